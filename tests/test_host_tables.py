"""Host-built tables of the tile walks (CPU only): the lane maps and the contact tables
stored by lane.

For every tile of hex radius W, and for the whole-cross-section tile where it exists:
* every column of the tile is computed by some lane, lanes take the columns in order,
  and a repeated column (an idle lane) sits next to its first lane;
* each lane's packed words hold the LDS words of that lane's column's side contacts:
  column kPadCols + its place in the tile's staged range, row 1 + dcell, rows 64 words
  apart, columns in blocks of 64 with ten rows each; a missing contact reads a word of
  row 1 of the zero pad block (block 0);
* no half-wave (32 lanes) reads two different words of one LDS bank (word mod 32) for
  one contact direction on the tiles of the benchmarked widths (W = 8 .. 32) and the
  smaller whole-cross-section tiles; where the lane budget (the tile width rounded up to
  64) leaves too few idle lanes (W = 4, 48, 64, the 817-column whole tile of W = 16) some
  remain, never more than with one lane per column in order.

The tables are printed by tests/host/table_dump.cpp, built here from the library's own
lattice source with the host compiler.
"""
import os
import shutil
import subprocess
from collections import defaultdict

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1401_2130_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
KBLK, KROWS, KPAD, HALF = 64, 10, 64, 32

# the offsets (dq, dr) of the 12 side contacts in the library's order
SIDE = [(1, 1), (2, -1), (1, -2), (-1, -1), (-2, 1), (-1, 2), (1, 0), (-1, 1), (0, -1), (0, 1), (-1, 0), (1, -1)]


def ring_word(row, lcol):
    return (lcol // KBLK) * KBLK * KROWS + row * KBLK + lcol % KBLK


@pytest.fixture(scope="module")
def dump(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime_api.h")):
        pytest.skip("needs g++ and the HIP headers")
    exe = str(tmp_path_factory.mktemp("tables") / "table_dump")
    cmd = [gxx, "-O1", "-std=c++17", "-D__HIP_PLATFORM_AMD__=1", f"-I{ROCM}/include", f"-I{CSRC}",
           f"-I{ROOT}/include", os.path.join(ROOT, "tests", "host", "table_dump.cpp"),
           os.path.join(CSRC, "lattice.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)

    def run(W):
        it = iter(subprocess.run([exe, str(W)], check=True, capture_output=True, text=True).stdout.split())
        C, nt, B = int(next(it)), int(next(it)), int(next(it))
        tiles = [tuple(int(next(it)) for _ in range(4)) for _ in range(nt)]
        lanes = [int(next(it)) for _ in range(nt * B)]
        packed = [int(next(it)) for _ in range(6 * nt * B)]
        nb = [int(next(it)) for _ in range(12 * C)]
        Bw = int(next(it))
        lanes_w = [int(next(it)) for _ in range(Bw)]
        packed_w = [int(next(it)) for _ in range(6 * Bw)]
        return dict(C=C, nt=nt, B=B, tiles=tiles, lanes=lanes, packed=packed, nb=nb, Bw=Bw, lanes_w=lanes_w,
                    packed_w=packed_w)
    return run


def conflicts_in_order(d, ts, te, hs, B):
    """Bank conflicts of the real contacts with one lane per column in order (the lanes
    beyond the tile on its first column), missing contacts counted as free."""
    C, nb = d["C"], d["nb"]
    cols = [c if c < te else ts for c in range(ts, ts + B)]
    n = 0
    for h0 in range(0, B, HALF):
        for i in range(12):
            per = defaultdict(set)
            for c in cols[h0:h0 + HALF]:
                col, dcp1 = nb[i * C + c] >> 2, nb[i * C + c] & 3
                if col < C:
                    v = ring_word(dcp1, col - hs + KPAD)
                    per[v % HALF].add(v)
            n += max([len(s) for s in per.values()] + [1]) - 1
    return n


def check_tile(d, ts, te, hs, lanes, word, B):
    """lanes: the lane map of one tile (B entries); word(j, l): packed word j of lane l."""
    C, nb = d["C"], d["nb"]
    assert len(lanes) == B and B % 64 == 0 and B >= te - ts
    # coverage and order: 0, then each lane repeats or advances by one; every column used
    assert lanes[0] == 0
    for a, b in zip(lanes, lanes[1:]):
        assert b in (a, a + 1)
    assert lanes[-1] == te - ts - 1
    # contents: the LDS word of each contact of each lane's column
    for l, off in enumerate(lanes):
        c = ts + off
        for i in range(12):
            v = (word(i // 2, l) >> (16 * (i % 2))) & 0xFFFF
            col, dcp1 = nb[i * C + c] >> 2, nb[i * C + c] & 3
            if col < C:
                assert v == ring_word(dcp1, col - hs + KPAD), (c, i)
            else:
                assert KBLK <= v < 2 * KBLK, (c, i, v)  # row 1 of the zero pad block
    # bank conflicts per half-wave and direction
    conflicts = 0
    for h0 in range(0, B, HALF):
        for i in range(12):
            per = defaultdict(set)
            for l in range(h0, h0 + HALF):
                v = (word(i // 2, l) >> (16 * (i % 2))) & 0xFFFF
                per[v % HALF].add(v)
            conflicts += max(len(s) for s in per.values()) - 1
    return conflicts


@pytest.mark.parametrize("W", [0, 1, 2, 3, 4, 5, 8, 12, 16, 18, 24, 32, 48, 64])
def test_tile_tables(dump, W):
    d = dump(W)
    B, nt = d["B"], d["nt"]
    assert d["C"] == 3 * W * (W + 1) + 1
    conflicts = in_order = 0
    for k, (ts, te, hs, he) in enumerate(d["tiles"]):
        lanes = d["lanes"][k * B:(k + 1) * B]
        conflicts += check_tile(d, ts, te, hs, lanes, lambda j, l: d["packed"][j * nt * B + k * B + l], B)
        in_order += conflicts_in_order(d, ts, te, hs, B)
    assert conflicts <= in_order
    if W not in (4, 48, 64):
        assert conflicts == 0


@pytest.mark.parametrize("W", [0, 1, 2, 4, 8, 12, 16, 17])
def test_whole_tile_tables(dump, W):
    d = dump(W)
    Bw, C = d["Bw"], d["C"]
    assert Bw == (C + 63) // 64 * 64  # W <= 17: at most 1,024 columns
    conflicts = check_tile(d, 0, C, 0, d["lanes_w"], lambda j, l: d["packed_w"][j * Bw + l], Bw)
    assert conflicts <= conflicts_in_order(d, 0, C, 0, Bw)
    if W not in (4, 16, 17):
        assert conflicts == 0


def test_no_whole_tile_beyond_1024_columns(dump):
    assert dump(18)["Bw"] == 0  # 1,027 columns


def test_contact_order_matches_the_lattice(dump):
    """The directions the tables are checked against are the lattice's own: a column's
    contact i lies at (q + dq_i, r + dr_i) on the hexagon (W = 3, centre column)."""
    d = dump(3)
    C, nb = d["C"], d["nb"]
    cols = [(q, r) for q in range(-3, 4) for r in range(-3, 4) if max(abs(q), abs(r), abs(q + r)) <= 3]
    assert len(cols) == C
    c0 = cols.index((0, 0))
    for i, (dq, dr) in enumerate(SIDE):
        assert cols[nb[i * C + c0] >> 2] == (dq, dr)
