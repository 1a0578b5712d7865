"""CPU oracle for the percolation inspection (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of ``bench.py`` may import
this package; the product path never does. The arithmetic lives in ``perc_oracle.c``
(plain C, FP64, one configuration per OpenMP thread as in Sec. II.B of the paper);
this module is argument marshalling with ``ctypes`` and numpy.

Functions and the passage of the paper each one follows:

* :class:`Lattice` -- modified FCC fiber lattice built from geometry (Sec. II.A,
  Fig. 1): 12 side contacts at the FCC nearest-neighbour distance, 2 end contacts
  along the column.
* :func:`philox4x32_10`, :meth:`Lattice.sample` -- Bernoulli(p) occupancy (Sec. II.A)
  from Philox4x32-10 (Salmon et al., SC'11), pinned by the generator's published
  known-answer outputs, uniformity tests, host/device equality and a shift identity of
  the key schedule against the closed forms of its Weyl increments.
* :meth:`Lattice.inspect_markov` -- Eq. (1)-(2) with the detector site of Sec. II.B,
  forward FP64 iteration plus the exact support that decides "non-zero probability".
* :meth:`Lattice.state_after` -- the same iteration for exactly K steps.
* :func:`eq3_backward`, :func:`first_passage_forward` -- Eq. (3)-(4) on any matrix.
* :meth:`Lattice.inspect_bfs`, :meth:`Lattice.inspect_uf` -- the plain reachability
  definition (independent pins).
* :meth:`Lattice.exhaustive` -- all 2^N configurations of a tiny lattice.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "perc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "_build", "liborc.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``perc_oracle.c`` into ``oracle/_build/liborc.so`` with gcc + OpenMP."""
    if not force and os.path.exists(_LIB_PATH):
        return _LIB_PATH
    os.makedirs(os.path.dirname(_LIB_PATH), exist_ok=True)
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = C.CDLL(_LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.orc_lattice_new.restype = vp
    lib.orc_lattice_new.argtypes = [C.c_int, C.c_int]
    lib.orc_lattice_new_ex.restype = vp
    lib.orc_lattice_new_ex.argtypes = [C.c_int, C.c_int, C.c_int]
    lib.orc_lattice_free.argtypes = [vp]
    for f in ("orc_lattice_sites", "orc_lattice_bonds", "orc_lattice_nnz"):
        getattr(lib, f).restype = i64
        getattr(lib, f).argtypes = [vp]
    lib.orc_lattice_coords.argtypes = [vp, vp, vp, vp]
    lib.orc_lattice_adjacency.argtypes = [vp, vp, vp]
    lib.orc_lattice_surfaces.argtypes = [vp, vp, vp]
    lib.orc_philox4x32_10.argtypes = [vp, vp, vp]
    lib.orc_threshold.restype = C.c_uint64
    lib.orc_threshold.argtypes = [dbl]
    lib.orc_sample.argtypes = [vp, dbl, C.c_uint64, i64, i64, vp]
    lib.orc_sample_fixed.argtypes = [vp, dbl, C.c_uint64, i64, i64, vp]
    lib.orc_first_passage_all.argtypes = [vp, vp, i32, vp]
    lib.orc_fixed_count.restype = i64
    lib.orc_fixed_count.argtypes = [i64, dbl]
    lib.orc_inspect_markov.argtypes = [vp, vp, i64, vp, vp, vp, C.c_int]
    lib.orc_state_after.argtypes = [vp, vp, i32, vp, vp]
    lib.orc_row_sums.argtypes = [vp, vp, vp, vp]
    lib.orc_eq3_backward.argtypes = [i64, vp, vp, vp, i32, i32, vp]
    lib.orc_first_passage_forward.argtypes = [i64, vp, vp, vp, i32, vp, i32, vp]
    lib.orc_inspect_bfs.argtypes = [vp, vp, i64, vp, vp, C.c_int]
    lib.orc_bfs_dist.argtypes = [vp, vp, vp]
    lib.orc_inspect_uf.argtypes = [vp, vp, i64, vp]
    lib.orc_exhaustive.argtypes = [vp, C.c_int, vp]
    lib.orc_num_threads.restype = C.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return int(_load().orc_num_threads())


def threshold(p: float) -> int:
    """floor(p * 2^32): a site is metallic iff its 32-bit draw is below this."""
    return int(_load().orc_threshold(float(p)))


def philox4x32_10(ctr, key) -> np.ndarray:
    lib = _load()
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib.orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


class Lattice:
    """Modified FCC fiber lattice of hex radius ``W`` and ``L`` (111) layers; with
    ``ends=False`` the regular FCC lattice of the same sites (no end contacts)."""

    def __init__(self, W: int, L: int, ends: bool = True):
        lib = _load()
        h = lib.orc_lattice_new_ex(int(W), int(L), 1 if ends else 0)
        self.ends = bool(ends)
        if not h:
            raise ValueError(f"oracle lattice W={W} L={L} rejected")
        self._h = h
        self.W, self.L = int(W), int(L)
        self.n = int(lib.orc_lattice_sites(h))
        self.words = (self.n + 31) // 32
        self.n_bonds = int(lib.orc_lattice_bonds(h))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and _lib is not None:
            _lib.orc_lattice_free(h)
            self._h = None

    # -- geometry -----------------------------------------------------------------
    def coords(self):
        q = np.zeros(self.n, np.int32); r = np.zeros(self.n, np.int32); k = np.zeros(self.n, np.int32)
        _lib.orc_lattice_coords(self._h, _ptr(q), _ptr(r), _ptr(k))
        return q, r, k

    def adjacency(self):
        nnz = int(_lib.orc_lattice_nnz(self._h))
        ptr = np.zeros(self.n + 1, np.int64); idx = np.zeros(max(nnz, 1), np.int32)
        _lib.orc_lattice_adjacency(self._h, _ptr(ptr), _ptr(idx))
        return ptr, idx[:nnz]

    def surfaces(self):
        s = np.zeros(self.n, np.uint8); f = np.zeros(self.n, np.uint8)
        _lib.orc_lattice_surfaces(self._h, _ptr(s), _ptr(f))
        return s.astype(bool), f.astype(bool)

    # -- occupancy -----------------------------------------------------------------
    def sample(self, p: float, seed: int, n_cfg: int, cfg0: int = 0) -> np.ndarray:
        bits = np.zeros((n_cfg, self.words), np.uint32)
        _check(_lib.orc_sample(self._h, float(p), int(seed) & (2**64 - 1), int(cfg0), int(n_cfg),
                               _ptr(bits)), "sample")
        return bits

    def sample_fixed(self, p: float, seed: int, n_cfg: int, cfg0: int = 0) -> np.ndarray:
        """Fixed-count ensemble: floor(N p + 1/2) metallic sites per configuration, the
        ones with the smallest 64-bit Philox keys (orc_sample_fixed)."""
        bits = np.zeros((n_cfg, self.words), np.uint32)
        _check(_lib.orc_sample_fixed(self._h, float(p), int(seed) & (2**64 - 1), int(cfg0), int(n_cfg),
                                     _ptr(bits)), "sample_fixed")
        return bits

    def _bits(self, bits) -> np.ndarray:
        b = np.ascontiguousarray(bits, dtype=np.uint32)
        if b.ndim == 1:
            b = b.reshape(1, -1)
        if b.shape[1] != self.words:
            raise ValueError(f"expected {self.words} words per configuration, got {b.shape[1]}")
        return b

    # -- the method ----------------------------------------------------------------
    def inspect_markov(self, bits, nthreads: int = 0):
        b = self._bits(bits)
        n_cfg = b.shape[0]
        perc = np.zeros(n_cfg, np.uint8); steps = np.zeros(n_cfg, np.int32)
        hm = np.zeros(n_cfg, np.float64)
        _check(_lib.orc_inspect_markov(self._h, _ptr(b), n_cfg, _ptr(perc), _ptr(steps), _ptr(hm),
                                       int(nthreads)), "inspect_markov")
        return perc, steps, hm

    def state_after(self, bits, K: int):
        b = self._bits(bits)
        x = np.zeros(self.n + 1, np.float64); reach = np.zeros(self.n + 1, np.uint8)
        _check(_lib.orc_state_after(self._h, _ptr(b[0]), int(K), _ptr(x), _ptr(reach)), "state_after")
        return x, reach.astype(bool)

    def first_passage_all(self, bits, M: int) -> np.ndarray:
        """out[s] = probability that the walk from tube s first reaches the detector at
        step M (Eq. 3 for every source), FP64; 0 for insulating tubes."""
        b = self._bits(bits)
        out = np.zeros(self.n, np.float64)
        _check(_lib.orc_first_passage_all(self._h, _ptr(b[0]), int(M), _ptr(out)), "first_passage_all")
        return out

    def row_sums(self, bits):
        b = self._bits(bits)
        sums = np.zeros(self.n + 1, np.float64); nr = np.zeros(1, np.int64)
        _check(_lib.orc_row_sums(self._h, _ptr(b[0]), _ptr(sums), _ptr(nr)), "row_sums")
        return sums[: int(nr[0])]

    # -- plain definition -------------------------------------------------------------
    def inspect_bfs(self, bits, nthreads: int = 0):
        b = self._bits(bits)
        n_cfg = b.shape[0]
        perc = np.zeros(n_cfg, np.uint8); steps = np.zeros(n_cfg, np.int32)
        _check(_lib.orc_inspect_bfs(self._h, _ptr(b), n_cfg, _ptr(perc), _ptr(steps), int(nthreads)),
               "inspect_bfs")
        return perc, steps

    def bfs_dist(self, bits):
        b = self._bits(bits)
        d = np.zeros(self.n, np.int32)
        _check(_lib.orc_bfs_dist(self._h, _ptr(b[0]), _ptr(d)), "bfs_dist")
        return d

    def inspect_uf(self, bits):
        b = self._bits(bits)
        perc = np.zeros(b.shape[0], np.uint8)
        _check(_lib.orc_inspect_uf(self._h, _ptr(b), b.shape[0], _ptr(perc)), "inspect_uf")
        return perc

    def exhaustive(self, method: str = "bfs") -> np.ndarray:
        """a[k] = number of percolating configurations with k metallic sites."""
        if self.n > 24:
            raise ValueError("exhaustive enumeration is limited to N <= 24")
        a = np.zeros(self.n + 1, np.int64)
        _check(_lib.orc_exhaustive(self._h, 1 if method == "markov" else 0, _ptr(a)), "exhaustive")
        return a


def pi_from_counts(a: np.ndarray, p: float) -> float:
    """Pi(p) = sum_k a_k p^k (1-p)^(N-k) for the exhaustive counts a_k."""
    n = len(a) - 1
    k = np.arange(n + 1)
    return float(np.sum(a * (p ** k) * ((1.0 - p) ** (n - k))))


def _csr_arrays(P_dense: np.ndarray):
    n = P_dense.shape[0]
    ptr = [0]; col = []; val = []
    for i in range(n):
        for j in range(n):
            if P_dense[i, j] != 0.0:
                col.append(j); val.append(float(P_dense[i, j]))
        ptr.append(len(col))
    return (np.asarray(ptr, np.int64), np.asarray(col, np.int32), np.asarray(val, np.float64))


def eq3_backward(P_dense: np.ndarray, j0: int, M: int) -> np.ndarray:
    """f[m-1, i] = P_i[first hit of j0 at step m] by Eq. (3)-(4), m = 1..M."""
    n = P_dense.shape[0]
    ptr, col, val = _csr_arrays(np.asarray(P_dense, np.float64))
    f = np.zeros((M, n), np.float64)
    _check(_load().orc_eq3_backward(n, _ptr(ptr), _ptr(col), _ptr(val), int(j0), int(M), _ptr(f)), "eq3")
    return f


def first_passage_forward(P_dense: np.ndarray, j0: int, x0, M: int) -> np.ndarray:
    """hit[m-1] = P_x0[first hit of j0 at step m] by the forward absorbing iteration."""
    n = P_dense.shape[0]
    ptr, col, val = _csr_arrays(np.asarray(P_dense, np.float64))
    x = np.ascontiguousarray(x0, np.float64)
    hit = np.zeros(M, np.float64)
    _check(_load().orc_first_passage_forward(n, _ptr(ptr), _ptr(col), _ptr(val), int(j0), _ptr(x), int(M),
                                             _ptr(hit)), "first_passage_forward")
    return hit
