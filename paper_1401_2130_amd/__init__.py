"""perc -- percolation inspection of carbon-nanotube fibers on MI355X (gfx950).

Thin ``ctypes`` binding of the C ABI in ``include/perc.h`` (``libperc.so``). The
functions keep the C names; arguments are marshalled from torch device tensors,
which serve only as device memory and streams. Every step of the inspection runs in
the HIP kernels of the library; there is no Python or CPU fallback: importing the
package raises when the library has not been built.

Conventions (see ``include/perc.h``): occupancy is ``int32`` tensors holding the
canonical bit words (``[n_cfg, words]``); decisions are ``uint8``, step counts
``int32``, first-hit probabilities ``float32``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np
import torch  # loaded first so that libperc.so binds to the same HIP runtime

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "_build", "libperc.so")

PERC_OK, PERC_EINVAL, PERC_ENOMEM, PERC_EHIP, PERC_EBUSY, PERC_ECANCELED, PERC_ECAP = 0, -1, -2, -3, -4, -5, -6
PERC_LATTICE_NO_END_CONTACTS = 1
FORM_AUTO, FORM_PLAIN, FORM_SPAN, FORM_PERSIST, FORM_SPAN2, FORM_PERSIST2, FORM_MIXED = 0, 1, 2, 3, 4, 5, 6
_FORMS = {"auto": FORM_AUTO, "plain": FORM_PLAIN, "span": FORM_SPAN, "persist": FORM_PERSIST, "span2": FORM_SPAN2,
          "persist2": FORM_PERSIST2, "mixed": FORM_MIXED}


class PercError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"perc error {code}: {msg}")
        self.code = code


class perc_options(C.Structure):
    _fields_ = [("form", C.c_int32), ("depth", C.c_int32), ("block", C.c_int32), ("grid", C.c_int32),
                ("graph_steps", C.c_int32)]


class perc_profile(C.Structure):
    _fields_ = [("step_launches", C.c_int64), ("step_ms", C.c_double), ("tube_steps", C.c_int64),
                ("persist_launches", C.c_int64), ("persist_ms", C.c_double), ("persist_tube_steps", C.c_int64)]


class perc_job(C.Structure):
    _fields_ = [("lat", C.c_void_p), ("occ_bits", C.c_void_p), ("p", C.c_double), ("seed", C.c_uint64),
                ("cfg", C.c_int64), ("group", C.c_int32)]


# perc_job as a numpy record, for building large job arrays without a Python loop
JOB_DTYPE = np.dtype({"names": ["lat", "occ_bits", "p", "seed", "cfg", "group"],
                      "formats": [np.uint64, np.uint64, np.float64, np.uint64, np.int64, np.int32],
                      "offsets": [getattr(perc_job, f).offset for f in ("lat", "occ_bits", "p", "seed", "cfg", "group")],
                      "itemsize": C.sizeof(perc_job)})


class perc_server_config(C.Structure):
    _fields_ = [("hbm_bytes", C.c_int64), ("max_slots", C.c_int32), ("tick_steps", C.c_int32), ("max_w", C.c_int32),
                ("host_only", C.c_int32), ("opt", perc_options), ("max_queue", C.c_int32), ("lookahead", C.c_int32)]


class perc_result(C.Structure):
    _fields_ = [("tag", C.c_uint64), ("W", C.c_int32), ("L", C.c_int32), ("p", C.c_double), ("seed", C.c_uint64),
                ("cfg", C.c_uint64), ("status", C.c_int32), ("perc", C.c_uint8), ("steps", C.c_int32),
                ("hit", C.c_float), ("t_arrive_ns", C.c_int64), ("t_admit_ns", C.c_int64), ("t_done_ns", C.c_int64)]


class perc_server_stats(C.Structure):
    _fields_ = [("queued", C.c_int64), ("in_flight", C.c_int64), ("completed", C.c_int64), ("ticks", C.c_int64),
                ("pool_bytes", C.c_int64), ("pool_used_bytes", C.c_int64), ("rejected", C.c_int64),
                ("cancelled", C.c_int64)]


class perc_request(C.Structure):
    _fields_ = [("t_arrive_ns", C.c_int64), ("W", C.c_int32), ("L", C.c_int32), ("p", C.c_double),
                ("seed", C.c_uint64), ("cfg", C.c_uint64), ("tag", C.c_uint64)]


class perc_pi_out(C.Structure):
    _fields_ = [("n_perc", C.c_int64), ("pi", C.c_double), ("bits", C.c_void_p), ("steps", C.c_void_p),
                ("hit", C.c_void_p)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1401_2130_amd/build.py` "
                          "(or __graft_entry__.build()); there is no fallback path")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, dbl = C.c_void_p, C.c_int64, C.c_int32, C.c_double
    lib.perc_lattice_create.restype = vp
    lib.perc_lattice_create.argtypes = [i32, i32]
    lib.perc_lattice_create_ex.restype = vp
    lib.perc_lattice_create_ex.argtypes = [i32, i32, i32]
    lib.perc_lattice_destroy.argtypes = [vp]
    for f in ("perc_lattice_sites", "perc_lattice_words", "perc_lattice_state_bytes"):
        getattr(lib, f).restype = i64
        getattr(lib, f).argtypes = [vp]
    lib.perc_lattice_columns.restype = i32
    lib.perc_lattice_columns.argtypes = [vp]
    lib.perc_site_coord.argtypes = [vp, i64, vp, vp, vp]
    lib.perc_site_neighbors.argtypes = [vp, i64, vp, vp]
    lib.perc_last_error.restype = C.c_char_p
    lib.perc_sample.argtypes = [vp, dbl, C.c_uint64, i64, i64, vp, vp]
    lib.perc_sample_fixed.argtypes = [vp, dbl, C.c_uint64, i64, i64, vp, vp]
    lib.perc_inspect.argtypes = [vp, vp, i64, vp, vp, vp]
    lib.perc_inspect_ex.argtypes = [vp, vp, i64, vp, vp, vp, C.POINTER(perc_options), vp]
    lib.perc_inspect_noalloc.argtypes = [vp, vp, i64, vp, vp, vp, vp]
    lib.perc_pi.argtypes = [vp, dbl, i64, C.c_uint64, C.POINTER(perc_pi_out), vp]
    lib.perc_pi_ex.argtypes = [vp, dbl, i64, C.c_uint64, C.POINTER(perc_pi_out), C.POINTER(perc_options), vp]
    lib.perc_state_after.argtypes = [vp, vp, i32, vp, vp, vp]
    lib.perc_first_passage.argtypes = [vp, vp, i32, vp, vp]
    lib.perc_first_passage_batch.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.perc_steps_hist.argtypes = [vp, vp, i64, i32, vp, vp]
    lib.perc_batch.argtypes = [C.POINTER(perc_job), i64, vp, vp, vp, vp, i32, C.POINTER(perc_options), vp]
    lib.perc_profile_enable.argtypes = [i32]
    lib.perc_profile_read.argtypes = [C.POINTER(perc_profile)]
    lib.perc_autotune.argtypes = [C.POINTER(perc_job), i64, i64, C.POINTER(perc_options), C.POINTER(dbl), vp]
    lib.perc_stream_copy.argtypes = [vp, vp, i64, i32, vp]
    lib.perc_trim.argtypes = []
    lib.perc_server_create.restype = vp
    lib.perc_server_create.argtypes = [C.POINTER(perc_server_config), vp]
    lib.perc_server_destroy.argtypes = [vp]
    lib.perc_server_submit.argtypes = [vp, i32, i32, dbl, C.c_uint64, C.c_uint64, C.c_uint64, i64]
    lib.perc_server_cancel.argtypes = [vp, C.c_uint64]
    lib.perc_server_tick.argtypes = [vp]
    lib.perc_server_poll.argtypes = [vp, C.POINTER(perc_result), i32]
    lib.perc_server_stats_read.argtypes = [vp, C.POINTER(perc_server_stats)]
    lib.perc_server_run.argtypes = [vp, C.POINTER(perc_request), i64, C.POINTER(perc_result)]
    return lib


_lib = _load()

EXPORTED = ("perc_lattice_create", "perc_lattice_create_ex", "perc_lattice_destroy", "perc_lattice_sites", "perc_lattice_words",
            "perc_lattice_columns", "perc_lattice_state_bytes", "perc_site_coord", "perc_site_neighbors",
            "perc_last_error", "perc_sample", "perc_sample_fixed", "perc_inspect", "perc_inspect_ex", "perc_inspect_noalloc",
            "perc_pi", "perc_pi_ex",
            "perc_batch", "perc_state_after", "perc_first_passage", "perc_first_passage_batch", "perc_steps_hist", "perc_profile_enable", "perc_profile_read", "perc_autotune",
            "perc_stream_copy", "perc_trim",
            "perc_server_create",
            "perc_server_destroy", "perc_server_submit", "perc_server_cancel", "perc_server_tick", "perc_server_poll",
            "perc_server_stats_read", "perc_server_run")


def perc_last_error() -> str:
    return _lib.perc_last_error().decode()


def _check(rc: int):
    if rc != PERC_OK:
        raise PercError(rc, perc_last_error())


def _stream(stream) -> Optional[int]:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dptr(t: Optional[torch.Tensor], dtype=None, numel=None) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected dtype {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"expected at least {numel} elements, got {t.numel()}")
    return t.data_ptr()


def _options(form="auto", depth=0, block=0, grid=0, graph_steps=0) -> perc_options:
    f = _FORMS[form] if isinstance(form, str) else int(form)
    return perc_options(f, int(depth), int(block), int(grid), int(graph_steps))


class Lattice:
    """Handle of ``perc_lattice_create_ex(W, L, flags)`` (destroyed with the object);
    ``ends=False`` gives the regular FCC lattice (PERC_LATTICE_NO_END_CONTACTS)."""

    def __init__(self, W: int, L: int, ends: bool = True):
        h = _lib.perc_lattice_create_ex(int(W), int(L), 0 if ends else PERC_LATTICE_NO_END_CONTACTS)
        self.ends = bool(ends)
        if not h:
            raise PercError(PERC_EINVAL, perc_last_error())
        self._h = h
        self._lib = _lib  # kept for the destructor at interpreter shutdown
        self.W, self.L = int(W), int(L)
        self.n = int(_lib.perc_lattice_sites(h))
        self.words = int(_lib.perc_lattice_words(h))
        self.columns = int(_lib.perc_lattice_columns(h))
        self.state_bytes = int(_lib.perc_lattice_state_bytes(h))

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = getattr(self, "_lib", None)
        if h and lib is not None:
            lib.perc_lattice_destroy(h)
            self._h = None

    def __repr__(self):
        return f"Lattice(W={self.W}, L={self.L}, sites={self.n}{'' if self.ends else ', regular FCC'})"


def perc_lattice_create(W: int, L: int) -> Lattice:
    return Lattice(W, L)


def perc_lattice_destroy(lat: Lattice) -> None:
    h = getattr(lat, "_h", None)
    if h:
        _lib.perc_lattice_destroy(h)
        lat._h = None


def perc_lattice_sites(lat: Lattice) -> int:
    return int(_lib.perc_lattice_sites(lat.handle))


def perc_lattice_words(lat: Lattice) -> int:
    return int(_lib.perc_lattice_words(lat.handle))


def perc_lattice_columns(lat: Lattice) -> int:
    return int(_lib.perc_lattice_columns(lat.handle))


def perc_lattice_state_bytes(lat: Lattice) -> int:
    return int(_lib.perc_lattice_state_bytes(lat.handle))


def perc_site_coord(lat: Lattice, s: int):
    q, r, k = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.perc_site_coord(lat.handle, int(s), C.byref(q), C.byref(r), C.byref(k)))
    return q.value, r.value, k.value


def perc_site_neighbors(lat: Lattice, s: int):
    buf = (C.c_int64 * 14)()
    cnt = C.c_int32()
    _check(_lib.perc_site_neighbors(lat.handle, int(s), buf, C.byref(cnt)))
    return list(buf[: cnt.value])


def perc_sample(lat: Lattice, p: float, seed: int, n_cfg: int, cfg0: int = 0, out: Optional[torch.Tensor] = None,
                stream=None) -> torch.Tensor:
    """Occupancy words [n_cfg, words] (int32 bit patterns) of the Philox stream."""
    if out is None:
        out = torch.empty((n_cfg, lat.words), dtype=torch.int32, device="cuda")
    _check(_lib.perc_sample(lat.handle, float(p), int(seed) & (2**64 - 1), int(cfg0), int(n_cfg),
                            _dptr(out, torch.int32, n_cfg * lat.words), _stream(stream)))
    return out


def perc_sample_fixed(lat: Lattice, p: float, seed: int, n_cfg: int, cfg0: int = 0,
                      out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Occupancy words [n_cfg, words] of the fixed-count ensemble: exactly
    floor(N p + 1/2) metallic tubes per configuration, chosen uniformly (Philox keys)."""
    if out is None:
        out = torch.empty((n_cfg, lat.words), dtype=torch.int32, device="cuda")
    _check(_lib.perc_sample_fixed(lat.handle, float(p), int(seed) & (2**64 - 1), int(cfg0), int(n_cfg),
                                  _dptr(out, torch.int32, n_cfg * lat.words), _stream(stream)))
    return out


def perc_inspect(lat: Lattice, occ: torch.Tensor, n_cfg: Optional[int] = None, perc=None, steps=None,
                 stream=None):
    """Decisions (uint8) and step counts (int32) of canonical occupancy words."""
    return perc_inspect_ex(lat, occ, n_cfg, perc=perc, steps=steps, hit=False, stream=stream)[:2]


def perc_inspect_ex(lat: Lattice, occ: torch.Tensor, n_cfg: Optional[int] = None, perc=None, steps=None,
                    hit=False, form="auto", depth=0, block=0, grid=0, graph_steps=0, stream=None):
    """As perc_inspect with an execution form and the first-hit probability (float32)."""
    if n_cfg is None:
        n_cfg = occ.numel() // lat.words
    dev = occ.device
    if perc is None:
        perc = torch.empty(n_cfg, dtype=torch.uint8, device=dev)
    if steps is None:
        steps = torch.empty(n_cfg, dtype=torch.int32, device=dev)
    hit_t = None
    if hit is True:
        hit_t = torch.empty(n_cfg, dtype=torch.float32, device=dev)
    elif isinstance(hit, torch.Tensor):
        hit_t = hit
    opt = _options(form, depth, block, grid, graph_steps)
    _check(_lib.perc_inspect_ex(lat.handle, _dptr(occ, torch.int32, n_cfg * lat.words), int(n_cfg),
                                _dptr(perc, torch.uint8, n_cfg), _dptr(steps, torch.int32, n_cfg),
                                _dptr(hit_t, torch.float32, n_cfg), C.byref(opt), _stream(stream)))
    return perc, steps, hit_t


def perc_inspect_noalloc(lat: Lattice, occ: torch.Tensor, perc: torch.Tensor, steps=None, hit=None,
                         n_cfg: Optional[int] = None, stream=None):
    """perc_inspect_ex in the span form with the library's fixed work array: the caller
    passes every output buffer; the call allocates nothing (synchronous)."""
    if n_cfg is None:
        n_cfg = occ.numel() // lat.words
    _check(_lib.perc_inspect_noalloc(lat.handle, _dptr(occ, torch.int32, n_cfg * lat.words), int(n_cfg),
                                     _dptr(perc, torch.uint8, n_cfg), _dptr(steps, torch.int32, n_cfg),
                                     _dptr(hit, torch.float32, n_cfg), _stream(stream)))
    return perc, steps, hit


def perc_pi(lat: Lattice, p: float, n_cfg: int, seed: int, bits=None, steps=None, hit=None, stream=None):
    """Pi(p) over configurations 0..n_cfg-1 of the Philox stream ``seed`` (synchronous)."""
    return perc_pi_ex(lat, p, n_cfg, seed, bits=bits, steps=steps, hit=hit, stream=stream)


def perc_pi_ex(lat: Lattice, p: float, n_cfg: int, seed: int, bits=None, steps=None, hit=None, form="auto",
               depth=0, block=0, grid=0, graph_steps=0, stream=None):
    out = perc_pi_out(0, 0.0, _dptr(bits, torch.uint8, n_cfg), _dptr(steps, torch.int32, n_cfg),
                      _dptr(hit, torch.float32, n_cfg))
    opt = _options(form, depth, block, grid, graph_steps)
    _check(_lib.perc_pi_ex(lat.handle, float(p), int(n_cfg), int(seed) & (2**64 - 1), C.byref(out), C.byref(opt),
                           _stream(stream)))
    return int(out.n_perc), float(out.pi)


def philox_jobs(lat: "Lattice", p: float, seed: int, n_cfg: int, cfg0: int = 0, group: int = -1) -> np.ndarray:
    """Jobs (lat, p, seed, cfg) for cfg = cfg0 .. cfg0+n_cfg-1 as a JOB_DTYPE array, the
    fast form of the job list for perc_batch / perc_autotune (concatenate several with
    numpy). The array holds the lattice's handle: keep the Lattice alive while it is used."""
    a = np.zeros(n_cfg, dtype=JOB_DTYPE)
    a["lat"] = lat.handle
    a["p"] = float(p)
    a["seed"] = int(seed) & (2**64 - 1)
    a["cfg"] = np.arange(cfg0, cfg0 + n_cfg, dtype=np.int64)
    a["group"] = group
    return a


def _job_array(jobs):
    """perc_job array of (lattice, occ[, group]) or (lattice, p, seed, cfg[, group]) tuples,
    or of a JOB_DTYPE numpy array (used in place), and what it points into (kept alive by
    the caller)."""
    if isinstance(jobs, np.ndarray):
        if jobs.dtype.names != JOB_DTYPE.names:
            raise TypeError("a numpy job array must have the fields of JOB_DTYPE")
        if jobs.dtype != JOB_DTYPE or not jobs.flags.c_contiguous:
            # numpy packs a structured dtype when it concatenates: copy the fields back
            # into the struct layout (padding zero)
            out = np.zeros(len(jobs), dtype=JOB_DTYPE)
            for name in JOB_DTYPE.names:
                out[name] = jobs[name]
            jobs = out
        return jobs.ctypes.data_as(C.POINTER(perc_job)), [jobs]
    n = len(jobs)
    arr = (perc_job * max(n, 1))()
    keep = []
    for j, job in enumerate(jobs):
        lat = job[0]
        if isinstance(job[1], torch.Tensor):
            keep.append(job[1])
            grp = int(job[2]) if len(job) > 2 else -1
            arr[j] = perc_job(lat.handle, _dptr(job[1], torch.int32, lat.words), 0.0, 0, 0, grp)
        else:
            p, seed, cfg = job[1], job[2], job[3]
            grp = int(job[4]) if len(job) > 4 else -1
            arr[j] = perc_job(lat.handle, None, float(p), int(seed) & (2**64 - 1), int(cfg), grp)
    return arr, keep


def perc_autotune(jobs, n_target: int = 0, stream=None) -> dict:
    """Time candidate execution settings on the sample ``jobs`` (tuples as perc_batch,
    without groups) and return the fastest as keyword options for perc_batch /
    perc_pi_ex / perc_inspect_ex (``form``, ``depth``, ``block``, ``graph_steps``) plus
    ``ms``; a single-shape sample also sets the choice for form="auto" at batch size
    about ``n_target``."""
    arr, keep = _job_array(jobs)
    best = perc_options()
    ms = C.c_double()
    _check(_lib.perc_autotune(arr, len(jobs), int(n_target), C.byref(best), C.byref(ms), _stream(stream)))
    names = {v: k for k, v in _FORMS.items()}
    return {"form": names[best.form], "depth": int(best.depth), "block": int(best.block),
            "graph_steps": int(best.graph_steps), "ms": float(ms.value)}


def perc_batch(jobs, n_groups: int = 0, perc=None, steps=None, hit=False, form="auto", depth=0, block=0, grid=0,
               graph_steps=0, stream=None):
    """Inspect a list of jobs of possibly different lattices in one batch.

    ``jobs``: sequence of (lattice, occ) with occ a device int32 word tensor of one
    configuration, or (lattice, p, seed, cfg[, group]) for a Philox draw. Returns
    (perc uint8, steps int32, hit float32 or None, group counts list)."""
    n = len(jobs)
    arr, keep = _job_array(jobs)
    if perc is None:
        perc = torch.empty(n, dtype=torch.uint8, device="cuda")
    if steps is None:
        steps = torch.empty(n, dtype=torch.int32, device="cuda")
    hit_t = torch.empty(n, dtype=torch.float32, device="cuda") if hit is True else (hit if isinstance(hit, torch.Tensor) else None)
    counts = (C.c_int64 * max(n_groups, 1))()
    opt = _options(form, depth, block, grid, graph_steps)
    _check(_lib.perc_batch(arr, n, _dptr(perc, torch.uint8, n), _dptr(steps, torch.int32, n),
                           _dptr(hit_t, torch.float32, n), counts if n_groups else None, int(n_groups), C.byref(opt),
                           _stream(stream)))
    return perc, steps, hit_t, list(counts[:n_groups])


def perc_stream_copy(src: torch.Tensor, dst: torch.Tensor, grid: int = 0, stream=None) -> None:
    """The streaming copy of the HBM ceiling measurement (src -> dst, same byte size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() < nbytes:
        raise ValueError("dst is smaller than src")
    _check(_lib.perc_stream_copy(_dptr(src), _dptr(dst), int(nbytes), int(grid), _stream(stream)))


def perc_trim() -> None:
    """Release the work buffer the library keeps between calls on the current device."""
    _check(_lib.perc_trim())


def perc_profile_enable(on: bool) -> None:
    _check(_lib.perc_profile_enable(1 if on else 0))


def perc_profile_read() -> dict:
    out = perc_profile()
    _check(_lib.perc_profile_read(C.byref(out)))
    return {"step_launches": int(out.step_launches), "step_ms": float(out.step_ms),
            "tube_steps": int(out.tube_steps), "persist_launches": int(out.persist_launches),
            "persist_ms": float(out.persist_ms), "persist_tube_steps": int(out.persist_tube_steps)}


def perc_state_after(lat: Lattice, occ: torch.Tensor, K: int, x=None, reach=None, stream=None):
    """Exactly K steps of one configuration: probabilities (N+1 float32) and reach (N+1 uint8)."""
    dev = occ.device
    if x is None:
        x = torch.empty(lat.n + 1, dtype=torch.float32, device=dev)
    if reach is None:
        reach = torch.empty(lat.n + 1, dtype=torch.uint8, device=dev)
    _check(_lib.perc_state_after(lat.handle, _dptr(occ, torch.int32, lat.words), int(K),
                                 _dptr(x, torch.float32, lat.n + 1), _dptr(reach, torch.uint8, lat.n + 1),
                                 _stream(stream)))
    return x, reach


def perc_first_passage(lat: Lattice, occ: torch.Tensor, M: int, f=None, stream=None):
    """First-passage probabilities at move M from every tube (N float32, canonical order)."""
    if f is None:
        f = torch.empty(max(lat.n, 1), dtype=torch.float32, device=occ.device)
    _check(_lib.perc_first_passage(lat.handle, _dptr(occ, torch.int32, lat.words), int(M),
                                   _dptr(f, torch.float32, lat.n), _stream(stream)))
    return f[: lat.n]


def perc_first_passage_batch(lat: Lattice, occ: torch.Tensor, M: int, n_cfg: Optional[int] = None, f=None,
                             stream=None):
    """First-passage probabilities at move M from every tube of n_cfg configurations
    ([n_cfg, N] float32)."""
    if n_cfg is None:
        n_cfg = occ.numel() // lat.words
    if f is None:
        f = torch.empty((n_cfg, lat.n), dtype=torch.float32, device=occ.device)
    _check(_lib.perc_first_passage_batch(lat.handle, _dptr(occ, torch.int32, n_cfg * lat.words), int(n_cfg), int(M),
                                         _dptr(f, torch.float32, n_cfg * lat.n), _stream(stream)))
    return f


def perc_steps_hist(perc: torch.Tensor, steps: torch.Tensor, nbins: int, hist=None, stream=None):
    """Histogram of m* over the percolating entries (bins 0 .. nbins-1, last bin open)."""
    n = perc.numel()
    if hist is None:
        hist = torch.zeros(nbins, dtype=torch.int64, device=perc.device)
    _check(_lib.perc_steps_hist(_dptr(perc, torch.uint8, n), _dptr(steps, torch.int32, n), int(n), int(nbins),
                                _dptr(hist, torch.int64, nbins), _stream(stream)))
    return hist


# ---------------------------------------------------------------------------------
# serving (continuous batching of single inspections)
# ---------------------------------------------------------------------------------

_RESULT_KEYS = ("tag", "W", "L", "p", "seed", "cfg", "status", "perc", "steps", "hit", "t_arrive_ns", "t_admit_ns",
                "t_done_ns")


def _result_dict(r: perc_result) -> dict:
    return {k: getattr(r, k) for k in _RESULT_KEYS}


class perc_server:
    """A serving instance (``perc_server_create``): requests of single configurations
    (W, L, p, seed, cfg) are admitted by HBM footprint as slots free up and advanced
    together, a tick at a time; the state of every admitted request stays on the GPU."""

    def __init__(self, hbm_bytes: int = 0, max_slots: int = 0, tick_steps: int = 0, max_w: int = 0,
                 host_only: bool = False, depth: int = 0, block: int = 0, grid: int = 0, max_queue: int = 0,
                 lookahead: int = 0, stream=None):
        cfg = perc_server_config(int(hbm_bytes), int(max_slots), int(tick_steps), int(max_w), 1 if host_only else 0,
                                 _options("span", depth, block, grid, 0), int(max_queue), int(lookahead))
        self._lib = _lib
        self._stream = stream  # the server works on this stream; keep it alive as long
        self.handle = _lib.perc_server_create(C.byref(cfg), None if host_only else _stream(stream))
        if not self.handle:
            raise PercError(PERC_EINVAL, perc_last_error())

    def __del__(self):
        h, lib = getattr(self, "handle", None), getattr(self, "_lib", None)
        if h and lib is not None:
            lib.perc_server_destroy(h)
            self.handle = None

    def submit(self, W: int, L: int, p: float, seed: int, cfg: int = 0, tag: int = 0, t_arrive_ns: int = -1):
        _check(_lib.perc_server_submit(self.handle, int(W), int(L), float(p), int(seed), int(cfg), int(tag),
                                       int(t_arrive_ns)))

    def cancel(self, tag: int) -> int:
        """Cancel the requests with this tag (queued: at once; in flight: at the next
        tick); returns how many were cancelled."""
        rc = _lib.perc_server_cancel(self.handle, int(tag))
        if rc < 0:
            _check(rc)
        return rc

    def tick(self) -> int:
        rc = _lib.perc_server_tick(self.handle)
        if rc < 0:
            _check(rc)
        return rc

    def poll(self, max_results: int = 4096) -> list:
        buf = (perc_result * max_results)()
        n = _lib.perc_server_poll(self.handle, buf, int(max_results))
        if n < 0:
            _check(n)
        return [_result_dict(buf[i]) for i in range(n)]

    def stats(self) -> dict:
        st = perc_server_stats()
        _check(_lib.perc_server_stats_read(self.handle, C.byref(st)))
        return {k: int(getattr(st, k)) for k, _ in perc_server_stats._fields_}

    def run(self, requests) -> list:
        """Serve a request stream natively (``perc_server_run``): requests are
        (t_arrive_s, W, L, p, seed, cfg, tag) with non-decreasing arrival offsets."""
        n = len(requests)
        reqs = (perc_request * max(n, 1))()
        for i, (t, W, L, p, seed, cfg, tag) in enumerate(requests):
            reqs[i] = perc_request(int(round(t * 1e9)), int(W), int(L), float(p), int(seed), int(cfg), int(tag))
        out = (perc_result * max(n, 1))()
        _check(_lib.perc_server_run(self.handle, reqs, n, out))
        return [_result_dict(out[i]) for i in range(n)]
