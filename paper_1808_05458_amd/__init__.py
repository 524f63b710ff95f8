"""Exact global minimum cut on one MI355X: Python binding of ``libmincut.so``.

Argument marshalling only.  Every step of the solve runs in the HIP kernels
behind the C ABI declared in ``include/mincut.h``; PyTorch provides device
memory and the stream.  There is no CPU fallback: if the library is not
built, every call raises.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
_LIB = os.path.join(_HERE, "libmincut.so")
_SOURCES = [os.path.join(_HERE, "csrc", "engine.hip")]
HEADER = os.path.join(_ROOT, "include", "mincut.h")

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-result", "-Wno-unused-value"]

MC_OK, MC_EINVAL, MC_ENOCUT, MC_EOVERFLOW, MC_ENOMEM, MC_EHIP, MC_EBUSY, MC_ESTATE = (
    0, -1, -2, -3, -4, -5, -6, -7)
MC_EINTERNAL = -8
MC_EMISMATCH = -9
MC_ETOOBIG = -10


def build() -> str:
    """Compile the HIP library for gfx950 (always recompiles)."""
    out = _LIB + ".tmp"
    cmd = ["hipcc", *HIPCC_FLAGS, *_SOURCES, "-o", out]
    subprocess.check_call(cmd, cwd=_ROOT)
    os.replace(out, _LIB)
    return _LIB


class MincutError(RuntimeError):
    def __init__(self, code: int, what: str):
        lib = _load()
        msg = lib.mc_strerror(code).decode()
        super().__init__(f"{what}: {msg} (code {code})")
        self.code = code


class Options(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("use_pr", ctypes.c_int32),
                ("use_viecut", ctypes.c_int32), ("region_waves", ctypes.c_int32),
                ("eager_blacklist", ctypes.c_int32), ("max_pops", ctypes.c_int32),
                ("max_rounds", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("force_fallback", ctypes.c_int32), ("whole_max", ctypes.c_int32),
                ("lp_sweeps", ctypes.c_int32), ("scan_mode", ctypes.c_int32),
                ("sweep_handoff", ctypes.c_int32), ("viecut_stop", ctypes.c_int32),
                ("viecut_levels", ctypes.c_int32), ("sweep_threads", ctypes.c_int32),
                ("sweep_groups", ctypes.c_int32), ("sort_tile", ctypes.c_int32),
                ("pr_triangle_deg", ctypes.c_int32), ("viecut_exact", ctypes.c_int32),
                ("approx_ppm", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_uint64),
                ("sweep_tail", ctypes.c_int32), ("sweep_pull", ctypes.c_int32),
                ("pq_order", ctypes.c_int32), ("scan_visits", ctypes.c_int32),
                ("use_tuned", ctypes.c_int32), ("emit_rows", ctypes.c_int32),
                ("sweep_seg", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [("best", Options), ("candidates", ctypes.c_int32), ("reps", ctypes.c_int32),
                ("best_ms", ctypes.c_double), ("default_ms", ctypes.c_double)]


class Stats(ctypes.Structure):
    _fields_ = [("rounds", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("unions_pr", ctypes.c_int64), ("pairs_scan", ctypes.c_int64),
                ("scans", ctypes.c_int64), ("pops", ctypes.c_int64),
                ("overflows", ctypes.c_int64), ("lambda_initial", ctypes.c_int64),
                ("lambda_viecut", ctypes.c_int64), ("ms", ctypes.c_double),
                ("n_round", ctypes.c_int32 * 64), ("nnz_round", ctypes.c_int64 * 64),
                ("sweep_phases", ctypes.c_int32), ("sweep_big_batches", ctypes.c_int32),
                ("sweep_singles", ctypes.c_int32 * 8), ("sweep_batches", ctypes.c_int32 * 8),
                ("sweep_cross", ctypes.c_int32 * 8), ("sweep_tail_pops", ctypes.c_int64)]

    def as_dict(self):
        r = min(self.rounds, 64)
        return {"rounds": self.rounds, "fallbacks": self.fallbacks,
                "unions_pr": self.unions_pr, "pairs_scan": self.pairs_scan,
                "scans": self.scans, "pops": self.pops, "overflows": self.overflows,
                "lambda_initial": self.lambda_initial, "lambda_viecut": self.lambda_viecut,
                "ms": self.ms, "n_round": list(self.n_round[:r]),
                "nnz_round": list(self.nnz_round[:r]),
                "sweep_big_batches": self.sweep_big_batches,
                "sweep_singles": list(self.sweep_singles[:self.sweep_phases]),
                "sweep_batches": list(self.sweep_batches[:self.sweep_phases]),
                "sweep_cross": list(self.sweep_cross[:self.sweep_phases]),
                "sweep_tail_pops": self.sweep_tail_pops}


class Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class Batch(ctypes.Structure):
    _fields_ = [("num_graphs", ctypes.c_int32), ("n_total", ctypes.c_int32),
                ("nnz_total", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("vtx_off", ctypes.c_void_p)]


class TimingEntry(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 24), ("launches", ctypes.c_int64),
                ("ms", ctypes.c_double), ("algo_bytes", ctypes.c_double)]


_lib = None


def library_path() -> str:
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        raise RuntimeError(
            f"{_LIB} is not built; run __graft_entry__.build() (hipcc, gfx950). "
            "There is no CPU fallback.")
    lib = ctypes.CDLL(_LIB)
    vp = ctypes.c_void_p
    lib.mc_options_default.argtypes = [vp]
    lib.mc_options_default.restype = None
    lib.mc_mincut.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mc_mincut.restype = ctypes.c_int
    lib.mc_mincut_noalloc.argtypes = [vp, vp, vp, vp, vp]
    lib.mc_mincut_noalloc.restype = ctypes.c_int
    lib.mc_mincut_batched.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mc_mincut_batched.restype = ctypes.c_int
    lib.mc_tune_batched.argtypes = [vp, vp, vp, ctypes.c_int32, vp]
    lib.mc_tune_batched.restype = ctypes.c_int
    lib.mc_tune_lookup.argtypes = [vp, vp]
    lib.mc_tune_lookup.restype = ctypes.c_int
    lib.mc_tune_clear.argtypes = []
    lib.mc_tune_clear.restype = None
    lib.mc_debug_first_round.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mc_debug_first_round.restype = ctypes.c_int
    lib.mc_debug_contract.argtypes = [vp, vp, ctypes.c_int32, vp, vp, vp, vp, vp]
    lib.mc_debug_contract.restype = ctypes.c_int
    lib.mc_debug_lp_sweep.argtypes = [vp, vp, vp, vp]
    lib.mc_debug_lp_sweep.restype = ctypes.c_int
    lib.mc_debug_pr_tests.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, vp]
    lib.mc_debug_pr_tests.restype = ctypes.c_int
    lib.mc_viecut_bound.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.mc_viecut_bound.restype = ctypes.c_int
    lib.mc_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.mc_workspace_bytes.restype = ctypes.c_size_t
    lib.mc_viecut_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    lib.mc_viecut_workspace_bytes.restype = ctypes.c_size_t
    lib.mc_release.argtypes = []
    lib.mc_release.restype = None
    lib.mc_strerror.argtypes = [ctypes.c_int]
    lib.mc_strerror.restype = ctypes.c_char_p
    lib.mc_timing_get.argtypes = [vp, ctypes.c_int]
    lib.mc_timing_get.restype = ctypes.c_int
    lib.mc_timing_reset.argtypes = []
    lib.mc_timing_reset.restype = None
    lib.mc_timing_focus.argtypes = [ctypes.c_char_p]
    lib.mc_timing_focus.restype = None
    lib.mc_server_cfg_default.argtypes = [vp]
    lib.mc_server_cfg_default.restype = None
    lib.mc_server_create.argtypes = [vp, vp]
    lib.mc_server_create.restype = ctypes.c_int
    lib.mc_server_submit.argtypes = [vp, vp, vp]
    lib.mc_server_submit.restype = ctypes.c_int
    lib.mc_server_wait.argtypes = [vp, ctypes.c_uint64, vp, vp, vp]
    lib.mc_server_wait.restype = ctypes.c_int
    lib.mc_server_destroy.argtypes = [vp]
    lib.mc_server_destroy.restype = ctypes.c_int
    _lib = lib
    return lib


class ServerCfg(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("small_max_nnz", ctypes.c_int64), ("max_batch_nnz", ctypes.c_int64),
                ("mem_budget", ctypes.c_int64),
                ("queue_cap", ctypes.c_int32), ("device", ctypes.c_int32),
                ("validate", ctypes.c_int32), ("reserved", ctypes.c_int32), ("opt", Options)]


class Request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("borrow", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p), ("w", ctypes.c_void_p)]


class Latency(ctypes.Structure):
    _fields_ = [("queue_ms", ctypes.c_double), ("solve_ms", ctypes.c_double),
                ("total_ms", ctypes.c_double), ("batch_graphs", ctypes.c_int32),
                ("lane", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Server:
    """The served form: host CSR requests, continuous batching over lanes.
    submit() returns a ticket; wait(ticket) returns (lambda, side, latency).
    With borrow=True the arrays are kept referenced here until wait()."""

    def __init__(self, opts: Optional[Options] = None, **cfg):
        lib = _load()
        c = ServerCfg()
        lib.mc_server_cfg_default(ctypes.byref(c))
        if opts is not None:
            c.opt = opts
        for k, v in cfg.items():
            if not hasattr(c, k):
                raise TypeError(f"unknown server setting {k}")
            setattr(c, k, v)
        self._lib = lib
        self._h = ctypes.c_void_p()
        rc = lib.mc_server_create(ctypes.byref(c), ctypes.byref(self._h))
        if rc != MC_OK:
            raise MincutError(rc, "mc_server_create")
        self._held = {}
        self._n = {}

    def submit(self, g, borrow: bool = True) -> int:
        rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
        col = np.ascontiguousarray(g.col, dtype=np.int32)
        w = np.ascontiguousarray(g.w, dtype=np.int32)
        r = Request(g.n, 1 if borrow else 0, len(col), rp.ctypes.data, col.ctypes.data, w.ctypes.data)
        t = ctypes.c_uint64(0)
        rc = self._lib.mc_server_submit(self._h, ctypes.byref(r), ctypes.byref(t))
        if rc != MC_OK:
            raise MincutError(rc, "mc_server_submit")
        if borrow:
            self._held[t.value] = (rp, col, w)
        self._n[t.value] = g.n
        return t.value

    def wait(self, ticket: int, want_side: bool = True):
        n = self._n.pop(ticket)
        side = np.zeros(n, np.uint8) if want_side else None
        lam = ctypes.c_int64(-1)
        lat = Latency()
        rc = self._lib.mc_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(lam),
                                      side.ctypes.data_as(ctypes.c_void_p) if side is not None else None,
                                      ctypes.byref(lat))
        self._held.pop(ticket, None)
        if rc != MC_OK:
            raise MincutError(rc, "mc_server_wait")
        return int(lam.value), side, lat.as_dict()

    def close(self):
        if self._h:
            self._lib.mc_server_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._held.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def options(**kw) -> Options:
    o = Options()
    _load().mc_options_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor on the GPU")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def mincut(row_ptr, col, w, *, want_side: bool = True, stream=None, opts: Optional[Options] = None,
           **kw):
    """lambda, side (uint8 tensor or None), stats dict for one graph whose
    CSR arrays are device tensors (int64 row_ptr, int32 col, int32 w)."""
    import torch
    lib = _load()
    n = row_ptr.numel() - 1
    g = Graph(n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"))
    o = opts if opts is not None else options(**kw)
    side = torch.empty(max(n, 1), dtype=torch.uint8, device=row_ptr.device) if want_side else None
    lam = ctypes.c_int64(-1)
    st = Stats()
    rc = lib.mc_mincut(ctypes.byref(g), _stream(stream), ctypes.byref(o), ctypes.byref(lam),
                       ctypes.c_void_p(side.data_ptr()) if side is not None else None,
                       ctypes.byref(st))
    if rc != MC_OK:
        raise MincutError(rc, "mc_mincut")
    return int(lam.value), side, st.as_dict()


def mincut_noalloc(row_ptr, col, w, side=None, *, stream=None, opts: Optional[Options] = None, **kw):
    """mc_mincut_noalloc: lambda of one graph (device tensors), solved in the
    library's fixed workspace.  `side`, if given, is a preallocated uint8
    device tensor of at least n entries that receives the side."""
    import torch
    lib = _load()
    n = row_ptr.numel() - 1
    g = Graph(n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"))
    o = opts if opts is not None else options(**kw)
    lam = ctypes.c_int64(-1)
    sp = None
    if side is not None:
        if side.numel() < n:
            raise ValueError("side must hold n entries")
        sp = _dev_ptr(side, torch.uint8, "side")
    rc = lib.mc_mincut_noalloc(ctypes.byref(g), _stream(stream), ctypes.byref(o), ctypes.byref(lam), sp)
    if rc != MC_OK:
        raise MincutError(rc, "mc_mincut_noalloc")
    return int(lam.value)


def mincut_batched(row_ptr, col, w, vtx_off: Sequence[int], *, want_side: bool = True,
                   stream=None, opts: Optional[Options] = None, **kw):
    """Solve all graphs of a packed CSR (global vertex ids; graph g owns
    vertices [vtx_off[g], vtx_off[g+1])).  Returns (lambdas int64 ndarray,
    sides uint8 tensor or None, stats dict)."""
    import torch
    lib = _load()
    voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    G = len(voff) - 1
    n = row_ptr.numel() - 1
    b = Batch(G, n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"),
              voff.ctypes.data_as(ctypes.c_void_p))
    o = opts if opts is not None else options(**kw)
    sides = torch.empty(max(n, 1), dtype=torch.uint8, device=row_ptr.device) if want_side else None
    lams = np.full(G, -1, np.int64)
    st = Stats()
    rc = lib.mc_mincut_batched(ctypes.byref(b), _stream(stream), ctypes.byref(o),
                               lams.ctypes.data_as(ctypes.c_void_p),
                               ctypes.c_void_p(sides.data_ptr()) if sides is not None else None,
                               ctypes.byref(st))
    if rc != MC_OK:
        raise MincutError(rc, "mc_mincut_batched")
    return lams, sides, st.as_dict()


def tune_batched(row_ptr, col, w, vtx_off: Sequence[int], *, reps: int = 2, stream=None,
                 opts: Optional[Options] = None, **kw):
    """Autotune the batched form on this batch (launch shapes, triangle
    tests, priority-queue order); the choice is also stored for the batch's
    size class, where solves with use_tuned=1 find it.  Returns (Options
    with the chosen settings, report dict)."""
    import torch
    lib = _load()
    voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    G = len(voff) - 1
    n = row_ptr.numel() - 1
    b = Batch(G, n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"),
              voff.ctypes.data_as(ctypes.c_void_p))
    o = opts if opts is not None else options(**kw)
    out = TuneResult()
    rc = lib.mc_tune_batched(ctypes.byref(b), _stream(stream), ctypes.byref(o), int(reps),
                             ctypes.byref(out))
    if rc != MC_OK:
        raise MincutError(rc, "mc_tune_batched")
    best = Options()
    ctypes.memmove(ctypes.byref(best), ctypes.byref(out.best), ctypes.sizeof(Options))
    report = {"candidates": out.candidates, "reps": out.reps, "best_ms": out.best_ms,
              "default_ms": out.default_ms, "sweep_threads": best.sweep_threads,
              "sweep_groups": best.sweep_groups, "sort_tile": best.sort_tile,
              "pr_triangle_deg": best.pr_triangle_deg, "pq_order": best.pq_order}
    return best, report


def tune_lookup(n_total: int, nnz_total: int, vtx_off: Sequence[int], opts: Optional[Options] = None):
    """The stored tuned settings for a batch of this size class (graph
    count len(vtx_off) - 1, n_total vertices, nnz_total entries) applied to
    a copy of opts (defaults if None), or None when none are stored."""
    lib = _load()
    voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    b = Batch(len(voff) - 1, int(n_total), int(nnz_total), None, None, None,
              voff.ctypes.data_as(ctypes.c_void_p))
    o = Options()
    if opts is not None:
        ctypes.memmove(ctypes.byref(o), ctypes.byref(opts), ctypes.sizeof(Options))
    else:
        lib.mc_options_default(ctypes.byref(o))
    rc = lib.mc_tune_lookup(ctypes.byref(b), ctypes.byref(o))
    if rc < 0:
        raise MincutError(rc, "mc_tune_lookup")
    return o if rc == 1 else None


def tune_clear():
    """Forget every stored tuned setting."""
    _load().mc_tune_clear()


def viecut_bound(row_ptr, col, w, vtx_off: Sequence[int], *, want_side: bool = True, stream=None,
                 opts: Optional[Options] = None, **kw):
    """The clustering upper bound alone for every graph of a packed CSR:
    (bounds int64 ndarray, sides uint8 tensor or None, levels run)."""
    import torch
    lib = _load()
    voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    G = len(voff) - 1
    n = row_ptr.numel() - 1
    b = Batch(G, n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"),
              voff.ctypes.data_as(ctypes.c_void_p))
    o = opts if opts is not None else options(**kw)
    sides = torch.empty(max(n, 1), dtype=torch.uint8, device=row_ptr.device) if want_side else None
    bounds = np.full(G, -1, np.int64)
    levels = ctypes.c_int32(0)
    rc = lib.mc_viecut_bound(ctypes.byref(b), _stream(stream), ctypes.byref(o),
                             bounds.ctypes.data_as(ctypes.c_void_p),
                             ctypes.c_void_p(sides.data_ptr()) if sides is not None else None,
                             ctypes.byref(levels))
    if rc != MC_OK:
        raise MincutError(rc, "mc_viecut_bound")
    return bounds, sides, int(levels.value)


def debug_lp_sweep(row_ptr, col, w, labels, *, stream=None):
    """One label-propagation sweep on one graph (device tensors); returns
    the new labels."""
    import torch
    lib = _load()
    n = row_ptr.numel() - 1
    g = Graph(n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"))
    lin = labels.to(torch.int32).contiguous()
    out = torch.empty_like(lin)
    rc = lib.mc_debug_lp_sweep(ctypes.byref(g), _dev_ptr(lin, torch.int32, "labels"),
                               ctypes.c_void_p(out.data_ptr()), _stream(stream))
    if rc != MC_OK:
        raise MincutError(rc, "mc_debug_lp_sweep")
    return out


def debug_pr_tests(row_ptr, col, w, lhat: int, max_deg: int = 64, *, stream=None):
    """Padberg-Rinaldi test outcomes per entry of one graph (device
    tensors): uint8 tensor of bits PR1 1, PR2 2, PR3 4, PR4 8."""
    import torch
    lib = _load()
    n = row_ptr.numel() - 1
    g = Graph(n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"))
    flags = torch.empty(max(col.numel(), 1), dtype=torch.uint8, device=row_ptr.device)
    rc = lib.mc_debug_pr_tests(ctypes.byref(g), _stream(stream), int(lhat), int(max_deg),
                               ctypes.c_void_p(flags.data_ptr()))
    if rc != MC_OK:
        raise MincutError(rc, "mc_debug_pr_tests")
    return flags[: col.numel()]


def debug_first_round(row_ptr, col, w, vtx_off, *, lhat_in=None, stream=None,
                      opts: Optional[Options] = None, **kw):
    """Union-find roots after the first round's tests and scans (blocks that
    round would contract) and the bound each graph used."""
    import torch
    lib = _load()
    voff = np.ascontiguousarray(np.asarray(vtx_off, dtype=np.int64))
    G = len(voff) - 1
    n = row_ptr.numel() - 1
    b = Batch(G, n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"),
              voff.ctypes.data_as(ctypes.c_void_p))
    o = opts if opts is not None else options(**kw)
    labels = torch.empty(max(n, 1), dtype=torch.int32, device=row_ptr.device)
    lh = np.zeros(G, np.int64)
    lin = None if lhat_in is None else np.ascontiguousarray(np.asarray(lhat_in, np.int64))
    rc = lib.mc_debug_first_round(ctypes.byref(b), _stream(stream), ctypes.byref(o),
                                  None if lin is None else lin.ctypes.data_as(ctypes.c_void_p),
                                  ctypes.c_void_p(labels.data_ptr()),
                                  lh.ctypes.data_as(ctypes.c_void_p))
    if rc != MC_OK:
        raise MincutError(rc, "mc_debug_first_round")
    return labels[:n], lh


def debug_contract(row_ptr, col, w, labels, n_new, *, stream=None):
    """The contraction kernels alone: (row_ptr, col, w) of the graph with
    every block of `labels` (int32 in [0, n_new)) contracted to one vertex."""
    import torch
    lib = _load()
    n = row_ptr.numel() - 1
    g = Graph(n, col.numel(), _dev_ptr(row_ptr, torch.int64, "row_ptr"),
              _dev_ptr(col, torch.int32, "col"), _dev_ptr(w, torch.int32, "w"))
    rp_o = torch.empty(n_new + 1, dtype=torch.int64, device=row_ptr.device)
    col_o = torch.empty(max(col.numel(), 1), dtype=torch.int32, device=row_ptr.device)
    w_o = torch.empty(max(col.numel(), 1), dtype=torch.int32, device=row_ptr.device)
    nnz = ctypes.c_int64(0)
    rc = lib.mc_debug_contract(ctypes.byref(g), _dev_ptr(labels, torch.int32, "labels"), n_new,
                               _stream(stream), ctypes.c_void_p(rp_o.data_ptr()),
                               ctypes.c_void_p(col_o.data_ptr()), ctypes.c_void_p(w_o.data_ptr()),
                               ctypes.byref(nnz))
    if rc != MC_OK:
        raise MincutError(rc, "mc_debug_contract")
    return rp_o, col_o[: nnz.value], w_o[: nnz.value]


def workspace_bytes(n_total: int, nnz_total: int, num_graphs: int = 1) -> int:
    return int(_load().mc_workspace_bytes(n_total, nnz_total, num_graphs))


def viecut_workspace_bytes(n_total: int, nnz_total: int, num_graphs: int = 1) -> int:
    return int(_load().mc_viecut_workspace_bytes(n_total, nnz_total, num_graphs))


def release():
    _load().mc_release()


def timing():
    lib = _load()
    arr = (TimingEntry * 64)()
    k = lib.mc_timing_get(arr, 64)
    return [{"name": arr[i].name.decode(), "launches": arr[i].launches, "ms": arr[i].ms,
             "algo_bytes": arr[i].algo_bytes} for i in range(min(k, 64))]


def timing_reset():
    _load().mc_timing_reset()


def timing_focus(name=None):
    """Time only the kernel class `name` (None: every class)."""
    _load().mc_timing_focus(name.encode() if name else None)


def to_device(g, device="cuda"):
    """Copy a host CSR (numpy arrays) to device tensors."""
    import torch
    return (torch.from_numpy(np.ascontiguousarray(g.row_ptr, np.int64)).to(device),
            torch.from_numpy(np.ascontiguousarray(g.col, np.int32)).to(device),
            torch.from_numpy(np.ascontiguousarray(g.w, np.int32)).to(device))
