"""CPU oracle for the exact global minimum cut (test infrastructure only).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never calls it and
shares no code with it.

Routes (see ``oracle.cpp`` for the passages each follows):
  bruteforce(g)        O1, enumeration of all sides (n <= 26)
  pair_connectivity(g) lambda(G, s, t) for all pairs by enumeration (n <= 20)
  stoer_wagner(g)      O2
  noi(g, seed)         O3, sequential Nagamochi-Ono-Ibaraki
  viecut(g, ...)       VieCut-style upper bound (Algorithm 2, first step)
  lp_sweep(g, labels)  its label-propagation step
  cut_value(g, side)   c(A) by definition
  contract(g, labels)  G with every block of `labels` contracted to one
                       vertex (Preliminaries, contraction G/(u,v)), numpy
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", _SRC,
                               "-o", _LIB + ".tmp"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp = ctypes.c_void_p
        lib.mco_cut_value.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.mco_bruteforce.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.mco_pair_connectivity.argtypes = [ctypes.c_int32, vp, vp, vp, vp]
        lib.mco_stoer_wagner.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
        lib.mco_noi.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_uint64, vp, vp, vp]
        lib.mco_matula.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_uint64, ctypes.c_int64, vp, vp, vp]
        lib.mco_pr_tests.argtypes = [ctypes.c_int32, vp, vp, vp, ctypes.c_int64, ctypes.c_int32, vp]
        lib.mco_lp_sweep.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp]
        i32 = ctypes.c_int32
        lib.mco_viecut.argtypes = [i32, vp, vp, vp, i32, i32, i32, i32, vp, vp, vp]
        _lib = lib
    return _lib


def _arrs(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    col = np.ascontiguousarray(g.col, dtype=np.int32)
    w = np.ascontiguousarray(g.w, dtype=np.int32)
    return rp, col, w


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def cut_value(g, side) -> int:
    rp, col, w = _arrs(g)
    s = np.ascontiguousarray(side, dtype=np.uint8)
    out = np.zeros(1, np.int64)
    _check(_load().mco_cut_value(g.n, _p(rp), _p(col), _p(w), _p(s), _p(out)), "cut_value")
    return int(out[0])


def bruteforce(g):
    rp, col, w = _arrs(g)
    lam = np.zeros(1, np.int64)
    side = np.zeros(g.n, np.uint8)
    _check(_load().mco_bruteforce(g.n, _p(rp), _p(col), _p(w), _p(lam), _p(side)), "bruteforce")
    return int(lam[0]), side


def pair_connectivity(g) -> np.ndarray:
    rp, col, w = _arrs(g)
    conn = np.zeros(g.n * g.n, np.int64)
    _check(_load().mco_pair_connectivity(g.n, _p(rp), _p(col), _p(w), _p(conn)),
           "pair_connectivity")
    return conn.reshape(g.n, g.n)


def stoer_wagner(g):
    rp, col, w = _arrs(g)
    lam = np.zeros(1, np.int64)
    side = np.zeros(g.n, np.uint8)
    _check(_load().mco_stoer_wagner(g.n, _p(rp), _p(col), _p(w), _p(lam), _p(side)),
           "stoer_wagner")
    return int(lam[0]), side


def noi(g, seed: int = 0):
    rp, col, w = _arrs(g)
    lam = np.zeros(1, np.int64)
    side = np.zeros(g.n, np.uint8)
    rounds = np.zeros(1, np.int32)
    _check(_load().mco_noi(g.n, _p(rp), _p(col), _p(w), ctypes.c_uint64(seed), _p(lam),
                           _p(side), _p(rounds)), "noi")
    return int(lam[0]), side, int(rounds[0])


def pr_tests(g, lhat: int, max_deg: int = 64):
    """Padberg-Rinaldi tests per entry (u, v), u < v: uint8 bits PR1 (1),
    PR2 (2), PR3 (4), PR4 (8); 0 for the other entries."""
    rp, col, w = _arrs(g)
    flags = np.zeros(len(col), np.uint8)
    _check(_load().mco_pr_tests(g.n, _p(rp), _p(col), _p(w), int(lhat), int(max_deg), _p(flags)), "pr_tests")
    return flags


def matula(g, eps_ppm: int, seed: int = 0):
    """Matula's (2+eps)-approximation, eps = eps_ppm / 10^6: (cut value, side,
    rounds); the value is a real cut of g."""
    rp, col, w = _arrs(g)
    lam = np.zeros(1, np.int64)
    side = np.zeros(g.n, np.uint8)
    rounds = np.zeros(1, np.int32)
    _check(_load().mco_matula(g.n, _p(rp), _p(col), _p(w), ctypes.c_uint64(seed), int(eps_ppm), _p(lam),
                              _p(side), _p(rounds)), "matula")
    return int(lam[0]), side, int(rounds[0])


def lp_sweep(g, labels):
    """One synchronous label-propagation sweep: each vertex takes the
    neighbour label of largest total weight, ties to the smallest label."""
    rp, col, w = _arrs(g)
    lin = np.ascontiguousarray(labels, dtype=np.int32)
    out = np.zeros(g.n, np.int32)
    _check(_load().mco_lp_sweep(g.n, _p(rp), _p(col), _p(w), _p(lin), _p(out)), "lp_sweep")
    return out


def viecut(g, sweeps: int = 2, stop_n: int = 2, max_levels: int = 32, exact_finish: bool = False):
    """VieCut-style upper bound: (lambda-hat, side, levels); exact_finish
    solves the last level graph exactly."""
    rp, col, w = _arrs(g)
    lam = np.zeros(1, np.int64)
    side = np.zeros(g.n, np.uint8)
    levels = np.zeros(1, np.int32)
    _check(_load().mco_viecut(g.n, _p(rp), _p(col), _p(w), sweeps, stop_n, max_levels, int(exact_finish),
                              _p(lam), _p(side), _p(levels)), "viecut")
    return int(lam[0]), side, int(levels[0])


def contract(g, labels):
    """Contract every block of `labels` (any integer per vertex; equal values
    form a block) into one vertex: parallel edges summed, edges inside a block
    dropped (Preliminaries, contraction G/(u,v)).  Returns (graph, block id
    per vertex); blocks are numbered in order of their smallest label."""
    import graphgen as gg
    lab = np.asarray(labels)
    uniq, blk = np.unique(lab, return_inverse=True)
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    a, b = blk[src], blk[g.col]
    keep = a < b
    if not keep.any():
        return gg.Graph(len(uniq), np.zeros(len(uniq) + 1, np.int64), np.zeros(0, np.int32),
                        np.zeros(0, np.int32), "contracted"), blk
    pairs = np.stack([a[keep], b[keep]], 1)
    keys, inv = np.unique(pairs, axis=0, return_inverse=True)
    wsum = np.zeros(len(keys), np.int64)
    np.add.at(wsum, inv.reshape(-1), g.w[keep].astype(np.int64))
    return gg.from_edges(len(uniq), keys, wsum, name="contracted"), blk
