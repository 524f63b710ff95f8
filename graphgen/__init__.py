"""Seeded synthetic graphs shaped like the paper's workloads.

The paper evaluates on random hyperbolic graphs and on k-cores of web and
social graphs (appendix, "Instances"); neither generator nor data is
available here, so these stand-ins are used: planted clusters (community
structure), Chung-Lu and R-MAT (heavy-tailed degrees), followed by the
paper's own preparation (k-core, then the largest connected component).

Nothing here computes any part of the minimum-cut method.  The heavy lifting
is in ``graphgen.cpp`` (built into ``libgraphgen.so``); all randomness is
counter-based and seeded, so every machine produces the same graphs.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")


def build(force: bool = True) -> str:
    """Compile the generator library with g++ (OpenMP)."""
    if force or not os.path.exists(_LIB):
        cmd = ["g++", "-O3", "-std=c++17", "-fopenmp", "-shared", "-fPIC",
               _SRC, "-o", _LIB + ".tmp"]
        subprocess.check_call(cmd)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Csr(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.POINTER(ctypes.c_int64)),
                ("col", ctypes.POINTER(ctypes.c_int32)),
                ("w", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.POINTER(_Csr)
        lib.gg_planted.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, P]
        lib.gg_chung_lu.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, P]
        lib.gg_rmat.argtypes = [ctypes.c_uint64, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                ctypes.c_int32, ctypes.c_int32, P]
        lib.gg_structured.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64,
                                      ctypes.c_int32, ctypes.c_int32, P]
        lib.gg_free.argtypes = [P]
        for f in (lib.gg_planted, lib.gg_chung_lu, lib.gg_rmat, lib.gg_structured):
            f.restype = ctypes.c_int
        _lib = lib
    return _lib


@dataclass
class Graph:
    """Symmetric CSR: row_ptr int64[n+1], col int32[nnz], w int32[nnz]."""
    n: int
    row_ptr: np.ndarray
    col: np.ndarray
    w: np.ndarray
    name: str = ""

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Undirected edge count (each edge is stored in both rows)."""
        return self.nnz // 2

    def src(self) -> np.ndarray:
        return np.repeat(np.arange(self.n, dtype=np.int32), np.diff(self.row_ptr))


def _take(call, name) -> Graph:
    lib = _load()
    out = _Csr()
    rc = call(ctypes.byref(out))
    if rc != 0:
        raise RuntimeError(f"graph generator failed ({name}): code {rc}")
    try:
        n, nnz = int(out.n), int(out.nnz)
        rp = np.ctypeslib.as_array(out.row_ptr, shape=(n + 1,)).copy()
        col = np.ctypeslib.as_array(out.col, shape=(max(nnz, 1),))[:nnz].copy()
        w = np.ctypeslib.as_array(out.w, shape=(max(nnz, 1),))[:nnz].copy()
    finally:
        lib.gg_free(ctypes.byref(out))
    return Graph(n, rp, col, w, name)


def planted(seed, n, k, p, inter_total=0, inter_min=1, inter_max=4, wmin=1, wmax=10,
            name="planted") -> Graph:
    lib = _load()
    return _take(lambda o: lib.gg_planted(seed, n, k, p, inter_total, inter_min, inter_max,
                                          wmin, wmax, o), name)


def chung_lu(seed, n, beta=2.5, avg_deg=16.0, wmin=1, wmax=1, kcore=0, lcc=True,
             name="chung_lu") -> Graph:
    lib = _load()
    return _take(lambda o: lib.gg_chung_lu(seed, n, beta, avg_deg, wmin, wmax, kcore,
                                           int(lcc), o), name)


def rmat(seed, scale, draws, a=0.57, b=0.19, c=0.19, kcore=0, lcc=True, name="rmat") -> Graph:
    lib = _load()
    return _take(lambda o: lib.gg_rmat(seed, scale, draws, a, b, c, kcore, int(lcc), o), name)


def complete(n, w=1) -> Graph:
    lib = _load()
    return _take(lambda o: lib.gg_structured(0, n, 0, w, w, o), f"K{n}")


def cycle(n, seed, wmin=1, wmax=10) -> Graph:
    lib = _load()
    return _take(lambda o: lib.gg_structured(1, n, seed, wmin, wmax, o), f"C{n}")


def two_cliques(a, k) -> Graph:
    lib = _load()
    return _take(lambda o: lib.gg_structured(2, 2 * a, 0, k, k, o), f"2K{a}+{k}")


def from_edges(n, edges, weights=None, name="edges") -> Graph:
    """Symmetric CSR from an undirected edge list (duplicates kept as given)."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    wt = np.ones(len(e), np.int64) if weights is None else np.asarray(weights, np.int64)
    src = np.concatenate([e[:, 0], e[:, 1]])
    dst = np.concatenate([e[:, 1], e[:, 0]])
    ww = np.concatenate([wt, wt])
    order = np.lexsort((dst, src))
    src, dst, ww = src[order], dst[order], ww[order]
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, src + 1, 1)
    rp = np.cumsum(rp)
    return Graph(n, rp, dst.astype(np.int32), ww.astype(np.int32), name)


# --------------------------------------------------------------------------
# Workload recipes.  Each is seeded; sizes follow the workload descriptions.

def _u01(seed: int, i: int) -> float:
    """SplitMix64-based uniform in [0,1) for recipe parameters."""
    z = (seed * 0x9E3779B97F4A7C15 + (i + 1) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = (z + 0x9E3779B97F4A7C15) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    z ^= z >> 31
    return (z >> 11) * 2.0 ** -53


def planted_4096() -> Graph:
    """8 clusters of 512, intra-cluster G(512, 0.04), 64 inter-cluster edges,
    weights uniform in [1, 10], seed 1."""
    return planted(1, 4096, 8, 0.04, inter_total=64, wmin=1, wmax=10, name="planted_4096")


def chung_lu_4m_8core(n_log2: int = 22) -> Graph:
    """Chung-Lu, n = 2^22, exponent 2.5, average degree 32, unit weights,
    8-core, largest component, seed 2."""
    return chung_lu(2, 1 << n_log2, 2.5, 32.0, 1, 1, kcore=8, lcc=True,
                    name=f"chung_lu_2^{n_log2}_8core")


def rmat_24_10core(scale: int = 24, draws_log2: int = 28) -> Graph:
    """R-MAT scale 24, 2^28 draws, (0.57, 0.19, 0.19, 0.05), multiplicity
    weights, 10-core, largest component, seed 3."""
    return rmat(3, scale, 1 << draws_log2, 0.57, 0.19, 0.19, kcore=10, lcc=True,
                name=f"rmat_{scale}_10core")


def batch_graph_params(g: int):
    """(n, clusters, intra degree) of graph g of the 4096-graph batch."""
    s = 4_000_000 + g
    n = int(round(math.exp(math.log(64) + _u01(s, 0) * (math.log(8192) - math.log(64)))))
    k = 2 + int(_u01(s, 1) * 15)
    d = 8.0 + _u01(s, 2) * 24.0
    return max(n, 2 * k), k, d


def batch_graph(g: int) -> Graph:
    """Graph g of the batch: planted clusters, n log-uniform in [64, 8192],
    2-16 clusters, intra degree uniform in [8, 32], 1-4 inter edges per
    cluster pair, weights in [1, 100]."""
    n, k, d = batch_graph_params(g)
    return planted(4_000_000 + g, n, k, -d, inter_total=0, inter_min=1, inter_max=4,
                   wmin=1, wmax=100, name=f"batch_{g}")


def served_request_params(i: int):
    s = 5_000_000 + i
    n = int(round(math.exp(math.log(2 ** 10) + _u01(s, 0) * (math.log(2 ** 20) - math.log(2 ** 10)))))
    return n


def served_request(i: int) -> Graph:
    """Request i of the served stream: Chung-Lu, exponent 2.5, average degree
    16, n log-uniform in [2^10, 2^20], weights in [1, 50], largest component."""
    n = served_request_params(i)
    return chung_lu(5_000_000 + i, n, 2.5, 16.0, 1, 50, kcore=0, lcc=True, name=f"served_{i}")


def pack(graphs):
    """Disjoint union as one CSR with global vertex ids, plus vertex and
    entry offsets per graph."""
    ns = [g.n for g in graphs]
    nz = [g.nnz for g in graphs]
    vo = np.zeros(len(graphs) + 1, np.int64)
    vo[1:] = np.cumsum(ns)
    eo = np.zeros(len(graphs) + 1, np.int64)
    eo[1:] = np.cumsum(nz)
    rp = np.zeros(vo[-1] + 1, np.int64)
    col = np.empty(eo[-1], np.int32)
    w = np.empty(eo[-1], np.int32)
    for i, g in enumerate(graphs):
        rp[vo[i]:vo[i + 1] + 1] = g.row_ptr + eo[i]
        col[eo[i]:eo[i + 1]] = g.col + vo[i]
        w[eo[i]:eo[i + 1]] = g.w
    return Graph(int(vo[-1]), rp, col, w, "packed"), vo, eo
