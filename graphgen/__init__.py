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


def _cached(name: str, make) -> Graph:
    """make(), or its copy saved under $MC_GRAPH_CACHE when that is set
    (plain .npy arrays; several runs of one command reuse a large graph)."""
    d = os.environ.get("MC_GRAPH_CACHE")
    if not d:
        return make()
    paths = [os.path.join(d, f"{name}.{k}.npy") for k in ("row_ptr", "col", "w")]
    if all(os.path.exists(q) for q in paths):
        rp, col, w = (np.load(q, allow_pickle=False) for q in paths)
        return Graph(len(rp) - 1, rp, col, w, name)
    g = make()
    os.makedirs(d, exist_ok=True)
    for q, arr in zip(paths, (g.row_ptr, g.col, g.w)):
        np.save(q + ".tmp.npy", arr, allow_pickle=False)
        os.replace(q + ".tmp.npy", q)
    return g


def planted_4096() -> Graph:
    """8 clusters of 512, intra-cluster G(512, 0.04), 64 inter-cluster edges,
    weights uniform in [1, 10], seed 1."""
    return planted(1, 4096, 8, 0.04, inter_total=64, wmin=1, wmax=10, name="planted_4096")


def chung_lu_4m_8core(n_log2: int = 22) -> Graph:
    """Chung-Lu, n = 2^22, exponent 2.5, average degree 32, unit weights,
    8-core, largest component, seed 2."""
    name = f"chung_lu_2^{n_log2}_8core"
    return _cached(name, lambda: chung_lu(2, 1 << n_log2, 2.5, 32.0, 1, 1, kcore=8, lcc=True, name=name))


def rmat_24_10core(scale: int = 24, draws_log2: int = 28) -> Graph:
    """R-MAT scale 24, 2^28 draws, (0.57, 0.19, 0.19, 0.05), multiplicity
    weights, 10-core, largest component, seed 3."""
    name = f"rmat_{scale}_10core"
    return _cached(name, lambda: rmat(3, scale, 1 << draws_log2, 0.57, 0.19, 0.19, kcore=10, lcc=True,
                                      name=name))


def _mix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 finaliser, elementwise on uint64."""
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def bridged_8cores(n_log2: int = 21, k: int = 3) -> Graph:
    """Two Chung-Lu graphs (n = 2^n_log2 each, exponent 2.5, average degree
    32, unit weights, seeds 6 and 7), each reduced to its 8-core and largest
    component, joined by k unit edges whose 2k endpoints are distinct, then
    every vertex id permuted (seed 8).  For k below 8 the minimum cut is the
    k bridges and lies below the minimum degree 8 (unless a half has a
    smaller cut of its own: the oracle decides)."""
    name = f"bridged_8cores_2^{n_log2}_k{k}"

    def make():
        a = chung_lu(6, 1 << n_log2, 2.5, 32.0, 1, 1, kcore=8, lcc=True)
        b = chung_lu(7, 1 << n_log2, 2.5, 32.0, 1, 1, kcore=8, lcc=True)
        n = a.n + b.n
        # bridge endpoints: the first k distinct picks on each side
        ends = []
        for side, h, off in ((0, a, 0), (1, b, a.n)):
            picks, i = [], 0
            while len(picks) < k:
                v = int(_mix64(np.array([8_000_000 + 1000 * side + i], np.uint64))[0] % np.uint64(h.n))
                if v not in picks:
                    picks.append(v)
                i += 1
            ends.append([off + v for v in picks])
        perm = np.argsort(_mix64(np.arange(n, dtype=np.uint64) + np.uint64(8 << 40)), kind="stable")
        src = np.concatenate([a.src(), b.src() + a.n, ends[0], ends[1]]).astype(np.int64)
        dst = np.concatenate([a.col, b.col + a.n, ends[1], ends[0]]).astype(np.int64)
        key = np.sort((perm[src] << 32) | perm[dst])
        del src, dst
        s2 = (key >> 32).astype(np.int32)
        col = (key & 0xFFFFFFFF).astype(np.int32)
        rp = np.zeros(n + 1, np.int64)
        rp[1:] = np.cumsum(np.bincount(s2, minlength=n))
        return Graph(n, rp, col, np.ones(len(col), np.int32), name)
    return _cached(name, make)


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
