"""GPU parity of the clustering upper bound (VieCut-style, the first step of
Algorithm 2): one label-propagation sweep equals the oracle's label for
label, the bound equals the oracle's bound exactly (both are deterministic:
synchronous sweeps with ties to the smallest label, fixed block numbering),
its side realises it, and the exact solve started from it still returns
the oracle's lambda."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import announce, check_side, random_graph

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_05458_amd as mc
    mc._load()
    yield


def _hub_graph(seed, n, hubs, hub_deg, extra, wmax):
    """`hubs` vertices joined to `hub_deg` random others each, plus `extra`
    random edges and a random path through all vertices; weights uniform in
    [1, wmax]; parallel entries kept."""
    rng = np.random.default_rng(seed)
    e = []
    for h in range(hubs):
        nb = rng.choice(np.arange(hubs, n), size=hub_deg, replace=False)
        e.append(np.stack([np.full(hub_deg, h), nb], 1))
    e.append(rng.integers(0, n, size=(extra, 2)))
    perm = rng.permutation(n)  # a path through every vertex keeps it connected
    e.append(np.stack([perm[:-1], perm[1:]], 1))
    e = np.concatenate(e)
    e = e[e[:, 0] != e[:, 1]]
    return gg.from_edges(n, e, rng.integers(1, wmax + 1, size=len(e)), name=f"hubs{hubs}x{hub_deg}")


def _lp_cases():
    rng = np.random.default_rng(31)
    cases = []
    for t in range(40):
        n = int(rng.integers(2, 60))
        g = random_graph(rng, n, float(rng.uniform(0.05, 0.9)), int(rng.choice([1, 4, 90])),
                         connected=bool(rng.random() < 0.8))
        cases.append((g, rng.integers(0, n, size=n)))
    # self-loops and parallel entries
    g = gg.from_edges(5, [(0, 0), (0, 1), (0, 1), (1, 2), (2, 3), (3, 3), (3, 4)], [50, 2, 2, 3, 1, 9, 1])
    cases.append((g, np.arange(5)))
    for i in (3, 140, 2000):
        g = gg.batch_graph(i)
        cases.append((g, np.arange(g.n)))
        cases.append((g, rng.integers(0, max(2, g.n // 50), size=g.n)))
    g = gg.chung_lu(7, 1 << 16, 2.5, 32.0, 1, 20, kcore=0, lcc=True)  # rows up to ~1400 entries
    cases.append((g, np.arange(g.n)))
    # rows longer than one workgroup pass (4096 entries): 2 to 5 passes
    g = _hub_graph(5, 30000, 3, 19000, 60000, 7)
    cases.append((g, np.arange(g.n)))
    cases.append((g, rng.integers(0, 25000, size=g.n)))
    cases.append((g, rng.integers(0, 3, size=g.n)))
    return cases


def test_lp_sweep_equals_oracle():
    import torch
    import paper_1808_05458_amd as mc
    for g, lab in _lp_cases():
        announce("lp sweep", g.name, g.n, g.nnz, int(np.diff(g.row_ptr).max()))
        rp, col, w = mc.to_device(g, "cuda")
        out = mc.debug_lp_sweep(rp, col, w, torch.from_numpy(lab.astype(np.int32)).cuda()).cpu().numpy()
        ref = oracle.lp_sweep(g, lab)
        assert np.array_equal(out, ref), (g.name, np.flatnonzero(out != ref)[:8])


def _bounds_equal(graphs, sweeps=2, stop=2, levels=32, exact=False, **extra):
    import paper_1808_05458_amd as mc
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    announce("viecut bound", len(graphs), packed.n, packed.m, sweeps, stop, levels, exact)
    bounds, sides, lv = mc.viecut_bound(rp, col, w, vo, lp_sweeps=sweeps, viecut_stop=stop,
                                        viecut_levels=levels, viecut_exact=int(exact), **extra)
    s = sides.cpu().numpy()
    most = 0
    for i, g in enumerate(graphs):
        b, _, l = oracle.viecut(g, sweeps=sweeps, stop_n=stop, max_levels=levels, exact_finish=exact)
        assert bounds[i] == b, (i, g.name, bounds[i], b)
        check_side(g, b, s[vo[i]:vo[i + 1]])
        most = max(most, l)
    assert lv == most
    return bounds


def test_viecut_hand_examples():
    spec = json.load(open(os.path.join(GOLDEN, "lp_examples.json")))
    graphs = []
    for ex in spec["bounds"]:
        if isinstance(ex["edges"], str):
            kind, *args = ex["edges"].split()
            graphs.append(gg.two_cliques(*map(int, args)) if kind == "two_cliques" else gg.complete(int(args[0])))
        else:
            e = np.array(ex["edges"])
            graphs.append(gg.from_edges(ex["n"], e[:, :2], e[:, 2]))
    for stop in sorted({ex.get("stop_n", 2) for ex in spec["bounds"]}):
        idx = [i for i, ex in enumerate(spec["bounds"]) if ex.get("stop_n", 2) == stop]
        b = _bounds_equal([graphs[i] for i in idx], stop=stop)
        assert list(b) == [spec["bounds"][i]["bound"] for i in idx]


def test_viecut_bound_batch_recipe():
    graphs = [gg.batch_graph(i) for i in range(0, 4096, 13)]
    _bounds_equal(graphs)


@pytest.mark.parametrize("sweeps,stop,levels", [(1, 2, 32), (3, 2, 32), (2, 64, 32), (2, 2, 1), (0, 2, 4)])
def test_viecut_bound_options(sweeps, stop, levels):
    graphs = [gg.batch_graph(i) for i in range(100, 160)]
    _bounds_equal(graphs, sweeps=sweeps, stop=stop, levels=levels)


def test_viecut_bound_mixed_shapes():
    rng = np.random.default_rng(8)
    graphs = [gg.planted_4096(), gg.two_cliques(9, 2), gg.complete(5),
              gg.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)]),  # disconnected: 0
              gg.from_edges(2, [(0, 1)], [9])]
    graphs += [random_graph(rng, int(rng.integers(3, 40)), 0.3, 20) for _ in range(30)]
    graphs.append(gg.chung_lu(9, 1 << 15, 2.5, 16.0, 1, 50, kcore=0, lcc=True))
    graphs.append(_hub_graph(6, 12000, 2, 9000, 30000, 40))
    _bounds_equal(graphs)


def test_exact_solve_from_viecut_bound():
    import paper_1808_05458_amd as mc
    graphs = [gg.batch_graph(i) for i in range(160)]
    refs = [oracle.noi(g, 5)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for opts in [dict(use_viecut=1), dict(use_viecut=1, scan_mode=2), dict(use_viecut=1, use_pr=0)]:
        announce("batch with viecut", opts)
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, **opts)
        s = sides.cpu().numpy()
        assert list(lams) == refs, opts
        for i, g in enumerate(graphs):
            check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])
    for g in [gg.planted_4096(), gg.chung_lu(9, 1 << 15, 2.5, 16.0, 1, 50, kcore=0, lcc=True),
              gg.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)])]:
        announce("single with viecut", g.name)
        rp, col, w = mc.to_device(g, "cuda")
        lam, side, st = mc.mincut(rp, col, w, use_viecut=1)
        assert lam == oracle.noi(g, 3)[0]
        assert st["lambda_viecut"] >= lam
        check_side(g, lam, side.cpu().numpy()[: g.n])


@pytest.mark.parametrize("stop,levels", [(64, 32), (2, 32), (256, 2), (16, 1)])
def test_viecut_exact_finish(stop, levels):
    # the last level graph of every graph solved exactly: graphs stop at
    # different levels, and those that stop early stay in the later level
    # graphs as they are
    graphs = [gg.batch_graph(i) for i in range(40, 160)] + [gg.planted_4096()]
    _bounds_equal(graphs, stop=stop, levels=levels, exact=True)


def test_viecut_exact_finish_mixed_shapes():
    rng = np.random.default_rng(18)
    graphs = [gg.two_cliques(9, 2), gg.complete(5), gg.from_edges(2, [(0, 1)], [9]),
              gg.from_edges(6, [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5)])]  # disconnected: 0
    graphs += [random_graph(rng, int(rng.integers(3, 40)), 0.3, 20) for _ in range(30)]
    graphs.append(gg.chung_lu(9, 1 << 15, 2.5, 16.0, 1, 50, kcore=0, lcc=True))
    bounds = _bounds_equal(graphs, stop=32, exact=True)
    # the exact finish reaches lambda where the levels stopped above it
    lams = [oracle.noi(g, 1)[0] for g in graphs]
    assert all(b >= l for b, l in zip(bounds, lams))
