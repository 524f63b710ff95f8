"""GPU tests of Matula's (2+eps)-approximation mode (approx_ppm): the answer
is a real cut (the side realises it) between lambda and the bound
lambda / (1/2 - eps); where lambda equals the minimum degree it is
exact; it never needs more rounds than the exact loop.  Several answers are
correct, so the oracle's own approximation is not compared value for value;
lambda comes from the exact oracle."""
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


def bound(lam, ppm):
    # lambda / (1/2 - eps), the guarantee of the paper's threshold
    return lam * 2_000_000 // (1_000_000 - 2 * ppm)


def _check_all(graphs, exact, vo, lams, sides, ppm):
    s = sides.cpu().numpy()
    for i, g in enumerate(graphs):
        a = int(lams[i])
        assert exact[i] <= a <= bound(exact[i], ppm), (g.name, exact[i], a)
        check_side(g, a, s[vo[i]:vo[i + 1]])


@pytest.mark.parametrize("ppm", [1, 100_000, 250_000, 490_000])
def test_random_graphs_packed(ppm):
    import paper_1808_05458_amd as mc
    rng = np.random.default_rng(31 + ppm % 101)
    graphs = [random_graph(rng, int(rng.integers(2, 15)), float(rng.uniform(0.15, 1.0)),
                           int(rng.choice([1, 3, 20, 100]))) for _ in range(300)]
    exact = [oracle.bruteforce(g)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    announce("matula random", ppm, len(graphs))
    lams, sides, st = mc.mincut_batched(rp, col, w, vo, approx_ppm=ppm)
    _check_all(graphs, exact, vo, lams, sides, ppm)


def test_fixtures_where_a_floor_threshold_breaks_the_bound():
    import paper_1808_05458_amd as mc
    fx = json.load(open(os.path.join(GOLDEN, "matula_examples.json")))["examples"]
    graphs = [gg.from_edges(ex["n"], ex["edges"], ex["weights"]) for ex in fx]
    exact = [oracle.bruteforce(g)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for ppm in sorted({ex["ppm"] for ex in fx}):
        announce("matula fixtures", ppm)
        for seed in (1, 2, 3):
            lams, sides, st = mc.mincut_batched(rp, col, w, vo, approx_ppm=ppm, seed=seed)
            _check_all(graphs, exact, vo, lams, sides, ppm)


def test_batch_sample_within_bound():
    import paper_1808_05458_amd as mc
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))["batch_4096"]["lambdas"]
    graphs = [gg.batch_graph(i) for i in range(200)]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for ppm in (100_000, 400_000):
        announce("matula batch", ppm)
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, approx_ppm=ppm)
        _check_all(graphs, gold[:200], vo, lams, sides, ppm)


@pytest.mark.parametrize("opts", [dict(), dict(whole_max=16), dict(use_pr=0), dict(scan_mode=2)])
def test_single_graphs_and_paths(opts):
    import paper_1808_05458_amd as mc
    for g in [gg.planted_4096(), gg.chung_lu(5, 1 << 14, avg_deg=16.0, wmin=1, wmax=20, name="cl14")]:
        lam = oracle.noi(g, 1)[0]
        rp, col, w = mc.to_device(g, "cuda")
        exact, _, st_e = mc.mincut(rp, col, w, **opts)
        assert exact == lam
        for ppm in (100_000, 300_000):
            announce("matula", g.name, opts, ppm)
            a, side, st = mc.mincut(rp, col, w, approx_ppm=ppm, **opts)
            assert lam <= a <= bound(lam, ppm)
            check_side(g, a, side.cpu().numpy()[: g.n])
            assert st["rounds"] <= st_e["rounds"] + 1


def test_exact_where_lambda_is_the_min_degree():
    # Chung-Lu 2^19 8-core: lambda = minimum degree = 8
    import paper_1808_05458_amd as mc
    g = gg.chung_lu_4m_8core(19)
    rp, col, w = mc.to_device(g, "cuda")
    announce("matula chung-lu 2^19")
    a, side, st = mc.mincut(rp, col, w, approx_ppm=100_000)
    assert a == 8
    check_side(g, a, side.cpu().numpy()[: g.n])


def test_rejects_eps_out_of_range():
    import paper_1808_05458_amd as mc
    g = gg.complete(5)
    rp, col, w = mc.to_device(g, "cuda")
    for ppm in (-1, 500_000):
        with pytest.raises(mc.MincutError) as e:
            mc.mincut(rp, col, w, approx_ppm=ppm)
        assert e.value.code == mc.MC_EINVAL
