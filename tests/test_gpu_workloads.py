"""GPU parity at the workloads' full sizes, in the configuration bench.py
times (default options, graph resident on the device): lambda equals the
stored oracle value (tests/golden/workloads.json, written by make_golden.py
with the sequential NOI oracle) and the returned side realises it."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import announce, check_side, solve

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


def _gold(name):
    return json.load(open(os.path.join(GOLDEN, "workloads.json")))[name]


def _single(name, make):
    gold = _gold(name)
    g = make()
    announce(name, g.n, g.m)
    assert (g.n, g.m) == (gold["n"], gold["m"]), "generator drifted"
    lam, side, st = solve(g)
    assert lam == gold["lambda"]
    check_side(g, lam, side)
    return st


def test_chung_lu_2_22_8core():
    _single("chung_lu_4m_8core", gg.chung_lu_4m_8core)


def test_batch_of_4096_graphs():
    import paper_1808_05458_amd as mc
    gold = _gold("batch_4096")
    graphs = [gg.batch_graph(i) for i in range(gold["graphs"])]
    packed, vo, eo = gg.pack(graphs)
    assert (packed.n, packed.m) == (gold["n"], gold["m"])
    announce("batch_4096", packed.n, packed.m)
    rp, col, w = mc.to_device(packed, "cuda")
    lams, sides, st = mc.mincut_batched(rp, col, w, vo)
    assert list(lams) == gold["lambdas"]
    s = sides.cpu().numpy()
    for i, g in enumerate(graphs):
        check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])


def test_rmat_scale20_10core():
    _single("rmat_20_10core", lambda: gg.rmat_24_10core(20, 24))


@pytest.mark.timeout(900)
def test_rmat_scale24_10core():
    # about 1.5 minutes of generation on the host, then the solve
    _single("rmat_24_10core", gg.rmat_24_10core)


@pytest.fixture(scope="module")
def bridged():
    gold = _gold("bridged_8cores_2^21_k3")
    g = gg.bridged_8cores(21, 3)
    assert (g.n, g.m) == (gold["n"], gold["m"]), "generator drifted"
    return g, gold


@pytest.mark.timeout(600)
@pytest.mark.parametrize("opts", [dict(), dict(sweep_tail=-1, sweep_pull=-1, emit_rows=-1, sweep_seg=-1),
                                  dict(sweep_pull=1, emit_rows=1), dict(sweep_pull=-1, sweep_seg=1)],
                         ids=["default", "sequential_tail_push_entry_emit", "pull_row_emit", "range_owned_push"])
def test_bridged_8cores_lambda_below_min_degree(bridged, opts):
    # two Chung-Lu 8-cores (about 2M vertices each) joined by 3 bridges: the
    # minimum cut (3) lies below the minimum degree (8), so the full-graph
    # sweeps, their grid-wide batches and the tail must keep the bridges
    # apart from everything else
    g, gold = bridged
    assert int(np.diff(g.row_ptr).min()) == 8 and gold["lambda"] == 3
    announce("bridged_8cores", g.n, g.m, opts)
    lam, side, st = solve(g, **opts)
    assert lam == gold["lambda"]
    check_side(g, lam, side)
