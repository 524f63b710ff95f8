"""GPU tests of the Padberg-Rinaldi triangle tests (PR3, PR4) and their use
in the solve: the per-entry outcomes of all four tests equal the oracle's bit
for bit (random graphs with parallel entries and rows out of order, the
row-length limit, workload shapes, several bounds), solves with the
triangle tests give the oracle's lambda with sides that realise it, and a
first round with them keeps lambda."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import announce, check_side, random_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_05458_amd as mc
    mc._load()
    yield


def _flags_equal(g, lhat, max_deg):
    import paper_1808_05458_amd as mc
    rp, col, w = mc.to_device(g, "cuda")
    got = mc.debug_pr_tests(rp, col, w, lhat, max_deg).cpu().numpy()
    want = oracle.pr_tests(g, lhat, max_deg)
    assert np.array_equal(got, want), (g.name, lhat, max_deg, np.flatnonzero(got != want)[:8])
    return want


def _shuffle_some_rows(g, rng):
    col, w = g.col.copy(), g.w.copy()
    for u in range(g.n):
        a, b = g.row_ptr[u], g.row_ptr[u + 1]
        if b - a > 1 and rng.random() < 0.3:
            p = rng.permutation(b - a)
            col[a:b], w[a:b] = col[a:b][p], w[a:b][p]
    return gg.Graph(g.n, g.row_ptr.copy(), col, w, g.name + "-shuffled")


def _sort_rows(g):
    col, w = g.col.copy(), g.w.copy()
    for u in range(g.n):
        a, b = g.row_ptr[u], g.row_ptr[u + 1]
        p = np.argsort(col[a:b], kind="stable")
        col[a:b], w[a:b] = col[a:b][p], w[a:b][p]
    return gg.Graph(g.n, g.row_ptr.copy(), col, w, g.name + "-sorted")


def test_flags_equal_oracle_on_random_graphs():
    rng = np.random.default_rng(606)
    seen = np.zeros(16, np.int64)
    for trial in range(300):
        n = int(rng.integers(2, 16))
        g = _sort_rows(random_graph(rng, n, float(rng.uniform(0.2, 1.0)), int(rng.choice([1, 2, 5, 30]))))
        if trial % 3 == 1:
            g = _shuffle_some_rows(g, rng)
        if trial % 5 == 2:  # parallel entries: the same edge listed twice
            e = np.concatenate([np.stack([g.src(), g.col], 1)[g.src() < g.col]] * 2)
            g = gg.from_edges(g.n, e, rng.integers(1, 4, size=len(e)), name="parallel")
        lam = oracle.bruteforce(g)[0] if g.n <= 14 else oracle.noi(g)[0]
        for lhat in (max(lam, 1), lam + 3):
            for max_deg in (3, 64, 100):
                f = _flags_equal(g, lhat, max_deg)
                np.add.at(seen, f, 1)
    # every combination of the four bits that occurs is compared; PR3 and PR4
    # both occurred
    assert seen[4:].sum() > 0 and seen[8:].sum() > 0


def test_flags_equal_oracle_on_workload_shapes():
    for g in [gg.planted_4096(), gg.batch_graph(7), gg.batch_graph(311),
              gg.chung_lu(9, 1 << 13, avg_deg=16.0, wmin=1, wmax=9, name="cl13")]:
        lam = oracle.noi(g, 1)[0]
        for lhat in (lam, lam + 10):
            announce("pr flags", g.name, lhat)
            _flags_equal(g, lhat, 64)
            _flags_equal(g, lhat, 100)
        # a contracted graph (sorted rows, summed parallel edges)
        lab = np.arange(g.n) // 3
        h, _ = oracle.contract(g, lab)
        _flags_equal(h, lam + 5, 64)


def test_solves_with_triangle_tests_equal_oracle():
    import paper_1808_05458_amd as mc
    graphs = [gg.batch_graph(i) for i in range(160)]
    refs = [oracle.noi(g, 5)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for opts in [dict(pr_triangle_deg=-64), dict(pr_triangle_deg=16, scan_mode=2),
                 dict(pr_triangle_deg=-64, whole_max=64), dict(pr_triangle_deg=-100), dict(pr_triangle_deg=0)]:
        announce("pr34 batch", opts)
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, **opts)
        assert list(lams) == refs, opts
        s = sides.cpu().numpy()
        for i, g in enumerate(graphs):
            check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])
    for g in [gg.planted_4096(), gg.chung_lu(9, 1 << 13, avg_deg=16.0, wmin=1, wmax=9, name="cl13")]:
        lam = oracle.noi(g, 1)[0]
        rp, col, w = mc.to_device(g, "cuda")
        for opts in [dict(pr_triangle_deg=-64), dict(pr_triangle_deg=-64, whole_max=16), dict(pr_triangle_deg=0)]:
            announce("pr34", g.name, opts)
            got, side, st = mc.mincut(rp, col, w, **opts)
            assert got == lam
            check_side(g, got, side.cpu().numpy()[: g.n])


def test_first_round_with_triangle_tests_keeps_lambda():
    # bounds above lambda: the round's unions (PR1-PR4 and scans together)
    # must leave a graph whose minimum cut is still lambda (the starting
    # bound is the smaller of the caller's and the minimum degree)
    import paper_1808_05458_amd as mc
    graphs = [gg.batch_graph(i) for i in range(120, 150)]
    lams = [oracle.noi(g, 5)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for margin in (1, 20, 200):
        announce("pr34 round", margin)
        lin = [l + margin for l in lams]
        labels, used = mc.debug_first_round(rp, col, w, vo, lhat_in=lin, pr_triangle_deg=-64)
        lab = labels.cpu().numpy()
        checked = 0
        for i, g in enumerate(graphs):
            h, _ = oracle.contract(g, lab[vo[i]:vo[i + 1]])
            assert used[i] <= lin[i]
            # a bound equal to lambda is already the answer (the minimum
            # degree or the caller's bound): then any contraction is allowed
            if lams[i] < used[i]:
                assert h.n >= 2, (i, margin)
                assert oracle.noi(h, 1)[0] == lams[i], (i, margin)
                checked += 1
        assert checked >= 8  # graphs whose minimum cut is below their minimum degree
