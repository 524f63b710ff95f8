"""Pins for the CPU oracle against facts fixed by the mathematics.

Each route (O1 enumeration, O2 Stoer-Wagner, O3 sequential NOI) is checked
against closed forms of textbook graphs, hand-worked fixtures, invariants of
the minimum cut (lambda <= minimum weighted degree, scaling, relabelling,
monotonicity under edge insertion and contraction) and against each other on
thousands of random tiny graphs.  A dropped term, a wrong sign or a
transposed index in any route breaks one of these.
"""
import itertools
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ROUTES = {
    "bruteforce": lambda g: oracle.bruteforce(g)[:2],
    "stoer_wagner": lambda g: oracle.stoer_wagner(g)[:2],
    "noi": lambda g: oracle.noi(g, 7)[:2],
}


def min_degree(g):
    deg = np.zeros(g.n, np.int64)
    src = g.src()
    keep = src != g.col
    np.add.at(deg, src[keep], g.w[keep])
    return int(deg.min())


def check_side(g, lam, side):
    side = np.asarray(side)
    assert 0 < side.sum() < g.n, "side must be a non-empty proper subset"
    assert oracle.cut_value(g, side) == lam


def random_graph(rng, n, density, wmax, connected=True):
    edges, ws = [], []
    for u, v in itertools.combinations(range(n), 2):
        if rng.random() < density:
            edges.append((u, v))
            ws.append(int(rng.integers(1, wmax + 1)))
    if connected:  # a random spanning path keeps it connected
        perm = rng.permutation(n)
        for a, b in zip(perm[:-1], perm[1:]):
            edges.append((int(a), int(b)))
            ws.append(int(rng.integers(1, wmax + 1)))
    if not edges:
        edges, ws = [(0, 1)], [1]
    return gg.from_edges(n, edges, ws)


# --------------------------------------------------------------- closed forms
@pytest.mark.parametrize("route", list(ROUTES))
@pytest.mark.parametrize("n,w", [(2, 1), (3, 1), (6, 1), (9, 1), (7, 5)])
def test_complete_graph(route, n, w):
    g = gg.complete(n, w)
    lam, side = ROUTES[route](g)
    assert lam == w * (n - 1)
    check_side(g, lam, side)


@pytest.mark.parametrize("route", list(ROUTES))
@pytest.mark.parametrize("n,seed", [(3, 1), (5, 2), (12, 3), (17, 4)])
def test_cycle_two_lightest(route, n, seed):
    g = gg.cycle(n, seed, 1, 20)
    # each cycle edge appears twice in the CSR; take weights per edge
    src = g.src()
    per_edge = np.sort(g.w[src < g.col])
    lam, side = ROUTES[route](g)
    assert lam == per_edge[0] + per_edge[1]
    check_side(g, lam, side)


@pytest.mark.parametrize("route", list(ROUTES))
def test_trees_min_edge(route):
    rng = np.random.default_rng(11)
    for trial in range(20):
        n = int(rng.integers(2, 14))
        edges = [(int(rng.integers(0, v)), v) for v in range(1, n)]
        ws = [int(x) for x in rng.integers(1, 30, size=n - 1)]
        g = gg.from_edges(n, edges, ws)
        lam, side = ROUTES[route](g)
        assert lam == min(ws)
        check_side(g, lam, side)


@pytest.mark.parametrize("route", list(ROUTES))
@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (3, 3), (4, 6), (5, 2)])
def test_complete_bipartite(route, a, b):
    edges = [(i, a + j) for i in range(a) for j in range(b)]
    g = gg.from_edges(a + b, edges)
    lam, side = ROUTES[route](g)
    assert lam == min(a, b)
    check_side(g, lam, side)


@pytest.mark.parametrize("route", list(ROUTES))
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_hypercube(route, d):
    n = 1 << d
    edges = [(v, v ^ (1 << i)) for v in range(n) for i in range(d) if v < v ^ (1 << i)]
    g = gg.from_edges(n, edges)
    lam, side = ROUTES[route](g)
    assert lam == d
    check_side(g, lam, side)


@pytest.mark.parametrize("route", list(ROUTES))
@pytest.mark.parametrize("a,k", [(4, 1), (5, 2), (6, 3), (6, 5), (6, 6), (8, 7)])
def test_two_cliques(route, a, k):
    # k < a: the k joining edges are the cheapest cut (a lone vertex without a
    # joining edge costs a-1 >= k).  k == a: a perfect matching, every vertex
    # has degree a and both the joining cut and every lone vertex cost a.
    g = gg.two_cliques(a, k)
    lam, side = ROUTES[route](g)
    assert lam == (k if k < a else a)
    check_side(g, lam, side)


@pytest.mark.parametrize("route", list(ROUTES))
def test_two_vertices_parallel(route):
    g = gg.from_edges(2, [(0, 1), (0, 1), (1, 0)], [3, 4, 5])
    lam, side = ROUTES[route](g)
    assert lam == 12
    assert list(side) in ([0, 1], [1, 0])


@pytest.mark.parametrize("route", list(ROUTES))
def test_disconnected_is_zero(route):
    g = gg.from_edges(7, [(0, 1), (1, 2), (3, 4), (4, 5), (5, 6), (6, 3)], [4, 4, 1, 1, 1, 1])
    lam, side = ROUTES[route](g)
    assert lam == 0
    check_side(g, lam, side)


def test_hand_examples():
    spec = json.load(open(os.path.join(GOLDEN, "hand_examples.json")))
    for ex in spec["graphs"]:
        e = np.array(ex["edges"])
        g = gg.from_edges(ex["n"], e[:, :2], e[:, 2])
        for route, f in ROUTES.items():
            lam, side = f(g)
            assert lam == ex["lambda"], (ex["name"], route)
            check_side(g, lam, side)
        # O1 returns one minimiser; it must be among the listed sides
        _, side = oracle.bruteforce(g)
        s = set(np.flatnonzero(side).tolist())
        comp = set(range(ex["n"])) - s
        listed = [set(x) for x in ex["sides"]]
        assert s in listed or comp in listed, ex["name"]


# --------------------------------------------------------- cross-route sweep
def test_routes_agree_on_random_tiny_graphs():
    rng = np.random.default_rng(2024)
    for trial in range(1500):
        n = int(rng.integers(2, 11))
        g = random_graph(rng, n, float(rng.uniform(0.1, 1.0)), int(rng.choice([1, 3, 10, 100])),
                         connected=bool(rng.random() < 0.9))
        lb, sb = oracle.bruteforce(g)
        ls, ss = oracle.stoer_wagner(g)
        ln, sn, _ = oracle.noi(g, trial)
        assert lb == ls == ln, (trial, lb, ls, ln)
        for s in (sb, ss, sn):
            check_side(g, lb, s)
        assert lb <= min_degree(g)


def test_bruteforce_max_size_and_pairs():
    rng = np.random.default_rng(5)
    g = random_graph(rng, 18, 0.3, 5)
    lb, sb = oracle.bruteforce(g)
    assert lb == oracle.stoer_wagner(g)[0] == oracle.noi(g)[0]
    conn = oracle.pair_connectivity(gg.from_edges(12, [(i, (i + 1) % 12) for i in range(12)]))
    # on a unit cycle every pair has connectivity 2
    assert (conn[~np.eye(12, dtype=bool)] == 2).all()


def test_pair_connectivity_properties():
    rng = np.random.default_rng(9)
    for trial in range(30):
        n = int(rng.integers(3, 10))
        g = random_graph(rng, n, 0.5, 7)
        conn = oracle.pair_connectivity(g)
        off = conn[~np.eye(n, dtype=bool)]
        assert (conn == conn.T).all()
        assert off.min() == oracle.bruteforce(g)[0]
        # ultrametric-like property of edge connectivity:
        # lambda(s,t) >= min(lambda(s,x), lambda(x,t)) for every x
        for s, t, x in itertools.permutations(range(n), 3):
            assert conn[s, t] >= min(conn[s, x], conn[x, t])
    # path: connectivity is the lightest edge between the two ends
    g = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)], [5, 2, 7])
    conn = oracle.pair_connectivity(g)
    assert conn[0, 1] == 5 and conn[0, 3] == 2 and conn[2, 3] == 7 and conn[1, 2] == 2


# ---------------------------------------------------------------- invariants
def test_invariants():
    rng = np.random.default_rng(77)
    for trial in range(150):
        n = int(rng.integers(3, 11))
        g = random_graph(rng, n, float(rng.uniform(0.2, 0.9)), 9)
        lam = oracle.bruteforce(g)[0]
        assert 1 <= lam <= min_degree(g)
        # scaling every weight by s scales lambda by s
        s = int(rng.integers(2, 6))
        gs = gg.Graph(g.n, g.row_ptr, g.col, g.w * s)
        assert oracle.noi(gs, trial)[0] == s * lam
        assert oracle.stoer_wagner(gs)[0] == s * lam
        # relabelling leaves lambda unchanged
        perm = rng.permutation(n)
        src = g.src()
        e = np.stack([perm[src], perm[g.col]], 1)
        keep = e[:, 0] < e[:, 1]
        gp = gg.from_edges(n, e[keep], g.w[keep])
        assert oracle.noi(gp, trial)[0] == lam
        # adding an edge never lowers lambda
        u, v = rng.choice(n, 2, replace=False)
        e2 = np.concatenate([np.stack([src, g.col], 1)[src < g.col], [[u, v]]])
        w2 = np.concatenate([g.w[src < g.col], [int(rng.integers(1, 5))]])
        assert oracle.noi(gg.from_edges(n, e2, w2), trial)[0] >= lam
        # contracting an edge never lowers lambda (when two or more remain)
        a, b = int(src[0]), int(g.col[0])
        relab = np.arange(n)
        relab[b] = a
        relab = np.unique(relab, return_inverse=True)[1]
        ce = np.stack([relab[src], relab[g.col]], 1)
        keep = ce[:, 0] < ce[:, 1]
        if n - 1 >= 2:
            gc = gg.from_edges(n - 1, ce[keep], g.w[keep])
            assert oracle.bruteforce(gc)[0] >= lam


def test_noi_seed_independent_on_workload_shapes():
    # shapes of the workloads, small: planted clusters and a power-law core
    graphs = [gg.batch_graph(g) for g in (1, 3, 4, 9)]
    graphs.append(gg.chung_lu(17, 3000, 2.5, 16.0, 1, 50, kcore=0, lcc=True))
    for g in graphs:
        lams = {oracle.noi(g, s)[0] for s in range(4)}
        assert len(lams) == 1
        lam = lams.pop()
        if g.n <= 2500:
            assert oracle.stoer_wagner(g)[0] == lam
        _, side, _ = oracle.noi(g, 1)
        check_side(g, lam, side)


@pytest.mark.slow
def test_stoer_wagner_equals_noi_on_planted_4096():
    g = gg.planted_4096()
    ls, ss = oracle.stoer_wagner(g)
    ln, sn, rounds = oracle.noi(g, 3)
    assert ls == ln
    check_side(g, ls, ss)
    check_side(g, ln, sn)


def test_contract_keeps_block_aligned_cuts():
    # a cut whose side is a union of blocks has the same value before and
    # after contraction; the contracted graph has one vertex per block
    rng = np.random.default_rng(41)
    for trial in range(40):
        n = int(rng.integers(4, 30))
        g = random_graph(rng, n, 0.3, 9)
        k = int(rng.integers(2, n + 1))
        labels = rng.integers(0, k, size=n)
        h, blk = oracle.contract(g, labels)
        assert h.n == len(np.unique(labels))
        for _ in range(5):
            pick = rng.random(h.n) < 0.5
            if pick.all() or not pick.any():
                continue
            assert oracle.cut_value(g, pick[blk]) == oracle.cut_value(h, pick)
    # hand example: path 0-1-2-3 with weights 1,2,3; blocks {0,1},{2,3}
    g = gg.from_edges(4, [(0, 1), (1, 2), (2, 3)], [1, 2, 3])
    h, blk = oracle.contract(g, [7, 7, 9, 9])
    assert h.n == 2 and h.nnz == 2 and list(h.w) == [2, 2]


# ------------------------------------------------ VieCut-style upper bound
def _fixture_graph(ex):
    if isinstance(ex["edges"], str):
        kind, *args = ex["edges"].split()
        return gg.two_cliques(*map(int, args)) if kind == "two_cliques" else gg.complete(int(args[0]))
    e = np.array(ex["edges"])
    return gg.from_edges(ex["n"], e[:, :2], e[:, 2])


def test_lp_sweep_hand_examples():
    spec = json.load(open(os.path.join(GOLDEN, "lp_examples.json")))
    for ex in spec["sweeps"]:
        g = _fixture_graph(ex)
        assert oracle.lp_sweep(g, ex["labels_in"]).tolist() == ex["labels_out"], ex["name"]


def test_viecut_hand_examples():
    spec = json.load(open(os.path.join(GOLDEN, "lp_examples.json")))
    for ex in spec["bounds"]:
        g = _fixture_graph(ex)
        lam, side, levels = oracle.viecut(g, stop_n=ex.get("stop_n", 2))
        assert (lam, levels) == (ex["bound"], ex["levels"]), ex["name"]
        assert oracle.cut_value(g, side) == lam and 0 < side.sum() < g.n, ex["name"]
        if "side" in ex:
            s = sorted(np.flatnonzero(side).tolist())
            other = sorted(set(range(g.n)) - set(ex["side"]))
            assert s in (ex["side"], other), ex["name"]


@pytest.mark.parametrize("a", [4, 5, 6, 8, 12])
def test_viecut_finds_the_bridge_between_cliques(a):
    # two sweeps turn each clique into one class, so the bound is exact
    lam, side, _ = oracle.viecut(gg.two_cliques(a, 1))
    assert lam == 1
    assert sorted([int(side.sum()), a]) == [a, a]


def test_lp_sweep_is_synchronous_and_label_invariant():
    # renaming labels by an increasing map commutes with a sweep (ties to the
    # smallest label are preserved); a vertex's new label is always one of
    # its neighbours' labels
    rng = np.random.default_rng(5)
    for trial in range(200):
        n = int(rng.integers(2, 30))
        g = random_graph(rng, n, float(rng.uniform(0.1, 0.8)), int(rng.choice([1, 5, 50])),
                         connected=bool(rng.random() < 0.8))
        lab = rng.integers(0, n, size=n).astype(np.int32)
        out = oracle.lp_sweep(g, lab)
        up = np.sort(rng.choice(10 * n, size=n, replace=False)).astype(np.int32)  # increasing map
        assert np.array_equal(oracle.lp_sweep(g, up[lab]), up[out]), trial
        src = g.src()
        for v in range(n):
            nb = g.col[(src == v) & (g.col != v)]
            if len(nb):
                assert out[v] in set(lab[nb].tolist())
            else:
                assert out[v] == lab[v]


def test_viecut_bound_properties_on_random_graphs():
    # lambda <= bound <= minimum degree, and the side realises the bound
    rng = np.random.default_rng(77)
    for trial in range(400):
        n = int(rng.integers(2, 14))
        g = random_graph(rng, n, float(rng.uniform(0.15, 1.0)), int(rng.choice([1, 3, 20])),
                         connected=bool(rng.random() < 0.9))
        lam = oracle.bruteforce(g)[0]
        for sweeps in (1, 2, 3):
            b, side, _ = oracle.viecut(g, sweeps=sweeps)
            assert lam <= b <= min_degree(g), (trial, sweeps)
            check_side(g, b, side)


def test_viecut_on_workload_shapes():
    for g in [gg.planted_4096()] + [gg.batch_graph(i) for i in range(0, 400, 37)]:
        lam = oracle.noi(g, 1)[0]
        b, side, levels = oracle.viecut(g)
        assert lam <= b <= min_degree(g), g.name
        assert oracle.cut_value(g, side) == b
        assert levels >= 1


# ------------------------------------------ Matula's (2+eps)-approximation
def matula_bound(lam, ppm):
    # the paper's guarantee: a round contracts the edges with q(e) >= k, k at
    # least (1/2 - eps) delta; a minimum-cut edge has q(e) <= lambda, so if
    # one is contracted then delta <= lambda / (1/2 - eps), and delta is a
    # cut the answer counts; if none is, the minimum cut survives to the end
    return lam * 2_000_000 // (1_000_000 - 2 * ppm)


@pytest.mark.parametrize("ppm", [1, 100_000, 250_000, 490_000])
def test_matula_is_a_cut_within_its_bound(ppm):
    rng = np.random.default_rng(900 + ppm % 97)
    for trial in range(300):
        n = int(rng.integers(2, 12))
        g = random_graph(rng, n, float(rng.uniform(0.1, 1.0)), int(rng.choice([1, 3, 10, 100])),
                         connected=bool(rng.random() < 0.9))
        lam = oracle.bruteforce(g)[0]
        a, side, _ = oracle.matula(g, ppm, trial)
        check_side(g, a, side)
        assert lam <= a <= matula_bound(lam, ppm), (trial, lam, a)
        assert a <= min_degree(g)


def test_matula_fixtures_where_a_floor_threshold_breaks_the_bound():
    # graphs on which contracting at q(e) >= floor((1/2 - eps) delta) answered
    # above lambda / (1/2 - eps); the paper's threshold keeps the bound
    fx = json.load(open(os.path.join(GOLDEN, "matula_examples.json")))["examples"]
    assert len(fx) >= 3
    for ex in fx:
        g = gg.from_edges(ex["n"], ex["edges"], ex["weights"])
        lam = oracle.bruteforce(g)[0]
        assert ex["floor_answer"] > matula_bound(lam, ex["ppm"])
        a, side, _ = oracle.matula(g, ex["ppm"], ex["seed"])
        check_side(g, a, side)
        assert lam <= a <= matula_bound(lam, ex["ppm"]), (ex["n"], lam, a)


def _hypercube(d):
    n = 1 << d
    return gg.from_edges(n, [(v, v ^ (1 << i)) for v in range(n) for i in range(d) if v < v ^ (1 << i)],
                         name=f"Q{d}")


def _kab(a, b):
    return gg.from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)], name=f"K{a},{b}")


@pytest.mark.parametrize("g", [gg.complete(9), gg.complete(6, 5), _hypercube(4), _kab(3, 7)],
                         ids=lambda g: g.name)
def test_matula_is_exact_when_lambda_is_the_min_degree(g):
    # the answer is a cut (>= lambda) and never above the minimum degree
    lam = oracle.bruteforce(g)[0] if g.n <= 20 else oracle.noi(g)[0]
    assert lam == min_degree(g)
    for ppm in (1, 100_000, 400_000):
        assert oracle.matula(g, ppm)[0] == lam


def test_matula_lowers_the_contraction_bound():
    # with the bound below the best cut a round contracts at least as much:
    # never more rounds than the exact loop on the same graphs, and fewer on
    # most of them (the exact loop's bound would give the same counts)
    graphs = [gg.planted_4096()] + [gg.batch_graph(i) for i in range(0, 400, 37)]
    fewer = 0
    for g in graphs:
        e, _, re_ = oracle.noi(g, 1)
        a, side, ra = oracle.matula(g, 100_000, 1)
        assert e <= a <= matula_bound(e, 100_000)
        assert oracle.cut_value(g, side) == a
        assert ra <= re_, g.name
        fewer += ra < re_
    assert fewer >= len(graphs) // 2


def test_matula_rejects_eps_out_of_range():
    with pytest.raises(ValueError):
        oracle.matula(gg.complete(4), 500_000)
    with pytest.raises(ValueError):
        oracle.matula(gg.complete(4), -1)


# ------------------------------------------------ Padberg-Rinaldi tests
PR1, PR2, PR3, PR4 = 1, 2, 4, 8


def _edge_entries(g):
    src = g.src()
    return [(int(e), int(src[e]), int(g.col[e])) for e in range(len(g.col)) if src[e] < g.col[e]]


def test_pr_tests_hand_examples():
    # a triangle whose light edge (0,1) sits beside two heavy ones
    g = gg.from_edges(3, [(0, 1), (0, 2), (1, 2)], [1, 5, 5])
    f = oracle.pr_tests(g, 6)
    e01 = [e for e, u, v in _edge_entries(g) if (u, v) == (0, 1)][0]
    # c(0) = c(1) = 6 < 2 (1 + 5); 1 + min(5, 5) = 6 >= 6; not PR1, not PR2
    assert f[e01] == PR3 | PR4
    assert oracle.pr_tests(g, 7)[e01] == PR3
    # K_n, unit weights: one edge plus n - 2 two-edge paths = n - 1 = lambda;
    # PR3 needs n - 1 < 4
    for n in (4, 5, 6, 8):
        g = gg.complete(n)
        f = oracle.pr_tests(g, n - 1)
        for e, u, v in _edge_entries(g):
            assert f[e] & PR4
            assert bool(f[e] & PR3) == (n <= 4)
            assert not f[e] & (PR1 | PR2)
        assert not any(oracle.pr_tests(g, n)[e] & PR4 for e, _, _ in _edge_entries(g))


def test_pr_tests_need_sorted_short_rows():
    g = gg.complete(6)
    f = oracle.pr_tests(g, 5, max_deg=4)  # rows of 5 entries exceed the limit
    assert not any(x & (PR3 | PR4) for x in f)
    # the same graph with row 0 listed backwards: its edges lose PR3/PR4
    col = g.col.copy()
    a, b = g.row_ptr[0], g.row_ptr[1]
    col[a:b] = col[a:b][::-1].copy()
    w = g.w.copy()
    w[a:b] = w[a:b][::-1].copy()
    h = gg.Graph(g.n, g.row_ptr.copy(), col, w, "K6-rev")
    f = oracle.pr_tests(h, 5)
    for e, u, v in _edge_entries(h):
        assert bool(f[e] & PR4) == (u != 0)


def test_pr_tests_are_sound_by_brute_force():
    # contracting a passing edge keeps the minimum cut: min(bound, delta,
    # lambda(G/e)) = lambda(G), with the bound a real cut (lambda itself, or
    # delta); so does contracting all passing edges at once, as a round does;
    # PR4 never claims more than the pair's connectivity
    rng = np.random.default_rng(4242)
    checked = {PR1: 0, PR2: 0, PR3: 0, PR4: 0}
    for trial in range(250):
        n = int(rng.integers(3, 10))
        g = random_graph(rng, n, float(rng.uniform(0.3, 1.0)), int(rng.choice([1, 2, 5, 20])))
        lam = oracle.bruteforce(g)[0]
        delta = min_degree(g)
        conn = oracle.pair_connectivity(g)
        for bound in {lam, delta}:
            f = oracle.pr_tests(g, bound)
            for e, u, v in _edge_entries(g):
                if f[e] & PR4:
                    assert conn[u, v] >= bound, (trial, u, v)
                if not f[e]:
                    continue
                lab = np.arange(g.n)
                lab[v] = u
                h, _ = oracle.contract(g, lab)
                lh = oracle.bruteforce(h)[0] if h.n >= 2 else bound
                assert min(bound, delta, lh) == lam, (trial, bound, f[e])
                for bit in checked:
                    checked[bit] += bool(f[e] & bit)
            # every passing edge at once
            parent = np.arange(g.n)

            def find(x):
                while parent[x] != x:
                    x = parent[x]
                return x
            for e, u, v in _edge_entries(g):
                if f[e]:
                    a, b = find(u), find(v)
                    parent[max(a, b)] = min(a, b)
            lab = np.array([find(x) for x in range(g.n)])
            h, _ = oracle.contract(g, lab)
            lh = oracle.bruteforce(h)[0] if h.n >= 2 else bound
            assert min(bound, delta, lh) == lam, (trial, bound, "all")
        # PR4's path sum never exceeds the pair's connectivity
        for e, u, v in _edge_entries(g):
            f1 = oracle.pr_tests(g, int(conn[u, v]) + 1)
            assert not f1[e] & PR4
    assert min(checked.values()) > 20, checked


# ----------------------------------- clustering bound with an exact finish
def test_viecut_exact_finish_without_levels_is_lambda():
    # no clustering level: the last level graph is G itself, solved exactly
    rng = np.random.default_rng(515)
    for trial in range(300):
        n = int(rng.integers(3, 13))
        g = random_graph(rng, n, float(rng.uniform(0.15, 1.0)), int(rng.choice([1, 3, 20])),
                         connected=bool(rng.random() < 0.9))
        lam = oracle.bruteforce(g)[0]
        b, side, levels = oracle.viecut(g, max_levels=0, exact_finish=True)
        assert levels == 0 and b == lam, trial
        check_side(g, b, side)


def test_viecut_exact_finish_never_worse():
    rng = np.random.default_rng(516)
    for trial in range(300):
        n = int(rng.integers(3, 14))
        g = random_graph(rng, n, float(rng.uniform(0.15, 1.0)), int(rng.choice([1, 3, 20])))
        lam = oracle.bruteforce(g)[0]
        for stop in (2, 4, 8):
            plain = oracle.viecut(g, stop_n=stop)[0]
            b, side, _ = oracle.viecut(g, stop_n=stop, exact_finish=True)
            assert lam <= b <= plain, (trial, stop)
            check_side(g, b, side)


def test_viecut_exact_finish_on_workload_shapes():
    # stopping the levels at 64 vertices leaves level graphs whose minimum
    # degree is far above lambda on some batch graphs; solving them exactly
    # recovers lambda (from the independent NOI route)
    lowered = 0
    for g in [gg.planted_4096()] + [gg.batch_graph(i) for i in range(0, 400, 37)]:
        lam = oracle.noi(g, 1)[0]
        plain = oracle.viecut(g, stop_n=64)[0]
        b, side, _ = oracle.viecut(g, stop_n=64, exact_finish=True)
        assert lam <= b <= plain
        assert oracle.cut_value(g, side) == b
        lowered += b < plain
        if g.name in ("batch_74", "batch_222"):
            assert plain > lam and b == lam, g.name
    assert lowered >= 2
