"""GPU parity: lambda from the HIP path equals the oracle's exactly (integer,
tolerance 0), and every returned side is checked by recomputing its cut
weight (sides are not unique, so identity is not compared)."""
import json
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import announce, check_side, random_graph, solve

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


def test_closed_forms():
    cases = [(gg.complete(8), 7), (gg.complete(12, 3), 33), (gg.two_cliques(10, 3), 3),
             (gg.two_cliques(7, 7), 7), (gg.from_edges(2, [(0, 1), (0, 1)], [3, 4]), 7)]
    cyc = gg.cycle(40, 5, 1, 30)
    pe = np.sort(cyc.w[cyc.src() < cyc.col])
    cases.append((cyc, int(pe[0] + pe[1])))
    d = 6
    cube = gg.from_edges(1 << d, [(v, v ^ (1 << i)) for v in range(1 << d) for i in range(d)
                                  if v < v ^ (1 << i)])
    cases.append((cube, d))
    for g, expect in cases:
        announce("closed form", g.name, g.n)
        lam, side, _ = solve(g)
        assert lam == expect, g.name
        check_side(g, lam, side)


def test_hand_examples():
    spec = json.load(open(os.path.join(GOLDEN, "hand_examples.json")))
    for ex in spec["graphs"]:
        announce("hand", ex["name"])
        e = np.array(ex["edges"])
        g = gg.from_edges(ex["n"], e[:, :2], e[:, 2])
        lam, side, _ = solve(g)
        assert lam == ex["lambda"], ex["name"]
        check_side(g, lam, side)


def test_random_tiny_graphs_against_enumeration():
    rng = np.random.default_rng(31)
    for t in range(300):
        n = int(rng.integers(2, 15))
        g = random_graph(rng, n, float(rng.uniform(0.15, 1.0)), int(rng.choice([1, 4, 50])),
                         connected=bool(rng.random() < 0.93))
        if t % 50 == 0:
            announce("tiny", t, n)
        lam, side, _ = solve(g)
        ref, _ = oracle.bruteforce(g)
        assert lam == ref, (t, lam, ref)
        check_side(g, lam, side)


@pytest.mark.parametrize("opts", [dict(pq_order=1), dict(pq_order=2), dict(pq_order=3),
                                  dict(whole_max=8, scan_mode=1, pq_order=1, scan_visits=2),
                                  dict(whole_max=8, scan_mode=1, pq_order=2, scan_visits=4, use_pr=0),
                                  dict(scan_mode=2, pq_order=3)],
                         ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()))
def test_queue_orders_and_repeated_visits_against_noi(opts):
    """The priority-queue orders (bucket queue, bucket stack, heap; section
    "Priority Queue Implementations") and repeated visits (section "Parallel
    CAPFOREST") change which pairs a round unites, never lambda: unweighted
    and few-valued weights give many equal keys, so the order decides."""
    rng = np.random.default_rng(17 + 3 * len(opts) + opts.get("pq_order", 0))
    for t in range(24):
        n = int(rng.integers(20, 400))
        g = random_graph(rng, n, float(rng.uniform(0.02, 0.25)), int(rng.choice([1, 2, 3])))
        if t % 8 == 0:
            announce("orders", opts, t, n, g.m)
        lam, side, _ = solve(g, **opts)
        ref, _, _ = oracle.noi(g, 2)
        assert lam == ref, (t, lam, ref, opts)
        check_side(g, lam, side)


@pytest.mark.parametrize("emit_rows", [1, -1])
def test_row_wise_emit_on_a_packed_batch(emit_rows):
    """The contraction's row-wise key emit (rows outside each graph's
    reference block only, skipped rows' entries as mirrors) and the
    entry-wise emit give the oracle's lambda on every graph of a packed
    batch, with sides that realise it."""
    import paper_1808_05458_amd as mc
    rng = np.random.default_rng(71 + emit_rows)
    graphs = [random_graph(rng, int(rng.integers(10, 300)), float(rng.uniform(0.03, 0.3)),
                           int(rng.choice([1, 3, 20]))) for _ in range(60)]
    refs = [oracle.noi(g, 1)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    announce("emit rows", emit_rows, packed.n, packed.m)
    lams, sides, st = mc.mincut_batched(rp, col, w, vo, emit_rows=emit_rows)
    assert list(lams) == refs
    s = sides.cpu().numpy()
    for i, g in enumerate(graphs):
        check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])


def test_queue_orders_are_refused_outside_their_range():
    import paper_1808_05458_amd as mc
    g = gg.complete(6)
    for bad in (dict(pq_order=4), dict(pq_order=-1), dict(scan_visits=-2)):
        with pytest.raises(mc.MincutError) as e:
            solve(g, **bad)
        assert e.value.code == mc.MC_EINVAL


def test_medium_graphs_against_noi():
    rng = np.random.default_rng(7)
    for t in range(40):
        n = int(rng.integers(30, 700))
        g = random_graph(rng, n, float(rng.uniform(0.01, 0.2)), int(rng.choice([1, 3, 20])))
        announce("medium", t, n, g.m)
        lam, side, _ = solve(g)
        ref, _, _ = oracle.noi(g, 2)
        assert lam == ref, (t, lam, ref)
        check_side(g, lam, side)


@pytest.mark.parametrize("opts", [dict(), dict(use_pr=0), dict(eager_blacklist=0),
                                  dict(force_fallback=1), dict(max_pops=3),
                                  dict(whole_max=16), dict(whole_max=16, use_pr=0),
                                  dict(whole_max=16, scan_mode=1),
                                  dict(whole_max=16, scan_mode=1, max_pops=5, use_pr=0),
                                  dict(whole_max=16, scan_mode=1, eager_blacklist=0),
                                  dict(whole_max=16, sweep_handoff=1),
                                  dict(whole_max=16, sweep_handoff=3, use_pr=0),
                                  dict(whole_max=16, sweep_handoff=1, sweep_tail=1),
                                  dict(whole_max=16, sweep_handoff=1, sweep_tail=1, use_pr=0),
                                  dict(whole_max=16, sweep_tail=-1),
                                  dict(whole_max=16, sweep_handoff=1, sweep_pull=1),
                                  dict(whole_max=16, sweep_handoff=2, sweep_pull=1, use_pr=0),
                                  dict(whole_max=16, sweep_pull=-1),
                                  dict(scan_mode=2), dict(scan_mode=2, max_pops=3),
                                  dict(scan_mode=2, eager_blacklist=0, use_pr=0),
                                  dict(pq_order=1), dict(pq_order=2, use_pr=0), dict(pq_order=3),
                                  dict(whole_max=16, scan_mode=1, pq_order=2),
                                  dict(whole_max=16, scan_mode=1, scan_visits=3, use_pr=0),
                                  dict(scan_mode=2, pq_order=1),
                                  dict(emit_rows=1), dict(emit_rows=1, whole_max=16, use_pr=0),
                                  dict(emit_rows=-1, whole_max=16),
                                  dict(whole_max=16, sweep_handoff=1, sweep_seg=1, sweep_pull=-1),
                                  dict(whole_max=16, sweep_handoff=1, sweep_seg=1, sweep_pull=-1, use_pr=0),
                                  dict(whole_max=16, sweep_handoff=1, sweep_seg=-1, sweep_pull=-1)])
def test_planted_4096_options(opts):
    g = gg.planted_4096()
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))["planted_4096"]
    assert g.n == gold["n"] and g.m == gold["m"]
    announce("planted_4096", opts)
    lam, side, st = solve(g, **opts)
    assert lam == gold["lambda"]
    check_side(g, lam, side)


def test_region_scans_on_power_law_core():
    # graphs above whole_max: full-graph sweeps (scan_mode 0) or region scans
    # with the sweep as fallback (scan_mode 1), on a power-law k-core
    g = gg.chung_lu(23, 20000, 2.5, 16.0, 1, 3, kcore=4, lcc=True)
    ref, _, _ = oracle.noi(g, 1)
    for opts in [dict(whole_max=64), dict(whole_max=64, use_pr=0),
                 dict(whole_max=64, sweep_handoff=4),
                 dict(whole_max=64, sweep_tail=-1), dict(whole_max=64, sweep_tail=1, use_pr=0),
                 dict(whole_max=64, sweep_handoff=4, sweep_tail=1),
                 dict(whole_max=64, sweep_handoff=4, sweep_pull=1), dict(whole_max=64, sweep_pull=-1, use_pr=0),
                 dict(whole_max=64, scan_mode=1), dict(whole_max=64, scan_mode=1, eager_blacklist=0),
                 dict(whole_max=64, scan_mode=1, max_pops=50),
                 dict(whole_max=64, scan_mode=1, use_pr=0),
                 dict(whole_max=64, scan_mode=1, pq_order=1), dict(whole_max=64, scan_mode=1, pq_order=2),
                 dict(whole_max=64, scan_mode=1, pq_order=3, scan_visits=2),
                 dict(whole_max=64, scan_mode=1, scan_visits=4, use_pr=0),
                 dict(whole_max=64, sweep_handoff=4, sweep_seg=1, sweep_pull=-1),
                 dict(whole_max=64, sweep_seg=1, sweep_pull=-1, use_pr=0), dict(whole_max=64, sweep_seg=-1)]:
        announce("chung_lu 20000", opts)
        lam, side, st = solve(g, **opts)
        assert lam == ref, opts
        check_side(g, lam, side)


def test_disconnected_and_edge_cases():
    announce("disconnected")
    g = gg.from_edges(9, [(0, 1), (1, 2), (2, 0), (3, 4), (4, 5), (5, 3), (6, 7), (7, 8), (8, 6)],
                      [5] * 9)
    lam, side, _ = solve(g)
    assert lam == 0
    check_side(g, lam, side)
    announce("isolated vertex")
    g = gg.from_edges(4, [(0, 1), (1, 2)], [2, 3])
    lam, side, _ = solve(g)
    assert lam == 0 and side[3] == 1
    announce("self loops and repeated entries")
    g = gg.from_edges(5, [(0, 1), (0, 1), (1, 2), (2, 3), (3, 4), (4, 0), (2, 2), (3, 3)],
                      [1, 1, 5, 5, 5, 5, 100, 7])
    lam, side, _ = solve(g)
    assert lam == oracle.bruteforce(g)[0]
    check_side(g, lam, side)
    announce("two vertices")
    g = gg.from_edges(2, [(0, 1)], [9])
    lam, side, _ = solve(g)
    assert lam == 9 and list(side) == [0, 1]


def test_ingest_chunk_forms_against_noi():
    # the weighted degrees come from two forms of the ingest: a chunk with
    # fewer than 64 row starts, light weights and no self-loop takes each
    # row's share from prefix sums; a chunk of short rows (a ring's degree-2
    # rows start more than 64 per chunk), one holding a self-loop or a
    # weight of 2^22 or more maps every entry to its row.  These graphs mix
    # all of them: lambda equals the sequential NOI oracle's, the reported
    # initial bound equals the minimum weighted degree summed on the host
    # (self-loops excluded), and the side realises lambda.
    rng = np.random.default_rng(11)
    for t in range(8):
        n = int(rng.integers(600, 2500))
        edges = [(i, (i + 1) % n) for i in range(n)]
        for h in rng.choice(n, size=4, replace=False):
            for v in rng.choice(n, size=int(rng.integers(200, 600)), replace=False):
                if v != h:
                    edges.append((int(h), int(v)))
        extra = rng.integers(0, n, size=(n // 2, 2))
        edges += [(int(a), int(b)) for a, b in extra if a != b]
        wts = rng.integers(1, 50, size=len(edges))
        wts[rng.choice(len(edges), size=6, replace=False)] = rng.integers(1 << 22, 1 << 24, size=6)
        loops = list(rng.choice(n, size=5, replace=False))
        if t % 2:  # a heavy self-loop on a vertex of least weighted degree
            g0 = gg.from_edges(n, edges, wts)
            s0 = np.repeat(np.arange(n), np.diff(g0.row_ptr))
            loops[0] = int(np.argmin(np.bincount(s0, weights=g0.w.astype(np.float64), minlength=n)))
        edges += [(int(v), int(v)) for v in loops]
        wts = np.concatenate([wts, rng.integers(1, 1000, size=5)])
        g = gg.from_edges(n, edges, wts)
        src = np.repeat(np.arange(n), np.diff(g.row_ptr))
        deg = np.bincount(src, weights=np.where(g.col != src, g.w, 0).astype(np.float64), minlength=n)
        ref = oracle.noi(g, 1)[0]
        announce("ingest chunk forms", t, n, g.m, ref)
        lam, side, st = solve(g)
        assert lam == ref
        check_side(g, lam, side)
        assert st["lambda_initial"] == int(deg.min())


def test_invalid_inputs_are_rejected():
    import torch
    import paper_1808_05458_amd as mc
    g = gg.complete(5)
    rp, col, w = mc.to_device(g, "cuda")
    bad = col.clone()
    bad[3] = 99
    announce("invalid col")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rp, bad, w)
    assert e.value.code == mc.MC_EINVAL
    announce("zero weight")
    w0 = w.clone()
    w0[0] = 0
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rp, col, w0)
    assert e.value.code == mc.MC_EINVAL
    announce("bad row_ptr")
    rpb = rp.clone()
    rpb[2] = rpb[3] + 1
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rpb, col, w)
    assert e.value.code == mc.MC_EINVAL
    announce("one vertex")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(torch.zeros(2, dtype=torch.int64, device="cuda"),
                  torch.zeros(0, dtype=torch.int32, device="cuda"),
                  torch.zeros(0, dtype=torch.int32, device="cuda"))
    assert e.value.code == mc.MC_ENOCUT
    announce("overflow")
    h = gg.from_edges(3, [(0, 1), (1, 2), (2, 0)], [1 << 30] * 3)
    rp, col, w = mc.to_device(h, "cuda")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rp, col, w)
    assert e.value.code == mc.MC_EOVERFLOW
    # the library still works after errors
    lam, side, _ = solve(gg.complete(6))
    assert lam == 5


def test_batched_workload_sample_against_noi():
    # 160 graphs of the 4096-graph batch recipe, in one packed solve, under
    # the default (LDS sweeps) and the one-pop-at-a-time whole scans
    import paper_1808_05458_amd as mc
    graphs = [gg.batch_graph(i) for i in range(160)]
    refs = [oracle.noi(g, 5)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for opts in [dict(), dict(scan_mode=2), dict(use_pr=0), dict(seed=2), dict(seed=3, scan_mode=2),
                 dict(seed=4, scan_mode=2)]:
        announce("batch sample", opts, packed.n, packed.m)
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, **opts)
        s = sides.cpu().numpy()
        assert list(lams) == refs, opts
        for i, g in enumerate(graphs):
            check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])


def test_batched_small_against_noi():
    import torch
    import paper_1808_05458_amd as mc
    graphs = [gg.batch_graph(i) for i in range(24)]
    graphs.append(gg.from_edges(6, [(0, 1), (1, 2), (3, 4), (4, 5)], [1, 1, 1, 1]))  # disconnected
    graphs.append(gg.complete(3))
    graphs.append(gg.from_edges(2, [(0, 1)], [17]))
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    announce("batched", len(graphs), packed.n, packed.m)
    lams, sides, st = mc.mincut_batched(rp, col, w, vo)
    s = sides.cpu().numpy()
    for i, g in enumerate(graphs):
        ref, _, _ = oracle.noi(g, 3)
        assert lams[i] == ref, (i, lams[i], ref)
        check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])
    # each graph alone gives the same lambda
    for i in (0, 5, 24, 26):
        lam, _, _ = solve(graphs[i])
        assert lam == lams[i]


def test_sweep_on_weighted_graphs_with_wide_buckets():
    # bound above 4096 makes the sweep's bucket queue hold several keys per
    # bucket (exact maximum search inside the top bucket)
    rng = np.random.default_rng(3)
    for t in range(6):
        n = int(rng.integers(200, 1500))
        g = random_graph(rng, n, float(rng.uniform(0.02, 0.1)), 5000)
        ref, _, _ = oracle.noi(g, 1)
        announce("wide buckets", t, n, ref)
        for opts in [dict(whole_max=16), dict(whole_max=16, use_pr=0),
                     dict(whole_max=16, sweep_handoff=2)]:
            lam, side, _ = solve(g, **opts)
            assert lam == ref, (t, opts)
            check_side(g, lam, side)


def test_sweep_on_larger_power_law_graph():
    g = gg.chung_lu(29, 200000, 2.5, 16.0, 1, 1, kcore=5, lcc=True)
    ref, _, _ = oracle.noi(g, 1)
    for opts in [dict(), dict(sweep_tail=-1), dict(sweep_tail=1, use_pr=0), dict(sweep_pull=1),
                 dict(sweep_pull=-1, sweep_tail=-1), dict(sweep_seg=1, sweep_pull=-1),
                 dict(sweep_seg=1, sweep_pull=-1, sweep_tail=-1, use_pr=0), dict(sweep_seg=-1)]:
        announce("chung_lu 200000 5-core", g.n, g.m, ref, opts)
        lam, side, st = solve(g, **opts)
        assert lam == ref, opts
        check_side(g, lam, side)
        assert st["rounds"] <= 6


def _round_is_sound(graphs, margins, **opts):
    """First round under a starting bound lambda + margin: contracting the
    GPU's blocks must keep a minimum cut (every cut below the bound)."""
    import paper_1808_05458_amd as mc
    lams = [oracle.noi(g, 5)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for margin in margins:
        lin = [l + margin for l in lams]
        labels, used = mc.debug_first_round(rp, col, w, vo, lhat_in=lin, **opts)
        lab = labels.cpu().numpy()
        # every label is a root: the relabelling that follows numbers blocks
        # by their root, so a vertex left at a non-root ancestor would be
        # contracted into a different block than the one checked here
        assert np.array_equal(lab[lab], lab), (margin, opts)
        nxt = []
        for i, g in enumerate(graphs):
            h, _ = oracle.contract(g, lab[vo[i]:vo[i + 1]])
            assert used[i] <= lin[i]
            if lams[i] < used[i]:
                assert h.n >= 2, (i, margin)
                assert oracle.noi(h, 1)[0] == lams[i], (i, margin, opts)
            nxt.append(h)
    return nxt


def test_round_soundness_batch_recipe():
    graphs = [gg.batch_graph(i) for i in range(120, 160)]
    announce("round soundness", len(graphs))
    for opts in [dict(), dict(scan_mode=2), dict(use_pr=0), dict(whole_max=64)]:
        _round_is_sound(graphs, [1, 20, 200], **opts)


def test_round_soundness_second_round():
    # second-round conditions: contracted, weighted graphs and a bound far
    # below their minimum degree
    graphs = [gg.batch_graph(i) for i in range(130, 150)]
    lams = [oracle.noi(g, 5)[0] for g in graphs]
    import paper_1808_05458_amd as mc
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    labels, used = mc.debug_first_round(rp, col, w, vo, lhat_in=[l + 20 for l in lams])
    lab = labels.cpu().numpy()
    g2 = [oracle.contract(g, lab[vo[i]:vo[i + 1]])[0] for i, g in enumerate(graphs)]
    keep = [i for i, h in enumerate(g2) if h.n > 2]
    announce("second round", len(keep))
    for opts in [dict(), dict(scan_mode=2), dict(use_pr=0)]:
        _round_is_sound([g2[i] for i in keep], [1, 20], **opts)


def test_contraction_kernels_equal_cpu_contraction():
    # emit + radix sort + merge + CSR against the numpy contraction, on
    # block structures of every size: few large blocks (long runs of equal
    # keys across tiles), many small ones, identity labels (merging
    # duplicates and dropping self-loops)
    import torch
    import paper_1808_05458_amd as mc
    rng = np.random.default_rng(12)
    cases = [gg.batch_graph(140), gg.chung_lu(31, 300000, 2.5, 16.0, 1, 9, kcore=0, lcc=True)]
    packed, vo, eo = gg.pack([gg.batch_graph(i) for i in range(100, 160)])
    cases.append(packed)
    cases.append(gg.from_edges(5, [(0, 1), (0, 1), (1, 2), (2, 2), (3, 4), (4, 0)], [1, 2, 3, 9, 4, 5]))
    # a hub whose row spans many ingest chunks, with every odd vertex
    # isolated (runs of empty rows inside chunks)
    leaves = np.arange(0, 24000, 2)
    leaves = leaves[leaves != 12000]
    cases.append(gg.from_edges(24001, [(12000, int(v)) for v in leaves], rng.integers(1, 9, size=len(leaves)),
                               name="hub-with-empty-rows"))
    # a long run of empty rows before a small dense part
    dense = [(50000 + i, 50000 + j) for i in range(40) for j in range(i + 1, 40)]
    cases.append(gg.from_edges(50040, dense, rng.integers(1, 5, size=len(dense)), name="empty-prefix"))
    for g in cases:
        for k in [1, 2, 3, 17, 1000, g.n]:
            k = min(k, g.n)
            lab = rng.integers(0, k, size=g.n) if k < g.n else np.arange(g.n)
            lab = np.unique(lab, return_inverse=True)[1].astype(np.int32)
            n_new = int(lab.max()) + 1
            announce("contract", g.name, g.n, k)
            rp, col, w = mc.to_device(g, "cuda")
            rpo, colo, wo = mc.debug_contract(rp, col, w, torch.from_numpy(lab).cuda(), n_new)
            h, blk = oracle.contract(g, lab)
            assert h.n == n_new
            assert np.array_equal(rpo.cpu().numpy(), h.row_ptr)
            assert np.array_equal(colo.cpu().numpy(), h.col)
            assert np.array_equal(wo.cpu().numpy(), h.w)


def _two_blobs(rng):
    """Two dense random blobs (weights 1..50) joined by one to three light
    edges: a minimum cut well below the minimum degree."""
    a, b = int(rng.integers(3, 9)), int(rng.integers(3, 9))
    e, w = [], []
    for off, k in ((0, a), (a, b)):
        for i in range(k):
            for j in range(i + 1, k):
                if rng.random() < 0.8:
                    e.append((off + i, off + j))
                    w.append(int(rng.integers(1, 51)))
        for i in range(k - 1):  # a path keeps each blob connected
            e.append((off + i, off + i + 1))
            w.append(int(rng.integers(10, 51)))
    for _ in range(int(rng.integers(1, 4))):
        e.append((int(rng.integers(0, a)), a + int(rng.integers(0, b))))
        w.append(int(rng.integers(1, 6)))
    return gg.from_edges(a + b, e, w)


_BLOCK_VARIANTS = [dict(), dict(use_pr=0), dict(whole_max=4, scan_mode=1), dict(whole_max=4, scan_mode=1, use_pr=0),
                   dict(scan_mode=2), dict(scan_mode=2, use_pr=0), dict(whole_max=4, sweep_handoff=1),
                   dict(whole_max=4, sweep_handoff=1, use_pr=0),
                   dict(whole_max=4, sweep_handoff=1, sweep_tail=1),
                   dict(whole_max=4, sweep_handoff=1, sweep_tail=1, use_pr=0),
                   dict(whole_max=4, sweep_handoff=1, sweep_tail=-1, use_pr=0),
                   dict(whole_max=4, sweep_handoff=1, sweep_pull=1, use_pr=0),
                   dict(whole_max=4, sweep_handoff=1, sweep_pull=1, sweep_tail=1),
                   dict(pr_triangle_deg=-64),
                   dict(pq_order=1, use_pr=0), dict(pq_order=2, use_pr=0), dict(pq_order=3),
                   dict(whole_max=4, scan_mode=1, pq_order=2, scan_visits=3, use_pr=0),
                   dict(whole_max=4, scan_mode=1, scan_visits=2),
                   dict(scan_mode=2, pq_order=1, use_pr=0),
                   dict(whole_max=4, sweep_handoff=1, sweep_seg=1, sweep_pull=-1, use_pr=0),
                   dict(whole_max=4, sweep_handoff=1, sweep_seg=1, sweep_pull=-1, sweep_tail=1)]


@pytest.mark.parametrize("opts", _BLOCK_VARIANTS, ids=lambda o: ",".join(f"{k}={v}" for k, v in o.items()) or "default")
def test_round_blocks_keep_every_minimum_cut(opts):
    """Per-step soundness of one round (section "Parallel CAPFOREST", Lemma 2;
    the Padberg-Rinaldi conditions): wherever the bound used exceeds lambda,
    every pair of vertices that the round puts in one block has pair
    connectivity above lambda (no minimum cut is cut), and with the scans
    alone (no tests) at least the bound (each union has q(e) >= the bound
    and q(e) is at most the pair's connectivity)."""
    import paper_1808_05458_amd as mc
    rng = np.random.default_rng(4242 + len(opts))
    graphs = [random_graph(rng, int(rng.integers(4, 17)), float(rng.uniform(0.2, 0.9)),
                           int(rng.choice([1, 5, 50]))) for _ in range(80)]
    graphs += [_two_blobs(rng) for _ in range(80)]  # lambda below the minimum degree
    lams = [oracle.bruteforce(g)[0] for g in graphs]
    conn = [oracle.pair_connectivity(g) for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    checked = 0
    for margin in (None, 1, 7):
        lin = None if margin is None else [l + margin for l in lams]
        announce("round blocks", opts, margin)
        labels, used = mc.debug_first_round(rp, col, w, vo, lhat_in=lin, **opts)
        lab = labels.cpu().numpy()
        for i, g in enumerate(graphs):
            if lams[i] >= used[i]:
                continue
            b = lab[vo[i]:vo[i + 1]]
            same = b[:, None] == b[None, :]
            np.fill_diagonal(same, False)
            c = conn[i][same]
            if c.size == 0:
                continue
            checked += 1
            assert c.min() > lams[i], (i, margin, opts, int(c.min()), lams[i])
            if opts.get("use_pr", 1) == 0:
                assert c.min() >= used[i], (i, margin, opts, int(c.min()), int(used[i]))
    assert checked >= 100, checked


def _shuffle_rows(g, seed):
    """The same graph with every row's entries in a random order."""
    rng = np.random.default_rng(seed)
    col, w = g.col.copy(), g.w.copy()
    for v in range(g.n):
        a, b = int(g.row_ptr[v]), int(g.row_ptr[v + 1])
        p = a + rng.permutation(b - a)
        col[a:b], w[a:b] = g.col[p], g.w[p]
    return gg.Graph(g.n, g.row_ptr.copy(), col, w, g.name + "_shuffled")


def test_range_owned_push_and_row_order():
    """The range-owned push relax (sweep_seg=1: every grid-wide push batch
    relaxed range by range in LDS) on a hub-heavy R-MAT core and a power-law
    core whose rows are in ascending order, and the same options on the same
    graphs with every row shuffled (the segment pass finds a batch row out of
    order, and that batch and the rest of the sweep go to the global form):
    the oracle's lambda and a side that realises it every time."""
    graphs = [gg.rmat(5, 15, 1 << 19, 0.57, 0.19, 0.19, kcore=6, lcc=True, name="rmat15"),
              gg.chung_lu(31, 60000, 2.3, 14.0, 1, 4, kcore=4, lcc=True)]
    for g in graphs:
        assert all(np.all(np.diff(g.col[g.row_ptr[v]:g.row_ptr[v + 1]]) >= 0) for v in range(0, g.n, 97))
        ref, _, _ = oracle.noi(g, 1)
        h = _shuffle_rows(g, 3)
        for opts in [dict(sweep_handoff=1, sweep_seg=1, sweep_pull=-1),
                     dict(sweep_handoff=1, sweep_seg=1, sweep_pull=-1, use_pr=0),
                     dict(sweep_handoff=8, sweep_seg=1, sweep_pull=-1, sweep_tail=-1), dict()]:
            for graph in (g, h):
                announce("range-owned push", graph.name, graph.n, graph.m, ref, opts)
                lam, side, st = solve(graph, **opts)
                assert lam == ref, (graph.name, opts)
                check_side(graph, lam, side)


def test_range_owned_push_in_packed_sweeps():
    """Several graphs above the LDS size swept in one packed solve (their
    sweeps run at once, sharing the segment table in turn), the range-owned
    relax forced, one graph's rows shuffled: every lambda equals the
    oracle's and every side realises it."""
    import paper_1808_05458_amd as mc
    graphs = [gg.rmat(7, 15, 1 << 19, 0.57, 0.19, 0.19, kcore=5, lcc=True, name="rmat15"),
              gg.chung_lu(37, 30000, 2.4, 12.0, 1, 5, kcore=3, lcc=True),
              _shuffle_rows(gg.chung_lu(41, 25000, 2.6, 10.0, 1, 3, kcore=3, lcc=True), 5),
              gg.planted_4096()]
    refs = [oracle.noi(g, 1)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    for opts in [dict(sweep_seg=1, sweep_pull=-1, sweep_handoff=1), dict(sweep_seg=1, sweep_pull=-1),
                 dict(sweep_seg=-1, sweep_handoff=1)]:
        announce("packed range-owned push", packed.n, packed.m, opts)
        lams, sides, st = mc.mincut_batched(rp, col, w, vo, **opts)
        assert list(lams) == refs, opts
        s = sides.cpu().numpy()
        for i, g in enumerate(graphs):
            check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])
