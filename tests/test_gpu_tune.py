"""GPU tests of the batched form's launch shapes and its autotuner: every
shape (LDS-sweep threads and workgroups per CU, radix-sort tile) gives the
oracle's lambdas and sides that realise them, and the autotuner returns one
of the candidate shapes, whose solve again equals the oracle."""
import json
import os

import pytest

import graphgen as gg
import oracle
from gpu_util import announce, check_side

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


@pytest.fixture(scope="module")
def sample():
    # 400 graphs of the 4096-graph batch, with their stored oracle lambdas
    import paper_1808_05458_amd as mc
    gold = json.load(open(os.path.join(GOLDEN, "workloads.json")))["batch_4096"]["lambdas"]
    graphs = [gg.batch_graph(i) for i in range(400)]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    return graphs, gold[:400], vo, (rp, col, w)


def _check(graphs, refs, vo, lams, sides):
    assert list(lams) == refs
    s = sides.cpu().numpy()
    for i, g in enumerate(graphs):
        check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])


@pytest.mark.parametrize("threads,groups,tile", [(128, 1, 2048), (128, 3, 4096), (256, 1, 8192),
                                                 (256, 2, 2048), (256, 3, 4096), (512, 2, 8192),
                                                 (512, 3, 4096)])
def test_launch_shapes_equal_oracle(sample, threads, groups, tile):
    import paper_1808_05458_amd as mc
    graphs, refs, vo, (rp, col, w) = sample
    announce("shape", threads, groups, tile)
    lams, sides, st = mc.mincut_batched(rp, col, w, vo, sweep_threads=threads, sweep_groups=groups,
                                        sort_tile=tile)
    _check(graphs, refs, vo, lams, sides)


def test_contraction_sort_tiles_on_a_large_graph():
    # the radix sort's tile on a single graph with many entries per round
    import paper_1808_05458_amd as mc
    g = gg.planted_4096()
    ref = oracle.noi(g, 1)[0]
    rp, col, w = mc.to_device(g, "cuda")
    for tile in (2048, 4096, 8192):
        announce("sort tile", tile)
        lam, side, st = mc.mincut(rp, col, w, sort_tile=tile, whole_max=16)
        assert lam == ref
        check_side(g, lam, side.cpu().numpy()[: g.n])


def test_autotuner_picks_a_candidate_that_equals_oracle(sample):
    import paper_1808_05458_amd as mc
    graphs, refs, vo, (rp, col, w) = sample
    announce("autotune", len(graphs))
    best, rep = mc.tune_batched(rp, col, w, vo, reps=1)
    assert rep["candidates"] >= 5 and rep["reps"] == 1
    assert rep["sweep_threads"] in (128, 256, 512)
    assert rep["sweep_groups"] in (2, 3)
    assert rep["sort_tile"] in (2048, 4096, 8192)
    assert rep["pr_triangle_deg"] in (0, 64, -64) and rep["pq_order"] in (0, 1, 2, 3)
    assert 0 < rep["best_ms"] <= rep["default_ms"]
    lams, sides, st = mc.mincut_batched(rp, col, w, vo, opts=best)
    _check(graphs, refs, vo, lams, sides)


def test_tuned_settings_are_kept_per_size_class(sample):
    """mc_tune_batched stores its choice under the batch's size class (bit
    lengths of graph count, vertex total, entry total); solves with
    use_tuned=1 in that class take it and still equal the oracle; another
    class finds nothing; mc_tune_clear forgets."""
    import paper_1808_05458_amd as mc
    graphs, refs, vo, (rp, col, w) = sample
    n, nnz = rp.numel() - 1, col.numel()
    mc.tune_clear()
    assert mc.tune_lookup(n, nnz, vo) is None
    best, rep = mc.tune_batched(rp, col, w, vo, reps=1)
    got = mc.tune_lookup(n, nnz, vo)
    assert got is not None
    for k in ("sweep_threads", "sweep_groups", "sort_tile", "pr_triangle_deg", "pq_order"):
        assert getattr(got, k) == getattr(best, k), k
    # the same class: a vertex and two entries fewer, same bit lengths
    if (n - 1).bit_length() == n.bit_length() and (nnz - 2).bit_length() == nnz.bit_length():
        assert mc.tune_lookup(n - 1, nnz - 2, vo) is not None
    # another class: twice the entries
    assert mc.tune_lookup(n, 2 * nnz, vo) is None
    announce("tuned solve", rep)
    lams, sides, st = mc.mincut_batched(rp, col, w, vo, use_tuned=1)
    _check(graphs, refs, vo, lams, sides)
    mc.tune_clear()
    assert mc.tune_lookup(n, nnz, vo) is None
