"""The entry point that allocates nothing (mc_mincut_noalloc) against the
entry point it is a variant of (mc_mincut), through the C ABI: lambda equal
(and equal to the oracle), every side realising it, on two calls in a row,
the second on a smaller graph; then its limits."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from gpu_util import announce, check_side

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_05458_amd as mc
    mc._load()
    yield


def _both(g, **opts):
    import torch
    import paper_1808_05458_amd as mc
    rp, col, w = mc.to_device(g, "cuda")
    side = torch.full((g.n,), 7, dtype=torch.uint8, device="cuda")
    lam_na = mc.mincut_noalloc(rp, col, w, side, **opts)
    torch.cuda.synchronize()
    lam, side_ref, _ = mc.mincut(rp, col, w, **opts)
    return lam_na, side.cpu().numpy(), lam, side_ref.cpu().numpy()[: g.n]


def test_noalloc_equals_mincut_on_two_calls_in_a_row():
    # a larger graph first, then a smaller one: the second call must not see
    # the first call's contents of the shared array
    first = gg.chung_lu(61, 80000, 2.5, 16.0, 1, 9, kcore=3, lcc=True, name="cl80k")
    second = gg.planted_4096()
    for g in (first, second):
        ref = oracle.noi(g, 1)[0]
        announce("noalloc", g.name, g.n, g.m)
        lam_na, side_na, lam, side = _both(g)
        assert lam_na == lam == ref, (g.name, lam_na, lam, ref)
        check_side(g, lam_na, side_na)
        check_side(g, lam, side)


def test_noalloc_options_and_small_graphs():
    rng = np.random.default_rng(17)
    for t in range(20):
        n = int(rng.integers(2, 40))
        e = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.3]
        e += [(i, i + 1) for i in range(n - 1)]
        g = gg.from_edges(n, e, rng.integers(1, 20, size=len(e)))
        ref = oracle.stoer_wagner(g)[0]
        for opts in [dict(), dict(whole_max=4, sweep_handoff=1), dict(scan_mode=1, whole_max=4),
                     dict(whole_max=4, sweep_handoff=1, sweep_seg=1, sweep_pull=-1)]:
            lam_na, side_na, lam, _ = _both(g, **opts)
            assert lam_na == lam == ref, (t, opts)
            check_side(g, lam_na, side_na)


def test_noalloc_limits():
    import paper_1808_05458_amd as mc
    g = gg.complete(6)
    rp, col, w = mc.to_device(g, "cuda")
    for bad in [dict(use_viecut=1)]:
        with pytest.raises(mc.MincutError) as e:
            mc.mincut_noalloc(rp, col, w, **bad)
        assert e.value.code == mc.MC_EINVAL
    # a graph whose workspace exceeds the fixed array: refused before any work
    big = gg.chung_lu_4m_8core(19)
    assert mc.workspace_bytes(big.n, big.nnz, 1) > 64 << 20
    rp, col, w = mc.to_device(big, "cuda")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut_noalloc(rp, col, w)
    assert e.value.code == mc.MC_ETOOBIG
    # and a good call afterwards
    assert mc.mincut_noalloc(*mc.to_device(gg.complete(7, 2), "cuda")) == 12
