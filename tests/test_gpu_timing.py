"""GPU tests of the kernel-class timing used by bench.py's roofline: every
class is timed by default; mc_timing_focus limits the events to one class;
the classes are read after the timed solves (mc_timing_get), and the
solves' results do not depend on timing."""
import pytest

import graphgen as gg
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
    mc.timing_focus(None)
    mc.timing_reset()


def test_focus_limits_timing_to_one_class():
    import paper_1808_05458_amd as mc
    g = gg.planted_4096()
    rp, col, w = mc.to_device(g, "cuda")
    announce("timing", g.n, g.m)
    mc.timing_focus(None)
    mc.timing_reset()
    lam0, side0, _ = mc.mincut(rp, col, w)
    for _ in range(2):
        lam, side, _ = mc.mincut(rp, col, w, timing=1)
        assert lam == lam0
        check_side(g, lam, side.cpu().numpy()[: g.n])
    every = mc.timing()
    names = {c["name"] for c in every}
    assert len(names) >= 5 and all(c["launches"] > 0 and c["ms"] > 0 for c in every)
    dom = max(every, key=lambda c: c["ms"])["name"]
    mc.timing_reset()
    mc.timing_focus(dom)
    for _ in range(3):
        lam, _, _ = mc.mincut(rp, col, w, timing=1)
        assert lam == lam0
    only = mc.timing()
    assert [c["name"] for c in only] == [dom]
    assert only[0]["launches"] > 0 and only[0]["ms"] > 0
    mc.timing_focus(None)
    mc.timing_reset()
    assert mc.timing() == []
