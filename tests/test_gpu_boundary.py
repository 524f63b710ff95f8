"""GPU tests of the boundary's calling conventions: calls on different
streams from different host threads are independent (each stream has its
own workspace), a caller-lent workspace gives the same results without a
library allocation, and the opt-in symmetry check rejects an asymmetric
CSR.  lambda is compared with the oracle exactly; sides by their weight."""
import threading

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


def test_two_streams_at_once_equal_their_solo_results():
    import torch
    import paper_1808_05458_amd as mc
    graphs = [gg.chung_lu_4m_8core(19), gg.chung_lu(41, 150000, 2.5, 16.0, 1, 9, kcore=3, lcc=True),
              gg.bridged_8cores(14, 2), gg.planted_4096()]
    refs = [oracle.noi(g, 1)[0] for g in graphs]
    dev = [mc.to_device(g, "cuda") for g in graphs]
    streams = [torch.cuda.Stream() for _ in graphs]
    solo = []
    for g, d, s in zip(graphs, dev, streams):
        announce("solo", g.name, g.n)
        lam, side, _ = mc.mincut(*d, stream=s)
        torch.cuda.synchronize()
        solo.append(lam)
    assert solo == refs
    out = [None] * len(graphs)
    errors = []

    def work(i):
        try:
            for _ in range(3):
                lam, side, _ = mc.mincut(*dev[i], stream=streams[i])
                out[i] = (lam, side)
        except Exception as e:  # reported below
            errors.append(e)

    announce("concurrent", len(graphs), "streams")
    th = [threading.Thread(target=work, args=(i,)) for i in range(len(graphs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for i, g in enumerate(graphs):
        lam, side = out[i]
        assert lam == refs[i], (g.name, lam, refs[i])
        check_side(g, lam, side.cpu().numpy()[: g.n])


def test_caller_workspace():
    import torch
    import paper_1808_05458_amd as mc
    graphs = [gg.batch_graph(i) for i in range(300, 340)]
    refs = [oracle.noi(g, 1)[0] for g in graphs]
    packed, vo, eo = gg.pack(graphs)
    rp, col, w = mc.to_device(packed, "cuda")
    need = mc.workspace_bytes(packed.n, packed.nnz, len(graphs))
    buf = torch.empty(need, dtype=torch.uint8, device="cuda")
    announce("caller workspace", need)
    for opts in [dict(), dict(whole_max=64), dict(scan_mode=1, whole_max=64)]:
        lams, sides, _ = mc.mincut_batched(rp, col, w, vo, workspace=buf.data_ptr(), workspace_bytes=need, **opts)
        assert list(lams) == refs, opts
        s = sides.cpu().numpy()
        for i, g in enumerate(graphs):
            check_side(g, int(lams[i]), s[vo[i]:vo[i + 1]])
    # too small: rejected before any kernel runs
    with pytest.raises(mc.MincutError) as e:
        mc.mincut_batched(rp, col, w, vo, workspace=buf.data_ptr(), workspace_bytes=need - 256)
    assert e.value.code == mc.MC_EINVAL
    # the clustering bound needs its own part after the core arrays
    vc = mc.viecut_workspace_bytes(packed.n, packed.nnz, len(graphs))
    big = torch.empty(need + vc, dtype=torch.uint8, device="cuda")
    lams, _, _ = mc.mincut_batched(rp, col, w, vo, use_viecut=1, workspace=big.data_ptr(),
                                   workspace_bytes=need + vc)
    assert list(lams) == refs
    with pytest.raises(mc.MincutError) as e:
        mc.mincut_batched(rp, col, w, vo, use_viecut=1, workspace=buf.data_ptr(), workspace_bytes=need)
    assert e.value.code == mc.MC_EINVAL


def test_symmetry_check():
    import torch
    import paper_1808_05458_amd as mc
    rng = np.random.default_rng(5)
    g = random_graph(rng, 300, 0.05, 9)
    rp, col, w = mc.to_device(g, "cuda")
    announce("symmetry: symmetric input")
    lam, side, _ = mc.mincut(rp, col, w, validate=1)
    assert lam == oracle.noi(g, 1)[0]
    # repeated entries are symmetric when both directions add up alike
    h = gg.from_edges(4, [(0, 1), (0, 1), (1, 2), (2, 3), (3, 0), (1, 1)], [2, 3, 4, 4, 4, 7])
    lam, _, _ = mc.mincut(*mc.to_device(h, "cuda"), validate=1)
    assert lam == oracle.bruteforce(h)[0]
    # one entry's weight changed: the pair's two directions differ
    w2 = w.clone()
    w2[7] += 1
    announce("symmetry: changed weight")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rp, col, w2, validate=1)
    assert e.value.code == mc.MC_EINVAL
    # one entry pointing elsewhere: a pair with one direction only
    u = int(np.searchsorted(g.row_ptr, 11, side="right") - 1)
    c2 = col.clone()
    c2[11] = (int(c2[11]) + 1) % g.n if (int(c2[11]) + 1) % g.n != u else (int(c2[11]) + 2) % g.n
    announce("symmetry: moved entry")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rp, c2, w, validate=1)
    assert e.value.code == mc.MC_EINVAL
    # packed graphs are checked too
    packed, vo, eo = gg.pack([gg.complete(6), gg.cycle(9, 3)])
    prp, pcol, pw = mc.to_device(packed, "cuda")
    lams, _, _ = mc.mincut_batched(prp, pcol, pw, vo, validate=1)
    assert list(lams) == [5, oracle.bruteforce(gg.cycle(9, 3))[0]]
    pw[int(packed.row_ptr[7])] += 3
    with pytest.raises(mc.MincutError) as e:
        mc.mincut_batched(prp, pcol, pw, vo, validate=1)
    assert e.value.code == mc.MC_EINVAL


def test_unaligned_entry_arrays():
    """Entry arrays that are not 16-byte aligned (views one to three entries
    into larger buffers, as a caller may pass): the same lambda as the
    oracle, single and packed, sides that realise it, and a column out of
    range is still refused."""
    import torch
    import paper_1808_05458_amd as mc
    g = gg.chung_lu(43, 20000, 2.5, 12.0, 1, 9, kcore=2, lcc=True)
    assert g.nnz % 512 != 0  # a ragged last chunk
    ref = oracle.noi(g, 1)[0]
    rp, col, w = mc.to_device(g, "cuda")

    def shifted(t, off, fill):
        buf = torch.full((t.numel() + off,), fill, dtype=t.dtype, device=t.device)
        buf[off:] = t
        return buf, buf[off:]

    for off_c, off_w in ((1, 1), (2, 3), (0, 1), (3, 0)):
        cb, c_v = shifted(col, off_c, 0)
        wb, w_v = shifted(w, off_w, 1)
        assert (c_v.data_ptr() | w_v.data_ptr()) % 16 != 0
        announce("unaligned entry arrays", off_c, off_w)
        lam, side, _ = mc.mincut(rp, c_v, w_v)
        assert lam == ref
        check_side(g, lam, side.cpu().numpy())
    # packed: two graphs, both arrays one entry off
    h = gg.cycle(9, 3)
    packed, vo, eo = gg.pack([g, h])
    prp, pcol, pw = mc.to_device(packed, "cuda")
    _, pc_v = shifted(pcol, 1, 0)
    _, pw_v = shifted(pw, 1, 1)
    announce("unaligned entry arrays, packed")
    lams, sides, _ = mc.mincut_batched(prp, pc_v, pw_v, vo)
    assert list(lams) == [ref, oracle.bruteforce(h)[0]]
    s = sides.cpu().numpy()
    check_side(g, int(lams[0]), s[vo[0]:vo[1]])
    # a column out of range in an unaligned array
    cb, c_v = shifted(col, 1, 0)
    cb[1 + 777] = g.n + 5
    _, w_v = shifted(w, 1, 1)
    announce("unaligned entry arrays, bad column")
    with pytest.raises(mc.MincutError) as e:
        mc.mincut(rp, c_v, w_v)
    assert e.value.code == mc.MC_EINVAL
