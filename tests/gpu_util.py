"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np

import graphgen as gg
import oracle


def solve(g, **opts):
    import paper_1808_05458_amd as mc
    rp, col, w = mc.to_device(g, "cuda")
    lam, side, stats = mc.mincut(rp, col, w, **opts)
    return lam, side.cpu().numpy()[: g.n], stats


def check_side(g, lam, side):
    side = np.asarray(side)
    assert side[0] == 0, "side must be normalised so that vertex 0 is on side 0"
    assert 0 < int(side.sum()) < g.n, "side must be a non-empty proper subset"
    assert oracle.cut_value(g, side) == lam, "side's recomputed cut weight must equal lambda"


def announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def random_graph(rng, n, density, wmax, connected=True):
    iu = np.triu_indices(n, 1)
    keep = rng.random(len(iu[0])) < density
    e = np.stack([iu[0][keep], iu[1][keep]], 1)
    if connected:
        perm = rng.permutation(n)
        e = np.concatenate([e, np.stack([perm[:-1], perm[1:]], 1)])
    if len(e) == 0:
        e = np.array([[0, 1]])
    ws = rng.integers(1, wmax + 1, size=len(e))
    return gg.from_edges(n, e, ws)
