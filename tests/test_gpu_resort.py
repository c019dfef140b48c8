"""The adaptive re-sort of a simulation's rebuilds (the bodies arrive in
the previous build's order, nearly sorted after a short step: Sec. 4.4)
against the full radix sort: the same trees bit for bit, step after step,
whether few or many bodies move."""
import numpy as np
import pytest
import torch

from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, say

pytestmark = pytest.mark.gpu

FIELDS = ["keys", "perm", "hkey", "level", "begin", "count", "next", "parent", "cmask",
          "mass", "com", "quad"]


def _trees(ctx, pos, vel, mass, leaf, dt, steps, mode, curve, opts):
    B.bh_ctx_set_sort(ctx, mode)
    B.bh_ctx_set_curve(ctx, curve)
    P, V, M = (torch.from_numpy(x).cuda() for x in (pos, vel, mass))
    B.bh_sim_init(ctx, P, V, M, leaf, 0.5, 0.005, opts)
    out = []
    for _ in range(steps):
        B.bh_leapfrog_step(ctx, dt)
        out.append(B.bh_tree_export(B.bh_sim_tree(ctx)))
    x = torch.empty_like(P)
    B.bh_sim_get(ctx, x, None, None)
    torch.cuda.synchronize()
    B.bh_ctx_set_sort(ctx, B.BH_SORT_ADAPTIVE)
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    return out, x.cpu().numpy()


# adaptive: whether the movers stay under a quarter of the bodies (the
# coincident clusters scatter, and a long step moves most bodies: both fall
# back to the full sort)
@pytest.mark.parametrize("kind,n,leaf,dt,curve,dtype,adaptive", [
    ("plummer", 30000, 16, 5e-4, B.BH_CURVE_MORTON, np.float32, True),
    ("plummer", 30000, 16, 5e-4, B.BH_CURVE_HILBERT, np.float32, True),
    ("clumpy", 20000, 8, 2e-3, B.BH_CURVE_MORTON, np.float32, True),
    ("coincident", 3000, 4, 1e-3, B.BH_CURVE_MORTON, np.float64, False),
    ("plummer", 8000, 1, 1e-3, B.BH_CURVE_HILBERT, np.float64, True),
    ("plummer", 20000, 16, 0.2, B.BH_CURVE_MORTON, np.float32, False),
])
def test_adaptive_resort_equals_full_sort(ctx, kind, n, leaf, dt, curve, dtype, adaptive):
    say(f"re-sort: {kind} n={n} leaf={leaf} dt={dt} curve={curve}")
    pos, vel, mass = case_bodies(kind, n, 9, dtype)
    opts = B.force_opts(walk=B.BH_WALK_GROUP)
    ad, xa = _trees(ctx, pos, vel, mass, leaf, dt, 4, B.BH_SORT_ADAPTIVE, curve, opts)
    fu, xf = _trees(ctx, pos, vel, mass, leaf, dt, 4, B.BH_SORT_FULL, curve, opts)
    moved = [t["movers"] for t in ad]
    say(f"  movers per step (adaptive): {moved}")
    assert all(t["movers"] == -1 for t in fu)
    for s, (a, f) in enumerate(zip(ad, fu)):
        for k in FIELDS:
            assert np.array_equal(a[k], f[k]), (s, k)
    assert np.array_equal(xa, xf)
    if adaptive:
        assert all(0 <= m < n // 4 for m in moved)  # the adaptive path ran
    else:
        assert all(m == -1 or 0 <= m < n // 4 for m in moved)


def test_simulation_repeats_bit_for_bit(ctx):
    """Two simulations of the same bodies on one context, one after the
    other, give the same trajectory: nothing of the first (such as the group
    walk's fallback predictions) carries into the second."""
    pos, vel, mass = case_bodies("plummer", 20000, 12, np.float32)
    opts = B.force_opts(walk=B.BH_WALK_GROUP)
    (_, x1), (_, x2) = (_trees(ctx, pos, vel, mass, 16, 1e-3, 3, B.BH_SORT_ADAPTIVE,
                               B.BH_CURVE_MORTON, opts) for _ in range(2))
    assert np.array_equal(x1, x2)


def test_sort_mode_is_checked(ctx):
    with pytest.raises(B.BHError) as e:
        B.bh_ctx_set_sort(ctx, 5)
    assert e.value.code == B.BH_E_INVALID
