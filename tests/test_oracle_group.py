"""Pins for the oracle's group walk (one acceptance decision per group of
consecutive sorted bodies)."""
import numpy as np

import oracle
from paper_2203_08966_amd import workloads as W

# a work cap no group reaches: every group keeps its group decisions
NO_CAP = 1 << 40


def _tree(n=6000, seed=3, leaf=8, kind="plummer"):
    b = W.plummer(n, seed) if kind == "plummer" else W.clumpy(n, seed, n_clumps=6)
    return b, oracle.build_all(b.pos, b.mass, leaf)


def test_group_of_one_is_the_per_body_walk():
    """G = 1: the box is the body, d_g = d; below theta = 1/sqrt(3) no
    accepted cell can contain the body, so this is the walk of Sec. 3."""
    b, bb = _tree()
    for theta in (0.3, 0.5):
        g = oracle.walk_group(bb, 0.01, group=1, theta=theta, cap=NO_CAP, split=False)
        w = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], theta, 0.01)
        np.testing.assert_array_equal(g.npp, w.npp)
        np.testing.assert_array_equal(g.npc, w.npc)
        np.testing.assert_allclose(g.acc, w.acc, rtol=1e-13, atol=0)
        np.testing.assert_allclose(g.phi, w.phi, rtol=1e-13, atol=0)


def test_group_of_one_budget_is_the_per_body_budget_walk():
    b, bb = _tree(seed=4)
    kc = oracle.cell_kc(bb)
    an = np.linalg.norm(oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"],
                                    0.4, 0.01).acc, axis=1)
    g = oracle.walk_group(bb, 0.01, group=1, mode=1, theta_max=0.9, tau=1e-3, kc=kc, anorm=an,
                          cap=NO_CAP, split=False)
    w = oracle.walk_kc(bb, 0.01, 0.9, 1e-3, kc, an)
    np.testing.assert_array_equal(g.npp, w.npp)
    np.testing.assert_array_equal(g.npc, w.npc)
    np.testing.assert_allclose(g.acc, w.acc, rtol=1e-13, atol=0)


def test_every_body_accounted_once_and_groups_only_tighten():
    """Every other body is covered exactly once by each group walk; a group
    decision accepts a cell only where each member's own test would, so the
    error falls and the work rises against the per-body walk."""
    b, bb = _tree(8000, 5, 8, "clumpy")
    n = len(b.mass)
    direct, _ = oracle.direct(bb["spos"], bb["smass"], 0.01)
    w = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.55, 0.01)

    def rms(a):
        e = np.linalg.norm(a - direct, axis=1) / np.linalg.norm(direct, axis=1)
        return np.sqrt(np.mean(e * e))
    prev = None
    for G in (1, 8, 64):
        g = oracle.walk_group(bb, 0.01, group=G, theta=0.55, split=False, cap=NO_CAP)
        assert np.all(g.ncov == n - 1)
        if prev is not None:
            assert np.all(g.npp + g.npc >= 0)
            assert rms(g.acc) <= rms(prev.acc) * 1.0001
            assert (g.npp + g.npc).sum() >= (prev.npp + prev.npc).sum()
        prev = g
    assert rms(prev.acc) < rms(w.acc)


def test_one_group_holding_everything_is_the_direct_sum():
    """A single group whose box covers every cell opens everything: the
    direct sum, particle-particle only."""
    b, bb = _tree(700, 6)
    g = oracle.walk_group(bb, 0.02, group=700, theta=0.9, split=False, cap=NO_CAP)
    d, phi = oracle.direct(bb["spos"], bb["smass"], 0.02)
    assert np.all(g.npc == 0) and np.all(g.npp == 699)
    np.testing.assert_allclose(g.acc, d, rtol=1e-12, atol=1e-14)


def test_ragged_target_range_and_box_geometry():
    """Groups start at t0; the last one is ragged.  Hand check of one
    decision: a far, light cell against a two-body group box."""
    b, bb = _tree(3000, 7)
    g_all = oracle.walk_group(bb, 0.01, group=64, theta=0.7, cap=6144, split=True)
    g_sub = oracle.walk_group(bb, 0.01, group=64, theta=0.7, target_range=(128, 1000),
                              cap=6144, split=True)
    # groups [128, 192) ... [896, 960) coincide; [960, 1000) is ragged
    np.testing.assert_array_equal(g_sub.npc[:832], g_all.npc[128:960])
    np.testing.assert_allclose(g_sub.acc[:832], g_all.acc[128:960], rtol=1e-13, atol=0)
    assert np.all(g_sub.ncov == 2999)
    rag = oracle.walk_group(bb, 0.01, group=40, theta=0.7, target_range=(960, 1000),
                            cap=6144, split=True)
    np.testing.assert_array_equal(g_sub.npc[832:], rag.npc)
    # group box: bodies at x = 0.1 and 0.3 (y = z = 0.5).  Bodies at
    # (0.8, 0.5, 0.5) and (0.8, 0.7, 0.5) share the level-2 cube
    # [0.75, 1) x [0.5, 0.75) x [0.5, 0.75) (side 0.25) and split below it;
    # their COM (0.8, 0.6, 0.5) lies at d_g = sqrt(0.26) from the box (the
    # box centre is farther, sqrt(0.37)).  Above theta = 0.25/d_g the cell is
    # one particle-cell term for both group bodies, below it two
    # particle-particle terms.
    pos = np.array([[0.1, 0.5, 0.5], [0.3, 0.5, 0.5], [0.8, 0.5, 0.5], [0.8, 0.7, 0.5],
                    [0.0, 0.0, 0.0], [0.99, 0.99, 0.99]])
    mass = np.array([1.0, 1.0, 0.5, 0.5, 1e-9, 1e-9])
    tb = oracle.build_all(pos, mass, 1)
    assert tb["L"] == 1.0 and np.all(tb["lo"] == 0.0)
    rank = np.empty(6, dtype=np.int64)
    rank[tb["perm"]] = np.arange(6)
    r0 = min(rank[0], rank[1])
    assert abs(rank[0] - rank[1]) == 1
    lim = 0.25 / np.sqrt(0.26)
    for theta, accepted in ((lim * 1.001, True), (lim * 0.999, False)):
        r = oracle.walk_group(tb, 0.0, group=2, theta=theta, target_range=(r0, r0 + 2),
                              cap=NO_CAP, split=True)
        assert np.all(r.ncov == 5)
        assert np.all(r.npc == (1 if accepted else 0))
        assert np.all(r.npp == (3 if accepted else 5))
        # the box lies on the plane y = 0.5, a face of the cube tested, but
        # the x axis separates them by far: no decision is near a threshold
        assert np.all(r.flag == 0)
    # within a relative 1e-5 of the angle threshold the group is flagged
    r = oracle.walk_group(tb, 0.0, group=2, theta=lim * (1 + 1e-7), target_range=(r0, r0 + 2),
                          cap=NO_CAP, split=True)
    assert np.all(r.flag == 1)


def test_work_cap_falls_back_to_the_per_body_walk():
    """A cap below every group's work turns the group walk into the per-body
    walk (both modes); an unreachable cap changes nothing."""
    b, bb = _tree(5000, 8, 8, "clumpy")
    theta = 0.5
    w = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], theta, 0.01)
    g = oracle.walk_group(bb, 0.01, group=64, theta=theta, split=False, cap=1)
    np.testing.assert_array_equal(g.npc, w.npc)
    np.testing.assert_allclose(g.acc, w.acc, rtol=1e-13, atol=0)
    kc = oracle.cell_kc(bb)
    an = np.linalg.norm(w.acc, axis=1)
    gb = oracle.walk_group(bb, 0.01, group=64, mode=1, theta_max=0.9, tau=1e-2, kc=kc,
                           anorm=an, cap=1, split=False)
    wb = oracle.walk_kc(bb, 0.01, 0.9, 1e-2, kc, an)
    np.testing.assert_array_equal(gb.npp, wb.npp)
    np.testing.assert_allclose(gb.acc, wb.acc, rtol=1e-13, atol=0)
    big = oracle.walk_group(bb, 0.01, group=64, theta=theta, split=False, cap=1 << 62)
    # the cap splits groups by their work: each group either keeps the group
    # walk or takes the per-body counts
    mid = oracle.walk_group(bb, 0.01, group=64, theta=theta, split=False, cap=3000)
    # (a group's work is npp + npc + 1 for each of its bodies: the body's
    # own particle-particle cell counts it too)
    work = big.npp + big.npc + 1
    fell = 0
    for k0 in range(0, 5000, 64):
        sl = slice(k0, min(k0 + 64, 5000))
        assert np.all(work[sl] == work[k0])
        src = w if work[k0] > 3000 else big
        fell += work[k0] > 3000
        np.testing.assert_array_equal(mid.npc[sl], src.npc[sl])
    assert 0 < fell < 5000 // 64


def _fill(rng, lo, hi, hole_lo, hole_hi, n):
    """n points uniform in the cube [lo, hi)^3 outside [hole_lo, hole_hi)^3."""
    out = []
    while len(out) < n:
        p = lo + (hi - lo) * rng.random(3)
        if not np.all((p >= hole_lo) & (p < hole_hi)):
            out.append(p)
    return np.array(out)


def test_split_cuts_a_straddling_group_at_the_jump():
    """Two clusters of 8 bodies, at the upper corner of the root's first
    octant and the lower corner of its last, are consecutive on the
    space-filling curve; filler bodies around them make their leaves deep
    (level 5 or more).  As one group of 16 their common cell is the root, more than
    two levels above their leaves, so the group is cut exactly between the
    clusters and each half is walked as a group of its own.  A cluster
    alone is not cut."""
    rng = np.random.default_rng(9)
    a = 0.497 + 0.0025 * rng.random((8, 3))          # octant 0, upper corner
    c = 0.5005 + 0.0025 * rng.random((8, 3))         # octant 7, lower corner
    fa = _fill(rng, 0.375, 0.5, 0.49, 0.5, 300)       # before a on the curve
    fc = _fill(rng, 0.5, 0.625, 0.5, 0.51, 300)       # after c
    pos = np.concatenate([a, c, fa, fc, [[0.01, 0.01, 0.01], [0.99, 0.99, 0.99]]])
    mass = np.full(len(pos), 1.0 / len(pos))
    bb = oracle.build_all(pos, mass, 8)
    rank = np.empty(len(pos), dtype=np.int64)
    rank[bb["perm"]] = np.arange(len(pos))
    ra, rc = np.sort(rank[:8]), np.sort(rank[8:16])
    assert ra[-1] + 1 == rc[0]                          # adjacent on the curve
    lv = oracle.leaf_levels(bb)
    assert lv[ra].min() >= 5 and lv[rc].min() >= 5           # deep leaves
    g0 = ra[0]
    kw = dict(group=16, theta=0.6, cap=NO_CAP)
    sp = oracle.walk_group(bb, 0.0, target_range=(g0, g0 + 16), split=True, **kw)
    nosp = oracle.walk_group(bb, 0.0, target_range=(g0, g0 + 16), split=False, **kw)
    h1 = oracle.walk_group(bb, 0.0, target_range=(g0, g0 + 8), split=False, **kw)
    h2 = oracle.walk_group(bb, 0.0, target_range=(g0 + 8, g0 + 16), split=False, **kw)
    np.testing.assert_array_equal(sp.npc, np.concatenate([h1.npc, h2.npc]))
    np.testing.assert_array_equal(sp.npp, np.concatenate([h1.npp, h2.npp]))
    np.testing.assert_allclose(sp.acc, np.concatenate([h1.acc, h2.acc]), rtol=1e-14, atol=0)
    assert (sp.npp + sp.npc).sum() < (nosp.npp + nosp.npc).sum()
    # one cluster as its own group: no cut
    one = oracle.walk_group(bb, 0.0, target_range=(g0, g0 + 8), split=True, **kw)
    np.testing.assert_array_equal(one.npc, h1.npc)
