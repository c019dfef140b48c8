"""Hand-computed pins of the error-budget acceptance test (the library's
criterion beside the opening angle of Sec. 3): a multi-body cell C is
accepted iff l^2 < theta_max^2 d^2, the body lies outside C, and
k_C M l^3 < tau |a_i| d^5 (k_C = 1 here).  In the group walk d is the
distance d_g from C's centre of mass to the group's bounding box and |a_i|
the smallest norm of the group's bodies.

Each pin places a two-mass cell (unequal masses, so the COM is not the
midpoint) at a distance that is neither 1 nor its side, computes the
threshold by hand, and checks that the decision flips between a relative
1e-3 below and above it.  A wrong power of d (d^4 for d^5), of the side
(l^2 for l^3), the mass squared, the body's own norm in place of the
group's smallest, or the body distance in place of the box distance all
move the threshold by far more than 1e-3 and fail here."""
import numpy as np
import pytest

import oracle

# Level-1 octant 0 of the root cube [0, 2)^3 holds the corner pin O and the
# two group bodies A, B; octant 7 holds the far corner pin Z and the cell
# C = [1.5, 2) x [1, 1.5) x [1, 1.5) (side 0.5, level 2) with C1 and C2.
O = (0.0, 0.0, 0.0)
A = (0.2, 0.7, 0.3)
B = (0.6, 0.4, 0.4)
C1 = (1.6, 1.1, 1.2)
C2 = (1.8, 1.4, 1.04)
Z = (1.98, 1.98, 1.98)
MC1, MC2 = 0.5, 0.25
SIDE = 0.5


def _system():
    pos = np.array([O, A, B, C1, C2, Z])
    mass = np.array([1e-9, 1.0, 1.0, MC1, MC2, 1e-9])
    tb = oracle.build_all(pos, mass, 1)
    assert tb["L"] == 2.0 and np.all(tb["lo"] == 0.0)
    rank = np.empty(6, dtype=np.int64)
    rank[tb["perm"]] = np.arange(6)
    # C is one level-2 cell holding exactly C1 and C2
    t = tb["tree"]
    c = [k for k in range(len(t["level"])) if t["level"][k] == 2 and t["count"][k] == 2
         and t["begin"][k] == min(rank[3], rank[4])]
    assert len(c) == 1
    return tb, rank, c[0]


def _com():
    return (MC1 * np.array(C1) + MC2 * np.array(C2)) / (MC1 + MC2)


def _norms(rank, a_of):
    """|a_i| per sorted rank (the walk's input), from a map body -> norm."""
    an = np.ones(6)
    for body, v in a_of.items():
        an[rank[body]] = v
    return an


def test_cell_under_test_in_closed_form():
    tb, rank, c = _system()
    M, com, Q = tb["mom"]
    assert M[c] == MC1 + MC2
    np.testing.assert_allclose(com[c], _com(), rtol=1e-15)
    kc = oracle.cell_kc(tb)
    assert kc[c] == pytest.approx((MC1 + MC2) * SIDE ** 3, rel=1e-15)


def test_per_body_budget_flips_at_hand_threshold():
    """Body A alone: accept C iff (M l^3) < tau |a_A| d^5, d = |A - COM_C|."""
    tb, rank, c = _system()
    kc = oracle.cell_kc(tb)
    a_A = 0.7
    an = _norms(rank, {1: a_A, 2: 5.0})
    d = np.linalg.norm(np.array(A) - _com())
    tau_star = (MC1 + MC2) * SIDE ** 3 / (a_A * d ** 5)
    # the octant-7 cell (side 1, 8x the coefficient) stays rejected here
    for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
        r = oracle.walk_kc(tb, 0.0, 10.0, tau_star * f, kc, an, targets=[rank[1]])
        assert r.ncov[0] == 5
        assert r.npc[0] == (1 if accepted else 0), f
        assert r.npp[0] == (3 if accepted else 5), f
        assert r.flag[0] == 0


def test_per_body_angle_limit_flips_at_side_over_distance():
    """With an unbounded budget the test is l^2 < theta_max^2 d^2: C is the
    first cell to pass as theta_max crosses l/d (octant 7, side 1, is about
    twice that ratio)."""
    tb, rank, c = _system()
    kc = oracle.cell_kc(tb)
    an = _norms(rank, {})
    d = np.linalg.norm(np.array(A) - _com())
    lim = SIDE / d
    for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
        r = oracle.walk_kc(tb, 0.0, lim * f, 1e30, kc, an, targets=[rank[1]])
        assert r.npc[0] == (1 if accepted else 0), f


def test_group_budget_flips_at_hand_threshold():
    """Group {A, B} (consecutive ranks): accept C for both iff
    M l^3 < tau min(|a_A|, |a_B|) d_g^5, with d_g the distance from C's COM
    to the box spanned by A and B."""
    tb, rank, c = _system()
    assert abs(rank[1] - rank[2]) == 1
    r0 = min(rank[1], rank[2])
    kc = oracle.cell_kc(tb)
    a_A, a_B = 1.3, 0.7
    an = _norms(rank, {1: a_A, 2: a_B})
    lo = np.minimum(A, B)
    hi = np.maximum(A, B)
    gap = np.maximum(0.0, np.maximum(lo - _com(), _com() - hi))
    dg = np.linalg.norm(gap)
    # the box's nearest corner is neither body: d_g is well below either
    # body's own distance
    assert dg < 0.95 * min(np.linalg.norm(np.array(A) - _com()),
                          np.linalg.norm(np.array(B) - _com()))
    tau_star = (MC1 + MC2) * SIDE ** 3 / (min(a_A, a_B) * dg ** 5)
    for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
        r = oracle.walk_group(tb, 0.0, group=2, mode=1, theta_max=10.0, tau=tau_star * f,
                              kc=kc, anorm=an, target_range=(r0, r0 + 2), cap=1 << 40,
                              split=False)
        assert np.all(r.ncov == 5)
        assert np.all(r.npc == (1 if accepted else 0)), f
        assert np.all(r.npp == (3 if accepted else 5)), f
        assert np.all(r.flag == 0)


def test_group_angle_limit_uses_the_box_distance():
    tb, rank, c = _system()
    r0 = min(rank[1], rank[2])
    kc = oracle.cell_kc(tb)
    an = _norms(rank, {})
    lo = np.minimum(A, B)
    hi = np.maximum(A, B)
    dg = np.linalg.norm(np.maximum(0.0, np.maximum(lo - _com(), _com() - hi)))
    for mode, kw in ((0, dict(theta=SIDE / dg)), (1, dict(theta_max=SIDE / dg, tau=1e30))):
        for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
            kw2 = {k: v * f if k in ("theta", "theta_max") else v for k, v in kw.items()}
            r = oracle.walk_group(tb, 0.0, group=2, mode=mode, kc=kc, anorm=an,
                                  target_range=(r0, r0 + 2), cap=1 << 40, split=False, **kw2)
            assert np.all(r.npc == (1 if accepted else 0)), (mode, f)


# ---- monopole terms (order 0): the budget also charges each cell the bound
# on the quadrupole term it drops, (7/2) |Q|_F / d^4

def _quad_frobenius_by_hand():
    """|Q|_F of C from its two masses: Q = sum m (3 y y^T - |y|^2 I), y
    about the COM (the convention of Sec. 2.2)."""
    Qm = np.zeros((3, 3))
    for p, m in ((C1, MC1), (C2, MC2)):
        y = np.array(p) - _com()
        Qm += m * (3.0 * np.outer(y, y) - (y @ y) * np.eye(3))
    return np.sqrt(np.sum(Qm * Qm))


def test_dropped_quadrupole_within_its_bound():
    """Far from C the monopole's error is its quadrupole term (the next
    terms fall off faster): in every direction it stays within
    (7/2) |Q|_F / d^4, and in the worst direction reaches a third of it (the
    bound of a cell whose Q has two equal eigenvalues is 3/sqrt(6) of |Q|_F
    along the axis, i.e. 0.35 of the bound)."""
    qf = _quad_frobenius_by_hand()
    rng = np.random.default_rng(3)
    ratios = []
    for _ in range(400):
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        d = 40.0
        x = _com() + d * u
        exact = np.zeros(3)
        for p, m in ((C1, MC1), (C2, MC2)):
            r = np.array(p) - x
            exact += m * r / np.linalg.norm(r) ** 3
        mono = (MC1 + MC2) * (_com() - x) / d ** 3
        ratios.append(np.linalg.norm(exact - mono) / (3.5 * qf / d ** 4))
    assert max(ratios) <= 1.0 + 1e-3
    assert max(ratios) > 0.3


def test_per_body_monopole_budget_flips_at_hand_threshold():
    """Body A alone, monopole terms: accept C iff
    M l^3 + (7/2) |Q|_F d < tau |a_A| d^5."""
    tb, rank, c = _system()
    M, com, Q = tb["mom"]
    qf = _quad_frobenius_by_hand()
    q = Q[c]
    np.testing.assert_allclose(np.sqrt(q[0] ** 2 + q[3] ** 2 + q[5] ** 2
                                       + 2 * (q[1] ** 2 + q[2] ** 2 + q[4] ** 2)), qf, rtol=1e-12)
    kc = oracle.cell_kc(tb)
    a_A = 0.7
    an = _norms(rank, {1: a_A, 2: 5.0})
    d = np.linalg.norm(np.array(A) - _com())
    tau_star = ((MC1 + MC2) * SIDE ** 3 + 3.5 * qf * d) / (a_A * d ** 5)
    # the quadrupole budget alone would accept well below this tau
    assert (MC1 + MC2) * SIDE ** 3 / (a_A * d ** 5) < 0.9 * tau_star
    for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
        r = oracle.walk_kc(tb, 0.0, 10.0, tau_star * f, kc, an, targets=[rank[1]], order=0)
        assert r.npc[0] == (1 if accepted else 0), f
        assert r.npp[0] == (3 if accepted else 5), f
        assert r.flag[0] == 0


def test_group_monopole_budget_flips_at_hand_threshold():
    """Group {A, B}, monopole terms: accept C for both iff
    M l^3 + (7/2) |Q|_F d_g < tau min |a| d_g^5."""
    tb, rank, c = _system()
    r0 = min(rank[1], rank[2])
    kc = oracle.cell_kc(tb)
    a_A, a_B = 1.3, 0.7
    an = _norms(rank, {1: a_A, 2: a_B})
    lo = np.minimum(A, B)
    hi = np.maximum(A, B)
    dg = np.linalg.norm(np.maximum(0.0, np.maximum(lo - _com(), _com() - hi)))
    qf = _quad_frobenius_by_hand()
    tau_star = ((MC1 + MC2) * SIDE ** 3 + 3.5 * qf * dg) / (min(a_A, a_B) * dg ** 5)
    for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
        r = oracle.walk_group(tb, 0.0, group=2, mode=1, theta_max=10.0, tau=tau_star * f,
                              kc=kc, anorm=an, target_range=(r0, r0 + 2), cap=1 << 40,
                              split=False, order=0)
        assert np.all(r.npc == (1 if accepted else 0)), f
        assert np.all(r.npp == (3 if accepted else 5)), f
        assert np.all(r.flag == 0)


# ---- mixed order: per cell the monopole where M l^3 + (7/2) |Q|_F d <
# tau a d^5, else the quadrupole where M l^3 < tau a d^5, else open

def _mixed_thresholds(a, d):
    qf = _quad_frobenius_by_hand()
    kc = (MC1 + MC2) * SIDE ** 3
    return kc / (a * d ** 5), (kc + 3.5 * qf * d) / (a * d ** 5)


def test_per_body_mixed_order_picks_the_cheaper_term():
    """Body A: above the monopole threshold C gives a monopole term, between
    the two thresholds a quadrupole term, below both it is opened; each
    accepted term is the one the walk of that single order computes."""
    tb, rank, c = _system()
    kc = oracle.cell_kc(tb)
    a_A = 0.7
    an = _norms(rank, {1: a_A, 2: 5.0})
    d = np.linalg.norm(np.array(A) - _com())
    tau_q, tau_m = _mixed_thresholds(a_A, d)
    assert tau_q < 0.9 * tau_m
    tau_mid = np.sqrt(tau_q * tau_m)
    args = (tb, 0.0, 10.0)
    cases = ((tau_m * (1 + 1e-3), 1, 0, 0), (tau_m * (1 - 1e-3), 1, 1, 2),
             (tau_mid, 1, 1, 2), (tau_q * (1 + 1e-3), 1, 1, 2), (tau_q * (1 - 1e-3), 0, 0, None))
    for tau, npc, npq, same_as in cases:
        r = oracle.walk_kc(*args, tau, kc, an, targets=[rank[1]], order=oracle.ORDER_MIXED)
        assert (r.npc[0], r.npq[0], r.flag[0]) == (npc, npq, 0), tau
        if same_as is not None:  # (the pins O and Z, of mass 1e-9, may be taken apart)
            ref = oracle.walk_kc(*args, tau, kc, an, targets=[rank[1]], order=same_as)
            assert ref.npc[0] == 1
            np.testing.assert_allclose(r.acc, ref.acc, rtol=1e-8)


def test_group_mixed_order_picks_the_cheaper_term():
    tb, rank, c = _system()
    r0 = min(rank[1], rank[2])
    kc = oracle.cell_kc(tb)
    a_A, a_B = 1.3, 0.7
    an = _norms(rank, {1: a_A, 2: a_B})
    lo = np.minimum(A, B)
    hi = np.maximum(A, B)
    dg = np.linalg.norm(np.maximum(0.0, np.maximum(lo - _com(), _com() - hi)))
    tau_q, tau_m = _mixed_thresholds(min(a_A, a_B), dg)
    kw = dict(group=2, mode=1, theta_max=10.0, kc=kc, anorm=an, target_range=(r0, r0 + 2),
              cap=1 << 40, split=False)
    for tau, npc, npq in ((tau_m * (1 + 1e-3), 1, 0), (tau_m * (1 - 1e-3), 1, 1),
                          (tau_q * (1 + 1e-3), 1, 1), (tau_q * (1 - 1e-3), 0, 0)):
        r = oracle.walk_group(tb, 0.0, tau=tau, order=oracle.ORDER_MIXED, **kw)
        assert np.all(r.npc == npc) and np.all(r.npq == npq) and np.all(r.flag == 0), tau


def test_mixed_order_accepts_what_the_quadrupole_budget_accepts():
    """The mixed walk opens exactly the cells the quadrupole budget opens (a
    monopole acceptance implies the quadrupole one): the same interaction
    counts for every body, with part of the terms monopoles; at a tau where
    no cell's quadrupole bound is small enough every term is a quadrupole,
    and the forces equal the quadrupole walk's."""
    from tests.conftest import case_bodies
    pos, _, mass = case_bodies("plummer", 3000, 31, np.float64)
    tb = oracle.build_all(pos, mass, 8)
    w = oracle.walk(tb["tree"], tb["mom"], tb["spos"], tb["smass"], tb["L"], 0.5, 0.01)
    an = np.linalg.norm(w.acc, axis=1)
    kc = oracle.cell_kc(tb)
    for tau in (1e-3, 1e-2):
        r2 = oracle.walk_kc(tb, 0.01, 1.2, tau, kc, an, order=2)
        rm = oracle.walk_kc(tb, 0.01, 1.2, tau, kc, an, order=oracle.ORDER_MIXED)
        np.testing.assert_array_equal(rm.npc, r2.npc)
        np.testing.assert_array_equal(rm.npp, r2.npp)
        assert np.all(r2.npq == r2.npc) and np.all(rm.npq <= rm.npc)
        assert 0.05 < 1 - rm.npq.sum() / rm.npc.sum() < 0.999
        g2 = oracle.walk_group(tb, 0.01, group=64, mode=1, theta_max=1.2, tau=tau, kc=kc,
                               anorm=an, cap=4096, split=True, order=2)
        gm = oracle.walk_group(tb, 0.01, group=64, mode=1, theta_max=1.2, tau=tau, kc=kc,
                               anorm=an, cap=4096, split=True, order=oracle.ORDER_MIXED)
        np.testing.assert_array_equal(gm.npc, g2.npc)
        np.testing.assert_array_equal(gm.npp, g2.npp)
    # tau so small that nearly every accepted cell fails its monopole
    # budget: where all of a body's terms are quadrupoles its force is the
    # quadrupole walk's, bit for bit
    rq = oracle.walk_kc(tb, 0.01, 1.2, 1e-9, kc, an, order=oracle.ORDER_MIXED)
    r2 = oracle.walk_kc(tb, 0.01, 1.2, 1e-9, kc, an, order=2)
    allq = rq.npq == rq.npc
    assert allq.mean() > 0.99
    np.testing.assert_array_equal(rq.acc[allq], r2.acc[allq])
