"""Pins for the oracle's direct sum, cell moments, multipole field and tree walk
(Sec. 2.1, Sec. 2.2, Sec. 3)."""
import numpy as np
import pytest

import oracle
from paper_2203_08966_amd import workloads as W


# ---------------------------------------------------------------- direct sum
def test_two_body_closed_form():
    """Two bodies: a_1 = m_2 (r_2 - r_1) / (r^2 + eps^2)^(3/2)."""
    pos = np.array([[0.1, -0.2, 0.3], [1.1, 0.6, -0.1]])
    mass = np.array([0.7, 1.9])
    eps = 0.05
    acc, phi = oracle.direct(pos, mass, eps)
    d = pos[1] - pos[0]
    s = np.sqrt(d @ d + eps * eps)
    np.testing.assert_allclose(acc[0], mass[1] * d / s ** 3, rtol=1e-15)
    np.testing.assert_allclose(acc[1], -mass[0] * d / s ** 3, rtol=1e-15)
    np.testing.assert_allclose(phi, [-mass[1] / s, -mass[0] / s], rtol=1e-15)


def test_momentum_conservation():
    """Pairwise antisymmetry: sum_i m_i a_i = 0 up to rounding."""
    b = W.plummer(1500, 17)
    m = b.mass * np.linspace(0.5, 1.5, b.n)
    acc, _ = oracle.direct(b.pos, m, 0.01)
    tot = (m[:, None] * acc).sum(0)
    assert np.linalg.norm(tot) <= 1e-13 * np.abs(m[:, None] * acc).sum()


def test_uniform_sphere_interior_field():
    """Inside a uniform ball of mass M and radius R: a = -M r / R^3.  The ball
    is a cubic lattice (spacing h) clipped to radius 1, probed at lattice
    vertices so that the nearest lattice points cancel by symmetry; R is the
    radius of the ball with the lattice's volume n h^3."""
    h = 1.0 / 16
    g = (np.arange(-16, 16) + 0.5) * h
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel(), Z.ravel()], 1)
    pts = pts[np.linalg.norm(pts, axis=1) < 1.0]
    n = len(pts)
    R = (3 * n * h ** 3 / (4 * np.pi)) ** (1 / 3)
    probe = np.array([[5 * h, 0.0, 0.0], [0.0, -8 * h, 0.0], [0.0, 0.0, 10 * h], [3 * h, 4 * h, -2 * h]])
    allp = np.concatenate([pts, probe])
    mass = np.concatenate([np.full(n, 1.0 / n), np.zeros(len(probe))])
    acc, _ = oracle.direct(allp, mass, 0.0, targets=np.arange(n, n + len(probe)))
    want = -probe / R ** 3
    err = np.linalg.norm(acc - want, axis=1) / np.linalg.norm(want, axis=1)
    assert np.all(err < 0.03), err


# ---------------------------------------------------------------- moments
def test_moments_two_masses_closed_form():
    """Masses m at +-s z: M = 2m, COM = 0, Q_zz = 4 m s^2, Q_xx = Q_yy = -2 m s^2."""
    m, s = 0.3, 0.25
    pos = np.array([[0.0, 0.0, s], [0.0, 0.0, -s]]) + 1e-9
    b = oracle.build_all(pos, np.array([m, m]), 8)
    M, com, Q = b["mom"]
    assert M[0] == 2 * m
    np.testing.assert_allclose(com[0], 1e-9, atol=1e-15)
    np.testing.assert_allclose(Q[0], [-2 * m * s * s, 0, 0, -2 * m * s * s, 0, 4 * m * s * s],
                               atol=1e-15)


def test_moments_root_and_traceless():
    b0 = W.two_spheres(3000, 8)
    bb = oracle.build_all(b0.pos, b0.mass, 4)
    M, com, Q = bb["mom"]
    assert abs(M[0] - b0.mass.sum()) <= 1e-14
    np.testing.assert_allclose(com[0], np.average(b0.pos, axis=0, weights=b0.mass), atol=1e-13)
    tr = Q[:, 0] + Q[:, 3] + Q[:, 5]
    scale = M * (bb["L"] * 2.0 ** -bb["tree"]["level"]) ** 2
    assert np.all(np.abs(tr) <= 1e-12 * scale)


def test_parallel_axis_composition():
    """A parent's moments equal its children's combined by the parallel-axis
    rule: M = sum M_c, COM = sum M_c com_c / M,
    Q = sum [Q_c + M_c (3 d d^T - |d|^2 I)], d = com_c - COM."""
    b0 = W.plummer(2000, 5)
    bb = oracle.build_all(b0.pos, b0.mass, 3)
    t = bb["tree"]
    M, com, Q = bb["mom"]
    iu = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]
    checked = 0
    for i in range(len(M)):
        if t["next"][i] == i + 1:
            continue
        kids = []
        c = i + 1
        while c < t["next"][i]:
            kids.append(c)
            c = t["next"][c]
        Mp = sum(M[c] for c in kids)
        cp = sum(M[c] * com[c] for c in kids) / Mp
        Qp = np.zeros(6)
        for c in kids:
            d = com[c] - cp
            D = 3 * np.outer(d, d) - (d @ d) * np.eye(3)
            Qp += Q[c] + M[c] * np.array([D[a, b] for a, b in iu])
        side = bb["L"] * 2.0 ** -t["level"][i]
        assert abs(Mp - M[i]) <= 1e-12 * M[i]
        np.testing.assert_allclose(cp, com[i], atol=1e-12 * side)
        np.testing.assert_allclose(Qp, Q[i], atol=1e-11 * M[i] * side * side)
        checked += 1
    assert checked > 100


# ---------------------------------------------------------------- multipole field
def _pair_and_target(z, s, m, order, theta=10.0):
    """Two masses m at (c, c, c +- s), target on the axis at height z above
    their midpoint, in another root octant, so that the pair is one cell that
    the walk accepts.  Returns (a, n_pc, n_pp)."""
    c = 0.25
    pos = np.array([[c, c, c + s], [c, c, c - s], [c, c, c + z]])
    mass = np.array([m, m, 0.0])
    bb = oracle.build_all(pos, mass, 2)
    r = oracle.barnes_hut(pos, mass, theta, 0.0, 2, order=order, targets=[2], built=bb)
    return r.acc[0], r.npc[0], r.npp[0]


def test_quadrupole_on_axis_closed_form():
    """On the axis of two masses m at +-s: exact a = -m/(z-s)^2 - m/(z+s)^2;
    monopole -2m/z^2; monopole+quadrupole -(2m/z^2)(1 + 3 s^2/z^2), whose
    remaining error is the next term, -(2m/z^2)(5 s^4/z^4) to leading order."""
    m, s = 0.4, 0.01
    for z in (0.3, 0.4, 0.6):
        a2, npc, npp = _pair_and_target(z, s, m, 2)
        assert npc == 1 and npp == 0
        a0, npc, npp = _pair_and_target(z, s, m, 0)
        assert npc == 1 and npp == 0
        exact = -m / (z - s) ** 2 - m / (z + s) ** 2
        np.testing.assert_allclose(a0[:2], 0, atol=1e-14)
        np.testing.assert_allclose(a0[2], -2 * m / z ** 2, rtol=1e-12)
        quad = -(2 * m / z ** 2) * (1 + 3 * s * s / z ** 2)
        np.testing.assert_allclose(a2[2], quad, rtol=1e-12)
        nxt = (2 * m / z ** 2) * 5 * s ** 4 / z ** 4
        assert abs(a2[2] - exact) <= 1.2 * nxt
        assert abs(a2[2] - exact) >= 0.8 * nxt


def test_error_slopes():
    """Relative p-c error falls like (size/d)^2 with the monopole and like
    (size/d)^3 with the quadrupole (dipole vanishes about the COM)."""
    rng = np.random.default_rng(1)
    cl = rng.random((12, 3)) * 0.05 + 100.0
    mass = np.concatenate([rng.random(12) + 0.5, [0.0]])
    direction = np.array([0.6, -0.48, 0.64])
    errs = {0: [], 2: []}
    ds = np.array([0.4, 0.8, 1.6, 3.2])
    for d in ds:
        tgt = cl.mean(0) + d * direction
        pos = np.concatenate([cl, tgt[None]])
        bb = oracle.build_all(pos, mass, 12)
        exact, _ = oracle.direct(pos, mass, 0.0, targets=[12])
        for order in (0, 2):
            r = oracle.barnes_hut(pos, mass, 100.0, 0.0, 12, order=order, targets=[12], built=bb)
            assert r.npc[0] >= 1
            errs[order].append(np.linalg.norm(r.acc[0] - exact[0]) / np.linalg.norm(exact[0]))
    s0 = np.polyfit(np.log(ds), np.log(errs[0]), 1)[0]
    s2 = np.polyfit(np.log(ds), np.log(errs[2]), 1)[0]
    assert -2.4 < s0 < -1.6, s0
    assert -3.4 < s2 < -2.6, s2


# ---------------------------------------------------------------- walk
def test_theta_zero_equals_direct():
    b = W.plummer(3000, 21)
    acc_d, phi_d = oracle.direct(b.pos, b.mass, 0.01)
    for leaf in (1, 8):
        r = oracle.barnes_hut(b.pos, b.mass, 0.0, 0.01, leaf)
        np.testing.assert_allclose(r.acc, acc_d, rtol=1e-12, atol=1e-12 * np.abs(acc_d).max())
        np.testing.assert_allclose(r.phi, phi_d, rtol=1e-12)
        assert np.all(r.npc == 0) and np.all(r.npp == b.n - 1)


def test_error_decreases_with_theta_and_order():
    b = W.plummer(4000, 22)
    acc_d, _ = oracle.direct(b.pos, b.mass, 0.01)
    bb = oracle.build_all(b.pos, b.mass, 8)
    prev = 0.0
    for th in (0.2, 0.35, 0.5, 0.7, 0.9):
        e2 = oracle.rms_rel(oracle.barnes_hut(b.pos, b.mass, th, 0.01, 8, built=bb).acc, acc_d)["rms"]
        e0 = oracle.rms_rel(oracle.barnes_hut(b.pos, b.mass, th, 0.01, 8, order=0, built=bb).acc, acc_d)["rms"]
        assert e2 > prev
        assert e2 < e0
        prev = e2


def test_coverage_invariant():
    """Every other body is accounted for exactly once: n_pp plus the bodies of
    accepted cells equals N-1 (N when theta >= 1/sqrt(3) lets an accepted cell
    hold the body itself)."""
    b = W.two_spheres(2500, 6)
    bb = oracle.build_all(b.pos, b.mass, 5)
    for th in (0.3, 0.5, 0.57):
        r = oracle.barnes_hut(b.pos, b.mass, th, 0.0, 5, built=bb)
        assert np.all(r.ncov == b.n - 1)
    r = oracle.barnes_hut(b.pos, b.mass, 1.5, 0.0, 5, built=bb)
    assert np.all((r.ncov == b.n - 1) | (r.ncov == b.n))


def test_root_leaf_and_tiny():
    pos = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    mass = np.array([1.0, 2.0, 3.0])
    acc_d, _ = oracle.direct(pos, mass, 0.1)
    r = oracle.barnes_hut(pos, mass, 0.5, 0.1, 8)  # the root is the only leaf
    np.testing.assert_allclose(r.acc, acc_d, rtol=1e-15)
    r1 = oracle.barnes_hut(pos[:1], mass[:1], 0.5, 0.1, 1)
    assert np.all(r1.acc == 0) and r1.npp[0] == 0


def test_guard_changes_nothing_below_inverse_sqrt3():
    """Below theta = 1/sqrt(3) no cell holding the body passes the opening
    angle test (its distance to the cell's COM is at most the cube's
    diagonal), so the containment guard leaves every result unchanged; at
    theta 1.0 it opens cells and changes counts."""
    from tests.conftest import case_bodies
    pos, _, mass = case_bodies("clumpy", 3000, 7, np.float64)
    ref = oracle.build_all(pos, mass, 8)
    args = (ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"])
    for theta in (0.3, 0.5, 0.57):
        r0 = oracle.walk(*args, theta, 0.01)
        r1 = oracle.walk(*args, theta, 0.01, guard_lo=ref["lo"])
        assert np.array_equal(r0.acc, r1.acc) and np.array_equal(r0.phi, r1.phi)
        assert np.array_equal(r0.npp, r1.npp) and np.array_equal(r0.npc, r1.npc)
    r0 = oracle.walk(*args, 1.0, 0.01)
    r1 = oracle.walk(*args, 1.0, 0.01, guard_lo=ref["lo"])
    assert (r1.npc != r0.npc).any()


def test_guard_opens_the_cell_holding_the_body():
    """Three bodies, leaf size 1, root cube [0, 2)^3: a light body A at 0.05
    (each coordinate) shares the octant [0, 1)^3 with a heavy body B at 0.95;
    C at 1.9 is alone in its octant.  At theta 0.9 that octant (side 1, COM
    about 1.56 from A) passes the opening angle test, so the paper's walk
    takes A's field from a multipole that holds A itself.  The guard opens
    it; what remains are two particle-particle terms, so A's acceleration is
    the direct sum."""
    pos = np.array([[0.05] * 3, [0.95] * 3, [1.9] * 3])
    mass = np.array([1e-3, 1.0, 0.5])
    ref = oracle.build_all(pos, mass, 1)
    assert ref["L"] == 2.0 and np.array_equal(ref["lo"], np.zeros(3))
    a_rank = int(np.where(ref["perm"] == 0)[0][0])
    args = (ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], 0.9, 0.0)
    plain = oracle.walk(*args, targets=np.array([a_rank]))
    guard = oracle.walk(*args, targets=np.array([a_rank]), guard_lo=ref["lo"])
    direct, _ = oracle.direct(pos, mass, 0.0)
    assert plain.npc[0] == 1 and guard.npc[0] == 0 and guard.npp[0] == 2
    np.testing.assert_allclose(guard.acc[0], direct[0], rtol=1e-14, atol=0)
    assert np.linalg.norm(plain.acc[0] - direct[0]) > 1e-3 * np.linalg.norm(direct[0])
