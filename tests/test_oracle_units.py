"""Pins for the oracle's standard-units scaling (Sec. 2.4) and the
two-cluster collision workload (Sec. 5)."""
import numpy as np
from scipy.spatial.distance import pdist

import oracle
from paper_2203_08966_amd import workloads as W


def _energies(x, v, m):
    """Kinetic energy and the unsoftened pair potential, each pair once,
    by a route of their own (scipy's pair distances)."""
    ek = 0.5 * float(np.einsum("i,ij,ij->", m, v, v))
    mm = pdist(m[:, None], lambda a, b: a[0] * b[0])
    return ek, -float(np.sum(mm / pdist(x)))


def test_two_body_closed_form():
    """Two bodies of masses 1 and 3: in standard units the masses are 1/4
    and 3/4, W = -m1 m2 / r = -1/2 gives r = 3/8, and E_kin = mu u^2 / 2 =
    1/4 with mu = m1 m2 = 3/16 gives |u| = sqrt(8/3); the separation and the
    relative velocity keep their directions, and the centre of mass is at
    rest at the origin."""
    pos = np.array([[0.3, -1.0, 2.0], [0.3, 1.0, 2.0]])  # separation along +y, length 2
    vel = np.array([[5.0, 0.0, 0.0], [1.0, 0.0, 0.0]])   # relative velocity along -x
    x, v, m, (ek, ep, M) = oracle.standard_units(pos, vel, np.array([1.0, 3.0]))
    assert M == 4.0
    np.testing.assert_allclose(m, [0.25, 0.75], rtol=0, atol=1e-15)
    r = 3.0 / 8.0
    u = np.sqrt(8.0 / 3.0)
    np.testing.assert_allclose(x, [[0, -0.75 * r, 0], [0, 0.25 * r, 0]], rtol=0, atol=1e-14)
    np.testing.assert_allclose(v, [[0.75 * u, 0, 0], [-0.25 * u, 0, 0]], rtol=0, atol=1e-14)
    # energies before the scalings: relative speed 4, separation 2
    assert abs(ek - 0.5 * (3.0 / 16.0) * 16.0) < 1e-14
    assert abs(ep - (-(3.0 / 16.0) / 2.0)) < 1e-15


def test_invariants_random_system():
    """Any system: total mass 1, centre of mass and momentum zero, E_kin =
    -E_pot / 2 and E = -1/4 (energies by an independent route), and the
    result is the shifted input scaled by one length and one velocity
    factor."""
    rng = np.random.default_rng(11)
    n = 300
    pos = rng.normal(size=(n, 3)) + 5.0
    vel = rng.normal(size=(n, 3)) * 0.3 - 1.0
    mass = rng.uniform(0.5, 2.0, n)
    x, v, m, _ = oracle.standard_units(pos, vel, mass)
    assert abs(m.sum() - 1.0) < 1e-14
    assert np.abs(m @ x).max() < 1e-14 and np.abs(m @ v).max() < 1e-14
    ek, ep = _energies(x, v, m)
    assert abs(ek + ep + 0.25) < 1e-13
    assert abs(2 * ek + ep) < 1e-13
    x0 = pos - (mass @ pos) / mass.sum()
    v0 = vel - (mass @ vel) / mass.sum()
    for y, y0 in ((x, x0), (v, v0)):
        beta = np.sum(y * y0) / np.sum(y0 * y0)
        assert np.abs(y - beta * y0).max() < 1e-13 * np.abs(y).max()
    np.testing.assert_allclose(m, mass / mass.sum(), rtol=1e-15)


def test_plummer_length_scale():
    """A Plummer sphere (mass 1, radius 1) has W = -3 pi / 32, so in standard
    units its lengths shrink by b = -2 W = 3 pi / 16 (finite sample and the
    mass cut-off at 0.999: within 3 %)."""
    b = W.plummer(8000, 5)
    x, _, _, (ek, ep, M) = oracle.standard_units(b.pos, b.vel, b.mass)
    assert abs(M - 1.0) < 1e-12
    assert abs(ep / (-3 * np.pi / 32) - 1) < 0.03
    assert abs(ek / (3 * np.pi / 64) - 1) < 0.05  # virial: E_kin = -W / 2
    x0 = b.pos - (b.mass @ b.pos)
    scale = np.median(np.linalg.norm(x, axis=1) / np.linalg.norm(x0, axis=1))
    assert abs(scale / (3 * np.pi / 16) - 1) < 0.03


def test_two_clusters_layout():
    """Two clusters of n/2 equal-mass bodies, centred at -/+ offset (1,1,1),
    at rest relative to each other, each with virial ratio about 1/2."""
    b = W.two_clusters(4000, 3, offset=2.0)
    assert b.n == 4000 and np.all(b.mass == 1.0 / 4000)
    h = 2000
    for sl, c in ((slice(0, h), -2.0), (slice(h, None), 2.0)):
        np.testing.assert_allclose(b.pos[sl].mean(0), [c, c, c], atol=1e-12)
        np.testing.assert_allclose(b.vel[sl].mean(0), [0, 0, 0], atol=1e-12)
        ek, ep = _energies(b.pos[sl], b.vel[sl], b.mass[sl])
        assert 0.4 < ek / -ep < 0.6
