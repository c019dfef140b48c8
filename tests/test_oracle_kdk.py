"""Pins for the oracle's KDK leapfrog and energy (Sec. 2.3, Sec. 2.4) and the
Plummer generator's closed forms."""
import numpy as np

import oracle
from paper_2203_08966_amd import workloads as W


def _direct_force(mass, eps):
    return lambda x: oracle.direct(x, mass, eps)[0]


def _circular_pair(m1=0.6, m2=0.4, a=1.0):
    M = m1 + m2
    w = np.sqrt(M / a ** 3)
    pos = np.array([[-m2 / M * a, 0, 0], [m1 / M * a, 0, 0]])
    vel = np.array([[0, -m2 / M * a * w, 0], [0, m1 / M * a * w, 0]])
    return pos, vel, np.array([m1, m2]), 2 * np.pi / w


def test_circular_orbit_period_and_energy():
    """Circular two-body orbit: after one period 2 pi sqrt(a^3/M) the bodies
    return to the start (error O(dt^2)); the energy error over the orbit is
    bounded, does not grow from one period to the next, and shrinks ~4x when
    dt halves (second order)."""
    pos, vel, mass, period = _circular_pair(a=1.0)
    pos = pos * np.array([1.0, 1.0, 1.0])
    vel = vel * 0.9  # eccentric orbit: the energy error is not constant
    e0 = sum(oracle.energy(pos, vel, mass, 0.0))
    res = []
    f = _direct_force(mass, 0.0)
    for nsteps in (200, 400):
        dt = period / nsteps
        x, v = pos, vel
        worst = []
        for _ in range(2):
            w = 0.0
            for _ in range(nsteps):
                x, v, _ = oracle.kdk(x, v, mass, dt, 1, f)
                w = max(w, abs(sum(oracle.energy(x, v, mass, 0.0)) - e0))
            worst.append(w)
        res.append(worst)
    (a1, a2), (b1, b2) = res
    assert a1 < 1e-2 * abs(e0)
    assert 3.0 < a1 / b1 < 5.0
    assert a2 < 1.5 * a1 and b2 < 1.5 * b1
    # circular orbit: return to the start after one period
    pos_c, vel_c, _, _ = _circular_pair(a=1.0)
    errs = []
    for nsteps in (200, 400):
        x, _, _ = oracle.kdk(pos_c, vel_c, mass, period / nsteps, nsteps, f)
        errs.append(np.abs(x - pos_c).max())
    assert errs[0] < 0.05 and 3.0 < errs[0] / errs[1] < 5.0


def test_time_reversal():
    """KDK is time-symmetric: n steps, reverse velocities, n steps -> start."""
    b = W.plummer(64, 3)
    mass = b.mass
    f = _direct_force(mass, 0.05)
    x, v, _ = oracle.kdk(b.pos, b.vel, mass, 1e-3, 50, f)
    x2, v2, _ = oracle.kdk(x, -v, mass, 1e-3, 50, f)
    np.testing.assert_allclose(x2, b.pos, atol=1e-12)
    np.testing.assert_allclose(-v2, b.vel, atol=1e-12)


def test_energy_drift_second_order_small_n():
    b = W.plummer(32, 9)
    f = _direct_force(b.mass, 0.05)
    e0 = sum(oracle.energy(b.pos, b.vel, b.mass, 0.05))
    d = []
    for dt in (4e-3, 2e-3):
        steps = int(round(0.4 / dt))
        x, v, _ = oracle.kdk(b.pos, b.vel, b.mass, dt, steps, f)
        d.append(abs(sum(oracle.energy(x, v, b.mass, 0.05)) - e0))
    assert d[0] < 1e-4 * abs(e0)
    assert 2.5 < d[0] / d[1] < 6.0


def test_two_body_potential_energy():
    pos = np.array([[0.0, 0, 0], [0.3, 0.4, 0]])
    mass = np.array([2.0, 3.0])
    ek, ep = oracle.energy(pos, np.zeros((2, 3)), mass, 0.1)
    assert ek == 0.0
    np.testing.assert_allclose(ep, -6.0 / np.sqrt(0.25 + 0.01), rtol=1e-15)


def test_plummer_closed_forms():
    """Plummer sphere (M = a = G = 1): E_kin = 3 pi/64, E_pot = -3 pi/32,
    half-mass radius (2^(2/3) - 1)^(-1/2) = 1.3048; statistical tolerance."""
    b = W.plummer(20000, 12)
    ek = 0.5 * np.sum(b.mass * np.sum(b.vel ** 2, axis=1))
    r = np.sort(np.linalg.norm(b.pos, axis=1))
    assert abs(r[b.n // 2] - 1.3048) < 0.04
    assert abs(ek - 3 * np.pi / 64) < 0.03 * 3 * np.pi / 64
    sub = W.plummer(4096, 12)
    ek4, ep4 = oracle.energy(sub.pos, sub.vel, sub.mass, 0.0)
    assert abs(ep4 + 3 * np.pi / 32) < 0.04 * 3 * np.pi / 32
    assert abs(np.sum(sub.mass) - 1.0) < 1e-12
    np.testing.assert_allclose(np.average(sub.pos, axis=0, weights=sub.mass), 0, atol=1e-14)
