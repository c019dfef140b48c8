"""GPU standard units (Sec. 2.4), the direct method (every pair, Sec. 3) and
the two-cluster collision (Sec. 5) against the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08966_amd import binding as B
from paper_2203_08966_amd import workloads as W
from tests.conftest import case_bodies, say

pytestmark = pytest.mark.gpu


def _units(ctx, pos, vel, mass):
    P, V, M = (torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (pos, vel, mass))
    st = B.bh_standard_units(ctx, P, V, M)
    return P.cpu().numpy(), V.cpu().numpy(), M.cpu().numpy(), st


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_standard_units_match_oracle(ctx, dtype):
    """Two clusters of 3000 (FP64) or 6000 (FP32) bodies: the scaled
    positions, velocities and masses and the energies before the scaling
    agree with the oracle's (FP64: to rounding; FP32: one rounding of each
    stored value, twice)."""
    n = 3000 if dtype == np.float64 else 6000
    b = W.two_clusters(n, 3)
    pos, vel, mass = (np.ascontiguousarray(a, dtype=dtype) for a in (b.pos, b.vel, b.mass))
    say(f"standard units: {n} bodies, {np.dtype(dtype).name}")
    x, v, m, st = _units(ctx, pos, vel, mass)
    xo, vo, mo, sto = oracle.standard_units(pos.astype(np.float64), vel.astype(np.float64),
                                            mass.astype(np.float64))
    tol = 1e-12 if dtype == np.float64 else 1e-6
    assert np.abs(x - xo).max() <= tol * np.abs(xo).max()
    assert np.abs(v - vo).max() <= tol * np.abs(vo).max()
    assert np.abs(m - mo).max() <= tol * mo.max()
    # FP32: the energies are taken from the shifted values as stored (FP32)
    np.testing.assert_allclose(st, sto, rtol=1e-12 if dtype == np.float64 else 1e-6)
    ek, ep = oracle.energy(x.astype(np.float64), v.astype(np.float64), m.astype(np.float64), 0.0)
    say(f"  E after scaling {ek + ep:.9f}, 2T/|W| {2 * ek / -ep:.9f}")
    assert abs(ek + ep + 0.25) <= (1e-12 if dtype == np.float64 else 1e-5)


def test_standard_units_two_body_closed_form(ctx):
    """Masses 1 and 3 two apart along y, relative velocity 4 along -x: in
    standard units the masses are 1/4 and 3/4, the separation 3/8 (W = -1/2)
    and the relative speed sqrt(8/3) (E_kin = 1/4), directions kept, centre
    of mass at rest at the origin."""
    pos = np.array([[0.3, -1.0, 2.0], [0.3, 1.0, 2.0]])
    vel = np.array([[5.0, 0.0, 0.0], [1.0, 0.0, 0.0]])
    x, v, m, st = _units(ctx, pos, vel, np.array([1.0, 3.0]))
    r, u = 3.0 / 8.0, np.sqrt(8.0 / 3.0)
    np.testing.assert_allclose(m, [0.25, 0.75], rtol=0, atol=1e-15)
    np.testing.assert_allclose(x, [[0, -0.75 * r, 0], [0, 0.25 * r, 0]], rtol=0, atol=1e-14)
    np.testing.assert_allclose(v, [[0.75 * u, 0, 0], [-0.25 * u, 0, 0]], rtol=0, atol=1e-14)
    np.testing.assert_allclose(st, [1.5, -3.0 / 32.0, 4.0], rtol=1e-14)


def test_direct_method_single_body(ctx):
    """One body: no force, so a step moves it by v dt; its energy is all
    kinetic."""
    P = torch.tensor([[0.5, -0.25, 2.0]], dtype=torch.float64, device="cuda")
    V = torch.tensor([[1.0, 2.0, -3.0]], dtype=torch.float64, device="cuda")
    M = torch.tensor([2.0], dtype=torch.float64, device="cuda")
    B.bh_sim_init(ctx, P, V, M, 8, 0.5, 0.0, _direct_opts())
    B.bh_leapfrog_step(ctx, 0.125)
    x, a = torch.empty_like(P), torch.empty_like(P)
    B.bh_sim_get(ctx, x, None, a)
    assert torch.equal(a.cpu(), torch.zeros(1, 3, dtype=torch.float64))
    assert torch.equal(x.cpu(), torch.tensor([[0.625, 0.0, 1.625]], dtype=torch.float64))
    assert B.bh_energy(ctx) == (14.0, 0.0)


def test_standard_units_errors(ctx):
    """A system at rest has no kinetic energy to scale (BH_E_INVALID); two
    bodies at one point make the unsoftened potential infinite
    (BH_E_NONFINITE)."""
    pos = np.random.default_rng(1).normal(size=(100, 3))
    mass = np.full(100, 0.01)
    with pytest.raises(B.BHError) as e:
        _units(ctx, pos, np.zeros_like(pos), mass)
    assert e.value.code == B.BH_E_INVALID
    pos2 = pos.copy()
    pos2[1] = pos2[0]
    with pytest.raises(B.BHError) as e:
        _units(ctx, pos2, np.ones_like(pos), mass)
    assert e.value.code == B.BH_E_NONFINITE


def _direct_opts():
    o = B.bh_force_opts_default()
    o.walk = B.BH_WALK_DIRECT
    return o


def test_direct_method_fp64_matches_oracle(ctx):
    """The direct method (no tree, every pair): 2048 Plummer bodies, FP64,
    eps 0.01, initial forces plus 5 KDK steps of dt 1e-3 against the oracle's
    KDK with its direct sum; the energy from the direct potential."""
    pos, vel, mass = case_bodies("plummer", 2048, 1, np.float64)
    eps, dt, steps = 0.01, 1e-3, 5
    say("direct method FP64: 2048 bodies, 5 steps")
    xo, vo, ao = oracle.kdk(pos, vel, mass, dt, steps, lambda x: oracle.direct(x, mass, eps)[0])
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    B.bh_sim_init(ctx, P, V, M, 8, 0.5, eps, _direct_opts())
    B.bh_sim_timing(ctx, True)
    for _ in range(steps):
        B.bh_leapfrog_step(ctx, dt)
    ms, n = B.bh_sim_timing_get(ctx)
    B.bh_sim_timing(ctx, False)
    # no tree builds: the build phase is two adjacent events (a tree build of
    # 2048 bodies takes several kernels, well over 20 us)
    assert n == steps and ms[1] / steps < 0.02 and ms[4] > 0
    x, v, a = torch.empty_like(P), torch.empty_like(V), torch.empty_like(P)
    B.bh_sim_get(ctx, x, v, a)
    torch.cuda.synchronize()
    x, v, a = x.cpu().numpy(), v.cpu().numpy(), a.cpu().numpy()
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-12)
    np.testing.assert_allclose(v, vo, rtol=0, atol=1e-10)
    e = np.linalg.norm(a - ao, axis=1) / np.linalg.norm(ao, axis=1)
    assert e.max() < 1e-11
    ek, ep = B.bh_energy(ctx)
    eko, epo = oracle.energy(xo, vo, mass, eps)
    assert abs(ek - eko) <= 1e-11 * abs(eko) and abs(ep - epo) <= 1e-11 * abs(epo)


def test_direct_method_fp32(ctx):
    """FP32 direct method (rsqrt, FP64 sums per tile of 256 sources): 5000
    clumpy bodies, accelerations against the FP64 direct sum, then 5 steps
    against the oracle's FP64 KDK."""
    pos, vel, mass = case_bodies("clumpy", 5000, 4, np.float32)
    eps, dt = 0.005, 5e-4
    say("direct method FP32: 5000 bodies")
    p64, v64, m64 = (a.astype(np.float64) for a in (pos, vel, mass))
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    B.bh_sim_init(ctx, P, V, M, 16, 0.5, eps, _direct_opts())
    a = torch.empty_like(P)
    B.bh_sim_get(ctx, acc=a)
    torch.cuda.synchronize()
    ao, _ = oracle.direct(p64, m64, eps)
    e = np.linalg.norm(a.cpu().numpy() - ao, axis=1) / np.linalg.norm(ao, axis=1)
    say(f"  rel err: rms {np.sqrt(np.mean(e ** 2)):.2e}  max {e.max():.2e}")
    assert np.sqrt(np.mean(e ** 2)) < 1e-6 and e.max() < 1e-4
    xo, vo, _ = oracle.kdk(p64, v64, m64, dt, 5, lambda x: oracle.direct(x, m64, eps)[0])
    for _ in range(5):
        B.bh_leapfrog_step(ctx, dt)
    x, v = torch.empty_like(P), torch.empty_like(V)
    B.bh_sim_get(ctx, x, v)
    torch.cuda.synchronize()
    assert np.abs(x.cpu().numpy() - xo).max() < 1e-5
    assert np.abs(v.cpu().numpy() - vo).max() < 1e-3


def test_forces_reject_direct(ctx):
    pos, _, mass = case_bodies("plummer", 1000, 2, np.float32)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, 16)
    acc = torch.empty_like(P)
    with pytest.raises(B.BHError) as e:
        B.bh_forces(t, 0.5, 0.01, acc, _direct_opts())
    assert e.value.code == B.BH_E_INVALID
    B.bh_tree_free(t)


def test_collision_energy_conservation(ctx):
    """Sec. 5's test problem at 4096 bodies in standard units, theta 0.5,
    dt 0.01, 100 steps, FP64: the tree code (per-body walk, quadrupoles) and
    the direct method both keep the total energy within 1 % (the level the
    paper calls satisfactory), and their energy changes agree in size."""
    b = W.two_clusters(4096, 7)
    P, V, M = (torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).cuda()
               for a in (b.pos, b.vel, b.mass))
    B.bh_standard_units(ctx, P, V, M)
    eps, dt, steps = 0.01, 0.01, 100
    say("collision: 4096 bodies, standard units, 100 steps of 0.01")
    changes = []
    for opts in (None, _direct_opts()):
        B.bh_sim_init(ctx, P, V, M, 8, 0.5, eps, opts)
        e0 = sum(B.bh_energy(ctx))
        for _ in range(steps):
            B.bh_leapfrog_step(ctx, dt)
        e1 = sum(B.bh_energy(ctx))
        changes.append(abs(e1 - e0) / abs(e0))
        say(f"  {'tree' if opts is None else 'direct'}: E0 {e0:.6f}  |dE/E| {changes[-1]:.2e}")
        assert abs(e0 + 0.25) < 0.01  # softening moves E0 slightly off -1/4
    assert max(changes) < 1e-2
    assert changes[0] < 10 * changes[1] + 1e-6
