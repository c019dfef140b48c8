"""GPU kick-drift-kick leapfrog and energy against the oracle (Sec. 2.3,
Sec. 2.4)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, say

pytestmark = pytest.mark.gpu


def _bh_force(mass, theta, eps, leaf):
    return lambda x: oracle.barnes_hut(x, mass, theta, eps, leaf).acc


# 4099: 3n odd, so the kicks' last component is outside their 16-byte vectors
@pytest.mark.parametrize("n", [4096, 4099])
def test_leapfrog_fp64_matches_oracle(ctx, n):
    """N=4096 (or 4099) Plummer, theta 0.5, eps 0.01, leaf 8, FP64: one force
    evaluation plus 10 KDK steps of dt 1e-3, against the oracle's KDK with
    its own tree rebuilt every step."""
    pos, vel, mass = case_bodies("plummer", n, 1, np.float64)
    theta, eps, leaf, dt, steps = 0.5, 0.01, 8, 1e-3, 10
    say(f"leapfrog FP64: {n} bodies, 10 steps")
    xo, vo, ao = oracle.kdk(pos, vel, mass, dt, steps, _bh_force(mass, theta, eps, leaf))
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    B.bh_sim_init(ctx, P, V, M, leaf, theta, eps)
    for _ in range(steps):
        B.bh_leapfrog_step(ctx, dt)
    x = torch.empty_like(P)
    v = torch.empty_like(V)
    a = torch.empty_like(P)
    B.bh_sim_get(ctx, x, v, a)
    torch.cuda.synchronize()
    x, v, a = x.cpu().numpy(), v.cpu().numpy(), a.cpu().numpy()
    np.testing.assert_allclose(x, xo, rtol=0, atol=1e-9)
    np.testing.assert_allclose(v, vo, rtol=0, atol=1e-7)
    e = np.linalg.norm(a - ao, axis=1) / np.linalg.norm(ao, axis=1)
    assert np.median(e) < 1e-10
    # energy: kinetic exact, potential from the walk's phi at the same tree
    ek, ep = B.bh_energy(ctx)
    ek_ref = 0.5 * np.sum(mass * np.sum(vo ** 2, axis=1))
    phi_ref = oracle.barnes_hut(xo, mass, theta, eps, leaf).phi
    ep_ref = 0.5 * np.sum(mass * phi_ref)
    assert abs(ek - ek_ref) <= 1e-9 * abs(ek_ref)
    assert abs(ep - ep_ref) <= 1e-9 * abs(ep_ref)


# 20001: 3n = 60003, three components after the kicks' last 16-byte vector
@pytest.mark.parametrize("n", [20000, 20001])
def test_leapfrog_fp32_short_run(ctx, n):
    pos, vel, mass = case_bodies("plummer", n, 2, np.float32)
    theta, eps, leaf, dt = 0.5, 0.005, 16, 5e-4
    say(f"leapfrog FP32: {n} bodies, 5 steps, vs FP64 oracle KDK")
    p64, v64, m64 = (a.astype(np.float64) for a in (pos, vel, mass))
    xo, vo, _ = oracle.kdk(p64, v64, m64, dt, 5, _bh_force(m64, theta, eps, leaf))
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    B.bh_sim_init(ctx, P, V, M, leaf, theta, eps)
    e0 = sum(B.bh_energy(ctx))
    B.bh_sim_timing(ctx, True)
    for _ in range(5):
        B.bh_leapfrog_step(ctx, dt)
    ms, steps = B.bh_sim_timing_get(ctx)
    B.bh_sim_timing(ctx, False)
    # phases: kick+drift, build, walk (with set-up), kick, walk kernel alone
    assert steps == 5 and all(t > 0 for t in ms) and ms[4] <= ms[2]
    x = torch.empty_like(P)
    v = torch.empty_like(V)
    B.bh_sim_get(ctx, x, v)
    torch.cuda.synchronize()
    dx = np.abs(x.cpu().numpy() - xo).max()
    dv = np.abs(v.cpu().numpy() - vo).max()
    say(f"  max |dx| {dx:.2e}  max |dv| {dv:.2e}")
    assert dx < 1e-5 and dv < 1e-3
    e1 = sum(B.bh_energy(ctx))
    assert abs(e1 - e0) < 1e-4 * abs(e0)


def test_energy_potential_on_demand(ctx):
    """Steps compute accelerations only; bh_energy then walks the current
    tree once more for the potential.  It equals the potential of a fresh
    simulation started from the final state (whose initial walk computes it),
    and a second call returns the same values."""
    pos, vel, mass = case_bodies("plummer", 8192, 5, np.float32)
    theta, eps, leaf, dt = 0.6, 0.01, 16, 1e-3
    say("energy on demand: 8192 bodies, 4 steps")
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    B.bh_sim_init(ctx, P, V, M, leaf, theta, eps)
    for _ in range(4):
        B.bh_leapfrog_step(ctx, dt)
    e1 = B.bh_energy(ctx)
    assert B.bh_energy(ctx) == e1
    x, v = torch.empty_like(P), torch.empty_like(V)
    B.bh_sim_get(ctx, x, v)
    B.bh_sim_init(ctx, x, v, M, leaf, theta, eps)
    e2 = B.bh_energy(ctx)
    assert e1[0] == e2[0]
    assert abs(e1[1] - e2[1]) <= 1e-6 * abs(e2[1])


def test_sim_state_errors(ctx):
    c2 = B.bh_ctx_create(0)
    with pytest.raises(B.BHError) as e:
        B.bh_leapfrog_step(c2, 1e-3)
    assert e.value.code == B.BH_E_STATE
    with pytest.raises(B.BHError) as e:
        B.bh_energy(c2)
    assert e.value.code == B.BH_E_STATE
    B.bh_ctx_destroy(c2)


@pytest.mark.parametrize("walk", [B.BH_WALK_BODY, B.BH_WALK_GROUP])
def test_recorded_steps_count_interactions(ctx, walk):
    """Steps recorded by bh_sim_timing also sum their walks' interaction
    counts: equal to the counts of the same walk repeated on each step's
    tree (no work cap, so a repeated group walk takes the same decisions)."""
    pos, vel, mass = case_bodies("plummer", 30000, 6, np.float32)
    theta, eps, leaf, dt = 0.6, 0.005, 16, 5e-4
    say(f"recorded step counts: 30000 bodies, walk {walk}")
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    o = B.force_opts(walk=walk, walk_cap=1 << 30)
    B.bh_sim_init(ctx, P, V, M, leaf, theta, eps, o)
    B.bh_leapfrog_step(ctx, dt)
    B.bh_sim_timing(ctx, True)
    pp = pc = 0
    for _ in range(3):
        B.bh_leapfrog_step(ctx, dt)
        t = B.bh_sim_tree(ctx)
        acc = torch.empty_like(P)
        npp = torch.zeros(30000, dtype=torch.int32, device="cuda")
        npc = torch.zeros(30000, dtype=torch.int32, device="cuda")
        B.bh_forces(t, theta, eps, acc, B.force_opts(walk=walk, walk_cap=1 << 30, n_pp=npp,
                                                      n_pc=npc))
        pp += int(npp.to(torch.int64).sum().item())
        pc += int(npc.to(torch.int64).sum().item())
    got = B.bh_sim_counts_get(ctx)
    _, steps = B.bh_sim_timing_get(ctx)
    B.bh_sim_timing(ctx, False)
    say(f"  recorded {got}, repeated walks {(pp, pc)}")
    assert steps == 3 and got == (pp, pc) and pc > 0
