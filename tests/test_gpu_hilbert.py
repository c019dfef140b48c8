"""The Peano-Hilbert ordering on the GPU (Sec. 4.4 names the curve as the
remedy for the Morton order's jumps; a method variant) against the oracle's
Hilbert build and walks: keys, permutation and every node array bit for
bit, FP64 moments to rounding, per-body and group walks."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, check_flagged, say
from tests.test_gpu_build import check_tree
from tests.test_gpu_group import CAP_BUDGET, CAP_THETA, FLAG_TOL, _check, _run
from tests.test_gpu_walk import run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture
def hctx(ctx):
    """The session context with the Hilbert curve for one test."""
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_HILBERT)
    yield ctx
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)


@pytest.mark.parametrize("kind,n,seed,leaf,dtype", [
    ("plummer", 4096, 1, 8, np.float64),
    ("plummer", 20000, 2, 16, np.float32),
    ("clumpy", 50000, 5, 16, np.float32),
    ("coincident", 3000, 6, 4, np.float64),
    ("plummer", 1, 1, 8, np.float32),
    ("plummer", 63, 2, 1, np.float32),
])
def test_hilbert_build_matches_oracle(hctx, kind, n, seed, leaf, dtype):
    say(f"hilbert build: {kind} n={n} leaf={leaf} {np.dtype(dtype).name}")
    pos, _, mass = case_bodies(kind, n, seed, dtype)
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), leaf, curve="hilbert")
    t = B.bh_build(hctx, torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda(), leaf)
    try:
        assert B.bh_tree_info_get(t)["curve"] == B.BH_CURVE_HILBERT
        check_tree(B.bh_tree_export(t), ref, leaf)
    finally:
        B.bh_tree_free(t)


@pytest.mark.parametrize("kind,n,dtype,theta,eps", [
    ("plummer", 20000, np.float32, 0.6, 0.005),
    ("clumpy", 20000, np.float32, 0.7, 1e-4),
    ("plummer", 4096, np.float64, 0.5, 0.01),
])
def test_hilbert_body_walk_matches_oracle(hctx, kind, n, dtype, theta, eps):
    say(f"hilbert per-body walk: {kind} n={n} {np.dtype(dtype).name} theta {theta}")
    pos, _, mass = case_bodies(kind, n, 3, dtype)
    acc, phi, npp, npc = run_gpu(hctx, pos, mass, 16, theta, eps)
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16, curve="hilbert")
    tol = 3e-6 if dtype == np.float32 else 1e-9
    r = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], theta, eps,
                    tol=tol)
    p = ref["perm"]
    a, cp, cc = acc[p].astype(np.float64), npp[p], npc[p]
    ok = r.flag == 0
    assert np.array_equal(cp[ok], r.npp[ok]) and np.array_equal(cc[ok], r.npc[ok])
    e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
    lim = (1e-5, 1e-4) if dtype == np.float32 else (1e-12, 1e-10)
    say(f"  rel err (unflagged): rms {np.sqrt(np.mean(e[ok] ** 2)):.2e} max {e[ok].max():.2e}")
    assert np.sqrt(np.mean(e[ok] ** 2)) <= lim[0] and e[ok].max() <= lim[1]
    check_flagged(ref, r.acc, a, r.flag, eps, 0.01)


def test_hilbert_group_walks_match_oracle(hctx):
    """Group walks over Hilbert groups (64 consecutive bodies along the
    curve): opening angle and error budget, with explicit work caps."""
    pos, _, mass = case_bodies("plummer", 20000, 11, np.float32)
    eps = 0.005
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16, curve="hilbert")
    say("hilbert group walk: theta 0.75")
    out = _run(hctx, pos, mass, 16, 0.75, eps, walk_cap=CAP_THETA)
    r = oracle.walk_group(ref, eps, group=B.BH_GROUP_BODIES, theta=0.75, tol=FLAG_TOL[np.float32],
                          cap=CAP_THETA, split=True)
    _check(ref, r, out, np.float32, eps)
    tau, tmax, fl = 10 ** -1.75, 1.5, 0.5
    w = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], 0.4, eps)
    an = np.empty(len(mass))
    an[ref["perm"]] = np.linalg.norm(w.acc, axis=1)
    an = an.astype(np.float32)
    say("hilbert group walk: error budget with floor")
    out = _run(hctx, pos, mass, 16, 0.5, eps, mac=B.BH_MAC_BUDGET, mlp_theta_max=tmax,
               mlp_log10_tau=np.log10(tau), acc_norm=an, mlp_acc_floor=fl, walk_cap=CAP_BUDGET)
    r = oracle.walk_group(ref, eps, group=B.BH_GROUP_BODIES, mode=1, theta_max=tmax, tau=tau,
                          kc=oracle.cell_kc(ref), anorm=an.astype(np.float64)[ref["perm"]],
                          tol=FLAG_TOL[np.float32], cap=CAP_BUDGET, split=True, floor=fl)
    _check(ref, r, out, np.float32, eps)


def test_hilbert_simulation_follows_morton(ctx):
    """A few KDK steps of the same system sorted along either curve: the
    per-body walks take the same decisions, so the trajectories agree to
    the FP32 rounding of the sums (taken in another order)."""
    pos, vel, mass = case_bodies("plummer", 20000, 4, np.float32)
    P, V, M = (torch.from_numpy(x).cuda() for x in (pos, vel, mass))
    out = {}
    for curve in (B.BH_CURVE_MORTON, B.BH_CURVE_HILBERT):
        B.bh_ctx_set_curve(ctx, curve)
        B.bh_sim_init(ctx, P, V, M, 16, 0.5, 0.005, B.force_opts())
        for _ in range(3):
            B.bh_leapfrog_step(ctx, 1e-3)
        x, a = torch.empty_like(P), torch.empty_like(P)
        B.bh_sim_get(ctx, x, None, a)
        torch.cuda.synchronize()
        out[curve] = (x.cpu().numpy().astype(np.float64), a.cpu().numpy().astype(np.float64))
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    (xm, am), (xh, ah) = out[B.BH_CURVE_MORTON], out[B.BH_CURVE_HILBERT]
    dx = np.abs(xh - xm).max()
    ea = np.linalg.norm(ah - am, axis=1) / np.linalg.norm(am, axis=1)
    say(f"  |x_H - x_M| max {dx:.2e}; acc rel diff rms {np.sqrt(np.mean(ea ** 2)):.2e}")
    assert dx < 1e-5
    assert np.sqrt(np.mean(ea ** 2)) < 1e-5


def test_simulation_keeps_its_curve(ctx):
    """The curve set when the simulation starts sorts every later rebuild
    of its steps, whatever the context's curve is set to afterwards."""
    pos, vel, mass = case_bodies("plummer", 5000, 6, np.float32)
    P, V, M = (torch.from_numpy(x).cuda() for x in (pos, vel, mass))
    for curve, other in ((B.BH_CURVE_HILBERT, B.BH_CURVE_MORTON),
                         (B.BH_CURVE_MORTON, B.BH_CURVE_HILBERT)):
        B.bh_ctx_set_curve(ctx, curve)
        B.bh_sim_init(ctx, P, V, M, 16, 0.5, 0.005, B.force_opts())
        B.bh_ctx_set_curve(ctx, other)
        try:
            for _ in range(2):
                B.bh_leapfrog_step(ctx, 1e-3)
            info = B.bh_tree_info_get(B.bh_sim_tree(ctx))
            torch.cuda.synchronize()
        finally:
            B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
        assert int(info["curve"]) == curve


def test_curve_is_checked(ctx):
    with pytest.raises(B.BHError) as e:
        B.bh_ctx_set_curve(ctx, 2)
    assert e.value.code == B.BH_E_INVALID
