"""The error budget with monopole terms (order 0) on the GPU against the
oracle: a cell is accepted iff M l^3 + (7/2) |Q|_F d < tau |a| d^5 (the
dropped quadrupole term of Sec. 2.2 bounded by (7/2) |Q|_F / d^4, added to
the budget of Sec. 3.2), per body and per group, over Morton and Hilbert
groups, with the per-body fallback of runs over the work cap; and the mixed
order (the monopole where that holds, else the quadrupole where
M l^3 < tau |a| d^5, else open), with its count of quadrupole terms."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08966_amd import binding as B
from tests.conftest import case_bodies, say
from tests.test_gpu_group import CAP_BUDGET, FLAG_TOL, MAX_FLAGGED, _check, _run
from tests.test_gpu_mlp import _compare, _gpu_walk, _oracle_anorm

pytestmark = pytest.mark.gpu


def _setup(kind, n, seed, curve="morton", eps=0.005):
    pos, _, mass = case_bodies(kind, n, seed, np.float32)
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16, curve=curve)
    an = _oracle_anorm(ref, eps).astype(np.float32)
    return pos, mass, ref, an


@pytest.mark.parametrize("kind,tau,tmax,fl", [
    ("plummer", 1e-2, 1.0, 0.0),
    ("clumpy", 10 ** -1.5, 1.5, 0.5),
])
def test_body_budget_mono_matches_oracle(ctx, kind, tau, tmax, fl):
    eps = 0.005
    pos, mass, ref, an = _setup(kind, 20000, 21)
    say(f"per-body monopole budget: {kind} 20000 bodies, tau {tau:.3g}, theta_max {tmax}, "
        f"floor {fl}")
    a, cp, cc = _gpu_walk(ctx, pos, mass, 16, eps, mac=B.BH_MAC_BUDGET, order=0,
                          mlp_theta_max=tmax, mlp_log10_tau=np.log10(tau), acc_norm=an,
                          mlp_acc_floor=fl)
    kc = oracle.cell_kc(ref)
    anr = an.astype(np.float64)[ref["perm"]]
    r = oracle.walk_kc(ref, eps, tmax, tau, kc, anr, floor=fl, order=0)
    # the quadrupole's bound is in effect: the quadrupole budget accepts more
    r2 = oracle.walk_kc(ref, eps, tmax, tau, kc, anr, floor=fl)
    assert np.mean(r.npc + r.npp > r2.npc + r2.npp) > 0.5
    _compare(ref, r, a, cp, cc, eps)


@pytest.mark.parametrize("curve", ["morton", "hilbert"])
def test_group_budget_mono_matches_oracle(ctx, curve):
    eps, tau, tmax, fl = 0.005, 10 ** -2.0, 1.5, 0.5
    pos, mass, ref, an = _setup("plummer", 20000, 22, curve)
    say(f"group monopole budget ({curve}): 20000 bodies, tau {tau:.3g}, floor {fl}")
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_HILBERT if curve == "hilbert" else B.BH_CURVE_MORTON)
    try:
        out = _run(ctx, pos, mass, 16, 0.5, eps, mac=B.BH_MAC_BUDGET, order=0, mlp_theta_max=tmax,
                   mlp_log10_tau=np.log10(tau), acc_norm=an, mlp_acc_floor=fl,
                   walk_cap=CAP_BUDGET)
    finally:
        B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    r = oracle.walk_group(ref, eps, group=B.BH_GROUP_BODIES, mode=1, order=0, theta_max=tmax,
                          tau=tau, kc=oracle.cell_kc(ref), anorm=an.astype(np.float64)[ref["perm"]],
                          tol=FLAG_TOL[np.float32], cap=CAP_BUDGET, split=True, floor=fl)
    _check(ref, r, out, np.float32, eps)


def test_group_budget_mono_work_cap(ctx):
    """A low work cap sends part of the runs to the per-body walk with the
    same criterion, exactly where the oracle's runs go."""
    eps, tau, tmax, cap = 0.005, 10 ** -2.0, 1.5, 1200
    pos, mass, ref, an = _setup("clumpy", 20000, 23)
    kw = dict(group=B.BH_GROUP_BODIES, mode=1, order=0, theta_max=tmax, tau=tau,
              kc=oracle.cell_kc(ref), anorm=an.astype(np.float64)[ref["perm"]],
              tol=FLAG_TOL[np.float32], split=True)
    r = oracle.walk_group(ref, eps, cap=cap, **kw)
    r0 = oracle.walk_group(ref, eps, cap=1 << 40, **kw)
    moved = np.mean((r.npp != r0.npp) | (r.npc != r0.npc))
    say(f"group monopole budget, work cap {cap}: {moved:.1%} of the bodies walked per body")
    assert 0.1 < moved < 0.9
    out = _run(ctx, pos, mass, 16, 0.5, eps, mac=B.BH_MAC_BUDGET, order=0, mlp_theta_max=tmax,
               mlp_log10_tau=np.log10(tau), acc_norm=an, walk_cap=cap)
    _check(ref, r, out, np.float32, eps)


def test_budget_orders_accepted_and_refused(ctx):
    """The budget runs in the FP32 walk of order 0 or 2; the learned
    criterion only in the quadrupole walk."""
    pos, _, mass = case_bodies("plummer", 3000, 24, np.float32)
    t = B.bh_build(ctx, torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda(), 16)
    acc = torch.empty(3000, 3, device="cuda")
    try:
        for order in (0, 2):
            B.bh_forces(t, 0.5, 0.005, acc, B.force_opts(mac=B.BH_MAC_BUDGET, order=order))
            torch.cuda.synchronize()
            assert torch.isfinite(acc).all()
        with pytest.raises(B.BHError):
            B.bh_forces(t, 0.5, 0.005, acc, B.force_opts(mac=B.BH_MAC_BUDGET, order=3))
        with pytest.raises(B.BHError):
            B.bh_forces(t, 0.5, 0.005, acc, B.force_opts(mac=B.BH_MAC_MLP, order=0))
    finally:
        B.bh_tree_free(t)
    p64 = torch.from_numpy(pos.astype(np.float64)).cuda()
    t = B.bh_build(ctx, p64, torch.from_numpy(mass.astype(np.float64)).cuda(), 16)
    try:
        with pytest.raises(B.BHError):
            B.bh_forces(t, 0.5, 0.005, torch.empty_like(p64),
                        B.force_opts(mac=B.BH_MAC_BUDGET, order=0))
    finally:
        B.bh_tree_free(t)


def _run_q(ctx, pos, mass, eps, curve=B.BH_CURVE_MORTON, **kw):
    """A walk with all four outputs and the quadrupole-term count."""
    B.bh_ctx_set_curve(ctx, curve)
    try:
        P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
        t = B.bh_build(ctx, P, M, 16)
    finally:
        B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    n = len(mass)
    acc = torch.empty_like(P)
    phi = torch.empty_like(M)
    cnt = [torch.zeros(n, dtype=torch.int32, device="cuda") for _ in range(3)]
    an = kw.pop("acc_norm", None)
    an_t = None if an is None else torch.from_numpy(an.astype(np.float32)).cuda()
    o = B.force_opts(phi=phi, n_pp=cnt[0], n_pc=cnt[1], n_pq=cnt[2], mlp_acc_norm=an_t, **kw)
    B.bh_forces(t, 0.5, eps, acc, o)
    torch.cuda.synchronize()
    B.bh_tree_free(t)
    return (acc.cpu().numpy().astype(np.float64), phi.cpu().numpy().astype(np.float64),
            *(c.cpu().numpy() for c in cnt))


def _check_q(ref, r, out, eps, max_flagged):
    """Unflagged bodies: identical counts (quadrupole terms included) and
    forces within the FP32 bounds; flagged bodies within the method's error."""
    from tests.conftest import check_flagged
    a, phi, cp, cc, cq = (x[ref["perm"]] for x in out)
    ok = r.flag == 0
    same = (cp == r.npp) & (cc == r.npc) & (cq == r.npq)
    say(f"  unflagged {ok.mean():.4f}, identical counts there {same[ok].mean():.4f}; "
        f"quadrupole terms {r.npq.sum() / max(r.npc.sum(), 1):.3f} of the cell terms")
    assert np.all(same[ok])
    e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
    assert np.sqrt(np.mean(e[ok] ** 2)) <= 1e-5 and e[ok].max() <= 1e-4
    check_flagged(ref, r.acc, a, r.flag, eps, max_flagged)


@pytest.mark.parametrize("kind,tau,tmax,fl", [
    ("plummer", 1e-2, 1.0, 0.0),
    ("clumpy", 10 ** -1.5, 1.5, 0.5),
])
def test_body_budget_mixed_matches_oracle(ctx, kind, tau, tmax, fl):
    eps = 0.005
    pos, mass, ref, an = _setup(kind, 20000, 25)
    say(f"per-body mixed-order budget: {kind}, tau {tau:.3g}, theta_max {tmax}, floor {fl}")
    out = _run_q(ctx, pos, mass, eps, mac=B.BH_MAC_BUDGET, order=B.BH_ORDER_MIXED,
                 mlp_theta_max=tmax, mlp_log10_tau=np.log10(tau), acc_norm=an, mlp_acc_floor=fl)
    r = oracle.walk_kc(ref, eps, tmax, tau, oracle.cell_kc(ref), an.astype(np.float64)[ref["perm"]],
                       floor=fl, order=oracle.ORDER_MIXED)
    assert 0.01 < r.npq.sum() / r.npc.sum() < 0.99  # both kinds of term present
    _check_q(ref, r, out, eps, 0.01)


@pytest.mark.parametrize("curve,cap", [("morton", CAP_BUDGET), ("hilbert", CAP_BUDGET),
                                       ("morton", 1200)])
def test_group_budget_mixed_matches_oracle(ctx, curve, cap):
    eps, tau, tmax, fl = 0.005, 10 ** -2.0, 1.5, 0.5
    pos, mass, ref, an = _setup("plummer" if cap == CAP_BUDGET else "clumpy", 20000, 26, curve)
    say(f"group mixed-order budget ({curve}, work cap {cap}): tau {tau:.3g}, floor {fl}")
    out = _run_q(ctx, pos, mass, eps,
                 curve=B.BH_CURVE_HILBERT if curve == "hilbert" else B.BH_CURVE_MORTON,
                 walk=B.BH_WALK_GROUP, mac=B.BH_MAC_BUDGET, order=B.BH_ORDER_MIXED,
                 mlp_theta_max=tmax, mlp_log10_tau=np.log10(tau), acc_norm=an,
                 mlp_acc_floor=fl, walk_cap=cap)
    kw = dict(group=B.BH_GROUP_BODIES, mode=1, order=oracle.ORDER_MIXED, theta_max=tmax, tau=tau,
              kc=oracle.cell_kc(ref), anorm=an.astype(np.float64)[ref["perm"]],
              tol=FLAG_TOL[np.float32], split=True, floor=fl)
    r = oracle.walk_group(ref, eps, cap=cap, **kw)
    if cap != CAP_BUDGET:  # part of the runs walked per body
        r0 = oracle.walk_group(ref, eps, cap=1 << 40, **kw)
        assert 0.1 < np.mean((r.npp != r0.npp) | (r.npc != r0.npc)) < 0.9
    assert 0.01 < r.npq.sum() / r.npc.sum() < 0.99
    _check_q(ref, r, out, eps, MAX_FLAGGED)


def test_quadrupole_count_by_order(ctx):
    """n_pq: every particle-cell term at order 2, none at order 0; the mixed
    order runs with the error budget only."""
    pos, _, mass = case_bodies("plummer", 3000, 27, np.float32)
    for walk in (B.BH_WALK_BODY, B.BH_WALK_GROUP):
        for order, mac in ((2, B.BH_MAC_THETA), (0, B.BH_MAC_THETA), (2, B.BH_MAC_BUDGET),
                           (0, B.BH_MAC_BUDGET)):
            _, _, cp, cc, cq = _run_q(ctx, pos, mass, 0.01, walk=walk, mac=mac, order=order)
            assert cc.sum() > 0
            np.testing.assert_array_equal(cq, cc if order == 2 else 0)
    t = B.bh_build(ctx, torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda(), 16)
    acc = torch.empty(3000, 3, device="cuda")
    try:
        for mac in (B.BH_MAC_THETA, B.BH_MAC_MLP, B.BH_MAC_THETA_GUARD):
            with pytest.raises(B.BHError):
                B.bh_forces(t, 0.5, 0.01, acc, B.force_opts(mac=mac, order=B.BH_ORDER_MIXED))
    finally:
        B.bh_tree_free(t)
