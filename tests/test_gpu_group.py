"""GPU group walk (one decision per group of BH_GROUP_BODIES bodies) against the
oracle's group walk."""
import numpy as np
import pytest
import torch

import oracle
from paper_2203_08966_amd import binding as B
from paper_2203_08966_amd import workloads as W
from tests.conftest import case_bodies, check_flagged, say

NO_CAP = 1 << 40

pytestmark = pytest.mark.gpu


def _run(ctx, pos, mass, leaf, theta, eps, **kw):
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, leaf)
    n = len(mass)
    acc = torch.empty_like(P)
    phi = torch.empty_like(M)
    npp = torch.zeros(n, dtype=torch.int32, device="cuda")
    npc = torch.zeros(n, dtype=torch.int32, device="cuda")
    an = kw.pop("acc_norm", None)
    an_t = None if an is None else torch.from_numpy(an).cuda()
    o = B.force_opts(walk=B.BH_WALK_GROUP, phi=phi, n_pp=npp, n_pc=npc, mlp_acc_norm=an_t, **kw)
    B.bh_forces(t, theta, eps, acc, o)
    torch.cuda.synchronize()
    B.bh_tree_free(t)
    return (acc.cpu().numpy().astype(np.float64), phi.cpu().numpy().astype(np.float64),
            npp.cpu().numpy(), npc.cpu().numpy())


# per-body relative error against the FP64 oracle: rms and max bounds of
# the FP32 and FP64 walks (as for the per-body walk)
TOL = {np.float32: (1e-5, 1e-4), np.float64: (1e-12, 1e-10)}
# relative margin around a decision threshold inside which the walk's
# arithmetic may decide either way.  FP32: the group box, the COM offset and
# the distance d_g^2 are each a few roundings (2^-24) of quantities up to
# about ten times d_g (large boxes), so d_g^2 is good to a few 1e-6; FP64 to
# about 1e-15, with the same factor.
FLAG_TOL = {np.float32: 1e-5, np.float64: 1e-9}
# share of bodies that may be flagged: one uncertain decision flags every
# body of its group (64), and a group takes some thousand decisions; the
# oracle flags 0-0.7 % of the bodies in these cases
MAX_FLAGGED = 0.02
# work caps stated by each test for both the library and the oracle (the
# method's definition: a run over the cap is walked per body)
CAP_THETA, CAP_BUDGET = 6144, 4096


def _check(ref, r, out, dtype, eps, max_flagged=MAX_FLAGGED):
    """Counts identical for every body of an unflagged group, forces within
    the walk's precision there; a flagged group may take a decision the other
    way, which swaps one approximation for another: bounded by the method's
    own error (check_flagged)."""
    rms_tol, max_tol = TOL[dtype]
    a, phi, cp, cc = (x[ref["perm"]] for x in out)
    ok = r.flag == 0
    same = (cp == r.npp) & (cc == r.npc)
    say(f"  unflagged {ok.mean():.4f}, identical counts there {same[ok].mean():.4f}")
    assert np.all(same[ok])
    e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
    ep = np.abs(phi - r.phi) / np.abs(r.phi)
    say(f"  rel err (unflagged): rms {np.sqrt(np.mean(e[ok] ** 2)):.3e} max {e[ok].max():.3e}")
    assert np.sqrt(np.mean(e[ok] ** 2)) <= rms_tol and e[ok].max() <= max_tol
    assert np.sqrt(np.mean(ep[ok] ** 2)) <= rms_tol
    check_flagged(ref, r.acc, a, r.flag, eps, max_flagged)


@pytest.mark.parametrize("kind,n,dtype,theta", [
    ("plummer", 20000, np.float32, 0.75),
    ("clumpy", 15000, np.float32, 0.6),
    ("plummer", 6000, np.float64, 0.8),
    ("two_spheres", 9000, np.float32, 1.0),
])
def test_group_walk_matches_oracle(ctx, kind, n, dtype, theta):
    pos, _, mass = case_bodies(kind, n, 11, dtype)
    eps, leaf = 0.005, 16
    say(f"group walk {kind} n={n} {np.dtype(dtype).name} theta {theta}")
    out = _run(ctx, pos, mass, leaf, theta, eps, walk_cap=CAP_THETA)
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), leaf)
    r = oracle.walk_group(ref, eps, group=B.BH_GROUP_BODIES, theta=theta, tol=FLAG_TOL[dtype],
                          cap=CAP_THETA, split=True)
    _check(ref, r, out, dtype, eps)


def test_group_walk_small_stack_same_result(ctx):
    """With a tiny LDS stack the opened subtrees take the stackless sweep:
    the same interactions (only their order differs)."""
    pos, _, mass = case_bodies("plummer", 12000, 12, np.float64)
    say("group walk: stack 1024 vs 8 vs 1 (FP64)")
    a0 = _run(ctx, pos, mass, 8, 0.7, 0.01)
    for cap in (8, 1):
        a1 = _run(ctx, pos, mass, 8, 0.7, 0.01, walk_stack=cap)
        np.testing.assert_array_equal(a0[2], a1[2])
        np.testing.assert_array_equal(a0[3], a1[3])
        e = np.linalg.norm(a0[0] - a1[0], axis=1) / np.linalg.norm(a0[0], axis=1)
        assert e.max() <= TOL[np.float64][1]


def test_group_walk_target_range_and_tiny_trees(ctx):
    pos, _, mass = case_bodies("plummer", 5000, 13, np.float64)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, 8)
    acc = torch.full_like(P, 5.0)
    B.bh_forces(t, 0.7, 0.01, acc, B.force_opts(walk=B.BH_WALK_GROUP, target_range=(100, 1337),
                                                 walk_cap=CAP_THETA))
    torch.cuda.synchronize()
    perm = B.bh_tree_export(t)["perm"].astype(np.int64)
    B.bh_tree_free(t)
    ref = oracle.build_all(pos, mass, 8)
    r = oracle.walk_group(ref, 0.01, group=B.BH_GROUP_BODIES, theta=0.7, target_range=(100, 1337),
                          tol=1e-9, cap=CAP_THETA, split=True)
    a = acc.cpu().numpy()
    ok = r.flag == 0
    e = np.linalg.norm(a[perm[100:1337]] - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
    assert ok.mean() >= 1 - MAX_FLAGGED and e[ok].max() <= TOL[np.float64][1]
    rest = np.setdiff1d(np.arange(5000), perm[100:1337])
    assert np.all(a[rest] == 5.0)
    # a root that is a leaf, and a single body
    for n in (10, 1):
        p, _, m = case_bodies("plummer", max(n, 2), 14, np.float64)
        p, m = p[:n].copy(), m[:n].copy()
        out = _run(ctx, p, m, 16, 0.7, 0.01)
        d, _ = oracle.direct(p, m, 0.01)
        np.testing.assert_allclose(out[0], d, rtol=1e-12, atol=1e-300)
        assert np.all(out[2] == n - 1) and np.all(out[3] == 0)


def test_group_budget_matches_oracle(ctx):
    pos, _, mass = case_bodies("plummer", 20000, 15, np.float32)
    eps, tau, tmax = 0.005, 10 ** -1.5, 1.2
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16)
    w = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], 0.4, eps)
    an = np.empty(20000)
    an[ref["perm"]] = np.linalg.norm(w.acc, axis=1)
    an = an.astype(np.float32)
    say(f"group budget walk: 20000 bodies, tau {tau:.3g}, theta_max {tmax}")
    out = _run(ctx, pos, mass, 16, 0.5, eps, mac=B.BH_MAC_BUDGET, mlp_theta_max=tmax,
               mlp_log10_tau=np.log10(tau), acc_norm=an, walk_cap=CAP_BUDGET)
    r = oracle.walk_group(ref, eps, group=B.BH_GROUP_BODIES, mode=1, theta_max=tmax, tau=tau,
                          kc=oracle.cell_kc(ref), anorm=an.astype(np.float64)[ref["perm"]],
                          tol=FLAG_TOL[np.float32], cap=CAP_BUDGET, split=True)
    _check(ref, r, out, np.float32, eps)


def test_group_budget_floor_matches_oracle(ctx):
    """The group error-budget walk with |a_i| floored at half the mean norm:
    a group's decision uses max(min |a_i|, floor)."""
    pos, _, mass = case_bodies("plummer", 20000, 15, np.float32)
    eps, tau, tmax, fl = 0.005, 10 ** -1.75, 1.5, 0.5
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16)
    w = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], 0.4, eps)
    an = np.empty(20000)
    an[ref["perm"]] = np.linalg.norm(w.acc, axis=1)
    an = an.astype(np.float32)
    say(f"group budget walk, floor {fl}: 20000 bodies, tau {tau:.3g}, theta_max {tmax}")
    out = _run(ctx, pos, mass, 16, 0.5, eps, mac=B.BH_MAC_BUDGET, mlp_theta_max=tmax,
               mlp_log10_tau=np.log10(tau), acc_norm=an, mlp_acc_floor=fl, walk_cap=CAP_BUDGET)
    args = dict(group=B.BH_GROUP_BODIES, mode=1, theta_max=tmax, tau=tau, kc=oracle.cell_kc(ref),
                anorm=an.astype(np.float64)[ref["perm"]], tol=FLAG_TOL[np.float32],
                cap=CAP_BUDGET, split=True)
    r = oracle.walk_group(ref, eps, floor=fl, **args)
    r0 = oracle.walk_group(ref, eps, **args)
    assert np.mean(r.npp + r.npc < r0.npp + r0.npc) > 0.05  # the floor is in effect
    _check(ref, r, out, np.float32, eps)


def test_group_walk_full_size_sampled(ctx):
    """The Plummer sphere of 2^20 bodies in the launch the benchmark times
    (FP32, quadrupole, leaf 16, eps 0.005): sampled groups against the
    oracle's group walk on the same groups."""
    b, cfg = W.config("c2")
    n = b.n
    theta = 0.75
    say(f"group walk full size: n={n}, theta {theta}, 24 sampled groups")
    out = _run(ctx, b.pos, b.mass, cfg["leaf"], theta, cfg["eps"], walk_cap=CAP_THETA)
    ref = oracle.build_all(b.pos.astype(np.float64), b.mass.astype(np.float64), cfg["leaf"])
    rng = np.random.default_rng(4)
    G = B.BH_GROUP_BODIES
    groups = rng.choice(n // G, 24, replace=False)
    a, phi, cp, cc = (x[ref["perm"]] for x in out)
    checked = 0
    for g in groups:
        r = oracle.walk_group(ref, cfg["eps"], group=B.BH_GROUP_BODIES, theta=theta,
                              target_range=(G * g, G * g + G), tol=FLAG_TOL[np.float32],
                              cap=CAP_THETA, split=True)
        sl = slice(G * g, G * g + G)
        if r.flag[0]:
            continue
        checked += 1
        assert np.array_equal(cp[sl], r.npp) and np.array_equal(cc[sl], r.npc)
        e = np.linalg.norm(a[sl] - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
        assert e.max() <= TOL[np.float32][1]
    say(f"  unflagged groups checked: {checked}")
    assert checked >= 12


@pytest.mark.parametrize("mode", [0, 1])
def test_group_walk_work_cap(ctx, mode):
    """With a low work cap part of the groups fall back to per-body
    decisions, exactly where the oracle's groups do.  The cap is the 70th
    percentile of the work of the uncapped oracle walk (a run's work is
    each of its bodies' npp + npc + 1), so that about 30 % of the bodies
    fall back."""
    pos, _, mass = case_bodies("clumpy", 20000, 16, np.float32)
    eps = 0.005
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), 16)
    G = B.BH_GROUP_BODIES
    if mode == 0:
        args = dict(group=G, theta=0.7, tol=FLAG_TOL[np.float32], split=True)
        kw = dict()
        theta = 0.7
    else:
        w = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], 0.4, eps)
        an = np.empty(20000)
        an[ref["perm"]] = np.linalg.norm(w.acc, axis=1)
        an = an.astype(np.float32)
        kw = dict(mac=B.BH_MAC_BUDGET, mlp_theta_max=1.0, mlp_log10_tau=-2.0, acc_norm=an)
        args = dict(group=G, mode=1, theta_max=1.0, tau=1e-2, kc=oracle.cell_kc(ref),
                    anorm=an.astype(np.float64)[ref["perm"]], tol=FLAG_TOL[np.float32],
                    split=True)
        theta = 0.5
    full = oracle.walk_group(ref, eps, cap=1 << 40, **args)
    cap = int(np.quantile(full.npp + full.npc + 1, 0.7))
    say(f"group walk work cap {cap}, mode {mode}")
    out = _run(ctx, pos, mass, 16, theta, eps, walk_cap=cap, **kw)
    r = oracle.walk_group(ref, eps, cap=cap, **args)
    fell = np.mean(full.npp + full.npc + 1 > cap)
    say(f"  fraction of bodies in groups over the cap: {fell:.3f}")
    assert 0.05 < fell < 0.95
    _check(ref, r, out, np.float32, eps)


def test_group_walk_repeat_is_bitwise_identical(ctx):
    """Later walks of the same tree with the same parameters walk the groups
    that exceeded the work cap per body straight away (the prediction made
    by the first walk); every result is unchanged bit for bit."""
    pos, _, mass = case_bodies("clumpy", 30000, 17, np.float32)
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, 16)
    outs = []
    for k in range(3):
        acc = torch.empty_like(P)
        npc = torch.zeros(30000, dtype=torch.int32, device="cuda")
        npp = torch.zeros(30000, dtype=torch.int32, device="cuda")
        B.bh_forces(t, 0.7, 0.005, acc, B.force_opts(walk=B.BH_WALK_GROUP, walk_cap=2000,
                                                      n_pp=npp, n_pc=npc))
        torch.cuda.synchronize()
        outs.append((acc.cpu().numpy(), npp.cpu().numpy(), npc.cpu().numpy()))
    B.bh_tree_free(t)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)


def test_group_walk_repeat_short_predictions(ctx):
    """With more than 4 groups per launched wavefront (2^22 bodies) a first
    excess is predicted for one walk only, then the group walk is tried
    again and the prediction doubles: walks 1-4 mix excesses found during
    the walk with predicted per-body walks, and every result is unchanged
    bit for bit.  A walk without a cap shows that groups did exceed it."""
    pos, _, mass = case_bodies("plummer", 1 << 22, 23, np.float32)
    n, cap = len(mass), 4096
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    say(f"repeat walks with short predictions: {n} bodies, cap {cap}")
    t = B.bh_build(ctx, P, M, 16)

    def walk(c):
        acc = torch.empty_like(P)
        npc = torch.zeros(n, dtype=torch.int32, device="cuda")
        npp = torch.zeros(n, dtype=torch.int32, device="cuda")
        B.bh_forces(t, 0.7, 0.005, acc, B.force_opts(walk=B.BH_WALK_GROUP, walk_cap=c,
                                                      n_pp=npp, n_pc=npc))
        torch.cuda.synchronize()
        return acc.cpu().numpy(), npp.cpu().numpy(), npc.cpu().numpy()

    outs = [walk(cap) for _ in range(4)]
    free = walk(1 << 30)
    B.bh_tree_free(t)
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert np.array_equal(a, b)
    fell = (outs[0][1] != free[1]) | (outs[0][2] != free[2])
    say(f"  bodies in groups over the cap: {fell.mean():.4f}")
    assert 0.0005 < fell.mean() < 0.5


def test_group_walk_prediction_after_rebuild(ctx):
    """After the tree object is rebuilt from moved bodies, a group predicted
    (by the previous walk) to exceed the work cap is walked per body even if
    it would now fit: every body's result is either the oracle's group-walk
    result or its per-body walk result at the same theta, and both occur."""
    pos, _, mass = case_bodies("clumpy", 20000, 16, np.float32)
    eps, cap, theta = 0.005, 2500, 0.7
    P, M = torch.from_numpy(pos).cuda(), torch.from_numpy(mass).cuda()
    t = B.bh_build(ctx, P, M, 16)
    n = len(mass)
    acc = torch.empty_like(P)
    npp = torch.zeros(n, dtype=torch.int32, device="cuda")
    npc = torch.zeros(n, dtype=torch.int32, device="cuda")
    o = B.force_opts(walk=B.BH_WALK_GROUP, walk_cap=cap, n_pp=npp, n_pc=npc)
    B.bh_forces(t, theta, eps, acc, o)  # makes the predictions
    rng = np.random.default_rng(5)
    pos2 = (pos + rng.normal(0, 1e-2, pos.shape)).astype(np.float32)
    P2 = torch.from_numpy(pos2).cuda()
    B.bh_build(ctx, P2, M, 16, tree=t)
    B.bh_forces(t, theta, eps, acc, o)
    torch.cuda.synchronize()
    B.bh_tree_free(t)
    ref = oracle.build_all(pos2.astype(np.float64), mass.astype(np.float64), 16)
    p = ref["perm"]
    a = acc.cpu().numpy().astype(np.float64)[p]
    cp, cc = npp.cpu().numpy()[p], npc.cpu().numpy()[p]
    rg = oracle.walk_group(ref, eps, group=B.BH_GROUP_BODIES, theta=theta, tol=FLAG_TOL[np.float32],
                           cap=cap, split=True)
    rb = oracle.walk(ref["tree"], ref["mom"], ref["spos"], ref["smass"], ref["L"], theta, eps)

    def same(r):
        e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
        return (cp == r.npp) & (cc == r.npc) & (e <= TOL[np.float32][1])
    sg, sb = same(rg), same(rb)
    only_b = sb & ~sg
    say(f"  group-walk results {sg.mean():.3f}, per-body only {only_b.mean():.3f}")
    assert np.mean(sg | sb) >= 0.99
    assert only_b.mean() > 0.005  # predicted groups walked per body
    assert sg.mean() > 0.5


def test_default_work_cap_by_criterion(ctx):
    """walk_cap = 0 means 6144 for the opening angle and 4096 for the error
    budget (the criteria's measured best caps): the defaults reproduce those
    caps bit for bit, and on the Plummer sphere of 2^20 bodies the other cap
    changes some results (groups lie between the two)."""
    b, cfg = W.config("c2")
    P = torch.from_numpy(np.ascontiguousarray(b.pos)).cuda()
    M = torch.from_numpy(np.ascontiguousarray(b.mass)).cuda()
    eps = cfg["eps"]
    t = B.bh_build(ctx, P, M, cfg["leaf"])
    acc = torch.empty_like(P)
    B.bh_forces(t, 0.5, eps, acc)
    an = acc.norm(dim=1).contiguous()
    say("default work caps: 2^20 bodies, opening angle and error budget")

    def walk(cap, **kw):
        out = torch.empty_like(P)
        B.bh_forces(t, 0.7, eps, out, B.force_opts(walk=B.BH_WALK_GROUP, walk_cap=cap, **kw))
        torch.cuda.synchronize()
        return out.cpu()
    budget = dict(mac=B.BH_MAC_BUDGET, mlp_log10_tau=-1.75, mlp_theta_max=1.5, mlp_acc_norm=an,
                  mlp_acc_floor=0.5)
    for kw, default, other in (({}, 6144, 4096), (budget, 4096, 6144)):
        a0 = walk(0, **kw)
        assert torch.equal(a0, walk(default, **kw))
        assert not torch.equal(a0, walk(other, **kw))
    B.bh_tree_free(t)


@pytest.mark.parametrize("curve,order,fl,log_tau", [
    ("morton", 2, 0.5, -1.75),
    ("hilbert", 0, 0.3, -2.0),   # the budget with monopole terms over Hilbert groups
])
def test_timed_path_budget_steps_match_oracle(ctx, curve, order, fl, log_tau):
    """The path the benchmark times: leapfrog steps with the group
    error-budget walk (quadrupole terms over Morton groups, or monopole
    terms over Hilbert groups), |a_i| floored at a fraction of the mean and
    taken from the previous step, a work cap, and the per-body predictions
    the steps carry from walk to walk.  Steps of dt = 0 keep the bodies in place (so every
    input of the oracle is the host's), while each step still rebuilds the
    tree in place, walks with the previous accelerations and kicks.  The
    oracle runs the same chain with its own accelerations: an estimate by a
    monopole group walk at theta 0.8 first, then one budget walk per step.
    After every step each body's force and counts equal the oracle's group
    walk or its per-body budget walk (a group predicted to exceed the cap is
    walked per body), except the groups that took a decision near a
    threshold in this step or hold a body that differed in the previous
    one (a flipped decision changes that body's |a_i|, and with it its
    group's next decisions)."""
    n, eps, leaf, cap, steps = 20000, 0.005, 16, 2000, 4
    tau, tmax, test = 10 ** log_tau, 1.5, 0.8
    pos, vel, mass = case_bodies("plummer", n, 19, np.float32)
    P, V, M = (torch.from_numpy(a).cuda() for a in (pos, vel, mass))
    o = B.force_opts(walk=B.BH_WALK_GROUP, mac=B.BH_MAC_BUDGET, order=order, walk_cap=cap,
                     mlp_log10_tau=np.log10(tau), mlp_theta_max=tmax, mlp_acc_floor=fl,
                     mlp_theta_est=test)
    say(f"timed path: {n} bodies, group budget walk of order {order} over {curve} groups, "
        f"cap {cap}, {steps} steps of dt 0")
    B.bh_ctx_set_curve(ctx, B.BH_CURVE_HILBERT if curve == "hilbert" else B.BH_CURVE_MORTON)
    try:
        B.bh_sim_init(ctx, P, V, M, leaf, 0.5, eps, o)
    finally:
        B.bh_ctx_set_curve(ctx, B.BH_CURVE_MORTON)
    ref = oracle.build_all(pos.astype(np.float64), mass.astype(np.float64), leaf, curve=curve)
    p = ref["perm"]
    kc = oracle.cell_kc(ref)
    G = B.BH_GROUP_BODIES
    est = oracle.walk_group(ref, eps, group=G, mode=0, order=0, theta=test, cap=cap, split=True,
                            tol=FLAG_TOL[np.float32])
    anorm = np.linalg.norm(est.acc, axis=1)
    exempt = est.flag != 0  # sorted order: bodies whose |a_i| may differ
    budget = dict(group=G, mode=1, theta_max=tmax, tau=tau, kc=kc, floor=fl, cap=cap,
                  split=True, tol=FLAG_TOL[np.float32], order=order)
    # groups over the cap (walked per body at once, then predicted for the
    # next steps) are part of this workload
    free = oracle.walk_group(ref, eps, anorm=anorm, **dict(budget, cap=NO_CAP))
    first = oracle.walk_group(ref, eps, anorm=anorm, **budget)
    over = np.mean((free.npp != first.npp) | (free.npc != first.npc))
    say(f"  bodies in groups over the cap at the start: {over:.3f}")
    assert over > 0.01
    for k in range(steps + 1):
        if k:
            B.bh_leapfrog_step(ctx, 0.0)
        a = torch.empty_like(P)
        B.bh_sim_get(ctx, None, None, a)
        torch.cuda.synchronize()
        a = a.cpu().numpy().astype(np.float64)[p]
        rg = oracle.walk_group(ref, eps, anorm=anorm, **budget)
        rb = oracle.walk_kc(ref, eps, tmax, tau, kc, anorm, floor=fl, order=order)

        def close(r):
            e = np.linalg.norm(a - r.acc, axis=1) / np.linalg.norm(r.acc, axis=1)
            return e <= TOL[np.float32][1]
        same_g, same_b = close(rg), close(rb)
        bad_group = np.repeat(np.add.reduceat(exempt | (rg.flag != 0), np.arange(0, n, G)) > 0,
                              G)[:n]
        match = same_g | same_b
        say(f"  step {k}: match {match.mean():.4f}, exempt groups hold {bad_group.mean():.4f}, "
            f"per-body results {np.mean(same_b & ~same_g):.4f}")
        assert np.all(match | bad_group)
        assert bad_group.mean() <= 0.05
        exempt = ~match
        # the oracle's next |a_i|: its own result where the GPU took the
        # group walk or the per-body walk, as the GPU did
        anorm = np.linalg.norm(np.where(same_b[:, None] & ~same_g[:, None], rb.acc, rg.acc),
                               axis=1)
