"""Pins for the oracle's network (gradients, Adam, the bf16 and fp16 views,
the pinball loss), the hash of the training-pair selection, and the error
budget with k_C = 1 (the relative criterion without a network).  The
learned criterion's features, labels, bound and decisions are pinned in
test_oracle_learned.py."""
import numpy as np
import pytest

import oracle
from oracle import mlp
from paper_2203_08966_amd import workloads as W


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(64, 10))
    y = rng.normal(size=64)
    th = mlp.init(1) + rng.normal(size=mlp.NPARAM) * 0.05
    g = mlp.grad(th, X, y)
    h = 1e-6
    idx = rng.choice(mlp.NPARAM, size=120, replace=False)
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss(th + e, X, y) - mlp.loss(th - e, X, y)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, k


def test_adam_first_step_closed_form():
    """First Adam step: m_hat = g, v_hat = g^2, so the update is
    lr * g / (|g| + eps)."""
    th = np.array([0.5, -1.0, 2.0])
    g = np.array([0.3, -2e-3, 0.0])
    opt = mlp.Adam(3, lr=1e-2, eps=1e-8)
    th1 = opt.step(th, g)
    np.testing.assert_allclose(th1, th - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)


def test_training_reduces_loss():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, size=(2048, 10))
    y = np.sin(2 * X[:, 0]) + X[:, 1] * X[:, 2]
    th = mlp.init(5)
    opt = mlp.Adam(mlp.NPARAM, lr=3e-3)
    l0 = mlp.loss(th, X, y)
    for ep in range(300):
        b = rng.choice(2048, 256, replace=False)
        th = opt.step(th, mlp.grad(th, X[b], y[b]))
    assert mlp.loss(th, X, y) < 0.2 * l0


def test_bf16_views_agree():
    """The numpy and C writings of the bf16 network agree; bf16 rounding is
    round-to-nearest-even on the top 16 bits."""
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2 ** -8) == 1.0           # tie -> even
    assert mlp.bf16(1.0 + 3 * 2 ** -8) == 1.0 + 2 ** -6
    rng = np.random.default_rng(3)
    th = mlp.init(9) + rng.normal(size=mlp.NPARAM) * 0.1
    X = rng.normal(size=(50, 10))
    a = mlp.forward_bf16(th, X)
    b = np.array([oracle.mlp_bf16(th, x) for x in X])
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
    full, _ = mlp.forward(th, X)
    assert np.max(np.abs(a - full)) < 0.05 * np.max(np.abs(full)) + 0.05


def test_f16_rounding_and_views_agree():
    """The C oracle's binary16 rounding (written from the format's
    definition) equals numpy's float16 conversion, ties to even, subnormals
    and overflow included; the numpy and C writings of the fp16 network
    agree."""
    cases = [1.0, 1.0 + 2 ** -11, 1.0 + 3 * 2 ** -11, -(1.0 + 2 ** -11), 65504.0, 65519.0,
             65520.0, 1e6, 2 ** -14, 2 ** -24, 2 ** -25, 3 * 2 ** -26, 1e-9, 0.0, -0.0]
    assert oracle.f16r(1.0 + 2 ** -11) == 1.0                 # tie -> even
    assert oracle.f16r(1.0 + 3 * 2 ** -11) == 1.0 + 2 ** -9
    assert oracle.f16r(65519.0) == 65504.0 and np.isinf(oracle.f16r(65520.0))
    assert oracle.f16r(2 ** -25) == 0.0 and oracle.f16r(3 * 2 ** -26) == 2 ** -24
    rng = np.random.default_rng(4)
    xs = np.concatenate([cases, rng.normal(size=2000) * 10.0 ** rng.uniform(-9, 5, 2000)])
    xs = xs.astype(np.float32).astype(np.float64)
    want = mlp.f16(xs)
    got = np.array([oracle.f16r(x) for x in xs])
    assert np.array_equal(got, want)
    th = mlp.init(9) + rng.normal(size=mlp.NPARAM) * 0.1
    X = rng.normal(size=(50, 10))
    a = mlp.forward_bf16(th, X, rnd=mlp.f16)
    b = np.array([oracle.mlp_f16(th, x) for x in X])
    np.testing.assert_allclose(a, b, rtol=1e-12, atol=1e-12)
    full, _ = mlp.forward(th, X)
    # 11 significant bits: closer to the full network than the bf16 view
    assert np.max(np.abs(a - full)) < np.max(np.abs(mlp.forward_bf16(th, X) - full))


def test_splitmix64_reference_outputs():
    """SplitMix64 with state 0: the first three outputs of the published
    generator (state advances by the golden gamma before each mix)."""
    gamma = 0x9E3779B97F4A7C15
    outs = [oracle.splitmix64((k * gamma) % 2 ** 64) for k in range(3)]
    assert outs == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_cell_kc_without_network():
    b = W.plummer(1000, 2)
    bb = oracle.build_all(b.pos, b.mass, 8)
    kc = oracle.cell_kc(bb)
    side = bb["L"] * 2.0 ** -bb["tree"]["level"]
    np.testing.assert_allclose(kc, bb["mom"][0] * side ** 3, rtol=1e-15)


def test_walk_kc_limits():
    """tau = 0 never accepts a cell: the direct sum; an unbounded tau accepts
    whenever l/d < theta_max (the body outside the cell): the theta walk at
    theta_max."""
    b = W.plummer(3000, 5)
    bb = oracle.build_all(b.pos, b.mass, 8)
    kc = oracle.cell_kc(bb)
    anorm = np.ones(3000)
    none = oracle.walk_kc(bb, 0.01, 0.55, 0.0, kc, anorm)
    direct = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.0, 0.01)
    np.testing.assert_allclose(none.acc, direct.acc, rtol=1e-13, atol=0)
    assert np.all(none.npc == 0)
    every = oracle.walk_kc(bb, 0.01, 0.55, 1e300, kc, anorm)
    th = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.55, 0.01)
    np.testing.assert_allclose(every.acc, th.acc, rtol=1e-13, atol=0)
    assert np.array_equal(every.npc, th.npc)
    # above 1/sqrt(3) the guard keeps every accepted cell away from the body:
    # every other body is accounted for exactly once
    wide = oracle.walk_kc(bb, 0.01, 0.95, 1e300, kc, anorm)
    assert np.all(wide.ncov == 2999)


def test_relative_criterion_beats_theta():
    """The error-budget criterion (k_C = 1) reaches a given rms relative
    error with fewer interactions than the opening angle (quadrupole walk,
    Plummer sphere)."""
    b = W.plummer(20000, 8)
    bb = oracle.build_all(b.pos, b.mass, 16)
    samp = np.arange(0, 20000, 10)
    rank = np.empty(20000, dtype=np.int64)
    rank[bb["perm"]] = np.arange(20000)
    ad, _ = oracle.direct(b.pos, b.mass, 0.005, samp)
    full = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.4, 0.005)
    anorm = np.linalg.norm(full.acc, axis=1)

    def rms(acc):
        e = np.linalg.norm(acc - ad, axis=1) / np.linalg.norm(ad, axis=1)
        return np.sqrt(np.mean(e * e))
    th = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.55, 0.005,
                     targets=rank[samp])
    kc = oracle.cell_kc(bb)
    best = None
    for tau in (3e-4, 1e-3, 3e-3):
        r = oracle.walk_kc(bb, 0.005, 1.0, tau, kc, anorm, targets=rank[samp])
        if rms(r.acc) <= rms(th.acc):
            best = r
    assert best is not None
    assert (best.npp + best.npc).mean() < 0.8 * (th.npp + th.npc).mean()


def test_pinball_gradient_and_quantile():
    """Pinball loss: the analytic gradient matches central differences, and
    for a constant network the bias derivative vanishes exactly at the
    label's q-quantile (the fraction of labels below it equals q)."""
    rng = np.random.default_rng(21)
    X = rng.normal(size=(80, 10))
    y = rng.normal(size=80)
    th = mlp.init(4) + rng.normal(size=mlp.NPARAM) * 0.05
    q = 0.9
    g = mlp.grad(th, X, y, q)
    h = 1e-7
    for k in rng.choice(mlp.NPARAM, size=80, replace=False):
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss(th + e, X, y, q) - mlp.loss(th - e, X, y, q)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-5 * max(1.0, abs(fd)) + 1e-8, k
    # constant network: output = b3; d loss / d b3 = frac(y < b3) - q
    c = np.zeros(mlp.NPARAM)
    ys = np.sort(rng.normal(size=1000))
    for b3, frac in ((ys[899] + 1e-9, 0.9), (ys[499] + 1e-9, 0.5), (ys[949] + 1e-9, 0.95)):
        c[-1] = b3
        gb = mlp.grad(c, np.zeros((1000, 10)), ys, q)[-1]
        assert abs(gb - (frac - q)) < 1e-12
    c[-1] = ys[899] + 1e-9
    assert abs(mlp.grad(c, np.zeros((1000, 10)), ys, q)[-1]) < 1e-12


def test_floored_norms_hand_example():
    """max(|a_i|, f <|a|>): norms 1, 2, 3, 10 have mean 4."""
    a = np.array([1.0, 2.0, 3.0, 10.0])
    np.testing.assert_array_equal(oracle.floored_norms(a, 0.0), a)
    np.testing.assert_array_equal(oracle.floored_norms(a, 0.5), [2.0, 2.0, 3.0, 10.0])
    np.testing.assert_array_equal(oracle.floored_norms(a, 3.0), [12.0] * 4)


def test_walk_kc_floor_touches_only_bodies_below_it():
    """Each body's decisions depend on its own |a_i| only: bodies at or above
    the floor walk exactly as without it; bodies below it walk as with
    |a_i| = the floor, which accepts at least as much (never more
    interactions).  A floor above every norm turns the test into an absolute
    error bound, the same as a constant |a|."""
    b = W.plummer(3000, 6)
    bb = oracle.build_all(b.pos, b.mass, 8)
    kc = oracle.cell_kc(bb)
    full = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.4, 0.01)
    an = np.linalg.norm(full.acc, axis=1)
    tau, tm = 1e-3, 1.0
    r0 = oracle.walk_kc(bb, 0.01, tm, tau, kc, an)
    rf = oracle.walk_kc(bb, 0.01, tm, tau, kc, an, floor=0.5)
    fl = 0.5 * an.mean()
    above = an >= fl
    assert 0.1 < (~above).mean() < 0.9
    np.testing.assert_array_equal(rf.acc[above], r0.acc[above])
    assert np.array_equal(rf.npp[above], r0.npp[above])
    w0, wf = r0.npp + r0.npc, rf.npp + rf.npc
    assert np.all(wf[~above] <= w0[~above]) and np.mean(wf[~above] < w0[~above]) > 0.5
    const = oracle.walk_kc(bb, 0.01, tm, tau, kc, np.full(3000, fl))
    big = oracle.walk_kc(bb, 0.01, tm, tau, kc, an, floor=an.max() / an.mean())
    lev = an.max()
    const_big = oracle.walk_kc(bb, 0.01, tm, tau, kc, np.full(3000, lev))
    np.testing.assert_array_equal(big.acc, const_big.acc)
    np.testing.assert_array_equal(rf.acc[~above], const.acc[~above])
