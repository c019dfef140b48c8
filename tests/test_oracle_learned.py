"""Pins of the oracle's learned acceptance criterion, one decision per
(group, cell): its features, its label, the bound on a reduced-precision
evaluation of the network, the decision, and the training pairs."""
import numpy as np
import pytest

import oracle
from oracle import mlp as OM
from paper_2203_08966_amd import workloads as W
from tests.test_oracle_budget import A, B, C1, C2, MC1, MC2, SIDE, _com, _norms, _system

NO_CAP = 1 << 40


def _two_masses(axis, s, m=0.5):
    """Cell moments of two masses m at +-s along ``axis`` about the origin."""
    y = np.zeros((2, 3))
    y[0, axis], y[1, axis] = s, -s
    Q = np.zeros((3, 3))
    for v in y:
        Q += m * (3 * np.outer(v, v) - v @ v * np.eye(3))
    return Q[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]


def test_features_geometry_closed_form():
    """Box [-1, 1]^3, cell of side l with its COM at (5, 0, 0): d_g = 4,
    d_c = 5, half-diagonal sqrt(3).  Two equal masses at +-s on z: the
    quadrupole is diag(-2, -2, 4) m s^2, so along n = x the projection is
    -2 m s^2 and |Q|_F = 2 sqrt(6) m s^2."""
    s, l, m, eps = 0.1, 0.5, 0.5, 0.3
    Q = _two_masses(2, s, m)
    centre = np.array([5.1, 0.05, 0.0])
    f = oracle.gfeatures([-1, -1, -1], [1, 1, 1], centre, l, [5, 0, 0], 2 * m, Q, 2, 1, eps)
    np.testing.assert_allclose(f[0], np.log2(l / 4), rtol=1e-14)
    np.testing.assert_allclose(f[1], np.log2(5 / 4), rtol=1e-14)
    np.testing.assert_allclose(f[2], np.sqrt(3) / (np.sqrt(3) + 4), rtol=1e-14)
    np.testing.assert_allclose(f[3], -2 * m * s * s / (2 * m * l * l), rtol=1e-12)
    np.testing.assert_allclose(f[4], 2 * np.sqrt(6) * m * s * s / (2 * m * l * l), rtol=1e-12)
    np.testing.assert_allclose(f[5], -0.1 / l, rtol=1e-12)              # (COM - centre).x
    np.testing.assert_allclose(f[6], np.hypot(0.1, 0.05) / l, rtol=1e-12)
    np.testing.assert_allclose(f[7], 1 / 21, rtol=1e-14)
    np.testing.assert_allclose(f[8], eps / 4, rtol=1e-14)
    assert f[9] == 1.0
    # along z the projection is +4 m s^2
    f = oracle.gfeatures([-1, -1, -1], [1, 1, 1], [0, 0, 5], l, [0, 0, 5], 2 * m, Q, 2, 0, eps)
    np.testing.assert_allclose(f[3], 4 * m * s * s / (2 * m * l * l), rtol=1e-12)
    assert f[9] == 0.0 and f[5] == 0.0


def test_features_invariant_under_scale_translation_and_axis_swap():
    rng = np.random.default_rng(1)
    bl = rng.normal(size=3)
    bu = bl + rng.random(3)
    centre = bu + 2 + rng.random(3)
    com = centre + 0.1 * rng.normal(size=3)
    Q = rng.normal(size=6)
    f = oracle.gfeatures(bl, bu, centre, 0.7, com, 1.3, Q, 17, 0, 0.05)
    k, t = 3.0, np.array([10.0, -4.0, 2.5])
    g = oracle.gfeatures(k * bl + t, k * bu + t, k * centre + t, k * 0.7, k * com + t, 1.3,
                         k * k * Q, 17, 0, k * 0.05)
    np.testing.assert_allclose(g, f, rtol=1e-12, atol=1e-13)
    # swap x and y everywhere (the quadrupole's components follow)
    sw = [1, 0, 2]
    Qm = np.array([[Q[0], Q[1], Q[2]], [Q[1], Q[3], Q[4]], [Q[2], Q[4], Q[5]]])[sw][:, sw]
    Qs = Qm[[0, 0, 0, 1, 1, 2], [0, 1, 2, 1, 2, 2]]
    h = oracle.gfeatures(bl[sw], bu[sw], centre[sw], 0.7, com[sw], 1.3, Qs, 17, 0, 0.05)
    np.testing.assert_allclose(h, f, rtol=1e-12, atol=1e-13)


def _axis_tree(zs, s=0.05, m=0.5):
    """Two masses m at (c, c, c +- s), c = 10.6 (one cell of side 0.25),
    and light bodies on the line x = y = c at z = c - zs; the root cube
    [0, 16)^3 from two corner pins."""
    c = 10.6
    pos = [[c, c, c + s], [c, c, c - s]] + [[c, c, c - z] for z in zs] + [[0.01, 0.01, 0.01],
                                                                           [15.9, 15.9, 15.9]]
    mass = [m, m] + [1e-12] * len(zs) + [1e-12, 1e-12]
    return oracle.build_all(np.array(pos, dtype=float), np.array(mass), 1)


def test_label_on_axis_closed_form():
    """Two equal masses at +-s on an axis and group bodies on the axis at
    distances z: the exact field is m/(z - s)^2 + m/(z + s)^2 and monopole
    plus quadrupole give (2m/z^2)(1 + 3 x^2), x = s/z, so the label of the
    pair cell, in units of M l^3 / d_g^5, is
    log10(((1 - x)^-2 + (1 + x)^-2)/2 - 1 - 3 x^2) + 3 log10(z / l) at the
    nearest body (d_g = its distance z for a box on the axis)."""
    s = 0.05
    for zs in ([0.31], [0.4, 0.55], [0.6, 0.7, 0.9]):
        bb = _axis_tree(zs, s)
        assert bb["L"] == 16.0
        rank = np.empty(len(bb["perm"]), dtype=np.int64)
        rank[bb["perm"]] = np.arange(len(bb["perm"]))
        r = np.sort(rank[2:2 + len(zs)])
        assert r[-1] - r[0] == len(zs) - 1  # consecutive on the curve
        t = bb["tree"]
        # the cells holding exactly the pair (a chain of one-child cells:
        # the same mass distribution, so the same label)
        pair = [c for c in range(len(t["next"])) if t["count"][c] == 2
                and set(bb["perm"][t["begin"][c]:t["begin"][c] + 2]) == {0, 1}]
        assert len(pair) >= 1
        feat, lab, node, cnt = oracle.group_samples(bb, 0.0, 0.0, 100.0, 1.0, 1,
                                                    group=len(zs), cap=64,
                                                    target_range=(r[0], r[-1] + 1))
        z, x = min(zs), s / min(zs)
        for c in pair:
            side = bb["L"] * 2.0 ** -t["level"][c]
            expect = (np.log10(((1 - x) ** -2 + (1 + x) ** -2) / 2 - 1 - 3 * x * x)
                      + 3 * np.log10(z / side))
            k = list(node[0, :cnt[0]]).index(c)
            assert abs(lab[0, k] - expect) < 1e-9, (lab[0, k], expect)


def _fp32_eval(params, f):
    """The network evaluated in float32 with bf16 operands, sums in the
    opposite order from the oracle's (a reduced-precision evaluation the
    bound must cover)."""
    p = OM.unpack(params)
    bf = OM.bf16 if hasattr(OM, "bf16") else None
    assert bf is not None
    fr = bf(np.asarray(f, dtype=np.float32))
    W1 = bf(p["W1"].astype(np.float32))
    b1 = bf(p["b1"].astype(np.float32))
    W2 = bf(p["W2"].astype(np.float32))
    b2 = p["b2"].astype(np.float32)
    w3 = p["w3"].astype(np.float32)
    b3 = np.float32(p["b3"][0])
    h1 = np.zeros(32, dtype=np.float32)
    for j in range(32):
        acc = np.float32(0)
        for k in reversed(range(10)):
            acc = np.float32(acc + np.float32(W1[j, k] * fr[k]))
        acc = np.float32(acc + b1[j])
        h1[j] = bf(np.float32(max(acc, 0)))
    out = np.float32(0)
    for u in reversed(range(32)):
        acc = b2[u]
        for j in reversed(range(32)):
            acc = np.float32(acc + np.float32(W2[u, j] * h1[j]))
        out = np.float32(out + w3[u] * np.float32(max(acc, 0)))
    return float(np.float32(out + b3))


def test_network_bound_covers_a_float32_evaluation():
    """For random networks and inputs, with a feature placed on a bf16
    rounding midpoint and perturbed by 1e-6 relative either way (an FP32
    feature's error), the FP32 evaluation (sums in another order) lies
    within the bound of the FP64 one; away from midpoints the bound is
    tiny."""
    rng = np.random.default_rng(3)
    flips, plain = 0, []
    for trial in range(60):
        params = OM.init(100 + trial)
        params[1376:1408] = rng.normal(0, 0.3, 32)   # b2
        params[1440] = rng.normal()
        f = rng.normal(size=10) * 2
        if trial % 2:
            k = rng.integers(10)  # one feature on a rounding midpoint of bf16
            v = np.float32(f[k])
            u = v.view(np.uint32) & np.uint32(0xFFFF0000)
            f[k] = float((u | np.uint32(0x8000)).view(np.float32))
        pred, delta = oracle.gnet_bound(params, f)
        for sgn in (-1, 1):
            got = _fp32_eval(params, f * (1 + sgn * 1e-6))
            assert abs(got - pred) <= delta + 1e-12, (trial, got, pred, delta)
            flips += abs(got - pred) > 1e-4
        if trial % 2 == 0:
            plain.append(delta)
    assert flips > 0  # some midpoint flips did move the output
    assert np.median(plain) < 1e-4  # no feature on a midpoint: only FP32 sums


def test_constant_network_decision_flips_at_hand_threshold():
    """A network that outputs the constant c (all weights 0, output bias c):
    the cell is accepted for the group iff 10^c M l^3 / d_g^5 < tau a_min.  The
    opening angle 0.5 keeps the octant cell above it (l/d_g 0.72) out, so
    the pair cell C (l/d_g 0.36) is the cell decided."""
    tb, rank, c = _system()
    r0 = min(rank[1], rank[2])
    a_A, a_B = 1.3, 0.7
    an = _norms(rank, {1: a_A, 2: a_B})
    lo, hi = np.minimum(A, B), np.maximum(A, B)
    dg = np.linalg.norm(np.maximum(0.0, np.maximum(lo - _com(), _com() - hi)))
    cval = -1.25
    params = np.zeros(OM.NPARAM)
    params[-1] = cval
    M = MC1 + MC2
    tau_star = 10 ** cval * M * SIDE ** 3 / (dg ** 5 * min(a_A, a_B))
    for f, accepted in ((1 + 1e-3, True), (1 - 1e-3, False)):
        r = oracle.walk_group(tb, 0.0, group=2, mode=2, theta_max=0.5, tau=tau_star * f,
                              anorm=an, params=params, target_range=(r0, r0 + 2), cap=NO_CAP,
                              split=False)
        assert np.all(r.ncov == 5)
        assert np.all(r.npc == (1 if accepted else 0)), f
        assert np.all(r.npp == (3 if accepted else 5)), f
        assert np.all(r.flag == 0)


def _tree(n=4000, seed=3, leaf=8):
    b = W.plummer(n, seed)
    return oracle.build_all(b.pos, b.mass, leaf)


def test_learned_limits_and_one_body_groups():
    """tau -> infinity: the group opening-angle walk at theta_max; tau -> 0:
    every cell opened, the direct sum; a cap below every run's work: each
    body walked as a group of one, which is what group size 1 gives."""
    bb = _tree()
    n = len(bb["smass"])
    params = OM.init(5)
    an = np.ones(n)
    kw = dict(group=64, cap=NO_CAP, split=True)
    big = oracle.walk_group(bb, 0.01, mode=2, theta_max=0.8, tau=1e300, anorm=an, params=params,
                            **kw)
    th = oracle.walk_group(bb, 0.01, mode=0, theta=0.8, **kw)
    np.testing.assert_array_equal(big.npc, th.npc)
    np.testing.assert_allclose(big.acc, th.acc, rtol=1e-13, atol=0)
    tiny = oracle.walk_group(bb, 0.01, mode=2, theta_max=0.8, tau=1e-300, anorm=an,
                             params=params, **kw)
    assert np.all(tiny.npc == 0) and np.all(tiny.npp == n - 1)
    one = oracle.walk_group(bb, 0.01, group=1, mode=2, theta_max=0.8, tau=1e-3, anorm=an,
                            params=params, cap=NO_CAP, split=False)
    fb = oracle.walk_group(bb, 0.01, group=64, mode=2, theta_max=0.8, tau=1e-3, anorm=an,
                           params=params, cap=0, split=False)
    np.testing.assert_array_equal(one.npc, fb.npc)
    np.testing.assert_allclose(one.acc, fb.acc, rtol=1e-13, atol=0)
    assert np.all(one.ncov == n - 1)


def test_group_samples_are_exactly_the_band_cells_of_the_walk():
    """Brute force: a multi-body cell is a candidate of a group iff its cube
    misses the box, theta_lo <= l/d_g < theta_max, and every proper ancestor
    (below the root) either meets the box or has l >= theta_lo d_g; with
    keep = 1 the samples are exactly these cells, in pre-order."""
    bb = _tree(1500, 4, 4)
    t = bb["tree"]
    M, com, Q = bb["mom"]
    G, tlo, tmax = 64, 0.4, 1.2
    feat, lab, node, cnt = oracle.group_samples(bb, 0.01, tlo, tmax, 1.0, 9, group=G, cap=4096)
    n = len(bb["smass"])
    m = len(t["next"])
    parent = t["parent"]
    for q in range(0, (n + G - 1) // G, 5):
        p = bb["spos"][q * G:min(n, q * G + G)]
        bl, bu = p.min(axis=0), p.max(axis=0)
        bc, bh = 0.5 * (bl + bu), 0.5 * (bu - bl)

        def geo(c):
            side = bb["L"] * 2.0 ** -t["level"][c]
            k = int(t["level"][c])
            pre = int(t["hkey"][c]) ^ (1 << (3 * k))
            ix = iy = iz = 0
            for lv in range(k):
                d = (pre >> (3 * (k - 1 - lv))) & 7
                ix, iy, iz = 2 * ix + (d >> 2 & 1), 2 * iy + (d >> 1 & 1), 2 * iz + (d & 1)
            centre = bb["lo"] + (np.array([ix, iy, iz]) + 0.5) * side
            overlap = np.all(np.abs(centre - bc) <= 0.5 * side + bh)
            dg = np.linalg.norm(np.maximum(np.abs(com[c] - bc) - bh, 0.0))
            return side, overlap, dg
        want = []
        for c in range(1, m):
            if t["count"][c] == 1:
                continue
            side, ov, dg = geo(c)
            if ov or not (tlo * dg <= side < tmax * dg):
                continue
            a, ok = parent[c], True
            while a > 0:
                sa, oa, da = geo(a)
                if not oa and sa < tlo * da:
                    ok = False
                    break
                a = parent[a]
            if ok:
                want.append(c)
        assert list(node[q, :cnt[q]]) == want, q
    # the features of a sample are those of its (box, cell)
    q = 3
    p = bb["spos"][q * G:q * G + G]
    c = node[q, 0]
    side = bb["L"] * 2.0 ** -t["level"][c]
    f = oracle.gfeatures(p.min(axis=0), p.max(axis=0), np.zeros(3) + 0.0, side, com[c], M[c],
                         Q[c], t["count"][c], t["next"][c] == c + 1, 0.01)
    np.testing.assert_allclose(feat[q, 0][[0, 1, 2, 3, 4, 7, 8, 9]], f[[0, 1, 2, 3, 4, 7, 8, 9]],
                               rtol=1e-14)
    assert np.all(np.isfinite(lab[:, :1][cnt > 0]))


@pytest.mark.parametrize("keep", [0.25])
def test_group_samples_keep_rate(keep):
    bb = _tree(3000, 6, 8)
    _, _, _, c_all = oracle.group_samples(bb, 0.01, 0.3, 1.0, 1.0, 2)
    _, _, _, c_keep = oracle.group_samples(bb, 0.01, 0.3, 1.0, keep, 2)
    frac = c_keep.sum() / c_all.sum()
    assert abs(frac - keep) < 0.05
