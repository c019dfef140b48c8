"""Pins of the octopole term (Sec. 2.2, the l = 3 term of the multipole
expansion): the moments against the Legendre sum they stand for, the
particle-cell field on the axis of two unequal masses in closed form, and
the error slope 4 of an order-3 expansion."""
import numpy as np

import oracle


def test_octopole_is_the_legendre_term():
    """-O:xxx / (6 r^7) equals -sum m |y|^3 P_3(cos g) / r^4 (P_3 the
    Legendre polynomial, g the angle between x and y) for random bodies and
    field points; O is symmetric and traceless."""
    rng = np.random.default_rng(4)
    pos = rng.normal(size=(9, 3)) * 0.2 + 3.0
    mass = rng.random(9) + 0.2
    bb = oracle.build_all(np.concatenate([pos, [[-9, -9, -9]]]), np.concatenate([mass, [0.0]]),
                          16)
    O = oracle.octopole(bb)
    c = 0  # the root holds every body
    com = bb["mom"][1][c]
    o = O[c]
    full = np.zeros((3, 3, 3))
    idx = [(0, 0, 0), (0, 0, 1), (0, 0, 2), (0, 1, 1), (0, 1, 2), (0, 2, 2), (1, 1, 1),
           (1, 1, 2), (1, 2, 2), (2, 2, 2)]
    for k, (a, b, cc) in enumerate(idx):
        for p in {(a, b, cc), (a, cc, b), (b, a, cc), (b, cc, a), (cc, a, b), (cc, b, a)}:
            full[p] = o[k]
    np.testing.assert_allclose(np.einsum("abb->a", full), 0.0, atol=1e-12 * np.abs(o).max())
    y = pos - com
    for _ in range(5):
        x = rng.normal(size=3) * 5.0
        r = np.linalg.norm(x)
        cosg = (y @ x) / (np.linalg.norm(y, axis=1) * r)
        p3 = 0.5 * (5 * cosg ** 3 - 3 * cosg)
        legendre = -np.sum(mass * np.linalg.norm(y, axis=1) ** 3 * p3) / r ** 4
        moment = -np.einsum("abc,a,b,c->", full, x, x, x) / (6 * r ** 7)
        np.testing.assert_allclose(moment, legendre, rtol=1e-12)


def test_on_axis_field_of_two_unequal_masses():
    """Masses m1 at +s1 and m2 at -s2 on the z axis with m1 s1 = m2 s2 (COM at
    the origin), field point on the axis at -z: along the axis toward the
    field point the masses sit at -s1 and +s2, so the expansion to order l
    gives a_z = sum_{k <= l} (k + 1) M_k / z^(k + 2) with
    M_k = m1 (-s1)^k + m2 s2^k (M_1 = 0).  The order-3 walk equals this to
    rounding, and its octopole term 4 M_3 / z^5 is not zero for unequal
    masses."""
    m1, m2, s1 = 0.3, 0.7, 0.07
    s2 = m1 * s1 / m2
    c = np.array([10.6, 10.6, 10.6])  # inside one cell of side 0.25
    for z in (0.5, 0.8, 1.3):
        pos = np.array([c + [0, 0, s1], c - [0, 0, s2], c - [0, 0, z], [0.01] * 3, [15.9] * 3])
        mass = np.array([m1, m2, 0.0, 0.0, 0.0])
        bb = oracle.build_all(pos, mass, 1)
        rank = np.empty(5, dtype=np.int64)
        rank[bb["perm"]] = np.arange(5)
        Mk = [m1 * (-s1) ** k + m2 * s2 ** k for k in range(5)]
        assert abs(Mk[1]) < 1e-15 and abs(Mk[3]) > 1e-6
        # the body sits below the pair: the field points up (+z), toward it
        for order, terms in ((2, (0, 2)), (3, (0, 2, 3))):
            r = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 10.0, 0.0,
                            order=order, targets=[rank[2]],
                            oct=oracle.octopole(bb) if order == 3 else None)
            assert r.npc[0] >= 1
            expect = sum((k + 1) * Mk[k] / z ** (k + 2) for k in terms)
            np.testing.assert_allclose(r.acc[0], [0, 0, expect], rtol=1e-12, atol=1e-12 * expect)
        exact = m1 / (z + s1) ** 2 + m2 / (z - s2) ** 2
        # what order 3 leaves is the l = 4 term, to leading order
        assert abs((exact - expect) / (5 * Mk[4] / z ** 6) - 1) < 0.2


def test_error_slope_four():
    """The relative particle-cell error falls like (size/d)^4 with the
    octopole (and like (size/d)^3 with the quadrupole on the same cluster)."""
    rng = np.random.default_rng(1)
    cl = rng.random((12, 3)) * 0.05 + 100.0
    mass = np.concatenate([rng.random(12) + 0.5, [0.0]])
    direction = np.array([0.6, -0.48, 0.64])
    errs = {2: [], 3: []}
    ds = np.array([0.4, 0.8, 1.6, 3.2])
    for d in ds:
        tgt = cl.mean(0) + d * direction
        pos = np.concatenate([cl, tgt[None]])
        bb = oracle.build_all(pos, mass, 12)
        exact, _ = oracle.direct(pos, mass, 0.0, targets=[12])
        for order in (2, 3):
            r = oracle.barnes_hut(pos, mass, 100.0, 0.0, 12, order=order, targets=[12], built=bb)
            assert r.npc[0] >= 1
            errs[order].append(np.linalg.norm(r.acc[0] - exact[0]) / np.linalg.norm(exact[0]))
    s2 = np.polyfit(np.log(ds), np.log(errs[2]), 1)[0]
    s3 = np.polyfit(np.log(ds), np.log(errs[3]), 1)[0]
    assert -3.4 < s2 < -2.6, s2
    assert -4.4 < s3 < -3.6, s3
    assert all(e3 < e2 for e2, e3 in zip(errs[2], errs[3]))


def test_order_three_walk_limits():
    """theta = 0 is still the direct sum; every other body is covered once
    (theta below 1/sqrt(3)); at equal theta the order-3 walk is more
    accurate than order 2."""
    from paper_2203_08966_amd import workloads as W
    b = W.plummer(3000, 21)
    bb = oracle.build_all(b.pos, b.mass, 8)
    O = oracle.octopole(bb)
    d, _ = oracle.direct(bb["spos"], bb["smass"], 0.01)
    r0 = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.0, 0.01,
                     order=3, oct=O)
    np.testing.assert_allclose(r0.acc, d, rtol=1e-12, atol=1e-12 * np.abs(d).max())
    e = {}
    for order in (2, 3):
        r = oracle.walk(bb["tree"], bb["mom"], bb["spos"], bb["smass"], bb["L"], 0.55, 0.01,
                        order=order, oct=O if order == 3 else None)
        assert np.all(r.ncov == 2999)
        er = np.linalg.norm(r.acc - d, axis=1) / np.linalg.norm(d, axis=1)
        e[order] = np.sqrt(np.mean(er * er))
    assert e[3] < 0.6 * e[2], e
