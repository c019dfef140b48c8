"""Pins of the Peano-Hilbert ordering (Sec. 4.4 names it as the remedy for
the jumps of the Morton order; a method variant): the curve itself against
a hand-drawn order and the properties that make a curve a Hilbert curve,
and the tree and walk over Hilbert-sorted bodies against the Morton ones,
which hold the same cells in another order."""
import itertools

import numpy as np
import pytest

import oracle
from paper_2203_08966_amd import workloads as W


def test_two_dimensional_curve_is_hilberts():
    """On a 4 x 4 grid the curve is Hilbert's own, drawn by hand: the first
    quadrant is entered at the origin and left upward, the two upper
    quadrants are traversed left to right, and the curve ends in the lower
    right corner (points listed as (x, y) in the order visited)."""
    drawn = [(0, 0), (1, 0), (1, 1), (0, 1), (0, 2), (0, 3), (1, 3), (1, 2),
             (2, 2), (2, 3), (3, 3), (3, 2), (3, 1), (2, 1), (2, 0), (3, 0)]
    assert [oracle.hilbert(p, 2) for p in drawn] == list(range(16))
    # order 1: the quadrants in the order the order-2 curve visits them
    assert [oracle.hilbert(p, 1) for p in [(0, 0), (0, 1), (1, 1), (1, 0)]] == [0, 1, 2, 3]


@pytest.mark.parametrize("bits", [1, 2, 3])
def test_three_dimensional_curve_properties(bits):
    """On the 2^bits grid per axis: a bijection onto 0 .. 8^bits - 1 that
    starts at the origin; consecutive cells share a face; every aligned cube
    of side 2^j covers one range of 8^j consecutive indices starting at a
    multiple of 8^j (the nesting that lets a key prefix name a cell)."""
    N = 1 << bits
    idx = {p: oracle.hilbert(p, bits) for p in itertools.product(range(N), repeat=3)}
    inv = {v: p for p, v in idx.items()}
    assert sorted(idx.values()) == list(range(N ** 3))
    assert inv[0] == (0, 0, 0)
    for k in range(N ** 3 - 1):
        assert sum(abs(a - b) for a, b in zip(inv[k], inv[k + 1])) == 1, k
    for j in range(1, bits + 1):
        side = 1 << j
        for corner in itertools.product(range(0, N, side), repeat=3):
            vals = sorted(idx[tuple(c + o for c, o in zip(corner, off))]
                          for off in itertools.product(range(side), repeat=3))
            assert vals[0] % side ** 3 == 0
            assert vals == list(range(vals[0], vals[0] + side ** 3))


def test_21_bit_key_prefix_names_the_cell():
    """With 21 bits per axis, two points share their first 3k key bits
    exactly when they lie in the same level-k cell (same q >> (21 - k) on
    every axis)."""
    rng = np.random.default_rng(3)
    for _ in range(300):
        k = int(rng.integers(0, 22))
        a = rng.integers(0, 1 << 21, size=3)
        sh = 21 - k
        b = ((a >> sh) << sh) | rng.integers(0, 1 << sh, size=3) if sh else a.copy()
        if k > 0 and rng.random() < 0.5:  # move b to a neighbouring level-k cell
            ax = int(rng.integers(0, 3))
            cell = (b[ax] >> sh) ^ 1
            b[ax] = (cell << sh) | (b[ax] & ((1 << sh) - 1))
        ka, kb = oracle.hilbert(tuple(a), 21), oracle.hilbert(tuple(b), 21)
        same_cell = all((a >> sh) == (b >> sh))
        assert ((ka >> (3 * sh)) == (kb >> (3 * sh))) == same_cell


@pytest.mark.parametrize("kind,n,leaf", [("plummer", 5000, 8), ("clumpy", 8000, 16),
                                          ("coincident", 2000, 4)])
def test_hilbert_tree_has_the_morton_cells(kind, n, leaf):
    """Sorting along either curve gives the same cells (same hashed key,
    level, bodies, child mask), only in another pre-order; the moments of a
    cell agree to rounding (its bodies are summed in another order)."""
    from tests.conftest import case_bodies
    pos, _, mass = case_bodies(kind, n, 5, np.float64)
    A = oracle.build_all(pos, mass, leaf)
    H = oracle.build_all(pos, mass, leaf, curve="hilbert")
    ta, th = A["tree"], H["tree"]
    assert len(ta["hkey"]) == len(th["hkey"])
    ia = {int(h): i for i, h in enumerate(ta["hkey"])}
    ih = {int(h): i for i, h in enumerate(th["hkey"])}
    assert ia.keys() == ih.keys()
    # Hilbert keys sorted, ties in input order
    assert np.all(np.diff(H["keys"].astype(np.float64)) >= 0)
    for h, i in ia.items():
        j = ih[h]
        assert ta["level"][i] == th["level"][j] and ta["count"][i] == th["count"][j]
        assert ta["cmask"][i] == th["cmask"][j]
        ba = A["perm"][ta["begin"][i]:ta["begin"][i] + ta["count"][i]]
        bh = H["perm"][th["begin"][j]:th["begin"][j] + th["count"][j]]
        assert set(ba.tolist()) == set(bh.tolist())
    order = np.array([ih[int(h)] for h in ta["hkey"]])
    Ma, ca, Qa = A["mom"]
    Mh, ch, Qh = H["mom"]
    np.testing.assert_allclose(Mh[order], Ma, rtol=1e-13)
    np.testing.assert_allclose(ch[order], ca, rtol=1e-12, atol=1e-13 * A["L"])
    side = A["L"] * 2.0 ** -ta["level"].astype(float)
    assert np.all(np.abs(Qh[order] - Qa) <= 1e-10 * (Ma * side * side)[:, None] + 1e-300)
    # parents and skip pointers describe the same tree
    for i in range(len(ta["hkey"])):
        p = ta["parent"][i]
        q = th["parent"][order[i]]
        assert (p < 0 and q < 0) or (q == order[p])


def test_hilbert_walk_makes_the_same_decisions():
    """The per-body walk over the Hilbert tree meets each cell under the same
    test as over the Morton tree: the same particle-particle and
    particle-cell counts for every body whose decisions are not within
    rounding of the threshold, and the same forces to rounding."""
    b = W.plummer(4000, 8)
    A = oracle.build_all(b.pos, b.mass, 8)
    H = oracle.build_all(b.pos, b.mass, 8, curve="hilbert")
    ra = oracle.barnes_hut(None, None, 0.6, 0.01, 8, built=A)
    rh = oracle.barnes_hut(None, None, 0.6, 0.01, 8, built=H)
    ok = (ra.flag == 0) & (rh.flag == 0)
    assert ok.mean() > 0.99
    assert np.array_equal(ra.npp[ok], rh.npp[ok]) and np.array_equal(ra.npc[ok], rh.npc[ok])
    e = np.linalg.norm(ra.acc[ok] - rh.acc[ok], axis=1) / np.linalg.norm(ra.acc[ok], axis=1)
    assert e.max() < 1e-12
