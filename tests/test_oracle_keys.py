"""Pins for the oracle's root cube, Morton keys and sort (Sec. 4.4, Sec. 4.7)."""
import json
import os

import numpy as np
import pytest

import oracle
from tests.conftest import GOLDEN


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def test_worked_example_2d_key():
    """Sec. 4.4 worked example: (3, 5) -> 27 with x more significant than y.
    Embedded in 3-D with z = 0, each octal digit of the 3-D key is twice the
    base-4 digit of the 2-D key (digit = 4 bx + 2 by + bz)."""
    g = _golden("morton_worked_example.json")
    bits = g["bits"]
    shift = 21 - bits
    k3 = oracle.interleave(g["x"] << shift, g["y"] << shift, 0)
    digits = [(k3 >> (3 * (20 - lvl))) & 7 for lvl in range(bits)]
    assert all(d % 2 == 0 for d in digits)
    k2 = 0
    for d in digits:
        k2 = 4 * k2 + d // 2
    assert k2 == g["key"]


def _octant_path(p, lo, L, levels):
    """Octant digits of a point, found geometrically: at each level compare
    the point with the midpoint of the cell that holds it."""
    lo = np.array(lo, dtype=float)
    side = float(L)
    out = []
    for _ in range(levels):
        half = side / 2
        b = [int(p[d] >= lo[d] + half) for d in range(3)]
        out.append(4 * b[0] + 2 * b[1] + b[2])
        lo = lo + half * np.array(b)
        side = half
    return out


def test_keys_match_geometric_octants():
    """Every octal digit of a key equals the octant the body occupies at that
    level, derived from cell midpoints (independent of the bit interleave)."""
    rng = np.random.default_rng(11)
    pos = rng.normal(size=(300, 3)) * [1.0, 3.0, 0.2] + [5.0, -2.0, 0.0]
    lo, L = oracle.root_cube(pos)
    k = oracle.keys(pos, lo, L)
    for i in range(pos.shape[0]):
        path = _octant_path(pos[i], lo, L, 21)
        kd = [(int(k[i]) >> (3 * (20 - l))) & 7 for l in range(21)]
        assert kd == path, i


def test_hashed_octant_labels():
    """Sec. 4.7 figure: cells 10..17 and 170..177; a point at the centre of each
    labelled cell must carry the label's digits at the top of its key."""
    g = _golden("hashed_octants.json")
    lo, L = np.zeros(3), 8.0
    for label, halves in g["labels"].items():
        c = np.zeros(3)
        side = L
        for h in halves:
            side /= 2
            c += side * np.array(h)
        c += side / 2
        k = oracle.keys(c[None, :], lo, L)[0]
        digits = label[1:]
        for lvl, ch in enumerate(digits):
            assert (int(k) >> (3 * (20 - lvl))) & 7 == int(ch, 8), label
        # hashed key of the cell: 1 followed by the octal digits
        hk = (1 << (3 * len(digits))) | (int(k) >> (3 * (21 - len(digits))))
        assert oct(hk)[2:] == label


def test_root_cube_contains_and_minimal():
    rng = np.random.default_rng(3)
    for trial in range(50):
        scale = 10.0 ** rng.uniform(-3, 3)
        pos = rng.normal(size=(int(rng.integers(1, 200)), 3)) * scale + rng.normal(size=3) * scale * 5
        lo, L = oracle.root_cube(pos)
        m, e = np.frexp(L)
        assert m == 0.5  # power of two
        assert np.all(pos >= lo) and np.all(pos < lo + L)
        assert np.all(np.fmod(lo, L / 2) == 0)
        # halving the side (with the corner snapped to L/4) never fits
        h = L / 2
        lo2 = np.floor(pos.min(0) / (h / 2)) * (h / 2)
        assert not np.all(pos.max(0) < lo2 + h)


def test_quadtree_figure_morton_order():
    """Sec. 4.4 figure: sorting the 21 points by key reproduces the drawn
    Morton polyline (fed in a shuffled order)."""
    g = _golden("quadtree21.json")
    pts = np.array(g["points_in_morton_order"])
    pos = np.column_stack([pts, np.full(len(pts), 0.5)])
    rng = np.random.default_rng(5)
    shuf = rng.permutation(len(pts))
    lo, L = oracle.root_cube(pos[shuf])
    assert L == g["root_side"] and list(lo[:2]) == g["root_lo"]
    k = oracle.keys(pos[shuf], lo, L)
    perm = oracle.sort(k)
    np.testing.assert_array_equal(shuf[perm], np.arange(len(pts)))


def test_sort_is_stable_and_sorted():
    rng = np.random.default_rng(9)
    k = rng.integers(0, 50, size=5000).astype(np.uint64)  # many ties
    perm = oracle.sort(k)
    ref = np.argsort(k, kind="stable")
    np.testing.assert_array_equal(perm, ref)


def test_key_quantisation_edges():
    """Bodies on a cell's lower face go to the upper cell; coordinates map to
    [0, 2^21 - 1]."""
    lo, L = np.zeros(3), 1.0
    pos = np.array([[0.0, 0.5, 1.0 - 2.0 ** -22], [0.5, 0.25, 0.75]])
    k = oracle.keys(pos, lo, L)
    q = (pos * 2 ** 21).astype(np.int64)
    q = np.minimum(q, 2 ** 21 - 1)
    for i in range(2):
        assert int(k[i]) == oracle.interleave(*map(int, q[i]))
    assert (int(k[0]) >> 60) & 7 == 0b011  # x lower, y upper, z upper
