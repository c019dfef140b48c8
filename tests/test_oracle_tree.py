"""Pins for the oracle's octree (Sec. 3 build by insertion; Sec. 4.2 pre-order
serialisation with child masks; Sec. 4.7 hashed keys)."""
import json
import os

import numpy as np
import pytest

import oracle
from tests.conftest import GOLDEN


def _tree_of(pos, leaf):
    b = oracle.build_all(pos, np.ones(len(pos)), leaf)
    return b


def test_quadtree_figure_levels():
    """Sec. 3 figure: 21 points, one body per leaf -> 31 cells, per level
    1, 4, 9, 9, 8; 21 leaves and 10 internal cells."""
    with open(os.path.join(GOLDEN, "quadtree21.json")) as f:
        g = json.load(f)
    pts = np.array(g["points_in_morton_order"])
    pos = np.column_stack([pts, np.full(len(pts), 0.5)])
    t = _tree_of(pos, 1)["tree"]
    lv = np.bincount(t["level"])
    assert list(lv) == g["nodes_per_level"]
    leaves = t["next"] == np.arange(1, len(t["next"]) + 1)
    assert leaves.sum() == g["leaves"] and (~leaves).sum() == g["internal"]
    assert np.all(t["count"][leaves] == 1)


def _insertion_tree(pos, leaf, lo, L):
    """The paper's build (Barnes-Hut loop body, 'Build Tree'): insert bodies
    one at a time into the leaf enclosing them; a leaf that now holds more
    than `leaf` bodies is split in half in each dimension and its bodies are
    pushed into the children.  Cells are tracked geometrically, by their
    integer coordinates at their level; splitting stops at level 21.
    Returns {(level, ix, iy, iz): count}."""
    cells = {(0, 0, 0, 0): []}
    is_leaf = {(0, 0, 0, 0): True}

    def child_of(cell, p):
        k, ix, iy, iz = cell
        side = L / 2 ** (k + 1)
        c = []
        for d, i in enumerate((ix, iy, iz)):
            mid = lo[d] + (2 * i + 1) * side
            c.append(2 * i + int(p[d] >= mid))
        return (k + 1, c[0], c[1], c[2])

    def insert(cell, j):
        while not is_leaf[cell]:
            cell = child_of(cell, pos[j])
            if cell not in cells:
                cells[cell] = []
                is_leaf[cell] = True
        cells[cell].append(j)
        if len(cells[cell]) > leaf and cell[0] < 21:
            is_leaf[cell] = False
            held = cells[cell]
            cells[cell] = []
            for h in held:
                insert(cell, h)

    for j in range(len(pos)):
        insert((0, 0, 0, 0), j)

    counts = {}

    def total(cell):
        if is_leaf[cell]:
            n = len(cells[cell])
        else:
            n = sum(total(c) for c in cells if c[0] == cell[0] + 1 and
                    (c[1] >> 1, c[2] >> 1, c[3] >> 1) == cell[1:])
        counts[cell] = n
        return n

    total((0, 0, 0, 0))
    return counts


def _cells_of(t):
    out = {}
    for h, k, c in zip(t["hkey"], t["level"], t["count"]):
        prefix = int(h) ^ (1 << (3 * int(k)))
        ix = iy = iz = 0
        for l in range(int(k)):
            d = (prefix >> (3 * (int(k) - 1 - l))) & 7
            ix, iy, iz = 2 * ix + (d >> 2), 2 * iy + ((d >> 1) & 1), 2 * iz + (d & 1)
        out[(int(k), ix, iy, iz)] = int(c)
    return out


@pytest.mark.parametrize("leaf", [1, 2, 3, 8])
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_matches_insertion_build(leaf, seed):
    """Brute force: the paper's insertion build (in any insertion order)
    yields the same set of cells and counts as the oracle's recursive split."""
    rng = np.random.default_rng(seed)
    n = 120
    pos = np.concatenate([rng.normal(size=(n - 20, 3)),
                          rng.normal(size=(20, 3)) * 1e-3 + 0.3])
    b = _tree_of(pos, leaf)
    order = rng.permutation(n)
    ins = _insertion_tree(pos[order], leaf, b["lo"], b["L"])
    assert _cells_of(b["tree"]) == ins


def test_coincident_bodies_cap_at_level_21():
    pos = np.zeros((10, 3))
    pos[5:] = 1.0
    t = _tree_of(pos, 2)["tree"]
    leaves = t["next"] == np.arange(1, len(t["next"]) + 1)
    assert set(t["level"][leaves]) == {21}
    assert sorted(t["count"][leaves]) == [5, 5]


def test_structure_invariants():
    rng = np.random.default_rng(4)
    pos = rng.standard_cauchy(size=(3000, 3))
    pos = np.clip(pos, -50, 50)
    for leaf in (1, 4, 16):
        b = _tree_of(pos, leaf)
        t, sk = b["tree"], b["keys"]
        m = len(t["hkey"])
        assert t["begin"][0] == 0 and t["count"][0] == len(pos) and t["parent"][0] == -1
        for i in range(m):
            k = int(t["level"][i])
            leaf_node = t["next"][i] == i + 1
            if leaf_node:
                assert t["count"][i] <= leaf or k == 21
                assert t["cmask"][i] == 0
            else:
                assert t["count"][i] > leaf and k < 21
                # children partition the parent's range, in octant order
                c, pos_ = i + 1, t["begin"][i]
                digits = []
                while c < t["next"][i]:
                    assert t["parent"][c] == i
                    assert t["hkey"][c] >> np.uint64(3) == t["hkey"][i]
                    assert t["begin"][c] == pos_
                    pos_ += t["count"][c]
                    digits.append(int(t["hkey"][c]) & 7)
                    c = t["next"][c]
                assert pos_ == t["begin"][i] + t["count"][i]
                assert digits == sorted(digits)
                assert t["cmask"][i] == sum(1 << d for d in digits)
            # every body in the cell carries the cell's key prefix
            b0, e0 = t["begin"][i], t["begin"][i] + t["count"][i]
            pref = sk[b0:e0] >> np.uint64(3 * (21 - k))
            assert np.all(pref == (t["hkey"][i] ^ np.uint64(1 << (3 * k))))
