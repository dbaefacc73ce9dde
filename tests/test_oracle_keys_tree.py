"""Pins for the oracle's root cube, Hilbert keys and flat octree (Sect. 3.4.1,
Sect. 3.4.6).  The Hilbert orientation itself is a reading (Skilling's transpose
form); what the paper fixes -- a space-filling curve through face-adjacent cells,
nested by level, and the two ordering properties of the flat tree -- is checked
here on exhaustive small grids and on seeded disks."""
import itertools

import numpy as np
import pytest

from paper_2310_20374_amd import inputs


def test_root_half_width(orc):
    z = np.zeros(3)
    assert orc.root_half_width(np.array([10.1, -3, 0]), z, z) == 16.0
    assert orc.root_half_width(np.array([8.0, 0, 0]), z, z) == 16.0     # strictly above
    assert orc.root_half_width(np.array([0.3, 0, 0]), z, z) == 0.5
    assert orc.root_half_width(np.array([0.0, 0, 0]), z, z) == 1.0
    assert orc.root_half_width(z, np.array([-7.99, 0, 0]), z) == 8.0


def test_quantize_edges(orc):
    L = 16.0
    assert orc.quantize(-16.0, L) == 0
    assert orc.quantize(0.0, L) == 1 << 20
    assert orc.quantize(16.0 - 1e-12, L) == (1 << 21) - 1
    assert orc.quantize(-16.0 + 2 * 16.0 / 2 ** 21, L) == 1
    # cell boundaries at every level fall on exact multiples of 2L/2^l
    for lev in range(1, 8):
        w = 2 * L / 2 ** lev
        for k in range(1, 2 ** lev):
            x = -L + k * w
            assert orc.quantize(x, L) >> (21 - lev) == k


@pytest.mark.parametrize("bits", [1, 2, 3, 4])
def test_hilbert_bijective_and_adjacent(orc, bits):
    side = 1 << bits
    pos = {}
    for cx, cy, cz in itertools.product(range(side), repeat=3):
        h = orc.hilbert_index(cx, cy, cz, bits)
        assert h not in pos
        pos[h] = (cx, cy, cz)
    assert sorted(pos) == list(range(side ** 3))
    for h in range(side ** 3 - 1):
        a, b = np.array(pos[h]), np.array(pos[h + 1])
        assert np.abs(a - b).sum() == 1, (h, pos[h], pos[h + 1])


def _cell_keys(orc, lev, L=16.0):
    """21-bit keys of the centres of every level-`lev` cell, cut to the level."""
    side = 1 << lev
    w = 2 * L / side
    cells = list(itertools.product(range(side), repeat=3))
    c = np.array(cells, dtype=np.float64)
    x, y, z = (-L + (c[:, k] + 0.5) * w for k in range(3))
    keys = orc.hilbert_keys(x, y, z, L)
    return np.array(cells), keys >> np.uint64(3 * (21 - lev))


@pytest.mark.parametrize("lev", [1, 2, 3, 4])
def test_key_prefix_is_a_hilbert_curve_at_every_level(orc, lev):
    cells, pref = _cell_keys(orc, lev)
    assert len(np.unique(pref)) == len(pref) == 8 ** lev
    order = np.argsort(pref)
    walk = cells[order]
    steps = np.abs(np.diff(walk, axis=0)).sum(axis=1)
    assert np.all(steps == 1)


def test_key_prefix_nesting(orc):
    """Every moonlet of a cell shares the cell's key prefix; the parent's prefix is
    the child's shifted by one digit (Sect. 3.4.6 ordering properties)."""
    rng = np.random.default_rng(3)
    L = 16.0
    pts = rng.uniform(-L, L, (4000, 3))
    keys = orc.hilbert_keys(pts[:, 0], pts[:, 1], pts[:, 2], L)
    q = np.array([[orc.quantize(v, L) for v in p] for p in pts[:300]])
    for lev in (1, 3, 6, 10):
        cell = q >> (21 - lev)
        pref = keys[:300] >> np.uint64(3 * (21 - lev))
        for i in range(300):
            same = np.all(cell == cell[i], axis=1)
            assert np.all(pref[same] == pref[i])
            other = ~same
            assert not np.any(pref[other] == pref[i])


def _check_tree(t, s):
    nc, n = t.ncells, t.n
    assert t.level[0] == 0 and t.first[0] == 0 and t.count[0] == n and t.parent[0] == -1
    # breadth-first by level, Hilbert (prefix) order within a level
    lv, pf = t.level.astype(np.int64), t.prefix
    for c in range(1, nc):
        assert (lv[c], pf[c]) > (lv[c - 1], pf[c - 1])
    leaves = t.nchild == 0
    assert np.all((t.count[leaves] <= s) | (t.level[leaves] == 21))
    assert np.all(t.count[~leaves] > s)
    # leaves tile the moonlets in tree order
    lf = np.where(leaves)[0]
    order = lf[np.argsort(t.first[lf])]
    assert t.first[order[0]] == 0
    assert np.all(t.first[order][1:] == (t.first[order] + t.count[order])[:-1])
    assert (t.first[order][-1] + t.count[order][-1]) == n
    for c in np.where(~leaves)[0]:
        ch = np.arange(t.child_first[c], t.child_first[c] + t.nchild[c])
        assert np.all(t.parent[ch] == c)
        assert np.all(t.level[ch] == t.level[c] + 1)
        assert t.count[ch].sum() == t.count[c]
        assert t.first[ch[0]] == t.first[c]
        assert np.all(t.first[ch][1:] == (t.first[ch] + t.count[ch])[:-1])
        assert np.all(t.prefix[ch] >> np.uint64(3) == t.prefix[c])
        assert 1 <= t.nchild[c] <= 8
    # order of children of different parents follows the parents' order
    # (second ordering property of the flat tree)
    for c in range(nc - 1):
        if t.nchild[c] and t.nchild[c + 1]:
            assert t.child_first[c] + t.nchild[c] == t.child_first[c + 1]
    # moonlets: sorted by (key, input index), and inside their cell's key range
    k = t.keys[t.perm]
    assert np.all((k[1:] > k[:-1]) | ((k[1:] == k[:-1]) & (t.perm[1:] > t.perm[:-1])))
    for c in range(nc):
        kk = k[t.first[c]: t.first[c] + t.count[c]] >> np.uint64(3 * (21 - t.level[c]))
        assert np.all(kk == t.prefix[c])


@pytest.mark.parametrize("s", [1, 4, 16, 52])
def test_tree_invariants_disk(orc, s):
    d = inputs.disk(3000, seed=1)
    t = orc.Tree(d["x"], d["y"], d["z"], s)
    assert t.L == 16.0
    _check_tree(t, s)


def test_tree_small_by_hand(orc):
    # four moonlets, s = 1: two in the (+,+,+) octant split once more
    x = np.array([1.0, 9.0, -5.0, 9.5])
    y = np.array([1.0, 9.0, -5.0, 1.0])
    z = np.array([1.0, 1.0, -5.0, 1.0])
    t = orc.Tree(x, y, z, 1)
    assert t.L == 16.0
    _check_tree(t, 1)
    # root -> 2 children (the (-,-,-) octant holds one moonlet, the (+,+,+) three)
    assert t.nchild[0] == 2
    lvl1 = np.where(t.level == 1)[0]
    assert sorted(t.count[lvl1].tolist()) == [1, 3]
    # no empty cells exist: every cell holds at least one moonlet
    assert np.all(t.count >= 1)


def test_tree_independent_of_insertion_order(orc):
    """Sect. 3.4.6: inserting in another order changes only the speed."""
    d = inputs.disk(2500, seed=2)
    t1 = orc.Tree(d["x"], d["y"], d["z"], 12)
    rng = np.random.default_rng(0)
    p = rng.permutation(len(d["x"]))
    t2 = orc.Tree(d["x"][p], d["y"][p], d["z"][p], 12)
    for f in ("level", "first", "count", "child_first", "nchild", "parent", "prefix"):
        assert np.array_equal(getattr(t1, f), getattr(t2, f)), f
    # same moonlets in the same cells (ties inside a leaf ordered by input index)
    assert np.array_equal(np.sort(p[t2.perm][:100]), np.sort(t1.perm[:100]))


def test_tree_depth_cap(orc):
    """Depth cap of 21 levels (the paper states none): more than s coincident moonlets
    stay in a depth-21 leaf."""
    x = np.full(5, 0.25); y = np.full(5, -0.5); z = np.full(5, 3.0)
    x = np.concatenate([x, [5.0]]); y = np.concatenate([y, [5.0]]); z = np.concatenate([z, [5.0]])
    t = orc.Tree(x, y, z, 2)
    _check_tree(t, 2)
    assert t.maxlevel == 21
    deep = np.where((t.level == 21) & (t.nchild == 0))[0]
    assert len(deep) == 1 and t.count[deep[0]] == 5
