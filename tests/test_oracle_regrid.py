"""Pins of the oracle's regridding and data migration (oracle/regrid.py,
Section 5.4, RDM-1..4):

* clustering: hand-derived boxes for two separated blobs (a hole in the
  signature), an L-shape (the strongest inflection of the signature, along
  y) and a full rectangle; on random tag sets, every tagged cell covered,
  boxes disjoint and tight (every face touches a tag), each box efficient
  or without an admissible cut;
* RDM-3: the new levels cover the refined tags of the level below and are
  properly nested with a margin (each new level-2 box, coarsened twice and
  grown by the default growth, then refined once, lies in new level 1), and
  form a valid hierarchy on which every AMRCFI window stays on the coarser
  level (the paper's one-cell growth does not at ratio 2: a pinned
  counter-example); blocked boxes are aligned to blocks of at least four
  cells, on random regrids at ratios 2 and 4;
* migration: the copy on common cells is exact, and cell averages of a
  polynomial of degree <= 4 per direction are reproduced on every new cell
  (AMRCFI is exact to that degree);
* vorticity: exact for velocities polynomial of degree <= 4 (the
  fourth-order gradient is) on valid cells away from the physical boundary
  (whose fill carries homogeneous data), ratios 2 and 4.
"""
import numpy as np
import pytest

from oracle import amr, regrid
from oracle.level import PAD
from tests.polyfix import Poly1


def test_two_blobs_split_at_the_hole():
    t = np.zeros((16, 16), bool)
    t[2:5, 3:6] = True
    t[10:13, 9:12] = True
    assert regrid.cluster(t) == [((2, 3), (4, 5)), ((10, 9), (12, 11))]


def test_l_shape_splits_at_the_strongest_inflection():
    t = np.zeros((16, 16), bool)
    t[0:4, 0:8] = True    # x 0..3, y 0..7
    t[0:12, 0:4] = True   # x 0..11, y 0..3
    # signature along y: 12 12 12 12 4 4 4 4 (second differences -8 at y = 3,
    # +8 at y = 4: jump 16); along x: 8 8 8 8 4 ... (jump 8): cut at y = 4
    assert regrid.cluster(t) == [((0, 0), (11, 3)), ((0, 4), (3, 7))]


def test_full_rectangle_is_one_box():
    t = np.zeros((8, 8, 8), bool)
    t[1:5, 2:7, 3:4] = True
    assert regrid.cluster(t) == [((1, 2, 3), (4, 6, 3))]


@pytest.mark.parametrize("dim,seed", [(2, 0), (2, 1), (2, 2), (3, 3)])
def test_clustering_properties_on_random_tags(dim, seed):
    rng = np.random.default_rng(seed)
    shape = (32, 24) if dim == 2 else (12, 10, 8)
    t = np.zeros(shape, bool)
    for _ in range(6):  # blobs of random size
        c = [rng.integers(0, n) for n in shape]
        r = [rng.integers(1, 5) for _ in shape]
        t[tuple(slice(max(0, a - b), a + b) for a, b in zip(c, r))] = True
    t |= rng.random(shape) < 0.02
    boxes = regrid.cluster(t, efficiency=0.7, min_side=2)
    cov = np.zeros(shape, int)
    for lo, hi in boxes:
        sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
        cov[sl] += 1
        sub = t[sl]
        for d in range(dim):  # tight
            assert sub.take(0, axis=d).any() and sub.take(-1, axis=d).any()
        eff = sub.sum() / sub.size
        if eff < 0.7:
            assert regrid._cut(t, lo, hi, 2) is None
    assert np.all(cov[t] == 1) and cov.max() == 1


def test_new_hierarchy_is_nested_and_covers_the_tags():
    r = 2
    shapes = [(16, 16), (32, 32)]
    t0 = np.zeros(shapes[0], bool)
    t0[6:9, 6:9] = True
    t1 = np.zeros(shapes[1], bool)
    t1[14:17, 15:20] = True
    new = regrid.new_boxes(shapes, [t0, t1], r)
    assert len(new) == 2 and new[0] and new[1]
    lev1 = np.zeros((32, 32), bool)
    for lo, hi in new[0]:
        lev1[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1] = True
    # tags of level 0 refined are in new level 1; tags of level 1 in new level 2
    assert lev1[np.kron(t0, np.ones((2, 2), bool))].all()
    lev2 = np.zeros((64, 64), bool)
    for lo, hi in new[1]:
        lev2[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1] = True
    assert lev2[np.kron(t1, np.ones((2, 2), bool))].all()
    # proper nesting with a margin: level-2 boxes coarsened twice and grown by
    # two cells (the default at ratio 2), refined to level 1, lie in level 1
    assert regrid.default_growth(2) == 2 and regrid.default_growth(4) == 1
    for lo, hi in new[1]:
        clo = [max(a // 4 - 2, 0) * 2 for a in lo]
        chi = [min(b // 4 + 2, 15) * 2 + 1 for b in hi]
        assert lev1[clo[0]:chi[0] + 1, clo[1]:chi[1] + 1].all()
    # a valid hierarchy (nesting, refinement) on which every AMRCFI and
    # refluxing window stays on the coarser level (composite_apply raises
    # otherwise)
    H = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], new[0], new[1]],
                      {(d, s): "D" for d in range(2) for s in (0, 1)})
    H.composite_apply([lev.zeros() for lev in H.levels], "poisson", 0.0)


def test_one_cell_growth_leaves_windows_off_the_coarser_level_at_ratio_2():
    # the paper's one-cell expansion nests the levels with one cell of level
    # 1 between levels 2 and 0, too little for the five-cell window
    shapes = [(16, 16), (32, 32)]
    t0 = np.zeros(shapes[0], bool)
    t1 = np.zeros(shapes[1], bool)
    t1[14:18, 14:18] = True
    new1 = regrid.new_boxes(shapes, [t0, t1], 2, grow=1)
    H = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], new1[0], new1[1]],
                      {(d, s): "D" for d in range(2) for s in (0, 1)})
    with pytest.raises(ValueError, match="window leaves"):
        H.composite_apply([lev.zeros() for lev in H.levels], "poisson", 0.0)
    new2 = regrid.new_boxes(shapes, [t0, t1], 2)
    H = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], new2[0], new2[1]],
                      {(d, s): "D" for d in range(2) for s in (0, 1)})
    H.composite_apply([lev.zeros() for lev in H.levels], "poisson", 0.0)


@pytest.mark.parametrize("ratio", [2, 4])
def test_default_growth_keeps_windows_on_random_regrids(ratio):
    for seed in range(4):
        rng = np.random.default_rng(seed)
        shapes = [(16, 16), (16 * ratio, 16 * ratio)]
        tags = [rng.random(s) < 0.01 for s in shapes]
        tags[1][tuple(slice(int(a), int(a) + 3 * ratio) for a in rng.integers(2 * ratio, 12 * ratio, 2))] = True
        new = regrid.new_boxes(shapes, tags, ratio)
        q = regrid.default_blocking(ratio) * ratio  # boxes aligned to blocks of q cells
        assert q >= 4
        for lo, hi in new[0] + new[1]:
            assert all(a % q == 0 and (c + 1) % q == 0 for a, c in zip(lo, hi))
        H = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))]] + [b for b in new if b],
                          {(d, s): "D" for d in range(2) for s in (0, 1)}, ratio=ratio)
        H.composite_apply([lev.zeros() for lev in H.levels], "poisson", 0.0)


P = [Poly1([0.3, -1.0, 0.5, 2.0, -1.5]), Poly1([1.0, 0.7, -2.0, 0.25, 1.0])]


def poly_avgs(lev):
    a = lev.zeros()
    a[lev.inner] = np.multiply.outer(P[0].avg(0.0, lev.h, lev.shape[0]), P[1].avg(0.0, lev.h, lev.shape[1]))
    return np.where(lev.mask, a, 0.0)


@pytest.mark.parametrize("ratio", [2, 4])
def test_migration_copies_and_reproduces_polynomials(ratio):
    bc = {(d, s): "D" for d in range(2) for s in (0, 1)}
    n1 = 16 * ratio
    old = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((4 * ratio, 4 * ratio), (10 * ratio - 1, 10 * ratio - 1))]],
                        bc, ratio=ratio)
    new = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((6 * ratio, 2 * ratio), (13 * ratio - 1, 8 * ratio - 1))]],
                        bc, ratio=ratio)
    rng = np.random.default_rng(5)
    U_old = [np.where(lev.mask, rng.normal(size=lev.pshape), 0.0) for lev in old.levels]
    U_new = regrid.migrate(old, new, U_old)
    common = new.levels[1].mask & old.levels[1].mask
    assert np.array_equal(U_new[1][common], U_old[1][common])
    assert np.array_equal(U_new[0][new.levels[0].mask], U_old[0][new.levels[0].mask])
    # polynomial data: every migrated cell equals the exact average
    U_old = [poly_avgs(lev) for lev in old.levels]
    U_new = regrid.migrate(old, new, U_old)
    want = poly_avgs(new.levels[1])
    assert np.abs(U_new[1] - want)[new.levels[1].mask].max() < 1e-12 * np.abs(want).max()
    assert n1 == new.levels[1].shape[0]


@pytest.mark.parametrize("ratio", [2, 4])
def test_vorticity_exact_on_polynomial_velocities(ratio):
    bc = {(d, s): "D" for d in range(2) for s in (0, 1)}
    H = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((4 * ratio, 4 * ratio), (11 * ratio - 1, 11 * ratio - 1))]],
                      bc, ratio=ratio)
    # u = (P0(x) P1(y), P1(x) P0(y)): omega = P1'(x) P0(y) - P0(x) P1'(y)
    U = [[], []]
    want = []
    for lev in H.levels:
        def avg(px, py):
            a = lev.zeros()
            a[lev.inner] = np.multiply.outer(px.avg(0.0, lev.h, lev.shape[0]), py.avg(0.0, lev.h, lev.shape[1]))
            return a
        U[0].append(np.where(lev.mask, avg(P[0], P[1]), 0.0))
        U[1].append(np.where(lev.mask, avg(P[1], P[0]), 0.0))
        w = avg(P[1].d1(), P[0]) - avg(P[0], P[1].d1())
        want.append(np.where(lev.mask, w, 0.0))
    W = regrid.vorticity(H, U)
    for l, lev in enumerate(H.levels):
        # away from the physical boundary (its fill carries homogeneous data)
        inner = np.zeros(lev.pshape, bool)
        inner[tuple(slice(PAD + 2, PAD + n - 2) for n in lev.shape)] = True
        valid = H.valid[l] & inner
        assert np.abs(W[l] - want[l])[valid].max() < 1e-9 * np.abs(want[l]).max(), l
