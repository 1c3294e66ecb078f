"""The library's host-side regridding (Section 5.4, RDM-2 and RDM-3:
amg_cluster, amg_regrid_boxes) against the oracle, bit-exact: the boxes are
integers, so every box, in order, must be the oracle's.  Random blob-and-
noise tag sets in 2D and 3D at several efficiencies and minimum sides, the
hand-made sets of the oracle's own pins, three-level RDM-3 chains at ratios
2 and 4 with the default and explicit growth and blocking, and the argument
checks.  No GPU: these calls touch no device."""
import os

import numpy as np
import pytest

from oracle import regrid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02663_amd", "libamg.so")


@pytest.fixture(scope="module")
def A():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2506_02663_amd import amg
    return amg


def blobs(shape, seed, nblob=6, noise=0.02):
    rng = np.random.default_rng(seed)
    t = np.zeros(shape, bool)
    for _ in range(nblob):
        c = [rng.integers(0, n) for n in shape]
        r = [rng.integers(1, 5) for _ in shape]
        t[tuple(slice(max(0, a - b), a + b) for a, b in zip(c, r))] = True
    t |= rng.random(shape) < noise
    return t


@pytest.mark.parametrize("shape,seed", [((32, 24), 0), ((32, 24), 1), ((17, 29), 2), ((64, 64), 3),
                                        ((12, 10, 8), 4), ((9, 13, 11), 5)])
@pytest.mark.parametrize("eff,min_side", [(0.5, 2), (0.75, 2), (0.9, 1), (0.9, 3)])
def test_cluster_matches_the_oracle(A, shape, seed, eff, min_side):
    t = blobs(shape, seed)
    assert A.cluster(t, eff, min_side) == regrid.cluster(t, eff, min_side)


def test_cluster_edge_cases(A):
    assert A.cluster(np.zeros((8, 8), bool)) == []
    full = np.ones((5, 7, 3), bool)
    assert A.cluster(full) == [((0, 0, 0), (4, 6, 2))]
    one = np.zeros((1, 1), bool)
    one[0, 0] = True
    assert A.cluster(one) == [((0, 0), (0, 0))]
    # every cell tagged on a checkerboard: cuts until the minimum side stops them
    cb = (np.add.outer(np.arange(8), np.arange(8)) % 2).astype(bool)
    assert A.cluster(cb, 0.9, 2) == regrid.cluster(cb, 0.9, 2)
    # the oracle's hand-derived cases
    t = np.zeros((16, 16), bool)
    t[0:4, 0:8] = True
    t[0:12, 0:4] = True
    assert A.cluster(t) == [((0, 0), (11, 3)), ((0, 4), (3, 7))]


@pytest.mark.parametrize("ratio", [2, 4])
@pytest.mark.parametrize("dim", [2, 3])
def test_regrid_boxes_matches_the_oracle(A, ratio, dim):
    base = (16, 12) if dim == 2 else (8, 8, 6)
    shapes = [tuple(n * ratio ** l for n in base) for l in range(3)]
    if dim == 3 and ratio == 4:
        shapes = shapes[:2]  # keep the level-2 grid small
    tags = [blobs(s, 10 + l, nblob=3, noise=0.005) for l, s in enumerate(shapes)]
    want = regrid.new_boxes(shapes, tags, ratio)
    got = A.regrid_boxes(base, ratio, tags)
    assert got == want
    assert all(len(b) for b in got)
    # explicit growth and blocking, including the paper's one-cell growth
    for grow, block in [(1, 1), (1, 2), (3, 1)]:
        assert A.regrid_boxes(base, ratio, tags, grow=grow, block=block) == \
            regrid.new_boxes(shapes, tags, ratio, grow=grow, block=block)


def test_regrid_boxes_empty_finest_tags(A):
    shapes = [(16, 16), (32, 32)]
    t0 = np.zeros(shapes[0], bool)
    t0[3:6, 9:12] = True
    t1 = np.zeros(shapes[1], bool)
    assert A.regrid_boxes((16, 16), 2, [t0, t1]) == regrid.new_boxes(shapes, [t0, t1], 2)


def test_argument_errors(A):
    t = np.ones((4, 4), bool)
    with pytest.raises(A.AmgError):
        A.cluster(t, efficiency=0.0)
    with pytest.raises(A.AmgError):
        A.cluster(t, min_side=0)
    with pytest.raises(A.AmgError):
        A.regrid_boxes((4, 4), 3, [t])
    with pytest.raises(A.AmgError):
        A.regrid_boxes((4, 4), 2, [t], grow=-1)
    with pytest.raises(A.AmgError):
        A.regrid_boxes((4, 4), 2, [t], block=65)
    # more boxes than room: AMG_EUNSUPPORTED, count still reported
    cb = (np.add.outer(np.arange(8), np.arange(8)) % 2).astype(bool)
    with pytest.raises(A.AmgError):
        A.cluster(cb, 1.0, 1, max_boxes=2)
