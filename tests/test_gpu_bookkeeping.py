"""Box and index bookkeeping, bit-exact against the oracle.

For every level of a set of layouts (one box, tiled boxes, boxes with gaps,
coarse-fine levels with two components, the two-level disk layout, the
three-level vortex layout, a batch of isolated boxes) the library's box table
(amg_box_info) must give, at every multigrid depth, exactly the boxes of the
oracle's coarsening (Level.hierarchy(): corners halved while every box stays
even, at least 8 wide and facing boxes stay apart), in the caller's order;
its component ids must be the oracle's face-connected labels (scipy's
ndimage.label) up to a relabelling that is one-to-one, and its singular
flags the oracle's pure-Neumann components.  The library is never used to
place a value here: only its tables are read."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle.level import PAD, Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd import workloads as W  # noqa: E402
from tests.gpuhelp import cf_level, gap_level, make_hier, tiled_level, unit_level  # noqa: E402


def check_level(H, L, lev, op, bottom_cells=0):
    info = H.level_info(L)
    depths = lev.hierarchy(bottom_cells)
    assert info.depths == len(depths)
    assert info.nboxes == len(lev.boxes)
    assert info.ncells == lev.ncells
    assert info.ncomp == lev.ncomp
    sing = set(lev.singular_components(op))
    assert info.nsingular == len(sing)
    for k, dl in enumerate(depths):
        got = [(b["lo"], b["hi"]) for b in H.boxes(L, k)]
        assert got == dl.boxes, k
    # components: one label per box, and a one-to-one map library -> oracle
    fwd, bwd = {}, {}
    for b in H.boxes(L, 0):
        sl = tuple(slice(PAD + l, PAD + h + 1) for l, h in zip(b["lo"], b["hi"]))
        labs = np.unique(lev.labels[sl])
        assert len(labs) == 1
        o = int(labs[0])
        assert fwd.setdefault(b["comp"], o) == o
        assert bwd.setdefault(o, b["comp"]) == b["comp"]
        assert bool(b["singular"]) == (o in sing)
    assert len(fwd) == lev.ncomp


LAYOUTS = {
    "one_box_2d": lambda: (unit_level(64, 2, "N"), "poisson"),
    "one_box_3d": lambda: (unit_level(32, 3, "D"), "helmholtz"),
    "tiled_2d": lambda: (tiled_level(32, 2, "N"), "poisson"),
    "tiled_3d": lambda: (tiled_level(32, 3, "N"), "poisson"),
    "cf_two_components": lambda: (cf_level("N", "N"), "poisson"),
    "cf_dirichlet": lambda: (cf_level("D", "N"), "poisson"),
    "gaps": lambda: (gap_level("D"), "helmholtz"),
}


@pytest.mark.parametrize("name", sorted(LAYOUTS))
def test_box_tables_match_the_oracle(name):
    lev, op = LAYOUTS[name]()
    c = 1e-3 if op == "helmholtz" else 0.0
    H, L = make_hier(lev, op, c)
    check_level(H, L, lev, op)


@pytest.mark.parametrize("bottom", [64, 256])
def test_box_tables_with_a_bottom_size(bottom):
    lev = tiled_level(32, 2, "N")
    H, L = make_hier(lev, "poisson", 0.0, bottom_cells=bottom)
    check_level(H, L, lev, "poisson", bottom)


def _multi(boxes, base, cf_modes, bc, op):
    H = A.Hierarchy(2, (base, base), 1.0 / base, len(boxes))
    for l, bl in enumerate(boxes):
        H.set_level_boxes(l, bl)
        if l:
            H.set_cf_mode(l, cf_modes)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.NEUMANN if bc == "N" else A.DIRICHLET)
    H.set_operator(A.POISSON if op == "poisson" else A.HELMHOLTZ, 0.0 if op == "poisson" else 1e-3)
    H.finalize()
    return H


@pytest.mark.parametrize("cf", ["N", "I"])
def test_two_level_disk_layout(cf):
    boxes = W.amr_two_level_boxes()
    H = _multi(boxes, 256, A.CF_NEUMANN if cf == "N" else A.CF_INTERP, "N", "poisson")
    phys = {(d, s): "N" for d in range(2) for s in (0, 1)}
    for l, bl in enumerate(boxes):
        n = 256 * 2 ** l
        lev = Level((n, n), 1.0 / n, bl, phys, cf if l else "D")
        check_level(H, l, lev, "poisson")
    assert H.level_info(1).ncomp == 2 and H.level_info(1).nboxes == 56


def test_three_level_vortex_layout():
    boxes, _ = W.three_level_vortex_boxes(0)
    H = _multi(boxes, 512, A.CF_INTERP, "D", "helmholtz")
    phys = {(d, s): "D" for d in range(2) for s in (0, 1)}
    for l, bl in enumerate(boxes):
        n = 512 * 2 ** l
        lev = Level((n, n), 1.0 / n, bl, phys, "I" if l else "D")
        check_level(H, l, lev, "helmholtz")


def test_isolated_boxes_each_coarsen_on_their_own():
    """A batch of isolated boxes: each box is its own domain (its corners are
    reported in its own index space, from 0) and coarsens on its own; at
    depth k the table lists, in the caller's order, the boxes whose own
    hierarchy reaches k."""
    sides = W.batched_boxes(48, seed=3)
    H = A.Hierarchy(2, (256, 256), 1.0 / 256, 1)
    boxes, x = [], 0
    for s in sides:
        boxes.append(((x, 0), (x + s - 1, s - 1)))
        x += s + 8
    H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    H.set_operator(A.HELMHOLTZ, 1e-3)
    H.finalize()
    info = H.level_info(0)
    assert info.ncomp == len(sides) and info.nboxes == len(sides)
    phys = {(d, e): "D" for d in range(2) for e in (0, 1)}
    own = [Level((s, s), 1.0 / 256, [((0, 0), (s - 1, s - 1))], phys).hierarchy() for s in sides]
    assert info.depths == max(len(o) for o in own)
    for k in range(info.depths):
        want = [o[k].boxes[0] for o in own if len(o) > k]
        got = [(b["lo"], b["hi"]) for b in H.boxes(0, k)]
        assert got == want, k
    assert len({b["comp"] for b in H.boxes(0, 0)}) == len(sides)
