"""The C-ABI library loads and exports every function include/amg.h
declares; host-only calls validate their arguments (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02663_amd", "libamg.so")


def declared():
    text = open(os.path.join(ROOT, "include", "amg.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(amg_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for must in ("amg_create", "amg_finalize", "amg_solve", "amg_apply_operator", "amg_vcycle", "amg_destroy"):
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def _create(L, dim, cells, h=None, lo=None, hi=None, ratio=2, nlevels=1):
    h = 1.0 / cells[0] if h is None else h
    lo = [0.0] * dim if lo is None else lo
    hi = [lo[d] + cells[d] * h for d in range(dim)] if hi is None else hi
    hd = ctypes.c_void_p()
    rc = L.amg_create(dim, (ctypes.c_double * dim)(*lo), (ctypes.c_double * dim)(*hi),
                      (ctypes.c_int32 * dim)(*cells), ratio, nlevels, ctypes.byref(hd))
    return rc, hd


def test_host_argument_checks(lib):
    from paper_2506_02663_amd import amg as A
    L = A.lib()
    assert _create(L, 4, [16] * 4)[0] == A.EINVAL                          # bad dim
    assert _create(L, 2, [16, 16], ratio=3)[0] == A.EINVAL                 # ratio
    assert _create(L, 2, [16, 16], h=-1.0)[0] == A.EINVAL                  # empty extent
    assert _create(L, 2, [16, 16], hi=[1.0, 0.5])[0] == A.EINVAL           # cells not cubes
    assert _create(L, 2, [2, 16], hi=[0.125, 1.0])[0] == A.EINVAL           # fewer than 4 cells
    assert _create(L, 2, [16, 16], nlevels=17)[0] == A.EINVAL
    rc, h = _create(L, 2, [16, 32], lo=[-1.0, 2.0], hi=[-0.5, 3.0])        # h = 1/32, origin off 0
    assert rc == A.OK
    assert L.amg_destroy(h) == A.OK
    rc, h = _create(L, 2, [16, 16])
    assert rc == A.OK
    assert L.amg_set_operator(h, A.HELMHOLTZ, -1.0) == A.EINVAL
    assert b"c > 0" in L.amg_last_error(h)
    assert L.amg_set_physical_bc(h, 2, 0, A.DIRICHLET) == A.EINVAL          # d >= dim
    assert L.amg_set_cf_mode(h, 0, A.CF_NEUMANN) == A.EINVAL                 # level 0 has no interface
    assert L.amg_set_bottom_cells(h, -1) == A.EINVAL
    assert L.amg_set_bottom_cells(h, 1025) == A.EINVAL                      # host inverse O(n^3)
    assert L.amg_set_bottom_cells(h, 512) == A.OK
    assert L.amg_set_bottom_solver(h, 2, 5) == A.EINVAL                      # no such bottom solver
    assert L.amg_set_bottom_solver(h, A.BOTTOM_ILU_GMRES, 0) == A.EINVAL      # GMRES steps 1..16
    assert L.amg_set_bottom_solver(h, A.BOTTOM_ILU_GMRES, 17) == A.EINVAL
    assert L.amg_set_bottom_solver(h, A.BOTTOM_ILU_GMRES, 5) == A.OK
    assert L.amg_set_tuning(h, 3, 2) == A.EINVAL                            # split switch is 0 or 1
    assert L.amg_set_tuning(h, 4, 2) == A.EINVAL                            # tail switch is 0 or 1
    assert L.amg_set_tuning(h, 4, 0) == A.OK
    assert L.amg_set_tuning(h, 5, 0) == A.EINVAL                            # no such key
    assert L.amg_solve(h, 0, 0, None, None, None, None, None, None) == A.EINVAL  # not finalized
    assert b"finalize" in L.amg_last_error(h)
    assert L.amg_destroy(h) == A.OK


# ---- layout rejection: amg_finalize validates on the host before it touches
# the device, so these run without a GPU.  Section 5.1: boxes are disjoint
# (eq. AMRHier), a finer level's boxes are unions of refined coarse cells
# (proper refinement, corners multiples of the ratio) and lie inside the
# level below (proper nesting, eq. validRegion); the fills read four cells of
# a row (eqs. velBCHomoDiri5th, Neumann5), so boxes have at least 4 cells per
# side; the interpolation window of the AMRCFI must lie on the coarse level.

def _layout(L, dim, n, levels, cf=None, bc=0, ratio=2):
    from paper_2506_02663_amd import amg as A
    rc, h = _create(L, dim, [n] * dim, nlevels=len(levels), ratio=ratio)
    assert rc == A.OK
    for d in range(dim):
        for s in (0, 1):
            assert L.amg_set_physical_bc(h, d, s, bc) == A.OK
    assert L.amg_set_operator(h, A.POISSON, 0.0) == A.OK
    for l, boxes in enumerate(levels):
        k = len(boxes)
        lo = (ctypes.c_int32 * (k * dim))(*[v for b in boxes for v in b[0]])
        hi = (ctypes.c_int32 * (k * dim))(*[v for b in boxes for v in b[1]])
        assert L.amg_set_level_boxes(h, l, k, lo, hi) == A.OK
        if l > 0 and cf is not None:
            assert L.amg_set_cf_mode(h, l, cf) == A.OK
    return h


def _finalize_code(L, h):
    rc = L.amg_finalize(h)
    msg = L.amg_last_error(h).decode()
    L.amg_destroy(h)
    return rc, msg


@pytest.mark.parametrize("case,want,text", [
    ("overlap", "ELAYOUT", "overlap"),
    ("gap_in_level0", "ELAYOUT", "cover"),
    ("outside_grid", "ELAYOUT", "leaves the grid"),
    ("side_below_4", "ELAYOUT", "< 4 cells"),
    ("unaligned_fine", "ELAYOUT", "not properly refined"),
    ("not_nested", "ELAYOUT", "not nested"),
    ("cfi_window_off_coarse", "EUNSUPPORTED", "interpolation window"),
    ("empty_level", "ELAYOUT", "no boxes"),
    ("periodic_one_side", "EINVAL", "periodic on one side only"),
    ("periodic_fine_touches_side", "EUNSUPPORTED", "touches the periodic side"),
    ("periodic_isolated", "EUNSUPPORTED", "isolated boxes with periodic"),
    ("unaligned_ratio4", "ELAYOUT", "not properly refined"),
    ("not_nested_ratio4", "ELAYOUT", "not nested"),
])
def test_layout_rejected_before_any_device_call(lib, case, want, text):
    from paper_2506_02663_amd import amg as A
    L = A.lib()
    full = [((0, 0), (31, 31))]
    if case == "overlap":
        h = _layout(L, 2, 32, [[((0, 0), (15, 31)), ((12, 0), (31, 31))]])
    elif case == "gap_in_level0":
        h = _layout(L, 2, 32, [[((0, 0), (15, 31)), ((20, 0), (31, 31))]])
    elif case == "outside_grid":
        h = _layout(L, 2, 32, [[((0, 0), (31, 35))]])
    elif case == "side_below_4":
        h = _layout(L, 2, 32, [full, [((8, 8), (10, 23))]])
    elif case == "unaligned_fine":
        h = _layout(L, 2, 32, [full, [((9, 8), (24, 23))]])
    elif case == "not_nested":
        # level 1 inside level 0's grid, level 2 reaching beyond level 1
        h = _layout(L, 2, 32, [full, [((16, 16), (31, 31))], [((24, 24), (71, 71))]])
    elif case == "cfi_window_off_coarse":
        # level 2 one coarse cell from the edge of level 1: the 5-cell
        # interpolation window of its ghosts leaves level 1
        h = _layout(L, 2, 32, [full, [((16, 16), (47, 47))], [((34, 34), (61, 61))]], cf=A.CF_INTERP)
    elif case == "empty_level":
        h = _layout(L, 2, 32, [full, []])
    elif case == "periodic_one_side":
        h = _layout(L, 2, 32, [full])
        assert L.amg_set_physical_bc(h, 1, 0, A.PERIODIC) == A.OK
    elif case == "periodic_fine_touches_side":
        h = _layout(L, 2, 32, [full, [((0, 16), (15, 31))]], bc=A.PERIODIC)
    elif case == "unaligned_ratio4":  # corners multiples of 2, not of 4
        h = _layout(L, 2, 32, [full, [((18, 16), (41, 47))]], ratio=4)
    elif case == "not_nested_ratio4":  # level 2 reaching beyond level 1 (ratio 4)
        h = _layout(L, 2, 16, [[((0, 0), (15, 15))], [((16, 16), (31, 31))], [((64, 64), (159, 159))]], ratio=4)
    elif case == "periodic_isolated":
        h = _layout(L, 2, 32, [full], bc=A.PERIODIC)
        assert L.amg_set_isolated_boxes(h, 0, 1) == A.OK
    rc, msg = _finalize_code(L, h)
    assert rc == getattr(A, want), (case, rc, msg)
    assert text in msg, (case, msg)
