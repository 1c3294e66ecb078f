"""Parity of the bottom-size option with the oracle: the exact coarsest
solve taken at the first depth whose components have at most B cells.  The
hierarchy, the bottom solve, whole V-cycles (forward and adjoint, Jacobi and
red-black) and solves match the oracle built with the same B; a B that
covers the level makes one V-cycle the exact solve; batches of isolated
boxes stop per box."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import (from_dev, make_hier, random_field, relerr, tiled_level, to_dev,  # noqa: E402
                           unit_level)

TOL64 = 1e-11

CASES = {
    "2d_dir_B256": (lambda: unit_level(64, 2, "D"), "helmholtz", 0.37, 256),
    "2d_neu_B256": (lambda: unit_level(64, 2, "N"), "poisson", 0.0, 256),
    "2d_tiled_B256": (lambda: tiled_level(32, 2, "N"), "poisson", 0.0, 256),
    "3d_neu_B512": (lambda: unit_level(32, 3, "N"), "poisson", 0.0, 512),
    "3d_dir_B512": (lambda: unit_level(32, 3, "D"), "helmholtz", 0.37, 512),
}


def _setup(name):
    mk, op, c0, B = CASES[name]
    lev = mk()
    c = c0 * lev.h if op == "helmholtz" else 0.0
    H, L = make_hier(lev, op, c, bottom_cells=B)
    return lev, op, c, B, H, L


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_bottom_and_vcycles(name):
    lev, op, c, B, H, L = _setup(name)
    levels = lev.hierarchy(B)
    assert len(levels) < len(lev.hierarchy())
    assert H.level_info(L).depths == len(levels)
    last = len(levels) - 1
    assert H.depth_size(L, last)[0] >= levels[-1].ncells
    for smoother, sm in (("jacobi", A.SMOOTH_JACOBI), ("rb", A.SMOOTH_RB)):
        for tr in (False, True):
            M = mg.MG(lev, op, c, smoother=smoother, transpose=tr, bottom_cells=B)
            assert len(M.levels) == len(levels)
            if not tr:
                bot = M.levels[-1]
                fb = bot.comp_mean(random_field(bot, 3), M.sing[-1])
                fbd = to_dev(H, L, last, fb)
                ebd = torch.zeros(H.depth_size(L, last)[0], dtype=torch.float64, device="cuda")
                H.bottom(L, fbd, ebd)
                torch.cuda.synchronize()
                assert relerr(from_dev(H, L, last, ebd, bot), M.bottom.solve(fb), bot.mask) < TOL64
            g = lev.comp_mean(random_field(lev, 4), M.sing[0])
            gd = to_dev(H, L, 0, g)
            e = torch.zeros_like(gd)
            (H.vcycle_adjoint if tr else H.vcycle)(L, gd, e, A.default_opts(smoother=sm))
            torch.cuda.synchronize()
            assert relerr(from_dev(H, L, 0, e, lev), M.vcycle(g), lev.mask) < TOL64, (smoother, tr)


@pytest.mark.parametrize("name", ["2d_neu_B256", "3d_dir_B512"])
def test_solves_fp64_and_mixed(name):
    lev, op, c, B, H, L = _setup(name)
    f = random_field(lev, 5)
    x_or, st = mg.solve(lev, f, op, c, tol_rel=1e-12, max_cycles=200, smoother="rb", bottom_cells=B)
    assert st["converged"]
    fdev = to_dev(H, L, 0, f)
    for prec, tol in ((A.FP64, TOL64), (A.MIXED, 1e-9)):
        x = torch.zeros_like(fdev)
        s = H.solve(L, x, fdev, None, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                        max_cycles=200))
        assert s["converged"]
        assert relerr(from_dev(H, L, 0, x, lev), x_or, lev.mask) < tol, prec
    # FP64 takes the oracle's cycles exactly
    x = torch.zeros_like(fdev)
    s = H.solve(L, x, fdev, None, A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                    max_cycles=200))
    assert s["cycles"] == st["cycles"]


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("poisson", "N")])
def test_bottom_covering_the_level_is_the_exact_solve(op, bc):
    lev = unit_level(16, 2, bc)
    c = 0.3 * lev.h if op == "helmholtz" else 0.0
    H, L = make_hier(lev, op, c, bottom_cells=256)
    assert H.level_info(L).depths == 1
    M = mg.MG(lev, op, c, bottom_cells=256)
    g = lev.comp_mean(random_field(lev, 6), M.sing[0])
    gd = to_dev(H, L, 0, g)
    e = torch.zeros_like(gd)
    H.vcycle(L, gd, e)
    torch.cuda.synchronize()
    Am, _ = mg.assemble(lev, op, c)
    got = from_dev(H, L, 0, e, lev)[lev.mask]
    if op == "helmholtz":
        want = np.linalg.solve(Am, g[lev.mask])
    else:
        want = np.linalg.lstsq(Am, g[lev.mask], rcond=None)[0]
        want -= want.mean()
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()


def test_isolated_boxes_stop_per_box():
    # isolated boxes of two shapes: 16^3 (bottom at 8^3 = 512 cells, one depth
    # above the layout's own) and 32 x 16 x 16 (1024 cells at depth 1, so it
    # halves once more, to 8 x 4 x 4); the two 16^3 boxes share one inverse
    boxes = [((0, 0, 0), (15, 15, 15)), ((32, 0, 0), (63, 15, 15)), ((0, 32, 0), (15, 47, 15))]
    h = 1 / 64
    H = A.Hierarchy(3, (64, 64, 64), h, 1)
    H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    for d in range(3):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.DIRICHLET)
    c = 0.4 * h
    H.set_operator(A.HELMHOLTZ, c)
    H.set_bottom_cells(512)
    H.finalize()
    sizes = [tuple(u - l + 1 for l, u in zip(lo, hi)) for lo, hi in boxes]
    fs = [np.random.default_rng(i).normal(size=n) for i, n in enumerate(sizes)]
    fdev = torch.tensor(H.pack(0, 0, lambda i, b: fs[i]), device="cuda")
    e = torch.zeros_like(fdev)
    H.vcycle(0, fdev, e, A.default_opts(smoother=A.SMOOTH_RB))
    torch.cuda.synchronize()
    got = H.unpack(0, 0, e.cpu().numpy())
    depths = []
    for i, n in enumerate(sizes):
        lev = Level(n, h, [((0,) * 3, tuple(k - 1 for k in n))], {(d, s): "D" for d in range(3) for s in (0, 1)})
        M = mg.MG(lev, "helmholtz", c, smoother="rb", bottom_cells=512)
        depths.append(len(M.levels))
        f = lev.zeros()
        f[lev.inner] = fs[i]
        want = M.vcycle(f)
        err = np.abs(got[i] - want[lev.inner]).max() / np.abs(want[lev.inner]).max()
        assert err < 1e-11, (i, err)
    assert depths == [2, 3, 2]
    assert H.level_info(0).depths == 3
