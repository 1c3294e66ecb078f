"""The paper's bottom solver of the pressure systems (Section 6.5),
ILU(0)-preconditioned GMRES(m), on the GPU against the oracle's
(oracle/mg.py, IluGmresBottom; pinned by ILU(0)'s defining property, the
direct solve at m = n and the minimal-residual property): the bottom solve
alone for m = 1, 3, 5 on bordered (pure-Neumann) and plain systems, several
boxes in one component, several components and 3D; one V-cycle with it;
whole solves in FP64 (the oracle's residual history) and mixed precision;
batched isolated boxes sharing one factorisation; the adjoint solve keeping
the exact transposed inverse."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import cf_level, from_dev, make_hier, random_field, relerr, tiled_level, to_dev, unit_level  # noqa: E402

LAYOUTS = {
    "2d_neumann": (lambda: unit_level(32, 2, "N"), "poisson", 0.0),
    "2d_dirichlet_helmholtz": (lambda: unit_level(32, 2, "D"), "helmholtz", 0.3 / 32),
    "2d_tiled_neumann": (lambda: tiled_level(32, 2, "N"), "poisson", 0.0),
    "2d_cf_two_components": (lambda: cf_level("N", "N"), "poisson", 0.0),
    "3d_neumann": (lambda: unit_level(16, 3, "N"), "poisson", 0.0),
}


@pytest.mark.parametrize("name", sorted(LAYOUTS))
@pytest.mark.parametrize("m", [1, 3, 5])
def test_bottom_solve_against_oracle(name, m):
    make, op, c = LAYOUTS[name]
    lev = make()
    H, L = make_hier(lev, op, c, bottom=(A.BOTTOM_ILU_GMRES, m))
    M = mg.MG(lev, op, c, bottom="ilu_gmres", bottom_iters=m)
    bot = M.levels[-1]
    f = bot.comp_mean(random_field(bot, 7), M.sing[-1])
    last = len(M.levels) - 1
    fd = to_dev(H, L, last, f)
    ed = torch.zeros(H.depth_size(L, last)[0], dtype=torch.float64, device="cuda")
    H.bottom(L, fd, ed)
    torch.cuda.synchronize()
    want = M.bottom.solve(f)
    assert relerr(from_dev(H, L, last, ed, bot), want, bot.mask) < 1e-11


@pytest.mark.parametrize("name", sorted(LAYOUTS))
def test_vcycle_and_solves_against_oracle(name):
    make, op, c = LAYOUTS[name]
    lev = make()
    H, L = make_hier(lev, op, c, bottom=(A.BOTTOM_ILU_GMRES, 5))
    M = mg.MG(lev, op, c, smoother="rb", bottom="ilu_gmres", bottom_iters=5)
    g = lev.comp_mean(random_field(lev, 9), M.sing[0])
    gd = to_dev(H, L, 0, g)
    e = torch.zeros_like(gd)
    H.vcycle(L, gd, e, A.default_opts(smoother=A.SMOOTH_RB))
    torch.cuda.synchronize()
    assert relerr(from_dev(H, L, 0, e, lev), M.vcycle(g), lev.mask) < 1e-11
    f = random_field(lev, 10)
    x_or, st_or = mg.solve(lev, f, op, c, smoother="rb", tol_rel=1e-12, max_cycles=100, mg=M)
    assert st_or["converged"]
    sing = lev.singular_components(op)
    want = lev.comp_mean(x_or, sing)
    fdev = to_dev(H, L, 0, f)
    for prec, tol in ((A.FP64, 1e-11), (A.MIXED, 1e-9)):
        x = torch.zeros_like(fdev)
        st = H.solve(L, x, fdev, None, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                        max_cycles=100))
        torch.cuda.synchronize()
        assert st["status"] == 0 and st["converged"], st
        assert relerr(lev.comp_mean(from_dev(H, L, 0, x, lev), sing), want, lev.mask) < tol, prec
        if prec == A.FP64:
            k = min(len(st["history"]), len(st_or["history"]))
            assert abs(len(st["history"]) - len(st_or["history"])) <= 1
            assert np.allclose(st["history"][:k], st_or["history"][:k], rtol=1e-6, atol=1e-13 * st_or["history"][0])


def test_batched_boxes_share_one_factorisation():
    """Isolated boxes of equal shape share one ILU(0) factorisation and run
    one GMRES per box: each box's solution equals its own oracle solve."""
    boxes = [((0, 0), (15, 15)), ((0, 0), (15, 15)), ((0, 0), (23, 15))]
    H = A.Hierarchy(2, (64, 64), 1 / 64, 1)
    H.set_level_boxes(0, boxes)
    H.set_isolated(0)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.NEUMANN)
    H.set_operator(A.POISSON, 0.0)
    H.set_bottom_solver(A.BOTTOM_ILU_GMRES, 4)
    H.finalize()
    rng = np.random.default_rng(11)
    fs = [rng.normal(size=(hi[0] - lo[0] + 1, hi[1] - lo[1] + 1)) for lo, hi in boxes]
    fs = [f - f.mean() for f in fs]
    fd = torch.tensor(H.pack(0, 0, lambda i, b: fs[i]), device="cuda")
    x = torch.zeros_like(fd)
    st = H.solve(0, x, fd, None, A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                max_cycles=100))
    torch.cuda.synchronize()
    assert st["status"] == 0 and st["converged"], st
    got = H.unpack(0, 0, x.cpu().numpy())
    for i, (lo, hi) in enumerate(boxes):
        n = (hi[0] - lo[0] + 1, hi[1] - lo[1] + 1)
        lev = Level(n, 1 / 64, [((0, 0), (n[0] - 1, n[1] - 1))], {(d, s): "N" for d in range(2) for s in (0, 1)})
        f = lev.zeros()
        f[lev.inner] = fs[i]
        M = mg.MG(lev, "poisson", 0.0, smoother="rb", bottom="ilu_gmres", bottom_iters=4)
        xo, so = mg.solve(lev, f, "poisson", 0.0, smoother="rb", tol_rel=1e-12, max_cycles=100, mg=M)
        want = lev.comp_mean(xo, [0])[lev.inner]
        g = got[i] - got[i].mean()
        assert np.abs(g - want).max() < 1e-10 * np.abs(want).max(), i


def test_adjoint_solve_keeps_the_exact_bottom():
    lev = unit_level(32, 2, "N")
    H, L = make_hier(lev, "poisson", 0.0, bottom=(A.BOTTOM_ILU_GMRES, 5))
    g = random_field(lev, 12)
    lam_or, st_or = mg.solve(lev, g, "poisson", 0.0, tol_rel=1e-12, max_cycles=200, smoother="rb", transpose=True)
    gd = to_dev(H, L, 0, g)
    lam = torch.zeros_like(gd)
    st = H.solve_adjoint(L, lam, gd, A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                    max_cycles=200))
    assert st["status"] == 0 and st["converged"], st
    assert relerr(from_dev(H, L, 0, lam, lev), lam_or, lev.mask) < 1e-11
