"""Adjoint of the level system on the GPU against the oracle: the transposed
operator element by element on every kind of ghost, one adjoint V-cycle
(Jacobi and red-black), whole adjoint solves in FP64 (same residual history)
and mixed precision, the Laplacian and dot product behind dJ/dc, the
autograd binding against the oracle's gradients and against finite
differences of GPU solves, batched isolated boxes, and a coefficient change
on a finalized hierarchy.  Layouts include periodic ones (the transposed
wrapped exchange)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd.autograd import level_solve  # noqa: E402
from tests.gpuhelp import (MIXED_BC, PERIODIC_X_BC, cf_level, faces_to_dev, from_dev, gap_level, make_hier,  # noqa: E402
                           random_faces, random_field, relerr, tiled_level, to_dev, unit_level)

TOL64 = 1e-11

LAYOUTS = {
    "2d_dir": lambda: unit_level(32, 2, "D"),
    "2d_neu": lambda: unit_level(32, 2, "N"),
    "2d_mixed": lambda: unit_level(32, 2, MIXED_BC),
    "2d_small": lambda: unit_level(8, 2, "D"),          # 8^2: boxes 4 wide one depth down
    "2d_tiled": lambda: tiled_level(32, 2, "N"),
    "2d_cf_dir": lambda: cf_level("D", "N"),
    "2d_cf_neu": lambda: cf_level("N", "D"),
    "2d_gap": lambda: gap_level("N"),
    "2d_ragged": lambda: Level((40, 24), 1 / 40, [((0, 0), (39, 23))],
                               {(d, s): "D" for d in range(2) for s in (0, 1)}),
    "3d_dir": lambda: unit_level(16, 3, "D"),
    "3d_neu_tiled": lambda: tiled_level(16, 3, "N"),
    "3d_mixed": lambda: Level((16, 16, 16), 1 / 16, [((0, 0, 0), (15, 15, 15))],
                              {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D", (2, 0): "N", (2, 1): "D"}),
    "2d_periodic_tiled": lambda: tiled_level(32, 2, "P"),
    "2d_periodic_x": lambda: unit_level(32, 2, PERIODIC_X_BC),
}
OPS = [("helmholtz", 0.37), ("poisson", 0.0)]


def _c(op, c, lev):
    return c * lev.h if op == "helmholtz" else 0.0


@pytest.mark.parametrize("name", list(LAYOUTS))
@pytest.mark.parametrize("op,c0", OPS)
def test_apply_transpose(name, op, c0):
    lev = LAYOUTS[name]()
    c = _c(op, c0, lev)
    H, L = make_hier(lev, op, c)
    lam = random_field(lev, 3)
    x = to_dev(H, L, 0, lam)
    y = torch.zeros_like(x)
    H.apply_transpose(L, x, y)
    torch.cuda.synchronize()
    assert relerr(from_dev(H, L, 0, y, lev), lev.apply_T(lam, op, c), lev.mask) < TOL64


@pytest.mark.parametrize("name", ["2d_dir", "2d_neu", "2d_mixed", "2d_small", "2d_cf_neu", "2d_gap", "3d_dir",
                                  "3d_mixed", "2d_periodic_tiled", "2d_periodic_x"])
@pytest.mark.parametrize("op,c0", OPS)
@pytest.mark.parametrize("smoother", ["jacobi", "rb"])
def test_adjoint_vcycle(name, op, c0, smoother):
    lev = LAYOUTS[name]()
    c = _c(op, c0, lev)
    H, L = make_hier(lev, op, c)
    M = mg.MG(lev, op, c, smoother=smoother, transpose=True)
    g = lev.comp_mean(random_field(lev, 4), M.sing[0])
    gd = to_dev(H, L, 0, g)
    e = torch.zeros_like(gd)
    sm = A.SMOOTH_JACOBI if smoother == "jacobi" else A.SMOOTH_RB
    H.vcycle_adjoint(L, gd, e, A.default_opts(smoother=sm))
    torch.cuda.synchronize()
    assert relerr(from_dev(H, L, 0, e, lev), M.vcycle(g), lev.mask) < TOL64


@pytest.mark.parametrize("name", ["2d_dir", "2d_neu", "2d_mixed", "2d_tiled", "2d_cf_dir", "2d_cf_neu", "2d_gap",
                                  "2d_ragged", "3d_dir", "3d_neu_tiled", "2d_periodic_tiled", "2d_periodic_x"])
@pytest.mark.parametrize("op,c0", OPS)
def test_adjoint_solve(name, op, c0):
    lev = LAYOUTS[name]()
    c = _c(op, c0, lev)
    H, L = make_hier(lev, op, c)
    g = random_field(lev, 5)
    lam_or, st_or = mg.solve(lev, g, op, c, tol_rel=1e-12, max_cycles=200, smoother="rb", transpose=True)
    assert st_or["converged"]
    gd = to_dev(H, L, 0, g)
    for prec, tol in ((A.FP64, TOL64), (A.MIXED, 1e-9)):
        lam = torch.zeros_like(gd)
        st = H.solve_adjoint(L, lam, gd, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                        max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        got = from_dev(H, L, 0, lam, lev)
        assert relerr(got, lam_or, lev.mask) < tol, (prec, st["cycles"], st_or["cycles"])
        if prec == A.FP64:
            hist, ho = np.array(st["history"]), np.array(st_or["history"])
            assert abs(len(hist) - len(ho)) <= 1
            k = min(len(hist), len(ho))
            assert np.allclose(hist[:k], ho[:k], rtol=1e-5, atol=1e-14 * ho[0])
        # face ghost cells come back zero (lam is the gradient in the packed layout)
        for a in H.unpack(L, 0, lam.cpu().numpy(), ghosts=True):
            inner = tuple(slice(2, -2) for _ in range(lev.dim))
            m = np.ones(a.shape, dtype=bool)
            m[inner] = False
            assert np.all(a[m] == 0.0)


@pytest.mark.parametrize("name", ["2d_mixed", "2d_cf_neu", "3d_dir"])
def test_laplacian_and_dot(name):
    lev = LAYOUTS[name]()
    H, L = make_hier(lev, "helmholtz", 0.3 * lev.h)
    u, v = random_field(lev, 6), random_field(lev, 7)
    fd = random_faces(lev, 8)
    ud, vd = to_dev(H, L, 0, u), to_dev(H, L, 0, v)
    y = torch.zeros_like(ud)
    H.apply_laplacian(L, ud, y, faces_to_dev(H, L, lev, fd))
    want = lev.laplacian(u, lev.ghosts(u, fd))
    assert relerr(from_dev(H, L, 0, y, lev), want, lev.mask) < TOL64
    d = H.dot(L, ud, vd)
    want = float((u[lev.mask] * v[lev.mask]).sum())
    assert abs(d - want) < 1e-13 * np.abs(u[lev.mask] * v[lev.mask]).sum()
    assert H.dot(L, ud, vd) == d  # fixed summation order


@pytest.mark.parametrize("name", ["2d_dir", "2d_cf_neu", "3d_mixed"])
def test_autograd_against_oracle(name):
    lev = LAYOUTS[name]()
    c = 0.4 * lev.h
    H, L = make_hier(lev, "helmholtz", c)
    f, t = random_field(lev, 9), random_field(lev, 10)
    fd = random_faces(lev, 11)
    fdd = faces_to_dev(H, L, lev, fd)
    fdev = to_dev(H, L, 0, f).requires_grad_(True)
    cdev = torch.tensor(c, dtype=torch.float64, requires_grad=True)
    tdev = to_dev(H, L, 0, t)
    mask = to_dev(H, L, 0, lev.mask.astype(float))
    opts = A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-13, max_cycles=200)
    x = level_solve(fdev, cdev, H, L, fdd, opts)
    J = 0.5 * (((x - tdev) * mask) ** 2).sum()
    J.backward()
    # oracle gradients
    u, _ = mg.solve(lev, f, "helmholtz", c, fd, tol_rel=1e-13, max_cycles=200)
    lam, _ = mg.solve(lev, u - t, "helmholtz", c, tol_rel=1e-13, max_cycles=200, transpose=True)
    gc = mg.grad_c(lev, lam, u, fd)
    assert relerr(from_dev(H, L, 0, fdev.grad, lev), lam, lev.mask) < 1e-9
    assert abs(cdev.grad.item() - gc) < 1e-8 * abs(gc)


def test_backward_uses_the_coefficient_of_its_forward():
    # two forward solves at different c on one hierarchy, then the backward of
    # the first: its gradients are the oracle's at the first c, and the
    # hierarchy keeps the coefficient it had before the backward
    lev = unit_level(32, 2, "D")
    c1, c2 = 0.3 * lev.h, 0.8 * lev.h
    H, L = make_hier(lev, "helmholtz", c1)
    f, t = random_field(lev, 21), random_field(lev, 22)
    fdev, tdev = to_dev(H, L, 0, f).requires_grad_(True), to_dev(H, L, 0, t)
    mask = to_dev(H, L, 0, lev.mask.astype(float))
    opts = A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-13, max_cycles=200)
    cdev = torch.tensor(c1, dtype=torch.float64, requires_grad=True)
    x1 = level_solve(fdev, cdev, H, L, None, opts)
    x2 = level_solve(fdev.detach(), c2, H, L, None, opts)
    assert H.c == c2
    J = 0.5 * (((x1 - tdev) * mask) ** 2).sum()
    J.backward()
    assert H.c == c2
    u, _ = mg.solve(lev, f, "helmholtz", c1, tol_rel=1e-13, max_cycles=200)
    lam, _ = mg.solve(lev, u - t, "helmholtz", c1, tol_rel=1e-13, max_cycles=200, transpose=True)
    assert relerr(from_dev(H, L, 0, fdev.grad, lev), lam, lev.mask) < 1e-9
    gc = mg.grad_c(lev, lam, u)
    assert abs(cdev.grad.item() - gc) < 1e-8 * abs(gc)
    del x2


def test_autograd_finite_differences_and_nu_chain():
    # dJ/dnu through c = gamma nu k by autograd, against central differences
    # of GPU solves (step 1e-6 relative); the hierarchy's coefficient is
    # changed in place between the solves
    lev = unit_level(32, 2, MIXED_BC)
    gamma, k = 0.5, lev.h
    nu0 = 1e-1
    H, L = make_hier(lev, "helmholtz", gamma * nu0 * k)
    f, t = random_field(lev, 12), random_field(lev, 13)
    fd = random_faces(lev, 14)
    fdd, fdev, tdev = faces_to_dev(H, L, lev, fd), to_dev(H, L, 0, f), to_dev(H, L, 0, t)
    mask = to_dev(H, L, 0, lev.mask.astype(float))
    opts = A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-14, max_cycles=300)

    def J(nu):
        x = level_solve(fdev, gamma * nu * k, H, L, fdd, opts)
        return 0.5 * (((x - tdev) * mask) ** 2).sum()

    nu = torch.tensor(nu0, dtype=torch.float64, requires_grad=True)
    J(nu).backward()
    eps = 1e-6 * nu0
    with torch.no_grad():
        fdiff = (J(torch.tensor(nu0 + eps, dtype=torch.float64)).item()
                 - J(torch.tensor(nu0 - eps, dtype=torch.float64)).item()) / (2 * eps)
    assert abs(nu.grad.item() - fdiff) < 1e-5 * abs(fdiff)


def test_set_coefficient_matches_fresh_hierarchy():
    lev = unit_level(32, 2, "D")
    c1, c2 = 0.3 * lev.h, 0.7 * lev.h
    H1, L = make_hier(lev, "helmholtz", c1)
    H1.set_coefficient(c2)
    H2, _ = make_hier(lev, "helmholtz", c2)
    f = to_dev(H1, L, 0, random_field(lev, 15))
    x1, x2 = torch.zeros_like(f), torch.zeros_like(f)
    s1 = H1.solve(L, x1, f, None, A.default_opts(precision=A.FP64, tol_rel=1e-12))
    s2 = H2.solve(L, x2, f, None, A.default_opts(precision=A.FP64, tol_rel=1e-12))
    assert s1["history"] == s2["history"]
    assert torch.equal(x1, x2)


def test_batched_isolated_adjoint():
    # independent boxes of several sizes in one hierarchy: each box's adjoint
    # solution equals the oracle's adjoint solve of that box alone
    sides = [16, 24, 40, 32, 16]
    h = 1.0 / 64
    c = 0.5 * 1e-3 * h
    H = A.Hierarchy(2, (256, 64), h, 1)
    boxes, x0 = [], 0
    for s in sides:
        boxes.append(((x0, 0), (x0 + s - 1, s - 1)))
        x0 += s
    H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    for d in range(2):
        for sd in (0, 1):
            H.set_physical_bc(d, sd, A.DIRICHLET)
    H.set_operator(A.HELMHOLTZ, c)
    H.finalize()
    rng = np.random.default_rng(16)
    gs = [rng.normal(size=(s, s)) for s in sides]
    gd = torch.tensor(H.pack(0, 0, lambda i, b: gs[i]), device="cuda")
    lam = torch.zeros_like(gd)
    st = H.solve_adjoint(0, lam, gd, A.default_opts(precision=A.FP64, tol_rel=1e-12, max_cycles=200))
    assert st["converged"]
    got = H.unpack(0, 0, lam.cpu().numpy())
    for i, s in enumerate(sides):
        lev = Level((s, s), h, [((0, 0), (s - 1, s - 1))], {(d, sd): "D" for d in range(2) for sd in (0, 1)})
        g = lev.zeros()
        g[lev.inner] = gs[i]
        want, _ = mg.solve(lev, g, "helmholtz", c, tol_rel=1e-13, max_cycles=200, transpose=True)
        err = np.abs(got[i] - want[lev.inner]).max() / np.abs(want).max()
        assert err < 1e-10, (i, s, err)
