"""Periodic boundaries (the domains of Section 7.3) on the GPU against the
oracle: gradient, divergence and the approximate projection on periodic
levels (wrap within one box, between boxes, periodic in one direction
only); composite solves and the composite projection over a periodic base
level with a refined patch inside; and at 256^2 the mixed-precision solves
of the periodic Poisson and Helmholtz systems against their exact solutions
by FFT division with the Laplacian's symbol (the closed form pinned in the
oracle's periodic tests).  Level solves, smoothers, V-cycles and adjoints on
periodic layouts are covered with every other layout by the parity and
adjoint tests."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import amr, proj  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import (PERIODIC_X_BC, faces_to_dev, from_dev, make_hier, random_faces,  # noqa: E402
                           random_field, relerr, tiled_level, to_dev, unit_level)

TOL64 = 1e-11

LAYOUTS = {
    "2d": lambda: unit_level(32, 2, "P"),
    "2d_tiled": lambda: tiled_level(32, 2, "P"),
    "2d_x_only": lambda: unit_level(32, 2, PERIODIC_X_BC),
    "3d_tiled": lambda: tiled_level(16, 3, "P"),
}


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_gradient_divergence_projection(name):
    lev = LAYOUTS[name]()
    lw, lp = proj.velocity_level(lev), proj.pressure_level(lev)
    Hw, L = make_hier(lw, "poisson", 0.0)
    Hp, _ = make_hier(lp, "poisson", 0.0)
    D = lev.dim
    phi = random_field(lp, 1)
    fdp = random_faces(lp, 2)
    ph = to_dev(Hp, L, 0, phi)
    gs = [torch.zeros_like(ph) for _ in range(D)]
    Hp.gradient([ph], [gs], [faces_to_dev(Hp, L, lp, fdp)], lev_lo=L)
    W = [random_field(lw, 3 + d) for d in range(D)]
    wb = [random_faces(lw, 7 + d) for d in range(D)]
    ws = [to_dev(Hw, L, 0, w) for w in W]
    div = torch.zeros_like(ws[0])
    Hw.divergence([ws], [div], [[faces_to_dev(Hw, L, lw, f) for f in wb]], lev_lo=L)
    torch.cuda.synchronize()
    want = proj.gradient(lp, phi, fdp)
    for d in range(D):
        assert relerr(from_dev(Hp, L, 0, gs[d], lp), want[d], lp.mask) < TOL64
    assert relerr(from_dev(Hw, L, 0, div, lw), proj.divergence(lw, W, wb), lw.mask) < TOL64
    U_o, phi_o, st_o = proj.project(lev, W, wb, tol_rel=1e-12, smoother="rb")
    assert st_o["converged"]
    for prec, tol in ((A.FP64, 1e-10), (A.MIXED, 1e-9)):
        ws = [to_dev(Hw, L, 0, w) for w in W]
        us = [torch.zeros_like(ws[0]) for _ in W]
        phd = torch.zeros_like(ws[0])
        st = A.project(Hw, Hp, [ws], [phd], [us], [[faces_to_dev(Hw, L, lw, f) for f in wb]],
                       A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        for d in range(D):
            assert relerr(from_dev(Hw, L, 0, us[d], lev), U_o[d], lev.mask) < tol, (prec, d)


BASE = ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((8, 8), (19, 23)), ((20, 8), (23, 15))]])


def gpu_hier(kind, op, c):
    base, h0, boxes = BASE
    H = A.Hierarchy(2, base, h0, len(boxes))
    for l, bl in enumerate(boxes):
        H.set_level_boxes(l, bl)
        if l:
            H.set_cf_mode(l, A.CF_INTERP)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.PERIODIC if kind == "P" else (A.DIRICHLET if kind == "D" else A.NEUMANN))
    H.set_operator(A.POISSON if op == "poisson" else A.HELMHOLTZ, c)
    H.finalize()
    return H


def rand_levels(OH, seed):
    rng = np.random.default_rng(seed)
    return [np.where(lev.mask, rng.normal(size=lev.pshape), 0.0) for lev in OH.levels]


def relmax(G, O, masks):
    num = max(np.abs(G[l] - O[l])[masks[l]].max() for l in range(len(G)))
    den = max(np.abs(O[l])[masks[l]].max() for l in range(len(G)))
    return num / den


@pytest.mark.parametrize("op,c", [("helmholtz", 0.01), ("poisson", 0.0)])
def test_composite_solve_on_a_periodic_base(op, c):
    base, h0, boxes = BASE
    OH = amr.Hierarchy(base, h0, boxes, {(d, s): "P" for d in range(2) for s in (0, 1)})
    H = gpu_hier("P", op, c)
    f = rand_levels(OH, 5)
    U_o, st_o = amr.composite_solve(OH, f, op, c, tol_rel=1e-12, max_cycles=200)
    assert st_o["converged"]
    if OH.singular(op):
        m = OH.composite_mean(U_o)
        U_o = [np.where(lev.mask, U_o[l] - m, 0.0) for l, lev in enumerate(OH.levels)]
    for prec, tol in ((A.FP64, 1e-10), (A.MIXED, 1e-9)):
        fs = [to_dev(H, l, 0, f[l]) for l in range(OH.nlev)]
        xs = [torch.zeros_like(t) for t in fs]
        st = H.solve_composite(xs, fs, None, A.default_opts(precision=prec, tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        got = [from_dev(H, l, 0, xs[l], OH.levels[l]) for l in range(OH.nlev)]
        if OH.singular(op):
            m = OH.composite_mean(got)
            got = [np.where(lev.mask, got[l] - m, 0.0) for l, lev in enumerate(OH.levels)]
        assert relmax(got, U_o, OH.valid) < tol, prec


def test_composite_projection_on_a_periodic_base():
    base, h0, boxes = BASE
    H_o = amr.Hierarchy(base, h0, boxes, {(d, s): "P" for d in range(2) for s in (0, 1)})
    Hw_o = proj.hierarchy_with(H_o, "D")
    Hp, Hw = gpu_hier("P", "poisson", 0.0), gpu_hier("P", "poisson", 0.0)
    nl = len(boxes)
    W = [rand_levels(Hw_o, 31 + d) for d in range(2)]
    U_o, _, st_o = proj.composite_project(H_o, W, None, tol_rel=1e-12, smoother="rb")
    assert st_o["converged"]
    for prec, tol in ((A.FP64, 1e-10), (A.MIXED, 1e-9)):
        ws = [[to_dev(Hw, l, 0, W[d][l]) for d in range(2)] for l in range(nl)]
        us = [[torch.zeros_like(ws[l][0]) for _ in range(2)] for l in range(nl)]
        phis = [torch.zeros_like(ws[l][0]) for l in range(nl)]
        st = A.project(Hw, Hp, ws, phis, us, None,
                       A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        for d in range(2):
            got = [from_dev(Hw, l, 0, us[l][d], Hw_o.levels[l]) for l in range(nl)]
            assert relmax(got, U_o[d], H_o.valid) < tol, (prec, d)


def fft_solution(f, h, op, c):
    """Exact solution of the periodic system on an n^2 grid: division of
    the Fourier coefficients by the symbol of (I - c L) or L (zero mode
    dropped for L)."""
    th = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) for n in f.shape], indexing="ij")
    lam = sum((32 * np.cos(t) - 2 * np.cos(2 * t) - 30) / (12 * h * h) for t in th)
    fh = np.fft.fftn(f)
    if op == "poisson":
        lam.flat[0] = 1.0
        uh = fh / lam
        uh.flat[0] = 0.0
    else:
        uh = fh / (1.0 - c * lam)
    return np.real(np.fft.ifftn(uh))


@pytest.mark.parametrize("op", ["poisson", "helmholtz"])
@pytest.mark.parametrize("tiled", [False, True])
def test_solves_at_256_equal_fft_solutions(op, tiled):
    n = 256
    lev = tiled_level(n, 2, "P") if tiled else unit_level(n, 2, "P")
    c = 0.0 if op == "poisson" else 0.5e-3 / n
    rng = np.random.default_rng(9)
    x = (np.arange(n) + 0.5) / n
    f = lev.zeros()
    f[lev.inner] = np.sin(2 * np.pi * x)[:, None] * np.cos(4 * np.pi * x)[None, :] + 1e-3 * rng.normal(size=(n, n))
    if op == "poisson":
        f[lev.inner] -= f[lev.inner].mean()
    want = fft_solution(f[lev.inner], lev.h, op, c)
    H, L = make_hier(lev, op, c)
    fd = to_dev(H, L, 0, f)
    for prec, tol in ((A.FP64, 1e-10), (A.MIXED, 1e-9)):
        xd = torch.zeros_like(fd)
        st = H.solve(L, xd, fd, None, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                       max_cycles=100))
        assert st["status"] == 0 and st["converged"], st
        got = from_dev(H, L, 0, xd, lev)[lev.inner]
        if op == "poisson":
            got = got - got.mean()
        assert np.abs(got - want).max() < tol * np.abs(want).max(), (prec, st["cycles"])
