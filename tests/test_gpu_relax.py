"""Parity of the over-relaxed red-black smoother (solve option omega_rb, the
step entry point's omega for red-black) with the oracle: single sweeps in
FP64 and FP32, whole V-cycles forward and adjoint, FP64 and mixed solves (the
FP64 solve takes the oracle's cycles), and the
option's range check."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import (cf_level, from_dev, gap_level, make_hier, random_field, relerr, tiled_level,  # noqa: E402
                           to_dev, unit_level)

TOL64 = 1e-11
W = 1.3
LAYOUTS = {
    "2d_dir": (lambda: unit_level(32, 2, "D"), "helmholtz", 0.37),
    "2d_neu": (lambda: unit_level(32, 2, "N"), "poisson", 0.0),
    "2d_cf_neu": (lambda: cf_level("N", "N"), "poisson", 0.0),
    "2d_gap": (lambda: gap_level("D"), "helmholtz", 0.37),
    "3d_neu_tiled": (lambda: tiled_level(16, 3, "N"), "poisson", 0.0),
    "3d_dir": (lambda: unit_level(16, 3, "D"), "helmholtz", 0.37),
}


def _setup(name):
    mk, op, c0 = LAYOUTS[name]
    lev = mk()
    c = c0 * lev.h if op == "helmholtz" else 0.0
    H, L = make_hier(lev, op, c)
    return lev, op, c, H, L


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_over_relaxed_sweeps(name):
    lev, op, c, H, L = _setup(name)
    e, f = random_field(lev, 1), random_field(lev, 2)
    want = mg.red_black(lev, e, f, op, c, lev.diagonal(op, c), 2, omega=W)
    for dt, tol in ((torch.float64, TOL64), (torch.float32, 2e-5)):
        ed, fdv = to_dev(H, L, 0, e, dt), to_dev(H, L, 0, f, dt)
        H.smooth(L, 0, ed, fdv, torch.zeros_like(ed), A.SMOOTH_RB, 2, W)
        torch.cuda.synchronize()
        assert relerr(from_dev(H, L, 0, ed, lev), want, lev.mask) < tol, str(dt)


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_over_relaxed_vcycles(name):
    lev, op, c, H, L = _setup(name)
    opts = A.default_opts(smoother=A.SMOOTH_RB, omega_rb=W, nu1=1, nu2=3)
    for tr in (False, True):
        M = mg.MG(lev, op, c, nu1=1, nu2=3, smoother="rb", transpose=tr, omega_rb=W)
        g = lev.comp_mean(random_field(lev, 3), M.sing[0])
        gd = to_dev(H, L, 0, g)
        e = torch.zeros_like(gd)
        (H.vcycle_adjoint if tr else H.vcycle)(L, gd, e, opts)
        torch.cuda.synchronize()
        assert relerr(from_dev(H, L, 0, e, lev), M.vcycle(g), lev.mask) < TOL64, tr


@pytest.mark.parametrize("name", ["2d_neu", "2d_cf_neu", "3d_neu_tiled", "3d_dir"])
def test_over_relaxed_solves(name):
    lev, op, c, H, L = _setup(name)
    f = random_field(lev, 4)
    x_or, st = mg.solve(lev, f, op, c, tol_rel=1e-12, max_cycles=200, smoother="rb", nu1=1, nu2=3, omega_rb=W)
    assert st["converged"]
    fdev = to_dev(H, L, 0, f)
    for prec, tol in ((A.FP64, TOL64), (A.MIXED, 1e-9)):
        x = torch.zeros_like(fdev)
        s = H.solve(L, x, fdev, None, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, omega_rb=W, nu1=1, nu2=3,
                                                        tol_rel=1e-12, max_cycles=200))
        assert s["converged"]
        assert relerr(from_dev(H, L, 0, x, lev), x_or, lev.mask) < tol, prec
        if prec == A.FP64:
            assert s["cycles"] == st["cycles"]


def test_relaxation_range_checked():
    lev, op, c, H, L = _setup("2d_dir")
    fdev = to_dev(H, L, 0, random_field(lev, 6))
    x = torch.zeros_like(fdev)
    for w in (0.0, 2.0, -1.0):
        with pytest.raises(A.AmgError):
            H.solve(L, x, fdev, None, A.default_opts(smoother=A.SMOOTH_RB, omega_rb=w))
