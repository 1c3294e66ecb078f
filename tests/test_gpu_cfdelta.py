"""Solvability by the coarse-fine face-data correction (eq.
correctingFaceAvg) on the GPU against the oracle: two singular components
with coarse-fine Neumann faces (no RHS shift), and a component without
coarse-fine faces (RHS shift), FP64 and mixed precision."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import (cf_level, faces_to_dev, from_dev, make_hier, random_faces, random_field,  # noqa: E402
                           relerr, to_dev, unit_level)


@pytest.mark.parametrize("name", ["cf", "full"])
@pytest.mark.parametrize("smoother", ["jacobi", "rb"])
def test_cf_delta_solve(name, smoother):
    lev = cf_level("N", "N") if name == "cf" else unit_level(32, 2, "N")
    H, L = make_hier(lev, "poisson", 0.0)
    f, fd = random_field(lev, 1), random_faces(lev, 2)
    x_or, st_or = mg.solve(lev, f, "poisson", 0.0, fd, tol_rel=1e-12, max_cycles=200, smoother=smoother,
                           cf_delta=True)
    assert st_or["converged"]
    sing = lev.singular_components("poisson")
    fdev, fdd = to_dev(H, L, 0, f), faces_to_dev(H, L, lev, fd)
    sm = A.SMOOTH_JACOBI if smoother == "jacobi" else A.SMOOTH_RB
    for prec, tol in ((A.FP64, 1e-11), (A.MIXED, 1e-9)):
        x = torch.zeros_like(fdev)
        st = H.solve(L, x, fdev, fdd, A.default_opts(precision=prec, smoother=sm, solvability=A.SOLV_CF_DELTA,
                                                     tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        got = lev.comp_mean(from_dev(H, L, 0, x, lev), sing)
        assert relerr(got, lev.comp_mean(x_or, sing), lev.mask) < tol
        assert np.allclose(st["defects"], st_or["defects"], rtol=1e-9, atol=1e-12)
        if prec == A.FP64:
            hist, ho = np.array(st["history"]), np.array(st_or["history"])
            assert abs(len(hist) - len(ho)) <= 1
            k = min(len(hist), len(ho))
            assert np.allclose(hist[:k], ho[:k], rtol=1e-5, atol=1e-14 * ho[0])
    # the caller's face data are not modified
    assert torch.equal(fdd, faces_to_dev(H, L, lev, fd))
