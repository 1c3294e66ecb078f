"""Tile tuning: the march length and row alignment change only how the work
is cut into launches, not the result (parity with the oracle for every
setting), and the autotuner picks one of its candidates."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import from_dev, random_field, relerr, to_dev, unit_level  # noqa: E402


def hier(n, dim, bc, op, c, march=None, align=None):
    H = A.Hierarchy(dim, (n,) * dim, 1.0 / n, 1)
    H.set_level_boxes(0, [((0,) * dim, (n - 1,) * dim)])
    for d in range(dim):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.DIRICHLET if bc == "D" else A.NEUMANN)
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
    if march:
        H.set_tuning(A.TUNE_MARCH2 if dim == 2 else A.TUNE_MARCH3, march)
    if align:
        H.set_tuning(A.TUNE_ROW_ALIGN, align)
    H.finalize()
    return H


@pytest.mark.parametrize("dim,n", [(2, 64), (3, 32)])
@pytest.mark.parametrize("march,align", [(2, None), (8, 64), (128, 2), (4096, None)])
def test_result_independent_of_tiling(dim, n, march, align):
    lev = unit_level(n, dim, "N")
    f = random_field(lev, 1)
    x_or, st_or = mg.solve(lev, f, "poisson", 0.0, None, tol_rel=1e-12, max_cycles=200, smoother="rb")
    H = hier(n, dim, "N", "poisson", 0.0, march, align)
    fd = to_dev(H, 0, 0, f)
    for prec, tol in ((A.FP64, 1e-11), (A.MIXED, 1e-9)):
        x = torch.zeros_like(fd)
        st = H.solve(0, x, fd, None, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                    max_cycles=200))
        assert st["converged"]
        sing = lev.singular_components("poisson")
        assert relerr(lev.comp_mean(from_dev(H, 0, 0, x, lev), sing), lev.comp_mean(x_or, sing), lev.mask) < tol


def test_autotune_picks_a_candidate():
    H = A.Hierarchy(3, (64,) * 3, 1 / 64, 1)
    H.set_level_boxes(0, [((0,) * 3, (63,) * 3)])
    H.set_operator(A.HELMHOLTZ, 1e-4)
    best, ms = H.autotune(0, A.F32, A.SMOOTH_RB, nreps=5)
    assert best in (4, 6, 8, 16, 32, 64, 128) and ms > 0
    H.finalize()
    f = torch.ones(H.depth_size(0, 0)[0], dtype=torch.float64, device="cuda")
    x = torch.zeros_like(f)
    assert H.solve(0, x, f)["converged"]
