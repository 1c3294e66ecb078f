"""Mixed-precision solves of right-hand sides far from unit size.

The outer loop stores the FP64 residual directly in FP32 when its max-norm
lies in 1e-20..1e30 and otherwise takes the FP64 residual plus a separate
scaling pass (the FP32 value of an unscaled residual could underflow or
overflow).  The second path is exercised here by scaling the RHS by 1e-24 and
1e32, in colour-split and interleaved storage, in 2D and 3D: the solution is
the scaled oracle solution (the systems are linear) to the mixed-precision
bar, and the solve takes the cycles of the unscaled one (to one cycle)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import from_dev, random_field, relerr, to_dev, unit_level  # noqa: E402


def _hier(lev, op, c, split):
    H = A.Hierarchy(lev.dim, lev.shape, lev.h, 1)
    H.set_level_boxes(0, lev.boxes)
    for (d, s), kind in lev.phys_bc.items():
        H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
    H.set_tuning(A.TUNE_SPLIT_RB, int(split))
    H.finalize()
    return H


CASES = [("2d_helmholtz", 64, 2, "D", "helmholtz"), ("3d_poisson", 32, 3, "N", "poisson")]


@pytest.mark.parametrize("split", [True, False])
@pytest.mark.parametrize("scale", [1e-24, 1e32])
@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_scaled_right_hand_side(case, scale, split):
    _, n, D, bc, op = case
    lev = unit_level(n, D, bc)
    c = 0.3 * lev.h if op == "helmholtz" else 0.0
    sing = lev.singular_components(op)
    f = lev.comp_mean(random_field(lev, 31), sing)
    x_or, st_or = mg.solve(lev, f, op, c, tol_rel=1e-12, max_cycles=100, smoother="rb")
    assert st_or["converged"]
    H = _hier(lev, op, c, split)
    assert H.level_info(0).split_rb == int(split)
    opts = A.default_opts(precision=A.MIXED, smoother=A.SMOOTH_RB, tol_rel=1e-10, max_cycles=100)
    cyc = []
    for s in (1.0, scale):
        fd = to_dev(H, 0, 0, f * s)
        x = torch.zeros_like(fd)
        st = H.solve(0, x, fd, None, opts)
        torch.cuda.synchronize()
        assert st["status"] == 0 and st["converged"], (s, st)
        assert st["r0"] > 0 and np.isfinite(st["rfinal"])
        got = lev.comp_mean(from_dev(H, 0, 0, x, lev), sing)
        assert relerr(got, s * lev.comp_mean(x_or, sing), lev.mask) < 1e-9, s
        cyc.append(st["cycles"])
    assert abs(cyc[0] - cyc[1]) <= 1, cyc
