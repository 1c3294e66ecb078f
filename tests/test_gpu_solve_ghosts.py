"""Mixed-precision level solves in which the outer FP64 residual forms the
ghosts of x where it reads them (no face data, every face filled uniformly
with both ghost layers from its own row): the x-face ghosts come from the
cells the lanes exchange, except at the high x face of a row of odd length,
which the block writes.  Checked on rows of odd and even length, 2D and 3D,
Dirichlet, Neumann and mixed conditions: the solution satisfies the oracle's
discrete system, and the ghosts of the returned solution equal the oracle's
fill of its cells (the solve fills them after its last cycle and the mean
shift)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import MIXED_BC, from_dev, ghost_values, make_hier, random_field, to_dev  # noqa: E402

MIXED3 = {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D", (2, 0): "D", (2, 1): "N"}


def _level(shape, bc):
    D = len(shape)
    bcs = bc if isinstance(bc, dict) else {(d, s): bc for d in range(D) for s in (0, 1)}
    return Level(shape, 1.0 / max(shape), [((0,) * D, tuple(n - 1 for n in shape))], bcs)


CASES = {
    # odd rows: no coarser depth, the exact bottom solve at depth 0
    "2d_37x20_D": ((37, 20), "D"),
    "2d_37x24_mixed": ((37, 24), MIXED_BC),
    "3d_13x8x8_N": ((13, 8, 8), "N"),
    # even rows: the V-cycle, with colour-split storage in 3D
    "2d_136x40_N": ((136, 40), "N"),
    "3d_40x16x24_mixed": ((40, 16, 24), MIXED3),
    "3d_32cubed_N": ((32, 32, 32), "N"),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("op", ["helmholtz", "poisson"])
def test_solution_and_its_ghosts_against_oracle(name, op):
    shape, bc = CASES[name]
    lev = _level(shape, bc)
    c = 0.37 * lev.h if op == "helmholtz" else 0.0
    H, L = make_hier(lev, op, c)
    f = random_field(lev, 5)
    fdev = to_dev(H, L, 0, f)
    x = torch.zeros_like(fdev)
    opts = A.default_opts(precision=A.MIXED, smoother=A.SMOOTH_RB, tol_rel=1e-10, max_cycles=100)
    st = H.solve(L, x, fdev, None, opts)
    assert st["status"] == 0 and st["converged"], st
    torch.cuda.synchronize()
    xs = from_dev(H, L, 0, x, lev)
    # the oracle's system (a singular component takes the solvability shift)
    fo = f.copy()
    sing = lev.singular_components(op)
    if sing:
        fo, _ = mg.solvability_shift(lev, fo, None, sing)
    r = fo - lev.apply(xs, op, c)
    r0 = np.abs(fo[lev.mask]).max()
    assert np.abs(r[lev.mask]).max() <= 2e-10 * r0, (np.abs(r[lev.mask]).max() / r0, st["cycles"])
    # every stored face ghost of the returned x is the fill of its cells
    G = lev.ghosts(xs, None)
    for g, o, m in ghost_values(H, L, 0, x, lev, G):
        assert np.allclose(np.where(m, 0.0, g), o, rtol=1e-12, atol=1e-12 * np.abs(o).max(initial=1.0))
