"""The FP32 V-cycle's coarse tail in one workgroup (AMG_TUNE_TAIL) against
the same solves launching every operation of every depth: the tail engages
where the layout allows it (level info), and mixed-precision solves with and
without it take the same number of cycles, with residual histories equal to
FP32 rounding and solutions equal to the solve tolerance; Dirichlet, Neumann
(singular: the mean removal inside the tail), mixed and periodic faces
(ghosts wrapping onto the box), Helmholtz and
Poisson, red-black and Jacobi smoothing, 2D and 3D, cubic and ragged boxes,
with the bottom at the layout's last depth or at a chosen size.  The
tail-on solves also match the oracle's (the default of every other mixed
parity test)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import MIXED_BC, from_dev, to_dev  # noqa: E402

CASES = {
    # name: (shape, bc, bottom_cells)
    "3d_32_D": ((32, 32, 32), "D", 0),
    "3d_32_N_bottom512": ((32, 32, 32), "N", 512),
    "3d_ragged_mixed": ((48, 32, 16), "M", 0),
    "2d_128_N": ((128, 128), "N", 0),
    "2d_128_D_bottom256": ((128, 128), "D", 256),
    "2d_64_mixed": ((64, 64), "M", 0),
    "2d_128_periodic": ((128, 128), "P", 0),
    "2d_128_periodic_x": ((128, 64), "PX", 0),
    "3d_32_periodic_xz": ((32, 32, 32), "PXZ", 0),
}


def bcs(D, kind):
    if kind == "M":
        b = dict(MIXED_BC)
        if D == 3:
            b.update({(2, 0): "D", (2, 1): "N"})
        return b
    if kind == "PX":  # periodic in x, Dirichlet / Neumann in y
        return {(0, 0): "P", (0, 1): "P", (1, 0): "D", (1, 1): "N"}
    if kind == "PXZ":  # periodic in x and z, Neumann in y (singular)
        return {(0, 0): "P", (0, 1): "P", (1, 0): "N", (1, 1): "N", (2, 0): "P", (2, 1): "P"}
    return {(d, s): kind for d in range(D) for s in (0, 1)}


def hier(shape, bc, op, c, bottom_cells, tail):
    D = len(shape)
    H = A.Hierarchy(D, shape, 1.0 / shape[0], 1)
    H.set_level_boxes(0, [((0,) * D, tuple(n - 1 for n in shape))])
    for (d, s), k in bc.items():
        H.set_physical_bc(d, s, {"D": A.DIRICHLET, "N": A.NEUMANN, "P": A.PERIODIC}[k])
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
    if bottom_cells:
        H.set_bottom_cells(bottom_cells)
    H.set_tuning(A.TUNE_TAIL, tail)
    H.finalize()
    return H


def rhs(lev, op, seed):
    rng = np.random.default_rng(seed)
    f = lev.zeros()
    f[lev.mask] = rng.normal(size=lev.ncells)
    if op == "poisson" and all(k in "NP" for k in lev.phys_bc.values()):
        f[lev.mask] -= f[lev.mask].mean()
    return f


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("op", ["helmholtz", "poisson"])
@pytest.mark.parametrize("smoother", ["rb", "jacobi"])
def test_tail_matches_the_launch_per_operation_cycle(name, op, smoother):
    shape, kind, bottom = CASES[name]
    D = len(shape)
    bc = bcs(D, kind)
    c = 1e-4 if op == "helmholtz" else 0.0
    lev = Level(shape, 1.0 / shape[0], [((0,) * D, tuple(n - 1 for n in shape))], bc)
    Hon = hier(shape, bc, op, c, bottom, 1)
    Hoff = hier(shape, bc, op, c, bottom, 0)
    assert Hon.level_info(0).tail_depth >= 1
    assert Hoff.level_info(0).tail_depth == -1
    sm = A.SMOOTH_RB if smoother == "rb" else A.SMOOTH_JACOBI
    opts = A.default_opts(precision=A.MIXED, smoother=sm, tol_rel=1e-10, max_cycles=200,
                          omega_rb=1.3 if op == "poisson" else 1.0)
    f = rhs(lev, op, 3)
    out = {}
    for key, H in (("on", Hon), ("off", Hoff)):
        x = to_dev(H, 0, 0, lev.zeros())
        st = H.solve(0, x, to_dev(H, 0, 0, f), None, opts)
        assert st["status"] == 0 and st["converged"], (key, st["cycles"])
        out[key] = (st, from_dev(H, 0, 0, x, lev))
    (s_on, x_on), (s_off, x_off) = out["on"], out["off"]
    assert s_on["cycles"] == s_off["cycles"]
    h_on, h_off = np.array(s_on["history"]), np.array(s_off["history"])
    assert np.all(np.abs(h_on - h_off) <= 1e-3 * h_off + 1e-12 * h_off[0])
    m = lev.mask
    scale = np.abs(x_off[m]).max()
    assert np.abs(x_on - x_off)[m].max() <= 1e-6 * scale


@pytest.mark.parametrize("shape,kind", [((32, 32), "N"), ((16, 16, 16), "M"), ((32, 32), "P")])
def test_tail_solve_matches_the_oracle(shape, kind):
    D = len(shape)
    bc = bcs(D, kind)
    lev = Level(shape, 1.0 / shape[0], [((0,) * D, tuple(n - 1 for n in shape))], bc)
    H = hier(shape, bc, "poisson", 0.0, 0, 1)
    assert H.level_info(0).tail_depth >= 1
    f = rhs(lev, "poisson", 5)
    x = to_dev(H, 0, 0, lev.zeros())
    st = H.solve(0, x, to_dev(H, 0, 0, f), None,
                 A.default_opts(precision=A.MIXED, smoother=A.SMOOTH_RB, tol_rel=1e-12, max_cycles=200))
    assert st["converged"]
    got = from_dev(H, 0, 0, x, lev)
    if D == 2:
        want = mg.direct_solve(lev, f, "poisson", 0.0)
    else:  # the dense referee would take half a minute at 16^3
        want, ost = mg.solve(lev, f, "poisson", 0.0, smoother="rb", tol_rel=1e-13, max_cycles=100)
        assert ost["converged"]
    m = lev.mask
    if all(k in "NP" for k in bc.values()):
        got[m] -= got[m].mean()
        want[m] -= want[m].mean()
    assert np.abs(got - want)[m].max() <= 1e-9 * np.abs(want[m]).max()
