"""The solve-time error contract of the C ABI, forced from the host:

* AMG_ENOTCONVERGED: max_cycles = 1 below the tolerance; x holds the last
  iterate (equal to the oracle's iterate after one cycle) and the stats are
  valid;
* AMG_ENONFINITE: a NaN or an Inf in the right-hand side (the max-norms map
  NaN to infinity, so neither vanishes in a max reduction);
* AMG_ESOLVABILITY: solvability enforcement off on a singular component
  whose mean defect (eq. velocity_disc_solvabilityCond) exceeds the stopping
  target: returned before any cycle with x untouched; below the target the
  solve runs.

Every case is an ordinary solve on valid buffers; the kernels run to their
normal end."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import amr, mg  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import from_dev, make_hier, random_field, relerr, to_dev, unit_level  # noqa: E402


@pytest.mark.parametrize("graph", [1, 0])
@pytest.mark.parametrize("prec", [A.FP64, A.MIXED])
def test_not_converged_returns_the_last_iterate(prec, graph):
    lev = unit_level(32, 2, "D")
    c = 0.5e-3 / 32
    f = random_field(lev, 11)
    H, L = make_hier(lev, "helmholtz", c)
    fdev = to_dev(H, L, 0, f)
    x = torch.zeros_like(fdev)
    st = H.solve(L, x, fdev, None, A.default_opts(precision=prec, tol_rel=1e-14, max_cycles=1, use_graph=graph))
    torch.cuda.synchronize()
    assert st["status"] == A.ENOTCONVERGED
    assert st["cycles"] == 1 and not st["converged"]
    assert len(st["history"]) == 2 and st["rfinal"] == st["history"][1]
    assert 0 < st["history"][1] < st["history"][0]
    x1, st_or = mg.solve(lev, f, "helmholtz", c, tol_rel=1e-14, max_cycles=1)
    assert st_or["cycles"] == 1
    tol = 1e-11 if prec == A.FP64 else 1e-6  # one FP32 V-cycle
    assert relerr(from_dev(H, L, 0, x, lev), x1, lev.mask) < tol
    assert abs(st["history"][1] - st_or["history"][1]) <= (1e-9 if prec == A.FP64 else 1e-4) * st_or["history"][1]


@pytest.mark.parametrize("bad", [float("nan"), float("inf")])
@pytest.mark.parametrize("prec", [A.FP64, A.MIXED])
@pytest.mark.parametrize("D", [2, 3])
def test_non_finite_right_hand_side(D, prec, bad):
    n = 32 if D == 2 else 16
    lev = unit_level(n, D, "D")
    f = random_field(lev, 12)
    f[tuple([n // 2 + 2] * D)] = bad
    H, L = make_hier(lev, "helmholtz", 1e-3)
    fdev = to_dev(H, L, 0, f)
    x = torch.zeros_like(fdev)
    with pytest.raises(A.AmgError) as e:
        H.solve(L, x, fdev, None, A.default_opts(precision=prec))
    assert e.value.code == A.ENONFINITE
    # the transposed (adjoint) solve checks its source the same way
    with pytest.raises(A.AmgError) as e:
        H.solve_adjoint(L, torch.zeros_like(fdev), fdev, A.default_opts(precision=prec))
    assert e.value.code == A.ENONFINITE


def _neumann_problem(shift):
    """32^2 pure-Neumann Poisson problem whose RHS has mean `shift` (the
    solvable part made mean-free first)."""
    lev = unit_level(32, 2, "N")
    f = random_field(lev, 13)
    f = lev.comp_mean(f, [0])
    f[lev.mask] += shift
    return lev, f


@pytest.mark.parametrize("prec", [A.FP64, A.MIXED])
def test_solvability_off_rejects_an_unreachable_target(prec):
    lev, f = _neumann_problem(1e-3)
    H, L = make_hier(lev, "poisson", 0.0)
    fdev = to_dev(H, L, 0, f)
    x0 = torch.full_like(fdev, 0.25)
    x = x0.clone()
    st = None
    with pytest.raises(A.AmgError) as e:
        st = H.solve(L, x, fdev, None, A.default_opts(precision=prec, solvability=A.SOLV_OFF, tol_rel=1e-10))
    assert st is None and e.value.code == A.ESOLVABILITY
    assert "mean defect" in str(e.value)
    # x untouched on the cells (ghosts are the library's)
    got, want = from_dev(H, L, 0, x, lev), from_dev(H, L, 0, x0, lev)
    assert np.array_equal(got[lev.mask], want[lev.mask])
    # the same data with enforcement (the default RHS shift) converges, and
    # reports the defect the oracle computes
    x = torch.zeros_like(fdev)
    st = H.solve(L, x, fdev, None, A.default_opts(precision=prec, tol_rel=1e-10))
    assert st["status"] == 0 and st["converged"]
    _, defects = mg.solvability_shift(lev, f, None, [0])
    assert np.allclose(st["defects"], defects, rtol=1e-9, atol=1e-15)


def test_solvability_off_with_a_defect_below_the_target_runs():
    # a defect below the tolerance: enforcement off still converges
    lev, f = _neumann_problem(1e-14)
    H, L = make_hier(lev, "poisson", 0.0)
    fdev = to_dev(H, L, 0, f)
    x = torch.zeros_like(fdev)
    st = H.solve(L, x, fdev, None, A.default_opts(precision=A.FP64, solvability=A.SOLV_OFF, tol_rel=1e-8))
    assert st["status"] == 0 and st["converged"]


def test_composite_solvability_off_rejects_an_unreachable_target():
    boxes = [[((0, 0), (31, 31))], [((16, 16), (47, 47))]]
    hier = amr.Hierarchy((32, 32), 1.0 / 32, boxes, {(d, s): "N" for d in range(2) for s in (0, 1)})
    H = A.Hierarchy(2, (32, 32), 1.0 / 32, 2)
    for l, bl in enumerate(boxes):
        H.set_level_boxes(l, bl)
    H.set_cf_mode(1, A.CF_INTERP)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.NEUMANN)
    H.set_operator(A.POISSON, 0.0)
    H.finalize()
    fs = [lev.zeros() for lev in hier.levels]
    for l, lev in enumerate(hier.levels):
        fs[l][lev.mask] = 1e-3  # mean 1e-3 over the whole domain: defect = 1e-3
    fd = [to_dev(H, l, 0, fs[l]) for l in range(2)]
    xs = [torch.zeros_like(t) for t in fd]
    with pytest.raises(A.AmgError) as e:
        H.solve_composite(xs, fd, None, A.default_opts(precision=A.FP64, solvability=A.SOLV_OFF))
    assert e.value.code == A.ESOLVABILITY
