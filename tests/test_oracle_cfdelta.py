"""Pins of the coarse-fine face-data correction for solvability (eq.
correctingFaceAvg): after the correction the discrete compatibility
condition holds on every singular component, the correction is one constant
on that component's coarse-fine faces and nothing elsewhere, the solve then
needs no right-hand-side shift and matches the direct solve with the
corrected data, and a component without coarse-fine faces falls back to the
right-hand-side shift."""
import numpy as np
import pytest

from oracle import mg
from oracle.level import Level


def cf_level():
    # an L-shape and a separate box inside a 32^2 grid: two components, both
    # with physical Neumann and coarse-fine Neumann faces
    boxes = [((0, 4), (15, 11)), ((16, 4), (23, 19)), ((4, 20), (11, 27))]
    return Level((32, 32), 1.0 / 32, boxes, {(d, s): "N" for d in range(2) for s in (0, 1)}, "N")


def data(lev, seed):
    rng = np.random.default_rng(seed)
    f = lev.zeros()
    f[lev.mask] = rng.normal(size=lev.ncells)
    fd = lev.zero_face_data()
    for k in fd:
        e = lev.row_end(*k)
        fd[k][e] = rng.normal(size=int(e.sum()))
    return f, fd


def test_correction_restores_compatibility():
    lev = cf_level()
    f, fd = data(lev, 1)
    comps = lev.singular_components("poisson")
    assert comps == [0, 1]
    f2, fd2, defects = mg.cf_delta_correction(lev, f, fd, comps)
    assert np.array_equal(f2, f)  # no RHS shift where coarse-fine faces exist
    hD, hD1 = lev.h ** 2, lev.h
    for c, defect in zip(comps, defects):
        sel = lev.labels == c
        assert abs(defect) > 1e-3  # random data are incompatible
        bsum = sum(fd2[(d, s)][lev.row_end(d, s) & sel].sum() for d in range(2) for s in (0, 1)) * hD1
        assert abs(hD * f[sel].sum() - bsum) < 1e-13 * (hD * np.abs(f[sel]).sum() + abs(bsum))
        deltas = []
        for d in range(2):
            for s in (0, 1):
                end = lev.row_end(d, s) & sel
                phys = lev.end_is_physical(d, s)
                diff = (fd2[(d, s)] - fd[(d, s)])
                assert np.all(diff[end & phys] == 0.0)
                deltas.append(diff[end & ~phys])
        dv = np.concatenate(deltas)
        assert dv.size > 0 and np.ptp(dv) < 1e-14 * abs(dv[0]) + 1e-300


@pytest.mark.parametrize("smoother", ["jacobi", "rb"])
def test_solve_with_corrected_data(smoother):
    lev = cf_level()
    f, fd = data(lev, 2)
    x, st = mg.solve(lev, f, "poisson", 0.0, fd, tol_rel=1e-12, max_cycles=200, smoother=smoother, cf_delta=True)
    assert st["converged"]
    assert np.array_equal(st["rhs"], f)
    fd2 = st["fd"]
    # the system with the corrected data is consistent: the residual of the
    # unshifted right-hand side vanishes
    r = f - lev.apply(x, "poisson", 0.0, fd2)
    assert np.abs(r[lev.mask]).max() < 1e-10 * np.abs(f).max()
    xd = mg.direct_solve(lev, f, "poisson", 0.0, fd2)
    comps = lev.singular_components("poisson")
    a, b = lev.comp_mean(x, comps), lev.comp_mean(xd, comps)
    assert np.abs(a - b)[lev.mask].max() < 1e-9 * np.abs(b).max()


def test_component_without_cf_faces_takes_the_rhs_shift():
    lev = Level((16, 16), 1 / 16, [((0, 0), (15, 15))], {(d, s): "N" for d in range(2) for s in (0, 1)}, "N")
    f, fd = data(lev, 3)
    x1, s1 = mg.solve(lev, f, "poisson", 0.0, fd, tol_rel=1e-12, cf_delta=True)
    x2, s2 = mg.solve(lev, f, "poisson", 0.0, fd, tol_rel=1e-12)
    # same shift up to the summation order of the defect
    assert np.abs(x1 - x2)[lev.mask].max() < 1e-12 * np.abs(x2).max()
    assert np.allclose(s1["defects"], s2["defects"], rtol=1e-13, atol=1e-15)
