"""Pins of the oracle's bottom-size rule: coarsening stops at the first depth
whose largest component has at most `bottom_cells` cells (the paper leaves
the bottom solver open; the coarsest depth is solved exactly).  The depth
counts follow from the rule by hand; a hierarchy of one depth makes one
V-cycle the exact solve, checked against numpy's dense solve of the probed
matrix; and the converged solution does not depend on where the hierarchy
stops."""
import numpy as np
import pytest

from oracle import mg
from oracle.level import Level


def full(n, D, bc):
    return Level((n,) * D, 1.0 / n, [((0,) * D, (n - 1,) * D)], {(d, s): bc for d in range(D) for s in (0, 1)})


def rand_cells(lev, seed):
    u = lev.zeros()
    u[lev.mask] = np.random.default_rng(seed).normal(size=lev.ncells)
    return u


@pytest.mark.parametrize("B,sides", [(0, [64, 32, 16, 8, 4]), (16, [64, 32, 16, 8, 4]), (64, [64, 32, 16, 8]),
                                     (256, [64, 32, 16]), (4095, [64, 32]), (4096, [64])])
def test_depths_single_box(B, sides):
    lev = full(64, 2, "N")
    assert [l.shape[0] for l in lev.hierarchy(B)] == sides


def test_depths_follow_the_largest_component():
    # two components: 16 x 32 and 8 x 32 cells (the gap of 8 stays >= 2 down to depth 2)
    lev = Level((64, 32), 1 / 64, [((0, 0), (15, 31)), ((24, 0), (31, 31))],
                {(d, s): "N" for d in range(2) for s in (0, 1)}, "N")
    assert lev.largest_component() == 512
    # depth 1: 8 x 16 = 128 and 4 x 16 = 64 cells; depth 2 would need sides >= 8
    assert len(lev.hierarchy(0)) == 2
    assert len(lev.hierarchy(512)) == 1
    assert len(lev.hierarchy(511)) == 2


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("poisson", "N")])
def test_one_depth_vcycle_is_the_exact_solve(op, bc):
    lev = full(16, 2, bc)
    c = 0.3 * lev.h if op == "helmholtz" else 0.0
    M = mg.MG(lev, op, c, bottom_cells=lev.ncells)
    assert len(M.levels) == 1
    f = lev.comp_mean(rand_cells(lev, 1), M.sing[0])
    e = M.vcycle(f)
    A, cells = mg.assemble(lev, op, c)
    if op == "helmholtz":
        want = np.linalg.solve(A, f[lev.mask])
    else:
        # the mean-free solution of the singular system
        want = np.linalg.lstsq(A, f[lev.mask], rcond=None)[0]
        want -= want.mean()
        assert abs(e[lev.mask].mean()) < 1e-13
    assert np.abs(e[lev.mask] - want).max() < 1e-10 * np.abs(want).max()


@pytest.mark.parametrize("op,bc,D,n,B", [("helmholtz", "D", 2, 64, 256), ("poisson", "N", 2, 64, 256),
                                          ("poisson", "N", 3, 16, 512)])
@pytest.mark.parametrize("smoother", ["jacobi", "rb"])
def test_bigger_bottom_same_solution_and_contracts(op, bc, D, n, B, smoother):
    lev = full(n, D, bc)
    c = 0.5 * lev.h if op == "helmholtz" else 0.0
    f = rand_cells(lev, 2)
    x0, s0 = mg.solve(lev, f, op, c, tol_rel=1e-12, max_cycles=100, smoother=smoother)
    x1, s1 = mg.solve(lev, f, op, c, tol_rel=1e-12, max_cycles=100, smoother=smoother, bottom_cells=B)
    assert s0["converged"] and s1["converged"]
    assert len(lev.hierarchy(B)) < len(lev.hierarchy())
    assert np.abs(x1 - x0)[lev.mask].max() < 1e-10 * np.abs(x0).max()
    # the two hierarchies contract alike (over the first cycles, before the
    # residual nears rounding level)
    worst = [np.max(np.array(s["history"])[1:9] / np.array(s["history"])[:8]) for s in (s0, s1)]
    assert worst[1] < 1.05 * worst[0] and worst[1] < 0.6
