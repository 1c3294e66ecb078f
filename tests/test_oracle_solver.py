"""Pins of the oracle's level operator and multigrid solver against what the
paper and the mathematics fix: polynomial reproduction (every stencil and
fill is exact on low-degree polynomials, so the discrete solution IS the cell
average of the polynomial), fourth-order convergence (Section 3),
solvability sums, the direct solve of the probe-assembled matrix, an
h-independent V-cycle factor, and independent bookkeeping checks."""
import math
from collections import deque

import numpy as np
import pytest

from oracle import mg
from oracle.level import Level, PAD
from tests.polyfix import Poly1, Trig1, problem


def unit_level(n, D, bc, h=None):
    h = h or 1.0 / n
    bcs = bc if isinstance(bc, dict) else {(d, s): bc for d in range(D) for s in (0, 1)}
    return Level((n,) * D, h, [((0,) * D, (n - 1,) * D)], bcs)


P4a = Poly1([0.3, -1.0, 0.5, 2.0, -1.5])
P4b = Poly1([1.0, 0.7, -2.0, 0.25, 1.0])
P3 = Poly1([-0.2, 1.1, 0.4, -0.9])


def relerr(a, b, lev):
    return np.abs(a - b)[lev.mask].max() / np.abs(b)[lev.mask].max()


MIXED = {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D"}


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("helmholtz", "N"), ("poisson", "D"),
                                   ("poisson", "N"), ("helmholtz", "mixed"), ("poisson", "mixed")])
def test_polynomial_reproduction_2d(op, bc):
    lev = unit_level(32, 2, MIXED if bc == "mixed" else bc)
    c = 0.7 / 32 if op == "helmholtz" else 0.0
    u, f, fd = problem(lev, [(P4a, P4b), (P3, P4a)], op, c)
    # the discrete operator applied to <p> gives <A p> exactly (rounding only)
    Au = lev.apply(u, op, c, fd)
    assert relerr(Au, f, lev) < 1e-10
    x, st = mg.solve(lev, f, op, c, fd, tol_rel=1e-13, max_cycles=80)
    assert st["converged"]
    sing = lev.singular_components(op)
    want = lev.comp_mean(u, sing)
    assert relerr(x, want, lev) < 1e-9
    if sing:
        # exact data satisfy the discrete compatibility condition exactly
        assert abs(st["defects"][0]) < 1e-11 * np.abs(f).max()


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("poisson", "N")])
def test_polynomial_reproduction_3d(op, bc):
    lev = unit_level(16, 3, bc)
    c = 0.3 / 16 if op == "helmholtz" else 0.0
    u, f, fd = problem(lev, [(P4a, P4b, P3), (P3, P4a, P4b)], op, c)
    x, st = mg.solve(lev, f, op, c, fd, tol_rel=1e-13, max_cycles=80)
    assert st["converged"]
    want = lev.comp_mean(u, lev.singular_components(op))
    assert relerr(x, want, lev) < 1e-9


def l_shape_level(cf, phys="D"):
    # an L-shaped level of two boxes inside a 32^2 grid, plus a separate box:
    # three kinds of row end (physical, coarse-fine, box-to-box) and two
    # face-connected components
    boxes = [((0, 4), (15, 11)), ((16, 4), (23, 19)), ((4, 20), (11, 27))]
    return Level((32, 32), 1.0 / 32, boxes, {(d, s): phys for d in range(2) for s in (0, 1)}, cf)


@pytest.mark.parametrize("op,cf", [("helmholtz", "D"), ("helmholtz", "N"), ("poisson", "N"), ("poisson", "D")])
def test_polynomial_reproduction_multibox_coarse_fine_faces(op, cf):
    lev = l_shape_level(cf, phys="N")
    assert lev.ncomp == 2
    c = 0.5 / 32 if op == "helmholtz" else 0.0
    u, f, fd = problem(lev, [(P4a, P4b), (P3, P3)], op, c)
    assert relerr(lev.apply(u, op, c, fd), f, lev) < 1e-10
    x, st = mg.solve(lev, f, op, c, fd, tol_rel=1e-13, max_cycles=100)
    assert st["converged"]
    sing = lev.singular_components(op)
    assert len(sing) == (2 if (op == "poisson" and cf == "N") else 0)
    assert relerr(x, lev.comp_mean(u, sing), lev) < 1e-9


@pytest.mark.parametrize("op,bc", [("poisson", "D"), ("helmholtz", "D"), ("poisson", "N")])
def test_fourth_order_convergence(op, bc):
    errs = []
    for n in (16, 32, 64):
        lev = unit_level(n, 2, bc)
        c = 0.05 if op == "helmholtz" else 0.0
        if bc == "N":
            terms = [(Trig1(2 * math.pi, math.pi / 2), Trig1(2 * math.pi, math.pi / 2))]  # cos cos
        else:
            terms = [(Trig1(math.pi), Trig1(2 * math.pi, 0.3))]
        u, f, fd = problem(lev, terms, op, c)
        x, st = mg.solve(lev, f, op, c, fd, tol_rel=1e-13, max_cycles=100)
        sing = lev.singular_components(op)
        err = lev.comp_mean(x - u, sing)
        errs.append((np.abs(err[lev.mask]).mean(), np.abs(err[lev.mask]).max()))
    for (a1, m1), (a2, m2) in zip(errs, errs[1:]):
        assert math.log2(a1 / a2) > 3.7     # L1: fourth order
        assert math.log2(m1 / m2) > 2.8     # Linf: third-order truncation on a codim-1 set


def test_solvability_sum_and_constant_null_vector():
    lev = l_shape_level("N", phys="N")
    rng = np.random.default_rng(3)
    u = lev.zeros()
    u[lev.mask] = rng.normal(size=lev.ncells)
    fd = lev.zero_face_data()
    for k in fd:
        fd[k][lev.row_end(*k)] = rng.normal(size=int(lev.row_end(*k).sum()))
    Lu = lev.apply(u, "poisson", 0.0, fd)
    h = lev.h
    for comp in range(lev.ncomp):
        sel = lev.labels == comp
        bsum = sum(fd[k][lev.row_end(*k) & sel].sum() for k in fd) * h
        lsum = Lu[sel].sum() * h * h
        assert abs(lsum - bsum) < 1e-12 * (np.abs(Lu[sel]).sum() * h * h)
    one = lev.zeros()
    one[lev.mask] = 1.0
    assert np.abs(lev.apply(one, "poisson", 0.0)[lev.mask]).max() < 1e-9


@pytest.mark.parametrize("op,bc,cf", [("helmholtz", "D", "D"), ("poisson", "N", "N"), ("poisson", "D", "N")])
def test_vcycle_solution_equals_direct_lu(op, bc, cf):
    lev = Level((16, 16), 1.0 / 16, [((0, 0), (7, 15)), ((8, 4), (15, 11))],
                {(d, s): bc for d in range(2) for s in (0, 1)}, cf)
    c = 0.4 / 16 if op == "helmholtz" else 0.0
    rng = np.random.default_rng(5)
    f = lev.zeros()
    f[lev.mask] = rng.normal(size=lev.ncells)
    fd = lev.zero_face_data()
    for k in fd:
        fd[k][lev.row_end(*k)] = rng.normal(size=int(lev.row_end(*k).sum()))
    xd = mg.direct_solve(lev, f, op, c, fd)
    x, st = mg.solve(lev, f, op, c, fd, tol_rel=1e-13, max_cycles=200)
    sing = lev.singular_components(op)
    assert relerr(lev.comp_mean(x, sing), lev.comp_mean(xd, sing), lev) < 1e-10
    # and the direct solution agrees with scipy's sparse LU of the same matrix
    import scipy.sparse.linalg as spla
    import scipy.sparse as sp
    M, cells = mg.assemble(lev, op, c)
    b = lev.apply(lev.zeros(), op, c, fd)[lev.mask]
    if not sing:
        xs = spla.splu(sp.csc_matrix(M)).solve(f[lev.mask] - b)
        assert np.abs(xs - xd[lev.mask]).max() < 1e-10 * np.abs(xs).max()


def test_vcycle_factor_independent_of_h():
    rates = []
    for n in (32, 64, 128):
        lev = unit_level(n, 2, "N")
        rng = np.random.default_rng(0)
        f = lev.zeros()
        f[lev.mask] = rng.normal(size=lev.ncells)
        _, st = mg.solve(lev, f, "poisson", 0.0, tol_rel=1e-9, max_cycles=8)
        hist = st["history"]
        rates.append((hist[-1] / hist[2]) ** (1.0 / (len(hist) - 3)))
    assert max(rates) < 0.5
    assert max(rates) / min(rates) < 1.25


def test_diagonal_equals_assembled_diagonal():
    for op, c in (("helmholtz", 0.3 / 16), ("poisson", 0.0)):
        lev = Level((16, 16), 1.0 / 16, [((0, 0), (7, 15)), ((8, 4), (15, 11))],
                    {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D"}, "N")
        M, cells = mg.assemble(lev, op, c)
        assert np.allclose(np.diag(M), lev.diagonal(op, c)[lev.mask], rtol=1e-13, atol=1e-9)


def test_components_match_breadth_first_search():
    rng = np.random.default_rng(7)
    for trial in range(5):
        boxes = []
        occ = np.zeros((48, 48), bool)
        for _ in range(12):
            lo = rng.integers(0, 10, size=2) * 4
            sz = rng.integers(1, 3, size=2) * 4
            hi = np.minimum(lo + sz, 48) - 1
            if occ[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1].any() or (hi - lo + 1).min() < 4:
                continue
            occ[lo[0]:hi[0] + 1, lo[1]:hi[1] + 1] = True
            boxes.append((tuple(lo), tuple(hi)))
        lev = Level((48, 48), 1 / 48, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)})
        # breadth-first search with face neighbours
        lab = -np.ones((48, 48), int)
        ncomp = 0
        for start in zip(*np.nonzero(occ)):
            if lab[start] >= 0:
                continue
            q = deque([start])
            lab[start] = ncomp
            while q:
                i, j = q.popleft()
                for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
                    a, b = i + di, j + dj
                    if 0 <= a < 48 and 0 <= b < 48 and occ[a, b] and lab[a, b] < 0:
                        lab[a, b] = ncomp
                        q.append((a, b))
            ncomp += 1
        assert lev.ncomp == ncomp
        got = lev.labels[lev.inner]
        # same partition up to relabelling
        pairs = set(zip(got[occ].tolist(), lab[occ].tolist()))
        assert len(pairs) == ncomp


def test_restriction_of_averages_and_prolongation_of_linears():
    fine = unit_level(16, 2, "D")
    coarse = fine.coarsen()
    term = [(P4a, P3)]
    uf, _, _ = problem(fine, term, "poisson", 0.0)
    uc, _, _ = problem(coarse, term, "poisson", 0.0)
    assert relerr(mg.restrict(fine, uf, coarse), uc, coarse) < 1e-13
    lin = [(Poly1([0.3, 1.7]), Poly1([1.0])), (Poly1([1.0]), Poly1([-0.4, 2.2]))]
    # linear functions vanishing on the boundary faces are not needed: the
    # interior of the coarse level reproduces exactly wherever both
    # neighbours are real cells
    lc, _, _ = problem(coarse, lin, "poisson", 0.0)
    lf, _, _ = problem(fine, lin, "poisson", 0.0)
    pf = mg.prolong(coarse, lc, fine)
    inner = (slice(PAD + 2, PAD + 14),) * 2
    assert np.abs(pf[inner] - lf[inner]).max() < 1e-13


def test_red_black_half_sweeps_touch_only_their_colour():
    lev = unit_level(16, 2, "D")
    D = lev.diagonal("poisson", 0.0)
    rng = np.random.default_rng(1)
    f = lev.zeros()
    f[lev.mask] = rng.normal(size=lev.ncells)
    red = lev.colour() & lev.mask
    e1 = lev.zeros()
    r = f - lev.apply(e1, "poisson", 0.0)
    e1[red] += r[red] / D[red]
    e2 = mg.red_black(lev, lev.zeros(), f, "poisson", 0.0, D, 1)
    assert np.array_equal(e1[red], e2[red])
    assert not np.array_equal(e2[~red & lev.mask], 0 * e2[~red & lev.mask])
