"""Pins of the oracle's composite (multi-level) operators: coarse-fine
interpolation weights in exact arithmetic, polynomial reproduction of the
composite operator and solve, conservation of the refluxed operator, and the
directly solved composite system as referee; refinement ratios 2 and 4
(eq. grids), the prolongation of corrections exact on linear functions."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import amr
from tests.polyfix import Poly1, problem


def avg_mono(k, a, b):
    return (Fr(b) ** (k + 1) - Fr(a) ** (k + 1)) / ((k + 1) * (Fr(b) - Fr(a)))


def test_centred_weights_match_hand_derived_values():
    # derived by hand for the centred window (child 0); child 1 is its mirror
    want0 = [Fr(-3, 128), Fr(11, 64), Fr(1), Fr(-11, 64), Fr(3, 128)]
    assert amr.cfi_weights_1d(0, 0) == want0
    assert amr.cfi_weights_1d(0, 1) == want0[::-1]


@pytest.mark.parametrize("shift", range(-2, 3))
@pytest.mark.parametrize("child", (0, 1))
def test_weights_exact_to_degree_4_and_not_5(shift, child):
    w = amr.cfi_weights_1d(shift, child)
    mp = 2 - shift
    x0 = Fr(mp) + Fr(child, 2)
    for k in range(6):
        data = [avg_mono(k, m, m + 1) for m in range(5)]
        got = sum(wi * di for wi, di in zip(w, data))
        assert (got == avg_mono(k, x0, x0 + Fr(1, 2))) == (k <= 4)


@pytest.mark.parametrize("shift", range(-2, 3))
def test_weights_are_conservative(shift):
    w0, w1 = amr.cfi_weights_1d(shift, 0), amr.cfi_weights_1d(shift, 1)
    mean = [(a + b) / 2 for a, b in zip(w0, w1)]
    assert mean == [Fr(1) if m == 2 - shift else Fr(0) for m in range(5)]


@pytest.mark.parametrize("shift", range(-2, 3))
@pytest.mark.parametrize("child", range(4))
def test_ratio4_weights_exact_to_degree_4_and_not_5(shift, child):
    w = amr.cfi_weights_1d(shift, child, 4)
    x0 = Fr(2 - shift) + Fr(child, 4)
    for k in range(6):
        data = [avg_mono(k, m, m + 1) for m in range(5)]
        got = sum(wi * di for wi, di in zip(w, data))
        assert (got == avg_mono(k, x0, x0 + Fr(1, 4))) == (k <= 4)


@pytest.mark.parametrize("shift", range(-2, 3))
def test_ratio4_weights_are_conservative_and_mirror(shift):
    ws = [amr.cfi_weights_1d(shift, a, 4) for a in range(4)]
    mean = [sum(col) / 4 for col in zip(*ws)]
    assert mean == [Fr(1) if m == 2 - shift else Fr(0) for m in range(5)]
    if shift == 0:  # the centred window is symmetric: child a mirrors child 3 - a
        for a in range(4):
            assert ws[a] == ws[3 - a][::-1]


@pytest.mark.parametrize("ratio", [2, 4])
def test_prolongation_exact_on_linear_functions(ratio):
    """The correction prolongation reproduces a linear function's cell
    averages at every child whose coarse neighbours are cells (a linear
    function's cell average is its value at the centre)."""
    from oracle.level import Level
    D = 2
    coarse = Level((8, 8), 1 / 8, [((0, 0), (7, 7))], {(d, s): "D" for d in range(D) for s in (0, 1)})
    n = 8 * ratio
    fine = Level((n, n), 1 / n, [((0, 0), (n - 1, n - 1))], {(d, s): "D" for d in range(D) for s in (0, 1)})
    lin = lambda x, y: 0.3 + 1.7 * x - 0.6 * y  # noqa: E731
    xc = (np.arange(8) + 0.5) / 8
    ec = coarse.zeros()
    ec[coarse.inner] = lin(xc[:, None], xc[None, :])
    got = amr.prolong_ratio(coarse, ec, fine, ratio)[fine.inner]
    xf = (np.arange(n) + 0.5) / n
    want = lin(xf[:, None], xf[None, :])
    inner = (slice(ratio, n - ratio), slice(ratio, n - ratio))  # children whose neighbours are cells
    assert np.abs(got[inner] - want[inner]).max() < 1e-13
    if ratio == 2:
        from oracle import mg
        assert np.array_equal(amr.prolong_ratio(coarse, ec, fine, 2), mg.prolong(coarse, ec, fine))


P4a = Poly1([0.3, -1.0, 0.5, 2.0, -1.5])
P4b = Poly1([1.0, 0.7, -2.0, 0.25, 1.0])
P3 = Poly1([-0.2, 1.1, 0.4, -0.9])


def two_level(bc):
    return amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((8, 8), (15, 23)), ((16, 8), (23, 15))]],
                         {(d, s): bc for d in range(2) for s in (0, 1)})


def three_level(bc):
    return amr.Hierarchy((16, 16), 1.0 / 16,
                         [[((0, 0), (15, 15))], [((4, 4), (27, 27))], [((16, 16), (31, 31))]],
                         {(d, s): bc for d in range(2) for s in (0, 1)})


def two_level_r4(bc):
    # ratio 4: level 1 on the 64^2 grid, an L of two boxes
    return amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((16, 16), (39, 47)), ((40, 16), (47, 31))]],
                         {(d, s): bc for d in range(2) for s in (0, 1)}, ratio=4)


def three_level_r4(bc):
    return amr.Hierarchy((8, 8), 1.0 / 8, [[((0, 0), (7, 7))], [((8, 8), (23, 23))], [((48, 48), (79, 79))]],
                         {(d, s): bc for d in range(2) for s in (0, 1)}, ratio=4)


def poly_data(H, op, c):
    us, fs, fds = [], [], []
    for lev in H.levels:
        u, f, fd = problem(lev, [(P4a, P4b), (P3, P4a)], op, c)
        us.append(u)
        fs.append(f)
        fds.append(fd)
    return us, fs, fds


def rel(U, V, H):
    num = max(np.abs(U[l] - V[l])[H.valid[l]].max() for l in range(H.nlev))
    return num / max(np.abs(V[l][H.valid[l]]).max() for l in range(H.nlev))


@pytest.mark.parametrize("make", [two_level, three_level, two_level_r4, three_level_r4])
@pytest.mark.parametrize("op,bc,c", [("helmholtz", "D", 0.5 / 16), ("poisson", "N", 0.0), ("poisson", "D", 0.0)])
def test_composite_reproduces_polynomials(make, op, bc, c):
    H = make(bc)
    us, fs, fds = poly_data(H, op, c)
    A = H.composite_apply(H.average_down_all(us), op, c, fds)
    assert rel(A, fs, H) < 1e-12
    U, st = amr.composite_solve(H, fs, op, c, fds, tol_rel=1e-12, max_cycles=80)
    assert st["converged"]
    if H.singular(op):
        m = H.composite_mean(us)
        us = [np.where(H.levels[l].mask, us[l] - m, 0.0) for l in range(H.nlev)]
        assert abs(st["defect"]) < 1e-12
    assert rel(U, us, H) < 1e-9


@pytest.mark.parametrize("make", [two_level, two_level_r4, three_level_r4])
def test_refluxed_operator_is_conservative(make):
    H = make("N")
    rng = np.random.default_rng(0)
    U = []
    for l, lev in enumerate(H.levels):
        u = lev.zeros()
        u[lev.mask] = rng.normal(size=lev.ncells)
        U.append(u)
    U = H.average_down_all(U)
    fds = []
    for lev in H.levels:
        fd = lev.zero_face_data()
        for k in fd:
            e = lev.end_is_physical(*k)
            fd[k][e] = rng.normal(size=int(e.sum()))
        fds.append(fd)
    L = H.composite_apply(U, "poisson", 0.0, fds)
    vol = sum(L[l][H.valid[l]].sum() * H.levels[l].h ** 2 for l in range(H.nlev))
    bnd = sum(fds[l][k][H.levels[l].end_is_physical(*k) & H.valid[l]].sum() * H.levels[l].h
              for l in range(H.nlev) for k in fds[l])
    scale = sum(np.abs(L[l][H.valid[l]]).sum() * H.levels[l].h ** 2 for l in range(H.nlev))
    assert abs(vol - bnd) < 1e-13 * scale


def corner(bc):
    # a fine box in a corner of the domain (interpolation windows shifted
    # along both directions next to it)
    return amr.Hierarchy((16, 8), 1.0 / 16, [[((0, 0), (15, 7))], [((0, 0), (7, 7))]],
                         {(d, s): bc for d in range(2) for s in (0, 1)})


def corner_r4(bc):
    return amr.Hierarchy((8, 8), 1.0 / 8, [[((0, 0), (7, 7))], [((0, 0), (15, 15))]],
                         {(d, s): bc for d in range(2) for s in (0, 1)}, ratio=4)


@pytest.mark.parametrize("make", [two_level, corner, corner_r4])
@pytest.mark.parametrize("op,bc,c", [("helmholtz", "D", 0.3 / 16), ("poisson", "N", 0.0), ("poisson", "D", 0.0)])
def test_composite_solve_equals_direct_solve(make, op, bc, c):
    H = make(bc)
    rng = np.random.default_rng(4)
    fs = []
    for lev in H.levels:
        f = lev.zeros()
        f[lev.mask] = rng.normal(size=lev.ncells)
        fs.append(f)
    U, st = amr.composite_solve(H, fs, op, c, None, tol_rel=1e-13, max_cycles=120)
    Ud = amr.composite_direct(H, fs, op, c, None)
    assert rel(U, Ud, H) < 1e-10


def test_nesting_is_checked():
    with pytest.raises(ValueError):  # not properly refined for ratio 4
        amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((18, 16), (41, 47))]],
                      {(d, s): "D" for d in range(2) for s in (0, 1)}, ratio=4)
    with pytest.raises(ValueError):
        amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((4, 4), (11, 11))], [((2, 2), (9, 9))]],
                      {(d, s): "D" for d in range(2) for s in (0, 1)})
