"""Pins of single smoothing sweeps and of the prolongation next to a face.

The smoothers are pinned against the textbook matrix forms, built in this
file from the probe-assembled matrix M of the homogeneous operator (whose
entries are pinned elsewhere: the printed Section 3 coefficients, the dense
solves and the folded diagonal):

* one weighted-Jacobi sweep (Section 6.5, omega = 2/3) is
  e + omega diag(M)^-1 (f - M e), with every cell reading the old iterate;
* one red-black sweep updates the cells whose global index sum is even
  (red) from e, then the odd (black) cells from the red-updated vector.

The colour sets come from the cells' global indices computed here, and a
box whose lower corner is odd makes the global parity differ from the
box-local one.  Each pin also checks that the plausible mistakes (black
first, a stale red half, omega on the wrong term) give a different result,
so the comparison has the power to catch them.

The prolongation (reading: face-neighbour linear interpolation) of a coarse
correction next to a physical face reads the first ghost layer of the
homogeneous fill (eqs. velBCHomoDiri5th and Neumann5).  That fill is exact
for cell averages of polynomials of degree <= 4 along the row whose datum
vanishes, so for such a polynomial p the child next to the face must equal
(1 - D/4) pbar_P + 1/4 sum_d pbar_(n_d), where the neighbour n_d beyond the
face is the exact average of p over the cell outside the domain.  Using the
second ghost layer, or a wrong fill, changes the value.
"""
import itertools

import numpy as np
import pytest

from oracle import mg
from oracle.level import PAD, Level
from tests.polyfix import Poly1


def unit_level(n, D, bc, boxes=None, shape=None):
    shape = shape or (n,) * D
    boxes = boxes or [((0,) * D, tuple(m - 1 for m in shape))]
    return Level(shape, 1.0 / n, boxes, {(d, s): bc for d in range(D) for s in (0, 1)})


def rand_cells(lev, seed):
    u = lev.zeros()
    u[lev.mask] = np.random.default_rng(seed).normal(size=lev.ncells)
    return u


LAYOUTS = [
    # one box, Dirichlet, Helmholtz
    ("helmholtz", lambda: unit_level(12, 2, "D")),
    # two boxes with a gap, one of them with an odd lower corner, Neumann
    ("poisson", lambda: unit_level(16, 2, "N", boxes=[((0, 0), (6, 15)), ((9, 3), (15, 12))])),
    # a box off the domain faces (coarse-fine faces of Dirichlet kind), odd corner
    ("poisson", lambda: Level((16, 16), 1 / 16, [((3, 5), (10, 14))],
                              {(d, s): "N" for d in range(2) for s in (0, 1)}, cf_kind="D")),
    # 3D, Neumann, Helmholtz
    ("helmholtz", lambda: unit_level(6, 3, "N")),
]


def _matrix(lev, op, c, transpose):
    M, cells = mg.assemble(lev, op, c)
    return (M.T.copy() if transpose else M), cells


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("case", range(len(LAYOUTS)))
def test_weighted_jacobi_sweep_is_the_matrix_form(case, transpose):
    op, mk = LAYOUTS[case]
    lev = mk()
    c = 0.3 * lev.h if op == "helmholtz" else 0.0
    M, _ = _matrix(lev, op, c, transpose)
    dg = np.diag(M)
    e, f = rand_cells(lev, 1), rand_cells(lev, 2)
    w = 2.0 / 3.0
    ev, fv = e[lev.mask], f[lev.mask]
    want = ev.copy()
    for _ in range(2):
        want = want + w * (fv - M @ want) / dg
    got = mg.jacobi(lev, e, f, op, c, lev.diagonal(op, c), w, 2, transpose=transpose)
    scale = np.abs(want).max()
    assert np.abs(got[lev.mask] - want).max() <= 1e-12 * scale
    assert np.all(got[~lev.mask] == 0.0)
    # omega applied to the whole update instead of the correction differs
    wrong = w * (ev + (fv - M @ ev) / dg)
    assert np.abs(wrong - mg.jacobi(lev, e, f, op, c, lev.diagonal(op, c), w, 1, transpose)[lev.mask]).max() > 1e-3


def _rb_matrix_form(M, ev, fv, red, sweeps, omega=1.0, order=(True, False), stale=False):
    dg = np.diag(M)
    e = ev.copy()
    for _ in range(sweeps):
        base = e.copy()
        for colour in order:
            sel = red if colour else ~red
            src = base if stale else e
            r = fv - M @ src
            e = e.copy()
            e[sel] = e[sel] + omega * r[sel] / dg[sel]
    return e


@pytest.mark.parametrize("transpose", [False, True])
@pytest.mark.parametrize("case", range(len(LAYOUTS)))
def test_red_black_sweep_is_the_matrix_form(case, transpose):
    op, mk = LAYOUTS[case]
    lev = mk()
    c = 0.3 * lev.h if op == "helmholtz" else 0.0
    M, cells = _matrix(lev, op, c, transpose)
    red = ((cells - PAD).sum(axis=1) % 2) == 0
    e, f = rand_cells(lev, 3), rand_cells(lev, 4)
    ev, fv = e[lev.mask], f[lev.mask]
    D = lev.diagonal(op, c)
    for omega in (1.0, 1.3):
        want = _rb_matrix_form(M, ev, fv, red, 2, omega)
        got = mg.red_black(lev, e, f, op, c, D, 2, transpose=transpose, omega=omega)
        scale = np.abs(want).max()
        assert np.abs(got[lev.mask] - want).max() <= 1e-12 * scale
    # the comparison separates the plausible misreadings
    ref = _rb_matrix_form(M, ev, fv, red, 1)
    for bad in (_rb_matrix_form(M, ev, fv, red, 1, order=(False, True)),
                _rb_matrix_form(M, ev, fv, red, 1, stale=True),
                _rb_matrix_form(M, ev, fv, ~red, 1)):
        assert np.abs(bad - ref).max() > 1e-6 * np.abs(ref).max()


def test_colours_follow_global_indices():
    """A box with an odd lower corner: its first cell (local 0, 0) is black."""
    lev = unit_level(16, 2, "D", boxes=[((3, 4), (10, 11))])
    col = lev.colour()
    assert not col[PAD + 3, PAD + 4] and col[PAD + 4, PAD + 4] and col[PAD + 3, PAD + 5]


# ----------------------------------------------------------------------
# prolongation next to a face

def _avg(poly, lo, h):
    return float(poly.avg(lo, h, 1)[0])


def _poly_for(kind, s):
    """A 1-D polynomial of degree <= 4 whose homogeneous datum vanishes on the
    face x = 0 (s = 0) or x = 1 (s = 1)."""
    t = Poly1([0.0, 1.0]) if s == 0 else Poly1([1.0, -1.0])  # distance to the face
    if kind == "D":
        # t (0.7 + 1.3 t - 0.9 t^2): zero at the face
        return _compose(t, [0.0, 0.7, 1.3, -0.9])
    # 0.4 + 1.1 t^2 - 0.5 t^3 + 0.2 t^4: zero derivative at the face
    return _compose(t, [0.4, 0.0, 1.1, -0.5, 0.2])


def _compose(t, coef):
    """sum_k coef[k] t(x)^k for a linear t, as a Poly1 in x."""
    out = np.zeros(len(coef))
    a, b = t.c  # t = a + b x
    for k, ck in enumerate(coef):
        # (a + b x)^k by the binomial theorem
        for j in range(k + 1):
            out[j] += ck * _binom(k, j) * a ** (k - j) * b ** j
    return Poly1(out)


def _binom(n, k):
    from math import comb
    return comb(n, k)


@pytest.mark.parametrize("D", [2, 3])
@pytest.mark.parametrize("kind", ["D", "N"])
def test_prolongation_next_to_a_face_reads_the_first_homogeneous_ghost(D, kind):
    n = 8
    coarse = unit_level(n, D, kind)
    fine = unit_level(2 * n, D, kind)
    H = coarse.h
    other = Poly1([0.3, 0.8, -0.6])  # any smooth profile along the other directions
    for d, s in itertools.product(range(D), (0, 1)):
        p = _poly_for(kind, s)
        ec = coarse.zeros()
        prof = [p if dd == d else other for dd in range(D)]
        avgs = [q.avg(0.0, H, n) for q in prof]
        grid = avgs[0]
        for a in avgs[1:]:
            grid = np.multiply.outer(grid, a)
        ec[coarse.inner] = grid
        pf = mg.prolong(coarse, ec, fine)
        i_face = 0 if s == 0 else n - 1
        # parents next to face (d, s), away from every other face
        for rest in itertools.product(range(2, n - 2), repeat=D - 1):
            P = list(rest)
            P.insert(d, i_face)
            for corner in itertools.product((0, 1), repeat=D):
                if corner[d] != s:
                    continue  # the child on the face's side reads the ghost
                val = (1.0 - D / 4.0) * ec[tuple(PAD + i for i in P)]
                for dd in range(D):
                    k = 1 if corner[dd] == 1 else -1
                    if dd == d:
                        # the coarse cell beyond the face: exact average of p there
                        lo = (P[dd] + k) * H
                        nb = _avg(prof[dd], lo, H)
                        for e2 in range(D):
                            if e2 != dd:
                                nb *= _avg(prof[e2], P[e2] * H, H)
                    else:
                        Q = list(P)
                        Q[dd] += k
                        nb = ec[tuple(PAD + i for i in Q)]
                    val += 0.25 * nb
                child = tuple(PAD + 2 * P[dd] + corner[dd] for dd in range(D))
                assert abs(pf[child] - val) <= 1e-13 * max(1.0, abs(val)), (d, s, P, corner)
    # the second ghost layer (the cell two beyond the face) gives another value
    p = _poly_for(kind, 0)
    assert abs(_avg(p, -H, H) - _avg(p, -2 * H, H)) > 1e-3
