"""Exact-arithmetic pins of the oracle's stencils and ghost fills.

The truth here is the cell average of a polynomial, computed in rational
arithmetic from its antiderivative; the oracle's formulas (Section 3) are
evaluated on Fractions and must reproduce it exactly up to the degree the
paper's order claims imply, and must fail one degree higher (so a dropped
term or a wrong coefficient cannot pass)."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import fv
from oracle.level import Level, PAD


def mono_avg(k, i, h):
    """Average of x^k over [i h, (i+1) h]."""
    a, b = i * h, (i + 1) * h
    return (b ** (k + 1) - a ** (k + 1)) / ((k + 1) * h)


def mono_val(k, x):
    return x ** k


def mono_der(k, x):
    return k * x ** (k - 1) if k else Fr(0)


def mono_d2_avg(k, i, h):
    return k * (k - 1) * mono_avg(k - 2, i, h) if k >= 2 else Fr(0)


H = Fr(1, 3)


@pytest.mark.parametrize("k", range(0, 8))
def test_laplacian_exact_to_degree_5(k):
    i = 5
    u = [mono_avg(k, j, H) for j in range(i - 2, i + 3)]
    got = fv.laplacian_1d(*u, H)
    assert (got == mono_d2_avg(k, i, H)) == (k <= 5)


@pytest.mark.parametrize("k", range(0, 7))
def test_gradient_exact_to_degree_4(k):
    i = 4
    got = fv.gradient_1d(mono_avg(k, i - 2, H), mono_avg(k, i - 1, H), mono_avg(k, i + 1, H),
                         mono_avg(k, i + 2, H), H)
    want = (mono_val(k, (i + 1) * H) - mono_val(k, i * H)) / H  # average of the derivative
    assert (got == want) == (k <= 4)


@pytest.mark.parametrize("k", range(0, 7))
def test_face_value_and_derivative(k):
    i = 4
    u = [mono_avg(k, j, H) for j in (i - 1, i, i + 1, i + 2)]
    xf = (i + 1) * H
    assert (fv.face_value(*u) == mono_val(k, xf)) == (k <= 3)
    assert (fv.face_derivative(*u, H) == mono_der(k, xf)) == (k <= 4)


def _interior(k):
    # boundary face at x = 0 is the HIGH face of cell -1; interior cells -1..-4
    return [mono_avg(k, -1 - j, H) for j in range(4)]


@pytest.mark.parametrize("k", range(0, 7))
def test_dirichlet_fill_exact_to_degree_4(k):
    g1, g2 = fv.dirichlet_ghosts(*_interior(k), mono_val(k, Fr(0)))
    exact = (g1 == mono_avg(k, 0, H)) and (g2 == mono_avg(k, 1, H))
    assert exact == (k <= 4)


@pytest.mark.parametrize("k", range(0, 7))
def test_neumann_fill_exact_to_degree_4(k):
    g1, g2 = fv.neumann_ghosts(*_interior(k), mono_der(k, Fr(0)), H)
    exact = (g1 == mono_avg(k, 0, H)) and (g2 == mono_avg(k, 1, H))
    assert exact == (k <= 4)


@pytest.mark.parametrize("k", range(0, 7))
def test_dirichlet_face_derivative_exact_to_degree_4(k):
    got = fv.dirichlet_face_normal_derivative(*_interior(k), mono_val(k, Fr(0)), H)
    assert (got == mono_der(k, Fr(0))) == (k <= 4)


def test_neumann_fill_makes_boundary_flux_equal_data():
    # For arbitrary interior values, the 4th-order face flux through the
    # boundary face computed with the Neumann ghosts equals the datum: this is
    # what makes the discrete solvability sums telescope.
    rng = np.random.default_rng(1)
    for _ in range(20):
        u = [Fr(int(v), 7) for v in rng.integers(-50, 50, size=4)]
        gn = Fr(int(rng.integers(-30, 30)), 11)
        g1, g2 = fv.neumann_ghosts(*u, gn, H)
        assert fv.face_derivative(u[1], u[0], g1, g2, H) == gn


def test_dirichlet_fill_flux_equals_printed_face_derivative():
    # two independently printed formulas of Section 3 agree identically
    rng = np.random.default_rng(2)
    for _ in range(20):
        u = [Fr(int(v), 5) for v in rng.integers(-50, 50, size=4)]
        g = Fr(int(rng.integers(-30, 30)), 13)
        g1, g2 = fv.dirichlet_ghosts(*u, g)
        assert fv.face_derivative(u[1], u[0], g1, g2, H) == fv.dirichlet_face_normal_derivative(*u, g, H)


@pytest.mark.parametrize("bc,first,second", [("D", Fr(-1087, 12), Fr(-403, 12)),
                                              ("N", Fr(-29, 2), Fr(-309, 10))])
def test_folded_diagonal_matches_hand_derived_rationals(bc, first, second):
    """Diagonal of the 1-D Laplacian with the fill folded in, in units of
    1/(12 h^2), next to a boundary: derived by hand in rational arithmetic
    from the fill coefficients; the oracle obtains it by probing."""
    n, h = 16, 1.0 / 16
    lev = Level((n,), h, [((0,), (n - 1,))], {(0, 0): bc, (0, 1): bc})
    D = lev.diagonal("poisson", 0.0)[lev.inner] * 12 * h * h
    assert D[0] == pytest.approx(float(first), abs=1e-12)
    assert D[1] == pytest.approx(float(second), abs=1e-12)
    assert D[-1] == pytest.approx(float(first), abs=1e-12)
    assert D[-2] == pytest.approx(float(second), abs=1e-12)
    assert np.allclose(D[2:-2], -30.0)
