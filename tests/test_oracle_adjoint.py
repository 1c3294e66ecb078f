"""Pins of the oracle's adjoint (transposed) level operator and adjoint solve
against the forward operator, which is pinned on its own: the dot-product
identity <A u, lam> = <u, A^T lam> on every kind of ghost (physical
Dirichlet and Neumann, coarse-fine face data, box-to-box exchange across
touching boxes and across gaps, interpolated coarse-fine ghosts), the
probe-assembled matrix, <A^-1 f, g> = <f, A^-T g> for the solves (pure
Neumann included), and the derivative with respect to the Helmholtz
coefficient against central finite differences."""
import numpy as np
import pytest

from oracle import mg
from oracle.level import Level


def full(n, D, bc):
    return Level((n,) * D, 1.0 / n, [((0,) * D, (n - 1,) * D)], {(d, s): bc for d in range(D) for s in (0, 1)})


MIXED = {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D"}


def layouts():
    out = {
        "2d_D": full(12, 2, "D"),
        "2d_N": full(12, 2, "N"),
        "2d_mixed": Level((12, 12), 1 / 12, [((0, 0), (11, 11))], MIXED),
        "3d_D": full(8, 3, "D"),
        "3d_N": full(8, 3, "N"),
        # two touching boxes (exchange) + a box across a one-cell gap
        "gap1_N": Level((24, 12), 1 / 24, [((0, 0), (7, 11)), ((8, 0), (13, 7)), ((15, 0), (22, 7))],
                        {(d, s): "N" for d in range(2) for s in (0, 1)}, "N"),
        # boxes inside the domain with coarse-fine face data (D and N)
        "cf_D": Level((24, 24), 1 / 24, [((4, 4), (11, 15)), ((12, 4), (19, 11))],
                      {(d, s): "N" for d in range(2) for s in (0, 1)}, "D"),
        "cf_N": Level((24, 24), 1 / 24, [((4, 4), (11, 15)), ((12, 4), (19, 11))],
                      {(d, s): "D" for d in range(2) for s in (0, 1)}, "N"),
        # interpolated coarse-fine ghosts (homogeneous: zero)
        "cf_I": Level((24, 24), 1 / 24, [((0, 4), (11, 15)), ((12, 4), (19, 11))],
                      {(d, s): "D" for d in range(2) for s in (0, 1)}, "I"),
        # gap of two and three cells between facing boxes
        "gap23_D": Level((30, 10), 1 / 30, [((0, 0), (5, 9)), ((8, 0), (13, 9)), ((17, 2), (22, 7))],
                         {(d, s): "D" for d in range(2) for s in (0, 1)}, "N"),
    }
    return out


LAY = layouts()


def rand_cells(lev, rng):
    u = lev.zeros()
    u[lev.mask] = rng.normal(size=lev.ncells)
    return u


def dot(a, b, lev):
    return float((a[lev.mask] * b[lev.mask]).sum())


@pytest.mark.parametrize("name", sorted(LAY))
@pytest.mark.parametrize("op,c", [("helmholtz", 0.37), ("poisson", 0.0)])
def test_dot_product_identity(name, op, c):
    lev = LAY[name]
    rng = np.random.default_rng(sum(map(ord, name)))
    c = c * lev.h  # c / h^2 of order 1/h: both parts of I - cL matter
    for _ in range(3):
        u, lam = rand_cells(lev, rng), rand_cells(lev, rng)
        lhs = dot(lev.apply(u, op, c), lam, lev)
        rhs = dot(u, lev.apply_T(lam, op, c), lev)
        scale = np.abs(lev.apply(u, op, c)[lev.mask]).sum() * np.abs(lam).max()
        assert abs(lhs - rhs) < 1e-14 * scale


@pytest.mark.parametrize("name", ["2d_mixed", "gap1_N", "cf_N", "cf_I"])
def test_transpose_equals_probed_matrix_transpose(name):
    lev = LAY[name]
    M, cells = mg.assemble(lev, "helmholtz", 0.2 * lev.h)
    MT = np.zeros_like(M)
    for j, cell in enumerate(cells):
        e = lev.zeros()
        e[tuple(cell)] = 1.0
        col = lev.apply_T(e, "helmholtz", 0.2 * lev.h)
        MT[:, j] = col[lev.mask]
        assert np.all(col[~lev.mask] == 0.0)
    assert np.abs(MT - M.T).max() < 1e-12 * np.abs(M).max()


def test_transpose_differs_from_operator():
    # the folded boundary rows make A non-symmetric: the pin above would not
    # notice an apply_T that returned A itself unless A != A^T here
    lev = LAY["2d_D"]
    M, _ = mg.assemble(lev, "poisson", 0.0)
    assert np.abs(M - M.T).max() > 1e-3 * np.abs(M).max()


@pytest.mark.parametrize("name,op", [("2d_D", "helmholtz"), ("2d_N", "poisson"), ("2d_mixed", "poisson"),
                                     ("3d_N", "poisson"), ("cf_N", "poisson"), ("gap1_N", "helmholtz")])
@pytest.mark.parametrize("smoother", ["jacobi", "rb"])
def test_adjoint_solve_identity(name, op, smoother):
    lev = LAY[name]
    c = 0.3 * lev.h if op == "helmholtz" else 0.0
    rng = np.random.default_rng(7)
    f, g = rand_cells(lev, rng), rand_cells(lev, rng)
    u, st = mg.solve(lev, f, op, c, tol_rel=1e-13, max_cycles=200, smoother=smoother)
    lam, sta = mg.solve(lev, g, op, c, tol_rel=1e-13, max_cycles=200, smoother=smoother, transpose=True)
    assert st["converged"] and sta["converged"]
    lhs, rhs = dot(u, g, lev), dot(f, lam, lev)
    assert abs(lhs - rhs) < 1e-10 * np.abs(u).max() * np.abs(g).sum()
    # the adjoint solution solves the transposed system (mean-free source on
    # singular components)
    sing = lev.singular_components(op)
    gs = lev.comp_mean(g, sing)
    assert np.abs(lev.apply_T(lam, op, c) - gs)[lev.mask].max() < 1e-11 * np.abs(gs).max() * 10
    if sing:
        assert np.abs(lev.comp_mean(lam, sing) - lam).max() < 1e-13 * np.abs(lam).max()


def test_adjoint_direct_solve():
    # the adjoint solve equals numpy's dense solve with the transposed matrix
    lev = LAY["cf_D"]
    c = 0.25 * lev.h
    M, cells = mg.assemble(lev, "helmholtz", c)
    rng = np.random.default_rng(3)
    g = rand_cells(lev, rng)
    lam, st = mg.solve(lev, g, "helmholtz", c, tol_rel=1e-14, max_cycles=200, transpose=True)
    want = np.linalg.solve(M.T, g[lev.mask])
    assert np.abs(lam[lev.mask] - want).max() < 1e-11 * np.abs(want).max()


@pytest.mark.parametrize("name", ["2d_D", "2d_mixed", "cf_N"])
def test_grad_c_matches_finite_differences(name):
    lev = LAY[name]
    rng = np.random.default_rng(11)
    f = rand_cells(lev, rng)
    t = rand_cells(lev, rng)
    fd = lev.zero_face_data()
    for k in fd:
        e = lev.row_end(*k)
        fd[k][e] = rng.normal(size=int(e.sum()))
    c = 0.4 * lev.h

    def J(cc):
        u, st = mg.solve(lev, f, "helmholtz", cc, fd, tol_rel=1e-14, max_cycles=200)
        return 0.5 * float(((u - t)[lev.mask] ** 2).sum()), u

    J0, u = J(c)
    lam, _ = mg.solve(lev, u - t, "helmholtz", c, tol_rel=1e-14, max_cycles=200, transpose=True)
    g = mg.grad_c(lev, lam, u, fd)
    eps = 1e-6 * c
    fdiff = (J(c + eps)[0] - J(c - eps)[0]) / (2 * eps)
    assert abs(g - fdiff) < 1e-6 * abs(fdiff)
    # and the gradient with respect to f is lam: a linear functional's
    # derivative along a random direction
    v = rand_cells(lev, rng)
    du = mg.solve(lev, v, "helmholtz", c, tol_rel=1e-14, max_cycles=200)[0]  # homogeneous part: no fd
    assert abs(dot(u - t, du, lev) - dot(lam, v, lev)) < 1e-9 * np.abs(lam).max() * np.abs(v).sum()


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("poisson", "N")])
def test_adjoint_vcycle_contracts(op, bc):
    lev = full(32, 2, bc)
    c = 0.5 * lev.h if op == "helmholtz" else 0.0
    g = rand_cells(lev, np.random.default_rng(5))
    _, st = mg.solve(lev, g, op, c, tol_rel=1e-12, max_cycles=60, transpose=True, smoother="rb")
    h = np.array(st["history"])
    assert st["converged"]
    assert np.max(h[1:] / h[:-1]) < 0.3
