"""Pins of the oracle's ILU(0)-preconditioned GMRES(m) bottom solver
(oracle/mg.py: ilu0, gmres_right, IluGmresBottom; the bottom solver of the
pressure systems in Section 6.5, after Saad's Iterative Methods, Alg. 9.5
and 10.4):

* ILU(0) on a matrix whose pattern admits no fill (tridiagonal, diagonally
  dominant: no pivoting either) equals the complete LU factorisation from
  scipy;
* ILU(0)'s defining property on the bottom matrices of 2D and 3D levels
  (Neumann bordered, Dirichlet, several boxes): (L U)_ij = K_ij on the
  pattern;
* GMRES with as many steps as unknowns is the direct solve; m steps give
  the smallest residual over the preconditioned Krylov space, computed by
  brute force (its explicit power basis, orthonormalised, least squares);
  the residual does not grow with m;
* inside the multigrid: solves with the GMRES bottom reach the solutions of
  the exact-bottom solves, and five GMRES steps keep the V-cycle's
  reduction close to the exact bottom's (the paper reports three to five
  steps suffice).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import mg
from oracle.level import Level


def test_ilu0_without_fill_is_the_complete_lu():
    rng = np.random.default_rng(0)
    n = 12
    K = np.diag(4.0 + rng.random(n)) + np.diag(-rng.random(n - 1), 1) + np.diag(-rng.random(n - 1), -1)
    P, L, U = scipy.linalg.lu(K)
    assert np.array_equal(P, np.eye(n))
    LU = mg.ilu0(K)
    assert np.allclose(np.tril(LU, -1), np.tril(L, -1), rtol=1e-14, atol=1e-15)
    assert np.allclose(np.triu(LU), U, rtol=1e-14, atol=1e-15)


def bottom_level(name):
    if name == "2d_neumann":
        return Level((8, 8), 1 / 8, [((0, 0), (7, 7))], {(d, s): "N" for d in range(2) for s in (0, 1)}), "poisson", 0.0
    if name == "2d_two_boxes":
        return (Level((16, 8), 1 / 16, [((0, 0), (7, 7)), ((8, 0), (15, 7))],
                      {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D"}), "helmholtz", 0.01)
    if name == "3d_dirichlet":
        return (Level((6, 6, 6), 1 / 6, [((0, 0, 0), (5, 5, 5))], {(d, s): "D" for d in range(3) for s in (0, 1)}),
                "poisson", 0.0)
    raise KeyError(name)


@pytest.mark.parametrize("name", ["2d_neumann", "2d_two_boxes", "3d_dirichlet"])
def test_ilu0_matches_the_matrix_on_its_pattern(name):
    lev, op, c = bottom_level(name)
    B = mg.IluGmresBottom(lev, op, c, 5)
    for idx, K, LU, sing in B.systems:
        L = np.tril(LU, -1) + np.eye(K.shape[0])
        U = np.triu(LU)
        pat = (np.abs(K) > 1e-12 * np.abs(K).max(axis=1, keepdims=True)) | np.eye(K.shape[0], dtype=bool)
        prod = L @ U
        assert np.abs(prod - K)[pat].max() < 1e-12 * np.abs(K).max()
        # and it is not the complete factorisation: fill outside the pattern
        assert np.abs(prod[~pat]).max() > 1e-6 * np.abs(K).max()
        assert sing == (op == "poisson" and name == "2d_neumann")


def test_gmres_with_n_steps_is_the_direct_solve():
    lev, op, c = bottom_level("2d_two_boxes")
    B = mg.IluGmresBottom(lev, op, c, 5)
    idx, K, LU, _ = B.systems[0]
    rng = np.random.default_rng(1)
    b = rng.normal(size=K.shape[0])
    x = mg.gmres_right(K, b, LU, K.shape[0])
    assert np.abs(x - np.linalg.solve(K, b)).max() < 1e-10 * np.abs(np.linalg.solve(K, b)).max()


@pytest.mark.parametrize("m", [1, 2, 3, 5])
def test_gmres_minimises_over_the_preconditioned_krylov_space(m):
    lev, op, c = bottom_level("2d_neumann")
    B = mg.IluGmresBottom(lev, op, c, m)
    idx, K, LU, sing = B.systems[0]
    rng = np.random.default_rng(2)
    b = rng.normal(size=K.shape[0])
    b[-1] = 0.0
    x = mg.gmres_right(K, b, LU, m)
    res = np.linalg.norm(b - K @ x)
    # brute force: C = K (LU)^-1, Krylov basis b, C b, ..., C^(m-1) b
    Lf = np.tril(LU, -1) + np.eye(K.shape[0])
    Uf = np.triu(LU)
    C = K @ np.linalg.solve(Uf, np.linalg.solve(Lf, np.eye(K.shape[0])))
    W = np.zeros((K.shape[0], m))
    v = b.copy()
    for j in range(m):
        W[:, j] = v
        v = C @ v
    Q, _ = np.linalg.qr(W)
    y = np.linalg.lstsq(C @ Q, b, rcond=None)[0]
    best = np.linalg.norm(b - C @ Q @ y)
    assert abs(res - best) <= 1e-9 * np.linalg.norm(b)
    if m > 1:
        prev = np.linalg.norm(b - K @ mg.gmres_right(K, b, LU, m - 1))
        assert res <= prev * (1 + 1e-12)


@pytest.mark.parametrize("name", ["2d_neumann_16", "2d_cf"])
def test_multigrid_with_the_gmres_bottom(name):
    if name == "2d_neumann_16":
        lev = Level((32, 32), 1 / 32, [((0, 0), (31, 31))], {(d, s): "N" for d in range(2) for s in (0, 1)})
        op, c = "poisson", 0.0
    else:  # coarse-fine Neumann faces, two components
        lev = Level((32, 32), 1 / 32, [((0, 4), (15, 11)), ((16, 4), (23, 19)), ((4, 20), (11, 27))],
                    {(d, s): "N" for d in range(2) for s in (0, 1)}, "N")
        op, c = "poisson", 0.0
    rng = np.random.default_rng(3)
    f = np.where(lev.mask, rng.normal(size=lev.pshape), 0.0)
    sing = lev.singular_components(op)
    x_ex, st_ex = mg.solve(lev, f, op, c, smoother="rb", tol_rel=1e-11, max_cycles=100)
    M = mg.MG(lev, op, c, smoother="rb", bottom="ilu_gmres", bottom_iters=5)
    x_gm, st_gm = mg.solve(lev, f, op, c, smoother="rb", tol_rel=1e-11, max_cycles=100, mg=M)
    assert st_ex["converged"] and st_gm["converged"]
    want = lev.comp_mean(x_ex, sing)
    got = lev.comp_mean(x_gm, sing)
    assert np.abs(got - want)[lev.mask].max() < 1e-9 * np.abs(want).max()
    # five steps keep the cycle count within a few of the exact bottom's
    assert st_gm["cycles"] <= st_ex["cycles"] + 3, (st_gm["cycles"], st_ex["cycles"])
