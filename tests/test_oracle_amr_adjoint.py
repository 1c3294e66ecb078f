"""Pins of the oracle's transposed composite operator and composite adjoint
solve against the forward composite operator and solve, which are pinned on
their own: the dot-product identity on two- and three-level hierarchies
(interpolated ghosts, refluxing, average-down, physical fills), equality with
the transpose of the probe-assembled composite matrix, <A^-1 f, g> =
<f, A^-T g> for the solves (pure Neumann included), and the derivative in
the Helmholtz coefficient against central finite differences."""
import numpy as np
import pytest

from oracle import amr, amr_adj

LAYOUTS = {
    "two_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((8, 8), (15, 23)), ((16, 8), (23, 15))]]),
    "three_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((4, 4), (27, 27))], [((16, 16), (31, 31))]]),
    "corner": ((16, 8), 1 / 16, [[((0, 0), (15, 7))], [((0, 0), (7, 7))]]),
    "boundary": ((32, 16), 1 / 32, [[((0, 0), (15, 15)), ((16, 0), (31, 15))],
                                   [((0, 0), (15, 15)), ((16, 0), (23, 11))]]),
    "two_level_r4": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((16, 16), (39, 47)), ((40, 16), (47, 31))]], 4),
    "three_level_r4": ((8, 8), 1 / 8, [[((0, 0), (7, 7))], [((8, 8), (23, 23))], [((48, 48), (79, 79))]], 4),
}
CASES = [("D", "helmholtz", 0.3), ("N", "poisson", 0.0), ("D", "poisson", 0.0), ("N", "helmholtz", 0.5)]


def hier(name, bc):
    base, h0, boxes, *ratio = LAYOUTS[name]
    return amr.Hierarchy(base, h0, boxes, {(d, s): bc for d in range(2) for s in (0, 1)}, *ratio)


def rand_valid(H, rng):
    return [np.where(H.valid[l], rng.normal(size=lev.pshape), 0.0) for l, lev in enumerate(H.levels)]


def vdot(H, a, b):
    return float(sum((a[l] * b[l])[H.valid[l]].sum() for l in range(H.nlev)))


@pytest.mark.parametrize("name", sorted(LAYOUTS))
@pytest.mark.parametrize("bc,op,c0", CASES)
def test_dot_product_identity(name, bc, op, c0):
    H = hier(name, bc)
    c = c0 * H.levels[0].h
    rng = np.random.default_rng(sum(map(ord, name)) + len(bc))
    for _ in range(2):
        u, lam = rand_valid(H, rng), rand_valid(H, rng)
        Au = H.composite_apply(H.average_down_all(u), op, c)
        lhs = vdot(H, Au, lam)
        rhs = vdot(H, u, amr_adj.composite_apply_T(H, lam, op, c))
        scale = sum(np.abs(Au[l][H.valid[l]]).sum() for l in range(H.nlev)) * max(np.abs(x).max() for x in lam)
        assert abs(lhs - rhs) < 1e-14 * scale


def test_transpose_equals_probed_matrix_transpose():
    H = hier("corner", "N")
    c = 0.2 / 16
    cells = [(l, tuple(p)) for l in range(H.nlev) for p in np.argwhere(H.valid[l])]
    n = len(cells)

    def vec(k):
        U = [lev.zeros() for lev in H.levels]
        l, p = cells[k]
        U[l][p] = 1.0
        return U
    M = np.zeros((n, n))
    MT = np.zeros((n, n))
    for j in range(n):
        A = H.composite_apply(H.average_down_all(vec(j)), "helmholtz", c)
        M[:, j] = [A[l][p] for l, p in cells]
        B = amr_adj.composite_apply_T(H, vec(j), "helmholtz", c)
        MT[:, j] = [B[l][p] for l, p in cells]
    assert np.abs(MT - M.T).max() < 1e-12 * np.abs(M).max()
    assert np.abs(M - M.T).max() > 1e-3 * np.abs(M).max()  # not symmetric: the pin has teeth


@pytest.mark.parametrize("name,bc,op,c0", [("two_level", "D", "helmholtz", 0.3), ("three_level", "N", "poisson", 0.0),
                                           ("two_level_r4", "N", "poisson", 0.0), ("three_level_r4", "D", "helmholtz", 0.3),
                                          ("three_level", "D", "helmholtz", 0.3), ("corner", "D", "poisson", 0.0),
                                          ("boundary", "N", "poisson", 0.0)])
def test_adjoint_solve_identity(name, bc, op, c0):
    H = hier(name, bc)
    c = c0 * H.levels[0].h
    rng = np.random.default_rng(5)
    f, g = rand_valid(H, rng), rand_valid(H, rng)
    u, st = amr.composite_solve(H, f, op, c, None, tol_rel=1e-13, max_cycles=200)
    lam, sta = amr_adj.composite_solve_T(H, g, op, c, tol_rel=1e-12, max_cycles=200)
    assert st["converged"] and sta["converged"]
    lhs, rhs = vdot(H, u, g), vdot(H, f, lam)
    assert abs(lhs - rhs) < 1e-9 * max(np.abs(x).max() for x in u) * sum(np.abs(x).sum() for x in g)
    h = np.array(sta["history"])
    assert np.max(h[1:] / h[:-1]) < 0.85


def test_grad_c_matches_finite_differences():
    H = hier("two_level", "D")
    rng = np.random.default_rng(7)
    f, t = rand_valid(H, rng), rand_valid(H, rng)
    fd = []
    for lev in H.levels:
        d = lev.zero_face_data()
        for k in d:
            e = lev.end_is_physical(*k)
            d[k][e] = rng.normal(size=int(e.sum()))
        fd.append(d)
    c = 0.4 / 16

    def J(cc):
        u, st = amr.composite_solve(H, f, "helmholtz", cc, fd, tol_rel=1e-14, max_cycles=300)
        return 0.5 * sum(((u[l] - t[l]) ** 2)[H.valid[l]].sum() for l in range(H.nlev)), u

    _, u = J(c)
    lam, _ = amr_adj.composite_solve_T(H, [u[l] - t[l] for l in range(H.nlev)], "helmholtz", c, tol_rel=1e-14,
                                       max_cycles=300)
    g = amr_adj.grad_c(H, lam, u, fd)
    eps = 1e-6 * c
    fdiff = (J(c + eps)[0] - J(c - eps)[0]) / (2 * eps)
    assert abs(g - fdiff) < 1e-6 * abs(fdiff)
