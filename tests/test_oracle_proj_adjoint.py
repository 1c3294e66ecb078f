"""Pins of the oracle's transposed gradient, divergence and projection
(oracle/proj_adj.py) against the forward operators of oracle/proj.py, which
are pinned on their own (exactness on polynomials, conservation):

* the dot-product identity <A x, y> = <x, A^T y> over the cells of a level
  (two boxes: exchange ghosts; a refined level with face-data ghosts) and
  over the valid cells of two- and three-level hierarchies (interpolated
  ghosts, refluxing of the divergence, average-down);
* equality with the transpose of the probe-assembled matrix of the forward
  operator on a small layout;
* the projection: <P w, u> = <w, P^T u> with the pure-Neumann solves done to
  a tight tolerance, on a level and over a hierarchy.

A transposed operator that dropped a ghost term, flipped a sign or read the
wrong side fails the identities (checked by perturbing the result)."""
import numpy as np
import pytest

from oracle import amr, proj, proj_adj
from oracle.level import Level


def level(name):
    if name == "box":
        return Level((16, 16), 1 / 16, [((0, 0), (15, 15))], {(d, s): "D" for d in range(2) for s in (0, 1)})
    if name == "two_boxes":
        return Level((16, 16), 1 / 16, [((0, 0), (7, 15)), ((8, 0), (15, 15))],
                     {(d, s): "D" for d in range(2) for s in (0, 1)})
    if name == "refined":  # face-data ghosts on the coarse-fine faces
        return Level((32, 32), 1 / 32, [((4, 8), (19, 23)), ((20, 8), (27, 15))],
                     {(d, s): "D" for d in range(2) for s in (0, 1)}, "D")
    if name == "box3d":
        return Level((8, 8, 8), 1 / 8, [((0, 0, 0), (7, 7, 7))], {(d, s): "D" for d in range(3) for s in (0, 1)})
    raise KeyError(name)


def rand(lev, rng):
    return np.where(lev.mask, rng.normal(size=lev.pshape), 0.0)


def cdot(lev, a, b):
    return float((a[lev.mask] * b[lev.mask]).sum())


NAMES = ["box", "two_boxes", "refined", "box3d"]


@pytest.mark.parametrize("name", NAMES)
def test_level_gradient_and_divergence_transposes(name):
    rng = np.random.default_rng(1)
    lev = level(name)
    lw, lp = proj.velocity_level(lev), proj.pressure_level(lev)
    D = lev.dim
    # G (phi's Neumann fill) and its transpose
    phi = rand(lp, rng)
    mu = [rand(lp, rng) for _ in range(D)]
    g = proj.gradient(lp, phi)
    lhs = sum(cdot(lp, g[d], mu[d]) for d in range(D))
    gt = proj_adj.gradient_T(lp, mu)
    rhs = cdot(lp, phi, gt)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0) * lev.ncells
    # D (the velocity's Dirichlet fill) and its transpose
    w = [rand(lw, rng) for _ in range(D)]
    lam = rand(lw, rng)
    lhs = cdot(lw, proj.divergence(lw, w), lam)
    dt = proj_adj.divergence_T(lw, lam)
    rhs = sum(cdot(lw, w[d], dt[d]) for d in range(D))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0) * lev.ncells
    # a perturbed transpose (one corner cell off) breaks the identity
    lhs_g = sum(cdot(lp, g[d], mu[d]) for d in range(D))
    bad = gt.copy()
    idx = tuple(np.argwhere(lp.mask)[0])
    bad[idx] += 0.1 * np.abs(gt).max()
    assert abs(lhs_g - cdot(lp, phi, bad)) > 1e-6 * (abs(lhs_g) + 1.0)


def _assemble(lev, fn, nin, nout):
    """Dense matrix of a linear map from nin fields on lev's cells to nout
    fields, by probing with unit vectors."""
    cells = np.argwhere(lev.mask)
    n = len(cells)
    M = np.zeros((nout * n, nin * n))
    for k in range(nin):
        for j, c in enumerate(cells):
            x = [lev.zeros() for _ in range(nin)]
            x[k][tuple(c)] = 1.0
            y = fn(x)
            M[:, k * n + j] = np.concatenate([y[m][lev.mask] for m in range(nout)])
    return M


def test_transposes_equal_the_probed_matrices():
    lev = Level((8, 8), 1 / 8, [((0, 0), (7, 7))], {(d, s): "D" for d in range(2) for s in (0, 1)})
    lw, lp = proj.velocity_level(lev), proj.pressure_level(lev)
    G = _assemble(lp, lambda x: proj.gradient(lp, x[0]), 1, 2)
    GT = _assemble(lp, lambda x: [proj_adj.gradient_T(lp, x)], 2, 1)
    assert np.abs(GT - G.T).max() < 1e-12 * np.abs(G).max()
    Dm = _assemble(lw, lambda x: [proj.divergence(lw, x)], 2, 1)
    DT = _assemble(lw, lambda x: proj_adj.divergence_T(lw, x[0]), 1, 2)
    assert np.abs(DT - Dm.T).max() < 1e-12 * np.abs(Dm).max()


def test_level_projection_transpose():
    rng = np.random.default_rng(2)
    lev = Level((16, 16), 1 / 16, [((0, 0), (15, 15))], {(d, s): "D" for d in range(2) for s in (0, 1)})
    w = [rand(lev, rng) for _ in range(2)]
    ub = [rand(lev, rng) for _ in range(2)]
    U, _, st = proj.project(lev, w, tol_rel=1e-14, max_cycles=300)
    assert st["converged"]
    PT, _, st = proj_adj.project_T(lev, ub, tol_rel=1e-14, max_cycles=300)
    assert st["converged"]
    lhs = sum(cdot(lev, U[d], ub[d]) for d in range(2))
    rhs = sum(cdot(lev, w[d], PT[d]) for d in range(2))
    assert abs(lhs - rhs) <= 1e-10 * sum(np.abs(w[d]).sum() for d in range(2))


HIERS = {
    "two_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((8, 8), (15, 23)), ((16, 8), (23, 15))]]),
    "three_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((4, 4), (27, 27))], [((16, 16), (31, 31))]]),
    "boundary": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((0, 0), (15, 15)), ((16, 0), (23, 11))]]),
    "two_level_r4": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((16, 16), (39, 47)), ((40, 16), (47, 31))]], 4),
}


def hier(name, kind):
    base, h0, boxes, *ratio = HIERS[name]
    return amr.Hierarchy(base, h0, boxes, {(d, s): kind for d in range(2) for s in (0, 1)}, *ratio)


def rand_levels(H, rng, valid=True):
    return [np.where(H.valid[l] if valid else H.levels[l].mask, rng.normal(size=lev.pshape), 0.0)
            for l, lev in enumerate(H.levels)]


@pytest.mark.parametrize("name", sorted(HIERS))
def test_composite_gradient_and_divergence_transposes(name):
    rng = np.random.default_rng(3)
    Hp, Hw = hier(name, "N"), hier(name, "D")
    D = Hp.dim
    phi = rand_levels(Hp, rng)
    mu = [rand_levels(Hp, rng) for _ in range(D)]
    G = proj.composite_gradient(Hp, phi)
    lhs = sum(proj_adj.valid_dot(Hp, G[d], mu[d]) for d in range(D))
    rhs = proj_adj.valid_dot(Hp, phi, proj_adj.composite_gradient_T(Hp, mu))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0) * 1e3
    w = [rand_levels(Hw, rng) for _ in range(D)]
    lam = rand_levels(Hw, rng)
    Dw = proj.composite_divergence(Hw, w)
    lhs = proj_adj.valid_dot(Hw, Dw, lam)
    DT = proj_adj.composite_divergence_T(Hw, lam)
    rhs = sum(proj_adj.valid_dot(Hw, w[d], DT[d]) for d in range(D))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0) * 1e3
    # covered cells of the input do not matter to the forward (averaged
    # down first), and the transpose is zero there
    for d in range(D):
        for l in range(Hw.nlev):
            assert np.all(DT[d][l][~Hw.valid[l]] == 0.0)


@pytest.mark.parametrize("name", ["two_level", "three_level", "two_level_r4"])
def test_composite_projection_transpose(name):
    rng = np.random.default_rng(4)
    H = hier(name, "D")
    w = [rand_levels(H, rng) for _ in range(2)]
    ub = [rand_levels(H, rng) for _ in range(2)]
    U, _, st = proj.composite_project(H, w, tol_rel=1e-13, max_cycles=400)
    assert st["converged"]
    PT, _, st = proj_adj.composite_project_T(H, ub, tol_rel=1e-13, max_cycles=400)
    assert st["converged"]
    lhs = sum(proj_adj.valid_dot(H, U[d], ub[d]) for d in range(2))
    rhs = sum(proj_adj.valid_dot(H, w[d], PT[d]) for d in range(2))
    scale = sum(np.abs(w[d][l]).sum() for d in range(2) for l in range(H.nlev))
    assert abs(lhs - rhs) <= 1e-9 * scale
