"""Pins of the oracle's periodic boundaries (oracle/level.py, kind 'P'; the
periodic domains of Section 7.3) against closed forms of the discrete
operators of eq. discreteOps on Fourier modes, which do not go through the
oracle's ghost code:

* on a periodic grid the stencils act on a mode exp(i theta.j) by their
  symbols: L by sum_d (32 cos theta_d - 2 cos 2 theta_d - 30) / (12 h^2),
  G_d and D by i (8 sin theta_d - sin 2 theta_d) / (6 h);
* the periodic Poisson and Helmholtz systems are diagonal in the discrete
  Fourier basis, so their solutions are FFT divisions by the symbol (the
  Poisson one with the zero mode set to zero);
* the approximate projection eq. appProj acts on a mode by
  I - g g^T / lambda (g the gradient symbol, lambda the Laplacian's);
* periodic in one direction, Dirichlet in the other: the operator
  separates into the periodic symbol plus a one-directional Dirichlet
  operator taken from a separate non-periodic level.

Also: the two-box level equals the one-box level (wrap across a box
boundary versus within a box), components join across the periodic side,
the transpose satisfies the dot-product identity and equals the probed
matrix's transpose, and a periodic ghost that is not a cell is rejected.
A wrap to the wrong cell (off by one, wrong side, second layer from the
first) breaks the eigen-relation at the boundary."""
import numpy as np
import pytest

from oracle import amr, mg, proj
from oracle.level import PAD, Level


def periodic_level(n, dim=2, boxes=None, h=None):
    boxes = boxes or [((0,) * dim, (n - 1,) * dim)]
    return Level((n,) * dim, h or 1.0 / n, boxes, {(d, s): "P" for d in range(dim) for s in (0, 1)})


def lap_symbol(theta, h):
    return sum((32 * np.cos(t) - 2 * np.cos(2 * t) - 30) / (12 * h * h) for t in theta)


def grad_symbol(t, h):
    return 1j * (8 * np.sin(t) - np.sin(2 * t)) / (6 * h)


def mode(lev, m):
    """exp(i theta.j) on the cells, theta_d = 2 pi m_d / n_d (padded)."""
    j = np.indices(lev.shape)
    theta = [2 * np.pi * m[d] / lev.shape[d] for d in range(lev.dim)]
    ph = sum(theta[d] * j[d] for d in range(lev.dim))
    out = np.zeros(lev.pshape, complex)
    out[lev.inner] = np.exp(1j * ph)
    return out, theta


@pytest.mark.parametrize("dim,n,m", [(2, 16, (1, 0)), (2, 16, (3, 5)), (2, 16, (8, 7)), (3, 8, (1, 2, 3))])
def test_laplacian_eigen_relation(dim, n, m):
    lev = periodic_level(n, dim)
    u, theta = mode(lev, m)
    lam = lap_symbol(theta, lev.h)
    for part in (np.real, np.imag):
        got = lev.apply(part(u), "poisson", 0.0)
        assert np.abs(got[lev.mask] - part(lam * u)[lev.mask]).max() < 1e-9 * abs(lam) + 1e-9


def test_two_boxes_equal_one_box():
    rng = np.random.default_rng(0)
    one = periodic_level(16)
    two = periodic_level(16, boxes=[((0, 0), (7, 15)), ((8, 0), (15, 15))])
    four = periodic_level(16, boxes=[((0, 0), (7, 7)), ((8, 0), (15, 7)), ((0, 8), (7, 15)), ((8, 8), (15, 15))])
    u = np.where(one.mask, rng.normal(size=one.pshape), 0.0)
    a = one.apply(u, "helmholtz", 0.01)
    assert np.array_equal(a, two.apply(u, "helmholtz", 0.01))
    assert np.array_equal(a, four.apply(u, "helmholtz", 0.01))
    assert one.ncomp == two.ncomp == four.ncomp == 1
    # translation invariance
    sh = np.zeros_like(u)
    sh[one.inner] = np.roll(u[one.inner], (3, -5), axis=(0, 1))
    b = np.zeros_like(u)
    b[one.inner] = np.roll(a[one.inner], (3, -5), axis=(0, 1))
    assert np.abs(one.apply(sh, "helmholtz", 0.01) - b).max() < 1e-12


def fft_solve(lev, f, op, c):
    fh = np.fft.fftn(f[lev.inner])
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(n) * 1.0 for n in lev.shape], indexing="ij")
    # fftfreq(n) * 2 pi = theta_d of each coefficient
    lam = lap_symbol(ks, lev.h)
    if op == "poisson":
        den = lam.copy()
        den.flat[0] = 1.0
        uh = fh / den
        uh.flat[0] = 0.0
    else:
        uh = fh / (1.0 - c * lam)
    out = lev.zeros()
    out[lev.inner] = np.real(np.fft.ifftn(uh))
    return out


@pytest.mark.parametrize("op", ["poisson", "helmholtz"])
@pytest.mark.parametrize("smoother", ["jacobi", "rb"])
def test_multigrid_solves_equal_fft_solves(op, smoother):
    rng = np.random.default_rng(1)
    lev = periodic_level(32)
    f = np.where(lev.mask, rng.normal(size=lev.pshape), 0.0)
    c = 0.0 if op == "poisson" else 0.05 / 32
    if op == "poisson":
        f[lev.mask] -= f[lev.mask].mean()
        assert lev.singular_components("poisson") == [0]
    else:
        assert lev.singular_components("helmholtz") == []
    x, st = mg.solve(lev, f, op, c, smoother=smoother, tol_rel=1e-13, max_cycles=200)
    assert st["converged"]
    want = fft_solve(lev, f, op, c)
    x = lev.comp_mean(x, lev.singular_components(op))
    assert np.abs(x - want)[lev.mask].max() < 1e-10 * np.abs(want).max()


def test_periodic_x_dirichlet_y_separates():
    n = 16
    lev = Level((n, n), 1 / n, [((0, 0), (n - 1, n - 1))], {(0, 0): "P", (0, 1): "P", (1, 0): "D", (1, 1): "D"})
    lev_y = Level((n, n), 1 / n, [((0, 0), (n - 1, n - 1))], {(0, 0): "D", (0, 1): "D", (1, 0): "D", (1, 1): "D"})
    rng = np.random.default_rng(2)
    g = rng.normal(size=n)
    for m in (0, 1, 5):
        t = 2 * np.pi * m / n
        cx = np.cos(t * np.arange(n))
        u = lev.zeros()
        u[lev.inner] = np.outer(cx, g)
        got = lev.apply(u, "poisson", 0.0)
        # the y part from the Dirichlet level: its y-Laplacian of the same
        # field, with its x-direction part removed by applying it to a field
        # constant in x and scaling by the x profile
        v = lev_y.zeros()
        v[lev_y.inner] = np.outer(np.ones(n), g)
        Gy = lev_y.ghosts(v)
        ly = lev_y.laplacian(v, Gy, dirs=[1])[lev_y.inner][0]
        want = lap_symbol([t], lev.h) * np.outer(cx, g) + np.outer(cx, ly)
        assert np.abs(got[lev.inner] - want).max() < 1e-9 * np.abs(want).max()
    assert lev.singular_components("poisson") == []


def test_components_join_across_the_periodic_side():
    bc = {(d, s): "P" for d in range(2) for s in (0, 1)}
    bc_np = {(0, 0): "D", (0, 1): "D", (1, 0): "P", (1, 1): "P"}
    boxes = [((0, 8), (31, 15)), ((0, 20), (31, 27))]  # full rows along x: x-periodic ghosts are cells
    lev = Level((32, 32), 1 / 32, boxes, {(0, 0): "P", (0, 1): "P", (1, 0): "D", (1, 1): "D"})
    assert lev.ncomp == 2
    full = [((0, 0), (31, 7)), ((0, 24), (31, 31))]  # touch across the y-periodic side only
    assert Level((32, 32), 1 / 32, full, bc_np).ncomp == 1
    assert Level((32, 32), 1 / 32, full, {k: "D" for k in bc}).ncomp == 2
    with pytest.raises(ValueError):  # x-periodic ghost of a box not spanning x is not a cell
        Level((32, 32), 1 / 32, [((0, 0), (15, 31))], bc)
    with pytest.raises(ValueError):
        Level((16, 16), 1 / 16, [((0, 0), (15, 15))], {(0, 0): "P", (0, 1): "D", (1, 0): "D", (1, 1): "D"})


def test_transpose_identity_and_probed_matrix():
    rng = np.random.default_rng(3)
    bc = {(0, 0): "P", (0, 1): "P", (1, 0): "N", (1, 1): "D"}
    lev = Level((8, 8), 1 / 8, [((0, 0), (3, 7)), ((4, 0), (7, 7))], bc)
    for op, c in (("poisson", 0.0), ("helmholtz", 0.03)):
        M, cells = mg.assemble(lev, op, c)
        MT = np.zeros_like(M)
        for j, cell in enumerate(cells):
            e = lev.zeros()
            e[tuple(cell)] = 1.0
            MT[:, j] = lev.apply_T(e, op, c)[lev.mask]
        assert np.abs(MT - M.T).max() < 1e-12 * np.abs(M).max()
        u = np.where(lev.mask, rng.normal(size=lev.pshape), 0.0)
        v = np.where(lev.mask, rng.normal(size=lev.pshape), 0.0)
        lhs = (lev.apply(u, op, c) * v)[lev.mask].sum()
        rhs = (u * lev.apply_T(v, op, c))[lev.mask].sum()
        assert abs(lhs - rhs) < 1e-12 * np.abs(M).max() * 64
    # the diagonal with periodic ghosts (no wrap contribution) is the probed one
    D = lev.diagonal("helmholtz", 0.03)
    M, cells = mg.assemble(lev, "helmholtz", 0.03)
    assert np.abs(D[lev.mask] - np.diag(M)).max() < 1e-12 * np.abs(M).max()


@pytest.mark.parametrize("m", [(1, 0), (2, 3), (5, 1)])
def test_projection_symbol(m):
    n = 16
    lev = periodic_level(n)
    e, theta = mode(lev, m)
    a = np.array([0.7 + 0.2j, -0.3 + 0.9j])
    W = [np.real(a[d] * e) for d in range(2)]
    U, _, st = proj.project(lev, W, tol_rel=1e-14, max_cycles=300)
    assert st["converged"]
    g = np.array([grad_symbol(t, lev.h) for t in theta])
    lam = lap_symbol(theta, lev.h)
    ah = a - g * (g @ a) / lam
    for d in range(2):
        want = np.real(ah[d] * e)
        assert np.abs(U[d] - want)[lev.mask].max() < 1e-10, d


def test_composite_hierarchy_on_a_periodic_base():
    """A refined patch inside a periodic base level: the composite solve's
    operator residual vanishes and the hierarchy's Poisson system is
    singular; a patch touching the periodic side is rejected."""
    bc = {(d, s): "P" for d in range(2) for s in (0, 1)}
    H = amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((8, 8), (19, 23))]], bc)
    assert H.singular("poisson") and not H.singular("helmholtz")
    rng = np.random.default_rng(4)
    f = [np.where(lev.mask, rng.normal(size=lev.pshape), 0.0) for lev in H.levels]
    U, st = amr.composite_solve(H, f, "helmholtz", 0.01, tol_rel=1e-12, max_cycles=100)
    assert st["converged"]
    R = amr.composite_residual(H, U, f, "helmholtz", 0.01)
    assert H.norm_inf(R) < 1e-10 * H.norm_inf(f)
    with pytest.raises(ValueError):
        amr.Hierarchy((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((0, 8), (15, 23))]], bc)
