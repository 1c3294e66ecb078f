"""Pins of the oracle's IMEX step (oracle/imex.py, eq. GePUP-IMEX with the
ARK4(3)6L[2]SA pair) and its convection operator (eq. convOp):

* the tableau: nodes equal the row sums of both parts, A_E strictly lower
  triangular, A_I singly diagonal with gamma = 1/4 and an explicit first
  stage, b = last row of A_I, and every order condition of an additive
  Runge-Kutta method of order 4 (both parts and all couplings), which a
  single wrong digit of a coefficient breaks;
* convection: fourth-order convergence of the cell averages of div(u u)
  against exact ones (face averages of the products by Gauss quadrature),
  2D and 3D; a scheme without the h^2/12 transverse term converges at
  second order only, so the rate pins that term; zero sum over the periodic
  grid (telescoping fluxes);
* the stage loop on a shear flow u = (f(y), 0) with a time-dependent
  forcing of the same form: convection and divergence vanish discretely,
  so the pressure is zero, the projection is the identity and each Fourier
  mode follows the additive step on y' = lambda y + g(t) in closed form,
  Y = (I - z A_I)^-1 (y0 + dt A_E g), y1 = Y_6 + dt (b - A_E[6]).g,
  z = nu lambda dt, computed from the tableau alone (a wrong coefficient
  index, gamma, weight or stage time fails).

Not pinned by a convergence rate in time: the step ends with w = P w* for
the approximate projection eq. appProj, which is not idempotent, so on a
coarse grid every step adds a spatial error that does not shrink with dt;
the nonlinear chain is pinned by its parts (convection above, gradient,
divergence and projection in their own tests) and the closed form above.
"""
import itertools

import numpy as np
import pytest

from oracle import imex
from oracle.level import Level


def plevel(n, dim=2):
    return Level((n,) * dim, 1.0 / n, [((0,) * dim, (n - 1,) * dim)],
                 {(d, s): "P" for d in range(dim) for s in (0, 1)})


def test_tableau_structure_and_order_conditions():
    AE, AI, b, c = np.array(imex.AE), np.array(imex.AI), np.array(imex.B), np.array(imex.C)
    assert np.abs(AE.sum(1) - c).max() < 1e-15 and np.abs(AI.sum(1) - c).max() < 1e-15
    assert np.all(np.triu(AE) == 0.0)
    assert np.all(np.triu(AI, 1) == 0.0) and AI[0, 0] == 0.0
    assert np.all(np.diag(AI)[1:] == imex.GAMMA) and imex.GAMMA == 0.25
    assert np.array_equal(b, AI[5]) and c[-1] == 1.0
    assert abs(b.sum() - 1) < 1e-15 and abs(b @ c - 1 / 2) < 1e-15
    assert abs(b @ c ** 2 - 1 / 3) < 1e-15 and abs(b @ c ** 3 - 1 / 4) < 1e-15
    for A1, A2 in itertools.product((AE, AI), repeat=2):
        assert abs(b @ (A1 @ c) - 1 / 6) < 1e-15
        assert abs(b @ (c * (A1 @ c)) - 1 / 8) < 1e-15
        assert abs(b @ (A1 @ c ** 2) - 1 / 12) < 1e-15
        assert abs(b @ (A1 @ (A2 @ c)) - 1 / 24) < 1e-15
    # a perturbed coefficient breaks a condition
    bad = AE.copy()
    bad[3, 1] *= 1 + 1e-6
    assert abs(b @ (bad @ c) - 1 / 6) > 1e-9 or abs(b @ (c * (bad @ c)) - 1 / 8) > 1e-9


# ---------------------------------------------------------------------------
TWO_PI = 2 * np.pi


def field2(x, y):
    u = np.sin(TWO_PI * x) * np.cos(TWO_PI * y) + 0.3 * np.cos(2 * TWO_PI * y)
    v = -np.cos(TWO_PI * x) * np.sin(TWO_PI * y) + 0.2 * np.sin(TWO_PI * x + 0.4)
    return [u, v]


def field3(x, y, z):
    u = np.sin(TWO_PI * x) * np.cos(TWO_PI * y) * np.cos(TWO_PI * z) + 0.2 * np.sin(TWO_PI * z)
    v = np.cos(TWO_PI * x) * np.sin(TWO_PI * y) * np.cos(TWO_PI * z) + 0.1
    w = -2 * np.cos(TWO_PI * x) * np.cos(TWO_PI * y) * np.sin(TWO_PI * z) + 0.3 * np.cos(TWO_PI * (x + y))
    return [u, v, w]


def gauss(m):
    p, w = np.polynomial.legendre.leggauss(m)
    return (p + 1) / 2, w / 2


def exact_averages(n, dim, fn, m=6):
    """Cell averages of fn's components and cell averages of div(u u_e)
    (from the exact face averages of the products), by tensor Gauss rules."""
    h = 1.0 / n
    p, w = gauss(m)
    idx = np.arange(n)
    # cell averages
    grids = np.meshgrid(*([(idx[:, None] + p[None, :]).ravel() * h] * dim), indexing="ij")
    vals = fn(*grids)
    def cell_avg(a):
        shp = []
        for _ in range(dim):
            shp += [n, m]
        a = a.reshape(shp)
        for k in range(dim):
            a = np.tensordot(a, w, axes=([k + 1], [0]))
        return a
    avg = [cell_avg(v) for v in vals]
    div = [np.zeros((n,) * dim) for _ in range(dim)]
    for d in range(dim):
        # face i + 1/2 along d at x_d = (i + 1) h, quadrature across
        axes = []
        for e in range(dim):
            if e == d:
                axes.append(((idx + 1) * h)[:, None].ravel())
            else:
                axes.append((idx[:, None] + p[None, :]).ravel() * h)
        g = np.meshgrid(*axes, indexing="ij")
        f = fn(*g)
        for e in range(dim):
            prod = f[d] * f[e]
            shp = []
            for k in range(dim):
                shp += [n, 1] if k == d else [n, m]
            a = prod.reshape(shp)
            for k in range(dim):
                a = np.tensordot(a, np.ones(1) if k == d else w, axes=([k + 1], [0]))
            div[e] += (a - np.roll(a, 1, axis=d)) / h
    return avg, div


@pytest.mark.parametrize("dim,ns,fn", [(2, (16, 32, 64), field2), (3, (8, 16, 32), field3)])
def test_convection_fourth_order(dim, ns, fn):
    errs = []
    for n in ns:
        lev = plevel(n, dim)
        avg, div = exact_averages(n, dim, fn)
        U = []
        for e in range(dim):
            a = lev.zeros()
            a[lev.inner] = avg[e]
            U.append(a)
        got = imex.convection(lev, U)
        errs.append(max(np.abs(got[e][lev.inner] - div[e]).max() for e in range(dim)))
        for e in range(dim):  # telescoping fluxes
            assert abs(got[e][lev.inner].sum()) < 1e-10 * n ** dim
    rates = [np.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    assert rates[-1] > 3.7, (errs, rates)


def additive_step(z, y0, gs, dt):
    """Closed form of the additive step on y' = lambda y + g(t) with the
    explicit part carrying g (gs[j] = g at the stage time t_n + c_j dt):
    stage values Y = (I - z A_I)^-1 (y0 + dt A_E gs), result
    Y_6 + dt sum_j (b_j - A_E[6,j]) gs_j."""
    AI, AE, b = np.array(imex.AI), np.array(imex.AE), np.array(imex.B)
    gs = np.asarray(gs, dtype=float)
    Y = np.linalg.solve(np.eye(6) - z * AI, y0 * np.ones(6) + dt * (AE @ gs))
    return Y[5] + dt * (b - AE[5]) @ gs


@pytest.mark.parametrize("forcing", [False, True])
def test_stage_loop_on_a_shear_flow_is_the_additive_step(forcing):
    """u = (f(y), 0) and g = (a(t) cos(2 pi k_g y), 0): every stage's
    convection, divergence and pressure vanish, and each Fourier mode follows
    the closed form above; a(t) = cos(omega t) with omega dt = 2 makes the
    stage values of g differ, so A_E and the final weights b - A_E[6] enter
    one by one."""
    n, nu, dt, t0 = 16, 0.02, 0.01, 0.3
    lev = plevel(n)
    y = (np.arange(n) + 0.5) / n
    modes = [(1, 0.8), (3, -0.5)]
    prof = sum(a * np.cos(TWO_PI * k * y) for k, a in modes)
    U = [lev.zeros(), lev.zeros()]
    U[0][lev.inner] = np.broadcast_to(prof[None, :], (n, n))
    gk, omega = 2, 2.0 / dt
    amp = [np.cos(omega * (t0 + cj * dt)) for cj in imex.C] if forcing else [0.0] * 6
    g = None
    if forcing:
        g = []
        for j in range(imex.NSTAGES):
            ga = lev.zeros()
            ga[lev.inner] = np.broadcast_to(amp[j] * np.cos(TWO_PI * gk * y)[None, :], (n, n))
            g.append([ga, lev.zeros()])
    out = imex.imex_step(lev, U, dt, nu, g=g, tol_rel=1e-13)
    assert np.abs(out[1][lev.inner]).max() < 1e-12
    got = out[0][lev.inner][0]
    lam = lambda k: (32 * np.cos(TWO_PI * k / n) - 2 * np.cos(2 * TWO_PI * k / n) - 30) * n * n / 12
    want = sum(additive_step(nu * lam(k) * dt, a, [0.0] * 6, dt) * np.cos(TWO_PI * k * y) for k, a in modes)
    if forcing:
        want = want + additive_step(nu * lam(gk) * dt, 0.0, amp, dt) * np.cos(TWO_PI * gk * y)
        # the stage values matter: g frozen at t_n gives a different result
        frozen = additive_step(nu * lam(gk) * dt, 0.0, [amp[0]] * 6, dt)
        assert abs(frozen - additive_step(nu * lam(gk) * dt, 0.0, amp, dt)) > 1e-4
    assert np.abs(got - want).max() < 1e-11
    # the factor is not the trivial one: one backward-Euler step differs by far more
    k, a = modes[1]
    z = nu * lam(k) * dt
    assert abs(additive_step(z, a, [0.0] * 6, dt) - a / (1 - z)) > 1e-5
