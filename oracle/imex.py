"""Oracle: one time step of the IMEX scheme eq. GePUP-IMEX (Section 4) on a
single level whose grid is periodic in every direction (the domains of
Section 7.3), with the convection operator of eq. convOp.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The ODE system eq. ODE-MOL, d<w>/dt = X(<u>, <q>, t) + nu L <w> with
X = <g> - Div<uu> - G<q>, is integrated by the ERK-ESDIRK additive
Runge-Kutta pair the paper cites, ARK4(3)6L[2]SA of Kennedy and Carpenter
(Appl. Numer. Math. 44, 2003): six stages, explicit tableau A_E, singly
diagonally implicit tableau A_I with diagonal gamma = 1/4 (first stage
explicit), shared weights b = last row of A_I (stiffly accurate) and nodes
c.  The coefficients are restated from that publication (the paper does
not print them); the tests pin them by the order conditions of an additive
method of order 4.

One step from <u>^n (= <w>^n), in the order eq. GePUP-IMEX gives:

* stage 1: w1 = u1 = w^n;
* stages s = 2..6: the pressure Poisson system L q^(s-1) = D(g^(s-1) -
  Div<uu>^(s-1)) (TLS-1), the stage's X^(s-1); then the Helmholtz systems
  (I - dt nu gamma L) w^(s) = w^n + dt sum_j A_E[s,j] X^(j) + dt nu sum_j
  A_I[s,j] L w^(j), j < s (TLS-2, per component), and u^(s) = P w^(s)
  (eq. appProj; TLS-3);
* after the last stage: X^(6) (one more pressure solve), w* = w^(6) + dt
  sum_j (b_j - A_E[6,j]) X^(j), u^(n+1) = P w*, w^(n+1) = u^(n+1).

Readings: on a periodic domain no boundary conditions enter (the paper's
conditions for w and q apply on walls only); the pressure system is the
singular periodic Poisson system, its right-hand side a divergence (zero
sum), solved to zero mean; the forcing g^(j) is evaluated at the stage time
t_n + c_j dt and passed in.
"""
import numpy as np

from . import mg, proj

# ARK4(3)6L[2]SA (Kennedy & Carpenter 2003), explicit and implicit parts.
C = [0.0, 1 / 2, 83 / 250, 31 / 50, 17 / 20, 1.0]
GAMMA = 1 / 4
AE = [
    [0.0] * 6,
    [1 / 2, 0, 0, 0, 0, 0],
    [13861 / 62500, 6889 / 62500, 0, 0, 0, 0],
    [-116923316275 / 2393684061468, -2731218467317 / 15368042101831, 9408046702089 / 11113171139209, 0, 0, 0],
    [-451086348788 / 2902428689909, -2682348792572 / 7519795681897, 12662868775082 / 11960479115383,
     3355817975965 / 11060851509271, 0, 0],
    [647845179188 / 3216320057751, 73281519250 / 8382639484533, 552539513391 / 3454668386233,
     3354512671639 / 8306763924573, 4040 / 17871, 0],
]
AI = [
    [0.0] * 6,
    [1 / 4, 1 / 4, 0, 0, 0, 0],
    [8611 / 62500, -1743 / 31250, 1 / 4, 0, 0, 0],
    [5012029 / 34652500, -654441 / 2922500, 174375 / 388108, 1 / 4, 0, 0],
    [15267082809 / 155376265600, -71443401 / 120774400, 730878875 / 902184768, 2285395 / 8070912, 1 / 4, 0],
    [82889 / 524892, 0, 15625 / 83664, 69875 / 102672, -2260 / 8211, 1 / 4],
]
B = list(AI[5])
NSTAGES = 6


def check_level(lev):
    if lev.ncells != int(np.prod(lev.shape)) or len(lev.periodic) != lev.dim:
        raise ValueError("the IMEX step needs one level covering a grid periodic in every direction")


def _p(a, d, k):
    """a[i + k e_d] on the periodic (unpadded) grid."""
    return np.roll(a, -k, axis=d)


def face_average(a, d):
    """<phi> on the face i + 1/2 e_d from cell averages (eq. cell2face,
    first row), stored at index i."""
    return (-_p(a, d, 2) + 7 * _p(a, d, 1) + 7 * a - _p(a, d, -1)) / 12


def convection(lev, U):
    """Div<uu> of eq. convOp on a periodic level: per component e, the sum
    over d of the differences of F<u_d, u_e> across the two faces normal to
    d, over h, where F<phi, psi> on a face is the product of the face
    averages plus h^2/12 times the products of their transverse centred
    differences (over 2h), summed over the transverse directions."""
    check_level(lev)
    D, h = lev.dim, lev.h
    u = [U[e][lev.inner] for e in range(D)]
    out = [np.zeros_like(u[0]) for _ in range(D)]
    for d in range(D):
        fa = [face_average(u[e], d) for e in range(D)]
        for e in range(D):
            F = fa[d] * fa[e]
            for dp in range(D):
                if dp == d:
                    continue
                gd = (_p(fa[d], dp, 1) - _p(fa[d], dp, -1)) / (2 * h)
                ge = (_p(fa[e], dp, 1) - _p(fa[e], dp, -1)) / (2 * h)
                F = F + h * h / 12 * gd * ge
            out[e] += (F - _p(F, d, -1)) / h
    res = []
    for e in range(D):
        a = lev.zeros()
        a[lev.inner] = out[e]
        res.append(a)
    return res


def laplacian(lev, w):
    """L w (eq. discreteOps c) with the level's (periodic) ghosts."""
    return lev.laplacian(w, lev.ghosts(w))


def explicit_term(lev, U, g, tol_rel, max_cycles):
    """X = g - Div<uu> - G q with L q = D(g - Div<uu>) (TLS-1).  Returns
    (X, q)."""
    D = lev.dim
    lp, lw = proj.pressure_level(lev), proj.velocity_level(lev)
    conv = convection(lev, U)
    V = [(g[e] if g is not None else 0.0) - conv[e] for e in range(D)]
    rhs = proj.divergence(lw, V)
    q, st = mg.solve(lp, rhs, "poisson", 0.0, None, tol_rel=tol_rel, max_cycles=max_cycles, smoother="rb")
    if not st["converged"]:
        raise RuntimeError("pressure solve did not converge")
    gq = proj.gradient(lp, q)
    return [np.where(lev.mask, V[e] - gq[e], 0.0) for e in range(D)], q


def imex_step(lev, Un, dt, nu, g=None, tol_rel=1e-12, max_cycles=200):
    """One step of eq. GePUP-IMEX.  Un: list of D padded arrays (u^n = w^n);
    g: None or g[j][e], the forcing at t_n + C[j] dt.  Returns u^(n+1)."""
    check_level(lev)
    D = lev.dim
    c = dt * nu * GAMMA
    Wn = [u.copy() for u in Un]
    W = [Wn]            # w^(j)
    Us = [Wn]           # u^(j)
    X, LW = [], []
    for s in range(1, NSTAGES):
        Xj, _ = explicit_term(lev, Us[s - 1], g[s - 1] if g is not None else None, tol_rel, max_cycles)
        X.append(Xj)
        LW.append([laplacian(lev, W[s - 1][e]) for e in range(D)])
        Ws = []
        for e in range(D):
            rhs = Wn[e].copy()
            for j in range(s):
                rhs = rhs + dt * AE[s][j] * X[j][e] + dt * nu * AI[s][j] * LW[j][e]
            rhs = np.where(lev.mask, rhs, 0.0)
            w, st = mg.solve(lev, rhs, "helmholtz", c, None, tol_rel=tol_rel, max_cycles=max_cycles,
                             smoother="rb")
            if not st["converged"]:
                raise RuntimeError("Helmholtz solve did not converge")
            Ws.append(w)
        W.append(Ws)
        U, _, st = proj.project(lev, Ws, tol_rel=tol_rel, max_cycles=max_cycles, smoother="rb")
        if not st["converged"]:
            raise RuntimeError("projection did not converge")
        Us.append(U)
    X6, _ = explicit_term(lev, Us[-1], g[NSTAGES - 1] if g is not None else None, tol_rel, max_cycles)
    X.append(X6)
    Wstar = []
    for e in range(D):
        w = W[-1][e].copy()
        for j in range(NSTAGES):
            w = w + dt * (B[j] - AE[NSTAGES - 1][j]) * X[j][e]
        Wstar.append(np.where(lev.mask, w, 0.0))
    Unew, _, st = proj.project(lev, Wstar, tol_rel=tol_rel, max_cycles=max_cycles, smoother="rb")
    if not st["converged"]:
        raise RuntimeError("projection did not converge")
    return Unew
