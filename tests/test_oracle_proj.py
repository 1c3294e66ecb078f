"""Pins of the oracle's discrete gradient, divergence and approximate
projection (single level and composite): exactness on polynomials of degree
<= 4 per variable (the operators, the fills and AMRCFI are exact there), a
divergence-free polynomial velocity left unchanged, the gradient of a
Neumann potential removed exactly, and conservation of the refluxed
composite divergence."""
import numpy as np
import pytest

from oracle import amr, fv, proj
from oracle.level import PAD, Level
from tests.polyfix import Poly1, problem

# phi0 = p(x) q(y) [r(z)] with zero normal derivative on the unit box
p = Poly1([0.0, 0.0, 3.0, -2.0])            # p' = 6x(1-x)
q = Poly1([0.0, 0.0, 1.0, -2.0, 1.0])       # y^2 (1-y)^2, q'(0) = q'(1) = 0
r = Poly1([0.5, 0.0, 3.0, -2.0])
# stream function P(x) Q(y): w_df = (P Q', -P' Q).  Every velocity
# component is of degree <= 3 along its own direction: the face averages of
# eq. (cell2face) that refluxing compares are exact to degree 3 only.
P = Poly1([0.0, -0.5, 0.0, 1.0])
Q = Poly1([0.1, 0.3, 1.0, 0.3])


def grad_terms(dim):
    f = [p, q, r][:dim]
    out = []
    for d in range(dim):
        t = list(f)
        t[d] = f[d].d1()
        out.append([tuple(t)])
    return out


def lap_terms(dim):
    f = [p, q, r][:dim]
    out = []
    for d in range(dim):
        t = list(f)
        t[d] = f[d].d2()
        out.append(tuple(t))
    return out


def df_terms(dim):
    if dim == 2:
        return [[(P, Q.d1())], [(-P.d1(), Q)]]
    # (P Q' R, -P' Q R, 0) with R a function of z only: divergence-free
    R = Poly1([1.0, 0.5, -0.25])
    return [[(P, Q.d1(), R)], [(-P.d1(), Q, R)], [(Poly1([0.0]), Poly1([0.0]), Poly1([0.0]))]]


def cells(lev, terms):
    return problem(lev, terms, "poisson", 0.0)[0]


def unit(n, dim, kind):
    return Level((n,) * dim, 1.0 / n, [((0,) * dim, (n - 1,) * dim)], {(d, s): kind for d in range(dim) for s in (0, 1)},
                 kind)


def rel(a, b, mask):
    return np.abs(a - b)[mask].max() / max(np.abs(b)[mask].max(), 1e-300)


@pytest.mark.parametrize("dim,n", [(2, 16), (3, 8)])
def test_gradient_and_divergence_exact_on_polynomials(dim, n):
    lp, lw = unit(n, dim, "N"), unit(n, dim, "D")
    f = [p, q, r][:dim]
    phi, _, fdp = problem(lp, [tuple(f)], "poisson", 0.0)
    G = proj.gradient(lp, phi, fdp)
    for d, terms in enumerate(grad_terms(dim)):
        assert rel(G[d], cells(lp, terms), lp.mask) < 1e-12
    # divergence of the polynomial velocity grad(phi0) + w_df
    W, wb = [], []
    for d in range(dim):
        terms = grad_terms(dim)[d] + df_terms(dim)[d]
        u, _, fd = problem(lw, terms, "poisson", 0.0)
        W.append(u)
        wb.append(fd)
    div = proj.divergence(lw, W, wb)
    want = cells(lw, lap_terms(dim))
    assert rel(div, want, lw.mask) < 1e-11


@pytest.mark.parametrize("dim,n", [(2, 32), (3, 16)])
def test_projection_removes_gradient_keeps_solenoidal_part(dim, n):
    lev = unit(n, dim, "D")
    lw = proj.velocity_level(lev)
    W, wb, want = [], [], []
    for d in range(dim):
        u, _, fd = problem(lw, grad_terms(dim)[d] + df_terms(dim)[d], "poisson", 0.0)
        W.append(u)
        wb.append(fd)
        want.append(cells(lw, df_terms(dim)[d]))
    U, phi, st = proj.project(lev, W, wb, tol_rel=1e-13)
    assert st["converged"]
    scale = max(np.abs(w[lev.mask]).max() for w in W)
    for d in range(dim):
        assert np.abs(U[d] - want[d])[lev.mask].max() < 1e-9 * scale


def test_divergence_free_field_is_unchanged():
    lev = unit(32, 2, "D")
    W, wb = [], []
    for t in df_terms(2):
        u, _, fd = problem(lev, t, "poisson", 0.0)
        W.append(u)
        wb.append(fd)
    U, phi, st = proj.project(lev, W, wb, tol_rel=1e-13)
    for d in range(2):
        assert np.abs(U[d] - W[d])[lev.mask].max() < 1e-10 * np.abs(W[d]).max()


def two_level(kind):
    return amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((8, 8), (15, 23)), ((16, 8), (23, 15))]],
                         {(d, s): kind for d in range(2) for s in (0, 1)})


def three_level(kind):
    return amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((4, 4), (27, 27))], [((16, 16), (31, 31))]],
                         {(d, s): kind for d in range(2) for s in (0, 1)})


def two_level_r4(kind):
    return amr.Hierarchy((16, 16), 1.0 / 16, [[((0, 0), (15, 15))], [((16, 16), (39, 47)), ((40, 16), (47, 31))]],
                         {(d, s): kind for d in range(2) for s in (0, 1)}, ratio=4)


@pytest.mark.parametrize("make", [two_level, three_level, two_level_r4])
def test_composite_projection_on_polynomials(make):
    H = make("D")
    Hw = proj.hierarchy_with(H, "D")
    W = [[None] * H.nlev for _ in range(2)]
    wb = [[None] * H.nlev for _ in range(2)]
    want = [[None] * H.nlev for _ in range(2)]
    for l, lev in enumerate(Hw.levels):
        for d in range(2):
            u, _, fd = problem(lev, grad_terms(2)[d] + df_terms(2)[d], "poisson", 0.0)
            W[d][l], wb[d][l] = u, fd
            want[d][l] = cells(lev, df_terms(2)[d])
    # composite divergence and gradient are exact
    div = proj.composite_divergence(Hw, W, wb)
    lap = [cells(lev, lap_terms(2)) for lev in Hw.levels]
    for l in range(H.nlev):
        assert rel(div[l], lap[l], H.valid[l]) < 1e-11
    Hp = proj.hierarchy_with(H, "N")
    phi = [cells(lev, [(p, q)]) for lev in Hp.levels]
    G = proj.composite_gradient(Hp, phi)
    for d in range(2):
        for l in range(H.nlev):
            assert rel(G[d][l], cells(Hp.levels[l], grad_terms(2)[d]), H.valid[l]) < 1e-12
    U, Phi, st = proj.composite_project(H, W, wb, tol_rel=1e-13)
    assert st["converged"]
    for d in range(2):
        for l in range(H.nlev):
            assert np.abs(U[d][l] - want[d][l])[H.valid[l]].max() < 1e-9


@pytest.mark.parametrize("make", [two_level, two_level_r4])
def test_composite_divergence_is_conservative(make):
    Hw = make("D")
    rng = np.random.default_rng(3)
    W = [[np.where(lev.mask, rng.normal(size=lev.pshape), 0.0) for lev in Hw.levels] for _ in range(2)]
    wb = []
    for d in range(2):
        per = []
        for lev in Hw.levels:
            fd = lev.zero_face_data()
            for k in fd:
                e = lev.end_is_physical(*k)
                fd[k][e] = rng.normal(size=int(e.sum()))
            per.append(fd)
        wb.append(per)
    div = proj.composite_divergence(Hw, W, wb)
    vol = sum(div[l][Hw.valid[l]].sum() * Hw.levels[l].h ** 2 for l in range(Hw.nlev))
    # boundary fluxes: face averages (eq. cell2face) on the physical faces of
    # valid cells, from each level's own cells and filled ghosts
    Wd = [Hw.average_down_all(W[d]) for d in range(2)]
    bnd = 0.0
    for l, lev in enumerate(Hw.levels):
        for d in range(2):
            cfv = Hw.amrcfi(l, Wd[d][l - 1]) if l else None
            G = lev.ghosts(Wd[d][l], wb[d][l], cfv)
            u = Wd[d][l]
            for s in (0, 1):
                ends = lev.end_is_physical(d, s) & Hw.valid[l]
                for pos in np.argwhere(ends):
                    pos = tuple(pos)

                    def v(k):
                        qq = list(pos)
                        qq[d] += k
                        qq = tuple(qq)
                        return u[qq] if lev.mask[qq] else G[(d, 1 if k > 0 else 0)][qq]
                    F = fv.face_value(v(-1), v(0), v(1), v(2)) if s else fv.face_value(v(-2), v(-1), v(0), v(1))
                    bnd += (1 if s else -1) * F * lev.h
    scale = sum(np.abs(div[l][Hw.valid[l]]).sum() * Hw.levels[l].h ** 2 for l in range(Hw.nlev))
    assert abs(vol - bnd) < 1e-13 * scale
