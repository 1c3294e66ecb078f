"""Oracle: the discrete gradient and divergence (Section 3, eq. discreteOps
a-b), the approximate projection P = I - G L^-1 D (eq. appProj) on one
level, and their composite forms over a hierarchy (Section 5.3, COH-1..4,
eq. comp_ProjOp).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper defers the projection's boundary treatment to another paper.
Readings taken:

* D acts on the velocity components with their ghosts filled by the
  Dirichlet fill (eq. velBCHomoDiri5th) from the face averages of the
  boundary velocity (data ``wb``, per component), coarse-fine ghosts by
  AMRCFI on a hierarchy (COH-1);
* phi solves the pure-Neumann Poisson equation L phi = D w with homogeneous
  Neumann data (the right-hand side shifted for solvability, phi mean-free);
* G acts on phi with its ghosts from the Neumann fill (eq. Neumann5),
  coarse-fine ghosts by AMRCFI;
* the projected velocity is u = w - G phi;
* composite D is in divergence form: its face fluxes are the face averages
  of eq. (cell2face, first row), and at a coarse-fine face the coarse flux is
  replaced by the mean of the fine fluxes (COH-3); composite G is not in
  divergence form (no refluxing).  Both average down onto covered cells
  (COH-4).
"""
import numpy as np

from . import amr, fv, mg
from .level import PAD, Level, _shift


# ---------------------------------------------------------------------------
# one level
def gradient(lev, phi, fd=None, cfv=None):
    """[G_d phi for d in directions], eq. (discreteOps a), ghosts of phi
    from the level's fill (fd: face data, cfv: interpolated ghosts)."""
    G = lev.ghosts(phi, fd, cfv)
    out = []
    for d in range(lev.dim):
        g = fv.gradient_1d(lev.neighbour(phi, G, d, -2), lev.neighbour(phi, G, d, -1),
                           lev.neighbour(phi, G, d, 1), lev.neighbour(phi, G, d, 2), lev.h)
        out.append(np.where(lev.mask, g, 0.0))
    return out


def divergence(lev, W, wb=None, cfvs=None):
    """D w = sum_d G_d w_d, eq. (discreteOps b); wb[d]: face data of
    component d for the level's fill, cfvs[d]: its interpolated ghosts."""
    out = lev.zeros()
    for d in range(lev.dim):
        G = lev.ghosts(W[d], wb[d] if wb else None, cfvs[d] if cfvs else None)
        out += fv.gradient_1d(lev.neighbour(W[d], G, d, -2), lev.neighbour(W[d], G, d, -1),
                              lev.neighbour(W[d], G, d, 1), lev.neighbour(W[d], G, d, 2), lev.h)
    return np.where(lev.mask, out, 0.0)


def _keep_periodic(bc, kind):
    return {k: ("P" if v == "P" else kind) for k, v in bc.items()}


def velocity_level(lev):
    """The same boxes with Dirichlet conditions on every non-periodic side
    (the velocity's fill)."""
    return Level(lev.shape, lev.h, lev.boxes, _keep_periodic(lev.phys_bc, "D"), "D")


def pressure_level(lev):
    """The same boxes with Neumann conditions on every non-periodic side
    (phi's fill)."""
    return Level(lev.shape, lev.h, lev.boxes, _keep_periodic(lev.phys_bc, "N"), "N")


def project(lev, W, wb=None, tol_rel=1e-12, max_cycles=200, smoother="jacobi"):
    """u = w - G phi with L phi = D w (pure Neumann, homogeneous data) on
    a level that covers its grid.  Returns (U, phi, solve stats)."""
    lw, lp = velocity_level(lev), pressure_level(lev)
    div = divergence(lw, W, wb)
    phi, st = mg.solve(lp, div, "poisson", 0.0, None, tol_rel=tol_rel, max_cycles=max_cycles, smoother=smoother)
    gp = gradient(lp, phi)
    return [np.where(lev.mask, W[d] - gp[d], 0.0) for d in range(lev.dim)], phi, st


# ---------------------------------------------------------------------------
# composite (hierarchy) forms
def hierarchy_with(H, kind):
    """A hierarchy with H's boxes and every non-periodic physical condition
    set to kind."""
    boxes = [lev.boxes for lev in H.levels]
    return amr.Hierarchy(H.levels[0].shape, H.levels[0].h, boxes, _keep_periodic(H.levels[0].phys_bc, kind),
                         H.ratio)


def composite_gradient(Hp, Phi):
    """G^comp phi: per-level gradients with AMRCFI ghosts, averaged down.
    Phi: per-level arrays (covered cells are replaced by averages first)."""
    Phi = Hp.average_down_all(Phi)
    comps = [[None] * Hp.nlev for _ in range(Hp.dim)]
    for l, lev in enumerate(Hp.levels):
        cfv = Hp.amrcfi(l, Phi[l - 1]) if l else None
        g = gradient(lev, Phi[l], None, cfv)
        for d in range(Hp.dim):
            comps[d][l] = g[d]
    return [Hp.average_down_all(c) for c in comps]


def composite_divergence(Hw, W, wb=None):
    """D^comp w: W[d][l] per component and level; wb[d][l] face data of the
    physical faces (None = zero).  Per-level divergence with AMRCFI ghosts,
    face-average fluxes refluxed at coarse-fine faces, averaged down."""
    D = Hw.dim
    W = [Hw.average_down_all(W[d]) for d in range(D)]
    out, ghosts = [], []
    for l, lev in enumerate(Hw.levels):
        Gl = []
        acc = lev.zeros()
        for d in range(D):
            cfv = Hw.amrcfi(l, W[d][l - 1]) if l else None
            G = lev.ghosts(W[d][l], wb[d][l] if wb else None, cfv)
            Gl.append(G)
            acc += fv.gradient_1d(lev.neighbour(W[d][l], G, d, -2), lev.neighbour(W[d][l], G, d, -1),
                                  lev.neighbour(W[d][l], G, d, 1), lev.neighbour(W[d][l], G, d, 2), lev.h)
        out.append(np.where(lev.mask, acc, 0.0))
        ghosts.append(Gl)
    for l in range(1, Hw.nlev):
        fine, coarse = Hw.levels[l], Hw.levels[l - 1]
        hc = coarse.h
        for pos, d, s in Hw.cf_faces(l):
            i = np.array(pos) - PAD
            Wc, Gc = W[d][l - 1], ghosts[l - 1][d]
            Wf, Gf = W[d][l], ghosts[l][d]

            def cval(off):
                q = np.array(pos)
                q[d] += off
                q = tuple(q)
                if coarse.mask[q]:
                    return Wc[q]
                return Gc[(d, 1 if off > 0 else 0)][q]

            # coarse face average of w_d on the face (d, s) of the cell
            Fc = fv.face_value(cval(-1), cval(0), cval(1), cval(2)) if s else \
                fv.face_value(cval(-2), cval(-1), cval(0), cval(1))
            rr = Hw.ratio
            jd = rr * i[d] + (rr if s else 0)
            trans = [e for e in range(D) if e != d]
            tot, nf = 0.0, 0
            for off in np.ndindex(*(rr,) * (D - 1)):
                q = np.zeros(D, int)
                q[d] = jd
                for e, o in zip(trans, off):
                    q[e] = rr * i[e] + o

                def fval(delta):
                    qq = q.copy()
                    qq[d] += delta
                    t = tuple(qq + PAD)
                    if fine.mask[t]:
                        return Wf[t]
                    return Gf[(d, 1 if delta >= 0 else 0)][t]
                tot += fv.face_value(fval(-2), fval(-1), fval(0), fval(1))
                nf += 1
            out[l - 1][pos] += (1 if s else -1) * (tot / nf - Fc) / hc
    return Hw.average_down_all(out)


def composite_project(H, W, wb=None, tol_rel=1e-12, max_cycles=200, smoother="jacobi"):
    """u = w - G^comp phi with L^comp phi = D^comp w (pure Neumann), eq.
    (comp_ProjOp).  Returns (U per component and level, Phi, stats)."""
    Hw, Hp = hierarchy_with(H, "D"), hierarchy_with(H, "N")
    div = composite_divergence(Hw, W, wb)
    Phi, st = amr.composite_solve(Hp, div, "poisson", 0.0, None, tol_rel=tol_rel, max_cycles=max_cycles,
                                  smoother=smoother)
    G = composite_gradient(Hp, Phi)
    U = [[np.where(H.levels[l].mask, W[d][l] - G[d][l], 0.0) for l in range(H.nlev)] for d in range(H.dim)]
    return [H.average_down_all(U[d]) for d in range(H.dim)], Phi, st
