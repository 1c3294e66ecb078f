"""Oracle: transposes of the discrete gradient and divergence (eq.
discreteOps a-b) and of the approximate projection (eq. appProj, composite
eq. comp_ProjOp), on one level and over a hierarchy (not in the paper: the
adjoint that carries a loss on the projected velocity back to the velocity
before projection).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Every operator here is the homogeneous (zero boundary data) linear map of
``oracle/proj.py``, taken from the values on the valid cells to the values
on the valid cells (covered cells of the input are averages of their
children, those of the output are redundant copies).  Its transpose
reverses the forward steps, each transposed, in the way
``oracle/amr_adj.py`` does it for the composite Laplacian:

* the one-direction gradient G_d u_i = sum_m a_m u_(i+m e_d) with
  a_(+-1) = +-8/(12h), a_(+-2) = -+1/(12h) is antisymmetric, so its
  transpose on the cells of a level is -G_d applied to the adjoint extended
  by zero; the weight a_m that the cell i puts on a ghost position i + m e_d
  goes into that ghost's adjoint;
* ghost adjoints of the physical (and face-data) fills go back onto the four
  cells each fill reads with the fill weights, those of interpolated ghosts
  onto the AMRCFI window of the level below;
* refluxing of the composite divergence (COH-3: the coarse face average of
  eq. cell2face, first row, replaced by the mean of the fine ones) spreads
  the adjoint of the refluxed coarse cell onto the coarse and fine values
  and ghosts those face averages read;
* the average-down of the input sends the adjoint of a covered cell to its
  children in equal parts, coarse to fine.

The projection's transpose is P^T = I - D^T L^-T G^T, with L^-T the adjoint
of the pure-Neumann solve (``mg.solve(transpose=True)`` on a level,
``amr_adj.composite_solve_T`` on a hierarchy), which already contains
the transposes of the solvability shift and of the mean removal.
"""
import numpy as np

from . import amr_adj, fv, mg, proj
from .level import PAD, _shift

# stencil weights of eq. discreteOps a, in units of 1/(12h): a[m] for m = -2..2
_A = {-2: 1.0, -1: -8.0, 1: 8.0, 2: -1.0}


def _grad_T_level(lev, mu, d, Gbar):
    """(G_d^T mu) on the cells of one level (homogeneous: the ghosts' share
    is added to Gbar, the per-side ghost adjoints of direction d)."""
    m = np.where(lev.mask, mu, 0.0)
    zero = {(e, s): lev.zeros() for e in range(lev.dim) for s in (0, 1)}
    out = -fv.gradient_1d(lev.neighbour(m, zero, d, -2), lev.neighbour(m, zero, d, -1),
                          lev.neighbour(m, zero, d, 1), lev.neighbour(m, zero, d, 2), lev.h)
    out = np.where(lev.mask, out, 0.0)
    k12 = 12.0 * lev.h
    for s in (0, 1):
        step = 1 if s == 1 else -1
        # position p is read by the cell p - k step with weight a[k step]
        contrib = (_A[step] * _shift(m, d, -step) + _A[2 * step] * _shift(m, d, -2 * step)) / k12
        Gbar[(d, s)] += np.where(lev.mask, 0.0, contrib)
    return out


def _ghosts_T(lev, Gbar, back):
    """Physical / face-data fill adjoints of one level onto its cells."""
    amr_adj._scatter_fill(lev, Gbar, back)


# ---------------------------------------------------------------------------
# one level (the level covers its grid: no interpolated ghosts)
def gradient_T(lp, Mu):
    """sum_d G_d^T Mu[d] on the cells of the level lp (phi's fill)."""
    Gbar = {(d, s): lp.zeros() for d in range(lp.dim) for s in (0, 1)}
    out = lp.zeros()
    for d in range(lp.dim):
        out += _grad_T_level(lp, Mu[d], d, Gbar)
    back = lp.zeros()
    _ghosts_T(lp, Gbar, back)
    return np.where(lp.mask, out + back, 0.0)


def divergence_T(lw, lam):
    """[G_d^T lam for d] on the cells of the level lw (the velocity's fill):
    the transpose of D w = sum_d G_d w_d."""
    out = []
    for d in range(lw.dim):
        Gbar = {(e, s): lw.zeros() for e in range(lw.dim) for s in (0, 1)}
        o = _grad_T_level(lw, lam, d, Gbar)
        back = lw.zeros()
        _ghosts_T(lw, Gbar, back)
        out.append(np.where(lw.mask, o + back, 0.0))
    return out


def project_T(lev, Ubar, tol_rel=1e-12, max_cycles=200, smoother="jacobi"):
    """P^T ubar = ubar - D^T L^-T G^T ubar for the level projection of
    proj.project (homogeneous velocity data)."""
    lw, lp = proj.velocity_level(lev), proj.pressure_level(lev)
    g = gradient_T(lp, Ubar)
    lam, st = mg.solve(lp, g, "poisson", 0.0, tol_rel=tol_rel, max_cycles=max_cycles, smoother=smoother,
                       transpose=True)
    dt = divergence_T(lw, lam)
    return [np.where(lev.mask, Ubar[d] - dt[d], 0.0) for d in range(lev.dim)], lam, st


# ---------------------------------------------------------------------------
# composite forms
def _down_T(H, Ubar):
    """Transpose of the average-down of the input: covered adjoints to the
    children in equal parts, coarse to fine; result on the valid cells."""
    Ubar = [u.copy() for u in Ubar]
    for l in range(1, H.nlev):
        fine, coarse = H.levels[l], H.levels[l - 1]
        cov = np.where(H.covered[l - 1], Ubar[l - 1], 0.0)
        Ubar[l] += np.where(fine.mask, amr_adj._children(fine, coarse, cov, H.ratio), 0.0)
        Ubar[l - 1] = np.where(H.covered[l - 1], 0.0, Ubar[l - 1])
    return [np.where(H.valid[l], Ubar[l], 0.0) for l in range(H.nlev)]


def _ghost_adjoints_to_cells(H, Gbars, Ubar):
    """Every level's ghost adjoints: fills onto the level, AMRCFI onto the
    level below (finest first)."""
    for l in range(H.nlev - 1, -1, -1):
        lev = H.levels[l]
        back = lev.zeros()
        _ghosts_T(lev, Gbars[l], back)
        Ubar[l] += np.where(lev.mask, back, 0.0)
        if l:
            Ubar[l - 1] += np.where(H.levels[l - 1].mask,
                                    amr_adj._amrcfi_T(H, l, amr_adj._interp_ghost_adjoint(lev, Gbars[l])), 0.0)


def composite_gradient_T(Hp, Mu):
    """Transpose of proj.composite_gradient as a map between valid cells:
    Mu[d][l] (read on valid cells) -> per-level adjoint of phi."""
    D = Hp.dim
    Ubar, Gbars = [], []
    for l, lev in enumerate(Hp.levels):
        Gbar = {(d, s): lev.zeros() for d in range(D) for s in (0, 1)}
        out = lev.zeros()
        for d in range(D):
            out += _grad_T_level(lev, np.where(Hp.valid[l], Mu[d][l], 0.0), d, Gbar)
        Ubar.append(out)
        Gbars.append(Gbar)
    _ghost_adjoints_to_cells(Hp, Gbars, Ubar)
    return _down_T(Hp, Ubar)


def composite_divergence_T(Hw, Lam):
    """Transpose of proj.composite_divergence as a map between valid cells:
    Lam[l] (read on valid cells) -> [per-level adjoint of w_d for d]."""
    D, nl = Hw.dim, Hw.nlev
    lam = [np.where(Hw.valid[l], Lam[l], 0.0) for l in range(nl)]
    Wbar = [[lev.zeros() for lev in Hw.levels] for _ in range(D)]
    Gbar = [[{(e, s): lev.zeros() for e in range(D) for s in (0, 1)} for lev in Hw.levels] for _ in range(D)]
    # refluxing (adjoint): out[l-1][pos] += sg (mean of fine face averages
    # - coarse face average) / hc, each face average eq. cell2face row 1
    fw = [-1.0, 7.0, 7.0, -1.0]  # (12 x) weights on the cells at offsets -1, 0, 1, 2 of a high face
    for l in range(1, nl):
        fine, coarse = Hw.levels[l], Hw.levels[l - 1]
        hc = coarse.h
        for pos, d, s in Hw.cf_faces(l):
            t = lam[l - 1][pos] * (1 if s else -1) / hc
            if t == 0.0:
                continue
            i = np.array(pos) - PAD

            def add(level, lv, q, side, wgt):
                # a value of the level, or the ghost of the given side that
                # the forward read there
                q = tuple(q)
                if lv.mask[q]:
                    Wbar[d][level][q] += wgt
                else:
                    Gbar[d][level][(d, side)][q] += wgt
            offs = [-1, 0, 1, 2] if s else [-2, -1, 0, 1]
            for o, wv in zip(offs, fw):
                q = np.array(pos)
                q[d] += o
                add(l - 1, coarse, q, 1 if o > 0 else 0, -t * wv / 12.0)
            rr = Hw.ratio
            jd = rr * i[d] + (rr if s else 0)
            trans = [e for e in range(D) if e != d]
            nf = rr ** (D - 1)
            for off in np.ndindex(*(rr,) * (D - 1)):
                q = np.zeros(D, int)
                q[d] = jd
                for e, o in zip(trans, off):
                    q[e] = rr * i[e] + o
                for delta, wv in zip((-2, -1, 0, 1), fw):
                    r = q.copy()
                    r[d] += delta
                    add(l, fine, r + PAD, 1 if delta >= 0 else 0, t * wv / (12.0 * nf))
    # per-level stencils and the ghosts of every component
    for d in range(D):
        for l, lev in enumerate(Hw.levels):
            Wbar[d][l] += _grad_T_level(lev, lam[l], d, Gbar[d][l])
        _ghost_adjoints_to_cells(Hw, Gbar[d], Wbar[d])
    return [_down_T(Hw, Wbar[d]) for d in range(D)]


def composite_project_T(H, Ubar, tol_rel=1e-12, max_cycles=200, smoother="jacobi"):
    """P^T ubar for the composite projection of proj.composite_project
    (homogeneous velocity data), as a map between valid cells."""
    Hw, Hp = proj.hierarchy_with(H, "D"), proj.hierarchy_with(H, "N")
    g = composite_gradient_T(Hp, Ubar)
    lam, st = amr_adj.composite_solve_T(Hp, g, "poisson", 0.0, tol_rel=tol_rel, max_cycles=max_cycles,
                                         smoother=smoother)
    dt = composite_divergence_T(Hw, lam)
    out = [[np.where(H.valid[l], Ubar[d][l] - dt[d][l], 0.0) for l in range(H.nlev)] for d in range(H.dim)]
    return out, lam, st


def valid_dot(H, A, B):
    """Plain sum over the valid cells of every level of A * B (per-level
    arrays)."""
    return float(sum((A[l][H.valid[l]] * B[l][H.valid[l]]).sum() for l in range(H.nlev)))

