"""Oracle: adjoint (transpose) of the composite operator over a hierarchy and
the composite adjoint solve (not in the paper).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The composite operator of Section 5.3 maps the values u_V on the valid cells
of all levels to (A^comp u)_V: extend u to the covered cells by averaging
down (COH-4), fill every level's ghosts (physical fills with zero data,
box-to-box copies, AMRCFI from the level below), apply each level's stencil,
reflux at valid coarse cells next to the finer level (COH-3), and take
u - cL (Helmholtz) or L (Poisson) on the valid cells.  Its transpose is the
reverse of these steps, each one transposed: the reflux spreads the output
adjoint of a coarse cell back onto the fine and coarse values and ghosts its
fluxes read; the stencil is applied to the adjoint extended by zero and
hands its weights on the ghosts to the ghost adjoints; physical fills send
those back onto the four cells they read; AMRCFI sends them back onto its
coarse window; and the adjoint of a covered cell goes to its children in
equal parts, coarse to fine.

Adjoint solve, multiplicative over levels in the order of the forward
composite cycle: each level correction runs one V-cycle of that level's
transposed multigrid on the transposed composite residual, adds it to the
level and its face-neighbour linear prolongation to the finer levels.  The
adjoint of a composite solution behaves like a cell integral rather than a
cell average (for a conservative operator A = W^-1 K with W the cell
volumes, A^T lam = g reads K W^-1 lam = g), so the transfers between levels
are the volume-weighted ones: a covered cell carries the SUM of its
children's residuals, and a correction prolonged to the next finer level is
divided by 2^D.  (With the forward transfers, mean and unscaled
prolongation, the cycle diverges on a three-level hierarchy.)
"""
import numpy as np

from . import fv, mg
from .amr import prolong_ratio, weights, window_shift
from .level import NEUMANN, DIRICHLET, PAD, PERIODIC, _shift, _wrap


def _scatter_fill(lev, Gbar, back):
    """Ghost adjoints of the physical (and face-data) fills of one level sent
    back onto the four cells each fill reads, with the fill weights."""
    unit = [[1.0 if m == j else 0.0 for m in range(4)] for j in range(4)]
    wd = [fv.dirichlet_ghosts(*unit[j], 0.0) for j in range(4)]
    wn = [fv.neumann_ghosts(*unit[j], 0.0, lev.h) for j in range(4)]
    for d in range(lev.dim):
        for s in (0, 1):
            step = 1 if s == 1 else -1
            end = lev.row_end(d, s)
            kinds = lev.end_kind(d, s)
            gb = Gbar[(d, s)]
            # ghost adjoint of the first / second ghost, seen at the row end;
            # a second ghost position that is a level cell is not a ghost
            mu1 = _shift(gb, d, step)
            mu2 = np.where(_shift(lev.mask, d, 2 * step), 0.0, _shift(gb, d, 2 * step))
            for kind, w in ((DIRICHLET, wd), (NEUMANN, wn)):
                sel = end & (kinds == kind)
                if not sel.any():
                    continue
                for j in range(4):
                    back += _shift(np.where(sel, w[j][0] * mu1 + w[j][1] * mu2, 0.0), d, j * step)
            # periodic ghosts copy the cells one and two steps on (mod n)
            sel = end & (kinds == PERIODIC)
            if sel.any():
                back += _wrap(np.where(sel, mu1, 0.0), d, -step)
                back += _wrap(np.where(sel, mu2, 0.0), d, -2 * step)


def _interp_ghost_adjoint(lev, Gbar):
    """Adjoint of the interpolated ghost values (one value per ghost cell,
    read through every (d, s) ghost array that holds it)."""
    cbar = lev.zeros()
    for d in range(lev.dim):
        for s in (0, 1):
            step = 1 if s == 1 else -1
            isi = lev.row_end(d, s) & (lev.end_kind(d, s) == "I")
            at1 = _shift(isi, d, -step)
            at2 = _shift(isi, d, -2 * step) & ~lev.mask
            cbar[at1] += Gbar[(d, s)][at1]
            cbar[at2] += Gbar[(d, s)][at2]
    return cbar


def _amrcfi_T(H, l, cbar):
    """Transpose of amrcfi(l, .): coarse-level adjoint from the interpolated
    ghost adjoints of level l."""
    fine, coarse = H.levels[l], H.levels[l - 1]
    out = coarse.zeros()
    D = fine.dim
    for pos in np.argwhere(H.cf_positions(l)):
        v = cbar[tuple(pos)]
        if v == 0.0:
            continue
        g = pos - PAD
        P = g // H.ratio
        a = g % H.ratio
        shifts = [window_shift(int(P[d]), coarse.shape[d]) for d in range(D)]
        lo = [int(P[d]) + shifts[d] - 2 for d in range(D)]
        w = np.array(1.0)
        for d in range(D):
            w = np.multiply.outer(w, np.array([float(x) for x in weights(H.ratio)[(shifts[d], int(a[d]))]]))
        sl = tuple(slice(PAD + lo[d], PAD + lo[d] + 5) for d in range(D))
        out[sl] += v * w
    return out


def composite_apply_T(H, Lam, op, c):
    """(A^comp)^T lam for lam on the valid cells of every level (other
    entries ignored); returns per-level arrays, zero off the valid cells."""
    nl, D = H.nlev, H.dim
    lam = [np.where(H.valid[l], Lam[l], 0.0) for l in range(nl)]
    Ubar = [lev.zeros() for lev in H.levels]
    Lbar = []
    for l, lev in enumerate(H.levels):
        if op == "helmholtz":
            Ubar[l] += lam[l]
            Lbar.append(-c * lam[l])
        elif op == "poisson":
            Lbar.append(lam[l].copy())
        else:
            raise ValueError(op)
    Gbar = [{(d, s): lev.zeros() for d in range(D) for s in (0, 1)} for lev in H.levels]
    # reflux (adjoint): L[l-1][pos] += sg (Ff - Fc) / hc
    for l in range(1, nl):
        fine, coarse = H.levels[l], H.levels[l - 1]
        hc, hf = coarse.h, fine.h
        for pos, d, s in H.cf_faces(l):
            t = Lbar[l - 1][pos] * (1 if s else -1) / hc
            if t == 0.0:
                continue
            i = np.array(pos) - PAD

            def add_c(off, wgt):
                q = np.array(pos)
                q[d] += off
                q = tuple(q)
                if coarse.mask[q]:
                    Ubar[l - 1][q] += wgt
                else:
                    Gbar[l - 1][(d, 1 if off > 0 else 0)][q] += wgt
            # Fc = (-v[+2] + 15 v[+1] - 15 v[0] + v[-1]) / 12hc on the face's cells
            cw = [1.0, -15.0, 15.0, -1.0]
            offs = [-1, 0, 1, 2] if s else [-2, -1, 0, 1]
            for o, wv in zip(offs, cw):
                add_c(o, -t * wv / (12 * hc))
            rr = H.ratio
            jd = rr * i[d] + (rr if s else 0)
            trans = [e for e in range(D) if e != d]
            nf = rr ** (D - 1)
            for off in np.ndindex(*(rr,) * (D - 1)):
                q = np.zeros(D, int)
                q[d] = jd
                for e, o in zip(trans, off):
                    q[e] = rr * i[e] + o
                for delta, wv in zip((-2, -1, 0, 1), cw):
                    r = q.copy()
                    r[d] += delta
                    tt = tuple(r + PAD)
                    val = t * wv / (12 * hf * nf)
                    if fine.mask[tt]:
                        Ubar[l][tt] += val
                    else:
                        Gbar[l][(d, 1 if delta >= 0 else 0)][tt] += val
    # level stencils (adjoint): symmetric stencil on Lbar extended by zero,
    # weights on ghost positions into the ghost adjoints
    k12 = [12.0 * lev.h ** 2 for lev in H.levels]
    for l, lev in enumerate(H.levels):
        zero = {(d, s): lev.zeros() for d in range(D) for s in (0, 1)}
        Ubar[l] += lev.laplacian(Lbar[l], zero)
        lb = np.where(lev.mask, Lbar[l], 0.0)
        for d in range(D):
            for s in (0, 1):
                step = 1 if s == 1 else -1
                # stencil at i reads position i + k step (k = 1 weight 16, k = 2 weight -1)
                contrib = 16.0 * _shift(lb, d, -step) - _shift(lb, d, -2 * step)
                Gbar[l][(d, s)] += np.where(lev.mask, 0.0, contrib) / k12[l]
    # ghosts (adjoint): physical fills onto the level, AMRCFI onto the level below
    for l in range(nl - 1, -1, -1):
        lev = H.levels[l]
        back = lev.zeros()
        _scatter_fill(lev, Gbar[l], back)
        Ubar[l] += np.where(lev.mask, back, 0.0)
        if l:
            Ubar[l - 1] += np.where(H.levels[l - 1].mask, _amrcfi_T(H, l, _interp_ghost_adjoint(lev, Gbar[l])), 0.0)
    # average-down (adjoint): covered adjoints to the children, coarse to fine
    for l in range(1, nl):
        fine, coarse = H.levels[l], H.levels[l - 1]
        cov = np.where(H.covered[l - 1], Ubar[l - 1], 0.0)
        Ubar[l] += np.where(fine.mask, _children(fine, coarse, cov, H.ratio), 0.0)
        Ubar[l - 1] = np.where(H.covered[l - 1], 0.0, Ubar[l - 1])
    return [np.where(H.valid[l], Ubar[l], 0.0) for l in range(nl)]


def _children(fine, coarse, a, ratio=2):
    """Fine array whose every cell holds 1/ratio^D of its parent's value in a."""
    out = fine.zeros()
    D = fine.dim
    ain = a[coarse.inner]
    fin = out[fine.inner]
    for corner in np.ndindex(*(ratio,) * D):
        fin[tuple(slice(k, None, ratio) for k in corner)] = ain / ratio ** D
    return out


def composite_residual_T(H, Lam, g, op, c):
    """g - A^T lam on the valid cells; a covered cell holds the sum of its
    children's values (finest first)."""
    AT = composite_apply_T(H, Lam, op, c)
    R = [np.where(H.valid[l], g[l] - AT[l], 0.0) for l in range(H.nlev)]
    for l in range(H.nlev - 1, 0, -1):
        H.average_down(R, l)
        R[l - 1] = np.where(H.covered[l - 1], R[l - 1] * H.ratio ** H.dim, R[l - 1])
    return R


def composite_solve_T(H, g, op, c, tol_rel=1e-10, tol_abs=0.0, max_cycles=100, nu1=2, nu2=2, smoother="jacobi"):
    """Adjoint composite solve (A^comp)^T lam = g on the valid cells, by the
    multiplicative level cycle described in the module docstring.

    Pure Neumann: A^comp has the constants as right null vector and the
    volume weights w (h_l^D per valid cell) as left null vector.  The forward
    solve shifts the right-hand side by a constant and returns the solution
    with zero volume-weighted mean, i.e. x = Z A^+ S f with
    S = Z = I - 1 w^T / (w^T 1); the gradient of J(x) in f is then
    S^T A^+T Z^T dJ/dx with S^T = Z^T = I - w 1^T / (w^T 1).  So the source
    is projected by Z^T (it then sums to zero) and lam by S^T (plain sum
    zero)."""
    MG = [mg.MG(lev, op, c, nu1, nu2, smoother, transpose=True) for lev in H.levels]
    sing = H.singular(op)
    g = [np.where(H.valid[l], g[l], 0.0) for l in range(H.nlev)]
    wts = [np.where(H.valid[l], H.levels[l].h ** H.dim, 0.0) for l in range(H.nlev)]
    wsum = sum(w.sum() for w in wts)

    def proj_w(a):
        tot = sum(a[l][H.valid[l]].sum() for l in range(H.nlev))
        return [np.where(H.valid[l], a[l] - wts[l] * tot / wsum, 0.0) for l in range(H.nlev)]

    if sing:
        g = proj_w(g)
    lam = [lev.zeros() for lev in H.levels]
    R = composite_residual_T(H, lam, g, op, c)
    hist = [H.norm_inf(R)]
    target = max(tol_rel * hist[0], tol_abs)
    order = list(range(H.nlev - 1, 0, -1)) + list(range(H.nlev))
    cycles = 0
    while hist[-1] > target and cycles < max_cycles:
        for l in order:
            R = composite_residual_T(H, lam, g, op, c)
            rl = R[l]
            if l == 0 and sing:
                rl = H.levels[0].comp_mean(rl, [0])
            s = float(np.abs(rl[H.levels[l].mask]).max()) or 1.0
            e = MG[l].vcycle(rl / s) * s
            lam[l] = lam[l] + np.where(H.valid[l], e, 0.0)
            E = e
            for m in range(l + 1, H.nlev):
                dU = prolong_ratio(H.levels[m - 1], E, H.levels[m], H.ratio) / H.ratio ** H.dim
                lam[m] = lam[m] + np.where(H.valid[m], dU, 0.0)
                E = dU
        if sing:
            lam = proj_w(lam)
        R = composite_residual_T(H, lam, g, op, c)
        hist.append(H.norm_inf(R))
        cycles += 1
    return lam, {"cycles": cycles, "history": hist, "converged": hist[-1] <= target}


def grad_c(H, Lam, U, fd=None):
    """dJ/dc for the composite Helmholtz solve: <lam, L^comp u> over the
    valid cells, L^comp u the composite Laplacian (refluxed) of the solution
    with its data (differentiate u - c L^comp u = f)."""
    Lu = H.composite_apply(H.average_down_all(U), "poisson", 0.0, fd)
    return float(sum((Lam[l] * Lu[l])[H.valid[l]].sum() for l in range(H.nlev)))
