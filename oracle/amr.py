"""Oracle: composite operators over an AMR hierarchy (Sections 5.2-5.3) and
the composite solve.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings taken where the paper points to other papers:

* Coarse-fine interpolation (AMRCFI, Section 5.2): the paper fixes only that
  it is polynomial, fifth-order, conservative, a fixed matrix per relative
  position, from coarse data.  Reading: a tensor product, per direction, of
  the quartic whose averages over five consecutive coarse cells equal the
  data; the child's value is the average of that quartic over the child.
  The five-cell window is centred on the parent and shifted by the least
  amount that keeps it inside the domain; the whole tensor window must lie
  in the coarse level (else the layout is rejected).
* Refluxing (COH-3): at a valid coarse cell, the coarse flux through a face
  that borders the next finer level is replaced by the mean of the fine
  fluxes through the fine faces covering it; every flux is the fourth-order
  face derivative of eq. (cell2face), fine ones taken with the interpolated
  ghosts.
* Average-down (COH-4, eq. AMR_avergingDownToCrse) puts on every coarse cell
  covered by the next level the mean of its r^D children (r the refinement
  ratio, 2 or 4).
* Composite solve (the paper cites an adaptive multigrid for the inverse of
  the composite operator): multiplicative correction by levels in V order,
  finest to level 1, then level 0, then level 1 to finest.  Each correction
  of level l recomputes the composite residual (data averaged down first,
  covered cells carrying the averaged finer residual), runs one V-cycle of
  level l's own multigrid on it (interpolated ghosts of a correction are
  zero), adds the correction to level l and its face-neighbour linear
  prolongation to every finer level.  After the sweep the data is averaged
  down.  (Correcting the fine levels only once per cycle, after level 0,
  diverges when a fine box sits in a corner of a Dirichlet domain: the fine
  correction ignores how its own values reach its interpolated ghosts
  through the averaged-down coarse cells.)
"""
from fractions import Fraction as Fr

import numpy as np

from . import fv, mg
from .level import PAD, Level, _shift


# ---------------------------------------------------------------------------
# AMRCFI weights
def _moment_matrix():
    """M[m][k] = average of x^k over the unit cell [m, m+1], m, k = 0..4."""
    return [[Fr((m + 1) ** (k + 1) - m ** (k + 1), k + 1) for k in range(5)] for m in range(5)]


def _solve_fraction(A, b):
    """Gaussian elimination in exact arithmetic (A square, list of lists)."""
    n = len(A)
    M = [list(row) + [bi] for row, bi in zip(A, b)]
    for c in range(n):
        p = next(r for r in range(c, n) if M[r][c] != 0)
        M[c], M[p] = M[p], M[c]
        for r in range(n):
            if r != c and M[r][c] != 0:
                f = M[r][c] / M[c][c]
                M[r] = [x - f * y for x, y in zip(M[r], M[c])]
    return [M[r][n] / M[r][r] for r in range(n)]


def cfi_weights_1d(shift, child, ratio=2):
    """Weights on the five window cells (left to right) giving the average,
    over child `child` (0 .. ratio-1 from the low end) of the parent, of the
    quartic with the given cell averages.  The window is the parent's cell
    moved by `shift` cells: window cell m = 0..4 covers [m, m+1] and the
    parent is window cell 2 - shift."""
    M = _moment_matrix()
    mp = 2 - shift
    x0 = Fr(mp) + Fr(child, ratio)
    x1 = x0 + Fr(1, ratio)
    # average of x^k over [x0, x1]
    c = [(x1 ** (k + 1) - x0 ** (k + 1)) / (k + 1) / (x1 - x0) for k in range(5)]
    # child average = c . a, with M a = U  =>  weights w = M^-T c
    MT = [[M[m][k] for m in range(5)] for k in range(5)]
    return _solve_fraction(MT, c)


_WR = {}


def weights(ratio):
    """{(shift, child): the five AMRCFI weights} for refinement ratio `ratio`."""
    if ratio not in _WR:
        _WR[ratio] = {(s, a): np.array([float(v) for v in cfi_weights_1d(s, a, ratio)])
                      for s in range(-2, 3) for a in range(ratio)}
    return _WR[ratio]


_W = weights(2)


def restrict_ratio(fine, r, coarse, ratio):
    """Mean of the ratio^D children of every coarse cell (average-down)."""
    rin = r[fine.inner]
    acc = np.zeros(coarse.shape)
    for corner in np.ndindex(*(ratio,) * fine.dim):
        acc += rin[tuple(slice(a, None, ratio) for a in corner)]
    out = coarse.zeros()
    out[coarse.inner] = acc / ratio ** fine.dim
    out[~coarse.mask] = 0.0
    return out


def prolong_ratio(coarse, ec, fine, ratio):
    """Face-neighbour linear interpolation of a coarse correction onto the
    children of a refinement by `ratio`: a child whose centre lies delta_d
    (in parent widths) from the parent's centre along d takes
    (1 - sum_d |delta_d|) e_P + sum_d |delta_d| e_(P + sign(delta_d) e_d)
    (ratio 2: delta = +-1/4, the multigrid prolongation)."""
    if ratio == 2:
        return mg.prolong(coarse, ec, fine)
    G = coarse.ghosts(ec)
    D = fine.dim
    out = fine.zeros()
    fin = out[fine.inner]
    nb = {(d, k): coarse.neighbour(ec, G, d, k) for d in range(D) for k in (-1, 1)}
    for corner in np.ndindex(*(ratio,) * D):
        delta = [(a + 0.5) / ratio - 0.5 for a in corner]
        val = (1.0 - sum(abs(t) for t in delta)) * ec
        for d in range(D):
            val = val + abs(delta[d]) * nb[(d, 1 if delta[d] > 0 else -1)]
        fin[tuple(slice(a, None, ratio) for a in corner)] = val[coarse.inner]
    out[~fine.mask] = 0.0
    return out


def window_shift(P, n):
    """Least shift keeping the five-cell window around coarse cell P inside
    [0, n)."""
    if P < 2:
        return 2 - P
    if P > n - 3:
        return (n - 3) - P
    return 0


# ---------------------------------------------------------------------------
class Hierarchy:
    """Levels 0..lmax of a block-structured hierarchy with refinement ratio
    `ratio` (2 or 4, eq. grids) between consecutive levels.

    base_shape : cells of level 0 per direction; h0 its cell size
    boxes      : list per level of (lo, hi) boxes (level 0 covers the grid)
    phys_bc    : {(d, s): 'D' | 'N' | 'P'} (a level above 0 may not touch a
                 periodic side)
    """

    def __init__(self, base_shape, h0, boxes, phys_bc, ratio=2):
        r = self.ratio = int(ratio)
        self.levels = []
        for l, bl in enumerate(boxes):
            shape = tuple(n * r ** l for n in base_shape)
            self.levels.append(Level(shape, h0 / r ** l, bl, phys_bc, "I" if l else "D"))
        self.dim = len(base_shape)
        self.nlev = len(self.levels)
        # covered[l]: cells of level l under level l+1
        self.covered = []
        for l in range(self.nlev):
            cov = np.zeros(self.levels[l].pshape, bool)
            if l + 1 < self.nlev:
                for lo, hi in self.levels[l + 1].boxes:
                    sl = tuple(slice(PAD + a // r, PAD + (b + 1) // r) for a, b in zip(lo, hi))
                    cov[sl] = True
            self.covered.append(cov)
        self.valid = [self.levels[l].mask & ~self.covered[l] for l in range(self.nlev)]
        self._check_nesting()

    def _check_nesting(self):
        for l in range(1, self.nlev):
            fine, coarse = self.levels[l], self.levels[l - 1]
            r = self.ratio
            for lo, hi in fine.boxes:
                if any(v % r for v in lo) or any((v + 1) % r for v in hi):
                    raise ValueError("level %d is not properly refined" % l)
            # every fine cell's parent is a cell of the coarse level
            par = np.zeros(coarse.pshape, bool)
            for lo, hi in fine.boxes:
                par[tuple(slice(PAD + a // r, PAD + (b + 1) // r) for a, b in zip(lo, hi))] = True
            if np.any(par & ~coarse.mask):
                raise ValueError("level %d is not nested in level %d" % (l, l - 1))

    # -- coarse-fine interpolation --------------------------------------
    def cf_positions(self, l):
        """Fine positions that serve as interpolated ghosts of level l: not
        in the level, inside the domain, one or two cells along an axis from
        a level cell."""
        lev = self.levels[l]
        near = np.zeros(lev.pshape, bool)
        for d in range(lev.dim):
            for k in (-2, -1, 1, 2):
                near |= _shift(lev.mask, d, k)
        return near & ~lev.mask & lev.inside

    def amrcfi(self, l, Uc):
        """Interpolated ghost values of level l (padded array, zero elsewhere)
        from the coarse level's data Uc (its covered cells must hold the
        averaged-down data)."""
        fine, coarse = self.levels[l], self.levels[l - 1]
        out = fine.zeros()
        D = fine.dim
        for pos in np.argwhere(self.cf_positions(l)):
            g = pos - PAD
            P = g // self.ratio
            a = g % self.ratio
            shifts = [window_shift(int(P[d]), coarse.shape[d]) for d in range(D)]
            lo = [int(P[d]) + shifts[d] - 2 for d in range(D)]
            win = Uc[tuple(slice(PAD + lo[d], PAD + lo[d] + 5) for d in range(D))]
            wm = coarse.mask[tuple(slice(PAD + lo[d], PAD + lo[d] + 5) for d in range(D))]
            if not wm.all():
                raise ValueError("interpolation window leaves level %d" % (l - 1))
            val = win
            for d in range(D):
                w = weights(self.ratio)[(shifts[d], int(a[d]))]
                val = np.tensordot(w, val, axes=([0], [0]))
            out[tuple(pos)] = float(val)
        return out

    # -- transfers --------------------------------------------------------
    def average_down(self, U, l):
        """Covered cells of level l-1 := mean of their children on level l."""
        fine, coarse = self.levels[l], self.levels[l - 1]
        avg = restrict_ratio(fine, np.where(fine.mask, U[l], 0.0), coarse, self.ratio)
        cov = self.covered[l - 1]
        U[l - 1] = np.where(cov, avg, U[l - 1])

    def average_down_all(self, U):
        U = [u.copy() for u in U]
        for l in range(self.nlev - 1, 0, -1):
            self.average_down(U, l)
        return U

    # -- composite operator ----------------------------------------------
    def cf_faces(self, l):
        """Faces between a valid cell of level l-1 and a cell covered by
        level l: list of (coarse cell index tuple (padded), d, s)."""
        coarse = self.levels[l - 1]
        cov = self.covered[l - 1]
        faces = []
        for d in range(coarse.dim):
            for s in (0, 1):
                k = 1 if s else -1
                sel = self.valid[l - 1] & _shift(cov, d, k)
                for pos in np.argwhere(sel):
                    faces.append((tuple(pos), d, s))
        return faces

    def composite_apply(self, U, op, c, fd=None):
        """A^comp U per level (COH-1..4).  U: padded arrays, covered cells
        holding averaged-down data.  fd: per-level physical face data (None =
        zero).  Returns per-level arrays; covered cells hold the average of
        the finer level's values."""
        L, G = [], []
        for l, lev in enumerate(self.levels):
            cfv = self.amrcfi(l, U[l - 1]) if l else None
            Gl = lev.ghosts(U[l], fd[l] if fd else None, cfv)
            G.append(Gl)
            L.append(lev.laplacian(U[l], Gl))
        for l in range(1, self.nlev):
            self._reflux(l, U, G, L)
        A = []
        for l, lev in enumerate(self.levels):
            a = U[l] - c * L[l] if op == "helmholtz" else L[l]
            A.append(np.where(lev.mask, a, 0.0))
        for l in range(self.nlev - 1, 0, -1):
            self.average_down(A, l)
        return A

    def _reflux(self, l, U, G, L):
        fine, coarse = self.levels[l], self.levels[l - 1]
        D = coarse.dim
        hc, hf = coarse.h, fine.h
        for pos, d, s in self.cf_faces(l):
            i = np.array(pos) - PAD
            k = 1 if s else -1

            def cval(off):
                q = np.array(pos)
                q[d] += off
                q = tuple(q)
                if coarse.mask[q]:
                    return U[l - 1][q]
                side = 1 if off > 0 else 0
                return G[l - 1][(d, side)][q]

            # coarse face derivative through the face (in +e_d direction)
            if s:  # face i + 1/2
                Fc = fv.face_derivative(cval(-1), cval(0), cval(1), cval(2), hc)
            else:  # face i - 1/2
                Fc = fv.face_derivative(cval(-2), cval(-1), cval(0), cval(1), hc)
            # fine faces covering it
            r = self.ratio
            jd = r * i[d] + (r if s else 0)  # fine index of the first cell past the face (+e_d side)
            tot = 0.0
            nf = 0
            trans = [e for e in range(D) if e != d]
            for off in np.ndindex(*(r,) * (D - 1)):
                q = np.zeros(D, int)
                q[d] = jd
                for e, o in zip(trans, off):
                    q[e] = r * i[e] + o

                def fval(delta):
                    qq = q.copy()
                    qq[d] += delta
                    t = tuple(qq + PAD)
                    if fine.mask[t]:
                        return U[l][t]
                    side = 1 if delta >= 0 else 0
                    return G[l][(d, side)][t]
                # face between fine cells jd-1 and jd, derivative along +e_d
                tot += fv.face_derivative(fval(-2), fval(-1), fval(0), fval(1), hf)
                nf += 1
            Ff = tot / nf
            L[l - 1][pos] += (1 if s else -1) * (Ff - Fc) / hc

    # -- norms and means --------------------------------------------------
    def norm_inf(self, R):
        return max(float(np.abs(R[l][self.valid[l]]).max()) if self.valid[l].any() else 0.0
                   for l in range(self.nlev))

    def composite_mean(self, U):
        vol = sum(self.valid[l].sum() * self.levels[l].h ** self.dim for l in range(self.nlev))
        tot = sum(U[l][self.valid[l]].sum() * self.levels[l].h ** self.dim for l in range(self.nlev))
        return tot / vol

    def singular(self, op):
        return op == "poisson" and all(v in ("N", "P") for v in self.levels[0].phys_bc.values())

    def solvability_shift(self, f, fd):
        """Shift every level's right-hand side by one constant so that the
        volume sum over valid cells equals the boundary-flux sum."""
        D = self.dim
        bsum = 0.0
        for l, lev in enumerate(self.levels):
            if fd is None:
                break
            for d in range(D):
                for s in (0, 1):
                    phys = lev.end_is_physical(d, s) & (lev.end_kind(d, s) != "P")
                    bsum += fd[l][(d, s)][phys & self.valid[l]].sum() * lev.h ** (D - 1)
        vol = sum(self.valid[l].sum() * self.levels[l].h ** D for l in range(self.nlev))
        tot = sum(f[l][self.valid[l]].sum() * self.levels[l].h ** D for l in range(self.nlev))
        delta = (tot - bsum) / vol
        return [np.where(self.levels[l].mask, f[l] - delta, 0.0) for l in range(self.nlev)], tot - bsum


def composite_residual(H, U, f, op, c, fd=None):
    A = H.composite_apply(U, op, c, fd)
    R = [np.where(H.levels[l].mask, f[l] - A[l], 0.0) for l in range(H.nlev)]
    # covered cells carry the averaged residual of the finer level
    for l in range(H.nlev - 1, 0, -1):
        H.average_down(R, l)
    return R


def correct_level(H, U, f, op, c, fd, MGl, l, sing):
    """One correction of level l: composite residual, a V-cycle of level l's
    multigrid on it (scaled by its max norm), the correction added to level
    l and prolonged onto every finer level."""
    U = H.average_down_all(U)
    R = composite_residual(H, U, f, op, c, fd)
    rl = R[l]
    if l == 0 and sing:
        rl = H.levels[0].comp_mean(rl, [0])
    s = float(np.abs(rl[H.levels[l].mask]).max()) or 1.0
    e = MGl.vcycle(rl / s) * s
    U[l] = U[l] + e
    E = e
    for m in range(l + 1, H.nlev):
        dU = prolong_ratio(H.levels[m - 1], E, H.levels[m], H.ratio)
        U[m] = U[m] + dU
        E = dU
    return U


def composite_solve(H, f, op, c, fd=None, tol_rel=1e-10, tol_abs=0.0, max_cycles=100, nu1=2, nu2=2,
                    smoother="jacobi", shift=True, omega_rb=1.0):
    """The composite cycle described in the module docstring, from U = 0
    (omega_rb: the red-black relaxation factor of the level cycles)."""
    MG = [mg.MG(lev, op, c, nu1, nu2, smoother, omega_rb=omega_rb) for lev in H.levels]
    sing = H.singular(op)
    defect = 0.0
    if sing and shift:
        f, defect = H.solvability_shift(f, fd)
    U = [lev.zeros() for lev in H.levels]
    R = composite_residual(H, U, f, op, c, fd)
    hist = [H.norm_inf(R)]
    target = max(tol_rel * hist[0], tol_abs)
    order = list(range(H.nlev - 1, 0, -1)) + list(range(H.nlev))
    cycles = 0
    while hist[-1] > target and cycles < max_cycles:
        for l in order:
            U = correct_level(H, U, f, op, c, fd, MG[l], l, sing)
        U = H.average_down_all(U)
        if sing:
            m = H.composite_mean(U)
            U = [np.where(H.levels[l].mask, U[l] - m, 0.0) for l in range(H.nlev)]
        R = composite_residual(H, U, f, op, c, fd)
        hist.append(H.norm_inf(R))
        cycles += 1
    return U, {"cycles": cycles, "history": hist, "converged": hist[-1] <= target, "defect": defect}


def composite_direct(H, f, op, c, fd=None):
    """Referee for small hierarchies: the composite system on the valid cells
    assembled by probing, solved directly (with a zero-mean constraint for
    the pure-Neumann Poisson case)."""
    cells = [(l, tuple(p)) for l in range(H.nlev) for p in np.argwhere(H.valid[l])]
    n = len(cells)
    sing = H.singular(op)
    if sing:
        f, _ = H.solvability_shift(f, fd)

    def apply(vec, data):
        U = [lev.zeros() for lev in H.levels]
        for k, (l, p) in enumerate(cells):
            U[l][p] = vec[k]
        U = H.average_down_all(U)
        A = H.composite_apply(U, op, c, data)
        return np.array([A[l][p] for l, p in cells])

    b = apply(np.zeros(n), fd)
    M = np.zeros((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        M[:, j] = apply(e, None)
    rhs = np.array([f[l][p] for l, p in cells]) - b
    if sing:
        w = np.array([H.levels[l].h ** H.dim for l, _ in cells])
        K = np.block([[M, w[:, None]], [w[None, :], np.zeros((1, 1))]])
        x = np.linalg.solve(K, np.concatenate([rhs, [0.0]]))[:n]
    else:
        x = np.linalg.solve(M, rhs)
    U = [lev.zeros() for lev in H.levels]
    for k, (l, p) in enumerate(cells):
        U[l][p] = x[k]
    return H.average_down_all(U)
