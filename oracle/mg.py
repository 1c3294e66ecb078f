"""Oracle: geometric multigrid for the level systems, Section 6.5, and the
outer residual-correction loop with per-component solvability.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

What the paper fixes (Section 6.5): restriction by "injection", prolongation
by "linear interpolation", weighted Jacobi with omega = 2/3 as the smoother.
The readings taken where it is silent:

* restriction of cell averages = the mean of the 2^D children, i.e. eq.
  (AMR_avergingDownToCrse) applied to residuals;
* prolongation = face-neighbour linear interpolation,
  e_child = (1 - D/4) e_P + 1/4 sum_d e_{P +- e_d}, the neighbour taken on the
  child's side; it reproduces linear functions and reads only the first
  (homogeneous) ghost layer of the coarse correction;
* Jacobi and red-black use the diagonal with the ghost fill folded in;
* red-black colours by the parity of the sum of global indices; each
  half-sweep updates its colour simultaneously (omega = 1), ghosts refilled
  before every sweep and half-sweep, red first;
* the coarsest depth is solved exactly (dense FP64 solve; for a component
  with a constant null vector, bordered with one zero-mean constraint);
* stopping: ||r_k||_inf <= max(tol_rel ||r_0||_inf, tol_abs), max-norm over
  the cells of the level (the composite max norm of Section 7).
"""
import numpy as np

from .level import PAD


def restrict(fine, r, coarse):
    """Mean of the 2^D children of every coarse cell."""
    out = coarse.zeros()
    n = fine.shape
    rin = r[fine.inner]
    acc = np.zeros(tuple(m // 2 for m in n))
    D = fine.dim
    for corner in np.ndindex(*(2,) * D):
        acc += rin[tuple(slice(a, None, 2) for a in corner)]
    out[coarse.inner] = acc / 2 ** D
    out[~coarse.mask] = 0.0
    return out


def prolong(coarse, ec, fine):
    """Face-neighbour linear interpolation of a coarse correction (with its
    homogeneous ghosts) to the fine cells."""
    G = coarse.ghosts(ec)
    D = fine.dim
    out = fine.zeros()
    fin = out[fine.inner]
    for corner in np.ndindex(*(2,) * D):
        val = (1.0 - D / 4.0) * ec
        for d in range(D):
            k = 1 if corner[d] == 1 else -1
            val = val + 0.25 * coarse.neighbour(ec, G, d, k)
        fin[tuple(slice(a, None, 2) for a in corner)] = val[coarse.inner]
    out[~fine.mask] = 0.0
    return out


def _A(lev, u, op, c, transpose):
    return lev.apply_T(u, op, c) if transpose else lev.apply(u, op, c)


def jacobi(lev, e, f, op, c, D, omega, nsweeps, transpose=False):
    for _ in range(nsweeps):
        r = f - _A(lev, e, op, c, transpose)
        e = e + omega * r / D
        e[~lev.mask] = 0.0
    return e


def red_black(lev, e, f, op, c, D, nsweeps, transpose=False, omega=1.0):
    """Red-black half-sweeps (reading R-4): each colour in turn takes omega
    times its Jacobi correction from the current iterate (omega = 1: plain;
    > 1 over-relaxed)."""
    red = lev.colour() & lev.mask
    black = ~lev.colour() & lev.mask
    for _ in range(nsweeps):
        for sel in (red, black):
            r = f - _A(lev, e, op, c, transpose)
            e = e.copy()
            e[sel] += omega * r[sel] / D[sel]
    return e


def assemble(lev, op, c):
    """Dense matrix of the homogeneous operator on the masked cells, column j
    obtained by applying it to the j-th unit vector (probing)."""
    cells = np.argwhere(lev.mask)
    n = len(cells)
    M = np.zeros((n, n))
    for j, cell in enumerate(cells):
        e = lev.zeros()
        e[tuple(cell)] = 1.0
        M[:, j] = lev.apply(e, op, c)[lev.mask]
    return M, cells


class Bottom:
    """Exact solve on the coarsest depth (the bottom solver of Section 6.5
    replaced by a direct FP64 solve).  transpose: solve with the transposed
    matrix (the adjoint system); the zero-mean border is the same."""

    def __init__(self, lev, op, c, transpose=False):
        self.lev = lev
        M, self.cells = assemble(lev, op, c)
        if transpose:
            M = M.T.copy()
        self.sing = lev.singular_components(op)
        n = M.shape[0]
        k = len(self.sing)
        B = np.zeros((n, k))
        lab = lev.labels[lev.mask]
        for j, comp in enumerate(self.sing):
            B[lab == comp, j] = 1.0
        self.K = np.block([[M, B], [B.T, np.zeros((k, k))]])
        self.n = n

    def solve(self, f):
        rhs = np.concatenate([f[self.lev.mask], np.zeros(self.K.shape[0] - self.n)])
        sol = np.linalg.solve(self.K, rhs)
        e = self.lev.zeros()
        e[self.lev.mask] = sol[: self.n]
        return e


def ilu0(K, drop=1e-12):
    """ILU(0) of the square matrix K (dense array) on its own pattern: the
    diagonal and the entries whose magnitude exceeds drop times the largest
    of their row (a bordered system's zero corner is a pivot too).
    Gaussian elimination in the i-k-j order (Saad, Iterative Methods, Alg.
    10.4) in which only positions of the pattern are ever written.  Returns
    the combined factors: strictly lower part of L (unit diagonal implied)
    and U on and above the diagonal, zero off the pattern."""
    n = K.shape[0]
    pat = (np.abs(K) > drop * np.abs(K).max(axis=1, keepdims=True)) | np.eye(n, dtype=bool)
    LU = np.where(pat, K, 0.0).astype(float)
    for i in range(1, n):
        for k in range(i):
            if not pat[i, k]:
                continue
            LU[i, k] /= LU[k, k]
            for j in range(k + 1, n):
                if pat[i, j]:
                    LU[i, j] -= LU[i, k] * LU[k, j]
    return LU


def ilu_apply(LU, v):
    """z = (L U)^-1 v: forward substitution with the unit lower factor, then
    back substitution with the upper one."""
    n = LU.shape[0]
    y = np.zeros(n)
    for i in range(n):
        y[i] = v[i] - LU[i, :i] @ y[:i]
    z = np.zeros(n)
    for i in range(n - 1, -1, -1):
        z[i] = (y[i] - LU[i, i + 1:] @ z[i + 1:]) / LU[i, i]
    return z


def gmres_right(K, b, LU, m, breakdown=1e-14):
    """m steps of GMRES from x0 = 0, preconditioned on the right by the ILU
    factors (Saad, Alg. 9.5): Arnoldi with modified Gram-Schmidt on
    K (LU)^-1, the least-squares problem min ||beta e1 - H y||, then
    x = (LU)^-1 V y.  Stops early when the new Arnoldi vector's norm falls
    below breakdown times ||b|| (the Krylov space is invariant)."""
    n = len(b)
    beta = float(np.linalg.norm(b))
    if beta == 0.0:
        return np.zeros(n)
    V = np.zeros((n, m + 1))
    H = np.zeros((m + 1, m))
    V[:, 0] = b / beta
    k = m
    for j in range(m):
        w = K @ ilu_apply(LU, V[:, j])
        for i in range(j + 1):
            H[i, j] = w @ V[:, i]
            w = w - H[i, j] * V[:, i]
        H[j + 1, j] = float(np.linalg.norm(w))
        if H[j + 1, j] <= breakdown * beta:
            k = j + 1
            break
        V[:, j + 1] = w / H[j + 1, j]
    rhs = np.zeros(k + 1)
    rhs[0] = beta
    y = np.linalg.lstsq(H[:k + 1, :k], rhs, rcond=None)[0]
    return ilu_apply(LU, V[:, :k] @ y)


class IluGmresBottom:
    """The paper's bottom solver for the pressure systems (Section 6.5):
    ILU(0)-preconditioned GMRES(m) at the coarsest depth, m steps from zero
    per call.  Each face-connected component is its own system (they do not
    couple), its unknowns ordered box by box in the level's box order, x
    fastest within a box; a component on which the operator has a constant
    null vector is bordered with one zero-mean constraint (last unknown)."""

    def __init__(self, lev, op, c, m):
        self.lev, self.m = lev, m
        M, cells = assemble(lev, op, c)
        pos = {tuple(q): i for i, q in enumerate(cells)}
        sing = set(lev.singular_components(op))
        self.systems = []
        for comp in range(lev.ncomp):
            order = []
            for lo, hi in lev.boxes:
                first = tuple(PAD + v for v in lo)
                if lev.labels[first] != comp:
                    continue
                rng = [range(PAD + a, PAD + b + 1) for a, b in zip(lo, hi)]
                for q in np.ndindex(*[len(r) for r in rng][::-1]):  # last axis slowest
                    order.append(pos[tuple(r[qi] for r, qi in zip(rng, q[::-1]))])
            idx = np.array(order)
            K = M[np.ix_(idx, idx)]
            if comp in sing:
                n = len(idx)
                K = np.block([[K, np.ones((n, 1))], [np.ones((1, n)), np.zeros((1, 1))]])
            self.systems.append((idx, K, ilu0(K), comp in sing))
        self.cells = cells

    def solve(self, f):
        fv = f[self.lev.mask]
        out = np.zeros(len(fv))
        for idx, K, LU, sing in self.systems:
            b = np.concatenate([fv[idx], [0.0]]) if sing else fv[idx]
            x = gmres_right(K, b, LU, self.m)
            out[idx] = x[: len(idx)]
        e = self.lev.zeros()
        e[self.lev.mask] = out
        return e


class MG:
    """V(nu1, nu2) cycle on the multigrid depths of one level.

    transpose=True gives the V-cycle of the adjoint system: the transposed
    operator at every depth (same diagonal, since a matrix and its transpose
    share it), the same restriction and prolongation, the transposed bottom
    matrix."""

    def __init__(self, lev, op, c, nu1=2, nu2=2, smoother="jacobi", omega=2.0 / 3.0, transpose=False,
                 bottom_cells=0, omega_rb=1.0, bottom="exact", bottom_iters=5):
        self.levels = lev.hierarchy(bottom_cells)
        self.op, self.c = op, c
        self.transpose = transpose
        self.nu1, self.nu2, self.smoother, self.omega, self.omega_rb = nu1, nu2, smoother, omega, omega_rb
        self.D = [l.diagonal(op, c) for l in self.levels]
        self.sing = [l.singular_components(op) for l in self.levels]
        if bottom == "ilu_gmres" and not transpose:
            self.bottom = IluGmresBottom(self.levels[-1], op, c, bottom_iters)
        else:
            self.bottom = Bottom(self.levels[-1], op, c, transpose)

    def smooth(self, k, e, f, n):
        lev = self.levels[k]
        if self.smoother == "jacobi":
            return jacobi(lev, e, f, self.op, self.c, self.D[k], self.omega, n, self.transpose)
        return red_black(lev, e, f, self.op, self.c, self.D[k], n, self.transpose, self.omega_rb)

    def vcycle(self, f, k=0):
        """Correction e with A_hom e ~= f on depth k (homogeneous ghosts)."""
        lev = self.levels[k]
        if k == len(self.levels) - 1:
            return self.bottom.solve(f)
        e = self.smooth(k, lev.zeros(), f, self.nu1)
        r = f - _A(lev, e, self.op, self.c, self.transpose)
        coarse = self.levels[k + 1]
        fc = restrict(lev, r, coarse)
        fc = coarse.comp_mean(fc, self.sing[k + 1])
        ec = self.vcycle(fc, k + 1)
        e = e + prolong(coarse, ec, lev)
        return self.smooth(k, e, f, self.nu2)


def solvability_shift(lev, f, fd, comps):
    """RHS shift so that on each listed component the sum of h^D f equals the
    sum of h^(D-1) g over its boundary faces (the discrete compatibility
    condition eq. velocity_disc_solvabilityCond, enforced on the right-hand
    side; the data g is the outward normal derivative).  Returns the shifted
    RHS and the defect of each component before the shift."""
    hD = lev.h ** lev.dim
    bsum = np.zeros(lev.ncomp)
    for d in range(lev.dim):
        for s in (0, 1):
            end = lev.row_end(d, s) & (lev.end_kind(d, s) != "P")  # periodic ends take no data
            if fd is not None:
                np.add.at(bsum, lev.labels[end], fd[(d, s)][end] * lev.h ** (lev.dim - 1))
    out = f.copy()
    defects = []
    for c in comps:
        sel = lev.labels == c
        defect = hD * f[sel].sum() - bsum[c]
        defects.append(defect)
        out[sel] -= defect / (sel.sum() * hD)
    return out, defects


def cf_delta_correction(lev, f, fd, comps):
    """Solvability by correcting the coarse-fine face data (eq.
    correctingFaceAvg): on each listed component that has coarse-fine
    (non-physical) Neumann faces, one constant delta is added to the face
    data of all of them so that the sum of h^D f equals the sum of
    h^(D-1) g over the component's boundary faces; a component without such
    faces takes the RHS shift instead.  Returns (f, fd, defects)."""
    hD, hD1 = lev.h ** lev.dim, lev.h ** (lev.dim - 1)
    fd = {k: (v.copy() if fd is not None else lev.zeros()) for k, v in (fd or lev.zero_face_data()).items()}
    f = f.copy()
    defects = []
    for c in comps:
        sel = lev.labels == c
        bsum, ncf = 0.0, 0
        cf_ends = []
        for d in range(lev.dim):
            for s in (0, 1):
                end = lev.row_end(d, s) & sel
                bsum += fd[(d, s)][end].sum() * hD1
                cf = end & ~lev.end_is_physical(d, s) & (lev.end_kind(d, s) == "N")
                ncf += int(cf.sum())
                cf_ends.append(((d, s), cf))
        defect = hD * f[sel].sum() - bsum
        defects.append(defect)
        if ncf:
            delta = defect / (hD1 * ncf)
            for k, cf in cf_ends:
                fd[k][cf] += delta
        else:
            f[sel] -= defect / (sel.sum() * hD)
    return f, fd, defects


def norm_inf(lev, a):
    return float(np.abs(a[lev.mask]).max()) if lev.ncells else 0.0


def solve(lev, f, op, c, fd=None, cfv=None, x0=None, nu1=2, nu2=2, smoother="jacobi",
          omega=2.0 / 3.0, tol_rel=1e-10, tol_abs=0.0, max_cycles=50, shift=True, mg=None, transpose=False,
          cf_delta=False, bottom_cells=0, omega_rb=1.0):
    """Outer residual-correction loop in FP64:
    r = f - A(x); s = ||r||_inf; e = V(r / s); x += s e; remove the mean of x
    on every singular component; stop by the max-norm criterion above.

    transpose=True solves the adjoint system A_hom^T x = f (homogeneous: no
    face data); on a singular component the right-hand side is first made
    mean-free, which is the RHS shift with zero face data."""
    if transpose and (fd is not None or cfv is not None):
        raise ValueError("the adjoint system is homogeneous")
    mg = mg or MG(lev, op, c, nu1, nu2, smoother, omega, transpose, bottom_cells, omega_rb)
    sing = mg.sing[0]
    defects = []
    if shift and sing and cf_delta:
        f, fd, defects = cf_delta_correction(lev, f, fd, sing)
    elif shift and sing:
        f, defects = solvability_shift(lev, f, fd, sing)
    x = lev.zeros() if x0 is None else x0.copy()
    hist = []
    r = f - _A(lev, x, op, c, transpose) if transpose else f - lev.apply(x, op, c, fd, cfv)
    r0 = norm_inf(lev, r)
    hist.append(r0)
    target = max(tol_rel * r0, tol_abs)
    cycles = 0
    while hist[-1] > target and cycles < max_cycles:
        r = lev.comp_mean(r, sing)
        s = norm_inf(lev, r)
        e = mg.vcycle(r / s)
        x = x + s * e
        x = lev.comp_mean(x, sing)
        r = f - _A(lev, x, op, c, transpose) if transpose else f - lev.apply(x, op, c, fd, cfv)
        hist.append(norm_inf(lev, r))
        cycles += 1
    return x, {"cycles": cycles, "history": hist, "converged": hist[-1] <= target,
               "defects": defects, "rhs": f, "fd": fd}


def direct_solve(lev, f, op, c, fd=None, cfv=None):
    """Referee for tiny grids: x = M^{-1}(f - b) where A x = M x + b is the
    affine operator assembled by probing; singular components bordered with
    a zero-mean constraint, the RHS shifted for solvability first."""
    sing = lev.singular_components(op)
    if sing:
        f, _ = solvability_shift(lev, f, fd, sing)
    b = lev.apply(lev.zeros(), op, c, fd, cfv)
    bot = Bottom(lev, op, c)
    return bot.solve(f - b)


def grad_c(lev, lam, u, fd=None, cfv=None):
    """Derivative of a loss J(u) with respect to the Helmholtz coefficient c,
    u the solution of (I - cL) u = f with data fd: differentiating
    u - c L(u) = f gives (I - c L_hom) du/dc = L(u), so
    dJ/dc = <lam, L(u)> with lam the adjoint solution for dJ/du and L(u) the
    Laplacian of u with its data (sum over the level's cells)."""
    Lu = lev.laplacian(u, lev.ghosts(u, fd, cfv))
    return float((lam[lev.mask] * Lu[lev.mask]).sum())
