"""Oracle: one refinement level of a block-structured AMR hierarchy.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Data model.  A level (or one multigrid depth of it) lives on a dense array
over the whole index space of its grid (Section 5.1, eq. grids), padded by
two cells on every side; a boolean mask marks the cells of the level's
boxes (eq. AMRHier).  Index ``i`` of the level maps to array position
``i + PAD``.  Axis d of an array is spatial direction d.

Ghost cells (Section 3, the paragraph on two ghost layers, and Figure 1(c)).
The stencils are axis-aligned, so a ghost value is only ever read along one
direction.  For every direction d and side s the oracle keeps a separate
ghost array ``G[(d, s)]``: where a row of masked cells along d ends at cell
e (e masked, e + s*e_d not), positions e + s*e_d and e + 2s*e_d receive the
first and second ghost of that row end.  The row end is on the physical
boundary when e + s*e_d lies outside the domain, and on the coarse-fine
interface otherwise.  Cells of other boxes of the same level are read
directly from the array (the exchange ghosts of Figure 1(c)).

Face data ``fd[(d, s)]`` holds, at the row-end cell e, the face average on
the face between e and e + s*e_d: the Dirichlet value, or the derivative
along the outward normal for Neumann (eqs. velBCHomoDiri5th, Neumann5).

Periodic boundaries (the domains of Section 7.3) pair the two sides of a
direction: a row end on such a side is kind 'P', and its first and second
ghosts are the cells of the level at e + s*e_d and e + 2s*e_d taken modulo
the grid size (cells of the level there are required); components connect
across the periodic boundary.
"""
import numpy as np
from scipy import ndimage

from . import fv

PAD = 2
DIRICHLET, NEUMANN, INTERP, PERIODIC = "D", "N", "I", "P"


def _shift(a, d, k):
    """b[i] = a[i + k e_d] on a padded array (wrap-around only touches
    positions that callers discard)."""
    return np.roll(a, -k, axis=d)


def _wrap(a, d, k):
    """b[i] = a[(i + k e_d) mod n] on the domain part of a padded array (the
    pad stays zero): the periodic neighbour."""
    inner = tuple(slice(PAD, -PAD) for _ in range(a.ndim))
    out = np.zeros_like(a)
    out[inner] = np.roll(a[inner], -k, axis=d)
    return out


class Level:
    """One level of the hierarchy, or one multigrid depth of one level.

    shape   : cells per direction of the level's whole grid (the domain)
    h       : cell size
    boxes   : list of (lo, hi) inclusive index tuples, eq. (AMRHier)
    phys_bc : {(d, s): 'D' | 'N' | 'P'} for the physical boundary, s = 0 low,
              1 high; 'P' (periodic) on both sides of a direction or neither
    cf_kind : 'D' | 'N' (face data on the coarse-fine interface, Definition
              6.1) or 'I' (ghosts from coarse-fine interpolation)
    """

    def __init__(self, shape, h, boxes, phys_bc, cf_kind=DIRICHLET):
        self.shape = tuple(int(n) for n in shape)
        self.dim = len(self.shape)
        self.h = float(h)
        self.boxes = [(tuple(int(v) for v in lo), tuple(int(v) for v in hi)) for lo, hi in boxes]
        self.phys_bc = dict(phys_bc)
        self.periodic = [d for d in range(self.dim) if self.phys_bc[(d, 0)] == PERIODIC]
        for d in range(self.dim):
            if (self.phys_bc[(d, 0)] == PERIODIC) != (self.phys_bc[(d, 1)] == PERIODIC):
                raise ValueError("periodic on one side of direction %d only" % d)
        self.cf_kind = cf_kind
        self.pshape = tuple(n + 2 * PAD for n in self.shape)
        self.inner = tuple(slice(PAD, PAD + n) for n in self.shape)
        self.mask = np.zeros(self.pshape, dtype=bool)
        for lo, hi in self.boxes:
            sl = tuple(slice(PAD + l, PAD + u + 1) for l, u in zip(lo, hi))
            if self.mask[sl].any():
                raise ValueError("boxes overlap")
            self.mask[sl] = True
        self.inside = np.zeros(self.pshape, dtype=bool)
        self.inside[self.inner] = True
        self.ncells = int(self.mask.sum())
        self._check_rows()
        self.labels, self.ncomp = ndimage.label(self.mask)  # face connectivity
        self.labels = self.labels - 1  # -1 outside the level, else 0..ncomp-1
        if self.periodic:
            self._join_periodic()
            for d in self.periodic:
                for s in (0, 1):
                    step = 1 if s else -1
                    pend = self.end_is_physical(d, s)
                    for k in (1, 2):
                        if np.any(pend & ~_wrap(self.mask, d, k * step)):
                            raise ValueError("a periodic ghost of direction %d is not a cell of the level" % d)

    def _join_periodic(self):
        """Merge the labels of cells that face each other across a periodic
        boundary (first and last cell of a row along that direction)."""
        par = list(range(self.ncomp))

        def find(x):
            while par[x] != x:
                x = par[x]
            return x

        for d in self.periodic:
            lo = [slice(None)] * self.dim
            hi = [slice(None)] * self.dim
            lo[d], hi[d] = PAD, PAD + self.shape[d] - 1
            a, b = self.labels[tuple(lo)], self.labels[tuple(hi)]
            both = (a >= 0) & (b >= 0)
            for x, y in zip(a[both], b[both]):
                rx, ry = find(int(x)), find(int(y))
                if rx != ry:
                    par[max(rx, ry)] = min(rx, ry)
        roots = sorted({find(c) for c in range(self.ncomp)})
        new = {r: i for i, r in enumerate(roots)}
        remap = np.array([new[find(c)] for c in range(self.ncomp)] + [-1])
        self.labels = remap[self.labels]  # -1 indexes the trailing -1
        self.ncomp = len(roots)

    # ------------------------------------------------------------------
    # bookkeeping
    def row_end(self, d, s):
        """Masked cells whose neighbour on side s along d is not masked."""
        step = 1 if s == 1 else -1
        return self.mask & ~_shift(self.mask, d, step)

    def end_is_physical(self, d, s):
        """Row ends whose outer neighbour lies outside the domain."""
        step = 1 if s == 1 else -1
        return self.row_end(d, s) & ~_shift(self.inside, d, step)

    def _check_rows(self):
        # The fills read the row-end cell and three cells behind it, so every
        # maximal row of masked cells must be at least 4 long.
        for d in range(self.dim):
            for s in (0, 1):
                step = 1 if s == 1 else -1
                end = self.row_end(d, s)
                for k in (1, 2, 3):
                    if np.any(end & ~_shift(self.mask, d, -k * step)):
                        raise ValueError("a row of cells is shorter than 4")

    def end_kind(self, d, s):
        """Array of fill kinds at row ends: 'D', 'N', 'P' or 'I' (None
        elsewhere)."""
        phys = self.end_is_physical(d, s)
        end = self.row_end(d, s)
        kinds = np.full(self.pshape, None, dtype=object)
        kinds[phys] = self.phys_bc[(d, s)]
        kinds[end & ~phys] = self.cf_kind
        return kinds

    def singular_components(self, op):
        """Components on which the operator has a constant null vector: the
        Poisson operator with no Dirichlet-type row end in the component
        (the pure-Neumann case of (TLS-1) and (TLS-3))."""
        if op != "poisson":
            return []
        has_dir = np.zeros(self.ncomp, dtype=bool)
        for d in range(self.dim):
            for s in (0, 1):
                kinds = self.end_kind(d, s)
                dirlike = (kinds == DIRICHLET) | (kinds == INTERP)
                has_dir[np.unique(self.labels[dirlike])] = True
        return [c for c in range(self.ncomp) if not has_dir[c]]

    def zeros(self):
        return np.zeros(self.pshape)

    def zero_face_data(self):
        return {(d, s): self.zeros() for d in range(self.dim) for s in (0, 1)}

    # ------------------------------------------------------------------
    # ghost fill (Section 3, eqs. velBCHomoDiri5th and Neumann5)
    def ghosts(self, u, fd=None, cfv=None, wrap=True):
        """Ghost arrays G[(d, s)] for the padded level array u.

        fd   : face data as described in the module docstring (None = zero,
               the homogeneous fill used for corrections)
        cfv  : padded array of coarse-fine interpolated ghost values for
               row ends of kind 'I' (None = zero)
        wrap : False leaves the ghosts of periodic row ends at zero
        """
        G = {}
        for d in range(self.dim):
            for s in (0, 1):
                step = 1 if s == 1 else -1
                end = self.row_end(d, s)
                kinds = self.end_kind(d, s)
                u0 = u
                u1 = _shift(u, d, -step)
                u2 = _shift(u, d, -2 * step)
                u3 = _shift(u, d, -3 * step)
                g = fd[(d, s)] if fd is not None else 0.0
                gd1, gd2 = fv.dirichlet_ghosts(u0, u1, u2, u3, g)
                gn1, gn2 = fv.neumann_ghosts(u0, u1, u2, u3, g, self.h)
                first = np.zeros(self.pshape)
                second = np.zeros(self.pshape)
                isd = end & (kinds == DIRICHLET)
                isn = end & (kinds == NEUMANN)
                first[isd], second[isd] = gd1[isd], gd2[isd]
                first[isn], second[isn] = gn1[isn], gn2[isn]
                isp = end & (kinds == PERIODIC)
                if wrap and isp.any():
                    first[isp] = _wrap(u, d, step)[isp]
                    second[isp] = _wrap(u, d, 2 * step)[isp]
                Gs = _shift(first, d, -step) + _shift(second, d, -2 * step)
                isi = end & (kinds == INTERP)
                if cfv is not None and isi.any():
                    # interpolated ghosts are properties of the ghost cell itself
                    at1 = _shift(isi, d, -step)
                    at2 = _shift(isi, d, -2 * step)
                    Gs[at1] = cfv[at1]
                    Gs[at2] = cfv[at2]
                G[(d, s)] = Gs
        return G

    def neighbour(self, u, G, d, k):
        """Value at i + k e_d as seen by the stencil at i: the level's own
        cell where masked, else the ghost of the matching side."""
        s = 1 if k > 0 else 0
        return np.where(_shift(self.mask, d, k), _shift(u, d, k), _shift(G[(d, s)], d, k))

    # ------------------------------------------------------------------
    # operators
    def laplacian(self, u, G, dirs=None):
        """Discrete Laplacian eq. (discreteOps c) on masked cells (0 elsewhere)."""
        out = self.zeros()
        for d in (range(self.dim) if dirs is None else dirs):
            out += fv.laplacian_1d(self.neighbour(u, G, d, -2), self.neighbour(u, G, d, -1), u,
                                   self.neighbour(u, G, d, 1), self.neighbour(u, G, d, 2), self.h)
        out[~self.mask] = 0.0
        return out

    def apply(self, u, op, c, fd=None, cfv=None):
        """A u: (I - c L) u for op 'helmholtz' (the (TLS-2) form, eq.
        GePUP-IMEX, c = gamma nu k) or L u for op 'poisson' (TLS-1/3), with
        the ghosts of u filled from fd / cfv first."""
        G = self.ghosts(u, fd, cfv)
        Lu = self.laplacian(u, G)
        if op == "helmholtz":
            out = u - c * Lu
        elif op == "poisson":
            out = Lu
        else:
            raise ValueError(op)
        out[~self.mask] = 0.0
        return out

    def apply_T(self, lam, op, c):
        """Transpose of the homogeneous operator: the A_T with
        <A_hom u, lam> = <u, A_T lam> for all u (the adjoint of the level
        system; not in the paper).

        The homogeneous A is "fill the ghosts from the level's own cells, then
        apply the stencil".  Its transpose applies the (symmetric) stencil to
        lam extended by zero, where the neighbour is a cell of the level
        (other boxes included: exchange ghosts are plain cells here), then
        sends every ghost's adjoint mu (the stencil weights the cells next to
        that ghost put on it) back to the cells the fill read, with the fill
        weights.  The fill weights are taken from the fill formulas
        themselves (applied to unit vectors), not retyped."""
        dim = self.dim
        zero = self.zeros()
        # stencil on lam extended by zero (G = 0 everywhere)
        Ltl = self.laplacian(lam, {(d, s): zero for d in range(dim) for s in (0, 1)})
        back = self.zeros()
        k12 = 12.0 * self.h * self.h
        unit = [[1.0 if m == j else 0.0 for m in range(4)] for j in range(4)]
        wd = [fv.dirichlet_ghosts(*unit[j], 0.0) for j in range(4)]
        wn = [fv.neumann_ghosts(*unit[j], 0.0, self.h) for j in range(4)]
        for d in range(dim):
            for s in (0, 1):
                step = 1 if s == 1 else -1
                end = self.row_end(d, s)
                kinds = self.end_kind(d, s)
                lam0 = np.where(self.mask, lam, 0.0)
                lam1 = _shift(lam0, d, -step)
                # stencil weights on the first ghost (from the end cell and the
                # next cell) and on the second ghost (from the end cell), at
                # the row end; a ghost position that is a cell of the level
                # is not a ghost (the neighbour() rule)
                g1_is_ghost = ~_shift(self.mask, d, step)
                g2_is_ghost = ~_shift(self.mask, d, 2 * step)
                mu1 = np.where(g1_is_ghost, (16.0 * lam0 - lam1) / k12, 0.0)
                mu2 = np.where(g2_is_ghost, -lam0 / k12, 0.0)
                for kind, w in ((DIRICHLET, wd), (NEUMANN, wn)):
                    sel = end & (kinds == kind)
                    if not sel.any():
                        continue
                    for j in range(4):
                        contrib = np.where(sel, w[j][0] * mu1 + w[j][1] * mu2, 0.0)
                        back += _shift(contrib, d, j * step)
                # a periodic ghost copies the cell one or two steps on,
                # modulo the grid: its adjoint goes back to that cell
                sel = end & (kinds == PERIODIC)
                if sel.any():
                    back += _wrap(np.where(sel, mu1, 0.0), d, -step)
                    back += _wrap(np.where(sel, mu2, 0.0), d, -2 * step)
        back[~self.mask] = 0.0
        if op == "helmholtz":
            out = lam - c * (Ltl + back)
        elif op == "poisson":
            out = Ltl + back
        else:
            raise ValueError(op)
        out[~self.mask] = 0.0
        return out

    def diagonal(self, op, c):
        """Coefficient of u_i in (A u)_i with the homogeneous ghost fill
        folded in.  Obtained by probing: along direction d the folded 1-D
        operator couples cells at most 3 apart, so unit vectors on every 7th
        cell of a row cannot disturb each other's diagonal entries.  A
        periodic ghost is a copy of another cell (rows have at least 4
        cells), so it carries no diagonal part and is left at zero."""
        idx = np.indices(self.pshape)
        Ldiag = self.zeros()
        for d in range(self.dim):
            for colour in range(7):
                probe = (self.mask & (idx[d] % 7 == colour)).astype(float)
                G = self.ghosts(probe, wrap=False)
                col = self.laplacian(probe, G, dirs=[d])
                sel = probe > 0
                Ldiag[sel] += col[sel]
        if op == "helmholtz":
            D = 1.0 - c * Ldiag
        else:
            D = Ldiag
        D[~self.mask] = 1.0
        return D

    # ------------------------------------------------------------------
    # multigrid coarsening
    def can_coarsen(self):
        """Halve while every box has even corners and even sides of at least 8,
        and while two boxes that face each other across a gap along an axis
        stay at least two cells apart after halving (a one-cell gap would let
        the radius-2 stencil of one box read the other box directly, coupling
        boxes that are not face-connected)."""
        if any(n % 2 for n in self.shape):
            return False
        for lo, hi in self.boxes:
            for l, u in zip(lo, hi):
                if l % 2 or (u + 1) % 2 or (u - l + 1) < 8:
                    return False
        for a, (alo, ahi) in enumerate(self.boxes):
            for blo, bhi in self.boxes[a + 1:]:
                for d in range(self.dim):
                    if any(max(alo[e], blo[e]) > min(ahi[e], bhi[e]) for e in range(self.dim) if e != d):
                        continue
                    gap = max(blo[d] - ahi[d] - 1, alo[d] - bhi[d] - 1)
                    if 0 < gap < 4:
                        return False
        return True

    def coarsen(self):
        boxes = [(tuple(l // 2 for l in lo), tuple((u + 1) // 2 - 1 for u in hi)) for lo, hi in self.boxes]
        return Level(tuple(n // 2 for n in self.shape), 2 * self.h, boxes, self.phys_bc, self.cf_kind)

    def largest_component(self):
        """Cells of the largest face-connected component."""
        return int(np.bincount(self.labels[self.mask]).max())

    def hierarchy(self, bottom_cells=0):
        """The multigrid depths: halve while can_coarsen() allows and, with
        bottom_cells > 0, while some component has more than bottom_cells
        cells (the depth that first has none is solved exactly)."""
        levels = [self]
        while levels[-1].can_coarsen() and not (bottom_cells and levels[-1].largest_component() <= bottom_cells):
            levels.append(levels[-1].coarsen())
        return levels

    # ------------------------------------------------------------------
    def colour(self):
        """Red (True) where the sum of the level's global indices is even."""
        idx = np.indices(self.pshape) - PAD
        return (idx.sum(axis=0) % 2) == 0

    def comp_mean(self, u, comps):
        """Subtract, on each listed component, the mean over its cells."""
        out = u.copy()
        for c in comps:
            sel = self.labels == c
            out[sel] -= u[sel].sum() / sel.sum()
        return out
