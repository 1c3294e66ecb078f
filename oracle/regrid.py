"""Oracle: regridding and data migration of an AMR hierarchy (Section 5.4,
RDM-1..4).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* RDM-1: cells of level l are tagged where the magnitude of the discrete
  vorticity reaches a threshold; the vorticity is taken from the composite
  gradient of the velocity components (eq. discreteOps a with the
  hierarchy's fills), 2D: G_x u_1 - G_y u_0, 3D: the norm of the curl.
* RDM-2: tagged cells are grouped into disjoint boxes by the clustering of
  Berger and Rigoutsos (1991), then refined by the ratio.
* RDM-3: for l = lmax-2 .. 0 the boxes of the new level l+2 are coarsened
  twice, grown by `grow` cells in every direction (clipped to the domain),
  and their cells joined to the tags of level l; clustering that set and
  refining gives the new level l+1.  The paper grows by one cell, which
  gives its nesting (one cell of level l+1 between levels l+2 and l).  The
  five-cell AMRCFI window (oracle/amr.py, never shifted off the coarser
  level) reaches three cells of level l+1 beyond the footprint of level
  l+2, so the default growth is the least g with g * ratio >= 3: one cell
  at ratio 4 (the paper's), two at ratio 2.
* Blocking (not in the paper): the fills need rows of at least four cells
  on every level, which a box around one tagged cell would break; so the
  tags of level l are clustered on the grid coarsened by a blocking factor
  b (a block is tagged when any of its cells is), and the boxes refined by
  b (clipped to the grid) and then by the ratio.  The default is the least
  b with b * ratio >= 4: two at ratio 2, one at ratio 4.
* Data migration: cells of the new hierarchy that the old one has on the
  same level take the old values; the others take AMRCFI (the conservative
  tensor quartic of oracle/amr.py) from the new coarser level, which holds
  the old data where the grids are common, levels in increasing order.

The clustering (the paper cites it without details; readings):

* a box is first shrunk to the bounding box of its tags and accepted when
  its efficiency (tags / cells) reaches ``efficiency``;
* otherwise it is cut into two along one direction at an index c (parts
  [lo, c-1] and [c, hi]), each part at least ``min_side`` long along the
  cut direction: at a hole of the tag signature (a slice without tags)
  closest to the box's centre; else at the strongest inflection of the
  signature (the largest jump of its second difference between two
  neighbouring slices, where the second difference changes sign); else at
  the middle of the longest side; ties go to the position closer to the
  centre, then to the lower direction, then to the lower index;
* a box that admits no cut is accepted as it is; parts are clustered
  recursively, the low part first.
"""
import numpy as np

from . import proj
from .amr import weights, window_shift
from .level import PAD


# ---------------------------------------------------------------------------
# RDM-1
def vorticity(H, U):
    """Per level, the vorticity of the velocity U[d][l] on the level's cells
    (2D: G_x u_1 - G_y u_0; 3D: the Euclidean norm of the curl)."""
    D = H.dim
    G = [proj.composite_gradient(H, U[d]) for d in range(D)]  # G[d][e][l] = G_e u_d
    out = []
    for l, lev in enumerate(H.levels):
        if D == 2:
            w = G[1][0][l] - G[0][1][l]
        else:
            cx = G[2][1][l] - G[1][2][l]
            cy = G[0][2][l] - G[2][0][l]
            cz = G[1][0][l] - G[0][1][l]
            w = np.sqrt(cx * cx + cy * cy + cz * cz)
        out.append(np.where(lev.mask, w, 0.0))
    return out


def tag_vorticity(H, U, eps):
    """Dense boolean arrays over each level's grid (unpadded): |omega| >= eps
    on the level's cells."""
    W = vorticity(H, U)
    return [(np.abs(W[l]) >= eps)[lev.inner] & lev.mask[lev.inner] for l, lev in enumerate(H.levels)]


# ---------------------------------------------------------------------------
# RDM-2: clustering
def _signature(tags, lo, hi, d):
    sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
    sub = tags[sl]
    axes = tuple(e for e in range(tags.ndim) if e != d)
    return sub.sum(axis=axes)


def _cut(tags, lo, hi, min_side):
    """(d, c) of the cut of box [lo, hi] (already the bounding box of its
    tags), or None."""
    D = tags.ndim
    centre = [(lo[d] + hi[d] + 1) / 2.0 for d in range(D)]

    def ok(d, c):
        return c - lo[d] >= min_side and hi[d] + 1 - c >= min_side

    # holes: slice index i without tags; cut at c = i
    best = None
    for d in range(D):
        sig = _signature(tags, lo, hi, d)
        for i, v in enumerate(sig):
            c = lo[d] + i
            if v == 0 and ok(d, c):
                key = (abs(c - centre[d]), d, c)
                if best is None or key < best:
                    best = key
    if best is not None:
        return best[1], best[2]
    # inflections: second difference lap[i] at slice i (interior slices);
    # a sign change between slices c-1 and c gives a cut at c
    best = None
    for d in range(D):
        sig = _signature(tags, lo, hi, d).astype(np.int64)
        n = len(sig)
        lap = {i: int(sig[i - 1] - 2 * sig[i] + sig[i + 1]) for i in range(1, n - 1)}
        for i in range(2, n - 1):
            a, b = lap[i - 1], lap[i]
            if a * b < 0:
                c = lo[d] + i
                if ok(d, c):
                    key = (-abs(b - a), abs(c - centre[d]), d, c)
                    if best is None or key < best:
                        best = key
    if best is not None:
        return best[2], best[3]
    # bisection of the longest side (lowest direction among equals)
    sides = [hi[d] - lo[d] + 1 for d in range(D)]
    d = int(np.argmax(sides))
    c = lo[d] + sides[d] // 2
    if ok(d, c):
        return d, c
    return None


def cluster(tags, efficiency=0.75, min_side=2):
    """Boxes (lo, hi) covering the tagged cells of the dense boolean array
    `tags` (Berger-Rigoutsos as read in the module docstring)."""
    out = []

    def rec(lo, hi):
        sl = tuple(slice(a, b + 1) for a, b in zip(lo, hi))
        idx = np.argwhere(tags[sl])
        if len(idx) == 0:
            return
        lo = tuple(int(a + v) for a, v in zip(lo, idx.min(axis=0)))
        hi = tuple(int(a + v) for a, v in zip(lo, idx.max(axis=0) - idx.min(axis=0)))
        vol = int(np.prod([b - a + 1 for a, b in zip(lo, hi)]))
        if len(idx) >= efficiency * vol:
            out.append((lo, hi))
            return
        cut = _cut(tags, lo, hi, min_side)
        if cut is None:
            out.append((lo, hi))
            return
        d, c = cut
        hi1 = list(hi)
        hi1[d] = c - 1
        lo2 = list(lo)
        lo2[d] = c
        rec(lo, tuple(hi1))
        rec(tuple(lo2), hi)

    rec(tuple(0 for _ in tags.shape), tuple(n - 1 for n in tags.shape))
    return out


# ---------------------------------------------------------------------------
# RDM-2..4
def _refine(boxes, r):
    return [(tuple(a * r for a in lo), tuple((b + 1) * r - 1 for b in hi)) for lo, hi in boxes]


def default_growth(ratio):
    """Cells of level l added around the coarsened boxes in RDM-3: the
    least g with g * ratio >= 3 (see the module docstring)."""
    return -(-3 // ratio)


def default_blocking(ratio):
    """Blocking factor of the clustering: the least b with b * ratio >= 4."""
    return -(-4 // ratio)


def blocked_cluster(tags, b, efficiency, min_side):
    """Boxes over the grid of `tags` from the clustering of its tags
    coarsened by b (a block tagged when any of its cells is), refined by b
    and clipped to the grid."""
    shape = tags.shape
    nb = [-(-n // b) for n in shape]
    tb = np.zeros(nb, bool)
    for pos in np.argwhere(tags):
        tb[tuple(int(p) // b for p in pos)] = True
    out = []
    for lo, hi in cluster(tb, efficiency, min_side):
        out.append((tuple(a * b for a in lo), tuple(min((c + 1) * b, n) - 1 for c, n in zip(hi, shape))))
    return out


def new_boxes(shapes, tags, ratio, efficiency=0.75, min_side=2, grow=None, block=None):
    """New boxes of levels 1..lmax from the tags of levels 0..lmax-1.
    shapes[l]: grid of level l; tags[l]: dense booleans over it; grow: cells
    of RDM-3's expansion (None: default_growth(ratio)); block: blocking
    factor (None: default_blocking(ratio)).  Returns a list per new level
    l = 1..lmax (an empty list: no boxes)."""
    g = default_growth(ratio) if grow is None else grow
    b = default_blocking(ratio) if block is None else block
    lmax = len(tags)
    new = [None] * (lmax + 1)
    new[lmax] = _refine(blocked_cluster(tags[lmax - 1], b, efficiency, min_side), ratio)
    for l in range(lmax - 2, -1, -1):
        t = tags[l].copy()
        for lo, hi in new[l + 2]:
            clo = [a // ratio // ratio - g for a in lo]
            chi = [b // ratio // ratio + g for b in hi]
            sl = tuple(slice(max(a, 0), min(b, n - 1) + 1) for a, b, n in zip(clo, chi, shapes[l]))
            t[sl] = True
        new[l + 1] = _refine(blocked_cluster(t, b, efficiency, min_side), ratio)
    return new[1:]


def migrate(H_old, H_new, U_old):
    """Data of the new hierarchy (padded arrays per level) from U_old (old
    levels, covered cells as stored): level 0 is copied; on every finer new
    level, AMRCFI from the new level below, then the cells the old level had
    copied over."""
    U = [H_new.levels[0].zeros()]
    U[0][H_new.levels[0].mask] = U_old[0][H_new.levels[0].mask]
    r = H_new.ratio
    for l in range(1, H_new.nlev):
        fine, coarse = H_new.levels[l], H_new.levels[l - 1]
        D = fine.dim
        out = fine.zeros()
        for pos in np.argwhere(fine.mask):
            g = pos - PAD
            P = g // r
            a = g % r
            shifts = [window_shift(int(P[d]), coarse.shape[d]) for d in range(D)]
            lo = [int(P[d]) + shifts[d] - 2 for d in range(D)]
            sl = tuple(slice(PAD + lo[d], PAD + lo[d] + 5) for d in range(D))
            if not coarse.mask[sl].all():
                raise ValueError("interpolation window leaves the new level %d" % (l - 1))
            val = U[l - 1][sl]
            for d in range(D):
                val = np.tensordot(weights(r)[(shifts[d], int(a[d]))], val, axes=([0], [0]))
            out[tuple(pos)] = float(val)
        if l < H_old.nlev:
            common = fine.mask & H_old.levels[l].mask
            out[common] = U_old[l][common]
        U.append(out)
    return U
