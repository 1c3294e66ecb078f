"""Test glue between the oracle's dense level arrays and the HIP library's
packed buffers (pure indexing; no solver arithmetic)."""
import numpy as np

from oracle.level import PAD, Level


def covers_domain(lev):
    return lev.ncells == int(np.prod(lev.shape))


def make_hier(lev, op, c, cf_mode=None, bottom_cells=0, bottom=None):
    """Hierarchy whose level `index` has the oracle level's boxes.  A level
    that does not cover its grid becomes level 1 of a two-level hierarchy
    (level 0 one box over the half-resolution grid).  bottom_cells: the
    exact-solve size of the multigrid hierarchy (0: the layout's own)."""
    import torch  # noqa: F401  (initialises the HIP runtime the library uses)
    from paper_2506_02663_amd import amg as A

    D = lev.dim
    if covers_domain(lev):
        H = A.Hierarchy(D, lev.shape, lev.h, 1)
        index = 0
    else:
        H = A.Hierarchy(D, tuple(n // 2 for n in lev.shape), 2 * lev.h, 2)
        H.set_level_boxes(0, [((0,) * D, tuple(n // 2 - 1 for n in lev.shape))])
        index = 1
        mode = {"D": A.CF_DIRICHLET, "N": A.CF_NEUMANN, "I": A.CF_INTERP}[cf_mode or lev.cf_kind]
        H.set_cf_mode(1, mode)
    H.set_level_boxes(index, lev.boxes)
    for (d, s), kind in lev.phys_bc.items():
        H.set_physical_bc(d, s, {"D": A.DIRICHLET, "N": A.NEUMANN, "P": A.PERIODIC}[kind])
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
    if bottom_cells:
        H.set_bottom_cells(bottom_cells)
    if bottom is not None:  # (kind, GMRES steps)
        H.set_bottom_solver(*bottom)
    H.finalize()
    return H, index


def _box_slices(b):
    return tuple(slice(PAD + l, PAD + h + 1) for l, h in zip(b["lo"], b["hi"]))


def to_dev(H, level, depth, dense, dtype=None):
    import torch
    dtype = dtype or torch.float64
    flat = H.pack(level, depth, lambda i, b: dense[_box_slices(b)])
    return torch.tensor(flat, dtype=dtype, device="cuda")


def from_dev(H, level, depth, t, lev):
    out = lev.zeros()
    arrs = H.unpack(level, depth, t.detach().cpu().double().numpy())
    for b, a in zip(H.boxes(level, depth), arrs):
        out[_box_slices(b)] = a
    return out


def faces_to_dev(H, level, lev, fd):
    import torch

    def get(i, b, d, s):
        sl = list(_box_slices(b))
        sl[d] = PAD + (b["hi"][d] if s else b["lo"][d])
        return fd[(d, s)][tuple(sl)]

    return torch.tensor(H.pack_faces(level, get), dtype=torch.float64, device="cuda")


def ghost_values(H, level, depth, t, lev, G):
    """(gpu, oracle) pairs of every stored face-strip ghost value."""
    gpu, want = [], []
    arrs = H.unpack(level, depth, t.detach().cpu().double().numpy(), ghosts=True)
    u_or = None
    for b, a in zip(H.boxes(level, depth), arrs):
        n = [h - l + 1 for l, h in zip(b["lo"], b["hi"])]
        for d in range(lev.dim):
            for s in (0, 1):
                for layer in (1, 2):
                    p = (b["hi"][d] + layer) if s else (b["lo"][d] - layer)
                    sl_g = [slice(2, 2 + m) for m in n]
                    sl_g[d] = 2 + (n[d] - 1 + layer if s else -layer)
                    sl_o = list(_box_slices(b))
                    sl_o[d] = PAD + p
                    sl_o = tuple(sl_o)
                    m = lev.mask[sl_o]
                    ov = np.where(m, 0.0, G[(d, s)][sl_o])
                    gpu.append((a[tuple(sl_g)], ov, m))
    return gpu


def random_field(lev, seed):
    rng = np.random.default_rng(seed)
    u = lev.zeros()
    u[lev.mask] = rng.normal(size=lev.ncells)
    return u


def random_faces(lev, seed):
    rng = np.random.default_rng(seed)
    fd = lev.zero_face_data()
    for k in fd:
        e = lev.row_end(*k)
        fd[k][e] = rng.normal(size=int(e.sum()))
    return fd


def relerr(a, b, mask):
    scale = max(np.abs(b[mask]).max(), 1e-300)
    return float(np.abs(a[mask] - b[mask]).max() / scale)


# ---- layouts shared by the GPU tests ---------------------------------------
def unit_level(n, D, bc):
    bcs = bc if isinstance(bc, dict) else {(d, s): bc for d in range(D) for s in (0, 1)}
    return Level((n,) * D, 1.0 / n, [((0,) * D, (n - 1,) * D)], bcs)


MIXED_BC = {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D"}
PERIODIC_X_BC = {(0, 0): "P", (0, 1): "P", (1, 0): "D", (1, 1): "N"}


def tiled_level(n=32, D=2, bc="D"):
    """Level 0 split into four boxes (box-to-box exchange everywhere)."""
    h = n // 2
    if D == 2:
        boxes = [((0, 0), (h - 1, h - 1)), ((h, 0), (n - 1, h - 1)), ((0, h), (h - 1, n - 1)), ((h, h), (n - 1, n - 1))]
    else:
        boxes = [((0, 0, 0), (h - 1, n - 1, n - 1)), ((h, 0, 0), (n - 1, h - 1, n - 1)),
                 ((h, h, 0), (n - 1, n - 1, h - 1)), ((h, h, h), (n - 1, n - 1, n - 1))]
    return Level((n,) * D, 1.0 / n, boxes, {(d, s): bc for d in range(D) for s in (0, 1)})


def cf_level(cf="D", phys="N"):
    """A level of three boxes inside a 32^2 grid: an L-shape and a separate
    box (two components; physical, coarse-fine and box-to-box row ends)."""
    boxes = [((0, 4), (15, 11)), ((16, 4), (23, 19)), ((4, 20), (11, 27))]
    return Level((32, 32), 1.0 / 32, boxes, {(d, s): phys for d in range(2) for s in (0, 1)}, cf)


def gap_level(cf="D"):
    """Boxes four cells apart along x (two cells one depth down: both ghost
    layers of each box lie in the gap) and a third box eight cells away."""
    boxes = [((0, 0), (15, 15)), ((20, 0), (35, 15)), ((0, 24), (15, 39))]
    return Level((48, 48), 1.0 / 48, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)}, cf)
