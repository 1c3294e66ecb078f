"""Python binding of the C ABI in include/amg.h (argument marshalling only).

Every numerical step runs in the HIP library ``libamg.so``; this module
passes device pointers of torch tensors and host arrays of box corners, and
converts between dense per-box arrays and the packed level layout (pure
indexing).  Importing it on a machine without the built library raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libamg.so")

OK, EINVAL, ELAYOUT, EUNSUPPORTED, ENOTCONVERGED, ENONFINITE, ESOLVABILITY, EDEVICE = range(8)
HELMHOLTZ, POISSON = 0, 1
DIRICHLET, NEUMANN, PERIODIC = 0, 1, 2
CF_DIRICHLET, CF_NEUMANN, CF_INTERP = 0, 1, 2
SMOOTH_JACOBI, SMOOTH_RB = 0, 1
FP64, MIXED = 0, 1
F64, F32 = 0, 1
SOLV_RHS_SHIFT, SOLV_OFF, SOLV_CF_DELTA = 0, 1, 2
BOTTOM_EXACT, BOTTOM_ILU_GMRES = 0, 1
CIC_VALUE, CIC_NORMAL_DERIVATIVE = 0, 1
T_SWEEP, T_FILL, T_RESTRICT, T_PROLONG, T_RESIDUAL, T_SWEEP_SPLIT, T_KINDS = range(7)
TUNE_MARCH2, TUNE_MARCH3, TUNE_ROW_ALIGN, TUNE_SPLIT_RB, TUNE_TAIL = range(5)
MAX_HISTORY, MAX_COMP = 128, 64


class LevelDesc(C.Structure):
    _fields_ = [("nboxes", C.c_int32), ("depths", C.c_int32), ("ncomp", C.c_int32), ("nsingular", C.c_int32),
                ("ncells", C.c_int64), ("nstored", C.c_int64), ("nface", C.c_int64), ("split_rb", C.c_int32),
                ("tail_depth", C.c_int32)]


class BoxDesc(C.Structure):
    _fields_ = [("lo", C.c_int32 * 3), ("hi", C.c_int32 * 3), ("offset", C.c_int64), ("stride", C.c_int64 * 3),
                ("face_offset", (C.c_int64 * 2) * 3), ("comp", C.c_int32), ("singular", C.c_int32)]


class SolveOpts(C.Structure):
    _fields_ = [("nu1", C.c_int32), ("nu2", C.c_int32), ("smoother", C.c_int32), ("precision", C.c_int32),
                ("solvability", C.c_int32), ("max_cycles", C.c_int32), ("omega", C.c_double),
                ("tol_rel", C.c_double), ("tol_abs", C.c_double), ("use_graph", C.c_int32), ("pad_", C.c_int32),
                ("omega_rb", C.c_double)]


class SolveStats(C.Structure):
    _fields_ = [("cycles", C.c_int32), ("converged", C.c_int32), ("r0", C.c_double), ("rfinal", C.c_double),
                ("history", C.c_double * MAX_HISTORY), ("ncomp", C.c_int32), ("used_graph", C.c_int32),
                ("pad_", C.c_int32), ("defect", C.c_double * MAX_COMP)]

    def as_dict(self):
        n = min(self.cycles + 1, MAX_HISTORY)
        return {"cycles": self.cycles, "converged": bool(self.converged), "r0": self.r0, "rfinal": self.rfinal,
                "history": list(self.history[:n]), "defects": list(self.defect[: self.ncomp]),
                "graph": bool(self.used_graph)}


class ImexStats(C.Structure):
    _fields_ = [("solves", C.c_int32), ("cycles", C.c_int32), ("max_cycles", C.c_int32), ("converged", C.c_int32),
                ("max_rel_residual", C.c_double)]

    def as_dict(self):
        return {"solves": self.solves, "cycles": self.cycles, "max_cycles": self.max_cycles,
                "converged": bool(self.converged), "max_rel_residual": self.max_rel_residual}


IMEX_C = (0.0, 1 / 2, 83 / 250, 31 / 50, 17 / 20, 1.0)  # stage nodes of ARK4(3)6L[2]SA

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libamg.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
        # torch first: its HIP runtime (same soname) then serves the library
        # too, so the process holds one runtime whichever module loads first
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int, C.c_double
        L.amg_create.argtypes = [i32, C.POINTER(C.c_double), C.POINTER(C.c_double), C.POINTER(C.c_int32), i32, i32,
                                 C.POINTER(vp)]
        L.amg_destroy.argtypes = [vp]
        L.amg_last_error.argtypes = [vp]
        L.amg_last_error.restype = C.c_char_p
        L.amg_set_level_boxes.argtypes = [vp, i32, i32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.amg_set_isolated_boxes.argtypes = [vp, i32, i32]
        L.amg_set_physical_bc.argtypes = [vp, i32, i32, i32]
        L.amg_set_cf_mode.argtypes = [vp, i32, i32]
        L.amg_set_bottom_cells.argtypes = [vp, i32]
        L.amg_set_bottom_solver.argtypes = [vp, i32, i32]
        L.amg_set_operator.argtypes = [vp, i32, dbl]
        L.amg_finalize.argtypes = [vp]
        L.amg_level_info.argtypes = [vp, i32, C.POINTER(LevelDesc)]
        L.amg_box_info.argtypes = [vp, i32, i32, i32, C.POINTER(BoxDesc)]
        L.amg_depth_size.argtypes = [vp, i32, i32, C.POINTER(C.c_int64), C.POINTER(C.c_int32)]
        L.amg_default_opts.argtypes = [C.POINTER(SolveOpts)]
        L.amg_default_opts.restype = None
        L.amg_solve.argtypes = [vp, i32, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(SolveOpts),
                                C.POINTER(SolveStats), vp]
        L.amg_apply_operator.argtypes = [vp, i32, vp, vp, vp, i32, vp]
        L.amg_fill_ghosts.argtypes = [vp, i32, i32, i32, vp, vp, vp]
        L.amg_residual.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.amg_smooth.argtypes = [vp, i32, i32, i32, i32, i32, dbl, vp, vp, vp, vp]
        L.amg_restrict.argtypes = [vp, i32, i32, i32, vp, vp, vp]
        L.amg_prolong.argtypes = [vp, i32, i32, i32, vp, vp, vp]
        L.amg_bottom.argtypes = [vp, i32, i32, vp, vp, vp]
        L.amg_vcycle.argtypes = [vp, i32, i32, C.POINTER(SolveOpts), vp, vp, vp]
        L.amg_timing_enable.argtypes = [vp, i32]
        L.amg_composite_residual.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp]
        L.amg_set_tuning.argtypes = [vp, i32, i32]
        L.amg_timing_read.argtypes = [vp, i32, C.POINTER(C.c_int64), C.POINTER(C.c_double), i32]
        L.amg_solve_adjoint.argtypes = [vp, i32, vp, vp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
        L.amg_vcycle_adjoint.argtypes = [vp, i32, i32, C.POINTER(SolveOpts), vp, vp, vp]
        L.amg_apply_transpose.argtypes = [vp, i32, vp, vp, vp]
        L.amg_apply_laplacian.argtypes = [vp, i32, vp, vp, vp, vp]
        L.amg_dot.argtypes = [vp, i32, vp, vp, C.POINTER(C.c_double), vp]
        L.amg_set_coefficient.argtypes = [vp, dbl]
        pp = C.POINTER(vp)
        L.amg_gradient.argtypes = [vp, i32, i32, pp, pp, pp, vp]
        L.amg_divergence.argtypes = [vp, i32, i32, pp, pp, pp, vp]
        L.amg_project.argtypes = [vp, vp, i32, i32, pp, pp, pp, pp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
        L.amg_solve_adjoint_composite.argtypes = [vp, i32, pp, pp, C.POINTER(SolveOpts), C.POINTER(SolveStats), vp]
        L.amg_composite_residual_adjoint.argtypes = [vp, i32, pp, pp, pp, vp]
        L.amg_composite_laplacian.argtypes = [vp, i32, pp, pp, pp, vp]
        L.amg_time_sweep.argtypes = [vp, i32, i32, i32, i32, vp, vp, vp, C.POINTER(C.c_double), vp]
        L.amg_autotune.argtypes = [vp, i32, i32, i32, i32, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.amg_dot_noalloc.argtypes = [vp, i32, vp, vp, vp, vp]
        L.amg_cic_face_data.argtypes = [vp, i32, C.POINTER(vp), dbl, dbl, i32, vp, vp, vp]
        L.amg_cic_correct.argtypes = [vp, i32, C.POINTER(vp), C.POINTER(C.c_double), vp]
        L.amg_gradient_transpose.argtypes = [vp, i32, i32, pp, pp, vp]
        L.amg_divergence_transpose.argtypes = [vp, i32, i32, pp, pp, vp]
        L.amg_project_adjoint.argtypes = [vp, vp, i32, i32, pp, pp, pp, C.POINTER(SolveOpts), C.POINTER(SolveStats),
                                          vp]
        L.amg_imex_step.argtypes = [vp, vp, dbl, dbl, pp, pp, C.POINTER(SolveOpts), C.POINTER(SolveOpts),
                                    C.POINTER(ImexStats), vp]
        L.amg_convection.argtypes = [vp, pp, pp, vp]
        i32p = C.POINTER(C.c_int32)
        L.amg_cluster.argtypes = [i32, i32p, C.POINTER(C.c_uint8), dbl, i32, i32, i32p, i32p, i32p]
        L.amg_dense_inverse.argtypes = [i32, C.POINTER(C.c_double), i32]
        L.amg_subcycle_schedule.argtypes = [i32, i32, dbl, dbl, i32, i32, i32, i32p, C.POINTER(ScEvent)]
        L.amg_regrid_boxes.argtypes = [i32, i32p, i32, i32, C.POINTER(C.c_void_p), dbl, i32, i32, i32, i32, i32p, i32p,
                                       i32p]
        L.amg_tag_vorticity.argtypes = [vp, i32, pp, dbl, C.POINTER(C.c_void_p), vp]
        L.amg_migrate.argtypes = [vp, vp, pp, pp, vp]
        _lib = L
    return _lib


class AmgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"amg error {code}: {msg}")
        self.code = code


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_opts(**kw):
    o = SolveOpts()
    lib().amg_default_opts(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Hierarchy:
    """A box layout and operator; owns the library handle."""

    def __init__(self, dim, base_cells, h0, nlevels=1, ratio=2, x_lo=None):
        """Level 0 has base_cells[d] cells of size h0 from x_lo (default 0)."""
        self.dim = dim
        h = C.c_void_p()
        base = (C.c_int32 * dim)(*base_cells)
        lo = [0.0] * dim if x_lo is None else [float(v) for v in x_lo]
        xlo = (C.c_double * dim)(*lo)
        xhi = (C.c_double * dim)(*[lo[d] + base_cells[d] * float(h0) for d in range(dim)])
        rc = lib().amg_create(dim, xlo, xhi, base, ratio, nlevels, C.byref(h))
        if rc:
            raise AmgError(rc, "amg_create")
        self.h = h
        self._layout = {}

    def close(self):
        if self.h:
            lib().amg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc:
            raise AmgError(rc, lib().amg_last_error(self.h).decode())
        return rc

    # ---- layout ----
    def set_level_boxes(self, level, boxes):
        n = len(boxes)
        lo = (C.c_int32 * (n * self.dim))(*[int(v) for b in boxes for v in b[0]])
        hi = (C.c_int32 * (n * self.dim))(*[int(v) for b in boxes for v in b[1]])
        self._check(lib().amg_set_level_boxes(self.h, level, n, lo, hi))

    def set_isolated(self, level, flag=True):
        self._check(lib().amg_set_isolated_boxes(self.h, level, int(flag)))

    def set_physical_bc(self, d, side, kind):
        self._check(lib().amg_set_physical_bc(self.h, d, side, kind))

    def set_cf_mode(self, level, mode):
        self._check(lib().amg_set_cf_mode(self.h, level, mode))

    def set_bottom_cells(self, cells):
        self._check(lib().amg_set_bottom_cells(self.h, int(cells)))

    def set_bottom_solver(self, kind, iters=5):
        """BOTTOM_EXACT or BOTTOM_ILU_GMRES with iters GMRES steps."""
        self._check(lib().amg_set_bottom_solver(self.h, int(kind), int(iters)))

    def set_operator(self, kind, c=0.0):
        self._check(lib().amg_set_operator(self.h, kind, float(c)))
        self.op_kind, self.c = kind, float(c)

    def set_tuning(self, key, value):
        self._check(lib().amg_set_tuning(self.h, key, int(value)))

    def autotune(self, level=0, dtype=F32, smoother=SMOOTH_RB, nreps=20):
        """Pick the tile march length by timing the finest sweep (before finalize)."""
        best = C.c_int()
        ms = C.c_double()
        self._check(lib().amg_autotune(self.h, level, dtype, smoother, nreps, C.byref(best), C.byref(ms)))
        return best.value, ms.value

    def finalize(self):
        self._check(lib().amg_finalize(self.h))

    def level_info(self, level=0):
        d = LevelDesc()
        self._check(lib().amg_level_info(self.h, level, C.byref(d)))
        return d

    def depth_size(self, level, depth):
        n = C.c_int64()
        nb = C.c_int32()
        self._check(lib().amg_depth_size(self.h, level, depth, C.byref(n), C.byref(nb)))
        return n.value, nb.value

    def boxes(self, level=0, depth=0):
        key = (level, depth)
        if key not in self._layout:
            _, nb = self.depth_size(level, depth)
            out = []
            for b in range(nb):
                d = BoxDesc()
                self._check(lib().amg_box_info(self.h, level, depth, b, C.byref(d)))
                out.append({"lo": tuple(d.lo[: self.dim]), "hi": tuple(d.hi[: self.dim]), "offset": d.offset,
                            "stride": tuple(d.stride[: self.dim]),
                            "face_offset": [[d.face_offset[k][s] for s in (0, 1)] for k in range(self.dim)],
                            "comp": d.comp, "singular": d.singular})
            self._layout[key] = out
        return self._layout[key]

    # ---- dense <-> packed (pure indexing) ----
    def _box_view(self, flat, b, ghosts=False):
        n = [hi - lo + 1 for lo, hi in zip(b["lo"], b["hi"])]
        st = b["stride"]
        rows = int(np.prod([m + 4 for m in n[1:]]))  # stored rows of the box
        blk = flat[b["offset"]: b["offset"] + rows * st[1]]
        shape = [m + 4 for m in n[1:]][::-1] + [st[1]]  # (z, y, padded x) in memory order
        blk = blk.reshape(shape)[..., : n[0] + 4]
        if ghosts:
            return blk
        return blk[tuple(slice(2, 2 + m) for m in n[::-1])]

    def pack(self, level, depth, get, dtype=np.float64):
        """Packed host array; get(b, box) returns the box's interior as an
        array indexed [x, y(, z)]."""
        n, _ = self.depth_size(level, depth)
        flat = np.zeros(n, dtype=dtype)
        for i, b in enumerate(self.boxes(level, depth)):
            self._box_view(flat, b)[...] = np.asarray(get(i, b)).T
        return flat

    def unpack(self, level, depth, flat, ghosts=False):
        """List of per-box arrays indexed [x, y(, z)] (with the two ghost
        layers if ghosts=True)."""
        flat = np.asarray(flat)
        return [self._box_view(flat, b, ghosts).T.copy() for b in self.boxes(level, depth)]

    def pack_faces(self, level, get):
        """Face-data host array; get(b, box, d, s) returns the face's values
        indexed by the transverse directions in increasing order."""
        info = self.level_info(level)
        flat = np.zeros(max(info.nface, 1))
        for i, b in enumerate(self.boxes(level, 0)):
            for d in range(self.dim):
                for s in (0, 1):
                    v = np.asarray(get(i, b, d, s), dtype=np.float64)
                    off = b["face_offset"][d][s]
                    # transverse directions in increasing order, the first fastest
                    flat[off: off + v.size] = v.T.reshape(-1)
        return flat

    # ---- solve and steps (torch device tensors) ----
    def _need(self, t, level, depth, name, dtypes=None):
        """Host-side check that a tensor matches the packed layout the kernels
        index (so no kernel is launched on a short or misplaced buffer)."""
        import torch
        if t is None:
            raise ValueError(f"{name} is required")
        if not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous device tensor")
        if dtypes is not None and t.dtype not in dtypes:
            raise ValueError(f"{name} has dtype {t.dtype}")
        n = self.depth_size(level, depth)[0]
        if t.numel() < n:
            raise ValueError(f"{name} has {t.numel()} elements, the layout needs {n}")

    def _need_faces(self, fd, level):
        import torch
        if fd is None:
            return
        if not fd.is_cuda or not fd.is_contiguous() or fd.dtype != torch.float64:
            raise ValueError("face data must be a contiguous float64 device tensor")
        if fd.numel() < self.level_info(level).nface:
            raise ValueError("face data too short")

    def solve(self, level, x, f, face_data=None, opts=None, stream=None):
        import torch
        self._need(x, level, 0, "x", (torch.float64,))
        self._need(f, level, 0, "f", (torch.float64,))
        self._need_faces(face_data, level)
        o = opts or default_opts()
        st = SolveStats()
        xs = (C.c_void_p * (level + 1))()
        fs = (C.c_void_p * (level + 1))()
        ds = (C.c_void_p * (level + 1))()
        xs[level] = x.data_ptr()
        fs[level] = f.data_ptr()
        ds[level] = face_data.data_ptr() if face_data is not None else None
        rc = lib().amg_solve(self.h, level, level, xs, fs, ds, C.byref(o), C.byref(st), stream or _stream())
        if rc and rc != ENOTCONVERGED:
            self._check(rc)
        out = st.as_dict()
        out["status"] = rc
        return out

    def _level_ptrs(self, ts, n):
        arr = (C.c_void_p * n)()
        for i, t in enumerate(ts):
            arr[i] = None if t is None else t.data_ptr()
        return arr

    def solve_composite(self, xs, fs, fds=None, opts=None):
        """Composite solve over levels 0..len(xs)-1 (one tensor per level)."""
        import torch
        n = len(xs)
        fds = fds or [None] * n
        for l in range(n):
            self._need(xs[l], l, 0, "x", (torch.float64,))
            self._need(fs[l], l, 0, "f", (torch.float64,))
            self._need_faces(fds[l], l)
        o = opts or default_opts()
        st = SolveStats()
        rc = lib().amg_solve(self.h, 0, n - 1, self._level_ptrs(xs, n), self._level_ptrs(fs, n),
                             self._level_ptrs(fds, n), C.byref(o), C.byref(st), _stream())
        if rc and rc != ENOTCONVERGED:
            self._check(rc)
        out = st.as_dict()
        out["status"] = rc
        return out

    def composite_residual(self, xs, fs, rs, fds=None):
        import torch
        n = len(xs)
        fds = fds or [None] * n
        for l in range(n):
            for t, nm in ((xs[l], "x"), (fs[l], "f"), (rs[l], "r")):
                self._need(t, l, 0, nm, (torch.float64,))
            self._need_faces(fds[l], l)
        self._check(lib().amg_composite_residual(self.h, n - 1, self._level_ptrs(xs, n), self._level_ptrs(fs, n),
                                                 self._level_ptrs(fds, n), self._level_ptrs(rs, n), _stream()))

    def apply_operator(self, level, x, y, face_data=None, homogeneous=False):
        import torch
        self._need(x, level, 0, "x", (torch.float64,))
        self._need(y, level, 0, "y", (torch.float64,))
        self._need_faces(face_data, level)
        self._check(lib().amg_apply_operator(self.h, level, _ptr(x), _ptr(face_data), _ptr(y), int(homogeneous),
                                             _stream()))

    @staticmethod
    def _dt(t):
        import torch
        return F64 if t.dtype == torch.float64 else F32

    def fill_ghosts(self, level, depth, u, face_data=None):
        self._need(u, level, depth, "u")
        self._need_faces(face_data, level)
        self._check(lib().amg_fill_ghosts(self.h, level, depth, self._dt(u), _ptr(u), _ptr(face_data), _stream()))

    def residual(self, level, depth, u, f, r):
        for t, nm in ((u, "u"), (f, "f"), (r, "r")):
            self._need(t, level, depth, nm, (u.dtype,))
        self._check(lib().amg_residual(self.h, level, depth, self._dt(u), _ptr(u), _ptr(f), _ptr(r), _stream()))

    def smooth(self, level, depth, u, f, tmp, smoother=SMOOTH_JACOBI, nsweeps=1, omega=None):
        """omega: the Jacobi weight (default 2/3) or the red-black relaxation
        factor (default 1)."""
        if omega is None:
            omega = 2.0 / 3.0 if smoother == SMOOTH_JACOBI else 1.0
        for t, nm in ((u, "u"), (f, "f"), (tmp, "tmp")):
            self._need(t, level, depth, nm, (u.dtype,))
        self._check(lib().amg_smooth(self.h, level, depth, self._dt(u), smoother, nsweeps, float(omega), _ptr(u),
                                     _ptr(f), _ptr(tmp), _stream()))

    def restrict(self, level, depth, r, fc):
        self._need(r, level, depth, "r")
        self._need(fc, level, depth + 1, "fc", (r.dtype,))
        self._check(lib().amg_restrict(self.h, level, depth, self._dt(r), _ptr(r), _ptr(fc), _stream()))

    def prolong(self, level, depth, ec, u):
        self._need(u, level, depth, "u")
        self._need(ec, level, depth + 1, "ec", (u.dtype,))
        self._check(lib().amg_prolong(self.h, level, depth, self._dt(u), _ptr(ec), _ptr(u), _stream()))

    def bottom(self, level, f, e):
        last = self.level_info(level).depths - 1
        self._need(f, level, last, "f")
        self._need(e, level, last, "e", (f.dtype,))
        self._check(lib().amg_bottom(self.h, level, self._dt(f), _ptr(f), _ptr(e), _stream()))

    def time_sweep(self, level, u, f, tmp, smoother=SMOOTH_JACOBI, n=50):
        """Average duration (ms) of the finest-depth smoothing kernel launched
        n times back to back (values meaningless: timing only)."""
        for t, nm in ((u, "u"), (f, "f"), (tmp, "tmp")):
            self._need(t, level, 0, nm, (u.dtype,))
        ms = C.c_double()
        self._check(lib().amg_time_sweep(self.h, level, self._dt(u), smoother, int(n), _ptr(u), _ptr(f), _ptr(tmp),
                                         C.byref(ms), _stream()))
        return ms.value

    def timing(self, on=True):
        self._check(lib().amg_timing_enable(self.h, int(on)))

    def timing_read(self, kind, reset=True):
        n = C.c_int64()
        ms = C.c_double()
        self._check(lib().amg_timing_read(self.h, kind, C.byref(n), C.byref(ms), int(reset)))
        return n.value, ms.value

    def vcycle(self, level, f, e, opts=None):
        self._need(f, level, 0, "f")
        self._need(e, level, 0, "e", (f.dtype,))
        o = opts or default_opts()
        self._check(lib().amg_vcycle(self.h, level, self._dt(f), C.byref(o), _ptr(f), _ptr(e), _stream()))

    # ---- adjoint ----
    def solve_adjoint(self, level, lam, g, opts=None):
        """A_h^T lam = g (lam: initial guess in, solution out, face ghosts 0)."""
        import torch
        self._need(lam, level, 0, "lam", (torch.float64,))
        self._need(g, level, 0, "g", (torch.float64,))
        o = opts or default_opts()
        st = SolveStats()
        rc = lib().amg_solve_adjoint(self.h, level, _ptr(lam), _ptr(g), C.byref(o), C.byref(st), _stream())
        if rc and rc != ENOTCONVERGED:
            self._check(rc)
        out = st.as_dict()
        out["status"] = rc
        return out

    def solve_adjoint_composite(self, lams, gs, opts=None):
        """(A^comp)^T lam = g over levels 0..len(lams)-1."""
        import torch
        n = len(lams)
        for l in range(n):
            self._need(lams[l], l, 0, "lam", (torch.float64,))
            self._need(gs[l], l, 0, "g", (torch.float64,))
        o = opts or default_opts()
        st = SolveStats()
        rc = lib().amg_solve_adjoint_composite(self.h, n - 1, self._level_ptrs(lams, n), self._level_ptrs(gs, n),
                                               C.byref(o), C.byref(st), _stream())
        if rc and rc != ENOTCONVERGED:
            self._check(rc)
        out = st.as_dict()
        out["status"] = rc
        return out

    def composite_laplacian(self, xs, ys, fds=None):
        import torch
        n = len(xs)
        fds = fds or [None] * n
        for l in range(n):
            self._need(xs[l], l, 0, "x", (torch.float64,))
            self._need(ys[l], l, 0, "y", (torch.float64,))
            self._need_faces(fds[l], l)
        self._check(lib().amg_composite_laplacian(self.h, n - 1, self._level_ptrs(xs, n), self._level_ptrs(fds, n),
                                                  self._level_ptrs(ys, n), _stream()))

    def composite_residual_adjoint(self, lams, gs, rs):
        import torch
        n = len(lams)
        for l in range(n):
            for t, nm in ((lams[l], "lam"), (gs[l], "g"), (rs[l], "r")):
                self._need(t, l, 0, nm, (torch.float64,))
        self._check(lib().amg_composite_residual_adjoint(self.h, n - 1, self._level_ptrs(lams, n),
                                                         self._level_ptrs(gs, n), self._level_ptrs(rs, n), _stream()))

    def vcycle_adjoint(self, level, f, e, opts=None):
        self._need(f, level, 0, "f")
        self._need(e, level, 0, "e", (f.dtype,))
        o = opts or default_opts()
        self._check(lib().amg_vcycle_adjoint(self.h, level, self._dt(f), C.byref(o), _ptr(f), _ptr(e), _stream()))

    def apply_transpose(self, level, x, y):
        import torch
        self._need(x, level, 0, "x", (torch.float64,))
        self._need(y, level, 0, "y", (torch.float64,))
        self._check(lib().amg_apply_transpose(self.h, level, _ptr(x), _ptr(y), _stream()))

    def apply_laplacian(self, level, x, y, face_data=None):
        import torch
        self._need(x, level, 0, "x", (torch.float64,))
        self._need(y, level, 0, "y", (torch.float64,))
        self._need_faces(face_data, level)
        self._check(lib().amg_apply_laplacian(self.h, level, _ptr(x), _ptr(face_data), _ptr(y), _stream()))

    def dot(self, level, a, b):
        import torch
        self._need(a, level, 0, "a", (torch.float64,))
        self._need(b, level, 0, "b", (torch.float64,))
        out = C.c_double()
        self._check(lib().amg_dot(self.h, level, _ptr(a), _ptr(b), C.byref(out), _stream()))
        return out.value

    def dot_noalloc(self, level, a, b, out):
        """out[0] = sum over the level's cells of a b, into the device tensor
        out (no allocation, no synchronisation)."""
        import torch
        self._need(a, level, 0, "a", (torch.float64,))
        self._need(b, level, 0, "b", (torch.float64,))
        if not out.is_cuda or out.dtype != torch.float64 or out.numel() < 1:
            raise ValueError("out must be a float64 device tensor of at least one element")
        self._check(lib().amg_dot_noalloc(self.h, level, _ptr(a), _ptr(b), _ptr(out), _stream()))

    def cic_face_data(self, level, coarse_hist, k, eta, face_data, face_data_dt=None, kind=CIC_VALUE):
        """Coarse-fine face data of `level` at t* = t_-1 + eta from
        coarse_hist[i] = the level-1 data at t_-i (i = 0..3) into face_data
        (and the time derivative into face_data_dt)."""
        import torch
        if len(coarse_hist) != 4:
            raise ValueError("four coarse time levels")
        for t in coarse_hist:
            self._need(t, level - 1, 0, "coarse data", (torch.float64,))
        self._need_faces(face_data, level)
        if face_data_dt is not None:
            self._need_faces(face_data_dt, level)
        arr = (C.c_void_p * 4)(*[t.data_ptr() for t in coarse_hist])
        self._check(lib().amg_cic_face_data(self.h, level, arr, float(k), float(eta), kind, _ptr(face_data),
                                            _ptr(face_data_dt), _stream()))

    def cic_correct(self, level, face_data):
        """Eq. correctingFaceAvg on the velocity face data (one buffer per
        component, corrected in place); returns the per-component deltas."""
        if len(face_data) != self.dim:
            raise ValueError("one face-data buffer per velocity component")
        for t in face_data:
            self._need_faces(t, level)
        arr = (C.c_void_p * self.dim)(*[t.data_ptr() for t in face_data])
        n = self.level_info(level).ncomp
        out = (C.c_double * max(n, 1))()
        self._check(lib().amg_cic_correct(self.h, level, arr, out, _stream()))
        return list(out[:n])

    def set_coefficient(self, c):
        self._check(lib().amg_set_coefficient(self.h, float(c)))
        self.c = float(c)

    # ---- gradient, divergence, projection ----
    # level lists start at level lev_lo; component lists are [level][d]
    def _comp_ptrs(self, lev_lo, comps, need=True):
        import torch
        n = (lev_lo + len(comps)) * self.dim
        arr = (C.c_void_p * max(n, 1))()
        for i, per in enumerate(comps):
            l = lev_lo + i
            for d in range(self.dim):
                t = None if per is None else per[d]
                if t is None:
                    if need:
                        raise ValueError("missing component")
                    continue
                self._need(t, l, 0, "component", (torch.float64,))
                arr[l * self.dim + d] = t.data_ptr()
        return arr

    def _lev_ptrs(self, lev_lo, ts, faces=False):
        import torch
        arr = (C.c_void_p * (lev_lo + len(ts)))()
        for i, t in enumerate(ts):
            if t is None:
                continue
            if faces:
                self._need_faces(t, lev_lo + i)
            else:
                self._need(t, lev_lo + i, 0, "array", (torch.float64,))
            arr[lev_lo + i] = t.data_ptr()
        return arr

    def gradient(self, phis, gs, fds=None, lev_lo=0):
        """gs[i][d] = G_d phis[i] on levels lev_lo.. (composite if more than one)."""
        n = len(phis)
        self._check(lib().amg_gradient(self.h, lev_lo, lev_lo + n - 1, self._lev_ptrs(lev_lo, phis),
                                       self._lev_ptrs(lev_lo, fds or [None] * n, True),
                                       self._comp_ptrs(lev_lo, gs), _stream()))

    def divergence(self, ws, outs, wbs=None, lev_lo=0):
        """outs[i] = D ws[i] (ws[i][d] components); wbs[i][d] face data or None."""
        n = len(ws)
        wb = None
        if wbs is not None:
            wb = (C.c_void_p * ((lev_lo + n) * self.dim))()
            for i, per in enumerate(wbs):
                for d in range(self.dim):
                    t = None if per is None else per[d]
                    if t is not None:
                        self._need_faces(t, lev_lo + i)
                        wb[(lev_lo + i) * self.dim + d] = t.data_ptr()
        self._check(lib().amg_divergence(self.h, lev_lo, lev_lo + n - 1, self._comp_ptrs(lev_lo, ws), wb,
                                         self._lev_ptrs(lev_lo, outs), _stream()))

    def gradient_transpose(self, mus, outs, lev_lo=0):
        """outs[i] = sum_d G_d^T mus[i][d] (mus' covered cells and ghosts are
        set to 0)."""
        n = len(outs)
        self._check(lib().amg_gradient_transpose(self.h, lev_lo, lev_lo + n - 1, self._comp_ptrs(lev_lo, mus),
                                                 self._lev_ptrs(lev_lo, outs), _stream()))

    def divergence_transpose(self, lams, outs, lev_lo=0):
        """outs[i][d] = G_d^T lams[i] (lams' covered cells and ghosts are set
        to 0)."""
        n = len(lams)
        self._check(lib().amg_divergence_transpose(self.h, lev_lo, lev_lo + n - 1, self._lev_ptrs(lev_lo, lams),
                                                   self._comp_ptrs(lev_lo, outs), _stream()))


def project_adjoint(Hw, Hp, ubars, lams, wbars, opts=None, lev_lo=0):
    """wbar = P^T ubar (see amg_project_adjoint); ubars[i][d] (covered cells
    and ghosts set to 0), lams[i] initial guess in, adjoint potential out;
    wbars may be ubars."""
    n = len(lams)
    o = opts or default_opts()
    st = SolveStats()
    rc = lib().amg_project_adjoint(Hw.h, Hp.h, lev_lo, lev_lo + n - 1, Hp._comp_ptrs(lev_lo, ubars),
                                   Hp._lev_ptrs(lev_lo, lams), Hw._comp_ptrs(lev_lo, wbars), C.byref(o), C.byref(st),
                                   _stream())
    if rc and rc != ENOTCONVERGED:
        Hp._check(rc)
    out = st.as_dict()
    out["status"] = rc
    return out


def project(Hw, Hp, ws, phis, us, wbs=None, opts=None, lev_lo=0):
    """u = w - G phi with L phi = D w (see amg_project); Hw: velocity fill,
    Hp: pure-Neumann Poisson hierarchy with the same boxes."""
    n = len(ws)
    wb = None
    if wbs is not None:
        wb = (C.c_void_p * ((lev_lo + n) * Hw.dim))()
        for i, per in enumerate(wbs):
            for d in range(Hw.dim):
                t = None if per is None else per[d]
                if t is not None:
                    Hw._need_faces(t, lev_lo + i)
                    wb[(lev_lo + i) * Hw.dim + d] = t.data_ptr()
    o = opts or default_opts()
    st = SolveStats()
    rc = lib().amg_project(Hw.h, Hp.h, lev_lo, lev_lo + n - 1, Hw._comp_ptrs(lev_lo, ws), wb,
                           Hp._lev_ptrs(lev_lo, phis), Hp._comp_ptrs(lev_lo, us), C.byref(o), C.byref(st), _stream())
    if rc and rc != ENOTCONVERGED:
        Hp._check(rc)
    out = st.as_dict()
    out["status"] = rc
    return out


def imex_step(Hv, Hp, dt, nu, us, gs=None, opts=None, opts_p=None):
    """One step of eq. GePUP-IMEX on one periodic box (see amg_imex_step):
    us[d] holds u^n on entry and u^(n+1) on return; gs: None or gs[j][d],
    the forcing at t_n + IMEX_C[j] dt; opts: the Helmholtz solves, opts_p:
    the Poisson solves (None: opts).  Returns the stats and status."""
    import torch
    arr = Hv._comp_ptrs(0, [us])
    g = None
    if gs is not None:
        if len(gs) != len(IMEX_C):
            raise ValueError("the forcing needs one entry per stage")
        g = (C.c_void_p * (len(IMEX_C) * Hv.dim))()
        for j, per in enumerate(gs):
            for d in range(Hv.dim):
                Hv._need(per[d], 0, 0, "forcing", (torch.float64,))
                g[j * Hv.dim + d] = per[d].data_ptr()
    o = opts or default_opts()
    op = C.byref(opts_p) if opts_p is not None else None
    st = ImexStats()
    rc = lib().amg_imex_step(Hv.h, Hp.h, float(dt), float(nu), arr, g, C.byref(o), op, C.byref(st), _stream())
    if rc and rc != ENOTCONVERGED:
        Hv._check(rc)
    out = st.as_dict()
    out["status"] = rc
    return out



def convection(H, us, outs):
    """outs[d] = (Div<uu>)_d of eq. convOp on one periodic box (see
    amg_convection)."""
    H._check(lib().amg_convection(H.h, H._comp_ptrs(0, [us]), H._comp_ptrs(0, [outs]), _stream()))


def _boxes_out(dim, n, lo, hi):
    return [(tuple(int(v) for v in lo[i * dim:(i + 1) * dim]), tuple(int(v) for v in hi[i * dim:(i + 1) * dim]))
            for i in range(n)]


SC_KINDS = ("synced", "regrid", "advance", "sync")  # AMG_SC_SYNCED .. AMG_SC_SYNC


class ScEvent(C.Structure):
    _fields_ = [("kind", C.c_int32), ("level", C.c_int32), ("t", C.c_double), ("dt", C.c_double),
                ("k_coarse", C.c_double), ("t_coarse", C.c_double)]


def subcycle_schedule(nlevels, ratio, t0, k0, ncoarse, regrid_every=0):
    """Algorithm 1's events (see amg_subcycle_schedule) as tuples (kind,
    level, t, dt, k_coarse, t_coarse), kind one of SC_KINDS."""
    n = C.c_int32()
    rc = lib().amg_subcycle_schedule(nlevels, ratio, float(t0), float(k0), ncoarse, regrid_every, 0, C.byref(n),
                                     None)
    if rc and rc != EUNSUPPORTED:
        raise AmgError(rc, "amg_subcycle_schedule failed")
    ev = (ScEvent * max(1, n.value))()
    rc = lib().amg_subcycle_schedule(nlevels, ratio, float(t0), float(k0), ncoarse, regrid_every, n.value,
                                     C.byref(n), ev)
    if rc:
        raise AmgError(rc, "amg_subcycle_schedule failed")
    return [(SC_KINDS[e.kind], e.level, e.t, e.dt, e.k_coarse, e.t_coarse) for e in ev[:n.value]]


def dense_inverse(a, threads=1):
    """The inverse of the square FP64 matrix a (see amg_dense_inverse: the
    bottom solve's factorisation, on the host)."""
    import numpy as np
    m = np.array(a, dtype=np.float64, order="C", copy=True)
    if m.ndim != 2 or m.shape[0] != m.shape[1]:
        raise ValueError("a square matrix is required")
    rc = lib().amg_dense_inverse(m.shape[0], m.ctypes.data_as(C.POINTER(C.c_double)), int(threads))
    if rc:
        raise AmgError(rc, "amg_dense_inverse failed")
    return m


def cluster(tags, efficiency=0.75, min_side=2, max_boxes=4096):
    """Boxes of the tagged cells of a dense boolean array indexed [x, y(, z)]
    (see amg_cluster)."""
    import numpy as np
    t = np.ascontiguousarray(np.asarray(tags, dtype=np.uint8).T)  # x fastest
    dim = t.ndim
    shape = (C.c_int32 * dim)(*np.asarray(tags).shape)
    nb = C.c_int32()
    lo = (C.c_int32 * (max_boxes * dim))()
    hi = (C.c_int32 * (max_boxes * dim))()
    rc = lib().amg_cluster(dim, shape, t.ctypes.data_as(C.POINTER(C.c_uint8)), float(efficiency), int(min_side),
                           max_boxes, C.byref(nb), lo, hi)
    if rc:
        raise AmgError(rc, "amg_cluster failed")
    return _boxes_out(dim, nb.value, lo, hi)


def regrid_boxes(base_cells, ratio, tags, efficiency=0.75, min_side=2, grow=0, block=0, max_boxes=4096):
    """Boxes of new levels 1..len(tags) from dense boolean tag arrays of
    levels 0..len(tags)-1, indexed [x, y(, z)] (see amg_regrid_boxes; grow,
    block = 0: the defaults)."""
    import numpy as np
    dim = len(base_cells)
    arrs = [np.ascontiguousarray(np.asarray(t, dtype=np.uint8).T) for t in tags]
    ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
    nt = len(arrs)
    nb = (C.c_int32 * nt)()
    lo = (C.c_int32 * (nt * max_boxes * dim))()
    hi = (C.c_int32 * (nt * max_boxes * dim))()
    rc = lib().amg_regrid_boxes(dim, (C.c_int32 * dim)(*base_cells), int(ratio), nt, ptrs, float(efficiency),
                                int(min_side), int(grow), int(block), max_boxes, nb, lo, hi)
    if rc:
        raise AmgError(rc, "amg_regrid_boxes failed")
    out = []
    for l in range(nt):
        off = l * max_boxes * dim
        out.append(_boxes_out(dim, nb[l], lo[off:off + max_boxes * dim], hi[off:off + max_boxes * dim]))
    return out


def tag_vorticity(H, us, eps, tags):
    """tags[l] (uint8 device tensors, one byte per cell of level l's grid, x
    fastest) from the velocity us[l][d] (see amg_tag_vorticity)."""
    n = len(tags)
    ptrs = (C.c_void_p * n)(*[t.data_ptr() for t in tags])
    H._check(lib().amg_tag_vorticity(H.h, n - 1, H._comp_ptrs(0, us), float(eps), ptrs, _stream()))


def migrate(H_old, H_new, u_old, u_new):
    """u_new[l] on the new hierarchy from u_old[l] (see amg_migrate)."""
    H_new._check(lib().amg_migrate(H_old.h, H_new.h, H_old._lev_ptrs(0, u_old), H_new._lev_ptrs(0, u_new), _stream()))
