"""torch.autograd binding of level and composite solves.

``level_solve(f, c, H, level, face_data, opts)`` returns x with
A x = f - b(face_data) on one level of the hierarchy H (the Helmholtz
system (I - cL) or the Poisson system L; pure-Neumann components solved for
the mean-free x after the right-hand-side shift).  It is differentiable in f
and, for the Helmholtz operator, in the coefficient c = gamma nu k, so a
caller that builds c from nu obtains dJ/dnu = gamma k dJ/dc by autograd.

Backward (the adjoint of the level system, not in the paper): lam solves
A_h^T lam = dJ/dx by the library's adjoint multigrid solve (mean-free source
and solution on singular components); dJ/df = lam and dJ/dc = <lam, L x>
with L the Laplacian of x with the solve's face data.  Only the cells of the
level carry gradient: the ghost entries of dJ/dx are ignored and those of
dJ/df are zero.  No gradient flows to the face data.  Every step runs in the
HIP library; this module only passes tensors.

``composite_solve(fs, c, H, face_data, opts)`` does the same for the
composite system over levels 0..len(fs)-1 (x on every level, covered cells
holding averages): backward solves the composite adjoint system, dJ/df_l =
lam_l (zero on covered cells) and dJ/dc = sum_l <lam_l, (L^comp x)_l>.
Gradients reach x through its valid cells only.

``project(ws, Hw, Hp, opts)`` returns the projected velocity u = P w of
eq. appProj (composite eq. comp_ProjOp over levels 0..len(ws)-1 when there
are several; ws[l][d] component d on level l), with homogeneous velocity
data.  P is linear, so backward needs no saved tensor: dJ/dw = P^T dJ/du by
the library's transposed gradient, adjoint pure-Neumann solve and transposed
divergence (amg_project_adjoint).

Checkpointing: ``level_solve`` and ``composite_solve`` take
``checkpoint=True`` to keep only their inputs (the right-hand sides, which
the caller holds anyway) instead of the solution on every level, and solve
again in backward when the solution is needed (for dJ/dc); the adjoint needs
no solution.  This trades one forward solve for the memory of the solutions
of all levels.
"""
import torch

from . import amg as A


class _coefficient:
    """Runs a backward with the Helmholtz coefficient of its forward solve
    (another forward on the same hierarchy may have changed it since) and
    puts the hierarchy's coefficient back afterwards."""

    def __init__(self, H, c):
        self.H, self.c, self.prev = H, c, None

    def __enter__(self):
        if self.H.op_kind == A.HELMHOLTZ and self.H.c != self.c:
            self.prev = self.H.c
            self.H.set_coefficient(self.c)

    def __exit__(self, *exc):
        if self.prev is not None:
            self.H.set_coefficient(self.prev)
        return False


class LevelSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, c, H, level, face_data, opts, checkpoint):
        if H.op_kind == A.HELMHOLTZ:
            cv = float(c)
            if cv != H.c:
                H.set_coefficient(cv)
        x = _level_forward(H, level, f, face_data, opts)
        ctx.H, ctx.level, ctx.face_data, ctx.opts = H, level, face_data, opts
        ctx.c_fwd = H.c  # the coefficient this solve used (the hierarchy may change it before backward)
        ctx.c_is_tensor = torch.is_tensor(c)
        ctx.c_meta = (c.dtype, c.device) if ctx.c_is_tensor else None
        ctx.checkpoint = bool(checkpoint)
        # checkpointing keeps the input (held by the caller anyway), not x
        ctx.save_for_backward(f if ctx.checkpoint else x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (saved,) = ctx.saved_tensors
        H, level = ctx.H, ctx.level
        with _coefficient(H, ctx.c_fwd):
            lam = torch.zeros_like(saved)
            st = H.solve_adjoint(level, lam, gx.contiguous(), ctx.opts)
            if st["status"] != 0:
                raise A.AmgError(st["status"], f"adjoint solve did not converge: {st}")
            gc = None
            if ctx.c_is_tensor and ctx.needs_input_grad[1] and H.op_kind == A.HELMHOLTZ:
                x = _level_forward(H, level, saved, ctx.face_data, ctx.opts) if ctx.checkpoint else saved.clone()
                y = torch.zeros_like(x)
                H.apply_laplacian(level, x, y, ctx.face_data)
                gc = torch.tensor(H.dot(level, lam, y), dtype=ctx.c_meta[0], device=ctx.c_meta[1])
        return lam, gc, None, None, None, None, None


def _level_forward(H, level, f, face_data, opts):
    x = torch.zeros_like(f)
    st = H.solve(level, x, f.contiguous(), face_data, opts)
    if st["status"] != 0:
        raise A.AmgError(st["status"], f"level solve did not converge: {st}")
    return x


def level_solve(f, c, H, level=0, face_data=None, opts=None, checkpoint=False):
    """x = A^-1 (f - b(face_data)), differentiable in f and (Helmholtz) c."""
    return LevelSolve.apply(f, c, H, level, face_data, opts, checkpoint)


def _composite_forward(H, fs, face_data, opts):
    xs = [torch.zeros_like(f) for f in fs]
    st = H.solve_composite(xs, [f.contiguous() for f in fs], face_data, opts)
    if st["status"] != 0:
        raise A.AmgError(st["status"], f"composite solve did not converge: {st}")
    return xs


class CompositeSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, H, face_data, opts, checkpoint, *fs):
        if H.op_kind == A.HELMHOLTZ:
            cv = float(c)
            if cv != H.c:
                H.set_coefficient(cv)
        xs = _composite_forward(H, fs, face_data, opts)
        ctx.H, ctx.face_data, ctx.opts = H, face_data, opts
        ctx.c_fwd = H.c
        ctx.c_meta = (c.dtype, c.device) if torch.is_tensor(c) else None
        ctx.checkpoint = bool(checkpoint)
        ctx.save_for_backward(*(fs if ctx.checkpoint else xs))
        return tuple(xs)

    @staticmethod
    def backward(ctx, *gxs):
        saved = ctx.saved_tensors
        H = ctx.H
        with _coefficient(H, ctx.c_fwd):
            lams = [torch.zeros_like(t) for t in saved]
            gs = [g.contiguous() if g is not None else torch.zeros_like(t) for g, t in zip(gxs, saved)]
            st = H.solve_adjoint_composite(lams, gs, ctx.opts)
            if st["status"] != 0:
                raise A.AmgError(st["status"], f"composite adjoint solve did not converge: {st}")
            gc = None
            if ctx.c_meta is not None and ctx.needs_input_grad[0] and H.op_kind == A.HELMHOLTZ:
                if ctx.checkpoint:
                    xx = _composite_forward(H, saved, ctx.face_data, ctx.opts)
                else:
                    xx = [x.clone() for x in saved]
                ys = [torch.zeros_like(x) for x in xx]
                H.composite_laplacian(xx, ys, ctx.face_data)
                tot = sum(H.dot(l, lams[l], ys[l]) for l in range(len(xx)))
                gc = torch.tensor(tot, dtype=ctx.c_meta[0], device=ctx.c_meta[1])
        return (gc, None, None, None, None, *lams)


def composite_solve(fs, c, H, face_data=None, opts=None, checkpoint=False):
    """[x_l] solving the composite system, differentiable in every f_l and
    (Helmholtz) c."""
    return list(CompositeSolve.apply(c, H, face_data, opts, checkpoint, *fs))


class Project(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Hw, Hp, opts, n, *ws):
        dim = Hw.dim
        # amg_project writes the ghosts (and covered cells) of its input: copies
        w = [[ws[l * dim + d].detach().clone() for d in range(dim)] for l in range(n)]
        phis = [torch.zeros_like(w[l][0]) for l in range(n)]
        us = [[torch.empty_like(w[l][d]) for d in range(dim)] for l in range(n)]
        st = A.project(Hw, Hp, w, phis, us, opts=opts)
        if st["status"] != 0:
            raise A.AmgError(st["status"], f"projection solve did not converge: {st}")
        ctx.Hw, ctx.Hp, ctx.opts, ctx.n = Hw, Hp, opts, n
        return tuple(us[l][d] for l in range(n) for d in range(dim))

    @staticmethod
    def backward(ctx, *gus):
        Hw, Hp, n = ctx.Hw, ctx.Hp, ctx.n
        dim = Hw.dim
        ub = [[gus[l * dim + d].detach().clone() for d in range(dim)] for l in range(n)]
        lams = [torch.zeros_like(ub[l][0]) for l in range(n)]
        st = A.project_adjoint(Hw, Hp, ub, lams, ub, ctx.opts)
        if st["status"] != 0:
            raise A.AmgError(st["status"], f"adjoint projection solve did not converge: {st}")
        return (None, None, None, None, *(ub[l][d] for l in range(n) for d in range(dim)))


def project(ws, Hw, Hp, opts=None):
    """u = P w (eq. appProj; composite over levels 0..len(ws)-1 if several),
    ws[l][d] the velocity component d on level l; returns us[l][d].
    Differentiable in w."""
    n, dim = len(ws), Hw.dim
    flat = Project.apply(Hw, Hp, opts, n, *(ws[l][d] for l in range(n) for d in range(dim)))
    return [[flat[l * dim + d] for d in range(dim)] for l in range(n)]
