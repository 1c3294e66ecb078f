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
    def forward(ctx, f, c, H, level, face_data, opts):
        if H.op_kind == A.HELMHOLTZ:
            cv = float(c)
            if cv != H.c:
                H.set_coefficient(cv)
        x = torch.zeros_like(f)
        st = H.solve(level, x, f.contiguous(), face_data, opts)
        if st["status"] != 0:
            raise A.AmgError(st["status"], f"level solve did not converge: {st}")
        ctx.H, ctx.level, ctx.face_data, ctx.opts = H, level, face_data, opts
        ctx.c_fwd = H.c  # the coefficient this solve used (the hierarchy may change it before backward)
        ctx.c_is_tensor = torch.is_tensor(c)
        ctx.c_meta = (c.dtype, c.device) if ctx.c_is_tensor else None
        ctx.save_for_backward(x)
        return x

    @staticmethod
    def backward(ctx, gx):
        (x,) = ctx.saved_tensors
        H, level = ctx.H, ctx.level
        with _coefficient(H, ctx.c_fwd):
            lam = torch.zeros_like(x)
            st = H.solve_adjoint(level, lam, gx.contiguous(), ctx.opts)
            if st["status"] != 0:
                raise A.AmgError(st["status"], f"adjoint solve did not converge: {st}")
            gc = None
            if ctx.c_is_tensor and ctx.needs_input_grad[1] and H.op_kind == A.HELMHOLTZ:
                xx = x.clone()
                y = torch.zeros_like(x)
                H.apply_laplacian(level, xx, y, ctx.face_data)
                gc = torch.tensor(H.dot(level, lam, y), dtype=ctx.c_meta[0], device=ctx.c_meta[1])
        return lam, gc, None, None, None, None


def level_solve(f, c, H, level=0, face_data=None, opts=None):
    """x = A^-1 (f - b(face_data)), differentiable in f and (Helmholtz) c."""
    return LevelSolve.apply(f, c, H, level, face_data, opts)


class CompositeSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, H, face_data, opts, *fs):
        if H.op_kind == A.HELMHOLTZ:
            cv = float(c)
            if cv != H.c:
                H.set_coefficient(cv)
        xs = [torch.zeros_like(f) for f in fs]
        st = H.solve_composite(xs, [f.contiguous() for f in fs], face_data, opts)
        if st["status"] != 0:
            raise A.AmgError(st["status"], f"composite solve did not converge: {st}")
        ctx.H, ctx.face_data, ctx.opts = H, face_data, opts
        ctx.c_fwd = H.c
        ctx.c_meta = (c.dtype, c.device) if torch.is_tensor(c) else None
        ctx.save_for_backward(*xs)
        return tuple(xs)

    @staticmethod
    def backward(ctx, *gxs):
        xs = ctx.saved_tensors
        H = ctx.H
        with _coefficient(H, ctx.c_fwd):
            lams = [torch.zeros_like(x) for x in xs]
            gs = [g.contiguous() if g is not None else torch.zeros_like(x) for g, x in zip(gxs, xs)]
            st = H.solve_adjoint_composite(lams, gs, ctx.opts)
            if st["status"] != 0:
                raise A.AmgError(st["status"], f"composite adjoint solve did not converge: {st}")
            gc = None
            if ctx.c_meta is not None and ctx.needs_input_grad[0] and H.op_kind == A.HELMHOLTZ:
                xx = [x.clone() for x in xs]
                ys = [torch.zeros_like(x) for x in xs]
                H.composite_laplacian(xx, ys, ctx.face_data)
                tot = sum(H.dot(l, lams[l], ys[l]) for l in range(len(xs)))
                gc = torch.tensor(tot, dtype=ctx.c_meta[0], device=ctx.c_meta[1])
        return (gc, None, None, None, *lams)


def composite_solve(fs, c, H, face_data=None, opts=None):
    """[x_l] solving the composite system, differentiable in every f_l and
    (Helmholtz) c."""
    return list(CompositeSolve.apply(c, H, face_data, opts, *fs))
