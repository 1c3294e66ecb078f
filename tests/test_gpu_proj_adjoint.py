"""Transposed gradient, divergence and projection on the GPU against the
oracle (oracle/proj_adj.py, pinned by dot-product identities): element by
element on levels (one box, two boxes, a refined level with face-data
ghosts, 3D) and over two- and three-level hierarchies (interpolated ghosts,
refluxing, average-down); the adjoint projection against the oracle's; and
the gradient of the vortex workload's loss (composite Helmholtz solves of
both velocity components, then the composite projection, then the
volume-weighted ||u - u_t||^2) in the forcing g and in nu, through the
autograd binding, on a reduced three-level hierarchy: against the oracle's
adjoint chain and against central finite differences (step 1e-6), with and
without checkpointing."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import amr, amr_adj, proj, proj_adj  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd import autograd as AG  # noqa: E402
from tests.gpuhelp import from_dev, make_hier, to_dev  # noqa: E402

TOL = 1e-12


def levels(name):
    bc = {(d, s): "D" for d in range(2) for s in (0, 1)}
    if name == "box":
        return Level((32, 32), 1 / 32, [((0, 0), (31, 31))], bc)
    if name == "two_boxes":
        return Level((32, 32), 1 / 32, [((0, 0), (15, 31)), ((16, 0), (31, 31))], bc)
    if name == "refined":
        return Level((32, 32), 1 / 32, [((4, 8), (19, 23)), ((20, 8), (27, 15))], bc, "D")
    if name == "box3d":
        return Level((16, 16, 16), 1 / 16, [((0, 0, 0), (15, 15, 15))], {(d, s): "D" for d in range(3) for s in (0, 1)})
    raise KeyError(name)


def rand(lev, seed):
    rng = np.random.default_rng(seed)
    return np.where(lev.mask, rng.normal(size=lev.pshape), 0.0)


def rel(got, want, mask):
    return float(np.abs(got - want)[mask].max() / max(np.abs(want)[mask].max(), 1e-300))


@pytest.mark.parametrize("name", ["box", "two_boxes", "refined", "box3d"])
def test_level_transposes(name):
    lev = levels(name)
    lw, lp = proj.velocity_level(lev), proj.pressure_level(lev)
    D = lev.dim
    Hp, L = make_hier(lp, "poisson", 0.0)
    Hw, _ = make_hier(lw, "poisson", 0.0)
    mu = [rand(lev, 10 + d) for d in range(D)]
    want = proj_adj.gradient_T(lp, mu)
    mus = [to_dev(Hp, L, 0, m) for m in mu]
    out = torch.zeros_like(mus[0])
    Hp.gradient_transpose([mus], [out], lev_lo=L)
    torch.cuda.synchronize()
    assert rel(from_dev(Hp, L, 0, out, lp), want, lp.mask) < TOL
    lam = rand(lev, 20)
    want = proj_adj.divergence_T(lw, lam)
    outs = [torch.zeros_like(mus[0]) for _ in range(D)]
    Hw.divergence_transpose([to_dev(Hw, L, 0, lam)], [outs], lev_lo=L)
    torch.cuda.synchronize()
    for d in range(D):
        assert rel(from_dev(Hw, L, 0, outs[d], lw), want[d], lw.mask) < TOL, d


HIERS = {
    "two_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((8, 8), (15, 23)), ((16, 8), (23, 15))]]),
    "three_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((4, 4), (27, 27))], [((16, 16), (31, 31))]]),
    "boundary": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((0, 0), (15, 15)), ((16, 0), (23, 11))]]),
    "two_boxes_c": ((32, 16), 1 / 32, [[((0, 0), (15, 15)), ((16, 0), (31, 15))],
                                      [((0, 0), (15, 15)), ((16, 0), (23, 11))]]),
}


def gpu_hier(name, kind, op=A.POISSON, c=0.0):
    base, h0, boxes = HIERS[name]
    H = A.Hierarchy(2, base, h0, len(boxes))
    for l, bl in enumerate(boxes):
        H.set_level_boxes(l, bl)
        if l:
            H.set_cf_mode(l, A.CF_INTERP)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
    H.set_operator(op, c)
    H.finalize()
    return H


def oracle_hier(name, kind):
    base, h0, boxes = HIERS[name]
    return amr.Hierarchy(base, h0, boxes, {(d, s): kind for d in range(2) for s in (0, 1)})


def rand_valid(OH, seed):
    rng = np.random.default_rng(seed)
    return [np.where(OH.valid[l], rng.normal(size=lev.pshape), 0.0) for l, lev in enumerate(OH.levels)]


def vrel(OH, got, want):
    num = max(np.abs(got[l] - want[l])[OH.valid[l]].max() for l in range(OH.nlev))
    den = max(np.abs(want[l])[OH.valid[l]].max() for l in range(OH.nlev))
    return num / den


@pytest.mark.parametrize("name", sorted(HIERS))
def test_composite_transposes(name):
    Op, Ow = oracle_hier(name, "N"), oracle_hier(name, "D")
    Hp, Hw = gpu_hier(name, "N"), gpu_hier(name, "D")
    nl = Op.nlev
    mu = [rand_valid(Op, 30 + d) for d in range(2)]
    want = proj_adj.composite_gradient_T(Op, mu)
    mus = [[to_dev(Hp, l, 0, mu[d][l]) for d in range(2)] for l in range(nl)]
    outs = [torch.zeros_like(mus[l][0]) for l in range(nl)]
    Hp.gradient_transpose(mus, outs)
    torch.cuda.synchronize()
    got = [from_dev(Hp, l, 0, outs[l], Op.levels[l]) for l in range(nl)]
    assert vrel(Op, got, want) < TOL
    for l in range(nl):  # zero off the valid cells
        assert np.all(got[l][Op.levels[l].mask & ~Op.valid[l]] == 0.0)
    lam = rand_valid(Ow, 40)
    want = proj_adj.composite_divergence_T(Ow, lam)
    lams = [to_dev(Hw, l, 0, lam[l]) for l in range(nl)]
    outs = [[torch.zeros_like(lams[l]) for _ in range(2)] for l in range(nl)]
    Hw.divergence_transpose(lams, outs)
    torch.cuda.synchronize()
    for d in range(2):
        got = [from_dev(Hw, l, 0, outs[l][d], Ow.levels[l]) for l in range(nl)]
        assert vrel(Ow, got, want[d]) < TOL, d


@pytest.mark.parametrize("name", ["two_level", "three_level"])
def test_composite_projection_adjoint(name):
    OH = oracle_hier(name, "D")
    Hw, Hp = gpu_hier(name, "D"), gpu_hier(name, "N")
    nl = OH.nlev
    ub = [rand_valid(OH, 50 + d) for d in range(2)]
    want, lam_o, st_o = proj_adj.composite_project_T(OH, ub, tol_rel=1e-13, max_cycles=400)
    assert st_o["converged"]
    ubs = [[to_dev(Hw, l, 0, ub[d][l]) for d in range(2)] for l in range(nl)]
    lams = [torch.zeros_like(ubs[l][0]) for l in range(nl)]
    wbs = [[torch.zeros_like(ubs[l][0]) for _ in range(2)] for l in range(nl)]
    st = A.project_adjoint(Hw, Hp, ubs, lams, wbs, A.default_opts(precision=A.FP64, tol_rel=1e-13,
                                                                  max_cycles=400))
    assert st["status"] == 0 and st["converged"], st
    for d in range(2):
        got = [from_dev(Hw, l, 0, wbs[l][d], OH.levels[l]) for l in range(nl)]
        assert vrel(OH, got, want[d]) < 1e-9, d
    # in place (wbar aliases ubar) gives the same values
    ubs2 = [[to_dev(Hw, l, 0, ub[d][l]) for d in range(2)] for l in range(nl)]
    lams2 = [torch.zeros_like(ubs2[l][0]) for l in range(nl)]
    A.project_adjoint(Hw, Hp, ubs2, lams2, ubs2, A.default_opts(precision=A.FP64, tol_rel=1e-13, max_cycles=400))
    for l in range(nl):
        for d in range(2):
            assert torch.equal(ubs2[l][d], wbs[l][d])


# ---------------------------------------------------------------------------
# the vortex workload's loss on a reduced three-level hierarchy
RBASE = 32
RBOXES = [[((0, 0), (31, 31))], [((16, 16), (47, 47))], [((40, 40), (71, 71))]]
K = 1.0 / RBASE
GAMMA = 0.5


_ORACLE = {}


class Chain:
    """Helmholtz solves of both components (Dirichlet, composite), the
    composite projection, and J = sum over valid cells of h^D (u - t)^2."""

    def __init__(self):
        bc = {(d, s): "D" for d in range(2) for s in (0, 1)}
        self.OH = amr.Hierarchy((RBASE, RBASE), 1.0 / RBASE, RBOXES, bc)
        self.Hh = self._gpu("D", A.HELMHOLTZ, GAMMA * 1e-2 * K)
        self.Hw = self._gpu("D", A.POISSON, 0.0)
        self.Hp = self._gpu("N", A.POISSON, 0.0)
        rng = np.random.default_rng(60)
        OH = self.OH
        self.w0 = [[np.where(OH.levels[l].mask, rng.normal(size=OH.levels[l].pshape), 0.0) for l in range(3)]
                   for _ in range(2)]
        for d in range(2):
            self.w0[d] = OH.average_down_all(self.w0[d])
        self.t = [rand_valid(OH, 61 + d) for d in range(2)]
        self.g = [rand_valid(OH, 63 + d) for d in range(2)]
        self.wts = [np.where(OH.valid[l], OH.levels[l].h ** 2, 0.0) for l in range(3)]
        self.opts = A.default_opts(precision=A.FP64, smoother=A.SMOOTH_RB, tol_rel=1e-13, max_cycles=300)

    def _gpu(self, kind, op, c):
        H = A.Hierarchy(2, (RBASE, RBASE), 1.0 / RBASE, 3)
        for l, bl in enumerate(RBOXES):
            H.set_level_boxes(l, bl)
            if l:
                H.set_cf_mode(l, A.CF_INTERP)
        for d in range(2):
            for s in (0, 1):
                H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
        H.set_operator(op, c)
        H.finalize()
        return H

    def dev(self, arrs, H=None):
        H = H or self.Hh
        return [to_dev(H, l, 0, arrs[l]) for l in range(3)]

    def loss(self, g_dev, nu, checkpoint=False):
        """J(g, nu) through the autograd binding; g_dev[d][l] device tensors."""
        c = GAMMA * nu * K
        xs = []
        for d in range(2):
            b = [self.w0d[d][l] + K * g_dev[d][l] for l in range(3)]
            xs.append(AG.composite_solve(b, c, self.Hh, None, self.opts, checkpoint=checkpoint))
        us = AG.project([[xs[d][l] for d in range(2)] for l in range(3)], self.Hw, self.Hp, self.opts)
        J = 0.0
        for d in range(2):
            for l in range(3):
                J = J + (self.wdev[l] * (us[l][d] - self.tdev[d][l]) ** 2).sum()
        return J

    def prepare(self):
        self.w0d = [self.dev(self.w0[d]) for d in range(2)]
        self.tdev = [self.dev(self.t[d]) for d in range(2)]
        self.wdev = self.dev(self.wts)

    def oracle_gradient(self, nu):
        """dJ/dg and dJ/dnu by the oracle's adjoint chain (computed once per
        nu for the module)."""
        if nu not in _ORACLE:
            _ORACLE[nu] = self._oracle_gradient(nu)
        return _ORACLE[nu]

    def _oracle_gradient(self, nu):
        OH, c = self.OH, GAMMA * nu * K
        X = []
        for d in range(2):
            b = [self.w0[d][l] + K * self.g[d][l] for l in range(3)]
            x, st = amr.composite_solve(OH, b, "helmholtz", c, None, tol_rel=1e-14, max_cycles=300)
            assert st["converged"]
            X.append(x)
        U, _, st = proj.composite_project(OH, X, tol_rel=1e-14, max_cycles=400)
        assert st["converged"]
        ub = [[np.where(OH.valid[l], 2 * self.wts[l] * (U[d][l] - self.t[d][l]), 0.0) for l in range(3)]
              for d in range(2)]
        wb, _, st = proj_adj.composite_project_T(OH, ub, tol_rel=1e-14, max_cycles=400)
        assert st["converged"]
        gg, gnu = [], 0.0
        for d in range(2):
            lam, st = amr_adj.composite_solve_T(OH, wb[d], "helmholtz", c, tol_rel=1e-14, max_cycles=300)
            assert st["converged"]
            gg.append([K * lam[l] for l in range(3)])
            gnu += GAMMA * K * amr_adj.grad_c(OH, lam, X[d])
        return gg, gnu


@pytest.mark.parametrize("checkpoint", [False, True])
def test_vortex_loss_gradient_against_oracle_and_differences(checkpoint):
    ch = Chain()
    ch.prepare()
    OH = ch.OH
    nu0 = 1e-2
    gd = [[t.clone().requires_grad_(True) for t in ch.dev(ch.g[d])] for d in range(2)]
    nu = torch.tensor(nu0, dtype=torch.float64, requires_grad=True)
    J = ch.loss(gd, nu, checkpoint)
    J.backward()
    gg, gnu = ch.oracle_gradient(nu0)
    for d in range(2):
        got = [from_dev(ch.Hh, l, 0, gd[d][l].grad, OH.levels[l]) for l in range(3)]
        assert vrel(OH, got, gg[d]) < 1e-8, d
        for l in range(3):  # no gradient on covered cells: they do not enter the loss
            assert np.all(got[l][OH.levels[l].mask & ~OH.valid[l]] == 0.0)
    assert abs(nu.grad.item() - gnu) < 1e-7 * abs(gnu)
    # central differences (step 1e-6 relative) in nu and along a random direction of g
    with torch.no_grad():
        eps = 1e-6 * nu0
        fd_nu = (ch.loss(gd, torch.tensor(nu0 + eps, dtype=torch.float64)).item()
                 - ch.loss(gd, torch.tensor(nu0 - eps, dtype=torch.float64)).item()) / (2 * eps)
        rng = np.random.default_rng(70)
        dirs = [ch.dev([np.where(OH.valid[l], rng.normal(size=OH.levels[l].pshape), 0.0) for l in range(3)])
                for d in range(2)]
        h = 1e-6
        gp = [[gd[d][l] + h * dirs[d][l] for l in range(3)] for d in range(2)]
        gm = [[gd[d][l] - h * dirs[d][l] for l in range(3)] for d in range(2)]
        fd_g = (ch.loss(gp, nu0).item() - ch.loss(gm, nu0).item()) / (2 * h)
    dir_grad = sum(float((gd[d][l].grad * dirs[d][l]).sum()) for d in range(2) for l in range(3))
    assert abs(nu.grad.item() - fd_nu) < 1e-5 * abs(fd_nu), (nu.grad.item(), fd_nu)
    assert abs(dir_grad - fd_g) < 1e-6 * abs(fd_g), (dir_grad, fd_g)


def test_checkpointing_gives_the_same_gradients_and_saves_no_solution():
    ch = Chain()
    ch.prepare()
    grads = []
    for checkpoint in (False, True):
        gd = [[t.clone().requires_grad_(True) for t in ch.dev(ch.g[d])] for d in range(2)]
        nu = torch.tensor(1e-2, dtype=torch.float64, requires_grad=True)
        J = ch.loss(gd, nu, checkpoint)
        J.backward()
        grads.append(([[t.grad.clone() for t in per] for per in gd], nu.grad.item()))
    for d in range(2):
        for l in range(3):
            assert torch.equal(grads[0][0][d][l], grads[1][0][d][l])
    assert grads[0][1] == grads[1][1]
    # the checkpointed solve keeps its inputs only
    b = [ch.w0d[0][l].clone().requires_grad_(True) for l in range(3)]
    xs = AG.composite_solve(b, GAMMA * 1e-2 * K, ch.Hh, None, ch.opts, checkpoint=True)
    saved = xs[0].grad_fn.saved_tensors
    assert len(saved) == 3 and all(s.data_ptr() == bb.data_ptr() for s, bb in zip(saved, b))
    xs2 = AG.composite_solve(b, GAMMA * 1e-2 * K, ch.Hh, None, ch.opts, checkpoint=False)
    saved2 = xs2[0].grad_fn.saved_tensors
    assert all(s.data_ptr() == x.data_ptr() for s, x in zip(saved2, xs2))
