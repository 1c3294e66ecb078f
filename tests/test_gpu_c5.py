"""The three-level vortex workload at full size (512^2 base, 64^2 boxes on
1024^2 and 2048^2 around two seeded Lamb-Oseen vortices): composite
Helmholtz solves of both velocity components, the composite projection and
composite adjoint solves on the GPU, in the configuration the benchmark
times (mixed precision, red-black V(2,2), 1e-10).  The oracle's composite
solvers are too slow at this size, its composite operators are not: every
GPU result is checked by evaluating the oracle's operators on it."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import amr, amr_adj, proj  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd import workloads as W  # noqa: E402
from tests.gpuhelp import from_dev, to_dev  # noqa: E402

BASE = 512
BOXES, CENTRES = W.three_level_vortex_boxes(0)
K = 1.0 / BASE
C_HELM = 0.5 * 1e-3 * K
OPTS = dict(precision=A.MIXED, smoother=A.SMOOTH_RB, tol_rel=1e-10, max_cycles=100)


def gpu_hier(kind, op, c=0.0):
    H = A.Hierarchy(2, (BASE, BASE), 1.0 / BASE, 3)
    for l, bl in enumerate(BOXES):
        H.set_level_boxes(l, bl)
        if l:
            H.set_cf_mode(l, A.CF_INTERP)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
    H.set_operator(op, c)
    H.finalize()
    return H


def inputs(OH):
    """b_d per level: cell averages of the vortices' velocity + k g_d."""
    B = [[None] * 3 for _ in range(2)]
    for l, lev in enumerate(OH.levels):
        n = lev.shape
        u, v = W.lamb_oseen_avg(CENTRES, (0, 0), n, lev.h)
        for d, comp in enumerate((u, v)):
            a = lev.zeros()
            a[lev.inner] = comp + K * W.smooth_field_avg((0, 0), n, lev.h, seed=10 + d)
            B[d][l] = np.where(lev.mask, a, 0.0)
    return B


def vmax(H, arrs):
    return max(np.abs(arrs[l][H.valid[l]]).max() for l in range(H.nlev))


def test_three_level_vortex_workload():
    OH = amr.Hierarchy((BASE, BASE), 1.0 / BASE, BOXES, {(d, s): "D" for d in range(2) for s in (0, 1)})
    print("levels", [len(b) for b in BOXES], "valid cells", [int(v.sum()) for v in OH.valid], flush=True)
    Hh = gpu_hier("D", A.HELMHOLTZ, C_HELM)
    B = inputs(OH)
    Wd = []
    for d in range(2):
        bs = [to_dev(Hh, l, 0, B[d][l]) for l in range(3)]
        xs = [torch.zeros_like(b) for b in bs]
        st = Hh.solve_composite(xs, bs, None, A.default_opts(**OPTS))
        assert st["status"] == 0 and st["converged"], st
        Wd.append([from_dev(Hh, l, 0, xs[l], OH.levels[l]) for l in range(3)])
        R = amr.composite_residual(OH, OH.average_down_all(Wd[d]), B[d], "helmholtz", C_HELM)
        print("helmholtz", d, st["cycles"], vmax(OH, R) / vmax(OH, B[d]), flush=True)
        assert vmax(OH, R) <= 2e-10 * vmax(OH, B[d])
    # composite projection of w
    Hw, Hp = gpu_hier("D", A.POISSON), gpu_hier("N", A.POISSON)
    ws = [[to_dev(Hw, l, 0, Wd[d][l]) for d in range(2)] for l in range(3)]
    us = [[torch.zeros_like(ws[l][0]) for _ in range(2)] for l in range(3)]
    phis = [torch.zeros_like(ws[l][0]) for l in range(3)]
    st = A.project(Hw, Hp, ws, phis, us, None, A.default_opts(**OPTS))
    assert st["status"] == 0 and st["converged"], st
    Hw_o, Hp_o = proj.hierarchy_with(OH, "D"), proj.hierarchy_with(OH, "N")
    div = proj.composite_divergence(Hw_o, Wd, None)
    phi = [from_dev(Hp, l, 0, phis[l], OH.levels[l]) for l in range(3)]
    div_s, _ = Hp_o.solvability_shift(div, None)
    R = amr.composite_residual(Hp_o, Hp_o.average_down_all(phi), div_s, "poisson", 0.0)
    print("projection", st["cycles"], vmax(OH, R) / vmax(OH, div_s), flush=True)
    assert vmax(OH, R) <= 2e-10 * vmax(OH, div_s)
    G = proj.composite_gradient(Hp_o, phi)
    Wa = [Hw_o.average_down_all(Wd[d]) for d in range(2)]
    for d in range(2):
        got = [from_dev(Hw, l, 0, us[l][d], OH.levels[l]) for l in range(3)]
        want = [np.where(OH.levels[l].mask, Wa[d][l] - G[d][l], 0.0) for l in range(3)]
        want = OH.average_down_all(want)
        err = max(np.abs(got[l] - want[l])[OH.valid[l]].max() for l in range(3)) / vmax(OH, want)
        assert err < 1e-11, err
    # composite adjoint of the Helmholtz solve for J = 1/2 |w - t|^2
    rng = np.random.default_rng(20)
    for d in range(2):
        g = [np.where(OH.valid[l], Wd[d][l] - 0.1 * rng.normal(size=OH.levels[l].pshape), 0.0) for l in range(3)]
        gd = [to_dev(Hh, l, 0, g[l]) for l in range(3)]
        lam = [torch.zeros_like(x) for x in gd]
        st = Hh.solve_adjoint_composite(lam, gd, A.default_opts(**OPTS))
        assert st["status"] == 0 and st["converged"], st
        lo = [from_dev(Hh, l, 0, lam[l], OH.levels[l]) for l in range(3)]
        R = amr_adj.composite_residual_T(OH, lo, g, "helmholtz", C_HELM)
        print("adjoint", d, st["cycles"], vmax(OH, R) / vmax(OH, g), flush=True)
        assert vmax(OH, R) <= 2e-10 * vmax(OH, g)


def test_vortex_projection_adjoint_full_size():
    """The adjoint of the composite projection on the full three-level
    layout, checked by the oracle's operators: the adjoint potential lam
    satisfies the oracle's transposed composite Poisson system with the
    oracle's G^T ubar as source (projected along the volume weights), and
    wbar = ubar - D^T lam with the oracle's D^T applied to the GPU's lam."""
    from oracle import proj_adj
    OH = amr.Hierarchy((BASE, BASE), 1.0 / BASE, BOXES, {(d, s): "D" for d in range(2) for s in (0, 1)})
    Hw, Hp = gpu_hier("D", A.POISSON), gpu_hier("N", A.POISSON)
    Hw_o, Hp_o = proj.hierarchy_with(OH, "D"), proj.hierarchy_with(OH, "N")
    rng = np.random.default_rng(30)
    ub = [[np.where(OH.valid[l], rng.normal(size=OH.levels[l].pshape), 0.0) for l in range(3)] for _ in range(2)]
    ubs = [[to_dev(Hw, l, 0, ub[d][l]) for d in range(2)] for l in range(3)]
    lams = [torch.zeros_like(ubs[l][0]) for l in range(3)]
    wbs = [[torch.zeros_like(ubs[l][0]) for _ in range(2)] for l in range(3)]
    st = A.project_adjoint(Hw, Hp, ubs, lams, wbs, A.default_opts(**OPTS))
    assert st["status"] == 0 and st["converged"], st
    lam = [from_dev(Hp, l, 0, lams[l], OH.levels[l]) for l in range(3)]
    g = proj_adj.composite_gradient_T(Hp_o, ub)
    wts = [np.where(OH.valid[l], OH.levels[l].h ** 2, 0.0) for l in range(3)]
    tot = sum(g[l][OH.valid[l]].sum() for l in range(3))
    gp = [np.where(OH.valid[l], g[l] - wts[l] * tot / sum(w.sum() for w in wts), 0.0) for l in range(3)]
    R = amr_adj.composite_residual_T(Hp_o, lam, gp, "poisson", 0.0)
    print("projection adjoint", st["cycles"], vmax(OH, R) / vmax(OH, gp), flush=True)
    assert vmax(OH, R) <= 2e-10 * vmax(OH, gp)
    dt = proj_adj.composite_divergence_T(Hw_o, lam)
    for d in range(2):
        got = [from_dev(Hw, l, 0, wbs[l][d], OH.levels[l]) for l in range(3)]
        want = [np.where(OH.valid[l], ub[d][l] - dt[d][l], 0.0) for l in range(3)]
        err = max(np.abs(got[l] - want[l])[OH.valid[l]].max() for l in range(3)) / vmax(OH, want)
        assert err < 1e-11, err
