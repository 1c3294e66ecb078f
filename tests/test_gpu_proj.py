"""Gradient, divergence and the approximate projection on the GPU against
the oracle: element by element on single levels (physical, coarse-fine and
box-to-box ghosts, 2D and 3D) and in composite form over two- and
three-level hierarchies (AMRCFI ghosts, refluxed divergence, average-down),
and whole projections in FP64 and mixed precision."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import amr, proj  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import (cf_level, faces_to_dev, from_dev, gap_level, make_hier, random_faces,  # noqa: E402
                           random_field, relerr, tiled_level, to_dev, unit_level)

TOL64 = 1e-11

LAYOUTS = {
    "2d": lambda k: unit_level(32, 2, k),
    "2d_ragged": lambda k: Level((40, 24), 1 / 40, [((0, 0), (39, 23))], {(d, s): k for d in range(2) for s in (0, 1)}),
    "2d_tiled": lambda k: tiled_level(32, 2, k),
    "2d_cf": lambda k: cf_level(k, k),
    "2d_gap": lambda k: Level(gap_level().shape, gap_level().h, gap_level().boxes,
                              {(d, s): k for d in range(2) for s in (0, 1)}, k),
    "3d": lambda k: unit_level(16, 3, k),
    "3d_tiled": lambda k: tiled_level(16, 3, k),
}


@pytest.mark.parametrize("name", list(LAYOUTS))
@pytest.mark.parametrize("kind", ["N", "D"])
def test_level_gradient(name, kind):
    lev = LAYOUTS[name](kind)
    H, L = make_hier(lev, "poisson", 0.0)
    phi = random_field(lev, 1)
    fd = random_faces(lev, 2)
    ph = to_dev(H, L, 0, phi)
    gs = [torch.zeros_like(ph) for _ in range(lev.dim)]
    H.gradient([ph], [gs], [faces_to_dev(H, L, lev, fd)], lev_lo=L)
    torch.cuda.synchronize()
    want = proj.gradient(lev, phi, fd)
    for d in range(lev.dim):
        assert relerr(from_dev(H, L, 0, gs[d], lev), want[d], lev.mask) < TOL64


@pytest.mark.parametrize("name", list(LAYOUTS))
def test_level_divergence(name):
    lev = LAYOUTS[name]("D")
    H, L = make_hier(lev, "poisson", 0.0)
    W = [random_field(lev, 3 + d) for d in range(lev.dim)]
    wb = [random_faces(lev, 7 + d) for d in range(lev.dim)]
    ws = [to_dev(H, L, 0, w) for w in W]
    out = torch.zeros_like(ws[0])
    H.divergence([ws], [out], [[faces_to_dev(H, L, lev, f) for f in wb]], lev_lo=L)
    torch.cuda.synchronize()
    assert relerr(from_dev(H, L, 0, out, lev), proj.divergence(lev, W, wb), lev.mask) < TOL64


COMPOSITE = {
    "two_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((8, 8), (15, 23)), ((16, 8), (23, 15))]]),
    "three_level": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((4, 4), (27, 27))], [((16, 16), (31, 31))]]),
    "corner": ((16, 8), 1 / 16, [[((0, 0), (15, 7))], [((0, 0), (7, 7))]]),
    "boundary": ((32, 16), 1 / 32, [[((0, 0), (15, 15)), ((16, 0), (31, 15))],
                                   [((0, 0), (15, 15)), ((16, 0), (23, 11))]]),
    "two_level_r4": ((16, 16), 1 / 16, [[((0, 0), (15, 15))], [((16, 16), (39, 47)), ((40, 16), (47, 31))]], 4),
}


def gpu_hier(base, h0, boxes, kind, ratio=2):
    H = A.Hierarchy(2, base, h0, len(boxes), ratio=ratio)
    for l, bl in enumerate(boxes):
        H.set_level_boxes(l, bl)
        if l:
            H.set_cf_mode(l, A.CF_INTERP)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
    H.set_operator(A.POISSON, 0.0)
    H.finalize()
    return H


def rand_levels(OH, seed):
    rng = np.random.default_rng(seed)
    out = []
    for lev in OH.levels:
        u = lev.zeros()
        u[lev.mask] = rng.normal(size=lev.ncells)
        out.append(u)
    return out


def rand_faces(OH, seed):
    rng = np.random.default_rng(seed)
    out = []
    for lev in OH.levels:
        fd = lev.zero_face_data()
        for k in fd:
            e = lev.end_is_physical(*k)
            fd[k][e] = rng.normal(size=int(e.sum()))
        out.append(fd)
    return out


def relmax(G, O, masks):
    num = max(np.abs(G[l] - O[l])[masks[l]].max() for l in range(len(G)))
    den = max(np.abs(O[l])[masks[l]].max() for l in range(len(G)))
    return num / den


@pytest.mark.parametrize("name", list(COMPOSITE))
def test_composite_gradient_and_divergence(name):
    base, h0, boxes, *rest = COMPOSITE[name]
    ratio = rest[0] if rest else 2
    Hp_o = amr.Hierarchy(base, h0, boxes, {(d, s): "N" for d in range(2) for s in (0, 1)}, ratio=ratio)
    Hw_o = amr.Hierarchy(base, h0, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)}, ratio=ratio)
    Hp, Hw = gpu_hier(base, h0, boxes, "N", ratio), gpu_hier(base, h0, boxes, "D", ratio)
    nl = len(boxes)
    phi = rand_levels(Hp_o, 1)
    ph = [to_dev(Hp, l, 0, phi[l]) for l in range(nl)]
    gs = [[torch.zeros_like(ph[l]) for _ in range(2)] for l in range(nl)]
    Hp.gradient(ph, gs)
    want = proj.composite_gradient(Hp_o, phi)
    for d in range(2):
        got = [from_dev(Hp, l, 0, gs[l][d], Hp_o.levels[l]) for l in range(nl)]
        assert relmax(got, want[d], [lev.mask for lev in Hp_o.levels]) < TOL64
    W = [rand_levels(Hw_o, 2 + d) for d in range(2)]
    wb = [rand_faces(Hw_o, 5 + d) for d in range(2)]
    ws = [[to_dev(Hw, l, 0, W[d][l]) for d in range(2)] for l in range(nl)]
    wbs = [[faces_to_dev(Hw, l, Hw_o.levels[l], wb[d][l]) for d in range(2)] for l in range(nl)]
    out = [torch.zeros_like(ws[l][0]) for l in range(nl)]
    Hw.divergence(ws, out, wbs)
    want = proj.composite_divergence(Hw_o, W, wb)
    got = [from_dev(Hw, l, 0, out[l], Hw_o.levels[l]) for l in range(nl)]
    assert relmax(got, want, [lev.mask for lev in Hw_o.levels]) < TOL64


@pytest.mark.parametrize("name", ["2d", "3d", "2d_ragged"])
def test_level_projection(name):
    lev = LAYOUTS[name]("D")
    lw, lp = proj.velocity_level(lev), proj.pressure_level(lev)
    Hw, L = make_hier(lw, "poisson", 0.0)
    Hp, _ = make_hier(lp, "poisson", 0.0)
    W = [random_field(lev, 11 + d) for d in range(lev.dim)]
    wb = [random_faces(lw, 21 + d) for d in range(lev.dim)]
    U_o, phi_o, st_o = proj.project(lev, W, wb, tol_rel=1e-12, smoother="rb")
    for prec, tol in ((A.FP64, TOL64), (A.MIXED, 1e-9)):
        ws = [to_dev(Hw, L, 0, w) for w in W]
        us = [torch.zeros_like(ws[0]) for _ in W]
        phi = torch.zeros_like(ws[0])
        st = A.project(Hw, Hp, [ws], [phi], [us], [[faces_to_dev(Hw, L, lw, f) for f in wb]],
                       A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        for d in range(lev.dim):
            assert relerr(from_dev(Hw, L, 0, us[d], lev), U_o[d], lev.mask) < tol, (prec, d)
        assert relerr(from_dev(Hp, L, 0, phi, lev), phi_o, lev.mask) < tol


@pytest.mark.parametrize("name", ["two_level", "three_level", "two_level_r4"])
def test_composite_projection(name):
    base, h0, boxes, *rest = COMPOSITE[name]
    ratio = rest[0] if rest else 2
    H_o = amr.Hierarchy(base, h0, boxes, {(d, s): "D" for d in range(2) for s in (0, 1)}, ratio=ratio)
    Hw_o = proj.hierarchy_with(H_o, "D")
    Hp, Hw = gpu_hier(base, h0, boxes, "N", ratio), gpu_hier(base, h0, boxes, "D", ratio)
    nl = len(boxes)
    W = [rand_levels(Hw_o, 31 + d) for d in range(2)]
    wb = [rand_faces(Hw_o, 41 + d) for d in range(2)]
    U_o, Phi_o, st_o = proj.composite_project(H_o, W, wb, tol_rel=1e-12, smoother="rb")
    assert st_o["converged"]
    for prec, tol in ((A.FP64, 1e-10), (A.MIXED, 1e-9)):
        ws = [[to_dev(Hw, l, 0, W[d][l]) for d in range(2)] for l in range(nl)]
        wbs = [[faces_to_dev(Hw, l, Hw_o.levels[l], wb[d][l]) for d in range(2)] for l in range(nl)]
        us = [[torch.zeros_like(ws[l][0]) for _ in range(2)] for l in range(nl)]
        phis = [torch.zeros_like(ws[l][0]) for l in range(nl)]
        st = A.project(Hw, Hp, ws, phis, us, wbs,
                       A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        for d in range(2):
            got = [from_dev(Hw, l, 0, us[l][d], Hw_o.levels[l]) for l in range(nl)]
            assert relmax(got, U_o[d], H_o.valid) < tol, (prec, d)
