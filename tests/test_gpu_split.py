"""Colour-split storage of the finest depth's red-black post-smoothing in
mixed-precision 3D solves (each colour in its own half array, so a
half-sweep streams only the cells it reads and writes): which depths take
it (3D, every face filled uniformly with both ghost layers from its row, even
sizes), solves with it against the same solves in interleaved storage
(AMG_TUNE_SPLIT_RB = 0) on single boxes with Dirichlet, Neumann and mixed
conditions, rows wider than one tile, a last x-tile two cells wide, batches
of isolated boxes and both relaxation factors; graph replays against direct
launches; a split solve against the oracle's discrete system; and the timing
entry point on a split depth.  Both storages evaluate the same expressions
on the same values."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd import workloads as W  # noqa: E402

MIXED3 = {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D", (2, 0): "D", (2, 1): "N"}


def build(shape, boxes, bc, split, isolated=False, op="helmholtz", c=None):
    n = max(shape)
    dim = len(shape)
    H = A.Hierarchy(dim, shape, 1.0 / n, 1)
    if isolated:
        H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    for d in range(dim):
        for s in (0, 1):
            kind = bc[(d, s)] if isinstance(bc, dict) else bc
            H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, 0.3 / n if c is None else c)
    H.set_tuning(A.TUNE_SPLIT_RB, 1 if split else 0)
    H.finalize()
    return H


CASES = {
    # name: (grid, boxes, bc, isolated)
    "cube16_D": ((16, 16, 16), [((0, 0, 0), (15, 15, 15))], "D", False),
    "cube32_N": ((32, 32, 32), [((0, 0, 0), (31, 31, 31))], "N", False),
    "mixed_24x16x20": ((24, 16, 20), [((0, 0, 0), (23, 15, 19))], MIXED3, False),
    "wide_136x8x12": ((136, 8, 12), [((0, 0, 0), (135, 7, 11))], "D", False),
    "wide_130x8x8": ((130, 8, 8), [((0, 0, 0), (129, 7, 7))], "N", False),  # last x-tile 2 wide
    "rows_264x16x16": ((264, 16, 16), [((0, 0, 0), (263, 15, 15))], MIXED3, False),
    "isolated": ((64, 64, 64), [((0, 0, 0), (15, 15, 15)), ((32, 0, 0), (55, 23, 31))], "N", True),
    # 2D: one wavefront per tile, marched along y
    "sq2d_64_D": ((64, 64), [((0, 0), (63, 63))], "D", False),
    "rect2d_96x64_N": ((96, 64), [((0, 0), (95, 63))], "N", False),
    "mixed2d_136x40": ((136, 40), [((0, 0), (135, 39))], MIXED3, False),
    "wide2d_130x16": ((130, 16), [((0, 0), (129, 15))], "D", False),  # last x-tile 2 wide
    "iso2d": ((512, 64), [((0, 0), (15, 23)), ((32, 0), (63, 31)), ((96, 0), (231, 47)), ((256, 0), (511, 63))],
              "D", True),
}


def rand_dev(H, seed, dtype=torch.float64):
    n, _ = H.depth_size(0, 0)
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(n, generator=g, dtype=torch.float64).to(dtype).cuda()


def opts(omega_rb=1.0, graph=1, nu1=1, nu2=3):
    return A.default_opts(precision=A.MIXED, smoother=A.SMOOTH_RB, tol_rel=1e-10, max_cycles=100, nu1=nu1, nu2=nu2,
                          omega_rb=omega_rb, use_graph=graph)


@pytest.mark.parametrize("name", list(CASES))
def test_split_layout_bits(name):
    shape, boxes, bc, iso = CASES[name]
    assert build(shape, boxes, bc, True, iso).level_info(0).split_rb == 1
    assert build(shape, boxes, bc, False, iso).level_info(0).split_rb == 0


def test_split_not_taken_on_interpolated_faces():
    # a refined patch: its faces inside the domain are coarse-fine faces,
    # filled from their own rows in the Dirichlet and Neumann modes (like
    # physical faces) and interpolated from the coarse level in the other
    for mode, want in ((A.CF_DIRICHLET, 1), (A.CF_NEUMANN, 1), (A.CF_INTERP, 0)):
        H = A.Hierarchy(3, (16, 16, 16), 1.0 / 16, 2)
        H.set_level_boxes(0, [((0, 0, 0), (15, 15, 15))])
        H.set_level_boxes(1, [((8, 8, 8), (23, 23, 23))])
        H.set_cf_mode(1, mode)
        H.set_operator(A.POISSON, 0.0)
        H.finalize()
        assert H.level_info(0).split_rb == 1
        assert H.level_info(1).split_rb == want, mode


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("op,omega_rb", [("helmholtz", 1.0), ("poisson", 1.3)])
def test_split_solves_match_interleaved(name, op, omega_rb):
    shape, boxes, bc, iso = CASES[name]
    if op == "poisson" and bc == "D":
        bc = "N"
    res = []
    for split in (True, False):
        H = build(shape, boxes, bc, split, iso, op=op)
        f = rand_dev(H, 5)
        x = torch.zeros_like(f)
        st = H.solve(0, x, f, None, opts(omega_rb))
        torch.cuda.synchronize()
        assert st["converged"], (name, split, st)
        res.append((st["cycles"], st["history"], H.unpack(0, 0, x.cpu().numpy())))
    assert res[0][0] == res[1][0], (name, res[0][0], res[1][0])
    for a, b in zip(res[0][1], res[1][1]):
        assert abs(a - b) <= 1e-5 * max(abs(b), 1e-300), (name, res[0][1], res[1][1])
    for a, b in zip(res[0][2], res[1][2]):
        assert np.abs(a - b).max() <= 1e-9 * np.abs(b).max(), (name, np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("nu1,nu2", [(1, 1), (2, 2), (1, 4), (0, 2), (3, 1)])
def test_split_cycle_shapes(nu1, nu2):
    shape, boxes, bc, iso = CASES["mixed_24x16x20"]
    res = []
    for split in (True, False):
        H = build(shape, boxes, bc, split, iso)
        f = rand_dev(H, 6)
        x = torch.zeros_like(f)
        st = H.solve(0, x, f, None, opts(nu1=nu1, nu2=nu2))
        torch.cuda.synchronize()
        assert st["converged"], st
        res.append((st["cycles"], H.unpack(0, 0, x.cpu().numpy())[0]))
    assert res[0][0] == res[1][0]
    assert np.abs(res[0][1] - res[1][1]).max() <= 1e-9 * np.abs(res[1][1]).max()


def test_split_not_taken_with_a_box_solved_at_depth_0():
    # an isolated 4^3 box cannot be halved: it is solved exactly at depth 0,
    # next to a box that is smoothed there
    boxes = [((0, 0, 0), (15, 15, 15)), ((24, 0, 0), (27, 3, 3))]
    res = []
    for split in (True, False):
        H = build((32, 32, 32), boxes, "D", split, True)
        assert H.level_info(0).split_rb == 0
        f = rand_dev(H, 8)
        x = torch.zeros_like(f)
        st = H.solve(0, x, f, None, opts())
        torch.cuda.synchronize()
        assert st["converged"], st
        res.append(x.cpu().numpy())
    assert np.array_equal(res[0], res[1])


def test_split_graph_replays_match_direct_launches_bitwise():
    shape, boxes, bc, iso = CASES["rows_264x16x16"]
    H = build(shape, boxes, bc, True, iso, op="poisson")
    f = rand_dev(H, 7)
    out = []
    for graph in (0, 1, 1, 0):
        x = torch.zeros_like(f)
        st = H.solve(0, x, f, None, opts(1.3, graph=graph))
        torch.cuda.synchronize()
        assert st["converged"] and st["graph"] == bool(graph)
        out.append((x.cpu().numpy().copy(), st["history"]))
        _ = (f * 2).sum().item()  # unrelated eager work between solves
    for x, hist in out[1:]:
        assert np.array_equal(x, out[0][0])
        assert hist == out[0][1]


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("poisson", "N")])
def test_split_solution_satisfies_oracle_system(op, bc):
    n = 32
    h = 1.0 / n
    c = 0.5e-4 * h if op == "helmholtz" else 0.0
    shape = (n,) * 3
    if op == "helmholtz":
        f = (1.0 + 12 * math.pi ** 2 * c) * W.sinprod_avg(shape, h) + W.noise(shape, 0)
    else:
        f = -12 * math.pi ** 2 * W.cosprod_avg(shape, h) + W.noise(shape, 1)
        f -= f.mean()
    H = build(shape, [((0,) * 3, (n - 1,) * 3)], bc, True, op=op, c=c)
    assert H.level_info(0).split_rb == 1
    fd = torch.tensor(H.pack(0, 0, lambda i, b: f), device="cuda")
    x = torch.zeros_like(fd)
    st = H.solve(0, x, fd, None, opts(1.3 if op == "poisson" else 1.0))
    assert st["status"] == 0 and st["converged"], st
    lev = Level(shape, h, [((0,) * 3, (n - 1,) * 3)], {(d, s): bc for d in range(3) for s in (0, 1)})
    xs = lev.zeros()
    xs[lev.inner] = H.unpack(0, 0, x.cpu().numpy())[0]
    fo = lev.zeros()
    fo[lev.inner] = f
    sing = lev.singular_components(op)
    if sing:
        fo, _ = mg.solvability_shift(lev, fo, None, sing)
    r = fo - lev.apply(xs, op, c)
    r0 = np.abs(fo[lev.mask]).max()
    assert np.abs(r[lev.mask]).max() <= 2e-10 * r0, (np.abs(r[lev.mask]).max() / r0, st["cycles"])


def test_time_sweep_on_split_depth():
    shape, boxes, bc, iso = CASES["cube32_N"]
    H = build(shape, boxes, bc, True, iso, op="poisson")
    n, _ = H.depth_size(0, 0)
    u = torch.zeros(n, dtype=torch.float32, device="cuda")
    f = torch.zeros_like(u)
    t = torch.zeros_like(u)
    ms = H.time_sweep(0, u, f, t, A.SMOOTH_RB, 8)
    assert ms > 0
    assert torch.isfinite(u).all() and torch.isfinite(t).all()


@pytest.mark.parametrize("shape", [(32, 32, 32), (64, 48)])
def test_split_poisson_keeps_outer_mean_shift(shape):
    """A right-hand side with a large mean: the split kernels subtract the
    outer residual's per-component mean as they read it, through the whole
    V-cycle (the coarse depths' own mean removals must not replace it).  The
    two storages evaluate the same expressions in the same order, so the
    solves agree bitwise (the shift of a coarse depth in its place changed
    the solution by a few 1e-12)."""
    box = [((0,) * len(shape), tuple(n - 1 for n in shape))]
    res = []
    for split in (True, False):
        H = build(shape, box, "N", split, op="poisson")
        assert H.level_info(0).split_rb == int(split)
        f = rand_dev(H, 9) + 5.0
        x = torch.zeros_like(f)
        st = H.solve(0, x, f, None, opts(1.3))
        torch.cuda.synchronize()
        assert st["converged"], st
        res.append((st["cycles"], H.unpack(0, 0, x.cpu().numpy())[0]))
    assert res[0][0] == res[1][0]
    assert np.array_equal(res[0][1], res[1][1]), np.abs(res[0][1] - res[1][1]).max() / np.abs(res[1][1]).max()
