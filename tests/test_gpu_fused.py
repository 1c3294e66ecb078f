"""The fused red-black sweep (both colours of an FP32 red-black sweep in one
launch, 3D) against the two half-sweep launches it replaces, on depths where
it applies: single boxes with Dirichlet, Neumann and mixed conditions, boxes
wider than one tile row, uneven tile counts, batches of isolated boxes, and
the 256^3 benchmark depth; and which depths take it (4-plane tiles, rows of
128 m or 128 m + (>= 4) cells, whole 4-row tiles, uniformly filled faces).
The fused form is opt-in (AMG_TUNE_FUSED_RB = 1); the two forms compute the
same expressions from the same values and agree to the last bits the
compiler's instruction selection may change."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2506_02663_amd import amg as A  # noqa: E402

MIXED3 = {(0, 0): "D", (0, 1): "N", (1, 0): "N", (1, 1): "D", (2, 0): "D", (2, 1): "N"}


def build(shape, boxes, bc, fused, isolated=False, op="helmholtz"):
    n = max(shape)
    H = A.Hierarchy(3, shape, 1.0 / n, 1)
    if isolated:
        H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    for d in range(3):
        for s in (0, 1):
            kind = bc[(d, s)] if isinstance(bc, dict) else bc
            H.set_physical_bc(d, s, A.DIRICHLET if kind == "D" else A.NEUMANN)
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, 0.3 / n)
    H.set_tuning(A.TUNE_FUSED_RB, 1 if fused else 0)
    H.finalize()
    return H


CASES = {
    # name: (grid, boxes, bc, isolated, fused bits expected at depths 0, 1)
    "cube16_D": ((16, 16, 16), [((0, 0, 0), (15, 15, 15))], "D", False, (1, 1)),
    "cube32_N": ((32, 32, 32), [((0, 0, 0), (31, 31, 31))], "N", False, (1, 1)),
    "mixed_24x16x20": ((24, 16, 20), [((0, 0, 0), (23, 15, 19))], MIXED3, False, (1, 0)),  # 12x8x10: a 2-plane tile
    "wide_136x8x12": ((136, 8, 12), [((0, 0, 0), (135, 7, 11))], "D", False, (1, 0)),     # 68x4x6: 4 rows -> 2
    "wide_130_off": ((130, 8, 8), [((0, 0, 0), (129, 7, 7))], "D", False, (0, 0)),         # last x-tile 2 wide
    "isolated": ((64, 64, 64), [((0, 0, 0), (15, 15, 15)), ((32, 0, 0), (55, 23, 31))], "N", True, (1, 1)),
}


def rand_dev(H, depth, seed, dtype=torch.float32):
    n, _ = H.depth_size(0, depth)
    g = torch.Generator(device="cpu").manual_seed(seed)
    return torch.randn(n, generator=g, dtype=torch.float64).to(dtype).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_fused_sweeps_match_half_sweeps(name):
    shape, boxes, bc, iso, bits = CASES[name]
    Hf = build(shape, boxes, bc, True, iso)
    Hs = build(shape, boxes, bc, False, iso)
    info = Hf.level_info(0)
    got_bits = tuple((info.fused_rb >> k) & 1 for k in range(2))
    assert got_bits == bits, (name, info.fused_rb)
    assert Hs.level_info(0).fused_rb == 0
    for depth in range(min(2, info.depths - 1)):
        u0, f = rand_dev(Hf, depth, 1), rand_dev(Hf, depth, 2)
        outs = []
        for H in (Hf, Hs):
            u, t = u0.clone(), torch.zeros_like(u0)
            H.smooth(0, depth, u, f, t, A.SMOOTH_RB, 3)
            torch.cuda.synchronize()
            outs.append(H.unpack(0, depth, u.double().cpu().numpy()))
        for a, b in zip(*outs):
            scale = np.abs(b).max()
            assert np.abs(a - b).max() <= 2e-6 * scale, (name, depth, np.abs(a - b).max() / scale)


def test_fused_benchmark_depth_256():
    n = 256
    box = [((0, 0, 0), (n - 1,) * 3)]
    Hf = build((n,) * 3, box, "N", True, op="poisson")
    Hs = build((n,) * 3, box, "N", False, op="poisson")
    assert Hf.level_info(0).fused_rb & 3 == 3
    u0, f = rand_dev(Hf, 0, 3), rand_dev(Hf, 0, 4)
    res = []
    for H in (Hf, Hs):
        u, t = u0.clone(), torch.zeros_like(u0)
        H.smooth(0, 0, u, f, t, A.SMOOTH_RB, 2)
        torch.cuda.synchronize()
        res.append(H.unpack(0, 0, u.double().cpu().numpy())[0])
    scale = np.abs(res[1]).max()
    assert np.abs(res[0] - res[1]).max() <= 2e-6 * scale


@pytest.mark.parametrize("name", ["cube32_N", "isolated", "mixed_24x16x20"])
def test_fused_mixed_solves_match(name):
    shape, boxes, bc, iso, _ = CASES[name]
    sols = []
    for fused in (True, False):
        H = build(shape, boxes, bc, fused, iso, op="poisson" if bc == "N" else "helmholtz")
        f = rand_dev(H, 0, 5, torch.float64)
        x = torch.zeros_like(f)
        st = H.solve(0, x, f, None, A.default_opts(precision=A.MIXED, smoother=A.SMOOTH_RB, tol_rel=1e-10,
                                                       max_cycles=100, nu1=1, nu2=3))
        assert st["converged"], st
        sols.append((st["cycles"], H.unpack(0, 0, x.cpu().numpy())))
    assert abs(sols[0][0] - sols[1][0]) <= 1
    for a, b in zip(sols[0][1], sols[1][1]):
        assert np.abs(a - b).max() <= 1e-8 * np.abs(b).max()
