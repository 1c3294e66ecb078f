"""Batched independent boxes (one level of isolated boxes of uneven sizes,
each its own domain): every multigrid step runs as one launch over all
boxes, boxes reach their coarsest depth at different depths.  Parity with
the oracle solving each box on its own."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import mg  # noqa: E402
from oracle.level import PAD, Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd import workloads as W  # noqa: E402

# sides 8m: coarsest sides 4 (16, 32), 6 (24, 48), 5 (40), 7 (56); one box
# of each size twice so that boxes share bottom inverses
SIDES = [16, 24, 40, 32, 48, 56, 24, 40]


def build(op, c, sides, bc="D"):
    h = 1.0 / 256
    H = A.Hierarchy(2, (256, 256), h, 1)
    boxes = []
    x = 0
    for s in sides:
        boxes.append(((x, 0), (x + s - 1, s - 1)))
        x += s + 8
    H.set_isolated(0)
    H.set_level_boxes(0, boxes)
    for d in range(2):
        for sd in (0, 1):
            H.set_physical_bc(d, sd, A.DIRICHLET if bc == "D" else A.NEUMANN)
    H.set_operator(A.HELMHOLTZ if op == "helmholtz" else A.POISSON, c)
    H.finalize()
    levs = [Level((s, s), h, [((0, 0), (s - 1, s - 1))], {(d, sd): bc for d in range(2) for sd in (0, 1)})
            for s in sides]
    return H, levs


def pack(H, arrs, dtype=torch.float64):
    return torch.tensor(H.pack(0, 0, lambda i, b: arrs[i]), dtype=dtype, device="cuda")


def unpack(H, t):
    return H.unpack(0, 0, t.detach().cpu().double().numpy())


@pytest.mark.parametrize("op,bc", [("helmholtz", "D"), ("poisson", "N"), ("poisson", "D")])
def test_batched_solve_matches_per_box_oracle(op, bc):
    c = 0.5e-3 / 256 * 40 if op == "helmholtz" else 0.0
    H, levs = build(op, c, SIDES, bc)
    info = H.level_info(0)
    assert info.nboxes == len(SIDES) and info.ncomp == len(SIDES)
    fs = [W.batched_rhs(s, 1.0 / 256, seed=i) for i, s in enumerate(SIDES)]
    fdev = pack(H, fs)
    for prec, tol in ((A.FP64, 1e-11), (A.MIXED, 1e-9)):
        x = torch.zeros_like(fdev)
        st = H.solve(0, x, fdev, None, A.default_opts(precision=prec, tol_rel=1e-12, max_cycles=200))
        assert st["status"] == 0 and st["converged"], st
        got = unpack(H, x)
        for i, lev in enumerate(levs):
            f = lev.zeros()
            f[lev.inner] = fs[i]
            want, sto = mg.solve(lev, f, op, c, tol_rel=1e-13, max_cycles=300)
            sing = lev.singular_components(op)
            g = lev.zeros()
            g[lev.inner] = got[i]
            g = lev.comp_mean(g, sing)
            want = lev.comp_mean(want, sing)
            err = np.abs(g - want)[lev.mask].max() / np.abs(want)[lev.mask].max()
            assert err < tol, (i, SIDES[i], prec, err)


def test_batched_vcycle_matches_per_box_oracle():
    """One V-cycle over boxes whose coarsest depths differ (0..3)."""
    op, c = "helmholtz", 0.3 / 256
    H, levs = build(op, c, SIDES)
    fs = [np.random.default_rng(i).normal(size=(s, s)) for i, s in enumerate(SIDES)]
    fdev = pack(H, fs)
    e = torch.zeros_like(fdev)
    H.vcycle(0, fdev, e)
    torch.cuda.synchronize()
    got = unpack(H, e)
    for i, lev in enumerate(levs):
        f = lev.zeros()
        f[lev.inner] = fs[i]
        want = mg.MG(lev, op, c).vcycle(f)
        err = np.abs(got[i] - want[lev.inner]).max() / np.abs(want[lev.inner]).max()
        assert err < 1e-11, (i, SIDES[i], err)
