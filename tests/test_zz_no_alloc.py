"""The allocation-free dot product (amg_dot_noalloc, per-tile partials in a
static device array) against amg_dot (the same kernels on the level's own
partial buffer): bitwise equal on two calls in a row, the second on a
smaller level (fewer tiles, so stale partials of the first call sit past
its range), in 3D and 2D; a graph that captures the call replays it to the
same value; a level with more tiles than the static array holds is
rejected."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import make_hier, random_field, to_dev, unit_level  # noqa: E402


def _pair(lev, seed):
    H, L = make_hier(lev, "helmholtz", 1e-3)
    a = to_dev(H, L, 0, random_field(lev, seed))
    b = to_dev(H, L, 0, random_field(lev, seed + 1))
    return H, L, a, b


def test_matches_dot_on_two_calls_second_smaller():
    big = _pair(unit_level(64, 3, "D"), 1)
    small = _pair(unit_level(32, 2, "N"), 3)
    assert big[0].depth_size(0, 0)[0] > small[0].depth_size(0, 0)[0]
    out = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for k, (H, L, a, b) in enumerate((big, small)):
        H.dot_noalloc(L, a, b, out[k:k + 1])
        torch.cuda.synchronize()
        want = H.dot(L, a, b)
        got = out[k].item()
        assert got == want, (k, got, want)
        assert np.isfinite(got) and got != 0.0
    # and once more on the big level after the small one
    H, L, a, b = big
    H.dot_noalloc(L, a, b, out[1:2])
    torch.cuda.synchronize()
    assert out[1].item() == out[0].item()


def test_captured_in_a_graph():
    H, L, a, b = _pair(unit_level(48, 2, "D"), 5)
    want = H.dot(L, a, b)
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        H.dot_noalloc(L, a, b, out)  # warm-up outside the capture
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        H.dot_noalloc(L, a, b, out)
    for _ in range(3):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert out.item() == want
        _ = (a * 2).sum().item()  # unrelated eager work between replays


def test_rejects_a_level_beyond_the_static_scratch():
    # 4200 isolated 16^2 boxes marched two rows at a time: 33600 tiles
    H = A.Hierarchy(2, (256, 256), 1.0 / 256, 1)
    H.set_isolated(0)
    H.set_level_boxes(0, [((0, 0), (15, 15))] * 4200)
    H.set_operator(A.HELMHOLTZ, 1e-3)
    H.set_tuning(A.TUNE_MARCH2, 2)
    H.finalize()
    n, _ = H.depth_size(0, 0)
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(A.AmgError) as e:
        H.dot_noalloc(0, a, a, out)
    assert e.value.code == A.EUNSUPPORTED and "static scratch" in str(e.value)
    assert H.dot(0, a, a) == 4200 * 256
