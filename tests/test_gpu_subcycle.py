"""Algorithm 1's schedule feeding the interface conditions (Section 6.2,
eq. timeInterp): for every level-1 advance of the schedule and every stage
time t* = t + c dt of the IMEX scheme, the coarse slices at t_coarse -
i k_coarse of a field cubic in time, interpolated by amg_cic_face_data at
the event's eta, give the face data (and its time derivative) of the field
at t* itself, to rounding: the schedule's slice bookkeeping and the time
interpolation agree, and t* always lies within the slices."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2506_02663_amd import amg as A  # noqa: E402
from tests.gpuhelp import to_dev  # noqa: E402
from oracle.level import Level  # noqa: E402

STAGES = (0.0, 0.5, 83 / 250, 31 / 50, 17 / 20, 1.0)


def P(t):  # cubic in time, and its derivative
    return 1.0 + 2.0 * t - t * t + 0.5 * t ** 3


def dP(t):
    return 2.0 - 2.0 * t + 1.5 * t * t


@pytest.mark.parametrize("ratio", [2, 4])
def test_schedule_times_feed_the_time_interpolation(ratio):
    base = (16, 16)
    fine_boxes = ([((0, 8), (15, 15)), ((16, 8), (23, 23)), ((8, 24), (15, 31))] if ratio == 2 else
                  [((0, 16), (31, 31)), ((32, 16), (47, 47)), ((16, 48), (31, 63))])
    H = A.Hierarchy(2, base, 1.0 / 16, 2, ratio=ratio)
    H.set_level_boxes(0, [((0, 0), (15, 15))])
    H.set_level_boxes(1, fine_boxes)
    H.set_cf_mode(1, A.CF_DIRICHLET)
    for d in range(2):
        for s in (0, 1):
            H.set_physical_bc(d, s, A.NEUMANN)
    H.set_operator(A.HELMHOLTZ, 1e-3)
    H.finalize()
    coarse = Level(base, 1.0 / 16, [((0, 0), (15, 15))], {(d, s): "N" for d in range(2) for s in (0, 1)})
    rng = np.random.default_rng(11)
    g = np.where(coarse.mask, rng.normal(size=coarse.pshape), 0.0)
    nface = H.level_info(1).nface

    def face(hist, k, eta):
        fd = torch.zeros(nface, dtype=torch.float64, device="cuda")
        dfd = torch.zeros(nface, dtype=torch.float64, device="cuda")
        H.cic_face_data(1, [to_dev(H, 0, 0, a) for a in hist], k, eta, fd, dfd, kind=A.CIC_VALUE)
        torch.cuda.synchronize()
        return fd.cpu().numpy(), dfd.cpu().numpy()

    events = A.subcycle_schedule(2, ratio, 0.0, 0.125, 2)
    fine = [e for e in events if e[0] == "advance" and e[1] == 1]
    assert len(fine) == 2 * ratio
    checked = 0
    for _, _, t, dt, kc, tc in fine:
        hist = [g * P(tc - i * kc) for i in range(4)]
        for c in STAGES:
            ts = t + c * dt
            eta = ts - (tc - kc)
            assert -1e-15 <= eta <= kc + 1e-15
            got, gotd = face(hist, kc, eta)
            # the field at t* itself: four equal slices interpolate to it exactly
            want, _ = face([g * P(ts)] * 4, kc, eta)
            wantd, _ = face([g * dP(ts)] * 4, kc, eta)
            scale = np.abs(want).max()
            assert np.abs(got - want).max() <= 1e-12 * scale
            assert np.abs(gotd - wantd).max() <= 1e-10 * max(1.0, np.abs(wantd).max())
            checked += 1
    assert checked == 2 * ratio * len(STAGES)
