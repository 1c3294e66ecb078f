"""The IMEX step of eq. GePUP-IMEX on a periodic level on the GPU (the
stage loop calling the solver as a black box) against the oracle:

* the convection operator eq. convOp element by element (2D, 3D, ragged
  sizes);
* one whole step against oracle.imex.imex_step, FP64 and mixed-precision
  solves, with and without forcing, 2D and 3D;
* at 256^2, a shear flow with time-dependent forcing against the closed
  form of the additive step on each Fourier mode (the pin of the oracle's
  loop, computed here from the tableau), and several steps of a
  four-vortex flow (Section 7.3's initial vorticity, velocity from the
  periodic stream function) staying finite with decaying energy;
* the error contract (non-periodic or tiled levels, bad arguments)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

from oracle import imex, proj  # noqa: E402
from oracle.level import Level  # noqa: E402
from paper_2506_02663_amd import amg as A  # noqa: E402
from paper_2506_02663_amd import workloads as W  # noqa: E402
from tests.gpuhelp import from_dev, relerr, to_dev  # noqa: E402

TWO_PI = 2 * np.pi


def plevel(shape):
    D = len(shape)
    return Level(shape, 1.0 / shape[0], [((0,) * D, tuple(n - 1 for n in shape))],
                 {(d, s): "P" for d in range(D) for s in (0, 1)})


def hiers(lev):
    D = lev.dim
    out = []
    for op in (A.HELMHOLTZ, A.POISSON):
        H = A.Hierarchy(D, lev.shape, lev.h, 1)
        H.set_level_boxes(0, lev.boxes)
        for d in range(D):
            for s in (0, 1):
                H.set_physical_bc(d, s, A.PERIODIC)
        H.set_operator(op, 1.0 if op == A.HELMHOLTZ else 0.0)
        H.finalize()
        out.append(H)
    return out


def smooth_field(lev, seed):
    rng = np.random.default_rng(seed)
    idx = np.indices(lev.shape)
    U = []
    for _ in range(lev.dim):
        a = lev.zeros()
        val = np.zeros(lev.shape)
        for _k in range(3):
            k = rng.integers(-2, 3, size=lev.dim)
            ph = sum(TWO_PI * k[d] * (idx[d] + 0.5) / lev.shape[d] for d in range(lev.dim))
            val += rng.normal() * np.cos(ph + rng.uniform(0, TWO_PI))
        a[lev.inner] = val
        U.append(a)
    return U


@pytest.mark.parametrize("shape", [(32, 32), (40, 24), (16, 16, 16), (12, 20, 8)])
def test_convection_against_oracle(shape):
    lev = plevel(shape)
    Hv, _ = hiers(lev)
    U = smooth_field(lev, 1)
    us = [to_dev(Hv, 0, 0, u) for u in U]
    outs = [torch.zeros_like(us[0]) for _ in U]
    A.convection(Hv, us, outs)
    torch.cuda.synchronize()
    want = imex.convection(lev, U)
    for d in range(lev.dim):
        assert relerr(from_dev(Hv, 0, 0, outs[d], lev), want[d], lev.mask) < 1e-12, d


def projected(lev, U):
    P, _, st = proj.project(lev, U, tol_rel=1e-13, smoother="rb")
    assert st["converged"]
    return P


@pytest.mark.parametrize("shape,forcing", [((32, 32), False), ((32, 32), True), ((16, 16, 16), False)])
def test_step_against_oracle(shape, forcing):
    lev = plevel(shape)
    Hv, Hp = hiers(lev)
    U0 = projected(lev, smooth_field(lev, 2))
    dt, nu = 0.4 * lev.h, 0.01
    g = None
    if forcing:
        rng = np.random.default_rng(3)
        base = smooth_field(lev, 4)
        g = [[np.where(lev.mask, base[d] * np.cos(5.0 * cj + d), 0.0) for d in range(lev.dim)] for cj in imex.C]
        assert rng is not None
    want = imex.imex_step(lev, U0, dt, nu, g=g, tol_rel=1e-12)
    for prec, tol in ((A.FP64, 1e-9), (A.MIXED, 1e-8)):
        us = [to_dev(Hv, 0, 0, u) for u in U0]
        gs = None if g is None else [[to_dev(Hv, 0, 0, a) for a in per] for per in g]
        st = A.imex_step(Hv, Hp, dt, nu, us, gs, A.default_opts(precision=prec, smoother=A.SMOOTH_RB,
                                                                  tol_rel=1e-12, max_cycles=100))
        torch.cuda.synchronize()
        assert st["status"] == 0 and st["converged"], st
        assert st["solves"] == 6 + 5 * lev.dim + 6
        for d in range(lev.dim):
            assert relerr(from_dev(Hv, 0, 0, us[d], lev), want[d], lev.mask) < tol, (prec, d)


def additive_step(z, y0, gs, dt):
    AI, AE, b = np.array(imex.AI), np.array(imex.AE), np.array(imex.B)
    gs = np.asarray(gs, dtype=float)
    Y = np.linalg.solve(np.eye(6) - z * AI, y0 * np.ones(6) + dt * (AE @ gs))
    return Y[5] + dt * (b - AE[5]) @ gs


@pytest.mark.parametrize("prec,tol", [(A.FP64, 1e-11), (A.MIXED, 1e-9)])
def test_shear_flow_at_256_is_the_closed_form(prec, tol):
    n, nu, dt, t0 = 256, 1e-3, 0.5 / 256, 0.1
    lev = plevel((n, n))
    Hv, Hp = hiers(lev)
    y = (np.arange(n) + 0.5) / n
    modes = [(1, 0.9), (7, -0.4), (40, 0.05)]
    prof = sum(a * np.cos(TWO_PI * k * y) for k, a in modes)
    u0 = lev.zeros()
    u0[lev.inner] = np.broadcast_to(prof[None, :], (n, n))
    gk, omega = 3, 2.0 / dt
    amp = [np.cos(omega * (t0 + cj * dt)) for cj in imex.C]
    us = [to_dev(Hv, 0, 0, u0), to_dev(Hv, 0, 0, lev.zeros())]
    gs = []
    for j in range(6):
        ga = lev.zeros()
        ga[lev.inner] = np.broadcast_to(amp[j] * np.cos(TWO_PI * gk * y)[None, :], (n, n))
        gs.append([to_dev(Hv, 0, 0, ga), to_dev(Hv, 0, 0, lev.zeros())])
    st = A.imex_step(Hv, Hp, dt, nu, us, gs, A.default_opts(precision=prec, smoother=A.SMOOTH_RB, tol_rel=1e-12,
                                                              max_cycles=100))
    torch.cuda.synchronize()
    assert st["status"] == 0 and st["converged"], st
    lam = lambda k: (32 * np.cos(TWO_PI * k / n) - 2 * np.cos(2 * TWO_PI * k / n) - 30) * n * n / 12
    want = sum(additive_step(nu * lam(k) * dt, a, [0.0] * 6, dt) * np.cos(TWO_PI * k * y) for k, a in modes)
    want = want + additive_step(nu * lam(gk) * dt, 0.0, amp, dt) * np.cos(TWO_PI * gk * y)
    got = from_dev(Hv, 0, 0, us[0], lev)[lev.inner]
    assert np.abs(got - want[None, :]).max() < tol * np.abs(want).max()
    assert np.abs(from_dev(Hv, 0, 0, us[1], lev)[lev.inner]).max() < tol


def test_four_vortex_steps_at_256():
    n = 256
    lev = plevel((n, n))
    Hv, Hp = hiers(lev)
    u, v = W.four_vortex_velocity(n)
    U = [lev.zeros(), lev.zeros()]
    U[0][lev.inner], U[1][lev.inner] = u, v
    us = [to_dev(Hv, 0, 0, a) for a in U]
    dt = 0.5 * lev.h / max(np.abs(u).max(), np.abs(v).max())
    energies = [sum(float((t * t).sum()) for t in us)]
    for _ in range(3):
        st = A.imex_step(Hv, Hp, dt, 1e-3, us, None, A.default_opts(smoother=A.SMOOTH_RB, tol_rel=1e-10,
                                                                    max_cycles=100))
        assert st["status"] == 0 and st["converged"], st
        energies.append(sum(float((t * t).sum()) for t in us))
    assert all(np.isfinite(energies))
    assert energies[-1] < energies[0] and energies[-1] > 0.9 * energies[0]


def test_error_contract():
    lev = plevel((32, 32))
    Hv, Hp = hiers(lev)
    us = [to_dev(Hv, 0, 0, lev.zeros()) for _ in range(2)]
    with pytest.raises(A.AmgError) as e:
        A.imex_step(Hv, Hp, -1.0, 0.01, us)
    assert e.value.code == A.EINVAL
    with pytest.raises(A.AmgError) as e:
        A.imex_step(Hp, Hv, 0.01, 0.01, us)  # operators swapped
    assert e.value.code == A.EINVAL
    tiled = Level((32, 32), 1 / 32, [((0, 0), (15, 31)), ((16, 0), (31, 31))],
                  {(d, s): "P" for d in range(2) for s in (0, 1)})
    Ht = A.Hierarchy(2, (32, 32), 1 / 32, 1)
    Ht.set_level_boxes(0, tiled.boxes)
    for d in range(2):
        for s in (0, 1):
            Ht.set_physical_bc(d, s, A.PERIODIC)
    Ht.set_operator(A.HELMHOLTZ, 1.0)
    Ht.finalize()
    ut = [to_dev(Ht, 0, 0, tiled.zeros()) for _ in range(2)]
    with pytest.raises(A.AmgError) as e:
        A.convection(Ht, ut, [torch.zeros_like(ut[0]) for _ in range(2)])
    assert e.value.code == A.EUNSUPPORTED
