"""Algorithm 1's time schedule (Section 6.2; amg_subcycle_schedule) against
the oracle's recursion in exact rational arithmetic: every event, in order,
for one to four levels at ratios 2 and 4, with and without periodic
regrids; the structure the recursion fixes (level l advances ratio^l times
per coarse step, each level's steps tile the coarse step without gaps, a
synchronisation follows the finer levels' catch-up, the synchronized start
ends at t0 + 3 k0); the interpolation offsets eta of eq. timeInterp stay in
[0, k_coarse] and place t* between the two newest coarse slices; times
stay exact over many steps; argument errors.  No GPU."""
import os
from fractions import Fraction

import pytest

from oracle import subcycle as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2506_02663_amd", "libamg.so")


@pytest.fixture(scope="module")
def A():
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    from paper_2506_02663_amd import amg
    return amg


def as_float(ev):
    return [(k, l, float(t), float(dt), float(kc), float(tc)) for k, l, t, dt, kc, tc in ev]


@pytest.mark.parametrize("nlevels", [1, 2, 3, 4])
@pytest.mark.parametrize("ratio", [2, 4])
@pytest.mark.parametrize("regrid_every", [0, 1, 3])
def test_schedule_matches_the_oracle(A, nlevels, ratio, regrid_every):
    # dyadic t0 and k0: every time is exact in binary
    t0, k0 = Fraction(5, 8), Fraction(1, 64)
    got = A.subcycle_schedule(nlevels, ratio, float(t0), float(k0), 4, regrid_every)
    want = as_float(S.schedule(nlevels, ratio, t0, k0, 4, regrid_every))
    assert got == want


def test_structure_of_one_coarse_step(A):
    nl, r, k0 = 3, 2, 0.5
    ev = A.subcycle_schedule(nl, r, 0.0, k0, 1)
    synced = [e for e in ev if e[0] == "synced"]
    assert len(synced) == 3 * r ** (nl - 1)
    assert synced[-1][2] + synced[-1][3] == 3 * k0  # the start ends at t0 + 3 k0
    adv = [e for e in ev if e[0] == "advance"]
    for l in range(nl):
        mine = [e for e in adv if e[1] == l]
        assert len(mine) == r ** l
        assert all(e[3] == k0 / r ** l for e in mine)
        # the steps of a level tile the coarse step
        ts = [e[2] for e in mine]
        assert ts[0] == 3 * k0 and all(b - a == k0 / r ** l for a, b in zip(ts, ts[1:]))
    # a level is advanced only after its coarser level has reached its end
    for i, e in enumerate(ev):
        if e[0] == "advance" and e[1] > 0:
            assert e[5] >= e[2] + e[3]  # the coarse slices reach the end of the fine step
    # a sync of level l follows the last advance of level l+1 in its step
    syncs = [i for i, e in enumerate(ev) if e[0] == "sync"]
    for i in syncs:
        l = ev[i][1]
        prev = [e for e in ev[:i] if e[0] == "advance" and e[1] == l + 1]
        assert prev[-1][2] + prev[-1][3] == ev[i][2]
    assert ev[-1][0] == "sync" and ev[-1][1] == 0


@pytest.mark.parametrize("ratio", [2, 4])
def test_eta_between_the_newest_coarse_slices(A, ratio):
    ev = A.subcycle_schedule(3, ratio, 0.0, 1.0 / 16, 3)
    oev = S.schedule(3, ratio, 0, Fraction(1, 16), 3)
    for e, o in zip(ev, oev):
        if e[0] != "advance" or e[1] == 0:
            continue
        for c in (0, Fraction(1, 2), Fraction(83, 250), Fraction(31, 50), Fraction(17, 20), 1):
            eta = S.eta(o, c)
            assert 0 <= eta <= o[4]
            # the library's event gives the same eta
            assert abs((e[2] + float(c) * e[3] - (e[5] - e[4])) - float(eta)) < 1e-15


def test_times_stay_exact_over_many_steps(A):
    # a non-dyadic step: times are t0 + n k_finest, no accumulated drift
    k0 = 0.1
    ev = A.subcycle_schedule(2, 4, 0.0, k0, 2000)
    last = [e for e in ev if e[0] == "advance" and e[1] == 0][-1]
    assert last[2] == pytest.approx(3 * k0 + 1999 * k0, rel=1e-15)
    fine = [e for e in ev if e[0] == "advance" and e[1] == 1]
    assert fine[-1][2] + fine[-1][3] == pytest.approx(3 * k0 + 2000 * k0, rel=1e-15)


def test_errors(A):
    import ctypes as C
    L = A.lib()
    n = C.c_int32()
    for args in [(0, 2, 0.0, 1.0, 1, 0), (9, 2, 0.0, 1.0, 1, 0), (2, 3, 0.0, 1.0, 1, 0), (2, 2, 0.0, 0.0, 1, 0),
                 (2, 2, 0.0, 1.0, -1, 0), (2, 2, 0.0, 1.0, 1, -1)]:
        assert L.amg_subcycle_schedule(*args, 0, C.byref(n), None) == A.EINVAL
    # too small a buffer: EUNSUPPORTED, the total still reported
    ev = (A.ScEvent * 4)()
    assert L.amg_subcycle_schedule(2, 2, 0.0, 1.0, 1, 0, 4, C.byref(n), ev) == A.EUNSUPPORTED
    assert n.value == len(S.schedule(2, 2, 0, 1, 1))


def test_oracle_pinned_by_hand():
    """Two levels, ratio 2, k0 = 1 from t0 = 0, two coarse steps, read off
    Algorithm 1 by hand: six synchronized steps of 1/2 to t = 3, then per
    coarse step the level-0 step, two level-1 steps interpolating from the
    level-0 slices ending at the coarse step's end, and the synchronisation."""
    h = Fraction(1, 2)
    want = [("synced", 1, i * h, h, 0, 0) for i in range(6)]
    for t in (3, 4):
        want += [("advance", 0, t, 1, 0, 0), ("advance", 1, t, h, 1, t + 1), ("advance", 1, t + h, h, 1, t + 1),
                 ("sync", 0, t + 1, 0, 0, 0)]
    assert S.schedule(2, 2, 0, 1, 2) == want
    # one level: no recursion, no synchronisation; a regrid before each step
    assert S.schedule(1, 4, 0, 1, 2, regrid_every=1) == [("synced", 0, 0, 1, 0, 0), ("synced", 0, 1, 1, 0, 0),
                                                          ("synced", 0, 2, 1, 0, 0), ("regrid", 0, 3, 0, 0, 0),
                                                          ("advance", 0, 3, 1, 0, 0), ("regrid", 0, 4, 0, 0, 0),
                                                          ("advance", 0, 4, 1, 0, 0)]
