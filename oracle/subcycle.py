"""The time schedule of Algorithm 1 (Section 6.2) and of its start, written
from the paper in exact rational arithmetic.  Test infrastructure only: the
tests compare the library's schedule with this one.

Algorithm 1 first advances the composite velocity by synchronized AMR
(Section 5.5: every level with the finest step k^lmax = k0 / r^lmax) from t0
to t0 + 3 k0, which fills the four time slices of eq. vel_slicing for every
level; then, per coarse step (while t^0 < t_e), it regrids if the criteria
hold and calls SingleLevelAdvance(0).  SingleLevelAdvance(l) advances level
l by one step k^l = k0 / r^l from t^l to t^l + k^l (for l > 0 with the
interface conditions of eq. GePUP-localized from the slices of level l-1),
then, for l < lmax, calls SingleLevelAdvance(l+1) while t^(l+1) is behind
the new t^l, and finally synchronizes levels l..lmax by the composite
projection (eq. comp_ProjOp).

Readings (the paper leaves them open):
- the regridding criterion is a fixed period: before coarse step j (j = 0,
  1, ...) when regrid_every > 0 and j is a multiple of it;
- the time interpolation of a level-l stage (l > 0) at t* = t^l + c k^l uses
  the slices of level l-1 at t_-i = t^(l-1) - i k^(l-1), t^(l-1) the newest
  (level l-1 has already advanced to or past t*), so eta = t* - t_-1 of eq.
  timeInterp lies in [0, k^(l-1)].

Events are tuples (kind, level, t, dt, k_coarse, t_coarse):
  ("synced", lmax, t, k^lmax, 0, 0): one synchronized AMR step of all levels;
  ("regrid", 0, t, 0, 0, 0);
  ("advance", l, t^l, k^l, k^(l-1), t^(l-1)) (level 0: k_coarse = t_coarse = 0);
  ("sync", l, t_sync, 0, 0, 0): the composite projection of levels l..lmax.
"""
from fractions import Fraction


def schedule(nlevels, ratio, t0, k0, ncoarse, regrid_every=0):
    """Algorithm 1's events for ncoarse coarse steps after the synchronized
    start (exact Fractions for the times)."""
    assert nlevels >= 1 and ratio >= 2 and ncoarse >= 0
    t0, k0 = Fraction(t0), Fraction(k0)
    lmax = nlevels - 1
    k = [k0 / ratio ** l for l in range(nlevels)]
    ev = []
    # line 1: synchronized AMR from t0 to t0 + 3 k0 with the finest step
    t = t0
    for _ in range(3 * ratio ** lmax):
        ev.append(("synced", lmax, t, k[lmax], Fraction(0), Fraction(0)))
        t += k[lmax]
    # line 2: every level at t0 + 3 k0
    tl = [t0 + 3 * k0] * nlevels

    def single_level_advance(l):
        kc = k[l - 1] if l > 0 else Fraction(0)
        tc = tl[l - 1] if l > 0 else Fraction(0)
        ev.append(("advance", l, tl[l], k[l], kc, tc))
        tsync = tl[l] + k[l]
        tl[l] = tsync
        if l < lmax:
            while tl[l + 1] < tsync:
                single_level_advance(l + 1)
            ev.append(("sync", l, tsync, Fraction(0), Fraction(0), Fraction(0)))

    for j in range(ncoarse):
        if regrid_every > 0 and j % regrid_every == 0:
            ev.append(("regrid", 0, tl[0], Fraction(0), Fraction(0), Fraction(0)))
        single_level_advance(0)
    return ev


def eta(event, c):
    """eta of eq. timeInterp for the stage at t* = t + c dt of a level-l
    advance (l > 0): t* minus the second newest slice of level l-1."""
    kind, l, t, dt, kc, tc = event
    assert kind == "advance" and l > 0
    return t + Fraction(c) * dt - (tc - kc)
