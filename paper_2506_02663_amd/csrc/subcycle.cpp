// Host side of Algorithm 1 (Section 6.2): the order and times of the level
// advances of the subcycled AMR method and of its synchronized start.  The
// library advances no level here; the events tell a driver which level to
// advance over which step, with the time slices of the next coarser level
// its interface conditions interpolate from (eq. timeInterp through
// amg_cic_face_data), and when to synchronise.
//
// Times are kept as integer counts of the finest step k0 / ratio^(nlevels-1),
// so the recursion's comparisons are exact; each event's time is t0 plus
// its count times that step.
#include <cstdint>
#include <vector>

#include "../../include/amg.h"

namespace {

struct Sched {
  int lmax = 0;
  double t0 = 0.0, kf = 0.0;
  std::vector<int64_t> steps;  // finest steps per step of each level
  std::vector<int64_t> tl;     // current time of each level, in finest steps
  amg_sc_event* out = nullptr;
  int cap = 0, n = 0;

  void emit(int kind, int level, int64_t t, int64_t dt, int64_t kc, int64_t tc) {
    if (n < cap) {
      amg_sc_event& e = out[n];
      e.kind = kind;
      e.level = level;
      e.t = t0 + (double)t * kf;
      e.dt = (double)dt * kf;
      e.k_coarse = (double)kc * kf;
      e.t_coarse = kind == AMG_SC_ADVANCE && level > 0 ? t0 + (double)tc * kf : 0.0;
    }
    ++n;
  }

  // SingleLevelAdvance(l): level l one step, then the finer levels up to its
  // new time, then the composite projection of levels l..lmax
  void advance(int l) {
    emit(AMG_SC_ADVANCE, l, tl[l], steps[l], l > 0 ? steps[l - 1] : 0, l > 0 ? tl[l - 1] : 0);
    const int64_t tsync = tl[l] + steps[l];
    tl[l] = tsync;
    if (l < lmax) {
      while (tl[l + 1] < tsync) advance(l + 1);
      emit(AMG_SC_SYNC, l, tsync, 0, 0, 0);
    }
  }
};

}  // namespace

extern "C" int amg_subcycle_schedule(int nlevels, int ratio, double t0, double k0, int ncoarse, int regrid_every,
                                     int max_events, int32_t* nevents, amg_sc_event* events) {
  if (nlevels < 1 || nlevels > 8 || (ratio != 2 && ratio != 4) || !(k0 > 0) || ncoarse < 0 ||
      regrid_every < 0 || max_events < 0 || !nevents || (max_events > 0 && !events))
    return AMG_EINVAL;
  Sched S;
  S.lmax = nlevels - 1;
  S.t0 = t0;
  int64_t fine = 1;
  for (int l = 0; l < S.lmax; ++l) fine *= ratio;
  S.kf = k0 / (double)fine;
  S.steps.resize(nlevels);
  for (int l = 0; l < nlevels; ++l) {
    int64_t s = 1;
    for (int m = l; m < S.lmax; ++m) s *= ratio;
    S.steps[l] = s;
  }
  S.out = events;
  S.cap = max_events;
  // line 1: synchronized AMR with the finest step up to t0 + 3 k0
  for (int64_t i = 0; i < 3 * fine; ++i) S.emit(AMG_SC_SYNCED, S.lmax, i, 1, 0, 0);
  // line 2: every level at t0 + 3 k0
  S.tl.assign(nlevels, 3 * fine);
  for (int j = 0; j < ncoarse; ++j) {
    if (regrid_every > 0 && j % regrid_every == 0) S.emit(AMG_SC_REGRID, 0, S.tl[0], 0, 0, 0);
    S.advance(0);
  }
  *nevents = S.n;
  return S.n > max_events ? AMG_EUNSUPPORTED : AMG_OK;
}
