// C ABI entry points (include/amg.h) and the solver driver: the V-cycle of
// Section 6.5 on the multigrid depths of one level, inside an outer
// residual-correction loop (FP64, or FP32 V-cycles inside FP64 iterative
// refinement), with the per-component solvability shift and mean removal.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <type_traits>
#include <vector>

#include "amg_internal.h"
#include "kernels.h"

using namespace amg;

namespace {

// device scalar slots of a level: residual norm, the constant 1, per-level
// norms of a composite cycle (level 0's array), per-level face-data sums
enum { S_NORM = 0, S_ONE = 1, S_LEV = 2, S_FD = 20, S_FSUM = 38, S_DELTA = 39, S_DOT = 40, S_COUNT = 41 };

#define HIPCHK(expr)                                                      \
  do {                                                                    \
    hipError_t e_ = (expr);                                               \
    if (e_ != hipSuccess) {                                               \
      H->err = std::string(#expr) + ": " + hipGetErrorString(e_);          \
      return AMG_EDEVICE;                                                 \
    }                                                                     \
  } while (0)

int fail(amg_hier* H, int code, const std::string& msg) {
  if (H) H->err = msg;
  return code;
}

// ---- static scratch of the allocation-free entry point ----------------------
// kNoAllocDoubles FP64 words of device memory that every GPU holds from the
// load of the library to the end of the process; amg_dot_noalloc keeps its
// per-tile partial sums there instead of in the level's partial buffer.  In
// host code the array's name is only a stand-in: its device address is looked
// up once per device (hipGetSymbolAddress) and that address is what kernels
// receive.
constexpr int64_t kNoAllocDoubles = 32768;  // 256 KiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];
constexpr int kMaxDevices = 64;
double* g_scratch_ptr[kMaxDevices] = {};

// the device address of `scratch` on the current device (looked up once per
// device, at amg_finalize or at the first allocation-free call there)
hipError_t scratch_address(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

template <typename T>
int upload(amg_hier* H, T** dst, const std::vector<T>& v) {
  size_t n = std::max<size_t>(v.size(), 1);
  HIPCHK(hipMalloc((void**)dst, n * sizeof(T)));
  if (!v.empty()) HIPCHK(hipMemcpy(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
  return AMG_OK;
}

template <typename T>
int zalloc(amg_hier* H, T** dst, size_t n) {
  n = std::max<size_t>(n, 1);
  HIPCHK(hipMalloc((void**)dst, n * sizeof(T)));
  HIPCHK(hipMemset(*dst, 0, n * sizeof(T)));
  return AMG_OK;
}

#define TRY(expr)               \
  do {                          \
    int rc_ = (expr);           \
    if (rc_ != AMG_OK) return rc_; \
  } while (0)

// A u = alpha u + beta * (sum of the 1-D stencils), eq. (discreteOps c)
template <typename T>
void coefs(const amg_hier* H, const Depth& D, T& alpha, T& beta) {
  const double K = 1.0 / (12.0 * D.h * D.h);
  if (H->op == AMG_HELMHOLTZ) {
    alpha = T(1);
    beta = T(-H->c * K);
  } else {
    alpha = T(0);
    beta = T(K);
  }
}

template <typename T>
struct Bufs;
template <>
struct Bufs<double> {
  static double* e(Depth& D) { return D.e64; }
  static double* f(Depth& D) { return D.f64; }
  static double* t(Depth& D) { return D.t64; }
};
template <>
struct Bufs<float> {
  static float* e(Depth& D) { return D.e32; }
  static float* f(Depth& D) { return D.f32; }
  static float* t(Depth& D) { return D.t32; }
};

// Struct holding one call's view of a level; tr: the adjoint system (the
// transposed operator at every depth)
struct Run {
  amg_hier* H;
  Level* L;
  int dim;
  hipStream_t st;
  bool tr = false;
};

// ghosts before an operator application: the fill of the homogeneous
// operator, or of its transpose
template <typename T>
void fill_op(const Run& R, const Depth& D, T* u) {
  if (R.tr)
    launch_fill_tr<T>(D, u, R.st);
  else
    launch_fill<T>(D, u, nullptr, R.st);
}

// event timing around launches of one kernel kind (finest depth only)
struct Timed {
  Timer* t;
  hipStream_t st;
  bool active;
  size_t idx;
  Timed(const Run& R, int kind, int depth) : t(&R.H->timer), st(R.st), active(false), idx(0) {
    if (!t->on || depth != 0 || t->next + 2 > t->pool.size()) return;
    active = true;
    idx = t->next;
    t->pending.push_back({kind, idx});
    (void)hipEventRecord(t->pool[idx], st);
    t->next += 2;
  }
  ~Timed() {
    if (active) (void)hipEventRecord(t->pool[idx + 1], st);
  }
};

// accumulate the durations of recorded event pairs (after the stream is idle)
void accumulate(Timer& t, const std::vector<std::pair<int, size_t>>& pairs) {
  for (auto& p : pairs) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.pool[p.second], t.pool[p.second + 1]) == hipSuccess) {
      t.count[p.first] += 1;
      t.total_ms[p.first] += ms;
    } else {
      (void)hipGetLastError();
    }
  }
}

void collect_timing(Timer& t) {
  accumulate(t, t.pending);
  t.pending.clear();
  t.next = t.base;
}

// per-component sums of the tile partials in L.partial (two fixed-order stages)
void comp_sums(const Run& R, const Depth& D, double* out, const double* in = nullptr) {
  Level& L = *R.L;
  const int nseg = (int)D.seg_ptr.size() - 1;
  launch_seg_reduce(in ? in : L.partial, D.d_seg, nseg, 0, L.partial2, false, R.st);
  launch_seg_reduce(L.partial2, D.d_cseg, L.ncomp, 0, out, false, R.st);
}

// max of the tile partials in L.partial
// host (may be null): pinned host memory that receives the maximum too
void global_max(const Run& R, const Depth& D, double* out, double* host = nullptr) {
  Level& L = *R.L;
  const int nseg = (int)D.seg_ptr.size() - 1;
  const int nt = (int)D.tiles.size();
  if (nt <= 16384) {  // one block over all tile partials
    launch_seg_reduce(L.partial, nullptr, 1, nt, out, true, R.st, host);
    return;
  }
  launch_seg_reduce(L.partial, D.d_seg, nseg, 0, L.partial2, true, R.st);
  launch_seg_reduce(L.partial2, nullptr, 1, nseg, out, true, R.st, host);
}

// Subtract the per-component mean on every singular component (depth k).
template <typename T>
void remove_mean(const Run& R, int k, T* a) {
  Level& L = *R.L;
  if (!L.nsingular) return;
  Depth& D = L.depths[k];
  // small depths: one launch, one block per component
  int64_t maxc = 0;
  for (int c = 0; c < L.ncomp; ++c) maxc = std::max<int64_t>(maxc, L.comp_cells[c] >> (R.dim * k));
  if (maxc <= 16384 && D.boxes.size() <= 64) {
    launch_comp_mean_small<T>(R.dim, D, L.ncomp, L.d_comp_flag, L.d_comp_cnt + (size_t)k * L.ncomp, a, R.st);
    return;
  }
  launch_tile_sum<T>(R.dim, D, a, L.partial, R.st);
  if (D.tiles.size() <= 1024) {  // every block re-sums at most 1024 tile sums
    launch_comp_mean_shift<T>(R.dim, D, L.partial, L.d_comp_flag, L.d_comp_cnt + (size_t)k * L.ncomp, a, R.st);
    return;
  }
  launch_comp_mean_delta(D, L.partial, L.d_comp_flag, L.d_comp_cnt + (size_t)k * L.ncomp, L.ncomp, L.d_delta, R.st);
  launch_comp_shift<T>(R.dim, D, a, L.d_delta, R.st);
}

// nsweeps homogeneous sweeps at depth k; `cur` holds the iterate (zero if
// from_zero), `oth` is the second buffer; both may be swapped.
template <typename T>
void smooth(const Run& R, int k, int smoother, int nsweeps, double omega, bool from_zero, T*& cur, T*& oth,
            const T* f) {
  Depth& D = R.L->depths[k];
  T alpha, beta;
  coefs<T>(R.H, D, alpha, beta);
  if (nsweeps <= 0) {
    if (from_zero) launch_zero<T>(cur, D.nstored, R.st);
    return;
  }
  // FP32 forward sweeps compute the ghosts of filled columns where they read
  // them: no fill launch when the depth has no other ghosts
  const int gr = (sizeof(T) == 4 && !R.tr) ? 1 : 0;
  const bool fill = !(gr && D.fill_only);
  if (smoother == AMG_SMOOTH_JACOBI) {
    for (int s = 0; s < nsweeps; ++s) {
      if (s == 0 && from_zero) {
        launch_jacobi<T>(R.dim, D, nullptr, f, cur, alpha, beta, (T)omega, true, R.st);
        continue;
      }
      if (fill) {
        Timed tm(R, AMG_T_FILL, k);
        fill_op<T>(R, D, cur);
      }
      {
        Timed tm(R, AMG_T_SWEEP, k);
        launch_jacobi<T>(R.dim, D, cur, f, oth, alpha, beta, (T)omega, false, R.st, gr);
      }
      if (R.tr) launch_band<T>(R.dim, D, 1, cur, oth, alpha, beta, -(T)omega * beta, 0, R.st);
      std::swap(cur, oth);
    }
  } else {
    for (int s = 0; s < nsweeps; ++s) {
      for (int col = 0; col < 2; ++col) {
        if (s == 0 && col == 0 && from_zero) {
          launch_rb<T>(R.dim, D, nullptr, f, cur, alpha, beta, (T)omega, 0, true, R.st);
          continue;
        }
        if (fill) {
          Timed tm(R, AMG_T_FILL, k);
          fill_op<T>(R, D, cur);
        }
        {
          Timed tm(R, AMG_T_SWEEP, k);
          launch_rb<T>(R.dim, D, cur, f, oth, alpha, beta, (T)omega, col, false, R.st, gr);
        }
        if (R.tr) launch_band<T>(R.dim, D, 2, cur, oth, alpha, beta, -(T)omega * beta, col, R.st);
        std::swap(cur, oth);
      }
    }
  }
}

// relaxation factor of the chosen smoother: the Jacobi weight, or the
// red-black half-sweeps' factor
inline double relax(const amg_solve_opts& o) { return o.smoother == AMG_SMOOTH_RB ? o.omega_rb : o.omega; }

// nsweeps red-black sweeps of a depth in colour-split storage: the iterate
// starts in buffer a (both halves), b is the second buffer; each half-sweep
// writes its colour's half into the buffer that does not hold it.  Returns
// the buffer that holds the final iterate (both halves).  fsc (may be null):
// fs holds the unscaled residual, read as (fs - fdl[comp]) / fsc[0].  xu
// (may be null): the last half-sweep adds su[0] times the final iterate to
// the FP64 array xu instead of storing it (the outer update fused into it),
// and the function returns null.
float* smooth_split(const Run* R, hipStream_t st, int dim, const Depth& D, int k, int nsweeps, float alpha,
                    float beta, float omega, const float* fs, float* a, float* b, const double* fsc = nullptr,
                    const double* fdl = nullptr, double* xu = nullptr, const double* su = nullptr) {
  const int64_t hs = D.nstored / 2;
  const float* h[2] = {a, a + hs};
  for (int s = 0; s < nsweeps; ++s)
    for (int col = 0; col < 2; ++col) {
      float* dst = (h[col] == a + col * hs ? b : a) + col * hs;
      if (xu && s == nsweeps - 1 && col == 1) {
        if (R) {
          Timed tm(*R, AMG_T_SWEEP, k);
          launch_rbs(dim, D, 3, h[0], h[1], fs + col * hs, dst, alpha, beta, omega, col, st, fsc, fdl, xu, su);
        } else {
          launch_rbs(dim, D, 3, h[0], h[1], fs + col * hs, dst, alpha, beta, omega, col, st, fsc, fdl, xu, su);
        }
        return nullptr;
      }
      if (R) {
        Timed tm(*R, AMG_T_SWEEP_SPLIT, k);
        launch_rbs(dim, D, 0, h[0], h[1], fs + col * hs, dst, alpha, beta, omega, col, st, fsc, fdl);
      } else {
        launch_rbs(dim, D, 0, h[0], h[1], fs + col * hs, dst, alpha, beta, omega, col, st, fsc, fdl);
      }
      h[col] = dst;
    }
  return const_cast<float*>(h[0]);
}

// Pre-smoothing of depth 0 in colour-split storage from e = 0: nsweeps
// red-black sweeps into buffer a (b: the second buffer).  The first
// half-sweep starts from zero and writes the red half; the second reads only
// the red half (its own colour is still zero) and writes the black half of
// the same buffer.  Returns the buffer that holds the iterate.
float* presmooth_split(const Run& R, const Depth& D, int nsweeps, float alpha, float beta, float omega,
                       const float* fs, float* a, float* b, const double* fsc, const double* fdl) {
  if (nsweeps <= 0) {
    launch_zero<float>(a, D.nstored, R.st);
    return a;
  }
  const int64_t hs = D.nstored / 2;
  {
    Timed tm(R, AMG_T_SWEEP, 0);
    launch_rbs(R.dim, D, 2, nullptr, nullptr, fs, a, alpha, beta, omega, 0, R.st, fsc, fdl);
  }
  {
    Timed tm(R, AMG_T_SWEEP, 0);
    launch_rbs(R.dim, D, 1, a, a + hs, fs + hs, a + hs, alpha, beta, omega, 1, R.st, fsc, fdl);
  }
  return smooth_split(&R, R.st, R.dim, D, 0, nsweeps - 1, alpha, beta, omega, fs, a, b, fsc, fdl);
}

// whether a mixed-precision solve runs depth 0 in colour-split storage (its
// right-hand side is then written split)
inline bool use_split(const amg_hier* H, const Depth& D0, const amg_solve_opts& o) {
  return D0.split_rb && D0.fs32 && o.smoother == AMG_SMOOTH_RB && o.nu2 > 0;
}

// First depth of the FP32 V-cycle's coarse tail (tail.hip), or -1: the
// first depth k >= 1 of at most 4096 cells from which every depth holds one
// box whose faces are filled uniformly or wrap onto it, and the coarsest is
// one exact system; at least one depth above the bottom.
// direction d of depth D's one box wraps onto the box itself (periodic, and
// the box spans the grid)
bool tail_wraps(const Depth& D, int d) { return D.periodic[d] && D.boxd[0].n[d] == D.dn[d]; }

// every face of depth D's one box filled uniformly from its own rows, or
// wrapping onto the box (an exchange face: column code 0)
bool tail_faces(const Depth& D, int dim) {
  for (int d = 0; d < dim; ++d)
    for (int s = 0; s < 2; ++s) {
      const uint8_t c = D.boxd[0].ucode[d][s];
      if (tail_wraps(D, d) ? c != 0 : (c != 5 && c != 6)) return false;
    }
  return true;
}

int tail_start(const Run& R, const amg_solve_opts& o) {
  const Level& L = *R.L;
  const int K = (int)L.depths.size();
  if (!R.H->tail || R.tr || L.ncomp != 1 || K < 3) return -1;
  if (o.smoother != AMG_SMOOTH_RB && o.smoother != AMG_SMOOTH_JACOBI) return -1;
  const Depth& B = L.depths[K - 1];
  if (B.boxes.size() != 1 || B.groups.size() != 1 || B.groups[0].ninst != 1 || !B.stiles.empty() ||
      !tail_faces(B, R.dim))
    return -1;
  int kt = -1;
  for (int k = K - 2; k >= 1; --k) {
    const Depth& D = L.depths[k];
    if (D.boxes.size() != 1 || !tail_faces(D, R.dim) || D.stiles.empty() || !D.groups.empty()) break;
    const BoxD& b = D.boxd[0];
    if ((int64_t)b.n[0] * b.n[1] * b.n[2] > kTailMaxCells || K - k > kTailMaxDepths) break;
    // LDS of both legs: two arrays of depth k, one of depth k + 1
    auto padded = [&](const BoxD& x) {
      return (size_t)(x.n[0] + 4) * (x.n[1] + 4) * (R.dim == 3 ? x.n[2] + 4 : 1) * sizeof(float);
    };
    if (2 * padded(b) + padded(L.depths[k + 1].boxd[0]) > tail_lds_limit()) break;
    kt = k;
  }
  return kt;
}

// The tail's three launches: down-leg (depths kt .. K-2), the bottom solve,
// up-leg; the result of depth kt lands in its e buffer.
void run_tail(const Run& R, const amg_solve_opts& o, int kt) {
  Level& L = *R.L;
  const int K = (int)L.depths.size();
  TailArgs A;
  memset(&A, 0, sizeof A);
  A.nd = K - kt;
  A.nu1 = o.nu1;
  A.nu2 = o.nu2;
  A.rb = o.smoother == AMG_SMOOTH_RB ? 1 : 0;
  A.singular = L.comp_singular[0] != 0;
  A.omega = (float)relax(o);
  for (int j = 0; j < A.nd; ++j) {
    Depth& D = L.depths[kt + j];
    TailDepth& T = A.d[j];
    T.b = D.boxd[0];
    T.e = D.e32;
    T.f = D.f32;
    coefs<float>(R.H, D, T.alpha, T.beta);
    T.cnt = (double)L.comp_cells[0] / std::pow(2.0, (double)(R.dim * (kt + j)));
    for (int d = 0; d < R.dim; ++d) T.wrap[d] = tail_wraps(D, d) ? 1 : 0;
  }
  Depth& B = L.depths[K - 1];
  launch_tail_down(R.dim, A, R.st);
  if (R.H->bottom_kind == AMG_BOTTOM_ILU_GMRES)
    launch_bottom_gmres<float>(B, L.d_mat, L.d_idx, B.f32, B.e32, R.H->bottom_iters, L.d_gws, R.st, B.t32);
  else
    launch_bottom<float>(B, L.d_mat, L.d_idx, B.f32, B.e32, false, R.st, B.t32);
  launch_tail_up(R.dim, A, R.st);
}

// One homogeneous V-cycle from e = 0; f0 is the depth-0 right-hand side, e0
// and t0 the two depth-0 buffers.  Returns the buffer that holds e.  With
// fs0 (FP32: the depth-0 right-hand side in colour-split storage, depth 0
// with split_rb; f0 is then not read) every depth-0 step runs in split
// storage and the returned e is split; with fsc0 fs0 holds the unscaled
// residual, which the split kernels read as (fs0 - fdl0[comp]) / fsc0[0];
// with xu (split only) the last half-sweep adds su[0] e to xu itself and
// the function returns null.
template <typename T>
T* vcycle(const Run& R, const amg_solve_opts& o, const T* f0, T* e0, T* t0, const float* fs0 = nullptr,
          const double* fsc0 = nullptr, const double* fdl0 = nullptr, double* xu = nullptr,
          const double* su = nullptr) {
  Level& L = *R.L;
  const int K = (int)L.depths.size();
  std::vector<T*> cur(K), oth(K);
  std::vector<const T*> f(K);
  for (int k = 0; k < K; ++k) {
    cur[k] = k ? Bufs<T>::e(L.depths[k]) : e0;
    oth[k] = k ? Bufs<T>::t(L.depths[k]) : t0;
    f[k] = k ? Bufs<T>::f(L.depths[k]) : f0;
  }
  // the coarse tail in three launches (FP32 forward cycles)
  const int kt = sizeof(T) == 4 ? tail_start(R, o) : -1;
  for (int k = 0; k < K; ++k) {
    Depth& D = L.depths[k];
    if (k == kt) {
      if constexpr (sizeof(T) == 4) {
        Timed tm(R, AMG_T_SWEEP, k);
        run_tail(R, o, k);
        cur[k] = D.e32;
      }
      break;
    }
    // boxes that end here: exact solve, written to both buffers of the depth
    if (!D.groups.empty()) {
      if (R.H->bottom_kind == AMG_BOTTOM_ILU_GMRES && !R.tr)  // the adjoint keeps the exact transposed inverse
        launch_bottom_gmres<T>(D, L.d_mat, L.d_idx, f[k], cur[k], R.H->bottom_iters, L.d_gws, R.st, oth[k]);
      else
        launch_bottom<T>(D, L.d_mat, L.d_idx, f[k], cur[k], R.tr, R.st, oth[k]);
    }
    if (k + 1 >= K || D.stiles.empty()) break;
    if constexpr (sizeof(T) == 4) {
      if (k == 0 && fs0) {
        T alpha, beta;
        coefs<T>(R.H, D, alpha, beta);
        float* s = presmooth_split(R, D, o.nu1, alpha, beta, (float)relax(o), fs0, cur[0], oth[0], fsc0, fdl0);
        if (s != cur[0]) std::swap(cur[0], oth[0]);
        {
          // the kernel writes the ghosts it reads itself: no fill launch
          Timed tm(R, AMG_T_RESTRICT, 0);
          launch_resid_restrict_s(R.dim, D, L.depths[1], cur[0], fs0, Bufs<T>::f(L.depths[1]), alpha, beta, R.st,
                                  fsc0, fdl0);
        }
        remove_mean<T>(R, 1, Bufs<T>::f(L.depths[1]));
        continue;
      }
    }
    smooth<T>(R, k, o.smoother, o.nu1, relax(o), true, cur[k], oth[k], f[k]);
    T alpha, beta;
    coefs<T>(R.H, D, alpha, beta);
    // below the finest depth the FP32 restriction writes the ghosts it reads
    // itself where every face is filled uniformly or wraps onto its box (no
    // fill launch)
    const int rgr = (sizeof(T) == 4 && !R.tr && k > 0 && D.wrap_fill) ? 1 : 0;
    if (!rgr) {
      Timed tm(R, AMG_T_FILL, k);
      fill_op<T>(R, D, cur[k]);
    }
    if (R.tr) {
      // residual of the transposed operator into the free buffer, then restrict
      launch_residual<T>(R.dim, D, false, cur[k], f[k], oth[k], alpha, beta, nullptr, R.st);
      launch_band<T>(R.dim, D, 0, cur[k], oth[k], alpha, beta, -beta, 0, R.st);
      launch_restrict<T>(R.dim, D, L.depths[k + 1], oth[k], Bufs<T>::f(L.depths[k + 1]), R.st);
    } else {
      Timed tm(R, AMG_T_RESTRICT, k);
      launch_resid_restrict<T>(R.dim, D, L.depths[k + 1], cur[k], f[k], Bufs<T>::f(L.depths[k + 1]), alpha, beta,
                               R.st, rgr);
    }
    remove_mean<T>(R, k + 1, Bufs<T>::f(L.depths[k + 1]));
  }
  for (int k = (kt > 0 ? kt - 1 : K - 2); k >= 0; --k) {
    Depth& D = L.depths[k];
    if (D.stiles.empty()) continue;
    // the FP32 prolongation into depths below the finest forms the coarse
    // ghosts it reads where the coarse faces are filled uniformly
    const int pgr = (sizeof(T) == 4 && !R.tr && k > 0 && L.depths[k + 1].wrap_fill) ? 1 : 0;
    if (!pgr) launch_fill<T>(L.depths[k + 1], cur[k + 1], nullptr, R.st);
    if constexpr (sizeof(T) == 4) {
      if (k == 0 && fs0) {
        // the prolongation writes the corrected iterate into the free buffer
        {
          Timed tm(R, AMG_T_PROLONG, k);
          launch_prolong_s(R.dim, D, L.depths[1], cur[1], cur[0], oth[0], R.st);
        }
        T alpha, beta;
        coefs<T>(R.H, D, alpha, beta);
        return smooth_split(&R, R.st, R.dim, D, 0, o.nu2, alpha, beta, (float)relax(o), fs0, oth[0], cur[0], fsc0,
                            fdl0, xu, su);
      }
    }
    {
      Timed tm(R, AMG_T_PROLONG, k);
      launch_prolong<T>(R.dim, D, L.depths[k + 1], cur[k + 1], cur[k], R.st, pgr);
    }
    smooth<T>(R, k, o.smoother, o.nu2, relax(o), false, cur[k], oth[k], f[k]);
  }
  return cur[0];
}

bool check_level(amg_hier* H, int level) {
  if (!H) return false;
  if (!H->finalized) {
    H->err = "amg_finalize has not been called";
    return false;
  }
  if (level < 0 || level >= H->nlevels) {
    H->err = "level out of range";
    return false;
  }
  return true;
}

hipStream_t stream_of(amg_hier* H, void* s) { return s ? (hipStream_t)s : H->own; }

void free_level(amg::Level& L) {
  for (auto& D : L.depths) {
    for (void* p : {(void*)D.d_box, (void*)D.d_codes, (void*)D.d_xsrc, (void*)D.d_chunks, (void*)D.d_tiles, (void*)D.d_stiles,
                    (void*)D.d_seg, (void*)D.d_cseg, (void*)D.d_cc_ptr, (void*)D.d_cc_idx, (void*)D.d_groups, (void*)D.d_band,
                    (void*)D.e64, (void*)D.f64, (void*)D.t64, (void*)D.e32, (void*)D.f32, (void*)D.t32, (void*)D.fs32, (void*)D.xg32})
      if (p) (void)hipFree(p);
  }
  if (L.d_gws) (void)hipFree(L.d_gws);
  for (void* p : {(void*)L.d_mat, (void*)L.d_idx, (void*)L.r64, (void*)L.fsh, (void*)L.partial, (void*)L.partial2, (void*)L.comp_sum,
                  (void*)L.scal, (void*)L.d_comp_flag, (void*)L.d_comp_cnt, (void*)L.d_delta, (void*)L.d_delta0, (void*)L.d_bsum,
                  (void*)L.d_defect, (void*)L.d_dfd, (void*)L.fdc, (void*)L.d_comp_ncf})
    if (p) (void)hipFree(p);
  if (L.h_scal) (void)hipHostFree(L.h_scal);
  const Composite& X = L.cmp;
  for (void* p : {(void*)L.E64, (void*)L.d_face_valid, (void*)X.d_w, (void*)X.d_cfi_dst, (void*)X.d_cfi_src,
                  (void*)X.d_cfi_w, (void*)X.d_avg, (void*)X.d_rfx_cell, (void*)X.d_rfx_ptr, (void*)X.d_rfx_face,
                  (void*)X.d_pro, (void*)L.A64, (void*)L.mu, (void*)X.d_cfi_e0, (void*)X.d_cfi_in,
                  (void*)X.d_cfi_layer, (void*)X.d_cfiT_elem, (void*)X.d_cfiT_ptr, (void*)X.d_cfiT_ent,
                  (void*)X.d_rfxTc_elem, (void*)X.d_rfxTc_ptr, (void*)X.d_rfxTc_src, (void*)X.d_rfxTc_coef,
                  (void*)X.d_rfxTf_elem, (void*)X.d_rfxTf_ptr, (void*)X.d_rfxTf_src, (void*)X.d_rfxTf_coef})
    if (p) (void)hipFree(p);
  for (int d = 0; d < 3; ++d)
    for (const Composite::GatherT* t : {&X.rfxVc[d], &X.rfxVf[d]})
      for (void* p : {(void*)t->d_elem, (void*)t->d_ptr, (void*)t->d_src, (void*)t->d_coef})
        if (p) (void)hipFree(p);
  for (auto& D : L.depths)
    for (void* p : {(void*)D.d_exT_elem, (void*)D.d_exT_slot, (void*)D.d_exT_ptr})
      if (p) (void)hipFree(p);
  const CicTable& T = L.cic;
  for (void* p : {(void*)T.d_fd, (void*)T.d_src, (void*)T.d_wsel, (void*)T.d_w, (void*)T.d_ncf, (void*)T.d_sum})
    if (p) (void)hipFree(p);
}

// ---- composite (multi-level) solve -------------------------------------------
struct Comp {
  amg_hier* H;
  int hi;  // finest level of the composite (level 0 is the coarsest)
  hipStream_t st;
  bool tr = false;  // the adjoint (transposed) composite system
  bool lap = false;  // comp_residual with F = NULL gives L^comp x (the Laplacian, whatever the operator)
  std::vector<double*> X, R;
  std::vector<const double*> F, FD;
};

// Composite residual (COH-1..4): average the data down, fill every level's
// ghosts (coarse-fine ones by interpolation from the level below), level
// residuals, refluxing at coarse cells next to finer levels, and the
// residual averaged down onto covered cells.  Norm (max over all cells of
// all levels, which equals the max over valid cells since covered cells
// hold averages) into level 0's S_NORM slot.
void comp_residual(Comp& C) {
  amg_hier* H = C.H;
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  for (int l = C.hi; l >= 1; --l) launch_avgdown(dim, H->levels[l].cmp, C.X[l], C.X[l - 1], C.st);
  for (int l = 0; l <= C.hi; ++l) {
    Level& L = H->levels[l];
    Depth& D = L.depths[0];
    launch_fill<double>(D, C.X[l], C.FD[l], C.st);
    if (l) launch_cfi(dim, L.cmp, C.X[l - 1], C.X[l], C.st);
    double a, b;
    coefs<double>(H, D, a, b);
    if (C.lap) {
      a = 0.0;
      b = 1.0 / (12.0 * D.h * D.h);
    }
    launch_residual<double>(dim, D, true, C.X[l], C.F[l], C.R[l], a, b, nullptr, C.st);
  }
  const double kappa = C.lap ? 1.0 : (H->op == AMG_HELMHOLTZ ? H->c : -1.0);
  for (int l = 1; l <= C.hi; ++l)
    launch_reflux(dim, H->levels[l].cmp, C.X[l - 1], C.X[l], C.R[l - 1], kappa, H->levels[l - 1].depths[0].h,
                  H->levels[l].depths[0].h, C.st);
  for (int l = C.hi; l >= 1; --l) launch_avgdown(dim, H->levels[l].cmp, C.R[l], C.R[l - 1], C.st);
  for (int l = 0; l <= C.hi; ++l) {
    Level& L = H->levels[l];
    Run R{H, &L, dim, C.st};
    launch_tile_absmax<double>(dim, L.depths[0], C.R[l], L.partial, C.st);
    global_max(R, L.depths[0], L0.scal + S_LEV + l);
  }
  launch_max_slots(L0.scal + S_LEV, C.hi + 1, L0.scal + S_NORM, C.st);
}

// one V-cycle of level l's multigrid on the residual Rl (scaled by the norm
// in `sc`); x += s e and E += s e
void comp_level_vcycle(Comp& C, int l, const amg_solve_opts& o, double* Rl, const double* sc) {
  amg_hier* H = C.H;
  Level& L = H->levels[l];
  Depth& D0 = L.depths[0];
  Run R{H, &L, H->dim, C.st, C.tr};
  if (o.precision == AMG_MIXED) {
    launch_to32(H->dim, D0, Rl, D0.f32, sc, C.st);
    float* e = vcycle<float>(R, o, D0.f32, D0.e32, D0.t32);
    launch_update2<float>(H->dim, D0, C.X[l], L.E64, e, sc, C.st);
  } else {
    double* e = vcycle<double>(R, o, Rl, D0.e64, D0.t64);
    launch_update2<double>(H->dim, D0, C.X[l], L.E64, e, H->levels[0].scal + S_ONE, C.st);
  }
}

// one correction of level l: composite residual, a V-cycle of level l's
// multigrid on it (scaled by its max norm over the level), x_l += s e, and
// the correction prolonged onto every finer level of the composite
void comp_correct(Comp& C, const amg_solve_opts& o, int l) {
  amg_hier* H = C.H;
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  comp_residual(C);
  if (l == 0 && L0.nsingular) {
    Run R0{H, &L0, dim, C.st};
    remove_mean<double>(R0, 0, C.R[0]);
    launch_tile_absmax<double>(dim, L0.depths[0], C.R[0], L0.partial, C.st);
    global_max(R0, L0.depths[0], L0.scal + S_LEV);
  }
  Level& L = H->levels[l];
  launch_zero<double>(L.E64, L.depths[0].nstored, C.st);
  comp_level_vcycle(C, l, o, C.R[l], L0.scal + S_LEV + l);
  for (int m = l + 1; m <= C.hi; ++m) {
    launch_fill<double>(H->levels[m - 1].depths[0], H->levels[m - 1].E64, nullptr, C.st);
    launch_amr_prolong(dim, H->levels[m].cmp, H->levels[m - 1].E64, C.X[m], H->levels[m].E64, C.st);
  }
}

// one composite cycle: corrections of the levels in V order (finest .. 1,
// 0, 1 .. finest), average-down, composite mean removal (pure Neumann), and
// the new composite residual and its norm
void comp_cycle(Comp& C, const amg_solve_opts& o) {
  amg_hier* H = C.H;
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  for (int l = C.hi; l >= 1; --l) comp_correct(C, o, l);
  for (int l = 0; l <= C.hi; ++l) comp_correct(C, o, l);
  for (int l = C.hi; l >= 1; --l) launch_avgdown(dim, H->levels[l].cmp, C.X[l], C.X[l - 1], C.st);
  if (L0.nsingular) {
    // composite mean over valid cells = mean over all level-0 cells, since
    // covered cells hold the averages of the finer levels
    Run R0{H, &L0, dim, C.st};
    launch_tile_sum<double>(dim, L0.depths[0], C.X[0], L0.partial, C.st);
    comp_sums(R0, L0.depths[0], L0.comp_sum);
    launch_comp_delta(L0.comp_sum, nullptr, L0.d_comp_flag, L0.d_comp_cnt, L0.ncomp, 1.0, 0.0, L0.d_delta, nullptr,
                      C.st);
    for (int l = 0; l <= C.hi; ++l) launch_sub_scalar(dim, H->levels[l].depths[0], C.X[l], L0.d_delta, C.st);
  }
  comp_residual(C);
}

// ---- composite adjoint (the transposed composite system) ---------------------
// R_l = g_l - (A^comp)^T lam on the valid cells (see the oracle's reverse of
// average-down, AMRCFI, fills, stencils and refluxing); covered cells of R end
// as the sum of their children's residuals (volume-weighted transfers of the
// adjoint), the max norm over valid cells in level 0's S_NORM slot and the
// per-level max (covered cells included) in S_LEV + l.
void comp_residual_T(Comp& C) {
  amg_hier* H = C.H;
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  const double lscale = H->op == AMG_HELMHOLTZ ? -H->c : 1.0;
  for (int l = 0; l < C.hi; ++l) launch_zero_covered(H->levels[l + 1].cmp, C.X[l], C.st);
  for (int l = 0; l <= C.hi; ++l) launch_zero<double>(H->levels[l].A64, H->levels[l].depths[0].nstored, C.st);
  for (int l = 1; l <= C.hi; ++l)
    launch_rfx_T(H->levels[l].cmp, C.X[l - 1], lscale, H->levels[l - 1].A64, H->levels[l].A64, C.st);
  for (int l = 0; l <= C.hi; ++l) {
    Level& L = H->levels[l];
    Depth& D = L.depths[0];
    double a, b;
    coefs<double>(H, D, a, b);
    launch_fill_tr<double>(D, C.X[l], C.st);
    launch_residual<double>(dim, D, true, C.X[l], C.F[l], C.R[l], a, b, nullptr, C.st);
    launch_band_ab(dim, D, C.X[l], L.A64, C.R[l], b, C.st);
    launch_exch_T(D, L.A64, C.R[l], C.st);
    launch_sub_array(dim, D, L.A64, C.R[l], C.st);
    if (l) launch_cfi_T(dim, L.cmp, C.X[l], L.A64, b, L.mu, C.R[l - 1], C.st);
  }
  const double down = 1.0 / std::pow((double)H->ratio, dim);  // 1 / children per coarse cell
  for (int l = 1; l <= C.hi; ++l) {
    launch_pass_down(H->levels[l].cmp, C.R[l - 1], C.R[l], down, C.st);
    launch_zero_covered(H->levels[l].cmp, C.R[l - 1], C.st);
  }
  for (int l = 0; l <= C.hi; ++l) {
    Level& L = H->levels[l];
    Run R{H, &L, dim, C.st};
    launch_tile_absmax<double>(dim, L.depths[0], C.R[l], L.partial, C.st);
    global_max(R, L.depths[0], L0.scal + S_LEV + l);
  }
  launch_max_slots(L0.scal + S_LEV, C.hi + 1, L0.scal + S_NORM, C.st);
  for (int l = C.hi; l >= 1; --l) {
    launch_sumdown(dim, H->levels[l].cmp, C.R[l], C.R[l - 1], 1.0, C.st);
    Level& L = H->levels[l - 1];
    Run R{H, &L, dim, C.st};
    launch_tile_absmax<double>(dim, L.depths[0], C.R[l - 1], L.partial, C.st);
    global_max(R, L.depths[0], L0.scal + S_LEV + l - 1);
  }
}

// a -= w (sum over valid cells of a) / (sum of w), w = h_l^D per valid cell:
// the projection of the pure-Neumann adjoint along the volume weights
void proj_w(Comp& C, double* const* a) {
  amg_hier* H = C.H;
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  for (int l = 0; l < C.hi; ++l) launch_zero_covered(H->levels[l + 1].cmp, a[l], C.st);
  for (int l = C.hi; l >= 1; --l) launch_sumdown(dim, H->levels[l].cmp, a[l], a[l - 1], 1.0, C.st);
  Run R0{H, &L0, dim, C.st};
  launch_tile_sum<double>(dim, L0.depths[0], a[0], L0.partial, C.st);
  comp_sums(R0, L0.depths[0], L0.comp_sum);  // level 0 is one component
  const double vol = (double)L0.ncells * std::pow(L0.depths[0].h, dim);
  for (int l = 0; l <= C.hi; ++l) {
    launch_set_scaled(L0.comp_sum, std::pow(H->levels[l].depths[0].h, dim) / vol, L0.scal + S_LEV + l, C.st);
    launch_sub_scalar(dim, H->levels[l].depths[0], a[l], L0.scal + S_LEV + l, C.st);
  }
  for (int l = 0; l < C.hi; ++l) launch_zero_covered(H->levels[l + 1].cmp, a[l], C.st);
}

void comp_correct_T(Comp& C, const amg_solve_opts& o, int l) {
  amg_hier* H = C.H;
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  comp_residual_T(C);
  if (l == 0 && L0.nsingular) {
    Run R0{H, &L0, dim, C.st};
    remove_mean<double>(R0, 0, C.R[0]);
    launch_tile_absmax<double>(dim, L0.depths[0], C.R[0], L0.partial, C.st);
    global_max(R0, L0.depths[0], L0.scal + S_LEV);
  }
  Level& L = H->levels[l];
  launch_zero<double>(L.E64, L.depths[0].nstored, C.st);
  comp_level_vcycle(C, l, o, C.R[l], L0.scal + S_LEV + l);
  const double down = 1.0 / std::pow((double)H->ratio, dim);  // 1 / children per coarse cell
  for (int m = l + 1; m <= C.hi; ++m) {
    launch_fill<double>(H->levels[m - 1].depths[0], H->levels[m - 1].E64, nullptr, C.st);
    launch_amr_prolong(dim, H->levels[m].cmp, H->levels[m - 1].E64, C.X[m], H->levels[m].E64, C.st, down);
  }
}

void comp_cycle_T(Comp& C, const amg_solve_opts& o) {
  amg_hier* H = C.H;
  for (int l = C.hi; l >= 1; --l) comp_correct_T(C, o, l);
  for (int l = 0; l <= C.hi; ++l) comp_correct_T(C, o, l);
  if (H->levels[0].nsingular) proj_w(C, C.X.data());
  comp_residual_T(C);
}

}  // namespace

// ============================================================================
extern "C" {

void amg_default_opts(amg_solve_opts* o) {
  if (!o) return;
  o->nu1 = 2;
  o->nu2 = 2;
  o->smoother = AMG_SMOOTH_JACOBI;
  o->precision = AMG_MIXED;
  o->solvability = AMG_SOLV_RHS_SHIFT;
  o->max_cycles = 100;
  o->omega = 2.0 / 3.0;
  o->tol_rel = 1e-10;
  o->tol_abs = 0.0;
  o->use_graph = 1;
  o->pad_ = 0;
  o->omega_rb = 1.0;
}

int amg_create(int dim, const double* x_lo, const double* x_hi, const int32_t* base_cells, int ratio, int nlevels,
               amg_hier** out) {
  if (!out) return AMG_EINVAL;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || !x_lo || !x_hi || !base_cells || (ratio != 2 && ratio != 4) || nlevels < 1 ||
      nlevels > 16)
    return AMG_EINVAL;
  double h0 = 0;
  for (int d = 0; d < dim; ++d) {
    if (base_cells[d] < 4 || !std::isfinite(x_lo[d]) || !std::isfinite(x_hi[d]) || !(x_hi[d] > x_lo[d]))
      return AMG_EINVAL;
    const double h = (x_hi[d] - x_lo[d]) / base_cells[d];
    if (d == 0) h0 = h;
    // cells are cubes (eq. grids): one h for every direction
    if (std::fabs(h - h0) > 1e-12 * h0) return AMG_EINVAL;
  }
  amg_hier* H = new amg_hier();
  H->dim = dim;
  for (int d = 0; d < dim; ++d) {
    H->base[d] = base_cells[d];
    H->x_lo[d] = x_lo[d];
  }
  H->h0 = h0;
  H->ratio = ratio;
  H->nlevels = nlevels;
  H->levels.resize(nlevels);
  *out = H;
  return AMG_OK;
}

int amg_destroy(amg_hier* H) {
  if (!H) return AMG_OK;
  for (auto& L : H->levels) L.graph.release();
  for (auto& L : H->levels) L.graphT.release();
  H->comp_graph.release();
  H->comp_graphT.release();
  for (auto& e : H->timer.pool) (void)hipEventDestroy(e);
  for (auto& L : H->levels) free_level(L);
  if (H->imex_ws) (void)hipFree(H->imex_ws);
  if (H->regrid_ws) (void)hipFree(H->regrid_ws);
  if (H->own) (void)hipStreamDestroy(H->own);
  delete H;
  return AMG_OK;
}

const char* amg_last_error(const amg_hier* H) { return H ? H->err.c_str() : "null handle"; }

int amg_set_level_boxes(amg_hier* H, int level, int nboxes, const int32_t* lo, const int32_t* hi) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (level < 0 || level >= H->nlevels || nboxes < 0 || (nboxes && (!lo || !hi)))
    return fail(H, AMG_EINVAL, "bad level or box arrays");
  auto& B = H->levels[level].boxes;
  B.assign(nboxes, Box());
  for (int b = 0; b < nboxes; ++b)
    for (int d = 0; d < 3; ++d) {
      B[b].lo[d] = d < H->dim ? lo[b * H->dim + d] : 0;
      B[b].hi[d] = d < H->dim ? hi[b * H->dim + d] : 0;
    }
  return AMG_OK;
}

int amg_set_isolated_boxes(amg_hier* H, int level, int isolated) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (level < 0 || level >= H->nlevels) return fail(H, AMG_EINVAL, "level out of range");
  H->levels[level].isolated = isolated != 0;
  return AMG_OK;
}

int amg_set_physical_bc(amg_hier* H, int d, int side, int type) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (d < 0 || d >= H->dim || side < 0 || side > 1 || (type != AMG_DIRICHLET && type != AMG_NEUMANN && type != AMG_PERIODIC))
    return fail(H, AMG_EINVAL, "bad boundary condition");
  H->phys_bc[d][side] = type;
  return AMG_OK;
}

int amg_set_cf_mode(amg_hier* H, int level, int mode) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (level < 1 || level >= H->nlevels || mode < AMG_CF_DIRICHLET || mode > AMG_CF_INTERP)
    return fail(H, AMG_EINVAL, "bad coarse-fine mode");
  H->levels[level].cf_mode = mode;
  return AMG_OK;
}

int amg_set_operator(amg_hier* H, int kind, double c) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (kind == AMG_HELMHOLTZ && !(c > 0)) return fail(H, AMG_EINVAL, "Helmholtz needs c > 0");
  if (kind != AMG_HELMHOLTZ && kind != AMG_POISSON) return fail(H, AMG_EINVAL, "bad operator");
  H->op = kind;
  H->c = kind == AMG_HELMHOLTZ ? c : 0.0;
  return AMG_OK;
}

int amg_set_tuning(amg_hier* H, int key, int value) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  switch (key) {
    case AMG_TUNE_MARCH2:
    case AMG_TUNE_MARCH3:
      if (value < 2 || value > 4096 || (value & 1)) return fail(H, AMG_EINVAL, "march length must be even, 2..4096");
      (key == AMG_TUNE_MARCH2 ? H->march2 : H->march3) = value;
      return AMG_OK;
    case AMG_TUNE_SPLIT_RB:
      if (value != 0 && value != 1) return fail(H, AMG_EINVAL, "split red-black switch must be 0 or 1");
      H->split_rb = value;
      return AMG_OK;
    case AMG_TUNE_TAIL:
      if (value != 0 && value != 1) return fail(H, AMG_EINVAL, "tail switch must be 0 or 1");
      H->tail = value;
      return AMG_OK;
    case AMG_TUNE_ROW_ALIGN:
      if (value < 2 || value > 256 || (value & (value - 1)))
        return fail(H, AMG_EINVAL, "alignment must be a power of two of at least 2");
      H->row_align = value;
      return AMG_OK;
  }
  return fail(H, AMG_EINVAL, "unknown tuning key");
}

int amg_set_bottom_cells(amg_hier* H, int cells) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (cells < 0 || cells > 1024) return fail(H, AMG_EINVAL, "bottom cells must be 0..1024");
  H->bottom_cells = cells;
  return AMG_OK;
}

int amg_set_bottom_solver(amg_hier* H, int kind, int iters) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "layout is final");
  if (kind != AMG_BOTTOM_EXACT && kind != AMG_BOTTOM_ILU_GMRES) return fail(H, AMG_EINVAL, "unknown bottom solver");
  if (kind == AMG_BOTTOM_ILU_GMRES && (iters < 1 || iters > 16))
    return fail(H, AMG_EINVAL, "GMRES steps must be 1..16");
  H->bottom_kind = kind;
  if (kind == AMG_BOTTOM_ILU_GMRES) H->bottom_iters = iters;
  return AMG_OK;
}

int amg_finalize(amg_hier* H) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "already final");
  // Host planning first (validation, tables, bottom factors, composite
  // tables), so a rejected layout is reported before any device call.
  std::vector<std::vector<double>> mats(H->nlevels);
  std::vector<std::vector<int64_t>> idxs(H->nlevels);
  for (int l = 0; l < H->nlevels; ++l) {
    Level& L = H->levels[l];
    if (L.boxes.empty()) return fail(H, AMG_ELAYOUT, "level " + std::to_string(l) + " has no boxes");
    std::string err;
    int rc = plan_level(H, l, err);
    if (rc != AMG_OK) return fail(H, rc, err);
    rc = build_bottom(H, l, err, mats[l], idxs[l]);
    if (rc != AMG_OK) return fail(H, rc, err);
    L.face_valid.assign((size_t)std::max<int64_t>(L.nface, 1), 1);  // build_composite marks covered faces
  }
  for (int l = 1; l < H->nlevels; ++l) {
    Level& L = H->levels[l];
    std::string err;
    int rc = AMG_OK;
    if (L.cf_mode == AMG_CF_INTERP)
      rc = build_composite(H, l, err);
    else if (!L.isolated && !H->levels[l - 1].isolated && build_cic(H, l, err) != AMG_OK) {
      // the interface conditions its face data may come from: a window off
      // the coarse level makes only amg_cic_face_data unavailable
      L.cic = CicTable();
      L.cic.err = err;
    }
    if (rc != AMG_OK) return fail(H, rc, err);
  }
  HIPCHK(hipStreamCreate(&H->own));
  tail_prepare();
  {
    double* sp = nullptr;  // the allocation-free entry point's scratch on this device
    HIPCHK(scratch_address(&sp));
  }
  for (int l = 0; l < H->nlevels; ++l) {
    Level& L = H->levels[l];
    const std::vector<double>& mats_l = mats[l];
    const std::vector<int64_t>& idx = idxs[l];
    TRY(upload(H, &L.d_mat, mats_l));
    L.nmat = mats_l.size();
    TRY(upload(H, &L.d_idx, idx));
    if (L.ngws > 0) TRY(zalloc(H, &L.d_gws, L.ngws));
    size_t maxpart = 1, maxseg = 1;
    for (auto& D : L.depths) {
      TRY(upload(H, &D.d_box, D.boxd));
      TRY(upload(H, &D.d_codes, D.codes));
      TRY(upload(H, &D.d_xsrc, D.xsrc));
      TRY(upload(H, &D.d_chunks, D.chunks));
      TRY(upload(H, &D.d_tiles, D.tiles));
      TRY(upload(H, &D.d_stiles, D.stiles));
      TRY(upload(H, &D.d_seg, D.seg_ptr));
      TRY(upload(H, &D.d_cseg, D.comp_seg_ptr));
      TRY(upload(H, &D.d_cc_ptr, D.chunk_comp_ptr));
      TRY(upload(H, &D.d_cc_idx, D.chunk_comp_idx));
      TRY(upload(H, &D.d_groups, D.groups));
      TRY(upload(H, &D.d_band, D.band));
      TRY(zalloc(H, &D.e64, D.nstored));
      TRY(zalloc(H, &D.f64, D.nstored));
      TRY(zalloc(H, &D.t64, D.nstored));
      TRY(zalloc(H, &D.e32, D.nstored));
      TRY(zalloc(H, &D.f32, D.nstored));
      TRY(zalloc(H, &D.t32, D.nstored));
      if (D.split_rb) TRY(zalloc(H, &D.fs32, D.nstored));
      if (D.split_rb) TRY(zalloc(H, &D.xg32, std::max<int64_t>(D.nxg, 1)));
      maxpart = std::max(maxpart, std::max(D.tiles.size(), D.chunks.size()));
      maxseg = std::max(maxseg, D.seg_ptr.size());
    }
    TRY(zalloc(H, &L.r64, L.depths[0].nstored));
    TRY(zalloc(H, &L.fsh, L.depths[0].nstored));
    TRY(zalloc(H, &L.partial, 2 * maxpart));  // per-tile max and per-tile sum of a residual
    TRY(zalloc(H, &L.partial2, maxseg));
    TRY(zalloc(H, &L.comp_sum, L.ncomp));
    TRY(zalloc(H, &L.d_delta, L.ncomp));
    TRY(zalloc(H, &L.d_delta0, L.ncomp));
    TRY(zalloc(H, &L.d_bsum, L.ncomp));
    TRY(zalloc(H, &L.d_defect, L.ncomp));
    TRY(zalloc(H, &L.d_dfd, L.ncomp));
    TRY(zalloc(H, &L.fdc, (size_t)std::max<int64_t>(L.nface, 1)));
    TRY(upload(H, &L.d_comp_ncf, L.comp_ncf));
    TRY(upload(H, &L.d_comp_flag, L.comp_singular));
    std::vector<double> cnt((size_t)L.depths.size() * L.ncomp);
    for (size_t k = 0; k < L.depths.size(); ++k)
      for (int c = 0; c < L.ncomp; ++c)
        cnt[k * L.ncomp + c] = (double)L.comp_cells[c] / std::pow(2.0, (double)(H->dim * k));
    TRY(upload(H, &L.d_comp_cnt, cnt));
    std::vector<double> sc(S_COUNT, 0.0);
    sc[S_ONE] = 1.0;
    TRY(upload(H, &L.scal, sc));
    HIPCHK(hipHostMalloc((void**)&L.h_scal, S_COUNT * sizeof(double), hipHostMallocDefault));
    TRY(zalloc(H, &L.E64, L.depths[0].nstored));
    TRY(zalloc(H, &L.A64, L.depths[0].nstored));
    {
      Depth& D0 = L.depths[0];
      TRY(upload(H, &D0.d_exT_elem, D0.exT_elem));
      TRY(upload(H, &D0.d_exT_slot, D0.exT_slot));
      TRY(upload(H, &D0.d_exT_ptr, D0.exT_ptr));
    }
  }
  // interface-condition tables of the face-data levels
  for (int l = 1; l < H->nlevels; ++l) {
    CicTable& T = H->levels[l].cic;
    if (T.fd.empty()) continue;
    std::vector<double> w(&T.w[0][0], &T.w[0][0] + 100);
    TRY(upload(H, &T.d_w, w));
    TRY(upload(H, &T.d_fd, T.fd));
    TRY(upload(H, &T.d_src, T.src));
    TRY(upload(H, &T.d_wsel, T.wsel));
    TRY(upload(H, &T.d_ncf, T.ncf));
    TRY(zalloc(H, &T.d_sum, (size_t)H->levels[l].ncomp));
  }
  // composite tables of every interpolated level against the one below
  for (int l = 1; l < H->nlevels; ++l) {
    Level& L = H->levels[l];
    if (L.cf_mode != AMG_CF_INTERP) continue;
    Composite& X = L.cmp;
    std::vector<double> w(&X.w[0][0], &X.w[0][0] + 100);
    TRY(upload(H, &X.d_w, w));
    TRY(upload(H, &X.d_cfi_dst, X.cfi_dst));
    TRY(upload(H, &X.d_cfi_src, X.cfi_src));
    TRY(upload(H, &X.d_cfi_w, X.cfi_w));
    TRY(upload(H, &X.d_avg, X.avg));
    TRY(upload(H, &X.d_rfx_cell, X.rfx_cell));
    TRY(upload(H, &X.d_rfx_ptr, X.rfx_ptr));
    TRY(upload(H, &X.d_rfx_face, X.rfx_face));
    TRY(upload(H, &X.d_pro, X.pro));
    TRY(upload(H, &X.d_cfi_e0, X.cfi_e0));
    TRY(upload(H, &X.d_cfi_in, X.cfi_in));
    TRY(upload(H, &X.d_cfi_layer, X.cfi_layer));
    TRY(upload(H, &X.d_cfiT_elem, X.cfiT_elem));
    TRY(upload(H, &X.d_cfiT_ptr, X.cfiT_ptr));
    TRY(upload(H, &X.d_cfiT_ent, X.cfiT_ent));
    TRY(upload(H, &X.d_rfxTc_elem, X.rfxTc_elem));
    TRY(upload(H, &X.d_rfxTc_ptr, X.rfxTc_ptr));
    TRY(upload(H, &X.d_rfxTc_src, X.rfxTc_src));
    TRY(upload(H, &X.d_rfxTc_coef, X.rfxTc_coef));
    TRY(upload(H, &X.d_rfxTf_elem, X.rfxTf_elem));
    TRY(upload(H, &X.d_rfxTf_ptr, X.rfxTf_ptr));
    TRY(upload(H, &X.d_rfxTf_src, X.rfxTf_src));
    TRY(upload(H, &X.d_rfxTf_coef, X.rfxTf_coef));
    for (int d = 0; d < H->dim; ++d)
      for (Composite::GatherT* t : {&X.rfxVc[d], &X.rfxVf[d]}) {
        TRY(upload(H, &t->d_elem, t->elem));
        TRY(upload(H, &t->d_ptr, t->ptr));
        TRY(upload(H, &t->d_src, t->src));
        TRY(upload(H, &t->d_coef, t->coef));
      }
    TRY(zalloc(H, &L.mu, X.cfi_dst.size()));
  }
  for (auto& L : H->levels) TRY(upload(H, &L.d_face_valid, L.face_valid));
  H->finalized = true;
  return AMG_OK;
}

int amg_level_info(const amg_hier* Hc, int level, amg_level_desc* out) {
  amg_hier* H = const_cast<amg_hier*>(Hc);
  if (!out || !check_level(H, level)) return AMG_EINVAL;
  const Level& L = H->levels[level];
  out->nboxes = (int32_t)L.boxes.size();
  out->depths = (int32_t)L.depths.size();
  out->ncomp = L.ncomp;
  out->nsingular = L.nsingular;
  out->ncells = L.ncells;
  out->nstored = L.depths[0].nstored;
  out->nface = L.nface;
  out->split_rb = L.depths[0].split_rb ? 1 : 0;
  {
    Run R{H, const_cast<Level*>(&L), H->dim, H->own};
    amg_solve_opts o;
    amg_default_opts(&o);
    out->tail_depth = tail_start(R, o);
  }
  return AMG_OK;
}

int amg_depth_size(const amg_hier* Hc, int level, int depth, int64_t* nstored, int32_t* nboxes) {
  amg_hier* H = const_cast<amg_hier*>(Hc);
  if (!check_level(H, level)) return AMG_EINVAL;
  const Level& L = H->levels[level];
  if (depth < 0 || depth >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  if (nstored) *nstored = L.depths[depth].nstored;
  if (nboxes) *nboxes = (int32_t)L.depths[depth].boxes.size();
  return AMG_OK;
}

int amg_box_info(const amg_hier* Hc, int level, int depth, int box, amg_box_desc* out) {
  amg_hier* H = const_cast<amg_hier*>(Hc);
  if (!out || !check_level(H, level)) return AMG_EINVAL;
  const Level& L = H->levels[level];
  if (depth < 0 || depth >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  const Depth& D = L.depths[depth];
  if (box < 0 || box >= (int)D.boxes.size()) return fail(H, AMG_EINVAL, "box out of range");
  memset(out, 0, sizeof *out);
  const BoxD& X = D.boxd[box];
  for (int d = 0; d < 3; ++d) {
    out->lo[d] = D.boxes[box].lo[d];
    out->hi[d] = D.boxes[box].hi[d];
    out->stride[d] = X.s[d];
    for (int s = 0; s < 2; ++s)
      out->face_offset[d][s] = (depth == 0 && d < H->dim) ? L.face_off[D.level_box[box] * 6 + d * 2 + s] : -1;
  }
  if (H->dim == 2) out->stride[2] = 0;
  out->offset = X.off;
  out->comp = X.comp;
  out->singular = L.comp_singular[X.comp];
  return AMG_OK;
}

int amg_apply_operator(amg_hier* H, int level, double* x, const double* face_data, double* y, int homogeneous,
                       void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!x || !y) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  Depth& D = L.depths[0];
  hipStream_t st = stream_of(H, stream);
  double alpha, beta;
  coefs<double>(H, D, alpha, beta);
  launch_fill<double>(D, x, homogeneous ? nullptr : face_data, st);
  launch_residual<double>(H->dim, D, true, x, nullptr, y, alpha, beta, nullptr, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_fill_ghosts(amg_hier* H, int level, int depth, int dtype, void* u, const double* face_data, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!u) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  if (depth < 0 || depth >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  if (depth > 0 && face_data) return fail(H, AMG_EINVAL, "face data only at depth 0");
  hipStream_t st = stream_of(H, stream);
  if (dtype == AMG_F64)
    launch_fill<double>(L.depths[depth], (double*)u, face_data, st);
  else
    launch_fill<float>(L.depths[depth], (float*)u, face_data, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_residual(amg_hier* H, int level, int depth, int dtype, const void* u, const void* f, void* r, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!u || !r) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  if (depth < 0 || depth >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  hipStream_t st = stream_of(H, stream);
  Depth& D = L.depths[depth];
  if (dtype == AMG_F64) {
    double a, b;
    coefs<double>(H, D, a, b);
    launch_residual<double>(H->dim, D, true, (const double*)u, (const double*)f, (double*)r, a, b, nullptr, st);
  } else {
    float a, b;
    coefs<float>(H, D, a, b);
    launch_residual<float>(H->dim, D, true, (const float*)u, (const float*)f, (float*)r, a, b, nullptr, st);
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_smooth(amg_hier* H, int level, int depth, int dtype, int smoother, int nsweeps, double omega, void* u,
               const void* f, void* tmp, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!u || !f || !tmp) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  if (depth < 0 || depth >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  if (smoother != AMG_SMOOTH_JACOBI && smoother != AMG_SMOOTH_RB) return fail(H, AMG_EINVAL, "bad smoother");
  Run R{H, &L, H->dim, stream_of(H, stream)};
  const size_t bytes = L.depths[depth].nstored * (dtype == AMG_F64 ? 8 : 4);
  if (dtype == AMG_F64) {
    double *cur = (double*)u, *oth = (double*)tmp;
    smooth<double>(R, depth, smoother, nsweeps, omega, false, cur, oth, (const double*)f);
    if (cur != u) HIPCHK(hipMemcpyAsync(u, cur, bytes, hipMemcpyDeviceToDevice, R.st));
  } else {
    float *cur = (float*)u, *oth = (float*)tmp;
    smooth<float>(R, depth, smoother, nsweeps, omega, false, cur, oth, (const float*)f);
    if (cur != u) HIPCHK(hipMemcpyAsync(u, cur, bytes, hipMemcpyDeviceToDevice, R.st));
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_restrict(amg_hier* H, int level, int depth, int dtype, const void* r, void* fc, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!r || !fc) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  if (depth < 0 || depth + 1 >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  hipStream_t st = stream_of(H, stream);
  if (dtype == AMG_F64)
    launch_restrict<double>(H->dim, L.depths[depth], L.depths[depth + 1], (const double*)r, (double*)fc, st);
  else
    launch_restrict<float>(H->dim, L.depths[depth], L.depths[depth + 1], (const float*)r, (float*)fc, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_prolong(amg_hier* H, int level, int depth, int dtype, const void* ec, void* u, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!ec || !u) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  if (depth < 0 || depth + 1 >= (int)L.depths.size()) return fail(H, AMG_EINVAL, "depth out of range");
  hipStream_t st = stream_of(H, stream);
  if (dtype == AMG_F64)
    launch_prolong<double>(H->dim, L.depths[depth], L.depths[depth + 1], (const double*)ec, (double*)u, st);
  else
    launch_prolong<float>(H->dim, L.depths[depth], L.depths[depth + 1], (const float*)ec, (float*)u, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_bottom(amg_hier* H, int level, int dtype, const void* f, void* e, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!f || !e) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  if (L.isolated && L.depths.size() > 1) {
    for (size_t k = 0; k + 1 < L.depths.size(); ++k)
      if (!L.depths[k].groups.empty()) return fail(H, AMG_EUNSUPPORTED, "boxes of this level end at several depths");
  }
  Depth& D = L.depths.back();
  hipStream_t st = stream_of(H, stream);
  const bool gm = H->bottom_kind == AMG_BOTTOM_ILU_GMRES;
  if (dtype == AMG_F64) {
    if (gm)
      launch_bottom_gmres<double>(D, L.d_mat, L.d_idx, (const double*)f, (double*)e, H->bottom_iters, L.d_gws, st);
    else
      launch_bottom<double>(D, L.d_mat, L.d_idx, (const double*)f, (double*)e, false, st);
  } else {
    if (gm)
      launch_bottom_gmres<float>(D, L.d_mat, L.d_idx, (const float*)f, (float*)e, H->bottom_iters, L.d_gws, st);
    else
      launch_bottom<float>(D, L.d_mat, L.d_idx, (const float*)f, (float*)e, false, st);
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_vcycle(amg_hier* H, int level, int dtype, const amg_solve_opts* opts, const void* f, void* e, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!f || !e) return fail(H, AMG_EINVAL, "bad arguments");
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  Level& L = H->levels[level];
  Run R{H, &L, H->dim, stream_of(H, stream)};
  Depth& D0 = L.depths[0];
  if (dtype == AMG_F64) {
    double* res = vcycle<double>(R, o, (const double*)f, (double*)e, D0.t64);
    if (res != e) HIPCHK(hipMemcpyAsync(e, res, D0.nstored * 8, hipMemcpyDeviceToDevice, R.st));
  } else {
    float* res = vcycle<float>(R, o, (const float*)f, (float*)e, D0.t32);
    if (res != e) HIPCHK(hipMemcpyAsync(e, res, D0.nstored * 4, hipMemcpyDeviceToDevice, R.st));
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

static int check_opts(amg_hier* H, const amg_solve_opts& o) {
  if (o.nu1 < 0 || o.nu2 < 0 || o.max_cycles < 0 || o.max_cycles > 100000 ||
      (o.smoother != AMG_SMOOTH_JACOBI && o.smoother != AMG_SMOOTH_RB) ||
      (o.precision != AMG_FP64 && o.precision != AMG_MIXED) || !(o.omega > 0) ||
      !(o.omega_rb > 0 && o.omega_rb < 2) ||
      (o.solvability != AMG_SOLV_RHS_SHIFT && o.solvability != AMG_SOLV_OFF && o.solvability != AMG_SOLV_CF_DELTA))
    return fail(H, AMG_EINVAL, "bad solve options");
  return AMG_OK;
}

static int make_comp(amg_hier* H, int lev_lo, int lev_hi, double* const* x, const double* const* f,
                     const double* const* face_data, void* stream, Comp& C) {
  if (lev_lo != 0) return fail(H, AMG_EUNSUPPORTED, "a composite solve starts at level 0");
  if (lev_hi < 1 || lev_hi >= H->nlevels) return fail(H, AMG_EINVAL, "level out of range");
  for (int l = 1; l <= lev_hi; ++l)
    if (H->levels[l].cf_mode != AMG_CF_INTERP)
      return fail(H, AMG_EINVAL, "levels of a composite solve take interpolated coarse-fine ghosts");
  C.H = H;
  C.hi = lev_hi;
  C.st = stream_of(H, stream);
  for (int l = 0; l <= lev_hi; ++l) {
    if (!x[l] || !f[l]) return fail(H, AMG_EINVAL, "null x or f");
    C.X.push_back(x[l]);
    C.F.push_back(f[l]);
    C.FD.push_back(face_data ? face_data[l] : nullptr);
    C.R.push_back(H->levels[l].r64);
  }
  return AMG_OK;
}

// Prepares the replay of one composite cycle (body) from a HIP graph
// captured on C.st, keyed on everything its launches bake in: the levels'
// buffers and the options (the coefficient and the timer release the graph
// when they change).  Returns false when the cycle is to run as direct
// launches (graphs off, timing on, or a capture that failed once).
static bool comp_graph_ready(amg_hier* H, GraphCache& G, const Comp& C, const amg_solve_opts& o,
                             const std::function<void()>& body) {
  if (o.use_graph == 0 || G.broken || H->timer.on) return false;
  std::vector<int64_t> key = {(int64_t)C.hi, o.precision, o.smoother, o.nu1, o.nu2, (int64_t)C.tr};
  int64_t ob;
  memcpy(&ob, &o.omega, sizeof ob);
  key.push_back(ob);
  memcpy(&ob, &o.omega_rb, sizeof ob);
  key.push_back(ob);
  for (int l = 0; l <= C.hi; ++l) {
    key.push_back((int64_t)(intptr_t)C.X[l]);
    key.push_back((int64_t)(intptr_t)C.R[l]);
    key.push_back((int64_t)(intptr_t)C.F[l]);
    key.push_back((int64_t)(intptr_t)C.FD[l]);
  }
  if (G.exec && G.key == key) return true;
  G.release();
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(C.st, hipStreamCaptureModeRelaxed);
  if (e == hipSuccess) {
    body();
    e = hipStreamEndCapture(C.st, &g);
  }
  hipGraphExec_t ex = nullptr;
  if (e == hipSuccess && g) e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess || !ex) {
    (void)hipGetLastError();
    if (g) (void)hipGraphDestroy(g);
    G.broken = true;  // direct launches from now on
    return false;
  }
  G.graph = g;
  G.exec = ex;
  G.key = key;
  return true;
}

static int composite_solve(amg_hier* H, int lev_lo, int lev_hi, double* const* x, const double* const* f,
                           const double* const* face_data, const amg_solve_opts* opts, amg_solve_stats* stats,
                           void* stream) {
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(H, o));
  Comp C;
  TRY(make_comp(H, lev_lo, lev_hi, x, f, face_data, stream, C));
  const int dim = H->dim;
  Level& L0 = H->levels[0];
  if (stats) memset(stats, 0, sizeof *stats);
  double comp_defect_mean = 0.0;
  // solvability of the pure-Neumann composite problem: one constant shift of
  // the right-hand side on every level (sums over valid cells and over the
  // physical faces of valid cells)
  if (L0.nsingular) {
    for (int l = 0; l <= C.hi; ++l)
      HIPCHK(hipMemcpyAsync(H->levels[l].fsh, C.F[l], H->levels[l].depths[0].nstored * sizeof(double),
                            hipMemcpyDeviceToDevice, C.st));
    for (int l = C.hi; l >= 1; --l) launch_avgdown(dim, H->levels[l].cmp, H->levels[l].fsh, H->levels[l - 1].fsh, C.st);
    Run R0{H, &L0, dim, C.st};
    launch_tile_sum<double>(dim, L0.depths[0], L0.fsh, L0.partial, C.st);
    comp_sums(R0, L0.depths[0], L0.scal + S_FSUM);
    for (int l = 0; l <= C.hi; ++l) {
      Level& L = H->levels[l];
      Depth& D = L.depths[0];
      if (C.FD[l] && !D.chunks.empty()) {
        launch_chunk_fdsum(D, C.FD[l], l < H->nlevels - 1 && l < C.hi ? L.d_face_valid : nullptr, L.partial, C.st);
        launch_seg_reduce(L.partial, nullptr, 1, (int)D.chunks.size(), L0.scal + S_FD + l, false, C.st);
      } else {
        launch_zero<double>(L0.scal + S_FD + l, 1, C.st);
      }
    }
    std::vector<double> hs(S_COUNT);
    HIPCHK(hipMemcpyAsync(hs.data(), L0.scal, S_COUNT * sizeof(double), hipMemcpyDeviceToHost, C.st));
    HIPCHK(hipStreamSynchronize(C.st));
    const double h0 = L0.depths[0].h;
    double g = 0.0;
    for (int l = 0; l <= C.hi; ++l) g += hs[S_FD + l] * std::pow(H->levels[l].depths[0].h, dim - 1);
    const double defect = hs[S_FSUM] * std::pow(h0, dim) - g;
    const double vol = (double)L0.ncells * std::pow(h0, dim);
    if (stats) {
      stats->ncomp = 1;
      stats->defect[0] = defect;
    }
    comp_defect_mean = std::fabs(defect) / vol;
    if (o.solvability != AMG_SOLV_OFF) {
      L0.h_scal[0] = defect / vol;
      HIPCHK(hipMemcpyAsync(L0.scal + S_DELTA, L0.h_scal, sizeof(double), hipMemcpyHostToDevice, C.st));
      for (int l = 0; l <= C.hi; ++l) {
        HIPCHK(hipMemcpyAsync(H->levels[l].fsh, C.F[l], H->levels[l].depths[0].nstored * sizeof(double),
                              hipMemcpyDeviceToDevice, C.st));
        launch_sub_scalar(dim, H->levels[l].depths[0], H->levels[l].fsh, L0.scal + S_DELTA, C.st);
        C.F[l] = H->levels[l].fsh;
      }
    }
  }
  auto read_norm = [&](double& v) -> int {
    HIPCHK(hipMemcpyAsync(L0.h_scal, L0.scal + S_NORM, sizeof(double), hipMemcpyDeviceToHost, C.st));
    HIPCHK(hipStreamSynchronize(C.st));
    v = L0.h_scal[0];
    return AMG_OK;
  };
  comp_residual(C);
  HIPCHK(hipGetLastError());
  double r0 = 0;
  TRY(read_norm(r0));
  if (!std::isfinite(r0)) return fail(H, AMG_ENONFINITE, "non-finite initial residual");
  const double target = std::max(o.tol_rel * r0, o.tol_abs);
  double rn = r0;
  int cycles = 0;
  if (stats) {
    stats->r0 = r0;
    stats->history[0] = r0;
  }
  // unenforced solvability: the volume-weighted mean of the composite
  // residual is defect / volume whatever x is (see level_solve)
  if (L0.nsingular && o.solvability == AMG_SOLV_OFF && comp_defect_mean > target) {
    char buf[160];
    snprintf(buf, sizeof buf, "mean defect %.3e exceeds the stopping target %.3e", comp_defect_mean, target);
    return fail(H, AMG_ESOLVABILITY, buf);
  }
  // the cycle is captured once into a HIP graph and replayed
  const bool use_graph = comp_graph_ready(H, H->comp_graph, C, o, [&]() { comp_cycle(C, o); });
  while (rn > target && cycles < o.max_cycles) {
    if (use_graph)
      HIPCHK(hipGraphLaunch(H->comp_graph.exec, C.st));
    else
      comp_cycle(C, o);
    HIPCHK(hipGetLastError());
    TRY(read_norm(rn));
    ++cycles;
    if (stats && cycles < AMG_MAX_HISTORY) stats->history[cycles] = rn;
    if (!std::isfinite(rn)) return fail(H, AMG_ENONFINITE, "non-finite residual");
  }
  if (stats) {
    stats->cycles = cycles;
    stats->rfinal = rn;
    stats->converged = rn <= target;
    stats->used_graph = use_graph && cycles > 0;
  }
  if (rn > target) return fail(H, AMG_ENOTCONVERGED, "max_cycles reached");
  return AMG_OK;
}

int amg_composite_residual(amg_hier* H, int lev_hi, double* const* x, const double* const* f,
                           const double* const* face_data, double* const* r, void* stream) {
  if (!H || !H->finalized) return fail(H, AMG_EINVAL, "amg_finalize has not been called");
  if (!x || !f || !r) return fail(H, AMG_EINVAL, "bad arguments");
  Comp C;
  TRY(make_comp(H, 0, lev_hi, x, f, face_data, stream, C));
  for (int l = 0; l <= lev_hi; ++l) {
    if (!r[l]) return fail(H, AMG_EINVAL, "null r");
    C.R[l] = r[l];
  }
  comp_residual(C);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

// the outer loop of a level solve (tr: of the adjoint system, homogeneous)
static int level_solve(amg_hier* H, int l, double* X, const double* F, const double* FD, const amg_solve_opts& o,
                       amg_solve_stats* stats, void* stream, bool tr) {
  Level& L = H->levels[l];
  if (l > 0 && L.cf_mode == AMG_CF_INTERP)
    return fail(H, AMG_EUNSUPPORTED, "a level with interpolated coarse-fine ghosts is solved in a composite solve");
  if (!X || !F) return fail(H, AMG_EINVAL, "null x or f");
  Run R{H, &L, H->dim, stream_of(H, stream), tr};
  Depth& D0 = L.depths[0];
  const int dim = H->dim;
  const double hD = std::pow(D0.h, dim), hD1 = std::pow(D0.h, dim - 1);
  if (stats) memset(stats, 0, sizeof *stats);

  // ---- solvability: defect per singular component and the RHS shift ----
  const double* frhs = F;
  if (L.nsingular) {
    launch_tile_sum<double>(dim, D0, F, L.partial, R.st);
    comp_sums(R, D0, L.comp_sum);
    const double* bsum = nullptr;
    if (FD) {
      launch_chunk_fdsum(D0, FD, nullptr, L.partial, R.st);
      launch_comp_sum(L.partial, D0.d_cc_ptr, D0.d_cc_idx, L.ncomp, L.d_bsum, R.st);
      bsum = L.d_bsum;
    }
    launch_comp_delta(L.comp_sum, bsum, L.d_comp_flag, L.d_comp_cnt, L.ncomp, hD, hD1, L.d_delta, L.d_defect, R.st);
    if (o.solvability == AMG_SOLV_CF_DELTA && !tr) {
      // eq. (correctingFaceAvg): the face data of coarse-fine Neumann faces
      // take the correction, the right-hand side only where there are none
      launch_cf_delta(L.d_defect, L.d_comp_flag, L.d_comp_ncf, L.d_comp_cnt, L.ncomp, hD, hD1, L.d_delta, L.d_dfd,
                      R.st);
      launch_fd_correct(D0, FD, L.d_dfd, L.fdc, R.st);
      FD = L.fdc;
    }
    if (o.solvability == AMG_SOLV_RHS_SHIFT || o.solvability == AMG_SOLV_CF_DELTA) {
      launch_shift_copy(dim, D0, F, L.fsh, L.d_delta, R.st);
      frhs = L.fsh;
    }
    if (stats) {
      std::vector<double> df(L.ncomp);
      HIPCHK(hipMemcpyAsync(df.data(), L.d_defect, L.ncomp * sizeof(double), hipMemcpyDeviceToHost, R.st));
      HIPCHK(hipStreamSynchronize(R.st));
      int j = 0;
      for (int c = 0; c < L.ncomp && j < AMG_MAX_COMP; ++c)
        if (L.comp_singular[c]) stats->defect[j++] = df[c];
      stats->ncomp = j;
    }
  }

  const bool mixed = o.precision == AMG_MIXED;
  double* Rb = mixed ? L.r64 : D0.f64;
  double alpha, beta;
  coefs<double>(H, D0, alpha, beta);
  // mixed precision: the residual kernel stores r in FP32 directly (the
  // conversion then scales it in place), unless its size is outside the
  // range where FP32 holds it comfortably
  bool direct32 = mixed && !tr;
  const bool split = mixed && !tr && use_split(H, D0, o);
  auto residual_norm = [&]() {
    if (tr) {
      launch_fill_tr<double>(D0, X, R.st);
      launch_residual<double>(dim, D0, true, X, frhs, Rb, alpha, beta, nullptr, R.st);
      launch_band<double>(dim, D0, 0, X, Rb, alpha, beta, -beta, 0, R.st);
      launch_tile_absmax<double>(dim, D0, Rb, L.partial, R.st);
    } else {
      // without face data on uniformly filled faces the residual kernel
      // writes the (homogeneous) ghosts of x it reads itself
      const int rgr = (direct32 && !FD && D0.wrap_fill) ? 1 : 0;
      if (!rgr) launch_fill<double>(D0, X, FD, R.st);
      Timed tm(R, AMG_T_RESIDUAL, 0);
      if (direct32)
        launch_residual32(dim, D0, X, frhs, split ? D0.fs32 : D0.f32, alpha, beta, L.partial, R.st, split, rgr);
      else
        launch_residual<double>(dim, D0, true, X, frhs, Rb, alpha, beta, L.partial, R.st);
    }
    global_max(R, D0, L.scal + S_NORM, L.h_scal);  // the host reads it after each cycle
  };
  // the norm kernel also stores the norm into h_scal[0] (pinned host
  // memory, system scope): no copy, only the wait
  auto read_norm = [&](double& v) -> int {
    HIPCHK(hipStreamSynchronize(R.st));
    v = L.h_scal[0];
    return AMG_OK;
  };
  residual_norm();
  HIPCHK(hipGetLastError());
  double r0 = 0;
  TRY(read_norm(r0));
  if (direct32 && std::isfinite(r0) && !(r0 > 1e-20 && r0 < 1e30)) {
    direct32 = false;
    residual_norm();
    TRY(read_norm(r0));
  }
  if (!std::isfinite(r0)) return fail(H, AMG_ENONFINITE, "non-finite initial residual");
  const double target = std::max(o.tol_rel * r0, o.tol_abs);
  double rn = r0;
  int cycles = 0;
  if (stats) {
    stats->r0 = r0;
    stats->history[0] = r0;
  }
  // Without enforcement the residual keeps the mean defect / (|c| h^D) on a
  // singular component c whatever x is (the discrete divergence theorem of
  // eq. velocity_disc_solvabilityCond), so a mean above the target can never
  // be reached.
  if (!tr && L.nsingular && o.solvability == AMG_SOLV_OFF) {
    std::vector<double> df(L.ncomp);
    HIPCHK(hipMemcpyAsync(df.data(), L.d_defect, L.ncomp * sizeof(double), hipMemcpyDeviceToHost, R.st));
    HIPCHK(hipStreamSynchronize(R.st));
    for (int c = 0; c < L.ncomp; ++c) {
      if (!L.comp_singular[c]) continue;
      const double m = std::fabs(df[c]) / ((double)L.comp_cells[c] * hD);
      if (m > target) {
        char buf[160];
        snprintf(buf, sizeof buf, "component %d: mean defect %.3e exceeds the stopping target %.3e", c, m, target);
        return fail(H, AMG_ESOLVABILITY, buf);
      }
    }
  }
  // one outer cycle: r -> V-cycle -> x += s e -> new residual and its norm
  // per-component means of the residual: from the per-tile sums the
  // residual kernel wrote next to its maxima (the transposed residual has
  // none: a separate sum pass)
  auto residual_mean = [&]() {
    if (tr) {
      launch_tile_sum<double>(dim, D0, Rb, L.partial, R.st);
      comp_sums(R, D0, L.comp_sum);
      launch_comp_delta(L.comp_sum, nullptr, L.d_comp_flag, L.d_comp_cnt, L.ncomp, 1.0, 0.0, L.d_delta0, nullptr,
                        R.st);
    } else {
      launch_comp_mean_delta(D0, L.partial + D0.tiles.size(), L.d_comp_flag, L.d_comp_cnt, L.ncomp, L.d_delta0, R.st);
    }
  };
  // The solution's mean on singular components does not change the
  // residual (the operator annihilates constants), so it is removed once
  // after the loop rather than after every cycle.
  auto body = [&]() {
    if (L.nsingular) residual_mean();
    if (mixed) {
      // the mean removal fused into the FP32 conversion
      // with depth 0 in split storage the residual kernel has stored r split
      // and the split kernels scale it as they read it (no conversion pass);
      // from the FP64 residual the conversion writes f split, scaled
      float* fs = split ? D0.fs32 : nullptr;
      const double* fsc = nullptr;
      const double* fdl = nullptr;
      if (direct32 && split) {
        fsc = L.scal + S_NORM;
        fdl = L.nsingular ? L.d_delta0 : nullptr;
      } else if (direct32) {
        launch_scale32(dim, D0, D0.f32, L.scal + S_NORM, R.st, L.nsingular ? L.d_delta0 : nullptr);
      } else {
        launch_to32(dim, D0, Rb, D0.f32, L.scal + S_NORM, R.st, L.nsingular ? L.d_delta0 : nullptr, fs);
      }
      // in split storage the V-cycle's last half-sweep applies x += s e
      float* e = vcycle<float>(R, o, D0.f32, D0.e32, D0.t32, fs, fsc, fdl, split ? X : nullptr,
                               split ? L.scal + S_NORM : nullptr);
      if (e) launch_update<float>(dim, D0, X, e, L.scal + S_NORM, R.st);
    } else {
      if (L.nsingular) launch_comp_shift<double>(dim, D0, Rb, L.d_delta0, R.st);
      double* e = vcycle<double>(R, o, D0.f64, D0.e64, D0.t64);
      launch_update<double>(dim, D0, X, e, L.scal + S_ONE, R.st);
    }
    residual_norm();
  };
  // the cycle is captured once into a HIP graph and replayed
  GraphCache& G = tr ? L.graphT : L.graph;
  // event timing needs per-launch events, which a replayed graph does not
  // provide: with timing on, the cycle runs as direct launches
  bool use_graph = o.use_graph != 0 && !G.broken && !H->timer.on;
  if (use_graph) {
    std::vector<int64_t> key = {(int64_t)direct32, (int64_t)(intptr_t)X, (int64_t)(intptr_t)frhs,
                                (int64_t)(intptr_t)FD, o.precision,
                                o.smoother, o.nu1, o.nu2, (int64_t)H->timer.on};
    int64_t ob;
    memcpy(&ob, &o.omega, sizeof ob);
    key.push_back(ob);
    memcpy(&ob, &o.omega_rb, sizeof ob);
    key.push_back(ob);
    if (!G.exec || G.key != key) {
      G.release();
      Timer& T = H->timer;
      const size_t p0 = T.pending.size();
      hipGraph_t g = nullptr;
      hipError_t e1 = hipStreamBeginCapture(R.st, hipStreamCaptureModeRelaxed);
      if (e1 == hipSuccess) {
        body();
        e1 = hipStreamEndCapture(R.st, &g);
      }
      hipGraphExec_t ex = nullptr;
      if (e1 == hipSuccess && g) e1 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
      if (e1 != hipSuccess || !ex) {
        (void)hipGetLastError();
        if (g) (void)hipGraphDestroy(g);
        G.broken = true;  // fall back to direct launches from now on
        use_graph = false;
        T.pending.resize(p0);
        T.next = T.base;
      } else {
        G.graph = g;
        G.exec = ex;
        G.key = key;
        // event pairs captured into the graph are re-recorded by every replay
        G.timed.assign(T.pending.begin() + p0, T.pending.end());
        T.pending.resize(p0);
        T.base = T.next;
      }
    }
  }
  while (rn > target && cycles < o.max_cycles) {
    if (use_graph)
      HIPCHK(hipGraphLaunch(G.exec, R.st));
    else
      body();
    HIPCHK(hipGetLastError());
    TRY(read_norm(rn));
    if (use_graph && H->timer.on) accumulate(H->timer, G.timed);
    ++cycles;
    if (stats && cycles < AMG_MAX_HISTORY) stats->history[cycles] = rn;
    if (!std::isfinite(rn)) return fail(H, AMG_ENONFINITE, "non-finite residual");
  }
  if (stats) {
    stats->cycles = cycles;
    stats->rfinal = rn;
    stats->converged = rn <= target;
    stats->used_graph = use_graph && cycles > 0;
  }
  if (H->timer.on) collect_timing(H->timer);
  remove_mean<double>(R, 0, X);
  if (tr)  // the adjoint solution as a gradient: zero outside the cells
    launch_fill_zero<double>(D0, X, R.st);
  else  // the residual kernels need not leave every ghost of x written, and
        // the mean shift moves the cells: ghosts of the returned solution
    launch_fill<double>(D0, X, FD, R.st);
  HIPCHK(hipGetLastError());
  if (rn > target) return fail(H, AMG_ENOTCONVERGED, "max_cycles reached");
  return AMG_OK;
}

int amg_solve(amg_hier* H, int lev_lo, int lev_hi, double* const* x, const double* const* f,
              const double* const* face_data, const amg_solve_opts* opts, amg_solve_stats* stats, void* stream) {
  if (!check_level(H, lev_lo)) return AMG_EINVAL;
  if (!x || !f) return fail(H, AMG_EINVAL, "bad arguments");
  if (lev_hi != lev_lo) return composite_solve(H, lev_lo, lev_hi, x, f, face_data, opts, stats, stream);
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(H, o));
  return level_solve(H, lev_lo, x[lev_lo], f[lev_lo], face_data ? face_data[lev_lo] : nullptr, o, stats, stream,
                     false);
}

int amg_solve_adjoint(amg_hier* H, int level, double* lam, const double* g, const amg_solve_opts* opts,
                      amg_solve_stats* stats, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!lam || !g) return fail(H, AMG_EINVAL, "bad arguments");
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(H, o));
  return level_solve(H, level, lam, g, nullptr, o, stats, stream, true);
}

int amg_composite_laplacian(amg_hier* H, int lev_hi, double* const* x, const double* const* face_data,
                            double* const* y, void* stream) {
  if (!H || !H->finalized) return fail(H, AMG_EINVAL, "amg_finalize has not been called");
  if (!x || !y) return fail(H, AMG_EINVAL, "bad arguments");
  Comp C;
  TRY(make_comp(H, 0, lev_hi, x, (const double* const*)x, face_data, stream, C));
  C.lap = true;
  for (int l = 0; l <= lev_hi; ++l) {
    if (!y[l] || y[l] == x[l]) return fail(H, AMG_EINVAL, "bad y");
    C.R[l] = y[l];
    C.F[l] = nullptr;
  }
  comp_residual(C);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_composite_residual_adjoint(amg_hier* H, int lev_hi, double* const* lam, const double* const* g,
                                   double* const* r, void* stream) {
  if (!H || !H->finalized) return fail(H, AMG_EINVAL, "amg_finalize has not been called");
  if (!lam || !g || !r) return fail(H, AMG_EINVAL, "bad arguments");
  Comp C;
  TRY(make_comp(H, 0, lev_hi, lam, g, nullptr, stream, C));
  C.tr = true;
  for (int l = 0; l <= lev_hi; ++l) {
    if (!r[l]) return fail(H, AMG_EINVAL, "null r");
    C.R[l] = r[l];
    // the source on the valid cells only
    HIPCHK(hipMemcpyAsync(H->levels[l].fsh, C.F[l], H->levels[l].depths[0].nstored * sizeof(double),
                          hipMemcpyDeviceToDevice, C.st));
    if (l < lev_hi) launch_zero_covered(H->levels[l + 1].cmp, H->levels[l].fsh, C.st);
    C.F[l] = H->levels[l].fsh;
  }
  comp_residual_T(C);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_solve_adjoint_composite(amg_hier* H, int lev_hi, double* const* lam, const double* const* g,
                                const amg_solve_opts* opts, amg_solve_stats* stats, void* stream) {
  if (!H || !H->finalized) return fail(H, AMG_EINVAL, "amg_finalize has not been called");
  if (!lam || !g) return fail(H, AMG_EINVAL, "bad arguments");
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(H, o));
  Comp C;
  TRY(make_comp(H, 0, lev_hi, lam, g, nullptr, stream, C));
  C.tr = true;
  Level& L0 = H->levels[0];
  if (stats) memset(stats, 0, sizeof *stats);
  // the source on the valid cells only (library copy); pure Neumann: its
  // projection along the volume weights
  std::vector<double*> G(C.hi + 1);
  for (int l = 0; l <= C.hi; ++l) {
    G[l] = H->levels[l].fsh;
    HIPCHK(hipMemcpyAsync(G[l], C.F[l], H->levels[l].depths[0].nstored * sizeof(double), hipMemcpyDeviceToDevice,
                          C.st));
  }
  for (int l = 0; l < C.hi; ++l) launch_zero_covered(H->levels[l + 1].cmp, G[l], C.st);
  if (L0.nsingular) proj_w(C, G.data());
  for (int l = 0; l <= C.hi; ++l) C.F[l] = G[l];
  auto read_norm = [&](double& v) -> int {
    HIPCHK(hipMemcpyAsync(L0.h_scal, L0.scal + S_NORM, sizeof(double), hipMemcpyDeviceToHost, C.st));
    HIPCHK(hipStreamSynchronize(C.st));
    v = L0.h_scal[0];
    return AMG_OK;
  };
  comp_residual_T(C);
  HIPCHK(hipGetLastError());
  double r0 = 0;
  TRY(read_norm(r0));
  if (!std::isfinite(r0)) return fail(H, AMG_ENONFINITE, "non-finite initial residual");
  const double target = std::max(o.tol_rel * r0, o.tol_abs);
  double rn = r0;
  int cycles = 0;
  if (stats) {
    stats->r0 = r0;
    stats->history[0] = r0;
  }
  const bool use_graph = comp_graph_ready(H, H->comp_graphT, C, o, [&]() { comp_cycle_T(C, o); });
  while (rn > target && cycles < o.max_cycles) {
    if (use_graph)
      HIPCHK(hipGraphLaunch(H->comp_graphT.exec, C.st));
    else
      comp_cycle_T(C, o);
    HIPCHK(hipGetLastError());
    TRY(read_norm(rn));
    ++cycles;
    if (stats && cycles < AMG_MAX_HISTORY) stats->history[cycles] = rn;
    if (!std::isfinite(rn)) return fail(H, AMG_ENONFINITE, "non-finite residual");
  }
  // the adjoint lives on the valid cells: covered cells and face ghosts 0
  for (int l = 0; l <= C.hi; ++l) {
    if (l < C.hi) launch_zero_covered(H->levels[l + 1].cmp, C.X[l], C.st);
    launch_fill_zero<double>(H->levels[l].depths[0], C.X[l], C.st);
  }
  HIPCHK(hipGetLastError());
  if (stats) {
    stats->cycles = cycles;
    stats->rfinal = rn;
    stats->converged = rn <= target;
    stats->used_graph = use_graph && cycles > 0;
  }
  if (rn > target) return fail(H, AMG_ENOTCONVERGED, "max_cycles reached");
  return AMG_OK;
}

int amg_vcycle_adjoint(amg_hier* H, int level, int dtype, const amg_solve_opts* opts, const void* f, void* e,
                       void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!f || !e) return fail(H, AMG_EINVAL, "bad arguments");
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(H, o));
  Level& L = H->levels[level];
  Run R{H, &L, H->dim, stream_of(H, stream), true};
  Depth& D0 = L.depths[0];
  if (dtype == AMG_F64) {
    double* res = vcycle<double>(R, o, (const double*)f, (double*)e, D0.t64);
    if (res != e) HIPCHK(hipMemcpyAsync(e, res, D0.nstored * 8, hipMemcpyDeviceToDevice, R.st));
  } else {
    float* res = vcycle<float>(R, o, (const float*)f, (float*)e, D0.t32);
    if (res != e) HIPCHK(hipMemcpyAsync(e, res, D0.nstored * 4, hipMemcpyDeviceToDevice, R.st));
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_apply_transpose(amg_hier* H, int level, double* x, double* y, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!x || !y || x == y) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  Depth& D = L.depths[0];
  hipStream_t st = stream_of(H, stream);
  double alpha, beta;
  coefs<double>(H, D, alpha, beta);
  launch_fill_tr<double>(D, x, st);
  launch_residual<double>(H->dim, D, true, x, nullptr, y, alpha, beta, nullptr, st);
  launch_band<double>(H->dim, D, 0, x, y, alpha, beta, beta, 0, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_apply_laplacian(amg_hier* H, int level, double* x, const double* face_data, double* y, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!x || !y || x == y) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  Depth& D = L.depths[0];
  hipStream_t st = stream_of(H, stream);
  launch_fill<double>(D, x, face_data, st);
  launch_residual<double>(H->dim, D, true, x, nullptr, y, 0.0, 1.0 / (12.0 * D.h * D.h), nullptr, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_dot(amg_hier* H, int level, const double* a, const double* b, double* out, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!a || !b || !out) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  Depth& D = L.depths[0];
  hipStream_t st = stream_of(H, stream);
  launch_tile_dot(H->dim, D, a, b, L.partial, st);
  launch_seg_reduce(L.partial, nullptr, 1, (int)D.tiles.size(), L.scal + S_DOT, false, st);
  HIPCHK(hipMemcpyAsync(L.h_scal + S_DOT, L.scal + S_DOT, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *out = L.h_scal[S_DOT];
  return AMG_OK;
}

int amg_dot_noalloc(amg_hier* H, int level, const double* a, const double* b, double* out, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!a || !b || !out) return fail(H, AMG_EINVAL, "bad arguments");
  Level& L = H->levels[level];
  Depth& D = L.depths[0];
  const int64_t nt = (int64_t)D.tiles.size();
  if (nt > kNoAllocDoubles)
    return fail(H, AMG_EUNSUPPORTED, "amg_dot_noalloc: the level has " + std::to_string(nt) +
                                         " tiles, the static scratch holds " + std::to_string(kNoAllocDoubles));
  double* sp = nullptr;
  HIPCHK(scratch_address(&sp));
  hipStream_t st = stream_of(H, stream);
  // every tile writes its own partial before the reduction reads it: nothing
  // of an earlier call's contents is read
  launch_tile_dot(H->dim, D, a, b, sp, st);
  launch_seg_reduce(sp, nullptr, 1, (int)nt, out, false, st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

static int check_cic(amg_hier* H, int level) {
  if (!check_level(H, level)) return AMG_EINVAL;
  const Level& L = H->levels[level];
  if (level < 1 || L.cf_mode == AMG_CF_INTERP || L.isolated || H->levels[level - 1].isolated)
    return fail(H, AMG_EINVAL, "interface conditions are for a refined level solved with face data");
  return AMG_OK;
}

int amg_cic_face_data(amg_hier* H, int level, const double* const* coarse, double k, double eta, int kind,
                      double* face_data, double* face_data_dt, void* stream) {
  TRY(check_cic(H, level));
  if (!coarse || !face_data || (kind != AMG_CIC_VALUE && kind != AMG_CIC_NORMAL_DERIVATIVE) || !(k > 0) ||
      !std::isfinite(eta))
    return fail(H, AMG_EINVAL, "bad arguments");
  for (int i = 0; i < 4; ++i)
    if (!coarse[i]) return fail(H, AMG_EINVAL, "null coarse data");
  // eq. timeInterp: the printed rows divided by 6 k^3; its columns belong to
  // t_-3, t_-2, t_-1, t_-0 (t* = t_-1 + eta), coarse[i] holds t_-i
  const double e = eta, e2 = eta * eta, e3 = e2 * eta, k2 = k * k, k3 = k2 * k, s = 1.0 / (6.0 * k3);
  const double r0[4] = {-e3 + k2 * e, 3 * e3 + 3 * k * e2 - 6 * k2 * e, -3 * e3 - 6 * k * e2 + 3 * k2 * e + 6 * k3,
                        e3 + 3 * k * e2 + 2 * k2 * e};
  const double r1[4] = {-3 * e2 + k2, 9 * e2 + 6 * k * e - 6 * k2, -9 * e2 - 12 * k * e + 3 * k2,
                        3 * e2 + 6 * k * e + 2 * k2};
  double tv[4], td[4];
  for (int i = 0; i < 4; ++i) {
    tv[i] = r0[3 - i] * s;
    td[i] = r1[3 - i] * s;
  }
  Level& L = H->levels[level];
  if (!L.cic.err.empty()) return fail(H, AMG_EUNSUPPORTED, L.cic.err);
  launch_cic(H->dim, L.cic, coarse, tv, td, kind, L.depths[0].h, face_data, face_data_dt, stream_of(H, stream));
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_cic_correct(amg_hier* H, int level, double* const* face_data, double* delta, void* stream) {
  TRY(check_cic(H, level));
  if (!face_data) return fail(H, AMG_EINVAL, "bad arguments");
  DPtrs fdv{};
  for (int d = 0; d < H->dim; ++d) {
    if (!face_data[d]) return fail(H, AMG_EINVAL, "null face data");
    fdv.p[d] = face_data[d];
  }
  Level& L = H->levels[level];
  hipStream_t st = stream_of(H, stream);
  if (L.cic.fd.empty()) {  // no coarse-fine face: nothing to correct
    if (delta)
      for (int c = 0; c < L.ncomp; ++c) delta[c] = 0.0;
    return AMG_OK;
  }
  launch_cic_correct(L.depths[0], L.ncomp, L.cic, fdv, st);
  if (delta) {
    HIPCHK(hipMemcpyAsync(delta, L.cic.d_sum, L.ncomp * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_set_coefficient(amg_hier* H, double c) {
  if (!H) return AMG_EINVAL;
  if (H->op != AMG_HELMHOLTZ) return fail(H, AMG_EINVAL, "the coefficient belongs to the Helmholtz operator");
  if (!(c > 0)) return fail(H, AMG_EINVAL, "Helmholtz needs c > 0");
  H->c = c;
  if (!H->finalized) return AMG_OK;
  for (int l = 0; l < H->nlevels; ++l) {
    Level& L = H->levels[l];
    std::string err;
    std::vector<double> mats;
    std::vector<int64_t> idx;
    const int rc = build_bottom(H, l, err, mats, idx);
    if (rc != AMG_OK) return fail(H, rc, err);
    if (mats.size() != L.nmat) return fail(H, AMG_EDEVICE, "bottom matrices changed size");
    if (!mats.empty()) HIPCHK(hipMemcpy(L.d_mat, mats.data(), mats.size() * sizeof(double), hipMemcpyHostToDevice));
    L.graph.release();
    L.graphT.release();
  }
  H->comp_graph.release();
  H->comp_graphT.release();
  return AMG_OK;
}

// ---- gradient, divergence, projection (eqs. discreteOps a-b, appProj,
// comp_ProjOp) ----------------------------------------------------------------
static int check_range(amg_hier* H, int lev_lo, int lev_hi) {
  if (!H || !H->finalized) return fail(H, AMG_EINVAL, "amg_finalize has not been called");
  if (lev_lo < 0 || lev_hi >= H->nlevels || lev_hi < lev_lo) return fail(H, AMG_EINVAL, "level out of range");
  if (lev_lo != lev_hi) {
    if (lev_lo != 0) return fail(H, AMG_EUNSUPPORTED, "a composite operator starts at level 0");
    for (int l = 1; l <= lev_hi; ++l)
      if (H->levels[l].cf_mode != AMG_CF_INTERP)
        return fail(H, AMG_EINVAL, "levels of a composite operator take interpolated coarse-fine ghosts");
  } else if (lev_lo > 0 && H->levels[lev_lo].cf_mode == AMG_CF_INTERP) {
    return fail(H, AMG_EUNSUPPORTED, "a level with interpolated coarse-fine ghosts is used in composite form");
  }
  return AMG_OK;
}

// the ghosts of level l's array u: the level's fill from face data fd, then
// (composite) AMRCFI from the level below
static void fill_level(amg_hier* H, int l, double* u, const double* fd, const double* uc, hipStream_t st) {
  Level& L = H->levels[l];
  launch_fill<double>(L.depths[0], u, fd, st);
  if (uc) launch_cfi(H->dim, L.cmp, uc, u, st);
}

static int gradient_impl(amg_hier* H, int lo, int hi, double* const* phi, const double* const* fd,
                         double* const* g, const double* const* w, hipStream_t st) {
  const int dim = H->dim;
  const bool comp = hi > lo;
  for (int l = lo; l <= hi; ++l) {
    if (!phi[l]) return fail(H, AMG_EINVAL, "null phi");
    for (int d = 0; d < dim; ++d)
      if (!g[l * dim + d] || (w && !w[l * dim + d])) return fail(H, AMG_EINVAL, "null component");
  }
  if (comp)
    for (int l = hi; l >= 1; --l) launch_avgdown(dim, H->levels[l].cmp, phi[l], phi[l - 1], st);
  for (int l = lo; l <= hi; ++l) {
    fill_level(H, l, phi[l], fd ? fd[l] : nullptr, comp && l > lo ? phi[l - 1] : nullptr, st);
    DPtrs gp{};
    CPtrs wp{};
    for (int d = 0; d < dim; ++d) {
      gp.p[d] = g[l * dim + d];
      wp.p[d] = w ? w[l * dim + d] : nullptr;
    }
    launch_grad(dim, H->levels[l].depths[0], phi[l], gp, wp, w != nullptr, st);
  }
  if (comp)
    for (int l = hi; l >= 1; --l)
      for (int d = 0; d < dim; ++d) launch_avgdown(dim, H->levels[l].cmp, g[l * dim + d], g[(l - 1) * dim + d], st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

static int divergence_impl(amg_hier* H, int lo, int hi, double* const* w, const double* const* wb,
                           double* const* out, hipStream_t st) {
  const int dim = H->dim;
  const bool comp = hi > lo;
  for (int l = lo; l <= hi; ++l) {
    if (!out[l]) return fail(H, AMG_EINVAL, "null output");
    for (int d = 0; d < dim; ++d)
      if (!w[l * dim + d]) return fail(H, AMG_EINVAL, "null component");
  }
  if (comp)
    for (int l = hi; l >= 1; --l)
      for (int d = 0; d < dim; ++d) launch_avgdown(dim, H->levels[l].cmp, w[l * dim + d], w[(l - 1) * dim + d], st);
  for (int l = lo; l <= hi; ++l) {
    CPtrs wp{};
    for (int d = 0; d < dim; ++d) {
      fill_level(H, l, w[l * dim + d], wb ? wb[l * dim + d] : nullptr, comp && l > lo ? w[(l - 1) * dim + d] : nullptr,
                 st);
      wp.p[d] = w[l * dim + d];
    }
    launch_div(dim, H->levels[l].depths[0], wp, out[l], st);
  }
  if (comp) {
    for (int l = 1; l <= hi; ++l) {
      CPtrs wc{}, wf{};
      for (int d = 0; d < dim; ++d) {
        wc.p[d] = w[(l - 1) * dim + d];
        wf.p[d] = w[l * dim + d];
      }
      launch_reflux_div(dim, H->levels[l].cmp, wc, wf, out[l - 1], H->levels[l - 1].depths[0].h, st);
    }
    for (int l = hi; l >= 1; --l) launch_avgdown(dim, H->levels[l].cmp, out[l], out[l - 1], st);
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_gradient(amg_hier* H, int lev_lo, int lev_hi, double* const* phi, const double* const* face_data,
                 double* const* g, void* stream) {
  TRY(check_range(H, lev_lo, lev_hi));
  if (!phi || !g) return fail(H, AMG_EINVAL, "bad arguments");
  return gradient_impl(H, lev_lo, lev_hi, phi, face_data, g, nullptr, stream_of(H, stream));
}

int amg_divergence(amg_hier* H, int lev_lo, int lev_hi, double* const* w, const double* const* face_data,
                   double* const* out, void* stream) {
  TRY(check_range(H, lev_lo, lev_hi));
  if (!w || !out) return fail(H, AMG_EINVAL, "bad arguments");
  return divergence_impl(H, lev_lo, lev_hi, w, face_data, out, stream_of(H, stream));
}

// the two hierarchies of a projection must share the packed layout of every level
static int same_layout(amg_hier* Hw, amg_hier* Hp, int lev_lo, int lev_hi) {
  if (Hw->dim != Hp->dim || Hw->nlevels != Hp->nlevels) return fail(Hp, AMG_EINVAL, "hierarchies differ");
  for (int l = lev_lo; l <= lev_hi; ++l) {
    const Depth& A0 = Hw->levels[l].depths[0];
    const Depth& B0 = Hp->levels[l].depths[0];
    if (A0.boxes.size() != B0.boxes.size() || A0.nstored != B0.nstored) return fail(Hp, AMG_EINVAL, "layouts differ");
    for (size_t b = 0; b < A0.boxes.size(); ++b)
      if (A0.boxd[b].off != B0.boxd[b].off || memcmp(A0.boxes[b].lo, B0.boxes[b].lo, sizeof(int) * 3) ||
          memcmp(A0.boxes[b].hi, B0.boxes[b].hi, sizeof(int) * 3))
        return fail(Hp, AMG_EINVAL, "layouts differ");
  }
  return AMG_OK;
}

int amg_project(amg_hier* Hw, amg_hier* Hp, int lev_lo, int lev_hi, double* const* w, const double* const* wb,
                double* const* phi, double* const* u, const amg_solve_opts* opts, amg_solve_stats* stats,
                void* stream) {
  TRY(check_range(Hw, lev_lo, lev_hi));
  TRY(check_range(Hp, lev_lo, lev_hi));
  if (!w || !phi || !u) return fail(Hp, AMG_EINVAL, "bad arguments");
  if (Hp->op != AMG_POISSON) return fail(Hp, AMG_EINVAL, "the potential's hierarchy must hold the Poisson operator");
  TRY(same_layout(Hw, Hp, lev_lo, lev_hi));
  hipStream_t st = stream_of(Hp, stream);
  std::vector<double*> div(lev_hi + 1, nullptr);
  for (int l = lev_lo; l <= lev_hi; ++l) div[l] = Hw->levels[l].fsh;
  int rc = divergence_impl(Hw, lev_lo, lev_hi, w, wb, div.data(), st);
  if (rc != AMG_OK) return fail(Hp, rc, Hw->err);
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(Hp, o));
  std::vector<const double*> f(div.begin(), div.end());
  if (lev_hi > lev_lo)
    rc = composite_solve(Hp, lev_lo, lev_hi, phi, f.data(), nullptr, &o, stats, st);
  else
    rc = level_solve(Hp, lev_lo, phi[lev_lo], f[lev_lo], nullptr, o, stats, st, false);
  if (rc != AMG_OK) return rc;
  return gradient_impl(Hp, lev_lo, lev_hi, phi, nullptr, u, w, st);
}

// ---- transposes of G, D and the projection -------------------------------
// Each is the homogeneous map between the valid cells of levels lo..hi (one
// level, or composite from level 0): its input's covered cells and ghosts
// are set to 0 (they do not enter the forward map), the output is 0 on
// covered cells.  Ghost adjoints of the gradient stencil go to the slots of
// the level's scratch array A64 (negated), refluxing (divergence) adds its
// share there too, and the scatter kernels send them on: fills (band),
// exchange copies, AMRCFI onto the level below.

// the input of a transpose: valid cells only, ghosts 0
static void clear_input(amg_hier* H, int l, int hi, double* a, hipStream_t st) {
  if (l < hi) launch_zero_covered(H->levels[l + 1].cmp, a, st);
  launch_fill_zero<double>(H->levels[l].depths[0], a, st);
}

// the ghost adjoints held (negated) in each level's A64 onto the cells of
// out: interior share, fills, exchange copies, AMRCFI onto the level below
static void scatter_slots(amg_hier* H, int lo, int hi, double* const* out, int stride, hipStream_t st) {
  const int dim = H->dim;
  for (int l = hi; l >= lo; --l) {
    Level& L = H->levels[l];
    Depth& D = L.depths[0];
    double* o = out[l * stride];
    launch_sub_array(dim, D, L.A64, o, st);
    launch_band_ab(dim, D, o, L.A64, o, 0.0, st);
    launch_exch_T(D, L.A64, o, st);
    if (l > lo) launch_cfi_T(dim, L.cmp, o, L.A64, 0.0, L.mu, out[(l - 1) * stride], st);
  }
}

// the average-down of the forward input, transposed: covered adjoints to
// the children in equal parts, coarse to fine
static void pass_down_all(amg_hier* H, int hi, double* const* out, int stride, hipStream_t st) {
  const double down = 1.0 / (1 << H->dim);
  for (int l = 1; l <= hi; ++l) {
    launch_pass_down(H->levels[l].cmp, out[(l - 1) * stride], out[l * stride], down, st);
    launch_zero_covered(H->levels[l].cmp, out[(l - 1) * stride], st);
  }
}

static int gradient_T_impl(amg_hier* H, int lo, int hi, double* const* mu, double* const* out, hipStream_t st) {
  const int dim = H->dim;
  for (int l = lo; l <= hi; ++l) {
    if (!out[l]) return fail(H, AMG_EINVAL, "null output");
    for (int d = 0; d < dim; ++d)
      if (!mu[l * dim + d]) return fail(H, AMG_EINVAL, "null component");
  }
  for (int l = lo; l <= hi; ++l) {
    Level& L = H->levels[l];
    CPtrs m{};
    for (int d = 0; d < dim; ++d) {
      clear_input(H, l, hi, mu[l * dim + d], st);
      m.p[d] = mu[l * dim + d];
    }
    // G_d is antisymmetric: its transpose on the cells is -G_d of the
    // zero-extended adjoint
    launch_div(dim, L.depths[0], m, out[l], st, -1.0);
    launch_zero<double>(L.A64, L.depths[0].nstored, st);
    launch_gslot(L.depths[0], m, -1, L.A64, st);
  }
  scatter_slots(H, lo, hi, out, 1, st);
  if (hi > lo) pass_down_all(H, hi, out, 1, st);
  for (int l = lo; l <= hi; ++l) launch_fill_zero<double>(H->levels[l].depths[0], out[l], st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

static int divergence_T_impl(amg_hier* H, int lo, int hi, double* const* lam, double* const* out, hipStream_t st) {
  const int dim = H->dim;
  for (int l = lo; l <= hi; ++l) {
    if (!lam[l]) return fail(H, AMG_EINVAL, "null lam");
    for (int d = 0; d < dim; ++d)
      if (!out[l * dim + d]) return fail(H, AMG_EINVAL, "null component");
  }
  for (int l = lo; l <= hi; ++l) {
    clear_input(H, l, hi, lam[l], st);
    DPtrs g{};
    for (int d = 0; d < dim; ++d) g.p[d] = out[l * dim + d];
    launch_grad(dim, H->levels[l].depths[0], lam[l], g, CPtrs{}, false, st, -1.0);
  }
  for (int d = 0; d < dim; ++d) {
    for (int l = lo; l <= hi; ++l)
      launch_zero<double>(H->levels[l].A64, H->levels[l].depths[0].nstored, st);
    for (int l = lo + 1; l <= hi; ++l)
      launch_rfxV_T(H->levels[l].cmp, d, lam[l - 1], -1.0, H->levels[l - 1].A64, H->levels[l].A64, st);
    for (int l = lo; l <= hi; ++l) {
      CPtrs m{};
      for (int e = 0; e < dim; ++e) m.p[e] = lam[l];
      launch_gslot(H->levels[l].depths[0], m, d, H->levels[l].A64, st);
    }
    scatter_slots(H, lo, hi, out + d, dim, st);
    if (hi > lo) pass_down_all(H, hi, out + d, dim, st);
  }
  for (int l = lo; l <= hi; ++l)
    for (int d = 0; d < dim; ++d) launch_fill_zero<double>(H->levels[l].depths[0], out[l * dim + d], st);
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_gradient_transpose(amg_hier* H, int lev_lo, int lev_hi, double* const* mu, double* const* out,
                           void* stream) {
  TRY(check_range(H, lev_lo, lev_hi));
  if (!mu || !out) return fail(H, AMG_EINVAL, "bad arguments");
  return gradient_T_impl(H, lev_lo, lev_hi, mu, out, stream_of(H, stream));
}

int amg_divergence_transpose(amg_hier* H, int lev_lo, int lev_hi, double* const* lam, double* const* out,
                             void* stream) {
  TRY(check_range(H, lev_lo, lev_hi));
  if (!lam || !out) return fail(H, AMG_EINVAL, "bad arguments");
  return divergence_T_impl(H, lev_lo, lev_hi, lam, out, stream_of(H, stream));
}

int amg_project_adjoint(amg_hier* Hw, amg_hier* Hp, int lev_lo, int lev_hi, double* const* ubar, double* const* lam,
                        double* const* wbar, const amg_solve_opts* opts, amg_solve_stats* stats, void* stream) {
  TRY(check_range(Hw, lev_lo, lev_hi));
  TRY(check_range(Hp, lev_lo, lev_hi));
  if (!ubar || !lam || !wbar) return fail(Hp, AMG_EINVAL, "bad arguments");
  TRY(same_layout(Hw, Hp, lev_lo, lev_hi));
  const int dim = Hp->dim;
  for (int l = lev_lo; l <= lev_hi; ++l) {
    if (!lam[l]) return fail(Hp, AMG_EINVAL, "null lam");
    for (int d = 0; d < dim; ++d)
      if (!ubar[l * dim + d] || !wbar[l * dim + d]) return fail(Hp, AMG_EINVAL, "null component");
  }
  hipStream_t st = stream_of(Hp, stream);
  amg_hier* H = Hp;  // the hierarchy that reports device errors
  // g = G^T ubar (the potential's fill), into the Poisson hierarchy's fsh
  std::vector<double*> g(lev_hi + 1, nullptr);
  for (int l = lev_lo; l <= lev_hi; ++l) g[l] = Hp->levels[l].fsh;
  TRY(gradient_T_impl(Hp, lev_lo, lev_hi, ubar, g.data(), st));
  // lam = L^-T g: the adjoint of the pure-Neumann solve (transposes of its
  // solvability shift and mean removal included)
  amg_solve_opts o;
  amg_default_opts(&o);
  if (opts) o = *opts;
  TRY(check_opts(Hp, o));
  int rc;
  if (lev_hi > lev_lo) {
    std::vector<const double*> gc(g.begin(), g.end());
    rc = amg_solve_adjoint_composite(Hp, lev_hi, lam, gc.data(), &o, stats, st);
  } else {
    rc = amg_solve_adjoint(Hp, lev_lo, lam[lev_lo], g[lev_lo], &o, stats, st);
  }
  if (rc != AMG_OK) return rc;
  // wbar = ubar - D^T lam (the velocity's fill); D^T lam into the velocity
  // hierarchy's depth-0 work buffers
  std::vector<double*> dt((lev_hi + 1) * dim, nullptr), lamv(lev_hi + 1, nullptr);
  for (int l = lev_lo; l <= lev_hi; ++l) {
    Depth& D = Hw->levels[l].depths[0];
    double* bufs[3] = {D.e64, D.f64, D.t64};
    for (int d = 0; d < dim; ++d) dt[l * dim + d] = bufs[d];
    // the solve leaves lam's ghosts and covered cells 0; a copy keeps the
    // caller's lam as the solve returned it
    lamv[l] = Hw->levels[l].fsh;
    HIPCHK(hipMemcpyAsync(lamv[l], lam[l], D.nstored * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  rc = divergence_T_impl(Hw, lev_lo, lev_hi, lamv.data(), dt.data(), st);
  if (rc != AMG_OK) return fail(Hp, rc, Hw->err);
  for (int l = lev_lo; l <= lev_hi; ++l) {
    Depth& D = Hw->levels[l].depths[0];
    for (int d = 0; d < dim; ++d) {
      double* wb = wbar[l * dim + d];
      if (wb != ubar[l * dim + d])
        HIPCHK(hipMemcpyAsync(wb, ubar[l * dim + d], D.nstored * sizeof(double), hipMemcpyDeviceToDevice, st));
      launch_sub_array(dim, D, dt[l * dim + d], wb, st);
      if (l < lev_hi) launch_zero_covered(Hw->levels[l + 1].cmp, wb, st);
    }
  }
  HIPCHK(hipGetLastError());
  return AMG_OK;
}

int amg_time_sweep(amg_hier* H, int level, int dtype, int smoother, int n, void* u, const void* f, void* tmp,
                   double* avg_ms, void* stream) {
  if (!check_level(H, level)) return AMG_EINVAL;
  if (!u || !f || !tmp || !avg_ms || n < 1 || u == tmp) return fail(H, AMG_EINVAL, "bad arguments");
  if (smoother != AMG_SMOOTH_JACOBI && smoother != AMG_SMOOTH_RB) return fail(H, AMG_EINVAL, "bad smoother");
  Level& L = H->levels[level];
  Depth& D = L.depths[0];
  hipStream_t st = stream_of(H, stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  auto run = [&](auto* cur, auto* oth, const auto* ff) {
    using T = std::remove_const_t<std::remove_pointer_t<decltype(ff)>>;
    T a, b;
    coefs<T>(H, D, a, b);
    (void)hipEventRecord(e0, st);
    if constexpr (sizeof(T) == 4) {
      // the form the mixed-precision solve post-smooths in: n half-sweeps
      // in colour-split storage (u, f and tmp taken as split arrays)
      if (smoother == AMG_SMOOTH_RB && D.split_rb) {
        const int64_t hs = D.nstored / 2;
        const float* h[2] = {cur, cur + hs};
        for (int i = 0; i < n; ++i) {
          const int col = i & 1;
          float* dst = (h[col] == cur + col * hs ? oth : cur) + col * hs;
          launch_rbs(H->dim, D, 0, h[0], h[1], ff + col * hs, dst, a, b, 1.0f, col, st);
          h[col] = dst;
        }
        (void)hipEventRecord(e1, st);
        return;
      }
    }
    for (int i = 0; i < n; ++i) {
      const int gr = sizeof(T) == 4 ? 1 : 0;  // the form the FP32 V-cycle launches
      if (smoother == AMG_SMOOTH_JACOBI)
        launch_jacobi<T>(H->dim, D, cur, ff, oth, a, b, T(2.0 / 3.0), false, st, gr);
      else
        launch_rb<T>(H->dim, D, cur, ff, oth, a, b, T(1), i & 1, false, st, gr);
      std::swap(cur, oth);
    }
    (void)hipEventRecord(e1, st);
  };
  if (dtype == AMG_F64)
    run((double*)u, (double*)tmp, (const double*)f);
  else
    run((float*)u, (float*)tmp, (const float*)f);
  hipError_t err = hipEventSynchronize(e1);
  float ms = 0.f;
  if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIPCHK(err);
  HIPCHK(hipGetLastError());
  *avg_ms = (double)ms / n;
  return AMG_OK;
}

int amg_autotune(amg_hier* H, int level, int dtype, int smoother, int nreps, int* best, double* best_ms) {
  if (!H) return AMG_EINVAL;
  if (H->finalized) return fail(H, AMG_EINVAL, "autotuning runs before amg_finalize");
  if (level < 0 || level >= H->nlevels || nreps < 1) return fail(H, AMG_EINVAL, "bad arguments");
  const int cands[] = {4, 6, 8, 16, 32, 64, 128};
  int arg = H->dim == 2 ? H->march2 : H->march3;
  double tbest = 1e300;
  for (int m : cands) {
    // a finalized copy of the layout with march length m
    amg_hier* T = nullptr;
    double xhi[3];
    for (int d = 0; d < H->dim; ++d) xhi[d] = H->x_lo[d] + H->base[d] * H->h0;
    int rc = amg_create(H->dim, H->x_lo, xhi, H->base, H->ratio, H->nlevels, &T);
    if (rc != AMG_OK) return fail(H, rc, "autotune: amg_create failed");
    for (int l = 0; l < H->nlevels && rc == AMG_OK; ++l) {
      T->levels[l].boxes = H->levels[l].boxes;
      T->levels[l].isolated = H->levels[l].isolated;
      T->levels[l].cf_mode = H->levels[l].cf_mode;
    }
    memcpy(T->phys_bc, H->phys_bc, sizeof H->phys_bc);
    T->op = H->op;
    T->c = H->c;
    T->row_align = H->row_align;
    T->bottom_cells = H->bottom_cells;
    T->bottom_kind = H->bottom_kind;
    T->bottom_iters = H->bottom_iters;
    T->split_rb = H->split_rb;
    T->march2 = T->march3 = m;
    rc = amg_finalize(T);
    if (rc != AMG_OK) {
      const std::string e = T->err;
      amg_destroy(T);
      return fail(H, rc, "autotune: " + e);
    }
    // marches below 8 are not tried for 3D sweeps in interleaved storage:
    // they time well back to back there but not inside the solves (the
    // colour-split sweep and 2D sweeps gain from them in the solves too)
    const bool split = dtype == AMG_F32 && smoother == AMG_SMOOTH_RB && T->levels[level].depths[0].split_rb;
    if (m < 8 && H->dim == 3 && !split) {
      amg_destroy(T);
      continue;
    }
    const size_t bytes = T->levels[level].depths[0].nstored * (dtype == AMG_F64 ? 8 : 4);
    void *u = nullptr, *f = nullptr, *t = nullptr;
    hipError_t e = hipMalloc(&u, bytes);
    if (e == hipSuccess) e = hipMalloc(&f, bytes);
    if (e == hipSuccess) e = hipMalloc(&t, bytes);
    if (e == hipSuccess) e = hipMemset(u, 0, bytes);
    if (e == hipSuccess) e = hipMemset(f, 0, bytes);
    double ms = 0.0;
    if (e == hipSuccess) {
      rc = amg_time_sweep(T, level, dtype, smoother, 4, u, f, t, &ms, nullptr);
      if (rc == AMG_OK) rc = amg_time_sweep(T, level, dtype, smoother, nreps, u, f, t, &ms, nullptr);
    }
    for (void* p : {u, f, t})
      if (p) (void)hipFree(p);
    const std::string terr = T->err;
    amg_destroy(T);
    if (e != hipSuccess) return fail(H, AMG_EDEVICE, std::string("autotune: ") + hipGetErrorString(e));
    if (rc != AMG_OK) return fail(H, rc, "autotune: " + terr);
    if (ms < tbest) {
      tbest = ms;
      arg = m;
    }
  }
  (H->dim == 2 ? H->march2 : H->march3) = arg;
  if (best) *best = arg;
  if (best_ms) *best_ms = tbest;
  return AMG_OK;
}

int amg_timing_enable(amg_hier* H, int on) {
  if (!H) return AMG_EINVAL;
  H->timer.on = on != 0;
  for (auto& L : H->levels) L.graph.release();  // recapture with or without events
  H->comp_graph.release();  // composite cycles run as direct launches while timing is on
  H->timer.pending.clear();
  H->timer.next = H->timer.base = 0;
  if (H->timer.on && H->timer.pool.empty()) {
    H->timer.pool.resize(8192);
    // timing-only events: no system-scope fence when they complete
    for (auto& e : H->timer.pool) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  return AMG_OK;
}

int amg_timing_read(amg_hier* H, int kind, int64_t* count, double* total_ms, int reset) {
  if (!H || kind < 0 || kind >= AMG_T_KINDS) return AMG_EINVAL;
  if (!H->timer.pending.empty()) {  // launches made outside a solve (step-level calls)
    (void)hipEventSynchronize(H->timer.pool[H->timer.pending.back().second + 1]);
    collect_timing(H->timer);
  }
  if (count) *count = H->timer.count[kind];
  if (total_ms) *total_ms = H->timer.total_ms[kind];
  if (reset) {
    H->timer.count[kind] = 0;
    H->timer.total_ms[kind] = 0.0;
  }
  return AMG_OK;
}

}  // extern "C"
