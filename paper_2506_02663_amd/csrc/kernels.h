// Launchers of the HIP kernels (kernels.hip), called by the solver driver.
#pragma once
#include <hip/hip_runtime.h>

#include "amg_internal.h"

namespace amg {
// The FP32 V-cycle's coarse tail in one workgroup (tail.hip): depths d[0]
// (the first tail depth) .. d[nd-1] (the exact bottom system), one box each,
// every face filled uniformly or periodic onto the box itself.  e / f: the depth's iterate and right-hand
// side buffers; cnt: the component's cells at the depth.
constexpr int kTailMaxDepths = 8;
constexpr int kTailMaxCells = 4096;  // cells of a tail depth (four per thread of its workgroup)
struct TailDepth {
  BoxD b;
  float* e;
  float* f;
  float alpha, beta;
  double cnt;
  int32_t wrap[3];  // direction d periodic with the box spanning the grid: its ghosts wrap onto itself
};
struct TailArgs {
  TailDepth d[kTailMaxDepths];
  int nd, nu1, nu2, rb, singular;
  float omega;
};
// LDS bytes of either leg (four arrays of the first depth, one of the second)
size_t tail_lds_bytes(int dim, const TailArgs& A);
// the largest dynamic LDS a tail leg may use on the current device
size_t tail_lds_limit();
// raises the tail kernels' dynamic LDS limit to it (before any capture)
void tail_prepare();
void launch_tail_down(int dim, const TailArgs& A, hipStream_t st);
void launch_tail_up(int dim, const TailArgs& A, hipStream_t st);
template <typename T>
void launch_fill(const Depth& D, T* u, const double* fd, hipStream_t st);
template <typename T>
void launch_fill_tr(const Depth& D, T* u, hipStream_t st);
template <typename T>
void launch_fill_zero(const Depth& D, T* u, hipStream_t st);
template <typename T>
void launch_band(int dim, const Depth& D, int mode, const T* u, T* out, T alpha, T beta, T scale, int col,
                 hipStream_t st);
void launch_tile_dot(int dim, const Depth& D, const double* a, const double* b, double* part, hipStream_t st);
// per-direction device pointers, passed by value
struct DPtrs {
  double* p[3];
};
struct CPtrs {
  const double* p[3];
};
// g[d] = scale G_d u, or w[d] - scale G_d u if sub
void launch_grad(int dim, const Depth& D, const double* u, DPtrs g, CPtrs w, bool sub, hipStream_t st,
                 double scale = 1.0);
// out = scale sum_d G_d w[d]
void launch_div(int dim, const Depth& D, CPtrs w, double* out, hipStream_t st, double scale = 1.0);
// coarse-fine interface conditions of a face-data level: fd (dfd may be
// null) at the table's entries from the coarse data hist[i] = phi(t_-i) with
// time weights tv (value) and td (derivative); kind 0 face averages, 1
// outward normal derivatives (h: the level's cell size)
void launch_cic(int dim, const CicTable& T, const double* const* hist, const double tv[4], const double td[4], int kind,
                double h, double* fd, double* dfd, hipStream_t st);
// eq. correctingFaceAvg on the velocity face data fdv.p[d] (T.d_sum receives
// the per-component deltas)
void launch_cic_correct(const Depth& D, int ncomp, const CicTable& T, DPtrs fdv, hipStream_t st);
// transposes of G and D: ghost-slot adjoints of the gradient stencil (ab
// -= weights times mu; mu.p[d] read along d; dir >= 0: faces normal to dir)
void launch_gslot(const Depth& D, CPtrs mu, int dir, double* ab, hipStream_t st);
// refluxing of the divergence (component d), transposed: abc / abf (levels
// l-1 / l) += lscale * d(correction) / d(element) * lam_c[refluxed cell]
void launch_rfxV_T(const Composite& X, int d, const double* lam_c, double lscale, double* abc, double* abf,
                   hipStream_t st);
void launch_reflux_div(int dim, const Composite& X, CPtrs wc, CPtrs wf, double* div, double hc, hipStream_t st);
template <typename T>
void launch_residual(int dim, const Depth& D, bool all, const T* u, const T* f, T* r, T alpha, T beta, double* part,
                     hipStream_t st);
// gr != 0 (FP32 only): filled ghost columns computed where they are read, no
// fill needed before the sweep for them
template <typename T>
void launch_jacobi(int dim, const Depth& D, const T* u, const T* f, T* out, T alpha, T beta, T omega, bool zero,
                   hipStream_t st, int gr = 0);
template <typename T>
void launch_rb(int dim, const Depth& D, const T* u, const T* f, T* out, T alpha, T beta, T omega, int col, bool zero,
               hipStream_t st, int gr = 0);
template <typename T>
// gr != 0 (F.uniform_fill): the kernel writes the ghosts it reads itself
// (no fill launch before it)
void launch_resid_restrict(int dim, const Depth& F, const Depth& C, const T* u, const T* f, T* fc, T alpha, T beta,
                           hipStream_t st, int gr = 0);
template <typename T>
void launch_restrict(int dim, const Depth& F, const Depth& C, const T* r, T* fc, hipStream_t st);
template <typename T>
// gr != 0 (C.uniform_fill): the coarse ghosts it reads are formed from the
// coarse rows (no fill launch on C before it)
void launch_prolong(int dim, const Depth& F, const Depth& C, const T* ec, T* u, hipStream_t st, int gr = 0);
template <typename T>
void launch_bottom(const Depth& D, const double* mats, const int64_t* idx, const T* f, T* e, bool tr, hipStream_t st,
                   T* e2 = nullptr);
// ILU(0)-preconditioned GMRES(iters) on every bottom system of D (tables
// planned with the ILU-GMRES bottom; ws: the level's Krylov workspace)
template <typename T>
void launch_bottom_gmres(const Depth& D, const double* mats, const int64_t* idx, const T* f, T* e, int iters,
                         double* ws, hipStream_t st, T* e2 = nullptr);
template <typename T>
void launch_tile_sum(int dim, const Depth& D, const T* a, double* part, hipStream_t st);
template <typename T>
void launch_tile_absmax(int dim, const Depth& D, const T* a, double* part, hipStream_t st);
void launch_reduce_max(const double* part, int n, double* out, hipStream_t st);
void launch_seg_reduce(const double* in, const int32_t* ptr, int nseg, int n, double* out, bool is_max,
                       hipStream_t st,
                       double* host = nullptr);
// delta[c] = flag[c] ? (sum of component c's tile partials) / cnt[c] : 0, one launch
void launch_comp_mean_delta(const Depth& D, const double* part, const int32_t* flag, const double* cnt, int ncomp,
                            double* delta, hipStream_t st);
void launch_comp_sum(const double* part, const int32_t* ptr, const int32_t* ids, int ncomp, double* out,
                     hipStream_t st);
void launch_comp_delta(const double* sum, const double* bsum, const int32_t* flag, const double* cnt, int ncomp,
                       double scale_sum, double scale_b, double* delta, double* defect, hipStream_t st);
template <typename T>
void launch_comp_shift(int dim, const Depth& D, T* a, const double* delta, hipStream_t st);
void launch_chunk_fdsum(const Depth& D, const double* fd, const uint8_t* valid, double* part, hipStream_t st);
// mean removal from the per-tile sums in one launch (each block re-sums its
// component's tile sums)
template <typename T>
void launch_comp_mean_shift(int dim, const Depth& D, const double* part, const int32_t* flag, const double* cnt, T* a,
                            hipStream_t st);
// per-component mean removal of a small depth in one launch (one block per component)
template <typename T>
void launch_comp_mean_small(int dim, const Depth& D, int ncomp, const int32_t* flag, const double* cnt, T* a,
                            hipStream_t st);
void launch_cf_delta(const double* defect, const int32_t* flag, const double* ncf, const double* cnt, int ncomp,
                     double hD, double hD1, double* delta, double* dfd, hipStream_t st);
void launch_fd_correct(const Depth& D, const double* fd, const double* dfd, double* out, hipStream_t st);
void launch_cfi(int dim, const Composite& X, const double* uc, double* uf, hipStream_t st);
void launch_avgdown(int dim, const Composite& X, const double* uf, double* uc, hipStream_t st);
void launch_reflux(int dim, const Composite& X, const double* uc, const double* uf, double* r, double kappa,
                   double hc, double hf, hipStream_t st);
void launch_amr_prolong(int dim, const Composite& X, const double* ec, double* u, double* ef, hipStream_t st,
                        double scale = 1.0);
// adjoint of the composite operator
void launch_zero_covered(const Composite& X, double* u, hipStream_t st);
void launch_sumdown(int dim, const Composite& X, const double* uf, double* uc, double scale, hipStream_t st);
void launch_rfx_T(const Composite& X, const double* lam_c, double lscale, double* abc, double* abf, hipStream_t st);
void launch_exch_T(const Depth& D, const double* ab, double* r, hipStream_t st);
void launch_cfi_T(int dim, const Composite& X, const double* lam_f, const double* abf, double beta, double* mu,
                  double* rc, hipStream_t st);
void launch_pass_down(const Composite& X, const double* rc, double* rf, double scale, hipStream_t st);
void launch_sub_array(int dim, const Depth& D, const double* a, double* r, hipStream_t st);
void launch_band_ab(int dim, const Depth& D, const double* u, const double* ab, double* out, double beta,
                    hipStream_t st);
void launch_max_slots(const double* in, int n, double* out, hipStream_t st);
void launch_sub_scalar(int dim, const Depth& D, double* a, const double* s, hipStream_t st);
template <typename T>
void launch_update2(int dim, const Depth& D, double* x, double* E, const T* e, const double* scal, hipStream_t st);
template <typename T>
void launch_update(int dim, const Depth& D, double* x, const T* e, const double* scal, hipStream_t st);
// r32 = (r - delta[component]) / scal[0] (delta may be NULL)
// the FP64 residual of all tiles stored unscaled in FP32 (r = f - A u, with
// the per-tile max and sum partials), and its in-place conversion
// r32 = (r32 - delta[comp]) / scal[0]
// split: r in colour-split storage (halves D.nstored / 2 apart); gr != 0
// (D.uniform_fill, homogeneous conditions): the kernel writes the ghosts of
// u it reads itself, so no fill launch is needed before it
void launch_residual32(int dim, const Depth& D, const double* u, const double* f, float* r, double alpha, double beta,
                       double* part, hipStream_t st, bool split = false, int gr = 0);
// fs (may be null): the result in colour-split storage instead of r32
// (two halves of D.nstored / 2 elements, element e of colour c at index
// e >> 1 of half c)
void launch_scale32(int dim, const Depth& D, float* r32, const double* scal, hipStream_t st, const double* delta,
                    float* fs = nullptr);
void launch_to32(int dim, const Depth& D, const double* r, float* r32, const double* scal, hipStream_t st,
                 const double* delta = nullptr, float* fs = nullptr);
// colour-split storage (FP32 depths with split_rb): red-black half-sweep
// of colour col of the iterate with halves h0, h1 into the half `out` (fc:
// half col of f; mode 0: plain, 1: half col of the iterate is zero, 2: the
// iterate is zero); residual fused with restriction from split u and f into
// the coarse f (interleaved); prolongation out = u + P ec (u, out split).  scal (may be null): f is the unscaled
// residual, read as (f - delta[comp]) / scal[0] (delta may be null).  Mode 3
// of the half-sweep: mode 0 with xu += su[0] * (the pair of the new value and
// the other colour) instead of writing `out` (the last half-sweep fused with
// the outer update; xu FP64 in the depth's interleaved layout).
void launch_rbs(int dim, const Depth& D, int mode, const float* h0, const float* h1, const float* fc, float* out,
                float alpha, float beta, float omega, int col, hipStream_t st, const double* scal = nullptr,
                const double* delta = nullptr, double* xu = nullptr, const double* su = nullptr);
void launch_resid_restrict_s(int dim, const Depth& F, const Depth& C, const float* u, const float* f, float* fc,
                             float alpha, float beta, hipStream_t st, const double* scal = nullptr,
                             const double* delta = nullptr);
void launch_prolong_s(int dim, const Depth& F, const Depth& C, const float* ec, const float* u, float* out,
                      hipStream_t st);
void launch_shift_copy(int dim, const Depth& D, const double* f, double* out, const double* delta, hipStream_t st);
void launch_set_scale(const double* src, double* dst, hipStream_t st);
void launch_set_scaled(const double* src, double f, double* dst, hipStream_t st);
template <typename T>
void launch_zero(T* a, int64_t n, hipStream_t st);
}  // namespace amg
