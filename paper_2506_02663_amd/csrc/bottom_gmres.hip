// The paper's bottom solver of the pressure systems (Section 6.5): m steps
// of GMRES from zero, preconditioned on the right by ILU(0), on every system
// of the coarsest depth (a component, or an isolated box; bordered with the
// zero-mean constraint when singular).  The host keeps B = K P and
// P = (L U)^-1 dense per system (one matrix-vector product per
// preconditioning), so one GMRES step is: w = B v_j, modified Gram-Schmidt
// against v_0..v_j, the new Arnoldi vector; then the small least-squares
// problem by Givens rotations and x = P (V y).  One block of 1024 threads per
// system instance (a product's rows split over 8 partial sums, the vector in
// LDS); the Krylov vectors live in a per-instance slice of the level's
// workspace, the Hessenberg matrix in LDS; sums in a fixed order.
#include <hip/hip_runtime.h>

#include "amg_internal.h"
#include "kernels.h"

namespace amg {

namespace {

constexpr int kThreads = 1024;          // 16 wavefronts per system
constexpr int kParts = 8;               // partial sums per row of a product
constexpr int kRows = kThreads / kParts;  // rows per pass of a product
constexpr int kMaxSteps = 16;

// sum over the block of one value per thread, fixed order (all threads get it)
__device__ double block_sum(double v, double* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < kThreads / 64; ++i) t += sh[i];
  __syncthreads();
  return t;
}

// y = M x for the column-major N x N matrix M: x is staged in LDS (xs), each
// row's sum split over kParts threads (coalesced column reads) and summed in
// a fixed order; y may alias nothing the call reads
__device__ void matvec(const double* __restrict__ M, const double* __restrict__ x, double* __restrict__ y, int N,
                       double* xs, double (*part)[kRows]) {
  const int tid = threadIdx.x;
  for (int c = tid; c < N; c += kThreads) xs[c] = x[c];
  __syncthreads();
  const int rl = tid % kRows, p = tid / kRows;
  for (int r0 = 0; r0 < N; r0 += kRows) {
    const int r = r0 + rl;
    double s = 0.0;
    if (r < N)
      for (int c = p; c < N; c += kParts) s += M[(int64_t)c * N + r] * xs[c];
    part[p][rl] = s;
    __syncthreads();
    if (p == 0 && r < N) {
      double t = 0.0;
      for (int q = 0; q < kParts; ++q) t += part[q][rl];
      y[r] = t;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_bottom_gmres(const BottomGroupD* __restrict__ groups,
                                                           const double* __restrict__ mats,
                                                           const int64_t* __restrict__ idx, const T* __restrict__ f,
                                                           T* __restrict__ e, T* __restrict__ e2, int m,
                                                           double* __restrict__ ws, double breakdown) {
  extern __shared__ double xs[];  // N doubles
  __shared__ double sh[kThreads / 64];
  __shared__ double part[kParts][kRows];
  __shared__ double Hs[kMaxSteps + 1][kMaxSteps];
  __shared__ double yv[kMaxSteps];
  const BottomGroupD G = groups[blockIdx.y];
  const int inst = blockIdx.x;
  if (inst >= G.ninst) return;  // uniform per block
  const int N = G.N, n = G.n;
  const int tid = threadIdx.x;
  const int64_t* id = idx + G.idx + (int64_t)inst * n;
  double* V = ws + G.ws + (int64_t)inst * (m + 1) * N;  // column j at V + j N
  const double* B = mats + G.ilub;
  const double* P = mats + G.ilup;

  // r0 = (f, 0) and beta = ||r0||
  double loc = 0.0;
  for (int r = tid; r < N; r += kThreads) {
    const double v = r < n ? (double)f[id[r]] : 0.0;
    V[r] = v;
    loc += v * v;
  }
  const double beta = sqrt(block_sum(loc, sh));
  if (beta == 0.0) {
    for (int r = tid; r < n; r += kThreads) {
      e[id[r]] = T(0);
      if (e2) e2[id[r]] = T(0);
    }
    return;
  }
  for (int r = tid; r < N; r += kThreads) V[r] /= beta;
  __syncthreads();
  int k = m;
  for (int j = 0; j < m; ++j) {
    double* w = V + (int64_t)(j + 1) * N;
    matvec(B, V + (int64_t)j * N, w, N, xs, part);
    for (int i = 0; i <= j; ++i) {  // modified Gram-Schmidt
      const double* vi = V + (int64_t)i * N;
      double pv = 0.0;
      for (int r = tid; r < N; r += kThreads) pv += w[r] * vi[r];
      const double h = block_sum(pv, sh);
      for (int r = tid; r < N; r += kThreads) w[r] -= h * vi[r];
      if (tid == 0) Hs[i][j] = h;
      __syncthreads();
    }
    double q = 0.0;
    for (int r = tid; r < N; r += kThreads) q += w[r] * w[r];
    const double hn = sqrt(block_sum(q, sh));
    if (tid == 0) Hs[j + 1][j] = hn;
    __syncthreads();
    if (hn <= breakdown * beta) {  // the Krylov space is invariant
      k = j + 1;
      break;
    }
    for (int r = tid; r < N; r += kThreads) w[r] /= hn;
    __syncthreads();
  }
  // min || beta e1 - H y || by Givens rotations, then back substitution
  if (tid == 0) {
    double g[kMaxSteps + 1];
    for (int i = 0; i <= k; ++i) g[i] = 0.0;
    g[0] = beta;
    for (int i = 0; i < k; ++i) {
      const double a = Hs[i][i], b = Hs[i + 1][i];
      const double rr = sqrt(a * a + b * b);
      const double cs = a / rr, sn = b / rr;
      for (int c = i; c < k; ++c) {
        const double t0 = Hs[i][c], t1 = Hs[i + 1][c];
        Hs[i][c] = cs * t0 + sn * t1;
        Hs[i + 1][c] = -sn * t0 + cs * t1;
      }
      const double t0 = g[i], t1 = g[i + 1];
      g[i] = cs * t0 + sn * t1;
      g[i + 1] = -sn * t0 + cs * t1;
    }
    for (int i = k - 1; i >= 0; --i) {
      double s = g[i];
      for (int c = i + 1; c < k; ++c) s -= Hs[i][c] * yv[c];
      yv[i] = s / Hs[i][i];
    }
  }
  __syncthreads();
  // u = V y into the last column (free after the last step), x = P u into
  // the first (free too), then the cells
  double* u = V + (int64_t)m * N;
  for (int r = tid; r < N; r += kThreads) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) s += V[(int64_t)i * N + r] * yv[i];
    u[r] = s;
  }
  __syncthreads();
  matvec(P, u, V, N, xs, part);
  for (int r = tid; r < n; r += kThreads) {
    const double s = V[r];
    e[id[r]] = (T)s;
    if (e2) e2[id[r]] = (T)s;
  }
}

}  // namespace

template <typename T>
void launch_bottom_gmres(const Depth& D, const double* mats, const int64_t* idx, const T* f, T* e, int iters,
                         double* ws, hipStream_t st, T* e2) {
  if (D.groups.empty()) return;
  int maxinst = 0, maxN = 1;
  for (auto& g : D.groups) {
    maxinst = std::max(maxinst, g.ninst);
    maxN = std::max(maxN, g.N);
  }
  const dim3 grid((unsigned)maxinst, (unsigned)D.groups.size());
  hipLaunchKernelGGL(k_bottom_gmres<T>, grid, dim3(kThreads), (size_t)maxN * sizeof(double), st, D.d_groups, mats,
                     idx, f, e, e2, iters, ws, 1e-14);
}

template void launch_bottom_gmres<double>(const Depth&, const double*, const int64_t*, const double*, double*, int,
                                          double*, hipStream_t, double*);
template void launch_bottom_gmres<float>(const Depth&, const double*, const int64_t*, const float*, float*, int,
                                         double*, hipStream_t, float*);

}  // namespace amg
