// The coarse tail of the FP32 V-cycle in three launches.  Below a depth of
// at most 4096 cells (16^3, 64^2) every multigrid operation is a few
// microseconds of launch and cache set-up around almost no work, ten of them
// per depth.  Where every depth from there down holds one box whose faces
// are all filled uniformly (both ghost layers from its own rows) or wrap
// onto the box itself (a periodic direction that the box spans), and the
// coarsest is one exact bottom system, one workgroup runs the whole
// down-leg in LDS (pre-smoothing from zero, residual and restriction, mean
// removal of a singular problem, depth after depth), the existing bottom
// kernel solves the coarsest system, and one workgroup runs the up-leg
// (prolongation, post-smoothing).  Each depth's box is staged in LDS with two
// ghost layers, filled there before every operator application; each thread
// keeps the LDS places, inverse diagonals and colours of its (at most four)
// cells in registers, and a half-sweep computes its new values before it
// writes them in place.  The arithmetic per cell is the tiled
// kernels' (the stencil in the same order, the same fills, folded diagonal,
// prolongation and mean removal), so the two paths agree to the rounding of
// the diagonal's and the mean's sums.
#include <hip/hip_runtime.h>

#include "amg_internal.h"
#include "kernels.h"
#include "stencil.h"

namespace amg {

namespace {

constexpr int kThreads = 1024;

// one tail depth's box in LDS: padded layout with two ghost layers, x fastest
template <int DIM>
struct Lay {
  int n[3], sy, sz;  // cells; strides of y and z in the padded layout
  float r0, r1;      // 1 / n[0], 1 / n[1]
  __device__ explicit Lay(const BoxD& b) {
    n[0] = b.n[0];
    n[1] = b.n[1];
    n[2] = DIM == 3 ? b.n[2] : 1;
    sy = n[0] + 4;
    sz = sy * (n[1] + 4);
    r0 = 1.0f / (float)n[0];
    r1 = 1.0f / (float)n[1];
  }
  __device__ int at(int x, int y, int z) const { return (x + 2) + (y + 2) * sy + (DIM == 3 ? (z + 2) * sz : 0); }
  __device__ int cells() const { return n[0] * n[1] * n[2]; }
  __device__ int padded() const { return sz * (DIM == 3 ? n[2] + 4 : 1); }
  __device__ int stride(int d) const { return d == 0 ? 1 : (d == 1 ? sy : sz); }
  // cell i (x fastest) of the box; the quotients come from the reciprocals
  // (exact: a box here has at most 4096 cells, so (i + 1/2) / n is at least
  // 1 / (2n) from an integer, far above the rounding of the product)
  __device__ void cell(int i, int& x, int& y, int& z) const {
    const int row = (int)(((float)i + 0.5f) * r0);
    x = i - row * n[0];
    if (DIM == 3) {
      z = (int)(((float)row + 0.5f) * r1);
      y = row - z * n[1];
    } else {
      y = row;
      z = 0;
    }
  }
};

// both ghost layers of every face: from the face rows (uniform fills), or,
// in a direction that wraps onto the box, the cells at the other end.  The
// faces' rows are spread over all threads at once (a ghost reads only cells
// of its own row, so the faces are independent).
template <int DIM>
__device__ void fill(const Lay<DIM>& L, const BoxD& b, const int32_t* wrap, float* u) {
  int rows[3];
#pragma unroll
  for (int d = 0; d < DIM; ++d) rows[d] = L.n[d == 0 ? 1 : 0] * (DIM == 3 ? L.n[d == 2 ? 1 : 2] : 1);
  const int total = 2 * (rows[0] + rows[1] + (DIM == 3 ? rows[2] : 0));
  for (int r = (int)threadIdx.x; r < total; r += kThreads) {
    // face (d, side) and row j of the item
    int d = 0, j = r;
#pragma unroll
    for (int k = 0; k < DIM - 1; ++k)
      if (d == k && j >= 2 * rows[k]) {
        j -= 2 * rows[k];
        d = k + 1;
      }
    const int side = j >= rows[d] ? 1 : 0;
    j -= side * rows[d];
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    const int m1 = L.n[d1];
    const int st = L.stride(d);
    const int in = side ? -st : st;
    int q[3] = {0, 0, 0};
    q[d] = side ? L.n[d] - 1 : 0;
    const int r2 = DIM == 3 ? (int)(((float)j + 0.5f) / (float)m1) : 0;
    q[d1] = j - r2 * m1;
    if (DIM == 3) q[d2] = r2;
    const int e0 = L.at(q[0], q[1], q[2]);
    if (wrap[d]) {  // ghost layer g is the cell g from the other end
      const int far = (L.n[d] - 1) * in;  // from the face cell to the other end of its row
      u[e0 - in] = u[e0 + far];
      u[e0 - 2 * in] = u[e0 + far - in];
      continue;
    }
    const uint8_t cd = b.ucode[d][side];
    const float u0 = u[e0], u1 = u[e0 + in], u2 = u[e0 + 2 * in], u3 = u[e0 + 3 * in];
    u[e0 - in] = ghost1<float>(cd, u0, u1, u2, u3);
    u[e0 - 2 * in] = ghost2<float>(cd, u0, u1, u2, u3);
  }
}

// inverse of the folded diagonal of cell (x, y, z)
template <int DIM>
__device__ float inv_diag(const Lay<DIM>& L, const BoxD& b, int x, int y, int z, float alpha, float beta) {
  float S = float(-30 * DIM);
  const int q[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int lo = q[d], hi = L.n[d] - 1 - q[d];
    if (lo < 2) S += fold<float>(b.ucode[d][0], lo);
    if (hi < 2) S += fold<float>(b.ucode[d][1], hi);
  }
  return 1.0f / (alpha + beta * S);
}

// (A u) at element e: alpha u + beta (the stencil sum), in the tiled sweep's order
template <int DIM>
__device__ float apply(const Lay<DIM>& L, const float* u, int e, float alpha, float beta) {
  const int sm = DIM == 3 ? L.sz : L.sy;  // the march direction of the tiled kernels
  float ls = 16.0f * (u[e - 1] + u[e + 1]) - (u[e - 2] + u[e + 2]) + 16.0f * (u[e - sm] + u[e + sm]) -
             (u[e - 2 * sm] + u[e + 2 * sm]) + float(-30 * DIM) * u[e];
  if (DIM == 3) ls += 16.0f * (u[e - L.sy] + u[e + L.sy]) - (u[e - 2 * L.sy] + u[e + 2 * L.sy]);
  return alpha * u[e] + beta * ls;
}

template <int DIM>
__device__ int colour(const BoxD& b, int x, int y, int z) {
  return (b.lo[0] + b.lo[1] + (DIM == 3 ? b.lo[2] : 0) + x + y + z) & 1;
}

// The cells a thread owns in a depth: cell i = threadIdx.x + k kThreads,
// k < kOwn (a tail depth has at most kOwn kThreads cells), with their LDS
// elements, inverse folded diagonals and colours kept in registers for the
// depth's sweeps.
constexpr int kOwn = 4;
static_assert(kOwn * kThreads >= kTailMaxCells, "a tail depth's cells exceed its workgroup's share");

template <int DIM>
struct Own {
  int e[kOwn];
  float iv[kOwn];
  int col[kOwn];  // red-black colour; -1: no cell
  __device__ Own(const Lay<DIM>& L, const BoxD& b, const TailDepth& D) {
#pragma unroll
    for (int k = 0; k < kOwn; ++k) {
      const int i = (int)threadIdx.x + k * kThreads;
      e[k] = 0;
      iv[k] = 0.0f;
      col[k] = -1;
      if (i < L.cells()) {
        int x, y, z;
        L.cell(i, x, y, z);
        e[k] = L.at(x, y, z);
        iv[k] = inv_diag<DIM>(L, b, x, y, z, D.alpha, D.beta);
        col[k] = colour<DIM>(b, x, y, z);
      }
    }
  }
};

// the first sweep from zero: red-black (colour 0 only) or Jacobi
template <int DIM>
__device__ void sweep_zero(const Own<DIM>& W, const float* f, float* u, int rb, float omega) {
#pragma unroll
  for (int k = 0; k < kOwn; ++k)
    if (W.col[k] >= 0) u[W.e[k]] = (!rb || W.col[k] == 0) ? omega * f[W.e[k]] * W.iv[k] : 0.0f;
}

// one red-black half-sweep of colour col (col < 0: a Jacobi sweep) in
// place: every new value is computed from the old iterate first, then
// written (the same values as a sweep from u into a second buffer)
template <int DIM>
__device__ void sweep(const Lay<DIM>& L, const Own<DIM>& W, const TailDepth& D, const float* f, float* u, int col,
                      float omega) {
  float nv[kOwn];
#pragma unroll
  for (int k = 0; k < kOwn; ++k) {
    nv[k] = 0.0f;
    if (W.col[k] >= 0 && (col < 0 || W.col[k] == col)) {
      const int e = W.e[k];
      const float Au = apply<DIM>(L, u, e, D.alpha, D.beta);
      nv[k] = u[e] + omega * (f[e] - Au) * W.iv[k];
    }
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kOwn; ++k)
    if (W.col[k] >= 0 && (col < 0 || W.col[k] == col)) u[W.e[k]] = nv[k];
}

// nsw sweeps on u in place (from zero: u is written first)
template <int DIM>
__device__ void smooth(const Lay<DIM>& L, const BoxD& b, const TailDepth& D, const Own<DIM>& W, const float* f,
                       float* u, int nsw, bool from_zero, int rb, float omega) {
  if (nsw <= 0) {
    if (from_zero) {
      for (int i = (int)threadIdx.x; i < L.padded(); i += kThreads) u[i] = 0.0f;
      __syncthreads();
    }
    return;
  }
  int h = 0;
  if (from_zero) {
    sweep_zero<DIM>(W, f, u, rb, omega);
    __syncthreads();
    h = 1;
  }
  const int nh = rb ? 2 * nsw : nsw;
  for (; h < nh; ++h) {
    fill<DIM>(L, b, D.wrap, u);
    __syncthreads();
    sweep<DIM>(L, W, D, f, u, rb ? (h & 1) : -1, omega);
    __syncthreads();
  }
}

template <int DIM>
__device__ void load(const Lay<DIM>& L, const BoxD& b, const float* __restrict__ g, float* s) {
#pragma unroll 4
  for (int i = (int)threadIdx.x; i < L.cells(); i += kThreads) {
    int x, y, z;
    L.cell(i, x, y, z);
    s[L.at(x, y, z)] = g[cell_index<DIM>(b, x, y, z)];
  }
}

template <int DIM>
__device__ void store(const Lay<DIM>& L, const BoxD& b, const float* s, float* __restrict__ g) {
#pragma unroll 4
  for (int i = (int)threadIdx.x; i < L.cells(); i += kThreads) {
    int x, y, z;
    L.cell(i, x, y, z);
    g[cell_index<DIM>(b, x, y, z)] = s[L.at(x, y, z)];
  }
}

// Down-leg: depth d[0] .. d[nd-2] pre-smoothed from zero, each restricted
// into the next; the smoothed iterates and the restricted right-hand sides
// are written to the depths' buffers (e, f).  LDS: the iterate u of the
// depth and the right-hand sides of the depth and the next, alternating.
template <int DIM>
__global__ void __launch_bounds__(kThreads) k_tail_down(TailArgs A) {
  extern __shared__ float lds[];
  __shared__ double sh[kThreads / 64];
  __shared__ double mean;
  const Lay<DIM> L0(A.d[0].b);
  float* U = lds;
  float* F[2] = {U + L0.padded(), U + 2 * L0.padded()};  // F[1] holds odd depths (at most d[1]'s size)
  load<DIM>(L0, A.d[0].b, A.d[0].f, F[0]);
  for (int k = 0; k + 1 < A.nd; ++k) {
    const TailDepth& D = A.d[k];
    const TailDepth& C = A.d[k + 1];
    const Lay<DIM> L(D.b), Lc(C.b);
    const float* f = F[k & 1];
    float* fc = F[(k + 1) & 1];
    const Own<DIM> W(L, D.b, D);
    __syncthreads();  // the first depth's right-hand side loaded
    float* u = U;
    smooth<DIM>(L, D.b, D, W, f, u, A.nu1, true, A.rb, A.omega);
    store<DIM>(L, D.b, u, D.e);
    fill<DIM>(L, D.b, D.wrap, u);
    __syncthreads();
    // residual and restriction: the mean of the 2^D children's residuals
#pragma unroll 4
    for (int i = (int)threadIdx.x; i < Lc.cells(); i += kThreads) {
      int X, Y, Z;
      Lc.cell(i, X, Y, Z);
      float acc = 0.0f;
#pragma unroll
      for (int a = 0; a < (1 << DIM); ++a) {
        const int e = L.at(2 * X + (a & 1), 2 * Y + ((a >> 1) & 1), DIM == 3 ? 2 * Z + ((a >> 2) & 1) : 0);
        acc += f[e] - apply<DIM>(L, u, e, D.alpha, D.beta);
      }
      fc[Lc.at(X, Y, Z)] = acc * float(DIM == 2 ? 0.25 : 0.125);
    }
    __syncthreads();
    if (A.singular) {  // the one component's mean, removed (as the small-depth mean removal)
      double v = 0.0;
      for (int i = (int)threadIdx.x; i < Lc.cells(); i += kThreads) {
        int X, Y, Z;
        Lc.cell(i, X, Y, Z);
        v += (double)fc[Lc.at(X, Y, Z)];
      }
      v = block_sum<double>(v, sh);
      if (threadIdx.x == 0) mean = v / C.cnt;
      __syncthreads();
      const double m = mean;
      for (int i = (int)threadIdx.x; i < Lc.cells(); i += kThreads) {
        int X, Y, Z;
        Lc.cell(i, X, Y, Z);
        const int e = Lc.at(X, Y, Z);
        fc[e] = (float)((double)fc[e] - m);
      }
      __syncthreads();
    }
    store<DIM>(Lc, C.b, fc, C.f);
    __syncthreads();
  }
}

// Up-leg: from the bottom's solution (in d[nd-1].e), for depth nd-2 .. 0:
// the iterate saved by the down-leg, plus the prolonged correction, then
// post-smoothing; the result of depth 0 goes to its buffer e.  LDS: the
// coarse correction, then u and f of the depth.
template <int DIM>
__global__ void __launch_bounds__(kThreads) k_tail_up(TailArgs A) {
  extern __shared__ float lds[];
  const Lay<DIM> L0(A.d[0].b), L1(A.d[1].b);
  float* Cb = lds;                // coarse correction (at most the second depth's size)
  float* U = Cb + L1.padded();
  float* F = U + L0.padded();
  {
    const TailDepth& B = A.d[A.nd - 1];
    load<DIM>(Lay<DIM>(B.b), B.b, B.e, Cb);
    __syncthreads();
  }
  for (int k = A.nd - 2; k >= 0; --k) {
    const TailDepth& D = A.d[k];
    const TailDepth& C = A.d[k + 1];
    const Lay<DIM> L(D.b), Lc(C.b);
    load<DIM>(L, D.b, D.e, U);
    load<DIM>(L, D.b, D.f, F);
    const Own<DIM> W(L, D.b, D);
    fill<DIM>(Lc, C.b, C.wrap, Cb);
    __syncthreads();
    // u += (1 - D/4) e_P + 1/4 sum_d e_(P + s_d e_d), s_d the child's side
#pragma unroll 4
    for (int i = (int)threadIdx.x; i < L.cells(); i += kThreads) {
      int x, y, z;
      L.cell(i, x, y, z);
      const int q = Lc.at(x >> 1, y >> 1, z >> 1);
      float common = float(1.0 - DIM * 0.25) * Cb[q] + 0.25f * Cb[q + ((y & 1) ? Lc.sy : -Lc.sy)];
      if (DIM == 3) common += 0.25f * Cb[q + ((z & 1) ? Lc.sz : -Lc.sz)];
      U[L.at(x, y, z)] += common + 0.25f * Cb[q + ((x & 1) ? 1 : -1)];
    }
    __syncthreads();
    smooth<DIM>(L, D.b, D, W, F, U, A.nu2, false, A.rb, A.omega);
    if (k == 0) {
      store<DIM>(L, D.b, U, D.e);
    } else {
      for (int i = (int)threadIdx.x; i < L.padded(); i += kThreads) Cb[i] = U[i];
      __syncthreads();
    }
  }
}

}  // namespace

size_t tail_lds_bytes(int dim, const TailArgs& A) {
  auto padded = [&](const BoxD& b) {
    return (size_t)(b.n[0] + 4) * (b.n[1] + 4) * (dim == 3 ? b.n[2] + 4 : 1);
  };
  return (2 * padded(A.d[0].b) + padded(A.d[1].b)) * sizeof(float);
}

size_t tail_lds_limit() {
  // the device's LDS per workgroup, less the legs' static LDS
  static size_t limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
                                                  hipSuccess)
      return (size_t)0;
    return v > 1024 ? (size_t)(v - 1024) : (size_t)0;
  }();
  return limit;
}

void tail_prepare() {
  // dynamic LDS above the default limit: ask for the device's (a failure
  // leaves the default, and a tail that needs more is not run)
  const size_t bytes = tail_lds_limit();
  for (const void* k : {(const void*)k_tail_down<2>, (const void*)k_tail_down<3>, (const void*)k_tail_up<2>,
                        (const void*)k_tail_up<3>})
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  (void)hipGetLastError();
}

void launch_tail_down(int dim, const TailArgs& A, hipStream_t st) {
  const size_t lds = tail_lds_bytes(dim, A);
  if (dim == 2)
    hipLaunchKernelGGL(k_tail_down<2>, dim3(1), dim3(kThreads), lds, st, A);
  else
    hipLaunchKernelGGL(k_tail_down<3>, dim3(1), dim3(kThreads), lds, st, A);
}

void launch_tail_up(int dim, const TailArgs& A, hipStream_t st) {
  const size_t lds = tail_lds_bytes(dim, A);
  if (dim == 2)
    hipLaunchKernelGGL(k_tail_up<2>, dim3(1), dim3(kThreads), lds, st, A);
  else
    hipLaunchKernelGGL(k_tail_up<3>, dim3(1), dim3(kThreads), lds, st, A);
}

}  // namespace amg
