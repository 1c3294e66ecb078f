// HIP kernels of the multigrid path for gfx950 (CDNA4).
//
// Every cell kernel walks a tile table that covers all boxes of one
// multigrid depth of one level, one workgroup per tile, one thread per cell
// (64-wide rows of x, the fastest direction, so each wavefront reads one
// coalesced row segment).  Ghost values are read from the two stored ghost
// layers; the diagonal of the operator with the ghost fill folded in is
// computed on the fly from per-face column codes, so no coefficient array
// is streamed.  All reductions are two-stage with a fixed order, so results
// are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "amg_internal.h"
#include "kernels.h"
#include "tiles.h"

namespace amg {

template <int DIM>
struct Shape;
template <>
struct Shape<2> {
  static constexpr int X = TILE2_X, Y = TILE2_Y, Z = 1;
};
template <>
struct Shape<3> {
  static constexpr int X = TILE3_X, Y = TILE3_Y, Z = TILE3_Z;
};

// Increment of the diagonal (in units of 1/(12 h^2)) from the ghost fill of
// one face, for the cell at distance `dist` (0 or 1) from that face.  The
// end cell reads ghost 1 with weight 16 and ghost 2 with weight -1; the next
// cell reads ghost 1 with weight -1.  Coefficients of the end cell / the
// next cell in the fills of eqs. (velBCHomoDiri5th) and (Neumann5):
// Dirichlet -77/12, -505/12 / 43/12; Neumann 5/10, -75/10 / 9/10.
template <typename T>
__device__ __forceinline__ T fold(uint8_t code, int dist) {
  const int kind = code & 3;
  if (kind == 0) return T(0);
  if (dist == 0) {
    if (kind == 1) return T(16.0 * (-77.0 / 12.0)) + ((code & 4) ? T(505.0 / 12.0) : T(0));
    return T(16.0 * 0.5) + ((code & 4) ? T(7.5) : T(0));
  }
  return kind == 1 ? T(-43.0 / 12.0) : T(-0.9);
}

struct Cell {
  int x, y, z;
  int64_t c;
  bool ok;
};

template <int DIM>
__device__ __forceinline__ Cell tile_cell(const TileD& t, const BoxD& b) {
  using S = Shape<DIM>;
  const int tid = threadIdx.x;
  Cell q;
  q.x = t.x0 + tid % S::X;
  q.y = t.y0 + (tid / S::X) % S::Y;
  q.z = DIM == 3 ? t.z0 + tid / (S::X * S::Y) : 0;
  q.ok = q.x < b.n[0] && q.y < b.n[1] && (DIM == 2 || q.z < b.n[2]);
  q.c = b.off + (q.x + 2) + (int64_t)(q.y + 2) * b.s[1] + (DIM == 3 ? (int64_t)(q.z + 2) * b.s[2] : 0);
  return q;
}

// sum over directions of (-u[-2] + 16u[-1] - 30u[0] + 16u[1] - u[2])
template <typename T, int DIM>
__device__ __forceinline__ T lap_sum(const T* __restrict__ u, int64_t c, const BoxD& b) {
  T u0 = u[c];
  T acc = T(-30 * DIM) * u0;
  acc += T(16) * (u[c - 1] + u[c + 1]) - (u[c - 2] + u[c + 2]);
  const int64_t sy = b.s[1];
  acc += T(16) * (u[c - sy] + u[c + sy]) - (u[c - 2 * sy] + u[c + 2 * sy]);
  if (DIM == 3) {
    const int64_t sz = b.s[2];
    acc += T(16) * (u[c - sz] + u[c + sz]) - (u[c - 2 * sz] + u[c + 2 * sz]);
  }
  return acc;
}

// -30 DIM plus the folded fill increments of the faces within two cells
template <typename T, int DIM>
__device__ __forceinline__ T diag_units(const Cell& q, const BoxD& b, const uint8_t* __restrict__ codes) {
  T S = T(-30 * DIM);
  const int p[3] = {q.x, q.y, q.z};
  for (int d = 0; d < DIM; ++d) {
    const int lo = p[d], hi = b.n[d] - 1 - p[d];
    if (lo >= 2 && hi >= 2) continue;
    int col;
    if (DIM == 2)
      col = d == 0 ? q.y : q.x;
    else
      col = d == 0 ? q.y + b.n[1] * q.z : (d == 1 ? q.x + b.n[0] * q.z : q.x + b.n[0] * q.y);
    if (lo < 2) S += fold<T>(codes[b.code_off[d][0] + col], lo);
    if (hi < 2) S += fold<T>(codes[b.code_off[d][1] + col], hi);
  }
  return S;
}

template <typename T>
__device__ __forceinline__ T block_sum(T v, T* sh) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  return r;  // valid in thread 0
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T* sh) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh[w] = v;
  __syncthreads();
  T r = T(0);
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, sh[i]);
  return r;
}

// ---------------------------------------------------------------------------
// ghost fill: one wavefront per chunk of up to 64 face columns
template <typename T>
__global__ void __launch_bounds__(256) k_fill(const ChunkD* __restrict__ chunks, int nchunks, T* __restrict__ u,
                                              const double* __restrict__ fd, double h) {
  const int ci = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (ci >= nchunks) return;
  const ChunkD ch = chunks[ci];
  if (lane >= ch.count) return;
  const int64_t g1 = ch.dst + (int64_t)lane * ch.cstride;
  const int64_t n = ch.nstride;
  const int64_t e = g1 - n;
  T v1 = T(0), v2 = T(0);
  if (ch.kind1 == G_FILL_D || ch.kind1 == G_FILL_N || ch.kind2 == G_FILL_D || ch.kind2 == G_FILL_N) {
    const T u0 = u[e], u1 = u[e - n], u2 = u[e - 2 * n], u3 = u[e - 3 * n];
    const T g = (fd && ch.fd >= 0) ? T(fd[ch.fd + lane]) : T(0);
    const int k = (ch.kind1 == G_FILL_D || ch.kind1 == G_FILL_N) ? ch.kind1 : ch.kind2;
    T f1, f2;
    if (k == G_FILL_D) {  // eq. (velBCHomoDiri5th); 75/3 = 25
      f1 = (T(-77) * u0 + T(43) * u1 - T(17) * u2 + T(3) * u3) * T(1.0 / 12.0) + T(5) * g;
      f2 = (T(-505) * u0 + T(335) * u1 - T(145) * u2 + T(27) * u3) * T(1.0 / 12.0) + T(25) * g;
    } else {  // eq. (Neumann5), g = outward normal derivative
      f1 = (T(5) * u0 + T(9) * u1 - T(5) * u2 + u3) * T(0.1) + T(1.2 * h) * g;
      f2 = (T(-75) * u0 + T(145) * u1 - T(75) * u2 + T(15) * u3) * T(0.1) + T(6.0 * h) * g;
    }
    if (ch.kind1 == G_FILL_D || ch.kind1 == G_FILL_N) v1 = f1;
    if (ch.kind2 == G_FILL_D || ch.kind2 == G_FILL_N) v2 = f2;
  }
  if (ch.kind1 == G_EXCH) v1 = u[ch.src1 + (int64_t)lane * ch.sstride1];
  if (ch.kind2 == G_EXCH) v2 = u[ch.src2 + (int64_t)lane * ch.sstride2];
  u[g1] = v1;
  u[g1 + n] = v2;
}

// ---------------------------------------------------------------------------
// r = f - A u  (A u = alpha u + beta lap_sum); optional per-tile max |r|
template <typename T, int DIM, bool PART>
__global__ void __launch_bounds__(256) k_residual(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                  const T* __restrict__ u, const T* __restrict__ f,
                                                  T* __restrict__ r, T alpha, T beta, double* __restrict__ part) {
  __shared__ T sh[4];
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  T v = T(0);
  if (q.ok) {
    const T Au = alpha * u[q.c] + beta * lap_sum<T, DIM>(u, q.c, b);
    v = f ? f[q.c] - Au : Au;  // f == NULL: the operator itself
    r[q.c] = v;
  }
  if (PART) {
    T av = fabs(v);
    av = (av == av) ? av : T(INFINITY);  // a NaN residual must not vanish in fmax
    T m = block_max<T>(av, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = (double)m;
  }
}

// weighted Jacobi sweep: out = u + omega (f - A u) / diag
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_jacobi(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                const uint8_t* __restrict__ codes, const T* __restrict__ u,
                                                const T* __restrict__ f, T* __restrict__ out, T alpha, T beta,
                                                T omega) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  const T uc = u[q.c];
  const T Au = alpha * uc + beta * lap_sum<T, DIM>(u, q.c, b);
  const T dg = alpha + beta * diag_units<T, DIM>(q, b, codes);
  out[q.c] = uc + omega * (f[q.c] - Au) / dg;
}

// first weighted-Jacobi sweep from a zero iterate: out = omega f / diag
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_jacobi0(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                 const uint8_t* __restrict__ codes, const T* __restrict__ f,
                                                 T* __restrict__ out, T alpha, T beta, T omega) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  const T dg = alpha + beta * diag_units<T, DIM>(q, b, codes);
  out[q.c] = omega * f[q.c] / dg;
}

// red-black half-sweep of colour `col` (parity of the sum of global indices):
// cells of that colour updated simultaneously from u, the others copied
template <typename T, int DIM, bool ZERO>
__global__ void __launch_bounds__(256) k_rb(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                            const uint8_t* __restrict__ codes, const T* __restrict__ u,
                                            const T* __restrict__ f, T* __restrict__ out, T alpha, T beta,
                                            int col) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  const int par = (b.lo[0] + q.x + b.lo[1] + q.y + (DIM == 3 ? b.lo[2] + q.z : 0)) & 1;
  const T uc = ZERO ? T(0) : u[q.c];
  if (par != col) {
    out[q.c] = uc;
    return;
  }
  const T Au = ZERO ? T(0) : alpha * uc + beta * lap_sum<T, DIM>(u, q.c, b);
  const T dg = alpha + beta * diag_units<T, DIM>(q, b, codes);
  out[q.c] = uc + (f[q.c] - Au) / dg;
}

// fused residual and restriction: fc = mean over the 2^DIM children of
// (f - A u); one thread per coarse cell
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_resid_restrict(const TileD* __restrict__ ctiles,
                                                        const BoxD* __restrict__ cboxes,
                                                        const BoxD* __restrict__ fboxes, const T* __restrict__ u,
                                                        const T* __restrict__ f, T* __restrict__ fc, T alpha,
                                                        T beta) {
  const TileD t = ctiles[blockIdx.x];
  const BoxD cb = cboxes[t.box];
  const Cell q = tile_cell<DIM>(t, cb);
  if (!q.ok) return;
  const BoxD fb = fboxes[cb.fine];
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    const int x = 2 * q.x + (a & 1), y = 2 * q.y + ((a >> 1) & 1), z = DIM == 3 ? 2 * q.z + ((a >> 2) & 1) : 0;
    const int64_t c = fb.off + (x + 2) + (int64_t)(y + 2) * fb.s[1] + (DIM == 3 ? (int64_t)(z + 2) * fb.s[2] : 0);
    acc += f[c] - (alpha * u[c] + beta * lap_sum<T, DIM>(u, c, fb));
  }
  fc[q.c] = acc * T(DIM == 2 ? 0.25 : 0.125);
}

// plain restriction: fc = mean of the 2^DIM children of r
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_restrict(const TileD* __restrict__ ctiles, const BoxD* __restrict__ cboxes,
                                                  const BoxD* __restrict__ fboxes, const T* __restrict__ r,
                                                  T* __restrict__ fc) {
  const TileD t = ctiles[blockIdx.x];
  const BoxD cb = cboxes[t.box];
  const Cell q = tile_cell<DIM>(t, cb);
  if (!q.ok) return;
  const BoxD fb = fboxes[cb.fine];
  T acc = T(0);
#pragma unroll
  for (int a = 0; a < (1 << DIM); ++a) {
    const int x = 2 * q.x + (a & 1), y = 2 * q.y + ((a >> 1) & 1), z = DIM == 3 ? 2 * q.z + ((a >> 2) & 1) : 0;
    const int64_t c = fb.off + (x + 2) + (int64_t)(y + 2) * fb.s[1] + (DIM == 3 ? (int64_t)(z + 2) * fb.s[2] : 0);
    acc += r[c];
  }
  fc[q.c] = acc * T(DIM == 2 ? 0.25 : 0.125);
}

// u += face-neighbour linear interpolation of the coarse correction:
// (1 - DIM/4) e_P + 1/4 sum_d e_{P + s_d e_d}, s_d the child's side
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_prolong(const TileD* __restrict__ ftiles, const BoxD* __restrict__ fboxes,
                                                 const BoxD* __restrict__ cboxes, const T* __restrict__ ec,
                                                 T* __restrict__ u) {
  const TileD t = ftiles[blockIdx.x];
  const BoxD fb = fboxes[t.box];
  const Cell q = tile_cell<DIM>(t, fb);
  if (!q.ok) return;
  const BoxD cb = cboxes[fb.coarse];
  const int px = q.x >> 1, py = q.y >> 1, pz = q.z >> 1;
  const int64_t p = cb.off + (px + 2) + (int64_t)(py + 2) * cb.s[1] + (DIM == 3 ? (int64_t)(pz + 2) * cb.s[2] : 0);
  T v = T(1.0 - DIM * 0.25) * ec[p];
  T nb = ec[p + ((q.x & 1) ? 1 : -1)] + ec[p + ((q.y & 1) ? cb.s[1] : -cb.s[1])];
  if (DIM == 3) nb += ec[p + ((q.z & 1) ? cb.s[2] : -cb.s[2])];
  u[q.c] += v + T(0.25) * nb;
}

// exact bottom solve: e = M f for every instance of every group
template <typename T>
__global__ void __launch_bounds__(256) k_bottom(const BottomGroupD* __restrict__ groups,
                                                const double* __restrict__ mats, const int64_t* __restrict__ idx,
                                                const T* __restrict__ f, T* __restrict__ e) {
  constexpr int NI = 8, KC = 512;
  __shared__ double xs[NI][KC];
  const BottomGroupD G = groups[blockIdx.y];
  const int r = blockIdx.x * 256 + threadIdx.x;
  if ((int)(blockIdx.x * 256) >= G.n) return;  // uniform per block
  const double* M = mats + G.mat;
  for (int i0 = 0; i0 < G.ninst; i0 += NI) {
    const int ni = min(NI, G.ninst - i0);
    double acc[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) acc[i] = 0.0;
    for (int k0 = 0; k0 < G.n; k0 += KC) {
      const int kc = min(KC, G.n - k0);
      __syncthreads();
      for (int j = threadIdx.x; j < ni * kc; j += 256) {
        const int i = j / kc, k = j % kc;
        xs[i][k] = (double)f[idx[G.idx + (int64_t)(i0 + i) * G.n + k0 + k]];
      }
      __syncthreads();
      if (r < G.n) {
        for (int k = 0; k < kc; ++k) {
          const double m = M[(int64_t)(k0 + k) * G.n + r];
#pragma unroll
          for (int i = 0; i < NI; ++i) acc[i] += m * xs[i][k];
        }
      }
    }
    if (r < G.n)
      for (int i = 0; i < ni; ++i) e[idx[G.idx + (int64_t)(i0 + i) * G.n + r]] = (T)acc[i];
  }
}

// ---------------------------------------------------------------------------
// reductions and vector updates (interior cells only)
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_tile_sum(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                  const T* __restrict__ a, double* __restrict__ part) {
  __shared__ double sh[4];
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  double v = q.ok ? (double)a[q.c] : 0.0;
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_tile_absmax(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                     const T* __restrict__ a, double* __restrict__ part) {
  __shared__ double sh[4];
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  double v = q.ok ? fabs((double)a[q.c]) : 0.0;
  v = block_max<double>(v, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// out[slot] = max of part[0..n); NaN propagates (fmax drops NaN, so count it)
__global__ void __launch_bounds__(256) k_reduce_max(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double sh[4];
  double v = 0.0;
  int bad = 0;
  for (int i = threadIdx.x; i < n; i += 256) {
    const double p = part[i];
    if (!(p <= 1e300)) bad = 1;
    v = fmax(v, p);
  }
  v = block_max<double>(v, sh);
  __syncthreads();
  __shared__ int anybad;
  if (threadIdx.x == 0) anybad = 0;
  __syncthreads();
  if (bad) atomicOr(&anybad, 1);
  __syncthreads();
  if (threadIdx.x == 0) *out = anybad ? __builtin_nan("") : v;
}

// per-component sums of tile partials in a fixed order; one block per component
__global__ void __launch_bounds__(256) k_comp_sum(const double* __restrict__ part, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ ids, double* __restrict__ out) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double v = 0.0;
  for (int j = ptr[c] + threadIdx.x; j < ptr[c + 1]; j += 256) v += part[ids[j]];
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) out[c] = v;
}

// a -= coef * sum[comp] on cells of components with flag[comp] != 0
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_comp_shift(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                    T* __restrict__ a, const double* __restrict__ delta) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  const double d = delta[b.comp];
  if (d != 0.0) a[q.c] = (T)((double)a[q.c] - d);
}

// per-component deltas: delta[c] = flag[c] ? (sum[c] - bsum[c]) * scale / cnt[c] : 0
__global__ void k_comp_delta(const double* __restrict__ sum, const double* __restrict__ bsum,
                             const int32_t* __restrict__ flag, const double* __restrict__ cnt, int ncomp,
                             double scale_sum, double scale_b, double* __restrict__ delta, double* __restrict__ defect) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncomp) return;
  double dv = 0.0;
  if (flag[c]) {
    const double df = sum[c] * scale_sum - (bsum ? bsum[c] * scale_b : 0.0);
    if (defect) defect[c] = df;
    dv = df / (cnt[c] * scale_sum);
  }
  delta[c] = dv;
}

// sum of face data over Neumann-filled ghost columns of each chunk
__global__ void __launch_bounds__(256) k_chunk_fdsum(const ChunkD* __restrict__ chunks, int nchunks,
                                                     const double* __restrict__ fd, double* __restrict__ part) {
  const int ci = blockIdx.x * 256 + threadIdx.x;
  if (ci >= nchunks) return;
  const ChunkD ch = chunks[ci];
  double s = 0.0;
  if (ch.kind1 == G_FILL_N && ch.fd >= 0)
    for (int i = 0; i < ch.count; ++i) s += fd[ch.fd + i];
  part[ci] = s;
}

// x += s e (x FP64, e FP32 or FP64), s = scal[0]
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_update(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                double* __restrict__ x, const T* __restrict__ e,
                                                const double* __restrict__ scal) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  x[q.c] += scal[0] * (double)e[q.c];
}

// r32 = fp32(r / s), s = scal[0]
template <int DIM>
__global__ void __launch_bounds__(256) k_to32(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                              const double* __restrict__ r, float* __restrict__ r32,
                                              const double* __restrict__ scal) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  r32[q.c] = (float)(r[q.c] / scal[0]);
}

// f_shift = f - delta[comp]
template <int DIM>
__global__ void __launch_bounds__(256) k_shift_copy(const TileD* __restrict__ tiles, const BoxD* __restrict__ boxes,
                                                    const double* __restrict__ f, double* __restrict__ out,
                                                    const double* __restrict__ delta) {
  const TileD t = tiles[blockIdx.x];
  const BoxD b = boxes[t.box];
  const Cell q = tile_cell<DIM>(t, b);
  if (!q.ok) return;
  out[q.c] = f[q.c] - delta[b.comp];
}

// scal[dst] = src[0] (device-side scalar copy, keeps the scale on the device)
__global__ void k_set_scale(const double* __restrict__ src, double* __restrict__ dst) { *dst = *src; }

// zero a whole buffer (used in place of memset nodes in captured graphs)
template <typename T>
__global__ void k_zero(T* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = T(0);
}

// ===========================================================================
// host-side launchers
namespace {
inline dim3 g1(size_t n) { return dim3((unsigned)n); }
}  // namespace

template <typename T>
void launch_fill(const Depth& D, T* u, const double* fd, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL(k_fill<T>, dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, u, fd, D.h);
}

template <typename T>
void launch_residual(int dim, const Depth& D, bool all, const T* u, const T* f, T* r, T alpha, T beta,
                     double* part, hipStream_t st) {
  const TileD* tl = all ? D.d_tiles : D.d_stiles;
  const size_t n = all ? D.tiles.size() : D.stiles.size();
  if (!n) return;
  if (dim == 2) {
    if (part)
      hipLaunchKernelGGL((k_residual<T, 2, true>), g1(n), dim3(256), 0, st, tl, D.d_box, u, f, r, alpha, beta, part);
    else
      hipLaunchKernelGGL((k_residual<T, 2, false>), g1(n), dim3(256), 0, st, tl, D.d_box, u, f, r, alpha, beta, part);
  } else {
    if (part)
      hipLaunchKernelGGL((k_residual<T, 3, true>), g1(n), dim3(256), 0, st, tl, D.d_box, u, f, r, alpha, beta, part);
    else
      hipLaunchKernelGGL((k_residual<T, 3, false>), g1(n), dim3(256), 0, st, tl, D.d_box, u, f, r, alpha, beta, part);
  }
}

template <typename T>
void launch_jacobi(int dim, const Depth& D, const T* u, const T* f, T* out, T alpha, T beta, T omega, bool zero,
                   hipStream_t st) {
  const size_t n = D.stiles.size();
  if (!n) return;
  if (dim == 2) {
    if (zero)
      hipLaunchKernelGGL((k_jacobi0<T, 2>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, f, out, alpha, beta,
                         omega);
    else
      hipLaunchKernelGGL((k_jacobi<T, 2>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, u, f, out, alpha,
                         beta, omega);
  } else {
    if (zero)
      hipLaunchKernelGGL((k_jacobi0<T, 3>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, f, out, alpha, beta,
                         omega);
    else
      hipLaunchKernelGGL((k_jacobi<T, 3>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, u, f, out, alpha,
                         beta, omega);
  }
}

template <typename T>
void launch_rb(int dim, const Depth& D, const T* u, const T* f, T* out, T alpha, T beta, int col, bool zero,
               hipStream_t st) {
  const size_t n = D.stiles.size();
  if (!n) return;
  if (dim == 2) {
    if (zero)
      hipLaunchKernelGGL((k_rb<T, 2, true>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, u, f, out, alpha,
                         beta, col);
    else
      hipLaunchKernelGGL((k_rb<T, 2, false>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, u, f, out, alpha,
                         beta, col);
  } else {
    if (zero)
      hipLaunchKernelGGL((k_rb<T, 3, true>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, u, f, out, alpha,
                         beta, col);
    else
      hipLaunchKernelGGL((k_rb<T, 3, false>), g1(n), dim3(256), 0, st, D.d_stiles, D.d_box, D.d_codes, u, f, out, alpha,
                         beta, col);
  }
}

template <typename T>
void launch_resid_restrict(int dim, const Depth& F, const Depth& C, const T* u, const T* f, T* fc, T alpha, T beta,
                           hipStream_t st) {
  const size_t n = C.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_resid_restrict<T, 2>), g1(n), dim3(256), 0, st, C.d_tiles, C.d_box, F.d_box, u, f, fc, alpha,
                       beta);
  else
    hipLaunchKernelGGL((k_resid_restrict<T, 3>), g1(n), dim3(256), 0, st, C.d_tiles, C.d_box, F.d_box, u, f, fc, alpha,
                       beta);
}

template <typename T>
void launch_restrict(int dim, const Depth& F, const Depth& C, const T* r, T* fc, hipStream_t st) {
  const size_t n = C.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_restrict<T, 2>), g1(n), dim3(256), 0, st, C.d_tiles, C.d_box, F.d_box, r, fc);
  else
    hipLaunchKernelGGL((k_restrict<T, 3>), g1(n), dim3(256), 0, st, C.d_tiles, C.d_box, F.d_box, r, fc);
}

template <typename T>
void launch_prolong(int dim, const Depth& F, const Depth& C, const T* ec, T* u, hipStream_t st) {
  const size_t n = F.stiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_prolong<T, 2>), g1(n), dim3(256), 0, st, F.d_stiles, F.d_box, C.d_box, ec, u);
  else
    hipLaunchKernelGGL((k_prolong<T, 3>), g1(n), dim3(256), 0, st, F.d_stiles, F.d_box, C.d_box, ec, u);
}

template <typename T>
void launch_bottom(const Depth& D, const double* mats, const int64_t* idx, const T* f, T* e, hipStream_t st) {
  if (D.groups.empty()) return;
  int maxn = 0;
  for (auto& g : D.groups) maxn = std::max(maxn, g.n);
  hipLaunchKernelGGL(k_bottom<T>, dim3((maxn + 255) / 256, (unsigned)D.groups.size()), dim3(256), 0, st, D.d_groups,
                     mats, idx, f, e);
}

template <typename T>
void launch_tile_sum(int dim, const Depth& D, const T* a, double* part, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (dim == 2)
    hipLaunchKernelGGL((k_tile_sum<T, 2>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, a, part);
  else
    hipLaunchKernelGGL((k_tile_sum<T, 3>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, a, part);
}

template <typename T>
void launch_tile_absmax(int dim, const Depth& D, const T* a, double* part, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (dim == 2)
    hipLaunchKernelGGL((k_tile_absmax<T, 2>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, a, part);
  else
    hipLaunchKernelGGL((k_tile_absmax<T, 3>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, a, part);
}

void launch_reduce_max(const double* part, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_max, dim3(1), dim3(256), 0, st, part, n, out);
}

void launch_comp_sum(const double* part, const int32_t* ptr, const int32_t* ids, int ncomp, double* out,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_comp_sum, dim3(ncomp), dim3(256), 0, st, part, ptr, ids, out);
}

void launch_comp_delta(const double* sum, const double* bsum, const int32_t* flag, const double* cnt, int ncomp,
                       double scale_sum, double scale_b, double* delta, double* defect, hipStream_t st) {
  hipLaunchKernelGGL(k_comp_delta, dim3((ncomp + 255) / 256), dim3(256), 0, st, sum, bsum, flag, cnt, ncomp, scale_sum,
                     scale_b, delta, defect);
}

template <typename T>
void launch_comp_shift(int dim, const Depth& D, T* a, const double* delta, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (dim == 2)
    hipLaunchKernelGGL((k_comp_shift<T, 2>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, a, delta);
  else
    hipLaunchKernelGGL((k_comp_shift<T, 3>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, a, delta);
}

void launch_chunk_fdsum(const Depth& D, const double* fd, double* part, hipStream_t st) {
  const int n = (int)D.chunks.size();
  hipLaunchKernelGGL(k_chunk_fdsum, dim3((n + 255) / 256), dim3(256), 0, st, D.d_chunks, n, fd, part);
}

template <typename T>
void launch_update(int dim, const Depth& D, double* x, const T* e, const double* scal, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (dim == 2)
    hipLaunchKernelGGL((k_update<T, 2>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, x, e, scal);
  else
    hipLaunchKernelGGL((k_update<T, 3>), g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, x, e, scal);
}

void launch_to32(int dim, const Depth& D, const double* r, float* r32, const double* scal, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (dim == 2)
    hipLaunchKernelGGL(k_to32<2>, g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, r, r32, scal);
  else
    hipLaunchKernelGGL(k_to32<3>, g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, r, r32, scal);
}

void launch_shift_copy(int dim, const Depth& D, const double* f, double* out, const double* delta, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (dim == 2)
    hipLaunchKernelGGL(k_shift_copy<2>, g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, f, out, delta);
  else
    hipLaunchKernelGGL(k_shift_copy<3>, g1(n), dim3(256), 0, st, D.d_tiles, D.d_box, f, out, delta);
}

void launch_set_scale(const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scale, dim3(1), dim3(1), 0, st, src, dst);
}

template <typename T>
void launch_zero(T* a, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n);
}

#define INST(T)                                                                                                   \
  template void launch_fill<T>(const Depth&, T*, const double*, hipStream_t);                                     \
  template void launch_residual<T>(int, const Depth&, bool, const T*, const T*, T*, T, T, double*, hipStream_t);  \
  template void launch_jacobi<T>(int, const Depth&, const T*, const T*, T*, T, T, T, bool, hipStream_t);          \
  template void launch_rb<T>(int, const Depth&, const T*, const T*, T*, T, T, int, bool, hipStream_t);            \
  template void launch_resid_restrict<T>(int, const Depth&, const Depth&, const T*, const T*, T*, T, T,           \
                                         hipStream_t);                                                            \
  template void launch_restrict<T>(int, const Depth&, const Depth&, const T*, T*, hipStream_t);                   \
  template void launch_prolong<T>(int, const Depth&, const Depth&, const T*, T*, hipStream_t);                    \
  template void launch_bottom<T>(const Depth&, const double*, const int64_t*, const T*, T*, hipStream_t);         \
  template void launch_tile_sum<T>(int, const Depth&, const T*, double*, hipStream_t);                            \
  template void launch_tile_absmax<T>(int, const Depth&, const T*, double*, hipStream_t);                         \
  template void launch_comp_shift<T>(int, const Depth&, T*, const double*, hipStream_t);                          \
  template void launch_update<T>(int, const Depth&, double*, const T*, const double*, hipStream_t);               \
  template void launch_zero<T>(T*, int64_t, hipStream_t);
INST(double)
INST(float)

}  // namespace amg
