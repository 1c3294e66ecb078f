// HIP kernels of the multigrid path for gfx950 (CDNA4).
//
// Layout of the work.  Every cell kernel walks a tile table covering all
// boxes of one multigrid depth of one level.  A tile is a column block that
// is marched along the last direction (y in 2D, z in 3D): in 2D one
// wavefront of 64 consecutive x cells, in 3D a 64 x 4 block of (x, y)
// columns (four wavefronts).  Each thread keeps the five values of its own
// column at offsets -2..+2 along the march direction in registers, so every
// cell value is fetched from memory once per sweep for that direction; the
// x (and y) neighbours are re-read from the L1/L2 caches, where the
// neighbouring columns just put them.  Blocks are ordered so that each of
// the 8 XCDs walks one contiguous part of the tile table (neighbouring tiles
// share that XCD's L2).
//
// Ghost values are read from the two stored ghost layers.  The diagonal of
// the operator with the ghost fill folded in is computed on the fly from
// per-face column codes (no coefficient array is streamed), and its inverse
// is a constant away from the faces.  All reductions are two-stage with a
// fixed order, so results are bitwise reproducible.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "amg_internal.h"
#include "kernels.h"
#include "stencil.h"
#include "tiles.h"

namespace amg {

// XCD-aware block order: the hardware hands consecutive workgroups to the 8
// XCDs in turn, so block b runs on XCD b % 8.  Block b takes tile
// (b % 8) * ceil(n/8) + b / 8: each XCD walks one contiguous eighth of the
// (spatially ordered) tile table.
__device__ __forceinline__ int tile_of_block(int n) {
  const int per = (n + 7) >> 3;
  const int t = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  return t < n ? t : -1;
}

template <int DIM>
constexpr int block_threads() {
  return DIM == 2 ? 64 : 256;
}

// One thread's column of a tile: cells (x, y, p) for p in [p0, p1), with p
// the coordinate along the march direction (y in 2D, z in 3D).
// Each thread owns two neighbouring x-columns (x, x+1), x even, so every
// row access is a 2-element vector load (rows are aligned: the first
// interior cell of every row sits on an even element).
struct Column {
  int x, y;        // x even; 2D: y unused
  int p0, p1;
  bool ok, ok1;    // cell x / cell x+1 inside the box
  int64_t base;    // element of (x, y, stored march index 0)
  int64_t sm;      // march stride
};

template <int DIM>
__device__ __forceinline__ Column column_at(const TileD& t, const BoxD& b, int tid) {
  Column c;
  c.x = t.x0 + 2 * (DIM == 2 ? tid : (tid & 63));
  c.y = DIM == 2 ? 0 : t.y0 + (tid >> 6);
  c.ok = c.x < b.n[0] && (DIM == 2 || c.y < b.n[1]);
  c.ok1 = c.ok && c.x + 1 < b.n[0];
  c.p0 = DIM == 2 ? t.y0 : t.z0;
  c.p1 = min(c.p0 + t.len, b.n[DIM - 1]);
  c.sm = b.s[DIM - 1];
  c.base = b.off + (c.x + 2) + (DIM == 3 ? (int64_t)(c.y + 2) * b.s[1] : 0);
  return c;
}

template <int DIM>
__device__ __forceinline__ Column column_of(const TileD& t, const BoxD& b) {
  return column_at<DIM>(t, b, (int)threadIdx.x);
}

// One x-column per thread over the same tiles (blocks of 128 threads in 2D,
// 512 in 3D): lanes of a wavefront take 64 consecutive x cells.
template <int DIM>
__device__ __forceinline__ Column column1_of(const TileD& t, const BoxD& b) {
  Column c;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  c.x = t.x0 + 64 * (w & 1) + lane;
  c.y = DIM == 2 ? 0 : t.y0 + (w >> 1);
  c.ok = c.x < b.n[0] && (DIM == 2 || c.y < b.n[1]);
  c.ok1 = false;
  c.p0 = DIM == 2 ? t.y0 : t.z0;
  c.p1 = min(c.p0 + t.len, b.n[DIM - 1]);
  c.sm = b.s[DIM - 1];
  c.base = b.off + (c.x + 2) + (DIM == 3 ? (int64_t)(c.y + 2) * b.s[1] : 0);
  return c;
}

template <typename T>
struct alignas(2 * sizeof(T)) Pair {
  T a, b;
};
template <typename T>
__device__ __forceinline__ Pair<T> ld2(const T* p) {
  return *reinterpret_cast<const Pair<T>*>(p);
}
template <typename T>
__device__ __forceinline__ void st2(T* p, T a, T b) {
  *reinterpret_cast<Pair<T>*>(p) = Pair<T>{a, b};
}
// Non-temporal forms, for the FP64 arrays of a mixed-precision solve that
// stream through once per cycle (the outer residual's x and f, the fused
// update's x): kept from displacing the FP32 cycle's iterate and right-hand
// side in the caches (the 256 MB Infinity Cache holds those at 256^3).
template <typename T>
__device__ __forceinline__ Pair<T> ld2nt(const T* p) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = __builtin_nontemporal_load(reinterpret_cast<const v2*>(p));
  return Pair<T>{v.x, v.y};
}
template <typename T>
__device__ __forceinline__ void st2nt(T* p, T a, T b) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = a;
  v.y = b;
  __builtin_nontemporal_store(v, reinterpret_cast<v2*>(p));
}


// red-black colour of cell (x, y, z) of a 3D box
__device__ __forceinline__ int colour_of(const BoxD& b, int x, int y, int z) {
  return (b.lo[0] + b.lo[1] + b.lo[2] + x + y + z) & 1;
}

// folded diagonal increments of the faces within two cells of (x, y, z)
template <typename T, int DIM>
__device__ __forceinline__ T fold_at(const BoxD& b, const uint8_t* __restrict__ codes, int x, int y, int z) {
  T S = T(0);
  const int p[3] = {x, y, z};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int lo = p[d], hi = b.n[d] - 1 - p[d];
    if (lo >= 2 && hi >= 2) continue;
    int col;
    if (DIM == 2)
      col = d == 0 ? y : x;
    else
      col = d == 0 ? y + b.n[1] * z : (d == 1 ? x + b.n[0] * z : x + b.n[0] * y);
    if (lo < 2) S += fold<T>(codes[b.code_off[d][0] + col], lo);
    if (hi < 2) S += fold<T>(codes[b.code_off[d][1] + col], hi);
  }
  return S;
}

// true if (x, y, z) is within two cells of some face (the folded band)
template <int DIM>
__device__ __forceinline__ bool near_face(const BoxD& b, int x, int y, int z) {
  bool r = x < 2 || x > b.n[0] - 3 || y < 2 || y > b.n[1] - 3;
  if (DIM == 3) r = r || z < 2 || z > b.n[2] - 3;
  return r;
}

// (16 (u[-1] + u[1]) - (u[-2] + u[2])) along the non-march directions
template <typename T, int DIM>
__device__ __forceinline__ T cross_sum(const T* __restrict__ u, int64_t c, const BoxD& b) {
  T acc = T(16) * (u[c - 1] + u[c + 1]) - (u[c - 2] + u[c + 2]);
  if (DIM == 3) {
    const int64_t sy = b.s[1];
    acc += T(16) * (u[c - sy] + u[c + sy]) - (u[c - 2 * sy] + u[c + 2 * sy]);
  }
  return acc;
}

// full stencil sum at c by direct loads (all directions)
template <typename T, int DIM>
__device__ __forceinline__ T lap_sum(const T* __restrict__ u, int64_t c, const BoxD& b) {
  const int64_t sm = b.s[DIM - 1];
  return cross_sum<T, DIM>(u, c, b) + T(16) * (u[c - sm] + u[c + sm]) - (u[c - 2 * sm] + u[c + 2 * sm]) +
         T(-30 * DIM) * u[c];
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
// stencil sweeps marched along the last direction
enum { OP_RESID = 0, OP_JACOBI = 1, OP_RB = 2, OP_RESTRICT = 3 };

// Inverse of the folded diagonal along one thread's column.  The faces
// across the march direction contribute a constant (from the per-face
// uniform code; a face with mixed codes is looked up cell by cell); the two
// faces at the ends of the march contribute only in the first and last two
// cells, from the column's own codes.
template <typename T, int DIM>
struct DiagColumn {
  T alpha, beta, Sfix, inv_mid, flo[2], fhi[2];
  bool mixed;
  int nm;
  __device__ __forceinline__ void init(const BoxD& b, const uint8_t* __restrict__ codes, int x, int y, T a, T be,
                                       bool ok) {
    alpha = a;
    beta = be;
    Sfix = T(-30 * DIM);
    mixed = false;
    const int q[2] = {x, y};
#pragma unroll
    for (int d = 0; d < DIM - 1; ++d) {
      const int lo = q[d], hi = b.n[d] - 1 - q[d];
      if (lo < 2) {
        const uint8_t cd = b.ucode[d][0];
        if (cd == 0xFF) mixed = true;
        else Sfix += fold<T>(cd, lo);
      }
      if (hi < 2) {
        const uint8_t cd = b.ucode[d][1];
        if (cd == 0xFF) mixed = true;
        else Sfix += fold<T>(cd, hi);
      }
    }
    constexpr int M = DIM - 1;
    nm = b.n[M];
    flo[0] = flo[1] = fhi[0] = fhi[1] = T(0);
    if (ok) {
      const int col = DIM == 2 ? x : x + b.n[0] * y;
      const uint8_t cl = codes[b.code_off[M][0] + col], ch = codes[b.code_off[M][1] + col];
      flo[0] = fold<T>(cl, 0);
      flo[1] = fold<T>(cl, 1);
      fhi[0] = fold<T>(ch, 0);
      fhi[1] = fold<T>(ch, 1);
    }
    inv_mid = T(1) / (alpha + beta * Sfix);
  }
  // p: march coordinate; (x, y, z) of the cell for the mixed-face lookup
  __device__ __forceinline__ T inv(const BoxD& b, const uint8_t* __restrict__ codes, int p, int x, int y,
                                   int z) const {
    if (mixed) return T(1) / (alpha + beta * (T(-30 * DIM) + fold_at<T, DIM>(b, codes, x, y, z)));
    if (p >= 2 && p <= nm - 3) return inv_mid;
    T S = Sfix;
    if (p < 2) S += p == 0 ? flo[0] : flo[1];  // selects: no indexed private array
    if (p > nm - 3) S += p == nm - 1 ? fhi[0] : fhi[1];
    return T(1) / (alpha + beta * S);
  }
};

// The two ghosts beyond the row end e0 (first four cells e0 + m in, m = 0..3)
// of the homogeneous fill of a column with code cd: eqs. (velBCHomoDiri5th)
// and (Neumann5) with zero data, computed where they are read instead of by a
// fill launch.  Returns false if the column is not filled (its ghosts are in
// memory); a second layer that is not filled from this row is read from memory.
template <typename T>
__device__ __forceinline__ bool gfill(uint8_t cd, const T* __restrict__ u, int64_t e0, int64_t in, T& g1, T& g2) {
  const T u0 = u[e0], u1 = u[e0 + in], u2 = u[e0 + 2 * in], u3 = u[e0 + 3 * in];
  const int kind = cd & 3;
  if (!kind) return false;
  if (kind == 1) {
    g1 = (T(-77) * u0 + T(43) * u1 - T(17) * u2 + T(3) * u3) * T(1.0 / 12.0);
    g2 = (cd & 4) ? (T(-505) * u0 + T(335) * u1 - T(145) * u2 + T(27) * u3) * T(1.0 / 12.0) : u[e0 - 2 * in];
  } else {
    g1 = (T(5) * u0 + T(9) * u1 - T(5) * u2 + u3) * T(0.1);
    g2 = (cd & 4) ? (T(-75) * u0 + T(145) * u1 - T(75) * u2 + T(15) * u3) * T(0.1) : u[e0 - 2 * in];
  }
  return true;
}

// Ghosts across the march direction of the cells x0..x0+nx-1, y0..y0+ny-1
// (3D; 2D: y0 = 0, ny = 1), march planes p0..p0+len-1, on faces filled
// uniformly (code uf), written into u by the block before its march
// (read-time fill): x faces for the rows that reach them, y faces (3D) for
// the columns that reach them.  Each of these ghosts is read only by the
// block that writes it.
template <typename T, int DIM, bool WRAP = false>
__device__ __forceinline__ void face_ghosts(const BoxD& b, T* __restrict__ u, int x0, int nx, int y0, int ny, int p0,
                                            int len, bool xfaces = true, const uint8_t* __restrict__ codes = nullptr,
                                            const int64_t* __restrict__ xsrc = nullptr) {
  // the ghosts of one column with code cd (e0: its cell at the face, in:
  // the inward stride)
  auto column = [&](uint8_t cd, int64_t e0, int64_t in) {
    if (cd & 3) {
      const T u0 = u[e0], u1 = u[e0 + in], u2 = u[e0 + 2 * in], u3 = u[e0 + 3 * in];
      u[e0 - in] = ghost1<T>(cd, u0, u1, u2, u3);
      if (cd & 4) u[e0 - 2 * in] = ghost2<T>(cd, u0, u1, u2, u3);
    }
  };
  // the same from the column's stored code at pos, its exchange sources
  // loaded with the code (-1: not an exchange column)
  auto column_at = [&](int64_t pos, int64_t e0, int64_t in) {
    const uint8_t cd = codes[pos];
    const int64_t s1 = xsrc[2 * pos], s2 = xsrc[2 * pos + 1];
    if (cd & 3) {
      column(cd, e0, in);
    } else if (s1 >= 0) {
      u[e0 - in] = u[s1];
      u[e0 - 2 * in] = u[s2];
    } else if (cd & kCodeZero) {
      u[e0 - in] = T(0);
      u[e0 - 2 * in] = T(0);
    }
  };
  // x faces: one thread per (row, side); with WRAP, a face that wraps onto
  // the box takes the row's cells at the other end (a compile-time switch:
  // reading the wrap bits costs the other kernels a memory round trip).
  // With codes, a face of several codes, or of exchange or zero columns,
  // goes column by column.
  const bool wx = WRAP && (b.wrap & 1);
  for (int side = 0; side < 2 && xfaces; ++side) {
    const uint8_t cd = b.ucode[0][side];
    const bool percol = codes && (cd == 0xFF || (cd & (kCodeExch | kCodeZero)));
    if (!wx && !percol && (cd == 0xFF || !(cd & 3))) continue;
    if (side == 0 ? x0 != 0 : x0 + nx != b.n[0]) continue;
    for (int r = (int)threadIdx.x; r < ny * len; r += (int)blockDim.x) {
      const int y = DIM == 3 ? y0 + r % ny : 0, p = p0 + r / ny;
      const int64_t e0 = cell_index<DIM>(b, side ? b.n[0] - 1 : 0, DIM == 3 ? y : p, DIM == 3 ? p : 0);
      const int64_t in = side ? -1 : 1;
      if (wx) {
        const int64_t far = (int64_t)(b.n[0] - 1) * in;
        u[e0 - in] = u[e0 + far];
        u[e0 - 2 * in] = u[e0 + far - in];
        continue;
      }
      if (percol) {
        const int64_t pos = (int64_t)b.code_off[0][side] + (DIM == 3 ? y + (int64_t)b.n[1] * p : p);
        column_at(pos, e0, in);
        continue;
      }
      column(cd, e0, in);
    }
  }
  if (DIM == 3) {
    const bool wy = WRAP && ((b.wrap >> 1) & 1);
    for (int side = 0; side < 2; ++side) {
      const uint8_t cd = b.ucode[1][side];
      const bool percol = codes && (cd == 0xFF || (cd & (kCodeExch | kCodeZero)));
      if (!wy && !percol && (cd == 0xFF || !(cd & 3))) continue;
      if (side == 0 ? y0 != 0 : y0 + ny != b.n[1]) continue;
      for (int r = (int)threadIdx.x; r < nx * len; r += (int)blockDim.x) {
        const int x = x0 + r % nx, p = p0 + r / nx;
        const int64_t e0 = cell_index<DIM>(b, x, side ? b.n[1] - 1 : 0, p);
        const int64_t in = (side ? -1 : 1) * (int64_t)b.s[1];
        if (wy) {
          const int64_t far = (int64_t)(b.n[1] - 1) * in;
          u[e0 - in] = u[e0 + far];
          u[e0 - 2 * in] = u[e0 + far - in];
          continue;
        }
        if (percol) {
          const int64_t pos = (int64_t)b.code_off[1][side] + x + (int64_t)b.n[0] * p;
          column_at(pos, e0, in);
          continue;
        }
        column(cd, e0, in);
      }
    }
  }
}

// Ghosts along the march direction of the tile's columns (the faces at the
// ends of the march), from each column's own code, on the faces the tile
// reaches; written by the block before its march like face_ghosts.
template <typename T, int DIM, bool WRAP = false>
__device__ __forceinline__ void march_ghosts(const TileD& t, const BoxD& b, const uint8_t* __restrict__ codes,
                                             T* __restrict__ u) {
  constexpr int M = DIM - 1;
  const int p0 = DIM == 2 ? t.y0 : t.z0, len = min(t.len, b.n[M] - p0);
  const int nx = min(TILE_X, b.n[0] - t.x0), ny = DIM == 3 ? min(TILE3_Y, b.n[1] - t.y0) : 1;
  const bool wm = WRAP && ((b.wrap >> M) & 1);  // the march direction wraps onto the box
  for (int side = 0; side < 2; ++side) {
    if (side == 0 ? p0 != 0 : p0 + len != b.n[M]) continue;
    for (int r = (int)threadIdx.x; r < nx * ny; r += (int)blockDim.x) {
      const int x = t.x0 + r % nx, y = DIM == 3 ? t.y0 + r / nx : 0;
      const int pe = side ? b.n[M] - 1 : 0;
      const int64_t e0 = DIM == 3 ? cell_index<3>(b, x, y, pe) : cell_index<2>(b, x, pe, 0);
      const int64_t in = (side ? -1 : 1) * (int64_t)b.s[M];
      if (wm) {  // ghost layer g is the cell g from the other end of the column
        const int64_t far = (int64_t)(b.n[M] - 1) * in;
        u[e0 - in] = u[e0 + far];
        u[e0 - 2 * in] = u[e0 + far - in];
        continue;
      }
      const uint8_t cd = codes[b.code_off[M][side] + (DIM == 2 ? x : x + b.n[0] * y)];
      if (!(cd & 3)) continue;
      const T u0 = u[e0], u1 = u[e0 + in], u2 = u[e0 + 2 * in], u3 = u[e0 + 3 * in];
      u[e0 - in] = ghost1<T>(cd, u0, u1, u2, u3);
      if (cd & 4) u[e0 - 2 * in] = ghost2<T>(cd, u0, u1, u2, u3);
    }
  }
}

// the same for the cells of one column tile (xfaces false: y faces only)
template <typename T, int DIM, bool WRAP = false>
__device__ __forceinline__ void tile_ghosts(const TileD& t, const BoxD& b, T* __restrict__ u, bool xfaces = true,
                                            const uint8_t* __restrict__ codes = nullptr,
                                            const int64_t* __restrict__ xsrc = nullptr) {
  const int p0 = DIM == 2 ? t.y0 : t.z0;
  face_ghosts<T, DIM, WRAP>(b, u, t.x0, min(TILE_X, b.n[0] - t.x0), DIM == 3 ? t.y0 : 0,
                            DIM == 3 ? min(TILE3_Y, b.n[1] - t.y0) : 1, p0, min(t.len, b.n[DIM - 1] - p0), xfaces,
                            codes, xsrc);
}

// OP_RESID : out = f - A u (f == NULL: out = A u); PART: per-tile max |out|
// OP_JACOBI: out = u + omega (f - A u) / diag
// OP_RB    : out = u + omega (f - A u) / diag on cells of colour `col`, else u (omega = 1: plain)
// with A u = alpha u + beta * (sum of the 1-D stencils of eq. discreteOps c).
// Along the march direction the neighbours come from the thread's register
// queue; across it they are re-read through the L1/L2 caches (the
// neighbouring columns of the same tile and of the neighbouring tiles of
// the same XCD have just fetched them).
// One cell per thread and step; the neighbours across the march direction
// are re-read through the L1/L2 caches (the neighbouring columns of the same
// tile and the neighbouring tiles on the same XCD have just fetched them).
//
// gr != 0: the ghosts of filled columns (physical and coarse-fine face-data
// faces, homogeneous) are computed where they are read (gfill), and those of
// a direction that wraps onto the box are read from its other end (WRAP), so
// no fill launch is needed before the sweep for them.  XF: so are those of
// exchange columns (copied from the cells xsrc names) and zero columns
// (the interpolated ghosts of a correction); without XF those come from
// memory.
template <typename T, int DIM, int OP, bool PART, bool WRAP, bool XF>
__global__ void __launch_bounds__(512) k_march1(const TileD* __restrict__ tiles, int ntiles,
                                                const BoxD* __restrict__ boxes, const uint8_t* __restrict__ codes,
                                                const T* u, const T* __restrict__ f, T* __restrict__ out,
                                                T alpha, T beta, T omega, int col, double* __restrict__ part,
                                                int gr, const int64_t* __restrict__ xsrc) {
  __shared__ double sh[8];
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  const Column C = column1_of<DIM>(t, b);
  // read-time fill across the march: a block whose tile touches a uniformly
  // filled x or y face writes the ghosts its cells read there (each such
  // ghost is read only by this tile) before marching; the input array is
  // complete when the kernel starts
  if (gr) {
    const int nx = min(TILE_X, b.n[0] - t.x0);
    const uint8_t ux0 = b.ucode[0][0], ux1 = b.ucode[0][1];
    // XF: also faces of exchange or zero columns, or of several codes
    const bool xf = XF ? ((ux0 != 0 && t.x0 == 0) || (ux1 != 0 && t.x0 + nx == b.n[0]))
                       : ((ux0 != 0xFF && (ux0 & 3) && t.x0 == 0) || (ux1 != 0xFF && (ux1 & 3) && t.x0 + nx == b.n[0]));
    const bool xw = WRAP && (b.wrap & 1) && (t.x0 == 0 || t.x0 + nx == b.n[0]);
    const bool yf = DIM == 3 && (t.y0 == 0 || t.y0 + TILE3_Y >= b.n[1]);
    if (xf || xw || yf) {  // block-uniform
      tile_ghosts<T, DIM, WRAP>(t, b, const_cast<T*>(u), true, XF ? codes : nullptr, XF ? xsrc : nullptr);
      __syncthreads();
    }
  }
  double vmax = 0.0, vsum = 0.0;
  if (C.ok) {
    const int64_t sm = C.sm;
    constexpr int M = DIM - 1;
    const int nm = b.n[M];
    int64_t c = C.base + (int64_t)(C.p0 + 2) * sm;
    // the march direction wraps onto the box: its ghosts are the column's
    // planes at the other end, read there (c0: plane 0 of the column)
    const bool wm = WRAP && gr && ((b.wrap >> M) & 1);
    const int64_t c0 = c - (int64_t)C.p0 * sm;
    T q0 = u[c - 2 * sm], q1 = u[c - sm], q2 = u[c], q3 = u[c + sm];
    if (wm) {
      if (C.p0 == 0) {
        q0 = u[c0 + (int64_t)(nm - 2) * sm];
        q1 = u[c0 + (int64_t)(nm - 1) * sm];
      } else if (C.p0 == 1) {
        q0 = u[c0 + (int64_t)(nm - 1) * sm];
      }
      if (C.p0 + 1 >= nm) q3 = u[c0 + (int64_t)(C.p0 + 1 - nm) * sm];
    }
    // march-direction ghosts of this column (homogeneous fill, if filled):
    // the low ones once here, the high ones from the register queue
    uint8_t chi = 0;
    T g2n = T(0);  // second high ghost, computed one step ahead
    T xh1 = T(0), xh2 = T(0);  // high ghosts of an exchange or zero column
    if (gr) {
      const int mcol = DIM == 2 ? C.x : C.x + b.n[0] * C.y;
      T g1, g2;
      if (C.p0 < 2) {
        const int64_t pos = (int64_t)b.code_off[M][0] + mcol;
        const uint8_t clo = codes[pos];
        bool got = gfill<T>(clo, u, c - (int64_t)C.p0 * sm, sm, g1, g2);
        if (XF && !got && (clo & (kCodeExch | kCodeZero))) {
          g1 = (clo & kCodeExch) ? u[xsrc[2 * pos]] : T(0);
          g2 = (clo & kCodeExch) ? u[xsrc[2 * pos + 1]] : T(0);
          got = true;
        }
        if (got) {
          if (C.p0 == 0) {
            q0 = g2;
            q1 = g1;
          } else {
            q0 = g1;
          }
        }
      }
      if (C.p1 + 2 > nm) {
        const int64_t pos = (int64_t)b.code_off[M][1] + mcol;
        chi = codes[pos];
        if (XF && (chi & kCodeExch)) {
          xh1 = u[xsrc[2 * pos]];
          xh2 = u[xsrc[2 * pos + 1]];
        }
        if ((chi & 3) && C.p0 + 1 >= nm && gfill<T>(chi, u, c + (int64_t)(nm - 1 - C.p0) * sm, -sm, g1, g2)) {
          q3 = g1;  // a one-cell tile at the end of the column
          g2n = g2;
        }
        if (XF && (chi & (kCodeExch | kCodeZero)) && C.p0 + 1 >= nm) q3 = xh1;
      }
    }
    const int hk = chi & 3;  // fill kind of the high march-direction face (0: ghosts in memory)
    const bool hx = XF && (chi & (kCodeExch | kCodeZero)) != 0;  // high ghosts from xh1, xh2
    DiagColumn<T, DIM> dg;
    if (OP != OP_RESID) dg.init(b, codes, C.x, C.y, alpha, beta, true);
    const int par0 = (b.lo[0] + C.x + (DIM == 3 ? b.lo[1] + C.y : 0) + b.lo[DIM - 1]) & 1;
    for (int p = C.p0; p < C.p1; ++p, c += sm) {
      T q4;
      if (hk && p + 2 == nm) {  // q0..q3 hold the last four cells of the column
        if (hk == 1) {
          q4 = (T(-77) * q3 + T(43) * q2 - T(17) * q1 + T(3) * q0) * T(1.0 / 12.0);
          g2n = (chi & 4) ? (T(-505) * q3 + T(335) * q2 - T(145) * q1 + T(27) * q0) * T(1.0 / 12.0)
                          : u[c + 3 * sm];
        } else {
          q4 = (T(5) * q3 + T(9) * q2 - T(5) * q1 + q0) * T(0.1);
          g2n = (chi & 4) ? (T(-75) * q3 + T(145) * q2 - T(75) * q1 + T(15) * q0) * T(0.1) : u[c + 3 * sm];
        }
      } else if (hk && p + 2 == nm + 1) {
        q4 = g2n;
      } else if (hx && p + 2 >= nm) {
        q4 = p + 2 == nm ? xh1 : xh2;
      } else if (wm && p + 2 >= nm) {
        q4 = u[c0 + (int64_t)(p + 2 - nm) * sm];
      } else {
        q4 = u[c + 2 * sm];
      }
      T ls = T(16) * (u[c - 1] + u[c + 1]) - (u[c - 2] + u[c + 2]) + T(16) * (q1 + q3) - (q0 + q4) +
             T(-30 * DIM) * q2;
      if (DIM == 3) {
        const int64_t sy = b.s[1];
        ls += T(16) * (u[c - sy] + u[c + sy]) - (u[c - 2 * sy] + u[c + 2 * sy]);
      }
      const T Au = alpha * q2 + beta * ls;
      if (OP == OP_RESID) {
        const T v = f ? f[c] - Au : Au;
        out[c] = v;
        if (PART) {
          double av = fabs((double)v);
          vmax = fmax(vmax, (av == av) ? av : (double)INFINITY);  // a NaN must not vanish in fmax
          vsum += (double)v;
        }
      } else if (OP == OP_JACOBI || (((par0 + p) & 1) == col)) {
        out[c] = q2 + omega * (f[c] - Au) *
                          dg.inv(b, codes, p, C.x, DIM == 2 ? p : C.y, DIM == 2 ? 0 : p);
      } else {
        out[c] = q2;
      }
      q0 = q1;
      q1 = q2;
      q2 = q3;
      q3 = q4;
    }
  }
  if (PART) {
    const double m = block_max<double>(vmax, sh);
    __syncthreads();
    const double sm = block_sum<double>(vsum, sh);
    if (threadIdx.x == 0) {
      part[ti] = m;
      part[ntiles + ti] = sm;
    }
  }
}

// Two cells (x, x+1) per thread and step.  x neighbours: the two cells on
// each side come from the adjacent lanes (shuffles); the end lanes of the
// wavefront read them from memory.  y neighbours (3D): vector loads through
// the caches.  OP_RESTRICT computes the residual like OP_RESID and averages
// it over the 2^DIM children of each coarse cell on the fly (x pairs inside
// the thread, z or y pairs over two steps, y pairs in 3D through LDS), so the
// fine residual is never stored: out is the coarse right-hand side.  TO:
// the element type of out (an FP64 residual may be stored in FP32).
template <typename T, int DIM, int OP, bool PART, typename TO = T, bool WRAP = false>
__global__ void __launch_bounds__(256) k_march(const TileD* __restrict__ tiles, int ntiles,
                                               const BoxD* __restrict__ boxes, const uint8_t* __restrict__ codes,
                                               const T* __restrict__ u, const T* __restrict__ f, TO* __restrict__ out,
                                               T alpha, T beta, T omega, int col, double* __restrict__ part,
                                               const BoxD* __restrict__ cboxes, int gr, int64_t shalf) {
  __shared__ double sh[4];
  __shared__ T R[2][64];
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  // gr != 0 (every face filled uniformly from its own rows, both layers):
  // no fill launch is needed before the kernel.  A block whose tile touches
  // a y face or an end of the march writes the ghosts its cells read there
  // first; the x-face ghosts are formed in registers by the lanes next to
  // the x faces from the cells the lanes exchange (below), except at the
  // high x face of a row of odd length (its last lane holds one cell), which
  // the block writes too.
  const bool xodd = gr && (b.n[0] & 1) && t.x0 + TILE_X >= b.n[0];
  if (gr) {
    const int p0 = DIM == 2 ? t.y0 : t.z0, nm = b.n[DIM - 1];
    if (xodd || (DIM == 3 && (t.y0 == 0 || t.y0 + TILE3_Y >= b.n[1])) || p0 == 0 || p0 + t.len >= nm) {
      tile_ghosts<T, DIM, WRAP>(t, b, const_cast<T*>(u), xodd);  // block-uniform branch
      march_ghosts<T, DIM, WRAP>(t, b, codes, const_cast<T*>(u));
      __syncthreads();
    }
  }
  // lanes whose pair ends at an x face (gr only)
  const bool gxlo = gr && t.x0 == 0, gxhi = gr && !(b.n[0] & 1);
  const uint8_t cxl = b.ucode[0][0], cxh = b.ucode[0][1];
  const Column C = column_of<DIM>(t, b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // lanes up to two cells past the box feed the x-neighbours of the last cells
  const bool has = C.x < b.n[0] + 2 && (DIM == 2 || C.y < b.n[1]);
  const int64_t sm = C.sm, sy = b.s[1];
  int64_t c = C.base + (int64_t)(C.p0 + 2) * sm;
  Pair<T> q0{}, q1{}, q2{}, q3{}, q4{};
  if (has) {
    q0 = ld2(u + c - 2 * sm);
    q1 = ld2(u + c - sm);
    q2 = ld2(u + c);
    q3 = ld2(u + c + sm);
  }
  // the outer FP64 residual of a mixed solve (FP32 output): x and f stream
  constexpr bool NT = OP == OP_RESID && sizeof(T) == 8 && sizeof(TO) == 4;
  DiagColumn<T, DIM> d0, d1;
  if (OP == OP_JACOBI || OP == OP_RB) {
    d0.init(b, codes, C.x, C.y, alpha, beta, C.ok);
    d1.init(b, codes, C.x + 1, C.y, alpha, beta, C.ok1);
  }
  const int par0 = (b.lo[0] + C.x + (DIM == 3 ? b.lo[1] + C.y : 0) + b.lo[DIM - 1]) & 1;
  double vmax = 0.0, vsum = 0.0;
  T acc = T(0);
  for (int p = C.p0; p < C.p1; ++p, c += sm) {
    if (has) q4 = NT ? ld2nt(u + c + 2 * sm) : ld2(u + c + 2 * sm);
    T La = __shfl_up(q2.a, 1, 64), Lb = __shfl_up(q2.b, 1, 64);
    T Ra = __shfl_down(q2.a, 1, 64), Rb = __shfl_down(q2.b, 1, 64);
    T o0 = T(0), o1 = T(0);
    if (C.ok) {
      const bool xlo = gxlo && C.x == 0, xhi = gxhi && C.x + 2 == b.n[0];
      if (lane == 0 && !xlo) {
        La = u[c - 2];
        Lb = u[c - 1];
      }
      if (lane == 63 && !xhi) {
        Ra = u[c + 2];
        Rb = u[c + 3];
      }
      // WRAP: an x direction that wraps onto the box takes the row's cells
      // at the other end
      const bool wx = WRAP && (b.wrap & 1);
      if (xlo && wx) {
        La = u[c + b.n[0] - 2];
        Lb = u[c + b.n[0] - 1];
      } else if (xlo) {  // cells -2, -1 from cells 0..3 (the next lane's pair)
        La = ghost2<T>(cxl, q2.a, q2.b, Ra, Rb);
        Lb = ghost1<T>(cxl, q2.a, q2.b, Ra, Rb);
      }
      if (xhi && wx) {
        Ra = u[c + 2 - b.n[0]];
        Rb = u[c + 3 - b.n[0]];
      } else if (xhi) {  // cells n, n + 1 from cells n - 1 .. n - 4 (the previous pair)
        const T g1 = ghost1<T>(cxh, q2.b, q2.a, Lb, La), g2 = ghost2<T>(cxh, q2.b, q2.a, Lb, La);
        Ra = g1;
        Rb = g2;
      }
      T s0 = T(16) * (Lb + q2.b) - (La + Ra) + T(16) * (q1.a + q3.a) - (q0.a + q4.a) + T(-30 * DIM) * q2.a;
      T s1 = T(16) * (q2.a + Ra) - (Lb + Rb) + T(16) * (q1.b + q3.b) - (q0.b + q4.b) + T(-30 * DIM) * q2.b;
      if (DIM == 3) {
        const Pair<T> ym1 = ld2(u + c - sy), yp1 = ld2(u + c + sy), ym2 = ld2(u + c - 2 * sy),
                      yp2 = ld2(u + c + 2 * sy);
        s0 += T(16) * (ym1.a + yp1.a) - (ym2.a + yp2.a);
        s1 += T(16) * (ym1.b + yp1.b) - (ym2.b + yp2.b);
      }
      const T A0 = alpha * q2.a + beta * s0, A1 = alpha * q2.b + beta * s1;
      Pair<T> fv{};
      if (OP != OP_RESID || f) fv = NT ? ld2nt(f + c) : ld2(f + c);
      if (OP == OP_RESID || OP == OP_RESTRICT) {
        o0 = f ? fv.a - A0 : A0;
        o1 = f ? fv.b - A1 : A1;
        if (PART) {
          double a0 = fabs((double)o0), a1 = C.ok1 ? fabs((double)o1) : 0.0;
          a0 = (a0 == a0) ? a0 : (double)INFINITY;  // a NaN must not vanish in fmax
          a1 = (a1 == a1) ? a1 : (double)INFINITY;
          vmax = fmax(vmax, fmax(a0, a1));
          vsum += (double)o0 + (C.ok1 ? (double)o1 : 0.0);
        }
      } else {
        const int cy = DIM == 2 ? p : C.y, cz = DIM == 2 ? 0 : p;
        const bool u0 = OP == OP_JACOBI || (((par0 + p) & 1) == col);
        const bool u1 = OP == OP_JACOBI || (((par0 + p + 1) & 1) == col);
        const T wgt = omega;
        o0 = u0 ? q2.a + wgt * (fv.a - A0) * d0.inv(b, codes, p, C.x, cy, cz) : q2.a;
        o1 = u1 ? q2.b + wgt * (fv.b - A1) * d1.inv(b, codes, p, C.x + 1, cy, cz) : q2.b;
      }
      if (OP != OP_RESTRICT) {
        if (OP == OP_RESID && shalf) {  // colour-split output, halves shalf apart
          const int cxo = DIM == 3 ? colour_of(b, C.x, C.y, p) : colour_of(b, C.x, p, 0);
          out[(cxo ? shalf : 0) + (c >> 1)] = (TO)o0;
          out[(cxo ? 0 : shalf) + (c >> 1)] = (TO)o1;
        } else if (C.ok1) {
          st2<TO>(out + c, (TO)o0, (TO)o1);
        } else {
          out[c] = (TO)o0;
        }
      }
    }
    if (OP == OP_RESTRICT) {
      acc += o0 + o1;  // x pair (fine sizes are even, so both cells exist)
      if ((p - C.p0) & 1) {
        if (DIM == 3) {
          if (w & 1) R[w >> 1][lane] = acc;
          __syncthreads();
          if (!(w & 1) && C.ok) {
            const BoxD cb = cboxes[b.coarse];
            out[cell_index<DIM>(cb, C.x >> 1, C.y >> 1, p >> 1)] = (TO)((acc + R[w >> 1][lane]) * T(0.125));
          }
          __syncthreads();
        } else if (C.ok) {
          const BoxD cb = cboxes[b.coarse];
          out[cell_index<DIM>(cb, C.x >> 1, p >> 1, 0)] = (TO)(acc * T(0.25));
        }
        acc = T(0);
      }
    }
    q0 = q1;
    q1 = q2;
    q2 = q3;
    q3 = q4;
  }
  if (PART) {
    const double m = block_max<double>(vmax, sh);
    __syncthreads();
    const double sm = block_sum<double>(vsum, sh);
    if (threadIdx.x == 0) {
      part[ti] = m;
      part[ntiles + ti] = sm;
    }
  }
}

// ---------------------------------------------------------------------------
// pointwise kernels over the same tiles (two columns per thread)
#define FOR_COLUMN(DIM_)                                             \
  const int ti = tile_of_block(ntiles);                             \
  if (ti < 0) return;                                               \
  const TileD t = tiles[ti];                                        \
  const BoxD b = boxes[t.box];                                      \
  const Column C = column_of<DIM_>(t, b);                           \
  if (C.ok)                                                         \
    for (int p = C.p0; p < C.p1; ++p)

// first sweep from a zero iterate: Jacobi out = omega f / diag; red-black
// (red half) out = omega f / diag on red cells, 0 on black ones
template <typename T, int DIM, bool RB>
__global__ void __launch_bounds__(256) k_sweep0(const TileD* __restrict__ tiles, int ntiles,
                                                const BoxD* __restrict__ boxes, const uint8_t* __restrict__ codes,
                                                const T* __restrict__ f, T* __restrict__ out, T alpha, T beta,
                                                T omega) {
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  const Column C = column_of<DIM>(t, b);
  if (!C.ok) return;
  DiagColumn<T, DIM> d0, d1;
  d0.init(b, codes, C.x, C.y, alpha, beta, true);
  d1.init(b, codes, C.x + 1, C.y, alpha, beta, C.ok1);
  const int par0 = (b.lo[0] + C.x + (DIM == 3 ? b.lo[1] + C.y : 0) + b.lo[DIM - 1]) & 1;
  const T w = omega;
  for (int p = C.p0; p < C.p1; ++p) {
    const int cy = DIM == 2 ? p : C.y, cz = DIM == 2 ? 0 : p;
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    const Pair<T> fv = C.ok1 ? ld2(f + c) : Pair<T>{f[c], T(0)};
    const bool red0 = !RB || (((par0 + p) & 1) == 0), red1 = !RB || (((par0 + p + 1) & 1) == 0);
    const T o0 = red0 ? w * fv.a * d0.inv(b, codes, p, C.x, cy, cz) : T(0);
    const T o1 = red1 ? w * fv.b * d1.inv(b, codes, p, C.x + 1, cy, cz) : T(0);
    if (C.ok1)
      st2(out + c, o0, o1);
    else
      out[c] = o0;
  }
}

// x += s e (x FP64, e FP32 or FP64), s = scal[0]
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_update(const TileD* __restrict__ tiles, int ntiles,
                                                const BoxD* __restrict__ boxes, double* __restrict__ x,
                                                const T* __restrict__ e, const double* __restrict__ scal) {
  const double s = scal[0];
  FOR_COLUMN(DIM) {
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    if (C.ok1) {
      const Pair<double> xv = ld2(x + c);
      const Pair<T> ev = ld2(e + c);
      st2(x + c, xv.a + s * (double)ev.a, xv.b + s * (double)ev.b);
    } else {
      x[c] += s * (double)e[c];
    }
  }
}

// the pair of cells (x, x + 1) at element c (x even; (x, y, z) with z = 0 in
// 2D) stored into split halves fs0, fs1
__device__ __forceinline__ void split_pair(float* __restrict__ fs0, float* __restrict__ fs1, const BoxD& b, int x,
                                           int y, int z, int64_t c, float a, float a1) {
  const int cx = colour_of(b, x, y, z);
  (cx ? fs1 : fs0)[c >> 1] = a;
  (cx ? fs0 : fs1)[c >> 1] = a1;
}

// r32 = fp32(r / s), s = scal[0]; with fs0, fs1 the result goes to split
// storage instead
template <int DIM>
__global__ void __launch_bounds__(256) k_to32(const TileD* __restrict__ tiles, int ntiles,
                                              const BoxD* __restrict__ boxes, const double* __restrict__ r,
                                              float* __restrict__ r32, const double* __restrict__ scal,
                                              const double* __restrict__ delta, float* __restrict__ fs0,
                                              float* __restrict__ fs1) {
  const double inv = 1.0 / scal[0];
  FOR_COLUMN(DIM) {
    const double dv = delta ? delta[b.comp] : 0.0;
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    if (C.ok1) {
      const Pair<double> rv = ld2(r + c);
      const float a = (float)((rv.a - dv) * inv), a1 = (float)((rv.b - dv) * inv);
      if (fs0)
        split_pair(fs0, fs1, b, C.x, DIM == 3 ? C.y : p, DIM == 3 ? p : 0, c, a, a1);
      else
        st2(r32 + c, a, a1);
    } else {
      r32[c] = (float)((r[c] - dv) * inv);
    }
  }
}

// r32 = (r32 - delta[comp]) / scal[0] in place (the FP64 residual stored
// unscaled in FP32 by the residual kernel; arithmetic in FP64); with fs0,
// fs1 the result goes to split storage instead
template <int DIM>
__global__ void __launch_bounds__(256) k_scale32(const TileD* __restrict__ tiles, int ntiles,
                                                 const BoxD* __restrict__ boxes, float* __restrict__ r32,
                                                 const double* __restrict__ scal, const double* __restrict__ delta,
                                                 float* __restrict__ fs0, float* __restrict__ fs1) {
  const double inv = 1.0 / scal[0];
  FOR_COLUMN(DIM) {
    const double dv = delta ? delta[b.comp] : 0.0;
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    if (C.ok1) {
      const Pair<float> rv = ld2(r32 + c);
      const float a = (float)(((double)rv.a - dv) * inv), a1 = (float)(((double)rv.b - dv) * inv);
      if (fs0)
        split_pair(fs0, fs1, b, C.x, DIM == 3 ? C.y : p, DIM == 3 ? p : 0, c, a, a1);
      else
        st2(r32 + c, a, a1);
    } else {
      r32[c] = (float)(((double)r32[c] - dv) * inv);
    }
  }
}

// a -= delta[comp] (components with a zero delta untouched)
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_comp_shift(const TileD* __restrict__ tiles, int ntiles,
                                                    const BoxD* __restrict__ boxes, T* __restrict__ a,
                                                    const double* __restrict__ delta) {
  FOR_COLUMN(DIM) {
    const double d = delta[b.comp];
    if (d == 0.0) break;
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    a[c] = (T)((double)a[c] - d);
    if (C.ok1) a[c + 1] = (T)((double)a[c + 1] - d);
  }
}

// Per-component mean removal from the per-tile sums in part (k_tile_reduce)
// in one launch: every block sums its component's tile sums itself, in one
// fixed order (a block-size stride, the same in every block of the launch),
// so all blocks of a component subtract the same mean, then shifts its own
// tile (for depths of few tiles, where the repeated sums are cheap and the
// launch saved is not).  In 3D the blocks have the 256 threads of
// k_comp_mean_delta and sum in its order; the 64-thread blocks of 2D sum in
// another order, so the two mean paths agree there to rounding only.
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_comp_mean_shift(const TileD* __restrict__ tiles, int ntiles,
                                                         const BoxD* __restrict__ boxes,
                                                         const double* __restrict__ part,
                                                         const int32_t* __restrict__ seg,
                                                         const int32_t* __restrict__ cseg,
                                                         const int32_t* __restrict__ flag,
                                                         const double* __restrict__ cnt, T* __restrict__ a) {
  __shared__ double sh[4];
  __shared__ double mean;
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  const int comp = b.comp;
  const int32_t fl = flag[comp], j0 = seg[cseg[comp]], j1 = seg[cseg[comp + 1]];
  if (!fl) return;  // block-uniform
  double v = 0.0;
  for (int j = j0 + (int)threadIdx.x; j < j1; j += (int)blockDim.x) v += part[j];
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) mean = v / (cnt[comp] * 1.0);
  __syncthreads();
  const double d = mean;
  if (d == 0.0) return;
  const Column C = column_of<DIM>(t, b);
  if (C.ok)
    for (int p = C.p0; p < C.p1; ++p) {
      const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
      a[c] = (T)((double)a[c] - d);
      if (C.ok1) a[c + 1] = (T)((double)a[c + 1] - d);
    }
}

// Per-component mean removal of a small depth in one launch: one block per
// component walks the cells of the component's boxes in a fixed order,
// sums, and subtracts sum / cells on singular components.
template <typename T, int DIM>
__global__ void __launch_bounds__(1024) k_comp_mean_small(int nboxes, const BoxD* __restrict__ boxes,
                                                          const int32_t* __restrict__ flag,
                                                          const double* __restrict__ cnt, T* __restrict__ a) {
  __shared__ double sh[16];
  __shared__ double mean;
  const int comp = blockIdx.x;
  if (!flag[comp]) return;
  double v = 0.0;
  for (int bi = 0; bi < nboxes; ++bi) {
    const BoxD b = boxes[bi];
    if (b.comp != comp) continue;
    const int n = b.n[0] * b.n[1] * (DIM == 3 ? b.n[2] : 1);
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
      const int x = i % b.n[0], r = i / b.n[0];
      v += (double)a[cell_index<DIM>(b, x, DIM == 3 ? r % b.n[1] : r, DIM == 3 ? r / b.n[1] : 0)];
    }
  }
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) mean = v / cnt[comp];
  __syncthreads();
  const double m = mean;
  for (int bi = 0; bi < nboxes; ++bi) {
    const BoxD b = boxes[bi];
    if (b.comp != comp) continue;
    const int n = b.n[0] * b.n[1] * (DIM == 3 ? b.n[2] : 1);
    for (int i = (int)threadIdx.x; i < n; i += (int)blockDim.x) {
      const int x = i % b.n[0], r = i / b.n[0];
      const int64_t c = cell_index<DIM>(b, x, DIM == 3 ? r % b.n[1] : r, DIM == 3 ? r / b.n[1] : 0);
      a[c] = (T)((double)a[c] - m);
    }
  }
}

// out = f - delta[comp]
template <int DIM>
__global__ void __launch_bounds__(256) k_shift_copy(const TileD* __restrict__ tiles, int ntiles,
                                                    const BoxD* __restrict__ boxes, const double* __restrict__ f,
                                                    double* __restrict__ out, const double* __restrict__ delta) {
  FOR_COLUMN(DIM) {
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    out[c] = f[c] - delta[b.comp];
    if (C.ok1) out[c + 1] = f[c + 1] - delta[b.comp];
  }
}

// per-tile sum (MAX = false) or max |.| (MAX = true) of the interior
template <typename T, int DIM, bool MAX>
__global__ void __launch_bounds__(256) k_tile_reduce(const TileD* __restrict__ tiles, int ntiles,
                                                     const BoxD* __restrict__ boxes, const T* __restrict__ a,
                                                     double* __restrict__ part) {
  __shared__ double sh[4];
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  const Column C = column_of<DIM>(t, b);
  double v = 0.0;
  if (C.ok)
    for (int p = C.p0; p < C.p1; ++p) {
      const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
      const double x0 = (double)a[c], x1 = C.ok1 ? (double)a[c + 1] : 0.0;
      if (MAX) {
        const double m = fmax(fabs(x0), fabs(x1));
        v = fmax(v, (x0 == x0 && x1 == x1) ? m : (double)INFINITY);  // a NaN must not vanish in fmax
      } else {
        v += x0 + x1;
      }
    }
  v = MAX ? block_max<double>(v, sh) : block_sum<double>(v, sh);
  if (threadIdx.x == 0) part[ti] = v;
}

// ---------------------------------------------------------------------------
// inter-depth transfers

// residual of the fine cell c, by direct loads
template <typename T, int DIM>
__device__ __forceinline__ T resid_at(const T* __restrict__ u, const T* __restrict__ f, int64_t c, const BoxD& fb,
                                      T alpha, T beta) {
  return f[c] - (alpha * u[c] + beta * lap_sum<T, DIM>(u, c, fb));
}

// fused residual and restriction: fc = mean over the 2^DIM children of
// (f - A u); marched over coarse tiles, two coarse cells per thread and step
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_resid_restrict(const TileD* __restrict__ tiles, int ntiles,
                                                        const BoxD* __restrict__ boxes,
                                                        const BoxD* __restrict__ fboxes, const T* __restrict__ u,
                                                        const T* __restrict__ f, T* __restrict__ fc, T alpha,
                                                        T beta) {
  FOR_COLUMN(DIM) {
    const int cy = DIM == 2 ? p : C.y, cz = DIM == 2 ? 0 : p;
    const BoxD fb = fboxes[b.fine];
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j == 1 && !C.ok1) break;
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < (1 << DIM); ++a)
        acc += resid_at<T, DIM>(u, f,
                                cell_index<DIM>(fb, 2 * (C.x + j) + (a & 1), 2 * cy + ((a >> 1) & 1),
                                                DIM == 3 ? 2 * cz + ((a >> 2) & 1) : 0),
                                fb, alpha, beta);
      fc[c + j] = acc * T(DIM == 2 ? 0.25 : 0.125);
    }
  }
}

// plain restriction: fc = mean of the 2^DIM children of r
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_restrict(const TileD* __restrict__ tiles, int ntiles,
                                                  const BoxD* __restrict__ boxes, const BoxD* __restrict__ fboxes,
                                                  const T* __restrict__ r, T* __restrict__ fc) {
  FOR_COLUMN(DIM) {
    const int cy = DIM == 2 ? p : C.y, cz = DIM == 2 ? 0 : p;
    const BoxD fb = fboxes[b.fine];
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j == 1 && !C.ok1) break;
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < (1 << DIM); ++a)
        acc += r[cell_index<DIM>(fb, 2 * (C.x + j) + (a & 1), 2 * cy + ((a >> 1) & 1),
                                 DIM == 3 ? 2 * cz + ((a >> 2) & 1) : 0)];
      fc[c + j] = acc * T(DIM == 2 ? 0.25 : 0.125);
    }
  }
}

// u += face-neighbour linear interpolation of the coarse correction:
// (1 - DIM/4) e_P + 1/4 sum_d e_{P + s_d e_d}, s_d the child's side;
// marched over fine tiles.  The thread's two cells x, x+1 share the parent.
// Neighbour of coarse cell q (coordinate pd along direction d) on side s
// (-1, +1); with gr != 0 (the coarse faces filled uniformly from their own
// rows) a neighbour beyond the box is its first ghost, formed from the row.
// (WRAP: a direction that wraps onto the coarse box takes the coarse cell at
// the other end of the row instead)
template <typename T, bool WRAP = false>
__device__ __forceinline__ T coarse_nb(const T* __restrict__ ec, const BoxD& cb, int64_t q, int d, int pd, int s,
                                       int gr) {
  const int64_t st = d == 0 ? 1 : cb.s[d];
  if (WRAP && gr && ((cb.wrap >> d) & 1)) {
    if (s < 0 && pd == 0) return ec[q + (int64_t)(cb.n[d] - 1) * st];
    if (s > 0 && pd == cb.n[d] - 1) return ec[q - (int64_t)(cb.n[d] - 1) * st];
    return ec[q + s * st];
  }
  if (gr && s < 0 && pd == 0) return ghost1<T>(cb.ucode[d][0], ec[q], ec[q + st], ec[q + 2 * st], ec[q + 3 * st]);
  if (gr && s > 0 && pd == cb.n[d] - 1)
    return ghost1<T>(cb.ucode[d][1], ec[q], ec[q - st], ec[q - 2 * st], ec[q - 3 * st]);
  return ec[q + s * st];
}

template <typename T, int DIM, bool WRAP = false>
__global__ void __launch_bounds__(256) k_prolong(const TileD* __restrict__ tiles, int ntiles,
                                                 const BoxD* __restrict__ boxes, const BoxD* __restrict__ cboxes,
                                                 const T* __restrict__ ec, T* __restrict__ u, int gr) {
  FOR_COLUMN(DIM) {
    const int cy = DIM == 2 ? p : C.y, cz = DIM == 2 ? 0 : p;
    const BoxD cb = cboxes[b.coarse];
    const int px = C.x >> 1, py = cy >> 1, pz = cz >> 1;
    const int64_t q = cell_index<DIM>(cb, px, py, pz);
    T common =
        T(1.0 - DIM * 0.25) * ec[q] + T(0.25) * coarse_nb<T, WRAP>(ec, cb, q, 1, py, (cy & 1) ? 1 : -1, gr);
    if (DIM == 3) common += T(0.25) * coarse_nb<T, WRAP>(ec, cb, q, 2, pz, (cz & 1) ? 1 : -1, gr);
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    u[c] += common + T(0.25) * coarse_nb<T, WRAP>(ec, cb, q, 0, px, -1, gr);
    if (C.ok1) u[c + 1] += common + T(0.25) * coarse_nb<T, WRAP>(ec, cb, q, 0, px, 1, gr);
  }
}

// ---------------------------------------------------------------------------
// Colour-split storage (FP32, 2D and 3D).  An array of a depth is kept as
// two halves of nstored / 2 elements: element e (of the interleaved layout)
// of colour c, c = (lo + x + y + z) mod 2, lives at index e >> 1 of half c.
// Box offsets, row lengths and plane sizes are even and every row starts on
// an even element, so the two cells of each aligned pair (e even, e + 1)
// have different colours and share the index e >> 1, and a cell's
// neighbours at distance 1 along y or z (the other colour) and at distance 2
// (its own colour) keep its index shifted by half the stride.  A red-black
// half-sweep of colour c then streams half c (the cell and its same-colour
// neighbours), the other half (its neighbours at distance 1) and half c of
// f, and writes only half c: two words per cell of the depth instead of the
// three of the interleaved out-of-place form, whose cache lines carry both
// colours.

// cell (x, y, z) (ghosts included) of a split array with halves h0, h1;
// zc: a colour whose interior cells are taken as zero (not read), -1: none
template <int DIM>
__device__ __forceinline__ float split_ld(const float* h0, const float* h1, const BoxD& b, int x, int y, int z,
                                          int zc) {
  const int k = colour_of(b, x, y, z);
  return k == zc ? 0.0f : (k ? h1 : h0)[cell_index<DIM>(b, x, y, z) >> 1];
}
template <int DIM>
__device__ __forceinline__ void split_st(float* h0, float* h1, const BoxD& b, int x, int y, int z, float v) {
  (colour_of(b, x, y, z) ? h1 : h0)[cell_index<DIM>(b, x, y, z) >> 1] = v;
}

// x-face ghost of row (y, z) of box b on side `side` (0 low, 1 high),
// layer 1 or 2, in the side buffer xg: the rows of a face are contiguous
__device__ __forceinline__ float* x_ghost(float* xg, const BoxD& b, int side, int y, int z, int layer) {
  return xg + b.xg + (int64_t)side * 2 * b.n[1] * b.n[2] + ((int64_t)z * b.n[1] + y) * 2 + (layer - 1);
}

// Read-time fill in split storage: the two ghost layers of every face of the
// box that the tile's cells read (every face filled uniformly, both layers
// from its own row), written before the march: the y and z faces into the
// input halves, the x faces into the side buffer xg (in the halves an x-face
// ghost is one word per row and half, which would dirty a cache line each);
// one thread per face row of the tile.  Each of these ghosts is read only by
// this tile (smoothed boxes have even sizes and marches are even, so the
// last tile of every row, column and march has at least 2 cells).  zc >= 0:
// the interior cells of colour zc are zero (their half is not read); the
// ghosts of both colours are written.
template <int DIM>
__device__ __forceinline__ void split_ghosts(const TileD& t, const BoxD& b, float* h0, float* h1, float* xg,
                                             int zc) {
  // the tile's cells: x, then (3D) its rows and planes, (2D) its rows
  const int lo[3] = {t.x0, t.y0, DIM == 3 ? t.z0 : 0};
  const int nn[3] = {min(TILE_X, b.n[0] - t.x0), DIM == 3 ? min(TILE3_Y, b.n[1] - t.y0) : min(t.len, b.n[1] - t.y0),
                     DIM == 3 ? min(t.len, b.n[2] - t.z0) : 1};
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    for (int side = 0; side < 2; ++side) {
      if (side == 0 ? lo[d] != 0 : lo[d] + nn[d] != b.n[d]) continue;
      const uint8_t cd = b.ucode[d][side];
      const int in = side ? -1 : 1, e = side ? b.n[d] - 1 : 0;
      for (int r = (int)threadIdx.x; r < nn[d1] * nn[d2]; r += (int)blockDim.x) {
        const int a1 = lo[d1] + r % nn[d1], a2 = lo[d2] + r / nn[d1];
        // (x, y, z) of the cell at distance m from the face cell along d
        auto at = [&](int m, int& x, int& y, int& z) {
          x = d == 0 ? e + m * in : (d1 == 0 ? a1 : a2);
          y = d == 1 ? e + m * in : (d1 == 1 ? a1 : a2);
          z = d == 2 ? e + m * in : a2;
        };
        float u[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
          int x, y, z;
          at(m, x, y, z);
          u[m] = split_ld<DIM>(h0, h1, b, x, y, z, zc);
        }
        const float g1 = ghost1<float>(cd, u[0], u[1], u[2], u[3]), g2 = ghost2<float>(cd, u[0], u[1], u[2], u[3]);
        if (d == 0) {
          *x_ghost(xg, b, side, a1, a2, 1) = g1;
          *x_ghost(xg, b, side, a1, a2, 2) = g2;
        } else {
          int x, y, z;
          at(-1, x, y, z);
          split_st<DIM>(h0, h1, b, x, y, z, g1);
          at(-2, x, y, z);
          split_st<DIM>(h0, h1, b, x, y, z, g2);
        }
      }
    }
  }
}

// -30 D plus the folded diagonal increments of the faces across the march
// at (x, y) (3D: x and y faces; 2D: x faces), added in the order of
// DiagColumn (uniformly filled faces).
template <int DIM>
__device__ __forceinline__ float split_sfix(const BoxD& b, int x, int y) {
  float S = float(-30 * DIM);
  const int q[2] = {x, y};
#pragma unroll
  for (int d = 0; d < DIM - 1; ++d) {
    const int lo = q[d], hi = b.n[d] - 1 - q[d];
    if (lo < 2) S += fold<float>(b.ucode[d][0], lo);
    if (hi < 2) S += fold<float>(b.ucode[d][1], hi);
  }
  return S;
}

// true if the tile touches a face of its box (its block writes ghosts)
template <int DIM>
__device__ __forceinline__ bool tile_at_face(const TileD& t, const BoxD& b) {
  if (DIM == 2) return t.x0 == 0 || t.x0 + TILE_X >= b.n[0] || t.y0 == 0 || t.y0 + t.len >= b.n[1];
  return t.x0 == 0 || t.x0 + TILE_X >= b.n[0] || t.y0 == 0 || t.y0 + TILE3_Y >= b.n[1] || t.z0 == 0 ||
         t.z0 + t.len >= b.n[2];
}

// One red-black half-sweep of colour `col` in split storage (the arithmetic
// of k_march1<OP_RB>): out_c = u_c + omega (f_c - A u)_c / diag on the cells
// of colour col, u given by its halves h0, h1; fc and out are half col of f
// and of the output.  MODE 1: the interior cells of colour col are zero (the
// second half-sweep after a first one from zero; only the ghosts of colour
// col are read from half col, which may be the output half); MODE 2: u is
// zero (the first half-sweep from zero, out_c = omega f_c / diag; h0, h1
// unused); MODE 3: as MODE 0, but instead of writing half col the kernel
// adds su[0] times both cells of every aligned pair (its own new value and
// the other colour's, which it reads anyway) to the FP64 array xu of the
// same layout: the last half-sweep of a V-cycle fused with the outer update.  3D: blocks of 4 wavefronts over the sweep tiles (128 x 4
// columns), lane i of wavefront w taking the colour-col cell of row
// (y0 + w, z) in the i-th aligned pair from x0; 2D: one wavefront per tile
// (128 columns, marched along y).  The cell's x alternates between x0 + 2i
// and x0 + 2i + 1 from plane to plane while its split index moves by one
// plane stride.  Along the march the thread keeps both halves at planes
// -2..+2 in registers; x (and y) neighbours are re-read through the caches.
template <int DIM, int MODE>
__global__ void __launch_bounds__(256) k_rbs(const TileD* __restrict__ tiles, int ntiles,
                                             const BoxD* __restrict__ boxes, const float* h0, const float* h1,
                                             const float* __restrict__ fc, float* __restrict__ out, float alpha,
                                             float beta, float omega, int col, float* xg,
                                             const double* __restrict__ scal, const double* __restrict__ delta,
                                             double* __restrict__ xu, const double* __restrict__ su) {
  constexpr int M = DIM - 1;  // march direction
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  if (MODE != 2 && tile_at_face<DIM>(t, b)) {  // block-uniform
    split_ghosts<DIM>(t, b, const_cast<float*>(h0), const_cast<float*>(h1), xg, MODE == 1 ? col : -1);
    __syncthreads();
  }
  // 3D: wavefront w takes row y0 + w of the tile; 2D: one wavefront per tile
  const int i = threadIdx.x & 63, y = DIM == 3 ? t.y0 + (int)(threadIdx.x >> 6) : 0;
  const int nxh = min(TILE_X, b.n[0] - t.x0) >> 1;
  if (i >= nxh || (DIM == 3 && y >= b.n[1])) return;
  const float* __restrict__ self = col ? h1 : h0;
  const float* __restrict__ oth = col ? h0 : h1;
  const int64_t sy = b.s[1] >> 1, sz = b.s[M] >> 1;
  const int z0 = DIM == 3 ? t.z0 : t.y0, z1 = min(z0 + t.len, b.n[M]), nz = b.n[M];
  // split index of the thread's cell at march plane z0 (x = x0 + 2i + parity)
  int64_t c = (b.off >> 1) + 1 + (t.x0 >> 1) + i + (DIM == 3 ? (int64_t)(y + 2) * sy : 0) + (int64_t)(z0 + 2) * sz;
  // x parity of the colour-col cell of the pair: (col + lo + x + y + z) even
  int par = (col + b.lo[0] + b.lo[1] + b.lo[2] + t.x0 + y + z0) & 1;
  const int xa = t.x0 + 2 * i;
  const float SfA = split_sfix<DIM>(b, xa, y), SfB = split_sfix<DIM>(b, xa + 1, y);
  const float imA = 1.0f / (alpha + beta * SfA), imB = 1.0f / (alpha + beta * SfB);
  const uint8_t zl = b.ucode[M][0], zh = b.ucode[M][1];
  const float flo0 = fold<float>(zl, 0), flo1 = fold<float>(zl, 1);
  const float fhi0 = fold<float>(zh, 0), fhi1 = fold<float>(zh, 1);
  // own colour at plane q / at a neighbour: MODE 1 reads only ghosts
  constexpr bool FULL = MODE == 0 || MODE == 3;  // reads both halves in full
  auto own = [&](int64_t j, bool ghost) { return (FULL || (MODE == 1 && ghost)) ? self[j] : 0.0f; };
  // scal != null: fc holds the unscaled residual; f = (r - delta) / scal[0],
  // evaluated in FP64 as the conversion kernel (k_scale32) would
  const double finv = scal ? 1.0 / scal[0] : 1.0, fdv = (scal && delta) ? delta[b.comp] : 0.0;
  auto fval = [&](int64_t j) { return scal ? (float)(((double)fc[j] - fdv) * finv) : fc[j]; };
  const double ssc = MODE == 3 ? su[0] : 0.0;
  float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, o0 = 0.0f, o1 = 0.0f, o2 = 0.0f, o3 = 0.0f;
  if (MODE != 2) {
    s0 = own(c - 2 * sz, z0 - 2 < 0);
    s1 = own(c - sz, z0 - 1 < 0);
    s2 = own(c, false);
    s3 = own(c + sz, z0 + 1 >= nz);
    o0 = oth[c - 2 * sz];
    o1 = oth[c - sz];
    o2 = oth[c];
    o3 = oth[c + sz];
  }
  for (int z = z0; z < z1; ++z, c += sz, par ^= 1) {
    float inv;
    if (z >= 2 && z <= nz - 3) {
      inv = par ? imB : imA;
    } else {
      float S = par ? SfB : SfA;
      if (z < 2) S += z == 0 ? flo0 : flo1;
      if (z > nz - 3) S += z == nz - 1 ? fhi0 : fhi1;
      inv = 1.0f / (alpha + beta * S);
    }
    if (MODE == 2) {
      out[c] = omega * fval(c) * inv;
      continue;
    }
    const int x = xa + par, nx0 = b.n[0];
    // the row of the side buffer: (y, z) in 3D, (z, 0) in 2D
    const int gy = DIM == 3 ? y : z, gz = DIM == 3 ? z : 0;
    const float s4 = own(c + 2 * sz, z + 2 >= nz), o4 = oth[c + 2 * sz];
    // x neighbours beyond the box come from the side buffer: one load each,
    // its address chosen per lane
    const float* a_on = par ? (x + 1 >= nx0 ? x_ghost(xg, b, 1, gy, gz, 1) : oth + c + 1)
                            : (x < 1 ? x_ghost(xg, b, 0, gy, gz, 1) : oth + c - 1);
    const float on = *a_on;
    const float xm1 = par ? o2 : on, xp1 = par ? on : o2;
    const float* a_m2 = x < 2 ? x_ghost(xg, b, 0, gy, gz, 2 - x) : self + c - 1;
    const float* a_p2 = x + 2 >= nx0 ? x_ghost(xg, b, 1, gy, gz, x + 3 - nx0) : self + c + 1;
    const float xm2 = (FULL || x < 2) ? *a_m2 : 0.0f;
    const float xp2 = (FULL || x + 2 >= nx0) ? *a_p2 : 0.0f;
    float ls = 16.0f * (xm1 + xp1) - (xm2 + xp2) + 16.0f * (o1 + o3) - (s0 + s4) + float(-30 * DIM) * s2;
    if (DIM == 3) {
      const float ym2 = own(c - 2 * sy, y < 2), yp2 = own(c + 2 * sy, y + 2 >= b.n[1]);
      ls += 16.0f * (oth[c - sy] + oth[c + sy]) - (ym2 + yp2);
    }
    const float Au = alpha * s2 + beta * ls;
    const float v = s2 + omega * (fval(c) - Au) * inv;
    if (MODE == 3) {
      // the pair (elements 2c, 2c + 1) holds this cell and the other
      // colour's final value o2: x += s e for both, as k_update
      double* xp = xu + 2 * c;
      const Pair<double> xv = ld2(xp);
      const float ea = par ? o2 : v, eb = par ? v : o2;
      st2nt(xp, xv.a + ssc * (double)ea, xv.b + ssc * (double)eb);
    } else {
      out[c] = v;
    }
    s0 = s1;
    s1 = s2;
    s2 = s3;
    s3 = s4;
    o0 = o1;
    o1 = o2;
    o2 = o3;
    o3 = o4;
  }
  (void)o0;
}

// the pair of cells (x, x + 1) at element e (x even) of a split array whose
// cell x has colour cx, in x order
__device__ __forceinline__ Pair<float> split_pair_ld(const float* h0, const float* h1, int64_t e, int cx) {
  return Pair<float>{(cx ? h1 : h0)[e >> 1], (cx ? h0 : h1)[e >> 1]};
}

// Residual fused with restriction on a split iterate (halves h0, h1) and a
// split right-hand side (halves f0, f1): the arithmetic of
// k_march<OP_RESTRICT>, after the block has written the ghosts of its tile
// (read-time fill, as in k_rbs: y/z faces into the iterate's halves, x faces
// into the side buffer).  Output: the coarse right-hand side, interleaved.
template <int DIM>
__global__ void __launch_bounds__(256) k_resid_restrict_s(const TileD* __restrict__ tiles, int ntiles,
                                                          const BoxD* __restrict__ boxes, const float* h0,
                                                          const float* h1, const float* __restrict__ f0,
                                                          const float* __restrict__ f1, float* __restrict__ out,
                                                          float alpha, float beta,
                                                          const BoxD* __restrict__ cboxes, float* xg,
                                                          const double* __restrict__ scal,
                                                          const double* __restrict__ delta) {
  __shared__ float R[2][64];
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  if (tile_at_face<DIM>(t, b)) {  // block-uniform
    split_ghosts<DIM>(t, b, const_cast<float*>(h0), const_cast<float*>(h1), xg, -1);
    __syncthreads();
  }
  const Column C = column_of<DIM>(t, b);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // lanes up to two cells past the box feed the x-neighbours of the last cells
  const bool has = C.x < b.n[0] + 2 && (DIM == 2 || C.y < b.n[1]);
  const int64_t sm = C.sm, sy = b.s[1];
  int64_t c = C.base + (int64_t)(C.p0 + 2) * sm;
  // colour of cell x at plane p; the row of the side buffer at plane p
  int cx = DIM == 3 ? colour_of(b, C.x, C.y, C.p0) : colour_of(b, C.x, C.p0, 0);
  auto xgh = [&](int side, int p, int layer) {
    return *x_ghost(xg, b, side, DIM == 3 ? C.y : p, DIM == 3 ? p : 0, layer);
  };
  // unscaled residual: f = (r - delta) / scal[0] in FP64, as k_scale32
  const double finv = scal ? 1.0 / scal[0] : 1.0, fdv = scal && delta ? delta[b.comp] : 0.0;
  Pair<float> q0{}, q1{}, q2{}, q3{}, q4{};
  if (has) {
    q0 = split_pair_ld(h0, h1, c - 2 * sm, cx);
    q1 = split_pair_ld(h0, h1, c - sm, cx ^ 1);
    q2 = split_pair_ld(h0, h1, c, cx);
    q3 = split_pair_ld(h0, h1, c + sm, cx ^ 1);
  }
  float acc = 0.0f;
  for (int p = C.p0; p < C.p1; ++p, c += sm, cx ^= 1) {
    if (has) q4 = split_pair_ld(h0, h1, c + 2 * sm, cx);
    // the lane whose pair is the x-high ghost pair feeds its left neighbour
    // from the side buffer
    Pair<float> sq = q2;
    if (C.x == b.n[0] && (DIM == 2 || C.y < b.n[1])) sq = Pair<float>{xgh(1, p, 1), xgh(1, p, 2)};
    float La = __shfl_up(sq.a, 1, 64), Lb = __shfl_up(sq.b, 1, 64);
    float Ra = __shfl_down(sq.a, 1, 64), Rb = __shfl_down(sq.b, 1, 64);
    float o0 = 0.0f, o1 = 0.0f;
    if (C.ok) {
      if (lane == 0) {
        if (C.x == 0) {
          La = xgh(0, p, 2);
          Lb = xgh(0, p, 1);
        } else {
          const Pair<float> l = split_pair_ld(h0, h1, c - 2, cx);
          La = l.a;
          Lb = l.b;
        }
      }
      if (lane == 63) {
        if (C.x + 2 == b.n[0]) {
          Ra = xgh(1, p, 1);
          Rb = xgh(1, p, 2);
        } else {
          const Pair<float> r = split_pair_ld(h0, h1, c + 2, cx);
          Ra = r.a;
          Rb = r.b;
        }
      }
      float s0 = 16.0f * (Lb + q2.b) - (La + Ra) + 16.0f * (q1.a + q3.a) - (q0.a + q4.a) + float(-30 * DIM) * q2.a;
      float s1 = 16.0f * (q2.a + Ra) - (Lb + Rb) + 16.0f * (q1.b + q3.b) - (q0.b + q4.b) + float(-30 * DIM) * q2.b;
      if (DIM == 3) {
        const Pair<float> ym1 = split_pair_ld(h0, h1, c - sy, cx ^ 1), yp1 = split_pair_ld(h0, h1, c + sy, cx ^ 1),
                          ym2 = split_pair_ld(h0, h1, c - 2 * sy, cx), yp2 = split_pair_ld(h0, h1, c + 2 * sy, cx);
        s0 += 16.0f * (ym1.a + yp1.a) - (ym2.a + yp2.a);
        s1 += 16.0f * (ym1.b + yp1.b) - (ym2.b + yp2.b);
      }
      const float A0 = alpha * q2.a + beta * s0, A1 = alpha * q2.b + beta * s1;
      Pair<float> fv = split_pair_ld(f0, f1, c, cx);
      if (scal) fv = Pair<float>{(float)(((double)fv.a - fdv) * finv), (float)(((double)fv.b - fdv) * finv)};
      o0 = fv.a - A0;
      o1 = fv.b - A1;
    }
    acc += o0 + o1;  // x pair (fine sizes are even, so both cells exist)
    if ((p - C.p0) & 1) {
      if (DIM == 3) {
        if (w & 1) R[w >> 1][lane] = acc;
        __syncthreads();
        if (!(w & 1) && C.ok) {
          const BoxD cb = cboxes[b.coarse];
          out[cell_index<3>(cb, C.x >> 1, C.y >> 1, p >> 1)] = (acc + R[w >> 1][lane]) * 0.125f;
        }
        __syncthreads();
      } else if (C.ok) {
        const BoxD cb = cboxes[b.coarse];
        out[cell_index<2>(cb, C.x >> 1, p >> 1, 0)] = acc * 0.25f;
      }
      acc = 0.0f;
    }
    q0 = q1;
    q1 = q2;
    q2 = q3;
    q3 = q4;
  }
}

// Prolongation in split storage: out = u + P ec (the arithmetic of
// k_prolong), u and out split (halves u0, u1 and o0, o1)
template <int DIM>
__global__ void __launch_bounds__(256) k_prolong_s(const TileD* __restrict__ tiles, int ntiles,
                                                   const BoxD* __restrict__ boxes, const BoxD* __restrict__ cboxes,
                                                   const float* __restrict__ ec, const float* __restrict__ u0,
                                                   const float* __restrict__ u1, float* __restrict__ o0,
                                                   float* __restrict__ o1) {
  FOR_COLUMN(DIM) {
    const int cy = DIM == 2 ? p : C.y, cz = DIM == 2 ? 0 : p;
    const BoxD cb = cboxes[b.coarse];
    const int64_t q = cell_index<DIM>(cb, C.x >> 1, cy >> 1, cz >> 1);
    float common = float(1.0 - DIM * 0.25) * ec[q] + 0.25f * ec[q + ((cy & 1) ? cb.s[1] : -cb.s[1])];
    if (DIM == 3) common += 0.25f * ec[q + ((cz & 1) ? cb.s[2] : -cb.s[2])];
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    const int cx = colour_of(b, C.x, cy, cz);
    const Pair<float> uv = split_pair_ld(u0, u1, c, cx);
    (cx ? o1 : o0)[c >> 1] = uv.a + (common + 0.25f * ec[q - 1]);
    (cx ? o0 : o1)[c >> 1] = uv.b + (common + 0.25f * ec[q + 1]);
  }
}

// ---------------------------------------------------------------------------
// ghost fill: one wavefront per chunk of up to 64 face columns.  MODE 0: the
// fill; 1: the ghosts of the transposed operator (filled columns 0,
// exchange copied; the fill's contribution is added by k_band instead);
// 2: every ghost 0
template <typename T, int MODE>
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
  if (MODE == 0 && (ch.kind1 == G_FILL_D || ch.kind1 == G_FILL_N || ch.kind2 == G_FILL_D || ch.kind2 == G_FILL_N)) {
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
  if (MODE != 2 && ch.kind1 == G_EXCH) v1 = u[ch.src1 + (int64_t)lane * ch.sstride1];
  if (MODE != 2 && ch.kind2 == G_EXCH) v2 = u[ch.src2 + (int64_t)lane * ch.sstride2];
  u[g1] = v1;
  u[g1 + n] = v2;
}

// exact bottom solve: e = M f (TR: e = M^T f, the adjoint system) for every
// instance of every group.  Both M and M^T are stored column-major, so the
// lanes of a column read consecutive rows.  A block takes 8 rows; its 32
// thread groups split the columns (group p takes columns p, p + 32, ...), so
// every thread has only n / 32 independent loads per instance batch, and the
// 32 partial sums of a row are added in LDS.
template <typename T, bool TR>
__global__ void __launch_bounds__(256) k_bottom(const BottomGroupD* __restrict__ groups,
                                                const double* __restrict__ mats, const int64_t* __restrict__ idx,
                                                const T* __restrict__ f, T* __restrict__ e, T* __restrict__ e2) {
  constexpr int NI = 8, KC = 512, RB = 8, KP = 32;
  __shared__ double xs[NI][KC];
  __shared__ double red[KP][NI][RB];
  const BottomGroupD G = groups[blockIdx.y];
  if ((int)(blockIdx.x * RB) >= G.n) return;  // uniform per block
  const int rl = (int)threadIdx.x % RB, part = (int)threadIdx.x / RB;
  const int r = blockIdx.x * RB + rl;
  const double* M = mats + (TR ? G.matT : G.mat);
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
#pragma unroll 4
        for (int k = part; k < kc; k += KP) {
          const double m = M[(int64_t)(k0 + k) * G.n + r];
#pragma unroll
          for (int i = 0; i < NI; ++i) acc[i] += m * xs[i][k];
        }
      }
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) red[part][i][rl] = acc[i];
    __syncthreads();
    if (part == 0 && r < G.n)
      for (int i = 0; i < ni; ++i) {
        double s = 0.0;
        for (int p = 0; p < KP; ++p) s += red[p][i][rl];
        const int64_t q = idx[G.idx + (int64_t)(i0 + i) * G.n + r];
        e[q] = (T)s;
        if (e2) e2[q] = (T)s;
      }
  }
}

// ---------------------------------------------------------------------------
// transposed operator (adjoint system): contribution of the ghost fill.
//
// The homogeneous operator reads the two ghosts of a filled column, which the
// fill computes from the first four cells of that row; the end cell puts
// weight 16 on ghost 1 and -1 on ghost 2, the next cell -1 on ghost 1.  The
// transpose therefore adds to the cell at distance p (0..3) from the face
//   w1[p] (16 l0 - l1) + w2[p] (-l0)   (units of 1 / 12 h^2),
// l0, l1 the first two cells of the row and w1, w2 the coefficients of the
// cell in the first and second ghost of eqs. (velBCHomoDiri5th) and
// (Neumann5).  The stencil part of the transpose is the stencil itself (it is
// symmetric) on the array whose filled ghosts are 0 (k_fill<T, true>).
// MODE 0: out += scale * delta (residual or operator); 1: Jacobi, out +=
// scale * delta / diag; 2: red-black, the same on cells of colour `col`.
__constant__ double kFillW[2][2][4] = {
    {{-77.0 / 12, 43.0 / 12, -17.0 / 12, 3.0 / 12}, {-505.0 / 12, 335.0 / 12, -145.0 / 12, 27.0 / 12}},
    {{0.5, 0.9, -0.5, 0.1}, {-7.5, 14.5, -7.5, 1.5}}};

template <typename T, int DIM, int MODE>
__global__ void __launch_bounds__(256) k_band(const BandChunkD* __restrict__ chunks, int nchunks,
                                              const BoxD* __restrict__ boxes, const uint8_t* __restrict__ codes,
                                              const T* __restrict__ u, T* __restrict__ out, T alpha, T beta, T scale,
                                              int col) {
  const int ci = blockIdx.x;
  if (ci >= nchunks) return;
  const BandChunkD ch = chunks[ci];
  if ((int)threadIdx.x >= ch.count) return;
  const BoxD b = boxes[ch.box];
  const int k = ch.start + (int)threadIdx.x;
  const int d = ch.face >> 1, s = ch.face & 1;
  int x[3] = {0, 0, 0};
  if (d == 0) {  // distance fastest: rows along x are contiguous
    const int p = k & 3, r = k >> 2;
    x[0] = s ? b.n[0] - 1 - p : p;
    x[1] = r % b.n[1];
    x[2] = r / b.n[1];
  } else if (d == 1) {
    const int r = k / b.n[0], p = r & 3;
    x[0] = k % b.n[0];
    x[1] = s ? b.n[1] - 1 - p : p;
    x[2] = r >> 2;
  } else {
    const int r = k / b.n[0], p = r / b.n[1];
    x[0] = k % b.n[0];
    x[1] = r % b.n[1];
    x[2] = s ? b.n[2] - 1 - p : p;
  }
  for (int f = 0; f < ch.face; ++f) {  // owned by an earlier filled face
    if (!((ch.fmask >> f) & 1)) continue;
    const int e = f >> 1;
    if (((f & 1) ? b.n[e] - 1 - x[e] : x[e]) < 4) return;
  }
  T delta = T(0);
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) {
    if (!((ch.fmask >> f) & 1)) continue;
    const int e = f >> 1, sd = f & 1;
    const int dist = sd ? b.n[e] - 1 - x[e] : x[e];
    if (dist >= 4) continue;
    int colx;
    if (DIM == 2)
      colx = e == 0 ? x[1] : x[0];
    else
      colx = e == 0 ? x[1] + b.n[1] * x[2] : (e == 1 ? x[0] + b.n[0] * x[2] : x[0] + b.n[0] * x[1]);
    const uint8_t cd = codes[b.code_off[e][sd] + colx];
    const int kind = cd & 3;
    if (!kind) continue;
    int y[3] = {x[0], x[1], x[2]};
    y[e] = sd ? b.n[e] - 1 : 0;
    const int64_t e0 = cell_index<DIM>(b, y[0], y[1], y[2]);
    const int64_t in = (e == 0 ? 1 : (int64_t)b.s[e]) * (sd ? -1 : 1);
    const T l0 = u[e0], l1 = u[e0 + in];
    delta += T(kFillW[kind - 1][0][dist]) * (T(16) * l0 - l1);
    if (cd & 4) delta -= T(kFillW[kind - 1][1][dist]) * l0;
  }
  const int64_t c = cell_index<DIM>(b, x[0], x[1], x[2]);
  if (MODE == 0) {
    out[c] += scale * delta;
    return;
  }
  if (MODE == 2 && ((b.lo[0] + x[0] + b.lo[1] + x[1] + (DIM == 3 ? b.lo[2] + x[2] : 0)) & 1) != col) return;
  out[c] += scale * delta / (alpha + beta * (T(-30 * DIM) + fold_at<T, DIM>(b, codes, x[0], x[1], x[2])));
}

// discrete gradient, eq. (discreteOps a): g[d] = (-u[+2] + 8 u[+1] - 8 u[-1]
// + u[-2]) / 12h along d, from u with its ghosts filled; w != NULL: g[d] =
// w[d] - that (the projection's correction u = w - G phi)
template <int DIM>
__global__ void __launch_bounds__(256) k_grad(const TileD* __restrict__ tiles, int ntiles,
                                              const BoxD* __restrict__ boxes, const double* __restrict__ u,
                                              DPtrs g, CPtrs w, bool sub, double inv12h) {
  FOR_COLUMN(DIM) {
    const int64_t c0 = C.base + (int64_t)(p + 2) * C.sm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j == 1 && !C.ok1) break;
      const int64_t c = c0 + j;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int64_t s = d == 0 ? 1 : (int64_t)b.s[d];
        const double v = (-u[c + 2 * s] + 8.0 * u[c + s] - 8.0 * u[c - s] + u[c - 2 * s]) * inv12h;
        g.p[d][c] = sub ? w.p[d][c] - v : v;
      }
    }
  }
}

// discrete divergence, eq. (discreteOps b): sum over d of the gradient of
// w[d] along d (ghosts of every component filled)
template <int DIM>
__global__ void __launch_bounds__(256) k_div(const TileD* __restrict__ tiles, int ntiles,
                                             const BoxD* __restrict__ boxes, CPtrs w, double* __restrict__ out,
                                             double inv12h) {
  FOR_COLUMN(DIM) {
    const int64_t c0 = C.base + (int64_t)(p + 2) * C.sm;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      if (j == 1 && !C.ok1) break;
      const int64_t c = c0 + j;
      double acc = 0.0;
#pragma unroll
      for (int d = 0; d < DIM; ++d) {
        const int64_t s = d == 0 ? 1 : (int64_t)b.s[d];
        const double* a = w.p[d];
        acc += (-a[c + 2 * s] + 8.0 * a[c + s] - 8.0 * a[c - s] + a[c - 2 * s]);
      }
      out[c] = acc * inv12h;
    }
  }
}

// Ghost-slot adjoints of the gradient stencil (the transposes of G and D):
// along the normal d of a face, the row-end cell e0 reads its first ghost
// with the weight a(sg) = 8 sg / 12h and its second with a(2 sg) = -sg / 12h,
// the next cell e1 reads the first ghost with a(2 sg) (sg = +1 on a high
// face, -1 on a low one; eq. discreteOps a).  ab[slot] -= sum of the weights
// times mu[cell] (ab holds the negated adjoint, the convention of the
// scatter kernels k_band_ab, k_exch_T and k_cfi_T, which subtract it).
// mu.p[d]: the array read along d; dir >= 0: faces normal to dir only.  One
// wavefront per chunk of ghost columns; every slot belongs to one chunk.
__global__ void __launch_bounds__(256) k_gslot(const ChunkD* __restrict__ chunks, int nchunks, CPtrs mu, int dir,
                                               double* __restrict__ ab, double inv12h) {
  const int ci = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (ci >= nchunks) return;
  const ChunkD ch = chunks[ci];
  if (lane >= ch.count || (dir >= 0 && ch.dir != dir)) return;
  const double* __restrict__ m = mu.p[ch.dir];
  const int64_t g1 = ch.dst + (int64_t)lane * ch.cstride, ns = ch.nstride;
  const double sg = ns > 0 ? 1.0 : -1.0;
  const double m0 = m[g1 - ns], m1 = m[g1 - 2 * ns];
  ab[g1] -= sg * (8.0 * m0 - m1) * inv12h;
  ab[g1 + ns] -= -sg * m0 * inv12h;
}

// ---------------------------------------------------------------------------
// coarse-fine interface conditions (CIC-1..3 of Section 6.3).  One thread per
// face-data entry of a coarse-fine face: the four fine cells across the face
// along the outward normal are interpolated (AMRCFI) from the coarse data of
// four earlier times, combined by eq. cell2face into the face average (kind
// 0, weights (-1, 7, 7, -1) / 12) or the outward normal derivative (kind 1,
// (1, -15, 15, -1) / 12h), and taken to the time t* by the two rows tw0, tw1
// of eq. timeInterp; every step is linear, so the coarse data are combined
// in time first.  fd[entry] = value at t*, dfd[entry] (may be null) = its
// time derivative.
struct CoarseHist {
  const double* p[4];  // phi(t_-i), i = 0..3
};
struct TimeW {
  double v[4], d[4];  // weights of phi(t_-i) for the value and the derivative
};
template <int DIM>
__global__ void __launch_bounds__(256) k_cic(int n, const int64_t* __restrict__ fdi, const int32_t* __restrict__ src,
                                             const uint8_t* __restrict__ wsel, const double* __restrict__ W,
                                             CoarseHist hist, TimeW tw, int kind, double inv12h,
                                             double* __restrict__ fd, double* __restrict__ dfd) {
  constexpr int NW = DIM == 2 ? 25 : 125;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const double cv[4] = {-1.0 / 12.0, 7.0 / 12.0, 7.0 / 12.0, -1.0 / 12.0};
  const double cd[4] = {inv12h, -15.0 * inv12h, 15.0 * inv12h, -inv12h};
  double a0 = 0.0, a1 = 0.0;
  for (int p = 0; p < 4; ++p) {
    const int q = j * 4 + p;
    const uint8_t* ws = wsel + (size_t)q * DIM;
    const int32_t* sr = src + (size_t)q * NW;
    double b0 = 0.0, b1 = 0.0;
    for (int m = 0; m < NW; ++m) {
      double w = W[5 * ws[0] + m % 5] * W[5 * ws[1] + (m / 5) % 5];
      if (DIM == 3) w *= W[5 * ws[2] + m / 25];
      const int32_t e = sr[m];
      double v = 0.0, dv = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double c = hist.p[i][e];
        v += tw.v[i] * c;
        dv += tw.d[i] * c;
      }
      b0 += w * v;
      b1 += w * dv;
    }
    const double cf = kind == 0 ? cv[p] : cd[p];
    a0 += cf * b0;
    a1 += cf * b1;
  }
  fd[fdi[j]] = a0;
  if (dfd) dfd[fdi[j]] = a1;
}

// eq. correctingFaceAvg on a velocity's face data (fdv.p[d]: component d):
// per component c, sum over its faces with face data (coarse-fine and
// physical) of the outward normal component, sign(outward) * fdv[normal
// direction]; then delta[c] = -sum / (coarse-fine entries of c), 0 without
// any.  One block per component, the component's chunks in list order.
__global__ void __launch_bounds__(256) k_cic_sum(const ChunkD* __restrict__ chunks, const int32_t* __restrict__ ptr,
                                                 const int32_t* __restrict__ idx, DPtrs fdv,
                                                 const double* __restrict__ ncf, double* __restrict__ delta) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  const int a = ptr[c], b = ptr[c + 1];
  double v = 0.0;
  for (int k = a * 64 + (int)threadIdx.x; k < b * 64; k += 256) {
    const ChunkD ch = chunks[idx[k >> 6]];
    const int lane = k & 63;
    if (lane >= ch.count || ch.fd < 0 || (ch.kind1 != G_FILL_D && ch.kind1 != G_FILL_N)) continue;
    v += (ch.nstride > 0 ? 1.0 : -1.0) * fdv.p[ch.dir][ch.fd + lane];
  }
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) delta[c] = ncf[c] > 0.0 ? -v / ncf[c] : 0.0;
}

// the correction: fdv[d] += sign(outward) * delta[component] on the
// coarse-fine face entries of faces normal to d
__global__ void __launch_bounds__(256) k_cic_fix(const ChunkD* __restrict__ chunks, int nchunks,
                                                 const BoxD* __restrict__ boxes, DPtrs fdv,
                                                 const double* __restrict__ delta) {
  const int ci = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (ci >= nchunks) return;
  const ChunkD ch = chunks[ci];
  if (lane >= ch.count || !ch.cf || ch.fd < 0 || (ch.kind1 != G_FILL_D && ch.kind1 != G_FILL_N)) return;
  fdv.p[ch.dir][ch.fd + lane] += (ch.nstride > 0 ? 1.0 : -1.0) * delta[boxes[ch.box].comp];
}

// per-tile sum of a * b over the interior (dot products)
template <int DIM>
__global__ void __launch_bounds__(256) k_tile_dot(const TileD* __restrict__ tiles, int ntiles,
                                                  const BoxD* __restrict__ boxes, const double* __restrict__ a,
                                                  const double* __restrict__ bb, double* __restrict__ part) {
  __shared__ double sh[4];
  const int ti = tile_of_block(ntiles);
  if (ti < 0) return;
  const TileD t = tiles[ti];
  const BoxD b = boxes[t.box];
  const Column C = column_of<DIM>(t, b);
  double v = 0.0;
  if (C.ok)
    for (int p = C.p0; p < C.p1; ++p) {
      const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
      v += a[c] * bb[c];
      if (C.ok1) v += a[c + 1] * bb[c + 1];
    }
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) part[ti] = v;
}

// segmented reduction in a fixed order: out[s] = sum (or max) of in over
// [ptr[s], ptr[s+1]); ptr == NULL means the single segment [0, n).  One
// block per segment.
template <bool MAX>
// host (may be null): pinned host memory that also receives the results,
// stored at system scope, so the host reads them after the stream's
// synchronisation without a copy
__global__ void __launch_bounds__(256) k_seg_reduce(const double* __restrict__ in, const int32_t* __restrict__ ptr,
                                                    int n, double* __restrict__ out, double* host) {
  __shared__ double sh[4];
  const int s = blockIdx.x;
  const int a = ptr ? ptr[s] : 0, b = ptr ? ptr[s + 1] : n;
  double v = 0.0;
  for (int j = a + (int)threadIdx.x; j < b; j += 256) v = MAX ? fmax(v, in[j]) : v + in[j];
  v = MAX ? block_max<double>(v, sh) : block_sum<double>(v, sh);
  if (threadIdx.x == 0) {
    out[s] = v;
    if (host) {
      __hip_atomic_store(host + s, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __threadfence_system();
    }
  }
}

// per-component sums of chunk partials in a fixed order; one block per component
__global__ void __launch_bounds__(256) k_comp_sum(const double* __restrict__ part, const int32_t* __restrict__ ptr,
                                                  const int32_t* __restrict__ ids, double* __restrict__ out) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  double v = 0.0;
  for (int j = ptr[c] + threadIdx.x; j < ptr[c + 1]; j += 256) v += part[ids[j]];
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) out[c] = v;
}

// per-component means of tile partials in one launch: block c sums the
// partials of component c's tiles (a contiguous range) in a fixed order and
// writes delta[c] = flag[c] ? sum / cnt[c] : 0
__global__ void __launch_bounds__(256) k_comp_mean_delta(const double* __restrict__ part,
                                                         const int32_t* __restrict__ seg,
                                                         const int32_t* __restrict__ cseg,
                                                         const int32_t* __restrict__ flag,
                                                         const double* __restrict__ cnt, double* __restrict__ delta) {
  __shared__ double sh[4];
  const int c = blockIdx.x;
  // the flag and the segment range are loaded together (one round trip less)
  const int32_t fl = flag[c], a = seg[cseg[c]], b = seg[cseg[c + 1]];
  if (!fl) {  // block-uniform
    if (threadIdx.x == 0) delta[c] = 0.0;
    return;
  }
  double v = 0.0;
  for (int j = a + (int)threadIdx.x; j < b; j += 256) v += part[j];
  v = block_sum<double>(v, sh);
  if (threadIdx.x == 0) delta[c] = v / (cnt[c] * 1.0);
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

// solvability by the coarse-fine face-data correction (eq. correctingFaceAvg):
// per singular component with coarse-fine Neumann faces, dfd = defect /
// (h^(D-1) ncf) and no RHS shift; otherwise the RHS shift of k_comp_delta
__global__ void k_cf_delta(const double* __restrict__ defect, const int32_t* __restrict__ flag,
                           const double* __restrict__ ncf, const double* __restrict__ cnt, int ncomp, double hD,
                           double hD1, double* __restrict__ delta, double* __restrict__ dfd) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncomp) return;
  double dv = 0.0, dq = 0.0;
  if (flag[c]) {
    if (ncf[c] > 0)
      dq = defect[c] / (hD1 * ncf[c]);
    else
      dv = defect[c] / (cnt[c] * hD);
  }
  delta[c] = dv;
  dfd[c] = dq;
}

// corrected face data: out = fd (0 if NULL) + dfd[component] on coarse-fine
// Neumann columns
__global__ void __launch_bounds__(256) k_fd_correct(const ChunkD* __restrict__ chunks, int nchunks,
                                                    const BoxD* __restrict__ boxes, const double* __restrict__ fd,
                                                    const double* __restrict__ dfd, double* __restrict__ out) {
  const int ci = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (ci >= nchunks) return;
  const ChunkD ch = chunks[ci];
  if (lane >= ch.count || ch.fd < 0) return;
  double v = fd ? fd[ch.fd + lane] : 0.0;
  if (ch.cf && ch.kind1 == G_FILL_N) v += dfd[boxes[ch.box].comp];
  out[ch.fd + lane] = v;
}

// sum of face data over Neumann-filled ghost columns of each chunk
__global__ void __launch_bounds__(256) k_chunk_fdsum(const ChunkD* __restrict__ chunks, int nchunks,
                                                     const double* __restrict__ fd, const uint8_t* __restrict__ valid,
                                                     double* __restrict__ part) {
  const int ci = blockIdx.x * 256 + threadIdx.x;
  if (ci >= nchunks) return;
  const ChunkD ch = chunks[ci];
  double s = 0.0;
  if (ch.kind1 == G_FILL_N && ch.fd >= 0)
    for (int i = 0; i < ch.count; ++i)
      if (!valid || valid[ch.fd + i]) s += fd[ch.fd + i];
  part[ci] = s;
}

// scal[dst] = src[0] (device-side scalar copy, keeps the scale on the device)
__global__ void k_set_scale(const double* __restrict__ src, double* __restrict__ dst) { *dst = *src; }
__global__ void k_set_scaled(const double* __restrict__ src, double f, double* __restrict__ dst) { *dst = f * *src; }

// zero a whole buffer (used in place of memset nodes in captured graphs)
template <typename T>
__global__ void k_zero(T* __restrict__ a, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = T(0);
}


// ---------------------------------------------------------------------------
// composite (multi-level) operator

// interpolated ghosts of the finer level: u_f[dst] = sum over the 5^DIM
// window of the tensor-product weights times the coarse values
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_cfi(int n, const int64_t* __restrict__ dst, const int32_t* __restrict__ src,
                                             const uint8_t* __restrict__ wsel, const double* __restrict__ W,
                                             const T* __restrict__ uc, T* __restrict__ uf) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  constexpr int NW = DIM == 2 ? 25 : 125;
  const int32_t* s = src + (int64_t)i * NW;
  const double* wx = W + 5 * wsel[i * DIM];
  const double* wy = W + 5 * wsel[i * DIM + 1];
  const double* wz = DIM == 3 ? W + 5 * wsel[i * DIM + 2] : nullptr;
  double acc = 0.0;
  for (int k = 0; k < (DIM == 3 ? 5 : 1); ++k) {
    double plane = 0.0;
    for (int j = 0; j < 5; ++j) {
      double row = 0.0;
#pragma unroll
      for (int m = 0; m < 5; ++m) row += wx[m] * (double)uc[s[k * 25 + j * 5 + m]];
      plane += wy[j] * row;
    }
    acc += (DIM == 3 ? wz[k] : 1.0) * plane;
  }
  uf[dst[i]] = (T)acc;
}

// sum of the r^DIM children of a coarse cell (the first child at e.fe)
template <typename T, int DIM>
__device__ __forceinline__ T children_sum(const AvgD& e, const T* __restrict__ uf, int r) {
  if (r == 2) {
    T s = uf[e.fe] + uf[e.fe + 1] + uf[e.fe + e.fs1] + uf[e.fe + e.fs1 + 1];
    if (DIM == 3)
      s += uf[e.fe + e.fs2] + uf[e.fe + e.fs2 + 1] + uf[e.fe + e.fs2 + e.fs1] + uf[e.fe + e.fs2 + e.fs1 + 1];
    return s;
  }
  T s = T(0);
  for (int cz = 0; cz < (DIM == 3 ? r : 1); ++cz)
    for (int cy = 0; cy < r; ++cy)
      for (int cx = 0; cx < r; ++cx) s += uf[e.fe + cx + (int64_t)cy * e.fs1 + (int64_t)cz * e.fs2];
  return s;
}

// coarse cell := mean of its r^DIM children
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_avgdown(int n, const AvgD* __restrict__ a, const T* __restrict__ uf,
                                                 T* __restrict__ uc, int r) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const AvgD e = a[i];
  const T s = children_sum<T, DIM>(e, uf, r);
  if (r == 2)
    uc[e.ce] = s * T(DIM == 2 ? 0.25 : 0.125);
  else
    uc[e.ce] = s * T(1.0 / (DIM == 2 ? r * r : r * r * r));
}

// refluxing: r[c] += kappa * sum over the cell's coarse-fine faces of
// (mean fine flux - coarse flux) / hc, fluxes = fourth-order derivatives
// along the normal n pointing into the finer level; ratio^(DIM-1) fine faces
// cover a coarse face
template <int DIM>
__global__ void __launch_bounds__(256) k_reflux(int ncell, const int64_t* __restrict__ cell,
                                                const int32_t* __restrict__ ptr, const RfxFaceD* __restrict__ faces,
                                                const double* __restrict__ uc, const double* __restrict__ uf,
                                                double* __restrict__ r, double kappa, double inv12hc, double inv12hf,
                                                double inv_hc, int ratio) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ncell) return;
  const int64_t c = cell[i];
  double corr = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const RfxFaceD F = faces[k];
    const int64_t n = F.csn;
    const double Fc = (-uc[c + 2 * n] + 15.0 * uc[c + n] - 15.0 * uc[c] + uc[c - n]) * inv12hc;
    const int64_t fn = F.fsn;
    const int nt = DIM == 2 ? ratio : ratio * ratio;
    double Ff = 0.0;
    for (int t = 0; t < nt; ++t) {
      const int64_t e = F.fe + (int64_t)(t % ratio) * F.ft0 + (int64_t)(t / ratio) * F.ft1;
      Ff += (-uf[e + fn] + 15.0 * uf[e] - 15.0 * uf[e - fn] + uf[e - 2 * fn]) * inv12hf;
    }
    Ff *= 1.0 / nt;
    corr += (Ff - Fc) * inv_hc;
  }
  r[c] += kappa * corr;
}

// refluxing of the divergence (COH-3 for eq. discreteOps b in divergence
// form): div[c] += sum over the cell's coarse-fine faces of
// sg (mean fine face average - coarse face average of w_d) / hc, face
// averages by eq. (cell2face, first row); w[d]: component d
template <int DIM>
__global__ void __launch_bounds__(256) k_reflux_div(int ncell, const int64_t* __restrict__ cell,
                                                    const int32_t* __restrict__ ptr,
                                                    const RfxFaceD* __restrict__ faces, CPtrs wc, CPtrs wf,
                                                    double* __restrict__ div,
                                                    double inv_hc, int ratio) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= ncell) return;
  const int64_t c = cell[i];
  double corr = 0.0;
  for (int k = ptr[i]; k < ptr[i + 1]; ++k) {
    const RfxFaceD F = faces[k];
    const double* uc = F.d == 0 ? wc.p[0] : (F.d == 1 ? wc.p[1] : wc.p[2]);
    const double* uf = F.d == 0 ? wf.p[0] : (F.d == 1 ? wf.p[1] : wf.p[2]);
    const int64_t n = F.csn;
    const double Fc = (-uc[c + 2 * n] + 7.0 * uc[c + n] + 7.0 * uc[c] - uc[c - n]) * (1.0 / 12.0);
    const int64_t fn = F.fsn;
    const int nt = DIM == 2 ? ratio : ratio * ratio;
    double Ff = 0.0;
    for (int t = 0; t < nt; ++t) {
      const int64_t e = F.fe + (int64_t)(t % ratio) * F.ft0 + (int64_t)(t / ratio) * F.ft1;
      Ff += (-uf[e + fn] + 7.0 * uf[e] + 7.0 * uf[e - fn] - uf[e - 2 * fn]) * (1.0 / 12.0);
    }
    Ff *= 1.0 / nt;
    corr += F.sg * (Ff - Fc) * inv_hc;
  }
  div[c] += corr;
}

// prolongation of a coarse correction onto the finer level (face-neighbour
// linear): a child whose centre lies delta_d parent widths from the
// parent's centre along d takes (1 - sum |delta_d|) E[P] + sum |delta_d|
// E[P + sign(delta_d) e_d] (ratio 2: delta = +-1/4); u += v, and ef = v
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_amr_prolong(int n, const ProlD* __restrict__ p, const T* __restrict__ ec,
                                                     T* __restrict__ u, T* __restrict__ ef, T scale, int r) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const ProlD q = p[i];
  const int a0 = q.child & 3, a1 = (q.child >> 2) & 3, a2 = (q.child >> 4) & 3;
  T v;
  if (r == 2) {
    v = T(1.0 - DIM * 0.25) * ec[q.pe] + T(0.25) * (ec[q.pe + (a0 ? 1 : -1)] + ec[q.pe + (a1 ? q.cs1 : -q.cs1)]);
    if (DIM == 3) v += T(0.25) * ec[q.pe + (a2 ? q.cs2 : -q.cs2)];
  } else {
    const T d0 = (T(a0) + T(0.5)) / T(r) - T(0.5), d1 = (T(a1) + T(0.5)) / T(r) - T(0.5);
    const T d2 = DIM == 3 ? (T(a2) + T(0.5)) / T(r) - T(0.5) : T(0);
    const T w0 = d0 < T(0) ? -d0 : d0, w1 = d1 < T(0) ? -d1 : d1, w2 = d2 < T(0) ? -d2 : d2;
    v = (T(1) - (w0 + w1 + w2)) * ec[q.pe];
    v += w0 * ec[q.pe + (d0 > T(0) ? 1 : -1)];
    v += w1 * ec[q.pe + (d1 > T(0) ? q.cs1 : -q.cs1)];
    if (DIM == 3) v += w2 * ec[q.pe + (d2 > T(0) ? q.cs2 : -q.cs2)];
  }
  v *= scale;
  u[q.fe] += v;
  if (ef) ef[q.fe] = v;
}

// ---------------------------------------------------------------------------
// adjoint of the composite operator (gathers over host-built transposes)

// a[e] = 0 on the coarse cells under the finer level
__global__ void __launch_bounds__(256) k_zero_covered(int n, const AvgD* __restrict__ a, double* __restrict__ u) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i < n) u[a[i].ce] = 0.0;
}

// coarse cell := scale * (sum of its r^DIM children)
template <int DIM>
__global__ void __launch_bounds__(256) k_sumdown(int n, const AvgD* __restrict__ a, const double* __restrict__ uf,
                                                 double* __restrict__ uc, double scale, int r) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const AvgD e = a[i];
  uc[e.ce] = children_sum<double, DIM>(e, uf, r) * scale;
}

// refluxing, transposed: out[elem[k]] += lscale * sum over entries of
// coef * lam[cell[src]]
__global__ void __launch_bounds__(256) k_rfx_T(int n, const int64_t* __restrict__ elem,
                                               const int32_t* __restrict__ ptr, const int32_t* __restrict__ src,
                                               const double* __restrict__ coef, const int64_t* __restrict__ cell,
                                               const double* __restrict__ lam, double lscale,
                                               double* __restrict__ out) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int j = ptr[k]; j < ptr[k + 1]; ++j) acc += coef[j] * lam[cell[src[j]]];
  out[elem[k]] += lscale * acc;
}

// exchange, transposed: r[source] -= sum of the adjoints in the ghost slots
// that copy it
__global__ void __launch_bounds__(256) k_exch_T(int n, const int64_t* __restrict__ elem,
                                                const int32_t* __restrict__ ptr, const int64_t* __restrict__ slot,
                                                const double* __restrict__ ab, double* __restrict__ r) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int j = ptr[k]; j < ptr[k + 1]; ++j) acc += ab[slot[j]];
  r[elem[k]] -= acc;
}

// adjoint of every interpolated ghost: the stencil weight its own row puts
// on it (beta (16 l0 - l1) for layer 1, -beta l0 for layer 2) plus what
// refluxing put in its slot
__global__ void __launch_bounds__(256) k_cfi_mu(int n, const int64_t* __restrict__ e0, const int32_t* __restrict__ in,
                                                const uint8_t* __restrict__ layer, const int64_t* __restrict__ dst,
                                                const double* __restrict__ lam, const double* __restrict__ ab,
                                                double beta, double* __restrict__ mu) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const double l0 = lam[e0[i]];
  const double v = layer[i] == 1 ? 16.0 * l0 - lam[e0[i] + in[i]] : -l0;
  mu[i] = beta * v + ab[dst[i]];
}

// AMRCFI, transposed: r[coarse window cell] -= sum of weight * mu
template <int DIM>
__global__ void __launch_bounds__(256) k_cfi_T(int n, const int64_t* __restrict__ elem, const int32_t* __restrict__ ptr,
                                               const int32_t* __restrict__ ent, const uint8_t* __restrict__ wsel,
                                               const double* __restrict__ W, const double* __restrict__ mu,
                                               double* __restrict__ r) {
  constexpr int NW = DIM == 2 ? 25 : 125;
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= n) return;
  double acc = 0.0;
  for (int j = ptr[k]; j < ptr[k + 1]; ++j) {
    const int i = ent[j] / NW, m = ent[j] % NW;
    double w = W[5 * wsel[i * DIM] + m % 5] * W[5 * wsel[i * DIM + 1] + (m / 5) % 5];
    if (DIM == 3) w *= W[5 * wsel[i * DIM + 2] + m / 25];
    acc += w * mu[i];
  }
  r[elem[k]] -= acc;
}

// adjoint of the average-down: rf[child] += scale * rc[parent] (scale =
// 1 / ratio^DIM)
__global__ void __launch_bounds__(256) k_pass_down(int n, const ProlD* __restrict__ p, const double* __restrict__ rc,
                                                   double* __restrict__ rf, double scale) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const ProlD q = p[i];
  rf[q.fe] += scale * rc[q.pe];
}

// r -= a on the interior (cells of the tiles)
template <int DIM>
__global__ void __launch_bounds__(256) k_sub_array(const TileD* __restrict__ tiles, int ntiles,
                                                   const BoxD* __restrict__ boxes, const double* __restrict__ a,
                                                   double* __restrict__ r) {
  FOR_COLUMN(DIM) {
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    r[c] -= a[c];
    if (C.ok1) r[c + 1] -= a[c + 1];
  }
}

// fill-band transpose for the composite adjoint: like k_band (residual mode,
// scale -1) with the ghost adjoints beta * (stencil weights) plus what
// refluxing put in the ghost slots (ab)
template <int DIM>
__global__ void __launch_bounds__(256) k_band_ab(const BandChunkD* __restrict__ chunks, int nchunks,
                                                 const BoxD* __restrict__ boxes, const uint8_t* __restrict__ codes,
                                                 const double* __restrict__ u, const double* __restrict__ ab,
                                                 double* __restrict__ out, double beta) {
  const int ci = blockIdx.x;
  if (ci >= nchunks) return;
  const BandChunkD ch = chunks[ci];
  if ((int)threadIdx.x >= ch.count) return;
  const BoxD b = boxes[ch.box];
  const int k = ch.start + (int)threadIdx.x;
  const int d = ch.face >> 1, s = ch.face & 1;
  int x[3] = {0, 0, 0};
  if (d == 0) {
    const int p = k & 3, r = k >> 2;
    x[0] = s ? b.n[0] - 1 - p : p;
    x[1] = r % b.n[1];
    x[2] = r / b.n[1];
  } else if (d == 1) {
    const int r = k / b.n[0], p = r & 3;
    x[0] = k % b.n[0];
    x[1] = s ? b.n[1] - 1 - p : p;
    x[2] = r >> 2;
  } else {
    const int r = k / b.n[0], p = r / b.n[1];
    x[0] = k % b.n[0];
    x[1] = r % b.n[1];
    x[2] = s ? b.n[2] - 1 - p : p;
  }
  for (int f = 0; f < ch.face; ++f) {
    if (!((ch.fmask >> f) & 1)) continue;
    const int e = f >> 1;
    if (((f & 1) ? b.n[e] - 1 - x[e] : x[e]) < 4) return;
  }
  double delta = 0.0;
#pragma unroll
  for (int f = 0; f < 2 * DIM; ++f) {
    if (!((ch.fmask >> f) & 1)) continue;
    const int e = f >> 1, sd = f & 1;
    const int dist = sd ? b.n[e] - 1 - x[e] : x[e];
    if (dist >= 4) continue;
    int colx;
    if (DIM == 2)
      colx = e == 0 ? x[1] : x[0];
    else
      colx = e == 0 ? x[1] + b.n[1] * x[2] : (e == 1 ? x[0] + b.n[0] * x[2] : x[0] + b.n[0] * x[1]);
    const uint8_t cd = codes[b.code_off[e][sd] + colx];
    const int kind = cd & 3;
    if (!kind) continue;
    int y[3] = {x[0], x[1], x[2]};
    y[e] = sd ? b.n[e] - 1 : 0;
    const int64_t e0 = cell_index<DIM>(b, y[0], y[1], y[2]);
    const int64_t in = (e == 0 ? 1 : (int64_t)b.s[e]) * (sd ? -1 : 1);
    const double l0 = u[e0], l1 = u[e0 + in];
    delta += kFillW[kind - 1][0][dist] * (beta * (16.0 * l0 - l1) + ab[e0 - in]);
    if (cd & 4) delta += kFillW[kind - 1][1][dist] * (-beta * l0 + ab[e0 - 2 * in]);
  }
  out[cell_index<DIM>(b, x[0], x[1], x[2])] -= delta;
}



// out = max over n slots
__global__ void k_max_slots(const double* __restrict__ in, int n, double* __restrict__ out) {
  double m = 0.0;
  for (int i = 0; i < n; ++i) m = fmax(m, in[i]);
  for (int i = 0; i < n; ++i)
    if (!(in[i] <= 1e308)) m = in[i];  // NaN / Inf propagate
  *out = m;
}

// a -= s[0] on every interior cell
template <int DIM>
__global__ void __launch_bounds__(256) k_sub_scalar(const TileD* __restrict__ tiles, int ntiles,
                                                    const BoxD* __restrict__ boxes, double* __restrict__ a,
                                                    const double* __restrict__ s) {
  const double v = s[0];
  FOR_COLUMN(DIM) {
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    a[c] -= v;
    if (C.ok1) a[c + 1] -= v;
  }
}

// x += s e and E += s e (FP64 x and E, e FP32 or FP64), s = scal[0]
template <typename T, int DIM>
__global__ void __launch_bounds__(256) k_update2(const TileD* __restrict__ tiles, int ntiles,
                                                 const BoxD* __restrict__ boxes, double* __restrict__ x,
                                                 double* __restrict__ E, const T* __restrict__ e,
                                                 const double* __restrict__ scal) {
  const double s = scal[0];
  FOR_COLUMN(DIM) {
    const int64_t c = C.base + (int64_t)(p + 2) * C.sm;
    const double v0 = s * (double)e[c];
    x[c] += v0;
    E[c] += v0;
    if (C.ok1) {
      const double v1 = s * (double)e[c + 1];
      x[c + 1] += v1;
      E[c + 1] += v1;
    }
  }
}

// ===========================================================================
// host-side launchers
namespace {
inline dim3 grid8(size_t n) { return dim3((unsigned)(8 * ((n + 7) / 8))); }
template <int DIM>
inline dim3 threads() {
  return dim3(block_threads<DIM>());
}
}  // namespace

#define DISPATCH_DIM(dim, KERNEL, ...)                                                   \
  do {                                                                                   \
    if ((dim) == 2)                                                                      \
      hipLaunchKernelGGL(KERNEL<2>, grid8(n), threads<2>(), 0, st, __VA_ARGS__);         \
    else                                                                                 \
      hipLaunchKernelGGL(KERNEL<3>, grid8(n), threads<3>(), 0, st, __VA_ARGS__);         \
  } while (0)

template <typename T>
void launch_fill(const Depth& D, T* u, const double* fd, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL((k_fill<T, 0>), dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, u, fd, D.h);
}

template <typename T>
void launch_fill_tr(const Depth& D, T* u, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL((k_fill<T, 1>), dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, u, nullptr, D.h);
}

template <typename T>
void launch_fill_zero(const Depth& D, T* u, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL((k_fill<T, 2>), dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, u, nullptr, D.h);
}

template <typename T>
void launch_band(int dim, const Depth& D, int mode, const T* u, T* out, T alpha, T beta, T scale, int col,
                 hipStream_t st) {
  const int n = (int)D.band.size();
  if (!n) return;
#define BAND_(DIM_, MODE_)                                                                                        \
  hipLaunchKernelGGL((k_band<T, DIM_, MODE_>), dim3(n), dim3(256), 0, st, D.d_band, n, D.d_box, D.d_codes, u, out, \
                     alpha, beta, scale, col)
  if (dim == 2) {
    if (mode == 0) {
      BAND_(2, 0);
    } else if (mode == 1) {
      BAND_(2, 1);
    } else {
      BAND_(2, 2);
    }
  } else {
    if (mode == 0) {
      BAND_(3, 0);
    } else if (mode == 1) {
      BAND_(3, 1);
    } else {
      BAND_(3, 2);
    }
  }
#undef BAND_
}

void launch_grad(int dim, const Depth& D, const double* u, DPtrs g, CPtrs w, bool sub, hipStream_t st,
                 double scale) {
  const size_t n = D.tiles.size();
  if (!n) return;
  DISPATCH_DIM(dim, k_grad, D.d_tiles, (int)n, D.d_box, u, g, w, sub, scale / (12.0 * D.h));
}

void launch_div(int dim, const Depth& D, CPtrs w, double* out, hipStream_t st, double scale) {
  const size_t n = D.tiles.size();
  if (!n) return;
  DISPATCH_DIM(dim, k_div, D.d_tiles, (int)n, D.d_box, w, out, scale / (12.0 * D.h));
}

void launch_cic(int dim, const CicTable& T, const double* const* hist, const double tv[4], const double td[4], int kind,
                double h, double* fd, double* dfd, hipStream_t st) {
  const int n = (int)T.fd.size();
  if (!n) return;
  CoarseHist ch;
  TimeW tw;
  for (int i = 0; i < 4; ++i) {
    ch.p[i] = hist[i];
    tw.v[i] = tv[i];
    tw.d[i] = td[i];
  }
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (dim == 2)
    hipLaunchKernelGGL(k_cic<2>, g, b, 0, st, n, T.d_fd, T.d_src, T.d_wsel, T.d_w, ch, tw, kind, 1.0 / (12.0 * h), fd,
                       dfd);
  else
    hipLaunchKernelGGL(k_cic<3>, g, b, 0, st, n, T.d_fd, T.d_src, T.d_wsel, T.d_w, ch, tw, kind, 1.0 / (12.0 * h), fd,
                       dfd);
}

void launch_cic_correct(const Depth& D, int ncomp, const CicTable& T, DPtrs fdv, hipStream_t st) {
  if (D.chunks.empty() || ncomp <= 0) return;
  hipLaunchKernelGGL(k_cic_sum, dim3(ncomp), dim3(256), 0, st, D.d_chunks, D.d_cc_ptr, D.d_cc_idx, fdv, T.d_ncf,
                     T.d_sum);
  const int n = (int)D.chunks.size();
  hipLaunchKernelGGL(k_cic_fix, dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, D.d_box, fdv, T.d_sum);
}

void launch_gslot(const Depth& D, CPtrs mu, int dir, double* ab, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL(k_gslot, dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, mu, dir, ab, 1.0 / (12.0 * D.h));
}

void launch_rfxV_T(const Composite& X, int d, const double* lam_c, double lscale, double* abc, double* abf,
                   hipStream_t st) {
  const Composite::GatherT* t[2] = {&X.rfxVc[d], &X.rfxVf[d]};
  double* out[2] = {abc, abf};
  for (int k = 0; k < 2; ++k) {
    const int n = (int)t[k]->elem.size();
    if (n)
      hipLaunchKernelGGL(k_rfx_T, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, t[k]->d_elem, t[k]->d_ptr,
                         t[k]->d_src, t[k]->d_coef, X.d_rfx_cell, lam_c, lscale, out[k]);
  }
}

void launch_reflux_div(int dim, const Composite& X, CPtrs wc, CPtrs wf, double* div, double hc, hipStream_t st) {
  const int n = (int)X.rfx_cell.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL(k_reflux_div<2>, dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_rfx_cell, X.d_rfx_ptr,
                       X.d_rfx_face, wc, wf, div, 1.0 / hc, X.r);
  else
    hipLaunchKernelGGL(k_reflux_div<3>, dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_rfx_cell, X.d_rfx_ptr,
                       X.d_rfx_face, wc, wf, div, 1.0 / hc, X.r);
}

void launch_tile_dot(int dim, const Depth& D, const double* a, const double* b, double* part, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  DISPATCH_DIM(dim, k_tile_dot, D.d_tiles, (int)n, D.d_box, a, b, part);
}

// FP32 sweeps run one cell per thread (k_march1), FP64 sweeps two (k_march):
// the faster of the two forms measured for each precision on gfx950.
template <typename T, int OP, bool PART>
struct MarchK {
  template <int DIM>
  static void go(const TileD* tl, size_t n, const Depth& D, const T* u, const T* f, T* out, T a, T b, T w, int col,
                 double* part, const BoxD* cboxes, hipStream_t st, int gr) {
    if (sizeof(T) == 4 && OP != OP_RESTRICT) {
      // the form that reads wrapped ghosts only where a box wraps
      // the forms that read wrapped ghosts, or form exchange and zero
      // ghosts, only where a box wraps or such columns exist
      const dim3 g = grid8(n), bs(DIM == 2 ? 128 : 512);
      const bool wr = gr && D.wrap, xf = gr && D.xfill;
      if (wr && xf)
        hipLaunchKernelGGL((k_march1<T, DIM, OP, PART, true, true>), g, bs, 0, st, tl, (int)n, D.d_box, D.d_codes, u,
                           f, out, a, b, w, col, part, gr, D.d_xsrc);
      else if (wr)
        hipLaunchKernelGGL((k_march1<T, DIM, OP, PART, true, false>), g, bs, 0, st, tl, (int)n, D.d_box, D.d_codes,
                           u, f, out, a, b, w, col, part, gr, D.d_xsrc);
      else if (xf)
        hipLaunchKernelGGL((k_march1<T, DIM, OP, PART, false, true>), g, bs, 0, st, tl, (int)n, D.d_box, D.d_codes,
                           u, f, out, a, b, w, col, part, gr, D.d_xsrc);
      else
        hipLaunchKernelGGL((k_march1<T, DIM, OP, PART, false, false>), g, bs, 0, st, tl, (int)n, D.d_box, D.d_codes,
                           u, f, out, a, b, w, col, part, gr, D.d_xsrc);
    } else if (gr && D.wrap) {  // the form that reads wrapped ghosts only where a box wraps
      hipLaunchKernelGGL((k_march<T, DIM, OP, PART, T, true>), grid8(n), threads<DIM>(), 0, st, tl, (int)n, D.d_box,
                         D.d_codes, u, f, out, a, b, w, col, part, cboxes, gr, (int64_t)0);
    } else {
      hipLaunchKernelGGL((k_march<T, DIM, OP, PART>), grid8(n), threads<DIM>(), 0, st, tl, (int)n, D.d_box, D.d_codes,
                         u, f, out, a, b, w, col, part, cboxes, gr, (int64_t)0);
    }
  }
};

template <typename T, int OP, bool PART>
void march(int dim, const TileD* tl, size_t n, const Depth& D, const T* u, const T* f, T* out, T a, T b, T w, int col,
           double* part, hipStream_t st, const BoxD* cboxes = nullptr, int gr = 0) {
  if (!n) return;
  if (dim == 2)
    MarchK<T, OP, PART>::template go<2>(tl, n, D, u, f, out, a, b, w, col, part, cboxes, st, gr);
  else
    MarchK<T, OP, PART>::template go<3>(tl, n, D, u, f, out, a, b, w, col, part, cboxes, st, gr);
}

template <typename T>
void launch_residual(int dim, const Depth& D, bool all, const T* u, const T* f, T* r, T alpha, T beta,
                     double* part, hipStream_t st) {
  const TileD* tl = all ? D.d_tiles : D.d_stiles;
  const size_t n = all ? D.tiles.size() : D.stiles.size();
  if (part)
    march<T, OP_RESID, true>(dim, tl, n, D, u, f, r, alpha, beta, T(0), 0, part, st);
  else
    march<T, OP_RESID, false>(dim, tl, n, D, u, f, r, alpha, beta, T(0), 0, nullptr, st);
}

template <typename T>
void launch_jacobi(int dim, const Depth& D, const T* u, const T* f, T* out, T alpha, T beta, T omega, bool zero,
                   hipStream_t st, int gr) {
  const size_t n = D.stiles.size();
  if (!n) return;
  if (zero) {
    if (dim == 2)
      hipLaunchKernelGGL((k_sweep0<T, 2, false>), grid8(n), threads<2>(), 0, st, D.d_stiles, (int)n, D.d_box, D.d_codes,
                         f, out, alpha, beta, omega);
    else
      hipLaunchKernelGGL((k_sweep0<T, 3, false>), grid8(n), threads<3>(), 0, st, D.d_stiles, (int)n, D.d_box, D.d_codes,
                         f, out, alpha, beta, omega);
    return;
  }
  march<T, OP_JACOBI, false>(dim, D.d_stiles, n, D, u, f, out, alpha, beta, omega, 0, nullptr, st, nullptr, gr);
}

template <typename T>
void launch_rb(int dim, const Depth& D, const T* u, const T* f, T* out, T alpha, T beta, T omega, int col, bool zero,
               hipStream_t st, int gr) {
  const size_t n = D.stiles.size();
  if (!n) return;
  if (zero) {
    if (dim == 2)
      hipLaunchKernelGGL((k_sweep0<T, 2, true>), grid8(n), threads<2>(), 0, st, D.d_stiles, (int)n, D.d_box, D.d_codes,
                         f, out, alpha, beta, omega);
    else
      hipLaunchKernelGGL((k_sweep0<T, 3, true>), grid8(n), threads<3>(), 0, st, D.d_stiles, (int)n, D.d_box, D.d_codes,
                         f, out, alpha, beta, omega);
    return;
  }
  march<T, OP_RB, false>(dim, D.d_stiles, n, D, u, f, out, alpha, beta, omega, col, nullptr, st, nullptr, gr);
}

template <typename T>
void launch_resid_restrict(int dim, const Depth& F, const Depth& C, const T* u, const T* f, T* fc, T alpha, T beta,
                           hipStream_t st, int gr) {
  // marched over the fine tiles of the boxes that continue to depth+1
  march<T, OP_RESTRICT, false>(dim, F.d_stiles, F.stiles.size(), F, u, f, fc, alpha, beta, T(0), 0, nullptr, st,
                               C.d_box, gr);
}

template <typename T>
void launch_restrict(int dim, const Depth& F, const Depth& C, const T* r, T* fc, hipStream_t st) {
  const size_t n = C.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_restrict<T, 2>), grid8(n), threads<2>(), 0, st, C.d_tiles, (int)n, C.d_box, F.d_box, r, fc);
  else
    hipLaunchKernelGGL((k_restrict<T, 3>), grid8(n), threads<3>(), 0, st, C.d_tiles, (int)n, C.d_box, F.d_box, r, fc);
}

template <typename T>
void launch_prolong(int dim, const Depth& F, const Depth& C, const T* ec, T* u, hipStream_t st, int gr) {
  const size_t n = F.stiles.size();
  if (!n) return;
  // the wrapped form only where a coarse box wraps onto itself
  if (gr && C.wrap) {
    if (dim == 2)
      hipLaunchKernelGGL((k_prolong<T, 2, true>), grid8(n), threads<2>(), 0, st, F.d_stiles, (int)n, F.d_box, C.d_box,
                         ec, u, gr);
    else
      hipLaunchKernelGGL((k_prolong<T, 3, true>), grid8(n), threads<3>(), 0, st, F.d_stiles, (int)n, F.d_box, C.d_box,
                         ec, u, gr);
    return;
  }
  if (dim == 2)
    hipLaunchKernelGGL((k_prolong<T, 2>), grid8(n), threads<2>(), 0, st, F.d_stiles, (int)n, F.d_box, C.d_box, ec, u,
                       gr);
  else
    hipLaunchKernelGGL((k_prolong<T, 3>), grid8(n), threads<3>(), 0, st, F.d_stiles, (int)n, F.d_box, C.d_box, ec, u,
                       gr);
}

template <typename T>
void launch_bottom(const Depth& D, const double* mats, const int64_t* idx, const T* f, T* e, bool tr,
                   hipStream_t st, T* e2) {
  if (D.groups.empty()) return;
  int maxn = 0;
  for (auto& g : D.groups) maxn = std::max(maxn, g.n);
  const dim3 grid((maxn + 7) / 8, (unsigned)D.groups.size());
  if (tr)
    hipLaunchKernelGGL((k_bottom<T, true>), grid, dim3(256), 0, st, D.d_groups, mats, idx, f, e, e2);
  else
    hipLaunchKernelGGL((k_bottom<T, false>), grid, dim3(256), 0, st, D.d_groups, mats, idx, f, e, e2);
}

template <typename T>
void launch_tile_sum(int dim, const Depth& D, const T* a, double* part, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_tile_reduce<T, 2, false>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n, D.d_box, a, part);
  else
    hipLaunchKernelGGL((k_tile_reduce<T, 3, false>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n, D.d_box, a, part);
}

template <typename T>
void launch_tile_absmax(int dim, const Depth& D, const T* a, double* part, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_tile_reduce<T, 2, true>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n, D.d_box, a, part);
  else
    hipLaunchKernelGGL((k_tile_reduce<T, 3, true>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n, D.d_box, a, part);
}

void launch_seg_reduce(const double* in, const int32_t* ptr, int nseg, int n, double* out, bool is_max,
                       hipStream_t st, double* host) {
  if (nseg <= 0) return;
  if (is_max)
    hipLaunchKernelGGL(k_seg_reduce<true>, dim3(nseg), dim3(256), 0, st, in, ptr, n, out, host);
  else
    hipLaunchKernelGGL(k_seg_reduce<false>, dim3(nseg), dim3(256), 0, st, in, ptr, n, out, host);
}

void launch_comp_mean_delta(const Depth& D, const double* part, const int32_t* flag, const double* cnt, int ncomp,
                            double* delta, hipStream_t st) {
  if (ncomp <= 0) return;
  hipLaunchKernelGGL(k_comp_mean_delta, dim3(ncomp), dim3(256), 0, st, part, D.d_seg, D.d_cseg, flag, cnt, delta);
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
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_comp_shift<T, 2>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n, D.d_box, a, delta);
  else
    hipLaunchKernelGGL((k_comp_shift<T, 3>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n, D.d_box, a, delta);
}

template <typename T>
void launch_comp_mean_shift(int dim, const Depth& D, const double* part, const int32_t* flag, const double* cnt, T* a,
                            hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_comp_mean_shift<T, 2>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n, D.d_box, part,
                       D.d_seg, D.d_cseg, flag, cnt, a);
  else
    hipLaunchKernelGGL((k_comp_mean_shift<T, 3>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n, D.d_box, part,
                       D.d_seg, D.d_cseg, flag, cnt, a);
}
template void launch_comp_mean_shift<float>(int, const Depth&, const double*, const int32_t*, const double*, float*,
                                            hipStream_t);
template void launch_comp_mean_shift<double>(int, const Depth&, const double*, const int32_t*, const double*, double*,
                                             hipStream_t);

template <typename T>
void launch_comp_mean_small(int dim, const Depth& D, int ncomp, const int32_t* flag, const double* cnt, T* a,
                            hipStream_t st) {
  if (D.tiles.empty() || ncomp <= 0) return;
  const int nb = (int)D.boxes.size();
  if (dim == 2)
    hipLaunchKernelGGL((k_comp_mean_small<T, 2>), dim3(ncomp), dim3(1024), 0, st, nb, D.d_box, flag, cnt, a);
  else
    hipLaunchKernelGGL((k_comp_mean_small<T, 3>), dim3(ncomp), dim3(1024), 0, st, nb, D.d_box, flag, cnt, a);
}
template void launch_comp_mean_small<float>(int, const Depth&, int, const int32_t*, const double*, float*, hipStream_t);
template void launch_comp_mean_small<double>(int, const Depth&, int, const int32_t*, const double*, double*,
                                             hipStream_t);

void launch_cf_delta(const double* defect, const int32_t* flag, const double* ncf, const double* cnt, int ncomp,
                     double hD, double hD1, double* delta, double* dfd, hipStream_t st) {
  hipLaunchKernelGGL(k_cf_delta, dim3((ncomp + 255) / 256), dim3(256), 0, st, defect, flag, ncf, cnt, ncomp, hD, hD1,
                     delta, dfd);
}

void launch_fd_correct(const Depth& D, const double* fd, const double* dfd, double* out, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL(k_fd_correct, dim3((n + 3) / 4), dim3(256), 0, st, D.d_chunks, n, D.d_box, fd, dfd, out);
}

void launch_chunk_fdsum(const Depth& D, const double* fd, const uint8_t* valid, double* part, hipStream_t st) {
  const int n = (int)D.chunks.size();
  if (!n) return;
  hipLaunchKernelGGL(k_chunk_fdsum, dim3((n + 255) / 256), dim3(256), 0, st, D.d_chunks, n, fd, valid, part);
}

void launch_cfi(int dim, const Composite& X, const double* uc, double* uf, hipStream_t st) {
  const int n = (int)X.cfi_dst.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_cfi<double, 2>), dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_cfi_dst, X.d_cfi_src,
                       X.d_cfi_w, X.d_w, uc, uf);
  else
    hipLaunchKernelGGL((k_cfi<double, 3>), dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_cfi_dst, X.d_cfi_src,
                       X.d_cfi_w, X.d_w, uc, uf);
}

void launch_avgdown(int dim, const Composite& X, const double* uf, double* uc, hipStream_t st) {
  const int n = (int)X.avg.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_avgdown<double, 2>), dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_avg, uf, uc, X.r);
  else
    hipLaunchKernelGGL((k_avgdown<double, 3>), dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_avg, uf, uc, X.r);
}

void launch_reflux(int dim, const Composite& X, const double* uc, const double* uf, double* r, double kappa,
                   double hc, double hf, hipStream_t st) {
  const int n = (int)X.rfx_cell.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL(k_reflux<2>, dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_rfx_cell, X.d_rfx_ptr,
                       X.d_rfx_face, uc, uf, r, kappa, 1.0 / (12 * hc), 1.0 / (12 * hf), 1.0 / hc, X.r);
  else
    hipLaunchKernelGGL(k_reflux<3>, dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_rfx_cell, X.d_rfx_ptr,
                       X.d_rfx_face, uc, uf, r, kappa, 1.0 / (12 * hc), 1.0 / (12 * hf), 1.0 / hc, X.r);
}

void launch_amr_prolong(int dim, const Composite& X, const double* ec, double* u, double* ef, hipStream_t st,
                        double scale) {
  const int n = (int)X.pro.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_amr_prolong<double, 2>), dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_pro, ec, u, ef,
                       scale, X.r);
  else
    hipLaunchKernelGGL((k_amr_prolong<double, 3>), dim3((n + 255) / 256), dim3(256), 0, st, n, X.d_pro, ec, u, ef,
                       scale, X.r);
}

#define GRID1(n) dim3((unsigned)(((n) + 255) / 256)), dim3(256)
void launch_zero_covered(const Composite& X, double* u, hipStream_t st) {
  const int n = (int)X.avg.size();
  if (n) hipLaunchKernelGGL(k_zero_covered, GRID1(n), 0, st, n, X.d_avg, u);
}
void launch_sumdown(int dim, const Composite& X, const double* uf, double* uc, double scale, hipStream_t st) {
  const int n = (int)X.avg.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL(k_sumdown<2>, GRID1(n), 0, st, n, X.d_avg, uf, uc, scale, X.r);
  else
    hipLaunchKernelGGL(k_sumdown<3>, GRID1(n), 0, st, n, X.d_avg, uf, uc, scale, X.r);
}
void launch_rfx_T(const Composite& X, const double* lam_c, double lscale, double* abc, double* abf, hipStream_t st) {
  int n = (int)X.rfxTc_elem.size();
  if (n)
    hipLaunchKernelGGL(k_rfx_T, GRID1(n), 0, st, n, X.d_rfxTc_elem, X.d_rfxTc_ptr, X.d_rfxTc_src, X.d_rfxTc_coef,
                       X.d_rfx_cell, lam_c, lscale, abc);
  n = (int)X.rfxTf_elem.size();
  if (n)
    hipLaunchKernelGGL(k_rfx_T, GRID1(n), 0, st, n, X.d_rfxTf_elem, X.d_rfxTf_ptr, X.d_rfxTf_src, X.d_rfxTf_coef,
                       X.d_rfx_cell, lam_c, lscale, abf);
}
void launch_exch_T(const Depth& D, const double* ab, double* r, hipStream_t st) {
  const int n = (int)D.exT_elem.size();
  if (n) hipLaunchKernelGGL(k_exch_T, GRID1(n), 0, st, n, D.d_exT_elem, D.d_exT_ptr, D.d_exT_slot, ab, r);
}
void launch_cfi_T(int dim, const Composite& X, const double* lam_f, const double* abf, double beta, double* mu,
                  double* rc, hipStream_t st) {
  const int n = (int)X.cfi_dst.size();
  if (!n) return;
  hipLaunchKernelGGL(k_cfi_mu, GRID1(n), 0, st, n, X.d_cfi_e0, X.d_cfi_in, X.d_cfi_layer, X.d_cfi_dst, lam_f, abf,
                     beta, mu);
  const int m = (int)X.cfiT_elem.size();
  if (!m) return;
  if (dim == 2)
    hipLaunchKernelGGL(k_cfi_T<2>, GRID1(m), 0, st, m, X.d_cfiT_elem, X.d_cfiT_ptr, X.d_cfiT_ent, X.d_cfi_w, X.d_w,
                       mu, rc);
  else
    hipLaunchKernelGGL(k_cfi_T<3>, GRID1(m), 0, st, m, X.d_cfiT_elem, X.d_cfiT_ptr, X.d_cfiT_ent, X.d_cfi_w, X.d_w,
                       mu, rc);
}
void launch_pass_down(const Composite& X, const double* rc, double* rf, double scale, hipStream_t st) {
  const int n = (int)X.pro.size();
  if (n) hipLaunchKernelGGL(k_pass_down, GRID1(n), 0, st, n, X.d_pro, rc, rf, scale);
}
void launch_sub_array(int dim, const Depth& D, const double* a, double* r, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  DISPATCH_DIM(dim, k_sub_array, D.d_tiles, (int)n, D.d_box, a, r);
}
void launch_band_ab(int dim, const Depth& D, const double* u, const double* ab, double* out, double beta,
                    hipStream_t st) {
  const int n = (int)D.band.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL(k_band_ab<2>, dim3(n), dim3(256), 0, st, D.d_band, n, D.d_box, D.d_codes, u, ab, out, beta);
  else
    hipLaunchKernelGGL(k_band_ab<3>, dim3(n), dim3(256), 0, st, D.d_band, n, D.d_box, D.d_codes, u, ab, out, beta);
}
#undef GRID1

void launch_max_slots(const double* in, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_max_slots, dim3(1), dim3(1), 0, st, in, n, out);
}

void launch_sub_scalar(int dim, const Depth& D, double* a, const double* s, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  DISPATCH_DIM(dim, k_sub_scalar, D.d_tiles, (int)n, D.d_box, a, s);
}

template <typename T>
void launch_update2(int dim, const Depth& D, double* x, double* E, const T* e, const double* scal, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_update2<T, 2>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n, D.d_box, x, E, e, scal);
  else
    hipLaunchKernelGGL((k_update2<T, 3>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n, D.d_box, x, E, e, scal);
}
template void launch_update2<float>(int, const Depth&, double*, double*, const float*, const double*, hipStream_t);
template void launch_update2<double>(int, const Depth&, double*, double*, const double*, const double*, hipStream_t);

template <typename T>
void launch_update(int dim, const Depth& D, double* x, const T* e, const double* scal, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  if (dim == 2)
    hipLaunchKernelGGL((k_update<T, 2>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n, D.d_box, x, e, scal);
  else
    hipLaunchKernelGGL((k_update<T, 3>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n, D.d_box, x, e, scal);
}

void launch_to32(int dim, const Depth& D, const double* r, float* r32, const double* scal, hipStream_t st,
                 const double* delta, float* fs) {
  const size_t n = D.tiles.size();
  if (!n) return;
  float* fs1 = fs ? fs + D.nstored / 2 : nullptr;
  DISPATCH_DIM(dim, k_to32, D.d_tiles, (int)n, D.d_box, r, r32, scal, delta, fs, fs1);
}

void launch_scale32(int dim, const Depth& D, float* r32, const double* scal, hipStream_t st, const double* delta,
                    float* fs) {
  const size_t n = D.tiles.size();
  if (!n) return;
  float* fs1 = fs ? fs + D.nstored / 2 : nullptr;
  DISPATCH_DIM(dim, k_scale32, D.d_tiles, (int)n, D.d_box, r32, scal, delta, fs, fs1);
}

template <int DIM>
void launch_rbs_d(const Depth& D, int mode, const float* h0, const float* h1, const float* fc, float* out,
                  float alpha, float beta, float omega, int col, hipStream_t st, const double* scal,
                  const double* delta, double* xu, const double* su) {
  const size_t n = D.stiles.size();
  const dim3 bs(DIM == 3 ? 256 : 64);
#define RBS_LAUNCH(MD)                                                                                         \
  hipLaunchKernelGGL((k_rbs<DIM, MD>), grid8(n), bs, 0, st, D.d_stiles, (int)n, D.d_box, h0, h1, fc, out, alpha, \
                     beta, omega, col, D.xg32, scal, delta, xu, su)
  if (mode == 0)
    RBS_LAUNCH(0);
  else if (mode == 1)
    RBS_LAUNCH(1);
  else if (mode == 2)
    RBS_LAUNCH(2);
  else
    RBS_LAUNCH(3);
#undef RBS_LAUNCH
}

void launch_rbs(int dim, const Depth& D, int mode, const float* h0, const float* h1, const float* fc, float* out,
                float alpha, float beta, float omega, int col, hipStream_t st, const double* scal,
                const double* delta, double* xu, const double* su) {
  if (D.stiles.empty()) return;
  if (dim == 2)
    launch_rbs_d<2>(D, mode, h0, h1, fc, out, alpha, beta, omega, col, st, scal, delta, xu, su);
  else
    launch_rbs_d<3>(D, mode, h0, h1, fc, out, alpha, beta, omega, col, st, scal, delta, xu, su);
}

void launch_resid_restrict_s(int dim, const Depth& F, const Depth& C, const float* u, const float* f, float* fc,
                             float alpha, float beta, hipStream_t st, const double* scal, const double* delta) {
  const size_t n = F.stiles.size();
  if (!n) return;
  const int64_t hs = F.nstored / 2;
  if (dim == 2)
    hipLaunchKernelGGL(k_resid_restrict_s<2>, grid8(n), threads<2>(), 0, st, F.d_stiles, (int)n, F.d_box, u, u + hs,
                       f, f + hs, fc, alpha, beta, C.d_box, F.xg32, scal, delta);
  else
    hipLaunchKernelGGL(k_resid_restrict_s<3>, grid8(n), threads<3>(), 0, st, F.d_stiles, (int)n, F.d_box, u, u + hs,
                       f, f + hs, fc, alpha, beta, C.d_box, F.xg32, scal, delta);
}

void launch_prolong_s(int dim, const Depth& F, const Depth& C, const float* ec, const float* u, float* out,
                      hipStream_t st) {
  const size_t n = F.stiles.size();
  if (!n) return;
  const int64_t hs = F.nstored / 2;
  if (dim == 2)
    hipLaunchKernelGGL(k_prolong_s<2>, grid8(n), threads<2>(), 0, st, F.d_stiles, (int)n, F.d_box, C.d_box, ec, u,
                       u + hs, out, out + hs);
  else
    hipLaunchKernelGGL(k_prolong_s<3>, grid8(n), threads<3>(), 0, st, F.d_stiles, (int)n, F.d_box, C.d_box, ec, u,
                       u + hs, out, out + hs);
}

void launch_residual32(int dim, const Depth& D, const double* u, const double* f, float* r, double alpha, double beta,
                       double* part, hipStream_t st, bool split, int gr) {
  const size_t n = D.tiles.size();
  if (!n) return;
  const int64_t sh = split ? D.nstored / 2 : 0;
  if (gr && D.wrap) {  // the form that reads wrapped ghosts only where a box wraps
    if (dim == 2)
      hipLaunchKernelGGL((k_march<double, 2, OP_RESID, true, float, true>), grid8(n), threads<2>(), 0, st, D.d_tiles,
                         (int)n, D.d_box, D.d_codes, u, f, r, alpha, beta, 0.0, 0, part, nullptr, gr, sh);
    else
      hipLaunchKernelGGL((k_march<double, 3, OP_RESID, true, float, true>), grid8(n), threads<3>(), 0, st, D.d_tiles,
                         (int)n, D.d_box, D.d_codes, u, f, r, alpha, beta, 0.0, 0, part, nullptr, gr, sh);
  } else if (dim == 2) {
    hipLaunchKernelGGL((k_march<double, 2, OP_RESID, true, float>), grid8(n), threads<2>(), 0, st, D.d_tiles, (int)n,
                       D.d_box, D.d_codes, u, f, r, alpha, beta, 0.0, 0, part, nullptr, gr, sh);
  } else {
    hipLaunchKernelGGL((k_march<double, 3, OP_RESID, true, float>), grid8(n), threads<3>(), 0, st, D.d_tiles, (int)n,
                       D.d_box, D.d_codes, u, f, r, alpha, beta, 0.0, 0, part, nullptr, gr, sh);
  }
}

void launch_shift_copy(int dim, const Depth& D, const double* f, double* out, const double* delta, hipStream_t st) {
  const size_t n = D.tiles.size();
  if (!n) return;
  DISPATCH_DIM(dim, k_shift_copy, D.d_tiles, (int)n, D.d_box, f, out, delta);
}

void launch_set_scale(const double* src, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scale, dim3(1), dim3(1), 0, st, src, dst);
}
void launch_set_scaled(const double* src, double f, double* dst, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scaled, dim3(1), dim3(1), 0, st, src, f, dst);
}

template <typename T>
void launch_zero(T* a, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_zero<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, a, n);
}

#define INST(T)                                                                                                   \
  template void launch_fill<T>(const Depth&, T*, const double*, hipStream_t);                                     \
  template void launch_fill_tr<T>(const Depth&, T*, hipStream_t);                                                 \
  template void launch_fill_zero<T>(const Depth&, T*, hipStream_t);                                               \
  template void launch_band<T>(int, const Depth&, int, const T*, T*, T, T, T, int, hipStream_t);                  \
  template void launch_residual<T>(int, const Depth&, bool, const T*, const T*, T*, T, T, double*, hipStream_t);  \
  template void launch_jacobi<T>(int, const Depth&, const T*, const T*, T*, T, T, T, bool, hipStream_t, int);     \
  template void launch_rb<T>(int, const Depth&, const T*, const T*, T*, T, T, T, int, bool, hipStream_t, int);    \
  template void launch_resid_restrict<T>(int, const Depth&, const Depth&, const T*, const T*, T*, T, T,           \
                                         hipStream_t, int);                                                       \
  template void launch_restrict<T>(int, const Depth&, const Depth&, const T*, T*, hipStream_t);                   \
  template void launch_prolong<T>(int, const Depth&, const Depth&, const T*, T*, hipStream_t, int);               \
  template void launch_bottom<T>(const Depth&, const double*, const int64_t*, const T*, T*, bool, hipStream_t, T*); \
  template void launch_tile_sum<T>(int, const Depth&, const T*, double*, hipStream_t);                            \
  template void launch_tile_absmax<T>(int, const Depth&, const T*, double*, hipStream_t);                         \
  template void launch_comp_shift<T>(int, const Depth&, T*, const double*, hipStream_t);                          \
  template void launch_update<T>(int, const Depth&, double*, const T*, const double*, hipStream_t);               \
  template void launch_zero<T>(T*, int64_t, hipStream_t);
INST(double)
INST(float)

}  // namespace amg
