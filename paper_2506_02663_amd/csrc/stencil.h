// Device helpers shared by the kernels: the folded diagonal increment of a
// filled face, the homogeneous ghost fills of a row, the element of a cell
// of a box, and a fixed-order block sum.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "amg_internal.h"

namespace amg {

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

// First and second ghost of a filled column with code cd from the first four
// cells of its row (u0 at the face): eqs. (velBCHomoDiri5th) and (Neumann5)
// with zero data.
template <typename T>
__device__ __forceinline__ T ghost1(uint8_t cd, T u0, T u1, T u2, T u3) {
  return (cd & 3) == 1 ? (T(-77) * u0 + T(43) * u1 - T(17) * u2 + T(3) * u3) * T(1.0 / 12.0)
                       : (T(5) * u0 + T(9) * u1 - T(5) * u2 + u3) * T(0.1);
}
template <typename T>
__device__ __forceinline__ T ghost2(uint8_t cd, T u0, T u1, T u2, T u3) {
  return (cd & 3) == 1 ? (T(-505) * u0 + T(335) * u1 - T(145) * u2 + T(27) * u3) * T(1.0 / 12.0)
                       : (T(-75) * u0 + T(145) * u1 - T(75) * u2 + T(15) * u3) * T(0.1);
}

// element of cell (x, y, z) in box b (0-based interior indices)
template <int DIM>
__device__ __forceinline__ int64_t cell_index(const BoxD& b, int x, int y, int z) {
  return b.off + (x + 2) + (int64_t)(y + 2) * b.s[1] + (DIM == 3 ? (int64_t)(z + 2) * b.s[2] : 0);
}

// sum over the block of one value per thread, in a fixed order (wavefront
// butterflies, then the wavefronts in turn); the result is valid in thread 0
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

}  // namespace amg
