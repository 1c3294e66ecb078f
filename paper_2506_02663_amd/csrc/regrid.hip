// Device side of regridding (Section 5.4): the vorticity tags of RDM-1 and
// the data migration onto a new hierarchy.
//
// Tags: the composite gradient of every velocity component (eq. discreteOps
// a with the hierarchy's fills, as amg_gradient), then per cell of level l
// the vorticity (2D: G_x u_1 - G_y u_0; 3D: the norm of the curl) against
// the threshold, written into a dense byte array over the level's grid
// (x fastest; 0 off the level).
//
// Migration: level 0 is copied; every finer new level, in increasing order,
// takes on each cell the old level's value where the old level has that
// cell, else AMRCFI (the conservative tensor quartic over the child, window
// centred on the parent and shifted into the domain) from the new level
// below.  One thread per cell; cell -> box lookups through dense owner maps
// of the levels read.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "amg_internal.h"

using namespace amg;

namespace {

int fail(amg_hier* H, int code, const std::string& msg) {
  if (H) H->err = msg;
  return code;
}

struct GridD {
  int32_t n[3];  // cells of the level's grid
};

// element of the cell (gx, gy, gz) of box X (2D: no plane term)
template <int DIM>
__device__ __forceinline__ int64_t elem_of(const BoxD& X, int gx, int gy, int gz) {
  int64_t e = X.off + (int64_t)(gx - X.lo[0] + 2) + (int64_t)(gy - X.lo[1] + 2) * X.s[1];
  if (DIM == 3) e += (int64_t)(gz - X.lo[2] + 2) * X.s[2];
  return e;
}

template <int DIM>
__global__ __launch_bounds__(256) void k_tag_vort(BoxD X, GridD G, const double* __restrict__ g01,
                                                  const double* __restrict__ g10, const double* __restrict__ g02,
                                                  const double* __restrict__ g20, const double* __restrict__ g12,
                                                  const double* __restrict__ g21, double eps,
                                                  uint8_t* __restrict__ tags) {
  // gde = G_e u_d: g01 = G_1 u_0, g10 = G_0 u_1, ...
  const int64_t cells = (int64_t)X.n[0] * X.n[1] * X.n[2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells) return;
  const int x = (int)(i % X.n[0]), y = (int)((i / X.n[0]) % X.n[1]), z = (int)(i / ((int64_t)X.n[0] * X.n[1]));
  const int gx = X.lo[0] + x, gy = X.lo[1] + y, gz = X.lo[2] + z;
  const int64_t o = elem_of<DIM>(X, gx, gy, gz);
  double w;
  if (DIM == 2) {
    w = fabs(g10[o] - g01[o]);
  } else {
    const double cx = g21[o] - g12[o], cy = g02[o] - g20[o], cz = g10[o] - g01[o];
    w = sqrt(cx * cx + cy * cy + cz * cz);
  }
  tags[gx + (int64_t)G.n[0] * (gy + (int64_t)G.n[1] * gz)] = w >= eps ? 1 : 0;
}

struct Migr {
  BoxD X;              // the new box
  GridD Gc;            // grid of the new level below
  int r;
  const int32_t* own_c;   // owner map of the new level below (box index or -1)
  const BoxD* box_c;
  const double* uc;
  const int32_t* own_o;   // owner map of the old level (null: none)
  const BoxD* box_o;
  const double* uo;
  const double* W;        // AMRCFI weights [(shift + 2) * r + child][5]
  double* un;
  int* err;
};

__device__ __forceinline__ int window_shift(int P, int n) { return P < 2 ? 2 - P : (P > n - 3 ? (n - 3) - P : 0); }

template <int DIM>
__global__ __launch_bounds__(256) void k_migrate(Migr M) {
  const BoxD& X = M.X;
  const int64_t cells = (int64_t)X.n[0] * X.n[1] * X.n[2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells) return;
  const int x = (int)(i % X.n[0]), y = (int)((i / X.n[0]) % X.n[1]), z = (int)(i / ((int64_t)X.n[0] * X.n[1]));
  const int g[3] = {X.lo[0] + x, X.lo[1] + y, DIM == 3 ? X.lo[2] + z : 0};
  const int64_t dst = elem_of<DIM>(X, g[0], g[1], g[2]);
  const int r = M.r;
  if (M.own_o) {  // the old level has the cell: copy
    const int32_t ob = M.own_o[(int64_t)g[0] + (int64_t)M.Gc.n[0] * r * ((int64_t)g[1] + (int64_t)M.Gc.n[1] * r * g[2])];
    if (ob >= 0) {
      M.un[dst] = M.uo[elem_of<DIM>(M.box_o[ob], g[0], g[1], g[2])];
      return;
    }
  }
  if (!M.own_c) {  // level 0: the old level 0 lacks the cell
    *M.err = 1;
    M.un[dst] = 0.0;
    return;
  }
  int lo[3] = {0, 0, 0};
  const double* w[3] = {nullptr, nullptr, nullptr};
  for (int d = 0; d < DIM; ++d) {
    const int P = g[d] / r, a = g[d] % r;
    const int sh = window_shift(P, M.Gc.n[d]);
    lo[d] = P + sh - 2;
    w[d] = M.W + 5 * ((sh + 2) * r + a);
  }
  double acc = 0.0;
  bool bad = false;
  for (int k = 0; k < (DIM == 3 ? 5 : 1); ++k) {
    double plane = 0.0;
    for (int j = 0; j < 5; ++j) {
      double row = 0.0;
      for (int m = 0; m < 5; ++m) {
        const int q0 = lo[0] + m, q1 = lo[1] + j, q2 = DIM == 3 ? lo[2] + k : 0;
        const int32_t cb = M.own_c[(int64_t)q0 + (int64_t)M.Gc.n[0] * ((int64_t)q1 + (int64_t)M.Gc.n[1] * q2)];
        if (cb < 0) {
          bad = true;
          continue;
        }
        row += w[0][m] * M.uc[elem_of<DIM>(M.box_c[cb], q0, q1, q2)];
      }
      plane += w[1][j] * row;
    }
    acc += (DIM == 3 ? w[2][k] : 1.0) * plane;
  }
  if (bad) *M.err = 1;
  M.un[dst] = acc;
}

// dense owner map (box index, -1 elsewhere) of depth 0 of a level
std::vector<int32_t> owner_map(const amg_hier* H, const Level& L, int64_t n[3]) {
  std::vector<int32_t> own((size_t)(n[0] * n[1] * n[2]), -1);
  const Depth& D = L.depths[0];
  for (size_t b = 0; b < D.boxes.size(); ++b) {
    const Box& B = D.boxes[b];
    for (int z = B.lo[2]; z <= B.hi[2]; ++z)
      for (int y = B.lo[1]; y <= B.hi[1]; ++y)
        for (int x = B.lo[0]; x <= B.hi[0]; ++x) own[x + n[0] * (y + n[1] * (int64_t)z)] = (int32_t)b;
  }
  (void)H;
  return own;
}

void grid_of(const amg_hier* H, int l, int64_t n[3]) {
  for (int d = 0; d < 3; ++d) {
    n[d] = d < H->dim ? H->base[d] : 1;
    for (int i = 0; i < l && d < H->dim; ++i) n[d] *= H->ratio;
  }
}

template <typename T>
int dev_copy(amg_hier* H, T** dst, const std::vector<T>& v, hipStream_t st) {
  if (hipMalloc(dst, std::max<size_t>(v.size(), 1) * sizeof(T)) != hipSuccess)
    return fail(H, AMG_EDEVICE, "hipMalloc failed");
  if (!v.empty() && hipMemcpyAsync(*dst, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(H, AMG_EDEVICE, "copy of a regrid table failed");
  return AMG_OK;
}

}  // namespace

extern "C" int amg_tag_vorticity(amg_hier* h, int lev_hi, double* const* u, double eps, uint8_t* const* tags,
                                 void* stream) {
  amg_hier* H = h;
  if (!h || !h->finalized) return fail(H, AMG_EINVAL, "amg_finalize has not been called");
  if (lev_hi < 0 || lev_hi >= h->nlevels || !u || !tags || !(eps >= 0)) return fail(H, AMG_EINVAL, "bad arguments");
  const int D = h->dim;
  for (int l = 0; l <= lev_hi; ++l) {
    if (!tags[l]) return fail(H, AMG_EINVAL, "null tag array");
    for (int d = 0; d < D; ++d)
      if (!u[l * D + d]) return fail(H, AMG_EINVAL, "null velocity component");
  }
  hipStream_t st = stream ? (hipStream_t)stream : h->own;
  // gradients G_e u_d of every level: D * D level buffers per level
  int64_t need = 0;
  std::vector<int64_t> base(lev_hi + 1);
  for (int l = 0; l <= lev_hi; ++l) {
    base[l] = need;
    need += (int64_t)D * D * h->levels[l].depths[0].nstored;
  }
  if (h->regrid_len < need) {
    if (h->regrid_ws) (void)hipFree(h->regrid_ws);
    h->regrid_ws = nullptr;
    h->regrid_len = 0;
    if (hipMalloc(&h->regrid_ws, need * sizeof(double)) != hipSuccess) return fail(H, AMG_EDEVICE, "hipMalloc failed");
    h->regrid_len = need;
  }
  auto grad = [&](int l, int d, int e) {
    return h->regrid_ws + base[l] + (int64_t)(d * D + e) * h->levels[l].depths[0].nstored;
  };
  for (int d = 0; d < D; ++d) {
    std::vector<double*> phi(lev_hi + 1), g((size_t)(lev_hi + 1) * D);
    for (int l = 0; l <= lev_hi; ++l) {
      phi[l] = u[l * D + d];
      for (int e = 0; e < D; ++e) g[(size_t)l * D + e] = grad(l, d, e);
    }
    const int rc = amg_gradient(h, 0, lev_hi, phi.data(), nullptr, g.data(), st);
    if (rc) return rc;
  }
  for (int l = 0; l <= lev_hi; ++l) {
    int64_t n[3];
    grid_of(h, l, n);
    if (hipMemsetAsync(tags[l], 0, (size_t)(n[0] * n[1] * n[2]), st) != hipSuccess)
      return fail(H, AMG_EDEVICE, "clearing the tags failed");
    const GridD G = {{(int32_t)n[0], (int32_t)n[1], (int32_t)n[2]}};
    const Depth& D0 = h->levels[l].depths[0];
    for (const BoxD& X : D0.boxd) {
      const int64_t cells = (int64_t)X.n[0] * X.n[1] * X.n[2];
      const dim3 grid((unsigned)((cells + 255) / 256));
      if (D == 2)
        hipLaunchKernelGGL(k_tag_vort<2>, grid, dim3(256), 0, st, X, G, grad(l, 0, 1), grad(l, 1, 0), nullptr, nullptr,
                           nullptr, nullptr, eps, tags[l]);
      else
        hipLaunchKernelGGL(k_tag_vort<3>, grid, dim3(256), 0, st, X, G, grad(l, 0, 1), grad(l, 1, 0), grad(l, 0, 2),
                           grad(l, 2, 0), grad(l, 1, 2), grad(l, 2, 1), eps, tags[l]);
      if (hipGetLastError() != hipSuccess) return fail(H, AMG_EDEVICE, "k_tag_vort launch failed");
    }
  }
  return AMG_OK;
}

extern "C" int amg_migrate(amg_hier* hold, amg_hier* hnew, double* const* u_old, double* const* u_new,
                           void* stream) {
  amg_hier* H = hnew;
  if (!hold || !hnew || !hold->finalized || !hnew->finalized) return fail(H, AMG_EINVAL, "both hierarchies must be final");
  if (hold->dim != hnew->dim || hold->ratio != hnew->ratio || hold->h0 != hnew->h0)
    return fail(H, AMG_EINVAL, "the hierarchies differ in dimension, ratio or cell size");
  for (int d = 0; d < hnew->dim; ++d)
    if (hold->base[d] != hnew->base[d]) return fail(H, AMG_EINVAL, "the hierarchies differ in their grids");
  if (!u_old || !u_new) return fail(H, AMG_EINVAL, "null level arrays");
  for (int l = 0; l < hold->nlevels; ++l)
    if (!u_old[l]) return fail(H, AMG_EINVAL, "null old level array");
  for (int l = 0; l < hnew->nlevels; ++l)
    if (!u_new[l]) return fail(H, AMG_EINVAL, "null new level array");
  const int dim = hnew->dim, r = hnew->ratio;
  for (int d = 0; d < dim; ++d)  // a five-cell interpolation window must fit in every coarser grid
    if (hnew->base[d] < 5) return fail(H, AMG_EUNSUPPORTED, "migration needs at least 5 level-0 cells per direction");
  hipStream_t st = stream ? (hipStream_t)stream : hnew->own;
  double W[20][5];
  cfi_weight_table(W, r);
  std::vector<double> Wv(&W[0][0], &W[0][0] + 100);
  double* dW = nullptr;
  int* derr = nullptr;
  std::vector<void*> scratch;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(st);
    for (void* p : scratch) (void)hipFree(p);
  };
  int rc = dev_copy(H, &dW, Wv, st);
  if (rc) return rc;
  scratch.push_back(dW);
  if ((rc = dev_copy(H, &derr, std::vector<int>(1, 0), st))) {
    cleanup();
    return rc;
  }
  scratch.push_back(derr);
  for (int l = 0; l < hnew->nlevels; ++l) {
    const Level& Ln = hnew->levels[l];
    int64_t n[3];
    grid_of(hnew, l, n);
    // the old level's owner map (copy source) and the new level below's
    int32_t *own_o = nullptr, *own_c = nullptr;
    if (l < hold->nlevels) {
      if ((rc = dev_copy(H, &own_o, owner_map(hold, hold->levels[l], n), st))) {
        cleanup();
        return rc;
      }
      scratch.push_back(own_o);
    }
    Migr M;
    memset(&M, 0, sizeof M);
    M.r = r;
    M.W = dW;
    M.err = derr;
    M.un = u_new[l];
    M.own_o = own_o;
    M.box_o = l < hold->nlevels ? hold->levels[l].depths[0].d_box : nullptr;
    M.uo = l < hold->nlevels ? u_old[l] : nullptr;
    int64_t nc[3] = {n[0], n[1], n[2]};
    if (l > 0) {
      grid_of(hnew, l - 1, nc);
      if ((rc = dev_copy(H, &own_c, owner_map(hnew, hnew->levels[l - 1], nc), st))) {
        cleanup();
        return rc;
      }
      scratch.push_back(own_c);
      M.own_c = own_c;
      M.box_c = hnew->levels[l - 1].depths[0].d_box;
      M.uc = u_new[l - 1];
    } else if (!own_o) {
      cleanup();
      return fail(H, AMG_EINVAL, "level 0 has no source");
    }
    // on level 0 every cell is copied: the coarse grid entries are the
    // level's own (owner lookups of the copy use Gc.n[.] * r, so divide)
    M.Gc.n[0] = (int32_t)(l > 0 ? nc[0] : n[0] / r);
    M.Gc.n[1] = (int32_t)(l > 0 ? nc[1] : n[1] / r);
    M.Gc.n[2] = (int32_t)(l > 0 ? nc[2] : std::max<int64_t>(n[2] / r, 1));
    if (l == 0 && (n[0] % r || n[1] % r || (dim == 3 && n[2] % r))) {
      cleanup();
      return fail(H, AMG_EUNSUPPORTED, "migration needs a level-0 grid divisible by the ratio");
    }
    for (const BoxD& X : Ln.depths[0].boxd) {
      M.X = X;
      const int64_t cells = (int64_t)X.n[0] * X.n[1] * X.n[2];
      const dim3 grid((unsigned)((cells + 255) / 256));
      if (dim == 2)
        hipLaunchKernelGGL(k_migrate<2>, grid, dim3(256), 0, st, M);
      else
        hipLaunchKernelGGL(k_migrate<3>, grid, dim3(256), 0, st, M);
      if (hipGetLastError() != hipSuccess) {
        cleanup();
        return fail(H, AMG_EDEVICE, "k_migrate launch failed");
      }
    }
  }
  int herr = 0;
  if (hipMemcpyAsync(&herr, derr, sizeof herr, hipMemcpyDeviceToHost, st) != hipSuccess) {
    cleanup();
    return fail(H, AMG_EDEVICE, "reading the migration flag failed");
  }
  cleanup();
  if (herr)
    return fail(H, AMG_EUNSUPPORTED,
                "a new cell has no source: an interpolation window leaves the new coarser level, or the old level 0 "
                "lacks a cell of the new one");
  return AMG_OK;
}
