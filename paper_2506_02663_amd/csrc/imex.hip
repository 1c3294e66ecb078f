// One time step of the IMEX scheme eq. GePUP-IMEX (Section 4) on a level
// that is one box covering a grid periodic in every direction (the domains
// of Section 7.3): the ERK-ESDIRK pair ARK4(3)6L[2]SA of Kennedy and
// Carpenter (2003) integrates d<w>/dt = X(<u>, <q>, t) + nu L <w>, with
// X = <g> - Div<uu> - G<q> (eq. ODE-MOL), the convection Div<uu> of eq.
// convOp, the pressure from L q = D(g - Div<uu>) (TLS-1), the stage
// Helmholtz systems (I - dt nu gamma L) w = rhs per component (TLS-2) and
// u = P w (eq. appProj, TLS-3).  The linear systems go through the level
// solver as a black box; the kernels here are the convection (wrapped
// indices on the one box: no ghosts) and the stage combinations.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <initializer_list>
#include <string>
#include <utility>
#include <vector>

#include "amg_internal.h"

using namespace amg;

namespace {

// ARK4(3)6L[2]SA: nodes, explicit and implicit tableaux, weights = last
// implicit row (stiffly accurate), diagonal gamma = 1/4.
constexpr int kStages = 6;
constexpr double kGamma = 0.25;
const double kAE[kStages][kStages] = {
    {0, 0, 0, 0, 0, 0},
    {0.5, 0, 0, 0, 0, 0},
    {13861.0 / 62500.0, 6889.0 / 62500.0, 0, 0, 0, 0},
    {-116923316275.0 / 2393684061468.0, -2731218467317.0 / 15368042101831.0, 9408046702089.0 / 11113171139209.0, 0,
     0, 0},
    {-451086348788.0 / 2902428689909.0, -2682348792572.0 / 7519795681897.0, 12662868775082.0 / 11960479115383.0,
     3355817975965.0 / 11060851509271.0, 0, 0},
    {647845179188.0 / 3216320057751.0, 73281519250.0 / 8382639484533.0, 552539513391.0 / 3454668386233.0,
     3354512671639.0 / 8306763924573.0, 4040.0 / 17871.0, 0}};
const double kAI[kStages][kStages] = {
    {0, 0, 0, 0, 0, 0},
    {0.25, 0.25, 0, 0, 0, 0},
    {8611.0 / 62500.0, -1743.0 / 31250.0, 0.25, 0, 0, 0},
    {5012029.0 / 34652500.0, -654441.0 / 2922500.0, 174375.0 / 388108.0, 0.25, 0, 0},
    {15267082809.0 / 155376265600.0, -71443401.0 / 120774400.0, 730878875.0 / 902184768.0, 2285395.0 / 8070912.0,
     0.25, 0},
    {82889.0 / 524892.0, 0, 15625.0 / 83664.0, 69875.0 / 102672.0, -2260.0 / 8211.0, 0.25}};

// the one box of depth 0: cell (x, y, z) at off + (x + 2) + (y + 2) s1 + (z + 2) s2
struct Geo {
  int64_t off;
  int32_t n[3];
  int32_t s1, s2;
};

struct In3 {
  const double* p[3];
};
struct Out3 {
  double* p[3];
};

constexpr int kMaxTerms = 12;
struct Combo {
  const double* src[kMaxTerms];
  double coef[kMaxTerms];
  int n;
};

__device__ __forceinline__ int wrap(int x, int n) { return x < 0 ? x + n : (x >= n ? x - n : x); }

// V_e = g_e + sign (Div<uu>)_e on every cell (g_e may be null: zero).
// Per direction d the flux F<u_d, u_e> on the two faces normal to d: the
// product of the face averages (eq. cell2face, first row) plus h^2/12 times
// the products of their centred transverse differences over 2h.
template <int DIM>
__global__ __launch_bounds__(256) void k_conv(Geo G, In3 U, In3 Gf, Out3 V, double h, double sign) {
  const int64_t cells = (int64_t)G.n[0] * G.n[1] * G.n[2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells) return;
  const int x = (int)(i % G.n[0]);
  const int y = (int)((i / G.n[0]) % G.n[1]);
  const int z = DIM == 3 ? (int)(i / ((int64_t)G.n[0] * G.n[1])) : 0;
  auto at = [&](int c, int px, int py, int pz) -> double {
    px = wrap(px, G.n[0]);
    py = wrap(py, G.n[1]);
    pz = DIM == 3 ? wrap(pz, G.n[2]) : 0;
    return U.p[c][G.off + (px + 2) + (int64_t)(py + 2) * G.s1 + (int64_t)(pz + 2) * G.s2];
  };
  // face average of component c on the high face along d of cell p
  auto fa = [&](int c, int d, const int p[3]) -> double {
    const int ex = d == 0, ey = d == 1, ez = d == 2;
    return (-at(c, p[0] + 2 * ex, p[1] + 2 * ey, p[2] + 2 * ez) + 7.0 * at(c, p[0] + ex, p[1] + ey, p[2] + ez) +
            7.0 * at(c, p[0], p[1], p[2]) - at(c, p[0] - ex, p[1] - ey, p[2] - ez)) *
           (1.0 / 12.0);
  };
  double acc[3] = {0.0, 0.0, 0.0};
  for (int d = 0; d < DIM; ++d)
    for (int side = 0; side < 2; ++side) {
      int p[3] = {x, y, z};
      if (!side) p[d] -= 1;  // the low face of the cell is the high face of its neighbour
      double f0[3];
      for (int c = 0; c < DIM; ++c) f0[c] = fa(c, d, p);
      double F[3];
      for (int e = 0; e < DIM; ++e) F[e] = f0[d] * f0[e];
      for (int dp = 0; dp < DIM; ++dp) {
        if (dp == d) continue;
        int pp[3] = {p[0], p[1], p[2]}, pm[3] = {p[0], p[1], p[2]};
        pp[dp] += 1;
        pm[dp] -= 1;
        double diff[3];
        for (int c = 0; c < DIM; ++c) diff[c] = fa(c, d, pp) - fa(c, d, pm);
        // h^2/12 * (diff_d / 2h) * (diff_e / 2h)
        for (int e = 0; e < DIM; ++e) F[e] += diff[d] * diff[e] * (1.0 / 48.0);
      }
      const double sg = side ? 1.0 : -1.0;
      for (int e = 0; e < DIM; ++e) acc[e] += sg * F[e];
    }
  const int64_t o = G.off + (x + 2) + (int64_t)(y + 2) * G.s1 + (int64_t)(z + 2) * G.s2;
  for (int e = 0; e < DIM; ++e) V.p[e][o] = (Gf.p[e] ? Gf.p[e][o] : 0.0) + sign * (acc[e] / h);
}

// dst = sum_k coef_k src_k on every cell (dst may be one of the sources)
__global__ __launch_bounds__(256) void k_combo(Geo G, double* dst, Combo cb) {
  const int64_t cells = (int64_t)G.n[0] * G.n[1] * G.n[2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cells) return;
  const int x = (int)(i % G.n[0]);
  const int y = (int)((i / G.n[0]) % G.n[1]);
  const int z = (int)(i / ((int64_t)G.n[0] * G.n[1]));
  const int64_t o = G.off + (x + 2) + (int64_t)(y + 2) * G.s1 + (int64_t)(z + 2) * G.s2;
  double s = 0.0;
  for (int k = 0; k < cb.n; ++k) s += cb.coef[k] * cb.src[k][o];
  dst[o] = s;
}

// *out = max over the cells of |v| (out cleared by the caller): per block a
// max over its share of the rows (a grid of at most kMaxAbsBlocks), then
// one atomic max on the bit pattern, which orders non-negative doubles (a
// NaN, positive, lands above infinity)
constexpr int kMaxAbsBlocks = 256;
__global__ __launch_bounds__(256) void k_maxabs(Geo G, const double* v, unsigned long long* out) {
  __shared__ double sh[4];
  // blocks stride over the rows (y, z), threads over x
  const int rows = G.n[1] * G.n[2];
  double m = 0.0;
  for (int r = (int)blockIdx.x; r < rows; r += (int)gridDim.x) {
    const int y = r % G.n[1], z = r / G.n[1];
    const double* row = v + G.off + 2 + (int64_t)(y + 2) * G.s1 + (int64_t)(z + 2) * G.s2;
    for (int x = (int)threadIdx.x; x < G.n[0]; x += (int)blockDim.x) {
      const double a = fabs(row[x]);
      const double c = (a == a) ? a : __longlong_as_double(0x7ff8000000000000LL);
      m = (c > m || c != c) ? c : m;
    }
  }
  for (int k = 32; k > 0; k >>= 1) {
    const double o = __shfl_xor(m, k, 64);
    m = (o > m || o != o) ? o : m;
  }
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = (sh[w] > m || sh[w] != sh[w]) ? sh[w] : m;
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
  }
}

int fail(amg_hier* H, int code, const std::string& msg) {
  if (H) H->err = msg;
  return code;
}

bool periodic_box(const amg_hier* H) {
  if (!H->finalized || H->nlevels != 1 || H->levels[0].isolated || H->levels[0].boxes.size() != 1) return false;
  const Box& B = H->levels[0].boxes[0];
  for (int d = 0; d < H->dim; ++d)
    if (H->phys_bc[d][0] != AMG_PERIODIC || H->phys_bc[d][1] != AMG_PERIODIC || B.lo[d] != 0 ||
        B.hi[d] != H->base[d] - 1)
      return false;
  return true;
}

Geo box_geo(const amg_hier* H) {
  const BoxD& X0 = H->levels[0].depths[0].boxd[0];
  Geo G;
  G.off = X0.off;
  G.n[0] = X0.n[0];
  G.n[1] = X0.n[1];
  G.n[2] = H->dim == 3 ? X0.n[2] : 1;
  G.s1 = X0.s[1];
  G.s2 = H->dim == 3 ? X0.s[2] : 0;
  return G;
}

}  // namespace

extern "C" int amg_convection(amg_hier* h, double* const* u, double* const* out, void* stream) {
  amg_hier* H = h;
  if (!h) return AMG_EINVAL;
  if (!u || !out) return fail(H, AMG_EINVAL, "null argument");
  if (!periodic_box(h))
    return fail(H, AMG_EUNSUPPORTED, "the convection operator needs one level of one box on a periodic grid");
  In3 Ui = {{nullptr, nullptr, nullptr}}, Gi = {{nullptr, nullptr, nullptr}};
  Out3 Vo = {{nullptr, nullptr, nullptr}};
  for (int d = 0; d < h->dim; ++d) {
    if (!u[d] || !out[d]) return fail(H, AMG_EINVAL, "null component");
    Ui.p[d] = u[d];
    Vo.p[d] = out[d];
    for (int e = 0; e < h->dim; ++e)
      if (out[d] == u[e]) return fail(H, AMG_EINVAL, "out may not alias u");
  }
  const Geo G = box_geo(h);
  const int64_t cells = (int64_t)G.n[0] * G.n[1] * G.n[2];
  hipStream_t st = stream ? (hipStream_t)stream : h->own;
  const double hh = h->levels[0].depths[0].h;
  if (h->dim == 2)
    hipLaunchKernelGGL(k_conv<2>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, G, Ui, Gi, Vo, hh, 1.0);
  else
    hipLaunchKernelGGL(k_conv<3>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, G, Ui, Gi, Vo, hh, 1.0);
  return hipGetLastError() == hipSuccess ? AMG_OK : fail(H, AMG_EDEVICE, "k_conv launch failed");
}

extern "C" int amg_imex_step(amg_hier* hv, amg_hier* hp, double dt, double nu, double* const* u,
                             const double* const* g, const amg_solve_opts* opts,
                             const amg_solve_opts* opts_p, amg_imex_stats* stats,
                             void* stream) {
  amg_hier* H = hv;
  if (!hv || !hp) return AMG_EINVAL;
  if (stats) memset(stats, 0, sizeof *stats);
  if (!u || !opts) return fail(H, AMG_EINVAL, "null argument");
  if (!opts_p) opts_p = opts;
  for (int d = 0; d < hv->dim; ++d)
    if (!u[d]) return fail(H, AMG_EINVAL, "null velocity component");
  if (!(dt > 0) || !(nu >= 0) || !std::isfinite(dt) || !std::isfinite(nu))
    return fail(H, AMG_EINVAL, "dt > 0 and nu >= 0 are required");
  if (hv->op != AMG_HELMHOLTZ || hp->op != AMG_POISSON)
    return fail(H, AMG_EINVAL, "hv takes the Helmholtz operator, hp the Poisson operator");
  if (hv->dim != hp->dim || hv->h0 != hp->h0)
    return fail(H, AMG_EINVAL, "the two hierarchies differ");
  for (int d = 0; d < hv->dim; ++d)
    if (hv->base[d] != hp->base[d]) return fail(H, AMG_EINVAL, "the two hierarchies differ");
  if (!periodic_box(hv) || !periodic_box(hp))
    return fail(H, AMG_EUNSUPPORTED, "the IMEX step needs one level of one box on a grid periodic in every direction");
  const int D = hv->dim;
  hipStream_t st = stream ? (hipStream_t)stream : hv->own;

  // the Helmholtz coefficient of every stage system
  const double c = dt * nu * kGamma;
  if (c > 0 && hv->c != c) {
    const int rc = amg_set_coefficient(hv, c);
    if (rc) return rc;
  }

  const Depth& D0 = hv->levels[0].depths[0];
  const Geo G = box_geo(hv);
  const int64_t N = D0.nstored;
  if (N != hp->levels[0].depths[0].nstored) return fail(H, AMG_EINVAL, "the two hierarchies differ");

  // workspace: w^n, w, the stage terms X_j and L w^(j), V, G q (D arrays
  // each), q, phi, the divergence and the stage right-hand side; one word
  // for the norm of a right-hand side
  const int narr = D * (1 + 1 + kStages + (kStages - 1) + 1 + 1) + 4;
  const int64_t need = (int64_t)narr * N + 1;
  if (hv->imex_len < need) {
    if (hv->imex_ws) (void)hipFree(hv->imex_ws);
    hv->imex_ws = nullptr;
    hv->imex_len = 0;
    hipError_t e = hipMalloc(&hv->imex_ws, need * sizeof(double));
    if (e != hipSuccess) return fail(H, AMG_EDEVICE, std::string("hipMalloc: ") + hipGetErrorString(e));
    e = hipMemset(hv->imex_ws, 0, need * sizeof(double));
    if (e != hipSuccess) return fail(H, AMG_EDEVICE, std::string("hipMemset: ") + hipGetErrorString(e));
    hv->imex_len = need;
  }
  double* ws = hv->imex_ws;
  int next = 0;
  auto take = [&]() { return ws + (int64_t)(next++) * N; };
  double *wn[3], *w[3], *Xs[kStages][3], *LW[kStages - 1][3], *V[3], *gq[3];
  for (int e = 0; e < D; ++e) wn[e] = take();
  for (int e = 0; e < D; ++e) w[e] = take();
  for (int j = 0; j < kStages; ++j)
    for (int e = 0; e < D; ++e) Xs[j][e] = take();
  for (int j = 0; j < kStages - 1; ++j)
    for (int e = 0; e < D; ++e) LW[j][e] = take();
  for (int e = 0; e < D; ++e) V[e] = take();
  for (int e = 0; e < D; ++e) gq[e] = take();
  double* q = take();
  double* phi = take();
  double* div = take();
  double* rhs = take();
  unsigned long long* dnorm = reinterpret_cast<unsigned long long*>(ws + (int64_t)narr * N);

  const int64_t cells = (int64_t)G.n[0] * G.n[1] * G.n[2];
  const dim3 grid((unsigned)((cells + 255) / 256)), block(256);
  int worst = AMG_OK;
  // ||b||_inf over the cells (one small reduction and a wait for it)
  auto rhs_norm = [&](const double* b, double& out) -> int {
    if (hipMemsetAsync(dnorm, 0, sizeof *dnorm, st) != hipSuccess) return fail(H, AMG_EDEVICE, "norm clear failed");
    const unsigned rows = (unsigned)G.n[1] * (unsigned)G.n[2];
    hipLaunchKernelGGL(k_maxabs, dim3(std::min<unsigned>(rows, kMaxAbsBlocks)), block, 0, st, G, b, dnorm);
    if (hipGetLastError() != hipSuccess) return fail(H, AMG_EDEVICE, "k_maxabs launch failed");
    unsigned long long bits = 0;
    if (hipMemcpyAsync(&bits, dnorm, sizeof bits, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(H, AMG_EDEVICE, "norm read failed");
    memcpy(&out, &bits, sizeof out);
    return AMG_OK;
  };
  // Every stage system starts from the previous stage's solution of the
  // same system and stops when ||r||_inf <= max(tol_rel ||b||_inf, tol_abs),
  // b its right-hand side: the test of a solve from zero, whose initial
  // residual is b.  A zero b has the zero solution (no solve).
  auto target_opts = [&](const amg_solve_opts* base, double bn, amg_solve_opts& o2) {
    o2 = *base;
    o2.tol_abs = std::max(base->tol_abs, base->tol_rel * bn);
    o2.tol_rel = 0.0;
  };
  auto account = [&](int rc, const amg_solve_stats& s, double bn) -> int {
    if (rc != AMG_OK && rc != AMG_ENOTCONVERGED) return rc;
    if (rc == AMG_ENOTCONVERGED) worst = AMG_ENOTCONVERGED;
    if (stats) {
      stats->solves += 1;
      stats->cycles += s.cycles;
      if (s.cycles > stats->max_cycles) stats->max_cycles = s.cycles;
      const double rel = bn > 0 ? s.rfinal / bn : 0.0;
      if (rel > stats->max_rel_residual) stats->max_rel_residual = rel;
    }
    return AMG_OK;
  };
  // the solve of (hier) x = b from the x it holds
  auto stage_solve = [&](amg_hier* hs, double* x, const double* b, const char* what) -> int {
    double bn = 0.0;
    int rc = rhs_norm(b, bn);
    if (rc) return rc;
    if (bn == 0.0) {
      if (hipMemsetAsync(x, 0, N * sizeof(double), st) != hipSuccess) return fail(H, AMG_EDEVICE, "clear failed");
      amg_solve_stats s0;
      memset(&s0, 0, sizeof s0);
      return account(AMG_OK, s0, 0.0);
    }
    amg_solve_opts o2;
    target_opts(hs == hp ? opts_p : opts, bn, o2);
    amg_solve_stats s;
    rc = account(amg_solve(hs, 0, 0, &x, &b, nullptr, &o2, &s, st), s, bn);
    if (rc) return fail(H, rc, std::string(what) + amg_last_error(hs));
    return AMG_OK;
  };
  auto combo = [&](double* dst, std::initializer_list<std::pair<const double*, double>> terms) -> int {
    Combo cb;
    memset(&cb, 0, sizeof cb);
    for (auto& t : terms) {
      if (t.second == 0.0) continue;
      cb.src[cb.n] = t.first;
      cb.coef[cb.n] = t.second;
      ++cb.n;
    }
    hipLaunchKernelGGL(k_combo, grid, block, 0, st, G, dst, cb);
    return hipGetLastError() == hipSuccess ? AMG_OK : fail(H, AMG_EDEVICE, "k_combo launch failed");
  };
  // X_j = g_j - Div<uu> - G q, L q = D(g_j - Div<uu>), from the current u
  auto explicit_term = [&](int j) -> int {
    In3 Ui = {{u[0], u[1], D == 3 ? u[2] : nullptr}};
    In3 Gi = {{nullptr, nullptr, nullptr}};
    if (g)
      for (int e = 0; e < D; ++e) Gi.p[e] = g[j * D + e];
    Out3 Vo = {{V[0], V[1], D == 3 ? V[2] : nullptr}};
    if (D == 2)
      hipLaunchKernelGGL(k_conv<2>, grid, block, 0, st, G, Ui, Gi, Vo, hv->levels[0].depths[0].h, -1.0);
    else
      hipLaunchKernelGGL(k_conv<3>, grid, block, 0, st, G, Ui, Gi, Vo, hv->levels[0].depths[0].h, -1.0);
    if (hipGetLastError() != hipSuccess) return fail(H, AMG_EDEVICE, "k_conv launch failed");
    int rc = amg_divergence(hv, 0, 0, V, nullptr, &div, st);
    if (rc) return rc;
    if ((rc = stage_solve(hp, q, div, "pressure solve: "))) return rc;
    rc = amg_gradient(hp, 0, 0, &q, nullptr, gq, st);
    if (rc) return fail(H, rc, std::string("pressure gradient: ") + amg_last_error(hp));
    for (int e = 0; e < D; ++e)
      if ((rc = combo(Xs[j][e], {{V[e], 1.0}, {gq[e], -1.0}}))) return rc;
    return AMG_OK;
  };
  // u = P w, the potential from the previous projection's (D w: the norm of
  // the potential's right-hand side; zero: u = w)
  auto project = [&]() -> int {
    double* wl[3] = {w[0], w[1], D == 3 ? w[2] : nullptr};
    int rc = amg_divergence(hv, 0, 0, wl, nullptr, &div, st);
    if (rc) return rc;
    double bn = 0.0;
    if ((rc = rhs_norm(div, bn))) return rc;
    if (bn == 0.0 && hipMemsetAsync(phi, 0, N * sizeof(double), st) != hipSuccess)
      return fail(H, AMG_EDEVICE, "clearing the potential failed");
    amg_solve_opts o2;
    target_opts(opts_p, bn, o2);
    amg_solve_stats s;
    rc = account(amg_project(hv, hp, 0, 0, wl, nullptr, &phi, u, &o2, &s, st), s, bn);
    if (rc) return fail(H, rc, std::string("projection: ") + amg_last_error(hp));
    return AMG_OK;
  };

  // stage 1: w = u = w^n; the pressure and the potential start from zero
  if (hipMemsetAsync(q, 0, N * sizeof(double), st) != hipSuccess ||
      hipMemsetAsync(phi, 0, N * sizeof(double), st) != hipSuccess)
    return fail(H, AMG_EDEVICE, "clearing the pressure failed");
  for (int e = 0; e < D; ++e) {
    if (hipMemcpyAsync(wn[e], u[e], N * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(w[e], u[e], N * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(H, AMG_EDEVICE, "copy of the initial velocity failed");
  }
  int rc;
  for (int s = 1; s < kStages; ++s) {
    const int j = s - 1;
    if ((rc = explicit_term(j))) return rc;
    for (int e = 0; e < D; ++e)
      if ((rc = amg_apply_laplacian(hv, 0, w[e], nullptr, LW[j][e], st))) return rc;
    for (int e = 0; e < D; ++e) {
      Combo cb;
      memset(&cb, 0, sizeof cb);
      cb.src[cb.n] = wn[e];
      cb.coef[cb.n++] = 1.0;
      for (int k = 0; k <= j; ++k) {
        if (kAE[s][k] != 0.0) {
          cb.src[cb.n] = Xs[k][e];
          cb.coef[cb.n++] = dt * kAE[s][k];
        }
        if (kAI[s][k] != 0.0 && nu != 0.0) {
          cb.src[cb.n] = LW[k][e];
          cb.coef[cb.n++] = dt * nu * kAI[s][k];
        }
      }
      if (c > 0) {
        hipLaunchKernelGGL(k_combo, grid, block, 0, st, G, rhs, cb);
        if (hipGetLastError() != hipSuccess) return fail(H, AMG_EDEVICE, "k_combo launch failed");
        // (I - c L) w^(s) = rhs from w^(s-1)
        if ((rc = stage_solve(hv, w[e], rhs, "Helmholtz solve: "))) return rc;
      } else {  // nu = 0: the stage system is the identity
        hipLaunchKernelGGL(k_combo, grid, block, 0, st, G, w[e], cb);
        if (hipGetLastError() != hipSuccess) return fail(H, AMG_EDEVICE, "k_combo launch failed");
      }
    }
    if ((rc = project())) return rc;
  }
  if ((rc = explicit_term(kStages - 1))) return rc;
  for (int e = 0; e < D; ++e) {
    Combo cb;
    memset(&cb, 0, sizeof cb);
    cb.src[cb.n] = w[e];
    cb.coef[cb.n++] = 1.0;
    for (int k = 0; k < kStages; ++k) {
      const double a = kAI[kStages - 1][k] - kAE[kStages - 1][k];  // b_k - A_E[6,k]
      if (a == 0.0) continue;
      cb.src[cb.n] = Xs[k][e];
      cb.coef[cb.n++] = dt * a;
    }
    hipLaunchKernelGGL(k_combo, grid, block, 0, st, G, w[e], cb);
    if (hipGetLastError() != hipSuccess) return fail(H, AMG_EDEVICE, "k_combo launch failed");
  }
  if ((rc = project())) return rc;
  if (stats) stats->converged = worst == AMG_OK;
  return worst;
}
