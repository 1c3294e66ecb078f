// Host side of the exact bottom solve (the coarsest multigrid depth).
//
// The paper uses weighted Jacobi (TLS-2) or ILU-preconditioned GMRES (TLS-1,
// TLS-3) at the coarsest multigrid level (Section 6.5); this library solves
// that level exactly instead.  Here the homogeneous operator of the coarsest
// depth -- the stencil of eq. (discreteOps c) with the ghost fills of eqs.
// (velBCHomoDiri5th) / (Neumann5) folded in -- is assembled row by row for
// each independent system (a face-connected component of a coupled level, or
// one isolated box), and inverted in FP64 by Gauss-Jordan elimination with
// partial pivoting.  A component on which the operator has a constant null
// vector is bordered with one zero-mean constraint; the top-left block of the
// bordered inverse maps a consistent right-hand side to the zero-mean
// solution.  Identical systems (isolated boxes of equal shape) share one
// inverse.
//
// With the paper's bottom solver selected (amg_set_bottom_solver,
// ILU(0)-preconditioned GMRES(m), Section 6.5), each system (bordered when
// singular) is also factorised incompletely: ILU(0) on its pattern (the
// diagonal and the entries above 1e-12 of their row's largest, elimination
// in the i-k-j order), and the factors are inverted into one dense
// preconditioning matrix P = (L U)^-1, so that a preconditioning is one
// matrix-vector product; B = K P, the right-preconditioned operator, is kept
// beside it.  Unknowns are ordered box by box, x fastest within a box.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <immintrin.h>
#include <map>
#include <string>
#include <thread>
#include <tuple>

#include "amg_internal.h"

namespace amg {

namespace {

// coefficient of the m-th cell behind the row end (m = 0 is the end cell) in
// the first / second ghost
const double kFillD[2][4] = {{-77.0 / 12, 43.0 / 12, -17.0 / 12, 3.0 / 12},
                             {-505.0 / 12, 335.0 / 12, -145.0 / 12, 27.0 / 12}};
const double kFillN[2][4] = {{5.0 / 10, 9.0 / 10, -5.0 / 10, 1.0 / 10},
                             {-75.0 / 10, 145.0 / 10, -75.0 / 10, 15.0 / 10}};

// ILU(0) of the dense row-major N x N matrix K in place (combined factors:
// unit lower L strictly below the diagonal, U on and above it); false if a
// pivot vanishes
bool ilu0(std::vector<double>& K, int N) {
  std::vector<std::vector<int>> cols(N);  // pattern per row, increasing
  for (int i = 0; i < N; ++i) {
    double mx = 0.0;
    for (int j = 0; j < N; ++j) mx = std::max(mx, std::fabs(K[(size_t)i * N + j]));
    for (int j = 0; j < N; ++j) {
      const double v = K[(size_t)i * N + j];
      if (j == i || std::fabs(v) > 1e-12 * mx)
        cols[i].push_back(j);
      else
        K[(size_t)i * N + j] = 0.0;
    }
  }
  std::vector<char> in(N, 0);
  for (int i = 1; i < N; ++i) {
    double* ri = &K[(size_t)i * N];
    for (int j : cols[i]) in[j] = 1;
    for (int k : cols[i]) {
      if (k >= i) break;
      const double piv = K[(size_t)k * N + k];
      if (piv == 0.0) return false;
      ri[k] /= piv;
      const double* rk = &K[(size_t)k * N];
      for (int j : cols[k])
        if (j > k && in[j]) ri[j] -= ri[k] * rk[j];
    }
    for (int j : cols[i]) in[j] = 0;
  }
  for (int i = 0; i < N; ++i)
    if (K[(size_t)i * N + i] == 0.0) return false;
  return true;
}

// barrier for the threads of one inversion (spinning; the waits are short)
struct SpinBarrier {
  explicit SpinBarrier(int n) : n_(n) {}
  void wait() {
    const int gen = gen_.load(std::memory_order_acquire);
    if (count_.fetch_add(1, std::memory_order_acq_rel) == n_ - 1) {
      count_.store(0, std::memory_order_relaxed);
      gen_.fetch_add(1, std::memory_order_acq_rel);
    } else {
      int spins = 0;
      while (gen_.load(std::memory_order_acquire) == gen)
        if (++spins > 1024) std::this_thread::yield();
    }
  }
  int n_;
  std::atomic<int> count_{0}, gen_{0};
};

// In-place Gauss-Jordan with partial pivoting of the row-major n x n matrix
// c[i][0..m) -= sum_q a[i][q] B[q][0..m) for R rows at once (B rows ldb
// apart): eight columns of each row accumulate in registers over q, so every
// element of B loaded serves R rows.  An AVX2 form where the host has it.
template <int R>
void rows_update_plain(double* const* c, const double* const* a, const double* __restrict__ B, int b, size_t ldb,
                       int m) {
  for (int j = 0; j < m; ++j)
    for (int i = 0; i < R; ++i) {
      double s = c[i][j];
      for (int q = 0; q < b; ++q) s -= a[i][q] * B[q * ldb + j];
      c[i][j] = s;
    }
}

template <int R>
__attribute__((target("avx2,fma"))) void rows_update_avx2(double* const* c, const double* const* a,
                                                            const double* __restrict__ B, int b, size_t ldb, int m) {
  int j = 0;
  for (; j + 8 <= m; j += 8) {
    __m256d acc[R][2];
    for (int i = 0; i < R; ++i) {
      acc[i][0] = _mm256_loadu_pd(c[i] + j);
      acc[i][1] = _mm256_loadu_pd(c[i] + j + 4);
    }
    for (int q = 0; q < b; ++q) {
      const double* bq = B + q * ldb + j;
      const __m256d b0 = _mm256_loadu_pd(bq), b1 = _mm256_loadu_pd(bq + 4);
      for (int i = 0; i < R; ++i) {
        const __m256d f = _mm256_broadcast_sd(a[i] + q);
        acc[i][0] = _mm256_fnmadd_pd(f, b0, acc[i][0]);
        acc[i][1] = _mm256_fnmadd_pd(f, b1, acc[i][1]);
      }
    }
    for (int i = 0; i < R; ++i) {
      _mm256_storeu_pd(c[i] + j, acc[i][0]);
      _mm256_storeu_pd(c[i] + j + 4, acc[i][1]);
    }
  }
  if (j < m) {
    double* cr[R];
    for (int i = 0; i < R; ++i) cr[i] = c[i] + j;
    rows_update_plain<R>(cr, a, B + j, b, ldb, m - j);
  }
}

// the same over column tiles of 256 (B's tile, b x 256, stays in L2)
template <int R>
void rows_update(bool avx2, double* const* c, const double* const* a, const double* B, int b, size_t ldb, int m) {
  constexpr int kTile = 256;
  for (int j0 = 0; j0 < m; j0 += kTile) {
    double* cc[R];
    for (int i = 0; i < R; ++i) cc[i] = c[i] + j0;
    if (avx2)
      rows_update_avx2<R>(cc, a, B + j0, b, ldb, std::min(kTile, m - j0));
    else
      rows_update_plain<R>(cc, a, B + j0, b, ldb, std::min(kTile, m - j0));
  }
}

// A into its inverse; false if A is singular.  Gauss-Jordan elimination with
// partial pivoting, in blocks of kPanel columns: the block's pivots come from
// an LU factorisation of its columns over the rows not yet pivotal (the
// pivots column-by-column elimination would pick), the same row swaps are
// applied to A and to X (the inverse being built, initially I), the pivot
// rows of the trailing columns of A and of X are multiplied by the inverse
// of the block's pivot block, and every other row subtracts its block
// entries times those rows (a product of a (n - b) x b and a b x (trailing)
// matrix).  `threads` > 1 splits the products by rows and columns.
bool invert(std::vector<double>& A, int n, int threads = 1) {
  constexpr int kPanel = 64;
  std::vector<double> X((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) X[(size_t)i * n + i] = 1.0;
  const int T = std::max(1, std::min(threads, n / 64));
  const bool avx2 = __builtin_cpu_supports("avx2") && __builtin_cpu_supports("fma");
  SpinBarrier bar(T);
  std::atomic<bool> singular{false};
  // the block's panel (rows k.. x b, LU in place), -A_KK^-1 (b x b), and the
  // new pivot rows K = A_KK^-1 [A_K,trailing | X_K] (b x (trailing + n))
  std::vector<double> P((size_t)n * kPanel), W((size_t)kPanel * kPanel), K((size_t)kPanel * 2 * n);
  std::vector<double> Li((size_t)kPanel * kPanel), Ui((size_t)kPanel * kPanel);
  std::vector<int> piv(kPanel);
  auto work = [&](int tid) {
    for (int k = 0; k < n; k += kPanel) {
      const int b = std::min(kPanel, n - k), rows = n - k;
      const int mt = n - k - b;  // trailing columns of A
      const int m = mt + n;      // and every column of X
      if (tid == 0) {
        for (int r = 0; r < rows; ++r)
          for (int c = 0; c < b; ++c) P[(size_t)r * b + c] = A[(size_t)(k + r) * n + k + c];
        for (int c = 0; c < b; ++c) {
          int p = c;
          double best = std::fabs(P[(size_t)c * b + c]);
          for (int r = c + 1; r < rows; ++r) {
            const double v = std::fabs(P[(size_t)r * b + c]);
            if (v > best) best = v, p = r;
          }
          if (best == 0.0) {
            singular.store(true);
            break;
          }
          piv[c] = p;
          if (p != c)
            for (int j = 0; j < b; ++j) std::swap(P[(size_t)p * b + j], P[(size_t)c * b + j]);
          const double d = 1.0 / P[(size_t)c * b + c];
          const double* pc = &P[(size_t)c * b];
          for (int r = c + 1; r < rows; ++r) {
            double* pr = &P[(size_t)r * b];
            const double f = (pr[c] *= d);
            if (f != 0.0)
              for (int j = c + 1; j < b; ++j) pr[j] -= f * pc[j];
          }
        }
        if (!singular.load()) {
          // the swaps on whole rows (A's block columns keep their values
          // from before the block: they are the multipliers below)
          for (int c = 0; c < b; ++c)
            if (piv[c] != c) {
              std::swap_ranges(&A[(size_t)(k + c) * n], &A[(size_t)(k + c) * n] + n, &A[(size_t)(k + piv[c]) * n]);
              std::swap_ranges(&X[(size_t)(k + c) * n], &X[(size_t)(k + c) * n] + n, &X[(size_t)(k + piv[c]) * n]);
            }
          // A_KK = L U (unit lower L below the diagonal of the panel's top
          // block, U on and above it); W = -U^-1 L^-1
          for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
              Li[(size_t)i * b + j] = i == j ? 1.0 : 0.0;
              Ui[(size_t)i * b + j] = 0.0;
            }
          for (int i = 0; i < b; ++i)
            for (int j = 0; j < i; ++j) {
              double s = 0.0;
              for (int q = j; q < i; ++q) s += P[(size_t)i * b + q] * Li[(size_t)q * b + j];
              Li[(size_t)i * b + j] = -s;
            }
          for (int i = b - 1; i >= 0; --i) {
            const double d = 1.0 / P[(size_t)i * b + i];
            Ui[(size_t)i * b + i] = d;
            for (int j = i + 1; j < b; ++j) {
              double s = 0.0;
              for (int q = i + 1; q <= j; ++q) s += P[(size_t)i * b + q] * Ui[(size_t)q * b + j];
              Ui[(size_t)i * b + j] = -s * d;
            }
          }
          for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j) {
              double s = 0.0;
              for (int q = std::max(i, j); q < b; ++q) s += Ui[(size_t)i * b + q] * Li[(size_t)q * b + j];
              W[(size_t)i * b + j] = -s;
            }
        }
      }
      if (T > 1) bar.wait();
      if (singular.load()) return;
      // K = 0 - W [A_K,trailing | X_K], by column ranges
      {
        const int per = ((m + T - 1) / T + 7) / 8 * 8, j0 = std::min(m, tid * per), j1 = std::min(m, j0 + per);
        for (int i = 0; i < b; ++i) std::fill(&K[(size_t)i * m + j0], &K[(size_t)i * m + j1], 0.0);
        // K columns c0..c1 from the rows k.. of src, starting at its column s0
        auto part = [&](int c0, int c1, const double* src, int s0) {
          if (c1 <= c0) return;
          const double* B = src + (size_t)k * n + s0;
          for (int i0 = 0; i0 < b; i0 += 4) {
            double* c[4];
            const double* a[4];
            const int R = std::min(4, b - i0);
            for (int i = 0; i < R; ++i) {
              c[i] = &K[(size_t)(i0 + i) * m + c0];
              a[i] = &W[(size_t)(i0 + i) * b];
            }
            if (R == 4)
              rows_update<4>(avx2, c, a, B, b, (size_t)n, c1 - c0);
            else
              for (int i = 0; i < R; ++i) rows_update<1>(avx2, c + i, a + i, B, b, (size_t)n, c1 - c0);
          }
        };
        part(j0, std::min(j1, mt), A.data(), k + b + j0);
        part(std::max(j0, mt), j1, X.data(), std::max(j0, mt) - mt);
      }
      if (T > 1) bar.wait();
      // every other row: [A_r,trailing | X_r] -= A_rK K, four rows at a
      // time (a group of four lies wholly in the pivot rows or out of them:
      // k is a multiple of four, and the last block runs to the last row);
      // the pivot rows take K
      for (int g = tid; g < (n + 3) / 4; g += T) {
        const int r0 = 4 * g, r1 = std::min(n, r0 + 4);
        if (r0 >= k && r0 < k + b) {
          for (int r = r0; r < r1; ++r) {
            const double* kr = &K[(size_t)(r - k) * m];
            std::copy(kr, kr + mt, &A[(size_t)r * n] + k + b);
            std::copy(kr + mt, kr + m, &X[(size_t)r * n]);
          }
          continue;
        }
        double* ca[4];
        double* cx[4];
        const double* aa[4];
        for (int r = r0; r < r1; ++r) {
          ca[r - r0] = &A[(size_t)r * n] + k + b;
          cx[r - r0] = &X[(size_t)r * n];
          aa[r - r0] = &A[(size_t)r * n] + k;
        }
        if (r1 - r0 == 4) {
          rows_update<4>(avx2, ca, aa, K.data(), b, (size_t)m, mt);
          rows_update<4>(avx2, cx, aa, K.data() + mt, b, (size_t)m, n);
        } else {
          for (int i = 0; i < r1 - r0; ++i) {
            rows_update<1>(avx2, ca + i, aa + i, K.data(), b, (size_t)m, mt);
            rows_update<1>(avx2, cx + i, aa + i, K.data() + mt, b, (size_t)m, n);
          }
        }
      }
      if (T > 1) bar.wait();
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& t : th) t.join();
  if (singular.load()) return false;
  A.swap(X);
  return true;
}

constexpr size_t kBatch = 8;                      // systems factorised at once
constexpr unsigned kHostThreads = 16;             // host threads of a batch at most
constexpr size_t kBatchBytes = (size_t)1 << 30;  // their matrices' bytes at once

// one bottom system: the assembled (bordered) matrix, replaced by its
// inverse; with the ILU-GMRES bottom also B = K P and P = (L U)^-1, both
// column-major
struct Job {
  int group = 0, m = 0, n = 0;
  std::vector<double> A, K, B, P;
  bool ok = true;
  std::string err;
};

void factorise(Job& J, int kind, int threads) {
  const int m = J.m;
  if (!invert(J.A, m, threads)) {
    J.ok = false;
    J.err = "singular bottom system";
    return;
  }
  if (kind != AMG_BOTTOM_ILU_GMRES) return;
  std::vector<double> LU = J.K;
  if (!ilu0(LU, m)) {
    J.ok = false;
    J.err = "ILU(0) of a bottom system met a zero pivot";
    return;
  }
  // P = (L U)^-1 by columns (forward then back substitution), then B = K P
  J.P.assign((size_t)m * m, 0.0);
  std::vector<double> y(m);
  for (int c = 0; c < m; ++c) {
    for (int i = 0; i < m; ++i) {
      double s = i == c ? 1.0 : 0.0;
      const double* ri = &LU[(size_t)i * m];
      for (int j = 0; j < i; ++j) s -= ri[j] * y[j];
      y[i] = s;
    }
    for (int i = m - 1; i >= 0; --i) {
      double s = y[i];
      const double* ri = &LU[(size_t)i * m];
      for (int j = i + 1; j < m; ++j) s -= ri[j] * J.P[(size_t)c * m + j];
      J.P[(size_t)c * m + i] = s / ri[i];
    }
  }
  J.B.assign((size_t)m * m, 0.0);
  for (int c = 0; c < m; ++c)
    for (int r = 0; r < m; ++r) {
      double s = 0.0;
      const double* kr = &J.K[(size_t)r * m];
      for (int j = 0; j < m; ++j)
        if (kr[j] != 0.0) s += kr[j] * J.P[(size_t)c * m + j];
      J.B[(size_t)c * m + r] = s;
    }
}

}  // namespace

int build_bottom(amg_hier* H, int l, std::string& err, std::vector<double>& mats, std::vector<int64_t>& idx) {
  Level& L = H->levels[l];
  const int dim = H->dim;
  L.ngws = 0;
  for (size_t k = 0; k < L.depths.size(); ++k) {
    Depth& D = L.depths[k];
    D.groups.clear();
    if (D.bottom_boxes.empty()) continue;
    // systems: lists of boxes (at this depth)
    std::vector<std::vector<int>> systems;
    if (L.isolated) {
      for (int b : D.bottom_boxes) systems.push_back({b});
    } else {
      std::vector<std::vector<int>> bycomp(L.ncomp);
      for (int b : D.bottom_boxes) bycomp[D.boxd[b].comp].push_back(b);
      for (auto& v : bycomp)
        if (!v.empty()) systems.push_back(v);
    }
    const double K = 1.0 / (12.0 * D.h * D.h);
    std::map<std::tuple<int, int, int>, int> shared;  // isolated: shape -> group
    std::vector<std::vector<int64_t>> group_elems;
    // systems waiting for their factorisation, run in parallel batches (at
    // most kBatch systems and kBatchBytes of matrices at once); results are
    // appended in the order the systems were met
    std::vector<Job> jobs;
    size_t pending = 0;
    auto flush = [&]() -> int {
      // one thread per system, the rest of the host's (at most
      // kHostThreads) inside the inversions
      const unsigned hw = std::max(1u, std::min(kHostThreads, std::thread::hardware_concurrency()));
      const int inner = jobs.empty() ? 1 : std::max<int>(1, (int)(hw / jobs.size()));
      std::vector<std::thread> th;
      for (size_t q = 1; q < jobs.size(); ++q)
        th.emplace_back(factorise, std::ref(jobs[q]), H->bottom_kind, inner);
      if (!jobs.empty()) factorise(jobs[0], H->bottom_kind, inner);
      for (auto& t : th) t.join();
      for (Job& J : jobs) {
        if (!J.ok) {
          err = J.err;
          return AMG_EUNSUPPORTED;
        }
        BottomGroupD& G = D.groups[J.group];
        const int64_t nn = J.n, m = J.m;
        // column-major top-left n x n block of the inverse, then its transpose
        const size_t base = mats.size();
        G.mat = (int64_t)base;
        G.matT = (int64_t)(base + (size_t)nn * nn);
        if (mats.capacity() < base + 2 * (size_t)nn * nn)
          mats.reserve(std::max(base + 2 * (size_t)nn * nn, 2 * mats.capacity()));
        mats.resize(base + (size_t)nn * nn);
        constexpr int64_t kT = 32;  // the block itself: transposed in 32 x 32 tiles
        for (int64_t c0 = 0; c0 < nn; c0 += kT)
          for (int64_t r0 = 0; r0 < nn; r0 += kT)
            for (int64_t r = r0; r < std::min(nn, r0 + kT); ++r)
              for (int64_t c = c0; c < std::min(nn, c0 + kT); ++c)
                mats[base + (size_t)c * nn + r] = J.A[(size_t)r * m + c];
        for (int64_t c = 0; c < nn; ++c)  // its transpose: the rows of A in order
          mats.insert(mats.end(), &J.A[(size_t)c * m], &J.A[(size_t)c * m] + nn);
        if (H->bottom_kind == AMG_BOTTOM_ILU_GMRES) {
          G.ilub = (int64_t)mats.size();
          G.ilup = G.ilub + m * m;
          mats.insert(mats.end(), J.B.begin(), J.B.end());
          mats.insert(mats.end(), J.P.begin(), J.P.end());
        }
      }
      jobs.clear();
      pending = 0;
      return AMG_OK;
    };
    for (auto& sys : systems) {
      // local numbering
      std::vector<int64_t> start(D.boxes.size(), -1);
      int64_t n = 0;
      for (int b : sys) {
        start[b] = n;
        n += (int64_t)D.boxd[b].n[0] * D.boxd[b].n[1] * D.boxd[b].n[2];
      }
      const int comp = D.boxd[sys[0]].comp;
      const bool sing = L.comp_singular[comp] != 0;
      // element indices of this instance
      std::vector<int64_t> elems;
      for (int b : sys) {
        const BoxD& X = D.boxd[b];
        for (int z = 0; z < X.n[2]; ++z)
          for (int y = 0; y < X.n[1]; ++y)
            for (int x = 0; x < X.n[0]; ++x)
              elems.push_back(X.off + (int64_t)(x + 2) * X.s[0] + (int64_t)(y + 2) * X.s[1] +
                              (dim == 3 ? (int64_t)(z + 2) * X.s[2] : 0));
      }
      if (L.isolated) {
        const BoxD& X = D.boxd[sys[0]];
        auto key = std::make_tuple(X.n[0], X.n[1], X.n[2]);
        auto it = shared.find(key);
        if (it != shared.end()) {
          D.groups[it->second].ninst += 1;
          auto& ge = group_elems[it->second];
          ge.insert(ge.end(), elems.begin(), elems.end());
          continue;
        }
      }
      if (n > 8192) {
        char buf[200];
        snprintf(buf, sizeof buf, "coarsest system of level %d has %lld unknowns (limit 8192)", l, (long long)n);
        err = buf;
        return AMG_EUNSUPPORTED;
      }
      const int m = (int)n + (sing ? 1 : 0);
      std::vector<double> A((size_t)m * m, 0.0);
      std::vector<double> Ks;  // the system itself (ILU-GMRES bottom)
      auto lidx = [&](int b, int x, int y, int z) -> int64_t {
        const BoxD& X = D.boxd[b];
        return start[b] + x + (int64_t)X.n[0] * (y + (int64_t)X.n[1] * z);
      };
      for (int b : sys) {
        const BoxD& X = D.boxd[b];
        const Box& B = D.boxes[b];
        for (int z = 0; z < X.n[2]; ++z)
          for (int y = 0; y < X.n[1]; ++y)
            for (int x = 0; x < X.n[0]; ++x) {
              int64_t row = lidx(b, x, y, z);
              double* R = &A[(size_t)row * m];
              int loc[3] = {x, y, z};
              R[row] += -30.0 * dim * K;
              for (int d = 0; d < dim; ++d) {
                int t0 = -1, t1 = -1;
                for (int e = 0; e < dim; ++e)
                  if (e != d) (t0 < 0 ? t0 : t1) = e;
                for (int o : {-2, -1, 1, 2}) {
                  double w = (o == 1 || o == -1) ? 16.0 * K : -1.0 * K;
                  int p = loc[d] + o;
                  if (p >= 0 && p < X.n[d]) {
                    int q[3] = {x, y, z};
                    q[d] = p;
                    R[lidx(b, q[0], q[1], q[2])] += w;
                    continue;
                  }
                  int s = o > 0 ? 1 : 0;
                  int layer = s ? p - (X.n[d] - 1) : -p;
                  size_t col = (size_t)loc[t0] + (size_t)X.n[t0] * (dim == 3 ? loc[t1] : 0);
                  const FaceCols& fc = D.faces[b * 6 + d * 2 + s];
                  uint8_t kind = layer == 1 ? fc.k1[col] : fc.k2[col];
                  if (kind == G_FILL_D || kind == G_FILL_N) {
                    const double* a = kind == G_FILL_D ? kFillD[layer - 1] : kFillN[layer - 1];
                    int e0 = s ? X.n[d] - 1 : 0;
                    for (int mm = 0; mm < 4; ++mm) {
                      int q[3] = {x, y, z};
                      q[d] = s ? e0 - mm : e0 + mm;
                      R[lidx(b, q[0], q[1], q[2])] += w * a[mm];
                    }
                  } else if (kind == G_EXCH) {
                    int j = layer == 1 ? fc.src1[col] : fc.src2[col];
                    const Box& C = D.boxes[j];
                    int g[3] = {B.lo[0] + x, B.lo[1] + y, B.lo[2] + z};
                    g[d] = B.lo[d] + p;
                    if (D.periodic[d]) g[d] = ((g[d] % D.dn[d]) + D.dn[d]) % D.dn[d];
                    if (start[j] < 0) {
                      err = "exchange source outside the bottom system";
                      return AMG_EUNSUPPORTED;
                    }
                    R[lidx(j, g[0] - C.lo[0], g[1] - C.lo[1], dim == 3 ? g[2] - C.lo[2] : 0)] += w;
                  }
                }
              }
            }
      }
      if (H->op == AMG_HELMHOLTZ) {
        for (int64_t i = 0; i < n; ++i)
          for (int64_t j = 0; j < n; ++j) A[(size_t)i * m + j] = (i == j ? 1.0 : 0.0) - H->c * A[(size_t)i * m + j];
      }
      if (sing) {
        for (int64_t i = 0; i < n; ++i) {
          A[(size_t)i * m + n] = 1.0;
          A[(size_t)n * m + i] = 1.0;
        }
      }
      if (H->bottom_kind == AMG_BOTTOM_ILU_GMRES) {
        if (m > 4096) {  // the GMRES kernel stages one vector of the system in LDS
          char b2[160];
          snprintf(b2, sizeof b2, "coarsest system of level %d has %d unknowns (ILU-GMRES bottom: at most 4096)", l, m);
          err = b2;
          return AMG_EUNSUPPORTED;
        }
        Ks = A;
      }
      // the group's place is fixed now; its matrices follow when the batch
      // of pending systems is factorised
      const size_t bytes = (H->bottom_kind == AMG_BOTTOM_ILU_GMRES ? 4 : 2) * (size_t)m * m * sizeof(double);
      if (!jobs.empty() && (jobs.size() >= kBatch || pending + bytes > kBatchBytes)) {
        const int rc = flush();
        if (rc != AMG_OK) return rc;
      }
      BottomGroupD G;
      memset(&G, 0, sizeof G);
      G.mat = G.matT = G.idx = G.ilub = G.ilup = G.ws = -1;
      G.n = (int32_t)n;
      G.N = m;
      G.ninst = 1;
      Job J;
      J.group = (int)D.groups.size();
      J.m = m;
      J.n = (int)n;
      J.A.swap(A);
      J.K.swap(Ks);
      jobs.push_back(std::move(J));
      pending += bytes;
      group_elems.push_back(elems);
      if (L.isolated) {
        const BoxD& X = D.boxd[sys[0]];
        shared[std::make_tuple(X.n[0], X.n[1], X.n[2])] = (int)D.groups.size();
      }
      D.groups.push_back(G);
    }
    {
      const int rc = flush();
      if (rc != AMG_OK) return rc;
    }
    // instances of one group are contiguous in the index pool
    for (size_t g = 0; g < D.groups.size(); ++g) {
      D.groups[g].idx = (int64_t)idx.size();
      idx.insert(idx.end(), group_elems[g].begin(), group_elems[g].end());
      if (H->bottom_kind == AMG_BOTTOM_ILU_GMRES) {  // m + 1 Krylov vectors per instance
        D.groups[g].ws = L.ngws;
        L.ngws += (int64_t)D.groups[g].ninst * (H->bottom_iters + 1) * D.groups[g].N;
      }
    }
  }
  return AMG_OK;
}

}  // namespace amg

extern "C" int amg_dense_inverse(int n, double* a, int threads) {
  if (n < 1 || !a || threads < 1) return AMG_EINVAL;
  std::vector<double> A(a, a + (size_t)n * n);
  if (!amg::invert(A, n, threads)) return AMG_EUNSUPPORTED;
  std::copy(A.begin(), A.end(), a);
  return AMG_OK;
}
