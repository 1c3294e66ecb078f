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
// A into its inverse; false if A is singular.  `threads` > 1 splits each
// column's row updates over that many threads (the pivot step runs on the
// first); every row's arithmetic is the same in any split.  Columns of A up
// to the current one are never read again, so only those right of it are
// updated.
bool invert(std::vector<double>& A, int n, int threads = 1) {
  std::vector<double> inv((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) inv[(size_t)i * n + i] = 1.0;
  const int T = std::max(1, std::min(threads, n / 64));
  SpinBarrier bar(T);
  std::atomic<bool> singular{false};
  auto work = [&](int tid) {
    for (int col = 0; col < n; ++col) {
      if (tid == 0) {
        int p = col;
        double best = std::fabs(A[(size_t)col * n + col]);
        for (int r = col + 1; r < n; ++r) {
          const double v = std::fabs(A[(size_t)r * n + col]);
          if (v > best) best = v, p = r;
        }
        if (best == 0.0) {
          singular.store(true);
        } else {
          if (p != col)
            for (int j = 0; j < n; ++j) {
              std::swap(A[(size_t)p * n + j], A[(size_t)col * n + j]);
              std::swap(inv[(size_t)p * n + j], inv[(size_t)col * n + j]);
            }
          const double d = 1.0 / A[(size_t)col * n + col];
          for (int j = col + 1; j < n; ++j) A[(size_t)col * n + j] *= d;
          for (int j = 0; j < n; ++j) inv[(size_t)col * n + j] *= d;
        }
      }
      if (T > 1) bar.wait();
      if (singular.load()) return;
      const double* ac = &A[(size_t)col * n];
      const double* ic = &inv[(size_t)col * n];
      for (int r = tid; r < n; r += T) {
        if (r == col) continue;
        const double f = A[(size_t)r * n + col];
        if (f == 0.0) continue;
        double* ar = &A[(size_t)r * n];
        double* ir = &inv[(size_t)r * n];
        for (int j = col + 1; j < n; ++j) ar[j] -= f * ac[j];
        for (int j = 0; j < n; ++j) ir[j] -= f * ic[j];
      }
      if (T > 1) bar.wait();
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < T; ++t) th.emplace_back(work, t);
  work(0);
  for (auto& t : th) t.join();
  if (singular.load()) return false;
  A.swap(inv);
  return true;
}

constexpr size_t kBatch = 8;                      // systems factorised at once
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
      // kBatch threads in all: one per system, the rest inside the inversions
      const int inner = jobs.empty() ? 1 : std::max<int>(1, (int)(kBatch / jobs.size()));
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
        mats.resize(base + 2 * (size_t)nn * nn);
        for (int64_t c = 0; c < nn; ++c)
          for (int64_t r = 0; r < nn; ++r) {
            mats[base + (size_t)c * nn + r] = J.A[(size_t)r * m + c];
            mats[G.matT + (size_t)c * nn + r] = J.A[(size_t)c * m + r];
          }
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
