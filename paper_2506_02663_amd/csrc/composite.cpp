// Host planner of the composite (multi-level) operator: the index tables of
// coarse-fine interpolation, average-down, refluxing and the prolongation of
// a coarse level's correction onto the next finer level.
//
//  * Coarse-fine interpolation (AMRCFI, Section 5.2): each interpolated ghost
//    of level l is a fixed combination of a 5^D window of level-(l-1) cells.
//    Per direction the weights give the average over the child of the
//    quartic whose averages over the five window cells equal the data; the
//    window is centred on the parent and shifted by the least amount that
//    keeps it inside the domain.  The weights are computed here by solving
//    the 5 x 5 moment system.
//  * Average-down (eq. AMR_avergingDownToCrse, COH-4): coarse cell := mean of
//    its r^D children (r the refinement ratio, 2 or 4).
//  * Refluxing (COH-3): at a valid coarse cell, the coarse flux through a face
//    bordering level l is replaced by the mean of the fine fluxes through the
//    fine faces covering it (fourth-order face derivatives, eq. cell2face).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "amg_internal.h"

namespace amg {

namespace {

// weights[(s + 2) * r + child][m]: five window cells m = 0..4, window
// shifted by s cells from the parent's centred position (parent = window
// cell 2 - s), child 0..r-1 from the parent's low end
void cfi_weights(double W[20][5], int r) {
  for (int s = -2; s <= 2; ++s)
    for (int a = 0; a < r; ++a) {
      // moment matrix M[m][k] = average of x^k over [m, m+1]; child average of
      // the quartic = c . coef with M coef = U, so the weights solve M^T w = c
      long double A[5][6];
      const long double x0 = (2 - s) + (long double)a / r, x1 = x0 + 1.0L / r;
      for (int k = 0; k < 5; ++k) {
        for (int m = 0; m < 5; ++m) A[k][m] = (std::pow((long double)(m + 1), k + 1) - std::pow((long double)m, k + 1)) / (k + 1);
        A[k][5] = (std::pow(x1, k + 1) - std::pow(x0, k + 1)) / ((k + 1) * (x1 - x0));
      }
      for (int c = 0; c < 5; ++c) {
        int p = c;
        for (int r = c + 1; r < 5; ++r)
          if (std::fabs(A[r][c]) > std::fabs(A[p][c])) p = r;
        for (int j = 0; j < 6; ++j) std::swap(A[c][j], A[p][j]);
        for (int r = 0; r < 5; ++r) {
          if (r == c) continue;
          const long double f = A[r][c] / A[c][c];
          for (int j = 0; j < 6; ++j) A[r][j] -= f * A[c][j];
        }
      }
      for (int m = 0; m < 5; ++m) W[(s + 2) * r + a][m] = (double)(A[m][5] / A[m][m]);
    }
}

struct Owner {  // dense map grid cell -> box at depth 0 of a level
  int dim;
  int64_t n[3];
  std::vector<int32_t> box;
  int32_t at(const int* g) const {
    for (int d = 0; d < dim; ++d)
      if (g[d] < 0 || g[d] >= n[d]) return -1;
    int64_t i = g[0] + n[0] * (g[1] + (dim == 3 ? n[1] * (int64_t)g[2] : 0));
    return box[i];
  }
};

Owner make_owner(const amg_hier* H, const Level& L, int l) {
  Owner o;
  o.dim = H->dim;
  for (int d = 0; d < 3; ++d) {
    o.n[d] = 1;
    if (d < H->dim) {
      o.n[d] = H->base[d];
      for (int i = 0; i < l; ++i) o.n[d] *= H->ratio;
    }
  }
  o.box.assign((size_t)(o.n[0] * o.n[1] * o.n[2]), -1);
  const Depth& D = L.depths[0];
  for (size_t b = 0; b < D.boxes.size(); ++b) {
    const Box& B = D.boxes[b];
    for (int z = B.lo[2]; z <= B.hi[2]; ++z)
      for (int y = B.lo[1]; y <= B.hi[1]; ++y)
        for (int x = B.lo[0]; x <= B.hi[0]; ++x) o.box[x + o.n[0] * (y + o.n[1] * (int64_t)z)] = (int32_t)b;
  }
  return o;
}

int64_t elem(const Depth& D, int b, const int* g, int dim) {
  const BoxD& X = D.boxd[b];
  const Box& B = D.boxes[b];
  int64_t e = X.off + (int64_t)(g[0] - B.lo[0] + 2) * X.s[0] + (int64_t)(g[1] - B.lo[1] + 2) * X.s[1];
  if (dim == 3) e += (int64_t)(g[2] - B.lo[2] + 2) * X.s[2];
  return e;
}

int floordiv(int v, int r) { return v >= 0 ? v / r : -((-v + r - 1) / r); }

}  // namespace

void cfi_weight_table(double W[20][5], int r) { cfi_weights(W, r); }

int build_composite(amg_hier* H, int l, std::string& err) {
  Level& F = H->levels[l];
  Level& C = H->levels[l - 1];
  Composite& X = F.cmp;
  const int dim = H->dim;
  char buf[256];
  const int r = H->ratio;
  X.r = r;
  cfi_weights(X.w, r);
  const Owner oc = make_owner(H, C, l - 1), of = make_owner(H, F, l);
  const Depth& DF = F.depths[0];
  const Depth& DC = C.depths[0];
  const int nwin = dim == 2 ? 25 : 125;

  // every fine cell's parent must be a cell of the coarse level (nesting)
  for (size_t b = 0; b < DF.boxes.size(); ++b) {
    const Box& B = DF.boxes[b];
    int g[3];
    for (g[2] = B.lo[2]; g[2] <= B.hi[2]; g[2] += (dim == 3 ? r : 1))
      for (g[1] = B.lo[1]; g[1] <= B.hi[1]; g[1] += r)
        for (g[0] = B.lo[0]; g[0] <= B.hi[0]; g[0] += r) {
          int p[3] = {g[0] / r, g[1] / r, dim == 3 ? g[2] / r : 0};
          if (oc.at(p) < 0) {
            snprintf(buf, sizeof buf, "level %d is not nested in level %d", l, l - 1);
            err = buf;
            return AMG_ELAYOUT;
          }
        }
  }

  // ---- coarse-fine interpolation of the ghost cells of kind ZERO ----
  X.cfi_dst.clear();
  X.cfi_src.clear();
  X.cfi_w.clear();
  for (size_t b = 0; b < DF.boxes.size(); ++b) {
    const Box& B = DF.boxes[b];
    for (int d = 0; d < dim; ++d) {
      int t[2] = {-1, -1}, k = 0;
      for (int e = 0; e < dim; ++e)
        if (e != d) t[k++] = e;
      const int n0 = B.n(t[0]);
      const int n1 = dim == 3 ? B.n(t[1]) : 1;
      for (int s = 0; s < 2; ++s) {
        const FaceCols& fc = DF.faces[b * 6 + d * 2 + s];
        for (int q1 = 0; q1 < n1; ++q1)
          for (int q0 = 0; q0 < n0; ++q0) {
            const size_t col = (size_t)q0 + (size_t)n0 * q1;
            for (int layer = 1; layer <= 2; ++layer) {
              const uint8_t kind = layer == 1 ? fc.k1[col] : fc.k2[col];
              if (kind != G_ZERO) continue;
              int g[3] = {0, 0, 0};
              g[d] = s ? B.hi[d] + layer : B.lo[d] - layer;
              g[t[0]] = B.lo[t[0]] + q0;
              if (dim == 3) g[t[1]] = B.lo[t[1]] + q1;
              X.cfi_dst.push_back(elem(DF, (int)b, g, dim));
              {
                int g0[3] = {g[0], g[1], g[2]};
                g0[d] = s ? B.hi[d] : B.lo[d];
                X.cfi_e0.push_back(elem(DF, (int)b, g0, dim));
                X.cfi_in.push_back((s ? -1 : 1) * DF.boxd[b].s[d]);
                X.cfi_layer.push_back((uint8_t)layer);
              }
              int lo[3] = {0, 0, 0};
              for (int e = 0; e < dim; ++e) {
                const int P = floordiv(g[e], r);
                const int N = (int)oc.n[e];
                int sh = 0;
                if (P < 2) sh = 2 - P;
                if (P > N - 3) sh = (N - 3) - P;
                lo[e] = P + sh - 2;
                X.cfi_w.push_back((uint8_t)((sh + 2) * r + (g[e] - r * P)));
              }
              for (int w = 0; w < nwin; ++w) {
                int q[3] = {lo[0] + w % 5, lo[1] + (w / 5) % 5, dim == 3 ? lo[2] + w / 25 : 0};
                const int cb = oc.at(q);
                if (cb < 0) {
                  snprintf(buf, sizeof buf, "interpolation window of level %d leaves level %d", l, l - 1);
                  err = buf;
                  return AMG_EUNSUPPORTED;
                }
                const int64_t e = elem(DC, cb, q, dim);
                if (e > INT32_MAX) {
                  err = "coarse level too large for 32-bit interpolation indices";
                  return AMG_EUNSUPPORTED;
                }
                X.cfi_src.push_back((int32_t)e);
              }
            }
          }
      }
    }
  }

  // ---- average-down (coarse cells under level l) ----
  X.avg.clear();
  std::vector<uint8_t> covered((size_t)(oc.n[0] * oc.n[1] * oc.n[2]), 0);
  for (size_t b = 0; b < DF.boxes.size(); ++b) {
    const Box& B = DF.boxes[b];
    const BoxD& Y = DF.boxd[b];
    int g[3];
    for (g[2] = B.lo[2]; g[2] <= B.hi[2]; g[2] += (dim == 3 ? r : 1))
      for (g[1] = B.lo[1]; g[1] <= B.hi[1]; g[1] += r)
        for (g[0] = B.lo[0]; g[0] <= B.hi[0]; g[0] += r) {
          int p[3] = {g[0] / r, g[1] / r, dim == 3 ? g[2] / r : 0};
          AvgD a;
          memset(&a, 0, sizeof a);
          a.ce = elem(DC, oc.at(p), p, dim);
          a.fe = elem(DF, (int)b, g, dim);
          a.fs1 = Y.s[1];
          a.fs2 = dim == 3 ? Y.s[2] : 0;
          X.avg.push_back(a);
          covered[p[0] + oc.n[0] * (p[1] + oc.n[1] * (int64_t)p[2])] = 1;
        }
  }
  auto is_cov = [&](const int* p) {
    for (int d = 0; d < dim; ++d)
      if (p[d] < 0 || p[d] >= oc.n[d]) return false;
    return covered[p[0] + oc.n[0] * (p[1] + oc.n[1] * (int64_t)p[2])] != 0;
  };

  // ---- refluxing at valid coarse cells next to level l ----
  X.rfx_cell.clear();
  X.rfx_ptr.assign(1, 0);
  X.rfx_face.clear();
  for (size_t b = 0; b < DC.boxes.size(); ++b) {
    const Box& B = DC.boxes[b];
    const BoxD& Y = DC.boxd[b];
    int i[3];
    for (i[2] = B.lo[2]; i[2] <= B.hi[2]; ++i[2])
      for (i[1] = B.lo[1]; i[1] <= B.hi[1]; ++i[1])
        for (i[0] = B.lo[0]; i[0] <= B.hi[0]; ++i[0]) {
          if (is_cov(i)) continue;
          size_t nf0 = X.rfx_face.size();
          for (int d = 0; d < dim; ++d)
            for (int sg = -1; sg <= 1; sg += 2) {
              int j[3] = {i[0], i[1], i[2]};
              j[d] += sg;
              if (!is_cov(j)) continue;
              // first fine cell past the face, transverse offset 0
              int f0[3] = {r * i[0], r * i[1], dim == 3 ? r * i[2] : 0};
              f0[d] = sg > 0 ? r * j[d] : r * j[d] + r - 1;
              const int fb = of.at(f0);
              if (fb < 0) {
                err = "refluxing: the fine cell past a coarse-fine face is not in the fine level";
                return AMG_ELAYOUT;
              }
              const BoxD& Z = DF.boxd[fb];
              RfxFaceD rf;
              memset(&rf, 0, sizeof rf);
              rf.fe = elem(DF, fb, f0, dim);
              rf.fsn = sg * Z.s[d];
              int t[2] = {-1, -1}, k = 0;
              for (int e = 0; e < dim; ++e)
                if (e != d) t[k++] = e;
              rf.ft0 = Z.s[t[0]];
              rf.ft1 = dim == 3 ? Z.s[t[1]] : 0;
              rf.csn = sg * Y.s[d];
              rf.d = d;
              rf.sg = sg;
              X.rfx_face.push_back(rf);
            }
          if (X.rfx_face.size() > nf0) {
            X.rfx_cell.push_back(elem(DC, (int)b, i, dim));
            X.rfx_ptr.push_back((int32_t)X.rfx_face.size());
          }
        }
  }

  // ---- transposes for the adjoint ----
  {
    // AMRCFI: coarse window cell -> (ghost, window cell) pairs
    const size_t ng = X.cfi_dst.size();
    std::vector<std::pair<int64_t, int32_t>> pairs;
    pairs.reserve(ng * nwin);
    for (size_t i = 0; i < ng; ++i)
      for (int m = 0; m < nwin; ++m) pairs.push_back({(int64_t)X.cfi_src[i * nwin + m], (int32_t)(i * nwin + m)});
    std::stable_sort(pairs.begin(), pairs.end(),
                     [](const std::pair<int64_t, int32_t>& a, const std::pair<int64_t, int32_t>& b) {
                       return a.first < b.first;
                     });
    X.cfiT_elem.clear();
    X.cfiT_ptr.assign(1, 0);
    X.cfiT_ent.clear();
    for (size_t k = 0; k < pairs.size(); ++k) {
      if (k == 0 || pairs[k].first != pairs[k - 1].first) {
        if (k) X.cfiT_ptr.push_back((int32_t)k);
        X.cfiT_elem.push_back(pairs[k].first);
      }
      X.cfiT_ent.push_back(pairs[k].second);
    }
    if (!pairs.empty()) X.cfiT_ptr.push_back((int32_t)pairs.size());
    // refluxing: d(correction at coarse cell i) / d(value at element), per
    // target element of each level; the correction is
    // (1/hc) sum_faces [mean_t Ff_t - Fc], fluxes (-v[+2] + 15 v[+1] - 15 v[0]
    // + v[-1]) / 12h along the face normal n
    const double hc = DC.h, hf = DF.h;
    const int nft = dim == 2 ? r : r * r;  // fine faces covering a coarse face
    const double nf = (double)nft;
    std::vector<std::pair<int64_t, std::pair<int32_t, double>>> tc, tf;
    const int cw[4] = {1, -15, 15, -1};  // offsets -1, 0, 1, 2 along n
    for (size_t i = 0; i + 1 < X.rfx_ptr.size(); ++i) {
      const int64_t c = X.rfx_cell[i];
      for (int k = X.rfx_ptr[i]; k < X.rfx_ptr[i + 1]; ++k) {
        const RfxFaceD& F = X.rfx_face[k];
        for (int o = 0; o < 4; ++o)
          tc.push_back({c + (int64_t)(o - 1) * F.csn, {(int32_t)i, -cw[o] / (12.0 * hc * hc)}});
        for (int t = 0; t < nft; ++t) {
          const int64_t e = F.fe + (int64_t)(t % r) * F.ft0 + (int64_t)(t / r) * F.ft1;
          // fine flux at the face: offsets -2, -1, 0, 1 from e along n
          for (int o = 0; o < 4; ++o)
            tf.push_back({e + (int64_t)(o - 2) * F.fsn, {(int32_t)i, cw[o] / (12.0 * hf * hc * nf)}});
        }
      }
    }
    auto build = [](std::vector<std::pair<int64_t, std::pair<int32_t, double>>>& v, std::vector<int64_t>& elem,
                    std::vector<int32_t>& ptr, std::vector<int32_t>& src, std::vector<double>& coef) {
      std::stable_sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
      elem.clear();
      ptr.assign(1, 0);
      src.clear();
      coef.clear();
      for (size_t k = 0; k < v.size(); ++k) {
        if (k == 0 || v[k].first != v[k - 1].first) {
          if (k) ptr.push_back((int32_t)k);
          elem.push_back(v[k].first);
        }
        src.push_back(v[k].second.first);
        coef.push_back(v[k].second.second);
      }
      if (!v.empty()) ptr.push_back((int32_t)v.size());
    };
    build(tc, X.rfxTc_elem, X.rfxTc_ptr, X.rfxTc_src, X.rfxTc_coef);
    build(tf, X.rfxTf_elem, X.rfxTf_ptr, X.rfxTf_src, X.rfxTf_coef);
    // refluxing of the divergence: the correction at coarse cell i is
    // (sg / hc) sum over its faces normal to d of [mean_t Ff_t - Fc], face
    // averages (-v[+2] + 7 v[+1] + 7 v[0] - v[-1]) / 12 along n
    const int vw[4] = {-1, 7, 7, -1};  // offsets -1, 0, 1, 2 along n
    for (int d = 0; d < dim; ++d) {
      std::vector<std::pair<int64_t, std::pair<int32_t, double>>> vc, vf;
      for (size_t i = 0; i + 1 < X.rfx_ptr.size(); ++i) {
        const int64_t c = X.rfx_cell[i];
        for (int k = X.rfx_ptr[i]; k < X.rfx_ptr[i + 1]; ++k) {
          const RfxFaceD& F = X.rfx_face[k];
          if (F.d != d) continue;
          for (int o = 0; o < 4; ++o)
            vc.push_back({c + (int64_t)(o - 1) * F.csn, {(int32_t)i, -F.sg * vw[o] / (12.0 * hc)}});
          for (int t = 0; t < nft; ++t) {
            const int64_t e = F.fe + (int64_t)(t % r) * F.ft0 + (int64_t)(t / r) * F.ft1;
            for (int o = 0; o < 4; ++o)
              vf.push_back({e + (int64_t)(o - 2) * F.fsn, {(int32_t)i, F.sg * vw[o] / (12.0 * hc * nf)}});
          }
        }
      }
      build(vc, X.rfxVc[d].elem, X.rfxVc[d].ptr, X.rfxVc[d].src, X.rfxVc[d].coef);
      build(vf, X.rfxVf[d].elem, X.rfxVf[d].ptr, X.rfxVf[d].src, X.rfxVf[d].coef);
    }
  }

  // ---- prolongation of a level-(l-1) correction onto level l ----
  X.pro.clear();
  for (size_t b = 0; b < DF.boxes.size(); ++b) {
    const Box& B = DF.boxes[b];
    int g[3];
    for (g[2] = B.lo[2]; g[2] <= B.hi[2]; ++g[2])
      for (g[1] = B.lo[1]; g[1] <= B.hi[1]; ++g[1])
        for (g[0] = B.lo[0]; g[0] <= B.hi[0]; ++g[0]) {
          int p[3] = {g[0] / r, g[1] / r, dim == 3 ? g[2] / r : 0};
          const int cb = oc.at(p);
          ProlD q;
          memset(&q, 0, sizeof q);
          q.fe = elem(DF, (int)b, g, dim);
          q.pe = elem(DC, cb, p, dim);
          q.cs1 = DC.boxd[cb].s[1];
          q.cs2 = dim == 3 ? DC.boxd[cb].s[2] : 0;
          q.child = (g[0] % r) | ((g[1] % r) << 2) | (dim == 3 ? ((g[2] % r) << 4) : 0);
          X.pro.push_back(q);
        }
  }

  // ---- physical face columns of level l-1 lying under level l ----
  C.face_valid.assign((size_t)std::max<int64_t>(C.nface, 1), 1);
  for (size_t b = 0; b < DC.boxes.size(); ++b) {
    const Box& B = DC.boxes[b];
    for (int d = 0; d < dim; ++d) {
      int t[2] = {-1, -1}, k = 0;
      for (int e = 0; e < dim; ++e)
        if (e != d) t[k++] = e;
      const int n0 = B.n(t[0]);
      const int n1 = dim == 3 ? B.n(t[1]) : 1;
      for (int s = 0; s < 2; ++s)
        for (int q1 = 0; q1 < n1; ++q1)
          for (int q0 = 0; q0 < n0; ++q0) {
            int i[3] = {0, 0, 0};
            i[d] = s ? B.hi[d] : B.lo[d];
            i[t[0]] = B.lo[t[0]] + q0;
            if (dim == 3) i[t[1]] = B.lo[t[1]] + q1;
            if (is_cov(i)) C.face_valid[C.face_off[b * 6 + d * 2 + s] + q0 + (int64_t)n0 * q1] = 0;
          }
    }
  }
  return AMG_OK;
}

int build_cic(amg_hier* H, int l, std::string& err) {
  Level& F = H->levels[l];
  Level& C = H->levels[l - 1];
  CicTable& T = F.cic;
  const int dim = H->dim;
  const int nwin = dim == 2 ? 25 : 125;
  char buf[256];
  const int r = H->ratio;
  cfi_weights(T.w, r);
  const Owner oc = make_owner(H, C, l - 1);
  const Depth& DF = F.depths[0];
  const Depth& DC = C.depths[0];
  T.fd.clear();
  T.src.clear();
  T.wsel.clear();
  T.ncf.assign(F.ncomp, 0.0);
  int64_t gn[3] = {1, 1, 1};  // cells of level l's grid
  for (int d = 0; d < dim; ++d) gn[d] = oc.n[d] * H->ratio;
  for (size_t b = 0; b < DF.boxes.size(); ++b) {
    const Box& B = DF.boxes[b];
    for (int d = 0; d < dim; ++d) {
      int t[2] = {-1, -1}, k = 0;
      for (int e = 0; e < dim; ++e)
        if (e != d) t[k++] = e;
      const int n0 = B.n(t[0]);
      const int n1 = dim == 3 ? B.n(t[1]) : 1;
      for (int s = 0; s < 2; ++s) {
        const int sg = s ? 1 : -1;
        const int p1 = s ? B.hi[d] + 1 : B.lo[d] - 1;
        if (p1 < 0 || p1 >= gn[d]) continue;  // physical face
        const FaceCols& fc = DF.faces[b * 6 + d * 2 + s];
        for (int q1 = 0; q1 < n1; ++q1)
          for (int q0 = 0; q0 < n0; ++q0) {
            const size_t col = (size_t)q0 + (size_t)n0 * q1;
            if (fc.k1[col] != G_FILL_D && fc.k1[col] != G_FILL_N) continue;  // another box of the level
            T.fd.push_back(F.face_off[b * 6 + d * 2 + s] + (int64_t)q0 + (int64_t)n0 * q1);
            T.ncf[DF.boxd[b].comp] += 1.0;
            // the row-end cell and the cells at -1, +1, +2 along the outward normal
            int e0[3] = {0, 0, 0};
            e0[d] = s ? B.hi[d] : B.lo[d];
            e0[t[0]] = B.lo[t[0]] + q0;
            if (dim == 3) e0[t[1]] = B.lo[t[1]] + q1;
            for (int m = -1; m <= 2; ++m) {
              int g[3] = {e0[0], e0[1], e0[2]};
              g[d] += m * sg;
              int lo[3] = {0, 0, 0};
              for (int e = 0; e < dim; ++e) {
                const int P = floordiv(g[e], r);
                const int N = (int)oc.n[e];
                int sh = 0;
                if (P < 2) sh = 2 - P;
                if (P > N - 3) sh = (N - 3) - P;
                lo[e] = P + sh - 2;
                T.wsel.push_back((uint8_t)((sh + 2) * r + (g[e] - r * P)));
              }
              for (int w = 0; w < nwin; ++w) {
                int q[3] = {lo[0] + w % 5, lo[1] + (w / 5) % 5, dim == 3 ? lo[2] + w / 25 : 0};
                const int cb = oc.at(q);
                if (cb < 0) {
                  snprintf(buf, sizeof buf, "interface-condition window of level %d leaves level %d", l, l - 1);
                  err = buf;
                  return AMG_EUNSUPPORTED;
                }
                const int64_t e = elem(DC, cb, q, dim);
                if (e > INT32_MAX) {
                  err = "coarse level too large for 32-bit interpolation indices";
                  return AMG_EUNSUPPORTED;
                }
                T.src.push_back((int32_t)e);
              }
            }
          }
      }
    }
  }
  return AMG_OK;
}

}  // namespace amg
