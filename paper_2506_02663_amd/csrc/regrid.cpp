// Host side of regridding (Section 5.4, RDM-2..4): the clustering of tagged
// cells into boxes (Berger and Rigoutsos 1991, as read below) and the
// construction of the new levels from the tags of the old ones.
//
// New levels: the tags of a level are clustered on its grid coarsened by a
// blocking factor b (a block is tagged when any of its cells is; boxes
// refined by b and clipped), so that every box spans at least b * ratio >= 4
// cells of the new level (the fills need rows of four cells).  RDM-3 grows
// the twice-coarsened boxes of level l+2 by g cells of level l; g * ratio >=
// 3 keeps every five-cell AMRCFI window of level l+2 on level l+1 (the
// paper grows by one cell, enough at ratio 4).
//
// Clustering of a box: shrink it to the bounding box of its tags; accept it
// when tags / cells reaches the efficiency; otherwise cut it in two along
// one direction at an index c (parts [lo, c-1] and [c, hi], each at least
// min_side long along the cut): at a slice without tags closest to the
// box's centre; else at the strongest inflection of the tag signature (the
// largest jump of its second difference between neighbouring slices where
// that difference changes sign); else at the middle of the longest side.
// Ties: closer to the centre, then the lower direction, then the lower
// index.  A box without an admissible cut is accepted; the low part is
// clustered first.  Tags are dense over a grid, x fastest.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../include/amg.h"

namespace {

struct TagGrid {
  int dim;
  int64_t n[3];
  const uint8_t* t;
  bool at(int x, int y, int z) const { return t[x + n[0] * (y + n[1] * (int64_t)z)] != 0; }
};

struct Cluster {
  const TagGrid& G;
  double eff;
  int min_side;
  std::vector<int> out;  // lo[3], hi[3] per box

  // tags per slice along d of the box
  std::vector<int64_t> signature(const int lo[3], const int hi[3], int d) const {
    std::vector<int64_t> sig(hi[d] - lo[d] + 1, 0);
    for (int z = lo[2]; z <= hi[2]; ++z)
      for (int y = lo[1]; y <= hi[1]; ++y)
        for (int x = lo[0]; x <= hi[0]; ++x)
          if (G.at(x, y, z)) {
            const int p[3] = {x, y, z};
            sig[p[d] - lo[d]] += 1;
          }
    return sig;
  }

  bool ok(const int lo[3], const int hi[3], int d, int c) const {
    return c - lo[d] >= min_side && hi[d] + 1 - c >= min_side;
  }

  // the cut (d, c) of a tight box, or false
  bool cut(const int lo[3], const int hi[3], int& bd, int& bc) const {
    const int D = G.dim;
    double centre[3];
    for (int d = 0; d < D; ++d) centre[d] = (lo[d] + hi[d] + 1) / 2.0;
    bool found = false;
    double bdist = 0;
    // holes
    for (int d = 0; d < D; ++d) {
      const std::vector<int64_t> sig = signature(lo, hi, d);
      for (size_t i = 0; i < sig.size(); ++i) {
        const int c = lo[d] + (int)i;
        if (sig[i] != 0 || !ok(lo, hi, d, c)) continue;
        const double dist = std::fabs(c - centre[d]);
        if (!found || dist < bdist || (dist == bdist && (d < bd || (d == bd && c < bc)))) {
          found = true;
          bdist = dist;
          bd = d;
          bc = c;
        }
      }
    }
    if (found) return true;
    // inflections
    int64_t bjump = 0;
    for (int d = 0; d < D; ++d) {
      const std::vector<int64_t> sig = signature(lo, hi, d);
      const int n = (int)sig.size();
      std::vector<int64_t> lap(n, 0);
      for (int i = 1; i + 1 < n; ++i) lap[i] = sig[i - 1] - 2 * sig[i] + sig[i + 1];
      for (int i = 2; i + 1 < n; ++i) {
        const int64_t a = lap[i - 1], b = lap[i];
        if (!((a < 0 && b > 0) || (a > 0 && b < 0))) continue;
        const int c = lo[d] + i;
        if (!ok(lo, hi, d, c)) continue;
        const int64_t jump = b > a ? b - a : a - b;
        const double dist = std::fabs(c - centre[d]);
        if (!found || jump > bjump ||
            (jump == bjump && (dist < bdist || (dist == bdist && (d < bd || (d == bd && c < bc)))))) {
          found = true;
          bjump = jump;
          bdist = dist;
          bd = d;
          bc = c;
        }
      }
    }
    if (found) return true;
    // bisection of the longest side
    int d = 0;
    for (int e = 1; e < D; ++e)
      if (hi[e] - lo[e] > hi[d] - lo[d]) d = e;
    const int c = lo[d] + (hi[d] - lo[d] + 1) / 2;
    if (!ok(lo, hi, d, c)) return false;
    bd = d;
    bc = c;
    return true;
  }

  void rec(const int lo0[3], const int hi0[3]) {
    int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    int64_t count = 0;
    bool any = false;
    for (int z = lo0[2]; z <= hi0[2]; ++z)
      for (int y = lo0[1]; y <= hi0[1]; ++y)
        for (int x = lo0[0]; x <= hi0[0]; ++x)
          if (G.at(x, y, z)) {
            const int p[3] = {x, y, z};
            for (int d = 0; d < 3; ++d) {
              if (!any || p[d] < lo[d]) lo[d] = p[d];
              if (!any || p[d] > hi[d]) hi[d] = p[d];
            }
            any = true;
            ++count;
          }
    if (!any) return;
    double vol = 1;
    for (int d = 0; d < G.dim; ++d) vol *= hi[d] - lo[d] + 1;
    int d = 0, c = 0;
    if ((double)count >= eff * vol || !cut(lo, hi, d, c)) {
      out.insert(out.end(), lo, lo + 3);
      out.insert(out.end(), hi, hi + 3);
      return;
    }
    int hi1[3] = {hi[0], hi[1], hi[2]}, lo2[3] = {lo[0], lo[1], lo[2]};
    hi1[d] = c - 1;
    lo2[d] = c;
    rec(lo, hi1);
    rec(lo2, hi);
  }
};

std::vector<int> cluster(const TagGrid& G, double eff, int min_side) {
  Cluster C{G, eff, min_side, {}};
  const int lo[3] = {0, 0, 0};
  const int hi[3] = {(int)G.n[0] - 1, (int)G.n[1] - 1, (int)G.n[2] - 1};
  C.rec(lo, hi);
  return C.out;
}

int write_boxes(const std::vector<int>& b, int dim, int scale, int max_boxes, int32_t* nboxes, int32_t* lo,
                int32_t* hi) {
  const int nb = (int)b.size() / 6;
  *nboxes = nb;
  if (nb > max_boxes) return AMG_EUNSUPPORTED;
  for (int i = 0; i < nb; ++i)
    for (int d = 0; d < dim; ++d) {
      lo[i * dim + d] = b[i * 6 + d] * scale;
      hi[i * dim + d] = (b[i * 6 + 3 + d] + 1) * scale - 1;
    }
  return AMG_OK;
}

bool check_args(int dim, const int32_t* shape, double eff, int min_side, int max_boxes) {
  if ((dim != 2 && dim != 3) || !shape || !(eff > 0 && eff <= 1) || min_side < 1 || max_boxes < 0) return false;
  for (int d = 0; d < dim; ++d)
    if (shape[d] < 1) return false;
  return true;
}

}  // namespace

extern "C" int amg_cluster(int dim, const int32_t* shape, const uint8_t* tags, double efficiency, int min_side,
                           int max_boxes, int32_t* nboxes, int32_t* lo, int32_t* hi) {
  if (!check_args(dim, shape, efficiency, min_side, max_boxes) || !tags || !nboxes || (max_boxes && (!lo || !hi)))
    return AMG_EINVAL;
  TagGrid G{dim, {shape[0], shape[1], dim == 3 ? shape[2] : 1}, tags};
  return write_boxes(cluster(G, efficiency, min_side), dim, 1, max_boxes, nboxes, lo, hi);
}

namespace {

// clustering of the tags of an n-cell grid coarsened by b; boxes refined by
// b and clipped to the grid
std::vector<int> blocked_cluster(int dim, const int64_t n[3], const uint8_t* t, int b, double eff, int min_side) {
  int64_t nb[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) nb[d] = (n[d] + b - 1) / b;
  std::vector<uint8_t> tb((size_t)(nb[0] * nb[1] * nb[2]), 0);
  for (int64_t z = 0; z < n[2]; ++z)
    for (int64_t y = 0; y < n[1]; ++y)
      for (int64_t x = 0; x < n[0]; ++x)
        if (t[x + n[0] * (y + n[1] * z)]) {
          const int64_t bz = dim == 3 ? z / b : 0;
          tb[x / b + nb[0] * (y / b + nb[1] * bz)] = 1;
        }
  std::vector<int> c = cluster(TagGrid{dim, {nb[0], nb[1], nb[2]}, tb.data()}, eff, min_side);
  for (size_t i = 0; i < c.size(); i += 6)
    for (int d = 0; d < dim; ++d) {
      c[i + d] *= b;
      c[i + 3 + d] = (int)std::min<int64_t>((int64_t)(c[i + 3 + d] + 1) * b, n[d]) - 1;
    }
  return c;
}

}  // namespace

extern "C" int amg_regrid_boxes(int dim, const int32_t* base_cells, int ratio, int ntag, const uint8_t* const* tags,
                                double efficiency, int min_side, int grow, int block, int max_boxes, int32_t* nboxes,
                                int32_t* lo, int32_t* hi) {
  if (!check_args(dim, base_cells, efficiency, min_side, max_boxes) || (ratio != 2 && ratio != 4) || ntag < 1 ||
      ntag > 15 || !tags || !nboxes || !lo || !hi || grow < 0 || block < 0 || block > 64)
    return AMG_EINVAL;
  const int g = grow ? grow : (3 + ratio - 1) / ratio;   // least g with g * ratio >= 3
  const int b = block ? block : (4 + ratio - 1) / ratio;  // least b with b * ratio >= 4
  for (int l = 0; l < ntag; ++l)
    if (!tags[l]) return AMG_EINVAL;
  // grid of level l: base * ratio^l
  auto grid = [&](int l, int64_t n[3]) {
    for (int d = 0; d < 3; ++d) {
      n[d] = d < dim ? base_cells[d] : 1;
      for (int i = 0; i < l && d < dim; ++i) n[d] *= ratio;
    }
  };
  std::vector<std::vector<int>> nb(ntag + 1);  // boxes of new level l at level l-1 resolution
  {
    int64_t n[3];
    grid(ntag - 1, n);
    nb[ntag] = blocked_cluster(dim, n, tags[ntag - 1], b, efficiency, min_side);
  }
  for (int l = ntag - 2; l >= 0; --l) {
    int64_t n[3];
    grid(l, n);
    std::vector<uint8_t> t(tags[l], tags[l] + n[0] * n[1] * n[2]);
    // boxes of new level l+2 (stored at level l+1 resolution) coarsened to
    // level l and grown by g cells, clipped to the grid
    const std::vector<int>& up = nb[l + 2];
    for (size_t i = 0; i < up.size(); i += 6) {
      int blo[3] = {0, 0, 0}, bhi[3] = {0, 0, 0};
      for (int d = 0; d < dim; ++d) {
        blo[d] = (int)std::max<int64_t>(up[i + d] / ratio - g, 0);
        bhi[d] = (int)std::min<int64_t>(up[i + 3 + d] / ratio + g, n[d] - 1);
      }
      for (int z = blo[2]; z <= bhi[2]; ++z)
        for (int y = blo[1]; y <= bhi[1]; ++y)
          for (int x = blo[0]; x <= bhi[0]; ++x) t[x + n[0] * (y + n[1] * (int64_t)z)] = 1;
    }
    nb[l + 1] = blocked_cluster(dim, n, t.data(), b, efficiency, min_side);
  }
  int rc = AMG_OK;
  for (int l = 1; l <= ntag; ++l) {
    const size_t off = (size_t)(l - 1) * max_boxes * dim;
    const int r2 = write_boxes(nb[l], dim, ratio, max_boxes, nboxes + (l - 1), lo + off, hi + off);
    if (r2 != AMG_OK) rc = r2;
  }
  return rc;
}
