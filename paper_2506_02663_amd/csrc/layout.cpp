// Host planner: validates a level's box layout and builds the tables the
// kernels walk -- box descriptors, ghost-column classification and chunks,
// tiles, component lists -- at every multigrid depth.
//
// Layout rules (Section 5.1): boxes are disjoint rectangles of the level's
// grid, eq. (AMRHier); a level > 0 is properly refined, eq. (pBlock), i.e.
// its corners are multiples of the refinement ratio.  The fills read four
// cells of the row that ends at a face, so every box has at least 4 cells
// per side.  A level is halved for the next multigrid depth while every box
// has even corners and even sides of at least 8 (an isolated box: even sides
// of at least 8) and, with a bottom size B set, while some component (an
// isolated box) has more than B cells.
//
// Periodic directions (the domains of Section 7.3) pair the two sides of the
// grid: a ghost beyond a periodic side is an exchange ghost whose source is
// the cell at its index modulo the grid size, and boxes touching across the
// side are face-connected.  Level 0 covers its grid, so every such source is
// a cell; a finer level may not touch a periodic side.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <numeric>

#include "amg_internal.h"
#include "tiles.h"

namespace amg {

namespace {

int64_t grid_cells(const amg_hier* H, int l, int d) {
  int64_t n = H->base[d];
  for (int i = 0; i < l; ++i) n *= H->ratio;
  return n;
}

bool touch(const Box& a, const Box& b, int dim) {
  // face contact: adjacent along one direction, overlapping with positive
  // extent in all others (corner or edge contact does not connect)
  for (int d = 0; d < dim; ++d) {
    bool adj = (a.hi[d] + 1 == b.lo[d]) || (b.hi[d] + 1 == a.lo[d]);
    if (!adj) continue;
    bool ok = true;
    for (int e = 0; e < dim; ++e) {
      if (e == d) continue;
      if (std::max(a.lo[e], b.lo[e]) > std::min(a.hi[e], b.hi[e])) ok = false;
    }
    if (ok) return true;
  }
  return false;
}

// face contact across a periodic side of direction d (grid size n): a ends
// at the last cell, b starts at cell 0 (or the other way round), overlapping
// with positive extent in all other directions
bool touch_periodic(const Box& a, const Box& b, int dim, int d, int64_t n) {
  if (!((a.hi[d] == n - 1 && b.lo[d] == 0) || (b.hi[d] == n - 1 && a.lo[d] == 0))) return false;
  for (int e = 0; e < dim; ++e)
    if (e != d && std::max(a.lo[e], b.lo[e]) > std::min(a.hi[e], b.hi[e])) return false;
  return true;
}

int64_t wrap(int64_t p, int64_t n) { return ((p % n) + n) % n; }

bool overlap(const Box& a, const Box& b, int dim) {
  for (int d = 0; d < dim; ++d)
    if (std::max(a.lo[d], b.lo[d]) > std::min(a.hi[d], b.hi[d])) return false;
  return true;
}

int find(std::vector<int>& p, int x) {
  while (p[x] != x) x = p[x] = p[p[x]];
  return x;
}

// transverse directions of face d, in increasing order
void transverse(int dim, int d, int t[2]) {
  int k = 0;
  t[0] = t[1] = -1;
  for (int e = 0; e < dim; ++e)
    if (e != d) t[k++] = e;
}

}  // namespace

int plan_level(amg_hier* H, int l, std::string& err) {
  Level& L = H->levels[l];
  const int dim = H->dim;
  const int nb = (int)L.boxes.size();
  char buf[256];
  if (nb == 0) {
    err = "level has no boxes";
    return AMG_ELAYOUT;
  }
  int64_t gn[3] = {1, 1, 1};
  for (int d = 0; d < dim; ++d) gn[d] = grid_cells(H, l, d);
  bool per[3] = {false, false, false};
  for (int d = 0; d < dim; ++d) {
    const bool p0 = H->phys_bc[d][0] == AMG_PERIODIC, p1 = H->phys_bc[d][1] == AMG_PERIODIC;
    if (p0 != p1) {
      snprintf(buf, sizeof buf, "direction %d is periodic on one side only", d);
      err = buf;
      return AMG_EINVAL;
    }
    per[d] = p0;
    if (per[d] && L.isolated) {
      err = "isolated boxes with periodic conditions are not supported";
      return AMG_EUNSUPPORTED;
    }
  }

  // ---- validation -----------------------------------------------------------
  int64_t vol = 0;
  for (int b = 0; b < nb; ++b) {
    const Box& B = L.boxes[b];
    int64_t v = 1;
    for (int d = 0; d < dim; ++d) {
      if (B.n(d) < 4) {
        snprintf(buf, sizeof buf, "box %d has %d < 4 cells along direction %d", b, B.n(d), d);
        err = buf;
        return AMG_ELAYOUT;
      }
      if (!L.isolated && (B.lo[d] < 0 || B.hi[d] >= gn[d])) {
        snprintf(buf, sizeof buf, "box %d leaves the grid of level %d", b, l);
        err = buf;
        return AMG_ELAYOUT;
      }
      if (l > 0 && per[d] && (B.lo[d] == 0 || B.hi[d] == gn[d] - 1)) {
        snprintf(buf, sizeof buf, "box %d of level %d touches the periodic side of direction %d", b, l, d);
        err = buf;
        return AMG_EUNSUPPORTED;
      }
      if (l > 0 && !L.isolated && (B.lo[d] % H->ratio || (B.hi[d] + 1) % H->ratio)) {
        snprintf(buf, sizeof buf, "box %d of level %d is not properly refined (corners not multiples of %d)", b, l,
                 H->ratio);
        err = buf;
        return AMG_ELAYOUT;
      }
      v *= B.n(d);
    }
    vol += v;
  }
  if (!L.isolated) {
    for (int a = 0; a < nb; ++a)
      for (int b = a + 1; b < nb; ++b)
        if (overlap(L.boxes[a], L.boxes[b], dim)) {
          snprintf(buf, sizeof buf, "boxes %d and %d overlap", a, b);
          err = buf;
          return AMG_ELAYOUT;
        }
    if (l == 0) {
      int64_t g = 1;
      for (int d = 0; d < dim; ++d) g *= gn[d];
      if (g != vol) {
        err = "level 0 must cover the whole grid";
        return AMG_ELAYOUT;
      }
    }
    // nesting (Section 5.1): the parents of every cell of level l are cells
    // of level l-1, i.e. each coarsened box is covered by the (disjoint)
    // boxes of level l-1
    if (l > 0 && !H->levels[l - 1].isolated) {
      const std::vector<Box>& CB = H->levels[l - 1].boxes;
      for (int b = 0; b < nb; ++b) {
        Box P;
        int64_t need = 1, got = 0;
        for (int d = 0; d < 3; ++d) {
          P.lo[d] = d < dim ? L.boxes[b].lo[d] / H->ratio : 0;
          P.hi[d] = d < dim ? (L.boxes[b].hi[d] + 1) / H->ratio - 1 : 0;
          if (d < dim) need *= P.n(d);
        }
        for (const Box& Q : CB) {
          int64_t v = 1;
          for (int d = 0; d < dim; ++d) v *= std::max(0, std::min(P.hi[d], Q.hi[d]) - std::max(P.lo[d], Q.lo[d]) + 1);
          got += v;
        }
        if (got != need) {
          snprintf(buf, sizeof buf, "level %d is not nested in level %d (box %d)", l, l - 1, b);
          err = buf;
          return AMG_ELAYOUT;
        }
      }
    }
  }
  L.ncells = vol;

  // ---- components (union-find over face contact) ------------------------------
  std::vector<int> par(nb);
  std::iota(par.begin(), par.end(), 0);
  if (!L.isolated)
    for (int a = 0; a < nb; ++a)
      for (int b = a + 1; b < nb; ++b)
        if (touch(L.boxes[a], L.boxes[b], dim)) par[find(par, a)] = find(par, b);
  for (int d = 0; d < dim; ++d)
    if (per[d])
      for (int a = 0; a < nb; ++a)
        for (int b = a + 1; b < nb; ++b)
          if (touch_periodic(L.boxes[a], L.boxes[b], dim, d, gn[d])) par[find(par, a)] = find(par, b);
  std::vector<int> root_id(nb, -1);
  L.box_comp.assign(nb, 0);
  L.ncomp = 0;
  for (int b = 0; b < nb; ++b) {
    int r = find(par, b);
    if (root_id[r] < 0) root_id[r] = L.ncomp++;
    L.box_comp[b] = root_id[r];
  }

  // ---- multigrid depths ---------------------------------------------------------
  std::vector<int> bottom(nb, 0);
  if (L.isolated) {
    for (int b = 0; b < nb; ++b) {
      int n[3] = {L.boxes[b].n(0), L.boxes[b].n(1), dim == 3 ? L.boxes[b].n(2) : 8};
      int k = 0;
      while (true) {
        bool ok = true;
        for (int d = 0; d < dim; ++d)
          if ((n[d] >> k) % 2 || (n[d] >> k) < 8) ok = false;
        if (ok && H->bottom_cells > 0) {  // small enough for the exact solve
          int64_t cells = 1;
          for (int d = 0; d < dim; ++d) cells *= n[d] >> k;
          if (cells <= H->bottom_cells) ok = false;
        }
        if (!ok) break;
        ++k;
      }
      bottom[b] = k;
    }
  } else {
    int k = 0;
    while (true) {
      bool ok = true;
      for (int d = 0; d < dim; ++d)
        if ((gn[d] >> k) % 2) ok = false;
      for (int b = 0; b < nb && ok; ++b)
        for (int d = 0; d < dim; ++d) {
          int lo = L.boxes[b].lo[d] >> k, n = L.boxes[b].n(d) >> k;
          if (lo % 2 || n % 2 || n < 8) ok = false;
        }
      // boxes facing each other across a gap must stay two cells apart
      // after halving, or the radius-2 stencil would couple them directly
      for (int a = 0; a < nb && ok; ++a)
        for (int b = a + 1; b < nb && ok; ++b)
          for (int d = 0; d < dim && ok; ++d) {
            bool facing = true;
            for (int e = 0; e < dim; ++e)
              if (e != d && std::max(L.boxes[a].lo[e], L.boxes[b].lo[e]) > std::min(L.boxes[a].hi[e], L.boxes[b].hi[e]))
                facing = false;
            if (!facing) continue;
            int gap = std::max(L.boxes[b].lo[d] - L.boxes[a].hi[d] - 1, L.boxes[a].lo[d] - L.boxes[b].hi[d] - 1) >> k;
            if (gap > 0 && gap < 4) ok = false;
          }
      if (ok && H->bottom_cells > 0) {  // every component small enough for the exact solve
        std::vector<int64_t> cc(L.ncomp, 0);
        for (int b = 0; b < nb; ++b) {
          int64_t v = 1;
          for (int d = 0; d < dim; ++d) v *= L.boxes[b].n(d) >> k;
          cc[L.box_comp[b]] += v;
        }
        if (*std::max_element(cc.begin(), cc.end()) <= H->bottom_cells) ok = false;
      }
      if (!ok) break;
      ++k;
    }
    std::fill(bottom.begin(), bottom.end(), k);
  }
  const int ndepth = 1 + *std::max_element(bottom.begin(), bottom.end());
  L.depths.assign(ndepth, Depth());

  const int gk1 = (L.cf_mode == AMG_CF_DIRICHLET) ? G_FILL_D : (L.cf_mode == AMG_CF_NEUMANN) ? G_FILL_N : G_ZERO;

  // face-data layout (depth 0 only)
  L.face_off.assign((size_t)nb * 6, -1);
  L.nface = 0;
  for (int b = 0; b < nb; ++b)
    for (int d = 0; d < dim; ++d)
      for (int s = 0; s < 2; ++s) {
        int t[2];
        transverse(dim, d, t);
        int64_t area = 1;
        for (int q = 0; q < dim - 1; ++q) area *= L.boxes[b].n(t[q]);
        L.face_off[b * 6 + d * 2 + s] = L.nface;
        L.nface += area;
      }

  std::vector<int> prev_index(nb, -1);  // box b's index at the previous depth
  for (int k = 0; k < ndepth; ++k) {
    Depth& D = L.depths[k];
    D.h = H->h0;
    for (int i = 0; i < l; ++i) D.h /= H->ratio;
    for (int i = 0; i < k; ++i) D.h *= 2;
    std::vector<int> cur_index(nb, -1);
    for (int b = 0; b < nb; ++b) {
      if (bottom[b] < k) continue;
      Box B;
      for (int d = 0; d < 3; ++d) {
        if (d < dim) {
          B.lo[d] = L.isolated ? 0 : (L.boxes[b].lo[d] >> k);
          B.hi[d] = B.lo[d] + (L.boxes[b].n(d) >> k) - 1;
        } else {
          B.lo[d] = B.hi[d] = 0;
        }
      }
      cur_index[b] = (int)D.boxes.size();
      D.boxes.push_back(B);
      D.level_box.push_back(b);
      if (bottom[b] == k) D.bottom_boxes.push_back(cur_index[b]);
    }
    const int nbk = (int)D.boxes.size();
    // storage: each box with two ghost layers, x fastest, box starts aligned to 64 elements
    D.boxd.resize(nbk);
    int64_t off = 0;
    for (int i = 0; i < nbk; ++i) {
      const Box& B = D.boxes[i];
      BoxD& X = D.boxd[i];
      memset(&X, 0, sizeof X);
      // rows padded to a multiple of A elements and the first interior cell
      // of every row placed on an A-element boundary (aligned row loads)
      const int64_t A = std::max(1, H->row_align);
      int64_t sx = ((B.n(0) + 4 + A - 1) / A) * A, sy = B.n(1) + 4;
      int64_t sz = dim == 3 ? B.n(2) + 4 : 1;
      off = ((off + 2 + A - 1) / A) * A - 2;
      X.off = off;
      X.n[0] = B.n(0);
      X.n[1] = B.n(1);
      X.n[2] = dim == 3 ? B.n(2) : 1;
      X.s[0] = 1;
      X.s[1] = (int32_t)sx;
      X.s[2] = (int32_t)(sx * sy);
      for (int d = 0; d < 3; ++d) X.lo[d] = B.lo[d];
      X.comp = L.box_comp[D.level_box[i]];
      X.fine = k > 0 ? prev_index[D.level_box[i]] : -1;
      X.coarse = -1;
      off += sx * sy * sz;
    }
    D.nstored = off + 64;
    if (k > 0) {
      Depth& F = L.depths[k - 1];
      for (int i = 0; i < nbk; ++i) F.boxd[D.boxd[i].fine].coarse = i;
    }
    // domain at this depth
    int64_t dn[3] = {1, 1, 1};
    for (int d = 0; d < dim; ++d) dn[d] = gn[d] >> k;
    for (int d = 0; d < 3; ++d) {
      D.dn[d] = (int32_t)dn[d];
      D.periodic[d] = per[d];
    }
    D.wrap = false;
    for (BoxD& X : D.boxd)
      for (int d = 0; d < dim; ++d)
        if (per[d] && X.n[d] == dn[d]) {
          X.wrap |= (uint8_t)(1 << d);
          D.wrap = true;
        }

    // ---- ghost-column classification ----
    D.faces.assign((size_t)nbk * 6, FaceCols());
    for (int i = 0; i < nbk; ++i) {
      const Box& B = D.boxes[i];
      for (int d = 0; d < dim; ++d) {
        int t[2];
        transverse(dim, d, t);
        int n0 = t[0] >= 0 ? B.n(t[0]) : 1;
        int n1 = (dim == 3) ? B.n(t[1]) : 1;
        for (int s = 0; s < 2; ++s) {
          FaceCols& fc = D.faces[i * 6 + d * 2 + s];
          size_t area = (size_t)n0 * n1;
          int p1 = s ? B.hi[d] + 1 : B.lo[d] - 1;
          bool phys = L.isolated ? true : ((p1 < 0 || p1 >= dn[d]) && !per[d]);
          uint8_t kk = phys ? ((H->phys_bc[d][s] == AMG_DIRICHLET) ? G_FILL_D : G_FILL_N) : gk1;
          fc.k1.assign(area, kk);
          fc.k2.assign(area, kk);
          fc.src1.assign(area, -1);
          fc.src2.assign(area, -1);
          if (L.isolated || phys) continue;
          for (int layer = 1; layer <= 2; ++layer) {
            int p = s ? B.hi[d] + layer : B.lo[d] - layer;
            const bool wrapped = p < 0 || p >= dn[d];  // beyond a periodic side
            if (wrapped) p = (int)wrap(p, dn[d]);
            for (int j = 0; j < nbk; ++j) {
              if (j == i && !wrapped) continue;
              const Box& C = D.boxes[j];
              if (p < C.lo[d] || p > C.hi[d]) continue;
              int a0 = std::max(B.lo[t[0]], C.lo[t[0]]), b0 = std::min(B.hi[t[0]], C.hi[t[0]]);
              if (a0 > b0) continue;
              int a1 = 0, b1 = 0;
              if (dim == 3) {
                a1 = std::max(B.lo[t[1]], C.lo[t[1]]);
                b1 = std::min(B.hi[t[1]], C.hi[t[1]]);
                if (a1 > b1) continue;
              }
              for (int q1 = a1; q1 <= b1; ++q1)
                for (int q0 = a0; q0 <= b0; ++q0) {
                  size_t col = (size_t)(q0 - B.lo[t[0]]) + (size_t)n0 * (dim == 3 ? (q1 - B.lo[t[1]]) : 0);
                  if (layer == 1) {
                    fc.k1[col] = G_EXCH;
                    fc.src1[col] = j;
                  } else {
                    fc.k2[col] = G_EXCH;
                    fc.src2[col] = j;
                  }
                }
            }
          }
        }
      }
    }
    // column codes
    D.codes.clear();
    for (int i = 0; i < nbk; ++i)
      for (int d = 0; d < 3; ++d)
        for (int s = 0; s < 2; ++s) {
          if (d >= dim) {
            D.boxd[i].code_off[d][s] = 0;
            continue;
          }
          FaceCols& fc = D.faces[i * 6 + d * 2 + s];
          D.boxd[i].code_off[d][s] = (int32_t)D.codes.size();
          uint8_t u0 = stored_code(fc.k1[0], fc.k2[0], fc.src1[0] == i);
          for (size_t c = 0; c < fc.k1.size(); ++c) {
            const uint8_t cc = stored_code(fc.k1[c], fc.k2[c], fc.src1[c] == i);
            D.codes.push_back(cc);
            if (cc != u0) u0 = 0xFF;
          }
          D.boxd[i].ucode[d][s] = u0;
        }
    if (D.codes.empty()) D.codes.push_back(0);
    D.xsrc.assign(2 * D.codes.size(), -1);

    // ---- band of the transposed fill: 4-deep slabs of faces with filled columns ----
    D.band.clear();
    for (int i = 0; i < nbk; ++i) {
      const Box& B = D.boxes[i];
      int fmask = 0;
      for (int d = 0; d < dim; ++d)
        for (int s = 0; s < 2; ++s) {
          const FaceCols& fc = D.faces[i * 6 + d * 2 + s];
          for (size_t c = 0; c < fc.k1.size(); ++c)
            if (column_code(fc.k1[c], fc.k2[c]) & 3) {
              fmask |= 1 << (d * 2 + s);
              break;
            }
        }
      for (int f = 0; f < 2 * dim; ++f) {
        if (!((fmask >> f) & 1)) continue;
        int64_t cells = 4;
        for (int e = 0; e < dim; ++e)
          if (e != f / 2) cells *= B.n(e);
        for (int64_t k = 0; k < cells; k += 256)
          D.band.push_back(BandChunkD{i, f, (int32_t)k, (int32_t)std::min<int64_t>(256, cells - k), fmask, 0});
      }
    }

    // ---- ghost chunks ----
    auto addr = [&](int box, int x, int y, int z) -> int64_t {  // global index -> element
      const BoxD& X = D.boxd[box];
      const Box& B = D.boxes[box];
      int64_t a = X.off + (int64_t)(x - B.lo[0] + 2) * X.s[0] + (int64_t)(y - B.lo[1] + 2) * X.s[1];
      if (dim == 3) a += (int64_t)(z - B.lo[2] + 2) * X.s[2];
      return a;
    };
    D.chunks.clear();
    std::vector<std::vector<int32_t>> comp_chunks(L.ncomp);
    for (int i = 0; i < nbk; ++i) {
      const Box& B = D.boxes[i];
      for (int d = 0; d < dim; ++d) {
        int t[2];
        transverse(dim, d, t);
        int n0 = B.n(t[0]);
        int n1 = (dim == 3) ? B.n(t[1]) : 1;
        for (int s = 0; s < 2; ++s) {
          FaceCols& fc = D.faces[i * 6 + d * 2 + s];
          int step = s ? 1 : -1;
          for (int q1 = 0; q1 < n1; ++q1) {
            int q0 = 0;
            while (q0 < n0) {
              size_t col = (size_t)q0 + (size_t)n0 * q1;
              int q = q0 + 1;
              while (q < n0 && q - q0 < 64) {
                size_t c2 = (size_t)q + (size_t)n0 * q1;
                if (fc.k1[c2] != fc.k1[col] || fc.k2[c2] != fc.k2[col] || fc.src1[c2] != fc.src1[col] ||
                    fc.src2[c2] != fc.src2[col])
                  break;
                ++q;
              }
              ChunkD ch;
              memset(&ch, 0, sizeof ch);
              int g[3] = {0, 0, 0};  // global index of the layer-1 ghost of the first column
              g[d] = s ? B.hi[d] + 1 : B.lo[d] - 1;
              g[t[0]] = B.lo[t[0]] + q0;
              if (dim == 3) g[t[1]] = B.lo[t[1]] + q1;
              ch.dst = addr(i, g[0], g[1], g[2]);
              ch.cstride = D.boxd[i].s[t[0]];
              ch.nstride = step * D.boxd[i].s[d];
              ch.dir = (uint8_t)d;
              ch.count = q - q0;
              ch.box = i;
              ch.kind1 = fc.k1[col];
              ch.kind2 = fc.k2[col];
              ch.src1 = ch.src2 = -1;
              if (fc.src1[col] >= 0) {
                int g1[3] = {g[0], g[1], g[2]};
                g1[d] = (int)wrap(g1[d], dn[d]);
                ch.src1 = addr(fc.src1[col], g1[0], g1[1], g1[2]);
                ch.sstride1 = D.boxd[fc.src1[col]].s[t[0]];
              }
              if (fc.src2[col] >= 0) {
                int g2[3] = {g[0], g[1], g[2]};
                g2[d] = (int)wrap(g2[d] + step, dn[d]);
                ch.src2 = addr(fc.src2[col], g2[0], g2[1], g2[2]);
                ch.sstride2 = D.boxd[fc.src2[col]].s[t[0]];
              }
              {
                const int p1 = s ? B.hi[d] + 1 : B.lo[d] - 1;
                ch.cf = (!L.isolated && p1 >= 0 && p1 < dn[d]) ? 1 : 0;
              }
              // the sources of exchange columns, for the sweeps' read-time fill
              for (int l = 0; l < ch.count; ++l) {
                const size_t pos = (size_t)D.boxd[i].code_off[d][s] + (size_t)(q0 + l) + (size_t)n0 * q1;
                if (D.codes[pos] != kCodeExch) continue;
                D.xsrc[2 * pos] = ch.src1 + (int64_t)l * ch.sstride1;
                D.xsrc[2 * pos + 1] = ch.src2 + (int64_t)l * ch.sstride2;
              }
              ch.fd = -1;
              if (k == 0 && (ch.kind1 == G_FILL_D || ch.kind1 == G_FILL_N))
                ch.fd = L.face_off[D.level_box[i] * 6 + d * 2 + s] + (int64_t)q0 + (int64_t)n0 * q1;
              comp_chunks[D.boxd[i].comp].push_back((int32_t)D.chunks.size());
              D.chunks.push_back(ch);
              q0 = q;
            }
          }
        }
      }
    }
    D.chunk_comp_ptr.assign(1, 0);
    D.chunk_comp_idx.clear();
    for (int c = 0; c < L.ncomp; ++c) {
      D.chunk_comp_idx.insert(D.chunk_comp_idx.end(), comp_chunks[c].begin(), comp_chunks[c].end());
      D.chunk_comp_ptr.push_back((int32_t)D.chunk_comp_idx.size());
    }

    // (the FP32 sweeps form the ghosts they read: filled columns from their
    // rows, a face that wraps onto its own box from the box's other end,
    // exchange columns from their sources, zero columns as zero)
    // every exchange code has its sources (else the column keeps its ghosts
    // in memory and the fill launch stays)
    bool sources = true;
    for (size_t pos = 0; pos < D.codes.size(); ++pos)
      if (D.codes[pos] == kCodeExch && (D.xsrc[2 * pos] < 0 || D.xsrc[2 * pos + 1] < 0)) {
        D.codes[pos] = 0;
        sources = false;
      }
    D.fill_only = sources;
    D.xfill = false;
    for (uint8_t c : D.codes)
      if (c & (kCodeExch | kCodeZero)) D.xfill = true;
    for (const ChunkD& ch : D.chunks) {
      const bool filled =
          (ch.kind1 == G_FILL_D || ch.kind1 == G_FILL_N) && (ch.kind2 == G_FILL_D || ch.kind2 == G_FILL_N);
      const bool exch = ch.kind1 == G_EXCH && ch.kind2 == G_EXCH;
      const bool zero = ch.kind1 == G_ZERO && ch.kind2 == G_ZERO;
      if (!filled && !exch && !zero) D.fill_only = false;
    }

    // ---- tiles (grouped by component, so each component is one range) ----
    D.tiles.clear();
    D.stiles.clear();
    // march length of this depth: long marches amortise each column's set-up,
    // but a depth must still give about kTargetTiles tiles to fill the chip;
    // always even, so restriction pairs never straddle two tiles
    int CH;
    {
      int64_t R = 0;  // tile rows: (x-tiles x y-tiles) x cells along the march direction
      for (int i = 0; i < nbk; ++i) {
        const BoxD& X = D.boxd[i];
        const int64_t base = (int64_t)((X.n[0] + TILE_X - 1) / TILE_X) * (dim == 3 ? (X.n[1] + TILE3_Y - 1) / TILE3_Y : 1);
        R += base * X.n[dim - 1];
      }
      const int cap = dim == 2 ? H->march2 : H->march3;
      int64_t m = R / kTargetTiles;
      m = std::max<int64_t>(2, std::min<int64_t>(cap, m));
      CH = (int)(m & ~int64_t(1));
    }
    D.march = CH;
    D.comp_seg_ptr.assign(1, 0);
    D.seg_ptr.assign(1, 0);
    for (int c = 0; c < L.ncomp; ++c) {
      const size_t first = D.tiles.size();
      for (int i = 0; i < nbk; ++i) {
        const BoxD& X = D.boxd[i];
        if (X.comp != c) continue;
        bool smooths = bottom[D.level_box[i]] > k;
        auto add = [&](int x0, int y0, int z0, int len) {
          TileD T;
          memset(&T, 0, sizeof T);
          T.box = i;
          T.x0 = x0;
          T.y0 = y0;
          T.z0 = z0;
          T.len = len;
          D.tiles.push_back(T);
          if (smooths) D.stiles.push_back(T);
        };
        if (dim == 2) {
          for (int y0 = 0; y0 < X.n[1]; y0 += CH)
            for (int x0 = 0; x0 < X.n[0]; x0 += TILE_X) add(x0, y0, 0, std::min(CH, X.n[1] - y0));
        } else {
          for (int z0 = 0; z0 < X.n[2]; z0 += CH)
            for (int y0 = 0; y0 < X.n[1]; y0 += TILE3_Y)
              for (int x0 = 0; x0 < X.n[0]; x0 += TILE_X) add(x0, y0, z0, std::min(CH, X.n[2] - z0));
        }
      }
      // reduction segments of at most kSeg tiles inside the component
      for (size_t a = first; a < D.tiles.size(); a += kSeg)
        D.seg_ptr.push_back((int32_t)std::min(D.tiles.size(), a + kSeg));
      D.comp_seg_ptr.push_back((int32_t)D.seg_ptr.size() - 1);
    }
    D.uniform_fill = D.fill_only;
    for (const BoxD& X : D.boxd)
      for (int d = 0; d < dim; ++d)
        for (int s = 0; s < 2; ++s)
          if (X.ucode[d][s] != 5 && X.ucode[d][s] != 6) D.uniform_fill = false;
    D.wrap_fill = D.fill_only;
    for (const BoxD& X : D.boxd)
      for (int d = 0; d < dim; ++d)
        for (int s = 0; s < 2; ++s)
          if (((X.wrap >> d) & 1) ? X.ucode[d][s] != 0 : (X.ucode[d][s] != 5 && X.ucode[d][s] != 6))
            D.wrap_fill = false;
    // colour-split storage (depth 0): every face filled uniformly with
    // both layers from its own row (the sweep computes all ghosts it reads),
    // even offsets, row lengths and plane sizes (each aligned pair of
    // elements holds one cell of each colour) and rows of an even number of
    // cells (a tile's columns pair up)
    // no box solved exactly at this depth (the bottom solve writes interleaved)
    bool split_ok = H->split_rb && k == 0 && D.fill_only && !D.stiles.empty() && D.bottom_boxes.empty() &&
                    (D.nstored % 2) == 0;
    for (const BoxD& X : D.boxd) {
      for (int d = 0; d < dim; ++d)
        for (int s = 0; s < 2; ++s)
          if (X.ucode[d][s] != 5 && X.ucode[d][s] != 6) split_ok = false;
      // even sizes (true of every box that is smoothed, since it coarsens)
      // with an even march give every last tile of a row, column or march at
      // least 2 cells, so no tile's stencil reaches a ghost another tile writes
      if ((X.off % 2) != 0 || (X.s[1] % 2) != 0 || (X.s[2] % 2) != 0 || (X.n[0] % 2) != 0 || (X.n[1] % 2) != 0 ||
          (dim == 3 && (X.n[2] % 2) != 0))
        split_ok = false;
    }
    D.split_rb = split_ok;
    D.nxg = 0;
    if (split_ok)
      for (BoxD& X : D.boxd) {
        X.xg = D.nxg;
        D.nxg += 4 * (int64_t)X.n[1] * X.n[2];
      }
    prev_index = cur_index;
  }

  // ---- singular components (Poisson, no Dirichlet-type column at depth 0) -----
  L.comp_singular.assign(L.ncomp, 0);
  L.comp_cells.assign(L.ncomp, 0);
  for (int b = 0; b < nb; ++b) {
    int64_t v = 1;
    for (int d = 0; d < dim; ++d) v *= L.boxes[b].n(d);
    L.comp_cells[L.box_comp[b]] += v;
  }
  if (H->op == AMG_POISSON) {
    std::vector<int> has_dir(L.ncomp, 0);
    Depth& D0 = L.depths[0];
    for (size_t i = 0; i < D0.boxes.size(); ++i)
      for (int d = 0; d < dim; ++d)
        for (int s = 0; s < 2; ++s) {
          const FaceCols& fc = D0.faces[i * 6 + d * 2 + s];
          for (size_t c = 0; c < fc.k1.size(); ++c)
            if (fc.k1[c] == G_FILL_D || fc.k1[c] == G_ZERO) has_dir[D0.boxd[i].comp] = 1;
        }
    for (int c = 0; c < L.ncomp; ++c) L.comp_singular[c] = !has_dir[c];
  }
  L.nsingular = (int)std::count(L.comp_singular.begin(), L.comp_singular.end(), 1);
  // exchange transpose at depth 0: every source cell with the ghost slots
  // that copy it
  {
    Depth& D0 = L.depths[0];
    std::vector<std::pair<int64_t, int64_t>> pairs;
    for (const ChunkD& ch : D0.chunks)
      for (int lane = 0; lane < ch.count; ++lane) {
        const int64_t g1 = ch.dst + (int64_t)lane * ch.cstride;
        if (ch.kind1 == G_EXCH) pairs.push_back({ch.src1 + (int64_t)lane * ch.sstride1, g1});
        if (ch.kind2 == G_EXCH) pairs.push_back({ch.src2 + (int64_t)lane * ch.sstride2, g1 + ch.nstride});
      }
    std::stable_sort(pairs.begin(), pairs.end(),
                     [](const std::pair<int64_t, int64_t>& a, const std::pair<int64_t, int64_t>& b) {
                       return a.first < b.first;
                     });
    D0.exT_elem.clear();
    D0.exT_slot.clear();
    D0.exT_ptr.assign(1, 0);
    for (size_t k = 0; k < pairs.size(); ++k) {
      if (k == 0 || pairs[k].first != pairs[k - 1].first) {
        if (k) D0.exT_ptr.push_back((int32_t)k);
        D0.exT_elem.push_back(pairs[k].first);
      }
      D0.exT_slot.push_back(pairs[k].second);
    }
    if (!pairs.empty()) D0.exT_ptr.push_back((int32_t)pairs.size());
  }
  L.comp_ncf.assign(L.ncomp, 0.0);
  for (const ChunkD& ch : L.depths[0].chunks)
    if (ch.cf && ch.kind1 == G_FILL_N && ch.fd >= 0) L.comp_ncf[L.depths[0].boxd[ch.box].comp] += ch.count;
  return AMG_OK;
}

}  // namespace amg
