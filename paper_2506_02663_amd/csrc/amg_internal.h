// Internal structures of the multigrid library: the tables the host planner
// builds once per layout and the kernels walk.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/amg.h"
#include "tiles.h"

namespace amg {

// ---- ghost kinds (per ghost layer of a face column) -------------------------
// FILL_D / FILL_N: fifth-order fill from the row that ends at the face, eqs.
// (velBCHomoDiri5th) / (Neumann5), with the face datum of that column.
// EXCH: the ghost lies in another box of the same level; copy its value.
// ZERO: coarse-fine interpolated ghost of a correction (homogeneous: 0).
enum GhostKind : uint8_t { G_ZERO = 0, G_FILL_D = 1, G_FILL_N = 2, G_EXCH = 3 };

// Column code read by the stencil kernels to fold the fill into the diagonal:
// bits 0-1 = fill kind of layer 1 (0 none, 1 Dirichlet, 2 Neumann), bit 2 =
// layer 2 is filled from the same row end.
inline uint8_t column_code(uint8_t k1, uint8_t k2) {
  uint8_t c = (k1 == G_FILL_D) ? 1 : (k1 == G_FILL_N) ? 2 : 0;
  if (c && k2 == k1) c |= 4;
  return c;
}

// Further bits of the stored column code, for the FP32 sweeps that form
// their ghosts where they read them: kCodeExch, both layers copy cells of
// another box (their elements in Depth::xsrc); kCodeZero, both layers are
// zero (the interpolated ghosts of a correction).  A column that copies
// cells of its own box (a periodic direction the box spans) keeps code 0.
constexpr uint8_t kCodeExch = 8, kCodeZero = 16;
inline uint8_t stored_code(uint8_t k1, uint8_t k2, bool own_box) {
  const uint8_t c = column_code(k1, k2);
  if (c) return c;
  if (k1 == G_EXCH && k2 == G_EXCH && !own_box) return kCodeExch;
  if (k1 == G_ZERO && k2 == G_ZERO) return kCodeZero;
  return 0;
}

struct BoxD {              // one box at one multigrid depth
  int64_t off;             // element offset of the stored corner (ghost -2,-2,-2)
  int32_t n[3];            // interior cells per direction (1 for unused dims)
  int32_t s[3];            // element strides
  int32_t lo[3];           // global lower corner at this depth (colouring)
  int32_t code_off[3][2];  // offset of each face's column codes
  int32_t comp;            // component id
  int32_t fine;            // index of the same box at depth-1 (-1 at depth 0)
  int32_t coarse;          // index at depth+1, -1 if the box ends here
  uint8_t ucode[3][2];     // column code shared by a whole face, 0xFF if the face mixes codes
  uint8_t wrap;            // bit d: direction d is periodic and the box spans the grid, so its ghosts
                           // in d are its own cells at the other end
  uint8_t pad;
  int64_t xg;              // colour-split depths: first element of the box's x-face ghost rows in Depth::xg32
};

struct TileD {             // a column block of one box, marched along the last direction
  int32_t box;
  int32_t x0, y0, z0;      // first cell (2D: y0 is the first row of the march)
  int32_t len;             // cells along the march direction
  int32_t pad[3];
};

struct ChunkD {            // up to 64 consecutive ghost columns of one face
  int64_t dst;             // element of the layer-1 ghost of the first column
  int64_t src1, src2;      // exchange sources of layers 1 and 2 (first column)
  int64_t fd;              // face-data element of the first column (-1: none)
  int32_t cstride;         // element stride between consecutive columns
  int32_t sstride1, sstride2;
  int32_t nstride;         // outward normal stride (elements, signed)
  int32_t count;           // columns in the chunk (<= 64)
  int32_t box;
  uint8_t kind1, kind2;
  uint8_t cf;              // 1: the face is not on the physical boundary
  uint8_t dir;             // direction d of the face normal
  uint8_t pad[4];
};

// Up to 256 cells of the band of one box face that the transposed ghost
// fill touches: the first four cells of every row ending at a face with
// filled (Dirichlet / Neumann) ghost columns.  Cells are numbered within the
// face's 4-deep slab; a cell within reach of several such faces belongs to
// the first of them (faces ordered d * 2 + side).
struct BandChunkD {
  int32_t box;
  int32_t face;   // d * 2 + side
  int32_t start;  // first slab cell of the chunk
  int32_t count;  // cells in the chunk (<= 256)
  int32_t fmask;  // bit f: face f of the box has filled ghost columns
  int32_t pad;
};

constexpr int kSeg = 2048;          // tiles per first-stage reduction segment
constexpr int64_t kTargetTiles = 512;  // tiles a depth should offer the 256 CUs (two each)

struct BottomGroupD {      // systems sharing one dense inverse
  int64_t mat;             // offset of the n x n inverse (column-major) in the matrix pool
  int64_t idx;             // offset of ninst*n element indices in the index pool
  int32_t n, ninst;
  int64_t matT;            // offset of its transpose (column-major) in the matrix pool
  // ILU(0)-GMRES bottom (amg_set_bottom_solver): the N x N system (N = n, or
  // n + 1 with the zero-mean border), K P and P = (L U)^-1 column-major in
  // the matrix pool, and the offset of its instances' Krylov vectors
  int64_t ilub, ilup, ws;
  int32_t N, pad;
};

// ---- composite (multi-level) tables -------------------------------------------
struct AvgD {     // one coarse cell under the finer level
  int64_t ce;     // coarse element
  int64_t fe;     // element of its child with the smallest indices
  int32_t fs1, fs2;  // fine strides along y and z
};

struct RfxFaceD {  // one coarse-fine face of a valid coarse cell
  int64_t fe;      // first fine cell past the face (transverse offset 0)
  int32_t fsn;     // fine stride along the normal n (pointing into the fine level)
  int32_t ft0, ft1;  // fine strides across the face
  int32_t csn;     // coarse stride along n
  int32_t d;       // direction of the normal
  int32_t sg;      // +1: n = +e_d, -1: n = -e_d
};

struct ProlD {     // one fine cell and its coarse parent
  int64_t fe, pe;
  int32_t cs1, cs2;  // coarse strides along y and z
  int32_t child;     // bits 2d..2d+1: the child's offset 0..ratio-1 in its parent along d
  int32_t pad;
};

struct Composite {  // tables of level l against level l-1 (l >= 1)
  int r = 2;        // refinement ratio against level l-1 (2 or 4)
  double w[20][5];  // interpolation weights, [(shift + 2) * r + child][window cell]
  std::vector<int64_t> cfi_dst;
  std::vector<int32_t> cfi_src;  // 5^D coarse elements per ghost
  std::vector<uint8_t> cfi_w;    // D weight-set indices per ghost
  std::vector<AvgD> avg;
  std::vector<int64_t> rfx_cell;  // coarse cells with coarse-fine faces
  std::vector<int32_t> rfx_ptr;   // CSR into rfx_face
  std::vector<RfxFaceD> rfx_face;
  std::vector<ProlD> pro;
  // transposes for the adjoint of the composite operator (gathers in a
  // fixed order): per interpolated ghost its row end, inward stride and layer;
  // AMRCFI by coarse target element; refluxing by target element of level
  // l-1 and of level l (coefficient times the adjoint of the refluxed cell)
  std::vector<int64_t> cfi_e0;
  std::vector<int32_t> cfi_in;
  std::vector<uint8_t> cfi_layer;
  std::vector<int64_t> cfiT_elem;
  std::vector<int32_t> cfiT_ptr, cfiT_ent;  // ent = ghost * 5^D + window cell
  std::vector<int64_t> rfxTc_elem, rfxTf_elem;
  std::vector<int32_t> rfxTc_ptr, rfxTf_ptr, rfxTc_src, rfxTf_src;  // src: index into rfx_cell
  std::vector<double> rfxTc_coef, rfxTf_coef;
  // refluxing of the divergence (face averages of eq. cell2face, first row),
  // transposed like the above, one table per face direction d (the
  // divergence refluxes component d through the faces normal to d)
  struct GatherT {
    std::vector<int64_t> elem;
    std::vector<int32_t> ptr, src;
    std::vector<double> coef;
    int64_t* d_elem = nullptr;
    int32_t *d_ptr = nullptr, *d_src = nullptr;
    double* d_coef = nullptr;
  };
  GatherT rfxVc[3], rfxVf[3];
  // device
  double* d_w = nullptr;
  int64_t* d_cfi_dst = nullptr;
  int32_t* d_cfi_src = nullptr;
  uint8_t* d_cfi_w = nullptr;
  AvgD* d_avg = nullptr;
  int64_t* d_rfx_cell = nullptr;
  int32_t* d_rfx_ptr = nullptr;
  RfxFaceD* d_rfx_face = nullptr;
  ProlD* d_pro = nullptr;
  int64_t* d_cfi_e0 = nullptr;
  int32_t* d_cfi_in = nullptr;
  uint8_t* d_cfi_layer = nullptr;
  int64_t* d_cfiT_elem = nullptr;
  int32_t *d_cfiT_ptr = nullptr, *d_cfiT_ent = nullptr;
  int64_t *d_rfxTc_elem = nullptr, *d_rfxTf_elem = nullptr;
  int32_t *d_rfxTc_ptr = nullptr, *d_rfxTf_ptr = nullptr, *d_rfxTc_src = nullptr, *d_rfxTf_src = nullptr;
  double *d_rfxTc_coef = nullptr, *d_rfxTf_coef = nullptr;
};

// ---- host-side description ---------------------------------------------------
struct Box {
  int lo[3], hi[3];
  int n(int d) const { return hi[d] - lo[d] + 1; }
};

struct FaceCols {          // classification of the ghost columns of one box face
  std::vector<uint8_t> k1, k2;
  std::vector<int32_t> src1, src2;  // source box of layers 1 and 2 (-1 none)
};

struct Depth {
  double h = 0;
  std::vector<Box> boxes;
  std::vector<BoxD> boxd;
  std::vector<int32_t> level_box;    // index of the box at depth 0
  std::vector<FaceCols> faces;       // [box*6 + d*2 + side]
  std::vector<uint8_t> codes;
  std::vector<ChunkD> chunks;
  std::vector<TileD> tiles;          // all boxes at this depth
  std::vector<TileD> stiles;         // boxes that smooth at this depth (not at their bottom)
  std::vector<int32_t> seg_ptr;       // reduction segments: ranges of at most kSeg tiles within one component
  std::vector<int32_t> comp_seg_ptr;  // segments of each component (range into seg_ptr)
  std::vector<int32_t> chunk_comp_ptr, chunk_comp_idx; // CSR: chunks of each component
  std::vector<BandChunkD> band;      // cells the transposed fill touches
  // exchange transpose (depth 0): source element -> ghost slots that copy it
  std::vector<int64_t> exT_elem, exT_slot;
  std::vector<int32_t> exT_ptr;
  int64_t* d_exT_elem = nullptr;
  int64_t* d_exT_slot = nullptr;
  int32_t* d_exT_ptr = nullptr;
  std::vector<int32_t> bottom_boxes; // boxes solved exactly at this depth
  std::vector<BottomGroupD> groups;
  int64_t nstored = 0;
  bool fill_only = false;  // the FP32 sweeps form every ghost they read (fills, wraps, exchanges, zeros)
  bool xfill = false;      // some column has an exchange or zero code (the sweeps' form that reads them)
  bool split_rb = false;   // colour-split storage (k_rbs) applies to this depth
  bool wrap = false;       // some box wraps onto itself in a periodic direction (BoxD::wrap)
  bool wrap_fill = false;  // every face filled uniformly from its own rows (codes 5, 6) or wrapping onto its box
  bool uniform_fill = false;  // every face of every box filled uniformly from its own rows, both ghost layers
  int march = 2;  // cells each tile marches along the last direction
  int32_t dn[3] = {1, 1, 1};  // cells of the grid per direction at this depth
  bool periodic[3] = {false, false, false};
  // exchange sources of the columns with kCodeExch: elements of the cells
  // that ghost layers 1 and 2 copy, at 2 i and 2 i + 1 for the column code i
  std::vector<int64_t> xsrc;
  // device copies
  BoxD* d_box = nullptr;
  uint8_t* d_codes = nullptr;
  int64_t* d_xsrc = nullptr;
  ChunkD* d_chunks = nullptr;
  TileD* d_tiles = nullptr;
  TileD* d_stiles = nullptr;
  int32_t *d_seg = nullptr, *d_cseg = nullptr, *d_cc_ptr = nullptr, *d_cc_idx = nullptr;
  BottomGroupD* d_groups = nullptr;
  BandChunkD* d_band = nullptr;
  // work buffers (FP64 and FP32): correction, right-hand side, second buffer
  double *e64 = nullptr, *f64 = nullptr, *t64 = nullptr;
  float *e32 = nullptr, *f32 = nullptr, *t32 = nullptr;
  float* fs32 = nullptr;  // right-hand side in colour-split storage (depth 0 with split_rb)
  // x-face ghosts of split depths, outside the split halves: per box, rows
  // (y, z) of the low face (2 layers) then of the high face; written by the
  // tiles at the x faces and read by their edge lanes
  float* xg32 = nullptr;
  int64_t nxg = 0;
};

struct GraphCache {  // the captured outer cycle of one level
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int64_t> key;
  std::vector<std::pair<int, size_t>> timed;  // event pairs inside the graph
  bool broken = false;
  void release() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
    key.clear();
    timed.clear();
  }
};

// Coarse-fine interface conditions of a level solved with face data (CIC-1..3
// of Section 6.3): per face-data entry on a coarse-fine face, the four fine
// cells across the face along the outward normal (two inside, two outside)
// and, for each, the 5^D window of coarse cells AMRCFI interpolates it from.
struct CicTable {
  std::vector<int64_t> fd;     // face-data entry
  std::vector<int32_t> src;    // [entry * 4 + cell] * 5^D coarse elements
  std::vector<uint8_t> wsel;   // [entry * 4 + cell] * D weight sets (of Composite::w)
  std::vector<double> ncf;     // coarse-fine face entries per component
  double w[20][5];  // as Composite::w
  int64_t* d_fd = nullptr;
  int32_t* d_src = nullptr;
  uint8_t* d_wsel = nullptr;
  double* d_w = nullptr;
  double* d_ncf = nullptr;
  double* d_sum = nullptr;     // per-component compatibility sums, then deltas
  std::string err;             // why the table could not be built (empty: built)
};

struct Level {
  CicTable cic;                     // coarse-fine interface conditions (face-data levels)
  GraphCache graph;                 // captured outer cycle of the level solve
  GraphCache graphT;                // the same for the adjoint solve
  Composite cmp;                    // against level l-1 (l >= 1)
  std::vector<uint8_t> face_valid;  // face-data entries not under level l+1
  uint8_t* d_face_valid = nullptr;
  double* E64 = nullptr;            // total correction of this level in a composite cycle
  double* A64 = nullptr;            // adjoint accumulator (composite adjoint)
  double* mu = nullptr;             // adjoints of the interpolated ghosts
  std::vector<Box> boxes;
  bool isolated = false;
  int cf_mode = AMG_CF_DIRICHLET;
  std::vector<Depth> depths;
  std::vector<int32_t> box_comp;
  std::vector<int32_t> comp_singular;
  std::vector<int64_t> comp_cells;
  std::vector<double> comp_ncf;      // coarse-fine Neumann face columns per component (depth 0)
  std::vector<int64_t> face_off;     // [box*6 + d*2 + side] element offset of face data
  int64_t nface = 0;
  int ncomp = 0, nsingular = 0;
  int64_t ncells = 0;
  // device
  double* d_mat = nullptr;
  int64_t* d_idx = nullptr;
  size_t nmat = 0;           // doubles in d_mat
  double* d_gws = nullptr;   // Krylov vectors of the ILU(0)-GMRES bottom
  int64_t ngws = 0;          // doubles in d_gws
  double* r64 = nullptr;     // outer residual
  double* fsh = nullptr;     // right-hand side after the solvability shift
  double* partial = nullptr; // tile partials (max over all depths)
  double* partial2 = nullptr; // segment partials
  double* comp_sum = nullptr;
  int32_t* d_comp_flag = nullptr;  // 1 on singular components
  double* d_comp_cnt = nullptr;    // cells per component at each depth [depth*ncomp + c]
  double* d_delta = nullptr;       // per-component shift
  double* d_delta0 = nullptr;      // per-component mean of the outer residual (kept through the V-cycle)
  double* d_bsum = nullptr;        // per-component sum of Neumann face data
  double* d_defect = nullptr;      // per-component solvability defect
  double* d_comp_ncf = nullptr;    // comp_ncf on the device
  double* d_dfd = nullptr;         // per-component face-data correction
  double* fdc = nullptr;           // corrected face data (nface)
  double* scal = nullptr;    // device scalars: norms history, scale
  double* h_scal = nullptr;  // pinned host mirror
};

}  // namespace amg

namespace amg {
// Optional per-kernel timing with HIP events recorded on the solve's stream
// around the launches of a few kernel kinds (finest depth only).
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> pool;
  size_t next = 0;
  size_t base = 0;  // events below base belong to a captured graph
  std::vector<std::pair<int, size_t>> pending;  // (kind, index of the start event)
  int64_t count[AMG_T_KINDS] = {};
  double total_ms[AMG_T_KINDS] = {};
};
}  // namespace amg

struct amg_hier {
  amg::Timer timer;
  int march2 = MARCH2_DEFAULT, march3 = MARCH3_DEFAULT;  // tile march lengths
  int row_align = ROW_ALIGN_DEFAULT;                       // row alignment of the packed layout (elements)
  int bottom_cells = 0;  // coarsening stops once every component has at most this many cells (0: off)
  int split_rb = 1;      // mixed-precision post-smoothing of depth 0 in colour-split storage where allowed
  int tail = 1;          // the FP32 V-cycle's coarse tail in one workgroup where allowed
  int dim = 2;
  int32_t base[3] = {1, 1, 1};
  double h0 = 1;         // cell size of level 0
  double x_lo[3] = {0, 0, 0};  // physical corner of the grid of level 0
  int ratio = 2;
  int nlevels = 1;
  int phys_bc[3][2] = {{0, 0}, {0, 0}, {0, 0}};
  int op = AMG_HELMHOLTZ;
  double c = 0;
  bool finalized = false;
  hipStream_t own = nullptr;  // used when the caller passes no stream
  amg::GraphCache comp_graph;   // captured cycle of the composite solve
  amg::GraphCache comp_graphT;  // the same for the composite adjoint solve
  int bottom_kind = AMG_BOTTOM_EXACT;  // coarsest-depth solver of forward V-cycles
  int bottom_iters = 5;                // GMRES steps per bottom solve (AMG_BOTTOM_ILU_GMRES)
  double* imex_ws = nullptr;  // stage storage of the IMEX step (allocated on its first call)
  double* regrid_ws = nullptr;  // gradients of the vorticity tagging (allocated on its first call)
  int64_t regrid_len = 0;
  int64_t imex_len = 0;
  std::vector<amg::Level> levels;
  std::string err;
};

namespace amg {
// planner (layout.cpp)
int plan_level(amg_hier* H, int l, std::string& err);
// composite tables of level l against level l-1 (composite.cpp)
int build_composite(amg_hier* H, int l, std::string& err);
// interface-condition table of a level solved with face data (composite.cpp)
int build_cic(amg_hier* H, int l, std::string& err);
// AMRCFI weights [(shift + 2) * r + child][window cell] (composite.cpp)
void cfi_weight_table(double W[20][5], int r);
// host assembly of the coarsest operator and its inverse (bottom.cpp)
int build_bottom(amg_hier* H, int l, std::string& err, std::vector<double>& mats, std::vector<int64_t>& idx);
}  // namespace amg
