/*
 * amg.h -- C ABI of the MI355X multigrid library for the fourth-order
 * finite-volume Helmholtz and Poisson systems of a block-structured AMR
 * hierarchy (Zhao & Zhang, arXiv 2506.02663).
 *
 * The operations follow the paper's statement of the problem:
 *   - hierarchy, levels and boxes ............ Section 5.1, eqs. (grids), (AMRHier)
 *   - operators (I - c L) and L .............. eq. (discreteOps c); (TLS-1..3) of
 *                                              Section 6.5; c = gamma nu k, eq. (GePUP-IMEX)
 *   - physical boundary conditions ........... eqs. (velBCHomoDiri5th), (Neumann5);
 *                                              the assignment of Section 4
 *   - coarse-fine conditions of a level ...... Definition 6.1, eq. (GePUP-localized)
 *   - solvability per connected component .... eqs. (GePUP-localized-solvability-
 *                                              condition), (velocity_disc_solvabilityCond)
 *   - the multigrid solver ................... Section 6.5
 *
 * Conventions shared by every call.
 *   Index space.  Level l has cell size h_l = h0 / ratio^l.  A box is given by
 *   its inclusive corners lo/hi in level-l indices (eq. AMRHier); cell i spans
 *   [x_lo + i h_l, x_lo + (i+1) h_l] in each direction (amg_create).
 *   Packed level buffer.  Every array of cell averages of a level (solution,
 *   right-hand side, output of an operator) is ONE device buffer holding all
 *   boxes of the level, each stored with two ghost layers on every side, x
 *   fastest.  amg_box_info gives, per box, the element offset of its stored
 *   corner (ghost index -2 in every direction) and its strides; the interior
 *   cell (i,j,k) (0-based within the box) is at
 *       offset + (i+2) stride[0] + (j+2) stride[1] + (k+2) stride[2].
 *   Ghost entries are written by the library; the caller leaves them alone.
 *   Face data.  One FP64 device buffer per level; for every box and every face
 *   (d, side) a dense array over the face's cells (transverse directions in
 *   increasing order, the first fastest) at the face_offset given by amg_box_info.  Entry
 *   = face average of the Dirichlet value, or of the derivative along the
 *   OUTWARD normal for Neumann, on faces that lie on the physical boundary or
 *   (for AMG_CF_DIRICHLET / AMG_CF_NEUMANN levels) on the coarse-fine
 *   interface.  Other entries are ignored.  NULL means all zero.
 *   Ownership.  The caller owns every buffer it passes (device memory); the
 *   library only reads inputs and writes outputs during the call, on the
 *   given stream (a hipStream_t passed as void*, NULL = default stream).  The
 *   library owns its workspace, allocated in amg_finalize and freed in
 *   amg_destroy; nothing is allocated on the solve path.
 *   Errors.  Every call returns AMG_OK (0) or a positive error code; the
 *   message of the last error is amg_last_error(h).  A failed call leaves
 *   outputs unspecified except where stated.
 *   Threading.  One hierarchy object must not be used from two host threads
 *   at once.  Results are bitwise reproducible for identical inputs on one
 *   device (all reductions have a fixed order).
 */
#ifndef AMG_H
#define AMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define AMG_OK 0
#define AMG_EINVAL 1          /* bad argument */
#define AMG_ELAYOUT 2         /* invalid box layout (overlap, nesting, alignment, size) */
#define AMG_EUNSUPPORTED 3    /* valid but not supported (e.g. box too small) */
#define AMG_ENOTCONVERGED 4   /* max_cycles reached; x holds the last iterate */
#define AMG_ENONFINITE 5      /* NaN or Inf in a residual */
#define AMG_ESOLVABILITY 6    /* Neumann defect above the stopping target with enforcement off */
#define AMG_EDEVICE 7         /* HIP runtime error */

/* operator kinds (Section 6.5) */
#define AMG_HELMHOLTZ 0 /* (I - c L), (TLS-2) */
#define AMG_POISSON 1   /* L, (TLS-1) and (TLS-3) */

/* boundary condition types */
#define AMG_DIRICHLET 0
#define AMG_NEUMANN 1
#define AMG_PERIODIC 2 /* both sides of a direction; the domains of Section 7.3 */

/* coarse-fine modes of a level */
#define AMG_CF_DIRICHLET 0 /* face averages given on the coarse-fine interface */
#define AMG_CF_NEUMANN 1   /* outward normal derivatives given there */
#define AMG_CF_INTERP 2    /* ghosts interpolated from level l-1 (composite solves) */

/* smoothers */
#define AMG_SMOOTH_JACOBI 0 /* weighted Jacobi, Section 6.5 */
#define AMG_SMOOTH_RB 1     /* red-black: Jacobi within each colour of (sum of indices) mod 2 */

/* precision modes */
#define AMG_FP64 0  /* every step in FP64 */
#define AMG_MIXED 1 /* FP32 V-cycle inside FP64 iterative refinement */

/* data types of the step-level entry points */
#define AMG_F64 0
#define AMG_F32 1

/* solvability modes for components with a constant null vector */
#define AMG_SOLV_RHS_SHIFT 0 /* shift the right-hand side to satisfy the discrete condition */
/* AMG_SOLV_OFF: do nothing; report the defect.  The residual of a singular
 * component has the mean defect / (|cells| h^D) whatever x is (the operator
 * maps every x to data of zero sum there, eq. velocity_disc_solvabilityCond),
 * so if that mean exceeds the stopping target max(tol_rel r0, tol_abs) the
 * solve cannot converge: it returns AMG_ESOLVABILITY before any cycle, x
 * unchanged, stats holding r0 and the defects. */
#define AMG_SOLV_OFF 1
/* eq. (correctingFaceAvg): add one constant delta to the Neumann face data of
 * every coarse-fine face of the component (|faces| delta h^(D-1) = defect);
 * a component without coarse-fine Neumann faces takes the RHS shift.  Level
 * solves only (a composite solve treats it as AMG_SOLV_RHS_SHIFT). */
#define AMG_SOLV_CF_DELTA 2

/* kernel kinds of the optional event timing (finest multigrid depth) */
#define AMG_T_SWEEP 0     /* one smoothing sweep or half-sweep (except the kind below) */
#define AMG_T_FILL 1      /* one ghost fill */
#define AMG_T_RESTRICT 2  /* fused residual and restriction */
#define AMG_T_PROLONG 3   /* prolongation and correction */
#define AMG_T_RESIDUAL 4  /* outer FP64 residual with its norm partials */
#define AMG_T_SWEEP_SPLIT 5 /* one red-black half-sweep in colour-split storage (not the first two from zero) */
#define AMG_T_KINDS 6

#define AMG_MAX_HISTORY 128
#define AMG_MAX_COMP 64

typedef struct amg_hier amg_hier;

typedef struct {
  int32_t nboxes;
  int32_t depths;      /* multigrid depths of this level (>= 1) */
  int32_t ncomp;       /* face-connected components */
  int32_t nsingular;   /* components with a constant null vector under the operator */
  int64_t ncells;      /* interior cells */
  int64_t nstored;     /* elements of the packed buffer */
  int64_t nface;       /* elements of the face-data buffer */
  int32_t split_rb;    /* bit k set: mixed-precision solves post-smooth depth k in colour-split storage */
  int32_t tail_depth;  /* first depth of the FP32 V-cycle's one-workgroup coarse tail (AMG_TUNE_TAIL) in
                          forward solves, -1: none */
} amg_level_desc;

typedef struct {
  int32_t lo[3], hi[3];       /* inclusive corners (level indices; unused dims 0) */
  int64_t offset;             /* element offset of the stored corner */
  int64_t stride[3];          /* element strides (stride[0] = 1) */
  int64_t face_offset[3][2];  /* element offset of each face's data */
  int32_t comp;               /* component id */
  int32_t singular;           /* 1 if that component is singular */
} amg_box_desc;

typedef struct {
  int32_t nu1, nu2;      /* pre- and post-smoothing sweeps */
  int32_t smoother;      /* AMG_SMOOTH_* */
  int32_t precision;     /* AMG_FP64 or AMG_MIXED */
  int32_t solvability;   /* AMG_SOLV_* */
  int32_t max_cycles;
  double omega;          /* weighted-Jacobi factor (2/3 in the paper) */
  double tol_rel;        /* stop when ||r||_inf <= max(tol_rel ||r0||_inf, tol_abs) */
  double tol_abs;
  int32_t use_graph;     /* 1: capture the outer cycle once into a HIP graph and replay it */
  int32_t pad_;
  double omega_rb;       /* red-black: each half-sweep adds omega_rb times its correction
                            (1: plain red-black; over-relaxation > 1), 0 < omega_rb < 2 */
} amg_solve_opts;

typedef struct {
  int32_t cycles;
  int32_t converged;
  double r0;                           /* ||f - A x0||_inf */
  double rfinal;                       /* ||f - A x||_inf at return */
  double history[AMG_MAX_HISTORY];     /* ||r||_inf after each cycle, history[0] = r0 */
  int32_t ncomp;
  int32_t used_graph;                  /* 1 if the cycles ran as replays of a captured HIP graph */
  int32_t pad_;
  double defect[AMG_MAX_COMP];         /* h^D sum f - h^(D-1) sum g per singular component, before the shift */
} amg_solve_stats;

/* Fills opts with the defaults: V(2,2), weighted Jacobi omega = 2/3, mixed
 * precision, RHS shift, tol_rel 1e-10, tol_abs 0, 100 cycles. */
void amg_default_opts(amg_solve_opts* opts);

/* Creates a hierarchy of nlevels levels over the box [x_lo, x_hi] (dim
 * entries each) of the physical domain, cut into base_cells[d] cells along
 * direction d at level 0, in dimension dim (2 or 3) with refinement ratio
 * `ratio` (2 or 4; the tests of Sections 7.4-7.5 take 4) between
 * consecutive levels, eq. (grids) of Section 5.1: cells are cubes, so
 * (x_hi[d] - x_lo[d]) / base_cells[d] must be the same h0 in every direction
 * (to 1e-12 relative), and level l has h0 / ratio^l.  Cell i of level l spans
 * [x_lo + i h_l, x_lo + (i+1) h_l].  *out receives the handle.
 * Errors: AMG_EINVAL (dim, ratio, nlevels outside 1..16, fewer than 4 cells,
 * an empty or non-finite extent, cells that are not cubes). */
int amg_create(int dim, const double* x_lo, const double* x_hi, const int32_t* base_cells, int ratio, int nlevels,
               amg_hier** out);

/* Frees the hierarchy and all its device workspace.  NULL is a no-op. */
int amg_destroy(amg_hier* h);

/* Message of the last failed call (a string owned by h, valid until the next
 * call on h). */
const char* amg_last_error(const amg_hier* h);

/* Sets the boxes of a level: lo and hi hold nboxes*dim inclusive corners
 * (eq. AMRHier), copied by the call.  Level 0 must cover the whole grid
 * unless the level is isolated. */
int amg_set_level_boxes(amg_hier* h, int level, int nboxes, const int32_t* lo, const int32_t* hi);

/* isolated != 0 makes every box of the level an independent domain with the
 * physical conditions on all its faces (a batch of independent solves that
 * share one launch per multigrid step). */
int amg_set_isolated_boxes(amg_hier* h, int level, int isolated);

/* Physical condition on the domain face (d, side), side 0 = low, 1 = high:
 * AMG_DIRICHLET (face averages of the value, eq. velBCHomoDiri5th),
 * AMG_NEUMANN (face averages of the outward normal derivative, eq.
 * Neumann5), the assignment of the boundary conditions to the velocity and
 * pressure systems in Section 4, or AMG_PERIODIC (the periodic domains of
 * Section 7.3: a ghost beyond the side is the cell at its index modulo the
 * grid size, no face data).  Default Dirichlet on every face.  Set before
 * amg_finalize.  Errors: AMG_EINVAL (d, side or type out of range, layout
 * final); amg_finalize returns AMG_EINVAL when a direction is periodic on
 * one side only, and AMG_EUNSUPPORTED when a level above 0 touches a
 * periodic side or a level of isolated boxes has a periodic direction. */
int amg_set_physical_bc(amg_hier* h, int d, int side, int type);

/* bottom solvers */
#define AMG_BOTTOM_EXACT 0     /* dense FP64 inverse of each coarsest system (default) */
#define AMG_BOTTOM_ILU_GMRES 1 /* ILU(0)-preconditioned GMRES(m), Section 6.5 */

/* Solver of the coarsest multigrid depth in forward V-cycles (Section 6.5):
 * AMG_BOTTOM_EXACT, or the paper's AMG_BOTTOM_ILU_GMRES: iters (1..16)
 * steps of GMRES from zero per bottom solve, preconditioned on the right by
 * the ILU(0) factorisation of each coarsest system (a component, or an
 * isolated box; bordered with the zero-mean constraint when the operator
 * is singular on it; pattern: the diagonal and the entries above 1e-12 of
 * their row's largest; unknowns box by box, x fastest).  The factors are
 * computed once by amg_finalize (and amg_set_coefficient) and kept as one
 * dense preconditioning matrix per system, so a preconditioning is a
 * matrix-vector product; the library adds (iters + 1) Krylov vectors per
 * system instance.  Adjoint solves keep the exact transposed inverse.  Set
 * before amg_finalize.  Errors: AMG_EINVAL (kind, iters, layout final);
 * amg_finalize returns AMG_EUNSUPPORTED if an ILU(0) pivot vanishes or a
 * coarsest system has more than 4096 unknowns. */
int amg_set_bottom_solver(amg_hier* h, int kind, int iters);

/* Coarse-fine mode of a level > 0 (default AMG_CF_DIRICHLET): the condition
 * its ghosts take on the coarse-fine interface.  AMG_CF_DIRICHLET /
 * AMG_CF_NEUMANN: the level is solved on its own with face data on the
 * interface (Definition 6.1 and the interface conditions of Section 6.3,
 * filled by eqs. velBCHomoDiri5th / Neumann5 like a physical face);
 * AMG_CF_INTERP: ghosts interpolated from level l-1 (the AMRCFI of Section
 * 5.2), for composite solves (COH-1..4 of Section 5.3).  Set before
 * amg_finalize.  Errors: AMG_EINVAL (level 0, mode out of range, final). */
int amg_set_cf_mode(amg_hier* h, int level, int mode);

/* Operator of every level: AMG_HELMHOLTZ (I - c L), c > 0, the implicit
 * stage operator of eq. GePUP-IMEX with c = gamma nu k ((TLS-2) of Section
 * 6.5; the caller computes c, since the tableau is not printed), or
 * AMG_POISSON L ((TLS-1) and (TLS-3); c ignored), with L the fourth-order
 * Laplacian of eq. discreteOps c.  Set before amg_finalize (a new c after it:
 * amg_set_coefficient).  Errors: AMG_EINVAL (kind, c <= 0 for Helmholtz,
 * layout final). */
int amg_set_operator(amg_hier* h, int kind, double c);

/* Tuning knobs of the kernels' work layout, set before amg_finalize:
 * AMG_TUNE_MARCH2 / AMG_TUNE_MARCH3: the longest march (cells a tile walks
 * along the last direction) in 2D / 3D, even, 2..4096; each multigrid depth
 * uses the longest even march up to it that still gives about 512 tiles; AMG_TUNE_ROW_ALIGN: rows of the packed
 * layout are padded so that every box row starts on a multiple of this many
 * elements (power of two, 2..256).  They change speed, not results. */
#define AMG_TUNE_MARCH2 0
#define AMG_TUNE_MARCH3 1
#define AMG_TUNE_ROW_ALIGN 2
/* AMG_TUNE_SPLIT_RB: 1 (default) lets the mixed-precision solve keep the
 * finest depth's correction and right-hand side in colour-split storage
 * (each colour in its own half array, so a red-black half-sweep moves only
 * the cells it reads and writes), in 2D and 3D, on depths whose faces are
 * all filled uniformly with both ghost layers from their own rows, whose
 * boxes have even sizes and where no box is solved exactly; 0 keeps the
 * interleaved storage.  The two forms give the same results (to the
 * rounding of FP32 sums). */
#define AMG_TUNE_SPLIT_RB 3
/* AMG_TUNE_TAIL: 1 (default) runs the coarse tail of the FP32 V-cycle of a
 * forward solve in three launches: from the first depth of at most 4096
 * cells (16^3, 64^2) down, where every depth holds one box whose faces are
 * all filled uniformly or periodic across the whole box, and the coarsest is
 * one exact system, one workgroup
 * smooths and restricts depth after depth in LDS, the bottom kernel solves,
 * and one workgroup prolongs and smooths back up; 0 launches every
 * operation of every depth.  The two forms give the same results (to the
 * rounding of FP32 sums). */
#define AMG_TUNE_TAIL 4
int amg_set_tuning(amg_hier* h, int key, int value);

/* Size of the exactly solved coarsest systems (Section 6.5 leaves the bottom
 * solver open; this library solves the coarsest depth exactly).  Coarsening
 * stops at the first depth where every component of a level (of an isolated
 * level: every box) has at most `cells` cells, or where the layout rule below
 * stops it; `cells` = 0 (the default) coarsens as far as the layout allows.
 * A larger bottom replaces the smallest, launch-bound depths by one dense
 * FP64 solve; it changes the multigrid hierarchy, hence the iterates (not
 * the converged solution).  0..1024 (the inverse is formed on the host in
 * O(cells^3)), set before amg_finalize.
 * Errors: AMG_EINVAL (range, or the layout is final). */
int amg_set_bottom_cells(amg_hier* h, int cells);

/* Validates the layout (disjoint boxes inside the grid, proper refinement
 * eq. (pBlock), boxes of at least 4 cells per side), labels components,
 * builds the multigrid depths (a level is halved while every box has even
 * corners and even sides of at least 8), the ghost, tile and bottom-solve
 * tables, factors the bottom systems, and allocates the workspace.
 * Errors: AMG_ELAYOUT, AMG_EUNSUPPORTED, AMG_EDEVICE. */
int amg_finalize(amg_hier* h);

/* Summary of level `level` after amg_finalize: its boxes (eq. AMRHier), the
 * multigrid depths the planner built (Section 6.5: a level is halved while
 * every box has even corners and even sides of at least 8), the
 * face-connected components and how many of them are singular (pure
 * Neumann: the constant null vector behind the solvability condition of
 * Section 6.4), cells, and the sizes of the packed level buffer and of the
 * face-data buffer.  *out is written by the call.  Errors: AMG_EINVAL (not
 * finalized, level out of range, out NULL). */
int amg_level_info(const amg_hier* h, int level, amg_level_desc* out);

/* Layout of box `box` of level `level` at multigrid depth `depth` (depth 0 is
 * the level itself; deeper layouts serve the step-level entry points): its
 * inclusive corners in that depth's index space (eq. AMRHier; depth k halves
 * the corners of depth k-1: lo / 2, (hi + 1) / 2 - 1), where it sits in the
 * packed buffer, where its face data sit, and its component.  Box order is
 * the order of amg_set_level_boxes at every depth.  *out is written by the
 * call.  A box of an isolated level (amg_set_isolated_boxes) is its own
 * domain: its corners are given in its own index space (lo = 0), and at depth
 * k the table lists, in order, only the boxes that coarsen that far.
 * Errors: AMG_EINVAL (not finalized, an index out of range). */
int amg_box_info(const amg_hier* h, int level, int depth, int box, amg_box_desc* out);
/* Elements of the packed buffer of (level, depth) and boxes at that depth. */
int amg_depth_size(const amg_hier* h, int level, int depth, int64_t* nstored, int32_t* nboxes);

/* Solves the level system A x = f on level `level` (lev_lo == lev_hi; the
 * coarse-fine interface takes the level's face data), or, with lev_lo = 0 <
 * lev_hi, the composite system over levels 0..lev_hi (levels >= 1 in mode
 * AMG_CF_INTERP): each cycle corrects level 0 by a V-cycle of its multigrid,
 * then every finer level by the prolonged coarse correction plus a V-cycle
 * of its own multigrid on its residual, averages down and recomputes the
 * composite residual (see amg_composite_residual); x holds the composite
 * solution (covered cells: averages of the finer level).  x: initial guess on
 * entry, solution on return, ghosts filled.  f, face_data as above.
 * On AMG_ENOTCONVERGED x holds the last iterate and stats are valid. */
int amg_solve(amg_hier* h, int lev_lo, int lev_hi, double* const* x, const double* const* f,
              const double* const* face_data, const amg_solve_opts* opts, amg_solve_stats* stats,
              void* stream);

/* Composite residual r = f - A^comp x over levels 0..lev_hi (COH-1..4 of
 * Section 5.3): x is averaged down onto covered cells (eq.
 * AMR_avergingDownToCrse), every level's ghosts are filled (coarse-fine ones
 * interpolated from the level below), the coarse fluxes through coarse-fine
 * faces are replaced by the mean fine fluxes (refluxing), and r on covered
 * cells is the average of the finer level's r.  x, f, face_data, r: one
 * packed FP64 buffer per level (face_data may be NULL or hold NULLs). */
int amg_composite_residual(amg_hier* h, int lev_hi, double* const* x, const double* const* f,
                           const double* const* face_data, double* const* r, void* stream);

/* y = A x on level `level` (FP64), ghosts of x filled from face_data
 * (homogeneous != 0: face data treated as zero).  x's ghosts are written. */
int amg_apply_operator(amg_hier* h, int level, double* x, const double* face_data, double* y,
                       int homogeneous, void* stream);

/* ---- step-level entry points (one multigrid step on caller buffers in the
 * packed layout of (level, depth); dtype AMG_F64 or AMG_F32).  They serve
 * the per-step parity tests; amg_solve chains the same kernels. ---------- */

/* Ghost fill of u: face data (FP64) at depth 0, or homogeneous if NULL. */
int amg_fill_ghosts(amg_hier* h, int level, int depth, int dtype, void* u, const double* face_data, void* stream);

/* r = f - A u on the interior; u's ghosts must be filled. */
int amg_residual(amg_hier* h, int level, int depth, int dtype, const void* u, const void* f, void* r, void* stream);

/* nsweeps homogeneous sweeps of the chosen smoother on u (ghosts refilled
 * before each sweep and half-sweep); tmp is a second buffer of the same
 * layout.  omega: the Jacobi weight, or the red-black relaxation factor of
 * each half-sweep (1: plain).  The result is in u. */
int amg_smooth(amg_hier* h, int level, int depth, int dtype, int smoother, int nsweeps, double omega,
               void* u, const void* f, void* tmp, void* stream);

/* f_coarse (depth+1) = mean of the 2^D children of r (depth). */
int amg_restrict(amg_hier* h, int level, int depth, int dtype, const void* r, void* f_coarse, void* stream);

/* u (depth) += face-neighbour linear interpolation of e (depth+1); the first
 * ghost layer of e must be filled (homogeneous). */
int amg_prolong(amg_hier* h, int level, int depth, int dtype, const void* e_coarse, void* u, void* stream);

/* Exact solve on the coarsest depth: e = A^-1 f (zero-mean per singular
 * component). */
int amg_bottom(amg_hier* h, int level, int dtype, const void* f, void* e, void* stream);

/* One homogeneous V(nu1,nu2) cycle from e = 0 on the level: e ~= A^-1 f. */
int amg_vcycle(amg_hier* h, int level, int dtype, const amg_solve_opts* opts, const void* f, void* e, void* stream);

/* ---- adjoint of the level system --------------------------------------------
 * Not in the paper: the derivative of a loss J(x) of a level solution
 * x = A^-1 (f - b(face data)) with respect to f is lam = A_h^-T dJ/dx, with
 * A_h the homogeneous operator (ghost fill with zero data, then the stencil
 * of eq. discreteOps c, as I - cL or L).  Its transpose applies the
 * (symmetric) stencil to lam with the filled ghosts set to zero and sends
 * each ghost's stencil weight back onto the four cells its fill read (eqs.
 * velBCHomoDiri5th, Neumann5); exchange ghosts are symmetric and stay
 * copies.  On a singular (pure-Neumann) component the source is made
 * mean-free first and lam is returned mean-free.  The derivative with
 * respect to the Helmholtz coefficient is dJ/dc = <lam, L x> (L with the
 * solve's face data), so dJ/dnu = gamma k <lam, L x> for c = gamma nu k. */

/* Solves A_h^T lam = g on level `level` (a level solved on its own, not
 * AMG_CF_INTERP) by the same outer loop and V-cycle as amg_solve with the
 * transposed operator at every depth (same diagonal, same restriction and
 * prolongation, transposed bottom matrix).  lam: initial guess on entry,
 * solution on return with its face ghost cells set to 0 (corner and row
 * padding entries are not written; starting from a zeroed buffer lam is the
 * gradient with respect to the packed f); g: packed FP64 buffer of the
 * level, read on the level's cells only.  Errors as amg_solve. */
int amg_solve_adjoint(amg_hier* h, int level, double* lam, const double* g, const amg_solve_opts* opts,
                      amg_solve_stats* stats, void* stream);

/* Composite adjoint: solves (A^comp)^T lam = g on the valid cells of levels
 * 0..lev_hi (levels >= 1 in AMG_CF_INTERP), A^comp the homogeneous composite
 * operator of amg_solve's composite form.  Its transpose reverses the
 * average-down (a covered cell's adjoint goes to its children in equal
 * parts), AMRCFI (ghost adjoints back onto the coarse window), the fills and
 * stencils (as for a level) and the refluxing (the adjoint of a refluxed
 * coarse cell onto the coarse and fine values its fluxes read).  The cycle
 * is the composite cycle of amg_solve with each level's transposed multigrid
 * and volume-weighted transfers (covered cells carry the sum of the finer
 * residual; prolonged corrections are divided by 2^D).  Pure Neumann: g is
 * projected along the volume weights w (h_l^D) so that it sums to zero, and
 * lam is returned with zero plain sum (the gradient in f of a solution that
 * amg_solve returns with zero volume-weighted mean).  lam[l]: initial guess
 * in, solution out (covered cells and face ghosts 0); g[l] read on valid
 * cells only.  Errors as amg_solve. */
int amg_solve_adjoint_composite(amg_hier* h, int lev_hi, double* const* lam, const double* const* g,
                                const amg_solve_opts* opts, amg_solve_stats* stats, void* stream);

/* y = L^comp x over levels 0..lev_hi: the composite Laplacian (COH-1..4,
 * refluxed, averaged down) of x with its face data, whatever operator the
 * hierarchy holds; x is averaged down and its ghosts written; y != x.  With x
 * a composite Helmholtz solution and lam its adjoint, dJ/dc = sum over levels
 * of <lam, y> (lam is zero on covered cells). */
int amg_composite_laplacian(amg_hier* h, int lev_hi, double* const* x, const double* const* face_data,
                            double* const* y, void* stream);

/* r = g - (A^comp)^T lam on the valid cells of levels 0..lev_hi (covered
 * cells of r: the sum of their children's values, the convention of the
 * adjoint cycle).  lam's covered cells are set to 0 and its ghosts written. */
int amg_composite_residual_adjoint(amg_hier* h, int lev_hi, double* const* lam, const double* const* g,
                                   double* const* r, void* stream);

/* One V(nu1,nu2) cycle of the adjoint system from e = 0: e ~= A_h^-T f. */
int amg_vcycle_adjoint(amg_hier* h, int level, int dtype, const amg_solve_opts* opts, const void* f, void* e,
                       void* stream);

/* y = A_h^T x (FP64) on depth 0 of `level`; x's ghosts are overwritten (zero
 * on filled columns, copies on exchange columns); x != y. */
int amg_apply_transpose(amg_hier* h, int level, double* x, double* y, void* stream);

/* y = L x (FP64): the Laplacian of eq. (discreteOps c) with x's ghosts filled
 * from face_data (NULL: zero data), whatever operator the hierarchy holds;
 * x != y.  With x a Helmholtz solution, dJ/dc = <lam, y>. */
int amg_apply_laplacian(amg_hier* h, int level, double* x, const double* face_data, double* y, void* stream);

/* *out = sum over the level's cells of a_i b_i (FP64, fixed summation order:
 * bitwise reproducible); synchronises the stream. */
int amg_dot(amg_hier* h, int level, const double* a, const double* b, double* out, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): amg_dot
 * without any allocation, host transfer or synchronisation.  *out (ONE
 * DEVICE double, written on the stream) = sum over the level's cells of
 * a_i b_i, bitwise equal to amg_dot's value (same kernels, same order).  The
 * per-tile partials live in a static 256 KiB device array that every GPU
 * holds until the process ends, so the level may have at most 32768 tiles
 * (AMG_EUNSUPPORTED beyond); every call fully overwrites what it reads, and
 * calls that overlap on one GPU (two streams, two threads) race on that
 * array.  Errors: AMG_EINVAL, AMG_EUNSUPPORTED, AMG_EDEVICE. */
int amg_dot_noalloc(amg_hier* h, int level, const double* a, const double* b, double* out, void* stream);

/* ---- gradient, divergence and the approximate projection --------------------
 * Eqs. (discreteOps a-b) on one level (lev_lo == lev_hi) or in composite form
 * over levels 0..lev_hi (COH-1..4 of Section 5.3: ghosts by the hierarchy's
 * fill and AMRCFI, the divergence refluxed with the face averages of eq.
 * cell2face, results averaged down onto covered cells).  Per-component
 * arrays are indexed [level * dim + d] from level 0 (entries below lev_lo are
 * not read); every buffer is a packed FP64 level buffer.  Inputs have their
 * ghosts written and, in composite form, their covered cells replaced by the
 * averages of the finer level. */

/* g[l*dim+d] = G_d phi[l]; phi's ghosts from the hierarchy's own fill
 * (face_data[l] may be NULL: zero data). */
int amg_gradient(amg_hier* h, int lev_lo, int lev_hi, double* const* phi, const double* const* face_data,
                 double* const* g, void* stream);

/* out[l] = D w = sum_d G_d w[l*dim+d]; component d's ghosts from the
 * hierarchy's fill with face_data[l*dim+d] (face averages of that component;
 * the array or its entries may be NULL). */
int amg_divergence(amg_hier* h, int lev_lo, int lev_hi, double* const* w, const double* const* face_data,
                   double* const* out, void* stream);

/* The approximate projection u = w - G phi, L phi = D w (eq. appProj, or eq.
 * comp_ProjOp in composite form).  hw: the hierarchy whose fill the velocity
 * components take (normally Dirichlet, face data wb = boundary velocity face
 * averages, [l*dim+d], may be NULL); hp: a hierarchy with the same boxes and
 * the Poisson operator with pure-Neumann conditions, which solves for phi
 * (homogeneous Neumann data, RHS shifted for solvability, mean-free phi) with
 * opts, reporting in stats.  phi[l]: initial guess in, potential out.
 * u[l*dim+d] may alias w.  AMG_EINVAL if the layouts differ. */
int amg_project(amg_hier* hw, amg_hier* hp, int lev_lo, int lev_hi, double* const* w, const double* const* wb,
                double* const* phi, double* const* u, const amg_solve_opts* opts, amg_solve_stats* stats,
                void* stream);

/* ---- transposes of G, D and the projection (not in the paper) ---------------
 * The adjoint that carries a loss on the projected velocity back to the
 * velocity before projection.  Each is the transpose of the homogeneous (zero
 * boundary data) linear map above, taken between the valid cells of levels
 * lev_lo..lev_hi (one level, or composite from level 0) in the plain inner
 * product sum over valid cells of a_i b_i: the forward maps read no covered
 * input cell (they average down first) and their covered outputs are copies.
 * G_d of eq. discreteOps a is antisymmetric, so its transpose on a level's
 * cells is -G_d of the adjoint extended by zero, plus the weights the stencil
 * puts on ghosts sent back through the fills (eqs. velBCHomoDiri5th,
 * Neumann5), exchange copies and AMRCFI; the composite divergence's
 * refluxing (COH-3, face averages of eq. cell2face) is transposed onto the
 * values and ghosts its face averages read, and the average-down of the
 * input onto the children of covered cells.  Inputs: their covered cells
 * and ghosts are set to 0 by the call.  Outputs: 0 on covered cells and on
 * ghosts.  Buffers are packed FP64 level buffers indexed as in
 * amg_gradient / amg_divergence; outputs must not alias inputs.  Errors:
 * AMG_EINVAL (range, null buffer), AMG_EUNSUPPORTED (composite not from
 * level 0). */

/* out[l] = sum_d G_d^T mu[l*dim+d], G with the hierarchy's fill. */
int amg_gradient_transpose(amg_hier* h, int lev_lo, int lev_hi, double* const* mu, double* const* out, void* stream);

/* out[l*dim+d] = G_d^T lam[l], the transpose of D w = sum_d G_d w_d with the
 * hierarchy's fill for every component. */
int amg_divergence_transpose(amg_hier* h, int lev_lo, int lev_hi, double* const* lam, double* const* out,
                             void* stream);

/* wbar = P^T ubar = ubar - D^T L^-T G^T ubar for the projection of
 * amg_project (hw, hp as there): G^T on hp, the adjoint pure-Neumann solve of
 * amg_solve_adjoint(_composite) on hp (it holds the transposes of the
 * solvability shift and the mean removal; opts, stats as there), D^T on hw.
 * lam[l]: initial guess in, the adjoint potential out.  ubar[l*dim+d]: its
 * covered cells and ghosts are set to 0; wbar may alias ubar (then it is
 * updated in place), covered cells of wbar are 0.  Uses the work buffers of
 * both hierarchies.  Errors as amg_project and amg_solve_adjoint. */
int amg_project_adjoint(amg_hier* hw, amg_hier* hp, int lev_lo, int lev_hi, double* const* ubar, double* const* lam,
                        double* const* wbar, const amg_solve_opts* opts, amg_solve_stats* stats, void* stream);

/* ---- coarse-fine interface conditions (CIC-1..3 of Section 6.3) -------------
 * The face data a refined level solved on its own (AMG_CF_DIRICHLET or
 * AMG_CF_NEUMANN) takes on its coarse-fine faces, from the data of level-1
 * at four earlier coarse times t_-i = t_-0 - i k (the history kept by the
 * subcycled time stepping, eq. vel_slicing):
 *   CIC-1 the face between a row-end cell e and the position beyond it has
 *         two fine cells on each side along the normal (e - n, e, e + n,
 *         e + 2n, n the outward unit step);
 *   CIC-2 their averages are interpolated from the coarse data by AMRCFI
 *         (Section 5.2, the tensor-product conservative quartic of the
 *         composite operators) and combined by eq. cell2face: the face
 *         average (AMG_CIC_VALUE, first row) or the face average of the
 *         outward normal derivative (AMG_CIC_NORMAL_DERIVATIVE, second row);
 *   CIC-3 eq. timeInterp takes them to t* = t_-1 + eta.
 * Readings of the printed time matrix: its columns belong to t_-3, t_-2,
 * t_-1, t_-0 (it puts weight 1 on t_-1 at eta = 0 and on t_-0 at eta = k),
 * and with the printed prefactor 1/(6k^3) its second row gives d/dt itself.
 * Every step is linear: the kernels combine the coarse data in time first,
 * which agrees with the paper's order to rounding. */
#define AMG_CIC_VALUE 0
#define AMG_CIC_NORMAL_DERIVATIVE 1

/* coarse[i] (i = 0..3): packed FP64 buffers of level-1 with the data at t_-i
 * (covered cells included: the history of level-1 itself); k > 0 the coarse
 * step, eta the offset of t* from t_-1.  Writes the entries of face_data
 * (the level's face-data layout) on its coarse-fine faces, and those of
 * face_data_dt (may be NULL) with the time derivative at t*; other entries
 * (physical faces) are left alone.  Errors: AMG_EINVAL (level 0, an
 * interpolated or isolated level, bad arguments), AMG_EUNSUPPORTED (a
 * coarse window of the interpolation leaves level-1; amg_finalize records
 * this instead of rejecting the layout), AMG_EDEVICE. */
int amg_cic_face_data(amg_hier* h, int level, const double* const* coarse, double k, double eta, int kind,
                      double* face_data, double* face_data_dt, void* stream);

/* Eq. correctingFaceAvg on the face data of a velocity of the level:
 * face_data[d] is the face-data buffer of velocity component d.  Per
 * face-connected component c, the outward normal face averages of its
 * coarse-fine and physical faces must sum to zero (eq.
 * velocity_disc_solvabilityCond; the faces of a level have one area); one
 * constant delta_c, -delta_c (coarse-fine faces of c) = that sum, is added
 * to the outward normal average of each of its coarse-fine faces (component
 * d on faces normal to d, with the outward sign).  delta (host, ncomp
 * values, may be NULL) receives the constants (the call then synchronises
 * the stream).  Errors as amg_cic_face_data. */
int amg_cic_correct(amg_hier* h, int level, double* const* face_data, double* delta, void* stream);

/* ---- the IMEX time step on one periodic level (Section 4) -------------------
 * The convection operator and one time step on a periodic box. */

/* out[d] = (Div<uu>)_d, the convection of eq. convOp: per direction the
 * difference across the cell of the face averages of the product u_d u_e,
 * each the product of the face averages (eq. cell2face) plus h^2/12 times
 * the products of their centred transverse differences.  h: one level of
 * one box on a grid periodic in every direction (neighbours wrap; ghosts
 * are not read).  u[d], out[d]: packed FP64 level buffers, out not aliasing
 * u; only cells are written.  Errors: AMG_EINVAL (null), AMG_EUNSUPPORTED
 * (layout). */
int amg_convection(amg_hier* h, double* const* u, double* const* out, void* stream);

typedef struct {
  int32_t solves;           /* linear solves run (TLS-1, TLS-2 per component, TLS-3) */
  int32_t cycles;           /* outer cycles over all of them */
  int32_t max_cycles;       /* most cycles of one solve */
  int32_t converged;        /* 1 if every solve converged */
  double max_rel_residual;  /* max over the solves of ||r||_inf / ||b||_inf at return */
} amg_imex_stats;

/* One step of eq. GePUP-IMEX with the ERK-ESDIRK pair ARK4(3)6L[2]SA of
 * Kennedy and Carpenter (2003, the scheme the paper cites; six stages,
 * gamma = 1/4, stiffly accurate) for the system eq. ODE-MOL on a level that
 * is one box covering a grid periodic in every direction (the domains of
 * Section 7.3, where no boundary data enter).  Per stage s = 2..6: X of
 * the previous stage from its velocity (convection eq. convOp, pressure
 * from L q = D(g - Div<uu>), TLS-1), the Helmholtz systems
 * (I - dt nu gamma L) w = w^n + dt sum A_E X + dt nu sum A_I L w per
 * component (TLS-2), then u = P w (eq. appProj, TLS-3); after the last
 * stage one more X, w* = w^(6) + dt sum (b - A_E[6]) X and u^(n+1) = P w*.
 * hv: Helmholtz hierarchy of the velocity (its coefficient is set to
 * dt nu / 4 by the call when it differs: bottom inverses are rebuilt on
 * the host, see amg_set_coefficient); hp: Poisson hierarchy with the same
 * box; both one level, periodic in every direction.  u[d]: packed FP64
 * level buffers, u^n on entry (taken as w^n), u^(n+1) on return.  g: NULL
 * (no forcing) or g[j*dim+d], the forcing's cell averages at t_n + c_j dt,
 * j = 0..5 (c = 0, 1/2, 83/250, 31/50, 17/20, 1).  opts: the Helmholtz
 * solves; opts_p: the Poisson solves of the pressure and the projection
 * (NULL: opts).  Each stage system starts from the previous stage's solution of
 * the same system (the pressure and the potential from zero at the first
 * stage, the velocity from w^n) and stops when ||r||_inf <= max(tol_rel
 * ||b||_inf, tol_abs), b its right-hand side: the test of a solve from
 * zero, whose initial residual is b.
 * The library keeps (15 dim + 4) level buffers of stage storage and one
 * word in hv, allocated on the first call.  Not graph-capturable (it allocates on its
 * first call and the solves synchronise).  Errors: AMG_EINVAL (null
 * argument, dt <= 0, nu < 0, operators or layouts that differ),
 * AMG_EUNSUPPORTED (not one periodic box on one level), errors of the
 * solves; AMG_ENOTCONVERGED if a solve did not converge (u still holds the
 * step's result). */
int amg_imex_step(amg_hier* hv, amg_hier* hp, double dt, double nu, double* const* u, const double* const* g,
                  const amg_solve_opts* opts, const amg_solve_opts* opts_p, amg_imex_stats* stats, void* stream);

/* The inverse of the dense row-major n x n FP64 matrix a, in place: the
 * factorisation behind the exact bottom solve (the coarsest depth's system,
 * Section 6.5 replaced by an exact solve), Gauss-Jordan elimination with
 * partial pivoting in blocks of 64 columns on up to `threads` host threads.
 * Host-only: no device call.  Errors: AMG_EINVAL (n < 1, null a, threads
 * < 1), AMG_EUNSUPPORTED (a zero pivot: a singular matrix; a is then left
 * unchanged). */
int amg_dense_inverse(int n, double* a, int threads);

/* ---- Algorithm 1's time schedule (Section 6.2) ------------------------------
 * The order and times of the level advances of the subcycled AMR method,
 * host-only (no device call, no level is advanced): a driver runs each
 * event with the level operations above.
 *   AMG_SC_SYNCED: one step dt = k0 / ratio^(nlevels-1) of synchronized AMR
 *     (Section 5.5: all levels together) from t; 3 ratio^(nlevels-1) of them
 *     take the hierarchy from t0 to t0 + 3 k0 (Algorithm 1, line 1), filling
 *     the four time slices of every level (eq. vel_slicing);
 *   AMG_SC_REGRID: regrid and migrate at t, before a coarse step (line 4;
 *     the criterion read here as a period of regrid_every coarse steps, 0:
 *     never);
 *   AMG_SC_ADVANCE: advance `level` by one step dt = k0 / ratio^level from
 *     t (SingleLevelAdvance, line 5); for level > 0 the interface
 *     conditions come from the slices of level-1 at t_coarse - i k_coarse,
 *     i = 0..3, so a stage at t* = t + c dt takes eta = t* - (t_coarse -
 *     k_coarse) in eq. timeInterp (0 <= eta <= k_coarse) with k = k_coarse;
 *   AMG_SC_SYNC: the composite projection of levels level..nlevels-1 at t
 *     (line 11), after the finer levels have caught up with `level`.
 * Per coarse step the events are those of SingleLevelAdvance(0)'s
 * recursion: level l advances ratio^l times. */
#define AMG_SC_SYNCED 0
#define AMG_SC_REGRID 1
#define AMG_SC_ADVANCE 2
#define AMG_SC_SYNC 3

typedef struct {
  int32_t kind;      /* AMG_SC_* */
  int32_t level;     /* the level advanced or synchronised from (SYNCED: the finest) */
  double t;          /* start time of the step, or the time of the regrid / synchronisation */
  double dt;         /* the step (0 for REGRID and SYNC) */
  double k_coarse;   /* ADVANCE of a level > 0: the step of level-1; else 0 */
  double t_coarse;   /* ADVANCE of a level > 0: the newest time slice of level-1; else 0 */
} amg_sc_event;

/* The events of Algorithm 1 from t0 (step k0 on level 0, refinement ratio
 * 2 or 4, 1 <= nlevels <= 8): the synchronized start, then ncoarse coarse
 * steps.  Times are t0 plus integer multiples of the finest step (no drift
 * over long runs).  events (host, max_events entries) receives at most
 * max_events of them, *nevents their total.  Errors: AMG_EINVAL (arguments),
 * AMG_EUNSUPPORTED (more events than max_events; *nevents is still the
 * total). */
int amg_subcycle_schedule(int nlevels, int ratio, double t0, double k0, int ncoarse, int regrid_every,
                          int max_events, int32_t* nevents, amg_sc_event* events);

/* ---- regridding and data migration (Section 5.4, RDM-1..4) -----------------
 * Clustering (RDM-2), as read from Berger and Rigoutsos (1991): a box is
 * shrunk to the bounding box of its tags and accepted when tags / cells
 * reaches `efficiency`; otherwise it is cut in two along one direction at
 * index c (parts [lo, c-1] and [c, hi], each at least min_side long along
 * the cut): at a slice without tags closest to the box's centre; else at
 * the strongest inflection of the tag signature (the largest jump of its
 * second difference where that changes sign between neighbouring slices);
 * else at the middle of the longest side; ties to the position closer to
 * the centre, then the lower direction, then the lower index; a box without
 * an admissible cut is accepted; the low part first.  Host-only: no device
 * call. */

/* Boxes of the tagged cells of the dense host array tags (shape[d] cells
 * per direction, x fastest, nonzero = tagged): *nboxes receives their
 * number, lo/hi (max_boxes * dim entries each) their inclusive corners.
 * Errors: AMG_EINVAL (dim, shape, efficiency outside (0, 1], min_side < 1,
 * null pointers), AMG_EUNSUPPORTED (more than max_boxes; *nboxes is still
 * the count). */
int amg_cluster(int dim, const int32_t* shape, const uint8_t* tags, double efficiency, int min_side, int max_boxes,
                int32_t* nboxes, int32_t* lo, int32_t* hi);

/* RDM-2..4: the boxes of new levels 1..ntag from the tags of levels
 * 0..ntag-1 (tags[l]: dense host array over level l's grid, base_cells
 * times ratio^l, x fastest): new level ntag clusters the tags of level
 * ntag-1; for l = ntag-2 .. 0 the boxes of new level l+2 coarsened twice and
 * grown by `grow` cells of level l (clipped to the grid) join the tags of
 * level l, and their clustering gives new level l+1; boxes are refined by
 * the ratio.  Every clustering runs on the level's grid coarsened by the
 * blocking factor `block` (a block is tagged when any of its cells is;
 * boxes refined by it and clipped).  grow = 0: the least g with g * ratio
 * >= 3 (every five-cell AMRCFI window of level l+2 then lies on level l+1;
 * the paper's one cell is that at ratio 4); block = 0: the least b with
 * b * ratio >= 4 (every box at least four cells wide, as the fills need).
 * nboxes[l-1]: boxes of new level l (0: none); lo/hi: per new level
 * max_boxes * dim entries.  Errors: AMG_EINVAL (arguments, ratio not 2 or
 * 4, grow < 0, block outside 0..64), AMG_EUNSUPPORTED (a level needs more
 * than max_boxes). */
int amg_regrid_boxes(int dim, const int32_t* base_cells, int ratio, int ntag, const uint8_t* const* tags,
                     double efficiency, int min_side, int grow, int block, int max_boxes, int32_t* nboxes, int32_t* lo, int32_t* hi);

/* RDM-1: tags[l] (device, one byte per cell of level l's grid, x fastest)
 * := 1 where the vorticity of the velocity u[l*dim+d] reaches eps on a cell
 * of level l, else 0 (also off the level), levels 0..lev_hi.  Vorticity:
 * 2D G_x u_1 - G_y u_0, 3D the norm of the curl, from the composite gradient
 * of each component (amg_gradient: the velocity's ghosts and covered cells
 * are written).  The library keeps dim^2 level buffers per level of
 * gradient storage, allocated on the first call.  Errors: AMG_EINVAL. */
int amg_tag_vorticity(amg_hier* h, int lev_hi, double* const* u, double eps, uint8_t* const* tags, void* stream);

/* Data migration onto a new hierarchy (Section 5.4): u_new[l] on every
 * cell of new level l := u_old[l] where old level l has the cell, else
 * AMRCFI from new level l-1 (levels in increasing order; level 0 is
 * copied).  Both hierarchies final, with the same dimension, grid, cell
 * size and ratio.  Allocates and frees its lookup tables; synchronises the
 * stream.  Errors: AMG_EINVAL, AMG_EUNSUPPORTED (an interpolation window
 * off new level l-1). */
int amg_migrate(amg_hier* h_old, amg_hier* h_new, double* const* u_old, double* const* u_new, void* stream);

/* Changes the Helmholtz coefficient c (> 0) of a finalized hierarchy: the
 * bottom inverses are recomputed on the host and captured graphs dropped.
 * Not on the hot path; AMG_EINVAL if the operator is not Helmholtz. */
int amg_set_coefficient(amg_hier* h, double c);

/* ---- measurement -------------------------------------------------------- */

/* on != 0: every later amg_solve records a HIP event before and after each
 * launch of the AMG_T_* kernels on the finest depth (on the solve's stream)
 * and accumulates their durations; creates the event pool on first use. */
int amg_timing_enable(amg_hier* h, int on);

/* Measurement of the dominant kernel: the finest-depth smoothing kernel of
 * `level` (one Jacobi sweep, or one red-black half-sweep alternating the
 * colours) launched n times back to back on the stream, u and tmp swapping
 * roles, with no ghost fill in between, bracketed by two HIP events;
 * *avg_ms = elapsed / n.  FP32 red-black on a depth whose mixed-precision
 * post-smoothing runs in colour-split storage (AMG_TUNE_SPLIT_RB) times that
 * split half-sweep, u, f and tmp taken as split arrays.  The values written
 * are not a smoothing result (ghosts are not refilled): for timing only.
 * u != tmp. */
int amg_time_sweep(amg_hier* h, int level, int dtype, int smoother, int n, void* u, const void* f, void* tmp,
                   double* avg_ms, void* stream);

/* Autotuning of the tile march length (cells a tile marches along the last
 * direction, AMG_TUNE_MARCH2/3) before amg_finalize: for each candidate
 * (4, 6, 8, 16, 32, 64, 128; from 8 for 3D sweeps in interleaved storage)
 * a finalized copy of the layout times the finest-depth
 * smoothing kernel of `level` (amg_time_sweep, nreps launches, zero data);
 * the fastest candidate is set on h.  *best, *best_ms (may be NULL) receive
 * it and its time per launch.  Allocates and frees device memory. */
int amg_autotune(amg_hier* h, int level, int dtype, int smoother, int nreps, int* best, double* best_ms);

/* Launch count and summed duration (ms) of kernel kind `kind` since the last
 * reset; reset != 0 clears the counters after reading.  Launches made by the
 * step-level calls (amg_smooth, ...) are waited for and collected first. */
int amg_timing_read(amg_hier* h, int kind, int64_t* count, double* total_ms, int reset);

#ifdef __cplusplus
}
#endif
#endif /* AMG_H */
