/*
 * stv.h - C ABI of the MI355X space-time Vanka multigrid library.
 *
 * The library solves J d = r (the linear system of one Newton or Oseen step of
 * the dG(k)-in-time, Q2/P1disc-in-space discretisation of the incompressible
 * Navier-Stokes equations, Section 4.1 eq. (4.1) of Anselmann & Bause,
 * "A geometric multigrid method for space-time finite element discretizations
 * of the Navier-Stokes equations and its application to 3d flow simulation")
 * by flexible GMRES preconditioned with a geometric multigrid V-cycle
 * (Algorithm 4.1) whose smoother is the cell-based space-time Vanka operator
 * (Section 4.2, eq. (4.6), with the damping of Section 5.3).
 *
 * Conventions shared by every entry point
 *   - Status: every int-returning call returns STV_OK (0) or a negative code
 *     below; the text of the last error of a context is stv_last_error().
 *     No C++ exception crosses this boundary.
 *   - Levels: index 0 is the coarsest level (the paper's g = 1, solved
 *     directly); index n_levels-1 is the finest (g = G).
 *   - Space-time vectors are FP64, time-inner: entry s*(k+1) + l holds
 *     spatial DoF s at temporal DoF l.  Vectors passed to the compute calls
 *     are DEVICE pointers owned by the caller; the calls are asynchronous on
 *     the context's stream unless stated otherwise.
 *   - Host arrays handed to stv_set_hierarchy are deep-copied; the caller may
 *     free them when the call returns.
 *   - One context serves one stream; calls on one context must not overlap
 *     from several host threads.
 */
#ifndef STV_H
#define STV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---- */
#define STV_OK 0
#define STV_EINVAL (-1)     /* invalid argument or malformed hierarchy      */
#define STV_ENOMEM (-2)     /* device or host allocation failed             */
#define STV_EHIP (-3)       /* a HIP runtime call failed                    */
#define STV_ESTATE (-4)     /* call made in the wrong state                 */
#define STV_ESINGULAR (-5)  /* zero pivot in a local or the coarse factor   */
#define STV_ENOCONV (-6)    /* GMRES hit max_it without reaching rtol       */
#define STV_ENUMERIC (-7)   /* NaN or Inf met in the Krylov process         */

/* ---- storage of the pre-computed cell inverses (Section 4.3) ---- */
#define STV_F64 0           /* stored and applied in FP64                   */
#define STV_F32 1           /* factorised in FP64, stored in FP32           */
#define STV_STORE_FULL 2    /* flag: keep every row of J_T^-1 (default keeps
                               only the rows of DoFs the cell owns, which are
                               the only ones the last-writer sweep uses)    */

/* ---- how a sweep combines the corrections of cells sharing a DoF ---- */
#define STV_LAST_WRITER 0   /* DoF takes the correction of the last cell in
                               loop order that contains it (Section 4.2)     */
#define STV_POU 1           /* average of the cells' corrections             */
#define STV_ADDITIVE 2      /* sum of the cells' corrections                 */

typedef struct stv_ctx stv_ctx;

/*
 * One level of the hierarchy (all pointers HOST, deep-copied).
 *   n_sdofs     spatial DoFs N_s of the level (space-time size N_s*(k+1)).
 *   bsr_rowptr  [n_sdofs+1] block-row pointers, bsr_rowptr[0] = 0.
 *   bsr_col     [nnzb] spatial column of each block, strictly increasing per row.
 *   bsr_val     [nnzb*(k+1)*(k+1)] block (s, s') row-major: entry i*(k+1)+l is
 *               J[(s, i), (s', l)] (test time DoF i, trial time DoF l).
 *   n_cells     cells of the level, in smoother loop order.
 *   n_ls        spatial DoFs per cell: dim*3^dim + dim + 1 (21 in 2d, 85 in 3d).
 *   cell_sdofs  [n_cells*n_ls] global spatial DoFs of each cell in local order:
 *               velocity component-major over the lexicographic Q2 nodes, then
 *               the dim+1 pressure modes (the spatial part of eq. (4.4)).
 *   P_*         spatial prolongation from level-1 to this level, CSR with
 *               n_sdofs rows and the coarser level's n_sdofs columns (identity
 *               in time).  Ignored (may be NULL) on level 0.
 * A pair of DoFs sharing a cell may be absent from the block pattern; its
 * block is then zero (in J and in every local Jacobian J_T).
 */
typedef struct stv_level {
  int32_t n_sdofs;
  const int32_t* bsr_rowptr;
  const int32_t* bsr_col;
  const double* bsr_val;
  int64_t nnzb;
  int32_t n_cells;
  int32_t n_ls;
  const int32_t* cell_sdofs;
  const int32_t* P_rowptr;
  const int32_t* P_col;
  const double* P_val;
  int64_t P_nnz;
} stv_level;

/* V(nu1, nu2) cycle parameters (Algorithm 4.1; damping omega of Section 5.3). */
typedef struct stv_mg_params {
  int32_t nu1;      /* pre-smoothing sweeps, >= 0                */
  int32_t nu2;      /* post-smoothing sweeps, >= 0               */
  double omega;     /* damping of every sweep, > 0               */
  int32_t mode;     /* STV_LAST_WRITER, STV_POU or STV_ADDITIVE  */
} stv_mg_params;

/* Flexible GMRES(restart) parameters. */
typedef struct stv_gmres_params {
  int32_t restart;      /* Krylov dimension per cycle, 1..256                  */
  int32_t max_it;       /* total Arnoldi steps allowed                         */
  double rtol;          /* stop when ||b - J x||_2 <= rtol ||b||_2             */
  int32_t use_x0;       /* 1: start from the x passed in; 0: from x = 0        */
  int32_t fixed_iters;  /* > 0: run exactly this many steps, ignore rtol       */
  stv_mg_params mg;     /* preconditioner                                     */
} stv_gmres_params;

/* Results of stv_gmres_solve.  history (optional, caller-owned host array of
 * history_cap doubles) receives ||r_j|| / ||b|| for j = 0 .. iters. */
typedef struct stv_gmres_info {
  int32_t iters;
  int32_t restarts;
  int32_t converged;
  double true_relres;
  double* history;
  int32_t history_cap;
  int32_t history_len;
} stv_gmres_info;

/* Create a context bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  The caller owns *out until
 * stv_destroy.  Errors: STV_EINVAL, STV_EHIP, STV_ENOMEM. */
int stv_create(stv_ctx** out, int device, void* hip_stream);

/* Free the context and all device memory it holds.  NULL is allowed. */
void stv_destroy(stv_ctx* ctx);

/* Text of the last error raised on this context ("" if none).  ctx may be
 * NULL, which returns the text of the last failed stv_create. */
const char* stv_last_error(const stv_ctx* ctx);

/* Host-only validation of a hierarchy (the checks stv_set_hierarchy runs
 * before touching the device): sizes, sorted unique block columns, cell DoFs
 * in range and distinct within a cell, every DoF in some cell, prolongation
 * shapes.
 * Writes a message naming the offending field into err (errlen bytes). */
int stv_validate_hierarchy(int n_levels, int dim, int k, const stv_level* lv,
                           char* err, size_t errlen);

/* Upload a hierarchy (levels 0..n_levels-1, 1 <= n_levels <= 16, dim 2 or 3,
 * 0 <= k <= 3).  Builds on the host the per-cell lists of owned DoFs (the
 * owner of a DoF is the last cell in loop order that contains it) and the
 * transposed prolongations.  Replaces any previous hierarchy and drops the
 * inverses.  Synchronises the stream.  Errors: STV_EINVAL, STV_ENOMEM, STV_EHIP. */
int stv_set_hierarchy(stv_ctx* ctx, int n_levels, int dim, int k, const stv_level* lv);

/* Upload n_inst independent hierarchies as one batch (same dim and k; each
 * instance i has n_levels[i] levels, levels[i] pointing to its level array,
 * index 0 the coarsest; every array is validated as in stv_set_hierarchy and
 * deep-copied).  The instances are packed into block-diagonal levels aligned
 * at their finest level: packed level D-1 (D = max n_levels) holds every
 * instance's finest level, instance i's own level l sits at packed level
 * D - n_levels[i] + l, its rows after those of the instances before it.
 * Every other call then acts on all instances at once: finest-level vectors
 * are the instances' vectors concatenated (stv_instance_layout gives each
 * offset), a V-cycle runs every instance's own V-cycle (an instance whose
 * coarsest level is packed level g is solved directly there), and
 * stv_gmres_solve runs an independent FGMRES per instance, in lockstep, each
 * with its own Krylov space, stopping test and true residual
 * (stv_instance_info).  A single hierarchy is the batch of one.  Replaces any
 * previous hierarchy.  Errors as stv_set_hierarchy (messages name the
 * instance); STV_EINVAL if a packed level exceeds 32-bit indexing. */
int stv_set_batch(stv_ctx* ctx, int n_inst, int dim, int k, const int* n_levels,
                  const stv_level* const* levels);

/* Where instance inst lives: its number of levels, the first spatial row
 * of its finest level in the packed finest level and its spatial row count
 * (vector elements: times k+1). */
int stv_instance_layout(stv_ctx* ctx, int inst, int* n_levels, int64_t* row_offset,
                        int64_t* n_rows);

/* Result of the last stv_gmres_solve for instance inst (iters, restarts,
 * converged, true_relres; no history). */
int stv_instance_info(stv_ctx* ctx, int inst, stv_gmres_info* info);

/* Extract every local Jacobian J_T (the submatrix of the level matrix on the
 * cell's DoFs, Section 4.2) on levels >= 1, invert it by Gauss-Jordan
 * elimination with partial pivoting in FP64 and store it (Section 4.3);
 * factor the coarsest matrix densely (its explicit inverse) in FP64; with
 * spatial factors on the coarsest level, the diagonal blocks of its
 * time-decoupled form are inverted instead (each the real form of a complex
 * matrix) and stv_coarse_solve applies them with the time transforms, so the
 * whole inverse is never formed.
 * With spatial factors on a level (stv_set_kron_factors) whose cell problems
 * fit one wavefront (n_ls = 21, k + 1 <= 3) and the owned-rows layout, the
 * level's inverses are stored time-decoupled: with D^-1 C = V T V^-1 (real
 * Jordan form), J_T^-1 = (I (x) V) Q^-1 (I (x) W), Q = M_T (x) T + A_T (x) I,
 * W = V^-1 D^-1, and Q^-1 is block diagonal in time, so one row of
 * (k+1)*n_ls values per owned spatial DoF is kept instead of k+1 rows (the
 * sweep applies the same J_T^-1).  The layout is fixed by the build that
 * made the store.
 * storage = STV_F64 or STV_F32, optionally | STV_STORE_FULL.  The stores
 * and the build's work buffers are owned by the context and kept between
 * builds of one hierarchy (remade when the storage flags or the coarse
 * algorithm change; a changed hierarchy frees them).  Synchronises the
 * stream.  On a zero pivot returns STV_ESINGULAR and, if non-NULL, sets
 * *bad_level and *bad_cell (bad_cell = -1 for the coarse matrix); the
 * inverses are then unusable until the next successful build.
 * Errors: STV_ESTATE (no hierarchy), STV_EINVAL, STV_ENOMEM, STV_EHIP. */
int stv_build_cell_inverses(stv_ctx* ctx, int storage, int* bad_level, int* bad_cell);

/* out = r - J_level d: the level residual that Algorithm 4.1 restricts to the
 * next coarser level and that every smoothing step of eq. (4.6) starts from.
 * r may be NULL (then out = -J d).  Device pointers, N_s*(k+1) doubles each,
 * time-inner; out must not alias r or d.  Asynchronous on the context's
 * stream.  Errors: STV_ESTATE (no hierarchy), STV_EINVAL (level out of range
 * or NULL d/out). */
int stv_residual(stv_ctx* ctx, int level, const double* r, const double* d, double* out);

/* n_sweeps damped Vanka sweeps on level >= 1, in place on d:
 *   rho = r - J d (once per sweep, from the pre-sweep iterate);
 *   for every cell T: c_T = omega J_T^-1 rho_T;
 *   d_j += c_T(j) with T chosen per mode (STV_LAST_WRITER: the owner of j).
 * eq. (4.6) with the damping of Section 5.3.  STV_POU and STV_ADDITIVE need
 * inverses stored with STV_STORE_FULL.  Errors: STV_ESTATE (no inverses or
 * incompatible storage), STV_EINVAL. */
int stv_vanka_sweep(stv_ctx* ctx, int level, const double* r, double* d,
                    int n_sweeps, double omega, int mode);

/* r_c = P^T rho (restriction to level-1; the transpose of the prolongation,
 * Section 4.1).  level >= 1; rho has the size of `level`, r_c of level-1. */
int stv_restrict(stv_ctx* ctx, int level, const double* rho, double* r_c);

/* d += P d_c (prolongation of a level-1 correction to `level` >= 1). */
int stv_prolongate_add(stv_ctx* ctx, int level, const double* d_c, double* d);

/* d = J_0^-1 r on the coarsest level (the direct coarse solve; for a batch,
 * the instances whose coarsest level is packed level 0). */
int stv_coarse_solve(stv_ctx* ctx, const double* r, double* d);

/* d = MG(r): one V(nu1, nu2) cycle on the finest level from d = 0
 * (Algorithm 4.1 read with the residual r_g - J_g d_g, the recursion result
 * assigned to d_{g-1}, prolongation of d_{g-1}, post-smoothing against the
 * original r_g).  r and d are finest-level device vectors, d must not alias r. */
int stv_vcycle(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p);

/* For callers that cannot allocate device memory (code under stream or HIP
 * graph capture, allocation-free serving loops): stv_vcycle with its level
 * work vectors (per level the residual, and the restricted right-hand side
 * and correction of every level below the finest; with STV_POU/STV_ADDITIVE
 * also the per-cell corrections) taken from a fixed device workspace of
 * 64 MiB that the library holds on every device it runs on until the process
 * ends, instead of the context's own buffers.  The call allocates nothing,
 * launches eagerly on the context's stream (never the captured graph) and is
 * not recorded by stv_set_timing.  Same arguments and results as stv_vcycle
 * (bitwise).  Every call on one device shares that workspace and leaves the
 * last call's values in it: calls that overlap on one device (several
 * contexts or streams) race, so the caller orders them.  Errors: as
 * stv_vcycle; STV_EINVAL if the hierarchy's work vectors exceed 64 MiB (the
 * message gives both sizes); STV_EHIP if the workspace has no address on the
 * context's device. */
int stv_vcycle_noalloc(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p);

/* Solve J x = b on the finest level by right-preconditioned flexible GMRES
 * (x = x0 + Z y with z_j = MG(v_j)), FP64 throughout: the linear solver of
 * every Newton step of Section 3 (its Newton linear system), preconditioned
 * by the V-cycle of Algorithm 4.1 (Section 4.1); the paper's robustness study
 * (Section 5.3) caps it at 1000 steps, which is max_it's usual value.  The
 * restart length is the caller's (the paper gives none).  A cycle ends when the
 * rotated residual estimate reaches rtol ||b|| or after `restart` steps; the
 * iterate is updated and the true residual decides convergence.  b and x are
 * device vectors.  Synchronises the stream.  Returns STV_ENOCONV (x holds the
 * last iterate) or STV_ENUMERIC (NaN/Inf) on failure; info is filled in all
 * cases where it is non-NULL. */
int stv_gmres_solve(stv_ctx* ctx, const double* b, double* x,
                    const stv_gmres_params* p, stv_gmres_info* info);

/* Adjoint solves: the same V-cycle and FGMRES for the transposed system
 * J^T x = b.  The level operators become J_g^T (built once per hierarchy on
 * first use), the smoother the Vanka sweep of J^T, whose local inverses
 * (J_T^T)^-1 = (J_T^-1)^T are the stored ones read transposed (so the
 * inverses must be built with STV_STORE_FULL), with the same owner rule;
 * the transfers are unchanged and the coarse solve applies the transposed
 * coarse inverse.  Last-writer mode only.  Errors as stv_vcycle /
 * stv_gmres_solve, and STV_ESTATE without full inverses. */
int stv_vcycle_transposed(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p);
int stv_gmres_solve_transposed(stv_ctx* ctx, const double* b, double* x,
                               const stv_gmres_params* p, stv_gmres_info* info);

/* Cellwise bilinear form of two device vectors of `level` (time-inner):
 *   out[T] = sum_l tw[l] sum_{alpha,beta} lam[s_alpha, l] K_T[alpha][beta] x[s_beta, l]
 * for every smoothed cell T of the level, with the spatial matrix
 * K_T = sum_{e = kptr[T]}^{kptr[T+1]-1} kw[e] Kref[kidx[e]] built from n_ref
 * reference matrices (n_ls x n_ls row-major each, in the spatial order of
 * eq. (4.4)).  With K_T the viscosity derivative of the cell's element
 * matrix this is the per-cell term lam_c^T K_c x_c of an adjoint gradient.
 * Kref, kptr, kidx, kw, tw are host arrays (copied); lam, x, out device
 * (out: one double per cell).  Synchronises.  Errors: STV_EINVAL. */
int stv_cell_contract(stv_ctx* ctx, int level, const double* lam, const double* x, int n_ref,
                      const double* Kref, const int32_t* kptr, const int32_t* kidx,
                      const double* kw, const double* tw, double* out);

/* out[k] = sum over cell cells[k]'s DoFs of lam times f[k] (f: host, n x
 * n_loc, cell-local order alpha*(k+1) + l); out is a device array of n
 * doubles.  Synchronises.  Errors: STV_EINVAL. */
int stv_cell_dot(stv_ctx* ctx, int level, const double* lam, int n, const int32_t* cells,
                 const double* f, double* out);

/* The cellwise gradient terms in one pass: for every smoothed cell T of
 * `level`,
 *   out[T] = sc * (the stv_cell_contract form of T) + sf * lam_T . f[k]
 * where the second term is present only for T = cells[k] (cells distinct,
 * f a host array of n x n_loc values in the cell-local order
 * alpha*(k+1) + l).  For an operator affine in each cell's viscosity, the
 * viscosity derivative of the local matrices of Sec. 2.3 eq. (2.5) as K_T,
 * sc = -1 and f the viscosity derivative of the right-hand side scaled by
 * sf, this is the adjoint gradient dL/dnu_T = -lam^T (dJ/dnu_T) x +
 * lam^T (db/dnu_T).  Host arrays are copied; lam, x, out are device arrays
 * (out: one double per cell).  Synchronises.  Errors: STV_EINVAL (a cell
 * out of range or listed twice, a non-finite scale, bad kptr/kidx). */
int stv_cell_gradient(stv_ctx* ctx, int level, const double* lam, const double* x, int n_ref,
                      const double* Kref, const int32_t* kptr, const int32_t* kidx,
                      const double* kw, const double* tw, double sc, int n,
                      const int32_t* cells, const double* f, double sf, double* out);

/* Cellwise terms added into a device vector y of `level` (time-inner):
 *   y[DoF j of cell cells[k]] += coef[k] * f[k][j]
 * for k < n (f: host, n x n_loc in the cell-local order alpha*(k+1) + l;
 * coef: host, n values) - the assembly of a right-hand side whose cell
 * contributions scale with a per-cell coefficient (Sec. 2.3: the load
 * vector of eq. (2.5) with a cellwise viscosity).  The terms of a DoF are
 * summed in list order by one thread (deterministic).  Synchronises.
 * Errors: STV_EINVAL. */
int stv_cell_scatter(stv_ctx* ctx, int level, int n, const int32_t* cells, const double* coef,
                     const double* f, double* y);

/* out[i] = a_i . b_i for every instance i of two finest-level device vectors
 * (out: host array of n_inst doubles).  Synchronises. */
int stv_dot(stv_ctx* ctx, const double* a, const double* b, double* out);

/* Copy the stored inverse of cell `cell` on `level` (>= 1) into the host array
 * out[n_loc*n_loc], row-major in the cell-local order of eq. (4.4)
 * (time-major: index l*n_ls + alpha), converted to FP64.  Rows not stored
 * (the default owned-rows storage) are written as NaN.  A time-decoupled
 * store (see stv_build_cell_inverses) is expanded on the host to the same
 * rows of J_T^-1.  Synchronises. */
int stv_get_cell_inverse(stv_ctx* ctx, int level, int cell, double* out);

/* Sizes of a level: spatial DoFs, cells, local DoFs per cell (n_loc), stored
 * inverse bytes of the level (0 before stv_build_cell_inverses). */
int stv_level_info(stv_ctx* ctx, int level, int64_t* n_sdofs, int64_t* n_cells,
                   int64_t* n_loc, int64_t* inverse_bytes);

/* Options (take effect at the next stv_build_cell_inverses):
 *   STV_OPT_COARSE_ALGO: how the coarsest matrix is inverted by Gauss-Jordan
 *   elimination with partial pivoting: 0 = chosen by size (default: 1 up
 *   to order 256, 3 above),
 *   1 = one level of narrow panels, each updating the whole matrix,
 *   2 = slabs of 64 (128 above order 5120) columns eliminated by narrow
 *   panels, then one rank-64 (128) update of the rest on the matrix cores
 *   (1 and 2 give the same pivots),
 *   3 = the slabs of 2 with panels of 16 columns whose pivot rows are chosen
 *   by a tournament: 64-row chunks propose rows by partial pivoting on their
 *   own rows and the proposals are merged by partial pivoting up a tree
 *   (the pivots can differ from 1 and 2; the inverse agrees to rounding).
 *   With spatial factors on the coarsest level (stv_set_kron_factors) the
 *   coarse inverse is assembled from the diagonal blocks of the operator in
 *   the real Jordan basis of its time matrix, each built as the real form
 *   of a complex matrix of order n_s; with 3 (and 0 above order 256) the
 *   tournament takes complex pivots there (16 per panel of 32 real
 *   columns), with 1 and 2 the real schedules run on the same real forms.
 * Errors: STV_EINVAL (unknown option or value). */
#define STV_OPT_COARSE_ALGO 1
/*   STV_OPT_GRAPH: 1 = the V-cycle (stv_vcycle and the preconditioner of
 *   stv_gmres_solve) is captured once into a HIP graph and replayed: one
 *   graph launch plus two vector copies instead of one launch per kernel.
 *   The graph is recaptured when the hierarchy, the inverses or the cycle
 *   parameters change.  Per-kernel timing then reports the whole replay
 *   (class 7) instead of the kernels inside it.  0 = eager launches
 *   (default).  Results are identical in both modes. */
#define STV_OPT_GRAPH 2
/*   STV_OPT_COARSE_OVERLAP: 1 (default) = the coarse factorisations run on
 *   an internal stream concurrently with the cell inverses; 0 = they run on
 *   the caller's stream before the cell inverses.  Same results. */
#define STV_OPT_COARSE_OVERLAP 3
/*   STV_OPT_INVERSE_CUS: while the coarse factorisation runs concurrently,
 *   the 3d complex cell-inverse kernel (one cell per compute unit) runs as at
 *   most this many resident workgroups striding over the cells, leaving the
 *   remaining compute units to the coarse chain; 0 (default) = no cap, -1 =
 *   five eighths of the device's compute units.  Same results. */
#define STV_OPT_INVERSE_CUS 4
/*   STV_OPT_COARSE_LOOKAHEAD: 1 (default) = in the complex-pivot coarse
 *   chain the next slab's columns are updated first and the other columns on
 *   an internal stream, concurrent with the next slab's panels; 0 = one
 *   update per slab on the chain's stream.  Same results. */
#define STV_OPT_COARSE_LOOKAHEAD 5
int stv_set_option(stv_ctx* ctx, int option, int64_t value);

/* Spatial factors of a level whose operator has time-independent
 * coefficients (the Oseen linearisation): every block (i, l) of the level
 * matrix is C[i][l] M(s, s') + delta_il tw[i] A(s, s') (C: (k+1)^2
 * row-major, tw: k+1).  mval and aval hold M and A in the level's block
 * pattern (one value per block, in the order of bsr_col; for a batch, the
 * packed level's order).  The library checks on the device that the factors
 * reproduce the stored blocks (to 1e-12 of the largest entry; otherwise
 * STV_EINVAL) and from then on computes the level's residual from them,
 * streaming two values per block instead of (k+1)^2; transposed solves keep
 * using the blocks.  mval = aval = NULL drops the factors.  Host arrays,
 * copied.  Synchronises. */
int stv_set_kron_factors(stv_ctx* ctx, int level, const double* mval, const double* aval,
                         const double* C, const double* tw);

/* Launch shapes of the level kernels of one level: spmv_rows = shape of the
 * residual (1..12, default 2): with the blocks, block rows per wavefront (5
 * to 12 act as 4); with spatial factors, (lanes per block row, blocks per
 * lane and round) = (4,4), (8,3), (8,4), (16,2), (16,4), (32,2) over one
 * list of (m, a) pairs per row (1..6), or the same six over two lists per
 * row, the blocks with a mass entry as (m, a) pairs and the others as a
 * alone (7..12: fewer bytes, more rounds); sweep_wgs = workgroups
 * of the Vanka sweep, 0 (default) for one wavefront per cell, otherwise a
 * persistent launch of that many workgroups whose wavefronts stride over the
 * cells.  The residual's summation order depends on spmv_rows (results
 * agree to rounding); the sweep's results do not depend on sweep_wgs.
 * Errors: STV_ESTATE (no hierarchy), STV_EINVAL. */
int stv_set_launch(stv_ctx* ctx, int level, int spmv_rows, int sweep_wgs);

/* Launch shapes of the transfers between `level` >= 1 and level-1: shape t
 * in 1..5 takes 2^(t-1) lanes per row (1, 2, 4, 8, 16), p_shape for the
 * prolongation P (rows of `level`), pt_shape for the restriction by its
 * transpose (rows of level-1); 0 keeps the current shape.  cur_p and cur_pt,
 * when non-NULL, receive the shapes in force afterwards.  The summation order
 * of a row depends on its shape (results agree to rounding).  Errors:
 * STV_ESTATE (no hierarchy), STV_EINVAL. */
int stv_transfer_shapes(stv_ctx* ctx, int level, int p_shape, int pt_shape, int* cur_p,
                        int* cur_pt);

/* Autotuner: on every smoothed level, time each residual shape (1..4 with
 * the blocks, 1..12 with spatial factors) and
 * each sweep shape (one wavefront per cell, or persistent
 * grids of 2, 4, 8, 16, 32 workgroups per compute unit) on the device, five
 * launches each after one untimed launch, and keep the fastest.  The same
 * for the transfers of every level with a prolongation: 1, 2, 4, 8 or 16
 * lanes per row, for P and for its transpose separately (without the
 * autotuner, the lanes follow the mean row length: 1 below 3 entries, then
 * 2, 4, 8, 16 below 6, 12, 24 and above; the transfers' summation order
 * depends on the lanes, results agree to rounding).  Needs the
 * inverses (the sweep is timed with the stored ones); uses temporary device
 * vectors; the hierarchy's data are not modified.  If choices is non-NULL
 * it receives, for level g < cap/2, choices[2g] = residual shape and
 * choices[2g+1] = sweep workgroups.  Synchronises the stream. */
int stv_autotune(stv_ctx* ctx, int* choices, int cap);

/* Per-kernel timing with HIP events on the context's stream.
 * stv_set_timing(ctx, 1) starts recording (and clears the counters);
 * stv_kernel_stats returns launches and total milliseconds of one kernel
 * class on one level (level = -1: all levels): 0 = Vanka cell sweep,
 * 1 = level residual / matrix-vector product, 2 = transfers, 3 = coarse
 * apply, 4 = Krylov vector kernels, 5 = cell inverse build, 6 = coarse
 * factorisation, 7 = V-cycle graph replay.  Synchronises the stream. */
int stv_set_timing(stv_ctx* ctx, int on);

/* Restricts the recording to the kernel classes whose bit (1 << class) is
 * set in class_mask and to the levels whose bit (1 << level) is set in
 * level_mask (default: all of both; launches not tied to a level count as
 * level 0).  Launches of the sweep, residual, transfer and coarse-apply
 * classes are timed by the kernel's own start and end stamps
 * (hipExtLaunchKernel events), the other classes by event records around
 * them.  Synchronises the stream.  Errors: STV_EINVAL (a class bit beyond
 * the last class). */
int stv_set_timing_filter(stv_ctx* ctx, unsigned class_mask, unsigned level_mask);
int stv_kernel_stats(stv_ctx* ctx, int kernel_class, int level, int64_t* launches,
                     double* total_ms);

#ifdef __cplusplus
}
#endif

#endif /* STV_H */
