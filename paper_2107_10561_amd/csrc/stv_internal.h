// Internal declarations of the space-time Vanka multigrid library: device
// data of a level, the context, and the host-side launchers of every kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cstdint>
#include <string>
#include <vector>

#include "stv.h"

namespace stv {

constexpr int kMaxLevels = 16;
constexpr int kMaxB = 4;             // k <= 3
constexpr int kMaxRestart = 256;
constexpr int kDotBlocks = 1024;     // partial sums per Krylov reduction
constexpr int kKrylovFuse = 8;       // basis vectors of a fused Gram-Schmidt update + products

enum KernelClass {
  KC_SWEEP = 0, KC_RESIDUAL, KC_TRANSFER, KC_COARSE, KC_KRYLOV, KC_INVERSE, KC_COARSE_FACTOR,
  KC_GRAPH, KC_COUNT
};

// Time decoupling of the cell problems of a level with spatial factors
// (cell matrix J_T = M_T (x) C + A_T (x) D, spatial index outer, D =
// diag(tw)): with D^-1 C = V T V^-1 (T real block diagonal, blocks of order
// sz[p] starting at time component first[p]),
//   J_T^-1 = (I (x) V) Q^-1 (I (x) W),  Q = M_T (x) T + A_T (x) I,  W = V^-1 D^-1.
// Q couples time components only inside a block; its inverse is stored per
// owned spatial DoF a as one row of B * n_loc values: for each block p, at
// columns off[p] + s (s < n_loc), Q^-1[(a, f), (s, f)] (f = first[p]), and
// for a pair also, at off[p] + n_loc + s, Q^-1[(a, f + 1), (s, f)] (the real
// and imaginary parts of the inverse of the complex block).  T, V, W are
// b x b, row-major.
struct CellSplit {
  int b, nblk;
  int sz[4], first[4], off[4];
  double T[16], V[16], W[16];
};

// Device arrays of one level.
struct DevLevel {
  int32_t n_s = 0, n_cells = 0, n_ls = 0;
  int64_t nnzb = 0;
  int32_t* rowptr = nullptr;      // [n_s+1]
  int32_t* col = nullptr;         // [nnzb]
  double* val = nullptr;          // [nnzb*b*b]
  int32_t* cell_sdofs = nullptr;  // [n_cells*n_ls]
  // owned DoFs: cell T owns own_loc[own_ptr[T] .. own_ptr[T+1]) (local alpha)
  int32_t* own_ptr = nullptr;     // [n_cells+1]
  uint8_t* own_loc = nullptr;     // [total owned]
  // incidence for the POU / additive modes: spatial DoF s belongs to cells
  // inc_cell[inc_ptr[s] .. inc_ptr[s+1]) at local index inc_loc[...]
  int32_t* inc_ptr = nullptr;
  int32_t* inc_cell = nullptr;
  uint8_t* inc_loc = nullptr;
  // prolongation from the coarser level (levels >= 1): P (n_s x n_s_coarse)
  // and its transpose, CSR
  int32_t* P_rowptr = nullptr; int32_t* P_col = nullptr; double* P_val = nullptr;
  int32_t* Pt_rowptr = nullptr; int32_t* Pt_col = nullptr; double* Pt_val = nullptr;
  int32_t n_s_coarse = 0;
  // transfer shapes (1..kTransferShapes: 2^(shape-1) lanes per row) of P and
  // of its transpose
  int p_shape = 1, pt_shape = 1;
  // block position of each cell DoF pair (levels >= 1), n_cells * n_ls^2
  int32_t* posmap = nullptr;
  // stored inverses (levels >= 1)
  int64_t* inv_off = nullptr;     // [n_cells] element offset of each cell's block
  void* inv_store = nullptr;
  int inv_ld = 0;                 // row stride of the stored rows (n_loc)
  int64_t inv_elems = 0;
  // work vectors (n_s*b each)
  double* rho = nullptr;
  double* r = nullptr;
  double* d = nullptr;
  double* corr = nullptr;         // [n_cells*n_loc] per-cell corrections (POU/additive)
  // host copies kept for validation / export
  std::vector<int32_t> h_own_ptr;
  std::vector<uint8_t> h_own_loc;
  std::vector<int32_t> h_csd;     // cell DoF lists (n_cells x n_ls)
  int64_t n_cells_all = 0;        // cells of every member, the coarse ones included
  // launch shapes (chosen by the autotuner or set explicitly)
  // transposed level matrix (built on first use by a transposed solve)
  int32_t* rowptr_t = nullptr; int32_t* col_t = nullptr; double* val_t = nullptr;
  // spatial factors (optional): blocks = C[i][l] M + delta_il tw[i] A
  double* kron_ma = nullptr;      // spatial factors (m, a), interleaved per block
  // the factors split per row for the residual: the blocks with m != 0 as
  // (m, a) pairs, then those with m = 0 as a only; kx_ptr holds both row
  // pointer arrays (n_s + 1 each), kx_col the two column lists (kx_n1 + the
  // rest), kx_val the 2 kx_n1 pair values followed by the a-only values
  int32_t* kx_ptr = nullptr;
  int32_t* kx_col = nullptr;
  double* kx_val = nullptr;
  int64_t kx_n1 = 0;
  int dec = 0;                    // the inverse store holds time-decoupled rows (CellSplit)
  int cx = 0;                     // inverses built from the complex decoupled block (plain store)
  CellSplit split{};
  // per lane j of the decoupled sweep: W[j % B][.] and V[j % B][.] (2B x 64,
  // row-major), and a code word: source lanes of u (bits 0-5, 6-11) and the
  // multipliers (2 bits per output: 0 = 0, 1 = +1, 3 = -1; from bit 12 for
  // the first source, from bit 12 + 2B for the second)
  double* dec_tab = nullptr;
  int32_t* dec_code = nullptr;
  double kron_C[16] = {}, kron_tw[4] = {};
  int spmv_rpw = 2;               // residual shape: 1..4 (blocks), 1..12 (factors)
  int sweep_wgs = 0;              // workgroups of a persistent sweep (0: one wavefront per cell)
};

// One dense coarse member: an instance whose coarsest level is stored in the
// packed level that holds rowptr/col/val, at spatial rows [row_off,
// row_off + n_s); its inverse (n_s*b square, row-major) sits at inv_off of
// the coarse store.
struct CoarseDesc {
  const int32_t* rowptr;
  const int32_t* col;
  const double* val;
  int32_t row_off, n_s;
  int64_t inv_off;
};

// Work buffers of a batched dense Gauss-Jordan inversion: each array holds
// one slice per matrix at the given stride (elements).
struct GjWork {
  double* A; int64_t sA;          // n x n matrices
  int* rpiv; uint8_t* used; int64_t sV;   // n pivot records / flags
  double* B; int64_t sB;          // pivot rows, max(nb, no) x n
  double* P; int64_t sP;          // two panel buffers, 2 x n x nb
  double* S; int64_t sS;          // two slab buffers, 2 x n x no
  double* Bin; int64_t sBin;      // pivot rows of a slab, nb x no
  // tournament schedule: candidate pivot rows of each workgroup and of the
  // merge tree's nodes, the two panel right factors (2 x nb x no) and the
  // arrival counters of the merge tree (sK per matrix)
  int* cand; int64_t sC;
  double* Z; int64_t sZ;
  unsigned* counter; int64_t sK;
};

// Dense Gauss-Jordan plan: algo 1 = one level of panels (width nb), 2 = slabs
// of no columns eliminated by panels of nb, 3 = slabs whose panels take
// tournament-chosen pivot rows; the matrix is padded to a multiple of pad;
// max_n is the largest supported order.  pair (algo 3 only): the matrix is
// the real form of a complex matrix (entry x of complex row i, column j at
// real rows 2i, 2i+1 and columns 2j, 2j+1 as [[Re x, -Im x], [Im x, Re x]])
// and the tournament chooses complex pivots, nb / 2 per panel of nb real
// columns.
struct GjPlan { int algo, cfg, nb, no, pad; int64_t max_n; bool pair; };

// One diagonal block of a coarse member's time-decoupled operator, built
// from the member's spatial factors in the real form of a complex matrix:
// B[2s + a, 2s' + c] = T[a][c] M(s, s') + delta_ac A(s, s') (a, c < 2).  A
// complex pair al +- i be has T = [[al, be], [-be, al]], the real form of the
// complex matrix al M + A - i be M; a real eigenvalue lambda has T = lambda I
// (two uncoupled copies of lambda M + A).
struct KronBlockDesc {
  const int32_t* rowptr; const int32_t* col; const double* ma;
  int32_t row_off, n_s;
  double t[4];
};

// A coarse member inverted through time decoupling: its inverse is
//   J^-1[(s, i), (s', l)] = sum_p sum_{a, c < sz_p} V[i][f_p + a] Binv_p[2s + a, 2s' + c] W[f_p + c][l]
// (Binv_p of order 2 n_s in real form; f_p = first[p]; time-inner rows
// s * b + i), applied from the blocks without being formed.  Binv_p is read
// where the elimination left it: Binv_p[i, j] = S_p[rpiv_p[i], rinv_p[j]]
// (S_p row-major with leading dimension ld_p; rinv_p the inverse of
// rpiv_p).  paired[p]: the block was eliminated with complex pivots, so its
// pivot records pair real rows 2r, 2r + 1 with real columns 2t, 2t + 1 and
// S_p keeps the exact 2 x 2 structure of the real form.  The member's rows
// start at spatial row row_off of its packed level.
struct KronCoarse {
  const double* S[4];
  const int* rpiv[4];
  const int* rinv[4];
  int64_t ld[4];
  int paired[4];
  int nblk;
  int sz[4], first[4];
  int32_t n_s, row_off;
  double V[16], W[16];
};

// The coarse members of one order, eliminated by one batched Gauss-Jordan:
// members (packed level, index in that level), their device descriptors,
// the elimination buffers and the inverse pivot permutations.
struct CoarseGroup {
  int64_t n0 = 0, np = 0;
  GjPlan plan{};
  std::vector<int> lev, idx;
  CoarseDesc* d_desc = nullptr;
  GjWork w{};
  int* rinv = nullptr;
  // blocks of time-decoupled members instead of whole members, each padded
  // with the identity to the group's order n0: their descriptors (desc then
  // holds n_s = block order, b = 1); a block's inverse stays in its slice of
  // w.A with its pivot records (not unpermuted)
  bool kron = false;
  std::vector<int> part;          // kron: which block of its member each slot is
  KronBlockDesc* d_kdesc = nullptr;
};

// Start and stop events for the next kernel launched through stv::launch:
// hipExtLaunchKernel stamps them at the kernel's own start and end, so a
// timed launch needs no marker packets around it.  The launch clears them.
struct LaunchEvents { hipEvent_t start = nullptr, stop = nullptr; };
extern thread_local LaunchEvents g_launch_events;

template <typename... P, typename... A>
inline void launch(void (*kernel)(P...), dim3 grid, dim3 block, uint32_t shm, hipStream_t s,
                   A... args) {
  const LaunchEvents ev = g_launch_events;
  g_launch_events = LaunchEvents{};
  hipExtLaunchKernelGGL(kernel, grid, block, shm, s, ev.start, ev.stop, 0u,
                        static_cast<P>(args)...);
}

// Results of the last solve for one instance.
struct InstInfo { int iters = 0, restarts = 0, converged = 0; double relres = 0.0; };

struct TimerPair { hipEvent_t a, b; int cls; int level; };

}  // namespace stv

struct stv_ctx {
  int device = 0;
  double* noalloc_ws = nullptr;   // this device's address of the fixed workspace (or NULL)
  hipStream_t stream = nullptr;
  hipStream_t side = nullptr;     // internal stream: coarse factorisation overlaps the cell inverses
  hipStream_t side2 = nullptr;    // internal stream: look-ahead updates of the coarse chain
  hipEvent_t ev_gj[2] = {nullptr, nullptr};
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  hipEvent_t ev_step[2] = {nullptr, nullptr};   // Arnoldi coefficients of a step reached the host
  std::string err;
  int n_levels = 0, dim = 0, k = 0, b = 0;
  stv::DevLevel lv[stv::kMaxLevels];
  bool have_hier = false;
  bool have_inv = false;
  int inv_fp32 = 0;
  int inv_full = 0;
  // instances: a single hierarchy is one instance; a batch packs many into
  // block-diagonal levels aligned at their finest level
  int n_inst = 0;
  std::vector<int> inst_levels;       // levels of each instance
  std::vector<int64_t> inst_row;      // first spatial row on the finest level (+ total)
  int64_t* seg_off = nullptr;         // device: first vector element per instance (+ total)
  int64_t max_seg = 0;                // longest instance vector on the finest level
  std::vector<stv::InstInfo> inst_info;
  // dense coarse members, per packed level: host descriptors of all of
  // them; device descriptors (and the largest order) of those whose inverse
  // is stored whole in coarse_inv
  std::vector<stv::CoarseDesc> h_coarse[stv::kMaxLevels];
  stv::CoarseDesc* d_coarse[stv::kMaxLevels] = {};
  int n_whole[stv::kMaxLevels] = {};
  int64_t coarse_max_n0[stv::kMaxLevels] = {};
  double* coarse_inv = nullptr;       // the whole inverses
  int64_t coarse_elems = 0;
  // inverse-build workspace, kept between builds of one hierarchy: the
  // store layout it was made for (full rows or owned rows, element type),
  // per-level cell statuses and scratch, the coarse groups (for the coarse
  // algorithm in cgroups_algo) and the report block (first flagged cell per
  // level, then one verdict per coarse member) with its pinned host mirror
  int inv_layout = -1, inv_type = -1;
  uint8_t* inv_status[stv::kMaxLevels] = {};
  double* inv_scratch[stv::kMaxLevels] = {};
  int inv_slots[stv::kMaxLevels] = {};
  std::vector<stv::CoarseGroup> cgroups;
  int cgroups_algo = -1;
  // coarse members inverted through time decoupling, per packed level:
  // applied from their blocks' inverses (device descriptors, one per member,
  // and the largest spatial order)
  std::vector<stv::KronCoarse> h_kc[stv::kMaxLevels];
  stv::KronCoarse* d_kc[stv::kMaxLevels] = {};
  int32_t kc_max_ns[stv::kMaxLevels] = {};
  int kc_max_blocks[stv::kMaxLevels] = {};
  int* inv_report = nullptr;
  int* h_report = nullptr;
  int n_report = 0;
  int coarse_algo = 0;          // STV_OPT_COARSE_ALGO
  int coarse_overlap = 1;       // STV_OPT_COARSE_OVERLAP
  int inverse_cus = 0;          // STV_OPT_INVERSE_CUS (0: no cap)
  int coarse_lookahead = 1;     // STV_OPT_COARSE_LOOKAHEAD
  int64_t scal_segs = 0;        // instances the scalar buffers are sized for
  // V-cycle replayed from a captured HIP graph (STV_OPT_GRAPH): the graph
  // reads g_in and writes g_out; it is captured on cap_stream and replayed
  // on the caller's stream, and recaptured when its key changes
  int transposed = 0;            // level operators act as J^T (adjoint solves)
  int use_graph = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t graph_exec = nullptr;
  double* g_in = nullptr;
  double* g_out = nullptr;
  int64_t graph_key[6] = {};    // generation, nu1, nu2, omega bits, mode, launches tuned
  int64_t generation = 0;       // bumped by every hierarchy / inverse change
  int64_t graph_replays = 0;
  // Krylov workspace (finest level)
  double* V = nullptr;          // (restart+1) x N
  double* Z = nullptr;          // restart x N
  double* w = nullptr;          // N
  double* rt = nullptr;         // N (true residual)
  double* partial = nullptr;    // kDotBlocks x 8
  double* scal = nullptr;       // device scalars
  double* hscal = nullptr;      // pinned host mirror
  double* hstep = nullptr;      // pinned: the coefficients of the next Arnoldi step (look-ahead)
  int ws_restart = 0;
  int64_t ws_n = 0;
  // timing
  bool timing = false;
  unsigned timing_mask = ~0u;     // kernel classes recorded while timing is on
  unsigned timing_levels = ~0u;   // levels recorded while timing is on
  std::vector<stv::TimerPair> pending;
  std::vector<hipEvent_t> pool;
  int64_t launches[stv::KC_COUNT][stv::kMaxLevels] = {};
  double total_ms[stv::KC_COUNT][stv::kMaxLevels] = {};
};

namespace stv {

// ---- kernel launchers (each returns the hipError_t of the launch) ----
// y = (r ? r : 0) + sx * (J x)
hipError_t launch_spmv(hipStream_t s, int b, const DevLevel& L, const double* r,
                       const double* x, double* y, double sx, bool transposed = false);
hipError_t launch_spmv_kron(hipStream_t s, int b, const DevLevel& L, const double* r,
                            const double* x, double* y, double sx);
hipError_t launch_kron_check(hipStream_t s, int b, const DevLevel& L, const double* ma,
                             const double* C, const double* tw, double* partial, int nblk);
// residual shapes available for a level (factors: lanes per row x blocks per lane)
int residual_shapes(const DevLevel& L);
hipError_t launch_bsr_transpose_vals(hipStream_t s, int b, const double* val, const int32_t* src,
                                     double* val_t, int64_t nnzb);
hipError_t launch_vanka_cells_t(hipStream_t s, int b, const DevLevel& L, const double* rho,
                                double* d, double omega, int zero_init, int fp32);
hipError_t launch_cell_contract(hipStream_t s, int b, const DevLevel& L, const double* lam,
                                const double* x, const double* Kref, const int32_t* kptr,
                                const int32_t* kidx, const double* kw, const double* tw,
                                double sc, const int32_t* fidx, const double* f, double sf,
                                double* out);
hipError_t launch_cell_scatter(hipStream_t s, const int64_t* dof, const int32_t* ptr,
                               const int32_t* ck, const int64_t* fi, const double* coef,
                               const double* f, int n_dof, double* y);
hipError_t launch_cell_dot(hipStream_t s, int b, const DevLevel& L, const double* lam,
                           const int32_t* cells, int n, const double* f, double* out);
hipError_t launch_dense_gemv_t(hipStream_t s, const CoarseDesc* desc, int cnt, int b,
                               int64_t max_n0, const double* inv, const double* x, double* y);
bool inverse_fits_regs(int b, int n_ls);
hipError_t launch_build_posmap(hipStream_t s, const DevLevel& L);
hipError_t launch_vanka_cells(hipStream_t s, int b, const DevLevel& L, const double* rho,
                              double* d, double omega, int zero_init, int fp32, int full);
hipError_t launch_vanka_cells_corr(hipStream_t s, int b, const DevLevel& L, const double* rho,
                                   double omega, int fp32);
hipError_t launch_vanka_combine(hipStream_t s, int b, const DevLevel& L, double* d, int pou);
// n_cu > 0 and reserve > 0 cap the grid of the one-wavefront inverse kernel
// (it strides over the cells) at the wavefronts per compute unit that leave
// `reserve` VGPRs free on every SIMD, so that the kernels of a concurrent
// stream find room beside it.
hipError_t launch_cell_inverses(hipStream_t s, int b, const DevLevel& L, int fp32, int full,
                                uint8_t* status, double* gscratch, int n_slots, int n_cu,
                                int reserve, int cu_cap = 0);
// transfers: shapes 1..kTransferShapes take 1, 2, 4, 8, 16 lanes per row;
// transfer_shape_for picks one from the mean row length
constexpr int kTransferShapes = 5;
int transfer_shape_for(int64_t nnz, int64_t n_rows);
hipError_t launch_restrict(hipStream_t s, int b, const DevLevel& L, const double* rho,
                           double* r_c);
hipError_t launch_prolongate_add(hipStream_t s, int b, const DevLevel& L, const double* d_c,
                                 double* d);
hipError_t launch_fill(hipStream_t s, double* x, int64_t n, double v);
hipError_t launch_copy(hipStream_t s, const double* x, double* y, int64_t n);
// dense coarse level
hipError_t launch_bsr_to_dense(hipStream_t s, int b, const CoarseDesc* desc, int cnt,
                               int32_t max_rows, double* A, int64_t sA, int64_t n);
GjPlan gj_plan(int64_t n, int algo /* 0 = choose by size */, bool pair);
// Second stream and events of the look-ahead of the complex-pivot slab
// schedule: the update of the columns other than the next slab's runs on s2
// beside the next slab's panels (next_ready: the next slab's columns are
// updated; done_rest: the other columns are).
struct GjAux {
  hipStream_t s2;
  hipEvent_t next_ready, done_rest;
};
hipError_t launch_gj(hipStream_t s, const GjPlan& p, const GjWork& w, int64_t n, int cnt,
                     const GjAux* aux = nullptr);
hipError_t launch_set_diag(hipStream_t s, const CoarseDesc* desc, int cnt, int b, double* A,
                           int64_t sA, int64_t n);
// dense blocks of time-decoupled coarse members (member z: kdesc[z])
hipError_t launch_kron_block_dense(hipStream_t s, const KronBlockDesc* kdesc, int cnt,
                                   int32_t max_rows, double* A, int64_t sA, int64_t n);
// d = J^-1 r (transposed: d = J^-T r) on the rows of time-decoupled
// coarse members, from their blocks' inverses
hipError_t launch_kron_coarse_apply(hipStream_t s, int b, const KronCoarse* kc, int cnt,
                                    int max_blocks, int32_t max_ns, int transposed,
                                    const double* r, double* d);
// rinv = the inverse of every member's pivot record rpiv (order n, real
// order n0 from desc); verdict[z] = 0 when member z's record is a
// permutation whose real columns pivot on real rows, else 1.
hipError_t launch_gj_invert_perm(hipStream_t s, const int* rpiv, int64_t sV, int64_t n,
                                 const CoarseDesc* desc, int cnt, int b, int* rinv,
                                 int* verdict);
// out[0] = the lowest index c < n with flag[c] != 0 (out[0] keeps its value
// when it is lower or no flag is set)
hipError_t launch_first_flag(hipStream_t s, const uint8_t* flag, int64_t n, int* out);
hipError_t launch_gj_unpermute(hipStream_t s, const double* S, int64_t sA, int64_t n,
                               const int* rpiv, const int* rinv, int64_t sV,
                               const CoarseDesc* desc, int cnt, int b, int64_t max_n0,
                               double* out);
hipError_t launch_dense_gemv(hipStream_t s, const CoarseDesc* desc, int cnt, int b,
                             int64_t max_n0, const double* inv, const double* x, double* y);
// Krylov helpers, per instance segment: V is row-major (m vectors of length
// n); segment z covers elements [seg[z], seg[z+1]); nseg segments, the
// longest of max_seg elements.  Scalars of segment z sit at z * stride.
struct Segs { const int64_t* seg; int nseg; int64_t max_seg; };
int seg_blocks(const Segs& g);   // partial-sum blocks per segment
hipError_t launch_multidot(hipStream_t s, const double* V, int m, const double* w, int64_t n,
                           const Segs& g, double* partial, double* out, int64_t ostride);
hipError_t launch_multiaxpy_dot(hipStream_t s, const double* V, int m, const double* coef,
                                int64_t cstride, double sign, double* w, int64_t n,
                                const Segs& g, double* partial, double* out, int64_t ostride);
hipError_t launch_multiaxpy_nrm(hipStream_t s, const double* V, int m, const double* coef,
                                int64_t cstride, double sign, double* w, int64_t n,
                                const Segs& g, double* partial, double* out, int64_t ostride);
hipError_t launch_multiaxpy(hipStream_t s, const double* V, int m, const double* coef,
                            int64_t cstride, double sign, double* w, int64_t n, const Segs& g);
hipError_t launch_scale_by_norm(hipStream_t s, const double* w, const double* nrm2,
                                int64_t nstride, double* v, const Segs& g);

}  // namespace stv
