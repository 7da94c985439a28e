// Host side of the space-time Vanka multigrid library: argument validation,
// hierarchy upload (owned-DoF lists, transposed prolongations), the inverse
// build, the smoother / V-cycle orchestration (Algorithm 4.1) and the flexible
// GMRES driver.  Every arithmetic step on vectors and matrices runs in the
// HIP kernels; the host only does index bookkeeping, the (k+1)-sized Givens
// and triangular solves of GMRES, and control flow.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "stv_internal.h"

// registers per lane that the complex-pivot elimination chain's largest
// kernel needs on a SIMD (its workgroups run beside the cell inverses; the
// panel kernel k_gj_tour_cx and the wide update k_gj_slab_update_cx128 are
// held to 128)
#ifndef STV_CHAIN_VGPRS
#define STV_CHAIN_VGPRS 128
#endif

using namespace stv;

thread_local stv::LaunchEvents stv::g_launch_events;

// Fixed device workspace of stv_vcycle_noalloc: the level work vectors of a
// V-cycle, so that the call allocates nothing.  Every device the library runs
// on holds its own copy until the process ends; host code reaches it only
// through the per-device address resolved at context creation (the name
// itself is a host-side stand-in, not a device address).
constexpr size_t kNoAllocDoubles = size_t(8) << 20;   // 64 MiB
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

std::string g_create_err;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (resolved once per
// device, with that device current).
hipError_t resolve_scratch(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_dev[device] = static_cast<double*>(ptr);
  }
  *out = g_scratch_dev[device];
  return hipSuccess;
}

int fail(stv_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  return code;
}

#define STV_HIP(call)                                                                       \
  do {                                                                                      \
    hipError_t e_ = (call);                                                                 \
    if (e_ != hipSuccess)                                                                   \
      return fail(ctx, e_ == hipErrorOutOfMemory ? STV_ENOMEM : STV_EHIP,                   \
                  std::string(#call) + " failed: " + hipGetErrorString(e_));                \
  } while (0)

#define STV_TRY(call)        \
  do {                       \
    int rc_ = (call);        \
    if (rc_ != STV_OK) return rc_; \
  } while (0)

template <typename T>
int dalloc(stv_ctx* ctx, T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, sizeof(T) * count);
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(ctx, STV_ENOMEM, "hipMalloc of " + std::to_string(sizeof(T) * count) +
                                     " bytes failed: " + hipGetErrorString(e));
  }
  return STV_OK;
}

template <typename T>
int upload(stv_ctx* ctx, T** p, const T* src, size_t count) {
  STV_TRY(dalloc(ctx, p, count));
  if (count) STV_HIP(hipMemcpy(*p, src, sizeof(T) * count, hipMemcpyHostToDevice));
  return STV_OK;
}

template <typename T>
void dfree(T*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void free_graph(stv_ctx* ctx) {
  if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
  if (ctx->graph) (void)hipGraphDestroy(ctx->graph);
  ctx->graph_exec = nullptr;
  ctx->graph = nullptr;
  dfree(ctx->g_in);
  dfree(ctx->g_out);
}

void free_coarse_groups(stv_ctx* ctx) {
  for (auto& G : ctx->cgroups) {
    dfree(G.d_desc); dfree(G.w.A); dfree(G.w.rpiv); dfree(G.w.used); dfree(G.w.B);
    dfree(G.w.P); dfree(G.w.S); dfree(G.w.Bin); dfree(G.rinv);
    dfree(G.w.cand); dfree(G.w.Z); dfree(G.w.counter);
    dfree(G.d_kdesc);
  }
  ctx->cgroups.clear();
  for (int g = 0; g < kMaxLevels; ++g) {
    ctx->h_kc[g].clear();
    dfree(ctx->d_kc[g]);
    ctx->kc_max_ns[g] = 0;
    ctx->kc_max_blocks[g] = 0;
  }
  ctx->cgroups_algo = -1;
  dfree(ctx->coarse_inv);
  ctx->coarse_elems = 0;
}

// Every stored inverse and the whole inverse-build workspace.
void free_inverses(stv_ctx* ctx) {
  ++ctx->generation;
  free_graph(ctx);
  for (int g = 0; g < kMaxLevels; ++g) {
    dfree(ctx->lv[g].inv_off);
    dfree(ctx->lv[g].inv_store);
    dfree(ctx->lv[g].dec_tab);
    dfree(ctx->lv[g].dec_code);
    ctx->lv[g].dec = 0;
    ctx->lv[g].inv_elems = 0;
    dfree(ctx->inv_status[g]);
    dfree(ctx->inv_scratch[g]);
    ctx->inv_slots[g] = 0;
  }
  ctx->inv_layout = ctx->inv_type = -1;
  free_coarse_groups(ctx);
  dfree(ctx->inv_report);
  if (ctx->h_report) (void)hipHostFree(ctx->h_report);
  ctx->h_report = nullptr;
  ctx->n_report = 0;
  ctx->have_inv = false;
}

void free_level(DevLevel& L) {
  dfree(L.rowptr); dfree(L.col); dfree(L.val); dfree(L.cell_sdofs);
  dfree(L.own_ptr); dfree(L.own_loc); dfree(L.inc_ptr); dfree(L.inc_cell); dfree(L.inc_loc);
  dfree(L.P_rowptr); dfree(L.P_col); dfree(L.P_val);
  dfree(L.Pt_rowptr); dfree(L.Pt_col); dfree(L.Pt_val);
  dfree(L.inv_off); dfree(L.inv_store); dfree(L.posmap); dfree(L.dec_tab); dfree(L.dec_code);
  dfree(L.rho); dfree(L.r); dfree(L.d); dfree(L.corr);
  dfree(L.rowptr_t); dfree(L.col_t); dfree(L.val_t);
  dfree(L.kron_ma); dfree(L.kx_ptr); dfree(L.kx_col); dfree(L.kx_val);
  L = DevLevel();
}

void free_workspace(stv_ctx* ctx) {
  dfree(ctx->V); dfree(ctx->Z); dfree(ctx->w); dfree(ctx->rt); dfree(ctx->partial);
  ctx->ws_restart = 0;
  ctx->ws_n = 0;
}

void free_hierarchy(stv_ctx* ctx) {
  free_inverses(ctx);
  for (int g = 0; g < kMaxLevels; ++g) {
    free_level(ctx->lv[g]);
    dfree(ctx->d_coarse[g]);
    ctx->h_coarse[g].clear();
    ctx->n_whole[g] = 0;
    ctx->coarse_max_n0[g] = 0;
  }
  free_workspace(ctx);
  dfree(ctx->seg_off);
  ctx->n_inst = 0;
  ctx->inst_levels.clear();
  ctx->inst_row.clear();
  ctx->inst_info.clear();
  ctx->max_seg = 0;
  ctx->have_hier = false;
  ctx->n_levels = 0;
}

// ---------------------------------------------------------------- timing
hipEvent_t get_event(stv_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Times one kernel class on one level while timing is on and the class is
// selected.  A scope holding exactly one launch made through stv::launch
// (one_launch) has that kernel stamp its own start and end; any other scope
// is bracketed by event records on its stream.
struct Timed {
  stv_ctx* ctx;
  int cls;
  int level;
  hipStream_t st;
  bool stamp = false;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(stv_ctx* c, int k, int g = 0, hipStream_t on = nullptr, bool one_launch = false)
      : ctx(c), cls(k), level(g), st(on ? on : c->stream) {
    if (!ctx->timing || !((ctx->timing_mask >> cls) & 1u) || !((ctx->timing_levels >> level) & 1u))
      return;
    a = get_event(ctx);
    if (one_launch) {
      b = get_event(ctx);
      g_launch_events = LaunchEvents{a, b};
      stamp = true;
    } else {
      (void)hipEventRecord(a, st);
    }
  }
  void done() {
    if (!a) return;
    if (stamp) {
      // the pair counts only when the launch took it
      const bool taken = g_launch_events.start != a;
      g_launch_events = LaunchEvents{};
      if (taken) {
        ctx->pending.push_back({a, b, cls, level});
      } else {
        ctx->pool.push_back(a);
        ctx->pool.push_back(b);
      }
    } else {
      b = get_event(ctx);
      (void)hipEventRecord(b, st);
      ctx->pending.push_back({a, b, cls, level});
    }
    a = b = nullptr;
  }
  ~Timed() {
    if (a && g_launch_events.start == a) g_launch_events = LaunchEvents{};
  }
};

void resolve_timers(stv_ctx* ctx) {
  for (auto& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      ctx->launches[t.cls][t.level] += 1;
      ctx->total_ms[t.cls][t.level] += ms;
    }
    ctx->pool.push_back(t.a);
    ctx->pool.push_back(t.b);
  }
  ctx->pending.clear();
}

// ---------------------------------------------------------------- validation
int n_ls_of(int dim) { return dim * (dim == 2 ? 9 : 27) + dim + 1; }

bool validate_impl(int n_levels, int dim, int k, const stv_level* lv, std::string& err) {
  auto bad = [&](int g, const std::string& m) {
    err = "level " + std::to_string(g) + ": " + m;
    return false;
  };
  if (n_levels < 1 || n_levels > kMaxLevels) {
    err = "n_levels must be in [1, 16]";
    return false;
  }
  if (dim != 2 && dim != 3) { err = "dim must be 2 or 3"; return false; }
  if (k < 0 || k > 3) { err = "k must be in [0, 3]"; return false; }
  if (!lv) { err = "levels pointer is NULL"; return false; }
  const int nls = n_ls_of(dim);
  for (int g = 0; g < n_levels; ++g) {
    const stv_level& L = lv[g];
    if (L.n_sdofs <= 0) return bad(g, "n_sdofs must be positive");
    if (L.n_cells <= 0) return bad(g, "n_cells must be positive");
    if (L.n_ls != nls) return bad(g, "n_ls must be dim*3^dim + dim + 1 = " + std::to_string(nls));
    if (!L.bsr_rowptr || !L.bsr_col || !L.bsr_val || !L.cell_sdofs)
      return bad(g, "bsr_rowptr/bsr_col/bsr_val/cell_sdofs must not be NULL");
    if (L.nnzb <= 0 || L.nnzb > INT32_MAX) return bad(g, "nnzb out of range");
    if (L.bsr_rowptr[0] != 0) return bad(g, "bsr_rowptr[0] must be 0");
    if ((int64_t)L.bsr_rowptr[L.n_sdofs] != L.nnzb)
      return bad(g, "bsr_rowptr[n_sdofs] must equal nnzb");
    for (int32_t s = 0; s < L.n_sdofs; ++s) {
      const int32_t a = L.bsr_rowptr[s], e = L.bsr_rowptr[s + 1];
      if (e < a) return bad(g, "bsr_rowptr must be non-decreasing (row " + std::to_string(s) + ")");
      for (int32_t q = a; q < e; ++q) {
        const int32_t c = L.bsr_col[q];
        if (c < 0 || c >= L.n_sdofs)
          return bad(g, "bsr_col out of range (row " + std::to_string(s) + ")");
        if (q > a && c <= L.bsr_col[q - 1])
          return bad(g, "bsr_col must be strictly increasing per row (row " + std::to_string(s) + ")");
      }
    }
    std::vector<uint8_t> seen((size_t)L.n_sdofs, 0);
    for (int64_t e = 0; e < (int64_t)L.n_cells * nls; ++e) {
      const int32_t s = L.cell_sdofs[e];
      if (s < 0 || s >= L.n_sdofs)
        return bad(g, "cell_sdofs out of range (cell " + std::to_string(e / nls) + ")");
      seen[(size_t)s] = 1;
    }
    // distinct DoFs per cell (cell pairs absent from the block pattern are zero)
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<int64_t> bad_cell(nth, -1);
    std::vector<int> bad_kind(nth, 0);
    std::vector<std::thread> th;
    for (unsigned t = 0; t < nth; ++t) {
      th.emplace_back([&, t]() {
        for (int64_t c = t; c < L.n_cells; c += nth) {
          const int32_t* sd = L.cell_sdofs + c * nls;
          for (int a = 0; a < nls && bad_cell[t] < 0; ++a) {
            for (int bb = a + 1; bb < nls; ++bb)
              if (sd[bb] == sd[a]) { bad_cell[t] = c; bad_kind[t] = 1; break; }
          }
          if (bad_cell[t] >= 0) return;
        }
      });
    }
    for (auto& x : th) x.join();
    for (unsigned t = 0; t < nth; ++t)
      if (bad_cell[t] >= 0)
        return bad(g, "repeated DoF in cell " + std::to_string(bad_cell[t]));
    for (int32_t s = 0; s < L.n_sdofs; ++s)
      if (!seen[(size_t)s]) return bad(g, "spatial DoF " + std::to_string(s) + " belongs to no cell");
    if (g > 0) {
      const stv_level& C = lv[g - 1];
      if (!L.P_rowptr || !L.P_col || !L.P_val)
        return bad(g, "P_rowptr/P_col/P_val must not be NULL on levels >= 1");
      if (L.P_rowptr[0] != 0 || (int64_t)L.P_rowptr[L.n_sdofs] != L.P_nnz || L.P_nnz < 0)
        return bad(g, "P_rowptr inconsistent with P_nnz");
      for (int32_t s = 0; s < L.n_sdofs; ++s) {
        if (L.P_rowptr[s + 1] < L.P_rowptr[s]) return bad(g, "P_rowptr must be non-decreasing");
        for (int32_t q = L.P_rowptr[s]; q < L.P_rowptr[s + 1]; ++q)
          if (L.P_col[q] < 0 || L.P_col[q] >= C.n_sdofs)
            return bad(g, "P_col out of range of the coarser level");
      }
    }
  }
  return true;
}

int check_ctx(stv_ctx* ctx, bool need_hier, bool need_inv) {
  if (!ctx) return STV_EINVAL;
  if (need_hier && !ctx->have_hier) return fail(ctx, STV_ESTATE, "no hierarchy set");
  if (need_inv && !ctx->have_inv) return fail(ctx, STV_ESTATE, "cell inverses not built");
  return STV_OK;
}

// ---------------------------------------------------------------- level ops
// y = r + sx J_g x: from the spatial factors when the level has them (and
// the operator is not transposed), else from the stored blocks.
int level_apply(stv_ctx* ctx, int g, const double* r, const double* x, double* y, double sx) {
  const DevLevel& L = ctx->lv[g];
  Timed t(ctx, KC_RESIDUAL, g, nullptr, true);
  if (L.kron_ma && !ctx->transposed)
    STV_HIP(launch_spmv_kron(ctx->stream, ctx->b, L, r, x, y, sx));
  else
    STV_HIP(launch_spmv(ctx->stream, ctx->b, L, r, x, y, sx, ctx->transposed != 0));
  t.done();
  return STV_OK;
}

int residual(stv_ctx* ctx, int g, const double* r, const double* x, double* y) {
  return level_apply(ctx, g, r, x, y, -1.0);
}

int matvec(stv_ctx* ctx, int g, const double* x, double* y) {
  return level_apply(ctx, g, nullptr, x, y, 1.0);
}

int cell_pass(stv_ctx* ctx, int g, const double* rho, double* d, double omega, int zero_init,
              int mode) {
  DevLevel& L = ctx->lv[g];
  const int b = ctx->b;
  if (ctx->transposed) {
    Timed t(ctx, KC_SWEEP, g, nullptr, true);
    STV_HIP(launch_vanka_cells_t(ctx->stream, b, L, rho, d, omega, zero_init, ctx->inv_fp32));
    t.done();
    return STV_OK;
  }
  if (mode == STV_LAST_WRITER) {
    Timed t(ctx, KC_SWEEP, g, nullptr, true);
    STV_HIP(launch_vanka_cells(ctx->stream, b, L, rho, d, omega, zero_init, ctx->inv_fp32,
                               ctx->inv_full));
    t.done();
    return STV_OK;
  }
  if (!L.corr) STV_TRY(dalloc(ctx, &L.corr, (size_t)L.n_cells * L.n_ls * b));
  if (zero_init) STV_HIP(launch_fill(ctx->stream, d, (int64_t)L.n_s * b, 0.0));
  Timed t(ctx, KC_SWEEP, g);
  STV_HIP(launch_vanka_cells_corr(ctx->stream, b, L, rho, omega, ctx->inv_fp32));
  STV_HIP(launch_vanka_combine(ctx->stream, b, L, d, mode == STV_POU ? 1 : 0));
  t.done();
  return STV_OK;
}

int check_mode(stv_ctx* ctx, int mode) {
  if (mode != STV_LAST_WRITER && mode != STV_POU && mode != STV_ADDITIVE)
    return fail(ctx, STV_EINVAL, "unknown sweep mode");
  if (mode != STV_LAST_WRITER && !ctx->inv_full)
    return fail(ctx, STV_ESTATE, "averaged/additive sweeps need inverses built with STV_STORE_FULL");
  return STV_OK;
}

int sweeps(stv_ctx* ctx, int g, const double* r, double* d, int n, double omega, int mode,
           bool d_is_zero) {
  DevLevel& L = ctx->lv[g];
  for (int s = 0; s < n; ++s) {
    if (s == 0 && d_is_zero) {
      STV_TRY(cell_pass(ctx, g, r, d, omega, 1, mode));   // rho = r when d = 0
    } else {
      STV_TRY(residual(ctx, g, r, d, L.rho));
      STV_TRY(cell_pass(ctx, g, L.rho, d, omega, 0, mode));
    }
  }
  return STV_OK;
}

// d = J_c^-1 r on the rows of every coarse member stored on level g: the
// members with a whole stored inverse by a dense product, the time-decoupled
// ones from their blocks' inverses.
int coarse_apply(stv_ctx* ctx, int g, const double* r, double* d) {
  const int nw = ctx->n_whole[g], nk = (int)ctx->h_kc[g].size();
  if (nw == 0 && nk == 0) return STV_OK;
  Timed t(ctx, KC_COARSE, g, nullptr, true);
  if (nw > 0 && ctx->transposed)
    STV_HIP(launch_dense_gemv_t(ctx->stream, ctx->d_coarse[g], nw, ctx->b, ctx->coarse_max_n0[g],
                                ctx->coarse_inv, r, d));
  else if (nw > 0)
    STV_HIP(launch_dense_gemv(ctx->stream, ctx->d_coarse[g], nw, ctx->b, ctx->coarse_max_n0[g],
                              ctx->coarse_inv, r, d));
  if (nk > 0)
    STV_HIP(launch_kron_coarse_apply(ctx->stream, ctx->b, ctx->d_kc[g], nk, ctx->kc_max_blocks[g],
                                     ctx->kc_max_ns[g], ctx->transposed ? 1 : 0, r, d));
  t.done();
  return STV_OK;
}

// One V-cycle on level g from d = 0.  Every member of a packed level is
// either smoothed there (it has a coarser level) or solved directly (level g
// is its coarsest); the two kinds own disjoint rows, the level operators are
// block diagonal over members, and the coarse rows are written after the
// smoother, which touches only its own cells' rows.
int vcycle_level(stv_ctx* ctx, int g, const double* r, double* d, const stv_mg_params& p) {
  DevLevel& L = ctx->lv[g];
  if (g == 0 || L.n_cells == 0) return coarse_apply(ctx, g, r, d);
  DevLevel& C = ctx->lv[g - 1];
  const int b = ctx->b;
  if (p.nu1 == 0) STV_HIP(launch_fill(ctx->stream, d, (int64_t)L.n_s * b, 0.0));
  STV_TRY(sweeps(ctx, g, r, d, p.nu1, p.omega, p.mode, true));
  STV_TRY(coarse_apply(ctx, g, r, d));
  STV_TRY(residual(ctx, g, r, d, L.rho));
  {
    Timed t(ctx, KC_TRANSFER, g, nullptr, true);
    STV_HIP(launch_restrict(ctx->stream, b, L, L.rho, C.r));
    t.done();
  }
  STV_TRY(vcycle_level(ctx, g - 1, C.r, C.d, p));
  {
    Timed t(ctx, KC_TRANSFER, g, nullptr, true);
    STV_HIP(launch_prolongate_add(ctx->stream, b, L, C.d, d));
    t.done();
  }
  STV_TRY(sweeps(ctx, g, r, d, p.nu2, p.omega, p.mode, false));
  return STV_OK;
}

// Capture one V-cycle (finest level, g_in -> g_out) into a HIP graph.  The
// capture runs the ordinary launch sequence on an internal stream with the
// per-kernel timers off; nothing in it allocates, synchronises or sets
// memory with a memset (zero fills are kernels).
int ensure_graph(stv_ctx* ctx, const stv_mg_params& p) {
  int64_t om = 0;
  std::memcpy(&om, &p.omega, sizeof(om));
  const int64_t key[6] = {ctx->generation, p.nu1, p.nu2, om, p.mode, ctx->transposed};
  if (ctx->graph_exec && std::equal(key, key + 6, ctx->graph_key)) return STV_OK;
  free_graph(ctx);
  const int G = ctx->n_levels - 1;
  const int64_t n = (int64_t)ctx->lv[G].n_s * ctx->b;
  STV_TRY(dalloc(ctx, &ctx->g_in, (size_t)n));
  STV_TRY(dalloc(ctx, &ctx->g_out, (size_t)n));
  if (p.mode != STV_LAST_WRITER)
    for (int g = 1; g < ctx->n_levels; ++g) {
      DevLevel& L = ctx->lv[g];
      if (L.n_cells > 0 && !L.corr) STV_TRY(dalloc(ctx, &L.corr, (size_t)L.n_cells * L.n_ls * ctx->b));
    }
  STV_HIP(hipStreamSynchronize(ctx->stream));
  const bool timing = ctx->timing;
  hipStream_t saved = ctx->stream;
  ctx->timing = false;
  ctx->stream = ctx->cap_stream;
  hipError_t e = hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeRelaxed);
  int rc = STV_OK;
  if (e == hipSuccess) {
    rc = vcycle_level(ctx, G, ctx->g_in, ctx->g_out, p);
    hipGraph_t gr = nullptr;
    const hipError_t e2 = hipStreamEndCapture(ctx->cap_stream, &gr);
    ctx->graph = gr;
    if (e2 != hipSuccess) e = e2;
  }
  ctx->stream = saved;
  ctx->timing = timing;
  if (rc != STV_OK) { free_graph(ctx); return rc; }
  if (e == hipSuccess) e = hipGraphInstantiate(&ctx->graph_exec, ctx->graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    free_graph(ctx);
    return fail(ctx, STV_EHIP, std::string("V-cycle graph capture failed: ") + hipGetErrorString(e));
  }
  std::copy(key, key + 6, ctx->graph_key);
  return STV_OK;
}

// d = MG(r) on the finest level: eager launches, or the captured graph.
int precond_apply(stv_ctx* ctx, const double* r, double* d, const stv_mg_params& p) {
  const int G = ctx->n_levels - 1;
  if (!ctx->use_graph) return vcycle_level(ctx, G, r, d, p);
  STV_TRY(ensure_graph(ctx, p));
  const int64_t n = (int64_t)ctx->lv[G].n_s * ctx->b;
  Timed t(ctx, KC_GRAPH, G);
  STV_HIP(launch_copy(ctx->stream, r, ctx->g_in, n));
  STV_HIP(hipGraphLaunch(ctx->graph_exec, ctx->stream));
  STV_HIP(launch_copy(ctx->stream, ctx->g_out, d, n));
  t.done();
  ++ctx->graph_replays;
  return STV_OK;
}

// Pattern and values of J^T on every level (once per hierarchy): the
// pattern by a counting sort of the block columns on the host, the values by
// a block-transposing gather on the device.
int ensure_transpose(stv_ctx* ctx) {
  const int b = ctx->b;
  for (int g = 0; g < ctx->n_levels; ++g) {
    DevLevel& L = ctx->lv[g];
    if (L.val_t) continue;
    std::vector<int32_t> rp((size_t)L.n_s + 1), cl((size_t)L.nnzb);
    STV_HIP(hipMemcpy(rp.data(), L.rowptr, sizeof(int32_t) * rp.size(), hipMemcpyDeviceToHost));
    STV_HIP(hipMemcpy(cl.data(), L.col, sizeof(int32_t) * cl.size(), hipMemcpyDeviceToHost));
    std::vector<int32_t> tp((size_t)L.n_s + 1, 0), tc((size_t)L.nnzb), src((size_t)L.nnzb);
    for (int64_t q = 0; q < L.nnzb; ++q) tp[(size_t)cl[(size_t)q] + 1]++;
    for (int32_t r = 0; r < L.n_s; ++r) tp[(size_t)r + 1] += tp[(size_t)r];
    std::vector<int32_t> fillp(tp.begin(), tp.end() - 1);
    for (int32_t r = 0; r < L.n_s; ++r)
      for (int32_t q = rp[(size_t)r]; q < rp[(size_t)r + 1]; ++q) {
        const int32_t c = cl[(size_t)q];
        tc[(size_t)fillp[(size_t)c]] = r;           // rows ascending: columns of J^T sorted
        src[(size_t)fillp[(size_t)c]++] = q;
      }
    int32_t* dsrc = nullptr;
    STV_TRY(upload(ctx, &L.rowptr_t, tp.data(), tp.size()));
    STV_TRY(upload(ctx, &L.col_t, tc.data(), tc.size()));
    STV_TRY(dalloc(ctx, &L.val_t, (size_t)L.nnzb * b * b));
    STV_TRY(upload(ctx, &dsrc, src.data(), src.size()));
    hipError_t e = launch_bsr_transpose_vals(ctx->stream, b, L.val, dsrc, L.val_t, L.nnzb);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    dfree(dsrc);
    if (e != hipSuccess) return fail(ctx, STV_EHIP, std::string("transpose failed: ") + hipGetErrorString(e));
  }
  return STV_OK;
}

int check_transposable(stv_ctx* ctx, int mode) {
  STV_TRY(check_ctx(ctx, true, true));
  if (!ctx->inv_full)
    return fail(ctx, STV_ESTATE, "transposed solves need inverses built with STV_STORE_FULL");
  if (mode != STV_LAST_WRITER)
    return fail(ctx, STV_EINVAL, "transposed solves use the last-writer sweep only");
  return ensure_transpose(ctx);
}

int check_mg(stv_ctx* ctx, const stv_mg_params* p) {
  if (!p) return fail(ctx, STV_EINVAL, "mg params NULL");
  if (p->nu1 < 0 || p->nu2 < 0 || p->nu1 > 64 || p->nu2 > 64)
    return fail(ctx, STV_EINVAL, "nu1/nu2 must be in [0, 64]");
  if (!(p->omega > 0.0) || !std::isfinite(p->omega))
    return fail(ctx, STV_EINVAL, "omega must be positive and finite");
  return check_mode(ctx, p->mode);
}

// ---------------------------------------------------------------- Krylov
int ensure_workspace(stv_ctx* ctx, int m) {
  const int64_t n = (int64_t)ctx->lv[ctx->n_levels - 1].n_s * ctx->b;
  if (ctx->ws_restart >= m && ctx->ws_n == n) return STV_OK;
  free_workspace(ctx);
  const Segs sg{ctx->seg_off, ctx->n_inst, ctx->max_seg};
  STV_TRY(dalloc(ctx, &ctx->V, (size_t)(m + 1) * n));
  STV_TRY(dalloc(ctx, &ctx->Z, (size_t)m * n));
  STV_TRY(dalloc(ctx, &ctx->w, (size_t)n));
  STV_TRY(dalloc(ctx, &ctx->rt, (size_t)n));
  STV_TRY(dalloc(ctx, &ctx->partial, (size_t)ctx->n_inst * seg_blocks(sg) * 8));
  ctx->ws_restart = m;
  ctx->ws_n = n;
  return STV_OK;
}

// Scalar buffers (device and pinned host mirror), S = instances, R = kScalR:
//   h1 (first Gram-Schmidt pass)   [0, S R)        instance z at z R
//   h2 (second pass)               [S R, 2 S R)
//   ||w||^2                        [2 S R, 2 S R + S)
//   scratch norms^2                [2 S R + S, 2 S R + 2 S)
//   y (host -> device)             [2 S R + 2 S, 3 S R + 2 S)
constexpr int kScalR = kMaxRestart + 2;
struct ScalLayout {
  int64_t S;
  int64_t h1(int64_t z) const { return z * kScalR; }
  int64_t h2(int64_t z) const { return S * kScalR + z * kScalR; }
  int64_t nrm() const { return 2 * S * kScalR; }
  int64_t aux() const { return 2 * S * kScalR + S; }
  int64_t y(int64_t z) const { return 2 * S * kScalR + 2 * S + z * kScalR; }
  int64_t total() const { return 3 * S * kScalR + 2 * S; }
};

int ensure_scalars(stv_ctx* ctx, int64_t S) {
  if (ctx->scal_segs >= S && ctx->scal) return STV_OK;
  dfree(ctx->scal);
  if (ctx->hscal) (void)hipHostFree(ctx->hscal);
  if (ctx->hstep) (void)hipHostFree(ctx->hstep);
  ctx->hscal = ctx->hstep = nullptr;
  ctx->scal_segs = 0;
  const ScalLayout lay{S};
  STV_TRY(dalloc(ctx, &ctx->scal, (size_t)lay.total()));
  if (hipHostMalloc((void**)&ctx->hscal, sizeof(double) * lay.total(), hipHostMallocDefault) !=
          hipSuccess ||
      hipHostMalloc((void**)&ctx->hstep, sizeof(double) * (lay.nrm() + S), hipHostMallocDefault) !=
          hipSuccess) {
    if (ctx->hscal) (void)hipHostFree(ctx->hscal);
    ctx->hscal = ctx->hstep = nullptr;
    return fail(ctx, STV_ENOMEM, "pinned allocation of the scalar buffer failed");
  }
  ctx->scal_segs = S;
  return STV_OK;
}

// out[z] = a_z . b_z for every instance segment z of two finest-level vectors
int dots_to_host(stv_ctx* ctx, const double* a, const double* b, int64_t n,
                 std::vector<double>& out) {
  const ScalLayout lay{ctx->scal_segs};
  const Segs sg{ctx->seg_off, ctx->n_inst, ctx->max_seg};
  Timed t(ctx, KC_KRYLOV);
  STV_HIP(launch_multidot(ctx->stream, a, 1, b, n, sg, ctx->partial, ctx->scal + lay.aux(), 1));
  t.done();
  STV_HIP(hipMemcpyAsync(ctx->hscal + lay.aux(), ctx->scal + lay.aux(),
                         sizeof(double) * ctx->n_inst, hipMemcpyDeviceToHost, ctx->stream));
  STV_HIP(hipStreamSynchronize(ctx->stream));
  out.assign(ctx->hscal + lay.aux(), ctx->hscal + lay.aux() + ctx->n_inst);
  return STV_OK;
}

// ---------------------------------------------------------------- set-up
// Pack n_inst hierarchies into block-diagonal levels aligned at the finest
// level: instance i with G_i levels occupies packed levels D-G_i .. D-1
// (D = max G_i), its own level l at packed level D-G_i+l, rows (and cells)
// in instance order.  A single hierarchy is the case n_inst = 1.
int setup_packed(stv_ctx* ctx, int n_inst, int dim, int k, const int* nlev,
                 const stv_level* const* lvs) {
  std::string msg;
  for (int i = 0; i < n_inst; ++i) {
    if (!validate_impl(nlev[i], dim, k, lvs[i], msg))
      return fail(ctx, STV_EINVAL, n_inst > 1 ? "instance " + std::to_string(i) + ": " + msg : msg);
  }
  int D = 0;
  for (int i = 0; i < n_inst; ++i) D = std::max(D, nlev[i]);
  const int b = k + 1;
  const int nls = n_ls_of(dim);
  // member i is present on packed level g from level g - (D - G_i) of its own
  auto local = [&](int i, int g) { return g - (D - nlev[i]); };
  // packed sizes must fit the 32-bit indices of the kernels
  for (int g = 0; g < D; ++g) {
    int64_t ns = 0, nz = 0, nc = 0, pz = 0;
    for (int i = 0; i < n_inst; ++i) {
      const int l = local(i, g);
      if (l < 0) continue;
      const stv_level& H = lvs[i][l];
      ns += H.n_sdofs;
      nz += H.nnzb;
      if (l > 0) { nc += H.n_cells; pz += H.P_nnz; }
    }
    if (ns * b >= INT32_MAX || nz >= INT32_MAX || nc * nls >= INT32_MAX || pz >= INT32_MAX)
      return fail(ctx, STV_EINVAL, "packed level " + std::to_string(g) + " exceeds 32-bit indexing");
  }
  STV_HIP(hipSetDevice(ctx->device));
  STV_HIP(hipStreamSynchronize(ctx->stream));
  free_hierarchy(ctx);
  STV_TRY(ensure_scalars(ctx, n_inst));
  ctx->n_levels = D;
  ctx->dim = dim;
  ctx->k = k;
  ctx->b = b;
  ctx->n_inst = n_inst;
  ctx->inst_levels.assign(nlev, nlev + n_inst);
  ctx->inst_info.assign((size_t)n_inst, InstInfo());
  std::vector<std::vector<int32_t>> roff((size_t)D, std::vector<int32_t>((size_t)n_inst, -1));
  for (int g = 0; g < D; ++g) {
    DevLevel& L = ctx->lv[g];
    // offsets of the members: rows, blocks, cells (smoothed members only)
    int32_t ns = 0;
    int64_t nz = 0, ncell = 0, ncell_all = 0, pnz = 0;
    std::vector<int64_t> zoff((size_t)n_inst, 0), coff((size_t)n_inst, -1), poff((size_t)n_inst, 0);
    for (int i = 0; i < n_inst; ++i) {
      const int l = local(i, g);
      if (l < 0) continue;
      const stv_level& H = lvs[i][l];
      roff[(size_t)g][(size_t)i] = ns;
      zoff[(size_t)i] = nz;
      ns += H.n_sdofs;
      nz += H.nnzb;
      ncell_all += H.n_cells;
      if (l > 0) {
        coff[(size_t)i] = ncell;
        ncell += H.n_cells;
        poff[(size_t)i] = pnz;
        pnz += H.P_nnz;
      }
    }
    L.n_s = ns;
    L.nnzb = nz;
    L.n_cells = (int32_t)ncell;
    L.n_cells_all = ncell_all;
    L.n_ls = nls;
    // block rows (column indices shifted by the member's first row)
    {
      std::vector<int32_t> rp((size_t)ns + 1, 0), cl;
      const bool shift = n_inst > 1;
      if (shift) cl.resize((size_t)nz);
      for (int i = 0; i < n_inst; ++i) {
        const int l = local(i, g);
        if (l < 0) continue;
        const stv_level& H = lvs[i][l];
        const int32_t r0 = roff[(size_t)g][(size_t)i];
        for (int32_t s = 0; s <= H.n_sdofs; ++s) rp[(size_t)r0 + s] = (int32_t)(zoff[(size_t)i] + H.bsr_rowptr[s]);
        if (shift)
          for (int64_t q = 0; q < H.nnzb; ++q) cl[(size_t)(zoff[(size_t)i] + q)] = H.bsr_col[q] + r0;
      }
      STV_TRY(upload(ctx, &L.rowptr, rp.data(), rp.size()));
      if (shift) STV_TRY(upload(ctx, &L.col, cl.data(), cl.size()));
      else STV_TRY(upload(ctx, &L.col, lvs[0][local(0, g)].bsr_col, (size_t)nz));
      STV_TRY(dalloc(ctx, &L.val, (size_t)nz * b * b));
      for (int i = 0; i < n_inst; ++i) {
        const int l = local(i, g);
        if (l < 0) continue;
        const stv_level& H = lvs[i][l];
        STV_HIP(hipMemcpy(L.val + zoff[(size_t)i] * b * b, H.bsr_val,
                          sizeof(double) * (size_t)H.nnzb * b * b, hipMemcpyHostToDevice));
      }
    }
    // cells of the smoothed members, their owned DoFs (the owner of a DoF is
    // the last cell in loop order that contains it) and the incidence lists
    {
      std::vector<int32_t> csd((size_t)ncell * nls);
      L.h_own_ptr.assign((size_t)ncell + 1, 0);
      L.h_own_loc.clear();
      std::vector<int32_t> ip((size_t)ns + 1, 0);
      for (int i = 0; i < n_inst; ++i) {
        const int l = local(i, g);
        if (l <= 0) continue;
        const stv_level& H = lvs[i][l];
        const int32_t r0 = roff[(size_t)g][(size_t)i];
        const int64_t c0 = coff[(size_t)i];
        std::vector<int32_t> owner((size_t)H.n_sdofs, -1);
        for (int32_t c = 0; c < H.n_cells; ++c)
          for (int a = 0; a < nls; ++a) owner[(size_t)H.cell_sdofs[(int64_t)c * nls + a]] = c;
        for (int32_t c = 0; c < H.n_cells; ++c) {
          for (int a = 0; a < nls; ++a) {
            const int32_t sd = H.cell_sdofs[(int64_t)c * nls + a];
            csd[(size_t)((c0 + c) * nls + a)] = sd + r0;
            if (owner[(size_t)sd] == c) L.h_own_loc.push_back((uint8_t)a);
            ip[(size_t)(r0 + sd) + 1]++;
          }
          L.h_own_ptr[(size_t)(c0 + c) + 1] = (int32_t)L.h_own_loc.size();
        }
      }
      for (int32_t r = 0; r < ns; ++r) ip[(size_t)r + 1] += ip[(size_t)r];
      std::vector<int32_t> fillp(ip.begin(), ip.end() - 1);
      std::vector<int32_t> icell((size_t)ip.back());
      std::vector<uint8_t> iloc((size_t)ip.back());
      for (int64_t c = 0; c < ncell; ++c)
        for (int a = 0; a < nls; ++a) {
          const int32_t r = csd[(size_t)(c * nls + a)];
          icell[(size_t)fillp[(size_t)r]] = (int32_t)c;
          iloc[(size_t)fillp[(size_t)r]++] = (uint8_t)a;
        }
      STV_TRY(upload(ctx, &L.cell_sdofs, csd.data(), csd.size()));
      L.h_csd = std::move(csd);
      STV_TRY(upload(ctx, &L.own_ptr, L.h_own_ptr.data(), L.h_own_ptr.size()));
      STV_TRY(upload(ctx, &L.own_loc, L.h_own_loc.data(), L.h_own_loc.size()));
      STV_TRY(upload(ctx, &L.inc_ptr, ip.data(), ip.size()));
      STV_TRY(upload(ctx, &L.inc_cell, icell.data(), icell.size()));
      STV_TRY(upload(ctx, &L.inc_loc, iloc.data(), iloc.size()));
    }
    if (ncell > 0) {
      STV_TRY(dalloc(ctx, &L.posmap, (size_t)ncell * nls * nls));
      STV_HIP(launch_build_posmap(ctx->stream, L));
    }
    const size_t nst = (size_t)ns * b;
    STV_TRY(dalloc(ctx, &L.rho, nst));
    if (g < D - 1) {
      STV_TRY(dalloc(ctx, &L.r, nst));
      STV_TRY(dalloc(ctx, &L.d, nst));
    }
    // prolongation from packed level g-1 (rows of coarse members stay empty)
    if (g > 0) {
      const int32_t nc = ctx->lv[g - 1].n_s;
      L.n_s_coarse = nc;
      std::vector<int32_t> prp((size_t)ns + 1, 0), pcl((size_t)pnz);
      std::vector<double> pvl((size_t)pnz);
      for (int i = 0; i < n_inst; ++i) {
        const int l = local(i, g);
        if (l <= 0) continue;
        const stv_level& H = lvs[i][l];
        const int32_t r0 = roff[(size_t)g][(size_t)i];
        const int32_t cc0 = roff[(size_t)g - 1][(size_t)i];
        const int64_t q0 = poff[(size_t)i];
        for (int32_t s = 0; s < H.n_sdofs; ++s)
          prp[(size_t)(r0 + s) + 1] = H.P_rowptr[s + 1] - H.P_rowptr[s];
        for (int64_t q = 0; q < H.P_nnz; ++q) {
          pcl[(size_t)(q0 + q)] = H.P_col[q] + cc0;
          pvl[(size_t)(q0 + q)] = H.P_val[q];
        }
      }
      for (int32_t r = 0; r < ns; ++r) prp[(size_t)r + 1] += prp[(size_t)r];
      STV_TRY(upload(ctx, &L.P_rowptr, prp.data(), prp.size()));
      STV_TRY(upload(ctx, &L.P_col, pcl.data(), pcl.size()));
      STV_TRY(upload(ctx, &L.P_val, pvl.data(), pvl.size()));
      // transpose (coarse rows, fine rows ascending within each)
      std::vector<int32_t> tp((size_t)nc + 1, 0);
      for (int64_t q = 0; q < pnz; ++q) tp[(size_t)pcl[(size_t)q] + 1]++;
      for (int32_t c = 0; c < nc; ++c) tp[(size_t)c + 1] += tp[(size_t)c];
      std::vector<int32_t> fillp(tp.begin(), tp.end() - 1);
      std::vector<int32_t> tc((size_t)pnz);
      std::vector<double> tv((size_t)pnz);
      for (int32_t r = 0; r < ns; ++r)
        for (int32_t q = prp[(size_t)r]; q < prp[(size_t)r + 1]; ++q) {
          const int32_t c = pcl[(size_t)q];
          tc[(size_t)fillp[(size_t)c]] = r;
          tv[(size_t)fillp[(size_t)c]++] = pvl[(size_t)q];
        }
      STV_TRY(upload(ctx, &L.Pt_rowptr, tp.data(), tp.size()));
      STV_TRY(upload(ctx, &L.Pt_col, tc.data(), tc.size()));
      STV_TRY(upload(ctx, &L.Pt_val, tv.data(), tv.size()));
      L.p_shape = transfer_shape_for(pnz, ns);
      L.pt_shape = transfer_shape_for(pnz, nc);
    }
    // the members solved directly on this level
    for (int i = 0; i < n_inst; ++i) {
      if (local(i, g) != 0) continue;
      CoarseDesc c{L.rowptr, L.col, L.val, roff[(size_t)g][(size_t)i], lvs[i][0].n_sdofs, 0};
      ctx->h_coarse[g].push_back(c);
      ctx->coarse_max_n0[g] = std::max<int64_t>(ctx->coarse_max_n0[g], (int64_t)c.n_s * b);
    }
  }
  // instance segments of the finest level
  ctx->inst_row.assign((size_t)n_inst + 1, 0);
  std::vector<int64_t> seg((size_t)n_inst + 1, 0);
  for (int i = 0; i < n_inst; ++i) {
    ctx->inst_row[(size_t)i] = roff[(size_t)D - 1][(size_t)i];
    ctx->inst_row[(size_t)i + 1] = roff[(size_t)D - 1][(size_t)i] + lvs[i][nlev[i] - 1].n_sdofs;
  }
  int64_t mx = 0;
  for (int i = 0; i <= n_inst; ++i) seg[(size_t)i] = ctx->inst_row[(size_t)i] * b;
  for (int i = 0; i < n_inst; ++i) mx = std::max(mx, seg[(size_t)i + 1] - seg[(size_t)i]);
  ctx->max_seg = mx;
  STV_TRY(upload(ctx, &ctx->seg_off, seg.data(), seg.size()));
  STV_HIP(hipStreamSynchronize(ctx->stream));
  ctx->have_hier = true;
  return STV_OK;
}

}  // namespace

// ============================================================== public ABI
extern "C" {

int stv_create(stv_ctx** out, int device, void* hip_stream) {
  g_create_err.clear();
  if (!out) { g_create_err = "out is NULL"; return STV_EINVAL; }
  *out = nullptr;
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    g_create_err = std::string("no HIP device: ") + hipGetErrorString(e);
    return STV_EHIP;
  }
  if (device < 0 || device >= ndev) { g_create_err = "device out of range"; return STV_EINVAL; }
  e = hipSetDevice(device);
  if (e != hipSuccess) { g_create_err = hipGetErrorString(e); return STV_EHIP; }
  stv_ctx* ctx = new (std::nothrow) stv_ctx();
  if (!ctx) { g_create_err = "host allocation failed"; return STV_ENOMEM; }
  ctx->device = device;
  ctx->stream = (hipStream_t)hip_stream;
  if (hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->side2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_gj[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_gj[1], hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_step[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_step[1], hipEventDisableTiming) != hipSuccess) {
    g_create_err = "creation of the internal stream/events failed";
    delete ctx;
    return STV_EHIP;
  }
  // the fixed workspace's address on this device; without it only
  // stv_vcycle_noalloc is unavailable (it then reports STV_EHIP)
  if (resolve_scratch(device, &ctx->noalloc_ws) != hipSuccess) {
    (void)hipGetLastError();
    ctx->noalloc_ws = nullptr;
  }
  if (ensure_scalars(ctx, 1) != STV_OK) {
    g_create_err = "allocation of the scalar buffers failed";
    dfree(ctx->scal);
    (void)hipStreamDestroy(ctx->side);
    (void)hipEventDestroy(ctx->ev_fork);
    (void)hipEventDestroy(ctx->ev_join);
    (void)hipEventDestroy(ctx->ev_step[0]);
    (void)hipEventDestroy(ctx->ev_step[1]);
    delete ctx;
    return STV_ENOMEM;
  }
  *out = ctx;
  return STV_OK;
}

void stv_destroy(stv_ctx* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipStreamSynchronize(ctx->stream);
  free_hierarchy(ctx);
  dfree(ctx->scal);
  if (ctx->hscal) (void)hipHostFree(ctx->hscal);
  if (ctx->hstep) (void)hipHostFree(ctx->hstep);
  for (auto& t : ctx->pending) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->cap_stream) {
    (void)hipStreamSynchronize(ctx->cap_stream);
    (void)hipStreamDestroy(ctx->cap_stream);
  }
  if (ctx->side2) {
    (void)hipStreamSynchronize(ctx->side2);
    (void)hipStreamDestroy(ctx->side2);
  }
  for (auto e : ctx->ev_gj)
    if (e) (void)hipEventDestroy(e);
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
  for (auto e : ctx->ev_step)
    if (e) (void)hipEventDestroy(e);
  delete ctx;
}

const char* stv_last_error(const stv_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

int stv_validate_hierarchy(int n_levels, int dim, int k, const stv_level* lv, char* err,
                           size_t errlen) {
  std::string msg;
  const bool ok = validate_impl(n_levels, dim, k, lv, msg);
  if (err && errlen) {
    std::snprintf(err, errlen, "%s", msg.c_str());
  }
  return ok ? STV_OK : STV_EINVAL;
}

int stv_set_hierarchy(stv_ctx* ctx, int n_levels, int dim, int k, const stv_level* lv) {
  if (!ctx) return STV_EINVAL;
  return setup_packed(ctx, 1, dim, k, &n_levels, &lv);
}

int stv_set_batch(stv_ctx* ctx, int n_inst, int dim, int k, const int* n_levels,
                  const stv_level* const* levels) {
  if (!ctx) return STV_EINVAL;
  if (n_inst < 1 || n_inst > 65535) return fail(ctx, STV_EINVAL, "n_inst must be in [1, 65535]");
  if (!n_levels || !levels) return fail(ctx, STV_EINVAL, "n_levels and levels must not be NULL");
  return setup_packed(ctx, n_inst, dim, k, n_levels, levels);
}

// Real block diagonalisation of the time matrix K = D^-1 C (D = diag(tw),
// b <= 4) of an operator C (x) M + D (x) A: K = V T V^-1 with T block
// diagonal, a 1 x 1 block per real eigenvalue and [[al, be], [-be, al]] per
// pair al +- i be (columns Re v, Im v of V).  Then
//   (C (x) M + D (x) A)^-1 = (V (x) I) blockdiag_p(T_p (x) M + I (x) A)^-1 (W (x) I)
// with W = V^-1 D^-1, so each block is inverted on its own.  Eigenvalues are
// the roots of the characteristic polynomial (Newton's identities for the
// coefficients, Durand-Kerner iterations for the roots), eigenvectors null
// vectors of K - lambda I by complete pivoting.  Returns false (use the
// whole matrix) when there would be a single real block, when K V = V T
// fails to working accuracy, or when V is ill-conditioned.  A single pair
// (dG(1)) is kept: its block is the real form of a complex matrix of order
// n_s, eliminated with complex pivots in half the panels.
struct TimeSplit {
  int nblk = 0;
  int sz[4] = {}, first[4] = {};
  double t[4][4] = {};   // per block, 2 x 2 row-major
  double T[16] = {};     // the whole b x b block diagonal T, row-major
  double V[16] = {}, W[16] = {};
};

static bool time_split(const double* C, const double* tw, int b, TimeSplit& out) {
  typedef std::complex<double> cd;
  if (b < 2 || b > 4) return false;
  double K[16];
  double kmax = 0.0;
  for (int i = 0; i < b; ++i) {
    if (!(tw[i] != 0.0)) return false;
    for (int l = 0; l < b; ++l) {
      K[i * b + l] = C[i * b + l] / tw[i];
      kmax = std::max(kmax, std::fabs(K[i * b + l]));
    }
  }
  if (!(kmax > 0.0) || !std::isfinite(kmax)) return false;
  // characteristic polynomial lambda^b + c[1] lambda^(b-1) + ... + c[b]
  double P[16], Q[16], ptr[5] = {}, c[5] = {1.0};
  for (int e = 0; e < b * b; ++e) P[e] = K[e];
  for (int k = 1; k <= b; ++k) {
    double tr = 0.0;
    for (int i = 0; i < b; ++i) tr += P[i * b + i];
    ptr[k] = tr;
    for (int i = 0; i < b; ++i)
      for (int l = 0; l < b; ++l) {
        double acc = 0.0;
        for (int j = 0; j < b; ++j) acc += P[i * b + j] * K[j * b + l];
        Q[i * b + l] = acc;
      }
    for (int e = 0; e < b * b; ++e) P[e] = Q[e];
  }
  for (int k = 1; k <= b; ++k) {
    double acc = ptr[k];
    for (int j = 1; j < k; ++j) acc += c[j] * ptr[k - j];
    c[k] = -acc / k;
  }
  auto poly = [&](cd z) {
    cd v = 1.0;
    for (int k = 1; k <= b; ++k) v = v * z + c[k];
    return v;
  };
  cd z[4];
  const cd seed(0.4, 0.9);
  cd pw = 1.0;
  for (int k = 0; k < b; ++k) { pw *= seed; z[k] = pw * kmax; }
  for (int it = 0; it < 500; ++it) {
    double delta = 0.0;
    for (int k = 0; k < b; ++k) {
      cd den = 1.0;
      for (int j = 0; j < b; ++j)
        if (j != k) den *= (z[k] - z[j]);
      if (std::abs(den) == 0.0) return false;
      const cd step = poly(z[k]) / den;
      z[k] -= step;
      delta = std::max(delta, std::abs(step));
    }
    if (delta <= 1e-15 * kmax) break;
  }
  // eigenvector of each root: null vector of K - lambda I
  auto null_vector = [&](cd lam, cd* v) {
    cd M[16];
    int cperm[4];
    for (int i = 0; i < b; ++i) {
      cperm[i] = i;
      for (int l = 0; l < b; ++l) M[i * b + l] = cd(K[i * b + l]) - (i == l ? lam : cd(0.0));
    }
    for (int k = 0; k < b - 1; ++k) {
      int pr = k, pc = k;
      double best = -1.0;
      for (int i = k; i < b; ++i)
        for (int l = k; l < b; ++l)
          if (std::abs(M[i * b + l]) > best) { best = std::abs(M[i * b + l]); pr = i; pc = l; }
      if (!(best > 0.0)) return false;
      for (int l = 0; l < b; ++l) std::swap(M[k * b + l], M[pr * b + l]);
      for (int i = 0; i < b; ++i) std::swap(M[i * b + k], M[i * b + pc]);
      std::swap(cperm[k], cperm[pc]);
      for (int i = k + 1; i < b; ++i) {
        const cd f = M[i * b + k] / M[k * b + k];
        for (int l = k; l < b; ++l) M[i * b + l] -= f * M[k * b + l];
      }
    }
    cd y[4];
    y[b - 1] = 1.0;
    for (int k = b - 2; k >= 0; --k) {
      cd acc = 0.0;
      for (int l = k + 1; l < b; ++l) acc += M[k * b + l] * y[l];
      y[k] = -acc / M[k * b + k];
    }
    double mx = 0.0;
    for (int k = 0; k < b; ++k) mx = std::max(mx, std::abs(y[k]));
    for (int k = 0; k < b; ++k) v[cperm[k]] = y[k] / mx;
    return true;
  };
  const double tol_im = 1e-9 * kmax;
  TimeSplit S;
  int col = 0;
  double T[16] = {};
  // real eigenvalues first, then one representative per pair
  for (int pass = 0; pass < 2; ++pass)
    for (int k = 0; k < b; ++k) {
      const bool real = std::fabs(z[k].imag()) <= tol_im;
      if ((pass == 0) != real) continue;
      if (!real && z[k].imag() < 0.0) continue;
      cd v[4];
      if (!null_vector(real ? cd(z[k].real(), 0.0) : z[k], v)) return false;
      if (S.nblk >= 4) return false;
      S.first[S.nblk] = col;
      if (real) {
        if (col + 1 > b) return false;
        for (int i = 0; i < b; ++i) S.V[i * b + col] = v[i].real();
        T[col * b + col] = z[k].real();
        S.sz[S.nblk] = 1;
        S.t[S.nblk][0] = z[k].real();
        col += 1;
      } else {
        if (col + 2 > b) return false;
        const double al = z[k].real(), be = z[k].imag();
        for (int i = 0; i < b; ++i) {
          S.V[i * b + col] = v[i].real();
          S.V[i * b + col + 1] = v[i].imag();
        }
        T[col * b + col] = al; T[col * b + col + 1] = be;
        T[(col + 1) * b + col] = -be; T[(col + 1) * b + col + 1] = al;
        S.sz[S.nblk] = 2;
        S.t[S.nblk][0] = al; S.t[S.nblk][1] = be; S.t[S.nblk][2] = -be; S.t[S.nblk][3] = al;
        col += 2;
      }
      ++S.nblk;
    }
  if (col != b || (S.nblk < 2 && S.sz[0] != 2)) return false;
  // K V = V T to working accuracy
  double dev = 0.0;
  for (int i = 0; i < b; ++i)
    for (int l = 0; l < b; ++l) {
      double kv = 0.0, vt = 0.0;
      for (int j = 0; j < b; ++j) {
        kv += K[i * b + j] * S.V[j * b + l];
        vt += S.V[i * b + j] * T[j * b + l];
      }
      dev = std::max(dev, std::fabs(kv - vt));
    }
  if (!(dev <= 1e-10 * kmax)) return false;
  for (int e = 0; e < b * b; ++e) S.T[e] = T[e];
  // W = V^-1 D^-1 (Gauss-Jordan with partial pivoting), conditioning check
  double A[16], I[16];
  for (int e = 0; e < b * b; ++e) { A[e] = S.V[e]; I[e] = 0.0; }
  for (int i = 0; i < b; ++i) I[i * b + i] = 1.0;
  double vnorm = 0.0;
  for (int i = 0; i < b; ++i) {
    double rs = 0.0;
    for (int l = 0; l < b; ++l) rs += std::fabs(S.V[i * b + l]);
    vnorm = std::max(vnorm, rs);
  }
  for (int k = 0; k < b; ++k) {
    int pr = k;
    for (int i = k + 1; i < b; ++i)
      if (std::fabs(A[i * b + k]) > std::fabs(A[pr * b + k])) pr = i;
    if (!(std::fabs(A[pr * b + k]) > 0.0)) return false;
    for (int l = 0; l < b; ++l) { std::swap(A[k * b + l], A[pr * b + l]); std::swap(I[k * b + l], I[pr * b + l]); }
    const double ip = 1.0 / A[k * b + k];
    for (int l = 0; l < b; ++l) { A[k * b + l] *= ip; I[k * b + l] *= ip; }
    for (int i = 0; i < b; ++i)
      if (i != k) {
        const double f = A[i * b + k];
        for (int l = 0; l < b; ++l) { A[i * b + l] -= f * A[k * b + l]; I[i * b + l] -= f * I[k * b + l]; }
      }
  }
  double inorm = 0.0;
  for (int i = 0; i < b; ++i) {
    double rs = 0.0;
    for (int l = 0; l < b; ++l) rs += std::fabs(I[i * b + l]);
    inorm = std::max(inorm, rs);
  }
  if (!(vnorm * inorm <= 1e8)) return false;
  for (int c2 = 0; c2 < b; ++c2)
    for (int l = 0; l < b; ++l) S.W[c2 * b + l] = I[c2 * b + l] / tw[l];
  out = S;
  return true;
}

// Coarse members grouped by order (one batched elimination per group), their
// buffers, the coarse inverse store and the member descriptors.  A member on
// a level with spatial factors whose time matrix splits (time_split) is
// inverted block by block: every block is built in real form of order 2 n_s
// (a pair is the real form of a complex matrix, a real eigenvalue two
// uncoupled copies), the blocks join one group per order, eliminated with
// complex pivots by the tournament, and the member is applied from their
// inverses (KronCoarse) instead of a whole stored inverse.
static int make_coarse_groups(stv_ctx* ctx) {
  const int b = ctx->b;
  std::vector<CoarseGroup>& groups = ctx->cgroups;
  for (int g = 0; g < kMaxLevels; ++g) ctx->h_kc[g].clear();
  // (level, index in h_kc[level]) of each time-decoupled member, in the
  // order of mblocks below
  std::vector<std::pair<int, size_t>> kref;
  // split of each level's time matrix (levels with spatial factors)
  std::vector<TimeSplit> split((size_t)ctx->n_levels);
  std::vector<bool> has_split((size_t)ctx->n_levels, false);
  for (int g = 0; g < ctx->n_levels; ++g)
    if (ctx->lv[g].kron_ma && !ctx->h_coarse[g].empty())
      has_split[(size_t)g] = time_split(ctx->lv[g].kron_C, ctx->lv[g].kron_tw, b, split[(size_t)g]);
  // whole members: one group per order; blocks of time-decoupled members:
  // one group, each block padded with the identity to the largest order
  // (the blocks then share every launch of one elimination chain)
  auto group_of = [&](int64_t order, bool kron) -> CoarseGroup& {
    for (auto& G : groups)
      if (G.kron == kron && G.n0 == order) return G;
    groups.emplace_back();
    groups.back().n0 = order;
    groups.back().kron = kron;
    return groups.back();
  };
  // block slots of the time-decoupled members: (group index, slot in group)
  struct BlockRef { size_t gi; size_t slot; };
  std::vector<std::vector<BlockRef>> mblocks;
  int64_t coarse_total = 0;
  for (int g = 0; g < ctx->n_levels; ++g)
    for (size_t q = 0; q < ctx->h_coarse[g].size(); ++q) {
      CoarseDesc& c = ctx->h_coarse[g][q];
      const int64_t n0 = (int64_t)c.n_s * b;
      if (!has_split[(size_t)g]) {
        c.inv_off = coarse_total;
        coarse_total += n0 * n0;
        CoarseGroup& G = group_of(n0, false);
        G.lev.push_back(g);
        G.idx.push_back((int)q);
        continue;
      }
      c.inv_off = -1;                // no whole inverse
      const TimeSplit& S = split[(size_t)g];
      KronCoarse R{};
      R.nblk = S.nblk;
      R.n_s = c.n_s;
      R.row_off = c.row_off;
      for (int e = 0; e < 16; ++e) { R.V[e] = S.V[e]; R.W[e] = S.W[e]; }
      std::vector<BlockRef> refs;
      for (int p = 0; p < S.nblk; ++p) {
        R.sz[p] = S.sz[p];
        R.first[p] = S.first[p];
        CoarseGroup& G = group_of(2 * (int64_t)c.n_s, true);
        G.lev.push_back(g);
        G.idx.push_back((int)q);
        G.part.push_back(p);
        refs.push_back({(size_t)(&G - groups.data()), G.lev.size() - 1});
      }
      mblocks.push_back(refs);
      kref.emplace_back(g, ctx->h_kc[g].size());
      ctx->h_kc[g].push_back(R);
    }
  ctx->coarse_elems = coarse_total;
  if (coarse_total > 0) STV_TRY(dalloc(ctx, &ctx->coarse_inv, (size_t)coarse_total));
  // per group: plan, descriptors, buffers
  for (size_t gi = 0; gi < groups.size(); ++gi) {
    CoarseGroup& G = groups[gi];
    G.plan = gj_plan(G.n0, ctx->coarse_algo, G.kron);
    G.np = (G.n0 + G.plan.pad - 1) / G.plan.pad * G.plan.pad;
    if (G.np > G.plan.max_n)
      return fail(ctx, STV_EINVAL, "coarse level larger than " + std::to_string(G.plan.max_n) + " unknowns");
    const int64_t cnt = (int64_t)G.lev.size(), np = G.np;
    const int64_t nbo = std::max(G.plan.nb, G.plan.no);
    GjWork& w = G.w;
    w = GjWork{};
    w.sA = np * np;
    w.sV = np;
    w.sB = nbo * np;
    w.sP = 2 * G.plan.nb * np;
    w.sS = 2 * (int64_t)G.plan.no * np;
    w.sBin = (int64_t)G.plan.nb * G.plan.no;
    std::vector<CoarseDesc> hd;
    if (!G.kron) {
      for (size_t m = 0; m < G.lev.size(); ++m) hd.push_back(ctx->h_coarse[G.lev[m]][(size_t)G.idx[m]]);
    } else {
      // blocks in real form (order 2 n_s each)
      std::vector<KronBlockDesc> kd;
      for (size_t m = 0; m < G.lev.size(); ++m) {
        const CoarseDesc& c = ctx->h_coarse[G.lev[m]][(size_t)G.idx[m]];
        CoarseDesc cb = c;
        cb.n_s = (int32_t)(2 * (int64_t)c.n_s);
        cb.inv_off = -1;
        hd.push_back(cb);
        const DevLevel& L = ctx->lv[G.lev[m]];
        KronBlockDesc k{};
        k.rowptr = L.rowptr;
        k.col = L.col;
        k.ma = L.kron_ma;
        k.row_off = c.row_off;
        k.n_s = c.n_s;
        // a real eigenvalue: two uncoupled copies (T = lambda I)
        const TimeSplit& S = split[(size_t)G.lev[m]];
        const int p = G.part[m];
        const bool pair = S.sz[p] == 2;
        k.t[0] = S.t[p][0];
        k.t[1] = pair ? S.t[p][1] : 0.0;
        k.t[2] = pair ? S.t[p][2] : 0.0;
        k.t[3] = pair ? S.t[p][3] : S.t[p][0];
        kd.push_back(k);
      }
      STV_TRY(upload(ctx, &G.d_kdesc, kd.data(), kd.size()));
    }
    STV_TRY(upload(ctx, &G.d_desc, hd.data(), hd.size()));
    STV_TRY(dalloc(ctx, &w.A, (size_t)(cnt * w.sA)));
    STV_TRY(dalloc(ctx, &w.rpiv, (size_t)(cnt * w.sV)));
    STV_TRY(dalloc(ctx, &w.used, (size_t)(cnt * w.sV)));
    STV_TRY(dalloc(ctx, &w.B, (size_t)(cnt * w.sB)));
    STV_TRY(dalloc(ctx, &w.P, (size_t)(cnt * w.sP)));
    STV_TRY(dalloc(ctx, &G.rinv, (size_t)(cnt * w.sV)));
    if (G.plan.no > 0) {
      STV_TRY(dalloc(ctx, &w.S, (size_t)(cnt * w.sS)));
      STV_TRY(dalloc(ctx, &w.Bin, (size_t)(cnt * w.sBin)));
    }
    if (G.plan.algo == 3) {
      // the workgroups' lists and, for the merge tree, the lists and
      // arrival counters of its nodes (fewer than a third more)
      w.sC = 2 * ((np + 255) / 256 * G.plan.nb);
      w.sZ = 2 * (int64_t)G.plan.nb * G.plan.no;
      w.sK = np / 64 + 8;
      STV_TRY(dalloc(ctx, &w.cand, (size_t)(cnt * w.sC)));
      STV_TRY(dalloc(ctx, &w.Z, (size_t)(cnt * w.sZ)));
      STV_TRY(dalloc(ctx, &w.counter, (size_t)(cnt * w.sK)));
    }
  }
  // time-decoupled members: where their blocks' inverses and pivot records
  // are left by the elimination
  for (size_t k = 0; k < kref.size(); ++k) {
    KronCoarse& R = ctx->h_kc[kref[k].first][kref[k].second];
    for (int p = 0; p < R.nblk; ++p) {
      const BlockRef& br = mblocks[k][(size_t)p];
      const CoarseGroup& G = groups[br.gi];
      const int64_t slot = (int64_t)br.slot;
      R.S[p] = G.w.A + slot * G.w.sA;
      R.rpiv[p] = G.w.rpiv + slot * G.w.sV;
      R.rinv[p] = G.rinv + slot * G.w.sV;
      R.ld[p] = G.np;
      R.paired[p] = G.plan.pair ? 1 : 0;
    }
  }
  // device descriptors per level: the members with a whole inverse (offsets
  // now known) and the time-decoupled ones
  for (int g = 0; g < ctx->n_levels; ++g) {
    dfree(ctx->d_coarse[g]);
    dfree(ctx->d_kc[g]);
    std::vector<CoarseDesc> whole;
    ctx->coarse_max_n0[g] = 0;
    for (const CoarseDesc& c : ctx->h_coarse[g])
      if (c.inv_off >= 0) {
        whole.push_back(c);
        ctx->coarse_max_n0[g] = std::max<int64_t>(ctx->coarse_max_n0[g], (int64_t)c.n_s * b);
      }
    ctx->n_whole[g] = (int)whole.size();
    if (!whole.empty()) STV_TRY(upload(ctx, &ctx->d_coarse[g], whole.data(), whole.size()));
    ctx->kc_max_ns[g] = 0;
    ctx->kc_max_blocks[g] = 0;
    for (const KronCoarse& R : ctx->h_kc[g]) {
      ctx->kc_max_ns[g] = std::max(ctx->kc_max_ns[g], R.n_s);
      ctx->kc_max_blocks[g] = std::max(ctx->kc_max_blocks[g], R.nblk);
    }
    if (!ctx->h_kc[g].empty())
      STV_TRY(upload(ctx, &ctx->d_kc[g], ctx->h_kc[g].data(), ctx->h_kc[g].size()));
  }
  return STV_OK;
}

// Stores of every cell's inverse rows for a layout (all rows or the owned
// rows) and element type: per-level row offsets and the store itself.
static int make_inverse_stores(stv_ctx* ctx, int fp32, int full) {
  const int b = ctx->b;
  for (int g = 0; g < ctx->n_levels; ++g) {
    DevLevel& L = ctx->lv[g];
    dfree(L.inv_off);
    dfree(L.inv_store);
    dfree(L.dec_tab);
    dfree(L.dec_code);
    L.inv_elems = 0;
    L.dec = 0;
    L.cx = 0;
    if (L.n_cells == 0) continue;
    const int n = L.n_ls * b;
    // with spatial factors, the owned-row layout of a level whose cell
    // problems fit one wavefront stores the time-decoupled inverse: one row
    // of n values per owned spatial DoF instead of b rows (CellSplit)
    L.dec = 0;
    TimeSplit S;
    if (!full && L.kron_ma && n <= 64 && inverse_fits_regs(b, L.n_ls) &&
        time_split(L.kron_C, L.kron_tw, b, S)) {
      CellSplit& c = L.split;
      c = CellSplit{};
      c.b = b;
      c.nblk = S.nblk;
      int o = 0;
      for (int p = 0; p < S.nblk; ++p) {
        c.sz[p] = S.sz[p];
        c.first[p] = S.first[p];
        c.off[p] = o;
        o += S.sz[p] * L.n_ls;
      }
      for (int e = 0; e < 16; ++e) {
        c.T[e] = S.T[e];
        c.V[e] = S.V[e];
        c.W[e] = S.W[e];
      }
      // the sweep's per-lane constants (stored column j = lane)
      std::vector<double> tab((size_t)2 * b * 64);
      std::vector<int32_t> code(64, 0);
      auto enc = [](int v) { return v == 1 ? 1 : v == -1 ? 3 : 0; };
      for (int lane = 0; lane < 64; ++lane) {
        const int jl = std::min(lane, n - 1), cl = jl % b, il = lane % b;
        for (int l = 0; l < b; ++l) {
          tab[(size_t)l * 64 + lane] = S.W[cl * b + l];
          tab[(size_t)(b + l) * 64 + lane] = S.V[il * b + l];
        }
        int srca = 0, srcb = 0, ca[4] = {}, cb[4] = {};
        for (int p = 0; p < S.nblk; ++p) {
          const int rel = lane - c.off[p], sz = S.sz[p], f = S.first[p];
          if (rel < 0 || rel >= sz * L.n_ls) continue;
          const bool im = rel >= L.n_ls;
          const int sp = im ? rel - L.n_ls : rel;
          srca = sp * b + f;
          srcb = sp * b + f + (sz == 2 ? 1 : 0);
          if (sz == 1) {
            ca[f] = 1;
          } else if (!im) {
            ca[f] = 1;
            cb[f + 1] = 1;
          } else {
            cb[f] = -1;
            ca[f + 1] = 1;
          }
        }
        int w = srca | (srcb << 6);
        for (int o = 0; o < b; ++o) w |= (enc(ca[o]) << (12 + 2 * o)) | (enc(cb[o]) << (12 + 2 * b + 2 * o));
        code[(size_t)lane] = w;
      }
      STV_TRY(upload(ctx, &L.dec_tab, tab.data(), tab.size()));
      STV_TRY(upload(ctx, &L.dec_code, code.data(), code.size()));
      L.dec = 1;
    }
    // a 3d dG(1) level with spatial factors whose time matrix has one complex
    // pair: the inverses are computed from the complex decoupled block (half
    // the pivot steps and flops of the real elimination); the owned-rows
    // layout stores them time-decoupled (one complex row per owned spatial
    // DoF, as the 2d split does), the full layout plainly
    if (!L.dec && L.kron_ma && b == 2 && L.n_ls == 85 && time_split(L.kron_C, L.kron_tw, b, S) &&
        S.nblk == 1 && S.sz[0] == 2 && S.T[0] == S.T[3] && S.T[1] == -S.T[2]) {
      CellSplit& c = L.split;
      c = CellSplit{};
      c.b = b;
      c.nblk = 1;
      c.sz[0] = 2;
      c.first[0] = 0;
      c.off[0] = 0;
      for (int e = 0; e < 16; ++e) {
        c.T[e] = S.T[e];
        c.V[e] = S.V[e];
        c.W[e] = S.W[e];
      }
      L.cx = 1;
      L.dec = full ? 0 : 1;
    }
    // rows stored densely (padding each row to a 128-byte boundary was
    // measured slower: the sweep reads whole cells as one contiguous stream)
    L.inv_ld = n;
    std::vector<int64_t> off((size_t)L.n_cells);
    int64_t tot = 0;
    for (int32_t c = 0; c < L.n_cells; ++c) {
      off[(size_t)c] = tot;
      const int no = L.h_own_ptr[(size_t)c + 1] - L.h_own_ptr[(size_t)c];
      const int rows = full ? n : L.dec ? no : no * b;
      tot += (int64_t)rows * L.inv_ld;
    }
    STV_TRY(upload(ctx, &L.inv_off, off.data(), off.size()));
    if (fp32) {
      float* p = nullptr;
      STV_TRY(dalloc(ctx, &p, (size_t)tot));
      L.inv_store = p;
    } else {
      double* p = nullptr;
      STV_TRY(dalloc(ctx, &p, (size_t)tot));
      L.inv_store = p;
    }
    L.inv_elems = tot;
  }
  return STV_OK;
}

int stv_build_cell_inverses(stv_ctx* ctx, int storage, int* bad_level, int* bad_cell) {
  STV_TRY(check_ctx(ctx, true, false));
  if (bad_level) *bad_level = -1;
  if (bad_cell) *bad_cell = -1;
  const int fp32 = storage & STV_F32;
  const int full = (storage & STV_STORE_FULL) ? 1 : 0;
  if (storage & ~(STV_F32 | STV_STORE_FULL)) return fail(ctx, STV_EINVAL, "unknown storage flags");
  STV_HIP(hipSetDevice(ctx->device));
  STV_HIP(hipStreamSynchronize(ctx->stream));
  if (ctx->side) STV_HIP(hipStreamSynchronize(ctx->side));
  ctx->have_inv = false;
  const int b = ctx->b;
  hipStream_t s = ctx->stream;
  // the coarse factorisations run on the internal stream, overlapping the
  // cell inverses, or on the caller's stream ahead of them
  hipStream_t side = ctx->coarse_overlap ? ctx->side : ctx->stream;

  // ---- workspace: made on the first build of a hierarchy and whenever the
  // layout, the element type or the coarse algorithm changes; a captured
  // V-cycle is dropped only when a buffer it reads moved
  int rc = STV_OK;
  bool moved = false;
  if (ctx->inv_layout != full || ctx->inv_type != fp32) {
    ctx->inv_layout = ctx->inv_type = -1;
    rc = make_inverse_stores(ctx, fp32, full);
    if (rc == STV_OK) {
      ctx->inv_layout = full;
      ctx->inv_type = fp32;
    }
    moved = true;
  }
  for (int g = 0; g < ctx->n_levels && rc == STV_OK; ++g) {
    const DevLevel& L = ctx->lv[g];
    if (L.n_cells == 0 || ctx->inv_status[g]) continue;
    rc = dalloc(ctx, &ctx->inv_status[g], (size_t)L.n_cells);
    if (rc == STV_OK && !inverse_fits_regs(b, L.n_ls)) {
      ctx->inv_slots[g] = std::min<int>(L.n_cells, 1024);
      rc = dalloc(ctx, &ctx->inv_scratch[g], (size_t)ctx->inv_slots[g] * L.n_ls * b * L.n_ls * b);
    }
  }
  if (rc == STV_OK && ctx->cgroups_algo != ctx->coarse_algo) {
    free_coarse_groups(ctx);
    rc = make_coarse_groups(ctx);
    if (rc == STV_OK) ctx->cgroups_algo = ctx->coarse_algo;
    moved = true;
  }
  int members = 0;
  for (const auto& G : ctx->cgroups) members += (int)G.lev.size();
  const int nrep = ctx->n_levels + members;
  if (rc == STV_OK && ctx->n_report != nrep) {
    dfree(ctx->inv_report);
    if (ctx->h_report) (void)hipHostFree(ctx->h_report);
    ctx->h_report = nullptr;
    ctx->n_report = 0;
    rc = dalloc(ctx, &ctx->inv_report, (size_t)nrep);
    if (rc == STV_OK &&
        hipHostMalloc((void**)&ctx->h_report, sizeof(int) * (size_t)nrep, hipHostMallocDefault) !=
            hipSuccess) {
      ctx->h_report = nullptr;
      rc = fail(ctx, STV_ENOMEM, "pinned host allocation of the build report failed");
    }
    if (rc == STV_OK) ctx->n_report = nrep;
  }
  if (rc != STV_OK) {
    free_inverses(ctx);
    return rc;
  }
  if (moved) {
    ++ctx->generation;
    free_graph(ctx);
  }
  ctx->inv_fp32 = fp32;
  ctx->inv_full = full;

  // ---- launch: cell inverses on the caller's stream, coarse factorisations
  // on the internal stream (it starts after everything queued before it);
  // the report starts at 0x7f7f7f7f ("no flagged cell") per level
  int* rep = ctx->inv_report;
  hipError_t e = hipMemsetAsync(rep, 0x7f, sizeof(int) * (size_t)nrep, s);
  hipStream_t inv = s;
  if (e == hipSuccess && side != s) {
    e = hipEventRecord(ctx->ev_fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(side, ctx->ev_fork, 0);
  }
  // while the coarse factorisations run beside them, the one-wavefront cell
  // inverses leave STV_CHAIN_VGPRS registers free on every SIMD: the
  // elimination chain's latency-bound workgroups then start at once instead
  // of waiting for the inverse kernel to drain whole compute units
  int n_cu = 0;
  if (STV_CHAIN_VGPRS > 0 && side != s && !ctx->cgroups.empty()) {
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, ctx->device) !=
        hipSuccess)
      n_cu = 0;
  }
  auto cell_inverses = [&]() {
    for (int g = 1; g < ctx->n_levels && e == hipSuccess; ++g) {
      const DevLevel& L = ctx->lv[g];
      if (L.n_cells == 0) continue;
      Timed t(ctx, KC_INVERSE, g, inv);
      e = launch_cell_inverses(inv, b, L, fp32, full, ctx->inv_status[g], ctx->inv_scratch[g],
                               ctx->inv_slots[g], n_cu, STV_CHAIN_VGPRS, ctx->inverse_cus);
      if (e == hipSuccess) e = launch_first_flag(inv, ctx->inv_status[g], L.n_cells, rep + g);
      t.done();
    }
  };
  if (side != s) cell_inverses();
  int mbase = ctx->n_levels;
  for (auto& G : ctx->cgroups) {
    if (e != hipSuccess) break;
    const int gb = G.kron ? 1 : b;   // a block's descriptor holds its order in n_s
    Timed t(ctx, KC_COARSE_FACTOR, 0, side);
    const int cnt = (int)G.lev.size();
    int32_t max_rows = 0;
    for (size_t m = 0; m < G.lev.size(); ++m)
      max_rows = std::max(max_rows, ctx->h_coarse[G.lev[m]][(size_t)G.idx[m]].n_s);
    e = launch_fill(side, G.w.A, cnt * G.w.sA, 0.0);
    if (e == hipSuccess)
      e = G.kron ? launch_kron_block_dense(side, G.d_kdesc, cnt, max_rows, G.w.A, G.w.sA, G.np)
                 : launch_bsr_to_dense(side, b, G.d_desc, cnt, max_rows, G.w.A, G.w.sA, G.np);
    if (e == hipSuccess) e = launch_set_diag(side, G.d_desc, cnt, gb, G.w.A, G.w.sA, G.np);
    if (e == hipSuccess) e = hipMemsetAsync(G.w.used, 0, (size_t)(cnt * G.w.sV), side);
    if (e == hipSuccess && G.w.counter)
      e = hipMemsetAsync(G.w.counter, 0, sizeof(unsigned) * (size_t)(cnt * G.w.sK), side);
    const GjAux aux{ctx->side2, ctx->ev_gj[0], ctx->ev_gj[1]};
    if (e == hipSuccess) e = launch_gj(side, G.plan, G.w, G.np, cnt, ctx->coarse_lookahead ? &aux : nullptr);
    // pivot records -> inverse permutations and verdicts, then the
    // unpermuted inverses (the blocks of time-decoupled members are applied
    // where the elimination left them, through their pivot records)
    if (e == hipSuccess)
      e = launch_gj_invert_perm(side, G.w.rpiv, G.w.sV, G.np, G.d_desc, cnt, gb, G.rinv,
                                rep + mbase);
    if (e == hipSuccess && !G.kron)
      e = launch_gj_unpermute(side, G.w.A, G.w.sA, G.np, G.w.rpiv, G.rinv, G.w.sV, G.d_desc, cnt,
                              gb, G.n0, ctx->coarse_inv);
    t.done();
    mbase += cnt;
  }
  if (side == s) {
    cell_inverses();
  } else {
    if (e == hipSuccess) e = hipEventRecord(ctx->ev_join, side);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->ev_join, 0);
  }
  if (e == hipSuccess)
    e = hipMemcpyAsync(ctx->h_report, rep, sizeof(int) * (size_t)nrep, hipMemcpyDeviceToHost, s);
  {
    // every stream drains on every path
    const hipError_t e1 = hipStreamSynchronize(s);
    const hipError_t e2 = hipStreamSynchronize(side);
    (void)hipStreamSynchronize(ctx->side2);
    if (e == hipSuccess) e = (e1 != hipSuccess) ? e1 : e2;
  }
  if (e != hipSuccess) {
    free_inverses(ctx);
    return fail(ctx, STV_EHIP, std::string("inverse build failed: ") + hipGetErrorString(e));
  }
  const int none = 0x7f7f7f7f;
  for (int g = 1; g < ctx->n_levels; ++g)
    if (ctx->lv[g].n_cells > 0 && ctx->h_report[g] != none) {
      if (bad_level) *bad_level = g;
      if (bad_cell) *bad_cell = ctx->h_report[g];
      return fail(ctx, STV_ESINGULAR, "zero pivot in J_T of level " + std::to_string(g) +
                                          " cell " + std::to_string(ctx->h_report[g]));
    }
  mbase = ctx->n_levels;
  for (const auto& G : ctx->cgroups) {
    for (size_t m = 0; m < G.lev.size(); ++m)
      if (ctx->h_report[mbase + (int)m] != 0) {
        if (bad_level) *bad_level = G.lev[m];
        if (bad_cell) *bad_cell = -1;
        return fail(ctx, STV_ESINGULAR,
                    "zero pivot in a coarse matrix (level " + std::to_string(G.lev[m]) + ")");
      }
    mbase += (int)G.lev.size();
  }
  ctx->have_inv = true;
  return STV_OK;
}

int stv_residual(stv_ctx* ctx, int level, const double* r, const double* d, double* out) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level out of range");
  if (!d || !out) return fail(ctx, STV_EINVAL, "d and out must not be NULL");
  if (out == d || out == r) return fail(ctx, STV_EINVAL, "out must not alias r or d");
  return residual(ctx, level, r, d, out);
}

int stv_vanka_sweep(stv_ctx* ctx, int level, const double* r, double* d, int n_sweeps,
                    double omega, int mode) {
  STV_TRY(check_ctx(ctx, true, true));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level must be in [1, n_levels)");
  if (!r || !d) return fail(ctx, STV_EINVAL, "r and d must not be NULL");
  if (n_sweeps < 0) return fail(ctx, STV_EINVAL, "n_sweeps must be >= 0");
  if (!(omega > 0.0) || !std::isfinite(omega)) return fail(ctx, STV_EINVAL, "omega must be positive");
  STV_TRY(check_mode(ctx, mode));
  return sweeps(ctx, level, r, d, n_sweeps, omega, mode, false);
}

int stv_restrict(stv_ctx* ctx, int level, const double* rho, double* r_c) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level must be in [1, n_levels)");
  Timed t(ctx, KC_TRANSFER, 0, nullptr, true);
  STV_HIP(launch_restrict(ctx->stream, ctx->b, ctx->lv[level], rho, r_c));
  t.done();
  return STV_OK;
}

int stv_prolongate_add(stv_ctx* ctx, int level, const double* d_c, double* d) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level must be in [1, n_levels)");
  Timed t(ctx, KC_TRANSFER, 0, nullptr, true);
  STV_HIP(launch_prolongate_add(ctx->stream, ctx->b, ctx->lv[level], d_c, d));
  t.done();
  return STV_OK;
}

int stv_coarse_solve(stv_ctx* ctx, const double* r, double* d) {
  STV_TRY(check_ctx(ctx, true, true));
  if (!r || !d || r == d) return fail(ctx, STV_EINVAL, "r, d must be distinct non-NULL vectors");
  return coarse_apply(ctx, 0, r, d);
}

int stv_vcycle(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p) {
  STV_TRY(check_ctx(ctx, true, true));
  STV_TRY(check_mg(ctx, p));
  if (!r || !d || r == d) return fail(ctx, STV_EINVAL, "r, d must be distinct non-NULL vectors");
  return precond_apply(ctx, r, d, *p);
}

int stv_vcycle_noalloc(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p) {
  STV_TRY(check_ctx(ctx, true, true));
  STV_TRY(check_mg(ctx, p));
  if (!r || !d || r == d) return fail(ctx, STV_EINVAL, "r, d must be distinct non-NULL vectors");
  if (!ctx->noalloc_ws)
    return fail(ctx, STV_EHIP, "the fixed V-cycle workspace has no address on this device");
  // the work vectors the context's own V-cycle keeps per level, carved from
  // the fixed workspace in 256-byte aligned pieces
  const int b = ctx->b;
  const bool corr = p->mode != STV_LAST_WRITER;
  auto piece = [](size_t n) { return (n + 31) / 32 * 32; };
  size_t need = 0;
  for (int g = 0; g < ctx->n_levels; ++g) {
    const DevLevel& L = ctx->lv[g];
    const size_t nst = (size_t)L.n_s * b;
    need += piece(nst);                                   // rho
    if (g < ctx->n_levels - 1) need += 2 * piece(nst);    // r, d
    if (corr && g > 0 && L.n_cells > 0) need += piece((size_t)L.n_cells * L.n_ls * b);
  }
  if (need > kNoAllocDoubles)
    return fail(ctx, STV_EINVAL,
                "the V-cycle needs " + std::to_string(need * 8) + " bytes of work vectors; "
                "stv_vcycle_noalloc holds at most " + std::to_string(kNoAllocDoubles * 8));
  struct Saved { double *rho, *r, *d, *corr; };
  Saved saved[kMaxLevels];
  double* cur = ctx->noalloc_ws;
  for (int g = 0; g < ctx->n_levels; ++g) {
    DevLevel& L = ctx->lv[g];
    saved[g] = Saved{L.rho, L.r, L.d, L.corr};
    const size_t nst = (size_t)L.n_s * b;
    L.rho = cur; cur += piece(nst);
    if (g < ctx->n_levels - 1) {
      L.r = cur; cur += piece(nst);
      L.d = cur; cur += piece(nst);
    }
    if (corr && g > 0 && L.n_cells > 0) {
      L.corr = cur;
      cur += piece((size_t)L.n_cells * L.n_ls * b);
    }
  }
  // eager launches on the caller's stream; no event records (the timer's
  // event pool may allocate), no graph
  const bool timing = ctx->timing;
  ctx->timing = false;
  const int rc = vcycle_level(ctx, ctx->n_levels - 1, r, d, *p);
  ctx->timing = timing;
  for (int g = 0; g < ctx->n_levels; ++g) {
    DevLevel& L = ctx->lv[g];
    L.rho = saved[g].rho;
    L.r = saved[g].r;
    L.d = saved[g].d;
    L.corr = saved[g].corr;
  }
  return rc;
}

int stv_gmres_solve(stv_ctx* ctx, const double* bvec, double* x, const stv_gmres_params* p,
                    stv_gmres_info* info) {
  STV_TRY(check_ctx(ctx, true, true));
  if (!p) return fail(ctx, STV_EINVAL, "params NULL");
  STV_TRY(check_mg(ctx, &p->mg));
  if (!bvec || !x || bvec == x) return fail(ctx, STV_EINVAL, "b, x must be distinct non-NULL vectors");
  if (p->restart < 1 || p->restart > kMaxRestart) return fail(ctx, STV_EINVAL, "restart must be in [1, 256]");
  if (p->max_it < 1) return fail(ctx, STV_EINVAL, "max_it must be >= 1");
  if (p->fixed_iters < 0) return fail(ctx, STV_EINVAL, "fixed_iters must be >= 0");
  if (!(p->rtol >= 0.0)) return fail(ctx, STV_EINVAL, "rtol must be >= 0");
  const int m = p->restart;
  STV_TRY(ensure_workspace(ctx, m));
  const int G = ctx->n_levels - 1;
  const int64_t n = ctx->ws_n;
  const int S = ctx->n_inst;
  const ScalLayout lay{ctx->scal_segs};
  const Segs sg{ctx->seg_off, S, ctx->max_seg};
  hipStream_t s = ctx->stream;
  double* hs = ctx->hscal;
  // every instance runs its own FGMRES; the instances advance in lockstep
  // (one V-cycle and one matrix product serve all of them) and an instance
  // that has stopped only carries its iterate along
  struct Inst {
    double bnorm = 0, target = 0, beta = 0;
    bool done = false, cyc = false;
    int iters = 0, restarts = 0, j_end = 0;
    std::vector<double> H, cs, sn, gv;
  };
  std::vector<Inst> in((size_t)S);
  int hist_len = 0;
  auto push_hist = [&](double v) {
    if (info && info->history && hist_len < info->history_cap) info->history[hist_len] = v;
    ++hist_len;
  };
  auto finish = [&](int rc) {
    int conv = 1, it = 0, rs = 0;
    double rr = 0.0;
    for (int z = 0; z < S; ++z) {
      const Inst& I = in[(size_t)z];
      const double rel = I.bnorm > 0 ? I.beta / I.bnorm : 0.0;
      InstInfo& o = ctx->inst_info[(size_t)z];
      o.iters = I.iters;
      o.restarts = I.restarts;
      o.relres = rel;
      o.converged = (rel <= p->rtol) ? 1 : 0;
      conv &= o.converged;
      it = std::max(it, I.iters);
      rs = std::max(rs, I.restarts);
      rr = std::isnan(rel) || std::isnan(rr) ? NAN : std::max(rr, rel);
    }
    if (info) {
      info->iters = it;
      info->restarts = rs;
      info->converged = conv;
      info->true_relres = rr;
      info->history_len = std::min(hist_len, info->history ? info->history_cap : 0);
    }
    resolve_timers(ctx);
    return rc;
  };
  auto inst_name = [&](int z) { return S > 1 ? " of instance " + std::to_string(z) : std::string(); };
  if (!p->use_x0) STV_HIP(launch_fill(s, x, n, 0.0));
  std::vector<double> v2;
  STV_TRY(dots_to_host(ctx, bvec, bvec, n, v2));
  for (int z = 0; z < S; ++z) {
    Inst& I = in[(size_t)z];
    I.bnorm = std::sqrt(v2[(size_t)z]);
    if (!std::isfinite(I.bnorm)) {
      I.beta = NAN;
      return finish(fail(ctx, STV_ENUMERIC, "NaN/Inf in the right-hand side" + inst_name(z)));
    }
    I.target = p->rtol * I.bnorm;
    if (I.bnorm == 0.0) {
      const int64_t o0 = ctx->inst_row[(size_t)z] * ctx->b, o1 = ctx->inst_row[(size_t)z + 1] * ctx->b;
      STV_HIP(launch_fill(s, x + o0, o1 - o0, 0.0));
      I.done = true;
    }
  }
  if (p->use_x0) {
    STV_TRY(residual(ctx, G, bvec, x, ctx->rt));
    STV_TRY(dots_to_host(ctx, ctx->rt, ctx->rt, n, v2));
  } else {
    // x = 0: the initial residual is b itself (b - J 0 = b exactly) and its
    // squared norms are those just reduced
    STV_HIP(hipMemcpyAsync(ctx->rt, bvec, sizeof(double) * (size_t)n, hipMemcpyDeviceToDevice, s));
  }
  double hmax = 0.0;
  for (int z = 0; z < S; ++z) {
    Inst& I = in[(size_t)z];
    if (I.bnorm == 0.0) { I.beta = 0.0; continue; }
    I.beta = std::sqrt(v2[(size_t)z]);
    if (!std::isfinite(I.beta))
      return finish(fail(ctx, STV_ENUMERIC, "NaN/Inf in the initial residual" + inst_name(z)));
    if (I.beta <= I.target && p->fixed_iters == 0) I.done = true;
    hmax = std::max(hmax, I.beta / I.bnorm);
  }
  push_hist(hmax);
  const int budget = p->fixed_iters > 0 ? p->fixed_iters : p->max_it;
  for (auto& I : in) {
    I.H.assign((size_t)(m + 1) * m, 0.0);
    I.cs.assign((size_t)m, 0.0);
    I.sn.assign((size_t)m, 0.0);
    I.gv.assign((size_t)m + 1, 0.0);
  }
  auto any_cycle = [&]() {
    for (const auto& I : in) if (I.cyc) return true;
    return false;
  };
  for (;;) {
    for (auto& I : in) {
      I.cyc = !I.done && I.iters < budget;
      I.j_end = 0;
    }
    if (!any_cycle()) break;
    for (int z = 0; z < S; ++z) {
      Inst& I = in[(size_t)z];
      std::fill(I.H.begin(), I.H.end(), 0.0);
      std::fill(I.gv.begin(), I.gv.end(), 0.0);
      I.gv[0] = I.beta;
      hs[lay.aux() + z] = I.cyc ? v2[(size_t)z] : 0.0;   // ||rt_z||^2 as reduced on the device
    }
    STV_HIP(hipMemcpyAsync(ctx->scal + lay.aux(), hs + lay.aux(), sizeof(double) * S,
                           hipMemcpyHostToDevice, s));
    {
      Timed t(ctx, KC_KRYLOV);
      STV_HIP(launch_scale_by_norm(s, ctx->rt, ctx->scal + lay.aux(), 1, ctx->V, sg));
      t.done();
    }
    // The device work of Arnoldi step j (preconditioner, product, CGS2,
    // normalisation) needs only v_j, which the device computed itself; the
    // host needs the step's coefficients only for the rotations and the
    // stopping test.  So step j + 1 is enqueued before step j's coefficients
    // are awaited, unless step j may end the cycle: then the host waits
    // first (a step enqueued but not taken only costs time, the iterate is
    // formed from the steps taken).  Each step's coefficients go to their
    // own pinned buffer (two in turn).
    int jmax = 0, enq = 0;
    double* hbuf[2] = {hs, ctx->hstep};
    auto enqueue = [&](int j) -> int {
      double* vj = ctx->V + (int64_t)j * n;
      double* zj = ctx->Z + (int64_t)j * n;
      STV_TRY(precond_apply(ctx, vj, zj, p->mg));
      STV_TRY(matvec(ctx, G, zj, ctx->w));
      {
        Timed t(ctx, KC_KRYLOV);
        // CGS2: h1 = V'w, w -= V h1, h2 = V'w, w -= V h2, ||w||.  Each update
        // is fused with the products that follow it (one pass over V and w
        // fewer each; the same blocks and order of operations as the separate
        // kernels), the first while V has at most kKrylovFuse columns.
        STV_HIP(launch_multidot(s, ctx->V, j + 1, ctx->w, n, sg, ctx->partial, ctx->scal + lay.h1(0), kScalR));
        if (j + 1 <= kKrylovFuse) {
          STV_HIP(launch_multiaxpy_dot(s, ctx->V, j + 1, ctx->scal + lay.h1(0), kScalR, -1.0, ctx->w, n, sg,
                                       ctx->partial, ctx->scal + lay.h2(0), kScalR));
        } else {
          STV_HIP(launch_multiaxpy(s, ctx->V, j + 1, ctx->scal + lay.h1(0), kScalR, -1.0, ctx->w, n, sg));
          STV_HIP(launch_multidot(s, ctx->V, j + 1, ctx->w, n, sg, ctx->partial, ctx->scal + lay.h2(0), kScalR));
        }
        STV_HIP(launch_multiaxpy_nrm(s, ctx->V, j + 1, ctx->scal + lay.h2(0), kScalR, -1.0, ctx->w, n, sg,
                                     ctx->partial, ctx->scal + lay.nrm(), 1));
        STV_HIP(launch_scale_by_norm(s, ctx->w, ctx->scal + lay.nrm(), 1, ctx->V + (int64_t)(j + 1) * n, sg));
        t.done();
      }
      STV_HIP(hipMemcpyAsync(hbuf[j & 1], ctx->scal, sizeof(double) * (lay.nrm() + S),
                             hipMemcpyDeviceToHost, s));
      STV_HIP(hipEventRecord(ctx->ev_step[j & 1], s));
      return STV_OK;
    };
    // whether some cycling instance may need a step after step j: a fixed
    // count not reached, or an estimate after step j (the current residual
    // |g_j| times the last step's reduction |s_{j-1}|) above three times the
    // target
    auto may_continue = [&](int j) {
      for (const auto& I : in) {
        if (!I.cyc) continue;
        if (I.iters + 1 >= budget) continue;
        if (p->fixed_iters > 0) return true;
        const double cur = std::fabs(I.gv[(size_t)j]);
        const double rate = j > 0 ? std::fabs(I.sn[(size_t)j - 1]) : 1.0;
        if (!(cur * rate <= 3.0 * I.target)) return true;
      }
      return false;
    };
    for (int j = 0; j < m && any_cycle(); ++j) {
      if (enq == j) {
        STV_TRY(enqueue(j));
        ++enq;
      }
      if (enq == j + 1 && j + 1 < m && may_continue(j)) {
        STV_TRY(enqueue(j + 1));
        ++enq;
      }
      STV_HIP(hipEventSynchronize(ctx->ev_step[j & 1]));
      const double* hj = hbuf[j & 1];
      jmax = j + 1;
      double hist = 0.0;
      bool any = false;
      for (int z = 0; z < S; ++z) {
        Inst& I = in[(size_t)z];
        if (!I.cyc) continue;
        auto Hij = [&](int i, int jj) -> double& { return I.H[(size_t)i * m + jj]; };
        for (int i = 0; i <= j; ++i) Hij(i, j) = hj[lay.h1(z) + i] + hj[lay.h2(z) + i];
        const double hn = std::sqrt(hj[lay.nrm() + z]);
        Hij(j + 1, j) = hn;
        for (int i = 0; i <= j + 1; ++i)
          if (!std::isfinite(Hij(i, j))) {
            I.beta = NAN;
            (void)hipStreamSynchronize(s);
            return finish(fail(ctx, STV_ENUMERIC, "NaN/Inf in the Arnoldi process at step " +
                                                      std::to_string(I.iters) + inst_name(z)));
          }
        const bool breakdown = hn == 0.0;
        for (int i = 0; i < j; ++i) {
          const double tmp = I.cs[(size_t)i] * Hij(i, j) + I.sn[(size_t)i] * Hij(i + 1, j);
          Hij(i + 1, j) = -I.sn[(size_t)i] * Hij(i, j) + I.cs[(size_t)i] * Hij(i + 1, j);
          Hij(i, j) = tmp;
        }
        const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
        I.cs[(size_t)j] = Hij(j, j) / den;
        I.sn[(size_t)j] = Hij(j + 1, j) / den;
        Hij(j, j) = den;
        Hij(j + 1, j) = 0.0;
        I.gv[(size_t)j + 1] = -I.sn[(size_t)j] * I.gv[(size_t)j];
        I.gv[(size_t)j] = I.cs[(size_t)j] * I.gv[(size_t)j];
        ++I.iters;
        I.j_end = j + 1;
        hist = std::max(hist, std::fabs(I.gv[(size_t)j + 1]) / I.bnorm);
        any = true;
        if (p->fixed_iters > 0) {
          if (I.iters >= p->fixed_iters || breakdown) I.cyc = false;
        } else if (std::fabs(I.gv[(size_t)j + 1]) <= I.target || I.iters >= p->max_it || breakdown) {
          I.cyc = false;
        }
      }
      if (any) push_hist(hist);
    }
    // x += Z y per instance, y = R^-1 g (back substitution on the rotated
    // Hessenberg matrix); instances without steps this cycle take y = 0
    for (int z = 0; z < S; ++z) {
      Inst& I = in[(size_t)z];
      double* yz = hs + lay.y(z);
      for (int i = 0; i < jmax; ++i) yz[i] = 0.0;
      for (int i = I.j_end - 1; i >= 0; --i) {
        double acc = I.gv[(size_t)i];
        for (int l = i + 1; l < I.j_end; ++l) acc -= I.H[(size_t)i * m + l] * yz[l];
        yz[i] = acc / I.H[(size_t)i * m + i];
      }
    }
    STV_HIP(hipMemcpyAsync(ctx->scal + lay.y(0), hs + lay.y(0), sizeof(double) * S * kScalR,
                           hipMemcpyHostToDevice, s));
    {
      Timed t(ctx, KC_KRYLOV);
      STV_HIP(launch_multiaxpy(s, ctx->Z, jmax, ctx->scal + lay.y(0), kScalR, 1.0, x, n, sg));
      t.done();
    }
    STV_TRY(residual(ctx, G, bvec, x, ctx->rt));
    STV_TRY(dots_to_host(ctx, ctx->rt, ctx->rt, n, v2));
    for (int z = 0; z < S; ++z) {
      Inst& I = in[(size_t)z];
      if (I.j_end == 0) continue;
      I.beta = std::sqrt(v2[(size_t)z]);
      ++I.restarts;
      if (!std::isfinite(I.beta))
        return finish(fail(ctx, STV_ENUMERIC, "NaN/Inf in the true residual" + inst_name(z)));
      if (p->fixed_iters == 0 && I.beta <= I.target) I.done = true;
      if (p->fixed_iters > 0 && I.iters >= p->fixed_iters) I.done = true;
      if (I.beta == 0.0) I.done = true;
    }
  }
  if (p->fixed_iters == 0)
    for (int z = 0; z < S; ++z) {
      const Inst& I = in[(size_t)z];
      if (I.bnorm > 0.0 && !(I.beta / I.bnorm <= p->rtol))
        return finish(fail(ctx, STV_ENOCONV, "GMRES did not reach rtol within max_it steps" + inst_name(z)));
    }
  return finish(STV_OK);
}

int stv_vcycle_transposed(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p) {
  if (!ctx) return STV_EINVAL;
  if (!p) return fail(ctx, STV_EINVAL, "mg params NULL");
  STV_TRY(check_transposable(ctx, p->mode));
  ctx->transposed = 1;
  const int rc = stv_vcycle(ctx, r, d, p);
  ctx->transposed = 0;
  return rc;
}

int stv_gmres_solve_transposed(stv_ctx* ctx, const double* bvec, double* x,
                               const stv_gmres_params* p, stv_gmres_info* info) {
  if (!ctx) return STV_EINVAL;
  if (!p) return fail(ctx, STV_EINVAL, "params NULL");
  STV_TRY(check_transposable(ctx, p->mg.mode));
  ctx->transposed = 1;
  const int rc = stv_gmres_solve(ctx, bvec, x, p, info);
  ctx->transposed = 0;
  return rc;
}

int stv_cell_contract(stv_ctx* ctx, int level, const double* lam, const double* x, int n_ref,
                      const double* Kref, const int32_t* kptr, const int32_t* kidx,
                      const double* kw, const double* tw, double* out) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels || ctx->lv[level].n_cells == 0)
    return fail(ctx, STV_EINVAL, "level out of range or without smoothed cells");
  if (!lam || !x || !Kref || !kptr || !kidx || !kw || !tw || !out || n_ref < 1)
    return fail(ctx, STV_EINVAL, "NULL argument or n_ref < 1");
  const DevLevel& L = ctx->lv[level];
  const int nls = L.n_ls;
  if (kptr[0] != 0) return fail(ctx, STV_EINVAL, "kptr[0] must be 0");
  for (int32_t c = 0; c < L.n_cells; ++c)
    if (kptr[c + 1] < kptr[c]) return fail(ctx, STV_EINVAL, "kptr must be non-decreasing");
  const int32_t ne = kptr[L.n_cells];
  for (int32_t e = 0; e < ne; ++e)
    if (kidx[e] < 0 || kidx[e] >= n_ref) return fail(ctx, STV_EINVAL, "kidx out of range");
  double *dK = nullptr, *dw = nullptr, *dtw = nullptr;
  int32_t *dp = nullptr, *di = nullptr;
  auto cleanup = [&]() { dfree(dK); dfree(dw); dfree(dtw); dfree(dp); dfree(di); };
  int rc = upload(ctx, &dK, Kref, (size_t)n_ref * nls * nls);
  if (rc == STV_OK) rc = upload(ctx, &dp, kptr, (size_t)L.n_cells + 1);
  if (rc == STV_OK) rc = upload(ctx, &di, kidx, (size_t)std::max(ne, 1));
  if (rc == STV_OK) rc = upload(ctx, &dw, kw, (size_t)std::max(ne, 1));
  if (rc == STV_OK) rc = upload(ctx, &dtw, tw, (size_t)ctx->b);
  if (rc != STV_OK) { cleanup(); return rc; }
  hipError_t e = launch_cell_contract(ctx->stream, ctx->b, L, lam, x, dK, dp, di, dw, dtw, 1.0,
                                      nullptr, nullptr, 0.0, out);
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  cleanup();
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(ctx, STV_EHIP, std::string("cell contraction failed: ") + hipGetErrorString(e));
  return STV_OK;
}

int stv_cell_gradient(stv_ctx* ctx, int level, const double* lam, const double* x, int n_ref,
                      const double* Kref, const int32_t* kptr, const int32_t* kidx,
                      const double* kw, const double* tw, double sc, int n,
                      const int32_t* cells, const double* f, double sf, double* out) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels || ctx->lv[level].n_cells == 0)
    return fail(ctx, STV_EINVAL, "level out of range or without smoothed cells");
  if (!lam || !x || !Kref || !kptr || !kidx || !kw || !tw || !out || n_ref < 1)
    return fail(ctx, STV_EINVAL, "NULL argument or n_ref < 1");
  if (n < 0 || (n > 0 && (!cells || !f))) return fail(ctx, STV_EINVAL, "bad cell list");
  if (!std::isfinite(sc) || !std::isfinite(sf)) return fail(ctx, STV_EINVAL, "sc and sf must be finite");
  const DevLevel& L = ctx->lv[level];
  const int nls = L.n_ls, N = nls * ctx->b;
  if (kptr[0] != 0) return fail(ctx, STV_EINVAL, "kptr[0] must be 0");
  for (int32_t c = 0; c < L.n_cells; ++c)
    if (kptr[c + 1] < kptr[c]) return fail(ctx, STV_EINVAL, "kptr must be non-decreasing");
  const int32_t ne = kptr[L.n_cells];
  for (int32_t e = 0; e < ne; ++e)
    if (kidx[e] < 0 || kidx[e] >= n_ref) return fail(ctx, STV_EINVAL, "kidx out of range");
  // the row of f that belongs to each cell (-1: none)
  std::vector<int32_t> fidx((size_t)L.n_cells, -1);
  for (int k = 0; k < n; ++k) {
    if (cells[k] < 0 || cells[k] >= L.n_cells) return fail(ctx, STV_EINVAL, "cell out of range");
    if (fidx[(size_t)cells[k]] >= 0) return fail(ctx, STV_EINVAL, "cells must be distinct");
    fidx[(size_t)cells[k]] = k;
  }
  double *dK = nullptr, *dw = nullptr, *dtw = nullptr, *df = nullptr;
  int32_t *dp = nullptr, *di = nullptr, *dfi = nullptr;
  auto cleanup = [&]() {
    dfree(dK); dfree(dw); dfree(dtw); dfree(dp); dfree(di); dfree(df); dfree(dfi);
  };
  int rc = upload(ctx, &dK, Kref, (size_t)n_ref * nls * nls);
  if (rc == STV_OK) rc = upload(ctx, &dp, kptr, (size_t)L.n_cells + 1);
  if (rc == STV_OK) rc = upload(ctx, &di, kidx, (size_t)std::max(ne, 1));
  if (rc == STV_OK) rc = upload(ctx, &dw, kw, (size_t)std::max(ne, 1));
  if (rc == STV_OK) rc = upload(ctx, &dtw, tw, (size_t)ctx->b);
  if (rc == STV_OK) rc = upload(ctx, &dfi, fidx.data(), fidx.size());
  if (rc == STV_OK && n > 0) rc = upload(ctx, &df, f, (size_t)n * N);
  if (rc != STV_OK) { cleanup(); return rc; }
  hipError_t e = launch_cell_contract(ctx->stream, ctx->b, L, lam, x, dK, dp, di, dw, dtw, sc,
                                      dfi, df, sf, out);
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  cleanup();
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(ctx, STV_EHIP, std::string("cell gradient failed: ") + hipGetErrorString(e));
  return STV_OK;
}

int stv_cell_scatter(stv_ctx* ctx, int level, int n, const int32_t* cells, const double* coef,
                     const double* f, double* y) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels || ctx->lv[level].n_cells == 0)
    return fail(ctx, STV_EINVAL, "level out of range or without smoothed cells");
  if (n < 0 || !y || (n > 0 && (!cells || !coef || !f))) return fail(ctx, STV_EINVAL, "bad arguments");
  if (n == 0) return STV_OK;
  const DevLevel& L = ctx->lv[level];
  const int b = ctx->b, nls = L.n_ls, N = nls * b;
  for (int k = 0; k < n; ++k)
    if (cells[k] < 0 || cells[k] >= L.n_cells) return fail(ctx, STV_EINVAL, "cell out of range");
  // (global DoF, list position k, entry of f) for every term, grouped by DoF
  // in the order of the list
  std::vector<std::pair<int64_t, int64_t>> terms;   // (global DoF, k * N + j)
  terms.reserve((size_t)n * N);
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < N; ++j) {
      const int a = j / b, l = j - a * b;
      const int64_t g = (int64_t)L.h_csd[(size_t)cells[k] * nls + a] * b + l;
      terms.emplace_back(g, (int64_t)k * N + j);
    }
  std::stable_sort(terms.begin(), terms.end(),
                   [](const auto& u, const auto& v) { return u.first < v.first; });
  std::vector<int64_t> dof, fi;
  std::vector<int32_t> ptr(1, 0), ck;
  for (size_t t = 0; t < terms.size(); ++t) {
    if (t == 0 || terms[t].first != terms[t - 1].first) {
      if (t) ptr.push_back((int32_t)fi.size());
      dof.push_back(terms[t].first);
    }
    fi.push_back(terms[t].second);
    ck.push_back((int32_t)(terms[t].second / N));
  }
  ptr.push_back((int32_t)fi.size());
  double *dc = nullptr, *df = nullptr;
  int64_t *dd = nullptr, *dfi = nullptr;
  int32_t *dp = nullptr, *dk = nullptr;
  auto cleanup = [&]() { dfree(dc); dfree(df); dfree(dd); dfree(dfi); dfree(dp); dfree(dk); };
  int rc = upload(ctx, &dc, coef, (size_t)n);
  if (rc == STV_OK) rc = upload(ctx, &df, f, (size_t)n * N);
  if (rc == STV_OK) rc = upload(ctx, &dd, dof.data(), dof.size());
  if (rc == STV_OK) rc = upload(ctx, &dfi, fi.data(), fi.size());
  if (rc == STV_OK) rc = upload(ctx, &dp, ptr.data(), ptr.size());
  if (rc == STV_OK) rc = upload(ctx, &dk, ck.data(), ck.size());
  if (rc != STV_OK) { cleanup(); return rc; }
  hipError_t e = launch_cell_scatter(ctx->stream, dd, dp, dk, dfi, dc, df, (int)dof.size(), y);
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  cleanup();
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(ctx, STV_EHIP, std::string("cell scatter failed: ") + hipGetErrorString(e));
  return STV_OK;
}

int stv_cell_dot(stv_ctx* ctx, int level, const double* lam, int n, const int32_t* cells,
                 const double* f, double* out) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels || ctx->lv[level].n_cells == 0)
    return fail(ctx, STV_EINVAL, "level out of range or without smoothed cells");
  if (n < 0 || (n > 0 && (!lam || !cells || !f || !out))) return fail(ctx, STV_EINVAL, "bad arguments");
  if (n == 0) return STV_OK;
  const DevLevel& L = ctx->lv[level];
  for (int k = 0; k < n; ++k)
    if (cells[k] < 0 || cells[k] >= L.n_cells) return fail(ctx, STV_EINVAL, "cell out of range");
  int32_t* dc = nullptr;
  double* df = nullptr;
  int rc = upload(ctx, &dc, cells, (size_t)n);
  if (rc == STV_OK) rc = upload(ctx, &df, f, (size_t)n * L.n_ls * ctx->b);
  if (rc != STV_OK) { dfree(dc); dfree(df); return rc; }
  hipError_t e = launch_cell_dot(ctx->stream, ctx->b, L, lam, dc, n, df, out);
  const hipError_t es = hipStreamSynchronize(ctx->stream);
  dfree(dc);
  dfree(df);
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(ctx, STV_EHIP, std::string("cell dot failed: ") + hipGetErrorString(e));
  return STV_OK;
}

int stv_dot(stv_ctx* ctx, const double* a, const double* bv, double* out) {
  STV_TRY(check_ctx(ctx, true, false));
  if (!a || !bv || !out) return fail(ctx, STV_EINVAL, "NULL argument");
  STV_TRY(ensure_workspace(ctx, 1));
  std::vector<double> v;
  STV_TRY(dots_to_host(ctx, a, bv, ctx->ws_n, v));
  for (int z = 0; z < ctx->n_inst; ++z) out[z] = v[(size_t)z];
  return STV_OK;
}

int stv_get_cell_inverse(stv_ctx* ctx, int level, int cell, double* out) {
  STV_TRY(check_ctx(ctx, true, true));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level must be in [1, n_levels)");
  DevLevel& L = ctx->lv[level];
  if (cell < 0 || cell >= L.n_cells) return fail(ctx, STV_EINVAL, "cell out of range");
  if (!out) return fail(ctx, STV_EINVAL, "out is NULL");
  const int b = ctx->b, nls = L.n_ls, n = nls * b;
  const int o0 = L.h_own_ptr[(size_t)cell], no = L.h_own_ptr[(size_t)cell + 1] - o0;
  const int R = ctx->inv_full ? n : L.dec ? no : no * b;
  const int ld = L.inv_ld;
  std::vector<int64_t> off(1);
  STV_HIP(hipMemcpy(off.data(), L.inv_off + cell, sizeof(int64_t), hipMemcpyDeviceToHost));
  std::vector<double> blk((size_t)R * ld);
  if (ctx->inv_fp32) {
    std::vector<float> f((size_t)R * ld);
    STV_HIP(hipMemcpy(f.data(), (const float*)L.inv_store + off[0], sizeof(float) * f.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < f.size(); ++i) blk[i] = f[i];
  } else {
    STV_HIP(hipMemcpy(blk.data(), (const double*)L.inv_store + off[0], sizeof(double) * blk.size(), hipMemcpyDeviceToHost));
  }
  for (int64_t e = 0; e < (int64_t)n * n; ++e) out[e] = NAN;
  if (L.dec) {
    // J_T^-1[(alpha, i), (beta, l)] = sum_{a, c} V[i][a] Q^-1[(alpha, a), (beta, c)] W[c][l]
    // with Q^-1 from the stored time-decoupled row of alpha
    const CellSplit& S = L.split;
    std::vector<double> q((size_t)b * b);
    for (int os = 0; os < no; ++os) {
      const int alpha = L.h_own_loc[(size_t)(o0 + os)];
      const double* row = &blk[(size_t)os * ld];
      for (int beta = 0; beta < nls; ++beta) {
        std::fill(q.begin(), q.end(), 0.0);   // Q^-1[(alpha, a), (beta, c)]
        for (int p = 0; p < S.nblk; ++p) {
          const int f = S.first[p];
          const double re = row[S.off[p] + beta];
          if (S.sz[p] == 1) {
            q[(size_t)f * b + f] = re;
          } else {
            const double im = row[S.off[p] + nls + beta];
            q[(size_t)f * b + f] = re;
            q[(size_t)f * b + f + 1] = -im;
            q[(size_t)(f + 1) * b + f] = im;
            q[(size_t)(f + 1) * b + f + 1] = re;
          }
        }
        for (int i = 0; i < b; ++i)
          for (int l = 0; l < b; ++l) {
            double acc = 0.0;
            for (int a = 0; a < b; ++a)
              for (int c = 0; c < b; ++c) acc += S.V[i * b + a] * q[(size_t)a * b + c] * S.W[c * b + l];
            out[(int64_t)(i * nls + alpha) * n + l * nls + beta] = acc;   // eq. (4.4) order
          }
      }
    }
    return STV_OK;
  }
  // stored row index -> internal local index (alpha*b + l)
  for (int o = 0; o < R; ++o) {
    int alpha, l;
    if (ctx->inv_full) { alpha = o / b; l = o % b; }
    else { alpha = L.h_own_loc[(size_t)(o0 + o / b)]; l = o % b; }
    const int row = l * nls + alpha;   // eq. (4.4) order
    for (int j = 0; j < n; ++j) {
      const int beta = j / b, lj = j % b;
      out[(int64_t)row * n + lj * nls + beta] = blk[(size_t)o * ld + j];   // stored row-major
    }
  }
  return STV_OK;
}

int stv_level_info(stv_ctx* ctx, int level, int64_t* n_sdofs, int64_t* n_cells, int64_t* n_loc,
                   int64_t* inverse_bytes) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level out of range");
  const DevLevel& L = ctx->lv[level];
  if (n_sdofs) *n_sdofs = L.n_s;
  if (n_cells) *n_cells = L.n_cells_all;
  if (n_loc) *n_loc = (int64_t)L.n_ls * ctx->b;
  if (inverse_bytes) *inverse_bytes = L.inv_elems * (ctx->inv_fp32 ? 4 : 8);
  return STV_OK;
}

int stv_instance_layout(stv_ctx* ctx, int inst, int* n_levels, int64_t* row_offset,
                        int64_t* n_rows) {
  STV_TRY(check_ctx(ctx, true, false));
  if (inst < 0 || inst >= ctx->n_inst) return fail(ctx, STV_EINVAL, "instance out of range");
  if (n_levels) *n_levels = ctx->inst_levels[(size_t)inst];
  if (row_offset) *row_offset = ctx->inst_row[(size_t)inst];
  if (n_rows) *n_rows = ctx->inst_row[(size_t)inst + 1] - ctx->inst_row[(size_t)inst];
  return STV_OK;
}

int stv_instance_info(stv_ctx* ctx, int inst, stv_gmres_info* info) {
  STV_TRY(check_ctx(ctx, true, false));
  if (inst < 0 || inst >= ctx->n_inst) return fail(ctx, STV_EINVAL, "instance out of range");
  if (!info) return fail(ctx, STV_EINVAL, "info is NULL");
  const InstInfo& o = ctx->inst_info[(size_t)inst];
  info->iters = o.iters;
  info->restarts = o.restarts;
  info->converged = o.converged;
  info->true_relres = o.relres;
  info->history_len = 0;
  return STV_OK;
}

int stv_set_launch(stv_ctx* ctx, int level, int spmv_rows, int sweep_wgs) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level out of range");
  if (spmv_rows < 1 || spmv_rows > 12) return fail(ctx, STV_EINVAL, "spmv_rows must be in [1, 12]");
  if (sweep_wgs < 0) return fail(ctx, STV_EINVAL, "sweep_wgs must be >= 0");
  STV_HIP(hipStreamSynchronize(ctx->stream));
  ctx->lv[level].spmv_rpw = spmv_rows;
  ctx->lv[level].sweep_wgs = sweep_wgs;
  ++ctx->generation;   // a captured V-cycle holds the old launch shapes
  free_graph(ctx);
  return STV_OK;
}

int stv_transfer_shapes(stv_ctx* ctx, int level, int p_shape, int pt_shape, int* cur_p,
                        int* cur_pt) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level out of range");
  if (p_shape < 0 || p_shape > kTransferShapes || pt_shape < 0 || pt_shape > kTransferShapes)
    return fail(ctx, STV_EINVAL, "transfer shapes must be in [0, 5]");
  DevLevel& L = ctx->lv[level];
  if (p_shape > 0 || pt_shape > 0) {
    STV_HIP(hipStreamSynchronize(ctx->stream));
    if (p_shape > 0) L.p_shape = p_shape;
    if (pt_shape > 0) L.pt_shape = pt_shape;
    ++ctx->generation;   // a captured V-cycle holds the old launch shapes
    free_graph(ctx);
  }
  if (cur_p) *cur_p = L.p_shape;
  if (cur_pt) *cur_pt = L.pt_shape;
  return STV_OK;
}

int stv_autotune(stv_ctx* ctx, int* choices, int cap) {
  STV_TRY(check_ctx(ctx, true, true));
  const int b = ctx->b;
  hipStream_t s = ctx->stream;
  int64_t nmax = 0;
  for (int g = 0; g < ctx->n_levels; ++g) nmax = std::max<int64_t>(nmax, (int64_t)ctx->lv[g].n_s * b);
  double *x = nullptr, *r = nullptr, *y = nullptr;
  auto cleanup = [&]() { dfree(x); dfree(r); dfree(y); };
  if (dalloc(ctx, &x, (size_t)nmax) != STV_OK || dalloc(ctx, &r, (size_t)nmax) != STV_OK ||
      dalloc(ctx, &y, (size_t)nmax) != STV_OK) {
    cleanup();
    return STV_ENOMEM;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch_fill(s, x, nmax, 1.0);
  if (e == hipSuccess) e = launch_fill(s, r, nmax, 0.5);
  // average milliseconds of reps launches of f after one untimed launch
  auto time_it = [&](auto&& f, double& ms) -> hipError_t {
    const int reps = 5;
    hipError_t er = f();
    if (er == hipSuccess) er = hipEventRecord(e0, s);
    for (int i = 0; i < reps && er == hipSuccess; ++i) er = f();
    if (er == hipSuccess) er = hipEventRecord(e1, s);
    if (er == hipSuccess) er = hipEventSynchronize(e1);
    float t = 0.f;
    if (er == hipSuccess) er = hipEventElapsedTime(&t, e0, e1);
    ms = t / reps;
    return er;
  };
  for (int g = 1; g < ctx->n_levels && e == hipSuccess; ++g) {
    DevLevel& L = ctx->lv[g];
    if (L.n_cells == 0) continue;
    int best_r = L.spmv_rpw;
    double best = 1e30;
    for (int rpw = 1; rpw <= residual_shapes(L) && e == hipSuccess; ++rpw) {
      L.spmv_rpw = rpw;
      double ms = 0;
      e = time_it([&]() {
        return L.kron_ma ? launch_spmv_kron(s, b, L, r, x, y, -1.0)
                        : launch_spmv(s, b, L, r, x, y, -1.0);
      }, ms);
      if (ms < best) { best = ms; best_r = rpw; }
    }
    L.spmv_rpw = best_r;
    int best_w = 0;
    best = 1e30;
    int cu = 256;
    (void)hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, ctx->device);
    const int full_grid = (L.n_cells + 3) / 4;
    const int cand[6] = {0, 2 * cu, 4 * cu, 8 * cu, 16 * cu, 32 * cu};
    for (int c = 0; c < 6 && e == hipSuccess; ++c) {
      if (c > 0 && cand[c] >= full_grid) break;
      L.sweep_wgs = cand[c];
      double ms = 0;
      e = time_it([&]() {
        return launch_vanka_cells(s, b, L, x, y, 0.7, 0, ctx->inv_fp32, ctx->inv_full);
      }, ms);
      if (ms < best) { best = ms; best_w = cand[c]; }
    }
    L.sweep_wgs = best_w;
  }
  // transfer shapes of every level with a prolongation, each direction alone
  for (int g = 1; g < ctx->n_levels && e == hipSuccess; ++g) {
    DevLevel& L = ctx->lv[g];
    if (!L.P_rowptr) continue;
    for (int dir = 0; dir < 2 && e == hipSuccess; ++dir) {
      int& shape = dir ? L.pt_shape : L.p_shape;
      int best_t = shape;
      double best = 1e30;
      for (int t = 1; t <= kTransferShapes && e == hipSuccess; ++t) {
        shape = t;
        double ms = 0;
        e = time_it([&]() {
          return dir ? launch_restrict(s, b, L, x, y) : launch_prolongate_add(s, b, L, x, y);
        }, ms);
        if (ms < best) { best = ms; best_t = t; }
      }
      shape = best_t;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const hipError_t es = hipStreamSynchronize(s);
  cleanup();
  if (e == hipSuccess) e = es;
  if (e != hipSuccess) return fail(ctx, STV_EHIP, std::string("autotune failed: ") + hipGetErrorString(e));
  ++ctx->generation;
  free_graph(ctx);
  if (choices)
    for (int g = 0; g < ctx->n_levels && 2 * g + 1 < cap; ++g) {
      choices[2 * g] = ctx->lv[g].spmv_rpw;
      choices[2 * g + 1] = ctx->lv[g].sweep_wgs;
    }
  return STV_OK;
}

int stv_set_kron_factors(stv_ctx* ctx, int level, const double* mval, const double* aval,
                         const double* C, const double* tw) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 0 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level out of range");
  DevLevel& L = ctx->lv[level];
  if (!mval && !aval) {   // drop the factors: back to the stored blocks
    STV_HIP(hipStreamSynchronize(ctx->stream));
    dfree(L.kron_ma); dfree(L.kx_ptr); dfree(L.kx_col); dfree(L.kx_val);
    L.kx_n1 = 0;
    ctx->cgroups_algo = -1;   // the coarse groups may refer to the factors
    ctx->inv_layout = -1;     // and the cell-inverse layout of the level
    ++ctx->generation;
    free_graph(ctx);
    return STV_OK;
  }
  if (!mval || !aval || !C || !tw) return fail(ctx, STV_EINVAL, "NULL argument");
  const int b = ctx->b;
  for (int e = 0; e < b * b; ++e)
    if (!std::isfinite(C[e])) return fail(ctx, STV_EINVAL, "C must be finite");
  for (int e = 0; e < b; ++e)
    if (!std::isfinite(tw[e])) return fail(ctx, STV_EINVAL, "tw must be finite");
  STV_HIP(hipStreamSynchronize(ctx->stream));
  double *dma = nullptr, *part = nullptr;
  const int nblk = 1024;
  auto drop = [&]() { dfree(dma); dfree(part); };
  std::vector<double> hma((size_t)2 * L.nnzb);
  for (int64_t q = 0; q < L.nnzb; ++q) {
    hma[(size_t)(2 * q)] = mval[q];
    hma[(size_t)(2 * q + 1)] = aval[q];
  }
  int rc = upload(ctx, &dma, hma.data(), hma.size());
  if (rc == STV_OK) rc = dalloc(ctx, &part, (size_t)2 * nblk);
  if (rc != STV_OK) { drop(); return rc; }
  // the factors must reproduce the stored blocks
  std::vector<double> hp((size_t)2 * nblk);
  hipError_t e = launch_kron_check(ctx->stream, b, L, dma, C, tw, part, nblk);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), part, sizeof(double) * hp.size(),
                                          hipMemcpyDeviceToHost, ctx->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
  dfree(part);
  if (e != hipSuccess) {
    drop();
    return fail(ctx, STV_EHIP, std::string("factor check failed: ") + hipGetErrorString(e));
  }
  double dev = 0.0, mag = 0.0;
  for (int i = 0; i < nblk; ++i) {
    dev = std::max(dev, hp[(size_t)2 * i]);
    mag = std::max(mag, hp[(size_t)2 * i + 1]);
  }
  if (!(dev <= 1e-12 * mag)) {
    drop();
    return fail(ctx, STV_EINVAL, "the factors do not reproduce the level's blocks (max deviation " +
                                     std::to_string(dev) + " of " + std::to_string(mag) + ")");
  }
  // the residual's split lists: per row the blocks with m != 0, then the
  // others (row order kept within each list)
  const int64_t ns = L.n_s;
  std::vector<int32_t> hrp((size_t)ns + 1), hcol((size_t)L.nnzb);
  e = hipMemcpy(hrp.data(), L.rowptr, sizeof(int32_t) * hrp.size(), hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(hcol.data(), L.col, sizeof(int32_t) * hcol.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    drop();
    return fail(ctx, STV_EHIP, std::string("reading the level pattern failed: ") + hipGetErrorString(e));
  }
  std::vector<int32_t> xptr((size_t)(2 * (ns + 1)), 0);
  int64_t n1 = 0;
  for (int64_t q = 0; q < L.nnzb; ++q) n1 += mval[q] != 0.0;
  const int64_t n2 = L.nnzb - n1;
  std::vector<int32_t> xcol((size_t)L.nnzb);
  std::vector<double> xval((size_t)(2 * n1 + n2));
  int64_t p1 = 0, p2 = 0;
  for (int64_t i = 0; i < ns; ++i) {
    xptr[(size_t)i] = (int32_t)p1;
    xptr[(size_t)(ns + 1 + i)] = (int32_t)p2;
    for (int32_t q = hrp[(size_t)i]; q < hrp[(size_t)i + 1]; ++q) {
      if (mval[q] != 0.0) {
        xcol[(size_t)p1] = hcol[(size_t)q];
        xval[(size_t)(2 * p1)] = mval[q];
        xval[(size_t)(2 * p1 + 1)] = aval[q];
        ++p1;
      } else {
        xcol[(size_t)(n1 + p2)] = hcol[(size_t)q];
        xval[(size_t)(2 * n1 + p2)] = aval[q];
        ++p2;
      }
    }
  }
  xptr[(size_t)ns] = (int32_t)p1;
  xptr[(size_t)(2 * ns + 1)] = (int32_t)p2;
  int32_t *dxp = nullptr, *dxc = nullptr;
  double* dxv = nullptr;
  rc = upload(ctx, &dxp, xptr.data(), xptr.size());
  if (rc == STV_OK) rc = upload(ctx, &dxc, xcol.data(), xcol.size());
  if (rc == STV_OK) rc = upload(ctx, &dxv, xval.data(), xval.size());
  if (rc != STV_OK) { drop(); dfree(dxp); dfree(dxc); dfree(dxv); return rc; }
  dfree(L.kron_ma); dfree(L.kx_ptr); dfree(L.kx_col); dfree(L.kx_val);
  L.kron_ma = dma;
  L.kx_ptr = dxp;
  L.kx_col = dxc;
  L.kx_val = dxv;
  L.kx_n1 = n1;
  ctx->cgroups_algo = -1;   // the coarse groups are regrouped at the next build
  ctx->inv_layout = -1;     // the cell inverses may be stored time-decoupled
  for (int i = 0; i < 16; ++i) L.kron_C[i] = i < b * b ? C[i] : 0.0;
  for (int i = 0; i < 4; ++i) L.kron_tw[i] = i < b ? tw[i] : 0.0;
  ++ctx->generation;
  free_graph(ctx);
  return STV_OK;
}

int stv_set_option(stv_ctx* ctx, int option, int64_t value) {
  if (!ctx) return STV_EINVAL;
  switch (option) {
    case STV_OPT_COARSE_ALGO:
      if (value < 0 || value > 3) return fail(ctx, STV_EINVAL, "coarse algorithm must be 0, 1, 2 or 3");
      ctx->coarse_algo = (int)value;
      return STV_OK;
    case STV_OPT_COARSE_OVERLAP:
      if (value < 0 || value > 1) return fail(ctx, STV_EINVAL, "overlap option must be 0 or 1");
      ctx->coarse_overlap = (int)value;
      return STV_OK;
    case STV_OPT_GRAPH:
      if (value < 0 || value > 1) return fail(ctx, STV_EINVAL, "graph option must be 0 or 1");
      ctx->use_graph = (int)value;
      return STV_OK;
    case STV_OPT_COARSE_LOOKAHEAD:
      if (value < 0 || value > 1) return fail(ctx, STV_EINVAL, "look-ahead option must be 0 or 1");
      ctx->coarse_lookahead = (int)value;
      return STV_OK;
    case STV_OPT_INVERSE_CUS:
      if (value < -1 || value > 65536) return fail(ctx, STV_EINVAL, "compute-unit cap must be in [-1, 65536]");
      ctx->inverse_cus = (int)value;
      return STV_OK;
    default:
      return fail(ctx, STV_EINVAL, "unknown option");
  }
}

int stv_set_timing(stv_ctx* ctx, int on) {
  if (!ctx) return STV_EINVAL;
  STV_HIP(hipStreamSynchronize(ctx->stream));
  resolve_timers(ctx);
  ctx->timing = on != 0;
  for (int c = 0; c < KC_COUNT; ++c)
    for (int g = 0; g < kMaxLevels; ++g) { ctx->launches[c][g] = 0; ctx->total_ms[c][g] = 0.0; }
  return STV_OK;
}

int stv_set_timing_filter(stv_ctx* ctx, unsigned class_mask, unsigned level_mask) {
  if (!ctx) return STV_EINVAL;
  if (class_mask >> KC_COUNT) return fail(ctx, STV_EINVAL, "unknown kernel class in the mask");
  STV_HIP(hipStreamSynchronize(ctx->stream));
  resolve_timers(ctx);
  ctx->timing_mask = class_mask;
  ctx->timing_levels = level_mask;
  return STV_OK;
}

int stv_kernel_stats(stv_ctx* ctx, int kernel_class, int level, int64_t* launches,
                     double* total_ms) {
  if (!ctx) return STV_EINVAL;
  if (kernel_class < 0 || kernel_class >= KC_COUNT) return fail(ctx, STV_EINVAL, "unknown kernel class");
  if (level < -1 || level >= kMaxLevels) return fail(ctx, STV_EINVAL, "level out of range");
  STV_HIP(hipStreamSynchronize(ctx->stream));
  resolve_timers(ctx);
  int64_t n = 0;
  double ms = 0.0;
  for (int g = 0; g < kMaxLevels; ++g)
    if (level < 0 || g == level) {
      n += ctx->launches[kernel_class][g];
      ms += ctx->total_ms[kernel_class][g];
    }
  if (launches) *launches = n;
  if (total_ms) *total_ms = ms;
  return STV_OK;
}

}  // extern "C"
