// Host side of the space-time Vanka multigrid library: argument validation,
// hierarchy upload (owned-DoF lists, transposed prolongations), the inverse
// build, the smoother / V-cycle orchestration (Algorithm 4.1) and the flexible
// GMRES driver.  Every arithmetic step on vectors and matrices runs in the
// HIP kernels; the host only does index bookkeeping, the (k+1)-sized Givens
// and triangular solves of GMRES, and control flow.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "stv_internal.h"

using namespace stv;

namespace {

std::string g_create_err;

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

void free_inverses(stv_ctx* ctx) {
  for (int g = 0; g < kMaxLevels; ++g) {
    dfree(ctx->lv[g].inv_off);
    dfree(ctx->lv[g].inv_store);
    ctx->lv[g].inv_elems = 0;
  }
  dfree(ctx->coarse_inv);
  ctx->have_inv = false;
}

void free_level(DevLevel& L) {
  dfree(L.rowptr); dfree(L.col); dfree(L.val); dfree(L.cell_sdofs);
  dfree(L.own_ptr); dfree(L.own_loc); dfree(L.inc_ptr); dfree(L.inc_cell); dfree(L.inc_loc);
  dfree(L.P_rowptr); dfree(L.P_col); dfree(L.P_val);
  dfree(L.Pt_rowptr); dfree(L.Pt_col); dfree(L.Pt_val);
  dfree(L.inv_off); dfree(L.inv_store); dfree(L.posmap);
  dfree(L.rho); dfree(L.r); dfree(L.d); dfree(L.corr);
  L = DevLevel();
}

void free_workspace(stv_ctx* ctx) {
  dfree(ctx->V); dfree(ctx->Z); dfree(ctx->w); dfree(ctx->rt); dfree(ctx->partial);
  ctx->ws_restart = 0;
  ctx->ws_n = 0;
}

void free_hierarchy(stv_ctx* ctx) {
  free_inverses(ctx);
  for (int g = 0; g < kMaxLevels; ++g) free_level(ctx->lv[g]);
  free_workspace(ctx);
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

struct Timed {
  stv_ctx* ctx;
  int cls;
  int level;
  hipStream_t st;
  hipEvent_t a = nullptr;
  Timed(stv_ctx* c, int k, int g = 0, hipStream_t on = nullptr)
      : ctx(c), cls(k), level(g), st(on ? on : c->stream) {
    if (ctx->timing) {
      a = get_event(ctx);
      (void)hipEventRecord(a, st);
    }
  }
  void done() {
    if (ctx->timing && a) {
      hipEvent_t b = get_event(ctx);
      (void)hipEventRecord(b, st);
      ctx->pending.push_back({a, b, cls, level});
      a = nullptr;
    }
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
int residual(stv_ctx* ctx, int g, const double* r, const double* x, double* y) {
  Timed t(ctx, KC_RESIDUAL, g);
  STV_HIP(launch_spmv(ctx->stream, ctx->b, ctx->lv[g], r, x, y, -1.0));
  t.done();
  return STV_OK;
}

int matvec(stv_ctx* ctx, int g, const double* x, double* y) {
  Timed t(ctx, KC_RESIDUAL, g);
  STV_HIP(launch_spmv(ctx->stream, ctx->b, ctx->lv[g], nullptr, x, y, 1.0));
  t.done();
  return STV_OK;
}

int cell_pass(stv_ctx* ctx, int g, const double* rho, double* d, double omega, int zero_init,
              int mode) {
  DevLevel& L = ctx->lv[g];
  const int b = ctx->b;
  if (mode == STV_LAST_WRITER) {
    Timed t(ctx, KC_SWEEP, g);
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

int coarse_apply(stv_ctx* ctx, const double* r, double* d) {
  Timed t(ctx, KC_COARSE);
  STV_HIP(launch_dense_gemv(ctx->stream, ctx->coarse_inv, ctx->n0, r, d));
  t.done();
  return STV_OK;
}

int vcycle_level(stv_ctx* ctx, int g, const double* r, double* d, const stv_mg_params& p) {
  if (g == 0) return coarse_apply(ctx, r, d);
  DevLevel& L = ctx->lv[g];
  DevLevel& C = ctx->lv[g - 1];
  const int b = ctx->b;
  if (p.nu1 == 0) STV_HIP(launch_fill(ctx->stream, d, (int64_t)L.n_s * b, 0.0));
  STV_TRY(sweeps(ctx, g, r, d, p.nu1, p.omega, p.mode, true));
  STV_TRY(residual(ctx, g, r, d, L.rho));
  {
    Timed t(ctx, KC_TRANSFER, g);
    STV_HIP(launch_restrict(ctx->stream, b, L, L.rho, C.r));
    t.done();
  }
  STV_TRY(vcycle_level(ctx, g - 1, C.r, C.d, p));
  {
    Timed t(ctx, KC_TRANSFER, g);
    STV_HIP(launch_prolongate_add(ctx->stream, b, L, C.d, d));
    t.done();
  }
  STV_TRY(sweeps(ctx, g, r, d, p.nu2, p.omega, p.mode, false));
  return STV_OK;
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
  STV_TRY(dalloc(ctx, &ctx->V, (size_t)(m + 1) * n));
  STV_TRY(dalloc(ctx, &ctx->Z, (size_t)m * n));
  STV_TRY(dalloc(ctx, &ctx->w, (size_t)n));
  STV_TRY(dalloc(ctx, &ctx->rt, (size_t)n));
  STV_TRY(dalloc(ctx, &ctx->partial, (size_t)kDotBlocks * 8));
  ctx->ws_restart = m;
  ctx->ws_n = n;
  return STV_OK;
}

// scal layout (device and pinned host mirror):
//   [0, R)        h1 (first Gram-Schmidt pass)
//   [R, 2R)       h2 (second pass)
//   [2R]          ||w||^2
//   [2R+1]        scratch norm^2
//   [3R, 4R)      y (host -> device)
constexpr int kScalR = kMaxRestart + 2;

int dot_to_host(stv_ctx* ctx, const double* a, const double* b, int64_t n, double* out) {
  Timed t(ctx, KC_KRYLOV);
  STV_HIP(launch_multidot(ctx->stream, a, 1, b, n, ctx->partial, ctx->scal + 2 * kScalR + 1));
  t.done();
  STV_HIP(hipMemcpyAsync(ctx->hscal + 2 * kScalR + 1, ctx->scal + 2 * kScalR + 1, sizeof(double),
                         hipMemcpyDeviceToHost, ctx->stream));
  STV_HIP(hipStreamSynchronize(ctx->stream));
  *out = ctx->hscal[2 * kScalR + 1];
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
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess) {
    g_create_err = "creation of the internal stream/events failed";
    delete ctx;
    return STV_EHIP;
  }
  if (hipMalloc((void**)&ctx->scal, sizeof(double) * 4 * kScalR) != hipSuccess ||
      hipHostMalloc((void**)&ctx->hscal, sizeof(double) * 4 * kScalR, hipHostMallocDefault) !=
          hipSuccess) {
    g_create_err = "allocation of the scalar buffers failed";
    if (ctx->scal) (void)hipFree(ctx->scal);
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
  for (auto& t : ctx->pending) { (void)hipEventDestroy(t.a); (void)hipEventDestroy(t.b); }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->side) {
    (void)hipStreamSynchronize(ctx->side);
    (void)hipStreamDestroy(ctx->side);
  }
  if (ctx->ev_fork) (void)hipEventDestroy(ctx->ev_fork);
  if (ctx->ev_join) (void)hipEventDestroy(ctx->ev_join);
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
  std::string msg;
  if (!validate_impl(n_levels, dim, k, lv, msg)) return fail(ctx, STV_EINVAL, msg);
  STV_HIP(hipSetDevice(ctx->device));
  STV_HIP(hipStreamSynchronize(ctx->stream));
  free_hierarchy(ctx);
  ctx->n_levels = n_levels;
  ctx->dim = dim;
  ctx->k = k;
  ctx->b = k + 1;
  const int b = ctx->b;
  for (int g = 0; g < n_levels; ++g) {
    const stv_level& H = lv[g];
    DevLevel& L = ctx->lv[g];
    L.n_s = H.n_sdofs;
    L.n_cells = H.n_cells;
    L.n_ls = H.n_ls;
    L.nnzb = H.nnzb;
    const int nls = H.n_ls;
    STV_TRY(upload(ctx, &L.rowptr, H.bsr_rowptr, (size_t)H.n_sdofs + 1));
    STV_TRY(upload(ctx, &L.col, H.bsr_col, (size_t)H.nnzb));
    STV_TRY(upload(ctx, &L.val, H.bsr_val, (size_t)H.nnzb * b * b));
    STV_TRY(upload(ctx, &L.cell_sdofs, H.cell_sdofs, (size_t)H.n_cells * nls));
    // owner of each spatial DoF: the last cell in loop order containing it
    std::vector<int32_t> owner((size_t)H.n_sdofs, -1);
    for (int32_t c = 0; c < H.n_cells; ++c)
      for (int a = 0; a < nls; ++a) owner[(size_t)H.cell_sdofs[(int64_t)c * nls + a]] = c;
    L.h_own_ptr.assign((size_t)H.n_cells + 1, 0);
    L.h_own_loc.clear();
    for (int32_t c = 0; c < H.n_cells; ++c) {
      for (int a = 0; a < nls; ++a)
        if (owner[(size_t)H.cell_sdofs[(int64_t)c * nls + a]] == c) L.h_own_loc.push_back((uint8_t)a);
      L.h_own_ptr[(size_t)c + 1] = (int32_t)L.h_own_loc.size();
    }
    STV_TRY(upload(ctx, &L.own_ptr, L.h_own_ptr.data(), L.h_own_ptr.size()));
    STV_TRY(upload(ctx, &L.own_loc, L.h_own_loc.data(), L.h_own_loc.size()));
    // incidence DoF -> (cell, local index), cells in loop order
    {
      std::vector<int32_t> ip((size_t)H.n_sdofs + 1, 0);
      for (int64_t e = 0; e < (int64_t)H.n_cells * nls; ++e) ip[(size_t)H.cell_sdofs[e] + 1]++;
      for (int32_t s = 0; s < H.n_sdofs; ++s) ip[(size_t)s + 1] += ip[(size_t)s];
      std::vector<int32_t> fillp(ip.begin(), ip.end() - 1);
      std::vector<int32_t> icell((size_t)ip.back());
      std::vector<uint8_t> iloc((size_t)ip.back());
      for (int32_t c = 0; c < H.n_cells; ++c)
        for (int a = 0; a < nls; ++a) {
          const int32_t s = H.cell_sdofs[(int64_t)c * nls + a];
          icell[(size_t)fillp[(size_t)s]] = c;
          iloc[(size_t)fillp[(size_t)s]++] = (uint8_t)a;
        }
      STV_TRY(upload(ctx, &L.inc_ptr, ip.data(), ip.size()));
      STV_TRY(upload(ctx, &L.inc_cell, icell.data(), icell.size()));
      STV_TRY(upload(ctx, &L.inc_loc, iloc.data(), iloc.size()));
    }
    if (g > 0) {
      STV_TRY(dalloc(ctx, &L.posmap, (size_t)H.n_cells * nls * nls));
      STV_HIP(launch_build_posmap(ctx->stream, L));
    }
    const size_t nst = (size_t)H.n_sdofs * b;
    STV_TRY(dalloc(ctx, &L.rho, nst));
    if (g < n_levels - 1) {
      STV_TRY(dalloc(ctx, &L.r, nst));
      STV_TRY(dalloc(ctx, &L.d, nst));
    }
    if (g > 0) {
      const int32_t nc = lv[g - 1].n_sdofs;
      L.n_s_coarse = nc;
      STV_TRY(upload(ctx, &L.P_rowptr, H.P_rowptr, (size_t)H.n_sdofs + 1));
      STV_TRY(upload(ctx, &L.P_col, H.P_col, (size_t)H.P_nnz));
      STV_TRY(upload(ctx, &L.P_val, H.P_val, (size_t)H.P_nnz));
      // transpose (coarse rows, fine rows ascending within each)
      std::vector<int32_t> tp((size_t)nc + 1, 0);
      for (int64_t q = 0; q < H.P_nnz; ++q) tp[(size_t)H.P_col[q] + 1]++;
      for (int32_t c = 0; c < nc; ++c) tp[(size_t)c + 1] += tp[(size_t)c];
      std::vector<int32_t> fillp(tp.begin(), tp.end() - 1);
      std::vector<int32_t> tc((size_t)H.P_nnz);
      std::vector<double> tv((size_t)H.P_nnz);
      for (int32_t s = 0; s < H.n_sdofs; ++s)
        for (int32_t q = H.P_rowptr[s]; q < H.P_rowptr[s + 1]; ++q) {
          const int32_t c = H.P_col[q];
          tc[(size_t)fillp[(size_t)c]] = s;
          tv[(size_t)fillp[(size_t)c]++] = H.P_val[q];
        }
      STV_TRY(upload(ctx, &L.Pt_rowptr, tp.data(), tp.size()));
      STV_TRY(upload(ctx, &L.Pt_col, tc.data(), tc.size()));
      STV_TRY(upload(ctx, &L.Pt_val, tv.data(), tv.size()));
    }
  }
  STV_HIP(hipStreamSynchronize(ctx->stream));
  ctx->have_hier = true;
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
  free_inverses(ctx);
  ctx->inv_fp32 = fp32;
  ctx->inv_full = full;
  const int b = ctx->b;
  hipStream_t s = ctx->stream;
  hipStream_t side = ctx->side;
  // ---- allocations (host-side offsets of every cell's stored rows)
  std::vector<uint8_t*> status((size_t)ctx->n_levels, nullptr);
  std::vector<double*> scratch((size_t)ctx->n_levels, nullptr);
  std::vector<int> slots((size_t)ctx->n_levels, 0);
  double *A = nullptr, *Bbuf = nullptr, *pbuf = nullptr, *Sbuf = nullptr, *Bin = nullptr;
  int *piv = nullptr, *rinv_d = nullptr;
  uint8_t* used = nullptr;
  auto cleanup = [&]() {
    for (auto& p : status) dfree(p);
    for (auto& p : scratch) dfree(p);
    dfree(A); dfree(Bbuf); dfree(pbuf); dfree(Sbuf); dfree(Bin); dfree(piv); dfree(rinv_d);
    dfree(used);
  };
  int rc = STV_OK;
  for (int g = 1; g < ctx->n_levels && rc == STV_OK; ++g) {
    DevLevel& L = ctx->lv[g];
    const int n = L.n_ls * b;
    std::vector<int64_t> off((size_t)L.n_cells);
    int64_t tot = 0;
    for (int32_t c = 0; c < L.n_cells; ++c) {
      off[(size_t)c] = tot;
      const int rows = full ? n : (L.h_own_ptr[(size_t)c + 1] - L.h_own_ptr[(size_t)c]) * b;
      tot += (int64_t)rows * n;
    }
    if ((rc = upload(ctx, &L.inv_off, off.data(), off.size())) != STV_OK) break;
    if (fp32) {
      float* p = nullptr;
      rc = dalloc(ctx, &p, (size_t)tot);
      L.inv_store = p;
    } else {
      double* p = nullptr;
      rc = dalloc(ctx, &p, (size_t)tot);
      L.inv_store = p;
    }
    if (rc != STV_OK) break;
    L.inv_elems = tot;
    if ((rc = dalloc(ctx, &status[(size_t)g], (size_t)L.n_cells)) != STV_OK) break;
    if (!inverse_fits_regs(b, L.n_ls)) {
      slots[(size_t)g] = std::min<int>(L.n_cells, 1024);
      rc = dalloc(ctx, &scratch[(size_t)g], (size_t)slots[(size_t)g] * n * n);
    }
  }
  DevLevel& L0 = ctx->lv[0];
  const int64_t n0 = (int64_t)L0.n_s * b;
  const GjPlan plan = gj_plan(n0, ctx->coarse_algo);
  const int64_t np = (n0 + plan.pad - 1) / plan.pad * plan.pad;
  if (rc == STV_OK && np > plan.max_n)
    rc = fail(ctx, STV_EINVAL, "coarse level larger than " + std::to_string(plan.max_n) + " unknowns");
  if (rc == STV_OK) {
    ctx->n0 = n0;
    const int64_t nbo = std::max(plan.nb, plan.no);
    if ((rc = dalloc(ctx, &A, (size_t)(np * np))) == STV_OK &&
        (rc = dalloc(ctx, &ctx->coarse_inv, (size_t)(n0 * n0))) == STV_OK &&
        (rc = dalloc(ctx, &Bbuf, (size_t)(nbo * np))) == STV_OK &&
        (rc = dalloc(ctx, &pbuf, (size_t)(2 * plan.nb * np))) == STV_OK &&
        (plan.no == 0 || (rc = dalloc(ctx, &Sbuf, (size_t)(2 * plan.no * np))) == STV_OK) &&
        (plan.no == 0 || (rc = dalloc(ctx, &Bin, (size_t)(plan.nb * plan.no))) == STV_OK) &&
        (rc = dalloc(ctx, &piv, (size_t)np)) == STV_OK &&
        (rc = dalloc(ctx, &used, (size_t)np)) == STV_OK)
      rc = dalloc(ctx, &rinv_d, (size_t)np);
  }
  if (rc != STV_OK) {
    cleanup();
    free_inverses(ctx);
    return rc;
  }
  // ---- launch: cell inverses on the caller's stream, coarse factorisation
  // on the internal stream (it starts after everything queued before it)
  hipError_t e = hipEventRecord(ctx->ev_fork, s);
  if (e == hipSuccess) e = hipStreamWaitEvent(side, ctx->ev_fork, 0);
  for (int g = 1; g < ctx->n_levels && e == hipSuccess; ++g) {
    Timed t(ctx, KC_INVERSE, g);
    e = launch_cell_inverses(s, b, ctx->lv[g], fp32, full, status[(size_t)g], scratch[(size_t)g],
                             slots[(size_t)g]);
    t.done();
  }
  {
    Timed t(ctx, KC_COARSE_FACTOR, 0, side);
    if (e == hipSuccess) e = launch_fill(side, A, np * np, 0.0);
    if (e == hipSuccess) e = launch_bsr_to_dense(side, b, L0, A, np);
    if (e == hipSuccess) e = launch_set_diag(side, A, np, n0, np);
    if (e == hipSuccess) e = hipMemsetAsync(used, 0, (size_t)np, side);
    if (e == hipSuccess) e = launch_gj(side, plan, A, np, piv, used, Bbuf, pbuf, Sbuf, Bin);
    t.done();
  }
  std::vector<int> hp((size_t)np);
  if (e == hipSuccess) e = hipMemcpyAsync(hp.data(), piv, sizeof(int) * np, hipMemcpyDeviceToHost, side);
  if (e == hipSuccess) e = hipStreamSynchronize(side);
  bool coarse_singular = false;
  std::vector<int> rinv((size_t)np, -1);
  if (e == hipSuccess) {
    for (int64_t p = 0; p < np; ++p) {
      const int r = hp[(size_t)p];
      if (r < 0 || r >= np || rinv[(size_t)r] >= 0) { coarse_singular = true; break; }
      rinv[(size_t)r] = (int)p;
    }
    // the real block must pivot within itself (the padding is an identity)
    for (int64_t p = 0; p < n0 && !coarse_singular; ++p)
      if (hp[(size_t)p] >= n0) coarse_singular = true;
    if (!coarse_singular) {
      Timed t(ctx, KC_COARSE_FACTOR, 0, side);
      e = hipMemcpyAsync(rinv_d, rinv.data(), sizeof(int) * np, hipMemcpyHostToDevice, side);
      if (e == hipSuccess) e = launch_gj_unpermute(side, A, np, ctx->coarse_inv, n0, piv, rinv_d);
      if (e == hipSuccess) e = hipStreamSynchronize(side);   // rinv (host) outlives the copy
      t.done();
    }
  }
  if (e == hipSuccess) e = hipEventRecord(ctx->ev_join, side);
  if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->ev_join, 0);
  std::vector<std::vector<uint8_t>> hs((size_t)ctx->n_levels);
  for (int g = 1; g < ctx->n_levels && e == hipSuccess; ++g) {
    hs[(size_t)g].resize((size_t)ctx->lv[g].n_cells);
    e = hipMemcpyAsync(hs[(size_t)g].data(), status[(size_t)g], hs[(size_t)g].size(),
                       hipMemcpyDeviceToHost, s);
  }
  {
    // both streams drain before any buffer is released, on every path
    const hipError_t e1 = hipStreamSynchronize(s);
    const hipError_t e2 = hipStreamSynchronize(side);
    if (e == hipSuccess) e = (e1 != hipSuccess) ? e1 : e2;
  }
  cleanup();
  if (e != hipSuccess) {
    free_inverses(ctx);
    return fail(ctx, STV_EHIP, std::string("inverse build failed: ") + hipGetErrorString(e));
  }
  for (int g = 1; g < ctx->n_levels; ++g)
    for (int32_t c = 0; c < ctx->lv[g].n_cells; ++c)
      if (hs[(size_t)g][(size_t)c]) {
        if (bad_level) *bad_level = g;
        if (bad_cell) *bad_cell = c;
        free_inverses(ctx);
        return fail(ctx, STV_ESINGULAR,
                    "zero pivot in J_T of level " + std::to_string(g) + " cell " + std::to_string(c));
      }
  if (coarse_singular) {
    if (bad_level) *bad_level = 0;
    if (bad_cell) *bad_cell = -1;
    free_inverses(ctx);
    return fail(ctx, STV_ESINGULAR, "zero pivot in the coarse matrix");
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
  Timed t(ctx, KC_TRANSFER);
  STV_HIP(launch_restrict(ctx->stream, ctx->b, ctx->lv[level], rho, r_c));
  t.done();
  return STV_OK;
}

int stv_prolongate_add(stv_ctx* ctx, int level, const double* d_c, double* d) {
  STV_TRY(check_ctx(ctx, true, false));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level must be in [1, n_levels)");
  Timed t(ctx, KC_TRANSFER);
  STV_HIP(launch_prolongate_add(ctx->stream, ctx->b, ctx->lv[level], d_c, d));
  t.done();
  return STV_OK;
}

int stv_coarse_solve(stv_ctx* ctx, const double* r, double* d) {
  STV_TRY(check_ctx(ctx, true, true));
  if (!r || !d || r == d) return fail(ctx, STV_EINVAL, "r, d must be distinct non-NULL vectors");
  return coarse_apply(ctx, r, d);
}

int stv_vcycle(stv_ctx* ctx, const double* r, double* d, const stv_mg_params* p) {
  STV_TRY(check_ctx(ctx, true, true));
  STV_TRY(check_mg(ctx, p));
  if (!r || !d || r == d) return fail(ctx, STV_EINVAL, "r, d must be distinct non-NULL vectors");
  return vcycle_level(ctx, ctx->n_levels - 1, r, d, *p);
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
  hipStream_t s = ctx->stream;
  double* hs = ctx->hscal;
  int iters = 0, restarts = 0, hist_len = 0;
  auto push_hist = [&](double v) {
    if (info && info->history && hist_len < info->history_cap) info->history[hist_len] = v;
    ++hist_len;
  };
  auto finish = [&](int conv, double relres, int rc) {
    if (info) {
      info->iters = iters;
      info->restarts = restarts;
      info->converged = conv;
      info->true_relres = relres;
      info->history_len = std::min(hist_len, info->history ? info->history_cap : 0);
    }
    resolve_timers(ctx);
    return rc;
  };
  if (!p->use_x0) STV_HIP(launch_fill(s, x, n, 0.0));
  double bn2 = 0.0;
  STV_TRY(dot_to_host(ctx, bvec, bvec, n, &bn2));
  const double bnorm = std::sqrt(bn2);
  if (!std::isfinite(bnorm)) return finish(0, NAN, fail(ctx, STV_ENUMERIC, "NaN/Inf in the right-hand side"));
  if (bnorm == 0.0) {
    STV_HIP(launch_fill(s, x, n, 0.0));
    STV_HIP(hipStreamSynchronize(s));
    return finish(1, 0.0, STV_OK);
  }
  const double target = p->rtol * bnorm;
  STV_TRY(residual(ctx, G, bvec, x, ctx->rt));
  double beta2 = 0.0;
  STV_TRY(dot_to_host(ctx, ctx->rt, ctx->rt, n, &beta2));
  double beta = std::sqrt(beta2);
  if (!std::isfinite(beta)) return finish(0, NAN, fail(ctx, STV_ENUMERIC, "NaN/Inf in the initial residual"));
  push_hist(beta / bnorm);
  bool converged = beta <= target && p->fixed_iters == 0;
  const int budget = p->fixed_iters > 0 ? p->fixed_iters : p->max_it;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1);
  auto Hij = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
  double* d_nrm = ctx->scal + 2 * kScalR;
  double* d_rt2 = ctx->scal + 2 * kScalR + 1;
  while (!converged && iters < budget) {
    std::fill(H.begin(), H.end(), 0.0);
    {
      Timed t(ctx, KC_KRYLOV);
      STV_HIP(launch_scale_by_norm(s, ctx->rt, d_rt2, ctx->V, n));   // d_rt2 = ||rt||^2
      t.done();
    }
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta;
    int j_end = 0;
    for (int j = 0; j < m; ++j) {
      double* vj = ctx->V + (int64_t)j * n;
      double* zj = ctx->Z + (int64_t)j * n;
      STV_TRY(vcycle_level(ctx, G, vj, zj, p->mg));
      STV_TRY(matvec(ctx, G, zj, ctx->w));
      {
        Timed t(ctx, KC_KRYLOV);
        STV_HIP(launch_multidot(s, ctx->V, j + 1, ctx->w, n, ctx->partial, ctx->scal));
        STV_HIP(launch_multiaxpy(s, ctx->V, j + 1, ctx->scal, -1.0, ctx->w, n));
        STV_HIP(launch_multidot(s, ctx->V, j + 1, ctx->w, n, ctx->partial, ctx->scal + kScalR));
        STV_HIP(launch_multiaxpy(s, ctx->V, j + 1, ctx->scal + kScalR, -1.0, ctx->w, n));
        STV_HIP(launch_multidot(s, ctx->w, 1, ctx->w, n, ctx->partial, d_nrm));
        STV_HIP(launch_scale_by_norm(s, ctx->w, d_nrm, ctx->V + (int64_t)(j + 1) * n, n));
        t.done();
      }
      STV_HIP(hipMemcpyAsync(hs, ctx->scal, sizeof(double) * (2 * kScalR + 1), hipMemcpyDeviceToHost, s));
      STV_HIP(hipStreamSynchronize(s));
      for (int i = 0; i <= j; ++i) Hij(i, j) = hs[i] + hs[kScalR + i];
      const double hn = std::sqrt(hs[2 * kScalR]);
      Hij(j + 1, j) = hn;
      for (int i = 0; i <= j + 1; ++i)
        if (!std::isfinite(Hij(i, j))) {
          resolve_timers(ctx);
          return finish(0, NAN, fail(ctx, STV_ENUMERIC, "NaN/Inf in the Arnoldi process at step " + std::to_string(iters)));
        }
      const bool breakdown = hn == 0.0;
      for (int i = 0; i < j; ++i) {
        const double tmp = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
        Hij(i + 1, j) = -sn[i] * Hij(i, j) + cs[i] * Hij(i + 1, j);
        Hij(i, j) = tmp;
      }
      const double den = std::hypot(Hij(j, j), Hij(j + 1, j));
      cs[j] = Hij(j, j) / den;
      sn[j] = Hij(j + 1, j) / den;
      Hij(j, j) = den;
      Hij(j + 1, j) = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      ++iters;
      j_end = j + 1;
      push_hist(std::fabs(gv[j + 1]) / bnorm);
      if (p->fixed_iters > 0) {
        if (iters >= p->fixed_iters || breakdown) break;
      } else if (std::fabs(gv[j + 1]) <= target || iters >= p->max_it || breakdown) {
        break;
      }
    }
    // y = R^-1 g (back substitution on the rotated Hessenberg matrix)
    std::vector<double> y((size_t)j_end);
    for (int i = j_end - 1; i >= 0; --i) {
      double acc = gv[i];
      for (int l = i + 1; l < j_end; ++l) acc -= Hij(i, l) * y[(size_t)l];
      y[(size_t)i] = acc / Hij(i, i);
    }
    for (int i = 0; i < j_end; ++i) hs[3 * kScalR + i] = y[(size_t)i];
    STV_HIP(hipMemcpyAsync(ctx->scal + 3 * kScalR, hs + 3 * kScalR, sizeof(double) * j_end,
                           hipMemcpyHostToDevice, s));
    {
      Timed t(ctx, KC_KRYLOV);
      STV_HIP(launch_multiaxpy(s, ctx->Z, j_end, ctx->scal + 3 * kScalR, 1.0, x, n));
      t.done();
    }
    STV_TRY(residual(ctx, G, bvec, x, ctx->rt));
    STV_TRY(dot_to_host(ctx, ctx->rt, ctx->rt, n, &beta2));
    beta = std::sqrt(beta2);
    ++restarts;
    if (!std::isfinite(beta)) return finish(0, NAN, fail(ctx, STV_ENUMERIC, "NaN/Inf in the true residual"));
    if (p->fixed_iters == 0 && beta <= target) converged = true;
    if (beta == 0.0) {
      converged = p->fixed_iters == 0 || iters >= p->fixed_iters;
      break;
    }
  }
  const double relres = beta / bnorm;
  const int conv = relres <= p->rtol ? 1 : 0;
  if (p->fixed_iters == 0 && !conv)
    return finish(0, relres, fail(ctx, STV_ENOCONV, "GMRES did not reach rtol within max_it steps"));
  return finish(conv, relres, STV_OK);
}

int stv_get_cell_inverse(stv_ctx* ctx, int level, int cell, double* out) {
  STV_TRY(check_ctx(ctx, true, true));
  if (level < 1 || level >= ctx->n_levels) return fail(ctx, STV_EINVAL, "level must be in [1, n_levels)");
  DevLevel& L = ctx->lv[level];
  if (cell < 0 || cell >= L.n_cells) return fail(ctx, STV_EINVAL, "cell out of range");
  if (!out) return fail(ctx, STV_EINVAL, "out is NULL");
  const int b = ctx->b, nls = L.n_ls, n = nls * b;
  const int o0 = L.h_own_ptr[(size_t)cell], no = L.h_own_ptr[(size_t)cell + 1] - o0;
  const int R = ctx->inv_full ? n : no * b;
  std::vector<int64_t> off(1);
  STV_HIP(hipMemcpy(off.data(), L.inv_off + cell, sizeof(int64_t), hipMemcpyDeviceToHost));
  std::vector<double> blk((size_t)R * n);
  if (ctx->inv_fp32) {
    std::vector<float> f((size_t)R * n);
    STV_HIP(hipMemcpy(f.data(), (const float*)L.inv_store + off[0], sizeof(float) * f.size(), hipMemcpyDeviceToHost));
    for (size_t i = 0; i < f.size(); ++i) blk[i] = f[i];
  } else {
    STV_HIP(hipMemcpy(blk.data(), (const double*)L.inv_store + off[0], sizeof(double) * blk.size(), hipMemcpyDeviceToHost));
  }
  for (int64_t e = 0; e < (int64_t)n * n; ++e) out[e] = NAN;
  // stored row index -> internal local index (alpha*b + l)
  for (int o = 0; o < R; ++o) {
    int alpha, l;
    if (ctx->inv_full) { alpha = o / b; l = o % b; }
    else { alpha = L.h_own_loc[(size_t)(o0 + o / b)]; l = o % b; }
    const int row = l * nls + alpha;   // eq. (4.4) order
    for (int j = 0; j < n; ++j) {
      const int beta = j / b, lj = j % b;
      out[(int64_t)row * n + lj * nls + beta] = blk[(size_t)o * n + j];   // stored row-major
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
  if (n_cells) *n_cells = L.n_cells;
  if (n_loc) *n_loc = (int64_t)L.n_ls * ctx->b;
  if (inverse_bytes) *inverse_bytes = L.inv_elems * (ctx->inv_fp32 ? 4 : 8);
  return STV_OK;
}

int stv_set_option(stv_ctx* ctx, int option, int64_t value) {
  if (!ctx) return STV_EINVAL;
  switch (option) {
    case STV_OPT_COARSE_ALGO:
      if (value < 0 || value > 2) return fail(ctx, STV_EINVAL, "coarse algorithm must be 0, 1 or 2");
      ctx->coarse_algo = (int)value;
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
