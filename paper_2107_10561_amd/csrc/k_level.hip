// Level kernels of the V-cycle: the block-sparse level residual, the Vanka
// cell sweep and the grid transfers.  Vectors are FP64 and time-inner
// (x[s*B + l], B = k+1 temporal DoFs per spatial DoF).
#include "stv_internal.h"

namespace stv {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// ---------------------------------------------------------------------------
// Level residual y = r + sx J x  (sx = -1: r - J x; r == nullptr: sx J x).
// One 64-lane wavefront per block row.  Lane (q_off, j) streams block column
// j of every (64/B)-th block of the row, so consecutive lanes read
// consecutive doubles of the row's value array; B partial sums per lane are
// folded across the wavefront at the end.
template <int B>
__global__ void __launch_bounds__(256) k_spmv(const int32_t* __restrict__ rowptr,
                                              const int32_t* __restrict__ col,
                                              const double* __restrict__ val,
                                              const double* __restrict__ r,
                                              const double* __restrict__ x,
                                              double* __restrict__ y, int32_t n_rows, double sx) {
  constexpr int NQ = 64 / B;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n_rows) return;  // uniform per wavefront
  const int qo = lane / B;
  const int j = lane - qo * B;
  const int32_t q0 = rowptr[row], q1 = rowptr[row + 1];
  double acc[B];
#pragma unroll
  for (int i = 0; i < B; ++i) acc[i] = 0.0;
  if (qo < NQ) {
#pragma unroll 2
    for (int32_t q = q0 + qo; q < q1; q += NQ) {
      const int32_t c = col[q];
      const double xv = x[(int64_t)c * B + j];
      const double* vb = val + (int64_t)q * (B * B) + j;
#pragma unroll
      for (int i = 0; i < B; ++i) acc[i] = fma(vb[i * B], xv, acc[i]);
    }
  }
#pragma unroll
  for (int i = 0; i < B; ++i) acc[i] = wave_sum(acc[i]);
  if (lane < B) {
    double a = acc[0];
#pragma unroll
    for (int i = 1; i < B; ++i)
      if (lane == i) a = acc[i];
    const int64_t o = (int64_t)row * B + lane;
    y[o] = r ? fma(sx, a, r[o]) : sx * a;
  }
}

hipError_t launch_spmv(hipStream_t s, int b, const DevLevel& L, const double* r, const double* x,
                       double* y, double sx) {
  dim3 grid((L.n_s + 3) / 4), block(256);
  switch (b) {
    case 1: k_spmv<1><<<grid, block, 0, s>>>(L.rowptr, L.col, L.val, r, x, y, L.n_s, sx); break;
    case 2: k_spmv<2><<<grid, block, 0, s>>>(L.rowptr, L.col, L.val, r, x, y, L.n_s, sx); break;
    case 3: k_spmv<3><<<grid, block, 0, s>>>(L.rowptr, L.col, L.val, r, x, y, L.n_s, sx); break;
    case 4: k_spmv<4><<<grid, block, 0, s>>>(L.rowptr, L.col, L.val, r, x, y, L.n_s, sx); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vanka cell sweep, last-writer form.  One wavefront per cell T:
//   rho_T  <- gather of the level residual on the cell's n_loc DoFs (LDS),
//   c      <- J_T^-1 rho_T for the rows of the DoFs T owns,
//   d_j    <- d_j + omega c_j  (or omega c_j for a zero initial iterate).
// Every DoF has exactly one owner (the last cell in loop order containing
// it), so the stores are disjoint: no atomics, deterministic.
// Inverse blocks are column-major per cell (element (i, j) at j*ld + i), so
// the lanes of one row chunk read consecutive addresses of a column.  When
// the cell has at most 32 stored rows, 64/R columns are read per step.
template <int B, typename TS>
__global__ void __launch_bounds__(64) k_vanka(const double* __restrict__ rho,
                                             double* __restrict__ d,
                                             const int32_t* __restrict__ csd, int n_ls,
                                             const int32_t* __restrict__ own_ptr,
                                             const uint8_t* __restrict__ own_loc,
                                             const int64_t* __restrict__ inv_off,
                                             const TS* __restrict__ store, double omega,
                                             int zero_init, int full) {
  extern __shared__ double sm[];
  const int n_loc = n_ls * B;
  double* xs = sm;
  double* part = sm + n_loc;
  const int T = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t* sd = csd + (int64_t)T * n_ls;
  for (int e = lane; e < n_loc; e += 64) {
    const int be = e / B;
    const int l = e - be * B;
    xs[e] = rho[(int64_t)sd[be] * B + l];
  }
  __syncthreads();
  const int o0 = own_ptr[T];
  const int R = (own_ptr[T + 1] - o0) * B;
  const TS* A = store + inv_off[T];
  if (!full && R <= 32) {
    const int S = 64 / R;
    const int i = lane % R;
    const int js = lane / R;
    double acc = 0.0;
    if (js < S) {
      const TS* Ai = A + i;
#pragma unroll 4
      for (int j = js; j < n_loc; j += S) acc = fma((double)Ai[(int64_t)j * R], xs[j], acc);
    }
    part[lane] = acc;
    __syncthreads();
    if (lane < R) {
      double sacc = 0.0;
      for (int t = 0; t < S; ++t) sacc += part[lane + t * R];
      const int o = lane / B;
      const int l = lane - o * B;
      const int64_t g = (int64_t)sd[own_loc[o0 + o]] * B + l;
      d[g] = zero_init ? omega * sacc : d[g] + omega * sacc;
    }
  } else {
    const int ld = full ? n_loc : R;
    for (int i0 = 0; i0 < R; i0 += 64) {
      const int i = i0 + lane;
      if (i < R) {
        const int o = i / B;
        const int l = i - o * B;
        const int alpha = own_loc[o0 + o];
        const TS* Ai = A + (full ? alpha * B + l : i);
        double acc = 0.0;
#pragma unroll 4
        for (int j = 0; j < n_loc; ++j) acc = fma((double)Ai[(int64_t)j * ld], xs[j], acc);
        const int64_t g = (int64_t)sd[alpha] * B + l;
        d[g] = zero_init ? omega * acc : d[g] + omega * acc;
      }
    }
  }
}

template <int B>
static hipError_t vanka_b(hipStream_t s, const DevLevel& L, const double* rho, double* d,
                          double omega, int zero_init, int fp32, int full) {
  const size_t shm = sizeof(double) * (size_t)(L.n_ls * B + 64);
  if (fp32)
    k_vanka<B, float><<<L.n_cells, 64, shm, s>>>(rho, d, L.cell_sdofs, L.n_ls, L.own_ptr,
                                                 L.own_loc, L.inv_off, (const float*)L.inv_store,
                                                 omega, zero_init, full);
  else
    k_vanka<B, double><<<L.n_cells, 64, shm, s>>>(rho, d, L.cell_sdofs, L.n_ls, L.own_ptr,
                                                  L.own_loc, L.inv_off,
                                                  (const double*)L.inv_store, omega, zero_init,
                                                  full);
  return hipGetLastError();
}

hipError_t launch_vanka_cells(hipStream_t s, int b, const DevLevel& L, const double* rho,
                              double* d, double omega, int zero_init, int fp32, int full) {
  switch (b) {
    case 1: return vanka_b<1>(s, L, rho, d, omega, zero_init, fp32, full);
    case 2: return vanka_b<2>(s, L, rho, d, omega, zero_init, fp32, full);
    case 3: return vanka_b<3>(s, L, rho, d, omega, zero_init, fp32, full);
    case 4: return vanka_b<4>(s, L, rho, d, omega, zero_init, fp32, full);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Averaged / additive forms: every cell writes its full damped correction
// omega J_T^-1 rho_T to corr[T*n_loc + (alpha*B + l)]; a second kernel sums,
// per DoF and in cell order, the corrections of the cells containing it.
template <int B, typename TS>
__global__ void __launch_bounds__(64) k_vanka_corr(const double* __restrict__ rho,
                                                  double* __restrict__ corr,
                                                  const int32_t* __restrict__ csd, int n_ls,
                                                  const int64_t* __restrict__ inv_off,
                                                  const TS* __restrict__ store, double omega) {
  extern __shared__ double sm[];
  const int n_loc = n_ls * B;
  const int T = blockIdx.x;
  const int lane = threadIdx.x;
  const int32_t* sd = csd + (int64_t)T * n_ls;
  for (int e = lane; e < n_loc; e += 64) {
    const int be = e / B;
    sm[e] = rho[(int64_t)sd[be] * B + (e - be * B)];
  }
  __syncthreads();
  const TS* A = store + inv_off[T];
  for (int i = lane; i < n_loc; i += 64) {
    double acc = 0.0;
    for (int j = 0; j < n_loc; ++j) acc = fma((double)A[(int64_t)j * n_loc + i], sm[j], acc);
    corr[(int64_t)T * n_loc + i] = omega * acc;
  }
}

template <int B>
__global__ void k_vanka_combine(const double* __restrict__ corr, double* __restrict__ d,
                                const int32_t* __restrict__ inc_ptr,
                                const int32_t* __restrict__ inc_cell,
                                const uint8_t* __restrict__ inc_loc, int n_s, int n_loc, int pou) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_s * B) return;
  const int s = (int)(idx / B);
  const int l = (int)(idx - (int64_t)s * B);
  const int e0 = inc_ptr[s], e1 = inc_ptr[s + 1];
  double acc = 0.0;
  for (int e = e0; e < e1; ++e) acc += corr[(int64_t)inc_cell[e] * n_loc + inc_loc[e] * B + l];
  if (pou) acc /= (double)(e1 - e0);
  d[idx] += acc;
}

hipError_t launch_vanka_cells_corr(hipStream_t s, int b, const DevLevel& L, const double* rho,
                                   double omega, int fp32) {
  const size_t shm = sizeof(double) * (size_t)(L.n_ls * b);
#define STV_CORR(BB)                                                                        \
  if (fp32)                                                                                 \
    k_vanka_corr<BB, float><<<L.n_cells, 64, shm, s>>>(rho, L.corr, L.cell_sdofs, L.n_ls,   \
                                                       L.inv_off, (const float*)L.inv_store, \
                                                       omega);                              \
  else                                                                                      \
    k_vanka_corr<BB, double><<<L.n_cells, 64, shm, s>>>(rho, L.corr, L.cell_sdofs, L.n_ls,  \
                                                        L.inv_off,                          \
                                                        (const double*)L.inv_store, omega);
  switch (b) {
    case 1: STV_CORR(1) break;
    case 2: STV_CORR(2) break;
    case 3: STV_CORR(3) break;
    case 4: STV_CORR(4) break;
    default: return hipErrorInvalidValue;
  }
#undef STV_CORR
  return hipGetLastError();
}

hipError_t launch_vanka_combine(hipStream_t s, int b, const DevLevel& L, double* d, int pou) {
  const int64_t n = (int64_t)L.n_s * b;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  const int n_loc = L.n_ls * b;
  switch (b) {
    case 1: k_vanka_combine<1><<<grid, block, 0, s>>>(L.corr, d, L.inc_ptr, L.inc_cell, L.inc_loc, L.n_s, n_loc, pou); break;
    case 2: k_vanka_combine<2><<<grid, block, 0, s>>>(L.corr, d, L.inc_ptr, L.inc_cell, L.inc_loc, L.n_s, n_loc, pou); break;
    case 3: k_vanka_combine<3><<<grid, block, 0, s>>>(L.corr, d, L.inc_ptr, L.inc_cell, L.inc_loc, L.n_s, n_loc, pou); break;
    case 4: k_vanka_combine<4><<<grid, block, 0, s>>>(L.corr, d, L.inc_ptr, L.inc_cell, L.inc_loc, L.n_s, n_loc, pou); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Transfers: y[row*B + l] (+)= sum_e val[e] x[col[e]*B + l] for a spatial CSR
// (identity in time).  Restriction uses the stored transpose of P, so both
// directions are gathers (no atomics).
template <int B>
__global__ void k_csr_time(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const double* __restrict__ val, const double* __restrict__ x,
                           double* __restrict__ y, int32_t n_rows, int accumulate) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n_rows * B) return;
  const int32_t row = (int32_t)(idx / B);
  const int l = (int)(idx - (int64_t)row * B);
  double acc = 0.0;
  for (int32_t e = rp[row]; e < rp[row + 1]; ++e) acc = fma(val[e], x[(int64_t)col[e] * B + l], acc);
  y[idx] = accumulate ? y[idx] + acc : acc;
}

static hipError_t csr_time(hipStream_t s, int b, const int32_t* rp, const int32_t* col,
                           const double* val, const double* x, double* y, int32_t n_rows,
                           int acc) {
  const int64_t n = (int64_t)n_rows * b;
  dim3 grid((unsigned)((n + 255) / 256)), block(256);
  switch (b) {
    case 1: k_csr_time<1><<<grid, block, 0, s>>>(rp, col, val, x, y, n_rows, acc); break;
    case 2: k_csr_time<2><<<grid, block, 0, s>>>(rp, col, val, x, y, n_rows, acc); break;
    case 3: k_csr_time<3><<<grid, block, 0, s>>>(rp, col, val, x, y, n_rows, acc); break;
    case 4: k_csr_time<4><<<grid, block, 0, s>>>(rp, col, val, x, y, n_rows, acc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_restrict(hipStream_t s, int b, const DevLevel& L, const double* rho,
                           double* r_c) {
  return csr_time(s, b, L.Pt_rowptr, L.Pt_col, L.Pt_val, rho, r_c, L.n_s_coarse, 0);
}

hipError_t launch_prolongate_add(hipStream_t s, int b, const DevLevel& L, const double* d_c,
                                 double* d) {
  return csr_time(s, b, L.P_rowptr, L.P_col, L.P_val, d_c, d, L.n_s, 1);
}

__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

__global__ void k_copy(const double* __restrict__ x, double* __restrict__ y, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}

hipError_t launch_fill(hipStream_t s, double* x, int64_t n, double v) {
  if (n <= 0) return hipSuccess;
  k_fill<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, n, v);
  return hipGetLastError();
}

hipError_t launch_copy(hipStream_t s, const double* x, double* y, int64_t n) {
  if (n <= 0) return hipSuccess;
  k_copy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(x, y, n);
  return hipGetLastError();
}

}  // namespace stv
