// Grid transfers of the V-cycle (Sec. 4.1: prolongation by interpolation
// between the nested spaces of consecutive levels, restriction by its
// transpose), identity in time: y (+)= (P (x) I_B) x for a spatial CSR matrix
// P and time-inner vectors (x[c*B + l], B = k+1 temporal DoFs per spatial
// DoF).  Restriction uses the stored transpose of P, so both directions are
// gathers (no atomics).
#include "stv_internal.h"

namespace stv {

// LPR lanes per spatial row (LPR in {1, 2, 4, 8, 16}; a row's lanes are
// consecutive and never straddle a row of 16 lanes) and all B time levels
// per lane.  Lane q of a row takes the row's entries e0 + q, e0 + q + LPR,
// ..., four per round with every load in flight, so consecutive lanes read
// consecutive column indices and values; the B entries of x at a column are
// adjacent.  The LPR partial sums are combined by lane exchanges (lane ^ M,
// M = LPR/2 .. 1), after which every lane of the row holds the row's sums, and
// lane q stores the time levels l with l % LPR == q.  For a given shape the
// order of the additions is fixed, so results are reproducible.
template <int B, int LPR>
__global__ void __launch_bounds__(256) k_csr_lanes(const int32_t* __restrict__ rp,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, int32_t n_rows,
                                                   int accumulate) {
  constexpr int U = 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t row = t / LPR;
  const int q = (int)(threadIdx.x & (LPR - 1));
  const bool live = row < n_rows;
  if (LPR == 1 && !live) return;
  int32_t e0 = 0, e1 = 0;
  if (live) {
    e0 = rp[row];
    e1 = rp[row + 1];
  }
  double acc[B];
#pragma unroll
  for (int l = 0; l < B; ++l) acc[l] = 0.0;
  for (int32_t e = e0 + q; e < e1; e += U * LPR) {
    int64_t c[U];
    double v[U], xv[U][B];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t eu = e + u * LPR;
      const bool ok = eu < e1;
      const int32_t ec = ok ? eu : e;   // e < e1: a valid entry of this row
      c[u] = col[ec];
      const double w = val[ec];
      v[u] = ok ? w : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int l = 0; l < B; ++l) xv[u][l] = x[c[u] * B + l];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int l = 0; l < B; ++l) acc[l] = fma(v[u], xv[u][l], acc[l]);
  }
  // every lane of the wavefront is here (no lane has returned when LPR > 1)
#pragma unroll
  for (int m = LPR / 2; m >= 1; m >>= 1)
#pragma unroll
    for (int l = 0; l < B; ++l) acc[l] += __shfl_xor(acc[l], m, 64);
  if (!live) return;
  double* yr = y + row * B;
#pragma unroll
  for (int l = 0; l < B; ++l)
    if (l % LPR == q) yr[l] = accumulate ? yr[l] + acc[l] : acc[l];
}

template <int B>
static void csr_shape(int lanes, dim3 grid, hipStream_t s, const int32_t* rp, const int32_t* col,
                      const double* val, const double* x, double* y, int32_t n_rows, int acc) {
  const dim3 block(256);
  switch (lanes) {
    case 1: launch(k_csr_lanes<B, 1>, grid, block, 0, s, rp, col, val, x, y, n_rows, acc); break;
    case 2: launch(k_csr_lanes<B, 2>, grid, block, 0, s, rp, col, val, x, y, n_rows, acc); break;
    case 4: launch(k_csr_lanes<B, 4>, grid, block, 0, s, rp, col, val, x, y, n_rows, acc); break;
    case 8: launch(k_csr_lanes<B, 8>, grid, block, 0, s, rp, col, val, x, y, n_rows, acc); break;
    default: launch(k_csr_lanes<B, 16>, grid, block, 0, s, rp, col, val, x, y, n_rows, acc); break;
  }
}

static hipError_t csr_time(hipStream_t s, int b, int shape, const int32_t* rp,
                           const int32_t* col, const double* val, const double* x, double* y,
                           int32_t n_rows, int acc) {
  if (shape < 1 || shape > kTransferShapes) return hipErrorInvalidValue;
  if (n_rows <= 0) return hipSuccess;
  const int lanes = 1 << (shape - 1);
  const dim3 grid((unsigned)(((int64_t)n_rows * lanes + 255) / 256));
  switch (b) {
    case 1: csr_shape<1>(lanes, grid, s, rp, col, val, x, y, n_rows, acc); break;
    case 2: csr_shape<2>(lanes, grid, s, rp, col, val, x, y, n_rows, acc); break;
    case 3: csr_shape<3>(lanes, grid, s, rp, col, val, x, y, n_rows, acc); break;
    case 4: csr_shape<4>(lanes, grid, s, rp, col, val, x, y, n_rows, acc); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int transfer_shape_for(int64_t nnz, int64_t n_rows) {
  // lanes per row about the mean row length: 1 below 3 entries, then 2, 4,
  // 8 and 16 for means below 6, 12, 24 and above
  const double mean = n_rows > 0 ? (double)nnz / (double)n_rows : 0.0;
  int shape = 1;
  for (double lim = 3.0; mean >= lim && shape < kTransferShapes; lim *= 2.0) ++shape;
  return shape;
}

hipError_t launch_restrict(hipStream_t s, int b, const DevLevel& L, const double* rho,
                           double* r_c) {
  return csr_time(s, b, L.pt_shape, L.Pt_rowptr, L.Pt_col, L.Pt_val, rho, r_c, L.n_s_coarse, 0);
}

hipError_t launch_prolongate_add(hipStream_t s, int b, const DevLevel& L, const double* d_c,
                                 double* d) {
  return csr_time(s, b, L.p_shape, L.P_rowptr, L.P_col, L.P_val, d_c, d, L.n_s, 1);
}

}  // namespace stv
