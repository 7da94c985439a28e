// Dense coarse level (the direct solve of Algorithm 4.1 on the coarsest
// grid): the level matrix is expanded to a dense FP64 array, inverted once by
// Gauss-Jordan elimination with partial pivoting (one pivot kernel and one
// rank-1 update kernel per step), and applied as a dense matrix-vector
// product in every V-cycle.
#include "stv_internal.h"

namespace stv {

template <int B>
__global__ void k_bsr_to_dense(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const double* __restrict__ val, double* __restrict__ A, int64_t n,
                               int32_t n_rows) {
  const int32_t row = blockIdx.x;
  if (row >= n_rows) return;
  for (int32_t q = rowptr[row] + threadIdx.x; q < rowptr[row + 1]; q += blockDim.x) {
    const int64_t c = col[q];
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int l = 0; l < B; ++l)
        A[((int64_t)row * B + i) * n + c * B + l] = val[(int64_t)q * B * B + i * B + l];
  }
}

hipError_t launch_bsr_to_dense(hipStream_t s, int b, const DevLevel& L, double* A, int64_t n) {
  switch (b) {
    case 1: k_bsr_to_dense<1><<<L.n_s, 64, 0, s>>>(L.rowptr, L.col, L.val, A, n, L.n_s); break;
    case 2: k_bsr_to_dense<2><<<L.n_s, 64, 0, s>>>(L.rowptr, L.col, L.val, A, n, L.n_s); break;
    case 3: k_bsr_to_dense<3><<<L.n_s, 64, 0, s>>>(L.rowptr, L.col, L.val, A, n, L.n_s); break;
    case 4: k_bsr_to_dense<4><<<L.n_s, 64, 0, s>>>(L.rowptr, L.col, L.val, A, n, L.n_s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Pivot search of column p (largest magnitude, lowest index on ties) and
// copies of the pivot row, old row p and column p.  piv[p] = r, or -1 when the
// column holds no nonzero finite candidate (singular).
__global__ void __launch_bounds__(1024) k_gj_pivot(const double* __restrict__ A, int64_t n, int p,
                                                   double* __restrict__ prow,
                                                   double* __restrict__ trow,
                                                   double* __restrict__ pcol, int* piv) {
  __shared__ double sb[16];
  __shared__ int si[16];
  __shared__ int rsh;
  const int tid = threadIdx.x;
  double best = -1.0;
  int bi = 0x7fffffff;
  for (int64_t i = p + tid; i < n; i += blockDim.x) {
    const double v = fabs(A[i * n + p]);
    if (v > best) { best = v; bi = (int)i; }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const double ob = __shfl_xor(best, off, 64);
    const int oi = __shfl_xor(bi, off, 64);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
  }
  if ((tid & 63) == 0) { sb[tid >> 6] = best; si[tid >> 6] = bi; }
  __syncthreads();
  if (tid == 0) {
    double b0 = sb[0];
    int i0 = si[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w)
      if (sb[w] > b0 || (sb[w] == b0 && si[w] < i0)) { b0 = sb[w]; i0 = si[w]; }
    const bool ok = (i0 < n) && (b0 > 0.0);
    rsh = (i0 < n) ? i0 : p;
    piv[p] = ok ? i0 : -1;
  }
  __syncthreads();
  const int64_t r = rsh;
  for (int64_t j = tid; j < n; j += blockDim.x) {
    prow[j] = A[r * n + j];
    trow[j] = A[(int64_t)p * n + j];
    pcol[j] = A[j * n + p];
  }
}

// Gauss-Jordan update of step p; element (i, j) depends only on its own old
// value and the copies made by k_gj_pivot.
__global__ void k_gj_update(double* __restrict__ A, int64_t n, int p,
                            const double* __restrict__ prow, const double* __restrict__ trow,
                            const double* __restrict__ pcol, const int* __restrict__ piv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j >= n) return;
  const int pr = piv[p];
  const int64_t r = pr >= 0 ? pr : p;
  const double pv = prow[p];
  const double ipiv = (pr >= 0 && pv != 0.0) ? 1.0 / pv : 0.0;
  double out;
  if (i == p) {
    out = (j == p) ? ipiv : prow[j] * ipiv;
  } else {
    const double f = ((i == r) ? pcol[p] : pcol[i]) * ipiv;
    const double src = (i == r) ? trow[j] : A[i * n + j];
    out = (j == p) ? -f : fma(-f, prow[j], src);
  }
  A[i * n + j] = out;
}

hipError_t launch_gj_step(hipStream_t s, double* A, int64_t n, int p, double* prow, double* trow,
                          double* pcol, int* piv) {
  k_gj_pivot<<<1, 1024, 0, s>>>(A, n, p, prow, trow, pcol, piv);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n), block(256);
  k_gj_update<<<grid, block, 0, s>>>(A, n, p, prow, trow, pcol, piv);
  return hipGetLastError();
}

__global__ void k_permute_cols(const double* __restrict__ A, double* __restrict__ out, int64_t n,
                               const int* __restrict__ sigma) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < n) out[i * n + j] = A[i * n + sigma[j]];
}

hipError_t launch_permute_cols(hipStream_t s, const double* A, double* out, int64_t n,
                               const int* sigma) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n), block(256);
  k_permute_cols<<<grid, block, 0, s>>>(A, out, n, sigma);
  return hipGetLastError();
}

// y = A x, one wavefront per row of the row-major dense inverse.
__global__ void __launch_bounds__(256) k_dense_gemv(const double* __restrict__ A, int64_t n,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const double* Ar = A + row * n;
  double acc = 0.0;
  for (int64_t j = lane; j < n; j += 64) acc = fma(Ar[j], x[j], acc);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[row] = acc;
}

hipError_t launch_dense_gemv(hipStream_t s, const double* A, int64_t n, const double* x,
                             double* y) {
  k_dense_gemv<<<(unsigned)((n + 3) / 4), 256, 0, s>>>(A, n, x, y);
  return hipGetLastError();
}

}  // namespace stv
