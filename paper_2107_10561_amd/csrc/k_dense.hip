// Dense coarse level (the direct solve of Algorithm 4.1 on the coarsest
// grid): the level matrix is expanded to a dense FP64 array (padded with an
// identity block to a multiple of the panel width), inverted once by blocked
// Gauss-Jordan elimination with partial pivoting, and applied as a dense
// matrix-vector product in every V-cycle.
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

// Blocked Gauss-Jordan inversion with partial pivoting.  Panel of NB columns
// [p0, p0+NB): one 1024-thread workgroup holds the n x NB panel in registers
// (thread t owns rows t + 1024 m) and runs NB elimination steps on it with
// full-row swaps inside the panel; the panel columns then hold the columns of
// the accumulated elimination matrix E.  Every other column j (earlier panels
// included) is then brought up to date at once: apply the panel's row swaps,
// then A(:, j) += (E - I)(:, panel) A(panel rows, j), a rank-NB update.
// piv[p] records the pivot row of step p (-1: no nonzero pivot).
template <int RPT, int NB>
__global__ void __launch_bounds__(1024) k_gj_panel(double* __restrict__ A, int64_t n, int p0,
                                                   int* __restrict__ piv) {
  __shared__ double wbest[2][16];
  __shared__ int widx[2][16];
  __shared__ double prow[2][NB];
  __shared__ double trow[2][NB];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double P[RPT][NB];
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const int64_t i = tid + 1024 * m;
#pragma unroll
    for (int t = 0; t < NB; ++t) P[m][t] = (i < n) ? A[i * n + p0 + t] : 0.0;
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int p = p0 + t;
    const int par = t & 1;
    double best = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int i = tid + 1024 * m;
      double v = 0.0;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c == t) v = P[m][c];
      v = fabs(v);
      if (i >= p && i < n && v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { wbest[par][wv] = best; widx[par][wv] = bi; }
    __syncthreads();
    best = wbest[par][0];
    bi = widx[par][0];
#pragma unroll
    for (int w2 = 1; w2 < 16; ++w2) {
      const double ob = wbest[par][w2];
      const int oi = widx[par][w2];
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const bool ok = (bi < n) && (best > 0.0);
    const int r = ok ? bi : p;
    // owners of rows r and p publish them
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int i = tid + 1024 * m;
      if (i == r) {
#pragma unroll
        for (int c = 0; c < NB; ++c) prow[par][c] = P[m][c];
      }
      if (i == p) {
#pragma unroll
        for (int c = 0; c < NB; ++c) trow[par][c] = P[m][c];
      }
    }
    if (tid == 0) piv[p] = ok ? r : -1;
    __syncthreads();
    const double pv = prow[par][t];
    const double ipiv = (ok && pv != 0.0) ? 1.0 / pv : 0.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const int i = tid + 1024 * m;
      if (i == p) {
#pragma unroll
        for (int c = 0; c < NB; ++c) P[m][c] = (c == t) ? ipiv : prow[par][c] * ipiv;
      } else {
        double own = 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c == t) own = P[m][c];
        const bool isr = (i == r);
        const double f = (isr ? trow[par][t] : own) * ipiv;
#pragma unroll
        for (int c = 0; c < NB; ++c) {
          const double src = isr ? trow[par][c] : P[m][c];
          P[m][c] = (c == t) ? -f : fma(-f, prow[par][c], src);
        }
      }
    }
  }
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const int64_t i = tid + 1024 * m;
    if (i < n) {
#pragma unroll
      for (int t = 0; t < NB; ++t) A[i * n + p0 + t] = P[m][t];
    }
  }
}

// Row swaps of the panel on every column outside it, then a copy of the
// panel rows of those columns (the right factor of the rank-NB update).
__global__ void k_gj_swap_copy(double* __restrict__ A, int64_t n, int p0, int nb,
                               const int* __restrict__ piv, double* __restrict__ Bbuf) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n || (j >= p0 && j < p0 + nb)) return;
  for (int t = 0; t < nb; ++t) {
    const int pr = piv[p0 + t];
    const int64_t r = pr >= 0 ? pr : p0 + t;
    const int64_t p = p0 + t;
    if (r != p) {
      const double a = A[p * n + j];
      A[p * n + j] = A[r * n + j];
      A[r * n + j] = a;
    }
  }
  for (int t = 0; t < nb; ++t) Bbuf[(int64_t)t * n + j] = A[(int64_t)(p0 + t) * n + j];
}

// A(i, j) += sum_t (E(i, p0+t) - delta) * Bbuf(t, j) for j outside the panel.
template <int NB>
__global__ void __launch_bounds__(256) k_gj_rank_update(double* __restrict__ A, int64_t n, int p0,
                                                        const double* __restrict__ Bbuf) {
  const int64_t j = (int64_t)blockIdx.x * 64 + (threadIdx.x & 63);
  const int64_t i0 = (int64_t)blockIdx.y * 16 + (threadIdx.x >> 6) * 4;
  if (j >= n || (j >= p0 && j < p0 + NB)) return;
  double bcol[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) bcol[t] = Bbuf[(int64_t)t * n + j];
#pragma unroll
  for (int di = 0; di < 4; ++di) {
    const int64_t i = i0 + di;
    if (i >= n) break;
    const double* Wi = A + i * n + p0;
    double acc = A[i * n + j];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const double w = Wi[t] - ((i == p0 + t) ? 1.0 : 0.0);
      acc = fma(w, bcol[t], acc);
    }
    A[i * n + j] = acc;
  }
}

template <int RPT, int NB>
static hipError_t gj_blocked(hipStream_t s, double* A, int64_t n, int* piv, double* Bbuf) {
  for (int64_t p0 = 0; p0 < n; p0 += NB) {
    k_gj_panel<RPT, NB><<<1, 1024, 0, s>>>(A, n, (int)p0, piv);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gj_swap_copy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(A, n, (int)p0, NB, piv, Bbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((n + 63) / 64), (unsigned)((n + 15) / 16));
    k_gj_rank_update<NB><<<grid, 256, 0, s>>>(A, n, (int)p0, Bbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// n must be a multiple of the panel width chosen here (the caller pads).
int gj_panel_width(int64_t n) {
  if (n <= 3072) return 8;
  if (n <= 6144) return 4;
  return 2;
}

hipError_t launch_gj_blocked(hipStream_t s, double* A, int64_t n, int* piv, double* Bbuf) {
  if (n <= 3072) return gj_blocked<3, 8>(s, A, n, piv, Bbuf);
  if (n <= 6144) return gj_blocked<6, 4>(s, A, n, piv, Bbuf);
  if (n <= 12288) return gj_blocked<12, 2>(s, A, n, piv, Bbuf);
  return hipErrorInvalidValue;
}

__global__ void k_set_diag(double* __restrict__ A, int64_t lda, int64_t from, int64_t to) {
  const int64_t i = from + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < to) A[i * lda + i] = 1.0;
}

hipError_t launch_set_diag(hipStream_t s, double* A, int64_t lda, int64_t from, int64_t to) {
  if (to <= from) return hipSuccess;
  k_set_diag<<<(unsigned)((to - from + 255) / 256), 256, 0, s>>>(A, lda, from, to);
  return hipGetLastError();
}

// out (n x n, compact) = columns sigma of the top-left n x n block of A (stride lda)
__global__ void k_permute_cols(const double* __restrict__ A, int64_t lda, double* __restrict__ out,
                               int64_t n, const int* __restrict__ sigma) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < n) out[i * n + j] = A[i * lda + sigma[j]];
}

hipError_t launch_permute_cols(hipStream_t s, const double* A, int64_t lda, double* out, int64_t n,
                               const int* sigma) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n), block(256);
  k_permute_cols<<<grid, block, 0, s>>>(A, lda, out, n, sigma);
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
