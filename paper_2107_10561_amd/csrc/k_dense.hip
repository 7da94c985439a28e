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

// Blocked Gauss-Jordan inversion with partial pivoting and no row
// interchanges: the pivot of step p is the largest-magnitude entry of column
// p among the rows not yet used as pivots (lowest row on ties), recorded as
// rpiv[p]; at the end A^-1(p, j) = S(rpiv[p], rinv[j]) for the in-place
// result S (rinv the inverse permutation).
// Panel of NB columns [p0, p0+NB), kept in a contiguous row-major buffer
// (n x NB): one 512-thread workgroup holds it in registers (thread t owns
// rows t + 512 m) and eliminates it.  The panel columns then hold the columns
// rpiv[p0..] of the accumulated elimination matrix E; every other column j
// (earlier panels included) is brought up to date at once by the rank-NB
// update  A(:, j) += (E - I)(:, rpiv[p0+t]) * A(rpiv[p0+t], j)  (pivot rows
// read before it), which also writes the eliminated panel back into A and
// copies the next panel's updated columns into the other panel buffer.
// rpiv[p] = -1 marks a step without a nonzero finite pivot (singular).
template <int RPT, int NB>
__global__ void __launch_bounds__(512) k_gj_panel(double* __restrict__ pbuf, int64_t n, int p0,
                                                  int* __restrict__ rpiv,
                                                  uint8_t* __restrict__ used) {
  // per step, each wavefront publishes its best candidate (magnitude, row)
  // together with that row's panel values; one barrier, then every thread
  // picks the winner among the 8 candidates (double-buffered by step parity)
  __shared__ double wbest[2][8];
  __shared__ int widx[2][8];
  __shared__ double wrow[2][8][NB];
  __shared__ int rloc[NB];     // pivot records, written to global memory once at the end
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  double P[RPT][NB];
  unsigned umask = 0;   // bit m: row tid + 512 m already used as a pivot
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const int64_t i = tid + 512 * m;
#pragma unroll
    for (int t = 0; t < NB; ++t) P[m][t] = (i < n) ? pbuf[i * NB + t] : 0.0;
    if (i >= n || used[i]) umask |= 1u << m;
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int par = t & 1;
    double best = -1.0;
    int bi = 0x7fffffff;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const double v = fabs(P[m][t]);
      if (!(umask & (1u << m)) && v > best) { best = v; bi = tid + 512 * m; }
    }
    // wave argmax (largest magnitude, lowest row on ties)
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    bi = __builtin_amdgcn_readfirstlane(bi);   // identical in every lane
    if (lane == 0) { wbest[par][wv] = best; widx[par][wv] = bi; }
    if (bi < 0x7fffffff) {
      const int mo = bi / 512;                 // wave-uniform: one scalar-branched write
#pragma unroll
      for (int m = 0; m < RPT; ++m)
        if (m == mo && tid == bi - 512 * m) {
#pragma unroll
          for (int c = 0; c < NB; ++c) wrow[par][wv][c] = P[m][c];
        }
    }
    __syncthreads();
    double mx = wbest[par][0];
    int cand = widx[par][0];
    int win = 0;
#pragma unroll
    for (int w2 = 1; w2 < 8; ++w2) {
      const double ob = wbest[par][w2];
      const int oi = widx[par][w2];
      if (ob > mx || (ob == mx && oi < cand)) { mx = ob; cand = oi; win = w2; }
    }
    cand = __builtin_amdgcn_readfirstlane(cand);
    win = __builtin_amdgcn_readfirstlane(win);
    const bool ok = (cand < n) && (mx > 0.0);
    if (tid == 0) rloc[t] = ok ? cand : -1;
    if (cand >= n) continue;  // uniform: no candidate row at all (singular, flagged)
    const int r = cand;
    double pr[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) pr[c] = wrow[par][win][c];
    const double pv = pr[t];
    const double ipiv = (pv != 0.0) ? 1.0 / pv : 0.0;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const bool isr = (tid + 512 * m == r);
      if (isr) umask |= 1u << m;
      // pivot row: (src 0, factor -1/piv); other rows: (own value, factor a_it/piv)
      const double f = isr ? -ipiv : P[m][t] * ipiv;
#pragma unroll
      for (int c = 0; c < NB; ++c)
        P[m][c] = (c == t) ? (isr ? ipiv : -f) : fma(-f, pr[c], isr ? 0.0 : P[m][c]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const int64_t i = tid + 512 * m;
    if (i < n) {
#pragma unroll
      for (int t = 0; t < NB; ++t) pbuf[i * NB + t] = P[m][t];
    }
  }
  if (tid < NB) {
    const int r = rloc[tid];
    rpiv[p0 + tid] = r;
    if (r >= 0) used[r] = 1;
  }
}

// First panel: columns [0, NB) of A into the row-major panel buffer.
__global__ void k_gj_load_panel(const double* __restrict__ A, int64_t n, int nb,
                                double* __restrict__ pbuf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nb) return;
  const int64_t i = e / nb;
  pbuf[e] = A[i * n + (e - i * nb)];
}

// Pivot rows of the panel as they were before its update (right factor).
__global__ void k_gj_gather_rows(const double* __restrict__ A, int64_t n, int p0, int nb,
                                 const int* __restrict__ rpiv, double* __restrict__ Bbuf) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  for (int t = 0; t < nb; ++t) {
    const int r = rpiv[p0 + t];
    Bbuf[(int64_t)t * n + j] = r >= 0 ? A[(int64_t)r * n + j] : 0.0;
  }
}

// A(i, j) += sum_t (P(i, t) - [i == rpiv[p0+t]]) * Bbuf(t, j) for j outside the
// panel, A(i, p0+t) = P(i, t) inside it, and the updated columns of the next
// panel are copied to pnext.  A workgroup handles 16 rows x 256 columns: the
// 16 x NB left factor is staged in LDS, each thread keeps its column of the
// right factor in registers, and the rows of A are read and written fully
// coalesced.
template <int NB>
__global__ void __launch_bounds__(256) k_gj_rank_update(double* __restrict__ A, int64_t n, int p0,
                                                        const int* __restrict__ rpiv,
                                                        const double* __restrict__ pcur,
                                                        const double* __restrict__ Bbuf,
                                                        double* __restrict__ pnext) {
  __shared__ double W[16][NB];
  const int64_t i0 = (int64_t)blockIdx.y * 16;
  for (int e = threadIdx.x; e < 16 * NB; e += 256) {
    const int di = e / NB, t = e - di * NB;
    const int64_t i = i0 + di;
    W[di][t] = (i < n) ? pcur[i * NB + t] - ((i == rpiv[p0 + t]) ? 1.0 : 0.0) : 0.0;
  }
  __syncthreads();
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  if (j >= p0 && j < p0 + NB) {
    for (int di = 0; di < 16; ++di) {
      const int64_t i = i0 + di;
      if (i >= n) break;
      A[i * n + j] = pcur[i * NB + (j - p0)];
    }
    return;
  }
  double bcol[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) bcol[t] = Bbuf[(int64_t)t * n + j];
  const bool nxt = (j >= p0 + NB && j < p0 + 2 * NB);
#pragma unroll 4
  for (int di = 0; di < 16; ++di) {
    const int64_t i = i0 + di;
    if (i >= n) break;
    double acc = A[i * n + j];
#pragma unroll
    for (int t = 0; t < NB; ++t) acc = fma(W[di][t], bcol[t], acc);
    A[i * n + j] = acc;
    if (nxt) pnext[i * NB + (j - p0 - NB)] = acc;
  }
}

template <int RPT, int NB>
static hipError_t gj_blocked(hipStream_t s, double* A, int64_t n, int* rpiv, uint8_t* used,
                             double* Bbuf, double* pbuf) {
  double* pb[2] = {pbuf, pbuf + n * NB};
  k_gj_load_panel<<<(unsigned)((n * NB + 255) / 256), 256, 0, s>>>(A, n, NB, pb[0]);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  int cur = 0;
  for (int64_t p0 = 0; p0 < n; p0 += NB, cur ^= 1) {
    k_gj_panel<RPT, NB><<<1, 512, 0, s>>>(pb[cur], n, (int)p0, rpiv, used);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gj_gather_rows<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(A, n, (int)p0, NB, rpiv, Bbuf);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((n + 15) / 16));
    k_gj_rank_update<NB><<<grid, 256, 0, s>>>(A, n, (int)p0, rpiv, pb[cur], Bbuf, pb[cur ^ 1]);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// n must be a multiple of the panel width chosen here (the caller pads).
int gj_panel_width(int64_t n) {
  if (n <= 2560) return 12;
  if (n <= 5120) return 8;
  return 4;
}

hipError_t launch_gj_blocked(hipStream_t s, double* A, int64_t n, int* rpiv, uint8_t* used,
                             double* Bbuf, double* pbuf) {
  if (n <= 2560) return gj_blocked<5, 12>(s, A, n, rpiv, used, Bbuf, pbuf);
  if (n <= 5120) return gj_blocked<10, 8>(s, A, n, rpiv, used, Bbuf, pbuf);
  if (n <= 12288) return gj_blocked<24, 4>(s, A, n, rpiv, used, Bbuf, pbuf);
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

// out (n x n, compact): out(i, j) = S(rpiv[i], rinv[j]) from the in-place
// result S (stride lda), which is the inverse of the original matrix.
__global__ void k_gj_unpermute(const double* __restrict__ S, int64_t lda, double* __restrict__ out,
                               int64_t n, const int* __restrict__ rpiv,
                               const int* __restrict__ rinv) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (j < n) out[i * n + j] = S[(int64_t)rpiv[i] * lda + rinv[j]];
}

hipError_t launch_gj_unpermute(hipStream_t s, const double* S, int64_t lda, double* out, int64_t n,
                               const int* rpiv, const int* rinv) {
  dim3 grid((unsigned)((n + 255) / 256), (unsigned)n), block(256);
  k_gj_unpermute<<<grid, block, 0, s>>>(S, lda, out, n, rpiv, rinv);
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
