// Batched extraction and inversion of the local space-time Jacobians J_T
// (Section 4.2: J_T is the submatrix of the level matrix on the cell's DoFs;
// Section 4.3: the inverses are pre-computed once per Jacobian and stored).
//
// One workgroup per cell: the n_loc x n_loc block is gathered from the
// block-sparse level matrix (binary search of each cell pair in its block
// row), inverted in place by Gauss-Jordan elimination with partial pivoting
// in FP64, and written out column-major, FP64 or FP32, keeping either every
// row or only the rows of the DoFs the cell owns.
// Blocks that fit are held in LDS; larger ones (3d, k >= 1) live in a global
// scratch slot per persistent workgroup, with the pivot row/column in LDS.
// Cell-local order inside the kernel is (alpha, l) -> alpha*B + l, matching
// the time-inner global layout.
#include "stv_internal.h"

namespace stv {

__device__ __forceinline__ int32_t find_block(const int32_t* __restrict__ col, int32_t lo,
                                              int32_t hi, int32_t key) {
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

template <int B>
__device__ void extract_block(double* A, int lda, const int32_t* __restrict__ rowptr,
                              const int32_t* __restrict__ col, const double* __restrict__ val,
                              const int32_t* __restrict__ sd, int n_ls) {
  const int npairs = n_ls * n_ls;
  for (int pr = threadIdx.x; pr < npairs; pr += blockDim.x) {
    const int a = pr / n_ls;
    const int bb = pr - a * n_ls;
    const int32_t row = sd[a];
    const int32_t pos = find_block(col, rowptr[row], rowptr[row + 1], sd[bb]);
    const double* blk = val + (int64_t)pos * (B * B);
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int l = 0; l < B; ++l) A[(int64_t)(a * B + i) * lda + bb * B + l] = blk[i * B + l];
  }
}

// In-place Gauss-Jordan inversion with partial pivoting of the n x n row-major
// matrix A (leading dimension lda).  Each step: every wavefront finds the
// pivot row r of column p redundantly (largest magnitude, lowest index on
// ties); the pivot row, old row p and column p are copied to LDS; then every
// element is rewritten from its own old value and the copies only, so no
// element is read by one thread and written by another within a step.
// pivrow[p] = r is recorded; the column order is restored at the store.
__device__ void gj_invert(double* A, int lda, int n, double* prow, double* trow, double* pcol,
                          int* pivrow, int* sing) {
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int nw = nt >> 6;
  for (int p = 0; p < n; ++p) {
    double best = -1.0;
    int bi = 0x7fffffff;
    for (int i = p + lane; i < n; i += 64) {
      const double v = fabs(A[(int64_t)i * lda + p]);
      if (v > best) { best = v; bi = i; }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
      const double ob = __shfl_xor(best, off, 64);
      const int oi = __shfl_xor(bi, off, 64);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    const int r = (bi < n) ? bi : p;   // no finite candidate (NaN column): flagged below
    for (int j = tid; j < n; j += nt) {
      prow[j] = A[(int64_t)r * lda + j];
      trow[j] = A[(int64_t)p * lda + j];
      pcol[j] = A[(int64_t)j * lda + p];
    }
    if (tid == 0) {
      pivrow[p] = r;
      if (bi >= n) *sing = 1;
    }
    __syncthreads();
    const double piv = prow[p];
    if (tid == 0 && !(piv != 0.0)) *sing = 1;
    const double ipiv = (piv != 0.0) ? 1.0 / piv : 0.0;
    for (int i = wv; i < n; i += nw) {
      double* Ai = A + (int64_t)i * lda;
      if (i == p) {
        for (int j = lane; j < n; j += 64) Ai[j] = (j == p) ? ipiv : prow[j] * ipiv;
      } else {
        const double f = ((i == r) ? pcol[p] : pcol[i]) * ipiv;
        const double* src = (i == r) ? trow : Ai;
        for (int j = lane; j < n; j += 64) Ai[j] = (j == p) ? -f : fma(-f, prow[j], src[j]);
      }
    }
    __syncthreads();
  }
}

// The row swaps of the elimination act as column swaps on the inverse,
// applied in reverse step order: inverse(:, j) = A(:, sigma[j]).
__device__ void gj_sigma(int* sigma, const int* pivrow, int n) {
  if (threadIdx.x == 0) {
    for (int j = 0; j < n; ++j) sigma[j] = j;
    for (int p = n - 1; p >= 0; --p) {
      const int q = pivrow[p];
      const int t = sigma[p];
      sigma[p] = sigma[q];
      sigma[q] = t;
    }
  }
  __syncthreads();
}

template <int B>
__device__ void store_inverse(const double* A, int lda, int n, const int* sigma,
                              const uint8_t* __restrict__ own_loc, int o0, int n_own, int full,
                              void* store, int64_t off, int fp32) {
  const int R = full ? n : n_own * B;
  const int64_t total = (int64_t)R * n;
  for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
    const int j = (int)(e / R);
    const int o = (int)(e - (int64_t)j * R);
    int i;
    if (full) {
      i = o;
    } else {
      const int os = o / B;
      i = own_loc[o0 + os] * B + (o - os * B);
    }
    const double v = A[(int64_t)i * lda + sigma[j]];
    if (fp32) ((float*)store)[off + e] = (float)v;
    else ((double*)store)[off + e] = v;
  }
}

template <int B>
__global__ void __launch_bounds__(256) k_inverse_lds(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ csd, int n_ls,
    const int32_t* __restrict__ own_ptr, const uint8_t* __restrict__ own_loc, int full,
    const int64_t* __restrict__ inv_off, void* store, int fp32, uint8_t* status) {
  extern __shared__ double sm[];
  __shared__ int sing;
  const int n = n_ls * B;
  const int lda = n | 1;
  double* A = sm;
  double* prow = A + (size_t)n * lda;
  double* trow = prow + n;
  double* pcol = trow + n;
  int* pivrow = (int*)(pcol + n);
  int* sigma = pivrow + n;
  const int T = blockIdx.x;
  if (threadIdx.x == 0) sing = 0;
  extract_block<B>(A, lda, rowptr, col, val, csd + (int64_t)T * n_ls, n_ls);
  __syncthreads();
  gj_invert(A, lda, n, prow, trow, pcol, pivrow, &sing);
  gj_sigma(sigma, pivrow, n);
  const int o0 = own_ptr[T];
  store_inverse<B>(A, lda, n, sigma, own_loc, o0, own_ptr[T + 1] - o0, full, store, inv_off[T],
                   fp32);
  if (threadIdx.x == 0) status[T] = (uint8_t)sing;
}

template <int B>
__global__ void __launch_bounds__(256) k_inverse_global(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ csd, int n_ls, int n_cells,
    const int32_t* __restrict__ own_ptr, const uint8_t* __restrict__ own_loc, int full,
    const int64_t* __restrict__ inv_off, void* store, int fp32, uint8_t* status,
    double* gscratch) {
  extern __shared__ double sm[];
  __shared__ int sing;
  const int n = n_ls * B;
  const int lda = n | 1;
  double* A = gscratch + (int64_t)blockIdx.x * n * lda;
  double* prow = sm;
  double* trow = prow + n;
  double* pcol = trow + n;
  int* pivrow = (int*)(pcol + n);
  int* sigma = pivrow + n;
  for (int T = blockIdx.x; T < n_cells; T += gridDim.x) {
    if (threadIdx.x == 0) sing = 0;
    extract_block<B>(A, lda, rowptr, col, val, csd + (int64_t)T * n_ls, n_ls);
    __threadfence_block();
    __syncthreads();
    gj_invert(A, lda, n, prow, trow, pcol, pivrow, &sing);
    gj_sigma(sigma, pivrow, n);
    const int o0 = own_ptr[T];
    store_inverse<B>(A, lda, n, sigma, own_loc, o0, own_ptr[T + 1] - o0, full, store,
                     inv_off[T], fp32);
    if (threadIdx.x == 0) status[T] = (uint8_t)sing;
    __syncthreads();
  }
}

static size_t lds_bytes_resident(int n) {
  const int lda = n | 1;
  return sizeof(double) * ((size_t)n * lda + 3 * (size_t)n) + sizeof(int) * 2 * (size_t)n;
}

// Largest LDS footprint used by one workgroup (the device offers 160 KiB).
constexpr size_t kLdsBudget = 150 * 1024;

bool inverse_fits_lds(int n) { return lds_bytes_resident(n) <= kLdsBudget; }

template <int B>
static hipError_t inverse_b(hipStream_t s, const DevLevel& L, int fp32, int full,
                            uint8_t* status, double* gscratch, int n_slots) {
  const int n = L.n_ls * B;
  if (inverse_fits_lds(n)) {
    const size_t shm = lds_bytes_resident(n);
    hipError_t e = hipFuncSetAttribute((const void*)k_inverse_lds<B>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    k_inverse_lds<B><<<L.n_cells, 256, shm, s>>>(L.rowptr, L.col, L.val, L.cell_sdofs, L.n_ls,
                                                 L.own_ptr, L.own_loc, full, L.inv_off,
                                                 L.inv_store, fp32, status);
  } else {
    const size_t shm = sizeof(double) * 3 * (size_t)n + sizeof(int) * 2 * (size_t)n;
    k_inverse_global<B><<<n_slots, 256, shm, s>>>(L.rowptr, L.col, L.val, L.cell_sdofs, L.n_ls,
                                                  L.n_cells, L.own_ptr, L.own_loc, full,
                                                  L.inv_off, L.inv_store, fp32, status,
                                                  gscratch);
  }
  return hipGetLastError();
}

hipError_t launch_cell_inverses(hipStream_t s, int b, const DevLevel& L, int fp32, int full,
                                uint8_t* status, double* gscratch, int n_slots) {
  switch (b) {
    case 1: return inverse_b<1>(s, L, fp32, full, status, gscratch, n_slots);
    case 2: return inverse_b<2>(s, L, fp32, full, status, gscratch, n_slots);
    case 3: return inverse_b<3>(s, L, fp32, full, status, gscratch, n_slots);
    case 4: return inverse_b<4>(s, L, fp32, full, status, gscratch, n_slots);
  }
  return hipErrorInvalidValue;
}

}  // namespace stv
