// FP64 vector kernels of flexible GMRES: several dot products against one
// vector in a single pass (classical Gram-Schmidt, applied twice), the
// matching multi-axpy, and normalisation.  Reductions use a fixed number of
// partial sums folded in a fixed order, so results are bitwise repeatable.
#include "stv_internal.h"

namespace stv {

constexpr int kGroup = 8;

// partial[blk*kGroup + k] = sum over this block's grid-stride slice of V_k . w
template <int NV>
__global__ void __launch_bounds__(256) k_multidot(const double* __restrict__ V, int64_t n,
                                                  const double* __restrict__ w,
                                                  double* __restrict__ partial) {
  __shared__ double red[NV][4];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double wi = w[i];
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = fma(V[(int64_t)k * n + i], wi, acc[k]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double v = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) red[k][wv] = v;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    partial[(int64_t)blockIdx.x * kGroup + k] = (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

// out[k] = sum_blk partial[blk*kGroup + k], pairwise in a fixed order.
__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partial,
                                                         int nblk, int nv,
                                                         double* __restrict__ out) {
  __shared__ double red[4];
  const int k = blockIdx.x;
  if (k >= nv) return;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += partial[(int64_t)b * kGroup + k];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[k] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_multidot(hipStream_t s, const double* V, int m, const double* w, int64_t n,
                           double* partial, double* out) {
  for (int k0 = 0; k0 < m; k0 += kGroup) {
    const int nv = (m - k0) < kGroup ? (m - k0) : kGroup;
    const double* Vk = V + (int64_t)k0 * n;
    const int nblk = kDotBlocks;
    switch (nv) {
      case 1: k_multidot<1><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      case 2: k_multidot<2><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      case 3: k_multidot<3><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      case 4: k_multidot<4><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      case 5: k_multidot<5><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      case 6: k_multidot<6><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      case 7: k_multidot<7><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
      default: k_multidot<8><<<nblk, 256, 0, s>>>(Vk, n, w, partial); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reduce_partials<<<nv, 256, 0, s>>>(partial, nblk, nv, out + k0);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// w += sign * sum_k coef[k] V_k
__global__ void __launch_bounds__(256) k_multiaxpy(const double* __restrict__ V, int m,
                                                   const double* __restrict__ coef, double sign,
                                                   double* __restrict__ w, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int k = 0; k < m; ++k) acc = fma(coef[k], V[(int64_t)k * n + i], acc);
  w[i] = fma(sign, acc, w[i]);
}

hipError_t launch_multiaxpy(hipStream_t s, const double* V, int m, const double* coef,
                            double sign, double* w, int64_t n) {
  if (m <= 0) return hipSuccess;
  k_multiaxpy<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(V, m, coef, sign, w, n);
  return hipGetLastError();
}

// v = w / sqrt(nrm2[0])
__global__ void k_scale_by_norm(const double* __restrict__ w, const double* __restrict__ nrm2,
                                double* __restrict__ v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double nr = sqrt(nrm2[0]);
  v[i] = nr > 0.0 ? w[i] / nr : 0.0;
}

hipError_t launch_scale_by_norm(hipStream_t s, const double* w, const double* nrm2, double* v,
                                int64_t n) {
  k_scale_by_norm<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(w, nrm2, v, n);
  return hipGetLastError();
}

}  // namespace stv
