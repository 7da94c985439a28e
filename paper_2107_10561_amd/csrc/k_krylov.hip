// FP64 vector kernels of flexible GMRES: several dot products against one
// vector in a single pass (classical Gram-Schmidt, applied twice), the
// matching multi-axpy, and normalisation.  A vector may hold several
// independent instances (segments): every reduction and update is done per
// segment with that segment's scalars.  Reductions use a fixed number of
// partial sums folded in a fixed order, so results are bitwise repeatable.
#include "stv_internal.h"

namespace stv {

constexpr int kGroup = 8;

int seg_blocks(const Segs& g) {
  // kDotBlocks shared among the instances, at least 4 each; for a batch also
  // enough that a thread of the longest instance takes about 16 elements
  // (instances of uneven length otherwise leave the longest ones a few
  // blocks)
  const int per = kDotBlocks / (g.nseg > 0 ? g.nseg : 1);
  int nb = per < 4 ? 4 : per;
  if (g.nseg > 1) {
    const int64_t by_len = (g.max_seg + 16 * 256 - 1) / (16 * 256);
    if (by_len > nb) nb = (int)(by_len < 65535 ? by_len : 65535);
  }
  return nb;
}

// partial[(z*nblk + blk)*kGroup + k] = sum over this block's slice of segment
// z of V_k . w
template <int NV>
__global__ void __launch_bounds__(256) k_multidot(const double* __restrict__ V, int64_t n,
                                                  const double* __restrict__ w,
                                                  const int64_t* __restrict__ seg,
                                                  double* __restrict__ partial) {
  __shared__ double red[NV][4];
  const int z = blockIdx.y;
  const int64_t lo = seg[z], hi = seg[z + 1];
  double acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) acc[k] = 0.0;
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
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
    partial[((int64_t)z * gridDim.x + blockIdx.x) * kGroup + k] =
        (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

// out[z*ostride + k] = sum_blk partial[(z*nblk + blk)*kGroup + k], pairwise in
// a fixed order.
__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ partial,
                                                         int nblk, int nv,
                                                         double* __restrict__ out,
                                                         int64_t ostride) {
  __shared__ double red[4];
  const int k = blockIdx.x, z = blockIdx.y;
  if (k >= nv) return;
  const double* pz = partial + (int64_t)z * nblk * kGroup;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) acc += pz[(int64_t)b * kGroup + k];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[(int64_t)z * ostride + k] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_multidot(hipStream_t s, const double* V, int m, const double* w, int64_t n,
                           const Segs& g, double* partial, double* out, int64_t ostride) {
  const int nblk = seg_blocks(g);
  for (int k0 = 0; k0 < m; k0 += kGroup) {
    const int nv = (m - k0) < kGroup ? (m - k0) : kGroup;
    const double* Vk = V + (int64_t)k0 * n;
    dim3 grid((unsigned)nblk, (unsigned)g.nseg);
    switch (nv) {
      case 1: k_multidot<1><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      case 2: k_multidot<2><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      case 3: k_multidot<3><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      case 4: k_multidot<4><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      case 5: k_multidot<5><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      case 6: k_multidot<6><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      case 7: k_multidot<7><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
      default: k_multidot<8><<<grid, 256, 0, s>>>(Vk, n, w, g.seg, partial); break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_reduce_partials<<<dim3((unsigned)nv, (unsigned)g.nseg), 256, 0, s>>>(partial, nblk, nv,
                                                                          out + k0, ostride);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// w += sign * sum_k coef[z*cstride + k] V_k on segment z
__global__ void __launch_bounds__(256) k_multiaxpy(const double* __restrict__ V, int m,
                                                   const double* __restrict__ coef,
                                                   int64_t cstride, double sign,
                                                   double* __restrict__ w, int64_t n,
                                                   const int64_t* __restrict__ seg) {
  const int z = blockIdx.y;
  const int64_t i = seg[z] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= seg[z + 1]) return;
  const double* cz = coef + (int64_t)z * cstride;
  double acc = 0.0;
  for (int k = 0; k < m; ++k) acc = fma(cz[k], V[(int64_t)k * n + i], acc);
  w[i] = fma(sign, acc, w[i]);
}

hipError_t launch_multiaxpy(hipStream_t s, const double* V, int m, const double* coef,
                            int64_t cstride, double sign, double* w, int64_t n, const Segs& g) {
  if (m <= 0) return hipSuccess;
  dim3 grid((unsigned)((g.max_seg + 255) / 256), (unsigned)g.nseg);
  k_multiaxpy<<<grid, 256, 0, s>>>(V, m, coef, cstride, sign, w, n, g.seg);
  return hipGetLastError();
}

// The update of one Gram-Schmidt pass fused with the products of the next
// (one read of V instead of two): on segment z
//   w <- w + sign * sum_k coef[z*cstride + k] V_k   (k < NV),
// then, with the updated w, the partial sums of V_k . w as k_multidot writes
// them (same blocks, same order of operations: the results equal those of
// k_multiaxpy followed by k_multidot).
template <int NV>
__global__ void __launch_bounds__(256) k_multiaxpy_dot(const double* __restrict__ V, int64_t n,
                                                       const double* __restrict__ coef,
                                                       int64_t cstride, double sign,
                                                       double* __restrict__ w,
                                                       const int64_t* __restrict__ seg,
                                                       double* __restrict__ partial) {
  __shared__ double red[NV][4];
  const int z = blockIdx.y;
  const int64_t lo = seg[z], hi = seg[z + 1];
  const double* cz = coef + (int64_t)z * cstride;
  double c[NV], acc[NV];
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    c[k] = cz[k];
    acc[k] = 0.0;
  }
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = V[(int64_t)k * n + i];
    double a = 0.0;
#pragma unroll
    for (int k = 0; k < NV; ++k) a = fma(c[k], v[k], a);
    const double wi = fma(sign, a, w[i]);
    w[i] = wi;
#pragma unroll
    for (int k = 0; k < NV; ++k) acc[k] = fma(v[k], wi, acc[k]);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) {
    double t = acc[k];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) red[k][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    const int k = threadIdx.x;
    partial[((int64_t)z * gridDim.x + blockIdx.x) * kGroup + k] =
        (red[k][0] + red[k][1]) + (red[k][2] + red[k][3]);
  }
}

// The second pass's update fused with the squared norm of its result:
// w <- w + sign * sum_k coef[z*cstride + k] V_k (any m), and the partial sums
// of w . w (slot 0), as k_multiaxpy followed by k_multidot of w with itself.
__global__ void __launch_bounds__(256) k_multiaxpy_nrm(const double* __restrict__ V, int m,
                                                       int64_t n, const double* __restrict__ coef,
                                                       int64_t cstride, double sign,
                                                       double* __restrict__ w,
                                                       const int64_t* __restrict__ seg,
                                                       double* __restrict__ partial) {
  __shared__ double red[4];
  const int z = blockIdx.y;
  const int64_t lo = seg[z], hi = seg[z + 1];
  const double* cz = coef + (int64_t)z * cstride;
  double acc = 0.0;
  for (int64_t i = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < hi;
       i += (int64_t)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int k = 0; k < m; ++k) a = fma(cz[k], V[(int64_t)k * n + i], a);
    const double wi = fma(sign, a, w[i]);
    w[i] = wi;
    acc = fma(wi, wi, acc);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) red[wv] = acc;
  __syncthreads();
  if (threadIdx.x == 0)
    partial[((int64_t)z * gridDim.x + blockIdx.x) * kGroup] = (red[0] + red[1]) + (red[2] + red[3]);
}

hipError_t launch_multiaxpy_dot(hipStream_t s, const double* V, int m, const double* coef,
                                int64_t cstride, double sign, double* w, int64_t n,
                                const Segs& g, double* partial, double* out, int64_t ostride) {
  if (m < 1 || m > kGroup) return hipErrorInvalidValue;
  const int nblk = seg_blocks(g);
  dim3 grid((unsigned)nblk, (unsigned)g.nseg);
#define STV_AXD(NN) k_multiaxpy_dot<NN><<<grid, 256, 0, s>>>(V, n, coef, cstride, sign, w, g.seg, partial)
  switch (m) {
    case 1: STV_AXD(1); break;
    case 2: STV_AXD(2); break;
    case 3: STV_AXD(3); break;
    case 4: STV_AXD(4); break;
    case 5: STV_AXD(5); break;
    case 6: STV_AXD(6); break;
    case 7: STV_AXD(7); break;
    default: STV_AXD(8); break;
  }
#undef STV_AXD
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_reduce_partials<<<dim3((unsigned)m, (unsigned)g.nseg), 256, 0, s>>>(partial, nblk, m, out,
                                                                        ostride);
  return hipGetLastError();
}

hipError_t launch_multiaxpy_nrm(hipStream_t s, const double* V, int m, const double* coef,
                                int64_t cstride, double sign, double* w, int64_t n,
                                const Segs& g, double* partial, double* out, int64_t ostride) {
  if (m < 1) return hipErrorInvalidValue;
  const int nblk = seg_blocks(g);
  k_multiaxpy_nrm<<<dim3((unsigned)nblk, (unsigned)g.nseg), 256, 0, s>>>(V, m, n, coef, cstride,
                                                                        sign, w, g.seg, partial);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_reduce_partials<<<dim3(1u, (unsigned)g.nseg), 256, 0, s>>>(partial, nblk, 1, out, ostride);
  return hipGetLastError();
}

// v = w / sqrt(nrm2[z*nstride]) on segment z (0 where the norm is 0)
__global__ void k_scale_by_norm(const double* __restrict__ w, const double* __restrict__ nrm2,
                                int64_t nstride, double* __restrict__ v,
                                const int64_t* __restrict__ seg) {
  const int z = blockIdx.y;
  const int64_t i = seg[z] + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= seg[z + 1]) return;
  const double nr = sqrt(nrm2[(int64_t)z * nstride]);
  v[i] = nr > 0.0 ? w[i] / nr : 0.0;
}

hipError_t launch_scale_by_norm(hipStream_t s, const double* w, const double* nrm2,
                                int64_t nstride, double* v, const Segs& g) {
  dim3 grid((unsigned)((g.max_seg + 255) / 256), (unsigned)g.nseg);
  k_scale_by_norm<<<grid, 256, 0, s>>>(w, nrm2, nstride, v, g.seg);
  return hipGetLastError();
}

}  // namespace stv
