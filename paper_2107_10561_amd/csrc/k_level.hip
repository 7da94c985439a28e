// Level kernels of the V-cycle: the block-sparse level residual, the Vanka
// cell sweep and the grid transfers.  Vectors are FP64 and time-inner
// (x[s*B + l], B = k+1 temporal DoFs per spatial DoF).
#include "stv_internal.h"
#include "wave.h"

namespace stv {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Partner value for lane ^ M inside a row of 16 lanes (M <= 8): DPP lane
// permutations (xor 1, xor 2 as quad permutations, xor 8 as a rotation of the
// row by 8) and, for xor 4, a swizzle in bit-mask mode.  Every source lane
// is inside the row, so the permutations need no old value.
template <int M>
__device__ __forceinline__ int xor_i32(int v) {
  static_assert(M == 1 || M == 2 || M == 4 || M == 8, "inside a row");
  if constexpr (M == 1) return __builtin_amdgcn_mov_dpp(v, 0xB1, 0xF, 0xF, true);   // quad_perm [1,0,3,2]
  if constexpr (M == 2) return __builtin_amdgcn_mov_dpp(v, 0x4E, 0xF, 0xF, true);   // quad_perm [2,3,0,1]
  if constexpr (M == 8) return __builtin_amdgcn_mov_dpp(v, 0x128, 0xF, 0xF, true);  // row_ror:8
  return __builtin_amdgcn_ds_swizzle(v, 0x101F);                                   // xor 4
}

template <int M>
__device__ __forceinline__ double xor_lane(double v) {
  const int lo = xor_i32<M>(__double2loint(v));
  const int hi = xor_i32<M>(__double2hiint(v));
  return __hiloint2double(hi, lo);
}

template <int M>
__device__ __forceinline__ float xor_lane(float v) {
  return __int_as_float(xor_i32<M>(__float_as_int(v)));
}

// x, y <- the lanes with bit M clear keep x and receive y's values of the
// partner lanes (lane ^ M) in y, and vice versa: one v_permlane{16,32}_swap
// per 32-bit word (M = 16: odd rows of x with even rows of y; M = 32: upper
// half of x with lower half of y).  Afterwards x + y is, in every lane, its
// own kept value plus its partner's sent one.
template <int M>
__device__ __forceinline__ void swap_words(unsigned& x, unsigned& y) {
  static_assert(M == 16 || M == 32, "across rows");
  if constexpr (M == 32) {
    const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
    x = r[0];
    y = r[1];
  }
}

template <int M>
__device__ __forceinline__ void swap_halves(double& x, double& y) {
  unsigned xl = (unsigned)__double2loint(x), xh = (unsigned)__double2hiint(x);
  unsigned yl = (unsigned)__double2loint(y), yh = (unsigned)__double2hiint(y);
  swap_words<M>(xl, yl);
  swap_words<M>(xh, yh);
  x = __hiloint2double((int)xh, (int)xl);
  y = __hiloint2double((int)yh, (int)yl);
}

template <int M>
__device__ __forceinline__ void swap_halves(float& x, float& y) {
  unsigned xw = __float_as_uint(x), yw = __float_as_uint(y);
  swap_words<M>(xw, yw);
  x = __uint_as_float(xw);
  y = __uint_as_float(yw);
}

// Transpose-reduce: NV (a power of two, 2..64) per-lane partial sums are
// summed over the wavefront; afterwards the lanes L with L / (64 / NV) == v
// hold the total of value v.  Each halving step exchanges half of the values
// with the partner lane, so the cost is about NV + log2(64 / NV) shuffles.
template <int CNT, int M, int NV>
__device__ __forceinline__ void fold_level(double (&p)[NV], int lane) {
  if constexpr (CNT > 1) {
    const bool hi = lane & M;
#pragma unroll
    for (int t = 0; t < CNT / 2; ++t) {
      const double keep = hi ? p[t + CNT / 2] : p[t];
      const double send = hi ? p[t] : p[t + CNT / 2];
      p[t] = keep + __shfl_xor(send, M, 64);
    }
    fold_level<CNT / 2, M / 2, NV>(p, lane);
  }
}

template <int NV>
__device__ __forceinline__ double fold(double (&p)[NV], int lane) {
  fold_level<NV, 32, NV>(p, lane);
  double u = p[0];
#pragma unroll
  for (int m = 32 / NV; m >= 1; m >>= 1) u += __shfl_xor(u, m, 64);
  return u;
}

// The same transpose-reduce (FP64 or FP32 values) with the exchanges done
// without LDS: across rows by lane-half swaps, inside a row by DPP and
// swizzle.  Every sum takes the same two operands as in fold, so the FP64
// results are identical.  LIVE marks the values that can be nonzero (bit v
// for value v): a pair of slots that are both known to be zero is not
// exchanged, which saves the padding of outputs per row up to a power of two.
template <int M, unsigned long long NEXT, int T, int H, int NV, typename V>
__device__ __forceinline__ void fold_swap_pairs(V (&p)[NV], int lane) {
  if constexpr (T < H) {
    if constexpr (((NEXT >> T) & 1ull) == 0) {
      p[T] = V(0);
    } else if constexpr (M >= 16) {
      V x = p[T], y = p[T + H];
      swap_halves<M>(x, y);
      p[T] = x + y;
    } else {
      const bool hi = lane & M;
      const V keep = hi ? p[T + H] : p[T];
      const V send = hi ? p[T] : p[T + H];
      p[T] = keep + xor_lane<M>(send);
    }
    fold_swap_pairs<M, NEXT, T + 1, H, NV>(p, lane);
  }
}

template <int CNT, int M, int NV, unsigned long long LIVE, typename V>
__device__ __forceinline__ void fold_swap_level(V (&p)[NV], int lane) {
  if constexpr (CNT > 1) {
    constexpr int H = CNT / 2;
    constexpr unsigned long long NEXT = (LIVE | (LIVE >> H)) & ((1ull << H) - 1ull);
    fold_swap_pairs<M, NEXT, 0, H, NV>(p, lane);
    fold_swap_level<H, M / 2, NV, NEXT>(p, lane);
  }
}

template <int NV, unsigned long long LIVE = (NV >= 64 ? ~0ull : (1ull << NV) - 1ull),
          typename V>
__device__ __forceinline__ V fold_swap(V (&p)[NV], int lane) {
  static_assert(NV >= 4 && NV <= 64, "the final exchanges stay inside a row");
  fold_swap_level<NV, 32, NV, LIVE>(p, lane);
  V u = p[0];
  if constexpr (NV <= 4) u += xor_lane<8>(u);
  if constexpr (NV <= 8) u += xor_lane<4>(u);
  if constexpr (NV <= 16) u += xor_lane<2>(u);
  if constexpr (NV <= 32) u += xor_lane<1>(u);
  return u;
}

// Live-value mask of G groups of P slots of which the first U are used.
constexpr unsigned long long live_slots(int G, int P, int U) {
  unsigned long long m = 0;
  for (int g = 0; g < G; ++g)
    for (int o = 0; o < U; ++o) m |= 1ull << (g * P + o);
  return m;
}

// ---------------------------------------------------------------------------
// Level residual y = r + sx J x  (sx = -1: r - J x; r == nullptr: sx J x).
// RPW consecutive block rows per 64-lane wavefront: the rows' blocks are
// contiguous, so lane (q_off, j) streams block column j of every (64/B)-th
// block of the whole range (consecutive lanes read consecutive doubles),
// keeping RPW*B partial sums that one transpose-reduce folds at the end.
// The rows per wavefront (1-4) are a per-level launch parameter: few rows
// leave lanes idle at the end of the range, many cost registers.
template <int B, int RPW>
__global__ void __launch_bounds__(256) k_spmv_rows(const int32_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, int32_t n_rows,
                                                   double sx) {
  constexpr int NQ = 64 / B;
  constexpr int NV = RPW * B;
  constexpr int NVP = NV <= 2 ? 2 : NV <= 4 ? 4 : NV <= 8 ? 8 : NV <= 16 ? 16 : 32;
  const int lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RPW;
  if (row0 >= n_rows) return;  // uniform per wavefront
  const int qo = lane / B;
  const int j = lane - qo * B;
  int32_t rp[RPW + 1];
#pragma unroll
  for (int t = 0; t <= RPW; ++t) rp[t] = rowptr[min(row0 + t, n_rows)];
  double acc[NVP];
#pragma unroll
  for (int v = 0; v < NVP; ++v) acc[v] = 0.0;
  if (qo < NQ) {
#pragma unroll 4
    for (int32_t q = rp[0] + qo; q < rp[RPW]; q += NQ) {
      const int32_t c = col[q];
      const double xv = x[(int64_t)c * B + j];
      const double* vb = val + (int64_t)q * (B * B) + j;
      int rr = 0;
#pragma unroll
      for (int t = 1; t < RPW; ++t) rr += (q >= rp[t]) ? 1 : 0;
#pragma unroll
      for (int i = 0; i < B; ++i) {
        const double pv = vb[i * B] * xv;
#pragma unroll
        for (int t = 0; t < RPW; ++t) acc[t * B + i] += (rr == t) ? pv : 0.0;
      }
    }
  }
  const double sum = fold<NVP>(acc, lane);
  constexpr int SPAN = 64 / NVP;
  const int v = lane / SPAN;
  if ((lane % SPAN) == 0 && v < NV) {
    const int t = v / B, i = v - (v / B) * B;
    const int row = row0 + t;
    if (row < n_rows) {
      const int64_t o = (int64_t)row * B + i;
      y[o] = r ? fma(sx, sum, r[o]) : sx * sum;
    }
  }
}

template <int B>
static hipError_t spmv_b(hipStream_t s, const DevLevel& L, bool tr, const double* r,
                         const double* x, double* y, double sx) {
  const int rpw = L.spmv_rpw < 4 ? L.spmv_rpw : 4;
  const int32_t* rp = tr ? L.rowptr_t : L.rowptr;
  const int32_t* cl = tr ? L.col_t : L.col;
  const double* vl = tr ? L.val_t : L.val;
  if (!rp || !cl || !vl) return hipErrorInvalidValue;
  dim3 grid((L.n_s + 4 * rpw - 1) / (4 * rpw)), block(256);
  switch (rpw) {
    case 1: launch(k_spmv_rows<B, 1>, dim3(grid), dim3(block), 0, s, rp, cl, vl, r, x, y, L.n_s, sx); break;
    case 2: launch(k_spmv_rows<B, 2>, dim3(grid), dim3(block), 0, s, rp, cl, vl, r, x, y, L.n_s, sx); break;
    case 3: launch(k_spmv_rows<B, 3>, dim3(grid), dim3(block), 0, s, rp, cl, vl, r, x, y, L.n_s, sx); break;
    case 4: launch(k_spmv_rows<B, 4>, dim3(grid), dim3(block), 0, s, rp, cl, vl, r, x, y, L.n_s, sx); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_spmv(hipStream_t s, int b, const DevLevel& L, const double* r, const double* x,
                       double* y, double sx, bool transposed) {
  switch (b) {
    case 1: return spmv_b<1>(s, L, transposed, r, x, y, sx);
    case 2: return spmv_b<2>(s, L, transposed, r, x, y, sx);
    case 3: return spmv_b<3>(s, L, transposed, r, x, y, sx);
    case 4: return spmv_b<4>(s, L, transposed, r, x, y, sx);
  }
  return hipErrorInvalidValue;
}

// Level residual from the spatial factors of an operator whose blocks are
// C[i][l] M + delta_il tw[i] A (time-independent coefficients): per block only
// the two scalars m = M(s, s') and a = A(s, s') are streamed.  SPLIT: a row's
// blocks come in two lists, those with m != 0 as one 16-byte (m, a) pair,
// then those with m = 0 (the velocity-pressure couplings of a mass matrix
// that acts on the velocity only) as a only, 8 bytes; otherwise one list of
// (m, a) pairs in the level's block order.  LPR lanes per block row
// (64 / LPR rows per wavefront): lane `sub` of a row takes the list's blocks
// sub, sub + LPR, ..., U of them per round, with every load of a round issued
// before the first is used (indices clamped into the list, the blocks past
// its end weighted by zero, instead of branches), and keeps only the B
// partial sums of its own row; the row's lanes then add their sums
// (butterfly over the LPR lanes).  LPR x U slots per round are matched to
// the typical row length by the autotuner.
struct KronCoef { double C[16]; double tw[4]; };

template <int B, int LPR, int U, bool SPLIT>
__global__ void __launch_bounds__(256) k_spmv_kron(const int32_t* __restrict__ rp1,
                                                   const int32_t* __restrict__ col1,
                                                   const double2* __restrict__ ma,
                                                   const int32_t* __restrict__ rp2,
                                                   const int32_t* __restrict__ col2,
                                                   const double* __restrict__ a2,
                                                   const double* __restrict__ r,
                                                   const double* __restrict__ x,
                                                   double* __restrict__ y, int32_t n_rows,
                                                   double sx, KronCoef K) {
  constexpr int RPWV = 64 / LPR;
  const int lane = threadIdx.x & 63, sub = lane % LPR;
  const int row = (blockIdx.x * 4 + (threadIdx.x >> 6)) * RPWV + lane / LPR;
  const bool live = row < n_rows;
  const int rr = live ? row : n_rows - 1;
  double rv = 0.0;
  if (r && live && sub < B) rv = r[(int64_t)rr * B + sub];
  double acc[B];
#pragma unroll
  for (int i = 0; i < B; ++i) acc[i] = 0.0;
  // blocks with a mass entry: (m, a)
  {
    const int32_t q0 = rp1[rr], q1 = rp1[rr + 1];
    const int nit = (q1 - q0 + U * LPR - 1) / (U * LPR);
    for (int it = 0; it < nit; ++it) {
      const int32_t qb = q0 + it * U * LPR + sub;
      int64_t c[U];
      double m[U], a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t q = qb + u * LPR;
        const bool v = q < q1;
        const int32_t qc = v ? q : q1 - 1;
        c[u] = col1[qc];
        const double2 f = ma[qc];
        m[u] = v ? f.x : 0.0;
        a[u] = v ? f.y : 0.0;
      }
      double xl[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int l = 0; l < B; ++l) xl[u][l] = x[c[u] * B + l];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < B; ++i) {
          double ci = 0.0;
#pragma unroll
          for (int l = 0; l < B; ++l) ci = fma(K.C[i * B + l], xl[u][l], ci);
          acc[i] = fma(m[u], ci, fma(a[u] * K.tw[i], xl[u][i], acc[i]));
        }
    }
  }
  // blocks without one: a only
  if constexpr (SPLIT) {
    const int32_t q0 = rp2[rr], q1 = rp2[rr + 1];
    const int nit = (q1 - q0 + U * LPR - 1) / (U * LPR);
    for (int it = 0; it < nit; ++it) {
      const int32_t qb = q0 + it * U * LPR + sub;
      int64_t c[U];
      double a[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int32_t q = qb + u * LPR;
        const bool v = q < q1;
        const int32_t qc = v ? q : q1 - 1;
        c[u] = col2[qc];
        const double f = a2[qc];
        a[u] = v ? f : 0.0;
      }
      double xl[U][B];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int l = 0; l < B; ++l) xl[u][l] = x[c[u] * B + l];
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int i = 0; i < B; ++i) acc[i] = fma(a[u] * K.tw[i], xl[u][i], acc[i]);
    }
  }
#pragma unroll
  for (int off = LPR / 2; off >= 1; off >>= 1)
#pragma unroll
    for (int i = 0; i < B; ++i) acc[i] += __shfl_xor(acc[i], off, 64);
  if (live && sub < B) {
    double s = acc[0];
#pragma unroll
    for (int i = 1; i < B; ++i) s = (sub == i) ? acc[i] : s;
    y[(int64_t)row * B + sub] = r ? fma(sx, s, rv) : sx * s;
  }
}

// residual shapes from the factors: (lanes per block row, blocks per lane and round)
// (shapes 7-12: the same on the split lists)
static constexpr int kKronShapes = 12;
static constexpr int kKronLpr[kKronShapes] = {4, 8, 8, 16, 16, 32, 4, 8, 8, 16, 16, 32};
static constexpr int kKronU[kKronShapes] = {4, 3, 4, 2, 4, 2, 4, 3, 4, 2, 4, 2};

int residual_shapes(const DevLevel& L) { return L.kron_ma ? kKronShapes : 4; }

template <int B>
static hipError_t spmv_kron_b(hipStream_t s, const DevLevel& L, const double* r, const double* x,
                              double* y, double sx) {
  KronCoef K{};
  for (int e = 0; e < B * B; ++e) K.C[e] = L.kron_C[e];
  for (int e = 0; e < B; ++e) K.tw[e] = L.kron_tw[e];
  const int sh = L.spmv_rpw - 1;
  if (sh < 0 || sh >= kKronShapes) return hipErrorInvalidValue;
  const int lpr = kKronLpr[sh], rows_per_wg = 4 * (64 / lpr);
  dim3 grid((L.n_s + rows_per_wg - 1) / rows_per_wg), block(256);
  const bool split = sh >= kKronShapes / 2;
  if (split && (!L.kx_ptr || !L.kx_col || !L.kx_val)) return hipErrorInvalidValue;
  const int64_t n1 = L.kx_n1;
  const int32_t* rp1 = split ? L.kx_ptr : L.rowptr;
  const int32_t* c1 = split ? L.kx_col : L.col;
  const double2* ma = (const double2*)(split ? L.kx_val : L.kron_ma);
  const int32_t* rp2 = split ? L.kx_ptr + (L.n_s + 1) : nullptr;
  const int32_t* c2 = split ? L.kx_col + n1 : nullptr;
  const double* a2 = split ? L.kx_val + 2 * n1 : nullptr;
#define STV_KRON(S, LP, UU, SP)                                                              \
  case S:                                                                                   \
    launch(k_spmv_kron<B, LP, UU, SP>, dim3(grid), dim3(block), 0, s, rp1, c1, ma, rp2, c2, a2, \
           r, x, y, L.n_s, sx, K);                                                          \
    break;
  switch (sh) {
    STV_KRON(0, 4, 4, false) STV_KRON(1, 8, 3, false) STV_KRON(2, 8, 4, false)
    STV_KRON(3, 16, 2, false) STV_KRON(4, 16, 4, false) STV_KRON(5, 32, 2, false)
    STV_KRON(6, 4, 4, true) STV_KRON(7, 8, 3, true) STV_KRON(8, 8, 4, true)
    STV_KRON(9, 16, 2, true) STV_KRON(10, 16, 4, true) STV_KRON(11, 32, 2, true)
    default: return hipErrorInvalidValue;
  }
#undef STV_KRON
  return hipGetLastError();
}

hipError_t launch_spmv_kron(hipStream_t s, int b, const DevLevel& L, const double* r,
                            const double* x, double* y, double sx) {
  switch (b) {
    case 1: return spmv_kron_b<1>(s, L, r, x, y, sx);
    case 2: return spmv_kron_b<2>(s, L, r, x, y, sx);
    case 3: return spmv_kron_b<3>(s, L, r, x, y, sx);
    case 4: return spmv_kron_b<4>(s, L, r, x, y, sx);
  }
  return hipErrorInvalidValue;
}

// Largest deviation of the stored blocks from C m + delta tw a, and the
// largest block entry: one (deviation, magnitude) pair per workgroup.
template <int B>
__global__ void __launch_bounds__(256) k_kron_check(const double* __restrict__ val,
                                                    const double2* __restrict__ ma,
                                                    int64_t nnzb, KronCoef K,
                                                    double* __restrict__ partial) {
  __shared__ double sd[4], sm[4];
  double dev = 0.0, mag = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < nnzb;
       q += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int l = 0; l < B; ++l) {
        const double v = val[q * B * B + i * B + l];
        const double2 f = ma[q];
        const double rec = K.C[i * B + l] * f.x + (i == l ? K.tw[i] * f.y : 0.0);
        dev = fmax(dev, fabs(v - rec));
        mag = fmax(mag, fabs(v));
      }
  }
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    dev = fmax(dev, __shfl_xor(dev, off, 64));
    mag = fmax(mag, __shfl_xor(mag, off, 64));
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) { sd[wv] = dev; sm[wv] = mag; }
  __syncthreads();
  if (threadIdx.x == 0) {
    partial[2 * blockIdx.x] = fmax(fmax(sd[0], sd[1]), fmax(sd[2], sd[3]));
    partial[2 * blockIdx.x + 1] = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
  }
}

hipError_t launch_kron_check(hipStream_t s, int b, const DevLevel& L, const double* ma_,
                             const double* C, const double* tw, double* partial, int nblk) {
  const double2* ma = (const double2*)ma_;
  KronCoef K{};
  for (int e = 0; e < b * b; ++e) K.C[e] = C[e];
  for (int e = 0; e < b; ++e) K.tw[e] = tw[e];
  switch (b) {
    case 1: k_kron_check<1><<<nblk, 256, 0, s>>>(L.val, ma, L.nnzb, K, partial); break;
    case 2: k_kron_check<2><<<nblk, 256, 0, s>>>(L.val, ma, L.nnzb, K, partial); break;
    case 3: k_kron_check<3><<<nblk, 256, 0, s>>>(L.val, ma, L.nnzb, K, partial); break;
    case 4: k_kron_check<4><<<nblk, 256, 0, s>>>(L.val, ma, L.nnzb, K, partial); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Values of the transposed level matrix: block qt of J^T is the transpose of
// block src[qt] of J (the pattern of J^T is built on the host).
template <int B>
__global__ void k_bsr_transpose_vals(const double* __restrict__ val,
                                     const int32_t* __restrict__ src, double* __restrict__ val_t,
                                     int64_t nnzb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nnzb * B * B) return;
  const int64_t qt = e / (B * B);
  const int ij = (int)(e - qt * (B * B));
  const int i = ij / B, l = ij - i * B;
  val_t[e] = val[(int64_t)src[qt] * (B * B) + l * B + i];
}

hipError_t launch_bsr_transpose_vals(hipStream_t s, int b, const double* val, const int32_t* src,
                                     double* val_t, int64_t nnzb) {
  const int64_t n = nnzb * b * b;
  const unsigned grid = (unsigned)((n + 255) / 256);
  switch (b) {
    case 1: k_bsr_transpose_vals<1><<<grid, 256, 0, s>>>(val, src, val_t, nnzb); break;
    case 2: k_bsr_transpose_vals<2><<<grid, 256, 0, s>>>(val, src, val_t, nnzb); break;
    case 3: k_bsr_transpose_vals<3><<<grid, 256, 0, s>>>(val, src, val_t, nnzb); break;
    case 4: k_bsr_transpose_vals<4><<<grid, 256, 0, s>>>(val, src, val_t, nnzb); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Vanka cell sweep.  One 64-lane wavefront per cell T (four cells per
// workgroup, no LDS, no barriers): lane j holds rho_T[j] for the columns
// j = lane + 64c of the cell-local order (alpha, l) -> alpha*B + l, gathered
// straight from the level residual.  The stored inverse rows are row-major,
// so each row is one contiguous, fully coalesced read.  Rows are taken G at
// a time with every load of a group issued before the first is used
// (indices clamped into the cell's block instead of branches, so that the
// loads do not serialise), and the G partial sums are folded by one
// transpose-reduce.  Last-writer form: only the rows of the DoFs the cell
// owns are computed; row r of the cell ends in lane r % 64, which also
// fetched the old iterate of that DoF at the start, and the cell's rows are
// stored in one pass (d_j += omega c_j, or = omega c_j for a zero initial
// iterate).  Every DoF has exactly one owner, so the stores are disjoint (no
// atomics, deterministic).  FULL: the store keeps every row of J_T^-1 and the
// owned ones are picked by their local index.  The row products and the
// transpose-reduce are in the precision of the store (FP32 products of an
// FP32 store and the residual rounded to FP32, summed in FP32), the update
// of the iterate in FP64.
template <int B, int NLS, typename TS, bool FULL>
__global__ void __launch_bounds__(256) k_vanka(const double* __restrict__ rho,
                                              double* __restrict__ d,
                                              const int32_t* __restrict__ csd,
                                              const int32_t* __restrict__ own_ptr,
                                              const uint8_t* __restrict__ own_loc,
                                              const int64_t* __restrict__ inv_off, int ld,
                                              const TS* __restrict__ store, double omega,
                                              int zero_init, int n_cells) {
  constexpr int N = B * NLS;
  constexpr int NC = (N + 63) / 64;        // 64-column chunks of a row
  constexpr int NOC = (NLS + 63) / 64;     // 64-lane chunks of the owned DoFs
  constexpr int RC = NC;                   // 64-lane chunks of the owned rows (R <= N)
  constexpr int G = NC == 1 ? 16 : 8;      // rows per group
  const int lane = threadIdx.x & 63;
  // one cell per wavefront and step; a grid smaller than the cell count makes
  // the launch persistent (each wavefront strides over the cells)
  // (the cell index is wave-uniform: its per-cell data sits in scalar registers)
  const int T0 = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  for (int T = T0; T < n_cells; T += gridDim.x * 4) {
    const int32_t* sd = csd + (int64_t)T * NLS;
    const int o0 = own_ptr[T];
    const int no = own_ptr[T + 1] - o0;
    if (no <= 0) continue;
    const int R = no * B;
    const TS* A = store + inv_off[T];
    double x[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      const int jc = j < N ? j : N - 1;
      const int be = jc / B;
      const double v = rho[(int64_t)sd[be] * B + (jc - be * B)];
      x[c] = j < N ? v : 0.0;
    }
    // the row products are in the precision of the store (see k_vanka_dec)
    TS xs[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) xs[c] = (TS)x[c];
    // owned DoFs, lane = owned index: local index and spatial DoF
    int ol[NOC], gs[NOC];
#pragma unroll
    for (int c = 0; c < NOC; ++c) {
      const int k = lane + 64 * c;
      ol[c] = own_loc[o0 + (k < no ? k : no - 1)];
      gs[c] = sd[ol[c]];
    }
    // the rows this lane stores (r = lane + 64 rc): DoF index and old value
    int64_t gi[RC];
    double dold[RC], res[RC];
#pragma unroll
    for (int rc = 0; rc < RC; ++rc) {
      const int r = lane + 64 * rc;
      const int rcl = r < R ? r : R - 1;
      const int os = rcl / B;
      int g = __shfl(gs[0], os & 63, 64);
      if constexpr (NOC > 1) {
        const int g1 = __shfl(gs[NOC - 1], os & 63, 64);
        g = os < 64 ? g : g1;
      }
      gi[rc] = (int64_t)g * B + (rcl - os * B);
      dold[rc] = zero_init ? 0.0 : d[gi[rc]];
      res[rc] = 0.0;
    }
    for (int r0 = 0; r0 < R; r0 += G) {
      TS a[G][NC];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const int row = min(r0 + t, R - 1);
        int srow = row;
        if constexpr (FULL) {
          const int os = row / B;
          int l = __builtin_amdgcn_readlane(ol[0], os & 63);
          if constexpr (NOC > 1) {
            const int l1 = __builtin_amdgcn_readlane(ol[NOC - 1], os & 63);
            l = os < 64 ? l : l1;
          }
          srow = l * B + (row - os * B);
        }
        // offsets inside the cell's block fit 32 bits: the loads address
        // from the block's (wave-uniform) base
        const unsigned ro = (unsigned)(srow * ld);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int j = lane + 64 * c;
          a[t][c] = A[ro + (unsigned)(j < N ? j : N - 1)];
        }
      }
      TS p[G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        TS acc = TS(0);
#pragma unroll
        for (int c = 0; c < NC; ++c) acc = fma(a[t][c], xs[c], acc);
        p[t] = acc;
      }
      const TS sum = fold_swap<G>(p, lane);   // row r0 + t in lanes t * (64 / G) ..
      // row r0 + t goes to lane (r0 + t) % 64 of chunk r0 / 64 (a group never
      // straddles two chunks: G divides 64)
      const int t = lane - (r0 & 63);
      const double v = (double)__shfl(sum, (t & (G - 1)) * (64 / G), 64);
      const int rcg = r0 >> 6;
#pragma unroll
      for (int rc = 0; rc < RC; ++rc)
        if (rc == rcg && t >= 0 && t < G) res[rc] = v;
    }
#pragma unroll
    for (int rc = 0; rc < RC; ++rc) {
      const int r = lane + 64 * rc;
      if (r < R) d[gi[rc]] = zero_init ? omega * res[rc] : fma(omega, res[rc], dold[rc]);
    }
  }
}

// ---------------------------------------------------------------------------
// Vanka cell sweep on time-decoupled inverses (CellSplit, last-writer form):
//   d_T <- d_T + omega (I (x) V) Q^-1 (I (x) W) rho_T   on the owned rows.
// One 64-lane wavefront per cell (B * NLS <= 64).  Lane j gathers rho_T[j]
// (local order alpha * B + l) and forms u = (I (x) W) rho_T in the same
// order (the B values of a spatial DoF by shuffles).  Lane j then takes the
// multipliers of stored column j: in block p (first time component f) at
// spatial DoF s, column j multiplies u[s, f] into output f; in the second
// half of a pair block (the imaginary part of the complex inverse) it
// multiplies -u[s, f + 1] into output f and u[s, f] into output f + 1, and
// in the first half u[s, f + 1] into output f + 1 as well: the real form of
// the complex product (the lane's constants come from the level's table,
// made with the store).  Each stored row (one owned spatial DoF) is one
// coalesced read and gives B per-lane products; 16 / BP rows at a time are
// folded by one transpose-reduce (slots of the padding outputs skipped),
// and the lane of DoF (k, i) combines the B outputs of row k with row i of
// V in FP64.  The products and the transpose-reduce are in the precision of
// the store: an FP32 store multiplies its values by the multipliers rounded
// to FP32 and sums in FP32, which halves the exchanges; the error this adds
// is of the order of the rounding of the stored values themselves.  Stores
// as in k_vanka.
// Occupancy the register allocation must leave room for (waves per SIMD):
// the sweep hides its load latency with waves; without spills the FP32 form
// fits 8, the FP64 form 6 (B = 1, 3) or 5 (B = 2).
template <int B, typename TS>
constexpr int dec_waves() {
  return sizeof(TS) == 4 ? 8 : (B == 2 ? 5 : 6);
}

template <int B, int NLS, typename TS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(dec_waves<B, TS>())))
k_vanka_dec(const double* __restrict__ rho,
                                                  double* __restrict__ d,
                                                  const int32_t* __restrict__ csd,
                                                  const int32_t* __restrict__ own_ptr,
                                                  const uint8_t* __restrict__ own_loc,
                                                  const int64_t* __restrict__ inv_off, int ld,
                                                  const TS* __restrict__ store, double omega,
                                                  int zero_init, int n_cells,
                                                  const double* __restrict__ tab,
                                                  const int32_t* __restrict__ code) {
  constexpr int N = B * NLS;
  static_assert(N <= 64 && NLS <= 64, "one wavefront per cell");
  constexpr int BP = B <= 2 ? 2 : 4;       // outputs per stored row, padded to a power of two
  constexpr int GN = 16 / BP;              // stored rows per transpose-reduce
  constexpr unsigned long long LIVE = live_slots(GN, BP, B);
  // stored rows loaded together: an interior cell owns about n_loc / 2
  // spatial DoFs, so one round of loads usually covers the cell (every load
  // in flight at once; each transpose-reduce waits only for its own rows)
  constexpr int GL = (B == 2 ? 2 : 3) * GN;
  const int lane = threadIdx.x & 63;
  const int jl = lane < N ? lane : N - 1;
  const int al = jl / B, cl = jl - al * B;   // spatial DoF and time component of lane j
  // per-lane constants of the level: W[cl][.], V[lane % B][.], the source
  // lanes of u and the multipliers of stored column j = lane
  double wl[B], vl[B];
#pragma unroll
  for (int l = 0; l < B; ++l) {
    wl[l] = tab[l * 64 + lane];
    vl[l] = tab[(B + l) * 64 + lane];
  }
  const int cd = code[lane];
  const int srca = cd & 63, srcb = (cd >> 6) & 63;
  // the multipliers 0, +1 or -1 of the two sources (2 bits each in the code
  // word): kept as constants for B <= 2, decoded per cell for B = 3, where
  // the registers they would hold cost a wavefront per SIMD
  constexpr bool DECODE = B == 3;
  double ca[DECODE ? 1 : B], cb[DECODE ? 1 : B];
#pragma unroll
  for (int o = 0; o < (DECODE ? 1 : B); ++o) {
    const int ea = (cd >> (12 + 2 * o)) & 3, eb = (cd >> (12 + 2 * B + 2 * o)) & 3;
    ca[o] = ea == 1 ? 1.0 : (ea == 3 ? -1.0 : 0.0);
    cb[o] = eb == 1 ? 1.0 : (eb == 3 ? -1.0 : 0.0);
  }
  // byte offset of the lane's column in a stored row, and of one row
  const unsigned jb = (unsigned)(jl * sizeof(TS)), rb = (unsigned)(ld * sizeof(TS));
  // the cell's offsets and its DoF list are fetched one cell ahead (a
  // persistent grid strides over the cells), so that a cell starts with its
  // row loads and its gather instead of a chain of dependent loads
  const int stride = gridDim.x * 4;
  int T = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  int o0n = 0, nxn = 0, sdn = 0;
  int64_t offn = 0;
  if (T < n_cells) {
    o0n = own_ptr[T];
    nxn = own_ptr[T + 1];
    offn = inv_off[T];
    sdn = csd[(int64_t)T * NLS + al];
  }
  for (; T < n_cells; T += stride) {
    const int o0 = o0n, no = nxn - o0n, sdv = sdn;
    const char* A = reinterpret_cast<const char*>(store + offn);
    const int Tn = T + stride;
    if (Tn < n_cells) {
      o0n = own_ptr[Tn];
      nxn = own_ptr[Tn + 1];
      offn = inv_off[Tn];
      sdn = csd[(int64_t)Tn * NLS + al];
    }
    if (no <= 0) continue;
    const int R = no * B;
    const double xv = rho[(int64_t)sdv * B + cl];
    const double x = lane < N ? xv : 0.0;
    double u = 0.0;
#pragma unroll
    for (int l = 0; l < B; ++l) u = fma(wl[l], __shfl(x, al * B + l, 64), u);
    const double ua = __shfl(u, srca, 64), ub = __shfl(u, srcb, 64);
    TS m[B];
#pragma unroll
    for (int o = 0; o < B; ++o) {
      if constexpr (DECODE) {
        const int ea = (cd >> (12 + 2 * o)) & 3, eb = (cd >> (12 + 2 * B + 2 * o)) & 3;
        const double ta = ea == 1 ? ua : (ea == 3 ? -ua : 0.0);
        const double tb = eb == 1 ? ub : (eb == 3 ? -ub : 0.0);
        m[o] = (TS)(ta + tb);
      } else {
        m[o] = (TS)fma(ca[o], ua, cb[o] * ub);
      }
    }
    // the owned DoF of each stored row (lane = owned index; its spatial
    // index from the lanes of its local DoF), the row this lane stores
    // (r = lane = k * B + i), its global index and old value
    const int ok = lane < no ? lane : no - 1;
    const int gs = __shfl(sdv, own_loc[o0 + ok] * B, 64);
    const int rl = lane < R ? lane : R - 1;
    const int kl = rl / B;
    const int64_t gi = (int64_t)__shfl(gs, kl, 64) * B + (rl - kl * B);
    const double dold = zero_init ? 0.0 : d[gi];
    double res = 0.0;
    for (int k0 = 0; k0 < no; k0 += GL) {
      TS a[GL];
#pragma unroll
      for (int t = 0; t < GL; ++t) {
        const unsigned row = (unsigned)min(k0 + t, no - 1);
        a[t] = *reinterpret_cast<const TS*>(A + (row * rb + jb));
      }
#pragma unroll
      for (int h = 0; h < GL / GN; ++h) {
        TS pp[16];
#pragma unroll
        for (int t = 0; t < GN; ++t)
#pragma unroll
          for (int o = 0; o < BP; ++o) pp[t * BP + o] = o < B ? a[h * GN + t] * m[o] : TS(0);
        // value t * BP + o in lanes 4 (t * BP + o) .. + 3
        const TS sum = fold_swap<16, LIVE>(pp, lane);
        const int kb = k0 + h * GN;
        const int kk = kl - kb;                  // this lane's row within the group
        const int kc = kk < 0 ? 0 : (kk >= GN ? GN - 1 : kk);
        double val = 0.0;
#pragma unroll
        for (int o = 0; o < B; ++o)
          val = fma(vl[o], (double)__shfl(sum, 4 * (kc * BP + o), 64), val);
        if (kk >= 0 && kk < GN) res = val;
      }
    }
    if (lane < R) d[gi] = zero_init ? omega * res : fma(omega, res, dold);
  }
}

// ---------------------------------------------------------------------------
// Vanka cell sweep on the complex time-decoupled store of a dG(1) level with
// one complex pair (built by k_inverse_cx): the stored row of owned spatial
// DoF a is Y_a. = (X^-1)_a. as [Re Y_a0 .. Re Y_a,n-1, Im Y_a0 .. Im Y_a,n-1],
// and with u = (I (x) W) rho_T (u_0 + i u_1 per spatial DoF c)
//   y_a = sum_c Y_ac (u_0c + i u_1c),  c_(a, i) = V_i0 Re y_a + V_i1 Im y_a:
// the same J_T^-1 rho_T = (I (x) V) Q^-1 (I (x) W) rho_T as the two plain rows
// of a, from half the stored values.  One wavefront per cell.  A stored row
// is read as one flat run of 2 NLS values, NF = 2 NLS / 64 (rounded up)
// coalesced loads: value v = 64 k + lane is Re Y_ac (v < NLS, c = v) or
// Im Y_ac (c = v - NLS), and the lane holds, per load, the two multipliers
// that put it into Re y_a and Im y_a (u_0c and u_1c for a real part, -u_1c
// and u_0c for an imaginary one), formed once per cell from its own
// 16-byte load of the time-inner pair rho_(c, 0..1).  G rows at a time give
// 2G sums (real and imaginary parts) folded by one transpose-reduce.  Output
// r = 2 os + i of the os-th owned DoF lands in lane r % 64, which fetched the
// DoF's old value at the start; stores as in k_vanka.  The complex products
// and the transpose-reduce are in the precision of the store, the
// recombination with V and the update in FP64.
template <int NLS, typename TS, int G>
__global__ void __launch_bounds__(256) k_vanka_cx(const double* __restrict__ rho,
                                                 double* __restrict__ d,
                                                 const int32_t* __restrict__ csd,
                                                 const int32_t* __restrict__ own_ptr,
                                                 const uint8_t* __restrict__ own_loc,
                                                 const int64_t* __restrict__ inv_off, int ld,
                                                 const TS* __restrict__ store, double omega,
                                                 int zero_init, int n_cells, CellSplit sp) {
  constexpr int B = 2;
  constexpr int NF = (2 * NLS + 63) / 64;    // flat 64-lane loads of a stored row
  constexpr int NOC = (NLS + 63) / 64;       // 64-lane chunks of the owned DoFs
  constexpr int RC = (B * NLS + 63) / 64;    // 64-lane chunks of the outputs
  const int lane = threadIdx.x & 63;
  const double w00 = sp.W[0], w01 = sp.W[1], w10 = sp.W[2], w11 = sp.W[3];
  const double v00 = sp.V[0], v01 = sp.V[1], v10 = sp.V[2], v11 = sp.V[3];
  // byte offsets of the lane's values in a stored row
  unsigned vb[NF];
#pragma unroll
  for (int k = 0; k < NF; ++k) {
    const int v = 64 * k + lane;
    vb[k] = (unsigned)((v < 2 * NLS ? v : 2 * NLS - 1) * sizeof(TS));
  }
  const unsigned rb = (unsigned)(ld * sizeof(TS));
  const int T0 = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  for (int T = T0; T < n_cells; T += gridDim.x * 4) {
    const int32_t* sd = csd + (int64_t)T * NLS;
    const int o0 = own_ptr[T];
    const int no = own_ptr[T + 1] - o0;
    if (no <= 0) continue;
    const int R = no * B;
    const char* A = reinterpret_cast<const char*>(store + inv_off[T]);
    // the multipliers of the lane's values: (into Re y, into Im y)
    TS mre[NF], mim[NF];
#pragma unroll
    for (int k = 0; k < NF; ++k) {
      const int v = 64 * k + lane;
      const bool ok = v < 2 * NLS;
      const bool im = v >= NLS;
      const int c = ok ? (im ? v - NLS : v) : 0;
      const double2 rr = *reinterpret_cast<const double2*>(&rho[(int64_t)sd[c] * B]);
      const double u0 = fma(w00, rr.x, w01 * rr.y), u1 = fma(w10, rr.x, w11 * rr.y);
      mre[k] = (TS)(ok ? (im ? -u1 : u0) : 0.0);
      mim[k] = (TS)(ok ? (im ? u0 : u1) : 0.0);
    }
    int gs[NOC];
#pragma unroll
    for (int c = 0; c < NOC; ++c) {
      const int k = lane + 64 * c;
      gs[c] = sd[own_loc[o0 + (k < no ? k : no - 1)]];
    }
    int64_t gi[RC];
    double dold[RC], res[RC];
#pragma unroll
    for (int rc = 0; rc < RC; ++rc) {
      const int r = lane + 64 * rc;
      const int rcl = r < R ? r : R - 1;
      const int os = rcl / B;
      int g = __shfl(gs[0], os & 63, 64);
      if constexpr (NOC > 1) {
        const int g1 = __shfl(gs[NOC - 1], os & 63, 64);
        g = os < 64 ? g : g1;
      }
      gi[rc] = (int64_t)g * B + (rcl - os * B);
      dold[rc] = zero_init ? 0.0 : d[gi[rc]];
      res[rc] = 0.0;
    }
    for (int k0 = 0; k0 < no; k0 += G) {
      TS a[G][NF];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        const unsigned ro = (unsigned)min(k0 + t, no - 1) * rb;
#pragma unroll
        for (int k = 0; k < NF; ++k) a[t][k] = *reinterpret_cast<const TS*>(A + (ro + vb[k]));
      }
      TS p[2 * G];
#pragma unroll
      for (int t = 0; t < G; ++t) {
        TS re = TS(0), im = TS(0);
#pragma unroll
        for (int k = 0; k < NF; ++k) {
          re = fma(a[t][k], mre[k], re);
          im = fma(a[t][k], mim[k], im);
        }
        p[2 * t] = re;
        p[2 * t + 1] = im;
      }
      const TS sum = fold_swap<2 * G>(p, lane);   // value e in lanes e (64 / 2G) ..
#pragma unroll
      for (int rc = 0; rc < RC; ++rc) {
        const int r = lane + 64 * rc;
        const int t = (r >> 1) - k0;
        const int tc = t < 0 ? 0 : (t >= G ? G - 1 : t);
        const double re = (double)__shfl(sum, (64 / (2 * G)) * (2 * tc), 64);
        const double im = (double)__shfl(sum, (64 / (2 * G)) * (2 * tc + 1), 64);
        const double val = (r & 1) ? fma(v10, re, v11 * im) : fma(v00, re, v01 * im);
        if (t >= 0 && t < G) res[rc] = val;
      }
    }
#pragma unroll
    for (int rc = 0; rc < RC; ++rc) {
      const int r = lane + 64 * rc;
      if (r < R) d[gi[rc]] = zero_init ? omega * res[rc] : fma(omega, res[rc], dold[rc]);
    }
  }
}

// rows per transpose-reduce of the complex sweep: 8 in FP64 (115 registers,
// four wavefronts per SIMD), 16 in FP32 (twice the rows in flight in about
// the same registers)
template <typename TS>
constexpr int cx_group() { return sizeof(TS) == 4 ? 16 : 8; }

template <int B, int NLS>
static hipError_t vanka_bn(hipStream_t s, const DevLevel& L, const double* rho, double* d,
                           double omega, int zero_init, int fp32, int full) {
  unsigned grid = (unsigned)((L.n_cells + 3) / 4);
  if (L.sweep_wgs > 0 && (unsigned)L.sweep_wgs < grid) grid = (unsigned)L.sweep_wgs;
  if constexpr (B * NLS <= 64) {
    if (L.dec) {
      if (full || L.split.b != B || !L.dec_tab || !L.dec_code) return hipErrorInvalidValue;
      if (fp32)
        launch(k_vanka_dec<B, NLS, float>, dim3(grid), dim3(256), 0, s, rho, d, L.cell_sdofs,
               L.own_ptr, L.own_loc, L.inv_off, L.inv_ld, (const float*)L.inv_store, omega,
               zero_init, L.n_cells, (const double*)L.dec_tab, (const int32_t*)L.dec_code);
      else
        launch(k_vanka_dec<B, NLS, double>, dim3(grid), dim3(256), 0, s, rho, d, L.cell_sdofs,
               L.own_ptr, L.own_loc, L.inv_off, L.inv_ld, (const double*)L.inv_store, omega,
               zero_init, L.n_cells, (const double*)L.dec_tab, (const int32_t*)L.dec_code);
      return hipGetLastError();
    }
  }
  if constexpr (B == 2 && NLS == 85) {
    if (L.dec && L.cx) {
      if (full) return hipErrorInvalidValue;
      if (fp32)
        launch(k_vanka_cx<NLS, float, cx_group<float>()>, dim3(grid), dim3(256), 0, s, rho, d,
               L.cell_sdofs, L.own_ptr, L.own_loc, L.inv_off, L.inv_ld,
               (const float*)L.inv_store, omega, zero_init, L.n_cells, L.split);
      else
        launch(k_vanka_cx<NLS, double, cx_group<double>()>, dim3(grid), dim3(256), 0, s, rho, d,
               L.cell_sdofs, L.own_ptr, L.own_loc, L.inv_off, L.inv_ld,
               (const double*)L.inv_store, omega, zero_init, L.n_cells, L.split);
      return hipGetLastError();
    }
  }
  if (L.dec) return hipErrorInvalidValue;
#define STV_VANKA(TS, F)                                                                     \
  launch(k_vanka<B, NLS, TS, F>, dim3(grid), dim3(256), 0, s, rho, d, L.cell_sdofs, L.own_ptr, L.own_loc,  \
                                              L.inv_off, L.inv_ld, (const TS*)L.inv_store, \
                                              omega, zero_init, L.n_cells)
  if (fp32) {
    if (full) STV_VANKA(float, true);
    else STV_VANKA(float, false);
  } else {
    if (full) STV_VANKA(double, true);
    else STV_VANKA(double, false);
  }
#undef STV_VANKA
  return hipGetLastError();
}

template <int B>
static hipError_t vanka_b(hipStream_t s, const DevLevel& L, const double* rho, double* d,
                          double omega, int zero_init, int fp32, int full) {
  if (L.n_ls == 21) return vanka_bn<B, 21>(s, L, rho, d, omega, zero_init, fp32, full);
  if (L.n_ls == 85) return vanka_bn<B, 85>(s, L, rho, d, omega, zero_init, fp32, full);
  return hipErrorInvalidValue;
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
// Vanka sweep of the transposed operator J^T.  Its local inverse is
// (J_T^T)^-1 = (J_T^-1)^T, the stored full inverse read transposed: with the
// residual rho_T of J^T in lane j = lane + 64c, the correction
// c_o = sum_j (J_T^-1)[j][o] rho_j of local DoF o = lane + 64c accumulates in
// lane o, stored row j after row j (each row one coalesced read, rho_j
// broadcast by readlane), 8 rows per round with all their loads in flight.
// The owner rule and the update are those of the forward sweep: lane o
// learns whether the cell owns its DoF from the cell's owned list, fetches
// the DoF's old value at the start and stores once.  Needs every stored row.
template <int B, int NLS, typename TS>
__global__ void __launch_bounds__(256) k_vanka_t(const double* __restrict__ rho,
                                                double* __restrict__ d,
                                                const int32_t* __restrict__ csd,
                                                const int32_t* __restrict__ own_ptr,
                                                const uint8_t* __restrict__ own_loc,
                                                const int64_t* __restrict__ inv_off, int ld,
                                                const TS* __restrict__ store, double omega,
                                                int zero_init, int n_cells) {
  constexpr int N = B * NLS;
  constexpr int NC = (N + 63) / 64;
  constexpr int NOC = (NLS + 63) / 64;
  constexpr int U = 8;
  const int lane = threadIdx.x & 63;
  const int T0 = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
  for (int T = T0; T < n_cells; T += gridDim.x * 4) {
    const int32_t* sd = csd + (int64_t)T * NLS;
    const int o0 = own_ptr[T];
    const int no = own_ptr[T + 1] - o0;
    if (no <= 0) continue;
    const TS* A = store + inv_off[T];
    double x[NC], acc[NC], dold[NC];
    int64_t gi[NC];
    bool own[NC];
    int ol[NOC];
#pragma unroll
    for (int c = 0; c < NOC; ++c) {
      const int k = lane + 64 * c;
      ol[c] = own_loc[o0 + (k < no ? k : no - 1)];
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int j = lane + 64 * c;
      const int jc = j < N ? j : N - 1;
      const int be = jc / B;
      const int64_t g = (int64_t)sd[be] * B + (jc - be * B);
      const double v = rho[g];
      x[c] = j < N ? v : 0.0;
      acc[c] = 0.0;
      gi[c] = g;
      own[c] = false;
    }
    // ownership of this lane's DoFs: compare their spatial index with the
    // cell's owned list (broadcast entry by entry)
    for (int k = 0; k < no; ++k) {
      int a = __builtin_amdgcn_readlane(ol[0], k & 63);
      if constexpr (NOC > 1) {
        const int a1 = __builtin_amdgcn_readlane(ol[NOC - 1], k & 63);
        a = k < 64 ? a : a1;
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int o = lane + 64 * c;
        own[c] = own[c] || (o < N && o / B == a);
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const double v = d[gi[c]];
      dold[c] = zero_init ? 0.0 : v;
    }
#pragma unroll 1
    for (int j0 = 0; j0 < N; j0 += U) {
      TS a[U][NC];
      double rj[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = j0 + u;
        const int jr = j < N ? j : N - 1;
        const unsigned ro = (unsigned)(jr * ld);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int o = lane + 64 * c;
          a[u][c] = A[ro + (unsigned)(o < N ? o : N - 1)];
        }
        // rho_j from its lane (chunk j / 64, uniform)
        double r = readlane_f64(x[0], jr & 63);
#pragma unroll
        for (int c = 1; c < NC; ++c) {
          const double rc = readlane_f64(x[c], jr & 63);
          r = (jr >> 6) == c ? rc : r;
        }
        rj[u] = j < N ? r : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = fma((double)a[u][c], rj[u], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
      if (own[c]) d[gi[c]] = zero_init ? omega * acc[c] : fma(omega, acc[c], dold[c]);
  }
}

template <int B, int NLS>
static hipError_t vanka_t_bn(hipStream_t s, const DevLevel& L, const double* rho, double* d,
                             double omega, int zero_init, int fp32) {
  unsigned grid = (unsigned)((L.n_cells + 3) / 4);
  if (L.sweep_wgs > 0 && (unsigned)L.sweep_wgs < grid) grid = (unsigned)L.sweep_wgs;
  if (fp32)
    launch(k_vanka_t<B, NLS, float>, dim3(grid), dim3(256), 0, s, rho, d, L.cell_sdofs, L.own_ptr, L.own_loc,
                                                  L.inv_off, L.inv_ld, (const float*)L.inv_store,
                                                  omega, zero_init, L.n_cells);
  else
    launch(k_vanka_t<B, NLS, double>, dim3(grid), dim3(256), 0, s, rho, d, L.cell_sdofs, L.own_ptr, L.own_loc,
                                                   L.inv_off, L.inv_ld,
                                                   (const double*)L.inv_store, omega, zero_init,
                                                   L.n_cells);
  return hipGetLastError();
}

template <int B>
static hipError_t vanka_t_b(hipStream_t s, const DevLevel& L, const double* rho, double* d,
                            double omega, int zero_init, int fp32) {
  if (L.n_ls == 21) return vanka_t_bn<B, 21>(s, L, rho, d, omega, zero_init, fp32);
  if (L.n_ls == 85) return vanka_t_bn<B, 85>(s, L, rho, d, omega, zero_init, fp32);
  return hipErrorInvalidValue;
}

hipError_t launch_vanka_cells_t(hipStream_t s, int b, const DevLevel& L, const double* rho,
                                double* d, double omega, int zero_init, int fp32) {
  switch (b) {
    case 1: return vanka_t_b<1>(s, L, rho, d, omega, zero_init, fp32);
    case 2: return vanka_t_b<2>(s, L, rho, d, omega, zero_init, fp32);
    case 3: return vanka_t_b<3>(s, L, rho, d, omega, zero_init, fp32);
    case 4: return vanka_t_b<4>(s, L, rho, d, omega, zero_init, fp32);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Cellwise bilinear forms of two level vectors.  out[T] = sum_l tw[l]
// sum_{alpha, beta} lam[alpha, l] K_T[alpha][beta] x[beta, l] with
// K_T = sum_e kw[e] Kref[kidx[e]] (e in [kptr[T], kptr[T+1]); n_ls x n_ls
// spatial reference matrices): one wavefront per cell, lane j = alpha*B + l
// forms (K_T x)_j with x broadcast from its lane, then a wavefront sum.
// With fidx (per cell: the row k of f that belongs to it, or -1) the cell's
// right-hand-side term is added in the same pass:
//   out[T] = sc * (the form above) + sf * sum_j lam[T's DoF j] f[k][j],
// f in the cell-local order alpha*B + l (the gradient of an outflow loss
// with respect to cell viscosities and an inflow amplitude).
template <int B, int NLS>
__global__ void __launch_bounds__(256) k_cell_contract(
    const double* __restrict__ lam, const double* __restrict__ x,
    const int32_t* __restrict__ csd, int n_cells, const double* __restrict__ Kref,
    const int32_t* __restrict__ kptr, const int32_t* __restrict__ kidx,
    const double* __restrict__ kw, const double* __restrict__ tw, double sc,
    const int32_t* __restrict__ fidx, const double* __restrict__ f, double sf,
    double* __restrict__ out) {
  constexpr int N = B * NLS;
  constexpr int NC = (N + 63) / 64;
  const int lane = threadIdx.x & 63;
  const int T = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (T >= n_cells) return;  // uniform per wavefront
  const int32_t* sd = csd + (int64_t)T * NLS;
  double xv[NC], lv[NC], y[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int j = lane + 64 * c;
    xv[c] = lv[c] = y[c] = 0.0;
    if (j < N) {
      const int be = j / B;
      const int64_t g = (int64_t)sd[be] * B + (j - be * B);
      xv[c] = x[g];
      lv[c] = lam[g];
    }
  }
  for (int e = kptr[T]; e < kptr[T + 1]; ++e) {
    const double* K = Kref + (int64_t)kidx[e] * NLS * NLS;
    const double w = kw[e];
#pragma unroll
    for (int cj = 0; cj < NC; ++cj) {
      const int jn = (N - 64 * cj) < 64 ? (N - 64 * cj) : 64;
      for (int jl = 0; jl < jn; ++jl) {
        const int j = 64 * cj + jl;
        const int beta = j / B, lj = j - beta * B;
        const double xj = w * __shfl(xv[cj], jl, 64);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int o = lane + 64 * c;
          if (o < N && (o - (o / B) * B) == lj) y[c] = fma(K[(o / B) * NLS + beta], xj, y[c]);
        }
      }
    }
  }
  double sacc = 0.0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const int o = lane + 64 * c;
    if (o < N) sacc = fma(tw[o - (o / B) * B] * lv[c], y[c], sacc);
  }
  sacc = wave_sum(sacc);
  double facc = 0.0;
  const int fk = fidx ? fidx[T] : -1;
  if (fk >= 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const int o = lane + 64 * c;
      if (o < N) facc = fma(lv[c], f[(int64_t)fk * N + o], facc);
    }
    facc = wave_sum(facc);
  }
  if (lane == 0) out[T] = fk >= 0 ? fma(sc, sacc, sf * facc) : sc * sacc;
}

// out[k] = sum_j lam[cell k's DoF j] f[k*N + j] (f in the cell-local order
// alpha*B + l) for the listed cells.
template <int B, int NLS>
__global__ void __launch_bounds__(256) k_cell_dot(const double* __restrict__ lam,
                                                  const int32_t* __restrict__ csd,
                                                  const int32_t* __restrict__ cells, int n,
                                                  const double* __restrict__ f,
                                                  double* __restrict__ out) {
  constexpr int N = B * NLS;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (k >= n) return;
  const int32_t* sd = csd + (int64_t)cells[k] * NLS;
  double acc = 0.0;
  for (int j = lane; j < N; j += 64) {
    const int be = j / B;
    acc = fma(lam[(int64_t)sd[be] * B + (j - be * B)], f[(int64_t)k * N + j], acc);
  }
  acc = wave_sum(acc);
  if (lane == 0) out[k] = acc;
}

hipError_t launch_cell_contract(hipStream_t s, int b, const DevLevel& L, const double* lam,
                                const double* x, const double* Kref, const int32_t* kptr,
                                const int32_t* kidx, const double* kw, const double* tw,
                                double sc, const int32_t* fidx, const double* f, double sf,
                                double* out) {
  const unsigned grid = (unsigned)((L.n_cells + 3) / 4);
#define STV_CC(BB, NN)                                                                    \
  k_cell_contract<BB, NN><<<grid, 256, 0, s>>>(lam, x, L.cell_sdofs, L.n_cells, Kref, kptr, \
                                               kidx, kw, tw, sc, fidx, f, sf, out)
  if (L.n_ls == 21) {
    switch (b) { case 1: STV_CC(1, 21); break; case 2: STV_CC(2, 21); break;
                 case 3: STV_CC(3, 21); break; case 4: STV_CC(4, 21); break;
                 default: return hipErrorInvalidValue; }
  } else if (L.n_ls == 85) {
    switch (b) { case 1: STV_CC(1, 85); break; case 2: STV_CC(2, 85); break;
                 case 3: STV_CC(3, 85); break; case 4: STV_CC(4, 85); break;
                 default: return hipErrorInvalidValue; }
  } else {
    return hipErrorInvalidValue;
  }
#undef STV_CC
  return hipGetLastError();
}

hipError_t launch_cell_dot(hipStream_t s, int b, const DevLevel& L, const double* lam,
                           const int32_t* cells, int n, const double* f, double* out) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 3) / 4);
#define STV_CD(BB, NN) k_cell_dot<BB, NN><<<grid, 256, 0, s>>>(lam, L.cell_sdofs, cells, n, f, out)
  if (L.n_ls == 21) {
    switch (b) { case 1: STV_CD(1, 21); break; case 2: STV_CD(2, 21); break;
                 case 3: STV_CD(3, 21); break; case 4: STV_CD(4, 21); break;
                 default: return hipErrorInvalidValue; }
  } else if (L.n_ls == 85) {
    switch (b) { case 1: STV_CD(1, 85); break; case 2: STV_CD(2, 85); break;
                 case 3: STV_CD(3, 85); break; case 4: STV_CD(4, 85); break;
                 default: return hipErrorInvalidValue; }
  } else {
    return hipErrorInvalidValue;
  }
#undef STV_CD
  return hipGetLastError();
}

// y[dof[i]] += sum_{e = ptr[i]}^{ptr[i+1]-1} coef[ck[e]] * f[fi[e]]: cellwise
// terms added into a vector by gathering, one thread per touched DoF, the
// terms of a DoF in the order of its list (deterministic, no atomics).
__global__ void k_cell_scatter(const int64_t* __restrict__ dof, const int32_t* __restrict__ ptr,
                               const int32_t* __restrict__ ck, const int64_t* __restrict__ fi,
                               const double* __restrict__ coef, const double* __restrict__ f,
                               int n_dof, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_dof) return;
  double acc = y[dof[i]];
  for (int e = ptr[i]; e < ptr[i + 1]; ++e) acc = fma(coef[ck[e]], f[fi[e]], acc);
  y[dof[i]] = acc;
}

hipError_t launch_cell_scatter(hipStream_t s, const int64_t* dof, const int32_t* ptr,
                               const int32_t* ck, const int64_t* fi, const double* coef,
                               const double* f, int n_dof, double* y) {
  if (n_dof <= 0) return hipSuccess;
  k_cell_scatter<<<(unsigned)((n_dof + 255) / 256), 256, 0, s>>>(dof, ptr, ck, fi, coef, f,
                                                                 n_dof, y);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Averaged / additive forms: every cell writes its full damped correction
// omega J_T^-1 rho_T to corr[T*n_loc + (alpha*B + l)] (needs every stored
// row); a second kernel sums, per DoF and in cell order, the corrections of
// the cells containing it.
template <int B, typename TS>
__global__ void __launch_bounds__(64) k_vanka_corr(const double* __restrict__ rho,
                                                  double* __restrict__ corr,
                                                  const int32_t* __restrict__ csd, int n_ls,
                                                  const int64_t* __restrict__ inv_off, int ld,
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
    for (int j = 0; j < n_loc; ++j) acc = fma((double)A[(int64_t)i * ld + j], sm[j], acc);
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
  if (pou && e1 > e0) acc /= (double)(e1 - e0);   // rows of directly solved members have no cell
  d[idx] += acc;
}

hipError_t launch_vanka_cells_corr(hipStream_t s, int b, const DevLevel& L, const double* rho,
                                   double omega, int fp32) {
  const size_t shm = sizeof(double) * (size_t)(L.n_ls * b);
#define STV_CORR(BB)                                                                        \
  if (fp32)                                                                                 \
    k_vanka_corr<BB, float><<<L.n_cells, 64, shm, s>>>(rho, L.corr, L.cell_sdofs, L.n_ls,   \
                                                       L.inv_off, L.inv_ld,                 \
                                                       (const float*)L.inv_store, omega);   \
  else                                                                                      \
    k_vanka_corr<BB, double><<<L.n_cells, 64, shm, s>>>(rho, L.corr, L.cell_sdofs, L.n_ls,  \
                                                        L.inv_off, L.inv_ld,                \
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
