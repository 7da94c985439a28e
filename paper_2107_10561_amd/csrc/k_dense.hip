// Dense coarse levels (the direct solve of Algorithm 4.1 on the coarsest
// grid): each coarse matrix is expanded to a dense FP64 array (padded with an
// identity block to a multiple of the panel width), inverted once by blocked
// Gauss-Jordan elimination with partial pivoting, and applied as a dense
// matrix-vector product in every V-cycle.  Every kernel takes a batch index in
// blockIdx.z: a group of equally sized coarse matrices (one per instance of a
// batched hierarchy) is inverted by the same launches, each matrix and work
// buffer at its own stride.
#include "stv_internal.h"
#include "wave.h"

namespace stv {

typedef double stv_d4 __attribute__((ext_vector_type(4)));

#ifndef STV_CHAIN_PRIO
#define STV_CHAIN_PRIO 3
#endif

// The kernels of the dense elimination chain run beside the cell-inverse
// kernels of the same build and are latency bound: their wavefronts take
// the higher issue priority on the SIMDs they share.
__device__ __forceinline__ void chain_priority() {
  if (STV_CHAIN_PRIO > 0) __builtin_amdgcn_s_setprio(STV_CHAIN_PRIO);
}

// Dense copy of member z's rows of its level matrix (columns shifted by the
// member's first row; the blocks of a member couple only its own rows).
template <int B>
__global__ void k_bsr_to_dense(const CoarseDesc* __restrict__ desc, double* __restrict__ A,
                               int64_t sA, int64_t n) {
  const CoarseDesc D = desc[blockIdx.z];
  const int32_t row = blockIdx.x;
  if (row >= D.n_s) return;
  double* Az = A + blockIdx.z * sA;
  const int32_t gr = D.row_off + row;
  for (int32_t q = D.rowptr[gr] + threadIdx.x; q < D.rowptr[gr + 1]; q += blockDim.x) {
    const int64_t c = D.col[q] - D.row_off;
#pragma unroll
    for (int i = 0; i < B; ++i)
#pragma unroll
      for (int l = 0; l < B; ++l)
        Az[((int64_t)row * B + i) * n + c * B + l] = D.val[(int64_t)q * B * B + i * B + l];
  }
}

hipError_t launch_bsr_to_dense(hipStream_t s, int b, const CoarseDesc* desc, int cnt,
                               int32_t max_rows, double* A, int64_t sA, int64_t n) {
  dim3 grid((unsigned)max_rows, 1, (unsigned)cnt);
  switch (b) {
    case 1: k_bsr_to_dense<1><<<grid, 64, 0, s>>>(desc, A, sA, n); break;
    case 2: k_bsr_to_dense<2><<<grid, 64, 0, s>>>(desc, A, sA, n); break;
    case 3: k_bsr_to_dense<3><<<grid, 64, 0, s>>>(desc, A, sA, n); break;
    case 4: k_bsr_to_dense<4><<<grid, 64, 0, s>>>(desc, A, sA, n); break;
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
// (n x NB): one TPB-thread workgroup holds it in registers (thread t owns
// rows t + TPB m) and eliminates it.  The panel columns then hold the columns
// rpiv[p0..] of the accumulated elimination matrix E; every other column j
// is brought up to date by the rank-NB update
//   A(:, j) += (E - I)(:, rpiv[p0+t]) * A(rpiv[p0+t], j)
// with the pivot rows read before it: the panel kernel copies those rows of
// the matrix being updated (S, ncs columns, row stride lds) to Bout once the
// pivots are known, since nothing else writes S while it runs.
// rpiv[p] = -1 marks a step without a nonzero finite pivot (singular).
template <int RPT, int NB, int TPB>
__global__ void __launch_bounds__(TPB) k_gj_panel(double* __restrict__ pbuf, int64_t sP, int64_t n,
                                                  int p0, int* __restrict__ rpiv,
                                                  uint8_t* __restrict__ used, int64_t sV,
                                                  const double* __restrict__ S, int64_t sS,
                                                  int64_t lds, int64_t ncs,
                                                  double* __restrict__ Bout, int64_t sBo) {
  pbuf += blockIdx.z * sP;
  rpiv += blockIdx.z * sV;
  used += blockIdx.z * sV;
  S += blockIdx.z * sS;
  Bout += blockIdx.z * sBo;
  // per step, each wavefront publishes its best candidate (magnitude, row)
  // together with that row's panel values; one barrier, then every thread
  // picks the winner among the NW candidates (double-buffered by step parity)
  constexpr int NW = TPB / 64;
  __shared__ double wbest[2][NW];
  __shared__ int widx[2][NW];
  __shared__ double wrow[2][NW][NB];
  __shared__ int rloc[NB];     // pivot records, written to global memory once at the end
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform, kept in an SGPR
  double P[RPT][NB];
  unsigned umask = 0;   // bit m: row tid + TPB m already used as a pivot
  // 32-bit offsets (n * NB < 2^28) let the loads and stores address from
  // the uniform base pointer instead of holding a 64-bit address per row
  const unsigned nu = (unsigned)n;
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const unsigned i = (unsigned)tid + TPB * m;
#pragma unroll
    for (int t = 0; t < NB; ++t) P[m][t] = (i < nu) ? pbuf[i * NB + t] : 0.0;
    if (i >= nu || used[i]) umask |= 1u << m;
  }
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int par = t & 1;
    double best = -1.0;
    int bm = -1;
#pragma unroll
    for (int m = 0; m < RPT; ++m) {
      const double v = fabs(P[m][t]);
      if (!(umask & (1u << m)) && v > best) { best = v; bm = m; }
    }
    int bi = bm >= 0 ? tid + TPB * bm : 0x7fffffff;
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
      const int mo = bi / TPB;                 // wave-uniform: one scalar-branched write
#pragma unroll
      for (int m = 0; m < RPT; ++m)
        if (m == mo && tid == bi - TPB * m) {
#pragma unroll
          for (int c = 0; c < NB; ++c) wrow[par][wv][c] = P[m][c];
        }
    }
    __syncthreads();
    double mx = wbest[par][0];
    int cand = widx[par][0];
    int win = 0;
#pragma unroll
    for (int w2 = 1; w2 < NW; ++w2) {
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
    const double pv = wrow[par][win][t];
    const double ipiv = (pv != 0.0) ? 1.0 / pv : 0.0;
    const int dr = r - tid;
    // pivot row: (src 0, factor -1/piv); other rows: (own value, factor a_it/piv)
    if constexpr (NB >= 16 && RPT <= NB) {
      // few rows, wide panel: the row factors stay in registers and the
      // pivot-row entries are read from LDS one column at a time (broadcast)
      double f[RPT];
      unsigned isr = 0;
#pragma unroll
      for (int m = 0; m < RPT; ++m) {
        const bool is = (dr == TPB * m);
        if (is) { umask |= 1u << m; isr |= 1u << m; }
        f[m] = is ? -ipiv : P[m][t] * ipiv;
      }
#pragma unroll
      for (int c = 0; c < NB; ++c) {
        const double prc = wrow[par][win][c];
#pragma unroll
        for (int m = 0; m < RPT; ++m) {
          const bool is = (isr >> m) & 1u;
          P[m][c] = (c == t) ? (is ? ipiv : -f[m]) : fma(-f[m], prc, is ? 0.0 : P[m][c]);
        }
      }
    } else {
      // the pivot row stays in registers
      double pr[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) pr[c] = wrow[par][win][c];
#pragma unroll
      for (int m = 0; m < RPT; ++m) {
        const bool is = (dr == TPB * m);
        if (is) umask |= 1u << m;
        const double f = is ? -ipiv : P[m][t] * ipiv;
#pragma unroll
        for (int c = 0; c < NB; ++c)
          P[m][c] = (c == t) ? (is ? ipiv : -f) : fma(-f, pr[c], is ? 0.0 : P[m][c]);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < RPT; ++m) {
    const unsigned i = (unsigned)tid + TPB * m;
    if (i < nu) {
#pragma unroll
      for (int t = 0; t < NB; ++t) pbuf[i * NB + t] = P[m][t];
    }
  }
  if (tid < NB) {
    const int r = rloc[tid];
    rpiv[p0 + tid] = r;
    if (r >= 0) used[r] = 1;
  }
  // pivot rows of S before the update (row r < n always holds when r >= 0)
  for (int64_t e = tid; e < NB * ncs; e += TPB) {
    const int t = (int)(e / ncs);
    const int64_t c = e - t * ncs;
    const int r = rloc[t];
    Bout[e] = r >= 0 ? S[(int64_t)r * lds + c] : 0.0;
  }
}

// out (rows x nb, row-major) = columns [c0, c0+nb) of A (row stride lda).
__global__ void k_gj_load_panel(const double* __restrict__ A, int64_t sA, int64_t lda,
                                int64_t rows, int64_t c0, int nb, double* __restrict__ out,
                                int64_t sO) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * nb) return;
  const int64_t i = e / nb;
  out[blockIdx.z * sO + e] = A[blockIdx.z * sA + i * lda + c0 + (e - i * nb)];
}

static hipError_t load_panel(hipStream_t s, int cnt, const double* A, int64_t sA, int64_t lda,
                             int64_t rows, int64_t c0, int nb, double* out, int64_t sO) {
  dim3 grid((unsigned)((rows * nb + 255) / 256), 1, (unsigned)cnt);
  k_gj_load_panel<<<grid, 256, 0, s>>>(A, sA, lda, rows, c0, nb, out, sO);
  return hipGetLastError();
}

// Pivot rows rpiv[p0..p0+nb) of A (n x n) before an update: Bbuf (nb x n);
// row t of the copy is blockIdx.y, so every load of the copy is independent.
__global__ void k_gj_gather_rows(const double* __restrict__ A, int64_t sA, int64_t n, int p0,
                                 const int* __restrict__ rpiv, int64_t sV,
                                 double* __restrict__ Bbuf, int64_t sB) {
  chain_priority();
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int t = blockIdx.y;
  A += blockIdx.z * sA;
  rpiv += blockIdx.z * sV;
  Bbuf += blockIdx.z * sB;
  // a record outside [0, n) (a missing pivot) gathers zeros; the pivot-record
  // check then reports the member
  const int r = rpiv[p0 + t];
  Bbuf[(int64_t)t * n + j] = (r >= 0 && r < n) ? A[(int64_t)r * n + j] : 0.0;
}

// A(i, j) += sum_t (P(i, t) - [i == rpiv[p0+t]]) * Bbuf(t, j) for j outside the
// panel, A(i, p0+t) = P(i, t) inside it, and the updated columns of the next
// panel are copied to pnext.  A workgroup handles 16 rows x 256 columns: the
// 16 x NB left factor is staged in LDS, each thread keeps its column of the
// right factor in registers, and the rows of A are read and written fully
// coalesced.
template <int NB>
__global__ void __launch_bounds__(256) k_gj_rank_update(double* __restrict__ A, int64_t sA,
                                                        int64_t n, int p0,
                                                        const int* __restrict__ rpiv, int64_t sV,
                                                        const double* __restrict__ pcur,
                                                        double* __restrict__ pnext, int64_t sP,
                                                        const double* __restrict__ Bbuf,
                                                        int64_t sB) {
  __shared__ double W[16][NB];
  A += blockIdx.z * sA;
  rpiv += blockIdx.z * sV;
  pcur += blockIdx.z * sP;
  pnext += blockIdx.z * sP;
  Bbuf += blockIdx.z * sB;
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

// One-level variant: every panel updates the whole matrix (rank NB).
template <int RPT, int NB, int TPB>
static hipError_t gj_blocked(hipStream_t s, const GjWork& w, int64_t n, int cnt) {
  double* pb[2] = {w.P, w.P + n * NB};
  hipError_t e = load_panel(s, cnt, w.A, w.sA, n, n, 0, NB, pb[0], w.sP);
  if (e != hipSuccess) return e;
  int cur = 0;
  for (int64_t p0 = 0; p0 < n; p0 += NB, cur ^= 1) {
    k_gj_panel<RPT, NB, TPB><<<dim3(1, 1, cnt), TPB, 0, s>>>(
        pb[cur], w.sP, n, (int)p0, w.rpiv, w.used, w.sV, w.A, w.sA, n, n, w.B, w.sB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((n + 255) / 256), (unsigned)((n + 15) / 16), (unsigned)cnt);
    k_gj_rank_update<NB><<<grid, 256, 0, s>>>(w.A, w.sA, n, (int)p0, w.rpiv, w.sV, pb[cur],
                                               pb[cur ^ 1], w.sP, w.B, w.sB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Two-level variant.  The columns are processed in slabs of NO: a slab is
// kept in its own contiguous buffer Sb (n x NO) and eliminated by panels of
// NB whose rank-NB updates touch only the slab; the slab then holds the
// columns rpiv[j0..j0+NO) of its accumulated elimination matrix, and the rest
// of the matrix takes one rank-NO update on the FP64 matrix cores.

// Rank-NB update inside the slab: Sb(i, c) += sum_t (pcur(i, t) - [i ==
// rp[t]]) Bin(t, c) for c outside [q0, q0+NB), Sb(i, q0+t) = pcur(i, t); the
// next panel's updated columns are copied to pnext.  64 rows per workgroup.
template <int NB, int NO>
__global__ void __launch_bounds__(256) k_gj_slab_inner(double* __restrict__ Sb, int64_t sS,
                                                       int64_t n, int q0,
                                                       const int* __restrict__ rp, int64_t sV,
                                                       const double* __restrict__ pcur,
                                                       double* __restrict__ pnext, int64_t sP,
                                                       const double* __restrict__ Bin,
                                                       int64_t sBin) {
  constexpr int RG = 256 / NO;   // row lanes per workgroup
  __shared__ double W[64][NB];
  Sb += blockIdx.z * sS;
  rp += blockIdx.z * sV;
  pcur += blockIdx.z * sP;
  pnext += blockIdx.z * sP;
  Bin += blockIdx.z * sBin;
  const int tid = threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.x * 64;
  for (int e = tid; e < 64 * NB; e += 256) {
    const int di = e / NB, t = e - di * NB;
    const int64_t i = i0 + di;
    W[di][t] = (i < n) ? pcur[i * NB + t] - ((i == rp[t]) ? 1.0 : 0.0) : 0.0;
  }
  __syncthreads();
  const int c = tid % NO, rq = tid / NO;
  const bool inpan = (c >= q0 && c < q0 + NB);
  const bool nxt = (c >= q0 + NB && c < q0 + 2 * NB);
  double bcol[NB];
#pragma unroll
  for (int t = 0; t < NB; ++t) bcol[t] = Bin[t * NO + c];
  for (int di = rq; di < 64; di += RG) {
    const int64_t i = i0 + di;
    if (i >= n) break;
    if (inpan) {
      Sb[i * NO + c] = pcur[i * NB + (c - q0)];
      continue;
    }
    double acc = Sb[i * NO + c];
#pragma unroll
    for (int t = 0; t < NB; ++t) acc = fma(W[di][t], bcol[t], acc);
    Sb[i * NO + c] = acc;
    if (nxt) pnext[i * NB + (c - q0 - NB)] = acc;
  }
}

// Rank-NO update of A (n x n, n a multiple of 64) outside the slab:
//   A(i, j) += sum_q (Sb(i, q) - [i == rp[q]]) Bg(q, j),
// the slab's own columns take Sb, and the next slab's updated columns are
// copied to Snext (and its first nbn columns to pnext).  One 64 x 64 tile per
// workgroup; each wavefront owns a 32 x 32 quarter as 2 x 2 accumulator tiles
// of v_mfma_f64_16x16x4f64 (lane l, register v of a tile holds element
// (4v + (l >> 4), l & 15)); the factors pass through LDS 32 columns of K at a
// time, which keeps four workgroups resident per compute unit.
template <int NO>
__global__ void __launch_bounds__(256) k_gj_slab_update(double* __restrict__ A, int64_t sA,
                                                        int64_t n, int64_t j0,
                                                        const int* __restrict__ rp, int64_t sV,
                                                        const double* __restrict__ Sb,
                                                        double* __restrict__ Snext, int64_t sS,
                                                        const double* __restrict__ Bg, int64_t sB,
                                                        double* __restrict__ pnext, int64_t sP,
                                                        int nbn) {
  constexpr int KC = 32;
  chain_priority();
  A += blockIdx.z * sA;
  rp += blockIdx.z * sV;
  Sb += blockIdx.z * sS;
  Snext += blockIdx.z * sS;
  Bg += blockIdx.z * sB;
  pnext += blockIdx.z * sP;
  __shared__ double Ws[64][KC + 1];
  __shared__ double Bs[KC][64 + 2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int64_t i0 = (int64_t)blockIdx.y * 64, jt = (int64_t)blockIdx.x * 64;
  if (jt >= j0 && jt < j0 + NO) {
    for (int e = tid; e < 64 * 32; e += 256) {
      const int r = e >> 5, c = 2 * (e & 31);
      *(double2*)&A[(i0 + r) * n + jt + c] = *(const double2*)&Sb[(i0 + r) * NO + (jt - j0) + c];
    }
    return;
  }
  const int rb = 32 * (w >> 1), cb = 32 * (w & 1), lr = lane >> 4, lc = lane & 15;
  stv_d4 acc[2][2];
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        acc[ti][tj][v] = A[(i0 + rb + 16 * ti + 4 * v + lr) * n + jt + cb + 16 * tj + lc];
  for (int kc = 0; kc < NO; kc += KC) {
    if (kc) __syncthreads();
    // 64 x KC of the left factor and KC x 64 of the right one, 16-byte loads
#pragma unroll
    for (int e = tid; e < 64 * KC / 2; e += 256) {
      const int r = e / (KC / 2), c = 2 * (e % (KC / 2));
      const double2 x = *(const double2*)&Sb[(i0 + r) * NO + kc + c];
      Ws[r][c] = x.x;
      Ws[r][c + 1] = x.y;
    }
#pragma unroll
    for (int e = tid; e < KC * 32; e += 256) {
      const int r = e >> 5, c = 2 * (e & 31);
      *(double2*)&Bs[r][c] = *(const double2*)&Bg[(int64_t)(kc + r) * n + jt + c];
    }
    __syncthreads();
    if (tid < KC) {
      const int r = rp[kc + tid];
      if (r >= i0 && r < i0 + 64) Ws[r - i0][tid] -= 1.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      double a[2], bv[2];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti) a[ti] = Ws[rb + 16 * ti + lc][4 * kk + lr];
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) bv[tj] = Bs[4 * kk + lr][cb + 16 * tj + lc];
#pragma unroll
      for (int ti = 0; ti < 2; ++ti)
#pragma unroll
        for (int tj = 0; tj < 2; ++tj)
          acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], bv[tj], acc[ti][tj], 0, 0, 0);
    }
  }
  const bool nxt = (jt >= j0 + NO && jt < j0 + 2 * NO);
#pragma unroll
  for (int ti = 0; ti < 2; ++ti)
#pragma unroll
    for (int tj = 0; tj < 2; ++tj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t i = i0 + rb + 16 * ti + 4 * v + lr;
        const int64_t j = jt + cb + 16 * tj + lc;
        A[i * n + j] = acc[ti][tj][v];
        if (nxt) {
          const int64_t c = j - j0 - NO;
          Snext[i * NO + c] = acc[ti][tj][v];
          if (c < nbn) pnext[i * nbn + c] = acc[ti][tj][v];
        }
      }
}

// The same rank-NO update for the real form of a complex matrix (rows and
// columns in pairs, every 2 x 2 block [[x, -y], [y, x]]): the left factor,
// the pivot rows and the result keep that structure exactly, so only the
// even row of each pair is computed, and the odd row is written from it
// (odd[2c] = -even[2c + 1], odd[2c + 1] = even[2c]; the partner column sits
// in the neighbouring lane).  Half the MFMAs of k_gj_slab_update: each
// wavefront owns 16 row pairs x 32 columns of the 64 x 64 tile.
template <int NO>
__global__ void __launch_bounds__(256) k_gj_slab_update_cx(double* __restrict__ A, int64_t sA,
                                                           int64_t n, int64_t j0,
                                                           const int* __restrict__ rp, int64_t sV,
                                                           const double* __restrict__ Sb,
                                                           double* __restrict__ Snext, int64_t sS,
                                                           const double* __restrict__ Bg,
                                                           int64_t sB, int ct0, int skip_at,
                                                           int skip_n) {
  constexpr int KC = 32;
  chain_priority();
  A += blockIdx.z * sA;
  rp += blockIdx.z * sV;
  Sb += blockIdx.z * sS;
  Snext += blockIdx.z * sS;
  Bg += blockIdx.z * sB;
  __shared__ double Ws[32][KC + 1];   // even rows of the tile
  __shared__ double Bs[KC][64 + 2];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // column tile: ct0 + x, skipping skip_n tiles from skip_at on (the launch
  // for the next slab's tiles and the one for all others)
  const int ct = ct0 + (int)blockIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * 64, jt = (int64_t)(ct < skip_at ? ct : ct + skip_n) * 64;
  if (jt >= j0 && jt < j0 + NO) {
    for (int e = tid; e < 64 * 32; e += 256) {
      const int r = e >> 5, c = 2 * (e & 31);
      *(double2*)&A[(i0 + r) * n + jt + c] = *(const double2*)&Sb[(i0 + r) * NO + (jt - j0) + c];
    }
    return;
  }
  const int rb = 16 * (w >> 1), cb = 32 * (w & 1), lr = lane >> 4, lc = lane & 15;
  stv_d4 acc[2];
#pragma unroll
  for (int tj = 0; tj < 2; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      acc[tj][v] = A[(i0 + 2 * (rb + 4 * v + lr)) * n + jt + cb + 16 * tj + lc];
  for (int kc = 0; kc < NO; kc += KC) {
    if (kc) __syncthreads();
#pragma unroll
    for (int e = tid; e < 32 * KC / 2; e += 256) {
      const int r = e / (KC / 2), c = 2 * (e % (KC / 2));
      const double2 x = *(const double2*)&Sb[(i0 + 2 * r) * NO + kc + c];
      Ws[r][c] = x.x;
      Ws[r][c + 1] = x.y;
    }
#pragma unroll
    for (int e = tid; e < KC * 32; e += 256) {
      const int r = e >> 5, c = 2 * (e & 31);
      *(double2*)&Bs[r][c] = *(const double2*)&Bg[(int64_t)(kc + r) * n + jt + c];
    }
    __syncthreads();
    if (tid < KC) {
      const int r = rp[kc + tid];
      if (r >= i0 && r < i0 + 64 && !(r & 1)) Ws[(r - i0) >> 1][tid] -= 1.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const double a = Ws[rb + lc][4 * kk + lr];
      double bv[2];
#pragma unroll
      for (int tj = 0; tj < 2; ++tj) bv[tj] = Bs[4 * kk + lr][cb + 16 * tj + lc];
#pragma unroll
      for (int tj = 0; tj < 2; ++tj)
        acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv[tj], acc[tj], 0, 0, 0);
    }
  }
  const bool nxt = (jt >= j0 + NO && jt < j0 + 2 * NO);
#pragma unroll
  for (int tj = 0; tj < 2; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + 2 * (rb + 4 * v + lr);
      const int64_t j = jt + cb + 16 * tj + lc;
      const double x = acc[tj][v];
      const double partner = __shfl_xor(x, 1, 64);
      const double odd = (j & 1) ? partner : -partner;
      A[i * n + j] = x;
      A[(i + 1) * n + j] = odd;
      if (nxt) {
        const int64_t c = j - j0 - NO;
        Snext[i * NO + c] = x;
        Snext[(i + 1) * NO + c] = odd;
      }
    }
}

// The even-row update with 128 x 128 tiles (n a multiple of 128): each
// wavefront owns 16 row pairs x 128 columns (8 accumulator tiles), and the
// factors pass through LDS 32 columns of K at a time.  Per multiply-add half
// the factor traffic of the 64 x 64 tiling, a quarter of its workgroups.
// Held to 128 registers (a few spill) so that its workgroups also run beside
// a cell-inverse workgroup of the concurrent stream, which leaves 128 per
// SIMD; the pivot-row buffer is in LDS sized at launch (kCx128Lds bytes), so
// that the register budget follows the attribute rather than the occupancy
// the static LDS alone would allow.
constexpr unsigned kCx128Lds = 32 * (128 + 2) * sizeof(double);
template <int NO>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_gj_slab_update_cx128(double* __restrict__ A, int64_t sA,
                                                              int64_t n, int64_t j0,
                                                              const int* __restrict__ rp,
                                                              int64_t sV,
                                                              const double* __restrict__ Sb,
                                                              double* __restrict__ Snext,
                                                              int64_t sS,
                                                              const double* __restrict__ Bg,
                                                              int64_t sB, int ct0, int skip_at,
                                                              int skip_n) {
  constexpr int KC = 32, TW = 128;
  chain_priority();
  A += blockIdx.z * sA;
  rp += blockIdx.z * sV;
  Sb += blockIdx.z * sS;
  Snext += blockIdx.z * sS;
  Bg += blockIdx.z * sB;
  __shared__ double Ws[64][KC + 1];      // even rows of the tile
  extern __shared__ double2 zdyn[];
  double(*Bs)[TW + 2] = reinterpret_cast<double(*)[TW + 2]>(zdyn);   // kCx128Lds bytes
  static_assert(KC * (TW + 2) * sizeof(double) == kCx128Lds, "launch-sized LDS");
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int ct = ct0 + (int)blockIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * TW, jt = (int64_t)(ct < skip_at ? ct : ct + skip_n) * TW;
  if (jt >= j0 && jt < j0 + NO) {
    for (int e = tid; e < TW * TW / 2; e += 256) {
      const int r = e / (TW / 2), c = 2 * (e % (TW / 2));
      *(double2*)&A[(i0 + r) * n + jt + c] = *(const double2*)&Sb[(i0 + r) * NO + (jt - j0) + c];
    }
    return;
  }
  const int rb = 16 * w, lr = lane >> 4, lc = lane & 15;
  stv_d4 acc[8];
#pragma unroll
  for (int tj = 0; tj < 8; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      acc[tj][v] = A[(i0 + 2 * (rb + 4 * v + lr)) * n + jt + 16 * tj + lc];
  for (int kc = 0; kc < NO; kc += KC) {
    if (kc) __syncthreads();
#pragma unroll
    for (int e = tid; e < 64 * KC / 2; e += 256) {
      const int r = e / (KC / 2), c = 2 * (e % (KC / 2));
      const double2 x = *(const double2*)&Sb[(i0 + 2 * r) * NO + kc + c];
      Ws[r][c] = x.x;
      Ws[r][c + 1] = x.y;
    }
#pragma unroll
    for (int e = tid; e < KC * TW / 2; e += 256) {
      const int r = e / (TW / 2), c = 2 * (e % (TW / 2));
      *(double2*)&Bs[r][c] = *(const double2*)&Bg[(int64_t)(kc + r) * n + jt + c];
    }
    __syncthreads();
    if (tid < KC) {
      const int r = rp[kc + tid];
      if (r >= i0 && r < i0 + TW && !(r & 1)) Ws[(r - i0) >> 1][tid] -= 1.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KC / 4; ++kk) {
      const double a = Ws[rb + lc][4 * kk + lr];
#pragma unroll
      for (int tj = 0; tj < 8; ++tj)
        acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, Bs[4 * kk + lr][16 * tj + lc], acc[tj],
                                                       0, 0, 0);
    }
  }
  const bool nxt = (jt >= j0 + NO && jt < j0 + 2 * NO);
#pragma unroll
  for (int tj = 0; tj < 8; ++tj)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t i = i0 + 2 * (rb + 4 * v + lr);
      const int64_t j = jt + 16 * tj + lc;
      const double x = acc[tj][v];
      const double partner = __shfl_xor(x, 1, 64);
      const double odd = (j & 1) ? partner : -partner;
      A[i * n + j] = x;
      A[(i + 1) * n + j] = odd;
      if (nxt) {
        const int64_t c = j - j0 - NO;
        Snext[i * NO + c] = x;
        Snext[(i + 1) * NO + c] = odd;
      }
    }
}

template <int RPT, int NB, int TPB, int NO>
static hipError_t gj_slab(hipStream_t s, const GjWork& w, int64_t n, int cnt) {
  double* sb[2] = {w.S, w.S + n * NO};
  double* pb[2] = {w.P, w.P + n * NB};
  hipError_t e = load_panel(s, cnt, w.A, w.sA, n, n, 0, NO, sb[0], w.sS);
  if (e == hipSuccess) e = load_panel(s, cnt, sb[0], w.sS, NO, n, 0, NB, pb[0], w.sP);
  if (e != hipSuccess) return e;
  int cs = 0, cp = 0;
  const unsigned nt = (unsigned)(n / 64);
  for (int64_t j0 = 0; j0 < n; j0 += NO, cs ^= 1) {
    for (int q0 = 0; q0 < NO; q0 += NB, cp ^= 1) {
      k_gj_panel<RPT, NB, TPB><<<dim3(1, 1, cnt), TPB, 0, s>>>(
          pb[cp], w.sP, n, (int)(j0 + q0), w.rpiv, w.used, w.sV, sb[cs], w.sS, NO, NO, w.Bin,
          w.sBin);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
      k_gj_slab_inner<NB, NO><<<dim3(nt, 1, cnt), 256, 0, s>>>(
          sb[cs], w.sS, n, q0, w.rpiv + j0 + q0, w.sV, pb[cp], pb[cp ^ 1], w.sP, w.Bin, w.sBin);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    k_gj_gather_rows<<<dim3((unsigned)((n + 255) / 256), NO, cnt), 256, 0, s>>>(
        w.A, w.sA, n, (int)j0, w.rpiv, w.sV, w.B, w.sB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gj_slab_update<NO><<<dim3(nt, nt, cnt), 256, 0, s>>>(
        w.A, w.sA, n, j0, w.rpiv + j0, w.sV, sb[cs], sb[cs ^ 1], w.sS, w.B, w.sB, pb[cp], w.sP, NB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// Slabs eliminated by panels whose pivot rows are chosen by a tournament
// (tall-skinny pivoting in the manner of communication-avoiding LU): every
// 64-row chunk proposes NB of its rows by partial pivoting on its own rows,
// groups of proposals are merged, again by partial pivoting on the proposed
// rows' panel values, up a tree, and the rows left at the root are the
// panel's pivots R, in the root's pivot order.  The root's LU factors give
// Z = Pb^-1 B'' for the pivot block Pb = S(R, panel) and B'' = S(R, :) with its
// panel columns replaced by the identity; the panel's elimination is then one
// block Gauss-Jordan step,
//   S(R[s], c) <- Z(s, c),
//   S(i, c)    <- [c outside the panel] S(i, c) - S(i, panel) Z(:, c)  (i not in R),
// which equals NB single steps with pivots (R[t], panel column t).  Every
// pivot decision runs inside one wavefront (DPP reductions, no workgroup
// barrier), and one launch per panel applies the previous panel's step,
// proposes the next panel's rows and, in the workgroup that arrives last,
// merges the proposals and computes the next Z.

// Partial pivoting over rows held by the lanes of one wavefront (all 64
// lanes active): lane l holds a row when `avail`, with panel values
// w[0..NB).  Step t takes the available lane of largest |w[t]| (lowest lane
// on ties) or, when no available lane has a positive |w[t]|, the lowest
// available lane (bit t of `zero` set), and eliminates column t from the
// other available lanes.  Lane t (< NB) returns in `mine` the lane taken at
// step t (-1: none left).  The lane taken at step s returns step = s; with
// LU it holds its multipliers in lmul[0..s) and its eliminated row in
// w[s..NB) (the rows taken, in step order, are L U).
template <int NB, bool LU>
__device__ __forceinline__ void wave_select(double (&w)[NB], bool avail, int& mine,
                                            unsigned& zero, double (&lmul)[NB], int& step) {
  const int lane = threadIdx.x & 63;
  mine = -1;
  zero = 0;
  step = -1;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const double v = avail ? fabs(w[t]) : -1.0;
    const double m = wave_max_f64(v);
    const bool nz = m > 0.0;
    int p;
    if (nz) {
      p = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(v == m));
    } else {
      zero |= 1u << t;
      const uint64_t am = __builtin_amdgcn_ballot_w64(avail);
      p = am ? (int)__builtin_ctzll(am) : -1;
    }
    p = __builtin_amdgcn_readfirstlane(p);
    if (lane == t) mine = p;
    if (p < 0) continue;
    if (lane == p) {
      avail = false;
      step = t;
    }
    if (nz) {
      double pr[NB];
#pragma unroll
      for (int c = t; c < NB; ++c) pr[c] = readlane_f64(w[c], p);
      const double f = w[t] * recip_f64(pr[t]);
      if (LU) lmul[t] = f;
      if (avail) {
#pragma unroll
        for (int c = t + 1; c < NB; ++c) w[c] = fma(-f, pr[c], w[c]);
      }
    }
  }
}

// One launch of the tournament schedule on slab S (n x NO, row-major) of
// every matrix z = blockIdx.z; 256 rows per workgroup, 16 wavefronts.
// UPDATE: apply the step of panel q0 (pivots rpiv[j0+q0..], factor Zc),
// then choose the pivots of panel q0+NB (if inside the slab); otherwise only
// choose the pivots of panel q0.  The choice writes rpiv, used and Zn.
template <int NB, int NO, bool UPDATE>
__global__ void __launch_bounds__(1024) k_gj_tour(double* __restrict__ S, int64_t sS, int64_t n,
                                                  int64_t j0, int q0, int* __restrict__ rpiv,
                                                  uint8_t* __restrict__ used, int64_t sV,
                                                  const double* __restrict__ Zc,
                                                  double* __restrict__ Zn, int64_t sZ,
                                                  int* __restrict__ cand, int64_t sC,
                                                  unsigned* __restrict__ counter, int64_t sK) {
  constexpr int RW = 256, NW = 16, FAN = 64 / NB, MAXL = 64, NH = NO / 64, RB = NH == 1 ? 16 : 4;
  chain_priority();
  static_assert(NB == 8 || NB == 16, "panel width");
  static_assert(64 * NO <= RW * (2 * NB + 1), "candidate rows fit the panel buffers");
  // the panel buffers (current panel of the workgroup's rows, next panel)
  // hold the root's candidate rows once the merge has started
  __shared__ double smem[RW * (2 * NB + 1)];
  double(*Acur)[NB] = reinterpret_cast<double(*)[NB]>(smem);
  double(*Anx)[NB + 1] = reinterpret_cast<double(*)[NB + 1]>(smem + RW * NB);
  double* Brow = smem;
  __shared__ int clist[4][NB];
  __shared__ int tl[2][MAXL * NB];
  __shared__ int rootg[64];
  __shared__ double LUs[NB][NB + 1];
  __shared__ int Ll[NB];
  __shared__ unsigned s_last;
  const int z = blockIdx.z;
  S += z * sS;
  rpiv += z * sV;
  used += z * sV;
  Zn += z * sZ;
  cand += z * sC;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t r0 = (int64_t)blockIdx.x * RW;
  const int qn = UPDATE ? q0 + NB : q0;     // panel whose pivots this launch chooses
  double dummy[NB];
  unsigned zf;
  int step, mine;
  if constexpr (UPDATE) {
    Zc += z * sZ;
    // this wavefront's rows wv + NW u; the loads of a batch are issued together
    double old[RB][NH];
    auto load_batch = [&](int u0) {
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int64_t i = r0 + wv + NW * (u0 + u);
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int c = lane + 64 * h;
          old[u][h] = (i < n && !(c >= q0 && c < q0 + NB)) ? S[i * NO + c] : 0.0;
        }
      }
    };
    load_batch(0);
    for (int e = tid; e < RW * NB; e += 1024) {
      const int di = e / NB, t = e - di * NB;
      const int64_t i = r0 + di;
      Acur[di][t] = i < n ? S[i * NO + q0 + t] : 0.0;
    }
    double zc[NH][NB];
#pragma unroll
    for (int h = 0; h < NH; ++h)
#pragma unroll
      for (int t = 0; t < NB; ++t) zc[h][t] = Zc[t * NO + lane + 64 * h];
    int rp[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) rp[t] = rpiv[j0 + q0 + t];
    __syncthreads();
#pragma unroll
    for (int u0 = 0; u0 < 16; u0 += RB) {
      if (u0) load_batch(u0);
#pragma unroll
      for (int u = 0; u < RB; ++u) {
        const int di = wv + NW * (u0 + u);
        const int64_t i = r0 + di;
        if (i >= n) break;
        int s = -1;
#pragma unroll
        for (int t = 0; t < NB; ++t) s = (rp[t] == i) ? t : s;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
          const int c = lane + 64 * h;
          double val;
          if (s >= 0) {
            val = Zc[(int64_t)s * NO + c];
          } else {
            double acc = old[u][h];
#pragma unroll
            for (int t = 0; t < NB; ++t) acc = fma(-Acur[di][t], zc[h][t], acc);
            val = acc;
          }
          S[i * NO + c] = val;
          if (c >= qn && c < qn + NB) Anx[di][c - qn] = val;
        }
      }
    }
    if (qn >= NO) return;                   // last panel of the slab
  } else {
    for (int e = tid; e < RW * NB; e += 1024) {
      const int di = e / NB, t = e - di * NB;
      const int64_t i = r0 + di;
      Anx[di][t] = i < n ? S[i * NO + qn + t] : 0.0;
    }
  }
  __syncthreads();
  // proposals of the four 64-row chunks, merged into one list of NB rows
  if (wv < 4) {
    const int di = 64 * wv + lane;
    const int64_t i = r0 + di;
    const bool av = i < n && !used[i];
    double w[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) w[t] = av ? Anx[di][t] : 0.0;
    wave_select<NB, false>(w, av, mine, zf, dummy, step);
    if (lane < NB) clist[wv][lane] = mine >= 0 ? 64 * wv + mine : -1;
  }
  __syncthreads();
  if (wv == 0) {
    const int li = lane / NB, sl = lane % NB;
    const int di = li < 4 ? clist[li][sl] : -1;
    const bool av = di >= 0;
    double w[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) w[t] = av ? Anx[di][t] : 0.0;
    wave_select<NB, false>(w, av, mine, zf, dummy, step);
    const int rs = __shfl(di, mine >= 0 ? mine : 0, 64);
    if (lane < NB) cand[(int64_t)blockIdx.x * NB + lane] = (mine >= 0 && rs >= 0) ? (int)(r0 + rs) : -1;
  }
  // the workgroup that arrives last merges every workgroup's list; one
  // device-scope release (after the barrier that orders this workgroup's
  // stores) and one acquire per workgroup
  __syncthreads();
  if (tid == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const unsigned last = (atomicAdd(counter + z * sK, 1u) == gridDim.x - 1) ? 1u : 0u;
    if (last) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      atomicExch(counter + z * sK, 0u);
    }
    s_last = last;
  }
  __syncthreads();
  if (!s_last) return;
  int m = (int)gridDim.x, cur = -1;        // cur < 0: lists in cand
  while (m > FAN) {
    const int nodes = (m + FAN - 1) / FAN, nxt = cur == 0 ? 1 : 0;
    for (int j = wv; j < nodes; j += NW) {
      const int li = j * FAN + lane / NB, sl = lane % NB;
      int g = -1;
      if (li < m) g = cur < 0 ? cand[(int64_t)li * NB + sl] : tl[cur][li * NB + sl];
      double w[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) w[t] = g >= 0 ? S[(int64_t)g * NO + qn + t] : 0.0;
      wave_select<NB, false>(w, g >= 0, mine, zf, dummy, step);
      const int gs = __shfl(g, mine >= 0 ? mine : 0, 64);
      if (lane < NB) tl[nxt][j * NB + lane] = mine >= 0 ? gs : -1;
    }
    __syncthreads();
    cur = nxt;
    m = nodes;
  }
  if (tid < 64) {
    const int li = tid / NB;
    rootg[tid] = li < m ? (cur < 0 ? cand[(int64_t)li * NB + tid % NB] : tl[cur][li * NB + tid % NB]) : -1;
  }
  __syncthreads();
  if (wv == 0) {
    // the root: its pivot rows, their LU factors
    const int g = rootg[lane];
    double w[NB], lmul[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      w[t] = g >= 0 ? S[(int64_t)g * NO + qn + t] : 0.0;
      lmul[t] = 0.0;
    }
    wave_select<NB, true>(w, g >= 0, mine, zf, lmul, step);
    const int gs = __shfl(g, mine >= 0 ? mine : 0, 64);
    if (lane < NB) {
      const bool ok = mine >= 0 && !((zf >> lane) & 1u);
      const int r = ok ? gs : -1;
      Ll[lane] = ok ? mine : -1;
      rpiv[j0 + qn + lane] = r;
      if (r >= 0) used[r] = 1;
    }
    if (step >= 0) {
#pragma unroll
      for (int c = 0; c < NB; ++c) LUs[step][c] = c < step ? lmul[c] : w[c];
    }
  } else {
    // meanwhile the other wavefronts stage the candidates' rows of the slab
    for (int e = tid - 64; e < 64 * NO; e += 1024 - 64) {
      const int l = e / NO, c = e - l * NO;
      const int g = rootg[l];
      Brow[e] = g >= 0 ? S[(int64_t)g * NO + c] : 0.0;
    }
  }
  __syncthreads();
  // Z = U^-1 L^-1 B'', one column per thread
  if (tid < NO) {
    const int c = tid;
    const bool inp = c >= qn && c < qn + NB;
    double y[NB];
#pragma unroll
    for (int s = 0; s < NB; ++s) {
      const int l = Ll[s];
      y[s] = inp ? ((c - qn == s) ? 1.0 : 0.0) : (l >= 0 ? Brow[l * NO + c] : 0.0);
    }
#pragma unroll
    for (int s = 1; s < NB; ++s)
#pragma unroll
      for (int t = 0; t < s; ++t) y[s] = fma(-LUs[s][t], y[t], y[s]);
#pragma unroll
    for (int s = NB - 1; s >= 0; --s) {
#pragma unroll
      for (int t = s + 1; t < NB; ++t) y[s] = fma(-LUs[s][t], y[t], y[s]);
      y[s] = y[s] / LUs[s][s];
    }
#pragma unroll
    for (int s = 0; s < NB; ++s) Zn[s * NO + c] = y[s];
  }
}

template <int NB, int NO>
static hipError_t gj_tour(hipStream_t s, const GjWork& w, int64_t n, int cnt) {
  double* sb[2] = {w.S, w.S + n * NO};
  double* zb[2] = {w.Z, w.Z + NB * NO};
  hipError_t e = load_panel(s, cnt, w.A, w.sA, n, n, 0, NO, sb[0], w.sS);
  if (e != hipSuccess) return e;
  const unsigned nwg = (unsigned)((n + 255) / 256), nt = (unsigned)(n / 64);
  int cs = 0, cz = 0;
  for (int64_t j0 = 0; j0 < n; j0 += NO, cs ^= 1) {
    k_gj_tour<NB, NO, false><<<dim3(nwg, 1, cnt), 1024, 0, s>>>(
        sb[cs], w.sS, n, j0, 0, w.rpiv, w.used, w.sV, nullptr, zb[cz], w.sZ, w.cand, w.sC,
        w.counter, w.sK);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    for (int q0 = 0; q0 < NO; q0 += NB, cz ^= 1) {
      k_gj_tour<NB, NO, true><<<dim3(nwg, 1, cnt), 1024, 0, s>>>(
          sb[cs], w.sS, n, j0, q0, w.rpiv, w.used, w.sV, zb[cz], zb[cz ^ 1], w.sZ, w.cand, w.sC,
          w.counter, w.sK);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    k_gj_gather_rows<<<dim3((unsigned)((n + 255) / 256), NO, cnt), 256, 0, s>>>(
        w.A, w.sA, n, (int)j0, w.rpiv, w.sV, w.B, w.sB);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_gj_slab_update<NO><<<dim3(nt, nt, cnt), 256, 0, s>>>(
        w.A, w.sA, n, j0, w.rpiv + j0, w.sV, sb[cs], sb[cs ^ 1], w.sS, w.B, w.sB, sb[cs ^ 1],
        w.sS, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Complex partial pivoting on a wavefront, as wave_select: lane l holds the
// complex row (wr[t], wi[t]), t < NB; the magnitude of a candidate is
// |Re| + |Im|; the multipliers are w[t] / p[t] with the complex quotient.
// With LU the lane taken at step s holds its multipliers in w[0..s) (column
// t of a lane is not read again once step t has eliminated it) and its
// eliminated row in w[s..NB).
template <int NB, bool LU>
__device__ __forceinline__ void wave_select_cx(double (&wr)[NB], double (&wi)[NB], bool avail,
                                               int& mine, unsigned& zero, int& step) {
  const int lane = threadIdx.x & 63;
  mine = -1;
  zero = 0;
  step = -1;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const double v = avail ? fabs(wr[t]) + fabs(wi[t]) : -1.0;
    const double m = wave_max_f64(v);
    const bool nz = m > 0.0;
    int p;
    if (nz) {
      p = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(v == m));
    } else {
      zero |= 1u << t;
      const uint64_t am = __builtin_amdgcn_ballot_w64(avail);
      p = am ? (int)__builtin_ctzll(am) : -1;
    }
    p = __builtin_amdgcn_readfirstlane(p);
    if (lane == t) mine = p;
    if (p < 0) continue;
    if (lane == p) {
      avail = false;
      step = t;
    }
    if (nz) {
      double pr[NB], pi[NB];
#pragma unroll
      for (int c = t; c < NB; ++c) {
        pr[c] = readlane_f64(wr[c], p);
        pi[c] = readlane_f64(wi[c], p);
      }
      const double d = recip_f64(fma(pr[t], pr[t], pi[t] * pi[t]));
      const double fr = fma(wr[t], pr[t], wi[t] * pi[t]) * d;
      const double fi = fma(wi[t], pr[t], -wr[t] * pi[t]) * d;
      if (avail) {
#pragma unroll
        for (int c = t + 1; c < NB; ++c) {
          wr[c] = fma(-fr, pr[c], fma(fi, pi[c], wr[c]));
          wi[c] = fma(-fr, pi[c], fma(-fi, pr[c], wi[c]));
        }
        if (LU) {
          wr[t] = fr;
          wi[t] = fi;
        }
      }
    }
  }
}

// Complex partial pivoting over the 256 threads of a workgroup, one
// candidate row per thread, with the results of wave_select_cx (mine, in the
// threads t < NB: the thread whose row was taken at step t).  At each step
// every wavefront proposes its best row (largest |Re| + |Im| in the column,
// lowest lane on ties) and stages it in LDS with its magnitude; after one
// barrier every thread takes the largest proposal (lowest wavefront on ties)
// and gathers its row: entry c read by lane c, then by readlane.  The staging
// alternates between two buffers: a thread writes a buffer again two steps
// later, after the barrier between, which every thread passes only once it
// has read the buffer.
template <int NB>
struct WgPickCx {
  double2 row[2][4][NB];
  double mag[2][4];
  int who[2][4];   // proposing thread, -1 when the wavefront has no nonzero
  int any[2][4];   // lowest thread of the wavefront still available, -1 if none
};

template <int NB, bool LU>
__device__ __forceinline__ void wg_select_cx(double (&wr)[NB], double (&wi)[NB], bool avail,
                                             int& mine, unsigned& zero, int& step,
                                             WgPickCx<NB>& sh) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  mine = -1;
  zero = 0;
  step = -1;
#pragma unroll
  for (int t = 0; t < NB; ++t) {
    const int b = t & 1;
    const double v = avail ? fabs(wr[t]) + fabs(wi[t]) : -1.0;
    const double m = wave_max_f64(v);
    const uint64_t hit = __builtin_amdgcn_ballot_w64(m > 0.0 && v == m);
    const uint64_t am = __builtin_amdgcn_ballot_w64(avail);
    const int pl = hit ? (int)__builtin_ctzll(hit) : -1;
    if (lane == pl) {
#pragma unroll
      for (int c = t; c < NB; ++c) sh.row[b][wv][c] = make_double2(wr[c], wi[c]);
    }
    if (lane == 0) {
      sh.mag[b][wv] = m;
      sh.who[b][wv] = pl >= 0 ? 64 * wv + pl : -1;
      sh.any[b][wv] = am ? 64 * wv + (int)__builtin_ctzll(am) : -1;
    }
    __syncthreads();
    double best = sh.mag[b][0];
    int bw = 0, first = sh.any[b][3];
#pragma unroll
    for (int w = 1; w < 4; ++w) {
      const double x = sh.mag[b][w];
      if (x > best) {
        best = x;
        bw = w;
      }
    }
#pragma unroll
    for (int w = 2; w >= 0; --w) {
      const int a = sh.any[b][w];
      first = a >= 0 ? a : first;
    }
    const bool nz = __builtin_amdgcn_readfirstlane(best > 0.0 ? 1 : 0) != 0;
    bw = __builtin_amdgcn_readfirstlane(bw);
    int p;
    if (nz) {
      p = sh.who[b][bw];
    } else {
      zero |= 1u << t;
      p = first;
    }
    p = __builtin_amdgcn_readfirstlane(p);
    if (tid == t) mine = p;
    if (p < 0) continue;
    if (tid == p) {
      avail = false;
      step = t;
    }
    if (nz) {
      // the pivot row, entry c in lane c, then by readlane to every lane
      // (entries before t are stale and not used)
      const double2 qv = sh.row[b][bw][lane < NB ? lane : 0];
      double qr[NB], qi[NB];
#pragma unroll
      for (int c = t; c < NB; ++c) {
        qr[c] = readlane_f64(qv.x, c);
        qi[c] = readlane_f64(qv.y, c);
      }
      const double d = recip_f64(fma(qr[t], qr[t], qi[t] * qi[t]));
      const double fr = fma(wr[t], qr[t], wi[t] * qi[t]) * d;
      const double fi = fma(wi[t], qr[t], -wr[t] * qi[t]) * d;
      if (avail) {
#pragma unroll
        for (int c = t + 1; c < NB; ++c) {
          wr[c] = fma(-fr, qr[c], fma(fi, qi[c], wr[c]));
          wi[c] = fma(-fr, qi[c], fma(-fi, qr[c], wi[c]));
        }
        if (LU) {
          wr[t] = fr;
          wi[t] = fi;
        }
      }
    }
  }
}

// The tournament schedule of k_gj_tour on the real form of complex matrices
// (complex row i = real rows 2i, 2i+1; see GjPlan::pair): the pivots are
// complex, 16 per panel of 32 real columns, chosen by complex partial
// pivoting on each workgroup's rows (wave_select_cx) and up a merge tree of
// the workgroups' proposals, 16 lists per node (wg_select_cx over their 256
// rows); the panel step is the complex block step
//   Z = P^-1 B'' (P = pivot rows x panel columns, B'' = pivot rows with the
//   panel columns replaced by the identity), pivot rows <- Z, other rows
//   <- row - (row's panel entries) Z,
// written back in real form.  Complex values are read from the even real
// row of a pair (Re x, -Im x) and both rows are written, so the pair keeps
// its structure exactly.  64 complex rows per workgroup (one chunk), four
// wavefronts: a workgroup needs one wavefront slot per SIMD, so it is
// placed next to the cell-inverse kernels that run concurrently instead of
// waiting for a whole compute unit to drain.  Z is stored complex,
// [16][NO / 2] pairs (re, im).  rpiv receives real rows (2r at real column
// 2t, 2r + 1 at 2t + 1); used flags both rows.
template <int NO, bool UPDATE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_gj_tour_cx(double* __restrict__ S, int64_t sS, int64_t n,
                                                     int64_t j0, int q0, int* __restrict__ rpiv,
                                                     uint8_t* __restrict__ used, int64_t sV,
                                                     const double* __restrict__ Zc,
                                                     double* __restrict__ Zn, int64_t sZ,
                                                     int* __restrict__ cand, int64_t sC,
                                                     unsigned* __restrict__ counter, int64_t sK,
                                                     const double* __restrict__ A, int64_t sA,
                                                     double* __restrict__ Bg, int64_t sB,
                                                     int ngwg) {
  constexpr int NB = 16, RC = 64, NW = 4, NT = 64 * NW, TFAN = NT / NB;
  chain_priority();
  // the last ngwg workgroups of the slab's last launch (ngwg > 0) gather the
  // slab's pivot rows of A (NO / ngwg rows each) for the update that follows,
  // beside the other workgroups' last panel step; rows without a record in
  // [0, n) gather zeros
  const int nwg = (int)gridDim.x - ngwg;
  if ((int)blockIdx.x >= nwg) {
    const int rows = NO / ngwg, z = blockIdx.z;
    const int* rp = rpiv + z * sV + j0;
    const double2* a2 = reinterpret_cast<const double2*>(A + z * sA);
    double2* b2 = reinterpret_cast<double2*>(Bg + z * sB);
    const int64_t h = n / 2;
    for (int t = ((int)blockIdx.x - nwg) * rows, te = t + rows; t < te; ++t) {
      const int r = rp[t];
      const bool ok = r >= 0 && r < n;
      for (int64_t c = threadIdx.x; c < h; c += NT)
        b2[(int64_t)t * h + c] = ok ? a2[(int64_t)r * h + c] : make_double2(0.0, 0.0);
    }
    return;
  }
  constexpr int NOC = NO / 2;                  // complex columns of the slab
  constexpr int LPR = NOC < 64 ? NOC : 64;     // lanes per row in the panel step
  constexpr int RPP = 64 / LPR;                // rows per wavefront and pass
  constexpr int NH = NOC / LPR;                // complex columns per lane
  constexpr int PASSES = RC / (NW * RPP);
  // the root stages the NB chosen rows (Brow) once they are known
  constexpr int NSM = RC * (2 * NB + 1) > NB * NOC ? RC * (2 * NB + 1) : NB * NOC;
  __shared__ double2 smem[NSM];
  double2(*Acur)[NB] = reinterpret_cast<double2(*)[NB]>(smem);
  double2(*Anx)[NB + 1] = reinterpret_cast<double2(*)[NB + 1]>(smem + RC * NB);
  double2* Brow = smem;
  // past Brow, once the chunk's rows (Acur, Anx) are done with: the candidate
  // rows of a merge and the pivot exchange of its selection
  int* candg = reinterpret_cast<int*>(smem + NB * NOC);
  WgPickCx<NB>& pick = *reinterpret_cast<WgPickCx<NB>*>(smem + NB * NOC + NT / 4);
  static_assert(NB * NOC + NT / 4 + (sizeof(WgPickCx<NB>) + 15) / 16 <= NSM, "LDS layout");
  // the previous panel's Z (UPDATE), in LDS sized at launch: kept out of
  // the static size, the register budget follows the four wavefronts per
  // SIMD the attribute asks for (128 registers) rather than the occupancy
  // the LDS would allow, so that a workgroup also fits beside a cell-inverse
  // workgroup of the concurrent stream
  extern __shared__ double2 zdyn[];
  double2(*Zs)[NOC] = reinterpret_cast<double2(*)[NOC]>(zdyn);
  __shared__ double2 LUs[NB][NB + 1];
  __shared__ double2 uinv[NB];                 // 1 / U(s, s)
  __shared__ int Ll[NB];
  __shared__ unsigned s_last;
  const int z = blockIdx.z;
  S += z * sS;
  rpiv += z * sV;
  used += z * sV;
  Zn += z * sZ;
  cand += z * sC;
  counter += z * sK;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t c0 = (int64_t)blockIdx.x * RC, nc = n / 2;
  const int qn = UPDATE ? q0 + 2 * NB : q0;    // real column of the panel chosen here
  const int q0c = q0 / 2, qnc = qn / 2;
  // complex value of entry (complex row ic, complex column cc)
  auto cval = [&](int64_t ic, int cc) {
    const double2 r = *reinterpret_cast<const double2*>(&S[2 * ic * NO + 2 * cc]);
    return make_double2(r.x, -r.y);
  };
  unsigned zf;
  int step, mine;
  // with a next panel, the update runs in two phases: the next panel's
  // columns of every row first (all threads), then, while wavefront 0
  // chooses the workgroup's proposal from them, wavefronts 1..3 update the
  // other columns
  const bool phased = UPDATE && qn < NO;
  if (UPDATE && phased) {
    Zc += z * sZ;
    const double2* Z2 = reinterpret_cast<const double2*>(Zc);
    constexpr int NR = NOC - NB;               // columns outside the next panel
    constexpr int E1 = RC * NB / NT;           // next-panel entries per thread
    constexpr int NT2 = NT - 64, G = 4;        // threads of the second phase, loads in flight
    static_assert(RC * NB % NT == 0, "next-panel entries per thread");
    double2 o1[E1];
#pragma unroll
    for (int i = 0; i < E1; ++i) {
      const int e = tid + NT * i, dx = e / NB, t = e - dx * NB;
      const int64_t ic = c0 + dx;
      o1[i] = ic < nc ? cval(ic, qnc + t) : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < RC * NB; e += NT) {
      const int dx = e / NB, t = e - dx * NB;
      const int64_t ic = c0 + dx;
      Acur[dx][t] = ic < nc ? cval(ic, q0c + t) : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < NB * NOC; e += NT) Zs[e / NOC][e % NOC] = Z2[e];
    int rp[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) rp[t] = rpiv[j0 + q0 + 2 * t] >> 1;   // -1 stays -1
    __syncthreads();
    // entry (row dx, complex column cc) from its old value o: the pivot rows
    // take their row of Z, the others o - (row's panel entries) Z
    auto upd = [&](int dx, int64_t ic, int cc, double2 o) {
      int s = -1;
#pragma unroll
      for (int t = 0; t < NB; ++t) s = (rp[t] == ic) ? t : s;
      double vr = o.x, vi = o.y;
      if (s >= 0) {
        const double2 v = Zs[s][cc];
        vr = v.x;
        vi = v.y;
      } else {
#pragma unroll
        for (int t = 0; t < NB; ++t) {
          const double2 a = Acur[dx][t];
          const double2 zz = Zs[t][cc];
          vr = fma(-a.x, zz.x, fma(a.y, zz.y, vr));
          vi = fma(-a.x, zz.y, fma(-a.y, zz.x, vi));
        }
      }
      *reinterpret_cast<double2*>(&S[2 * ic * NO + 2 * cc]) = make_double2(vr, -vi);
      *reinterpret_cast<double2*>(&S[(2 * ic + 1) * NO + 2 * cc]) = make_double2(vi, vr);
      return make_double2(vr, vi);
    };
#pragma unroll
    for (int i = 0; i < E1; ++i) {
      const int e = tid + NT * i, dx = e / NB, t = e - dx * NB;
      const int64_t ic = c0 + dx;
      Anx[dx][t] = ic < nc ? upd(dx, ic, qnc + t, o1[i]) : make_double2(0.0, 0.0);
    }
    __syncthreads();
    if (wv > 0) {
      for (int e0 = tid - 64; e0 < RC * NR; e0 += NT2 * G) {
        double2 o2[G];
        int dxs[G], ccs[G];
        bool ok[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
          const int e = e0 + NT2 * g;
          const int dx = e < RC * NR ? e / NR : 0, k = e - dx * NR;
          const int cc = k < qnc ? k : k + NB;
          const int64_t ic = c0 + dx;
          dxs[g] = dx;
          ccs[g] = cc;
          ok[g] = e < RC * NR && ic < nc;
          o2[g] = (ok[g] && !(cc >= q0c && cc < q0c + NB)) ? cval(ic, cc) : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int g = 0; g < G; ++g)
          if (ok[g]) (void)upd(dxs[g], c0 + dxs[g], ccs[g], o2[g]);
      }
    }
  } else if constexpr (UPDATE) {
    Zc += z * sZ;
    const double2* Z2 = reinterpret_cast<const double2*>(Zc);
    const int cl = lane % LPR, rl = lane / LPR;
    // this thread's rows and their old values (zero in the panel's columns)
    double2 old[PASSES][NH];
#pragma unroll
    for (int u = 0; u < PASSES; ++u) {
      const int64_t ic = c0 + rl + RPP * (wv + NW * u);
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int cc = cl + LPR * h;
        old[u][h] = (ic < nc && !(cc >= q0c && cc < q0c + NB)) ? cval(ic, cc) : make_double2(0.0, 0.0);
      }
    }
    for (int e = tid; e < RC * NB; e += NT) {
      const int dx = e / NB, t = e - dx * NB;
      const int64_t ic = c0 + dx;
      Acur[dx][t] = ic < nc ? cval(ic, q0c + t) : make_double2(0.0, 0.0);
    }
    for (int e = tid; e < NB * NOC; e += NT) Zs[e / NOC][e % NOC] = Z2[e];
    int rp[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) rp[t] = rpiv[j0 + q0 + 2 * t] >> 1;   // -1 stays -1
    __syncthreads();
#pragma unroll
    for (int u = 0; u < PASSES; ++u) {
      const int dx = rl + RPP * (wv + NW * u);
      const int64_t ic = c0 + dx;
      if (ic >= nc) continue;
      int s = -1;
#pragma unroll
      for (int t = 0; t < NB; ++t) s = (rp[t] == ic) ? t : s;
#pragma unroll
      for (int h = 0; h < NH; ++h) {
        const int cc = cl + LPR * h;
        double vr, vi;
        if (s >= 0) {
          const double2 v = Z2[s * NOC + cc];
          vr = v.x;
          vi = v.y;
        } else {
          vr = old[u][h].x;
          vi = old[u][h].y;
#pragma unroll
          for (int t = 0; t < NB; ++t) {
            const double2 a = Acur[dx][t];
            const double2 zz = Zs[t][cc];
            vr = fma(-a.x, zz.x, fma(a.y, zz.y, vr));
            vi = fma(-a.x, zz.y, fma(-a.y, zz.x, vi));
          }
        }
        *reinterpret_cast<double2*>(&S[2 * ic * NO + 2 * cc]) = make_double2(vr, -vi);
        *reinterpret_cast<double2*>(&S[(2 * ic + 1) * NO + 2 * cc]) = make_double2(vi, vr);
        if (cc >= qnc && cc < qnc + NB) Anx[dx][cc - qnc] = make_double2(vr, vi);
      }
    }
    if (qn >= NO) return;                      // last panel of the slab
  } else {
    for (int e = tid; e < RC * NB; e += NT) {
      const int dx = e / NB, t = e - dx * NB;
      const int64_t ic = c0 + dx;
      Anx[dx][t] = ic < nc ? cval(ic, qnc + t) : make_double2(0.0, 0.0);
    }
  }
  if (!phased) __syncthreads();
  // the workgroup's proposal: NB rows by partial pivoting on its rows
  if (wv == 0) {
    const int64_t ic = c0 + lane;
    const bool av = ic < nc && !used[2 * ic];
    double wr[NB], wi[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const double2 v = av ? Anx[lane][t] : make_double2(0.0, 0.0);
      wr[t] = v.x;
      wi[t] = v.y;
    }
    wave_select_cx<NB, false>(wr, wi, av, mine, zf, step);
    if (lane < NB) cand[(int64_t)blockIdx.x * NB + lane] = mine >= 0 ? (int)(c0 + mine) : -1;
  }
  // merge tree over the workgroups' lists, TFAN children per node: the last
  // child to arrive at a node merges the children's lists into the node's
  // (wg_select_cx over their rows, one per thread, children in index order),
  // so the nodes of one level merge in parallel; the last arrival at the top
  // level (at most TFAN lists) goes on to the root.  Lists of level l follow
  // those of level l - 1 in cand; counters of a level follow those of the
  // level below.
  static_assert(TFAN * NB == NT, "a merge takes one candidate row per thread");
  int m = nwg;                   // lists at the current level
  int node = (int)blockIdx.x;    // this workgroup's list there
  int64_t lev = 0, cb = 0;       // first list and first counter of the level
  for (;;) {
    const bool top = m <= TFAN;
    const int parent = top ? 0 : node / TFAN;
    const int nchild = top ? m : min(TFAN, m - parent * TFAN);
    __syncthreads();
    if (tid == 0) {
      // release this workgroup's rows and list; the last arrival acquires
      // its siblings'
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      unsigned* cn = counter + cb + parent;
      const unsigned last = (atomicAdd(cn, 1u) == (unsigned)nchild - 1u) ? 1u : 0u;
      if (last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        atomicExch(cn, 0u);
      }
      s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    if (top) break;
    const int64_t nlev = lev + m;
    {
      const int k = tid / NB;
      const int g = k < nchild ? cand[(lev + parent * TFAN + k) * NB + tid % NB] : -1;
      candg[tid] = g;
      double wr[NB], wi[NB];
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        const double2 v = g >= 0 ? cval(g, qnc + t) : make_double2(0.0, 0.0);
        wr[t] = v.x;
        wi[t] = v.y;
      }
      wg_select_cx<NB, false>(wr, wi, g >= 0, mine, zf, step, pick);
      if (tid < NB) cand[(nlev + parent) * NB + tid] = mine >= 0 ? candg[mine] : -1;
    }
    cb += (m + TFAN - 1) / TFAN;
    lev = nlev;
    node = parent;
    m = (m + TFAN - 1) / TFAN;
  }
  {
    // the root: its pivot rows, their complex LU factors
    const int k = tid / NB;
    const int g = k < m ? cand[(lev + k) * NB + tid % NB] : -1;
    candg[tid] = g;
    double wr[NB], wi[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const double2 v = g >= 0 ? cval(g, qnc + t) : make_double2(0.0, 0.0);
      wr[t] = v.x;
      wi[t] = v.y;
    }
    wg_select_cx<NB, true>(wr, wi, g >= 0, mine, zf, step, pick);
    if (tid < NB) {
      const bool ok = mine >= 0 && !((zf >> tid) & 1u);
      const int r = ok ? candg[mine] : -1;
      Ll[tid] = ok ? mine : -1;
      rpiv[j0 + qn + 2 * tid] = ok ? 2 * r : -1;
      rpiv[j0 + qn + 2 * tid + 1] = ok ? 2 * r + 1 : -1;
      if (ok) {
        used[2 * (int64_t)r] = 1;
        used[2 * (int64_t)r + 1] = 1;
      }
    }
    if (step >= 0) {
#pragma unroll
      for (int c = 0; c < NB; ++c) LUs[step][c] = make_double2(wr[c], wi[c]);
    }
  }
  __syncthreads();
  if (tid < NB) {
    const double2 u = LUs[tid][tid];
    const double d = 1.0 / fma(u.x, u.x, u.y * u.y);
    uinv[tid] = make_double2(u.x * d, -u.y * d);
  }
  // the chosen rows, in pivot order
  for (int e = tid; e < NB * NOC; e += NT) {
    const int sl = e / NOC, cc = e - sl * NOC;
    const int l = Ll[sl];
    const int g = l >= 0 ? candg[l] : -1;
    Brow[e] = g >= 0 ? cval(g, cc) : make_double2(0.0, 0.0);
  }
  __syncthreads();
  // Z = U^-1 L^-1 B'': four threads per complex column (a quad of lanes),
  // thread j of the quad holding rows j, j + 4, j + 8, j + 12; each
  // substitution step takes the finished row from its owner by a quad
  // broadcast.  Threads past the last column compute on zeros and store
  // nothing.
  {
    constexpr int TPC = 4, RPT = NB / TPC;
    static_assert(NT / TPC >= NOC, "one quad per complex column");
    const int j = tid & (TPC - 1);
    const int cq = tid / TPC;
    const bool cok = cq < NOC;
    const int cc = cok ? cq : 0;
    const bool inp = cc >= qnc && cc < qnc + NB;
    double yr[RPT], yi[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int s = r * TPC + j;
      const double2 v = !cok ? make_double2(0.0, 0.0)
                        : inp ? make_double2((cc - qnc == s) ? 1.0 : 0.0, 0.0)
                              : (Ll[s] >= 0 ? Brow[s * NOC + cc] : make_double2(0.0, 0.0));
      yr[r] = v.x;
      yi[r] = v.y;
    }
    // forward: the multipliers below the diagonal (unit lower factor)
#pragma unroll
    for (int s = 0; s < NB - 1; ++s) {
      const int ro = s / TPC, jo = s % TPC;
      const double br = quad_bcast_f64(yr[ro], jo), bi = quad_bcast_f64(yi[ro], jo);
#pragma unroll
      for (int r = ro; r < RPT; ++r) {
        if (r == ro && j <= jo) continue;
        const double2 f = LUs[r * TPC + j][s];
        yr[r] = fma(-f.x, br, fma(f.y, bi, yr[r]));
        yi[r] = fma(-f.x, bi, fma(-f.y, br, yi[r]));
      }
    }
    // backward: the upper factor, its diagonal by the stored reciprocals
#pragma unroll
    for (int s = NB - 1; s >= 0; --s) {
      const int ro = s / TPC, jo = s % TPC;
      const double2 ui = uinv[s];
      const double qr = fma(yr[ro], ui.x, -yi[ro] * ui.y);
      const double qi = fma(yr[ro], ui.y, yi[ro] * ui.x);
      const double br = quad_bcast_f64(qr, jo), bi = quad_bcast_f64(qi, jo);
      if (j == jo) {
        yr[ro] = br;
        yi[ro] = bi;
      }
#pragma unroll
      for (int r = 0; r <= ro; ++r) {
        if (r == ro && j >= jo) continue;
        const double2 f = LUs[r * TPC + j][s];
        yr[r] = fma(-f.x, br, fma(f.y, bi, yr[r]));
        yi[r] = fma(-f.x, bi, fma(-f.y, br, yi[r]));
      }
    }
    if (cok) {
      double2* Z2 = reinterpret_cast<double2*>(Zn);
#pragma unroll
      for (int r = 0; r < RPT; ++r) Z2[(r * TPC + j) * NOC + cc] = make_double2(yr[r], yi[r]);
    }
  }
}

template <int NO>
static hipError_t gj_tour_cx(hipStream_t s, const GjWork& w, int64_t n, int cnt,
                             const GjAux* aux) {
  constexpr int NBR = 32;                      // real columns per panel
  constexpr unsigned zbytes = (NBR / 2) * (NO / 2) * sizeof(double2);   // Z of a panel
  double* sb[2] = {w.S, w.S + n * NO};
  double* zb[2] = {w.Z, w.Z + NBR * NO};
  hipError_t e = load_panel(s, cnt, w.A, w.sA, n, n, 0, NO, sb[0], w.sS);
  if (e != hipSuccess) return e;
  // 128 real rows per workgroup; the proposals fit the candidate buffer
  // (w.sC = 32 per 256 real rows) and the merge tree (at most 512 lists)
  const unsigned nwg = (unsigned)((n + 127) / 128), nt = (unsigned)(n / 64);
  int cs = 0, cz = 0;
  for (int64_t j0 = 0; j0 < n; j0 += NO, cs ^= 1) {
    k_gj_tour_cx<NO, false><<<dim3(nwg, 1, cnt), 256, 0, s>>>(
        sb[cs], w.sS, n, j0, 0, w.rpiv, w.used, w.sV, nullptr, zb[cz], w.sZ, w.cand, w.sC,
        w.counter, w.sK, nullptr, 0, nullptr, 0, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // slabs of 64: the last launch also gathers the slab's pivot rows of A
    // (one launch fewer per slab), which needs the previous slab's update of
    // the other columns finished; slabs of 128 gather after it, so that the
    // last panel step is not held back by that update
    constexpr bool kFuse = NO == 64;
    for (int q0 = 0; q0 < NO; q0 += NBR, cz ^= 1) {
      const bool last = q0 + NBR >= NO;
      if (kFuse && last && aux && j0 > 0 &&
          (e = hipStreamWaitEvent(s, aux->done_rest, 0)) != hipSuccess)
        return e;
      const int ng = (kFuse && last) ? NO / 4 : 0;
      k_gj_tour_cx<NO, true><<<dim3(nwg + (unsigned)ng, 1, cnt), 256, zbytes, s>>>(
          sb[cs], w.sS, n, j0, q0, w.rpiv, w.used, w.sV, zb[cz], zb[cz ^ 1], w.sZ, w.cand, w.sC,
          w.counter, w.sK, w.A, w.sA, w.B, w.sB, ng);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (!kFuse) {
      // the gather reads whole rows of A: the previous slab's update of the
      // other columns must have finished
      if (aux && j0 > 0 && (e = hipStreamWaitEvent(s, aux->done_rest, 0)) != hipSuccess) return e;
      k_gj_gather_rows<<<dim3((unsigned)((n + 255) / 256), NO, cnt), 256, 0, s>>>(
          w.A, w.sA, n, (int)j0, w.rpiv, w.sV, w.B, w.sB);
      if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // 128 x 128 tiles when the order allows (slabs of 128), else 64 x 64
    const bool big = NO % 128 == 0 && n % 128 == 0;
    const int TS = big ? 128 : 64;
    const unsigned ntt = (unsigned)(n / TS);
    const int nst = (int)(NO / TS), nxt0 = (int)((j0 + NO) / TS);
    const int nnext = j0 + NO < n ? nst : 0;
    auto update = [&](unsigned gx, int ct0, int skip_at, int skip_n, hipStream_t st) {
      if (big)
        k_gj_slab_update_cx128<NO><<<dim3(gx, ntt, cnt), 256, kCx128Lds, st>>>(
            w.A, w.sA, n, j0, w.rpiv + j0, w.sV, sb[cs], sb[cs ^ 1], w.sS, w.B, w.sB, ct0, skip_at,
            skip_n);
      else
        k_gj_slab_update_cx<NO><<<dim3(gx, ntt, cnt), 256, 0, st>>>(
            w.A, w.sA, n, j0, w.rpiv + j0, w.sV, sb[cs], sb[cs ^ 1], w.sS, w.B, w.sB, ct0, skip_at,
            skip_n);
      return hipGetLastError();
    };
    if (!aux || nnext == 0) {
      if ((e = update(ntt, 0, (int)ntt, 0, s)) != hipSuccess) return e;
      continue;
    }
    // look-ahead: the next slab's columns first (its panels start at once),
    // the other columns on the second stream, concurrent with those panels
    if ((e = update((unsigned)nnext, nxt0, (int)ntt, 0, s)) != hipSuccess) return e;
    if ((e = hipEventRecord(aux->next_ready, s)) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(aux->s2, aux->next_ready, 0)) != hipSuccess) return e;
    if ((e = update(ntt - (unsigned)nnext, 0, nxt0, nnext, aux->s2)) != hipSuccess) return e;
    if ((e = hipEventRecord(aux->done_rest, aux->s2)) != hipSuccess) return e;
  }
  if (aux && n > NO && (e = hipStreamWaitEvent(s, aux->done_rest, 0)) != hipSuccess) return e;
  return hipSuccess;
}

// Panel configurations (panel width, threads, rows per thread, slab width);
// the largest order each one holds is RPT * TPB.
struct GjCfg { int nb, tpb, rpt, no; };
static const GjCfg kCfg1[3] = {{12, 512, 5, 0}, {8, 512, 10, 0}, {4, 768, 15, 0}};
static const GjCfg kCfg2[3] = {{8, 512, 5, 64}, {8, 512, 10, 64}, {4, 768, 15, 128}};

GjPlan gj_plan(int64_t n, int algo, bool pair) {
  GjPlan p{};
  p.algo = algo == 0 ? ((n > 256) ? 3 : 1) : algo;
  if (p.algo == 3) {
    // tournament panels of 16 (16 complex pivots, 32 real columns, for the
    // real form of a complex matrix) in slabs of 64 (128 above order 5120);
    // the merge tree holds up to 256 workgroup lists of 256 real rows
    p.cfg = n > 5120 ? 1 : 0;
    p.pair = pair;
    p.nb = pair ? 32 : 16;
    p.no = p.cfg ? 128 : 64;
    p.pad = p.no;
    p.max_n = 65536;
    return p;
  }
  const GjCfg* cfg = p.algo == 1 ? kCfg1 : kCfg2;
  p.cfg = 2;
  for (int c = 0; c < 3; ++c) {
    const int pad = p.algo == 1 ? cfg[c].nb : cfg[c].no;
    if ((n + pad - 1) / pad * pad <= (int64_t)cfg[c].rpt * cfg[c].tpb) { p.cfg = c; break; }
  }
  p.nb = cfg[p.cfg].nb;
  p.no = cfg[p.cfg].no;
  p.pad = p.algo == 1 ? p.nb : p.no;
  p.max_n = (int64_t)cfg[p.cfg].rpt * cfg[p.cfg].tpb;
  return p;
}

// cnt matrices of order n (a multiple of plan.pad, at most plan.max_n) at
// the strides of w.
hipError_t launch_gj(hipStream_t s, const GjPlan& p, const GjWork& w, int64_t n, int cnt,
                     const GjAux* aux) {
  if (n > p.max_n || n % p.pad || cnt < 1 || (p.pair && (p.algo != 3 || n % 2)))
    return hipErrorInvalidValue;
  if (p.algo == 1) {
    switch (p.cfg) {
      case 0: return gj_blocked<5, 12, 512>(s, w, n, cnt);
      case 1: return gj_blocked<10, 8, 512>(s, w, n, cnt);
      default: return gj_blocked<15, 4, 768>(s, w, n, cnt);
    }
  }
  if (p.algo == 3 && p.pair)
    return p.cfg ? gj_tour_cx<128>(s, w, n, cnt, aux) : gj_tour_cx<64>(s, w, n, cnt, aux);
  if (p.algo == 3)
    return p.cfg ? gj_tour<16, 128>(s, w, n, cnt) : gj_tour<16, 64>(s, w, n, cnt);
  switch (p.cfg) {
    case 0: return gj_slab<5, 8, 512, 64>(s, w, n, cnt);
    case 1: return gj_slab<10, 8, 512, 64>(s, w, n, cnt);
    default: return gj_slab<15, 4, 768, 128>(s, w, n, cnt);
  }
}

// Identity on the padding rows [n_s*b, n) of every member.
__global__ void k_set_diag(const CoarseDesc* __restrict__ desc, int b, double* __restrict__ A,
                           int64_t sA, int64_t n) {
  const int64_t i = (int64_t)desc[blockIdx.z].n_s * b + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) A[blockIdx.z * sA + i * n + i] = 1.0;
}

hipError_t launch_set_diag(hipStream_t s, const CoarseDesc* desc, int cnt, int b, double* A,
                           int64_t sA, int64_t n) {
  dim3 grid((unsigned)((n + 255) / 256), 1, (unsigned)cnt);
  k_set_diag<<<grid, 256, 0, s>>>(desc, b, A, sA, n);
  return hipGetLastError();
}

// Dense diagonal block of a time-decoupled coarse member (kdesc[z]) in real
// form: B[2s + a, 2s' + c] = T[a][c] m + delta_ac a (a, c < 2) for every
// block (s, s') of the member's spatial pattern; one workgroup per spatial
// row, two 16-byte stores per block.
__global__ void k_kron_block_dense(const KronBlockDesc* __restrict__ kdesc,
                                   double* __restrict__ A, int64_t sA, int64_t n) {
  const KronBlockDesc D = kdesc[blockIdx.z];
  const int32_t row = blockIdx.x;
  if (row >= D.n_s) return;
  double* Az = A + blockIdx.z * sA;
  const int32_t gr = D.row_off + row;
  for (int32_t q = D.rowptr[gr] + threadIdx.x; q < D.rowptr[gr + 1]; q += blockDim.x) {
    const int64_t c = D.col[q] - D.row_off;
    const double m = D.ma[2 * (int64_t)q], a = D.ma[2 * (int64_t)q + 1];
    *reinterpret_cast<double2*>(&Az[2 * (int64_t)row * n + 2 * c]) =
        make_double2(fma(D.t[0], m, a), D.t[1] * m);
    *reinterpret_cast<double2*>(&Az[(2 * (int64_t)row + 1) * n + 2 * c]) =
        make_double2(D.t[2] * m, fma(D.t[3], m, a));
  }
}

hipError_t launch_kron_block_dense(hipStream_t s, const KronBlockDesc* kdesc, int cnt,
                                   int32_t max_rows, double* A, int64_t sA, int64_t n) {
  dim3 grid((unsigned)max_rows, 1, (unsigned)cnt);
  k_kron_block_dense<<<grid, 64, 0, s>>>(kdesc, A, sA, n);
  return hipGetLastError();
}

// d = J^-1 r for time-decoupled coarse members (kc[z]) from their blocks'
// inverses, without forming J^-1: with z(s', q) = sum_l W[q][l] r(s', l),
//   y_p(s, a) = sum_{s', c < sz_p} Binv_p[2s + a, 2s' + c] z(s', f_p + c),
//   d(s, i)   = sum_p sum_{a < sz_p} V[i][f_p + a] y_p(s, a).
// Binv_p is read where the elimination left it, Binv_p[i, j] =
// S_p[rpiv_p[i], rinv_p[j]]: row 2s of Binv_p is row rpiv_p[2s] of S_p, and
// S_p's columns 2c, 2c + 1 belong to the spatial column s' = rpiv_p[2c] / 2
// (pivot records pair real rows 2r, 2r + 1 with real columns 2t, 2t + 1).
// The block of a complex pair is the real form of a complex matrix, every
// 2 x 2 block [[x, -y], [y, x]] (exactly so: the elimination keeps the
// structure), so its even rows hold the whole inverse: with
// (e0, e1) = (Binv_p[2s, 2s'], Binv_p[2s, 2s' + 1]),
//   y(s, 0) += e0 z0 + e1 z1,  y(s, 1) += e0 z1 - e1 z0.
// The block of a real eigenvalue holds two uncoupled copies; its even rows
// and columns are read.  So the complex inverse is read once (half the
// bytes of the real form of order b n_s).  A block eliminated with real
// pivots (paired[p] = 0: the schedules for small orders) has no such
// pairing: there every real column c of S_p belongs to Binv_p's column
// j = rpiv_p[c] (s' = j / 2, time component j % 2), and both rows of the
// pair are read.  One workgroup per spatial row s: thread t takes the
// columns t, t + 256, ... (coalesced), z is formed from r on the way (r
// stays in the caches), the partial sums meet in LDS and the first b
// threads form d(s, .).
template <int B>
__global__ void __launch_bounds__(256) k_kron_coarse_gemv(const KronCoarse* __restrict__ kc,
                                                         const double* __restrict__ r,
                                                         double* __restrict__ d) {
  const KronCoarse* K = kc + blockIdx.z;
  const int32_t n_s = K->n_s;
  const int32_t s = blockIdx.x;
  if (s >= n_s) return;
  const int nblk = K->nblk;
  const double* rz = r + (int64_t)K->row_off * B;
  double acc[B][2];
#pragma unroll
  for (int p = 0; p < B; ++p) {
    acc[p][0] = acc[p][1] = 0.0;
    if (p >= nblk) continue;
    const int f = K->first[p];
    const bool pair = K->sz[p] == 2;
    const int* rp = K->rpiv[p];
    const double* row = K->S[p] + (int64_t)rp[2 * s] * K->ld[p];
    double w0[B], w1[B];
#pragma unroll
    for (int l = 0; l < B; ++l) {
      w0[l] = K->W[f * B + l];
      w1[l] = pair ? K->W[(f + 1) * B + l] : 0.0;
    }
    if (!K->paired[p]) {
      const double* row1 = pair ? K->S[p] + (int64_t)rp[2 * s + 1] * K->ld[p] : row;
      for (int32_t c = threadIdx.x; c < 2 * n_s; c += 256) {
        const int j = rp[c];
        const int64_t sp = j >> 1;
        const bool odd = j & 1;
        if (odd && !pair) continue;            // the second copy of a real block
        double zc = 0.0;
#pragma unroll
        for (int l = 0; l < B; ++l) zc = fma(odd ? w1[l] : w0[l], rz[sp * B + l], zc);
        acc[p][0] = fma(row[c], zc, acc[p][0]);
        if (pair) acc[p][1] = fma(row1[c], zc, acc[p][1]);
      }
      continue;
    }
    for (int32_t c = threadIdx.x; c < n_s; c += 256) {
      const int64_t sp = rp[2 * c] >> 1;
      double z0 = 0.0, z1 = 0.0;
#pragma unroll
      for (int l = 0; l < B; ++l) {
        const double v = rz[sp * B + l];
        z0 = fma(w0[l], v, z0);
        z1 = fma(w1[l], v, z1);
      }
      if (pair) {
        const double2 e = *reinterpret_cast<const double2*>(row + 2 * (int64_t)c);
        acc[p][0] = fma(e.x, z0, fma(e.y, z1, acc[p][0]));
        acc[p][1] = fma(e.x, z1, fma(-e.y, z0, acc[p][1]));
      } else {
        acc[p][0] = fma(row[2 * (int64_t)c], z0, acc[p][0]);
      }
    }
  }
  __shared__ double red[4][B][2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int p = 0; p < B; ++p)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      double v = acc[p][a];
#pragma unroll
      for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
      if (lane == 0) red[wv][p][a] = v;
    }
  __syncthreads();
  if (threadIdx.x < B) {
    const int i = threadIdx.x;
    double out = 0.0;
    for (int p = 0; p < nblk; ++p) {
      const int f = K->first[p];
      for (int a = 0; a < K->sz[p]; ++a) {
        const double y = (red[0][p][a] + red[1][p][a]) + (red[2][p][a] + red[3][p][a]);
        out = fma(K->V[i * B + f + a], y, out);
      }
    }
    d[((int64_t)K->row_off + s) * B + i] = out;
  }
}

// Block p's part of d = J^-T r for the same members (the direct solve of the
// transposed coarse matrix): with u(s, q) = sum_i V[i][q] r(s, i),
//   w_p(s', c) = sum_{s, a < sz_p} Binv_p[2s + a, 2s' + c] u(s, f_p + a),
//   d(s', l) (+)= sum_{c < sz_p} W[f_p + c][l] w_p(s', c)
// (assigned for p = 0, added for p > 0: one launch per block, in order).
// For a pair, from the even rows, w(s', 0) += e0 u0 - e1 u1 and
// w(s', 1) += e1 u0 + e0 u1.  Thread per column pair 2t, 2t + 1 of S_p
// (coalesced), which belongs to s' = rpiv_p[2t] / 2; the even rows 2rho of
// S_p in order, row 2rho being row 2s of Binv_p for s = rinv_p[2rho] / 2.
// A block eliminated with real pivots: thread per s', its columns
// rinv_p[2s'], rinv_p[2s' + 1] of S_p, every row rho of S_p (row
// i = rinv_p[rho] of Binv_p: s = i / 2, time component i % 2).
template <int B>
__global__ void __launch_bounds__(256) k_kron_coarse_gemv_t(const KronCoarse* __restrict__ kc,
                                                           int p, const double* __restrict__ r,
                                                           double* __restrict__ d) {
  const KronCoarse* K = kc + blockIdx.z;
  const int32_t n_s = K->n_s;
  const int32_t t = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x);
  if (t >= n_s || p >= K->nblk) return;
  const int f = K->first[p];
  const bool pair = K->sz[p] == 2;
  const int* rp = K->rpiv[p];
  const int* ri = K->rinv[p];
  const double* S = K->S[p];
  const int64_t ld = K->ld[p];
  const double* rz = r + (int64_t)K->row_off * B;
  double v0[B], v1[B];
#pragma unroll
  for (int i = 0; i < B; ++i) {
    v0[i] = K->V[i * B + f];
    v1[i] = pair ? K->V[i * B + f + 1] : 0.0;
  }
  double w0 = 0.0, w1 = 0.0;
  if (!K->paired[p]) {
    const int64_t c0 = ri[2 * t], c1 = pair ? ri[2 * t + 1] : c0;
    for (int32_t rho = 0; rho < 2 * n_s; ++rho) {
      const int i = ri[rho];
      const int64_t s = i >> 1;
      const bool odd = i & 1;
      if (odd && !pair) continue;              // the second copy of a real block
      double u = 0.0;
#pragma unroll
      for (int q = 0; q < B; ++q) u = fma(odd ? v1[q] : v0[q], rz[s * B + q], u);
      const double* Sr = S + (int64_t)rho * ld;
      w0 = fma(Sr[c0], u, w0);
      if (pair) w1 = fma(Sr[c1], u, w1);
    }
    double* dz = d + ((int64_t)K->row_off + t) * B;
#pragma unroll
    for (int l = 0; l < B; ++l) {
      double out = K->W[f * B + l] * w0;
      if (pair) out = fma(K->W[(f + 1) * B + l], w1, out);
      dz[l] = p > 0 ? dz[l] + out : out;
    }
    return;
  }
#pragma unroll 4
  for (int32_t rho = 0; rho < n_s; ++rho) {
    const int64_t s = ri[2 * rho] >> 1;
    double u0 = 0.0, u1 = 0.0;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const double v = rz[s * B + i];
      u0 = fma(v0[i], v, u0);
      u1 = fma(v1[i], v, u1);
    }
    const double* e = S + 2 * (int64_t)rho * ld + 2 * (int64_t)t;
    if (pair) {
      const double2 ee = *reinterpret_cast<const double2*>(e);
      w0 = fma(ee.x, u0, fma(-ee.y, u1, w0));
      w1 = fma(ee.y, u0, fma(ee.x, u1, w1));
    } else {
      w0 = fma(e[0], u0, w0);
    }
  }
  const int64_t sp = rp[2 * t] >> 1;
  double* dz = d + ((int64_t)K->row_off + sp) * B;
#pragma unroll
  for (int l = 0; l < B; ++l) {
    double out = K->W[f * B + l] * w0;
    if (pair) out = fma(K->W[(f + 1) * B + l], w1, out);
    dz[l] = p > 0 ? dz[l] + out : out;
  }
}

hipError_t launch_kron_coarse_apply(hipStream_t s, int b, const KronCoarse* kc, int cnt,
                                    int max_blocks, int32_t max_ns, int transposed,
                                    const double* r, double* d) {
  if (cnt < 1 || max_ns < 1) return hipSuccess;
  if (b < 2 || b > 4) return hipErrorInvalidValue;
  if (!transposed) {
    const dim3 grid((unsigned)max_ns, 1, (unsigned)cnt);
    if (b == 2) launch(k_kron_coarse_gemv<2>, grid, dim3(256), 0, s, kc, r, d);
    else if (b == 3) launch(k_kron_coarse_gemv<3>, grid, dim3(256), 0, s, kc, r, d);
    else launch(k_kron_coarse_gemv<4>, grid, dim3(256), 0, s, kc, r, d);
    return hipGetLastError();
  }
  const dim3 grid((unsigned)((max_ns + 255) / 256), 1, (unsigned)cnt);
  for (int p = 0; p < max_blocks; ++p) {
    if (b == 2) launch(k_kron_coarse_gemv_t<2>, grid, dim3(256), 0, s, kc, p, r, d);
    else if (b == 3) launch(k_kron_coarse_gemv_t<3>, grid, dim3(256), 0, s, kc, p, r, d);
    else launch(k_kron_coarse_gemv_t<4>, grid, dim3(256), 0, s, kc, p, r, d);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Member z's inverse (n0 x n0, row-major, at desc.inv_off of out):
// out(i, j) = S(rpiv[i], rinv[j]) from the in-place result S (order n).
__global__ void k_gj_unpermute(const double* __restrict__ S, int64_t sA, int64_t n,
                               const int* __restrict__ rpiv, const int* __restrict__ rinv,
                               int64_t sV, const CoarseDesc* __restrict__ desc, int b,
                               double* __restrict__ out) {
  const CoarseDesc D = desc[blockIdx.z];
  const int64_t n0 = (int64_t)D.n_s * b;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (i >= n0 || j >= n0) return;
  const int* rp = rpiv + blockIdx.z * sV;
  const int* ri = rinv + blockIdx.z * sV;
  const int r = rp[i], c = ri[j];   // -1 only in a record the verdict rejects
  out[D.inv_off + i * n0 + j] =
      (r >= 0 && c >= 0) ? S[blockIdx.z * sA + (int64_t)r * n + c] : __builtin_nan("");
}

// One workgroup per member: rinv <- -1, then rinv[rpiv[p]] = p for every
// valid entry; a duplicate row, an entry outside [0, n) or a padding row
// taken by a real column sets the member's verdict.
__global__ void __launch_bounds__(1024) k_gj_invert_perm(const int* __restrict__ rpiv, int64_t sV,
                                                         int64_t n,
                                                         const CoarseDesc* __restrict__ desc,
                                                         int b, int* __restrict__ rinv,
                                                         int* __restrict__ verdict) {
  __shared__ int bad;
  const int z = blockIdx.x;
  const int64_t n0 = (int64_t)desc[z].n_s * b;
  const int* rp = rpiv + z * sV;
  int* ri = rinv + z * sV;
  if (threadIdx.x == 0) bad = 0;
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) ri[p] = -1;
  __syncthreads();
  for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
    const int r = rp[p];
    bool ok = r >= 0 && r < n && !(p < n0 && r >= n0);
    if (ok) ok = atomicCAS(&ri[r], -1, (int)p) == -1;
    if (!ok) atomicOr(&bad, 1);
  }
  __syncthreads();
  if (threadIdx.x == 0) verdict[z] = bad;
}

hipError_t launch_gj_invert_perm(hipStream_t s, const int* rpiv, int64_t sV, int64_t n,
                                 const CoarseDesc* desc, int cnt, int b, int* rinv,
                                 int* verdict) {
  k_gj_invert_perm<<<(unsigned)cnt, 1024, 0, s>>>(rpiv, sV, n, desc, b, rinv, verdict);
  return hipGetLastError();
}

__global__ void k_first_flag(const uint8_t* __restrict__ flag, int64_t n, int* out) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n && flag[c]) atomicMin(out, (int)c);
}

hipError_t launch_first_flag(hipStream_t s, const uint8_t* flag, int64_t n, int* out) {
  if (n <= 0) return hipSuccess;
  k_first_flag<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(flag, n, out);
  return hipGetLastError();
}

hipError_t launch_gj_unpermute(hipStream_t s, const double* S, int64_t sA, int64_t n,
                               const int* rpiv, const int* rinv, int64_t sV,
                               const CoarseDesc* desc, int cnt, int b, int64_t max_n0,
                               double* out) {
  dim3 grid((unsigned)((max_n0 + 255) / 256), (unsigned)max_n0, (unsigned)cnt), block(256);
  k_gj_unpermute<<<grid, block, 0, s>>>(S, sA, n, rpiv, rinv, sV, desc, b, out);
  return hipGetLastError();
}

// y = A x on every member's rows: one wavefront per row of a member's
// row-major dense inverse (member z in blockIdx.z).
__global__ void __launch_bounds__(256) k_dense_gemv(const CoarseDesc* __restrict__ desc, int b,
                                                    const double* __restrict__ inv,
                                                    const double* __restrict__ x,
                                                    double* __restrict__ y) {
  const CoarseDesc D = desc[blockIdx.z];
  const int64_t n0 = (int64_t)D.n_s * b;
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n0) return;
  const int64_t vo = (int64_t)D.row_off * b;
  const double* Ar = inv + D.inv_off + row * n0;
  const double* xz = x + vo;
  double acc = 0.0;
  for (int64_t j = lane; j < n0; j += 64) acc = fma(Ar[j], xz[j], acc);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) y[vo + row] = acc;
}

// y = A^T x on every member's rows (the direct solve of the transposed
// coarse matrix, (A^T)^-1 = (A^-1)^T): thread per column, coalesced over the
// columns of each row of the stored inverse.
__global__ void __launch_bounds__(256) k_dense_gemv_t(const CoarseDesc* __restrict__ desc, int b,
                                                      const double* __restrict__ inv,
                                                      const double* __restrict__ x,
                                                      double* __restrict__ y) {
  const CoarseDesc D = desc[blockIdx.z];
  const int64_t n0 = (int64_t)D.n_s * b;
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n0) return;
  const int64_t vo = (int64_t)D.row_off * b;
  const double* A = inv + D.inv_off;
  const double* xz = x + vo;
  double acc = 0.0;
  for (int64_t i = 0; i < n0; ++i) acc = fma(A[i * n0 + j], xz[i], acc);
  y[vo + j] = acc;
}

hipError_t launch_dense_gemv_t(hipStream_t s, const CoarseDesc* desc, int cnt, int b,
                               int64_t max_n0, const double* inv, const double* x, double* y) {
  if (cnt < 1) return hipSuccess;
  dim3 grid((unsigned)((max_n0 + 255) / 256), 1, (unsigned)cnt);
  launch(k_dense_gemv_t, dim3(grid), dim3(256), 0, s, desc, b, inv, x, y);
  return hipGetLastError();
}

hipError_t launch_dense_gemv(hipStream_t s, const CoarseDesc* desc, int cnt, int b,
                             int64_t max_n0, const double* inv, const double* x, double* y) {
  if (cnt < 1) return hipSuccess;
  dim3 grid((unsigned)((max_n0 + 3) / 4), 1, (unsigned)cnt);
  launch(k_dense_gemv, dim3(grid), dim3(256), 0, s, desc, b, inv, x, y);
  return hipGetLastError();
}

}  // namespace stv
