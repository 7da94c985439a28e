// Dense coarse levels (the direct solve of Algorithm 4.1 on the coarsest
// grid): each coarse matrix is expanded to a dense FP64 array (padded with an
// identity block to a multiple of the panel width), inverted once by blocked
// Gauss-Jordan elimination with partial pivoting, and applied as a dense
// matrix-vector product in every V-cycle.  Every kernel takes a batch index in
// blockIdx.z: a group of equally sized coarse matrices (one per instance of a
// batched hierarchy) is inverted by the same launches, each matrix and work
// buffer at its own stride.
#include "stv_internal.h"

namespace stv {

typedef double stv_d4 __attribute__((ext_vector_type(4)));

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

// Pivot rows rpiv[p0..p0+nb) of A (n x n) before an update: Bbuf (nb x n).
__global__ void k_gj_gather_rows(const double* __restrict__ A, int64_t sA, int64_t n, int p0,
                                 int nb, const int* __restrict__ rpiv, int64_t sV,
                                 double* __restrict__ Bbuf, int64_t sB) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  A += blockIdx.z * sA;
  rpiv += blockIdx.z * sV;
  Bbuf += blockIdx.z * sB;
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
    k_gj_gather_rows<<<dim3((unsigned)((n + 255) / 256), 1, cnt), 256, 0, s>>>(
        w.A, w.sA, n, (int)j0, NO, w.rpiv, w.sV, w.B, w.sB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_gj_slab_update<NO><<<dim3(nt, nt, cnt), 256, 0, s>>>(
        w.A, w.sA, n, j0, w.rpiv + j0, w.sV, sb[cs], sb[cs ^ 1], w.sS, w.B, w.sB, pb[cp], w.sP, NB);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Panel configurations (panel width, threads, rows per thread, slab width);
// the largest order each one holds is RPT * TPB.
struct GjCfg { int nb, tpb, rpt, no; };
static const GjCfg kCfg1[3] = {{12, 512, 5, 0}, {8, 512, 10, 0}, {4, 768, 15, 0}};
static const GjCfg kCfg2[3] = {{8, 512, 5, 64}, {8, 512, 10, 64}, {4, 768, 15, 128}};

GjPlan gj_plan(int64_t n, int algo) {
  GjPlan p{};
  p.algo = algo == 0 ? ((n > 256) ? 2 : 1) : algo;
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
hipError_t launch_gj(hipStream_t s, const GjPlan& p, const GjWork& w, int64_t n, int cnt) {
  if (n > p.max_n || n % p.pad || cnt < 1) return hipErrorInvalidValue;
  if (p.algo == 1) {
    switch (p.cfg) {
      case 0: return gj_blocked<5, 12, 512>(s, w, n, cnt);
      case 1: return gj_blocked<10, 8, 512>(s, w, n, cnt);
      default: return gj_blocked<15, 4, 768>(s, w, n, cnt);
    }
  }
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
  out[D.inv_off + i * n0 + j] = S[blockIdx.z * sA + (int64_t)rp[i] * n + ri[j]];
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
  k_dense_gemv_t<<<grid, 256, 0, s>>>(desc, b, inv, x, y);
  return hipGetLastError();
}

hipError_t launch_dense_gemv(hipStream_t s, const CoarseDesc* desc, int cnt, int b,
                             int64_t max_n0, const double* inv, const double* x, double* y) {
  if (cnt < 1) return hipSuccess;
  dim3 grid((unsigned)((max_n0 + 3) / 4), 1, (unsigned)cnt);
  k_dense_gemv<<<grid, 256, 0, s>>>(desc, b, inv, x, y);
  return hipGetLastError();
}

}  // namespace stv
