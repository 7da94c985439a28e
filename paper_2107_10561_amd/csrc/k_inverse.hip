// Batched extraction and inversion of the local space-time Jacobians J_T
// (Section 4.2: J_T is the submatrix of the level matrix on the cell's DoFs;
// Section 4.3: the inverses are pre-computed once per Jacobian and stored).
//
// One workgroup per cell.  The n x n block (n = B * NLS) lives in registers:
// wave w holds rows i = w + NW*k, lane holds columns j = lane + 64*c.  The
// block is gathered from the block-sparse level matrix through the cell's
// block-position map (absent pairs are zero), inverted by Gauss-Jordan
// elimination with partial pivoting in FP64,
// and written row-major, FP64 or FP32, keeping either every row or only the
// rows of the DoFs the cell owns.  Each elimination step exchanges only the
// pivot column and two rows through LDS (double-buffered, two barriers).
// Cell-local order inside the kernel is (alpha, l) -> alpha*B + l, matching
// the time-inner global layout.
#include "stv_internal.h"
#include "wave.h"

namespace stv {

__device__ __forceinline__ int32_t find_block(const int32_t* __restrict__ col, int32_t lo,
                                              int32_t hi, int32_t key) {
  const int32_t end = hi;
  while (lo < hi) {
    const int32_t mid = (lo + hi) >> 1;
    if (col[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (lo < end && col[lo] == key) ? lo : -1;
}

// Block position of every cell DoF pair (alpha, beta) in the block-sparse
// level matrix (-1 when the pair is absent, i.e. a zero block); built once
// per hierarchy, it turns the extraction of J_T into independent loads.
__global__ void k_build_posmap(const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const int32_t* __restrict__ csd, int n_ls, int64_t n_pairs,
                               int32_t* __restrict__ posmap) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_pairs) return;
  const int64_t per = (int64_t)n_ls * n_ls;
  const int64_t T = e / per;
  const int pr = (int)(e - T * per);
  const int a = pr / n_ls;
  const int32_t* sd = csd + T * n_ls;
  const int32_t row = sd[a];
  posmap[e] = find_block(col, rowptr[row], rowptr[row + 1], sd[pr - a * n_ls]);
}

hipError_t launch_build_posmap(hipStream_t s, const DevLevel& L) {
  const int64_t n = (int64_t)L.n_cells * L.n_ls * L.n_ls;
  k_build_posmap<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(L.rowptr, L.col, L.cell_sdofs,
                                                            L.n_ls, n, L.posmap);
  return hipGetLastError();
}

typedef double stv_d4 __attribute__((ext_vector_type(4)));

// Blocked Gauss-Jordan inversion on FP64 matrix cores.  The block, padded
// with an identity to NP = 16*NT, lives in the accumulator layout of
// v_mfma_f64_16x16x4f64: wave w holds tile row w, and lane l, register v of
// tile tj holds element (16w + 4v + (l >> 4), 16tj + (l & 15)).
// Pivot panels of 4 columns are eliminated by wave 0 in LDS with partial
// pivoting over the rows not yet used as pivots (no row interchanges: the
// pivot row of step p is recorded as rpiv[p]).  The panel's effect on every
// other column is the rank-4 update A += W B with W = (E - I)(:, pivot rows)
// and B = the pivot rows before the panel, one MFMA per 16x16 tile.  At the
// end element (rho, q) of the in-place result belongs to row rinv[rho] and
// column rpiv[q] of the inverse.
template <int B, int NLS>
__global__ void __launch_bounds__(((B * NLS + 15) / 16) * 64)
__attribute__((amdgpu_waves_per_eu((((B * NLS + 15) / 16) + 3) / 4, 8))) k_inverse_mfma(
    const int32_t* __restrict__ posmap, const double* __restrict__ val,
    const int32_t* __restrict__ own_ptr, const uint8_t* __restrict__ own_loc, int full,
    const int64_t* __restrict__ inv_off, int ld, void* store, int fp32, uint8_t* status) {
  constexpr int N = B * NLS;
  constexpr int NT = (N + 15) / 16;
  constexpr int NP = 16 * NT;
  constexpr int NCH = (NP + 63) / 64;
  __shared__ double panel[NP][4];
  __shared__ double brow[4][NP];
  __shared__ int rpiv[NP];
  __shared__ int rinv[NP];
  __shared__ uint8_t used[NP];
  __shared__ int rowmap[N];
  __shared__ int sing;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = tid >> 6;
  const int lr = lane >> 4;   // row offset inside a 4-row group
  const int lc = lane & 15;   // column inside a tile
  const int T = blockIdx.x;
  const int32_t* pos = posmap + (int64_t)T * (NLS * NLS);

  if (tid == 0) sing = 0;
  for (int i = tid; i < NP; i += NT * 64) used[i] = 0;
  for (int i = tid; i < N; i += NT * 64) rowmap[i] = full ? i : -1;
  __syncthreads();
  if (!full) {
    const int o0 = own_ptr[T], no = own_ptr[T + 1] - o0;
    for (int e = tid; e < no * B; e += NT * 64) {
      const int os = e / B;
      rowmap[own_loc[o0 + os] * B + (e - os * B)] = e;
    }
  }

  stv_d4 acc[NT];
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + 4 * v + lr;
      const int col = 16 * tj + lc;
      double x;
      if (row < N && col < N) {
        const int al = row / B, be = col / B;
        const int32_t q = pos[al * NLS + be];
        x = q >= 0 ? val[(int64_t)q * (B * B) + (row - al * B) * B + (col - be * B)] : 0.0;
      } else {
        x = (row == col) ? 1.0 : 0.0;
      }
      acc[tj][v] = x;
    }
  }

  // tile column tc is a run-time index: the accumulator tiles are selected
  // by compile-time comparisons so that they stay in registers
#pragma unroll 1
  for (int tc = 0; tc < NT; ++tc) {
    for (int q4 = 0; q4 < 4; ++q4) {
      const int c0 = 4 * q4;          // first panel column inside tile column tc
      const int p0 = 16 * tc + c0;
      // (a) panel columns -> LDS
      if (lc >= c0 && lc < c0 + 4) {
#pragma unroll
        for (int tj = 0; tj < NT; ++tj)
          if (tj == tc) {
#pragma unroll
            for (int v = 0; v < 4; ++v) panel[16 * w + 4 * v + lr][lc - c0] = acc[tj][v];
          }
      }
      __syncthreads();
      // (b) wave 0 eliminates the panel (partial pivoting over unused rows)
      if (w == 0) {
        for (int t = 0; t < 4; ++t) {
          const int p = p0 + t;
          double best = -1.0;
          int bi = 0x7fffffff;
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) {
            const int rho = lane + 64 * ch;
            if (rho < NP && !used[rho]) {
              const double v = fabs(panel[rho][t]);
              if (v > best) { best = v; bi = rho; }
            }
          }
          // the largest magnitude (DPP max), then the lowest row holding it:
          // read from the single lane that has it, or a DPP min over ties
          const double m = wave_max_f64(best);
          const uint64_t tied = __builtin_amdgcn_ballot_w64(bi < NP && best == m);
          int r;
          if (tied == 0)
            r = 0x7fffffff;
          else if (NCH == 1 || (tied & (tied - 1)) == 0)
            r = __builtin_amdgcn_readlane(bi, (int)__builtin_ctzll(tied));
          else
            r = wave_min_i32(best == m ? bi : 0x7fffffff);
          r = __builtin_amdgcn_readfirstlane(r);
          if (r >= NP) {   // no finite candidate (NaN column): lowest unused row
            int u = 0x7fffffff;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
              const int rho = lane + 64 * ch;
              if (rho < NP && !used[rho]) u = min(u, rho);
            }
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) u = min(u, __shfl_xor(u, off, 64));
            r = u;
            if (lane == 0) sing = 1;
          }
          const double piv = panel[r][t];
          if (lane == 0) {
            if (!(m > 0.0) || !(piv != 0.0)) sing = 1;
            rpiv[p] = r;
            used[r] = 1;
          }
          const double ipiv = (piv != 0.0) ? 1.0 / piv : 0.0;
          double pr[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) pr[c] = panel[r][c];
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch) {
            const int rho = lane + 64 * ch;
            if (rho < NP) {
              if (rho == r) {
#pragma unroll
                for (int c = 0; c < 4; ++c) panel[rho][c] = (c == t) ? ipiv : pr[c] * ipiv;
              } else {
                const double f = panel[rho][t] * ipiv;
#pragma unroll
                for (int c = 0; c < 4; ++c)
                  panel[rho][c] = (c == t) ? -f : fma(-f, pr[c], panel[rho][c]);
              }
            }
          }
        }
      }
      __syncthreads();
      // (c) the owners publish the four pivot rows as they were before the panel
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = rpiv[p0 + t];
        if (w == (r >> 4) && lr == (r & 3)) {
          const int vr = (r & 15) >> 2;
#pragma unroll
          for (int tj = 0; tj < NT; ++tj) {
            const stv_d4 a4 = acc[tj];
            const double x = vr == 0 ? a4[0] : vr == 1 ? a4[1] : vr == 2 ? a4[2] : a4[3];
            brow[t][16 * tj + lc] = x;
          }
        }
      }
      __syncthreads();
      // (d) rank-4 update of every tile, then the panel columns take the
      // eliminated panel values
      {
        const int rho = 16 * w + lc;
        const int t = lr;
        const double a = panel[rho][t] - ((rho == rpiv[p0 + t]) ? 1.0 : 0.0);
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          const double bv = brow[lr][16 * tj + lc];
          acc[tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[tj], 0, 0, 0);
        }
        if (lc >= c0 && lc < c0 + 4) {
#pragma unroll
          for (int tj = 0; tj < NT; ++tj)
            if (tj == tc) {
#pragma unroll
              for (int v = 0; v < 4; ++v) acc[tj][v] = panel[16 * w + 4 * v + lr][lc - c0];
            }
        }
      }
      __syncthreads();
    }
  }
  // row of the inverse held by in-place row rho, and the store
  for (int p = tid; p < NP; p += NT * 64) rinv[rpiv[p]] = p;
  if (tid == 0) status[T] = (uint8_t)sing;
  __syncthreads();
  const int64_t off = inv_off[T];
#pragma unroll
  for (int tj = 0; tj < NT; ++tj) {
    const int q = 16 * tj + lc;
    const int j = rpiv[q];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int rho = 16 * w + 4 * v + lr;
      const int p = rinv[rho];
      if (p < N && j < N) {
        const int o = rowmap[p];
        if (o >= 0) {
          const int64_t e = off + (int64_t)o * ld + j;
          if (fp32) ((float*)store)[e] = (float)acc[tj][v];
          else ((double*)store)[e] = acc[tj][v];
        }
      }
    }
  }
}

// Stores row r of the block (r uniform) into dst[0 .. 16 NT): the lanes of
// group r & 3 hold it in tile row r >> 4, register (r >> 2) & 3, one value
// per tile column.  Each case stores from its own registers, so no
// accumulator is ever selected by a run-time index (the empty asm statement
// ending each case keeps the compiler from merging the cases into one store
// of a run-time-indexed element, which would move the block to scratch).
template <int NT>
__device__ __forceinline__ void store_row(const stv_d4 (&acc)[NT][NT], int r, double* dst, int lr,
                                          int lc) {
  if (lr != (r & 3)) return;
  switch (r >> 2) {
#define STV_ROW_CASE(S)                                                                     \
  case S:                                                                                   \
    if constexpr (S < 4 * NT) {                                                             \
      _Pragma("unroll") for (int tj = 0; tj < NT; ++tj) dst[16 * tj + lc] = acc[S >> 2][tj][S & 3]; \
      asm volatile("; row case %0" ::"n"(S));                                               \
    }                                                                                       \
    break;
    STV_ROW_CASE(0) STV_ROW_CASE(1) STV_ROW_CASE(2) STV_ROW_CASE(3)
    STV_ROW_CASE(4) STV_ROW_CASE(5) STV_ROW_CASE(6) STV_ROW_CASE(7)
    STV_ROW_CASE(8) STV_ROW_CASE(9) STV_ROW_CASE(10) STV_ROW_CASE(11)
    STV_ROW_CASE(12) STV_ROW_CASE(13) STV_ROW_CASE(14) STV_ROW_CASE(15)
#undef STV_ROW_CASE
    default: break;
  }
}

// The same Gauss-Jordan inversion with one wavefront per cell, for orders up
// to 64: the whole identity-padded block (NT x NT tiles) sits in this
// wavefront's accumulators, so no step needs a workgroup barrier.  Per panel
// of 4 columns:
//  - the panel moves through LDS into one row per lane; its four pivots are
//    chosen by pivot_lane and the pivot row is broadcast by readlane;
//  - the four pivot rows as they were before the panel go to LDS; the panel
//    columns take their eliminated values directly and see B = 0;
//  - the rank-4 update A += W B is one MFMA per tile, the panel's own tile
//    column first so that the next panel can start while the rest run.
// The in-place result is permuted as in k_inverse_mfma.
// DEC: the cell matrix is Q = M_T (x) T + A_T (x) I of the CellSplit sp,
// gathered from the spatial factors (val = (m, a) per block position), and
// the store takes its time-decoupled owned rows (sp describes one diagonal
// block of a level's split: B = its order in time).  keep_status: a cell's
// status is only raised, so that the launches of several blocks combine.

template <int B, int NLS, bool DEC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_inverse_wave(const int32_t* __restrict__ posmap, const double* __restrict__ val,
               const int32_t* __restrict__ own_ptr, const uint8_t* __restrict__ own_loc, int full,
               const int64_t* __restrict__ inv_off, int ld, void* store, int fp32,
               uint8_t* status, int n_cells, CellSplit sp, int keep_status) {
  constexpr int N = B * NLS;
  constexpr int NT = (N + 15) / 16;
  constexpr int NP = 16 * NT;
  static_assert(NP <= 64, "one wavefront holds at most 64 rows");
  __shared__ int spos[NLS * NLS];
  __shared__ double panel[NP][4];
  __shared__ double brow[4][NP];
  __shared__ int rpiv[NP];
  __shared__ int rinv[NP];
  __shared__ int rowmap[NP];
  // DEC: T[a][c] and the first stored column of the inverse entries with
  // row component a and column component c (-1: not stored)
  __shared__ double tco[B * B];
  __shared__ int cmap[B * B];
  if constexpr (DEC) {
    if (threadIdx.x == 0) {
#pragma unroll
      for (int e = 0; e < B * B; ++e) {
        tco[e] = sp.T[e];
        cmap[e] = -1;
      }
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        if (p >= sp.nblk) break;
        const int f = sp.first[p];
        for (int a = 0; a < sp.sz[p]; ++a) cmap[f * B + f + a] = sp.off[p] + a * NLS;
      }
    }
  }
  // grid-stride over the cells: a capped grid leaves room on every SIMD
  // for the kernels of a concurrent stream
  for (int T = blockIdx.x; T < n_cells; T += gridDim.x) {
    wave_lds_sync();   // the previous cell's LDS reads come first
    // the lane index passes through an empty asm statement each cell, so the
    // per-lane index arithmetic stays inside the loop instead of being
    // hoisted and held in registers across it
    int lane = (int)threadIdx.x;
    asm volatile("" : "+v"(lane));
    const int lr = lane >> 4;
    const int lc = lane & 15;

    // J_T: the cell's block positions through LDS, then every value load at
    // once (indices clamped into the block, the padding and absent blocks
    // selected afterwards)
    {
      constexpr int NPOS = NLS * NLS;
      const int32_t* pos = posmap + (int64_t)T * NPOS;
      int32_t q[(NPOS + 63) / 64];
#pragma unroll
      for (int i = 0; i < (NPOS + 63) / 64; ++i) {
        const int e = lane + 64 * i;
        q[i] = pos[e < NPOS ? e : NPOS - 1];
      }
#pragma unroll
      for (int i = 0; i < (NPOS + 63) / 64; ++i)
        if (lane + 64 * i < NPOS) spos[lane + 64 * i] = q[i];
    }
    wave_lds_sync();
    stv_d4 acc[NT][NT];
#pragma unroll
    for (int ti = 0; ti < NT; ++ti) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 16 * ti + 4 * v + lr;
        const int rc = row < N ? row : N - 1;
        const int ra = rc / B;
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          const int col = 16 * tj + lc;
          const int cc = col < N ? col : N - 1;
          const int be = cc / B;
          const int32_t q = spos[ra * NLS + be];
          double x;
          if constexpr (DEC) {
            const double2 ma = *reinterpret_cast<const double2*>(&val[2 * (int64_t)(q > 0 ? q : 0)]);
            const int ar = rc - ra * B, ac = cc - be * B;
            x = fma(tco[ar * B + ac], ma.x, ar == ac ? ma.y : 0.0);
          } else {
            x = val[(int64_t)(q > 0 ? q : 0) * (B * B) + (rc - ra * B) * B + (cc - be * B)];
          }
          // bitwise predicates and a value select: no branch for the load to
          // sink into
          const bool inb = (row < N) & (col < N);
          const bool keep = inb & (q >= 0);
          const double pad = ((!inb) & (row == col)) ? 1.0 : 0.0;
          acc[ti][tj][v] = keep ? x : pad;
        }
      }
    }

    bool used = lane >= NP;   // this lane's row has been a pivot row
    int mypiv = 0;            // lane p: pivot row of column p
    bool sing = false;
    const int prow = lane < NP ? lane : NP - 1;
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
#pragma unroll 1
      for (int q4 = 0; q4 < 4; ++q4) {
        const int c0 = 4 * q4;
        const bool pcol = (unsigned)(lc - c0) < 4u;   // lane holds a panel column
        // panel columns -> LDS, read back one row per lane
        wave_lds_sync();
        if (pcol) {
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) panel[16 * ti + 4 * v + lr][lc - c0] = acc[ti][tc][v];
        }
        wave_lds_sync();
        double pv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) pv[c] = panel[prow][c];
        int rk[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          int r = pivot_lane(pv[t], !used);
          if (r < 0) {   // no finite candidate (NaN column): lowest unused row
            r = (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(!used));
            sing = true;
          }
          r = __builtin_amdgcn_readfirstlane(r);
          double pr[4];
#pragma unroll
          for (int c = 0; c < 4; ++c) pr[c] = readlane_f64(pv[c], r);
          const double piv = pr[t];
          if (!(piv != 0.0)) sing = true;
          const double ipiv = (piv != 0.0) ? recip_f64(piv) : 0.0;
          // pivot row: pr * ipiv (ipiv in column t); other rows: pv - f pr
          // (-f in column t), both as fma(-g, pr, pv') with pv' = 0 in the
          // pivot row
          const bool me = lane == r;
          const double g = me ? -ipiv : pv[t] * ipiv;
#pragma unroll
          for (int c = 0; c < 4; ++c) pv[c] = (c == t) ? -g : fma(-g, pr[c], me ? 0.0 : pv[c]);
          used = used || me;
          if (lane == 16 * tc + c0 + t) mypiv = r;
          rk[t] = r;
        }
        // the pivot rows as they were before the panel
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
          const int r = k == 0 ? rk[0] : k == 1 ? rk[1] : k == 2 ? rk[2] : rk[3];
          store_row<NT>(acc, r, &brow[k][0], lr, lc);
        }
        if (lane < NP) {
#pragma unroll
          for (int c = 0; c < 4; ++c) panel[lane][c] = pv[c];
        }
        wave_lds_sync();
        // W = (E - I)(:, pivot rows) and B in the operand layouts of the MFMA;
        // the panel columns take the eliminated values and see B = 0
        const int rsel = lr == 0 ? rk[0] : lr == 1 ? rk[1] : lr == 2 ? rk[2] : rk[3];
        double a[NT], b[NT];
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
          a[ti] = panel[16 * ti + lc][lr] - ((16 * ti + lc == rsel) ? 1.0 : 0.0);
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          const double bv = brow[lr][16 * tj + lc];
          b[tj] = (tj == tc && pcol) ? 0.0 : bv;
        }
        if (pcol) {
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[ti][tc][v] = panel[16 * ti + 4 * v + lr][lc - c0];
        }
#pragma unroll
        for (int ti = 0; ti < NT; ++ti)
          acc[ti][tc] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tc], acc[ti][tc], 0, 0, 0);
#pragma unroll
        for (int tj = 0; tj < NT; ++tj) {
          if (tj == tc) continue;
#pragma unroll
          for (int ti = 0; ti < NT; ++ti)
            acc[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ti], b[tj], acc[ti][tj], 0, 0, 0);
        }
      }
    }

    // row of the inverse held by in-place row rho, owned rows, and the store
    wave_lds_sync();
    if (lane < NP) {
      rpiv[lane] = mypiv;
      rinv[mypiv] = lane;
      rowmap[lane] = (full && lane < N) ? lane : -1;
    }
    wave_lds_sync();
    if (!full) {
      const int o0 = own_ptr[T], no = own_ptr[T + 1] - o0;
      for (int e = lane; e < no * B; e += 64) {
        const int os = e / B;
        rowmap[own_loc[o0 + os] * B + (e - os * B)] = DEC ? os : e;
      }
    }
    if (lane == 0 && (!keep_status || sing)) status[T] = (uint8_t)sing;
    wave_lds_sync();
    const int64_t off = inv_off[T];
#pragma unroll
    for (int tj = 0; tj < NT; ++tj) {
      const int j = rpiv[16 * tj + lc];
#pragma unroll
      for (int ti = 0; ti < NT; ++ti) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int p = rinv[16 * ti + 4 * v + lr];
          if (p < N && j < N) {
            const int o = rowmap[p];
            int col = j;
            if constexpr (DEC) {
              const int be = j / B, base = cmap[(j - be * B) * B + p % B];
              col = base >= 0 ? base + be : -1;
            }
            if (o >= 0 && col >= 0) {
              const int64_t e = off + (int64_t)o * ld + col;
              if (fp32) ((float*)store)[e] = (float)acc[ti][tj][v];
              else ((double*)store)[e] = acc[ti][tj][v];
            }
          }
        }
      }
    }
  }
}

// Stores the row of the complex block held in local tile row rl >> 4,
// register (rl >> 2) & 3 by the lanes of group rl & 3 (rl uniform, < 16 TR)
// into dst[16 tj + lc] for the TC local tile columns, as (re, im) pairs.  As
// in store_row, every case reads its own registers.
template <int TR, int TC>
__device__ __forceinline__ void store_row_cx(const stv_d4 (&ar)[TR][TC],
                                             const stv_d4 (&ai)[TR][TC], int rl,
                                             double2* dst, int lr, int lc) {
  if (lr != (rl & 3)) return;
  switch (rl >> 2) {
#define STV_CX_CASE(S)                                                                   \
  case S:                                                                                \
    if constexpr (S < 4 * TR) {                                                          \
      _Pragma("unroll") for (int tj = 0; tj < TC; ++tj)                                  \
        dst[16 * tj + lc] = make_double2(ar[S >> 2][tj][S & 3], ai[S >> 2][tj][S & 3]);  \
      asm volatile("; cx row case %0" ::"n"(S));                                         \
    }                                                                                    \
    break;
    STV_CX_CASE(0) STV_CX_CASE(1) STV_CX_CASE(2) STV_CX_CASE(3)
    STV_CX_CASE(4) STV_CX_CASE(5) STV_CX_CASE(6) STV_CX_CASE(7)
    STV_CX_CASE(8) STV_CX_CASE(9) STV_CX_CASE(10) STV_CX_CASE(11)
#undef STV_CX_CASE
    default: break;
  }
}

// Cell inverses of a dG(1) level with spatial factors through its complex
// time-decoupled block (Section 4.3's J_T^-1, computed in half the pivot
// steps and half the flops of the real block).  With D^-1 C = V T V^-1 and
// T = [[t00, t01], [t10, t00]] (one complex pair),
//   J_T^-1 = (I (x) V) Q^-1 (I (x) W),  Q = M_T (x) T + A_T (x) I,  W = V^-1 D^-1,
// and Q is the real form of the complex matrix X = (t00 M_T + A_T) + i t10 M_T
// of order n_ls, so Q^-1 is the real form of Y = X^-1 and
//   J_T^-1[(a, i), (c, l)] = V_i0 (Re Y_ac W_0l - Im Y_ac W_1l)
//                          + V_i1 (Im Y_ac W_0l + Re Y_ac W_1l).
// Y is computed by Gauss-Jordan elimination with complex partial pivoting
// (largest |Re| + |Im| among the rows not yet used, lowest row on ties; no
// row interchanges, as in k_inverse_mfma).  dec = 0: the rows of J_T^-1 are
// stored in the plain layout (owned or all rows, FP64 or FP32), the same rows
// the real elimination stores; dec = 1: the owned-rows layout keeps, per
// owned spatial DoF a, the row Y_a. as [Re Y_a0 .. Re Y_a,n-1, Im Y_a0 ..
// Im Y_a,n-1] (half the values of a's two rows of J_T^-1; the sweep applies
// V and W).
// Four wavefronts per cell on a 2 x 2 grid of the tiles: X, identity-padded
// to NP = 16 NT, sits in their accumulators in the v_mfma_f64_16x16x4f64
// layout, wave (wr, wc) holding tile rows TR wr .. and tile columns TC wc ..
// (real and imaginary parts in separate tiles).  Per panel of 4 columns
// every wavefront reads the panel from LDS and chooses the same pivots (no
// broadcast needed), the owners publish the pivot rows as they were before
// the panel, and the rank-4 complex update is four real MFMAs per tile.
// The grid strides over the cells.
template <int NLS>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1)))
k_inverse_cx(const int32_t* __restrict__ posmap, const double* __restrict__ ma,
             const int32_t* __restrict__ own_ptr, const uint8_t* __restrict__ own_loc, int full,
             const int64_t* __restrict__ inv_off, int ld, void* store, int fp32,
             uint8_t* status, int n_cells, CellSplit sp, int dec) {
  constexpr int N = NLS;
  constexpr int NT = (N + 15) / 16;
  constexpr int NP = 16 * NT;
  constexpr int NW = 4;
  constexpr int TR = NT / 2, TC = NT / 2;   // local tile rows and columns
  constexpr int RPW = 16 * TR;              // rows (and columns) per wavefront
  static_assert(NT % 2 == 0 && NP <= 128 && TR <= 3, "2 x 2 wavefronts, at most 96 rows");
  __shared__ double2 pin[NP][4];            // panel columns before elimination
  __shared__ double2 pw[NW][NP][4];         // each wavefront's eliminated panel
  __shared__ double2 brow[4][NP];           // the pivot rows before the panel
  __shared__ int rpiv[NP];
  __shared__ int rinv[NP];
  __shared__ int rowmap[2 * NP];            // local DoF a * 2 + i -> stored row (-1: none)
  const int tid = threadIdx.x;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wr = w >> 1, wc = w & 1;
  const double t00 = sp.T[0], t10 = sp.T[2];
  for (int T = blockIdx.x; T < n_cells; T += gridDim.x) {
    int lane = tid & 63;
    asm volatile("" : "+v"(lane));
    const int lr = lane >> 4;
    const int lc = lane & 15;

    // X from the spatial factors (m, a) of every cell pair, identity padding
    const int32_t* pos = posmap + (int64_t)T * (NLS * NLS);
    stv_d4 ar[TR][TC], ai[TR][TC];
#pragma unroll
    for (int ti = 0; ti < TR; ++ti) {
      int32_t q[TC][4];
#pragma unroll
      for (int tj = 0; tj < TC; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = RPW * wr + 16 * ti + 4 * v + lr, col = RPW * wc + 16 * tj + lc;
          const int rc = row < N ? row : N - 1, cc = col < N ? col : N - 1;
          q[tj][v] = pos[rc * NLS + cc];
        }
#pragma unroll
      for (int tj = 0; tj < TC; ++tj)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = RPW * wr + 16 * ti + 4 * v + lr, col = RPW * wc + 16 * tj + lc;
          const int32_t qq = q[tj][v];
          const double2 mav = *reinterpret_cast<const double2*>(&ma[2 * (int64_t)(qq > 0 ? qq : 0)]);
          const bool inb = (row < N) & (col < N);
          const bool keep = inb & (qq >= 0);
          const double pad = ((!inb) & (row == col)) ? 1.0 : 0.0;
          ar[ti][tj][v] = keep ? fma(t00, mav.x, mav.y) : pad;
          ai[ti][tj][v] = keep ? t10 * mav.x : 0.0;
        }
    }

    // candidate rows of this lane in the pivot searches: lane and lane + 64
    const bool has1 = lane + 64 < NP;
    const int l1 = has1 ? lane + 64 : 0;
    bool used0 = false, used1 = !has1;
    int mypiv0 = 0, mypiv1 = 0;             // pivot rows of columns lane, lane + 64
    bool sing = false;
#pragma unroll
    for (int tc = 0; tc < NT; ++tc) {
      const bool own_tc = wc == tc / TC;     // this wavefront holds tile column tc
#pragma unroll 1
      for (int q4 = 0; q4 < 4; ++q4) {
        const int c0 = 4 * q4, p0 = 16 * tc + c0;
        if (p0 >= N) continue;                 // identity columns of the padding (below)
        const bool pcol = (unsigned)(lc - c0) < 4u;   // lane holds a panel column
        if (own_tc && pcol) {
#pragma unroll
          for (int ti = 0; ti < TR; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v)
              pin[RPW * wr + 16 * ti + 4 * v + lr][lc - c0] =
                  make_double2(ar[ti][tc % TC][v], ai[ti][tc % TC][v]);
        }
        __syncthreads();
        double2 pv0[4], pv1[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          pv0[c] = pin[lane][c];
          pv1[c] = has1 ? pin[l1][c] : make_double2(0.0, 0.0);
        }
        int rk[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const double m0 = fabs(pv0[t].x) + fabs(pv0[t].y);
          const double m1 = fabs(pv1[t].x) + fabs(pv1[t].y);
          const double b0 = (!used0 && m0 == m0) ? m0 : -1.0;
          const double b1 = (!used1 && m1 == m1) ? m1 : -1.0;
          const double mx = wave_max_f64(fmax(b0, b1));
          int r;
          if (mx > 0.0) {
            const uint64_t k0 = __builtin_amdgcn_ballot_w64(b0 == mx);
            r = k0 ? (int)__builtin_ctzll(k0)
                   : 64 + (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(b1 == mx));
          } else {
            // no nonzero finite candidate: the lowest unused row (singular)
            const uint64_t u0 = __builtin_amdgcn_ballot_w64(!used0);
            r = u0 ? (int)__builtin_ctzll(u0)
                   : 64 + (int)__builtin_ctzll(__builtin_amdgcn_ballot_w64(!used1));
            sing = true;
          }
          r = __builtin_amdgcn_readfirstlane(r);
          double2 pr[4];
          if (r < 64) {
#pragma unroll
            for (int c = 0; c < 4; ++c)
              pr[c] = make_double2(readlane_f64(pv0[c].x, r), readlane_f64(pv0[c].y, r));
          } else {
#pragma unroll
            for (int c = 0; c < 4; ++c)
              pr[c] = make_double2(readlane_f64(pv1[c].x, r - 64), readlane_f64(pv1[c].y, r - 64));
          }
          const double2 piv = pr[t];
          const double den = fma(piv.x, piv.x, piv.y * piv.y);
          if (!(den > 0.0)) sing = true;
          const double id = den > 0.0 ? recip_f64(den) : 0.0;
          const double2 ip = make_double2(piv.x * id, -piv.y * id);   // 1 / piv
          // pivot row: pr * ip (ip in column t); other rows: pv - f pr (-f in
          // column t), f = pv[t] ip; both as pv' - g pr with pv' = 0 in the
          // pivot row and g = -ip there
          const bool me0 = lane == r, me1 = lane + 64 == r;
          const double2 g0 = me0 ? make_double2(-ip.x, -ip.y)
                                 : make_double2(fma(pv0[t].x, ip.x, -pv0[t].y * ip.y),
                                                fma(pv0[t].x, ip.y, pv0[t].y * ip.x));
          const double2 g1 = me1 ? make_double2(-ip.x, -ip.y)
                                 : make_double2(fma(pv1[t].x, ip.x, -pv1[t].y * ip.y),
                                                fma(pv1[t].x, ip.y, pv1[t].y * ip.x));
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const double2 a0 = me0 ? make_double2(0.0, 0.0) : pv0[c];
            const double2 a1 = me1 ? make_double2(0.0, 0.0) : pv1[c];
            pv0[c] = (c == t) ? make_double2(-g0.x, -g0.y)
                              : make_double2(fma(-g0.x, pr[c].x, fma(g0.y, pr[c].y, a0.x)),
                                             fma(-g0.x, pr[c].y, fma(-g0.y, pr[c].x, a0.y)));
            pv1[c] = (c == t) ? make_double2(-g1.x, -g1.y)
                              : make_double2(fma(-g1.x, pr[c].x, fma(g1.y, pr[c].y, a1.x)),
                                             fma(-g1.x, pr[c].y, fma(-g1.y, pr[c].x, a1.y)));
          }
          used0 = used0 || me0;
          used1 = used1 || me1;
          if (lane == p0 + t) mypiv0 = r;
          if (lane + 64 == p0 + t) mypiv1 = r;
          rk[t] = r;
        }
        // the pivot rows as they were before the panel (from their owners,
        // each wavefront its tile columns)
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
          const int r = k == 0 ? rk[0] : k == 1 ? rk[1] : k == 2 ? rk[2] : rk[3];
          if (r / RPW == wr)
            store_row_cx<TR, TC>(ar, ai, r - RPW * wr, &brow[k][RPW * wc], lr, lc);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          pw[w][lane][c] = pv0[c];
          if (has1) pw[w][l1][c] = pv1[c];
        }
        __syncthreads();
        // W = (E - I)(:, pivot rows) and B in the operand layouts; the panel
        // columns take the eliminated values and see B = 0
        const int rsel = lr == 0 ? rk[0] : lr == 1 ? rk[1] : lr == 2 ? rk[2] : rk[3];
        double wre[TR], wim[TR], nwi[TR];
#pragma unroll
        for (int ti = 0; ti < TR; ++ti) {
          const int rho = RPW * wr + 16 * ti + lc;
          const double2 e = pw[w][rho][lr];
          wre[ti] = e.x - ((rho == rsel) ? 1.0 : 0.0);
          wim[ti] = e.y;
          nwi[ti] = -e.y;
        }
        double br[TC], bi[TC];
#pragma unroll
        for (int tj = 0; tj < TC; ++tj) {
          const double2 bv = brow[lr][RPW * wc + 16 * tj + lc];
          const bool z = own_tc && (tj == tc % TC) && pcol;
          br[tj] = z ? 0.0 : bv.x;
          bi[tj] = z ? 0.0 : bv.y;
        }
        if (own_tc && pcol) {
#pragma unroll
          for (int ti = 0; ti < TR; ++ti)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const double2 e = pw[w][RPW * wr + 16 * ti + 4 * v + lr][lc - c0];
              ar[ti][tc % TC][v] = e.x;
              ai[ti][tc % TC][v] = e.y;
            }
        }
        // the panel's own tile column first (the next panel reads it)
#pragma unroll
        for (int k = 0; k < TC; ++k) {
          const int tj = (tc % TC + k) % TC;
#pragma unroll
          for (int ti = 0; ti < TR; ++ti) {
            ar[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wre[ti], br[tj], ar[ti][tj], 0, 0, 0);
            ar[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(nwi[ti], bi[tj], ar[ti][tj], 0, 0, 0);
            ai[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wre[ti], bi[tj], ai[ti][tj], 0, 0, 0);
            ai[ti][tj] = __builtin_amdgcn_mfma_f64_16x16x4f64(wim[ti], br[tj], ai[ti][tj], 0, 0, 0);
          }
        }
      }
    }

    // the padding columns after the last panel are identity columns: each
    // pivots on its own (never used) row
    constexpr int PEND = (N + 3) / 4 * 4;
    if (lane >= PEND) mypiv0 = lane;
    if (lane + 64 >= PEND) mypiv1 = lane + 64;
    // element (rho, q) of the in-place result is Y[rinv[rho]][rpiv[q]]
    if (w == 0) {
      rpiv[lane] = mypiv0;
      rinv[mypiv0] = lane;
      if (has1) {
        rpiv[l1] = mypiv1;
        rinv[mypiv1] = l1;
      }
    }
    for (int e = tid; e < 2 * NP; e += 64 * NW) rowmap[e] = (full && e < 2 * N) ? e : -1;
    if (tid == 0) status[T] = (uint8_t)sing;
    __syncthreads();
    if (!full) {
      const int o0 = own_ptr[T], no = own_ptr[T + 1] - o0;
      if (dec) {
        for (int e = tid; e < no; e += 64 * NW) rowmap[own_loc[o0 + e]] = e;
      } else {
        for (int e = tid; e < no * 2; e += 64 * NW) rowmap[own_loc[o0 + (e >> 1)] * 2 + (e & 1)] = e;
      }
    }
    __syncthreads();
    const int64_t off = inv_off[T];
    if (dec) {
#pragma unroll
      for (int tj = 0; tj < TC; ++tj) {
        const int c = rpiv[RPW * wc + 16 * tj + lc];
#pragma unroll
        for (int ti = 0; ti < TR; ++ti) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int a = rinv[RPW * wr + 16 * ti + 4 * v + lr];
            const int o = (a < N && c < N) ? rowmap[a] : -1;
            if (o >= 0) {
              const int64_t e = off + (int64_t)o * ld + c;
              if (fp32) {
                ((float*)store)[e] = (float)ar[ti][tj][v];
                ((float*)store)[e + N] = (float)ai[ti][tj][v];
              } else {
                ((double*)store)[e] = ar[ti][tj][v];
                ((double*)store)[e + N] = ai[ti][tj][v];
              }
            }
          }
        }
      }
      continue;
    }
#pragma unroll
    for (int tj = 0; tj < TC; ++tj) {
      const int c = rpiv[RPW * wc + 16 * tj + lc];
#pragma unroll
      for (int ti = 0; ti < TR; ++ti) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int a = rinv[RPW * wr + 16 * ti + 4 * v + lr];
          if (a < N && c < N) {
            const double re = ar[ti][tj][v], im = ai[ti][tj][v];
            const double x0 = fma(re, sp.W[0], -im * sp.W[2]);   // Re Y W_0l - Im Y W_1l, l = 0
            const double y0 = fma(im, sp.W[0], re * sp.W[2]);    // Im Y W_0l + Re Y W_1l, l = 0
            const double x1 = fma(re, sp.W[1], -im * sp.W[3]);
            const double y1 = fma(im, sp.W[1], re * sp.W[3]);
#pragma unroll
            for (int i = 0; i < 2; ++i) {
              const int o = rowmap[a * 2 + i];
              if (o < 0) continue;
              const double v0 = fma(sp.V[2 * i], x0, sp.V[2 * i + 1] * y0);
              const double v1 = fma(sp.V[2 * i], x1, sp.V[2 * i + 1] * y1);
              const int64_t e = off + (int64_t)o * ld + 2 * c;
              if (fp32)
                *reinterpret_cast<float2*>(&((float*)store)[e]) = make_float2((float)v0, (float)v1);
              else
                *reinterpret_cast<double2*>(&((double*)store)[e]) = make_double2(v0, v1);
            }
          }
        }
      }
    }
  }
}

// Fallback for blocks too large for registers (n > 256): the same
// elimination on a global scratch copy, one persistent workgroup per slot.
__global__ void __launch_bounds__(256) k_inverse_global(
    const int32_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const int32_t* __restrict__ csd, int B, int NLS, int n_cells,
    const int32_t* __restrict__ own_ptr, const uint8_t* __restrict__ own_loc, int full,
    const int64_t* __restrict__ inv_off, int ld, void* store, int fp32, uint8_t* status,
    double* gscratch) {
  extern __shared__ double sm[];
  __shared__ int sing;
  const int n = B * NLS;
  double* A = gscratch + (int64_t)blockIdx.x * n * n;
  double* prow = sm;
  double* trow = prow + n;
  double* pcol = trow + n;
  int* pivrow = (int*)(pcol + n);
  int* sigma = pivrow + n;
  int* rowmap = sigma + n;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wv = tid >> 6, nw = nt >> 6;
  for (int T = blockIdx.x; T < n_cells; T += gridDim.x) {
    const int32_t* sd = csd + (int64_t)T * NLS;
    if (tid == 0) sing = 0;
    for (int64_t e = tid; e < (int64_t)n * n; e += nt) {
      const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
      const int al = i / B, be = j / B;
      const int32_t row = sd[al];
      const int32_t q = find_block(col, rowptr[row], rowptr[row + 1], sd[be]);
      A[e] = q >= 0 ? val[(int64_t)q * B * B + (i - al * B) * B + (j - be * B)] : 0.0;
    }
    for (int i = tid; i < n; i += nt) rowmap[i] = full ? i : -1;
    __syncthreads();
    if (!full) {
      const int o0 = own_ptr[T], no = own_ptr[T + 1] - o0;
      for (int e = tid; e < no * B; e += nt) rowmap[own_loc[o0 + e / B] * B + e % B] = e;
    }
    for (int p = 0; p < n; ++p) {
      double best = -1.0;
      int bi = 0x7fffffff;
      for (int i = p + lane; i < n; i += 64) {
        const double v = fabs(A[(int64_t)i * n + p]);
        if (v > best) { best = v; bi = i; }
      }
      for (int off = 32; off >= 1; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      const int r = (bi < n) ? bi : p;
      for (int j = tid; j < n; j += nt) {
        prow[j] = A[(int64_t)r * n + j];
        trow[j] = A[(int64_t)p * n + j];
        pcol[j] = A[(int64_t)j * n + p];
      }
      if (tid == 0) {
        pivrow[p] = r;
        if (!(best > 0.0)) sing = 1;
      }
      __syncthreads();
      const double piv = prow[p];
      const double ipiv = (piv != 0.0) ? 1.0 / piv : 0.0;
      for (int i = wv; i < n; i += nw) {
        double* Ai = A + (int64_t)i * n;
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
    if (tid == 0) {
      for (int j = 0; j < n; ++j) sigma[j] = j;
      for (int p = n - 1; p >= 0; --p) {
        const int q = pivrow[p];
        const int t = sigma[p];
        sigma[p] = sigma[q];
        sigma[q] = t;
      }
      status[T] = (uint8_t)sing;
    }
    __syncthreads();
    const int64_t off = inv_off[T];
    for (int64_t e = tid; e < (int64_t)n * n; e += nt) {
      const int i = (int)(e / n), j = (int)(e - (int64_t)i * n);
      const int o = rowmap[i];
      if (o < 0) continue;
      const double v = A[(int64_t)i * n + sigma[j]];
      if (fp32) ((float*)store)[off + (int64_t)o * ld + j] = (float)v;
      else ((double*)store)[off + (int64_t)o * ld + j] = v;
    }
    __syncthreads();
  }
}

bool inverse_fits_regs(int b, int n_ls) {
  return (n_ls == 21 && b >= 1 && b <= 4) || (n_ls == 85 && b >= 1 && b <= 3);
}


// Wavefronts per compute unit of kernel f that leave `reserve` VGPRs free
// on each of the four SIMDs (a SIMD holds 512 per lane, allocated in
// granules of 8); 0 when the kernel's register count is not available.
template <typename K>
static int waves_leaving(K f, int reserve) {
  hipFuncAttributes a{};
  if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(f)) != hipSuccess) return 0;
  const int regs = (a.numRegs + 7) / 8 * 8;
  if (regs <= 0 || regs > 512) return 0;
  const int per_simd = std::min(8, (512 - reserve) / regs);
  return per_simd > 0 ? 4 * per_simd : 0;
}

template <int B, int NLS>
static hipError_t inv_mfma(hipStream_t s, const DevLevel& L, int fp32, int full, uint8_t* status,
                           int n_cu, int reserve) {
  constexpr int NT = (B * NLS + 15) / 16;
  if constexpr (NT <= 4) {
    int grid = L.n_cells;
    if (L.dec) {
      if (!L.kron_ma || L.split.b != B) return hipErrorInvalidValue;
      // one launch per diagonal block of the split: the real block of a
      // real eigenvalue (order n_loc) or the real form of a pair (2 n_loc)
      if constexpr (2 * NLS <= 64) {
        for (int p = 0; p < L.split.nblk; ++p) {
          const int sz = L.split.sz[p], f = L.split.first[p];
          CellSplit one{};
          one.b = sz;
          one.nblk = 1;
          one.sz[0] = sz;
          one.first[0] = 0;
          one.off[0] = L.split.off[p];
          for (int a = 0; a < sz; ++a)
            for (int c = 0; c < sz; ++c) one.T[a * sz + c] = L.split.T[(f + a) * B + f + c];
          int g = L.n_cells;
          if (sz == 1) {
            if (n_cu > 0 && reserve > 0) {
              static const int per_cu = waves_leaving(k_inverse_wave<1, NLS, true>, reserve);
              if (per_cu > 0) g = std::min(g, n_cu * per_cu);
            }
            k_inverse_wave<1, NLS, true><<<g, 64, 0, s>>>(L.posmap, L.kron_ma, L.own_ptr,
                                                          L.own_loc, full, L.inv_off, L.inv_ld,
                                                          L.inv_store, fp32, status, L.n_cells,
                                                          one, p > 0);
          } else {
            if (n_cu > 0 && reserve > 0) {
              static const int per_cu = waves_leaving(k_inverse_wave<2, NLS, true>, reserve);
              if (per_cu > 0) g = std::min(g, n_cu * per_cu);
            }
            k_inverse_wave<2, NLS, true><<<g, 64, 0, s>>>(L.posmap, L.kron_ma, L.own_ptr,
                                                          L.own_loc, full, L.inv_off, L.inv_ld,
                                                          L.inv_store, fp32, status, L.n_cells,
                                                          one, p > 0);
          }
          const hipError_t e = hipGetLastError();
          if (e != hipSuccess) return e;
        }
        return hipSuccess;
      }
      return hipErrorInvalidValue;
    }
    if (n_cu > 0 && reserve > 0) {
      static const int per_cu = waves_leaving(k_inverse_wave<B, NLS, false>, reserve);
      if (per_cu > 0) grid = std::min(grid, n_cu * per_cu);
    }
    k_inverse_wave<B, NLS, false><<<grid, 64, 0, s>>>(L.posmap, L.val, L.own_ptr, L.own_loc, full,
                                                      L.inv_off, L.inv_ld, L.inv_store, fp32,
                                                      status, L.n_cells, CellSplit{}, 0);
    return hipGetLastError();
  } else {
    k_inverse_mfma<B, NLS><<<L.n_cells, NT * 64, 0, s>>>(L.posmap, L.val, L.own_ptr, L.own_loc,
                                                       full, L.inv_off, L.inv_ld, L.inv_store, fp32,
                                                         status);
    return hipGetLastError();
  }
}

hipError_t launch_cell_inverses(hipStream_t s, int b, const DevLevel& L, int fp32, int full,
                                uint8_t* status, double* gscratch, int n_slots, int n_cu,
                                int reserve, int cu_cap) {
  if (L.cx) {
    // the complex decoupled build of a 3d dG(1) level: four wavefronts of
    // up to 512 registers per cell, one cell per compute unit at a time;
    // beside a concurrent coarse chain (n_cu > 0) a cap leaves the other
    // compute units to the chain (the grid then strides over the cells);
    // cu_cap < 0: five eighths of the compute units
    if (b != 2 || L.n_ls != 85 || !L.kron_ma || L.split.nblk != 1 || L.split.sz[0] != 2)
      return hipErrorInvalidValue;
    (void)reserve;
    int grid = L.n_cells;
    const int cap = cu_cap < 0 ? (n_cu * 5) / 8 : cu_cap;
    if (n_cu > 0 && cap > 0) grid = std::min(grid, cap);
    k_inverse_cx<85><<<grid, 256, 0, s>>>(L.posmap, L.kron_ma, L.own_ptr, L.own_loc, full,
                                                L.inv_off, L.inv_ld, L.inv_store, fp32, status,
                                                L.n_cells, L.split, L.dec && !full ? 1 : 0);
    return hipGetLastError();
  }
  if (L.n_ls == 21) {
    switch (b) {
      case 1: return inv_mfma<1, 21>(s, L, fp32, full, status, n_cu, reserve);
      case 2: return inv_mfma<2, 21>(s, L, fp32, full, status, n_cu, reserve);
      case 3: return inv_mfma<3, 21>(s, L, fp32, full, status, n_cu, reserve);
      case 4: return inv_mfma<4, 21>(s, L, fp32, full, status, n_cu, reserve);
    }
  } else if (L.n_ls == 85) {
    switch (b) {
      case 1: return inv_mfma<1, 85>(s, L, fp32, full, status, n_cu, reserve);
      case 2: return inv_mfma<2, 85>(s, L, fp32, full, status, n_cu, reserve);
      case 3: return inv_mfma<3, 85>(s, L, fp32, full, status, n_cu, reserve);
      default: break;
    }
  }
  const int n = L.n_ls * b;
  const size_t shm = sizeof(double) * 3 * (size_t)n + sizeof(int) * 3 * (size_t)n;
  k_inverse_global<<<n_slots, 256, shm, s>>>(L.rowptr, L.col, L.val, L.cell_sdofs, b, L.n_ls,
                                             L.n_cells, L.own_ptr, L.own_loc, full, L.inv_off,
                                             L.inv_ld, L.inv_store, fp32, status, gscratch);
  return hipGetLastError();
}

}  // namespace stv
