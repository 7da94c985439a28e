/*
 * Native helpers of the seeded problem generator: the block-sparse pattern of
 * a level (all pairs of spatial degrees of freedom that share a cell) and the
 * scatter of per-cell element contributions into the space-time blocks.
 *
 * Space-time block of the spatial pair (alpha, beta) of one cell, test time
 * index i, trial time index l (dG(k) with a Lagrange basis at the right
 * Gauss-Radau nodes, time-independent coefficients):
 *     Ct[i][l] * Me[alpha][beta] + (i == l) * tw[i] * Ae[alpha][beta]
 * where Ct is the time-derivative-plus-jump matrix, tw = tau * Radau weights,
 * Me the velocity mass part and Ae the spatial Oseen operator of the cell.
 *
 * This file builds inputs only; it holds no step of the multigrid solver.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Pass 1: count, for each spatial row, an upper bound of its column entries.
 * cell_sdofs: n_cells x n_ls (int32).  bound[n_sdofs] is written. */
void stgen_row_bounds(int32_t n_sdofs, int32_t n_cells, int32_t n_ls,
                      const int32_t* cell_sdofs, int64_t* bound) {
  memset(bound, 0, sizeof(int64_t) * (size_t)n_sdofs);
  for (int64_t c = 0; c < n_cells; ++c)
    for (int a = 0; a < n_ls; ++a) bound[cell_sdofs[c * n_ls + a]] += n_ls;
}

/* Pass 2: fill the (unsorted, duplicated) candidate columns, then sort and
 * make them unique per row.  scratch has sum(bound) entries; bptr[n_sdofs+1]
 * is the prefix sum of bound.  On return rowptr[n_sdofs+1] holds the unique
 * counts' prefix sum and the unique columns sit compacted at the front of
 * scratch (the caller copies rowptr[n] entries out). */
void stgen_pattern(int32_t n_sdofs, int32_t n_cells, int32_t n_ls,
                   const int32_t* cell_sdofs, const int64_t* bptr,
                   const uint8_t* kind, int n_kinds, const uint8_t* coupling,
                   int32_t* scratch, int64_t* fill, int64_t* rowptr) {
  /* kind[s] classifies spatial DoF s; coupling[kr * n_kinds + kc] != 0 keeps
   * the blocks between kinds kr (row) and kc (column). */
  for (int64_t r = 0; r < n_sdofs; ++r) fill[r] = bptr[r];
  for (int64_t c = 0; c < n_cells; ++c) {
    const int32_t* sd = cell_sdofs + c * n_ls;
    for (int a = 0; a < n_ls; ++a) {
      int32_t row = sd[a];
      const uint8_t* cp = coupling + (size_t)kind[row] * n_kinds;
      for (int bb = 0; bb < n_ls; ++bb)
        if (cp[kind[sd[bb]]]) scratch[fill[row]++] = sd[bb];
    }
  }
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t r = 0; r < n_sdofs; ++r) {
    int32_t* seg = scratch + bptr[r];
    int64_t n;
    n = fill[r] - bptr[r];
    qsort(seg, (size_t)n, sizeof(int32_t), cmp_i32);
    int64_t u = 0;
    for (int64_t e = 0; e < n; ++e)
      if (u == 0 || seg[e] != seg[u - 1]) seg[u++] = seg[e];
    fill[r] = u;
  }
  rowptr[0] = 0;
  int64_t w = 0;
  for (int64_t r = 0; r < n_sdofs; ++r) {
    const int32_t* seg = scratch + bptr[r];
    if (w != bptr[r]) memmove(scratch + w, seg, sizeof(int32_t) * (size_t)fill[r]);
    w += fill[r];
    rowptr[r + 1] = w;
  }
}

static int64_t find_col(const int32_t* col, int64_t lo, int64_t hi, int32_t key) {
  const int64_t end = hi;
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (col[mid] < key) lo = mid + 1; else hi = mid;
  }
  return (lo < end && col[lo] == key) ? lo : -1;
}

/* Scatter a chunk of cells [c0, c0+nc) whose element operators Ae are given
 * (nc x n_ls x n_ls, row = test, col = trial).  Me (n_ls x n_ls) is the same
 * for every cell of the level.  Cells of one colour (cell parity per axis)
 * share no degree of freedom, so each colour is scattered in parallel.
 * colour[c] in [0, n_colours). val is nnzb x b x b, row-major per block. */
void stgen_scatter(int32_t n_ls, int32_t b, const int32_t* cell_sdofs,
                   int64_t c0, int64_t nc, const uint8_t* colour, int n_colours,
                   const double* Ae, const double* Me, const double* Ct,
                   const double* tw, const int64_t* rowptr, const int32_t* col,
                   double* val, int64_t* dropped_nonzeros) {
  /* Pairs absent from the pattern must carry exactly zero; any nonzero
   * contribution to such a pair is counted in *dropped_nonzeros. */
  int64_t dropped = 0;
  for (int col_id = 0; col_id < n_colours; ++col_id) {
#pragma omp parallel for schedule(static) reduction(+ : dropped)
    for (int64_t t = 0; t < nc; ++t) {
      int64_t c = c0 + t;
      if (colour[c] != col_id) continue;
      const int32_t* sd = cell_sdofs + c * n_ls;
      const double* A = Ae + t * (int64_t)n_ls * n_ls;
      for (int a = 0; a < n_ls; ++a) {
        int32_t row = sd[a];
        for (int bb = 0; bb < n_ls; ++bb) {
          int64_t pos = find_col(col, rowptr[row], rowptr[row + 1], sd[bb]);
          double m = Me[a * n_ls + bb], aa = A[a * n_ls + bb];
          if (pos < 0) {
            if (m != 0.0 || aa != 0.0) ++dropped;
            continue;
          }
          double* blk = val + pos * (int64_t)b * b;
          for (int i = 0; i < b; ++i)
            for (int l = 0; l < b; ++l)
              blk[i * b + l] += Ct[i * b + l] * m + (i == l ? tw[i] * aa : 0.0);
        }
      }
    }
  }
  *dropped_nonzeros = dropped;
}
