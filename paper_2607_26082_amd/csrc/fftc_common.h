// Device helpers shared by the kernel translation units of libfftc.
#pragma once

#include "fftc_internal.h"

namespace fftc {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Adds the columns of a table of per-block partials (P columns of nrow values, column q at
// q * ld) into acc[0..P): thread t takes rows t, t + blockDim.x, t + 2 blockDim.x, ... in that
// order (the fixed order the solver's reductions have).  Consecutive lanes read consecutive
// rows, and four rows of every column are loaded before any is added, so their loads are in
// flight together.
template <int P, int NV>
__device__ __forceinline__ void sum_cols(const double* __restrict__ tab, long long ld, long long nrow,
                                         double (&acc)[NV]) {
  static_assert(P <= NV, "more columns than accumulators");
  constexpr int U = 4;
  const long long bd = blockDim.x;
  for (long long b0 = threadIdx.x; b0 < nrow; b0 += U * bd) {
    double v[U][P];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const long long b = b0 + k * bd;
#pragma unroll
      for (int q = 0; q < P; ++q) v[k][q] = b < nrow ? tab[q * ld + b] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (b0 + k * bd < nrow)
#pragma unroll
        for (int q = 0; q < P; ++q) acc[q] += v[k][q];
  }
}

// Gaussian elimination with partial pivoting on the augmented N x (N + 1) system G, solution in
// y; false (y = 0) when a pivot is not positive in magnitude.  Every index is a compile-time
// constant (row swaps are selects), so G stays in registers instead of private memory.
template <int N>
__device__ __forceinline__ bool solve_pivoted(double (&G)[N][N + 1], double (&y)[N]) {
#pragma unroll
  for (int r = 0; r < N; ++r) y[r] = 0.0;
#pragma unroll
  for (int col = 0; col < N; ++col) {
    int piv = col;
    double best = fabs(G[col][col]);
#pragma unroll
    for (int r = col + 1; r < N; ++r)
      if (fabs(G[r][col]) > best) {
        best = fabs(G[r][col]);
        piv = r;
      }
    if (!(best > 0.0)) return false;
#pragma unroll
    for (int r = col + 1; r < N; ++r)
      if (r == piv)
#pragma unroll
        for (int q = 0; q < N + 1; ++q) {
          const double t = G[col][q];
          G[col][q] = G[r][q];
          G[r][q] = t;
        }
#pragma unroll
    for (int r = col + 1; r < N; ++r) {
      const double f = G[r][col] / G[col][col];
#pragma unroll
      for (int q = col; q < N + 1; ++q) G[r][q] -= f * G[col][q];
    }
  }
#pragma unroll
  for (int r = N - 1; r >= 0; --r) {
    double s = G[r][N];
#pragma unroll
    for (int q = r + 1; q < N; ++q) s -= G[r][q] * y[q];
    y[r] = s / G[r][r];
  }
  return true;
}

// Block-wide sum of NV doubles; result valid in thread 0.  Fixed reduction order.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* sh /* >= NV*16 */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = wave_sum(v[q]);
  __syncthreads();
  if (lane == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) sh[q * 16 + wid] = v[q];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += sh[q * 16 + w];
      v[q] = s;
    }
  }
  __syncthreads();
}

// Contiguous node range of this block, with blocks of one XCD (workgroups are dealt
// round-robin to the 8 XCDs) owning one contiguous slab, so that the y/z neighbours a
// block reads are produced by blocks on the same XCD and hit its L2.
__device__ __forceinline__ void xcd_chunk(long long total, long long& lo, long long& hi) {
  const int G = gridDim.x, b = blockIdx.x;
  const int lb = (G % 8 == 0) ? (b % 8) * (G / 8) + b / 8 : b;
  const long long chunk = (total + G - 1) / G;
  lo = (long long)lb * chunk;
  hi = lo + chunk < total ? lo + chunk : total;
}

__device__ __forceinline__ int mirror_coord(const Geo& g, int x, int J) {
  if (g.periodic[J]) return x < 0 ? x + g.N[J] : (x >= g.N[J] ? x - g.N[J] : x);
  return x < 0 ? -x : (x > g.n[J] ? 2 * g.n[J] - x : x);
}

__device__ __forceinline__ bool is_antisym(const Geo& g, int c, const int xyz[3]) {
#pragma unroll
  for (int J = 0; J < 3; ++J) {
    if (g.periodic[J]) continue;
    if (xyz[J] == 0 && ((g.aface >> (c * 6 + J * 2 + 0)) & 1)) return true;
    if (xyz[J] == g.n[J] && ((g.aface >> (c * 6 + J * 2 + 1)) & 1)) return true;
  }
  return false;
}

__device__ __forceinline__ int bcount(const Geo& g, const int xyz[3]) {
  int b = 0;
#pragma unroll
  for (int J = 0; J < 3; ++J)
    if (!g.periodic[J] && (xyz[J] == 0 || xyz[J] == g.n[J])) ++b;
  return b;
}

static inline int grid_for(long long n, int cap) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (int)(b < cap ? b : cap);
}

// First Piola-Kirchhoff stress of the Saint-Venant-Kirchhoff law (finite strain, Section 5.2,
// eq 29; the law of Section 5.4) from the displacement gradient G (G[r][s] = d u_r / d x_s):
// F = I + G, Green-Lagrange E = (G + G^T + G^T G) / 2, S = l tr(E) I + 2 m E, P = F S.
template <typename T>
__device__ __forceinline__ void svk_pk1(const T (&G)[3][3], T l, T m, T (&P)[3][3]) {
  T E[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = a; b < 3; ++b) {
      E[a][b] = T(0.5) * (G[a][b] + G[b][a] + G[0][a] * G[0][b] + G[1][a] * G[1][b] + G[2][a] * G[2][b]);
      E[b][a] = E[a][b];
    }
  const T lt = l * (E[0][0] + E[1][1] + E[2][2]);
  T S[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) S[a][b] = T(2) * m * E[a][b] + (a == b ? lt : T(0));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) P[i][j] = S[i][j] + G[i][0] * S[0][j] + G[i][1] * S[1][j] + G[i][2] * S[2][j];
}

// blocks of kBlock threads for one wavefront per relation
static inline int rel_grid(long long m) { return (int)((m + (kBlock / 64) - 1) / (kBlock / 64)); }

}  // namespace fftc
