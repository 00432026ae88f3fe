// HIP kernels of libfftc for CDNA4 (gfx950), 64-wide wavefronts.
//
// One fixed-point iteration (paper Algorithm 1 / Algorithm 2, eq 3 and eq 9):
//   k_residual   stress at both TETRA2 integration points of the 8 voxels around
//                each node, nodal divergence (boundary weight 2^b), proj_P for strong
//                DOFs and contact nodes, reference-medium term, FP64 partial norms
//   k_weak       proj_P of the average relations (eq 14)
//   k_control    equilibrium test (eq 5), contact active-set update, Anderson flags
//   k_anderson_r / k_alpha   residual store, FP64 Gram matrix, constrained LS
//   k_dtt        per-axis DTT passes (Tables 2-3) in LDS; the z pass applies the Green
//                operator between its forward and inverse transforms (eq 3-4)
//   k_proj_*     proj_U: average relations (eq 11), contact radial projection, strong DOFs
#include "fftc_internal.h"
#include "fftc_launch.h"
#include "fftc_dtt.h"

#include <math.h>
#include <type_traits>
#include <algorithm>
#include <atomic>

namespace fftc {

// ---------------------------------------------------------------------------
// small helpers
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
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

// ---------------------------------------------------------------------------
// Residual of one node: p = 2^b div_D(C : grad^s_D u) summed over in-cell voxels,
// and K0 u = -2^b div_D(R0 : grad_D u) from the closed-form Paux stencil applied to
// the symmetric extension of u.  Optionally the stress norm and mean-stress sums of
// the tetrahedra owned by this node (T1 of voxel n, T2 of voxel n - e_x).
// ---------------------------------------------------------------------------
template <typename T, bool SIG>
__device__ __forceinline__ void node_eval(const Geo& g, const T* __restrict__ u, const T* __restrict__ lam,
                                          const T* __restrict__ mu, int i, int j, int k, T p[3], T k0[3],
                                          double& sn, double ms[6]) {
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  // 13 same-parity neighbours (self + 12 face diagonals), mirrored at the faces
  T nb[27][3];
  const int xm = mirror_coord(g, i - 1, 0), xp = mirror_coord(g, i + 1, 0);
  const int ym = mirror_coord(g, j - 1, 1), yp = mirror_coord(g, j + 1, 1);
  const int zm = mirror_coord(g, k - 1, 2), zp = mirror_coord(g, k + 1, 2);
  const int xs[3] = {xm, i, xp}, ys[3] = {ym, j, yp}, zs[3] = {zm, k, zp};
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int nrm = (dx != 0) + (dy != 0) + (dz != 0);
        if (nrm != 0 && nrm != 2) continue;
        const long long idx = (long long)xs[dx + 1] + (long long)Nx * ((long long)ys[dy + 1] + (long long)Ny * zs[dz + 1]);
        const int q = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) nb[q][c] = u[c * Nn + idx];
      }

  T F[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    int vx = i - ax, vy = j - ay, vz = k - az;
    bool inside = true;
    if (g.periodic[0]) { if (vx < 0) vx += g.n[0]; } else inside &= (vx >= 0 && vx < g.n[0]);
    if (g.periodic[1]) { if (vy < 0) vy += g.n[1]; } else inside &= (vy >= 0 && vy < g.n[1]);
    if (g.periodic[2]) { if (vz < 0) vz += g.n[2]; } else inside &= (vz >= 0 && vz < g.n[2]);
    if (!inside) continue;
    const long long vid = (long long)vx + (long long)g.n[0] * ((long long)vy + (long long)g.n[1] * vz);
    const T l = lam[vid], m = mu[vid];
    // gradient on the tetrahedron of this voxel that contains the node
    T G[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) G[r][s] = T(0);
    const int par = (ax + ay + az) & 1;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
      if (((cx + cy + cz) & 1) != par) continue;
      const int q = (cx - ax + 1) + 3 * (cy - ay + 1) + 9 * (cz - az + 1);
      const T sx = T(cx ? 0.5 : -0.5), sy = T(cy ? 0.5 : -0.5), sz = T(cz ? 0.5 : -0.5);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        G[r][0] += sx * nb[q][r];
        G[r][1] += sy * nb[q][r];
        G[r][2] += sz * nb[q][r];
      }
    }
    const T tr = G[0][0] + G[1][1] + G[2][2];
    const T s00 = l * tr + T(2) * m * G[0][0];
    const T s11 = l * tr + T(2) * m * G[1][1];
    const T s22 = l * tr + T(2) * m * G[2][2];
    const T s01 = m * (G[0][1] + G[1][0]);
    const T s02 = m * (G[0][2] + G[2][0]);
    const T s12 = m * (G[1][2] + G[2][1]);
    // nodal force: (1/2 IP weight) * B_node^T sigma with B_node = (2a - 1)/2
    const T bx = T(ax ? 0.25 : -0.25), by = T(ay ? 0.25 : -0.25), bz = T(az ? 0.25 : -0.25);
    F[0] += bx * s00 + by * s01 + bz * s02;
    F[1] += bx * s01 + by * s11 + bz * s12;
    F[2] += bx * s02 + by * s12 + bz * s22;
    if (SIG && (a == 0 || a == 1)) {
      const double d00 = s00, d11 = s11, d22 = s22, d01 = s01, d02 = s02, d12 = s12;
      sn += 0.5 * (d00 * d00 + d11 * d11 + d22 * d22 + 2.0 * (d01 * d01 + d02 * d02 + d12 * d12));
      ms[0] += 0.5 * d00; ms[1] += 0.5 * d11; ms[2] += 0.5 * d22;
      ms[3] += 0.5 * d12; ms[4] += 0.5 * d02; ms[5] += 0.5 * d01;
    }
  }
  const int xyz[3] = {i, j, k};
  const int b = bcount(g, xyz);
  const T w2b = T(1 << b);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const int q0 = 13;
    const T sxy = nb[0 + 0 + 9][c] + nb[2 + 0 + 9][c] + nb[0 + 6 + 9][c] + nb[2 + 6 + 9][c];
    const T sxz = nb[0 + 3 + 0][c] + nb[2 + 3 + 0][c] + nb[0 + 3 + 18][c] + nb[2 + 3 + 18][c];
    const T syz = nb[1 + 0 + 0][c] + nb[1 + 6 + 0][c] + nb[1 + 0 + 18][c] + nb[1 + 6 + 18][c];
    const T kk = T(g.st[c][0]) * nb[q0][c] + T(g.st[c][1]) * sxy + T(g.st[c][2]) * sxz + T(g.st[c][3]) * syz;
    const bool A = is_antisym(g, c, xyz);
    p[c] = A ? T(0) : -w2b * F[c];
    k0[c] = A ? T(0) : kk;
  }
}

// ---------------------------------------------------------------------------
// Residual pass
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual(Geo g, Bufs<T> B, ContactDev ct, DevState* st,
                                                     double* __restrict__ part, int force, int write_p) {
  __shared__ double sh[kPartStride * 16];
  if (!force && st->done) return;
  double acc[kPartStride];
#pragma unroll
  for (int q = 0; q < kPartStride; ++q) acc[q] = 0.0;
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  const int cur = ct.on ? st->vpar : 0;
  long long lo, hi;
  xcd_chunk(Nn, lo, hi);
  for (long long node = lo + threadIdx.x; node < hi; node += blockDim.x) {
    const int nd = (int)node;
    const int r = nd / Nx;
    const int i = nd - r * Nx;
    const int k = r / Ny, j = r - k * Ny;
    T p[3], k0[3];
    double sn = 0.0, ms[6] = {0, 0, 0, 0, 0, 0};
    node_eval<T, true>(g, B.u, B.lam, B.mu, i, j, k, p, k0, sn, ms);
    acc[1] += sn;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[2 + q] += ms[q];
    const uint8_t m = B.mask[node];
    if (ct.on && (m & M_FACE)) {
      const int xyz[3] = {i, j, k};
      const long long f = (long long)xyz[ct.b1] + (long long)g.N[ct.b1] * xyz[ct.b2];
      const double X0 = i + (double)B.u[node], X1 = j + (double)B.u[Nn + node], X2 = k + (double)B.u[2 * Nn + node];
      const double d0 = X0 - ct.center[0], d1 = X1 - ct.center[1], d2 = X2 - ct.center[2];
      const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
      const double gap = rr - ct.radius;
      const double n0 = -d0 / rr, n1 = -d1 / rr, n2 = -d2 / rr;
      const double pn = (double)p[0] * n0 + (double)p[1] * n1 + (double)p[2] * n2;
      const int b = bcount(g, xyz);
      const double fnc = -pn / (double)(1 << b);
      const uint8_t inC = ct.C[f];
      if (inC) {
        p[0] = (T)((double)p[0] - pn * n0);
        p[1] = (T)((double)p[1] - pn * n1);
        p[2] = (T)((double)p[2] - pn * n2);
      }
      ct.V[cur][f] = (uint8_t)(((!inC) && gap < 0.0) ? 1 : 0) | (uint8_t)((inC && fnc > 0.0) ? 2 : 0);
      ct.fnc[f] = fnc;
      ct.gap[f] = gap;
      acc[0] += (double)p[0] * p[0] + (double)p[1] * p[1] + (double)p[2] * p[2];
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (m & (M_STRONG << c)) p[c] = T(0);
        else if (!(m & (M_WEAK << c))) acc[0] += (double)p[c] * p[c];
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) B.X[c * Nn + node] = write_p ? p[c] : p[c] + k0[c];
  }
  block_sum<kPartStride>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < kPartStride; ++q) part[blockIdx.x * kPartStride + q] = acc[q];
}

// Residual only (no norms) for a list of nodes: used by the weak projection and reactions.
template <typename T>
__device__ __forceinline__ void node_p(const Geo& g, const Bufs<T>& B, long long node, T p[3], int& b) {
  const int Nx = g.N[0], Ny = g.N[1];
  const int i = (int)(node % Nx);
  const long long r = node / Nx;
  const int j = (int)(r % Ny), k = (int)(r / Ny);
  T k0[3];
  double sn = 0.0, ms[6];
  node_eval<T, false>(g, B.u, B.lam, B.mu, i, j, k, p, k0, sn, ms);
  const int xyz[3] = {i, j, k};
  b = bcount(g, xyz);
}

// proj_P of the average relations (eq 14) on the physical residual 2^-b p.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_weak(Geo g, Bufs<T> B, WeakDev w, DevState* st, int force) {
  if (!force && st->done) return;
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= w.m) return;
  const int c = w.comp[r];
  const int k = weak_size(w, r);
  double phys[8], wb[8];
  double sum = 0.0;
  for (int s = 0; s < k; ++s) {
    T p[3];
    int b;
    node_p<T>(g, B, w.nodes[r * w.k + s], p, b);
    wb[s] = (double)(1 << b);
    phys[s] = (double)p[c] / wb[s];
    sum += phys[s];
  }
  const double mean = sum / k;
  double pn = 0.0;
  for (int s = 0; s < k; ++s) {
    const long long node = w.nodes[r * w.k + s];
    const double pnew = (phys[s] - mean) * wb[s];
    pn += pnew * pnew;
    B.X[c * g.Nn + node] = (T)((double)B.X[c * g.Nn + node] - mean * wb[s]);
  }
  w.part[r] = pn;
  w.react[r] = -sum;
}

// ---------------------------------------------------------------------------
// Control: equilibrium test, contact update, Anderson flags (one block)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void k_control(DevState* st, const double* __restrict__ part, int nblk,
                                                    const double* __restrict__ wpart, long long nweak, ContactDev ct,
                                                    int pstride) {
  __shared__ double sh[kPartStrideD * 16];
  __shared__ int flags[4];
  if (st->done) return;
  double acc[kPartStrideD];
#pragma unroll
  for (int q = 0; q < kPartStrideD; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
    for (int q = 0; q < pstride; ++q) acc[q] += part[b * pstride + q];
  for (long long r = threadIdx.x; r < nweak; r += blockDim.x) acc[0] += wpart[r];
  block_sum<kPartStrideD>(acc, sh);
  if (threadIdx.x == 0) {
    st->pnorm2 = acc[0];
    st->snorm2 = acc[1];
    for (int q = 0; q < 6; ++q) st->ms[q] = acc[2 + q];
    if (pstride > kPartStride)
      for (int q = 0; q < 6; ++q) st->sing[q] = acc[8 + q];
    flags[0] = flags[1] = 0;
  }
  __syncthreads();
  // contact: compare V with the previous iteration, test emptiness
  if (ct.on) {
    const int cur = st->vpar;
    int differ = 0, nonempty = 0;
    for (long long f = threadIdx.x; f < ct.nface; f += blockDim.x) {
      const uint8_t v = ct.V[cur][f];
      nonempty |= (v != 0);
      differ |= (v != ct.V[cur ^ 1][f]);
    }
    if (differ) atomicOr(&flags[0], 1);
    if (nonempty) atomicOr(&flags[1], 1);
    __syncthreads();
  }
  __shared__ int decide, s_done, changed;
  if (threadIdx.x == 0) {
    const double pn = st->pnorm2, sn = st->snorm2;
    double res;
    if (pn == 0.0) res = 0.0;
    else if (sn == 0.0) res = INFINITY;
    else res = sqrt(pn) / sqrt(sn);
    st->residual = res;
    decide = 0;
    changed = 0;
    s_done = 0;
    const int nonempty = ct.on ? flags[1] : 0;
    st->vnonempty = nonempty;
    if (!isfinite(pn) || !isfinite(sn)) {
      st->status = ST_NAN;
      s_done = 1;
    } else if (res < st->tol && !nonempty) {
      st->status = ST_CONVERGED;
      s_done = 1;
    } else if (st->it >= st->max_iter) {
      st->status = ST_NOCONV;
      s_done = 1;
    } else {
      if (ct.on && st->have_prev && !flags[0] && nonempty && res < st->gate) decide = 1;
    }
    if (s_done) st->done = 1;
  }
  __syncthreads();
  if (s_done) return;
  if (ct.on) {
    if (decide) {
      const int cur = st->vpar;
      int ch = 0;
      for (long long f = threadIdx.x; f < ct.nface; f += blockDim.x) {
        const uint8_t v = ct.V[cur][f];
        const uint8_t old = ct.C[f];
        const uint8_t nw = (uint8_t)((old || (v & 1)) && !(v & 2));
        if (nw != old) {
          ct.C[f] = nw;
          ch = 1;
        }
      }
      if (ch) atomicOr(&changed, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      if (decide) {
        st->updates += 1;
        if (changed) {
          st->i_local = 0;
          st->restarts += 1;
        }
      }
      st->have_prev = 1;
      st->vpar ^= 1;
    }
  }
  if (threadIdx.x == 0) {
    const int i = st->i_local;
    st->store_r = (st->acv == 2) && (i > 0);
    st->accel = (st->acv == 2) && (i >= 4) && (i % st->period == 0);
    st->accel_ok = 0;
  }
}

// ---------------------------------------------------------------------------
// Anderson: R_{i-1 mod 4} = p~ - S_{i-1 mod 4}; Gram partials when accelerating
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_anderson_r(Bufs<T> B, long long n3, DevState* st,
                                                       double* __restrict__ gpart) {
  __shared__ double sh[10 * 16];
  if (st->done) return;
  const int store = st->store_r, accel = st->accel;
  if (!store && !accel) return;
  const int i = st->i_local;
  const int s = (i + 3) & 3;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  T* Rs = B.R[s];
  const T* Ss = B.S[s];
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    T r[4];
    if (store) {
      r[s] = B.X[e] - Ss[e];
      Rs[e] = r[s];
    }
    if (accel) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q != s || !store) r[q] = B.R[q][e];
      int t = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a; b < 4; ++b) acc[t++] += (double)r[a] * (double)r[b];
    }
  }
  if (!accel) return;
  block_sum<10>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 10; ++q) gpart[blockIdx.x * 10 + q] = acc[q];
}

// alpha = argmin |sum a_k R_k|, sum a_k = 1, from the regularised FP64 Gram matrix.
__global__ __launch_bounds__(kBlock) void k_alpha(DevState* st, const double* __restrict__ gpart, int nblk) {
  __shared__ double sh[10 * 16];
  if (st->done || !st->accel) return;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int q = 0; q < 10; ++q) acc[q] += gpart[b * 10 + q];
  block_sum<10>(acc, sh);
  if (threadIdx.x != 0) return;
  double G[4][5];
  int t = 0;
  for (int a = 0; a < 4; ++a)
    for (int b = a; b < 4; ++b) {
      G[a][b] = acc[t];
      G[b][a] = acc[t];
      ++t;
    }
  for (int a = 0; a < 4; ++a)
    for (int b = 0; b < 4; ++b) st->gram[a * 4 + b] = G[a][b];
  const double tr = G[0][0] + G[1][1] + G[2][2] + G[3][3];
  for (int a = 0; a < 4; ++a) {
    G[a][a] += 1e-14 * tr / 4.0;
    G[a][4] = 1.0;
  }
  // Gaussian elimination with partial pivoting
  bool ok = true;
  for (int col = 0; col < 4 && ok; ++col) {
    int piv = col;
    double best = fabs(G[col][col]);
    for (int r = col + 1; r < 4; ++r)
      if (fabs(G[r][col]) > best) {
        best = fabs(G[r][col]);
        piv = r;
      }
    if (!(best > 0.0)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int q = 0; q < 5; ++q) {
        const double tmp = G[col][q];
        G[col][q] = G[piv][q];
        G[piv][q] = tmp;
      }
    for (int r = col + 1; r < 4; ++r) {
      const double f = G[r][col] / G[col][col];
      for (int q = col; q < 5; ++q) G[r][q] -= f * G[col][q];
    }
  }
  double y[4] = {0, 0, 0, 0};
  if (ok) {
    for (int r = 3; r >= 0; --r) {
      double s = G[r][4];
      for (int q = r + 1; q < 4; ++q) s -= G[r][q] * y[q];
      y[r] = s / G[r][r];
    }
    const double sy = y[0] + y[1] + y[2] + y[3];
    ok = isfinite(sy) && sy != 0.0 && isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]) && isfinite(y[3]);
    if (ok)
      for (int a = 0; a < 4; ++a) st->alpha[a] = y[a] / sy;
  }
  st->accel_ok = ok ? 1 : 0;
}

// ---------------------------------------------------------------------------
// Batched per-axis discrete trigonometric transforms in LDS
// ---------------------------------------------------------------------------
template <typename T, int R>
__device__ __forceinline__ void dft_small(cplx<T> (&a)[R], int sgn) {
  if constexpr (R == 2) {
    const cplx<T> t0 = cadd(a[0], a[1]), t1 = csub(a[0], a[1]);
    a[0] = t0;
    a[1] = t1;
  } else if constexpr (R == 3) {
    const T c1 = T(-0.5), s1 = T(sgn) * T(0.86602540378443864676);
    const cplx<T> sum = cadd(a[1], a[2]), dif = csub(a[1], a[2]);
    const cplx<T> m = {a[0].re + c1 * sum.re, a[0].im + c1 * sum.im};
    const cplx<T> rot = {-s1 * dif.im, s1 * dif.re};   // i * s1 * dif
    a[0] = cadd(a[0], sum);
    a[1] = cadd(m, rot);
    a[2] = csub(m, rot);
  } else if constexpr (R == 4) {
    const cplx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const cplx<T> t2 = cadd(a[1], a[3]), d = csub(a[1], a[3]);
    const cplx<T> t3 = {-T(sgn) * d.im, T(sgn) * d.re};   // sgn * i * d
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(sgn) * T(0.95105651629515357212), s2 = T(sgn) * T(0.58778525229247312917);
    const cplx<T> b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
    const cplx<T> d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    const cplx<T> m1 = {a[0].re + c1 * b1.re + c2 * b2.re, a[0].im + c1 * b1.im + c2 * b2.im};
    const cplx<T> m2 = {a[0].re + c2 * b1.re + c1 * b2.re, a[0].im + c2 * b1.im + c1 * b2.im};
    // rotations i*(s1 d1 + s2 d2) and i*(s2 d1 - s1 d2)
    const cplx<T> r1 = {-(s1 * d1.im + s2 * d2.im), s1 * d1.re + s2 * d2.re};
    const cplx<T> r2 = {-(s2 * d1.im - s1 * d2.im), s2 * d1.re - s1 * d2.re};
    a[0] = {a[0].re + b1.re + b2.re, a[0].im + b1.im + b2.im};
    a[1] = cadd(m1, r1);
    a[4] = csub(m1, r1);
    a[2] = cadd(m2, r2);
    a[3] = csub(m2, r2);
  }
}

// One Stockham stage of radix R over L lines of length n (single LDS buffer,
// register staging between a read phase and a write phase).
template <typename T, int R, int EPT>
__device__ __forceinline__ void fft_stage(cplx<T>* buf, int cstride, int L, int n, int Ns, int sgn,
                                          const cplx<T>* __restrict__ tw) {
  constexpr int MAXW = (EPT + R - 1) / R;
  const int nb = n / R;
  const int total = L * nb;
  cplx<T> v[MAXW][R];
#pragma unroll
  for (int t = 0; t < MAXW; ++t) {
    const int w = threadIdx.x + t * kBlock;
    if (w < total) {
      const int line = w / nb, jj = w - line * nb;
      const cplx<T>* src = buf + line * cstride + jj;
#pragma unroll
      for (int q = 0; q < R; ++q) v[t][q] = src[q * nb];
    }
  }
  __syncthreads();
  const int step = n / (Ns * R);
#pragma unroll
  for (int t = 0; t < MAXW; ++t) {
    const int w = threadIdx.x + t * kBlock;
    if (w < total) {
      const int line = w / nb, jj = w - line * nb;
      const int kk = jj % Ns;
      if (Ns > 1) {
#pragma unroll
        for (int q = 1; q < R; ++q) {
          cplx<T> f = tw[4 * (q * kk * step)];
          if (sgn > 0) f.im = -f.im;
          v[t][q] = cmul(v[t][q], f);
        }
      }
      dft_small<T, R>(v[t], sgn);
      cplx<T>* dst = buf + line * cstride + (jj / Ns) * Ns * R + kk;
#pragma unroll
      for (int q = 0; q < R; ++q) dst[q * Ns] = v[t][q];
    }
  }
  __syncthreads();
}

template <typename T, int EPT>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, int cstride, int L, const AxisPlan& ap, int sgn) {
  const cplx<T>* tw = (const cplx<T>*)ap.tw;
  int Ns = 1;
  for (int s = 0; s < ap.nrad; ++s) {
    const int r = ap.rad[s];
    if (r == 4) fft_stage<T, 4, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else if (r == 2) fft_stage<T, 2, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else if (r == 3) fft_stage<T, 3, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else fft_stage<T, 5, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    Ns *= r;
  }
}

// FFT direction of each (type, forward/inverse): -1 = e^{-i}, +1 = e^{+i}
__device__ __forceinline__ int fft_sign(int type, int inv) {
  if (!inv) return (type == T_DCT3 || type == T_DST3) ? +1 : -1;
  return (type == T_DFT) ? +1 : -1;
}

// Symbol of the Paux stencil for component c from per-axis s = sin^2(theta/2),
// q = cos^2(theta/2): M = 4 sum_J a_J (s_J q_K q_L + q_J s_K s_L) -- the factored form of
// d + 4 (e_xy Cx Cy + e_xz Cx Cz + e_yz Cy Cz), exact at theta = 0 and (pi, pi, pi).
__device__ __forceinline__ double paux_symbol(const double a[3], double sx, double qx, double sy, double qy,
                                              double sz, double qz) {
  return 4.0 * (a[0] * (sx * qy * qz + qx * sy * sz) + a[1] * (sy * qx * qz + qy * sx * sz) +
                a[2] * (sz * qx * qy + qz * sx * sy));
}

// Residual-form update in the last inverse pass: delta = K0^+ e - (I - Pi) u, u += delta,
// at node (i, j, k) of component c.
template <typename T>
__device__ __forceinline__ void dtt_update(const DttArgs<T>& a, int c, int i, int j, int k, long long addr, T v) {
  double d = (double)v;
  const int sg = a.g.sing[c];
  if (sg) {
    const double s0 = a.st->sing[2 * c], s1 = a.st->sing[2 * c + 1];
    const int parity = (i + j + k) & 1;
    d -= a.g.sing_scale[c] * (s0 + ((sg & 2) ? (parity ? -s1 : s1) : 0.0));
  }
  a.u64[addr] += d;
  a.delta[addr] = (T)d;
}

// Pre-processing: complex input z_k (k < n) of the length-n FFT from the real line x.
template <typename T>
__device__ __forceinline__ cplx<T> dtt_pre(int type, int inv, const T* x, int n, int k, const cplx<T>* tw) {
  if (type == T_DCT1) {
    const int j0 = 2 * k, j1 = 2 * k + 1;
    const T a = x[j0 <= n ? j0 : 2 * n - j0];
    const T b = x[j1 <= n ? j1 : 2 * n - j1];
    return {a, b};
  }
  if (type == T_DST1) {
    const int j0 = 2 * k, j1 = 2 * k + 1;
    const T a = (j0 == 0 || j0 == n) ? T(0) : (j0 < n ? x[j0] : -x[2 * n - j0]);
    const T b = (j1 == n) ? T(0) : (j1 < n ? x[j1] : -x[2 * n - j1]);
    return {a, b};
  }
  if (type == T_DFT) {
    if (!inv) return {x[k], T(0)};
    if (k == 0) return {x[0], T(0)};
    if (2 * k == n) return {x[k], T(0)};
    if (2 * k < n) return {x[k], x[n - k]};
    return {x[n - k], -x[k]};
  }
  if (!inv) {
    // DCT3 / DST3 forward: W_k = e^{+i pi k / 2n} (a - i b)
    T a, b;
    if (type == T_DCT3) {
      a = x[k];
      b = (k == 0) ? T(0) : x[n - k];
    } else {
      a = x[n - k];
      b = (k == 0) ? T(0) : x[k];
    }
    const cplx<T> w = cconj(tw[k]);
    return cmul(w, cplx<T>{a, -b});
  }
  // inverse of DCT3 (DCT2) / of DST3 (DST2 via alternating signs): reordered real input
  const int h = (n + 1) / 2;
  if (k < h) return {x[2 * k], T(0)};
  const T v = x[2 * n - 1 - 2 * k];
  return {type == T_DST3 ? -v : v, T(0)};
}

// Post-processing: real output at storage index m (0..N-1) from the FFT result Z.
template <typename T>
__device__ __forceinline__ T dtt_post(int type, int inv, const cplx<T>* Z, int n, int m, const cplx<T>* tw) {
  if (type == T_DCT1 || type == T_DST1) {
    if (type == T_DST1 && (m == 0 || m == n)) return T(0);
    const cplx<T> Zm = Z[m == n ? 0 : m];
    const cplx<T> Zc = cconj(Z[m == 0 ? 0 : n - m]);
    const cplx<T> E = {(Zm.re + Zc.re) * T(0.5), (Zm.im + Zc.im) * T(0.5)};
    const cplx<T> D = {(Zm.re - Zc.re) * T(0.5), (Zm.im - Zc.im) * T(0.5)};
    const cplx<T> O = {D.im, -D.re};   // D / i
    const cplx<T> Y = cadd(E, cmul(tw[2 * m], O));
    const T s = inv ? T(1) / T(2 * n) : T(1);
    return (type == T_DCT1 ? Y.re : -Y.im) * s;
  }
  if (type == T_DFT) {
    if (inv) return Z[m].re / T(n);
    return (2 * m <= n) ? Z[m].re : Z[n - m].im;
  }
  if (!inv) {
    if (m >= n) return T(0);
    const int h = (m & 1) ? (n - 1 - (m - 1) / 2) : (m / 2);
    const T v = Z[h].re;
    return (type == T_DST3 && (m & 1)) ? -v : v;
  }
  // inverse: DCT2 (nodes 0..n-1) or DST2 (nodes 1..n), scaled by 1/2n
  if (type == T_DCT3) {
    if (m >= n) return T(0);
    return cmul(tw[m], Z[m]).re / T(n);
  }
  if (m == 0) return T(0);
  const int kk = n - m;
  return cmul(tw[kk], Z[kk]).re / T(n);
}


template <typename T, int EPT>
__global__ __launch_bounds__(kBlock) void k_dtt(DttArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (!a.force && a.st->done) return;
  const int c = blockIdx.y;
  const int n = a.ap.n, N = a.ap.N, L = a.ap.L;
  const int Nx = a.g.N[0], Ny = a.g.N[1];
  const long long Nn = a.g.Nn;
  const int axis = a.axis;
  const long long nlines = axis == 0 ? (long long)Ny * a.g.N[2] : axis == 1 ? (long long)Nx * a.g.N[2] : (long long)Nx * Ny;
  const long long stride = axis == 0 ? 1 : axis == 1 ? Nx : (long long)Nx * Ny;
  const long long l0 = (long long)blockIdx.x * L;
  const int cstride = n + 1, rstride = N + 1;
  cplx<T>* cb = (cplx<T>*)smem;
  T* rb = (T*)(smem + sizeof(cplx<T>) * (size_t)L * cstride);
  const cplx<T>* tw = (const cplx<T>*)a.ap.tw;
  const int type = a.types[c];
  auto off = [&](long long l) -> long long {
    if (axis == 0) return l * Nx;
    if (axis == 1) return (l / Nx) * ((long long)Nx * Ny) + (l % Nx);
    return l;
  };
  const long long cbase = (long long)c * Nn;
  // phase 1: gather the real lines into LDS (each node once)
  const int inv_first = (a.mode == PASS_INV);
  {
    const int total = L * N;
    int slot = 0, acc_ok = 0;
    double al[4] = {0, 0, 0, 0};
    if (a.src == SRC_ANDERSON) {
      slot = a.st->i_local & 3;
      acc_ok = a.st->accel_ok;
      if (acc_ok)
        for (int q = 0; q < 4; ++q) al[q] = a.st->alpha[q];
    }
    for (int w = threadIdx.x; w < total; w += kBlock) {
      int l, m;
      if (axis == 0) { l = w / N; m = w - l * N; } else { m = w / L; l = w - m * L; }
      const long long lg = l0 + l;
      T v = T(0);
      if (lg < nlines) {
        const long long addr = cbase + off(lg) + (long long)m * stride;
        if (a.src == SRC_ANDERSON) {
          if (acc_ok) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < 4; ++q) s += al[q] * ((double)a.B.S[q][addr] + (double)a.B.R[q][addr]);
            v = (T)s;
          } else {
            v = a.B.X[addr];
          }
          if (a.store_s) a.B.S[slot][addr] = v;
        } else if (a.src == SRC_DELTA) {
          v = a.dp2[a.st->it & 1][addr];
          if (a.st->accel_ok)
            v = v - ((T)a.st->gamma[0] * a.dY[0][addr] + (T)a.st->gamma[1] * a.dY[1][addr] +
                     (T)a.st->gamma[2] * a.dY[2][addr]);
          a.de[addr] = v;
        } else {
          v = a.in[addr];
        }
      }
      rb[l * rstride + m] = v;
    }
  }
  __syncthreads();
  // phase 2 + 3: pre-process and FFT
  {
    const int sg = fft_sign(type, inv_first);
    for (int w = threadIdx.x; w < L * n; w += kBlock) {
      const int l = w / n, k = w - l * n;
      cb[l * cstride + k] = dtt_pre<T>(type, inv_first, rb + l * rstride, n, k, tw);
    }
    __syncthreads();
    fft_lines<T, EPT>(cb, cstride, L, a.ap, sg);
  }
  if (a.mode == PASS_FWD_GREEN_INV) {
    // forward post-processing, Green operator M^-1, back into LDS
    const double* sxT = a.cosT + ((c * 3 + 0) * 2 + 0) * a.maxN;
    const double* qxT = a.cosT + ((c * 3 + 0) * 2 + 1) * a.maxN;
    const double* syT = a.cosT + ((c * 3 + 1) * 2 + 0) * a.maxN;
    const double* qyT = a.cosT + ((c * 3 + 1) * 2 + 1) * a.maxN;
    const double* szT = a.cosT + ((c * 3 + 2) * 2 + 0) * a.maxN;
    const double* qzT = a.cosT + ((c * 3 + 2) * 2 + 1) * a.maxN;
    for (int w = threadIdx.x; w < L * N; w += kBlock) {
      const int l = w / N, m = w - l * N;
      const long long lg = l0 + l;
      T v = dtt_post<T>(type, 0, cb + l * cstride, n, m, tw);
      if (lg < nlines) {
        const int mx = (int)(lg % Nx), my = (int)(lg / Nx);
        const double M = paux_symbol(a.g.ac[c], sxT[mx], qxT[mx], syT[my], qyT[my], szT[m], qzT[m]);
        v = (M > a.thr[c]) ? (T)((double)v / M) : T(0);
      } else {
        v = T(0);
      }
      rb[l * rstride + m] = v;
    }
    __syncthreads();
    const int itype = type;
    const int sg = fft_sign(itype, 1);
    for (int w = threadIdx.x; w < L * n; w += kBlock) {
      const int l = w / n, k = w - l * n;
      cb[l * cstride + k] = dtt_pre<T>(itype, 1, rb + l * rstride, n, k, tw);
    }
    __syncthreads();
    fft_lines<T, EPT>(cb, cstride, L, a.ap, sg);
  }
  // phase 4: post-process and write
  const int inv_out = (a.mode != PASS_FWD);
  {
    const int total = L * N;
    for (int w = threadIdx.x; w < total; w += kBlock) {
      int l, m;
      if (axis == 0) { l = w / N; m = w - l * N; } else { m = w / L; l = w - m * L; }
      const long long lg = l0 + l;
      if (lg >= nlines) continue;
      const T v = dtt_post<T>(type, inv_out, cb + l * cstride, n, m, tw);
      const long long addr = cbase + off(lg) + (long long)m * stride;
      if (a.dst == DST_UPDATE) {
        int xi, yj, zk;
        if (axis == 0) { xi = m; yj = (int)(lg % Ny); zk = (int)(lg / Ny); }
        else if (axis == 1) { xi = (int)(lg % Nx); yj = m; zk = (int)(lg / Nx); }
        else { xi = (int)(lg % Nx); yj = (int)(lg / Nx); zk = m; }
        dtt_update<T>(a, c, xi, yj, zk, addr, v);
      } else {
        a.buf[addr] = v;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// DTT pass with a compile-time length (non-periodic axes, n in {16,32,48,64,96,128,256})
// ---------------------------------------------------------------------------
template <typename T, int NF, int NTH, int TY = -1>
__global__ __launch_bounds__(NTH) void k_dtt2(DttArgs<T> a) {
  using S = DttShape<NF, NTH>;
  constexpr int LB = S::LB, NN = S::NN, CS = S::CS, RS = S::RS, NT = S::NT;
  extern __shared__ __align__(16) unsigned char smem[];
  if (!a.force && a.st->done) return;
  // Blocks are dispatched to the 8 XCDs round-robin in linear order; renumber them so that
  // every XCD works on a contiguous range of (chunk, plane, component) and the chunks that
  // share 128-byte lines of a y or z line meet in one L2.
  unsigned bxi, byi, c;
  {
    const unsigned G = gridDim.x * gridDim.y * gridDim.z;
    const unsigned p = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
    const unsigned q = G / 8, r = G % 8, xcd = p % 8, slot = p / 8;
    const unsigned L = xcd * q + (xcd < r ? xcd : r) + slot;
    bxi = L % gridDim.x;
    byi = (L / gridDim.x) % gridDim.y;
    c = L / (gridDim.x * gridDim.y);
  }
  const int axis = a.axis;
  const int Nx = a.g.N[0], Ny = a.g.N[1];
  long long base;
  int nl, lstride, estride;
  if (axis == 0) {
    const int y0 = (int)bxi * LB;
    nl = Ny - y0;
    base = ((long long)(int)byi * Ny + y0) * Nx;
    lstride = Nx;
    estride = 1;
  } else if (axis == 1) {
    const int x0 = (int)bxi * LB;
    nl = Nx - x0;
    base = (long long)(int)byi * Nx * Ny + x0;
    lstride = 1;
    estride = Nx;
  } else {
    const int x0 = (int)bxi * LB;
    nl = Nx - x0;
    base = (long long)(int)byi * Nx + x0;
    lstride = 1;
    estride = Nx * Ny;
  }
  base += (long long)c * a.g.Nn;
  T* rb = (T*)smem;
  cplx<T>* cb = (cplx<T>*)smem;
  // twiddles e^{-2 pi i s / 4NF} staged in LDS after the line buffer: s <= 2 NF covers the
  // pre- and post-processing, and the FFT folds its larger indices onto that range
  cplx<T>* tws = (cplx<T>*)smem + LB * CS;
  {
    const cplx<T>* twg = (const cplx<T>*)a.ap.tw;
    for (int s = threadIdx.x; s <= 2 * NF; s += NT) tws[s] = twg[s];
  }
  const cplx<T>* tw = tws;
  // TY >= 0: every component of this pass has transform type TY (fixed at compile time)
  const int type = TY >= 0 ? TY : a.types[c];
  const unsigned tid = threadIdx.x;
  constexpr int TL = NF / FftPlan<NF>::R1;   // threads per line in the FFT passes
  constexpr int NB = FftPlan<NF>::R1;        // body nodes (m < NF) per thread: LB NF = NT NB
  // Node ownership, the same in every phase: thread tid owns NB body nodes of the block's LB
  // lines and, when tid < LB, the last node (m = NF) of line tid.  y and z lines: the line
  // l = tid % LB is fixed and m = tid / LB + i TL, so that consecutive threads take
  // consecutive x.  x lines: m = tid % NF is fixed and l = tid / NF + i NT / NF (NF dividing
  // NT), else the flat index tid + i NT split into (line, node).  Offsets within one component
  // field fit in 32 bits (3 x nodes < 2^32 is checked at set-up).
  auto body = [&](auto mk, int i, unsigned& l, unsigned& m) {
    if constexpr (decltype(mk)::value == 1) {
      l = tid % LB;
      m = tid / LB + (unsigned)(i * TL);
    } else if constexpr (NT % NF == 0) {
      l = tid / NF + (unsigned)(i * (NT / NF));
      m = tid % NF;
    } else {
      const unsigned w = tid + (unsigned)(i * NT);
      l = w / NF;
      m = w % NF;
    }
  };
  // the element loops are compiled once per ownership map (axis is uniform), so that the
  // fixed line or node of a thread is loop-invariant
  auto by_map = [&](auto&& f) {
    if (axis != 0) f(std::integral_constant<int, 1>{});
    else f(std::integral_constant<int, 0>{});
  };
  const unsigned ls = (unsigned)lstride, es = (unsigned)estride;
  const bool has_tail = tid < (unsigned)LB;
  const bool tail_ok = has_tail && (int)tid < nl;
  const unsigned tail_off = tid * ls + (unsigned)NF * es;
  // gather the real lines into LDS: all loads of a thread are issued before any store (the
  // stores of S or e would otherwise hold back the next loads: the pointers may alias)
  auto gather = [&](auto fetch, auto keep) {
    by_map([&](auto mk) {
      T vals[NB + 1];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        vals[i] = ((int)l < nl) ? fetch(l * ls + m * es) : T(0);
      }
      vals[NB] = tail_ok ? fetch(tail_off) : T(0);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        if ((int)l < nl) keep(l * ls + m * es, vals[i]);
      }
      if (tail_ok) keep(tail_off, vals[NB]);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        rb[l * RS + m] = vals[i];
      }
      if (has_tail) rb[tid * RS + NF] = vals[NB];
    });
  };
  if (a.src == SRC_ANDERSON) {
    const int slot = a.st->i_local & 3;
    const int acc_ok = a.st->accel_ok;
    double al[4] = {0, 0, 0, 0};
    if (acc_ok)
      for (int q = 0; q < 4; ++q) al[q] = a.st->alpha[q];
    T* Sout = a.B.S[slot] + base;
    const int store_s = a.store_s;
    const T *S0 = a.B.S[0] + base, *S1 = a.B.S[1] + base, *S2 = a.B.S[2] + base, *S3 = a.B.S[3] + base;
    const T *R0 = a.B.R[0] + base, *R1 = a.B.R[1] + base, *R2 = a.B.R[2] + base, *R3 = a.B.R[3] + base;
    const T* X = a.B.X + base;
    const double al0 = al[0], al1 = al[1], al2 = al[2], al3 = al[3];
    gather(
        [&](unsigned off) -> T {
          if (acc_ok) {
            double s = al0 * ((double)S0[off] + (double)R0[off]);
            s += al1 * ((double)S1[off] + (double)R1[off]);
            s += al2 * ((double)S2[off] + (double)R2[off]);
            s += al3 * ((double)S3[off] + (double)R3[off]);
            return (T)s;
          }
          return X[off];
        },
        [&](unsigned off, T v) {
          if (store_s) Sout[off] = v;
        });
  } else if (a.src == SRC_DELTA) {
    const T* pcur = a.dp2[a.st->it & 1] + base;
    const int acc_ok = a.st->accel_ok;
    const T g0 = acc_ok ? (T)a.st->gamma[0] : T(0), g1 = acc_ok ? (T)a.st->gamma[1] : T(0),
            g2 = acc_ok ? (T)a.st->gamma[2] : T(0);
    const T *y0 = a.dY[0] + base, *y1 = a.dY[1] + base, *y2 = a.dY[2] + base;
    T* de = a.de + base;
    gather(
        [&](unsigned off) -> T {
          T v = pcur[off];
          if (acc_ok) v = v - (g0 * y0[off] + g1 * y1[off] + g2 * y2[off]);
          return v;
        },
        [&](unsigned off, T v) { de[off] = v; });
  } else {
    const T* in = a.in + base;
    gather([&](unsigned off) -> T { return in[off]; }, [&](unsigned, T) {});
  }
  __syncthreads();
  const int inv_first = (a.mode == PASS_INV);
  {
    auto ld = [&](int l, int k) { return pre_ct<T, NF>(type, inv_first, rb + l * RS, k, tw); };
    if (fft_sign(type, inv_first) < 0) fft_ct<T, NF, -1, NT>(cb, CS, tw, ld);
    else fft_ct<T, NF, +1, NT>(cb, CS, tw, ld);
  }
  if (a.mode == PASS_FWD_GREEN_INV) {
    // (z lines: block = x chunk bxi of the y plane byi)
    const double* sxT = a.cosT + ((c * 3 + 0) * 2 + 0) * a.maxN;
    const double* qxT = a.cosT + ((c * 3 + 0) * 2 + 1) * a.maxN;
    const double* syT = a.cosT + ((c * 3 + 1) * 2 + 0) * a.maxN;
    const double* qyT = a.cosT + ((c * 3 + 1) * 2 + 1) * a.maxN;
    const double* szT = a.cosT + ((c * 3 + 2) * 2 + 0) * a.maxN;
    const double* qzT = a.cosT + ((c * 3 + 2) * 2 + 1) * a.maxN;
    // symbol in the transform's precision: M = qz A(x, y) + sz B(x, y) with
    // A = 4 (a0 sx qy + a1 sy qx + a2 sx sy), B = 4 (a0 qx sy + a1 qy sx + a2 qx qy)
    const T sy = (T)syT[(int)byi], qy = (T)qyT[(int)byi];
    const T a0 = (T)a.g.ac[c][0], a1 = (T)a.g.ac[c][1], a2 = (T)a.g.ac[c][2];
    const T thr = (T)a.thr[c];
    const unsigned x0 = bxi * LB;
    auto green = [&](unsigned l, unsigned m) -> T {
      const T v = post_ct<T, NF>(type, 0, cb + l * CS, m, tw);
      const T sx = (T)sxT[x0 + l], qx = (T)qxT[x0 + l];
      const T A = T(4) * (a0 * sx * qy + a1 * sy * qx + a2 * sx * sy);
      const T B = T(4) * (a0 * qx * sy + a1 * qy * sx + a2 * qx * qy);
      const T M = (T)qzT[m] * A + (T)szT[m] * B;
      return (M > thr) ? v / M : T(0);
    };
    T vals[NB + 1];
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      unsigned l, m;
      body(std::integral_constant<int, 1>{}, i, l, m);
      vals[i] = ((int)l < nl) ? green(l, m) : T(0);
    }
    vals[NB] = tail_ok ? green(tid, NF) : T(0);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      unsigned l, m;
      body(std::integral_constant<int, 1>{}, i, l, m);
      rb[l * RS + m] = vals[i];
    }
    if (has_tail) rb[tid * RS + NF] = vals[NB];
    __syncthreads();
    auto ld = [&](int l, int k) { return pre_ct<T, NF>(type, 1, rb + l * RS, k, tw); };
    if (fft_sign(type, 1) < 0) fft_ct<T, NF, -1, NT>(cb, CS, tw, ld);
    else fft_ct<T, NF, +1, NT>(cb, CS, tw, ld);
  }
  // post-process and scatter
  const int inv_out = (a.mode != PASS_FWD);
  if (a.dst == DST_UPDATE) {
    // residual form, last inverse pass: read every old u of the thread first, then write u
    // and delta
    const double* u64r = a.u64 + base;
    double* u64w = a.u64 + base;
    T* dw = a.delta + base;
    // delta = K0^+ e minus the singular-mode part (I - Pi) u (null modes of K0), whose
    // coefficients are read once
    const int sg = a.g.sing[c];
    const double sc = a.g.sing_scale[c];
    const double s0 = sg ? a.st->sing[2 * c] : 0.0, s1 = sg ? a.st->sing[2 * c + 1] : 0.0;
    auto upd = [&](T v, unsigned l, unsigned m, unsigned off, double old) {
      double d = (double)v;
      if (sg) {
        const unsigned lg = bxi * LB + l;
        const unsigned parity = (m + lg + byi) & 1u;   // (i + j + k) mod 2 on every axis
        d -= sc * (s0 + ((sg & 2) ? (parity ? -s1 : s1) : 0.0));
      }
      u64w[off] = old + d;
      dw[off] = (T)d;
    };
    auto update = [&](auto mk, auto guarded) {
      constexpr bool G = decltype(guarded)::value;
      double uo[NB + 1];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        uo[i] = (!G || (int)l < nl) ? u64r[l * ls + m * es] : 0.0;
      }
      uo[NB] = tail_ok ? u64r[tail_off] : 0.0;
      // (the LDS reads are in bounds for every line of the block: only the stores are guarded)
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        const T v = post_ct<T, NF>(type, inv_out, cb + l * CS, m, tw);
        if (!G || (int)l < nl) upd(v, l, m, l * ls + m * es, uo[i]);
      }
      if (tail_ok) upd(post_ct<T, NF>(type, inv_out, cb + tid * CS, NF, tw), tid, NF, tail_off, uo[NB]);
    };
    if (axis != 0) update(std::integral_constant<int, 1>{}, std::true_type{});
    else if (nl >= LB) update(std::integral_constant<int, 0>{}, std::false_type{});
    else update(std::integral_constant<int, 0>{}, std::true_type{});
    return;
  }
  T* out = a.buf + base;
  // guarded: some lines of the block lie beyond the grid (last chunk only); x lines of a
  // full block take the unguarded copy, where the thread's fixed node is loop-invariant
  auto store = [&](auto mk, auto guarded) {
#pragma unroll
    for (int i = 0; i < NB; ++i) {
      unsigned l, m;
      body(mk, i, l, m);
      const T v = post_ct<T, NF>(type, inv_out, cb + l * CS, m, tw);
      if (!decltype(guarded)::value || (int)l < nl) out[l * ls + m * es] = v;
    }
  };
  if (axis != 0) store(std::integral_constant<int, 1>{}, std::true_type{});
  else if (nl >= LB) store(std::integral_constant<int, 0>{}, std::false_type{});
  else store(std::integral_constant<int, 0>{}, std::true_type{});
  if (tail_ok) out[tail_off] = post_ct<T, NF>(type, inv_out, cb + tid * CS, NF, tw);
}

// ---------------------------------------------------------------------------
// proj_U kernels and bookkeeping
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_weak(Geo g, T* u, WeakDev w, DevState* st, int force) {
  if (!force && st->done) return;
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= w.m) return;
  const int c = w.comp[r];
  const int k = weak_size(w, r);
  double s = 0.0;
  for (int q = 0; q < k; ++q) s += (double)u[c * g.Nn + w.nodes[r * w.k + q]];
  const double corr = w.val[r] - s / k;
  for (int q = 0; q < k; ++q) {
    const long long idx = c * g.Nn + w.nodes[r * w.k + q];
    u[idx] = (T)((double)u[idx] + corr);
  }
}

// radial projection of the active contact nodes onto the sphere (proj_U of eq 28)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_contact(Geo g, T* u, ContactDev ct, DevState* st, int force) {
  if (!force && st->done) return;
  const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f >= ct.nface || !ct.C[f]) return;
  int xyz[3];
  xyz[ct.axis] = ct.side ? g.n[ct.axis] : 0;
  xyz[ct.b1] = (int)(f % g.N[ct.b1]);
  xyz[ct.b2] = (int)(f / g.N[ct.b1]);
  const long long node = xyz[0] + (long long)g.N[0] * (xyz[1] + (long long)g.N[1] * xyz[2]);
  double d[3], r2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    d[c] = xyz[c] + (double)u[c * g.Nn + node] - ct.center[c];
    r2 += d[c] * d[c];
  }
  const double r = sqrt(r2);
  for (int c = 0; c < 3; ++c) u[c * g.Nn + node] = (T)(ct.center[c] + ct.radius * d[c] / r - xyz[c]);
}

// initial active set C = {g < 0} from the current u (start of an increment)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_contact_init(Geo g, const T* u, ContactDev ct) {
  const long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (f >= ct.nface) return;
  int xyz[3];
  xyz[ct.axis] = ct.side ? g.n[ct.axis] : 0;
  xyz[ct.b1] = (int)(f % g.N[ct.b1]);
  xyz[ct.b2] = (int)(f / g.N[ct.b1]);
  const long long node = xyz[0] + (long long)g.N[0] * (xyz[1] + (long long)g.N[1] * xyz[2]);
  double r2 = 0.0;
  for (int c = 0; c < 3; ++c) {
    const double d = xyz[c] + (double)u[c * g.Nn + node] - ct.center[c];
    r2 += d * d;
  }
  ct.C[f] = (sqrt(r2) - ct.radius < 0.0) ? 1 : 0;
  ct.V[0][f] = 0;
  ct.V[1][f] = 0;
}

// strong proj_U and the end-of-iteration counters
template <typename T>
__global__ __launch_bounds__(kBlock) void k_finish(Geo g, T* u, StrongDev s, DevState* st, int advance) {
  if (st->done) return;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < s.m; e += (long long)gridDim.x * blockDim.x)
    u[s.comp[e] * g.Nn + s.node[e]] = (T)s.val[e];
  if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
    st->it += 1;
    st->i_local += 1;
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_strong_scatter(Geo g, T* u, StrongDev s) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < s.m; e += (long long)gridDim.x * blockDim.x)
    u[s.comp[e] * g.Nn + s.node[e]] = (T)s.val[e];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reactions(Geo g, Bufs<T> B, StrongDev s, double* out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= s.m) return;
  T p[3];
  int b;
  node_p<T>(g, B, s.node[e], p, b);
  out[e] = -(double)p[s.comp[e]] / (double)(1 << b);
}

// elementwise conversion / utility kernels
template <typename A, typename Bt>
__global__ __launch_bounds__(kBlock) void k_convert(const A* __restrict__ in, Bt* __restrict__ out, long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = (Bt)in[e];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero_amask(Geo g, T* u) {
  for (long long node = blockIdx.x * (long long)blockDim.x + threadIdx.x; node < g.Nn;
       node += (long long)gridDim.x * blockDim.x) {
    const int i = (int)(node % g.N[0]);
    const long long r = node / g.N[0];
    const int xyz[3] = {i, (int)(r % g.N[1]), (int)(r / g.N[1])};
    for (int c = 0; c < 3; ++c)
      if (is_antisym(g, c, xyz)) u[c * g.Nn + node] = T(0);
  }
}

// stiffness check: finite values, mu >= 0, 3 lam + 2 mu >= 0; max lam, max mu
__global__ __launch_bounds__(kBlock) void k_check_stiffness(const double* lam, const double* mu, long long nv,
                                                            double* out /* per block: bad, maxl, maxm */) {
  __shared__ double sh[3 * 64];
  double bad = 0.0, ml = -INFINITY, mm = -INFINITY;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nv; e += (long long)gridDim.x * blockDim.x) {
    const double l = lam[e], m = mu[e];
    if (!isfinite(l) || !isfinite(m)) bad = fmax(bad, 2.0);
    else if (m < 0.0 || 3.0 * l + 2.0 * m < 0.0) bad = fmax(bad, 1.0);
    ml = fmax(ml, l);
    mm = fmax(mm, m);
  }
  for (int o = 32; o > 0; o >>= 1) {
    bad = fmax(bad, __shfl_xor(bad, o, 64));
    ml = fmax(ml, __shfl_xor(ml, o, 64));
    mm = fmax(mm, __shfl_xor(mm, o, 64));
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    sh[wid] = bad;
    sh[64 + wid] = ml;
    sh[128 + wid] = mm;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      sh[0] = fmax(sh[0], sh[w]);
      sh[64] = fmax(sh[64], sh[64 + w]);
      sh[128] = fmax(sh[128], sh[128 + w]);
    }
    out[blockIdx.x * 3 + 0] = sh[0];
    out[blockIdx.x * 3 + 1] = sh[64];
    out[blockIdx.x * 3 + 2] = sh[128];
  }
}

// Anderson on the displacement (ACV_U): flags at the start of the iteration, then the
// accelerated combination and the solution store after the residual store and LS.
__global__ void k_flags_u(DevState* st) {
  if (st->done) return;
  const int i = st->i_local;
  st->store_r = (i > 0);
  st->accel = (i >= 4) && (i % st->period == 0);
  st->accel_ok = 0;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_combine_u(Bufs<T> B, long long n3, DevState* st) {
  if (st->done) return;
  const int slot = st->i_local & 3, ok = st->accel_ok;
  double al[4];
  for (int q = 0; q < 4; ++q) al[q] = ok ? st->alpha[q] : 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    T v = B.u[e];
    if (ok) {
      double s = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) s += al[q] * ((double)B.S[q][e] + (double)B.R[q][e]);
      v = (T)s;
      B.u[e] = v;
    }
    B.S[slot][e] = v;
  }
}

// Contact force along the face normal: -side_sign * sum over C of f_nc n_c[axis] (FP64).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_contact_force(Geo g, const T* u, ContactDev ct, double* out) {
  __shared__ double sh[2 * 16];
  double acc[2] = {0.0, 0.0};
  for (long long f = blockIdx.x * (long long)blockDim.x + threadIdx.x; f < ct.nface; f += (long long)gridDim.x * blockDim.x) {
    if (!ct.C[f]) continue;
    int xyz[3];
    xyz[ct.axis] = ct.side ? g.n[ct.axis] : 0;
    xyz[ct.b1] = (int)(f % g.N[ct.b1]);
    xyz[ct.b2] = (int)(f / g.N[ct.b1]);
    const long long node = xyz[0] + (long long)g.N[0] * (xyz[1] + (long long)g.N[1] * xyz[2]);
    double d[3], r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      d[c] = xyz[c] + (double)u[c * g.Nn + node] - ct.center[c];
      r2 += d[c] * d[c];
    }
    const double nca = -d[ct.axis] / sqrt(r2);
    acc[0] += ct.fnc[f] * nca;
    acc[1] += 1.0;
  }
  block_sum<2>(acc, sh);
  if (threadIdx.x == 0) {
    out[2 * blockIdx.x] = acc[0];
    out[2 * blockIdx.x + 1] = acc[1];
  }
}

// Re-arm the iteration state for `iters` more iterations (fixed-count runs).
__global__ void k_extend(DevState* st, int iters, double tol) {
  st->done = 0;
  st->status = ST_RUNNING;
  st->max_iter = st->it + iters;
  st->tol = tol;
}

// ===========================================================================
// Residual-form iteration (FP32 fields, FP64 displacement).  The same fixed point as
// above with ACV_P, rearranged exactly: with y_i = p_i + K0 u_i the Green input of the
// paper's iteration, e_i = x_i - K0 u_i is residual-sized, u_{i+1} = Pi u_i + K0^+ e_i,
// and Anderson runs in difference form on
//   R_i = p_i + K0 delta_i - e_{i-1},  dR = R_i - R_{i-1},  dY = p_i - p_{i-1} + K0 delta_i,
//   e_i = p_i - sum_j gamma_j dY_j,  gamma = argmin |R_i - sum_j gamma_j dR_j|.
// Only residual-sized quantities pass through FP32 transforms.
// ===========================================================================

// K0 f at a node for the three components (Paux stencil, mirrored neighbours)
template <typename T>
__device__ __forceinline__ void stencil_k0(const Geo& g, const T* __restrict__ f, int i, int j, int k, T out[3]) {
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  const int xs[3] = {mirror_coord(g, i - 1, 0), i, mirror_coord(g, i + 1, 0)};
  const int ys[3] = {mirror_coord(g, j - 1, 1), j, mirror_coord(g, j + 1, 1)};
  const int zs[3] = {mirror_coord(g, k - 1, 2), k, mirror_coord(g, k + 1, 2)};
  auto at = [&](int c, int dx, int dy, int dz) {
    return f[c * Nn + (long long)xs[dx + 1] + (long long)Nx * ((long long)ys[dy + 1] + (long long)Ny * zs[dz + 1])];
  };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const T sxy = at(c, -1, -1, 0) + at(c, 1, -1, 0) + at(c, -1, 1, 0) + at(c, 1, 1, 0);
    const T sxz = at(c, -1, 0, -1) + at(c, 1, 0, -1) + at(c, -1, 0, 1) + at(c, 1, 0, 1);
    const T syz = at(c, 0, -1, -1) + at(c, 0, 1, -1) + at(c, 0, -1, 1) + at(c, 0, 1, 1);
    out[c] = T(g.st[c][0]) * at(c, 0, 0, 0) + T(g.st[c][1]) * sxy + T(g.st[c][2]) * sxz + T(g.st[c][3]) * syz;
  }
}

// p = 2^b div_D(sigma) from an FP64 displacement: neighbour differences are formed in
// FP64 and rounded once, the stress and divergence arithmetic is in T.
template <typename T, bool SIG>
__device__ __forceinline__ void node_eval_d(const Geo& g, const double* __restrict__ u, const T* __restrict__ lam,
                                            const T* __restrict__ mu, int i, int j, int k, T p[3], double& sn,
                                            double ms[6]) {
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  const int xs[3] = {mirror_coord(g, i - 1, 0), i, mirror_coord(g, i + 1, 0)};
  const int ys[3] = {mirror_coord(g, j - 1, 1), j, mirror_coord(g, j + 1, 1)};
  const int zs[3] = {mirror_coord(g, k - 1, 2), k, mirror_coord(g, k + 1, 2)};
  const long long self = (long long)i + (long long)Nx * ((long long)j + (long long)Ny * k);
  double u0[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) u0[c] = u[c * Nn + self];
  T nb[27][3];
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int nrm = (dx != 0) + (dy != 0) + (dz != 0);
        if (nrm != 2) continue;
        const long long idx = (long long)xs[dx + 1] + (long long)Nx * ((long long)ys[dy + 1] + (long long)Ny * zs[dz + 1]);
        const int q = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) nb[q][c] = (T)(u[c * Nn + idx] - u0[c]);
      }
#pragma unroll
  for (int c = 0; c < 3; ++c) nb[13][c] = T(0);
  T F[3] = {T(0), T(0), T(0)};
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
    int vx = i - ax, vy = j - ay, vz = k - az;
    bool inside = true;
    if (g.periodic[0]) { if (vx < 0) vx += g.n[0]; } else inside &= (vx >= 0 && vx < g.n[0]);
    if (g.periodic[1]) { if (vy < 0) vy += g.n[1]; } else inside &= (vy >= 0 && vy < g.n[1]);
    if (g.periodic[2]) { if (vz < 0) vz += g.n[2]; } else inside &= (vz >= 0 && vz < g.n[2]);
    if (!inside) continue;
    const long long vid = (long long)vx + (long long)g.n[0] * ((long long)vy + (long long)g.n[1] * vz);
    const T l = lam[vid], m = mu[vid];
    T G[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) G[r][s] = T(0);
    const int par = (ax + ay + az) & 1;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
      if (((cx + cy + cz) & 1) != par) continue;
      const int q = (cx - ax + 1) + 3 * (cy - ay + 1) + 9 * (cz - az + 1);
      const T sx = T(cx ? 0.5 : -0.5), sy = T(cy ? 0.5 : -0.5), sz = T(cz ? 0.5 : -0.5);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        G[r][0] += sx * nb[q][r];
        G[r][1] += sy * nb[q][r];
        G[r][2] += sz * nb[q][r];
      }
    }
    const T tr = G[0][0] + G[1][1] + G[2][2];
    const T s00 = l * tr + T(2) * m * G[0][0];
    const T s11 = l * tr + T(2) * m * G[1][1];
    const T s22 = l * tr + T(2) * m * G[2][2];
    const T s01 = m * (G[0][1] + G[1][0]);
    const T s02 = m * (G[0][2] + G[2][0]);
    const T s12 = m * (G[1][2] + G[2][1]);
    const T bx = T(ax ? 0.25 : -0.25), by = T(ay ? 0.25 : -0.25), bz = T(az ? 0.25 : -0.25);
    F[0] += bx * s00 + by * s01 + bz * s02;
    F[1] += bx * s01 + by * s11 + bz * s12;
    F[2] += bx * s02 + by * s12 + bz * s22;
    if (SIG && (a == 0 || a == 1)) {
      const double d00 = s00, d11 = s11, d22 = s22, d01 = s01, d02 = s02, d12 = s12;
      sn += 0.5 * (d00 * d00 + d11 * d11 + d22 * d22 + 2.0 * (d01 * d01 + d02 * d02 + d12 * d12));
      ms[0] += 0.5 * d00; ms[1] += 0.5 * d11; ms[2] += 0.5 * d22;
      ms[3] += 0.5 * d12; ms[4] += 0.5 * d02; ms[5] += 0.5 * d01;
    }
  }
  const int xyz[3] = {i, j, k};
  const T w2b = T(1 << bcount(g, xyz));
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = is_antisym(g, c, xyz) ? T(0) : -w2b * F[c];
}

// forward-transform weight of a node in the singular coefficients (DCT1 ends 1, interior 2; DFT 1)
__device__ __forceinline__ double sing_weight(const Geo& g, const int xyz[3]) {
  double w = 1.0;
#pragma unroll
  for (int J = 0; J < 3; ++J)
    if (!g.periodic[J] && xyz[J] > 0 && xyz[J] < g.n[J]) w *= 2.0;
  return w;
}

// Per-node part of the residual pass of the residual-form iteration, once p is known:
// singular-mode coefficients of u, contact bookkeeping or constraint masking, the norm of
// p, p itself, and (ACV_P, from the second iteration on) R_i = p_i + K0 delta_i - e_{i-1}
// with its differences.  kd = K0 delta at the node (read only when kd_used).
// Node inputs of the tail that do not depend on p: mask, e_{i-1}, p_{i-1}, R_{i-1}.
template <typename T>
struct TailIn {
  uint8_t m;
  T e[3], pp[3], rp[3];
};

template <typename T>
__device__ __forceinline__ void tail_load(const DeltaBufs<T>& D, long long Nn, bool kd_used, int il, const T* pp,
                                          const T* Rp, long long node, TailIn<T>& t) {
  t.m = D.mask[node];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    t.e[c] = T(0);
    t.pp[c] = T(0);
    t.rp[c] = T(0);
    if (kd_used) {
      t.e[c] = D.e[c * Nn + node];
      if (il >= 2) {
        t.pp[c] = pp[c * Nn + node];
        t.rp[c] = Rp[c * Nn + node];
      }
    }
  }
}

template <typename T>
__device__ __forceinline__ void delta_tail(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, int cur,
                                           bool kd_used, int il, int slot, T* pc, T* Rc, int i, int j, int k,
                                           long long node, T p[3], const T kd[3], const TailIn<T>& tin,
                                           double* acc) {
  const long long Nn = g.Nn;
  const int xyz[3] = {i, j, k};
  // singular-mode coefficients of u (projection Pi of the update)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (!g.sing[c]) continue;
    const double wu = sing_weight(g, xyz) * D.u[c * Nn + node];
    acc[8 + 2 * c] += wu;
    if (g.sing[c] & 2) acc[9 + 2 * c] += ((i + j + k) & 1) ? -wu : wu;
  }
  const uint8_t m = tin.m;
  if (ct.on && (m & M_FACE)) {
    const long long f = (long long)xyz[ct.b1] + (long long)g.N[ct.b1] * xyz[ct.b2];
    const double X0 = i + D.u[node], X1 = j + D.u[Nn + node], X2 = k + D.u[2 * Nn + node];
    const double d0 = X0 - ct.center[0], d1 = X1 - ct.center[1], d2 = X2 - ct.center[2];
    const double rr = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const double gap = rr - ct.radius;
    const double n0 = -d0 / rr, n1 = -d1 / rr, n2 = -d2 / rr;
    const double pn = (double)p[0] * n0 + (double)p[1] * n1 + (double)p[2] * n2;
    const double fnc = -pn / (double)(1 << bcount(g, xyz));
    const uint8_t inC = ct.C[f];
    if (inC) {
      p[0] = (T)((double)p[0] - pn * n0);
      p[1] = (T)((double)p[1] - pn * n1);
      p[2] = (T)((double)p[2] - pn * n2);
    }
    ct.V[cur][f] = (uint8_t)(((!inC) && gap < 0.0) ? 1 : 0) | (uint8_t)((inC && fnc > 0.0) ? 2 : 0);
    ct.fnc[f] = fnc;
    ct.gap[f] = gap;
    acc[0] += (double)p[0] * p[0] + (double)p[1] * p[1] + (double)p[2] * p[2];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (m & (M_STRONG << c)) p[c] = T(0);
      else if (!(m & (M_WEAK << c))) acc[0] += (double)p[c] * p[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) pc[c * Nn + node] = p[c];
  if (kd_used) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long e = c * Nn + node;
      const T Ri = p[c] + kd[c] - tin.e[c];
      Rc[e] = Ri;
      if (il >= 2) {
        D.dR[slot][e] = Ri - tin.rp[c];
        D.dY[slot][e] = p[c] - tin.pp[c] + kd[c];
      }
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_residual_d(Geo g, DeltaBufs<T> D, ContactDev ct, DevState* st,
                                                       double* __restrict__ part) {
  __shared__ double sh[kPartStrideD * 16];
  if (st->done) return;
  double acc[kPartStrideD];
#pragma unroll
  for (int q = 0; q < kPartStrideD; ++q) acc[q] = 0.0;
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  const int cur = ct.on ? st->vpar : 0;
  const int il = st->i_local, par = st->it & 1, acvp = (st->acv == 2);
  const int slot = (il + 1) % 3;   // (il - 2) mod 3
  const bool kd_used = acvp && il >= 1;
  T* pc = D.p[par];
  const T* pp = D.p[par ^ 1];
  T* Rc = D.R[par];
  const T* Rp = D.R[par ^ 1];
  long long lo, hi;
  xcd_chunk(Nn, lo, hi);
  for (long long node = lo + threadIdx.x; node < hi; node += blockDim.x) {
    const int nd = (int)node;
    const int r = nd / Nx;
    const int i = nd - r * Nx;
    const int k = r / Ny, j = r - k * Ny;
    T p[3];
    double sn = 0.0, ms[6] = {0, 0, 0, 0, 0, 0};
    node_eval_d<T, true>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
    acc[1] += sn;
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[2 + q] += ms[q];
    T kd[3] = {T(0), T(0), T(0)};
    if (kd_used) stencil_k0<T>(g, D.delta, i, j, k, kd);
    TailIn<T> tin;
    tail_load<T>(D, Nn, kd_used, il, pp, Rp, node, tin);
    delta_tail<T>(g, D, ct, cur, kd_used, il, slot, pc, Rc, i, j, k, node, p, kd, tin, acc);
  }
  block_sum<kPartStrideD>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < kPartStrideD; ++q) part[blockIdx.x * kPartStrideD + q] = acc[q];
}

// ---------------------------------------------------------------------------
// The same residual pass, tiled: a block owns a kTX x kTY column of nodes and marches
// along z over a segment of node planes.  Node planes of u (FP64) and of delta (with the
// stencil's mirrored / periodic halo) sit in LDS with a one-node halo; the stresses of the
// two tetrahedra of every voxel of a layer are formed once per block (differences of u
// taken in FP64 against the voxel's corner 000, then rounded) and serve the two node
// planes that bound the layer.  Every voxel's stress-norm and mean-stress terms are
// counted by the one block whose node column and segment contain its corner 000.
// ---------------------------------------------------------------------------
constexpr int kTX = 31, kTY = 7;                // 217 nodes; 32 x 8 = 256 voxels per layer
constexpr int kHX = kTX + 2, kHY = kTY + 2;   // node tile with halo: x0-1 .. x0+kTX
constexpr int kVX = kTX + 1, kVY = kTY + 1;   // voxels x0-1 .. x0+kTX-1
constexpr int kPlane = 3 * kHY * kHX;         // values of one staged node plane
constexpr int kPR = (kPlane + 255) / 256;     // of them per thread

// slot of node plane p in the four-plane ring of delta planes (p may be -1)
__device__ __forceinline__ int ring4(int p) { return p & 3; }

template <typename T>
__global__ __launch_bounds__(256) void k_residual_dt(Geo g, DeltaBufs<T> D, ContactDev ct, DevState* st,
                                                     double* __restrict__ part, TileGrid tg) {
  __shared__ double su[2][3][kHY][kHX];
  __shared__ T sdl[4][3][kHY][kHX];
  __shared__ T ss[2][12][kVY][kVX];   // stress component q of the voxels of a layer
  __shared__ double sh[kPartStrideD * 16];
  if (st->done) return;
  const int tid = threadIdx.x;
  // contiguous ranges of tiles per XCD (blocks go to the 8 XCDs round-robin), so that
  // neighbouring tiles share their halo lines in one L2
  int b;
  {
    const unsigned G = gridDim.x, p = blockIdx.x;
    const unsigned q = G / 8, r = G % 8, xcd = p % 8, slot = p / 8;
    b = (int)(xcd * q + (xcd < r ? xcd : r) + slot);
  }
  const int bx = b % tg.tx, by = (b / tg.tx) % tg.ty, bz = b / (tg.tx * tg.ty);
  const int x0 = bx * kTX, y0 = by * kTY;
  const int Nx = g.N[0], Ny = g.N[1], Nz = g.N[2];
  const int nx = g.n[0], ny = g.n[1], nz = g.n[2];
  const int zb = bz * tg.seg;
  const int ze = min(zb + tg.seg, Nz);
  const int Nn = (int)g.Nn;
  const int cur = ct.on ? st->vpar : 0;
  const int il = st->i_local, par = st->it & 1, acvp = (st->acv == 2);
  const int slot = (il + 1) % 3;
  const bool kd_used = acvp && il >= 1;
  T* pc = D.p[par];
  const T* pp = D.p[par ^ 1];
  T* Rc = D.R[par];
  const T* Rp = D.R[par ^ 1];
  double acc[kPartStrideD];
#pragma unroll
  for (int q = 0; q < kPartStrideD; ++q) acc[q] = 0.0;

  // Node planes are fetched into registers one step ahead and committed to LDS the next
  // step.  u: su[pz & 1], nodes outside the grid read as 0 (no voxel uses them); delta:
  // sdl[pz mod 4] with the stencil's halo (mirror or periodic image).
  double ru[kPR];
  T rd[kPR];
  auto fetch = [&](int pz) {
    int gz = pz;
    bool okz = true;
    if (g.periodic[2]) gz = (pz + Nz) % Nz;
    else okz = pz >= 0 && pz < Nz;
    const int mz = mirror_coord(g, pz, 2);
    const bool okm = mz >= 0 && mz < Nz;
#pragma unroll
    for (int r = 0; r < kPR; ++r) {
      const int e = tid + 256 * r;
      ru[r] = 0.0;
      rd[r] = T(0);
      if (e < kPlane) {
        const int c = e / (kHY * kHX), q = e - c * (kHY * kHX);
        const int hy = q / kHX, hx = q - hy * kHX;
        int gx = x0 - 1 + hx, gy = y0 - 1 + hy;
        bool ok = okz;
        if (g.periodic[0]) gx = (gx + Nx) % Nx;
        else ok = ok && gx >= 0 && gx < Nx;
        if (g.periodic[1]) gy = (gy + Ny) % Ny;
        else ok = ok && gy >= 0 && gy < Ny;
        if (ok) ru[r] = D.u[c * Nn + gx + Nx * (gy + Ny * gz)];
        if (kd_used) {
          const int mx = mirror_coord(g, x0 - 1 + hx, 0), my = mirror_coord(g, y0 - 1 + hy, 1);
          if (okm && mx >= 0 && mx < Nx && my >= 0 && my < Ny) rd[r] = D.delta[c * Nn + mx + Nx * (my + Ny * mz)];
        }
      }
    }
  };
  auto commit = [&](int pz) {
    double* du = &su[pz & 1][0][0][0];
    T* dd = &sdl[ring4(pz)][0][0][0];
#pragma unroll
    for (int r = 0; r < kPR; ++r) {
      const int e = tid + 256 * r;
      if (e < kPlane) {
        du[e] = ru[r];
        if (kd_used) dd[e] = rd[r];
      }
    }
  };
  // Every thread owns one voxel of a layer (kVX * kVY = 256): local (vlx, vly).
  const int vly = tid / kVX, vlx = tid - (tid / kVX) * kVX;
  const int vux = x0 - 1 + vlx, vuy = y0 - 1 + vly;   // unwrapped voxel coordinates
  int vxw = vux, vyw = vuy;
  bool vok = true;
  if (g.periodic[0]) vxw = (vux + nx) % nx;
  else vok = vux >= 0 && vux < nx;
  if (g.periodic[1]) vyw = (vuy + ny) % ny;
  else vok = vok && vuy >= 0 && vuy < ny;
  // Lame values of this thread's voxel in layer lz (fetched one step ahead)
  auto fetch_lm = [&](int lz, T& l, T& m, bool& ok) {
    int vz = lz;
    ok = vok;
    if (g.periodic[2]) vz = (lz + nz) % nz;
    else ok = ok && lz >= 0 && lz < nz;
    l = T(0);
    m = T(0);
    if (ok) {
      const int vid = vxw + nx * (vyw + ny * vz);
      l = D.lam[vid];
      m = D.mu[vid];
    }
  };
  // voxel layer lz (between node planes lz and lz+1, held in su[lz & 1] and su[(lz+1) & 1])
  auto layer = [&](int lz, bool own_z, T l, T m, bool ok) {
    const int lo = lz & 1, hi = (lz + 1) & 1;
    {
      const int ly = vly, lx = vlx;
      T (*out)[kVY][kVX] = ss[lz & 1];
      const int ux = vux, uy = vuy;
      if (!ok) {
#pragma unroll
        for (int q = 0; q < 12; ++q) out[q][ly][lx] = T(0);
        return;
      }
      T d[8][3];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double ref = su[lo][c][ly][lx];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
          d[cc][c] = cc == 0 ? T(0) : (T)(su[cz ? hi : lo][c][ly + cy][lx + cx] - ref);
        }
      }
      const bool own = own_z && ux >= x0 && ux < x0 + kTX && ux < nx && uy >= y0 && uy < y0 + kTY && uy < ny;
      T vs[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        T G[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q) G[r][q] = T(0);
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
          if (((cx + cy + cz) & 1) != t) continue;
          const T sx = T(cx ? 0.5 : -0.5), sy = T(cy ? 0.5 : -0.5), sz = T(cz ? 0.5 : -0.5);
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            G[r][0] += sx * d[cc][r];
            G[r][1] += sy * d[cc][r];
            G[r][2] += sz * d[cc][r];
          }
        }
        const T tr = G[0][0] + G[1][1] + G[2][2];
        const T s00 = l * tr + T(2) * m * G[0][0];
        const T s11 = l * tr + T(2) * m * G[1][1];
        const T s22 = l * tr + T(2) * m * G[2][2];
        const T s01 = m * (G[0][1] + G[1][0]);
        const T s02 = m * (G[0][2] + G[2][0]);
        const T s12 = m * (G[1][2] + G[2][1]);
        out[t * 6 + 0][ly][lx] = s00;
        out[t * 6 + 1][ly][lx] = s11;
        out[t * 6 + 2][ly][lx] = s22;
        out[t * 6 + 3][ly][lx] = s01;
        out[t * 6 + 4][ly][lx] = s02;
        out[t * 6 + 5][ly][lx] = s12;
        if (own) {
          // the voxel's two tetrahedra in T, added to the FP64 block sums once per voxel
          vs[0] += s00 * s00 + s11 * s11 + s22 * s22 + T(2) * (s01 * s01 + s02 * s02 + s12 * s12);
          vs[1] += s00;
          vs[2] += s11;
          vs[3] += s22;
          vs[4] += s12;
          vs[5] += s02;
          vs[6] += s01;
        }
      }
      if (own)
#pragma unroll
        for (int q = 0; q < 7; ++q) acc[1 + q] += 0.5 * (double)vs[q];
    }
  };
  const int nlx = tid % kTX, nly = tid / kTX;
  const bool nact = tid < kTX * kTY && x0 + nlx < Nx && y0 + nly < Ny;
  TailIn<T> tin;
  auto nodes = [&](int z) {
    if (!nact) return;
    const int lx = nlx, ly = nly;
    const int i = x0 + lx, j = y0 + ly;
    T F[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      // voxel (i - ax, j - ay, z - az): local voxel (lx + 1 - ax, ly + 1 - ay), layer z - az;
      // the node is its corner (ax, ay, az), in tetrahedron T1 (even) or T2 (odd)
      const int q0 = ((ax + ay + az) & 1) * 6, vy = ly + 1 - ay, vx = lx + 1 - ax;
      T (*sv)[kVY][kVX] = ss[(z - az) & 1];
      const T s00 = sv[q0 + 0][vy][vx], s11 = sv[q0 + 1][vy][vx], s22 = sv[q0 + 2][vy][vx];
      const T s01 = sv[q0 + 3][vy][vx], s02 = sv[q0 + 4][vy][vx], s12 = sv[q0 + 5][vy][vx];
      const T bxw = T(ax ? 0.25 : -0.25), byw = T(ay ? 0.25 : -0.25), bzw = T(az ? 0.25 : -0.25);
      F[0] += bxw * s00 + byw * s01 + bzw * s02;
      F[1] += bxw * s01 + byw * s11 + bzw * s12;
      F[2] += bxw * s02 + byw * s12 + bzw * s22;
    }
    const int xyz[3] = {i, j, z};
    const T w2b = T(1 << bcount(g, xyz));
    T p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = is_antisym(g, c, xyz) ? T(0) : -w2b * F[c];
    T kd[3] = {T(0), T(0), T(0)};
    if (kd_used) {
      const int zm = ring4(z - 1), z0 = ring4(z), zp = ring4(z + 1);
      const int hx = lx + 1, hy = ly + 1;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const T sxy = sdl[z0][c][hy - 1][hx - 1] + sdl[z0][c][hy - 1][hx + 1] + sdl[z0][c][hy + 1][hx - 1] +
                      sdl[z0][c][hy + 1][hx + 1];
        const T sxz = sdl[zm][c][hy][hx - 1] + sdl[zm][c][hy][hx + 1] + sdl[zp][c][hy][hx - 1] +
                      sdl[zp][c][hy][hx + 1];
        const T syz = sdl[zm][c][hy - 1][hx] + sdl[zm][c][hy + 1][hx] + sdl[zp][c][hy - 1][hx] +
                      sdl[zp][c][hy + 1][hx];
        kd[c] = T(g.st[c][0]) * sdl[z0][c][hy][hx] + T(g.st[c][1]) * sxy + T(g.st[c][2]) * sxz +
                T(g.st[c][3]) * syz;
      }
    }
    const long long node = (long long)i + (long long)Nx * ((long long)j + (long long)Ny * z);
    delta_tail<T>(g, D, ct, cur, kd_used, il, slot, pc, Rc, i, j, z, node, p, kd, tin, acc);
  };

  T lcur, mcur, lnext, mnext;
  bool okcur, oknext;
  fetch(zb - 1);
  commit(zb - 1);
  fetch(zb);
  commit(zb);
  fetch(zb + 1);
  fetch_lm(zb - 1, lcur, mcur, okcur);
  fetch_lm(zb, lnext, mnext, oknext);
  __syncthreads();
  layer(zb - 1, false, lcur, mcur, okcur);
  __syncthreads();
  // Per step, plane z + 1 is committed with no barrier before it: its u slot was last read
  // by layer(z - 1), and its delta slot (four-plane ring) by nodes(z - 2), both before the
  // barrier that follows layer(z - 1).  The stress slot written by layer(z) was last read by
  // nodes(z - 1), which precedes the barrier before layer(z).
  for (int z = zb; z < ze; ++z) {
    commit(z + 1);
    if (z + 2 <= ze) fetch(z + 2);
    lcur = lnext;
    mcur = mnext;
    okcur = oknext;
    if (z + 1 < ze) fetch_lm(z + 1, lnext, mnext, oknext);
    if (nact) {
      const long long node = (long long)(x0 + nlx) + (long long)Nx * ((long long)(y0 + nly) + (long long)Ny * z);
      tail_load<T>(D, g.Nn, kd_used, il, pp, Rp, node, tin);
    }
    __syncthreads();
    layer(z, true, lcur, mcur, okcur);
    __syncthreads();
    nodes(z);
  }
  block_sum<kPartStrideD>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < kPartStrideD; ++q) part[blockIdx.x * kPartStrideD + q] = acc[q];
}

// proj_P of the average relations on p (and on the quantities linear in p)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_weak_d(Geo g, DeltaBufs<T> D, WeakDev w, DevState* st) {
  if (st->done) return;
  const long long r = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (r >= w.m) return;
  const int c = w.comp[r];
  const int il = st->i_local, par = st->it & 1, acvp = (st->acv == 2);
  const int slot = (il + 1) % 3;
  const int ks = weak_size(w, r);
  double phys[8], wb[8];
  double sum = 0.0;
  for (int s = 0; s < ks; ++s) {
    const long long node = w.nodes[r * w.k + s];
    const int i = (int)(node % g.N[0]);
    const long long q = node / g.N[0];
    const int j = (int)(q % g.N[1]), k = (int)(q / g.N[1]);
    T p[3];
    double sn = 0.0, ms[6];
    node_eval_d<T, false>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
    const int xyz[3] = {i, j, k};
    wb[s] = (double)(1 << bcount(g, xyz));
    phys[s] = (double)p[c] / wb[s];
    sum += phys[s];
  }
  const double mean = sum / ks;
  double pn = 0.0;
  for (int s = 0; s < ks; ++s) {
    const long long e = c * g.Nn + w.nodes[r * w.k + s];
    const double pnew = (phys[s] - mean) * wb[s];
    pn += pnew * pnew;
    const T sh = (T)(mean * wb[s]);
    D.p[par][e] = (T)pnew;
    if (acvp && il >= 1) {
      D.R[par][e] -= sh;
      if (il >= 2) {
        D.dR[slot][e] -= sh;
        D.dY[slot][e] -= sh;
      }
    }
  }
  w.part[r] = pn;
  w.react[r] = -sum;
}

// Gram matrix of the R differences and their products with R_i (accelerating iterations)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram3(DeltaBufs<T> D, long long n3, DevState* st, double* __restrict__ gpart) {
  __shared__ double sh[9 * 16];
  if (st->done || !st->accel) return;
  const T* Ri = D.R[st->it & 1];
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    const double a0 = D.dR[0][e], a1 = D.dR[1][e], a2 = D.dR[2][e], r = Ri[e];
    acc[0] += a0 * a0; acc[1] += a0 * a1; acc[2] += a0 * a2;
    acc[3] += a1 * a1; acc[4] += a1 * a2; acc[5] += a2 * a2;
    acc[6] += a0 * r; acc[7] += a1 * r; acc[8] += a2 * r;
  }
  block_sum<9>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 9; ++q) gpart[blockIdx.x * 9 + q] = acc[q];
}

__global__ __launch_bounds__(kBlock) void k_alpha3(DevState* st, const double* __restrict__ gpart, int nblk) {
  __shared__ double sh[9 * 16];
  if (st->done || !st->accel) return;
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x)
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] += gpart[b * 9 + q];
  block_sum<9>(acc, sh);
  if (threadIdx.x != 0) return;
  double G[3][4] = {{acc[0], acc[1], acc[2], acc[6]}, {acc[1], acc[3], acc[4], acc[7]}, {acc[2], acc[4], acc[5], acc[8]}};
  const double tr = G[0][0] + G[1][1] + G[2][2];
  for (int a = 0; a < 3; ++a) G[a][a] += 1e-14 * tr / 3.0;
  bool ok = true;
  for (int col = 0; col < 3 && ok; ++col) {
    int piv = col;
    double best = fabs(G[col][col]);
    for (int r = col + 1; r < 3; ++r)
      if (fabs(G[r][col]) > best) {
        best = fabs(G[r][col]);
        piv = r;
      }
    if (!(best > 0.0)) {
      ok = false;
      break;
    }
    if (piv != col)
      for (int q = 0; q < 4; ++q) {
        const double t = G[col][q];
        G[col][q] = G[piv][q];
        G[piv][q] = t;
      }
    for (int r = col + 1; r < 3; ++r) {
      const double f = G[r][col] / G[col][col];
      for (int q = col; q < 4; ++q) G[r][q] -= f * G[col][q];
    }
  }
  double y[3] = {0, 0, 0};
  if (ok) {
    for (int r = 2; r >= 0; --r) {
      double s = G[r][3];
      for (int q = r + 1; q < 3; ++q) s -= G[r][q] * y[q];
      y[r] = s / G[r][r];
    }
    ok = isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]);
  }
  if (ok)
    for (int a = 0; a < 3; ++a) st->gamma[a] = y[a];
  st->accel_ok = ok ? 1 : 0;
}

// proj_U of the residual-form path on the FP64 displacement; the increment follows
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_d(Geo g, DeltaBufs<T> D, StrongDev s, WeakDev w, ContactDev ct,
                                                   DevState* st, int force) {
  if (!force && st->done) return;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  // strong DOFs
  if (e < s.m) {
    const long long idx = s.comp[e] * g.Nn + s.node[e];
    const double old = D.u[idx];
    D.u[idx] = s.val[e];
    D.delta[idx] = (T)((double)D.delta[idx] + (s.val[e] - old));
  }
  // average relations
  if (e < w.m) {
    const int c = w.comp[e];
    const int k = weak_size(w, e);
    double sum = 0.0;
    for (int q = 0; q < k; ++q) sum += D.u[c * g.Nn + w.nodes[e * w.k + q]];
    const double corr = w.val[e] - sum / k;
    for (int q = 0; q < k; ++q) {
      const long long idx = c * g.Nn + w.nodes[e * w.k + q];
      D.u[idx] += corr;
      D.delta[idx] = (T)((double)D.delta[idx] + corr);
    }
  }
  // contact nodes: radial projection onto the sphere
  if (ct.on && e < ct.nface && ct.C[e]) {
    int xyz[3];
    xyz[ct.axis] = ct.side ? g.n[ct.axis] : 0;
    xyz[ct.b1] = (int)(e % g.N[ct.b1]);
    xyz[ct.b2] = (int)(e / g.N[ct.b1]);
    const long long node = xyz[0] + (long long)g.N[0] * (xyz[1] + (long long)g.N[1] * xyz[2]);
    double d[3], r2 = 0.0;
    for (int c = 0; c < 3; ++c) {
      d[c] = xyz[c] + D.u[c * g.Nn + node] - ct.center[c];
      r2 += d[c] * d[c];
    }
    const double rr = sqrt(r2);
    for (int c = 0; c < 3; ++c) {
      const long long idx = c * g.Nn + node;
      const double nw = ct.center[c] + ct.radius * d[c] / rr - xyz[c];
      D.delta[idx] = (T)((double)D.delta[idx] + (nw - D.u[idx]));
      D.u[idx] = nw;
    }
  }
}

template <typename T>
__global__ void k_advance(DevState* st) {
  if (st->done) return;
  st->it += 1;
  st->i_local += 1;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_reactions_d(Geo g, DeltaBufs<T> D, StrongDev s, double* out) {
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= s.m) return;
  const long long node = s.node[e];
  const int i = (int)(node % g.N[0]);
  const long long q = node / g.N[0];
  const int j = (int)(q % g.N[1]), k = (int)(q / g.N[1]);
  T p[3];
  double sn = 0.0, ms[6];
  node_eval_d<T, false>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
  const int xyz[3] = {i, j, k};
  out[e] = -(double)p[s.comp[e]] / (double)(1 << bcount(g, xyz));
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
static inline int grid_for(long long n, int cap) {
  long long b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  return (int)(b < cap ? b : cap);
}

template <typename T>
void launch_residual(const Geo& g, const Bufs<T>& B, const ContactDev& ct, DevState* st, double* part, int nblk,
                     int force, int write_p, hipStream_t s) {
  hipLaunchKernelGGL(k_residual<T>, dim3(nblk), dim3(kBlock), 0, s, g, B, ct, st, part, force, write_p);
}

template <typename T>
void launch_weak(const Geo& g, const Bufs<T>& B, const WeakDev& w, DevState* st, int force, hipStream_t s) {
  if (w.m == 0) return;
  hipLaunchKernelGGL(k_weak<T>, dim3(grid_for(w.m, 1 << 30)), dim3(kBlock), 0, s, g, B, w, st, force);
}

void launch_control(DevState* st, const double* part, int nblk, const double* wpart, long long nweak,
                    const ContactDev& ct, int pstride, hipStream_t s) {
  hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, s, st, part, nblk, wpart, nweak, ct, pstride);
}

template <typename T>
void launch_anderson(const Bufs<T>& B, long long n3, DevState* st, double* gpart, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_anderson_r<T>, dim3(nblk), dim3(kBlock), 0, s, B, n3, st, gpart);
  hipLaunchKernelGGL(k_alpha, dim3(1), dim3(kBlock), 0, s, st, gpart, nblk);
}

template <typename T>
size_t dtt_smem(const AxisPlan& ap) {
  return sizeof(cplx<T>) * (size_t)ap.L * (ap.n + 1) + sizeof(T) * (size_t)ap.L * (ap.N + 1);
}

template <typename T, int NF, int NTH, int TY = -1>
static void launch_dtt2(const DttArgs<T>& a, hipStream_t s) {
  using S = DttShape<NF, NTH>;
  const int Nx = a.g.N[0], Ny = a.g.N[1], Nz = a.g.N[2];
  dim3 grid;
  if (a.axis == 0) grid = dim3((Ny + S::LB - 1) / S::LB, Nz, 3);
  else if (a.axis == 1) grid = dim3((Nx + S::LB - 1) / S::LB, Nz, 3);
  else grid = dim3((Nx + S::LB - 1) / S::LB, Ny, 3);
  const size_t sm = sizeof(cplx<T>) * ((size_t)S::LB * S::CS + 2 * NF + 1);
  hipLaunchKernelGGL((k_dtt2<T, NF, NTH, TY>), grid, dim3(S::NT), sm, s, a);
}

// Passes of the long lines with one transform type for all components get a kernel with
// that type fixed at compile time (no per-element type dispatch).
template <typename T, int NF, int NTH>
static void launch_dtt2_typed(const DttArgs<T>& a, hipStream_t s) {
  if constexpr (NF == 128 || NF == 256) {
    const int t0 = a.types[0];
    if (a.types[1] == t0 && a.types[2] == t0) {
      switch (t0) {
        case T_DCT1: launch_dtt2<T, NF, NTH, T_DCT1>(a, s); return;
        case T_DCT3: launch_dtt2<T, NF, NTH, T_DCT3>(a, s); return;
        case T_DST1: launch_dtt2<T, NF, NTH, T_DST1>(a, s); return;
        case T_DST3: launch_dtt2<T, NF, NTH, T_DST3>(a, s); return;
        default: break;
      }
    }
  }
  launch_dtt2<T, NF, NTH>(a, s);
}

template <typename T>
void launch_dtt(const DttArgs<T>& a, int ept, hipStream_t s) {
  if (!a.g.periodic[a.axis] && !a.generic) {
    // block size chosen by the host autotuner (a.nt): FP64 128 or 256 threads, FP32 256 or 512
    constexpr int NLO = sizeof(T) == 8 ? 128 : 256;
    constexpr int NHI = sizeof(T) == 8 ? 256 : 512;
    const bool hi = a.nt >= NHI;
#define FFTC_DTT_CASE(L)                                   \
  case L:                                                  \
    if (hi) launch_dtt2_typed<T, L, NHI>(a, s);            \
    else launch_dtt2_typed<T, L, NLO>(a, s);               \
    return;
    switch (a.ap.n) {
      FFTC_DTT_CASE(16)
      FFTC_DTT_CASE(32)
      FFTC_DTT_CASE(48)
      FFTC_DTT_CASE(64)
      FFTC_DTT_CASE(96)
      FFTC_DTT_CASE(128)
      FFTC_DTT_CASE(256)
      default: break;
    }
#undef FFTC_DTT_CASE
  }
  const int Nx = a.g.N[0], Ny = a.g.N[1], Nz = a.g.N[2];
  const long long nlines = a.axis == 0 ? (long long)Ny * Nz : a.axis == 1 ? (long long)Nx * Nz : (long long)Nx * Ny;
  const long long nb = (nlines + a.ap.L - 1) / a.ap.L;
  const size_t sm = dtt_smem<T>(a.ap);
  if (dtt_ept(ept, a.ap) <= 8)
    hipLaunchKernelGGL((k_dtt<T, 8>), dim3((unsigned)nb, 3), dim3(kBlock), sm, s, a);
  else
    hipLaunchKernelGGL((k_dtt<T, 16>), dim3((unsigned)nb, 3), dim3(kBlock), sm, s, a);
}

template <typename T>
void launch_proj(const Geo& g, T* u, const WeakDev& w, const ContactDev& ct, const StrongDev& sd, DevState* st,
                 int advance, int force, hipStream_t s) {
  if (w.m > 0) hipLaunchKernelGGL(k_proj_weak<T>, dim3(grid_for(w.m, 1 << 30)), dim3(kBlock), 0, s, g, u, w, st, force);
  if (ct.on)
    hipLaunchKernelGGL(k_proj_contact<T>, dim3(grid_for(ct.nface, 1 << 30)), dim3(kBlock), 0, s, g, u, ct, st, force);
  if (force) {
    if (sd.m > 0) hipLaunchKernelGGL(k_strong_scatter<T>, dim3(grid_for(sd.m, 1024)), dim3(kBlock), 0, s, g, u, sd);
  } else {
    hipLaunchKernelGGL(k_finish<T>, dim3(grid_for(sd.m, 1024)), dim3(kBlock), 0, s, g, u, sd, st, advance);
  }
}

template <typename T>
void launch_flags_combine(const Bufs<T>& B, long long n3, DevState* st, int which, hipStream_t s) {
  if (which == 0) hipLaunchKernelGGL(k_flags_u, dim3(1), dim3(1), 0, s, st);
  else hipLaunchKernelGGL(k_combine_u<T>, dim3(grid_for(n3, 2048)), dim3(kBlock), 0, s, B, n3, st);
}

template <typename T>
void launch_contact_force(const Geo& g, const T* u, const ContactDev& ct, double* out, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_force<T>, dim3(nblk), dim3(kBlock), 0, s, g, u, ct, out);
}

TileGrid residual_tiles(const Geo& g);

template <typename T>
int launch_delta_residual(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, DevState* st, double* part,
                          int nblk, hipStream_t s) {
  const TileGrid tg = residual_tiles(g);
  if (tg.tx > 0) {
    nblk = tg.tx * tg.ty * tg.nseg;
    hipLaunchKernelGGL(k_residual_dt<T>, dim3(nblk), dim3(256), 0, s, g, D, ct, st, part, tg);
  } else {
    hipLaunchKernelGGL(k_residual_d<T>, dim3(nblk), dim3(kBlock), 0, s, g, D, ct, st, part);
  }
  return nblk;
}

template <typename T>
void launch_delta_control(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, const WeakDev& w, DevState* st,
                          const double* part, const double* wpart, int nblk, hipStream_t s) {
  if (w.m > 0) hipLaunchKernelGGL(k_weak_d<T>, dim3(grid_for(w.m, 1 << 30)), dim3(kBlock), 0, s, g, D, w, st);
  hipLaunchKernelGGL(k_control, dim3(1), dim3(kBlock), 0, s, st, part, nblk, wpart, w.m, ct, kPartStrideD);
}

// Blocks of the tiled residual pass resident on the current device at once (blocks per CU
// at the kernel's register and LDS use, times the CU count), queried once per device.
static int residual_resident() {
  static std::atomic<int> cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 512;
  int r = cache[dev].load(std::memory_order_relaxed);
  if (!r) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_residual_dt<float>, 256, 0) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    r = per_cu * cus;
    cache[dev].store(r, std::memory_order_relaxed);   // every thread computes the same value
  }
  return r;
}

// Tile grid of the tiled residual pass: tiles of kTX x kTY node columns, z split into
// segments, at most 2048 blocks (the partial-sum rows); tx = 0 when the node plane alone
// needs more tiles than that.  A block marches its segment's planes plus two planes of
// prologue, and the blocks run in rounds of the resident count, so the split taken is the
// one with the fewest (rounds x planes per block); ties go to fewer segments.
TileGrid residual_tiles(const Geo& g) {
  TileGrid t{0, 0, 0, 0};
  const int tx = (g.N[0] + kTX - 1) / kTX, ty = (g.N[1] + kTY - 1) / kTY;
  if ((long long)tx * ty > 2048) return t;
  const int Nz = g.N[2];
  const int maxseg = std::max(1, std::min(Nz, 2048 / (tx * ty)));
  const long long resident = residual_resident();
  long long best = -1;
  int bseg = Nz;
  for (int ns = 1; ns <= maxseg; ++ns) {
    const int seg = (Nz + ns - 1) / ns;
    const long long blocks = (long long)tx * ty * ((Nz + seg - 1) / seg);
    const long long cost = (blocks + resident - 1) / resident * (seg + 2);
    if (best < 0 || cost < best) {
      best = cost;
      bseg = seg;
    }
  }
  t.tx = tx;
  t.ty = ty;
  t.seg = bseg;
  t.nseg = (Nz + bseg - 1) / bseg;
  return t;
}

template <typename T>
void launch_delta_anderson(const DeltaBufs<T>& D, long long n3, DevState* st, double* gpart, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_gram3<T>, dim3(nblk), dim3(kBlock), 0, s, D, n3, st, gpart);
  hipLaunchKernelGGL(k_alpha3, dim3(1), dim3(kBlock), 0, s, st, gpart, nblk);
}

template <typename T>
void launch_delta_proj(const Geo& g, const DeltaBufs<T>& D, const StrongDev& sd, const WeakDev& w,
                       const ContactDev& ct, DevState* st, int force, int advance, hipStream_t s) {
  long long m = sd.m > w.m ? sd.m : w.m;
  if (ct.on && ct.nface > m) m = ct.nface;
  if (m > 0) hipLaunchKernelGGL(k_proj_d<T>, dim3(grid_for(m, 1 << 30)), dim3(kBlock), 0, s, g, D, sd, w, ct, st, force);
  if (advance) hipLaunchKernelGGL(k_advance<T>, dim3(1), dim3(1), 0, s, st);
}

template <typename T>
void launch_reactions_d(const Geo& g, const DeltaBufs<T>& D, const StrongDev& sd, double* out, hipStream_t s) {
  if (sd.m == 0) return;
  hipLaunchKernelGGL(k_reactions_d<T>, dim3(grid_for(sd.m, 1 << 30)), dim3(kBlock), 0, s, g, D, sd, out);
}

template <typename T>
void launch_weak_d_stage(const Geo& g, const DeltaBufs<T>& D, const WeakDev& w, DevState* st, hipStream_t s) {
  if (w.m > 0) hipLaunchKernelGGL(k_weak_d<T>, dim3(grid_for(w.m, 1 << 30)), dim3(kBlock), 0, s, g, D, w, st);
}

template <typename T>
void launch_contact_init(const Geo& g, const T* u, const ContactDev& ct, hipStream_t s) {
  hipLaunchKernelGGL(k_contact_init<T>, dim3(grid_for(ct.nface, 1 << 30)), dim3(kBlock), 0, s, g, u, ct);
}

template <typename T>
void launch_reactions(const Geo& g, const Bufs<T>& B, const StrongDev& sd, double* out, hipStream_t s) {
  if (sd.m == 0) return;
  hipLaunchKernelGGL(k_reactions<T>, dim3(grid_for(sd.m, 1 << 30)), dim3(kBlock), 0, s, g, B, sd, out);
}

template <typename A, typename Bt>
void launch_convert(const A* in, Bt* out, long long n, hipStream_t s) {
  hipLaunchKernelGGL((k_convert<A, Bt>), dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, in, out, n);
}

template <typename T>
void launch_zero_amask(const Geo& g, T* u, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_amask<T>, dim3(grid_for(g.Nn, 8192)), dim3(kBlock), 0, s, g, u);
}

void launch_extend(DevState* st, int iters, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_extend, dim3(1), dim3(1), 0, s, st, iters, tol);
}

void launch_check_stiffness(const double* lam, const double* mu, long long nv, double* out, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_check_stiffness, dim3(nblk), dim3(kBlock), 0, s, lam, mu, nv, out);
}

#define FFTC_INST(T)                                                                                              \
  template void launch_residual<T>(const Geo&, const Bufs<T>&, const ContactDev&, DevState*, double*, int, int,   \
                                   int, hipStream_t);                                                                  \
  template void launch_weak<T>(const Geo&, const Bufs<T>&, const WeakDev&, DevState*, int, hipStream_t);         \
  template void launch_anderson<T>(const Bufs<T>&, long long, DevState*, double*, int, hipStream_t);             \
  template void launch_dtt<T>(const DttArgs<T>&, int, hipStream_t);                                                \
  template size_t dtt_smem<T>(const AxisPlan&);                                                                    \
  template void launch_proj<T>(const Geo&, T*, const WeakDev&, const ContactDev&, const StrongDev&, DevState*,   \
                               int, int, hipStream_t);                                                            \
  template void launch_contact_init<T>(const Geo&, const T*, const ContactDev&, hipStream_t);                     \
  template void launch_contact_force<T>(const Geo&, const T*, const ContactDev&, double*, int, hipStream_t);     \
  template void launch_reactions<T>(const Geo&, const Bufs<T>&, const StrongDev&, double*, hipStream_t);         \
  template void launch_zero_amask<T>(const Geo&, T*, hipStream_t);                                                 \
  template void launch_flags_combine<T>(const Bufs<T>&, long long, DevState*, int, hipStream_t);

FFTC_INST(double)
FFTC_INST(float)
template void launch_convert<double, double>(const double*, double*, long long, hipStream_t);
template void launch_convert<double, float>(const double*, float*, long long, hipStream_t);
template void launch_convert<float, double>(const float*, double*, long long, hipStream_t);
template int launch_delta_residual<float>(const Geo&, const DeltaBufs<float>&, const ContactDev&, DevState*, double*,
                                          int, hipStream_t);
template void launch_delta_control<float>(const Geo&, const DeltaBufs<float>&, const ContactDev&, const WeakDev&,
                                          DevState*, const double*, const double*, int, hipStream_t);
template void launch_delta_anderson<float>(const DeltaBufs<float>&, long long, DevState*, double*, int, hipStream_t);
template void launch_delta_proj<float>(const Geo&, const DeltaBufs<float>&, const StrongDev&, const WeakDev&,
                                       const ContactDev&, DevState*, int, int, hipStream_t);
template void launch_reactions_d<float>(const Geo&, const DeltaBufs<float>&, const StrongDev&, double*, hipStream_t);

}  // namespace fftc
