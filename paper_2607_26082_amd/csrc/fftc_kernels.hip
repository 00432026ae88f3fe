// HIP kernels of libfftc for CDNA4 (gfx950), 64-wide wavefronts.
//
// One fixed-point iteration (paper Algorithm 1 / Algorithm 2, eq 3 and eq 9):
//   k_residual   stress at both TETRA2 integration points of the 8 voxels around
//                each node, nodal divergence (boundary weight 2^b), proj_P for strong
//                DOFs and contact nodes, reference-medium term, FP64 partial norms
//   k_weak       proj_P of the relations on several nodes (eq 14, eq 17)
//   k_control    equilibrium test (eq 5), contact active-set update, Anderson flags
//   k_anderson_r / k_alpha   residual store, FP64 Gram matrix, constrained LS
//   (the per-axis DTT passes, Tables 2-3, are in fftc_dtt_kernels.h; the residual-form
//    iteration of the FP32 path is in fftc_residual.hip)
//   k_proj_*     proj_U: relations (eq 11, eq 15), contact radial projection, strong DOFs
#include "fftc_internal.h"
#include "fftc_launch.h"
#include "fftc_common.h"

#include <math.h>
#include <algorithm>

namespace fftc {


// ---------------------------------------------------------------------------
// Residual of one node: p = 2^b div_D(C : grad^s_D u) summed over in-cell voxels,
// and K0 u = -2^b div_D(R0 : grad_D u) from the closed-form Paux stencil applied to
// the symmetric extension of u.  Optionally the stress norm and mean-stress sums of
// the tetrahedra owned by this node (T1 of voxel n, T2 of voxel n - e_x).
// ---------------------------------------------------------------------------
template <typename T, bool SIG, bool FS = false>
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
    // nodal force: (1/2 IP weight) * B_node^T sigma with B_node = (2a - 1)/2
    const T bx = T(ax ? 0.25 : -0.25), by = T(ay ? 0.25 : -0.25), bz = T(az ? 0.25 : -0.25);
    if constexpr (FS) {
      // finite strain: the non-symmetric PK1 stress, nodal force row r = B . P[r][:]
      T P[3][3];
      svk_pk1<T>(G, l, m, P);
#pragma unroll
      for (int r = 0; r < 3; ++r) F[r] += bx * P[r][0] + by * P[r][1] + bz * P[r][2];
      if (SIG && (a == 0 || a == 1)) {
        double q = 0.0;
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < 3; ++c) q += (double)P[r][c] * (double)P[r][c];
        sn += 0.5 * q;
        ms[0] += 0.5 * (double)P[0][0]; ms[1] += 0.5 * (double)P[1][1]; ms[2] += 0.5 * (double)P[2][2];
        ms[3] += 0.5 * (double)P[1][2]; ms[4] += 0.5 * (double)P[0][2]; ms[5] += 0.5 * (double)P[0][1];
      }
      continue;
    }
    const T tr = G[0][0] + G[1][1] + G[2][2];
    const T s00 = l * tr + T(2) * m * G[0][0];
    const T s11 = l * tr + T(2) * m * G[1][1];
    const T s22 = l * tr + T(2) * m * G[2][2];
    const T s01 = m * (G[0][1] + G[1][0]);
    const T s02 = m * (G[0][2] + G[2][0]);
    const T s12 = m * (G[1][2] + G[2][1]);
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

// HEX1 (Section 3.1.2): the gradient of the trilinear interpolant at the centre of each of
// the 8 voxels around the node, B_corner = (2a - 1, 2b - 1, 2c - 1) / 4, one integration point
// of weight 1; p = -2^b sum B_node^T sigma, and the reference term K0 u = 2^b sum B_node^T
// sigma0 with sigma0 = R0 : G of the Paux or the isotropic medium, both over in-cell voxels.
template <typename T, bool SIG, bool FS = false>
__device__ __forceinline__ void node_eval_hex(const Geo& g, const T* __restrict__ u, const T* __restrict__ lam,
                                              const T* __restrict__ mu, int i, int j, int k, T p[3], T k0[3],
                                              double& sn, double ms[6]) {
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  const int xs[3] = {mirror_coord(g, i - 1, 0), i, mirror_coord(g, i + 1, 0)};
  const int ys[3] = {mirror_coord(g, j - 1, 1), j, mirror_coord(g, j + 1, 1)};
  const int zs[3] = {mirror_coord(g, k - 1, 2), k, mirror_coord(g, k + 1, 2)};
  T F[3] = {T(0), T(0), T(0)}, F0[3] = {T(0), T(0), T(0)};
  const T l0 = (T)g.lam0, m0 = (T)g.mu0;
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
      for (int q = 0; q < 3; ++q) G[r][q] = T(0);
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
      // corner cc of the voxel sits at node offset (cx - ax, cy - ay, cz - az)
      const long long idx = (long long)xs[cx - ax + 1] + (long long)Nx * ((long long)ys[cy - ay + 1] + (long long)Ny * zs[cz - az + 1]);
      const T bx = T(cx ? 0.25 : -0.25), by = T(cy ? 0.25 : -0.25), bz = T(cz ? 0.25 : -0.25);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T v = u[r * Nn + idx];
        G[r][0] += bx * v;
        G[r][1] += by * v;
        G[r][2] += bz * v;
      }
    }
    T P[3][3], P0[3][3];
    if constexpr (FS) {
      svk_pk1<T>(G, l, m, P);
    } else {
      const T tr = G[0][0] + G[1][1] + G[2][2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) P[r][q] = m * (G[r][q] + G[q][r]) + (r == q ? l * tr : T(0));
    }
    if (g.iso) {
      const T tr = G[0][0] + G[1][1] + G[2][2];
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) P0[r][q] = m0 * (G[r][q] + G[q][r]) + (r == q ? l0 * tr : T(0));
    } else {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 3; ++q) P0[r][q] = T(2) * m0 * G[r][q] + (r == q ? l0 * G[r][r] : T(0));
    }
    const T bx = T(ax ? 0.25 : -0.25), by = T(ay ? 0.25 : -0.25), bz = T(az ? 0.25 : -0.25);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      F[r] += bx * P[r][0] + by * P[r][1] + bz * P[r][2];
      F0[r] += bx * P0[r][0] + by * P0[r][1] + bz * P0[r][2];
    }
    if (SIG && a == 0) {   // the voxel whose corner 000 is this node
      double q = 0.0;
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) q += (double)P[r][c] * (double)P[r][c];
      sn += q;
      ms[0] += (double)P[0][0]; ms[1] += (double)P[1][1]; ms[2] += (double)P[2][2];
      ms[3] += (double)P[1][2]; ms[4] += (double)P[0][2]; ms[5] += (double)P[0][1];
    }
  }
  const int xyz[3] = {i, j, k};
  const T w2b = T(1 << bcount(g, xyz));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const bool A = is_antisym(g, c, xyz);
    p[c] = A ? T(0) : -w2b * F[c];
    k0[c] = A ? T(0) : w2b * F0[c];
  }
}

// node evaluation of the scheme in use (runtime dispatch for the kernels off the hot path)
template <typename T, bool SIG>
__device__ __forceinline__ void node_eval_any(const Geo& g, const T* __restrict__ u, const T* __restrict__ lam,
                                              const T* __restrict__ mu, int i, int j, int k, T p[3], T k0[3],
                                              double& sn, double ms[6]) {
  if (g.hex) {
    if (g.fs) node_eval_hex<T, SIG, true>(g, u, lam, mu, i, j, k, p, k0, sn, ms);
    else node_eval_hex<T, SIG, false>(g, u, lam, mu, i, j, k, p, k0, sn, ms);
  } else {
    if (g.fs) node_eval<T, SIG, true>(g, u, lam, mu, i, j, k, p, k0, sn, ms);
    else node_eval<T, SIG, false>(g, u, lam, mu, i, j, k, p, k0, sn, ms);
  }
}

// ---------------------------------------------------------------------------
// Residual pass
// ---------------------------------------------------------------------------
template <typename T, bool FS, bool HEX>
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
    if constexpr (HEX) node_eval_hex<T, true, FS>(g, B.u, B.lam, B.mu, i, j, k, p, k0, sn, ms);
    else node_eval<T, true, FS>(g, B.u, B.lam, B.mu, i, j, k, p, k0, sn, ms);
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
    for (int q = 0; q < kPartStride; ++q) part[q * kPartRows + blockIdx.x] = acc[q];
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
  node_eval_any<T, false>(g, B.u, B.lam, B.mu, i, j, k, p, k0, sn, ms);
  const int xyz[3] = {i, j, k};
  b = bcount(g, xyz);
}

// proj_P of the relations on several nodes on the physical residual q = 2^-b p (eq 14,
// eq 17): f = (wa . q) / (wa . wb), q -= wb f over the support.  One wavefront per relation,
// one lane per support node; the residual of every support node is formed again from u.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_weak(Geo g, Bufs<T> B, WeakDev w, DevState* st, int force) {
  if (!force && st->done) return;
  const long long r = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  if (r >= w.m) return;   // uniform over the wavefront
  const int lane = threadIdx.x & 63;
  const long long o0 = w.off[r];
  const bool act = lane < w.off[r + 1] - o0;
  const int c = w.comp[r];
  long long node = 0;
  double wa = 0.0, wb = 0.0, q = 0.0, scale = 1.0;
  if (act) {
    node = w.nodes[o0 + lane];
    wa = w.wa[o0 + lane];
    wb = w.wb[o0 + lane];
    T p[3];
    int b;
    node_p<T>(g, B, node, p, b);
    scale = (double)(1 << b);
    q = (double)p[c] / scale;
  }
  const double num = wave_sum(wa * q), den = wave_sum(wa * wb), sb = wave_sum(wb);
  const double f = num / den;
  const double pnew = (q - wb * f) * scale;
  const double pn = wave_sum(act ? pnew * pnew : 0.0);
  if (act) {
    const long long e = c * g.Nn + node;
    B.X[e] = (T)((double)B.X[e] - wb * f * scale);
  }
  if (lane == 0) {
    w.part[r] = pn;
    w.react[r] = -f * sb;
  }
}

// ---------------------------------------------------------------------------
// Control: equilibrium test, contact update, Anderson flags (one block)
// ---------------------------------------------------------------------------
// Face-node byte arrays (active set C, the V_gap / V_react flags V) are walked 16 bytes per
// lane, kFaceU chunks in flight per thread; the bytes past the last whole chunk one at a time.
// The workspace carve aligns these arrays to 256 bytes; misaligned ones are walked bytewise.
constexpr int kFaceU = 4;

__device__ __forceinline__ long long face_chunks(const ContactDev& ct, const uint8_t* a, const uint8_t* b) {
  return (((uintptr_t)a | (uintptr_t)b) & 15) ? 0 : ct.nface >> 4;
}

// chunk c of a byte array, zero past the last whole chunk
__device__ __forceinline__ uint4 face_chunk(const uint8_t* p, long long c, long long nch) {
  return c < nch ? reinterpret_cast<const uint4*>(p)[c] : make_uint4(0, 0, 0, 0);
}

// Algorithm 2's active-set update C <- (C u V_gap) \ V_react on four face nodes at once
// (one byte each: C in {0, 1}, V bit 0 = in V_gap, bit 1 = in V_react)
__device__ __forceinline__ unsigned active_bytes(unsigned c, unsigned v) {
  unsigned r = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const unsigned cj = (c >> (8 * j)) & 0xffu, vj = (v >> (8 * j)) & 0xffu;
    r |= (unsigned)((cj || (vj & 1u)) && !(vj & 2u)) << (8 * j);
  }
  return r;
}

// FP32 form's stagnation test: iterations without a halving of the residual, below this cap
constexpr int kStallWindow = 100;
constexpr double kStallCap = 1e-2;

__global__ __launch_bounds__(kBlock) void k_control(DevState* st, const double* __restrict__ part, int nblk,
                                                    const double* __restrict__ wpart, long long nweak, ContactDev ct,
                                                    int pstride) {
  __shared__ double sh[kPartStrideD * 16];
  __shared__ int flags[4];
  __shared__ int decide, s_done, changed;
  if (st->done) return;
  // the state this step reads, loaded once up front (independent loads; reading the fields
  // back after the stores and barriers below made a chain of dependent round trips)
  const int vpar = st->vpar, it = st->it, max_iter = st->max_iter, have_prev = st->have_prev;
  const int acv = st->acv, period = st->period, i_local0 = st->i_local, fine0 = st->fine;
  const double tol = st->tol, gate = st->gate, refine_below = st->refine_below;
  const double best_res = st->best_res;
  const int best_it = st->best_it;
  // the FP32 form's incremental pass forms no stress norm: the last full pass's is kept, and
  // such a pass never ends the solve (the exit test is taken on a pass from u)
  const bool inc = res_pass(st) == PASS_INC;
  const double sn_kept = st->snorm2;
  double acc[kPartStrideD];
#pragma unroll
  for (int q = 0; q < kPartStrideD; ++q) acc[q] = 0.0;
  if (pstride == kPartStrideD) sum_cols<kPartStrideD>(part, kPartRows, nblk, acc);
  else sum_cols<kPartStride>(part, kPartRows, nblk, acc);
  {
    double w0[1] = {acc[0]};
    sum_cols<1>(wpart, 0, nweak, w0);
    acc[0] = w0[0];
  }
  // contact: compare V with the previous iteration, test emptiness (read before the block
  // sum so that these loads overlap it)
  int differ = 0, nonempty = 0;
  if (ct.on) {
    const uint8_t* Vc = ct.V[vpar];
    const uint8_t* Vp = ct.V[vpar ^ 1];
    const long long nch = face_chunks(ct, Vc, Vp);
    for (long long c0 = threadIdx.x; c0 < nch; c0 += kFaceU * blockDim.x) {
      uint4 a[kFaceU], b[kFaceU];
#pragma unroll
      for (int k = 0; k < kFaceU; ++k) {
        a[k] = face_chunk(Vc, c0 + k * blockDim.x, nch);
        b[k] = face_chunk(Vp, c0 + k * blockDim.x, nch);
      }
#pragma unroll
      for (int k = 0; k < kFaceU; ++k) {
        nonempty |= (a[k].x | a[k].y | a[k].z | a[k].w) != 0;
        differ |= ((a[k].x ^ b[k].x) | (a[k].y ^ b[k].y) | (a[k].z ^ b[k].z) | (a[k].w ^ b[k].w)) != 0;
      }
    }
    for (long long f = 16 * nch + threadIdx.x; f < ct.nface; f += blockDim.x) {
      const uint8_t v = Vc[f];
      nonempty |= (v != 0);
      differ |= (v != Vp[f]);
    }
  }
  if (threadIdx.x == 0) flags[0] = flags[1] = 0;
  block_sum<kPartStrideD>(acc, sh);   // ends with a barrier
  if (ct.on) {
    if (differ) atomicOr(&flags[0], 1);
    if (nonempty) atomicOr(&flags[1], 1);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double pn = acc[0], sn = inc ? sn_kept : acc[1];
    st->pnorm2 = pn;
    st->snorm2 = sn;
    for (int q = 0; q < 6; ++q) st->ms[q] = acc[2 + q];
    if (pstride > kPartStride)
      for (int q = 0; q < 6; ++q) st->sing[q] = acc[8 + q];
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
    } else if (res < tol && !nonempty && !inc) {
      st->status = ST_CONVERGED;
      s_done = 1;
    } else if (it >= max_iter) {
      st->status = ST_NOCONV;
      s_done = 1;
    } else {
      if (ct.on && have_prev && !flags[0] && nonempty && res < gate) decide = 1;
      // FP32 form: below the refinement threshold the residual pass forms its stresses in
      // FP64 from the next iteration on, and so it does once the residual, below 1e-2, has not
      // halved in 100 iterations: on high-contrast cells the FP32 stresses hold the residual
      // above the threshold (measured: a contrast-90 indentation cell at 1.1e-5 after 4000
      // iterations, 703 with the FP64 stresses from 1e-3 on).  The Anderson history is kept:
      // its unaccelerated restart iterations amplify the error on cells where the plain map
      // diverges (measured on a homogeneous block: 1e-5 -> 0.26 within four iterations).
      if (refine_below > 0.0 && !fine0) {
        int bit = best_it;
        if (res < 0.5 * best_res) {
          st->best_res = res;
          st->best_it = bit = it;
        }
        if (res < refine_below || (res < kStallCap && it - bit > kStallWindow)) st->fine = 1;
      }
      // an incremental pass below the tolerance: the remaining passes are from u
      if (inc && res < tol) st->inc_k = 0;
    }
    if (s_done) st->done = 1;
  }
  __syncthreads();
  if (s_done) return;
  int i_local = i_local0;
  if (ct.on) {
    if (decide) {
      int ch = 0;
      const uint8_t* Vc = ct.V[vpar];
      const long long nch = face_chunks(ct, Vc, ct.C);
      for (long long c0 = threadIdx.x; c0 < nch; c0 += kFaceU * blockDim.x) {
        uint4 v[kFaceU], o[kFaceU];
#pragma unroll
        for (int k = 0; k < kFaceU; ++k) {
          v[k] = face_chunk(Vc, c0 + k * blockDim.x, nch);
          o[k] = face_chunk(ct.C, c0 + k * blockDim.x, nch);
        }
#pragma unroll
        for (int k = 0; k < kFaceU; ++k) {
          const uint4 nw = make_uint4(active_bytes(o[k].x, v[k].x), active_bytes(o[k].y, v[k].y),
                                      active_bytes(o[k].z, v[k].z), active_bytes(o[k].w, v[k].w));
          if (nw.x != o[k].x || nw.y != o[k].y || nw.z != o[k].z || nw.w != o[k].w) {
            reinterpret_cast<uint4*>(ct.C)[c0 + k * blockDim.x] = nw;   // only chunks < nch differ
            ch = 1;
          }
        }
      }
      for (long long f = 16 * nch + threadIdx.x; f < ct.nface; f += blockDim.x) {
        const uint8_t v = Vc[f];
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
          i_local = 0;
          st->i_local = 0;
          st->restarts += 1;
        }
      }
      st->have_prev = 1;
      st->vpar = vpar ^ 1;
    }
  }
  if (threadIdx.x == 0) {
    st->store_r = (acv == 2) && (i_local > 0);
    st->accel = (acv == 2) && (i_local >= 4) && (i_local % period == 0);
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
    for (int q = 0; q < 10; ++q) gpart[q * kPartRows + blockIdx.x] = acc[q];
}

// alpha = argmin |sum a_k R_k|, sum a_k = 1, from the regularised FP64 Gram matrix.
__global__ __launch_bounds__(kBlock) void k_alpha(DevState* st, const double* __restrict__ gpart, int nblk) {
  __shared__ double sh[10 * 16];
  if (st->done || !st->accel) return;
  double acc[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) acc[q] = 0.0;
  sum_cols<10>(gpart, kPartRows, nblk, acc);
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
  double y[4];
  bool ok = solve_pivoted<4>(G, y);
  if (ok) {
    const double sy = y[0] + y[1] + y[2] + y[3];
    ok = isfinite(sy) && sy != 0.0 && isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]) && isfinite(y[3]);
    if (ok)
      for (int a = 0; a < 4; ++a) st->alpha[a] = y[a] / sy;
  }
  st->accel_ok = ok ? 1 : 0;
}


// ---------------------------------------------------------------------------
// Isotropic reference medium on a cell periodic on every axis (eq 4, Section 3.2.4).  After
// the forward half-complex transforms of the three axes, storage index m of an axis of n
// voxels holds the cosine part of frequency m (2m <= n) or the sine part of frequency n - m
// (as the imaginary part of the DFT).  Per frequency class (k1, k2, k3), 0 <= k_J <= n_J / 2,
// the up to eight cosine/sine combinations of each component give the complex coefficients
// at (theta1, +-theta2, +-theta3); each is solved with the HEX1 symbol
// M = mu0 |d|^2 I + (lam0 + mu0) d d^T, d_J = 2 sin(theta_J / 2) prod_{K != J} cos(theta_K / 2)
// (real, so its inverse acts on real and imaginary parts alike; 0 where |d| = 0: theta = 0
// and the hourglass lines), and the combinations are formed back.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void ipow(int n, double& re, double& im) {   // i^n
  const int r = n & 3;
  re = r == 0 ? 1.0 : (r == 2 ? -1.0 : 0.0);
  im = r == 1 ? 1.0 : (r == 3 ? -1.0 : 0.0);
}

__global__ __launch_bounds__(kBlock) void k_green_iso(Geo g, double* buf, DevState* st, int force) {
  if (!force && st->done) return;
  const int nn[3] = {g.n[0], g.n[1], g.n[2]};
  const int h1 = nn[0] / 2 + 1, h2 = nn[1] / 2 + 1, h3 = nn[2] / 2 + 1;
  const long long cls = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (cls >= (long long)h1 * h2 * h3) return;
  const int kk[3] = {(int)(cls % h1), (int)((cls / h1) % h2), (int)(cls / ((long long)h1 * h2))};
  int np[3], idx[3][2];
#pragma unroll
  for (int J = 0; J < 3; ++J) {
    np[J] = (kk[J] == 0 || 2 * kk[J] == nn[J]) ? 1 : 2;
    idx[J][0] = kk[J];
    idx[J][1] = nn[J] - kk[J];
  }
  const long long Nn = g.Nn;
  const int Nx = g.N[0], Ny = g.N[1];
  double Tv[3][2][2][2], Tu[3][2][2][2];
  for (int c = 0; c < 3; ++c)
    for (int a1 = 0; a1 < 2; ++a1)
      for (int a2 = 0; a2 < 2; ++a2)
        for (int a3 = 0; a3 < 2; ++a3) {
          Tu[c][a1][a2][a3] = 0.0;
          Tv[c][a1][a2][a3] = 0.0;
          if (a1 < np[0] && a2 < np[1] && a3 < np[2])
            Tv[c][a1][a2][a3] = buf[c * Nn + idx[0][a1] + (long long)Nx * (idx[1][a2] + (long long)Ny * idx[2][a3])];
        }
  const double bcoef = (g.lam0 + g.mu0) / (g.lam0 + 2.0 * g.mu0);
  const double two_pi = 6.283185307179586476925286766559;
  for (int s2i = 0; s2i < np[1]; ++s2i)
    for (int s3i = 0; s3i < np[2]; ++s3i) {
      const double sg[3] = {1.0, s2i ? -1.0 : 1.0, s3i ? -1.0 : 1.0};
      double Xr[3], Xi[3];
      for (int c = 0; c < 3; ++c) {
        Xr[c] = Xi[c] = 0.0;
        for (int a1 = 0; a1 < np[0]; ++a1)
          for (int a2 = 0; a2 < np[1]; ++a2)
            for (int a3 = 0; a3 < np[2]; ++a3) {
              double wr, wi;
              ipow(a1 + a2 + a3, wr, wi);
              const double sgn = (a2 ? sg[1] : 1.0) * (a3 ? sg[2] : 1.0);
              Xr[c] += sgn * wr * Tv[c][a1][a2][a3];
              Xi[c] += sgn * wi * Tv[c][a1][a2][a3];
            }
      }
      double th[3], d[3];
      for (int J = 0; J < 3; ++J) th[J] = sg[J] * two_pi * kk[J] / nn[J];
      for (int J = 0; J < 3; ++J)
        d[J] = 2.0 * sin(0.5 * th[J]) * cos(0.5 * th[(J + 1) % 3]) * cos(0.5 * th[(J + 2) % 3]);
      const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
      double Ur[3] = {0.0, 0.0, 0.0}, Ui[3] = {0.0, 0.0, 0.0};
      if (d2 > 1e-13) {
        const double dr = d[0] * Xr[0] + d[1] * Xr[1] + d[2] * Xr[2];
        const double di = d[0] * Xi[0] + d[1] * Xi[1] + d[2] * Xi[2];
        const double inv = 1.0 / (g.mu0 * d2);
        for (int c = 0; c < 3; ++c) {
          Ur[c] = (Xr[c] - bcoef * d[c] * dr / d2) * inv;
          Ui[c] = (Xi[c] - bcoef * d[c] * di / d2) * inv;
        }
      }
      // T[a] = (1 / number of sign combinations) Re(sum_s conj(w_a(s)) U(s))
      for (int c = 0; c < 3; ++c)
        for (int a1 = 0; a1 < np[0]; ++a1)
          for (int a2 = 0; a2 < np[1]; ++a2)
            for (int a3 = 0; a3 < np[2]; ++a3) {
              double wr, wi;
              ipow(a1 + a2 + a3, wr, wi);
              const double sgn = (a2 ? sg[1] : 1.0) * (a3 ? sg[2] : 1.0);
              Tu[c][a1][a2][a3] += sgn * (wr * Ur[c] + wi * Ui[c]);
            }
    }
  const double inv_ns = 1.0 / (np[1] * np[2]);
  for (int c = 0; c < 3; ++c)
    for (int a1 = 0; a1 < np[0]; ++a1)
      for (int a2 = 0; a2 < np[1]; ++a2)
        for (int a3 = 0; a3 < np[2]; ++a3)
          buf[c * Nn + idx[0][a1] + (long long)Nx * (idx[1][a2] + (long long)Ny * idx[2][a3])] =
              Tu[c][a1][a2][a3] * inv_ns;
}

// The isotropic medium under normal-mixed faces (no periodic axis; on every face the normal
// component and the tangential ones have opposite symmetries).  On each axis the normal and
// the tangential components then use complementary transforms (DCT1/DST1 or DCT3/DST3) with
// the same angle at the same storage index, and one frequency (k1, k2, k3) holds the
// coefficients of all three components at node index (k1, k2, k3).  Derivatives map the
// cosine of a tangential component to the sine of the normal one with a minus sign and back
// with a plus sign, so the symbol is S M S, with M the real periodic symbol above and
// S = diag(s_J), s_J = +1 where the normal component is sine-type and -1 where it is
// cosine-type.  A component absent at a frequency (a DST1 line at k = 0 or n) decouples there
// (its factor of d vanishes) and is left untouched.
__global__ __launch_bounds__(kBlock) void k_green_iso_dtt(Geo g, double* buf, DevState* st, int force) {
  if (!force && st->done) return;
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (e >= g.Nn) return;
  const int Nx = g.N[0], Ny = g.N[1];
  const int k[3] = {(int)(e % Nx), (int)((e / Nx) % Ny), (int)(e / ((long long)Nx * Ny))};
  double th[3], sg[3];
  bool pres[3] = {true, true, true};
#pragma unroll
  for (int J = 0; J < 3; ++J) {
    const int half = g.iso_axis[J] & 1, nsin = (g.iso_axis[J] >> 1) & 1;
    th[J] = 3.14159265358979323846264338327950288 * (k[J] + (half ? 0.5 : 0.0)) / g.n[J];
    sg[J] = nsin ? 1.0 : -1.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int sine = (c == J) ? nsin : !nsin;
      const int lo = (!half && sine) ? 1 : 0;
      const int hi = (half || sine) ? g.n[J] - 1 : g.n[J];
      pres[c] = pres[c] && k[J] >= lo && k[J] <= hi;
    }
  }
  double X[3], d[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) X[c] = pres[c] ? sg[c] * buf[c * g.Nn + e] : 0.0;
#pragma unroll
  for (int J = 0; J < 3; ++J)
    d[J] = 2.0 * sin(0.5 * th[J]) * cos(0.5 * th[(J + 1) % 3]) * cos(0.5 * th[(J + 2) % 3]);
  const double d2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
  double U[3] = {0.0, 0.0, 0.0};
  if (d2 > 1e-13) {
    const double bcoef = (g.lam0 + g.mu0) / (g.lam0 + 2.0 * g.mu0);
    const double dX = d[0] * X[0] + d[1] * X[1] + d[2] * X[2];
    const double inv = 1.0 / (g.mu0 * d2);
#pragma unroll
    for (int c = 0; c < 3; ++c) U[c] = (X[c] - bcoef * d[c] * dX / d2) * inv;
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    if (pres[c]) buf[c * g.Nn + e] = sg[c] * U[c];
}

void launch_green_iso(const Geo& g, double* buf, DevState* st, int force, hipStream_t s) {
  if (g.iso == 2) {
    hipLaunchKernelGGL(k_green_iso_dtt, dim3(grid_for(g.Nn, 1 << 30)), dim3(kBlock), 0, s, g, buf, st, force);
    return;
  }
  const long long ncls = (long long)(g.n[0] / 2 + 1) * (g.n[1] / 2 + 1) * (g.n[2] / 2 + 1);
  hipLaunchKernelGGL(k_green_iso, dim3(grid_for(ncls, 1 << 30)), dim3(kBlock), 0, s, g, buf, st, force);
}

// ---------------------------------------------------------------------------
// proj_U kernels and bookkeeping
// ---------------------------------------------------------------------------
// proj_U of the relations (eq 11, eq 15): u += wd (val - wa . u) / (wa . wd) over the support.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_weak(Geo g, T* u, WeakDev w, DevState* st, int force) {
  if (!force && st->done) return;
  const long long r = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  if (r >= w.m) return;
  const int lane = threadIdx.x & 63;
  const long long o0 = w.off[r];
  const bool act = lane < w.off[r + 1] - o0;
  long long e = 0;
  double wa = 0.0, wd = 0.0, v = 0.0;
  if (act) {
    e = w.comp[r] * g.Nn + w.nodes[o0 + lane];
    wa = w.wa[o0 + lane];
    wd = w.wd[o0 + lane];
    v = (double)u[e];
  }
  const double num = wave_sum(wa * v), den = wave_sum(wa * wd);
  const double corr = (w.val[r] - num) / den;
  if (act) u[e] = (T)(v + wd * corr);
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
__global__ __launch_bounds__(kBlock) void k_convert(const A* __restrict__ in, Bt* __restrict__ out, long long n,
                                                    double f) {
  if (f == 1.0) {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
      out[e] = (Bt)in[e];
  } else {
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
      out[e] = (Bt)((double)in[e] * f);
  }
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

// Stiffness intake: per voxel (lam, mu), or (E, nu) when enu, of type Ti -> lam, mu of the
// working type To in the workspace, with the checks finite values, mu >= 0 and 3 lam + 2 mu >= 0
// (for E, nu: E >= 0 and -1 < nu < 1/2); per block: worst check (2 non-finite, 1 out of range),
// max lam, max mu.  Fixed reduction order.
template <typename Ti, typename To>
__global__ __launch_bounds__(kBlock) void k_stiffness_in(const Ti* __restrict__ a, const Ti* __restrict__ b, int enu,
                                                         long long nv, To* __restrict__ lam, To* __restrict__ mu,
                                                         double* __restrict__ out) {
  __shared__ double sh[3 * 64];
  double bad = 0.0, ml = -INFINITY, mm = -INFINITY;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < nv; e += (long long)gridDim.x * blockDim.x) {
    const double x = (double)a[e], y = (double)b[e];
    double l = x, m = y;
    if (enu) {
      l = m = 0.0;
      if (!isfinite(x) || !isfinite(y)) {
        bad = fmax(bad, 2.0);
      } else if (x < 0.0 || !(y > -1.0 && y < 0.5)) {
        bad = fmax(bad, 1.0);
      } else {
        l = x * y / ((1.0 + y) * (1.0 - 2.0 * y));
        m = x / (2.0 * (1.0 + y));
      }
    } else if (!isfinite(l) || !isfinite(m)) {
      bad = fmax(bad, 2.0);
    } else if (m < 0.0 || 3.0 * l + 2.0 * m < 0.0) {
      bad = fmax(bad, 1.0);
    }
    lam[e] = (To)l;
    mu[e] = (To)m;
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

// x *= s over n values (length unit of the ABI <-> voxel units)
__global__ __launch_bounds__(kBlock) void k_scale(double* __restrict__ x, long long n, double s) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    x[e] *= s;
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

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
template <typename T>
void launch_residual(const Geo& g, const Bufs<T>& B, const ContactDev& ct, DevState* st, double* part, int nblk,
                     int force, int write_p, hipStream_t s) {
  if (g.hex) {
    if (g.fs) hipLaunchKernelGGL((k_residual<T, true, true>), dim3(nblk), dim3(kBlock), 0, s, g, B, ct, st, part, force, write_p);
    else hipLaunchKernelGGL((k_residual<T, false, true>), dim3(nblk), dim3(kBlock), 0, s, g, B, ct, st, part, force, write_p);
  } else {
    if (g.fs) hipLaunchKernelGGL((k_residual<T, true, false>), dim3(nblk), dim3(kBlock), 0, s, g, B, ct, st, part, force, write_p);
    else hipLaunchKernelGGL((k_residual<T, false, false>), dim3(nblk), dim3(kBlock), 0, s, g, B, ct, st, part, force, write_p);
  }
}

template <typename T>
void launch_weak(const Geo& g, const Bufs<T>& B, const WeakDev& w, DevState* st, int force, hipStream_t s) {
  if (w.m == 0) return;
  hipLaunchKernelGGL(k_weak<T>, dim3(rel_grid(w.m)), dim3(kBlock), 0, s, g, B, w, st, force);
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
void launch_proj(const Geo& g, T* u, const WeakDev& w, const ContactDev& ct, const StrongDev& sd, DevState* st,
                 int advance, int force, hipStream_t s) {
  if (w.m > 0) hipLaunchKernelGGL(k_proj_weak<T>, dim3(rel_grid(w.m)), dim3(kBlock), 0, s, g, u, w, st, force);
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
void launch_convert(const A* in, Bt* out, long long n, hipStream_t s, double f) {
  hipLaunchKernelGGL((k_convert<A, Bt>), dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, in, out, n, f);
}

template <typename T>
void launch_zero_amask(const Geo& g, T* u, hipStream_t s) {
  hipLaunchKernelGGL(k_zero_amask<T>, dim3(grid_for(g.Nn, 8192)), dim3(kBlock), 0, s, g, u);
}

void launch_extend(DevState* st, int iters, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_extend, dim3(1), dim3(1), 0, s, st, iters, tol);
}

void launch_stiffness_in(const void* a, const void* b, int in_f32, int enu, long long nv, void* lam, void* mu,
                         int out_f32, double* out, int nblk, hipStream_t s) {
  if (in_f32 && out_f32)
    hipLaunchKernelGGL((k_stiffness_in<float, float>), dim3(nblk), dim3(kBlock), 0, s, (const float*)a, (const float*)b, enu,
                       nv, (float*)lam, (float*)mu, out);
  else if (in_f32)
    hipLaunchKernelGGL((k_stiffness_in<float, double>), dim3(nblk), dim3(kBlock), 0, s, (const float*)a, (const float*)b,
                       enu, nv, (double*)lam, (double*)mu, out);
  else if (out_f32)
    hipLaunchKernelGGL((k_stiffness_in<double, float>), dim3(nblk), dim3(kBlock), 0, s, (const double*)a,
                       (const double*)b, enu, nv, (float*)lam, (float*)mu, out);
  else
    hipLaunchKernelGGL((k_stiffness_in<double, double>), dim3(nblk), dim3(kBlock), 0, s, (const double*)a,
                       (const double*)b, enu, nv, (double*)lam, (double*)mu, out);
}

void launch_scale(double* x, long long n, double f, hipStream_t s) {
  hipLaunchKernelGGL(k_scale, dim3(grid_for(n, 8192)), dim3(kBlock), 0, s, x, n, f);
}

#define FFTC_INST(T)                                                                                              \
  template void launch_residual<T>(const Geo&, const Bufs<T>&, const ContactDev&, DevState*, double*, int, int,   \
                                   int, hipStream_t);                                                                  \
  template void launch_weak<T>(const Geo&, const Bufs<T>&, const WeakDev&, DevState*, int, hipStream_t);         \
  template void launch_anderson<T>(const Bufs<T>&, long long, DevState*, double*, int, hipStream_t);             \
  template void launch_proj<T>(const Geo&, T*, const WeakDev&, const ContactDev&, const StrongDev&, DevState*,   \
                               int, int, hipStream_t);                                                            \
  template void launch_contact_init<T>(const Geo&, const T*, const ContactDev&, hipStream_t);                     \
  template void launch_contact_force<T>(const Geo&, const T*, const ContactDev&, double*, int, hipStream_t);     \
  template void launch_reactions<T>(const Geo&, const Bufs<T>&, const StrongDev&, double*, hipStream_t);         \
  template void launch_zero_amask<T>(const Geo&, T*, hipStream_t);                                                 \
  template void launch_flags_combine<T>(const Bufs<T>&, long long, DevState*, int, hipStream_t);

FFTC_INST(double)
FFTC_INST(float)
template void launch_convert<double, double>(const double*, double*, long long, hipStream_t, double);
template void launch_convert<double, float>(const double*, float*, long long, hipStream_t, double);
template void launch_convert<float, double>(const float*, double*, long long, hipStream_t, double);

}  // namespace fftc
