// Residual-form iteration kernels of libfftc (FP32 fields, FP64 displacement) for CDNA4.
#include "fftc_internal.h"
#include "fftc_launch.h"
#include "fftc_common.h"

#include <math.h>
#include <algorithm>
#include <atomic>

namespace fftc {

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
// FP64 and rounded once to TS, the stress and divergence arithmetic is in TS (T, or FP64 for
// the refining passes of the FP32 form), and p is rounded to T.
template <typename T, bool SIG, bool FS = false, typename TS = T>
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
  TS nb[27][3];
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
        for (int c = 0; c < 3; ++c) nb[q][c] = (TS)(u[c * Nn + idx] - u0[c]);
      }
#pragma unroll
  for (int c = 0; c < 3; ++c) nb[13][c] = TS(0);
  TS F[3] = {TS(0), TS(0), TS(0)};
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
    const TS l = (TS)lam[vid], m = (TS)mu[vid];
    TS G[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int s = 0; s < 3; ++s) G[r][s] = TS(0);
    const int par = (ax + ay + az) & 1;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
      if (((cx + cy + cz) & 1) != par) continue;
      const int q = (cx - ax + 1) + 3 * (cy - ay + 1) + 9 * (cz - az + 1);
      const TS sx = TS(cx ? 0.5 : -0.5), sy = TS(cy ? 0.5 : -0.5), sz = TS(cz ? 0.5 : -0.5);
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        G[r][0] += sx * nb[q][r];
        G[r][1] += sy * nb[q][r];
        G[r][2] += sz * nb[q][r];
      }
    }
    const TS bx = TS(ax ? 0.25 : -0.25), by = TS(ay ? 0.25 : -0.25), bz = TS(az ? 0.25 : -0.25);
    if constexpr (FS) {
      TS P[3][3];
      svk_pk1<TS>(G, l, m, P);
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
    const TS tr = G[0][0] + G[1][1] + G[2][2];
    const TS s00 = l * tr + TS(2) * m * G[0][0];
    const TS s11 = l * tr + TS(2) * m * G[1][1];
    const TS s22 = l * tr + TS(2) * m * G[2][2];
    const TS s01 = m * (G[0][1] + G[1][0]);
    const TS s02 = m * (G[0][2] + G[2][0]);
    const TS s12 = m * (G[1][2] + G[2][1]);
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
  const TS w2b = TS(1 << bcount(g, xyz));
#pragma unroll
  for (int c = 0; c < 3; ++c) p[c] = is_antisym(g, c, xyz) ? T(0) : (T)(-w2b * F[c]);
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
// p, p itself, and (ACV_P, from the second iteration on) dY_i = p_i - p_{i-1} + K0 delta_i and
// R_i = p_i + K0 delta_i - e_{i-1} = dY_i + c_{i-1}, with c = p - e the correction of the last
// Anderson combination (0 after a plain iteration).  R_i goes to a ring of four, from which the
// Gram pass forms the differences with the same FP32 subtraction.  kd = K0 delta at the node
// (read only when kd_used).
// INC: p holds the increment dp_i (the divergence term of the stresses of delta_i) and p_i is
// p_{i-1} + dp_i; dY and R are formed from dp_i itself, so that they carry no cancellation
// against |p| (p_i - p_{i-1} in FP32 is rounding noise once the iteration stagnates).
// Node inputs of the tail that do not depend on p: mask, c_{i-1}, p_{i-1}.
template <typename T>
struct TailIn {
  uint8_t m;
  T cw;   // 1 after an accelerating iteration, else 0 (c is then p_{i-1}, read in its place)
  T c[3], pp[3];
};

template <typename T>
__device__ __forceinline__ void tail_load(const DeltaBufs<T>& D, long long Nn, bool kd_used, bool inc, int ecomb,
                                          const T* pp, long long node, TailIn<T>& t) {
  t.m = D.mask[node];
  // a uniform choice of source (no branch around the loads): after a plain iteration c is 0
  // and the second load of p_{i-1} is served by the cache.  The pass from u applies cw in
  // the tail, so its loads stay in flight over the layer's stresses (applied here, the pass
  // took 0.82 instead of 0.72 ms at 256^3); the incremental pass, which fetches these inputs
  // one step ahead, applies it here (0.53 against 0.55 ms per iteration, measured).
  const T* cs = ecomb ? D.e : pp;
  t.cw = ecomb ? T(1) : T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    t.c[c] = T(0);
    t.pp[c] = T(0);
    if (kd_used || inc) t.pp[c] = pp[c * Nn + node];
    if (kd_used) t.c[c] = inc ? t.cw * cs[c * Nn + node] : cs[c * Nn + node];
  }
  if (inc) t.cw = T(1);
}

// GEN = false: no rigid obstacle and no singular modes (both checked by the launcher).
template <typename T, bool GEN, bool INC = false>
__device__ __forceinline__ void delta_tail(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, int cur,
                                           bool kd_used, int il, int slot, T* pc, T* Rc, int i, int j, int k,
                                           long long node, T p[3], const T kd[3], const TailIn<T>& tin,
                                           double* acc) {
  static_assert(!(GEN && INC), "the incremental pass has no contact or singular modes");
  const long long Nn = g.Nn;
  const int xyz[3] = {i, j, k};
  // singular-mode coefficients of u (projection Pi of the update)
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (!GEN || !g.sing[c]) continue;
    const double wu = sing_weight(g, xyz) * D.u[c * Nn + node];
    acc[8 + 2 * c] += wu;
    if (g.sing[c] & 2) acc[9 + 2 * c] += ((i + j + k) & 1) ? -wu : wu;
  }
  const uint8_t m = tin.m;
  // dp: p_i - p_{i-1} as formed (INC: the increment itself, after the masking below)
  T dp[3];
  if (GEN && ct.on && (m & M_FACE)) {
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
#pragma unroll
    for (int c = 0; c < 3; ++c) dp[c] = p[c] - tin.pp[c];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (m & (M_STRONG << c)) p[c] = T(0);
      if constexpr (INC) {
        dp[c] = p[c];
        p[c] = tin.pp[c] + dp[c];
      } else {
        dp[c] = p[c] - tin.pp[c];
      }
      if (!(m & (M_WEAK << c))) acc[0] += (double)p[c] * p[c];
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) pc[c * Nn + node] = p[c];
  if (kd_used) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long e = c * Nn + node;
      // At a DOF held at 0 by a Dirichlet face p is 0 and K0 delta is taken from the
      // symmetric image; the transforms drop these entries, but they stay in the Gram matrix
      // of the differences (measured: zeroing them makes the FP32 least squares less robust).
      const T y = dp[c] + kd[c];
      Rc[e] = y + tin.cw * tin.c[c];
      if (il >= 2) D.dY[slot][e] = y;
    }
  }
}

// TS: stress arithmetic (T, or FP64 once the residual is below the refinement threshold);
// the instance whose kind is not the state's pass of this iteration returns at once (this
// untiled pass has no incremental form: its problems take the full pass every iteration).
template <typename T, bool FS, typename TS>
__global__ __launch_bounds__(kBlock) void k_residual_d(Geo g, DeltaBufs<T> D, ContactDev ct, DevState* st,
                                                       double* __restrict__ part) {
  __shared__ double sh[kPartStrideD * 16];
  if (st->done || res_pass(st) != (sizeof(TS) == 8 ? PASS_U64 : PASS_U)) return;
  double acc[kPartStrideD];
#pragma unroll
  for (int q = 0; q < kPartStrideD; ++q) acc[q] = 0.0;
  const int Nx = g.N[0], Ny = g.N[1];
  const long long Nn = g.Nn;
  const int cur = ct.on ? st->vpar : 0;
  const int il = st->i_local, par = st->it & 1, acvp = (st->acv == 2), ecomb = st->accel_ok;
  const int slot = (il + 1) % 3;   // (il - 2) mod 3
  const bool kd_used = acvp && il >= 1;
  T* pc = D.p[par];
  const T* pp = D.p[par ^ 1];
  T* Rc = D.R[il & 3];
  long long lo, hi;
  xcd_chunk(Nn, lo, hi);
  for (long long node = lo + threadIdx.x; node < hi; node += blockDim.x) {
    const int nd = (int)node;
    const int r = nd / Nx;
    const int i = nd - r * Nx;
    const int k = r / Ny, j = r - k * Ny;
    T p[3];
    double sn = 0.0, ms[6] = {0, 0, 0, 0, 0, 0};
    node_eval_d<T, true, FS, TS>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
    acc[1] += sn;
    T kd[3] = {T(0), T(0), T(0)};
    if (kd_used) stencil_k0<T>(g, D.delta, i, j, k, kd);
    TailIn<T> tin;
    tail_load<T>(D, Nn, kd_used, false, ecomb, pp, node, tin);
    delta_tail<T, true>(g, D, ct, cur, kd_used, il, slot, pc, Rc, i, j, k, node, p, kd, tin, acc);
  }
  block_sum<kPartStrideD>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < kPartStrideD; ++q) part[q * kPartRows + blockIdx.x] = acc[q];
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

// INC: the incremental pass (small strain, no contact or singular modes): the stresses are
// those of delta_i, formed in T from the delta planes, and p_i = p_{i-1} + their divergence
// term; u is not read and no stress norm is formed (the control keeps the last full pass's).
// The small-strain pass with contact or singular modes (GEN, T stresses) is held to three
// waves per SIMD, the residency the tile grid assumes (it needed one register granule more:
// two blocks per CU ran the grid in two rounds).
template <typename T, bool FS, bool GEN, typename TS, bool INC = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu((GEN && !FS && sizeof(TS) == 4) ? 3 : 1)))
void k_residual_dt(Geo g, DeltaBufs<T> D, ContactDev ct, DevState* st, double* __restrict__ part, TileGrid tg) {
  static_assert(!INC || (!FS && !GEN && sizeof(TS) == sizeof(T)), "incremental pass: small strain, T stresses");
  constexpr int NQ = FS ? 9 : 6;      // stored stress components per tetrahedron (PK1: all nine)
  __shared__ double su_raw[INC ? 1 : 2 * 3 * kHY * kHX];
  double (*su)[3][kHY][kHX] = reinterpret_cast<double (*)[3][kHY][kHX]>(su_raw);
  __shared__ T sdl[4][3][kHY][kHX];
  __shared__ TS ss[2][2 * NQ][kVY][kVX];   // stress component q of the voxels of a layer (in TS)
  // the final block sum reuses the stress buffer (block_sum starts with a barrier)
  static_assert(sizeof(ss) >= sizeof(double) * kPartStrideD * 16, "block-sum scratch");
  double* sh = reinterpret_cast<double*>(&ss[0][0][0][0]);
  if (st->done || res_pass(st) != (INC ? PASS_INC : (sizeof(TS) == 8 ? PASS_U64 : PASS_U))) return;
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
  const int il = st->i_local, par = st->it & 1, acvp = (st->acv == 2), ecomb = st->accel_ok;
  const int slot = (il + 1) % 3;
  const bool kd_used = acvp && il >= 1;
  const bool dl = INC || kd_used;   // delta planes staged
  T* pc = D.p[par];
  const T* pp = D.p[par ^ 1];
  T* Rc = D.R[il & 3];
  double acc[kPartStrideD];
#pragma unroll
  for (int q = 0; q < kPartStrideD; ++q) acc[q] = 0.0;

  // Node planes are fetched into registers one step ahead and committed to LDS the next
  // step.  u: su[pz & 1], nodes outside the grid read as 0 (no voxel uses them); delta:
  // sdl[pz mod 4] with the stencil's halo (mirror or periodic image).
  double ru[INC ? 1 : kPR];
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
      if constexpr (!INC) ru[r] = 0.0;
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
        if constexpr (!INC)
          if (ok) ru[r] = D.u[c * Nn + gx + Nx * (gy + Ny * gz)];
        if (dl) {
          const int mx = mirror_coord(g, x0 - 1 + hx, 0), my = mirror_coord(g, y0 - 1 + hy, 1);
          if (okm && mx >= 0 && mx < Nx && my >= 0 && my < Ny) rd[r] = D.delta[c * Nn + mx + Nx * (my + Ny * mz)];
        }
      }
    }
  };
  auto commit = [&](int pz) {
    double* du = INC ? nullptr : &su[pz & 1][0][0][0];
    T* dd = &sdl[ring4(pz)][0][0][0];
#pragma unroll
    for (int r = 0; r < kPR; ++r) {
      const int e = tid + 256 * r;
      if (e < kPlane) {
        if constexpr (!INC) du[e] = ru[r];
        if (dl) dd[e] = rd[r];
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
      TS (*out)[kVY][kVX] = ss[lz & 1];
      const int ux = vux, uy = vuy;
      if (!ok) {
#pragma unroll
        for (int q = 0; q < 2 * NQ; ++q) out[q][ly][lx] = TS(0);
        return;
      }
      const TS lt = (TS)l, mt = (TS)m;
      TS d[8][3];
      if constexpr (INC) {
        // differences of delta (T) against the voxel's corner 000
        const int s0 = ring4(lz), s1 = ring4(lz + 1);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const T ref = sdl[s0][c][ly][lx];
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) {
            const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
            d[cc][c] = cc == 0 ? TS(0) : (TS)(sdl[cz ? s1 : s0][c][ly + cy][lx + cx] - ref);
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double ref = su[lo][c][ly][lx];
#pragma unroll
          for (int cc = 0; cc < 8; ++cc) {
            const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
            d[cc][c] = cc == 0 ? TS(0) : (TS)(su[cz ? hi : lo][c][ly + cy][lx + cx] - ref);
          }
        }
      }
      const bool own = !INC && own_z && ux >= x0 && ux < x0 + kTX && ux < nx && uy >= y0 && uy < y0 + kTY && uy < ny;
      TS vs = TS(0);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        TS G[3][3];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int q = 0; q < 3; ++q) G[r][q] = TS(0);
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) {
          const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
          if (((cx + cy + cz) & 1) != t) continue;
          const TS sx = TS(cx ? 0.5 : -0.5), sy = TS(cy ? 0.5 : -0.5), sz = TS(cz ? 0.5 : -0.5);
#pragma unroll
          for (int r = 0; r < 3; ++r) {
            G[r][0] += sx * d[cc][r];
            G[r][1] += sy * d[cc][r];
            G[r][2] += sz * d[cc][r];
          }
        }
        if constexpr (FS) {
          TS P[3][3];
          svk_pk1<TS>(G, lt, mt, P);
#pragma unroll
          for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c) out[t * 9 + r * 3 + c][ly][lx] = P[r][c];
          if (own) {
#pragma unroll
            for (int r = 0; r < 3; ++r)
#pragma unroll
              for (int c = 0; c < 3; ++c) vs += P[r][c] * P[r][c];
          }
          continue;
        }
        const TS tr = G[0][0] + G[1][1] + G[2][2];
        const TS s00 = lt * tr + TS(2) * mt * G[0][0];
        const TS s11 = lt * tr + TS(2) * mt * G[1][1];
        const TS s22 = lt * tr + TS(2) * mt * G[2][2];
        const TS s01 = mt * (G[0][1] + G[1][0]);
        const TS s02 = mt * (G[0][2] + G[2][0]);
        const TS s12 = mt * (G[1][2] + G[2][1]);
        out[t * 6 + 0][ly][lx] = s00;
        out[t * 6 + 1][ly][lx] = s11;
        out[t * 6 + 2][ly][lx] = s22;
        out[t * 6 + 3][ly][lx] = s01;
        out[t * 6 + 4][ly][lx] = s02;
        out[t * 6 + 5][ly][lx] = s12;
        // the voxel's two tetrahedra in T, added to the FP64 block sum once per voxel
        if (own) vs += s00 * s00 + s11 * s11 + s22 * s22 + TS(2) * (s01 * s01 + s02 * s02 + s12 * s12);
      }
      if (own) acc[1] += 0.5 * (double)vs;
    }
  };
  const int nlx = tid % kTX, nly = tid / kTX;
  const bool nact = tid < kTX * kTY && x0 + nlx < Nx && y0 + nly < Ny;
  TailIn<T> tin;
  auto nodes = [&](int z) {
    if (!nact) return;
    const int lx = nlx, ly = nly;
    const int i = x0 + lx, j = y0 + ly;
    TS F[3] = {TS(0), TS(0), TS(0)};
#pragma unroll
    for (int a = 0; a < 8; ++a) {
      const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
      // voxel (i - ax, j - ay, z - az): local voxel (lx + 1 - ax, ly + 1 - ay), layer z - az;
      // the node is its corner (ax, ay, az), in tetrahedron T1 (even) or T2 (odd)
      const int q0 = ((ax + ay + az) & 1) * NQ, vy = ly + 1 - ay, vx = lx + 1 - ax;
      TS (*sv)[kVY][kVX] = ss[(z - az) & 1];
      const TS bxw = TS(ax ? 0.25 : -0.25), byw = TS(ay ? 0.25 : -0.25), bzw = TS(az ? 0.25 : -0.25);
      if constexpr (FS) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
          F[r] += bxw * sv[q0 + 3 * r][vy][vx] + byw * sv[q0 + 3 * r + 1][vy][vx] + bzw * sv[q0 + 3 * r + 2][vy][vx];
        continue;
      }
      const TS s00 = sv[q0 + 0][vy][vx], s11 = sv[q0 + 1][vy][vx], s22 = sv[q0 + 2][vy][vx];
      const TS s01 = sv[q0 + 3][vy][vx], s02 = sv[q0 + 4][vy][vx], s12 = sv[q0 + 5][vy][vx];
      F[0] += bxw * s00 + byw * s01 + bzw * s02;
      F[1] += bxw * s01 + byw * s11 + bzw * s12;
      F[2] += bxw * s02 + byw * s12 + bzw * s22;
    }
    const int xyz[3] = {i, j, z};
    const TS w2b = TS(1 << bcount(g, xyz));
    T p[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) p[c] = is_antisym(g, c, xyz) ? T(0) : (T)(-w2b * F[c]);
    T kd[3] = {T(0), T(0), T(0)};
    if (kd_used) {
      const int zm = ring4(z - 1), z0 = ring4(z), zp = ring4(z + 1);
      const int hx = lx + 1, hy = ly + 1;
      // one component at a time: keeps the 13 LDS reads of a component, not all 39, in
      // flight (194 -> 155 VGPRs, three waves per SIMD instead of two)
#pragma unroll 1
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
    delta_tail<T, GEN, INC>(g, D, ct, cur, kd_used, il, slot, pc, Rc, i, j, z, node, p, kd, tin, acc);
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
  // the incremental pass (fewer registers) fetches the tail inputs one step ahead
  TailIn<T> tnext;
  auto tail_at = [&](int z, TailIn<T>& t) {
    const long long node = (long long)(x0 + nlx) + (long long)Nx * ((long long)(y0 + nly) + (long long)Ny * z);
    tail_load<T>(D, g.Nn, kd_used, INC, ecomb, pp, node, t);
  };
  if (INC && nact) tail_at(zb, tnext);
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
    if constexpr (INC) {
      tin = tnext;
      if (nact && z + 1 < ze) tail_at(z + 1, tnext);
    } else {
      if (nact) tail_at(z, tin);
    }
    __syncthreads();
    layer(z, true, lcur, mcur, okcur);
    __syncthreads();
    nodes(z);
  }
  block_sum<kPartStrideD>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < kPartStrideD; ++q) part[q * kPartRows + blockIdx.x] = acc[q];
  // rows the control sums beyond this grid (another instance's larger grid): cleared
  if (blockIdx.x == 0)
    for (int q = 0; q < kPartStrideD; ++q)
      for (int r = (int)gridDim.x + tid; r < tg.rows; r += 256) part[q * kPartRows + r] = 0.0;
}

// Mean stress of the residual-form iterate, once, when the solve is reported: per voxel the
// stresses of its two tetrahedra as the tiled residual pass forms them (differences of the
// FP64 displacement against corner 000, rounded to T; the stress arithmetic in T), added in T
// and weighted by the integration-point weight 1/2 into FP64 block sums.  Components in the
// order xx, yy, zz, yz, xz, xy (first Piola-Kirchhoff for finite strain).
template <typename T, bool FS>
__global__ __launch_bounds__(kBlock) void k_mean_stress_d(Geo g, const double* __restrict__ u,
                                                          const T* __restrict__ lam, const T* __restrict__ mu,
                                                          double* __restrict__ part) {
  __shared__ double sh[6 * 16];
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  const int nx = g.n[0], ny = g.n[1];
  const long long Nn = g.Nn;
  long long lo, hi;
  xcd_chunk(g.Nv, lo, hi);
  for (long long v = lo + threadIdx.x; v < hi; v += blockDim.x) {
    const int vx = (int)(v % nx);
    const long long r = v / nx;
    const int vy = (int)(r % ny), vz = (int)(r / ny);
    double uc[8][3];
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      int x = vx + (cc & 1), y = vy + ((cc >> 1) & 1), z = vz + ((cc >> 2) & 1);
      if (x == g.N[0]) x = 0;   // only on a periodic axis, where there are n nodes
      if (y == g.N[1]) y = 0;
      if (z == g.N[2]) z = 0;
      const long long node = (long long)x + (long long)g.N[0] * ((long long)y + (long long)g.N[1] * z);
#pragma unroll
      for (int c = 0; c < 3; ++c) uc[cc][c] = u[c * Nn + node];
    }
    const T l = lam[v], m = mu[v];
    T vs[6] = {T(0), T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      T G[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) G[a][b] = T(0);
#pragma unroll
      for (int cc = 1; cc < 8; ++cc) {
        const int cx = cc & 1, cy = (cc >> 1) & 1, cz = (cc >> 2) & 1;
        if (((cx + cy + cz) & 1) != t) continue;
        const T sx = T(cx ? 0.5 : -0.5), sy = T(cy ? 0.5 : -0.5), sz = T(cz ? 0.5 : -0.5);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const T d = (T)(uc[cc][a] - uc[0][a]);
          G[a][0] += sx * d;
          G[a][1] += sy * d;
          G[a][2] += sz * d;
        }
      }
      if constexpr (FS) {
        T P[3][3];
        svk_pk1<T>(G, l, m, P);
        vs[0] += P[0][0];
        vs[1] += P[1][1];
        vs[2] += P[2][2];
        vs[3] += P[1][2];
        vs[4] += P[0][2];
        vs[5] += P[0][1];
      } else {
        const T tr = G[0][0] + G[1][1] + G[2][2];
        vs[0] += l * tr + T(2) * m * G[0][0];
        vs[1] += l * tr + T(2) * m * G[1][1];
        vs[2] += l * tr + T(2) * m * G[2][2];
        vs[3] += m * (G[1][2] + G[2][1]);
        vs[4] += m * (G[0][2] + G[2][0]);
        vs[5] += m * (G[0][1] + G[1][0]);
      }
    }
#pragma unroll
    for (int q = 0; q < 6; ++q) acc[q] += 0.5 * (double)vs[q];
  }
  block_sum<6>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 6; ++q) part[blockIdx.x * 6 + q] = acc[q];
}

// proj_P of the relations on several nodes (eq 14, eq 17) on p and on the quantities linear
// in p (R, and the difference dY): one wavefront per relation, one lane per support node.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_weak_d(Geo g, DeltaBufs<T> D, WeakDev w, DevState* st) {
  if (st->done) return;
  const long long r = (blockIdx.x * (long long)blockDim.x + threadIdx.x) >> 6;
  if (r >= w.m) return;   // uniform over the wavefront
  const int lane = threadIdx.x & 63;
  const int c = w.comp[r];
  const int il = st->i_local, par = st->it & 1, acvp = (st->acv == 2);
  const int slot = (il + 1) % 3;
  const long long o0 = w.off[r];
  const bool act = lane < w.off[r + 1] - o0;
  long long node = 0;
  double wa = 0.0, wb = 0.0, q = 0.0, scale = 1.0;
  if (act) {
    node = w.nodes[o0 + lane];
    wa = w.wa[o0 + lane];
    wb = w.wb[o0 + lane];
    const int i = (int)(node % g.N[0]);
    const long long t = node / g.N[0];
    const int j = (int)(t % g.N[1]), k = (int)(t / g.N[1]);
    T p[3];
    double sn = 0.0, ms[6];
    // the stresses in the precision the residual pass of this iteration used
    if (st->fine) {
      if (g.fs) node_eval_d<T, false, true, double>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
      else node_eval_d<T, false, false, double>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
    } else {
      if (g.fs) node_eval_d<T, false, true>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
      else node_eval_d<T, false, false>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
    }
    const int xyz[3] = {i, j, k};
    scale = (double)(1 << bcount(g, xyz));
    q = (double)p[c] / scale;
  }
  const double num = wave_sum(wa * q), den = wave_sum(wa * wb), sb = wave_sum(wb);
  const double f = num / den;
  const double pnew = (q - wb * f) * scale;
  const double pn = wave_sum(act ? pnew * pnew : 0.0);
  if (act) {
    const long long e = c * g.Nn + node;
    const T sh = (T)(wb * f * scale);
    D.p[par][e] = (T)pnew;
    if (acvp && il >= 1) {
      D.R[il & 3][e] -= sh;
      if (il >= 2) D.dY[slot][e] -= sh;
    }
  }
  if (lane == 0) {
    w.part[r] = pn;
    w.react[r] = -f * sb;
  }
}

// Gram matrix of the R differences and their products with R_i (accelerating iterations).
// The difference formed at local iteration j >= 2, R_j - R_{j-1} (FP32), pairs with the Y
// difference in slot (j + 1) mod 3; the three latest, j = i, i-1, i-2, come from the ring of
// four R fields (acceleration starts at i = 4, so all four are of the current run).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_gram3(DeltaBufs<T> D, long long n3, DevState* st, double* __restrict__ gpart) {
  __shared__ double sh[9 * 16];
  if (st->done || !st->accel) return;
  const int il = st->i_local;
  const T* Ri = D.R[il & 3];
  const T *Ra[3], *Rb[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int j = il - k, slot = (j + 1) % 3;
    Ra[slot] = D.R[j & 3];
    Rb[slot] = D.R[(j + 3) & 3];
  }
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n3; e += (long long)gridDim.x * blockDim.x) {
    const T d0 = Ra[0][e] - Rb[0][e], d1 = Ra[1][e] - Rb[1][e], d2 = Ra[2][e] - Rb[2][e];
    const double a0 = d0, a1 = d1, a2 = d2, r = Ri[e];
    acc[0] += a0 * a0; acc[1] += a0 * a1; acc[2] += a0 * a2;
    acc[3] += a1 * a1; acc[4] += a1 * a2; acc[5] += a2 * a2;
    acc[6] += a0 * r; acc[7] += a1 * r; acc[8] += a2 * r;
  }
  block_sum<9>(acc, sh);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < 9; ++q) gpart[q * kPartRows + blockIdx.x] = acc[q];
}

__global__ __launch_bounds__(kBlock) void k_alpha3(DevState* st, const double* __restrict__ gpart, int nblk) {
  __shared__ double sh[9 * 16];
  if (st->done || !st->accel) return;
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  sum_cols<9>(gpart, kPartRows, nblk, acc);
  block_sum<9>(acc, sh);
  if (threadIdx.x != 0) return;
  double G[3][4] = {{acc[0], acc[1], acc[2], acc[6]}, {acc[1], acc[3], acc[4], acc[7]}, {acc[2], acc[4], acc[5], acc[8]}};
  const double tr = G[0][0] + G[1][1] + G[2][2];
  for (int a = 0; a < 3; ++a) G[a][a] += 1e-14 * tr / 3.0;
  double y[3];
  bool ok = solve_pivoted<3>(G, y);
  if (ok) ok = isfinite(y[0]) && isfinite(y[1]) && isfinite(y[2]);
  if (ok)
    for (int a = 0; a < 3; ++a) st->gamma[a] = y[a];
  st->accel_ok = ok ? 1 : 0;
}

// The iteration counters move on in the last kernel of an iteration (its first thread; the
// other threads of that kernel read only the done flag), which saves a launch.
__device__ __forceinline__ void advance_iteration(DevState* st, int advance) {
  if (advance && blockIdx.x == 0 && threadIdx.x == 0) {
    st->it += 1;
    st->i_local += 1;
  }
}

// proj_U of the residual-form path on the FP64 displacement; the increment follows
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_d(Geo g, DeltaBufs<T> D, StrongDev s, WeakDev w, ContactDev ct,
                                                   DevState* st, int force, int advance) {
  if (!force && st->done) return;
  advance_iteration(st, advance);
  const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  // strong DOFs
  if (e < s.m) {
    const long long idx = s.comp[e] * g.Nn + s.node[e];
    const double old = D.u[idx];
    D.u[idx] = s.val[e];
    D.delta[idx] = (T)((double)D.delta[idx] + (s.val[e] - old));
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

// proj_U of the relations (eq 11, eq 15) on the FP64 displacement, the increment follows
template <typename T>
__global__ __launch_bounds__(kBlock) void k_proj_rel_d(Geo g, DeltaBufs<T> D, WeakDev w, DevState* st, int force,
                                                       int advance) {
  if (!force && st->done) return;
  advance_iteration(st, advance);
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
    v = D.u[e];
  }
  const double num = wave_sum(wa * v), den = wave_sum(wa * wd);
  const double corr = (w.val[r] - num) / den;
  if (act) {
    D.u[e] = v + wd * corr;
    D.delta[e] = (T)((double)D.delta[e] + wd * corr);
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
  // reactions are multipliers: the stresses here are formed in FP64 (p rounded once)
  T p[3];
  double sn = 0.0, ms[6];
  if (g.fs) node_eval_d<T, false, true, double>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
  else node_eval_d<T, false, false, double>(g, D.u, D.lam, D.mu, i, j, k, p, sn, ms);
  const int xyz[3] = {i, j, k};
  out[e] = -(double)p[s.comp[e]] / (double)(1 << bcount(g, xyz));
}

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
TileGrid residual_tiles(const Geo& g, bool inc);
TileGrid residual_tiles_fp64(const Geo& g, bool gen);

template <typename T, typename TS>
int launch_delta_residual_ts(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, DevState* st, double* part,
                             int nblk, const TileGrid& tg, hipStream_t s) {
  if (tg.tx > 0) {
    nblk = tg.tx * tg.ty * tg.nseg;
    const bool gen = ct.on || g.sing[0] || g.sing[1] || g.sing[2];
    if (g.fs && gen) hipLaunchKernelGGL((k_residual_dt<T, true, true, TS>), dim3(nblk), dim3(256), 0, s, g, D, ct, st, part, tg);
    else if (g.fs) hipLaunchKernelGGL((k_residual_dt<T, true, false, TS>), dim3(nblk), dim3(256), 0, s, g, D, ct, st, part, tg);
    else if (gen) hipLaunchKernelGGL((k_residual_dt<T, false, true, TS>), dim3(nblk), dim3(256), 0, s, g, D, ct, st, part, tg);
    else hipLaunchKernelGGL((k_residual_dt<T, false, false, TS>), dim3(nblk), dim3(256), 0, s, g, D, ct, st, part, tg);
  } else {
    if (g.fs) hipLaunchKernelGGL((k_residual_d<T, true, TS>), dim3(nblk), dim3(kBlock), 0, s, g, D, ct, st, part);
    else hipLaunchKernelGGL((k_residual_d<T, false, TS>), dim3(nblk), dim3(kBlock), 0, s, g, D, ct, st, part);
  }
  return nblk;
}

// The pass with T stresses, (refine) the pass with FP64 stresses and (inc) the incremental
// pass; the device state selects the one that works, the others return at once.  All write
// the partial rows the control step reads (the returned count).  inc is taken only for tiled
// small-strain problems without contact or singular modes (the caller's eligibility test).
template <typename T>
int launch_delta_residual(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, DevState* st, double* part,
                          int nblk, int refine, int inc, hipStream_t s) {
  const bool gen = ct.on || g.sing[0] || g.sing[1] || g.sing[2];
  const bool use_inc = inc && !g.fs && !gen;
  // each pass on the grid for its own resident count (the incremental one's taken only when
  // its segments are long enough); the control sums the largest count of rows, and a pass on
  // a smaller grid clears the rows beyond it
  TileGrid tf = residual_tiles(g, false);
  TileGrid ti = use_inc ? residual_tiles(g, true) : tf;
  TileGrid tu = refine ? residual_tiles_fp64(g, gen) : tf;
  if (tf.tx > 0) {
    const int rows = std::max(tf.rows, std::max(ti.rows, tu.rows));
    tf.rows = ti.rows = tu.rows = rows;
  }
  const int rows = launch_delta_residual_ts<T, T>(g, D, ct, st, part, nblk, tf, s);
  if (refine) launch_delta_residual_ts<T, double>(g, D, ct, st, part, nblk, tu, s);
  if (use_inc && ti.tx > 0)
    hipLaunchKernelGGL((k_residual_dt<T, false, false, T, true>), dim3(ti.tx * ti.ty * ti.nseg), dim3(256), 0, s, g, D,
                       ct, st, part, ti);
  return tf.tx > 0 ? tf.rows : rows;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_diff(const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ out,
                                                 long long n) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    out[e] = a[e] - b[e];
}

template <typename T>
void launch_diff(const T* a, const T* b, T* out, long long n, hipStream_t s) {
  const int nblk = (int)std::max<long long>(1, std::min<long long>(4096, (n + kBlock - 1) / kBlock));
  hipLaunchKernelGGL(k_diff<T>, dim3(nblk), dim3(kBlock), 0, s, a, b, out, n);
}

template <typename T>
int launch_mean_stress_d(const Geo& g, const DeltaBufs<T>& D, double* part, hipStream_t s) {
  const int nblk = (int)std::max<long long>(1, std::min<long long>(1024, (g.Nv + kBlock - 1) / kBlock));
  if (g.fs) hipLaunchKernelGGL((k_mean_stress_d<T, true>), dim3(nblk), dim3(kBlock), 0, s, g, D.u, D.lam, D.mu, part);
  else hipLaunchKernelGGL((k_mean_stress_d<T, false>), dim3(nblk), dim3(kBlock), 0, s, g, D.u, D.lam, D.mu, part);
  return nblk;
}

template <typename T>
void launch_delta_control(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, const WeakDev& w, DevState* st,
                          const double* part, const double* wpart, int nblk, hipStream_t s) {
  if (w.m > 0) hipLaunchKernelGGL(k_weak_d<T>, dim3(rel_grid(w.m)), dim3(kBlock), 0, s, g, D, w, st);
  launch_control(st, part, nblk, wpart, w.m, ct, kPartStrideD, s);
}

// Blocks of the tiled residual pass resident on the current device at once (blocks per CU
// at the kernel's register and LDS use, times the CU count), queried once per device and
// instance: the pass with T stresses, the incremental one, or one with FP64 stresses.
template <bool FS, bool GEN, typename TS, bool INC>
static int residual_resident() {
  static std::atomic<int> cache[64] = {};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 512;
  int r = cache[dev].load(std::memory_order_relaxed);
  if (!r) {
    int per_cu = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_residual_dt<float, FS, GEN, TS, INC>, 256, 0) !=
            hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
    r = per_cu * cus;
    cache[dev].store(r, std::memory_order_relaxed);   // every thread computes the same value
  }
  return r;
}

// segment length with the fewest (rounds x planes per block) for a resident count; ties go to
// fewer segments
static int tile_split(const Geo& g, int tx, int ty, long long resident) {
  const int Nz = g.N[2];
  const int maxseg = std::max(1, std::min(Nz, kPartRows / (tx * ty)));
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
  return bseg;
}

static TileGrid tile_grid(const Geo& g, int tx, int ty, int seg) {
  TileGrid t{tx, ty, 0, seg, 0};
  t.nseg = (g.N[2] + seg - 1) / seg;
  t.rows = tx * ty * t.nseg;
  return t;
}

// Tile grid of the tiled residual pass: tiles of kTX x kTY node columns, z split into
// segments, at most kPartRows blocks (the partial-sum rows); tx = 0 when the node plane alone
// needs more tiles than that.  A block marches its segment's planes plus two planes of
// prologue, and the blocks run in rounds of the resident count, so the split taken is the
// one with the fewest (rounds x planes per block); ties go to fewer segments.  inc: the split
// for the resident count of the incremental pass is taken when its segments are at least 8
// planes long (shorter ones add more prologue reads than the extra blocks save: measured at
// 64^3, 2-plane segments on 990 blocks against 3-plane ones on 660; at 128^3 the 13-plane
// segments on 950 blocks beat 17-plane ones on 760, 0.099 -> 0.089 ms).
TileGrid residual_tiles(const Geo& g, bool inc) {
  const int tx = (g.N[0] + kTX - 1) / kTX, ty = (g.N[1] + kTY - 1) / kTY;
  if ((long long)tx * ty > kPartRows) return TileGrid{0, 0, 0, 0, 0};
  // finite strain: the PK1 instances hold two blocks per CU (LDS), the small-strain ones three
  int bseg = tile_split(g, tx, ty,
                        g.fs ? residual_resident<true, false, float, false>() : residual_resident<false, false, float, false>());
  if (inc) {
    const int iseg = tile_split(g, tx, ty, residual_resident<false, false, float, true>());
    if (iseg >= 8) bseg = iseg;
  }
  return tile_grid(g, tx, ty, bseg);
}

// Tile grid of the pass with FP64 stresses, split for its own resident count (one or two
// blocks per CU against three or four for the FP32 instances): on another pass's grid it ran
// in two rounds.  gen: the instance for contact or singular modes.
TileGrid residual_tiles_fp64(const Geo& g, bool gen) {
  const int tx = (g.N[0] + kTX - 1) / kTX, ty = (g.N[1] + kTY - 1) / kTY;
  if ((long long)tx * ty > kPartRows) return TileGrid{0, 0, 0, 0, 0};
  int resident;
  if (g.fs) resident = gen ? residual_resident<true, true, double, false>() : residual_resident<true, false, double, false>();
  else resident = gen ? residual_resident<false, true, double, false>() : residual_resident<false, false, double, false>();
  return tile_grid(g, tx, ty, tile_split(g, tx, ty, resident));
}

template <typename T>
void launch_delta_anderson(const DeltaBufs<T>& D, long long n3, DevState* st, double* gpart, int nblk, hipStream_t s) {
  hipLaunchKernelGGL(k_gram3<T>, dim3(nblk), dim3(kBlock), 0, s, D, n3, st, gpart);
  hipLaunchKernelGGL(k_alpha3, dim3(1), dim3(kBlock), 0, s, st, gpart, nblk);
}

template <typename T>
void launch_delta_proj(const Geo& g, const DeltaBufs<T>& D, const StrongDev& sd, const WeakDev& w,
                       const ContactDev& ct, DevState* st, int force, int advance, hipStream_t s) {
  long long m = sd.m;
  if (ct.on && ct.nface > m) m = ct.nface;
  const int rel = w.m > 0;
  if (m > 0)
    hipLaunchKernelGGL(k_proj_d<T>, dim3(grid_for(m, 1 << 30)), dim3(kBlock), 0, s, g, D, sd, w, ct, st, force,
                       advance && !rel);
  if (rel) hipLaunchKernelGGL(k_proj_rel_d<T>, dim3(rel_grid(w.m)), dim3(kBlock), 0, s, g, D, w, st, force, advance);
  if (advance && m == 0 && !rel) hipLaunchKernelGGL(k_advance<T>, dim3(1), dim3(1), 0, s, st);
}

template <typename T>
void launch_reactions_d(const Geo& g, const DeltaBufs<T>& D, const StrongDev& sd, double* out, hipStream_t s) {
  if (sd.m == 0) return;
  hipLaunchKernelGGL(k_reactions_d<T>, dim3(grid_for(sd.m, 1 << 30)), dim3(kBlock), 0, s, g, D, sd, out);
}

template <typename T>
void launch_weak_d_stage(const Geo& g, const DeltaBufs<T>& D, const WeakDev& w, DevState* st, hipStream_t s) {
  if (w.m > 0) hipLaunchKernelGGL(k_weak_d<T>, dim3(rel_grid(w.m)), dim3(kBlock), 0, s, g, D, w, st);
}

template int launch_delta_residual<float>(const Geo&, const DeltaBufs<float>&, const ContactDev&, DevState*, double*,
                                          int, int, int, hipStream_t);
template void launch_delta_control<float>(const Geo&, const DeltaBufs<float>&, const ContactDev&, const WeakDev&,
                                          DevState*, const double*, const double*, int, hipStream_t);
template void launch_delta_anderson<float>(const DeltaBufs<float>&, long long, DevState*, double*, int, hipStream_t);
template void launch_delta_proj<float>(const Geo&, const DeltaBufs<float>&, const StrongDev&, const WeakDev&,
                                       const ContactDev&, DevState*, int, int, hipStream_t);
template void launch_diff<float>(const float*, const float*, float*, long long, hipStream_t);
template int launch_mean_stress_d<float>(const Geo&, const DeltaBufs<float>&, double*, hipStream_t);
template void launch_reactions_d<float>(const Geo&, const DeltaBufs<float>&, const StrongDev&, double*, hipStream_t);

}  // namespace fftc
