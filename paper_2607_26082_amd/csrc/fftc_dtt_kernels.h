// Per-axis DTT pass kernels (Tables 2-3, eq 7) and their launchers, instantiated per
// precision by fftc_dtt64.hip and fftc_dtt32.hip.
#pragma once

#include "fftc_internal.h"
#include "fftc_launch.h"
#include "fftc_dtt.h"
#include "fftc_common.h"

#include <math.h>
#include <type_traits>

namespace fftc {

// ---------------------------------------------------------------------------
// Batched per-axis discrete trigonometric transforms in LDS
// ---------------------------------------------------------------------------
// cos(2 pi k / R) and sin(2 pi k / R), k = 1 .. (R - 1) / 2, of the odd prime radices 7, 11, 13
template <int R> struct OddRadix;
template <> struct OddRadix<7> {
  static constexpr double c[3] = {0.6234898018587336, -0.22252093395631434, -0.900968867902419};
  static constexpr double s[3] = {0.7818314824680298, 0.9749279121818236, 0.43388373911755823};
};
template <> struct OddRadix<11> {
  static constexpr double c[5] = {0.8412535328311812, 0.41541501300188644, -0.142314838273285, -0.654860733945285,
                                  -0.9594929736144974};
  static constexpr double s[5] = {0.5406408174555976, 0.9096319953545183, 0.9898214418809328, 0.7557495743542583,
                                  0.28173255684142967};
};
template <> struct OddRadix<13> {
  static constexpr double c[6] = {0.8854560256532099, 0.5680647467311559, 0.120536680255323, -0.35460488704253545,
                                  -0.7485107481711012, -0.970941817426052};
  static constexpr double s[6] = {0.4647231720437685, 0.8229838658936564, 0.992708874098054, 0.9350162426854148,
                                  0.6631226582407952, 0.23931566428755768};
};

// Length-R DFT, R an odd prime, X_m = sum_j a_j e^{i sgn 2 pi j m / R}: with b_j = a_j + a_{R-j}
// and d_j = a_j - a_{R-j} (j = 1 .. H), X_m and X_{R-m} are A_m +- i sgn S_m, where
// A_m = a_0 + sum_j cos(2 pi j m / R) b_j and S_m = sum_j sin(2 pi j m / R) d_j.
template <typename T, int R>
__device__ __forceinline__ void dft_odd(cplx<T> (&a)[R], int sgn) {
  constexpr int H = (R - 1) / 2;
  cplx<T> b[H], d[H];
#pragma unroll
  for (int j = 1; j <= H; ++j) {
    b[j - 1] = cadd(a[j], a[R - j]);
    d[j - 1] = csub(a[j], a[R - j]);
  }
  cplx<T> x[R];
  x[0] = a[0];
#pragma unroll
  for (int j = 0; j < H; ++j) x[0] = cadd(x[0], b[j]);
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    cplx<T> A = a[0], S = {T(0), T(0)};
#pragma unroll
    for (int j = 1; j <= H; ++j) {
      const int k = (j * m) % R;
      const T cv = T(k <= H ? OddRadix<R>::c[k - 1] : OddRadix<R>::c[R - k - 1]);
      const T sv = T(k <= H ? OddRadix<R>::s[k - 1] : -OddRadix<R>::s[R - k - 1]);
      A = {A.re + cv * b[j - 1].re, A.im + cv * b[j - 1].im};
      S = {S.re + sv * d[j - 1].re, S.im + sv * d[j - 1].im};
    }
    const cplx<T> B = {-T(sgn) * S.im, T(sgn) * S.re};   // i sgn S
    x[m] = cadd(A, B);
    x[R - m] = csub(A, B);
  }
#pragma unroll
  for (int q = 0; q < R; ++q) a[q] = x[q];
}

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
  } else {
    dft_odd<T, R>(a, sgn);
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

// BIG: the plan has a radix 7, 11 or 13 (a separate kernel instance, so that the register
// budget of those stages does not lower the occupancy of the 2-3-5 lengths)
template <typename T, int EPT, bool BIG>
__device__ __forceinline__ void fft_lines(cplx<T>* buf, int cstride, int L, const AxisPlan& ap, int sgn) {
  const cplx<T>* tw = (const cplx<T>*)ap.tw;
  int Ns = 1;
  for (int s = 0; s < ap.nrad; ++s) {
    const int r = ap.rad[s];
    if (r == 4) fft_stage<T, 4, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else if (r == 2) fft_stage<T, 2, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else if (r == 3) fft_stage<T, 3, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else if (!BIG || r == 5) fft_stage<T, 5, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    else if constexpr (BIG) {
      if (r == 7) fft_stage<T, 7, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
      else if (r == 11) fft_stage<T, 11, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
      else fft_stage<T, 13, EPT>(buf, cstride, L, ap.n, Ns, sgn, tw);
    }
    Ns *= r;
  }
}

__host__ __device__ inline bool plan_has_big_radix(const AxisPlan& ap) {
  for (int s = 0; s < ap.nrad; ++s)
    if (ap.rad[s] > 5) return true;
  return false;
}

// FFT direction of each (type, forward/inverse): -1 = e^{-i}, +1 = e^{+i}
__device__ __forceinline__ int fft_sign(int type, int inv) {
  if (!inv) return (type == T_DCT3 || type == T_DST3) ? +1 : -1;
  return (type == T_DFT) ? +1 : -1;
}

// Symbol of the Paux stencil for component c from per-axis s = sin^2(theta/2),
// q = cos^2(theta/2): M = 4 sum_J a_J (s_J q_K q_L + q_J s_K s_L) -- the factored form of
// d + 4 (e_xy Cx Cy + e_xz Cx Cz + e_yz Cy Cz), exact at theta = 0 and (pi, pi, pi).
// HEX1 (hex = 1) keeps the first term of each pair only: M = 4 sum_J a_J s_J q_K q_L, the
// centre-gradient symbol, which also vanishes on the hourglass lines (two angles equal to pi).
__device__ __forceinline__ double paux_symbol(const double a[3], double sx, double qx, double sy, double qy,
                                              double sz, double qz, int hex) {
  const double h = hex ? 0.0 : 1.0;
  return 4.0 * (a[0] * (sx * qy * qz + h * qx * sy * sz) + a[1] * (sy * qx * qz + h * qy * sx * sz) +
                a[2] * (sz * qx * qy + h * qz * sx * sy));
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


template <typename T, int EPT, bool BIG>
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
          if (a.st->accel_ok) {
            const T k = (T)a.st->gamma[0] * a.dY[0][addr] + (T)a.st->gamma[1] * a.dY[1][addr] +
                        (T)a.st->gamma[2] * a.dY[2][addr];
            v = v - k;
            a.de[addr] = k;   // c = p - e, stored only when it is not 0
          }
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
    fft_lines<T, EPT, BIG>(cb, cstride, L, a.ap, sg);
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
        const double M = paux_symbol(a.g.ac[c], sxT[mx], qxT[mx], syT[my], qyT[my], szT[m], qzT[m], a.g.hex);
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
    fft_lines<T, EPT, BIG>(cb, cstride, L, a.ap, sg);
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
  // stores of S or c would otherwise hold back the next loads: the pointers may alias).
  // fetch(off, k) returns the value to transform and sets k, the value keep(off, v, k) may store.
  auto gather = [&](auto fetch, auto keep) {
    by_map([&](auto mk) {
      T vals[NB + 1], kv[NB + 1];
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        kv[i] = T(0);
        vals[i] = ((int)l < nl) ? fetch(l * ls + m * es, kv[i]) : T(0);
      }
      kv[NB] = T(0);
      vals[NB] = tail_ok ? fetch(tail_off, kv[NB]) : T(0);
#pragma unroll
      for (int i = 0; i < NB; ++i) {
        unsigned l, m;
        body(mk, i, l, m);
        if ((int)l < nl) keep(l * ls + m * es, vals[i], kv[i]);
      }
      if (tail_ok) keep(tail_off, vals[NB], kv[NB]);
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
        [&](unsigned off, T&) -> T {
          if (acc_ok) {
            double s = al0 * ((double)S0[off] + (double)R0[off]);
            s += al1 * ((double)S1[off] + (double)R1[off]);
            s += al2 * ((double)S2[off] + (double)R2[off]);
            s += al3 * ((double)S3[off] + (double)R3[off]);
            return (T)s;
          }
          return X[off];
        },
        [&](unsigned off, T v, T) {
          if (store_s) Sout[off] = v;
        });
  } else if (a.src == SRC_DELTA) {
    const T* pcur = a.dp2[a.st->it & 1] + base;
    const int acc_ok = a.st->accel_ok;
    const T g0 = acc_ok ? (T)a.st->gamma[0] : T(0), g1 = acc_ok ? (T)a.st->gamma[1] : T(0),
            g2 = acc_ok ? (T)a.st->gamma[2] : T(0);
    const T *y0 = a.dY[0] + base, *y1 = a.dY[1] + base, *y2 = a.dY[2] + base;
    T* de = a.de + base;
    // e = p - c with c = sum_j gamma_j dY_j; c is stored (only when it is not 0): the next
    // residual pass forms R = dY + c, with no cancellation against |p|.  p, dY and c are
    // touched once here; on fields larger than the last-level cache (nontemp) non-temporal
    // loads and store keep that cache for the transform buffer t, which the y forward pass
    // reads next (0.150 -> 0.115 ms at 256^3; at 128^3, where everything fits, they made this
    // pass slower)
    if (a.nontemp) {
      gather(
          [&](unsigned off, T& k) -> T {
            T v = __builtin_nontemporal_load(pcur + off);
            if (acc_ok) {
              k = g0 * __builtin_nontemporal_load(y0 + off) + g1 * __builtin_nontemporal_load(y1 + off) +
                  g2 * __builtin_nontemporal_load(y2 + off);
              v = v - k;
            }
            return v;
          },
          [&](unsigned off, T, T k) {
            if (acc_ok) __builtin_nontemporal_store(k, de + off);
          });
    } else {
      gather(
          [&](unsigned off, T& k) -> T {
            T v = pcur[off];
            if (acc_ok) {
              k = g0 * y0[off] + g1 * y1[off] + g2 * y2[off];
              v = v - k;
            }
            return v;
          },
          [&](unsigned off, T, T k) {
            if (acc_ok) de[off] = k;
          });
    }
  } else {
    const T* in = a.in + base;
    gather([&](unsigned off, T&) -> T { return in[off]; }, [&](unsigned, T, T) {});
  }
  __syncthreads();
  const int inv_first = (a.mode == PASS_INV);
  {
    auto ld = [&](int l, int k) { return pre_ct<T, NF>(type, inv_first, rb + l * RS, k, tw); };
    if (fft_sign(type, inv_first) < 0) fft_ct<T, NF, -1, NT>(cb, CS, tw, ld);
    else fft_ct<T, NF, +1, NT>(cb, CS, tw, ld);
  }
  if (a.mode == PASS_FWD_GREEN_INV) {
    // (z lines: block = x chunk bxi of the y plane byi); symbol tables in T
    const T* tab;
    if constexpr (sizeof(T) == 4) tab = a.cosT32;
    else tab = a.cosT;
    const T* sxT = tab + ((c * 3 + 0) * 2 + 0) * a.maxN;
    const T* qxT = tab + ((c * 3 + 0) * 2 + 1) * a.maxN;
    const T* syT = tab + ((c * 3 + 1) * 2 + 0) * a.maxN;
    const T* qyT = tab + ((c * 3 + 1) * 2 + 1) * a.maxN;
    const T* szT = tab + ((c * 3 + 2) * 2 + 0) * a.maxN;
    const T* qzT = tab + ((c * 3 + 2) * 2 + 1) * a.maxN;
    // symbol in the transform's precision: M = qz A(x, y) + sz B(x, y) with
    // A = 4 (a0 sx qy + a1 sy qx + a2 sx sy), B = 4 (a0 qx sy + a1 qy sx + a2 qx qy)
    const T sy = (T)syT[(int)byi], qy = (T)qyT[(int)byi];
    const T a0 = (T)a.g.ac[c][0], a1 = (T)a.g.ac[c][1], a2 = (T)a.g.ac[c][2];
    // the second-tetrahedron terms of the TETRA2 symbol; 0 for HEX1 (centre gradient)
    const T e0 = a.g.hex ? T(0) : a0, e1 = a.g.hex ? T(0) : a1, e2 = a.g.hex ? T(0) : a2;
    const T thr = (T)a.thr[c];
    const unsigned x0 = bxi * LB;
    auto green = [&](unsigned l, unsigned m) -> T {
      const T v = post_ct<T, NF>(type, 0, cb + l * CS, m, tw);
      const T sx = (T)sxT[x0 + l], qx = (T)qxT[x0 + l];
      const T A = T(4) * (a0 * sx * qy + a1 * sy * qx + e2 * sx * sy);
      const T B = T(4) * (e0 * qx * sy + e1 * qy * sx + a2 * qx * qy);
      const T M = (T)qzT[m] * A + (T)szT[m] * B;
      if constexpr (sizeof(T) == 4) {
        // FP32: times the hardware reciprocal (1 ulp) in place of the IEEE division sequence
        return (M > thr) ? v * __builtin_amdgcn_rcpf(M) : T(0);
      } else {
        return (M > thr) ? v / M : T(0);
      }
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
  const bool big = plan_has_big_radix(a.ap);
  if (dtt_ept(ept, a.ap) <= 8) {
    if (big) hipLaunchKernelGGL((k_dtt<T, 8, true>), dim3((unsigned)nb, 3), dim3(kBlock), sm, s, a);
    else hipLaunchKernelGGL((k_dtt<T, 8, false>), dim3((unsigned)nb, 3), dim3(kBlock), sm, s, a);
  } else {
    if (big) hipLaunchKernelGGL((k_dtt<T, 16, true>), dim3((unsigned)nb, 3), dim3(kBlock), sm, s, a);
    else hipLaunchKernelGGL((k_dtt<T, 16, false>), dim3((unsigned)nb, 3), dim3(kBlock), sm, s, a);
  }
}

}  // namespace fftc
