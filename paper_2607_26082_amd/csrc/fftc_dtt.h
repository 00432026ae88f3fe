// Per-axis discrete trigonometric transforms with compile-time lengths (CDNA4).
//
// Every transform of Table 2 (DCT1, DCT3, DST1, DST3 and their inverses DCT1, DCT2,
// DST1, DST2) is computed with one complex FFT of length n (the voxel count of the
// axis) plus O(n) pre- and post-processing:
//   DCT1 / DST1: real FFT of the even / odd 2n-periodic extension, packed as n complex
//                points (even samples in the real part, odd samples in the imaginary part)
//   DCT2 / DCT3: reordering of the samples (even indices ascending, odd descending) and a
//                quarter-wave twiddle e^{-/+ i pi k / 2n}
//   DST2 / DST3: DCT2 / DCT3 with alternating signs and reversed indices.
// The FFT runs in registers, two radix passes (8, 12 or 16 points per thread) joined by
// one LDS exchange, Stockham order.  One block transforms LB lines of one component.
#pragma once

#include "fftc_internal.h"

namespace fftc {

template <typename T>
struct cplx {
  T re, im;
};
template <typename T>
__device__ __forceinline__ cplx<T> cmul(cplx<T> a, cplx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ cplx<T> cconj(cplx<T> a) { return {a.re, -a.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> cadd(cplx<T> a, cplx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ cplx<T> csub(cplx<T> a, cplx<T> b) { return {a.re - b.re, a.im - b.im}; }

// ---- compile-time cos/sin of 2 pi m / R (octant reduction + Taylor series) ----
constexpr double ct_poly_cos(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
constexpr double ct_poly_sin(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 14; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
// cos and sin of 2 pi m / R for integer m, R
constexpr double ct_cos(long m, long R) {
  m = ((m % R) + R) % R;
  // angle = 2 pi m / R in [0, 2 pi); reduce with 8 m / R octants
  const double PI = 3.14159265358979323846264338327950288;
  const long e = 8 * m;
  const long oct = e / R;            // 0..7
  const double rem = (double)(e - oct * R) / (double)R;   // [0, 1) fraction of an octant
  const double a = rem * PI / 4.0;
  const double c = ct_poly_cos(a), s = ct_poly_sin(a);
  const double c2 = ct_poly_cos(PI / 4.0 - a), s2 = ct_poly_sin(PI / 4.0 - a);
  switch (oct) {
    case 0: return c;
    case 1: return s2;
    case 2: return -s;
    case 3: return -c2;
    case 4: return -c;
    case 5: return -s2;
    case 6: return s;
    default: return c2;
  }
}

// ---- small DFTs in registers, sign SGN (-1 forward, +1 backward) ----
template <typename T, int R, int SGN>
__device__ __forceinline__ void sdft(cplx<T> (&a)[R]) {
  if constexpr (R == 1) {
  } else if constexpr (R == 2) {
    const cplx<T> t0 = cadd(a[0], a[1]), t1 = csub(a[0], a[1]);
    a[0] = t0;
    a[1] = t1;
  } else if constexpr (R == 3) {
    const T c1 = T(-0.5), s1 = T(SGN) * T(0.86602540378443864676);
    const cplx<T> sum = cadd(a[1], a[2]), dif = csub(a[1], a[2]);
    const cplx<T> m = {a[0].re + c1 * sum.re, a[0].im + c1 * sum.im};
    const cplx<T> rot = {-s1 * dif.im, s1 * dif.re};
    a[0] = cadd(a[0], sum);
    a[1] = cadd(m, rot);
    a[2] = csub(m, rot);
  } else if constexpr (R == 4) {
    const cplx<T> t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
    const cplx<T> t2 = cadd(a[1], a[3]), d = csub(a[1], a[3]);
    const cplx<T> t3 = {-T(SGN) * d.im, T(SGN) * d.re};
    a[0] = cadd(t0, t2);
    a[2] = csub(t0, t2);
    a[1] = cadd(t1, t3);
    a[3] = csub(t1, t3);
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);
    const T s1 = T(SGN) * T(0.95105651629515357212), s2 = T(SGN) * T(0.58778525229247312917);
    const cplx<T> b1 = cadd(a[1], a[4]), b2 = cadd(a[2], a[3]);
    const cplx<T> d1 = csub(a[1], a[4]), d2 = csub(a[2], a[3]);
    const cplx<T> m1 = {a[0].re + c1 * b1.re + c2 * b2.re, a[0].im + c1 * b1.im + c2 * b2.im};
    const cplx<T> m2 = {a[0].re + c2 * b1.re + c1 * b2.re, a[0].im + c2 * b1.im + c1 * b2.im};
    const cplx<T> r1 = {-(s1 * d1.im + s2 * d2.im), s1 * d1.re + s2 * d2.re};
    const cplx<T> r2 = {-(s2 * d1.im - s1 * d2.im), s2 * d1.re - s1 * d2.re};
    a[0] = {a[0].re + b1.re + b2.re, a[0].im + b1.im + b2.im};
    a[1] = cadd(m1, r1);
    a[4] = csub(m1, r1);
    a[2] = cadd(m2, r2);
    a[3] = csub(m2, r2);
  } else {
    // R = A * B, A in {4, 2, 3}: X[k1 + A k2] = sum_q W_B^{q k2} W_R^{q k1} sum_r x[q + B r] W_A^{r k1}
    constexpr int A = (R % 4 == 0) ? 4 : ((R % 2 == 0) ? 2 : ((R % 3 == 0) ? 3 : 5));
    constexpr int B = R / A;
    cplx<T> t[R];
#pragma unroll
    for (int q = 0; q < B; ++q) {
      cplx<T> s[A];
#pragma unroll
      for (int r = 0; r < A; ++r) s[r] = a[q + B * r];
      sdft<T, A, SGN>(s);
#pragma unroll
      for (int k1 = 0; k1 < A; ++k1) {
        if (q * k1 == 0) {
          t[q + B * k1] = s[k1];
        } else {
          const cplx<T> w = {T(ct_cos(q * k1, R)), T(SGN) * T(ct_cos(q * k1 * 4 - R, 4 * R))};
          t[q + B * k1] = cmul(s[k1], w);
        }
      }
    }
#pragma unroll
    for (int k1 = 0; k1 < A; ++k1) {
      cplx<T> s[B];
#pragma unroll
      for (int q = 0; q < B; ++q) s[q] = t[q + B * k1];
      sdft<T, B, SGN>(s);
#pragma unroll
      for (int k2 = 0; k2 < B; ++k2) a[k1 + A * k2] = s[k2];
    }
  }
}

// FFT plan of each supported length: first radix R1 (one butterfly per thread), second R2
template <int NF>
struct FftPlan;
template <> struct FftPlan<16> { static constexpr int R1 = 4, R2 = 4; };
template <> struct FftPlan<32> { static constexpr int R1 = 8, R2 = 4; };
template <> struct FftPlan<48> { static constexpr int R1 = 12, R2 = 4; };
template <> struct FftPlan<64> { static constexpr int R1 = 8, R2 = 8; };
template <> struct FftPlan<96> { static constexpr int R1 = 12, R2 = 8; };
template <> struct FftPlan<128> { static constexpr int R1 = 16, R2 = 8; };
template <> struct FftPlan<256> { static constexpr int R1 = 16, R2 = 16; };

// ---- pre / post processing with compile-time length ----
template <typename T, int NF>
__device__ __forceinline__ cplx<T> pre_ct(int type, int inv, const T* x, int k, const cplx<T>* tw) {
  constexpr int n = NF;
  if (type == T_DCT1) {
    const int j0 = 2 * k, j1 = 2 * k + 1;
    return {x[j0 <= n ? j0 : 2 * n - j0], x[j1 <= n ? j1 : 2 * n - j1]};
  }
  if (type == T_DST1) {
    const int j0 = 2 * k, j1 = 2 * k + 1;
    const T a = (j0 == 0 || j0 == n) ? T(0) : (j0 < n ? x[j0] : -x[2 * n - j0]);
    const T b = (j1 == n) ? T(0) : (j1 < n ? x[j1] : -x[2 * n - j1]);
    return {a, b};
  }
  if (!inv) {
    T a, b;
    if (type == T_DCT3) {
      a = x[k];
      b = (k == 0) ? T(0) : x[n - k];
    } else {
      a = x[n - k];
      b = (k == 0) ? T(0) : x[k];
    }
    return cmul(cconj(tw[k]), cplx<T>{a, -b});
  }
  constexpr int h = (n + 1) / 2;
  if (k < h) return {x[2 * k], T(0)};
  const T v = x[2 * n - 1 - 2 * k];
  return {type == T_DST3 ? -v : v, T(0)};
}

// LDS index of complex element i of a line: one padding slot after every R1 elements, so
// that the strided accesses of both FFT passes and of the post-processing fall on
// distinct LDS banks.
template <int NF>
__device__ __forceinline__ unsigned cpad(unsigned i) { return i + i / (unsigned)FftPlan<NF>::R1; }

template <typename T, int NF>
__device__ __forceinline__ T post_ct(int type, int inv, const cplx<T>* Zb, int m, const cplx<T>* tw) {
  constexpr int n = NF;
  auto Z = [&](int i) { return Zb[cpad<NF>(i)]; };
  if (type == T_DCT1 || type == T_DST1) {
    if (type == T_DST1 && (m == 0 || m == n)) return T(0);
    const cplx<T> Zm = Z(m == n ? 0 : m);
    const cplx<T> Zc = cconj(Z(m == 0 ? 0 : n - m));
    const cplx<T> E = {(Zm.re + Zc.re) * T(0.5), (Zm.im + Zc.im) * T(0.5)};
    const cplx<T> D = {(Zm.re - Zc.re) * T(0.5), (Zm.im - Zc.im) * T(0.5)};
    const cplx<T> O = {D.im, -D.re};
    const cplx<T> Y = cadd(E, cmul(tw[2 * m], O));
    const T s = inv ? T(1.0 / (2.0 * n)) : T(1);
    return (type == T_DCT1 ? Y.re : -Y.im) * s;
  }
  if (!inv) {
    if (m >= n) return T(0);
    const int hh = (m & 1) ? (n - 1 - (m - 1) / 2) : (m / 2);
    const T v = Z(hh).re;
    return (type == T_DST3 && (m & 1)) ? -v : v;
  }
  if (type == T_DCT3) {
    if (m >= n) return T(0);
    return cmul(tw[m], Z(m)).re * T(1.0 / n);
  }
  if (m == 0) return T(0);
  const int kk = n - m;
  return cmul(tw[kk], Z(kk)).re * T(1.0 / n);
}

// Complex FFT of LB lines of length NF held in LDS (cb, line stride CS); the first pass
// reads its inputs through `load(l, k)` (pre-processing) instead of from cb.  On return
// the result is in cb in natural order.  tw: e^{-2 pi i s / 4NF} for s = 0 .. 2 NF.  Must be
// called by all NT threads.
template <typename T, int NF, int SGN, int NT, typename Loader>
__device__ __forceinline__ void fft_ct(cplx<T>* cb, int CS, const cplx<T>* __restrict__ tw, Loader load) {
  constexpr int R1 = FftPlan<NF>::R1, R2 = FftPlan<NF>::R2;
  constexpr int TL = NF / R1;          // threads per line
  constexpr int LB = NT / TL;          // lines per block
  constexpr int B2 = NF / R2;          // butterflies per line in pass 2
  constexpr int W2 = (B2 + TL - 1) / TL;
  const int tid = threadIdx.x;
  const int l = tid / TL, t = tid - l * TL;
  // pass 1: butterfly j = t, inputs k = t + q * TL, no twiddle (Ns = 1)
  cplx<T> a[R1];
#pragma unroll
  for (int q = 0; q < R1; ++q) a[q] = load(l, t + q * TL);
  sdft<T, R1, SGN>(a);
  __syncthreads();   // all inputs read (cb may alias the input staging)
#pragma unroll
  for (int q = 0; q < R1; ++q) cb[l * CS + cpad<NF>(t * R1 + q)] = a[q];
  __syncthreads();
  // pass 2: Ns = R1, butterflies j = t + w * TL
  cplx<T> b[W2][R2];
#pragma unroll
  for (int w = 0; w < W2; ++w) {
    const int j = t + w * TL;
    if (j < B2) {
      const int kk = j % R1;
#pragma unroll
      for (int q = 0; q < R2; ++q) {
        cplx<T> v = cb[l * CS + cpad<NF>(j + q * B2)];
        if (q > 0) {
          // W_{R1 R2}^{q kk} = e^{SGN 2 pi i q kk / NF}; the table holds e^{-2 pi i s / 4NF}
          // for s <= 2 NF only, and q kk < NF: past NF / 2 use e^{-i pi} = -1.  At kk = 0 the
          // factor is the table's exact (1, 0), so no lane takes a separate path.
          const int jj = q * kk;
          const bool hi = jj > NF / 2;
          cplx<T> f = tw[4 * (hi ? jj - NF / 2 : jj)];
          if (hi) f = {-f.re, -f.im};
          if (SGN > 0) f.im = -f.im;
          v = cmul(v, f);
        }
        b[w][q] = v;
      }
      sdft<T, R2, SGN>(b[w]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < W2; ++w) {
    const int j = t + w * TL;
    if (j < B2) {
      const int kk = j % R1;
      const int base = (j / R1) * R1 * R2 + kk;
#pragma unroll
      for (int q = 0; q < R2; ++q) cb[l * CS + cpad<NF>(base + q * R1)] = b[w][q];
    }
  }
  __syncthreads();
  (void)LB;
}

template <int NF, int NTHREADS>
struct DttShape {
  static constexpr int R1 = FftPlan<NF>::R1;
  static constexpr int TL = NF / R1;
  static constexpr int NT = NTHREADS;
  static constexpr int LB = NT / TL;
  static constexpr int NN = NF + 1;     // nodes on a non-periodic line
  static constexpr int CS = NF + NF / R1 + 1;   // complex line stride in LDS (padded, see cpad)
  static constexpr int RS = NF + 1;     // real line stride in LDS (staging aliases the complex buffer)
};

}  // namespace fftc
