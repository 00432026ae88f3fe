// Warm-start network: input channels, forward, backward and Adam on gfx950.
//
// The GEMM-shaped steps use v_mfma_f32_16x16x16_bf16 (BF16 operands, FP32
// accumulation).  Operand layout of that instruction for a 64-lane wave, with
// lane = r + 16 q (r < 16, q < 4) and element e < 4 of the 4-vector:
//   A (16 x 16, row i, column k):  i = r, k = 4 q + e
//   B (16 x 16, row k, column j):  k = 4 q + e, j = r
//   D (16 x 16 FP32, row i, col j): i = 4 q + e, j = r
// The contractions of the network:
//   k_gemm   out[node][o] = sum_k phi(node, k) P[o][k] + sum_c X[node][c] Q[o][c] + bias[o]
//            (rows = 16 nodes per tile; the cosine basis phi is formed on the fly
//            from per-axis tables in LDS), with a fused epilogue (GELU, or the
//            GELU derivative of a stored pre-activation);
//   k_reduce R[row][col] = sum_node L(node, row) X(node, col) (K = nodes, L an
//            activation), written as per-wave partials that k_sum_groups and k_sum
//            add in a fixed order;
//   k_ana_*  the analysis onto the cosine modes, sum_node phi_k(node) X(node, c),
//            separably: one axis at a time (x, then y, then z) in FP32.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>

#include "../../include/fftc_nn.h"
#include "fftc_nn_internal.h"

namespace nnk {

constexpr int kW = FFTC_NN_WIDTH;     // 32
constexpr int kH = FFTC_NN_HIDDEN;    // 64
constexpr int kCh = FFTC_NN_CHANNELS; // 16
constexpr int kCin = 12;
constexpr int kCout = 3;
constexpr int kMaxN = 257;
constexpr int kMaxM = 6;
constexpr int kKPMax = 224;                 // 6^3 = 216 modes padded to 16
constexpr int kTabMax = 3 * kMaxN * kMaxM;  // cosine tables, floats
constexpr int kRedGrid = 256;               // workgroups of a reduction
constexpr int kSumGroup = 32;               // per-wave partials summed per group (first pass)
constexpr int kSumGroupsMax = (4 * kRedGrid + kSumGroup - 1) / kSumGroup;
constexpr int kPartCols = kKPMax * kW;      // largest partial (rows x cols) per wave
constexpr int kGemmGrid = 1024;
constexpr int kHeadBlock = 256;

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma16(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

__device__ __host__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

struct Dims {
  int N[3];
  int Nn;
  int m, M3, KP, ksteps;
};

// --------------------------------------------------------------------------
// GEMM over node tiles
// --------------------------------------------------------------------------

enum { EPI_STORE = 0, EPI_GELU = 1, EPI_GELU_Z = 2, EPI_DGELU = 3 };

// Mode k of the m^3 cosine basis as packed per-axis indices kx | ky << 8 | kz << 16, or -1
// for the padding modes k >= m^3 (built once per block; the basis loops then need no
// division by the runtime m).
__device__ __forceinline__ void mode_table(int* sK, int KP, int m, int M3) {
  for (int k = threadIdx.x; k < KP; k += blockDim.x)
    sK[k] = k < M3 ? ((k % m) | (((k / m) % m) << 8) | ((k / (m * m)) << 16)) : -1;
}

struct GemmArgs {
  Dims d;
  const uint16_t* x;     // [Nn][KX]
  const uint16_t* q;     // QT ? [KX][NO] : [NO][KX]
  const uint16_t* p;     // [NO][KP] basis coefficients (BASIS only)
  const float* bias;     // [NO] or null
  const float* tab;      // cosine tables x | y | z, each [N][m]
  const uint16_t* zaux;  // [Nn][NO] pre-activation (EPI_DGELU)
  uint16_t* out;         // [Nn][NO]
  uint16_t* zout;        // [Nn][NO] (EPI_GELU_Z)
};

template <int NO, int KX, bool BASIS, int EPI, bool QT>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs a) {
  __shared__ __align__(16) uint16_t sQ[NO * KX];
  __shared__ __align__(16) uint16_t sP[BASIS ? NO * kKPMax : 4];
  __shared__ float sBias[NO];
  __shared__ float sT[BASIS ? kTabMax : 1];
  __shared__ int sK[BASIS ? kKPMax : 1];
  const int tid = threadIdx.x;
  for (int i = tid; i < NO * KX; i += 256) {
    const int o = i / KX, c = i % KX;
    sQ[i] = QT ? a.q[c * NO + o] : a.q[i];
  }
  for (int i = tid; i < NO; i += 256) sBias[i] = a.bias ? a.bias[i] : 0.0f;
  const int KP = a.d.KP, m = a.d.m, M3 = a.d.M3;
  const int Nx = a.d.N[0], Ny = a.d.N[1];
  if (BASIS) {
    for (int i = tid; i < NO * KP; i += 256) sP[i] = a.p[i];
    const int nt = (a.d.N[0] + a.d.N[1] + a.d.N[2]) * m;
    for (int i = tid; i < nt; i += 256) sT[i] = a.tab[i];
    mode_table(sK, KP, m, M3);
  }
  __syncthreads();
  const int lane = tid & 63, w = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int Nn = a.d.Nn;
  const int ntiles = (Nn + 15) >> 4;
  for (int tile = blockIdx.x * 4 + w; tile < ntiles; tile += gridDim.x * 4) {
    const int node = tile * 16 + r;
    const bool valid = node < Nn;
    f4 acc[NO / 16];
#pragma unroll
    for (int t = 0; t < NO / 16; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    if (BASIS) {
      const int x = node % Nx, y = (node / Nx) % Ny, z = node / (Nx * Ny);
      const int tx = x * m, ty = (Nx + y) * m, tz = (Nx + Ny + z) * m;
      for (int ks = 0; ks < a.d.ksteps; ++ks) {
        s4 av;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int kk = sK[ks * 16 + q * 4 + e];
          float v = 0.0f;
          if (valid && kk >= 0) v = sT[tz + (kk >> 16)] * sT[ty + ((kk >> 8) & 255)] * sT[tx + (kk & 255)];
          av[e] = (short)f2bf(v);
        }
#pragma unroll
        for (int t = 0; t < NO / 16; ++t) {
          const s4 bv = *(const s4*)&sP[(t * 16 + r) * KP + ks * 16 + q * 4];
          acc[t] = mfma16(av, bv, acc[t]);
        }
      }
    }
#pragma unroll
    for (int ks = 0; ks < KX / 16; ++ks) {
      s4 av = s4{0, 0, 0, 0};
      if (valid) av = *(const s4*)&a.x[(size_t)node * KX + ks * 16 + q * 4];
#pragma unroll
      for (int t = 0; t < NO / 16; ++t) {
        const s4 bv = *(const s4*)&sQ[(t * 16 + r) * KX + ks * 16 + q * 4];
        acc[t] = mfma16(av, bv, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < NO / 16; ++t) {
      const int col = t * 16 + r;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int nd = tile * 16 + q * 4 + e;
        if (nd >= Nn) continue;
        const size_t o = (size_t)nd * NO + col;
        const float v = acc[t][e] + sBias[col];
        if (EPI == EPI_STORE) {
          a.out[o] = f2bf(v);
        } else if (EPI == EPI_GELU || EPI == EPI_GELU_Z) {
          if (EPI == EPI_GELU_Z) a.zout[o] = f2bf(v);
          a.out[o] = f2bf(gelu(v));
        } else {
          a.out[o] = f2bf(v * gelu_grad(bf2f(a.zaux[o])));
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// reductions over nodes
// --------------------------------------------------------------------------

struct RedArgs {
  Dims d;
  const uint16_t* l;   // [Nn][RL] row source (activation rows)
  const uint16_t* x;   // [Nn][C]
  float* part;         // [waves][RL][CP]
};

// R[row][col] = sum_node l[node][row] x[node][col], CP = C + ONES (the ones column sums the rows).
template <int RL, int C, bool ONES>
__global__ __launch_bounds__(256) void k_reduce(RedArgs a) {
  constexpr int CT = C / 16 + (ONES ? 1 : 0);
  constexpr int RT = RL / 16;
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int r = lane & 15, q = lane >> 4;
  const int Nn = a.d.Nn;
  f4 acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int nchunks = (Nn + 15) >> 4;
  for (int chunk = blockIdx.x * 4 + w; chunk < nchunks; chunk += gridDim.x * 4) {
    int nd[4];
    bool ok[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      nd[e] = chunk * 16 + q * 4 + e;
      ok[e] = nd[e] < Nn;
    }
    s4 bv[CT];
#pragma unroll
    for (int ct = 0; ct < C / 16; ++ct)
#pragma unroll
      for (int e = 0; e < 4; ++e) bv[ct][e] = ok[e] ? (short)a.x[(size_t)nd[e] * C + ct * 16 + r] : (short)0;
    if (ONES) {
#pragma unroll
      for (int e = 0; e < 4; ++e) bv[CT - 1][e] = (ok[e] && r == 0) ? (short)0x3f80 : (short)0;
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      s4 av;
#pragma unroll
      for (int e = 0; e < 4; ++e) av[e] = ok[e] ? (short)a.l[(size_t)nd[e] * RL + rt * 16 + r] : (short)0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) acc[rt][ct] = mfma16(av, bv[ct], acc[rt][ct]);
    }
  }
  constexpr int CP = C + (ONES ? 1 : 0);
  const size_t wg = (size_t)blockIdx.x * 4 + w;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int col = ct * 16 + r;
      if (col < CP) {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int row = rt * 16 + q * 4 + e;
          a.part[(wg * RL + row) * CP + col] = acc[rt][ct][e];
        }
      }
    }
  }
}

// Fixed-order sum of the per-wave partials, in two passes so that many waves share the
// work: k_sum_groups adds each run of kSumGroup consecutive waves (grid.y = group, one
// thread per output), k_sum adds the group sums in order; col < ncols goes to
// dst[row][col] (leading dimension ldd), col == bias_col to dst_bias[row].
__global__ void k_sum_groups(const float* part, int waves, int RCP, double* grp) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= RCP) return;
  const int w0 = (int)blockIdx.y * kSumGroup;
  const int w1 = min(waves, w0 + kSumGroup);
  double s = 0.0;
  for (int w = w0; w < w1; ++w) s += part[(size_t)w * RCP + i];
  grp[(size_t)blockIdx.y * RCP + i] = s;
}

__global__ void k_sum(const double* grp, int groups, int R, int CP, int rows, float scale, float* dst, int ldd,
                      int ncols, float* dst_bias, int bias_col) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= R * CP) return;
  const int row = i / CP, col = i % CP;
  if (row >= rows) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += grp[(size_t)g * R * CP + i];
  const float v = (float)(s * scale);
  if (col < ncols) dst[row * ldd + col] = v;
  else if (col == bias_col && dst_bias) dst_bias[row] = v;
}

// --------------------------------------------------------------------------
// separable analysis onto the cosine modes
// --------------------------------------------------------------------------
// dst[k][c] = scale sum_node phi_k(node) X[node][c] with phi_k(x, y, z) = cx(x, kx) cy(y, ky)
// cz(z, kz), k = kx + m (ky + m kz): one axis at a time, each sum in a fixed order, FP32.
// Rows KP > k >= m^3 of dst are zero.

// x: one block per (y, z) line: A1[line][kx][c] = sum_x cx(x, kx) X[(x, y, z)][c]
__global__ __launch_bounds__(256) void k_ana_x(Dims d, const float* tab, const uint16_t* X, float* A1) {
  __shared__ uint16_t sX[kMaxN * kW];
  __shared__ float sC[kMaxN * kMaxM];
  const int Nx = d.N[0], m = d.m, line = blockIdx.x;
  const uint16_t* row = X + (size_t)line * Nx * kW;
  for (int i = threadIdx.x; i < Nx * kW; i += blockDim.x) sX[i] = row[i];
  for (int i = threadIdx.x; i < Nx * m; i += blockDim.x) sC[i] = tab[i];
  __syncthreads();
  const int t = threadIdx.x;
  if (t >= m * kW) return;
  const int kx = t / kW, c = t % kW;
  float s = 0.0f;
  for (int x = 0; x < Nx; ++x) s += sC[x * m + kx] * bf2f(sX[x * kW + c]);
  A1[(size_t)line * m * kW + t] = s;
}

// y: one block per (z, ky): A2[z][ky][kx][c] = sum_y cy(y, ky) A1[(y, z)][kx][c]
__global__ __launch_bounds__(256) void k_ana_y(Dims d, const float* tab, const float* A1, float* A2) {
  const int Nx = d.N[0], Ny = d.N[1], m = d.m;
  const int z = blockIdx.x / m, ky = blockIdx.x % m, t = threadIdx.x;
  if (t >= m * kW) return;
  const float* cy = tab + Nx * m;
  float s = 0.0f;
  for (int y = 0; y < Ny; ++y) s += cy[y * m + ky] * A1[((size_t)z * Ny + y) * m * kW + t];
  A2[((size_t)z * m + ky) * m * kW + t] = s;
}

// z: one block per (kz, ky): dst[k][c] = scale sum_z cz(z, kz) A2[z][ky][kx][c]
__global__ __launch_bounds__(256) void k_ana_z(Dims d, const float* tab, const float* A2, float scale, float* dst,
                                               int ldd) {
  const int Nx = d.N[0], Ny = d.N[1], Nz = d.N[2], m = d.m;
  const int kz = blockIdx.x / m, ky = blockIdx.x % m, t = threadIdx.x;
  if (blockIdx.x == 0)
    for (int i = t; i < (d.KP - d.M3) * kW; i += blockDim.x) dst[(d.M3 + i / kW) * ldd + i % kW] = 0.0f;
  if (t >= m * kW) return;
  const float* cz = tab + (Nx + Ny) * m;
  float s = 0.0f;
  for (int z = 0; z < Nz; ++z) s += cz[z * m + kz] * A2[((size_t)z * m + ky) * m * kW + t];
  const int kx = t / kW, c = t % kW;
  dst[(kx + m * (ky + m * kz)) * ldd + c] = s * scale;
}

// --------------------------------------------------------------------------
// mode mixing
// --------------------------------------------------------------------------

// yh[k][o] = sum_c Ws[k][o][c] xh[k][c]  ->  P[o][k] (BF16, zero for k >= M3)
__global__ void k_mix_fwd(const float* Ws, const float* xh, int M3, int KP, uint16_t* P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kW * KP) return;
  const int o = i / KP, k = i % KP;
  float s = 0.0f;
  if (k < M3)
    for (int c = 0; c < kW; ++c) s += Ws[(k * kW + o) * kW + c] * xh[k * kW + c];
  P[o * KP + k] = f2bf(s);
}

// dxh[k][c] = (1/Nn) sum_o Ws[k][o][c] dyh[k][o]  ->  P[c][k] (BF16)
__global__ void k_mix_bwd_dx(const float* Ws, const float* dyh, int M3, int KP, float inv_nn, uint16_t* P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= kW * KP) return;
  const int c = i / KP, k = i % KP;
  float s = 0.0f;
  if (k < M3)
    for (int o = 0; o < kW; ++o) s += Ws[(k * kW + o) * kW + c] * dyh[k * kW + o];
  P[c * KP + k] = f2bf(s * inv_nn);
}

// dWs[k][o][c] = dyh[k][o] xh[k][c]
__global__ void k_mix_bwd_dw(const float* dyh, const float* xh, int M3, float* dWs) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M3 * kW * kW) return;
  const int k = i / (kW * kW), o = (i / kW) % kW, c = i % kW;
  dWs[i] = dyh[k * kW + o] * xh[k * kW + c];
}

// --------------------------------------------------------------------------
// output layer, loss and its gradient
// --------------------------------------------------------------------------

struct HeadArgs {
  int Nn;
  const float* w2;        // Wp2[3][64] then bp2[3]
  const uint16_t* h;      // [Nn][64]
  float* y;               // [Nn][3] or null
  double* u0;             // [3][Nn] or null
  const double* base;     // [3][Nn] or null: u0 = base + s_u y
  double s_u;
  // training
  const uint16_t* hpre;   // [Nn][64]
  const float* target;    // [3][Nn]
  const float* tinv;      // 1 / sum t^2
  uint16_t* dy16;         // [Nn][16]
  uint16_t* dhpre;        // [Nn][64]
  double* lpart;          // per block
};

template <bool TRAIN>
__global__ __launch_bounds__(kHeadBlock) void k_head(HeadArgs a) {
  __shared__ float sW[kCout * kH + kCout];
  __shared__ double sred[kHeadBlock / 64];
  const int tid = threadIdx.x;
  for (int i = tid; i < kCout * kH + kCout; i += kHeadBlock) sW[i] = a.w2[i];
  __syncthreads();
  const int node = blockIdx.x * kHeadBlock + tid;
  double l = 0.0;
  if (node < a.Nn) {
    float h[kH];
    const uint4* hp = (const uint4*)(a.h + (size_t)node * kH);
#pragma unroll
    for (int v = 0; v < kH / 8; ++v) {
      const uint4 u = hp[v];
      const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        h[v * 8 + 2 * e] = __uint_as_float(wd[e] << 16);
        h[v * 8 + 2 * e + 1] = __uint_as_float(wd[e] & 0xffff0000u);
      }
    }
    float y[kCout];
#pragma unroll
    for (int c = 0; c < kCout; ++c) {
      float s = sW[kCout * kH + c];
#pragma unroll
      for (int j = 0; j < kH; ++j) s += sW[c * kH + j] * h[j];
      y[c] = s;
    }
    if (!TRAIN) {
#pragma unroll
      for (int c = 0; c < kCout; ++c) {
        if (a.y) a.y[(size_t)node * kCout + c] = y[c];
        if (a.u0)
          a.u0[(size_t)c * a.Nn + node] = (a.base ? a.base[(size_t)c * a.Nn + node] : 0.0) + a.s_u * (double)y[c];
      }
    } else {
      const float ti = *a.tinv;
      float dy[kCout];
#pragma unroll
      for (int c = 0; c < kCout; ++c) {
        const float d = y[c] - a.target[(size_t)c * a.Nn + node];
        l += (double)d * d;
        dy[c] = 2.0f * d * ti;
      }
      uint32_t pk[8];
      pk[0] = (uint32_t)f2bf(dy[0]) | ((uint32_t)f2bf(dy[1]) << 16);
      pk[1] = (uint32_t)f2bf(dy[2]);
#pragma unroll
      for (int e = 2; e < 8; ++e) pk[e] = 0u;
      uint4* dp = (uint4*)(a.dy16 + (size_t)node * kCh);
      dp[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
      dp[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
      const uint4* zp = (const uint4*)(a.hpre + (size_t)node * kH);
      uint4* op = (uint4*)(a.dhpre + (size_t)node * kH);
#pragma unroll
      for (int v = 0; v < kH / 8; ++v) {
        const uint4 u = zp[v];
        const uint32_t wd[4] = {u.x, u.y, u.z, u.w};
        uint32_t ow[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          uint16_t hv[2];
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const int j = v * 8 + 2 * e + s;
            const float z = __uint_as_float(s ? (wd[e] & 0xffff0000u) : (wd[e] << 16));
            float g = 0.0f;
#pragma unroll
            for (int c = 0; c < kCout; ++c) g += sW[c * kH + j] * dy[c];
            hv[s] = f2bf(g * gelu_grad(z));
          }
          ow[e] = (uint32_t)hv[0] | ((uint32_t)hv[1] << 16);
        }
        op[v] = make_uint4(ow[0], ow[1], ow[2], ow[3]);
      }
    }
  }
  if (TRAIN) {
    for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off, 64);
    if ((tid & 63) == 0) sred[tid >> 6] = l;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int i = 0; i < kHeadBlock / 64; ++i) s += sred[i];
      a.lpart[blockIdx.x] = s;
    }
  }
}

// per-block sums of t^2 over a [3][Nn] FP32 target
__global__ __launch_bounds__(256) void k_sq_partial(const float* t, long long n, double* part) {
  __shared__ double sred[4];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
    const double v = t[i];
    s += v * v;
  }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// per-block sums of b^2 over the first-iterate channels 9..11 of the input
__global__ __launch_bounds__(256) void k_sq_feat(const uint16_t* feat, int Nn, double* part) {
  __shared__ double sred[4];
  double s = 0.0;
  for (int i = blockIdx.x * 256 + threadIdx.x; i < Nn; i += gridDim.x * 256)
#pragma unroll
    for (int c = 9; c < 12; ++c) {
      const double v = bf2f(feat[(size_t)i * kCh + c]);
      s += v * v;
    }
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sred[0] + sred[1] + sred[2] + sred[3];
}

// single wave: tsum = sum part, tinv = 1 / tsum
__global__ void k_sq_final(const double* part, int nb, double* tsum, float* tinv) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 64) s += part[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (threadIdx.x == 0) {
    *tsum = s;
    *tinv = (float)(1.0 / s);
  }
}

__global__ void k_loss_final(const double* lpart, int nb, const double* tsum, double* loss) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 64) s += lpart[i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (threadIdx.x == 0) *loss = s / *tsum;
}

// --------------------------------------------------------------------------
// optimiser and weight images
// --------------------------------------------------------------------------

__global__ void k_adam(float* p, const float* g, float* mo, float* ve, long long P, float lr, float b1, float b2,
                       float eps, float bc1, float bc2) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= P) return;
  const float gi = g[i];
  const float mi = b1 * mo[i] + (1.0f - b1) * gi;
  const float vi = b2 * ve[i] + (1.0f - b2) * gi * gi;
  mo[i] = mi;
  ve[i] = vi;
  p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
}

struct Offsets {
  long long Wl, bl, blk0, blk_stride, Ws, Wb, cb, Wp1, bp1, Wp2, bp2, total;
};

// BF16 images: Wl as [32][16] (inputs 9..15 zero) | W_b [32][32] per block | Wp1 [64][32]
__global__ void k_images(const float* p, Offsets off, int blocks, uint16_t* img) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int nl = kW * kCh, nb = kW * kW, np = kH * kW;
  if (i < nl) {
    const int o = i / kCh, c = i % kCh;
    img[i] = c < kCin ? f2bf(p[off.Wl + o * kCin + c]) : (uint16_t)0;
    return;
  }
  int j = i - nl;
  if (j < blocks * nb) {
    const int b = j / nb;
    img[i] = f2bf(p[off.blk0 + b * off.blk_stride + off.Wb + j % nb]);
    return;
  }
  j -= blocks * nb;
  if (j < np) img[i] = f2bf(p[off.Wp1 + j]);
}

__global__ void k_zero_f(float* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0f;
}

// --------------------------------------------------------------------------
// input channels
// --------------------------------------------------------------------------

__device__ __forceinline__ void young_poisson(double l, double u, double& E, double& nu) {
  const double den = l + u;
  if (den > 0.0) {
    E = u * (3.0 * l + 2.0 * u) / den;
    nu = l / (2.0 * den);
  } else {
    E = 0.0;
    nu = 0.0;
  }
}

__device__ __forceinline__ double load_lame(const void* p, int fp64, long long i) {
  return fp64 ? ((const double*)p)[i] : (double)((const float*)p)[i];
}

__global__ __launch_bounds__(256) void k_emax_partial(FeatArgs a) {
  __shared__ double sred[4];
  double mx = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < a.Nv; i += (long long)gridDim.x * 256) {
    double E, nu;
    young_poisson(load_lame(a.lam, a.fp64, i), load_lame(a.mu, a.fp64, i), E, nu);
    mx = fmax(mx, E);
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
  if ((threadIdx.x & 63) == 0) sred[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) a.scratch[blockIdx.x] = fmax(fmax(sred[0], sred[1]), fmax(sred[2], sred[3]));
}

__global__ void k_emax_final(FeatArgs a, int nb) {
  double mx = 0.0;
  for (int i = threadIdx.x; i < nb; i += 64) mx = fmax(mx, a.scratch[i]);
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_down(mx, off, 64));
  if (threadIdx.x == 0) a.scratch[256] = mx > 0.0 ? mx : 1.0;
}

__global__ __launch_bounds__(256) void k_features(FeatArgs a) {
  const long long nd = (long long)blockIdx.x * 256 + threadIdx.x;
  if (nd >= a.Nn) return;
  const int x = (int)(nd % a.N[0]), y = (int)((nd / a.N[0]) % a.N[1]), z = (int)(nd / ((long long)a.N[0] * a.N[1]));
  const int X[3] = {x, y, z};
  double Es = 0.0, ns = 0.0;
  int cnt = 0;
  for (int dz = -1; dz <= 0; ++dz)
    for (int dy = -1; dy <= 0; ++dy)
      for (int dx = -1; dx <= 0; ++dx) {
        int v[3] = {x + dx, y + dy, z + dz};
        bool in = true;
        for (int J = 0; J < 3; ++J) {
          if (a.periodic[J]) v[J] = (v[J] + a.n[J]) % a.n[J];
          else if (v[J] < 0 || v[J] >= a.n[J]) in = false;
        }
        if (!in) continue;
        const long long vi = v[0] + (long long)a.n[0] * (v[1] + (long long)a.n[1] * v[2]);
        double E, nu;
        young_poisson(load_lame(a.lam, a.fp64, vi), load_lame(a.mu, a.fp64, vi), E, nu);
        Es += E;
        ns += nu;
        ++cnt;
      }
  float f[kCh];
  for (int c = 0; c < kCh; ++c) f[c] = 0.0f;
  f[0] = (float)(Es / cnt / a.scratch[256]);
  for (int c = 0; c < 3; ++c) f[9 + c] = (float)(a.u1[c * a.Nn + nd] / a.s_u);
  f[1] = (float)(ns / cnt);
  const uint8_t mk = a.mask[nd];
  for (int c = 0; c < 3; ++c) {
    bool fixed = (mk >> c) & 1;
    for (int J = 0; J < 3; ++J) {
      if (a.periodic[J]) continue;
      if (X[J] == 0 && ((a.aface >> (c * 6 + J * 2 + 0)) & 1)) fixed = true;
      if (X[J] == a.n[J] && ((a.aface >> (c * 6 + J * 2 + 1)) & 1)) fixed = true;
    }
    f[2 + c] = fixed ? 1.0f : 0.0f;
  }
  if (a.has_sphere) {
    const int ax = a.face / 2;
    const int idx = (a.face % 2) ? a.n[ax] : 0;
    if (X[ax] == idx) {
      const double ddx = x - a.center[0], ddy = y - a.center[1], ddz = z - a.center[2];
      const double g = sqrt(ddx * ddx + ddy * ddy + ddz * ddz) - a.radius;
      f[8] = (float)tanh(g / (8.0 * a.s_u));
    }
  }
  uint32_t pk[8];
  for (int e = 0; e < 8; ++e) pk[e] = (uint32_t)f2bf(f[2 * e]) | ((uint32_t)f2bf(f[2 * e + 1]) << 16);
  uint4* out = (uint4*)(a.feat + nd * kCh);
  out[0] = make_uint4(pk[0], pk[1], pk[2], pk[3]);
  out[1] = make_uint4(pk[4], pk[5], pk[6], pk[7]);
}

// prescribed values of strong constraints (the mask channel is set by k_features)
__global__ void k_feat_strong(FeatArgs a) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= a.ms) return;
  a.feat[a.snode[e] * kCh + 5 + a.scomp[e]] = f2bf((float)(a.sval[e] / a.s_u));
}

void launch_features(const FeatArgs& a, hipStream_t s) {
  const int nb = (int)std::min<long long>(256, (a.Nv + 255) / 256);
  hipLaunchKernelGGL(k_emax_partial, dim3(nb), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_emax_final, dim3(1), dim3(64), 0, s, a, nb);
  hipLaunchKernelGGL(k_features, dim3((unsigned)((a.Nn + 255) / 256)), dim3(256), 0, s, a);
  if (a.ms > 0) hipLaunchKernelGGL(k_feat_strong, dim3((unsigned)((a.ms + 255) / 256)), dim3(256), 0, s, a);
}

}  // namespace nnk

// ==========================================================================
// C ABI
// ==========================================================================

using namespace nnk;

// Training target of the learned start: t = (u* - u1) / s_u in FP32 (u* a converged solve,
// u1 the first iterate the input channels carry).
__global__ __launch_bounds__(256) void k_target(const double* __restrict__ u, const double* __restrict__ u1, long long n,
                                                double inv_su, float* __restrict__ t) {
  for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    t[e] = (float)((u[e] - u1[e]) * inv_su);
}

struct fftc_nn {
  int m = 6, blocks = 4, M3 = 216, KP = 224, ksteps = 14;
  Offsets off{};
  long long P = 0;
  // state
  float *p = nullptr, *g = nullptr, *mo = nullptr, *ve = nullptr;
  uint16_t* img = nullptr;
  long long img_n = 0;
  int step = 0;
  int state_bound = 0;
  // workspace
  int bound = 0, training = 0;
  Dims d{};
  hipStream_t stream = nullptr;
  float* tab = nullptr;
  uint16_t* xs = nullptr;     // activations x_0..x_B (training) or 2 ping-pong buffers
  uint16_t* zs = nullptr;     // pre-activations z_1..z_B (training)
  uint16_t *h = nullptr, *hpre = nullptr, *dy16 = nullptr, *dhpre = nullptr, *dz = nullptr;
  float *xh = nullptr, *dyh = nullptr, *part = nullptr;
  uint16_t* P16 = nullptr;
  double *dsc = nullptr;      // small FP64 scratch: partials, tsum, loss
  double* grp = nullptr;      // group sums of the reduction partials
  float *ana1 = nullptr, *ana2 = nullptr;   // separable analysis: after x, after y
  float* tinv = nullptr;
  std::string err;
};

namespace {

constexpr size_t kAlign = 256;

size_t al(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

Offsets make_offsets(int M3, int blocks) {
  Offsets o{};
  o.Wl = 0;
  o.bl = kW * kCin;
  o.blk0 = o.bl + kW;
  o.Ws = 0;
  o.Wb = (long long)M3 * kW * kW;
  o.cb = o.Wb + kW * kW;
  o.blk_stride = o.cb + kW;
  o.Wp1 = o.blk0 + blocks * o.blk_stride;
  o.bp1 = o.Wp1 + kH * kW;
  o.Wp2 = o.bp1 + kH;
  o.bp2 = o.Wp2 + kCout * kH;
  o.total = o.bp2 + kCout;
  return o;
}

int nfail(fftc_nn* nn, int code, const std::string& msg) {
  if (nn) nn->err = msg;
  return code;
}

#define NNCHK(nn, call)                                                                           \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) return nfail(nn, FFTC_E_HIP, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

size_t ws_layout(const fftc_nn* nn, const int N[3], int training, size_t* off /* >= 20 */) {
  const size_t Nn = (size_t)N[0] * N[1] * N[2];
  const size_t act = al(2 * Nn * kW);
  size_t o = 0;
  int q = 0;
  off[q++] = o; o += al(4 * (size_t)(N[0] + N[1] + N[2]) * nn->m);               // tab
  off[q++] = o; o += (training ? (nn->blocks + 1) : 2) * act;                    // xs
  off[q++] = o; o += training ? nn->blocks * act : 0;                            // zs
  off[q++] = o; o += al(2 * Nn * kH);                                            // h
  off[q++] = o; o += training ? al(2 * Nn * kH) : 0;                             // hpre
  off[q++] = o; o += training ? al(2 * Nn * kCh) : 0;                            // dy16
  off[q++] = o; o += training ? al(2 * Nn * kH) : 0;                             // dhpre
  off[q++] = o; o += training ? 2 * act : 0;                                     // dz
  off[q++] = o; o += al(4 * (size_t)std::max(nn->blocks, 1) * nn->KP * kW);      // xh
  off[q++] = o; o += al(4 * (size_t)nn->KP * kW);                                // dyh
  off[q++] = o; o += al(4 * (size_t)kRedGrid * 4 * std::max(nn->KP * kW, kH * (kW + 1)));  // part
  off[q++] = o; o += al(2 * (size_t)kW * nn->KP);                                // P16
  const size_t nhead = (Nn + kHeadBlock - 1) / kHeadBlock;
  off[q++] = o; o += al(8 * (std::max<size_t>(nhead, 1024) + 16));              // dsc
  off[q++] = o; o += al(16);                                                     // tinv
  off[q++] = o; o += al(8 * (size_t)kSumGroupsMax * std::max(nn->KP * kW, kH * (kW + 1)));  // grp
  off[q++] = o; o += al(4 * (size_t)N[1] * N[2] * nn->m * kW);                   // ana1
  off[q++] = o; o += al(4 * (size_t)N[2] * nn->m * nn->m * kW);                  // ana2
  return o;
}

Dims dims_of(const fftc_nn* nn) { return nn->d; }

uint16_t* xbuf(fftc_nn* nn, int i) { return nn->xs + (size_t)i * (al(2 * (size_t)nn->d.Nn * kW) / 2); }
uint16_t* zbuf(fftc_nn* nn, int i) { return nn->zs + (size_t)i * (al(2 * (size_t)nn->d.Nn * kW) / 2); }
uint16_t* dzbuf(fftc_nn* nn, int i) { return nn->dz + (size_t)i * (al(2 * (size_t)nn->d.Nn * kW) / 2); }

const uint16_t* img_Wl(const fftc_nn* nn) { return nn->img; }
const uint16_t* img_W(const fftc_nn* nn, int b) { return nn->img + kW * kCh + (size_t)b * kW * kW; }
const uint16_t* img_Wp1(const fftc_nn* nn) { return nn->img + kW * kCh + (size_t)nn->blocks * kW * kW; }

int gemm_grid(const fftc_nn* nn) {
  const int ntiles = (nn->d.Nn + 15) / 16;
  return std::max(1, std::min(kGemmGrid, (ntiles + 3) / 4));
}

int red_grid(const fftc_nn* nn) {
  const int nchunks = (nn->d.Nn + 15) / 16;
  return std::max(1, std::min(kRedGrid, (nchunks + 3) / 4));
}

template <int NO, int KX, bool BASIS, int EPI, bool QT>
void gemm(fftc_nn* nn, const uint16_t* x, const uint16_t* q, const uint16_t* p, const float* bias,
          const uint16_t* zaux, uint16_t* out, uint16_t* zout) {
  GemmArgs a{dims_of(nn), x, q, p, bias, nn->tab, zaux, out, zout};
  hipLaunchKernelGGL((k_gemm<NO, KX, BASIS, EPI, QT>), dim3(gemm_grid(nn)), dim3(256), 0, nn->stream, a);
}

// separable analysis of X [Nn][kW] onto the modes: dst [KP][ldd], scaled
void analysis(fftc_nn* nn, const uint16_t* X, float scale, float* dst, int ldd) {
  const Dims d = dims_of(nn);
  hipLaunchKernelGGL(k_ana_x, dim3(d.N[1] * d.N[2]), dim3(256), 0, nn->stream, d, (const float*)nn->tab, X, nn->ana1);
  hipLaunchKernelGGL(k_ana_y, dim3(d.N[2] * d.m), dim3(256), 0, nn->stream, d, (const float*)nn->tab,
                     (const float*)nn->ana1, nn->ana2);
  hipLaunchKernelGGL(k_ana_z, dim3(d.m * d.m), dim3(256), 0, nn->stream, d, (const float*)nn->tab,
                     (const float*)nn->ana2, scale, dst, ldd);
}

// reduce then sum: rows valid `rows`, scale, destination mapping as k_sum
template <int RL, int C, bool ONES>
void reduce(fftc_nn* nn, const uint16_t* l, const uint16_t* x, int rows, float scale, float* dst, int ldd,
            int ncols, float* dst_bias) {
  RedArgs a{dims_of(nn), l, x, nn->part};
  const int G = red_grid(nn);
  hipLaunchKernelGGL((k_reduce<RL, C, ONES>), dim3(G), dim3(256), 0, nn->stream, a);
  const int R = RL;
  const int CP = C + (ONES ? 1 : 0);
  const int waves = 4 * G, groups = (waves + kSumGroup - 1) / kSumGroup;
  hipLaunchKernelGGL(k_sum_groups, dim3((R * CP + 255) / 256, groups), dim3(256), 0, nn->stream,
                     (const float*)nn->part, waves, R * CP, nn->grp);
  hipLaunchKernelGGL(k_sum, dim3((R * CP + 255) / 256), dim3(256), 0, nn->stream, (const double*)nn->grp, groups, R,
                     CP, rows, scale, dst, ldd, ncols, dst_bias, ONES ? C : -1);
}

// forward pass; training keeps every activation and pre-activation
void forward(fftc_nn* nn, const uint16_t* feat) {
  const bool tr = nn->training;
  const float* p = nn->p;
  const Offsets& o = nn->off;
  gemm<kW, kCh, false, EPI_STORE, false>(nn, feat, img_Wl(nn), nullptr, p + o.bl, nullptr, xbuf(nn, 0), nullptr);
  int cur = 0;
  const int KPW = nn->KP * kW;
  for (int b = 0; b < nn->blocks; ++b) {
    const float* blk = p + o.blk0 + b * o.blk_stride;
    const int nxt = tr ? b + 1 : (cur ^ 1);
    float* xh = nn->xh + (size_t)(tr ? b : 0) * KPW;
    analysis(nn, xbuf(nn, cur), 1.0f / (float)nn->d.Nn, xh, kW);
    hipLaunchKernelGGL(k_mix_fwd, dim3((KPW + 255) / 256), dim3(256), 0, nn->stream, blk + o.Ws, (const float*)xh,
                       nn->M3, nn->KP, nn->P16);
    if (tr)
      gemm<kW, kW, true, EPI_GELU_Z, false>(nn, xbuf(nn, cur), img_W(nn, b), nn->P16, blk + o.cb, nullptr,
                                            xbuf(nn, nxt), zbuf(nn, b));
    else
      gemm<kW, kW, true, EPI_GELU, false>(nn, xbuf(nn, cur), img_W(nn, b), nn->P16, blk + o.cb, nullptr,
                                          xbuf(nn, nxt), nullptr);
    cur = nxt;
  }
  if (tr)
    gemm<kH, kW, false, EPI_GELU_Z, false>(nn, xbuf(nn, cur), img_Wp1(nn), nullptr, p + o.bp1, nullptr, nn->h,
                                           nn->hpre);
  else
    gemm<kH, kW, false, EPI_GELU, false>(nn, xbuf(nn, cur), img_Wp1(nn), nullptr, p + o.bp1, nullptr, nn->h,
                                         nullptr);
}

int check_grid(const int32_t N[3]) {
  for (int J = 0; J < 3; ++J)
    if (N[J] < 2 || N[J] > kMaxN) return 0;
  return 1;
}

}  // namespace

extern "C" {

int fftc_nn_create(fftc_nn_h* out, int32_t modes, int32_t blocks) {
  if (!out) return FFTC_E_ARG;
  *out = nullptr;
  if (modes < 1 || modes > kMaxM || blocks < 0 || blocks > 8) return FFTC_E_UNSUPPORTED;
  fftc_nn* nn = new (std::nothrow) fftc_nn();
  if (!nn) return FFTC_E_ARG;
  nn->m = modes;
  nn->blocks = blocks;
  nn->M3 = modes * modes * modes;
  nn->ksteps = (nn->M3 + 15) / 16;
  nn->KP = 16 * nn->ksteps;
  nn->off = make_offsets(nn->M3, blocks);
  nn->P = nn->off.total;
  nn->img_n = kW * kCh + (long long)blocks * kW * kW + kH * kW;
  *out = nn;
  return FFTC_OK;
}

void fftc_nn_destroy(fftc_nn_h nn) { delete nn; }

int fftc_nn_num_params(fftc_nn_h nn, int64_t* count) {
  if (!nn || !count) return FFTC_E_ARG;
  *count = nn->P;
  return FFTC_OK;
}

int fftc_nn_state_bytes(fftc_nn_h nn, size_t* bytes) {
  if (!nn || !bytes) return FFTC_E_ARG;
  *bytes = 4 * al(4 * (size_t)nn->P) + al(2 * (size_t)nn->img_n);
  return FFTC_OK;
}

int fftc_nn_bind_state(fftc_nn_h nn, void* state_dev, size_t bytes, void* stream) {
  if (!nn || !state_dev) return FFTC_E_ARG;
  size_t need;
  fftc_nn_state_bytes(nn, &need);
  if (bytes < need) return nfail(nn, FFTC_E_WORKSPACE, "state buffer too small");
  if ((uintptr_t)state_dev % kAlign) return nfail(nn, FFTC_E_ARG, "state buffer must be 256-byte aligned");
  char* b = (char*)state_dev;
  const size_t fp = al(4 * (size_t)nn->P);
  nn->p = (float*)b;
  nn->g = (float*)(b + fp);
  nn->mo = (float*)(b + 2 * fp);
  nn->ve = (float*)(b + 3 * fp);
  nn->img = (uint16_t*)(b + 4 * fp);
  nn->stream = (hipStream_t)stream;
  hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((nn->P + 255) / 256)), dim3(256), 0, nn->stream, nn->g, nn->P);
  hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((nn->P + 255) / 256)), dim3(256), 0, nn->stream, nn->mo, nn->P);
  hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((nn->P + 255) / 256)), dim3(256), 0, nn->stream, nn->ve, nn->P);
  nn->step = 0;
  nn->state_bound = 1;
  NNCHK(nn, hipGetLastError());
  return FFTC_OK;
}

int fftc_nn_workspace_bytes(fftc_nn_h nn, const int32_t N[3], int32_t training, size_t* bytes) {
  if (!nn || !N || !bytes) return FFTC_E_ARG;
  if (!check_grid(N)) return FFTC_E_UNSUPPORTED;
  size_t off[20];
  const int Nc[3] = {N[0], N[1], N[2]};
  *bytes = ws_layout(nn, Nc, training, off);
  return FFTC_OK;
}

int fftc_nn_bind(fftc_nn_h nn, const int32_t N[3], int32_t training, void* ws_dev, size_t bytes, void* stream) {
  if (!nn || !N || !ws_dev) return FFTC_E_ARG;
  if (!check_grid(N)) return nfail(nn, FFTC_E_UNSUPPORTED, "node grid must have 2..257 nodes per axis");
  if ((long long)N[0] * N[1] * N[2] >= (1ll << 31) / kH) return nfail(nn, FFTC_E_UNSUPPORTED, "grid too large");
  if ((uintptr_t)ws_dev % kAlign) return nfail(nn, FFTC_E_ARG, "workspace must be 256-byte aligned");
  size_t off[20];
  const int Nc[3] = {N[0], N[1], N[2]};
  const size_t need = ws_layout(nn, Nc, training, off);
  if (bytes < need) return nfail(nn, FFTC_E_WORKSPACE, "workspace too small");
  char* b = (char*)ws_dev;
  int q = 0;
  nn->tab = (float*)(b + off[q++]);
  nn->xs = (uint16_t*)(b + off[q++]);
  nn->zs = (uint16_t*)(b + off[q++]);
  nn->h = (uint16_t*)(b + off[q++]);
  nn->hpre = (uint16_t*)(b + off[q++]);
  nn->dy16 = (uint16_t*)(b + off[q++]);
  nn->dhpre = (uint16_t*)(b + off[q++]);
  nn->dz = (uint16_t*)(b + off[q++]);
  nn->xh = (float*)(b + off[q++]);
  nn->dyh = (float*)(b + off[q++]);
  nn->part = (float*)(b + off[q++]);
  nn->P16 = (uint16_t*)(b + off[q++]);
  nn->dsc = (double*)(b + off[q++]);
  nn->tinv = (float*)(b + off[q++]);
  nn->grp = (double*)(b + off[q++]);
  nn->ana1 = (float*)(b + off[q++]);
  nn->ana2 = (float*)(b + off[q++]);
  nn->training = training ? 1 : 0;
  nn->stream = (hipStream_t)stream;
  nn->d.N[0] = N[0];
  nn->d.N[1] = N[1];
  nn->d.N[2] = N[2];
  nn->d.Nn = N[0] * N[1] * N[2];
  nn->d.m = nn->m;
  nn->d.M3 = nn->M3;
  nn->d.KP = nn->KP;
  nn->d.ksteps = nn->ksteps;
  // cosine tables phi_k(i) = cos(pi k (i + 1/2) / N_J), per axis [N_J][m]
  std::vector<float> tab;
  for (int J = 0; J < 3; ++J)
    for (int i = 0; i < N[J]; ++i)
      for (int k = 0; k < nn->m; ++k) tab.push_back((float)cos(M_PI * k * (i + 0.5) / N[J]));
  NNCHK(nn, hipMemcpyAsync(nn->tab, tab.data(), 4 * tab.size(), hipMemcpyHostToDevice, nn->stream));
  NNCHK(nn, hipStreamSynchronize(nn->stream));
  nn->bound = 1;
  return FFTC_OK;
}

int fftc_nn_set_params(fftc_nn_h nn, const float* params_dev) {
  if (!nn || !params_dev) return FFTC_E_ARG;
  if (!nn->state_bound) return nfail(nn, FFTC_E_STATE, "state not bound");
  NNCHK(nn, hipMemcpyAsync(nn->p, params_dev, 4 * nn->P, hipMemcpyDeviceToDevice, nn->stream));
  hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((nn->P + 255) / 256)), dim3(256), 0, nn->stream, nn->mo, nn->P);
  hipLaunchKernelGGL(k_zero_f, dim3((unsigned)((nn->P + 255) / 256)), dim3(256), 0, nn->stream, nn->ve, nn->P);
  hipLaunchKernelGGL(k_images, dim3((unsigned)((nn->img_n + 255) / 256)), dim3(256), 0, nn->stream,
                     (const float*)nn->p, nn->off, nn->blocks, nn->img);
  nn->step = 0;
  NNCHK(nn, hipGetLastError());
  return FFTC_OK;
}

int fftc_nn_get_params(fftc_nn_h nn, float* params_dev) {
  if (!nn || !params_dev) return FFTC_E_ARG;
  if (!nn->state_bound) return nfail(nn, FFTC_E_STATE, "state not bound");
  NNCHK(nn, hipMemcpyAsync(params_dev, nn->p, 4 * nn->P, hipMemcpyDeviceToDevice, nn->stream));
  return FFTC_OK;
}

int fftc_nn_get_grad(fftc_nn_h nn, float* grad_dev) {
  if (!nn || !grad_dev) return FFTC_E_ARG;
  if (!nn->state_bound) return nfail(nn, FFTC_E_STATE, "state not bound");
  NNCHK(nn, hipMemcpyAsync(grad_dev, nn->g, 4 * nn->P, hipMemcpyDeviceToDevice, nn->stream));
  return FFTC_OK;
}

int fftc_nn_forward(fftc_nn_h nn, const uint16_t* feat_dev, float* y_dev, double s_u, const double* base_dev,
                    double* u0_dev) {
  if (!nn || !feat_dev) return FFTC_E_ARG;
  if (!nn->state_bound || !nn->bound) return nfail(nn, FFTC_E_STATE, "state and workspace must be bound");
  const int tr = nn->training;
  nn->training = 0;
  // inference uses the ping-pong buffers even on a training workspace
  forward(nn, feat_dev);
  nn->training = tr;
  HeadArgs a{};
  a.Nn = nn->d.Nn;
  a.w2 = nn->p + nn->off.Wp2;
  a.h = nn->h;
  a.y = y_dev;
  a.u0 = u0_dev;
  a.base = base_dev;
  a.s_u = s_u;
  hipLaunchKernelGGL(k_head<false>, dim3((nn->d.Nn + kHeadBlock - 1) / kHeadBlock), dim3(kHeadBlock), 0, nn->stream,
                     a);
  NNCHK(nn, hipGetLastError());
  return FFTC_OK;
}

int fftc_nn_train_step(fftc_nn_h nn, const uint16_t* feat_dev, const float* target_dev, double* loss_dev) {
  if (!nn || !feat_dev || !target_dev) return FFTC_E_ARG;
  if (!nn->state_bound || !nn->bound) return nfail(nn, FFTC_E_STATE, "state and workspace must be bound");
  if (!nn->training) return nfail(nn, FFTC_E_STATE, "workspace was bound without training");
  hipStream_t s = nn->stream;
  const Offsets& o = nn->off;
  const int Nn = nn->d.Nn;
  const int B = nn->blocks;
  const int KPW = nn->KP * kW;
  forward(nn, feat_dev);
  // 1 / sum t^2
  const int nsq = 256;
  // dsc: [0] sum t^2, [1] loss, from [8] per-block partials (t^2 first, then the loss)
  double* tsum = nn->dsc;
  double* lossd = nn->dsc + 1;
  double* dpart = nn->dsc + 8;
  hipLaunchKernelGGL(k_sq_partial, dim3(nsq), dim3(256), 0, s, target_dev, 3ll * Nn, dpart);
  hipLaunchKernelGGL(k_sq_feat, dim3(nsq), dim3(256), 0, s, feat_dev, Nn, dpart + nsq);
  hipLaunchKernelGGL(k_sq_final, dim3(1), dim3(64), 0, s, (const double*)dpart, 2 * nsq, tsum, nn->tinv);
  // output layer: loss, dy, dhpre
  const int nh = (Nn + kHeadBlock - 1) / kHeadBlock;
  HeadArgs a{};
  a.Nn = Nn;
  a.w2 = nn->p + o.Wp2;
  a.h = nn->h;
  a.hpre = nn->hpre;
  a.target = target_dev;
  a.tinv = nn->tinv;
  a.dy16 = nn->dy16;
  a.dhpre = nn->dhpre;
  a.lpart = dpart;   // the t^2 partials are consumed above
  hipLaunchKernelGGL(k_head<true>, dim3(nh), dim3(kHeadBlock), 0, s, a);
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, (const double*)dpart, nh, (const double*)tsum,
                     loss_dev ? loss_dev : lossd);
  float* g = nn->g;
  // Wp2, bp2 from dy (rows 0..2 of the 16-wide dy) and h
  reduce<kCh, kH, true>(nn, nn->dy16, nn->h, kCout, 1.0f, g + o.Wp2, kH, kH, g + o.bp2);
  // Wp1, bp1 from dhpre and x_B
  reduce<kH, kW, true>(nn, nn->dhpre, xbuf(nn, B), kH, 1.0f, g + o.Wp1, kW, kW, g + o.bp1);
  // dx_B = dhpre Wp1, then through GELU of block B (or into the lift when B = 0)
  uint16_t* dcur = dzbuf(nn, 0);
  if (B > 0)
    gemm<kW, kH, false, EPI_DGELU, true>(nn, nn->dhpre, img_Wp1(nn), nullptr, nullptr, zbuf(nn, B - 1), dcur,
                                         nullptr);
  else
    gemm<kW, kH, false, EPI_STORE, true>(nn, nn->dhpre, img_Wp1(nn), nullptr, nullptr, nullptr, dcur, nullptr);
  int side = 0;
  for (int b = B - 1; b >= 0; --b) {
    float* gb = g + o.blk0 + b * o.blk_stride;
    const float* pb = nn->p + o.blk0 + b * o.blk_stride;
    const float* xh = nn->xh + (size_t)b * KPW;
    // dyh = sum_i phi(i) dz(i)
    analysis(nn, dcur, 1.0f, nn->dyh, kW);
    // W_b, c_b
    reduce<kW, kW, true>(nn, dcur, xbuf(nn, b), kW, 1.0f, gb + o.Wb, kW, kW, gb + o.cb);
    hipLaunchKernelGGL(k_mix_bwd_dw, dim3((nn->M3 * kW * kW + 255) / 256), dim3(256), 0, s, (const float*)nn->dyh,
                       xh, nn->M3, gb + o.Ws);
    hipLaunchKernelGGL(k_mix_bwd_dx, dim3((KPW + 255) / 256), dim3(256), 0, s, pb + o.Ws, (const float*)nn->dyh,
                       nn->M3, nn->KP, 1.0f / (float)Nn, nn->P16);
    uint16_t* dnext = dzbuf(nn, side ^ 1);
    if (b > 0)
      gemm<kW, kW, true, EPI_DGELU, true>(nn, dcur, img_W(nn, b), nn->P16, nullptr, zbuf(nn, b - 1), dnext,
                                          nullptr);
    else
      gemm<kW, kW, true, EPI_STORE, true>(nn, dcur, img_W(nn, b), nn->P16, nullptr, nullptr, dnext, nullptr);
    side ^= 1;
    dcur = dnext;
  }
  // lift: Wl (9 of the 16 input columns), bl
  reduce<kW, kCh, true>(nn, dcur, feat_dev, kW, 1.0f, g + o.Wl, kCin, kCin, g + o.bl);
  NNCHK(nn, hipGetLastError());
  return FFTC_OK;
}

int fftc_nn_adam_step(fftc_nn_h nn, float lr, float beta1, float beta2, float eps) {
  if (!nn) return FFTC_E_ARG;
  if (!nn->state_bound) return nfail(nn, FFTC_E_STATE, "state not bound");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f && lr >= 0.f))
    return nfail(nn, FFTC_E_ARG, "invalid Adam hyper-parameters");
  nn->step += 1;
  const float bc1 = (float)(1.0 - pow((double)beta1, nn->step));
  const float bc2 = (float)(1.0 - pow((double)beta2, nn->step));
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((nn->P + 255) / 256)), dim3(256), 0, nn->stream, nn->p,
                     (const float*)nn->g, nn->mo, nn->ve, nn->P, lr, beta1, beta2, eps, bc1, bc2);
  hipLaunchKernelGGL(k_images, dim3((unsigned)((nn->img_n + 255) / 256)), dim3(256), 0, nn->stream,
                     (const float*)nn->p, nn->off, nn->blocks, nn->img);
  NNCHK(nn, hipGetLastError());
  return FFTC_OK;
}

int fftc_nn_make_target(const double* u_dev, const double* u1_dev, int64_t count, double s_u, float* target_dev,
                        void* stream) {
  if (!u_dev || !u1_dev || !target_dev || count < 0 || !(s_u > 0.0)) return FFTC_E_ARG;
  if (count == 0) return FFTC_OK;
  const unsigned nb = (unsigned)std::min<long long>((count + 255) / 256, 8192);
  hipLaunchKernelGGL(k_target, dim3(nb), dim3(256), 0, (hipStream_t)stream, u_dev, u1_dev, (long long)count,
                     1.0 / s_u, target_dev);
  return hipGetLastError() == hipSuccess ? FFTC_OK : FFTC_E_HIP;
}

const char* fftc_nn_last_error(fftc_nn_h nn) { return nn ? nn->err.c_str() : "null network"; }

}  // extern "C"
