// Internal declarations shared by the kernels and the host runtime of libfftc.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fftc {

enum DttType { T_DCT1 = 0, T_DCT3 = 1, T_DST1 = 2, T_DST3 = 3, T_DFT = 4 };
enum PassMode { PASS_FWD = 0, PASS_INV = 1, PASS_FWD_GREEN_INV = 2 };
enum SrcMode { SRC_BUF = 0, SRC_ANDERSON = 1, SRC_DELTA = 2 };
enum DstMode { DST_BUF = 0, DST_UPDATE = 1 };

constexpr int kMaxRadices = 16;
constexpr int kBlock = 256;          // threads per block of every streaming kernel
constexpr int kPartStride = 8;       // doubles per block partial of the residual pass
constexpr int kPartStrideD = 14;     // residual-form pass: + 6 singular-mode sums of u
// Per-block partial sums are stored by column: value q of block b at q * kPartRows + b, so that
// the one-block kernels that add them up read consecutive blocks on consecutive lanes.
constexpr int kPartRows = 2048;      // most blocks of a launch that leaves partial sums
constexpr int kMaxSets = 64;

// node mask bits
constexpr uint8_t M_STRONG = 1;      // << comp
constexpr uint8_t M_WEAK = 8;        // << comp
constexpr uint8_t M_FACE = 64;       // potential contact node

// blocks of the tiled residual pass: tx * ty node-column tiles, nseg z segments of seg planes;
// rows = partial-sum rows the control step reads (>= the blocks; the extra ones are cleared)
struct TileGrid {
  int tx, ty, nseg, seg, rows;
};

struct Geo {
  int n[3];            // voxels per axis
  int N[3];            // nodes per axis
  int periodic[3];
  long long Nn;        // nodes
  long long Nv;        // voxels
  int aface;           // bit (c*6 + J*2 + f): component c antisymmetric on face (J, f)
  // Paux reference stencil per component: diagonal, xy-, xz-, yz-plane face-diagonal coefficients
  double st[3][4];
  // axis coefficients of the Paux medium per component: a[c][J] = 2 mu0 + lam0 delta_cJ
  double ac[3][3];
  // singular modes (symbol zero) per component: bit 0 theta = 0, bit 1 theta = (pi, pi, pi)
  int sing[3];
  double sing_scale[3];   // inverse-transform factor of one singular coefficient (prod 1/2n or 1/n)
  int fs;                 // finite strain: Saint-Venant-Kirchhoff PK1 in place of the linear stress
  int hex;                // HEX1 scheme (centre gradient, one integration point) instead of TETRA2
  int iso;                // isotropic reference medium: 1 periodic cell, 2 normal-mixed DTT faces
  // normal-mixed faces, per axis: bit 0 half frequencies (DCT3/DST3), bit 1 the normal component
  // is sine-type (DST) and the tangential ones cosine-type (the reverse when 0)
  int iso_axis[3];
  double lam0, mu0;       // reference medium
};

// Device-resident iteration state (one per handle, in the workspace).
struct DevState {
  int done, status, it, i_local;
  int store_r, accel, accel_ok, acv;
  int have_prev, updates, restarts, vpar;
  int period, max_iter, contact, nC;
  int vnonempty, fine, inc_k, best_it;  // fine: the FP32 form forms stresses in FP64 (sticky);
                                        // inc_k > 0: incremental passes, a full one every inc_k;
                                        // best_it: iteration of best_res
  double tol, gate, residual, pnorm2;
  double snorm2, refine_below;
  double ms[6];
  double gram[16];
  double alpha[4];
  double sing[6];     // singular-mode coefficients of u (comp, {theta = 0, theta = pi})
  double gamma[3];    // difference-form Anderson coefficients
  double best_res;    // FP32 form: residual at the last halving (stagnation test of the refinement)
};

enum StatusCode { ST_RUNNING = 0, ST_CONVERGED = 1, ST_NOCONV = 2, ST_NAN = 3 };

// Residual pass of the FP32 form's current iteration: PASS_U = stresses of u in FP32,
// PASS_INC = p_{i-1} plus the divergence of the stresses of delta_i, PASS_U64 = stresses of u
// in FP64 (below the refinement threshold).  The launched instances and the control kernel
// take the same decision from the same state.
enum ResPass { PASS_U = 0, PASS_INC = 1, PASS_U64 = 2 };
__device__ __forceinline__ int res_pass(const DevState* st) {
  if (st->fine) return PASS_U64;
  return (st->inc_k > 0 && st->it % st->inc_k != 0) ? PASS_INC : PASS_U;
}

struct AxisPlan {
  int n;                   // transform length (voxels on the axis)
  int N;                   // nodes on a line
  int nrad;
  int rad[kMaxRadices];
  int L;                   // lines per block
  const void* tw;          // e^{-2 pi i t / 4n}, t = 0..4n-1, as (re, im) pairs of the working type
};

// Runtime-length transform kernel: each Stockham stage of radix R holds its L n / R
// butterflies in registers, ceil(EPT / R) per thread, so a block covers ceil(EPT / R) kBlock
// of them.  Elements per thread for a plan: the precision's default (8 FP64, 16 FP32), or 16
// when the block's L n points exceed 8 kBlock (lines longer than 2048 points).
__host__ __device__ inline int dtt_ept(int ept, const AxisPlan& ap) {
  return (ept <= 8 && (long long)ap.L * ap.n <= 8LL * kBlock) ? 8 : 16;
}
// true when every stage of the plan is covered by one block
__host__ __device__ inline bool dtt_covered(int ept, const AxisPlan& ap) {
  const int e = dtt_ept(ept, ap);
  for (int s = 0; s < ap.nrad; ++s) {
    const int r = ap.rad[s];
    if ((long long)ap.L * ap.n / r > (long long)((e + r - 1) / r) * kBlock) return false;
  }
  return true;
}

template <typename T>
struct Bufs {
  T* u;        // displacement (also the transform buffer)
  T* X;        // p~ written by the residual pass
  T* S[4];
  T* R[4];
  const T* lam;
  const T* mu;
  const uint8_t* mask;
};

struct ContactDev {
  int on;
  int axis, side;          // contact face
  int b1, b2;              // in-plane axes (b1 < b2)
  long long nface;
  double center[3];
  double radius;
  uint8_t* C;              // active set per face node
  uint8_t* V[2];           // V_gap (bit 0) / V_react (bit 1), current/previous
  double* fnc;             // normal reaction per face node
  double* gap;             // gap per face node
};

struct StrongDev {
  long long m;
  const long long* node;
  const int8_t* comp;
  const double* val;
};

// Relations on several nodes (averages, eq 10-14; smoothly applied conditions, eq 15-17):
// relation r on component comp[r] has the support nodes[off[r] .. off[r+1]) (at most
// kMaxRelSlots, one wavefront lane per node) with per-node weights: wa its kinematic row
// (wa . u = val), wb the distribution of its multiplier onto nodal forces (a column of B in
// eq 23), wd the direction along which proj_U moves the support.
constexpr int kMaxRelSlots = 64;

struct WeakDev {
  long long m;
  const long long* off;     // m + 1 slot offsets
  const long long* nodes;   // flat node per slot
  const double* wa;
  const double* wb;
  const double* wd;
  const int8_t* comp;
  const double* val;
  double* part;             // per relation partial ||p||^2 after projection
  double* react;            // per relation total reaction
};

template <typename T>
struct DttArgs {
  Geo g;
  int axis, mode, src;
  AxisPlan ap;                 // this axis
  int types[3];                // per component on this axis
  T* buf;                      // in/out node-shaped field
  const T* in;                 // forward source when src == SRC_BUF and in != buf
  Bufs<T> B;                   // Anderson buffers (src == SRC_ANDERSON)
  int store_s;
  DevState* st;
  int force;
  // Green (z pass)
  const double* cosT;          // [3 comps][3 axes][2][maxN]: sin^2(theta/2), cos^2(theta/2)
  const float* cosT32;         // the same, rounded to FP32
  int maxN;
  int inv_types[3];
  double thr[3];
  int generic;                 // force the runtime-length kernel
  int nt;                      // threads per block of the compile-time-length kernel
  // residual-form (FP32) iteration
  int dst;                     // DST_BUF or DST_UPDATE (x inverse pass: delta and FP64 u update)
  const T* dp2[2];             // p ping-pong buffers (SRC_DELTA, selected by iteration parity)
  const T* dY[3];              // Y-difference ring (SRC_DELTA)
  T* de;                       // correction c = p - e written by the x forward pass (SRC_DELTA)
  int nontemp;                 // SRC_DELTA: the fields exceed the last-level cache (non-temporal access)
  double* u64;                 // FP64 displacement (DST_UPDATE)
  T* delta;                    // displacement increment (DST_UPDATE)
};

// Fields of the residual-form iteration
template <typename T>
struct DeltaBufs {
  double* u;                 // displacement (FP64)
  T* delta;                  // u_i - u_{i-1}
  T* e;                      // c = p - e of the last combination: sum_j gamma_j dY_j
  T* p[2];                   // residual after proj_P (ping-pong by iteration parity)
  T* R[4];                   // R_i = p_i + K0 delta_i - e_{i-1} = dY_i + c_{i-1}, ring (i & 3)
  T* dY[3];                  // Y differences (ring of 3)
  T* t;                      // transform buffer
  const T* lam;
  const T* mu;
  const uint8_t* mask;
};

}  // namespace fftc
