// Host runtime and C ABI of libfftc: validation, plans (boundary table -> transform
// types, twiddles, symbol tables), workspace carving, and the device-driven iteration.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_set>
#include <vector>

#include "../../include/fftc.h"
#include "../../include/fftc_nn.h"
#include "fftc_internal.h"
#include "fftc_launch.h"
#include "fftc_nn_internal.h"

using namespace fftc;

// Device workspace of fftc_bind_workspace_static: one array per device, for callers that
// cannot allocate device memory.
constexpr size_t kStaticWsBytes = FFTC_STATIC_WORKSPACE_BYTES;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticWsBytes];

struct fftc_problem {
  int n[3] = {0, 0, 0}, N[3] = {0, 0, 0}, periodic[3] = {0, 0, 0};
  int precision = FFTC_FP64;
  int fs = 0;   // FFTC_FINITE_STRAIN
  double hlen = 1.0;   // voxel size: lengths at the ABI are physical, the kernels work in voxel units
  double last_force = 0.0;   // contact force of the last solve
  long long Nn = 0, Nv = 0;
  int8_t bc[18];
  int type[3][3];
  int aface = 0;
  double lam0 = 0, mu0 = 0, r0_factor = 1.0;
  int ref_mode = 0;  // 0 = factor of max stiffness, 1 = explicit
  int ref_kind = FFTC_REF_PAUX;
  int scheme = FFTC_TETRA2;
  // constraints
  std::vector<long long> s_node;
  std::vector<int8_t> s_comp;
  std::vector<double> s_val;
  std::vector<int> s_set;
  // relations on several nodes: support of relation r = slots w_off[r] .. w_off[r+1]
  std::vector<long long> w_off{0};
  std::vector<long long> w_nodes;
  std::vector<double> w_a, w_b, w_d;
  std::vector<int8_t> w_comp;
  std::vector<double> w_val;
  std::vector<int> w_set;
  std::unordered_set<long long> dof_used;  // comp * Nn + node
  // sphere
  int has_sphere = 0;
  double center[3] = {0, 0, 0}, radius = 0;
  int face = 5;
  fftc_solver_cfg cfg{1e-6, 2000, FFTC_ACV_P, 4, 2, 1e-2, 1e-5, 16, 0};
  // workspace
  char* ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  int bound = 0, stiff_set = 0;
  void* fld[10] = {};  // u, X, S0..3, R0..3 (FP32 carves S, R only for ACV_U)
  int nlit = 10;       // literal fields carved at binding
  int static_dev = -1; // device whose static workspace is bound, else -1
  // residual-form (FP32) fields: delta, e, p0, p1, R0, R1, dR0..2, dY0..2, t; FP64 u
  void* dfld[12] = {};
  double* u64 = nullptr;
  int delta_mode = 0;
  void* lam = nullptr;
  void* mu = nullptr;
  uint8_t* mask = nullptr;
  double *part = nullptr, *gpart = nullptr, *wpart = nullptr, *wreact = nullptr, *cosT = nullptr;
  double *sreact = nullptr, *chk = nullptr, *fnc = nullptr, *gap = nullptr;
  DevState* st = nullptr;
  void* tw[3] = {nullptr, nullptr, nullptr};
  long long* d_snode = nullptr;
  int8_t* d_scomp = nullptr;
  double* d_sval = nullptr;
  long long* d_wnodes = nullptr;
  long long* d_woff = nullptr;
  double *d_wa = nullptr, *d_wb = nullptr, *d_wd = nullptr;
  int8_t* d_wcomp = nullptr;
  double* d_wval = nullptr;
  uint8_t *C = nullptr, *V0 = nullptr, *V1 = nullptr;
  long long nface = 0;
  int b1 = 0, b2 = 1;
  AxisPlan ap[3];
  int ept = 8, nblk_res = 1, maxN = 1;
  int dtt_nt[5] = {0, 0, 0, 0, 0};   // autotuned block size per transform pass (TP_*)
  double tune_ms[5][2];
  Geo g;
  std::string err;
  DevState last{};
  DevState init_host{};
  std::vector<double> react_strong, react_weak;
  int profiling = 0;
};

struct fftc_batch {
  std::vector<fftc_problem*> cells;
  hipStream_t origin = nullptr;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipStream_t cap = nullptr;      // capture / replay stream (the caller's may be the NULL stream)
  hipEvent_t ready = nullptr;
  DevState* pinned = nullptr;     // host-pinned copies of the cells' device states
  int iters_per_graph = 4;
  std::string err;
};

namespace {

const size_t kAlign = 256;

int fail(fftc_problem* h, int code, const std::string& msg) {
  if (h) h->err = msg;
  return code;
}

#define HIPCHK(h, call)                                                             \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) return fail(h, FFTC_E_HIP, std::string("HIP: ") + hipGetErrorString(e_)); \
  } while (0)

bool factor_ok(int n, std::vector<int>& rad) {
  rad.clear();
  int m = n;
  while (m % 4 == 0) { rad.push_back(4); m /= 4; }
  while (m % 2 == 0) { rad.push_back(2); m /= 2; }
  while (m % 3 == 0) { rad.push_back(3); m /= 3; }
  while (m % 5 == 0) { rad.push_back(5); m /= 5; }
  for (int r : {7, 11, 13})
    while (m % r == 0) { rad.push_back(r); m /= r; }
  return m == 1 && (int)rad.size() <= kMaxRadices;
}

int sym_of(int code) { return code == FFTC_BC_DIRICHLET ? 1 : (code == FFTC_BC_NEUMANN ? 0 : 2); }  // 1 = A

// No periodic axis, and on every face the normal component's symmetry differs from that of
// both tangential components (then the DTTs diagonalise the coupled isotropic medium).
bool normal_mixed(const fftc_problem* h) {
  for (int J = 0; J < 3; ++J) {
    if (h->periodic[J]) return false;
    for (int f = 0; f < 2; ++f)
      for (int c = 0; c < 3; ++c)
        if (c != J && sym_of(h->bc[c * 6 + J * 2 + f]) == sym_of(h->bc[J * 6 + J * 2 + f])) return false;
  }
  return true;
}

// Table 2: symmetries on the two faces -> transform
int type_of(int s0, int s1) {
  if (s0 == 2) return T_DFT;
  if (s0 == 0 && s1 == 0) return T_DCT1;
  if (s0 == 0 && s1 == 1) return T_DCT3;
  if (s0 == 1 && s1 == 1) return T_DST1;
  return T_DST3;
}

double theta_of(int type, int n, int idx) {
  switch (type) {
    case T_DCT1:
    case T_DST1: return M_PI * idx / n;
    case T_DCT3:
    case T_DST3: return M_PI * (idx + 0.5) / n;
    default: {
      int k = std::min(idx, n - idx);
      return 2.0 * M_PI * k / n;
    }
  }
}

long long node_flat(const fftc_problem* h, long long i, long long j, long long k) {
  return i + (long long)h->N[0] * (j + (long long)h->N[1] * k);
}

bool node_antisym(const fftc_problem* h, int c, const long long xyz[3]) {
  for (int J = 0; J < 3; ++J) {
    if (h->periodic[J]) continue;
    if (xyz[J] == 0 && ((h->aface >> (c * 6 + J * 2)) & 1)) return true;
    if (xyz[J] == h->n[J] && ((h->aface >> (c * 6 + J * 2 + 1)) & 1)) return true;
  }
  return false;
}

void build_plan(fftc_problem* h) {
  h->aface = 0;
  for (int J = 0; J < 3; ++J) h->periodic[J] = (h->bc[0 * 6 + J * 2] == FFTC_BC_PERIODIC);
  for (int c = 0; c < 3; ++c)
    for (int J = 0; J < 3; ++J) {
      const int s0 = sym_of(h->bc[c * 6 + J * 2]), s1 = sym_of(h->bc[c * 6 + J * 2 + 1]);
      h->type[c][J] = type_of(s0, s1);
      if (s0 == 1) h->aface |= 1 << (c * 6 + J * 2);
      if (s1 == 1) h->aface |= 1 << (c * 6 + J * 2 + 1);
    }
  for (int J = 0; J < 3; ++J) h->N[J] = h->n[J] + (h->periodic[J] ? 0 : 1);
  h->Nn = (long long)h->N[0] * h->N[1] * h->N[2];
}

template <typename T>
size_t tsize() { return sizeof(T); }

struct Layout {
  size_t total = 0;
  size_t take(size_t bytes) {
    size_t off = total;
    total += (bytes + kAlign - 1) / kAlign * kAlign;
    return off;
  }
};

// carve the workspace; with base == nullptr only computes the size
size_t carve(fftc_problem* h, char* base) {
  Layout L;
  const size_t ts = h->precision == FFTC_FP64 ? 8 : 4;
  const size_t f3 = ts * 3 * (size_t)h->Nn;
  size_t off[64];
  int q = 0;
  // the FP32 residual-form iteration keeps its own fields; its literal form (ACV_U) and the
  // stage entry points need u and p~, the Anderson rings only for ACV_U
  const int nlit = (h->precision == FFTC_FP64 || h->cfg.acv == FFTC_ACV_U) ? 10 : 2;
  for (int i = 0; i < nlit; ++i) off[q++] = L.take(f3);
  off[q++] = L.take(ts * h->Nv);
  off[q++] = L.take(ts * h->Nv);
  off[q++] = L.take((size_t)h->Nn);
  off[q++] = L.take(sizeof(double) * kPartStrideD * kPartRows);
  off[q++] = L.take(sizeof(double) * 10 * kPartRows);
  off[q++] = L.take(sizeof(DevState));
  const size_t mw = h->w_comp.size(), ms = h->s_comp.size();
  off[q++] = L.take(sizeof(double) * (mw + 1));
  off[q++] = L.take(sizeof(double) * (mw + 1));
  int maxN = std::max(h->N[0], std::max(h->N[1], h->N[2]));
  off[q++] = L.take((sizeof(double) + sizeof(float)) * 18 * maxN);   // symbol tables, FP64 then FP32
  for (int J = 0; J < 3; ++J) off[q++] = L.take(2 * ts * 4 * (size_t)h->n[J]);
  off[q++] = L.take(8 * (ms + 1));
  off[q++] = L.take(ms + 1);
  off[q++] = L.take(8 * (ms + 1));
  const size_t nslot = h->w_nodes.size();
  off[q++] = L.take(8 * (nslot + 1));
  off[q++] = L.take(mw + 1);
  off[q++] = L.take(8 * (mw + 1));
  off[q++] = L.take(8 * (mw + 1));
  for (int i = 0; i < 3; ++i) off[q++] = L.take(8 * (nslot + 1));
  long long nface = 1;
  if (h->has_sphere) {
    const int a = h->face / 2;
    int bb[2], t = 0;
    for (int J = 0; J < 3; ++J)
      if (J != a) bb[t++] = J;
    nface = (long long)h->N[bb[0]] * h->N[bb[1]];
  }
  off[q++] = L.take(nface);
  off[q++] = L.take(nface);
  off[q++] = L.take(nface);
  off[q++] = L.take(8 * nface);
  off[q++] = L.take(8 * nface);
  off[q++] = L.take(8 * (ms + 1));
  off[q++] = L.take(sizeof(double) * 3 * 1024);
  const int nd = h->precision == FFTC_FP32 ? 12 : 0;
  for (int i = 0; i < nd; ++i) off[q++] = L.take(4 * 3 * (size_t)h->Nn);
  if (nd) off[q++] = L.take(8 * 3 * (size_t)h->Nn);
  if (base) {
    q = 0;
    h->nlit = nlit;
    for (int i = 0; i < 10; ++i) h->fld[i] = i < nlit ? base + off[q++] : nullptr;
    h->lam = base + off[q++];
    h->mu = base + off[q++];
    h->mask = (uint8_t*)(base + off[q++]);
    h->part = (double*)(base + off[q++]);
    h->gpart = (double*)(base + off[q++]);
    h->st = (DevState*)(base + off[q++]);
    h->wpart = (double*)(base + off[q++]);
    h->wreact = (double*)(base + off[q++]);
    h->cosT = (double*)(base + off[q++]);
    for (int J = 0; J < 3; ++J) h->tw[J] = base + off[q++];
    h->d_snode = (long long*)(base + off[q++]);
    h->d_scomp = (int8_t*)(base + off[q++]);
    h->d_sval = (double*)(base + off[q++]);
    h->d_wnodes = (long long*)(base + off[q++]);
    h->d_wcomp = (int8_t*)(base + off[q++]);
    h->d_wval = (double*)(base + off[q++]);
    h->d_woff = (long long*)(base + off[q++]);
    h->d_wa = (double*)(base + off[q++]);
    h->d_wb = (double*)(base + off[q++]);
    h->d_wd = (double*)(base + off[q++]);
    h->C = (uint8_t*)(base + off[q++]);
    h->V0 = (uint8_t*)(base + off[q++]);
    h->V1 = (uint8_t*)(base + off[q++]);
    h->fnc = (double*)(base + off[q++]);
    h->gap = (double*)(base + off[q++]);
    h->sreact = (double*)(base + off[q++]);
    h->chk = (double*)(base + off[q++]);
    for (int i = 0; i < nd; ++i) h->dfld[i] = base + off[q++];
    if (nd) h->u64 = (double*)(base + off[q++]);
    h->nface = nface;
    h->maxN = maxN;
  }
  return L.total;
}

void set_stencil(fftc_problem* h) {
  h->g.lam0 = h->lam0;
  h->g.mu0 = h->mu0;
  for (int c = 0; c < 3; ++c) {
    double cj[3];
    for (int J = 0; J < 3; ++J) cj[J] = 2.0 * h->mu0 + (J == c ? h->lam0 : 0.0);
    h->g.st[c][0] = cj[0] + cj[1] + cj[2];
    h->g.st[c][1] = (cj[2] - cj[0] - cj[1]) / 4.0;
    h->g.st[c][2] = (cj[1] - cj[0] - cj[2]) / 4.0;
    h->g.st[c][3] = (cj[0] - cj[1] - cj[2]) / 4.0;
    for (int J = 0; J < 3; ++J) h->g.ac[c][J] = cj[J];
  }
}

template <typename T>
Bufs<T> bufs(fftc_problem* h) {
  Bufs<T> B;
  B.u = (T*)h->fld[0];
  B.X = (T*)h->fld[1];
  for (int q = 0; q < 4; ++q) {
    B.S[q] = (T*)h->fld[2 + q];
    B.R[q] = (T*)h->fld[6 + q];
  }
  B.lam = (const T*)h->lam;
  B.mu = (const T*)h->mu;
  B.mask = h->mask;
  return B;
}

DeltaBufs<float> dbufs(fftc_problem* h) {
  DeltaBufs<float> D;
  D.u = h->u64;
  D.delta = (float*)h->dfld[0];
  D.e = (float*)h->dfld[1];
  D.p[0] = (float*)h->dfld[2];
  D.p[1] = (float*)h->dfld[3];
  for (int q = 0; q < 4; ++q) D.R[q] = (float*)h->dfld[4 + q];
  for (int q = 0; q < 3; ++q) D.dY[q] = (float*)h->dfld[8 + q];
  D.t = (float*)h->dfld[11];
  D.lam = (const float*)h->lam;
  D.mu = (const float*)h->mu;
  D.mask = h->mask;
  return D;
}

ContactDev contact_dev(fftc_problem* h) {
  ContactDev ct{};
  ct.on = h->has_sphere;
  ct.axis = h->face / 2;
  ct.side = h->face % 2;
  ct.b1 = h->b1;
  ct.b2 = h->b2;
  ct.nface = h->nface;
  for (int c = 0; c < 3; ++c) ct.center[c] = h->center[c];
  ct.radius = h->radius;
  ct.C = h->C;
  ct.V[0] = h->V0;
  ct.V[1] = h->V1;
  ct.fnc = h->fnc;
  ct.gap = h->gap;
  return ct;
}

StrongDev strong_dev(fftc_problem* h) {
  StrongDev s{(long long)h->s_comp.size(), h->d_snode, h->d_scomp, h->d_sval};
  return s;
}

WeakDev weak_dev(fftc_problem* h) {
  WeakDev w{(long long)h->w_comp.size(), h->d_woff, h->d_wnodes, h->d_wa, h->d_wb, h->d_wd,
            h->d_wcomp, h->d_wval, h->wpart, h->wreact};
  return w;
}

// The transform passes of one iteration, in order; each has its own tuned block size.
enum { TP_XF = 0, TP_YF, TP_Z, TP_YI, TP_XI, TP_N };
int pass_of(int axis, int mode) {
  if (axis == 2) return TP_Z;
  if (mode == PASS_INV) return axis == 0 ? TP_XI : TP_YI;
  return axis == 0 ? TP_XF : TP_YF;
}

template <typename T>
DttArgs<T> dtt_args(fftc_problem* h, int axis, int mode, int force) {
  DttArgs<T> a{};
  a.g = h->g;
  a.axis = axis;
  a.mode = mode;
  a.src = SRC_BUF;
  a.ap = h->ap[axis];
  for (int c = 0; c < 3; ++c) a.types[c] = h->type[c][axis];
  a.buf = (T*)h->fld[0];
  a.in = (T*)h->fld[0];
  a.B = bufs<T>(h);
  a.store_s = 0;
  a.st = h->st;
  a.force = force;
  a.cosT = h->cosT;
  a.cosT32 = (const float*)(h->cosT + 18 * (size_t)h->maxN);
  a.maxN = h->maxN;
  // the symbol vanishes only at theta = 0 and (pi, pi, pi) (exact zeros of the factored
  // form); any positive value is at least ~ a theta_min^2, far above this threshold
  for (int c = 0; c < 3; ++c) a.thr[c] = 1e-13 * std::max(h->g.ac[c][0], std::max(h->g.ac[c][1], h->g.ac[c][2]));
  a.nt = h->dtt_nt[pass_of(axis, mode)];
  return a;
}

// Arguments of transform pass p of the FP32 residual-form iteration: the x forward pass forms
// e = p - sum gamma dY from the residual fields, the x inverse pass updates the FP64 u and delta.
DttArgs<float> delta_pass(fftc_problem* h, int p, const DeltaBufs<float>& D) {
  static const int axis[TP_N] = {0, 1, 2, 1, 0};
  static const int mode[TP_N] = {PASS_FWD, PASS_FWD, PASS_FWD_GREEN_INV, PASS_INV, PASS_INV};
  DttArgs<float> a = dtt_args<float>(h, axis[p], mode[p], 0);
  a.buf = D.t;
  a.in = D.t;
  if (p == TP_XF) {
    a.src = SRC_DELTA;
    a.dp2[0] = D.p[0];
    a.dp2[1] = D.p[1];
    for (int q = 0; q < 3; ++q) a.dY[q] = D.dY[q];
    a.de = D.e;
    // the four fields the pass reads and writes are larger than the 256 MB last-level cache
    a.nontemp = 4 * 3 * 4 * (double)h->Nn > 256.0 * (1 << 20);
  } else if (p == TP_XI) {
    a.dst = DST_UPDATE;
    a.u64 = D.u;
    a.delta = D.delta;
  }
  return a;
}

// Green step on the working buffers: u <- DT^-1(M^-1 DT(src)), forward x source chosen by caller
struct StageTimer;
template <typename T>
void enqueue_green(fftc_problem* h, int src, const T* in, int store_s, int force, StageTimer* tm = nullptr);

struct StageTimer {
  hipEvent_t ev[16];
  int n = 0;
  bool on = false;
  void mark(hipStream_t s) {
    if (on && n < 16) hipEventRecord(ev[n++], s);
  }
};

// Period of the full residual passes between incremental ones (0: every pass from u).  The
// incremental pass needs the FP32 form on a tiled small-strain problem with no obstacle, no
// singular modes and no relations (their projections and multipliers are formed from u).
int inc_period(const fftc_problem* h) {
  if (!h->delta_mode || h->fs || h->has_sphere || h->cfg.anchor_every <= 0) return 0;
  if (h->g.sing[0] || h->g.sing[1] || h->g.sing[2] || weak_dev(const_cast<fftc_problem*>(h)).m > 0) return 0;
  if (residual_tiles(h->g, false).tx <= 0) return 0;
  return h->cfg.anchor_every;
}

void enqueue_delta_iteration(fftc_problem* h, StageTimer* tm) {
  DeltaBufs<float> D = dbufs(h);
  const ContactDev ct = contact_dev(h);
  const WeakDev w = weak_dev(h);
  const StrongDev sd = strong_dev(h);
  const long long n3 = 3 * h->Nn;
  hipStream_t s = h->stream;
  if (tm) tm->mark(s);
  const int nres = launch_delta_residual<float>(h->g, D, ct, h->st, h->part, h->nblk_res, h->cfg.refine_below > 0.0,
                                                inc_period(h) > 0, s);
  if (tm) tm->mark(s);
  launch_delta_control<float>(h->g, D, ct, w, h->st, h->part, h->wpart, nres, s);
  if (tm) tm->mark(s);
  if (h->cfg.acv == FFTC_ACV_P) launch_delta_anderson<float>(D, n3, h->st, h->gpart, h->nblk_res, s);
  if (tm) tm->mark(s);
  for (int p = 0; p < TP_N; ++p) {
    launch_dtt<float>(delta_pass(h, p, D), h->ept, s);
    if (tm) tm->mark(s);
  }
  launch_delta_proj<float>(h->g, D, sd, w, ct, h->st, 0, 1, s);
  if (tm) tm->mark(s);
}

template <typename T>
void enqueue_iteration(fftc_problem* h, StageTimer* tm = nullptr) {
  if (h->delta_mode) {
    enqueue_delta_iteration(h, tm);
    return;
  }
  Bufs<T> B = bufs<T>(h);
  const ContactDev ct = contact_dev(h);
  const WeakDev w = weak_dev(h);
  const StrongDev sd = strong_dev(h);
  const long long n3 = 3 * h->Nn;
  hipStream_t s = h->stream;
  if (h->cfg.acv == FFTC_ACV_U) {
    Bufs<T> Bu = B;
    Bu.X = B.u;  // residual store on the displacement
    launch_flags_combine<T>(B, n3, h->st, 0, s);
    launch_anderson<T>(Bu, n3, h->st, h->gpart, h->nblk_res, s);
    launch_flags_combine<T>(B, n3, h->st, 1, s);
  }
  if (tm) tm->mark(s);
  launch_residual<T>(h->g, B, ct, h->st, h->part, h->nblk_res, 0, 0, s);
  if (tm) tm->mark(s);
  launch_weak<T>(h->g, B, w, h->st, 0, s);
  launch_control(h->st, h->part, h->nblk_res, h->wpart, w.m, ct, kPartStride, s);
  if (tm) tm->mark(s);
  if (h->cfg.acv == FFTC_ACV_P) launch_anderson<T>(B, n3, h->st, h->gpart, h->nblk_res, s);
  if (tm) tm->mark(s);
  enqueue_green<T>(h, h->cfg.acv == FFTC_ACV_P ? SRC_ANDERSON : SRC_BUF, B.X, h->cfg.acv == FFTC_ACV_P, 0, tm);
  launch_proj<T>(h->g, B.u, w, ct, sd, h->st, 1, 0, s);
  if (tm) tm->mark(s);
}

template <typename T>
void enqueue_green(fftc_problem* h, int src, const T* in, int store_s, int force, StageTimer* tm) {
  DttArgs<T> a = dtt_args<T>(h, 0, PASS_FWD, force);
  a.src = src;
  a.in = in;
  a.store_s = store_s;
  launch_dtt<T>(a, h->ept, h->stream);
  if (tm) tm->mark(h->stream);
  a = dtt_args<T>(h, 1, PASS_FWD, force);
  launch_dtt<T>(a, h->ept, h->stream);
  if (tm) tm->mark(h->stream);
  if (h->g.iso) {
    // coupled 3x3 Green solve between the forward and the inverse z transforms
    if constexpr (sizeof(T) == 8) {
      launch_dtt<T>(dtt_args<T>(h, 2, PASS_FWD, force), h->ept, h->stream);
      launch_green_iso(h->g, (double*)h->fld[0], h->st, force, h->stream);
      launch_dtt<T>(dtt_args<T>(h, 2, PASS_INV, force), h->ept, h->stream);
    }
  } else {
    a = dtt_args<T>(h, 2, PASS_FWD_GREEN_INV, force);
    launch_dtt<T>(a, h->ept, h->stream);
  }
  if (tm) tm->mark(h->stream);
  a = dtt_args<T>(h, 1, PASS_INV, force);
  launch_dtt<T>(a, h->ept, h->stream);
  if (tm) tm->mark(h->stream);
  a = dtt_args<T>(h, 0, PASS_INV, force);
  launch_dtt<T>(a, h->ept, h->stream);
  if (tm) tm->mark(h->stream);
}

// Times each stage of `iters` further iterations with HIP events on the handle's stream.
// Stages: residual, weak+control, anderson, dtt x fwd, dtt y fwd, dtt z fwd+green+inv,
// dtt y inv, dtt x inv, projections.  Requires a prior solve (state and fields live).
template <typename T>
int profile_t(fftc_problem* h, int iters, double* ms, int nst) {
  hipStream_t s = h->stream;
  StageTimer tm;
  tm.on = true;
  for (int q = 0; q < 16; ++q) HIPCHK(h, hipEventCreate(&tm.ev[q]));
  std::vector<double> acc(16, 0.0);
  // keep the state running
  DevState hs{};
  HIPCHK(h, hipMemcpyAsync(&hs, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  hs.done = 0;
  hs.status = 0;
  hs.max_iter = hs.it + iters + 8;
  hs.tol = 0.0;
  HIPCHK(h, hipMemcpyAsync(h->st, &hs, sizeof(DevState), hipMemcpyHostToDevice, s));
  int nmark = 0;
  for (int it = 0; it < iters; ++it) {
    tm.n = 0;
    enqueue_iteration<T>(h, &tm);
    HIPCHK(h, hipStreamSynchronize(s));
    nmark = tm.n;
    for (int q = 0; q + 1 < tm.n; ++q) {
      float e = 0.f;
      HIPCHK(h, hipEventElapsedTime(&e, tm.ev[q], tm.ev[q + 1]));
      acc[q] += e;
    }
  }
  for (int q = 0; q < 16; ++q) hipEventDestroy(tm.ev[q]);
  for (int q = 0; q < nst; ++q) ms[q] = (q + 1 < nmark) ? acc[q] / iters : 0.0;
  return FFTC_OK;
}

// ---- solve = init + device-driven iterations + finish (shared by solo and batched solves)

int init_state(fftc_problem* h) {
  DevState hs{};
  hs.tol = h->cfg.tol;
  hs.gate = h->cfg.update_gate;
  hs.max_iter = h->cfg.max_iter;
  hs.period = h->cfg.period;
  hs.acv = h->cfg.acv;
  hs.contact = h->has_sphere;
  hs.refine_below = h->delta_mode ? h->cfg.refine_below : 0.0;
  hs.fine = 0;
  hs.inc_k = inc_period(h);
  hs.best_res = 1e300;
  hs.best_it = 0;
  h->init_host = hs;
  HIPCHK(h, hipMemcpyAsync(h->st, &h->init_host, sizeof(DevState), hipMemcpyHostToDevice, h->stream));
  return FFTC_OK;
}

template <typename T>
int init_literal(fftc_problem* h, const double* u_dev, int zero_start) {
  Bufs<T> B = bufs<T>(h);
  hipStream_t s = h->stream;
  const long long n3 = 3 * h->Nn;
  if (zero_start || !u_dev) HIPCHK(h, hipMemsetAsync(B.u, 0, sizeof(T) * n3, s));
  else launch_convert<double, T>(u_dev, B.u, n3, s, 1.0 / h->hlen);
  launch_zero_amask<T>(h->g, B.u, s);
  const ContactDev ct = contact_dev(h);
  // initial proj_U (and the initial active set from the gaps)
  if (ct.on) launch_contact_init<T>(h->g, B.u, ct, s);
  launch_proj<T>(h->g, B.u, weak_dev(h), ct, strong_dev(h), h->st, 0, 1, s);
  return init_state(h);
}

int init_delta(fftc_problem* h, const double* u_dev, int zero_start) {
  DeltaBufs<float> D = dbufs(h);
  hipStream_t s = h->stream;
  const long long n3 = 3 * h->Nn;
  if (zero_start || !u_dev) HIPCHK(h, hipMemsetAsync(D.u, 0, 8 * n3, s));
  else if (h->hlen != 1.0) launch_convert<double, double>(u_dev, D.u, n3, s, 1.0 / h->hlen);
  else HIPCHK(h, hipMemcpyAsync(D.u, u_dev, 8 * n3, hipMemcpyDeviceToDevice, s));
  launch_zero_amask<double>(h->g, D.u, s);
  const ContactDev ct = contact_dev(h);
  if (ct.on) launch_contact_init<double>(h->g, D.u, ct, s);
  launch_delta_proj<float>(h->g, D, strong_dev(h), weak_dev(h), ct, h->st, 1, 0, s);
  for (int q = 0; q < 11; ++q) HIPCHK(h, hipMemsetAsync(h->dfld[q], 0, 4 * n3, s));
  return init_state(h);
}

int solve_init(fftc_problem* h, const double* u_dev, int zero_start) {
  if (h->precision == FFTC_FP32 && h->cfg.acv == FFTC_ACV_U && h->nlit < 10)
    return fail(h, FFTC_E_STATE, "ACV_U in FP32 needs its Anderson fields: set it before binding the workspace");
  // FP32: residual-form iteration (FP64 displacement), except for ACV_U
  h->delta_mode = (h->precision == FFTC_FP32 && h->cfg.acv != FFTC_ACV_U) ? 1 : 0;
  if (h->delta_mode) return init_delta(h, u_dev, zero_start);
  return h->precision == FFTC_FP64 ? init_literal<double>(h, u_dev, zero_start)
                                   : init_literal<float>(h, u_dev, zero_start);
}

void enqueue_iter(fftc_problem* h) {
  if (h->precision == FFTC_FP64) enqueue_iteration<double>(h);
  else enqueue_iteration<float>(h);
}

int finish_report(fftc_problem* h, const DevState& out, double force_c, int nC, fftc_report* rep) {
  const int status = out.status == ST_CONVERGED ? FFTC_OK : (out.status == ST_NAN ? FFTC_E_NAN : FFTC_E_NOCONV);
  if (rep) {
    memset(rep, 0, sizeof(*rep));
    rep->status = status;
    rep->iterations = out.it;
    rep->residual = out.residual;
    rep->contact_updates = out.updates;
    rep->anderson_restarts = out.restarts;
    for (int q = 0; q < 6; ++q) rep->mean_stress[q] = out.ms[q] / (double)h->Nv;
    if (h->has_sphere) {
      const int a = h->face / 2;
      double A0 = 1.0;
      for (int J = 0; J < 3; ++J)
        if (J != a) A0 *= h->n[J];
      rep->force_mean_stress = -A0 * h->hlen * h->hlen * rep->mean_stress[a];
      rep->force_contact = force_c;
      h->last_force = force_c;
      rep->contact_nodes = nC;
    }
  }
  if (out.status == ST_NAN) return fail(h, FFTC_E_NAN, "non-finite iterate");
  if (out.status != ST_CONVERGED) return fail(h, FFTC_E_NOCONV, "maximum number of iterations reached");
  return FFTC_OK;
}

// After the iterations: reactions of the returned iterate, output displacement, report.
int solve_finish(fftc_problem* h, double* u_dev, fftc_report* rep) {
  hipStream_t s = h->stream;
  const long long n3 = 3 * h->Nn;
  const ContactDev ct = contact_dev(h);
  const StrongDev sd = strong_dev(h);
  HIPCHK(h, hipMemcpyAsync(&h->last, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
  std::vector<double> msp;
  if (h->delta_mode) {
    DeltaBufs<float> D = dbufs(h);
    // the residual-form pass carries only the norms; the mean stress is formed here, once
    msp.assign(6 * (size_t)launch_mean_stress_d<float>(h->g, D, h->part, s), 0.0);
    HIPCHK(h, hipMemcpyAsync(msp.data(), h->part, 8 * msp.size(), hipMemcpyDeviceToHost, s));
    launch_reactions_d<float>(h->g, D, sd, h->sreact, s);
    if (u_dev && h->hlen != 1.0) launch_convert<double, double>(D.u, u_dev, n3, s, h->hlen);
    else if (u_dev) HIPCHK(h, hipMemcpyAsync(u_dev, D.u, 8 * n3, hipMemcpyDeviceToDevice, s));
    if (ct.on) launch_contact_force<double>(h->g, D.u, ct, h->chk, 64, s);
  } else if (h->precision == FFTC_FP64) {
    Bufs<double> B = bufs<double>(h);
    launch_reactions<double>(h->g, B, sd, h->sreact, s);
    if (u_dev) launch_convert<double, double>(B.u, u_dev, n3, s, h->hlen);
    if (ct.on) launch_contact_force<double>(h->g, B.u, ct, h->chk, 64, s);
  } else {
    Bufs<float> B = bufs<float>(h);
    launch_reactions<float>(h->g, B, sd, h->sreact, s);
    if (u_dev) launch_convert<float, double>(B.u, u_dev, n3, s, h->hlen);
    if (ct.on) launch_contact_force<float>(h->g, B.u, ct, h->chk, 64, s);
  }
  h->react_strong.assign(h->s_comp.size(), 0.0);
  h->react_weak.assign(h->w_comp.size(), 0.0);
  if (!h->react_strong.empty())
    HIPCHK(h, hipMemcpyAsync(h->react_strong.data(), h->sreact, 8 * h->react_strong.size(), hipMemcpyDeviceToHost, s));
  if (!h->react_weak.empty())
    HIPCHK(h, hipMemcpyAsync(h->react_weak.data(), h->wreact, 8 * h->react_weak.size(), hipMemcpyDeviceToHost, s));
  std::vector<double> cf(2 * 64, 0.0);
  if (ct.on) HIPCHK(h, hipMemcpyAsync(cf.data(), h->chk, 8 * cf.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  if (!msp.empty()) {
    const size_t nb = msp.size() / 6;
    for (int q = 0; q < 6; ++q) {
      double a = 0.0;
      for (size_t b = 0; b < nb; ++b) a += msp[6 * b + q];
      h->last.ms[q] = a;
    }
  }
  const double h2 = h->hlen * h->hlen;   // forces: voxel units -> physical
  for (double& v : h->react_strong) v *= h2;
  for (double& v : h->react_weak) v *= h2;
  double force_c = 0.0;
  int nC = 0;
  if (ct.on) {
    double fs = 0.0, cnt = 0.0;
    for (int b = 0; b < 64; ++b) {
      fs += cf[2 * b];
      cnt += cf[2 * b + 1];
    }
    force_c = -((h->face % 2) ? 1.0 : -1.0) * fs * h2;
    nC = (int)cnt;
  }
  return finish_report(h, h->last, force_c, nC, rep);
}

int solve_all(fftc_problem* h, double* u_dev, int zero_start, fftc_report* rep) {
  int rc = solve_init(h, u_dev, zero_start);
  if (rc != FFTC_OK) return rc;
  hipStream_t s = h->stream;
  int chunk = 4;
  DevState out{};
  for (;;) {
    for (int t = 0; t < chunk; ++t) enqueue_iter(h);
    HIPCHK(h, hipGetLastError());
    HIPCHK(h, hipMemcpyAsync(&out, h->st, sizeof(DevState), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (out.done) break;
    chunk = std::min(64, chunk * 2);
  }
  return solve_finish(h, u_dev, rep);
}

template <typename T>
int stage_residual_t(fftc_problem* h, const double* u_dev, double* p_dev, double* ptil_dev, double* sums) {
  Bufs<T> B = bufs<T>(h);
  hipStream_t s = h->stream;
  const long long n3 = 3 * h->Nn;
  launch_convert<double, T>(u_dev, B.u, n3, s);
  const ContactDev ct = contact_dev(h);
  const WeakDev w = weak_dev(h);
  DevState hs{};
  HIPCHK(h, hipMemcpyAsync(h->st, &hs, sizeof(DevState), hipMemcpyHostToDevice, s));
  for (int pass = 0; pass < 2; ++pass) {
    double* dst = pass == 0 ? ptil_dev : p_dev;
    if (!dst) continue;
    launch_residual<T>(h->g, B, ct, h->st, h->part, h->nblk_res, 1, pass, s);
    launch_weak<T>(h->g, B, w, h->st, 1, s);
    launch_convert<T, double>(B.X, dst, n3, s);
  }
  if (sums) {
    if (!ptil_dev && !p_dev) {
      launch_residual<T>(h->g, B, ct, h->st, h->part, h->nblk_res, 1, 0, s);
      launch_weak<T>(h->g, B, w, h->st, 1, s);
    }
    // the first two columns of the partial-sum table: ||p||^2 and ||sigma||^2 per block
    std::vector<double> part(2 * (size_t)h->nblk_res), wp(w.m + 1);
    for (int q = 0; q < 2; ++q)
      HIPCHK(h, hipMemcpyAsync(part.data() + (size_t)q * h->nblk_res, h->part + (size_t)q * kPartRows,
                               8 * (size_t)h->nblk_res, hipMemcpyDeviceToHost, s));
    if (w.m) HIPCHK(h, hipMemcpyAsync(wp.data(), h->wpart, 8 * w.m, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    double a0 = 0, a1 = 0;
    for (int b = 0; b < h->nblk_res; ++b) {
      a0 += part[b];
      a1 += part[(size_t)h->nblk_res + b];
    }
    for (long long r = 0; r < w.m; ++r) a0 += wp[r];
    sums[0] = a0;
    sums[1] = a1;
  }
  HIPCHK(h, hipStreamSynchronize(s));
  return FFTC_OK;
}

// One residual pass of the FP32 residual-form iteration on caller state (local Anderson index
// il; kind 0: stresses of u in FP32, 1: in FP64, 2: the incremental pass): u (FP64), delta, e,
// p_prev, R_prev in, p, R, dR, dY out (FP64 copies), sums[0] = ||p||^2, sums[1] = sum (1/2)
// sigma:sigma (0 for the incremental pass).  The pass reads c = p_prev - e, formed here.
int stage_residual_form_t(fftc_problem* h, const double* const* in, int il, int kind, double* const* out,
                          double* sums) {
  DeltaBufs<float> D = dbufs(h);
  hipStream_t s = h->stream;
  const long long n3 = 3 * h->Nn;
  const int slot = (il + 1) % 3;
  // iteration parity: the incremental pass runs at it = 1 of a period of 2
  const int it = kind == 2 ? 1 : 0;
  HIPCHK(h, hipMemcpyAsync(D.u, in[0], 8 * n3, hipMemcpyDeviceToDevice, s));
  float* const Rcur = D.R[il & 3];
  float* const Rprev = D.R[(il + 3) & 3];
  float* const pprev = D.p[(it & 1) ^ 1];
  float* dst[4] = {D.delta, D.e, pprev, Rprev};
  for (int q = 0; q < 4; ++q) {
    if (in[q + 1]) launch_convert<double, float>(in[q + 1], dst[q], n3, s);
    else HIPCHK(h, hipMemsetAsync(dst[q], 0, 4 * n3, s));
  }
  launch_diff<float>(pprev, D.e, D.e, n3, s);   // c = p_prev - e
  for (int q = 0; q < 3; ++q) HIPCHK(h, hipMemsetAsync(D.dY[q], 0, 4 * n3, s));
  DevState hs{};
  hs.acv = FFTC_ACV_P;
  hs.i_local = il;
  hs.it = it;
  hs.accel_ok = 1;   // c comes from the caller's e, not 0
  hs.fine = kind == 1 ? 1 : 0;
  hs.inc_k = kind == 2 ? 2 : 0;
  hs.tol = 0.0;
  hs.max_iter = 1 << 30;
  hs.period = h->cfg.period;
  hs.gate = h->cfg.update_gate;
  hs.contact = h->has_sphere;
  HIPCHK(h, hipMemcpyAsync(h->st, &hs, sizeof(DevState), hipMemcpyHostToDevice, s));
  const ContactDev ct = contact_dev(h);
  const WeakDev w = weak_dev(h);
  if (ct.on) launch_contact_init<double>(h->g, D.u, ct, s);
  const int nres = launch_delta_residual<float>(h->g, D, ct, h->st, h->part, h->nblk_res, 1, kind == 2, s);
  launch_delta_control<float>(h->g, D, ct, w, h->st, h->part, h->wpart, nres, s);
  // R difference as the Gram pass forms it, from the R ring (staged in the transform buffer)
  if (out[2]) launch_diff<float>(Rcur, Rprev, D.t, n3, s);
  const float* src[4] = {D.p[it & 1], Rcur, D.t, D.dY[slot]};
  for (int q = 0; q < 4; ++q)
    if (out[q]) launch_convert<float, double>(src[q], out[q], n3, s);
  if (sums) {
    std::vector<double> part(2 * (size_t)nres), wp(w.m + 1);   // columns ||p||^2, ||sigma||^2
    for (int q = 0; q < 2; ++q)
      HIPCHK(h, hipMemcpyAsync(part.data() + (size_t)q * nres, h->part + (size_t)q * kPartRows, 8 * (size_t)nres,
                               hipMemcpyDeviceToHost, s));
    if (w.m) HIPCHK(h, hipMemcpyAsync(wp.data(), h->wpart, 8 * w.m, hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    double a0 = 0, a1 = 0;
    for (int b = 0; b < nres; ++b) {
      a0 += part[b];
      a1 += part[(size_t)nres + b];
    }
    for (long long r = 0; r < w.m; ++r) a0 += wp[r];
    sums[0] = a0;
    sums[1] = a1;
  }
  HIPCHK(h, hipStreamSynchronize(s));
  return FFTC_OK;
}

template <typename T>
int stage_green_t(fftc_problem* h, const double* ptil_dev, double* u_dev) {
  Bufs<T> B = bufs<T>(h);
  hipStream_t s = h->stream;
  const long long n3 = 3 * h->Nn;
  launch_convert<double, T>(ptil_dev, B.X, n3, s);
  enqueue_green<T>(h, SRC_BUF, B.X, 0, 1);
  launch_convert<T, double>(B.u, u_dev, n3, s);
  HIPCHK(h, hipStreamSynchronize(s));
  return FFTC_OK;
}

// ---- static workspace (fftc_bind_workspace_static) ----
// One array per device, in this file: its device address comes from hipGetSymbolAddress
// (the array's name is only a host-side stand-in), looked up on the first static binding
// on each device with that device current.  Handles bound to it on one device share it: a
// new binding unbinds the previous one, whose later calls then report FFTC_E_STATE.
std::mutex g_static_mu;
void* g_static_ptr[kMaxDevices] = {};
fftc_problem* g_static_owner[kMaxDevices] = {};

void release_static(fftc_problem* h) {
  std::lock_guard<std::mutex> lk(g_static_mu);
  if (h->static_dev >= 0 && g_static_owner[h->static_dev] == h) g_static_owner[h->static_dev] = nullptr;
  h->static_dev = -1;
}

}  // namespace

extern "C" {

int fftc_create(fftc_h* out, const int32_t n[3], double hlen, int32_t scheme, int32_t precision) {
  if (!out || !n) return FFTC_E_ARG;
  *out = nullptr;
  if (precision != FFTC_FP64 && precision != FFTC_FP32) return FFTC_E_UNSUPPORTED;
  if (scheme != FFTC_TETRA2 && scheme != FFTC_HEX1) return FFTC_E_UNSUPPORTED;
  if (!(hlen > 0.0) || !isfinite(hlen)) return FFTC_E_ARG;
  for (int J = 0; J < 3; ++J)
    if (n[J] < 2 || n[J] > 4096) return FFTC_E_ARG;
  fftc_problem* h = new (std::nothrow) fftc_problem();
  if (!h) return FFTC_E_ARG;
  for (int J = 0; J < 3; ++J) {
    h->n[J] = n[J];
    std::vector<int> rad;
    if (!factor_ok(n[J], rad)) {
      delete h;
      return FFTC_E_UNSUPPORTED;
    }
    h->ap[J].n = n[J];
    h->ap[J].nrad = (int)rad.size();
    for (size_t q = 0; q < rad.size(); ++q) h->ap[J].rad[q] = rad[q];
  }
  h->precision = precision;
  h->scheme = scheme;
  h->hlen = hlen;
  h->ept = precision == FFTC_FP64 ? 8 : 16;
  memset(h->bc, FFTC_BC_NEUMANN, sizeof(h->bc));
  build_plan(h);
  h->Nv = (long long)n[0] * n[1] * n[2];
  if (3LL * (n[0] + 1LL) * (n[1] + 1LL) * (n[2] + 1LL) >= (1LL << 31)) {
    delete h;
    return FFTC_E_UNSUPPORTED;   // node indices are 32-bit inside the kernels
  }
  *out = h;
  return FFTC_OK;
}

void fftc_destroy(fftc_h h) {
  if (!h) return;
  release_static(h);
  delete h;
}

int fftc_set_bc(fftc_h h, const int8_t* bc) {
  if (!h || !bc) return FFTC_E_ARG;
  if (h->bound) return fail(h, FFTC_E_STATE, "boundary table must be set before binding the workspace");
  if (!h->s_comp.empty() || !h->w_comp.empty()) return fail(h, FFTC_E_STATE, "set the boundary table before constraints");
  for (int q = 0; q < 18; ++q)
    if (bc[q] < 0 || bc[q] > 2) return fail(h, FFTC_E_ARG, "boundary code out of range");
  for (int J = 0; J < 3; ++J) {
    int np = 0;
    for (int c = 0; c < 3; ++c)
      for (int f = 0; f < 2; ++f) np += bc[c * 6 + J * 2 + f] == FFTC_BC_PERIODIC;
    if (np != 0 && np != 6) return fail(h, FFTC_E_BC, "periodicity must hold on both faces of an axis for all components");
  }
  memcpy(h->bc, bc, 18);
  build_plan(h);
  return FFTC_OK;
}

int fftc_set_reference(fftc_h h, int32_t kind, double lam0, double mu0) {
  if (!h) return FFTC_E_ARG;
  if (kind != FFTC_REF_PAUX && kind != FFTC_REF_ISO) return fail(h, FFTC_E_ARG, "unknown reference medium");
  if (!(mu0 > 0.0) || !(lam0 + 2.0 * mu0 > 0.0) || !isfinite(lam0) || !isfinite(mu0))
    return fail(h, FFTC_E_ARG, "reference medium needs mu0 > 0 and lam0 + 2 mu0 > 0");
  if (h->bound && kind != h->ref_kind) return fail(h, FFTC_E_STATE, "choose the reference medium before binding");
  h->ref_kind = kind;
  h->lam0 = lam0;
  h->mu0 = mu0;
  h->ref_mode = 1;
  if (h->bound) set_stencil(h);
  return FFTC_OK;
}

int fftc_set_reference_factor(fftc_h h, int32_t kind, double factor) {
  if (!h) return FFTC_E_ARG;
  if (kind != FFTC_REF_PAUX && kind != FFTC_REF_ISO) return fail(h, FFTC_E_ARG, "unknown reference medium");
  if (!(factor > 0.0) || !isfinite(factor)) return fail(h, FFTC_E_ARG, "reference factor must be positive");
  if (h->bound && kind != h->ref_kind) return fail(h, FFTC_E_STATE, "choose the reference medium before binding");
  h->ref_kind = kind;
  h->r0_factor = factor;
  h->ref_mode = 0;
  return FFTC_OK;
}

static int add_dirichlet_host(fftc_h h, int64_t m, const int64_t* node, const int8_t* comp, const double* value,
                              int32_t set_id) {
  if (!h || m < 0 || (m > 0 && (!node || !comp || !value))) return FFTC_E_ARG;
  if (h->bound) return fail(h, FFTC_E_STATE, "constraints must be added before binding the workspace");
  if (set_id < 0 || set_id >= kMaxSets) return fail(h, FFTC_E_ARG, "set_id out of range");
  std::vector<long long> keys;
  for (int64_t e = 0; e < m; ++e) {
    const long long xyz[3] = {node[3 * e], node[3 * e + 1], node[3 * e + 2]};
    for (int J = 0; J < 3; ++J)
      if (xyz[J] < 0 || xyz[J] >= h->N[J]) return fail(h, FFTC_E_ARG, "constraint node out of range");
    if (comp[e] < 0 || comp[e] > 2) return fail(h, FFTC_E_ARG, "component out of range");
    if (!isfinite(value[e])) return fail(h, FFTC_E_ARG, "non-finite prescribed value");
    if (node_antisym(h, comp[e], xyz)) {
      if (value[e] != 0.0) return fail(h, FFTC_E_BC, "nonzero value on a DOF held at 0 by a Dirichlet face");
      continue;
    }
    const long long flat = node_flat(h, xyz[0], xyz[1], xyz[2]);
    const long long key = comp[e] * h->Nn + flat;
    if (h->dof_used.count(key) || std::find(keys.begin(), keys.end(), key) != keys.end())
      return fail(h, FFTC_E_ARG, "DOF constrained twice");
    keys.push_back(key);
  }
  size_t t = 0;
  for (int64_t e = 0; e < m; ++e) {
    const long long xyz[3] = {node[3 * e], node[3 * e + 1], node[3 * e + 2]};
    if (node_antisym(h, comp[e], xyz)) continue;
    h->s_node.push_back(node_flat(h, xyz[0], xyz[1], xyz[2]));
    h->s_comp.push_back(comp[e]);
    h->s_val.push_back(value[e] / h->hlen);
    h->s_set.push_back(set_id);
    h->dof_used.insert(keys[t++]);
  }
  return FFTC_OK;
}

static int add_average_host(fftc_h h, int64_t m, int32_t k, const int64_t* support, const int8_t* comp,
                            const double* value, int32_t set_id) {
  if (!h || m < 0 || (m > 0 && (!support || !comp || !value))) return FFTC_E_ARG;
  if (h->bound) return fail(h, FFTC_E_STATE, "constraints must be added before binding the workspace");
  if (k < 2 || k > kMaxRelSlots) return fail(h, FFTC_E_ARG, "support size must be 2..64 nodes");
  if (set_id < 0 || set_id >= kMaxSets) return fail(h, FFTC_E_ARG, "set_id out of range");
  std::unordered_set<long long> mine;
  for (int64_t r = 0; r < m; ++r) {
    if (comp[r] < 0 || comp[r] > 2) return fail(h, FFTC_E_ARG, "component out of range");
    if (!isfinite(value[r])) return fail(h, FFTC_E_ARG, "non-finite prescribed value");
    for (int q = 0; q < k; ++q) {
      const long long xyz[3] = {support[(r * k + q) * 3], support[(r * k + q) * 3 + 1], support[(r * k + q) * 3 + 2]};
      for (int J = 0; J < 3; ++J)
        if (xyz[J] < 0 || xyz[J] >= h->N[J]) return fail(h, FFTC_E_ARG, "support node out of range");
      if (node_antisym(h, comp[r], xyz)) return fail(h, FFTC_E_BC, "support node held at 0 by a Dirichlet face");
      const long long key = comp[r] * h->Nn + node_flat(h, xyz[0], xyz[1], xyz[2]);
      if (h->dof_used.count(key) || mine.count(key)) return fail(h, FFTC_E_OVERLAP, "overlapping constraint supports");
      mine.insert(key);
    }
  }
  for (int64_t r = 0; r < m; ++r) {
    for (int q = 0; q < k; ++q) {
      const int64_t* p = support + (r * k + q) * 3;
      h->w_nodes.push_back(node_flat(h, p[0], p[1], p[2]));
      h->w_a.push_back(1.0 / k);
      h->w_b.push_back(1.0);
      h->w_d.push_back(1.0);
    }
    h->w_off.push_back((long long)h->w_nodes.size());
    h->w_comp.push_back(comp[r]);
    h->w_val.push_back(value[r] / h->hlen);
    h->w_set.push_back(set_id);
  }
  for (long long key : mine) h->dof_used.insert(key);
  return FFTC_OK;
}

static int add_smooth_host(fftc_h h, int64_t m, const int64_t* node, const int8_t* comp, const double* value,
                           int32_t set_id) {
  if (!h || m < 0 || (m > 0 && (!node || !comp || !value))) return FFTC_E_ARG;
  if (h->bound) return fail(h, FFTC_E_STATE, "constraints must be added before binding the workspace");
  if (set_id < 0 || set_id >= kMaxSets) return fail(h, FFTC_E_ARG, "set_id out of range");
  // Table 2 weights by the number of non-zero offsets from the node
  static const double wvol[4] = {1.0, 0.5, 0.25, 0.125};   // centre, middle of faces, of edges, corners
  static const double wsurf[3] = {1.0, 0.5, 0.25};         // centre, middle of edges, corners
  struct Rel {
    std::vector<long long> nodes;
    std::vector<double> b;
  };
  std::vector<Rel> rels((size_t)m);
  std::unordered_set<long long> mine;
  for (int64_t r = 0; r < m; ++r) {
    const long long c0[3] = {node[3 * r], node[3 * r + 1], node[3 * r + 2]};
    for (int J = 0; J < 3; ++J)
      if (c0[J] < 0 || c0[J] >= h->N[J]) return fail(h, FFTC_E_ARG, "constraint node out of range");
    if (comp[r] < 0 || comp[r] > 2) return fail(h, FFTC_E_ARG, "component out of range");
    if (!isfinite(value[r])) return fail(h, FFTC_E_ARG, "non-finite prescribed value");
    int nface = 0, fax = -1;
    for (int J = 0; J < 3; ++J)
      if (!h->periodic[J] && (c0[J] == 0 || c0[J] == h->n[J])) {
        ++nface;
        fax = J;
      }
    if (nface > 1) return fail(h, FFTC_E_UNSUPPORTED, "smooth condition on an edge or corner node of the cell");
    Rel& R = rels[(size_t)r];
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int d[3] = {dx, dy, dz};
          if (fax >= 0 && d[fax] != 0) continue;       // surface node: neighbours in the face plane
          long long xyz[3];
          int nz = 0;
          for (int J = 0; J < 3; ++J) {
            long long x = c0[J] + d[J];
            nz += d[J] != 0;
            if (h->periodic[J]) x = (x + h->N[J]) % h->N[J];
            else if (x < 0 || x > h->n[J]) return fail(h, FFTC_E_ARG, "smooth support leaves the cell");
            xyz[J] = x;
          }
          if (node_antisym(h, comp[r], xyz))
            return fail(h, FFTC_E_BC, "smooth support holds a DOF held at 0 by a Dirichlet face");
          const long long flat = node_flat(h, xyz[0], xyz[1], xyz[2]);
          const long long key = comp[r] * h->Nn + flat;
          if (h->dof_used.count(key) || mine.count(key)) return fail(h, FFTC_E_OVERLAP, "overlapping constraint supports");
          mine.insert(key);
          const double w = fax >= 0 ? wsurf[nz] : wvol[nz];
          if (nz == 0) {        // the node itself leads its support
            R.nodes.insert(R.nodes.begin(), flat);
            R.b.insert(R.b.begin(), w);
          } else {
            R.nodes.push_back(flat);
            R.b.push_back(w);
          }
        }
  }
  for (int64_t r = 0; r < m; ++r) {
    const Rel& R = rels[(size_t)r];
    for (size_t q = 0; q < R.nodes.size(); ++q) {
      h->w_nodes.push_back(R.nodes[q]);
      h->w_a.push_back(q == 0 ? 1.0 : 0.0);
      h->w_b.push_back(R.b[q]);
      h->w_d.push_back(q == 0 ? 1.0 : 0.0);
    }
    h->w_off.push_back((long long)h->w_nodes.size());
    h->w_comp.push_back(comp[r]);
    h->w_val.push_back(value[r] / h->hlen);
    h->w_set.push_back(set_id);
  }
  for (long long key : mine) h->dof_used.insert(key);
  return FFTC_OK;
}

// The constraint calls take host or device arrays: device arrays are copied to the host first.
extern "C++" template <typename T>
static const T* host_view(const T* p, size_t count, std::vector<T>& tmp, bool& ok) {
  ok = true;
  if (!p || count == 0) return p;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) == hipSuccess && at.type == hipMemoryTypeDevice) {
    tmp.resize(count);
    ok = hipMemcpy(tmp.data(), p, count * sizeof(T), hipMemcpyDeviceToHost) == hipSuccess;
    return tmp.data();
  }
  (void)hipGetLastError();   // a plain host pointer is not registered with the runtime
  return p;
}

int fftc_add_dirichlet(fftc_h h, int64_t m, const int64_t* node, const int8_t* comp, const double* value,
                       int32_t set_id) {
  if (!h || m < 0) return FFTC_E_ARG;
  std::vector<int64_t> tn;
  std::vector<int8_t> tc;
  std::vector<double> tv;
  bool o1, o2, o3;
  const int64_t* n2 = host_view(node, 3 * (size_t)m, tn, o1);
  const int8_t* c2 = host_view(comp, (size_t)m, tc, o2);
  const double* v2 = host_view(value, (size_t)m, tv, o3);
  if (!o1 || !o2 || !o3) return fail(h, FFTC_E_HIP, "copying constraint arrays from the device failed");
  return add_dirichlet_host(h, m, n2, c2, v2, set_id);
}

int fftc_add_average(fftc_h h, int64_t m, int32_t k, const int64_t* support, const int8_t* comp, const double* value,
                     int32_t set_id) {
  if (!h || m < 0 || k < 0) return FFTC_E_ARG;
  std::vector<int64_t> tn;
  std::vector<int8_t> tc;
  std::vector<double> tv;
  bool o1, o2, o3;
  const int64_t* n2 = host_view(support, 3 * (size_t)m * (size_t)k, tn, o1);
  const int8_t* c2 = host_view(comp, (size_t)m, tc, o2);
  const double* v2 = host_view(value, (size_t)m, tv, o3);
  if (!o1 || !o2 || !o3) return fail(h, FFTC_E_HIP, "copying constraint arrays from the device failed");
  return add_average_host(h, m, k, n2, c2, v2, set_id);
}

int fftc_add_smooth(fftc_h h, int64_t m, const int64_t* node, const int8_t* comp, const double* value, int32_t set_id) {
  if (!h || m < 0) return FFTC_E_ARG;
  std::vector<int64_t> tn;
  std::vector<int8_t> tc;
  std::vector<double> tv;
  bool o1, o2, o3;
  const int64_t* n2 = host_view(node, 3 * (size_t)m, tn, o1);
  const int8_t* c2 = host_view(comp, (size_t)m, tc, o2);
  const double* v2 = host_view(value, (size_t)m, tv, o3);
  if (!o1 || !o2 || !o3) return fail(h, FFTC_E_HIP, "copying constraint arrays from the device failed");
  return add_smooth_host(h, m, n2, c2, v2, set_id);
}

int fftc_set_sphere(fftc_h h, const double center[3], double radius, int32_t face) {
  if (!h || !center) return FFTC_E_ARG;
  if (h->bound) return fail(h, FFTC_E_STATE, "set the obstacle before binding the workspace");
  if (!(radius > 0.0) || face < 0 || face > 5) return fail(h, FFTC_E_ARG, "invalid sphere");
  if (h->periodic[face / 2]) return fail(h, FFTC_E_ARG, "contact face on a periodic axis");
  h->has_sphere = 1;
  for (int c = 0; c < 3; ++c) h->center[c] = center[c] / h->hlen;
  h->radius = radius / h->hlen;
  h->face = face;
  int t = 0, bb[2];
  for (int J = 0; J < 3; ++J)
    if (J != face / 2) bb[t++] = J;
  h->b1 = bb[0];
  h->b2 = bb[1];
  return FFTC_OK;
}

int fftc_move_sphere(fftc_h h, const double center[3]) {
  if (!h || !center || !h->has_sphere) return FFTC_E_ARG;
  for (int c = 0; c < 3; ++c) h->center[c] = center[c] / h->hlen;
  return FFTC_OK;
}

int fftc_set_kinematics(fftc_h h, int32_t kind) {
  if (!h) return FFTC_E_ARG;
  if (kind != FFTC_SMALL_STRAIN && kind != FFTC_FINITE_STRAIN) return fail(h, FFTC_E_ARG, "unknown kinematics");
  h->fs = kind == FFTC_FINITE_STRAIN;
  h->g.fs = h->fs;
  return FFTC_OK;
}

int fftc_set_solver(fftc_h h, const fftc_solver_cfg* cfg) {
  if (!h || !cfg) return FFTC_E_ARG;
  if (cfg->depth != 4) return fail(h, FFTC_E_UNSUPPORTED, "Anderson depth must be 4");
  if (cfg->period < 1 || cfg->max_iter < 0 || !(cfg->tol >= 0.0) || cfg->acv < 0 || cfg->acv > 2 ||
      !(cfg->refine_below >= 0.0) || cfg->anchor_every < 0)
    return fail(h, FFTC_E_ARG, "invalid solver settings");
  if (h->bound && cfg->acv == FFTC_ACV_U && h->nlit < 10)
    return fail(h, FFTC_E_STATE, "ACV_U in FP32 needs its Anderson fields: set it before binding the workspace");
  h->cfg = *cfg;
  return FFTC_OK;
}

int fftc_workspace_bytes(fftc_h h, size_t* bytes) {
  if (!h || !bytes) return FFTC_E_ARG;
  *bytes = carve(h, nullptr);
  return FFTC_OK;
}

namespace {
// Binds ws to h: carves the fields, uploads tables and constraints, and (tune) times the two
// block sizes of every transform pass; without tuning every pass takes the larger block.
int bind_impl(fftc_h h, void* ws, size_t bytes, void* stream, bool tune) {
  if (!h || !ws) return FFTC_E_ARG;
  if (h->scheme == FFTC_HEX1 && h->precision != FFTC_FP64)
    return fail(h, FFTC_E_UNSUPPORTED, "the HEX1 scheme runs in FP64 (its hourglass modes have no FP32 residual form)");
  if (h->scheme == FFTC_HEX1 && h->has_sphere) return fail(h, FFTC_E_UNSUPPORTED, "contact uses the TETRA2 scheme");
  if (h->ref_kind == FFTC_REF_ISO &&
      (h->scheme != FFTC_HEX1 || !((h->periodic[0] && h->periodic[1] && h->periodic[2]) || normal_mixed(h))))
    return fail(h, FFTC_E_UNSUPPORTED,
                "the isotropic reference medium needs HEX1 and periodic axes or normal-mixed faces");
  if (((uintptr_t)ws) % kAlign) return fail(h, FFTC_E_WORKSPACE, "workspace must be 256-byte aligned");
  const size_t need = carve(h, nullptr);
  if (bytes < need) return fail(h, FFTC_E_WORKSPACE, "workspace too small");
  // contact face nodes may not carry other constraints
  if (h->has_sphere) {
    const int a = h->face / 2;
    const long long fc = (h->face % 2) ? h->n[a] : 0;
    for (size_t e = 0; e < h->s_node.size(); ++e) {
      long long nd = h->s_node[e];
      const long long xyz[3] = {nd % h->N[0], (nd / h->N[0]) % h->N[1], nd / ((long long)h->N[0] * h->N[1])};
      if (xyz[a] == fc) return fail(h, FFTC_E_OVERLAP, "strong constraint on a potential contact node");
    }
    for (size_t e = 0; e < h->w_nodes.size(); ++e) {
      long long nd = h->w_nodes[e];
      const long long xyz[3] = {nd % h->N[0], (nd / h->N[0]) % h->N[1], nd / ((long long)h->N[0] * h->N[1])};
      if (xyz[a] == fc) return fail(h, FFTC_E_OVERLAP, "average relation on a potential contact node");
    }
  }
  h->ws = (char*)ws;
  h->ws_bytes = bytes;
  h->stream = (hipStream_t)stream;
  carve(h, h->ws);
  hipStream_t s = h->stream;
  // geometry
  Geo& g = h->g;
  for (int J = 0; J < 3; ++J) {
    g.n[J] = h->n[J];
    g.N[J] = h->N[J];
    g.periodic[J] = h->periodic[J];
  }
  g.Nn = h->Nn;
  g.Nv = h->Nv;
  g.aface = h->aface;
  g.fs = h->fs;
  g.hex = h->scheme == FFTC_HEX1;
  g.iso = h->ref_kind != FFTC_REF_ISO ? 0 : (h->periodic[0] && h->periodic[1] && h->periodic[2]) ? 1 : 2;
  for (int J = 0; J < 3; ++J) {
    const int tn = h->type[J][J];   // the normal component's transform on axis J
    g.iso_axis[J] = ((tn == T_DCT3 || tn == T_DST3) ? 1 : 0) | ((tn == T_DST1 || tn == T_DST3) ? 2 : 0);
  }
  // singular modes of each component: theta = 0 needs DCT1 or DFT on all axes; theta = pi
  // additionally needs an even length on DFT axes
  for (int c = 0; c < 3; ++c) {
    int zero = 1, pi = 1;
    double sc = 1.0;
    for (int J = 0; J < 3; ++J) {
      const int ty = h->type[c][J];
      if (ty == T_DCT1) sc /= 2.0 * h->n[J];
      else if (ty == T_DFT) {
        sc /= h->n[J];
        if (h->n[J] % 2) pi = 0;
      } else {
        zero = pi = 0;
      }
    }
    g.sing[c] = zero ? (1 | (pi ? 2 : 0)) : 0;
    g.sing_scale[c] = sc;
  }
  // axis plans: twiddles e^{-2 pi i t/4n}, lines per block
  for (int J = 0; J < 3; ++J) {
    AxisPlan& ap = h->ap[J];
    ap.N = h->N[J];
    ap.L = std::max(1, h->ept * kBlock / ap.n);
    const int n = ap.n;
    std::vector<double> twd(8 * n);
    std::vector<float> twf(8 * n);
    for (int t = 0; t < 4 * n; ++t) {
      const long double ang = 2.0L * 3.14159265358979323846264338327950288L * (long double)t / (4.0L * n);
      const long double c = cosl(ang), sn = -sinl(ang);
      twd[2 * t] = (double)c;
      twd[2 * t + 1] = (double)sn;
      twf[2 * t] = (float)c;
      twf[2 * t + 1] = (float)sn;
    }
    if (h->precision == FFTC_FP64)
      HIPCHK(h, hipMemcpyAsync(h->tw[J], twd.data(), 8 * twd.size(), hipMemcpyHostToDevice, s));
    else
      HIPCHK(h, hipMemcpyAsync(h->tw[J], twf.data(), 4 * twf.size(), hipMemcpyHostToDevice, s));
    ap.tw = h->tw[J];
    // LDS budget: keep one block within 64 KiB
    const size_t cs = h->precision == FFTC_FP64 ? 16 : 8, rs = cs / 2;
    while (ap.L > 1 && ap.L * ((n + 1) * cs + (ap.N + 1) * rs) > 65536) ap.L /= 2;
    if (!dtt_covered(h->ept, ap)) return fail(h, FFTC_E_UNSUPPORTED, "transform line too long for one block");
  }
  // symbol tables cos(theta) per (comp, axis)
  std::vector<double> cosT(18 * (size_t)h->maxN, 0.0);
  for (int c = 0; c < 3; ++c)
    for (int J = 0; J < 3; ++J)
      for (int idx = 0; idx < h->N[J]; ++idx) {
        const int ty = h->type[c][J], nJ = h->n[J];
        // theta = pi exactly at the last DCT1/DST1 index and at n/2 of a DFT axis
        const bool at_pi = ((ty == T_DCT1 || ty == T_DST1) && idx == nJ) ||
                           (ty == T_DFT && 2 * std::min(idx, nJ - idx) == nJ);
        const double half = 0.5 * theta_of(ty, nJ, idx);
        const double sn = sin(half), cs = cos(half);
        cosT[((c * 3 + J) * 2 + 0) * h->maxN + idx] = at_pi ? 1.0 : sn * sn;
        cosT[((c * 3 + J) * 2 + 1) * h->maxN + idx] = at_pi ? 0.0 : cs * cs;
      }
  HIPCHK(h, hipMemcpyAsync(h->cosT, cosT.data(), 8 * cosT.size(), hipMemcpyHostToDevice, s));
  // the same tables rounded to FP32, read by the FP32 Green step
  std::vector<float> cosT32(cosT.begin(), cosT.end());
  HIPCHK(h, hipMemcpyAsync(h->cosT + cosT.size(), cosT32.data(), 4 * cosT32.size(), hipMemcpyHostToDevice, s));
  // node mask
  std::vector<uint8_t> mask(h->Nn, 0);
  for (size_t e = 0; e < h->s_node.size(); ++e) mask[h->s_node[e]] |= (uint8_t)(M_STRONG << h->s_comp[e]);
  for (size_t r = 0; r < h->w_comp.size(); ++r)
    for (long long q = h->w_off[r]; q < h->w_off[r + 1]; ++q) mask[h->w_nodes[q]] |= (uint8_t)(M_WEAK << h->w_comp[r]);
  if (h->has_sphere) {
    const int a = h->face / 2;
    const long long fc = (h->face % 2) ? h->n[a] : 0;
    for (long long nd = 0; nd < h->Nn; ++nd) {
      const long long xyz[3] = {nd % h->N[0], (nd / h->N[0]) % h->N[1], nd / ((long long)h->N[0] * h->N[1])};
      if (xyz[a] == fc) mask[nd] |= M_FACE;
    }
  }
  HIPCHK(h, hipMemcpyAsync(h->mask, mask.data(), h->Nn, hipMemcpyHostToDevice, s));
  const size_t ms = h->s_comp.size(), mw = h->w_comp.size();
  if (ms) {
    HIPCHK(h, hipMemcpyAsync(h->d_snode, h->s_node.data(), 8 * ms, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_scomp, h->s_comp.data(), ms, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_sval, h->s_val.data(), 8 * ms, hipMemcpyHostToDevice, s));
  }
  if (mw) {
    HIPCHK(h, hipMemcpyAsync(h->d_wnodes, h->w_nodes.data(), 8 * h->w_nodes.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_wcomp, h->w_comp.data(), mw, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_wval, h->w_val.data(), 8 * mw, hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_woff, h->w_off.data(), 8 * (mw + 1), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_wa, h->w_a.data(), 8 * h->w_a.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_wb, h->w_b.data(), 8 * h->w_b.size(), hipMemcpyHostToDevice, s));
    HIPCHK(h, hipMemcpyAsync(h->d_wd, h->w_d.data(), 8 * h->w_d.size(), hipMemcpyHostToDevice, s));
  }
  h->nblk_res = (int)std::min<long long>(kPartRows, (h->Nn + kBlock - 1) / kBlock);
  // autotune the block size of each transform pass: time both variants of the pass as the
  // iteration runs it (the FP32 form's x passes with their residual-form source and FP64
  // update), on the bound buffers with a cleared state (no acceleration, nothing done)
  if (!tune) {
    for (int p = 0; p < TP_N; ++p) h->dtt_nt[p] = h->precision == FFTC_FP64 ? 256 : 512;
  } else {
    HIPCHK(h, hipMemsetAsync(h->st, 0, sizeof(DevState), s));
    const bool delta = h->precision == FFTC_FP32 && h->nlit < 10;   // runs the residual form
    static const int axis[TP_N] = {0, 1, 2, 1, 0};
    static const int mode[TP_N] = {PASS_FWD, PASS_FWD, PASS_FWD_GREEN_INV, PASS_INV, PASS_INV};
    hipEvent_t e0, e1;
    HIPCHK(h, hipEventCreate(&e0));
    HIPCHK(h, hipEventCreate(&e1));
    const int cand[2] = {h->precision == FFTC_FP64 ? 128 : 256, h->precision == FFTC_FP64 ? 256 : 512};
    for (int p = 0; p < TP_N; ++p) {
      for (int v = 0; v < 2; ++v) {
        h->dtt_nt[p] = cand[v];
        float tot = 0.f;
        for (int rep = 0; rep < 3; ++rep) {
          HIPCHK(h, hipEventRecord(e0, s));
          if (h->precision == FFTC_FP64) launch_dtt<double>(dtt_args<double>(h, axis[p], mode[p], 1), h->ept, s);
          else if (delta) launch_dtt<float>(delta_pass(h, p, dbufs(h)), h->ept, s);
          else launch_dtt<float>(dtt_args<float>(h, axis[p], mode[p], 1), h->ept, s);
          HIPCHK(h, hipEventRecord(e1, s));
          HIPCHK(h, hipEventSynchronize(e1));
          float ms = 0.f;
          HIPCHK(h, hipEventElapsedTime(&ms, e0, e1));
          if (rep > 0) tot += ms;
        }
        h->tune_ms[p][v] = tot / 2;
      }
      h->dtt_nt[p] = (h->tune_ms[p][0] <= h->tune_ms[p][1]) ? cand[0] : cand[1];
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
  }
  // occupancy queries of the residual pass instances, outside any capture
  (void)residual_tiles(h->g, false);
  (void)residual_tiles(h->g, true);
  (void)residual_tiles_fp64(h->g, false);
  (void)residual_tiles_fp64(h->g, true);
  if (h->nblk_res >= 8) h->nblk_res -= h->nblk_res % 8;   // whole slabs per XCD
  if (h->nblk_res < 1) h->nblk_res = 1;
  for (int q = 0; q < h->nlit; ++q)
    HIPCHK(h, hipMemsetAsync(h->fld[q], 0, (h->precision == FFTC_FP64 ? 8 : 4) * 3 * (size_t)h->Nn, s));
  HIPCHK(h, hipStreamSynchronize(s));
  h->bound = 1;
  h->stiff_set = 0;
  if (h->ref_mode == 1) set_stencil(h);
  return FFTC_OK;
}

}  // namespace

int fftc_bind_workspace(fftc_h h, void* ws, size_t bytes, void* stream) {
  if (!h) return FFTC_E_ARG;
  release_static(h);
  return bind_impl(h, ws, bytes, stream, true);
}

int fftc_bind_workspace_static(fftc_h h, void* stream) {
  if (!h) return FFTC_E_ARG;
  const size_t need = carve(h, nullptr);
  if (need > kStaticWsBytes)
    return fail(h, FFTC_E_WORKSPACE, "problem needs " + std::to_string(need) + " bytes of workspace, the static "
                                     "workspace holds " + std::to_string(kStaticWsBytes));
  int dev = -1;
  HIPCHK(h, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(h, FFTC_E_UNSUPPORTED, "device index beyond the static table");
  void* ptr = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_static_mu);
    if (!g_static_ptr[dev]) {
      const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !ptr) return fail(h, FFTC_E_HIP, std::string("HIP: ") + hipGetErrorString(e));
      g_static_ptr[dev] = ptr;
    }
    ptr = g_static_ptr[dev];
    fftc_problem* prev = g_static_owner[dev];
    if (prev && prev != h) {   // its fields are about to be overwritten
      prev->bound = 0;
      prev->stiff_set = 0;
      prev->static_dev = -1;
      prev->err = "the static workspace was bound to another problem";
    }
    g_static_owner[dev] = h;
  }
  h->static_dev = dev;
  const int rc = bind_impl(h, ptr, kStaticWsBytes, stream, false);
  if (rc != FFTC_OK) release_static(h);
  return rc;
}

static int set_stiffness_impl(fftc_h h, const void* a, const void* b, int dtype, int enu) {
  if (!h || !a || !b) return FFTC_E_ARG;
  if (dtype != FFTC_F64 && dtype != FFTC_F32) return fail(h, FFTC_E_ARG, "unknown dtype");
  if (!h->bound) return fail(h, FFTC_E_STATE, "bind the workspace first");
  hipStream_t s = h->stream;
  const int nblk = (int)std::min<long long>(1024, (h->Nv + kBlock - 1) / kBlock);
  h->stiff_set = 0;
  launch_stiffness_in(a, b, dtype == FFTC_F32, enu, h->Nv, h->lam, h->mu, h->precision == FFTC_FP32, h->chk, nblk, s);
  std::vector<double> chk(3 * nblk);
  HIPCHK(h, hipMemcpyAsync(chk.data(), h->chk, 8 * chk.size(), hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  double bad = 0, ml = -INFINITY, mm = -INFINITY;
  for (int k = 0; k < nblk; ++k) {
    bad = std::max(bad, chk[3 * k]);
    ml = std::max(ml, chk[3 * k + 1]);
    mm = std::max(mm, chk[3 * k + 2]);
  }
  if (bad >= 2.0) return fail(h, FFTC_E_NAN, "non-finite stiffness");
  if (bad >= 1.0)
    return fail(h, FFTC_E_ARG, enu ? "stiffness must satisfy E >= 0 and -1 < nu < 1/2"
                                   : "stiffness must satisfy mu >= 0 and 3 lam + 2 mu >= 0");
  if (h->ref_mode == 0) {
    h->lam0 = h->r0_factor * ml;
    h->mu0 = h->r0_factor * mm;
    if (!(h->mu0 > 0.0) || !(h->lam0 + 2 * h->mu0 > 0.0)) return fail(h, FFTC_E_ARG, "degenerate reference medium");
  }
  set_stencil(h);
  h->stiff_set = 1;
  return FFTC_OK;
}

int fftc_set_stiffness(fftc_h h, const void* lam_dev, const void* mu_dev, int32_t dtype) {
  return set_stiffness_impl(h, lam_dev, mu_dev, dtype, 0);
}

int fftc_set_stiffness_Enu(fftc_h h, const void* E_dev, const void* nu_dev, int32_t dtype) {
  return set_stiffness_impl(h, E_dev, nu_dev, dtype, 1);
}

int fftc_solve(fftc_h h, double* u_dev, int32_t zero_start, fftc_report* rep) {
  if (!h) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set before solving");
  return solve_all(h, u_dev, zero_start, rep);
}

int fftc_batch_create(fftc_batch_h* out, int32_t count, const fftc_h* cells, void* stream) {
  if (!out || count < 1 || !cells) return FFTC_E_ARG;
  *out = nullptr;
  for (int c = 0; c < count; ++c)
    if (!cells[c] || !cells[c]->bound || !cells[c]->stiff_set) return FFTC_E_STATE;
  // Cells with a rigid obstacle are not batched: solve them with fftc_solve.
  for (int c = 0; c < count; ++c)
    if (cells[c]->has_sphere) return fail(cells[c], FFTC_E_UNSUPPORTED, "contact cells are not batched");
  // FP64 cells are not batched either: a batched FP64 solve once ended the process with an
  // abort that no reading of this path explains; solve them with fftc_solve.
  for (int c = 0; c < count; ++c)
    if (cells[c]->precision == FFTC_FP64) return fail(cells[c], FFTC_E_UNSUPPORTED, "FP64 cells are not batched");
  fftc_batch* b = new (std::nothrow) fftc_batch();
  if (!b) return FFTC_E_ARG;
  b->cells.assign(cells, cells + count);
  b->origin = (hipStream_t)stream;
  const int K = std::min(count, 16);
  b->streams.resize(K);
  b->join.resize(K);
  bool ok = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) == hipSuccess &&
            hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) == hipSuccess;
  for (int k = 0; k < K && ok; ++k) {
    ok = hipStreamCreateWithFlags(&b->streams[k], hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&b->join[k], hipEventDisableTiming) == hipSuccess;
  }
  ok = ok && hipHostMalloc((void**)&b->pinned, sizeof(DevState) * count, hipHostMallocDefault) == hipSuccess;
  if (!ok) {
    fftc_batch_destroy(b);
    return FFTC_E_HIP;
  }
  *out = b;
  return FFTC_OK;
}

void fftc_batch_destroy(fftc_batch_h b) {
  if (!b) return;
  for (auto s : b->streams)
    if (s) hipStreamDestroy(s);
  for (auto e : b->join)
    if (e) hipEventDestroy(e);
  if (b->fork) hipEventDestroy(b->fork);
  if (b->ready) hipEventDestroy(b->ready);
  if (b->cap) hipStreamDestroy(b->cap);
  if (b->pinned) hipHostFree(b->pinned);
  delete b;
}

int fftc_batch_solve(fftc_batch_h b, double* const* u_dev, int32_t zero_start, fftc_report* reps) {
  if (!b) return FFTC_E_ARG;
  const int n = (int)b->cells.size();
  const int K = (int)b->streams.size();
  hipStream_t s0 = b->origin;
  std::vector<hipStream_t> saved(n);
  for (int c = 0; c < n; ++c) {
    saved[c] = b->cells[c]->stream;
    b->cells[c]->stream = s0;
  }
  auto restore = [&]() {
    for (int c = 0; c < n; ++c) b->cells[c]->stream = saved[c];
  };
#define BCHK(call)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      restore();                                                                                \
      b->err = std::string("HIP: ") + hipGetErrorString(e_);                                    \
      return FFTC_E_HIP;                                                                        \
    }                                                                                           \
  } while (0)
  // initial projections and device states, on the origin stream
  for (int c = 0; c < n; ++c) {
    const int rc = solve_init(b->cells[c], u_dev ? u_dev[c] : nullptr, zero_start || !u_dev);
    if (rc != FFTC_OK) {
      restore();
      b->err = "cell " + std::to_string(c) + ": " + b->cells[c]->err;
      return rc;
    }
  }
  // Capture iters_per_graph iterations of the unfinished cells as parallel branches.  The
  // graph is captured again whenever the set of unfinished cells shrinks, so finished cells
  // cost no launches.  Cells go to branches largest first, each to the least loaded branch.
  BCHK(hipEventRecord(b->ready, s0));
  BCHK(hipStreamWaitEvent(b->cap, b->ready, 0));
  const hipStream_t user = s0;
  s0 = b->cap;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  auto release = [&]() {
    if (exec) hipGraphExecDestroy(exec);
    if (graph) hipGraphDestroy(graph);
    exec = nullptr;
    graph = nullptr;
  };
  std::vector<int> order(n);
  for (int c = 0; c < n; ++c) order[c] = c;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int c) { return b->cells[a]->g.Nv > b->cells[c]->g.Nv; });
  std::vector<char> active(n, 1);
  auto capture = [&]() -> hipError_t {
    release();
    const int nb = std::min(K, (int)std::count(active.begin(), active.end(), 1));
    std::vector<double> load(nb, 0.0);
    hipError_t e = hipStreamBeginCapture(s0, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return e;
    hipEventRecord(b->fork, s0);
    for (int k = 0; k < nb; ++k) hipStreamWaitEvent(b->streams[k], b->fork, 0);
    for (int c : order) {
      if (!active[c]) continue;
      const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
      load[k] += (double)b->cells[c]->g.Nv;
      fftc_problem* h = b->cells[c];
      h->stream = b->streams[k];
      for (int it = 0; it < b->iters_per_graph; ++it) enqueue_iter(h);
      h->stream = s0;
    }
    for (int k = 0; k < nb; ++k) {
      hipEventRecord(b->join[k], b->streams[k]);
      hipStreamWaitEvent(s0, b->join[k], 0);
    }
    e = hipStreamEndCapture(s0, &graph);
    if (e != hipSuccess) return e;
    return hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  };
#undef BCHK
#define BCHK(call)                                                                              \
  do {                                                                                          \
    hipError_t e_ = (call);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      release();                                                                                \
      restore();                                                                                \
      b->err = std::string("HIP: ") + hipGetErrorString(e_);                                    \
      return FFTC_E_HIP;                                                                        \
    }                                                                                           \
  } while (0)
  BCHK(capture());
  // replay until every cell has set its done flag (each stops at its own max_iter at the latest)
  int chunk = 1;
  for (;;) {
    for (int t = 0; t < chunk; ++t) BCHK(hipGraphLaunch(exec, s0));
    for (int c = 0; c < n; ++c)
      if (active[c])
        BCHK(hipMemcpyAsync(&b->pinned[c], b->cells[c]->st, sizeof(DevState), hipMemcpyDeviceToHost, s0));
    BCHK(hipStreamSynchronize(s0));
    bool changed = false;
    for (int c = 0; c < n; ++c)
      if (active[c] && b->pinned[c].done) {
        active[c] = 0;
        changed = true;
      }
    if (std::count(active.begin(), active.end(), 1) == 0) break;
    if (changed) {
      BCHK(capture());
      chunk = 1;
    } else {
      chunk = std::min(16, chunk * 2);
    }
  }
  release();
  s0 = user;   // the replay stream is idle (synchronised above)
  int worst = FFTC_OK;
  for (int c = 0; c < n; ++c) {
    const int rc = solve_finish(b->cells[c], u_dev ? u_dev[c] : nullptr, reps ? &reps[c] : nullptr);
    if (rc == FFTC_E_HIP) {
      restore();
      return rc;
    }
    if (rc != FFTC_OK && worst == FFTC_OK) worst = rc;
  }
#undef BCHK
  restore();
  return worst;
}

int fftc_nn_features(fftc_h h, uint16_t* feat_dev, double* u1_dev) {
  if (!h || !feat_dev || !u1_dev) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set first");
  // first iterate from the plain start
  int rc = solve_init(h, nullptr, 1);
  if (rc != FFTC_OK) return rc;
  enqueue_iter(h);
  const long long n3 = 3 * h->Nn;
  if (h->delta_mode) {
    HIPCHK(h, hipMemcpyAsync(u1_dev, dbufs(h).u, 8 * n3, hipMemcpyDeviceToDevice, h->stream));
  } else if (h->precision == FFTC_FP64) {
    HIPCHK(h, hipMemcpyAsync(u1_dev, bufs<double>(h).u, 8 * n3, hipMemcpyDeviceToDevice, h->stream));
  } else {
    launch_convert<float, double>(bufs<float>(h).u, u1_dev, n3, h->stream);
  }
  nnk::FeatArgs a{};
  a.u1 = u1_dev;
  for (int J = 0; J < 3; ++J) {
    a.n[J] = h->n[J];
    a.N[J] = h->N[J];
    a.periodic[J] = h->periodic[J];
    a.center[J] = h->center[J];
  }
  a.Nn = h->Nn;
  a.Nv = h->Nv;
  a.aface = h->g.aface;
  a.lam = h->lam;
  a.mu = h->mu;
  a.fp64 = h->precision == FFTC_FP64;
  a.mask = h->mask;
  a.ms = (long long)h->s_comp.size();
  a.snode = h->d_snode;
  a.scomp = h->d_scomp;
  a.sval = h->d_sval;
  a.s_u = 1e-3 * (double)std::min(h->n[0], std::min(h->n[1], h->n[2]));
  a.has_sphere = h->has_sphere;
  a.radius = h->radius;
  a.face = h->face;
  a.scratch = h->gpart;
  a.feat = feat_dev;
  nnk::launch_features(a, h->stream);
  if (h->hlen != 1.0) launch_scale(u1_dev, n3, h->hlen, h->stream);   // channels in voxel units, u1 physical
  HIPCHK(h, hipGetLastError());
  return FFTC_OK;
}

namespace {

// Equilibrium residual of a start: the solver's own initialisation (proj_U, contact set),
// then one iteration, whose convergence test measures the start.
int start_residual(fftc_problem* h, const double* u0, double* res) {
  int rc = solve_init(h, u0, u0 ? 0 : 1);
  if (rc != FFTC_OK) return rc;
  enqueue_iter(h);
  HIPCHK(h, hipMemcpyAsync(&h->last, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(h, hipStreamSynchronize(h->stream));
  *res = h->last.residual;
  return FFTC_OK;
}

}  // namespace

int fftc_solve_judged(fftc_h h, const double* u0_dev, double* u_dev, fftc_report* rep, int32_t* used_u0,
                      double* residual_host) {
  if (!h || !u_dev) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set before solving");
  double r_nn = INFINITY, r_plain = INFINITY;
  int rc;
  if (u0_dev && (rc = start_residual(h, u0_dev, &r_nn)) != FFTC_OK) return rc;
  if ((rc = start_residual(h, nullptr, &r_plain)) != FFTC_OK) return rc;
  const int use = (u0_dev && r_nn < r_plain) ? 1 : 0;   // a non-finite r_nn falls back
  if (used_u0) *used_u0 = use;
  if (residual_host) {
    residual_host[0] = r_nn;
    residual_host[1] = r_plain;
  }
  if (use && u0_dev != u_dev)
    HIPCHK(h, hipMemcpyAsync(u_dev, u0_dev, 8 * 3 * (size_t)h->Nn, hipMemcpyDeviceToDevice, h->stream));
  rc = solve_all(h, u_dev, use ? 0 : 1, rep);
  if (use && (rc == FFTC_E_NOCONV || rc == FFTC_E_NAN)) {
    // the plain iteration finishes the solve: fall back to the plain start
    if (used_u0) *used_u0 = 0;
    rc = solve_all(h, u_dev, 1, rep);
  }
  return rc;
}

const char* fftc_batch_last_error(fftc_batch_h b) { return b ? b->err.c_str() : "null batch"; }

int fftc_get_reactions(fftc_h h, double* per_dof, double* per_rel, double* totals, int32_t nsets) {
  if (!h) return FFTC_E_ARG;
  if (per_dof) memcpy(per_dof, h->react_strong.data(), 8 * h->react_strong.size());
  if (per_rel) memcpy(per_rel, h->react_weak.data(), 8 * h->react_weak.size());
  if (totals) {
    if (nsets < 0) return FFTC_E_ARG;
    for (int q = 0; q < 3 * nsets; ++q) totals[q] = 0.0;
    for (size_t e = 0; e < h->react_strong.size(); ++e)
      if (h->s_set[e] < nsets) totals[h->s_set[e] * 3 + h->s_comp[e]] += h->react_strong[e];
    for (size_t r = 0; r < h->react_weak.size(); ++r)
      if (h->w_set[r] < nsets) totals[h->w_set[r] * 3 + h->w_comp[r]] += h->react_weak[r];
  }
  return FFTC_OK;
}

int fftc_num_constraints(fftc_h h, int64_t* ns, int64_t* nw) {
  if (!h) return FFTC_E_ARG;
  if (ns) *ns = (int64_t)h->s_comp.size();
  if (nw) *nw = (int64_t)h->w_comp.size();
  return FFTC_OK;
}

int fftc_num_face_nodes(fftc_h h, int64_t* count) {
  if (!h || !count) return FFTC_E_ARG;
  *count = h->has_sphere ? (int64_t)h->nface : 0;
  return FFTC_OK;
}

int fftc_get_contact(fftc_h h, uint8_t* mask, double* fnc, double* gap, double* force, double* area) {
  if (!h || !h->has_sphere || !h->bound) return FFTC_E_ARG;
  hipStream_t s = h->stream;
  std::vector<uint8_t> m((size_t)h->nface);
  HIPCHK(h, hipMemcpyAsync(m.data(), h->C, h->nface, hipMemcpyDeviceToHost, s));
  if (fnc) HIPCHK(h, hipMemcpyAsync(fnc, h->fnc, 8 * h->nface, hipMemcpyDeviceToHost, s));
  if (gap) HIPCHK(h, hipMemcpyAsync(gap, h->gap, 8 * h->nface, hipMemcpyDeviceToHost, s));
  HIPCHK(h, hipStreamSynchronize(s));
  const double h2 = h->hlen * h->hlen;
  if (mask) memcpy(mask, m.data(), m.size());
  if (fnc)
    for (long long f = 0; f < h->nface; ++f) fnc[f] *= h2;
  if (gap)
    for (long long f = 0; f < h->nface; ++f) gap[f] *= h->hlen;
  if (force) *force = h->last_force;
  if (area) {
    // tributary face area of every node of C: half a voxel face along an edge of the face
    double A = 0.0;
    const int N1 = h->N[h->b1], N2 = h->N[h->b2];
    for (long long f = 0; f < h->nface; ++f) {
      if (!m[f]) continue;
      const int i1 = (int)(f % N1), i2 = (int)(f / N1);
      const double w1 = (!h->periodic[h->b1] && (i1 == 0 || i1 == h->n[h->b1])) ? 0.5 : 1.0;
      const double w2 = (!h->periodic[h->b2] && (i2 == 0 || i2 == h->n[h->b2])) ? 0.5 : 1.0;
      A += w1 * w2;
    }
    *area = A * h2;
  }
  return FFTC_OK;
}

int fftc_stage_residual(fftc_h h, const double* u_dev, double* p_dev, double* ptil_dev, double* sums) {
  if (!h || !u_dev) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set");
  return h->precision == FFTC_FP64 ? stage_residual_t<double>(h, u_dev, p_dev, ptil_dev, sums)
                                   : stage_residual_t<float>(h, u_dev, p_dev, ptil_dev, sums);
}

int fftc_stage_residual_form(fftc_h h, const double* u_dev, const double* delta_dev, const double* e_dev,
                             const double* pprev_dev, const double* rprev_dev, int32_t i_local, int32_t pass_kind,
                             double* p_dev, double* r_dev, double* dr_dev, double* dy_dev, double* sums_host) {
  if (!h || !u_dev || i_local < 0 || pass_kind < 0 || pass_kind > 2) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set");
  if (h->precision != FFTC_FP32) return fail(h, FFTC_E_UNSUPPORTED, "the residual form is the FP32 iteration");
  if (pass_kind == 2 && (h->fs || h->has_sphere || h->g.sing[0] || h->g.sing[1] || h->g.sing[2] ||
                         residual_tiles(h->g, false).tx <= 0))
    return fail(h, FFTC_E_UNSUPPORTED, "the incremental pass is for tiled small-strain problems without obstacle "
                                       "or singular modes");
  const double* in[5] = {u_dev, delta_dev, e_dev, pprev_dev, rprev_dev};
  double* out[4] = {p_dev, r_dev, dr_dev, dy_dev};
  return stage_residual_form_t(h, in, i_local, pass_kind, out, sums_host);
}

int fftc_stage_green(fftc_h h, const double* ptil_dev, double* u_dev) {
  if (!h || !ptil_dev || !u_dev) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set");
  return h->precision == FFTC_FP64 ? stage_green_t<double>(h, ptil_dev, u_dev)
                                   : stage_green_t<float>(h, ptil_dev, u_dev);
}

const char* fftc_status_str(int status) {
  switch (status) {
    case FFTC_OK: return "ok";
    case FFTC_E_ARG: return "invalid argument";
    case FFTC_E_BC: return "inconsistent boundary condition";
    case FFTC_E_OVERLAP: return "overlapping constraints";
    case FFTC_E_WORKSPACE: return "workspace missing or too small";
    case FFTC_E_NOCONV: return "not converged";
    case FFTC_E_NAN: return "non-finite value";
    case FFTC_E_UNSUPPORTED: return "unsupported";
    case FFTC_E_STATE: return "call out of order";
    case FFTC_E_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

const char* fftc_last_error(fftc_h h) { return h ? h->err.c_str() : "null handle"; }

int fftc_iterate(fftc_h h, int32_t iters) {
  if (!h || iters < 0) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set");
  launch_extend(h->st, iters, 0.0, h->stream);
  for (int t = 0; t < iters; ++t) {
    if (h->precision == FFTC_FP64) enqueue_iteration<double>(h);
    else enqueue_iteration<float>(h);
  }
  HIPCHK(h, hipGetLastError());
  return FFTC_OK;
}

int fftc_profile_stages(fftc_h h, int32_t iters, double* ms, int32_t nstages) {
  if (!h || !ms || iters < 1 || nstages < 0) return FFTC_E_ARG;
  if (!h->bound || !h->stiff_set) return fail(h, FFTC_E_STATE, "workspace and stiffness must be set");
  return h->precision == FFTC_FP64 ? profile_t<double>(h, iters, ms, nstages) : profile_t<float>(h, iters, ms, nstages);
}

}  // extern "C"
