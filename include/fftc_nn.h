/*
 * fftc_nn -- learned warm start for the fftc solver (MI355X, gfx950).
 *
 * The paper closes (Section 6) by naming a better initial guess of the
 * fixed-point iteration as a way to cut its cost.  This part of the library
 * supplies one: a small neural operator on the solver's node grid maps the
 * problem data (stiffness, prescribed DOFs and values, obstacle gap) to an
 * initial displacement, the solver starts from it, and a judge falls back to
 * the plain start when the network's start is worse.  The iteration always
 * finishes the solve, so the network changes the cost, never the converged
 * answer beyond the solver tolerance.
 *
 * Network (width W = 32, head H = 64, m modes per axis, B blocks):
 *   x0  = f Wl^T + bl                                  (12 -> 32, per node)
 *   x_b = GELU(S_b(x_{b-1}) + x_{b-1} W_b^T + c_b)      b = 1..B
 *   h   = GELU(x_B Wp1^T + bp1);  y = h Wp2^T + bp2     (32 -> 64 -> 3)
 *   S(x)[i, o] = sum_k phi_k(i) sum_c Ws[k, o, c] xh[k, c],
 *   xh[k, c]   = (1 / Nn) sum_i phi_k(i) x[i, c],
 *   phi_k(i)   = cos(pi kx (x + 1/2) / Nx) cos(pi ky (y + 1/2) / Ny) cos(pi kz (z + 1/2) / Nz),
 *   k = (kz m + ky) m + kx with every index below m;  GELU(z) = z Phi(z) (erf form).
 * The network predicts a correction of the solver's own first iterate u1 (one
 * iteration from the plain start, i.e. the reference medium's response to the
 * prescribed data): the start is u0 = u1 + s_u y with s_u = 1e-3 min(n).
 * Training minimises the squared L2 misfit sum (y - t)^2 / (sum t^2 + sum b^2) to
 * t = (u* - u1) / s_u, u* a converged solve, relative to the size of the whole
 * field (b = u1 / s_u as stored in the input channels), with Adam (Kingma & Ba,
 * Algorithm 1).
 *
 * Arithmetic: GEMM-shaped steps (lift, spectral synthesis + pointwise term,
 * head, and every weight-gradient reduction over nodes) run on BF16 MFMA with
 * FP32 accumulation; activations are stored as BF16; the mode mixing, the
 * output layer, the loss and Adam run in FP32.
 *
 * Parameter vector (FP32, in this order, each row-major):
 *   Wl[32][12], bl[32], then per block b: Ws_b[m^3][32][32] (mode, out, in),
 *   W_b[32][32], c_b[32]; then Wp1[64][32], bp1[64], Wp2[3][64], bp2[3].
 *   Gradients use the same layout.
 *
 * Input channels (FFTC_NN_CHANNELS = 16 BF16 values per node, node-major,
 * channels 12..15 zero):
 *   0 E / max E, E averaged over the voxels around the node; 1 nu averaged
 *   likewise; 2-4 per component 1 where the DOF is prescribed (Dirichlet
 *   face or strong constraint); 5-7 per component prescribed value / s_u;
 *   8 on the contact face of a rigid sphere tanh(g / (8 s_u)) with g = |X - O| - R
 *   the gap of the undeformed node, else 0; 9-11 the first iterate u1 / s_u.
 *
 * Conventions are those of fftc.h: int status returns, *_dev device pointers
 * borrowed for the call, caller-owned device memory (a persistent state
 * buffer and a per-grid workspace), all device work on the bound stream.
 */
#ifndef FFTC_NN_H
#define FFTC_NN_H

#include <stddef.h>
#include <stdint.h>

#include "fftc.h"

#ifdef __cplusplus
extern "C" {
#endif

#define FFTC_NN_CHANNELS 16
#define FFTC_NN_WIDTH 32
#define FFTC_NN_HIDDEN 64

typedef struct fftc_nn* fftc_nn_h;

/* Network with m modes per axis (1..6) and `blocks` spectral blocks (0..8).
 * Host-side object; no device memory is touched. */
int fftc_nn_create(fftc_nn_h* out, int32_t modes, int32_t blocks);
void fftc_nn_destroy(fftc_nn_h nn);
int fftc_nn_num_params(fftc_nn_h nn, int64_t* count);

/* Persistent state: FP32 parameters, gradients, Adam moments and the BF16
 * weight images the kernels read.  The caller owns the buffer (256-byte
 * aligned, size from fftc_nn_state_bytes); binding it zeroes the gradients
 * and moments (enqueued on `stream`).  FFTC_E_WORKSPACE if too small. */
int fftc_nn_state_bytes(fftc_nn_h nn, size_t* bytes);
int fftc_nn_bind_state(fftc_nn_h nn, void* state_dev, size_t bytes, void* stream);

/* Per-grid workspace for a node grid N[3] = (Nx, Ny, Nz) (each 2..257).
 * training != 0 reserves what the backward pass needs.  Rebinding to
 * another grid keeps the state. */
int fftc_nn_workspace_bytes(fftc_nn_h nn, const int32_t N[3], int32_t training, size_t* bytes);
int fftc_nn_bind(fftc_nn_h nn, const int32_t N[3], int32_t training, void* ws_dev, size_t bytes,
                 void* stream);

/* Copy parameters in or out (FP32 device vector in the layout above).
 * Setting them refreshes the BF16 images and clears the Adam moments and
 * step counter. */
int fftc_nn_set_params(fftc_nn_h nn, const float* params_dev);
int fftc_nn_get_params(fftc_nn_h nn, float* params_dev);
int fftc_nn_get_grad(fftc_nn_h nn, float* grad_dev);

/* Input channels of a bound solver problem (stiffness set), written to
 * feat_dev[Nn][FFTC_NN_CHANNELS] (BF16 bits, round to nearest even) on the
 * problem's stream.  Runs the solver's initialisation and one iteration from
 * the plain start (Algorithm 1; Algorithm 2 with a sphere) and writes that
 * first iterate to u1_dev (FP64 component-planar [3][Nn], required); the
 * handle's iteration state is left there (the next solve starts afresh). */
int fftc_nn_features(fftc_h prob, uint16_t* feat_dev, double* u1_dev);

/* Forward pass on the bound grid.  y_dev (may be NULL): FP32 [Nn][3] network
 * output; u0_dev (may be NULL): FP64 component-planar [3][Nn] start
 * base + s_u * y, with base_dev the first iterate of fftc_nn_features (NULL
 * reads as zero). */
int fftc_nn_forward(fftc_nn_h nn, const uint16_t* feat_dev, float* y_dev, double s_u, const double* base_dev,
                    double* u0_dev);

/* One training sample: forward, loss and backward on a workspace bound with
 * training != 0.  target_dev: FP32 component-planar [3][Nn],
 * t = (u* - u1) / s_u (not all zero).  The gradient of the loss replaces the stored gradient;
 * loss_dev (may be NULL) receives the loss as one FP64 value. */
int fftc_nn_train_step(fftc_nn_h nn, const uint16_t* feat_dev, const float* target_dev, double* loss_dev);

/* Adam update of the parameters with the stored gradient (step counter
 * advanced first; bias corrections 1 - beta^step), then BF16 images
 * refreshed. */
int fftc_nn_adam_step(fftc_nn_h nn, float lr, float beta1, float beta2, float eps);

/* Training target t = (u* - u1) / s_u as FP32 (count values, component-planar like the
 * displacement) on the HIP stream given: u_dev a converged solve, u1_dev the first iterate of
 * fftc_nn_features, both FP64 device arrays.  Errors: FFTC_E_ARG, FFTC_E_HIP. */
int fftc_nn_make_target(const double* u_dev, const double* u1_dev, int64_t count, double s_u, float* target_dev,
                        void* stream);

/* Message of the last failing call on this network. */
const char* fftc_nn_last_error(fftc_nn_h nn);

/* Judged start (the plain iteration always finishes the solve): measures the
 * equilibrium residual of the projected start proj_U(u0) and of the plain
 * start, solves from u0 when its residual is smaller and from the plain
 * start otherwise.  A solve from u0 that does not converge (FFTC_E_NOCONV or
 * FFTC_E_NAN: with an obstacle, a start can hold a contact set the iteration
 * does not leave within max_iter) is repeated from the plain start, and its
 * result and report are those of that repeat.  *used_u0 = 1 when the returned
 * solution comes from u0; residual_host (may be NULL) receives {residual of u0,
 * residual of the plain start}.  Other arguments as fftc_solve. */
int fftc_solve_judged(fftc_h h, const double* u0_dev, double* u_dev, fftc_report* rep, int32_t* used_u0,
                      double* residual_host);

#ifdef __cplusplus
}
#endif

#endif
