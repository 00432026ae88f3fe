// Host-callable launchers of the libfftc kernels (instantiated for float and double).
#pragma once
#include "fftc_internal.h"

namespace fftc {

template <typename T>
void launch_residual(const Geo& g, const Bufs<T>& B, const ContactDev& ct, DevState* st, double* part, int nblk,
                     int force, int write_p, hipStream_t s);
template <typename T>
void launch_weak(const Geo& g, const Bufs<T>& B, const WeakDev& w, DevState* st, int force, hipStream_t s);
void launch_control(DevState* st, const double* part, int nblk, const double* wpart, long long nweak,
                    const ContactDev& ct, int pstride, hipStream_t s);
// Residual-form iteration, first half: the residual pass (returns the number of block
// partial rows it wrote), then the average relations and the control step over those rows.
// refine: also launch the FP64-stress pass (taken once the state's refinement flag is set);
// inc: also launch the incremental pass (taken between the state's full passes).
template <typename T>
int launch_delta_residual(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, DevState* st, double* part,
                          int nblk, int refine, int inc, hipStream_t s);
template <typename T>
void launch_delta_control(const Geo& g, const DeltaBufs<T>& D, const ContactDev& ct, const WeakDev& w, DevState* st,
                          const double* part, const double* wpart, int nblk, hipStream_t s);
// Tile grid of the tiled residual pass on the current device.  Its first call on a device
// queries the kernel's occupancy, which must not happen under stream capture: call it once
// outside capture (the workspace binding does) before capturing iterations.
TileGrid residual_tiles(const Geo& g, bool inc);
TileGrid residual_tiles_fp64(const Geo& g, bool gen);
template <typename T>
void launch_delta_anderson(const DeltaBufs<T>& D, long long n3, DevState* st, double* gpart, int nblk, hipStream_t s);
template <typename T>
void launch_delta_proj(const Geo& g, const DeltaBufs<T>& D, const StrongDev& sd, const WeakDev& w,
                       const ContactDev& ct, DevState* st, int force, int advance, hipStream_t s);
// out = a - b elementwise (FP32 R differences for the stage entry)
template <typename T>
void launch_diff(const T* a, const T* b, T* out, long long n, hipStream_t s);
// Mean stress of the residual-form iterate: per-block sums of the six components (xx, yy, zz,
// yz, xz, xy) times the voxel volume, rows of 6 in part; returns the number of rows.
template <typename T>
int launch_mean_stress_d(const Geo& g, const DeltaBufs<T>& D, double* part, hipStream_t s);
template <typename T>
void launch_reactions_d(const Geo& g, const DeltaBufs<T>& D, const StrongDev& sd, double* out, hipStream_t s);
template <typename T>
void launch_anderson(const Bufs<T>& B, long long n3, DevState* st, double* gpart, int nblk, hipStream_t s);
template <typename T>
void launch_flags_combine(const Bufs<T>& B, long long n3, DevState* st, int which, hipStream_t s);
template <typename T>
size_t dtt_smem(const AxisPlan& ap);
template <typename T>
void launch_dtt(const DttArgs<T>& a, int ept, hipStream_t s);
template <typename T>
void launch_proj(const Geo& g, T* u, const WeakDev& w, const ContactDev& ct, const StrongDev& sd, DevState* st,
                 int advance, int force, hipStream_t s);
template <typename T>
void launch_contact_init(const Geo& g, const T* u, const ContactDev& ct, hipStream_t s);
template <typename T>
void launch_contact_force(const Geo& g, const T* u, const ContactDev& ct, double* out, int nblk, hipStream_t s);
template <typename T>
void launch_reactions(const Geo& g, const Bufs<T>& B, const StrongDev& sd, double* out, hipStream_t s);
// out = (B)(in * f)
template <typename A, typename B>
void launch_convert(const A* in, B* out, long long n, hipStream_t s, double f = 1.0);
template <typename T>
void launch_zero_amask(const Geo& g, T* u, hipStream_t s);
void launch_extend(DevState* st, int iters, double tol, hipStream_t s);
// Isotropic reference medium on a cell periodic on every axis: Green solve on the forward
// half-complex coefficients of the three components (FP64).
void launch_green_iso(const Geo& g, double* buf, DevState* st, int force, hipStream_t s);
// Stiffness intake (lam, mu or E, nu; FP32 or FP64 in and out) with its checks, per-block
// (worst check, max lam, max mu) rows in out.
void launch_stiffness_in(const void* a, const void* b, int in_f32, int enu, long long nv, void* lam, void* mu,
                         int out_f32, double* out, int nblk, hipStream_t s);
void launch_scale(double* x, long long n, double f, hipStream_t s);

}  // namespace fftc
