// Internal interface between the solver API and the warm-start network kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nnk {

// Input channels of one problem (layout and meaning in include/fftc_nn.h).
struct FeatArgs {
  int n[3], N[3], periodic[3];
  long long Nn, Nv;
  int aface;               // bit (c*6 + J*2 + f): component c held at 0 on face (J, f)
  const void* lam;         // voxel Lame fields, FP64 or FP32
  const void* mu;
  int fp64;
  const uint8_t* mask;     // node mask, bit (1 << c): strong constraint on component c
  long long ms;            // strong constraints
  const long long* snode;
  const int8_t* scomp;
  const double* sval;
  double s_u;              // displacement unit of the value channels
  int has_sphere;
  double center[3], radius;
  int face;
  const double* u1;        // first iterate, FP64 [3][Nn]
  double* scratch;         // >= 257 doubles of device scratch
  uint16_t* feat;          // [Nn][16] BF16
};

void launch_features(const FeatArgs& a, hipStream_t s);

}  // namespace nnk
