// FP32 instances of the DTT pass kernels.
#include "fftc_dtt_kernels.h"

namespace fftc {
template void launch_dtt<float>(const DttArgs<float>&, int, hipStream_t);
template size_t dtt_smem<float>(const AxisPlan&);
}  // namespace fftc
