// FP64 instances of the DTT pass kernels.
#include "fftc_dtt_kernels.h"

namespace fftc {
template void launch_dtt<double>(const DttArgs<double>&, int, hipStream_t);
template size_t dtt_smem<double>(const AxisPlan&);
}  // namespace fftc
