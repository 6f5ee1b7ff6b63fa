// FP32 tier of the sweep kernels: hardware reciprocal for divisions and the
// fused multiply-adds written out in the shared device functions.
#include "sweep_kernels.h"

namespace mhd {
template hipError_t launch_fluid<float>(const SweepParams<float>&, int, const LaunchTuning&, hipStream_t);
template bool fused_cfl_possible<float>(int);
template hipError_t launch_magnetic<float>(const SweepParams<float>&, int, const LaunchTuning&, hipStream_t);
template hipError_t launch_magfluid<float>(const SweepParams<float>&, int, const LaunchTuning&, hipStream_t);
template hipError_t launch_magmagfluid<float>(const SweepParams<float>&, int, const LaunchTuning&, hipStream_t);
template hipError_t launch_batch_op<float>(const BatchParams<float>&, int, int, int, hipStream_t);
}  // namespace mhd
