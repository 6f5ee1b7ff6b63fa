// FP64 tier of the sweep kernels.  Built without contraction (see
// build.py): every product and sum is rounded as written, with IEEE
// division, which reproduces a plain evaluation of each formula.
#include "sweep_kernels.h"

namespace mhd {
template hipError_t launch_fluid<double>(const SweepParams<double>&, int, const LaunchTuning&, hipStream_t);
template bool fused_cfl_possible<double>(int);
template hipError_t launch_magnetic<double>(const SweepParams<double>&, int, const LaunchTuning&, hipStream_t);
template hipError_t launch_magfluid<double>(const SweepParams<double>&, int, const LaunchTuning&, hipStream_t);
template hipError_t launch_magmagfluid<double>(const SweepParams<double>&, int, const LaunchTuning&, hipStream_t);
template hipError_t launch_batch_op<double>(const BatchParams<double>&, int, int, int, hipStream_t);
}  // namespace mhd
