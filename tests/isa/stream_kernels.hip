// The streaming kernels as lbm_step launches them by default, compiled on
// their own so that a CPU test can read their register use from the
// assembly (test_isa.py).
#include "../../paper_2211_03160_amd/csrc/kernels.hpp"

namespace lbm {
template __global__ void stream_kernel<StF32, 4, true, 5, 0>(StreamArgs<StF32>);
template __global__ void stream_kernel<StF32, 4, false, 5, 0>(StreamArgs<StF32>);
template __global__ void stream_kernel<StF16, 4, true, 3, 0>(StreamArgs<StF16>);
template __global__ void stream_kernel<StBF16, 4, true, 4, 0>(StreamArgs<StBF16>);
template __global__ void stream_kernel<StMix, 4, true, 4, 0>(StreamArgs<StMix>);
template __global__ void batch_stream_kernel<StF32, 8, true, 5, 0>(BatchStreamArgs<StF32>);
template __global__ void step_kernel<2, StF32>(StepArgs<StF32>);
template __global__ void step_kernel<3, StF32>(StepArgs<StF32>);
template __global__ void stream3_kernel<StF32>(Stream3Args<StF32>);
}  // namespace lbm
