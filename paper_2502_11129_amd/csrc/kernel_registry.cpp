// Table of compiled rollout kernel variants.
#include "launch.h"

namespace simk {

hipError_t launch_rollout_8_1_16(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_8_1_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_12_1_16(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_12_1_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_16_1_16(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_16_2_16(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_16_1_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_20_1_8(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_20_2_8(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_20_1_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_24_1_8(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_24_2_8(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_24_2_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_24_1_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_28_2_8(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_28_2_2(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_28_2_4(const BinArgs&, const ModelParams&, hipStream_t);
hipError_t launch_rollout_28_2_12(const BinArgs&, const ModelParams&, hipStream_t);

const KernelVariant kKernelVariants[] = {
    {8, 1, 16, launch_rollout_8_1_16},
    {8, 1, 2, launch_rollout_8_1_2},
    {12, 1, 16, launch_rollout_12_1_16},
    {12, 1, 2, launch_rollout_12_1_2},
    {16, 1, 16, launch_rollout_16_1_16},
    {16, 2, 16, launch_rollout_16_2_16},
    {16, 1, 2, launch_rollout_16_1_2},
    {20, 1, 8, launch_rollout_20_1_8},
    {20, 2, 8, launch_rollout_20_2_8},
    {20, 1, 2, launch_rollout_20_1_2},
    {24, 1, 8, launch_rollout_24_1_8},
    {24, 2, 8, launch_rollout_24_2_8},
    {24, 2, 2, launch_rollout_24_2_2},
    {24, 1, 2, launch_rollout_24_1_2},
    {28, 2, 8, launch_rollout_28_2_8},
    {28, 2, 2, launch_rollout_28_2_2},
    {28, 2, 4, launch_rollout_28_2_4},
    {28, 2, 12, launch_rollout_28_2_12},
};
const int kNumKernelVariants = sizeof(kKernelVariants) / sizeof(kKernelVariants[0]);

}  // namespace simk
