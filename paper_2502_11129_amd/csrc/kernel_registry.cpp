// Table of compiled rollout kernel variants.
#include "launch.h"

namespace simk {

#define SIMK_DECLARE(NVC, SB, NCR) \
  hipError_t launch_rollout_##NVC##_##SB##_##NCR(const BinArgs&, const ModelParams&, hipStream_t);
#define SIMK_DECLARE_BALL(NVC, SB, NCR) \
  hipError_t launch_rollout_ball_##NVC##_##SB##_##NCR(const BinArgs&, const ModelParams&, hipStream_t);
#define SIMK_DECLARE_SELF(NVC, SB, NCR) \
  hipError_t launch_rollout_self_##NVC##_##SB##_##NCR(const BinArgs&, const ModelParams&, hipStream_t);
#define SIMK_DECLARE_TREE(NVC, SB, NCR) \
  hipError_t launch_rollout_tree_##NVC##_##SB##_##NCR(const BinArgs&, const ModelParams&, hipStream_t);
#define SIMK_ENTRY_TREE(NVC, SB, NCR) {NVC, SB, NCR, 0, 0, launch_rollout_tree_##NVC##_##SB##_##NCR},
#define SIMK_ENTRY(NVC, SB, NCR) {NVC, SB, NCR, 0, 0, launch_rollout_##NVC##_##SB##_##NCR},
#define SIMK_ENTRY_BALL(NVC, SB, NCR) {NVC, SB, NCR, 1, 0, launch_rollout_ball_##NVC##_##SB##_##NCR},
#define SIMK_ENTRY_SELF(NVC, SB, NCR) {NVC, SB, NCR, 0, 1, launch_rollout_self_##NVC##_##SB##_##NCR},

// Plane-only kernels, kernels whose variants carry a ball, and kernels with
// self-collision.
#define SIMK_PLANE(X)                                                                        \
  X(8, 1, 16) X(8, 1, 2) X(12, 1, 16) X(12, 1, 2) X(16, 1, 16) X(16, 2, 16) X(16, 1, 2) X(16, 2, 8) X(16, 1, 8)    \
  X(20, 1, 8) X(20, 2, 8) X(20, 1, 2) X(20, 1, 4) X(24, 1, 8) X(24, 2, 8) X(24, 2, 2) X(24, 1, 2)        \
  X(28, 2, 8) X(28, 2, 2) X(28, 2, 4) X(28, 2, 12)
#define SIMK_BALL(X) X(12, 1, 8) X(12, 1, 2) X(16, 1, 8) X(20, 1, 8) X(24, 1, 8) X(28, 1, 8) X(28, 2, 8)
#define SIMK_SELF(X) X(12, 1, 8) X(12, 1, 2) X(16, 1, 8) X(20, 1, 8) X(24, 1, 8) X(24, 2, 8) X(28, 2, 8)

// Plane-only kernels that factor M~ tree-sparsely (L^T L) instead of the
// dense Gauss-Jordan sweep.
#define SIMK_TREE(X) X(24, 2, 8)

SIMK_PLANE(SIMK_DECLARE)
SIMK_TREE(SIMK_DECLARE_TREE)
SIMK_BALL(SIMK_DECLARE_BALL)
SIMK_SELF(SIMK_DECLARE_SELF)

const KernelVariant kKernelVariants[] = {SIMK_PLANE(SIMK_ENTRY) SIMK_BALL(SIMK_ENTRY_BALL) SIMK_SELF(SIMK_ENTRY_SELF)};
const int kNumKernelVariants = sizeof(kKernelVariants) / sizeof(kKernelVariants[0]);
const KernelVariant kTreeKernelVariants[] = {SIMK_TREE(SIMK_ENTRY_TREE)};
const int kNumTreeKernelVariants = sizeof(kTreeKernelVariants) / sizeof(kTreeKernelVariants[0]);

}  // namespace simk
