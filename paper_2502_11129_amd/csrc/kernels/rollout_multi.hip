// One launch for all bins of a population whose bins are all 32-body
// kernels of the default contact budgets (the autotuned packing of the
// uneven-morphology trees).  Each workgroup finds its bin from the block
// ranges and runs that family's step loop; the LDS area is the largest
// family's, shared by all.
#include "../rollout_kernel.hpp"
#include "../launch.h"

namespace simk {

#define SIMK_MULTI_FAMILIES(X) X(16, 2, 16) X(20, 2, 8) X(24, 2, 8) X(28, 2, 8)

#define SIMK_MULTI_ENTRY(NVC, SB, NCR) {NVC, SB, NCR},
const MultiFamily kMultiFamilies[] = {SIMK_MULTI_FAMILIES(SIMK_MULTI_ENTRY)};
const int kNumMultiFamilies = sizeof(kMultiFamilies) / sizeof(kMultiFamilies[0]);

#define SIMK_MULTI_SIZE(NVC, SB, NCR) sizeof(GroupLds<NVC, SB, NCR>),
constexpr size_t kMultiSizes[] = {SIMK_MULTI_FAMILIES(SIMK_MULTI_SIZE)};
constexpr size_t max_size(size_t i = 0) {
  return i + 1 == sizeof(kMultiSizes) / sizeof(kMultiSizes[0]) ? kMultiSizes[i]
         : (kMultiSizes[i] > max_size(i + 1) ? kMultiSizes[i] : max_size(i + 1));
}
constexpr size_t kMultiLdsBytes = max_size() * kVarPerWave;

__global__ __launch_bounds__(64) void rollout_multi_kernel(MultiArgs m, ModelParams P) {
  __shared__ __attribute__((aligned(16))) char smem[kMultiLdsBytes];
  const int blk = blockIdx.x;
  int bi = 0;
  while (bi + 1 < m.nbins && blk >= m.block_start[bi + 1]) ++bi;  // uniform over the workgroup
  const int local = blk - m.block_start[bi];
  int kind = 0;
#define SIMK_MULTI_CASE(NVC, SB, NCR)                                                                  \
  if (m.kind[bi] == kind)                                                                            \
    rollout_body<NVC, SB, NCR>(m.bin[bi], P, local, reinterpret_cast<GroupLds<NVC, SB, NCR>*>(smem)); \
  ++kind;
  SIMK_MULTI_FAMILIES(SIMK_MULTI_CASE)
}

hipError_t launch_rollout_multi(const MultiArgs& m, const ModelParams& p, int blocks, hipStream_t st) {
  if (blocks <= 0) return hipSuccess;
  hipLaunchKernelGGL(rollout_multi_kernel, dim3(blocks), dim3(64), 0, st, m, p);
  return hipGetLastError();
}

}  // namespace simk
