// Registry of the compiled rollout kernel variants (host side).
#pragma once
#include <hip/hip_runtime.h>

#include "sim_layout.h"

namespace simk {

typedef hipError_t (*launch_fn)(const BinArgs&, const ModelParams&, hipStream_t);

struct KernelVariant {
  int nvc;   // DoF capacity (rows of the inverse held per variant)
  int sb;    // body slots per lane (body capacity 16 * sb)
  int ncr;   // contacts whose solver rows stay in registers
  launch_fn fn;
};

extern const KernelVariant kKernelVariants[];
extern const int kNumKernelVariants;

}  // namespace simk
