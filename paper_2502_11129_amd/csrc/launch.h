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
  int ball;  // 1: variants carry a ball (box-and-ball scene)
  int self;  // 1: contacts between the boxes of one robot
  launch_fn fn;
};

extern const KernelVariant kKernelVariants[];
extern const int kNumKernelVariants;

// The multi-bin kernel: its family list (nvc, sb, ncr per kind index) and launcher.
struct MultiFamily { int nvc, sb, ncr; };
extern const MultiFamily kMultiFamilies[];
extern const int kNumMultiFamilies;
hipError_t launch_rollout_multi(const MultiArgs& m, const ModelParams& p, int blocks, hipStream_t st);

}  // namespace simk
