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
// Plane-only kernels with the tree-sparse factorisation of M~ (same shapes as
// entries of kKernelVariants; chosen by sim_options.gpu_factorization).
extern const KernelVariant kTreeKernelVariants[];
extern const int kNumTreeKernelVariants;

// The multi-bin kernel: its family list (nvc, sb, ncr per kind index) and launcher.
struct MultiFamily { int nvc, sb, ncr; };
extern const MultiFamily kMultiFamilies[];
extern const int kNumMultiFamilies;
hipError_t launch_rollout_multi(const MultiArgs& m, const ModelParams& p, int blocks, hipStream_t st);

// Device-side state transfer between a bin's packed layout and the caller's
// variant-CSR arrays (map: int4 per packed variant, see state_kernels.hip).
hipError_t launch_state_gather(int m, const int* map, const float* qb, const float* vb, const long long* kb, float* q,
                               float* v, int64_t* k, hipStream_t st);
hipError_t launch_state_scatter(int m, const int* map, const float* q, const float* v, const int64_t* k, float* qb,
                                float* vb, long long* kb, unsigned* status, hipStream_t st);
hipError_t launch_counters_gather(int m, const int* map, const unsigned long long* cnt, const unsigned* status_b,
                                  uint64_t* rows_contact, uint64_t* rows_clamp, uint32_t* status, hipStream_t st);

}  // namespace simk
