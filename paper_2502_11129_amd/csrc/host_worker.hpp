// Host-thread worker for the CPU/GPU split of a population (the concurrent
// CPU part of the hybrid scheme, paper Sec. 6).  Single precision, same
// equations as the GPU kernel, one variant per task.  It reads the packed
// records that sim_create prepared and owns a host copy of the state of the
// variants it runs.
#pragma once
#include <cstdint>
#include <vector>

#include "sim_layout.h"

namespace simk {

struct HostVariantView {
  const int* hdr;        // HW_WORDS
  const float* hdrf;     // HF_WORDS
  const float* body;     // nbc * BW_WORDS
  const float* q0;       // kQStride
  const float* v0;       // kVStride
  int self_collision;    // contacts between the boxes of the robot
  int tree_factor;       // factorise M~ by the tree-sparse L^T L (else dense Cholesky)
};

struct HostVariantState {
  float q[kQStride];
  float v[kVStride];
  long long k = 0;
  unsigned status = 0;
  float x0 = 0.f, y0 = 0.f;
  unsigned long long rows_contact = 0, rows_clamp = 0;
};

// Reset to (q0, v0, k = 0) and run T steps.
void host_rollout(const HostVariantView& m, const ModelParams& P, int T, HostVariantState& st);

// Fitness of a finished state.
float host_fitness(const HostVariantView& m, const HostVariantState& st);

}  // namespace simk
