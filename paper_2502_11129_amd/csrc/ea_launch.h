// Launchers of the evolutionary-loop kernels (host side of ea_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace eak {

struct VaryArgs {
  int mu, n_off;
  uint64_t seed;
  int generation;
  const int32_t* nh;
  const int8_t *par, *fac, *axs;
  const float* cpg;
  const float* fit;
  int32_t* nh_out;
  int8_t *par_out, *fac_out, *axs_out;
  float* cpg_out;
};

struct GatherArgs {
  int k;
  const int32_t* idx;
  int n_a, n_b;
  const int32_t *nh_a, *nh_b;
  const int8_t *par_a, *fac_a, *axs_a, *par_b, *fac_b, *axs_b;
  const float *cpg_a, *cpg_b, *fit_a, *fit_b;
  int32_t* nh_out;
  int8_t *par_out, *fac_out, *axs_out;
  float* cpg_out;
  float* fit_out;  // may be NULL: fitness not gathered
};

hipError_t launch_vary(const VaryArgs& a, hipStream_t s);
hipError_t launch_tune_perturb(int n, const int32_t* nh, const float* cpg, uint64_t seed, int generation, int round,
                               float* out, hipStream_t s);
hipError_t launch_tune_accept(int n, float* cpg_base, float* fit_base, const float* cpg_cand, const float* fit_cand,
                              hipStream_t s);
hipError_t launch_gather(const GatherArgs& a, hipStream_t s);

}  // namespace eak
