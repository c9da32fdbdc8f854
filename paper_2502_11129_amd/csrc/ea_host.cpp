// Host side of the C ABI in include/ea.h: argument checks and launches.
#include <hip/hip_runtime.h>

#include <string>

#include "ea.h"
#include "ea_launch.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& m) {
  g_err = m;
  return code;
}

int launched(hipError_t e, const char* what) {
  if (e == hipSuccess) return EA_OK;
  return fail(EA_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace

extern "C" {

int ea_vary(int32_t mu, const int32_t* nh, const int8_t* parent, const int8_t* face, const int8_t* axis,
            const float* cpg, const float* fitness, int32_t n_off, uint64_t seed, int32_t generation,
            int32_t* nh_out, int8_t* parent_out, int8_t* face_out, int8_t* axis_out, float* cpg_out, void* stream) {
  if (mu < 1 || n_off < 0 || generation < 0) return fail(EA_E_INVALID, "need mu >= 1, n_off >= 0, generation >= 0");
  if (n_off == 0) return EA_OK;
  if (!nh || !parent || !face || !axis || !cpg || !fitness || !nh_out || !parent_out || !face_out || !axis_out ||
      !cpg_out)
    return fail(EA_E_INVALID, "a genotype or fitness array is NULL");
  eak::VaryArgs a{mu, n_off, seed, generation, nh, parent, face, axis, cpg, fitness,
                  nh_out, parent_out, face_out, axis_out, cpg_out};
  return launched(eak::launch_vary(a, (hipStream_t)stream), "ea_vary launch");
}

int ea_tune_perturb(int32_t n, const int32_t* nh, const float* cpg, uint64_t seed, int32_t generation, int32_t round,
                    float* cpg_out, void* stream) {
  if (n < 0 || generation < 0 || round < 0) return fail(EA_E_INVALID, "need n, generation, round >= 0");
  if (n == 0) return EA_OK;
  if (!nh || !cpg || !cpg_out) return fail(EA_E_INVALID, "nh, cpg or cpg_out is NULL");
  return launched(eak::launch_tune_perturb(n, nh, cpg, seed, generation, round, cpg_out, (hipStream_t)stream),
                  "ea_tune_perturb launch");
}

int ea_tune_accept(int32_t n, float* cpg_base, float* fit_base, const float* cpg_cand, const float* fit_cand,
                   void* stream) {
  if (n < 0) return fail(EA_E_INVALID, "need n >= 0");
  if (n == 0) return EA_OK;
  if (!cpg_base || !fit_base || !cpg_cand || !fit_cand) return fail(EA_E_INVALID, "an array is NULL");
  return launched(eak::launch_tune_accept(n, cpg_base, fit_base, cpg_cand, fit_cand, (hipStream_t)stream),
                  "ea_tune_accept launch");
}

int ea_gather(int32_t k, const int32_t* idx, int32_t n_a, const int32_t* nh_a, const int8_t* parent_a,
              const int8_t* face_a, const int8_t* axis_a, const float* cpg_a, const float* fit_a, int32_t n_b,
              const int32_t* nh_b, const int8_t* parent_b, const int8_t* face_b, const int8_t* axis_b,
              const float* cpg_b, const float* fit_b, int32_t* nh_out, int8_t* parent_out, int8_t* face_out,
              int8_t* axis_out, float* cpg_out, float* fit_out, void* stream) {
  if (k < 0 || n_a < 0 || n_b < 0) return fail(EA_E_INVALID, "need k, n_a, n_b >= 0");
  if (k == 0) return EA_OK;
  if (!idx || !nh_out || !parent_out || !face_out || !axis_out || !cpg_out)
    return fail(EA_E_INVALID, "idx or an output array is NULL");
  if (n_a > 0 && (!nh_a || !parent_a || !face_a || !axis_a || !cpg_a || (fit_out && !fit_a)))
    return fail(EA_E_INVALID, "an array of source a is NULL");
  if (n_b > 0 && (!nh_b || !parent_b || !face_b || !axis_b || !cpg_b || (fit_out && !fit_b)))
    return fail(EA_E_INVALID, "an array of source b is NULL");
  eak::GatherArgs a{k, idx, n_a, n_b, nh_a, nh_b, parent_a, face_a, axis_a, parent_b, face_b, axis_b,
                    cpg_a, cpg_b, fit_a, fit_b, nh_out, parent_out, face_out, axis_out, cpg_out, fit_out};
  return launched(eak::launch_gather(a, (hipStream_t)stream), "ea_gather launch");
}

const char* ea_last_error(void) { return g_err.c_str(); }

}  // extern "C"
