// Device-side state transfer between a bin's packed layout (q, v: 32 floats
// per packed variant; k, status, counters per packed variant) and the
// caller's variant-CSR layout in device memory (sim_get_state /
// sim_set_state / sim_counters with where = SIM_DEVICE).
//
// map[s] of packed variant s: (user index, offset of its q entries, offset of
// its v entries, nq | nv << 16), built by sim_create and uploaded by sim_bind.
// One thread per (packed variant, entry); every access is bounded by the
// variant's own nq / nv.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "launch.h"

namespace simk {

namespace {

constexpr int kEntries = 32;  // kQStride == kVStride

__global__ __launch_bounds__(256) void state_gather_kernel(int m, const int4* __restrict__ map,
                                                           const float* __restrict__ qb,
                                                           const float* __restrict__ vb,
                                                           const long long* __restrict__ kb, float* q, float* v,
                                                           int64_t* k) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = t / kEntries;
  const int j = (int)(t % kEntries);
  if (s >= m) return;
  const int4 e = map[s];
  const int nq = e.w & 0xffff, nv = e.w >> 16;
  if (q && j < nq) q[(int64_t)e.y + j] = qb[s * kEntries + j];
  if (v && j < nv) v[(int64_t)e.z + j] = vb[s * kEntries + j];
  if (k && j == 0) k[e.x] = kb[s];
}

__global__ __launch_bounds__(256) void state_scatter_kernel(int m, const int4* __restrict__ map,
                                                            const float* __restrict__ q,
                                                            const float* __restrict__ v,
                                                            const int64_t* __restrict__ k, float* qb, float* vb,
                                                            long long* kb, unsigned* status) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t s = t / kEntries;
  const int j = (int)(t % kEntries);
  if (s >= m) return;
  const int4 e = map[s];
  const int nq = e.w & 0xffff, nv = e.w >> 16;
  qb[s * kEntries + j] = j < nq ? q[(int64_t)e.y + j] : 0.f;
  vb[s * kEntries + j] = j < nv ? v[(int64_t)e.z + j] : 0.f;
  if (j == 0) {
    if (k) kb[s] = k[e.x];
    status[s] = 0u;
  }
}

__global__ __launch_bounds__(256) void counters_gather_kernel(int m, const int4* __restrict__ map,
                                                              const unsigned long long* __restrict__ cnt,
                                                              const unsigned* __restrict__ st, uint64_t* rows_contact,
                                                              uint64_t* rows_clamp, uint32_t* status) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= m) return;
  const int u = map[s].x;
  if (rows_contact) rows_contact[u] = cnt[2 * s];
  if (rows_clamp) rows_clamp[u] = cnt[2 * s + 1];
  if (status) status[u] = st[s];
}

unsigned blocks_for(int64_t threads) { return (unsigned)((threads + 255) / 256); }

}  // namespace

hipError_t launch_state_gather(int m, const int* map, const float* qb, const float* vb, const long long* kb, float* q,
                               float* v, int64_t* k, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(state_gather_kernel, dim3(blocks_for((int64_t)m * kEntries)), dim3(256), 0, st, m,
                     reinterpret_cast<const int4*>(map), qb, vb, kb, q, v, k);
  return hipGetLastError();
}

hipError_t launch_state_scatter(int m, const int* map, const float* q, const float* v, const int64_t* k, float* qb,
                                float* vb, long long* kb, unsigned* status, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(state_scatter_kernel, dim3(blocks_for((int64_t)m * kEntries)), dim3(256), 0, st, m,
                     reinterpret_cast<const int4*>(map), q, v, k, qb, vb, kb, status);
  return hipGetLastError();
}

hipError_t launch_counters_gather(int m, const int* map, const unsigned long long* cnt, const unsigned* status_b,
                                  uint64_t* rows_contact, uint64_t* rows_clamp, uint32_t* status, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(counters_gather_kernel, dim3(blocks_for(m)), dim3(256), 0, st, m,
                     reinterpret_cast<const int4*>(map), cnt, status_b, rows_contact, rows_clamp, status);
  return hipGetLastError();
}

}  // namespace simk
