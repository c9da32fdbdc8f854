// Peak probes (include/probe.h): FP32 FMA issue, BF16 MFMA issue and a
// plain copy, each timed with HIP events around one launch; and the rollout
// kernel's sine/cosine evaluated elementwise for accuracy checks.
#include <hip/hip_runtime.h>

#include <string>

#include "../../../include/probe.h"
#include "rollout_kernel.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kThreads = 256;
constexpr int kChains = 8;

__global__ __launch_bounds__(kThreads) void fma_probe_kernel(float* sink, int iters) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  float a[kChains];
#pragma unroll
  for (int i = 0; i < kChains; ++i) a[i] = 1.0f + 1e-7f * (float)(gid + i);
  const float m = 0.9999999f, c = 1e-7f;
#pragma unroll 8
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int i = 0; i < kChains; ++i) a[i] = fmaf(a[i], m, c);
  }
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < kChains; ++i) s += a[i];
  sink[gid] = s;
}

__global__ __launch_bounds__(kThreads) void mfma_probe_kernel(float* sink, int iters) {
  const int gid = blockIdx.x * kThreads + threadIdx.x;
  bf16x8 a, b;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    a[i] = (__bf16)(1.0f + 0.001f * (float)((gid + i) & 7));
    b[i] = (__bf16)(0.5f - 0.001f * (float)((gid + 3 * i) & 7));
  }
  f32x4 acc[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
  for (int k = 0; k < iters; ++k) {
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[j], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 4; ++j) s += acc[j][0] + acc[j][1] + acc[j][2] + acc[j][3];
  sink[gid] = s;
}

__global__ __launch_bounds__(kThreads) void copy_probe_kernel(const uint4* __restrict__ src, uint4* __restrict__ dst,
                                                              size_t n) {
  const size_t stride = (size_t)gridDim.x * kThreads;
  for (size_t i = (size_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kThreads) void sincos_probe_kernel(const float* __restrict__ x, float* __restrict__ sn,
                                                                float* __restrict__ cs, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < n) {
    float a, b;
    simk::sincos_moderate(x[i], &a, &b);
    sn[i] = a;
    cs[i] = b;
  }
}

// Times one launch (the lambda) between two events on `st`; milliseconds.
template <class F>
int timed(hipStream_t st, F launch, float* ms) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return fail(PROBE_E_DEVICE, "event create failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return fail(PROBE_E_DEVICE, "event create failed");
  }
  hipError_t e = hipEventRecord(e0, st);
  if (e == hipSuccess) {
    launch();
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipEventRecord(e1, st);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return fail(PROBE_E_DEVICE, std::string("probe launch: ") + hipGetErrorString(e));
  return PROBE_OK;
}

}  // namespace

extern "C" {

int probe_fp32_fma(float* sink, int32_t blocks, int32_t iters, void* stream, double* tflops) {
  if (!sink || !tflops || blocks < 1 || iters < 1) return fail(PROBE_E_INVALID, "probe_fp32_fma: bad argument");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float ms = 0.f;
  const int rc = timed(st, [&] { fma_probe_kernel<<<blocks, kThreads, 0, st>>>(sink, iters); }, &ms);
  if (rc) return rc;
  const double flops = 2.0 * kChains * (double)iters * (double)blocks * kThreads;
  *tflops = flops / (ms * 1e-3) / 1e12;
  return PROBE_OK;
}

int probe_bf16_mfma(float* sink, int32_t blocks, int32_t iters, void* stream, double* tflops) {
  if (!sink || !tflops || blocks < 1 || iters < 1) return fail(PROBE_E_INVALID, "probe_bf16_mfma: bad argument");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  float ms = 0.f;
  const int rc = timed(st, [&] { mfma_probe_kernel<<<blocks, kThreads, 0, st>>>(sink, iters); }, &ms);
  if (rc) return rc;
  const double waves = (double)blocks * (kThreads / 64);
  const double flops = 16.0 * 16.0 * 32.0 * 2.0 * 4.0 * (double)iters * waves;
  *tflops = flops / (ms * 1e-3) / 1e12;
  return PROBE_OK;
}

int probe_copy(const void* src, void* dst, size_t bytes, void* stream, double* gbs) {
  if (!src || !dst || !gbs || bytes == 0 || bytes % 16 != 0) return fail(PROBE_E_INVALID, "probe_copy: bad argument");
  const char* s = static_cast<const char*>(src);
  const char* d = static_cast<const char*>(dst);
  if (s < d + bytes && d < s + bytes) return fail(PROBE_E_INVALID, "probe_copy: buffers overlap");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const size_t n = bytes / 16;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(PROBE_E_DEVICE, "probe_copy: device query failed");
  const size_t want = (n + kThreads - 1) / kThreads;
  const int blocks = (int)(want < (size_t)cus * 16 ? want : (size_t)cus * 16);
  float ms = 0.f;
  const int rc = timed(st, [&] {
    copy_probe_kernel<<<blocks, kThreads, 0, st>>>(static_cast<const uint4*>(src), static_cast<uint4*>(dst), n);
  }, &ms);
  if (rc) return rc;
  *gbs = 2.0 * (double)bytes / (ms * 1e-3) / 1e9;
  return PROBE_OK;
}

int probe_sincos(const float* x, float* sn, float* cs, int64_t n, void* stream) {
  if (!x || !sn || !cs || n < 1 || n > ((int64_t)1 << 31)) return fail(PROBE_E_INVALID, "probe_sincos: bad argument");
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
  sincos_probe_kernel<<<blocks, kThreads, 0, st>>>(x, sn, cs, n);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PROBE_E_DEVICE, std::string("probe_sincos launch: ") + hipGetErrorString(e));
  return PROBE_OK;
}

const char* probe_last_error(void) { return g_err.c_str(); }

}  // extern "C"
