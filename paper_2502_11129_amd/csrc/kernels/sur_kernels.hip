// Kernels of the learned fitness surrogate: genotype features, BF16 MFMA
// products with fused bias/GELU/GELU' epilogues, the prediction head and its
// deterministic reductions, Adam with BF16 weight copies, and top-k selection.
//
// Matrix products use v_mfma_f32_16x16x32_bf16 (gfx950): a wave multiplies a
// 16x32 BF16 tile of A by a 32x16 tile of B into a 16x16 FP32 tile.  Lane l
// supplies row (l mod 16) of A and column (l mod 16) of B, eight consecutive
// k each (k = 8 floor(l/16) ...); it receives rows 4 floor(l/16) + i,
// i = 0..3, of column (l mod 16) of the result.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "../sur_launch.h"

namespace surk {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------------------- scalar helpers
__device__ inline uint16_t f2bf(float f) {
  // round to nearest even; NaN stays NaN (quiet bit set)
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint32_t b) { return __uint_as_float((b & 0xffffu) << 16); }

__device__ inline float gelu(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_grad(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) + z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// ----------------------------------------------------------------------------- GEMM
constexpr int BM = 64, BN = 64, BK = 32;
constexpr int LS = BK + 8;  // LDS row stride in BF16 elements (80 bytes: keeps 16-byte alignment)
constexpr uint16_t kOne = 0x3F80;
constexpr uint16_t kNaN = 0x7FC0;

// Stage the logical 64 x 32 tile (rows r0.., k0..) of an operand into S[row][k].
// kRowK: element (r, k) at P[srow(r) * ld + k]; kRowM: at P[srow(k) * ld + r].
// Rows >= R and k >= K read as zero; logical row onesRow reads as one and the
// rows after it as zero (its stored width is onesRow, a multiple of 8).  A
// gathered stored row outside [0, rows) reads as NaN.
template <int L>
__device__ inline void load_tile(uint16_t* S, const uint16_t* __restrict__ P, int ld, const int32_t* __restrict__ gather,
                                 int64_t rows, int onesRow, int R, int K, int r0, int k0, int t) {
  if (L == kRowK) {
    const int r = t >> 2, c = (t & 3) * 8, gr = r0 + r, gk = k0 + c;
    uint4 v = make_uint4(0, 0, 0, 0);
    if (gr < R && gk < K) {
      if (onesRow >= 0 && gr >= onesRow) {
        if (gr == onesRow) {
          uint16_t e[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (gk + j < K) ? kOne : 0;
          v = *reinterpret_cast<uint4*>(e);
        }
      } else {
        const int64_t srow = gather ? gather[gr] : gr;
        const uint16_t* p = P + srow * ld + gk;
        if (gather && (srow < 0 || srow >= rows)) {
          uint16_t e[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (gk + j < K) ? kNaN : 0;
          v = *reinterpret_cast<uint4*>(e);
        } else if (gk + 8 <= K) {
          v = *reinterpret_cast<const uint4*>(p);
        } else {
          uint16_t e[8];
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (gk + j < K) ? p[j] : 0;
          v = *reinterpret_cast<uint4*>(e);
        }
      }
    }
    *reinterpret_cast<uint4*>(&S[r * LS + c]) = v;
  } else {
    const int kk = t >> 3, c = (t & 7) * 8, gk = k0 + kk, gr = r0 + c;
    uint16_t e[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) e[j] = 0;
    if (gk < K && gr < R) {
      if (onesRow >= 0 && gr >= onesRow) {
#pragma unroll
        for (int j = 0; j < 8; ++j) e[j] = (gr + j == onesRow) ? kOne : 0;
      } else {
        const int64_t srow = gather ? gather[gk] : gk;
        const uint16_t* p = P + srow * ld + gr;
        if (gather && (srow < 0 || srow >= rows)) {
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (gr + j < R) ? kNaN : 0;
        } else if (gr + 8 <= R) {
          *reinterpret_cast<uint4*>(e) = *reinterpret_cast<const uint4*>(p);
        } else {
#pragma unroll
          for (int j = 0; j < 8; ++j) e[j] = (gr + j < R) ? p[j] : 0;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) S[(c + j) * LS + kk] = e[j];
  }
}

template <int AL, int BL, int EPI>
__global__ __launch_bounds__(256) void gemm_kernel(GemmArgs a) {
  __shared__ __attribute__((aligned(16))) uint16_t As[BM * LS];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[BN * LS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  // K range of this layer (the whole of K unless the product is split)
  const int kchunk = a.ksplit > 1 ? ((a.K + a.ksplit - 1) / a.ksplit + BK - 1) / BK * BK : a.K;
  const int kbeg = blockIdx.z * kchunk;
  const int kend = min(a.K, kbeg + kchunk);
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    load_tile<AL>(As, a.A, a.lda, a.gatherA, a.rowsA, a.onesRow, a.M, a.K, m0, k0, t);
    load_tile<BL>(Bs, a.B, a.ldb, nullptr, 0, -1, a.N, a.K, n0, k0, t);
    __syncthreads();
    bf16x8 af[2], bfr[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const uint4 ua = *reinterpret_cast<const uint4*>(&As[(wm + i * 16 + (lane & 15)) * LS + 8 * (lane >> 4)]);
      const uint4 ub = *reinterpret_cast<const uint4*>(&Bs[(wn + i * 16 + (lane & 15)) * LS + 8 * (lane >> 4)]);
      af[i] = __builtin_bit_cast(bf16x8, ua);
      bfr[i] = __builtin_bit_cast(bf16x8, ub);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn + j * 16 + (lane & 15);
        if (m >= a.M || n >= a.N) continue;
        const float v = acc[i][j][r];
        const int64_t o = (int64_t)m * a.ldc + n;
        if (EPI == kEpiGelu) {
          const float z = v + a.bias[n];
          if (a.zout) a.zout[o] = z;
          a.hout[o] = f2bf(gelu(z));
        } else if (EPI == kEpiGeluGrad) {
          const float z = a.zin[(int64_t)m * a.ldz + n];
          a.hout[o] = f2bf(v * gelu_grad(z));
        } else if (a.ksplit > 1) {
          a.partial[(size_t)blockIdx.z * a.M * a.N + (size_t)m * a.N + n] = v;
        } else {
          a.fout[o] = v;
        }
      }
}

// Sum of the split-K layers in layer order (deterministic): out[m][n] = sum_z partial[z][m][n].
__global__ __launch_bounds__(256) void splitk_reduce_kernel(int M, int N, int layers, const float* __restrict__ partial,
                                                            float* __restrict__ out, int ldc) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)M * N) return;
  float s = 0.f;
  for (int z = 0; z < layers; ++z) s += partial[(size_t)z * M * N + i];
  const int m = (int)(i / N), n = (int)(i % N);
  out[(int64_t)m * ldc + n] = s;
}

template <int AL, int BL, int EPI>
static hipError_t launch_gemm(const GemmArgs& a, hipStream_t s) {
  const int layers = (EPI == kEpiF32 && a.ksplit > 1) ? a.ksplit : 1;
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, layers);
  hipLaunchKernelGGL((gemm_kernel<AL, BL, EPI>), grid, dim3(256), 0, s, a);
  if (layers > 1) {
    const int64_t total = (int64_t)a.M * a.N;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, a.M, a.N, layers,
                       a.partial, a.fout, a.ldc);
  }
  return hipGetLastError();
}

hipError_t gemm(int al, int bl, int epi, const GemmArgs& a, hipStream_t s) {
  if (a.M <= 0 || a.N <= 0) return hipSuccess;
  // the combinations the surrogate uses
  if (al == kRowK && bl == kRowK && epi == kEpiGelu) return launch_gemm<kRowK, kRowK, kEpiGelu>(a, s);
  if (al == kRowK && bl == kRowK && epi == kEpiGeluGrad) return launch_gemm<kRowK, kRowK, kEpiGeluGrad>(a, s);
  if (al == kRowM && bl == kRowM && epi == kEpiF32) return launch_gemm<kRowM, kRowM, kEpiF32>(a, s);
  if (al == kRowK && bl == kRowK && epi == kEpiF32) return launch_gemm<kRowK, kRowK, kEpiF32>(a, s);
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------------------------- features
// One thread per candidate.  Every value is formed in double and rounded to
// float, then to BF16 (the same two roundings for every feature).
__global__ __launch_bounds__(64) void features_kernel(int64_t n, const int32_t* __restrict__ nh,
                                                      const int8_t* __restrict__ parent,
                                                      const int8_t* __restrict__ face,
                                                      const int8_t* __restrict__ axis,
                                                      const float* __restrict__ cpg, uint16_t* __restrict__ X) {
  __shared__ uint8_t dep_s[64][24], limb_s[64][24], size_s[64][24];
  const int t = threadIdx.x;
  const int64_t i = (int64_t)blockIdx.x * 64 + t;
  if (i >= n) return;
  uint8_t* dep = dep_s[t];
  uint8_t* limb = limb_s[t];
  uint8_t* sz = size_s[t];
  const int h = nh[i];
  bool ok = h >= 1 && h <= kMaxH;
  const int8_t* P = parent + i * kMaxH;
  const int8_t* Fc = face + i * kMaxH;
  const int8_t* Ax = axis + i * kMaxH;
  const float* C = cpg + i * kMaxH * 3;

  float f[kFeat];
#pragma unroll
  for (int c = 0; c < kFeat; ++c) f[c] = 0.f;
  dep[0] = 0;
  limb[0] = 0;
#pragma unroll
  for (int b = 0; b <= kMaxH; ++b) sz[b] = 0;
  int nz = 0, maxd = 0;
  int cnt[5] = {0, 0, 0, 0, 0};
  float occ[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int j = 0; j < kMaxH; ++j) {
    if (j < h && ok) {
      const int p = P[j], fc = Fc[j], ax = Ax[j];
      if (p < 0 || p > j || fc < 0 || fc > 3 || ax < 0 || ax > 1) {
        ok = false;
      } else {
        const int d = dep[p] + 1;
        dep[j + 1] = (uint8_t)d;
        limb[j + 1] = (uint8_t)(p == 0 ? j + 1 : limb[p]);
        sz[limb[j + 1]] += 1;
        maxd = d > maxd ? d : maxd;
#pragma unroll
        for (int q = 0; q < 5; ++q) cnt[q] += (d == q + 1);
        if (p == 0) {
#pragma unroll
          for (int q = 0; q < 4; ++q)
            if (fc == q) occ[q] = 1.f;
        }
        nz += (ax == 0);
        f[j] = (float)(double)C[j * 3 + 0];
        f[20 + j] = (float)((double)C[j * 3 + 1] / 6.0);
        f[40 + j] = (float)((double)C[j * 3 + 2] / 6.283185307179586);
        f[60 + j] = ax == 0 ? 1.f : -1.f;
        f[80 + j] = (float)((double)d / 4.0);
      }
    }
  }
  if (ok) {
    f[100] = (float)((double)h / 20.0);
    f[101] = (float)((double)nz / 20.0);
    f[102] = (float)((double)(h - nz) / 20.0);
    f[103] = (float)((double)maxd / 4.0);
#pragma unroll
    for (int q = 0; q < 5; ++q) f[104 + q] = (float)((double)cnt[q] / 20.0);
    float hist[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < kMaxH; ++j) {
      if (j < h && P[j] == 0) {
        const int s = sz[j + 1];
        const int bin = s == 1 ? 0 : s == 2 ? 1 : s <= 4 ? 2 : s <= 8 ? 3 : 4;
#pragma unroll
        for (int q = 0; q < 5; ++q)
          if (bin == q) hist[q] += 0.25f;
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) f[109 + q] = hist[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) f[114 + q] = occ[q];
  } else {
#pragma unroll
    for (int c = 0; c < kFeat; ++c) f[c] = __builtin_nanf("");
  }
  uint4* out = reinterpret_cast<uint4*>(X + i * kFeat);
#pragma unroll
  for (int q = 0; q < kFeat / 8; ++q) {
    uint32_t w[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) w[e] = (uint32_t)f2bf(f[8 * q + 2 * e]) | ((uint32_t)f2bf(f[8 * q + 2 * e + 1]) << 16);
    out[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

hipError_t features(int64_t n, const int32_t* nh, const int8_t* parent, const int8_t* face, const int8_t* axis,
                    const float* cpg, uint16_t* X, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 63) / 64;
  hipLaunchKernelGGL(features_kernel, dim3((unsigned)blocks), dim3(64), 0, s, n, nh, parent, face, axis, cpg, X);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- head
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One wave per row; lane l owns hidden units 4l .. 4l+3.
__global__ __launch_bounds__(256) void head_kernel(int n, const uint16_t* __restrict__ h3, const float* __restrict__ w4,
                                                   const float* __restrict__ b4, float* __restrict__ y_out,
                                                   const float* __restrict__ target, const int32_t* __restrict__ idx,
                                                   int64_t rows, const float* __restrict__ z3, float* __restrict__ r,
                                                   float* __restrict__ dy, uint16_t* __restrict__ dz3) {
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (row >= n) return;
  const uint2 hv = *reinterpret_cast<const uint2*>(h3 + (int64_t)row * kHid + 4 * lane);
  const float4 wv = *reinterpret_cast<const float4*>(w4 + 4 * lane);
  float s = bf2f(hv.x) * wv.x + bf2f(hv.x >> 16) * wv.y + bf2f(hv.y) * wv.z + bf2f(hv.y >> 16) * wv.w;
  s = wave_sum(s);
  const float y = s + b4[0];
  if (target == nullptr) {
    if (lane == 0) y_out[row] = y;
    return;
  }
  const int64_t ti = idx ? (int64_t)idx[row] : (int64_t)row;
  const float rr = (ti >= 0 && ti < rows) ? y - target[ti] : __builtin_nanf("");
  const float d = 2.0f * rr / (float)n;
  if (lane == 0) {
    y_out[row] = y;
    r[row] = rr;
    dy[row] = d;
  }
  const float4 zv = *reinterpret_cast<const float4*>(z3 + (int64_t)row * kHid + 4 * lane);
  const uint32_t o0 = f2bf(d * wv.x * gelu_grad(zv.x)) | ((uint32_t)f2bf(d * wv.y * gelu_grad(zv.y)) << 16);
  const uint32_t o1 = f2bf(d * wv.z * gelu_grad(zv.z)) | ((uint32_t)f2bf(d * wv.w * gelu_grad(zv.w)) << 16);
  *reinterpret_cast<uint2*>(dz3 + (int64_t)row * kHid + 4 * lane) = make_uint2(o0, o1);
}

hipError_t head(int n, const uint16_t* h3, const float* w4, const float* b4, float* y_out, const float* target,
                const int32_t* idx, int64_t rows, const float* z3, float* r, float* dy, uint16_t* dz3, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(head_kernel, dim3((n + 3) / 4), dim3(256), 0, s, n, h3, w4, b4, y_out, target, idx, rows, z3, r,
                     dy, dz3);
  return hipGetLastError();
}

// Column c < 256: sum_m h3[m][c] dy[m]; c = 256: sum dy; c = 257: sum r^2.
constexpr int kHeadCols = kHid + 2;

__global__ __launch_bounds__(320) void head_partial_kernel(int n, const uint16_t* __restrict__ h3,
                                                           const float* __restrict__ dy, const float* __restrict__ r,
                                                           float* __restrict__ partial) {
  const int c = threadIdx.x;
  if (c >= kHeadCols) return;
  const int r0 = blockIdx.x * kHeadChunk;
  const int r1 = min(n, r0 + kHeadChunk);
  float s = 0.f;
  if (c < kHid) {
    for (int m = r0; m < r1; ++m) s += bf2f(h3[(int64_t)m * kHid + c]) * dy[m];
  } else if (c == kHid) {
    for (int m = r0; m < r1; ++m) s += dy[m];
  } else {
    for (int m = r0; m < r1; ++m) s += r[m] * r[m];
  }
  partial[blockIdx.x * kHeadCols + c] = s;
}

__global__ __launch_bounds__(320) void head_final_kernel(int n, int chunks, const float* __restrict__ partial,
                                                         float* __restrict__ gW4, float* __restrict__ gb4,
                                                         float* __restrict__ loss) {
  const int c = threadIdx.x;
  if (c >= kHeadCols) return;
  float s = 0.f;
  for (int q = 0; q < chunks; ++q) s += partial[q * kHeadCols + c];
  if (c < kHid) gW4[c] = s;
  else if (c == kHid) gb4[0] = s;
  else if (loss) loss[0] = s / (float)n;
}

hipError_t head_reduce(int n, const uint16_t* h3, const float* dy, const float* r, float* partial, float* gW4,
                       float* gb4, float* loss, hipStream_t s) {
  const int chunks = (n + kHeadChunk - 1) / kHeadChunk;
  hipLaunchKernelGGL(head_partial_kernel, dim3(chunks), dim3(320), 0, s, n, h3, dy, r, partial);
  hipLaunchKernelGGL(head_final_kernel, dim3(1), dim3(320), 0, s, n, chunks, partial, gW4, gb4, loss);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- Adam + BF16 copies
struct Copies {
  uint16_t *wt1, *wt2, *wt3, *wb2, *wb3;
  float* w4f;
};

// wt_l[o][i] (forward operand) and wb_l[i][o] (backward operand) hold bf16(W_l[i][o]).
__device__ inline void write_copy(int i, float val, const Copies& c) {
  const uint16_t b = f2bf(val);
  if (i < kOffB1) {
    const int in = i / kHid, o = i % kHid;
    c.wt1[o * kFeat + in] = b;
  } else if (i >= kOffW2 && i < kOffB2) {
    const int j = i - kOffW2, in = j / kHid, o = j % kHid;
    c.wt2[o * kHid + in] = b;
    c.wb2[j] = b;
  } else if (i >= kOffW3 && i < kOffB3) {
    const int j = i - kOffW3, in = j / kHid, o = j % kHid;
    c.wt3[o * kHid + in] = b;
    c.wb3[j] = b;
  } else if (i >= kOffW4 && i < kOffB4) {
    c.w4f[i - kOffW4] = bf2f(b);
  }
}

__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ g, float c1, float c2, float lr, float b1,
                                                   float omb1, float b2, float omb2, float eps, Copies cp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kNParams) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + omb1 * gi;
  const float vi = b2 * v[i] + omb2 * gi * gi;
  const float mh = mi / c1, vh = vi / c2;
  const float pi = p[i] - lr * mh / (sqrtf(vh) + eps);
  m[i] = mi;
  v[i] = vi;
  p[i] = pi;
  write_copy(i, pi, cp);
}

__global__ __launch_bounds__(256) void refresh_kernel(const float* __restrict__ p, Copies cp) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= kNParams) return;
  write_copy(i, p[i], cp);
}

hipError_t adam(float* p, float* m, float* v, const float* g, int64_t t, double lr, double b1, double b2, double eps,
                uint16_t* wt1, uint16_t* wt2, uint16_t* wt3, uint16_t* wb2, uint16_t* wb3, float* w4f,
                hipStream_t s) {
  // 1 - beta and the bias corrections 1 - beta^t are formed in double, then rounded once
  const float c1 = (float)(1.0 - pow(b1, (double)t));
  const float c2 = (float)(1.0 - pow(b2, (double)t));
  Copies cp{wt1, wt2, wt3, wb2, wb3, w4f};
  hipLaunchKernelGGL(adam_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, p, m, v, g, c1, c2, (float)lr,
                     (float)b1, (float)(1.0 - b1), (float)b2, (float)(1.0 - b2), (float)eps, cp);
  return hipGetLastError();
}

hipError_t refresh_copies(const float* p, uint16_t* wt1, uint16_t* wt2, uint16_t* wt3, uint16_t* wb2,
                          uint16_t* wb3, float* w4f, hipStream_t s) {
  Copies cp{wt1, wt2, wt3, wb2, wb3, w4f};
  hipLaunchKernelGGL(refresh_kernel, dim3((kNParams + 255) / 256), dim3(256), 0, s, p, cp);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- top-k
// Order-preserving key: larger score -> larger key; NaN -> 0 (below -inf), -0 -> +0.
__device__ inline uint32_t score_key(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0u;
  if (u == 0x80000000u) u = 0u;
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

__global__ __launch_bounds__(256) void topk_init_kernel(uint32_t* hist, uint32_t* state, uint32_t k) {
  hist[threadIdx.x] = 0;
  if (threadIdx.x < 4) state[threadIdx.x] = threadIdx.x == 2 ? k : 0u;
}

__global__ __launch_bounds__(256) void topk_hist_kernel(int64_t n, const float* __restrict__ s,
                                                        const uint32_t* __restrict__ state, uint32_t* hist,
                                                        int shift) {
  __shared__ uint32_t lh[256];
  const int t = threadIdx.x;
  lh[t] = 0;
  __syncthreads();
  const uint32_t prefix = state[0], mask = state[1];
  for (int64_t i = (int64_t)blockIdx.x * 256 + t; i < n; i += (int64_t)gridDim.x * 256) {
    const uint32_t k = score_key(s[i]);
    if ((k & mask) == prefix) atomicAdd(&lh[(k >> shift) & 255u], 1u);
  }
  __syncthreads();
  if (lh[t]) atomicAdd(&hist[t], lh[t]);
}

// Pick the digit of the k-th largest key among those matching the prefix.
__global__ __launch_bounds__(256) void topk_select_kernel(uint32_t* hist, uint32_t* state, int shift) {
  __shared__ uint32_t c[256];
  const int t = threadIdx.x;
  c[t] = hist[t];
  hist[t] = 0;
  __syncthreads();
  if (t == 0) {
    const uint32_t kleft = state[2];
    uint32_t above = 0;
    int d = 255;
    for (; d > 0; --d) {
      if (above + c[d] >= kleft) break;
      above += c[d];
    }
    state[0] = state[0] | ((uint32_t)d << shift);
    state[1] = state[1] | (255u << shift);
    state[2] = kleft - above;
  }
}

// Inclusive scan of one value per thread over a 256-thread block.
__device__ inline uint32_t block_scan(uint32_t v, uint32_t* sh) {
  const int t = threadIdx.x;
  sh[t] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const uint32_t a = t >= off ? sh[t - off] : 0u;
    __syncthreads();
    sh[t] += a;
    __syncthreads();
  }
  const uint32_t r = sh[t];
  __syncthreads();
  return r;
}

// Per block of kTopkBlock scores: (#key > T, #key == T), packed as gt << 16 | eq.
__global__ __launch_bounds__(256) void topk_count_kernel(int64_t n, const float* __restrict__ s,
                                                         const uint32_t* __restrict__ state, uint32_t* blocks) {
  __shared__ uint32_t sh[256];
  const uint32_t T = state[0];
  const int64_t base = (int64_t)blockIdx.x * kTopkBlock + 4 * threadIdx.x;
  uint32_t gt = 0, eq = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j < n) {
      const uint32_t k = score_key(s[base + j]);
      gt += k > T;
      eq += k == T;
    }
  }
  const uint32_t tot = block_scan((gt << 16) | eq, sh);
  if (threadIdx.x == 255) blocks[blockIdx.x] = tot;
}

// Exclusive prefix over blocks of the greater and equal counts (one block).
__global__ __launch_bounds__(256) void topk_scan_kernel(int64_t nb, uint32_t* blocks, uint32_t* pre) {
  __shared__ uint32_t sh[256];
  __shared__ uint32_t carry_gt, carry_eq;
  const int t = threadIdx.x;
  if (t == 0) carry_gt = carry_eq = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += 256) {
    const int64_t b = b0 + t;
    const uint32_t v = b < nb ? blocks[b] : 0u;
    const uint32_t gt_in = block_scan(v >> 16, sh);
    const uint32_t eq_in = block_scan(v & 0xffffu, sh);
    const uint32_t cg = carry_gt, ce = carry_eq;
    if (b < nb) {
      pre[2 * b] = cg + gt_in - (v >> 16);
      pre[2 * b + 1] = ce + eq_in - (v & 0xffffu);
    }
    __syncthreads();
    if (t == 255) {
      carry_gt = cg + gt_in;
      carry_eq = ce + eq_in;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void topk_write_kernel(int64_t n, const float* __restrict__ s,
                                                         const uint32_t* __restrict__ state,
                                                         const uint32_t* __restrict__ pre, int32_t* __restrict__ out) {
  __shared__ uint32_t sh[256];
  const uint32_t T = state[0], keq = state[2];
  const int64_t base = (int64_t)blockIdx.x * kTopkBlock + 4 * threadIdx.x;
  uint32_t key[4];
  uint32_t gt = 0, eq = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    key[j] = base + j < n ? score_key(s[base + j]) : 0u;
    const bool in = base + j < n;
    gt += in && key[j] > T;
    eq += in && key[j] == T;
  }
  const uint32_t inc = block_scan((gt << 16) | eq, sh);
  uint32_t rg = pre[2 * blockIdx.x] + (inc >> 16) - gt;
  uint32_t re = pre[2 * blockIdx.x + 1] + (inc & 0xffffu) - eq;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    if (base + j >= n) break;
    if (key[j] > T) {
      out[rg + (re < keq ? re : keq)] = (int32_t)(base + j);
      ++rg;
    } else if (key[j] == T) {
      if (re < keq) out[rg + re] = (int32_t)(base + j);
      ++re;
    }
  }
}

hipError_t topk(int64_t n, const float* scores, int64_t k, int32_t* out, const TopkScratch& ws, hipStream_t s) {
  if (k <= 0 || n <= 0) return hipSuccess;
  hipLaunchKernelGGL(topk_init_kernel, dim3(1), dim3(256), 0, s, ws.hist, ws.state, (uint32_t)k);
  const int64_t hb = (n + 255) / 256;
  const unsigned hist_blocks = (unsigned)(hb < 2048 ? hb : 2048);
  for (int pass = 0; pass < 4; ++pass) {
    const int shift = 24 - 8 * pass;
    hipLaunchKernelGGL(topk_hist_kernel, dim3(hist_blocks), dim3(256), 0, s, n, scores, ws.state, ws.hist, shift);
    hipLaunchKernelGGL(topk_select_kernel, dim3(1), dim3(256), 0, s, ws.hist, ws.state, shift);
  }
  const int64_t nb = (n + kTopkBlock - 1) / kTopkBlock;
  uint32_t* counts = ws.blocks;
  uint32_t* pre = ws.blocks + nb;
  hipLaunchKernelGGL(topk_count_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, scores, ws.state, counts);
  hipLaunchKernelGGL(topk_scan_kernel, dim3(1), dim3(256), 0, s, nb, counts, pre);
  hipLaunchKernelGGL(topk_write_kernel, dim3((unsigned)nb), dim3(256), 0, s, n, scores, ws.state, pre, out);
  return hipGetLastError();
}

// ----------------------------------------------------------------------------- top-k without allocation
// Scratch of topk_noalloc: the histogram (256 words), the state (4 words, padded
// to 64) and the per-block counts and prefixes (3 words per kTopkBlock scores)
// of one selection over at most kTopkStaticMax scores.  A file-scope device
// array: each GPU the library runs on holds its own copy until the process
// ends; every call on a GPU uses that GPU's copy, so calls that overlap on one
// GPU race.  topk_init_kernel clears what must start at zero.
constexpr int64_t kTopkStaticWords = 256 + 64 + 3 * (kTopkStaticMax / kTopkBlock);
static __device__ __align__(256) uint32_t scratch[kTopkStaticWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// Device address of the current GPU's scratch copy, taken once per device (the
// array's name in host code is only a stand-in for the symbol).
static hipError_t static_scratch(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<uint32_t*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t topk_noalloc(int64_t n, const float* scores, int64_t k, int32_t* out, hipStream_t s) {
  if (n > kTopkStaticMax) return hipErrorInvalidValue;
  uint32_t* base = nullptr;
  const hipError_t e = static_scratch(&base);
  if (e != hipSuccess) return e;
  const TopkScratch ws{base, base + 256, base + 256 + 64};
  return topk(n, scores, k, out, ws, s);
}

// ----------------------------------------------------------------------------- target standardisation
// One block: mean and (population) standard deviation accumulated in double
// in a fixed order, then z = (y - mean) / std.  stats = (mean, std).
__global__ __launch_bounds__(1024) void standardize_kernel(int64_t n, const float* __restrict__ y,
                                                           float* __restrict__ z, double* __restrict__ stats) {
  __shared__ double sh[1024];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int64_t i = t; i < n; i += 1024) s += (double)y[i];
  sh[t] = s;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  const double mean = sh[0] / (double)n;
  __syncthreads();
  double q = 0.0;
  for (int64_t i = t; i < n; i += 1024) {
    const double d = (double)y[i] - mean;
    q += d * d;
  }
  sh[t] = q;
  __syncthreads();
  for (int off = 512; off > 0; off >>= 1) {
    if (t < off) sh[t] += sh[t + off];
    __syncthreads();
  }
  const double sd = sqrt(sh[0] / (double)n);
  const double inv = sd > 0.0 ? 1.0 / sd : 1.0;
  for (int64_t i = t; i < n; i += 1024) z[i] = (float)(((double)y[i] - mean) * inv);
  if (t == 0) {
    stats[0] = mean;
    stats[1] = sd;
  }
}

hipError_t standardize(int64_t n, const float* y, float* z, double* stats, hipStream_t s) {
  hipLaunchKernelGGL(standardize_kernel, dim3(1), dim3(1024), 0, s, n, y, z, stats);
  return hipGetLastError();
}

}  // namespace surk
