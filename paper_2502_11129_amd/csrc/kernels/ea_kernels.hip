// Variation and selection kernels of the evolutionary outer loop: one thread
// per offspring (a genotype is at most 20 hinges: every edit is a short
// sequential walk in registers).  Random numbers come from Philox4x32-10
// (Salmon, Moraes, Dror, Shaw, SC 2011) keyed by the seed, counter
// (offspring, generation, block, row); float arithmetic uses explicitly
// rounded operations so the results are the same on any IEEE machine.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../ea_launch.h"

namespace eak {

struct u4 { uint32_t x, y, z, w; };

__device__ __forceinline__ u4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = 0xD2511F53u * c0, hi0 = __umulhi(0xD2511F53u, c0);
    const uint32_t lo1 = 0xCD9E8D57u * c2, hi1 = __umulhi(0xCD9E8D57u, c2);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;  // the bump after the last round is unused
    k1 += 0xBB67AE85u;
  }
  return {c0, c1, c2, c3};
}

__device__ __forceinline__ float unif(uint32_t x) { return (float)(x >> 8) * 5.9604644775390625e-8f; }  // 2^-24
__device__ __forceinline__ int below(uint32_t x, int n) { return (int)(((uint64_t)x * (uint64_t)n) >> 32); }
__device__ __forceinline__ float signed_unit(uint32_t x) { return __fsub_rn(__fmul_rn(2.f, unif(x)), 1.f); }

constexpr int H = 20;
constexpr float kTwoPi = 6.28318548202514648f;  // float32(2 pi)
constexpr float kPMorph = 0.3f, kPCpg = 0.2f;

struct Geno {
  int nh;
  int par[H], fac[H], axs[H];
  float cpg[H][3];
};

__device__ __forceinline__ float move_clamped(float v, float t, float sig, float lo, float hi) {
  return fminf(hi, fmaxf(lo, __fadd_rn(v, __fmul_rn(sig, t))));
}
__device__ __forceinline__ float move_wrapped(float v, float t, float sig) {
  float p = __fadd_rn(v, __fmul_rn(sig, t));
  if (p < 0.f) p = __fadd_rn(p, kTwoPi);
  else if (p >= kTwoPi) p = __fsub_rn(p, kTwoPi);
  return p;
}
__device__ __forceinline__ void perturb(float* row, uint32_t a, uint32_t b, uint32_t c, float sa, float so, float sp) {
  row[0] = move_clamped(row[0], signed_unit(a), sa, 0.f, 1.f);
  row[1] = move_clamped(row[1], signed_unit(b), so, 1.f, 6.f);
  row[2] = move_wrapped(row[2], signed_unit(c), sp);
}

// higher fitness wins; NaN loses; ties to the lower index
__device__ __forceinline__ int better(const float* f, int a, int b) {
  const float fa = f[a], fb = f[b];
  const bool na = fa != fa, nb = fb != fb;
  if (na && nb) return a < b ? a : b;
  if (na) return b;
  if (nb) return a;
  if (fa > fb) return a;
  if (fb > fa) return b;
  return a < b ? a : b;
}

__device__ void add_leaf(Geno& g, uint32_t word, int flag, float A, float om, float ph) {
  if (g.nh >= H) return;
  int depth[H + 1];
  unsigned used[H + 1];
  depth[0] = 0;
  for (int b = 0; b <= g.nh; ++b) used[b] = 0u;
  for (int j = 0; j < g.nh; ++j) {
    depth[j + 1] = depth[g.par[j]] + 1;
    used[g.par[j]] |= 1u << g.fac[j];
  }
  // free slots in body order, faces in code order (core 0..3, bricks 0, 2, 3)
  int count = 0;
  for (int b = 0; b <= g.nh; ++b) {
    if (depth[b] >= 4) continue;
    const unsigned allowed = b == 0 ? 0xFu : 0xDu;
    count += __builtin_popcount(allowed & ~used[b]);
  }
  if (count == 0) return;
  int pick = below(word, count);
  for (int b = 0; b <= g.nh; ++b) {
    if (depth[b] >= 4) continue;
    unsigned fr = (b == 0 ? 0xFu : 0xDu) & ~used[b];
    const int c = __builtin_popcount(fr);
    if (pick < c) {
      for (; pick > 0; --pick) fr &= fr - 1;
      const int j = g.nh;
      g.par[j] = b;
      g.fac[j] = __builtin_ctz(fr);
      g.axs[j] = flag;
      g.cpg[j][0] = A; g.cpg[j][1] = om; g.cpg[j][2] = ph;
      g.nh += 1;
      return;
    }
    pick -= c;
  }
}

__device__ void remove_leaf(Geno& g, uint32_t word) {
  if (g.nh <= 4) return;
  unsigned parents = 0u;  // bodies with a child
  for (int j = 0; j < g.nh; ++j) parents |= 1u << g.par[j];
  const unsigned all = ((2u << g.nh) - 1u) & ~1u;  // bricks 1..nh
  unsigned lv = all & ~parents;
  int pick = below(word, __builtin_popcount(lv));
  for (; pick > 0; --pick) lv &= lv - 1;
  const int L = __builtin_ctz(lv);  // body L, hinge L - 1
  for (int j = L - 1; j < g.nh - 1; ++j) {
    g.par[j] = g.par[j + 1]; g.fac[j] = g.fac[j + 1]; g.axs[j] = g.axs[j + 1];
    g.cpg[j][0] = g.cpg[j + 1][0]; g.cpg[j][1] = g.cpg[j + 1][1]; g.cpg[j][2] = g.cpg[j + 1][2];
  }
  for (int j = 0; j < g.nh - 1; ++j)
    if (g.par[j] > L) g.par[j] -= 1;
  g.nh -= 1;
}

__device__ __forceinline__ void load(Geno& g, int i, const int32_t* nh, const int8_t* par, const int8_t* fac,
                                     const int8_t* axs, const float* cpg) {
  // a malformed genotype is clamped into range (never indexed out of bounds);
  // valid ones pass unchanged
  g.nh = min(max((int)nh[i], 0), H);
#pragma unroll
  for (int j = 0; j < H; ++j) {
    g.par[j] = min(max((int)par[(size_t)i * H + j], 0), j);
    g.fac[j] = min(max((int)fac[(size_t)i * H + j], 0), 3);
    g.axs[j] = min(max((int)axs[(size_t)i * H + j], 0), 1);
#pragma unroll
    for (int c = 0; c < 3; ++c) g.cpg[j][c] = cpg[((size_t)i * H + j) * 3 + c];
  }
}

__device__ __forceinline__ void store(const Geno& g, int i, int32_t* nh, int8_t* par, int8_t* fac, int8_t* axs,
                                      float* cpg) {
  nh[i] = g.nh;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const bool live = j < g.nh;
    par[(size_t)i * H + j] = (int8_t)(live ? g.par[j] : -1);
    fac[(size_t)i * H + j] = (int8_t)(live ? g.fac[j] : -1);
    axs[(size_t)i * H + j] = (int8_t)(live ? g.axs[j] : -1);
#pragma unroll
    for (int c = 0; c < 3; ++c) cpg[((size_t)i * H + j) * 3 + c] = live ? g.cpg[j][c] : 0.f;
  }
}

__global__ __launch_bounds__(64) void vary_kernel(VaryArgs a) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= a.n_off) return;
  const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32), g = (uint32_t)a.generation;
  const u4 x = philox((uint32_t)i, g, 0u, 0u, k0, k1);
  const int p1 = better(a.fit, below(x.x, a.mu), below(x.y, a.mu));
  const int p2 = better(a.fit, below(x.z, a.mu), below(x.w, a.mu));
  Geno o;
  load(o, p1, a.nh, a.par, a.fac, a.axs, a.cpg);
  // crossover of controller rows
  const u4 xc = philox((uint32_t)i, g, 1u, 0u, k0, k1);
  const int nh2 = a.nh[p2];
  for (int j = 0; j < o.nh; ++j)
    if (((xc.x >> j) & 1u) && j < nh2) {
#pragma unroll
      for (int c = 0; c < 3; ++c) o.cpg[j][c] = a.cpg[((size_t)p2 * H + j) * 3 + c];
    }
  // body mutation
  if (unif(xc.y) < kPMorph) {
    const int op = below(xc.z, 3);
    if (op == 0) {
      const u4 xn = philox((uint32_t)i, g, 2u, 0u, k0, k1);
      add_leaf(o, xc.w, (int)(xn.w & 1u), unif(xn.x), __fadd_rn(1.f, __fmul_rn(5.f, unif(xn.y))),
               __fmul_rn(kTwoPi, unif(xn.z)));
    } else if (op == 1) {
      remove_leaf(o, xc.w);
    } else {
      o.axs[below(xc.w, o.nh)] ^= 1;
    }
  }
  // controller mutation
  for (int j = 0; j < o.nh; ++j) {
    const u4 xr = philox((uint32_t)i, g, 3u, (uint32_t)j, k0, k1);
    if (unif(xr.x) < kPCpg) perturb(o.cpg[j], xr.y, xr.z, xr.w, 0.1f, 0.5f, 0.5f);
  }
  store(o, i, a.nh_out, a.par_out, a.fac_out, a.axs_out, a.cpg_out);
}

__global__ __launch_bounds__(256) void tune_perturb_kernel(int n, const int32_t* __restrict__ nh,
                                                           const float* __restrict__ cpg, uint64_t seed,
                                                           int generation, int round, float* __restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;  // one thread per (genotype, row)
  if (t >= n * H) return;
  const int i = t / H, j = t % H;
  float row[3] = {cpg[(size_t)t * 3], cpg[(size_t)t * 3 + 1], cpg[(size_t)t * 3 + 2]};
  if (j < nh[i]) {
    const u4 xr = philox((uint32_t)i, (uint32_t)generation, 64u + (uint32_t)round, (uint32_t)j, (uint32_t)seed,
                         (uint32_t)(seed >> 32));
    perturb(row, xr.x, xr.y, xr.z, 0.05f, 0.25f, 0.25f);
  } else {
    row[0] = row[1] = row[2] = 0.f;
  }
  out[(size_t)t * 3] = row[0];
  out[(size_t)t * 3 + 1] = row[1];
  out[(size_t)t * 3 + 2] = row[2];
}

__global__ __launch_bounds__(256) void tune_accept_kernel(int n, float* __restrict__ cpg_base,
                                                          float* __restrict__ fit_base,
                                                          const float* __restrict__ cpg_cand,
                                                          const float* __restrict__ fit_cand) {
  const int i = blockIdx.x * 256 + threadIdx.x;  // one thread per genotype
  if (i >= n) return;
  const float fb = fit_base[i], fc = fit_cand[i];
  if (fc > fb || (fb != fb && fc == fc)) {
    for (int e = 0; e < H * 3; ++e) cpg_base[(size_t)i * H * 3 + e] = cpg_cand[(size_t)i * H * 3 + e];
    fit_base[i] = fc;
  }
}

__global__ __launch_bounds__(64) void gather_kernel(GatherArgs a) {
  const int r = blockIdx.x * 64 + threadIdx.x;
  if (r >= a.k) return;
  const int p = a.idx[r];
  const bool from_a = p >= 0 && p < a.n_a;
  const bool from_b = p >= a.n_a && p < a.n_a + a.n_b;
  Geno g;
  float f = __int_as_float(0x7fc00000);
  if (from_a) {
    load(g, p, a.nh_a, a.par_a, a.fac_a, a.axs_a, a.cpg_a);
    if (a.fit_out) f = a.fit_a[p];
  } else if (from_b) {
    load(g, p - a.n_a, a.nh_b, a.par_b, a.fac_b, a.axs_b, a.cpg_b);
    if (a.fit_out) f = a.fit_b[p - a.n_a];
  } else {
    g.nh = 0;
  }
  store(g, r, a.nh_out, a.par_out, a.fac_out, a.axs_out, a.cpg_out);
  if (a.fit_out) a.fit_out[r] = f;
}

hipError_t launch_vary(const VaryArgs& a, hipStream_t s) {
  if (a.n_off > 0) hipLaunchKernelGGL(vary_kernel, dim3((a.n_off + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_tune_perturb(int n, const int32_t* nh, const float* cpg, uint64_t seed, int generation, int round,
                               float* out, hipStream_t s) {
  const long long t = (long long)n * H;
  if (t > 0)
    hipLaunchKernelGGL(tune_perturb_kernel, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, n, nh, cpg, seed,
                       generation, round, out);
  return hipGetLastError();
}

hipError_t launch_tune_accept(int n, float* cpg_base, float* fit_base, const float* cpg_cand, const float* fit_cand,
                              hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(tune_accept_kernel, dim3((n + 255) / 256), dim3(256), 0, s, n, cpg_base, fit_base, cpg_cand,
                       fit_cand);
  return hipGetLastError();
}

hipError_t launch_gather(const GatherArgs& a, hipStream_t s) {
  if (a.k > 0) hipLaunchKernelGGL(gather_kernel, dim3((a.k + 63) / 64), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace eak
