// Launchers of the surrogate kernels (defined in kernels/sur_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace surk {

constexpr int kFeat = 128;
constexpr int kHid = 256;
constexpr int kMaxH = 20;
constexpr int kNParams = 164865;
// offsets of the flat parameter vector
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kFeat * kHid;
constexpr int kOffW2 = kOffB1 + kHid;
constexpr int kOffB2 = kOffW2 + kHid * kHid;
constexpr int kOffW3 = kOffB2 + kHid;
constexpr int kOffB3 = kOffW3 + kHid * kHid;
constexpr int kOffW4 = kOffB3 + kHid;
constexpr int kOffB4 = kOffW4 + kHid;
static_assert(kOffB4 + 1 == kNParams, "parameter layout");

// Rows of the head reduction handled per block.
constexpr int kHeadChunk = 128;
// Elements per block of the top-k compaction.
constexpr int kTopkBlock = 1024;

enum ALayout { kRowK = 0, kRowM = 1 };      // stored row = m (k contiguous) | stored row = k (m contiguous)
enum Epilogue { kEpiGelu = 0, kEpiGeluGrad = 1, kEpiF32 = 2 };

// C = A B (+ epilogue) on BF16 MFMA with FP32 accumulation.
struct GemmArgs {
  int M, N, K;
  const uint16_t* A;
  int lda;
  const int32_t* gatherA;  // optional: stored row r of A is gatherA[r]
  int64_t rowsA;           // with gatherA: stored rows available; other indices read as NaN
  int onesRow;             // logical row m == onesRow of A is all ones (-1: none)
  const uint16_t* B;
  int ldb;
  // epilogues
  const float* bias;  // kEpiGelu: z = acc + bias[n]
  float* zout;        // kEpiGelu: optional z
  uint16_t* hout;     // kEpiGelu: bf16 GELU(z); kEpiGeluGrad: bf16(acc * GELU'(zin))
  const float* zin;   // kEpiGeluGrad
  int ldz;
  float* fout;        // kEpiF32
  int ldc;
  // kEpiF32 only: split the reduction dimension K over `ksplit` workgroup
  // layers; layer z writes its partial product to partial + z * M * N (row
  // stride N) and a second pass sums the layers in order into fout
  int ksplit;
  float* partial;
};

hipError_t gemm(int alayout, int blayout, int epi, const GemmArgs& a, hipStream_t s);

hipError_t features(int64_t n, const int32_t* nh, const int8_t* parent, const int8_t* face, const int8_t* axis,
                    const float* cpg, uint16_t* X, hipStream_t s);

// Prediction head y = h3 . w4 + b4.  Predict mode (target == NULL): y_out[i].
// Training mode: y, r = y - target[idx[i]] (NaN when idx[i] is outside
// [0, rows)), dy = 2 r / n, and the BF16
// gradient of the last hidden pre-activation dz3 = bf16(dy w4 GELU'(z3)).
hipError_t head(int n, const uint16_t* h3, const float* w4, const float* b4, float* y_out, const float* target,
                const int32_t* idx, int64_t rows, const float* z3, float* r, float* dy, uint16_t* dz3, hipStream_t s);
// Deterministic reductions of the head: grad W4, grad b4 and the loss.
hipError_t head_reduce(int n, const uint16_t* h3, const float* dy, const float* r, float* partial, float* gW4,
                       float* gb4, float* loss, hipStream_t s);

hipError_t adam(float* p, float* m, float* v, const float* g, int64_t t, double lr, double b1, double b2, double eps,
                uint16_t* wt1, uint16_t* wt2, uint16_t* wt3, uint16_t* wb2, uint16_t* wb3, float* w4f,
                hipStream_t s);
// Refresh the BF16 weight copies from the masters (after an upload).
hipError_t refresh_copies(const float* p, uint16_t* wt1, uint16_t* wt2, uint16_t* wt3, uint16_t* wb2,
                          uint16_t* wb3, float* w4f, hipStream_t s);

// Top-k: radix select of the threshold key, then an index-ordered compaction.
struct TopkScratch {
  uint32_t* hist;     // [256]
  uint32_t* state;    // [4]: prefix, mask, k remaining, unused
  uint32_t* blocks;   // [3 * nblocks]: per block (#greater << 16 | #equal), then exclusive prefixes (2 per block)
};
hipError_t topk(int64_t n, const float* scores, int64_t k, int32_t* out, const TopkScratch& ws, hipStream_t s);
// The same selection with its scratch in a static device array of the library
// (no allocation, no workspace argument); n <= kTopkStaticMax.
constexpr int64_t kTopkStaticMax = int64_t(1) << 24;
hipError_t topk_noalloc(int64_t n, const float* scores, int64_t k, int32_t* out, hipStream_t s);

// z = (y - mean) / std over n values (std of the population; 1 when zero); stats = (mean, std).
hipError_t standardize(int64_t n, const float* y, float* z, double* stats, hipStream_t s);

}  // namespace surk
