/*
 * sur.h -- C ABI of the learned fitness surrogate that pre-screens candidate
 * robots before exact simulation.
 *
 * The paper runs an evolutionary search whose cost is dominated by
 * simulation (Sec. 1 and Sec. 3: the evaluation of each candidate is a
 * simulation run).  This library adds a small multilayer perceptron that
 * predicts a candidate's fitness from a 128-value feature vector of its
 * genotype, so that only the best-ranked fraction of a large candidate pool is
 * simulated exactly; the simulator (sim.h) stays the judge of every kept
 * candidate.
 *
 * Network: 128 -> 256 -> 256 -> 256 -> 1, GELU(z) = z * Phi(z) (exact erf) on
 * the hidden layers, linear head.  Parameters are FP32 masters in one flat
 * array of SUR_N_PARAMS floats:
 *   W1 [128][256], b1 [256], W2 [256][256], b2 [256], W3 [256][256], b3 [256],
 *   W4 [256][1],   b4 [1]          (W_l[i][o]: input i -> output o, row-major)
 * Matrix products run on BF16 MFMA with FP32 accumulation.  BF16 rounding
 * (round to nearest even) happens at exactly these points: the feature
 * vector, every weight copy used by a product, every hidden activation
 * GELU(z), and every hidden-layer gradient dL/dz that feeds a product.
 * Pre-activations z, the prediction, dL/dy, gradients of parameters and the
 * optimiser state stay FP32.
 *
 * Training minimises the mean squared error over a batch with Adam (Kingma
 * and Ba 2015): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps), t counted from 1.
 *
 * Conventions (as in sim.h)
 *  - Return value SUR_OK (0) or a negative SUR_E_* code; sur_last_error()
 *    gives the message of the last failing call on a handle.
 *  - Device memory is the caller's: sur_bind attaches a workspace of at least
 *    sur_workspace_bytes(); all other device pointers (features, genotypes,
 *    scores, indices) are caller-owned device memory.
 *  - Every device call is ordered on the hipStream_t passed as void* (NULL =
 *    null stream) and returns without synchronising, except calls that
 *    read or write host memory, which synchronise that stream.
 *  - Handles are not thread-safe.
 */
#ifndef SUR_H_
#define SUR_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SUR_OK 0
#define SUR_E_INVALID (-1)
#define SUR_E_NOMEM (-2)
#define SUR_E_DEVICE (-3)
#define SUR_E_STATE (-4)

#define SUR_N_FEAT 128
#define SUR_HIDDEN 256
#define SUR_MAX_HINGES 20
#define SUR_N_PARAMS 164865

typedef struct {
  int32_t max_batch; /* largest training batch (rows), 1..65536                  */
  int32_t reserved;
  double lr;         /* Adam step size (the surrogate trains with 1e-3)            */
  double beta1;      /* 0.9                                                        */
  double beta2;      /* 0.999                                                      */
  double eps;        /* 1e-8                                                       */
} sur_config;       /* the kernels use float(x) and float(1 - beta), formed in double */

typedef struct sur_handle sur_handle;

/* Host only: validate the configuration (0 < lr, 0 <= beta < 1, eps > 0). */
int sur_create(const sur_config* cfg, sur_handle** out);

/* Device workspace: parameters, Adam moments, BF16 weight copies, gradients and
 * the activations of one training batch. */
int sur_workspace_bytes(const sur_handle* h, size_t* bytes);

/* Attach the workspace and upload the initial parameters (host float
 * [SUR_N_PARAMS], drawn by the caller), zero the Adam moments, t = 0. */
int sur_bind(sur_handle* h, void* dev_workspace, size_t bytes, const float* init_params, void* stream);

/*
 * Genotype -> features (device to device).  A genotype describes a core box
 * with nh in [1, 20] bricks: brick j+1 hangs off body parent[j] (< j+1) on
 * face face[j] (0 +x, 1 -x, 2 +y, 3 -y of the parent frame) through a hinge
 * about the brick's z (axis[j] = 0) or y (axis[j] = 1) axis, driven by
 * cpg[j] = (A, omega, phi).  Arrays (device, row per candidate, entries past
 * nh ignored): nh int32 [n]; parent, face, axis int8 [n][20]; cpg float
 * [n][20][3].  Output X: BF16 [n][128] (uint16 bit patterns):
 *   [0,20) A_j   [20,40) omega_j/6   [40,60) phi_j/(2 pi)   (zero padded)
 *   [60,80) +1 hinge about z, -1 about y, 0 padding   [80,100) depth_j/4
 *   100 nh/20, 101 (#z hinges)/20, 102 (#y hinges)/20, 103 max depth/4
 *   [104,109) number of bodies at depth 1..5, /20
 *   [109,114) histogram of limb sizes (subtrees hanging off the core) over
 *             {1, 2, 3-4, 5-8, >=9}, 0.25 per limb
 *   [114,118) core faces +x, -x, +y, -y in use (0/1)   [118,128) zero
 * An invalid genotype row (nh out of range, parent not earlier, face or axis
 * out of range) produces a row of NaN rather than an error. */
int sur_features(sur_handle* h, int64_t n, const int32_t* nh, const int8_t* parent, const int8_t* face,
                 const int8_t* axis, const float* cpg, uint16_t* X, void* stream);

/* Predictions y [n] (device float) for rows X[idx[i]] (idx device int32 [n],
 * or NULL for rows 0..n-1) with the current parameters.  X holds x_rows rows
 * (x_rows >= n when idx is NULL); an index outside [0, x_rows) gives a NaN
 * prediction.  Any n >= 0. */
int sur_predict(sur_handle* h, int64_t n, const uint16_t* X, int64_t x_rows, const int32_t* idx, float* y,
                void* stream);

/* One Adam step on the batch X[idx[i]], target[idx[i]], i < batch
 * (1 <= batch <= max_batch; idx device int32 [batch]; X and target device
 * arrays of x_rows rows).  An index outside [0, x_rows) makes the loss and the
 * gradient NaN (and so the parameters after the step).  loss: device float
 * [1] receiving the batch loss before the step, may be NULL. */
int sur_train_step(sur_handle* h, int32_t batch, const uint16_t* X, int64_t x_rows, const float* target,
                   const int32_t* idx, float* loss, void* stream);

/* One epoch: consecutive batches of `batch` rows of the permutation perm
 * (device int32 [n], drawn by the caller, entries in [0, x_rows)); the last
 * batch may be smaller.  losses: device float [ceil(n / batch)] or NULL. */
int sur_train_epoch(sur_handle* h, int64_t n, const uint16_t* X, int64_t x_rows, const float* target,
                    const int32_t* perm, int32_t batch, float* losses, void* stream);

/* Adam update with a caller-supplied gradient (device float [SUR_N_PARAMS]);
 * the step used by sur_train_step after it has computed the gradient. */
int sur_adam_step(sur_handle* h, const float* grad, void* stream);

/* Gradient of the batch loss left by the last sur_train_step (host or device
 * float [SUR_N_PARAMS], where = 0 host / 1 device). */
int sur_get_grad(const sur_handle* h, float* out, int where, void* stream);

/* Parameters, Adam moments (host float [SUR_N_PARAMS] each, any may be NULL)
 * and the step count t.  sur_set_state also refreshes the BF16 weight copies. */
int sur_get_state(const sur_handle* h, float* params, float* m, float* v, int64_t* t, void* stream);
int sur_set_state(sur_handle* h, const float* params, const float* m, const float* v, int64_t t, void* stream);

/*
 * Indices of the k largest scores (device float [n]) in ascending index
 * order, into out (device int32 [k]); 0 <= k <= n.  Ties at the threshold go
 * to the lower indices; NaN ranks below every number and -0 equals +0.
 * Needs no workspace beyond the handle's.
 */
int sur_topk(sur_handle* h, int64_t n, const float* scores, int64_t k, int32_t* out, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * selection as sur_topk, with the same result, without a handle or workspace.
 * Its scratch (histogram, selection state, per-block counts) is a static
 * device array of the library, SUR_TOPK_NOALLOC_MAX scores' worth (≈ 193 KiB),
 * one copy per GPU, held until the process ends; the call allocates nothing.
 * Every call on a GPU shares that GPU's copy: calls that overlap on one GPU
 * (concurrent streams, threads) race and must be serialised by the caller.
 * scores: device float [n]; out: device int32 [k]; stream as in sur_topk.
 * n > SUR_TOPK_NOALLOC_MAX, k outside [0, n] or NULL arrays give
 * SUR_E_INVALID without touching the device; a HIP error gives SUR_E_DEVICE.
 * err: optional host buffer of err_len bytes for the message (NULL allowed).
 */
#define SUR_TOPK_NOALLOC_MAX 16777216
int sur_topk_noalloc(int64_t n, const float* scores, int64_t k, int32_t* out, void* stream, char* err,
                     size_t err_len);

/* Training targets in standard units: z[i] = (y[i] - mean) / std over the n
 * values (device float arrays; z may alias y), std the population standard
 * deviation (taken as 1 when it is zero).  stats: host double [2] receiving
 * (mean, std), or NULL (then the call does not synchronise).  n >= 1. */
int sur_standardize(sur_handle* h, int64_t n, const float* y, float* z, double* stats, void* stream);

void sur_destroy(sur_handle* h);
const char* sur_last_error(const sur_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* SUR_H_ */
