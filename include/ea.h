/*
 * ea.h -- C ABI of the evolutionary outer loop's variation and selection
 * kernels (MI355X, gfx950).
 *
 * The paper motivates GPU simulation by evolutionary robotics: Revolve2
 * evolves robot bodies and their controllers, with Lamarckian (memetic)
 * controller learning inside each generation (Sec. 1).  It fixes no
 * operator; these are the ones of this library, on the genotype layout of
 * sur.h (hinge j joins body j+1 to parent[j] on face[j] -- 0 +x, 1 -x, 2 +y,
 * 3 -y of the parent -- with axis flag axis[j] -- 0 child z, 1 child y;
 * cpg[j] = (A, omega, phi); rows j >= nh are padding: -1 and 0):
 *
 *  - random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel
 *    Random Numbers: As Easy as 1, 2, 3", SC 2011) keyed by the 64-bit seed,
 *    counter (offspring, generation, block, row); a uniform is
 *    (x >> 8) 2^-24, an index below n is the high half of x n;
 *  - parents: two binary tournaments (higher fitness wins, NaN loses, ties
 *    to the lower index);
 *  - crossover: first parent's body; controller row j from the second
 *    parent when bit j of a random word is set and j < its hinge count;
 *  - body mutation (probability 0.3): add a leaf brick on a uniformly chosen
 *    free slot of a body of depth < 4 (core faces +-x, +-y; brick faces +x,
 *    +-y; at most 20 hinges), remove a uniformly chosen childless brick (at
 *    least 4 hinges remain; later bodies renumbered), or flip one hinge's
 *    axis;
 *  - controller mutation: each row with probability 0.2 moves (A, omega,
 *    phi) by (0.1, 0.5, 0.5) t, t uniform in [-1, 1), A clamped to [0, 1],
 *    omega to [1, 6], phi wrapped into [0, 2 pi), in float32 without fused
 *    operations (results are bit-reproducible on any IEEE host);
 *  - Lamarckian tuning: every row moves by (0.05, 0.25, 0.25) t with the
 *    same clamps; a candidate replaces the base controller when its fitness
 *    is strictly higher (or the base's is NaN and the candidate's is not).
 * Survivor selection (the mu best of parents then offspring) is sur_topk
 * over the concatenated fitness followed by ea_gather.
 *
 * Conventions: every array argument is DEVICE memory owned by the caller;
 * work is ordered on the given stream (void*, NULL = null stream); nothing
 * is allocated.  Return value: EA_OK or a negative EA_E_* code, with a
 * message from ea_last_error() (per host thread).  Input and output arrays
 * must not overlap.
 */
#ifndef EA_H_
#define EA_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EA_OK 0
#define EA_E_INVALID (-1) /* bad argument (nothing was launched) */
#define EA_E_DEVICE (-2)  /* HIP launch error                     */

/* Offspring 0..n_off-1 of generation `generation` from mu parents:
 * parents nh [mu], parent/face/axis [mu][20] int8, cpg [mu][20][3] float,
 * fitness [mu]; offspring in the same layout.  mu >= 1, n_off >= 0. */
int ea_vary(int32_t mu, const int32_t* nh, const int8_t* parent, const int8_t* face, const int8_t* axis,
            const float* cpg, const float* fitness, int32_t n_off, uint64_t seed, int32_t generation,
            int32_t* nh_out, int8_t* parent_out, int8_t* face_out, int8_t* axis_out, float* cpg_out, void* stream);

/* Lamarckian candidates: cpg_out[i] = every live row of cpg[i] moved (tuning
 * round `round` of generation `generation`); padding rows are written 0. */
int ea_tune_perturb(int32_t n, const int32_t* nh, const float* cpg, uint64_t seed, int32_t generation,
                    int32_t round, float* cpg_out, void* stream);

/* Keep improving candidates: where fit_cand[i] > fit_base[i] (or fit_base[i]
 * is NaN and fit_cand[i] is not), cpg_base[i] = cpg_cand[i] and fit_base[i] =
 * fit_cand[i] (in place). */
int ea_tune_accept(int32_t n, float* cpg_base, float* fit_base, const float* cpg_cand, const float* fit_cand,
                   void* stream);

/* out[r] = source position idx[r]: positions below n_a read genotype and
 * fitness from the a arrays, the others from the b arrays at idx - n_a.
 * Positions outside [0, n_a + n_b) are rejected by the kernel: the row is
 * written as padding with NaN fitness. */
int ea_gather(int32_t k, const int32_t* idx, int32_t n_a, const int32_t* nh_a, const int8_t* parent_a,
              const int8_t* face_a, const int8_t* axis_a, const float* cpg_a, const float* fit_a, int32_t n_b,
              const int32_t* nh_b, const int8_t* parent_b, const int8_t* face_b, const int8_t* axis_b,
              const float* cpg_b, const float* fit_b, int32_t* nh_out, int8_t* parent_out, int8_t* face_out,
              int8_t* axis_out, float* cpg_out, float* fit_out, void* stream);

const char* ea_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* EA_H_ */
