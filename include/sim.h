/*
 * sim.h -- C ABI of the MI355X batched robot-variant simulator.
 *
 * Problem statement (arXiv 2502.11129, Sec. 4 "Simulation Parameters" and
 * Sec. 5): a population of N simulation "variants" is advanced for S steps;
 * Sec. 6 splits such a population between CPU and GPU.  Here a variant is an
 * articulated tree of boxes joined by hinges, driven by a sine-wave central
 * pattern generator through a PD loop, on a ground plane with friction; its
 * fitness is the horizontal displacement of its core box after the run.
 *
 * One call advances every variant of a handle on the GPU; all per-step work
 * (kinematics, composite-rigid-body mass matrix, recursive Newton-Euler bias,
 * contact detection -- box-plane, and optionally a free ball (the
 * box-and-ball scene of Sec. 5) and contacts between a robot's own boxes --,
 * inversion of the implicit-PD mass matrix, fixed-iteration projected
 * Gauss-Seidel over actuator-clamp and contact rows, semi-implicit Euler)
 * runs inside one persistent HIP kernel per DoF bin.
 *
 * Conventions shared by every entry point
 *  - Return value: SIM_OK (0) or a negative SIM_E_* code; sim_last_error()
 *    returns a message for the last failing call on that handle.
 *  - A per-variant numerical failure (non-finite state) is NOT an error: the
 *    variant is frozen, a status bit is set and its fitness reads NaN.
 *  - Ownership: sim_create deep-copies the descriptor; caller arrays may be
 *    freed afterwards.  Device memory is owned by the caller: the library
 *    uses only the workspace handed to sim_bind (query its size with
 *    sim_workspace_bytes) plus a few events and streams of its own.
 *  - Streams: every device call is ordered on the hipStream_t passed in
 *    (void*; NULL = the null stream).  where=SIM_HOST transfers synchronise
 *    that stream before returning.
 *  - Variant order in and out is always the caller's order; packing by
 *    degrees of freedom is internal.
 *  - Handles are not thread-safe: use one handle per host thread.
 */
#ifndef SIM_H_
#define SIM_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_E_INVALID (-1) /* bad argument or model (nothing was changed)        */
#define SIM_E_NOMEM (-2)   /* workspace smaller than sim_workspace_bytes()       */
#define SIM_E_DEVICE (-3)  /* HIP runtime error (sticky for the handle)          */
#define SIM_E_STATE (-4)   /* call out of order (e.g. step before sim_bind)      */
#define SIM_E_HOST (-5)    /* host workers failed on some variants (host-only runs) */

#define SIM_ROOT_FREE 0  /* 6-DoF floating core                                 */
#define SIM_ROOT_FIXED 1 /* core welded to root_pose (tests)                    */

#define SIM_HOST 0
#define SIM_DEVICE 1

/* Status bits of a variant. */
#define SIM_STATUS_NONFINITE 1u /* a non-finite value appeared; variant frozen  */
#define SIM_STATUS_CONTACTS 4u  /* more than 256 self-collision contacts; frozen */

/*
 * Model descriptor.  All arrays are host memory in variant-CSR layout:
 * body b of variant i is global body body_offset[i] + b; body 0 is the core.
 *  parent[nb]           variant-local parent index, -1 for the core, parent < child
 *  half_ext[nb*3]       box half extents (m), > 0
 *  mass[nb]             kg, > 0
 *  anchor_parent[nb*3]  hinge point in the parent frame (face centre)
 *  anchor_child[nb*3]   the same point in the child frame
 *  rest_quat[nb*4]      parent <- child rotation at theta = 0 (w,x,y,z), unit
 *  axis[nb*3]           hinge axis in the child frame, unit
 *  cpg[nb*3]            (A, omega, phi): target angle A sin(omega t + phi)
 *  mu[n]                Coulomb friction coefficient of each variant, >= 0
 *  q0, v0               initial state, CSR over variants:
 *                       FREE : q = (p0[3], Q0[4] wxyz, theta[nh]), v = (w_body[3], v_body[3], thetadot[nh])
 *                       FIXED: q = theta[nh], v = thetadot[nh]
 *  root_pose[n*7]       FIXED roots only: (p0, Q0); may be NULL for FREE
 *  ball[n*2]            optional (NULL = none): every variant carries one free
 *                       solid sphere of (radius, mass), inertia 2/5 m r^2 --
 *                       the box-and-ball scene of Sec. 5.  Its state follows
 *                       the robot's in q0/v0: q += (centre[3], Q[4] wxyz),
 *                       v += (w_world[3], v_centre_world[3]).  Contacts after
 *                       the box corners: ball-plane (the sphere's lowest
 *                       point), then ball-box for every box in body order
 *                       (closest box point; a centre inside a box leaves
 *                       through the nearest face), normal from box to ball,
 *                       Coulomb friction on the relative velocity.  The
 *                       DoF total (ball included) must stay <= 28;
 *                       single_launch does not cover ball populations.
 *  self_collision       != 0: contacts between the boxes of one robot that
 *                       are not joined by a hinge: every corner of either
 *                       box strictly inside the other (after the box-plane
 *                       corners, pairs a < b in order, corners of a then of
 *                       b).  A pair shares one normal, the separating axis
 *                       of least overlap among the two boxes' 3 + 3 face
 *                       normals and the 9 normalised cross products of
 *                       their edge directions (a cross product with squared
 *                       norm below 1e-6 is skipped; the first of equal
 *                       overlaps wins), pointing out of the penetrated box;
 *                       a corner's depth is how far it lies inside that
 *                       box's extent along the normal.  Rows act on the
 *                       relative velocity (corner's box minus penetrated
 *                       box) with the same soft normal and Coulomb disk; a
 *                       row no DoF can move (J M~^-1 J^T < 1e-9) is inert.
 *                       A pair that intersects with no corner of either
 *                       box inside the other gets, when an edge pair's
 *                       overlap beats the least face overlap by more than
 *                       1e-5 m + 5 %, one contact at the midpoint of the
 *                       two facing edges' closest points (normal that
 *                       axis, depth its overlap); otherwise the face
 *                       contacts: the incident face (the other box's face
 *                       most anti-parallel to the reference face's normal;
 *                       reference = the first face axis within 1e-5 m of
 *                       the least face overlap) clipped to the reference
 *                       face, the clipped vertices below it, depth along
 *                       the reference normal.  A variant with more than
 *                       256 such contacts in a step freezes with
 *                       SIM_STATUS_CONTACTS.  Not combined with a ball.
 * Per-model constants: PD gains kp, kd (actuator torque limit tau_max), soft
 * contact stiffness and damping in acceleration units per contact row,
 * time step dt, gravity vector, and the solver sweep count pgs_iters (part
 * of the problem definition, never tuned).
 */
typedef struct {
  int32_t n_variants;
  int32_t root_type;
  const int32_t* body_offset;
  const int32_t* parent;
  const float* half_ext;
  const float* mass;
  const float* anchor_parent;
  const float* anchor_child;
  const float* rest_quat;
  const float* axis;
  const float* cpg;
  const float* mu;
  const float* q0;
  const float* v0;
  const float* root_pose;
  float kp, kd, tau_max, k_contact, b_contact, dt;
  float gravity[3];
  int32_t pgs_iters;
  const float* ball;
  int32_t self_collision;
} sim_model_desc;

/*
 * Options (may be NULL = defaults).  None of them changes results (same
 * arithmetic in every configuration); they choose how the population is laid
 * out and launched, and are what the autotuner searches over.
 *  contacts_in_registers  contacts per variant whose solver rows stay in
 *                         registers, for every bin (0 = ncr_by_nvc, else the
 *                         first compiled kernel of the bin); contacts beyond
 *                         it spill to the workspace
 *  use_graph              != 0: sim_rollout replays a captured hipGraph
 *  steps_per_launch       simulation steps per kernel launch (0 = 1000)
 *  streams                concurrent streams the bins are spread over, by
 *                         longest-first assignment (0 = one per bin; 1 = the
 *                         caller's stream only)
 *  min_body_slots         0 or 16: smallest body capacity that holds each
 *                         variant; 32: every variant in 32-body kernels (fewer
 *                         bins)
 *  ncr_by_nvc[6]          per DoF capacity 8, 12, 16, 20, 24, 28: contacts in
 *                         registers (0 = the bin's first compiled kernel)
 *  time_launches          != 0: every bin's launches are bracketed by HIP
 *                         events on the bin's stream (sim_launch_times)
 *  single_launch          != 0: all bins in one launch per chunk of steps, the
 *                         most expensive bins' workgroups first (needs every
 *                         bin to be a 32-body kernel of the default contact
 *                         budget with nv capacity 16..28, at most 8 bins; else
 *                         sim_create fails); streams is then ignored
 *  host_factorization     factorisation of M~ in the host worker
 *                         (sim_rollout_host, the host share of
 *                         sim_rollout_split): SIM_FACTOR_DENSE (0) dense
 *                         Cholesky, SIM_FACTOR_TREE (1) the tree-sparse L^T L
 *                         factorisation over the DoF tree (Featherstone's
 *                         branch-induced sparsity: every step touches only
 *                         a DoF's ancestors); the two agree to rounding.
 *                         The GPU kernels form the dense inverse unless
 *                         gpu_factorization says otherwise.
 *  min_nv_capacity        0 or a DoF capacity (8, 12, ..., 28): variants with
 *                         fewer DoFs go to bins of this capacity (fewer bins)
 *  slots32_min_nvc        with min_body_slots = 32: only bins of this DoF
 *                         capacity and above use 32-body kernels (0 = all);
 *                         smaller capacities keep the smallest body capacity
 *                         that holds each variant
 *  gpu_factorization      SIM_FACTOR_DENSE (0): every kernel inverts M~ by a
 *                         dense symmetric Gauss-Jordan sweep in registers;
 *                         SIM_FACTOR_TREE (1): bins whose shape has a
 *                         tree-sparse kernel (plane-only, nv capacity 24, 32
 *                         bodies, 8 contacts in registers) factor M~ = L^T L
 *                         over the DoF tree in LDS and form M~^-1 by two
 *                         triangular solves per DoF; other bins, and every
 *                         bin under single_launch, keep the sweep
 *                         (sim_bin_factorization tells which).  The two agree
 *                         to rounding.
 *  host_fault_items       for failure-handling tests: the first
 *                         host_fault_items variants taken by the host workers
 *                         of a host or split rollout fail as if their worker
 *                         had raised an error (0 = none)
 */
typedef struct {
  int32_t contacts_in_registers;
  int32_t use_graph;
  int32_t steps_per_launch;
  int32_t streams;
  int32_t min_body_slots;
  int32_t ncr_by_nvc[6];
  int32_t time_launches;
  int32_t single_launch;
  int32_t host_factorization;
  int32_t min_nv_capacity;
  int32_t slots32_min_nvc;
  int32_t gpu_factorization;
  int32_t host_fault_items;
} sim_options;

#define SIM_FACTOR_DENSE 0
#define SIM_FACTOR_TREE 1

typedef struct sim_handle sim_handle;

/* Validate the descriptor and pack it by DoF bins (host only, no device work).
 * Errors: SIM_E_INVALID with a message in sim_last_error(NULL).  Limits:
 * 1..32 bodies per variant and nv <= 28 degrees of freedom (the ball's six
 * included), i.e. at most 22 hinges under a free core (16 with a ball) and
 * 28 under a fixed root; the populations of the method have at most 20
 * hinges (nv <= 26).  pgs_iters >= 1, dt > 0. */
int sim_create(const sim_model_desc* desc, const sim_options* opts, sim_handle** out);

/* Bytes of device workspace the handle needs (256-byte aligned base). */
int sim_workspace_bytes(const sim_handle* h, size_t* bytes);

/* Attach a caller-owned device workspace of at least sim_workspace_bytes()
 * and upload the packed model and the initial state on `stream`.  May be
 * called again with another workspace (the previous one is no longer used;
 * a captured rollout graph is dropped and captured again on the next graph
 * rollout); every variant restarts from its initial state. */
int sim_bind(sim_handle* h, void* dev_workspace, size_t bytes, void* stream);

/* Advance every (non-frozen) variant by n_steps >= 0 steps. */
int sim_step_batch(sim_handle* h, int32_t n_steps, void* stream);

/* Reset every variant to (q0, v0, k = 0), run T >= 0 steps and compute the
 * fitness (core xy displacement at T relative to k = 0). */
int sim_rollout(sim_handle* h, int32_t T, void* stream);

/* Fitness of every variant, user order: ||xy_core(k) - xy_core(0)||, NaN for
 * frozen variants.  out: [n_variants] floats in host (where=SIM_HOST) or
 * device (SIM_DEVICE) memory. */
int sim_fitness(const sim_handle* h, float* out, int where, void* stream);

/* Current state in the q0/v0 CSR layout and step counters [n_variants].
 * where = SIM_HOST: host arrays, the call synchronises `stream`; SIM_DEVICE:
 * device arrays, written by kernels ordered on `stream` (no sync).  Any of
 * q, v, k may be NULL. */
int sim_get_state(const sim_handle* h, float* q, float* v, int64_t* k, int where, void* stream);
/* Overwrite the state (and, if k != NULL, the step counters) from arrays in
 * the same layout, host (SIM_HOST, synchronising) or device (SIM_DEVICE,
 * stream-ordered); clears the status bits.  q and v are required. */
int sim_set_state(sim_handle* h, const float* q, const float* v, const int64_t* k, int where, void* stream);

/* Per-variant counters since the last reset: active contact rows (sum over
 * steps of the number of active contacts), actuator-clamp rows that ended a
 * step engaged, and status bits, into host (SIM_HOST, synchronising) or
 * device (SIM_DEVICE, stream-ordered) arrays; any pointer may be NULL. */
int sim_counters(const sim_handle* h, uint64_t* rows_contact, uint64_t* rows_clamp, uint32_t* status,
                 int where, void* stream);

/* Timings of a split rollout, seconds (paper Sec. 6 "Results" measures). */
typedef struct {
  double combined_s; /* wall clock of the concurrent run, including the merge of host results */
  double gpu_s;      /* GPU share: first launch to completion (HIP events)                    */
  double host_s;     /* host share: first thread start to last thread end                     */
  int32_t n_gpu, n_host, host_threads;
  int32_t n_requeued; /* host-share variants no host worker finished, re-run on the GPU */
} sim_split_times;

/* Rollout of T steps with the population split between the GPU and host
 * threads (paper Sec. 6: pilot benchmark, allocation, concurrent execution).
 * n_host variants, taken from the tail of every DoF bin in proportion to the
 * bin's size, run on host_threads CPU threads (single precision, same step)
 * while the others run on the GPU; both start together.  When the call
 * returns (it synchronises `stream`), fitness, state and counters of every
 * variant are as after sim_rollout.  0 <= n_host <= n_variants;
 * host_threads >= 1.  `times` may be NULL.  A host worker that fails (an
 * error raised while it simulates a variant, or a thread that cannot start)
 * drops out and the others carry on; whatever no host worker finished is
 * re-queued on the GPU after the GPU share (times->n_requeued), so the
 * result still covers every variant. */
int sim_rollout_split(sim_handle* h, int32_t T, int32_t n_host, int32_t host_threads, void* stream,
                      sim_split_times* times);

/* Host-only rollout of every variant on host_threads CPU threads, without any
 * device work and without touching the device state (sim_bind not needed).
 * fitness: [n_variants] host floats, user order; may be NULL.  seconds: wall
 * clock of the run; may be NULL.  If host workers fail on some variants
 * there is no other device to take them: SIM_E_HOST, with the count in
 * sim_last_error(h), and fitness is not written. */
int sim_rollout_host(sim_handle* h, int32_t T, int32_t host_threads, float* fitness, double* seconds);

/* Description of the packing: number of bins and, per bin, (nv capacity,
 * body capacity, contacts in registers, variants).  info has 4*max_bins ints. */
int sim_bins(const sim_handle* h, int32_t* n_bins, int32_t* info, int32_t max_bins);

/* Bin of every variant (user order), an index into the sim_bins order.
 * bin: [n_variants] ints.  Host only. */
int sim_variant_bins(const sim_handle* h, int32_t* bin);

/* Consecutive chunks of the population, in user order, such that a handle
 * created for each chunk alone (same options) needs at most
 * max_workspace_bytes of workspace: chunk c holds the variants
 * [c ? chunk_end[c - 1] : 0, chunk_end[c]).  For populations whose workspace
 * exceeds the device memory (the paper caps N per scene for that reason):
 * create, bind and run one handle per chunk; per-variant results do not
 * depend on the chunking.  chunk_end has max_chunks ints; *n_chunks receives
 * the count.  Errors: SIM_E_NOMEM if one variant alone exceeds the cap;
 * SIM_E_INVALID if max_chunks is too small (*n_chunks still receives the
 * count).  Host only. */
int sim_chunk_plan(const sim_handle* h, size_t max_workspace_bytes, int32_t* n_chunks, int32_t* chunk_end,
                   int32_t max_chunks);

/* Factorisation of M~ in each bin's kernel (sim_bins order):
 * SIM_FACTOR_DENSE or SIM_FACTOR_TREE (see sim_options.gpu_factorization).
 * factorization has max_bins ints; *n_bins receives the bin count.  Host
 * only. */
int sim_bin_factorization(const sim_handle* h, int32_t* n_bins, int32_t* factorization, int32_t max_bins);

/* With time_launches set: per bin (in sim_bins order), the milliseconds
 * between the start of its first and the end of its last launch in the most
 * recent sim_step_batch / sim_rollout, and the number of launches (with
 * single_launch every bin reports the shared launches).  Any output may be
 * NULL.  Synchronises on the recorded events. */
int sim_launch_times(const sim_handle* h, int32_t* n_bins, float* ms, int32_t* launches, int32_t max_bins);

/* The compiled kernel variants: per variant (nv capacity, body capacity,
 * contacts in registers, 1 if its variants carry a ball, 1 if it handles
 * self-collision).  info has 5*max_variants ints; *n receives the total
 * count.  Host only. */
int sim_kernel_variants(int32_t* n, int32_t* info, int32_t max_variants);

/*
 * Allocation of a population between the GPU and host threads (paper Sec. 6:
 * pilot benchmark, then a share for each side), host only, no device work.
 * Inputs: n variants; the measured GPU time gpu_s[k] of pilot rollouts of
 * gpu_n[k] variants (n_points >= 1 points, gpu_n ascending, > 0); the host
 * time per variant of the thread pool for the same steps (host_s_per_variant
 * > 0).  GPU time of m variants is modelled by the measured curve: flat below
 * the first point, piecewise linear between points, extended with the last
 * segment's slope; host time of h variants is h * host_s_per_variant.
 * Outputs (any may be NULL):
 *   n_host_paper     the paper's rule: each side's share is inversely
 *                    proportional to its time for the whole population,
 *                    n_host = round(n * t_gpu(n) / (t_gpu(n) + t_host(n)))
 *   n_host_makespan  the smallest h minimising max(t_gpu(n - h), t_host(h))
 *   makespan_paper_s, makespan_opt_s: modelled makespans of the two
 * For a linear GPU curve through the origin both rules give the same h.
 * Errors: SIM_E_INVALID, message in sim_last_error(NULL). */
int sim_split_allocation(int32_t n, const int32_t* gpu_n, const double* gpu_s, int32_t n_points,
                         double host_s_per_variant, int32_t* n_host_paper, int32_t* n_host_makespan,
                         double* makespan_paper_s, double* makespan_opt_s);

/* Pilot measurements and the resulting allocation (paper Sec. 6 "Initial
 * Benchmarking"): GPU rollouts of T_pilot steps for 1, 1/2, 1/4, 1/8 and
 * 1/16 of every bin (HIP events on `stream`, after one warm-up), and a host
 * rollout of host_sample variants spread over the bins on host_threads
 * threads.  Leaves every variant reset to its initial state (as after
 * sim_bind).  Synchronises `stream`.  If host workers fail on pilot
 * variants the host rate is unknown: SIM_E_HOST. */
typedef struct {
  int32_t n_host_paper, n_host_makespan;
  double makespan_paper_s, makespan_opt_s; /* modelled, for T_pilot steps                */
  double host_s_per_variant;               /* measured                                   */
  int32_t gpu_points, reserved;
  int32_t gpu_n[8];
  double gpu_s[8];                         /* measured, ascending gpu_n                   */
} sim_split_plan;
int sim_plan_split(sim_handle* h, int32_t T_pilot, int32_t host_threads, int32_t host_sample, void* stream,
                   sim_split_plan* plan);

void sim_destroy(sim_handle* h);

/* Message of the last failing call on h (or of the last failed sim_create
 * when h is NULL).  Valid until the next call on that handle. */
const char* sim_last_error(const sim_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* SIM_H_ */
