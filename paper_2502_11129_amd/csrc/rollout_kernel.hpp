// Persistent per-variant rollout kernel for gfx950 (CDNA4, wave64).
//
// Mapping: one variant per 16-lane DPP row, four variants per wave, one wave
// per workgroup.  Degree of freedom d lives in lane d % 16, slot d / 16;
// body b lives in lane b % 16, slot b / 16.  All cross-lane traffic of a
// variant stays inside its row: reductions and broadcasts use DPP
// (quad_perm, row_half_mirror, row_mirror, row_newbcast), bulk exchanges go
// through a per-variant LDS area fenced at wavefront scope (no s_barrier).
//
// One step (t_k = k dt), for every variant in parallel:
//   1. CPG targets; forward kinematics level by level down the tree, together
//      with body spatial velocities and bias accelerations (frame: world axes
//      at the current core origin);
//   2. recursive Newton-Euler bias force and composite-rigid-body inertias
//      (one backward sweep up the tree); mass matrix by CRBA; the
//      linearly-implicit PD term dt (kd + dt kp) on the hinge diagonal;
//   3. explicit inverse of that matrix by a symmetric Gauss-Jordan sweep with
//      rotating columns (rows in registers, pivot column broadcast via LDS);
//   4. free velocity v + dt Mt^-1 (a - b_a v - c);
//   5. box-plane contact detection (8 corners per box, active iff z < 0) and
//      per-contact rows J (normal z, tangents x, y), W = Mt^-1 J^T, D = J W;
//   6. K sweeps of projected Gauss-Seidel: actuator-clamp rows then contact
//      rows (soft normal in acceleration units, Coulomb disk friction);
//   7. semi-implicit Euler; non-finite check freezes the variant.
// Ball kernels (BALL = true; the box-and-ball scene of Sec. 5) add one free
// sphere per variant: its six DoFs (world angular velocity, centre velocity)
// follow the robot's, its mass-matrix block is the constant diag(I, I, I, m,
// m, m) and its bias is gravity; after the box corners come a ball-plane
// contact and ball-box contacts (closest box point, or the nearest face when
// the centre is inside a box), whose rows project the relative velocity ball
// minus box on the normal and two tangents.
// Self-collision kernels (SELF = true) add, after the corner list, every
// corner of a box strictly inside another box of the same robot not joined
// to it by a hinge (pairs in order, a bounding-sphere test first); a pair
// shares the least-overlap separating-axis normal, a corner's depth is its
// distance inside the other box's extent along it, rows act on the relative
// velocity, and a row no DoF can move is inert.  A pair with no corner inside
// that intersects across two edges gets one contact at the crossing.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim_layout.h"

namespace simk {

// ----------------------------------------------------------------------------
// Row-local (16-lane) primitives.
// ----------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// inclusive prefix sum over the 16 lanes of a row (lanes shifted in from
// outside the row contribute 0)
__device__ __forceinline__ int row_scan_incl(int x) {
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, false);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xF, 0xF, false);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xF, 0xF, false);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xF, 0xF, false);  // row_shr:8
  return x;
}
template <int L>
__device__ __forceinline__ int row_bcast_i(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x150 + L, 0xF, 0xF, false);  // row_newbcast:L
}
// Sum over the 16 lanes of a row; every lane gets the bitwise-same value.
__device__ __forceinline__ float row_sum(float x) {
  x += dpp<0xB1>(x);   // quad_perm [1,0,3,2]
  x += dpp<0x4E>(x);   // quad_perm [2,3,0,1]
  x += dpp<0x141>(x);  // row_half_mirror
  x += dpp<0x140>(x);  // row_mirror
  return x;
}

// Value of lane L of the row, broadcast to the row (row_newbcast:L).
template <int L>
__device__ __forceinline__ float row_bcast(float x) {
  return dpp<0x150 + L>(x);
}

// ----------------------------------------------------------------------------
// Small 3D helpers.
// ----------------------------------------------------------------------------
struct f3 { float x, y, z; };
__device__ __forceinline__ f3 mk(float a, float b, float c) { return {a, b, c}; }
__device__ __forceinline__ f3 operator+(f3 a, f3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ f3 operator-(f3 a, f3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ f3 operator*(f3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
__device__ __forceinline__ float dot3(f3 a, f3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ f3 cross3(f3 a, f3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
// 1/x from the hardware reciprocal (1 ulp) refined by one Newton step
__device__ __forceinline__ float recip(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(fmaf(-x, r, 1.f), r, r);
}

// sin and cos of a moderate angle (joint angles, CPG phases in [0, 2 pi)):
// Cody-Waite reduction by the nearest multiple k of pi/2 (pi/2 split into
// its float value and the remainder), then the Taylor series of sin and cos
// on |r| <= pi/4 up to r^9 and r^10, whose next terms stay below 2e-9; the
// quadrant k mod 4 swaps and signs the pair.  About half an ulp of absolute
// error, against about 1e-6 for the hardware v_sin/v_cos, whose bias
// accumulates over tens of thousands of steps.
__device__ __forceinline__ void sincos_moderate(float x, float* sn, float* cs) {
  const float k = rintf(x * 0.636619772f);
  float r = fmaf(-k, 1.57079637f, x);
  r = fmaf(-k, -4.37113883e-8f, r);
  const float r2 = r * r;
  float ps = fmaf(r2, (float)(1.0 / 362880.0), (float)(-1.0 / 5040.0));
  ps = fmaf(r2, ps, (float)(1.0 / 120.0));
  ps = fmaf(r2, ps, (float)(-1.0 / 6.0));
  const float s = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, (float)(-1.0 / 3628800.0), (float)(1.0 / 40320.0));
  pc = fmaf(r2, pc, (float)(-1.0 / 720.0));
  pc = fmaf(r2, pc, (float)(1.0 / 24.0));
  pc = fmaf(r2, pc, -0.5f);
  const float c = fmaf(r2, pc, 1.f);
  const int q = (int)k & 3;
  const float a = (q & 1) ? c : s;
  const float b = (q & 1) ? s : c;
  *sn = (q & 2) ? -a : a;
  *cs = ((q + 1) & 2) ? -b : b;
}

struct m33 { float m[9]; };
// column c (0..2, may differ across lanes) of R as a weighted sum with 0/1
// weights (entries are finite): selects between elements of one array are
// folded by the compiler into a dynamically indexed load, which would move R
// into scratch memory
__device__ __forceinline__ f3 mcol(const m33& R, int c) {
  const float w0 = c == 0 ? 1.f : 0.f, w1 = c == 1 ? 1.f : 0.f, w2 = c == 2 ? 1.f : 0.f;
  return {R.m[0] * w0 + R.m[1] * w1 + R.m[2] * w2, R.m[3] * w0 + R.m[4] * w1 + R.m[5] * w2,
          R.m[6] * w0 + R.m[7] * w1 + R.m[8] * w2};
}
__device__ __forceinline__ f3 mul(const m33& R, f3 v) {
  return {R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
          R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z};
}
__device__ __forceinline__ f3 mulT(const m33& R, f3 v) {
  return {R.m[0] * v.x + R.m[3] * v.y + R.m[6] * v.z, R.m[1] * v.x + R.m[4] * v.y + R.m[7] * v.z,
          R.m[2] * v.x + R.m[5] * v.y + R.m[8] * v.z};
}
__device__ __forceinline__ m33 matmul(const m33& A, const m33& B) {
  m33 C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}
__device__ __forceinline__ m33 quat_rot(float w, float x, float y, float z) {
  m33 R;
  R.m[0] = 1.f - 2.f * (y * y + z * z); R.m[1] = 2.f * (x * y - w * z); R.m[2] = 2.f * (x * z + w * y);
  R.m[3] = 2.f * (x * y + w * z); R.m[4] = 1.f - 2.f * (x * x + z * z); R.m[5] = 2.f * (y * z - w * x);
  R.m[6] = 2.f * (x * z - w * y); R.m[7] = 2.f * (y * z + w * x); R.m[8] = 1.f - 2.f * (x * x + y * y);
  return R;
}
// Rotation about unit axis u by the angle whose sine / cosine are s, c (Rodrigues).
__device__ __forceinline__ m33 axis_rot_acc(f3 u, float s, float c) {
  float C = 1.f - c;
  m33 R;
  R.m[0] = c + u.x * u.x * C; R.m[1] = u.x * u.y * C - u.z * s; R.m[2] = u.x * u.z * C + u.y * s;
  R.m[3] = u.y * u.x * C + u.z * s; R.m[4] = c + u.y * u.y * C; R.m[5] = u.y * u.z * C - u.x * s;
  R.m[6] = u.z * u.x * C - u.y * s; R.m[7] = u.z * u.y * C + u.x * s; R.m[8] = c + u.z * u.z * C;
  return R;
}

// One step of a unit quaternion q by the rotation vector phi:
// q <- normalize(q (x) exp(phi)) (RIGHT: phi in the body frame) or
// normalize(exp(phi) (x) q) (phi in the world frame), exp(phi) = (cos(a/2),
// sin(a/2) phi / a), a = |phi|.  Formed as q + dq with dq = (cos(a/2) - 1) q +
// q (x) (0, u) (resp. (0, u) (x) q), u = sin(a/2) phi / a and cos(a/2) - 1 =
// -2 sin^2(a/4), so each component takes one rounding, that of a small
// increment added to it; the norm is then brought back to 1 along q by
// q -= q (|q|^2 - 1) / 2 (one fused multiply-add per component).  Multiplying
// by the float value of cos(a/2) (1 - 2^-24 for the rates of these robots) and
// by a float 1 / |q| instead rounds every component in the same direction step
// after step, which turns the orientation by ~3e-8 rad per step.
template <bool RIGHT>
__device__ __forceinline__ void quat_step(float (&q)[4], f3 phi) {
  const float an = sqrtf(dot3(phi, phi));
  float cm1 = 0.f, us = 0.5f;  // cos(a/2) - 1 and sin(a/2) / a (limits at a -> 0)
  if (an >= 1e-8f) {
    float s4, c4;
    sincosf(0.25f * an, &s4, &c4);
    cm1 = -2.f * s4 * s4;
    us = 2.f * s4 * c4 / an;
  }
  const float ux = phi.x * us, uy = phi.y * us, uz = phi.z * us;
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  float d[4];
  d[0] = -(x * ux + y * uy + z * uz);
  if (RIGHT) {  // q (x) (0, u) = (-q.u, w u + q x u)
    d[1] = w * ux + (y * uz - z * uy);
    d[2] = w * uy + (z * ux - x * uz);
    d[3] = w * uz + (x * uy - y * ux);
  } else {      // (0, u) (x) q = (-u.q, w u + u x q)
    d[1] = w * ux + (uy * z - uz * y);
    d[2] = w * uy + (uz * x - ux * z);
    d[3] = w * uz + (ux * y - uy * x);
  }
  float n[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) n[i] = q[i] + fmaf(cm1, q[i], d[i]);
  const float e = fmaf(n[0], n[0], fmaf(n[1], n[1], fmaf(n[2], n[2], fmaf(n[3], n[3], -1.f))));
  const float h = -0.5f * e;
#pragma unroll
  for (int i = 0; i < 4; ++i) q[i] = fmaf(n[i], h, n[i]);
}

// Spatial vectors (angular; linear at the frame origin), world axes at p0.
struct sv { f3 a, l; };
// motion cross product  V x_m U
__device__ __forceinline__ sv crm(const sv& V, const sv& U) {
  return {cross3(V.a, U.a), cross3(V.a, U.l) + cross3(V.l, U.a)};
}
// force cross product  V x_f F
__device__ __forceinline__ sv crf(const sv& V, const sv& F) {
  return {cross3(V.a, F.a) + cross3(V.l, F.l), cross3(V.a, F.l)};
}
// Rigid-body inertia about the frame origin: mass, first moment h = m c,
// rotational inertia Io (symmetric: xx, yy, zz, xy, xz, yz).
struct sinertia { float m; f3 h; float I[6]; };
__device__ __forceinline__ f3 symmul(const float* I, f3 w) {
  return {I[0] * w.x + I[3] * w.y + I[4] * w.z, I[3] * w.x + I[1] * w.y + I[5] * w.z,
          I[4] * w.x + I[5] * w.y + I[2] * w.z};
}
__device__ __forceinline__ sv imul(const sinertia& J, const sv& V) {
  return {symmul(J.I, V.a) + cross3(J.h, V.l), V.l * J.m - cross3(J.h, V.a)};
}

// ----------------------------------------------------------------------------
// Per-variant LDS area.
// ----------------------------------------------------------------------------
template <int NVC, int SB, int NCR, bool BALL = false, bool SELF = false, bool TREE = false>
struct alignas(16) GroupLds {
  static constexpr int NBC = 16 * SB;
  static constexpr int MST = NVC + 1;                 // padded row stride of the matrices
  static constexpr int A_BODY = NBC * 24;             // forward: R9 p3 V6 A6; backward: C10 F6
  static constexpr int A_MAT = NVC * MST;             // assembled M~, later M~^-1 (rotated columns)
  static constexpr int A_WORDS = A_BODY > A_MAT ? A_BODY : A_MAT;
  static_assert(A_MAT % 4 == 0, "the matrix area is cleared with 16-byte stores");
  float A[A_WORDS];
  float WO[NBC][12];        // hinge axis w, linear part (o - p0) x w of its motion S, composite force C S
  int par[NBC];
  int ccount[NBC];          // active-corner mask per body
  float cl[NCR][(BALL || SELF) ? kListWordsBall : kListWords];  // contact list entries (ListWord)
  float cs[NCR][12];        // per-contact solver scalars
  float sth[NVC], cth[NVC], thd[NVC];  // sin theta, cos theta, thetadot by DoF
  float cvec[NVC];          // bias c by DoF
  float cb[2][2 * NVC + 16];  // doubled broadcast buffers of the pivot column (+ a sink
                              // for the lanes past the last DoF, which store unmasked)
  int lv[2 * NBC + 4];      // level lists (bodies in depth order, then level starts), staged per launch
  float brad[SELF ? NBC : 1];  // bounding-sphere radius |h| per body (self-collision), staged per launch
  // self-collision: body pairs not joined by a hinge, in order (a | b << 8),
  // built per launch; the step's bounding-sphere candidates among them
  uint16_t spair[SELF ? NBC * (NBC - 1) / 2 : 1];
  uint16_t scand[SELF ? NBC * (NBC - 1) / 2 : 1];
  // tree-sparse factorisation: the negated inverse (rows of M~^-1 in natural
  // column order), each DoF's path mask (itself and its ancestors) and the
  // reciprocal diagonal of the factor
  float X[TREE ? NVC * MST : 1];
  unsigned pm[TREE ? NVC : 1];
  float dinv[TREE ? NVC : 1];
};

// ----------------------------------------------------------------------------
// Contact rows.  The inverse is held negated in natural column order:
// Mi[s][c] = -(M~^-1)[d][c] for the lane's DoF d = lane + 16 s.  The entries of
// a vector multiplied by it are broadcast from their owner lanes (DoF c lives
// in lane c mod 16, slot c / 16) by DPP, without LDS.
// Builds J (normal z, tangents x, y) of the point x for the lane's DoF slots,
// W = M~^-1 J^T, the row denominators and cross terms, and the solver scalars.
// ----------------------------------------------------------------------------
// Column C of three mat-vecs: y_k[s] += Mi[s][C] * x_k(DoF C), with x_k(DoF C)
// read from lane C mod 16 of the row by the multiply-add itself
// (v_fmac_f32 with a row_newbcast DPP source), so the broadcast costs no
// separate move.  Same single rounding as fmaf(Mi, x, y).  The leading s_nop
// gives the two wait states a DPP source needs after a VALU write, which the
// compiler does not track across inline assembly.  Every lane of an active row
// takes part (row-uniform control flow), as DPP reads require.
template <int L>
__device__ __forceinline__ void fmac3_bcast(const float (&m)[1], float xa, float xb, float xc, float (&ya)[1],
                                            float (&yb)[1], float (&yc)[1]) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %3, %6 row_newbcast:%7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, %4, %6 row_newbcast:%7 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, %5, %6 row_newbcast:%7 row_mask:0xf bank_mask:0xf"
      : "+v"(ya[0]), "+v"(yb[0]), "+v"(yc[0])
      : "v"(xa), "v"(xb), "v"(xc), "v"(m[0]), "n"(L));
}
template <int L>
__device__ __forceinline__ void fmac3_bcast(const float (&m)[2], float xa, float xb, float xc, float (&ya)[2],
                                            float (&yb)[2], float (&yc)[2]) {
  asm("s_nop 1\n\t"
      "v_fmac_f32_dpp %0, %6, %9 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %1, %6, %10 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %2, %7, %9 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %3, %7, %10 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %4, %8, %9 row_newbcast:%11 row_mask:0xf bank_mask:0xf\n\t"
      "v_fmac_f32_dpp %5, %8, %10 row_newbcast:%11 row_mask:0xf bank_mask:0xf"
      : "+v"(ya[0]), "+v"(ya[1]), "+v"(yb[0]), "+v"(yb[1]), "+v"(yc[0]), "+v"(yc[1])
      : "v"(xa), "v"(xb), "v"(xc), "v"(m[0]), "v"(m[1]), "n"(L));
}

template <int S, int NVC, int C = 0>
__device__ __forceinline__ void matvec_bcast3(const float (&Mi)[S][NVC], const float (&a)[S], const float (&b)[S],
                                              const float (&c)[S], float (&ya)[S], float (&yb)[S], float (&yc)[S]) {
  static_assert(S == 1 || S == 2, "at most 32 DoF slots per variant");
  if constexpr (C < NVC) {
    float m[S];
#pragma unroll
    for (int s = 0; s < S; ++s) m[s] = Mi[s][C];
    fmac3_bcast<C % 16>(m, a[C / 16], b[C / 16], c[C / 16], ya, yb, yc);
    matvec_bcast3<S, NVC, C + 1>(Mi, a, b, c, ya, yb, yc);
  }
}

template <int S, int NVC, int C = 0>
__device__ __forceinline__ void matvec_bcast1(const float (&Mi)[S][NVC], const float (&a)[S], float (&ya)[S]) {
  if constexpr (C < NVC) {
    const float va = row_bcast<C % 16>(a[C / 16]);
#pragma unroll
    for (int s = 0; s < S; ++s) ya[s] = fmaf(Mi[s][C], va, ya[s]);
    matvec_bcast1<S, NVC, C + 1>(Mi, a, ya);
  }
}

// Scalars of one contact's Gauss-Seidel rows, fixed for the step (the row
// laws of contact_row rearranged so that the quantities that do not depend on
// the sweep's velocity leave its dependent chain); s1 = 1 / (D_n (1 + kb dt)),
// s5 = 1 / (dt D_x), s6 = 1 / (dt D_y):
//   [0] k d s1, [1] kb s1, [2] kb s1 dt D_n   (normal row)
//   [3] s5 dt D_xn, [4] s6 dt D_yn            (tangential change per normal change)
//   [5] s5, [6] s6
//   [7..9] lambda_n, lambda_x, lambda_y       (cold start)
// guard: a self-contact row no DoF can move (D < 1e-9) is inert, its gains 0.
__device__ __forceinline__ void solver_scalars(float kd, float Dn, float Dx, float Dy, float Dxn, float Dyn,
                                               float kb, float dt, bool guard, float (&scal)[10]) {
  float s1 = recip(Dn * (1.f + kb * dt));
  float s5 = recip(dt * Dx), s6 = recip(dt * Dy);
  if (guard) {
    if (!(Dn >= 1e-9f)) s1 = 0.f;
    if (!(Dx >= 1e-9f)) s5 = 0.f;
    if (!(Dy >= 1e-9f)) s6 = 0.f;
  }
  const float a1 = kb * s1;
  scal[0] = kd * s1;
  scal[1] = a1;
  scal[2] = a1 * (dt * Dn);
  scal[3] = s5 * (dt * Dxn);
  scal[4] = s6 * (dt * Dyn);
  scal[5] = s5;
  scal[6] = s6;
  scal[7] = 0.f;
  scal[8] = 0.f;
  scal[9] = 0.f;
}

template <int S, int NVC>
__device__ __forceinline__ void build_rows(const float (&Mi)[S][NVC], const f3 (&ang)[S], const f3 (&cst)[S],
                                           const int (&bodyOfDof)[S], int lane, f3 x, unsigned anc, float kc,
                                           float kb, float dt, float (&Jn)[S], float (&Jx)[S], float (&Jy)[S],
                                           float (&Wn)[S], float (&Wx)[S], float (&Wy)[S], float (&scal)[10]) {
  float nJn[S], nJx[S], nJy[S];  // sign of the held inverse folded in
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const bool on = (bodyOfDof[s] < 0) || ((anc >> bodyOfDof[s]) & 1u);
    const f3 J = cross3(ang[s], x) + cst[s];
    Jn[s] = on ? J.z : 0.f;
    Jx[s] = on ? J.x : 0.f;
    Jy[s] = on ? J.y : 0.f;
    nJn[s] = -Jn[s]; nJx[s] = -Jx[s]; nJy[s] = -Jy[s];
    Wn[s] = 0.f; Wx[s] = 0.f; Wy[s] = 0.f;
  }
  matvec_bcast3<S, NVC>(Mi, nJn, nJx, nJy, Wn, Wx, Wy);
  float pn = 0.f, px = 0.f, py = 0.f, pxn = 0.f, pyn = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    pn = fmaf(Jn[s], Wn[s], pn);
    px = fmaf(Jx[s], Wx[s], px);
    py = fmaf(Jy[s], Wy[s], py);
    pxn = fmaf(Jx[s], Wn[s], pxn);
    pyn = fmaf(Jy[s], Wn[s], pyn);
  }
  const float Dn = row_sum(pn), Dx = row_sum(px), Dy = row_sum(py);
  const float Dxn = row_sum(pxn), Dyn = row_sum(pyn);
  solver_scalars(kc * (-x.z), Dn, Dx, Dy, Dxn, Dyn, kb, dt, false, scal);
}

// Orthonormal tangents of a unit normal n (Duff et al., "Building an
// Orthonormal Basis, Revisited", JCGT 2017); n = +z gives +x and +y exactly.
__device__ __forceinline__ void tangents(f3 n, f3& t1, f3& t2) {
  const float sign = copysignf(1.f, n.z);
  const float a = -1.f / (sign + n.z);
  const float b = n.x * n.y * a;
  t1 = mk(1.f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  t2 = mk(b, sign + n.y * n.y * a, -n.y);
}

// Rows of one contact of a ball or self-collision kernel: the relative
// velocity (point of the bodies in `plus` minus point of the bodies in
// `minus`, plus the ball's point when `ball`) projected on the normal n and
// tangents t1, t2; depth d.  A DoF's sign is its body's bit in plus minus its
// bit in minus (root DoFs count as body 0, the core).  bodyOfDof: -1 root or
// padding DoF, -2 ball DoF, else the hinge's body.
template <int S, int NVC>
__device__ __forceinline__ void build_rows_gen(const float (&Mi)[S][NVC], const f3 (&ang)[S], const f3 (&cst)[S],
                                               const int (&bodyOfDof)[S], f3 x, f3 n, float depth, unsigned plus,
                                               unsigned minus, bool ball, bool guard, float kc, float kb, float dt,
                                               float (&Jn)[S], float (&Jx)[S], float (&Jy)[S], float (&Wn)[S],
                                               float (&Wx)[S], float (&Wy)[S], float (&scal)[10]) {
  f3 t1, t2;
  tangents(n, t1, t2);
  float nJn[S], nJx[S], nJy[S];
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int bd = bodyOfDof[s];
    float coef;
    if (bd == -2) {
      coef = ball ? 1.f : 0.f;
    } else {
      const int b = bd < 0 ? 0 : bd;
      coef = (float)((int)((plus >> b) & 1u) - (int)((minus >> b) & 1u));
    }
    const f3 J = (cross3(ang[s], x) + cst[s]) * coef;
    Jn[s] = dot3(n, J);
    Jx[s] = dot3(t1, J);
    Jy[s] = dot3(t2, J);
    nJn[s] = -Jn[s]; nJx[s] = -Jx[s]; nJy[s] = -Jy[s];
    Wn[s] = 0.f; Wx[s] = 0.f; Wy[s] = 0.f;
  }
  matvec_bcast3<S, NVC>(Mi, nJn, nJx, nJy, Wn, Wx, Wy);
  float pn = 0.f, px = 0.f, py = 0.f, pxn = 0.f, pyn = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    pn = fmaf(Jn[s], Wn[s], pn);
    px = fmaf(Jx[s], Wx[s], px);
    py = fmaf(Jy[s], Wy[s], py);
    pxn = fmaf(Jx[s], Wn[s], pxn);
    pyn = fmaf(Jy[s], Wn[s], pyn);
  }
  const float Dn = row_sum(pn), Dx = row_sum(px), Dy = row_sum(py);
  const float Dxn = row_sum(pxn), Dyn = row_sum(pyn);
  // a self-contact row no DoF can move is inert: zero gains keep its
  // multipliers at 0 (the normal's 0 also zeroes the friction limit)
  solver_scalars(kc * depth, Dn, Dx, Dy, Dxn, Dyn, kb, dt, guard, scal);
}

// One contact list entry (ListWord layout); plane-only kernels store the
// first four words.
template <bool GEN>
__device__ __forceinline__ void put_contact(float* e, f3 x, unsigned plus, unsigned minus, f3 n, float depth,
                                            int kind) {
  e[CL_X] = x.x; e[CL_X + 1] = x.y; e[CL_X + 2] = x.z;
  e[CL_ANC] = __uint_as_float(plus);
  if (GEN) {
    e[CL_N] = n.x; e[CL_N + 1] = n.y; e[CL_N + 2] = n.z;
    e[CL_DEPTH] = depth;
    e[CL_KIND] = (float)kind;
    e[CL_MINUS] = __uint_as_float(minus);
  }
}

// A point x strictly inside a box (centre p, rotation R, half extents h).
__device__ __forceinline__ bool point_in_box(f3 x, f3 p, const m33& R, f3 h) {
  const f3 l = mulT(R, x - p);
  return fabsf(l.x) < h.x && fabsf(l.y) < h.y && fabsf(l.z) < h.z;
}

// Half-width of a box (rotation R, half extents h) along a unit direction u.
__device__ __forceinline__ float box_radius(const m33& R, f3 h, f3 u) {
  return h.x * fabsf(u.x * R.m[0] + u.y * R.m[3] + u.z * R.m[6]) +
         h.y * fabsf(u.x * R.m[1] + u.y * R.m[4] + u.z * R.m[7]) +
         h.z * fabsf(u.x * R.m[2] + u.y * R.m[5] + u.z * R.m[8]);
}

// Least-overlap separating axis of boxes P and Q (P's face normals, Q's, then
// the cross products of P's column i with Q's column j, normalised, skipped
// when |cross|^2 < 1e-6; first smallest overlap wins), pointing from Q to P.
__device__ __forceinline__ f3 sat_axis(f3 pP, const m33& RP, f3 hP, f3 pQ, const m33& RQ, f3 hQ) {
  const f3 d = pP - pQ;
  f3 best = mk(0.f, 0.f, 1.f);
  float best_o = __int_as_float(0x7f800000);
  auto consider = [&](f3 u) {
    const float o = box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - fabsf(dot3(u, d));
    if (o < best_o) { best_o = o; best = u; }
  };
#pragma unroll
  for (int k = 0; k < 3; ++k) consider(mcol(RP, k));
#pragma unroll
  for (int k = 0; k < 3; ++k) consider(mcol(RQ, k));
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const f3 c = cross3(mcol(RP, i), mcol(RQ, j));
      const float n2 = dot3(c, c);
      if (n2 < 1e-6f) continue;
      consider(c * (1.f / sqrtf(n2)));
    }
  return dot3(best, d) < 0.f ? best * -1.f : best;
}

// An edge pair takes the contact from the face axes only when its overlap
// beats the least face overlap by 1e-5 m plus 5 % of it (edges in parallel
// planes give an edge-pair axis along the face normal with the same overlap).
__device__ __forceinline__ bool edge_beats_face(float edge_o, float face_o) {
  return edge_o < face_o - 1e-5f - 0.05f * face_o;
}

// Contact of two intersecting boxes P and Q with no corner of either inside
// the other (two edges crossing): when the least overlap over the 15 axes of
// sat_axis is positive and belongs to the cross product of P's edge direction
// i and Q's j, beating the least face overlap by the margin, the midpoint of
// the closest points of the two edges facing each other along it (P's on the
// side of Q, Q's on the side of P), normal from Q towards P, depth the
// overlap.  False in every other case.
__device__ __forceinline__ bool edge_contact(f3 pP, const m33& RP, f3 hP, f3 pQ, const m33& RQ, f3 hQ, f3& x, f3& n,
                                             float& depth, int& face) {
  const f3 d = pP - pQ;
  f3 best = mk(0.f, 0.f, 1.f);
  float best_o = __int_as_float(0x7f800000);
  int bi = -1, bj = -1;
  float fo[6];
  auto consider = [&](f3 u, int i, int j) {
    const float o = box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - fabsf(dot3(u, d));
    if (o < best_o) { best_o = o; best = u; bi = i; bj = j; }
    return o;
  };
#pragma unroll
  for (int k = 0; k < 3; ++k) fo[k] = consider(mcol(RP, k), -1, -1);
#pragma unroll
  for (int k = 0; k < 3; ++k) fo[3 + k] = consider(mcol(RQ, k), -1, -1);
  const float face_o = best_o;
  float edge_o = __int_as_float(0x7f800000);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const f3 c = cross3(mcol(RP, i), mcol(RQ, j));
      const float n2 = dot3(c, c);
      if (n2 < 1e-6f) continue;
      edge_o = fminf(edge_o, consider(c * (1.f / sqrtf(n2)), i, j));
    }
  // the face case: the boxes intersect and no edge pair beats the least face
  // overlap by the margin; the reference is the first face axis within 1e-5 m
  // of the least face overlap
  face = -1;
  if (face_o > 0.f && edge_o > 0.f && !edge_beats_face(edge_o, face_o)) {
#pragma unroll
    for (int f = 5; f >= 0; --f)
      if (fo[f] <= face_o + 1e-5f) face = f;
  }
  if (!(best_o > 0.f) || bi < 0 || !edge_beats_face(best_o, face_o)) return false;
  if (dot3(best, d) < 0.f) best = best * -1.f;
  const float hp[3] = {hP.x, hP.y, hP.z}, hq[3] = {hQ.x, hQ.y, hQ.z};
  f3 cP = pP, cQ = pQ;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const f3 aP = mcol(RP, k), aQ = mcol(RQ, k);
    if (k != bi) cP = cP + aP * (dot3(best, aP) > 0.f ? -hp[k] : hp[k]);
    if (k != bj) cQ = cQ + aQ * (dot3(best, aQ) < 0.f ? -hq[k] : hq[k]);
  }
  // edge half lengths by selection (no run-time indexing of the arrays)
  const float lP = bi == 0 ? hp[0] : (bi == 1 ? hp[1] : hp[2]);
  const float lQ = bj == 0 ? hq[0] : (bj == 1 ? hq[1] : hq[2]);
  const f3 eP = mcol(RP, bi), eQ = mcol(RQ, bj), r = cP - cQ;
  const float b = dot3(eP, eQ), c = dot3(eP, r), f = dot3(eQ, r);
  float t = fminf(lP, fmaxf(-lP, (b * f - c) / (1.f - b * b)));
  const float s = fminf(lQ, fmaxf(-lQ, f + b * t));
  t = fminf(lP, fmaxf(-lP, b * s - c));
  x = ((cP + eP * t) + (cQ + eQ * s)) * 0.5f;
  n = best;
  depth = best_o;
  return true;
}

// Face contacts of two intersecting boxes with no corner of either inside the
// other when no edge pair beats the least face overlap by the margin (an edge
// or a face of one box pushed through a face of the other): the reference
// face is the face of the box owning the first face axis (P's, then Q's)
// within 1e-5 m of the least face overlap, on the side of the other box (normal n out of it, centre cR, in-plane axes ar1,
// ar2 with half extents e1, e2); the incident face is the other box's face
// most anti-parallel to n (centre cI, axes ai1, ai2, half extents f1, f2);
// the face index (0..2: P's axes, 3..5: Q's) comes from edge_contact.
struct FaceClip {
  f3 n, cR, ar1, ar2, cI, ai1, ai2;
  float e1, e2, f1, f2;
  bool on_q;  // the points belong to Q (else to P)
};
__device__ __forceinline__ void face_setup(f3 pP, const m33& RP, f3 hP, f3 pQ, const m33& RQ, f3 hQ,
                                                    int face, FaceClip& F) {
  const f3 d = pP - pQ;
  f3 best = face == 0 ? mcol(RP, 0) : face == 1 ? mcol(RP, 1) : face == 2 ? mcol(RP, 2)
          : face == 3 ? mcol(RQ, 0) : face == 4 ? mcol(RQ, 1) : mcol(RQ, 2);
  if (dot3(best, d) < 0.f) best = best * -1.f;
  const bool refP = face < 3;
  const int k = refP ? face : face - 3;
  const m33& RR = refP ? RP : RQ;
  const m33& RI = refP ? RQ : RP;
  const f3 hR = refP ? hP : hQ, hI = refP ? hQ : hP;
  const f3 pR = refP ? pP : pQ, pI = refP ? pQ : pP;
  F.n = refP ? best * -1.f : best;
  F.on_q = refP;
  const float hRk = k == 0 ? hR.x : (k == 1 ? hR.y : hR.z);
  F.cR = pR + F.n * hRk;
  F.ar1 = mcol(RR, k == 0 ? 1 : 0);
  F.ar2 = mcol(RR, k == 2 ? 1 : 2);
  F.e1 = k == 0 ? hR.y : hR.x;
  F.e2 = k == 2 ? hR.y : hR.z;
  int js = 0;
  float bc = -1.f;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const float c = fabsf(dot3(mcol(RI, j), F.n));
    if (c > bc) { bc = c; js = j; }
  }
  const f3 aj = js == 0 ? mcol(RI, 0) : (js == 1 ? mcol(RI, 1) : mcol(RI, 2));
  const float hIj = js == 0 ? hI.x : (js == 1 ? hI.y : hI.z);
  const float sg = dot3(aj, F.n) > 0.f ? -1.f : 1.f;
  F.cI = pI + aj * (sg * hIj);
  F.ai1 = js == 0 ? mcol(RI, 1) : mcol(RI, 0);
  F.ai2 = js == 2 ? mcol(RI, 1) : mcol(RI, 2);
  F.f1 = js == 0 ? hI.y : hI.x;
  F.f2 = js == 2 ? hI.y : hI.z;
}
// Candidate c (0..23) of the clipped incident face, in the fixed order:
// incident corners inside the reference rectangle (0..3), rectangle corners
// inside the incident face carried onto it (4..7), crossings of incident edge
// e = (c - 8) / 4 with rectangle edge line (c - 8) % 4 (8..23); true when the
// candidate exists and lies below the reference face, with its point and
// depth n . (cR - x).
__device__ __forceinline__ bool face_candidate(const FaceClip& F, int c, f3& x, float& depth) {
  auto corner = [&](int q) { return F.cI + (F.ai1 * ((q & 1) ? F.f1 : -F.f1) + F.ai2 * ((q & 2) ? F.f2 : -F.f2)); };
  bool ok = false;
  if (c < 4) {
    x = corner(c);
    const f3 r = x - F.cR;
    ok = fabsf(dot3(r, F.ar1)) < F.e1 && fabsf(dot3(r, F.ar2)) < F.e2;
  } else if (c < 8) {
    const int q = c - 4;
    const float m11 = dot3(F.ai1, F.ar1), m12 = dot3(F.ai2, F.ar1), m21 = dot3(F.ai1, F.ar2),
                m22 = dot3(F.ai2, F.ar2);
    const float det = m11 * m22 - m12 * m21;
    const f3 r0 = F.cI - F.cR;
    const float bs = ((q & 1) ? F.e1 : -F.e1) - dot3(r0, F.ar1), bt = ((q & 2) ? F.e2 : -F.e2) - dot3(r0, F.ar2);
    const float uu = (bs * m22 - m12 * bt) / det, ww = (m11 * bt - m21 * bs) / det;
    x = F.cI + (F.ai1 * uu + F.ai2 * ww);
    ok = fabsf(uu) < F.f1 && fabsf(ww) < F.f2;
  } else {
    const int e = (c - 8) >> 2, l = (c - 8) & 3;
    const int ia = e == 0 ? 0 : (e == 1 ? 1 : (e == 2 ? 3 : 2)), ib = e == 0 ? 1 : (e == 1 ? 3 : (e == 2 ? 2 : 0));
    const f3 A = corner(ia), B = corner(ib);
    const f3 rA = A - F.cR, rB = B - F.cR;
    const float sA = dot3(rA, F.ar1), tA = dot3(rA, F.ar2), sB = dot3(rB, F.ar1), tB = dot3(rB, F.ar2);
    const bool sline = l < 2;
    const float cval = l == 0 ? -F.e1 : (l == 1 ? F.e1 : (l == 2 ? -F.e2 : F.e2));
    const float a0 = sline ? sA : tA, a1 = sline ? sB : tB;
    if (a1 != a0) {
      const float lam = (cval - a0) / (a1 - a0);
      const float other = sline ? tA + lam * (tB - tA) : sA + lam * (sB - sA);
      x = A + (B - A) * lam;
      ok = lam > 0.f && lam < 1.f && fabsf(other) < (sline ? F.e2 : F.e1);
    }
  }
  depth = dot3(F.n, F.cR - x);
  return ok && depth > 0.f;
}

// Corner c (bits x, y, z = signs) of a box with pose (R, p) and half extents h.
__device__ __forceinline__ f3 box_corner(const m33& R, f3 p, f3 h, int c) {
  const f3 s = mk((c & 1) ? h.x : -h.x, (c & 2) ? h.y : -h.y, (c & 4) ? h.z : -h.z);
  return mk(p.x + R.m[0] * s.x + R.m[1] * s.y + R.m[2] * s.z, p.y + R.m[3] * s.x + R.m[4] * s.y + R.m[5] * s.z,
            p.z + R.m[6] * s.x + R.m[7] * s.y + R.m[8] * s.z);
}

// Sphere (centre c, radius r) against a box (centre p, rotation R, half
// extents h): with l = R^T (c - p), outside the box the closest box point q,
// contact iff |c - q| < r, normal (c - q) / |c - q|, depth r - |c - q|; a
// centre inside or on the box leaves through the nearest face (first of
// equals in x, y, z order), depth r + its distance.  Point: c - r n.
__device__ __forceinline__ bool sphere_box(f3 c, float r, f3 p, const m33& R, f3 h, f3& x, f3& n, float& depth) {
  const f3 l = mulT(R, c - p);
  const bool inside = fabsf(l.x) <= h.x && fabsf(l.y) <= h.y && fabsf(l.z) <= h.z;
  if (!inside) {
    const f3 q = mk(fmaxf(-h.x, fminf(h.x, l.x)), fmaxf(-h.y, fminf(h.y, l.y)), fmaxf(-h.z, fminf(h.z, l.z)));
    const f3 d = c - (p + mul(R, q));
    const float dist = sqrtf(dot3(d, d));
    if (!(dist < r)) return false;
    n = d * (1.f / dist);
    depth = r - dist;
  } else {
    const float gx = h.x - fabsf(l.x), gy = h.y - fabsf(l.y), gz = h.z - fabsf(l.z);
    int kb = 0;
    float gap = gx;
    if (gy < gap) { gap = gy; kb = 1; }
    if (gz < gap) { gap = gz; kb = 2; }
    const float sgn = (kb == 0 ? l.x : kb == 1 ? l.y : l.z) >= 0.f ? 1.f : -1.f;
    const f3 nl = mk(kb == 0 ? sgn : 0.f, kb == 1 ? sgn : 0.f, kb == 2 ? sgn : 0.f);
    const f3 nw = mul(R, nl);
    n = nw * (1.f / sqrtf(dot3(nw, nw)));
    depth = r + gap;
  }
  x = c - n * r;
  return true;
}

// One contact of one Gauss-Seidel sweep: soft normal row, then the two
// friction rows together (Jacobi within the pair), projected on the disk
// |lambda_t| <= mu lambda_n.  lam[0..2] are read and updated.  With the
// scalars of solver_scalars the laws read
//   lambda_n' = max(0, [0] - [1] u_n + [2] lambda_n),
//   g_x = lambda_x - [5] u_x - [3] (lambda_n' - lambda_n)   (same for y),
//   lambda_t' = g min(1, mu lambda_n' / |g|),
// the oracle's laws with the products regrouped; the terms that do not
// depend on u are formed beside the dependent chain, and the projection is
// branch-free.
template <int S>
__device__ __forceinline__ void contact_row(float (&vp)[S], const float (&Jn)[S], const float (&Jx)[S],
                                            const float (&Jy)[S], const float (&Wn)[S], const float (&Wx)[S],
                                            const float (&Wy)[S], const float (&sc)[10], float (&lam)[3],
                                            float mu, float dt) {
  float pn = 0.f, px = 0.f, py = 0.f;
#pragma unroll
  for (int s = 0; s < S; ++s) {
    pn = fmaf(Jn[s], vp[s], pn);
    px = fmaf(Jx[s], vp[s], px);
    py = fmaf(Jy[s], vp[s], py);
  }
  const float ln0 = lam[0], lx0 = lam[1], ly0 = lam[2];
  const float c0 = fmaf(sc[2], ln0, sc[0]);
  const float un = row_sum(pn), ux = row_sum(px), uy = row_sum(py);
  const float gxp = fmaf(-sc[5], ux, lx0), gyp = fmaf(-sc[6], uy, ly0);
  const float ln = fmaxf(0.f, fmaf(-sc[1], un, c0));
  const float dn = ln - ln0;
  const float gx = fmaf(-sc[3], dn, gxp), gy = fmaf(-sc[4], dn, gyp);
  const float edn = fmaf(dt, ln, -dt * ln0);
#pragma unroll
  for (int s = 0; s < S; ++s) vp[s] = fmaf(Wn[s], edn, vp[s]);
  const float gn2 = fmaf(gx, gx, gy * gy);
  const float scale = fminf(1.f, (mu * ln) * __builtin_amdgcn_rsqf(gn2));
  const float nx = gx * scale, ny = gy * scale;
  const float edx = fmaf(dt, nx, -dt * lx0), edy = fmaf(dt, ny, -dt * ly0);
  lam[0] = ln; lam[1] = nx; lam[2] = ny;
#pragma unroll
  for (int s = 0; s < S; ++s) vp[s] = fmaf(Wx[s], edx, fmaf(Wy[s], edy, vp[s]));
}

// Smallest value over the 16 lanes of a row (every lane gets it); integer,
// so each step is one DPP move and one min with no float canonicalisation.
__device__ __forceinline__ int row_min_i(int x) {
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false));   // quad_perm [1,0,3,2]
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false));   // quad_perm [2,3,0,1]
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false));  // row_half_mirror
  x = min(x, __builtin_amdgcn_update_dpp(0, x, 0x140, 0xF, 0xF, false));  // row_mirror
  return x;
}

// ----------------------------------------------------------------------------
// The kernel.
// ----------------------------------------------------------------------------
// A budget of 256 registers (two waves per SIMD) for the families that fit it
// without spills: one DoF slot per lane with at most 2 contacts in registers,
// and the 16-DoF families with 8; and for the 20-DoF, 16-body families with 2
// or 4 contacts in registers, which spill 24 and 48 registers per lane at
// 256 but run faster at two waves per SIMD: with 2, the whole rollout of the
// 8192 random trees is 5 % faster than with the single-wave 32-body kernel,
// with 4 another 3 % (more contacts stay out of the workspace; 5 is no
// faster, 6 slower).  The 24- and 28-DoF families spill 196 and 272 bytes
// there and run slower.  Their LDS areas then admit two waves per SIMD with
// 16 body slots and 1.5 with 32.  The others may use the whole register file
// and run one wave per SIMD.
template <int NVC, int SB, int NCR>
struct WavesPerSimd {
  static constexpr int value =
      ((SB == 1 && NCR <= 2 && NVC <= 20) || (SB == 1 && NCR == 4 && NVC == 20) || (NCR == 8 && NVC == 16)) ? 2
                                                                                                             : 1;
};

// One workgroup (one wave, four variants) of a bin: `block` is the
// workgroup's index within the bin, lds_all the four variants' LDS areas.
template <int NVC, int SB, int NCR, bool BALL = false, bool SELF = false, bool TREE = false>
__device__ __forceinline__ void rollout_body(const BinArgs& a, const ModelParams& P, int block,
                                             GroupLds<NVC, SB, NCR, BALL, SELF, TREE>* lds_all) {
  constexpr int S = (NVC + 15) / 16;
  constexpr int NBC = 16 * SB;
  constexpr int MAXC = max_contacts(NBC, BALL, SELF);
  constexpr bool GEN = BALL || SELF;  // general contact entries and rows
  constexpr int CLW = GEN ? kListWordsBall : kListWords;
  using L = GroupLds<NVC, SB, NCR, BALL, SELF, TREE>;
  static_assert(!TREE || (NVC >= 8 && NVC <= 32), "path masks are 32-bit; the first six DoFs are held apart");
  constexpr int MST = L::MST;

  const int lane = threadIdx.x & 15;
  const int grp = threadIdx.x >> 4;
  const int vid = block * kVarPerWave + grp;
  if (vid >= a.n) return;  // whole rows leave together
  L& sh = lds_all[grp];

  // ---- per-variant header (uniform within the row) ----
  const int* hdr = a.hdr + (size_t)vid * HW_WORDS;
  const int nb = hdr[HW_NB], nv = hdr[HW_NV], r0 = hdr[HW_R0], maxdepth = hdr[HW_MAXDEPTH];
  const int nvr = BALL ? hdr[HW_NVR] : nv;  // robot DoFs (the ball's follow)
  const float* hf = a.hdrf + (size_t)vid * HF_WORDS;
  const float mu = hf[HF_MU];
  const float rball = BALL ? hf[HF_BALLR] : 0.f, mball = BALL ? hf[HF_BALLM] : 0.f;
  const float iball = 0.4f * mball * rball * rball;  // solid sphere
  const float* bodyv = a.body + (size_t)vid * NBC * BW_WORDS;
  const int* lvl = a.lvl + (size_t)vid * a.lvl_stride;  // bodies in level order, then level offsets
  float* ovf = a.ovf + (size_t)vid * a.ovf_stride;
  float* ovf_list = ovf;
  float* ovf_scal = ovf + MAXC * CLW;
  float* ovf_rows = ovf_scal + MAXC * kOvfScal;

  const float dt = P.dt, kp = P.kp, kd = P.kd, tmax = P.tau_max, kc = P.k_contact, bc = P.b_contact;
  const float ba = kd + dt * kp;
  const float kb = bc + kc * dt;
  const double dtd = (double)dt;

  // ---- state ----
  float vS[S], thS[S];
  float p0[3], Q0[4];
  float pb[3] = {0.f, 0.f, 0.f}, Qb[4] = {1.f, 0.f, 0.f, 0.f};  // ball centre and orientation
  long long kstep;
  unsigned status;
  unsigned long long cnt_contact, cnt_clamp;
  {
    const float* qsrc = (a.reset ? a.q0 : a.q) + (size_t)vid * kQStride;
    const float* vsrc = (a.reset ? a.v0 : a.v) + (size_t)vid * kVStride;
    const int qh = (r0 == 6) ? 7 : 0;  // offset of theta in q
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      vS[s] = (d < nv) ? vsrc[d] : 0.f;
      thS[s] = (d >= r0 && d < nvr) ? qsrc[qh + d - r0] : 0.f;
    }
    if (BALL) {
      const int qb = hdr[HW_NQR];
      pb[0] = qsrc[qb]; pb[1] = qsrc[qb + 1]; pb[2] = qsrc[qb + 2];
      Qb[0] = qsrc[qb + 3]; Qb[1] = qsrc[qb + 4]; Qb[2] = qsrc[qb + 5]; Qb[3] = qsrc[qb + 6];
    }
    if (r0 == 6) {
      p0[0] = qsrc[0]; p0[1] = qsrc[1]; p0[2] = qsrc[2];
      Q0[0] = qsrc[3]; Q0[1] = qsrc[4]; Q0[2] = qsrc[5]; Q0[3] = qsrc[6];
    } else {
      p0[0] = hf[HF_ROOTP]; p0[1] = hf[HF_ROOTP + 1]; p0[2] = hf[HF_ROOTP + 2];
      Q0[0] = hf[HF_ROOTQ]; Q0[1] = hf[HF_ROOTQ + 1]; Q0[2] = hf[HF_ROOTQ + 2]; Q0[3] = hf[HF_ROOTQ + 3];
    }
    if (a.reset) {
      kstep = 0; status = 0; cnt_contact = 0; cnt_clamp = 0;
    } else {
      kstep = a.k[vid]; status = a.status[vid];
      cnt_contact = a.cnt[2 * vid]; cnt_clamp = a.cnt[2 * vid + 1];
    }
  }
  if (a.reset && lane == 0) {
    a.xy0[2 * vid] = (r0 == 6) ? p0[0] : 0.f;
    a.xy0[2 * vid + 1] = (r0 == 6) ? p0[1] : 0.f;
  }
  unsigned ancS[SB];  // ancestors-or-self mask of the lane's body slots (CRBA)
#pragma unroll
  for (int t = 0; t < SB; ++t) {
    const int b = lane + 16 * t;
    ancS[t] = 0u;
    if (b < nb) {
      sh.par[b] = __float_as_int(bodyv[b * BW_WORDS + BW_PARENT]);
      ancS[t] = __float_as_uint(bodyv[b * BW_WORDS + BW_ANCESTORS]);
    }
  }
  for (int j = lane; j < 2 * NBC + 4; j += 16) sh.lv[j] = lvl[j];
  if constexpr (TREE) {
    // path mask of every DoF (the DoF and its ancestors in the DoF tree): the
    // free root's six DoFs form a chain, a hinge sits under its parent body's
    // hinge and under the whole root, the ball's DoFs and the padding stand
    // alone.  Ancestors carry lower indices (parents precede children).
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      const int b = lane + 16 * t;
      if (b >= 1 && b < nb && r0 + b - 1 < NVC)
        sh.pm[r0 + b - 1] = (r0 == 6 ? 0x3Fu : 0u) | (((ancS[t] & ~1u) >> 1) << r0);
    }
    for (int d = lane; d < NVC; d += 16) {
      if (r0 == 6 && d < 6) sh.pm[d] = (2u << d) - 1u;
      else if (d >= nvr) sh.pm[d] = 1u << d;
    }
  }
  int npairs = 0;  // row-uniform
  if (SELF) {
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      const int b = lane + 16 * t;
      if (b < nb) {
        const float* rec = bodyv + (size_t)b * BW_WORDS;
        const f3 h = mk(rec[BW_HALF], rec[BW_HALF + 1], rec[BW_HALF + 2]);
        sh.brad[b] = sqrtf(dot3(h, h));
      }
    }
    wave_sync();  // parents staged above
    // the pair table: for each a the lanes take b = a + 1 + lane (+16), a DPP
    // scan places the pairs not joined by a hinge in order
    for (int ia = 0; ia < nb - 1; ++ia) {
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int ib = ia + 1 + lane + 16 * t;
        const int ok = (ib < nb && sh.par[ib] != ia) ? 1 : 0;
        const int incl = row_scan_incl(ok);
        if (ok) sh.spair[npairs + incl - 1] = (uint16_t)(ia | (ib << 8));
        npairs += row_bcast_i<15>(incl);
      }
    }
  }
  wave_sync();

  for (int it = 0; it < a.n_steps; ++it) {
    if (status) break;  // frozen variants stop (row-uniform)

    // =====================================================================
    // 1. forward kinematics, spatial velocities and bias accelerations, body
    //    by body down the tree; the lanes of a row take the bodies of one
    //    depth level at a time.  Corner tests of each body.
    // =====================================================================
#pragma unroll
    for (int s = 0; s < S; ++s) {  // every joint's sine and cosine at once, off the level chain
      const int d = lane + 16 * s;
      float sn, cn;
      sincos_moderate(thS[s], &sn, &cn);
      if (d < NVC) { sh.sth[d] = sn; sh.cth[d] = cn; sh.thd[d] = vS[s]; }
    }
    f3 wb = mk(row_bcast<0>(vS[0]), row_bcast<1>(vS[0]), row_bcast<2>(vS[0]));
    f3 vb = mk(row_bcast<3>(vS[0]), row_bcast<4>(vS[0]), row_bcast<5>(vS[0]));
    if (r0 != 6) { wb = mk(0.f, 0.f, 0.f); vb = wb; }
    const m33 R0 = quat_rot(Q0[0], Q0[1], Q0[2], Q0[3]);
    const f3 P0 = mk(p0[0], p0[1], p0[2]);
#pragma unroll
    for (int t = 0; t < SB; ++t) sh.ccount[lane + 16 * t] = 0;
    wave_sync();

    for (int lev = 0; lev <= maxdepth; ++lev) {
      const int i1 = sh.lv[NBC + lev + 1];
      for (int i = sh.lv[NBC + lev] + lane; i < i1; i += 16) {
        const int b = sh.lv[i];
        const float* rec = bodyv + (size_t)b * BW_WORDS;
        m33 R;
        f3 p, w, o, sl = mk(0.f, 0.f, 0.f);
        sv V, A;
        if (b == 0) {
          R = R0;
          p = P0;
          w = mk(0.f, 0.f, 0.f);
          o = P0;
          V.a = mul(R0, wb);
          V.l = mul(R0, vb);
          A.a = mk(0.f, 0.f, 0.f);
          A.l = mk(-P.g[0], -P.g[1], -P.g[2]);  // gravity as a base acceleration
        } else {
          const int lam = sh.par[b];
          const float* pr = &sh.A[lam * 24];
          m33 Rl;
#pragma unroll
          for (int k2 = 0; k2 < 9; ++k2) Rl.m[k2] = pr[k2];
          const f3 pl = mk(pr[9], pr[10], pr[11]);
          const sv Vl = {mk(pr[12], pr[13], pr[14]), mk(pr[15], pr[16], pr[17])};
          const sv Al = {mk(pr[18], pr[19], pr[20]), mk(pr[21], pr[22], pr[23])};
          const int dof = r0 + b - 1;
          const float sn = sh.sth[dof], cs = sh.cth[dof], thd = sh.thd[dof];
          const f3 u = mk(rec[BW_AXIS], rec[BW_AXIS + 1], rec[BW_AXIS + 2]);
          const m33 E = matmul(quat_rot(rec[BW_RQ], rec[BW_RQ + 1], rec[BW_RQ + 2], rec[BW_RQ + 3]),
                               axis_rot_acc(u, sn, cs));
          R = matmul(Rl, E);
          o = pl + mul(Rl, mk(rec[BW_AP], rec[BW_AP + 1], rec[BW_AP + 2]));
          p = o - mul(R, mk(rec[BW_AC], rec[BW_AC + 1], rec[BW_AC + 2]));
          w = mul(R, u);
          sl = cross3(o - P0, w);
          const sv St = {w * thd, sl * thd};
          V = {Vl.a + St.a, Vl.l + St.l};
          const sv c = crm(Vl, St);
          A = {Al.a + c.a, Al.l + c.l};
        }
        float* dst = &sh.A[b * 24];
#pragma unroll
        for (int k2 = 0; k2 < 9; ++k2) dst[k2] = R.m[k2];
        dst[9] = p.x; dst[10] = p.y; dst[11] = p.z;
        dst[12] = V.a.x; dst[13] = V.a.y; dst[14] = V.a.z; dst[15] = V.l.x; dst[16] = V.l.y; dst[17] = V.l.z;
        dst[18] = A.a.x; dst[19] = A.a.y; dst[20] = A.a.z; dst[21] = A.l.x; dst[22] = A.l.y; dst[23] = A.l.z;
        sh.WO[b][0] = w.x; sh.WO[b][1] = w.y; sh.WO[b][2] = w.z;
        sh.WO[b][3] = sl.x; sh.WO[b][4] = sl.y; sh.WO[b][5] = sl.z;
        // box-plane contact: 8 corners, bits (x, y, z) of the corner index = sign
        if (b >= 1 || r0 == 6) {
          const f3 h = mk(rec[BW_HALF], rec[BW_HALF + 1], rec[BW_HALF + 2]);
          unsigned msk = 0u;
#pragma unroll
          for (int cn = 0; cn < 8; ++cn) {
            const float z = p.z + R.m[6] * ((cn & 1) ? h.x : -h.x) + R.m[7] * ((cn & 2) ? h.y : -h.y) +
                            R.m[8] * ((cn & 4) ? h.z : -h.z);
            if (z < 0.f) msk |= 1u << cn;
          }
          sh.ccount[b] = (int)msk;
        }
      }
      wave_sync();
    }
    // contact list in (body, corner) order: prefix over bodies of the popcounts
    int nc = 0;
    {
      // active corners per body, exclusive prefix over bodies by a DPP scan
      // across the row (slot 0 holds bodies 0..15, slot 1 bodies 16..31)
      int off[SB];
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int b = lane + 16 * t;
        const int cnt = (b < nb) ? __builtin_popcount((unsigned)sh.ccount[b]) : 0;
        const int incl = row_scan_incl(cnt);
        off[t] = nc + incl - cnt;
        nc += row_bcast_i<15>(incl);
      }
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int b = lane + 16 * t;
        if (b < nb) {
          const unsigned msk = (unsigned)sh.ccount[b];
          if (msk) {
            const float* pr = &sh.A[b * 24];
            const float* rec = bodyv + (size_t)b * BW_WORDS;
            const f3 h = mk(rec[BW_HALF], rec[BW_HALF + 1], rec[BW_HALF + 2]);
            const unsigned anc = __float_as_uint(rec[BW_ANCESTORS]);
            int idx = off[t];
            for (int cn = 0; cn < 8; ++cn) {
              if (msk & (1u << cn)) {
                const f3 sv3 = mk((cn & 1) ? h.x : -h.x, (cn & 2) ? h.y : -h.y, (cn & 4) ? h.z : -h.z);
                const f3 x = mk(pr[9] + pr[0] * sv3.x + pr[1] * sv3.y + pr[2] * sv3.z,
                                pr[10] + pr[3] * sv3.x + pr[4] * sv3.y + pr[5] * sv3.z,
                                pr[11] + pr[6] * sv3.x + pr[7] * sv3.y + pr[8] * sv3.z);
                const f3 up = mk(0.f, 0.f, 1.f);
                if (idx < NCR) put_contact<GEN>(&sh.cl[idx][0], x, anc, 0u, up, -x.z, 0);
                else put_contact<GEN>(&ovf_list[idx * CLW], x, anc, 0u, up, -x.z, 0);
                ++idx;
              }
            }
          }
        }
      }
    }
    int nself = 0;
    if (SELF) {
      // (i) bounding spheres of every pair, 16 pairs at a time; the
      // candidates are compacted in pair order (conservative test: every
      // corner hit passes it)
      int ncand = 0;
      for (int k0 = 0; k0 < npairs; k0 += 16) {
        const int k = k0 + lane;
        int cand = 0;
        uint16_t pr = 0;
        if (k < npairs) {
          pr = sh.spair[k];
          const int ia = pr & 0xff, ib = pr >> 8;
          const float* pa = &sh.A[ia * 24];
          const float* pb = &sh.A[ib * 24];
          const f3 d = mk(pb[9] - pa[9], pb[10] - pa[10], pb[11] - pa[11]);
          const float rr = sh.brad[ia] + sh.brad[ib];
          cand = dot3(d, d) <= rr * rr * 1.0001f ? 1 : 0;
        }
        if (__builtin_amdgcn_ballot_w64(cand != 0) == 0) continue;  // no candidate in any row of the wave
        const int incl = row_scan_incl(cand);
        if (cand) sh.scand[ncand + incl - 1] = pr;
        ncand += row_bcast_i<15>(incl);
      }
      wave_sync();  // candidates written by other lanes of the row
      // (ii) the candidates' corner tests, one pair per lane; hits placed in
      // pair order by a DPP scan, corners of a then of b
      for (int c0 = 0; c0 < ncand; c0 += 16) {
        const int ci = c0 + lane;
        unsigned hits = 0u;  // bits 0..7: corners of a in b, 8..15: corners of b in a, 16: edge-edge
        unsigned fmask = 0u;  // face contacts: the clipped incident face's candidates that exist
        int face = -1;        // their reference face (edge_contact's face case)
        f3 ex = mk(0.f, 0.f, 0.f), en = ex;  // the edge-edge contact's point and normal (towards a)
        float ed = 0.f;
        int ia = 0, ib = 0;
        m33 Ra, Rb;
        f3 Pa = mk(0.f, 0.f, 0.f), Pb = Pa, ha = Pa, hb = Pa;
        if (ci < ncand) {
          const uint16_t pr = sh.scand[ci];
          ia = pr & 0xff;
          ib = pr >> 8;
          const float* pa = &sh.A[ia * 24];
          const float* pb = &sh.A[ib * 24];
#pragma unroll
          for (int k2 = 0; k2 < 9; ++k2) Ra.m[k2] = pa[k2];
#pragma unroll
          for (int k2 = 0; k2 < 9; ++k2) Rb.m[k2] = pb[k2];
          Pa = mk(pa[9], pa[10], pa[11]);
          Pb = mk(pb[9], pb[10], pb[11]);
          const float* reca = bodyv + (size_t)ia * BW_WORDS;
          const float* recb = bodyv + (size_t)ib * BW_WORDS;
          ha = mk(reca[BW_HALF], reca[BW_HALF + 1], reca[BW_HALF + 2]);
          hb = mk(recb[BW_HALF], recb[BW_HALF + 1], recb[BW_HALF + 2]);
          for (int c = 0; c < 8; ++c)
            if (point_in_box(box_corner(Ra, Pa, ha, c), Pb, Rb, hb)) hits |= 1u << c;
          for (int c = 0; c < 8; ++c)
            if (point_in_box(box_corner(Rb, Pb, hb, c), Pa, Ra, ha)) hits |= 1u << (8 + c);
          // no corner inside: two crossing edges, if the boxes intersect there (bit
          // 16), or else an edge or face through a face (the clipped incident face)
          if (hits == 0u && edge_contact(Pa, Ra, ha, Pb, Rb, hb, ex, en, ed, face)) hits = 1u << 16;
          else if (hits == 0u && face >= 0) {
            FaceClip F;
            face_setup(Pa, Ra, ha, Pb, Rb, hb, face, F);
#pragma unroll 1
            for (int c = 0; c < 24; ++c) {
              f3 x;
              float dep;
              if (face_candidate(F, c, x, dep)) fmask |= 1u << c;
            }
          }
        }
        if (__builtin_amdgcn_ballot_w64((hits | fmask) != 0u) == 0) continue;  // no hit in any row of the wave
        const int cnt = __builtin_popcount(hits) + __builtin_popcount(fmask);
        const int incl = row_scan_incl(cnt);
        if (hits | fmask) {
          int idx = nc + incl - cnt;
          const unsigned anca = __float_as_uint(bodyv[(size_t)ia * BW_WORDS + BW_ANCESTORS]);
          const unsigned ancb = __float_as_uint(bodyv[(size_t)ib * BW_WORDS + BW_ANCESTORS]);
          if (fmask) {  // the clipped incident face again (same inputs, same points)
            FaceClip F;
            face_setup(Pa, Ra, ha, Pb, Rb, hb, face, F);
            const unsigned plus = F.on_q ? ancb : anca, minus = F.on_q ? anca : ancb;
#pragma unroll 1
            for (int c = 0; c < 24; ++c) {
              if (!((fmask >> c) & 1u)) continue;
              f3 x;
              float dep;
              face_candidate(F, c, x, dep);
              if (idx < NCR) put_contact<GEN>(&sh.cl[idx][0], x, plus, minus, F.n, dep, 3);
              else if (idx < MAXC) put_contact<GEN>(&ovf_list[idx * CLW], x, plus, minus, F.n, dep, 3);
              ++idx;
            }
          }
          if (hits == (1u << 16)) {
            if (idx < NCR) put_contact<GEN>(&sh.cl[idx][0], ex, anca, ancb, en, ed, 3);
            else if (idx < MAXC) put_contact<GEN>(&ovf_list[idx * CLW], ex, anca, ancb, en, ed, 3);
            hits = 0u;
          }
          const f3 u = sat_axis(Pa, Ra, ha, Pb, Rb, hb);  // from b towards a
          for (int c = 0; c < 16; ++c) {
            if (!((hits >> c) & 1u)) continue;
            const bool aside = c < 8;  // a corner of a inside b
            const f3 x = aside ? box_corner(Ra, Pa, ha, c) : box_corner(Rb, Pb, hb, c - 8);
            const f3 n = aside ? u : u * -1.f;
            const float depth = aside ? dot3(n, Pb) + box_radius(Rb, hb, n) - dot3(n, x)
                                      : dot3(n, Pa) + box_radius(Ra, ha, n) - dot3(n, x);
            const unsigned plus = aside ? anca : ancb, minus = aside ? ancb : anca;
            if (idx < NCR) put_contact<GEN>(&sh.cl[idx][0], x, plus, minus, n, depth, 3);
            else if (idx < MAXC) put_contact<GEN>(&ovf_list[idx * CLW], x, plus, minus, n, depth, 3);
            ++idx;
          }
        }
        const int tot = row_bcast_i<15>(incl);
        nc += tot;
        nself += tot;
      }
      if (nself > kMaxSelfContacts) {  // row-uniform: more than the list holds, freeze
        status |= 4u;
        break;
      }
    }
    if (BALL) {
      // the ball after the boxes: plane first (row-uniform), then every box
      // in body order (a scan over the body lanes); the box poses are in sh.A
      const f3 cb = mk(pb[0], pb[1], pb[2]);
      if (cb.z - rball < 0.f) {
        if (lane == 0) {
          const f3 x = mk(cb.x, cb.y, cb.z - rball);
          if (nc < NCR) put_contact<GEN>(&sh.cl[nc][0], x, 0u, 0u, mk(0.f, 0.f, 1.f), -x.z, 1);
          else put_contact<GEN>(&ovf_list[nc * CLW], x, 0u, 0u, mk(0.f, 0.f, 1.f), -x.z, 1);
        }
        ++nc;
      }
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int b = lane + 16 * t;
        f3 x = mk(0.f, 0.f, 0.f), n = x;
        float depth = 0.f;
        bool hit = false;
        if (b < nb) {
          const float* pr = &sh.A[b * 24];
          m33 R;
#pragma unroll
          for (int k2 = 0; k2 < 9; ++k2) R.m[k2] = pr[k2];
          const float* rec = bodyv + (size_t)b * BW_WORDS;
          hit = sphere_box(cb, rball, mk(pr[9], pr[10], pr[11]), R,
                           mk(rec[BW_HALF], rec[BW_HALF + 1], rec[BW_HALF + 2]), x, n, depth);
        }
        const int cnt = hit ? 1 : 0;
        const int incl = row_scan_incl(cnt);
        if (hit) {
          const int idx = nc + incl - cnt;
          const unsigned anc = __float_as_uint(bodyv[(size_t)b * BW_WORDS + BW_ANCESTORS]);
          if (idx < NCR) put_contact<GEN>(&sh.cl[idx][0], x, 0u, anc, n, depth, 2);
          else put_contact<GEN>(&ovf_list[idx * CLW], x, 0u, anc, n, depth, 2);
        }
        nc += row_bcast_i<15>(incl);
      }
    }
    __threadfence_block();  // overflow list entries are read by other lanes of the row
    wave_sync();

    // =====================================================================
    // 2. backward sweep, level by level up the tree: body inertia about p0
    //    and Newton-Euler force f = I A + V x* (I V); composite inertia C
    //    and force F of each subtree; hinge bias S.F and C S for CRBA
    // =====================================================================
    // each body's own inertia about p0 and Newton-Euler force first, for all
    // bodies at once (they need no child), in place of the body's kinematics
#pragma unroll
    for (int t = 0; t < SB; ++t) {
      const int b = lane + 16 * t;
      if (b < nb) {
        const float* rec = bodyv + (size_t)b * BW_WORDS;
        float* own = &sh.A[b * 24];
        sinertia C;
        sv F;
        {
          m33 R;
#pragma unroll
          for (int k2 = 0; k2 < 9; ++k2) R.m[k2] = own[k2];
          const f3 c = mk(own[9], own[10], own[11]) - P0;
          const sv V = {mk(own[12], own[13], own[14]), mk(own[15], own[16], own[17])};
          const sv A = {mk(own[18], own[19], own[20]), mk(own[21], own[22], own[23])};
          const float m = rec[BW_MASS];
          const f3 h = mk(rec[BW_HALF], rec[BW_HALF + 1], rec[BW_HALF + 2]);
          const float ix = m / 3.f * (h.y * h.y + h.z * h.z), iy = m / 3.f * (h.x * h.x + h.z * h.z),
                      iz = m / 3.f * (h.x * h.x + h.y * h.y);
          const float cc = dot3(c, c);
          C.m = m;
          C.h = c * m;
          C.I[0] = R.m[0] * R.m[0] * ix + R.m[1] * R.m[1] * iy + R.m[2] * R.m[2] * iz + m * (cc - c.x * c.x);
          C.I[1] = R.m[3] * R.m[3] * ix + R.m[4] * R.m[4] * iy + R.m[5] * R.m[5] * iz + m * (cc - c.y * c.y);
          C.I[2] = R.m[6] * R.m[6] * ix + R.m[7] * R.m[7] * iy + R.m[8] * R.m[8] * iz + m * (cc - c.z * c.z);
          C.I[3] = R.m[0] * R.m[3] * ix + R.m[1] * R.m[4] * iy + R.m[2] * R.m[5] * iz - m * c.x * c.y;
          C.I[4] = R.m[0] * R.m[6] * ix + R.m[1] * R.m[7] * iy + R.m[2] * R.m[8] * iz - m * c.x * c.z;
          C.I[5] = R.m[3] * R.m[6] * ix + R.m[4] * R.m[7] * iy + R.m[5] * R.m[8] * iz - m * c.y * c.z;
          const sv IV = imul(C, V), IA = imul(C, A);
          const sv x = crf(V, IV);
          F = {IA.a + x.a, IA.l + x.l};
        }
        own[0] = C.m; own[1] = C.h.x; own[2] = C.h.y; own[3] = C.h.z;
#pragma unroll
        for (int k2 = 0; k2 < 6; ++k2) own[4 + k2] = C.I[k2];
        own[10] = F.a.x; own[11] = F.a.y; own[12] = F.a.z;
        own[13] = F.l.x; own[14] = F.l.y; own[15] = F.l.z;
      }
    }
    wave_sync();
    // then the subtrees level by level up the tree
    for (int lev = maxdepth; lev >= 0; --lev) {
      const int i1 = sh.lv[NBC + lev + 1];
      for (int i = sh.lv[NBC + lev] + lane; i < i1; i += 16) {
        const int b = sh.lv[i];
        const float* rec = bodyv + (size_t)b * BW_WORDS;
        float* own = &sh.A[b * 24];
        sinertia C;
        sv F;
        C.m = own[0];
        C.h = mk(own[1], own[2], own[3]);
#pragma unroll
        for (int k2 = 0; k2 < 6; ++k2) C.I[k2] = own[4 + k2];
        F.a = mk(own[10], own[11], own[12]);
        F.l = mk(own[13], own[14], own[15]);
        unsigned ch = __float_as_uint(rec[BW_CHILDREN]);
        while (ch) {
          const int c = __builtin_ctz(ch);
          ch &= ch - 1;
          const float* src = &sh.A[c * 24];
          C.m += src[0];
          C.h = C.h + mk(src[1], src[2], src[3]);
#pragma unroll
          for (int k2 = 0; k2 < 6; ++k2) C.I[k2] += src[4 + k2];
          F.a = F.a + mk(src[10], src[11], src[12]);
          F.l = F.l + mk(src[13], src[14], src[15]);
        }
        own[0] = C.m; own[1] = C.h.x; own[2] = C.h.y; own[3] = C.h.z;
#pragma unroll
        for (int k2 = 0; k2 < 6; ++k2) own[4 + k2] = C.I[k2];
        own[10] = F.a.x; own[11] = F.a.y; own[12] = F.a.z;
        own[13] = F.l.x; own[14] = F.l.y; own[15] = F.l.z;
        if (b >= 1) {
          const sv Sb = {mk(sh.WO[b][0], sh.WO[b][1], sh.WO[b][2]), mk(sh.WO[b][3], sh.WO[b][4], sh.WO[b][5])};
          sh.cvec[r0 + b - 1] = dot3(Sb.a, F.a) + dot3(Sb.l, F.l);
          const sv Fc = imul(C, Sb);
          sh.WO[b][6] = Fc.a.x; sh.WO[b][7] = Fc.a.y; sh.WO[b][8] = Fc.a.z;
          sh.WO[b][9] = Fc.l.x; sh.WO[b][10] = Fc.l.y; sh.WO[b][11] = Fc.l.z;
        }
      }
      wave_sync();
    }
    // root bias and root rows of M from the total composite (lanes 0..5)
    float mroot[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) mroot[i] = 0.f;
    if (r0 == 6 && lane < 6) {
      const float* src = &sh.A[0];
      const float m = src[0];
      const f3 hw = mk(src[1], src[2], src[3]);
      float Iw[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) Iw[i] = src[4 + i];
      const f3 Fa = mk(src[10], src[11], src[12]), Fl = mk(src[13], src[14], src[15]);
      const f3 ca = mulT(R0, Fa), cl = mulT(R0, Fl);
      const int i = lane;
      sh.cvec[i] = (i < 3) ? (i == 0 ? ca.x : i == 1 ? ca.y : ca.z) : (i == 3 ? cl.x : i == 4 ? cl.y : cl.z);
      // M_rr = [[R^T Io R, [h_b]x], [[h_b]x^T, m 1]] with h_b = R^T h; column j of [h_b]x is h_b x e_j
      const f3 hb = mulT(R0, hw);
      const f3 hx0 = cross3(hb, mk(1.f, 0.f, 0.f)), hx1 = cross3(hb, mk(0.f, 1.f, 0.f)),
               hx2 = cross3(hb, mk(0.f, 0.f, 1.f));
      if (i < 3) {
        const f3 e = mcol(R0, i);  // R0 e_i (column i)
        const f3 row = mulT(R0, symmul(Iw, e));             // row i of R^T Io R
        mroot[0] = row.x; mroot[1] = row.y; mroot[2] = row.z;
        mroot[3] = (i == 0) ? hx0.x : (i == 1) ? hx0.y : hx0.z;
        mroot[4] = (i == 0) ? hx1.x : (i == 1) ? hx1.y : hx1.z;
        mroot[5] = (i == 0) ? hx2.x : (i == 1) ? hx2.y : hx2.z;
      } else {
        const int r = i - 3;  // row r of [h_b]x^T = column r of [h_b]x
        const f3 col = (r == 0) ? hx0 : (r == 1) ? hx1 : hx2;
        mroot[0] = col.x; mroot[1] = col.y; mroot[2] = col.z;
        mroot[3] = (r == 0) ? m : 0.f; mroot[4] = (r == 1) ? m : 0.f; mroot[5] = (r == 2) ? m : 0.f;
      }
    }
    if (BALL && lane < 6)  // ball: bias -m g on the centre velocity, none on the spin
      sh.cvec[nvr + lane] = lane < 3 ? 0.f : -mball * (lane == 3 ? P.g[0] : lane == 4 ? P.g[1] : P.g[2]);
    wave_sync();  // composite reads done; the area becomes the assembled matrix
    {
      float4* a4 = reinterpret_cast<float4*>(sh.A);  // A is 16-byte aligned (first member)
      for (int e = lane; e < (NVC * MST + 3) / 4; e += 16) a4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    wave_sync();
    {
      float* Ml = sh.A;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        if (d >= nv && d < NVC) Ml[d * MST + d] = 1.f;  // identity padding
        if (BALL && d >= nvr && d < nv) Ml[d * MST + d] = (d - nvr < 3) ? iball : mball;
      }
      if (r0 == 6 && lane < 6) {
#pragma unroll
        for (int j = 0; j < 6; ++j) Ml[lane * MST + j] = mroot[j];
      }
#pragma unroll
      for (int t = 0; t < SB; ++t) {
        const int b = lane + 16 * t;
        if (b >= 1 && b < nb) {
          const int d = r0 + b - 1;
          const sv Fcb = {mk(sh.WO[b][6], sh.WO[b][7], sh.WO[b][8]), mk(sh.WO[b][9], sh.WO[b][10], sh.WO[b][11])};
          // the hinges of b and its ancestors (the core has none), by the
          // ancestor mask: no pointer chase through LDS
          unsigned am = ancS[t] & ~1u;
          while (am) {
            const int j = __builtin_ctz(am);
            am &= am - 1u;
            const int dj = r0 + j - 1;
            const f3 wj = mk(sh.WO[j][0], sh.WO[j][1], sh.WO[j][2]);
            const f3 slj = mk(sh.WO[j][3], sh.WO[j][4], sh.WO[j][5]);
            float val = dot3(wj, Fcb.a) + dot3(slj, Fcb.l);
            if (j == b) val += dt * ba;
            Ml[d * MST + dj] = val;
            Ml[dj * MST + d] = val;
          }
          if (r0 == 6) {
            const f3 ra = mulT(R0, Fcb.a), rl = mulT(R0, Fcb.l);
            const float rv[6] = {ra.x, ra.y, ra.z, rl.x, rl.y, rl.z};
#pragma unroll
            for (int i = 0; i < 6; ++i) {
              Ml[d * MST + i] = rv[i];
              Ml[i * MST + d] = rv[i];
            }
          }
        }
      }
    }
    wave_sync();
    float Mi[S][NVC];
    float cS[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      const int dr = d < NVC ? d : 0;
#pragma unroll
      for (int j = 0; j < NVC; ++j) Mi[s][j] = sh.A[dr * MST + j];
      cS[s] = (d < nv) ? sh.cvec[d] : 0.f;
    }

    if constexpr (TREE) {
      // ===================================================================
      // 3. (tree-sparse alternative) M~ = L^T L with L lower triangular and
      //    row i of L nonzero only on i's path (i and its ancestors), so
      //    factoring from the last DoF to the first creates no fill-in
      //    (Featherstone's branch-induced sparsity).  The factor overwrites
      //    the lower triangle of the assembled matrix; each pivot's ancestor
      //    rows are updated by their owner lanes along their own paths.  Then
      //    every lane forms the column of M~^-1 of its own DoF c by two
      //    triangular solves in its own row of X: L^T y = e_c (y lives on
      //    c's path) and L x = y (x is row c too, M~^-1 being symmetric).
      // ===================================================================
      // The first six DoFs (the free root's chain, on every path) are held in
      // registers or read in one batch; the hinge ancestors of a DoF are
      // taken up to four at a time (one LDS round trip), any deeper rest one
      // by one.
      constexpr int R6 = 6;
      constexpr unsigned kRootBits = (1u << R6) - 1u;
      constexpr int HB = 4;
      unsigned pmS[S];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        pmS[s] = d < nv ? sh.pm[d] : 0u;
      }
      // first HB set bits of m (removed from m), with their validity
      auto take = [](unsigned& m, int (&jj)[HB], bool (&ok)[HB]) {
#pragma unroll
        for (int p = 0; p < HB; ++p) {
          ok[p] = m != 0u;
          jj[p] = ok[p] ? __builtin_ctz(m) : 0;
          m &= m - 1u;
        }
      };
#pragma unroll 1
      for (int k = nv - 1; k >= 0; --k) {
        const unsigned ak = sh.pm[k] & ~(1u << k);  // ancestors of k
        const float lkk = sqrtf(sh.A[k * MST + k]);
        const float r = recip(lkk);
        float lk[S];
        bool in[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int d = lane + 16 * s;
          in[s] = (ak >> d) & 1u;
          lk[s] = in[s] ? sh.A[k * MST + d] * r : 0.f;  // L[k][d]
          if (in[s]) sh.A[k * MST + d] = lk[s];
          if (d == k) {
            sh.A[k * MST + k] = lkk;
            sh.dinv[k] = r;
          }
        }
        wave_sync();
        // rows d of k's ancestors: A[d][j] -= L[k][d] L[k][j] along d's path
        const float* rk = &sh.A[k * MST];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          if (in[s]) {
            const int d = lane + 16 * s;
            float* rd = &sh.A[d * MST];
            float a0[R6], b0[R6], ah[HB], bh[HB];
            int jj[HB];
            bool ok[HB];
            unsigned mh = pmS[s] & ~kRootBits;
            take(mh, jj, ok);
#pragma unroll
            for (int j = 0; j < R6; ++j) { a0[j] = rk[j]; b0[j] = rd[j]; }
#pragma unroll
            for (int p = 0; p < HB; ++p) { ah[p] = rk[jj[p]]; bh[p] = rd[jj[p]]; }
#pragma unroll
            for (int j = 0; j < R6; ++j)
              if ((pmS[s] >> j) & 1u) rd[j] = fmaf(-lk[s], a0[j], b0[j]);
#pragma unroll
            for (int p = 0; p < HB; ++p)
              if (ok[p]) rd[jj[p]] = fmaf(-lk[s], ah[p], bh[p]);
            while (mh) {
              const int j = __builtin_ctz(mh);
              mh &= mh - 1u;
              rd[j] = fmaf(-lk[s], rk[j], rd[j]);
            }
          }
        }
        wave_sync();
      }
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        if (d < NVC) {
#pragma unroll
          for (int j = 0; j < NVC; ++j) sh.X[d * MST + j] = (j == d && d < nv) ? 1.f : 0.f;
        }
      }
      // the factor's first six rows and reciprocal diagonal (uniform per variant)
      float L6[R6][R6], di6[R6];
      unsigned pm6[R6];
#pragma unroll
      for (int i = 0; i < R6; ++i) {
        di6[i] = sh.dinv[i < nv ? i : 0];
        pm6[i] = i < nv ? sh.pm[i] : 0u;
#pragma unroll
        for (int j = 0; j < i; ++j) L6[i][j] = sh.A[i * MST + j];
      }
      // L^T y = e_c, c the lane's DoF: y lives on c's path; its hinge part
      // from c upwards with the root entries of the right-hand side kept in
      // registers, then the six root entries
      float y6[S][R6];
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        float br[R6];
#pragma unroll
        for (int j = 0; j < R6; ++j) br[j] = (j == d) ? 1.f : 0.f;
        if (d < nv) {
          float* xr = &sh.X[d * MST];
          const unsigned mr = pmS[s] & kRootBits;
          unsigned mh = pmS[s] & ~kRootBits;
          while (mh) {
            const int i = 31 - __builtin_clz(mh);
            mh &= ~(1u << i);
            const float yi = xr[i] * sh.dinv[i];
            xr[i] = yi;
            const float* li = &sh.A[i * MST];
#pragma unroll
            for (int j = 0; j < R6; ++j)
              if ((mr >> j) & 1u) br[j] = fmaf(-li[j], yi, br[j]);
            unsigned an = mh;  // the rest of the path: i's hinge ancestors
            float lh[HB], xh[HB];
            int jj[HB];
            bool ok[HB];
            take(an, jj, ok);
#pragma unroll
            for (int p = 0; p < HB; ++p) { lh[p] = li[jj[p]]; xh[p] = xr[jj[p]]; }
#pragma unroll
            for (int p = 0; p < HB; ++p)
              if (ok[p]) xr[jj[p]] = fmaf(-lh[p], yi, xh[p]);
            while (an) {
              const int j = __builtin_ctz(an);
              an &= an - 1u;
              xr[j] = fmaf(-li[j], yi, xr[j]);
            }
          }
        }
#pragma unroll
        for (int i = R6 - 1; i >= 0; --i) {
          const bool on = d < nv && ((pmS[s] >> i) & 1u);
          y6[s][i] = on ? br[i] * di6[i] : 0.f;
#pragma unroll
          for (int j = 0; j < i; ++j) br[j] = fmaf(-L6[i][j], y6[s][i], br[j]);
        }
      }
      // L x = y over the DoFs in order: the root entries of x in registers,
      // then each hinge DoF along its ancestors
      int dr[S];
#pragma unroll
      for (int s = 0; s < S; ++s) dr[s] = (lane + 16 * s) < NVC ? lane + 16 * s : 0;
      float x6[S][R6];
#pragma unroll
      for (int i = 0; i < R6; ++i) {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          float acc = y6[s][i];
#pragma unroll
          for (int j = 0; j < i; ++j)
            if ((pm6[i] >> j) & 1u) acc = fmaf(-L6[i][j], x6[s][j], acc);
          x6[s][i] = i < nv ? acc * di6[i] : 0.f;
          if (lane + 16 * s < NVC) sh.X[dr[s] * MST + i] = x6[s][i];
        }
      }
#pragma unroll 1
      for (int i = R6; i < nv; ++i) {
        const float* li = &sh.A[i * MST];
        const float di = sh.dinv[i];
        const unsigned pi = sh.pm[i];
        float l0[R6];
#pragma unroll
        for (int j = 0; j < R6; ++j) l0[j] = li[j];
        unsigned an = pi & ~kRootBits & ~(1u << i);
        float lh[HB], xh[S][HB];
        int jj[HB];
        bool ok[HB];
        take(an, jj, ok);
        float acc[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          acc[s] = sh.X[dr[s] * MST + i];
#pragma unroll
          for (int p = 0; p < HB; ++p) xh[s][p] = sh.X[dr[s] * MST + jj[p]];
        }
#pragma unroll
        for (int p = 0; p < HB; ++p) lh[p] = ok[p] ? li[jj[p]] : 0.f;
#pragma unroll
        for (int s = 0; s < S; ++s) {
#pragma unroll
          for (int j = 0; j < R6; ++j)
            if ((pi >> j) & 1u) acc[s] = fmaf(-l0[j], x6[s][j], acc[s]);
#pragma unroll
          for (int p = 0; p < HB; ++p) acc[s] = fmaf(-lh[p], xh[s][p], acc[s]);
        }
        while (an) {
          const int j = __builtin_ctz(an);
          an &= an - 1u;
          const float l = li[j];
#pragma unroll
          for (int s = 0; s < S; ++s) acc[s] = fmaf(-l, sh.X[dr[s] * MST + j], acc[s]);
        }
#pragma unroll
        for (int s = 0; s < S; ++s)
          if (lane + 16 * s < NVC) sh.X[dr[s] * MST + i] = acc[s] * di;
      }
      // registers and X hold the inverse negated, natural column order
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
#pragma unroll
        for (int j = 0; j < NVC; ++j) {
          Mi[s][j] = d < NVC ? -sh.X[dr[s] * MST + j] : 0.f;
          if (d < NVC) sh.X[d * MST + j] = Mi[s][j];
        }
      }
    } else {
      // =====================================================================
      // 3. inverse by a symmetric Gauss-Jordan sweep over the nv real pivots,
      //    rows in registers, columns rotating by one per pivot (register
      //    column j of step k holds original column (k + j) mod NVC).  The
      //    pivot column is broadcast through a doubled LDS buffer.  Pivot row
      //    k uses the symmetric column values: a_kj - (1 - 1/d) a_jk.
      //    Result: -M~^-1 with register column j <-> column (nv + j) mod NVC.
      //    Software-pipelined: the first updated column of step k is column 0
      //    of step k + 1, so it is broadcast (and read back into the other
      //    register set) before the rest of step k's updates, which hide the
      //    LDS round trip; the arithmetic is that of the plain sweep.
      // =====================================================================
      {
        float ckA[NVC], ckB[NVC];  // pivot column of the current / next step
        // Store positions of the lane's rows in a broadcast buffer: row d at d
        // and d + NVC; a slot past the last DoF writes both copies into the
        // sink at 2 NVC + (d - NVC) < 2 NVC + 16, so the stores need no branch
        // (a branch there splits the step and lets the compiler sink its
        // updates below the next step's reads).
        int cb_lo[S], cb_hi[S];
  #pragma unroll
        for (int s = 0; s < S; ++s) {
          const int d = lane + 16 * s;
          cb_lo[s] = d < NVC ? d : NVC + d;
          cb_hi[s] = d < NVC ? d + NVC : NVC + d;
        }
  #pragma unroll
        for (int s = 0; s < S; ++s) { sh.cb[0][cb_lo[s]] = Mi[s][0]; sh.cb[0][cb_hi[s]] = Mi[s][0]; }
        wave_sync();
  #pragma unroll
        for (int j = 0; j < NVC; ++j) ckA[j] = sh.cb[0][j];
        auto pivot_step = [&](int k, const float (&ck)[NVC], float (&nck)[NVC]) {
          const float pinv = recip(ck[0]);
          float f[S];
          bool piv[S];
  #pragma unroll
          for (int s = 0; s < S; ++s) {
            piv[s] = (lane + 16 * s) == k;
            f[s] = piv[s] ? 1.f - pinv : Mi[s][0] * pinv;
          }
  #pragma unroll
          for (int s = 0; s < S; ++s) Mi[s][0] = fmaf(-f[s], ck[1], Mi[s][1]);
          float* cbn = sh.cb[(k + 1) & 1];
  #pragma unroll
          for (int s = 0; s < S; ++s) { cbn[cb_lo[s]] = Mi[s][0]; cbn[cb_hi[s]] = Mi[s][0]; }
          wave_sync();
  #pragma unroll
          for (int j = 0; j < NVC; ++j) nck[j] = cbn[k + 1 + j];  // k + 1 <= NVC: inside the doubled buffer
          // keep the scheduler from hoisting the next step's chain above this
          // step's updates (which would leave the reads' latency exposed)
          __builtin_amdgcn_sched_barrier(0);
  #pragma unroll
          for (int j = 2; j < NVC; ++j) {
  #pragma unroll
            for (int s = 0; s < S; ++s) Mi[s][j - 1] = fmaf(-f[s], ck[j], Mi[s][j]);
          }
  #pragma unroll
          for (int s = 0; s < S; ++s) Mi[s][NVC - 1] = piv[s] ? -pinv : f[s];
          __builtin_amdgcn_sched_barrier(0);
        };
        // whole pairs of steps (no branch between a step's reads and their use,
        // so the compiler keeps them ahead of the step's updates), then an odd
        // last step
        int k = 0;
  #pragma unroll 1
        for (; k + 1 < nv; k += 2) {
          pivot_step(k, ckA, ckB);
          pivot_step(k + 1, ckB, ckA);
        }
        if (k < nv) pivot_step(k, ckA, ckB);
      }
      // the assembled matrix is dead: keep the (negated, rotated) inverse in LDS
      // for the clamp rows, which need single columns chosen at run time, and
      // reload the registers in natural column order for the mat-vecs
      wave_sync();
  #pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        if (d < NVC) {
  #pragma unroll
          for (int j = 0; j < NVC; ++j) sh.A[d * MST + j] = Mi[s][j];
        }
      }
      wave_sync();
  #pragma unroll
      for (int s = 0; s < S; ++s) {
        const int dr = (lane + 16 * s) < NVC ? lane + 16 * s : 0;
  #pragma unroll
        for (int c = 0; c < NVC; ++c) {
          const int j = c - nv + (c < nv ? NVC : 0);  // register column of original column c
          Mi[s][c] = sh.A[dr * MST + j];
        }
      }
    }
    // the negated inverse in LDS: rotated columns after the sweep, natural
    // after the tree-sparse solves
    const float* const Ainv = TREE ? &sh.X[0] : &sh.A[0];
    float Dd[S];  // own diagonal of M~^-1
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      int cidx = d - nv;
      cidx += (cidx < 0) ? NVC : 0;
      if (TREE) cidx = d < NVC ? d : 0;
      Dd[s] = (d < nv) ? -Ainv[d * MST + cidx] : 0.f;
    }

    // =====================================================================
    // 4. control and free velocity
    // =====================================================================
    const double tk = (double)kstep * dtd;
    float aS[S], nrhs[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      const bool hinge = d >= r0 && d < nvr;
      const int b = hinge ? d - r0 + 1 : 0;
      const float* rec = bodyv + (size_t)b * BW_WORDS;
      double ph = (double)rec[BW_CPG + 1] * tk + (double)rec[BW_CPG + 2];
      ph -= 6.283185307179586 * floor(ph * 0.15915494309189535);
      float sph, cph;
      sincos_moderate((float)ph, &sph, &cph);  // phase reduced to [0, 2 pi)
      const float target = rec[BW_CPG] * sph;
      aS[s] = hinge ? kp * (target - thS[s]) : 0.f;
      float rhs = -dt * cS[s];
      if (hinge) rhs += dt * (aS[s] - ba * vS[s]);
      if (d >= nv) rhs = 0.f;
      nrhs[s] = -rhs;  // sign of the held inverse
    }
    float vp[S];
#pragma unroll
    for (int s = 0; s < S; ++s) vp[s] = vS[s];
    matvec_bcast1<S, NVC>(Mi, nrhs, vp);

    // =====================================================================
    // 5. contact rows
    // =====================================================================
    // per-DoF geometry of the point Jacobian: J_d(x) = ang_d x x + cst_d (zero off the path)
    f3 ang[S], cst[S];
    int bodyOfDof[S];
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      bodyOfDof[s] = -1;
      if (r0 == 6 && d < 3) {
        ang[s] = mcol(R0, d);
        cst[s] = mk(0.f, 0.f, 0.f) - cross3(ang[s], P0);
      } else if (r0 == 6 && d < 6) {
        ang[s] = mk(0.f, 0.f, 0.f);
        cst[s] = mcol(R0, d - 3);
      } else if (d < nvr) {
        const int b = d - r0 + 1;
        bodyOfDof[s] = b;
        ang[s] = mk(sh.WO[b][0], sh.WO[b][1], sh.WO[b][2]);
        // w x (x - o) = w x x + (o - p0) x w + p0 x w
        cst[s] = (mk(0.f, 0.f, 0.f) - cross3(ang[s], P0)) + mk(sh.WO[b][3], sh.WO[b][4], sh.WO[b][5]);
      } else if (BALL && d < nv) {
        // ball: spin e_k gives e_k x (x - cb), centre velocity e_k gives e_k
        const int k = d - nvr;
        const f3 e = mk((k % 3) == 0 ? 1.f : 0.f, (k % 3) == 1 ? 1.f : 0.f, (k % 3) == 2 ? 1.f : 0.f);
        bodyOfDof[s] = -2;
        ang[s] = k < 3 ? e : mk(0.f, 0.f, 0.f);
        cst[s] = k < 3 ? mk(0.f, 0.f, 0.f) - cross3(e, mk(pb[0], pb[1], pb[2])) : e;
      } else {
        ang[s] = mk(0.f, 0.f, 0.f);
        cst[s] = mk(0.f, 0.f, 0.f);
      }
    }
    float JnR[NCR][S], JxR[NCR][S], JyR[NCR][S], WnR[NCR][S], WxR[NCR][S], WyR[NCR][S];
    // The contacts' solver scalars and multipliers: in registers for the
    // single-wave families of 20 DoFs and more with at most 8 contacts in
    // registers (above 256 registers anyway, with room left below 512; their
    // sweeps would otherwise wait on an LDS read at every contact), else in
    // LDS: the smaller families fit 256 registers and run two waves per SIMD,
    // which the 80 more registers would cost them.
    constexpr bool SREG = WavesPerSimd<NVC, SB, NCR>::value == 1 && NVC >= 20 && NCR <= 8;
    float scR[SREG ? NCR : 1][10];
#pragma unroll
    for (int c = 0; c < NCR; ++c) {
      if (c < nc) {
        const f3 x = mk(sh.cl[c][CL_X], sh.cl[c][CL_X + 1], sh.cl[c][CL_X + 2]);
        const unsigned anc = __float_as_uint(sh.cl[c][CL_ANC]);
        float scal[10];
        if constexpr (GEN) {
          const int kind = (int)sh.cl[c][CL_KIND];
          build_rows_gen<S, NVC>(Mi, ang, cst, bodyOfDof, x, mk(sh.cl[c][CL_N], sh.cl[c][CL_N + 1], sh.cl[c][CL_N + 2]),
                                 sh.cl[c][CL_DEPTH], anc, __float_as_uint(sh.cl[c][CL_MINUS]), kind == 1 || kind == 2,
                                 kind == 3, kc, kb, dt, JnR[c], JxR[c], JyR[c], WnR[c], WxR[c], WyR[c], scal);
        }
        else
          build_rows<S, NVC>(Mi, ang, cst, bodyOfDof, lane, x, anc, kc, kb, dt, JnR[c], JxR[c], JyR[c], WnR[c],
                             WxR[c], WyR[c], scal);
#pragma unroll
        for (int i = 0; i < 10; ++i) {
          if constexpr (SREG) scR[c][i] = scal[i];
          else sh.cs[c][i] = scal[i];  // identical in every lane
        }
      } else {
#pragma unroll
        for (int s = 0; s < S; ++s) {
          JnR[c][s] = JxR[c][s] = JyR[c][s] = 0.f;
          WnR[c][s] = WxR[c][s] = WyR[c][s] = 0.f;
        }
        if constexpr (SREG) {
#pragma unroll
          for (int i = 0; i < 10; ++i) scR[c][i] = 0.f;
        }
      }
    }
    // contacts beyond the register budget: rows and scalars go to the workspace.
    // Each lane stores and later reloads only values it computed itself (the
    // scalars are identical in all lanes), so no cross-lane visibility is needed.
    for (int c = NCR; c < nc; ++c) {
      const float* e = &ovf_list[c * CLW];
      const f3 x = mk(e[CL_X], e[CL_X + 1], e[CL_X + 2]);
      const unsigned anc = __float_as_uint(e[CL_ANC]);
      float Jn[S], Jx[S], Jy[S], Wn[S], Wx[S], Wy[S], scal[10];
      if constexpr (GEN) {
        const int kind = (int)e[CL_KIND];
        build_rows_gen<S, NVC>(Mi, ang, cst, bodyOfDof, x, mk(e[CL_N], e[CL_N + 1], e[CL_N + 2]), e[CL_DEPTH], anc,
                               __float_as_uint(e[CL_MINUS]), kind == 1 || kind == 2, kind == 3, kc, kb, dt, Jn, Jx,
                               Jy, Wn, Wx, Wy, scal);
      }
      else
        build_rows<S, NVC>(Mi, ang, cst, bodyOfDof, lane, x, anc, kc, kb, dt, Jn, Jx, Jy, Wn, Wx, Wy, scal);
      float* rows = ovf_rows + (size_t)c * 6 * NVC;
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        if (d < NVC) {
          rows[0 * NVC + d] = Jn[s]; rows[1 * NVC + d] = Jx[s]; rows[2 * NVC + d] = Jy[s];
          rows[3 * NVC + d] = Wn[s]; rows[4 * NVC + d] = Wx[s]; rows[5 * NVC + d] = Wy[s];
        }
      }
      float* sd = ovf_scal + (size_t)c * kOvfScal;
#pragma unroll
      for (int i = 0; i < 10; ++i) sd[i] = scal[i];
    }

    // =====================================================================
    // 6. projected Gauss-Seidel
    // =====================================================================
    float Dl[S];    // actuator clamp corrections Delta, held by the DoF's owner lane/slot
    float rden[S];  // 1 / (1 - b_a dt D_jj), fixed for the step
#pragma unroll
    for (int s = 0; s < S; ++s) {
      Dl[s] = 0.f;
      rden[s] = 1.f / (1.f - ba * dt * Dd[s]);
    }
    constexpr int kNoRow = 1 << 20;
    for (int sweep = 0; sweep < P.K; ++sweep) {
      // (i) actuator clamp rows in hinge order.  Every remaining row is
      // evaluated against the current velocity; rows whose new Delta equals
      // the old one are no-ops, so only the lowest changing row is applied,
      // and the rest re-evaluated after it: the same result as visiting every
      // row in order.
      int last = -1;  // row-uniform: last hinge DoF applied in this sweep
      while (true) {
        int first = kNoRow;
        float ndv[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int d = lane + 16 * s;
          const float u0 = fmaf(dt * Dd[s], Dl[s], vp[s]);
          const float sv_ = aS[s] - ba * u0;
          // the part of the PD law beyond the torque limit, scaled
          const float over = sv_ > tmax ? sv_ - tmax : (sv_ < -tmax ? sv_ + tmax : 0.f);
          const float nd = over != 0.f ? over * rden[s] : 0.f;
          ndv[s] = nd;
          if (d >= r0 && d < nvr && d > last && nd != Dl[s]) first = min(first, d);
        }
        if (__builtin_amdgcn_ballot_w64(first < kNoRow) == 0) break;  // no row of any variant changes
        first = row_min_i(first);
        if (first < kNoRow) {  // row-uniform
          const int j = first;
          float dl = 0.f;
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const bool own = (lane + 16 * s) == j;
            dl += own ? ndv[s] - Dl[s] : 0.f;
            Dl[s] = own ? ndv[s] : Dl[s];
          }
          dl = row_sum(dl);
          int cj = j - nv;
          cj += (cj < 0) ? NVC : 0;
          if (TREE) cj = j;
          const float e = dt * dl;  // v+ -= dt M~^-1 e_j dl, inverse held negated
#pragma unroll
          for (int s = 0; s < S; ++s) {
            const int d = lane + 16 * s;
            const float mcol = Ainv[(d < NVC ? d : NVC - 1) * MST + cj];  // unmasked read
            vp[s] = fmaf(d < NVC ? mcol : 0.f, e, vp[s]);
          }
          last = j;
        }
      }
      // (ii) contact rows in (body, corner) order
#pragma unroll
      for (int c = 0; c < NCR; ++c) {
        if (c < nc) {
          float sc[10], lam[3];
#pragma unroll
          for (int i = 0; i < 10; ++i) sc[i] = SREG ? scR[c][i] : sh.cs[c][i];
          lam[0] = sc[7]; lam[1] = sc[8]; lam[2] = sc[9];
          contact_row<S>(vp, JnR[c], JxR[c], JyR[c], WnR[c], WxR[c], WyR[c], sc, lam, mu, dt);
          if constexpr (SREG) {
            scR[c][7] = lam[0]; scR[c][8] = lam[1]; scR[c][9] = lam[2];
          } else {
            sh.cs[c][7] = lam[0]; sh.cs[c][8] = lam[1]; sh.cs[c][9] = lam[2];
          }
        }
      }
      for (int c = NCR; c < nc; ++c) {
        const float* rows = ovf_rows + (size_t)c * 6 * NVC;
        float Jn[S], Jx[S], Jy[S], Wn[S], Wx[S], Wy[S];
#pragma unroll
        for (int s = 0; s < S; ++s) {
          const int d = lane + 16 * s;
          const bool ok = d < NVC;
          Jn[s] = ok ? rows[0 * NVC + d] : 0.f; Jx[s] = ok ? rows[1 * NVC + d] : 0.f;
          Jy[s] = ok ? rows[2 * NVC + d] : 0.f; Wn[s] = ok ? rows[3 * NVC + d] : 0.f;
          Wx[s] = ok ? rows[4 * NVC + d] : 0.f; Wy[s] = ok ? rows[5 * NVC + d] : 0.f;
        }
        float* sd = ovf_scal + (size_t)c * kOvfScal;
        float sc[10], lam[3];
#pragma unroll
        for (int i = 0; i < 10; ++i) sc[i] = sd[i];
        lam[0] = sc[7]; lam[1] = sc[8]; lam[2] = sc[9];
        contact_row<S>(vp, Jn, Jx, Jy, Wn, Wx, Wy, sc, lam, mu, dt);
        sd[7] = lam[0]; sd[8] = lam[1]; sd[9] = lam[2];
      }
    }

    // =====================================================================
    // 7. semi-implicit Euler, failure check, counters
    // =====================================================================
    const f3 wn = mk(row_bcast<0>(vp[0]), row_bcast<1>(vp[0]), row_bcast<2>(vp[0]));
    const f3 vn = mk(row_bcast<3>(vp[0]), row_bcast<4>(vp[0]), row_bcast<5>(vp[0]));
    float thN[S];
    float bad = 0.f, nclamp = 0.f;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      const bool hinge = d >= r0 && d < nvr;
      thN[s] = hinge ? fmaf(dt, vp[s], thS[s]) : 0.f;
      if (d < nv && !(isfinite(vp[s]) && isfinite(thN[s]))) bad = 1.f;
      if (hinge && Dl[s] != 0.f) nclamp += 1.f;
    }
    float p0n[3] = {p0[0], p0[1], p0[2]}, Q0n[4] = {Q0[0], Q0[1], Q0[2], Q0[3]};
    if (r0 == 6) {
      const f3 dp = mul(R0, vn);
      p0n[0] = fmaf(dt, dp.x, p0[0]); p0n[1] = fmaf(dt, dp.y, p0[1]); p0n[2] = fmaf(dt, dp.z, p0[2]);
      quat_step<true>(Q0n, wn * dt);  // body-frame rate
      bool ok = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) ok = ok && isfinite(p0n[i]);
#pragma unroll
      for (int i = 0; i < 4; ++i) ok = ok && isfinite(Q0n[i]);
      if (!ok) bad = 1.f;
    }
    float pbn[3] = {pb[0], pb[1], pb[2]}, Qbn[4] = {Qb[0], Qb[1], Qb[2], Qb[3]};
    if (BALL) {
      // ball velocities from their owner lanes (the bias vector is dead by now)
#pragma unroll
      for (int s = 0; s < S; ++s) {
        const int d = lane + 16 * s;
        if (d >= nvr && d < nv) sh.cvec[d] = vp[s];
      }
      wave_sync();
      const f3 wbn = mk(sh.cvec[nvr], sh.cvec[nvr + 1], sh.cvec[nvr + 2]);
      const f3 vbn = mk(sh.cvec[nvr + 3], sh.cvec[nvr + 4], sh.cvec[nvr + 5]);
      wave_sync();  // read before the next step's writes
      pbn[0] = fmaf(dt, vbn.x, pb[0]); pbn[1] = fmaf(dt, vbn.y, pb[1]); pbn[2] = fmaf(dt, vbn.z, pb[2]);
      // world angular velocity: Q <- exp(dt w) Q
      quat_step<false>(Qbn, wbn * dt);  // world-frame rate
      bool ok = true;
#pragma unroll
      for (int i = 0; i < 3; ++i) ok = ok && isfinite(pbn[i]);
#pragma unroll
      for (int i = 0; i < 4; ++i) ok = ok && isfinite(Qbn[i]);
      if (!ok) bad = 1.f;
    }
    const float badsum = row_sum(bad);
    const float clampsum = row_sum(nclamp);
    if (badsum > 0.f) {
      status |= 1u;  // non-finite state: freeze
      break;
    }
#pragma unroll
    for (int s = 0; s < S; ++s) { vS[s] = vp[s]; thS[s] = thN[s]; }
#pragma unroll
    for (int i = 0; i < 3; ++i) p0[i] = p0n[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) Q0[i] = Q0n[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) pb[i] = pbn[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) Qb[i] = Qbn[i];
    kstep += 1;
    cnt_contact += (unsigned long long)nc;
    cnt_clamp += (unsigned long long)clampsum;
  }

  // ---- write back ----
  {
    float* qdst = a.q + (size_t)vid * kQStride;
    float* vdst = a.v + (size_t)vid * kVStride;
    const int qh = (r0 == 6) ? 7 : 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
      const int d = lane + 16 * s;
      if (d < nv) vdst[d] = vS[s];
      if (d >= r0 && d < nvr) qdst[qh + d - r0] = thS[s];
    }
    if (BALL && lane == 0) {
      const int qb = hdr[HW_NQR];
      qdst[qb] = pb[0]; qdst[qb + 1] = pb[1]; qdst[qb + 2] = pb[2];
      qdst[qb + 3] = Qb[0]; qdst[qb + 4] = Qb[1]; qdst[qb + 5] = Qb[2]; qdst[qb + 6] = Qb[3];
    }
    if (lane == 0) {
      if (r0 == 6) {
        qdst[0] = p0[0]; qdst[1] = p0[1]; qdst[2] = p0[2];
        qdst[3] = Q0[0]; qdst[4] = Q0[1]; qdst[5] = Q0[2]; qdst[6] = Q0[3];
      }
      a.k[vid] = kstep;
      a.status[vid] = status;
      const float dx = p0[0] - a.xy0[2 * vid], dy = p0[1] - a.xy0[2 * vid + 1];
      a.fit[vid] = status ? __int_as_float(0x7fc00000) : ((r0 == 6) ? sqrtf(dx * dx + dy * dy) : 0.f);
      a.cnt[2 * vid] = cnt_contact;
      a.cnt[2 * vid + 1] = cnt_clamp;
    }
  }
}

template <int NVC, int SB, int NCR, bool BALL = false, bool SELF = false, bool TREE = false>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(WavesPerSimd<NVC, SB, NCR>::value)))
void rollout_kernel(BinArgs a, ModelParams P) {
  __shared__ GroupLds<NVC, SB, NCR, BALL, SELF, TREE> lds_all[kVarPerWave];
  rollout_body<NVC, SB, NCR, BALL, SELF, TREE>(a, P, blockIdx.x, lds_all);
}

}  // namespace simk
