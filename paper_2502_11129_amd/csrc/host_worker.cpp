// Host-thread worker: one variant per task, single precision, the same step
// as the GPU kernel (spatial forward/backward passes, CRBA, implicit-PD
// diagonal, contact rows, fixed-iteration Gauss-Seidel, semi-implicit Euler).
// The system is factorised here rather than inverted (a serial CPU has no
// reason to form the inverse), by a dense Cholesky or, as an option, by the
// tree-sparse L^T L factorisation that touches only a DoF's ancestors;
// clamp-row columns are solved only when a clamp engages.
// A ball (when the variant has one) adds six DoFs after the robot's (world
// spin, centre velocity), a ball-plane contact and ball-box contacts;
// self-collision adds the corners of a box strictly inside another box of the
// same robot not joined to it by a hinge, and, for a pair with no corner
// inside that intersects across two edges, one edge-edge contact.
#include "host_worker.hpp"

#include <cmath>
#include <algorithm>
#include <cstring>

namespace simk {
namespace {

struct V3 { float x, y, z; };
inline V3 v3(float a, float b, float c) { return {a, b, c}; }
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(V3 a, float s) { return {a.x * s, a.y * s, a.z * s}; }
inline float dotp(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 crs(V3 a, V3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
struct M3 { float m[9]; };
inline V3 mv(const M3& R, V3 v) {
  return {R.m[0] * v.x + R.m[1] * v.y + R.m[2] * v.z, R.m[3] * v.x + R.m[4] * v.y + R.m[5] * v.z,
          R.m[6] * v.x + R.m[7] * v.y + R.m[8] * v.z};
}
inline V3 mtv(const M3& R, V3 v) {
  return {R.m[0] * v.x + R.m[3] * v.y + R.m[6] * v.z, R.m[1] * v.x + R.m[4] * v.y + R.m[7] * v.z,
          R.m[2] * v.x + R.m[5] * v.y + R.m[8] * v.z};
}
inline M3 mm(const M3& A, const M3& B) {
  M3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}
inline M3 qrot(float w, float x, float y, float z) {
  return {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y),
           2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x),
           2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
}
// q <- normalize(q (x) exp(phi)) (right: phi in the body frame) or
// normalize(exp(phi) (x) q) (phi in the world frame), formed as q + dq with
// dq = (cos(a/2) - 1) q + q (x) (0, u) (resp. (0, u) (x) q), u = sin(a/2) phi / a,
// cos(a/2) - 1 = -2 sin^2(a/4), then pulled back to unit norm along q by
// q -= q (|q|^2 - 1) / 2: each component takes the rounding of one small
// increment, not that of a product with cos(a/2) ~ 1 - 2^-24 and with a float
// 1 / |q|, which rounds every component the same way step after step.
inline void quat_step(float* q, V3 phi, bool right) {
  const float an = std::sqrt(dotp(phi, phi));
  float cm1 = 0.f, us = 0.5f;
  if (an >= 1e-8f) {
    const float s4 = std::sin(0.25f * an), c4 = std::cos(0.25f * an);
    cm1 = -2.f * s4 * s4;
    us = 2.f * s4 * c4 / an;
  }
  const float ux = phi.x * us, uy = phi.y * us, uz = phi.z * us;
  const float w = q[0], x = q[1], y = q[2], z = q[3];
  float d[4];
  d[0] = -(x * ux + y * uy + z * uz);
  if (right) {
    d[1] = w * ux + (y * uz - z * uy); d[2] = w * uy + (z * ux - x * uz); d[3] = w * uz + (x * uy - y * ux);
  } else {
    d[1] = w * ux + (uy * z - uz * y); d[2] = w * uy + (uz * x - ux * z); d[3] = w * uz + (ux * y - uy * x);
  }
  float n[4];
  for (int i = 0; i < 4; ++i) n[i] = q[i] + std::fma(cm1, q[i], d[i]);
  const float e = std::fma(n[0], n[0], std::fma(n[1], n[1], std::fma(n[2], n[2], std::fma(n[3], n[3], -1.f))));
  for (int i = 0; i < 4; ++i) q[i] = std::fma(n[i], -0.5f * e, n[i]);
}
inline M3 arot(V3 u, float s, float c) {
  const float C = 1.f - c;
  return {{c + u.x * u.x * C, u.x * u.y * C - u.z * s, u.x * u.z * C + u.y * s,
           u.y * u.x * C + u.z * s, c + u.y * u.y * C, u.y * u.z * C - u.x * s,
           u.z * u.x * C - u.y * s, u.z * u.y * C + u.x * s, c + u.z * u.z * C}};
}
struct SV { V3 a, l; };
inline SV crm(const SV& V, const SV& U) { return {crs(V.a, U.a), crs(V.a, U.l) + crs(V.l, U.a)}; }
inline SV crf(const SV& V, const SV& F) { return {crs(V.a, F.a) + crs(V.l, F.l), crs(V.a, F.l)}; }
struct Inertia { float m; V3 h; float I[6]; };  // about p0: xx yy zz xy xz yz
inline V3 sym(const float* I, V3 w) {
  return {I[0] * w.x + I[3] * w.y + I[4] * w.z, I[3] * w.x + I[1] * w.y + I[5] * w.z,
          I[4] * w.x + I[5] * w.y + I[2] * w.z};
}
inline SV imul(const Inertia& J, const SV& V) { return {sym(J.I, V.a) + crs(J.h, V.l), V.l * J.m - crs(J.h, V.a)}; }

constexpr int NB = kMaxBodies;
constexpr int NV = 28;

struct Work {
  M3 R[NB];
  V3 p[NB], w[NB], o[NB];
  SV V[NB], A[NB], F[NB];
  Inertia C[NB];
  float M[NV * NV], L[NV * NV], c[NV], a[NV], vf[NV], vp[NV];
  int lam[NV];  // parent of each DoF in the DoF tree (-1 at a root), tree factorisation only
  float Wc[NV][NV];
  bool haveWc[NV];
  float Dl[NV];
  // contacts
  int ncap = 0;
  std::vector<float> J, W, scal;  // per contact: 3 * NV each; scalars 10
};

void chol_solve(int n, const float* L, const float* b, float* x) {
  float y[NV];
  for (int i = 0; i < n; ++i) {
    float s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * NV + k] * y[k];
    y[i] = s / L[i * NV + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    float s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * NV + i] * x[k];
    x[i] = s / L[i * NV + i];
  }
}

// Tree-sparse factorisation M = L^T L (Featherstone, "Rigid Body Dynamics
// Algorithms", 2008, Sec. 6.5).  Every DoF's parent lam[k] has a smaller index,
// and M[i][j] = 0 unless one of i, j is an ancestor of the other (branch-induced
// sparsity), so L is lower triangular with L[k][i] != 0 only for i an ancestor
// of k or k itself.  From the last DoF back: L[k][k] = sqrt of what is left of
// M[k][k], the row of k along its ancestors is divided by it, and the outer
// product of that row is taken off the ancestors' block.  Only the ancestor
// entries of M (lower triangle, row stride NV) are read; L is written in the
// same places.  Returns false on a non-positive pivot.
bool tree_factor(int n, const int* lam, const float* M, float* L) {
  for (int k = 0; k < n; ++k) {
    L[k * NV + k] = M[k * NV + k];
    for (int i = lam[k]; i >= 0; i = lam[i]) L[k * NV + i] = M[k * NV + i];
  }
  for (int k = n - 1; k >= 0; --k) {
    const float pivot = L[k * NV + k];
    if (!(pivot > 0.f)) return false;
    const float lkk = std::sqrt(pivot);
    L[k * NV + k] = lkk;
    for (int i = lam[k]; i >= 0; i = lam[i]) L[k * NV + i] /= lkk;
    for (int i = lam[k]; i >= 0; i = lam[i]) {
      const float lki = L[k * NV + i];
      for (int j = i; j >= 0; j = lam[j]) L[i * NV + j] -= lki * L[k * NV + j];
    }
  }
  return true;
}

// x = M^-1 b with M = L^T L from tree_factor: L^T y = b from the leaves
// towards the roots (each DoF, once final, is taken off its ancestors), then
// L x = y from the roots out (each DoF needs only its ancestors).
void tree_solve(int n, const int* lam, const float* L, const float* b, float* x) {
  float y[NV];
  for (int i = 0; i < n; ++i) y[i] = b[i];
  for (int k = n - 1; k >= 0; --k) {
    y[k] /= L[k * NV + k];
    for (int i = lam[k]; i >= 0; i = lam[i]) y[i] -= L[k * NV + i] * y[k];
  }
  for (int k = 0; k < n; ++k) {
    float s = y[k];
    for (int i = lam[k]; i >= 0; i = lam[i]) s -= L[k * NV + i] * x[i];
    x[k] = s / L[k * NV + k];
  }
}

// Orthonormal tangents of a unit normal (Duff et al., JCGT 2017).
void tangent_pair(V3 n, V3& t1, V3& t2) {
  const float sign = std::copysign(1.f, n.z);
  const float a = -1.f / (sign + n.z);
  const float b = n.x * n.y * a;
  t1 = v3(1.f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  t2 = v3(b, sign + n.y * n.y * a, -n.y);
}

// Sphere against box: closest box point (or the nearest face for a centre
// inside), normal from the box to the ball, point c - r n.
bool sphere_box(V3 c, float r, V3 p, const M3& R, V3 h, V3& x, V3& n, float& depth) {
  const V3 l = mtv(R, c - p);
  const bool inside = std::fabs(l.x) <= h.x && std::fabs(l.y) <= h.y && std::fabs(l.z) <= h.z;
  if (!inside) {
    const V3 q = v3(std::fmax(-h.x, std::fmin(h.x, l.x)), std::fmax(-h.y, std::fmin(h.y, l.y)),
                    std::fmax(-h.z, std::fmin(h.z, l.z)));
    const V3 d = c - (p + mv(R, q));
    const float dist = std::sqrt(dotp(d, d));
    if (!(dist < r)) return false;
    n = d * (1.f / dist);
    depth = r - dist;
  } else {
    const float g[3] = {h.x - std::fabs(l.x), h.y - std::fabs(l.y), h.z - std::fabs(l.z)};
    const float lc[3] = {l.x, l.y, l.z};
    int kb = 0;
    for (int k = 1; k < 3; ++k)
      if (g[k] < g[kb]) kb = k;
    const float sgn = lc[kb] >= 0.f ? 1.f : -1.f;
    const V3 nw = mv(R, v3(kb == 0 ? sgn : 0.f, kb == 1 ? sgn : 0.f, kb == 2 ? sgn : 0.f));
    n = nw * (1.f / std::sqrt(dotp(nw, nw)));
    depth = r + g[kb];
  }
  x = c - n * r;
  return true;
}

// A point strictly inside a box.
bool point_in_box(V3 x, V3 p, const M3& R, V3 h) {
  const V3 l = mtv(R, x - p);
  return std::fabs(l.x) < h.x && std::fabs(l.y) < h.y && std::fabs(l.z) < h.z;
}
V3 column(const M3& R, int k) { return v3(R.m[k], R.m[3 + k], R.m[6 + k]); }
float box_radius(const M3& R, V3 h, V3 u) {
  return h.x * std::fabs(dotp(u, column(R, 0))) + h.y * std::fabs(dotp(u, column(R, 1))) +
         h.z * std::fabs(dotp(u, column(R, 2)));
}
// Least-overlap separating axis of boxes P and Q (faces of P, of Q, edge
// crosses with |cross|^2 >= 1e-6), pointing from Q to P.
V3 sat_axis(V3 pP, const M3& RP, V3 hP, V3 pQ, const M3& RQ, V3 hQ) {
  const V3 d = pP - pQ;
  V3 best = v3(0, 0, 1);
  float best_o = INFINITY;
  auto consider = [&](V3 u) {
    const float o = box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - std::fabs(dotp(u, d));
    if (o < best_o) { best_o = o; best = u; }
  };
  for (int k = 0; k < 3; ++k) consider(column(RP, k));
  for (int k = 0; k < 3; ++k) consider(column(RQ, k));
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3 c = crs(column(RP, i), column(RQ, j));
      const float n2 = dotp(c, c);
      if (n2 < 1e-6f) continue;
      consider(c * (1.f / std::sqrt(n2)));
    }
  return dotp(best, d) < 0.f ? best * -1.f : best;
}

// Contact of two intersecting boxes with no corner of either inside the
// other: when the least overlap over the 15 axes of sat_axis is positive and
// belongs to the cross product of P's edge direction i and Q's j, the
// midpoint of the closest points of the two edges facing each other along it
// (P's on the side of Q, Q's on the side of P), normal from Q towards P, depth
// the overlap, when the edge pair beats the least face overlap by the margin
// of edge_beats_face.  False in every other case.
// An edge pair takes the contact from the face axes only when its overlap
// beats the least face overlap by 1e-5 m plus 5 % of it.
bool edge_beats_face(float edge_o, float face_o) { return edge_o < face_o - 1e-5f - 0.05f * face_o; }

bool edge_contact(V3 pP, const M3& RP, V3 hP, V3 pQ, const M3& RQ, V3 hQ, V3& x, V3& n, float& depth) {
  const V3 d = pP - pQ;
  float best_o = INFINITY;
  V3 best = v3(0, 0, 1);
  int bi = -1, bj = -1;
  auto consider = [&](V3 u, int i, int j) {
    const float o = box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - std::fabs(dotp(u, d));
    if (o < best_o) { best_o = o; best = u; bi = i; bj = j; }
  };
  for (int k = 0; k < 3; ++k) consider(column(RP, k), -1, -1);
  for (int k = 0; k < 3; ++k) consider(column(RQ, k), -1, -1);
  const float face_o = best_o;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3 c = crs(column(RP, i), column(RQ, j));
      const float n2 = dotp(c, c);
      if (n2 < 1e-6f) continue;
      consider(c * (1.f / std::sqrt(n2)), i, j);
    }
  if (!(best_o > 0.f) || bi < 0 || !edge_beats_face(best_o, face_o)) return false;
  if (dotp(best, d) < 0.f) best = best * -1.f;
  const float hp[3] = {hP.x, hP.y, hP.z}, hq[3] = {hQ.x, hQ.y, hQ.z};
  V3 cP = pP, cQ = pQ;
  for (int k = 0; k < 3; ++k) {
    if (k != bi) cP = cP + column(RP, k) * (dotp(best, column(RP, k)) > 0.f ? -hp[k] : hp[k]);
    if (k != bj) cQ = cQ + column(RQ, k) * (dotp(best, column(RQ, k)) < 0.f ? -hq[k] : hq[k]);
  }
  const V3 eP = column(RP, bi), eQ = column(RQ, bj), r = cP - cQ;
  const float b = dotp(eP, eQ), c = dotp(eP, r), f = dotp(eQ, r);
  auto clampv = [](float v, float lo, float hi) { return v < lo ? lo : (v > hi ? hi : v); };
  float t = clampv((b * f - c) / (1.f - b * b), -hp[bi], hp[bi]);
  const float s = clampv(f + b * t, -hq[bj], hq[bj]);
  t = clampv(b * s - c, -hp[bi], hp[bi]);
  x = ((cP + eP * t) + (cQ + eQ * s)) * 0.5f;
  n = best;
  depth = best_o;
  return true;
}

// Face contacts of two intersecting boxes with no corner of either inside the
// other when no edge pair beats the least face overlap by the margin: the
// incident face clipped to the reference face, the clipped vertices below it,
// in the fixed candidate order (incident corners inside the rectangle,
// rectangle corners inside the incident face, crossings of the incident
// edges with the rectangle's edge lines); writes up to 24, returns how many;
// the points belong to P when inc = 0, to Q when inc = 1; normal n out of the
// reference face.
int face_contacts(V3 pP, const M3& RP, V3 hP, V3 pQ, const M3& RQ, V3 hQ, V3* xs, float* depths, V3& n,
                  int& inc) {
  const V3 d = pP - pQ;
  float best_o = INFINITY;
  V3 best = v3(0, 0, 1);
  int face = -1;
  auto overlap = [&](V3 u) { return box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - std::fabs(dotp(u, d)); };
  float fo[6];
  for (int f = 0; f < 6; ++f) {
    fo[f] = overlap(column(f < 3 ? RP : RQ, f % 3));
    if (fo[f] < best_o) best_o = fo[f];
  }
  for (int f = 5; f >= 0; --f)  // the first face axis within 1e-5 m of the least
    if (fo[f] <= best_o + 1e-5f) face = f;
  best = column(face < 3 ? RP : RQ, face % 3);
  float edge_o = INFINITY;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3 c = crs(column(RP, i), column(RQ, j));
      const float n2 = dotp(c, c);
      if (n2 < 1e-6f) continue;
      edge_o = std::min(edge_o, overlap(c * (1.f / std::sqrt(n2))));
    }
  if (!(best_o > 0.f) || !(edge_o > 0.f) || edge_beats_face(edge_o, best_o)) return 0;
  if (dotp(best, d) < 0.f) best = best * -1.f;
  const bool refP = face < 3;
  const int k = face % 3;
  const M3& RR = refP ? RP : RQ;
  const M3& RI = refP ? RQ : RP;
  const float hR[3] = {refP ? hP.x : hQ.x, refP ? hP.y : hQ.y, refP ? hP.z : hQ.z};
  const float hI[3] = {refP ? hQ.x : hP.x, refP ? hQ.y : hP.y, refP ? hQ.z : hP.z};
  const V3 pR = refP ? pP : pQ, pI = refP ? pQ : pP;
  n = refP ? best * -1.f : best;
  inc = refP ? 1 : 0;
  const V3 cR = pR + n * hR[k];
  const int r1 = k == 0 ? 1 : 0, r2 = k == 2 ? 1 : 2;
  const V3 ar1 = column(RR, r1), ar2 = column(RR, r2);
  const float e1 = hR[r1], e2 = hR[r2];
  int js = 0;
  float bc = -1.f;
  for (int j = 0; j < 3; ++j) {
    const float c = std::fabs(dotp(column(RI, j), n));
    if (c > bc) { bc = c; js = j; }
  }
  const float sg = dotp(column(RI, js), n) > 0.f ? -1.f : 1.f;
  const V3 cI = pI + column(RI, js) * (sg * hI[js]);
  const int i1 = js == 0 ? 1 : 0, i2 = js == 2 ? 1 : 2;
  const V3 ai1 = column(RI, i1), ai2 = column(RI, i2);
  const float f1 = hI[i1], f2 = hI[i2];
  auto st = [&](V3 x, float& s, float& t) { const V3 r = x - cR; s = dotp(r, ar1); t = dotp(r, ar2); };
  int m = 0;
  auto keep = [&](V3 x) {
    const float dep = dotp(n, cR - x);
    if (dep > 0.f) { xs[m] = x; depths[m] = dep; ++m; }
  };
  V3 cor[4];
  for (int c = 0; c < 4; ++c) cor[c] = cI + (ai1 * ((c & 1) ? f1 : -f1) + ai2 * ((c & 2) ? f2 : -f2));
  for (int c = 0; c < 4; ++c) {
    float s, t;
    st(cor[c], s, t);
    if (std::fabs(s) < e1 && std::fabs(t) < e2) keep(cor[c]);
  }
  {
    const float m11 = dotp(ai1, ar1), m12 = dotp(ai2, ar1), m21 = dotp(ai1, ar2), m22 = dotp(ai2, ar2);
    const float det = m11 * m22 - m12 * m21;
    float s0, t0;
    st(cI, s0, t0);
    for (int c = 0; c < 4; ++c) {
      const float bs = ((c & 1) ? e1 : -e1) - s0, bt = ((c & 2) ? e2 : -e2) - t0;
      const float uu = (bs * m22 - m12 * bt) / det, ww = (m11 * bt - m21 * bs) / det;
      if (std::fabs(uu) < f1 && std::fabs(ww) < f2) keep(cI + (ai1 * uu + ai2 * ww));
    }
  }
  const int ea[4] = {0, 1, 3, 2}, eb[4] = {1, 3, 2, 0};
  for (int e = 0; e < 4; ++e) {
    const V3 A = cor[ea[e]], Bv = cor[eb[e]];
    float sA, tA, sB, tB;
    st(A, sA, tA);
    st(Bv, sB, tB);
    for (int l = 0; l < 4; ++l) {
      const bool sline = l < 2;
      const float cval = l == 0 ? -e1 : (l == 1 ? e1 : (l == 2 ? -e2 : e2));
      const float a0 = sline ? sA : tA, a1 = sline ? sB : tB;
      if (a1 == a0) continue;
      const float lam = (cval - a0) / (a1 - a0);
      if (!(lam > 0.f && lam < 1.f)) continue;
      const float other = sline ? tA + lam * (tB - tA) : sA + lam * (sB - sA);
      if (std::fabs(other) < (sline ? e2 : e1)) keep(A + (Bv - A) * lam);
    }
  }
  return m;
}

bool step(const HostVariantView& m, const ModelParams& P, HostVariantState& st, Work& wk) {
  const int nb = m.hdr[HW_NB], nv = m.hdr[HW_NV], r0 = m.hdr[HW_R0], nh = nb - 1;
  const int nvr = m.hdr[HW_NVR], nqr = m.hdr[HW_NQR];
  const bool ball = nv > nvr;
  const float rball = m.hdrf[HF_BALLR], mball = m.hdrf[HF_BALLM], iball = 0.4f * mball * rball * rball;
  const V3 cb = ball ? v3(st.q[nqr], st.q[nqr + 1], st.q[nqr + 2]) : v3(0, 0, 0);
  const float dt = P.dt, kp = P.kp, kd = P.kd, tmax = P.tau_max, kc = P.k_contact, bcn = P.b_contact;
  const float ba = kd + dt * kp, kb = bcn + kc * dt, mu = m.hdrf[HF_MU];
  const float* rec = m.body;
  auto B = [&](int b, int w) { return rec[b * BW_WORDS + w]; };
  auto Bi = [&](int b, int w) { int x; std::memcpy(&x, &rec[b * BW_WORDS + w], 4); return x; };
  float* q = st.q;
  float* v = st.v;
  const int qh = r0 ? 7 : 0;
  V3 P0;
  M3 R0;
  if (r0) { P0 = v3(q[0], q[1], q[2]); R0 = qrot(q[3], q[4], q[5], q[6]); }
  else {
    P0 = v3(m.hdrf[HF_ROOTP], m.hdrf[HF_ROOTP + 1], m.hdrf[HF_ROOTP + 2]);
    R0 = qrot(m.hdrf[HF_ROOTQ], m.hdrf[HF_ROOTQ + 1], m.hdrf[HF_ROOTQ + 2], m.hdrf[HF_ROOTQ + 3]);
  }
  const V3 wb = r0 ? v3(v[0], v[1], v[2]) : v3(0, 0, 0), vb = r0 ? v3(v[3], v[4], v[5]) : v3(0, 0, 0);
  // forward pass
  for (int b = 0; b < nb; ++b) {
    if (b == 0) {
      wk.R[0] = R0; wk.p[0] = P0; wk.w[0] = v3(0, 0, 0); wk.o[0] = P0;
      wk.V[0] = {mv(R0, wb), mv(R0, vb)};
      wk.A[0] = {v3(0, 0, 0), v3(-P.g[0], -P.g[1], -P.g[2])};
      continue;
    }
    const int l = Bi(b, BW_PARENT);
    const float th = q[qh + b - 1], thd = v[r0 + b - 1];
    const V3 u = v3(B(b, BW_AXIS), B(b, BW_AXIS + 1), B(b, BW_AXIS + 2));
    const M3 E = mm(qrot(B(b, BW_RQ), B(b, BW_RQ + 1), B(b, BW_RQ + 2), B(b, BW_RQ + 3)), arot(u, std::sin(th), std::cos(th)));
    wk.R[b] = mm(wk.R[l], E);
    wk.o[b] = wk.p[l] + mv(wk.R[l], v3(B(b, BW_AP), B(b, BW_AP + 1), B(b, BW_AP + 2)));
    wk.p[b] = wk.o[b] - mv(wk.R[b], v3(B(b, BW_AC), B(b, BW_AC + 1), B(b, BW_AC + 2)));
    wk.w[b] = mv(wk.R[b], u);
    const SV St = {wk.w[b] * thd, crs(wk.o[b] - P0, wk.w[b]) * thd};
    wk.V[b] = {wk.V[l].a + St.a, wk.V[l].l + St.l};
    const SV cc = crm(wk.V[l], St);
    wk.A[b] = {wk.A[l].a + cc.a, wk.A[l].l + cc.l};
  }
  // backward pass: inertia, force, composites (children have larger indices)
  for (int b = 0; b < nb; ++b) {
    const M3& R = wk.R[b];
    const float mm_ = B(b, BW_MASS);
    const V3 h = v3(B(b, BW_HALF), B(b, BW_HALF + 1), B(b, BW_HALF + 2));
    const float ix = mm_ / 3.f * (h.y * h.y + h.z * h.z), iy = mm_ / 3.f * (h.x * h.x + h.z * h.z),
                iz = mm_ / 3.f * (h.x * h.x + h.y * h.y);
    const V3 c = wk.p[b] - P0;
    const float cc = dotp(c, c);
    Inertia J;
    J.m = mm_;
    J.h = c * mm_;
    J.I[0] = R.m[0] * R.m[0] * ix + R.m[1] * R.m[1] * iy + R.m[2] * R.m[2] * iz + mm_ * (cc - c.x * c.x);
    J.I[1] = R.m[3] * R.m[3] * ix + R.m[4] * R.m[4] * iy + R.m[5] * R.m[5] * iz + mm_ * (cc - c.y * c.y);
    J.I[2] = R.m[6] * R.m[6] * ix + R.m[7] * R.m[7] * iy + R.m[8] * R.m[8] * iz + mm_ * (cc - c.z * c.z);
    J.I[3] = R.m[0] * R.m[3] * ix + R.m[1] * R.m[4] * iy + R.m[2] * R.m[5] * iz - mm_ * c.x * c.y;
    J.I[4] = R.m[0] * R.m[6] * ix + R.m[1] * R.m[7] * iy + R.m[2] * R.m[8] * iz - mm_ * c.x * c.z;
    J.I[5] = R.m[3] * R.m[6] * ix + R.m[4] * R.m[7] * iy + R.m[5] * R.m[8] * iz - mm_ * c.y * c.z;
    const SV IV = imul(J, wk.V[b]), IA = imul(J, wk.A[b]);
    const SV x = crf(wk.V[b], IV);
    wk.C[b] = J;
    wk.F[b] = {IA.a + x.a, IA.l + x.l};
  }
  for (int b = nb - 1; b >= 1; --b) {
    const int l = Bi(b, BW_PARENT);
    wk.C[l].m += wk.C[b].m;
    wk.C[l].h = wk.C[l].h + wk.C[b].h;
    for (int i = 0; i < 6; ++i) wk.C[l].I[i] += wk.C[b].I[i];
    wk.F[l].a = wk.F[l].a + wk.F[b].a;
    wk.F[l].l = wk.F[l].l + wk.F[b].l;
  }
  // bias and mass matrix (CRBA)
  std::memset(wk.M, 0, sizeof(wk.M));
  if (r0) {
    const V3 ca = mtv(R0, wk.F[0].a), cl = mtv(R0, wk.F[0].l);
    wk.c[0] = ca.x; wk.c[1] = ca.y; wk.c[2] = ca.z; wk.c[3] = cl.x; wk.c[4] = cl.y; wk.c[5] = cl.z;
    const Inertia& T = wk.C[0];
    const V3 hb = mtv(R0, T.h);
    for (int i = 0; i < 3; ++i) {
      const V3 e = v3(R0.m[i], R0.m[3 + i], R0.m[6 + i]);
      const V3 row = mtv(R0, sym(T.I, e));
      wk.M[i * NV + 0] = row.x; wk.M[i * NV + 1] = row.y; wk.M[i * NV + 2] = row.z;
    }
    const V3 hx[3] = {crs(hb, v3(1, 0, 0)), crs(hb, v3(0, 1, 0)), crs(hb, v3(0, 0, 1))};
    for (int j = 0; j < 3; ++j) {
      const float col[3] = {hx[j].x, hx[j].y, hx[j].z};
      for (int i = 0; i < 3; ++i) {
        wk.M[i * NV + 3 + j] = col[i];   // [h_b]x
        wk.M[(3 + j) * NV + i] = col[i]; // its transpose
      }
      wk.M[(3 + j) * NV + 3 + j] = T.m;
    }
  }
  for (int b = 1; b < nb; ++b) {
    const int d = r0 + b - 1;
    const SV Sb = {wk.w[b], crs(wk.o[b] - P0, wk.w[b])};
    wk.c[d] = dotp(Sb.a, wk.F[b].a) + dotp(Sb.l, wk.F[b].l);
    const SV Fc = imul(wk.C[b], Sb);
    for (int j = b; j >= 1; j = Bi(j, BW_PARENT)) {
      const int dj = r0 + j - 1;
      const SV Sj = {wk.w[j], crs(wk.o[j] - P0, wk.w[j])};
      float val = dotp(Sj.a, Fc.a) + dotp(Sj.l, Fc.l);
      if (j == b) val += dt * ba;
      wk.M[d * NV + dj] = val;
      wk.M[dj * NV + d] = val;
    }
    if (r0) {
      const V3 ra = mtv(R0, Fc.a), rl = mtv(R0, Fc.l);
      const float rv[6] = {ra.x, ra.y, ra.z, rl.x, rl.y, rl.z};
      for (int i = 0; i < 6; ++i) { wk.M[d * NV + i] = rv[i]; wk.M[i * NV + d] = rv[i]; }
    }
  }
  if (ball)  // constant block diag(I, I, I, m, m, m), bias -m g on the centre velocity
    for (int k = 0; k < 6; ++k) {
      wk.M[(nvr + k) * NV + nvr + k] = k < 3 ? iball : mball;
      wk.c[nvr + k] = k < 3 ? 0.f : -mball * P.g[k - 3];
    }
  const bool tree = m.tree_factor != 0;
  if (tree) {
    // DoF tree: the free root's six DoFs in a chain (their block is dense), a
    // hinge under its parent body's hinge (under the root's last DoF for a
    // child of the core), the ball's DoFs on their own (a diagonal block)
    for (int d = 0; d < r0; ++d) wk.lam[d] = d - 1;
    for (int b = 1; b < nb; ++b) {
      const int l = Bi(b, BW_PARENT);
      wk.lam[r0 + b - 1] = l == 0 ? r0 - 1 : r0 + l - 1;
    }
    for (int d = nvr; d < nv; ++d) wk.lam[d] = -1;
    if (!tree_factor(nv, wk.lam, wk.M, wk.L)) return false;
  } else {
    // dense Cholesky M = L L^T
    for (int j = 0; j < nv; ++j) {
      float s = wk.M[j * NV + j];
      for (int k = 0; k < j; ++k) s -= wk.L[j * NV + k] * wk.L[j * NV + k];
      if (!(s > 0.f)) return false;
      wk.L[j * NV + j] = std::sqrt(s);
      for (int i = j + 1; i < nv; ++i) {
        float t = wk.M[i * NV + j];
        for (int k = 0; k < j; ++k) t -= wk.L[i * NV + k] * wk.L[j * NV + k];
        wk.L[i * NV + j] = t / wk.L[j * NV + j];
      }
    }
  }
  auto solve = [&](const float* rhs_, float* x) {
    if (tree) tree_solve(nv, wk.lam, wk.L, rhs_, x);
    else chol_solve(nv, wk.L, rhs_, x);
  };
  // control and free velocity
  const double tk = double(st.k) * double(dt);
  float rhs[NV];
  for (int d = 0; d < nv; ++d) rhs[d] = -dt * wk.c[d];
  for (int j = 0; j < nh; ++j) {
    const int b = j + 1;
    double ph = double(B(b, BW_CPG + 1)) * tk + double(B(b, BW_CPG + 2));
    ph -= 6.283185307179586 * std::floor(ph * 0.15915494309189535);
    const float target = B(b, BW_CPG) * std::sin(float(ph));
    wk.a[j] = kp * (target - q[qh + j]);
    rhs[r0 + j] += dt * (wk.a[j] - ba * v[r0 + j]);
  }
  solve(rhs, wk.vf);
  for (int d = 0; d < nv; ++d) wk.vf[d] += v[d];
  // contacts: rows (n, t1, t2) of the relative velocity; a robot DoF's sign
  // is its body's bit in `plus` minus its bit in `minus` (root DoFs: body 0),
  // the ball's DoFs take `bsign`
  int nc = 0;
  auto add_contact = [&](V3 x, V3 n, float depth, unsigned plus, unsigned minus, float bsign, bool guard = false) {
    if (nc >= wk.ncap) {
      wk.ncap = nc + 16;
      wk.J.resize((size_t)wk.ncap * 3 * NV);
      wk.W.resize((size_t)wk.ncap * 3 * NV);
      wk.scal.resize((size_t)wk.ncap * 10);
    }
    float* J = &wk.J[(size_t)nc * 3 * NV];
    float* W = &wk.W[(size_t)nc * 3 * NV];
    float* sc = &wk.scal[(size_t)nc * 10];
    V3 t1, t2;
    tangent_pair(n, t1, t2);
    auto sign = [&](int b) { return (float)((int)((plus >> b) & 1u) - (int)((minus >> b) & 1u)); };
    for (int d = 0; d < nv; ++d) {
      V3 col;
      if (r0 && d < 3) col = crs(v3(R0.m[d], R0.m[3 + d], R0.m[6 + d]), x - P0) * sign(0);
      else if (r0 && d < 6) col = v3(R0.m[d - 3], R0.m[3 + d - 3], R0.m[6 + d - 3]) * sign(0);
      else if (d < nvr) {
        const int hb = d - r0 + 1;
        col = crs(wk.w[hb], x - wk.o[hb]) * sign(hb);
      } else {
        const int k = d - nvr;
        const V3 e = v3(k % 3 == 0 ? 1.f : 0.f, k % 3 == 1 ? 1.f : 0.f, k % 3 == 2 ? 1.f : 0.f);
        col = (k < 3 ? crs(e, x - cb) : e) * bsign;
      }
      J[d] = dotp(n, col); J[NV + d] = dotp(t1, col); J[2 * NV + d] = dotp(t2, col);
    }
    float D[3];
    for (int r = 0; r < 3; ++r) {
      solve(J + r * NV, W + r * NV);
      float s2 = 0.f;
      for (int d = 0; d < nv; ++d) s2 += J[r * NV + d] * W[r * NV + d];
      D[r] = s2;
    }
    sc[0] = kc * depth;
    sc[1] = 1.f / (D[0] * (1.f + kb * dt));
    sc[2] = dt * D[0];
    sc[3] = 1.f / (dt * D[1]);
    sc[4] = 1.f / (dt * D[2]);
    sc[5] = sc[6] = sc[7] = 0.f;
    if (guard) {  // a self-contact row no DoF can move is inert (zero gain)
      if (!(D[0] >= 1e-9f)) sc[1] = 0.f;
      if (!(D[1] >= 1e-9f)) sc[3] = 0.f;
      if (!(D[2] >= 1e-9f)) sc[4] = 0.f;
    }
    ++nc;
  };
  for (int b = (r0 ? 0 : 1); b < nb; ++b) {
    const V3 h = v3(B(b, BW_HALF), B(b, BW_HALF + 1), B(b, BW_HALF + 2));
    unsigned anc;
    { int x = Bi(b, BW_ANCESTORS); std::memcpy(&anc, &x, 4); }
    for (int cn = 0; cn < 8; ++cn) {
      const V3 s = v3((cn & 1) ? h.x : -h.x, (cn & 2) ? h.y : -h.y, (cn & 4) ? h.z : -h.z);
      const V3 x = wk.p[b] + mv(wk.R[b], s);
      if (!(x.z < 0.f)) continue;
      add_contact(x, v3(0, 0, 1), -x.z, anc, 0u, 0.f);
    }
  }
  if (m.self_collision) {
    // pairs a < b not joined by a hinge: corners of a inside b, then of b inside a
    int nself = 0;
    auto half = [&](int b) { return v3(B(b, BW_HALF), B(b, BW_HALF + 1), B(b, BW_HALF + 2)); };
    for (int a = 0; a < nb; ++a)
      for (int b = a + 1; b < nb; ++b) {
        if (Bi(b, BW_PARENT) == a) continue;
        V3 u{0, 0, 0};
        bool have_u = false;
        for (int side = 0; side < 2; ++side) {
          const int pb = side ? b : a, qb = side ? a : b;
          const V3 hp = half(pb), hq = half(qb);
          unsigned ancp, ancq;
          { int x0 = Bi(pb, BW_ANCESTORS); std::memcpy(&ancp, &x0, 4); }
          { int x0 = Bi(qb, BW_ANCESTORS); std::memcpy(&ancq, &x0, 4); }
          for (int cn = 0; cn < 8; ++cn) {
            const V3 s = v3((cn & 1) ? hp.x : -hp.x, (cn & 2) ? hp.y : -hp.y, (cn & 4) ? hp.z : -hp.z);
            const V3 x = wk.p[pb] + mv(wk.R[pb], s);
            if (!point_in_box(x, wk.p[qb], wk.R[qb], hq)) continue;
            if (!have_u) {  // the pair's normal, from b towards a
              u = sat_axis(wk.p[a], wk.R[a], half(a), wk.p[b], wk.R[b], half(b));
              have_u = true;
            }
            const V3 n = side ? u * -1.f : u;
            const float depth = dotp(n, wk.p[qb]) + box_radius(wk.R[qb], hq, n) - dotp(n, x);
            add_contact(x, n, depth, ancp, ancq, 0.f, true);
            ++nself;
          }
        }
        if (!have_u) {  // no corner inside: two crossing edges, if the boxes intersect there
          V3 x, n;
          float depth;
          unsigned anca, ancb;
          { int x0 = Bi(a, BW_ANCESTORS); std::memcpy(&anca, &x0, 4); }
          { int x0 = Bi(b, BW_ANCESTORS); std::memcpy(&ancb, &x0, 4); }
          if (edge_contact(wk.p[a], wk.R[a], half(a), wk.p[b], wk.R[b], half(b), x, n, depth)) {
            add_contact(x, n, depth, anca, ancb, 0.f, true);
            ++nself;
          } else {  // or an edge or face pushed through a face: the clipped incident face
            V3 xs[24];
            float ds[24];
            int inc = 0;
            const int mc = face_contacts(wk.p[a], wk.R[a], half(a), wk.p[b], wk.R[b], half(b), xs, ds, n, inc);
            for (int i = 0; i < mc; ++i) {
              add_contact(xs[i], n, ds[i], inc ? ancb : anca, inc ? anca : ancb, 0.f, true);
              ++nself;
            }
          }
        }
      }
    if (nself > kMaxSelfContacts) {
      st.status |= 4u;
      return true;  // frozen, state unchanged
    }
  }
  if (ball) {
    if (cb.z - rball < 0.f) {
      const V3 x = v3(cb.x, cb.y, cb.z - rball);
      add_contact(x, v3(0, 0, 1), -x.z, 0u, 0u, 1.f);
    }
    for (int b = 0; b < nb; ++b) {
      V3 x, n;
      float depth;
      if (!sphere_box(cb, rball, wk.p[b], wk.R[b], v3(B(b, BW_HALF), B(b, BW_HALF + 1), B(b, BW_HALF + 2)), x, n, depth))
        continue;
      unsigned anc;
      { int xi = Bi(b, BW_ANCESTORS); std::memcpy(&anc, &xi, 4); }
      add_contact(x, n, depth, 0u, anc, 1.f);
    }
  }
  // fixed-iteration Gauss-Seidel
  for (int d = 0; d < nv; ++d) wk.vp[d] = wk.vf[d];
  for (int j = 0; j < nh; ++j) { wk.Dl[j] = 0.f; wk.haveWc[j] = false; }
  auto clamp_col = [&](int j) -> const float* {
    if (!wk.haveWc[j]) {
      float e[NV] = {0};
      e[r0 + j] = 1.f;
      solve(e, wk.Wc[j]);
      wk.haveWc[j] = true;
    }
    return wk.Wc[j];
  };
  for (int it = 0; it < P.K; ++it) {
    for (int j = 0; j < nh; ++j) {
      // a clamp row with no correction and an unsaturated law is a no-op
      const float u_plain = wk.vp[r0 + j];
      if (wk.Dl[j] == 0.f) {
        const float s0 = wk.a[j] - ba * u_plain;
        if (s0 <= tmax && s0 >= -tmax) continue;
      }
      const float* Wj = clamp_col(j);
      const float Dj = Wj[r0 + j];
      const float u0 = wk.vp[r0 + j] + dt * Dj * wk.Dl[j];
      const float s = wk.a[j] - ba * u0;
      const float den = 1.f - ba * dt * Dj;
      float nd = 0.f;
      if (s > tmax) nd = (s - tmax) / den;
      else if (s < -tmax) nd = (s + tmax) / den;
      const float dl = nd - wk.Dl[j];
      for (int d = 0; d < nv; ++d) wk.vp[d] -= dt * Wj[d] * dl;
      wk.Dl[j] = nd;
    }
    for (int ci = 0; ci < nc; ++ci) {
      const float* J = &wk.J[(size_t)ci * 3 * NV];
      const float* W = &wk.W[(size_t)ci * 3 * NV];
      float* sc = &wk.scal[(size_t)ci * 10];
      float un = 0.f;
      for (int d = 0; d < nv; ++d) un += J[d] * wk.vp[d];
      const float u0 = un - sc[2] * sc[5];
      float ln = (sc[0] - kb * u0) * sc[1];
      if (ln < 0.f) ln = 0.f;
      const float dn = ln - sc[5];
      for (int d = 0; d < nv; ++d) wk.vp[d] += dt * W[d] * dn;
      sc[5] = ln;
      float ux = 0.f, uy = 0.f;
      for (int d = 0; d < nv; ++d) { ux += J[NV + d] * wk.vp[d]; uy += J[2 * NV + d] * wk.vp[d]; }
      float gx = sc[6] - ux * sc[3], gy = sc[7] - uy * sc[4];
      const float gn2 = gx * gx + gy * gy, lim = mu * ln;
      if (gn2 > lim * lim) { const float r = lim / std::sqrt(gn2); gx *= r; gy *= r; }
      const float ex = dt * (gx - sc[6]), ey = dt * (gy - sc[7]);
      for (int d = 0; d < nv; ++d) wk.vp[d] += W[NV + d] * ex + W[2 * NV + d] * ey;
      sc[6] = gx; sc[7] = gy;
    }
  }
  // semi-implicit Euler
  float qn[kQStride];
  std::memcpy(qn, q, sizeof(qn));
  for (int j = 0; j < nh; ++j) qn[qh + j] = q[qh + j] + dt * wk.vp[r0 + j];
  if (r0) {
    const V3 dp = mv(R0, v3(wk.vp[3], wk.vp[4], wk.vp[5]));
    qn[0] = q[0] + dt * dp.x; qn[1] = q[1] + dt * dp.y; qn[2] = q[2] + dt * dp.z;
    quat_step(qn + 3, v3(wk.vp[0], wk.vp[1], wk.vp[2]) * dt, true);  // body-frame rate
  }
  if (ball) {  // world velocities: p += dt v, Q <- exp(dt w) Q
    qn[nqr] = q[nqr] + dt * wk.vp[nvr + 3];
    qn[nqr + 1] = q[nqr + 1] + dt * wk.vp[nvr + 4];
    qn[nqr + 2] = q[nqr + 2] + dt * wk.vp[nvr + 5];
    quat_step(qn + nqr + 3, v3(wk.vp[nvr], wk.vp[nvr + 1], wk.vp[nvr + 2]) * dt, false);  // world-frame rate
  }
  for (int i = 0; i < nqr + (ball ? 7 : 0); ++i)
    if (!std::isfinite(qn[i])) return false;
  for (int d = 0; d < nv; ++d)
    if (!std::isfinite(wk.vp[d])) return false;
  std::memcpy(q, qn, sizeof(qn));
  for (int d = 0; d < nv; ++d) v[d] = wk.vp[d];
  st.k += 1;
  st.rows_contact += (unsigned long long)nc;
  for (int j = 0; j < nh; ++j) st.rows_clamp += (wk.Dl[j] != 0.f);
  return true;
}

}  // namespace

void host_rollout(const HostVariantView& m, const ModelParams& P, int T, HostVariantState& st) {
  std::memcpy(st.q, m.q0, sizeof(st.q));
  std::memcpy(st.v, m.v0, sizeof(st.v));
  st.k = 0;
  st.status = 0;
  st.rows_contact = st.rows_clamp = 0;
  const int r0 = m.hdr[HW_R0];
  st.x0 = r0 ? st.q[0] : 0.f;
  st.y0 = r0 ? st.q[1] : 0.f;
  Work wk;
  for (int t = 0; t < T; ++t) {
    if (!step(m, P, st, wk)) {
      st.status |= 1u;
      break;
    }
    if (st.status) break;
  }
}

float host_fitness(const HostVariantView& m, const HostVariantState& st) {
  if (st.status) return std::nanf("");
  if (!m.hdr[HW_R0]) return 0.f;
  const float dx = st.q[0] - st.x0, dy = st.q[1] - st.y0;
  return std::sqrt(dx * dx + dy * dy);
}

}  // namespace simk
