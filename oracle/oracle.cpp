// FP64 reference simulator -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct CPU implementation of one step of the
// batched box-and-hinge robot simulation: kinematics, the mass matrix as an
// explicit sum over body Jacobians, the bias force from body accelerations at
// zero generalised acceleration, a textbook Cholesky, box-plane contact rows,
// the fixed-iteration projected Gauss-Seidel solve over actuator-clamp and
// contact rows, and semi-implicit Euler.  Only the test-suite, the smoke check
// and the CPU-baseline leg of the benchmark load this library; the product
// path never does.  It shares no code with the HIP library: it parses the
// model arrays itself.
//
// What the paper fixes: the problem statement -- a population of "variants"
// simulated for a number of steps (Sec. 4 "Simulation Parameters", Sec. 5),
// split across CPU and GPU (Sec. 6).  The paper is silent on the physics; the
// equations below are the textbook definitions named in each function.
// Dense mass matrix: kinetic energy T = 1/2 v^T M v with body Jacobians
// (Featherstone, Rigid Body Dynamics Algorithms, 2008, ch. 2 and 6); bias
// force by Kane's method; contact: linearly-implicit soft normal in
// acceleration units, Coulomb disk friction, sequential impulses.
//
// Optional ball (the box-and-ball scene of Sec. 5): a free solid sphere per
// variant, generalised velocity = world angular velocity and world velocity of
// its centre (so its mass matrix block is constant and its bias is gravity
// alone), state appended after the robot's.  Contacts: ball-plane (the
// sphere's lowest point) and ball-box against every box of the robot (closest
// point of the box to the centre; a centre inside a box is pushed out through
// the nearest face), normal from the box to the ball, relative velocity ball
// minus box, friction in the tangent plane of the orthonormal basis of Duff
// et al., "Building an Orthonormal Basis, Revisited", JCGT 6(1), 2017.
//
// Optional self-collision (body-body contact between the boxes of one robot):
// for every pair of boxes not joined by a hinge, each corner of either box
// strictly inside the other is a contact.  The pair shares one normal, the
// separating-axis direction of least overlap (the 3 + 3 face normals and the 9
// edge-pair cross products, near-parallel edge pairs skipped; first of equals),
// oriented away from the penetrated box; a corner's depth is how far it lies
// inside the penetrated box's extent along that normal.  Rows act on the
// relative velocity (corner's box minus penetrated box) at the corner; a row
// no degree of freedom can move (J M^-1 J^T < 1e-9) is inert.  A pair that
// intersects with no corner of either box inside the other, and whose least
// overlap is along an edge-pair cross product (two edges crossing), gets one
// contact instead: the midpoint of the closest points of the two crossing
// edges, normal that axis (towards the first box of the pair), depth the
// overlap along it.  An edge passing through a face with no corner inside
// (least overlap along a face normal) gives no contact.
//
// The library is templated on the scalar so a float instance can measure how
// sensitive a trajectory is to single precision.  An RK4 mode (no contact, no
// solver) integrates the smooth dynamics for the energy/momentum pins.

#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <cstdint>
#include <cstring>
#include <memory>
#include <thread>
#include <vector>

namespace {

template <class T> using V3 = std::array<T, 3>;
template <class T> using M3 = std::array<T, 9>;  // row-major

template <class T> V3<T> add(const V3<T>& a, const V3<T>& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
template <class T> V3<T> sub(const V3<T>& a, const V3<T>& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
template <class T> V3<T> scl(const V3<T>& a, T s) { return {a[0] * s, a[1] * s, a[2] * s}; }
template <class T> T dot(const V3<T>& a, const V3<T>& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
template <class T> V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
template <class T> V3<T> mv(const M3<T>& m, const V3<T>& v) {
  return {m[0] * v[0] + m[1] * v[1] + m[2] * v[2], m[3] * v[0] + m[4] * v[1] + m[5] * v[2],
          m[6] * v[0] + m[7] * v[1] + m[8] * v[2]};
}
template <class T> V3<T> mtv(const M3<T>& m, const V3<T>& v) {  // m^T v
  return {m[0] * v[0] + m[3] * v[1] + m[6] * v[2], m[1] * v[0] + m[4] * v[1] + m[7] * v[2],
          m[2] * v[0] + m[5] * v[1] + m[8] * v[2]};
}
template <class T> M3<T> mm(const M3<T>& a, const M3<T>& b) {
  M3<T> c{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) c[3 * i + j] += a[3 * i + k] * b[3 * k + j];
  return c;
}
template <class T> M3<T> tr(const M3<T>& a) { return {a[0], a[3], a[6], a[1], a[4], a[7], a[2], a[5], a[8]}; }

// Hamilton quaternion (w,x,y,z) -> rotation matrix (world <- body).
template <class T> M3<T> quat_to_rot(const T* q) {
  T w = q[0], x = q[1], y = q[2], z = q[3];
  return {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
          2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
          2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
}
// Rodrigues: rotation by angle th about unit axis u.
template <class T> M3<T> axis_angle(const V3<T>& u, T th) {
  T c = std::cos(th), s = std::sin(th), C = 1 - c;
  return {c + u[0] * u[0] * C, u[0] * u[1] * C - u[2] * s, u[0] * u[2] * C + u[1] * s,
          u[1] * u[0] * C + u[2] * s, c + u[1] * u[1] * C, u[1] * u[2] * C - u[0] * s,
          u[2] * u[0] * C - u[1] * s, u[2] * u[1] * C + u[0] * s, c + u[2] * u[2] * C};
}
template <class T> void quat_mul(const T* a, const T* b, T* out) {
  T r[4] = {a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
            a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
            a[0] * b[2] - a[1] * b[3] + a[2] * b[0] + a[3] * b[1],
            a[0] * b[3] + a[1] * b[2] - a[2] * b[1] + a[3] * b[0]};
  for (int i = 0; i < 4; ++i) out[i] = r[i];
}
template <class T> void quat_normalize(T* q) {
  T n = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
  for (int i = 0; i < 4; ++i) q[i] /= n;
}
// exp map of a rotation vector phi: (cos|phi|/2, sin(|phi|/2) phi/|phi|); (1, phi/2) when tiny.
template <class T> void quat_exp(const V3<T>& phi, T* out) {
  T a = std::sqrt(dot(phi, phi));
  if (a < T(1e-8)) {
    out[0] = 1; out[1] = phi[0] / 2; out[2] = phi[1] / 2; out[3] = phi[2] / 2;
  } else {
    T s = std::sin(a / 2) / a;
    out[0] = std::cos(a / 2); out[1] = phi[0] * s; out[2] = phi[1] * s; out[3] = phi[2] * s;
  }
}

// A point x strictly inside a box (centre p, rotation R, half extents h).
template <class T> bool point_in_box(const V3<T>& x, const V3<T>& p, const M3<T>& R, const V3<T>& h) {
  V3<T> l = mtv(R, sub(x, p));
  for (int k = 0; k < 3; ++k)
    if (!(std::abs(l[k]) < h[k])) return false;
  return true;
}

// Half-width of a box (rotation R, half extents h) along a unit direction u.
template <class T> T box_radius(const M3<T>& R, const V3<T>& h, const V3<T>& u) {
  T r = 0;
  for (int k = 0; k < 3; ++k) r += h[k] * std::abs(u[0] * R[k] + u[1] * R[3 + k] + u[2] * R[6 + k]);
  return r;
}

// Separating-axis direction of least overlap between boxes P and Q: axes
// P's face normals (columns of RP), Q's, then cross products of P's column i
// with Q's column j (i-major), normalised, skipped when |cross|^2 < 1e-6;
// overlap = rP + rQ - |u . (pP - pQ)|; the first smallest wins; the result
// points from Q towards P (+ when u . (pP - pQ) = 0).
template <class T> V3<T> sat_axis(const V3<T>& pP, const M3<T>& RP, const V3<T>& hP, const V3<T>& pQ,
                                  const M3<T>& RQ, const V3<T>& hQ) {
  const V3<T> d = sub(pP, pQ);
  V3<T> best{0, 0, 1};
  T best_o = T(INFINITY);
  auto consider = [&](V3<T> u) {
    T o = box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - std::abs(dot(u, d));
    if (o < best_o) { best_o = o; best = u; }
  };
  for (int k = 0; k < 3; ++k) consider(V3<T>{RP[k], RP[3 + k], RP[6 + k]});
  for (int k = 0; k < 3; ++k) consider(V3<T>{RQ[k], RQ[3 + k], RQ[6 + k]});
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      V3<T> c = cross(V3<T>{RP[i], RP[3 + i], RP[6 + i]}, V3<T>{RQ[j], RQ[3 + j], RQ[6 + j]});
      T n2 = dot(c, c);
      if (n2 < T(1e-6)) continue;
      consider(scl(c, T(1) / std::sqrt(n2)));
    }
  if (dot(best, d) < 0) best = scl(best, T(-1));
  return best;
}

// An edge-pair axis takes the contact from the face axes only when its
// overlap is smaller than the least face overlap by more than 1e-5 m plus 5 %
// of that face overlap (a long edge barely tilted across a face is a face
// case, as in the common fudge-factor rule of box-box clipping).
constexpr double kEdgeMarginAbs = 1e-5, kEdgeMarginRel = 0.05;
template <class T> bool edge_beats_face(T edge_o, T face_o) {
  return edge_o < face_o - T(kEdgeMarginAbs) - T(kEdgeMarginRel) * face_o;
}

// Edge-edge contact of boxes P and Q that intersect although no corner of
// either lies inside the other (two edges crossing).  The 15 candidate axes
// and their overlaps are those of sat_axis; when every candidate overlaps
// (the boxes intersect) and the least overlap belongs to the cross product
// of P's edge direction i and Q's edge direction j, the contact is the
// midpoint of the closest points of the two edges that face each other
// along it: P's edge parallel to its axis i on the side of Q, Q's edge
// parallel to its axis j on the side of P.  Normal u from Q towards P,
// depth = the overlap along u.  The edge pair must beat the least face
// overlap by the margin of edge_beats_face.  Returns false in every other
// case.
template <class T> bool edge_contact(const V3<T>& pP, const M3<T>& RP, const V3<T>& hP, const V3<T>& pQ,
                                     const M3<T>& RQ, const V3<T>& hQ, V3<T>& x, V3<T>& n, T& depth) {
  const V3<T> d = sub(pP, pQ);
  T best_o = T(INFINITY);
  V3<T> best{0, 0, 1};
  int bi = -1, bj = -1;
  auto axis = [](const M3<T>& R, int k) { return V3<T>{R[k], R[3 + k], R[6 + k]}; };
  auto consider = [&](const V3<T>& u, int i, int j) {
    const T o = box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - std::abs(dot(u, d));
    if (o < best_o) { best_o = o; best = u; bi = i; bj = j; }
  };
  for (int k = 0; k < 3; ++k) consider(axis(RP, k), -1, -1);
  for (int k = 0; k < 3; ++k) consider(axis(RQ, k), -1, -1);
  const T face_o = best_o;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3<T> c = cross(axis(RP, i), axis(RQ, j));
      const T n2 = dot(c, c);
      if (n2 < T(1e-6)) continue;
      consider(scl(c, T(1) / std::sqrt(n2)), i, j);
    }
  // an edge pair only when it beats every face axis by the margin (a cross
  // product along a face normal, edges in parallel planes, stays a face case)
  if (!(best_o > 0) || bi < 0 || !edge_beats_face(best_o, face_o)) return false;
  if (dot(best, d) < 0) best = scl(best, T(-1));
  // the edges facing each other: P's towards -u, Q's towards +u
  V3<T> cP = pP, cQ = pQ;
  for (int k = 0; k < 3; ++k) {
    if (k != bi) cP = add(cP, scl(axis(RP, k), (dot(best, axis(RP, k)) > 0 ? -hP[k] : hP[k])));
    if (k != bj) cQ = add(cQ, scl(axis(RQ, k), (dot(best, axis(RQ, k)) < 0 ? -hQ[k] : hQ[k])));
  }
  // closest points of the segments cP + t eP (|t| <= hP[bi]) and cQ + s eQ (|s| <= hQ[bj])
  const V3<T> eP = axis(RP, bi), eQ = axis(RQ, bj), r = sub(cP, cQ);
  const T b = dot(eP, eQ), c = dot(eP, r), f = dot(eQ, r);
  auto clampv = [](T v, T lo, T hi) { return v < lo ? lo : (v > hi ? hi : v); };
  T t = clampv((b * f - c) / (1 - b * b), -hP[bi], hP[bi]);
  const T s = clampv(f + b * t, -hQ[bj], hQ[bj]);
  t = clampv(b * s - c, -hP[bi], hP[bi]);
  x = scl(add(add(cP, scl(eP, t)), add(cQ, scl(eQ, s))), T(0.5));
  n = best;
  depth = best_o;
  return true;
}

// Face contacts of boxes P and Q that intersect although no corner of either
// lies inside the other, when no edge-pair axis beats the least face overlap
// by the margin of edge_beats_face (an edge or a face of one box pushed through a face of the
// other without a corner inside).  The box R owning the first face axis (P's
// axes, then Q's) whose overlap is within 1e-5 m of the least gives the
// reference face: its face on the side of the other box I, outward normal n
// (from R towards I), centre cR, rectangle of R's other two half extents
// along R's other two axes (ascending).  I's incident face is its face whose
// outward normal is most anti-parallel to n (I's axis with the largest
// |a . n|, first of equals).  The contacts are the vertices of the incident
// face clipped to the reference rectangle (coordinates in the reference
// plane) that lie below the reference face, depth = n . (cR - x) > 0, taken
// in this order: incident-face corners strictly inside the rectangle (corner
// bits: sign of I's first, then second in-face axis), rectangle corners
// strictly inside the incident face, carried onto the incident face (same
// bits for R's axes), then crossings strictly inside both edges of each
// incident-face edge (corners 0-1, 1-3, 3-2, 2-0) with the rectangle's edge
// lines s = -e1, s = +e1, t = -e2, t = +e2.  Every point belongs to I and
// takes the normal n.  Returns the number of contacts written (at most 24
// candidates, at most 8 of them for a convex clip); inc = 0 when I is P, 1
// when I is Q.
template <class T> int face_contacts(const V3<T>& pP, const M3<T>& RP, const V3<T>& hP, const V3<T>& pQ,
                                     const M3<T>& RQ, const V3<T>& hQ, V3<T>* xs, T* depths, V3<T>& n, int& inc) {
  const V3<T> d = sub(pP, pQ);
  T best_o = T(INFINITY);
  V3<T> best{0, 0, 1};
  int face = -1;
  auto axis = [](const M3<T>& R, int k) { return V3<T>{R[k], R[3 + k], R[6 + k]}; };
  auto overlap = [&](const V3<T>& u) {
    return box_radius(RP, hP, u) + box_radius(RQ, hQ, u) - std::abs(dot(u, d));
  };
  T fo[6];
  for (int f = 0; f < 6; ++f) {
    fo[f] = overlap(axis(f < 3 ? RP : RQ, f % 3));
    if (fo[f] < best_o) best_o = fo[f];
  }
  // the reference: the first face axis (P's, then Q's) within 1e-5 m of the
  // least face overlap (parallel faces of two boxes tie exactly)
  for (int f = 5; f >= 0; --f)
    if (fo[f] <= best_o + T(1e-5)) face = f;
  best = axis(face < 3 ? RP : RQ, face % 3);
  T edge_o = T(INFINITY);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const V3<T> c = cross(axis(RP, i), axis(RQ, j));
      const T n2 = dot(c, c);
      if (n2 < T(1e-6)) continue;
      edge_o = std::min(edge_o, overlap(scl(c, T(1) / std::sqrt(n2))));
    }
  // the boxes intersect (every axis overlaps) and no edge pair beats the
  // least face overlap by the margin
  if (!(best_o > 0) || !(edge_o > 0) || edge_beats_face(edge_o, best_o)) return 0;
  if (dot(best, d) < 0) best = scl(best, T(-1));  // from Q towards P
  const bool refP = face < 3;
  const int k = face % 3;
  const M3<T>& RR = refP ? RP : RQ;
  const M3<T>& RI = refP ? RQ : RP;
  const V3<T>& hR = refP ? hP : hQ;
  const V3<T>& hI = refP ? hQ : hP;
  const V3<T>& pR = refP ? pP : pQ;
  const V3<T>& pI = refP ? pQ : pP;
  n = refP ? scl(best, T(-1)) : best;
  inc = refP ? 1 : 0;
  const V3<T> cR = add(pR, scl(n, hR[k]));
  const int r1 = k == 0 ? 1 : 0, r2 = k == 2 ? 1 : 2;
  const V3<T> ar1 = axis(RR, r1), ar2 = axis(RR, r2);
  const T e1 = hR[r1], e2 = hR[r2];
  int js = 0;
  T bestc = -1;
  for (int j = 0; j < 3; ++j) {
    const T c = std::abs(dot(axis(RI, j), n));
    if (c > bestc) { bestc = c; js = j; }
  }
  const T sg = dot(axis(RI, js), n) > 0 ? T(-1) : T(1);
  const V3<T> cI = add(pI, scl(axis(RI, js), sg * hI[js]));
  const int i1 = js == 0 ? 1 : 0, i2 = js == 2 ? 1 : 2;
  const V3<T> ai1 = axis(RI, i1), ai2 = axis(RI, i2);
  const T f1 = hI[i1], f2 = hI[i2];
  auto st = [&](const V3<T>& x, T& s, T& t) { const V3<T> r = sub(x, cR); s = dot(r, ar1); t = dot(r, ar2); };
  int m = 0;
  auto keep = [&](const V3<T>& x) {
    const T dep = dot(n, sub(cR, x));
    if (dep > 0) { xs[m] = x; depths[m] = dep; ++m; }
  };
  V3<T> cor[4];
  for (int c = 0; c < 4; ++c)
    cor[c] = add(cI, add(scl(ai1, (c & 1) ? f1 : -f1), scl(ai2, (c & 2) ? f2 : -f2)));
  // incident-face corners inside the rectangle
  for (int c = 0; c < 4; ++c) {
    T s, t;
    st(cor[c], s, t);
    if (std::abs(s) < e1 && std::abs(t) < e2) keep(cor[c]);
  }
  // rectangle corners inside the incident face, on the incident face
  {
    const T m11 = dot(ai1, ar1), m12 = dot(ai2, ar1), m21 = dot(ai1, ar2), m22 = dot(ai2, ar2);
    const T det = m11 * m22 - m12 * m21;
    T s0, t0;
    st(cI, s0, t0);
    for (int c = 0; c < 4; ++c) {
      const T bs = ((c & 1) ? e1 : -e1) - s0, bt = ((c & 2) ? e2 : -e2) - t0;
      const T uu = (bs * m22 - m12 * bt) / det, ww = (m11 * bt - m21 * bs) / det;
      if (std::abs(uu) < f1 && std::abs(ww) < f2) keep(add(cI, add(scl(ai1, uu), scl(ai2, ww))));
    }
  }
  // crossings of the incident-face edges with the rectangle's edge lines
  const int ea[4] = {0, 1, 3, 2}, eb[4] = {1, 3, 2, 0};
  for (int e = 0; e < 4; ++e) {
    const V3<T>& A = cor[ea[e]];
    const V3<T>& B = cor[eb[e]];
    T sA, tA, sB, tB;
    st(A, sA, tA);
    st(B, sB, tB);
    for (int l = 0; l < 4; ++l) {
      const bool sline = l < 2;
      const T cval = (l == 0) ? -e1 : (l == 1) ? e1 : (l == 2) ? -e2 : e2;
      const T a0 = sline ? sA : tA, a1 = sline ? sB : tB;
      if (a1 == a0) continue;
      const T lam = (cval - a0) / (a1 - a0);
      if (!(lam > 0 && lam < 1)) continue;
      const T other = sline ? tA + lam * (tB - tA) : sA + lam * (sB - sA);
      if (std::abs(other) < (sline ? e2 : e1)) keep(add(A, scl(sub(B, A), lam)));
    }
  }
  return m;
}

// ----------------------------------------------------------------------------
// Textbook dense Cholesky (lower, L L^T = A) and the two triangular solves.
// ----------------------------------------------------------------------------
template <class T> bool cholesky(int n, const T* A, T* L) {
  for (int i = 0; i < n * n; ++i) L[i] = 0;
  for (int j = 0; j < n; ++j) {
    T s = A[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0)) return false;
    L[j * n + j] = std::sqrt(s);
    for (int i = j + 1; i < n; ++i) {
      T t = A[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / L[j * n + j];
    }
  }
  return true;
}
template <class T> void chol_solve(int n, const T* L, const T* b, T* x) {
  std::vector<T> y(n);
  for (int i = 0; i < n; ++i) {
    T s = b[i];
    for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
    y[i] = s / L[i * n + i];
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = y[i];
    for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
    x[i] = s / L[i * n + i];
  }
}

// ----------------------------------------------------------------------------
// Model, parsed from the flat variant-CSR arrays.
// ----------------------------------------------------------------------------
struct Params {
  double kp, kd, tau_max, k_contact, b_contact, dt, g[3];
  int K;
  int root_fixed;
  int self_collision = 0;
};

template <class T> struct Body {
  int parent;
  V3<T> half, anchor_parent, anchor_child, axis;
  M3<T> rest;  // parent <- child rest rotation
  T mass;
  V3<T> Ib;    // principal inertia of the box about its centre
  T A, omega, phi;
};

template <class T> struct Variant {
  std::vector<Body<T>> bodies;
  std::vector<std::vector<int>> path;  // ancestors-or-self (hinge bodies only, root excluded)
  T mu;
  int nh, nq, nv, r0;                  // r0 = number of root DoFs (6 or 0); nq, nv include the ball
  int nqr, nvr;                        // robot coordinates only (the ball's follow)
  bool ball = false;
  T ball_r = 0, ball_m = 0, ball_I = 0;  // radius, mass, 2/5 m r^2
  T root_p[3], root_q[4];              // FIXED root pose
  std::vector<T> q0, v0;
};

template <class T> struct State {
  std::vector<T> q, v;
  int64_t k = 0;
  uint32_t status = 0;
  T x0 = 0, y0 = 0;
  uint64_t rows_contact = 0, rows_clamp = 0;
  // closest approach to the ground plane, over the steps taken since the last
  // reset or set_state, of a box corner or of the ball (|height|, metres):
  // bookkeeping for the tests, no part of the dynamics
  double plane_margin = std::numeric_limits<double>::infinity();
};

template <class T> struct Kin {
  std::vector<M3<T>> R;
  std::vector<V3<T>> p, w, o;
  V3<T> p0;
  M3<T> R0;
  V3<T> cb{};  // ball centre
};

// Orthonormal tangents (t1, t2) of a unit normal n (Duff et al. 2017).
template <class T> void tangent_basis(const V3<T>& n, V3<T>& t1, V3<T>& t2) {
  T sign = std::copysign(T(1), n[2]);
  T a = T(-1) / (sign + n[2]);
  T b = n[0] * n[1] * a;
  t1 = {1 + sign * n[0] * n[0] * a, sign * b, -sign * n[0]};
  t2 = {b, sign + n[1] * n[1] * a, -n[1]};
}

// Sphere (centre c, radius r) against a box (centre p, rotation R world <- box,
// half extents h).  With l = R^T (c - p) the centre in the box frame: outside
// the box, the closest box point q = p + R clamp(l, -h, h), contact iff
// |c - q| < r, normal (c - q)/|c - q|, depth r - |c - q|.  Centre inside or on
// the box: the face nearest to the centre (first of equals in x, y, z order),
// its outward normal R (+-e_k) normalised, depth r + distance to it.  Returns
// the normal (box -> ball), the contact point c - r n (the sphere's deepest
// point) and the depth.
template <class T> bool sphere_box(const V3<T>& c, T r, const V3<T>& p, const M3<T>& R, const V3<T>& h,
                                   V3<T>& x, V3<T>& n, T& depth) {
  V3<T> l = mtv(R, sub(c, p));
  bool inside = true;
  for (int k = 0; k < 3; ++k) inside = inside && std::abs(l[k]) <= h[k];
  if (!inside) {
    V3<T> cl;
    for (int k = 0; k < 3; ++k) cl[k] = std::max(-h[k], std::min(h[k], l[k]));
    V3<T> d = sub(c, add(p, mv(R, cl)));
    T dist = std::sqrt(dot(d, d));
    if (!(dist < r)) return false;
    n = scl(d, T(1) / dist);
    depth = r - dist;
  } else {
    int kb = 0;
    T gap = h[0] - std::abs(l[0]);
    for (int k = 1; k < 3; ++k)
      if (h[k] - std::abs(l[k]) < gap) { gap = h[k] - std::abs(l[k]); kb = k; }
    V3<T> nl{0, 0, 0};
    nl[kb] = l[kb] >= 0 ? T(1) : T(-1);
    n = mv(R, nl);
    n = scl(n, T(1) / std::sqrt(dot(n, n)));
    depth = r + gap;
  }
  x = sub(c, scl(n, r));
  return true;
}

template <class T> struct Sim {
  Params P;
  std::vector<Variant<T>> var;
  std::vector<State<T>> st;

  // Forward kinematics (composition of rigid transforms along the tree).
  void fk(const Variant<T>& V, const T* q, Kin<T>& kin) const {
    int nb = (int)V.bodies.size();
    kin.R.resize(nb); kin.p.resize(nb); kin.w.resize(nb); kin.o.resize(nb);
    const T* th;
    if (V.r0 == 6) {
      kin.p0 = {q[0], q[1], q[2]};
      kin.R0 = quat_to_rot(q + 3);
      th = q + 7;
    } else {
      kin.p0 = {V.root_p[0], V.root_p[1], V.root_p[2]};
      kin.R0 = quat_to_rot(V.root_q);
      th = q;
    }
    kin.R[0] = kin.R0; kin.p[0] = kin.p0; kin.w[0] = {0, 0, 0}; kin.o[0] = kin.p0;
    if (V.ball) kin.cb = {q[V.nqr], q[V.nqr + 1], q[V.nqr + 2]};
    for (int i = 1; i < nb; ++i) {
      const Body<T>& B = V.bodies[i];
      int l = B.parent;
      kin.R[i] = mm(mm(kin.R[l], B.rest), axis_angle(B.axis, th[i - 1]));
      kin.o[i] = add(kin.p[l], mv(kin.R[l], B.anchor_parent));
      kin.p[i] = sub(kin.o[i], mv(kin.R[i], B.anchor_child));
      kin.w[i] = mv(kin.R[i], B.axis);
    }
  }

  int dof_of_body(const Variant<T>& V, int b) const { return V.r0 + b - 1; }

  // World Jacobian of the velocity of a point x rigidly attached to body i
  // (3 x nv, row-major): J_p(x) = [-[x-p0]x R0, R0, w_j x (x - o_j) for hinges on path].
  void point_jacobian(const Variant<T>& V, const Kin<T>& kin, int i, const V3<T>& x, T* J) const {
    int nv = V.nv;
    for (int k = 0; k < 3 * nv; ++k) J[k] = 0;
    if (V.r0 == 6) {
      V3<T> r = sub(x, kin.p0);
      for (int c = 0; c < 3; ++c) {
        V3<T> Rc = {kin.R0[c], kin.R0[3 + c], kin.R0[6 + c]};  // column c of R0
        V3<T> a = cross(Rc, r);                                 // angular column: Rc x r
        for (int rr = 0; rr < 3; ++rr) {
          J[rr * nv + c] = a[rr];
          J[rr * nv + 3 + c] = Rc[rr];
        }
      }
    }
    for (int j : V.path[i]) {
      V3<T> c = cross(kin.w[j], sub(x, kin.o[j]));
      int d = dof_of_body(V, j);
      for (int rr = 0; rr < 3; ++rr) J[rr * nv + d] = c[rr];
    }
  }
  // World Jacobian of the velocity of a point x moving with the ball (3 x nv):
  // columns of the ball's angular velocity e_k x (x - cb), of its centre velocity e_k.
  void ball_point_jacobian(const Variant<T>& V, const Kin<T>& kin, const V3<T>& x, T* J) const {
    int nv = V.nv;
    for (int k = 0; k < 3 * nv; ++k) J[k] = 0;
    V3<T> r = sub(x, kin.cb);
    for (int k = 0; k < 3; ++k) {
      V3<T> e{0, 0, 0};
      e[k] = 1;
      V3<T> a = cross(e, r);
      for (int rr = 0; rr < 3; ++rr) {
        J[rr * nv + V.nvr + k] = a[rr];
        J[rr * nv + V.nvr + 3 + k] = e[rr];
      }
    }
  }
  void ball_angular_jacobian(const Variant<T>& V, T* J) const {
    int nv = V.nv;
    for (int k = 0; k < 3 * nv; ++k) J[k] = 0;
    for (int k = 0; k < 3; ++k) J[k * nv + V.nvr + k] = 1;
  }
  // Angular-velocity Jacobian of body i (3 x nv): [R0, 0, w_j on path].
  void angular_jacobian(const Variant<T>& V, const Kin<T>& kin, int i, T* J) const {
    int nv = V.nv;
    for (int k = 0; k < 3 * nv; ++k) J[k] = 0;
    if (V.r0 == 6)
      for (int rr = 0; rr < 3; ++rr)
        for (int c = 0; c < 3; ++c) J[rr * nv + c] = kin.R0[3 * rr + c];
    for (int j : V.path[i]) {
      int d = dof_of_body(V, j);
      for (int rr = 0; rr < 3; ++rr) J[rr * nv + d] = kin.w[j][rr];
    }
  }
  M3<T> world_inertia(const Body<T>& B, const M3<T>& R) const {
    M3<T> D{B.Ib[0], 0, 0, 0, B.Ib[1], 0, 0, 0, B.Ib[2]};
    return mm(mm(R, D), tr(R));
  }

  // Mass matrix by definition: M = sum_i m_i Jv_i^T Jv_i + Jw_i^T I_i Jw_i.
  void mass_matrix(const Variant<T>& V, const Kin<T>& kin, T* M) const {
    int nv = V.nv, nb = (int)V.bodies.size();
    std::vector<T> Jv(3 * nv), Jw(3 * nv);
    for (int k = 0; k < nv * nv; ++k) M[k] = 0;
    for (int i = 0; i < nb; ++i) {
      const Body<T>& B = V.bodies[i];
      point_jacobian(V, kin, i, kin.p[i], Jv.data());
      angular_jacobian(V, kin, i, Jw.data());
      M3<T> I = world_inertia(B, kin.R[i]);
      for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
          T s = 0;
          for (int r = 0; r < 3; ++r) s += B.mass * Jv[r * nv + a] * Jv[r * nv + b];
          V3<T> Ja = {Jw[a], Jw[nv + a], Jw[2 * nv + a]}, Jb = {Jw[b], Jw[nv + b], Jw[2 * nv + b]};
          s += dot(Ja, mv(I, Jb));
          M[a * nv + b] += s;
        }
    }
    if (V.ball) {  // the ball as one more body, isotropic inertia
      ball_point_jacobian(V, kin, kin.cb, Jv.data());
      ball_angular_jacobian(V, Jw.data());
      for (int a = 0; a < nv; ++a)
        for (int b = 0; b < nv; ++b) {
          T s = 0;
          for (int r = 0; r < 3; ++r) s += V.ball_m * Jv[r * nv + a] * Jv[r * nv + b] + V.ball_I * Jw[r * nv + a] * Jw[r * nv + b];
          M[a * nv + b] += s;
        }
    }
  }

  // Bias force by Kane's method: c = sum_i Jv_i^T m_i (abar_i - g) + Jw_i^T (I_i alphabar_i + w_i x I_i w_i),
  // with abar, alphabar the body accelerations at zero generalised acceleration.
  void bias(const Variant<T>& V, const Kin<T>& kin, const T* v, const T* g, T* c) const {
    int nv = V.nv, nb = (int)V.bodies.size();
    std::vector<V3<T>> om(nb), al(nb), pd(nb), ac(nb);
    if (V.r0 == 6) {
      om[0] = mv(kin.R0, V3<T>{v[0], v[1], v[2]});
      pd[0] = mv(kin.R0, V3<T>{v[3], v[4], v[5]});
      al[0] = {0, 0, 0};
      ac[0] = cross(om[0], pd[0]);
    } else {
      om[0] = pd[0] = al[0] = ac[0] = {0, 0, 0};
    }
    for (int i = 1; i < nb; ++i) {
      int l = V.bodies[i].parent;
      T thd = v[dof_of_body(V, i)];
      V3<T> wt = scl(kin.w[i], thd);
      om[i] = add(om[l], wt);
      al[i] = add(al[l], cross(om[l], wt));
      V3<T> r1 = sub(kin.o[i], kin.p[l]), r2 = sub(kin.p[i], kin.o[i]);
      ac[i] = add(add(add(ac[l], cross(al[l], r1)), cross(om[l], cross(om[l], r1))),
                  add(cross(al[i], r2), cross(om[i], cross(om[i], r2))));
      pd[i] = add(add(pd[l], cross(om[l], r1)), cross(om[i], r2));
    }
    std::vector<T> Jv(3 * nv), Jw(3 * nv);
    for (int k = 0; k < nv; ++k) c[k] = 0;
    V3<T> gv = {g[0], g[1], g[2]};
    for (int i = 0; i < nb; ++i) {
      const Body<T>& B = V.bodies[i];
      point_jacobian(V, kin, i, kin.p[i], Jv.data());
      angular_jacobian(V, kin, i, Jw.data());
      M3<T> I = world_inertia(B, kin.R[i]);
      V3<T> f = scl(sub(ac[i], gv), B.mass);
      V3<T> n = add(mv(I, al[i]), cross(om[i], mv(I, om[i])));
      for (int k = 0; k < nv; ++k)
        for (int r = 0; r < 3; ++r) c[k] += Jv[r * nv + k] * f[r] + Jw[r * nv + k] * n[r];
    }
    if (V.ball) {
      // centre acceleration and angular acceleration are the generalised
      // accelerations themselves: zero at zero generalised acceleration
      ball_point_jacobian(V, kin, kin.cb, Jv.data());
      ball_angular_jacobian(V, Jw.data());
      V3<T> om_b = {v[V.nvr], v[V.nvr + 1], v[V.nvr + 2]};
      V3<T> f = scl(sub(V3<T>{0, 0, 0}, gv), V.ball_m);
      V3<T> n = cross(om_b, scl(om_b, V.ball_I));
      for (int k = 0; k < nv; ++k)
        for (int r = 0; r < 3; ++r) c[k] += Jv[r * nv + k] * f[r] + Jw[r * nv + k] * n[r];
    }
  }

  // kind 0: box corner - plane (body, corner); 1: ball - plane; 2: ball - box (body);
  // 3: corner `corner` of box `body` inside box `other` (self-collision)
  struct Contact {
    int body, corner, kind = 0, other = -1;
    V3<T> x, n{0, 0, 1};
    T depth;
    std::vector<T> J[3], W[3];  // rows: 0 = normal (z), 1 = x, 2 = y
    T D[3];
    T lam[3];
  };

  // Rows of a contact in the slots (t1, t2, n) = (x, y, z) of a 3 x nv matrix:
  // plane contacts take world x, y, z; ball-box and box-box contacts project
  // the relative velocity Jacobian (ball or corner's box minus the other box
  // at the contact point) on (t1, t2, n).
  void contact_jacobian(const Variant<T>& V, const Kin<T>& kin, const Contact& ct, T* Jp) const {
    const int nv = V.nv;
    if (ct.kind == 0) {
      point_jacobian(V, kin, ct.body, ct.x, Jp);
    } else if (ct.kind == 1) {
      ball_point_jacobian(V, kin, ct.x, Jp);
    } else {
      std::vector<T> Ja(3 * nv), Jb(3 * nv);
      if (ct.kind == 2) {
        ball_point_jacobian(V, kin, ct.x, Ja.data());
        point_jacobian(V, kin, ct.body, ct.x, Jb.data());
      } else {
        point_jacobian(V, kin, ct.body, ct.x, Ja.data());
        point_jacobian(V, kin, ct.other, ct.x, Jb.data());
      }
      V3<T> t1, t2;
      tangent_basis(ct.n, t1, t2);
      const V3<T> dirs[3] = {t1, t2, ct.n};
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < nv; ++k) {
          T s = 0;
          for (int c = 0; c < 3; ++c) s += dirs[r][c] * (Ja[c * nv + k] - Jb[c * nv + k]);
          Jp[r * nv + k] = s;
        }
    }
  }

  // Active corners in (body, corner) order: corner c has sign bits (x,y,z) = bits 0,1,2.
  void detect(const Variant<T>& V, const Kin<T>& kin, std::vector<Contact>& out) const {
    out.clear();
    int nb = (int)V.bodies.size();
    for (int i = (V.r0 == 6 ? 0 : 1); i < nb; ++i) {
      const Body<T>& B = V.bodies[i];
      for (int c = 0; c < 8; ++c) {
        V3<T> s = {(c & 1) ? B.half[0] : -B.half[0], (c & 2) ? B.half[1] : -B.half[1],
                   (c & 4) ? B.half[2] : -B.half[2]};
        V3<T> x = add(kin.p[i], mv(kin.R[i], s));
        if (x[2] < 0) {
          Contact C;
          C.body = i; C.corner = c; C.x = x; C.depth = -x[2];
          out.push_back(std::move(C));
        }
      }
    }
    if (P.self_collision) {
      // pairs a < b not joined by a hinge; corners of a inside b, then of b inside a
      for (int a = 0; a < nb; ++a)
        for (int b = a + 1; b < nb; ++b) {
          if (V.bodies[b].parent == a) continue;
          const std::size_t first = out.size();
          for (int side = 0; side < 2; ++side) {
            const int pb = side ? b : a, qb = side ? a : b;
            const Body<T>& BP = V.bodies[pb];
            for (int c = 0; c < 8; ++c) {
              V3<T> sc = {(c & 1) ? BP.half[0] : -BP.half[0], (c & 2) ? BP.half[1] : -BP.half[1],
                          (c & 4) ? BP.half[2] : -BP.half[2]};
              V3<T> x = add(kin.p[pb], mv(kin.R[pb], sc));
              if (point_in_box(x, kin.p[qb], kin.R[qb], V.bodies[qb].half)) {
                Contact C;
                C.body = pb; C.other = qb; C.corner = c; C.kind = 3;
                C.x = x;
                out.push_back(std::move(C));
              }
            }
          }
          if (out.size() == first) {
            // no corner inside: two crossing edges, if the boxes intersect there
            Contact C;
            if (edge_contact(kin.p[a], kin.R[a], V.bodies[a].half, kin.p[b], kin.R[b], V.bodies[b].half, C.x, C.n,
                             C.depth)) {
              C.body = a; C.other = b; C.corner = -3; C.kind = 3;
              out.push_back(std::move(C));
              continue;
            }
            // or an edge or face pushed through a face: the clipped incident face
            V3<T> xs[24];
            T ds[24];
            V3<T> fn;
            int inc = 0;
            const int m = face_contacts(kin.p[a], kin.R[a], V.bodies[a].half, kin.p[b], kin.R[b], V.bodies[b].half,
                                        xs, ds, fn, inc);
            for (int i = 0; i < m; ++i) {
              Contact F;
              F.body = inc ? b : a; F.other = inc ? a : b; F.corner = -4; F.kind = 3;
              F.x = xs[i]; F.n = fn; F.depth = ds[i];
              out.push_back(std::move(F));
            }
            continue;
          }
          // the pair's normal (from b towards a) and each corner's depth along it
          const V3<T> u = sat_axis(kin.p[a], kin.R[a], V.bodies[a].half, kin.p[b], kin.R[b], V.bodies[b].half);
          for (std::size_t k = first; k < out.size(); ++k) {
            Contact& C = out[k];
            C.n = C.body == a ? u : scl(u, T(-1));
            const int q = C.other;
            const T support = dot(C.n, kin.p[q]) + box_radius(kin.R[q], V.bodies[q].half, C.n);
            C.depth = support - dot(C.n, C.x);
          }
        }
    }
    if (!V.ball) return;
    // the ball after the boxes: plane first, then every box in body order
    if (kin.cb[2] - V.ball_r < 0) {
      Contact C;
      C.body = -1; C.corner = -1; C.kind = 1;
      C.x = {kin.cb[0], kin.cb[1], kin.cb[2] - V.ball_r};
      C.depth = -C.x[2];
      out.push_back(std::move(C));
    }
    for (int i = 0; i < nb; ++i) {
      Contact C;
      if (sphere_box(kin.cb, V.ball_r, kin.p[i], kin.R[i], V.bodies[i].half, C.x, C.n, C.depth)) {
        C.body = i; C.corner = -2; C.kind = 2;
        out.push_back(std::move(C));
      }
    }
  }

  // One step k -> k+1 of variant vi.
  void step(int vi) {
    const Variant<T>& V = var[vi];
    State<T>& S = st[vi];
    if (S.status) return;
    const Params& P = this->P;
    const int nv = V.nv, nh = V.nh, r0 = V.r0;
    const T dt = T(P.dt), kp = T(P.kp), kd = T(P.kd), tmax = T(P.tau_max);
    const T kc = T(P.k_contact), bc = T(P.b_contact);
    const T g[3] = {T(P.g[0]), T(P.g[1]), T(P.g[2])};
    const T* q = S.q.data();
    const T* v = S.v.data();
    const T* th = q + (r0 == 6 ? 7 : 0);

    // 1. kinematics
    Kin<T> kin;
    fk(V, q, kin);
    // 2-3. mass matrix and bias force
    std::vector<T> M(nv * nv), c(nv), L(nv * nv);
    mass_matrix(V, kin, M.data());
    bias(V, kin, v, g, c.data());
    // 4. linearly-implicit PD: Mt = M + dt*b_a*S, b_a = kd + dt*kp
    const T ba = kd + dt * kp;
    for (int j = 0; j < nh; ++j) M[(r0 + j) * nv + (r0 + j)] += dt * ba;
    if (!cholesky(nv, M.data(), L.data())) { S.status |= 2u; return; }
    // control: theta*_j = A sin(omega t + phi), a_j = kp (theta* - theta)
    const double t = double(S.k) * P.dt;
    std::vector<T> a(nh), rhs(nv), vf(nv);
    for (int j = 0; j < nh; ++j) {
      const Body<T>& B = V.bodies[j + 1];
      T target = B.A * T(std::sin(double(B.omega) * t + double(B.phi)));
      a[j] = kp * (target - th[j]);
    }
    for (int k = 0; k < nv; ++k) rhs[k] = -dt * c[k];
    for (int j = 0; j < nh; ++j) rhs[r0 + j] += dt * (a[j] - ba * v[r0 + j]);
    chol_solve(nv, L.data(), rhs.data(), vf.data());
    for (int k = 0; k < nv; ++k) vf[k] += v[k];

    // 5. contacts and their rows
    std::vector<Contact> C;
    detect(V, kin, C);
    for (int i = (r0 == 6 ? 0 : 1); i < (int)V.bodies.size(); ++i)
      for (int cn = 0; cn < 8; ++cn) {
        const V3<T> sc = {(cn & 1) ? V.bodies[i].half[0] : -V.bodies[i].half[0],
                          (cn & 2) ? V.bodies[i].half[1] : -V.bodies[i].half[1],
                          (cn & 4) ? V.bodies[i].half[2] : -V.bodies[i].half[2]};
        S.plane_margin = std::min(S.plane_margin, std::abs(double(add(kin.p[i], mv(kin.R[i], sc))[2])));
      }
    if (V.ball) S.plane_margin = std::min(S.plane_margin, std::abs(double(kin.cb[2] - V.ball_r)));
    int nself = 0;
    for (const auto& ct : C) nself += ct.kind == 3;
    if (nself > 256) { S.status |= 4u; return; }  // more self-collision contacts than allowed: frozen
    std::vector<T> Jp(3 * nv);
    const int rowsel[3] = {2, 0, 1};  // normal = world z, then world x, y
    for (auto& ct : C) {
      contact_jacobian(V, kin, ct, Jp.data());
      for (int r = 0; r < 3; ++r) {
        ct.J[r].assign(Jp.begin() + rowsel[r] * nv, Jp.begin() + (rowsel[r] + 1) * nv);
        ct.W[r].resize(nv);
        chol_solve(nv, L.data(), ct.J[r].data(), ct.W[r].data());
        T d = 0;
        for (int k = 0; k < nv; ++k) d += ct.J[r][k] * ct.W[r][k];
        ct.D[r] = d;
        ct.lam[r] = 0;
      }
    }
    // clamp rows: W_j = Mt^{-1} e_j, D_j = (Mt^{-1})_jj
    std::vector<std::vector<T>> Wc(nh, std::vector<T>(nv));
    std::vector<T> Dc(nh), Delta(nh, T(0));
    std::vector<T> e(nv);
    for (int j = 0; j < nh; ++j) {
      std::fill(e.begin(), e.end(), T(0));
      e[r0 + j] = 1;
      chol_solve(nv, L.data(), e.data(), Wc[j].data());
      Dc[j] = Wc[j][r0 + j];
    }

    // 6-7. fixed-iteration projected Gauss-Seidel, cold start
    std::vector<T> vp = vf;
    auto dotv = [&](const std::vector<T>& x) { T s = 0; for (int k = 0; k < nv; ++k) s += x[k] * vp[k]; return s; };
    const T kb = bc + kc * dt;
    for (int it = 0; it < P.K; ++it) {
      for (int j = 0; j < nh; ++j) {  // (i) actuator clamp rows
        T u0 = vp[r0 + j] + dt * Dc[j] * Delta[j];
        T s = a[j] - ba * u0;
        T den = 1 - ba * dt * Dc[j];
        T nd = 0;
        if (s > tmax) nd = (s - tmax) / den;
        else if (s < -tmax) nd = (s + tmax) / den;
        T dl = nd - Delta[j];
        for (int k = 0; k < nv; ++k) vp[k] -= dt * Wc[j][k] * dl;
        Delta[j] = nd;
      }
      for (auto& ct : C) {             // (ii) contacts
        if (ct.kind == 3 && !(ct.D[0] >= T(1e-9))) continue;  // a self-contact row nothing can move
        T u = dotv(ct.J[0]);
        T u0 = u - dt * ct.D[0] * ct.lam[0];
        T ln = (kc * ct.depth - kb * u0) / (ct.D[0] * (1 + kb * dt));
        if (ln < 0) ln = 0;
        for (int k = 0; k < nv; ++k) vp[k] += dt * ct.W[0][k] * (ln - ct.lam[0]);
        ct.lam[0] = ln;
        T ux = dotv(ct.J[1]), uy = dotv(ct.J[2]);
        T gx = ct.lam[1] - ux / (dt * ct.D[1]);
        T gy = ct.lam[2] - uy / (dt * ct.D[2]);
        if (ct.kind == 3) {  // self-contact friction rows nothing can move stay inert
          if (!(ct.D[1] >= T(1e-9))) gx = 0;
          if (!(ct.D[2] >= T(1e-9))) gy = 0;
        }
        T gn = std::sqrt(gx * gx + gy * gy), lim = V.mu * ln;
        if (gn > lim) { gx *= lim / gn; gy *= lim / gn; }
        for (int k = 0; k < nv; ++k) vp[k] += dt * (ct.W[1][k] * (gx - ct.lam[1]) + ct.W[2][k] * (gy - ct.lam[2]));
        ct.lam[1] = gx; ct.lam[2] = gy;
      }
    }
    uint64_t nclamp = 0;
    for (int j = 0; j < nh; ++j) nclamp += (Delta[j] != 0);

    // 8. semi-implicit Euler
    std::vector<T> qn(S.q), vn(vp);
    T* thn = qn.data() + (r0 == 6 ? 7 : 0);
    for (int j = 0; j < nh; ++j) thn[j] = th[j] + dt * vp[r0 + j];
    if (r0 == 6) {
      V3<T> dp = mv(kin.R0, V3<T>{vp[3], vp[4], vp[5]});
      for (int k = 0; k < 3; ++k) qn[k] = q[k] + dt * dp[k];
      T dq[4];
      quat_exp(V3<T>{dt * vp[0], dt * vp[1], dt * vp[2]}, dq);
      quat_mul(q + 3, dq, qn.data() + 3);
      quat_normalize(qn.data() + 3);
    }
    if (V.ball) {  // world-frame velocities: p += dt v, Q <- exp(dt w) Q
      const int qb = V.nqr, vb = V.nvr;
      for (int k = 0; k < 3; ++k) qn[qb + k] = q[qb + k] + dt * vp[vb + 3 + k];
      T dq[4];
      quat_exp(V3<T>{dt * vp[vb], dt * vp[vb + 1], dt * vp[vb + 2]}, dq);
      quat_mul(dq, q + qb + 3, qn.data() + qb + 3);
      quat_normalize(qn.data() + qb + 3);
    }
    // 9. failure check: a non-finite state freezes the variant
    bool ok = true;
    for (T x : qn) ok = ok && std::isfinite(double(x));
    for (T x : vn) ok = ok && std::isfinite(double(x));
    if (!ok) { S.status |= 1u; return; }
    S.q.swap(qn); S.v.swap(vn);
    S.k += 1;
    S.rows_contact += C.size();
    S.rows_clamp += nclamp;
  }

  // ---- smooth dynamics for the RK4 mode (no contact; explicit clamped PD or zero torque) ----
  // Extended off the unit sphere so RK4 stays 4th order: the rotation is read from Q/|Q|.
  void accel(const Variant<T>& V, const T* qin, const T* v, double t, bool pd, T* vdot) const {
    int nv = V.nv, nh = V.nh, r0 = V.r0;
    std::vector<T> qv(qin, qin + V.nq);
    if (r0 == 6) quat_normalize(qv.data() + 3);
    const T* q = qv.data();
    Kin<T> kin;
    fk(V, q, kin);
    std::vector<T> M(nv * nv), c(nv), L(nv * nv), f(nv);
    T g[3] = {T(P.g[0]), T(P.g[1]), T(P.g[2])};
    mass_matrix(V, kin, M.data());
    bias(V, kin, v, g, c.data());
    for (int k = 0; k < nv; ++k) f[k] = -c[k];
    if (pd) {
      const T* th = q + (r0 == 6 ? 7 : 0);
      for (int j = 0; j < nh; ++j) {
        const Body<T>& B = V.bodies[j + 1];
        T target = B.A * T(std::sin(double(B.omega) * t + double(B.phi)));
        T tau = T(P.kp) * (target - th[j]) - T(P.kd) * v[r0 + j];
        tau = std::max(-T(P.tau_max), std::min(T(P.tau_max), tau));
        f[r0 + j] += tau;
      }
    }
    cholesky(nv, M.data(), L.data());
    chol_solve(nv, L.data(), f.data(), vdot);
  }
  // time derivative of q given v: pdot = R0 v_b, Qdot = 1/2 Q (0, w_b), thetadot
  void qdot(const Variant<T>& V, const T* q, const T* v, T* out) const {
    int nh = V.nh;
    if (V.r0 == 6) {
      T qn[4] = {q[3], q[4], q[5], q[6]};
      quat_normalize(qn);
      M3<T> R0 = quat_to_rot(qn);
      V3<T> dp = mv(R0, V3<T>{v[3], v[4], v[5]});
      for (int k = 0; k < 3; ++k) out[k] = dp[k];
      T w[4] = {0, v[0], v[1], v[2]}, qd[4];
      quat_mul(q + 3, w, qd);
      for (int k = 0; k < 4; ++k) out[3 + k] = qd[k] / 2;
      for (int j = 0; j < nh; ++j) out[7 + j] = v[6 + j];
    } else {
      for (int j = 0; j < nh; ++j) out[j] = v[j];
    }
    if (V.ball) {  // pdot = v, Qdot = 1/2 (0, w) Q
      const int qb = V.nqr, vb = V.nvr;
      for (int k = 0; k < 3; ++k) out[qb + k] = v[vb + 3 + k];
      T w[4] = {0, v[vb], v[vb + 1], v[vb + 2]}, qd[4];
      quat_mul(w, q + qb + 3, qd);
      for (int k = 0; k < 4; ++k) out[qb + 3 + k] = qd[k] / 2;
    }
  }
  void rk4_step(int vi, bool pd) {
    const Variant<T>& V = var[vi];
    State<T>& S = st[vi];
    int nq = V.nq, nv = V.nv;
    double h = P.dt, t = double(S.k) * h;
    std::vector<T> q0 = S.q, v0 = S.v, kq[4], kv[4], qt(nq), vt(nv);
    for (int s = 0; s < 4; ++s) { kq[s].resize(nq); kv[s].resize(nv); }
    const double cs[4] = {0, 0.5, 0.5, 1};
    for (int s = 0; s < 4; ++s) {
      for (int k = 0; k < nq; ++k) qt[k] = q0[k] + (s ? T(cs[s] * h) * kq[s - 1][k] : T(0));
      for (int k = 0; k < nv; ++k) vt[k] = v0[k] + (s ? T(cs[s] * h) * kv[s - 1][k] : T(0));
      qdot(V, qt.data(), vt.data(), kq[s].data());
      accel(V, qt.data(), vt.data(), t + cs[s] * h, pd, kv[s].data());
    }
    for (int k = 0; k < nq; ++k) S.q[k] = q0[k] + T(h / 6) * (kq[0][k] + 2 * kq[1][k] + 2 * kq[2][k] + kq[3][k]);
    for (int k = 0; k < nv; ++k) S.v[k] = v0[k] + T(h / 6) * (kv[0][k] + 2 * kv[1][k] + 2 * kv[2][k] + kv[3][k]);
    if (V.r0 == 6) quat_normalize(S.q.data() + 3);
    if (V.ball) quat_normalize(S.q.data() + V.nqr + 3);
    S.k += 1;
  }

  // Energy (kinetic + gravitational) and linear / angular momentum about the world origin.
  void invariants(int vi, T* out) const {
    const Variant<T>& V = var[vi];
    const State<T>& S = st[vi];
    int nv = V.nv, nb = (int)V.bodies.size();
    Kin<T> kin;
    fk(V, S.q.data(), kin);
    std::vector<T> Jv(3 * nv), Jw(3 * nv);
    T E = 0;
    V3<T> Pm{0, 0, 0}, Lm{0, 0, 0}, gv = {T(P.g[0]), T(P.g[1]), T(P.g[2])};
    for (int i = 0; i < nb; ++i) {
      const Body<T>& B = V.bodies[i];
      point_jacobian(V, kin, i, kin.p[i], Jv.data());
      angular_jacobian(V, kin, i, Jw.data());
      V3<T> vel{0, 0, 0}, om{0, 0, 0};
      for (int r = 0; r < 3; ++r)
        for (int k = 0; k < nv; ++k) { vel[r] += Jv[r * nv + k] * S.v[k]; om[r] += Jw[r * nv + k] * S.v[k]; }
      M3<T> I = world_inertia(B, kin.R[i]);
      E += B.mass * dot(vel, vel) / 2 + dot(om, mv(I, om)) / 2 - B.mass * dot(gv, kin.p[i]);
      Pm = add(Pm, scl(vel, B.mass));
      Lm = add(Lm, add(cross(kin.p[i], scl(vel, B.mass)), mv(I, om)));
    }
    if (V.ball) {
      const int vb = V.nvr;
      V3<T> vel = {S.v[vb + 3], S.v[vb + 4], S.v[vb + 5]}, om = {S.v[vb], S.v[vb + 1], S.v[vb + 2]};
      E += V.ball_m * dot(vel, vel) / 2 + V.ball_I * dot(om, om) / 2 - V.ball_m * dot(gv, kin.cb);
      Pm = add(Pm, scl(vel, V.ball_m));
      Lm = add(Lm, add(cross(kin.cb, scl(vel, V.ball_m)), scl(om, V.ball_I)));
    }
    out[0] = E;
    for (int r = 0; r < 3; ++r) { out[1 + r] = Pm[r]; out[4 + r] = Lm[r]; }
  }

  T fitness(int vi) const {
    const State<T>& S = st[vi];
    if (S.status) return T(NAN);
    T dx, dy;
    if (var[vi].r0 == 6) { dx = S.q[0] - S.x0; dy = S.q[1] - S.y0; }
    else { dx = 0; dy = 0; }
    return std::sqrt(dx * dx + dy * dy);
  }

  void reset(int vi) {
    const Variant<T>& V = var[vi];
    State<T>& S = st[vi];
    S.q = V.q0; S.v = V.v0; S.k = 0; S.status = 0; S.rows_contact = S.rows_clamp = 0;
    S.plane_margin = std::numeric_limits<double>::infinity();
    S.x0 = V.r0 == 6 ? V.q0[0] : T(0);
    S.y0 = V.r0 == 6 ? V.q0[1] : T(0);
  }
};

// Run f(i) for i in [0, n) on nthreads threads (contiguous blocks, static split).
template <class F> void parallel_for(int n, int nthreads, F f) {
  if (nthreads <= 1 || n <= 1) {
    for (int i = 0; i < n; ++i) f(i);
    return;
  }
  nthreads = std::min(nthreads, n);
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t)
    pool.emplace_back([=, &f] {
      for (int i = t; i < n; i += nthreads) f(i);
    });
  for (auto& th : pool) th.join();
}

struct Handle {
  int precision;  // 64 or 32
  std::unique_ptr<Sim<double>> d;
  std::unique_ptr<Sim<float>> f;
};

template <class T>
void parse(Sim<T>& S, int n, const int32_t* body_offset, const int32_t* parent, const float* half,
           const float* mass, const float* ap, const float* ac, const float* rq, const float* axis,
           const float* cpg, const float* mu, const float* q0, const float* v0, const float* root_pose,
           const float* ball, const double* params, int root_fixed, int K, int self_collision) {
  S.P = Params{params[0], params[1], params[2], params[3], params[4], params[5],
               {params[6], params[7], params[8]}, K, root_fixed, self_collision};
  S.var.resize(n);
  S.st.resize(n);
  int64_t qo = 0, vo = 0;
  for (int i = 0; i < n; ++i) {
    Variant<T>& V = S.var[i];
    int b0 = body_offset[i], nb = body_offset[i + 1] - b0;
    V.bodies.resize(nb);
    V.path.resize(nb);
    V.nh = nb - 1;
    V.r0 = root_fixed ? 0 : 6;
    V.nqr = V.nh + (root_fixed ? 0 : 7);
    V.nvr = V.nh + V.r0;
    V.ball = ball != nullptr;
    if (V.ball) {
      V.ball_r = T(ball[2 * i]);
      V.ball_m = T(ball[2 * i + 1]);
      V.ball_I = T(2) / T(5) * V.ball_m * V.ball_r * V.ball_r;
    }
    V.nq = V.nqr + (V.ball ? 7 : 0);
    V.nv = V.nvr + (V.ball ? 6 : 0);
    V.mu = T(mu[i]);
    for (int k = 0; k < 3; ++k) V.root_p[k] = T(root_pose[7 * i + k]);
    for (int k = 0; k < 4; ++k) V.root_q[k] = T(root_pose[7 * i + 3 + k]);
    for (int b = 0; b < nb; ++b) {
      Body<T>& B = V.bodies[b];
      int gb = b0 + b;
      B.parent = parent[gb];
      for (int k = 0; k < 3; ++k) {
        B.half[k] = T(half[3 * gb + k]);
        B.anchor_parent[k] = T(ap[3 * gb + k]);
        B.anchor_child[k] = T(ac[3 * gb + k]);
        B.axis[k] = T(axis[3 * gb + k]);
      }
      T qq[4] = {T(rq[4 * gb]), T(rq[4 * gb + 1]), T(rq[4 * gb + 2]), T(rq[4 * gb + 3])};
      B.rest = quat_to_rot(qq);
      B.mass = T(mass[gb]);
      T hx = B.half[0], hy = B.half[1], hz = B.half[2];
      B.Ib = {B.mass / 3 * (hy * hy + hz * hz), B.mass / 3 * (hx * hx + hz * hz), B.mass / 3 * (hx * hx + hy * hy)};
      B.A = T(cpg[3 * gb]); B.omega = T(cpg[3 * gb + 1]); B.phi = T(cpg[3 * gb + 2]);
      for (int j = b; j > 0; j = parent[b0 + j]) V.path[b].push_back(j);
    }
    V.q0.assign(q0 + qo, q0 + qo + V.nq);
    V.v0.assign(v0 + vo, v0 + vo + V.nv);
    qo += V.nq;
    vo += V.nv;
    S.reset(i);
  }
}

}  // namespace

extern "C" {

// Create a reference simulator.  params = [kp, kd, tau_max, k_contact, b_contact, dt, gx, gy, gz];
// ball = [radius, mass] per variant, or NULL for no ball; self_collision != 0
// adds the vertex-face contacts between boxes of one robot not joined by a hinge.
void* orc_create(int n, const int32_t* body_offset, const int32_t* parent, const float* half,
                 const float* mass, const float* anchor_parent, const float* anchor_child,
                 const float* rest_quat, const float* axis, const float* cpg, const float* mu,
                 const float* q0, const float* v0, const float* root_pose, const float* ball,
                 const double* params, int root_fixed, int pgs_iters, int precision, int self_collision) {
  auto* h = new Handle();
  h->precision = precision;
  if (precision == 32) {
    h->f.reset(new Sim<float>());
    parse(*h->f, n, body_offset, parent, half, mass, anchor_parent, anchor_child, rest_quat, axis, cpg, mu,
          q0, v0, root_pose, ball, params, root_fixed, pgs_iters, self_collision);
  } else {
    h->d.reset(new Sim<double>());
    parse(*h->d, n, body_offset, parent, half, mass, anchor_parent, anchor_child, rest_quat, axis, cpg, mu,
          q0, v0, root_pose, ball, params, root_fixed, pgs_iters, self_collision);
  }
  return h;
}

void orc_destroy(void* hp) { delete static_cast<Handle*>(hp); }

#define ORC_DISPATCH(h, ...)                                          \
  do {                                                                \
    if ((h)->precision == 32) { auto& S = *(h)->f; __VA_ARGS__; }     \
    else { auto& S = *(h)->d; __VA_ARGS__; }                          \
  } while (0)

// Advance every variant by n steps (variants spread over nthreads threads).
void orc_step(void* hp, int n_steps, int nthreads) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, parallel_for((int)S.var.size(), nthreads, [&](int i) { for (int s = 0; s < n_steps; ++s) S.step(i); }));
}
// Same for a subset of variants (indices).
void orc_step_subset(void* hp, int n_idx, const int32_t* idx, int n_steps, int nthreads) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, parallel_for(n_idx, nthreads, [&](int i) { for (int s = 0; s < n_steps; ++s) S.step(idx[i]); }));
}
void orc_reset(void* hp) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, for (int i = 0; i < (int)S.var.size(); ++i) S.reset(i));
}
// RK4 on the smooth dynamics (contact ignored); pd != 0 applies the explicit clamped PD torque.
void orc_rk4(void* hp, int n_steps, int pd, int nthreads) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, parallel_for((int)S.var.size(), nthreads, [&](int i) { for (int s = 0; s < n_steps; ++s) S.rk4_step(i, pd != 0); }));
}
void orc_fitness(void* hp, double* out) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, for (int i = 0; i < (int)S.var.size(); ++i) out[i] = double(S.fitness(i)));
}
// State in variant-CSR order (same layout as the model's q0 / v0).
void orc_get_state(void* hp, double* q, double* v, int64_t* k, uint32_t* status) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, {
    int64_t qo = 0, vo = 0;
    for (int i = 0; i < (int)S.var.size(); ++i) {
      for (size_t j = 0; j < S.st[i].q.size(); ++j) q[qo + j] = double(S.st[i].q[j]);
      for (size_t j = 0; j < S.st[i].v.size(); ++j) v[vo + j] = double(S.st[i].v[j]);
      qo += S.st[i].q.size(); vo += S.st[i].v.size();
      if (k) k[i] = S.st[i].k;
      if (status) status[i] = S.st[i].status;
    }
  });
}
void orc_set_state(void* hp, const double* q, const double* v, const int64_t* k) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, {
    int64_t qo = 0, vo = 0;
    for (int i = 0; i < (int)S.var.size(); ++i) {
      auto& st = S.st[i];
      for (size_t j = 0; j < st.q.size(); ++j) st.q[j] = q[qo + j];
      for (size_t j = 0; j < st.v.size(); ++j) st.v[j] = v[vo + j];
      qo += st.q.size(); vo += st.v.size();
      if (k) st.k = k[i];
      st.status = 0;
      st.plane_margin = std::numeric_limits<double>::infinity();
    }
  });
}
// Closest approach of a box corner or the ball to the plane, per variant, over
// the steps since the last reset / set_state (infinity before the first step).
void orc_plane_margin(void* hp, double* out) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, for (int i = 0; i < (int)S.var.size(); ++i) out[i] = S.st[i].plane_margin);
}
void orc_counters(void* hp, uint64_t* rows_contact, uint64_t* rows_clamp) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, for (int i = 0; i < (int)S.var.size(); ++i) {
    rows_contact[i] = S.st[i].rows_contact; rows_clamp[i] = S.st[i].rows_clamp;
  });
}
// Invariants of variant vi at its current state: [E, Px, Py, Pz, Lx, Ly, Lz].
void orc_invariants(void* hp, int vi, double* out) {
  auto* h = static_cast<Handle*>(hp);
  ORC_DISPATCH(h, {
    decltype(S.var[0].mu) tmp[7];
    S.invariants(vi, tmp);
    for (int k = 0; k < 7; ++k) out[k] = double(tmp[k]);
  });
}

// ---- probes of single pieces, for the unit tests (double precision handles only) ----
// Body poses of variant vi at generalised position q: R [nb*9], p [nb*3], hinge axes w and anchors o [nb*3].
int orc_fk(void* hp, int vi, const double* q, double* R, double* p, double* w, double* o) {
  auto* h = static_cast<Handle*>(hp);
  if (h->precision != 64) return -1;
  auto& S = *h->d;
  Kin<double> kin;
  S.fk(S.var[vi], q, kin);
  for (size_t b = 0; b < kin.R.size(); ++b) {
    for (int k = 0; k < 9; ++k) R[9 * b + k] = kin.R[b][k];
    for (int k = 0; k < 3; ++k) { p[3 * b + k] = kin.p[b][k]; w[3 * b + k] = kin.w[b][k]; o[3 * b + k] = kin.o[b][k]; }
  }
  return 0;
}
// Mass matrix M [nv*nv] and bias c [nv] at (q, v), gravity from the model.
int orc_dynamics(void* hp, int vi, const double* q, const double* v, double* M, double* c) {
  auto* h = static_cast<Handle*>(hp);
  if (h->precision != 64) return -1;
  auto& S = *h->d;
  Kin<double> kin;
  S.fk(S.var[vi], q, kin);
  S.mass_matrix(S.var[vi], kin, M);
  S.bias(S.var[vi], kin, v, S.P.g, c);
  return 0;
}
// Active contacts at q: returns count (<= max); body, corner, point x [3], depth, rows J [3*nv] (n, x, y).
// corner: 0..7 box corner, -1 ball-plane, -2 ball-box (body = the box), -3
// edge-edge contact of boxes `body` and `other` (normal towards `body`); other:
// the penetrated box of a self-collision contact (corner `corner` of `body`), else -1;
// normal n [3] (towards the ball / the corner's box).
int orc_contacts(void* hp, int vi, const double* q, int max, int32_t* body, int32_t* corner, double* x,
                 double* depth, double* J, double* normal, int32_t* other) {
  auto* h = static_cast<Handle*>(hp);
  if (h->precision != 64) return -1;
  auto& S = *h->d;
  const auto& V = S.var[vi];
  Kin<double> kin;
  S.fk(V, q, kin);
  std::vector<Sim<double>::Contact> C;
  S.detect(V, kin, C);
  int nv = V.nv, n = std::min<int>(max, (int)C.size());
  std::vector<double> Jp(3 * nv);
  const int rowsel[3] = {2, 0, 1};
  for (int i = 0; i < n; ++i) {
    body[i] = C[i].body; corner[i] = C[i].corner; depth[i] = C[i].depth; other[i] = C[i].other;
    for (int k = 0; k < 3; ++k) { x[3 * i + k] = C[i].x[k]; normal[3 * i + k] = C[i].n[k]; }
    S.contact_jacobian(V, kin, C[i], Jp.data());
    for (int r = 0; r < 3; ++r)
      for (int k = 0; k < nv; ++k) J[(3 * i + r) * nv + k] = Jp[rowsel[r] * nv + k];
  }
  return (int)C.size();
}
// The library's edge-edge contact of two boxes (poses: centre [3], rotation
// row-major [9], half extents [3]), exposed for its pins: returns 1 and the
// contact point, normal (towards box P) and depth, or 0 when it gives none.
int orc_edge_contact(const double* pP, const double* RP, const double* hP, const double* pQ, const double* RQ,
                     const double* hQ, double* x, double* n, double* depth) {
  V3<double> a{pP[0], pP[1], pP[2]}, b{pQ[0], pQ[1], pQ[2]}, ha{hP[0], hP[1], hP[2]}, hb{hQ[0], hQ[1], hQ[2]};
  M3<double> Ra, Rb;
  for (int k = 0; k < 9; ++k) { Ra[k] = RP[k]; Rb[k] = RQ[k]; }
  V3<double> xx, nn;
  double d = 0;
  if (!edge_contact(a, Ra, ha, b, Rb, hb, xx, nn, d)) return 0;
  for (int k = 0; k < 3; ++k) { x[k] = xx[k]; n[k] = nn[k]; }
  *depth = d;
  return 1;
}

// face_contacts on two boxes (row-major rotations); returns the count m and
// writes m points x[3 m], depths[m], the normal n[3] and inc (0: the points
// belong to P, 1: to Q).
int orc_face_contacts(const double* pP, const double* RP, const double* hP, const double* pQ, const double* RQ,
                      const double* hQ, double* x, double* depth, double* n, int* inc) {
  V3<double> a{pP[0], pP[1], pP[2]}, b{pQ[0], pQ[1], pQ[2]}, ha{hP[0], hP[1], hP[2]}, hb{hQ[0], hQ[1], hQ[2]};
  M3<double> Ra, Rb;
  for (int k = 0; k < 9; ++k) { Ra[k] = RP[k]; Rb[k] = RQ[k]; }
  V3<double> xs[24], nn;
  double ds[24];
  int ic = 0;
  const int m = face_contacts(a, Ra, ha, b, Rb, hb, xs, ds, nn, ic);
  for (int i = 0; i < m; ++i) {
    for (int k = 0; k < 3; ++k) x[3 * i + k] = xs[i][k];
    depth[i] = ds[i];
  }
  for (int k = 0; k < 3; ++k) n[k] = nn[k];
  *inc = ic;
  return m;
}

// The library's own Cholesky, exposed so a test can compare it with LAPACK.
int orc_cholesky(int n, const double* A, double* L) { return cholesky(n, A, L) ? 0 : -1; }

}  // extern "C"
