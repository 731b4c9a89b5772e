// Per-pair device code: Moeller screening with exact decisions, and the hand-derived
// derivatives of the two interval ends.
//
// Notation (Sec. 1): T_a = (u0,u1,u2), T_b = (v0,v1,v2); n_a = (u1-u0) x (u2-u0),
// n_b = (v1-v0) x (v2-v0); D = n_a x n_b spans the intersection line L; t(P) = D.P/|D|.
// d_k = n_b.(u_k - v0) are T_a's plane sides against T_b, e_k = n_a.(v_k - u0) T_b's
// against T_a.  Each triangle's cut is a segment with two endpoints, each either a vertex on
// the other plane or the lerp u_p + lam (u_q - u_p), lam = d_p / (d_p - d_q), on an edge whose
// ends lie strictly on opposite sides (the appendix's case table).  I_a = [t_a^0, t_a^1] and
// I_b by min/max, and Eq. 1 gives t_c^0 = t_a^0 - t_b^1, t_c^1 = t_a^1 - t_b^0.
//
// Exact flag.  For P on edge (p, q) of T_a and Q on edge (r, s) of T_b (an on-plane vertex p
// is the edge (p, q) with lam = 0 for any q off the plane), both on L:
//     det[q-p, r-p, s-p] = D.(Q-P)/|D|^2 * (d_q - d_p) * (e_s - e_r) * |D|... up to a positive
// factor: substituting p = P - lam (q-p) and r = Q - mu (s-r) leaves det[q-p, Q-P, s-r], and
// with Q - P parallel to D, (q-p).(D x (s-r)) = (n_b.(q-p)) (n_a.(s-r)) because n_a.(q-p) = 0
// and n_b.(s-r) = 0.  Hence sign(t(Q) - t(P)) = sign(orient(p,q,r,s)) sign(d_q - d_p)
// sign(e_s - e_r), where the last two signs are known exactly from the classification.
// The open interval (t_c^0, t_c^1) contains 0 iff some T_a endpoint lies strictly after
// some T_b endpoint and some strictly before: four exact orientation signs decide it.
//
// Derivatives.  All four endpoints lie on L, so d t(P) = Dh . dP with the line direction
// Dh = D/|D| held fixed (its variation is orthogonal to Dh and P - Q is parallel to Dh).  For a
// lerp endpoint  dP = (1-lam) du_p + lam du_q + (u_q - u_p) dlam,
// dlam = (d_p dd_q - d_q dd_p) / (d_p - d_q)^2, and d_x = det[v1-v0, v2-v0, x-v0] has partials
// n_b (x), (v2-v0) x (x-v0) (v1), (x-v0) x (v1-v0) (v2) and minus their sum (v0).  So each
// endpoint adds 3-vectors at five vertex slots; a = dt_c^0 and b = dt_c^1 are two such sums.
#pragma once

#include "device_math.h"
#include "predicates.h"

namespace ttie {

enum { PAIR_NONE = 0, PAIR_HIT = 1, PAIR_ADJACENT = 2, PAIR_BAD_FRAME = 3, PAIR_COPLANAR = 4, PAIR_DEFER = 5 };
enum { STATUS_OK = 0, STATUS_INVALID = 1, STATUS_INDEX = 2, STATUS_NONFINITE = 3, STATUS_CAPACITY = 4, STATUS_UNSUPPORTED = 7,
       STATUS_INTERNAL = 8 };

// Geometry of a screened pair: kept for every intersecting pair.
struct HitGeom {
  int64_t key;      // (i << 32) | j
  int32_t pair;     // index into the candidate list
  uint32_t desc;    // endpoint descriptors and min/max picks
  double t0, t1;    // Eq. 1 interval ends (already scaled for the appendix half)
  double da[3];     // d_k = n_b.(u_k - v0) as used by the lerps
  double db[3];     // e_k = n_a.(v_k - u0)
};

// Descriptor layout: endpoint k (0,1) of cut c (0 = T_a on plane b, 1 = T_b on plane a) at
// bit 8c + 4k: vertex p in bits 0-1, q in bits 2-3 (q = 3: the endpoint is vertex p itself).
// Bits 16..19: which endpoint is the min of I_a, the max of I_a, the min of I_b, the max of
// I_b.
__device__ __forceinline__ int desc_p(uint32_t d, int c, int k) { return (d >> (8 * c + 4 * k)) & 3; }
__device__ __forceinline__ int desc_q(uint32_t d, int c, int k) { return (d >> (8 * c + 4 * k + 2)) & 3; }
__device__ __forceinline__ int desc_pick(uint32_t d, int which) { return (d >> (16 + which)) & 1; }

struct Cut {
  int s[3];        // exact side signs
  int p[2], q[2];  // q = 3: on-plane vertex
  int straddle;
};

// The appendix's case table: lone vertex k on its side gives the edges (k, k+1) and (k, k+2)
// in index order; one vertex on the plane gives that vertex and the crossing of the
// opposite edge.
__device__ __forceinline__ Cut make_cut(int s0, int s1, int s2) {
  Cut c;
  c.s[0] = s0; c.s[1] = s1; c.s[2] = s2;
  const int pos = (s0 > 0) + (s1 > 0) + (s2 > 0);
  const int neg = (s0 < 0) + (s1 < 0) + (s2 < 0);
  c.straddle = pos > 0 && neg > 0;
  c.p[0] = c.p[1] = 0;
  c.q[0] = c.q[1] = 3;
  if (!c.straddle) return c;
  if (pos == 2 || neg == 2) {
    const int lone = pos == 2 ? -1 : 1;
    const int k = s0 == lone ? 0 : (s1 == lone ? 1 : 2);
    c.p[0] = k; c.q[0] = k == 0 ? 1 : 0;
    c.p[1] = k; c.q[1] = k == 2 ? 1 : 2;
  } else {
    const int k = s0 == 0 ? 0 : (s1 == 0 ? 1 : 2);
    c.p[0] = k; c.q[0] = 3;
    // crossing of the opposite edge, written from the next vertex as the appendix does:
    // vertex 0 on the plane -> (1,2); vertex 1 -> (2,0); vertex 2 -> (0,1)
    c.p[1] = (k + 1) % 3; c.q[1] = (k + 2) % 3;
  }
  return c;
}

// Sign of t(end 1) - t(end 0) for the cut of A by the plane of B, with D = n_A x n_B (the
// cut of B by the plane of A has the opposite sign).  Both ends lie on the line, so
// end 1 - end 0 = mu D; crossing it with the first edge e1 = (k, k1) within A's plane gives
// mu |n_A|^2 (n_B . e1) = lambda n_A . (e1 x e2) with lambda > 0.  n_B . e1 has the sign of
// the side of k1 (k is on the other side or on the plane), and n_A . (e1 x e2) is +|n_A|^2
// when (k, k1, k2) runs in the triangle's own order.
__device__ __forceinline__ int seg_order(const Cut& c) {
  const int k = c.p[0];
  const int k1 = c.q[0] != 3 ? c.q[0] : c.p[1];
  const int s1 = k1 == 0 ? c.s[0] : (k1 == 1 ? c.s[1] : c.s[2]);
  return (k1 == (k == 2 ? 0 : k + 1)) ? s1 : -s1;
}

struct Tri64 {
  double p[3][3];
};

// exact plane sides of the three vertices of `cut` against the plane of `pl`.  Without
// kExact a sign the FP64 filter cannot certify returns false (the pair is deferred).
template <bool kExact>
__device__ __forceinline__ bool plane_sides(const Tri64& pl, const Tri64& cut, int s[3], double d[3], int& status) {
  const V3<double> o{pl.p[0][0], pl.p[0][1], pl.p[0][2]};
  const V3<double> e1 = V3<double>{pl.p[1][0], pl.p[1][1], pl.p[1][2]} - o;
  const V3<double> e2 = V3<double>{pl.p[2][0], pl.p[2][1], pl.p[2][2]} - o;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const V3<double> w = V3<double>{cut.p[k][0], cut.p[k][1], cut.p[k][2]} - o;
    double det, bound;
    orient_fp64(e1, e2, w, det, bound);
    if (fabs(det) > bound) {
      s[k] = det > 0 ? 1 : -1;
      d[k] = det;
    } else if (bound == 0.0) {
      // every monomial has an exactly zero difference factor: the determinant is exactly 0
      s[k] = 0;
      d[k] = 0.0;
    } else {
      if (!kExact) return false;
      OrientResult r = orient_exact(pl.p[0], pl.p[1], pl.p[2], cut.p[k]);
      if (r.overflow) status = STATUS_UNSUPPORTED;
      s[k] = r.sign;
      d[k] = r.value;
    }
  }
  return true;
}

// register selects: the candidates are passed by value so that a runtime index becomes a
// conditional move instead of a runtime address into a local array (which spills it)
__device__ __forceinline__ int pick(int a, int b, int c, int i) { return i == 0 ? a : (i == 1 ? b : c); }
__device__ __forceinline__ double pick(double a, double b, double c, int i) { return i == 0 ? a : (i == 1 ? b : c); }
__device__ __forceinline__ int seli(const int (&a)[3], int i) { return pick(a[0], a[1], a[2], i); }
__device__ __forceinline__ double seld(const double (&a)[3], int i) { return pick(a[0], a[1], a[2], i); }
__device__ __forceinline__ V3<double> selv(const Tri64& T, int i) {
  return V3<double>{pick(T.p[0][0], T.p[1][0], T.p[2][0], i), pick(T.p[0][1], T.p[1][1], T.p[2][1], i),
                    pick(T.p[0][2], T.p[1][2], T.p[2][2], i)};
}

// the vertex paired with an on-plane vertex to form a degenerate edge: any vertex off the plane
__device__ __forceinline__ int partner(const Cut& c, int k) {
  const int p = k == 0 ? c.p[0] : c.p[1], q = k == 0 ? c.q[0] : c.q[1];
  return q != 3 ? q : (seli(c.s, (p + 1) % 3) != 0 ? (p + 1) % 3 : (p + 2) % 3);
}

// sign of orient(p, q, r, s) = det[q-p, r-p, s-p]; 2 when only the exact path could tell
// and kExact is off
template <bool kExact>
__device__ __forceinline__ int orient_sign(const V3<double>& p, const V3<double>& q, const V3<double>& r,
                                           const V3<double>& s, int& status) {
  double det, bound;
  orient_fp64(q - p, r - p, s - p, det, bound);
  if (fabs(det) > bound) return det > 0 ? 1 : -1;
  if (bound == 0.0) return 0;
  if (!kExact) return 2;
  const double P[3] = {p.x, p.y, p.z}, Q[3] = {q.x, q.y, q.z}, R[3] = {r.x, r.y, r.z}, S[3] = {s.x, s.y, s.z};
  OrientResult o = orient_exact(P, Q, R, S);
  if (o.overflow) status = STATUS_UNSUPPORTED;
  return o.sign;
}

// Sign of the 2D orientation of (a, b, c) with coordinate k dropped; 2 when only the exact path
// could tell and kExact is off.  It is orient((a', 0), (b', 0), (c', 0), (0, 0, 1)) on the
// dropped points, whose determinant is exactly the 2D one, so the filter and the exact path
// of the 3D predicate decide it.
template <bool kExact>
__device__ __forceinline__ int orient2_sign(const V3<double>& a, const V3<double>& b, const V3<double>& c, int k,
                                            int& status) {
  const auto drop = [k](const V3<double>& p) {
    return k == 0 ? V3<double>{p.y, p.z, 0.0} : (k == 1 ? V3<double>{p.z, p.x, 0.0} : V3<double>{p.x, p.y, 0.0});
  };
  return orient_sign<kExact>(drop(a), drop(b), drop(c), V3<double>{0.0, 0.0, 1.0}, status);
}

// Two triangles in one plane: the paper's reduction gives no segment and T = 0.  Their
// interiors overlap exactly when no edge line separates them (for convex polygons with
// disjoint interiors, the line through some edge of one leaves the other in its closed outer
// half-plane).  Decided with exact 2D orientations after dropping the coordinate A's FP64
// normal leans on most (or, if A has no area there, the next coordinate where it has some).
// Returns PAIR_COPLANAR, PAIR_NONE, or PAIR_DEFER when kExact is off and a sign needs the
// exact path.
template <bool kExact>
__device__ __forceinline__ int coplanar_kind(const Tri64& A, const Tri64& B, int& status) {
  const V3<double> a[3] = {selv(A, 0), selv(A, 1), selv(A, 2)};
  const V3<double> b[3] = {selv(B, 0), selv(B, 1), selv(B, 2)};
  const V3<double> n = cross(a[1] - a[0], a[2] - a[0]);
  const double nx = fabs(n.x), ny = fabs(n.y), nz = fabs(n.z);
  const int k0 = nx >= ny && nx >= nz ? 0 : (ny >= nz ? 1 : 2);
  int k = k0, sa = 0;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    k = (k0 + t) % 3;
    sa = orient2_sign<kExact>(a[0], a[1], a[2], k, status);
    if (sa != 0) break;
  }
  if (sa == 2) return PAIR_DEFER;
  if (sa == 0) return PAIR_NONE;  // A has no area
  const int sb = orient2_sign<kExact>(b[0], b[1], b[2], k, status);
  if (sb == 2) return PAIR_DEFER;
  if (sb == 0) return PAIR_NONE;  // B has no area
  // (fully unrolled, so every vertex index is a constant and nothing lives in scratch)
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const V3<double>* P = side == 0 ? a : b;
    const V3<double>* Q = side == 0 ? b : a;
    const int sp = side == 0 ? sa : sb;  // P's interior: edge orientations of sign sp
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      bool separates = true;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const int o = orient2_sign<kExact>(P[e], P[(e + 1) % 3], Q[j], k, status);
        if (o == 2) return PAIR_DEFER;
        separates &= o * sp <= 0;
      }
      if (separates) return PAIR_NONE;
    }
  }
  return PAIR_COPLANAR;
}

// Line direction D = n_a x n_b of a pair (Sec. 1: the intersection line of the two planes).
// The normals and D are rounded exactly as written, with no fused multiply-adds, so that the
// one discrete decision taken on rounded values -- D exactly (0, 0, 0), a degenerate frame --
// is the same wherever the definition is evaluated in float64.  (The exact D of a hit is never
// zero: both triangles straddle the other's plane.  Only rounded normals that come out parallel
// give a zero.)  A non-zero D is then multiplied by 2^-e, e the exponent of its largest
// component: exact, D/|D| unchanged, and |D|^2 stays finite and non-zero over the whole
// coordinate domain (components of order 2^-600 would underflow when squared).
__device__ __forceinline__ bool line_direction(const Tri64& A, const Tri64& B, V3<double>& D) {
#pragma clang fp contract(off)
  const double a1x = A.p[1][0] - A.p[0][0], a1y = A.p[1][1] - A.p[0][1], a1z = A.p[1][2] - A.p[0][2];
  const double a2x = A.p[2][0] - A.p[0][0], a2y = A.p[2][1] - A.p[0][1], a2z = A.p[2][2] - A.p[0][2];
  const double b1x = B.p[1][0] - B.p[0][0], b1y = B.p[1][1] - B.p[0][1], b1z = B.p[1][2] - B.p[0][2];
  const double b2x = B.p[2][0] - B.p[0][0], b2y = B.p[2][1] - B.p[0][1], b2z = B.p[2][2] - B.p[0][2];
  const double nax = a1y * a2z - a1z * a2y, nay = a1z * a2x - a1x * a2z, naz = a1x * a2y - a1y * a2x;
  const double nbx = b1y * b2z - b1z * b2y, nby = b1z * b2x - b1x * b2z, nbz = b1x * b2y - b1y * b2x;
  const double dx = nay * nbz - naz * nby, dy = naz * nbx - nax * nbz, dz = nax * nby - nay * nbx;
  const double m = fmax(fabs(dx), fmax(fabs(dy), fabs(dz)));
  if (!(m > 0.0)) {
    D = V3<double>{0.0, 0.0, 0.0};
    return false;
  }
  const int e = ilogb(m);
  D = V3<double>{ldexp(dx, -e), ldexp(dy, -e), ldexp(dz, -e)};
  return true;
}

struct Screen {
  int kind;  // PAIR_*
  uint32_t desc;
  double t0, t1;
  double da[3], db[3];
};

// The exact flag of two straddling cuts (sign(t(Q) - t(P)) for every pair of ends from four
// orientation signs, see the header): 1 when the open interval of Eq. 1 contains 0, 0 when it
// does not, 2 when a sign needs the exact path and kExact is off.
template <bool kExact>
__device__ __forceinline__ int cuts_intersect(const Tri64& A, const Tri64& B, const Cut& ca, const Cut& cb,
                                              int& status) {
  bool after = false, before = false;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int p = ca.p[i], q = partner(ca, i);
    const V3<double> P = selv(A, p), Q = selv(A, q);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int r = cb.p[j], s = partner(cb, j);
      // sign(t(Q) - t(P)) = sign(orient(p,q,r,s)) * sign(d_q - d_p) * sign(e_s - e_r)
      const int o = orient_sign<kExact>(P, Q, selv(B, r), selv(B, s), status);
      if (o == 2) return 2;
      const int tau = o * seli(ca.s, q) * seli(cb.s, s);
      after |= tau < 0;   // t(P) > t(Q)
      before |= tau > 0;  // t(P) < t(Q)
    }
  }
  return (after && before) ? 1 : 0;
}

// cuts_intersect for two cuts with no vertex on the other plane.  Each cut then has a lone
// vertex whose two edges carry the segment's ends (make_cut's table), so all four orientations
// share P (T_a's lone vertex) and R (T_b's): det[Q - P, R - P, S - P] is taken as
// (Q - P) x (R - P) dotted with S - P, two cross products for four determinants.  The caller
// passes the vertices in cut order -- P, T_a's two other vertices Q[0], Q[1] in the table's
// order with their sides sq; R, S[0], S[1] likewise -- so nothing is selected at run time.
// Each determinant's value, filter bound and verdict are orient_sign's, taken in the same
// order, so the result is cuts_intersect's.
struct LoneCut {
  int k, q0, q1;  // the lone vertex and the other two, in make_cut's order
};
__device__ __forceinline__ LoneCut lone_cut(int s0, int s1, int s2) {
  const int pos = (s0 > 0) + (s1 > 0) + (s2 > 0);
  const int lone = pos == 2 ? -1 : 1;
  LoneCut c;
  c.k = s0 == lone ? 0 : (s1 == lone ? 1 : 2);
  c.q0 = c.k == 0 ? 1 : 0;
  c.q1 = c.k == 2 ? 1 : 2;
  return c;
}

__device__ __forceinline__ int cuts_intersect_lone(const V3<double>& P, const V3<double> (&Q)[2], const int (&sq)[2],
                                                   const V3<double>& R, const V3<double> (&S)[2],
                                                   const int (&ss)[2]) {
  const V3<double> e2 = R - P;
  const V3<double> w[2] = {S[0] - P, S[1] - P};
  bool after = false, before = false;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const V3<double> e1 = Q[i] - P;
    const V3<double> n = cross(e1, e2);
    const double nx = fabs(e1.y * e2.z) + fabs(e1.z * e2.y);
    const double ny = fabs(e1.z * e2.x) + fabs(e1.x * e2.z);
    const double nz = fabs(e1.x * e2.y) + fabs(e1.y * e2.x);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double det = dot(n, w[j]);
      const double bound = kOrientErr * (nx * fabs(w[j].x) + ny * fabs(w[j].y) + nz * fabs(w[j].z));
      int o;
      if (fabs(det) > bound) o = det > 0 ? 1 : -1;
      else if (bound == 0.0) o = 0;  // every monomial has a zero factor: exactly 0
      else return 2;
      const int tau = o * sq[i] * ss[j];
      after |= tau < 0;
      before |= tau > 0;
    }
  }
  return (after && before) ? 1 : 0;
}

// FP64 interval ends of a hit on pair-local coordinates (origin u0), from its cuts and the
// plane sides out.da, out.db; fills out's descriptor and t0, t1 and its kind (PAIR_HIT, or
// PAIR_BAD_FRAME when the rounded line direction is 0).
__device__ __forceinline__ void interval_ends(const Tri64& A, const Tri64& B, const Cut& ca, const Cut& cb,
                                              double half, Screen& out) {
  const V3<double> o = selv(A, 0);
  V3<double> D;
  const bool frame = line_direction(A, B, D);
  const double len = sqrt(dot(D, D));
  double ta[2], tb[2];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    V3<double> P = selv(A, ca.p[k]) - o;
    if (ca.q[k] != 3) {
      const double dp = seld(out.da, ca.p[k]), dq = seld(out.da, ca.q[k]);
      P = P + (dp / (dp - dq)) * (selv(A, ca.q[k]) - selv(A, ca.p[k]));
    }
    ta[k] = dot(D, P);
    V3<double> Q = selv(B, cb.p[k]) - o;
    if (cb.q[k] != 3) {
      const double ep = seld(out.db, cb.p[k]), eq = seld(out.db, cb.q[k]);
      Q = Q + (ep / (ep - eq)) * (selv(B, cb.q[k]) - selv(B, cb.p[k]));
    }
    tb[k] = dot(D, Q);
  }
  // which end of each segment comes first along D, decided exactly (never from the rounded
  // t values, which can misorder two ends closer than their rounding error)
  const int amin = seg_order(ca) < 0 ? 1 : 0, amax = 1 - amin;
  const int bmin = seg_order(cb) > 0 ? 1 : 0, bmax = 1 - bmin;
  uint32_t desc = 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    desc |= (uint32_t)(ca.p[k] | (ca.q[k] << 2)) << (4 * k);
    desc |= (uint32_t)(cb.p[k] | (cb.q[k] << 2)) << (8 + 4 * k);
  }
  desc |= (uint32_t)amin << 16 | (uint32_t)amax << 17 | (uint32_t)bmin << 18 | (uint32_t)bmax << 19;
  out.desc = desc;
  if (!frame) {
    out.kind = PAIR_BAD_FRAME;
    return;
  }
  const double inv = half / len;
  out.t0 = ((amin ? ta[1] : ta[0]) - (bmax ? tb[1] : tb[0])) * inv;
  out.t1 = ((amax ? ta[1] : ta[0]) - (bmin ? tb[1] : tb[0])) * inv;
  out.kind = PAIR_HIT;
}

// Full screening of one non-adjacent pair in FP64 with exact decisions.  Without kExact,
// a pair needing the exact fallback for any sign comes back as PAIR_DEFER.
template <bool kExact>
__device__ __forceinline__ Screen screen_pair(const Tri64& A, const Tri64& B, double half, int& status) {
  Screen out;
  out.kind = PAIR_NONE;
  out.desc = 0;
  out.t0 = out.t1 = 0.0;
  int sa[3], sb[3];
  // T_a cut by the plane of T_b first, as the appendix does
  if (!plane_sides<kExact>(B, A, sa, out.da, status)) {
    out.kind = PAIR_DEFER;
    return out;
  }
  if ((sa[0] | sa[1] | sa[2]) == 0) {  // A lies in B's plane (or B has no area)
    out.kind = coplanar_kind<kExact>(A, B, status);
    return out;
  }
  const Cut ca = make_cut(sa[0], sa[1], sa[2]);
  if (!ca.straddle) return out;
  if (!plane_sides<kExact>(A, B, sb, out.db, status)) {
    out.kind = PAIR_DEFER;
    return out;
  }
  const Cut cb = make_cut(sb[0], sb[1], sb[2]);
  if (!cb.straddle) return out;
  const int x = cuts_intersect<kExact>(A, B, ca, cb, status);
  if (x == 2) out.kind = PAIR_DEFER;
  if (x == 1) interval_ends(A, B, ca, cb, half, out);
  return out;
}

// screen_pair for a pair whose exact plane sides are known to straddle both ways (sa: T_a's
// against T_b's plane, sb: the converse, as the FP64 pass of the first stage found them): the
// plane distances are computed only for a hit, by the same FP64 arithmetic that gave the
// signs, so every result is the one screen_pair gives.
template <bool kExact>
__device__ __forceinline__ Screen screen_pair_sides(const Tri64& A, const Tri64& B, const int (&sa)[3],
                                                    const int (&sb)[3], double half, int& status) {
  Screen out;
  out.kind = PAIR_NONE;
  out.desc = 0;
  out.t0 = out.t1 = 0.0;
  const Cut ca = make_cut(sa[0], sa[1], sa[2]), cb = make_cut(sb[0], sb[1], sb[2]);
  const int x = cuts_intersect<kExact>(A, B, ca, cb, status);
  if (x == 2) out.kind = PAIR_DEFER;
  if (x != 1) return out;
  int s2[3];
  if (!plane_sides<kExact>(B, A, s2, out.da, status) || !plane_sides<kExact>(A, B, s2, out.db, status)) {
    out.kind = PAIR_DEFER;
    return out;
  }
  interval_ends(A, B, ca, cb, half, out);
  return out;
}

// ------------------------------------------------------------------------------------------
// Derivatives of t_c^0 and t_c^1 (a and b, 18 each, slots u0,u1,u2,v0,v1,v2) for a hit.
// X holds pair-local coordinates in scalar S; dstored the FP64 plane sides of the screening.
// ------------------------------------------------------------------------------------------
// by-value selects for any scalar (see pick above) and slot accumulation with static indices
template <class T> __device__ __forceinline__ T pickt(T a, T b, T c, int i) { return i == 0 ? a : (i == 1 ? b : c); }
template <class S> __device__ __forceinline__ V3<S> pick3(const V3<S> (&v)[3], int i) {
  return V3<S>{pickt(v[0].x, v[1].x, v[2].x, i), pickt(v[0].y, v[1].y, v[2].y, i), pickt(v[0].z, v[1].z, v[2].z, i)};
}
template <class S> __device__ __forceinline__ void add_at(V3<S> (&out)[6], int slot, const V3<S>& v) {
#pragma unroll
  for (int k = 0; k < 6; ++k)
    if (k == slot) out[k] = out[k] + v;
}

// adds sgn * Dh . dP for endpoint (p, q) of the cut triangle C (slots cs..cs+2) against the
// plane of triangle P (slots ps..ps+2), d the cut triangle's plane sides, n the plane normal
template <class S>
__device__ __forceinline__ void add_endpoint(V3<S> (&out)[6], S sgn, int p, int q, const V3<S> (&C)[3],
                                             const V3<S> (&P)[3], const S (&d)[3], const V3<S>& n, const V3<S>& Dh,
                                             int cs, int ps) {
  if (q == 3) {
    add_at(out, cs + p, sgn * Dh);
    return;
  }
  const V3<S> Cp = pick3(C, p), Cq = pick3(C, q);
  const S dp = pickt(d[0], d[1], d[2], p), dq = pickt(d[0], d[1], d[2], q);
  const S den = dp - dq;
  const S lam = dp / den;
  const S w = dot(Dh, Cq - Cp) / (den * den);
  const S one = Sc<S>::c(1.0);
  add_at(out, cs + p, sgn * ((one - lam) * Dh - (w * dq) * n));
  add_at(out, cs + q, sgn * (lam * Dh + (w * dp) * n));
  const V3<S> Y = dp * (Cq - P[0]) - dq * (Cp - P[0]);
  const V3<S> g1 = w * cross(P[2] - P[0], Y);
  const V3<S> g2 = w * cross(Y, P[1] - P[0]);
  out[ps + 1] = out[ps + 1] + sgn * g1;
  out[ps + 2] = out[ps + 2] + sgn * g2;
  out[ps + 0] = out[ps + 0] - sgn * ((w * den) * n + g1 + g2);
}

// X: the pair's coordinates relative to u0 and multiplied by 2^-e (see local_coords); a and b
// are homogeneous of degree 0 in the coordinates, so the scaling changes nothing but the range
// of the intermediate values, which then neither under- nor overflows in float32.  The plane
// sides are of degree 3, so the stored ones are scaled by 2^-3e to match.
template <class S>
__device__ __forceinline__ void interval_grads(const V3<S> (&X)[6], const double dstored_a[3],
                                               const double dstored_b[3], int e, uint32_t desc, double half,
                                               S a[18], S b[18]) {
  const V3<S> U[3] = {X[0], X[1], X[2]};
  const V3<S> V[3] = {X[3], X[4], X[5]};
  const V3<S> na = cross(U[1] - U[0], U[2] - U[0]);
  const V3<S> nb = cross(V[1] - V[0], V[2] - V[0]);
  const V3<S> D = cross(na, nb);
  const S len = Sc<S>::sqrt_(dot(D, D));
  const V3<S> Dh = (Sc<S>::c(1.0) / len) * D;
  S da[3], db[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    // the screening's values (exact where the filter failed); tangents from the formula
    da[k] = Sc<S>::with_value(dot(nb, U[k] - V[0]), ldexp(dstored_a[k], -3 * e));
    db[k] = Sc<S>::with_value(dot(na, V[k] - U[0]), ldexp(dstored_b[k], -3 * e));
  }
  V3<S> ga[6], gb[6];
  const S zero = Sc<S>::c(0.0);
#pragma unroll
  for (int k = 0; k < 6; ++k) ga[k] = gb[k] = V3<S>{zero, zero, zero};
  const S pos = Sc<S>::c(half), neg = Sc<S>::c(-half);
  const int amin = desc_pick(desc, 0), amax = desc_pick(desc, 1);
  const int bmin = desc_pick(desc, 2), bmax = desc_pick(desc, 3);
  // a = d(t(P_amin) - t(Q_bmax)), b = d(t(P_amax) - t(Q_bmin))
  add_endpoint(ga, pos, desc_p(desc, 0, amin), desc_q(desc, 0, amin), U, V, da, nb, Dh, 0, 3);
  add_endpoint(ga, neg, desc_p(desc, 1, bmax), desc_q(desc, 1, bmax), V, U, db, na, Dh, 3, 0);
  add_endpoint(gb, pos, desc_p(desc, 0, amax), desc_q(desc, 0, amax), U, V, da, nb, Dh, 0, 3);
  add_endpoint(gb, neg, desc_p(desc, 1, bmin), desc_q(desc, 1, bmin), V, U, db, na, Dh, 3, 0);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    a[3 * k] = ga[k].x; a[3 * k + 1] = ga[k].y; a[3 * k + 2] = ga[k].z;
    b[3 * k] = gb[k].x; b[3 * k + 1] = gb[k].y; b[3 * k + 2] = gb[k].z;
  }
}

// 2x2 core M of the per-pair Hessian J^T M J for each PSD mode (see ttie.h), in FP64.
__device__ __forceinline__ void hessian_core(int mode, double t0, double t1, double aa, double bb, double ab,
                                             double M[3]) {
  const double s = t0 * t1;
  if (mode == 0) {  // per part
    const double na = sqrt(aa), nb = sqrt(bb);
    const bool ok = na > 0.0 && nb > 0.0;
    M[0] = 2.0 * t1 * t1 + (ok ? 2.0 * fabs(s) * nb / na : 0.0);
    M[1] = ok ? 2.0 * s : 0.0;
    M[2] = 2.0 * t0 * t0 + (ok ? 2.0 * fabs(s) * na / nb : 0.0);
    return;
  }
  if (mode == 2) {  // paper-literal
    M[0] = 2.0 * t1 * t1;
    M[1] = 8.0 * s * ab > 0.0 ? 4.0 * s : 0.0;
    M[2] = 2.0 * t0 * t0;
    return;
  }
  M[0] = 2.0 * t1 * t1;
  M[1] = 4.0 * s;
  M[2] = 2.0 * t0 * t0;
  if (mode != 1) return;  // raw Eq. 4
  // nearest PSD: the non-zero spectrum of J^T M J is that of K = G^1/2 M G^1/2 with the Gram
  // matrix G = J J^T; clamp K's eigenvalues and map back with the pseudo-inverse root of G.
  auto eig2 = [](double p, double r, double q, double& l0, double& l1, double& c, double& sn) {
    const double m = 0.5 * (p + q), h = 0.5 * (p - q);
    const double rad = sqrt(h * h + r * r);
    l0 = m + rad;
    l1 = m - rad;
    if (rad == 0.0) {
      c = 1.0; sn = 0.0;
    } else {  // eigenvector of l0: (h + rad, r) or (r, rad - h), whichever is larger
      double vx, vy;
      if (h >= 0) { vx = h + rad; vy = r; } else { vx = r; vy = rad - h; }
      const double nv = sqrt(vx * vx + vy * vy);
      c = vx / nv; sn = vy / nv;
    }
  };
  double g0, g1, gc, gs;
  eig2(aa, ab, bb, g0, g1, gc, gs);
  const double gmax = fmax(fabs(g0), fabs(g1));
  const double tol = 1e-14 * gmax;
  const double r0 = g0 > tol ? sqrt(g0) : 0.0, r1 = g1 > tol ? sqrt(g1) : 0.0;
  const double i0 = r0 > 0 ? 1.0 / r0 : 0.0, i1 = r1 > 0 ? 1.0 / r1 : 0.0;
  // R = [[gc, -gs],[gs, gc]] (columns: eigenvectors); root = R diag R^T
  auto sym = [&](double e0, double e1, double out[3]) {
    out[0] = gc * gc * e0 + gs * gs * e1;
    out[1] = gc * gs * (e0 - e1);
    out[2] = gs * gs * e0 + gc * gc * e1;
  };
  double Sq[3], Si[3];
  sym(r0, r1, Sq);
  sym(i0, i1, Si);
  auto mul = [](const double A[3], const double B[3], double C[4]) {  // C = A B (2x2 row-major)
    C[0] = A[0] * B[0] + A[1] * B[1];
    C[1] = A[0] * B[1] + A[1] * B[2];
    C[2] = A[1] * B[0] + A[2] * B[1];
    C[3] = A[1] * B[1] + A[2] * B[2];
  };
  double T[4], K[3];
  mul(Sq, M, T);  // Sq M
  K[0] = T[0] * Sq[0] + T[1] * Sq[1];
  K[1] = T[0] * Sq[1] + T[1] * Sq[2];
  K[2] = T[2] * Sq[1] + T[3] * Sq[2];
  double k0, k1, kc, ks;
  eig2(K[0], K[1], K[2], k0, k1, kc, ks);
  k0 = fmax(k0, 0.0);
  k1 = fmax(k1, 0.0);
  double Kp[3] = {kc * kc * k0 + ks * ks * k1, kc * ks * (k0 - k1), ks * ks * k0 + kc * kc * k1};
  mul(Si, Kp, T);  // Si K+
  M[0] = T[0] * Si[0] + T[1] * Si[1];
  M[1] = T[0] * Si[1] + T[1] * Si[2];
  M[2] = T[2] * Si[1] + T[3] * Si[2];
}

}  // namespace ttie
