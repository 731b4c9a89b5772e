// TTIE CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, FP64 reference for the triangle-triangle intersection energy (TTIE) of
// "Differentiable 3D Triangle-Triangle Intersection Energy".  It exists to check the HIP
// path; only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load
// it.  It shares no code with the GPU library: different arithmetic (forward-mode dual
// numbers, the appendix's formulas), different exact predicates (interval filter +
// arbitrary-precision dyadic fallback), different assembly (ordered maps).
//
// What it computes, per candidate pair (i, j) with T_a = tris[i] = (u0,u1,u2) and
// T_b = tris[j] = (v0,v1,v2), degrees of freedom ordered (u0,u1,u2,v0,v1,v2):
//   * Moeller's reduction (Sec. 1, Fig. 1; appendix function `intersects`): the plane of
//     one triangle cuts the other into a segment whose endpoints are either a vertex lying
//     on the plane or the lerp (d_q p - d_p q)/(d_q - d_p) along a crossing edge.
//   * the line frame of the appendix: D = n_a x n_b normalised, reference point A = mean
//     of the four endpoints, t = D.(S - A); intervals I_a, I_b by min/max.
//   * Eq. 1: t_c^0 = t_a^0 - t_b^1, t_c^1 = t_a^1 - t_b^0 (the appendix additionally halves
//     both; selectable).
//   * the open-interval criterion after Eq. 1 (0 in (t_c^0, t_c^1)), decided exactly.
//   * Eq. 2: T = (t_c^0 t_c^1)^2 on intersecting pairs, 0 otherwise.
//   * Eq. 3 gradient and all higher derivatives by forward-mode dual numbers (the
//     differentiation technique of the appendix), nested for Hessian-vector products.
//   * Eq. 4 inexact Hessian and its PSD projections built from the eigenanalysis of Sec. 1.1
//     as dense 18x18 matrices, with eigenvalues from a cyclic Jacobi sweep.
//   * energy / gradient / 3x3-block sparse Hessian assembly by plain ordered summation.
//
// Readings where the paper is silent (documented with the build):
//   - plane-side signs are the exact signs of the orientation determinant
//     det[p1-p0, p2-p0, x-p0]; an FP64 distance whose sign disagrees with the exact sign is
//     replaced by the exact value (rounded), so lerp weights stay in [0,1];
//   - the intersection flag is the exact open-interval test on the exact endpoints;
//   - the two ends of each segment are ordered along D exactly (the min/max of the interval
//     ends): with the segment's endpoints E0 on edge (k, k1) (or E0 = the on-plane vertex k and
//     E1 on the opposite edge (k1, k2)), t(E1) - t(E0) has the sign of the orientation of
//     (k, k1, k2) in the triangle times the side of k1 (negated for T_b, whose cut lies on the
//     plane of T_a and D = n_a x n_b), so two different endpoints never tie;
//   - pairs sharing a vertex index are "adjacent" and carry no energy;
//   - a hit whose FP64 line direction D = n_a x n_b (normals and D rounded as written, no fused
//     operations) is exactly (0, 0, 0) is reported with status 3 and T = 0: the exact D of a
//     hit is never zero (both triangles straddle the other's plane), so this happens only
//     when the rounded normals come out parallel;
//   - two triangles lying in one plane have no segment and no line, so T = 0 (the paper sets
//     coplanar pairs aside); when their interiors overlap the pair is reported with status 4,
//     still with T = 0, so that a caller can see where the energy is blind.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ============================================================================================
// Exact arithmetic: arbitrary-precision integers and dyadic rationals m * 2^e.
// Every finite double, and every sum, difference and product of them, is such a number.
// ============================================================================================
struct BigInt {
  int sign = 0;                 // -1, 0, +1
  std::vector<uint32_t> mag;    // little-endian base 2^32, no leading zero limbs
};

void trim(std::vector<uint32_t>& m) {
  while (!m.empty() && m.back() == 0) m.pop_back();
}

int cmp_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  if (a.size() != b.size()) return a.size() < b.size() ? -1 : 1;
  for (size_t k = a.size(); k-- > 0;)
    if (a[k] != b[k]) return a[k] < b[k] ? -1 : 1;
  return 0;
}

std::vector<uint32_t> add_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> r(std::max(a.size(), b.size()) + 1, 0);
  uint64_t carry = 0;
  for (size_t k = 0; k < r.size(); ++k) {
    uint64_t s = carry;
    if (k < a.size()) s += a[k];
    if (k < b.size()) s += b[k];
    r[k] = (uint32_t)s;
    carry = s >> 32;
  }
  trim(r);
  return r;
}

// |a| - |b| with |a| >= |b|
std::vector<uint32_t> sub_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  std::vector<uint32_t> r(a.size(), 0);
  int64_t borrow = 0;
  for (size_t k = 0; k < a.size(); ++k) {
    int64_t s = (int64_t)a[k] - borrow - (k < b.size() ? (int64_t)b[k] : 0);
    borrow = s < 0 ? 1 : 0;
    if (s < 0) s += ((int64_t)1 << 32);
    r[k] = (uint32_t)s;
  }
  trim(r);
  return r;
}

std::vector<uint32_t> mul_mag(const std::vector<uint32_t>& a, const std::vector<uint32_t>& b) {
  if (a.empty() || b.empty()) return {};
  std::vector<uint32_t> r(a.size() + b.size() + 1, 0);
  for (size_t i = 0; i < a.size(); ++i) {
    uint64_t carry = 0;
    for (size_t j = 0; j < b.size(); ++j) {
      uint64_t cur = (uint64_t)a[i] * b[j] + r[i + j] + carry;
      r[i + j] = (uint32_t)cur;
      carry = cur >> 32;
    }
    size_t k = i + b.size();
    while (carry) {
      uint64_t cur = (uint64_t)r[k] + carry;
      r[k] = (uint32_t)cur;
      carry = cur >> 32;
      ++k;
    }
  }
  trim(r);
  return r;
}

std::vector<uint32_t> shl_mag(const std::vector<uint32_t>& a, int64_t bits) {
  if (a.empty() || bits == 0) return a;
  size_t limbs = (size_t)(bits / 32);
  int rem = (int)(bits % 32);
  std::vector<uint32_t> r(a.size() + limbs + 1, 0);
  for (size_t k = 0; k < a.size(); ++k) {
    uint64_t v = (uint64_t)a[k] << rem;
    r[k + limbs] |= (uint32_t)v;
    r[k + limbs + 1] |= (uint32_t)(v >> 32);
  }
  trim(r);
  return r;
}

BigInt big_add(const BigInt& a, const BigInt& b) {
  if (a.sign == 0) return b;
  if (b.sign == 0) return a;
  BigInt r;
  if (a.sign == b.sign) {
    r.sign = a.sign;
    r.mag = add_mag(a.mag, b.mag);
    return r;
  }
  int c = cmp_mag(a.mag, b.mag);
  if (c == 0) return r;
  if (c > 0) {
    r.sign = a.sign;
    r.mag = sub_mag(a.mag, b.mag);
  } else {
    r.sign = b.sign;
    r.mag = sub_mag(b.mag, a.mag);
  }
  return r;
}

struct Dyadic {   // value = m * 2^e
  BigInt m;
  int64_t e = 0;
};

Dyadic dy(double x) {
  Dyadic r;
  if (x == 0.0) return r;
  int k = 0;
  double f = std::frexp(std::fabs(x), &k);          // |x| = f * 2^k, f in [0.5, 1)
  uint64_t mant = (uint64_t)std::ldexp(f, 53);      // exact: f has at most 53 significant bits
  r.m.sign = x < 0 ? -1 : 1;
  r.m.mag = {(uint32_t)mant, (uint32_t)(mant >> 32)};
  trim(r.m.mag);
  r.e = (int64_t)k - 53;
  return r;
}

Dyadic operator+(const Dyadic& a, const Dyadic& b) {
  if (a.m.sign == 0) return b;
  if (b.m.sign == 0) return a;
  Dyadic r;
  r.e = std::min(a.e, b.e);
  BigInt am = a.m, bm = b.m;
  am.mag = shl_mag(am.mag, a.e - r.e);
  bm.mag = shl_mag(bm.mag, b.e - r.e);
  r.m = big_add(am, bm);
  return r;
}
Dyadic operator-(const Dyadic& a) {
  Dyadic r = a;
  r.m.sign = -r.m.sign;
  return r;
}
Dyadic operator-(const Dyadic& a, const Dyadic& b) { return a + (-b); }
Dyadic operator*(const Dyadic& a, const Dyadic& b) {
  Dyadic r;
  if (a.m.sign == 0 || b.m.sign == 0) return r;
  r.m.sign = a.m.sign * b.m.sign;
  r.m.mag = mul_mag(a.m.mag, b.m.mag);
  r.e = a.e + b.e;
  return r;
}
int sgn(const Dyadic& a) { return a.m.sign; }

// Nearest-ish double (within one unit in the last place): only used to replace an FP64
// value whose sign is known to be wrong.
double to_double(const Dyadic& a) {
  if (a.m.sign == 0) return 0.0;
  const auto& m = a.m.mag;
  int64_t top_bits = (int64_t)(m.size() - 1) * 32 + (32 - __builtin_clz(m.back()));
  int64_t shift = std::max<int64_t>(0, top_bits - 64);
  // take the top 64 bits
  uint64_t v = 0;
  for (int64_t bit = top_bits - 1; bit >= shift; --bit) {
    uint32_t limb = m[(size_t)(bit / 32)];
    v = (v << 1) | ((limb >> (bit % 32)) & 1u);
  }
  return a.m.sign * std::ldexp((double)v, (int)(a.e + shift));
}

// ============================================================================================
// Interval arithmetic with outward rounding.  Under round-to-nearest the exact result of
// +, -, * lies within one ulp of the rounded one, so stepping each rounded bound one ulp
// outwards gives a guaranteed enclosure.
// ============================================================================================
struct Iv {
  double lo, hi;
};
const double kInf = std::numeric_limits<double>::infinity();
Iv iv(double x) { return {x, x}; }
Iv operator+(Iv a, Iv b) { return {std::nextafter(a.lo + b.lo, -kInf), std::nextafter(a.hi + b.hi, kInf)}; }
Iv operator-(Iv a, Iv b) { return {std::nextafter(a.lo - b.hi, -kInf), std::nextafter(a.hi - b.lo, kInf)}; }
Iv operator*(Iv a, Iv b) {
  double p[4] = {a.lo * b.lo, a.lo * b.hi, a.hi * b.lo, a.hi * b.hi};
  double lo = p[0], hi = p[0];
  for (double q : p) {
    if (std::isnan(q)) return {-kInf, kInf};
    lo = std::min(lo, q);
    hi = std::max(hi, q);
  }
  return {std::nextafter(lo, -kInf), std::nextafter(hi, kInf)};
}
// sign of the enclosed value if the enclosure proves it, else 2 (unknown)
int iv_sign(Iv a) {
  if (a.lo > 0) return 1;
  if (a.hi < 0) return -1;
  return 2;
}

// ============================================================================================
// Forward-mode dual numbers: value plus N tangents.  Nesting Dual<Dual<double,1>,18> gives
// second directional derivatives.
// ============================================================================================
template <class T, int N>
struct Dual {
  T v{};
  std::array<T, N> d{};
};

template <class T> struct is_dual { static constexpr bool value = false; };
template <class T, int N> struct is_dual<Dual<T, N>> { static constexpr bool value = true; };

template <class T, int N> Dual<T, N> operator+(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v + b.v;
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v - b.v;
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <class T, int N> Dual<T, N> operator-(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = -a.v;
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <class T, int N> Dual<T, N> operator*(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v * b.v;
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <class T, int N> Dual<T, N> operator*(double s, const Dual<T, N>& a) {
  Dual<T, N> r; r.v = s * a.v;
  for (int k = 0; k < N; ++k) r.d[k] = s * a.d[k];
  return r;
}
template <class T, int N> Dual<T, N> operator/(const Dual<T, N>& a, const Dual<T, N>& b) {
  Dual<T, N> r; r.v = a.v / b.v;
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] * b.v - a.v * b.d[k]) / (b.v * b.v);
  return r;
}
template <class T, int N> Dual<T, N> dsqrt(const Dual<T, N>& a);
inline double dsqrt(double a) { return std::sqrt(a); }
template <class T, int N> Dual<T, N> dsqrt(const Dual<T, N>& a) {
  Dual<T, N> r; r.v = dsqrt(a.v);
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] / (2.0 * r.v);
  return r;
}
inline double val(double a) { return a; }
template <class T, int N> double val(const Dual<T, N>& a) { return val(a.v); }
// overwrite the innermost value, keeping every tangent
inline void set_val(double& a, double x) { a = x; }
template <class T, int N> void set_val(Dual<T, N>& a, double x) { set_val(a.v, x); }

// ============================================================================================
// 3-vectors over any scalar
// ============================================================================================
template <class S> struct V3 { S x, y, z; };
template <class S> V3<S> operator+(const V3<S>& a, const V3<S>& b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class S> V3<S> operator-(const V3<S>& a, const V3<S>& b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class S> V3<S> scale(const S& s, const V3<S>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class S> V3<S> scale(double s, const V3<S>& a) { return {s * a.x, s * a.y, s * a.z}; }
template <class S> S dot(const V3<S>& a, const V3<S>& b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class S> V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <class S> V3<S> div(const V3<S>& a, const S& s) { return {a.x / s, a.y / s, a.z / s}; }

// orientation determinant det[b-a, c-a, p-a] = ((b-a) x (c-a)) . (p-a): the (unnormalised)
// signed distance of p from the plane of (a, b, c)
template <class S> S orient(const V3<S>& a, const V3<S>& b, const V3<S>& c, const V3<S>& p) {
  return dot(cross(b - a, c - a), p - a);
}

V3<Iv> to_iv(const double* p) { return {iv(p[0]), iv(p[1]), iv(p[2])}; }
V3<Dyadic> to_dy(const double* p) { return {dy(p[0]), dy(p[1]), dy(p[2])}; }

struct Side {
  int sign;        // exact sign of orient(plane, point)
  bool exact;      // the exact value below was computed
  Dyadic value;    // exact orient value (only when `exact`)
};

Side side(const double* a, const double* b, const double* c, const double* p) {
  int s = iv_sign(orient(to_iv(a), to_iv(b), to_iv(c), to_iv(p)));
  if (s != 2) return {s, false, {}};
  Dyadic e = orient(to_dy(a), to_dy(b), to_dy(c), to_dy(p));
  return {sgn(e), true, e};
}

// ============================================================================================
// The cut of a triangle by the other triangle's plane, per the appendix case analysis.
// ============================================================================================
struct Cut {
  bool straddle = false;
  int s[3] = {0, 0, 0};          // exact side signs of the cut triangle's vertices
  // endpoint k: on-plane vertex p[k] when q[k] < 0, else the crossing of edge (p[k], q[k])
  int p[2] = {0, 0}, q[2] = {-1, -1};
};

Cut classify(const int s[3]) {
  Cut c;
  int pos = 0, neg = 0, zero = 0;
  for (int i = 0; i < 3; ++i) {
    c.s[i] = s[i];
    if (s[i] > 0) ++pos; else if (s[i] < 0) ++neg; else ++zero;
  }
  if (!(pos > 0 && neg > 0)) return c;
  c.straddle = true;
  if (pos == 2 || neg == 2) {
    int lone_sign = pos == 2 ? -1 : 1;       // the vertex alone on its side
    int k = s[0] == lone_sign ? 0 : (s[1] == lone_sign ? 1 : 2);
    // lone 0: (0,1),(0,2); lone 1: (1,0),(1,2); lone 2: (2,0),(2,1)
    static const int other[3][2] = {{1, 2}, {0, 2}, {0, 1}};
    c.p[0] = k; c.q[0] = other[k][0];
    c.p[1] = k; c.q[1] = other[k][1];
  } else {  // one positive, one negative, one on the plane
    if (s[0] == 0) { c.p[0] = 0; c.q[0] = -1; c.p[1] = 1; c.q[1] = 2; }
    else if (s[1] == 0) { c.p[0] = 1; c.q[0] = -1; c.p[1] = 2; c.q[1] = 0; }
    else { c.p[0] = 2; c.q[0] = -1; c.p[1] = 0; c.q[1] = 1; }
  }
  return c;
}


// ============================================================================================
// Exact intersection flag.  The open interval (t_c^0, t_c^1) of Eq. 1 contains 0 iff some
// endpoint of I_a lies strictly after some endpoint of I_b and some endpoint of I_a lies
// strictly before some endpoint of I_b.  Every such comparison is the sign of D.(S_a - S_b)
// (t is D.S up to a positive factor and a common offset), with D = n_a x n_b and endpoints
// written as exact rationals num/den.  An interval enclosure settles it when it can; the
// dyadic evaluation of the same expression settles the rest.
// ============================================================================================
template <class S> S one();
template <> Iv one<Iv>() { return iv(1.0); }
template <> Dyadic one<Dyadic>() { return dy(1.0); }

template <class S> struct RatPoint { V3<S> num; S den; };

// endpoint k of a cut, with d[] the plane-side values of the cut triangle's vertices
template <class S>
RatPoint<S> rat_end(const Cut& c, int k, const V3<S> X[3], const S d[3]) {
  if (c.q[k] < 0) return {X[c.p[k]], one<S>()};
  const int p = c.p[k], q = c.q[k];
  return {scale(d[q], X[p]) - scale(d[p], X[q]), d[q] - d[p]};
}

// exact sign of the endpoint's denominator: 1 for an on-plane vertex, else sign(d_q - d_p),
// which is sign(d_q) because d_p and d_q have opposite signs on a crossing edge
int den_sign(const Cut& c, int k) { return c.q[k] < 0 ? 1 : c.s[c.q[k]]; }

// sign of (D.num_a) den_b - (D.num_b) den_a
template <class S>
S cmp_expr(const V3<S>& D, const RatPoint<S>& A, const RatPoint<S>& B) {
  return dot(D, A.num) * B.den - dot(D, B.num) * A.den;
}

struct Tri { const double* p[3]; };

template <class S>
void load_tri(const Tri& t, V3<S> out[3], V3<S> (*conv)(const double*)) {
  for (int k = 0; k < 3; ++k) out[k] = conv(t.p[k]);
}

// sign of t(S_a[i]) - t(S_b[j]) for all four endpoint pairs
void endpoint_order(const Tri& ta, const Tri& tb, const Cut& ca, const Cut& cb, int sig[2][2]) {
  V3<Iv> U[3], V[3];
  load_tri(ta, U, to_iv);
  load_tri(tb, V, to_iv);
  Iv da[3], db[3];
  for (int k = 0; k < 3; ++k) {
    da[k] = orient(V[0], V[1], V[2], U[k]);   // T_a's vertices against the plane of T_b
    db[k] = orient(U[0], U[1], U[2], V[k]);   // T_b's vertices against the plane of T_a
  }
  V3<Iv> D = cross(cross(U[1] - U[0], U[2] - U[0]), cross(V[1] - V[0], V[2] - V[0]));
  bool need_exact = false;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      int s = iv_sign(cmp_expr(D, rat_end(ca, i, U, da), rat_end(cb, j, V, db)));
      sig[i][j] = s == 2 ? 2 : s * den_sign(ca, i) * den_sign(cb, j);
      need_exact |= (s == 2);
    }
  if (!need_exact) return;
  V3<Dyadic> Ue[3], Ve[3];
  load_tri(ta, Ue, to_dy);
  load_tri(tb, Ve, to_dy);
  Dyadic dae[3], dbe[3];
  for (int k = 0; k < 3; ++k) {
    dae[k] = orient(Ve[0], Ve[1], Ve[2], Ue[k]);
    dbe[k] = orient(Ue[0], Ue[1], Ue[2], Ve[k]);
  }
  V3<Dyadic> De = cross(cross(Ue[1] - Ue[0], Ue[2] - Ue[0]), cross(Ve[1] - Ve[0], Ve[2] - Ve[0]));
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      if (sig[i][j] == 2)
        sig[i][j] = sgn(cmp_expr(De, rat_end(ca, i, Ue, dae), rat_end(cb, j, Ve, dbe))) *
                    den_sign(ca, i) * den_sign(cb, j);
}

bool exact_flag(const int sig[2][2]) {
  bool after = false, before = false;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) {
      after |= sig[i][j] > 0;
      before |= sig[i][j] < 0;
    }
  return after && before;
}

// ============================================================================================
// Dual-number stage: the appendix computation of the two segments and of t_c, carried out on
// any scalar S (Dual<double,18> for the gradient, Dual<Dual<double,1>,18> for Hv).
// ============================================================================================
template <class S>
V3<S> seg_point(const Cut& c, int k, const V3<S> C[3], const S d[3]) {
  if (c.q[k] < 0) return C[c.p[k]];
  const int p = c.p[k], q = c.q[k];
  return div(scale(d[q], C[p]) - scale(d[p], C[q]), d[q] - d[p]);   // (d_q C_p - d_p C_q)/(d_q - d_p)
}

int sign_of(double v) { return v > 0 ? 1 : (v < 0 ? -1 : 0); }

// appendix `intersects(P, C, seg0, seg1)`: the plane of triangle P cuts triangle C
template <class S>
void intersects(const V3<S> P[3], const V3<S> C[3], const Tri& tp, const Tri& tc, const Cut& cut, V3<S> seg[2]) {
  V3<S> n = cross(P[1] - P[0], P[2] - P[0]);
  S len = dsqrt(dot(n, n));
  V3<S> nh = div(n, len);
  S d[3];
  for (int i = 0; i < 3; ++i) {
    d[i] = dot(nh, C[i] - P[i]);
    if (sign_of(val(d[i])) != cut.s[i]) {
      // FP64 rounding put the vertex on the wrong side: use the exact distance instead
      Dyadic e = orient(to_dy(tp.p[0]), to_dy(tp.p[1]), to_dy(tp.p[2]), to_dy(tc.p[i]));
      set_val(d[i], to_double(e) / val(len));
    }
  }
  seg[0] = seg_point(cut, 0, C, d);
  seg[1] = seg_point(cut, 1, C, d);
}

// sign of t(endpoint 1) - t(endpoint 0) of a cut along D = n_a x n_b, from the exact sides.
// For T_a cut by the plane of T_b, write E1 - E0 = mu D; within the plane of T_a the 2D cross
// product with the edge e1 = k1 - k gives mu (n_a.(e1 x D)) = lambda n_a.(e1 x e2) with
// lambda > 0, and n_a.(e1 x D) = |n_a|^2 (n_b.e1), whose sign is the side of k1 (k lies on the
// other side or on the plane).  For T_b the same steps give the opposite sign.
int seg_order(const Cut& c, bool cut_of_b) {
  const int k = c.p[0];
  const int k1 = c.q[0] >= 0 ? c.q[0] : c.p[1];
  const int orientation = ((k1 - k + 3) % 3 == 1) ? 1 : -1;  // (k, k1, k2) cyclic in the triangle
  const int o = orientation * c.s[k1];
  return cut_of_b ? -o : o;
}

template <class S>
bool interval_ends(const V3<S> U[3], const V3<S> V[3], const Tri& ta, const Tri& tb, const Cut& ca,
                   const Cut& cb, double half, S& tc0, S& tc1) {
  V3<S> Sa[2], Sb[2];
  intersects(V, U, tb, ta, ca, Sa);   // T_a's segment on the plane of T_b
  intersects(U, V, ta, tb, cb, Sb);   // T_b's segment on the plane of T_a
  V3<S> un = cross(U[1] - U[0], U[2] - U[0]);
  V3<S> vn = cross(V[1] - V[0], V[2] - V[0]);
  V3<S> D = cross(un, vn);
  // The line frame is undefined only when the FP64 direction is exactly (0, 0, 0).  Otherwise
  // D is first multiplied by 2^-e, e the exponent of its largest component: an exact scaling
  // (in two factors, so that neither over- nor underflows) that leaves D/|D| unchanged and
  // keeps |D|^2 finite and non-zero over the whole coordinate domain.
  const double m = std::max(std::fabs(val(D.x)), std::max(std::fabs(val(D.y)), std::fabs(val(D.z))));
  if (!(m > 0.0)) return false;
  const int e = std::ilogb(m);
  D = scale(std::ldexp(1.0, -(e / 2)), D);
  D = scale(std::ldexp(1.0, -(e - e / 2)), D);
  S len = dsqrt(dot(D, D));
  D = div(D, len);
  V3<S> A = scale(0.25, Sa[0] + Sa[1] + Sb[0] + Sb[1]);
  S t00 = dot(D, Sa[0] - A), t01 = dot(D, Sa[1] - A);
  S t10 = dot(D, Sb[0] - A), t11 = dot(D, Sb[1] - A);
  const bool a_up = seg_order(ca, false) > 0;  // t(Sa[1]) > t(Sa[0])
  const bool b_up = seg_order(cb, true) > 0;
  S ta0 = a_up ? t00 : t01, ta1 = a_up ? t01 : t00;
  S tb0 = b_up ? t10 : t11, tb1 = b_up ? t11 : t10;
  tc0 = half * (ta0 - tb1);
  tc1 = half * (ta1 - tb0);
  return true;
}

// ============================================================================================
// Per-pair evaluation
// ============================================================================================
enum { ST_NONE = 0, ST_HIT = 1, ST_ADJACENT = 2, ST_BAD_FRAME = 3, ST_COPLANAR = 4 };
enum { PSD_PER_PART = 0, PSD_NEAREST = 1, PSD_PAPER_LITERAL = 2, PSD_RAW_EQ4 = 3 };

struct Classified {
  int status = ST_NONE;
  Cut ca, cb;
};

// ============================================================================================
// Coplanar overlap.  When every vertex of T_a lies on the plane of T_b (and T_b has area) the
// two triangles share one plane; Moeller's reduction yields no segment and the energy is 0.
// Their interiors overlap exactly when no edge line separates them: for two convex polygons
// with disjoint interiors some line through an edge of one of them leaves the other in its
// closed outer half-plane.  Decided in exact arithmetic after dropping a coordinate that
// keeps the triangles' area (the exact normal of T_a has a non-zero component there).
// ============================================================================================
// 2D orientation of (a, b, c) with coordinate k dropped, exactly
int orient2_exact(const double* a, const double* b, const double* c, int k) {
  const int u = (k + 1) % 3, v = (k + 2) % 3;
  const Dyadic r = (dy(b[u]) - dy(a[u])) * (dy(c[v]) - dy(a[v])) - (dy(b[v]) - dy(a[v])) * (dy(c[u]) - dy(a[u]));
  return sgn(r);
}

bool coplanar_overlap(const Tri& ta, const Tri& tb) {
  int k = 0, sa = 0;
  while (k < 3 && (sa = orient2_exact(ta.p[0], ta.p[1], ta.p[2], k)) == 0) ++k;
  if (sa == 0) return false;  // T_a has no area
  const int sb = orient2_exact(tb.p[0], tb.p[1], tb.p[2], k);
  if (sb == 0) return false;  // T_b has no area
  for (int side = 0; side < 2; ++side) {
    const Tri& P = side == 0 ? ta : tb;
    const Tri& Q = side == 0 ? tb : ta;
    const int sp = side == 0 ? sa : sb;  // P's interior lies where the edge orientation has sign sp
    for (int e = 0; e < 3; ++e) {
      bool separates = true;
      for (int j = 0; j < 3; ++j)
        if (sp * orient2_exact(P.p[e], P.p[(e + 1) % 3], Q.p[j], k) > 0) separates = false;
      if (separates) return false;
    }
  }
  return true;
}

// exact classification: straddle tests for both cuts, then the exact interval-overlap flag
Classified classify_pair(const Tri& ta, const Tri& tb) {
  Classified r;
  int s[3];
  for (int k = 0; k < 3; ++k) s[k] = side(tb.p[0], tb.p[1], tb.p[2], ta.p[k]).sign;
  if (s[0] == 0 && s[1] == 0 && s[2] == 0) {
    if (coplanar_overlap(ta, tb)) r.status = ST_COPLANAR;
    return r;
  }
  r.ca = classify(s);
  if (!r.ca.straddle) return r;
  for (int k = 0; k < 3; ++k) s[k] = side(ta.p[0], ta.p[1], ta.p[2], tb.p[k]).sign;
  r.cb = classify(s);
  if (!r.cb.straddle) return r;
  int sig[2][2];
  endpoint_order(ta, tb, r.ca, r.cb, sig);
  if (exact_flag(sig)) r.status = ST_HIT;
  return r;
}

using D18 = Dual<double, 18>;
using DD18 = Dual<Dual<double, 1>, 18>;

struct PairOut {
  int status = ST_NONE;
  double t0 = 0, t1 = 0, T = 0;
  double a[18] = {}, b[18] = {}, g[18] = {};
};

PairOut eval_pair(const Tri& ta, const Tri& tb, double half) {
  PairOut o;
  Classified c = classify_pair(ta, tb);
  o.status = c.status;
  if (c.status != ST_HIT) return o;
  V3<D18> U[3], V[3];
  for (int k = 0; k < 3; ++k) {
    const double* pu = ta.p[k];
    const double* pv = tb.p[k];
    D18* cu[3] = {&U[k].x, &U[k].y, &U[k].z};
    D18* cv[3] = {&V[k].x, &V[k].y, &V[k].z};
    for (int c3 = 0; c3 < 3; ++c3) {
      cu[c3]->v = pu[c3];
      cu[c3]->d[3 * k + c3] = 1.0;
      cv[c3]->v = pv[c3];
      cv[c3]->d[9 + 3 * k + c3] = 1.0;
    }
  }
  D18 tc0, tc1;
  if (!interval_ends(U, V, ta, tb, c.ca, c.cb, half, tc0, tc1)) {
    o.status = ST_BAD_FRAME;
    return o;
  }
  D18 p = tc0 * tc1;
  D18 T = p * p;                                   // Eq. 2
  o.t0 = tc0.v;
  o.t1 = tc1.v;
  o.T = T.v;
  for (int k = 0; k < 18; ++k) {
    o.a[k] = tc0.d[k];
    o.b[k] = tc1.d[k];
    o.g[k] = T.d[k];
  }
  return o;
}

// exact Hessian-vector product of T for one hit pair: forward-over-forward nested duals
bool hvp_pair(const Tri& ta, const Tri& tb, double half, const double v18[18], double out[18]) {
  Classified c = classify_pair(ta, tb);
  for (int k = 0; k < 18; ++k) out[k] = 0.0;
  if (c.status != ST_HIT) return false;
  V3<DD18> U[3], V[3];
  for (int k = 0; k < 3; ++k) {
    DD18* cu[3] = {&U[k].x, &U[k].y, &U[k].z};
    DD18* cv[3] = {&V[k].x, &V[k].y, &V[k].z};
    for (int c3 = 0; c3 < 3; ++c3) {
      cu[c3]->v.v = ta.p[k][c3];
      cu[c3]->v.d[0] = v18[3 * k + c3];
      cu[c3]->d[3 * k + c3].v = 1.0;
      cv[c3]->v.v = tb.p[k][c3];
      cv[c3]->v.d[0] = v18[9 + 3 * k + c3];
      cv[c3]->d[9 + 3 * k + c3].v = 1.0;
    }
  }
  DD18 tc0, tc1;
  if (!interval_ends(U, V, ta, tb, c.ca, c.cb, half, tc0, tc1)) return false;
  DD18 p = tc0 * tc1;
  DD18 T = p * p;
  for (int k = 0; k < 18; ++k) out[k] = T.d[k].d[0];
  return true;
}

// ============================================================================================
// Symmetric eigen-decomposition by cyclic Jacobi rotations (dense n x n, n <= 18).
// ============================================================================================
void jacobi_eig(int n, double* A /*n*n, destroyed*/, double* w, double* Q /*n*n columns*/) {
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) Q[i * n + j] = i == j ? 1.0 : 0.0;
  double fro = 0;
  for (int i = 0; i < n * n; ++i) fro += A[i] * A[i];
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off <= 1e-34 * fro || off == 0.0) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {   // columns p, q
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {   // rows p, q
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
        for (int k = 0; k < n; ++k) {
          double qkp = Q[k * n + p], qkq = Q[k * n + q];
          Q[k * n + p] = c * qkp - s * qkq;
          Q[k * n + q] = s * qkp + c * qkq;
        }
      }
  }
  for (int i = 0; i < n; ++i) w[i] = A[i * n + i];
}

// replace M (18x18 symmetric) by Q max(L, 0) Q^T
void project_psd(double* M) {
  double A[324], w[18], Q[324];
  std::memcpy(A, M, sizeof(A));
  jacobi_eig(18, A, w, Q);
  for (int i = 0; i < 18; ++i)
    for (int j = 0; j < 18; ++j) {
      double s = 0;
      for (int k = 0; k < 18; ++k)
        if (w[k] > 0) s += Q[i * 18 + k] * w[k] * Q[j * 18 + k];
      M[i * 18 + j] = s;
    }
}

// Eq. 4 and its variants as a dense 18x18 matrix, following the three-part split of the
// eigenanalysis in Sec. 1.1
void pair_hessian(const PairOut& o, int psd_mode, double* H) {
  const double t0 = o.t0, t1 = o.t1;
  double P1[324], P2[324], P3[324];
  for (int i = 0; i < 18; ++i)
    for (int j = 0; j < 18; ++j) {
      P1[i * 18 + j] = 2.0 * t1 * t1 * o.a[i] * o.a[j];
      P2[i * 18 + j] = 2.0 * t0 * t0 * o.b[i] * o.b[j];
      P3[i * 18 + j] = 4.0 * t0 * t1 * (o.b[i] * o.a[j] + o.a[i] * o.b[j]);
    }
  if (psd_mode == PSD_PER_PART) project_psd(P3);
  if (psd_mode == PSD_PAPER_LITERAL) {
    double ab = 0;
    for (int k = 0; k < 18; ++k) ab += o.a[k] * o.b[k];
    if (!(8.0 * t0 * t1 * ab > 0.0))
      for (double& x : P3) x = 0.0;
  }
  for (int i = 0; i < 324; ++i) H[i] = P1[i] + P2[i] + P3[i];
  if (psd_mode == PSD_NEAREST) project_psd(H);
}

// ============================================================================================
// Whole-problem evaluation and assembly
// ============================================================================================
struct Mesh {
  const double* x;
  int64_t nv;
  const int32_t* tris;
  int64_t nt;
  Tri tri(int64_t t) const {
    return {{x + 3 * (int64_t)tris[3 * t], x + 3 * (int64_t)tris[3 * t + 1], x + 3 * (int64_t)tris[3 * t + 2]}};
  }
  // Pairs sharing a vertex index are "adjacent" (Sec. 1) and carry no energy.  With
  // vertex_adjacent set, a pair sharing exactly one vertex is evaluated like any other (the
  // shared vertex lies exactly on both planes); pairs sharing an edge stay adjacent.
  bool vertex_adjacent = false;
  int shared(int64_t i, int64_t j) const {  // distinct vertex ids of triangle i found in triangle j
    int n = 0;
    for (int a = 0; a < 3; ++a) {
      const int32_t v = tris[3 * i + a];
      bool dup = false;
      for (int a2 = 0; a2 < a; ++a2) dup = dup || tris[3 * i + a2] == v;
      if (dup) continue;
      for (int b = 0; b < 3; ++b)
        if (tris[3 * j + b] == v) {
          ++n;
          break;
        }
    }
    return n;
  }
  bool adjacent(int64_t i, int64_t j) const {
    const int n = shared(i, j);
    return n >= 2 || (n == 1 && !vertex_adjacent);
  }
};

struct HitRec {
  int64_t pair;
  int32_t vid[6];
  PairOut o;
  std::vector<double> H;   // 18x18
};

struct EvalResult {
  std::vector<uint8_t> flags;
  std::vector<double> tpair, Tpair;
  std::vector<HitRec> hits;
  double E = 0;
  std::vector<double> G;
  std::vector<int32_t> row_ptr, col_idx;
  std::vector<double> vals;
  int error = 0;
};

int n_threads_or_default(int n) {
#ifdef _OPENMP
  return n > 0 ? n : omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

EvalResult* evaluate(const Mesh& m, const int32_t* pairs, int64_t np, int interval_mode, int psd_mode,
                     int want_hessian, int nthreads) {
  auto* R = new EvalResult;
  const double half = interval_mode == 1 ? 0.5 : 1.0;
  R->flags.assign(np, 0);
  R->tpair.assign(2 * np, 0.0);
  R->Tpair.assign(np, 0.0);
  for (int64_t p = 0; p < np; ++p) {
    int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
    if (i < 0 || j < 0 || i >= m.nt || j >= m.nt || i == j) {
      R->error = 1;
      return R;
    }
  }
  int nth = n_threads_or_default(nthreads);
  std::vector<std::vector<HitRec>> local(nth);
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nth)
  for (int64_t p = 0; p < np; ++p) {
    int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
    if (m.adjacent(i, j)) {
      R->flags[p] = ST_ADJACENT;
      continue;
    }
    PairOut o = eval_pair(m.tri(i), m.tri(j), half);
    R->flags[p] = (uint8_t)o.status;
    if (o.status != ST_HIT) continue;
    R->tpair[2 * p] = o.t0;
    R->tpair[2 * p + 1] = o.t1;
    R->Tpair[p] = o.T;
    HitRec h;
    h.pair = p;
    for (int k = 0; k < 3; ++k) {
      h.vid[k] = m.tris[3 * i + k];
      h.vid[3 + k] = m.tris[3 * j + k];
    }
    h.o = o;
    if (want_hessian) {
      h.H.assign(324, 0.0);
      pair_hessian(o, psd_mode, h.H.data());
    }
#ifdef _OPENMP
    local[omp_get_thread_num()].push_back(std::move(h));
#else
    local[0].push_back(std::move(h));
#endif
  }
  for (auto& l : local)
    for (auto& h : l) R->hits.push_back(std::move(h));
  std::sort(R->hits.begin(), R->hits.end(), [](const HitRec& a, const HitRec& b) { return a.pair < b.pair; });

  // energy: plain sum over the pair list in order (Eq. 2 summed over all candidate pairs)
  double E = 0;
  for (int64_t p = 0; p < np; ++p) E += R->Tpair[p];
  R->E = E;
  // gradient: each hit's 18-vector added to its six vertices
  R->G.assign(3 * m.nv, 0.0);
  for (const auto& h : R->hits)
    for (int k = 0; k < 6; ++k)
      for (int c = 0; c < 3; ++c) R->G[3 * h.vid[k] + c] += h.o.g[3 * k + c];
  // Hessian: 3x3 blocks keyed by (row vertex, column vertex), full symmetric storage
  if (want_hessian) {
    std::map<std::pair<int32_t, int32_t>, std::array<double, 9>> blocks;
    for (const auto& h : R->hits)
      for (int k = 0; k < 6; ++k)
        for (int l = 0; l < 6; ++l) {
          auto& B = blocks[{h.vid[k], h.vid[l]}];
          for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) B[3 * r + c] += h.H[(3 * k + r) * 18 + (3 * l + c)];
        }
    R->row_ptr.assign(m.nv + 1, 0);
    for (const auto& kv : blocks) R->row_ptr[kv.first.first + 1]++;
    for (int64_t v = 0; v < m.nv; ++v) R->row_ptr[v + 1] += R->row_ptr[v];
    for (const auto& kv : blocks) {   // std::map iterates rows, then columns, ascending
      R->col_idx.push_back(kv.first.second);
      for (double x : kv.second) R->vals.push_back(x);
    }
  }
  return R;
}

// ============================================================================================
// Broad phase: the canonical candidate set {(i, j) : i < j, no shared vertex index, and (for
// the box method) closed FP64 bounding boxes overlapping on all three axes}.
// ============================================================================================
std::vector<int32_t> pairs_brute(const Mesh& m) {
  std::vector<int32_t> out;
  for (int64_t i = 0; i < m.nt; ++i)
    for (int64_t j = i + 1; j < m.nt; ++j)
      if (!m.adjacent(i, j)) {
        out.push_back((int32_t)i);
        out.push_back((int32_t)j);
      }
  return out;
}

// x_end (nullable): boxes cover each triangle at x and at x_end (swept candidates)
std::vector<int32_t> pairs_boxes(const Mesh& m, const double* x_end = nullptr) {
  std::vector<double> lo(3 * m.nt), hi(3 * m.nt);
  double ext = 0;
  for (int64_t t = 0; t < m.nt; ++t) {
    Tri tr = m.tri(t);
    for (int c = 0; c < 3; ++c) {
      lo[3 * t + c] = std::min({tr.p[0][c], tr.p[1][c], tr.p[2][c]});
      hi[3 * t + c] = std::max({tr.p[0][c], tr.p[1][c], tr.p[2][c]});
      if (x_end)
        for (int k = 0; k < 3; ++k) {
          const double e = x_end[3 * (int64_t)m.tris[3 * t + k] + c];
          lo[3 * t + c] = std::min(lo[3 * t + c], e);
          hi[3 * t + c] = std::max(hi[3 * t + c], e);
        }
      ext = std::max(ext, hi[3 * t + c] - lo[3 * t + c]);
    }
  }
  if (m.nt == 0) return {};
  // uniform grid with cells as large as the largest box extent: overlapping boxes share a cell
  double h = ext > 0 ? ext : 1.0;
  double org[3] = {lo[0], lo[1], lo[2]};
  for (int64_t t = 0; t < m.nt; ++t)
    for (int c = 0; c < 3; ++c) org[c] = std::min(org[c], lo[3 * t + c]);
  std::vector<std::pair<int64_t, int32_t>> cells;
  for (int64_t t = 0; t < m.nt; ++t) {
    int64_t a[3], b[3];
    for (int c = 0; c < 3; ++c) {
      a[c] = (int64_t)std::floor((lo[3 * t + c] - org[c]) / h);
      b[c] = (int64_t)std::floor((hi[3 * t + c] - org[c]) / h);
    }
    for (int64_t x = a[0]; x <= b[0]; ++x)
      for (int64_t y = a[1]; y <= b[1]; ++y)
        for (int64_t z = a[2]; z <= b[2]; ++z)
          cells.push_back({(x * 2097152 + y) * 2097152 + z, (int32_t)t});
  }
  std::sort(cells.begin(), cells.end());
  std::vector<std::pair<int32_t, int32_t>> cand;
  for (size_t s = 0; s < cells.size();) {
    size_t e = s;
    while (e < cells.size() && cells[e].first == cells[s].first) ++e;
    for (size_t u = s; u < e; ++u)
      for (size_t w = u + 1; w < e; ++w) {
        int32_t i = cells[u].second, j = cells[w].second;
        if (i > j) std::swap(i, j);
        bool ov = true;
        for (int c = 0; c < 3; ++c)
          ov = ov && lo[3 * i + c] <= hi[3 * j + c] && lo[3 * j + c] <= hi[3 * i + c];
        if (ov && !m.adjacent(i, j)) cand.push_back({i, j});
      }
    s = e;
  }
  std::sort(cand.begin(), cand.end());
  cand.erase(std::unique(cand.begin(), cand.end()), cand.end());
  std::vector<int32_t> out;
  out.reserve(2 * cand.size());
  for (auto& pq : cand) {
    out.push_back(pq.first);
    out.push_back(pq.second);
  }
  return out;
}

// ============================================================================================
// Inexact Newton loop (the abstract's optimization route; its parameters are not given in
// the paper): H = the PSD Hessian, (H + mu I) d = -g by Jacobi-preconditioned CG from d = 0
// with mu = mu_rel * mean diagonal entry over the rows holding blocks, then Armijo
// backtracking on E along d with candidates from boxes swept from x to x + d.
// ============================================================================================
struct NewtonParams {
  int steps, pcg_iters;
  double pcg_tol, mu_rel, armijo_c, beta;
  int max_halvings, interval_mode, psd_mode, nthreads;
};

void bsr_apply(const EvalResult& R, int64_t nv, const std::vector<double>& v, double mu, std::vector<double>& out) {
  for (int64_t r = 0; r < nv; ++r)
    for (int a = 0; a < 3; ++a) {
      double acc = mu * v[3 * r + a];
      for (int32_t k = R.row_ptr[r]; k < R.row_ptr[r + 1]; ++k)
        for (int b = 0; b < 3; ++b) acc += R.vals[9 * (size_t)k + 3 * a + b] * v[3 * (size_t)R.col_idx[k] + b];
      out[3 * r + a] = acc;
    }
}

double dotv(const std::vector<double>& a, const std::vector<double>& b) {
  double s = 0;
  for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
  return s;
}

// Positions stay in the coordinate domain of the exact predicates (0, or magnitude in
// [2^-200, 2^200]): a trial coordinate of smaller magnitude (a far vertex reached by a
// truncated solve with a vanishing component) is set to 0.
double flush_tiny(double v) { return std::fabs(v) < 0x1p-200 ? 0.0 : v; }

int newton(double* x, int64_t nv, const int32_t* tris, int64_t nt, const NewtonParams& P, double* energies,
           double* alphas, int* pcg_iters_out) {
  int done = 0;
  std::vector<double> xt(3 * nv);
  for (int k = 0; k < P.steps; ++k) {
    Mesh m{x, nv, tris, nt};
    std::vector<int32_t> pl = pairs_boxes(m);
    EvalResult* R = evaluate(m, pl.data(), (int64_t)pl.size() / 2, P.interval_mode, P.psd_mode, 1, P.nthreads);
    const double E = R->E;
    energies[k] = E;
    if (E == 0.0) {
      delete R;
      done = k;
      for (int j = k; j <= P.steps; ++j) energies[j] = 0.0;
      return done;
    }
    // Jacobi-PCG on (H + mu I) d = -g
    double dsum = 0, dcnt = 0;
    std::vector<double> diag(3 * nv, 0.0);
    for (int64_t r = 0; r < nv; ++r)
      for (int32_t q = R->row_ptr[r]; q < R->row_ptr[r + 1]; ++q)
        if (R->col_idx[q] == r)
          for (int a = 0; a < 3; ++a) {
            diag[3 * r + a] = R->vals[9 * (size_t)q + 4 * a];
            dsum += diag[3 * r + a];
            dcnt += 1;
          }
    const double mu = P.mu_rel * (dcnt > 0 ? dsum / dcnt : 1.0);
    std::vector<double> b(3 * nv), d(3 * nv, 0.0), r(3 * nv), z(3 * nv), p(3 * nv), q(3 * nv), dinv(3 * nv);
    for (int64_t i = 0; i < 3 * nv; ++i) {
      b[i] = -R->G[i];
      const double dg = diag[i] + mu;
      dinv[i] = dg > 0 ? 1.0 / dg : 1.0;
      r[i] = b[i];
      z[i] = dinv[i] * r[i];
      p[i] = z[i];
    }
    double rz = dotv(r, z);
    const double bb = dotv(b, b);
    int it = 0;
    for (; it < P.pcg_iters; ++it) {
      bsr_apply(*R, nv, p, mu, q);
      const double pq = dotv(p, q);
      if (!(pq > 0)) break;
      const double alpha = rz / pq;
      for (int64_t i = 0; i < 3 * nv; ++i) {
        d[i] += alpha * p[i];
        r[i] -= alpha * q[i];
        z[i] = dinv[i] * r[i];
      }
      const double rzn = dotv(r, z), rr = dotv(r, r);
      if (rr <= P.pcg_tol * P.pcg_tol * bb) {
        ++it;
        break;
      }
      const double beta = rz > 0 ? rzn / rz : 0.0;
      for (int64_t i = 0; i < 3 * nv; ++i) p[i] = z[i] + beta * p[i];
      rz = rzn;
    }
    if (pcg_iters_out) pcg_iters_out[k] = it;
    double gd = 0;
    for (int64_t i = 0; i < 3 * nv; ++i) gd += R->G[i] * d[i];
    delete R;
    // Armijo backtracking with candidates swept from x to x + d
    std::vector<double> xe(3 * nv);
    for (int64_t i = 0; i < 3 * nv; ++i) xe[i] = flush_tiny(x[i] + d[i]);
    std::vector<int32_t> sw = pairs_boxes(m, xe.data());
    double alpha = 1.0;
    for (int h = 0; h < P.max_halvings; ++h) {
      for (int64_t i = 0; i < 3 * nv; ++i) xt[i] = flush_tiny(x[i] + alpha * d[i]);
      Mesh mt{xt.data(), nv, tris, nt};
      EvalResult* Rt = evaluate(mt, sw.data(), (int64_t)sw.size() / 2, P.interval_mode, P.psd_mode, 0, P.nthreads);
      const double Et = Rt->E;
      delete Rt;
      if (Et <= E + P.armijo_c * alpha * gd) break;
      if (h + 1 < P.max_halvings) alpha *= P.beta;
    }
    if (alphas) alphas[k] = alpha;
    for (int64_t i = 0; i < 3 * nv; ++i) x[i] = xt[i];
    done = k + 1;
  }
  Mesh m{x, nv, tris, nt};
  std::vector<int32_t> pl = pairs_boxes(m);
  EvalResult* R = evaluate(m, pl.data(), (int64_t)pl.size() / 2, P.interval_mode, P.psd_mode, 0, P.nthreads);
  energies[P.steps] = R->E;
  delete R;
  return done;
}

}  // namespace

// ============================================================================================
// C entry points (ctypes)
// ============================================================================================
extern "C" {

// threads the parallel loops use by default
int ttie_oracle_threads(void) { return n_threads_or_default(0); }

// exact sign of det[b-a, c-a, p-a]
int ttie_oracle_orient_sign(const double* a, const double* b, const double* c, const double* p) {
  return side(a, b, c, p).sign;
}

// single pair: X = (u0,u1,u2,v0,v1,v2) coordinates; returns the status
int ttie_oracle_pair(const double* X, int interval_mode, int psd_mode, double* t01, double* T, double* a,
                     double* b, double* g, double* H) {
  Tri ta{{X, X + 3, X + 6}}, tb{{X + 9, X + 12, X + 15}};
  PairOut o = eval_pair(ta, tb, interval_mode == 1 ? 0.5 : 1.0);
  if (t01) { t01[0] = o.t0; t01[1] = o.t1; }
  if (T) *T = o.T;
  for (int k = 0; k < 18; ++k) {
    if (a) a[k] = o.a[k];
    if (b) b[k] = o.b[k];
    if (g) g[k] = o.g[k];
  }
  if (H) {
    if (o.status == ST_HIT) pair_hessian(o, psd_mode, H);
    else std::memset(H, 0, 324 * sizeof(double));
  }
  return o.status;
}

int ttie_oracle_pair_hvp(const double* X, int interval_mode, const double* v, double* out) {
  Tri ta{{X, X + 3, X + 6}}, tb{{X + 9, X + 12, X + 15}};
  return hvp_pair(ta, tb, interval_mode == 1 ? 0.5 : 1.0, v, out) ? 1 : 0;
}

void ttie_oracle_eig(int n, const double* A, double* w, double* Q) {
  std::vector<double> tmp(A, A + n * n);
  jacobi_eig(n, tmp.data(), w, Q);
}

int32_t* ttie_oracle_pairs(const double* x, int64_t nv, const int32_t* tris, int64_t nt, int method,
                           int vertex_adjacent, int64_t* n_out) {
  Mesh m{x, nv, tris, nt};
  m.vertex_adjacent = vertex_adjacent != 0;
  std::vector<int32_t> p = method == 0 ? pairs_brute(m) : pairs_boxes(m);
  *n_out = (int64_t)(p.size() / 2);
  int32_t* out = (int32_t*)std::malloc(std::max<size_t>(1, p.size()) * sizeof(int32_t));
  if (!p.empty()) std::memcpy(out, p.data(), p.size() * sizeof(int32_t));
  return out;
}

void ttie_oracle_free(void* p) { std::free(p); }

// candidates with boxes swept from x to x_end
int32_t* ttie_oracle_pairs_swept(const double* x, const double* x_end, int64_t nv, const int32_t* tris, int64_t nt,
                                 int64_t* n_out) {
  Mesh m{x, nv, tris, nt};
  std::vector<int32_t> p = pairs_boxes(m, x_end);
  *n_out = (int64_t)(p.size() / 2);
  int32_t* out = (int32_t*)std::malloc(std::max<size_t>(1, p.size()) * sizeof(int32_t));
  if (!p.empty()) std::memcpy(out, p.data(), p.size() * sizeof(int32_t));
  return out;
}

// x is updated in place; energies has steps + 1 entries (the last at the final x)
int ttie_oracle_newton(double* x, int64_t nv, const int32_t* tris, int64_t nt, int steps, int pcg_iters,
                       double pcg_tol, double mu_rel, double armijo_c, double beta, int max_halvings,
                       int interval_mode, int psd_mode, int nthreads, double* energies, double* alphas,
                       int* pcg_iters_out) {
  NewtonParams P{steps, pcg_iters, pcg_tol, mu_rel, armijo_c, beta, max_halvings, interval_mode, psd_mode,
                 nthreads};
  return newton(x, nv, tris, nt, P, energies, alphas, pcg_iters_out);
}

void* ttie_oracle_eval(const double* x, int64_t nv, const int32_t* tris, int64_t nt, const int32_t* pairs,
                       int64_t np, int interval_mode, int psd_mode, int want_hessian, int nthreads,
                       int vertex_adjacent) {
  Mesh m{x, nv, tris, nt};
  m.vertex_adjacent = vertex_adjacent != 0;
  return evaluate(m, pairs, np, interval_mode, psd_mode, want_hessian, nthreads);
}

int ttie_oracle_eval_sizes(void* h, int64_t* n_hits, int64_t* nnzb) {
  auto* R = (EvalResult*)h;
  *n_hits = (int64_t)R->hits.size();
  *nnzb = (int64_t)R->col_idx.size();
  return R->error;
}

void ttie_oracle_eval_fetch(void* h, uint8_t* flags, double* tpair, double* Tpair, double* E, double* G,
                            int64_t* hit_pair, double* hit_t, double* hit_a, double* hit_b, double* hit_g,
                            double* hit_H, int32_t* row_ptr, int32_t* col_idx, double* vals) {
  auto* R = (EvalResult*)h;
  size_t np = R->flags.size();
  if (flags) std::memcpy(flags, R->flags.data(), np);
  if (tpair) std::memcpy(tpair, R->tpair.data(), 2 * np * sizeof(double));
  if (Tpair) std::memcpy(Tpair, R->Tpair.data(), np * sizeof(double));
  if (E) *E = R->E;
  if (G) std::memcpy(G, R->G.data(), R->G.size() * sizeof(double));
  for (size_t k = 0; k < R->hits.size(); ++k) {
    const HitRec& r = R->hits[k];
    if (hit_pair) hit_pair[k] = r.pair;
    if (hit_t) { hit_t[2 * k] = r.o.t0; hit_t[2 * k + 1] = r.o.t1; }
    for (int c = 0; c < 18; ++c) {
      if (hit_a) hit_a[18 * k + c] = r.o.a[c];
      if (hit_b) hit_b[18 * k + c] = r.o.b[c];
      if (hit_g) hit_g[18 * k + c] = r.o.g[c];
    }
    if (hit_H && !r.H.empty()) std::memcpy(hit_H + 324 * k, r.H.data(), 324 * sizeof(double));
  }
  if (row_ptr && !R->row_ptr.empty()) std::memcpy(row_ptr, R->row_ptr.data(), R->row_ptr.size() * sizeof(int32_t));
  if (col_idx && !R->col_idx.empty()) std::memcpy(col_idx, R->col_idx.data(), R->col_idx.size() * sizeof(int32_t));
  if (vals && !R->vals.empty()) std::memcpy(vals, R->vals.data(), R->vals.size() * sizeof(double));
}

void ttie_oracle_eval_free(void* h) { delete (EvalResult*)h; }

// Hv summed over the pair list.  mode 0: exact Hessian of the energy (nested duals);
// mode 1: the psd_mode Hessian of the hits (dense 18x18 per pair).
int ttie_oracle_hvp(const double* x, int64_t nv, const int32_t* tris, int64_t nt, const int32_t* pairs,
                    int64_t np, const double* v, int interval_mode, int mode, int psd_mode, double* Hv,
                    int nthreads, int vertex_adjacent) {
  Mesh m{x, nv, tris, nt};
  m.vertex_adjacent = vertex_adjacent != 0;
  const double half = interval_mode == 1 ? 0.5 : 1.0;
  std::memset(Hv, 0, 3 * nv * sizeof(double));
  int nth = n_threads_or_default(nthreads);
  std::vector<std::vector<std::pair<int64_t, std::array<double, 18>>>> local(nth);
#pragma omp parallel for schedule(dynamic, 1024) num_threads(nth)
  for (int64_t p = 0; p < np; ++p) {
    int64_t i = pairs[2 * p], j = pairs[2 * p + 1];
    if (m.adjacent(i, j)) continue;
    int32_t vid[6];
    for (int k = 0; k < 3; ++k) { vid[k] = tris[3 * i + k]; vid[3 + k] = tris[3 * j + k]; }
    double v18[18], out[18];
    for (int k = 0; k < 6; ++k)
      for (int c = 0; c < 3; ++c) v18[3 * k + c] = v[3 * vid[k] + c];
    bool hit;
    if (mode == 0) {
      hit = hvp_pair(m.tri(i), m.tri(j), half, v18, out);
    } else {
      PairOut o = eval_pair(m.tri(i), m.tri(j), half);
      hit = o.status == ST_HIT;
      if (hit) {
        double H[324];
        pair_hessian(o, psd_mode, H);
        for (int r = 0; r < 18; ++r) {
          double s = 0;
          for (int c = 0; c < 18; ++c) s += H[18 * r + c] * v18[c];
          out[r] = s;
        }
      }
    }
    if (!hit) continue;
    std::array<double, 18> o18;
    std::memcpy(o18.data(), out, sizeof(out));
#ifdef _OPENMP
    local[omp_get_thread_num()].push_back({p, o18});
#else
    local[0].push_back({p, o18});
#endif
  }
  std::vector<std::pair<int64_t, std::array<double, 18>>> all;
  for (auto& l : local) all.insert(all.end(), l.begin(), l.end());
  std::sort(all.begin(), all.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
  for (auto& e : all) {
    int64_t i = pairs[2 * e.first], j = pairs[2 * e.first + 1];
    for (int k = 0; k < 6; ++k) {
      int32_t vtx = k < 3 ? tris[3 * i + k] : tris[3 * j + k - 3];
      for (int c = 0; c < 3; ++c) Hv[3 * vtx + c] += e.second[3 * k + c];
    }
  }
  return 0;
}

}  // extern "C"
