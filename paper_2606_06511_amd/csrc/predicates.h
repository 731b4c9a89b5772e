// Exact orientation predicate on the GPU.
//
// orient(a, b, c, p) = det[b - a, c - a, p - a] = ((b - a) x (c - a)) . (p - a) is the
// (unnormalised) signed distance of p from the plane through a, b, c.  Its sign decides the
// plane sides of Moeller's reduction (Sec. 1) and -- through the identity used in pair.h --
// the order of the segment endpoints on the intersection line, so all intersection flags
// reduce to signs of this one polynomial of degree 3.
//
// Evaluation: an FP64 semi-static filter first.  With differences, the cross product and
// the dot product rounded in FP64 (eps = 2^-53), every one of the six monomials of the
// determinant passes through at most 8 roundings, so |fl(det) - det| <= gamma_8 * perm with
// perm = sum of |monomials| (computed from the rounded differences; the bound below keeps
// a margin for perm's own rounding).  When |fl(det)| exceeds that bound its sign is exact.
// When perm is exactly 0 every monomial has a zero difference factor (a difference of
// doubles rounds to 0 only when it is 0, and products cannot underflow on the input domain),
// so the determinant is exactly 0.
// Otherwise the determinant is recomputed exactly from the 24 signed triple products of the
// raw coordinates (det[b-a,c-a,p-a] = D(b,c,p) - D(a,b,c) + D(a,b,p) - D(a,c,p) with
// D(x,y,z) = x.(y x z)) in a two's-complement fixed-point accumulator spanning the exponent
// range of those products.  On the documented input domain (every coordinate 0 or of
// magnitude in [2^-200, 2^200]) nothing underflows in the filter and the accumulator
// (kLimbs x 64 bits) always suffices.
#pragma once

#include "device_math.h"

namespace ttie {

constexpr double kEps = 1.1102230246251565e-16;  // 2^-53
constexpr double kOrientErr = 9.0 * kEps;         // > gamma_8 plus the rounding of perm
constexpr int kLimbs = 24;                        // 1536-bit accumulator

struct OrientResult {
  double value;  // FP64 determinant, or the exact one rounded when the filter failed
  int sign;      // exact sign
  int exact;     // 1 if the exact path ran
  int overflow;  // 1 if the exact accumulator was too narrow (outside the input domain)
};

// FP64 determinant and its error bound, from the plane's edge vectors (e1, e2) = (b-a, c-a)
// and w = p - a, all rounded differences.
__device__ __forceinline__ void orient_fp64(const V3<double>& e1, const V3<double>& e2, const V3<double>& w,
                                            double& det, double& bound) {
  V3<double> n = cross(e1, e2);
  det = dot(n, w);
  const double nx = fabs(e1.y * e2.z) + fabs(e1.z * e2.y);
  const double ny = fabs(e1.z * e2.x) + fabs(e1.x * e2.z);
  const double nz = fabs(e1.x * e2.y) + fabs(e1.y * e2.x);
  bound = kOrientErr * (nx * fabs(w.x) + ny * fabs(w.y) + nz * fabs(w.z));
}

// |x| = m * 2^e with an integer mantissa m (53 bits for normal numbers)
struct Mant {
  uint64_t m;
  int e;
  int s;
};

__device__ __forceinline__ Mant decompose(double x) {
  const uint64_t bits = (uint64_t)__double_as_longlong(x);
  const int ef = (int)((bits >> 52) & 0x7ff);
  const uint64_t frac = bits & ((1ull << 52) - 1);
  Mant r;
  r.s = x > 0 ? 1 : (x < 0 ? -1 : 0);
  if (ef == 0) {
    r.m = frac;
    r.e = -1074;
  } else {
    r.m = frac | (1ull << 52);
    r.e = ef - 1075;
  }
  return r;
}

// exact determinant sign (and a rounded value) by fixed-point accumulation
__device__ __noinline__ OrientResult orient_exact(const double* a, const double* b, const double* c,
                                                   const double* p) {
  // D(b,c,p) - D(a,b,c) + D(a,b,p) - D(a,c,p); D(x,y,z) = sum over permutations (i,j,k) of
  // sgn * x_i y_j z_k
  const double* trip[4][3] = {{b, c, p}, {a, b, c}, {a, b, p}, {a, c, p}};
  const int tsgn[4] = {1, -1, 1, -1};
  const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 2, 0}, {1, 0, 2}, {2, 0, 1}, {2, 1, 0}};
  const int psgn[6] = {1, -1, 1, -1, 1, -1};

  int emin = 1 << 30, emax = -(1 << 30);
  for (int t = 0; t < 4; ++t)
    for (int q = 0; q < 6; ++q) {
      Mant x = decompose(trip[t][0][perm[q][0]]);
      Mant y = decompose(trip[t][1][perm[q][1]]);
      Mant z = decompose(trip[t][2][perm[q][2]]);
      if (x.s * y.s * z.s == 0) continue;
      const int e = x.e + y.e + z.e;
      emin = min(emin, e);
      emax = max(emax, e);
    }
  OrientResult r{0.0, 0, 1, 0};
  if (emin > emax) return r;  // every monomial is zero
  // products are < 2^159; 24 of them add < 5 bits; one sign bit
  const int bits = emax - emin + 159 + 5 + 1;
  const int nl = (bits + 63) / 64;
  if (nl > kLimbs) {
    r.overflow = 1;
    return r;
  }
  uint64_t acc[kLimbs];
  for (int k = 0; k < kLimbs; ++k) acc[k] = 0;

  for (int t = 0; t < 4; ++t)
    for (int q = 0; q < 6; ++q) {
      Mant x = decompose(trip[t][0][perm[q][0]]);
      Mant y = decompose(trip[t][1][perm[q][1]]);
      Mant z = decompose(trip[t][2][perm[q][2]]);
      const int s = x.s * y.s * z.s * tsgn[t] * psgn[q];
      if (s == 0) continue;
      // 159-bit product as three limbs
      const uint64_t lo = x.m * y.m, hi = __umul64hi(x.m, y.m);
      const uint64_t l0 = lo * z.m, l1 = __umul64hi(lo, z.m);
      const uint64_t h0 = hi * z.m, h1 = __umul64hi(hi, z.m);
      uint64_t p0 = l0, p1 = l1 + h0;
      uint64_t p2 = h1 + (p1 < h0 ? 1 : 0);
      // shift into place
      const int sh = x.e + y.e + z.e - emin;
      const int ls = sh >> 6, bs = sh & 63;
      uint64_t w[4];
      if (bs == 0) {
        w[0] = p0; w[1] = p1; w[2] = p2; w[3] = 0;
      } else {
        w[0] = p0 << bs;
        w[1] = (p1 << bs) | (p0 >> (64 - bs));
        w[2] = (p2 << bs) | (p1 >> (64 - bs));
        w[3] = p2 >> (64 - bs);
      }
      if (s > 0) {
        uint64_t carry = 0;
        for (int k = ls; k < nl; ++k) {
          const uint64_t add = (k - ls < 4) ? w[k - ls] : 0;
          const uint64_t s1 = acc[k] + add;
          const uint64_t c1 = s1 < add ? 1 : 0;
          const uint64_t s2 = s1 + carry;
          const uint64_t c2 = s2 < carry ? 1 : 0;
          acc[k] = s2;
          carry = c1 | c2;
          if (k - ls >= 3 && carry == 0) break;
        }
      } else {
        uint64_t borrow = 0;
        for (int k = ls; k < nl; ++k) {
          const uint64_t sub = (k - ls < 4) ? w[k - ls] : 0;
          const uint64_t d1 = acc[k] - sub;
          const uint64_t b1 = acc[k] < sub ? 1 : 0;
          const uint64_t d2 = d1 - borrow;
          const uint64_t b2 = d1 < borrow ? 1 : 0;
          acc[k] = d2;
          borrow = b1 | b2;
          if (k - ls >= 3 && borrow == 0) break;
        }
      }
    }

  const bool neg = (acc[nl - 1] >> 63) != 0;
  if (neg) {  // magnitude = two's complement negation over the nl limbs
    uint64_t carry = 1;
    for (int k = 0; k < nl; ++k) {
      const uint64_t v = ~acc[k] + carry;
      carry = (carry && v == 0) ? 1 : 0;
      acc[k] = v;
    }
  }
  int top = -1;
  for (int k = nl - 1; k >= 0; --k)
    if (acc[k] != 0) {
      top = k;
      break;
    }
  if (top < 0) return r;  // exactly zero
  r.sign = neg ? -1 : 1;
  // top two limbs give the value to within one part in 2^63
  double mag = (double)acc[top];
  if (top > 0) mag = mag * 18446744073709551616.0 + (double)acc[top - 1];
  const int shift = emin + 64 * (top > 0 ? top - 1 : 0);
  r.value = r.sign * ldexp(mag, shift);
  return r;
}

// Filtered exact orientation of p against the plane (a, b, c).
__device__ __forceinline__ OrientResult orient(const double* a, const double* b, const double* c, const double* p) {
  const V3<double> A{a[0], a[1], a[2]};
  const V3<double> e1 = V3<double>{b[0], b[1], b[2]} - A;
  const V3<double> e2 = V3<double>{c[0], c[1], c[2]} - A;
  const V3<double> w = V3<double>{p[0], p[1], p[2]} - A;
  double det, bound;
  orient_fp64(e1, e2, w, det, bound);
  if (fabs(det) > bound) return {det, det > 0 ? 1 : -1, 0, 0};
  if (bound == 0.0) return {0.0, 0, 0, 0};
  return orient_exact(a, b, c, p);
}

}  // namespace ttie
