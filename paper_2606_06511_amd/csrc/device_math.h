// Small device-side value types: 3-vectors over any scalar and a forward-mode dual number
// (value + one directional tangent) used to differentiate the gradient code along a vector.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ttie {

template <class S>
struct V3 {
  S x, y, z;
};

template <class S> __device__ __forceinline__ V3<S> operator+(const V3<S>& a, const V3<S>& b) {
  return {a.x + b.x, a.y + b.y, a.z + b.z};
}
template <class S> __device__ __forceinline__ V3<S> operator-(const V3<S>& a, const V3<S>& b) {
  return {a.x - b.x, a.y - b.y, a.z - b.z};
}
template <class S> __device__ __forceinline__ V3<S> operator*(const S& s, const V3<S>& a) {
  return {s * a.x, s * a.y, s * a.z};
}
template <class S> __device__ __forceinline__ S dot(const V3<S>& a, const V3<S>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <class S> __device__ __forceinline__ V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// Forward-mode dual number v + d*eps.
template <class T>
struct Dual {
  T v, d;
};
template <class T> __device__ __forceinline__ Dual<T> operator+(Dual<T> a, Dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a, Dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator-(Dual<T> a) { return {-a.v, -a.d}; }
template <class T> __device__ __forceinline__ Dual<T> operator*(Dual<T> a, Dual<T> b) {
  return {a.v * b.v, a.d * b.v + a.v * b.d};
}
template <class T> __device__ __forceinline__ Dual<T> operator/(Dual<T> a, Dual<T> b) {
  T inv = T(1) / b.v;
  return {a.v * inv, (a.d - a.v * inv * b.d) * inv};
}

// Scalar traits: construction from a constant, the value part, square root.
template <class S> struct Sc;
template <> struct Sc<double> {
  __device__ static double c(double x) { return x; }
  __device__ static double val(double x) { return x; }
  __device__ static double sqrt_(double x) { return sqrt(x); }
  // the value is replaced, the (absent) tangent kept
  __device__ static double with_value(double, double v) { return v; }
};
template <> struct Sc<float> {
  __device__ static float c(double x) { return (float)x; }
  __device__ static double val(float x) { return x; }
  __device__ static float sqrt_(float x) { return sqrtf(x); }
  __device__ static float with_value(float, double v) { return (float)v; }
};
template <class T> struct Sc<Dual<T>> {
  __device__ static Dual<T> c(double x) { return {Sc<T>::c(x), T(0)}; }
  __device__ static double val(Dual<T> x) { return Sc<T>::val(x.v); }
  __device__ static Dual<T> sqrt_(Dual<T> x) {
    T r = Sc<T>::sqrt_(x.v);
    return {r, x.d / (T(2) * r)};
  }
  __device__ static Dual<T> with_value(Dual<T> f, double v) { return {Sc<T>::c(v), f.d}; }
};

}  // namespace ttie
