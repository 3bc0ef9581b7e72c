// Forward-mode dual numbers x + x' e (e^2 = 0), used to differentiate the
// pointwise operator D at quadrature points only (paper: the remark after
// Eq. (2) -- forward mode is preferred when D's input and output have the
// same length, and MFEM's own dual-number type is the example).  Templated on
// the real type so the same D runs in FP64 and FP32.
#pragma once
#include <hip/hip_runtime.h>

namespace feod {

template <class T>
struct dual {
  T v;  // value
  T d;  // tangent (directional derivative)
};

template <class T> __device__ __forceinline__ dual<T> operator+(dual<T> a, dual<T> b) { return {a.v + b.v, a.d + b.d}; }
template <class T> __device__ __forceinline__ dual<T> operator-(dual<T> a, dual<T> b) { return {a.v - b.v, a.d - b.d}; }
template <class T> __device__ __forceinline__ dual<T> operator*(dual<T> a, dual<T> b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
template <class T> __device__ __forceinline__ dual<T> operator/(dual<T> a, dual<T> b) {
  T inv = T(1) / b.v;
  return {a.v * inv, (a.d - a.v * inv * b.d) * inv};
}
template <class T> __device__ __forceinline__ dual<T> operator+(dual<T> a, T s) { return {a.v + s, a.d}; }
template <class T> __device__ __forceinline__ dual<T> operator*(dual<T> a, T s) { return {a.v * s, a.d * s}; }
template <class T> __device__ __forceinline__ dual<T> operator*(T s, dual<T> a) { return {a.v * s, a.d * s}; }

// Real-valued overloads so the pointwise code can be written once for T and dual<T>.
__device__ __forceinline__ double fe_pow(double x, double r) { return pow(x, r); }
__device__ __forceinline__ float fe_pow(float x, float r) { return powf(x, r); }

}  // namespace feod
