// The pointwise operator D of the finite element operator decomposition
// (paper, Fig. 1): at one quadrature point, the regularised p-Laplacian flux
//     F(g) = (eps^2 + |g|^2)^r g,   r = (p-2)/2,
// written once for a generic scalar S (T for the residual, dual<T> for the
// Jacobian action: evaluating F on g + g' e yields J_D g' exactly, Eq. (2)).
#pragma once
#include "dual.hpp"
#include "kernel_api.hpp"

namespace feod {

// a^r for the exponents the p-Laplacian workloads use, by sqrt chains where
// possible; POW_GENERIC falls back to pow() (PowKind is in kernel_api.hpp).

// 1/sqrt(x): the hardware reciprocal square root refined by Newton steps on
// f(y) = 1/y^2 - x (y <- y (3 - x y^2) / 2), two for FP64, none for FP32
// (already within an ulp there).
__device__ __forceinline__ double fe_rsqrt(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = y * (1.5 - hx * y * y);
  y = y * (1.5 - hx * y * y);
  return y;
}
__device__ __forceinline__ float fe_rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }

// 1/x: the hardware reciprocal refined by Newton steps on f(y) = 1/y - x
// (y <- y + y (1 - x y)), two for FP64, one for FP32.  Within about an ulp,
// and a third of the instructions of a correctly rounded division.
__device__ __forceinline__ double fe_rcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
  y = __builtin_fma(y, __builtin_fma(-x, y, 1.0), y);
  return y;
}
__device__ __forceinline__ float fe_rcp(float x) {
  const float y = __builtin_amdgcn_rcpf(x);
  return __builtin_fmaf(y, __builtin_fmaf(-x, y, 1.0f), y);
}

// a^r and, for dual numbers, d(a^r) = r a^(r-1) da, without divisions:
//   r = 1/2:  a^r = a t, t = a^(-1/2);  d = t da / 2
//   r = 1/4:  a^r = s u, s = a t, u = s^(-1/2);  d = a^r t^2 da / 4
// a = 0 happens only with eps = 0 where the gradient vanishes (p >= 2 there).
// Then a^r = 0 for r > 0, and the tangent of F = a^r g tends to 0 (its size
// is at most max(1, p-1) a^r), so both parts are 0; the chains above would
// give 0 * inf = NaN.
template <int PK, class T>
__device__ __forceinline__ T apow(T a, T r) {
  if constexpr (PK == POW_ZERO) return T(1);
  else if constexpr (PK == POW_QUARTER) {
    const T s = a * fe_rsqrt(a);
    const T c = s * fe_rsqrt(s);
    return a > T(0) ? c : T(0);
  } else if constexpr (PK == POW_HALF) {
    const T c = a * fe_rsqrt(a);
    return a > T(0) ? c : T(0);
  } else if constexpr (PK == POW_ONE) return a;
  else return fe_pow(a, r);  // pow(0, r) = 0 for r > 0; r < 0 needs eps > 0
}

template <int PK, class T>
__device__ __forceinline__ dual<T> apow(dual<T> a, T r) {
  if constexpr (PK == POW_ZERO) {
    return {T(1), T(0)};
  } else if constexpr (PK == POW_QUARTER) {
    const T t = fe_rsqrt(a.v);
    const T s = a.v * t;
    const T c = s * fe_rsqrt(s);
    const T d = T(0.25) * c * t * t * a.d;
    return {a.v > T(0) ? c : T(0), a.v > T(0) ? d : T(0)};
  } else if constexpr (PK == POW_HALF) {
    const T t = fe_rsqrt(a.v);
    const T c = a.v * t, d = T(0.5) * t * a.d;
    return {a.v > T(0) ? c : T(0), a.v > T(0) ? d : T(0)};
  } else if constexpr (PK == POW_ONE) {
    return a;
  } else {
    const T pv = fe_pow(a.v, r);
    return {pv, a.v > T(0) ? r * pv / a.v * a.d : T(0)};
  }
}

template <class T> __device__ __forceinline__ T value_of(T x) { return x; }
template <class T> __device__ __forceinline__ T value_of(dual<T> x) { return x.v; }

// F = a^r g with a = eps2 + |g|^2.
template <int PK, class S, class T>
__device__ __forceinline__ void flux(const S g[3], T eps2, T r, S F[3]) {
  S a = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + eps2;
  S c = apow<PK>(a, r);
  F[0] = c * g[0];
  F[1] = c * g[1];
  F[2] = c * g[2];
}

// The tangent of F written out by hand (no dual numbers), for measuring what
// the dual-number evaluation costs: dF = a^r dg + 2 r a^(r-1) (g . dg) g, with
// a^r and 2 r a^(r-1) from the same reciprocal-square-root chains as apow.
template <int PK, class T>
__device__ __forceinline__ void flux_tangent_hand(const T g[3], const T dg[3], T eps2, T r, T dF[3]) {
  const T a = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + eps2;
  const T gd = g[0] * dg[0] + g[1] * dg[1] + g[2] * dg[2];
  T c, k;  // a^r and 2 r a^(r-1); both 0 at a = 0 (eps = 0, zero gradient), see apow
  if constexpr (PK == POW_ZERO) {
    c = T(1);
    k = T(0);
  } else if constexpr (PK == POW_QUARTER) {
    const T t = fe_rsqrt(a), s = a * t;
    c = s * fe_rsqrt(s);
    k = T(0.5) * c * t * t;
    c = a > T(0) ? c : T(0);
    k = a > T(0) ? k : T(0);
  } else if constexpr (PK == POW_HALF) {
    const T t = fe_rsqrt(a);
    c = a > T(0) ? a * t : T(0);
    k = a > T(0) ? t : T(0);
  } else if constexpr (PK == POW_ONE) {
    c = a;
    k = T(2);
  } else {
    c = fe_pow(a, r);
    k = a > T(0) ? T(2) * r * c / a : T(0);
  }
  const T kg = k * gd;
#pragma unroll
  for (int i = 0; i < 3; ++i) dF[i] = c * dg[i] + kg * g[i];
}

// Energy density W(g) = (1/p) a^(p/2) = a * a^r / p and the scalar a^r.
template <int PK, class T>
__device__ __forceinline__ void density(const T g[3], T eps2, T r, T inv_p, T* W, T* coef) {
  T a = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + eps2;
  T c = apow<PK>(a, r);
  *W = a * c * inv_p;
  *coef = c;
}

}  // namespace feod
