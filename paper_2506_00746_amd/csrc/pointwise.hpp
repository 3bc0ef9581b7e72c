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

__device__ __forceinline__ double one_like(double) { return 1.0; }
__device__ __forceinline__ float one_like(float) { return 1.0f; }
template <class T> __device__ __forceinline__ dual<T> one_like(dual<T>) { return {T(1), T(0)}; }

template <class S, class T>
__device__ __forceinline__ S apow(S a, T r, int kind) {
  switch (kind) {
    case POW_ZERO: return one_like(a);
    case POW_QUARTER: return fe_sqrt(fe_sqrt(a));
    case POW_HALF: return fe_sqrt(a);
    case POW_ONE: return a;
    default: return fe_pow(a, r);
  }
}

template <class T> __device__ __forceinline__ T value_of(T x) { return x; }
template <class T> __device__ __forceinline__ T value_of(dual<T> x) { return x.v; }

// F = a^r g with a = eps2 + |g|^2; also returns a^r (value) through coef.
template <class S, class T>
__device__ __forceinline__ void flux(const S g[3], T eps2, T r, int kind, S F[3]) {
  S a = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + eps2;
  S c = apow(a, r, kind);
  F[0] = c * g[0];
  F[1] = c * g[1];
  F[2] = c * g[2];
}

// Energy density W(g) = (1/p) a^(p/2) = a * a^r / p and the scalar a^r.
template <class T>
__device__ __forceinline__ void density(const T g[3], T eps2, T r, int kind, T inv_p, T* W, T* coef) {
  T a = g[0] * g[0] + g[1] * g[1] + g[2] * g[2] + eps2;
  T c = apow(a, r, kind);
  *W = a * c * inv_p;
  *coef = c;
}

}  // namespace feod
