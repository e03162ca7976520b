// usp_dual.h -- forward-mode dual numbers for the pathwise adjoint.
//
// Dual<N> carries a value and N partial derivatives.  The scalar chains of
// the cell state and of the relaxation temperatures are short functions of
// a handful of inputs, so their Jacobians are evaluated by running the
// same templated device functions on Dual<N> (one pass, N directions); the
// adjoint kernels then contract those Jacobians with the incoming adjoints.
// Comparisons look at values only, so every branch is the one the FP64
// evaluation takes.
#pragma once
#include "usp_internal.h"

namespace usp {

// the overloads below live in namespace usp; keep the plain double ones
// visible beside them for the code of this namespace
using ::cbrt;
using ::exp;
using ::expm1;
using ::fabs;
using ::fmax;
using ::fmin;
using ::log;
using ::log1p;
using ::pow;
using ::sqrt;

template <int N>
struct Dual {
  double v;
  double d[N];
  __device__ Dual() {}
  __device__ Dual(double x) : v(x) {
#pragma unroll
    for (int k = 0; k < N; ++k) d[k] = 0.0;
  }
  __device__ static Dual var(double x, int k) {
    Dual r(x);
    r.d[k] = 1.0;
    return r;
  }
};

#define USP_DUAL_UNARY(name, val, der)                          \
  template <int N>                                              \
  __device__ __forceinline__ Dual<N> name(const Dual<N>& a) {   \
    Dual<N> r;                                                  \
    r.v = val;                                                  \
    const double g = der;                                       \
    _Pragma("unroll") for (int k = 0; k < N; ++k) r.d[k] = g * a.d[k]; \
    return r;                                                   \
  }

template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a) {
  Dual<N> r;
  r.v = -a.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = -a.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v + b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] + b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v - b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] - b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v * b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = a.d[k] * b.v + a.v * b.d[k];
  return r;
}
template <int N>
__device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, const Dual<N>& b) {
  Dual<N> r;
  r.v = a.v / b.v;
  const double ib = 1.0 / b.v;
#pragma unroll
  for (int k = 0; k < N; ++k) r.d[k] = (a.d[k] - r.v * b.d[k]) * ib;
  return r;
}
template <int N> __device__ __forceinline__ Dual<N> operator+(const Dual<N>& a, double b) { return a + Dual<N>(b); }
template <int N> __device__ __forceinline__ Dual<N> operator+(double a, const Dual<N>& b) { return Dual<N>(a) + b; }
template <int N> __device__ __forceinline__ Dual<N> operator-(const Dual<N>& a, double b) { return a - Dual<N>(b); }
template <int N> __device__ __forceinline__ Dual<N> operator-(double a, const Dual<N>& b) { return Dual<N>(a) - b; }
template <int N> __device__ __forceinline__ Dual<N> operator*(const Dual<N>& a, double b) { return a * Dual<N>(b); }
template <int N> __device__ __forceinline__ Dual<N> operator*(double a, const Dual<N>& b) { return Dual<N>(a) * b; }
template <int N> __device__ __forceinline__ Dual<N> operator/(const Dual<N>& a, double b) { return a / Dual<N>(b); }
template <int N> __device__ __forceinline__ Dual<N> operator/(double a, const Dual<N>& b) { return Dual<N>(a) / b; }

template <int N> __device__ __forceinline__ bool operator<(const Dual<N>& a, const Dual<N>& b) { return a.v < b.v; }
template <int N> __device__ __forceinline__ bool operator>(const Dual<N>& a, const Dual<N>& b) { return a.v > b.v; }
template <int N> __device__ __forceinline__ bool operator<=(const Dual<N>& a, const Dual<N>& b) { return a.v <= b.v; }
template <int N> __device__ __forceinline__ bool operator>=(const Dual<N>& a, const Dual<N>& b) { return a.v >= b.v; }

USP_DUAL_UNARY(sqrt, ::sqrt(a.v), 0.5 / r.v)
USP_DUAL_UNARY(exp, ::exp(a.v), r.v)
USP_DUAL_UNARY(expm1, ::expm1(a.v), r.v + 1.0)
USP_DUAL_UNARY(log, ::log(a.v), 1.0 / a.v)
USP_DUAL_UNARY(log1p, ::log1p(a.v), 1.0 / (1.0 + a.v))
USP_DUAL_UNARY(cbrt, ::cbrt(a.v), 1.0 / (3.0 * r.v * r.v))
USP_DUAL_UNARY(fabs, ::fabs(a.v), a.v < 0.0 ? -1.0 : 1.0)
#undef USP_DUAL_UNARY

template <int N>
__device__ __forceinline__ Dual<N> pow(const Dual<N>& a, const Dual<N>& b) {
  return exp(b * log(a));
}
template <int N>
__device__ __forceinline__ Dual<N> fmin(const Dual<N>& a, const Dual<N>& b) { return b.v < a.v ? b : a; }
template <int N>
__device__ __forceinline__ Dual<N> fmax(const Dual<N>& a, const Dual<N>& b) { return b.v > a.v ? b : a; }

}  // namespace usp
