// usp_device.h -- device-side building blocks of libusp (gfx950).
#pragma once

#include <math.h>

#include "usp_internal.h"

namespace usp {

// ---------------------------------------------------------------------------
// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11):
// ten rounds of two 32x32->64 products; the key advances by two Weyl
// constants between rounds.  Key = seed, counter = (c0, c1, c2, c3).
// ---------------------------------------------------------------------------
struct U4 {
  uint32_t w[4];
};

// Four floats in global memory.  Loads through a pointer of this type are
// global (not flat) loads even where the compiler has lost track of where
// a generic pointer points (an opaque scalar copy of it, for instance):
// they then count only against the vector-memory counter, so waiting for
// them does not also wait for LDS traffic.
typedef float F4 __attribute__((ext_vector_type(4)));
typedef F4 __attribute__((address_space(1))) GlobalF4;
typedef CellRec __attribute__((address_space(1))) GlobalRec;
typedef CellPCoef __attribute__((address_space(1))) GlobalPCoef;
typedef double __attribute__((address_space(1))) GlobalD;
// p[k] of a cell-state plane, as a global load
__device__ __forceinline__ double ldg(const double* p, int64_t k) { return ((const GlobalD*)p)[k]; }

__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint64_t seed) {
  // The key is the same on every lane: every caller passes its launch's
  // seed.  An opaque scalar copy per call keeps the compiler from hoisting
  // the ten round keys out of the particle loops: hoisted, they overflow
  // the scalar registers and come back by one VALU readlane each;
  // recomputed, they are twenty scalar adds.
  uint32_t k0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)seed);
  uint32_t k1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(seed >> 32));
  asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // one 32x32->64 product per multiplier (a single v_mad_u64_u32)
    const uint64_t p0 = (uint64_t)0xD2511F53u * c0, p1 = (uint64_t)0xCD9E8D57u * c2;
    const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
    const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{{c0, c1, c2, c3}};
}

// uniform (w + 1/2) 2^-32 in (0,1), exact in double
__device__ __forceinline__ double u01d(uint32_t w) { return ((double)w + 0.5) * 0x1p-32; }

// ln u for the same u in single precision.  Below 1 - 2^-7 the hardware
// base-2 logarithm (v_log_f32) of the float u, times ln 2: the rounding of
// u to float (2^-24) dominates, ~4e-6 relative at worst, the same as the
// library logf (both measured against FP64 over 2^24 random words); above
// it ln(1 - v) = -v (1 + v/2 + v^2/3 + v^3/4 + v^4/5) with v = 1 - u formed
// exactly from ~w (truncation below 1e-10 relative).
__device__ __forceinline__ float logu(uint32_t w, float) {
  if (w < 0xFE000000u) return __builtin_amdgcn_logf(((float)w + 0.5f) * 0x1p-32f) * 0.69314718055994531f;
  const float v = ((float)(~w) + 0.5f) * 0x1p-32f;
  return -v * (1.0f + v * (0.5f + v * (1.0f / 3.0f + v * (0.25f + v * 0.2f))));
}
__device__ __forceinline__ double logu(uint32_t w, double) { return log(u01d(w)); }

// (sin, cos)(2 pi u) for the same u
// sin and cos of |x| <= pi/3 by their Taylor series in nested form,
// cos x = 1 - x^2/(1*2) (1 - x^2/(3*4) (1 - ...)) and likewise sin x / x
// with (2*3), (4*5), ...; NT terms leave a truncation below 4e-9 (NT = 5,
// float) or 1e-18 (NT = 9, double) on that interval.
template <typename T, int NT>
__device__ __forceinline__ void sincos_series(T x, T* s, T* c) {
  const T x2 = x * x;
  T cc = T(1), ss = T(1);
#pragma unroll
  for (int k = NT; k >= 1; --k) {
    cc = T(1) - x2 * T(1.0 / double((2 * k - 1) * (2 * k))) * cc;
    ss = T(1) - x2 * T(1.0 / double((2 * k) * (2 * k + 1))) * ss;
  }
  *c = cc;
  *s = x * ss;
}
// In single precision: the quarter turn q nearest to u and the remainder
// u - q/4 in [-1/8, 1/8] turns are formed exactly from w (wrapping 32-bit
// arithmetic); the hardware sine and cosine (v_sin_f32, v_cos_f32 take
// their argument in turns) of the remainder, within 1.3e-7 of FP64 over
// 2^24 random words; then a rotation by q quarter turns.
__device__ __forceinline__ void sincos2pi(uint32_t w, float* s, float* c) {
  const uint32_t q = ((w + 0x20000000u) >> 30) & 3u;
  const int32_t r = (int32_t)(w - (q << 30));
  const float rev = ((float)r + 0.5f) * 0x1p-32f;
  const float st = __builtin_amdgcn_sinf(rev), ct = __builtin_amdgcn_cosf(rev);
  const float a = (q & 1u) ? ct : st, b = (q & 1u) ? st : ct;
  *s = (q == 1u || q == 0u) ? a : -a;
  *c = (q == 0u || q == 3u) ? b : -b;
}
__device__ __forceinline__ void sincos2pi(uint32_t w, double* s, double* c) {
  sincospi(u01d(w) * 2.0, s, c);
}

// a / b for the coefficient chain.  In single precision: a times the
// hardware reciprocal (v_rcp_f32, 1 ulp), within 2 ulp of the quotient for
// |b| between 2^-126 and 2^126 (the chain divides physical quantities far
// inside that range), two instructions where the compiler's denormal-safe
// 2.5-ulp expansion takes eight; in FP64 (and for the dual numbers of the
// adjoint) the division itself.
template <typename T>
__device__ __forceinline__ T qdiv(T a, T b) {
  return a / b;
}
__device__ __forceinline__ float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// two standard normals from two words (Box-Muller)
template <typename T>
__device__ __forceinline__ void box_muller(uint32_t wa, uint32_t wb, T* g1, T* g2) {
  T r = sqrt(T(-2) * logu(wa, T()));
  T s, c;
  sincos2pi(wb, &s, &c);
  *g1 = r * c;
  *g2 = r * s;
}

// ---------------------------------------------------------------------------
// Gas model in reduced units (temperatures in K, energies per R).
// ---------------------------------------------------------------------------
// e^x and e^x - 1 for the gas-model terms.  FP64: the library.  FP32: the
// hardware base-2 exponential (v_exp_f32) of x log2(e), with the rounding of
// the product carried as a first-order correction (x log2 e = t + r exactly
// to FP32 working precision, 2^(t + r) = 2^t (1 + r ln 2)), about 2 ulp;
// e^x - 1 takes the library below |x| = 1, where the subtraction would lose
// bits (above it, at most 1.6x the exponential's relative error).
template <typename T>
__device__ __forceinline__ T gm_exp(T x) { return exp(x); }
template <typename T>
__device__ __forceinline__ T gm_expm1(T x) { return expm1(x); }
template <>
__device__ __forceinline__ float gm_exp<float>(float x) {
  const float hi = 1.44269502162933349609375f, lo = 1.925963033500011e-08f;
  const float t = x * hi;
  const float r = fmaf(x, hi, -t) + x * lo;
  const float e = __builtin_amdgcn_exp2f(t);
  return e * (1.0f + r * 0.693147180559945309f);  // inf stays inf
}
template <>
__device__ __forceinline__ float gm_expm1<float>(float x) {
  if (fabsf(x) < 1.0f) return expm1f(x);
  return gm_exp(x) - 1.0f;
}

// mean harmonic-oscillator level 1/(e^{theta/T} - 1) = e_vib/(R theta)
template <typename T>
__device__ __forceinline__ T mlevel(T theta, T Temp) {
  if (!(Temp > T(0))) return T(0);
  const T x = qdiv(theta, Temp);
  if (x > T(700)) return T(0);
  return qdiv(T(1), gm_expm1(x));
}

// Rescaled translational temperature: root of
//   (3/2 + a) T + b theta m(T) = 3/2 T_tr + a T_rot + b theta m(T_vib)
// (the energy balance behind the gamma coefficients of Sec. III.A.1),
// safeguarded Newton on [0, rhs/(3/2 + a)].  With x = theta/T and
// m = 1/(e^x - 1), dm/dT = x^2 m (1 + m)/T, so one expm1 per iteration
// gives both f and f'.
template <typename T>
__device__ __forceinline__ T tcheck(T theta, T Ttr, T Trot, T Tvib, T a, T b) {
  const T ca = T(1.5) + a;
  const T rhs = T(1.5) * Ttr + a * Trot + b * theta * mlevel(theta, Tvib);
  T hi = qdiv(rhs, ca), lo = T(0);
  if (!(hi > T(0))) return T(0);
  T t = qdiv(T(1.5) * Ttr + a * Trot, ca);
  if (!(t > T(0) && t <= hi)) t = hi;
  const T tol = sizeof(T) == 4 ? T(3e-7) : T(1e-14);
  for (int it = 0; it < 40; ++it) {
    const T x = qdiv(theta, t);
    // m(T) and c_v,vib/R; e^x overflows to inf for large x, giving m = 0
    const T m = x > T(700) ? T(0) : qdiv(T(1), gm_expm1(x));
    const T cv = x * x * m * (T(1) + m);
    const T f = ca * t + b * theta * m - rhs;
    if (f > T(0)) hi = t; else lo = t;
    const T fp = ca + b * cv;
    T tn = t - qdiv(f, fp);
    if (!(tn > lo && tn < hi)) tn = T(0.5) * (lo + hi);
    const T dt = fabs(tn - t);
    t = tn;
    if (dt <= tol * t) break;
  }
  return t;
}

// Secant heat capacity c_v,vib(T_1)/R between T_c and T_v (Sec. III.A.1),
// evaluated without cancellation:
//   xa xb e^{-xa} ((1 - e^{-d})/d) / ((1 - e^{-xa})(1 - e^{-xb})),
// xa <= xb the two values of theta/T, d = xb - xa.
template <typename T>
__device__ __forceinline__ T cbar_R(T theta, T Tc, T Tv) {
  if (!(Tc > T(0))) return T(0);
  if (!(Tv > T(0))) {
    const T xa = qdiv(theta, Tc);
    return xa > T(700) ? T(0) : qdiv(xa, gm_expm1(xa));
  }
  const T x1 = qdiv(theta, Tc), x2 = qdiv(theta, Tv);
  const T xa = fmin(x1, x2), xb = fmax(x1, x2);
  if (xa > T(700)) return T(0);
  const T d = qdiv(theta * fabs(Tc - Tv), Tc * Tv);
  const T h = d < T(1e-3) ? T(1) - d * (T(0.5) - d * (T(1) / T(6) - d * T(1) / T(24)))
                          : qdiv(-gm_expm1(-d), d);
  const T ea = gm_exp(-xa);
  const T oa = -gm_expm1(-xa), ob = -gm_expm1(-xb);
  return qdiv(xa * (xb * h) * ea, oa * ob);
}

// Eucken Prandtl number (Sec. IV.B)
__device__ __forceinline__ double prandtl(const GasP& g, double T) {
  if (g.pr_model == USP_PR_CONST) return g.Pr_const;
  double xi = 0.0;
  if (T > 0.0) {
    const double x = g.theta / T;
    xi = x > 700.0 ? 0.0 : x / expm1(x);
    if (g.pr_model == USP_PR_EUCKEN_STANDARD) xi *= 2.0;
  }
  return (14.0 + 2.0 * xi) / (19.0 + 2.0 * xi);
}

__device__ __forceinline__ double zrot(const GasP& g, double T) {
  if (g.zrot_model == USP_ZROT_CONST) return g.Z_rot;
  const double r = g.T_star / T;
  return g.Z_rot_inf / (1.0 + 0.5 * pow(PI, 1.5) * sqrt(r) + (PI + 0.25 * PI * PI) * r);
}

__device__ __forceinline__ double zvib(const GasP& g, double T) {
  if (g.zvib_model == USP_ZVIB_CONST) return g.Z_vib;
  const double mw = (g.C1 / pow(T, g.omega)) * exp(g.C2 * pow(T, -1.0 / 3.0));
  const double ht = (PI * g.d_ref * g.d_ref / g.sigma_vib) * pow(g.T_ref / T, g.omega - 0.5);
  return mw + ht;
}

// ---------------------------------------------------------------------------
// Grid: edge k of an axis in the stored precision S, formed with explicitly
// rounded FP64 operations (no contraction), so host and device agree bit
// for bit.  The index along an axis is the number of interior edges at or
// below v; -1 outside [e_0, e_n).
// ---------------------------------------------------------------------------
template <typename S>
__device__ __forceinline__ S edge(double o, double d, int k) {
  return (S)__dadd_rn(o, __dmul_rn((double)k, d));
}

// (id = 1/d gives the first guess.  The stored edges lie within a small
// fraction of a cell of o + k d, so the guess is normally right or off by
// one and the common path checks it against its two edges; otherwise the
// correction loops make the index exact against the edge table.)
template <typename S>
__device__ __forceinline__ int axis_index(S v, double o, double d, double id, int n) {
  if (!(v >= edge<S>(o, d, 0)) || v >= edge<S>(o, d, n)) return -1;
  int k = (int)floor(((double)v - o) * id);
  k = k < 0 ? 0 : (k > n - 1 ? n - 1 : k);
  const S e0 = edge<S>(o, d, k), e1 = edge<S>(o, d, k + 1);
  if (e0 <= v && v < e1) return k;
  if (v < e0 && k > 0 && edge<S>(o, d, k - 1) <= v) return k - 1;
  if (v >= e1 && k < n - 1 && v < edge<S>(o, d, k + 2)) return k + 1;
  while (k > 0 && edge<S>(o, d, k) > v) --k;
  while (k < n - 1 && edge<S>(o, d, k + 1) <= v) ++k;
  return k;
}

template <typename S>
__device__ __forceinline__ int32_t cell_of(const GridP& g, S x, S y) {
  if (g.dim == 1) return axis_index<S>(y, g.y0, g.dy, g.idy, g.ny);
  const int ix = axis_index<S>(x, g.x0, g.dx, g.idx, g.nx);
  const int iy = axis_index<S>(y, g.y0, g.dy, g.idy, g.ny);
  if (ix < 0 || iy < 0) return -1;
  return iy * g.nx + ix;
}

extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_or_u32(unsigned int);

// Event bits that name a counter (bit k: counter k).
constexpr uint32_t EVENT_MASK = USP_NCOUNTERS >= 32 ? 0xFFFFFFFFu : ((1u << USP_NCOUNTERS) - 1u);

// Bitwise OR of v over the active lanes of the wave, as a wave-uniform value.
__device__ __forceinline__ uint32_t wave_or(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)__ockl_wfred_or_u32(v));
}

// 64-bit event counter
__device__ __forceinline__ void count_event(int64_t* counters, int k, int64_t v = 1) {
  if (counters) atomicAdd((unsigned long long*)&counters[k], (unsigned long long)v);
}

// Events of the active lanes of a wave, one atomic per event kind: bit k of
// `ev` marks event k for this lane; `extra` adds a small per-lane count
// (< 16) to event `extra_k`.
__device__ __forceinline__ void flush_events(int64_t* counters, uint32_t ev, int extra_k = -1,
                                             int extra = 0) {
  if (!counters) return;
  const int lane = threadIdx.x & 63;
  const uint64_t active = __ballot(1);
  const int leader = __ffsll((long long)active) - 1;
  if (!__ballot(ev != 0u || extra != 0)) return;
  for (uint32_t rest = wave_or(ev) & EVENT_MASK; rest; rest &= rest - 1u) {
    const int k = __builtin_ctz(rest);
    const uint64_t m = __ballot((ev >> k) & 1u);
    if (lane == leader) atomicAdd((unsigned long long*)&counters[k], (unsigned long long)__popcll(m));
  }
  if (extra_k >= 0) {
    unsigned long long tot = 0;
    for (int b = 0; b < 4; ++b) tot += (unsigned long long)__popcll(__ballot((extra >> b) & 1)) << b;
    if (tot && lane == leader) atomicAdd((unsigned long long*)&counters[extra_k], tot);
  }
}

// A workgroup's event counts in LDS (c == nullptr when no counters are
// kept): flush_events adds to them with LDS atomics, and the workgroup adds
// them to the global counters after its last barrier.
struct WgCounters {
  unsigned long long* c;
};

__device__ __forceinline__ void flush_events(WgCounters w, uint32_t ev, int extra_k = -1,
                                             int extra = 0) {
  if (!w.c) return;
  const int lane = threadIdx.x & 63;
  const uint64_t active = __ballot(1);
  const int leader = __ffsll((long long)active) - 1;
  if (!__ballot(ev != 0u || extra != 0)) return;
  for (uint32_t rest = wave_or(ev) & EVENT_MASK; rest; rest &= rest - 1u) {
    const int k = __builtin_ctz(rest);
    const uint64_t m = __ballot((ev >> k) & 1u);
    if (lane == leader) atomicAdd(&w.c[k], (unsigned long long)__popcll(m));
  }
  if (extra_k >= 0) {
    unsigned long long tot = 0;
    for (int b = 0; b < 4; ++b) tot += (unsigned long long)__popcll(__ballot((extra >> b) & 1)) << b;
    if (tot && lane == leader) atomicAdd(&w.c[extra_k], tot);
  }
}

// Zero the workgroup's counts (before a barrier that precedes their use).
__device__ __forceinline__ void wg_counters_init(unsigned long long* c) {
  if (threadIdx.x < USP_NCOUNTERS) c[threadIdx.x] = 0ull;
}

// Add the workgroup's counts to the global counters and zero them (after a
// barrier that follows their last use; the next use must follow another).
__device__ __forceinline__ void wg_counters_flush(unsigned long long* c, int64_t* counters) {
  if (counters && threadIdx.x < USP_NCOUNTERS && c[threadIdx.x]) {
    atomicAdd((unsigned long long*)&counters[threadIdx.x], c[threadIdx.x]);
    c[threadIdx.x] = 0ull;
  }
}

// ---------------------------------------------------------------------------
// wave64 / block reductions in a fixed order (deterministic)
// ---------------------------------------------------------------------------
// FP64 sum over the 16 lanes of each row by DPP row permutes (swap of
// neighbours, of pairs, mirror within 8, mirror within 16); every lane of
// the row ends with the same bits (each step adds two operands whose
// roles are mirrored in the partner lane).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_f64<0x141>(v);  // row_half_mirror
  v += dpp_f64<0x140>(v);  // row_mirror
  return v;
}

// FP64 sum over a whole wave (all 64 lanes active): the four row sums,
// then (r0 + r1) + (r2 + r3); the result is uniform.  The rows are
// combined by the gfx950 row swaps: v_permlane16_swap exchanges rows 1 and
// 3 of its first operand with rows 0 and 2 of its second, so swapping a
// value with itself leaves rows (r0, r0, r2, r2) and (r1, r1, r3, r3),
// whose sum is r0 + r1 in rows 0-1 and r2 + r3 in rows 2-3;
// v_permlane32_swap exchanges rows 2-3 of the first with rows 0-1 of the
// second, which then sum to (r0 + r1) + (r2 + r3) in every lane (FP64
// addition commutes, so each lane has the same bits).
__device__ __forceinline__ double wave_swap_add(double v, bool rows32) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto l = rows32 ? __builtin_amdgcn_permlane32_swap(lo, lo, false, false)
                        : __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = rows32 ? __builtin_amdgcn_permlane32_swap(hi, hi, false, false)
                        : __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(h[0], l[0]) + __hiloint2double(h[1], l[1]);
}
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  v = wave_swap_add(v, false);
  return wave_swap_add(v, true);
}

}  // namespace usp
