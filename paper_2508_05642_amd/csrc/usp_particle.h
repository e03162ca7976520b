// usp_particle.h -- per-particle and per-cell device functions of the
// USP-FPM update: the particle update (Secs. III.A-III.B), the
// conservation scheme (Sec. IV.C) and the free flight with boundaries.
// Shared by the separate phase kernels and the fused update kernel, so
// both produce the same bits.
//
// Precision: the particle update runs in the state precision S (float for
// FP32 states, double for FP64 states); reconstruction weights, all cell
// quantities and the discrete vibrational decisions are FP64.
#pragma once
#include "usp_device.h"

namespace usp {

// Negative-binomial NB(r, p) (failures before the r-th success) and
// binomial B(n, p) draws by sequential CDF inversion: the smallest k with
// u < F(k).  The pmf recurrences and the order of every FP64 operation are
// fixed (no contraction) so that decisions are reproducible.
__device__ __forceinline__ int sample_nb(double u, int r, double p) {
#pragma clang fp contract(off)
  const double q = 1.0 - p;
  double pk = 1.0;
  for (int i = 0; i < r; ++i) pk = pk * p;
  double F = pk;
  int k = 0;
  while (u >= F && k < NB_KMAX) {
    double t = q * (double)(r + k);
    t = t / (double)(k + 1);
    pk = pk * t;
    F = F + pk;
    k = k + 1;
  }
  return k;
}

__device__ __forceinline__ int sample_b(double u, int n, double p) {
#pragma clang fp contract(off)
  if (n <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  const double q = 1.0 - p;
  double pk = 1.0;
  for (int i = 0; i < n; ++i) pk = pk * q;
  const double ratio = p / q;
  double F = pk;
  int k = 0;
  while (u >= F && k < n) {
    double t = ratio * (double)(n - k);
    t = t / (double)(k + 1);
    pk = pk * t;
    F = F + pk;
    k = k + 1;
  }
  return k;
}

// sin and cos of 0 <= x <= pi/3 (series of usp_device.h)
__device__ __forceinline__ void sincos_third(float x, float* s, float* c) {
  sincos_series<float, 5>(x, s, c);
}
__device__ __forceinline__ void sincos_third(double x, double* s, double* c) {
  sincos_series<double, 9>(x, s, c);
}

// smallest and largest eigenvalue of a symmetric 3x3 (trigonometric form:
// lambda = q + 2 p cos(phi + 2 pi k/3), phi = acos(det B / 2)/3 in
// [0, pi/3]; cos(phi + 2 pi/3) = -(cos phi + sqrt(3) sin phi)/2)
template <typename T>
__device__ __forceinline__ void eig_minmax(const T P[6], T* lmin, T* lmax) {
  const T p1 = P[3] * P[3] + P[4] * P[4] + P[5] * P[5];
  if (p1 == T(0)) {
    *lmin = fmin(P[0], fmin(P[1], P[2]));
    *lmax = fmax(P[0], fmax(P[1], P[2]));
    return;
  }
  const T q = (P[0] + P[1] + P[2]) / T(3);
  const T a = P[0] - q, b = P[1] - q, c = P[2] - q;
  const T p2 = a * a + b * b + c * c + T(2) * p1;
  const T p = sqrt(p2 / T(6));
  const T ip = T(1) / p;
  const T b11 = a * ip, b22 = b * ip, b33 = c * ip, b12 = P[3] * ip, b13 = P[4] * ip,
          b23 = P[5] * ip;
  const T det = b11 * (b22 * b33 - b23 * b23) - b12 * (b12 * b33 - b23 * b13) +
                b13 * (b12 * b23 - b22 * b13);
  T r = det / T(2);
  r = fmin(T(1), fmax(T(-1), r));
  const T phi = acos(r) / T(3);
  T sn, cs;
  sincos_third(phi, &sn, &cs);
  *lmax = q + T(2) * p * cs;
  *lmin = q - p * (cs + T(1.7320508075688772935) * sn);
}

// Cell-level coefficients (FP64, from the cell state).
struct CellCoef {
  double a, b, al, oma2, nu, r2, A2, Pr, dt;
  bool keep;  // refit root with the sign of al (else by the Prandtl number)
};

// Per-particle coefficients of the update.
template <typename T>
struct PartCoef {
  T L[6];          // Cholesky factor of Lambda = tau D_tr
  T al;            // alpha_tr = alpha_rot = alpha_vib
  double oma2;     // 1 - alpha^2 (FP64: it feeds the discrete decisions)
  T Trot_rel, mstar;
  T margin;        // smallest relative pivot of the accepted factor
  bool skip, fallback, nu_zero, clamp_rot, clamp_m;
};

// Cholesky with the smallest relative pivot min(d2/S_yy, d3/S_zz) returned.
template <typename T>
__device__ __forceinline__ bool chol3m(const T S[6], T L[6], T* margin) {
  if (!(S[0] > T(0))) return false;
  const T l11 = sqrt(S[0]);
  const T l21 = qdiv(S[3], l11), l31 = qdiv(S[4], l11);
  const T d2 = S[1] - l21 * l21;
  if (!(d2 > T(0))) return false;
  const T l22 = sqrt(d2);
  const T l32 = qdiv(S[5] - l31 * l21, l22);
  const T d3 = S[2] - l31 * l31 - l32 * l32;
  if (!(d3 > T(0))) return false;
  L[0] = l11; L[1] = l21; L[2] = l22; L[3] = l31; L[4] = l32; L[5] = sqrt(d3);
  *margin = fmin(qdiv(d2, S[1]), qdiv(d3, S[2]));
  return true;
}

// The chain of Secs. III.A.1-III.A.3 for one particle: rescaled
// temperature and gamma coefficients from the interpolated temperatures,
// relaxation temperatures (eqs. T_tr_USP, T_rot_USP, T_vib_USP), the
// diffusion tensor (eq. D_tr) and its Cholesky test, and on failure the nu
// clamp and alpha refit (eqs. nu_USP_positivity, alpha_USP_positivity_1..4).
// Without REFIT a failed test returns at once with `fallback` set (the FP32
// first pass hands such particles to the FP64 chain, so it never needs the
// refit, nor the cell inputs only the refit reads).
template <typename T, bool REFIT = true>
__device__ PartCoef<T> particle_coef(T R, T Th, T Ttr, T Trot, T Tvib, const T P[6],
                                     const CellCoef& cc) {
  PartCoef<T> r;
  r.skip = r.fallback = r.nu_zero = r.clamp_rot = r.clamp_m = false;
  r.margin = T(1);
  const T a = (T)cc.a, b = (T)cc.b;
  T al = (T)cc.al;
  double oma2d = cc.oma2;
  T nu = (T)cc.nu;
  // A vibrational exchange factor b below 1e-12 (tau_vib above ~1e12 time
  // steps: the Millikan-White number of a cold gas) leaves the gammas'
  // vibrational parts, b c_v,vib/D, and the shift of T-check from (3/2 T_tr
  // + a T_rot)/(3/2 + a) below 1e-7 K for temperatures up to 1e5 K (c_v,vib
  // <= R, e_vib/R <= T), far under FP32 resolution: they are taken as 0.
  T g1, g2, g3;
  if (b < T(1e-12)) {
    g1 = qdiv(T(3) * a, T(1.5) + a);
    g2 = g3 = T(0);
  } else {
    const T Tc = tcheck<T>(Th, Ttr, Trot, Tvib, a, b);
    const T cb = cbar_R<T>(Th, Tc, Tvib);
    const T D = T(1.5) + a + b * cb;
    g1 = qdiv(T(3) * a, D); g2 = qdiv(T(3) * b * cb, D); g3 = qdiv(T(2) * a * b * cb, D);
  }
  const T Xtr = g1 * (Ttr - Trot) + g2 * (Ttr - Tvib);
  const T Xrot = g1 * (Ttr - Trot) - g3 * (Trot - Tvib);
  const T Xvib = g2 * (Ttr - Tvib) + g3 * (Trot - Tvib);
  const T mvib = mlevel<T>(Th, Tvib);
  T oma2 = (T)oma2d;
  T Ttr_rel = Ttr - qdiv(Xtr, T(1.5) * oma2);
  T Trot_rel = Trot + qdiv(Xrot, oma2);
  T mstar = mvib + qdiv(Xvib, oma2 * Th);
  const T RT = R * Ttr;
  T Lam[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) Lam[k] = R * Ttr_rel + nu * (P[k] - RT);
#pragma unroll
  for (int k = 3; k < 6; ++k) Lam[k] = nu * P[k];
  bool ok = chol3m<T>(Lam, r.L, &r.margin);
  if (!REFIT && !ok) {
    r.fallback = true;
    return r;
  }
  if (!ok) {
    r.fallback = true;
    if (!(Ttr_rel > T(0))) {
      r.skip = true;
      return r;
    }
    T lmin, lmax;
    eig_minmax<T>(P, &lmin, &lmax);
    const T RTr = R * Ttr_rel;
    const T shrink = T(1) - T(1.0 / 1048576.0);
    if (nu <= T(0)) {
      if (lmax > RT) nu = fmax(nu, -RTr / (lmax - RT) * shrink);
    } else {
      if (lmin < RT) nu = fmin(nu, RTr / (RT - lmin) * shrink);
    }
    double a2 = ((double)nu - cc.r2) / ((double)nu - 1.0);
    a2 = fmin(1.0, fmax(0.0, a2));
    const double ap = sqrt(a2), am = -ap;
    const double Prp = cc.A2 * (1.0 - ap * ap * ap) / (cc.dt * (1.0 + ap * ap * ap));
    const double Prm = cc.A2 * (1.0 - am * am * am) / (cc.dt * (1.0 + am * am * am));
    if (cc.keep) al = (T)(cc.al < 0.0 ? am : ap);
    else al = (T)((fabs(Prm - cc.Pr) < fabs(Prp - cc.Pr)) ? am : ap);
    oma2d = 1.0 - a2;
    if (!(oma2d > 0.0)) {
      r.skip = true;
      return r;
    }
    oma2 = (T)oma2d;
    Ttr_rel = Ttr - qdiv(Xtr, T(1.5) * oma2);
    Trot_rel = Trot + qdiv(Xrot, oma2);
    mstar = mvib + qdiv(Xvib, oma2 * Th);
#pragma unroll
    for (int k = 0; k < 3; ++k) Lam[k] = R * Ttr_rel + nu * (P[k] - RT);
#pragma unroll
    for (int k = 3; k < 6; ++k) Lam[k] = nu * P[k];
    ok = chol3m<T>(Lam, r.L, &r.margin);
    if (!ok) {
      r.nu_zero = true;
      if (Ttr_rel > T(0)) {
        const T s0 = sqrt(R * Ttr_rel);
        r.L[0] = s0; r.L[1] = T(0); r.L[2] = s0; r.L[3] = T(0); r.L[4] = T(0); r.L[5] = s0;
      } else {
        r.skip = true;
        return r;
      }
    }
  }
  if (Trot_rel < T(0)) { Trot_rel = T(0); r.clamp_rot = true; }
  if (mstar < T(0)) { mstar = T(0); r.clamp_m = true; }
  r.al = al;
  r.oma2 = oma2d;
  r.Trot_rel = Trot_rel;
  r.mstar = mstar;
  return r;
}

// A particle's stored position (x used in 2D, y in 1D and 2D) and id (the
// key of its random streams), as the update reads them: from the particle
// arrays, or from a stage that holds them.
template <typename S>
struct PartPos {
  S x, y;
  uint32_t pid;
};

template <typename S>
__device__ __forceinline__ PartPos<S> load_pos(const PartP<S>& p, int64_t i, int dim) {
  PartPos<S> q;
  q.x = dim == 2 ? p.x[i] : S(0);
  q.y = dim >= 1 ? p.y[i] : S(0);
  q.pid = p.pid[i];
  return q;
}

// Stencil of a particle: the quadrant of its position in its cell selects
// one of the four precomputed stencils (see k_stencil); weights are the
// offsets from the cell centre over the signed spacing.
struct Stencil {
  int64_t c10, c01, c11;
  double wx, wy;
  bool hx, hy, hxy;
};

template <typename S>
__device__ __forceinline__ Stencil particle_stencil(const GridP& g, int32_t bits, int32_t c,
                                                    const PartPos<S>& q) {
  Stencil st;
  st.c10 = st.c01 = st.c11 = c;
  st.wx = st.wy = 0.0;
  st.hx = st.hy = st.hxy = false;
  if (g.dim == 0) return st;
  const int nx = g.nx;
  int cj = c, ci = 0;
  if (g.dim == 2) {
    // the row from an FP64 estimate of c / nx (off by at most one for any
    // int32 index), corrected against the remainder
    cj = (int)((double)c * g.inx);
    int r = c - cj * nx;
    if (r < 0) { --cj; r += nx; } else if (r >= nx) { ++cj; r -= nx; }
    ci = r;
  }
  // cell centre with explicitly rounded operations (no contraction)
  const double dyv = (double)q.y - __dadd_rn(g.y0, __dmul_rn(cj + 0.5, g.dy));
  double dxv = 0.0;
  int qd = dyv >= 0.0 ? 2 : 0;
  if (g.dim == 2) {
    dxv = (double)q.x - __dadd_rn(g.x0, __dmul_rn(ci + 0.5, g.dx));
    qd |= dxv >= 0.0 ? 1 : 0;
  }
  const int f = (bits >> (5 * qd)) & 31;
  const int tx = (f & 3) == 1 ? 1 : ((f & 3) == 2 ? -1 : 0);
  const int ty = ((f >> 2) & 3) == 1 ? 1 : (((f >> 2) & 3) == 2 ? -1 : 0);
  // weights: the offset over the signed spacing (times 1/dx, 1/dy)
  if (ty) { st.hy = true; st.wy = (ty > 0 ? dyv : -dyv) * g.idy; st.c01 = (int64_t)(cj + ty) * nx + ci; }
  if (tx) { st.hx = true; st.wx = (tx > 0 ? dxv : -dxv) * g.idx; st.c10 = (int64_t)cj * nx + ci + tx; }
  if ((f >> 4) & 1) { st.hxy = true; st.c11 = (int64_t)(cj + ty) * nx + ci + tx; }
  return st;
}

// first-order polynomial reconstruction from the FP64 planes
__device__ __forceinline__ double interp_planes(const double* __restrict__ cs, int64_t M, int f,
                                                int64_t c, const Stencil& st) {
  const double* F = cs + (int64_t)f * M;
  const double f00 = ldg(F, c);
  double phi = f00;
  const double f10 = ldg(F, st.c10), f01 = ldg(F, st.c01);
  if (st.hx) phi += (f10 - f00) * st.wx;
  if (st.hy) phi += (f01 - f00) * st.wy;
  if (st.hxy) phi += (f00 - f10 - f01 + ldg(F, st.c11)) * st.wx * st.wy;
  return phi;
}

__device__ __forceinline__ CellCoef coef_planes(const double* __restrict__ cs, int64_t M, int64_t c,
                                                bool keep) {
  CellCoef cc;
  cc.keep = keep;
  cc.a = ldg(cs, CS_A * M + c); cc.b = ldg(cs, CS_B * M + c); cc.al = ldg(cs, CS_ALPHA * M + c);
  cc.oma2 = ldg(cs, CS_OMA2 * M + c); cc.nu = ldg(cs, CS_NU * M + c); cc.r2 = ldg(cs, CS_R2 * M + c);
  cc.A2 = 2.0 * ldg(cs, CS_MUP * M + c); cc.Pr = ldg(cs, CS_PR * M + c); cc.dt = ldg(cs, CS_DT * M + c);
  return cc;
}

// FP64 values at the particle: U, Pi, and the floored temperatures
__device__ __forceinline__ bool fields_planes(const double* __restrict__ cs, int64_t M, int64_t c,
                                              const Stencil& st, double U[3], double P[6],
                                              double Tk[3]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) U[k] = interp_planes(cs, M, CS_UX + k, c, st);
#pragma unroll
  for (int k = 0; k < 6; ++k) P[k] = interp_planes(cs, M, CS_PXX + k, c, st);
  bool clamped = false;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    Tk[k] = interp_planes(cs, M, CS_TTR + k, c, st);
    const double fl = 0.05 * ldg(cs, (CS_TTR + k) * M + c);
    if (Tk[k] < fl) { Tk[k] = fl; clamped = true; }
  }
  return clamped;
}

// Velocity, rotational energy and level of one particle: the values an
// update reads (`in`) or produces (changed == false: the particle keeps its
// state because its cell or the particle itself is skipped).
template <typename S>
struct PartNew {
  S cx, cy, cz, erot;
  int vib;
  bool changed;
};

template <typename S>
__device__ __forceinline__ PartNew<S> load_state(const PartP<S>& p, int64_t i) {
  PartNew<S> v;
  v.cx = p.cx[i]; v.cy = p.cy[i]; v.cz = p.cz[i]; v.erot = p.erot[i]; v.vib = p.vib[i];
  v.changed = false;
  return v;
}

// Draws and the velocity (eq. update_ci), rotational (eq. update_erot) and
// vibrational (eq. update_evib) updates of particle i.
template <typename S, typename T>
__device__ __forceinline__ void update_particle(uint32_t id, const PartNew<S>& in, const T U[3],
                                                const PartCoef<T>& pc, T R, uint64_t seed,
                                                uint32_t step, uint32_t* ev, PartNew<S>* o) {
  const U4 w0 = philox(id, step, TAG_COLLIDE, 0u, seed);
  const U4 w1 = philox(id, step, TAG_COLLIDE, 1u, seed);
  T G1, G2, G3, G4;
  box_muller<T>(w0.w[0], w0.w[1], &G1, &G2);
  box_muller<T>(w0.w[2], w0.w[3], &G3, &G4);
  const T al = pc.al, oma2 = (T)pc.oma2;
  const T* L = pc.L;
  const T sq = sqrt(oma2);
  const T Cx = (T)in.cx - U[0], Cy = (T)in.cy - U[1], Cz = (T)in.cz - U[2];
  o->cx = (S)(U[0] + al * Cx + sq * (L[0] * G1));
  o->cy = (S)(U[1] + al * Cy + sq * (L[1] * G1 + L[2] * G2));
  o->cz = (S)(U[2] + al * Cz + sq * (L[3] * G1 + L[4] * G2 + L[5] * G3));
  const T half = T(0.5) * R * pc.Trot_rel * oma2;
  const T root = sqrt((T)in.erot) * al + sqrt(half) * G4;
  o->erot = (S)(half + root * root);
  // discrete decisions in FP64
  const int I = in.vib;
  const double ms = (double)pc.mstar;
  const double pNB = 1.0 / (1.0 + ms * pc.oma2);
  double pB = (1.0 + ms) * pc.oma2;
  if (pB > 1.0) { pB = 1.0; *ev |= 1u << USP_CNT_PB_CLAMP; }
  int nI = I + sample_nb(u01d(w1.w[0]), I + 1, pNB) - sample_b(u01d(w1.w[1]), I, pB);
  if (nI > VIB_MAX) { nI = VIB_MAX; *ev |= 1u << USP_CNT_VIB_SAT; }
  o->vib = nI;
  o->changed = true;
}

__device__ __forceinline__ void note_coef_events(const PartCoef<float>& a, uint32_t* ev) {
  if (a.fallback) *ev |= 1u << USP_CNT_CHOL_FALLBACK;
  if (a.nu_zero) *ev |= 1u << USP_CNT_NU_ZERO;
  if (a.skip) *ev |= 1u << USP_CNT_TREL_SKIP;
  if (a.clamp_rot || a.clamp_m) *ev |= 1u << USP_CNT_TREL_CLAMP;
}
__device__ __forceinline__ void note_coef_events(const PartCoef<double>& a, uint32_t* ev) {
  if (a.fallback) *ev |= 1u << USP_CNT_CHOL_FALLBACK;
  if (a.nu_zero) *ev |= 1u << USP_CNT_NU_ZERO;
  if (a.skip) *ev |= 1u << USP_CNT_TREL_SKIP;
  if (a.clamp_rot || a.clamp_m) *ev |= 1u << USP_CNT_TREL_CLAMP;
}

// First-order FPM update of particle i in cell c (Sec. II.C) from the FP64
// cell planes (no reconstruction); the Cholesky test and the level jumps in
// FP64, the four normals and the velocity and rotational-energy update in
// the state precision: the velocity by eq.
// conventionial-velo and the rotational energy by eq. conventionial-erot
// (the USP-FPM algebra with alpha = exp(-dt/tau)); the level by Gillespie's
// direct method for the master-equation rates omega_{I,I-1} = 2 I/(tau
// (1-q)), omega_{I,I+1} = 2 (I+1) q/(tau (1-q)), q = exp(-Theta/T_vib^rel) =
// m_rel/(1+m_rel).  Draws: block 0 of (pid, step, collide) for the four
// normals, blocks 1, 2, ... two uniforms per jump attempt, at most
// FPM_MAX_JUMPS attempts (then VIB_SAT).  A failed Cholesky test of the
// cell's Lambda falls back to nu = 0.
constexpr int FPM_MAX_JUMPS = 4096;

template <typename S>
__device__ __forceinline__ PartNew<S> collide_fpm(const GridP& g, const GasP& gas,
                                                 const double* __restrict__ cs,
                                                 const PartPos<S>& pq, int32_t c,
                                                 const PartNew<S>& in, uint64_t seed,
                                                 uint32_t step, uint32_t* evp) {
#pragma clang fp contract(off)
  PartNew<S> o;
  o.changed = false;
  const int64_t M = g.M;
  const double R = gas.R;
  double U[3], P[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) U[k] = ldg(cs, (CS_UX + k) * M + c);
#pragma unroll
  for (int k = 0; k < 6; ++k) P[k] = ldg(cs, (CS_PXX + k) * M + c);
  const double Ttr = ldg(cs, CS_TTR * M + c);
  const double al = ldg(cs, CS_ALPHA * M + c), oma2 = ldg(cs, CS_OMA2 * M + c), nu = ldg(cs, CS_NU * M + c);
  const double dtc = ldg(cs, CS_DT * M + c), tau = ldg(cs, CS_FPM_TAU * M + c);
  const double Ttr_rel = ldg(cs, CS_FPM_TTR_REL * M + c);
  double Trot_rel = ldg(cs, CS_FPM_TROT_REL * M + c), mrel = ldg(cs, CS_FPM_MREL * M + c);
  uint32_t ev = 0;
  const double RT = R * Ttr;
  double Lam[6], L[6], margin;
#pragma unroll
  for (int k = 0; k < 3; ++k) Lam[k] = R * Ttr_rel + nu * (P[k] - RT);
#pragma unroll
  for (int k = 3; k < 6; ++k) Lam[k] = nu * P[k];
  if (!chol3m<double>(Lam, L, &margin)) {
    ev |= (1u << USP_CNT_CHOL_FALLBACK) | (1u << USP_CNT_NU_ZERO);
    if (!(Ttr_rel > 0.0)) {
      *evp |= ev | (1u << USP_CNT_TREL_SKIP);
      return o;
    }
    const double s0 = sqrt(R * Ttr_rel);
    L[0] = s0; L[1] = 0.0; L[2] = s0; L[3] = 0.0; L[4] = 0.0; L[5] = s0;
  }
  if (Trot_rel < 0.0) { Trot_rel = 0.0; ev |= 1u << USP_CNT_TREL_CLAMP; }
  if (mrel < 0.0) { mrel = 0.0; ev |= 1u << USP_CNT_TREL_CLAMP; }
  const uint32_t id = pq.pid;
  const U4 w0 = philox(id, step, TAG_COLLIDE, 0u, seed);
  {
    // the draws and the update in the state precision (the decisions
    // above and the level jumps below stay in FP64)
    using T = S;
    T G1, G2, G3, G4;
    box_muller<T>(w0.w[0], w0.w[1], &G1, &G2);
    box_muller<T>(w0.w[2], w0.w[3], &G3, &G4);
    const T u0 = (T)U[0], u1 = (T)U[1], u2 = (T)U[2], a = (T)al;
    const T sq = sqrt((T)oma2);
    T Lt[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) Lt[k] = (T)L[k];
    const T Cx = (T)in.cx - u0, Cy = (T)in.cy - u1, Cz = (T)in.cz - u2;
    o.cx = (S)(u0 + a * Cx + sq * (Lt[0] * G1));
    o.cy = (S)(u1 + a * Cy + sq * (Lt[1] * G1 + Lt[2] * G2));
    o.cz = (S)(u2 + a * Cz + sq * (Lt[3] * G1 + Lt[4] * G2 + Lt[5] * G3));
    const T half = T(0.5) * (T)R * (T)Trot_rel * (T)oma2;
    const T root = sqrt((T)in.erot) * a + sqrt(half) * G4;
    o.erot = (S)(half + root * root);
  }
  // Gillespie: waiting time -ln(U1)/W, then up with probability
  // omega_up/W = (I+1) q / ((I+1) q + I)
  const double q = mrel / (1.0 + mrel);
  int I = in.vib;
  double t = 0.0;
  U4 w = w0;
  for (int k = 0; k < FPM_MAX_JUMPS; ++k) {
    const double wu = (double)(I + 1) * q, wd = (double)I;
    const double W = 2.0 * (wu + wd) / (tau * (1.0 - q));
    if (!(W > 0.0)) break;
    if ((k & 1) == 0) w = philox(id, step, TAG_COLLIDE, 1u + (uint32_t)(k >> 1), seed);
    const uint32_t a = (k & 1) ? w.w[2] : w.w[0], b = (k & 1) ? w.w[3] : w.w[1];
    const double dtv = -log(u01d(a)) / W;
    if (t + dtv > dtc) break;
    if (u01d(b) < wu / (wu + wd)) ++I;
    else --I;
    t += dtv;
    if (k == FPM_MAX_JUMPS - 1) ev |= 1u << USP_CNT_VIB_SAT;
  }
  if (I > VIB_MAX) { I = VIB_MAX; ev |= 1u << USP_CNT_VIB_SAT; }
  o.vib = I;
  o.changed = true;
  *evp |= ev;
  return o;
}

// Particle update of particle i in cell c (Secs. III.A-III.B).
// FP32 state, first pass: fields from the packed cell records (16-byte
// loads), FP32 reconstruction and coefficient chain.  When the Cholesky
// test of the diffusion tensor fails, or passes with a relative pivot below
// 1e-4, the particle is left unchanged with *esc set and no coefficient
// events: collide_esc then redoes it with every branch taken in FP64.
template <bool FPM>
__device__ __forceinline__ PartNew<float> collide_f32(const GridP& g, const GasP& gas,
                                                     const double* __restrict__ cs,
                                                     const PartPos<float>& q, int32_t c,
                                                     const PartNew<float>& in, uint64_t seed,
                                                     uint32_t step, uint32_t* evp, bool* esc) {
  *esc = false;
  if constexpr (FPM) return collide_fpm<float>(g, gas, cs, q, c, in, seed, step, evp);
  PartNew<float> o;
  o.changed = false;
  const int64_t M = g.M;
  const GlobalRec* __restrict__ rec = (const GlobalRec*)cell_records(cs, M);
  const GlobalF4* r4 = (const GlobalF4*)(rec + c);
  const F4 q4 = r4[3];  // fl[3], stencil
  const F4 q5 = r4[4];  // a, b, al, nu
  const GlobalRec& own = rec[c];
  if (own.collide == 0) return o;
  const Stencil st = particle_stencil<float>(g, __float_as_int(q4.w), c, q);
  // fields at the particle: each stencil cell's 12 fields added in with its
  // bilinear weight as its record arrives (the four records are never live
  // at once); the weights are those of f00 + (f10 - f00) wx + (f01 - f00) wy
  // + (f00 - f10 - f01 + f11) wx wy with the missing terms dropped
  const float wx = (float)st.wx, wy = (float)st.wy, wxy = (float)(st.wx * st.wy);
  const float w11 = st.hxy ? wxy : 0.0f;
  const float w10 = (st.hx ? wx : 0.0f) - w11;
  const float w01 = (st.hy ? wy : 0.0f) - w11;
  const float w00 = 1.0f - (st.hx ? wx : 0.0f) - (st.hy ? wy : 0.0f) + w11;
  float v12[12];
  auto add12 = [&](int64_t cc, float w, bool first) {
    const GlobalF4* v = (const GlobalF4*)(rec + cc);
    const F4 a0 = v[0], a1 = v[1], a2 = v[2];
    const float f[12] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w, a2.x, a2.y, a2.z, a2.w};
#pragma unroll
    for (int k = 0; k < 12; ++k) v12[k] = first ? w * f[k] : fmaf(w, f[k], v12[k]);
  };
  add12(c, w00, true);
  add12(st.c10, w10, false);
  add12(st.c01, w01, false);
  add12(st.c11, w11, false);
  float U[3] = {v12[0], v12[1], v12[2]};
  float Tk[3] = {v12[3], v12[4], v12[5]};
  float P[6] = {v12[6], v12[7], v12[8], v12[9], v12[10], v12[11]};
  const float fl[3] = {q4.x, q4.y, q4.z};
  uint32_t ev = 0;
  bool clamped = false;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (Tk[k] < fl[k]) { Tk[k] = fl[k]; clamped = true; }
  if (clamped) ev |= 1u << USP_CNT_INTERP_CLAMP;
  CellCoef cc;
  cc.a = q5.x; cc.b = q5.y; cc.al = q5.z; cc.nu = q5.w;
  // the refit's inputs (r2, 2 mu/p, Pr, dt, the sign rule) stay unread: a
  // failed test goes to the FP64 chain
  cc.oma2 = own.oma2;
  const PartCoef<float> pc =
      particle_coef<float, false>((float)gas.R, (float)gas.theta, Tk[0], Tk[1], Tk[2], P, cc);
  if (pc.fallback || pc.margin < 1e-4f) {
    *esc = true;
    *evp |= ev;
    return o;
  }
  note_coef_events(pc, &ev);
  if (!pc.skip) update_particle<float, float>(q.pid, in, U, pc, (float)gas.R, seed, step, &ev, &o);
  *evp |= ev;
  return o;
}

// FP32 state, second pass for the particles collide_f32 escalated: U, Pi
// and the temperatures interpolated from the FP64 planes with the same
// stencil, the coefficient chain with its Cholesky test and fallback in
// FP64, then the update in FP32 (the interpolation clamp was reported by
// the first pass).
__device__ __forceinline__ PartNew<float> collide_esc(const GridP& g, const GasP& gas,
                                                     const double* __restrict__ cs,
                                                     const PartPos<float>& q, int32_t c,
                                                     const PartNew<float>& in, uint64_t seed,
                                                     uint32_t step, uint32_t* evp) {
  PartNew<float> o;
  o.changed = false;
  const int64_t M = g.M;
  const Stencil st = particle_stencil<float>(g, cell_records(cs, M)[c].stencil, c, q);
  double Ud[3], Pd[6], Td[3];
  fields_planes(cs, M, c, st, Ud, Pd, Td);
  const CellCoef cd = coef_planes(cs, M, c, gas.alpha_keep != 0);
  const PartCoef<double> pd = particle_coef<double>(gas.R, gas.theta, Td[0], Td[1], Td[2], Pd, cd);
  PartCoef<float> pc;
#pragma unroll
  for (int k = 0; k < 6; ++k) pc.L[k] = (float)pd.L[k];
  pc.al = (float)pd.al; pc.oma2 = pd.oma2; pc.Trot_rel = (float)pd.Trot_rel;
  pc.mstar = (float)pd.mstar; pc.margin = (float)pd.margin;
  pc.skip = pd.skip; pc.fallback = pd.fallback; pc.nu_zero = pd.nu_zero;
  pc.clamp_rot = pd.clamp_rot; pc.clamp_m = pd.clamp_m;
  uint32_t ev = 0;
  note_coef_events(pc, &ev);
  const float U[3] = {(float)Ud[0], (float)Ud[1], (float)Ud[2]};
  if (!pc.skip) update_particle<float, float>(q.pid, in, U, pc, (float)gas.R, seed, step, &ev, &o);
  *evp |= ev;
  return o;
}

// Both passes in one call.
template <bool FPM>
__device__ __forceinline__ PartNew<float> collide_one(const GridP& g, const GasP& gas,
                                                     const double* __restrict__ cs,
                                                     const PartPos<float>& q, int32_t c,
                                                     const PartNew<float>& in, uint64_t seed,
                                                     uint32_t step, uint32_t* evp) {
  bool esc;
  PartNew<float> o = collide_f32<FPM>(g, gas, cs, q, c, in, seed, step, evp, &esc);
  if (esc) o = collide_esc(g, gas, cs, q, c, in, seed, step, evp);
  return o;
}

// FP64 state: fields and coefficients from the FP64 planes.
template <bool FPM>
__device__ __forceinline__ PartNew<double> collide_one(const GridP& g, const GasP& gas,
                                                      const double* __restrict__ cs,
                                                      const PartPos<double>& q, int32_t c,
                                                      const PartNew<double>& in, uint64_t seed,
                                                      uint32_t step, uint32_t* evp) {
  if constexpr (FPM) return collide_fpm<double>(g, gas, cs, q, c, in, seed, step, evp);
  PartNew<double> o;
  o.changed = false;
  const int64_t M = g.M;
  if (ldg(cs, CS_COLLIDE * M + c) == 0.0) return o;
  const Stencil st = particle_stencil<double>(g, cell_records(cs, M)[c].stencil, c, q);
  double U[3], P[6], Tk[3];
  uint32_t ev = fields_planes(cs, M, c, st, U, P, Tk) ? (1u << USP_CNT_INTERP_CLAMP) : 0u;
  const CellCoef cc = coef_planes(cs, M, c, gas.alpha_keep != 0);
  const PartCoef<double> pc = particle_coef<double>(gas.R, gas.theta, Tk[0], Tk[1], Tk[2], P, cc);
  note_coef_events(pc, &ev);
  if (!pc.skip) update_particle<double, double>(q.pid, in, U, pc, gas.R, seed, step, &ev, &o);
  *evp |= ev;
  return o;
}

// The coefficient chain of cell c at the cell's own temperatures and Pi
// (the per-cell reading), FP64, packed for the particle update.
__device__ __forceinline__ CellPCoef cell_pcoef(const GasP& gas, const double* __restrict__ cs,
                                                int64_t M, int64_t c) {
  CellPCoef r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.L[k] = 0.0;
  r.al = r.oma2 = r.Trot_rel = r.mstar = 0.0;
  r.flags = 0; r.pad[0] = r.pad[1] = r.pad[2] = 0;
  if (cs[CS_COLLIDE * M + c] == 0.0) return r;
  const CellCoef cc = coef_planes(cs, M, c, gas.alpha_keep != 0);
  double P[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) P[k] = cs[(CS_PXX + k) * M + c];
  const PartCoef<double> pc = particle_coef<double>(gas.R, gas.theta, cs[CS_TTR * M + c],
                                                    cs[CS_TROT * M + c], cs[CS_TVIB * M + c], P, cc);
  r.flags = (pc.skip ? PC_SKIP : 0) | (pc.fallback ? PC_FALLBACK : 0) |
            (pc.nu_zero ? PC_NU_ZERO : 0) | (pc.clamp_rot ? PC_CLAMP_ROT : 0) |
            (pc.clamp_m ? PC_CLAMP_M : 0);
  if (pc.skip) return r;
#pragma unroll
  for (int k = 0; k < 6; ++k) r.L[k] = pc.L[k];
  r.al = pc.al; r.oma2 = pc.oma2; r.Trot_rel = pc.Trot_rel; r.mstar = pc.mstar;
  return r;
}

// Particle update with the coefficients of the cell (USP_GAMMA_CELL): U
// interpolated as the per-particle chain does (FP32 from the packed
// records for FP32 states, FP64 from the planes for FP64 states), every
// other coefficient from the cell's record; the coefficient events are
// those of the cell, counted for each of its particles.
template <typename S>
__device__ __forceinline__ PartNew<S> collide_cell(const GridP& g, const GasP& gas,
                                                   const double* __restrict__ cs,
                                                   const PartPos<S>& q, int32_t c,
                                                   const PartNew<S>& in, uint64_t seed,
                                                   uint32_t step, uint32_t* evp) {
  PartNew<S> o;
  o.changed = false;
  const int64_t M = g.M;
  const CellRec* __restrict__ rec = cell_records(cs, M);
  if (rec[c].collide == 0) return o;
  const Stencil st = particle_stencil<S>(g, rec[c].stencil, c, q);
  S U[3];
  if constexpr (sizeof(S) == 4) {
    const F4 a = ((const GlobalF4*)(rec + c))[0], b = ((const GlobalF4*)(rec + st.c10))[0];
    const F4 d = ((const GlobalF4*)(rec + st.c01))[0], e = ((const GlobalF4*)(rec + st.c11))[0];
    const float f00[3] = {a.x, a.y, a.z}, f10[3] = {b.x, b.y, b.z};
    const float f01[3] = {d.x, d.y, d.z}, f11[3] = {e.x, e.y, e.z};
    const float wx = (float)st.wx, wy = (float)st.wy, wxy = (float)(st.wx * st.wy);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float phi = f00[k];
      if (st.hx) phi += (f10[k] - f00[k]) * wx;
      if (st.hy) phi += (f01[k] - f00[k]) * wy;
      if (st.hxy) phi += (f00[k] - f10[k] - f01[k] + f11[k]) * wxy;
      U[k] = phi;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 3; ++k) U[k] = interp_planes(cs, M, CS_UX + k, c, st);
  }
  const GlobalPCoef& cp = ((const GlobalPCoef*)cell_pcoefs(cs, M))[c];
  PartCoef<S> pc;
  const int32_t f = cp.flags;
  pc.skip = (f & PC_SKIP) != 0; pc.fallback = (f & PC_FALLBACK) != 0;
  pc.nu_zero = (f & PC_NU_ZERO) != 0; pc.clamp_rot = (f & PC_CLAMP_ROT) != 0;
  pc.clamp_m = (f & PC_CLAMP_M) != 0;
#pragma unroll
  for (int k = 0; k < 6; ++k) pc.L[k] = (S)cp.L[k];
  pc.al = (S)cp.al; pc.oma2 = cp.oma2; pc.Trot_rel = (S)cp.Trot_rel; pc.mstar = (S)cp.mstar;
  pc.margin = S(1);
  uint32_t ev = 0;
  note_coef_events(pc, &ev);
  if (!pc.skip) update_particle<S, S>(q.pid, in, U, pc, (S)gas.R, seed, step, &ev, &o);
  *evp |= ev;
  return o;
}

// The particle update of a kernel variant (MODE_*): the per-particle chain
// (FP32: both passes), the first-order FPM method, or the cell's chain.
template <int MODE, typename S>
__device__ __forceinline__ PartNew<S> collide_mode(const GridP& g, const GasP& gas,
                                                   const double* __restrict__ cs,
                                                   const PartPos<S>& q, int32_t c,
                                                   const PartNew<S>& in, uint64_t seed,
                                                   uint32_t step, uint32_t* evp) {
  if constexpr (MODE == MODE_CELL) return collide_cell<S>(g, gas, cs, q, c, in, seed, step, evp);
  else return collide_one<MODE == MODE_FPM>(g, gas, cs, q, c, in, seed, step, evp);
}

// ---------------------------------------------------------------------------
// Conservation (Sec. IV.C): one wave per cell.  The serial vibrational
// picks run on an LDS copy of the cell's levels (cells up to CONS_LDS
// particles; larger cells pick in global memory).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// One level up (+1) or down (-1) for level byte b, by an integer atomic on
// the aligned 32-bit word that holds it (LDS or global).  The caller's
// acceptance keeps every level within [0, VIB_MAX], so no carry or borrow
// reaches a neighbouring byte, and the atomics commute.
__device__ __forceinline__ void level_step(uint8_t* b, int dir) {
  const uintptr_t a = (uintptr_t)b;
  uint32_t* w = (uint32_t*)(a & ~(uintptr_t)3);
  const uint32_t one = 1u << (8 * (unsigned)(a & 3));
  if (dir > 0) atomicAdd(w, one);
  else atomicSub(w, one);
}

// The vibrational correction of Sec. IV.C, |I_delta| single-level moves on
// particles picked uniformly at random (draw j: counter (cell, step, 2, j/4),
// word j%4; a decrement that hits level 0, or an increment that hits the top
// level, is redrawn).  The draws are sequential by definition; here a wave
// evaluates 64 consecutive draws at once and reproduces the sequential
// outcome exactly: draw j on particle k is accepted iff the level of k,
// after the accepted earlier draws on k, still allows the move, i.e. iff
// dup < L (decrement) or L + dup < VIB_MAX (increment), dup being the number
// of earlier draws of the chunk on k; only the first |I_delta| accepted draws
// are applied, each as one level step.  When no level can reach VIB_MAX
// (`low`), every increment is accepted and dup is not needed.  Gives up
// after 64 N draws or when a decrement is impossible.  Returns 1 if any
// level changed; *SI is updated.  Called by a whole wave.
__device__ int wave_picks(uint8_t* lv, int64_t N, int64_t Id, int64_t* SI_io, uint32_t c,
                          uint32_t step, uint64_t seed, bool low, int64_t* counters) {
  const int lane = threadIdx.x & 63;
  const int64_t maxatt = 64 * N;
  int64_t att = 0, SI = *SI_io;
  uint32_t jbase = 1;
  int moved = 0;
  const double Nd = (double)N;
  const int kbits = N > 1 ? 64 - __clzll((long long)(N - 1)) : 0;  // bits of the keys
  while (Id != 0) {
    if (att >= maxatt || (Id < 0 && SI == 0)) {
      if (lane == 0) count_event(counters, USP_CNT_PICK_FAIL);
      break;
    }
    const int64_t need = Id > 0 ? Id : -Id;
    const bool valid = att + lane < maxatt;
    const uint32_t j = jbase + (uint32_t)lane;
    const U4 w = philox(c, step, TAG_CONSERVE, j >> 2, seed);
    const uint32_t wj = (j & 3) == 0 ? w.w[0] : (j & 3) == 1 ? w.w[1] : (j & 3) == 2 ? w.w[2] : w.w[3];
    int64_t k = (int64_t)floor(u01d(wj) * Nd);
    if (k >= N) k = N - 1;
    const int kk = (int)k;
    bool acc;
    if (Id > 0 && low) {
      acc = valid;
    } else {
      // the earlier lanes that drew the same particle: the lanes whose key
      // agrees with this lane's in every bit (one ballot per bit of N - 1)
      uint64_t same = ~0ull;
      for (int b = 0; b < kbits; ++b) {
        const uint32_t bit = ((uint32_t)kk >> b) & 1u;
        const uint64_t bm = __ballot(bit);
        same &= bit ? bm : ~bm;
      }
      const int dup = __popcll(same & ((1ull << lane) - 1ull));
      const int L = valid ? (int)lv[k] : 0;
      acc = valid && (Id > 0 ? (L + dup < VIB_MAX) : (dup < L));
    }
    const uint64_t accm = __ballot(acc);
    const int nacc = __popcll(accm);
    uint64_t applied;
    int consumed;
    if (nacc >= need) {
      // lane of the need-th accepted draw: the last draw made
      uint64_t m = accm;
      for (int64_t t = 1; t < need; ++t) m &= m - 1;
      const int cut = __ffsll((long long)m) - 1;
      applied = accm & (cut == 63 ? ~0ull : ((2ull << cut) - 1ull));
      consumed = cut + 1;
    } else {
      applied = accm;
      consumed = (int)__popcll(__ballot(valid));
    }
    const int napp = (int)__popcll(applied);
    wave_sync_lds();
    if ((applied >> lane) & 1ull) level_step(lv + k, Id > 0 ? 1 : -1);
    wave_sync_lds();
    if (napp) moved = 1;
    SI += Id > 0 ? napp : -napp;
    Id += Id > 0 ? -napp : napp;
    att += consumed;
    jbase += (uint32_t)consumed;
  }
  *SI_io = SI;
  return moved;
}

// The inputs of the conservation of cell c taken from the cell state, and
// the cell's draw for the rounding of I_delta: requested together, before
// the cell's sums, so that one memory round trip covers them all.
struct ConsIn {
  double Un[3];           // U^n
  double evib_t, erot_t;  // the cell targets of the vibrational and rotational energy
  double E0;              // e_tr^n + e_rot^n + e_vib^n
  double u0;              // uniform draw (counter (c, step, conserve, 0), word 0)
  bool collide;
};

__device__ __forceinline__ ConsIn cons_in(const double* __restrict__ cs, int64_t M, int64_t c,
                                          uint32_t step, uint64_t seed) {
  ConsIn a;
  a.collide = cs[CS_COLLIDE * M + c] != 0.0;
  a.Un[0] = cs[CS_UX * M + c]; a.Un[1] = cs[CS_UY * M + c]; a.Un[2] = cs[CS_UZ * M + c];
  a.evib_t = cs[CS_EVIB_NEW * M + c]; a.erot_t = cs[CS_EROT_NEW * M + c];
  a.E0 = cs[CS_ETR * M + c] + cs[CS_EROT * M + c] + cs[CS_EVIB * M + c];
  a.u0 = u01d(philox((uint32_t)c, step, TAG_CONSERVE, 0u, seed).w[0]);
  return a;
}

// The per-cell quantities of the conservation of Sec. IV.C, computed from
// the cell's post-collision sums and applied to each particle afterwards.
struct ConsScalars {
  double Un[3];   // U^n, the velocity scaling's target mean
  double Us[3];   // U*, the post-collision mean
  double frot;    // rotational factor (0: no rotational scaling)
  double sc;      // velocity factor (0: no velocity scaling)
  int moved;      // a level was changed by the picks
};

// Post-collision sums of the particles [i0, i1) taken by one lane (i0 =
// its first index, stride `stride`): s = (sum C_x, C_y, C_z, |C|^2 with C =
// c - U^n, sum e_rot, sum I) and the largest level; vx[i - base] etc. (LDS
// or global).  With copy, the levels are also copied to lv[i - o0].
template <typename PS>
__device__ __forceinline__ void cons_sums(const double Un[3], int64_t i0, int64_t i1,
                                          int64_t stride, const PS* vcx, const PS* vcy,
                                          const PS* vcz, const PS* verot, const uint8_t* vvib,
                                          int64_t base, uint8_t* lv, int64_t o0, bool copy,
                                          double s[6], int* lmax) {
  for (int64_t i = i0; i < i1; i += stride) {
    const int64_t j = i - base;
    const double d0 = (double)vcx[j] - Un[0], d1 = (double)vcy[j] - Un[1],
                 d2 = (double)vcz[j] - Un[2];
    s[0] += d0; s[1] += d1; s[2] += d2;
    s[3] += d0 * d0 + d1 * d1 + d2 * d2;
    s[4] += (double)verot[j];
    const uint8_t v = vvib[j];
    s[5] += (double)v;
    *lmax = v > *lmax ? v : *lmax;
    if (copy) lv[i - o0] = v;
  }
}

// The conservation of cell c from its wave-reduced sums s (uniform on the
// wave) and largest level lmax: (i) the vibrational correction, |I_delta|
// single-level moves by wave_picks on the cell's levels lv, (ii) the
// rotational factor to the cell target, (iii) the velocity factor about U*
// toward U^n that restores momentum and total energy with the energies
// actually reached.  Called by a whole wave; the result is uniform.
__device__ __forceinline__ ConsScalars cons_scalars(const GasP& gas, const ConsIn& in, int64_t c,
                                                    int64_t N, const double s[6], int lmax,
                                                    uint8_t* lv, uint64_t seed, uint32_t step,
                                                    int64_t* counters) {
  const int lane = threadIdx.x & 63;
  ConsScalars r;
  r.Un[0] = in.Un[0]; r.Un[1] = in.Un[1]; r.Un[2] = in.Un[2];
  const double evib_t = in.evib_t, erot_t = in.erot_t, E0 = in.E0;
  const double Nd = (double)N, iN = 1.0 / Nd;
  const double m1[3] = {s[0] * iN, s[1] * iN, s[2] * iN};
  const double RTh = gas.R * gas.theta;
  // (i) vibrational levels: I_delta = floor(N (e_target - e*)/(R theta) + U),
  // then |I_delta| single-level moves on randomly picked particles
  int64_t SI = (int64_t)s[5];
  const double X = Nd * evib_t / RTh - (double)SI;
  // the first-order FPM method keeps the levels and rotational energies it
  // sampled and conserves momentum and total energy through the velocities
  const bool fpm = gas.scheme == USP_SCHEME_FPM;
  const int64_t Id0 = fpm ? 0 : (int64_t)floor(X + in.u0);
  // no level can reach VIB_MAX through these increments
  const int64_t need0 = Id0 > 0 ? Id0 : 0;
  const bool low = !__ballot((int64_t)lmax + need0 >= VIB_MAX);
  r.moved = wave_picks(lv, N, Id0, &SI, (uint32_t)c, step, seed, low, counters);
  // the cell scalars, the same on every lane (wave-uniform inputs)
  r.frot = 0.0; r.sc = 0.0;
  const double etr_s = 0.5 * (s[3] * iN - (m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2]));
  // (ii) rotational scaling to the cell target
  const double erot_s = s[4] * iN;
  double erot_a = erot_s;
  int skips = 0;
  if (fpm) {
    // the sampled rotational energies stand
  } else if (erot_s > 0.0 && erot_t > 0.0) {
    r.frot = erot_t / erot_s;
    erot_a = erot_t;
  } else {
    ++skips;
  }
  // (iii) velocity scaling about U*, toward U^n (momentum and energy)
  const double evib_a = (double)SI * RTh * iN;
  const double s2 = (E0 - erot_a - evib_a) / etr_s;
  if (etr_s > 0.0 && s2 > 0.0) r.sc = sqrt(s2);
  else ++skips;
  if (lane == 0)
    for (int k = 0; k < skips; ++k) count_event(counters, USP_CNT_CONS_SKIP);
  r.Us[0] = r.Un[0] + m1[0]; r.Us[1] = r.Un[1] + m1[1]; r.Us[2] = r.Un[2] + m1[2];
  return r;
}

// The conservation's scalings of particle i (vx[i - base] etc.).
template <typename S, typename PS>
__device__ __forceinline__ void cons_apply(const ConsScalars& r, int64_t j, PS* vcx, PS* vcy,
                                           PS* vcz, PS* verot) {
  if (r.frot > 0.0) verot[j] = (S)((double)verot[j] * r.frot);
  if (r.sc > 0.0) {
    vcx[j] = (S)(r.Un[0] + r.sc * ((double)vcx[j] - r.Us[0]));
    vcy[j] = (S)(r.Un[1] + r.sc * ((double)vcy[j] - r.Us[1]));
    vcz[j] = (S)(r.Un[2] + r.sc * ((double)vcz[j] - r.Us[2]));
  }
}

// Conservation of one cell by one wave (Sec. IV.C).  The cell's particles
// are [o0, o1); their post-collision values sit at vx[i - base] etc.
// (LDS or global).  The vibrational picks run on `lv`, the cell's levels
// (LDS or global); if `copy` is set, vx's levels are first copied to lv and
// copied back after the picks.
template <typename S, typename PS>
__device__ __forceinline__ void conserve_cell(const GasP& gas, const ConsIn& in, int64_t c,
                                              int64_t o0, int64_t o1, PS* vcx, PS* vcy, PS* vcz,
                                              PS* verot, uint8_t* vvib, int64_t base, uint8_t* lv,
                                              bool copy, uint64_t seed, uint32_t step,
                                              int64_t* counters) {
  const int lane = threadIdx.x & 63;
  const int64_t N = o1 - o0;
  double s[6] = {0, 0, 0, 0, 0, 0};
  int lmax = 0;
  cons_sums<PS>(in.Un, o0 + lane, o1, 64, vcx, vcy, vcz, verot, vvib, base, lv, o0, copy, s,
                &lmax);
#pragma unroll
  for (int k = 0; k < 6; ++k) s[k] = wave_sum(s[k]);
  wave_sync_lds();
  const ConsScalars r = cons_scalars(gas, in, c, N, s, lmax, lv, seed, step, counters);
  wave_sync_lds();
  for (int64_t i = o0 + lane; i < o1; i += 64) {
    const int64_t j = i - base;
    if (copy && r.moved) vvib[j] = lv[i - o0];
    cons_apply<S, PS>(r, j, vcx, vcy, vcz, verot);
  }
}

// Wall re-emission draws for bounce `b`: blocks (2b, 2b+1) of the wall
// stream.  Normal speed from the flux-weighted half-range Maxwellian,
// tangential components Gaussian, exponential rotational energy and a
// Boltzmann level, all at the wall temperature.
__device__ __forceinline__ void wall_draw(const GasP& gas, double Tw, uint64_t seed, uint32_t pid,
                                          uint32_t step, int b, double* cn, double* ta, double* tb,
                                          double* er, int* lv) {
  const U4 w0 = philox(pid, step, TAG_WALL, (uint32_t)(2 * b), seed);
  const U4 w1 = philox(pid, step, TAG_WALL, (uint32_t)(2 * b + 1), seed);
  const double R = gas.R, sig = sqrt(R * Tw);
  *cn = sqrt(-2.0 * R * Tw * log(u01d(w0.w[0])));
  const double r = sqrt(-2.0 * log(u01d(w0.w[1])));
  double sn, cs;
  sincospi(2.0 * u01d(w0.w[2]), &sn, &cs);
  *ta = sig * r * cs;
  *tb = sig * r * sn;
  *er = -R * Tw * log(u01d(w0.w[3]));
  const double l = floor(log(u01d(w1.w[0])) / (-gas.theta / Tw));
  *lv = l > (double)VIB_MAX ? VIB_MAX : (int)l;
}

template <typename S>
__device__ __forceinline__ S settle(double v, double lo, double hi) {
  S vs = (S)v;
  const S los = (S)lo, his = (S)hi;
  if (vs >= his) vs = nextafter(his, (S)(-INFINITY));
  if (vs < los) vs = los;
  return vs;
}

// Free flight of particle i over dt with its post-collision values (cx0,
// cy0, cz0, er0, lv0): body-force kick, then straight flight with
// periodic, specular, outflow/free-stream and diffuse-wall boundaries (wall
// re-emission continues the remaining flight time).  Writes position,
// velocity, rot/vib state and the new cell (or -1 on deletion) to p.
// Surface sampling of one diffuse re-emission: the momentum and energy the
// particle gives the wall, per unit mass, added in fixed point to its
// element with integer atomics (order-independent sums).  (nx, ny) is the
// unit normal into the gas; side 4 is the cylinder.
__device__ __forceinline__ void surf_add(unsigned long long* a, double v, double scale) {
  atomicAdd(a, (unsigned long long)__double2ll_rn(v * scale));
}

__device__ __forceinline__ void surf_record(const GridP& g, const BcP& bc, int side, double x,
                                         double y, double nx, double ny, double cix, double ciy,
                                         double ciz, double eri, int lvi, double cox, double coy,
                                         double coz, double ero, int lvo) {
  int64_t e;
  double tx, ty;
  if (side == USP_SIDE_YLO || side == USP_SIDE_YHI) {
    int64_t ix = 0;
    if (g.dim == 2) {
      const double f = floor((x - g.x0) / g.dx);
      ix = f < 0.0 ? 0 : (f >= (double)g.nx ? g.nx - 1 : (int64_t)f);
    }
    e = (side == USP_SIDE_YLO ? 0 : g.nx) + ix;
    nx = 0.0; ny = side == USP_SIDE_YLO ? 1.0 : -1.0; tx = 1.0; ty = 0.0;
  } else if (side == USP_SIDE_XLO || side == USP_SIDE_XHI) {
    const double f = floor((y - g.y0) / g.dy);
    const int64_t iy = f < 0.0 ? 0 : (f >= (double)g.ny ? g.ny - 1 : (int64_t)f);
    e = 2 * (int64_t)g.nx + (side == USP_SIDE_XLO ? 0 : g.ny) + iy;
    nx = side == USP_SIDE_XLO ? 1.0 : -1.0; ny = 0.0; tx = 0.0; ty = 1.0;
  } else {
    if (bc.surf_nbody <= 0) return;
    const double th = atan2(fabs(ny), -nx);
    const double f = floor(th * (double)bc.surf_nbody / M_PI);
    const int64_t ib = f < 0.0 ? 0 : (f >= (double)bc.surf_nbody ? bc.surf_nbody - 1 : (int64_t)f);
    e = 2 * (int64_t)g.nx + 2 * (int64_t)g.ny + ib;
    // tangent along increasing Theta on either half
    if (ny >= 0.0) { tx = ny; ty = -nx; } else { tx = -ny; ty = nx; }
  }
  unsigned long long* a = bc.surf + e * USP_SURF_NQ;
  const double dx = cix - cox, dy = ciy - coy, dz = ciz - coz;
  atomicAdd(a + USP_SURF_HITS, 1ull);
  surf_add(a + USP_SURF_PX, dx, USP_SURF_P_SCALE);
  surf_add(a + USP_SURF_PY, dy, USP_SURF_P_SCALE);
  surf_add(a + USP_SURF_PZ, dz, USP_SURF_P_SCALE);
  surf_add(a + USP_SURF_PN, -(dx * nx + dy * ny), USP_SURF_P_SCALE);
  surf_add(a + USP_SURF_PT, dx * tx + dy * ty, USP_SURF_P_SCALE);
  surf_add(a + USP_SURF_ETR,
           0.5 * ((cix * cix + ciy * ciy + ciz * ciz) - (cox * cox + coy * coy + coz * coz)),
           USP_SURF_E_SCALE);
  surf_add(a + USP_SURF_EROT, eri - ero, USP_SURF_E_SCALE);
  atomicAdd(a + USP_SURF_QVIB, (unsigned long long)(long long)(lvi - lvo));
}

// q holds the particle's stored position and id; with WPOS they are also
// written to slot i (a caller whose arrays do not hold them yet), the
// position of a deleted particle unchanged.
template <typename S, bool WPOS = false, typename CNT>
__device__ __forceinline__ void advect_one(const GridP& g, const GasP& gas, const BcP& bc,
                                           double dt, const PartP<S>& p, int64_t i,
                                           const PartPos<S>& q, S cx0, S cy0, S cz0, S er0,
                                           int lv0, uint64_t seed, uint32_t step,
                                           CNT counters) {
  // body-force kick, rounded to storage as the state is, then the flight
  double cx = (double)(S)((double)cx0 + bc.g[0] * dt);
  double cy = (double)(S)((double)cy0 + bc.g[1] * dt);
  double cz = (double)(S)((double)cz0 + bc.g[2] * dt);
  double x = g.dim == 2 ? (double)q.x : 0.0, y = (double)q.y;
  double er = (double)er0;
  int lv = lv0;
  const double xlo = (double)(S)g.x0, xhi = (double)edge<S>(g.x0, g.dx, g.nx);
  const double ylo = (double)(S)g.y0, yhi = (double)edge<S>(g.y0, g.dy, g.ny);
  double t = dt;
  int bounces = 0, events = 0;
  bool deleted = false;
  uint32_t ev = 0;
  const uint32_t id = q.pid;
  if (WPOS) p.pid[i] = id;
  for (;;) {
    double th = INFINITY;
    int side = -1;
    if (g.dim == 2) {
      if (cx < 0.0 && x + cx * t < xlo) { const double tt = (xlo - x) / cx; if (tt < th) { th = tt; side = USP_SIDE_XLO; } }
      if (cx > 0.0 && x + cx * t >= xhi) { const double tt = (xhi - x) / cx; if (tt < th) { th = tt; side = USP_SIDE_XHI; } }
    }
    if (cy < 0.0 && y + cy * t < ylo) { const double tt = (ylo - y) / cy; if (tt < th) { th = tt; side = USP_SIDE_YLO; } }
    if (cy > 0.0 && y + cy * t >= yhi) { const double tt = (yhi - y) / cy; if (tt < th) { th = tt; side = USP_SIDE_YHI; } }
    // the body can only be reached within t if |p| <= r + |c| t, and
    // |c| <= |cx| + |cy|: a cheap, slightly widened pre-test (the exact
    // test below decides)
    const double px = x - bc.cyl_xc, py = y - bc.cyl_yc;
    const double reach = bc.cyl_r + (fabs(cx) + fabs(cy)) * t;
    if (g.dim == 2 && bc.cyl && px * px + py * py <= reach * reach * (1.0 + 1e-9)) {
      const double A = cx * cx + cy * cy, B = px * cx + py * cy;
      const double C = px * px + py * py - bc.cyl_r * bc.cyl_r;
      if (B < 0.0 && A > 0.0) {
        double tt = -1.0;
        if (C <= 0.0) tt = 0.0;
        else {
          const double disc = B * B - A * C;
          if (disc > 0.0) tt = (-B - sqrt(disc)) / A;
        }
        if (tt >= 0.0 && tt <= t && tt < th) { th = tt; side = 4; }
      }
    }
    if (side < 0) { x += cx * t; y += cy * t; break; }
    if (th < 0.0) th = 0.0;
    if (th > t) th = t;
    x += cx * th;
    y += cy * th;
    t -= th;
    if (++events > 4 * MAX_BOUNCE) { ev |= 1u << USP_CNT_BOUNCE_LIMIT; break; }
    const int kind = side == 4 ? USP_BC_DIFFUSE : bc.kind[side];
    if (side == USP_SIDE_XLO) x = xlo;
    if (side == USP_SIDE_XHI) x = xhi;
    if (side == USP_SIDE_YLO) y = ylo;
    if (side == USP_SIDE_YHI) y = yhi;
    if (kind == USP_BC_FREESTREAM || kind == USP_BC_OUTFLOW) { deleted = true; break; }
    if (kind == USP_BC_PERIODIC) {
      if (side == USP_SIDE_XLO) x = xhi;
      else if (side == USP_SIDE_XHI) x = xlo;
      else if (side == USP_SIDE_YLO) y = yhi;
      else y = ylo;
      continue;
    }
    if (kind == USP_BC_SPECULAR) {
      if (side == USP_SIDE_XLO || side == USP_SIDE_XHI) cx = -cx; else cy = -cy;
      continue;
    }
    if (bounces >= MAX_BOUNCE) { ev |= 1u << USP_CNT_BOUNCE_LIMIT; break; }
    double cn, ta, tb, ner;
    int nlv;
    const double Tw = side == 4 ? bc.cyl_Tw : bc.Tw[side];
    wall_draw(gas, Tw, seed, id, step, bounces, &cn, &ta, &tb, &ner, &nlv);
    ++bounces;
    const double cix = cx, ciy = cy, ciz = cz, eri = er;
    const int lvi = lv;
    er = ner;
    lv = nlv;
    double nxv = 0.0, nyv = 0.0;
    if (side == USP_SIDE_YLO || side == USP_SIDE_YHI) {
      cy = side == USP_SIDE_YLO ? cn : -cn;
      cx = ta; cz = tb;
    } else if (side == USP_SIDE_XLO || side == USP_SIDE_XHI) {
      cx = side == USP_SIDE_XLO ? cn : -cn;
      cy = ta; cz = tb;
    } else {
      nxv = x - bc.cyl_xc;
      nyv = y - bc.cyl_yc;
      const double nn = sqrt(nxv * nxv + nyv * nyv);
      nxv /= nn;
      nyv /= nn;
      x = bc.cyl_xc + bc.cyl_r * nxv;
      y = bc.cyl_yc + bc.cyl_r * nyv;
      cx = cn * nxv - ta * nyv;
      cy = cn * nyv + ta * nxv;
      cz = tb;
    }
    if (bc.surf)
      surf_record(g, bc, side, x, y, nxv, nyv, cix, ciy, ciz, eri, lvi, cx, cy, cz, er, lv);
  }
  if (deleted) {
    // a deleted particle keeps its position and its values before the flight
    p.cell[i] = -1;
    p.cx[i] = cx0; p.cy[i] = cy0; p.cz[i] = cz0; p.erot[i] = er0; p.vib[i] = (uint8_t)lv0;
    if (WPOS) {
      if (g.dim == 2) p.x[i] = q.x;
      p.y[i] = q.y;
    }
    ev |= 1u << USP_CNT_DELETED;
  } else {
    S xs = S(0);
    if (g.dim == 2) { xs = settle<S>(x, xlo, xhi); p.x[i] = xs; }
    const S ys = settle<S>(y, ylo, yhi);
    p.y[i] = ys;
    p.cx[i] = (S)cx;
    p.cy[i] = (S)cy;
    p.cz[i] = (S)cz;
    p.erot[i] = (S)er;
    p.vib[i] = (uint8_t)lv;
    p.cell[i] = cell_of<S>(g, xs, ys);
  }
  flush_events(counters, ev, USP_CNT_WALL_HITS, bounces);
}

}  // namespace usp
