// usp_cell.h -- per-cell device functions: the moments of a cell on a row
// of 16 lanes and the cell state with its packed record.  Shared by the
// phase kernels and the batched (0D) kernel.
#pragma once
#include "usp_device.h"

namespace usp {

// Moments of one cell (Sec. II.A): U = <c>, then central second and third
// moments about U, per unit mass.  One pass over 16 lanes per cell: sums of
// d = c - c_0 (c_0 = the cell's first particle; d is of the order of the
// thermal speed, and for an FP32 state it is exact in FP64, while for an
// FP64 state it carries one rounding) and of its products, turned into
// central moments with m = <d>:
//   sum C_i C_j = S_ij - N m_i m_j,
//   sum |C|^2 C_i = S3_i - m_i tr S - 2 (S m)_i + 2 N |m|^2 m_i,
//   sum C_i e = S_ie - m_i sum e.
// FP64 sums reduced by a fixed butterfly (deterministic).
// One particle's inputs held in the state precision while its loads are in
// flight (half the registers of FP64 for an FP32 state); widened exactly
// when summed.
template <typename PS>
struct MomIn {
  PS c0, c1, c2, e;
  uint32_t I;
};

template <typename PS>
__device__ __forceinline__ MomIn<PS> mom_load(const PS* cx, const PS* cy, const PS* cz,
                                              const PS* er, const uint8_t* vb, int64_t i) {
  return MomIn<PS>{cx[i], cy[i], cz[i], er[i], (uint32_t)vb[i]};
}

template <typename PS>
__device__ __forceinline__ void mom_add(const MomIn<PS>& a, double r0, double r1, double r2,
                                        double* s) {
  const double d0 = (double)a.c0 - r0, d1 = (double)a.c1 - r1, d2 = (double)a.c2 - r2;
  const double e = (double)a.e, I = (double)a.I;
  const double q = d0 * d0 + d1 * d1 + d2 * d2;
  s[0] += d0; s[1] += d1; s[2] += d2;
  s[3] += d0 * d0; s[4] += d1 * d1; s[5] += d2 * d2;
  s[6] += d0 * d1; s[7] += d0 * d2; s[8] += d1 * d2;
  s[9] += q * d0; s[10] += q * d1; s[11] += q * d2;
  s[12] += e; s[13] += d0 * e; s[14] += d1 * e; s[15] += d2 * e;
  s[16] += I; s[17] += d0 * I; s[18] += d1 * I; s[19] += d2 * I;
}

constexpr int MOM_LANES = 16;

__device__ __forceinline__ void moments_from_sums(const double s[20], int64_t N, double r0,
                                                  double r1, double r2, double v[NMOM]);

// The NMOM moments of the particles [o0, o1) (array indices) on one row of
// 16 lanes (sub = lane in the row; all 16 lanes call); every lane of the
// row returns the same v.  With G, slot i is the particle perm[i] of the
// arrays (a binning that left the particles in place).
template <typename PS, bool G = false>
__device__ __forceinline__ void row_moments(const PS* cx, const PS* cy, const PS* cz,
                                            const PS* er, const uint8_t* vb, int64_t o0,
                                            int64_t o1, int sub, double v[NMOM],
                                            const uint32_t* perm = nullptr) {
  const int64_t N = o1 - o0;
  auto at = [&](int64_t i) -> int64_t {
    if constexpr (G) return (int64_t)perm[i];
    else return i;
  };
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (N > 0) {
    const int64_t j = at(o0);
    r0 = (double)cx[j]; r1 = (double)cy[j]; r2 = (double)cz[j];
  }
  double s[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) s[k] = 0.0;
  // a lane takes i, i + 16, i + 32, ... in order; four at a time (all
  // loads issued before the sums), then the rest one at a time
  int64_t i = o0 + sub;
  for (; i + 3 * MOM_LANES < o1; i += 4 * MOM_LANES) {
    int64_t j[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) j[k] = at(i + k * MOM_LANES);
    MomIn<PS> a[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] = mom_load<PS>(cx, cy, cz, er, vb, j[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) mom_add(a[k], r0, r1, r2, s);
  }
  for (; i < o1; i += MOM_LANES) mom_add(mom_load<PS>(cx, cy, cz, er, vb, at(i)), r0, r1, r2, s);
#pragma unroll
  for (int k = 0; k < 20; ++k) s[k] = row16_sum(s[k]);
  moments_from_sums(s, N, r0, r1, r2, v);
}

// The NMOM moments of N particles from their 20 sums shifted by (r0, r1,
// r2) (the first particle's velocity): the sums of d, d_i d_j, |d|^2 d_i,
// e, d_i e, I, d_i I of mom_add.
__device__ __forceinline__ void moments_from_sums(const double s[20], int64_t N, double r0,
                                                  double r1, double r2, double v[NMOM]) {
  if (N == 0) {
#pragma unroll
    for (int k = 0; k < NMOM; ++k) v[k] = 0.0;
    return;
  }
  const double Nd = (double)N, invN = 1.0 / Nd;
  const double m[3] = {s[0] * invN, s[1] * invN, s[2] * invN};
  const double Sm[3] = {s[3] * m[0] + s[6] * m[1] + s[7] * m[2],
                        s[6] * m[0] + s[4] * m[1] + s[8] * m[2],
                        s[7] * m[0] + s[8] * m[1] + s[5] * m[2]};
  const double tr = s[3] + s[4] + s[5], mm = m[0] * m[0] + m[1] * m[1] + m[2] * m[2];
  v[M_N] = Nd;
  v[M_UX] = r0 + m[0]; v[M_UY] = r1 + m[1]; v[M_UZ] = r2 + m[2];
  v[M_PXX] = s[3] * invN - m[0] * m[0];
  v[M_PYY] = s[4] * invN - m[1] * m[1];
  v[M_PZZ] = s[5] * invN - m[2] * m[2];
  v[M_PXY] = s[6] * invN - m[0] * m[1];
  v[M_PXZ] = s[7] * invN - m[0] * m[2];
  v[M_PYZ] = s[8] * invN - m[1] * m[2];
  v[M_EROT] = s[12] * invN;
  v[M_IBAR] = s[16] * invN;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[M_QTRX + k] = 0.5 * (s[9 + k] - m[k] * tr - 2.0 * Sm[k] + 2.0 * Nd * mm * m[k]) * invN;
    v[M_QROTX + k] = (s[13 + k] - m[k] * s[12]) * invN;
    v[M_QIX + k] = (s[17 + k] - m[k] * s[16]) * invN;
  }
}

// Lane sub of the row stores moments sub and sub + 16 of cell c.
__device__ __forceinline__ void store_moments(double* mom, int64_t M, int64_t c, int sub,
                                              const double v[NMOM]) {
  double w0 = 0.0, w1 = 0.0;
#pragma unroll
  for (int k = 0; k < NMOM; ++k) {
    if (k == sub) w0 = v[k];
    if (k == sub + MOM_LANES) w1 = v[k];
  }
  mom[sub * M + c] = w0;
  if (sub + MOM_LANES < NMOM) mom[(sub + MOM_LANES) * M + c] = w1;
}

// Per-cell state (Secs. II.A, III.A.1, III.A.2, IV.A, IV.B) of cell c from
// its moments m: temperatures, viscosity, tau_c, Z's, Pr, alpha, nu, a, b,
// the energy targets, and the collide / stencil-usable flags.
__device__ __forceinline__ void cell_state(const GridP& g, const GasP& gas, const double m[NMOM],
                                           int64_t c, double dtc, double v[NCS],
                                           int64_t* counters) {
  const double R = gas.R, Th = gas.theta;
#pragma unroll
  for (int k = 0; k < NCS; ++k) v[k] = 0.0;
  const double N = m[M_N];
  const double vol = g.volume[c];
  v[CS_NP] = N;
  v[CS_NDENS] = vol > 0.0 ? N * g.fnum / vol : 0.0;
  v[CS_UX] = m[M_UX];
  v[CS_UY] = m[M_UY];
  v[CS_UZ] = m[M_UZ];
#pragma unroll
  for (int k = 0; k < 6; ++k) v[CS_PXX + k] = m[M_PXX + k];
  const double trP = v[CS_PXX] + v[CS_PYY] + v[CS_PZZ];
  const double ibar = m[M_IBAR];
  const double erot = m[M_EROT];
  const double Ttr = trP / (3.0 * R), Trot = erot / R;
  const double Tvib = ibar > 0.0 ? Th / log1p(1.0 / ibar) : 0.0;
  v[CS_TTR] = Ttr; v[CS_TROT] = Trot; v[CS_TVIB] = Tvib;
  v[CS_ETR] = 0.5 * trP; v[CS_EROT] = erot; v[CS_EVIB] = ibar * R * Th;
  v[CS_DT] = dtc;
  // a NaN or infinite velocity or rotational energy in the cell makes its
  // sums non-finite: such a cell is not collided, and it is counted
  const bool finite = isfinite(v[CS_UX]) && isfinite(v[CS_UY]) && isfinite(v[CS_UZ]) &&
                      isfinite(trP) && isfinite(erot);
  if (N >= 1.0 && !finite) count_event(counters, USP_CNT_NONFINITE);
  const bool collide = N >= 2.0 && Ttr > 0.0 && finite && vol > 0.0;
  if (collide && gas.scheme == USP_SCHEME_FPM) {
    // first-order FPM (Secs. II.B-II.C): nu from Pr, tau = 2 mu (1-nu)/p,
    // the update factor exp(-dt/tau) and the cell relaxation temperatures
    // of eqs. T_tr_FPM, T_rot_FPM, T_vib_FPM
    const double mu = gas.mu_ref * pow(Ttr / gas.T_ref, gas.omega);
    const double mup = mu / (v[CS_NDENS] * KB * Ttr);
    const double tauc = gas.K * mup;
    const double zr = zrot(gas, Ttr), zv = zvib(gas, Ttr);
    const double Pr = prandtl(gas, Ttr);
    const double nu = 1.0 - 3.0 / (2.0 * Pr);
    const double tau = 2.0 * mup * (1.0 - nu);
    const double fr = tau / (2.0 * zr * tauc), fv = tau / (2.0 * zv * tauc);
    const double mv = mlevel<double>(Th, Tvib), mt = mlevel<double>(Th, Ttr);
    v[CS_MU] = mu; v[CS_MUP] = mup; v[CS_TAUC] = tauc;
    v[CS_ZROT] = zr; v[CS_ZVIB] = zv; v[CS_PR] = Pr;
    v[CS_ALPHA] = exp(-dtc / tau);
    v[CS_OMA2] = -expm1(-2.0 * dtc / tau);
    v[CS_NU] = nu;
    v[CS_EROT_NEW] = erot;
    v[CS_EVIB_NEW] = v[CS_EVIB];
    v[CS_FPM_TAU] = tau;
    v[CS_FPM_TTR_REL] = Ttr + (2.0 / 3.0) * (fr * (Trot - Ttr) + fv * Th * (mv - mt));
    v[CS_FPM_TROT_REL] = Trot + fr * (Ttr - Trot);
    v[CS_FPM_MREL] = mv + fv * (mt - mv);
    v[CS_COLLIDE] = 1.0;
    const int cut = g.flags ? (g.flags[c] & (USP_FLAG_SOLID | USP_FLAG_CUT)) : 0;
    v[CS_NBR_OK] = cut ? 0.0 : 1.0;
  } else if (collide) {
    const double mu = gas.mu_ref * pow(Ttr / gas.T_ref, gas.omega);
    const double mup = mu / (v[CS_NDENS] * KB * Ttr);
    const double tauc = gas.K * mup;
    const double zr = zrot(gas, Ttr), zv = zvib(gas, Ttr);
    const double Pr = prandtl(gas, Ttr);
    const double A = 2.0 * mup;
    const double r3 = (A - Pr * dtc) / (A + Pr * dtc);
    const double r2 = (A - dtc) / (A + dtc);
    const double al = cbrt(r3);
    // 1 - alpha^2 = (1 - r3)(1 + alpha)/(1 + alpha + alpha^2), no cancellation
    const double oma2 = (2.0 * Pr * dtc / (A + Pr * dtc)) * (1.0 + al) / (1.0 + al + al * al);
    const double nu = (r2 - al * al) / oma2;
    const double a = dtc / (dtc + 2.0 * zr * tauc);
    const double b = dtc / (dtc + 2.0 * zv * tauc);
    const double Tc = tcheck<double>(Th, Ttr, Trot, Tvib, a, b);
    const double cb = cbar_R<double>(Th, Tc, Tvib);
    const double D = 1.5 + a + b * cb;
    const double g1 = 3.0 * a / D, g2 = 3.0 * b * cb / D, g3 = 2.0 * a * b * cb / D;
    v[CS_MU] = mu; v[CS_MUP] = mup; v[CS_TAUC] = tauc;
    v[CS_ZROT] = zr; v[CS_ZVIB] = zv; v[CS_PR] = Pr;
    v[CS_A] = a; v[CS_B] = b; v[CS_R2] = r2; v[CS_R3] = r3;
    v[CS_ALPHA] = al; v[CS_OMA2] = oma2; v[CS_NU] = nu;
    v[CS_EROT_NEW] = erot + R * (g1 * (Ttr - Trot) - g3 * (Trot - Tvib));
    v[CS_EVIB_NEW] = v[CS_EVIB] + R * (g2 * (Ttr - Tvib) + g3 * (Trot - Tvib));
    v[CS_COLLIDE] = 1.0;
    const int cut = g.flags ? (g.flags[c] & (USP_FLAG_SOLID | USP_FLAG_CUT)) : 0;
    v[CS_NBR_OK] = cut ? 0.0 : 1.0;
  } else if (N >= 1.0) {
    count_event(counters, USP_CNT_CELL_SKIP);
  }
}

// The FP64 planes of cell c and its packed record (stencil word 0; the
// stencil pass fills it in 1D and 2D).
__device__ __forceinline__ void store_cell_state(double* cs, int64_t M, int64_t c,
                                                 const double v[NCS]) {
#pragma unroll
  for (int k = 0; k < NCS; ++k) cs[k * M + c] = v[k];
  CellRec r;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    r.U[k] = (float)v[CS_UX + k];
    r.T[k] = (float)v[CS_TTR + k];
    r.fl[k] = (float)(0.05 * v[CS_TTR + k]);
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) r.P[k] = (float)v[CS_PXX + k];
  r.stencil = 0;
  r.a = (float)v[CS_A]; r.b = (float)v[CS_B]; r.al = (float)v[CS_ALPHA]; r.nu = (float)v[CS_NU];
  r.oma2 = v[CS_OMA2]; r.r2 = v[CS_R2]; r.A2 = 2.0 * v[CS_MUP]; r.Pr = v[CS_PR]; r.dt = v[CS_DT];
  r.collide = v[CS_COLLIDE] != 0.0 ? 1 : 0;
  r.pad = 0;
  cell_records(cs, M)[c] = r;
}

}  // namespace usp
