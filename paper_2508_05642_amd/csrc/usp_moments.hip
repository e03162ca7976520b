// usp_moments.hip -- per-cell moments and the per-cell USP-FPM state.
#include "usp_device.h"

namespace usp {

constexpr int CELL_BLOCK = 256;

// Moments of one cell (Sec. II.A): U = <c>, then central second and third
// moments about U, per unit mass.  One wave per cell and one pass: sums of
// d = c - c_0 (c_0 = the cell's first particle, so every d is exact in
// FP64 and of the order of the thermal speed) and of its products, turned
// into central moments with m = <d>:
//   sum C_i C_j = S_ij - N m_i m_j,
//   sum |C|^2 C_i = S3_i - m_i tr S - 2 (S m)_i + 2 N |m|^2 m_i,
//   sum C_i e = S_ie - m_i sum e.
// FP64 sums reduced by a fixed butterfly (deterministic).
template <typename S>
__device__ __forceinline__ void mom_add(const PartP<S>& p, int64_t i, double r0, double r1,
                                        double r2, double* s) {
  const double d0 = (double)p.cx[i] - r0, d1 = (double)p.cy[i] - r1, d2 = (double)p.cz[i] - r2;
  const double e = (double)p.erot[i], I = (double)p.vib[i];
  const double q = d0 * d0 + d1 * d1 + d2 * d2;
  s[0] += d0; s[1] += d1; s[2] += d2;
  s[3] += d0 * d0; s[4] += d1 * d1; s[5] += d2 * d2;
  s[6] += d0 * d1; s[7] += d0 * d2; s[8] += d1 * d2;
  s[9] += q * d0; s[10] += q * d1; s[11] += q * d2;
  s[12] += e; s[13] += d0 * e; s[14] += d1 * e; s[15] += d2 * e;
  s[16] += I; s[17] += d0 * I; s[18] += d1 * I; s[19] += d2 * I;
}

// 16 lanes per cell, four cells per wave (every lane stays active for the
// row permutes; lanes of cells past M carry zeros).
constexpr int MOM_LANES = 16;

template <typename S>
__global__ __launch_bounds__(CELL_BLOCK) void k_moments(GridP g, PartP<S> p, const int64_t* offsets,
                                                        double* mom) {
  const int64_t M = g.M;
  const int64_t c = ((int64_t)blockIdx.x * CELL_BLOCK + threadIdx.x) / MOM_LANES;
  const int sub = threadIdx.x & (MOM_LANES - 1);
  const bool valid = c < M;
  const int64_t o0 = valid ? offsets[c] : 0, o1 = valid ? offsets[c + 1] : 0, N = o1 - o0;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (N > 0) { r0 = (double)p.cx[o0]; r1 = (double)p.cy[o0]; r2 = (double)p.cz[o0]; }
  double s[20];
#pragma unroll
  for (int k = 0; k < 20; ++k) s[k] = 0.0;
  int64_t i = o0 + sub;
  for (; i + MOM_LANES < o1; i += 2 * MOM_LANES) {
    mom_add<S>(p, i, r0, r1, r2, s);
    mom_add<S>(p, i + MOM_LANES, r0, r1, r2, s);
  }
  if (i < o1) mom_add<S>(p, i, r0, r1, r2, s);
#pragma unroll
  for (int k = 0; k < 20; ++k) s[k] = row16_sum(s[k]);
  if (!valid) return;
  double v[NMOM];
  if (N == 0) {
#pragma unroll
    for (int k = 0; k < NMOM; ++k) v[k] = 0.0;
  } else {
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
  // lane k of the row stores moments k and k + 16
  double w0 = 0.0, w1 = 0.0;
#pragma unroll
  for (int k = 0; k < NMOM; ++k) {
    if (k == sub) w0 = v[k];
    if (k == sub + MOM_LANES) w1 = v[k];
  }
  mom[sub * M + c] = w0;
  if (sub + MOM_LANES < NMOM) mom[(sub + MOM_LANES) * M + c] = w1;
}

// Per-cell state (Secs. II.A, III.A.1, III.A.2, IV.A, IV.B).
__global__ void k_reconstruct(GridP g, GasP gas, const double* mom, double dt,
                              const double* dt_cell, double* cs, int64_t* counters) {
  const int64_t M = g.M;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  const double R = gas.R, Th = gas.theta;
  double v[NCS];
#pragma unroll
  for (int k = 0; k < NCS; ++k) v[k] = 0.0;
  const double N = mom[M_N * M + c];
  const double vol = g.volume[c];
  v[CS_NP] = N;
  v[CS_NDENS] = vol > 0.0 ? N * g.fnum / vol : 0.0;
  v[CS_UX] = mom[M_UX * M + c];
  v[CS_UY] = mom[M_UY * M + c];
  v[CS_UZ] = mom[M_UZ * M + c];
#pragma unroll
  for (int k = 0; k < 6; ++k) v[CS_PXX + k] = mom[(M_PXX + k) * M + c];
  const double trP = v[CS_PXX] + v[CS_PYY] + v[CS_PZZ];
  const double ibar = mom[M_IBAR * M + c];
  const double erot = mom[M_EROT * M + c];
  const double Ttr = trP / (3.0 * R), Trot = erot / R;
  const double Tvib = ibar > 0.0 ? Th / log1p(1.0 / ibar) : 0.0;
  v[CS_TTR] = Ttr; v[CS_TROT] = Trot; v[CS_TVIB] = Tvib;
  v[CS_ETR] = 0.5 * trP; v[CS_EROT] = erot; v[CS_EVIB] = ibar * R * Th;
  const double dtc = dt_cell ? dt_cell[c] : dt;
  v[CS_DT] = dtc;
  const bool collide = N >= 2.0 && Ttr > 0.0 && isfinite(Ttr) && vol > 0.0;
  if (collide) {
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

// Quadrant stencils of the reconstruction (Sec. III.B), one thread per
// cell, after the cell state: quadrant q = (x >= x_i) + 2 (y >= y_j) keeps
// the x neighbour direction tx and y direction ty (toward the quadrant,
// else the opposite side, else none) and whether the diagonal cell
// completes the cross term.  Field: 2 bits tx (1: +1, 2: -1), 2 bits ty,
// 1 bit cross, 5 bits per quadrant.
__global__ void k_stencil(GridP g, double* cs) {
  const int64_t M = g.M;
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M || g.dim == 0) return;
  const int nx = g.nx;
  const int ci = g.dim == 2 ? (int)(c % nx) : 0;
  const int cj = g.dim == 2 ? (int)(c / nx) : (int)c;
  auto ok = [&](int ii, int jj) -> bool {
    if (ii < 0 || jj < 0 || ii >= g.nx || jj >= g.ny) return false;
    return cs[CS_NBR_OK * M + (int64_t)jj * nx + ii] != 0.0;
  };
  int32_t bits = 0;
  for (int q = 0; q < 4; ++q) {
    const int sx = (q & 1) ? 1 : -1, sy = (q & 2) ? 1 : -1;
    int ty = 0, tx = 0;
    if (ok(ci, cj + sy)) ty = sy;
    else if (ok(ci, cj - sy)) ty = -sy;
    if (g.dim == 2) {
      if (ok(ci + sx, cj)) tx = sx;
      else if (ok(ci - sx, cj)) tx = -sx;
    }
    const int cross = (tx && ty && ok(ci + tx, cj + ty)) ? 1 : 0;
    const int f = (tx == 1 ? 1 : tx == -1 ? 2 : 0) | ((ty == 1 ? 1 : ty == -1 ? 2 : 0) << 2) | (cross << 4);
    bits |= f << (5 * q);
  }
  cell_records(cs, M)[c].stencil = bits;
}

template <typename S>
hipError_t launch_moments(const GridP& g, const PartP<S>& p, const int64_t* offsets, double* mom,
                          hipStream_t st) {
  k_moments<S><<<cdiv(g.M * MOM_LANES, CELL_BLOCK), CELL_BLOCK, 0, st>>>(g, p, offsets, mom);
  return hipGetLastError();
}

hipError_t launch_reconstruct(const GridP& g, const GasP& gas, const double* mom, double dt,
                              const double* dt_cell, double* cs, int64_t* counters, hipStream_t st) {
  k_reconstruct<<<cdiv(g.M, 128), 128, 0, st>>>(g, gas, mom, dt, dt_cell, cs, counters);
  k_stencil<<<cdiv(g.M, 256), 256, 0, st>>>(g, cs);
  return hipGetLastError();
}

template hipError_t launch_moments<float>(const GridP&, const PartP<float>&, const int64_t*,
                                          double*, hipStream_t);
template hipError_t launch_moments<double>(const GridP&, const PartP<double>&, const int64_t*,
                                           double*, hipStream_t);

}  // namespace usp
