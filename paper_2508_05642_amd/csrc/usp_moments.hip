// usp_moments.hip -- per-cell moments and the per-cell USP-FPM state.
#include "usp_device.h"

namespace usp {

constexpr int CELL_BLOCK = 256;
constexpr int CELL_WAVES = CELL_BLOCK / 64;

// Moments of one cell (Sec. II.A): U = <c>, then central second and third
// moments about U, per unit mass.  One wave per cell, two passes over its
// particles, FP64 sums reduced by a fixed butterfly (deterministic).
template <typename S>
__global__ __launch_bounds__(CELL_BLOCK) void k_moments(GridP g, PartP<S> p, const int64_t* offsets,
                                                        double* mom) {
  const int64_t M = g.M;
  const int64_t c = (int64_t)blockIdx.x * CELL_WAVES + (threadIdx.x >> 6);
  if (c >= M) return;
  const int lane = threadIdx.x & 63;
  const int64_t o0 = offsets[c], o1 = offsets[c + 1], N = o1 - o0;
  if (N == 0) {
    if (lane < NMOM) mom[lane * M + c] = 0.0;
    return;
  }
  double s1[3] = {0.0, 0.0, 0.0};
  for (int64_t i = o0 + lane; i < o1; i += 64) {
    s1[0] += (double)p.cx[i];
    s1[1] += (double)p.cy[i];
    s1[2] += (double)p.cz[i];
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) s1[k] = wave_sum(s1[k]);
  const double invN = 1.0 / (double)N;
  const double Ux = s1[0] * invN, Uy = s1[1] * invN, Uz = s1[2] * invN;
  double s[17];
#pragma unroll
  for (int k = 0; k < 17; ++k) s[k] = 0.0;
  for (int64_t i = o0 + lane; i < o1; i += 64) {
    const double Cx = (double)p.cx[i] - Ux, Cy = (double)p.cy[i] - Uy, Cz = (double)p.cz[i] - Uz;
    const double e = (double)p.erot[i], I = (double)p.vib[i];
    const double hC2 = 0.5 * (Cx * Cx + Cy * Cy + Cz * Cz);
    s[0] += Cx * Cx; s[1] += Cy * Cy; s[2] += Cz * Cz;
    s[3] += Cx * Cy; s[4] += Cx * Cz; s[5] += Cy * Cz;
    s[6] += e; s[7] += I;
    s[8] += hC2 * Cx; s[9] += hC2 * Cy; s[10] += hC2 * Cz;
    s[11] += Cx * e; s[12] += Cy * e; s[13] += Cz * e;
    s[14] += Cx * I; s[15] += Cy * I; s[16] += Cz * I;
  }
#pragma unroll
  for (int k = 0; k < 17; ++k) s[k] = wave_sum(s[k]);
  if (lane == 0) {
    mom[M_N * M + c] = (double)N;
    mom[M_UX * M + c] = Ux;
    mom[M_UY * M + c] = Uy;
    mom[M_UZ * M + c] = Uz;
  }
  if (lane < 17) {
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 17; ++k)
      if (k == lane) v = s[k];
    mom[(M_PXX + lane) * M + c] = v * invN;
  }
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
  k_moments<S><<<cdiv(g.M, CELL_WAVES), CELL_BLOCK, 0, st>>>(g, p, offsets, mom);
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
