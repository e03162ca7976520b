/*
 * usp_oracle.c -- plain FP64 CPU reference of one USP-FPM time step.
 *
 * TEST INFRASTRUCTURE ONLY (see usp_oracle.h).  Each function follows one
 * passage of arXiv 2508.05642 and is written as directly as possible: plain
 * loops, FP64 everywhere, no blocking or fusion.  Where the paper leaves a
 * detail open, the reading taken is stated at the point of use.
 *
 * Where the state is stored in single precision (f32 = 1), every value
 * written back to a particle array is rounded to float, exactly as a single
 * precision particle store would hold it; all arithmetic stays in FP64.
 */
#include "usp_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846

void orc_set_threads(int32_t n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int32_t orc_get_threads(void) {
#ifdef _OPENMP
  return (int32_t)omp_get_max_threads();
#else
  return 1;
#endif
}

static double store(double v, int32_t f32) { return f32 ? (double)(float)v : v; }

/* ======================================================================== */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11).  Ten rounds of two 32x32->64 multiplies, the   */
/* key advanced by the two Weyl constants between rounds.                   */
/* ======================================================================== */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
  uint32_t k[2] = {key[0], key[1]};
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k[0] += W0;
      k[1] += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c[0];
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c[2];
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c[1] ^ k[0];
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c[3] ^ k[1];
    uint32_t n3 = lo0;
    c[0] = n0; c[1] = n1; c[2] = n2; c[3] = n3;
  }
  out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* Four uniforms in (0,1) from counter (c0, step, tag, block), key = seed.  */
/* u = (w + 1/2) 2^-32 is exact in double.                                  */
static void draw4(uint64_t seed, uint32_t c0, uint64_t step, uint32_t tag, uint32_t block,
                  double u[4]) {
  uint32_t ctr[4] = {c0, (uint32_t)step, tag, block};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  uint32_t w[4];
  orc_philox4x32_10(ctr, key, w);
  for (int i = 0; i < 4; ++i) u[i] = ((double)w[i] + 0.5) * (1.0 / 4294967296.0);
}

/* stream tags */
enum { TAG_COLLIDE = 0, TAG_WALL = 1, TAG_CONSERVE = 2, TAG_INJECT = 3, TAG_FACE = 5 };

/* The four standard normals G1..G4 of the collision update of each       */
/* particle (Box-Muller on block 0 of its collide stream), as orc_collide */
/* draws them: G[4 i + k].                                                 */
void orc_collide_normals(uint64_t seed, uint64_t step, int64_t n, const uint32_t* pid,
                         double* G) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double u[4];
    draw4(seed, pid[i], step, TAG_COLLIDE, 0, u);
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    G[4 * i + 0] = r0 * cos(2.0 * PI * u[1]);
    G[4 * i + 1] = r0 * sin(2.0 * PI * u[1]);
    G[4 * i + 2] = r1 * cos(2.0 * PI * u[3]);
    G[4 * i + 3] = r1 * sin(2.0 * PI * u[3]);
  }
}

/* ======================================================================== */
/* Gas model                                                                */
/* ======================================================================== */
double orc_R(const orc_gas* g) { return ORC_KB / g->m; }

/* Harmonic-oscillator specific vibrational energy (Sec. II.A). */
double orc_e_vib(const orc_gas* g, double T) {
  if (T <= 0.0) return 0.0;
  return orc_R(g) * g->theta_vib / expm1(g->theta_vib / T);
}

/* c_v,vib = d e_vib / dT.  The paper prints the denominator as sinh(x);  */
/* the derivative of e_vib (and the Grad-17 factor of Sec. V.A.1) require */
/* sinh^2(x), which is what is used here.                                 */
double orc_cv_vib(const orc_gas* g, double T) {
  if (T <= 0.0) return 0.0;
  double x = g->theta_vib / (2.0 * T);
  if (x > 300.0) return 0.0;
  double s = sinh(x);
  return orc_R(g) * x * x / (s * s);
}

/* VSS power-law viscosity (Sec. IV.A), evaluated at T_tr. */
double orc_viscosity(const orc_gas* g, double T) { return g->mu_ref * pow(T / g->T_ref, g->omega); }

/* tau_c = K mu/p with K the VSS factor of eq. tau_c (Sec. IV.A). */
double orc_tau_c_factor(const orc_gas* g) {
  double a = g->alpha_vss, w = g->omega;
  return a * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) / (5.0 * (a + 1.0) * (a + 2.0));
}

/* Rotational collision number: constant, or Parker's law (Sec. V.C). */
double orc_zrot(const orc_gas* g, double T) {
  if (g->zrot_model == ORC_ZROT_CONST) return g->Z_rot;
  double r = g->T_star / T;
  return g->Z_rot_inf / (1.0 + 0.5 * pow(PI, 1.5) * sqrt(r) + (PI + 0.25 * PI * PI) * r);
}

/* Vibrational collision number: constant, or Millikan-White plus the     */
/* high-temperature correction (Sec. V.C).                                */
double orc_zvib(const orc_gas* g, double T) {
  if (g->zvib_model == ORC_ZVIB_CONST) return g->Z_vib;
  double mw = (g->C1 / pow(T, g->omega)) * exp(g->C2 * pow(T, -1.0 / 3.0));
  double ht = (PI * g->d_ref * g->d_ref / g->sigma_vib) * pow(g->T_ref / T, g->omega - 0.5);
  return mw + ht;
}

/* Eucken Prandtl number (Sec. IV.B).  "printed": xi = x/(e^x-1) as the  */
/* paper prints it; "standard": xi = 2x/(e^x-1).                          */
double orc_prandtl(const orc_gas* g, double T) {
  if (g->pr_model == ORC_PR_CONST) return g->Pr_const;
  double xi = 0.0;
  if (T > 0.0) {
    double x = g->theta_vib / T;
    xi = (x > 700.0) ? 0.0 : x / expm1(x);
    if (g->pr_model == ORC_PR_EUCKEN_STANDARD) xi *= 2.0;
  }
  return (14.0 + 2.0 * xi) / (19.0 + 2.0 * xi);
}

/* Rescaled translational temperature (Sec. III.A.1).  The paper defines  */
/* it through gamma coefficients that themselves depend on it; the        */
/* consistent reading (App. C, with tau_rot in the rotational bracket) is */
/* the root of the monotone scalar equation                               */
/*   e_tr(T) + a e_rot(T) + b e_vib(T) = e_tr(T_tr) + a e_rot(T_rot)      */
/*                                       + b e_vib(T_vib),                */
/* a = dt/(dt+2 tau_rot), b = dt/(dt+2 tau_vib).  Solved by safeguarded   */
/* Newton on the bracket [0, rhs/((3/2+a)R)].                             */
double orc_tcheck(const orc_gas* g, double Ttr, double Trot, double Tvib, double a, double b) {
  double R = orc_R(g);
  double rhs = 1.5 * R * Ttr + a * R * Trot + b * orc_e_vib(g, Tvib);
  double lo = 0.0, hi = rhs / ((1.5 + a) * R);
  if (!(hi > 0.0)) return 0.0;
  double T = hi;
  for (int it = 0; it < 200; ++it) {
    double f = (1.5 + a) * R * T + b * orc_e_vib(g, T) - rhs;
    if (f > 0.0) hi = T; else lo = T;
    double fp = (1.5 + a) * R + b * orc_cv_vib(g, T);
    double Tn = T - f / fp;
    if (!(Tn > lo && Tn < hi)) Tn = 0.5 * (lo + hi);
    if (fabs(Tn - T) <= 1e-15 * T) { T = Tn; break; }
    T = Tn;
  }
  return T;
}

/* gamma_tr-rot, gamma_tr-vib, gamma_rot-vib (Sec. III.A.1), with c_v,vib */
/* at T_1 taken as the secant of e_vib between T_check and T_vib.  When   */
/* the two temperatures are within 3e-6 relative, the secant is replaced  */
/* by c_v,vib at their midpoint (error O(dT^2), below FP64 rounding of    */
/* the secant there).                                                     */
void orc_gammas(const orc_gas* g, double Ttr, double Trot, double Tvib, double a, double b,
                double out[3], double* out_tcheck) {
  double R = orc_R(g);
  double cvt = 1.5 * R, cvr = R;
  double Tc = orc_tcheck(g, Ttr, Trot, Tvib, a, b);
  double cbar;
  if (fabs(Tc - Tvib) <= 3e-6 * fmax(Tc, Tvib))
    cbar = orc_cv_vib(g, 0.5 * (Tc + Tvib));
  else
    cbar = (orc_e_vib(g, Tc) - orc_e_vib(g, Tvib)) / (Tc - Tvib);
  double D = cvt + a * cvr + b * cbar;
  out[0] = 2.0 * a * cvt * cvr / D;
  out[1] = 2.0 * b * cvt * cbar / D;
  out[2] = 2.0 * a * b * cvr * cbar / D;
  if (out_tcheck) *out_tcheck = Tc;
}

/* Eigenvalues of a symmetric 3x3 matrix, ascending (trigonometric closed  */
/* form).  P = (xx, yy, zz, xy, xz, yz).                                   */
void orc_eigvals_sym3(const double P[6], double out[3]) {
  double a11 = P[0], a22 = P[1], a33 = P[2], a12 = P[3], a13 = P[4], a23 = P[5];
  double p1 = a12 * a12 + a13 * a13 + a23 * a23;
  if (p1 == 0.0) {
    double e[3] = {a11, a22, a33};
    for (int i = 0; i < 3; ++i)
      for (int j = i + 1; j < 3; ++j)
        if (e[j] < e[i]) { double t = e[i]; e[i] = e[j]; e[j] = t; }
    out[0] = e[0]; out[1] = e[1]; out[2] = e[2];
    return;
  }
  double q = (a11 + a22 + a33) / 3.0;
  double p2 = (a11 - q) * (a11 - q) + (a22 - q) * (a22 - q) + (a33 - q) * (a33 - q) + 2.0 * p1;
  double p = sqrt(p2 / 6.0);
  double b11 = (a11 - q) / p, b22 = (a22 - q) / p, b33 = (a33 - q) / p;
  double b12 = a12 / p, b13 = a13 / p, b23 = a23 / p;
  double det = b11 * (b22 * b33 - b23 * b23) - b12 * (b12 * b33 - b23 * b13) +
               b13 * (b12 * b23 - b22 * b13);
  double r = det / 2.0;
  if (r < -1.0) r = -1.0;
  if (r > 1.0) r = 1.0;
  double phi = acos(r) / 3.0;
  double l1 = q + 2.0 * p * cos(phi);
  double l3 = q + 2.0 * p * cos(phi + 2.0 * PI / 3.0);
  double l2 = 3.0 * q - l1 - l3;
  out[0] = l3; out[1] = l2; out[2] = l1;
}

/* ======================================================================== */
/* Grid geometry                                                            */
/* ======================================================================== */
static int64_t ncells(const orc_grid* gr) { return (int64_t)gr->nx * gr->ny; }

/* Edge k of an axis, in the precision the positions are stored in. */
static double edge(double o, double d, int k, int32_t f32) {
  double e = o + (double)k * d;
  return store(e, f32);
}

/* Index along an axis: the number of interior edges e_1..e_{n-1} at or   */
/* below v; -1 if v lies outside [e_0, e_n).  Edges are monotone, so the  */
/* count is found by bisection.                                           */
static int axis_index(double v, double o, double d, int n, int32_t f32) {
  if (!(v >= edge(o, d, 0, f32)) || v >= edge(o, d, n, f32)) return -1;
  int lo = 0, hi = n - 1; /* answer in [lo, hi] */
  while (lo < hi) {
    int mid = (lo + hi + 1) / 2;
    if (edge(o, d, mid, f32) <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

static int32_t cell_of(const orc_grid* gr, double x, double y, int32_t f32) {
  if (gr->dim == 1) return axis_index(y, gr->y0, gr->dy, gr->ny, f32);
  int ix = axis_index(x, gr->x0, gr->dx, gr->nx, f32);
  int iy = axis_index(y, gr->y0, gr->dy, gr->ny, f32);
  if (ix < 0 || iy < 0) return -1;
  return iy * gr->nx + ix;
}

/* ======================================================================== */
/* Bin: cell of every particle, stable counting sort by cell.               */
/* Particles marked -1 (left the domain) or found in a solid cell are       */
/* dropped.  In dim 0 the cell array is the problem id and is kept.         */
/* ======================================================================== */
int orc_bin(const orc_grid* gr, const orc_parts* src, orc_parts* dst, int64_t* offsets,
            int32_t f32, int64_t* counters) {
  int64_t M = ncells(gr), n = src->n;
  int32_t* key = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  if (!key) return -1;
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = src->cell[i];
    if (c >= 0) {
      if (gr->dim == 0) {
        if (c >= M) { free(key); return -1; }
      } else {
        c = cell_of(gr, src->x ? src->x[i] : 0.0, src->y[i], f32);
      }
    }
    if (c >= 0 && gr->flags && (gr->flags[c] & ORC_FLAG_SOLID)) {
      c = -1;
      if (counters) counters[ORC_CNT_SOLID_DROP] += 1;
    }
    key[i] = c;
  }
  for (int64_t c = 0; c <= M; ++c) offsets[c] = 0;
  for (int64_t i = 0; i < n; ++i)
    if (key[i] >= 0) offsets[key[i] + 1] += 1;
  for (int64_t c = 0; c < M; ++c) offsets[c + 1] += offsets[c];
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(M > 0 ? M : 1));
  if (!fill) { free(key); return -1; }
  for (int64_t c = 0; c < M; ++c) fill[c] = offsets[c];
  for (int64_t i = 0; i < n; ++i) {
    int32_t c = key[i];
    if (c < 0) continue;
    int64_t j = fill[c]++;
    if (src->x && dst->x) dst->x[j] = src->x[i];
    if (src->y && dst->y) dst->y[j] = src->y[i];
    dst->cx[j] = src->cx[i];
    dst->cy[j] = src->cy[i];
    dst->cz[j] = src->cz[i];
    dst->erot[j] = src->erot[i];
    dst->vib[j] = src->vib[i];
    dst->pid[j] = src->pid[i];
    dst->cell[j] = c;
  }
  dst->n = offsets[M];
  dst->next_pid = src->next_pid;
  free(fill);
  free(key);
  return 0;
}

/* ======================================================================== */
/* Moments (Sec. II.A): per cell, U = <c>, then central moments about U.    */
/* Quantities are per unit mass (the cell's particles have equal weight).   */
/* ======================================================================== */
int orc_moments(const orc_grid* gr, const orc_gas* gas, const orc_parts* p,
                const int64_t* offsets, double* mom) {
  (void)gas;
  int64_t M = ncells(gr);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < M; ++c) {
    int64_t o0 = offsets[c], o1 = offsets[c + 1], N = o1 - o0;
    double v[ORC_NMOM];
    for (int k = 0; k < ORC_NMOM; ++k) v[k] = 0.0;
    if (N > 0) {
      double sx = 0, sy = 0, sz = 0;
      for (int64_t i = o0; i < o1; ++i) { sx += p->cx[i]; sy += p->cy[i]; sz += p->cz[i]; }
      double Ux = sx / N, Uy = sy / N, Uz = sz / N;
      double s[ORC_NMOM];
      for (int k = 0; k < ORC_NMOM; ++k) s[k] = 0.0;
      for (int64_t i = o0; i < o1; ++i) {
        double Cx = p->cx[i] - Ux, Cy = p->cy[i] - Uy, Cz = p->cz[i] - Uz;
        double C2 = Cx * Cx + Cy * Cy + Cz * Cz;
        double e = p->erot[i], I = (double)p->vib[i];
        s[ORC_M_PXX] += Cx * Cx; s[ORC_M_PYY] += Cy * Cy; s[ORC_M_PZZ] += Cz * Cz;
        s[ORC_M_PXY] += Cx * Cy; s[ORC_M_PXZ] += Cx * Cz; s[ORC_M_PYZ] += Cy * Cz;
        s[ORC_M_EROT] += e; s[ORC_M_IBAR] += I;
        s[ORC_M_QTRX] += 0.5 * C2 * Cx; s[ORC_M_QTRY] += 0.5 * C2 * Cy; s[ORC_M_QTRZ] += 0.5 * C2 * Cz;
        s[ORC_M_QROTX] += Cx * e; s[ORC_M_QROTY] += Cy * e; s[ORC_M_QROTZ] += Cz * e;
        s[ORC_M_QIX] += Cx * I; s[ORC_M_QIY] += Cy * I; s[ORC_M_QIZ] += Cz * I;
      }
      for (int k = ORC_M_PXX; k < ORC_NMOM; ++k) v[k] = s[k] / N;
      v[ORC_M_N] = (double)N;
      v[ORC_M_UX] = Ux; v[ORC_M_UY] = Uy; v[ORC_M_UZ] = Uz;
    }
    for (int k = 0; k < ORC_NMOM; ++k) mom[(int64_t)k * M + c] = v[k];
  }
  return 0;
}

/* ======================================================================== */
/* Field sampling: per cell, the plain sums over its particles of 1, c,    */
/* c_i c_j, eps_rot, I, |c|^2 c/2, c eps_rot and c I, added to the running  */
/* sums of the sampled steps (time averages of the cylinder case, Sec. V.C).*/
/* ======================================================================== */
int orc_sample_fields(const orc_grid* gr, const orc_parts* p, const int64_t* offsets,
                      double* acc) {
  int64_t M = ncells(gr);
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < M; ++c) {
    double s[ORC_NSAMP];
    for (int k = 0; k < ORC_NSAMP; ++k) s[k] = 0.0;
    for (int64_t i = offsets[c]; i < offsets[c + 1]; ++i) {
      double v[3] = {p->cx[i], p->cy[i], p->cz[i]};
      double e = p->erot[i], I = (double)p->vib[i];
      double h = 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
      s[0] += 1.0;
      for (int k = 0; k < 3; ++k) {
        s[1 + k] += v[k];
        s[4 + k] += v[k] * v[k];
        s[12 + k] += h * v[k];
        s[15 + k] += v[k] * e;
        s[18 + k] += v[k] * I;
      }
      s[7] += v[0] * v[1];
      s[8] += v[0] * v[2];
      s[9] += v[1] * v[2];
      s[10] += e;
      s[11] += I;
    }
    for (int k = 0; k < ORC_NSAMP; ++k) acc[(int64_t)k * M + c] += s[k];
  }
  return 0;
}

/* ======================================================================== */
/* Cell state: temperatures, transport, and the USP-FPM cell coefficients.  */
/*   T_tr = tr(Pi)/(3R), T_rot = e_rot/R, T_vib from the mean level.        */
/*   mu(T_tr), p = n k T_tr, tau_c, Z's, Pr (Secs. IV.A, IV.B, V.C).         */
/*   alpha = cbrt of the heat-flux factor (eq. USP-FPM_alpha_tr; the real,  */
/*   sign-preserving cube root), nu from eq. USP-FPM_nu.                    */
/*   Cell energy targets for the conservation step from eqs. e_rot/e_vib    */
/*   relax (Sec. III.A.1) at the cell temperatures.                         */
/* ======================================================================== */
int orc_cellstate(const orc_grid* gr, const orc_gas* g, const double* mom, double dt,
                  const double* dt_cell, double* cs) {
  int64_t M = ncells(gr);
  double R = orc_R(g), Th = g->theta_vib;
  double K = orc_tau_c_factor(g);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < M; ++c) {
    double v[ORC_NCS];
    for (int k = 0; k < ORC_NCS; ++k) v[k] = 0.0;
    double N = mom[(int64_t)ORC_M_N * M + c];
    double vol = gr->volume[c];
    v[ORC_CS_NP] = N;
    v[ORC_CS_NDENS] = (vol > 0.0) ? N * gr->fnum / vol : 0.0;
    v[ORC_CS_UX] = mom[(int64_t)ORC_M_UX * M + c];
    v[ORC_CS_UY] = mom[(int64_t)ORC_M_UY * M + c];
    v[ORC_CS_UZ] = mom[(int64_t)ORC_M_UZ * M + c];
    for (int k = 0; k < 6; ++k) v[ORC_CS_PXX + k] = mom[(int64_t)(ORC_M_PXX + k) * M + c];
    double trP = v[ORC_CS_PXX] + v[ORC_CS_PYY] + v[ORC_CS_PZZ];
    double ibar = mom[(int64_t)ORC_M_IBAR * M + c];
    v[ORC_CS_TTR] = trP / (3.0 * R);
    v[ORC_CS_TROT] = mom[(int64_t)ORC_M_EROT * M + c] / R;
    v[ORC_CS_TVIB] = (ibar > 0.0) ? Th / log1p(1.0 / ibar) : 0.0;
    v[ORC_CS_ETR] = 0.5 * trP;
    v[ORC_CS_EROT] = mom[(int64_t)ORC_M_EROT * M + c];
    v[ORC_CS_EVIB] = ibar * R * Th;
    double dtc = dt_cell ? dt_cell[c] : dt;
    v[ORC_CS_DT] = dtc;
    double Ttr = v[ORC_CS_TTR];
    /* a cell whose sums are not finite (a NaN or infinite velocity or
       rotational energy among its particles) is not collided */
    int finite = isfinite(v[ORC_CS_UX]) && isfinite(v[ORC_CS_UY]) && isfinite(v[ORC_CS_UZ]) &&
                 isfinite(trP) && isfinite(v[ORC_CS_EROT]);
    int collide = (N >= 2.0) && (Ttr > 0.0) && finite && (vol > 0.0);
    if (collide) {
      double mu = orc_viscosity(g, Ttr);
      double pres = v[ORC_CS_NDENS] * ORC_KB * Ttr;
      double mup = mu / pres;
      double tauc = K * mup;
      double zr = orc_zrot(g, Ttr), zv = orc_zvib(g, Ttr);
      double Pr = orc_prandtl(g, Ttr);
      double Trot = v[ORC_CS_TROT], Tvib = v[ORC_CS_TVIB];
      v[ORC_CS_MU] = mu; v[ORC_CS_MUP] = mup; v[ORC_CS_TAUC] = tauc;
      v[ORC_CS_ZROT] = zr; v[ORC_CS_ZVIB] = zv; v[ORC_CS_PR] = Pr;
      if (g->scheme == ORC_SCHEME_FPM) {
        /* first-order FPM (Secs. II.B-II.C): nu from Pr, tau = 2 mu (1-nu)/p, */
        /* the update factor exp(-dt/tau) and the relaxation temperatures of */
        /* eqs. T_tr_FPM, T_rot_FPM, T_vib_FPM (cell values)                 */
        double nu = 1.0 - 3.0 / (2.0 * Pr);
        double tau = 2.0 * mup * (1.0 - nu);
        double al = exp(-dtc / tau);
        double oma2 = -expm1(-2.0 * dtc / tau);
        double fr = tau / (2.0 * zr * tauc), fv = tau / (2.0 * zv * tauc);
        double mv = orc_e_vib(g, Tvib) / (R * Th), mt = orc_e_vib(g, Ttr) / (R * Th);
        double Ttr_rel = Ttr + (2.0 / 3.0) * (fr * (Trot - Ttr) + fv * Th * (mv - mt));
        double Trot_rel = Trot + fr * (Ttr - Trot);
        double mrel = mv + fv * (mt - mv);
        v[ORC_CS_ALPHA] = al; v[ORC_CS_OMA2] = oma2; v[ORC_CS_NU] = nu;
        v[ORC_CS_EROT_NEW] = v[ORC_CS_EROT];
        v[ORC_CS_EVIB_NEW] = v[ORC_CS_EVIB];
        v[ORC_CS_FPM_TAU] = tau;
        v[ORC_CS_FPM_TTR_REL] = Ttr_rel;
        v[ORC_CS_FPM_TROT_REL] = Trot_rel;
        v[ORC_CS_FPM_MREL] = mrel;
      } else {
        double A = 2.0 * mup;
        double r3 = (A - Pr * dtc) / (A + Pr * dtc);
        double r2 = (A - dtc) / (A + dtc);
        double al = cbrt(r3);
        double oma2 = 1.0 - al * al;
        double nu = (r2 - al * al) / oma2;
        double a = dtc / (dtc + 2.0 * zr * tauc);
        double b = dtc / (dtc + 2.0 * zv * tauc);
        double gm[3];
        orc_gammas(g, Ttr, Trot, Tvib, a, b, gm, NULL);
        v[ORC_CS_A] = a; v[ORC_CS_B] = b; v[ORC_CS_R2] = r2; v[ORC_CS_R3] = r3;
        v[ORC_CS_ALPHA] = al; v[ORC_CS_OMA2] = oma2; v[ORC_CS_NU] = nu;
        v[ORC_CS_EROT_NEW] = v[ORC_CS_EROT] + gm[0] * (Ttr - Trot) - gm[2] * (Trot - Tvib);
        v[ORC_CS_EVIB_NEW] = v[ORC_CS_EVIB] + gm[1] * (Ttr - Tvib) + gm[2] * (Trot - Tvib);
      }
      v[ORC_CS_COLLIDE] = 1.0;
      int cut = gr->flags ? (gr->flags[c] & (ORC_FLAG_SOLID | ORC_FLAG_CUT)) : 0;
      v[ORC_CS_NBR_OK] = cut ? 0.0 : 1.0;
    }
    for (int k = 0; k < ORC_NCS; ++k) cs[(int64_t)k * M + c] = v[k];
  }
  return 0;
}

/* ======================================================================== */
/* First-order polynomial reconstruction on a uniform grid (Sec. III.B).    */
/* phi = C00 + Cx (x-x_i) + Cy (y-y_j) + Cxy (x-x_i)(y-y_j), the stencil     */
/* being the cell and its neighbours toward the particle's quadrant.  Per   */
/* axis, an unusable neighbour (outside the grid, cut or solid, or with     */
/* fewer than 2 particles) is replaced by the opposite one; with neither,   */
/* that axis has no slope.  The cross term needs the diagonal cell too.     */
/* ======================================================================== */
static int nbr_ok(const orc_grid* gr, const double* cs, int i, int j) {
  if (i < 0 || j < 0 || i >= gr->nx || j >= gr->ny) return 0;
  int64_t M = ncells(gr);
  return cs[(int64_t)ORC_CS_NBR_OK * M + (int64_t)j * gr->nx + i] != 0.0;
}

double orc_interp(const orc_grid* gr, const double* cs, int field, int32_t cell, double x,
                  double y) {
  int64_t M = ncells(gr);
  const double* f = cs + (int64_t)field * M;
  if (gr->dim == 0) return f[cell];
  int nx = gr->nx;
  int i = (gr->dim == 2) ? cell % nx : 0;
  int j = (gr->dim == 2) ? cell / nx : cell;
  double f00 = f[cell];
  double dyv = y - (gr->y0 + (j + 0.5) * gr->dy);
  int sy = (dyv >= 0.0) ? 1 : -1;
  int ty = 0;
  if (nbr_ok(gr, cs, i, j + sy)) ty = sy;
  else if (nbr_ok(gr, cs, i, j - sy)) ty = -sy;
  if (gr->dim == 1) {
    double phi = f00;
    if (ty) phi += (f[(int64_t)(j + ty) * nx + i] - f00) * dyv / (ty * gr->dy);
    return phi;
  }
  double dxv = x - (gr->x0 + (i + 0.5) * gr->dx);
  int sx = (dxv >= 0.0) ? 1 : -1;
  int tx = 0;
  if (nbr_ok(gr, cs, i + sx, j)) tx = sx;
  else if (nbr_ok(gr, cs, i - sx, j)) tx = -sx;
  double phi = f00;
  double hx = tx * gr->dx, hy = ty * gr->dy;
  double f10 = tx ? f[(int64_t)j * nx + i + tx] : 0.0;
  double f01 = ty ? f[(int64_t)(j + ty) * nx + i] : 0.0;
  if (tx) phi += (f10 - f00) * dxv / hx;
  if (ty) phi += (f01 - f00) * dyv / hy;
  if (tx && ty && nbr_ok(gr, cs, i + tx, j + ty)) {
    double f11 = f[(int64_t)(j + ty) * nx + i + tx];
    phi += (f00 - f10 - f01 + f11) * dxv * dyv / (hx * hy);
  }
  return phi;
}

/* ======================================================================== */
/* Negative-binomial and binomial draws by sequential CDF inversion: the    */
/* smallest k with u < F(k).  NB(r, p) counts failures before the r-th      */
/* success (mean r(1-p)/p, as used in Sec. III.A.2).  The pmf recurrences   */
/* and the order of every FP64 operation are fixed so that two faithful     */
/* implementations take identical decisions.                                */
/* ======================================================================== */
#define NB_KMAX 512
int32_t orc_sample_nb(double u, int32_t r, double p) {
  double q = 1.0 - p;
  double pk = 1.0;
  for (int32_t i = 0; i < r; ++i) pk = pk * p;
  double F = pk;
  int32_t k = 0;
  while (u >= F && k < NB_KMAX) {
    double t = q * (double)(r + k);
    t = t / (double)(k + 1);
    pk = pk * t;
    F = F + pk;
    k = k + 1;
  }
  return k;
}

int32_t orc_sample_b(double u, int32_t n, double p) {
  if (n <= 0 || p <= 0.0) return 0;
  if (p >= 1.0) return n;
  double q = 1.0 - p;
  double pk = 1.0;
  for (int32_t i = 0; i < n; ++i) pk = pk * q;
  double ratio = p / q;
  double F = pk;
  int32_t k = 0;
  while (u >= F && k < n) {
    double t = ratio * (double)(n - k);
    t = t / (double)(k + 1);
    pk = pk * t;
    F = F + pk;
    k = k + 1;
  }
  return k;
}

/* 3x3 lower Cholesky of a symmetric matrix L = (xx,yy,zz,xy,xz,yz);     */
/* fails when a pivot is not strictly positive.                          */
static int chol3(const double S[6], double L[6]) {
  /* L = (l11, l21, l22, l31, l32, l33) */
  if (!(S[0] > 0.0)) return 0;
  double l11 = sqrt(S[0]);
  double l21 = S[3] / l11;
  double l31 = S[4] / l11;
  double d2 = S[1] - l21 * l21;
  if (!(d2 > 0.0)) return 0;
  double l22 = sqrt(d2);
  double l32 = (S[5] - l31 * l21) / l22;
  double d3 = S[2] - l31 * l31 - l32 * l32;
  if (!(d3 > 0.0)) return 0;
  double l33 = sqrt(d3);
  L[0] = l11; L[1] = l21; L[2] = l22; L[3] = l31; L[4] = l32; L[5] = l33;
  return 1;
}

/* ======================================================================== */
/* Collision: the per-particle USP-FPM update (Secs. III.A.2, III.A.3 and   */
/* the flow chart of Sec. IV.D).                                            */
/* ======================================================================== */
/* First-order FPM update of the particles of cell c (Sec. II.C): cell    */
/* values throughout (no reconstruction); velocity by eq.                */
/* conventionial-velo and rotation by eq. conventionial-erot (the same   */
/* algebra as the USP-FPM updates with alpha = exp(-dt/tau)); the level  */
/* by Gillespie's direct method for the jump rates of the master          */
/* equation, omega_{I,I-1} = 2 I / (tau (1-q)), omega_{I,I+1} = 2 (I+1) q */
/* / (tau (1-q)), q = exp(-Theta/T_vib^rel) = m_rel/(1+m_rel).  Draws:    */
/* block 0 of (pid, step, collide) for the four normals, then blocks 1, */
/* 2, ... two uniforms per jump attempt.  At most FPM_MAX_JUMPS attempts; */
/* a cap or a level beyond the top counts as VIB_SAT.  A failed Cholesky */
/* test of the cell's Lambda falls back to nu = 0.                        */
#define FPM_MAX_JUMPS 4096
static void fpm_cell(const orc_grid* gr, const orc_gas* g, const double* cs, int64_t c,
                     int64_t o0, int64_t o1, orc_parts* p, uint64_t seed, uint64_t step,
                     int32_t f32, int64_t* lc) {
  int64_t M = ncells(gr);
  double R = orc_R(g);
  double U[3], P[6];
  for (int k = 0; k < 3; ++k) U[k] = cs[(int64_t)(ORC_CS_UX + k) * M + c];
  for (int k = 0; k < 6; ++k) P[k] = cs[(int64_t)(ORC_CS_PXX + k) * M + c];
  const double Ttr = cs[(int64_t)ORC_CS_TTR * M + c];
  const double al = cs[(int64_t)ORC_CS_ALPHA * M + c], oma2 = cs[(int64_t)ORC_CS_OMA2 * M + c];
  const double nu = cs[(int64_t)ORC_CS_NU * M + c], dtc = cs[(int64_t)ORC_CS_DT * M + c];
  const double tau = cs[(int64_t)ORC_CS_FPM_TAU * M + c];
  const double Ttr_rel = cs[(int64_t)ORC_CS_FPM_TTR_REL * M + c];
  double Trot_rel = cs[(int64_t)ORC_CS_FPM_TROT_REL * M + c];
  double mrel = cs[(int64_t)ORC_CS_FPM_MREL * M + c];
  const int64_t n = o1 - o0;
  double Lam[6], L[6];
  const double RT = R * Ttr;
  for (int k = 0; k < 3; ++k) Lam[k] = R * Ttr_rel + nu * (P[k] - RT);
  for (int k = 3; k < 6; ++k) Lam[k] = nu * P[k];
  if (!chol3(Lam, L)) {
    lc[ORC_CNT_CHOL_FALLBACK] += n;
    lc[ORC_CNT_NU_ZERO] += n;
    if (!(Ttr_rel > 0.0)) { lc[ORC_CNT_TREL_SKIP] += n; return; }
    double s0 = sqrt(R * Ttr_rel);
    L[0] = s0; L[1] = 0.0; L[2] = s0; L[3] = 0.0; L[4] = 0.0; L[5] = s0;
  }
  if (Trot_rel < 0.0) { Trot_rel = 0.0; lc[ORC_CNT_TREL_CLAMP] += n; }
  if (mrel < 0.0) { mrel = 0.0; lc[ORC_CNT_TREL_CLAMP] += n; }
  const double q = mrel / (1.0 + mrel);
  for (int64_t i = o0; i < o1; ++i) {
    double u[4];
    draw4(seed, p->pid[i], step, TAG_COLLIDE, 0, u);
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    double G1 = r0 * cos(2.0 * PI * u[1]), G2 = r0 * sin(2.0 * PI * u[1]);
    double G3 = r1 * cos(2.0 * PI * u[3]), G4 = r1 * sin(2.0 * PI * u[3]);
    double sq = sqrt(oma2);
    double Cx = p->cx[i] - U[0], Cy = p->cy[i] - U[1], Cz = p->cz[i] - U[2];
    double ncx = U[0] + al * Cx + sq * (L[0] * G1);
    double ncy = U[1] + al * Cy + sq * (L[1] * G1 + L[2] * G2);
    double ncz = U[2] + al * Cz + sq * (L[3] * G1 + L[4] * G2 + L[5] * G3);
    double half = 0.5 * R * Trot_rel * oma2;
    double root = sqrt(p->erot[i]) * al + sqrt(half) * G4;
    double ne = half + root * root;
    /* Gillespie: waiting time -ln(U1)/W, then up with probability */
    /* omega_up/W = (I+1) q / ((I+1) q + I)                         */
    int32_t I = p->vib[i];
    double t = 0.0;
    double w[4];
    for (int k = 0; k < FPM_MAX_JUMPS; ++k) {
      const double wu = (double)(I + 1) * q, wd = (double)I;
      const double W = 2.0 * (wu + wd) / (tau * (1.0 - q));
      if (!(W > 0.0)) break;
      if ((k & 1) == 0) draw4(seed, p->pid[i], step, TAG_COLLIDE, (uint32_t)(1 + (k >> 1)), w);
      const double u1 = w[2 * (k & 1)], u2 = w[2 * (k & 1) + 1];
      const double dtv = -log(u1) / W;
      if (t + dtv > dtc) break;
      if (u2 < wu / (wu + wd)) ++I; else --I;
      t += dtv;
      if (k == FPM_MAX_JUMPS - 1) lc[ORC_CNT_VIB_SAT] += 1;
    }
    if (I > ORC_VIB_MAX) { I = ORC_VIB_MAX; lc[ORC_CNT_VIB_SAT] += 1; }
    p->cx[i] = store(ncx, f32);
    p->cy[i] = store(ncy, f32);
    p->cz[i] = store(ncz, f32);
    p->erot[i] = store(ne, f32);
    p->vib[i] = I;
  }
}

/* ======================================================================== */
/* Per-particle coefficients of one particle (Secs. III.A.1-III.A.3): the   */
/* gamma coefficients at the interpolated temperatures, the relaxation      */
/* temperatures (eqs. T_tr_USP, T_rot_USP, T_vib_USP) with the cell's       */
/* alpha and nu, the tensor Lambda = R T_tr^rel I + nu (Pi - R T_tr I)      */
/* (tau times the diffusion tensor of eq. D_tr) and its Cholesky test.      */
/* When the test fails: nu is moved into the positive-definite range of     */
/* eq. nu_USP_positivity (bounds at the relaxation temperature of the cell  */
/* coefficients, kept 2^-20 inside so the re-test can pass), alpha^2        */
/* refitted by eq. alpha_USP_positivity_1 (clamped to [0, 1]), the sign of  */
/* alpha chosen by the Prandtl number of eq. alpha_USP_positivity_3 that is */
/* closer to the cell's (ties: +; with ORC_ALPHA_SIGN_KEEP the sign of the  */
/* cell's alpha instead), alpha_rot = alpha_vib = alpha_tr (eq.             */
/* alpha_USP_positivity_4), the relaxation temperatures recomputed with the */
/* new 1 - alpha^2 and Lambda re-tested; a second failure sets nu = 0       */
/* (Lambda = R T_tr^rel I, alpha kept).  T_tr^rel <= 0 (before or after    */
/* the refit) or 1 - alpha^2 = 0 after it skips the particle.               */
/* Cell inputs: a, b (eqs. of the gammas), alpha, 1 - alpha^2, nu, r2 =     */
/* (2mu/p - dt)/(2mu/p + dt), A2 = 2 mu/p, the cell's Pr and dt.            */
/* ======================================================================== */
void orc_particle_coef(const orc_gas* g, double Ttr, double Trot, double Tvib, const double P[6],
                       double a, double b, double al_cell, double oma2_cell, double nu_cell,
                       double r2, double A2, double Pr, double dtc, orc_pcoef* out) {
  double R = orc_R(g), Th = g->theta_vib;
  double gm[3];
  orc_gammas(g, Ttr, Trot, Tvib, a, b, gm, NULL);
  /* energy handed on by each mode in one step (eqs. e_*_relax) */
  double Xtr = gm[0] * (Ttr - Trot) + gm[1] * (Ttr - Tvib);
  double Xrot = gm[0] * (Ttr - Trot) - gm[2] * (Trot - Tvib);
  double Xvib = gm[1] * (Ttr - Tvib) + gm[2] * (Trot - Tvib);
  double al = al_cell, oma2 = oma2_cell, nu = nu_cell;
  /* relaxation temperatures, eqs. T_tr_USP, T_rot_USP, T_vib_USP */
  double Ttr_rel = Ttr - Xtr / (oma2 * 1.5 * R);
  double Trot_rel = Trot + Xrot / (oma2 * R);
  double mstar = orc_e_vib(g, Tvib) / (R * Th) + Xvib / (oma2 * R * Th);
  /* diffusion tensor (times tau), eq. D_tr, and its Cholesky test */
  double RT = R * Ttr;
  double Lam[6], L[6] = {0, 0, 0, 0, 0, 0};
  for (int k = 0; k < 3; ++k) Lam[k] = R * Ttr_rel + nu * (P[k] - RT);
  for (int k = 3; k < 6; ++k) Lam[k] = nu * P[k];
  int ok = chol3(Lam, L);
  int skip = 0, fallback = 0, nu_zero = 0;
  out->nu_bound = 0.0;
  if (!ok) {
    fallback = 1;
    if (!(Ttr_rel > 0.0)) {
      skip = 1;
    } else {
      /* nu clamped into the positive-definite range, eq.            */
      /* nu_USP_positivity; kept a hair inside the bound so the     */
      /* re-test can pass.                                          */
      double ev[3];
      orc_eigvals_sym3(P, ev);
      double RTr = R * Ttr_rel;
      const double shrink = 1.0 - 1.0 / 1048576.0;
      if (nu <= 0.0) {
        if (ev[2] > RT) {
          out->nu_bound = -RTr / (ev[2] - RT);
          nu = fmax(nu, -RTr / (ev[2] - RT) * shrink);
        }
      } else {
        if (ev[0] < RT) {
          out->nu_bound = RTr / (RT - ev[0]);
          nu = fmin(nu, RTr / (RT - ev[0]) * shrink);
        }
      }
      /* alpha refit, eqs. alpha_USP_positivity_1..4 */
      double a2 = (nu - r2) / (nu - 1.0);
      if (a2 < 0.0) a2 = 0.0;
      if (a2 > 1.0) a2 = 1.0;
      double ap = sqrt(a2), am = -sqrt(a2);
      double Prp = A2 * (1.0 - ap * ap * ap) / (dtc * (1.0 + ap * ap * ap));
      double Prm = A2 * (1.0 - am * am * am) / (dtc * (1.0 + am * am * am));
      if (g->alpha_sign == ORC_ALPHA_SIGN_KEEP)
        al = al_cell < 0.0 ? am : ap;
      else
        al = (fabs(Prm - Pr) < fabs(Prp - Pr)) ? am : ap;
      oma2 = 1.0 - a2;
      if (!(oma2 > 0.0)) {
        skip = 1;
      } else {
        Ttr_rel = Ttr - Xtr / (oma2 * 1.5 * R);
        Trot_rel = Trot + Xrot / (oma2 * R);
        mstar = orc_e_vib(g, Tvib) / (R * Th) + Xvib / (oma2 * R * Th);
        for (int k = 0; k < 3; ++k) Lam[k] = R * Ttr_rel + nu * (P[k] - RT);
        for (int k = 3; k < 6; ++k) Lam[k] = nu * P[k];
        ok = chol3(Lam, L);
        if (!ok) {
          nu_zero = 1;
          nu = 0.0;
          if (Ttr_rel > 0.0) {
            double s0 = sqrt(R * Ttr_rel);
            L[0] = s0; L[1] = 0.0; L[2] = s0; L[3] = 0.0; L[4] = 0.0; L[5] = s0;
            ok = 1;
          } else {
            skip = 1;
          }
        }
      }
    }
  }
  for (int k = 0; k < 6; ++k) out->L[k] = L[k];
  out->al = al;
  out->oma2 = oma2;
  out->nu = nu;
  out->Ttr_rel = Ttr_rel;
  out->Trot_rel = Trot_rel;
  out->mstar = mstar;
  out->fallback = fallback;
  out->nu_zero = nu_zero;
  out->skip = skip;
}

int orc_collide(const orc_grid* gr, const orc_gas* g, const double* cs, const int64_t* offsets,
                orc_parts* p, uint64_t seed, uint64_t step, int32_t f32, int64_t* counters) {
  int64_t M = ncells(gr);
  double R = orc_R(g);
  int64_t cnt[ORC_NCNT];
  memset(cnt, 0, sizeof(cnt));
#pragma omp parallel
  {
    int64_t lc[ORC_NCNT];
    memset(lc, 0, sizeof(lc));
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < M; ++c) {
      int64_t o0 = offsets[c], o1 = offsets[c + 1];
      if (o1 == o0) continue;
      if (cs[(int64_t)ORC_CS_COLLIDE * M + c] == 0.0) {
        lc[ORC_CNT_CELL_SKIP] += 1;
        double trP = cs[(int64_t)ORC_CS_PXX * M + c] + cs[(int64_t)ORC_CS_PYY * M + c] +
                     cs[(int64_t)ORC_CS_PZZ * M + c];
        if (!(isfinite(cs[(int64_t)ORC_CS_UX * M + c]) && isfinite(cs[(int64_t)ORC_CS_UY * M + c]) &&
              isfinite(cs[(int64_t)ORC_CS_UZ * M + c]) && isfinite(trP) &&
              isfinite(cs[(int64_t)ORC_CS_EROT * M + c])))
          lc[ORC_CNT_NONFINITE] += 1;
        continue;
      }
      if (g->scheme == ORC_SCHEME_FPM) {
        fpm_cell(gr, g, cs, c, o0, o1, p, seed, step, f32, lc);
        continue;
      }
      const double a = cs[(int64_t)ORC_CS_A * M + c], b = cs[(int64_t)ORC_CS_B * M + c];
      const double al_cell = cs[(int64_t)ORC_CS_ALPHA * M + c];
      const double oma2_cell = cs[(int64_t)ORC_CS_OMA2 * M + c];
      const double nu_cell = cs[(int64_t)ORC_CS_NU * M + c];
      const double r2 = cs[(int64_t)ORC_CS_R2 * M + c];
      const double A2 = 2.0 * cs[(int64_t)ORC_CS_MUP * M + c];
      const double Pr = cs[(int64_t)ORC_CS_PR * M + c];
      const double dtc = cs[(int64_t)ORC_CS_DT * M + c];
      for (int64_t i = o0; i < o1; ++i) {
        double px = p->x ? p->x[i] : 0.0, py = p->y ? p->y[i] : 0.0;
        /* interpolate U, T_tr, T_rot, T_vib, Pi to the particle */
        double U[3], T[3], P[6];
        for (int k = 0; k < 3; ++k) U[k] = orc_interp(gr, cs, ORC_CS_UX + k, (int32_t)c, px, py);
        if (g->gamma_scope == ORC_GAMMA_CELL) {
          /* the per-cell reading: the chain at the cell's own values */
          for (int k = 0; k < 3; ++k) T[k] = cs[(int64_t)(ORC_CS_TTR + k) * M + c];
          for (int k = 0; k < 6; ++k) P[k] = cs[(int64_t)(ORC_CS_PXX + k) * M + c];
        } else {
          for (int k = 0; k < 3; ++k) T[k] = orc_interp(gr, cs, ORC_CS_TTR + k, (int32_t)c, px, py);
          for (int k = 0; k < 6; ++k) P[k] = orc_interp(gr, cs, ORC_CS_PXX + k, (int32_t)c, px, py);
          /* guard: an extrapolated temperature may not fall below 5% of */
          /* the cell's own value (the paper has no limiter)             */
          int clamped = 0;
          for (int k = 0; k < 3; ++k) {
            double floorv = 0.05 * cs[(int64_t)(ORC_CS_TTR + k) * M + c];
            if (T[k] < floorv) { T[k] = floorv; clamped = 1; }
          }
          if (clamped) lc[ORC_CNT_INTERP_CLAMP] += 1;
        }
        double Ttr = T[0], Trot = T[1], Tvib = T[2];
        orc_pcoef pc;
        orc_particle_coef(g, Ttr, Trot, Tvib, P, a, b, al_cell, oma2_cell, nu_cell, r2, A2, Pr,
                          dtc, &pc);
        if (pc.fallback) lc[ORC_CNT_CHOL_FALLBACK] += 1;
        if (pc.nu_zero) lc[ORC_CNT_NU_ZERO] += 1;
        int skip = pc.skip;
        double al = pc.al, oma2 = pc.oma2, Trot_rel = pc.Trot_rel, mstar = pc.mstar;
        const double* L = pc.L;
        if (skip) { lc[ORC_CNT_TREL_SKIP] += 1; continue; }
        if (Trot_rel < 0.0) { Trot_rel = 0.0; lc[ORC_CNT_TREL_CLAMP] += 1; }
        if (mstar < 0.0) { mstar = 0.0; lc[ORC_CNT_TREL_CLAMP] += 1; }
        /* draws: two Philox blocks keyed by (pid, step, collide) */
        double u[8];
        draw4(seed, p->pid[i], step, TAG_COLLIDE, 0, u);
        draw4(seed, p->pid[i], step, TAG_COLLIDE, 1, u + 4);
        double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
        double G1 = r0 * cos(2.0 * PI * u[1]), G2 = r0 * sin(2.0 * PI * u[1]);
        double G3 = r1 * cos(2.0 * PI * u[3]), G4 = r1 * sin(2.0 * PI * u[3]);
        /* velocity, eq. update_ci, with sqrt(tau) d = L */
        double sq = sqrt(oma2);
        double Cx = p->cx[i] - U[0], Cy = p->cy[i] - U[1], Cz = p->cz[i] - U[2];
        double ncx = U[0] + al * Cx + sq * (L[0] * G1);
        double ncy = U[1] + al * Cy + sq * (L[1] * G1 + L[2] * G2);
        double ncz = U[2] + al * Cz + sq * (L[3] * G1 + L[4] * G2 + L[5] * G3);
        /* rotational energy, eq. update_erot */
        double half = 0.5 * R * Trot_rel * oma2;
        double root = sqrt(p->erot[i]) * al + sqrt(half) * G4;
        double ne = half + root * root;
        /* vibrational level, eq. update_evib */
        int32_t I = p->vib[i];
        double pNB = 1.0 / (1.0 + mstar * oma2);
        double pB = (1.0 + mstar) * oma2;
        if (pB > 1.0) { pB = 1.0; lc[ORC_CNT_PB_CLAMP] += 1; }
        int32_t nI = I + orc_sample_nb(u[4], I + 1, pNB) - orc_sample_b(u[5], I, pB);
        if (nI > ORC_VIB_MAX) { nI = ORC_VIB_MAX; lc[ORC_CNT_VIB_SAT] += 1; }
        p->cx[i] = store(ncx, f32);
        p->cy[i] = store(ncy, f32);
        p->cz[i] = store(ncz, f32);
        p->erot[i] = store(ne, f32);
        p->vib[i] = nI;
      }
    }
#pragma omp critical
    for (int k = 0; k < ORC_NCNT; ++k) cnt[k] += lc[k];
  }
  if (counters)
    for (int k = 0; k < ORC_NCNT; ++k) counters[k] += cnt[k];
  return 0;
}

/* ======================================================================== */
/* Conservation scheme (Sec. IV.C), per cell, in the order vibration,       */
/* rotation, velocity.  I_delta = floor(N (e_vib^{n+1}-e_vib^*)/(R Theta)+U)*/
/* (the integer part taken as floor, so the rounding is unbiased); levels   */
/* are moved one at a time on randomly picked particles (a level-0 pick for */
/* a decrement is redrawn).  The velocity scale uses the energies actually  */
/* reached after the vibrational and rotational corrections, so the total  */
/* energy is conserved to rounding.                                         */
/* ======================================================================== */
int orc_conserve(const orc_grid* gr, const orc_gas* g, const double* cs, const int64_t* offsets,
                 orc_parts* p, uint64_t seed, uint64_t step, int32_t f32, int64_t* counters) {
  int64_t M = ncells(gr);
  double R = orc_R(g), RTh = orc_R(g) * g->theta_vib;
  (void)R;
  int64_t cnt[ORC_NCNT];
  memset(cnt, 0, sizeof(cnt));
#pragma omp parallel
  {
    int64_t lc[ORC_NCNT];
    memset(lc, 0, sizeof(lc));
#pragma omp for schedule(dynamic, 16)
    for (int64_t c = 0; c < M; ++c) {
      int64_t o0 = offsets[c], o1 = offsets[c + 1], N = o1 - o0;
      if (N == 0 || cs[(int64_t)ORC_CS_COLLIDE * M + c] == 0.0) continue;
      double Un[3] = {cs[(int64_t)ORC_CS_UX * M + c], cs[(int64_t)ORC_CS_UY * M + c],
                      cs[(int64_t)ORC_CS_UZ * M + c]};
      double S1[3] = {0, 0, 0}, S2 = 0, Se = 0;
      int64_t SI = 0;
      for (int64_t i = o0; i < o1; ++i) {
        double d0 = p->cx[i] - Un[0], d1 = p->cy[i] - Un[1], d2 = p->cz[i] - Un[2];
        S1[0] += d0; S1[1] += d1; S1[2] += d2;
        S2 += d0 * d0 + d1 * d1 + d2 * d2;
        Se += p->erot[i];
        SI += p->vib[i];
      }
      double m1[3] = {S1[0] / N, S1[1] / N, S1[2] / N};
      double Us[3] = {Un[0] + m1[0], Un[1] + m1[1], Un[2] + m1[2]};
      double etr_s = 0.5 * (S2 / N - (m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2]));
      /* (i) vibrational levels (USP-FPM only: the first-order FPM      */
      /* method keeps the levels and rotational energies it sampled and  */
      /* conserves momentum and total energy through the velocities)     */
      const int fpm = g->scheme == ORC_SCHEME_FPM;
      double X = (double)N * cs[(int64_t)ORC_CS_EVIB_NEW * M + c] / RTh - (double)SI;
      double u4[4];
      draw4(seed, (uint32_t)c, step, TAG_CONSERVE, 0, u4);
      int64_t Id = fpm ? 0 : (int64_t)floor(X + u4[0]);
      int64_t att = 0, maxatt = 64 * N;
      uint32_t j = 1;
      while (Id != 0) {
        if (att >= maxatt || (Id < 0 && SI == 0)) { lc[ORC_CNT_PICK_FAIL] += 1; break; }
        draw4(seed, (uint32_t)c, step, TAG_CONSERVE, j >> 2, u4);
        double uu = u4[j & 3];
        j++;
        att++;
        int64_t k = (int64_t)floor(uu * (double)N);
        if (k >= N) k = N - 1;
        int32_t* lv = &p->vib[o0 + k];
        if (Id > 0) {
          if (*lv < ORC_VIB_MAX) { *lv += 1; SI += 1; Id -= 1; }
        } else {
          if (*lv > 0) { *lv -= 1; SI -= 1; Id += 1; }
        }
      }
      /* (ii) rotational scaling */
      double erot_s = Se / N, erot_t = cs[(int64_t)ORC_CS_EROT_NEW * M + c];
      double erot_a = erot_s;
      if (fpm) {
        /* nothing: the sampled rotational energies stand */
      } else if (erot_s > 0.0 && erot_t > 0.0) {
        double f = erot_t / erot_s;
        for (int64_t i = o0; i < o1; ++i) p->erot[i] = store(p->erot[i] * f, f32);
        erot_a = erot_t;
      } else {
        lc[ORC_CNT_CONS_SKIP] += 1;
      }
      /* (iii) velocity scaling about U*, toward U^n */
      double evib_a = (double)SI * RTh / N;
      double E0 = cs[(int64_t)ORC_CS_ETR * M + c] + cs[(int64_t)ORC_CS_EROT * M + c] +
                  cs[(int64_t)ORC_CS_EVIB * M + c];
      double s2 = (E0 - erot_a - evib_a) / etr_s;
      if (etr_s > 0.0 && s2 > 0.0) {
        double s = sqrt(s2);
        for (int64_t i = o0; i < o1; ++i) {
          p->cx[i] = store(Un[0] + s * (p->cx[i] - Us[0]), f32);
          p->cy[i] = store(Un[1] + s * (p->cy[i] - Us[1]), f32);
          p->cz[i] = store(Un[2] + s * (p->cz[i] - Us[2]), f32);
        }
      } else {
        lc[ORC_CNT_CONS_SKIP] += 1;
      }
    }
#pragma omp critical
    for (int k = 0; k < ORC_NCNT; ++k) cnt[k] += lc[k];
  }
  if (counters)
    for (int k = 0; k < ORC_NCNT; ++k) counters[k] += cnt[k];
  return 0;
}

/* ======================================================================== */
/* Free flight x += c dt (Sec. II.C) with boundaries.                       */
/* Diffuse walls re-emit from the wall Maxwellian (full accommodation): the */
/* normal speed from the flux-weighted half-range distribution, tangential  */
/* components Gaussian, rotational energy exponential and the level         */
/* geometric at the wall temperature; the flight continues for the time    */
/* left.  Free-stream and outflow faces remove the particle.                */
/* ======================================================================== */
static void wall_draw(const orc_gas* g, double Tw, uint64_t seed, uint32_t pid, uint64_t step,
                      int bounce, double* cn, double* ta, double* tb, double* er, int32_t* lv) {
  double u[8];
  draw4(seed, pid, step, TAG_WALL, (uint32_t)(2 * bounce), u);
  draw4(seed, pid, step, TAG_WALL, (uint32_t)(2 * bounce + 1), u + 4);
  double R = orc_R(g);
  double sig = sqrt(R * Tw);
  *cn = sqrt(-2.0 * R * Tw * log(u[0]));
  double r = sqrt(-2.0 * log(u[1]));
  *ta = sig * r * cos(2.0 * PI * u[2]);
  *tb = sig * r * sin(2.0 * PI * u[2]);
  *er = -R * Tw * log(u[3]);
  double lvl = floor(log(u[4]) / (-g->theta_vib / Tw));
  *lv = (lvl > ORC_VIB_MAX) ? ORC_VIB_MAX : (int32_t)lvl;
}

/* domain extent along an axis in stored precision */
static double lo_edge(double o, int32_t f32) { return store(o, f32); }

static int inside_cyl(const orc_bc* bc, double x, double y) {
  if (!bc->cyl) return 0;
  double dx = x - bc->cyl_xc, dy = y - bc->cyl_yc;
  return dx * dx + dy * dy < bc->cyl_r * bc->cyl_r;
}

/* final position: round to storage precision, keep inside [lo, hi) */
static double settle(double v, double lo, double hi, int32_t f32) {
  if (f32) {
    float vf = (float)v, lof = (float)lo, hif = (float)hi;
    if (vf >= hif) vf = nextafterf(hif, -INFINITY);
    if (vf < lof) vf = lof;
    return (double)vf;
  }
  if (v >= hi) v = nextafter(hi, -INFINITY);
  if (v < lo) v = lo;
  return v;
}

/* One diffuse re-emission into the surface sums (see usp_oracle.h).      */
static void surf_fix_add(int64_t* a, double v, double scale) {
  int64_t q = llrint(v * scale);
#pragma omp atomic
  *a += q;
}

static void surface_sample(const orc_grid* gr, const orc_bc* bc, int side, double x,
                           double y, const double cin[3], double ein, int32_t lin,
                           const double cout[3], double eout, int32_t lout) {
  int64_t e;
  double n[2], t[2];
  if (side == ORC_SIDE_YLO || side == ORC_SIDE_YHI) {
    int64_t ix = 0;
    if (gr->dim == 2) {
      double f = floor((x - gr->x0) / gr->dx);
      ix = (f < 0.0) ? 0 : (f >= gr->nx) ? gr->nx - 1 : (int64_t)f;
    }
    e = ((side == ORC_SIDE_YLO) ? 0 : gr->nx) + ix;
    n[0] = 0.0; n[1] = (side == ORC_SIDE_YLO) ? 1.0 : -1.0;
    t[0] = 1.0; t[1] = 0.0;
  } else if (side == ORC_SIDE_XLO || side == ORC_SIDE_XHI) {
    double f = floor((y - gr->y0) / gr->dy);
    int64_t iy = (f < 0.0) ? 0 : (f >= gr->ny) ? gr->ny - 1 : (int64_t)f;
    e = 2 * (int64_t)gr->nx + ((side == ORC_SIDE_XLO) ? 0 : gr->ny) + iy;
    n[0] = (side == ORC_SIDE_XLO) ? 1.0 : -1.0; n[1] = 0.0;
    t[0] = 0.0; t[1] = 1.0;
  } else {
    if (bc->surf_nbody <= 0) return;
    /* outward unit normal of the circle at the hit point */
    double ux = x - bc->cyl_xc, uy = y - bc->cyl_yc;
    double r = sqrt(ux * ux + uy * uy);
    n[0] = ux / r; n[1] = uy / r;
    /* Theta from the upstream point (-r, 0), growing over either half */
    double theta = atan2(fabs(n[1]), -n[0]);
    double f = floor(theta * bc->surf_nbody / PI);
    int64_t ib = (f < 0.0) ? 0 : (f >= bc->surf_nbody) ? bc->surf_nbody - 1 : (int64_t)f;
    e = 2 * (int64_t)gr->nx + 2 * (int64_t)gr->ny + ib;
    /* d(point)/dTheta direction: upper half (n_y >= 0) and its mirror */
    if (n[1] >= 0.0) { t[0] = n[1]; t[1] = -n[0]; }
    else { t[0] = -n[1]; t[1] = n[0]; }
  }
  int64_t* a = bc->surf + e * ORC_SURF_NQ;
  double d[3] = {cin[0] - cout[0], cin[1] - cout[1], cin[2] - cout[2]};
#pragma omp atomic
  a[ORC_SURF_HITS] += 1;
  surf_fix_add(a + ORC_SURF_PX, d[0], ORC_SURF_P_SCALE);
  surf_fix_add(a + ORC_SURF_PY, d[1], ORC_SURF_P_SCALE);
  surf_fix_add(a + ORC_SURF_PZ, d[2], ORC_SURF_P_SCALE);
  surf_fix_add(a + ORC_SURF_PN, -(d[0] * n[0] + d[1] * n[1]), ORC_SURF_P_SCALE);
  surf_fix_add(a + ORC_SURF_PT, d[0] * t[0] + d[1] * t[1], ORC_SURF_P_SCALE);
  double kin = cin[0] * cin[0] + cin[1] * cin[1] + cin[2] * cin[2];
  double kout = cout[0] * cout[0] + cout[1] * cout[1] + cout[2] * cout[2];
  surf_fix_add(a + ORC_SURF_ETR, 0.5 * (kin - kout), ORC_SURF_E_SCALE);
  surf_fix_add(a + ORC_SURF_EROT, ein - eout, ORC_SURF_E_SCALE);
#pragma omp atomic
  a[ORC_SURF_QVIB] += (int64_t)(lin - lout);
}

static void flight(const orc_grid* gr, const orc_gas* g, const orc_bc* bc, double dt,
                   orc_parts* p, int64_t i, uint64_t seed, uint64_t step, int32_t f32,
                   int64_t* lc) {
  double x = p->x ? p->x[i] : 0.0, y = p->y[i];
  double cx = p->cx[i], cy = p->cy[i], cz = p->cz[i];
  double er = p->erot[i];
  int32_t lv = p->vib[i];
  int changed_int = 0;
  const double xlo = lo_edge(gr->x0, f32), xhi = edge(gr->x0, gr->dx, gr->nx, f32);
  const double ylo = lo_edge(gr->y0, f32), yhi = edge(gr->y0, gr->dy, gr->ny, f32);
  double t = dt;
  int bounces = 0, events = 0, deleted = 0;
  for (;;) {
    /* earliest boundary crossing within the time left; on a tie the     */
    /* first candidate in the order xlo, xhi, ylo, yhi, cylinder wins     */
    double th = INFINITY;
    int side = -1;
    if (gr->dim == 2) {
      if (cx < 0.0 && x + cx * t < xlo) { double tt = (xlo - x) / cx; if (tt < th) { th = tt; side = ORC_SIDE_XLO; } }
      if (cx > 0.0 && x + cx * t >= xhi) { double tt = (xhi - x) / cx; if (tt < th) { th = tt; side = ORC_SIDE_XHI; } }
    }
    if (cy < 0.0 && y + cy * t < ylo) { double tt = (ylo - y) / cy; if (tt < th) { th = tt; side = ORC_SIDE_YLO; } }
    if (cy > 0.0 && y + cy * t >= yhi) { double tt = (yhi - y) / cy; if (tt < th) { th = tt; side = ORC_SIDE_YHI; } }
    if (gr->dim == 2 && bc->cyl) {
      /* entry into the circle: |p + c t|^2 = r^2 while moving inward */
      double px = x - bc->cyl_xc, py = y - bc->cyl_yc;
      double A = cx * cx + cy * cy, B = px * cx + py * cy;
      double C = px * px + py * py - bc->cyl_r * bc->cyl_r;
      if (B < 0.0 && A > 0.0) {
        double tt = -1.0;
        if (C <= 0.0) tt = 0.0;
        else {
          double disc = B * B - A * C;
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
    if (++events > 4 * ORC_MAX_BOUNCE) { lc[ORC_CNT_BOUNCE_LIMIT] += 1; break; }
    int kind = (side == 4) ? ORC_BC_DIFFUSE : bc->kind[side];
    if (side == ORC_SIDE_XLO) x = xlo;
    if (side == ORC_SIDE_XHI) x = xhi;
    if (side == ORC_SIDE_YLO) y = ylo;
    if (side == ORC_SIDE_YHI) y = yhi;
    if (kind == ORC_BC_FREESTREAM || kind == ORC_BC_OUTFLOW) { deleted = 1; break; }
    if (kind == ORC_BC_PERIODIC) {
      if (side == ORC_SIDE_XLO) x = xhi;
      else if (side == ORC_SIDE_XHI) x = xlo;
      else if (side == ORC_SIDE_YLO) y = yhi;
      else y = ylo;
      continue;
    }
    if (kind == ORC_BC_SPECULAR) {
      if (side == ORC_SIDE_XLO || side == ORC_SIDE_XHI) cx = -cx; else cy = -cy;
      continue;
    }
    /* diffuse re-emission */
    if (bounces >= ORC_MAX_BOUNCE) { lc[ORC_CNT_BOUNCE_LIMIT] += 1; break; }
    double cn, ta, tb, ner;
    int32_t nlv;
    double Tw = (side == 4) ? bc->cyl_Tw : bc->Tw[side];
    wall_draw(g, Tw, seed, p->pid[i], step, bounces, &cn, &ta, &tb, &ner, &nlv);
    bounces++;
    lc[ORC_CNT_WALL_HITS] += 1;
    double cin[3] = {cx, cy, cz}, ein = er;
    int32_t lin = lv;
    double hx = x, hy = y;   /* the hit point */
    er = ner; lv = nlv; changed_int = 1;
    if (side == ORC_SIDE_YLO || side == ORC_SIDE_YHI) {
      cy = (side == ORC_SIDE_YLO) ? cn : -cn;
      cx = ta; cz = tb;
    } else if (side == ORC_SIDE_XLO || side == ORC_SIDE_XHI) {
      cx = (side == ORC_SIDE_XLO) ? cn : -cn;
      cy = ta; cz = tb;
    } else {
      double nxv = x - bc->cyl_xc, nyv = y - bc->cyl_yc;
      double nn = sqrt(nxv * nxv + nyv * nyv);
      nxv /= nn; nyv /= nn;
      x = bc->cyl_xc + bc->cyl_r * nxv;
      y = bc->cyl_yc + bc->cyl_r * nyv;
      cx = cn * nxv - ta * nyv;
      cy = cn * nyv + ta * nxv;
      cz = tb;
    }
    if (bc->surf) {
      double cout[3] = {cx, cy, cz};
      surface_sample(gr, bc, side, hx, hy, cin, ein, lin, cout, er, lv);
    }
  }
  (void)changed_int;
  if (deleted) {
    p->cell[i] = -1;
    lc[ORC_CNT_DELETED] += 1;
    return;
  }
  if (gr->dim == 2) p->x[i] = settle(x, xlo, xhi, f32);
  p->y[i] = settle(y, ylo, yhi, f32);
  p->cx[i] = store(cx, f32);
  p->cy[i] = store(cy, f32);
  p->cz[i] = store(cz, f32);
  p->erot[i] = store(er, f32);
  p->vib[i] = lv;
  p->cell[i] = cell_of(gr, p->x ? p->x[i] : 0.0, p->y[i], f32);
}

/* ---- free-stream injection ---------------------------------------------- */
/* Number flux of a drifting Maxwellian through a face, per unit area.     */
static double flux_per_area(double n, double R, double T, double Un) {
  double s = Un / sqrt(2.0 * R * T);
  return n * sqrt(R * T / (2.0 * PI)) * (exp(-s * s) + sqrt(PI) * s * (1.0 + erf(s)));
}

/* Dimensionless inward normal speed u = v_n / sqrt(2RT) drawn from the   */
/* density proportional to u exp(-(u-s)^2) on u > 0 (the flux-weighted    */
/* drifting Maxwellian), s = U_n/sqrt(2RT).  Exact: for s >= 0 the density */
/* in w = u - s splits into w e^{-w^2} (w>0), s e^{-w^2} (w>0) and         */
/* (w+s) e^{-w^2} on (-s,0), picked by their masses; for s < 0 the density */
/* u e^{-u^2} e^{-2|s|u} is sampled by rejection.                          */
double orc_inflow_speed(uint64_t seed, uint64_t step, uint32_t pid, double s) {
  double ub[4], ua[4];
  draw4(seed, pid, step, TAG_INJECT, 1, ub);
  if (s >= 0.0) {
    double mA1 = 0.5, mA2 = 0.5 * sqrt(PI) * s;
    double mB = 0.5 * (sqrt(PI) * s * erf(s) - (1.0 - exp(-s * s)));
    if (mB < 0.0) mB = 0.0;
    double v = ub[2] * (mA1 + mA2 + mB);
    if (v < mA1) {
      draw4(seed, pid, step, TAG_INJECT, 2, ua);
      return sqrt(-log(ua[0])) + s;
    }
    if (v < mA1 + mA2) {
      draw4(seed, pid, step, TAG_INJECT, 2, ua);
      double G = sqrt(-2.0 * log(ua[0])) * cos(2.0 * PI * ua[1]);
      return fabs(G) / sqrt(2.0) + s;
    }
    double w = 0.0;
    for (uint32_t att = 0; att < 10000; ++att) {
      draw4(seed, pid, step, TAG_INJECT, 2 + att, ua);
      w = s * sqrt(ua[0]) - s;
      if (ua[1] < exp(-w * w)) break;
    }
    return w + s;
  }
  double sg = -s, t = 0.0;
  for (uint32_t att = 0; att < 10000; ++att) {
    draw4(seed, pid, step, TAG_INJECT, 2 + att, ua);
    if (sg < 1.0) {
      t = sqrt(-log(ua[0]));
      if (ua[1] < exp(-2.0 * sg * t)) break;
    } else {
      t = (-log(ua[0]) - log(ua[1])) / (2.0 * sg);
      if (ua[2] < exp(-t * t)) break;
    }
  }
  return t;
}

static void inject(const orc_grid* gr, const orc_gas* g, const orc_bc* bc, double dt, orc_parts* p,
                   uint64_t seed, uint64_t step, int32_t f32, int64_t* counters) {
  if (gr->dim != 2) return;
  int nx = gr->nx, ny = gr->ny;
  int64_t nf = 2 * (int64_t)ny + 2 * (int64_t)nx;
  double R = orc_R(g), T = bc->fs_T, sig = sqrt(R * T), vs = sqrt(2.0 * R * T);
  const double xlo = store(gr->x0, f32), xhi = edge(gr->x0, gr->dx, nx, f32);
  const double ylo = store(gr->y0, f32), yhi = edge(gr->y0, gr->dy, ny, f32);
  int64_t* cnt = (int64_t*)calloc((size_t)nf, sizeof(int64_t));
  int64_t total = 0;
  for (int64_t f = 0; f < nf; ++f) {
    int side = (f < ny) ? 0 : (f < 2 * ny) ? 1 : (f < 2 * ny + nx) ? 2 : 3;
    if (bc->kind[side] != ORC_BC_FREESTREAM) continue;
    double Un = (side == 0) ? bc->fs_U[0] : (side == 1) ? -bc->fs_U[0]
              : (side == 2) ? bc->fs_U[1] : -bc->fs_U[1];
    double area = (side < 2 ? gr->dy : gr->dx) * bc->depth;
    double lam = flux_per_area(bc->fs_n, R, T, Un) * area * dt / gr->fnum;
    double u4[4];
    draw4(seed, (uint32_t)f, step, TAG_FACE, 0, u4);
    cnt[f] = (int64_t)floor(lam + u4[0]);
    total += cnt[f];
  }
  int64_t avail = p->cap - p->n;
  if (total > avail) {
    counters[ORC_CNT_CAPACITY] += total - avail;
    total = avail;
  }
  int64_t k = 0;
  for (int64_t f = 0; f < nf && k < total; ++f) {
    int side = (f < ny) ? 0 : (f < 2 * ny) ? 1 : (f < 2 * ny + nx) ? 2 : 3;
    int64_t loc = (side == 0) ? f : (side == 1) ? f - ny : (side == 2) ? f - 2 * ny : f - 2 * ny - nx;
    double Un = (side == 0) ? bc->fs_U[0] : (side == 1) ? -bc->fs_U[0]
              : (side == 2) ? bc->fs_U[1] : -bc->fs_U[1];
    for (int64_t q = 0; q < cnt[f] && k < total; ++q, ++k) {
      int64_t i = p->n + k;
      uint32_t pid = (uint32_t)(p->next_pid + (uint64_t)k);
      double u[8];
      draw4(seed, pid, step, TAG_INJECT, 0, u);
      draw4(seed, pid, step, TAG_INJECT, 1, u + 4);
      double vn = orc_inflow_speed(seed, step, pid, Un / vs) * vs;
      double rr = sqrt(-2.0 * log(u[4]));
      double ga = sig * rr * cos(2.0 * PI * u[5]), gb = sig * rr * sin(2.0 * PI * u[5]);
      double x, y, cx, cy, cz = bc->fs_U[2] + gb;
      if (side < 2) {
        x = (side == 0) ? xlo : xhi;
        y = gr->y0 + ((double)loc + u[0]) * gr->dy;
        cx = (side == 0) ? vn : -vn;
        cy = bc->fs_U[1] + ga;
      } else {
        y = (side == 2) ? ylo : yhi;
        x = gr->x0 + ((double)loc + u[0]) * gr->dx;
        cy = (side == 2) ? vn : -vn;
        cx = bc->fs_U[0] + ga;
      }
      double tf = u[1] * dt;
      x += cx * tf;
      y += cy * tf;
      double lvl = floor(log(u[3]) / (-g->theta_vib / T));
      p->x[i] = store(x, f32);
      p->y[i] = store(y, f32);
      p->cx[i] = store(cx, f32);
      p->cy[i] = store(cy, f32);
      p->cz[i] = store(cz, f32);
      p->erot[i] = store(-R * T * log(u[2]), f32);
      p->vib[i] = (lvl > ORC_VIB_MAX) ? ORC_VIB_MAX : (int32_t)lvl;
      p->pid[i] = pid;
      int out = !(p->x[i] >= xlo && p->x[i] < xhi && p->y[i] >= ylo && p->y[i] < yhi) ||
                inside_cyl(bc, p->x[i], p->y[i]);
      p->cell[i] = out ? -1 : cell_of(gr, p->x[i], p->y[i], f32);
      if (out) counters[ORC_CNT_DELETED] += 1;
    }
  }
  p->n += total;
  p->next_pid += (uint64_t)total;
  counters[ORC_CNT_INJECTED] += total;
  free(cnt);
}

int orc_advect(const orc_grid* gr, const orc_gas* g, const orc_bc* bc, double dt, orc_parts* p,
               uint64_t seed, uint64_t step, int32_t f32, int64_t* counters) {
  if (gr->dim == 0) return 0;
  int64_t cnt[ORC_NCNT];
  memset(cnt, 0, sizeof(cnt));
  int64_t n = p->n;
#pragma omp parallel
  {
    int64_t lc[ORC_NCNT];
    memset(lc, 0, sizeof(lc));
#pragma omp for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      if (p->cell[i] < 0) continue;
      /* body-force kick, then the flight */
      p->cx[i] = store(p->cx[i] + bc->g[0] * dt, f32);
      p->cy[i] = store(p->cy[i] + bc->g[1] * dt, f32);
      p->cz[i] = store(p->cz[i] + bc->g[2] * dt, f32);
      flight(gr, g, bc, dt, p, i, seed, step, f32, lc);
    }
#pragma omp critical
    for (int k = 0; k < ORC_NCNT; ++k) cnt[k] += lc[k];
  }
  inject(gr, g, bc, dt, p, seed, step, f32, cnt);
  if (counters)
    for (int k = 0; k < ORC_NCNT; ++k) counters[k] += cnt[k];
  return 0;
}

/* ======================================================================== */
/* One full step: bin, moments, cell state, collide, conserve, advect.      */
/* After the call, *p holds the state (the two buffers are swapped as      */
/* needed).                                                                 */
/* ======================================================================== */
int orc_step(const orc_grid* gr, const orc_gas* g, const orc_bc* bc, double dt,
             const double* dt_cell, orc_parts* p, orc_parts* p_alt, int64_t* offsets, double* mom,
             double* cs, uint64_t seed, uint64_t step, int32_t nsteps, int32_t f32,
             int64_t* counters) {
  for (int32_t s = 0; s < nsteps; ++s) {
    uint64_t st = step + (uint64_t)s;
    if (orc_bin(gr, p, p_alt, offsets, f32, counters)) return -1;
    orc_parts tmp = *p;
    *p = *p_alt;
    *p_alt = tmp;
    orc_moments(gr, g, p, offsets, mom);
    orc_cellstate(gr, g, mom, dt, dt_cell, cs);
    orc_collide(gr, g, cs, offsets, p, seed, st, f32, counters);
    orc_conserve(gr, g, cs, offsets, p, seed, st, f32, counters);
    orc_advect(gr, g, bc, dt, p, seed, st, f32, counters);
  }
  return 0;
}
