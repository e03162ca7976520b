/*
 * usp_oracle.h -- plain FP64 CPU reference of one time step of the unified
 * stochastic particle Fokker-Planck-Master (USP-FPM) method for a diatomic
 * gas (Kim & Jun, arXiv 2508.05642).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the oracle that the GPU path is
 * checked against.  Only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark may load it.  It shares no source with the GPU
 * library and is written for clarity, not speed: every phase is a plain loop
 * over cells or particles in FP64, in the order the paper states.
 *
 * Paper map (sections / equations of arXiv 2508.05642):
 *   gas model           Sec. II.A (energies, heat capacities, Landau-Teller),
 *                       Sec. IV.A (VSS viscosity, mean collision time),
 *                       Sec. IV.B (Eucken Prandtl number),
 *                       Sec. V.C  (Parker Z_rot, Millikan-White + high-T Z_vib)
 *   energy targets      Sec. III.A.1, eqs. e_tr/e_rot/e_vib relax, gamma
 *                       coefficients, T_1 secant, rescaled T_tr
 *   particle update     Sec. III.A.2, eqs. update_ci, USP-FPM_alpha_tr,
 *                       USP-FPM_nu, T_tr_USP, update_erot, T_rot_USP,
 *                       update_evib (NB/B parameters), T_vib_USP
 *   positivity          Sec. III.A.3, eqs. nu_USP_positivity,
 *                       alpha_USP_positivity_1..4
 *   reconstruction      Sec. III.B (uniform grid, quadrant stencils)
 *   conservation        Sec. IV.C
 *   step order          Sec. IV.D (collision-step flow chart)
 *   free flight         Sec. II.C (x^{n+1} = x^n + c^n dt)
 *
 * Parity unpinned (the paper fixes no value to check these against; only
 * the GPU/oracle parity tests and the invariants below cover them):
 *   - orc_conserve's order of the vibrational picks (which particle gets a
 *     level step, draw by draw): the total I_delta and the level bounds are
 *     pinned, the choice of particles is not;
 *   - orc_interp's rule at boundaries and solid cells (which neighbour a
 *     quadrant stencil falls back to): pinned only by exactness on bilinear
 *     fields where the whole stencil exists and on linear fields next to an
 *     unusable cell.
 */
#ifndef USP_ORACLE_H
#define USP_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_KB 1.380649e-23

/* ---- model switches ---------------------------------------------------- */
enum { ORC_ZROT_CONST = 0, ORC_ZROT_PARKER = 1 };
enum { ORC_ZVIB_CONST = 0, ORC_ZVIB_MW_HT = 1 };
enum { ORC_PR_EUCKEN_PRINTED = 0, ORC_PR_EUCKEN_STANDARD = 1, ORC_PR_CONST = 2 };

/* ---- boundary kinds ---------------------------------------------------- */
enum { ORC_BC_PERIODIC = 0, ORC_BC_DIFFUSE = 1, ORC_BC_SPECULAR = 2,
       ORC_BC_FREESTREAM = 3, ORC_BC_OUTFLOW = 4 };
enum { ORC_SIDE_XLO = 0, ORC_SIDE_XHI = 1, ORC_SIDE_YLO = 2, ORC_SIDE_YHI = 3 };

/* ---- cell flags -------------------------------------------------------- */
#define ORC_FLAG_SOLID 1u   /* cell lies entirely inside the body            */
#define ORC_FLAG_CUT   2u   /* cell is cut by the body surface               */

/* ---- event counters (same meaning as the GPU library's) ---------------- */
enum {
  ORC_CNT_PB_CLAMP = 0,      /* p_B > 1 clamped to 1                          */
  ORC_CNT_CHOL_FALLBACK = 1, /* first Cholesky test failed: nu/alpha refit    */
  ORC_CNT_NU_ZERO = 2,       /* second Cholesky test failed: nu = 0           */
  ORC_CNT_TREL_SKIP = 3,     /* T_tr^rel <= 0: particle left unchanged        */
  ORC_CNT_TREL_CLAMP = 4,    /* T_rot^rel < 0 or m* < 0 clamped to 0          */
  ORC_CNT_VIB_SAT = 5,       /* vibrational level clamped at ORC_VIB_MAX      */
  ORC_CNT_INTERP_CLAMP = 6,  /* interpolated temperature raised to the floor  */
  ORC_CNT_CONS_SKIP = 7,     /* a conservation scaling skipped (bad factor)   */
  ORC_CNT_PICK_FAIL = 8,     /* vib correction gave up before I_delta = 0     */
  ORC_CNT_CELL_SKIP = 9,     /* occupied cell skipped (N_p < 2 or T_tr <= 0)  */
  ORC_CNT_INJECTED = 10,     /* particles created at free-stream faces        */
  ORC_CNT_DELETED = 11,      /* particles removed at free-stream faces        */
  ORC_CNT_WALL_HITS = 12,    /* diffuse re-emissions                          */
  ORC_CNT_BOUNCE_LIMIT = 13, /* flight stopped at the re-emission limit       */
  ORC_CNT_CAPACITY = 14,     /* injections dropped for lack of capacity       */
  ORC_CNT_SOLID_DROP = 15,   /* particle found in a solid cell, removed       */
  ORC_CNT_NONFINITE = 16,    /* occupied cell with non-finite sums (skipped)  */
  ORC_NCNT = 17
};

#define ORC_VIB_MAX 255
#define ORC_MAX_BOUNCE 8

/* ---- gas ---------------------------------------------------------------- */
typedef struct {
  double m;          /* molecular mass [kg]                                 */
  double theta_vib;  /* characteristic vibrational temperature [K]          */
  double T_ref;      /* viscosity reference temperature [K]                 */
  double mu_ref;     /* viscosity at T_ref [Pa s]                           */
  double omega;      /* viscosity index c_omega                             */
  double alpha_vss;  /* VSS scattering parameter c_alpha (1 = VHS)          */
  int32_t zrot_model;
  double Z_rot;      /* constant Z_rot                                      */
  double Z_rot_inf;  /* Parker limit                                        */
  double T_star;     /* Parker characteristic temperature [K]               */
  int32_t zvib_model;
  double Z_vib;      /* constant Z_vib                                      */
  double C1, C2;     /* Millikan-White constants                            */
  double sigma_vib;  /* high-temperature vibrational cross-section [m^2]    */
  double d_ref;      /* reference diameter [m]                              */
  int32_t pr_model;
  double Pr_const;
  int32_t scheme;    /* ORC_SCHEME_USP or ORC_SCHEME_FPM                    */
  int32_t gamma_scope; /* ORC_GAMMA_PARTICLE or ORC_GAMMA_CELL               */
  int32_t alpha_sign;  /* ORC_ALPHA_SIGN_PR or ORC_ALPHA_SIGN_KEEP           */
} orc_gas;

/* USP-FPM (Secs. III-IV) or the first-order FPM method (Secs. II.B-II.C) */
enum { ORC_SCHEME_USP = 0, ORC_SCHEME_FPM = 1 };
/* Readings of the USP-FPM particle update.  gamma_scope: the temperatures */
/* and Pi of the coefficient chain (gammas, relaxation temperatures,       */
/* diffusion tensor and its refit) are interpolated to the particle        */
/* (PARTICLE, the flow chart of Sec. IV.D) or are the cell's own (CELL; U  */
/* is interpolated in both).  alpha_sign: after a refit, the root of eq.   */
/* alpha_USP_positivity_2 whose Prandtl number is closer to the cell's     */
/* (PR) or the one with the sign of the cell's alpha (KEEP; 0 counts +).   */
enum { ORC_GAMMA_PARTICLE = 0, ORC_GAMMA_CELL = 1 };
enum { ORC_ALPHA_SIGN_PR = 0, ORC_ALPHA_SIGN_KEEP = 1 };

/* ---- grid --------------------------------------------------------------- */
typedef struct {
  int32_t dim;       /* 0: cells are independent boxes, 1: y only, 2: x,y   */
  int32_t nx, ny;    /* cells along x and y (dim 0: nx = number of cells)   */
  double x0, y0, dx, dy;
  double fnum;       /* real molecules per simulated particle               */
  const double* volume;        /* [M] cell volumes [m^3]                    */
  const uint8_t* flags;        /* [M] ORC_FLAG_* (may be NULL)              */
} orc_grid;

/* ---- boundaries --------------------------------------------------------- */
typedef struct {
  int32_t kind[4];   /* per side, ORC_BC_*                                  */
  double Tw[4];      /* diffuse-wall temperature per side [K]               */
  double fs_n;       /* free-stream number density [1/m^3]                  */
  double fs_T;       /* free-stream temperature, all modes [K]              */
  double fs_U[3];    /* free-stream velocity [m/s]                          */
  double depth;      /* z extent used for face areas and volumes [m]        */
  int32_t cyl;       /* 1: a cylinder (circle in x,y) is present            */
  double cyl_xc, cyl_yc, cyl_r, cyl_Tw;
  double g[3];       /* body acceleration [m/s^2]                           */
  int64_t* surf;     /* surface sums [element][ORC_SURF_NQ] or NULL         */
  int32_t surf_nbody;/* angular elements on the cylinder                    */
} orc_bc;

/* ---- sampling (the N_sampling phase of Sec. V.C) ------------------------- */
/* Surface elements: ylo wall by x cell [0, nx), yhi [nx, 2nx), xlo by y    */
/* cell [2nx, 2nx+ny), xhi [2nx+ny, 2nx+2ny), cylinder by the angle from   */
/* the upstream stagnation point, Theta in [0, pi], in surf_nbody bins.    */
/* Per element, per diffuse re-emission, per unit mass, fixed point:       */
/* hits; c_in - c_out (x, y, z); its components along -n and t (n: normal  */
/* into the gas, t: +x on y walls, +y on x walls, increasing Theta on the  */
/* cylinder); (|c_in|^2 - |c_out|^2)/2; eps_in - eps_out; I_in - I_out.    */
enum {
  ORC_SURF_HITS = 0, ORC_SURF_PX, ORC_SURF_PY, ORC_SURF_PZ, ORC_SURF_PN, ORC_SURF_PT,
  ORC_SURF_ETR, ORC_SURF_EROT, ORC_SURF_QVIB, ORC_SURF_NQ
};
#define ORC_SURF_P_SCALE 65536.0   /* fixed-point units per m/s   */
#define ORC_SURF_E_SCALE 16.0      /* fixed-point units per J/kg  */
/* Field sums: N, sum c, sum c_i c_j (xx yy zz xy xz yz), sum eps_rot,      */
/* sum I, sum |c|^2 c / 2, sum c eps_rot, sum c I; plane-major [k][M].       */
#define ORC_NSAMP 21

/* ---- particles (FP64 structure of arrays) ------------------------------- */
typedef struct {
  int64_t n, cap;
  double *x, *y, *cx, *cy, *cz, *erot;
  int32_t* vib;
  int32_t* cell;
  uint32_t* pid;
  uint64_t next_pid;
} orc_parts;

/* ---- moment planes, mom[k*M + c] ---------------------------------------- */
enum {
  ORC_M_N = 0, ORC_M_UX, ORC_M_UY, ORC_M_UZ,
  ORC_M_PXX, ORC_M_PYY, ORC_M_PZZ, ORC_M_PXY, ORC_M_PXZ, ORC_M_PYZ,
  ORC_M_EROT, ORC_M_IBAR,
  ORC_M_QTRX, ORC_M_QTRY, ORC_M_QTRZ,       /* (1/2) <C^2 C_i>               */
  ORC_M_QROTX, ORC_M_QROTY, ORC_M_QROTZ,    /* <C_i eps_rot>                 */
  ORC_M_QIX, ORC_M_QIY, ORC_M_QIZ,          /* <C_i I>  (times R Theta = q_vib) */
  ORC_NMOM
};

/* ---- cell-state planes, cs[k*M + c] ------------------------------------- */
enum {
  ORC_CS_NP = 0, ORC_CS_NDENS,
  ORC_CS_UX, ORC_CS_UY, ORC_CS_UZ,
  ORC_CS_TTR, ORC_CS_TROT, ORC_CS_TVIB,
  ORC_CS_PXX, ORC_CS_PYY, ORC_CS_PZZ, ORC_CS_PXY, ORC_CS_PXZ, ORC_CS_PYZ,
  ORC_CS_ETR, ORC_CS_EROT, ORC_CS_EVIB,
  ORC_CS_MU, ORC_CS_MUP, ORC_CS_TAUC, ORC_CS_ZROT, ORC_CS_ZVIB, ORC_CS_PR,
  ORC_CS_DT, ORC_CS_A, ORC_CS_B, ORC_CS_R2, ORC_CS_R3,
  ORC_CS_ALPHA, ORC_CS_OMA2, ORC_CS_NU,
  ORC_CS_EROT_NEW, ORC_CS_EVIB_NEW,
  ORC_CS_COLLIDE, ORC_CS_NBR_OK,
  /* first-order FPM only: tau = 2 mu (1 - nu)/p and the cell relaxation */
  /* temperatures (eqs. T_tr_FPM, T_rot_FPM) and level (eq. T_vib_FPM)   */
  ORC_CS_FPM_TAU, ORC_CS_FPM_TTR_REL, ORC_CS_FPM_TROT_REL, ORC_CS_FPM_MREL,
  ORC_NCS
};

/* ---- counter-based generator (Salmon et al., SC'11) --------------------- */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* ---- gas model ---------------------------------------------------------- */
double orc_R(const orc_gas* g);
double orc_e_vib(const orc_gas* g, double T);
double orc_cv_vib(const orc_gas* g, double T);
double orc_viscosity(const orc_gas* g, double T);
double orc_tau_c_factor(const orc_gas* g);
double orc_zrot(const orc_gas* g, double T);
double orc_zvib(const orc_gas* g, double T);
double orc_prandtl(const orc_gas* g, double T);
double orc_tcheck(const orc_gas* g, double Ttr, double Trot, double Tvib, double a, double b);
void orc_gammas(const orc_gas* g, double Ttr, double Trot, double Tvib,
                double a, double b, double out_gamma[3], double* out_tcheck);
void orc_eigvals_sym3(const double P[6], double out[3]);

/* Per-particle coefficients of Secs. III.A.1-III.A.3 with the positivity
   fallback of Sec. III.A.3 (see usp_oracle.c).  L: lower Cholesky factor
   (l11, l21, l22, l31, l32, l33) of Lambda = tau D_tr; al, oma2: alpha and
   1 - alpha^2 after any refit; nu: the nu used (0 after the second
   fallback); nu_bound: the bound of eq. nu_USP_positivity on the side of
   the cell's nu (0 when the first test passed or the bound does not apply);
   Ttr_rel, Trot_rel, mstar: relaxation temperatures and mean level before
   the clamps to 0 of the update; flags: the first test failed (fallback),
   the re-test failed (nu_zero), the particle is left unchanged (skip). */
typedef struct {
  double L[6];
  double al, oma2, nu, nu_bound, Ttr_rel, Trot_rel, mstar;
  int32_t fallback, nu_zero, skip;
} orc_pcoef;
void orc_particle_coef(const orc_gas* g, double Ttr, double Trot, double Tvib, const double P[6],
                       double a, double b, double al_cell, double oma2_cell, double nu_cell,
                       double r2, double A2, double Pr, double dtc, orc_pcoef* out);

/* ---- one step, phase by phase ------------------------------------------- */
int orc_bin(const orc_grid* grid, const orc_parts* src, orc_parts* dst,
            int64_t* offsets, int32_t f32, int64_t* counters);
int orc_moments(const orc_grid* grid, const orc_gas* gas, const orc_parts* p,
                const int64_t* offsets, double* mom);
int orc_cellstate(const orc_grid* grid, const orc_gas* gas, const double* mom,
                  double dt, const double* dt_cell, double* cs);
double orc_interp(const orc_grid* grid, const double* cs, int field,
                  int32_t cell, double x, double y);
int orc_collide(const orc_grid* grid, const orc_gas* gas, const double* cs,
                const int64_t* offsets, orc_parts* p, uint64_t seed, uint64_t step,
                int32_t f32, int64_t* counters);
int orc_conserve(const orc_grid* grid, const orc_gas* gas, const double* cs,
                 const int64_t* offsets, orc_parts* p, uint64_t seed, uint64_t step,
                 int32_t f32, int64_t* counters);
void orc_collide_normals(uint64_t seed, uint64_t step, int64_t n, const uint32_t* pid,
                         double* G);
int orc_sample_fields(const orc_grid* grid, const orc_parts* p, const int64_t* offsets,
                      double* acc);
int orc_advect(const orc_grid* grid, const orc_gas* gas, const orc_bc* bc, double dt,
               orc_parts* p, uint64_t seed, uint64_t step, int32_t f32, int64_t* counters);
int orc_step(const orc_grid* grid, const orc_gas* gas, const orc_bc* bc, double dt,
             const double* dt_cell, orc_parts* p, orc_parts* p_alt, int64_t* offsets,
             double* mom, double* cs, uint64_t seed, uint64_t step, int32_t nsteps,
             int32_t f32, int64_t* counters);

/* ---- single-draw helpers exposed for distribution pins ------------------ */
int32_t orc_sample_nb(double u, int32_t r, double p);
int32_t orc_sample_b(double u, int32_t n, double p);
double orc_inflow_speed(uint64_t seed, uint64_t step, uint32_t pid, double s);

void orc_set_threads(int32_t n);
int32_t orc_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
