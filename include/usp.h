/*
 * usp.h -- C ABI of libusp, the MI355X (gfx950) implementation of one time
 * step of the unified stochastic particle Fokker-Planck-Master (USP-FPM)
 * method for a diatomic gas (Kim & Jun, arXiv 2508.05642).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Arrays named in usp_particles, usp_grid and the plane buffers are DEVICE
 *   pointers owned by the caller; the library allocates nothing.  Scratch
 *   space is a caller buffer of usp_workspace_bytes() bytes.
 * - Structs themselves (usp_gas, usp_grid, usp_bc, usp_particles) live in
 *   HOST memory and are read during the call only.
 * - `stream` is a hipStream_t (passed as void*).  Every call except
 *   usp_check enqueues work on it and returns without synchronising.
 *   Nothing is copied between host and device, so those calls may be
 *   captured in a HIP graph.
 * - The live particle count and the next free particle id are device
 *   scalars (usp_particles.count[0], count[1]); kernels read them on the
 *   device, so no step needs a host round trip.
 * - Return value: USP_OK, or a negative usp_status detected on the host
 *   before anything is enqueued (USP_EINVAL), or a HIP launch error
 *   (USP_EDEVICE).  Non-fatal physics events are counted on the device in
 *   the caller's int64 counters[USP_NCOUNTERS] (see enum below); usp_check
 *   turns the counts of non-finite values and dropped injections into the
 *   statuses USP_ENUMERIC and USP_ECAPACITY.
 * - Cells are numbered c = j*nx + i (dim 2), c = j (dim 1, nx = 1), or are
 *   independent boxes c = 0..nx-1 (dim 0, ny = 1).  M = nx*ny.
 * - Plane buffers are FP64, plane-major: buf[k*M + c].
 */
#ifndef USP_H
#define USP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t usp_status;
#define USP_OK 0
#define USP_EINVAL -1      /* null pointer, bad size or dimension, dt <= 0 */
#define USP_EDEVICE -2     /* a HIP launch or runtime error */
#define USP_ECAPACITY -3   /* usp_check: injections were dropped for lack of capacity */
#define USP_ENUMERIC -4    /* usp_check: a NaN or infinite value in the state */
#define USP_EUNSUPPORTED -5
#define USP_ESCRATCH -6    /* usp_update_noalloc: needs more than its fixed scratch */

#define USP_F32 0
#define USP_F64 1

/* model switches (Sec. V.C for the temperature-dependent collision numbers,
   Sec. IV.B for the Eucken Prandtl number) */
#define USP_ZROT_CONST 0
#define USP_ZROT_PARKER 1
#define USP_ZVIB_CONST 0
#define USP_ZVIB_MW_HT 1
#define USP_PR_EUCKEN_PRINTED 0   /* xi_vib = x/(e^x - 1) as printed */
#define USP_PR_EUCKEN_STANDARD 1  /* xi_vib = 2x/(e^x - 1) */
#define USP_PR_CONST 2

/* particle scheme: the USP-FPM method (Secs. III-IV) or the first-order
   FPM method (Secs. II.B-II.C: alpha = exp(-dt/tau), tau = 2 mu (1-nu)/p,
   nu = 1 - 3/(2 Pr), cell relaxation temperatures of eqs. T_tr_FPM,
   T_rot_FPM, T_vib_FPM, vibrational jumps by Gillespie's direct method;
   its conservation keeps the sampled rotational energies and levels and
   conserves momentum and total energy through the velocities) */
#define USP_SCHEME_USP 0
#define USP_SCHEME_FPM 1

/* reading switches of the USP-FPM particle update (the defaults are the
   reading the paper's flow chart of Sec. IV.D gives; the first-order FPM
   scheme ignores both):
   gamma_scope -- the temperatures and Pi that enter the gamma coefficients,
     T-check, the relaxation temperatures (eqs. T_tr_USP, T_rot_USP,
     T_vib_USP), the diffusion tensor (eq. D_tr) and its positivity refit
     are interpolated to each particle (USP_GAMMA_PARTICLE: the chain runs
     per particle, after the interpolation) or are the cell's own
     (USP_GAMMA_CELL: the chain runs once per cell, in FP64, inside
     usp_reconstruct; the mean velocity U is still interpolated);
   alpha_sign -- of the two roots of eq. alpha_USP_positivity_2 after a
     refit, the one whose Prandtl number (eq. alpha_USP_positivity_3) is
     closer to the cell's (USP_ALPHA_SIGN_PR; ties: +) or the one with the
     sign of the cell's alpha = cbrt(r3) (USP_ALPHA_SIGN_KEEP; alpha = 0
     counts as +). */
#define USP_GAMMA_PARTICLE 0
#define USP_GAMMA_CELL 1
#define USP_ALPHA_SIGN_PR 0
#define USP_ALPHA_SIGN_KEEP 1

/* boundary kinds, per domain side */
#define USP_BC_PERIODIC 0
#define USP_BC_DIFFUSE 1     /* isothermal wall, full accommodation */
#define USP_BC_SPECULAR 2    /* symmetry plane */
#define USP_BC_FREESTREAM 3  /* particles leaving are removed; free stream injected */
#define USP_BC_OUTFLOW 4     /* particles leaving are removed */
#define USP_SIDE_XLO 0
#define USP_SIDE_XHI 1
#define USP_SIDE_YLO 2
#define USP_SIDE_YHI 3

/* cell flags */
#define USP_FLAG_SOLID 1u  /* inside the body: particles found there are removed */
#define USP_FLAG_CUT 2u    /* cut by the body: collides, but is not a stencil neighbour */

/* device event counters (int64 each) */
enum {
  USP_CNT_PB_CLAMP = 0,      /* binomial p_B > 1 clamped to 1 (Sec. III.A.2 caveat) */
  USP_CNT_CHOL_FALLBACK = 1, /* Cholesky test failed; nu/alpha refit (Sec. III.A.3) */
  USP_CNT_NU_ZERO = 2,       /* refit still not positive definite; nu = 0 */
  USP_CNT_TREL_SKIP = 3,     /* T_tr^rel <= 0: particle not updated */
  USP_CNT_TREL_CLAMP = 4,    /* T_rot^rel < 0 or mean level m* < 0 set to 0 */
  USP_CNT_VIB_SAT = 5,       /* level clamped at 255 */
  USP_CNT_INTERP_CLAMP = 6,  /* interpolated temperature raised to 5% of the cell's */
  USP_CNT_CONS_SKIP = 7,     /* a conservation scaling was skipped */
  USP_CNT_PICK_FAIL = 8,     /* vibrational correction stopped early */
  USP_CNT_CELL_SKIP = 9,     /* occupied cell skipped (fewer than 2 particles, T <= 0) */
  USP_CNT_INJECTED = 10,     /* particles created at free-stream faces */
  USP_CNT_DELETED = 11,      /* particles removed at free-stream/outflow faces */
  USP_CNT_WALL_HITS = 12,    /* diffuse re-emissions */
  USP_CNT_BOUNCE_LIMIT = 13, /* flight stopped at the re-emission limit */
  USP_CNT_CAPACITY = 14,     /* injections dropped: capacity reached */
  USP_CNT_SOLID_DROP = 15,   /* particles found in a solid cell and removed */
  USP_CNT_NONFINITE = 16,    /* occupied cells with non-finite moments (not collided),
                                plus the values usp_check finds */
  USP_NCOUNTERS = 17
};

/* Gas model.  Sec. II.A (harmonic oscillator, Landau-Teller relaxation
   times tau_rot = Z_rot tau_c, tau_vib = Z_vib tau_c), Sec. IV.A (viscosity
   mu = mu_ref (T/T_ref)^omega and mean collision time tau_c = K mu/p with the
   VSS factor K(alpha_vss, omega)), Sec. IV.B (Prandtl number), Sec. V.C
   (Parker and Millikan-White + high-temperature collision numbers). */
typedef struct {
  double m;          /* molecular mass [kg]; R = k_B/m */
  double theta_vib;  /* characteristic vibrational temperature [K] */
  double T_ref;      /* viscosity reference temperature [K] */
  double mu_ref;     /* viscosity at T_ref [Pa s] */
  double omega;      /* viscosity index */
  double alpha_vss;  /* VSS scattering parameter (1 = VHS) */
  int32_t zrot_model;
  double Z_rot, Z_rot_inf, T_star;
  int32_t zvib_model;
  double Z_vib, C1, C2, sigma_vib, d_ref;
  int32_t pr_model;
  double Pr_const;
  int32_t scheme;    /* USP_SCHEME_USP or USP_SCHEME_FPM */
  int32_t gamma_scope; /* USP_GAMMA_PARTICLE or USP_GAMMA_CELL */
  int32_t alpha_sign;  /* USP_ALPHA_SIGN_PR or USP_ALPHA_SIGN_KEEP */
} usp_gas;

/* Uniform Cartesian grid (the uniform grid of Sec. III.B).  volume and flags
   are DEVICE arrays of M entries; flags may be NULL. */
typedef struct {
  int32_t dim;       /* 0: independent boxes, 1: y only, 2: x and y */
  int32_t nx, ny;
  double x0, y0, dx, dy;
  double fnum;       /* real molecules per simulated particle */
  const double* volume;
  const uint8_t* flags;
} usp_grid;

/* Boundaries (host struct).  The paper names diffuse isothermal walls, a
   symmetry plane and a free stream (Secs. V.B, V.C); kinds per side.
   Surface sampling (the wall fluxes behind the surface coefficients C_f,
   C_h, the drag and the peak heat flux of Sec. V.C): when `surf` is not
   NULL every diffuse re-emission adds the momentum and energy that the
   particle gives the wall to its surface element, see USP_SURF_* below. */
typedef struct {
  int32_t kind[4];   /* USP_BC_* for xlo, xhi, ylo, yhi */
  double Tw[4];      /* diffuse-wall temperature per side [K] */
  double fs_n;       /* free-stream number density [1/m^3] */
  double fs_T;       /* free-stream temperature, all modes [K] */
  double fs_U[3];    /* free-stream velocity [m/s] */
  double depth;      /* z extent [m] used for injection face areas */
  int32_t cyl;       /* 1: a cylinder (a circle in x,y) is present */
  double cyl_xc, cyl_yc, cyl_r, cyl_Tw;
  double g[3];       /* body acceleration [m/s^2], applied before the flight */
  int64_t* surf;     /* DEVICE int64[usp_surf_elements() * USP_SURF_NQ] or NULL */
  int32_t surf_nbody;/* angular elements on the cylinder (0: body not sampled) */
} usp_bc;

/* Surface elements: ylo wall [0, nx) by the x cell of the hit point, yhi
   wall [nx, 2nx), xlo wall [2nx, 2nx+ny) by the y cell, xhi wall
   [2nx+ny, 2nx+2ny), cylinder [2nx+2ny, +surf_nbody) by the angle
   Theta = atan2(|y - yc|, xc - x) in [0, pi] from the upstream stagnation
   point, surf_nbody equal bins (the two halves of a full cylinder share a
   bin).  Per element USP_SURF_NQ int64 sums, row-major surf[e*NQ + q],
   accumulated with integer atomics in fixed point, so the totals do not
   depend on the order of the hits.  Per hit, with c_in/c_out the velocity
   before/after the re-emission and n the unit normal into the gas (t the
   tangent: +x on the y walls, +y on the x walls, increasing Theta on the
   cylinder), all per unit mass:
     HITS  1
     PX, PY, PZ  (c_in - c_out) * USP_SURF_P_SCALE      [m/s -> fixed]
     PN  -(c_in - c_out).n * USP_SURF_P_SCALE  (pressure part)
     PT   (c_in - c_out).t * USP_SURF_P_SCALE  (shear part)
     ETR  (|c_in|^2 - |c_out|^2)/2 * USP_SURF_E_SCALE   [J/kg -> fixed]
     EROT (eps_in - eps_out) * USP_SURF_E_SCALE
     QVIB I_in - I_out  (quanta; energy R theta_vib each)
   each value rounded to the nearest integer (ties to even) before it is
   added.  Multiply by m * fnum / (area * time) for fluxes.  The caller
   zeroes the buffer; sums overflow only past ~1e9 hits per element. */
enum {
  USP_SURF_HITS = 0, USP_SURF_PX = 1, USP_SURF_PY = 2, USP_SURF_PZ = 3,
  USP_SURF_PN = 4, USP_SURF_PT = 5, USP_SURF_ETR = 6, USP_SURF_EROT = 7,
  USP_SURF_QVIB = 8, USP_SURF_NQ = 9
};
#define USP_SURF_P_SCALE 65536.0
#define USP_SURF_E_SCALE 16.0

/* Particle state (Sec. II.A: position, velocity, rotational energy,
   vibrational level), structure of arrays in DEVICE memory, `capacity`
   entries each.  x is unused (may be NULL) unless dim = 2; y unused unless
   dim >= 1.  Floating arrays hold float (USP_F32) or double (USP_F64).
   count is a device int64[2]: live particle count, next particle id. */
typedef struct {
  int32_t prec;
  int64_t capacity;
  void* x;
  void* y;
  void* cx;
  void* cy;
  void* cz;
  void* erot;        /* rotational energy per unit mass [J/kg] */
  uint8_t* vib;      /* vibrational level I (energy I R theta_vib) */
  int32_t* cell;     /* cell index; -1 marks a removed particle */
  uint32_t* pid;     /* particle id: the random-stream key */
  int64_t* count;
} usp_particles;

/* ---- plane layouts ------------------------------------------------------ */
/* Moment planes (Sec. II.A, per unit mass, central about U):
   N, U(3), Pi(6: xx yy zz xy xz yz), e_rot, mean level, q_tr(3) =
   (1/2)<C^2 C>, q_rot(3) = <C eps_rot>, <C I>(3) (times R theta = q_vib). */
#define USP_NMOM 21
/* Cell-state buffer: USP_NCS FP64 planes (names: usp_cs_name(k)) followed
   by one packed 128-byte record per cell that the particle update reads
   and one 96-byte record per cell of the coefficients the particle update
   takes from the cell under USP_GAMMA_CELL; usp_cellstate_bytes() gives
   its size. */
#define USP_NCS 39
/* Field-sampling planes: running sums over sampled steps of the per-cell
   raw particle sums (the time averages of the cylinder case, Sec. V.C):
   N, sum c(3), sum c_i c_j(6: xx yy zz xy xz yz), sum eps_rot, sum I,
   sum (1/2)|c|^2 c(3), sum c eps_rot(3), sum c I(3). */
#define USP_NSAMP 21

const char* usp_status_str(usp_status s);
const char* usp_mom_name(int32_t k);
const char* usp_cs_name(int32_t k);
const char* usp_counter_name(int32_t k);
const char* usp_version(void);

/* Bytes of the cell-state buffer `cs` for this grid (0 if the grid is
   invalid). */
size_t usp_cellstate_bytes(const usp_grid* grid);

/* Number of surface elements for this grid and bc (2 nx + 2 ny +
   bc->surf_nbody), or 0 if an argument is invalid. */
int64_t usp_surf_elements(const usp_grid* grid, const usp_bc* bc);

/* Bytes of scratch the caller passes as `ws` to usp_bin, usp_advect,
   usp_update and usp_step for this grid and particle capacity. */
size_t usp_workspace_bytes(const usp_grid* grid, int64_t capacity);

/* Bin (the per-cell organisation the collision step of Sec. IV.D loops
   over): cell of each live particle from its position (dim >= 1; cell =
   number of cell edges, in the stored precision, at or below the
   coordinate) or from in->cell (dim 0); particles marked -1 or in a solid
   cell are dropped; the rest are written to `out` sorted by cell, stable in
   input order.  offsets: device int64[M+1], cell c owns [offsets[c],
   offsets[c+1]).  out->count[0] becomes the kept count, out->count[1] =
   in->count[1].  in and out must not alias.
   in_offsets (device int64[M+1], may be NULL, may alias offsets): when the
   input's first in_offsets[M] particles are the output of an earlier bin
   with these offsets (updated in place since, as usp_step does, with any
   later particles appended), the fast route that exploits it is taken.
   On that route the prefix particles' in->cell must be current (the cell of
   the position, or -1 if removed, as usp_advect and usp_update leave it):
   their cells are taken from in->cell, not recomputed from positions.
   Appended particles, and every particle when in_offsets is NULL, are
   binned from their positions.  NULL means nothing is known. */
usp_status usp_bin(const usp_grid* grid, const usp_particles* in, usp_particles* out,
                   int64_t* offsets, const int64_t* in_offsets, void* ws, size_t ws_bytes,
                   int64_t* counters, void* stream);

/* The bin of usp_bin without moving the particles: perm (device
   uint32[out->capacity]) receives, for every output slot j, the input index
   of the particle usp_bin would place there; out->cell[j] receives its cell;
   offsets and out->count as usp_bin sets them.  The other arrays of `out`
   are left as they are.  Same arguments and errors as usp_bin otherwise.
   With usp_moments_gather and usp_update_gather this is the step without
   the copy of the particle state into the binned order (usp_step uses it). */
usp_status usp_bin_gather(const usp_grid* grid, const usp_particles* in, usp_particles* out,
                          int64_t* offsets, const int64_t* in_offsets, uint32_t* perm, void* ws,
                          size_t ws_bytes, int64_t* counters, void* stream);

/* usp_moments of the state usp_bin would have produced, reading slot j from
   in[perm[j]] (perm and offsets from usp_bin_gather).  Bit-identical to
   usp_bin followed by usp_moments.  Errors: USP_EINVAL for a null
   argument. */
usp_status usp_moments_gather(const usp_grid* grid, const usp_particles* in, const uint32_t* perm,
                              const int64_t* offsets, double* mom, void* stream);

/* usp_update of the state usp_bin would have produced, reading slot j from
   in[perm[j]] and writing the whole result state in slot order to `out`
   (whose cells and count usp_bin_gather set), injection included.  in and
   out must differ; bit-identical to usp_bin followed by usp_update.
   ev_begin, ev_end (hipEvent_t, may be NULL): when given, recorded on
   `stream` immediately before and after the launch of the particle kernel
   itself (not the tile-index and injection kernels around it), so that a
   caller can time that kernel alone.
   Errors: USP_EINVAL for a null or inconsistent argument, in == out, or a
   short ws. */
usp_status usp_update_gather(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                             const double* cs, const int64_t* offsets, const usp_particles* in,
                             const uint32_t* perm, usp_particles* out, void* ws, size_t ws_bytes,
                             uint64_t seed, uint64_t step, int64_t* counters, void* ev_begin,
                             void* ev_end, void* stream);

/* Moments (Sec. II.A) of every cell from a binned state: mom = device
   double[USP_NMOM*M].  One pass per cell over sums shifted by the cell's
   first particle (for FP32 states every shifted difference is exact in
   FP64), accumulated in FP64 in a fixed order (deterministic); the central
   moments follow from the shifted sums. */
usp_status usp_moments(const usp_grid* grid, const usp_particles* p, const int64_t* offsets,
                       double* mom, void* stream);

/* Field sampling (the N_sampling phase of Sec. V.C): acc (device
   double[USP_NSAMP*M], plane-major, zeroed by the caller before the first
   sample) += the raw particle sums of each cell formed from the moment
   planes `mom` of usp_moments (N, N U, N (Pi + U U), N e_rot, N I_mean,
   N ((1/2)|U|^2 U + Pi U + tr(Pi) U/2 + q_tr), N (U e_rot + q_rot),
   N (U I_mean + <C I>)).  Thread per cell, no atomics: deterministic.
   To sample every step, call usp_step with nsteps = 1 and this after it
   (mom then holds the step's pre-collision moments). */
usp_status usp_sample_fields(const usp_grid* grid, const double* mom, double* acc,
                             void* stream);

/* Cell state (Secs. II.A, III.A.1, III.A.2, IV.A, IV.B): temperatures,
   viscosity, tau_c, Z's, Pr, the USP-FPM coefficients alpha (eq.
   USP-FPM_alpha_tr), nu (eq. USP-FPM_nu), a = dt/(dt + 2 tau_rot), b =
   dt/(dt + 2 tau_vib), the cell energy targets of eqs. e_rot/e_vib_relax and
   the stencil usability flag and quadrant stencils used by the
   reconstruction (Sec. III.B).  cs = device buffer of usp_cellstate_bytes().  dt_cell (device, M) overrides dt per cell
   when not NULL (independent 0D boxes). */
usp_status usp_reconstruct(const usp_grid* grid, const usp_gas* gas, const double* mom,
                           double dt, const double* dt_cell, double* cs, int64_t* counters,
                           void* stream);

/* Collision (Secs. III.A.2, III.A.3, flow chart of Sec. IV.D): for every
   particle of a colliding cell, the first-order polynomial reconstruction of
   U, T_tr, T_rot, T_vib, Pi at its position, the relaxation temperatures
   (eqs. T_tr_USP, T_rot_USP, T_vib_USP), the diffusion tensor (eq. D_tr)
   with its Cholesky test and positivity fallback, and the velocity (eq.
   update_ci), rotational (eq. update_erot) and vibrational (eq.
   update_evib) updates.  Random numbers: Philox4x32-10 keyed by `seed`,
   counter (pid, step, 0, block).  In-place on p (binned). */
usp_status usp_collide(const usp_grid* grid, const usp_gas* gas, const double* cs,
                       const int64_t* offsets, usp_particles* p, uint64_t seed, uint64_t step,
                       int64_t* counters, void* stream);

/* Conservation (Sec. IV.C), per colliding cell: integer vibrational
   correction by random level moves, rotational scaling to the cell target,
   velocity scaling conserving momentum and total energy.  Picks draw from
   Philox counter (cell, step, 2, j).  In-place on p (binned). */
usp_status usp_conserve(const usp_grid* grid, const usp_gas* gas, const double* cs,
                        const int64_t* offsets, usp_particles* p, uint64_t seed, uint64_t step,
                        int64_t* counters, void* stream);

/* Advection (free flight x += c dt, Sec. II.C) with body force and the
   boundaries of usp_bc; diffuse re-emissions draw from counter (pid, step,
   1, block).  Removed particles get cell -1; survivors get their new cell.
   Free-stream faces then inject new particles after the live ones (ids
   count[1], count[1]+1, ...; draws from (face, step, 5, 0) and (pid, step, 3,
   block)); count[] is advanced on the device.  With bc->surf set, every
   diffuse re-emission is added to its surface element (see usp_bc).
   No-op for dim 0. */
usp_status usp_advect(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                      usp_particles* p, uint64_t seed, uint64_t step, void* ws, size_t ws_bytes,
                      int64_t* counters, void* stream);

/* The particle phase of a step in one pass: usp_collide, usp_conserve and
   usp_advect (with injection) fused, bit-identical to calling the three in
   that order (Secs. III.A-III.B, IV.C and the flow chart of Sec. IV.D).
   p must be binned with `offsets` (count[0] == offsets[M], as usp_bin
   leaves it); particles past offsets[M] are not updated.  cs from
   usp_reconstruct of the same state.  bc and dt > 0 are required for
   dim >= 1; for dim 0 bc may be NULL and dt is unused (no flight).  A
   workgroup owns the cells whose first particle lies in one window of
   particle slots: its LDS stage (2048 FP32 / 1024 FP64 slots) less 1.25x
   the mean slots per cell (capacity / M), kept within 1/8..7/8 of the
   stage; tile boundaries go to `ws`.
   Errors: USP_EINVAL for a null or inconsistent argument or a short ws. */
usp_status usp_update(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                      const double* cs, const int64_t* offsets, usp_particles* p,
                      void* ws, size_t ws_bytes, uint64_t seed, uint64_t step,
                      int64_t* counters, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid allocation): the
   fused particle phase of usp_update with its scratch (the tile index and
   the injection's face counts, offsets and totals) in a fixed device array
   of USP_NOALLOC_SCRATCH_BYTES inside the library instead of a caller
   workspace.  Same arguments, results (the same kernels: bit-identical to
   usp_update) and errors as usp_update, less ws and ws_bytes; the call
   allocates nothing.  Each GPU holds its own copy of the array from the
   first call on it until the process ends; its address is looked up once
   per GPU on that first call.  Calls on one GPU share the array: calls that
   may overlap on one GPU (different streams, or one stream from several
   host threads without ordering) race and must not be issued.  Nothing in
   the array needs to start at zero (every call writes what it reads).
   Returns USP_ESCRATCH when the grid's faces and the capacity's tile index
   need more than the array holds (about 2.6e5 tiles: e.g. 4.0e8 particle
   slots for the cylinder's cells, whose launch bound is a 1527-slot
   window), USP_EDEVICE when the array's
   address cannot be found. */
#define USP_NOALLOC_SCRATCH_BYTES (1 << 20)
usp_status usp_update_noalloc(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc,
                              double dt, const double* cs, const int64_t* offsets,
                              usp_particles* p, uint64_t seed, uint64_t step, int64_t* counters,
                              void* stream);

/* nsteps full steps of independent 0D cells (dim 0) in few launches: per
   step the moments and cell state of each cell (Secs. II.A, III.A, IV.A,
   IV.B), the particle update and the conservation (Secs. III.A-III.B, IV.C),
   with no rebin (0D particles never change cell).  A workgroup owns a tile
   of whole cells and keeps their particles in LDS for all the steps of a
   launch; the tiles are dispatched by descending particle count (the tile
   order goes to `ws`).  Bit-identical to usp_step on the same state.
   p must be binned with `offsets` (count[0] == offsets[M]; a first
   usp_bin or usp_step leaves it so).  dt_cell (device double[M], may be
   NULL) overrides dt per cell.  mom and cs as for usp_moments /
   usp_reconstruct; they describe the last step's pre-collision state on
   return.  tile: particle slots per tile window (512, 1024 or 2048; 0 =
   1024; FP64 states: 0 or 512).  steps_per_launch: steps each launch runs
   (0 = all nsteps in one launch).  Errors: USP_EINVAL for dim != 0, a
   null or inconsistent argument, a tile value not listed, or a short ws. */
usp_status usp_batch(const usp_grid* grid, const usp_gas* gas, double dt, const double* dt_cell,
                     usp_particles* p, const int64_t* offsets, double* mom, double* cs, void* ws,
                     size_t ws_bytes, int32_t tile, int32_t steps_per_launch, uint64_t seed,
                     uint64_t step, int32_t nsteps, int64_t* counters, void* stream);

/* nsteps full steps (bin, moments, reconstruct, then the fused particle
   phase of usp_update) starting at step index `step`; in 0D only the first
   step bins.  p and p_alt are the two particle buffers;
   on return *p describes the buffer that holds the state (the two structs
   are swapped as needed); the two buffers must have equal capacities (the
   state moves between them every step) and distinct arrays, and ws is sized
   for that capacity.  offsets, mom, cs as above (they describe the last
   step's pre-collision state on return).  in_offsets (may be NULL, may
   alias offsets) is passed to the first step's usp_bin: when *p is the
   state a previous step or bin left (segments in in_offsets), the first
   bin takes the fast route too; later steps always do. */
usp_status usp_step(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                    const double* dt_cell, usp_particles* p, usp_particles* p_alt,
                    int64_t* offsets, const int64_t* in_offsets, double* mom, double* cs,
                    void* ws, size_t ws_bytes, uint64_t seed, uint64_t step, int32_t nsteps,
                    int64_t* counters, void* stream);

/* State check (the USP_ENUMERIC and USP_ECAPACITY statuses): scans the
   live particles of p (count[0], read on the device) for NaN or infinite
   x, y (as the grid uses them), cx, cy, cz and erot, and, when not NULL,
   the moment planes mom (USP_NMOM*M) and the FP64 cell-state planes cs
   (USP_NCS*M) of the occupied cells; the number of non-finite values found
   is added to counters[USP_CNT_NONFINITE] (counters is required).  Unlike
   every other entry point this call WAITS for `stream` (it copies the
   counters to the host), so it cannot be captured in a HIP graph.
   Returns USP_ENUMERIC if counters[USP_CNT_NONFINITE] is then non-zero
   (cells flagged by usp_reconstruct count too), else USP_ECAPACITY if
   counters[USP_CNT_CAPACITY] is non-zero, else USP_OK; *nonfinite (host,
   may be NULL) receives the number of values this scan found.  Errors:
   USP_EINVAL for a null or inconsistent argument, USP_EDEVICE for a HIP
   error. */
usp_status usp_check(const usp_grid* grid, const usp_particles* p, const double* mom,
                     const double* cs, int64_t* counters, int64_t* nonfinite, void* stream);

/* ---- pathwise adjoint (1D, FP64 state, USP-FPM scheme) -------------------
   Gradients of two time-averaged outputs of a run with respect to the
   collision-model parameters theta = (Z_rot, omega, mu_ref) (constant
   collision numbers; Sec. IV.A viscosity and tau_c, Sec. III.A.1 relaxation
   times), taken along the path of the run with every discrete outcome held
   fixed: cells and bin order, vibrational levels after the jumps (Sec.
   III.A.2) and the picks (Sec. IV.C), the stencil and the 5% temperature
   floor (Sec. III.B), the Cholesky test (a particle whose test fails keeps
   its post-collision state as a constant, Sec. III.A.3), the clamp of
   T_rot^rel, the skips of the conservation scalings, and every boundary
   event of the flight (a particle that meets a wall keeps its re-emitted
   velocity, energy and level as constants; its position after the flight
   follows the time of its first hit, the flights between walls after it
   keeping their durations).  The outputs, for a run of K steps, area =
   volume[0]/dy:
     J0 = w_mdot * sum over steps of sum_i c_x,i at the start of the step,
     J1 = w_tau * sum over steps of sum over particles whose flight meets a
          boundary of (c_x after the kick - c_x after the flight),
   with the weights given by the caller (m fnum/(area K) gives the mass flow
   per unit depth, m fnum/(2 area K dt) the mean shear of the two walls).
   Adjoint arrays `lam` are device double[2][5][capacity]: objective, then
   y, cx, cy, cz, erot, then particle slot.  Requires particle ids below
   capacity (1D runs create no particles).  Errors: USP_EINVAL for a grid
   that is not 1D, a non-FP64 state, the first-order FPM scheme, a
   temperature-dependent collision-number model, a reading switch other
   than USP_GAMMA_PARTICLE and USP_ALPHA_SIGN_PR, or short buffers. */
size_t usp_tape_bytes(const usp_grid* grid, int64_t capacity);
size_t usp_adjoint_ws_bytes(const usp_grid* grid, int64_t capacity);

/* One full step (the bits of usp_step) that also writes the tape of the
   step (bin permutation, binned pre-collision state, cell state, states
   after the collision and after the conservation) into `tape`
   (usp_tape_bytes); aws (usp_adjoint_ws_bytes) is scratch.  p and p_alt
   are swapped as usp_step swaps them; equal capacities; in_offsets as for
   usp_step. */
usp_status usp_step_taped(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                          usp_particles* p, usp_particles* p_alt, int64_t* offsets,
                          const int64_t* in_offsets, double* mom, double* cs, void* ws,
                          size_t ws_bytes, uint64_t seed, uint64_t step, void* tape,
                          size_t tape_bytes, void* aws, size_t aws_bytes, int64_t* counters,
                          void* stream);

/* The step recorded in `tape` (taken at step index `step` with `seed`)
   reversed: lam_in is the adjoint of the state after the step (slots as
   the step left them), lam_out receives the adjoint of the state before it
   (slots as they were before its bin), the step's own output terms
   included; grad (device double[2][3], objective-major) is incremented by
   the step's parameter terms.  lam_in and lam_out must differ.  Fixed-order
   reductions: deterministic. */
usp_status usp_adjoint_step(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                            const void* tape, size_t tape_bytes, int64_t capacity, uint64_t seed,
                            uint64_t step, const double* lam_in, double* lam_out, double w_mdot,
                            double w_tau, double* grad, void* aws, size_t aws_bytes,
                            void* stream);

#ifdef __cplusplus
}
#endif
#endif
