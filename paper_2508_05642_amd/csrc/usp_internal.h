// usp_internal.h -- shared declarations of libusp's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/usp.h"

namespace usp {

// moment planes, mom[k*M + c] (per unit mass, central about U)
enum Mom {
  M_N = 0, M_UX, M_UY, M_UZ, M_PXX, M_PYY, M_PZZ, M_PXY, M_PXZ, M_PYZ, M_EROT, M_IBAR,
  M_QTRX, M_QTRY, M_QTRZ, M_QROTX, M_QROTY, M_QROTZ, M_QIX, M_QIY, M_QIZ, NMOM
};
static_assert(NMOM == USP_NMOM, "moment plane count");

// cell-state planes, cs[k*M + c]
enum Cs {
  CS_NP = 0, CS_NDENS, CS_UX, CS_UY, CS_UZ, CS_TTR, CS_TROT, CS_TVIB,
  CS_PXX, CS_PYY, CS_PZZ, CS_PXY, CS_PXZ, CS_PYZ, CS_ETR, CS_EROT, CS_EVIB,
  CS_MU, CS_MUP, CS_TAUC, CS_ZROT, CS_ZVIB, CS_PR, CS_DT, CS_A, CS_B, CS_R2, CS_R3,
  CS_ALPHA, CS_OMA2, CS_NU, CS_EROT_NEW, CS_EVIB_NEW, CS_COLLIDE, CS_NBR_OK,
  // first-order FPM only: tau and the cell relaxation temperatures / level
  CS_FPM_TAU, CS_FPM_TTR_REL, CS_FPM_TROT_REL, CS_FPM_MREL, NCS
};
static_assert(NCS == USP_NCS, "cell-state plane count");

// Packed per-cell record for the particle update, stored after the FP64
// cell-state planes: the reconstructed fields and temperature floors in
// FP32, the quadrant stencils, and the cell coefficients.
struct alignas(16) CellRec {
  float U[3], T[3], P[6];  // interpolated fields (16-byte loads: 0..2)
  float fl[3];             // temperature floors, 5% of the cell values
  int32_t stencil;         // 4 quadrants x 5 bits: tx (2), ty (2), cross (1)
  float a, b, al, nu;
  double oma2, r2, A2, Pr, dt;
  int32_t collide, pad;
};
static_assert(sizeof(CellRec) == 128, "cell record size");

// Coefficients of the particle update taken from the cell (the per-cell
// reading of the coefficient chain): the chain of Secs. III.A.1-III.A.3
// at the cell's temperatures and Pi, in FP64.
struct alignas(16) CellPCoef {
  double L[6];             // Cholesky factor of Lambda
  double al, oma2, Trot_rel, mstar;
  int32_t flags, pad[3];   // PC_* bits
};
static_assert(sizeof(CellPCoef) == 96, "cell coefficient record size");
enum : int32_t { PC_SKIP = 1, PC_FALLBACK = 2, PC_NU_ZERO = 4, PC_CLAMP_ROT = 8, PC_CLAMP_M = 16 };

// bytes of the cell-state buffer: FP64 planes, then one CellRec per cell,
// then one CellPCoef per cell
__host__ __device__ inline size_t cellstate_bytes(int64_t M) {
  return (size_t)M * (NCS * sizeof(double) + sizeof(CellRec) + sizeof(CellPCoef));
}
__host__ __device__ inline CellRec* cell_records(double* cs, int64_t M) { return (CellRec*)(cs + (size_t)NCS * M); }
__host__ __device__ inline const CellRec* cell_records(const double* cs, int64_t M) {
  return (const CellRec*)(cs + (size_t)NCS * M);
}
__host__ __device__ inline CellPCoef* cell_pcoefs(double* cs, int64_t M) {
  return (CellPCoef*)(cell_records(cs, M) + M);
}
__host__ __device__ inline const CellPCoef* cell_pcoefs(const double* cs, int64_t M) {
  return (const CellPCoef*)(cell_records(cs, M) + M);
}

constexpr int VIB_MAX = 255;
constexpr int MAX_BOUNCE = 8;
constexpr int NB_KMAX = 512;
constexpr double KB = 1.380649e-23;
constexpr double PI = 3.14159265358979323846;

// stream tags of the counter-based generator
enum Tag : uint32_t { TAG_COLLIDE = 0, TAG_WALL = 1, TAG_CONSERVE = 2, TAG_INJECT = 3, TAG_FACE = 5 };

// Scalars the kernels need, passed by value (one copy per launch).
struct GasP {
  double R, theta, T_ref, mu_ref, omega, K;  // K = tau_c / (mu/p)
  int zrot_model; double Z_rot, Z_rot_inf, T_star;
  int zvib_model; double Z_vib, C1, C2, sigma_vib, d_ref;
  int pr_model; double Pr_const;
  int scheme;  // USP_SCHEME_USP or USP_SCHEME_FPM
  int gamma_cell, alpha_keep;  // USP_GAMMA_CELL, USP_ALPHA_SIGN_KEEP
};

// particle-update variants of the kernels: the USP-FPM chain per particle,
// the first-order FPM method, the USP-FPM chain taken from the cell
enum : int { MODE_USP = 0, MODE_FPM = 1, MODE_CELL = 2 };
inline int update_mode(const GasP& gas) {
  return gas.scheme == USP_SCHEME_FPM ? MODE_FPM : gas.gamma_cell ? MODE_CELL : MODE_USP;
}

struct GridP {
  int dim, nx, ny;
  int64_t M;
  double x0, y0, dx, dy, fnum;
  double idx, idy;  // 1/dx, 1/dy (first guess of a cell index; stencil weights)
  double inx;       // 1/nx (first guess of a cell's row)
  const double* volume;
  const uint8_t* flags;
};

struct BcP {
  int kind[4];
  double Tw[4];
  double fs_n, fs_T, fs_U[3], depth;
  int cyl;
  double cyl_xc, cyl_yc, cyl_r, cyl_Tw;
  double g[3];
  unsigned long long* surf;  // surface sums [element][USP_SURF_NQ] or null
  int surf_nbody;
};

template <typename S>
struct PartP {
  S *x, *y, *cx, *cy, *cz, *erot;
  uint8_t* vib;
  int32_t* cell;
  uint32_t* pid;
  int64_t* count;
  int64_t capacity;
};

// host-side argument checks of usp_update (without its workspace)
bool update_args_ok(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                    const double* cs, const int64_t* offsets, const usp_particles* p);

GasP make_gas(const usp_gas* g);
GridP make_grid(const usp_grid* g);
BcP make_bc(const usp_bc* b);
template <typename S> PartP<S> make_parts(const usp_particles* p);

// workspace layout (byte offsets into the caller's scratch buffer)
struct WsLayout {
  size_t key, perm, blocksums, t9, cell_i32, old_off, far_off, far, face_cnt, face_off, misc,
      tiles, chunk_off, chunk_part, cons_scal, total;
};
// Cells split into chunks for the per-cell reductions (grids whose cells
// are far larger than a workgroup's share): slots per chunk, partial sums
// per chunk, bytes of a cell's conservation scalars, and the most chunks a
// binned state of `capacity` slots in M cells can have.
constexpr int BIG_CHUNK = 512;
constexpr int BIG_PARTS = 20;
constexpr size_t CONS_SCALAR_BYTES = 80;
inline int64_t chunks_max(int64_t capacity, int64_t M) {
  return (capacity + BIG_CHUNK - 1) / BIG_CHUNK + M;
}
// LDS stage of the fused particle phase, in particle slots (FP32 / FP64
// state), and the smallest tile window (the tile index array is sized for it)
constexpr int UPDATE_STAGE_F32 = 2048;
constexpr int UPDATE_STAGE_F64 = 1024;
constexpr int UPDATE_TILE_MIN = 128;
WsLayout ws_layout(int64_t M, int64_t capacity, int nfaces);
int n_faces(const GridP& g);

// launchers (return hipError_t of the last launch)
template <typename S>
hipError_t launch_bin(const GridP& g, const PartP<S>& in, const PartP<S>& out, int64_t* offsets,
                      const int64_t* in_offsets, char* ws, const WsLayout& L, int64_t* counters,
                      hipStream_t st, uint32_t* gather_perm = nullptr);
template <typename S>
hipError_t launch_moments(const GridP& g, const PartP<S>& p, const int64_t* offsets, double* mom,
                          hipStream_t st, const uint32_t* gather_perm = nullptr);
// the particle update's coefficients of every cell (MODE_CELL only; else
// nothing)
hipError_t launch_cell_coef(const GridP& g, const GasP& gas, double* cs, hipStream_t st);
hipError_t launch_reconstruct(const GridP& g, const GasP& gas, const double* mom, double dt,
                              const double* dt_cell, double* cs, int64_t* counters, hipStream_t st);
hipError_t launch_sample_fields(const GridP& g, const double* mom, double* acc, hipStream_t st);
template <typename S>
hipError_t launch_collide(const GridP& g, const GasP& gas, const double* cs, const int64_t* offsets,
                          const PartP<S>& p, uint64_t seed, uint64_t step, int64_t* counters,
                          hipStream_t st);
// The moments and the conservation with every cell split into chunks of
// BIG_CHUNK slots (same quantities, partial sums combined in chunk order;
// the conservation reuses the chunk index of the moments).
template <typename S>
hipError_t launch_moments_split(const GridP& g, const PartP<S>& p, const int64_t* offsets,
                                double* mom, char* ws, const WsLayout& L, hipStream_t st);
template <typename S>
hipError_t launch_conserve_split(const GridP& g, const GasP& gas, const double* cs,
                                 const int64_t* offsets, const PartP<S>& p, uint64_t seed,
                                 uint64_t step, char* ws, const WsLayout& L, int64_t* counters,
                                 hipStream_t st);
template <typename S>
hipError_t launch_conserve(const GridP& g, const GasP& gas, const double* cs,
                           const int64_t* offsets, const PartP<S>& p, uint64_t seed, uint64_t step,
                           int64_t* counters, hipStream_t st);
template <typename S>
hipError_t launch_advect(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const PartP<S>& p, uint64_t seed, uint64_t step, char* ws,
                         const WsLayout& L, int64_t* counters, hipStream_t st);

template <typename S>
hipError_t launch_inject(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const PartP<S>& p, uint64_t seed, uint64_t step, char* ws,
                         const WsLayout& L, int64_t* counters, hipStream_t st);
// The fused particle phase on p (binned), or, with gather_perm, on the
// particles of `src` in the order gather_perm gives (slot j holds
// src[gather_perm[j]]), the results written to p (whose cells the
// gathering bin has set).
template <typename S>
hipError_t launch_update(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const double* cs, const int64_t* offsets, const PartP<S>& p,
                         uint64_t seed, uint64_t step, char* ws, const WsLayout& L,
                         int64_t* counters, hipStream_t st, const PartP<S>* src = nullptr,
                         const uint32_t* gather_perm = nullptr, hipEvent_t ev_begin = nullptr,
                         hipEvent_t ev_end = nullptr);
// Adds to *found the number of NaN or infinite values among the live
// particles' floating arrays and, when given, the moment and FP64
// cell-state planes of the occupied cells.
template <typename S>
hipError_t launch_check(const GridP& g, const PartP<S>& p, const double* mom, const double* cs,
                        int64_t* found, hipStream_t st);

// first[t] (t = 0..ntiles) = first cell of tile t: the cells whose first
// particle slot lies in [t T, (t+1) T).  With stage > 0 the window T is
// update_tile(stage, offsets[M], M), taken on the device from the binned
// count (the given T must be the window of a count at least as large, so
// that ntiles tiles cover it); with stage = 0 it is T as given.
hipError_t launch_tiles(const int64_t* offsets, int64_t M, int64_t T, int64_t ntiles,
                        int32_t* first, hipStream_t st, int stage = 0);
template <typename S>
hipError_t launch_batch(const GridP& g, const GasP& gas, double dt, const double* dt_cell,
                        double* mom, double* cs, const int64_t* offsets, const PartP<S>& p,
                        int tile, int steps_per_launch, uint64_t seed, uint64_t step,
                        int nsteps, char* ws, const WsLayout& L, int64_t* counters,
                        hipStream_t st);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Tile window of the fused particle phase: a tile holds the cells whose
// first particle lies in one window, so it spans the window plus the part
// of its last cell past the window's end.  The window is the stage less
// 13/8 of the mean particles per cell (n / M), kept within [stage/8,
// 7 stage/8], so that most tiles fit the stage.  It shrinks as n grows:
// the window of the capacity bounds the number of tiles any count needs.
__host__ __device__ inline int64_t update_tile(int stage, int64_t n, int64_t M) {
  const int64_t ppc = M > 0 ? (n + M - 1) / M : stage;
  int64_t t = stage - ppc - ppc / 2 - ppc / 8;
  const int64_t lo = stage / 8, hi = stage - stage / 8;
  if (t < lo) t = lo;
  if (t > hi) t = hi;
  return t < UPDATE_TILE_MIN ? UPDATE_TILE_MIN : t;
}

}  // namespace usp
