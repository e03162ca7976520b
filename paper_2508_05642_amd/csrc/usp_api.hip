// usp_api.hip -- C ABI of libusp: argument checks, workspace layout,
// dispatch on the state precision, and the full step.
#include <string.h>

#include "usp_internal.h"

namespace usp {

GasP make_gas(const usp_gas* g) {
  GasP p;
  p.R = KB / g->m;
  p.theta = g->theta_vib;
  p.T_ref = g->T_ref;
  p.mu_ref = g->mu_ref;
  p.omega = g->omega;
  const double a = g->alpha_vss, w = g->omega;
  p.K = a * (5.0 - 2.0 * w) * (7.0 - 2.0 * w) / (5.0 * (a + 1.0) * (a + 2.0));
  p.zrot_model = g->zrot_model; p.Z_rot = g->Z_rot; p.Z_rot_inf = g->Z_rot_inf; p.T_star = g->T_star;
  p.zvib_model = g->zvib_model; p.Z_vib = g->Z_vib; p.C1 = g->C1; p.C2 = g->C2;
  p.sigma_vib = g->sigma_vib; p.d_ref = g->d_ref;
  p.pr_model = g->pr_model; p.Pr_const = g->Pr_const;
  p.scheme = g->scheme;
  p.gamma_cell = g->gamma_scope == USP_GAMMA_CELL ? 1 : 0;
  p.alpha_keep = g->alpha_sign == USP_ALPHA_SIGN_KEEP ? 1 : 0;
  return p;
}

GridP make_grid(const usp_grid* g) {
  GridP p;
  p.dim = g->dim; p.nx = g->nx; p.ny = g->ny;
  p.M = (int64_t)g->nx * g->ny;
  p.x0 = g->x0; p.y0 = g->y0; p.dx = g->dx; p.dy = g->dy; p.fnum = g->fnum;
  p.idx = g->dx > 0.0 ? 1.0 / g->dx : 0.0;
  p.idy = g->dy > 0.0 ? 1.0 / g->dy : 0.0;
  p.inx = g->nx > 0 ? 1.0 / g->nx : 0.0;
  p.volume = g->volume; p.flags = g->flags;
  return p;
}

BcP make_bc(const usp_bc* b) {
  BcP p;
  memset(&p, 0, sizeof(p));
  if (!b) {
    for (int k = 0; k < 4; ++k) p.kind[k] = USP_BC_PERIODIC;
    return p;
  }
  for (int k = 0; k < 4; ++k) { p.kind[k] = b->kind[k]; p.Tw[k] = b->Tw[k]; }
  p.fs_n = b->fs_n; p.fs_T = b->fs_T;
  for (int k = 0; k < 3; ++k) { p.fs_U[k] = b->fs_U[k]; p.g[k] = b->g[k]; }
  p.depth = b->depth;
  p.cyl = b->cyl; p.cyl_xc = b->cyl_xc; p.cyl_yc = b->cyl_yc; p.cyl_r = b->cyl_r; p.cyl_Tw = b->cyl_Tw;
  p.surf = (unsigned long long*)b->surf;
  p.surf_nbody = b->surf_nbody;
  return p;
}

template <typename S>
PartP<S> make_parts(const usp_particles* q) {
  PartP<S> p;
  p.x = (S*)q->x; p.y = (S*)q->y; p.cx = (S*)q->cx; p.cy = (S*)q->cy; p.cz = (S*)q->cz;
  p.erot = (S*)q->erot; p.vib = q->vib; p.cell = q->cell; p.pid = q->pid; p.count = q->count;
  p.capacity = q->capacity;
  return p;
}
template PartP<float> make_parts<float>(const usp_particles*);
template PartP<double> make_parts<double>(const usp_particles*);

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

WsLayout ws_layout(int64_t M, int64_t capacity, int nfaces) {
  WsLayout L;
  size_t o = 0;
  L.key = o; o = align256(o + sizeof(int32_t) * (size_t)capacity);
  L.perm = o; o = align256(o + sizeof(uint32_t) * (size_t)capacity);
  L.blocksums = o; o = align256(o + sizeof(int64_t) * (size_t)(cdiv(M, 1024) + 1));
  L.t9 = o; o = align256(o + sizeof(int32_t) * 9 * (size_t)M);
  L.cell_i32 = o; o = align256(o + sizeof(int32_t) * 7 * (size_t)M);
  L.old_off = o; o = align256(o + sizeof(int64_t) * (size_t)(M + 1));
  L.far_off = o; o = align256(o + sizeof(int64_t) * (size_t)(M + 1));
  L.far = o; o = align256(o + sizeof(int32_t) * 4 * (size_t)capacity);
  L.face_cnt = o; o = align256(o + sizeof(int32_t) * (size_t)(nfaces + 1));
  L.face_off = o; o = align256(o + sizeof(int64_t) * (size_t)(nfaces + 1));
  L.misc = o; o = align256(o + sizeof(int64_t) * 8);
  L.tiles = o; o = align256(o + sizeof(int32_t) * (size_t)(cdiv(capacity, UPDATE_TILE_MIN) + 2));
  L.chunk_off = o; o = align256(o + sizeof(int64_t) * (size_t)(M + 1));
  L.chunk_part = o; o = align256(o + sizeof(double) * BIG_PARTS * (size_t)chunks_max(capacity, M));
  L.cons_scal = o; o = align256(o + CONS_SCALAR_BYTES * (size_t)M);
  L.total = o;
  return L;
}

}  // namespace usp

using namespace usp;

namespace {

bool grid_ok(const usp_grid* g) {
  if (!g || g->nx <= 0 || g->ny <= 0 || !g->volume) return false;
  if (g->dim < 0 || g->dim > 2) return false;
  if (g->dim == 0 && g->ny != 1) return false;
  if (g->dim == 1 && g->nx != 1) return false;
  if (g->dim >= 1 && !(g->dy > 0.0)) return false;
  if (g->dim == 2 && !(g->dx > 0.0)) return false;
  if (!(g->fnum > 0.0)) return false;
  if ((int64_t)g->nx * g->ny > (int64_t)INT32_MAX) return false;
  return true;
}

bool parts_ok(const usp_particles* p, const usp_grid* g) {
  if (!p || !p->cx || !p->cy || !p->cz || !p->erot || !p->vib || !p->cell || !p->pid || !p->count)
    return false;
  if (p->prec != USP_F32 && p->prec != USP_F64) return false;
  if (p->capacity <= 0 || p->capacity > (int64_t)UINT32_MAX) return false;
  if (g->dim >= 1 && !p->y) return false;
  if (g->dim == 2 && !p->x) return false;
  return true;
}

bool gas_ok(const usp_gas* g) {
  return g && g->m > 0.0 && g->theta_vib > 0.0 && g->T_ref > 0.0 && g->mu_ref > 0.0 &&
         g->alpha_vss > 0.0 && (g->scheme == USP_SCHEME_USP || g->scheme == USP_SCHEME_FPM) &&
         (g->gamma_scope == USP_GAMMA_PARTICLE || g->gamma_scope == USP_GAMMA_CELL) &&
         (g->alpha_sign == USP_ALPHA_SIGN_PR || g->alpha_sign == USP_ALPHA_SIGN_KEEP);
}

// Free-stream faces need a temperature and a depth; the surface element
// count must not be negative.  A null bc passes (callers that require one
// check it themselves).
bool bc_ok(const usp_bc* b, const usp_grid* grid) {
  if (!b) return true;
  if (b->surf_nbody < 0) return false;
  if (grid->dim == 2)
    for (int k = 0; k < 4; ++k)
      if (b->kind[k] == USP_BC_FREESTREAM && !(b->fs_T > 0.0 && b->depth > 0.0)) return false;
  return true;
}

usp_status hip_status(hipError_t e) { return e == hipSuccess ? USP_OK : USP_EDEVICE; }

}  // namespace

// The host-side argument checks of usp_update, less the workspace.
bool usp::update_args_ok(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                         const double* cs, const int64_t* offsets, const usp_particles* p) {
  if (!grid_ok(grid) || !gas_ok(gas) || !parts_ok(p, grid) || !cs || !offsets) return false;
  if (grid->dim >= 1 && (!bc || !(dt > 0.0))) return false;
  return bc_ok(bc, grid);
}

namespace {

template <typename S>
usp_status do_bin(const usp_grid* grid, const usp_particles* in, usp_particles* out,
                  int64_t* offsets, const int64_t* in_offsets, void* ws, int64_t* counters,
                  hipStream_t st) {
  const GridP g = make_grid(grid);
  const WsLayout L = ws_layout(g.M, in->capacity, n_faces(g));
  return hip_status(launch_bin<S>(g, make_parts<S>(in), make_parts<S>(out), offsets, in_offsets,
                                  (char*)ws, L, counters, st));
}

template <typename S>
usp_status do_step(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                   const double* dt_cell, usp_particles* p, usp_particles* p_alt,
                   int64_t* offsets, const int64_t* in_offsets, double* mom, double* cs,
                   void* ws, uint64_t seed, uint64_t step, int32_t nsteps, int64_t* counters,
                   hipStream_t st) {
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  const BcP bp = make_bc(bc);
  // the two buffers swap every step (equal capacities)
  const int64_t cap = p->capacity;
  const WsLayout L = ws_layout(g.M, cap, n_faces(g));
  char* w = (char*)ws;
  // Cells far larger than the fused particle phase's LDS stage (mean slots
  // per cell above it) would give whole cells to single workgroups: such
  // grids run the separate phase kernels, which spread every particle over
  // the chip, after a copying bin, with the moments and the conservation's
  // sums split over chunks of each cell.
  const int stage = sizeof(S) == 4 ? UPDATE_STAGE_F32 : UPDATE_STAGE_F64;
  const bool big_cells = cdiv(cap, g.M) > stage;
  for (int32_t s = 0; s < nsteps; ++s) {
    const uint64_t sn = step + (uint64_t)s;
    if (big_cells) {
      hipError_t e = hipSuccess;
      if (s == 0 || g.dim != 0) {
        const PartP<S> in = make_parts<S>(p), out = make_parts<S>(p_alt);
        if ((e = launch_bin<S>(g, in, out, offsets, s > 0 ? offsets : in_offsets, w, L, counters,
                               st)) != hipSuccess)
          return USP_EDEVICE;
        const usp_particles tmp = *p;
        *p = *p_alt;
        *p_alt = tmp;
      }
      // the per-cell reductions split over chunks of each cell
      const PartP<S> q = make_parts<S>(p);
      if ((e = launch_moments_split<S>(g, q, offsets, mom, w, L, st)) != hipSuccess)
        return USP_EDEVICE;
      if ((e = launch_reconstruct(g, gp, mom, dt, dt_cell, cs, counters, st)) != hipSuccess)
        return USP_EDEVICE;
      if ((e = launch_collide<S>(g, gp, cs, offsets, q, seed, sn, counters, st)) != hipSuccess)
        return USP_EDEVICE;
      if ((e = launch_conserve_split<S>(g, gp, cs, offsets, q, seed, sn, w, L, counters, st)) !=
          hipSuccess)
        return USP_EDEVICE;
      if (g.dim != 0 &&
          (e = launch_advect<S>(g, gp, bp, dt, q, seed, sn, w, L, counters, st)) != hipSuccess)
        return USP_EDEVICE;
      continue;
    }
    // from the second step on, the input is the previous step's binned
    // state (segments in `offsets`) followed by the injected particles; in
    // 0D nothing moves between cells, so only the first step bins
    hipError_t e = hipSuccess;
    if (s == 0 || g.dim != 0) {
      // the bin records the new order without moving the particles; the
      // moments and the particle phase read them through it, and the
      // particle phase writes the whole state in the new order to p_alt
      uint32_t* gperm = (uint32_t*)(w + L.perm);
      const PartP<S> in = make_parts<S>(p), out = make_parts<S>(p_alt);
      if ((e = launch_bin<S>(g, in, out, offsets, s > 0 ? offsets : in_offsets, w, L, counters, st,
                             gperm)) != hipSuccess)
        return USP_EDEVICE;
      if ((e = launch_moments<S>(g, in, offsets, mom, st, gperm)) != hipSuccess) return USP_EDEVICE;
      if ((e = launch_reconstruct(g, gp, mom, dt, dt_cell, cs, counters, st)) != hipSuccess)
        return USP_EDEVICE;
      if ((e = launch_update<S>(g, gp, bp, dt, cs, offsets, out, seed, sn, w, L, counters, st, &in,
                                gperm)) != hipSuccess)
        return USP_EDEVICE;
      const usp_particles tmp = *p;
      *p = *p_alt;
      *p_alt = tmp;
      continue;
    }
    const PartP<S> q = make_parts<S>(p);
    if ((e = launch_moments<S>(g, q, offsets, mom, st)) != hipSuccess) return USP_EDEVICE;
    if ((e = launch_reconstruct(g, gp, mom, dt, dt_cell, cs, counters, st)) != hipSuccess) return USP_EDEVICE;
    if ((e = launch_update<S>(g, gp, bp, dt, cs, offsets, q, seed, sn, w, L, counters, st)) != hipSuccess)
      return USP_EDEVICE;
  }
  return USP_OK;
}

const char* kMomNames[USP_NMOM] = {"N", "UX", "UY", "UZ", "PXX", "PYY", "PZZ", "PXY", "PXZ",
                                   "PYZ", "EROT", "IBAR", "QTRX", "QTRY", "QTRZ", "QROTX",
                                   "QROTY", "QROTZ", "QIX", "QIY", "QIZ"};
const char* kCsNames[USP_NCS] = {
    "NP", "NDENS", "UX", "UY", "UZ", "TTR", "TROT", "TVIB", "PXX", "PYY", "PZZ", "PXY",
    "PXZ", "PYZ", "ETR", "EROT", "EVIB", "MU", "MUP", "TAUC", "ZROT", "ZVIB", "PR", "DT",
    "A", "B", "R2", "R3", "ALPHA", "OMA2", "NU", "EROT_NEW", "EVIB_NEW", "COLLIDE", "NBR_OK",
    "FPM_TAU", "FPM_TTR_REL", "FPM_TROT_REL", "FPM_MREL"};
const char* kCntNames[USP_NCOUNTERS] = {
    "PB_CLAMP", "CHOL_FALLBACK", "NU_ZERO", "TREL_SKIP", "TREL_CLAMP", "VIB_SAT",
    "INTERP_CLAMP", "CONS_SKIP", "PICK_FAIL", "CELL_SKIP", "INJECTED", "DELETED",
    "WALL_HITS", "BOUNCE_LIMIT", "CAPACITY", "SOLID_DROP", "NONFINITE"};

}  // namespace

extern "C" {

const char* usp_status_str(usp_status s) {
  switch (s) {
    case USP_OK: return "ok";
    case USP_EINVAL: return "invalid argument";
    case USP_EDEVICE: return "HIP device error";
    case USP_ECAPACITY: return "particle capacity exceeded (injections dropped)";
    case USP_ENUMERIC: return "NaN or infinite value in the state";
    case USP_ESCRATCH: return "problem too large for the fixed scratch of usp_update_noalloc";
    case USP_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* usp_mom_name(int32_t k) { return (k >= 0 && k < USP_NMOM) ? kMomNames[k] : ""; }
const char* usp_cs_name(int32_t k) { return (k >= 0 && k < USP_NCS) ? kCsNames[k] : ""; }
const char* usp_counter_name(int32_t k) {
  return (k >= 0 && k < USP_NCOUNTERS) ? kCntNames[k] : "";
}
const char* usp_version(void) { return "libusp 0.1 (gfx950)"; }

size_t usp_cellstate_bytes(const usp_grid* grid) {
  if (!grid_ok(grid)) return 0;
  return cellstate_bytes((int64_t)grid->nx * grid->ny);
}

int64_t usp_surf_elements(const usp_grid* grid, const usp_bc* bc) {
  if (!grid_ok(grid) || !bc || bc->surf_nbody < 0) return 0;
  return 2 * (int64_t)grid->nx + 2 * (int64_t)grid->ny + bc->surf_nbody;
}

size_t usp_workspace_bytes(const usp_grid* grid, int64_t capacity) {
  if (!grid_ok(grid) || capacity <= 0) return 0;
  const GridP g = make_grid(grid);
  return ws_layout(g.M, capacity, n_faces(g)).total;
}

usp_status usp_bin(const usp_grid* grid, const usp_particles* in, usp_particles* out,
                   int64_t* offsets, const int64_t* in_offsets, void* ws, size_t ws_bytes,
                   int64_t* counters, void* stream) {
  if (!grid_ok(grid) || !parts_ok(in, grid) || !parts_ok(out, grid) || !offsets || !ws) return USP_EINVAL;
  if (in->prec != out->prec || out->capacity < in->capacity) return USP_EINVAL;
  if (in->cx == out->cx || in->count == out->count) return USP_EINVAL;
  if (ws_bytes < usp_workspace_bytes(grid, in->capacity)) return USP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  return in->prec == USP_F32 ? do_bin<float>(grid, in, out, offsets, in_offsets, ws, counters, st)
                             : do_bin<double>(grid, in, out, offsets, in_offsets, ws, counters, st);
}

usp_status usp_bin_gather(const usp_grid* grid, const usp_particles* in, usp_particles* out,
                          int64_t* offsets, const int64_t* in_offsets, uint32_t* perm, void* ws,
                          size_t ws_bytes, int64_t* counters, void* stream) {
  if (!grid_ok(grid) || !parts_ok(in, grid) || !parts_ok(out, grid) || !offsets || !ws || !perm)
    return USP_EINVAL;
  if (in->prec != out->prec || out->capacity < in->capacity) return USP_EINVAL;
  if (in->cx == out->cx || in->count == out->count) return USP_EINVAL;
  const int64_t cap = out->capacity;
  if (ws_bytes < usp_workspace_bytes(grid, cap)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const WsLayout L = ws_layout(g.M, cap, n_faces(g));
  hipStream_t st = (hipStream_t)stream;
  return hip_status(in->prec == USP_F32
      ? launch_bin<float>(g, make_parts<float>(in), make_parts<float>(out), offsets, in_offsets,
                          (char*)ws, L, counters, st, perm)
      : launch_bin<double>(g, make_parts<double>(in), make_parts<double>(out), offsets, in_offsets,
                           (char*)ws, L, counters, st, perm));
}

usp_status usp_moments_gather(const usp_grid* grid, const usp_particles* in, const uint32_t* perm,
                              const int64_t* offsets, double* mom, void* stream) {
  if (!grid_ok(grid) || !parts_ok(in, grid) || !perm || !offsets || !mom) return USP_EINVAL;
  const GridP g = make_grid(grid);
  hipStream_t st = (hipStream_t)stream;
  return hip_status(in->prec == USP_F32
      ? launch_moments<float>(g, make_parts<float>(in), offsets, mom, st, perm)
      : launch_moments<double>(g, make_parts<double>(in), offsets, mom, st, perm));
}

usp_status usp_update_gather(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                             const double* cs, const int64_t* offsets, const usp_particles* in,
                             const uint32_t* perm, usp_particles* out, void* ws, size_t ws_bytes,
                             uint64_t seed, uint64_t step, int64_t* counters, void* ev_begin,
                             void* ev_end, void* stream) {
  if (!grid_ok(grid) || !gas_ok(gas) || !parts_ok(in, grid) || !parts_ok(out, grid) || !cs ||
      !offsets || !ws || !perm)
    return USP_EINVAL;
  if (in->prec != out->prec || in->cx == out->cx || out->capacity < in->capacity) return USP_EINVAL;
  if (grid->dim >= 1 && (!bc || !(dt > 0.0))) return USP_EINVAL;
  if (!bc_ok(bc, grid)) return USP_EINVAL;
  if (ws_bytes < usp_workspace_bytes(grid, out->capacity)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  const BcP bp = make_bc(bc);
  const WsLayout L = ws_layout(g.M, out->capacity, n_faces(g));
  hipStream_t st = (hipStream_t)stream;
  if (in->prec == USP_F32) {
    const PartP<float> src = make_parts<float>(in);
    return hip_status(launch_update<float>(g, gp, bp, dt, cs, offsets, make_parts<float>(out), seed,
                                           step, (char*)ws, L, counters, st, &src, perm,
                                           (hipEvent_t)ev_begin, (hipEvent_t)ev_end));
  }
  const PartP<double> src = make_parts<double>(in);
  return hip_status(launch_update<double>(g, gp, bp, dt, cs, offsets, make_parts<double>(out), seed,
                                          step, (char*)ws, L, counters, st, &src, perm,
                                          (hipEvent_t)ev_begin, (hipEvent_t)ev_end));
}

usp_status usp_moments(const usp_grid* grid, const usp_particles* p, const int64_t* offsets,
                       double* mom, void* stream) {
  if (!grid_ok(grid) || !parts_ok(p, grid) || !offsets || !mom) return USP_EINVAL;
  const GridP g = make_grid(grid);
  hipStream_t st = (hipStream_t)stream;
  return hip_status(p->prec == USP_F32 ? launch_moments<float>(g, make_parts<float>(p), offsets, mom, st)
                                       : launch_moments<double>(g, make_parts<double>(p), offsets, mom, st));
}

usp_status usp_sample_fields(const usp_grid* grid, const double* mom, double* acc,
                             void* stream) {
  if (!grid_ok(grid) || !mom || !acc) return USP_EINVAL;
  return hip_status(launch_sample_fields(make_grid(grid), mom, acc, (hipStream_t)stream));
}

usp_status usp_reconstruct(const usp_grid* grid, const usp_gas* gas, const double* mom,
                           double dt, const double* dt_cell, double* cs, int64_t* counters,
                           void* stream) {
  if (!grid_ok(grid) || !gas_ok(gas) || !mom || !cs) return USP_EINVAL;
  if (!dt_cell && !(dt > 0.0)) return USP_EINVAL;
  return hip_status(launch_reconstruct(make_grid(grid), make_gas(gas), mom, dt, dt_cell, cs,
                                       counters, (hipStream_t)stream));
}

usp_status usp_collide(const usp_grid* grid, const usp_gas* gas, const double* cs,
                       const int64_t* offsets, usp_particles* p, uint64_t seed, uint64_t step,
                       int64_t* counters, void* stream) {
  if (!grid_ok(grid) || !gas_ok(gas) || !cs || !offsets || !parts_ok(p, grid)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  hipStream_t st = (hipStream_t)stream;
  return hip_status(p->prec == USP_F32
                        ? launch_collide<float>(g, gp, cs, offsets, make_parts<float>(p), seed, step, counters, st)
                        : launch_collide<double>(g, gp, cs, offsets, make_parts<double>(p), seed, step, counters, st));
}

usp_status usp_conserve(const usp_grid* grid, const usp_gas* gas, const double* cs,
                        const int64_t* offsets, usp_particles* p, uint64_t seed, uint64_t step,
                        int64_t* counters, void* stream) {
  if (!grid_ok(grid) || !gas_ok(gas) || !cs || !offsets || !parts_ok(p, grid)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  hipStream_t st = (hipStream_t)stream;
  return hip_status(p->prec == USP_F32
                        ? launch_conserve<float>(g, gp, cs, offsets, make_parts<float>(p), seed, step, counters, st)
                        : launch_conserve<double>(g, gp, cs, offsets, make_parts<double>(p), seed, step, counters, st));
}

usp_status usp_advect(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                      usp_particles* p, uint64_t seed, uint64_t step, void* ws, size_t ws_bytes,
                      int64_t* counters, void* stream) {
  if (!grid_ok(grid) || !gas_ok(gas) || !bc || !parts_ok(p, grid) || !ws) return USP_EINVAL;
  if (!(dt > 0.0) || !bc_ok(bc, grid)) return USP_EINVAL;
  if (ws_bytes < usp_workspace_bytes(grid, p->capacity)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  const BcP bp = make_bc(bc);
  const WsLayout L = ws_layout(g.M, p->capacity, n_faces(g));
  hipStream_t st = (hipStream_t)stream;
  return hip_status(p->prec == USP_F32
                        ? launch_advect<float>(g, gp, bp, dt, make_parts<float>(p), seed, step, (char*)ws, L, counters, st)
                        : launch_advect<double>(g, gp, bp, dt, make_parts<double>(p), seed, step, (char*)ws, L, counters, st));
}

usp_status usp_update(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                      const double* cs, const int64_t* offsets, usp_particles* p, void* ws,
                      size_t ws_bytes, uint64_t seed, uint64_t step, int64_t* counters,
                      void* stream) {
  if (!update_args_ok(grid, gas, bc, dt, cs, offsets, p) || !ws) return USP_EINVAL;
  if (ws_bytes < usp_workspace_bytes(grid, p->capacity)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  const BcP bp = make_bc(bc);
  const WsLayout L = ws_layout(g.M, p->capacity, n_faces(g));
  hipStream_t st = (hipStream_t)stream;
  return hip_status(p->prec == USP_F32
                        ? launch_update<float>(g, gp, bp, dt, cs, offsets, make_parts<float>(p), seed, step, (char*)ws, L, counters, st)
                        : launch_update<double>(g, gp, bp, dt, cs, offsets, make_parts<double>(p), seed, step, (char*)ws, L, counters, st));
}

usp_status usp_batch(const usp_grid* grid, const usp_gas* gas, double dt, const double* dt_cell,
                     usp_particles* p, const int64_t* offsets, double* mom, double* cs, void* ws,
                     size_t ws_bytes, int32_t tile, int32_t steps_per_launch, uint64_t seed,
                     uint64_t step, int32_t nsteps, int64_t* counters, void* stream) {
  if (!grid_ok(grid) || grid->dim != 0 || !gas_ok(gas) || !parts_ok(p, grid)) return USP_EINVAL;
  if (!offsets || !mom || !cs || !ws || nsteps < 0 || steps_per_launch < 0) return USP_EINVAL;
  if (!dt_cell && !(dt > 0.0)) return USP_EINVAL;
  if (tile != 0 && tile != 512 && tile != 1024 && tile != 2048) return USP_EINVAL;
  if (p->prec == USP_F64 && tile != 0 && tile != 512) return USP_EINVAL;
  if (ws_bytes < usp_workspace_bytes(grid, p->capacity)) return USP_EINVAL;
  const GridP g = make_grid(grid);
  const GasP gp = make_gas(gas);
  const WsLayout L = ws_layout(g.M, p->capacity, n_faces(g));
  hipStream_t st = (hipStream_t)stream;
  return hip_status(p->prec == USP_F32
                        ? launch_batch<float>(g, gp, dt, dt_cell, mom, cs, offsets, make_parts<float>(p), tile, steps_per_launch, seed, step, nsteps, (char*)ws, L, counters, st)
                        : launch_batch<double>(g, gp, dt, dt_cell, mom, cs, offsets, make_parts<double>(p), tile, steps_per_launch, seed, step, nsteps, (char*)ws, L, counters, st));
}

usp_status usp_step(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                    const double* dt_cell, usp_particles* p, usp_particles* p_alt,
                    int64_t* offsets, const int64_t* in_offsets, double* mom, double* cs,
                    void* ws, size_t ws_bytes, uint64_t seed, uint64_t step, int32_t nsteps,
                    int64_t* counters, void* stream) {
  if (!grid_ok(grid) || !gas_ok(gas) || !parts_ok(p, grid) || !parts_ok(p_alt, grid)) return USP_EINVAL;
  if (!offsets || !mom || !cs || !ws || nsteps < 0) return USP_EINVAL;
  // the state moves between the two buffers every step, so both must hold
  // the same number of slots (the bin copies up to the input's capacity)
  if (p->prec != p_alt->prec || p_alt->capacity != p->capacity || p->cx == p_alt->cx ||
      p->count == p_alt->count)
    return USP_EINVAL;
  if (grid->dim >= 1 && (!bc || !(dt > 0.0))) return USP_EINVAL;
  if (!bc_ok(bc, grid)) return USP_EINVAL;
  if (!dt_cell && !(dt > 0.0)) return USP_EINVAL;
  if (ws_bytes < usp_workspace_bytes(grid, p_alt->capacity)) return USP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  return p->prec == USP_F32
             ? do_step<float>(grid, gas, bc, dt, dt_cell, p, p_alt, offsets, in_offsets, mom, cs, ws, seed, step, nsteps, counters, st)
             : do_step<double>(grid, gas, bc, dt, dt_cell, p, p_alt, offsets, in_offsets, mom, cs, ws, seed, step, nsteps, counters, st);
}

usp_status usp_check(const usp_grid* grid, const usp_particles* p, const double* mom,
                     const double* cs, int64_t* counters, int64_t* nonfinite, void* stream) {
  if (!grid_ok(grid) || !parts_ok(p, grid) || !counters) return USP_EINVAL;
  const GridP g = make_grid(grid);
  hipStream_t st = (hipStream_t)stream;
  int64_t* found = counters + USP_CNT_NONFINITE;
  int64_t before[USP_NCOUNTERS];
  if (hipMemcpyAsync(before, counters, sizeof(before), hipMemcpyDeviceToHost, st) != hipSuccess)
    return USP_EDEVICE;
  const hipError_t e = p->prec == USP_F32
      ? launch_check<float>(g, make_parts<float>(p), mom, cs, found, st)
      : launch_check<double>(g, make_parts<double>(p), mom, cs, found, st);
  if (e != hipSuccess) return USP_EDEVICE;
  int64_t after[USP_NCOUNTERS];
  if (hipMemcpyAsync(after, counters, sizeof(after), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return USP_EDEVICE;
  if (nonfinite) *nonfinite = after[USP_CNT_NONFINITE] - before[USP_CNT_NONFINITE];
  if (after[USP_CNT_NONFINITE] > 0) return USP_ENUMERIC;
  if (after[USP_CNT_CAPACITY] > 0) return USP_ECAPACITY;
  return USP_OK;
}

}  // extern "C"
