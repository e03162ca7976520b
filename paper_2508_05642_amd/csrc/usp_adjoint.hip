// usp_adjoint.hip -- pathwise adjoint of the 1D step (FP64 state, USP-FPM
// scheme) with respect to the collision-model parameters (Z_rot, omega,
// mu_ref), for time-averaged outputs: the mass flow (sum of c_x at the
// start of every step) and the wall shear (c_x given to the walls).
//
// The derivative is taken along the path of the run with every discrete
// outcome held fixed: cells and bin order, vibrational levels after the
// jumps (Sec. III.A.2) and the picks (Sec. IV.C), the stencil and the 5%
// temperature floor of the reconstruction (Sec. III.B), the Cholesky test
// (a particle whose test fails keeps its post-collision state as a
// constant, Sec. III.A.3), the clamp of T_rot^rel, the skips of the
// conservation scalings, and every boundary event of the flight (a particle
// whose flight meets a boundary keeps its post-flight state as a
// constant).  The random normals are the run's own draws.
//
// Forward: usp_step_taped runs one step with the separate phase kernels
// (same bits as usp_step) and keeps a tape: the bin permutation, the binned
// pre-collision state, the cell state, and the states after the collision
// and after the conservation.  Reverse (usp_adjoint_step), per step:
//   K1  wave per cell: flight and conservation reversed;
//   K2  thread per particle: the particle update reversed (the scalar chain
//       of the relaxation temperatures through Dual<6> Jacobians), giving
//       adjoints of the particle and of the fields of its stencil cells;
//   K3  a wave per (objective, field, cell) sums the stencil contributions
//       in a fixed order; then a thread per cell reverses the cell state
//       (Dual<6> Jacobian of its coefficients), giving adjoints of the
//       moments and per-cell parameter partials;
//   K4  thread per particle: moments reversed, mass-flow source, and the
//       bin permutation undone;
//   K5  one workgroup: parameter partials summed in a fixed order.
// No floating-point atomics: the result is deterministic.
#include "usp_dual.h"
#include "usp_particle.h"

namespace usp {

// ---- tape and scratch layouts ---------------------------------------------
struct TapeLayout {
  size_t perm, y, cx, cy, cz, erot, vib, cell, pid, ccx, ccy, ccz, cerot, kcx, kcy, kcz, kerot,
      kvib, fcy, offsets, cs, total;
};

static size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

static TapeLayout tape_layout(int64_t M, int64_t cap) {
  TapeLayout t;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o = al256(o + bytes); return r; };
  const size_t d = (size_t)cap * 8;
  t.perm = take((size_t)cap * 4);
  t.y = take(d); t.cx = take(d); t.cy = take(d); t.cz = take(d); t.erot = take(d);
  t.vib = take((size_t)cap); t.cell = take((size_t)cap * 4); t.pid = take((size_t)cap * 4);
  t.ccx = take(d); t.ccy = take(d); t.ccz = take(d); t.cerot = take(d);
  t.kcx = take(d); t.kcy = take(d); t.kcz = take(d); t.kerot = take(d); t.kvib = take((size_t)cap);
  t.fcy = take(d);
  t.offsets = take((size_t)(M + 1) * 8);
  t.cs = take(cellstate_bytes(M));
  t.total = o;
  return t;
}

// cell-field adjoint slots: U(3), Pi(6), T_tr, T_rot, T_vib (the twelve a
// neighbour also reads), then a, b, alpha, 1-alpha^2, nu of the own cell
enum { CF_U = 0, CF_P = 3, CF_T = 9, CF_A = 12, CF_B = 13, CF_AL = 14, CF_OMA2 = 15, CF_NU = 16,
       NOWN = 17, NNBR = 12 };
// conservation's cell adjoints: U^n(3), the rotational target, E0
enum { CC_U = 0, CC_EROT_NEW = 3, CC_E0 = 4, NCONS = 5 };
// moment adjoints: U(3), Pi(6), e_rot
enum { AM_U = 0, AM_P = 3, AM_EROT = 9, NAMOM = 10 };
// particle adjoint fields (lam arrays [2][5][cap]): y, cx, cy, cz, erot
enum { LY = 0, LCX = 1, LE = 4, NLAM = 5 };
constexpr int NOBJ = 2, NPAR = 3;

struct AdjWsLayout {
  size_t lam1, own, nbr, nbrc, cons, csum, lmom, gcell, map, total;
};

static AdjWsLayout adj_ws_layout(int64_t M, int64_t cap) {
  AdjWsLayout w;
  size_t o = 0;
  auto take = [&](size_t bytes) { const size_t r = o; o = al256(o + bytes); return r; };
  w.lam1 = take((size_t)NOBJ * NLAM * cap * 8);
  w.own = take((size_t)NOBJ * NOWN * cap * 8);
  w.nbr = take((size_t)NOBJ * NNBR * cap * 8);
  w.nbrc = take((size_t)cap * 4);
  w.cons = take((size_t)NOBJ * NCONS * M * 8);
  w.csum = take((size_t)NOBJ * NOWN * M * 8);
  w.lmom = take((size_t)NOBJ * NAMOM * M * 8);
  w.gcell = take((size_t)NOBJ * NPAR * M * 8);
  w.map = take((size_t)cap * 4);
  w.total = o;
  return w;
}

struct TapeP {
  const int32_t* perm;
  const double *y, *cx, *cy, *cz, *erot;
  const uint8_t* vib;
  const int32_t* cell;
  const uint32_t* pid;
  const double *ccx, *ccy, *ccz, *cerot;
  const double *kcx, *kcy, *kcz, *kerot;
  const uint8_t* kvib;
  const double* fcy;  // y velocity after the flight
  const int64_t* offsets;
  const double* cs;
};

static TapeP tape_ptrs(const char* base, const TapeLayout& t) {
  TapeP p;
  p.perm = (const int32_t*)(base + t.perm);
  p.y = (const double*)(base + t.y); p.cx = (const double*)(base + t.cx);
  p.cy = (const double*)(base + t.cy); p.cz = (const double*)(base + t.cz);
  p.erot = (const double*)(base + t.erot); p.vib = (const uint8_t*)(base + t.vib);
  p.cell = (const int32_t*)(base + t.cell); p.pid = (const uint32_t*)(base + t.pid);
  p.ccx = (const double*)(base + t.ccx); p.ccy = (const double*)(base + t.ccy);
  p.ccz = (const double*)(base + t.ccz); p.cerot = (const double*)(base + t.cerot);
  p.kcx = (const double*)(base + t.kcx); p.kcy = (const double*)(base + t.kcy);
  p.kcz = (const double*)(base + t.kcz); p.kerot = (const double*)(base + t.kerot);
  p.kvib = (const uint8_t*)(base + t.kvib);
  p.fcy = (const double*)(base + t.fcy);
  p.offsets = (const int64_t*)(base + t.offsets);
  p.cs = (const double*)(base + t.cs);
  return p;
}

// the tape's binned state as a particle view (read only)
__device__ __forceinline__ PartP<double> tape_parts(const TapeP& t, int64_t cap) {
  PartP<double> p;
  p.x = nullptr;
  p.y = const_cast<double*>(t.y);
  p.cx = const_cast<double*>(t.cx); p.cy = const_cast<double*>(t.cy);
  p.cz = const_cast<double*>(t.cz); p.erot = const_cast<double*>(t.erot);
  p.vib = const_cast<uint8_t*>(t.vib); p.cell = const_cast<int32_t*>(t.cell);
  p.pid = const_cast<uint32_t*>(t.pid);
  p.count = nullptr;
  p.capacity = cap;
  return p;
}

// ---- forward with tape ------------------------------------------------------
__global__ void k_pid_map(const uint32_t* __restrict__ pid, const int64_t* __restrict__ count,
                          int64_t cap, int32_t* __restrict__ map) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count[0]) return;
  const uint32_t q = pid[i];
  if ((int64_t)q < cap) map[q] = (int32_t)i;
}

__global__ void k_perm(const uint32_t* __restrict__ pid, const int64_t* __restrict__ count,
                       int64_t cap, const int32_t* __restrict__ map, int32_t* __restrict__ perm) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= count[0]) return;
  const uint32_t q = pid[j];
  perm[j] = (int64_t)q < cap ? map[q] : -1;
}

// device-to-device copy on the stream; the first failure is kept in *e
static void copy_d(void* dst, const void* src, size_t bytes, hipStream_t st, hipError_t* e) {
  const hipError_t r = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, st);
  if (*e == hipSuccess) *e = r;
}

// Several device-to-device copies in one launch (the tape copies of a
// phase): blockIdx.y picks the copy; 8-byte words where both ends allow it,
// bytes otherwise.
constexpr int COPY_MAX = 8;
struct CopyList {
  void* dst[COPY_MAX];
  const void* src[COPY_MAX];
  size_t bytes[COPY_MAX];
  int n;
};

__global__ __launch_bounds__(256) void k_copy_many(CopyList L) {
  const int k = blockIdx.y;
  if (k >= L.n) return;
  const size_t n = L.bytes[k];
  const size_t t0 = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  const uintptr_t a = (uintptr_t)L.dst[k] | (uintptr_t)L.src[k];
  if ((a & 7) == 0) {
    uint64_t* d = (uint64_t*)L.dst[k];
    const uint64_t* s = (const uint64_t*)L.src[k];
    const size_t w = n / 8;
    for (size_t i = t0; i < w; i += stride) d[i] = s[i];
    uint8_t* db = (uint8_t*)L.dst[k];
    const uint8_t* sb = (const uint8_t*)L.src[k];
    for (size_t i = w * 8 + t0; i < n; i += stride) db[i] = sb[i];
  } else {
    uint8_t* d = (uint8_t*)L.dst[k];
    const uint8_t* s = (const uint8_t*)L.src[k];
    for (size_t i = t0; i < n; i += stride) d[i] = s[i];
  }
}

struct CopyBatch {
  CopyList L{};
  void add(void* dst, const void* src, size_t bytes) {
    L.dst[L.n] = dst; L.src[L.n] = src; L.bytes[L.n] = bytes; ++L.n;
  }
  void launch(hipStream_t st, hipError_t* e) {
    if (L.n == 0) return;
    size_t mx = 0;
    for (int k = 0; k < L.n; ++k) mx = L.bytes[k] > mx ? L.bytes[k] : mx;
    const size_t blocks = (mx / 8 + 255) / 256;
    const unsigned gx = (unsigned)(blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks));
    k_copy_many<<<dim3(gx, (unsigned)L.n), 256, 0, st>>>(L);
    const hipError_t r = hipGetLastError();
    if (*e == hipSuccess) *e = r;
    L.n = 0;
  }
};

// One full step of a 1D FP64 state through the separate phase kernels (the
// bits of usp_step), keeping the tape.
static hipError_t step_taped(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                             const PartP<double>& in, const PartP<double>& out, int64_t* offsets,
                             const int64_t* in_offsets, double* mom, double* cs, char* ws,
                             const WsLayout& L, uint64_t seed,
                             uint64_t step, char* tape, const TapeLayout& T, int32_t* map,
                             int64_t* counters, hipStream_t st) {
  const int64_t cap = out.capacity;
  const int grid_p = (int)cdiv(cap, 256);
  k_pid_map<<<grid_p, 256, 0, st>>>(in.pid, in.count, cap, map);
  hipError_t e = launch_bin<double>(g, in, out, offsets, in_offsets, ws, L, counters, st);
  if (e != hipSuccess) return e;
  k_perm<<<grid_p, 256, 0, st>>>(out.pid, out.count, cap, map, (int32_t*)(tape + T.perm));
  hipError_t ce = hipSuccess;
  const size_t d = (size_t)cap * 8;
  CopyBatch cb;
  cb.add(tape + T.y, out.y, d);
  cb.add(tape + T.cx, out.cx, d);
  cb.add(tape + T.cy, out.cy, d);
  cb.add(tape + T.cz, out.cz, d);
  cb.add(tape + T.erot, out.erot, d);
  cb.add(tape + T.vib, out.vib, (size_t)cap);
  cb.add(tape + T.cell, out.cell, (size_t)cap * 4);
  cb.add(tape + T.pid, out.pid, (size_t)cap * 4);
  cb.launch(st, &ce);
  if ((e = launch_moments<double>(g, out, offsets, mom, st)) != hipSuccess) return e;
  if ((e = launch_reconstruct(g, gas, mom, dt, nullptr, cs, counters, st)) != hipSuccess) return e;
  cb.add(tape + T.offsets, offsets, (size_t)(g.M + 1) * 8);
  cb.add(tape + T.cs, cs, cellstate_bytes(g.M));
  cb.launch(st, &ce);
  if ((e = launch_collide<double>(g, gas, cs, offsets, out, seed, step, counters, st)) != hipSuccess)
    return e;
  cb.add(tape + T.ccx, out.cx, d);
  cb.add(tape + T.ccy, out.cy, d);
  cb.add(tape + T.ccz, out.cz, d);
  cb.add(tape + T.cerot, out.erot, d);
  cb.launch(st, &ce);
  if ((e = launch_conserve<double>(g, gas, cs, offsets, out, seed, step, counters, st)) != hipSuccess)
    return e;
  cb.add(tape + T.kcx, out.cx, d);
  cb.add(tape + T.kcy, out.cy, d);
  cb.add(tape + T.kcz, out.cz, d);
  cb.add(tape + T.kerot, out.erot, d);
  cb.add(tape + T.kvib, out.vib, (size_t)cap);
  cb.launch(st, &ce);
  if (ce != hipSuccess) return ce;
  if ((e = launch_advect<double>(g, gas, bc, dt, out, seed, step, ws, L, counters, st)) != hipSuccess)
    return e;
  // the y velocity after the flight, for the hit-time derivative of the
  // particles that met a wall (1D: no particle is created or removed)
  copy_d(tape + T.fcy, out.cy, d, st, &ce);
  return ce;
}

// ---- shared pieces of the reverse -------------------------------------------
// Does the flight of a particle at y with post-kick velocity cy meet a
// boundary within dt (the first test of the free flight, 1D)?
__device__ __forceinline__ bool flight_event_1d(const GridP& g, double y, double cy, double dt) {
  const double ylo = (double)(double)g.y0, yhi = (double)edge<double>(g.y0, g.dy, g.ny);
  return (cy < 0.0 && y + cy * dt < ylo) || (cy > 0.0 && y + cy * dt >= yhi);
}

// T-check with the gradient of the root: the value is the FP64 solve; the
// derivative is that of one Newton step taken at the root (implicit
// function theorem).
template <int N>
__device__ __forceinline__ Dual<N> tcheck_dual(double th, const Dual<N>& Ttr, const Dual<N>& Trot,
                                               const Dual<N>& Tvib, const Dual<N>& a,
                                               const Dual<N>& b) {
  const double t = tcheck<double>(th, Ttr.v, Trot.v, Tvib.v, a.v, b.v);
  if (!(t > 0.0)) return Dual<N>(0.0);
  const Dual<N> ca = 1.5 + a;
  const Dual<N> rhs = 1.5 * Ttr + a * Trot + b * th * mlevel<Dual<N>>(Dual<N>(th), Tvib);
  const double x = th / t;
  const double m = x > 700.0 ? 0.0 : 1.0 / expm1(x);
  const double cv = x * x * m * (1.0 + m);
  const Dual<N> f = ca * t + b * (th * m) - rhs;
  const Dual<N> fp = ca + b * cv;
  Dual<N> r = Dual<N>(t) - f / fp;
  r.v = t;
  return r;
}

// (T_tr^rel, T_rot^rel) of a particle (Sec. III.A.1, eqs. T_tr_USP,
// T_rot_USP) as functions of (T_tr, T_rot, T_vib, a, b, 1 - alpha^2).
__device__ __forceinline__ void trel_dual(double th, double Ttr, double Trot, double Tvib, double a,
                                          double b, double oma2, Dual<6>* Ttr_rel,
                                          Dual<6>* Trot_rel) {
  using D6 = Dual<6>;
  const D6 tt = D6::var(Ttr, 0), tr = D6::var(Trot, 1), tv = D6::var(Tvib, 2);
  const D6 aa = D6::var(a, 3), bb = D6::var(b, 4), om = D6::var(oma2, 5);
  const D6 Tc = tcheck_dual<6>(th, tt, tr, tv, aa, bb);
  const D6 cb = cbar_R<D6>(D6(th), Tc, tv);
  const D6 D = 1.5 + aa + bb * cb;
  const D6 g1 = 3.0 * aa / D, g2 = 3.0 * bb * cb / D, g3 = 2.0 * aa * bb * cb / D;
  const D6 Xtr = g1 * (tt - tr) + g2 * (tt - tv);
  const D6 Xrot = g1 * (tt - tr) - g3 * (tr - tv);
  *Ttr_rel = tt - Xtr / (1.5 * om);
  *Trot_rel = tr + Xrot / om;
}

// templated Eucken Prandtl number (the forward's prandtl())
template <typename T>
__device__ __forceinline__ T prandtl_t(const GasP& g, T Ttr) {
  if (g.pr_model == USP_PR_CONST) return T(g.Pr_const);
  T xi = T(0.0);
  if (Ttr > T(0.0)) {
    const T x = g.theta / Ttr;
    xi = x > T(700.0) ? T(0.0) : x / expm1(x);
    if (g.pr_model == USP_PR_EUCKEN_STANDARD) xi = 2.0 * xi;
  }
  return (14.0 + 2.0 * xi) / (19.0 + 2.0 * xi);
}

// The cell coefficients the particle update and conservation read (the
// forward's cell_state, USP-FPM branch, constant collision numbers) as
// functions of (T_tr, T_rot, T_vib, Z_rot, omega, mu_ref):
// out = a, b, alpha, 1 - alpha^2, nu, e_rot target.
__device__ __forceinline__ void cell_coef_dual(const GasP& gas, double alpha_vss, double nd,
                                               double dtc, double Ttr, double Trot, double Tvib,
                                               Dual<6> out[6]) {
  using D6 = Dual<6>;
  const double R = gas.R, Th = gas.theta;
  const D6 tt = D6::var(Ttr, 0), tr = D6::var(Trot, 1), tv = D6::var(Tvib, 2);
  const D6 zr = D6::var(gas.Z_rot, 3), om = D6::var(gas.omega, 4), mr = D6::var(gas.mu_ref, 5);
  const D6 K = alpha_vss * (5.0 - 2.0 * om) * (7.0 - 2.0 * om) /
               (5.0 * (alpha_vss + 1.0) * (alpha_vss + 2.0));
  const D6 mu = mr * pow(tt / gas.T_ref, om);
  const D6 mup = mu / (nd * KB * tt);
  const D6 tauc = K * mup;
  const D6 Pr = prandtl_t<D6>(gas, tt);
  const D6 A = 2.0 * mup;
  const D6 r3 = (A - Pr * dtc) / (A + Pr * dtc);
  const D6 r2 = (A - dtc) / (A + dtc);
  const D6 al = cbrt(r3);
  const D6 oma2 = (2.0 * Pr * dtc / (A + Pr * dtc)) * (1.0 + al) / (1.0 + al + al * al);
  const D6 nu = (r2 - al * al) / oma2;
  const D6 a = dtc / (dtc + 2.0 * zr * tauc);
  const D6 b = dtc / (dtc + 2.0 * gas.Z_vib * tauc);
  const D6 Tc = tcheck_dual<6>(Th, tt, tr, tv, a, b);
  const D6 cb = cbar_R<D6>(D6(Th), Tc, tv);
  const D6 D = 1.5 + a + b * cb;
  const D6 g1 = 3.0 * a / D, g3 = 2.0 * a * b * cb / D;
  out[0] = a; out[1] = b; out[2] = al; out[3] = oma2; out[4] = nu;
  out[5] = R * tr + R * (g1 * (tt - tr) - g3 * (tr - tv));
}

// reverse of the 3x3 Cholesky factor L = chol(S) (both packed as in chol3m)
__device__ __forceinline__ void chol3_reverse(const double L[6], const double lL[6], double lS[6]) {
  const double l11 = L[0], l21 = L[1], l22 = L[2], l31 = L[3], l32 = L[4], l33 = L[5];
  const double ld3 = lL[5] / (2.0 * l33);
  const double l32t = lL[4] - 2.0 * l32 * ld3;
  lS[2] = ld3;
  lS[5] = l32t / l22;
  const double l31t = lL[3] - 2.0 * l31 * ld3 - l21 * l32t / l22;
  const double l22t = lL[2] - l32 * l32t / l22;
  const double ld2 = l22t / (2.0 * l22);
  lS[1] = ld2;
  const double l21t = lL[1] - 2.0 * l21 * ld2 - l31 * l32t / l22;
  lS[3] = l21t / l11;
  lS[4] = l31t / l11;
  const double l11t = lL[0] - (l21 * l21t + l31 * l31t) / l11;
  lS[0] = l11t / (2.0 * l11);
}

__device__ __forceinline__ double& lam_at(double* lam, int o, int f, int64_t cap, int64_t i) {
  return lam[((int64_t)o * NLAM + f) * cap + i];
}

// ---- K1: flight and conservation reversed, wave per cell ----------------------
__global__ __launch_bounds__(256) void k_adj_flight_conserve(GridP g, GasP gas, BcP bc, double dt,
                                                             TapeP T, int64_t cap,
                                                             const double* __restrict__ lam_in,
                                                             double* __restrict__ lam1,
                                                             double* __restrict__ cons,
                                                             double w_tau) {
  const int lane = threadIdx.x & 63;
  const int64_t c = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t M = g.M;
  if (c >= M) return;
  const int64_t o0 = T.offsets[c], o1 = T.offsets[c + 1], N = o1 - o0;
  for (int o = 0; o < NOBJ; ++o)
    if (lane < NCONS) cons[((int64_t)o * NCONS + lane) * M + c] = 0.0;
  if (N == 0) return;
  const double* cs = T.cs;
  const bool coll = cs[CS_COLLIDE * M + c] != 0.0;
  // adjoint of the post-conservation state (o, component) of particle i.
  // A particle whose flight meets a wall leaves with the re-emitted
  // velocity, energy and level (constants of the path); its position after
  // the flight is y_wall,last + c_y,f (dt - t_between - t_1), with t_1 =
  // (y_wall,1 - y)/c_y the first hit time, c_y the velocity after the kick
  // and c_y,f the final one: d y_f/d y = c_y,f/c_y, d y_f/d c_y = c_y,f
  // t_1/c_y.
  const double ylo = (double)g.y0, yhi = (double)edge<double>(g.y0, g.dy, g.ny);
  auto post = [&](int64_t i, int o, double lc[3], double* le, double* ly) {
    const double ck[3] = {T.kcx[i] + bc.g[0] * dt, T.kcy[i] + bc.g[1] * dt, T.kcz[i] + bc.g[2] * dt};
    if (flight_event_1d(g, T.y[i], ck[1], dt)) {
      const double lyf = lam_at(const_cast<double*>(lam_in), o, LY, cap, i);
      const double r = T.fcy[i] / ck[1];
      const double t1 = ((ck[1] < 0.0 ? ylo : yhi) - T.y[i]) / ck[1];
      lc[0] = o == 1 ? w_tau : 0.0; lc[1] = lyf * r * t1; lc[2] = 0.0; *le = 0.0; *ly = lyf * r;
      return;
    }
    const double lyv = lam_at(const_cast<double*>(lam_in), o, LY, cap, i);
    lc[0] = lam_at(const_cast<double*>(lam_in), o, LCX, cap, i);
    lc[1] = lam_at(const_cast<double*>(lam_in), o, LCX + 1, cap, i) + dt * lyv;
    lc[2] = lam_at(const_cast<double*>(lam_in), o, LCX + 2, cap, i);
    *le = lam_at(const_cast<double*>(lam_in), o, LE, cap, i);
    *ly = lyv;
  };
  if (!coll) {
    for (int64_t i = o0 + lane; i < o1; i += 64)
      for (int o = 0; o < NOBJ; ++o) {
        double lc[3], le, ly;
        post(i, o, lc, &le, &ly);
        for (int k = 0; k < 3; ++k) lam_at(lam1, o, LCX + k, cap, i) = lc[k];
        lam_at(lam1, o, LE, cap, i) = le;
        lam_at(lam1, o, LY, cap, i) = ly;
      }
    return;
  }
  // forward scalars of the conservation (the forward's own sums)
  const double Un[3] = {cs[CS_UX * M + c], cs[CS_UY * M + c], cs[CS_UZ * M + c]};
  double s[5] = {0, 0, 0, 0, 0};
  double SIp = 0.0;
  for (int64_t i = o0 + lane; i < o1; i += 64) {
    const double d0 = T.ccx[i] - Un[0], d1 = T.ccy[i] - Un[1], d2 = T.ccz[i] - Un[2];
    s[0] += d0; s[1] += d1; s[2] += d2;
    s[3] += d0 * d0 + d1 * d1 + d2 * d2;
    s[4] += T.cerot[i];
    SIp += (double)T.kvib[i];
  }
  for (int k = 0; k < 5; ++k) s[k] = wave_sum(s[k]);
  SIp = wave_sum(SIp);
  const double Nd = (double)N;
  const double m1[3] = {s[0] / Nd, s[1] / Nd, s[2] / Nd};
  const double etr_s = 0.5 * (s[3] / Nd - (m1[0] * m1[0] + m1[1] * m1[1] + m1[2] * m1[2]));
  const double erot_s = s[4] / Nd, erot_t = cs[CS_EROT_NEW * M + c];
  const bool rot = erot_s > 0.0 && erot_t > 0.0;
  const double frot = rot ? erot_t / erot_s : 1.0;
  const double erot_a = rot ? erot_t : erot_s;
  const double RTh = gas.R * gas.theta;
  const double evib_a = SIp * RTh / Nd;
  const double E0 = cs[CS_ETR * M + c] + cs[CS_EROT * M + c] + cs[CS_EVIB * M + c];
  const double s2 = (E0 - erot_a - evib_a) / etr_s;
  const bool vel = etr_s > 0.0 && s2 > 0.0;
  const double sc = vel ? sqrt(s2) : 0.0;
  const double Us[3] = {Un[0] + m1[0], Un[1] + m1[1], Un[2] + m1[2]};
  for (int o = 0; o < NOBJ; ++o) {
    // reverse sums over the cell
    double r[5] = {0, 0, 0, 0, 0};  // Lambda_e, L_sc, sum lc (3)
    for (int64_t i = o0 + lane; i < o1; i += 64) {
      double lc[3], le, ly;
      post(i, o, lc, &le, &ly);
      r[0] += le * T.cerot[i];
      r[1] += lc[0] * (T.ccx[i] - Us[0]) + lc[1] * (T.ccy[i] - Us[1]) + lc[2] * (T.ccz[i] - Us[2]);
      r[2] += lc[0]; r[3] += lc[1]; r[4] += lc[2];
    }
    for (int k = 0; k < 5; ++k) r[k] = wave_sum(r[k]);
    double l_erot_t = 0.0, l_erot_s = 0.0;
    if (rot) {
      const double lfrot = r[0];
      l_erot_t = lfrot / erot_s;
      l_erot_s = -lfrot * frot / erot_s;
    }
    double lE0 = 0.0, letr = 0.0, lUs[3] = {0, 0, 0}, lUn[3] = {0, 0, 0};
    if (vel) {
      const double ls2 = r[1] / (2.0 * sc);
      lE0 = ls2 / etr_s;
      const double lerot_a = -ls2 / etr_s;
      letr = -ls2 * s2 / etr_s;
      for (int k = 0; k < 3; ++k) { lUs[k] = -sc * r[2 + k]; lUn[k] = r[2 + k]; }
      if (rot) l_erot_t += lerot_a; else l_erot_s += lerot_a;
    }
    for (int64_t i = o0 + lane; i < o1; i += 64) {
      double lc[3], le, ly;
      post(i, o, lc, &le, &ly);
      const double cst[3] = {T.ccx[i], T.ccy[i], T.ccz[i]};
      for (int k = 0; k < 3; ++k) {
        const double v = (vel ? sc * lc[k] : lc[k]) + letr * (cst[k] - Us[k]) / Nd + lUs[k] / Nd;
        lam_at(lam1, o, LCX + k, cap, i) = v;
      }
      lam_at(lam1, o, LE, cap, i) = (rot ? frot * le : le) + l_erot_s / Nd;
      lam_at(lam1, o, LY, cap, i) = ly;
    }
    if (lane == 0) {
      double* cc = cons + (int64_t)o * NCONS * M;
      for (int k = 0; k < 3; ++k) cc[(CC_U + k) * M + c] = lUn[k];
      cc[CC_EROT_NEW * M + c] = l_erot_t;
      cc[CC_E0 * M + c] = lE0;
    }
  }
}

// ---- K2: the particle update reversed, thread per particle --------------------
__global__ __launch_bounds__(256) void k_adj_collide(GridP g, GasP gas, TapeP T, int64_t cap,
                                                     uint64_t seed, uint32_t step,
                                                     double* __restrict__ lam1,
                                                     double* __restrict__ own,
                                                     double* __restrict__ nbr,
                                                     int32_t* __restrict__ nbrc) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = g.M;
  if (i >= T.offsets[M]) return;
  const int32_t c = T.cell[i];
  const double* cs = T.cs;
  for (int o = 0; o < NOBJ; ++o) {
    for (int f = 0; f < NOWN; ++f) own[((int64_t)o * NOWN + f) * cap + i] = 0.0;
    for (int f = 0; f < NNBR; ++f) nbr[((int64_t)o * NNBR + f) * cap + i] = 0.0;
  }
  nbrc[i] = -1;
  if (cs[CS_COLLIDE * M + c] == 0.0) return;  // identity: lam1 already holds the adjoint
  const PartP<double> p = tape_parts(T, cap);
  const Stencil st = particle_stencil<double>(g, cell_records(cs, M)[c].stencil, c,
                                              load_pos(p, i, g.dim));
  double U[3], P[6], Tk[3];
  fields_planes(cs, M, c, st, U, P, Tk);
  bool floored[3];
  for (int k = 0; k < 3; ++k) floored[k] = Tk[k] == 0.05 * cs[(CS_TTR + k) * M + c] &&
                                           interp_planes(cs, M, CS_TTR + k, c, st) < Tk[k];
  const CellCoef cc = coef_planes(cs, M, c, false);  // the adjoint takes the Prandtl-number rule
  const PartCoef<double> pc = particle_coef<double>(gas.R, gas.theta, Tk[0], Tk[1], Tk[2], P, cc);
  if (pc.fallback) {
    // held fixed: no adjoint reaches the pre-collision values through it
    for (int o = 0; o < NOBJ; ++o)
      for (int k = 0; k < 4; ++k) lam_at(lam1, o, LCX + k, cap, i) = 0.0;
    return;
  }
  const double R = gas.R;
  Dual<6> Ttr_rel, Trot_rel;
  trel_dual(gas.theta, Tk[0], Tk[1], Tk[2], cc.a, cc.b, cc.oma2, &Ttr_rel, &Trot_rel);
  const bool rclamp = pc.clamp_rot;
  // draws (the forward's)
  const U4 w0 = philox(T.pid[i], step, TAG_COLLIDE, 0u, seed);
  double G1, G2, G3, G4;
  box_muller<double>(w0.w[0], w0.w[1], &G1, &G2);
  box_muller<double>(w0.w[2], w0.w[3], &G3, &G4);
  const double al = cc.al, oma2 = cc.oma2, nu = cc.nu, sq = sqrt(oma2);
  const double* L = pc.L;
  const double v[3] = {L[0] * G1, L[1] * G1 + L[2] * G2, L[3] * G1 + L[4] * G2 + L[5] * G3};
  const double cin[3] = {T.cx[i], T.cy[i], T.cz[i]}, ein = T.erot[i];
  const double Trr = pc.Trot_rel;
  const double half = 0.5 * R * Trr * oma2;
  const double se = sqrt(ein), sh = sqrt(half);
  const double root = se * al + sh * G4;
  const int ty = st.hy ? (int)(st.c01 - c) : 0;
  if (st.hy) nbrc[i] = (int32_t)st.c01;
  for (int o = 0; o < NOBJ; ++o) {
    double lcp[3];
    for (int k = 0; k < 3; ++k) lcp[k] = lam_at(lam1, o, LCX + k, cap, i);
    const double lep = lam_at(lam1, o, LE, cap, i);
    double lU[3], lc[3], lP[6] = {0, 0, 0, 0, 0, 0}, lT[3] = {0, 0, 0};
    double lal = 0.0, lsq = 0.0;
    double lL[6];
    for (int k = 0; k < 3; ++k) {
      lU[k] = (1.0 - al) * lcp[k];
      lc[k] = al * lcp[k];
      lal += lcp[k] * (cin[k] - U[k]);
      lsq += lcp[k] * v[k];
    }
    const double lv0 = sq * lcp[0], lv1 = sq * lcp[1], lv2 = sq * lcp[2];
    lL[0] = lv0 * G1; lL[1] = lv1 * G1; lL[2] = lv1 * G2;
    lL[3] = lv2 * G1; lL[4] = lv2 * G2; lL[5] = lv2 * G3;
    // rotational energy
    double lhalf = lep;
    const double lroot = 2.0 * root * lep;
    const double le = se > 0.0 ? lroot * al / (2.0 * se) : 0.0;
    lal += lroot * se;
    if (sh > 0.0) lhalf += lroot * G4 / (2.0 * sh);
    const double lTrr = rclamp ? 0.0 : lhalf * 0.5 * R * oma2;
    double loma2 = lhalf * 0.5 * R * Trr + lsq / (2.0 * sq);
    // Lambda = R T_tr^rel I + nu (Pi - R T_tr I), its Cholesky factor
    double lS[6];
    chol3_reverse(L, lL, lS);
    const double lTtr_rel = R * (lS[0] + lS[1] + lS[2]);
    double lnu = 0.0;
    for (int k = 0; k < 3; ++k) lnu += lS[k] * (P[k] - R * Tk[0]);
    for (int k = 3; k < 6; ++k) lnu += lS[k] * P[k];
    for (int k = 0; k < 6; ++k) lP[k] += nu * lS[k];
    lT[0] += -nu * R * (lS[0] + lS[1] + lS[2]);
    // relaxation temperatures: inputs (T_tr, T_rot, T_vib, a, b, 1-alpha^2)
    double lin6[6];
    for (int k = 0; k < 6; ++k) lin6[k] = lTtr_rel * Ttr_rel.d[k] + lTrr * Trot_rel.d[k];
    lT[0] += lin6[0]; lT[1] += lin6[1]; lT[2] += lin6[2];
    const double la = lin6[3], lb = lin6[4];
    loma2 += lin6[5];
    // floors and the reconstruction (Sec. III.B, 1D: own cell and c01)
    double* ow = own + (int64_t)o * NOWN * cap;
    double* nb = nbr + (int64_t)o * NNBR * cap;
    double lw = 0.0;
    auto scatter = [&](int f, int plane, double lf) {
      const double* F = cs + (int64_t)plane * M;
      if (st.hy) {
        ow[(int64_t)f * cap + i] += (1.0 - st.wy) * lf;
        nb[(int64_t)f * cap + i] += st.wy * lf;
        lw += (F[st.c01] - F[c]) * lf;
      } else {
        ow[(int64_t)f * cap + i] += lf;
      }
    };
    for (int k = 0; k < 3; ++k) scatter(CF_U + k, CS_UX + k, lU[k]);
    for (int k = 0; k < 6; ++k) scatter(CF_P + k, CS_PXX + k, lP[k]);
    for (int k = 0; k < 3; ++k) {
      if (floored[k]) ow[(int64_t)(CF_T + k) * cap + i] += 0.05 * lT[k];
      else scatter(CF_T + k, CS_TTR + k, lT[k]);
    }
    ow[(int64_t)CF_A * cap + i] = la;
    ow[(int64_t)CF_B * cap + i] = lb;
    ow[(int64_t)CF_AL * cap + i] = lal;
    ow[(int64_t)CF_OMA2 * cap + i] = loma2;
    ow[(int64_t)CF_NU * cap + i] = lnu;
    for (int k = 0; k < 3; ++k) lam_at(lam1, o, LCX + k, cap, i) = lc[k];
    lam_at(lam1, o, LE, cap, i) = le;
    if (ty != 0) lam_at(lam1, o, LY, cap, i) += lw / ((double)ty * g.dy);
  }
}

// lane 0 of K3: the cell state reversed for objective o
__device__ __forceinline__ void cell_reverse(const GasP& gas, int64_t c, int64_t M, int o,
                                             const double lf[NOWN], const Dual<6> co[6],
                                             const double* __restrict__ cons,
                                             double* __restrict__ lmom,
                                             double* __restrict__ gcell) {
  {
    const double R = gas.R;
    const double* cc = cons + (int64_t)o * NCONS * M;
    double lU[3], lP[6];
    for (int k = 0; k < 3; ++k) lU[k] = lf[CF_U + k] + cc[(CC_U + k) * M + c];
    for (int k = 0; k < 6; ++k) lP[k] = lf[CF_P + k];
    const double lE0 = cc[CC_E0 * M + c];
    // coefficients (a, b, alpha, 1-alpha^2, nu, e_rot target) of (T_tr,
    // T_rot, T_vib, Z_rot, omega, mu_ref)
    const double lout[6] = {lf[CF_A], lf[CF_B], lf[CF_AL], lf[CF_OMA2], lf[CF_NU],
                            cc[CC_EROT_NEW * M + c]};
    double lin[6] = {0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 6; ++q)
      for (int k = 0; k < 6; ++k) lin[k] += lout[q] * co[q].d[k];
    const double lTtr = lf[CF_T] + lin[0];
    const double lTrot = lf[CF_T + 1] + lin[1];
    // T_tr = tr(Pi)/(3R), T_rot = e_rot/R, E0 = tr(Pi)/2 + e_rot + I R theta
    for (int k = 0; k < 3; ++k) lP[k] += lTtr / (3.0 * R) + 0.5 * lE0;
    double* lm = lmom + (int64_t)o * NAMOM * M;
    for (int k = 0; k < 3; ++k) lm[(AM_U + k) * M + c] = lU[k];
    for (int k = 0; k < 6; ++k) lm[(AM_P + k) * M + c] = lP[k];
    lm[AM_EROT * M + c] = lTrot / R + lE0;
    for (int k = 0; k < NPAR; ++k) gcell[((int64_t)o * NPAR + k) * M + c] = lin[3 + k];
  }
}

// ---- K3: cell adjoints, then the cell state reversed ---------------------------
// K3a: one wave per (objective, field, cell): the cell's own particles'
// contributions plus those of the neighbouring cells' particles whose
// stencil reads it (1D: cells c-1 and c+1), in a fixed order.
__global__ __launch_bounds__(256) void k_adj_cell_sums(int64_t M, TapeP T, int64_t cap,
                                                       const double* __restrict__ own,
                                                       const double* __restrict__ nbr,
                                                       const int32_t* __restrict__ nbrc,
                                                       double* __restrict__ csum) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (w >= (int64_t)NOBJ * NOWN * M) return;
  const int64_t c = w % M, of = w / M;
  const int o = (int)(of / NOWN), f = (int)(of % NOWN);
  const int64_t o0 = T.offsets[c], o1 = T.offsets[c + 1];
  double s = 0.0;
  if (T.cs[CS_COLLIDE * M + c] != 0.0) {
    const double* ow = own + ((int64_t)o * NOWN + f) * cap;
    for (int64_t i = o0 + lane; i < o1; i += 64) s += ow[i];
    if (f < NNBR) {
      const double* nb = nbr + ((int64_t)o * NNBR + f) * cap;
      const int64_t lo_n = c > 0 ? T.offsets[c - 1] : o0;
      const int64_t hi_n = c + 1 < M ? T.offsets[c + 2] : o1;
      for (int64_t i = lo_n + lane; i < o0; i += 64)
        if (nbrc[i] == c) s += nb[i];
      for (int64_t i = o1 + lane; i < hi_n; i += 64)
        if (nbrc[i] == c) s += nb[i];
    }
  }
  s = wave_sum(s);
  if (lane == 0) csum[of * M + c] = s;
}

// K3b: thread per cell: the cell state reversed (Dual<6> Jacobian of the
// coefficients), giving moment adjoints and per-cell parameter partials.
__global__ __launch_bounds__(64) void k_adj_cellstate(GridP g, GasP gas, double alpha_vss,
                                                      TapeP T, const double* __restrict__ csum,
                                                      const double* __restrict__ cons,
                                                      double* __restrict__ lmom,
                                                      double* __restrict__ gcell) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = g.M;
  if (c >= M) return;
  const double* cs = T.cs;
  for (int o = 0; o < NOBJ; ++o) {
    for (int k = 0; k < NAMOM; ++k) lmom[((int64_t)o * NAMOM + k) * M + c] = 0.0;
    for (int k = 0; k < NPAR; ++k) gcell[((int64_t)o * NPAR + k) * M + c] = 0.0;
  }
  if (cs[CS_COLLIDE * M + c] == 0.0) return;
  Dual<6> co[6];
  cell_coef_dual(gas, alpha_vss, cs[CS_NDENS * M + c], cs[CS_DT * M + c], cs[CS_TTR * M + c],
                 cs[CS_TROT * M + c], cs[CS_TVIB * M + c], co);
  for (int o = 0; o < NOBJ; ++o) {
    double lf[NOWN];
    for (int f = 0; f < NOWN; ++f) lf[f] = csum[((int64_t)o * NOWN + f) * M + c];
    cell_reverse(gas, c, M, o, lf, co, cons, lmom, gcell);
  }
}

// ---- K4: moments reversed, mass-flow source, bin undone -----------------------
__global__ __launch_bounds__(256) void k_adj_moments(GridP g, TapeP T, int64_t cap,
                                                     const double* __restrict__ lam1,
                                                     const double* __restrict__ lmom,
                                                     double* __restrict__ lam_out, double w_mdot) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t M = g.M;
  if (i >= T.offsets[M]) return;
  const int32_t c = T.cell[i];
  const double* cs = T.cs;
  const double N = (double)(T.offsets[c + 1] - T.offsets[c]);
  const double d[3] = {T.cx[i] - cs[CS_UX * M + c], T.cy[i] - cs[CS_UY * M + c],
                       T.cz[i] - cs[CS_UZ * M + c]};
  const int32_t j = T.perm[i];
  if (j < 0) return;
  for (int o = 0; o < NOBJ; ++o) {
    const double* lm = lmom + (int64_t)o * NAMOM * M;
    double lP[6];
    for (int k = 0; k < 6; ++k) lP[k] = lm[(AM_P + k) * M + c];
    // Pi = <C C>: xx yy zz xy xz yz
    const double gP[3] = {2.0 * d[0] * lP[0] + d[1] * lP[3] + d[2] * lP[4],
                          2.0 * d[1] * lP[1] + d[0] * lP[3] + d[2] * lP[5],
                          2.0 * d[2] * lP[2] + d[0] * lP[4] + d[1] * lP[5]};
    for (int k = 0; k < 3; ++k) {
      double v = lam_at(const_cast<double*>(lam1), o, LCX + k, cap, i) +
                 (lm[(AM_U + k) * M + c] + gP[k]) / N;
      if (o == 0 && k == 0) v += w_mdot;
      lam_at(lam_out, o, LCX + k, cap, j) = v;
    }
    lam_at(lam_out, o, LE, cap, j) =
        lam_at(const_cast<double*>(lam1), o, LE, cap, i) + lm[AM_EROT * M + c] / N;
    lam_at(lam_out, o, LY, cap, j) = lam_at(const_cast<double*>(lam1), o, LY, cap, i);
  }
}

// ---- K5: parameter partials summed in a fixed order -------------------------
__global__ __launch_bounds__(256) void k_adj_grad(int64_t M, const double* __restrict__ gcell,
                                                  double* __restrict__ grad) {
  __shared__ double red[256];
  for (int q = 0; q < NOBJ * NPAR; ++q) {
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < M; c += 256) s += gcell[(int64_t)q * M + c];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) grad[q] += red[0];
    __syncthreads();
  }
}

static hipError_t adjoint_step(const GridP& g, const GasP& gas, const BcP& bc, double alpha_vss,
                               double dt, const TapeP& T, int64_t cap, uint64_t seed,
                               uint64_t step, const double* lam_in, double* lam_out,
                               double w_mdot, double w_tau, double* grad, char* aws,
                               const AdjWsLayout& W, hipStream_t st) {
  double* lam1 = (double*)(aws + W.lam1);
  double* own = (double*)(aws + W.own);
  double* nbr = (double*)(aws + W.nbr);
  int32_t* nbrc = (int32_t*)(aws + W.nbrc);
  double* cons = (double*)(aws + W.cons);
  double* lmom = (double*)(aws + W.lmom);
  double* gcell = (double*)(aws + W.gcell);
  const int cells = (int)cdiv(g.M, 4);
  const int parts = (int)cdiv(cap, 256);
  k_adj_flight_conserve<<<cells, 256, 0, st>>>(g, gas, bc, dt, T, cap, lam_in, lam1, cons, w_tau);
  k_adj_collide<<<parts, 256, 0, st>>>(g, gas, T, cap, seed, (uint32_t)step, lam1, own, nbr, nbrc);
  double* csum = (double*)(aws + W.csum);
  k_adj_cell_sums<<<(int)cdiv((int64_t)NOBJ * NOWN * g.M, 4), 256, 0, st>>>(g.M, T, cap, own, nbr,
                                                                            nbrc, csum);
  k_adj_cellstate<<<(int)cdiv(g.M, 64), 64, 0, st>>>(g, gas, alpha_vss, T, csum, cons, lmom, gcell);
  k_adj_moments<<<parts, 256, 0, st>>>(g, T, cap, lam1, lmom, lam_out, w_mdot);
  k_adj_grad<<<1, 256, 0, st>>>(g.M, gcell, grad);
  return hipGetLastError();
}

}  // namespace usp

using namespace usp;

namespace {

bool adj_setup_ok(const usp_grid* grid, const usp_gas* gas) {
  if (!grid || !gas || grid->dim != 1 || grid->nx != 1 || grid->ny <= 0 || !grid->volume) return false;
  if (!(grid->dy > 0.0) || !(grid->fnum > 0.0)) return false;
  if (gas->scheme != USP_SCHEME_USP) return false;
  // the reverse pass differentiates the per-particle chain with the
  // Prandtl-number sign rule
  if (gas->gamma_scope != USP_GAMMA_PARTICLE || gas->alpha_sign != USP_ALPHA_SIGN_PR) return false;
  if (gas->zrot_model != USP_ZROT_CONST || gas->zvib_model != USP_ZVIB_CONST) return false;
  return gas->m > 0.0 && gas->theta_vib > 0.0 && gas->T_ref > 0.0 && gas->mu_ref > 0.0 &&
         gas->alpha_vss > 0.0;
}

}  // namespace

extern "C" {

size_t usp_tape_bytes(const usp_grid* grid, int64_t capacity) {
  if (!grid || grid->dim != 1 || grid->ny <= 0 || capacity <= 0) return 0;
  return tape_layout((int64_t)grid->nx * grid->ny, capacity).total;
}

size_t usp_adjoint_ws_bytes(const usp_grid* grid, int64_t capacity) {
  if (!grid || grid->dim != 1 || grid->ny <= 0 || capacity <= 0) return 0;
  return adj_ws_layout((int64_t)grid->nx * grid->ny, capacity).total;
}

usp_status usp_step_taped(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                          usp_particles* p, usp_particles* p_alt, int64_t* offsets,
                          const int64_t* in_offsets, double* mom, double* cs, void* ws,
                          size_t ws_bytes, uint64_t seed, uint64_t step, void* tape,
                          size_t tape_bytes, void* aws, size_t aws_bytes, int64_t* counters,
                          void* stream) {
  if (!adj_setup_ok(grid, gas) || !bc || !p || !p_alt || !offsets || !mom || !cs || !ws || !tape ||
      !aws)
    return USP_EINVAL;
  if (p->prec != USP_F64 || p_alt->prec != USP_F64 || !(dt > 0.0)) return USP_EINVAL;
  if (p->capacity != p_alt->capacity || p->cx == p_alt->cx || !p->y || !p_alt->y) return USP_EINVAL;
  if (bc->surf_nbody < 0) return USP_EINVAL;
  const int64_t cap = p->capacity;
  if (ws_bytes < usp_workspace_bytes(grid, cap) || tape_bytes < usp_tape_bytes(grid, cap) ||
      aws_bytes < usp_adjoint_ws_bytes(grid, cap))
    return USP_EINVAL;
  const GridP g = make_grid(grid);
  const TapeLayout T = tape_layout(g.M, cap);
  const AdjWsLayout W = adj_ws_layout(g.M, cap);
  const WsLayout L = ws_layout(g.M, cap, n_faces(g));
  hipStream_t st = (hipStream_t)stream;
  const hipError_t e = step_taped(g, make_gas(gas), make_bc(bc), dt, make_parts<double>(p),
                                  make_parts<double>(p_alt), offsets, in_offsets, mom, cs,
                                  (char*)ws, L, seed,
                                  step, (char*)tape, T, (int32_t*)((char*)aws + W.map), counters, st);
  if (e != hipSuccess) return USP_EDEVICE;
  const usp_particles tmp = *p;
  *p = *p_alt;
  *p_alt = tmp;
  return USP_OK;
}

usp_status usp_adjoint_step(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                            const void* tape, size_t tape_bytes, int64_t capacity, uint64_t seed,
                            uint64_t step, const double* lam_in, double* lam_out, double w_mdot,
                            double w_tau, double* grad, void* aws, size_t aws_bytes,
                            void* stream) {
  if (!adj_setup_ok(grid, gas) || !bc || !tape || !lam_in || !lam_out || !grad || !aws)
    return USP_EINVAL;
  if (lam_in == lam_out || !(dt > 0.0) || capacity <= 0) return USP_EINVAL;
  if (tape_bytes < usp_tape_bytes(grid, capacity) || aws_bytes < usp_adjoint_ws_bytes(grid, capacity))
    return USP_EINVAL;
  const GridP g = make_grid(grid);
  const TapeLayout T = tape_layout(g.M, capacity);
  const AdjWsLayout W = adj_ws_layout(g.M, capacity);
  const hipError_t e = adjoint_step(g, make_gas(gas), make_bc(bc), gas->alpha_vss, dt,
                                    tape_ptrs((const char*)tape, T), capacity, seed, step, lam_in,
                                    lam_out, w_mdot, w_tau, grad, (char*)aws, W,
                                    (hipStream_t)stream);
  return e == hipSuccess ? USP_OK : USP_EDEVICE;
}

}  // extern "C"
