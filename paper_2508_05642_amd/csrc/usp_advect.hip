// usp_advect.hip -- free flight with boundaries, and free-stream injection.
//
// Flight arithmetic is FP64 for both state precisions (a few dozen FP64
// operations per particle); the result is rounded to the stored precision
// and kept inside the domain.
#include "usp_particle.h"

namespace usp {

constexpr int ADV_BLOCK = 256;

template <typename S>
__global__ __launch_bounds__(ADV_BLOCK) void k_advect(GridP g, GasP gas, BcP bc, double dt,
                                                      PartP<S> p, uint64_t seed, uint32_t step,
                                                      int64_t* counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.count[0]) return;
  if (p.cell[i] < 0) return;
  advect_one<S>(g, gas, bc, dt, p, i, load_pos(p, i, g.dim), p.cx[i], p.cy[i], p.cz[i], p.erot[i],
                p.vib[i], seed, step, counters);
}

// ---- free-stream injection ------------------------------------------------
__host__ __device__ inline int face_side(int64_t f, int nx, int ny) {
  return f < ny ? 0 : (f < 2 * ny ? 1 : (f < 2 * ny + nx ? 2 : 3));
}

__host__ __device__ inline double inward_speed(const BcP& bc, int side) {
  return side == 0 ? bc.fs_U[0] : side == 1 ? -bc.fs_U[0] : side == 2 ? bc.fs_U[1] : -bc.fs_U[1];
}

// expected injections through one face per step: number flux of a drifting
// Maxwellian n sqrt(RT/2pi) (e^{-s^2} + sqrt(pi) s (1 + erf s)), s = U_n/sqrt(2RT)
__host__ __device__ inline double face_lambda(const GridP& g, double R, const BcP& bc, double dt,
                                              int side) {
  const double T = bc.fs_T, Un = inward_speed(bc, side);
  const double s = Un / sqrt(2.0 * R * T);
  const double flux = bc.fs_n * sqrt(R * T / (2.0 * PI)) * (exp(-s * s) + sqrt(PI) * s * (1.0 + erf(s)));
  const double area = (side < 2 ? g.dy : g.dx) * bc.depth;
  return flux * area * dt / g.fnum;
}

__global__ void k_inject_count(GridP g, GasP gas, BcP bc, double dt, uint64_t seed, uint32_t step,
                               int64_t nf, int32_t* face_cnt) {
  const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= nf) return;
  const int side = face_side(f, g.nx, g.ny);
  int32_t n = 0;
  if (bc.kind[side] == USP_BC_FREESTREAM) {
    const double lam = face_lambda(g, gas.R, bc, dt, side);
    const U4 w = philox((uint32_t)f, step, TAG_FACE, 0u, seed);
    n = (int32_t)floor(lam + u01d(w.w[0]));
  }
  face_cnt[f] = n;
}

// one block: exclusive scan of the face counts; capacity check; the block's
// results go to misc = {injections this step, first slot, first id}
__global__ __launch_bounds__(256) void k_inject_scan(const int32_t* face_cnt, int64_t nf,
                                                     int64_t* face_off, int64_t* count,
                                                     int64_t capacity, int64_t* misc,
                                                     int64_t* counters) {
  __shared__ int64_t wsum[4];
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nf; b0 += 256) {
    const int64_t j = b0 + threadIdx.x;
    const int64_t v = j < nf ? face_cnt[j] : 0;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int64_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
      const int64_t y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wid] = x;
    __syncthreads();
    int64_t base = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
      if (w < wid) base += wsum[w];
      tot += wsum[w];
    }
    if (j < nf) face_off[j] = carry + base + x - v;
    __syncthreads();
    carry += tot;
  }
  if (threadIdx.x == 0) {
    face_off[nf] = carry;
    const int64_t n = count[0];
    const int64_t avail = capacity - n;
    const int64_t take = carry > avail ? avail : carry;
    if (counters) {
      if (carry > take) counters[USP_CNT_CAPACITY] += carry - take;
      counters[USP_CNT_INJECTED] += take;
    }
    misc[0] = take;
    misc[1] = n;
    misc[2] = count[1];
  }
}

// Dimensionless inward normal speed u = v_n/sqrt(2RT), density u e^{-(u-s)^2}
// on u > 0.  s >= 0: mixture of w e^{-w^2} (w > 0), s e^{-w^2} (w > 0) and
// (w + s) e^{-w^2} on (-s, 0) with w = u - s, chosen by their masses; s < 0:
// rejection from u e^{-u^2} (|s| < 1) or from u e^{-2|s|u} (|s| >= 1).
__device__ double inflow_speed(uint64_t seed, uint32_t step, uint32_t pid, double s) {
  const U4 b1 = philox(pid, step, TAG_INJECT, 1u, seed);
  if (s >= 0.0) {
    const double mA1 = 0.5, mA2 = 0.5 * sqrt(PI) * s;
    double mB = 0.5 * (sqrt(PI) * s * erf(s) - (1.0 - exp(-s * s)));
    if (mB < 0.0) mB = 0.0;
    const double v = u01d(b1.w[2]) * (mA1 + mA2 + mB);
    if (v < mA1) {
      const U4 a = philox(pid, step, TAG_INJECT, 2u, seed);
      return sqrt(-log(u01d(a.w[0]))) + s;
    }
    if (v < mA1 + mA2) {
      const U4 a = philox(pid, step, TAG_INJECT, 2u, seed);
      double sn, cs;
      sincospi(2.0 * u01d(a.w[1]), &sn, &cs);
      const double G = sqrt(-2.0 * log(u01d(a.w[0]))) * cs;
      return fabs(G) / sqrt(2.0) + s;
    }
    double w = 0.0;
    for (uint32_t att = 0; att < 10000; ++att) {
      const U4 a = philox(pid, step, TAG_INJECT, 2u + att, seed);
      w = s * sqrt(u01d(a.w[0])) - s;
      if (u01d(a.w[1]) < exp(-w * w)) break;
    }
    return w + s;
  }
  const double sg = -s;
  double t = 0.0;
  for (uint32_t att = 0; att < 10000; ++att) {
    const U4 a = philox(pid, step, TAG_INJECT, 2u + att, seed);
    if (sg < 1.0) {
      t = sqrt(-log(u01d(a.w[0])));
      if (u01d(a.w[1]) < exp(-2.0 * sg * t)) break;
    } else {
      t = (-log(u01d(a.w[0])) - log(u01d(a.w[1]))) / (2.0 * sg);
      if (u01d(a.w[2]) < exp(-t * t)) break;
    }
  }
  return t;
}

template <typename S>
__global__ __launch_bounds__(ADV_BLOCK) void k_inject(GridP g, GasP gas, BcP bc, double dt,
                                                      PartP<S> p, uint64_t seed, uint32_t step,
                                                      const int64_t* face_off, int64_t nf,
                                                      const int64_t* misc, int64_t* counters) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= misc[0]) return;
  // face f with face_off[f] <= k < face_off[f+1]
  int64_t lo = 0, hi = nf - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (face_off[mid] <= k) lo = mid; else hi = mid - 1;
  }
  const int64_t f = lo;
  const int side = face_side(f, g.nx, g.ny);
  const int64_t loc = side == 0 ? f : side == 1 ? f - g.ny : side == 2 ? f - 2 * g.ny : f - 2 * g.ny - g.nx;
  const int64_t slot = misc[1] + k;
  const uint32_t id = (uint32_t)(misc[2] + k);
  const double R = gas.R, T = bc.fs_T, sig = sqrt(R * T), vs = sqrt(2.0 * R * T);
  const U4 b0 = philox(id, step, TAG_INJECT, 0u, seed);
  const U4 b1 = philox(id, step, TAG_INJECT, 1u, seed);
  const double vn = inflow_speed(seed, step, id, inward_speed(bc, side) / vs) * vs;
  const double rr = sqrt(-2.0 * log(u01d(b1.w[0])));
  double sn, cs;
  sincospi(2.0 * u01d(b1.w[1]), &sn, &cs);
  const double ga = sig * rr * cs, gb = sig * rr * sn;
  const double xlo = (double)(S)g.x0, xhi = (double)edge<S>(g.x0, g.dx, g.nx);
  const double ylo = (double)(S)g.y0, yhi = (double)edge<S>(g.y0, g.dy, g.ny);
  double x, y, cx, cy;
  const double cz = bc.fs_U[2] + gb;
  if (side < 2) {
    x = side == 0 ? xlo : xhi;
    y = g.y0 + ((double)loc + u01d(b0.w[0])) * g.dy;
    cx = side == 0 ? vn : -vn;
    cy = bc.fs_U[1] + ga;
  } else {
    y = side == 2 ? ylo : yhi;
    x = g.x0 + ((double)loc + u01d(b0.w[0])) * g.dx;
    cy = side == 2 ? vn : -vn;
    cx = bc.fs_U[0] + ga;
  }
  const double tf = u01d(b0.w[1]) * dt;
  x += cx * tf;
  y += cy * tf;
  const double lvl = floor(log(u01d(b0.w[3])) / (-gas.theta / T));
  const S xs = (S)x, ys = (S)y;
  p.x[slot] = xs;
  p.y[slot] = ys;
  p.cx[slot] = (S)cx;
  p.cy[slot] = (S)cy;
  p.cz[slot] = (S)cz;
  p.erot[slot] = (S)(-R * T * log(u01d(b0.w[2])));
  p.vib[slot] = (uint8_t)(lvl > (double)VIB_MAX ? VIB_MAX : (int)lvl);
  p.pid[slot] = id;
  const double xd = (double)xs, yd = (double)ys;
  bool out = !(xd >= xlo && xd < xhi && yd >= ylo && yd < yhi);
  if (!out && bc.cyl) {
    const double ddx = xd - bc.cyl_xc, ddy = yd - bc.cyl_yc;
    out = ddx * ddx + ddy * ddy < bc.cyl_r * bc.cyl_r;
  }
  p.cell[slot] = out ? -1 : cell_of<S>(g, xs, ys);
  if (out) count_event(counters, USP_CNT_DELETED);
}

__global__ void k_inject_finish(int64_t* count, const int64_t* misc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    count[0] = misc[1] + misc[0];
    count[1] = misc[2] + misc[0];
  }
}

int n_faces(const GridP& g) { return g.dim == 2 ? 2 * (g.nx + g.ny) : 0; }

// Free-stream injection of one step: per-face counts, their scan (with the
// capacity check) and the new particles appended after the current ones.
template <typename S>
hipError_t launch_inject(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const PartP<S>& p, uint64_t seed, uint64_t step, char* ws,
                         const WsLayout& L, int64_t* counters, hipStream_t st) {
  const int64_t nf = n_faces(g);
  bool any = false;
  int64_t bound = 0;
  for (int64_t f = 0; f < nf; ++f) {
    const int side = face_side(f, g.nx, g.ny);
    if (bc.kind[side] != USP_BC_FREESTREAM) continue;
    any = true;
    bound += (int64_t)floor(face_lambda(g, gas.R, bc, dt, side)) + 1;
  }
  if (!any) return hipGetLastError();
  int32_t* face_cnt = (int32_t*)(ws + L.face_cnt);
  int64_t* face_off = (int64_t*)(ws + L.face_off);
  int64_t* misc = (int64_t*)(ws + L.misc);
  k_inject_count<<<cdiv(nf, 256), 256, 0, st>>>(g, gas, bc, dt, seed, (uint32_t)step, nf, face_cnt);
  k_inject_scan<<<1, 256, 0, st>>>(face_cnt, nf, face_off, p.count, p.capacity, misc, counters);
  if (bound > 0)
    k_inject<S><<<cdiv(bound, ADV_BLOCK), ADV_BLOCK, 0, st>>>(g, gas, bc, dt, p, seed, (uint32_t)step,
                                                             face_off, nf, misc, counters);
  k_inject_finish<<<1, 64, 0, st>>>(p.count, misc);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_advect(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const PartP<S>& p, uint64_t seed, uint64_t step, char* ws,
                         const WsLayout& L, int64_t* counters, hipStream_t st) {
  if (g.dim == 0) return hipSuccess;
  k_advect<S><<<cdiv(p.capacity, ADV_BLOCK), ADV_BLOCK, 0, st>>>(g, gas, bc, dt, p, seed,
                                                                (uint32_t)step, counters);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_inject<S>(g, gas, bc, dt, p, seed, step, ws, L, counters, st);
}

template hipError_t launch_inject<float>(const GridP&, const GasP&, const BcP&, double,
                                         const PartP<float>&, uint64_t, uint64_t, char*,
                                         const WsLayout&, int64_t*, hipStream_t);
template hipError_t launch_inject<double>(const GridP&, const GasP&, const BcP&, double,
                                          const PartP<double>&, uint64_t, uint64_t, char*,
                                          const WsLayout&, int64_t*, hipStream_t);
template hipError_t launch_advect<float>(const GridP&, const GasP&, const BcP&, double,
                                         const PartP<float>&, uint64_t, uint64_t, char*,
                                         const WsLayout&, int64_t*, hipStream_t);
template hipError_t launch_advect<double>(const GridP&, const GasP&, const BcP&, double,
                                          const PartP<double>&, uint64_t, uint64_t, char*,
                                          const WsLayout&, int64_t*, hipStream_t);

}  // namespace usp
