// usp_update.hip -- the particle phase of a step in one pass over a binned
// state: the particle update (Secs. III.A-III.B), the conservation scheme
// (Sec. IV.C) and the free flight with boundaries.
//
// A workgroup owns a tile: the cells whose first particle lies in one
// window of TILE particle slots (so whole cells, ~TILE particles).  Three
// phases separated by workgroup barriers:
//   A  particle update, one thread per particle, into an LDS stage;
//   B  conservation, one wave per cell, on the stage;
//   C  free flight, one thread per particle, from the stage; the state is
//      written to HBM once.
// Tiles with more particles than the stage holds run the same phases in
// place in global memory.  The arithmetic is that of the separate phase
// kernels (shared device functions), in the same order, so the result is
// bit-identical to running them one after the other.
#include "usp_particle.h"

namespace usp {

constexpr int UPD_BLOCK = 256;
constexpr int UPD_WAVES = UPD_BLOCK / 64;

template <typename S> struct UpdCfg;
template <> struct UpdCfg<float> { static constexpr int TILE = UPDATE_TILE_F32, STAGE = 2048; };
template <> struct UpdCfg<double> { static constexpr int TILE = UPDATE_TILE_F64, STAGE = 1024; };

__global__ void k_fill_first(int32_t* first, int64_t n, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) first[t] = v;
}

// first[t] = the smallest cell c with offsets[c] >= t * T (tiles past the
// last particle keep the prefilled M): cell c owns the tiles t with
// offsets[c-1] < t T <= offsets[c].
__global__ void k_tile_first(const int64_t* __restrict__ offsets, int64_t M, int64_t T,
                             int64_t ntiles, int32_t* first) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c > M) return;
  const int64_t lo = c == 0 ? 0 : offsets[c - 1] / T + 1;
  int64_t hi = offsets[c] / T;
  if (hi > ntiles) hi = ntiles;
  for (int64_t t = lo; t <= hi; ++t) first[t] = (int32_t)c;
}

// First and second pass of the particle update: in FP32 the first pass
// flags the particles that need the FP64 chain (see collide_f32); the FP64
// state has a single pass.
__device__ __forceinline__ PartNew<float> update_first(const GridP& g, const GasP& gas,
                                                      const double* cs, const PartP<float>& p,
                                                      int64_t i, int32_t c, uint64_t seed,
                                                      uint32_t step, uint32_t* ev, bool* esc) {
  return collide_f32(g, gas, cs, p, i, c, seed, step, ev, esc);
}
__device__ __forceinline__ PartNew<double> update_first(const GridP& g, const GasP& gas,
                                                       const double* cs, const PartP<double>& p,
                                                       int64_t i, int32_t c, uint64_t seed,
                                                       uint32_t step, uint32_t* ev, bool* esc) {
  *esc = false;
  return collide_one(g, gas, cs, p, i, c, seed, step, ev);
}
__device__ __forceinline__ PartNew<float> update_second(const GridP& g, const GasP& gas,
                                                       const double* cs, const PartP<float>& p,
                                                       int64_t i, int32_t c, uint64_t seed,
                                                       uint32_t step, uint32_t* ev) {
  return collide_esc(g, gas, cs, p, i, c, seed, step, ev);
}
__device__ __forceinline__ PartNew<double> update_second(const GridP&, const GasP&, const double*,
                                                        const PartP<double>&, int64_t, int32_t,
                                                        uint64_t, uint32_t, uint32_t*) {
  PartNew<double> o;
  o.changed = false;
  return o;
}

// The three phases of one tile; vx* = stage (LDS, indexed i - base) or the
// particle arrays themselves (base 0).  esc/nesc: LDS list of the
// particles of the current chunk (CAP slots) left for the second pass.
template <typename S, bool STAGED, int CAP>
__device__ __forceinline__ void tile_pass(const GridP& g, const GasP& gas, const BcP& bc,
                                          double dt, const double* __restrict__ cs,
                                          const int64_t* __restrict__ offsets, const PartP<S>& p,
                                          int64_t c0, int64_t c1, int64_t i0, int64_t i1,
                                          S* vcx, S* vcy, S* vcz, S* ver, uint8_t* vvb,
                                          int64_t base, uint16_t* esc_list, int* nesc,
                                          uint64_t seed, uint32_t step, bool advect,
                                          int64_t* counters) {
  const int64_t M = g.M;
  auto put = [&](int64_t i, PartNew<S> o) {
    if (STAGED) {
      if (!o.changed) {
        o.cx = p.cx[i]; o.cy = p.cy[i]; o.cz = p.cz[i]; o.erot = p.erot[i]; o.vib = p.vib[i];
      }
      const int64_t j = i - base;
      vcx[j] = o.cx; vcy[j] = o.cy; vcz[j] = o.cz; ver[j] = o.erot; vvb[j] = (uint8_t)o.vib;
    } else if (o.changed) {
      p.cx[i] = o.cx; p.cy[i] = o.cy; p.cz[i] = o.cz; p.erot[i] = o.erot;
      p.vib[i] = (uint8_t)o.vib;
    }
  };
  // A: particle update, in chunks of CAP particles (one chunk when staged):
  // first pass thread per particle, then the listed particles' second pass
  for (int64_t cb = i0; cb < i1; cb += CAP) {
    const int64_t ce = cb + CAP < i1 ? cb + CAP : i1;
    if (threadIdx.x == 0) *nesc = 0;
    __syncthreads();
    for (int64_t i = cb + threadIdx.x; i < ce; i += UPD_BLOCK) {
      const int32_t c = p.cell[i];
      uint32_t ev = 0;
      bool esc = false;
      PartNew<S> o;
      o.changed = false;
      // The cell-state planes are read only on the second pass; opaque
      // copies of their base and stride keep the compiler from holding
      // every plane's address live across the loop.
      GridP gl = g;
      const double* csl = cs;
      asm volatile("" : "+s"(csl), "+s"(gl.M));
      if (c >= 0) o = update_first(gl, gas, csl, p, i, c, seed, step, &ev, &esc);
      if (esc) esc_list[atomicAdd(nesc, 1)] = (uint16_t)(i - cb);
      else put(i, o);
      flush_events(counters, ev);
    }
    __syncthreads();
    const int ne = *nesc;
    for (int k = threadIdx.x; k < ne; k += UPD_BLOCK) {
      const int64_t i = cb + esc_list[k];
      uint32_t ev = 0;
      put(i, update_second(g, gas, cs, p, i, p.cell[i], seed, step, &ev));
      flush_events(counters, ev);
    }
    __syncthreads();
  }
  // B: conservation, wave per cell
  const int wid = threadIdx.x >> 6;
  for (int64_t c = c0 + wid; c < c1; c += UPD_WAVES) {
    const int64_t o0 = offsets[c], o1 = offsets[c + 1];
    if (o1 == o0 || cs[CS_COLLIDE * M + c] == 0.0) continue;
    conserve_cell<S, S>(gas, cs, M, c, o0, o1, vcx, vcy, vcz, ver, vvb, base,
                        vvb + (o0 - base), false, seed, step, counters);
  }
  __syncthreads();
  // C: free flight (1D and 2D), state written back once
  for (int64_t i = i0 + threadIdx.x; i < i1; i += UPD_BLOCK) {
    const int64_t j = i - base;
    const S cx = vcx[j], cy = vcy[j], cz = vcz[j], er = ver[j];
    const int lv = vvb[j];
    if (advect && p.cell[i] >= 0) {
      advect_one<S>(g, gas, bc, dt, p, i, cx, cy, cz, er, lv, seed, step, counters);
    } else if (STAGED) {
      p.cx[i] = cx; p.cy[i] = cy; p.cz[i] = cz; p.erot[i] = er; p.vib[i] = (uint8_t)lv;
    }
  }
}

template <typename S>
__global__ __launch_bounds__(UPD_BLOCK, 4) void k_update(GridP g, GasP gas, BcP bc, double dt,
                                                      const double* __restrict__ cs,
                                                      const int64_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ first,
                                                      PartP<S> p, uint64_t seed, uint32_t step,
                                                      int advect, int64_t* counters) {
  constexpr int CAP = UpdCfg<S>::STAGE;
  __shared__ S scx[CAP], scy[CAP], scz[CAP], ser[CAP];
  __shared__ uint8_t svb[CAP];
  __shared__ uint16_t esc_list[CAP];
  __shared__ int nesc;
  const int64_t t = blockIdx.x;
  const int64_t c0 = first[t], c1 = first[t + 1];
  if (c0 >= c1) return;
  const int64_t i0 = offsets[c0], i1 = offsets[c1];
  if (i1 - i0 <= CAP)
    tile_pass<S, true, CAP>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1, scx, scy, scz, ser,
                            svb, i0, esc_list, &nesc, seed, step, advect != 0, counters);
  else
    tile_pass<S, false, CAP>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1, p.cx, p.cy, p.cz,
                             p.erot, p.vib, 0, esc_list, &nesc, seed, step, advect != 0,
                             counters);
}

template <typename S>
hipError_t launch_update(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const double* cs, const int64_t* offsets, const PartP<S>& p,
                         uint64_t seed, uint64_t step, char* ws, const WsLayout& L,
                         int64_t* counters, hipStream_t st) {
  constexpr int T = UpdCfg<S>::TILE;
  const int64_t ntiles = cdiv(p.capacity, T);
  int32_t* first = (int32_t*)(ws + L.tiles);
  k_fill_first<<<cdiv(ntiles + 1, 256), 256, 0, st>>>(first, ntiles + 1, (int32_t)g.M);
  k_tile_first<<<cdiv(g.M + 1, 256), 256, 0, st>>>(offsets, g.M, T, ntiles, first);
  k_update<S><<<ntiles, UPD_BLOCK, 0, st>>>(g, gas, bc, dt, cs, offsets, first, p, seed,
                                            (uint32_t)step, g.dim != 0 ? 1 : 0, counters);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || g.dim == 0) return e;
  return launch_inject<S>(g, gas, bc, dt, p, seed, step, ws, L, counters, st);
}

template hipError_t launch_update<float>(const GridP&, const GasP&, const BcP&, double,
                                         const double*, const int64_t*, const PartP<float>&,
                                         uint64_t, uint64_t, char*, const WsLayout&, int64_t*,
                                         hipStream_t);
template hipError_t launch_update<double>(const GridP&, const GasP&, const BcP&, double,
                                          const double*, const int64_t*, const PartP<double>&,
                                          uint64_t, uint64_t, char*, const WsLayout&, int64_t*,
                                          hipStream_t);

}  // namespace usp
