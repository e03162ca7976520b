// usp_update.hip -- the particle phase of a step in one pass over a binned
// state: the particle update (Secs. III.A-III.B), the conservation scheme
// (Sec. IV.C) and the free flight with boundaries.
//
// A workgroup owns a tile: the cells whose first particle lies in one
// window of particle slots (so whole cells; the window is sized from the
// mean slots per cell by update_tile).  A gathering launch first loads the
// tile's particles through the bin's permutation.  Three phases separated
// by workgroup barriers:
//   A  particle update, one thread per particle, into an LDS stage;
//   B  conservation, one wave per cell, on the stage;
//   C  free flight, one thread per particle, from the stage; the state is
//      written to HBM once.
// Tiles with more particles than the stage holds run the same phases in
// place in global memory.  The arithmetic is that of the separate phase
// kernels (shared device functions), in the same order, so the result is
// bit-identical to running them one after the other.
#include "usp_tile.h"

namespace usp {

template <typename S> struct UpdCfg;
template <> struct UpdCfg<float> { static constexpr int STAGE = UPDATE_STAGE_F32; };
template <> struct UpdCfg<double> { static constexpr int STAGE = UPDATE_STAGE_F64; };

__global__ void k_fill_first(int32_t* first, int64_t n, int32_t v) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) first[t] = v;
}

// first[t] = the smallest cell c with offsets[c] >= t * T (tiles past the
// last particle keep the prefilled M): cell c owns the tiles t with
// offsets[c-1] < t T <= offsets[c].
__device__ __forceinline__ void tile_first(const int64_t* __restrict__ offsets, int64_t T,
                                           int64_t ntiles, int32_t* first, int64_t c) {
  const int64_t lo = c == 0 ? 0 : offsets[c - 1] / T + 1;
  int64_t hi = offsets[c] / T;
  if (hi > ntiles) hi = ntiles;
  for (int64_t t = lo; t <= hi; ++t) first[t] = (int32_t)c;
}

__global__ void k_tile_first(const int64_t* __restrict__ offsets, int64_t M, int64_t T,
                             int64_t ntiles, int32_t* first) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= M) tile_first(offsets, T, ntiles, first, c);
}

// Both passes in one block for grids of at most TILES_SMALL cells and tiles
// (launch-bound steps); the barrier orders the fill before the starts.
constexpr int64_t TILES_SMALL = 4096;
__global__ __launch_bounds__(256) void k_tiles_small(const int64_t* __restrict__ offsets, int64_t M,
                                                     int64_t T, int64_t ntiles, int32_t* first) {
  for (int64_t t = threadIdx.x; t <= ntiles; t += blockDim.x) first[t] = (int32_t)M;
  __syncthreads();
  for (int64_t c = threadIdx.x; c <= M; c += blockDim.x) tile_first(offsets, T, ntiles, first, c);
}

// The three phases of one tile; st = LDS stage or the particle arrays.
// With G the stage (or, for a tile past the stage, the arrays of p) was
// filled by the gather prologue, so phase A updates it in place.
template <typename S, bool STAGED, int CAP, bool FPM, bool G>
__device__ __forceinline__ void tile_pass(const GridP& g, const GasP& gas, const BcP& bc,
                                          double dt, const double* __restrict__ cs,
                                          const int64_t* __restrict__ offsets, const PartP<S>& p,
                                          int64_t c0, int64_t c1, int64_t i0, int64_t i1,
                                          const Stage<S>& st, uint16_t* esc_list, int* nesc,
                                          uint64_t seed, uint32_t step, bool advect,
                                          int64_t* counters, WgCounters wc) {
  // A: particle update, global inputs into the stage (or in place); the
  // per-particle events of A and C go to the workgroup's counts
  if constexpr (G && STAGED)
    tile_update<S, CAP, true, FPM>(g, gas, cs, p, i0, i1, st, st, esc_list, nesc, seed, step, wc);
  else
    tile_update<S, CAP, !STAGED, FPM>(g, gas, cs, p, i0, i1, global_stage(p), st, esc_list, nesc,
                                      seed, step, wc);
  // B: conservation, wave per cell
  tile_conserve<S>(gas, cs, g.M, offsets, c0, c1, st, seed, step, counters);
  __syncthreads();
  // C: free flight (1D and 2D), state written back once
  for (int64_t i = i0 + threadIdx.x; i < i1; i += UPD_BLOCK) {
    const PartNew<S> v = st.load(i);
    if (advect && p.cell[i] >= 0) {
      advect_one<S>(g, gas, bc, dt, p, i, v.cx, v.cy, v.cz, v.erot, v.vib, seed, step, wc);
    } else if (STAGED) {
      p.cx[i] = v.cx; p.cy[i] = v.cy; p.cz[i] = v.cz; p.erot[i] = v.erot; p.vib[i] = (uint8_t)v.vib;
    }
  }
}

// Gather prologue of a tile (G): slot i takes particle perm[i] of src;
// velocities, rotational energy and level go to the stage, positions and
// ids to p (p's cells were set by the gathering bin).  Each thread loads
// GATHER_U slots' indices, then all their fields, then stores them, so
// that many scattered loads are in flight at once.
constexpr int GATHER_U = 4;

template <typename S>
__device__ __forceinline__ void tile_gather(const GridP& g, const PartP<S>& src,
                                            const uint32_t* __restrict__ perm, const PartP<S>& p,
                                            int64_t i0, int64_t i1, const Stage<S>& st) {
  for (int64_t b = i0 + threadIdx.x; b < i1; b += GATHER_U * UPD_BLOCK) {
    uint32_t j[GATHER_U];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) {
      const int64_t i = b + k * UPD_BLOCK;
      j[k] = i < i1 ? perm[i] : 0u;
    }
    PartNew<S> v[GATHER_U];
    S xs[GATHER_U], ys[GATHER_U];
    uint32_t id[GATHER_U];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) {
      if (b + k * UPD_BLOCK < i1) {
        v[k] = load_state(src, j[k]);
        xs[k] = g.dim == 2 ? src.x[j[k]] : S(0);
        ys[k] = g.dim >= 1 ? src.y[j[k]] : S(0);
        id[k] = src.pid[j[k]];
      }
    }
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) {
      const int64_t i = b + k * UPD_BLOCK;
      if (i < i1) {
        st.store(i, v[k]);
        if (g.dim == 2) p.x[i] = xs[k];
        if (g.dim >= 1) p.y[i] = ys[k];
        p.pid[i] = id[k];
      }
    }
  }
  __syncthreads();
}

template <typename S, bool FPM, bool G>
__global__ __launch_bounds__(UPD_BLOCK, 4) void k_update(GridP g, GasP gas, BcP bc, double dt,
                                                      const double* __restrict__ cs,
                                                      const int64_t* __restrict__ offsets,
                                                      const int32_t* __restrict__ first,
                                                      PartP<S> p, uint64_t seed, uint32_t step,
                                                      int advect, int64_t* counters, PartP<S> src,
                                                      const uint32_t* __restrict__ perm) {
  constexpr int CAP = UpdCfg<S>::STAGE;
  __shared__ S scx[CAP], scy[CAP], scz[CAP], ser[CAP];
  __shared__ uint8_t svb[CAP];
  __shared__ uint16_t esc_list[CAP];
  __shared__ int nesc;
  __shared__ unsigned long long wcnt[USP_NCOUNTERS];
  const int64_t t = blockIdx.x;
  const int64_t c0 = first[t], c1 = first[t + 1];
  if (c0 >= c1) return;
  const int64_t i0 = offsets[c0], i1 = offsets[c1];
  wg_counters_init(wcnt);  // ordered before use by the first barrier of A
  const WgCounters wc{counters ? wcnt : nullptr};
  if (i1 - i0 <= CAP) {
    Stage<S> st;
    st.cx = scx; st.cy = scy; st.cz = scz; st.erot = ser; st.vib = svb; st.base = i0;
    if constexpr (G) tile_gather<S>(g, src, perm, p, i0, i1, st);
    tile_pass<S, true, CAP, FPM, G>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1, st, esc_list,
                                    &nesc, seed, step, advect != 0, counters, wc);
  } else {
    if constexpr (G) tile_gather<S>(g, src, perm, p, i0, i1, global_stage(p));
    tile_pass<S, false, CAP, FPM, G>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1,
                                     global_stage(p), esc_list, &nesc, seed, step, advect != 0,
                                     counters, wc);
  }
  __syncthreads();
  wg_counters_flush(wcnt, counters);
}

hipError_t launch_tiles(const int64_t* offsets, int64_t M, int64_t T, int64_t ntiles,
                        int32_t* first, hipStream_t st) {
  if (M < TILES_SMALL && ntiles < TILES_SMALL) {
    k_tiles_small<<<1, 256, 0, st>>>(offsets, M, T, ntiles, first);
    return hipGetLastError();
  }
  k_fill_first<<<cdiv(ntiles + 1, 256), 256, 0, st>>>(first, ntiles + 1, (int32_t)M);
  k_tile_first<<<cdiv(M + 1, 256), 256, 0, st>>>(offsets, M, T, ntiles, first);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_update(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const double* cs, const int64_t* offsets, const PartP<S>& p,
                         uint64_t seed, uint64_t step, char* ws, const WsLayout& L,
                         int64_t* counters, hipStream_t st, const PartP<S>* src,
                         const uint32_t* gather_perm, hipEvent_t ev_begin, hipEvent_t ev_end) {
  const int64_t T = update_tile(UpdCfg<S>::STAGE, p.capacity, g.M);
  const int64_t ntiles = cdiv(p.capacity, T);
  int32_t* first = (int32_t*)(ws + L.tiles);
  if (launch_tiles(offsets, g.M, T, ntiles, first, st) != hipSuccess) return hipGetLastError();
  const uint32_t s32 = (uint32_t)step;
  const int adv = g.dim != 0 ? 1 : 0;
  const bool fpm = gas.scheme == USP_SCHEME_FPM;
  const PartP<S> sp = src ? *src : p;
  if (ev_begin && hipEventRecord(ev_begin, st) != hipSuccess) return hipGetLastError();
  if (gather_perm && fpm)
    k_update<S, true, true><<<ntiles, UPD_BLOCK, 0, st>>>(g, gas, bc, dt, cs, offsets, first, p, seed,
                                                          s32, adv, counters, sp, gather_perm);
  else if (gather_perm)
    k_update<S, false, true><<<ntiles, UPD_BLOCK, 0, st>>>(g, gas, bc, dt, cs, offsets, first, p, seed,
                                                           s32, adv, counters, sp, gather_perm);
  else if (fpm)
    k_update<S, true, false><<<ntiles, UPD_BLOCK, 0, st>>>(g, gas, bc, dt, cs, offsets, first, p, seed,
                                                           s32, adv, counters, sp, nullptr);
  else
    k_update<S, false, false><<<ntiles, UPD_BLOCK, 0, st>>>(g, gas, bc, dt, cs, offsets, first, p,
                                                            seed, s32, adv, counters, sp, nullptr);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && ev_end) e = hipEventRecord(ev_end, st);
  if (e != hipSuccess || g.dim == 0) return e;
  return launch_inject<S>(g, gas, bc, dt, p, seed, step, ws, L, counters, st);
}

template hipError_t launch_update<float>(const GridP&, const GasP&, const BcP&, double,
                                         const double*, const int64_t*, const PartP<float>&,
                                         uint64_t, uint64_t, char*, const WsLayout&, int64_t*,
                                         hipStream_t, const PartP<float>*, const uint32_t*,
                                         hipEvent_t, hipEvent_t);
template hipError_t launch_update<double>(const GridP&, const GasP&, const BcP&, double,
                                          const double*, const int64_t*, const PartP<double>&,
                                          uint64_t, uint64_t, char*, const WsLayout&, int64_t*,
                                          hipStream_t, const PartP<double>*, const uint32_t*,
                                          hipEvent_t, hipEvent_t);

}  // namespace usp
