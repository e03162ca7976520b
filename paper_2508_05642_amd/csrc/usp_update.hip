// usp_update.hip -- the particle phase of a step in one pass over a binned
// state: the particle update (Secs. III.A-III.B), the conservation scheme
// (Sec. IV.C) and the free flight with boundaries.
//
// A workgroup of 8 waves owns a tile: the cells whose first particle lies
// in one window of particle slots (so whole cells; the window is sized from
// the mean particles per cell by update_tile).  A gathering launch first loads
// the tile's particles through the bin's permutation into LDS: velocities,
// rotational energy and level, and also position, id and new cell, so that
// the later phases touch global memory only for the cell records and the
// final write.  Three phases separated by workgroup barriers:
//   A  particle update, one thread per particle, into the LDS stage;
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
__device__ __forceinline__ int64_t tile_window(const int64_t* __restrict__ offsets, int64_t M,
                                               int64_t T, int stage) {
  return stage > 0 ? update_tile(stage, offsets[M], M) : T;
}

__device__ __forceinline__ void tile_first(const int64_t* __restrict__ offsets, int64_t T,
                                           int64_t ntiles, int32_t* first, int64_t c) {
  const int64_t lo = c == 0 ? 0 : offsets[c - 1] / T + 1;
  int64_t hi = offsets[c] / T;
  if (hi > ntiles) hi = ntiles;
  for (int64_t t = lo; t <= hi; ++t) first[t] = (int32_t)c;
}

__global__ void k_tile_first(const int64_t* __restrict__ offsets, int64_t M, int64_t T,
                             int64_t ntiles, int32_t* first, int stage) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c <= M) tile_first(offsets, tile_window(offsets, M, T, stage), ntiles, first, c);
}

// Both passes in one block for grids of at most TILES_SMALL cells and tiles
// (launch-bound steps); the barrier orders the fill before the starts.
constexpr int64_t TILES_SMALL = 4096;
__global__ __launch_bounds__(256) void k_tiles_small(const int64_t* __restrict__ offsets, int64_t M,
                                                     int64_t T, int64_t ntiles, int32_t* first,
                                                     int stage) {
  for (int64_t t = threadIdx.x; t <= ntiles; t += blockDim.x) first[t] = (int32_t)M;
  __syncthreads();
  const int64_t W = tile_window(offsets, M, T, stage);
  for (int64_t c = threadIdx.x; c <= M; c += blockDim.x) tile_first(offsets, W, ntiles, first, c);
}

// The fused kernel's workgroup: 8 waves, two workgroups per CU (their LDS
// stages fill it), 4 waves per SIMD.
constexpr int KU_BLOCK = 512;
constexpr int KU_WAVES = KU_BLOCK / 64;

// Positions, ids and new cells of a gathered tile's slots, in LDS next to
// the stage (slot i at i - base): the update and the flight read them there
// instead of from the output arrays.
template <typename S>
struct PosStage {
  S *x, *y;
  uint32_t* pid;
  int32_t* cell;
  int64_t base;
  __device__ __forceinline__ PartPos<S> load(int64_t i) const {
    const int64_t j = i - base;
    PartPos<S> q;
    q.x = x[j]; q.y = y[j]; q.pid = pid[j];
    return q;
  }
};

// Gather prologue of a tile (G): slot i takes particle perm[i] of src;
// velocities, rotational energy and level go to the stage; positions, ids
// and the slot's new cell (set by the gathering bin in p) go to the LDS
// position stage (POS) or, for a tile past the stage, positions and ids to
// p.  Each thread loads GATHER_U slots' indices (and cells), then all
// their fields, then stores them, so that many scattered loads are in
// flight at once.
constexpr int GATHER_U = 4;

template <typename S, bool POS>
__device__ __forceinline__ void tile_gather(const GridP& g, const PartP<S>& src,
                                            const uint32_t* __restrict__ perm, const PartP<S>& p,
                                            int64_t i0, int64_t i1, const Stage<S>& st,
                                            const PosStage<S>& ps) {
  for (int64_t b = i0 + threadIdx.x; b < i1; b += GATHER_U * KU_BLOCK) {
    uint32_t j[GATHER_U];
    int32_t cl[GATHER_U];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) {
      const int64_t i = b + k * KU_BLOCK;
      j[k] = i < i1 ? perm[i] : 0u;
      if (POS) cl[k] = i < i1 ? p.cell[i] : 0;
    }
    // every lane loads all GATHER_U slots, array by array (a slot past the
    // tile reads particle 0, in bounds, and stores nothing): no load waits
    // on a per-slot branch, and each array's base address is fetched once
    PartNew<S> v[GATHER_U];
    S xs[GATHER_U], ys[GATHER_U];
    uint32_t id[GATHER_U];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) v[k].cx = src.cx[j[k]];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) v[k].cy = src.cy[j[k]];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) v[k].cz = src.cz[j[k]];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) v[k].erot = src.erot[j[k]];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) v[k].vib = src.vib[j[k]];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) {
      v[k].changed = false;
      xs[k] = S(0);
      ys[k] = S(0);
    }
    if (g.dim == 2) {
#pragma unroll
      for (int k = 0; k < GATHER_U; ++k) xs[k] = src.x[j[k]];
    }
    if (g.dim >= 1) {
#pragma unroll
      for (int k = 0; k < GATHER_U; ++k) ys[k] = src.y[j[k]];
    }
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) id[k] = src.pid[j[k]];
#pragma unroll
    for (int k = 0; k < GATHER_U; ++k) {
      const int64_t i = b + k * KU_BLOCK;
      if (i < i1) {
        st.store(i, v[k]);
        if (POS) {
          const int64_t l = i - ps.base;
          ps.x[l] = xs[k]; ps.y[l] = ys[k]; ps.pid[l] = id[k]; ps.cell[l] = cl[k];
        } else {
          if (g.dim == 2) p.x[i] = xs[k];
          if (g.dim >= 1) p.y[i] = ys[k];
          p.pid[i] = id[k];
        }
      }
    }
  }
  __syncthreads();
}

// The three phases of one tile; st = LDS stage or the particle arrays.
// With G the stage (or, for a tile past the stage, the arrays of p) was
// filled by the gather prologue, so phase A updates it in place; with POS
// the positions, ids and cells are read from the LDS position stage.
//   A  particle update, thread per particle, into the stage (the particles
//      the FP32 first pass lists get the FP64 second pass);
//   B  conservation, wave per cell, on the stage;
//   C  free flight, thread per particle, writing the state once.
template <typename S, bool STAGED, int CAP, int MODE, bool G, bool POS>
__device__ __forceinline__ void tile_pass(const GridP& g, const GasP& gas, const BcP& bc,
                                          double dt, const double* __restrict__ cs,
                                          const int64_t* __restrict__ offsets, const PartP<S>& p,
                                          int64_t c0, int64_t c1, int64_t i0, int64_t i1,
                                          const Stage<S>& st, const PosStage<S>& ps,
                                          uint16_t* esc_list, int* nesc, uint64_t seed,
                                          uint32_t step, bool advect, int64_t* counters,
                                          WgCounters wc) {
  // A: inputs from the stage the gather filled, or from the arrays of p
  // (in place when the tile is past the stage)
  constexpr bool SAME = !STAGED || G;
  const Stage<S> src = (G && STAGED) ? st : global_stage(p);
  for (int64_t cb = i0; cb < i1; cb += CAP) {
    const int64_t ce = cb + CAP < i1 ? cb + CAP : i1;
    if (threadIdx.x == 0) *nesc = 0;
    __syncthreads();
    for (int64_t i = cb + threadIdx.x; i < ce; i += KU_BLOCK) {
      const int32_t c = POS ? ps.cell[i - ps.base] : p.cell[i];
      const PartNew<S> in = src.load(i);
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
      if (c >= 0) {
        const PartPos<S> q = POS ? ps.load(i) : load_pos(p, i, g.dim);
        o = update_first<MODE>(gl, gas, csl, q, c, in, seed, step, &ev, &esc);
      }
      if (esc) esc_list[atomicAdd(nesc, 1)] = (uint16_t)(i - cb);
      else if (o.changed) st.store(i, o);
      else if (!SAME) st.store(i, in);
      flush_events(wc, ev);
    }
    __syncthreads();
    const int ne = *nesc;
    for (int k = threadIdx.x; k < ne; k += KU_BLOCK) {
      const int64_t i = cb + esc_list[k];
      const PartNew<S> in = src.load(i);
      uint32_t ev = 0;
      const PartPos<S> q = POS ? ps.load(i) : load_pos(p, i, g.dim);
      const int32_t c = POS ? ps.cell[i - ps.base] : p.cell[i];
      const PartNew<S> o = update_second(g, gas, cs, q, c, in, seed, step, &ev);
      if (o.changed) st.store(i, o);
      else if (!SAME) st.store(i, in);
      flush_events(wc, ev);
    }
    __syncthreads();
  }
  // B: conservation, wave per cell
  // the wave's index, made wave-uniform so that the per-cell work of the
  // conservation (loads, draws, integer arithmetic) runs on the scalar unit
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t c = c0 + wid; c < c1; c += KU_WAVES) {
    const int64_t o0 = offsets[c], o1 = offsets[c + 1];
    const ConsIn in = cons_in(cs, g.M, c, step, seed);
    if (o1 == o0 || !in.collide) continue;
    conserve_cell<S, S>(gas, in, c, o0, o1, st.cx, st.cy, st.cz, st.erot, st.vib, st.base,
                        st.vib + (o0 - st.base), false, seed, step, counters);
  }
  __syncthreads();
  // C: free flight (1D and 2D), state written back once
  for (int64_t i = i0 + threadIdx.x; i < i1; i += KU_BLOCK) {
    const PartNew<S> v = st.load(i);
    const int32_t c = POS ? ps.cell[i - ps.base] : p.cell[i];
    if (advect && c >= 0) {
      const PartPos<S> q = POS ? ps.load(i) : load_pos(p, i, g.dim);
      advect_one<S, POS>(g, gas, bc, dt, p, i, q, v.cx, v.cy, v.cz, v.erot, v.vib, seed, step,
                         wc);
    } else if (STAGED) {
      p.cx[i] = v.cx; p.cy[i] = v.cy; p.cz[i] = v.cz; p.erot[i] = v.erot; p.vib[i] = (uint8_t)v.vib;
      if (POS) {
        const PartPos<S> q = ps.load(i);
        if (g.dim == 2) p.x[i] = q.x;
        if (g.dim >= 1) p.y[i] = q.y;
        p.pid[i] = q.pid;
      }
    }
  }
}

template <typename S, int MODE, bool G>
__global__ __launch_bounds__(KU_BLOCK, 4) void k_update(GridP g, GasP gas, BcP bc, double dt,
                                                     const double* __restrict__ cs,
                                                     const int64_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ first,
                                                     PartP<S> p, uint64_t seed, uint32_t step,
                                                     int advect, int64_t* counters, PartP<S> src,
                                                     const uint32_t* __restrict__ perm) {
  constexpr int CAP = UpdCfg<S>::STAGE;
  constexpr int PCAP = G ? CAP : 1;
  __shared__ S scx[CAP], scy[CAP], scz[CAP], ser[CAP];
  __shared__ uint8_t svb[CAP];
  __shared__ uint16_t esc_list[CAP];
  __shared__ S spx[PCAP], spy[PCAP];
  __shared__ uint32_t spid[PCAP];
  __shared__ int32_t scell[PCAP];
  __shared__ int nesc;
  __shared__ unsigned long long wcnt[USP_NCOUNTERS];
  const int64_t t = blockIdx.x;
  const int64_t c0 = first[t], c1 = first[t + 1];
  if (c0 >= c1) return;
  const int64_t i0 = offsets[c0], i1 = offsets[c1];
  wg_counters_init(wcnt);  // ordered before use by the first barrier of A
  const WgCounters wc{counters ? wcnt : nullptr};
  PosStage<S> ps;
  ps.x = spx; ps.y = spy; ps.pid = spid; ps.cell = scell; ps.base = i0;
  if (i1 - i0 <= CAP) {
    Stage<S> st;
    st.cx = scx; st.cy = scy; st.cz = scz; st.erot = ser; st.vib = svb; st.base = i0;
    if constexpr (G) {
      tile_gather<S, true>(g, src, perm, p, i0, i1, st, ps);
      tile_pass<S, true, CAP, MODE, G, true>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1, st, ps,
                                            esc_list, &nesc, seed, step, advect != 0, counters,
                                            wc);
    } else {
      tile_pass<S, true, CAP, MODE, G, false>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1, st,
                                             ps, esc_list, &nesc, seed, step, advect != 0,
                                             counters, wc);
    }
  } else {
    if constexpr (G) tile_gather<S, false>(g, src, perm, p, i0, i1, global_stage(p), ps);
    tile_pass<S, false, CAP, MODE, G, false>(g, gas, bc, dt, cs, offsets, p, c0, c1, i0, i1,
                                            global_stage(p), ps, esc_list, &nesc, seed, step,
                                            advect != 0, counters, wc);
  }
  __syncthreads();
  wg_counters_flush(wcnt, counters);
}

hipError_t launch_tiles(const int64_t* offsets, int64_t M, int64_t T, int64_t ntiles,
                        int32_t* first, hipStream_t st, int stage) {
  if (M < TILES_SMALL && ntiles < TILES_SMALL) {
    k_tiles_small<<<1, 256, 0, st>>>(offsets, M, T, ntiles, first, stage);
    return hipGetLastError();
  }
  k_fill_first<<<cdiv(ntiles + 1, 256), 256, 0, st>>>(first, ntiles + 1, (int32_t)M);
  k_tile_first<<<cdiv(M + 1, 256), 256, 0, st>>>(offsets, M, T, ntiles, first, stage);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_update(const GridP& g, const GasP& gas, const BcP& bc, double dt,
                         const double* cs, const int64_t* offsets, const PartP<S>& p,
                         uint64_t seed, uint64_t step, char* ws, const WsLayout& L,
                         int64_t* counters, hipStream_t st, const PartP<S>* src,
                         const uint32_t* gather_perm, hipEvent_t ev_begin, hipEvent_t ev_end) {
  // the launch covers a full state; the window itself comes from the
  // binned count on the device
  const int64_t T = update_tile(UpdCfg<S>::STAGE, p.capacity, g.M);
  const int64_t ntiles = cdiv(p.capacity, T);
  int32_t* first = (int32_t*)(ws + L.tiles);
  if (launch_tiles(offsets, g.M, T, ntiles, first, st, UpdCfg<S>::STAGE) != hipSuccess)
    return hipGetLastError();
  const uint32_t s32 = (uint32_t)step;
  const int adv = g.dim != 0 ? 1 : 0;
  const int mode = update_mode(gas);
  const PartP<S> sp = src ? *src : p;
  if (ev_begin && hipEventRecord(ev_begin, st) != hipSuccess) return hipGetLastError();
#define USP_K_UPDATE(MODE, G, PERM)                                                             \
  k_update<S, MODE, G><<<ntiles, KU_BLOCK, 0, st>>>(g, gas, bc, dt, cs, offsets, first, p, seed, \
                                                   s32, adv, counters, sp, PERM)
  if (gather_perm) {
    if (mode == MODE_FPM) USP_K_UPDATE(MODE_FPM, true, gather_perm);
    else if (mode == MODE_CELL) USP_K_UPDATE(MODE_CELL, true, gather_perm);
    else USP_K_UPDATE(MODE_USP, true, gather_perm);
  } else {
    if (mode == MODE_FPM) USP_K_UPDATE(MODE_FPM, false, nullptr);
    else if (mode == MODE_CELL) USP_K_UPDATE(MODE_CELL, false, nullptr);
    else USP_K_UPDATE(MODE_USP, false, nullptr);
  }
#undef USP_K_UPDATE
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
