// usp_batch.hip -- many independent 0D cells advanced several steps per
// launch (the persistent form of the step for dim 0).
//
// In 0D no particle changes cell and no cell reads a neighbour, so a
// workgroup that owns a tile of whole cells can run step after step without
// any grid-wide synchronisation: per step the moments and cell state of its
// cells (16 lanes per cell), the particle update (thread per particle) and
// the conservation (wave per cell), all on an LDS stage that holds the
// tile's velocities, rotational energies and levels from the first step to
// the last.  Tiles larger than the stage run in place in global memory.
// Every phase calls the device functions of the step kernels in the same
// order, so the result is bit-identical to usp_step on the same state.
#include "usp_tile.h"

namespace usp {

template <typename S, bool STAGED, int CAP, int MODE>
__device__ __forceinline__ void batch_tile(const GridP& g, const GasP& gas, double dt,
                                           const double* dt_cell, double* mom, double* cs,
                                           const int64_t* __restrict__ offsets,
                                           const PartP<S>& p, int64_t c0, int64_t c1,
                                           int64_t i0, int64_t i1, const Stage<S>& st,
                                           uint16_t* esc_list, int* nesc, uint64_t seed,
                                           uint64_t step0, int nsteps, int64_t* counters,
                                           unsigned long long* wcnt) {
  // per-particle events of the update go to the workgroup's counts, which
  // are added to the global counters after every step
  const WgCounters wc{counters ? wcnt : nullptr};
  if (STAGED) {
    for (int64_t i = i0 + threadIdx.x; i < i1; i += UPD_BLOCK) st.store(i, load_state(p, i));
    __syncthreads();
  }
  for (int s = 0; s < nsteps; ++s) {
    const uint32_t step = (uint32_t)(step0 + (uint64_t)s);
    tile_cells<S>(g, gas, dt, dt_cell, mom, cs, offsets, c0, c1, st, counters);
    __syncthreads();
    if constexpr (MODE == MODE_CELL) {
      for (int64_t c = c0 + threadIdx.x; c < c1; c += UPD_BLOCK)
        cell_pcoefs(cs, g.M)[c] = cell_pcoef(gas, cs, g.M, c);
      __syncthreads();
    }
    tile_update<S, CAP, true, MODE>(g, gas, cs, p, i0, i1, st, st, esc_list, nesc, seed, step,
                                   wc);
    tile_conserve<S>(gas, cs, g.M, offsets, c0, c1, st, seed, step, counters);
    __syncthreads();
    wg_counters_flush(wcnt, counters);
  }
  if (STAGED) {
    for (int64_t i = i0 + threadIdx.x; i < i1; i += UPD_BLOCK) {
      const PartNew<S> v = st.load(i);
      p.cx[i] = v.cx; p.cy[i] = v.cy; p.cz[i] = v.cz; p.erot[i] = v.erot; p.vib[i] = (uint8_t)v.vib;
    }
  }
}

// CAP = stage size (twice the tile window); WPE = waves per SIMD the
// register budget is held to (what the stage's LDS allows).
template <typename S, int CAP, int WPE, int MODE>
__global__ __launch_bounds__(UPD_BLOCK, WPE) void k_batch(GridP g, GasP gas, double dt,
                                                          const double* dt_cell, double* mom,
                                                          double* cs,
                                                          const int64_t* __restrict__ offsets,
                                                          const int32_t* __restrict__ first,
                                                          const int32_t* __restrict__ order,
                                                          PartP<S> p, uint64_t seed,
                                                          uint64_t step0, int nsteps,
                                                          int64_t* counters) {
  __shared__ S scx[CAP], scy[CAP], scz[CAP], ser[CAP];
  __shared__ uint8_t svb[CAP];
  __shared__ uint16_t esc_list[CAP];
  __shared__ int nesc;
  __shared__ unsigned long long wcnt[USP_NCOUNTERS];
  const int64_t t = order[blockIdx.x];
  const int64_t c0 = first[t], c1 = first[t + 1];
  if (c0 >= c1) return;
  const int64_t i0 = offsets[c0], i1 = offsets[c1];
  wg_counters_init(wcnt);  // ordered before use by the barriers ahead of the first update
  if (i1 - i0 <= CAP) {
    Stage<S> st;
    st.cx = scx; st.cy = scy; st.cz = scz; st.erot = ser; st.vib = svb; st.base = i0;
    batch_tile<S, true, CAP, MODE>(g, gas, dt, dt_cell, mom, cs, offsets, p, c0, c1, i0, i1, st,
                             esc_list, &nesc, seed, step0, nsteps, counters, wcnt);
  } else {
    batch_tile<S, false, CAP, MODE>(g, gas, dt, dt_cell, mom, cs, offsets, p, c0, c1, i0, i1,
                              global_stage(p), esc_list, &nesc, seed, step0, nsteps, counters, wcnt);
  }
}

// Dispatch order of a batched launch: the tiles by descending particle
// count (ties by index), so that the heaviest tiles start first and the
// launch, in which every workgroup keeps its tile for all its steps, does
// not end on a heavy tile started late.  One block, a bitonic sort of
// (count, index) keys in LDS; more than ORDER_MAX tiles keep launch order.
constexpr int ORDER_MAX = 8192;

__global__ __launch_bounds__(1024) void k_tile_order(const int64_t* __restrict__ offsets,
                                                     const int32_t* __restrict__ first,
                                                     int64_t ntiles, int32_t* order) {
  __shared__ unsigned long long key[ORDER_MAX];
  const int n = (int)ntiles;
  if (ntiles > ORDER_MAX) {
    for (int64_t t = threadIdx.x; t < ntiles; t += blockDim.x) order[t] = (int32_t)t;
    return;
  }
  int P = 1;
  while (P < n) P <<= 1;
  for (int t = threadIdx.x; t < P; t += blockDim.x) {
    unsigned long long k = ~0ull;  // padding sorts last
    if (t < n) {
      const int64_t w = offsets[first[t + 1]] - offsets[first[t]];
      const uint32_t wc = w > 0xFFFFFFF0LL ? 0xFFFFFFF0u : (uint32_t)w;
      k = ((unsigned long long)(0xFFFFFFFFu - wc) << 32) | (uint32_t)t;
    }
    key[t] = k;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int t = threadIdx.x; t < P; t += blockDim.x) {
        const int u = t ^ j;
        if (u > t) {
          const unsigned long long a = key[t], b = key[u];
          if ((a > b) == ((t & k) == 0)) {
            key[t] = b;
            key[u] = a;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < n; t += blockDim.x) order[t] = (int32_t)(key[t] & 0xFFFFFFFFull);
}

template <typename S, int TILE, int WPE>
static hipError_t batch_launches(const GridP& g, const GasP& gas, double dt,
                                 const double* dt_cell, double* mom, double* cs,
                                 const int64_t* offsets, const PartP<S>& p, int spl,
                                 uint64_t seed, uint64_t step, int nsteps, int32_t* first,
                                 int64_t* counters, hipStream_t st) {
  const int64_t ntiles = cdiv(p.capacity, TILE);
  hipError_t e = launch_tiles(offsets, g.M, TILE, ntiles, first, st);
  // the order follows first[] in the workspace (sized for 128-slot windows)
  int32_t* order = first + ntiles + 1;
  if (e == hipSuccess) {
    k_tile_order<<<1, 1024, 0, st>>>(offsets, first, ntiles, order);
    e = hipGetLastError();
  }
  for (int s = 0; s < nsteps && e == hipSuccess; s += spl) {
    const int k = nsteps - s < spl ? nsteps - s : spl;
    const int mode = update_mode(gas);
#define USP_K_BATCH(MODE)                                                                     \
  k_batch<S, 2 * TILE, WPE, MODE><<<ntiles, UPD_BLOCK, 0, st>>>(                               \
      g, gas, dt, dt_cell, mom, cs, offsets, first, order, p, seed, step + (uint64_t)s, k, counters)
    if (mode == MODE_FPM) USP_K_BATCH(MODE_FPM);
    else if (mode == MODE_CELL) USP_K_BATCH(MODE_CELL);
    else USP_K_BATCH(MODE_USP);
#undef USP_K_BATCH
    e = hipGetLastError();
  }
  return e;
}

template <typename S>
hipError_t launch_batch(const GridP& g, const GasP& gas, double dt, const double* dt_cell,
                        double* mom, double* cs, const int64_t* offsets, const PartP<S>& p,
                        int tile, int steps_per_launch, uint64_t seed, uint64_t step,
                        int nsteps, char* ws, const WsLayout& L, int64_t* counters,
                        hipStream_t st) {
  int32_t* first = (int32_t*)(ws + L.tiles);
  const int spl = steps_per_launch > 0 ? steps_per_launch : (nsteps > 0 ? nsteps : 1);
  if (nsteps <= 0) return hipSuccess;
  if constexpr (sizeof(S) == 4) {
    if (tile == 512)
      return batch_launches<S, 512, 4>(g, gas, dt, dt_cell, mom, cs, offsets, p, spl, seed, step,
                                       nsteps, first, counters, st);
    if (tile == 2048)
      return batch_launches<S, 2048, 2>(g, gas, dt, dt_cell, mom, cs, offsets, p, spl, seed, step,
                                        nsteps, first, counters, st);
    return batch_launches<S, 1024, 4>(g, gas, dt, dt_cell, mom, cs, offsets, p, spl, seed, step,
                                      nsteps, first, counters, st);
  } else {
    return batch_launches<S, 512, 4>(g, gas, dt, dt_cell, mom, cs, offsets, p, spl, seed, step,
                                     nsteps, first, counters, st);
  }
}

template hipError_t launch_batch<float>(const GridP&, const GasP&, double, const double*, double*,
                                        double*, const int64_t*, const PartP<float>&, int, int,
                                        uint64_t, uint64_t, int, char*, const WsLayout&, int64_t*,
                                        hipStream_t);
template hipError_t launch_batch<double>(const GridP&, const GasP&, double, const double*, double*,
                                         double*, const int64_t*, const PartP<double>&, int, int,
                                         uint64_t, uint64_t, int, char*, const WsLayout&,
                                         int64_t*, hipStream_t);

}  // namespace usp
