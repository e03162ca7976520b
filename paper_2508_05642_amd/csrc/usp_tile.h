// usp_tile.h -- phases of a tile of whole cells owned by one workgroup:
// the particle update (thread per particle), conservation (wave per cell),
// the free flight (thread per particle), and the per-cell moments and cell
// state (16 lanes per cell).  Used by the fused particle phase and by the
// batched 0D solve; the arithmetic is that of the separate phase kernels
// (the same device functions in the same order).
#pragma once
#include "usp_cell.h"
#include "usp_particle.h"

namespace usp {

constexpr int UPD_BLOCK = 256;
constexpr int UPD_WAVES = UPD_BLOCK / 64;

// Where a tile's velocities, rotational energies and levels live: an LDS
// stage indexed i - base, or the particle arrays themselves (base 0).
template <typename S>
struct Stage {
  S *cx, *cy, *cz, *erot;
  uint8_t* vib;
  int64_t base;
  __device__ __forceinline__ PartNew<S> load(int64_t i) const {
    const int64_t j = i - base;
    PartNew<S> v;
    v.cx = cx[j]; v.cy = cy[j]; v.cz = cz[j]; v.erot = erot[j]; v.vib = vib[j];
    v.changed = false;
    return v;
  }
  __device__ __forceinline__ void store(int64_t i, const PartNew<S>& v) const {
    const int64_t j = i - base;
    cx[j] = v.cx; cy[j] = v.cy; cz[j] = v.cz; erot[j] = v.erot; vib[j] = (uint8_t)v.vib;
  }
};

template <typename S>
__device__ __forceinline__ Stage<S> global_stage(const PartP<S>& p) {
  Stage<S> s;
  s.cx = p.cx; s.cy = p.cy; s.cz = p.cz; s.erot = p.erot; s.vib = p.vib; s.base = 0;
  return s;
}

// First and second pass of the particle update (MODE_*): in FP32 the
// first pass of the per-particle chain flags the particles that need the
// FP64 chain (see collide_f32); the FP64 state, the first-order FPM method
// and the cell's chain have a single pass.
template <int MODE>
__device__ __forceinline__ PartNew<float> update_first(const GridP& g, const GasP& gas,
                                                      const double* cs, const PartPos<float>& q,
                                                      int32_t c, const PartNew<float>& in,
                                                      uint64_t seed, uint32_t step, uint32_t* ev,
                                                      bool* esc) {
  if constexpr (MODE == MODE_CELL) {
    *esc = false;
    return collide_cell<float>(g, gas, cs, q, c, in, seed, step, ev);
  } else {
    return collide_f32<MODE == MODE_FPM>(g, gas, cs, q, c, in, seed, step, ev, esc);
  }
}
template <int MODE>
__device__ __forceinline__ PartNew<double> update_first(const GridP& g, const GasP& gas,
                                                       const double* cs, const PartPos<double>& q,
                                                       int32_t c, const PartNew<double>& in,
                                                       uint64_t seed, uint32_t step, uint32_t* ev,
                                                       bool* esc) {
  *esc = false;
  return collide_mode<MODE, double>(g, gas, cs, q, c, in, seed, step, ev);
}
__device__ __forceinline__ PartNew<float> update_second(const GridP& g, const GasP& gas,
                                                       const double* cs, const PartPos<float>& q,
                                                       int32_t c, const PartNew<float>& in,
                                                       uint64_t seed, uint32_t step,
                                                       uint32_t* ev) {
  return collide_esc(g, gas, cs, q, c, in, seed, step, ev);
}
__device__ __forceinline__ PartNew<double> update_second(const GridP&, const GasP&, const double*,
                                                        const PartPos<double>&, int32_t,
                                                        const PartNew<double>&, uint64_t,
                                                        uint32_t, uint32_t*) {
  PartNew<double> o;
  o.changed = false;
  return o;
}

// Particle update of [i0, i1): inputs from src, results to dst (unchanged
// particles are copied unless src and dst are the same storage, SAME).  In
// chunks of CAP particles: first pass thread per particle; the particles
// it lists (esc_list/nesc, LDS) get the second pass.  Positions and ids
// are read from p.
template <typename S, int CAP, bool SAME, int MODE, typename CNT>
__device__ __forceinline__ void tile_update(const GridP& g, const GasP& gas,
                                            const double* __restrict__ cs, const PartP<S>& p,
                                            int64_t i0, int64_t i1, const Stage<S>& src,
                                            const Stage<S>& dst, uint16_t* esc_list, int* nesc,
                                            uint64_t seed, uint32_t step, CNT counters) {
  for (int64_t cb = i0; cb < i1; cb += CAP) {
    const int64_t ce = cb + CAP < i1 ? cb + CAP : i1;
    if (threadIdx.x == 0) *nesc = 0;
    __syncthreads();
    for (int64_t i = cb + threadIdx.x; i < ce; i += UPD_BLOCK) {
      const int32_t c = p.cell[i];
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
      if (c >= 0)
        o = update_first<MODE>(gl, gas, csl, load_pos(p, i, g.dim), c, in, seed, step, &ev, &esc);
      if (esc) esc_list[atomicAdd(nesc, 1)] = (uint16_t)(i - cb);
      else if (o.changed) dst.store(i, o);
      else if (!SAME) dst.store(i, in);
      flush_events(counters, ev);
    }
    __syncthreads();
    const int ne = *nesc;
    for (int k = threadIdx.x; k < ne; k += UPD_BLOCK) {
      const int64_t i = cb + esc_list[k];
      const PartNew<S> in = src.load(i);
      uint32_t ev = 0;
      const PartNew<S> o = update_second(g, gas, cs, load_pos(p, i, g.dim), p.cell[i], in, seed,
                                         step, &ev);
      if (o.changed) dst.store(i, o);
      else if (!SAME) dst.store(i, in);
      flush_events(counters, ev);
    }
    __syncthreads();
  }
}

// Conservation of the cells [c0, c1), wave per cell, on st.
template <typename S>
__device__ __forceinline__ void tile_conserve(const GasP& gas, const double* __restrict__ cs,
                                              int64_t M, const int64_t* __restrict__ offsets,
                                              int64_t c0, int64_t c1, const Stage<S>& st,
                                              uint64_t seed, uint32_t step, int64_t* counters) {
  // the wave's index, made wave-uniform so that the per-cell work of the
  // conservation (loads, draws, integer arithmetic) runs on the scalar unit
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (int64_t c = c0 + wid; c < c1; c += UPD_WAVES) {
    const int64_t o0 = offsets[c], o1 = offsets[c + 1];
    const ConsIn in = cons_in(cs, M, c, step, seed);
    if (o1 == o0 || !in.collide) continue;
    conserve_cell<S, S>(gas, in, c, o0, o1, st.cx, st.cy, st.cz, st.erot, st.vib, st.base,
                        st.vib + (o0 - st.base), false, seed, step, counters);
  }
}

// Moments and cell state of the cells [c0, c1) from st, 16 lanes per cell
// (each row of 16 lanes takes every 16th cell); the planes and records go
// to mom and cs.
template <typename S>
__device__ __forceinline__ void tile_cells(const GridP& g, const GasP& gas, double dt,
                                           const double* dt_cell, double* mom, double* cs,
                                           const int64_t* __restrict__ offsets, int64_t c0,
                                           int64_t c1, const Stage<S>& st, int64_t* counters) {
  const int row = threadIdx.x / MOM_LANES, sub = threadIdx.x & (MOM_LANES - 1);
  const int64_t M = g.M;
  for (int64_t c = c0 + row; c < c1; c += UPD_BLOCK / MOM_LANES) {
    const int64_t o0 = offsets[c] - st.base, o1 = offsets[c + 1] - st.base;
    double v[NMOM];
    row_moments<S>(st.cx, st.cy, st.cz, st.erot, st.vib, o0, o1, sub, v);
    store_moments(mom, M, c, sub, v);
    if (sub == 0) {
      double w[NCS];
      cell_state(g, gas, v, c, dt_cell ? dt_cell[c] : dt, w, counters);
      store_cell_state(cs, M, c, w);
    }
  }
}

}  // namespace usp
