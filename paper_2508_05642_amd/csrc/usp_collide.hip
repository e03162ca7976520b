// usp_collide.hip -- kernels of the separate particle-update and
// conservation phases (device functions in usp_particle.h).
#include "usp_particle.h"

namespace usp {

constexpr int PART_BLOCK = 256;
constexpr int CONS_BLOCK = 256;

// One thread per particle.
template <typename S, int MODE>
__global__ __launch_bounds__(PART_BLOCK) void k_collide(GridP g, GasP gas,
                                                        const double* __restrict__ cs, PartP<S> p,
                                                        uint64_t seed, uint32_t step,
                                                        int64_t* counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.count[0]) return;
  const int32_t c = p.cell[i];
  if (c < 0) return;
  uint32_t ev = 0;
  const PartNew<S> o = collide_mode<MODE, S>(g, gas, cs, load_pos(p, i, g.dim), c,
                                             load_state(p, i), seed, step, &ev);
  if (o.changed) {
    p.cx[i] = o.cx; p.cy[i] = o.cy; p.cz[i] = o.cz; p.erot[i] = o.erot;
    p.vib[i] = (uint8_t)o.vib;
  }
  flush_events(counters, ev);
}

// The coefficient chain once per cell (USP_GAMMA_CELL), thread per cell.
__global__ void k_cell_coef(GridP g, GasP gas, double* cs) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= g.M) return;
  cell_pcoefs(cs, g.M)[c] = cell_pcoef(gas, cs, g.M, c);
}

hipError_t launch_cell_coef(const GridP& g, const GasP& gas, double* cs, hipStream_t st) {
  if (update_mode(gas) != MODE_CELL) return hipSuccess;
  k_cell_coef<<<cdiv(g.M, 128), 128, 0, st>>>(g, gas, cs);
  return hipGetLastError();
}

constexpr int CONS_WAVES = CONS_BLOCK / 64;
constexpr int CONS_LDS = 2048;

template <typename S>
__global__ __launch_bounds__(CONS_BLOCK) void k_conserve(GridP g, GasP gas, const double* __restrict__ cs,
                                                         const int64_t* offsets, PartP<S> p,
                                                         uint64_t seed, uint32_t step,
                                                         int64_t* counters) {
  __shared__ uint8_t lv_s[CONS_WAVES][CONS_LDS];
  // the wave's index, made wave-uniform so that the per-cell work of the
  // conservation (loads, draws, integer arithmetic) runs on the scalar unit
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t M = g.M;
  const int64_t c = (int64_t)blockIdx.x * CONS_WAVES + wid;
  if (c >= M) return;
  const int64_t o0 = offsets[c], o1 = offsets[c + 1], N = o1 - o0;
  const ConsIn in = cons_in(cs, M, c, step, seed);
  if (N == 0 || !in.collide) return;
  // levels staged in LDS for the picks (cells up to CONS_LDS particles)
  const bool staged = N <= CONS_LDS;
  conserve_cell<S, S>(gas, in, c, o0, o1, p.cx, p.cy, p.cz, p.erot, p.vib, 0,
                      staged ? lv_s[wid] : p.vib + o0, staged, seed, step, counters);
}

template <typename S>
hipError_t launch_collide(const GridP& g, const GasP& gas, const double* cs, const int64_t* offsets,
                          const PartP<S>& p, uint64_t seed, uint64_t step, int64_t* counters,
                          hipStream_t st) {
  (void)offsets;
  const int64_t nb = cdiv(p.capacity, PART_BLOCK);
  const uint32_t s32 = (uint32_t)step;
  const int mode = update_mode(gas);
  if (mode == MODE_FPM) k_collide<S, MODE_FPM><<<nb, PART_BLOCK, 0, st>>>(g, gas, cs, p, seed, s32, counters);
  else if (mode == MODE_CELL) k_collide<S, MODE_CELL><<<nb, PART_BLOCK, 0, st>>>(g, gas, cs, p, seed, s32, counters);
  else k_collide<S, MODE_USP><<<nb, PART_BLOCK, 0, st>>>(g, gas, cs, p, seed, s32, counters);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_conserve(const GridP& g, const GasP& gas, const double* cs,
                           const int64_t* offsets, const PartP<S>& p, uint64_t seed, uint64_t step,
                           int64_t* counters, hipStream_t st) {
  k_conserve<S><<<cdiv(g.M, CONS_WAVES), CONS_BLOCK, 0, st>>>(g, gas, cs, offsets, p, seed, (uint32_t)step, counters);
  return hipGetLastError();
}

template hipError_t launch_collide<float>(const GridP&, const GasP&, const double*, const int64_t*,
                                          const PartP<float>&, uint64_t, uint64_t, int64_t*,
                                          hipStream_t);
template hipError_t launch_collide<double>(const GridP&, const GasP&, const double*, const int64_t*,
                                           const PartP<double>&, uint64_t, uint64_t, int64_t*,
                                           hipStream_t);
template hipError_t launch_conserve<float>(const GridP&, const GasP&, const double*,
                                           const int64_t*, const PartP<float>&, uint64_t, uint64_t,
                                           int64_t*, hipStream_t);
template hipError_t launch_conserve<double>(const GridP&, const GasP&, const double*,
                                            const int64_t*, const PartP<double>&, uint64_t,
                                            uint64_t, int64_t*, hipStream_t);

}  // namespace usp
