// usp_bigcell.hip -- the per-cell reductions of Sec. IV.D for cells far
// larger than a workgroup's share of the chip (a single 0D cell of 1e5
// particles): the moments of Sec. II.A and the conservation of Sec. IV.C
// with each cell's particles split into chunks of CHUNK slots, one wave a
// chunk, and the chunks' partial sums combined in chunk order (the result
// does not depend on the launch).  The picks of the conservation stay the
// sequential draws of the cell (one wave, wave_picks), and the scalings
// are applied by one thread per particle.
#include "usp_cell.h"
#include "usp_particle.h"

namespace usp {

constexpr int CHUNK = BIG_CHUNK;
constexpr int BIG_BLOCK = 256;
constexpr int BIG_WAVES = BIG_BLOCK / 64;
constexpr int NPART = BIG_PARTS;  // partial sums per chunk (moments 20; conservation 6 + lmax)
static_assert(sizeof(ConsScalars) <= CONS_SCALAR_BYTES, "conservation scalar record size");

// chunk_off[c] = first chunk of cell c (cdiv(N_c, CHUNK) chunks each);
// chunk_off[M] = total.  One block: each thread sums a contiguous run of
// cells, then the runs' totals are scanned in LDS.
__global__ __launch_bounds__(256) void k_chunk_offsets(const int64_t* __restrict__ offsets,
                                                       int64_t M, int64_t* chunk_off) {
  __shared__ int64_t run[256];
  const int64_t per = (M + 255) / 256;
  const int64_t c0 = threadIdx.x * per, c1 = c0 + per < M ? c0 + per : M;
  int64_t t = 0;
  for (int64_t c = c0; c < c1; ++c) t += (offsets[c + 1] - offsets[c] + CHUNK - 1) / CHUNK;
  run[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t a = 0;
    for (int k = 0; k < 256; ++k) {
      const int64_t v = run[k];
      run[k] = a;
      a += v;
    }
  }
  __syncthreads();
  int64_t a = run[threadIdx.x];
  for (int64_t c = c0; c < c1; ++c) {
    chunk_off[c] = a;
    a += (offsets[c + 1] - offsets[c] + CHUNK - 1) / CHUNK;
  }
  // the last thread's running sum is the total (threads past M have no cells)
  if (threadIdx.x == 255) chunk_off[M] = a;
}

// The cell of chunk k: the last c with chunk_off[c] <= k (binary search).
__device__ __forceinline__ int64_t chunk_cell(const int64_t* __restrict__ chunk_off, int64_t M,
                                              int64_t k) {
  int64_t lo = 0, hi = M;  // chunk_off[lo] <= k < chunk_off[hi]
  while (hi - lo > 1) {
    const int64_t mid = (lo + hi) >> 1;
    if (chunk_off[mid] <= k) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Moments, first level: wave per chunk, the 20 sums of its slots shifted
// by the cell's first particle, reduced over the wave in a fixed order.
template <typename S>
__global__ __launch_bounds__(BIG_BLOCK) void k_mom_chunks(PartP<S> p,
                                                          const int64_t* __restrict__ offsets,
                                                          const int64_t* __restrict__ chunk_off,
                                                          int64_t M, int64_t nmax, double* part) {
  const int lane = threadIdx.x & 63;
  const int64_t k = (int64_t)blockIdx.x * BIG_WAVES + (threadIdx.x >> 6);
  if (k >= nmax || k >= chunk_off[M]) return;
  const int64_t c = chunk_cell(chunk_off, M, k);
  const int64_t o0 = offsets[c], o1 = offsets[c + 1];
  const int64_t a = o0 + (k - chunk_off[c]) * CHUNK;
  const int64_t b = a + CHUNK < o1 ? a + CHUNK : o1;
  const double r0 = (double)p.cx[o0], r1 = (double)p.cy[o0], r2 = (double)p.cz[o0];
  double s[NPART];
#pragma unroll
  for (int q = 0; q < NPART; ++q) s[q] = 0.0;
  for (int64_t i = a + lane; i < b; i += 64)
    mom_add(mom_load<S>(p.cx, p.cy, p.cz, p.erot, p.vib, i), r0, r1, r2, s);
#pragma unroll
  for (int q = 0; q < NPART; ++q) s[q] = wave_sum(s[q]);
  if (lane < NPART) {
    double w = 0.0;
#pragma unroll
    for (int q = 0; q < NPART; ++q)
      if (q == lane) w = s[q];
    part[k * NPART + lane] = w;
  }
}

// Moments, second level: thread per cell, its chunks' sums in chunk order.
template <typename S>
__global__ void k_mom_cells(PartP<S> p, const int64_t* __restrict__ offsets,
                            const int64_t* __restrict__ chunk_off, int64_t M,
                            const double* __restrict__ part, double* mom) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  const int64_t o0 = offsets[c], N = offsets[c + 1] - o0;
  double s[NPART];
#pragma unroll
  for (int q = 0; q < NPART; ++q) s[q] = 0.0;
  for (int64_t k = chunk_off[c]; k < chunk_off[c + 1]; ++k)
#pragma unroll
    for (int q = 0; q < NPART; ++q) s[q] += part[k * NPART + q];
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (N > 0) { r0 = (double)p.cx[o0]; r1 = (double)p.cy[o0]; r2 = (double)p.cz[o0]; }
  double v[NMOM];
  moments_from_sums(s, N, r0, r1, r2, v);
#pragma unroll
  for (int q = 0; q < NMOM; ++q) mom[q * M + c] = v[q];
}

// Conservation, first level: wave per chunk of a colliding cell, the
// post-collision sums about U^n and the largest level.
template <typename S>
__global__ __launch_bounds__(BIG_BLOCK) void k_cons_chunks(GridP g, const double* __restrict__ cs,
                                                           PartP<S> p,
                                                           const int64_t* __restrict__ offsets,
                                                           const int64_t* __restrict__ chunk_off,
                                                           int64_t nmax, double* part) {
  const int lane = threadIdx.x & 63;
  const int64_t M = g.M;
  const int64_t k = (int64_t)blockIdx.x * BIG_WAVES + (threadIdx.x >> 6);
  if (k >= nmax || k >= chunk_off[M]) return;
  const int64_t c = chunk_cell(chunk_off, M, k);
  if (cs[CS_COLLIDE * M + c] == 0.0) return;
  const int64_t o0 = offsets[c], o1 = offsets[c + 1];
  const int64_t a = o0 + (k - chunk_off[c]) * CHUNK;
  const int64_t b = a + CHUNK < o1 ? a + CHUNK : o1;
  const double Un[3] = {cs[CS_UX * M + c], cs[CS_UY * M + c], cs[CS_UZ * M + c]};
  double s[6] = {0, 0, 0, 0, 0, 0};
  int lmax = 0;
  cons_sums<S>(Un, a + lane, b, 64, p.cx, p.cy, p.cz, p.erot, p.vib, 0, nullptr, o0, false, s,
               &lmax);
#pragma unroll
  for (int q = 0; q < 6; ++q) s[q] = wave_sum(s[q]);
  // the wave's largest level: a fixed butterfly of integer maxima
  int m = lmax;
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(m, off, 64);
    m = o > m ? o : m;
  }
  if (lane < 7) {
    double w = (double)m;
#pragma unroll
    for (int q = 0; q < 6; ++q)
      if (q == lane) w = s[q];
    part[k * NPART + lane] = w;
  }
}

// Conservation, second level: wave per colliding cell, the chunks' sums in
// chunk order, then the picks on the cell's levels (global) and the
// scalars of the scalings.
template <typename S>
__global__ __launch_bounds__(BIG_BLOCK) void k_cons_cells(GridP g, GasP gas,
                                                          const double* __restrict__ cs,
                                                          PartP<S> p,
                                                          const int64_t* __restrict__ offsets,
                                                          const int64_t* __restrict__ chunk_off,
                                                          const double* __restrict__ part,
                                                          ConsScalars* scal, uint64_t seed,
                                                          uint32_t step, int64_t* counters) {
  const int lane = threadIdx.x & 63;
  const int64_t M = g.M;
  const int64_t c = (int64_t)blockIdx.x * BIG_WAVES + (threadIdx.x >> 6);
  if (c >= M) return;
  const int64_t o0 = offsets[c], N = offsets[c + 1] - o0;
  ConsScalars r;
  r.frot = 0.0; r.sc = 0.0; r.moved = 0;
  if (N == 0 || cs[CS_COLLIDE * M + c] == 0.0) {
    if (lane == 0) scal[c] = r;
    return;
  }
  double s[6] = {0, 0, 0, 0, 0, 0};
  double lm = 0.0;
  for (int64_t k = chunk_off[c]; k < chunk_off[c + 1]; ++k) {
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] += part[k * NPART + q];
    lm = fmax(lm, part[k * NPART + 6]);
  }
  r = cons_scalars(gas, cons_in(cs, M, c, step, seed), c, N, s, (int)lm, p.vib + o0, seed, step,
                   counters);
  if (lane == 0) scal[c] = r;
}

// Conservation, the scalings: thread per particle of the binned state.
template <typename S>
__global__ void k_cons_apply(PartP<S> p, const ConsScalars* __restrict__ scal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.count[0]) return;
  const int32_t c = p.cell[i];
  if (c < 0) return;
  const ConsScalars r = scal[c];
  cons_apply<S, S>(r, i, p.cx, p.cy, p.cz, p.erot);
}

template <typename S>
hipError_t launch_moments_split(const GridP& g, const PartP<S>& p, const int64_t* offsets,
                                double* mom, char* ws, const WsLayout& L, hipStream_t st) {
  int64_t* chunk_off = (int64_t*)(ws + L.chunk_off);
  double* part = (double*)(ws + L.chunk_part);
  const int64_t nmax = chunks_max(p.capacity, g.M);
  k_chunk_offsets<<<1, 256, 0, st>>>(offsets, g.M, chunk_off);
  k_mom_chunks<S><<<cdiv(nmax, BIG_WAVES), BIG_BLOCK, 0, st>>>(p, offsets, chunk_off, g.M, nmax,
                                                               part);
  k_mom_cells<S><<<cdiv(g.M, 128), 128, 0, st>>>(p, offsets, chunk_off, g.M, part, mom);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_conserve_split(const GridP& g, const GasP& gas, const double* cs,
                                 const int64_t* offsets, const PartP<S>& p, uint64_t seed,
                                 uint64_t step, char* ws, const WsLayout& L, int64_t* counters,
                                 hipStream_t st) {
  const int64_t* chunk_off = (const int64_t*)(ws + L.chunk_off);  // from the moments
  double* part = (double*)(ws + L.chunk_part);
  ConsScalars* scal = (ConsScalars*)(ws + L.cons_scal);
  const int64_t nmax = chunks_max(p.capacity, g.M);
  k_cons_chunks<S><<<cdiv(nmax, BIG_WAVES), BIG_BLOCK, 0, st>>>(g, cs, p, offsets, chunk_off,
                                                                nmax, part);
  k_cons_cells<S><<<cdiv(g.M, BIG_WAVES), BIG_BLOCK, 0, st>>>(g, gas, cs, p, offsets, chunk_off,
                                                              part, scal, seed, (uint32_t)step,
                                                              counters);
  k_cons_apply<S><<<cdiv(p.capacity, 256), 256, 0, st>>>(p, scal);
  return hipGetLastError();
}

template hipError_t launch_moments_split<float>(const GridP&, const PartP<float>&, const int64_t*,
                                                double*, char*, const WsLayout&, hipStream_t);
template hipError_t launch_moments_split<double>(const GridP&, const PartP<double>&,
                                                 const int64_t*, double*, char*, const WsLayout&,
                                                 hipStream_t);
template hipError_t launch_conserve_split<float>(const GridP&, const GasP&, const double*,
                                                 const int64_t*, const PartP<float>&, uint64_t,
                                                 uint64_t, char*, const WsLayout&, int64_t*,
                                                 hipStream_t);
template hipError_t launch_conserve_split<double>(const GridP&, const GasP&, const double*,
                                                  const int64_t*, const PartP<double>&, uint64_t,
                                                  uint64_t, char*, const WsLayout&, int64_t*,
                                                  hipStream_t);

}  // namespace usp
