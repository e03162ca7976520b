// usp_moments.hip -- per-cell moments and the per-cell USP-FPM state.
#include "usp_cell.h"

namespace usp {

constexpr int CELL_BLOCK = 256;

// 16 lanes per cell, four cells per wave (every lane stays active for the
// row permutes; lanes of cells past M carry zeros).
template <typename S, bool G>
__global__ __launch_bounds__(CELL_BLOCK) void k_moments(GridP g, PartP<S> p, const int64_t* offsets,
                                                        double* mom, const uint32_t* perm) {
  const int64_t M = g.M;
  const int64_t c = ((int64_t)blockIdx.x * CELL_BLOCK + threadIdx.x) / MOM_LANES;
  const int sub = threadIdx.x & (MOM_LANES - 1);
  const bool valid = c < M;
  const int64_t o0 = valid ? offsets[c] : 0, o1 = valid ? offsets[c + 1] : 0;
  double v[NMOM];
  row_moments<S, G>(p.cx, p.cy, p.cz, p.erot, p.vib, o0, o1, sub, v, perm);
  if (valid) store_moments(mom, M, c, sub, v);
}

// Per-cell state of cell c.
__device__ __forceinline__ void reconstruct_cell(const GridP& g, const GasP& gas, const double* mom,
                                                 double dt, const double* dt_cell, double* cs,
                                                 int64_t* counters, int64_t c) {
  const int64_t M = g.M;
  double m[NMOM], v[NCS];
#pragma unroll
  for (int k = 0; k < NMOM; ++k) m[k] = mom[k * M + c];
  cell_state(g, gas, m, c, dt_cell ? dt_cell[c] : dt, v, counters);
  store_cell_state(cs, M, c, v);
}

// Per-cell state, one thread per cell.
__global__ void k_reconstruct(GridP g, GasP gas, const double* mom, double dt,
                              const double* dt_cell, double* cs, int64_t* counters) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < g.M) reconstruct_cell(g, gas, mom, dt, dt_cell, cs, counters, c);
}

// Quadrant stencils of the reconstruction (Sec. III.B), one thread per
// cell, after the cell state: quadrant q = (x >= x_i) + 2 (y >= y_j) keeps
// the x neighbour direction tx and y direction ty (toward the quadrant,
// else the opposite side, else none) and whether the diagonal cell
// completes the cross term.  Field: 2 bits tx (1: +1, 2: -1), 2 bits ty,
// 1 bit cross, 5 bits per quadrant.
__device__ __forceinline__ void stencil_cell(const GridP& g, double* cs, int64_t c) {
  const int64_t M = g.M;
  const int nx = g.nx;
  const int ci = g.dim == 2 ? (int)(c % nx) : 0;
  const int cj = g.dim == 2 ? (int)(c / nx) : (int)c;
  auto ok = [&](int ii, int jj) -> bool {
    if (ii < 0 || jj < 0 || ii >= g.nx || jj >= g.ny) return false;
    return cs[CS_NBR_OK * M + (int64_t)jj * nx + ii] != 0.0;
  };
  int32_t bits = 0;
  for (int q = 0; q < 4; ++q) {
    const int sx = (q & 1) ? 1 : -1, sy = (q & 2) ? 1 : -1;
    int ty = 0, tx = 0;
    if (ok(ci, cj + sy)) ty = sy;
    else if (ok(ci, cj - sy)) ty = -sy;
    if (g.dim == 2) {
      if (ok(ci + sx, cj)) tx = sx;
      else if (ok(ci - sx, cj)) tx = -sx;
    }
    const int cross = (tx && ty && ok(ci + tx, cj + ty)) ? 1 : 0;
    const int f = (tx == 1 ? 1 : tx == -1 ? 2 : 0) | ((ty == 1 ? 1 : ty == -1 ? 2 : 0) << 2) | (cross << 4);
    bits |= f << (5 * q);
  }
  cell_records(cs, M)[c].stencil = bits;
}

__global__ void k_stencil(GridP g, double* cs) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c < g.M && g.dim != 0) stencil_cell(g, cs, c);
}

// Grids of at most CELL_SMALL cells (launch-bound steps): the cell state and
// then the stencils in one block, the barrier between them standing in for
// the launch boundary (the stencils read the neighbours' usability).
constexpr int64_t CELL_SMALL = 256;
__global__ __launch_bounds__(256) void k_cell_state_small(GridP g, GasP gas, const double* mom,
                                                          double dt, const double* dt_cell,
                                                          double* cs, int64_t* counters) {
  for (int64_t c = threadIdx.x; c < g.M; c += blockDim.x)
    reconstruct_cell(g, gas, mom, dt, dt_cell, cs, counters, c);
  if (g.dim == 0) return;
  __syncthreads();
  for (int64_t c = threadIdx.x; c < g.M; c += blockDim.x) stencil_cell(g, cs, c);
}

// Field sampling: the raw particle sums of each cell, N <f(c)>, formed
// from the central moment planes (c = U + C) and added to the running sums.
// Thread per cell, plain read-modify-write: deterministic.
__global__ void k_sample_fields(int64_t M, const double* __restrict__ mom,
                                double* __restrict__ acc) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= M) return;
  const double N = mom[M_N * M + c];
  if (N == 0.0) return;
  double U[3], P[6], qt[3], qr[3], qi[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    U[k] = mom[(M_UX + k) * M + c];
    qt[k] = mom[(M_QTRX + k) * M + c];
    qr[k] = mom[(M_QROTX + k) * M + c];
    qi[k] = mom[(M_QIX + k) * M + c];
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) P[k] = mom[(M_PXX + k) * M + c];
  const double er = mom[M_EROT * M + c], Ib = mom[M_IBAR * M + c];
  // Pi as a full matrix: xx yy zz xy xz yz
  const double PU[3] = {P[0] * U[0] + P[3] * U[1] + P[4] * U[2],
                        P[3] * U[0] + P[1] * U[1] + P[5] * U[2],
                        P[4] * U[0] + P[5] * U[1] + P[2] * U[2]};
  const double hU2 = 0.5 * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]);
  const double htr = 0.5 * (P[0] + P[1] + P[2]);
  double v[USP_NSAMP];
  v[0] = 1.0;
  v[1] = U[0]; v[2] = U[1]; v[3] = U[2];
  v[4] = P[0] + U[0] * U[0]; v[5] = P[1] + U[1] * U[1]; v[6] = P[2] + U[2] * U[2];
  v[7] = P[3] + U[0] * U[1]; v[8] = P[4] + U[0] * U[2]; v[9] = P[5] + U[1] * U[2];
  v[10] = er; v[11] = Ib;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    v[12 + k] = (hU2 + htr) * U[k] + PU[k] + qt[k];
    v[15 + k] = U[k] * er + qr[k];
    v[18 + k] = U[k] * Ib + qi[k];
  }
#pragma unroll
  for (int k = 0; k < USP_NSAMP; ++k) acc[k * M + c] += N * v[k];
}

hipError_t launch_sample_fields(const GridP& g, const double* mom, double* acc, hipStream_t st) {
  k_sample_fields<<<cdiv(g.M, 256), 256, 0, st>>>(g.M, mom, acc);
  return hipGetLastError();
}

template <typename S>
hipError_t launch_moments(const GridP& g, const PartP<S>& p, const int64_t* offsets, double* mom,
                          hipStream_t st, const uint32_t* gather_perm) {
  const int64_t nb = cdiv(g.M * MOM_LANES, CELL_BLOCK);
  if (gather_perm)
    k_moments<S, true><<<nb, CELL_BLOCK, 0, st>>>(g, p, offsets, mom, gather_perm);
  else
    k_moments<S, false><<<nb, CELL_BLOCK, 0, st>>>(g, p, offsets, mom, nullptr);
  return hipGetLastError();
}

hipError_t launch_reconstruct(const GridP& g, const GasP& gas, const double* mom, double dt,
                              const double* dt_cell, double* cs, int64_t* counters, hipStream_t st) {
  if (g.M <= CELL_SMALL) {
    k_cell_state_small<<<1, 256, 0, st>>>(g, gas, mom, dt, dt_cell, cs, counters);
  } else {
    k_reconstruct<<<cdiv(g.M, 128), 128, 0, st>>>(g, gas, mom, dt, dt_cell, cs, counters);
    k_stencil<<<cdiv(g.M, 256), 256, 0, st>>>(g, cs);
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the coefficient chain per cell, when the particle update takes it
  // from the cell
  return launch_cell_coef(g, gas, cs, st);
}

template hipError_t launch_moments<float>(const GridP&, const PartP<float>&, const int64_t*,
                                          double*, hipStream_t, const uint32_t*);
template hipError_t launch_moments<double>(const GridP&, const PartP<double>&, const int64_t*,
                                           double*, hipStream_t, const uint32_t*);

}  // namespace usp
