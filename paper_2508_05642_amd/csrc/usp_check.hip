// usp_check.hip -- the scan behind usp_check: counts NaN and infinite
// values in a particle state and in the moment and cell-state planes, so
// that a caller can turn a run gone wrong into a status instead of letting
// the non-finite values spread.
#include "usp_internal.h"

namespace usp {

template <typename S>
__global__ void k_check_parts(GridP g, PartP<S> p, int64_t* found) {
  int64_t n = p.count[0];
  n = n < 0 ? 0 : (n > p.capacity ? p.capacity : n);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // whole waves run every iteration, so the ballot sees every lane
  const int64_t nr = (n + stride - 1) / stride * stride;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride) {
    int bad = 0;
    if (i < n) {
      bad += !isfinite((double)p.cx[i]);
      bad += !isfinite((double)p.cy[i]);
      bad += !isfinite((double)p.cz[i]);
      bad += !isfinite((double)p.erot[i]);
      if (g.dim >= 1) bad += !isfinite((double)p.y[i]);
      if (g.dim == 2) bad += !isfinite((double)p.x[i]);
    }
    // at most 6 per particle: count each bit of the per-lane sum
    for (int b = 0; b < 3; ++b) {
      const uint64_t m = __ballot((bad >> b) & 1);
      if (m && (threadIdx.x & 63) == 0)
        atomicAdd((unsigned long long*)found, (unsigned long long)__popcll(m) << b);
    }
  }
}

// Thread per cell: the planes of an occupied cell (count plane >= 1, or
// itself not finite).
__global__ void k_check_planes(const double* __restrict__ v, int nplanes, int count_plane,
                               int64_t M, int64_t* found) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int bad = 0;
  if (c < M) {
    const double N = v[(int64_t)count_plane * M + c];
    if (!(N < 1.0)) {
      for (int k = 0; k < nplanes; ++k) bad += !isfinite(v[(int64_t)k * M + c]);
    }
  }
  // up to 64 per cell: count each bit of the per-lane sum
  for (int b = 0; b < 7; ++b) {
    const uint64_t m = __ballot((bad >> b) & 1);
    if (m && (threadIdx.x & 63) == 0)
      atomicAdd((unsigned long long*)found, (unsigned long long)__popcll(m) << b);
  }
}

template <typename S>
hipError_t launch_check(const GridP& g, const PartP<S>& p, const double* mom, const double* cs,
                        int64_t* found, hipStream_t st) {
  const int64_t blocks = cdiv(p.capacity, 256) < 4096 ? cdiv(p.capacity, 256) : 4096;
  k_check_parts<S><<<blocks, 256, 0, st>>>(g, p, found);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t cb = cdiv(g.M, 256);
  if (mom) {
    k_check_planes<<<cb, 256, 0, st>>>(mom, NMOM, M_N, g.M, found);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (cs) {
    k_check_planes<<<cb, 256, 0, st>>>(cs, NCS, CS_NP, g.M, found);
    e = hipGetLastError();
  }
  return e;
}

template hipError_t launch_check<float>(const GridP&, const PartP<float>&, const double*,
                                        const double*, int64_t*, hipStream_t);
template hipError_t launch_check<double>(const GridP&, const PartP<double>&, const double*,
                                         const double*, int64_t*, hipStream_t);

}  // namespace usp
