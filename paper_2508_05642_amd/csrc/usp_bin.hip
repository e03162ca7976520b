// usp_bin.hip -- binning: stable counting sort of particles by cell.
//
// 1. key + histogram: cell of every live particle (integer atomics only,
//    one per run of equal keys in a wave);
// 2. exclusive scan of the histogram -> cell offsets (reduce, top, down);
// 3. slot claim: each particle takes a slot in its cell's range with an
//    atomic cursor (order inside a cell is arbitrary at this point);
// 4. per-cell sort of the claimed input indices, ascending (one wave per
//    cell by rank counting; a block per cell above 1024 particles): this
//    restores input order inside every cell, so the result is the stable sort;
// 5. gather of every state array through the permutation.
// All results are deterministic: the only atomics are integer ones and the
// per-cell sort removes their ordering.
#include "usp_device.h"

namespace usp {

constexpr int BIN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = BIN_BLOCK * SCAN_ITEMS;
constexpr int SORT_LDS = 4096;

__global__ void k_fill_i32(int32_t* p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Runs of equal keys in consecutive lanes of a wave (particles arrive
// mostly sorted by cell, so a wave holds a few long runs).  Returns the
// lane of this lane's run head and, for heads, the run length.
__device__ __forceinline__ void wave_runs(int32_t key, int* head_lane, int* run_len) {
  const int lane = threadIdx.x & 63;
  const int32_t prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || key != prev;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  *head_lane = 63 - __clzll(heads & upto);
  const uint64_t above = heads & ~upto;
  const int next = above ? (__ffsll((long long)above) - 1) : 64;
  *run_len = head ? next - lane : 0;
}

template <typename S>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin_key(GridP g, PartP<S> in, int32_t* key,
                                                       int32_t* counts, int64_t* counters) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = i < in.count[0];
  int32_t c = -1;
  if (live) {
    c = in.cell[i];
    if (c >= 0) {
      if (g.dim == 0) {
        if (c >= g.M) c = -1;
      } else {
        c = cell_of<S>(g, g.dim == 2 ? in.x[i] : S(0), in.y[i]);
      }
    }
    if (c >= 0 && g.flags && (g.flags[c] & USP_FLAG_SOLID)) {
      c = -1;
      count_event(counters, USP_CNT_SOLID_DROP);
    }
    key[i] = c;
  }
  // one atomic per run of equal keys
  int hl, len;
  wave_runs(c, &hl, &len);
  if (len > 0 && c >= 0) atomicAdd(&counts[c], len);
}

// ---- exclusive scan of int32 counts into int64 offsets -------------------
__device__ __forceinline__ int64_t block_exclusive_scan(int64_t v, int64_t* total) {
  __shared__ int64_t wsum[BIN_BLOCK / 64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t x = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[wid] = x;
  __syncthreads();
  int64_t base = 0, tot = 0;
  for (int w = 0; w < BIN_BLOCK / 64; ++w) {
    if (w < wid) base += wsum[w];
    tot += wsum[w];
  }
  __syncthreads();
  *total = tot;
  return base + x - v;
}

__global__ __launch_bounds__(BIN_BLOCK) void k_scan_reduce(const int32_t* counts, int64_t M,
                                                           int64_t* blocksums) {
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t j = base + (int64_t)k * BIN_BLOCK + threadIdx.x;
    if (j < M) s += counts[j];
  }
  int64_t tot;
  block_exclusive_scan(s, &tot);
  if (threadIdx.x == 0) blocksums[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums in place; total -> offsets[M]
// and the output particle count
__global__ __launch_bounds__(BIN_BLOCK) void k_scan_top(int64_t* blocksums, int64_t nb,
                                                        int64_t* offsets, int64_t M,
                                                        int64_t* out_count, const int64_t* in_count) {
  int64_t carry = 0;
  for (int64_t b0 = 0; b0 < nb; b0 += BIN_BLOCK) {
    const int64_t j = b0 + threadIdx.x;
    const int64_t v = j < nb ? blocksums[j] : 0;
    int64_t tot;
    const int64_t ex = block_exclusive_scan(v, &tot);
    if (j < nb) blocksums[j] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) {
    offsets[M] = carry;
    out_count[0] = carry;
    out_count[1] = in_count[1];
  }
}

__global__ __launch_bounds__(BIN_BLOCK) void k_scan_down(const int32_t* counts, int64_t M,
                                                         const int64_t* blocksums,
                                                         int64_t* offsets) {
  // blocked arrangement: thread t owns SCAN_ITEMS consecutive entries
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t j = base + k;
    v[k] = j < M ? counts[j] : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t run = blocksums[blockIdx.x] + block_exclusive_scan(s, &tot);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t j = base + k;
    if (j < M) offsets[j] = run;
    run += v[k];
  }
}

__global__ __launch_bounds__(BIN_BLOCK) void k_claim(const int32_t* key, const int64_t* count,
                                                     const int64_t* offsets, int32_t* cursor,
                                                     uint32_t* perm) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int32_t c = i < count[0] ? key[i] : -1;
  // the run head claims slots for its whole run; members follow in order
  int hl, len;
  wave_runs(c, &hl, &len);
  int32_t base = 0;
  if (len > 0 && c >= 0) base = atomicAdd(&cursor[c], len);
  base = __shfl(base, hl, 64);
  if (c >= 0) perm[offsets[c] + base + ((threadIdx.x & 63) - hl)] = (uint32_t)i;
}

// Ascending sort network in which every compare-exchange puts the smaller
// value at the lower index (the bitonic merge with a mirrored first step).
// Entries at and beyond n are treated as +infinity and never move, so any
// pair whose partner lies beyond n is skipped and no padding is needed.
template <bool LDS>
__device__ __forceinline__ void sort_net(uint32_t* a, int n) {
  int npow = 1;
  while (npow < n) npow <<= 1;
  for (int k = 2; k <= npow; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < npow; i += blockDim.x) {
        const int p = (j == (k >> 1)) ? (i ^ (k - 1)) : (i ^ j);
        if (p > i && p < n) {
          const uint32_t u = a[i], w = a[p];
          if (w < u) { a[i] = w; a[p] = u; }
        }
      }
      if (!LDS) __threadfence_block();
      __syncthreads();
    }
  }
}

// One wave sorts one cell's slot list (distinct input indices) by rank
// counting: each lane holds K entries in registers; every entry's rank is
// the number of entries below it, counted against all entries broadcast one
// at a time with readlane.  Entries beyond n hold UINT32_MAX and never count.
template <int K>
__device__ __forceinline__ void wave_rank_sort(uint32_t* seg, int n) {
  const int lane = threadIdx.x & 63;
  uint32_t v[K];
  int r[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = k * 64 + lane;
    v[k] = j < n ? seg[j] : 0xFFFFFFFFu;
    r[k] = 0;
  }
#pragma unroll
  for (int s = 0; s < K; ++s) {
    const int lim = n - s * 64 < 64 ? n - s * 64 : 64;
    for (int l = 0; l < lim; ++l) {
      const uint32_t w = (uint32_t)__builtin_amdgcn_readlane((int)v[s], l);
#pragma unroll
      for (int k = 0; k < K; ++k) r[k] += (w < v[k]) ? 1 : 0;
    }
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int j = k * 64 + lane;
    if (j < n) seg[r[k]] = v[k];
  }
}

constexpr int WAVE_SORT_MAX = 1024;

__global__ __launch_bounds__(BIN_BLOCK) void k_segsort_wave(const int64_t* offsets, int64_t M,
                                                            uint32_t* perm) {
  const int64_t c = (int64_t)blockIdx.x * (BIN_BLOCK / 64) + (threadIdx.x >> 6);
  if (c >= M) return;
  const int64_t o0 = offsets[c];
  const int n = (int)(offsets[c + 1] - o0);
  if (n <= 1 || n > WAVE_SORT_MAX) return;
  uint32_t* seg = perm + o0;
  if (n <= 64) wave_rank_sort<1>(seg, n);
  else if (n <= 128) wave_rank_sort<2>(seg, n);
  else if (n <= 256) wave_rank_sort<4>(seg, n);
  else if (n <= 512) wave_rank_sort<8>(seg, n);
  else wave_rank_sort<16>(seg, n);
}

// cells above WAVE_SORT_MAX: one block per cell, sort network in LDS (or in
// global memory beyond SORT_LDS entries)
__global__ __launch_bounds__(BIN_BLOCK) void k_segsort_big(const int64_t* offsets, uint32_t* perm) {
  __shared__ uint32_t s[SORT_LDS];
  const int64_t c = blockIdx.x;
  const int64_t o0 = offsets[c];
  const int n = (int)(offsets[c + 1] - o0);
  if (n <= WAVE_SORT_MAX) return;
  uint32_t* seg = perm + o0;
  if (n <= SORT_LDS) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = seg[i];
    __syncthreads();
    sort_net<true>(s, n);
    for (int i = threadIdx.x; i < n; i += blockDim.x) seg[i] = s[i];
  } else {
    sort_net<false>(seg, n);
  }
}

template <typename S>
__global__ __launch_bounds__(BIN_BLOCK) void k_gather(PartP<S> in, PartP<S> out,
                                                      const uint32_t* perm, const int32_t* key,
                                                      int has_x, int has_y) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= out.count[0]) return;
  const uint32_t i = perm[p];
  if (has_x) out.x[p] = in.x[i];
  if (has_y) out.y[p] = in.y[i];
  out.cx[p] = in.cx[i];
  out.cy[p] = in.cy[i];
  out.cz[p] = in.cz[i];
  out.erot[p] = in.erot[i];
  out.vib[p] = in.vib[i];
  out.pid[p] = in.pid[i];
  out.cell[p] = key[i];
}

template <typename S>
hipError_t launch_bin(const GridP& g, const PartP<S>& in, const PartP<S>& out, int64_t* offsets,
                      char* ws, const WsLayout& L, int64_t* counters, hipStream_t st) {
  int32_t* key = (int32_t*)(ws + L.key);
  int32_t* cursor = (int32_t*)(ws + L.cursor);
  uint32_t* perm = (uint32_t*)(ws + L.perm);
  int64_t* blocksums = (int64_t*)(ws + L.blocksums);
  const int64_t M = g.M;
  const int64_t cap = in.capacity;
  const int64_t nb = cdiv(M, SCAN_TILE);
  k_fill_i32<<<cdiv(M, 256), 256, 0, st>>>(cursor, 0, M);
  k_bin_key<S><<<cdiv(cap, BIN_BLOCK), BIN_BLOCK, 0, st>>>(g, in, key, cursor, counters);
  k_scan_reduce<<<nb, BIN_BLOCK, 0, st>>>(cursor, M, blocksums);
  k_scan_top<<<1, BIN_BLOCK, 0, st>>>(blocksums, nb, offsets, M, out.count, in.count);
  k_scan_down<<<nb, BIN_BLOCK, 0, st>>>(cursor, M, blocksums, offsets);
  k_fill_i32<<<cdiv(M, 256), 256, 0, st>>>(cursor, 0, M);
  k_claim<<<cdiv(cap, BIN_BLOCK), BIN_BLOCK, 0, st>>>(key, in.count, offsets, cursor, perm);
  k_segsort_wave<<<cdiv(M, BIN_BLOCK / 64), BIN_BLOCK, 0, st>>>(offsets, M, perm);
  k_segsort_big<<<M, BIN_BLOCK, 0, st>>>(offsets, perm);
  k_gather<S><<<cdiv(cap, BIN_BLOCK), BIN_BLOCK, 0, st>>>(in, out, perm, key, g.dim == 2,
                                                          g.dim >= 1);
  return hipGetLastError();
}

template hipError_t launch_bin<float>(const GridP&, const PartP<float>&, const PartP<float>&,
                                      int64_t*, char*, const WsLayout&, int64_t*, hipStream_t);
template hipError_t launch_bin<double>(const GridP&, const PartP<double>&, const PartP<double>&,
                                       int64_t*, char*, const WsLayout&, int64_t*, hipStream_t);

}  // namespace usp
