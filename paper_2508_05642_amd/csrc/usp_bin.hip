// usp_bin.hip -- binning: stable counting sort of particles by cell.
//
// The output order is fixed by definition: particles sorted by cell, in
// input order inside a cell, removed particles dropped.  Two routes give it:
//
// * Binned input (the usual case: the previous step's sorted state, whose
//   segment offsets are passed in, followed by a tail of injected
//   particles).  A particle of old cell k lands in k + d with d in a small
//   neighbour set, so a new cell's particles come from at most 9 source
//   segments, which appear in ascending order in the input.  One wave per
//   source segment ranks its particles inside each group with ballots
//   (k_bin_group); one thread per new cell turns the group counts into
//   positions, interleaving the rare far moves by input index
//   (k_cell_bases); one wave per source segment then writes every particle
//   straight to its final slot (k_bin_scatter).  No atomics, no sorting.
// * The tail, and every particle when no input offsets are given: slots are
//   claimed after the cell's prefix particles with one integer atomic per
//   run of equal keys, and each cell's claimed indices are sorted ascending
//   (restoring input order) before the copy.
// All results are deterministic.
#include "usp_device.h"

namespace usp {

constexpr int BIN_BLOCK = 256;
constexpr int SCAN_ITEMS = 4;
constexpr int SCAN_TILE = BIN_BLOCK * SCAN_ITEMS;
constexpr int SORT_LDS = 4096;
constexpr int BIN_U = 4;
// grids of at most this many cells launch independent bin kernels together
constexpr int64_t BIN_MERGE_MAX = 4096;  // chunks of 64 particles per load batch of the grouped bin

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

// Each block adds up the totals of the blocks before it (at most a few
// hundred, read from L2), then scans its own tile; the last block writes the
// total to offsets[M] and the output particle count.
__global__ __launch_bounds__(BIN_BLOCK) void k_scan_down(const int32_t* counts, int64_t M,
                                                         const int64_t* blocksums,
                                                         int64_t* offsets, int64_t* out_count,
                                                         const int64_t* in_count) {
  int64_t before = 0;
  for (int64_t b = threadIdx.x; b < (int64_t)blockIdx.x; b += BIN_BLOCK) before += blocksums[b];
  int64_t block_base;
  block_exclusive_scan(before, &block_base);
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
  int64_t run = block_base + block_exclusive_scan(s, &tot);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t j = base + k;
    if (j < M) offsets[j] = run;
    run += v[k];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    offsets[M] = block_base + tot;
    if (out_count) {
      out_count[0] = block_base + tot;
      out_count[1] = in_count[1];
    }
  }
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

// ---------------------------------------------------------------------------
// Neighbour groups.  A particle of old cell k whose new cell is c = k + d
// with d in D (the cell itself and its 8 neighbours in 2D, up to 4 cells
// either way in 1D) belongs
// to group d; any other destination is a far move.  D is listed in
// descending order, so the source cells k = c - d of a new cell c come in
// ascending order, which is input order for a binned input.
// ---------------------------------------------------------------------------
struct Nbr {
  int n;
  int d[9];
};

__host__ __device__ inline Nbr nbr_set(const GridP& g) {
  Nbr r;
  if (g.dim == 2 && g.nx >= 3) {
    const int nx = g.nx;
    const int v[9] = {nx + 1, nx, nx - 1, 1, 0, -1, -nx + 1, -nx, -nx - 1};
    r.n = 9;
    for (int k = 0; k < 9; ++k) r.d[k] = v[k];
  } else if (g.dim == 1) {
    // along y a particle may cross several cells in a step: nine groups,
    // moves of up to four cells either way
    r.n = 9;
    for (int k = 0; k < 9; ++k) r.d[k] = 4 - k;
  } else {
    r.n = 3;
    r.d[0] = 1; r.d[1] = 0; r.d[2] = -1;
    for (int k = 3; k < 9; ++k) r.d[k] = 0;
  }
  return r;
}

constexpr int GRP_FAR = 9;
constexpr int GRP_GONE = 15;

// Group of a move by d cells: the index of d in nb.d, else GRP_FAR.  In 2D
// (nx >= 3) the members are d = r nx + dx with r, dx in {1, 0, -1}, listed
// as q = 3 (1 - r) + (1 - dx), and r is fixed by the sign of d beyond +-1;
// in 1D and 0D nb.d counts down by one from nb.d[0].
__device__ __forceinline__ int nbr_group(const GridP& g, const Nbr& nb, int64_t d) {
  if (g.dim == 2 && g.nx >= 3) {
    const int64_t r = d >= 2 ? 1 : (d <= -2 ? -1 : 0);
    const int64_t dx = d - r * g.nx;
    return (dx >= -1 && dx <= 1) ? (int)(3 * (1 - r) + (1 - dx)) : GRP_FAR;
  }
  const int64_t q = (int64_t)nb.d[0] - d;
  return (q >= 0 && q < nb.n) ? (int)q : GRP_FAR;
}

template <typename S>
__device__ __forceinline__ int32_t new_key(const GridP& g, const PartP<S>& in, int64_t i,
                                           bool* solid) {
  int32_t c = in.cell[i];
  *solid = false;
  if (c >= 0) {
    if (g.dim == 0) {
      if (c >= g.M) c = -1;
    } else {
      c = cell_of<S>(g, g.dim == 2 ? in.x[i] : S(0), in.y[i]);
    }
  }
  if (c >= 0 && g.flags && (g.flags[c] & USP_FLAG_SOLID)) {
    c = -1;
    *solid = true;
  }
  return c;
}

__device__ __forceinline__ int64_t sorted_len(const int64_t* old_off, int64_t M, const int64_t* count) {
  const int64_t a = old_off[M], b = count[0];
  return a < b ? (a > 0 ? a : 0) : b;
}

// A: one wave per old cell k.  New cell of every particle of the segment,
// its group, and its rank among the earlier particles of the segment in the
// same group (64 at a time with ballots).  Writes grp[i] = rank << 4 | group,
// the group counts T9[k][.], and appends far moves to an unordered list.
template <typename S>
__device__ __forceinline__ void bin_group(const GridP& g, const Nbr& nb, const PartP<S>& in,
                                          const int64_t* old_off, int32_t* grp, int32_t* T9,
                                          int32_t* far_cnt, int32_t* far_c, int32_t* far_i,
                                          int32_t* far_total, int64_t* counters, int64_t blk) {
  const int64_t M = g.M;
  const int64_t k = blk * (BIN_BLOCK / 64) + (threadIdx.x >> 6);
  if (k >= M) return;
  const int lane = threadIdx.x & 63;
  const int64_t ns = sorted_len(old_off, M, in.count);
  int64_t lo = old_off[k], hi = old_off[k + 1];
  lo = lo < 0 ? 0 : (lo > ns ? ns : lo);
  hi = hi < lo ? lo : (hi > ns ? ns : hi);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  int running[10];
#pragma unroll
  for (int q = 0; q < 10; ++q) running[q] = 0;
  // BIN_U chunks of 64 at a time: their cell and flag loads are issued
  // together, ahead of the ranking, which needs no memory
  for (int64_t base = lo; base < hi; base += 64 * BIN_U) {
    int32_t cc[BIN_U];
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      const int64_t i = base + u * 64 + lane;
      // a binned prefix carries its current cells (the flight rewrote them
      // from the new positions); only the solid-cell test remains
      cc[u] = i < hi ? in.cell[i] : -1;
      if (g.dim == 0 && cc[u] >= M) cc[u] = -1;
    }
    uint32_t solid = 0;
    if (g.flags) {
#pragma unroll
      for (int u = 0; u < BIN_U; ++u)
        if (cc[u] >= 0 && (g.flags[cc[u]] & USP_FLAG_SOLID)) solid |= 1u << u;
    }
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      if (base + u * 64 >= hi) break;
      const int64_t i = base + u * 64 + lane;
      const bool active = i < hi;
      int grpid = 14;  // inactive lane
      int32_t c = cc[u];
      if (active) {
        if (solid & (1u << u)) {
          c = -1;
          count_event(counters, USP_CNT_SOLID_DROP);
        }
        grpid = c < 0 ? GRP_GONE : nbr_group(g, nb, (int64_t)c - k);
      }
      // ranks within each group present in the wave (the others add nothing)
      const uint32_t present = wave_or(grpid < 10 ? (1u << grpid) : 0u);
      int rank = 0;
#pragma unroll
      for (int q = 0; q < 10; ++q) {
        if (present & (1u << q)) {
          const uint64_t m = __ballot(grpid == q);
          if (grpid == q) rank = running[q] + __popcll(m & lt);
          running[q] += __popcll(m);
        }
      }
      if (active) grp[i] = (rank << 4) | grpid;
      if (grpid == GRP_FAR) {
        const int j = atomicAdd(far_total, 1);
        far_c[j] = c;
        far_i[j] = (int32_t)i;
        atomicAdd(&far_cnt[c], 1);
      }
    }
  }
  if (lane < nb.n) {
    int v = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      if (q == lane) v = running[q];
    T9[k * 9 + lane] = v;
  }
}

// Keys of the unsorted tail [ns, n) (injected particles, or every particle
// when the input is not binned): one atomic per run of equal keys.
template <typename S>
__device__ __forceinline__ void tail_key(const GridP& g, const PartP<S>& in, const int64_t* old_off,
                                         int32_t* key, int32_t* tail_cnt, int32_t* tail_cells,
                                         int32_t* n_tail_cells, int64_t* counters, int64_t blk,
                                         int64_t nblk) {
  const int64_t M = g.M;
  const int64_t ns = sorted_len(old_off, M, in.count), n = in.count[0];
  const int lane = threadIdx.x & 63;
  const int64_t stride = nblk * BIN_BLOCK;
  for (int64_t b = ns + blk * BIN_BLOCK + (threadIdx.x & ~63); b < n; b += stride) {
    const int64_t i = b + lane;
    int32_t c = -1;
    if (i < n) {
      bool solid;
      c = new_key<S>(g, in, i, &solid);
      if (solid) count_event(counters, USP_CNT_SOLID_DROP);
      key[i] = c;
    }
    int hl, len;
    wave_runs(c, &hl, &len);
    // the run that opens a cell's tail also lists the cell
    if (len > 0 && c >= 0 && atomicAdd(&tail_cnt[c], len) == 0)
      tail_cells[atomicAdd(n_tail_cells, 1)] = c;
  }
}

template <typename S>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin_group(GridP g, Nbr nb, PartP<S> in,
                                                         const int64_t* old_off, int32_t* grp,
                                                         int32_t* T9, int32_t* far_cnt,
                                                         int32_t* far_c, int32_t* far_i,
                                                         int32_t* far_total, int64_t* counters) {
  bin_group<S>(g, nb, in, old_off, grp, T9, far_cnt, far_c, far_i, far_total, counters, blockIdx.x);
}

template <typename S>
__global__ __launch_bounds__(BIN_BLOCK) void k_tail_key(GridP g, PartP<S> in, const int64_t* old_off,
                                                        int32_t* key, int32_t* tail_cnt,
                                                        int32_t* tail_cells, int32_t* n_tail_cells,
                                                        int64_t* counters) {
  tail_key<S>(g, in, old_off, key, tail_cnt, tail_cells, n_tail_cells, counters, blockIdx.x,
              gridDim.x);
}

// On small grids, where the step is launch-bound, the two run side by side
// in one launch (they touch disjoint arrays): the first ngroup blocks group
// the binned prefix, the rest key the tail.  (On large grids the separate
// launches are faster.)
template <typename S>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin_group_tail(GridP g, Nbr nb, PartP<S> in,
                                                              const int64_t* old_off, int32_t* key,
                                                              int32_t* T9, int32_t* far_cnt,
                                                              int32_t* far_c, int32_t* far_i,
                                                              int32_t* far_total, int32_t* tail_cnt,
                                                              int32_t* tail_cells,
                                                              int32_t* n_tail_cells,
                                                              int64_t* counters, int64_t ngroup) {
  const int64_t blk = blockIdx.x;
  if (blk < ngroup)
    bin_group<S>(g, nb, in, old_off, key, T9, far_cnt, far_c, far_i, far_total, counters, blk);
  else
    tail_key<S>(g, in, old_off, key, tail_cnt, tail_cells, n_tail_cells, counters, blk - ngroup,
                (int64_t)gridDim.x - ngroup);
}

// Far moves into per-cell lists (the order inside a list is fixed later).
__global__ __launch_bounds__(BIN_BLOCK) void k_far_place(const int32_t* far_total,
                                                         const int32_t* far_c, const int32_t* far_i,
                                                         const int64_t* far_off, int32_t* far_cur,
                                                         int32_t* far_list) {
  const int nt = *far_total;
  for (int j = blockIdx.x * BIN_BLOCK + threadIdx.x; j < nt; j += gridDim.x * BIN_BLOCK) {
    const int32_t c = far_c[j];
    far_list[far_off[c] + atomicAdd(&far_cur[c], 1)] = far_i[j];
  }
}

// B2: the far moves into each cell in ascending input index.  Each wave
// takes cpw cells (1, or 64 on large grids, whose far moves are sparse) and
// sorts their lists of 2..FAR_SORT entries in its share of LDS, one list at
// a time (bitonic network, distinct keys, so the result is the unique sorted
// list); longer lists are left to the insertion sort of k_cell_bases.
constexpr int FAR_SORT = 512;

__global__ __launch_bounds__(BIN_BLOCK) void k_far_sort(const int64_t* __restrict__ far_off,
                                                        int64_t M, int32_t* far_list, int cpw) {
  __shared__ int32_t keys[BIN_BLOCK / 64][FAR_SORT];
  const int lane = threadIdx.x & 63;
  // lanes below cpw read one cell's list bounds each; the wave then sorts
  // the lists of 2..FAR_SORT entries among them one after another
  const int64_t cl = ((int64_t)blockIdx.x * (BIN_BLOCK / 64) + (threadIdx.x >> 6)) * cpw + lane;
  int64_t f0l = 0, nl = 0;
  if (lane < cpw && cl < M) {
    f0l = far_off[cl];
    nl = far_off[cl + 1] - f0l;
  }
  uint64_t todo = __ballot(nl >= 2 && nl <= FAR_SORT);
  int32_t* v = keys[threadIdx.x >> 6];
  while (todo) {
    const int src = __ffsll((long long)todo) - 1;
    todo &= todo - 1;
    const int64_t f0 = __shfl(f0l, src, 64);
    const int64_t n = __shfl(nl, src, 64);
    int P = 2;
    while (P < n) P <<= 1;
    for (int t = lane; t < P; t += 64) v[t] = t < n ? far_list[f0 + t] : INT32_MAX;
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int k = 2; k <= P; k <<= 1) {
      for (int j = k >> 1; j > 0; j >>= 1) {
        for (int t = lane; t < P; t += 64) {
          const int u = t ^ j;
          if (u > t) {
            const int32_t a = v[t], b = v[u];
            if ((a > b) == ((t & k) == 0)) {
              v[t] = b;
              v[u] = a;
            }
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
      }
    }
    for (int t = lane; t < n; t += 64) far_list[f0 + t] = v[t];
    // the next list reuses this wave's keys
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  }
}

// C: one thread per new cell c.  The source groups (k = c - d, ascending k)
// and the far moves into c (ascending index) interleave in input order;
// T9[k][q] becomes the group's first position inside c, far_base the far
// moves' positions.  cnt_total[c] = prefix particles + tail particles.
__global__ __launch_bounds__(BIN_BLOCK) void k_cell_bases(GridP g, Nbr nb, const int64_t* old_off,
                                                          const int64_t* count, int32_t* T9,
                                                          const int64_t* far_off, int32_t* far_list,
                                                          int32_t* far_base, const int32_t* tail_cnt,
                                                          int32_t* nontail, int32_t* cnt_total) {
  const int64_t M = g.M;
  const int64_t c = (int64_t)blockIdx.x * BIN_BLOCK + threadIdx.x;
  if (c >= M) return;
  const int64_t ns = sorted_len(old_off, M, count);
  const int64_t f0 = far_off[c], f1 = far_off[c + 1];
  for (int64_t a = f0 + 1; a < f1; ++a) {  // insertion sort (lists longer than FAR_SORT)
    const int32_t v = far_list[a];
    int64_t b = a - 1;
    while (b >= f0 && far_list[b] > v) { far_list[b + 1] = far_list[b]; --b; }
    far_list[b + 1] = v;
  }
  int32_t run = 0;
  int64_t fp = f0;
  for (int q = 0; q < nb.n; ++q) {
    const int64_t k = c - nb.d[q];
    if (k < 0 || k >= M) continue;
    int64_t kstart = old_off[k];
    kstart = kstart < 0 ? 0 : (kstart > ns ? ns : kstart);
    while (fp < f1 && far_list[fp] < kstart) far_base[fp++] = run++;
    const int32_t cnt = T9[k * 9 + q];
    T9[k * 9 + q] = run;
    run += cnt;
  }
  while (fp < f1) far_base[fp++] = run++;
  nontail[c] = run;
  cnt_total[c] = run + tail_cnt[c];
}

template <typename S>
__device__ __forceinline__ void copy_particle(const PartP<S>& in, const PartP<S>& out, int64_t i,
                                              int64_t p, int32_t c, bool has_x, bool has_y) {
  if (has_x) out.x[p] = in.x[i];
  if (has_y) out.y[p] = in.y[i];
  out.cx[p] = in.cx[i];
  out.cy[p] = in.cy[i];
  out.cz[p] = in.cz[i];
  out.erot[p] = in.erot[i];
  out.vib[p] = in.vib[i];
  out.pid[p] = in.pid[i];
  out.cell[p] = c;
}

// Output slot p of input particle i: copied (G = false), or, for a binning
// that leaves the particles where they are (G = true), recorded as
// gperm[p] = i with the new cell in out.cell[p].
template <bool G, typename S>
__device__ __forceinline__ void place(const PartP<S>& in, const PartP<S>& out, uint32_t* gperm,
                                      int64_t i, int64_t p, int32_t c, bool has_x, bool has_y) {
  if constexpr (G) {
    gperm[p] = (uint32_t)i;
    out.cell[p] = c;
  } else {
    copy_particle<S>(in, out, i, p, c, has_x, has_y);
  }
}

// E: one wave per old cell; every grouped particle goes straight to
// offsets[c] + (group base in c) + (rank in group).
template <typename S, bool G>
__global__ __launch_bounds__(BIN_BLOCK) void k_bin_scatter(GridP g, Nbr nb, PartP<S> in, PartP<S> out,
                                                           uint32_t* gperm,
                                                           const int64_t* old_off, const int32_t* grp,
                                                           const int32_t* T9, const int64_t* offsets) {
  const int64_t M = g.M;
  const int64_t k = (int64_t)blockIdx.x * (BIN_BLOCK / 64) + (threadIdx.x >> 6);
  if (k >= M) return;
  const int lane = threadIdx.x & 63;
  const int64_t ns = sorted_len(old_off, M, in.count);
  int64_t lo = old_off[k], hi = old_off[k + 1];
  // lane q < nb.n holds the first slot of group q and its cell (loaded
  // beside the segment bounds, which it does not depend on)
  int64_t gbase = 0;
  int32_t gcell = 0;
  if (lane < nb.n) {
    int dq = 0;
#pragma unroll
    for (int q = 0; q < 9; ++q)
      if (q == lane) dq = nb.d[q];
    const int64_t c = k + dq;
    if (c >= 0 && c < M) {
      gcell = (int32_t)c;
      gbase = offsets[c] + T9[k * 9 + lane];
    }
  }
  lo = lo < 0 ? 0 : (lo > ns ? ns : lo);
  hi = hi < lo ? lo : (hi > ns ? ns : hi);
  const bool hx = g.dim == 2, hy = g.dim >= 1;
  // the group words of BIN_U chunks are loaded before any of them is placed
  // (the stores could alias them as far as the compiler knows)
  for (int64_t base = lo; base < hi; base += 64 * BIN_U) {
    int32_t gw[BIN_U];
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      const int64_t i = base + u * 64 + lane;
      gw[u] = i < hi ? grp[i] : GRP_GONE;
    }
#pragma unroll
    for (int u = 0; u < BIN_U; ++u) {
      const int64_t i = base + u * 64 + lane;
      const int32_t gv = gw[u];
      const int q = gv & 15;
      const int64_t b = __shfl(gbase, q < 9 ? q : 0, 64);
      const int32_t c = __shfl(gcell, q < 9 ? q : 0, 64);
      if (i < hi && q < nb.n) place<G, S>(in, out, gperm, i, b + (gv >> 4), c, hx, hy);
    }
  }
}

// far moves: each list entry finds its position inside its cell
template <typename S, bool G>
__device__ __forceinline__ void far_scatter(const GridP& g, const PartP<S>& in, const PartP<S>& out,
                                            uint32_t* gperm, const int32_t* far_total,
                                            const int32_t* far_c, const int32_t* far_i,
                                            const int64_t* far_off, const int32_t* far_list,
                                            const int32_t* far_base, const int64_t* offsets,
                                            int blk, int nblk) {
  const int nt = *far_total;
  for (int j = blk * BIN_BLOCK + threadIdx.x; j < nt; j += nblk * BIN_BLOCK) {
    const int32_t c = far_c[j], i = far_i[j];
    int64_t fp = far_off[c];
    const int64_t f1 = far_off[c + 1];
    while (fp < f1 && far_list[fp] != i) ++fp;
    if (fp < f1) place<G, S>(in, out, gperm, i, offsets[c] + far_base[fp], c, g.dim == 2, g.dim >= 1);
  }
}

// tail: slots after the prefix particles of each cell, claimed per run
__device__ __forceinline__ void tail_claim(int64_t M, const int64_t* old_off, const int64_t* count,
                                           const int32_t* key, const int64_t* offsets,
                                           const int32_t* nontail, int32_t* cursor, uint32_t* perm,
                                           int64_t blk, int64_t nblk) {
  const int64_t ns = sorted_len(old_off, M, count), n = count[0];
  const int lane = threadIdx.x & 63;
  const int64_t stride = nblk * BIN_BLOCK;
  for (int64_t b = ns + blk * BIN_BLOCK + (threadIdx.x & ~63); b < n; b += stride) {
    const int64_t i = b + lane;
    const int32_t c = i < n ? key[i] : -1;
    int hl, len;
    wave_runs(c, &hl, &len);
    int32_t base = 0;
    if (len > 0 && c >= 0) base = atomicAdd(&cursor[c], len);
    base = __shfl(base, hl, 64);
    if (c >= 0) perm[offsets[c] + nontail[c] + base + (lane - hl)] = (uint32_t)i;
  }
}

template <typename S, bool G>
__global__ __launch_bounds__(BIN_BLOCK) void k_far_scatter(GridP g, PartP<S> in, PartP<S> out,
                                                           uint32_t* gperm,
                                                           const int32_t* far_total,
                                                           const int32_t* far_c, const int32_t* far_i,
                                                           const int64_t* far_off,
                                                           const int32_t* far_list,
                                                           const int32_t* far_base,
                                                           const int64_t* offsets) {
  far_scatter<S, G>(g, in, out, gperm, far_total, far_c, far_i, far_off, far_list, far_base, offsets,
                    blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(BIN_BLOCK) void k_tail_claim(int64_t M, const int64_t* old_off,
                                                          const int64_t* count, const int32_t* key,
                                                          const int64_t* offsets,
                                                          const int32_t* nontail, int32_t* cursor,
                                                          uint32_t* perm) {
  tail_claim(M, old_off, count, key, offsets, nontail, cursor, perm, blockIdx.x, gridDim.x);
}

// Far moves and tail claims side by side in one launch on small grids
// (disjoint slots): the first nfar blocks place the far moves, the rest
// claim the tail's slots.
template <typename S, bool G>
__global__ __launch_bounds__(BIN_BLOCK) void k_far_tail(GridP g, PartP<S> in, PartP<S> out,
                                                        uint32_t* gperm, const int32_t* far_total,
                                                        const int32_t* far_c, const int32_t* far_i,
                                                        const int64_t* far_off,
                                                        const int32_t* far_list,
                                                        const int32_t* far_base,
                                                        const int64_t* old_off, const int32_t* key,
                                                        const int64_t* offsets,
                                                        const int32_t* nontail, int32_t* cursor,
                                                        uint32_t* perm, int nfar) {
  const int blk = blockIdx.x;
  if (blk < nfar)
    far_scatter<S, G>(g, in, out, gperm, far_total, far_c, far_i, far_off, far_list, far_base,
                      offsets, blk, nfar);
  else
    tail_claim(g.M, old_off, in.count, key, offsets, nontail, cursor, perm, blk - nfar,
               (int64_t)gridDim.x - nfar);
}

// One wave sorts one cell's tail slot list (distinct input indices) by rank
// counting and copies each particle to its rank's slot: each lane holds K
// entries; an entry's rank is the number of entries below it, counted
// against all entries broadcast with readlane.
template <int K, bool G, typename S>
__device__ __forceinline__ void wave_rank_copy(const uint32_t* seg, int n, int64_t dst0,
                                               const PartP<S>& in, const PartP<S>& out,
                                               uint32_t* gperm, int32_t c, bool hx, bool hy) {
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
    if (j < n) place<G, S>(in, out, gperm, v[k], dst0 + r[k], c, hx, hy);
  }
}

constexpr int WAVE_SORT_MAX = 1024;

// one wave per listed cell (grid-stride over the list of cells with a tail)
template <typename S, bool G>
__global__ __launch_bounds__(BIN_BLOCK) void k_tail_sort_copy(GridP g, PartP<S> in, PartP<S> out,
                                                              const int64_t* offsets,
                                                              const int32_t* nontail,
                                                              uint32_t* perm,
                                                              const int32_t* tail_cells,
                                                              const int32_t* n_tail_cells) {
  const int nl = *n_tail_cells;
  const int w0 = blockIdx.x * (BIN_BLOCK / 64) + (threadIdx.x >> 6);
  for (int w = w0; w < nl; w += gridDim.x * (BIN_BLOCK / 64)) {
    const int64_t c = tail_cells[w];
    const int64_t t0 = offsets[c] + nontail[c];
    const int n = (int)(offsets[c + 1] - t0);
    if (n <= 0 || n > WAVE_SORT_MAX) continue;
    const bool hx = g.dim == 2, hy = g.dim >= 1;
    const uint32_t* seg = perm + t0;
    if (n <= 64) wave_rank_copy<1, G, S>(seg, n, t0, in, out, perm, (int32_t)c, hx, hy);
    else if (n <= 128) wave_rank_copy<2, G, S>(seg, n, t0, in, out, perm, (int32_t)c, hx, hy);
    else if (n <= 256) wave_rank_copy<4, G, S>(seg, n, t0, in, out, perm, (int32_t)c, hx, hy);
    else if (n <= 512) wave_rank_copy<8, G, S>(seg, n, t0, in, out, perm, (int32_t)c, hx, hy);
    else wave_rank_copy<16, G, S>(seg, n, t0, in, out, perm, (int32_t)c, hx, hy);
  }
}

// tails above WAVE_SORT_MAX: one block per cell, sort network in LDS (or in
// global memory beyond SORT_LDS entries), then the copy
template <typename S, bool G>
__global__ __launch_bounds__(BIN_BLOCK) void k_tail_sort_copy_big(GridP g, PartP<S> in, PartP<S> out,
                                                                  const int64_t* offsets,
                                                                  const int32_t* nontail,
                                                                  uint32_t* perm,
                                                                  const int32_t* tail_cells,
                                                                  const int32_t* n_tail_cells) {
  __shared__ uint32_t s[SORT_LDS];
  const int nl = *n_tail_cells;
  for (int w = blockIdx.x; w < nl; w += gridDim.x) {
    const int64_t c = tail_cells[w];
    const int64_t t0 = offsets[c] + nontail[c];
    const int n = (int)(offsets[c + 1] - t0);
    if (n <= WAVE_SORT_MAX) continue;
    uint32_t* seg = perm + t0;
    const bool hx = g.dim == 2, hy = g.dim >= 1;
    if (n <= SORT_LDS) {
      for (int i = threadIdx.x; i < n; i += blockDim.x) s[i] = seg[i];
      __syncthreads();
      sort_net<true>(s, n);
      for (int i = threadIdx.x; i < n; i += blockDim.x) place<G, S>(in, out, perm, s[i], t0 + i, (int32_t)c, hx, hy);
      __syncthreads();
    } else {
      sort_net<false>(seg, n);
      for (int i = threadIdx.x; i < n; i += blockDim.x) place<G, S>(in, out, perm, seg[i], t0 + i, (int32_t)c, hx, hy);
    }
  }
}

// Bin set-up, thread per cell: the input offsets [0, M] copied (the output
// offsets may be the same buffer) and the four per-cell counters and two
// totals cleared.
__global__ void k_bin_init(const int64_t* src, int64_t* dst, int64_t M, int32_t* a, int32_t* b,
                           int32_t* c, int32_t* d, int32_t* scalar, int32_t* scalar2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i <= M) dst[i] = src ? src[i] : 0;
  if (i < M) { a[i] = 0; b[i] = 0; c[i] = 0; d[i] = 0; }
  if (i == 0) { *scalar = 0; *scalar2 = 0; }
}

// The three scan passes in one block, for M <= SCAN_TILE (the 1D and 0D
// grids, where the step is launch-bound); same results as the three kernels.
__global__ __launch_bounds__(BIN_BLOCK) void k_scan_small(const int32_t* counts, int64_t M,
                                                          int64_t* offsets, int64_t* out_count,
                                                          const int64_t* in_count) {
  const int64_t base = (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int64_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t j = base + k;
    v[k] = j < M ? counts[j] : 0;
    s += v[k];
  }
  int64_t tot;
  int64_t run = block_exclusive_scan(s, &tot);
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t j = base + k;
    if (j < M) offsets[j] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) {
    offsets[M] = tot;
    if (out_count) {
      out_count[0] = tot;
      out_count[1] = in_count[1];
    }
  }
}

static void launch_scan(const int32_t* cnt, int64_t M, int64_t* out_off, int64_t* blocksums,
                        int64_t* out_count, const int64_t* in_count, hipStream_t st) {
  const int64_t nb = cdiv(M, SCAN_TILE);
  if (nb <= 1) {
    k_scan_small<<<1, BIN_BLOCK, 0, st>>>(cnt, M, out_off, out_count, in_count);
    return;
  }
  k_scan_reduce<<<nb, BIN_BLOCK, 0, st>>>(cnt, M, blocksums);
  k_scan_down<<<nb, BIN_BLOCK, 0, st>>>(cnt, M, blocksums, out_off, out_count, in_count);
}

template <typename S, bool G>
static hipError_t bin_launches(const GridP& g, const PartP<S>& in, const PartP<S>& out,
                               int64_t* offsets, const int64_t* in_offsets, char* ws,
                               const WsLayout& L, uint32_t* perm, int64_t* counters,
                               hipStream_t st) {
  int32_t* key = (int32_t*)(ws + L.key);
  int64_t* blocksums = (int64_t*)(ws + L.blocksums);
  int32_t* T9 = (int32_t*)(ws + L.t9);
  int32_t* tail_cnt = (int32_t*)(ws + L.cell_i32);
  int32_t* cursor = tail_cnt + g.M;
  int32_t* far_cnt = cursor + g.M;
  int32_t* far_cur = far_cnt + g.M;
  int32_t* nontail = far_cur + g.M;
  int32_t* cnt_total = nontail + g.M;
  int64_t* old_off = (int64_t*)(ws + L.old_off);
  int64_t* far_off = (int64_t*)(ws + L.far_off);
  int32_t* far_c = (int32_t*)(ws + L.far);
  int32_t* far_i = far_c + in.capacity;
  int32_t* far_list = far_i + in.capacity;
  int32_t* far_base = far_list + in.capacity;
  int32_t* far_total = (int32_t*)(ws + L.misc) + 8;
  int32_t* n_tail_cells = (int32_t*)(ws + L.misc) + 9;
  int32_t* tail_cells = cnt_total + g.M;
  const int64_t M = g.M;
  const Nbr nb = nbr_set(g);
  const int TAIL_GRID = 512;
  k_bin_init<<<cdiv(M + 1, 256), 256, 0, st>>>(in_offsets, old_off, M, tail_cnt, cursor, far_cnt,
                                                far_cur, far_total, n_tail_cells);
  const bool merged = M <= BIN_MERGE_MAX;
  const int64_t ngroup = cdiv(M, BIN_BLOCK / 64);
  if (merged) {
    k_bin_group_tail<S><<<ngroup + TAIL_GRID, BIN_BLOCK, 0, st>>>(
        g, nb, in, old_off, key, T9, far_cnt, far_c, far_i, far_total, tail_cnt, tail_cells,
        n_tail_cells, counters, ngroup);
  } else {
    k_bin_group<S><<<ngroup, BIN_BLOCK, 0, st>>>(g, nb, in, old_off, key, T9, far_cnt, far_c, far_i,
                                                 far_total, counters);
    k_tail_key<S><<<TAIL_GRID, BIN_BLOCK, 0, st>>>(g, in, old_off, key, tail_cnt, tail_cells,
                                                   n_tail_cells, counters);
  }
  launch_scan(far_cnt, M, far_off, blocksums, nullptr, nullptr, st);
  k_far_place<<<64, BIN_BLOCK, 0, st>>>(far_total, far_c, far_i, far_off, far_cur, far_list);
  const int far_cpw = M >= 64 * 1024 ? 64 : 1;
  k_far_sort<<<cdiv(M, (BIN_BLOCK / 64) * far_cpw), BIN_BLOCK, 0, st>>>(far_off, M, far_list,
                                                                       far_cpw);
  k_cell_bases<<<cdiv(M, BIN_BLOCK), BIN_BLOCK, 0, st>>>(g, nb, old_off, in.count, T9, far_off,
                                                          far_list, far_base, tail_cnt, nontail,
                                                          cnt_total);
  launch_scan(cnt_total, M, offsets, blocksums, out.count, in.count, st);
  k_bin_scatter<S, G><<<cdiv(M, BIN_BLOCK / 64), BIN_BLOCK, 0, st>>>(g, nb, in, out, perm, old_off, key, T9,
                                                                   offsets);
  const int FAR_GRID = 64;
  if (merged) {
    k_far_tail<S, G><<<FAR_GRID + TAIL_GRID, BIN_BLOCK, 0, st>>>(
        g, in, out, perm, far_total, far_c, far_i, far_off, far_list, far_base, old_off, key,
        offsets, nontail, cursor, perm, FAR_GRID);
  } else {
    k_far_scatter<S, G><<<FAR_GRID, BIN_BLOCK, 0, st>>>(g, in, out, perm, far_total, far_c, far_i,
                                                       far_off, far_list, far_base, offsets);
    k_tail_claim<<<TAIL_GRID, BIN_BLOCK, 0, st>>>(M, old_off, in.count, key, offsets, nontail,
                                                  cursor, perm);
  }
  k_tail_sort_copy<S, G><<<TAIL_GRID, BIN_BLOCK, 0, st>>>(g, in, out, offsets, nontail, perm,
                                                       tail_cells, n_tail_cells);
  k_tail_sort_copy_big<S, G><<<TAIL_GRID, BIN_BLOCK, 0, st>>>(g, in, out, offsets, nontail, perm,
                                                           tail_cells, n_tail_cells);
  return hipGetLastError();
}

// Copying bin (gather_perm null), or the same order recorded in
// gather_perm[slot] = input index with out.cell and out.count set and the
// particles left in place.
template <typename S>
hipError_t launch_bin(const GridP& g, const PartP<S>& in, const PartP<S>& out, int64_t* offsets,
                      const int64_t* in_offsets, char* ws, const WsLayout& L, int64_t* counters,
                      hipStream_t st, uint32_t* gather_perm) {
  if (gather_perm)
    return bin_launches<S, true>(g, in, out, offsets, in_offsets, ws, L, gather_perm, counters, st);
  return bin_launches<S, false>(g, in, out, offsets, in_offsets, ws, L, (uint32_t*)(ws + L.perm),
                                counters, st);
}

template hipError_t launch_bin<float>(const GridP&, const PartP<float>&, const PartP<float>&,
                                      int64_t*, const int64_t*, char*, const WsLayout&, int64_t*,
                                      hipStream_t, uint32_t*);
template hipError_t launch_bin<double>(const GridP&, const PartP<double>&, const PartP<double>&,
                                       int64_t*, const int64_t*, char*, const WsLayout&, int64_t*,
                                       hipStream_t, uint32_t*);

}  // namespace usp
