// usp_noalloc.hip -- usp_update_noalloc: the fused particle phase of
// usp_update with its scratch (the tile index and the injection's face
// counts, offsets and totals) in a fixed device array instead of a caller
// workspace, for callers that cannot allocate device memory.
#include <mutex>

#include "usp_internal.h"

namespace usp {
namespace {

// The scratch array: one copy per GPU, held until the process ends.  In
// host code `scratch` names a host-side stand-in, never its device copy:
// kernels and copies get the address hipGetSymbolAddress gives for the
// current device (scratch_ptr below).
static __device__ __align__(256) char scratch[USP_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char* scratch_dev[MAX_DEVICES];

// Device address of the scratch array on the current device, looked up once
// per device (with that device current) and cached; nullptr on error.
char* scratch_ptr() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_dev[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return nullptr;
    scratch_dev[dev] = (char*)p;
  }
  return scratch_dev[dev];
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

// The parts of the workspace layout the fused particle phase uses, packed
// for this grid and capacity: face counts, face offsets, injection totals,
// and the tile index of the window update_tile gives.  Returns the bytes
// needed.
template <typename S>
size_t noalloc_layout(const GridP& g, int64_t capacity, WsLayout* L) {
  const int stage = sizeof(S) == 4 ? UPDATE_STAGE_F32 : UPDATE_STAGE_F64;
  const int64_t ntiles = cdiv(capacity, update_tile(stage, capacity, g.M));
  const int nf = n_faces(g);
  size_t o = 0;
  *L = WsLayout{};
  L->face_cnt = o; o = align256(o + sizeof(int32_t) * (size_t)(nf + 1));
  L->face_off = o; o = align256(o + sizeof(int64_t) * (size_t)(nf + 1));
  L->misc = o; o = align256(o + sizeof(int64_t) * 8);
  L->tiles = o; o = align256(o + sizeof(int32_t) * (size_t)(ntiles + 2));
  L->total = o;
  return o;
}

template <typename S>
usp_status noalloc_update(const usp_grid* grid, const usp_gas* gas, const usp_bc* bc, double dt,
                          const double* cs, const int64_t* offsets, usp_particles* p,
                          uint64_t seed, uint64_t step, int64_t* counters, hipStream_t st) {
  const GridP g = make_grid(grid);
  WsLayout L;
  if (noalloc_layout<S>(g, p->capacity, &L) > (size_t)USP_NOALLOC_SCRATCH_BYTES)
    return USP_ESCRATCH;
  char* ws = scratch_ptr();
  if (!ws) return USP_EDEVICE;
  const hipError_t e = launch_update<S>(g, make_gas(gas), make_bc(bc), dt, cs, offsets,
                                        make_parts<S>(p), seed, step, ws, L, counters, st);
  return e == hipSuccess ? USP_OK : USP_EDEVICE;
}

}  // namespace
}  // namespace usp

using namespace usp;

extern "C" usp_status usp_update_noalloc(const usp_grid* grid, const usp_gas* gas,
                                         const usp_bc* bc, double dt, const double* cs,
                                         const int64_t* offsets, usp_particles* p, uint64_t seed,
                                         uint64_t step, int64_t* counters, void* stream) {
  // the argument checks of usp_update (there is no ws to check)
  if (!update_args_ok(grid, gas, bc, dt, cs, offsets, p)) return USP_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  return p->prec == USP_F32
             ? noalloc_update<float>(grid, gas, bc, dt, cs, offsets, p, seed, step, counters, st)
             : noalloc_update<double>(grid, gas, bc, dt, cs, offsets, p, seed, step, counters, st);
}
