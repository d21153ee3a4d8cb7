// Host-side internals shared by the library's translation units: the
// simulation object, its workspace layout and the error helpers.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbf.h"
#include "lbf_device.hpp"

namespace lbfi {

// Record the error text of the calling thread and return `code`.
int fail(int code, const char* fmt, ...);

#define HIP_TRY(expr)                                                                 \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return ::lbfi::fail(LBF_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));   \
  } while (0)

constexpr size_t kAlign = 256;

inline size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Plane stride in floats.  Plane-major (rb = 0): the node count rounded up
// to 64, plus `pad`.  Row blocks of rb rows: rb rows of nx rounded up to 64,
// plus `pad`.  Which HBM channels the 34 planes of a step hit at one time
// depends on this stride; the autotuner picks the pad per size and layout.
inline long long plane_stride(int nx, int ny, int pad, int rb) {
  return (long long)round_up((size_t)nx * (size_t)(rb ? rb : ny), 64) + pad;
}

// Planes of one state array: the 27 distributions, then the 9 lagged planes.
constexpr int kStateSlots = 27 + 9;

inline int num_blocks(int ny, int rb) { return rb ? (ny + rb - 1) / rb : 1; }

// Floats from an array's base to its end when its last block holds `planes`
// planes (block stride gs).
inline long long array_floats(int nblk, long long gs, long long P, int planes) {
  return (long long)(nblk - 1) * gs + (long long)planes * P;
}

constexpr int kMaxPlanePad = 65536;

// Kernels address each block of planes with 32-bit byte offsets.
// Plane-major: the 27 distribution planes must span less than 4 GiB.
constexpr long long kMaxPlane = (0xFFFFFFFFLL / (4LL * 27)) / 64 * 64;
// Row blocks: a whole state array must.
constexpr long long kMaxStateFloats = 0xFFFFFFFFLL / 4;

inline bool valid_row_block(int rb) {
  return rb == 0 || rb == 1 || rb == 2 || rb == 4 || rb == 8 || rb == 16 || rb == 32;
}

// Every byte offset the kernels form fits 32 bits (and every node index an
// int): plane-major, the 27 distribution planes; row blocks, a whole state
// array.
inline bool fits_offsets(int nx, int ny, int pad, int rb) {
  const long long P = plane_stride(nx, ny, pad, rb);
  if (!rb) return P <= kMaxPlane;
  return array_floats(num_blocks(ny, rb), kStateSlots * P, P, kStateSlots) <= kMaxStateFloats;
}

// Worst-case number of per-block partial sums: 64-wide strips, 1 row each.
inline size_t max_blocks(int nx, int ny) { return ((size_t)(nx + 63) / 64) * (size_t)ny; }

// Rows per chunk of the column-profile partial sums.
constexpr int kProfileChunk = 64;

struct Layout {
  size_t dist[2], lag[2], stat, fields, wall, red[2], redfinal, prof, total;
  int wstride;
};

Layout make_layout(int nx, int ny, int pad, int rb);

}  // namespace lbfi

struct lbf_sim {
  lbf_params prm;
  lbf::Geo G;
  lbf::Phys ph;
  lbfi::Layout L;
  hipStream_t stream;
  char* ws;
  bool owns_ws;
  int cur;           // which distribution / lag buffer holds the current state
  bool have_geo, have_init;
  bool from_fields;  // the state was set by lbf_init_fields (not loaded)
  int tile_x, tile_y;
  long long step;
  bool have_budget;  // red[0] holds the budget of the last step
  int budget_blocks;
  bool timing;
  double last_ms;
  hipEvent_t ev0, ev1;
  double* host_red;  // pinned host buffer for reductions
};

namespace lbfi {

inline float* fptr(lbf_sim* s, size_t off) { return reinterpret_cast<float*>(s->ws + off); }
inline double* dptr(lbf_sim* s, size_t off) { return reinterpret_cast<double*>(s->ws + off); }

// Launch the step kernel (MODE_STEP, MODE_FIELDS or MODE_STEP_MOM) with the
// simulation's tile shape on explicit buffers, on stream `st`.
int launch_step_args(lbf_sim* s, int mode, bool red, lbf::BufArgs B, hipStream_t st);

}  // namespace lbfi
