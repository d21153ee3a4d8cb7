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

// Plane stride: nx * ny rounded up to 64 floats (256 bytes).
// Floats between consecutive planes: the node count rounded up to 64, plus
// `pad` (a multiple of 64).  Which HBM channels the 34 planes of a step hit
// at one time depends on this stride; the autotuner picks the pad per size.
inline long long plane_stride(int nx, int ny, int pad) {
  return (long long)round_up((size_t)nx * ny, 64) + pad;
}

constexpr int kMaxPlanePad = 65536;

// Kernels address each block of planes with 32-bit byte offsets: the 27
// distribution planes must span less than 4 GiB.
constexpr long long kMaxPlane = (0xFFFFFFFFLL / (4LL * 27)) / 64 * 64;

// Worst-case number of per-block partial sums: 64-wide strips, 1 row each.
inline size_t max_blocks(int nx, int ny) { return ((size_t)(nx + 63) / 64) * (size_t)ny; }

// Rows per chunk of the column-profile partial sums.
constexpr int kProfileChunk = 64;

struct Layout {
  size_t dist[2], lag[2], stat, fields, wall, red[2], redfinal, prof, total;
  int wstride;
};

Layout make_layout(int nx, int ny);

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
