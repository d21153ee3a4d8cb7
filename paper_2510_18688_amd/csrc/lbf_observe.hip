// Column and row profiles of the current state (C ABI; contract in
// include/lbf.h).  The figure-level observables of the freezing runs (front
// height and final solid height, Sec. 4.2 and Table 1; drop height on a
// curved substrate, Sec. 4.4; radius and height of the three-phase contact
// line, Fig. 6; solid fraction against the Fourier number, Fig. 13) are sums
// and level crossings of the ice fraction f_s and of the phase-change
// fraction chi along columns and rows.  The read-out pass of the step kernel
// writes the fields; these kernels reduce them in FP64, in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "lbf.h"
#include "lbf_device.hpp"
#include "lbf_sim.hpp"

using namespace lbf;
using namespace lbfi;

namespace {

// Highest crossing of the level 1/2 between rows y and y + 1 (value v at y,
// vn at y + 1): the linear interpolate when v >= 1/2 > vn; the top row itself
// when it is at or above the level.
__device__ __forceinline__ void crossing(float v, float vn, bool top_row, int y, double& best) {
  if (v >= 0.5f && (top_row || vn < 0.5f))
    best = top_row ? (double)y : (double)y + ((double)v - 0.5) / ((double)v - (double)vn);
}

// Per column and chunk of kProfileChunk rows: sums of f_s and chi and the
// highest level crossings of each inside the chunk.
__global__ __launch_bounds__(256) void k_col_partial(Geo G, const float* __restrict__ fields,
                                                     double* __restrict__ part) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, ch = blockIdx.y;
  if (x >= G.nx) return;
  const size_t P = (size_t)G.PF;   // read-out planes are plane-major
  const float* fs = fields + (size_t)LBF_FIELD_FS * P;
  const float* chi = fields + (size_t)LBF_FIELD_CHI * P;
  const int y0 = ch * kProfileChunk, y1 = min(y0 + kProfileChunk, G.ny);
  double s_ice = 0.0, s_pcm = 0.0, top_pcm = -1.0, top_ice = -1.0;
  for (int y = y0; y < y1; ++y) {
    const size_t k = (size_t)y * G.nx + x;
    const bool top_row = y + 1 >= G.ny;
    const float a = fs[k], c = chi[k];
    const float an = top_row ? 0.0f : fs[k + G.nx], cn = top_row ? 0.0f : chi[k + G.nx];
    s_ice += a;
    s_pcm += c;
    crossing(c, cn, top_row, y, top_pcm);
    crossing(a, an, top_row, y, top_ice);
  }
  double* o = part + ((size_t)ch * G.nx + x) * 4;
  o[0] = s_ice;
  o[1] = s_pcm;
  o[2] = top_pcm;
  o[3] = top_ice;
}

// Per column: chunk partials summed in chunk order; highest crossing.
__global__ __launch_bounds__(256) void k_col_final(Geo G, const double* __restrict__ part,
                                                   int nchunk, double* __restrict__ col) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  if (x >= G.nx) return;
  double s_ice = 0.0, s_pcm = 0.0, top_pcm = -1.0, top_ice = -1.0;
  for (int ch = 0; ch < nchunk; ++ch) {
    const double* o = part + ((size_t)ch * G.nx + x) * 4;
    s_ice += o[0];
    s_pcm += o[1];
    top_pcm = fmax(top_pcm, o[2]);
    top_ice = fmax(top_ice, o[3]);
  }
  col[LBF_COL_ICE * G.nx + x] = s_ice;
  col[LBF_COL_PCM * G.nx + x] = s_pcm;
  col[LBF_COL_PCM_TOP * G.nx + x] = top_pcm;
  col[LBF_COL_ICE_TOP * G.nx + x] = top_ice;
}

// Per row (one workgroup of 256 lanes): sums of f_s and chi and the outer
// 1/2-crossings of each (leftmost rising, rightmost falling edge, linear
// interpolation; the domain edge node itself when it is at or above 1/2);
// lanes stride over x, then a fixed-order tree (sums) and min / max (edges).
__global__ __launch_bounds__(256) void k_row_profiles(Geo G, const float* __restrict__ fields,
                                                      double* __restrict__ row) {
  __shared__ double s[6][256];
  const int y = blockIdx.x, l = threadIdx.x;
  const size_t P = (size_t)G.PF;   // read-out planes are plane-major
  const float* fs = fields + (size_t)LBF_FIELD_FS * P + (size_t)y * G.nx;
  const float* chi = fields + (size_t)LBF_FIELD_CHI * P + (size_t)y * G.nx;
  const double none_left = 1e300, none_right = -1e300;
  double a = 0.0, c = 0.0;
  double cl = none_left, cr = none_right, al = none_left, ar = none_right;
  for (int x = l; x < G.nx; x += 256) {
    const float va = fs[x], vc = chi[x];
    a += va;
    c += vc;
    const bool first = x == 0, last = x + 1 >= G.nx;
    const float pa = first ? 0.0f : fs[x - 1], pc = first ? 0.0f : chi[x - 1];
    const float na = last ? 0.0f : fs[x + 1], nc = last ? 0.0f : chi[x + 1];
    if (vc >= 0.5f && (first || pc < 0.5f))
      cl = fmin(cl, first ? 0.0 : (double)x - ((double)vc - 0.5) / ((double)vc - (double)pc));
    if (vc >= 0.5f && (last || nc < 0.5f))
      cr = fmax(cr, last ? (double)x : (double)x + ((double)vc - 0.5) / ((double)vc - (double)nc));
    if (va >= 0.5f && (first || pa < 0.5f))
      al = fmin(al, first ? 0.0 : (double)x - ((double)va - 0.5) / ((double)va - (double)pa));
    if (va >= 0.5f && (last || na < 0.5f))
      ar = fmax(ar, last ? (double)x : (double)x + ((double)va - 0.5) / ((double)va - (double)na));
  }
  s[0][l] = a;
  s[1][l] = c;
  s[2][l] = cl;
  s[3][l] = cr;
  s[4][l] = al;
  s[5][l] = ar;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (l < w) {
      s[0][l] += s[0][l + w];
      s[1][l] += s[1][l + w];
      s[2][l] = fmin(s[2][l], s[2][l + w]);
      s[3][l] = fmax(s[3][l], s[3][l + w]);
      s[4][l] = fmin(s[4][l], s[4][l + w]);
      s[5][l] = fmax(s[5][l], s[5][l + w]);
    }
    __syncthreads();
  }
  if (l == 0) {
    row[LBF_ROW_ICE * G.ny + y] = s[0][0];
    row[LBF_ROW_PCM * G.ny + y] = s[1][0];
    row[LBF_ROW_PCM_LEFT * G.ny + y] = s[2][0] == none_left ? -1.0 : s[2][0];
    row[LBF_ROW_PCM_RIGHT * G.ny + y] = s[3][0] == none_right ? -1.0 : s[3][0];
    row[LBF_ROW_ICE_LEFT * G.ny + y] = s[4][0] == none_left ? -1.0 : s[4][0];
    row[LBF_ROW_ICE_RIGHT * G.ny + y] = s[5][0] == none_right ? -1.0 : s[5][0];
  }
}

}  // namespace

extern "C" {

int lbf_profiles(lbf_sim* s, double* col, double* row, int32_t dst_on_device) {
  if (!s || !col || !row) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  // read-out fields of the current state
  BufArgs B{};
  B.din = fptr(s, s->L.dist[s->cur]);
  B.dout = fptr(s, s->L.dist[1 - s->cur]);
  B.lin = fptr(s, s->L.lag[s->cur]);
  B.lout = fptr(s, s->L.lag[1 - s->cur]);
  B.stat = fptr(s, s->L.stat);
  B.wallT = fptr(s, s->L.wall);
  B.wstride = s->L.wstride;
  B.fields = fptr(s, s->L.fields);
  B.red = nullptr;
  int rc = launch_step_args(s, MODE_FIELDS, false, B, s->stream);
  if (rc) return rc;
  const int nx = s->G.nx, ny = s->G.ny;
  const int nchunk = (ny + kProfileChunk - 1) / kProfileChunk;
  double* part = dptr(s, s->L.prof);
  double* dcol = part + (size_t)nchunk * nx * 4;
  double* drow = dcol + LBF_NCOL * (size_t)nx;
  const float* F = fptr(s, s->L.fields);
  hipLaunchKernelGGL(k_col_partial, dim3((nx + 255) / 256, nchunk), dim3(256), 0, s->stream,
                     s->G, F, part);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_col_final, dim3((nx + 255) / 256), dim3(256), 0, s->stream, s->G,
                     (const double*)part, nchunk, dcol);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_row_profiles, dim3(ny), dim3(256), 0, s->stream, s->G, F, drow);
  HIP_TRY(hipGetLastError());
  const hipMemcpyKind kind = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  HIP_TRY(hipMemcpyAsync(col, dcol, LBF_NCOL * (size_t)nx * sizeof(double), kind, s->stream));
  HIP_TRY(hipMemcpyAsync(row, drow, LBF_NROW * (size_t)ny * sizeof(double), kind, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

}  // extern "C"
