// Cahn-Hilliard smoothing of a binary solid image (contract in
// include/lbf_pre.h).  One fused pass per Euler step: a workgroup loads its
// tile of c with a two-node halo into LDS, computes the chemical potential
// on the tile plus a one-node ring, and updates c on the tile, so HBM sees
// one read and one write of c per node and step (the halo re-reads hit L2:
// tiles are dealt to the XCDs in contiguous bands).  Each lane owns columns
// of the boxes and slides a window of registers along them.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "lbf_pre.h"
#include "lbf_sim.hpp"
#include "lbf_step.hpp"

using lbfi::fail;

// Scratch of the allocation-free entry point (lbf_ch_smooth_noalloc): the two
// planes of c for images of up to kStaticNodesCH nodes.  Every device the
// library runs on holds its own copy (32 MiB) from the module's load until
// the process ends.  In host code the array's name is not a device address:
// kernels and copies use the per-device address that hipGetSymbolAddress
// returns.
constexpr long long kStaticNodesCH = 1LL << 22;
static __device__ __align__(256) float scratch[2 * kStaticNodesCH];

namespace {

constexpr long long kMaxNodesCH = 0x7FFFFFFFLL;

// tiles: 64 x 16 nodes in 2D, 32 x 8 x 4 in 3D (1024 nodes, 4 per lane)
constexpr int kTX2 = 64, kTY2 = 16;
constexpr int kTX3 = 32, kTY3 = 8, kTZ3 = 4;

struct ChGeo {
  int n[3];
  int per[3];
};

// Index of v along an axis of n nodes: wrapped (any offset), or clamped to
// the first and last node (the mirror ghost).
__device__ __forceinline__ int wrap_or_clamp(int v, int n, int periodic) {
  if (v >= 0 && v < n) return v;   // interior: no division
  if (periodic) {
    v %= n;
    return v < 0 ? v + n : v;
  }
  return v < 0 ? 0 : n - 1;
}

// 6 sum_i w_i (X(x + c_i) - X(x)) over an LDS box with row length SX and
// plane size SXY: D2Q9 (DIM 2) or D3Q19 (DIM 3) weights.
template <int DIM, int SX, int SXY>
__device__ __forceinline__ float lds_laplacian(const float* X, int i) {
  const float xc = X[i];
  float axis = 0.0f, diag = 0.0f;
  constexpr int zlo = DIM == 3 ? -1 : 0, zhi = DIM == 3 ? 1 : 0;
#pragma unroll
  for (int dz = zlo; dz <= zhi; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
      for (int dx = -1; dx <= 1; ++dx) {
        const int m = (dx != 0) + (dy != 0) + (dz != 0);
        if (m == 0 || m == 3) continue;
        const float v = X[i + dz * SXY + dy * SX + dx] - xc;
        if (m == 1) axis += v;
        else diag += v;
      }
  // D2Q9: 1/9 axes, 1/36 diagonals; D3Q19: 1/18 axes, 1/36 face diagonals
  constexpr float wa = DIM == 3 ? 1.0f / 18.0f : 1.0f / 9.0f;
  return 6.0f * (wa * axis + (1.0f / 36.0f) * diag);
}

// The 2D step with the work laid out by columns: lane (tx, ty) of a 64 x 4
// block owns column tx of the tile and a run of consecutive rows, and slides
// a 3 x 3 window of registers up its column, so each stencil reads three new
// LDS values instead of nine and the box indices are formed once per column.
// Same operands, in the same order, as lds_laplacian<2, ...>.
template <int TX, int TY>
__global__ __launch_bounds__(256) void k_ch_step2(ChGeo G, const float* __restrict__ c,
                                                  float* __restrict__ cn, float A, float kappa,
                                                  float dtM, int ntx, int ntiles) {
  static_assert(TX == 64 && TY % 4 == 0, "64 lanes per row, four row groups");
  constexpr int LX = TX + 4, LY = TY + 4;   // c box, halo 2
  constexpr int MX = TX + 2, MY = TY + 2;   // mu box, halo 1
  constexpr float wa = 1.0f / 9.0f, wd = 1.0f / 36.0f;
  __shared__ float cs[LX * LY];
  __shared__ float ms[MX * MY];
  const int t = lbf::xcd_tile(blockIdx.x, ntiles);
  const int x0 = (t % ntx) * TX, y0 = (t / ntx) * TY;
  const int nx = G.n[0], ny = G.n[1];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  {
    const int gx = wrap_or_clamp(x0 + tx - 2, nx, G.per[0]);
    for (int ly = ty; ly < LY; ly += 4) {
      const int gy = wrap_or_clamp(y0 + ly - 2, ny, G.per[1]);
      cs[ly * LX + tx] = c[gy * nx + gx];
    }
    const int e = threadIdx.x;   // the last four columns of the box
    if (e < 4 * LY) {
      const int lx = TX + (e & 3), ly = e >> 2;
      const int gx2 = wrap_or_clamp(x0 + lx - 2, nx, G.per[0]);
      const int gy2 = wrap_or_clamp(y0 + ly - 2, ny, G.per[1]);
      cs[ly * LX + lx] = c[gy2 * nx + gx2];
    }
  }
  __syncthreads();
  {
    // mu on rows [r0, r1) of column tx; the window holds c rows my .. my + 2
    // of box columns tx .. tx + 2 (centre (my + 1, tx + 1))
    constexpr int RG = (MY + 3) / 4;
    const int r0 = ty * RG, r1 = min(r0 + RG, MY);
    float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, b0 = 0.0f, b1 = 0.0f, b2 = 0.0f;
    if (r0 < r1) {
      a0 = cs[r0 * LX + tx]; a1 = cs[r0 * LX + tx + 1]; a2 = cs[r0 * LX + tx + 2];
      b0 = cs[(r0 + 1) * LX + tx]; b1 = cs[(r0 + 1) * LX + tx + 1]; b2 = cs[(r0 + 1) * LX + tx + 2];
    }
    for (int my = r0; my < r1; ++my) {
      const float c0 = cs[(my + 2) * LX + tx], c1 = cs[(my + 2) * LX + tx + 1],
                  c2 = cs[(my + 2) * LX + tx + 2];
      const float xc = b1;
      float axis = 0.0f, diag = 0.0f;
      diag += a0 - xc; axis += a1 - xc; diag += a2 - xc;
      axis += b0 - xc; axis += b2 - xc;
      diag += c0 - xc; axis += c1 - xc; diag += c2 - xc;
      const float lap = 6.0f * (wa * axis + wd * diag);
      ms[my * MX + tx] = A * (xc * xc * xc - xc) - kappa * lap;
      a0 = b0; a1 = b1; a2 = b2;
      b0 = c0; b1 = c1; b2 = c2;
    }
    const int e = threadIdx.x;   // the last two columns of the mu box
    if (e < 2 * MY) {
      const int mx = TX + (e & 1), my = e >> 1;
      const int j = (my + 1) * LX + mx + 1;
      const float cc = cs[j];
      ms[my * MX + mx] = A * (cc * cc * cc - cc) - kappa * lds_laplacian<2, LX, LX * LY>(cs, j);
    }
  }
  __syncthreads();
  if ((!G.per[0] && (x0 == 0 || x0 + TX >= nx)) || (!G.per[1] && (y0 == 0 || y0 + TY >= ny))) {
    // beyond a mirror wall the potential is that of the first node
    for (int i = threadIdx.x; i < MX * MY; i += 256) {
      const int mx = i % MX, my = i / MX;
      const int gx = x0 + mx - 1, gy = y0 + my - 1;
      const int sx = G.per[0] ? gx : min(max(gx, 0), nx - 1);
      const int sy = G.per[1] ? gy : min(max(gy, 0), ny - 1);
      if (sx != gx || sy != gy) ms[i] = ms[(sy - y0 + 1) * MX + sx - x0 + 1];
    }
    __syncthreads();
  }
  {
    // update on rows [o0, o0 + TY / 4) of column tx; window over mu rows
    constexpr int RO = TY / 4;
    const int o0 = ty * RO, gx = x0 + tx;
    float a0 = ms[o0 * MX + tx], a1 = ms[o0 * MX + tx + 1], a2 = ms[o0 * MX + tx + 2];
    float b0 = ms[(o0 + 1) * MX + tx], b1 = ms[(o0 + 1) * MX + tx + 1],
          b2 = ms[(o0 + 1) * MX + tx + 2];
    for (int oy = o0; oy < o0 + RO; ++oy) {
      const float c0 = ms[(oy + 2) * MX + tx], c1 = ms[(oy + 2) * MX + tx + 1],
                  c2 = ms[(oy + 2) * MX + tx + 2];
      const float xc = b1;
      float axis = 0.0f, diag = 0.0f;
      diag += a0 - xc; axis += a1 - xc; diag += a2 - xc;
      axis += b0 - xc; axis += b2 - xc;
      diag += c0 - xc; axis += c1 - xc; diag += c2 - xc;
      const float lap = 6.0f * (wa * axis + wd * diag);
      const int gy = y0 + oy;
      if (gx < nx && gy < ny) cn[gy * nx + gx] = cs[(oy + 2) * LX + tx + 2] + dtM * lap;
      a0 = b0; a1 = b1; a2 = b2;
      b0 = c0; b1 = c1; b2 = c2;
    }
  }
}

// Laplacian of the centre of three 3 x 3 slices (z - 1, z, z + 1; entry
// 3 (dy + 1) + dx + 1) with the D3Q19 weights, accumulated in the order of
// lds_laplacian<3, ...>.
__device__ __forceinline__ float slice_laplacian19(const float* p, const float* q,
                                                   const float* r) {
  const float xc = q[4];
  float axis = 0.0f, diag = 0.0f;
  diag += p[1] - xc; diag += p[3] - xc; axis += p[4] - xc; diag += p[5] - xc; diag += p[7] - xc;
  diag += q[0] - xc; axis += q[1] - xc; diag += q[2] - xc;
  axis += q[3] - xc; axis += q[5] - xc;
  diag += q[6] - xc; axis += q[7] - xc; diag += q[8] - xc;
  diag += r[1] - xc; diag += r[3] - xc; axis += r[4] - xc; diag += r[5] - xc; diag += r[7] - xc;
  return 6.0f * ((1.0f / 18.0f) * axis + (1.0f / 36.0f) * diag);
}

// the 3 x 3 neighbourhood of (x, y) in slice z of an LDS box
template <int SX, int SXY>
__device__ __forceinline__ void load_slice(const float* X, int x, int y, int z, float* out) {
#pragma unroll
  for (int dy = -1; dy <= 1; ++dy)
#pragma unroll
    for (int dx = -1; dx <= 1; ++dx) out[(dy + 1) * 3 + dx + 1] = X[z * SXY + (y + dy) * SX + x + dx];
}

// The 3D step with the work laid out by columns along z: a lane owns an
// (x, y) column of a box and slides three slices of its 3 x 3 neighbourhood
// up the column, so each stencil reads nine new LDS values instead of
// eighteen and the box indices are formed once per column.
template <int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_ch_step3(ChGeo G, const float* __restrict__ c,
                                                  float* __restrict__ cn, float A, float kappa,
                                                  float dtM, int ntx, int nty, int ntiles) {
  static_assert(TX * TY == 256, "one output column per lane");
  constexpr int LX = TX + 4, LY = TY + 4, LZ = TZ + 4;   // c box, halo 2
  constexpr int MX = TX + 2, MY = TY + 2, MZ = TZ + 2;   // mu box, halo 1
  __shared__ float cs[LX * LY * LZ];
  __shared__ float ms[MX * MY * MZ];
  const int t = lbf::xcd_tile(blockIdx.x, ntiles);
  const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY, z0 = (t / (ntx * nty)) * TZ;
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  for (int col = threadIdx.x; col < LX * LY; col += 256) {
    const int lx = col % LX, ly = col / LX;
    const int gx = wrap_or_clamp(x0 + lx - 2, nx, G.per[0]);
    const int gy = wrap_or_clamp(y0 + ly - 2, ny, G.per[1]);
#pragma unroll
    for (int lz = 0; lz < LZ; ++lz) {
      const int gz = wrap_or_clamp(z0 + lz - 2, nz, G.per[2]);
      cs[(lz * LY + ly) * LX + lx] = c[(gz * ny + gy) * nx + gx];   // < 2^31 nodes
    }
  }
  __syncthreads();
  for (int col = threadIdx.x; col < MX * MY; col += 256) {
    const int mx = col % MX, my = col / MX;
    float p[9], q[9], r[9];
    load_slice<LX, LX * LY>(cs, mx + 1, my + 1, 0, p);
    load_slice<LX, LX * LY>(cs, mx + 1, my + 1, 1, q);
#pragma unroll
    for (int mz = 0; mz < MZ; ++mz) {
      load_slice<LX, LX * LY>(cs, mx + 1, my + 1, mz + 2, r);
      const float cc = q[4];
      ms[(mz * MY + my) * MX + mx] = A * (cc * cc * cc - cc) - kappa * slice_laplacian19(p, q, r);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        p[k] = q[k];
        q[k] = r[k];
      }
    }
  }
  __syncthreads();
  const bool at_wall = (!G.per[0] && (x0 == 0 || x0 + TX >= nx)) ||
                       (!G.per[1] && (y0 == 0 || y0 + TY >= ny)) ||
                       (!G.per[2] && (z0 == 0 || z0 + TZ >= nz));
  if (at_wall) {
    // beyond a mirror wall the potential is that of the first node
    for (int i = threadIdx.x; i < MX * MY * MZ; i += 256) {
      const int mx = i % MX, my = (i / MX) % MY, mz = i / (MX * MY);
      const int gx = x0 + mx - 1, gy = y0 + my - 1, gz = z0 + mz - 1;
      const int sx = G.per[0] ? gx : min(max(gx, 0), nx - 1);
      const int sy = G.per[1] ? gy : min(max(gy, 0), ny - 1);
      const int sz = G.per[2] ? gz : min(max(gz, 0), nz - 1);
      if (sx != gx || sy != gy || sz != gz)
        ms[i] = ms[((sz - z0 + 1) * MY + sy - y0 + 1) * MX + sx - x0 + 1];
    }
    __syncthreads();
  }
  {
    const int ox = threadIdx.x % TX, oy = threadIdx.x / TX;
    const int gx = x0 + ox, gy = y0 + oy;
    float p[9], q[9], r[9];
    load_slice<MX, MX * MY>(ms, ox + 1, oy + 1, 0, p);
    load_slice<MX, MX * MY>(ms, ox + 1, oy + 1, 1, q);
#pragma unroll
    for (int oz = 0; oz < TZ; ++oz) {
      load_slice<MX, MX * MY>(ms, ox + 1, oy + 1, oz + 2, r);
      const int gz = z0 + oz;
      if (gx < nx && gy < ny && gz < nz)
        cn[(gz * ny + gy) * nx + gx] = cs[((oz + 2) * LY + oy + 2) * LX + ox + 2] +
                                       dtM * slice_laplacian19(p, q, r);
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        p[k] = q[k];
        q[k] = r[k];
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_ch_init(const uint8_t* __restrict__ s,
                                                 float* __restrict__ c, int N) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < N) c[k] = s[k] ? 1.0f : -1.0f;
}

__global__ __launch_bounds__(256) void k_ch_final(const float* __restrict__ c,
                                                  float* __restrict__ phi0, int N) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k < N) phi0[k] = fminf(fmaxf(0.5f * (1.0f + c[k]), 0.0f), 1.0f);
}

size_t plane_bytes(long long n) { return ((size_t)n * 4 + 255) / 256 * 256; }

int ceil_div(int a, int b) { return (a + b - 1) / b; }

// Checks shared by both entry points.
int ch_validate(const lbf_ch_params* p, int32_t iterations) {
  if (!p) return fail(LBF_EINVAL, "NULL argument");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(LBF_EINVAL, "image size %d x %d x %d", p->nx, p->ny, p->nz);
  const long long n = (long long)p->nx * p->ny * p->nz;
  if (n > kMaxNodesCH) return fail(LBF_EINVAL, "image of %lld nodes exceeds 2^31 - 1", n);
  if (iterations < 0) return fail(LBF_EINVAL, "iterations %d", iterations);
  if (!(p->A >= 0.0) || !(p->kappa >= 0.0) || !(p->mobility >= 0.0) || !(p->dt > 0.0) ||
      !std::isfinite(p->A) || !std::isfinite(p->kappa) || !std::isfinite(p->mobility) ||
      !std::isfinite(p->dt))
    return fail(LBF_EINVAL, "A, kappa, mobility must be >= 0 and dt > 0, all finite");
  const double lmax = 16.0 / 3.0;
  const double amp = p->dt * p->mobility * lmax * (2.0 * p->A + p->kappa * lmax);
  if (amp > 2.0)
    return fail(LBF_EINVAL, "dt = %g is outside the explicit scheme's stability bound "
                            "(dt M 16/3 (2 A + kappa 16/3) = %g > 2)", p->dt, amp);
  return LBF_OK;
}

// The smoothing itself on two planes c0, c1 of at least plane_bytes(n) each
// (c1 also stages a host image and, when phi0 is host memory, the result).
// Stream-ordered; synchronises only when host memory is read or written.
int ch_run(const lbf_ch_params* p, const uint8_t* solid, bool solid_on_device, float* phi0,
           bool phi0_on_device, int32_t iterations, hipStream_t st, float* c0, float* c1) {
  const int N = p->nx * p->ny * p->nz;
  float* c[2] = {c0, c1};
  const int nb = (N + 255) / 256;
  const ChGeo G{{p->nx, p->ny, p->nz},
                {p->periodic[0] ? 1 : 0, p->periodic[1] ? 1 : 0, p->periodic[2] ? 1 : 0}};
  const bool is3d = p->nz > 1;
  const int ntx = ceil_div(p->nx, is3d ? kTX3 : kTX2), nty = ceil_div(p->ny, is3d ? kTY3 : kTY2);
  const int ntz = is3d ? ceil_div(p->nz, kTZ3) : 1;
  const int ntiles = ntx * nty * ntz;
  const float A = (float)p->A, kap = (float)p->kappa, dtM = (float)(p->dt * p->mobility);
  const uint8_t* s = solid;
  if (!solid_on_device) {
    HIP_TRY(hipMemcpyAsync(c[1], solid, (size_t)N, hipMemcpyHostToDevice, st));
    s = (const uint8_t*)c[1];
  }
  hipLaunchKernelGGL(k_ch_init, dim3(nb), dim3(256), 0, st, s, c[0], N);
  HIP_TRY(hipGetLastError());
  int cur = 0;
  for (int it = 0; it < iterations; ++it) {
    if (is3d)
      hipLaunchKernelGGL((k_ch_step3<kTX3, kTY3, kTZ3>), dim3(ntiles), dim3(256), 0, st, G,
                         c[cur], c[1 - cur], A, kap, dtM, ntx, nty, ntiles);
    else
      hipLaunchKernelGGL((k_ch_step2<kTX2, kTY2>), dim3(ntiles), dim3(256), 0, st, G, c[cur],
                         c[1 - cur], A, kap, dtM, ntx, ntiles);
    HIP_TRY(hipGetLastError());
    cur = 1 - cur;
  }
  float* dst = phi0_on_device ? phi0 : c[1 - cur];
  hipLaunchKernelGGL(k_ch_final, dim3(nb), dim3(256), 0, st, c[cur], dst, N);
  HIP_TRY(hipGetLastError());
  if (!phi0_on_device)
    HIP_TRY(hipMemcpyAsync(phi0, dst, (size_t)N * 4, hipMemcpyDeviceToHost, st));
  if (!phi0_on_device || !solid_on_device) HIP_TRY(hipStreamSynchronize(st));
  return LBF_OK;
}

// Address of `scratch` per device, looked up once per device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices];

int scratch_on_current_device(float** out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LBF_EINVAL, "device %d: the scratch table holds devices 0..%d", dev,
                kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(LBF_EHIP, "hipGetSymbolAddress(scratch) on device %d failed: %s", dev,
                  hipGetErrorString(e));
    g_scratch[dev] = (float*)p;
  }
  *out = g_scratch[dev];
  return LBF_OK;
}

}  // namespace

extern "C" {

size_t lbf_ch_workspace_bytes(int32_t nx, int32_t ny, int32_t nz) {
  if (nx < 1 || ny < 1 || nz < 1) return 0;
  const long long n = (long long)nx * ny * nz;
  if (n > kMaxNodesCH) return 0;
  // c, two ping-pong planes; a host image is staged in the second one
  return 2 * plane_bytes(n);
}

int lbf_ch_smooth(const lbf_ch_params* p, const uint8_t* solid, int32_t solid_on_device,
                  float* phi0, int32_t phi0_on_device, int32_t iterations, void* stream,
                  void* workspace, size_t workspace_bytes) {
  if (!solid || !phi0) return fail(LBF_EINVAL, "NULL argument");
  int rc = ch_validate(p, iterations);
  if (rc != LBF_OK) return rc;
  const long long n = (long long)p->nx * p->ny * p->nz;
  const size_t need = lbf_ch_workspace_bytes(p->nx, p->ny, p->nz);
  hipStream_t st = (hipStream_t)stream;
  char* ws = (char*)workspace;
  bool owns = false;
  if (ws) {
    if (workspace_bytes < need || (uintptr_t)ws % 256)
      return fail(LBF_ENOMEM, "workspace too small or not 256-byte aligned");
  } else {
    if (hipMalloc((void**)&ws, need) != hipSuccess) return fail(LBF_ENOMEM, "hipMalloc failed");
    owns = true;
  }
  const size_t pb = plane_bytes(n);
  rc = ch_run(p, solid, solid_on_device != 0, phi0, phi0_on_device != 0, iterations, st,
              (float*)ws, (float*)(ws + pb));
  if (owns) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(ws);
  }
  return rc;
}

size_t lbf_ch_noalloc_max_nodes(void) { return (size_t)kStaticNodesCH; }

int lbf_ch_smooth_noalloc(const lbf_ch_params* p, const uint8_t* solid_dev, float* phi0_dev,
                          int32_t iterations, void* stream) {
  if (!solid_dev || !phi0_dev) return fail(LBF_EINVAL, "NULL argument");
  int rc = ch_validate(p, iterations);
  if (rc != LBF_OK) return rc;
  const long long n = (long long)p->nx * p->ny * p->nz;
  if (n > kStaticNodesCH)
    return fail(LBF_EINVAL, "image of %lld nodes exceeds the allocation-free limit of %lld "
                            "nodes (use lbf_ch_smooth with a workspace)", n, kStaticNodesCH);
  float* c = nullptr;
  rc = scratch_on_current_device(&c);
  if (rc != LBF_OK) return rc;
  // every node of both planes that the smoothing reads is written first
  // (k_ch_init fills c0 from the image), so nothing needs clearing
  return ch_run(p, solid_dev, true, phi0_dev, true, iterations, (hipStream_t)stream, c,
                c + plane_bytes(n) / sizeof(float));
}

}  // extern "C"
