// Cahn-Hilliard smoothing of a binary solid image (contract in
// include/lbf_pre.h).  One fused pass per Euler step: a workgroup loads its
// tile of c with a two-node halo into LDS, computes the chemical potential
// on the tile plus a one-node ring, and updates c on the tile, so HBM sees
// one read and one write of c per node and step (the halo re-reads hit L2:
// tiles are dealt to the XCDs in contiguous bands).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "lbf_pre.h"
#include "lbf_sim.hpp"
#include "lbf_step.hpp"

using lbfi::fail;

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

// One Euler step on a TX x TY x TZ tile (TZ = 1 and no z halo in 2D).
template <int DIM, int TX, int TY, int TZ>
__global__ __launch_bounds__(256) void k_ch_step(ChGeo G, const float* __restrict__ c,
                                                 float* __restrict__ cn, float A, float kappa,
                                                 float dtM, int ntx, int nty, int ntiles) {
  constexpr int HZ = DIM == 3 ? 1 : 0;
  constexpr int LX = TX + 4, LY = TY + 4, LZ = TZ + 4 * HZ;   // c box, halo 2
  constexpr int MX = TX + 2, MY = TY + 2, MZ = TZ + 2 * HZ;   // mu box, halo 1
  __shared__ float cs[LX * LY * LZ];
  __shared__ float ms[MX * MY * MZ];
  const int t = lbf::xcd_tile(blockIdx.x, ntiles);
  const int x0 = (t % ntx) * TX, y0 = ((t / ntx) % nty) * TY, z0 = (t / (ntx * nty)) * TZ;
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  for (int i = threadIdx.x; i < LX * LY * LZ; i += 256) {
    const int lx = i % LX, ly = (i / LX) % LY, lz = i / (LX * LY);
    const int gx = wrap_or_clamp(x0 + lx - 2, nx, G.per[0]);
    const int gy = wrap_or_clamp(y0 + ly - 2, ny, G.per[1]);
    const int gz = DIM == 3 ? wrap_or_clamp(z0 + lz - 2, nz, G.per[2]) : 0;
    cs[i] = c[(gz * ny + gy) * nx + gx];   // < 2^31 nodes
  }
  __syncthreads();
  for (int i = threadIdx.x; i < MX * MY * MZ; i += 256) {
    const int mx = i % MX, my = (i / MX) % MY, mz = i / (MX * MY);
    const int j = ((mz + HZ) * LY + my + 1) * LX + mx + 1;
    const float cc = cs[j];
    ms[i] = A * (cc * cc * cc - cc) - kappa * lds_laplacian<DIM, LX, LX * LY>(cs, j);
  }
  __syncthreads();
  // beyond a mirror wall the potential is that of the first node (its
  // ghost); the source is always an in-domain node of the same box.  Only
  // tiles whose ring reaches past a wall have such cells.
  const bool at_wall = (!G.per[0] && (x0 == 0 || x0 + TX >= nx)) ||
                       (!G.per[1] && (y0 == 0 || y0 + TY >= ny)) ||
                       (DIM == 3 && !G.per[2] && (z0 == 0 || z0 + TZ >= nz));
  if (at_wall) {
    for (int i = threadIdx.x; i < MX * MY * MZ; i += 256) {
      const int mx = i % MX, my = (i / MX) % MY, mz = i / (MX * MY);
      const int gx = x0 + mx - 1, gy = y0 + my - 1, gz = z0 + mz - HZ;
      const int sx = G.per[0] ? gx : min(max(gx, 0), nx - 1);
      const int sy = G.per[1] ? gy : min(max(gy, 0), ny - 1);
      const int sz = (DIM == 3 && !G.per[2]) ? min(max(gz, 0), nz - 1) : gz;
      if (sx != gx || sy != gy || sz != gz)
        ms[i] = ms[((sz - z0 + HZ) * MY + sy - y0 + 1) * MX + sx - x0 + 1];
    }
    __syncthreads();
  }
  for (int o = threadIdx.x; o < TX * TY * TZ; o += 256) {
    const int ox = o % TX, oy = (o / TX) % TY, oz = o / (TX * TY);
    const int gx = x0 + ox, gy = y0 + oy, gz = z0 + oz;
    if (gx >= nx || gy >= ny || gz >= nz) continue;
    const int j = ((oz + 2 * HZ) * LY + oy + 2) * LX + ox + 2;
    const int m = ((oz + HZ) * MY + oy + 1) * MX + ox + 1;
    cn[(gz * ny + gy) * nx + gx] = cs[j] + dtM * lds_laplacian<DIM, MX, MX * MY>(ms, m);
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
  if (!p || !solid || !phi0) return fail(LBF_EINVAL, "NULL argument");
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
  const int N = (int)n;
  const size_t pb = plane_bytes(n);
  float* c[2] = {(float*)ws, (float*)(ws + pb)};
  const int nb = (N + 255) / 256;
  const ChGeo G{{p->nx, p->ny, p->nz},
                {p->periodic[0] ? 1 : 0, p->periodic[1] ? 1 : 0, p->periodic[2] ? 1 : 0}};
  const bool is3d = p->nz > 1;
  const int ntx = ceil_div(p->nx, is3d ? kTX3 : kTX2), nty = ceil_div(p->ny, is3d ? kTY3 : kTY2);
  const int ntz = is3d ? ceil_div(p->nz, kTZ3) : 1;
  const int ntiles = ntx * nty * ntz;
  const float A = (float)p->A, kap = (float)p->kappa, dtM = (float)(p->dt * p->mobility);
  auto run = [&]() -> int {
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
        hipLaunchKernelGGL((k_ch_step<3, kTX3, kTY3, kTZ3>), dim3(ntiles), dim3(256), 0, st, G,
                           c[cur], c[1 - cur], A, kap, dtM, ntx, nty, ntiles);
      else
        hipLaunchKernelGGL((k_ch_step<2, kTX2, kTY2, 1>), dim3(ntiles), dim3(256), 0, st, G,
                           c[cur], c[1 - cur], A, kap, dtM, ntx, nty, ntiles);
      HIP_TRY(hipGetLastError());
      cur = 1 - cur;
    }
    float* dst = phi0_on_device ? phi0 : c[1 - cur];
    hipLaunchKernelGGL(k_ch_final, dim3(nb), dim3(256), 0, st, c[cur], dst, N);
    HIP_TRY(hipGetLastError());
    if (!phi0_on_device)
      HIP_TRY(hipMemcpyAsync(phi0, dst, (size_t)N * 4, hipMemcpyDeviceToHost, st));
    if (!phi0_on_device || !solid_on_device || owns) HIP_TRY(hipStreamSynchronize(st));
    return LBF_OK;
  };
  const int rc = run();
  if (owns) {
    (void)hipStreamSynchronize(st);
    (void)hipFree(ws);
  }
  return rc;
}

}  // extern "C"
