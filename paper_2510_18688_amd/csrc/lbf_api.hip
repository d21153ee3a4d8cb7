// C ABI of liblbf (declarations and contracts in include/lbf.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "lbf.h"
#include "lbf_device.hpp"
#include "lbf_sim.hpp"
#include "lbf_step.hpp"

using namespace lbf;

namespace lbfi {

thread_local char g_err[512];

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
  return code;
}

static_assert(NDIST + NLAG == kStateSlots, "a state array holds the distributions and lags");

// Each parity's state is one array of row blocks (the 27 distribution planes,
// then the 9 lagged ones); the static planes use the same block structure, so
// a node has one index in all of them.  The read-out planes stay plane-major.
Layout make_layout(int nx, int ny, int pad, int rb) {
  Layout L{};
  const long long P = plane_stride(nx, ny, pad, rb);
  const int nblk = num_blocks(ny, rb);
  const long long gs = kStateSlots * P;
  const size_t PF = round_up((size_t)nx * ny, 64) * sizeof(float);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t o = off;
    off = round_up(off + bytes, kAlign);
    return o;
  };
  const size_t sb = (size_t)array_floats(nblk, gs, P, kStateSlots) * sizeof(float);
  for (int c = 0; c < 2; ++c) {
    L.dist[c] = take(sb);
    L.lag[c] = L.dist[c] + (size_t)NDIST * P * sizeof(float);
  }
  L.stat = take((size_t)array_floats(nblk, gs, P, NSTAT) * sizeof(float));
  L.fields = take(NFIELD * PF);
  L.wstride = (int)round_up((size_t)std::max(nx, ny), 64);
  L.wall = take(4 * (size_t)L.wstride * sizeof(float));
  const size_t redb = max_blocks(nx, ny) * NRED * sizeof(double);
  L.red[0] = take(redb);
  L.red[1] = take(redb);
  L.redfinal = take(2 * NRED * sizeof(double));
  // column-profile partials (4 per column and chunk of rows), then the
  // column and row profiles
  const size_t nchunk = ((size_t)ny + kProfileChunk - 1) / kProfileChunk;
  L.prof = take((nchunk * nx * 4 + LBF_NCOL * (size_t)nx + LBF_NROW * (size_t)ny) *
                sizeof(double));
  L.total = off;
  return L;
}

}  // namespace lbfi

using namespace lbfi;

namespace {

BufArgs make_args(lbf_sim* s) {
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
  return B;
}

int validate(const lbf_params* p) {
  if (!p) return fail(LBF_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1) return fail(LBF_EINVAL, "lattice size %d x %d", p->nx, p->ny);
  if (p->plane_pad < 0 || p->plane_pad > kMaxPlanePad || p->plane_pad % 64)
    return fail(LBF_EINVAL, "plane_pad %d (a multiple of 64 in [0, %d])", p->plane_pad,
                kMaxPlanePad);
  if (!valid_row_block(p->row_block))
    return fail(LBF_EINVAL, "row_block %d (0, 1, 2, 4, 8, 16 or 32)", p->row_block);
  if (!fits_offsets(p->nx, p->ny, p->plane_pad, p->row_block))
    return fail(LBF_EINVAL,
                "lattice of %d x %d nodes exceeds the 32-bit offset limit of its layout "
                "(row_block %d)", p->nx, p->ny, p->row_block);
  const double pos[] = {p->rho_l, p->rho_g, p->rho_s, p->mu_l, p->mu_g, p->mu_s, p->lam_l,
                        p->lam_g, p->lam_s, p->cp_l, p->cp_g, p->cp_s, p->eps, p->mobility,
                        p->rho_ref};
  for (double v : pos)
    if (!(v > 0.0) || !std::isfinite(v))
      return fail(LBF_EINVAL, "densities, viscosities, conductivities, heat capacities, eps, "
                              "mobility and rho_ref must be positive and finite");
  if (!(p->pcm_floor >= 0.0 && p->pcm_floor < 1.0))
    return fail(LBF_EINVAL, "pcm_floor must be in [0, 1) (got %g)", p->pcm_floor);
  if (!(p->latent >= 0.0) || !(p->sigma >= 0.0))
    return fail(LBF_EINVAL, "latent heat and surface tension must be non-negative");
  for (int w = 0; w < 4; ++w)
    if (p->thermal_bc[w] != LBF_ADIABATIC && p->thermal_bc[w] != LBF_DIRICHLET)
      return fail(LBF_EINVAL, "thermal_bc[%d] = %d", w, p->thermal_bc[w]);
  if (p->mrt != 0 && p->mrt != 1) return fail(LBF_EINVAL, "mrt = %d", p->mrt);
  if (p->check_every < 0) return fail(LBF_EINVAL, "check_every = %d", p->check_every);
  if (p->phi_src_mdot != 0 && p->phi_src_mdot != 1)
    return fail(LBF_EINVAL, "phi_src_mdot = %d", p->phi_src_mdot);
  for (int a = 0; a < 2; ++a)
    if (!std::isfinite(p->grav[a]) || !std::isfinite(p->u_solid[a]))
      return fail(LBF_EINVAL, "grav and u_solid must be finite");
  if (p->mrt && !(p->s_b >= 0.0 && p->s_b < 2.0 && p->s_q >= 0.0 && p->s_q < 2.0 &&
                  p->s_g >= 0.0 && p->s_g < 2.0))
    return fail(LBF_EINVAL, "MRT rates s_b = %g, s_q = %g, s_g = %g must be in [0, 2)", p->s_b,
                p->s_q, p->s_g);
  const double cpref = 2.0 * p->cp_s * p->cp_l / (p->cp_s + p->cp_l);
  const double kmin = std::min({p->rho_l, p->rho_g, p->rho_s}) *
                      std::min({p->cp_l, p->cp_g, p->cp_s});
  if (p->rho_ref * cpref > kmin * (1.0 + 1e-12))
    return fail(LBF_EINVAL,
                "rho_ref * C_p,ref = %g exceeds the smallest nodal heat capacity %g: the "
                "enthalpy scheme would be unstable",
                p->rho_ref * cpref, kmin);
  return LBF_OK;
}

void fill_phys(const lbf_params* p, Phys& ph) {
  ph.rho_l = (float)p->rho_l; ph.rho_g = (float)p->rho_g; ph.rho_s = (float)p->rho_s;
  ph.mu_l = (float)p->mu_l; ph.mu_g = (float)p->mu_g; ph.mu_s = (float)p->mu_s;
  ph.lam_l = (float)p->lam_l; ph.lam_g = (float)p->lam_g; ph.lam_s = (float)p->lam_s;
  ph.cp_l = (float)p->cp_l; ph.cp_g = (float)p->cp_g; ph.cp_s = (float)p->cp_s;
  ph.latent = (float)p->latent;
  ph.T_m = (float)p->T_m;
  ph.cos_psi = (float)p->cos_psi;
  ph.T_sub = (float)p->T_substrate;
  ph.a3 = (float)(3.0 * p->sigma / p->eps);
  ph.kap = (float)(3.0 * p->eps * p->sigma / 8.0);
  ph.tau_g = (float)(3.0 * p->mobility + 0.5);
  ph.inv_tau_g = (float)(1.0 / (3.0 * p->mobility + 0.5));
  ph.pg = (float)(1.0 - 0.5 / (3.0 * p->mobility + 0.5));
  const double Eref = p->rho_ref * 2.0 * p->cp_s * p->cp_l / (p->cp_s + p->cp_l);
  ph.Eref = (float)Eref;
  ph.three_over_Eref = (float)(3.0 / Eref);
  ph.mdot_coef = (float)(1.0 - p->rho_s / p->rho_l);
  ph.pcm_floor = (float)p->pcm_floor;
  ph.inv_pcm_span = (float)(1.0 / (1.0 - p->pcm_floor));
  ph.latch = p->latch_fs ? 1 : 0;
  ph.src_tau_a = p->h_src_tau_a ? 1 : 0;
  ph.subfix = p->substrate_fixed ? 1 : 0;
  ph.mrt = p->mrt ? 1 : 0;
  ph.phi_src_flow = p->phi_src_mdot ? 0 : 1;
  ph.s_b = p->mrt ? (float)p->s_b : 0.0f;
  ph.s_q = p->mrt ? (float)p->s_q : 0.0f;
  ph.s_g = p->mrt ? (float)p->s_g : 0.0f;
  for (int a = 0; a < 2; ++a) {
    ph.grav[a] = (float)p->grav[a];
    ph.vsol[a] = (float)p->u_solid[a];
  }
  ph.grav[2] = ph.vsol[2] = 0.0f;
}

// ---------------------------------------------------------------- kernels
__global__ void k_lap_static(Geo G, float* stat) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const float* phi0 = stat + ST_PHI0 * G.P;
  const float c = phi0[nidx(G, x, y)];
  float lap = 0.0f;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int xx = map_axis(x + cx(i), G.nx, G.px), yy = map_axis(y + cy(i), G.ny, G.py);
    lap += wgt(i) * (phi0[nidx(G, xx, yy)] - c);
  }
  stat[ST_LAP0 * G.P + nidx(G, x, y)] = 6.0f * lap;
}

// Held temperature per node from a byte mask and a temperature field (both
// staged in device memory, plane-major): T where the mask is set, NaN
// elsewhere.
__global__ void k_set_thold(Geo G, const uint8_t* mask, const float* T, float* stat) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const int k = y * G.nx + x;
  stat[ST_THOLD * G.P + nidx(G, x, y)] = mask[k] ? T[k] : __builtin_nanf("");
}

// Equilibrium populations of the initial state, in post-stream form, into
// `tmp` (NDIST planes of a state array); `in` holds phi (plane 0) and T
// (plane 1), plane-major, PF apart.
__global__ void k_init_eq(Geo G, Phys ph, const float* stat, const float* in, float* tmp) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const long long P = G.P;
  const int kf = y * G.nx + x;
  const int k = nidx(G, x, y);
  const float* phi = in;
  const float* T0 = in + G.PF;
  const float pc = phi[kf];
  float lap = 0.0f;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int xx = map_axis(x + cx(i), G.nx, G.px), yy = map_axis(y + cy(i), G.ny, G.py);
    lap += wgt(i) * (phi[yy * G.nx + xx] - pc);
  }
  lap *= 6.0f;
  const float phi0 = stat[ST_PHI0 * P + k];
  const float mu = chem_pot(ph, pc, lap, phi0, stat[ST_CTH * P + k], stat[ST_LAP0 * P + k], 0.0f,
                            0.0f);
  const float C = clampf(0.5f * (1.0f - phi0 + pc), 0.0f, 1.0f);
  const float Cp = clampf((C - ph.pcm_floor) * ph.inv_pcm_span, 0.0f, 1.0f);
  const float chi = clampf(Cp, 0.0f, 1.0f - phi0);
  const float Kliq = zeta(phi0, C, ph.rho_s, ph.rho_l, ph.rho_g) *
                     zeta(phi0, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float Tk = T0[kf];
  const float rhoH = Kliq * (Tk - ph.T_m) + Kliq * ph.T_m + chi * ph.rho_l * ph.latent;
  const float ET = ph.Eref * Tk;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    tmp[i * P + k] = 0.0f;
    tmp[(9 + i) * P + k] = (i == 0 ? pc : 0.0f) + (wgt(i) - (i == 0 ? 1.0f : 0.0f)) * mu;
    tmp[(18 + i) * P + k] = (i == 0) ? rhoH - ET + wgt(0) * ET : wgt(i) * ET;
  }
}

// Inverse of the pull: post-collision populations whose pull gives `tmp`.
// The rest populations g_0, h_0 (which do not move) become the high parts
// (lagged planes) of their float-float storage, with zero low parts.
__global__ void k_unstream(Geo G, Phys ph, const float* tmp, float* dst, float* stat, float* lag,
                           const float* wallT, int wstride) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= G.nx || y >= G.ny) return;
  const long long P = G.P;
  const int k = nidx(G, x, y);
  dst[k] = tmp[k];
  // rest populations as float-float: 16-bit high parts (one plane), the
  // exact remainders in the distribution planes
  const float g0 = tmp[9 * P + k], h0 = tmp[18 * P + k];
  const float gh = hi16(g0), hh = hi16(h0);
  lag[LAG_GHI * P + k] = __builtin_bit_cast(float, pack_hi(gh, hh));
  lag[LAG_HHI * P + k] = 0.0f;
  dst[9 * P + k] = g0 - gh;
  dst[18 * P + k] = h0 - hh;
  if (ph.phi_src_flow) {
    // the step keeps the previous step's phi in place of (phi u)_x: recover it
    // from the caller's (phi u) and u (any value serves where u = 0)
    const float jx = lag[LAG_JX * P + k], jy = lag[LAG_JY * P + k];
    const float ux = lag[LAG_UX * P + k], uy = lag[LAG_UY * P + k];
    float ph_prev = 0.0f;
    if (fabsf(ux) >= fabsf(uy)) {
      if (ux != 0.0f) ph_prev = jx / ux;
    } else {
      ph_prev = jy / uy;
    }
    lag[LAG_JX * P + k] = ph_prev;
    lag[LAG_JY * P + k] = 0.0f;
  }
#pragma unroll
  for (int j = 1; j < 9; ++j) {
    // destination of population j leaving (x, y)
    int dx = x + cx(j), dy = y + cy(j), wall = -1;
    if (dy < 0 || dy >= G.ny) {
      if (G.py) dy = dy < 0 ? dy + G.ny : dy - G.ny;
      else wall = dy < 0 ? 0 : 1;
    }
    if (wall < 0 && (dx < 0 || dx >= G.nx)) {
      if (G.px) dx = dx < 0 ? dx + G.nx : dx - G.nx;
      else wall = dx < 0 ? 2 : 3;
    }
    if (wall < 0) {
      const int d = nidx(G, dx, dy);
      dst[j * P + k] = tmp[j * P + d];
      dst[(9 + j) * P + k] = tmp[(9 + j) * P + d];
      dst[(18 + j) * P + k] = tmp[(18 + j) * P + d];
    } else {
      const int i = opp(j);   // the population that node (x, y) pulls back
      dst[j * P + k] = tmp[i * P + k];
      dst[(9 + j) * P + k] = tmp[(9 + i) * P + k];
      if ((G.tmask >> wall) & 1) {
        const float Tw = wallT[wall * wstride + (wall < 2 ? x : y)];
        dst[(18 + j) * P + k] = 2.0f * wgt(i) * ph.Eref * Tw - tmp[(18 + i) * P + k];
      } else {
        dst[(18 + j) * P + k] = tmp[(18 + i) * P + k];
      }
    }
  }
}

// Fixed-order sum of per-block partials (one block of 256 threads).
__global__ void k_reduce_blocks(const double* part, int nblocks, double* out) {
  __shared__ double s[256];
  for (int j = 0; j < NRED; ++j) {
    double v = (j == 4) ? 0.0 : 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      const double t = part[(size_t)b * NRED + j];
      v = (j == 4) ? fmax(v, t) : v + t;
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w)
        s[threadIdx.x] = (j == 4) ? fmax(s[threadIdx.x], s[threadIdx.x + w])
                                  : s[threadIdx.x] + s[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = s[0];
    __syncthreads();
  }
}

// Measurement aid: the step kernel's HBM access pattern without its
// arithmetic.  Same strips (xcd_tile order, WX columns, CY rows, even tile
// rows marching up and odd ones down) and the same buffer loads and
// non-temporal stores; every plane the step reads is copied to the plane it
// writes, the static planes are only read (their sum guards a store that
// never happens, so the loads stay).
template <int WX>
__global__ __launch_bounds__(WX) void k_copy_probe(Geo G, Phys ph, BufArgs A, int CY, int nbx,
                                                   int ntiles) {
  const Bufs B = make_bufs(A, G);
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int bx = t % nbx, by = t / nbx;
  const int x = bx * WX + (int)threadIdx.x;
  if (x >= G.nx) return;
  const int y0 = by * CY, y1 = min(y0 + CY, G.ny);
  const bool up = !(by & 1);
  const int P = G.P;
  const bool flow = ph.phi_src_flow != 0;
  float acc = 0.0f;
  for (int it = 0; it < y1 - y0; ++it) {
    const int y = up ? y0 + it : y1 - 1 - it;
    const int k = nidx(G, x, y);
    float v[27 + NLAG];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      v[i] = ldp(B.fin, i, P, k);
      v[9 + i] = ldp(B.gin, i, P, k);
      v[18 + i] = ldp(B.hin, i, P, k);
    }
#pragma unroll
    for (int j = 0; j < NLAG; ++j) {
      const bool used = j != LAG_HHI && (flow ? j != LAG_JY : j < LAG_UX);
      v[27 + j] = used ? ldp(B.lin, j, P, k) : 0.0f;
    }
    acc += ldp(B.stat, ST_PHI0, P, k) + ldp(B.stat, ST_CTH, P, k);
    if (ph.subfix == 2) acc += ldp(B.stat, ST_THOLD, P, k);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      stp(B.fout, i, P, k, v[i]);
      stp(B.gout, i, P, k, v[9 + i]);
      stp(B.hout, i, P, k, v[18 + i]);
    }
#pragma unroll
    for (int j = 0; j < NLAG; ++j) {
      const bool used = j != LAG_HHI && (flow ? j != LAG_JY : j < LAG_UX);
      if (used) stp(B.lout, j, P, k, v[27 + j]);
    }
  }
  if (acc == -1.0e30f) stp(B.lout, LAG_FS, P, nidx(G, x, y0), acc);
}

// ------------------------------------------------------------ launches
int grid_blocks(const lbf_sim* s, dim3& grid) {
  grid = dim3((s->G.nx + s->tile_x - 1) / s->tile_x, (s->G.ny + s->tile_y - 1) / s->tile_y, 1);
  return (int)(grid.x * grid.y);
}

template <int WX, bool MRT>
void launch_collide(const lbf_sim* s, int mode, bool red, BufArgs B, hipStream_t st, dim3 grid,
                    int nbx, int nt) {
  const dim3 block(WX);
  if (mode == MODE_STEP && !red)
    hipLaunchKernelGGL((step_kernel<WX, MODE_STEP, false, MRT>), grid, block, 0, st, s->G, s->ph,
                       B, s->tile_y, nbx, nt);
  else if (mode == MODE_STEP && red)
    hipLaunchKernelGGL((step_kernel<WX, MODE_STEP, true, MRT>), grid, block, 0, st, s->G, s->ph,
                       B, s->tile_y, nbx, nt);
  else if (mode == MODE_FIELDS && !red)
    hipLaunchKernelGGL((step_kernel<WX, MODE_FIELDS, false, MRT>), grid, block, 0, st, s->G,
                       s->ph, B, s->tile_y, nbx, nt);
  else
    hipLaunchKernelGGL((step_kernel<WX, MODE_FIELDS, true, MRT>), grid, block, 0, st, s->G,
                       s->ph, B, s->tile_y, nbx, nt);
}

template <int WX>
int launch_wx(lbf_sim* s, int mode, bool red, BufArgs B, hipStream_t st) {
  dim3 g2;
  const int nt = grid_blocks(s, g2);
  const int nbx = (int)g2.x;
  const dim3 grid(nt);
  if (mode == MODE_STEP_MOM)   // the adjoint's recomputation (BGK only)
    hipLaunchKernelGGL((step_kernel<WX, MODE_STEP_MOM, false>), grid, dim3(WX), 0, st, s->G,
                       s->ph, B, s->tile_y, nbx, nt);
  else if (s->ph.mrt)
    launch_collide<WX, true>(s, mode, red, B, st, grid, nbx, nt);
  else
    launch_collide<WX, false>(s, mode, red, B, st, grid, nbx, nt);
  HIP_TRY(hipGetLastError());
  return LBF_OK;
}

int launch_step(lbf_sim* s, int mode, bool red, double* red_buf) {
  BufArgs B = make_args(s);
  B.red = red_buf;
  return launch_step_args(s, mode, red, B, s->stream);
}

}  // namespace

int lbfi::launch_step_args(lbf_sim* s, int mode, bool red, BufArgs B, hipStream_t st) {
  switch (s->tile_x) {
    case 64: return launch_wx<64>(s, mode, red, B, st);
    case 128: return launch_wx<128>(s, mode, red, B, st);
    case 256: return launch_wx<256>(s, mode, red, B, st);
    case 512: return launch_wx<512>(s, mode, red, B, st);
    default: return fail(LBF_EINVAL, "tile_x %d", s->tile_x);
  }
}

namespace {

dim3 node_grid(const lbf_sim* s) { return dim3((s->G.nx + 255) / 256, s->G.ny, 1); }

int copy_in(lbf_sim* s, void* dst, const void* src, size_t bytes, int on_device) {
  HIP_TRY(hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         s->stream));
  if (!on_device) HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

// Copy one plane between a plain array of nx * ny values (`flat`) and the
// plane that starts at `plane` in a state or static array (row blocks, or
// plane-major), on the simulation's stream.  `to_plane` gives the direction.
int plane_copy(lbf_sim* s, float* plane, float* flat, bool to_plane, hipMemcpyKind kind) {
  const Geo& G = s->G;
  const size_t n = (size_t)G.nx * G.ny;
  if (G.nblk == 1) {
    HIP_TRY(hipMemcpyAsync(to_plane ? plane : flat, to_plane ? flat : plane, n * sizeof(float),
                           kind, s->stream));
    return LBF_OK;
  }
  const size_t rb = (size_t)G.rmask + 1, full = (size_t)G.ny / rb, rem = (size_t)G.ny - full * rb;
  const size_t w = rb * G.nx * sizeof(float), pitch = (size_t)G.GS * sizeof(float);
  if (full)
    HIP_TRY(hipMemcpy2DAsync(to_plane ? plane : flat, to_plane ? pitch : w,
                             to_plane ? flat : plane, to_plane ? w : pitch, w, full, kind,
                             s->stream));
  if (rem) {
    float* pb = plane + full * G.GS;
    float* fb = flat + full * rb * G.nx;
    HIP_TRY(hipMemcpyAsync(to_plane ? pb : fb, to_plane ? fb : pb, rem * G.nx * sizeof(float),
                           kind, s->stream));
  }
  return LBF_OK;
}

// Zero the lagged planes of state buffer c (every block).
int zero_lags(lbf_sim* s, int c) {
  HIP_TRY(hipMemset2DAsync(fptr(s, s->L.lag[c]), (size_t)s->G.GS * sizeof(float), 0,
                           NLAG * (size_t)s->G.P * sizeof(float), (size_t)s->G.nblk, s->stream));
  return LBF_OK;
}

// Plane copy from caller memory (host or device) into a state or static
// plane; a host source is released when this returns.
int plane_in(lbf_sim* s, float* plane, const float* src, int on_device) {
  int rc = plane_copy(s, plane, const_cast<float*>(src), true,
                      on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice);
  if (rc) return rc;
  if (!on_device) HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

// Stability check of lbf_step: fixed-order sum of the partials a step wrote
// for the state it read (time level `level`), then non-finite count and
// max |u| on the host.
int check_stable(lbf_sim* s, const double* part, long long level) {
  dim3 grid;
  const int nb = grid_blocks(s, grid);
  double* fin = dptr(s, s->L.redfinal) + NRED;
  hipLaunchKernelGGL(k_reduce_blocks, dim3(1), dim3(256), 0, s->stream, part, nb, fin);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(s->host_red + NRED, fin, NRED * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const double bad = s->host_red[NRED + LBF_RED_NONFINITE];
  const double umax = s->host_red[NRED + LBF_RED_UMAX];
  if (bad > 0 || !(umax <= 0.3))
    return fail(LBF_EUNSTABLE, "unstable at time level %lld: %g non-finite nodes, max |u| = %g",
                level, bad, umax);
  return LBF_OK;
}

}  // namespace

// ================================================================ C ABI
extern "C" {

const char* lbf_last_error(void) { return g_err; }

size_t lbf_workspace_bytes(int32_t nx, int32_t ny, int32_t plane_pad, int32_t row_block) {
  if (nx < 1 || ny < 1 || plane_pad < 0 || plane_pad > kMaxPlanePad || plane_pad % 64) return 0;
  if (!valid_row_block(row_block) || !fits_offsets(nx, ny, plane_pad, row_block)) return 0;
  return make_layout(nx, ny, plane_pad, row_block).total;
}

int lbf_create(const lbf_params* params, void* stream, void* workspace, size_t workspace_bytes,
               lbf_sim** out) {
  if (!out) return fail(LBF_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(params);
  if (rc) return rc;
  lbf_sim* s = new (std::nothrow) lbf_sim();
  if (!s) return fail(LBF_ENOMEM, "host allocation failed");
  s->prm = *params;
  s->G.nx = params->nx;
  s->G.ny = params->ny;
  s->G.px = params->periodic_x ? 1 : 0;
  s->G.py = params->periodic_y ? 1 : 0;
  s->G.tmask = 0;
  for (int w = 0; w < 4; ++w) {
    s->G.tbc[w] = params->thermal_bc[w];
    if (params->thermal_bc[w] == LBF_DIRICHLET) s->G.tmask |= 1 << w;
  }
  const int rb = params->row_block;
  s->G.P = (int)plane_stride(params->nx, params->ny, params->plane_pad, rb);
  s->G.GS = kStateSlots * s->G.P;
  s->G.nblk = num_blocks(params->ny, rb);
  s->G.rbs = 31;
  if (rb)
    for (s->G.rbs = 0; (1 << s->G.rbs) < rb; ++s->G.rbs) {
    }
  s->G.rmask = rb ? rb - 1 : 0x7fffffff;
  s->G.PF = (int)round_up((size_t)params->nx * params->ny, 64);
  fill_phys(params, s->ph);
  s->L = make_layout(params->nx, params->ny, params->plane_pad, rb);
  s->stream = (hipStream_t)stream;
  const size_t need = s->L.total;
  if (workspace) {
    if (workspace_bytes < need) {
      delete s;
      return fail(LBF_ENOMEM, "workspace of %zu bytes, %zu needed", workspace_bytes, need);
    }
    if ((uintptr_t)workspace % kAlign) {
      delete s;
      return fail(LBF_EINVAL, "workspace not 256-byte aligned");
    }
    s->ws = (char*)workspace;
    s->owns_ws = false;
  } else {
    if (hipMalloc((void**)&s->ws, need) != hipSuccess) {
      delete s;
      return fail(LBF_ENOMEM, "hipMalloc of %zu bytes failed", need);
    }
    s->owns_ws = true;
  }
  s->tile_x = params->nx >= 128 ? 128 : 64;
  s->tile_y = 32;
  if (hipHostMalloc((void**)&s->host_red, 2 * NRED * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
    lbf_destroy(s);
    return fail(LBF_EHIP, "host buffer / event creation failed");
  }
  // wall profiles start at zero
  if (hipMemsetAsync(s->ws + s->L.wall, 0, 4 * (size_t)s->L.wstride * sizeof(float), s->stream) !=
      hipSuccess) {
    lbf_destroy(s);
    return fail(LBF_EHIP, "hipMemsetAsync failed");
  }
  *out = s;
  return LBF_OK;
}

void lbf_destroy(lbf_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  if (s->owns_ws && s->ws) (void)hipFree(s->ws);
  if (s->host_red) (void)hipHostFree(s->host_red);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  delete s;
}

int lbf_set_geometry(lbf_sim* s, const float* phi0, const float* cos_theta, int32_t on_device) {
  if (!s || !phi0 || !cos_theta) return fail(LBF_EINVAL, "NULL argument");
  float* stat = fptr(s, s->L.stat);
  int rc = plane_in(s, stat + ST_PHI0 * (size_t)s->G.P, phi0, on_device);
  if (rc) return rc;
  rc = plane_in(s, stat + ST_CTH * (size_t)s->G.P, cos_theta, on_device);
  if (rc) return rc;
  hipLaunchKernelGGL(k_lap_static, node_grid(s), dim3(256), 0, s->stream, s->G, stat);
  HIP_TRY(hipGetLastError());
  s->have_geo = true;
  s->have_init = false;
  return LBF_OK;
}

int lbf_set_isothermal(lbf_sim* s, const uint8_t* mask, const float* T_hold, int32_t on_device) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  if (!mask) {
    s->ph.subfix = s->prm.substrate_fixed ? 1 : 0;
    return LBF_OK;
  }
  if (!T_hold) return fail(LBF_EINVAL, "T_hold is NULL");
  const size_t n = (size_t)s->G.nx * s->G.ny;
  // stage both arrays in the read-out planes (free between calls)
  float* stage = fptr(s, s->L.fields);
  uint8_t* mstage = reinterpret_cast<uint8_t*>(stage + s->G.PF);
  int rc = copy_in(s, stage, T_hold, n * sizeof(float), on_device);
  if (rc) return rc;
  rc = copy_in(s, mstage, mask, n, on_device);
  if (rc) return rc;
  hipLaunchKernelGGL(k_set_thold, node_grid(s), dim3(256), 0, s->stream, s->G,
                     (const uint8_t*)mstage, (const float*)stage, fptr(s, s->L.stat));
  HIP_TRY(hipGetLastError());
  s->ph.subfix = 2;
  return LBF_OK;
}

int lbf_set_wall_temperature(lbf_sim* s, int32_t wall, const float* Tw, int32_t n,
                             int32_t on_device) {
  if (!s || !Tw) return fail(LBF_EINVAL, "NULL argument");
  if (wall < 0 || wall > 3) return fail(LBF_EINVAL, "wall %d", wall);
  const int need = wall < 2 ? s->G.nx : s->G.ny;
  if (n != need) return fail(LBF_EINVAL, "wall %d needs %d values, got %d", wall, need, n);
  float* w = fptr(s, s->L.wall) + (size_t)wall * s->L.wstride;
  return copy_in(s, w, Tw, (size_t)n * sizeof(float), on_device);
}

int lbf_init_fields(lbf_sim* s, const float* phi, const float* T, int32_t on_device) {
  if (!s || !phi || !T) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_geo) return fail(LBF_ESTATE, "lbf_set_geometry must precede lbf_init_fields");
  const size_t n = (size_t)s->G.nx * s->G.ny;
  float* stage = fptr(s, s->L.fields);
  int rc = copy_in(s, stage, phi, n * sizeof(float), on_device);
  if (rc) return rc;
  rc = copy_in(s, stage + s->G.PF, T, n * sizeof(float), on_device);
  if (rc) return rc;
  s->cur = 0;
  float* tmp = fptr(s, s->L.dist[1]);
  hipLaunchKernelGGL(k_init_eq, node_grid(s), dim3(256), 0, s->stream, s->G, s->ph,
                     (const float*)fptr(s, s->L.stat), (const float*)stage, tmp);
  HIP_TRY(hipGetLastError());
  // the lagged planes of every block, in both buffers: planes a step does
  // not write (the high part of h_0, which shares g_0's plane, and (phi u)_y
  // under the flow-divergence source) then stay zero, and a saved state does
  // not depend on what the workspace held
  for (int c = 0; c < 2; ++c) {
    int rc = zero_lags(s, c);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_unstream, node_grid(s), dim3(256), 0, s->stream, s->G, s->ph,
                     (const float*)tmp, fptr(s, s->L.dist[0]), fptr(s, s->L.stat),
                     fptr(s, s->L.lag[0]), (const float*)fptr(s, s->L.wall), s->L.wstride);
  HIP_TRY(hipGetLastError());
  s->step = 0;
  s->have_budget = false;
  s->have_init = true;
  s->from_fields = true;
  return LBF_OK;
}

int lbf_set_poststream_state(lbf_sim* s, const float* dist, const float* lag, int64_t step,
                              int32_t on_device) {
  if (!s || !dist || !lag) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_geo) return fail(LBF_ESTATE, "lbf_set_geometry must precede the state");
  const size_t n = (size_t)s->G.nx * s->G.ny;
  int rc0 = zero_lags(s, 1 - s->cur);
  if (rc0) return rc0;
  float* tmp = fptr(s, s->L.dist[1 - s->cur]);
  for (int pl = 0; pl < NDIST; ++pl) {
    int rc = plane_in(s, tmp + (size_t)pl * s->G.P, dist + pl * n, on_device);
    if (rc) return rc;
  }
  float* lg = fptr(s, s->L.lag[s->cur]);
  // planes f_s, Q, (phi u), p, u of the caller's order; the high parts of
  // the rest populations come from dist
  const int dst_plane[7] = {LAG_FS, LAG_Q, LAG_JX, LAG_JY, LAG_P, LAG_UX, LAG_UY};
  for (int pl = 0; pl < 7; ++pl) {
    int rc = plane_in(s, lg + (size_t)dst_plane[pl] * s->G.P, lag + pl * n, on_device);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k_unstream, node_grid(s), dim3(256), 0, s->stream, s->G, s->ph,
                     (const float*)tmp, fptr(s, s->L.dist[s->cur]), fptr(s, s->L.stat),
                     fptr(s, s->L.lag[s->cur]), (const float*)fptr(s, s->L.wall), s->L.wstride);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->step = step;
  s->have_budget = false;
  s->have_init = true;
  s->from_fields = false;
  return LBF_OK;
}

int lbf_step(lbf_sim* s, int32_t nsteps) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  if (nsteps < 0) return fail(LBF_EINVAL, "nsteps %d", nsteps);
  if (!s->have_init) return fail(LBF_ESTATE, "lbf_init_fields must precede lbf_step");
  if (nsteps == 0) return LBF_OK;
  if (s->timing) HIP_TRY(hipEventRecord(s->ev0, s->stream));
  const int k = s->prm.check_every;
  for (int it = 0; it < nsteps; ++it) {
    const bool last = it == nsteps - 1;
    // a checking step reduces the state it reads (time level s->step)
    const bool chk = k > 0 && s->step % k == 0;
    double* rb = last ? dptr(s, s->L.red[0]) : (chk ? dptr(s, s->L.red[1]) : nullptr);
    int rc = launch_step(s, MODE_STEP, last || chk, rb);
    if (rc) return rc;
    s->cur = 1 - s->cur;
    s->step++;
    if (chk) {
      rc = check_stable(s, rb, s->step - 1);
      if (rc) {
        dim3 grid;
        s->budget_blocks = grid_blocks(s, grid);
        s->have_budget = last;
        return rc;
      }
    }
  }
  if (s->timing) {
    HIP_TRY(hipEventRecord(s->ev1, s->stream));
    HIP_TRY(hipEventSynchronize(s->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->last_ms = ms / nsteps;
  }
  dim3 grid;
  s->budget_blocks = grid_blocks(s, grid);
  s->have_budget = true;
  return LBF_OK;
}

int lbf_read_fields(lbf_sim* s, float* dst, int32_t dst_on_device) {
  if (!s || !dst) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  int rc = launch_step(s, MODE_FIELDS, false, nullptr);
  if (rc) return rc;
  const size_t n = (size_t)s->G.nx * s->G.ny;
  const float* F = fptr(s, s->L.fields);
  for (int f = 0; f < LBF_NFIELDS; ++f)
    HIP_TRY(hipMemcpyAsync(dst + f * n, F + f * (size_t)s->G.PF, n * sizeof(float),
                           dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

int lbf_read_field(lbf_sim* s, int32_t field_id, float* dst, int32_t dst_on_device) {
  if (!s || !dst) return fail(LBF_EINVAL, "NULL argument");
  if (field_id < 0 || field_id >= LBF_NFIELDS) return fail(LBF_EINVAL, "field %d", field_id);
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  int rc = launch_step(s, MODE_FIELDS, false, nullptr);
  if (rc) return rc;
  const size_t n = (size_t)s->G.nx * s->G.ny;
  HIP_TRY(hipMemcpyAsync(dst, fptr(s, s->L.fields) + field_id * (size_t)s->G.PF, n * sizeof(float),
                         dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

int lbf_reduce(lbf_sim* s, double* out) {
  if (!s || !out) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  int rc = launch_step(s, MODE_FIELDS, true, dptr(s, s->L.red[1]));
  if (rc) return rc;
  dim3 grid;
  const int nb = grid_blocks(s, grid);
  double* fin = dptr(s, s->L.redfinal);
  hipLaunchKernelGGL(k_reduce_blocks, dim3(1), dim3(256), 0, s->stream,
                     (const double*)dptr(s, s->L.red[1]), nb, fin + NRED);
  HIP_TRY(hipGetLastError());
  if (s->have_budget) {
    hipLaunchKernelGGL(k_reduce_blocks, dim3(1), dim3(256), 0, s->stream,
                       (const double*)dptr(s, s->L.red[0]), s->budget_blocks, fin);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipMemcpyAsync(s->host_red, fin, 2 * NRED * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const double* cur = s->host_red + NRED;
  const double* bud = s->host_red;
  for (int j = 0; j < LBF_NRED; ++j) out[j] = cur[j];
  out[LBF_RED_SRC_PHI] = s->have_budget ? bud[6] : 0.0;
  out[LBF_RED_SRC_HEAT] = s->have_budget ? bud[7] : 0.0;
  out[LBF_RED_RESET] = s->have_budget ? bud[9] : 0.0;
  out[LBF_RED_WALL_FLUX] = s->step > 0 ? cur[8] : 0.0;
  out[LBF_RED_STEP] = (double)s->step;
  if (out[LBF_RED_NONFINITE] > 0 || !(out[LBF_RED_UMAX] <= 0.3))
    return fail(LBF_EUNSTABLE, "unstable: %g non-finite nodes, max |u| = %g",
                out[LBF_RED_NONFINITE], out[LBF_RED_UMAX]);
  return LBF_OK;
}

int lbf_set_tile(lbf_sim* s, int32_t tile_x, int32_t tile_y) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  if (tile_x != 64 && tile_x != 128 && tile_x != 256 && tile_x != 512)
    return fail(LBF_EINVAL, "tile_x must be 64, 128, 256 or 512 (got %d)", tile_x);
  if (tile_y < 1 || tile_y > CY_MAX)
    return fail(LBF_EINVAL, "tile_y must be in [1, %d] (got %d)", CY_MAX, tile_y);
  s->tile_x = tile_x;
  s->tile_y = tile_y;
  return LBF_OK;
}

int lbf_get_tile(const lbf_sim* s, int32_t* tile_x, int32_t* tile_y) {
  if (!s || !tile_x || !tile_y) return fail(LBF_EINVAL, "NULL argument");
  *tile_x = s->tile_x;
  *tile_y = s->tile_y;
  return LBF_OK;
}

// The saved state holds each plane's nx * ny values back to back (not the
// workspace's padded stride), so it loads into a simulation of the same
// lattice whatever its plane_pad.
constexpr long long kStateMagic = 0x6c626674LL;

size_t lbf_state_bytes(const lbf_sim* s) {
  if (!s) return 0;
  return (size_t)(NDIST + NLAG) * s->G.nx * s->G.ny * sizeof(float) + 64;
}

int lbf_save_state(lbf_sim* s, void* dst, size_t cap) {
  if (!s || !dst) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  const size_t need = lbf_state_bytes(s);
  if (cap < need) return fail(LBF_ENOMEM, "state needs %zu bytes", need);
  char* d = (char*)dst;
  const size_t n = (size_t)s->G.nx * s->G.ny, nb = n * sizeof(float);
  // the distributions, then the lagged planes: the state array's planes in order
  float* st = fptr(s, s->L.dist[s->cur]);
  for (int pl = 0; pl < kStateSlots; ++pl) {
    int rc = plane_copy(s, st + (size_t)pl * s->G.P, (float*)d + pl * n, false,
                        hipMemcpyDeviceToDevice);
    if (rc) return rc;
  }
  const size_t db = NDIST * nb, lb = NLAG * nb;
  long long hdr[8] = {kStateMagic, s->step, s->G.nx, s->G.ny, 0, 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(d + db + lb, hdr, sizeof hdr, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

int lbf_load_state(lbf_sim* s, const void* src, size_t bytes) {
  if (!s || !src) return fail(LBF_EINVAL, "NULL argument");
  const size_t need = lbf_state_bytes(s);
  if (bytes < need) return fail(LBF_EINVAL, "state of %zu bytes, %zu needed", bytes, need);
  const char* d = (const char*)src;
  const size_t n = (size_t)s->G.nx * s->G.ny, nb = n * sizeof(float);
  const size_t db = NDIST * nb, lb = NLAG * nb;
  long long hdr[8];
  HIP_TRY(hipMemcpyAsync(hdr, d + db + lb, sizeof hdr, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (hdr[0] != kStateMagic || hdr[2] != s->G.nx || hdr[3] != s->G.ny)
    return fail(LBF_EINVAL, "state buffer does not match this lattice");
  if (!s->have_geo) return fail(LBF_ESTATE, "lbf_set_geometry must precede lbf_load_state");
  float* st = fptr(s, s->L.dist[s->cur]);
  for (int pl = 0; pl < kStateSlots; ++pl) {
    int rc = plane_copy(s, st + (size_t)pl * s->G.P, (float*)d + pl * n, true,
                        hipMemcpyDeviceToDevice);
    if (rc) return rc;
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->step = hdr[1];
  s->have_init = true;
  s->have_budget = false;
  s->from_fields = false;
  return LBF_OK;
}

int lbf_set_timing(lbf_sim* s, int32_t on) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  s->timing = on != 0;
  return LBF_OK;
}

double lbf_last_step_kernel_ms(const lbf_sim* s) { return s ? s->last_ms : 0.0; }

int lbf_copy_probe(lbf_sim* s, int32_t launches, double* ms_per_launch,
                   double* bytes_per_launch) {
  if (!s || !ms_per_launch || !bytes_per_launch) return fail(LBF_EINVAL, "NULL argument");
  if (launches < 1) return fail(LBF_EINVAL, "launches %d", launches);
  if (!s->have_init) return fail(LBF_ESTATE, "the state must be set before lbf_copy_probe");
  dim3 g2;
  const int nt = grid_blocks(s, g2);
  const int nbx = (int)g2.x;
  BufArgs B = make_args(s);
  HIP_TRY(hipEventRecord(s->ev0, s->stream));
  for (int i = 0; i < launches; ++i) {
    switch (s->tile_x) {
      case 64:
        hipLaunchKernelGGL(k_copy_probe<64>, dim3(nt), dim3(64), 0, s->stream, s->G, s->ph, B,
                           s->tile_y, nbx, nt);
        break;
      case 128:
        hipLaunchKernelGGL(k_copy_probe<128>, dim3(nt), dim3(128), 0, s->stream, s->G, s->ph, B,
                           s->tile_y, nbx, nt);
        break;
      case 512:
        hipLaunchKernelGGL(k_copy_probe<512>, dim3(nt), dim3(512), 0, s->stream, s->G, s->ph, B,
                           s->tile_y, nbx, nt);
        break;
      default:
        hipLaunchKernelGGL(k_copy_probe<256>, dim3(nt), dim3(256), 0, s->stream, s->G, s->ph, B,
                           s->tile_y, nbx, nt);
        break;
    }
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipEventRecord(s->ev1, s->stream));
  HIP_TRY(hipEventSynchronize(s->ev1));
  float ms = 0.0f;
  HIP_TRY(hipEventElapsedTime(&ms, s->ev0, s->ev1));
  *ms_per_launch = (double)ms / launches;
  const int lag = s->ph.phi_src_flow ? NLAG - 2 : NLAG - 3;   // planes in use
  const int stat = 2 + (s->ph.subfix == 2 ? 1 : 0);
  *bytes_per_launch = (double)s->G.nx * s->G.ny * 4.0 * (2.0 * (NDIST + lag) + stat);
  return LBF_OK;
}

}  // extern "C"

// ================================================================ batch
struct lbf_batch {
  std::vector<lbf_sim*> sims;
  hipStream_t stream;
  int tile_x, tile_y;
  bool mrt;                      // some lattice uses MRT: launch the kernel with its branches
  int grid;                      // persistent workgroups
  InstDesc* d_desc;
  int2* d_items;
  int nitems;
  std::vector<InstDesc> h_desc;  // host copy (source of the uploads)
  std::vector<int> desc_cur;     // sims' parity the descriptors were built for
  bool built;                    // work list, grid and graph match the tile shape
  hipGraphExec_t graph;          // kGraphSteps launches, parities alternating
  bool have_graph;
  hipStream_t capture;           // private stream the graph is recorded on (the
                                 // legacy default stream cannot be captured)
  bool timing;
  double last_ms;
  hipEvent_t ev0, ev1;
};

namespace {

constexpr int kGraphSteps = 32;

void batch_free_graph(lbf_batch* b) {
  if (b->have_graph) (void)hipGraphExecDestroy(b->graph);
  b->have_graph = false;
}

// Descriptors for the sims' current parities (A[0] steps the current state).
int batch_upload_desc(lbf_batch* b) {
  const int n = (int)b->sims.size();
  b->h_desc.assign(n, InstDesc{});
  for (int i = 0; i < n; ++i) {
    lbf_sim* s = b->sims[i];
    InstDesc& d = b->h_desc[i];
    d.G = s->G;
    d.ph = s->ph;
    for (int p = 0; p < 2; ++p) {
      const int c = s->cur ^ p;
      BufArgs A{};
      A.din = fptr(s, s->L.dist[c]);
      A.dout = fptr(s, s->L.dist[1 - c]);
      A.lin = fptr(s, s->L.lag[c]);
      A.lout = fptr(s, s->L.lag[1 - c]);
      A.stat = fptr(s, s->L.stat);
      A.wallT = fptr(s, s->L.wall);
      A.wstride = s->L.wstride;
      d.A[p] = A;
    }
    d.CY = b->tile_y;
    d.nbx = (s->G.nx + b->tile_x - 1) / b->tile_x;
  }
  HIP_TRY(hipMemcpyAsync(b->d_desc, b->h_desc.data(), n * sizeof(InstDesc),
                         hipMemcpyHostToDevice, b->stream));
  HIP_TRY(hipStreamSynchronize(b->stream));
  // recorded only once the device copy is in place
  for (int i = 0; i < n; ++i) b->desc_cur[i] = b->sims[i]->cur;
  return LBF_OK;
}

// Work list (tiles of every lattice, larger lattices first) and grid for the
// current tile shape.
int batch_build(lbf_batch* b) {
  const int n = (int)b->sims.size();
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int c) {
    return (long long)b->sims[a]->G.nx * b->sims[a]->G.ny >
           (long long)b->sims[c]->G.nx * b->sims[c]->G.ny;
  });
  std::vector<int2> items;
  for (int i : order) {
    const int nbx = (b->sims[i]->G.nx + b->tile_x - 1) / b->tile_x;
    const int nby = (b->sims[i]->G.ny + b->tile_y - 1) / b->tile_y;
    for (int t = 0; t < nbx * nby; ++t) items.push_back(make_int2(i, t));
  }
  HIP_TRY(hipStreamSynchronize(b->stream));
  batch_free_graph(b);
  if (b->d_items) (void)hipFree(b->d_items);
  b->d_items = nullptr;
  if (!b->d_desc) HIP_TRY(hipMalloc((void**)&b->d_desc, n * sizeof(InstDesc)));
  HIP_TRY(hipMalloc((void**)&b->d_items, items.size() * sizeof(int2)));
  HIP_TRY(hipMemcpyAsync(b->d_items, items.data(), items.size() * sizeof(int2),
                         hipMemcpyHostToDevice, b->stream));
  b->nitems = (int)items.size();
  int dev = 0, ncu = 0, per_cu = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
  // as many workgroups as fit on the device at once (register- and
  // LDS-limited), never many more than there are items
  b->mrt = false;
  for (lbf_sim* sm : b->sims) b->mrt = b->mrt || sm->ph.mrt;
  const void* kern = nullptr;
  switch (b->tile_x) {
    case 64:
      kern = b->mrt ? reinterpret_cast<const void*>(batch_step_kernel<64, true>)
                    : reinterpret_cast<const void*>(batch_step_kernel<64, false>);
      break;
    case 128:
      kern = b->mrt ? reinterpret_cast<const void*>(batch_step_kernel<128, true>)
                    : reinterpret_cast<const void*>(batch_step_kernel<128, false>);
      break;
    default:
      kern = b->mrt ? reinterpret_cast<const void*>(batch_step_kernel<256, true>)
                    : reinterpret_cast<const void*>(batch_step_kernel<256, false>);
      break;
  }
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, b->tile_x, 0));
  per_cu = std::max(per_cu, 1);
  b->grid = std::max(8, std::min(per_cu * ncu, (b->nitems + 7) / 8 * 8));
  b->grid = (b->grid + 7) / 8 * 8;
  b->built = true;
  return batch_upload_desc(b);
}

template <int WX>
void batch_launch_wx(lbf_batch* b, int parity, hipStream_t st) {
  if (b->mrt)   // some lattice of the batch uses MRT: the kernel with the MRT branches
    hipLaunchKernelGGL((batch_step_kernel<WX, true>), dim3(b->grid), dim3(WX), 0, st,
                       (const InstDesc*)b->d_desc, (const int2*)b->d_items, b->nitems, parity);
  else
    hipLaunchKernelGGL((batch_step_kernel<WX, false>), dim3(b->grid), dim3(WX), 0, st,
                       (const InstDesc*)b->d_desc, (const int2*)b->d_items, b->nitems, parity);
}

int batch_launch(lbf_batch* b, int parity, hipStream_t st) {
  switch (b->tile_x) {
    case 64: batch_launch_wx<64>(b, parity, st); break;
    case 128: batch_launch_wx<128>(b, parity, st); break;
    default: batch_launch_wx<256>(b, parity, st); break;
  }
  HIP_TRY(hipGetLastError());
  return LBF_OK;
}

}  // namespace

extern "C" {

int lbf_batch_create(lbf_sim* const* sims, int32_t n, lbf_batch** out) {
  if (!out) return fail(LBF_EINVAL, "out is NULL");
  *out = nullptr;
  if (!sims || n < 1) return fail(LBF_EINVAL, "a batch needs at least one simulation");
  for (int i = 0; i < n; ++i) {
    if (!sims[i]) return fail(LBF_EINVAL, "simulation %d is NULL", i);
    if (!sims[i]->have_init) return fail(LBF_ESTATE, "simulation %d is not initialised", i);
    if (sims[i]->stream != sims[0]->stream)
      return fail(LBF_EINVAL, "all simulations of a batch must share one stream");
    for (int j = 0; j < i; ++j)
      if (sims[j] == sims[i]) return fail(LBF_EINVAL, "simulation %d appears twice", i);
  }
  lbf_batch* b = new (std::nothrow) lbf_batch();
  if (!b) return fail(LBF_ENOMEM, "host allocation failed");
  try {
    b->sims.assign(sims, sims + n);
    b->desc_cur.assign(n, -1);
  } catch (const std::bad_alloc&) {
    delete b;
    return fail(LBF_ENOMEM, "host allocation failed");
  }
  b->stream = sims[0]->stream;
  b->tile_x = 128;
  b->tile_y = 32;
  if (hipEventCreate(&b->ev0) != hipSuccess || hipEventCreate(&b->ev1) != hipSuccess ||
      hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking) != hipSuccess) {
    lbf_batch_destroy(b);
    return fail(LBF_EHIP, "event / stream creation failed");
  }
  *out = b;
  return LBF_OK;
}

int lbf_batch_set_tile(lbf_batch* b, int32_t tile_x, int32_t tile_y) {
  if (!b) return fail(LBF_EINVAL, "batch is NULL");
  if (tile_x != 64 && tile_x != 128 && tile_x != 256)
    return fail(LBF_EINVAL, "tile_x must be 64, 128 or 256 (got %d)", tile_x);
  if (tile_y < 1 || tile_y > CY_MAX)
    return fail(LBF_EINVAL, "tile_y must be in [1, %d] (got %d)", CY_MAX, tile_y);
  if (tile_x != b->tile_x || tile_y != b->tile_y) b->built = false;
  b->tile_x = tile_x;
  b->tile_y = tile_y;
  return LBF_OK;
}

int lbf_batch_step(lbf_batch* b, int32_t nsteps) {
  if (!b) return fail(LBF_EINVAL, "batch is NULL");
  if (nsteps < 0) return fail(LBF_EINVAL, "nsteps %d", nsteps);
  if (nsteps == 0) return LBF_OK;
  for (size_t i = 0; i < b->sims.size(); ++i)
    if (!b->sims[i]->have_init)
      return fail(LBF_ESTATE, "simulation %zu of the batch has no state (new geometry without "
                              "lbf_init_fields or a loaded state)", i);
  try {   // the work-item list and descriptors are built in host vectors
    if (!b->built) {
      int rc = batch_build(b);
      if (rc) return rc;
    } else {
      for (size_t i = 0; i < b->sims.size(); ++i)
        if (b->sims[i]->cur != b->desc_cur[i]) {
          int rc = batch_upload_desc(b);
          if (rc) return rc;
          break;
        }
    }
  } catch (const std::bad_alloc&) {
    return fail(LBF_ENOMEM, "host allocation failed");
  }
  if (b->timing) HIP_TRY(hipEventRecord(b->ev0, b->stream));
  int done = 0;
  if (nsteps >= kGraphSteps) {
    if (!b->have_graph) {
      // one graph of kGraphSteps persistent launches, parities alternating
      hipGraph_t g = nullptr;
      HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
      int rc = LBF_OK;
      for (int k = 0; k < kGraphSteps && rc == LBF_OK; ++k) rc = batch_launch(b, k & 1, b->capture);
      const hipError_t ec = hipStreamEndCapture(b->capture, &g);
      if (rc == LBF_OK && ec != hipSuccess)
        rc = fail(LBF_EHIP, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
      if (rc == LBF_OK && hipGraphInstantiate(&b->graph, g, nullptr, nullptr, 0) != hipSuccess)
        rc = fail(LBF_EHIP, "hipGraphInstantiate failed");
      if (g) (void)hipGraphDestroy(g);   // the executable graph keeps its own copy
      if (rc) return rc;
      b->have_graph = true;
    }
    // kGraphSteps is even: each replay leaves every parity where it started
    while (nsteps - done >= kGraphSteps) {
      HIP_TRY(hipGraphLaunch(b->graph, b->stream));
      done += kGraphSteps;
    }
  }
  for (int k = 0; done < nsteps; ++k, ++done) {
    int rc = batch_launch(b, k & 1, b->stream);
    if (rc) return rc;
  }
  if (b->timing) {
    HIP_TRY(hipEventRecord(b->ev1, b->stream));
    HIP_TRY(hipEventSynchronize(b->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, b->ev0, b->ev1));
    b->last_ms = ms / nsteps;
  }
  for (lbf_sim* s : b->sims) {
    s->cur ^= nsteps & 1;
    s->step += nsteps;
    s->have_budget = false;
  }
  return LBF_OK;
}

int lbf_batch_set_timing(lbf_batch* b, int32_t on) {
  if (!b) return fail(LBF_EINVAL, "batch is NULL");
  b->timing = on != 0;
  return LBF_OK;
}

double lbf_batch_last_step_ms(const lbf_batch* b) { return b ? b->last_ms : 0.0; }

int32_t lbf_batch_items(const lbf_batch* b) { return b && b->built ? b->nitems : 0; }

void lbf_batch_destroy(lbf_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  batch_free_graph(b);
  if (b->d_desc) (void)hipFree(b->d_desc);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->ev0) (void)hipEventDestroy(b->ev0);
  if (b->ev1) (void)hipEventDestroy(b->ev1);
  if (b->capture) (void)hipStreamDestroy(b->capture);
  delete b;
}

}  // extern "C"
