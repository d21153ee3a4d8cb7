// C ABI of the three-dimensional (D3Q19) coupled step (contracts in
// include/lbf3.h).  Two kernels per step, one node per lane: the moments pass
// pulls g and h and stores phi, f_s and rho for the stencils (and, with the
// flow-divergence phase-field source, the divergence of the previous step's
// velocity from its eighteen neighbours); the step pass
// pulls f, g and h, accumulates the 3D stencils from those planes, collides
// and stores the next state.  Workgroups are dealt to the XCDs in contiguous
// bands of nodes so that the y and z neighbours a band reads stay in one L2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "lbf3.h"
#include "lbf3_device.hpp"
#include "lbf_sim.hpp"
#include "lbf_step.hpp"

using namespace lbf3;
using lbfi::fail;

namespace {

constexpr size_t kAlign3 = 256;
size_t up3(size_t v, size_t a) { return (v + a - 1) / a * a; }
// 19 planes per buffer resource with 32-bit byte offsets
constexpr long long kMaxNodes3 = (0xFFFFFFFFLL / (4LL * NQ)) / 64 * 64;
constexpr int kRed3 = 6;   // sum g, sum h, sum f_s, liquid PCM, max |u|, non-finite

struct Layout3 {
  size_t dist[2], lag[2], stat, mom, fields, red, redfinal, total;
  size_t P;       // plane stride inside a block
  size_t GS;      // block stride (one block: unused)
  size_t AS;      // floats of one of the f, g, h arrays
  size_t PL;      // plane stride of the linear arrays
  int nblk;       // row blocks
  int nblocks;    // workgroups of a pass
};

bool valid_row_block3(int rb) {
  return rb == 0 || rb == 1 || rb == 2 || rb == 4 || rb == 8 || rb == 16 || rb == 32 || rb == 64;
}

// Row blocks: rb rows of nx nodes per block, the block stride the power of
// two at or above the 19 planes of the f, g and h arrays; rb = 0: one block
// (plane-major, plane stride the node count rounded up to 64 plus the pad).
Layout3 make_layout3(int nx, int ny, int nz, int pad, int rb) {
  Layout3 L{};
  const size_t n = (size_t)nx * ny * nz, rows = (size_t)ny * nz;
  L.PL = up3(n, 64);
  if (rb) {
    L.P = up3((size_t)rb * nx, 64) + pad;
    L.nblk = (int)((rows + rb - 1) / rb);
    L.GS = 1;
    while (L.GS < NQ * L.P) L.GS <<= 1;
  } else {
    L.P = up3(n, 64) + pad;
    L.nblk = 1;
    L.GS = NQ * L.P;
  }
  const size_t base = (size_t)(L.nblk - 1) * L.GS;
  L.AS = base + NQ * L.P;
  L.nblocks = (int)((n + 255) / 256);
  size_t off = 0;
  auto take = [&](size_t b) {
    size_t o = off;
    off = up3(off + b, kAlign3);
    return o;
  };
  L.dist[0] = take(3 * L.AS * sizeof(float));
  L.dist[1] = take(3 * L.AS * sizeof(float));
  L.lag[0] = take((base + NLAG * L.P) * sizeof(float));
  L.lag[1] = take((base + NLAG * L.P) * sizeof(float));
  L.stat = take((base + NSTAT * L.P) * sizeof(float));
  L.mom = take(5 * L.PL * sizeof(float));   // 16-byte records, then the div u plane
  L.fields = take(NFIELD * L.PL * sizeof(float));
  L.red = take((size_t)L.nblocks * kRed3 * sizeof(double));
  L.redfinal = take(kRed3 * sizeof(double));
  L.total = off;
  return L;
}

__device__ __forceinline__ void coords(const Geo3& G, int k, int& x, int& y, int& z) {
  x = k % G.n[0];
  const int r = k / G.n[0];
  y = r % G.n[1];
  z = r / G.n[1];
}

__device__ __forceinline__ int node_of_block(int nblocks) {
  return lbf::xcd_tile(blockIdx.x, nblocks) * 256 + threadIdx.x;
}

// Node of position q of the step pass's order: strips of S rows, each walked
// slab by slab in z (x fastest within a slab's part of the strip), so the
// stencil's z neighbours were touched S nx nodes earlier; S >= ny is the
// plain x-fastest order.  A bijection of [0, N).
__device__ __forceinline__ int node_in_strips(const Geo3& G, int q) {
  const int nx = G.n[0], ny = G.n[1], nz = G.n[2];
  const int S = min(G.strip, ny);
  const int full = ny / S;
  const int per = S * nx * nz;
  if (q < full * per) {
    const int s = q / per, rem = q - s * per;
    const int z = rem / (S * nx), r = rem - z * S * nx;
    return (z * ny + s * S) * nx + r;
  }
  const int rows = ny - full * S, rem = q - full * per;
  const int z = rem / (rows * nx), r = rem - z * rows * nx;
  return (z * ny + full * S) * nx + r;
}

__global__ __launch_bounds__(256) void k3_lap_static(Geo3 G, float* stat, int N) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  int x, y, z;
  coords(G, k, x, y, z);
  const uint32_t s = sidx3(G, x, y, z);
  const float* phi0 = stat + ST_PHI0 * (size_t)G.P;
  const float c = phi0[s];
  float lap = 0.0f;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    const int xx = nb3(x + cx(i), G.n[0], G.per[0]), yy = nb3(y + cy(i), G.n[1], G.per[1]);
    const int zz = nb3(z + cz(i), G.n[2], G.per[2]);
    lap += wgt(i) * (phi0[sidx3(G, xx, yy, zz)] - c);
  }
  stat[ST_LAP0 * (size_t)G.P + s] = 6.0f * lap;
}

// Equilibria of the initial state in post-stream form (tmp: the f, g, h
// arrays); `in` holds phi (plane 0) and T (plane 1), linear, PL apart.
__global__ __launch_bounds__(256) void k3_init_eq(Geo3 G, Phys ph, const float* stat,
                                                  const float* in, float* tmp, int N) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  int x, y, z;
  coords(G, k, x, y, z);
  const size_t P = G.P, AS = G.AS;
  const uint32_t s = sidx3(G, x, y, z);
  const float pc = in[k];
  float lap = 0.0f;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    const int xx = nb3(x + cx(i), G.n[0], G.per[0]), yy = nb3(y + cy(i), G.n[1], G.per[1]);
    const int zz = nb3(z + cz(i), G.n[2], G.per[2]);
    lap += wgt(i) * (in[((size_t)zz * G.n[1] + yy) * G.n[0] + xx] - pc);
  }
  lap *= 6.0f;
  const float phi0 = stat[ST_PHI0 * P + s];
  const float mu = lbf::chem_pot(ph, pc, lap, phi0, stat[ST_CTH * P + s], stat[ST_LAP0 * P + s],
                                 0.0f, 0.0f);
  const float C = lbf::clampf(0.5f * (1.0f - phi0 + pc), 0.0f, 1.0f);
  const float Cp = lbf::clampf((C - ph.pcm_floor) * ph.inv_pcm_span, 0.0f, 1.0f);
  const float chi = lbf::clampf(Cp, 0.0f, 1.0f - phi0);
  const float Kliq = lbf::zeta(phi0, C, ph.rho_s, ph.rho_l, ph.rho_g) *
                     lbf::zeta(phi0, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float Tk = in[(size_t)G.PL + k];
  const float rhoH = Kliq * (Tk - ph.T_m) + Kliq * ph.T_m + chi * ph.rho_l * ph.latent;
  const float ET = ph.Eref * Tk;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    tmp[i * P + s] = 0.0f;
    tmp[AS + i * P + s] = (i == 0 ? pc : 0.0f) + (wgt(i) - (i == 0 ? 1.0f : 0.0f)) * mu;
    tmp[2 * AS + i * P + s] = (i == 0) ? rhoH - ET + wgt(0) * ET : wgt(i) * ET;
  }
}

// Inverse of the pull: post-collision populations whose pull gives `tmp`;
// the rest populations become the high parts of their float-float storage.
__global__ __launch_bounds__(256) void k3_unstream(Geo3 G, Phys ph, const float* tmp, float* dst,
                                                   float* lag, int N) {
  const int k = blockIdx.x * 256 + threadIdx.x;
  if (k >= N) return;
  int x, y, z;
  coords(G, k, x, y, z);
  const size_t P = G.P, AS = G.AS;
  const size_t s = sidx3(G, x, y, z);
  dst[s] = tmp[s];
  lag[LAG_GHI * P + s] = tmp[AS + s];
  lag[LAG_HHI * P + s] = tmp[2 * AS + s];
  dst[AS + s] = 0.0f;
  dst[2 * AS + s] = 0.0f;
  for (int j = 1; j < NQ; ++j) {
    // destination of population j leaving the node; the face of its wall
    const int v[3] = {x + cx(j), y + cy(j), z + cz(j)};
    int d[3];
    int face = -1;
    for (int a = 2; a >= 0; --a) {
      d[a] = v[a];
      if (v[a] < 0 || v[a] >= G.n[a]) {
        if (G.per[a]) d[a] = v[a] < 0 ? v[a] + G.n[a] : v[a] - G.n[a];
        else if (face < 0) face = 2 * a + (v[a] < 0 ? 0 : 1);
      }
    }
    if (face < 0) {
      const size_t dk = sidx3(G, d[0], d[1], d[2]);
      for (int b = 0; b < 3; ++b) dst[b * AS + j * P + s] = tmp[b * AS + j * P + dk];
    } else {
      const int i = opp(j);   // the population the node pulls back
      dst[j * P + s] = tmp[i * P + s];
      dst[AS + j * P + s] = tmp[AS + i * P + s];
      const float hb = tmp[2 * AS + i * P + s];
      dst[2 * AS + j * P + s] =
          ((G.tmask >> face) & 1) ? 2.0f * wgt(i) * ph.Eref * G.Tw[face] - hb : hb;
    }
  }
}

// Moments pass: phi, f_s, rho of the state read, for the stencils.
// With the flow-divergence source it walks the step pass's strip order: the
// divergence reads the z neighbours' velocity, which is then still in L2.
__global__ __launch_bounds__(256) void k3_moments(Geo3 G, Phys ph, BufArgs3 A, int N, int nblocks) {
  const int q = node_of_block(nblocks);
  if (q >= N) return;
  const int k = ph.phi_src_flow ? node_in_strips(G, q) : q;
  int x, y, z;
  coords(G, k, x, y, z);
  const Bufs3 B = make_bufs3(A, G);
  Pull19 n;
  pull19(G, x, y, z, n);
  const int s = (int)(n.k4 >> 2);   // storage index of the node
  float gv[NQ], hv[NQ];
  pull_gh3(G, ph, B, n, gv, hv);
  // the flow-divergence phase-field source: div u of the previous step, kept
  // for the step pass (which reads it instead of gathering the velocity again)
  float dl = 0.0f;
  if (ph.phi_src_flow) {
    dl = div3(G, B, n);
    lbf::stp(B.mom, MOM_DIVU, G.PL, k, dl);
  }
  Mom m;
  node_moments3(G, ph, B, (uint32_t)s, gv, hv, lbf::ldp(B.stat, ST_PHI0, G.P, s), m, dl);
  st_rec(B.mom, (uint32_t)k * 16u, m.phi, m.fs, m.rho, lbf::ldp(B.lin, LAG_P, G.P, s));
}

// Step pass (READOUT = false) or read-out of the fields with FP64 block sums
// (READOUT = true).
template <bool READOUT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8))) void k3_step(
    Geo3 G, Phys ph, BufArgs3 A, float* fields, double* red, int N, int nblocks) {
  const int q = node_of_block(nblocks);
  const bool act = q < N;
  const int k = act ? node_in_strips(G, q) : q;
  double v[kRed3] = {0, 0, 0, 0, 0, 0};
  if (act) {
    int x, y, z;
    coords(G, k, x, y, z);
    const Bufs3 B = make_bufs3(A, G);
    const size_t PL = G.PL;
    Pull19 n;
    pull19(G, x, y, z, n);
    const int s = (int)(n.k4 >> 2);   // storage index of the node
    float gv[NQ], hv[NQ], fv[NQ];
    pull_gh3(G, ph, B, n, gv, hv);
    const float phi0 = lbf::ldp(B.stat, ST_PHI0, G.P, s);
    const float dl = ph.phi_src_flow ? lbf::ldp(B.mom, MOM_DIVU, G.PL, k) : 0.0f;
    Mom m;
    node_moments3(G, ph, B, (uint32_t)s, gv, hv, phi0, m, dl);
    Stencil3 S;
    stencils3(G, B, n, m.phi, m.fs, S);
    pull_f3(G, B, n, fv);
    const float jprev[3] = {lbf::ldp(B.lin, LAG_JX, G.P, s), lbf::ldp(B.lin, LAG_JY, G.P, s),
                            lbf::ldp(B.lin, LAG_JZ, G.P, s)};
    const float ref_h = lbf::ldp(B.lin, LAG_HHI, G.P, s);
    Post3 o;
    collide3(ph, m, S, phi0, lbf::ldp(B.stat, ST_CTH, G.P, s), lbf::ldp(B.stat, ST_LAP0, G.P, s),
             jprev, ref_h, fv, gv, hv, o);
    if (!READOUT) {
#pragma unroll
      for (int i = 0; i < NQ; ++i) {
        lbf::stp(B.fout, i, G.P, s, fv[i]);
        lbf::stp(B.gout, i, G.P, s, gv[i]);
        lbf::stp(B.hout, i, G.P, s, hv[i]);
      }
      lbf::stp(B.lout, LAG_FS, G.P, s, m.fs);
      lbf::stp(B.lout, LAG_Q, G.P, s, o.Q);
      lbf::stp(B.lout, LAG_JX, G.P, s, o.j[0]);
      lbf::stp(B.lout, LAG_JY, G.P, s, o.j[1]);
      lbf::stp(B.lout, LAG_JZ, G.P, s, o.j[2]);
      lbf::stp(B.lout, LAG_P, G.P, s, o.p);
      lbf::stp(B.lout, LAG_GHI, G.P, s, o.ghi);
      lbf::stp(B.lout, LAG_HHI, G.P, s, o.hhi);
      if (ph.phi_src_flow) {
        lbf::stp(B.lout, LAG_UX, G.P, s, o.u[0]);
        lbf::stp(B.lout, LAG_UY, G.P, s, o.u[1]);
        lbf::stp(B.lout, LAG_UZ, G.P, s, o.u[2]);
      }
    } else {
      const float mu = lbf::chem_pot(ph, m.phi, S.lphi, phi0, lbf::ldp(B.stat, ST_CTH, G.P, s),
                                     lbf::ldp(B.stat, ST_LAP0, G.P, s), m.fs, S.lfs);
      const float out[NFIELD] = {m.phi, m.T, 1.0f - m.fs, m.fs, o.u[0], o.u[1], o.u[2], o.p,
                                 m.rhoH, mu, m.C, m.chi, m.rho, m.ref_g + m.sg};
#pragma unroll
      for (int f = 0; f < NFIELD; ++f) fields[f * PL + k] = out[f];
      const float um = sqrtf(o.u[0] * o.u[0] + o.u[1] * o.u[1] + o.u[2] * o.u[2]);
      v[0] = (double)m.ref_g + (double)m.sg;
      v[1] = (double)ref_h + (double)m.sh;
      v[2] = m.fs;
      v[3] = m.chi - m.fs;
      v[4] = um;
      v[5] = (!isfinite(m.phi) || !isfinite(m.T) || !isfinite(um) || !isfinite(o.p)) ? 1.0 : 0.0;
    }
  }
  if (READOUT) {
    __shared__ double s[4][kRed3];
#pragma unroll
    for (int j = 0; j < kRed3; ++j)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double t = __shfl_down(v[j], off, 64);
        v[j] = (j == 4) ? fmax(v[j], t) : v[j] + t;
      }
    const int l = threadIdx.x;
    if ((l & 63) == 0)
      for (int j = 0; j < kRed3; ++j) s[l >> 6][j] = v[j];
    __syncthreads();
    if (l < kRed3) {
      double t = s[0][l];
      for (int w = 1; w < 4; ++w) t = (l == 4) ? fmax(t, s[w][l]) : t + s[w][l];
      red[(size_t)lbf::xcd_tile(blockIdx.x, nblocks) * kRed3 + l] = t;
    }
  }
}

__global__ void k3_reduce_final(const double* part, int nblocks, double* out) {
  __shared__ double s[256];
  for (int j = 0; j < kRed3; ++j) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) {
      const double t = part[(size_t)b * kRed3 + j];
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

// Every byte offset a kernel forms fits 32 bits: 19 planes of the
// plane-major layout, or one whole f, g or h array of row blocks.
bool fits3(int nx, int ny, int nz, int pad, int rb) {
  const long long n = (long long)nx * ny * nz;
  if (n > kMaxNodes3 || (long long)up3((size_t)n, 64) + pad > kMaxNodes3) return false;
  if (!rb) return true;
  return make_layout3(nx, ny, nz, pad, rb).AS * 4ull <= 0xFFFFFFFFull;
}

int validate3(const lbf3_params* p) {
  if (!p) return fail(LBF_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1 || p->nz < 1)
    return fail(LBF_EINVAL, "lattice size %d x %d x %d", p->nx, p->ny, p->nz);
  if (p->plane_pad < 0 || p->plane_pad > lbfi::kMaxPlanePad || p->plane_pad % 64)
    return fail(LBF_EINVAL, "plane_pad %d (a multiple of 64 in [0, %d])", p->plane_pad,
                lbfi::kMaxPlanePad);
  if (!valid_row_block3(p->row_block))
    return fail(LBF_EINVAL, "row_block %d (0, 1, 2, 4, 8, 16, 32 or 64)", p->row_block);
  if (!fits3(p->nx, p->ny, p->nz, p->plane_pad, p->row_block))
    return fail(LBF_EINVAL, "lattice of %lld nodes exceeds the 32-bit offset limit of its layout "
                "(row_block %d)", (long long)p->nx * p->ny * p->nz, p->row_block);
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
  for (int f = 0; f < 6; ++f)
    if (p->thermal_bc[f] != LBF_ADIABATIC && p->thermal_bc[f] != LBF_DIRICHLET)
      return fail(LBF_EINVAL, "thermal_bc[%d] = %d", f, p->thermal_bc[f]);
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p->grav[a]) || !std::isfinite(p->u_solid[a]))
      return fail(LBF_EINVAL, "grav and u_solid must be finite");
  if (p->phi_src_mdot != 0 && p->phi_src_mdot != 1)
    return fail(LBF_EINVAL, "phi_src_mdot = %d", p->phi_src_mdot);
  const double cpref = 2.0 * p->cp_s * p->cp_l / (p->cp_s + p->cp_l);
  const double kmin = std::min({p->rho_l, p->rho_g, p->rho_s}) *
                      std::min({p->cp_l, p->cp_g, p->cp_s});
  if (p->rho_ref * cpref > kmin * (1.0 + 1e-12))
    return fail(LBF_EINVAL, "rho_ref * C_p,ref = %g exceeds the smallest nodal heat capacity %g: "
                            "the enthalpy scheme would be unstable", p->rho_ref * cpref, kmin);
  return LBF_OK;
}

void fill_phys3(const lbf3_params* p, Phys& ph) {
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
  ph.phi_src_flow = p->phi_src_mdot ? 0 : 1;
  for (int a = 0; a < 3; ++a) {
    ph.grav[a] = (float)p->grav[a];
    ph.vsol[a] = (float)p->u_solid[a];
  }
}

}  // namespace

struct lbf3_sim {
  lbf3_params prm;
  Geo3 G;
  Phys ph;
  Layout3 L;
  hipStream_t stream;
  char* ws;
  bool owns_ws, have_geo, have_init, timing;
  int cur;
  long long step;
  double last_ms;
  hipEvent_t ev0, ev1;
  double* host_red;
};

namespace {

float* fp3(lbf3_sim* s, size_t off) { return reinterpret_cast<float*>(s->ws + off); }

int N3(const lbf3_sim* s) { return s->G.n[0] * s->G.n[1] * s->G.n[2]; }

BufArgs3 args3(lbf3_sim* s, int c) {
  BufArgs3 A{};
  A.din = fp3(s, s->L.dist[c]);
  A.dout = fp3(s, s->L.dist[1 - c]);
  A.lin = fp3(s, s->L.lag[c]);
  A.lout = fp3(s, s->L.lag[1 - c]);
  A.stat = fp3(s, s->L.stat);
  A.mom = fp3(s, s->L.mom);
  return A;
}

// Copy one plane between a plain array of nx ny nz values (`flat`) and the
// plane that starts at `plane` in a state or static array, on the
// simulation's stream; `to_plane` gives the direction.
int plane_copy3(lbf3_sim* s, float* plane, float* flat, bool to_plane, hipMemcpyKind kind) {
  const size_t n = (size_t)N3(s);
  if (s->L.nblk == 1) {
    HIP_TRY(hipMemcpyAsync(to_plane ? plane : flat, to_plane ? flat : plane, n * sizeof(float),
                           kind, s->stream));
    return LBF_OK;
  }
  const size_t nx = s->G.n[0], rb = (size_t)s->G.rmask + 1, rows = n / nx;
  const size_t full = rows / rb, rem = rows - full * rb;
  const size_t w = rb * nx * sizeof(float), pitch = s->L.GS * sizeof(float);
  if (full)
    HIP_TRY(hipMemcpy2DAsync(to_plane ? plane : flat, to_plane ? pitch : w,
                             to_plane ? flat : plane, to_plane ? w : pitch, w, full, kind,
                             s->stream));
  if (rem) {
    float* pb = plane + full * s->L.GS;
    float* fb = flat + full * rb * nx;
    HIP_TRY(hipMemcpyAsync(to_plane ? pb : fb, to_plane ? fb : pb, rem * nx * sizeof(float), kind,
                           s->stream));
  }
  return LBF_OK;
}

// Start of plane j (0 .. 56 distributions, then 57 .. 67 lagged) of state
// buffer c.
float* state_plane3(lbf3_sim* s, int c, int j) {
  if (j < NDIST)
    return fp3(s, s->L.dist[c]) + (size_t)(j / NQ) * s->L.AS + (size_t)(j % NQ) * s->L.P;
  return fp3(s, s->L.lag[c]) + (size_t)(j - NDIST) * s->L.P;
}

// Zero the lagged planes of state buffer c (every block).
int zero_lags3(lbf3_sim* s, int c) {
  const size_t w = NLAG * s->L.P * sizeof(float);
  HIP_TRY(hipMemset2DAsync(fp3(s, s->L.lag[c]), s->L.nblk > 1 ? s->L.GS * sizeof(float) : w, 0, w,
                           (size_t)s->L.nblk, s->stream));
  return LBF_OK;
}

int copy3(lbf3_sim* s, void* dst, const void* src, size_t bytes, int on_device) {
  if (hipMemcpyAsync(dst, src, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                     s->stream) != hipSuccess)
    return fail(LBF_EHIP, "hipMemcpyAsync failed");
  if (!on_device && hipStreamSynchronize(s->stream) != hipSuccess)
    return fail(LBF_EHIP, "hipStreamSynchronize failed");
  return LBF_OK;
}

int launch_pair(lbf3_sim* s, bool readout) {
  const int N = N3(s), nb = s->L.nblocks;
  BufArgs3 A = args3(s, s->cur);
  hipLaunchKernelGGL(k3_moments, dim3(nb), dim3(256), 0, s->stream, s->G, s->ph, A, N, nb);
  HIP_TRY(hipGetLastError());
  if (readout)
    hipLaunchKernelGGL((k3_step<true>), dim3(nb), dim3(256), 0, s->stream, s->G, s->ph, A,
                       fp3(s, s->L.fields), reinterpret_cast<double*>(s->ws + s->L.red), N, nb);
  else
    hipLaunchKernelGGL((k3_step<false>), dim3(nb), dim3(256), 0, s->stream, s->G, s->ph, A,
                       (float*)nullptr, (double*)nullptr, N, nb);
  HIP_TRY(hipGetLastError());
  return LBF_OK;
}

}  // namespace

extern "C" {

size_t lbf3_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t plane_pad,
                            int32_t row_block) {
  if (nx < 1 || ny < 1 || nz < 1) return 0;
  if (plane_pad < 0 || plane_pad > lbfi::kMaxPlanePad || plane_pad % 64) return 0;
  if (!valid_row_block3(row_block) || !fits3(nx, ny, nz, plane_pad, row_block)) return 0;
  return make_layout3(nx, ny, nz, plane_pad, row_block).total;
}

int lbf3_create(const lbf3_params* params, void* stream, void* workspace, size_t workspace_bytes,
                lbf3_sim** out) {
  if (!out) return fail(LBF_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate3(params);
  if (rc) return rc;
  lbf3_sim* s = new (std::nothrow) lbf3_sim();
  if (!s) return fail(LBF_ENOMEM, "host allocation failed");
  s->prm = *params;
  s->G.n[0] = params->nx; s->G.n[1] = params->ny; s->G.n[2] = params->nz;
  s->G.tmask = 0;
  s->G.strip = 16;   // measured best of 2 .. 32 rows on 256^3 and the fracture
  for (int a = 0; a < 3; ++a) s->G.per[a] = params->periodic[a] ? 1 : 0;
  for (int f = 0; f < 6; ++f) {
    if (params->thermal_bc[f] == LBF_DIRICHLET) s->G.tmask |= 1 << f;
    s->G.Tw[f] = (float)params->wall_T[f];
  }
  fill_phys3(params, s->ph);
  const int rb = params->row_block;
  s->L = make_layout3(params->nx, params->ny, params->nz, params->plane_pad, rb);
  s->G.P = (int)s->L.P;
  s->G.rbs = 31;
  s->G.gss = 31;
  if (rb) {
    for (s->G.rbs = 0; (1 << s->G.rbs) < rb; ++s->G.rbs) {
    }
    for (s->G.gss = 0; ((size_t)1 << s->G.gss) < s->L.GS; ++s->G.gss) {
    }
  }
  s->G.rmask = rb ? rb - 1 : 0x7fffffff;
  s->G.nblk = s->L.nblk;
  s->G.RBN = rb * params->nx;
  s->G.AS = (int)s->L.AS;
  s->G.PL = (int)s->L.PL;
  s->stream = (hipStream_t)stream;
  if (workspace) {
    if (workspace_bytes < s->L.total || (uintptr_t)workspace % kAlign3) {
      delete s;
      return fail(LBF_ENOMEM, "workspace too small or not 256-byte aligned");
    }
    s->ws = (char*)workspace;
  } else {
    if (hipMalloc((void**)&s->ws, s->L.total) != hipSuccess) {
      delete s;
      return fail(LBF_ENOMEM, "hipMalloc failed");
    }
    s->owns_ws = true;
  }
  if (hipHostMalloc((void**)&s->host_red, kRed3 * sizeof(double), hipHostMallocDefault) !=
          hipSuccess ||
      hipEventCreate(&s->ev0) != hipSuccess || hipEventCreate(&s->ev1) != hipSuccess) {
    lbf3_destroy(s);
    return fail(LBF_EHIP, "host buffer / event creation failed");
  }
  *out = s;
  return LBF_OK;
}

void lbf3_destroy(lbf3_sim* s) {
  if (!s) return;
  if (s->stream) (void)hipStreamSynchronize(s->stream);
  else (void)hipDeviceSynchronize();
  if (s->owns_ws && s->ws) (void)hipFree(s->ws);
  if (s->host_red) (void)hipHostFree(s->host_red);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  delete s;
}

int lbf3_set_geometry(lbf3_sim* s, const float* phi0, const float* cth, int32_t on_device) {
  if (!s || !phi0 || !cth) return fail(LBF_EINVAL, "NULL argument");
  float* stat = fp3(s, s->L.stat);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  int rc = plane_copy3(s, stat + ST_PHI0 * s->L.P, const_cast<float*>(phi0), true, kind);
  if (rc) return rc;
  rc = plane_copy3(s, stat + ST_CTH * s->L.P, const_cast<float*>(cth), true, kind);
  if (rc) return rc;
  if (!on_device) HIP_TRY(hipStreamSynchronize(s->stream));
  hipLaunchKernelGGL(k3_lap_static, dim3(s->L.nblocks), dim3(256), 0, s->stream, s->G, stat,
                     N3(s));
  HIP_TRY(hipGetLastError());
  s->have_geo = true;
  s->have_init = false;
  return LBF_OK;
}

int lbf3_init_fields(lbf3_sim* s, const float* phi, const float* T, int32_t on_device) {
  if (!s || !phi || !T) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_geo) return fail(LBF_ESTATE, "lbf3_set_geometry must precede lbf3_init_fields");
  const size_t n = (size_t)N3(s);
  float* stage = fp3(s, s->L.fields);
  int rc = copy3(s, stage, phi, n * sizeof(float), on_device);
  if (rc) return rc;
  rc = copy3(s, stage + s->L.PL, T, n * sizeof(float), on_device);
  if (rc) return rc;
  s->cur = 0;
  float* tmp = fp3(s, s->L.dist[1]);
  hipLaunchKernelGGL(k3_init_eq, dim3(s->L.nblocks), dim3(256), 0, s->stream, s->G, s->ph,
                     (const float*)fp3(s, s->L.stat), (const float*)stage, tmp, N3(s));
  HIP_TRY(hipGetLastError());
  // both buffers' lagged planes start at zero, so a saved state does not
  // depend on what the workspace held
  for (int c = 0; c < 2; ++c) {
    rc = zero_lags3(s, c);
    if (rc) return rc;
  }
  hipLaunchKernelGGL(k3_unstream, dim3(s->L.nblocks), dim3(256), 0, s->stream, s->G, s->ph,
                     (const float*)tmp, fp3(s, s->L.dist[0]), fp3(s, s->L.lag[0]), N3(s));
  HIP_TRY(hipGetLastError());
  s->step = 0;
  s->have_init = true;
  return LBF_OK;
}

int lbf3_step(lbf3_sim* s, int32_t nsteps) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  if (nsteps < 0) return fail(LBF_EINVAL, "nsteps %d", nsteps);
  if (!s->have_init) return fail(LBF_ESTATE, "lbf3_init_fields must precede lbf3_step");
  if (nsteps == 0) return LBF_OK;
  if (s->timing) HIP_TRY(hipEventRecord(s->ev0, s->stream));
  for (int it = 0; it < nsteps; ++it) {
    int rc = launch_pair(s, false);
    if (rc) return rc;
    s->cur = 1 - s->cur;
    s->step++;
  }
  if (s->timing) {
    HIP_TRY(hipEventRecord(s->ev1, s->stream));
    HIP_TRY(hipEventSynchronize(s->ev1));
    float ms = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms, s->ev0, s->ev1));
    s->last_ms = ms / nsteps;
  }
  return LBF_OK;
}

int lbf3_read_fields(lbf3_sim* s, float* dst, int32_t dst_on_device) {
  if (!s || !dst) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  int rc = launch_pair(s, true);
  if (rc) return rc;
  const size_t n = (size_t)N3(s);
  for (int f = 0; f < NFIELD; ++f)
    HIP_TRY(hipMemcpyAsync(dst + f * n, fp3(s, s->L.fields) + f * s->L.PL, n * sizeof(float),
                           dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

int lbf3_reduce(lbf3_sim* s, double* out) {
  if (!s || !out) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  int rc = launch_pair(s, true);
  if (rc) return rc;
  double* fin = reinterpret_cast<double*>(s->ws + s->L.redfinal);
  hipLaunchKernelGGL(k3_reduce_final, dim3(1), dim3(256), 0, s->stream,
                     (const double*)(s->ws + s->L.red), s->L.nblocks, fin);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(s->host_red, fin, kRed3 * sizeof(double), hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  for (int j = 0; j < LBF_NRED; ++j) out[j] = 0.0;
  for (int j = 0; j < kRed3; ++j) out[j] = s->host_red[j];
  out[LBF_RED_STEP] = (double)s->step;
  if (out[LBF_RED_NONFINITE] > 0 || !(out[LBF_RED_UMAX] <= 0.3))
    return fail(LBF_EUNSTABLE, "unstable: %g non-finite nodes, max |u| = %g",
                out[LBF_RED_NONFINITE], out[LBF_RED_UMAX]);
  return LBF_OK;
}

// The saved state holds each plane's nx * ny * nz values back to back, so it
// loads into a simulation of the same lattice whatever its plane_pad.
constexpr long long kState3Magic = 0x6c626634LL;

size_t lbf3_state_bytes(const lbf3_sim* s) {
  if (!s) return 0;
  return (size_t)(NDIST + NLAG) * N3(s) * sizeof(float) + 64;
}

int lbf3_save_state(lbf3_sim* s, void* dst, size_t cap) {
  if (!s || !dst) return fail(LBF_EINVAL, "NULL argument");
  if (!s->have_init) return fail(LBF_ESTATE, "not initialised");
  const size_t need = lbf3_state_bytes(s);
  if (cap < need) return fail(LBF_ENOMEM, "state needs %zu bytes", need);
  char* d = (char*)dst;
  const size_t n = (size_t)N3(s), nb = n * sizeof(float);
  const size_t db = NDIST * nb, lb = NLAG * nb;
  for (int j = 0; j < NDIST + NLAG; ++j) {
    int rc = plane_copy3(s, state_plane3(s, s->cur, j), (float*)d + j * n, false,
                         hipMemcpyDeviceToDevice);
    if (rc) return rc;
  }
  long long hdr[8] = {kState3Magic, s->step, s->G.n[0], s->G.n[1], s->G.n[2], 0, 0, 0};
  HIP_TRY(hipMemcpyAsync(d + db + lb, hdr, sizeof hdr, hipMemcpyHostToDevice, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return LBF_OK;
}

int lbf3_load_state(lbf3_sim* s, const void* src, size_t bytes) {
  if (!s || !src) return fail(LBF_EINVAL, "NULL argument");
  const size_t need = lbf3_state_bytes(s);
  if (bytes < need) return fail(LBF_EINVAL, "state of %zu bytes, %zu needed", bytes, need);
  if (!s->have_geo) return fail(LBF_ESTATE, "lbf3_set_geometry must precede lbf3_load_state");
  const char* d = (const char*)src;
  const size_t n = (size_t)N3(s), nb = n * sizeof(float);
  const size_t db = NDIST * nb, lb = NLAG * nb;
  long long hdr[8];
  HIP_TRY(hipMemcpyAsync(hdr, d + db + lb, sizeof hdr, hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (hdr[0] != kState3Magic || hdr[2] != s->G.n[0] || hdr[3] != s->G.n[1] ||
      hdr[4] != s->G.n[2])
    return fail(LBF_EINVAL, "state buffer does not match this lattice");
  for (int j = 0; j < NDIST + NLAG; ++j) {
    int rc = plane_copy3(s, state_plane3(s, s->cur, j), (float*)d + j * n, true,
                         hipMemcpyDeviceToDevice);
    if (rc) return rc;
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->step = hdr[1];
  s->have_init = true;
  return LBF_OK;
}

int lbf3_set_strip(lbf3_sim* s, int32_t rows) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  if (rows < 1) return fail(LBF_EINVAL, "rows %d", rows);
  s->G.strip = rows;
  return LBF_OK;
}

int lbf3_set_timing(lbf3_sim* s, int32_t on) {
  if (!s) return fail(LBF_EINVAL, "sim is NULL");
  s->timing = on != 0;
  return LBF_OK;
}

double lbf3_last_step_ms(const lbf3_sim* s) { return s ? s->last_ms : 0.0; }

}  // extern "C"
