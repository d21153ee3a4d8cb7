// Fused coupled step: one kernel pass per time step.
//
// A block of WX lanes owns a strip of WX columns and marches up CY rows.
// Each lane keeps the pulled g and h of its current row in registers.  For
// the 9-point stencils of phi, f_s, rho (and the lagged p) the block keeps a
// ring of four rows of those values in LDS, WX + 2 wide; the row above the
// current one is computed (pull + moments) one iteration ahead, so the
// moments of every node are computed once per block, plus one halo row at
// each end of the strip and the two halo columns.  One barrier per row.
#pragma once
#include "lbf_device.hpp"

namespace lbf {

template <int WX>
struct StepShared {
  float v[4][4][WX + 2];   // [phi, fs, rho, p_prev][ring slot][column]
  double red[WX / 64][NRED];
};

// Moments of node (xx, yy), written into LDS column `col` of ring slot
// `slot`.  The pulled g/h and moments are returned for the lane's own node.
template <int WX>
__device__ __forceinline__ void node_into_ring(const Geo& G, const Phys& ph, const Bufs& B,
                                               StepShared<WX>& sh, int xx, int yy, int slot,
                                               int col, float* gv, float* hv, Mom& m,
                                               float& flux, float& Qp) {
  pull_gh(G, ph, B, xx, yy, gv, hv, flux);
  float sg = 0.0f, shh = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    sg += gv[i];
    shh += hv[i];
  }
  const int k = yy * G.nx + xx;
  const long long P = G.P;
  const float fsp = B.lin[LAG_FS * P + k];
  Qp = B.lin[LAG_Q * P + k];
  const float phi0 = B.stat[ST_PHI0 * P + k];
  moments(ph, sg, shh, fsp, Qp, phi0, m);
  sh.v[0][slot][col] = m.phi;
  sh.v[1][slot][col] = m.fs;
  sh.v[2][slot][col] = m.rho;
  sh.v[3][slot][col] = B.lin[LAG_P * P + k];
}

template <int WX>
__device__ __forceinline__ void halo_into_ring(const Geo& G, const Phys& ph, const Bufs& B,
                                               StepShared<WX>& sh, int xx, int yy, int slot,
                                               int col) {
  float gv[9], hv[9], flux = 0.0f, Qp;
  Mom m;
  node_into_ring<WX>(G, ph, B, sh, xx, yy, slot, col, gv, hv, m, flux, Qp);
}

// One strip (bx, by) of the lattice.  MODE_STEP writes the next state;
// MODE_FIELDS writes the read-out fields of the current state.  With RED,
// per-block FP64 partial sums go to `red_out` (NRED doubles).
template <int WX, int MODE, bool RED>
__device__ void step_strip(const Geo& G, const Phys& ph, const Bufs& B, int bx, int by, int CY,
                           double* red_out, StepShared<WX>& sh) {
  const int l = threadIdx.x;
  const int x0 = bx * WX;
  const int x = x0 + l;
  const bool act = x < G.nx;
  const int lastl = min(WX, G.nx - x0) - 1;
  const int y0 = by * CY;
  const int y1 = min(y0 + CY, G.ny);
  const int xl = map_axis(x0 - 1, G.nx, G.px);
  const int xr = map_axis(x0 + lastl + 1, G.nx, G.px);
  const long long P = G.P;

  double a_sg = 0, a_sh = 0, a_fs = 0, a_liq = 0, a_umax = 0, a_bad = 0;
  double a_sphi = 0, a_heat = 0, a_flux = 0, a_reset = 0;

  float cg[9], ch[9], cflux = 0.0f, cQp = 0.0f;
  Mom cm;
  // prologue: rows y0 - 1 (halo) and y0
  {
    const int r = map_axis(y0 - 1, G.ny, G.py);
    const int slot = (y0 + 3) & 3;
    if (act) {
      float gv[9], hv[9], fl = 0.0f, q;
      Mom m;
      node_into_ring<WX>(G, ph, B, sh, x, r, slot, l + 1, gv, hv, m, fl, q);
    }
    if (l == 0) halo_into_ring<WX>(G, ph, B, sh, xl, r, slot, 0);
    if (l == lastl) halo_into_ring<WX>(G, ph, B, sh, xr, r, slot, lastl + 2);
  }
  {
    const int slot = y0 & 3;
    if (act) node_into_ring<WX>(G, ph, B, sh, x, y0, slot, l + 1, cg, ch, cm, cflux, cQp);
    if (l == 0) halo_into_ring<WX>(G, ph, B, sh, xl, y0, slot, 0);
    if (l == lastl) halo_into_ring<WX>(G, ph, B, sh, xr, y0, slot, lastl + 2);
  }

  for (int y = y0; y < y1; ++y) {
    // moments of the row above, one iteration ahead
    float ng[9], nh[9], nflux = 0.0f, nQp = 0.0f;
    Mom nm;
    {
      const int r = map_axis(y + 1, G.ny, G.py);
      const int slot = (y + 1) & 3;
      if (act) node_into_ring<WX>(G, ph, B, sh, x, r, slot, l + 1, ng, nh, nm, nflux, nQp);
      if (l == 0) halo_into_ring<WX>(G, ph, B, sh, xl, r, slot, 0);
      if (l == lastl) halo_into_ring<WX>(G, ph, B, sh, xr, r, slot, lastl + 2);
    }
    __syncthreads();
    if (act) {
      const int k = y * G.nx + x;
      Stencil S;
      const int sm1 = (y + 3) & 3, s0 = y & 3, sp1 = (y + 1) & 3;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int slot = cy(i) == 0 ? s0 : (cy(i) > 0 ? sp1 : sm1);
        const int col = l + 1 + cx(i);
        S.phi[i] = sh.v[0][slot][col];
        S.fs[i] = sh.v[1][slot][col];
        S.rho[i] = sh.v[2][slot][col];
        S.p[i] = sh.v[3][slot][col];
      }
      float fv[9];
      pull_f(G, B, x, y, fv);
      const float phi0 = B.stat[ST_PHI0 * P + k];
      const float cth = B.stat[ST_CTH * P + k];
      const float lap0 = B.stat[ST_LAP0 * P + k];
      const float jxp = B.lin[LAG_JX * P + k];
      const float jyp = B.lin[LAG_JY * P + k];
      if (RED) {
        float sg = 0.0f, shh = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          sg += cg[i];
          shh += ch[i];
        }
        a_sg += sg;
        a_sh += shh;
        a_flux += cflux;
        a_fs += cm.fs;
        a_liq += cm.chi - cm.fs;
      }
      Post o;
      if (MODE == MODE_STEP) {
        collide_node<true>(ph, cm, S, phi0, cth, lap0, cQp, jxp, jyp, fv, cg, ch, o);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          B.dout[i * P + k] = fv[i];
          B.dout[(9 + i) * P + k] = cg[i];
          B.dout[(18 + i) * P + k] = ch[i];
        }
        B.lout[LAG_FS * P + k] = cm.fs;
        B.lout[LAG_Q * P + k] = o.Q;
        B.lout[LAG_JX * P + k] = o.jx;
        B.lout[LAG_JY * P + k] = o.jy;
        B.lout[LAG_P * P + k] = o.p;
        if (RED) {
          a_sphi += (double)cm.phi * (double)cm.mdot;
          a_heat += o.heat_src;
          a_reset += o.reset;
        }
      } else {
        collide_node<false>(ph, cm, S, phi0, cth, lap0, cQp, jxp, jyp, fv, cg, ch, o);
        float sg = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) sg += cg[i];
        float* F = B.fields;
        F[0 * P + k] = cm.phi;
        F[1 * P + k] = cm.T;
        F[2 * P + k] = 1.0f - cm.fs;
        F[3 * P + k] = cm.fs;
        F[4 * P + k] = o.ux;
        F[5 * P + k] = o.uy;
        F[6 * P + k] = o.p;
        F[7 * P + k] = cm.rhoH;
        F[8 * P + k] = o.mu;
        F[9 * P + k] = cm.C;
        F[10 * P + k] = cm.chi;
        F[11 * P + k] = cm.rho;
        F[12 * P + k] = sg;
      }
      if (RED) {
        const float um = sqrtf(o.ux * o.ux + o.uy * o.uy);
        a_umax = fmax(a_umax, (double)um);
        if (!isfinite(cm.phi) || !isfinite(cm.T) || !isfinite(um) || !isfinite(o.p)) a_bad += 1;
      }
    }
    // rotate the row registers
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      cg[i] = ng[i];
      ch[i] = nh[i];
    }
    cm = nm;
    cflux = nflux;
    cQp = nQp;
  }

  if (RED) {
    double v[NRED] = {a_sg, a_sh, a_fs, a_liq, a_umax, a_bad, a_sphi, a_heat, a_flux, a_reset, 0.0};
    // wavefront tree, then across the block's wavefronts, in fixed order
#pragma unroll
    for (int j = 0; j < NRED; ++j) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_down(v[j], off, 64);
        v[j] = (j == 4) ? fmax(v[j], o) : v[j] + o;
      }
    }
    const int wv = l >> 6;
    if ((l & 63) == 0) {
#pragma unroll
      for (int j = 0; j < NRED; ++j) sh.red[wv][j] = v[j];
    }
    __syncthreads();
    if (l < NRED) {
      double s = sh.red[0][l];
      for (int w = 1; w < WX / 64; ++w) s = (l == 4) ? fmax(s, sh.red[w][l]) : s + sh.red[w][l];
      red_out[l] = s;
    }
  }
}

// Single-lattice step kernel: grid (ceil(nx / WX), ceil(ny / CY)).
template <int WX, int MODE, bool RED>
__global__ __launch_bounds__(WX) void step_kernel(Geo G, Phys ph, Bufs B, int CY) {
  __shared__ StepShared<WX> sh;
  const int bx = blockIdx.x, by = blockIdx.y;
  double* red = RED ? B.red + (size_t)(by * gridDim.x + bx) * NRED : nullptr;
  step_strip<WX, MODE, RED>(G, ph, B, bx, by, CY, red, sh);
}

}  // namespace lbf
