// Fused coupled step: one kernel pass per time step.
//
// A block of WX lanes owns a strip of WX columns and marches up CY rows.
// Each lane keeps the pulled g and h of its current row in registers.  For
// the 9-point stencils of phi, f_s, rho (and the lagged p) the block keeps a
// ring of four rows of those values in LDS, WX + 2 wide; the row above the
// current one is computed (pull + moments) one iteration ahead, so the
// moments of every node are computed once per block, plus one halo row at
// each end of the strip.  The two halo columns of all CY + 2 rows are
// computed up front by the whole block (one node per lane) and copied into
// the ring row by row, so no lane diverges per row.  One barrier per row.
#pragma once
#include "lbf_device.hpp"

namespace lbf {

constexpr int CY_MAX = 256;

template <int WX>
struct StepShared {
  float v[4][4][WX + 2];        // [phi, fs, rho, p_prev][ring slot][column]
  float halo[4][2][CY_MAX + 2]; // [field][left, right][row - (y0 - 1)]
  double red[WX / 64][NRED];
};

// Moments of node (xx, yy): pulled g and h, liquid weight, enthalpy map,
// mass source, order parameter and density; the four stencil inputs are
// returned in st[].
__device__ __forceinline__ void node_moments(const Geo& G, const Phys& ph, const Bufs& B, int xx,
                                             int yy, float* gv, float* hv, Mom& m, float& flux,
                                             float& Qp, float& ref_h, float* st) {
  pull_gh(G, ph, B, xx, yy, gv, hv, flux);
  // sums of the small stored values first (rest populations are deviations)
  float sg = gv[0], shh = hv[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    sg += gv[i];
    shh += hv[i];
  }
  const int k = yy * G.nx + xx;
  const float fsp = ldp(B.lin, LAG_FS, G.P, k);
  Qp = ldp(B.lin, LAG_Q, G.P, k);
  const float phi0 = ldp(B.stat, ST_PHI0, G.P, k);
  const float ref_g = ldp(B.lin, LAG_GHI, G.P, k);
  ref_h = ldp(B.lin, LAG_HHI, G.P, k);
  moments(ph, ref_g, sg, ref_h, shh, fsp, Qp, phi0, m);
  st[0] = m.phi;
  st[1] = m.fs;
  st[2] = m.rho;
  st[3] = ldp(B.lin, LAG_P, G.P, k);
}

// One strip (bx, by) of the lattice.  MODE_STEP writes the next state;
// MODE_FIELDS writes the read-out fields of the current state.  With RED,
// per-block FP64 partial sums go to `red_out` (NRED doubles).
template <int WX, int MODE, bool RED, bool RECOMP>
__device__ __forceinline__ void step_strip(const Geo& G, const Phys& ph, const Bufs& B, int bx,
                                           int by, int CY, double* red_out, StepShared<WX>& sh) {
  const int l = threadIdx.x;
  const int x0 = bx * WX;
  const int x = x0 + l;
  const bool act = x < G.nx;
  const int lastl = min(WX, G.nx - x0) - 1;
  const int y0 = by * CY;
  const int y1 = min(y0 + CY, G.ny);
  const int P = G.P;

  double a_sg = 0, a_sh = 0, a_fs = 0, a_liq = 0, a_umax = 0, a_bad = 0;
  double a_sphi = 0, a_heat = 0, a_flux = 0, a_reset = 0;

  // halo columns x0 - 1 and x0 + lastl + 1 for rows y0 - 1 .. y1, one node per lane
  {
    const int xl = map_axis(x0 - 1, G.nx, G.px);
    const int xr = map_axis(x0 + lastl + 1, G.nx, G.px);
    const int nh = 2 * (y1 - y0 + 2);
    for (int t = l; t < nh; t += WX) {
      const int side = t & 1, r = t >> 1;
      float gv[9], hv[9], fl = 0.0f, q, rh, st[4];
      Mom m;
      node_moments(G, ph, B, side ? xr : xl, map_axis(y0 - 1 + r, G.ny, G.py), gv, hv, m, fl,
                   q, rh, st);
#pragma unroll
      for (int f = 0; f < 4; ++f) sh.halo[f][side][r] = st[f];
    }
  }

  float cg[9], ch[9], cflux = 0.0f, cQp = 0.0f, crh = 0.0f;
  Mom cm;
  // own columns of rows y0 - 1 (halo row) and y0
  if (act) {
    float gv[9], hv[9], fl = 0.0f, q, rh, st[4];
    Mom m;
    node_moments(G, ph, B, x, map_axis(y0 - 1, G.ny, G.py), gv, hv, m, fl, q, rh, st);
#pragma unroll
    for (int f = 0; f < 4; ++f) sh.v[f][(y0 + 3) & 3][l + 1] = st[f];
    node_moments(G, ph, B, x, y0, cg, ch, cm, cflux, cQp, crh, st);
#pragma unroll
    for (int f = 0; f < 4; ++f) sh.v[f][y0 & 3][l + 1] = st[f];
  }
  __syncthreads();
  // lane 0 places the left halo column, the last active lane the right one
  // (both, for a one-column strip)
  if (l == 0) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      sh.v[f][(y0 + 3) & 3][0] = sh.halo[f][0][0];
      sh.v[f][y0 & 3][0] = sh.halo[f][0][1];
    }
  }
  if (l == lastl) {
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      sh.v[f][(y0 + 3) & 3][lastl + 2] = sh.halo[f][1][0];
      sh.v[f][y0 & 3][lastl + 2] = sh.halo[f][1][1];
    }
  }

  for (int y = y0; y < y1; ++y) {
    // moments of the row above, one iteration ahead (with RECOMP only its
    // stencil inputs are kept; the row's own moments are recomputed when it
    // collides, trading L2 re-reads for registers)
    float ng[9], nh[9], nflux = 0.0f, nQp = 0.0f, nrh = 0.0f;
    Mom nm;
    const int slot_n = (y + 1) & 3;
    if (act) {
      float st[4];
      node_moments(G, ph, B, x, map_axis(y + 1, G.ny, G.py), ng, nh, nm, nflux, nQp, nrh, st);
#pragma unroll
      for (int f = 0; f < 4; ++f) sh.v[f][slot_n][l + 1] = st[f];
    }
    if (RECOMP && act && y > y0) {
      float st[4];
      cflux = 0.0f;
      node_moments(G, ph, B, x, y, cg, ch, cm, cflux, cQp, crh, st);
    }
    if (l == 0 || l == lastl) {
      const int r = y + 1 - (y0 - 1);
#pragma unroll
      for (int f = 0; f < 4; ++f) {
        if (l == 0) sh.v[f][slot_n][0] = sh.halo[f][0][r];
        if (l == lastl) sh.v[f][slot_n][lastl + 2] = sh.halo[f][1][r];
      }
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
      const float phi0 = ldp(B.stat, ST_PHI0, P, k);
      const float cth = ldp(B.stat, ST_CTH, P, k);
      const float lap0 = ldp(B.stat, ST_LAP0, P, k);
      const float jxp = ldp(B.lin, LAG_JX, P, k);
      const float jyp = ldp(B.lin, LAG_JY, P, k);
      if (RED) {
        // node totals: reference plus the small stored sums
        a_sg += (double)cm.ref_g + (double)cm.sg;
        a_sh += (double)crh + (double)cm.sh;
        a_flux += cflux;
        a_fs += cm.fs;
        a_liq += cm.chi - cm.fs;
      }
      Post o;
      if (MODE == MODE_STEP) {
        collide_node<true>(ph, cm, S, phi0, cth, lap0, cQp, jxp, jyp, crh, fv, cg, ch, o);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          stp(B.dout, i, P, k, fv[i]);
          stp(B.dout, 9 + i, P, k, cg[i]);
          stp(B.dout, 18 + i, P, k, ch[i]);
        }
        stp(B.lout, LAG_FS, P, k, cm.fs);
        stp(B.lout, LAG_Q, P, k, o.Q);
        stp(B.lout, LAG_JX, P, k, o.jx);
        stp(B.lout, LAG_JY, P, k, o.jy);
        stp(B.lout, LAG_P, P, k, o.p);
        stp(B.lout, LAG_GHI, P, k, o.ghi);
        stp(B.lout, LAG_HHI, P, k, o.hhi);
        if (RED) {
          a_sphi += (double)cm.phi * (double)cm.mdot;
          a_heat += o.heat_src;
          a_reset += o.reset;
        }
      } else {
        collide_node<false>(ph, cm, S, phi0, cth, lap0, cQp, jxp, jyp, crh, fv, cg, ch, o);
        const float sg = cm.ref_g + cm.sg;
        stp(B.fields, 0, P, k, cm.phi);
        stp(B.fields, 1, P, k, cm.T);
        stp(B.fields, 2, P, k, 1.0f - cm.fs);
        stp(B.fields, 3, P, k, cm.fs);
        stp(B.fields, 4, P, k, o.ux);
        stp(B.fields, 5, P, k, o.uy);
        stp(B.fields, 6, P, k, o.p);
        stp(B.fields, 7, P, k, cm.rhoH);
        stp(B.fields, 8, P, k, o.mu);
        stp(B.fields, 9, P, k, cm.C);
        stp(B.fields, 10, P, k, cm.chi);
        stp(B.fields, 11, P, k, cm.rho);
        stp(B.fields, 12, P, k, sg);
      }
      if (RED) {
        const float um = sqrtf(o.ux * o.ux + o.uy * o.uy);
        a_umax = fmax(a_umax, (double)um);
        if (!isfinite(cm.phi) || !isfinite(cm.T) || !isfinite(um) || !isfinite(o.p)) a_bad += 1;
      }
    }
    if (!RECOMP) {
      // rotate the row registers
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        cg[i] = ng[i];
        ch[i] = nh[i];
      }
      cm = nm;
      cflux = nflux;
      cQp = nQp;
      crh = nrh;
    }
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

#ifndef LBF_RECOMP
#define LBF_RECOMP 0
#endif
// Minimum waves per SIMD the register allocator is asked to keep.
#ifndef LBF_WAVES
#define LBF_WAVES 2
#endif

// Single-lattice step kernel: grid (ceil(nx / WX), ceil(ny / CY)).
template <int WX, int MODE, bool RED>
__global__ __launch_bounds__(WX) __attribute__((amdgpu_waves_per_eu(LBF_WAVES, 8))) void
step_kernel(Geo G, Phys ph, BufArgs A, int CY) {
  __shared__ StepShared<WX> sh;
  const Bufs B = make_bufs(A, G.P);
  const int bx = blockIdx.x, by = blockIdx.y;
  double* red = RED ? A.red + (size_t)(by * gridDim.x + bx) * NRED : nullptr;
  step_strip<WX, MODE, RED, LBF_RECOMP != 0>(G, ph, B, bx, by, CY, red, sh);
}

}  // namespace lbf
