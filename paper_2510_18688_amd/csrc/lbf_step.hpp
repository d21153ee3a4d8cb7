// Fused coupled step: one kernel pass per time step.
//
// A block of WX lanes owns a strip of WX columns and marches up CY rows.
// Each lane keeps the pulled g and h of its current row in registers.  For
// the 9-point stencils of phi, f_s, rho, the lagged p and the static phi0
// (its Laplacian is formed here rather than stored) the block keeps a ring
// of four rows of those values in LDS, WX + 2 wide; the row above the
// current one is computed (pull + moments) one iteration ahead, so the
// moments of every node are computed once per block, plus one halo row at
// each end of the strip.  The two halo columns of all CY + 2 rows are
// computed up front by the whole block (one node per lane) and copied into
// the ring row by row, so no lane diverges per row.  One barrier per row.
// When the phase-field source takes the divergence of the previous step's
// velocity, that velocity sits in a second four-row ring, filled two rows
// ahead of the moments that read it, so each node's velocity is loaded
// once per block instead of once per stencil neighbour.
#pragma once
#include "lbf_device.hpp"

namespace lbf {

constexpr int CY_MAX = 256;
// strips of at least this many rows take the previous step's velocity from
// the LDS ring, shorter ones gather it (the same values, the same bits)
constexpr int kRingRows = 4;
// values per node in the stencil ring: phi, f_s, rho, p of the previous step
// and the static phi0 (whose Laplacian is taken from the ring, not stored)
constexpr int NSV = 5;

template <int WX>
struct StepShared {
  float v[NSV][4][WX + 2];        // [phi, fs, rho, p_prev, phi0][ring slot][column]
  float halo[NSV][2][CY_MAX + 2]; // [field][left, right][row - (y0 - 1)]
  float u[2][4][WX + 2];          // previous step's velocity [x, y][ring slot][column]
  double red[WX / 64][NRED];
};



// Everything a node's moments read from memory.
struct NodeIn {
  float g[9], h[9];
  float flux, fsp, Qp, phi0, ghi, hhi, pprev;
  float dlag;   // divergence of the previous step's velocity at the node
                // (phase-field source from the flow's divergence)
  float uxc, uyc;   // the previous step's velocity at the node itself (same source)
};

// Isotropic divergence 3 sum_i w_i c_i . u(x + c_i) from the velocity
// components at the eight neighbours (ux[i], uy[i] at x + c_i; the entries
// off the component's axis are not read).  Every product is rounded on its
// own and the grouping is fixed: a node's moments are formed in several
// inlined places (strip rows, halo rows and columns, the batched kernel),
// and a contraction chosen differently in one of them would make the state
// depend on the launch shape.
__device__ __forceinline__ float div9(const float* ux, const float* uy) {
#pragma clang fp contract(off)
  // axis neighbours (weight 1/9), then diagonals (1/36)
  const float ax = (ux[1] - ux[3]) + (uy[2] - uy[4]);
  const float dg = ((ux[5] + uy[5]) + (uy[6] - ux[6])) - ((ux[7] + uy[7]) + (uy[8] - ux[8]));
  return 3.0f * ((1.0f / 9.0f) * ax + (1.0f / 36.0f) * dg);
}

// With the phase-field source from the flow's divergence and `gather_u`,
// also gather the previous step's velocity at the eight neighbours (periodic
// wrap or the mirror ghost, as for every stencil) and form its divergence;
// without `gather_u` the caller supplies in.dlag (from the velocity ring).
__device__ __forceinline__ void node_load(const Geo& G, const Phys& ph, const Bufs& B, int xx,
                                          int yy, NodeIn& in, bool gather_u = true) {
  in.flux = 0.0f;
  pull_gh(G, ph, B, xx, yy, in.g, in.h, in.flux);
  const int k = nidx(G, xx, yy);
  in.fsp = ldp(B.lin, LAG_FS, G.P, k);
  in.Qp = ldp(B.lin, LAG_Q, G.P, k);
  in.phi0 = ldp(B.stat, ST_PHI0, G.P, k);
  {
    // both high parts in one plane
    const uint32_t hp = __builtin_bit_cast(uint32_t, ldp(B.lin, LAG_GHI, G.P, k));
    in.ghi = unpack_ghi(hp);
    in.hhi = unpack_hhi(hp);
  }
  in.pprev = ldp(B.lin, LAG_P, G.P, k);
  in.dlag = 0.0f;
  if (ph.phi_src_flow && gather_u) {
    in.uxc = ldp(B.lin, LAG_UX, G.P, k);
    in.uyc = ldp(B.lin, LAG_UY, G.P, k);
    float ux[9], uy[9];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const int kk = nidx(G, map_axis(xx + cx(i), G.nx, G.px), map_axis(yy + cy(i), G.ny, G.py));
      ux[i] = cx(i) ? ldp(B.lin, LAG_UX, G.P, kk) : 0.0f;
      uy[i] = cy(i) ? ldp(B.lin, LAG_UY, G.P, kk) : 0.0f;
    }
    in.dlag = div9(ux, uy);
  }
}

// Divergence of the previous step's velocity at column l of ring row `row`
// (rows row - 1, row, row + 1 of the velocity ring; the same neighbours and
// arithmetic as the gather in node_load, so both give the same bits).
template <int WX>
__device__ __forceinline__ float ring_div(const StepShared<WX>& sh, int l, int row) {
  float ux[9], uy[9];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const int slot = (row + cy(i)) & 3, col = l + 1 + cx(i);
    ux[i] = cx(i) ? sh.u[0][slot][col] : 0.0f;
    uy[i] = cy(i) ? sh.u[1][slot][col] : 0.0f;
  }
  return div9(ux, uy);
}

// Previous step's velocity of one ring row: a lane's own node, and for the
// first and last active lanes the halo column beyond them (x wrapped or
// mirrored like every stencil neighbour).
struct URow {
  float x, y;      // at the lane's node
  float lx, ly;    // left halo column (lane 0)
  float rx, ry;    // right halo column (last active lane)
};

__device__ __forceinline__ void urow_load(const Geo& G, const Bufs& B, int x, int xl, int xr,
                                          int yy, bool left, bool right, URow& u) {
  const int row = nidx(G, 0, yy);
  u.x = ldp(B.lin, LAG_UX, G.P, row + x);
  u.y = ldp(B.lin, LAG_UY, G.P, row + x);
  if (left) {
    u.lx = ldp(B.lin, LAG_UX, G.P, row + xl);
    u.ly = ldp(B.lin, LAG_UY, G.P, row + xl);
  }
  if (right) {
    u.rx = ldp(B.lin, LAG_UX, G.P, row + xr);
    u.ry = ldp(B.lin, LAG_UY, G.P, row + xr);
  }
}

template <int WX>
__device__ __forceinline__ void urow_store(StepShared<WX>& sh, int l, int lastl, int row,
                                           const URow& u) {
  const int s = row & 3;
  sh.u[0][s][l + 1] = u.x;
  sh.u[1][s][l + 1] = u.y;
  if (l == 0) {
    sh.u[0][s][0] = u.lx;
    sh.u[1][s][0] = u.ly;
  }
  if (l == lastl) {
    sh.u[0][s][lastl + 2] = u.rx;
    sh.u[1][s][lastl + 2] = u.ry;
  }
}

// Moments of a loaded node: liquid weight, enthalpy map, mass source, order
// parameter and density; the four stencil inputs are returned in st[].
__device__ __forceinline__ void node_finish(const Phys& ph, const NodeIn& in, Mom& m, float* st) {
  // sums of the small stored values first (rest populations are deviations)
  float sg = in.g[0], shh = in.h[0];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    sg += in.g[i];
    shh += in.h[i];
  }
  moments(ph, in.ghi, sg, in.hhi, shh, in.fsp, in.Qp, in.phi0, m, in.dlag);
  st[0] = m.phi;
  st[1] = m.fs;
  st[2] = m.rho;
  st[3] = in.pprev;
}

// Flow populations and node data the collision reads.  With the phase-field
// source from the flow's divergence the previous step's (phi u) is not
// stored: the previous step's phi is (in the plane of (phi u)_x) and the
// velocity is anyway, and their product is the stored (phi u) bit for bit.
struct FlowIn {
  float f[9];
  float cth, lap0, jxp, jyp, thold;   // jxp: phi of the previous step in that case
};

// LAP0 = false leaves lap0 to the caller (the step kernel takes it from its
// stencil ring).
template <bool LAP0 = true>
__device__ __forceinline__ void flow_load(const Geo& G, const Phys& ph, const Bufs& B, int x,
                                          int y, FlowIn& in) {
  pull_f(G, B, x, y, in.f);
  const int k = nidx(G, x, y);
  in.cth = ldp(B.stat, ST_CTH, G.P, k);
  in.lap0 = LAP0 ? ldp(B.stat, ST_LAP0, G.P, k) : 0.0f;
  in.jxp = ldp(B.lin, LAG_JX, G.P, k);
  in.jyp = ph.phi_src_flow ? 0.0f : ldp(B.lin, LAG_JY, G.P, k);
  // the per-node held temperature is read only when that region is in use
  in.thold = ph.subfix == 2 ? ldp(B.stat, ST_THOLD, G.P, k) : 0.0f;
}

// One strip (bx, by) of the lattice.  MODE_STEP writes the next state;
// MODE_FIELDS writes the read-out fields of the current state.  With RED,
// per-block FP64 partial sums go to `red_out` (NRED doubles).
template <int WX, int MODE, bool RED, bool MRT = false>
__device__ __forceinline__ void step_strip(const Geo& G, const Phys& ph, const Bufs& B, int bx,
                                           int by, int CY, int dir, double* red_out,
                                           StepShared<WX>& sh) {
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
  // (the prologue's loads, up to the first rows', at the raised priority of
  // a load phase: see the main loop)
  __builtin_amdgcn_s_setprio(1);
  {
    const int xl = map_axis(x0 - 1, G.nx, G.px);
    const int xr = map_axis(x0 + lastl + 1, G.nx, G.px);
    const int nh = 2 * (y1 - y0 + 2);
    for (int t = l; t < nh; t += WX) {
      const int side = t & 1, r = t >> 1;
      NodeIn in;
      Mom m;
      float st[NSV];
      node_load(G, ph, B, side ? xr : xl, map_axis(y0 - 1 + r, G.ny, G.py), in);
      node_finish(ph, in, m, st);
      st[4] = in.phi0;
#pragma unroll
      for (int f = 0; f < NSV; ++f) sh.halo[f][side][r] = st[f];
    }
  }

  // March from ys in direction dir (+1 up, -1 down).  Software pipeline:
  // the populations of the row two ahead and the flow populations of the
  // next row are requested one iteration before they are used.
  const int ys = dir > 0 ? y0 : y1 - 1;
  const int nrow = y1 - y0;
  NodeIn cin, ain;   // current row; row ahead (in flight)
  FlowIn fin;        // flow data of the current row (in flight)
  FlowIn fnx;        // flow data of the next row, in flight
  Mom cm;
  // velocity ring (divergence source only): rows ys .. ys + 2 dir now, the
  // row after them in flight; the moments of rows ys - dir and ys gather
  // their neighbours' velocity themselves, and so does a ghost row beyond a
  // y wall (its moments are the mirrored row's, whose divergence is taken
  // around that row, not around the ghost row's place in the ring)
  // (a strip of a few rows gathers every row: the ring's fill and its
  // barrier-ordered stores would cost more than they save)
  const bool uring = ph.phi_src_flow != 0 && nrow >= kRingRows;
  auto ring_row = [&](int r) { return uring && (G.py || (r >= 0 && r < G.ny)); };
  const int xl = map_axis(x0 - 1, G.nx, G.px);
  const int xr = map_axis(x0 + lastl + 1, G.nx, G.px);
  URow un;
  if (act && uring) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      URow u0;
      urow_load(G, B, x, xl, xr, map_axis(ys + r * dir, G.ny, G.py), l == 0, l == lastl, u0);
      urow_store(sh, l, lastl, ys + r * dir, u0);
    }
    if (nrow > 1)
      urow_load(G, B, x, xl, xr, map_axis(ys + 3 * dir, G.ny, G.py), l == 0, l == lastl, un);
  }
  if (act) {
    NodeIn bin;
    Mom m;
    float st[NSV];
    node_load(G, ph, B, x, map_axis(ys - dir, G.ny, G.py), bin);
    node_load(G, ph, B, x, ys, cin);
    node_load(G, ph, B, x, map_axis(ys + dir, G.ny, G.py), ain, !ring_row(ys + dir));
    flow_load<false>(G, ph, B, x, ys, fin);
    __builtin_amdgcn_s_setprio(0);
    node_finish(ph, bin, m, st);
    st[4] = bin.phi0;
#pragma unroll
    for (int f = 0; f < NSV; ++f) sh.v[f][(ys - dir) & 3][l + 1] = st[f];
    node_finish(ph, cin, cm, st);
    st[4] = cin.phi0;
#pragma unroll
    for (int f = 0; f < NSV; ++f) sh.v[f][ys & 3][l + 1] = st[f];
  }
  __syncthreads();
  // lane 0 places the left halo column, the last active lane the right one
  // (both, for a one-column strip)
  if (l == 0) {
#pragma unroll
    for (int f = 0; f < NSV; ++f) {
      sh.v[f][(ys - dir) & 3][0] = sh.halo[f][0][ys - dir - (y0 - 1)];
      sh.v[f][ys & 3][0] = sh.halo[f][0][ys - (y0 - 1)];
    }
  }
  if (l == lastl) {
#pragma unroll
    for (int f = 0; f < NSV; ++f) {
      sh.v[f][(ys - dir) & 3][lastl + 2] = sh.halo[f][1][ys - dir - (y0 - 1)];
      sh.v[f][ys & 3][lastl + 2] = sh.halo[f][1][ys - (y0 - 1)];
    }
  }

  for (int it = 0; it < nrow; ++it) {
    const int y = ys + it * dir;
    const int ya = y + dir;
    const int slot_n = ya & 3;
    const bool more = it + 1 < nrow;
    // moments of the row ahead from the data requested last iteration, then
    // the request for the row after it
    Mom am;
    NodeIn next_c;
    if (act) {
      float st[NSV];
      if (uring) {
        // rows y, ya, ya + dir of the velocity ring were filled before the
        // last barrier; the row after them (slot of y - dir, no longer read)
        // is stored now and the next one requested
        if (ring_row(ya)) {
          ain.dlag = ring_div(sh, l, ya);
          ain.uxc = sh.u[0][ya & 3][l + 1];
          ain.uyc = sh.u[1][ya & 3][l + 1];
        }
        if (more) {
          urow_store(sh, l, lastl, y + 3 * dir, un);
          if (it + 2 < nrow) {
            __builtin_amdgcn_s_setprio(1);   // a load phase (see below)
            urow_load(G, B, x, xl, xr, map_axis(y + 4 * dir, G.ny, G.py), l == 0, l == lastl, un);
            __builtin_amdgcn_s_setprio(0);
          }
        }
      }
      node_finish(ph, ain, am, st);
      st[4] = ain.phi0;
#pragma unroll
      for (int f = 0; f < NSV; ++f) sh.v[f][slot_n][l + 1] = st[f];
      next_c = ain;
      if (more) {
        // the next rows' loads go out at a raised wave priority, so that a
        // wave about to issue them is scheduled before waves in their
        // collision (with the velocity ring's and the prologue's loads
        // raised too: 2048^2 step 0.2372 -> 0.2317 ms, 4096 x 2048 medium
        // 0.5332 -> 0.5224 ms; the same bits)
        __builtin_amdgcn_s_setprio(1);
        node_load(G, ph, B, x, map_axis(ya + dir, G.ny, G.py), ain, !ring_row(ya + dir));
        flow_load<false>(G, ph, B, x, ya, fnx);   // before this row's collision
        __builtin_amdgcn_s_setprio(0);
      }
    }
    if (l == 0 || l == lastl) {
      const int r = ya - (y0 - 1);
#pragma unroll
      for (int f = 0; f < NSV; ++f) {
        if (l == 0) sh.v[f][slot_n][0] = sh.halo[f][0][r];
        if (l == lastl) sh.v[f][slot_n][lastl + 2] = sh.halo[f][1][r];
      }
    }
    __syncthreads();
    if (act) {
      const int k = nidx(G, x, y);
      Stencil S;
      const int sm1 = (y - 1) & 3, s0 = y & 3, sp1 = (y + 1) & 3;
#pragma unroll
      for (int i = 0; i < 9; ++i) {
        const int slot = cy(i) == 0 ? s0 : (cy(i) > 0 ? sp1 : sm1);
        const int col = l + 1 + cx(i);
        S.phi[i] = sh.v[0][slot][col];
        S.fs[i] = sh.v[1][slot][col];
        S.rho[i] = sh.v[2][slot][col];
        S.p[i] = sh.v[3][slot][col];
      }
      // static Laplacian of phi0 on the same ring (mirror ghosts at walls)
      float lap = 0.0f;
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const int slot = cy(i) == 0 ? s0 : (cy(i) > 0 ? sp1 : sm1);
        lap += wgt(i) * (sh.v[4][slot][l + 1 + cx(i)] - cin.phi0);
      }
      const float lap0 = 6.0f * lap;
      float* fv = fin.f;
      float* cg = cin.g;
      float* ch = cin.h;
      const float phi0 = cin.phi0, cQp = cin.Qp, crh = cin.hhi;
      // lagged (phi u): stored, or the product of the previous step's phi and u
      const float jxp = ph.phi_src_flow ? fin.jxp * cin.uxc : fin.jxp;
      const float jyp = ph.phi_src_flow ? fin.jxp * cin.uyc : fin.jyp;
      if (RED) {
        a_sg += (double)cm.ref_g + (double)cm.sg;
        a_sh += (double)crh + (double)cm.sh;
        a_flux += cin.flux;
        a_fs += cm.fs;
        a_liq += cm.chi - cm.fs;
      }
      Post o;
      if (MODE != MODE_FIELDS) {
        collide_node<true, MRT>(ph, cm, S, phi0, fin.cth, lap0, cQp, jxp, jyp, crh,
                                fin.thold, fv, cg, ch, o);
#pragma unroll
        for (int i = 0; i < 9; ++i) {
          stp(B.fout, i, P, k, fv[i]);
          stp(B.gout, i, P, k, cg[i]);
          stp(B.hout, i, P, k, ch[i]);
        }
        stp(B.lout, LAG_FS, P, k, cm.fs);
        stp(B.lout, LAG_Q, P, k, o.Q);
        if (ph.phi_src_flow) {
          stp(B.lout, LAG_JX, P, k, cm.phi);
        } else {
          stp(B.lout, LAG_JX, P, k, o.jx);
          stp(B.lout, LAG_JY, P, k, o.jy);
        }
        stp(B.lout, LAG_P, P, k, o.p);
        stp(B.lout, LAG_GHI, P, k, __builtin_bit_cast(float, pack_hi(o.ghi, o.hhi)));
        if (ph.phi_src_flow) {
          stp(B.lout, LAG_UX, P, k, o.ux);
          stp(B.lout, LAG_UY, P, k, o.uy);
        }
        if (MODE == MODE_STEP_MOM) {
          stp(B.fields, 0, P, k, cm.phi);
          stp(B.fields, 1, P, k, cm.fs);
          stp(B.fields, 2, P, k, cm.rho);
        }
        if (RED) {
          a_sphi += (double)cm.phi * (double)cm.divu;
          a_heat += o.heat_src;
          a_reset += o.reset;
        }
      } else {
        collide_node<false, MRT>(ph, cm, S, phi0, fin.cth, lap0, cQp, jxp, jyp, crh,
                                 fin.thold, fv, cg, ch, o);
        // read-out planes are plane-major whatever the state's layout
        const int kf = y * G.nx + x, PF = G.PF;
        stp(B.fields, 0, PF, kf, cm.phi);
        stp(B.fields, 1, PF, kf, cm.T);
        stp(B.fields, 2, PF, kf, 1.0f - cm.fs);
        stp(B.fields, 3, PF, kf, cm.fs);
        stp(B.fields, 4, PF, kf, o.ux);
        stp(B.fields, 5, PF, kf, o.uy);
        stp(B.fields, 6, PF, kf, o.p);
        stp(B.fields, 7, PF, kf, cm.rhoH);
        stp(B.fields, 8, PF, kf, o.mu);
        stp(B.fields, 9, PF, kf, cm.C);
        stp(B.fields, 10, PF, kf, cm.chi);
        stp(B.fields, 11, PF, kf, cm.rho);
        stp(B.fields, 12, PF, kf, cm.ref_g + cm.sg);
      }
      if (RED) {
        const float um = sqrtf(o.ux * o.ux + o.uy * o.uy);
        a_umax = fmax(a_umax, (double)um);
        if (!isfinite(cm.phi) || !isfinite(cm.T) || !isfinite(um) || !isfinite(o.p)) a_bad += 1;
      }
      // request the next row's flow data; rotate the row registers
      if (more) fin = fnx;
      cin = next_c;
      cm = am;
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

// Minimum waves per SIMD the register allocator is asked to keep.
constexpr int kWaves = 2;

// Tile of a workgroup: workgroups are dealt to the 8 XCDs round-robin, so
// workgroup w runs on XCD w % 8; tiles are handed out so that each XCD
// owns a contiguous band of ntiles / 8 tiles (row-major: strips side by side,
// then up the lattice), keeping the columns and rows that neighbouring
// strips share inside one L2.
__device__ __forceinline__ int xcd_tile(int w, int ntiles) {
  const int xcd = w & 7, local = w >> 3;
  return xcd * (ntiles >> 3) + min(xcd, ntiles & 7) + local;
}

// Single-lattice step kernel: 1D grid of nbx * nby workgroups.  Strips in
// even tile rows march up, odd ones down, so two strips that share halo rows
// reach them at the same time.
template <int WX, int MODE, bool RED, bool MRT = false>
__global__ __launch_bounds__(WX) __attribute__((amdgpu_waves_per_eu(kWaves, 8))) void
step_kernel(Geo G, Phys ph, BufArgs A, int CY, int nbx, int ntiles) {
  __shared__ StepShared<WX> sh;
  const Bufs B = make_bufs(A, G);
  const int t = xcd_tile(blockIdx.x, ntiles);
  const int bx = t % nbx, by = t / nbx;
  double* red = RED ? A.red + (size_t)t * NRED : nullptr;
  step_strip<WX, MODE, RED, MRT>(G, ph, B, bx, by, CY, (by & 1) ? -1 : 1, red, sh);
}

}  // namespace lbf

namespace lbf {

// One lattice of a batch: geometry, constants, and its buffers for both
// ping-pong parities (A[p] steps the state that parity p reads).
struct InstDesc {
  Geo G;
  Phys ph;
  BufArgs A[2];
  int CY, nbx;
};

// Persistent batched step: a fixed grid walks the work list of (instance,
// tile) items of every lattice of the batch.  In round r workgroup b takes
// item r * gridDim.x + xcd_tile(b, gridDim.x), so each XCD receives a
// contiguous run of items (neighbouring tiles of one lattice) per round.
template <int WX, bool MRT = false>
__global__ __launch_bounds__(WX) __attribute__((amdgpu_waves_per_eu(kWaves, 8))) void
batch_step_kernel(const InstDesc* __restrict__ D, const int2* __restrict__ items, int nitems,
                  int parity) {
  __shared__ StepShared<WX> sh;
  const int G = gridDim.x;
  const int slot = xcd_tile(blockIdx.x, G);
  for (int base = 0; base < nitems; base += G) {
    const int w = base + slot;
    if (w >= nitems) break;
    const int2 item = items[w];
    const Geo geo = D[item.x].G;
    const Phys ph = D[item.x].ph;
    const BufArgs args = D[item.x].A[parity];
    const int CY = D[item.x].CY, nbx = D[item.x].nbx;
    const Bufs B = make_bufs(args, geo);
    const int bx = item.y % nbx, by = item.y / nbx;
    __syncthreads();   // the LDS ring of the previous item is free
    step_strip<WX, MODE_STEP, false, MRT>(geo, ph, B, bx, by, CY, (by & 1) ? -1 : 1, nullptr,
                                          sh);
  }
}

}  // namespace lbf
