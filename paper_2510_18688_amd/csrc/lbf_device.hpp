// Device-side building blocks of the coupled D2Q9 freezing step (gfx950).
//
// Layout in HBM (structure of arrays, FP32, plane stride P floats):
//   distributions  27 planes: f_0..f_8 (flow), g_0..g_8 (phase), h_0..h_8
//                  (enthalpy), stored post-collision: a step pulls
//                  X_i(x) = X_i*(x - c_i) and writes X_i*(x) of the next step
//                  at the node itself, so every store is row-coalesced and
//                  aligned and the pull loads are row-coalesced with a
//                  +-1 element shift;
//   lagged fields  9 planes: f_s, Q = rho C_p T mdot, (phi u)_x, (phi u)_y, p
//                  of the previous step, the high parts of g_0 and h_0, and
//                  the previous step's velocity u_x, u_y (written and read only
//                  when the phase-field source takes its divergence; then the
//                  (phi u)_x plane holds phi and (phi u)_y is not used);
//   static fields  4 planes: phi0, cos(theta), lap(phi0), and the temperature
//                  of the per-node isothermal region (NaN where not held).
// Both distributions and lagged fields are double-buffered (ping-pong).
// Storage is deviation-form: f^eq vanishes at the rest state (p = 0, u = 0)
// exactly; the moving g_i, h_i (i > 0) carry only O(mu) and O(rho_ref C_p T)
// values.  The rest populations g_0 ~ phi and h_0 ~ rho H hold the O(1) part
// and never move: each is an unevaluated float-float sum hi + lo (hi in a
// lagged plane, lo in the distribution plane) renormalised every step with an
// exact two-sum, so the order parameter and the enthalpy are carried to ~48
// bits while every sum and relaxation is formed from small deviations.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbf {

constexpr int NDIST = 27;
constexpr int NLAG = 9;
constexpr int NSTAT = 4;
constexpr int NFIELD = 13;
constexpr int NRED = 11;

// lagged planes: f_s, Q = rho C_p T mdot, (phi u)_x, (phi u)_y, p of the
// previous step, the high parts of the rest populations g_0, h_0, and the
// previous step's velocity.  When the phase-field source takes the flow's
// divergence (the velocity planes in use), the (phi u)_x plane holds the
// previous step's phi instead and the (phi u)_y plane is unused: (phi u) is
// their product.
enum {
  LAG_FS = 0, LAG_Q = 1, LAG_JX = 2, LAG_JY = 3, LAG_P = 4, LAG_GHI = 5, LAG_HHI = 6,
  LAG_UX = 7, LAG_UY = 8
};
// static planes: phi0, cos(theta), lap(phi0), held temperature (NaN: free)
enum { ST_PHI0 = 0, ST_CTH = 1, ST_LAP0 = 2, ST_THOLD = 3 };
// MODE_STEP_MOM: a step that also stores phi, f_s and rho of the state it
// reads (planes 0-2 of the fields buffer), for the reverse sweep's stencils
enum { MODE_STEP = 0, MODE_FIELDS = 1, MODE_STEP_MOM = 2 };

// D2Q9 (Sec. 3.1): c_0 = 0, c_1..4 axis-aligned counter-clockwise from +x,
// c_5..8 diagonal counter-clockwise from (1,1); weights 4/9, 1/9, 1/36.
__host__ __device__ constexpr int cx(int i) {
  return (i == 1 || i == 5 || i == 8) ? 1 : ((i == 3 || i == 6 || i == 7) ? -1 : 0);
}
__host__ __device__ constexpr int cy(int i) {
  return (i == 2 || i == 5 || i == 6) ? 1 : ((i == 4 || i == 7 || i == 8) ? -1 : 0);
}
__host__ __device__ constexpr int opp(int i) {
  return i == 0 ? 0 : (i <= 4 ? ((i + 1) % 4) + 1 : ((i - 3) % 4) + 5);
}
__host__ __device__ constexpr float wgt(int i) {
  return i == 0 ? 4.0f / 9.0f : (i <= 4 ? 1.0f / 9.0f : 1.0f / 36.0f);
}

// Values at the D2Q9 velocities of the moment polynomials that an MRT
// collision relaxes away from the BGK rate: energy -4 + 3c^2, energy square
// 4 - 21/2 c^2 + 9/2 c^4, energy fluxes (-5 + 3c^2) c_x, (-5 + 3c^2) c_y,
// stresses c_x^2 - c_y^2, c_x c_y.
__host__ __device__ constexpr float mrt_e(int i) { return i == 0 ? -4.0f : (i <= 4 ? -1.0f : 2.0f); }
__host__ __device__ constexpr float mrt_eps(int i) { return i == 0 ? 4.0f : (i <= 4 ? -2.0f : 1.0f); }
__host__ __device__ constexpr float mrt_qx(int i) { return i <= 4 ? -2.0f * cx(i) : (float)cx(i); }
__host__ __device__ constexpr float mrt_qy(int i) { return i <= 4 ? -2.0f * cy(i) : (float)cy(i); }
__host__ __device__ constexpr float mrt_pxx(int i) { return (float)(cx(i) * cx(i) - cy(i) * cy(i)); }
__host__ __device__ constexpr float mrt_pxy(int i) { return (float)(cx(i) * cy(i)); }

// Lattice geometry and boundary types.
struct Geo {
  int nx, ny;
  int px, py;        // periodic flags
  int tbc[4];        // per wall: 0 adiabatic, 1 Dirichlet (bottom, top, left, right)
  int tmask;         // bit w set when wall w is Dirichlet
  int P;             // plane stride in floats (every byte offset fits 32 bits)
  // Row blocks: rows rb i .. rb i + rb - 1 of every plane of a state array
  // (27 distributions, then 9 lagged planes) lie in block i, GS floats after
  // block i - 1; inside a block each plane's rows are back to back, P floats
  // after the previous plane's.  rbs = log2 rb, rmask = rb - 1; the plain
  // plane-major layout is one block (rbs 31, rmask 0x7fffffff).
  int GS;            // block stride in floats
  int rbs, rmask;
  int nblk;          // number of blocks
  int PF;            // plane stride of the read-out planes (plane-major)
};

// Index of node (x, y) in every plane of a state array, and in the static
// planes (same block structure).
__host__ __device__ __forceinline__ int nidx(const Geo& G, int x, int y) {
  return (y >> G.rbs) * G.GS + (y & G.rmask) * G.nx + x;
}

// Physical constants in the form the kernels use them.
struct Phys {
  float rho_l, rho_g, rho_s, mu_l, mu_g, mu_s, lam_l, lam_g, lam_s, cp_l, cp_g, cp_s;
  float latent, T_m, cos_psi, T_sub;
  float a3;          // 3 sigma / eps
  float kap;         // 3 eps sigma / 8
  float tau_g;       // Mbar / c_s^2 + 1/2
  float inv_tau_g;   // 1 / tau_g
  float pg;          // 1 - 1 / (2 tau_g)
  float Eref;        // rho_ref C_p,ref
  float three_over_Eref;
  float mdot_coef;   // 1 - rho_s / rho_l
  float pcm_floor;   // liquid weight below which a node holds no phase-change material
  float inv_pcm_span; // 1 / (1 - pcm_floor)
  int latch, src_tau_a;
  int subfix;        // isothermal region: 0 none, 1 nodes with phi0 >= 1/2 at
                     // T_sub, 2 the per-node plane ST_THOLD (NaN: not held)
  int mrt;           // 1: MRT flow and phase-field collisions
  int phi_src_flow;  // div u of the phase-field source: 0 mdot, 1 the
                     // divergence of the previous step's velocity
  float s_b, s_q;    // MRT bulk and energy-flux rates of f (0: 1/tau_f)
  float s_g;         // MRT rate of the moments of g above first order (0: 1/tau_g)
  float grav[3];     // body force G = rho grav
  float vsol[3];     // solid-phase velocity u_s of the drag
};

// Buffers of one lattice.  Device arrays are addressed through buffer
// resources: a lane supplies the 32-bit byte offset of its node and the
// plane offset rides in a scalar register, so no 64-bit address arithmetic
// is spent per access (and out-of-range offsets read zero instead of
// faulting).
typedef __amdgpu_buffer_rsrc_t Rsrc;

struct Bufs {
  // distributions, one resource per population block of 9 planes, so that
  // the plane offsets (scalar operands) are shared by f, g and h
  Rsrc fin, gin, hin;    // post-collision of the previous step
  Rsrc fout, gout, hout; // written by a step
  Rsrc lin;           // NLAG planes of the previous step
  Rsrc lout;          // NLAG planes, written by a step
  Rsrc stat;          // NSTAT planes
  Rsrc fields;        // NFIELD planes (read-out mode)
  const float* wallT; // 4 profiles, each `wstride` floats
  int wstride;
  double* red;        // per-block partial sums, NRED each
};

__device__ __forceinline__ Rsrc make_rsrc(const void* p, uint32_t bytes) {
  // gfx9 family: raw 32-bit data, offset addressing
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), 0, (int)bytes, 0x00020000);
}

// Plain pointers of one lattice, as the host passes them.
struct BufArgs {
  const float* din;
  float* dout;
  const float* lin;
  float* lout;
  const float* stat;
  float* fields;
  const float* wallT;
  int wstride;
  double* red;
};

// Bytes from a resource's base to the end of its array: the base holds
// `planes` planes of the last block (all earlier blocks lie before them).
__device__ __forceinline__ uint32_t block_extent(const Geo& G, int planes) {
  return (uint32_t)(((size_t)(G.nblk - 1) * G.GS + (size_t)planes * G.P) * 4u);
}

__device__ __forceinline__ Bufs make_bufs(const BufArgs& a, const Geo& G) {
  const size_t P = (size_t)G.P;
  const uint32_t e9 = block_extent(G, 9);
  Bufs B;
  B.fin = make_rsrc(a.din, e9);
  B.gin = make_rsrc(a.din + 9 * P, e9);
  B.hin = make_rsrc(a.din + 18 * P, e9);
  B.fout = make_rsrc(a.dout, e9);
  B.gout = make_rsrc(a.dout + 9 * P, e9);
  B.hout = make_rsrc(a.dout + 18 * P, e9);
  B.lin = make_rsrc(a.lin, block_extent(G, NLAG));
  B.lout = make_rsrc(a.lout, block_extent(G, NLAG));
  B.stat = make_rsrc(a.stat, block_extent(G, NSTAT));
  // read-out planes (plane-major, PF apart), or the 3 moment planes of a
  // recomputed step (state indexing, P apart)
  const size_t fe = (NFIELD * (size_t)G.PF > 3 * P ? NFIELD * (size_t)G.PF : 3 * P) * 4u;
  B.fields = make_rsrc(a.fields, a.fields ? (uint32_t)fe : 0u);
  B.wallT = a.wallT;
  B.wstride = a.wstride;
  B.red = a.red;
  return B;
}

// load plane `plane` at node index `k`
__device__ __forceinline__ float ldp(Rsrc r, int plane, int P, int k) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                       r, (uint32_t)k * 4u, (uint32_t)plane * (uint32_t)P * 4u, 0));
}
// load at an absolute element index
__device__ __forceinline__ float lda(Rsrc r, uint32_t elem) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, elem * 4u, 0, 0));
}
// Store cache policy: non-temporal (2; the new state is not re-read in this
// pass) with the SC1 scope bit (16).  Measured against non-temporal alone:
// 1.8 % faster on the 2048^2 step, 0.7 % on the 4096 x 2048 medium, the same
// on the D3Q19 passes; no policy, SC0 or SC0 + NT were 3-5 % slower.  The
// stored values and every result are the same bits under each policy.
constexpr int kStorePolicy = 16 | 2;
__device__ __forceinline__ void stp(Rsrc r, int plane, int P, int k, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (uint32_t)k * 4u,
                                        (uint32_t)plane * (uint32_t)P * 4u, kStorePolicy);
}

// Reciprocal with the hardware approximation (1 ulp), used for every per-node
// division: the FP32 path's accuracy is set by its storage, not by this.
__device__ __forceinline__ float rcp(float v) { return __builtin_amdgcn_rcpf(v); }

// High parts of the float-float rest populations are kept to 16 bits (the
// upper half of their FP32 pattern, i.e. truncated to a bfloat16 value), so
// that the high parts of g_0 and h_0 share one 32-bit plane.
__device__ __forceinline__ float hi16(float v) {
  return __builtin_bit_cast(float, __builtin_bit_cast(uint32_t, v) & 0xFFFF0000u);
}
__device__ __forceinline__ uint32_t pack_hi(float ghi, float hhi) {
  return (__builtin_bit_cast(uint32_t, ghi) >> 16) | (__builtin_bit_cast(uint32_t, hhi) & 0xFFFF0000u);
}
__device__ __forceinline__ float unpack_ghi(uint32_t p) { return __builtin_bit_cast(float, p << 16); }
__device__ __forceinline__ float unpack_hhi(uint32_t p) {
  return __builtin_bit_cast(float, p & 0xFFFF0000u);
}

// Exact two-sum: hi + d = s + err with s = fl(hi + d) (no reassociation of
// these additions is allowed, and none involves a product to contract).
__device__ __forceinline__ void two_sum(float hi, float d, float& s, float& err) {
  s = hi + d;
  const float bb = s - hi;
  err = (hi - (s - bb)) + (d - bb);
}

// Renormalise a float-float pair (reference hi, deviation d) to a 16-bit high
// part and an FP32 low part: hi' = hi16(fl(hi + d)), lo' the rest.  s - hi'
// is exact (the two agree in sign and exponent), so the pair carries the sum
// to within one rounding of lo' (|lo'| < 2^-8 |hi'|).
__device__ __forceinline__ void renorm16(float hi, float d, float& hi_out, float& lo_out) {
  float s, err;
  two_sum(hi, d, s, err);
  hi_out = hi16(s);
  lo_out = (s - hi_out) + err;
}

__device__ __forceinline__ float clampf(float v, float lo, float hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Mixing rule (Sec. 2): zeta = s zeta_s + (1 - s)[C zeta_l + (1 - C) zeta_g].
__device__ __forceinline__ float zeta(float s, float C, float zs, float zl, float zg) {
  return s * zs + (1.0f - s) * (C * zl + (1.0f - C) * zg);
}

// Node index of a stencil neighbour: periodic wrap or mirror ghost.
__device__ __forceinline__ int map_axis(int v, int n, int periodic) {
  if (v < 0) return periodic ? v + n : 0;
  if (v >= n) return periodic ? v - n : n - 1;
  return v;
}

// Source coordinate of a pull along one axis: v - c for c in {-1, 0, 1};
// periodic wrap, or -1 when the link crosses a wall.
__device__ __forceinline__ int pull_axis(int v, int c, int n, int periodic) {
  int s = v - c;
  if (s < 0) return periodic ? s + n : -1;
  if (s >= n) return periodic ? s - n : -1;
  return s;
}

// Pull sources of one node: the byte offset of x - c_i for each direction
// (the node itself when the link crosses a wall) and masks of the wall
// links.  Every population plane uses the same nine offsets; the plane
// offset is a scalar operand of the load.
struct Pull9 {
  uint32_t off[9];
  uint32_t k4;      // byte offset of the node itself
  uint32_t wmask;   // bit i: link i crosses a wall
  uint32_t ymask;   // bit i: the crossing is through a bottom/top wall
};

__device__ __forceinline__ void pull9(const Geo& G, int x, int y, Pull9& p) {
  const int sx[3] = {pull_axis(x, -1, G.nx, G.px), x, pull_axis(x, 1, G.nx, G.px)};
  const int sy[3] = {pull_axis(y, -1, G.ny, G.py), y, pull_axis(y, 1, G.ny, G.py)};
  const int k = nidx(G, x, y);
  p.k4 = (uint32_t)k * 4u;
  p.wmask = 0u;
  p.ymask = 0u;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xs = sx[cx(i) + 1], ys = sy[cy(i) + 1];
    const bool wy = ys < 0, w = wy || xs < 0;
    p.off[i] = w ? p.k4 : (uint32_t)nidx(G, xs, ys) * 4u;
    p.wmask |= (uint32_t)w << i;
    p.ymask |= (uint32_t)wy << i;
  }
}

__device__ __forceinline__ float ldo(Rsrc r, uint32_t voff, int plane, int P) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(
                                       r, voff, (uint32_t)plane * (uint32_t)P * 4u, 0));
}

// Pull the phase-field and enthalpy populations of node (x, y): bounce-back
// for g and for h on adiabatic walls, anti-bounce-back with the wall
// temperature for h on Dirichlet walls (a link through a bottom/top wall
// takes that wall even at a corner).  `flux` gains the energy that the
// Dirichlet links bring in.
__device__ __forceinline__ void pull_gh(const Geo& G, const Phys& ph, const Bufs& B, int x,
                                        int y, float* gv, float* hv, float& flux) {
  Pull9 n;
  pull9(G, x, y, n);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    gv[i] = ldo(B.gin, n.off[i], i, G.P);
    hv[i] = ldo(B.hin, n.off[i], i, G.P);
  }
  if (n.wmask) {
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      if ((n.wmask >> i) & 1u) {
        const int j = opp(i);
        gv[i] = ldo(B.gin, n.k4, j, G.P);
        const float hb = ldo(B.hin, n.k4, j, G.P);
        const int wall = ((n.ymask >> i) & 1u) ? (cy(i) > 0 ? 0 : 1) : (cx(i) > 0 ? 2 : 3);
        if ((G.tmask >> wall) & 1) {
          const float Tw = B.wallT[wall * B.wstride + (wall < 2 ? x : y)];
          hv[i] = -hb + 2.0f * wgt(i) * ph.Eref * Tw;
          flux += hv[i] - hb;
        } else {
          hv[i] = hb;
        }
      }
    }
  }
}

__device__ __forceinline__ void pull_f(const Geo& G, const Bufs& B, int x, int y, float* fv) {
  Pull9 n;
  pull9(G, x, y, n);
#pragma unroll
  for (int i = 0; i < 9; ++i) fv[i] = ldo(B.fin, n.off[i], i, G.P);
  if (n.wmask) {
#pragma unroll
    for (int i = 1; i < 9; ++i)
      if ((n.wmask >> i) & 1u) fv[i] = ldo(B.fin, n.k4, opp(i), G.P);
  }
}

// Node-local moments: liquid weight, phase-change fraction, total enthalpy,
// enthalpy map, ice fraction, mass source, order parameter and density.
// dphi = phi - ref_g and dH = rho H - ref_h keep the small parts.
struct Mom {
  float C, chi, rhoH, T, fs, fstot, mdot, divu, phi, rho, Ksol, Kliq, dphi, dH;
  float ref_g, sg, sh;   // references and stored sums (for exact global sums)
  // intermediate values and branch decisions, read only by the reverse sweep
  // (dead code in the forward kernels)
  float Craw, Cpraw, Cp, chi1, fl, fl_m, span;
  bool sol, liq;
};

// ref_g, ref_h: references of the rest populations; sg, sh: sums of the
// stored populations (rest population as its deviation); dlag: the
// divergence of the previous step's velocity at the node (used when the
// phase-field source takes div u from the flow).
__device__ __forceinline__ void moments(const Phys& ph, float ref_g, float sg, float ref_h,
                                        float sh, float fs_prev, float Q_prev, float phi0,
                                        Mom& m, float dlag = 0.0f) {
  const float phihat = ref_g + sg;
  const float Craw = 0.5f * (1.0f - phi0 + phihat);
  const float C = clampf(Craw, 0.0f, 1.0f);
  // phase-change fraction: liquid weight above the floor, latched by the
  // previous ice fraction, at most the non-solid fraction
  const float Cpraw = (C - ph.pcm_floor) * ph.inv_pcm_span;
  const float Cp = clampf(Cpraw, 0.0f, 1.0f);
  const float chi1 = ph.latch ? fmaxf(Cp, fs_prev) : Cp;
  const float chi = clampf(chi1, 0.0f, 1.0f - phi0);
  // total enthalpy with the lagged source (Sec. 3.3)
  const float dH = sh + 0.5f * Q_prev;
  const float rhoH = ref_h + dH;
  // enthalpy map (Sec. 2, Hfl) for a node with phase-change fraction chi
  const float s_sol = fminf(1.0f, phi0 + chi);
  const float Kliq = zeta(phi0, C, ph.rho_s, ph.rho_l, ph.rho_g) *
                     zeta(phi0, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float Ksol = zeta(s_sol, C, ph.rho_s, ph.rho_l, ph.rho_g) *
                     zeta(s_sol, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float Es = Ksol * ph.T_m;
  const float El = Kliq * ph.T_m + chi * ph.rho_l * ph.latent;
  // three branches (solid below E_s, liquid above E_l, mushy between; an
  // empty mushy interval counts as liquid), evaluated without divergence
  const bool sol = rhoH < Es, liq = !sol && rhoH > El;
  const float span = El - Es;
  const float fl_m = (El > Es) ? (rhoH - Es) * rcp(span) : 1.0f;
  const float fl = sol ? 0.0f : (liq ? 1.0f : fl_m);
  const float T = sol ? rhoH * rcp(Ksol) : (liq ? ph.T_m + (rhoH - El) * rcp(Kliq) : ph.T_m);
  const float fs = chi * (1.0f - fl);
  const float fstot = fminf(1.0f, phi0 + fs);
  const float mdot = ph.mdot_coef * (fs - fs_prev);   // eq1, backward difference
  m.C = C;
  m.chi = chi;
  m.rhoH = rhoH;
  m.T = T;
  m.fs = fs;
  m.fstot = fstot;
  m.mdot = mdot;
  // div u of the phase-field equation: the model's mdot, or the flow's own
  // divergence of the previous step
  const float divu = ph.phi_src_flow ? dlag : mdot;
  m.divu = divu;
  // Sec. 3.2: phi = phihat / (1 - div u / 2), formed on the deviation from
  // the reference
  const float hd = 0.5f * divu;   // exact
  m.dphi = __builtin_fmaf(hd, ref_g, sg) * rcp(1.0f - hd);
  m.phi = ref_g + m.dphi;
  m.dH = dH;
  m.ref_g = ref_g;
  m.sg = sg;
  m.sh = sh;
  m.rho = zeta(fstot, C, ph.rho_s, ph.rho_l, ph.rho_g);
  m.Ksol = Ksol;
  m.Kliq = Kliq;
  m.Craw = Craw;
  m.Cpraw = Cpraw;
  m.Cp = Cp;
  m.chi1 = chi1;
  m.fl = fl;
  m.fl_m = fl_m;
  m.span = span;
  m.sol = sol;
  m.liq = liq;
}

// Chemical potential, derivative of the free energy eq44.
__device__ __forceinline__ float chem_pot(const Phys& ph, float phi, float lap_phi, float phi0,
                                          float cth, float lap_phi0, float fs, float lap_fs) {
  const float a = ph.a3, k = ph.kap;
  float m = a * phi * (phi * phi - 1.0f) - k * lap_phi;
  m += 3.0f * a * phi0 * phi0 * phi + a * cth * phi0 * (3.0f * phi * phi + phi0 * phi0 - 1.0f) -
       k * cth * lap_phi0;
  m += 3.0f * a * fs * fs * phi + a * ph.cos_psi * fs * (3.0f * phi * phi + fs * fs - 1.0f) -
       k * ph.cos_psi * lap_fs;
  return m;
}

// Isothermal region (R21 and its per-node form): whether the node is held,
// and at which temperature.  `thold` is the node's ST_THOLD value (read only
// when subfix == 2).
__device__ __forceinline__ bool held_node(const Phys& ph, float phi0, float thold, float& Tw) {
  if (ph.subfix == 2) {
    Tw = thold;
    return !__builtin_isnan(thold);
  }
  Tw = ph.T_sub;
  return ph.subfix == 1 && phi0 >= 0.5f;
}

// Enthalpy of a node held at temperature Tw: frozen at or below T_m.
__device__ __forceinline__ float enthalpy_at(const Phys& ph, float Tw, float Ksol, float Kliq,
                                             float chi) {
  if (Tw <= ph.T_m) return Ksol * Tw;
  return Kliq * (Tw - ph.T_m) + Kliq * ph.T_m + chi * ph.rho_l * ph.latent;
}

// Stencil neighbourhood of one node: values of phi, f_s, rho and the lagged
// p at the 9 lattice points x + c_i (ghosts already mapped).
struct Stencil {
  float phi[9], fs[9], rho[9], p[9];
};

// Outputs of the per-node collision.
struct Post {
  float ux, uy, p, mu, Q, jx, jy;
  float heat_src, reset;
  float ghi;    // new high part of g_0 (gv[0] holds the low part)
  float hhi;    // new high part of h_0 (hv[0] holds the low part)
};

// Collision of the three populations at one node (Sec. 3.1-3.3), in place
// on fv, gv, hv (gv[0], hv[0] as deviations from the node's references).
// When `collide` is false only the diagnostics are filled.
// MRT: compile the MRT branches (taken when ph.mrt is set); BGK-only
// simulations run the instantiation without them.
template <bool COLLIDE, bool MRT = false>
__device__ __forceinline__ void collide_node(const Phys& ph, const Mom& m, const Stencil& S,
                                             float phi0, float cth, float lap_phi0, float Q_prev,
                                             float jx_prev, float jy_prev, float ref_h, float thold,
                                             float* fv, float* gv, float* hv, Post& o) {
  // isotropic stencils (factor 1/c_s^2 = 3 for the gradient, 2/c_s^2 = 6 for
  // the Laplacian)
  float gphx = 0, gphy = 0, lphi = 0, lfs = 0, grx = 0, gry = 0, gpx = 0, gpy = 0;
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const float w = wgt(i);
    gphx += w * cx(i) * S.phi[i];
    gphy += w * cy(i) * S.phi[i];
    lphi += w * (S.phi[i] - S.phi[0]);
    lfs += w * (S.fs[i] - S.fs[0]);
    grx += w * cx(i) * S.rho[i];
    gry += w * cy(i) * S.rho[i];
    gpx += w * cx(i) * S.p[i];
    gpy += w * cy(i) * S.p[i];
  }
  gphx *= 3.0f; gphy *= 3.0f; lphi *= 6.0f; lfs *= 6.0f;
  grx *= 3.0f; gry *= 3.0f; gpx *= 3.0f; gpy *= 3.0f;

  const float phi = m.phi, rho = m.rho, C = m.C, fstot = m.fstot, mdot = m.mdot, T = m.T;
  const float mu_v = zeta(fstot, C, ph.mu_s, ph.mu_l, ph.mu_g);
  const float lam = zeta(fstot, C, ph.lam_s, ph.lam_l, ph.lam_g);
  const float cp = zeta(fstot, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float inv_rho = rcp(rho);
  const float tau_f = 3.0f * mu_v * inv_rho + 0.5f;
  const float tau_a = lam * ph.three_over_Eref + 0.5f;
  const float inv_tau_a = rcp(tau_a);
  const float inv_tau_s = 2.0f - inv_tau_a;           // 1/tau_s + 1/tau_a = 2

  const float mu = chem_pot(ph, phi, lphi, phi0, cth, lap_phi0, m.fs, lfs);
  // total force F = F_s + G: F_s = mu grad phi, G = rho g
  const float Fx = mu * gphx + rho * ph.grav[0], Fy = mu * gphy + rho * ph.grav[1];
  float mx = 0, my = 0, sum_nz = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    mx += cx(i) * fv[i];
    my += cy(i) * fv[i];
    if (i) sum_nz += fv[i];
  }
  const float usx = (mx + 0.5f * Fx) * inv_rho, usy = (my + 0.5f * Fy) * inv_rho;
  const float fdx = fstot * (ph.vsol[0] - usx), fdy = fstot * (ph.vsol[1] - usy);  // drag
  const float ux = usx + 0.5f * fdx, uy = usy + 0.5f * fdy;
  const float Sm = rho * mdot + ux * grx + uy * gry;
  const float Ftx = Fx - gpx + (1.0f / 3.0f) * grx, Fty = Fy - gpy + (1.0f / 3.0f) * gry;
  const float uu = ux * ux + uy * uy;
  const float uFt = ux * Ftx + uy * Fty;
  const float F0 = wgt(0) * (Sm - 3.0f * uFt);
  // the rest population's non-equilibrium part (tau - 1/2) F_0: tau = tau_f,
  // or 1/s_b under MRT (the density, e and epsilon moments it projects on
  // relax at s_b)
  const bool mrt_b = MRT && ph.mrt && ph.s_b > 0.0f;
  const float tau_0 = mrt_b ? rcp(ph.s_b) : tau_f;
  const float p = (1.0f / 3.0f) / (1.0f - wgt(0)) *
                  (sum_nz + 0.5f * Sm + (tau_0 - 0.5f) * F0 - 1.5f * wgt(0) * rho * uu);
  o.ux = ux; o.uy = uy; o.p = p; o.mu = mu;
  const float jx = phi * ux, jy = phi * uy;
  o.jx = jx; o.jy = jy;
  const float rhocp = rho * cp;
  const float Q = rhocp * T * mdot;
  o.Q = Q;
  o.heat_src = 0.0f;
  o.reset = 0.0f;
  if (!COLLIDE) return;

  // flow: pressure-based equilibrium and forcing (Sec. 3.1)
  const float inv_tau_f = rcp(tau_f);
  const float pf = 1.0f - 0.5f * inv_tau_f;
  const float rfx = rho * fdx + Fx, rfy = rho * fdy + Fy;
  if (!MRT || !ph.mrt) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cu = cx(i) * ux + cy(i) * uy;
      const float cF = cx(i) * rfx + cy(i) * rfy;
      const float cFt = cx(i) * Ftx + cy(i) * Fty;
      const float feq = 3.0f * p * (wgt(i) - (i == 0 ? 1.0f : 0.0f)) +
                        rho * wgt(i) * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
      const float Fi = wgt(i) * (Sm + 3.0f * cF + 9.0f * cu * cFt - 3.0f * uFt);
      fv[i] = fv[i] - (fv[i] - feq) * inv_tau_f + pf * Fi;
    }
  } else {
    // MRT in the orthogonal basis (density, e, epsilon, j, q, p_xx, p_xy):
    // the BGK update plus, for the moments relaxing at s_b (density, e,
    // epsilon) and s_q (q_x, q_y), -(s_k - 1/tau_f) r_k / |r_k|^2 d_k with
    // d_k = sum_i r_k(c_i) (f_i - f_i^eq + F_i / 2)
    float d[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cu = cx(i) * ux + cy(i) * uy;
      const float cF = cx(i) * rfx + cy(i) * rfy;
      const float cFt = cx(i) * Ftx + cy(i) * Fty;
      const float feq = 3.0f * p * (wgt(i) - (i == 0 ? 1.0f : 0.0f)) +
                        rho * wgt(i) * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
      const float Fi = wgt(i) * (Sm + 3.0f * cF + 9.0f * cu * cFt - 3.0f * uFt);
      const float neq = fv[i] - feq + 0.5f * Fi;
      fv[i] = fv[i] - inv_tau_f * neq + Fi;
      d[0] += neq;
      d[1] += mrt_e(i) * neq;
      d[2] += mrt_eps(i) * neq;
      d[3] += mrt_qx(i) * neq;
      d[4] += mrt_qy(i) * neq;
    }
    const float db = (mrt_b ? ph.s_b : inv_tau_f) - inv_tau_f;
    const float dq = (ph.s_q > 0.0f ? ph.s_q : inv_tau_f) - inv_tau_f;
#pragma unroll
    for (int i = 0; i < 9; ++i)
      fv[i] -= db * ((1.0f / 9.0f) * d[0] + (1.0f / 36.0f) * (mrt_e(i) * d[1] + mrt_eps(i) * d[2])) +
               dq * (1.0f / 12.0f) * (mrt_qx(i) * d[3] + mrt_qy(i) * d[4]);
  }
  // phase field (Sec. 3.2)
  const float inv_tau_g = ph.inv_tau_g;
  const float pg = ph.pg;
  const float djx = jx - jx_prev, djy = jy - jy_prev;
  const float pm = phi * m.divu;
  // chemical-potential parts of g^eq; the rest term from the same rounded
  // products, so that the equilibria sum to phi (as for the enthalpy below)
  const float mu1 = wgt(1) * mu, mu5 = wgt(5) * mu;
  const float mrest = 4.0f * mu1 + 4.0f * mu5;
  if (!(MRT && ph.mrt && ph.s_g > 0.0f)) {
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cj = cx(i) * jx + cy(i) * jy;
      // rest population: equilibrium relative to the node's reference
      const float geq = (i == 0 ? m.dphi - mrest : (i <= 4 ? mu1 : mu5)) + 3.0f * wgt(i) * cj;
      const float Gi = wgt(i) * (3.0f * (cx(i) * djx + cy(i) * djy) + pm);
      gv[i] = gv[i] - (gv[i] - geq) * inv_tau_g + pg * Gi;
    }
  } else {
    // MRT: the BGK update plus -(s_g - 1/tau_g) r_k / |r_k|^2 d_k over the
    // moments above first order (e, epsilon, q_x, q_y, p_xx, p_xy), with
    // d_k = sum_i r_k(c_i) (g_i - g_i^eq + G_i / 2)
    float d[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cj = cx(i) * jx + cy(i) * jy;
      const float geq = (i == 0 ? m.dphi - mrest : (i <= 4 ? mu1 : mu5)) + 3.0f * wgt(i) * cj;
      const float Gi = wgt(i) * (3.0f * (cx(i) * djx + cy(i) * djy) + pm);
      const float neq = gv[i] - geq + 0.5f * Gi;
      gv[i] = gv[i] - inv_tau_g * neq + Gi;
      d[0] += mrt_e(i) * neq;
      d[1] += mrt_eps(i) * neq;
      d[2] += mrt_qx(i) * neq;
      d[3] += mrt_qy(i) * neq;
      d[4] += mrt_pxx(i) * neq;
      d[5] += mrt_pxy(i) * neq;
    }
    const float dg = ph.s_g - inv_tau_g;
#pragma unroll
    for (int i = 0; i < 9; ++i)
      gv[i] -= dg * ((1.0f / 36.0f) * (mrt_e(i) * d[0] + mrt_eps(i) * d[1]) +
                     (1.0f / 12.0f) * (mrt_qx(i) * d[2] + mrt_qy(i) * d[3]) +
                     0.25f * (mrt_pxx(i) * d[4] + mrt_pxy(i) * d[5]));
  }
  // renormalise g_0 = hi + lo (16-bit hi, FP32 lo)
  renorm16(m.ref_g, gv[0], o.ghi, gv[0]);
  // enthalpy, TRT (Sec. 3.3, eq22)
  const float ET = ph.Eref * T;
  const float cT = rhocp * T;
  // The equilibria must sum to rho H.  In FP32, (1 - w_0) rho_ref C_p,ref T
  // and the eight rounded products w_i rho_ref C_p,ref T differ by a bias of
  // about 2e-8 of the product (1 - w_0 rounds low against the weights' sum),
  // which every collision would add to the node's energy; the rest term is
  // therefore formed from the same rounded products as the moving ones.
  const float E1 = wgt(1) * ET, E5 = wgt(5) * ET;
  const float Erest = 4.0f * E1 + 4.0f * E5;   // each 4x product exact
  float heq[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float cu = cx(i) * ux + cy(i) * uy;
    // rest population relative to the node's reference: rhoH - ref_h = dH
    heq[i] = (i == 0) ? m.dH - Erest - 1.5f * wgt(0) * cT * uu
                      : (i <= 4 ? E1 : E5) + wgt(i) * cT * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
  }
  const float ps = ph.src_tau_a ? (1.0f - 0.5f * inv_tau_a) : (1.0f - 0.5f * inv_tau_s);
  float hn[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int j = opp(i);
    const float ha = 0.5f * (hv[i] - hv[j]), hs = 0.5f * (hv[i] + hv[j]);
    const float ea = 0.5f * (heq[i] - heq[j]), es = 0.5f * (heq[i] + heq[j]);
    hn[i] = hv[i] - (ha - ea) * inv_tau_a - (hs - es) * inv_tau_s + ps * wgt(i) * Q;
  }
  o.heat_src = 0.5f * Q_prev * inv_tau_s + ps * Q;
  float Tw;
  if (held_node(ph, phi0, thold, Tw)) {
    // isothermal region: reset to the equilibrium at the held temperature
    // (rest population relative to its reference)
    const float rH = enthalpy_at(ph, Tw, m.Ksol, m.Kliq, m.chi);
    const float EW = ph.Eref * Tw;
    const float W1 = wgt(1) * EW, W5 = wgt(5) * EW;
    float before = 0.0f, after = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      before += hn[i];
      const float e = (i == 0) ? (rH - ref_h) - (4.0f * W1 + 4.0f * W5) : (i <= 4 ? W1 : W5);
      after += e;
      hn[i] = e;
    }
    o.reset = after - before;
  }
#pragma unroll
  for (int i = 1; i < 9; ++i) hv[i] = hn[i];
  // renormalise h_0 = hi + lo (16-bit hi, FP32 lo)
  renorm16(ref_h, hn[0], o.hhi, hv[0]);
}

}  // namespace lbf
