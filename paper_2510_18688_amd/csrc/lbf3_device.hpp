// Device-side building blocks of the three-dimensional (D3Q19) coupled step.
//
// Layout in HBM (structure of arrays, FP32).  Rows of nx nodes are numbered
// z ny + y; the state arrays (f, g, h, lagged, static) group them in blocks
// of rb rows holding every plane of the array, each plane's rows back to
// back (plane stride P floats inside a block, block stride GS, a power of
// two), so node (x, y, z) has storage index (row >> log2 rb) GS +
// (row mod rb) nx + x in all of them; rb = ny nz (one block) is plane-major.
// The moments records and the read-out planes are indexed by the linear node
// id (z ny + y) nx + x, plane stride PL.
//   distributions 57 planes: f_0..f_18, g_0..g_18, h_0..h_18, post-collision,
//                 stored at the node that wrote them (pull scheme); the rest
//                 populations g_0, h_0 hold the low parts of float-float
//                 values whose high parts are lagged planes;
//   lagged       11 planes: f_s, Q = rho C_p T mdot, (phi u)_x, _y, _z, p of
//                 the previous step, high parts of g_0 and h_0, and the
//                 previous step's velocity (read and written only when the
//                 phase-field source takes its divergence);
//   static        3 planes: phi0, cos(theta), lap(phi0);
//   moments       per node a 16-byte record (phi, f_s, rho, lagged p) and one
//                 plane of div u, written by the moments pass.
// The node-local moments, the chemical potential and the mixing rule are the
// dimension-free functions of the two-dimensional step (lbf_device.hpp).
#pragma once
#include "lbf_device.hpp"

namespace lbf3 {

using lbf::Mom;
using lbf::Phys;
using lbf::Rsrc;

constexpr int NQ = 19;
constexpr int NDIST = 3 * NQ;
constexpr int NLAG = 11;
constexpr int NSTAT = 3;
constexpr int NFIELD = 14;
enum { LAG_FS = 0, LAG_Q, LAG_JX, LAG_JY, LAG_JZ, LAG_P, LAG_GHI, LAG_HHI, LAG_UX, LAG_UY, LAG_UZ };
// plane of div u behind the records in the moments buffer (in units of P floats)
constexpr int MOM_DIVU = 4;
enum { ST_PHI0 = 0, ST_CTH = 1, ST_LAP0 = 2 };

// D3Q19 (Sec. 3.1): rest, six axis directions, twelve face diagonals, in the
// printed order; weights 1/3, 1/18, 1/36.
__host__ __device__ constexpr int cx(int i) {
  return (i == 1 || i == 7 || i == 9 || i == 11 || i == 13) ? 1
         : (i == 2 || i == 8 || i == 10 || i == 12 || i == 14) ? -1 : 0;
}
__host__ __device__ constexpr int cy(int i) {
  return (i == 3 || i == 7 || i == 10 || i == 15 || i == 17) ? 1
         : (i == 4 || i == 8 || i == 9 || i == 16 || i == 18) ? -1 : 0;
}
__host__ __device__ constexpr int cz(int i) {
  return (i == 5 || i == 11 || i == 14 || i == 15 || i == 18) ? 1
         : (i == 6 || i == 12 || i == 13 || i == 16 || i == 17) ? -1 : 0;
}
__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }
__host__ __device__ constexpr float wgt(int i) {
  return i == 0 ? 1.0f / 3.0f : (i <= 6 ? 1.0f / 18.0f : 1.0f / 36.0f);
}

struct Geo3 {
  int n[3];          // nx, ny, nz
  int per[3];        // periodic flags
  int tmask;         // bit f: face f is Dirichlet (0 x-low .. 5 z-high)
  int strip;         // rows per strip of the step pass's node order (>= ny: x-fastest)
  int P;             // plane stride inside a block (floats)
  int rbs, rmask;    // log2 and rb - 1 of the rows per block (31, 0x7fffffff: one block)
  int gss;           // log2 of the block stride GS (31: one block)
  int nblk;          // blocks
  int RBN;           // nodes per block (rb nx)
  int AS;            // floats from one state array to the next (f, g, h)
  int PL;            // plane stride of the linear arrays (records, read-out)
  float Tw[6];       // face temperatures
};

// Storage index of node (x, y, z) in the state and static arrays.
__host__ __device__ __forceinline__ uint32_t sidx3(const Geo3& G, int x, int y, int z) {
  const int row = z * G.n[1] + y;
  return ((uint32_t)(row >> G.rbs) << G.gss) + (uint32_t)(row & G.rmask) * G.n[0] + x;
}

// Linear node id of a storage index.
__host__ __device__ __forceinline__ uint32_t lin_of(const Geo3& G, uint32_t s) {
  return (s >> G.gss) * (uint32_t)G.RBN + (s & ((1u << G.gss) - 1u));
}

struct Bufs3 {
  Rsrc fin, gin, hin, fout, gout, hout, lin, lout, stat, mom;
};

struct BufArgs3 {
  const float* din;
  float* dout;
  const float* lin;
  float* lout;
  const float* stat;
  float* mom;        // per node a 16-byte record (phi, f_s, rho of the state read,
                     // p of the step before), then a plane of div u (MOM_DIVU),
                     // written by the moments pass
};

// Bytes from a state array's base to its end when its last block holds
// `planes` planes.
__device__ __forceinline__ uint32_t extent3(const Geo3& G, int planes) {
  return (uint32_t)((((size_t)(G.nblk - 1) << G.gss) + (size_t)planes * G.P) * 4u);
}

__device__ __forceinline__ Bufs3 make_bufs3(const BufArgs3& a, const Geo3& G) {
  const size_t AS = (size_t)G.AS;
  const uint32_t e = extent3(G, NQ);
  Bufs3 B;
  B.fin = lbf::make_rsrc(a.din, e);
  B.gin = lbf::make_rsrc(a.din + AS, e);
  B.hin = lbf::make_rsrc(a.din + 2 * AS, e);
  B.fout = lbf::make_rsrc(a.dout, a.dout ? e : 0u);
  B.gout = lbf::make_rsrc(a.dout ? a.dout + AS : nullptr, a.dout ? e : 0u);
  B.hout = lbf::make_rsrc(a.dout ? a.dout + 2 * AS : nullptr, a.dout ? e : 0u);
  B.lin = lbf::make_rsrc(a.lin, extent3(G, NLAG));
  B.lout = lbf::make_rsrc(a.lout, a.lout ? extent3(G, NLAG) : 0u);
  B.stat = lbf::make_rsrc(a.stat, extent3(G, NSTAT));
  B.mom = lbf::make_rsrc(a.mom, 5u * (uint32_t)G.PL * 4u);
  return B;
}

// Pull sources of one node: byte offset of x - c_i (the node itself across a
// wall), the wall mask, and the node's coordinates (a wall link's face is
// recomputed from them: a link leaving through several walls takes the z
// face, else the y face, else the x face).
struct Pull19 {
  uint32_t off[NQ];
  uint32_t k4;
  uint32_t wmask;
  int x, y, z;
};

// Face of the wall that link i of node (x, y, z) crosses (low face when
// c > 0: the source x - c lies below the lattice).
__device__ __forceinline__ int wall_face(const Geo3& G, int x, int y, int z, int i) {
  const int sz = z - cz(i), sy = y - cy(i);
  if (!G.per[2] && (sz < 0 || sz >= G.n[2])) return cz(i) > 0 ? 4 : 5;
  if (!G.per[1] && (sy < 0 || sy >= G.n[1])) return cy(i) > 0 ? 2 : 3;
  return cx(i) > 0 ? 0 : 1;
}

__device__ __forceinline__ int src_axis(int v, int c, int n, int periodic, bool& out) {
  int s = v - c;
  out = false;
  if (s < 0) {
    if (periodic) return s + n;
    out = true;
    return v;
  }
  if (s >= n) {
    if (periodic) return s - n;
    out = true;
    return v;
  }
  return s;
}

__device__ __forceinline__ void pull19(const Geo3& G, int x, int y, int z, Pull19& p) {
  const uint32_t k = sidx3(G, x, y, z);
  p.k4 = k * 4u;
  p.wmask = 0u;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    bool ox, oy, oz;
    const int sx = src_axis(x, cx(i), G.n[0], G.per[0], ox);
    const int sy = src_axis(y, cy(i), G.n[1], G.per[1], oy);
    const int sz = src_axis(z, cz(i), G.n[2], G.per[2], oz);
    const bool w = ox || oy || oz;
    p.off[i] = w ? p.k4 : sidx3(G, sx, sy, sz) * 4u;
    p.wmask |= (uint32_t)w << i;
  }
  p.x = x;
  p.y = y;
  p.z = z;
}

// Pulled g of a node (bounce-back at every wall).
__device__ __forceinline__ void pull_g3(const Geo3& G, const Bufs3& B, const Pull19& n,
                                        float* gv) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) gv[i] = lbf::ldo(B.gin, n.off[i], i, G.P);
  if (n.wmask) {
#pragma unroll
    for (int i = 1; i < NQ; ++i)
      if ((n.wmask >> i) & 1u) gv[i] = lbf::ldo(B.gin, n.k4, opp(i), G.P);
  }
}

// Pulled h of a node (bounce-back; anti-bounce-back with the face
// temperature on Dirichlet faces).
__device__ __forceinline__ void pull_h3(const Geo3& G, const Phys& ph, const Bufs3& B,
                                        const Pull19& n, float* hv) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) hv[i] = lbf::ldo(B.hin, n.off[i], i, G.P);
  if (n.wmask) {
#pragma unroll
    for (int i = 1; i < NQ; ++i) {
      if ((n.wmask >> i) & 1u) {
        const float hb = lbf::ldo(B.hin, n.k4, opp(i), G.P);
        const int f = wall_face(G, n.x, n.y, n.z, i);
        hv[i] = ((G.tmask >> f) & 1) ? -hb + 2.0f * wgt(i) * ph.Eref * G.Tw[f] : hb;
      }
    }
  }
}

__device__ __forceinline__ void pull_gh3(const Geo3& G, const Phys& ph, const Bufs3& B,
                                         const Pull19& n, float* gv, float* hv) {
  pull_g3(G, B, n, gv);
  pull_h3(G, ph, B, n, hv);
}

__device__ __forceinline__ void pull_f3(const Geo3& G, const Bufs3& B, const Pull19& n,
                                        float* fv) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) fv[i] = lbf::ldo(B.fin, n.off[i], i, G.P);
  if (n.wmask) {
#pragma unroll
    for (int i = 1; i < NQ; ++i)
      if ((n.wmask >> i) & 1u) fv[i] = lbf::ldo(B.fin, n.k4, opp(i), G.P);
  }
}

// Node moments from the pulled g, h and the lagged fields; dlag is the
// divergence of the previous step's velocity (used with the flow-divergence
// phase-field source).
__device__ __forceinline__ void node_moments3(const Geo3& G, const Phys& ph, const Bufs3& B,
                                              uint32_t k, const float* gv, const float* hv,
                                              float phi0, Mom& m, float dlag = 0.0f) {
  float sg = gv[0], sh = hv[0];
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    sg += gv[i];
    sh += hv[i];
  }
  const float ghi = lbf::ldp(B.lin, LAG_GHI, G.P, (int)k);
  const float hhi = lbf::ldp(B.lin, LAG_HHI, G.P, (int)k);
  const float fsp = lbf::ldp(B.lin, LAG_FS, G.P, (int)k);
  const float Qp = lbf::ldp(B.lin, LAG_Q, G.P, (int)k);
  lbf::moments(ph, ghi, sg, hhi, sh, fsp, Qp, phi0, m, dlag);
}



// Neighbour index for the stencils: wrap, or the mirror ghost at a wall.
__device__ __forceinline__ int nb3(int v, int n, int periodic) {
  if (v < 0) return periodic ? v + n : 0;
  if (v >= n) return periodic ? v - n : n - 1;
  return v;
}

// Isotropic divergence 3 sum_i w_i c_i . u(x + c_i) of the previous step's
// velocity at one node, over the same neighbours as the stencils (the pull
// offsets, the mirror ghost for a link that crosses a wall).  Fixed grouping
// and no contraction: axis neighbours (weight 1/18), then face diagonals
// (1/36).
__device__ __forceinline__ float div3(const Geo3& G, const Bufs3& B, const Pull19& n) {
#pragma clang fp contract(off)
  float ax = 0.0f, dg = 0.0f;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    uint32_t o = n.off[opp(i)];
    if ((n.wmask >> opp(i)) & 1u) {
      const int xx = nb3(n.x + cx(i), G.n[0], G.per[0]);
      const int yy = nb3(n.y + cy(i), G.n[1], G.per[1]);
      const int zz = nb3(n.z + cz(i), G.n[2], G.per[2]);
      o = sidx3(G, xx, yy, zz) * 4u;
    }
    float c = 0.0f;
    if (cx(i)) c = c + (float)cx(i) * lbf::ldo(B.lin, o, LAG_UX, G.P);
    if (cy(i)) c = c + (float)cy(i) * lbf::ldo(B.lin, o, LAG_UY, G.P);
    if (cz(i)) c = c + (float)cz(i) * lbf::ldo(B.lin, o, LAG_UZ, G.P);
    if (i <= 6) ax = ax + c;
    else dg = dg + c;
  }
  return 3.0f * ((1.0f / 18.0f) * ax + (1.0f / 36.0f) * dg);
}

// The moments pass's record of a node: phi, f_s, rho and the lagged p.
struct MomRec {
  float v[4];
};

// Four dword accesses at consecutive offsets, which the compiler merges into
// one 16-byte access.
__device__ __forceinline__ MomRec ld_rec(Rsrc r, uint32_t off) {
  MomRec m;
#pragma unroll
  for (int c = 0; c < 4; ++c)
    m.v[c] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off + 4u * c, 0u, 0));
  return m;
}

__device__ __forceinline__ void st_rec(Rsrc r, uint32_t off, float a, float b, float c, float d) {
  const float v[4] = {a, b, c, d};
#pragma unroll
  for (int j = 0; j < 4; ++j)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v[j]), r, off + 4u * j, 0u, 0);
}

// Stencil sums of one node: gradients of phi, rho, p_prev; Laplacians of phi
// and f_s (isotropic D3Q19 stencils: factor 3 for the gradient, 6 for the
// Laplacian).
struct Stencil3 {
  float gph[3], gr[3], gp[3], lphi, lfs;
};

// The neighbour x + c_i is the pull source of direction opp(i), so the
// pull's offsets serve the stencil; only where that link crosses a wall does
// the stencil need its own (mirror-ghost) neighbour.
__device__ __forceinline__ void stencils3(const Geo3& G, const Bufs3& B, const Pull19& n,
                                          float phic, float fsc, Stencil3& S) {
  float gph[3] = {0, 0, 0}, gr[3] = {0, 0, 0}, gp[3] = {0, 0, 0}, lphi = 0, lfs = 0;
#pragma unroll
  for (int i = 1; i < NQ; ++i) {
    // linear id of the neighbour (the records are linear)
    uint32_t kn = lin_of(G, n.off[opp(i)] >> 2);
    if ((n.wmask >> opp(i)) & 1u) {
      const int xx = nb3(n.x + cx(i), G.n[0], G.per[0]);
      const int yy = nb3(n.y + cy(i), G.n[1], G.per[1]);
      const int zz = nb3(n.z + cz(i), G.n[2], G.per[2]);
      kn = ((uint32_t)zz * G.n[1] + yy) * G.n[0] + xx;
    }
    // one 16-byte record per neighbour: phi, f_s, rho, p_prev
    const MomRec r = ld_rec(B.mom, kn * 16u);
    const float vphi = r.v[0], vfs = r.v[1], vrho = r.v[2], vp = r.v[3];
    const float w = wgt(i);
    const float c[3] = {(float)cx(i), (float)cy(i), (float)cz(i)};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      gph[a] += w * c[a] * vphi;
      gr[a] += w * c[a] * vrho;
      gp[a] += w * c[a] * vp;
    }
    lphi += w * (vphi - phic);
    lfs += w * (vfs - fsc);
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    S.gph[a] = 3.0f * gph[a];
    S.gr[a] = 3.0f * gr[a];
    S.gp[a] = 3.0f * gp[a];
  }
  S.lphi = 6.0f * lphi;
  S.lfs = 6.0f * lfs;
}

struct Post3 {
  float u[3], p, Q, j[3], ghi, hhi;
};

// Node quantities of one collision that do not depend on the population
// index: velocity, pressure, forces and relaxation rates.
struct Coll3 {
  float u[3], rf[3], Ft[3], j[3], dj[3];
  float Sm, uu, uFt, p, rho, ift, pf, mu, pm, Q, ET, cT, inv_tau_a, inv_tau_s, ps;
};

// Velocity and pressure from the pulled f (Sec. 3.1: the forced velocity
// with the solid drag, the pressure from the non-rest populations), the
// chemical potential, and the rates of the three collisions.
__device__ __forceinline__ void collide3_prepare(const Phys& ph, const Mom& m, const Stencil3& S,
                                                 float phi0, float cth, float lap_phi0,
                                                 const float* jprev, const float* fv, Coll3& c) {
  const float phi = m.phi, rho = m.rho, C = m.C, fstot = m.fstot, mdot = m.mdot, T = m.T;
  const float mu_v = lbf::zeta(fstot, C, ph.mu_s, ph.mu_l, ph.mu_g);
  const float lam = lbf::zeta(fstot, C, ph.lam_s, ph.lam_l, ph.lam_g);
  const float cp = lbf::zeta(fstot, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float inv_rho = lbf::rcp(rho);
  const float tau_f = 3.0f * mu_v * inv_rho + 0.5f;
  c.inv_tau_a = lbf::rcp(lam * ph.three_over_Eref + 0.5f);
  c.inv_tau_s = 2.0f - c.inv_tau_a;
  c.mu = lbf::chem_pot(ph, phi, S.lphi, phi0, cth, lap_phi0, m.fs, S.lfs);
  float F[3], mm[3] = {0, 0, 0}, snz = 0;
#pragma unroll
  for (int a = 0; a < 3; ++a) F[a] = c.mu * S.gph[a] + rho * ph.grav[a];   // F_s + G
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    mm[0] += cx(i) * fv[i];
    mm[1] += cy(i) * fv[i];
    mm[2] += cz(i) * fv[i];
    if (i) snz += fv[i];
  }
  float fd[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float us = (mm[a] + 0.5f * F[a]) * inv_rho;
    fd[a] = fstot * (ph.vsol[a] - us);
    c.u[a] = us + 0.5f * fd[a];
    c.Ft[a] = F[a] - S.gp[a] + (1.0f / 3.0f) * S.gr[a];
    c.rf[a] = rho * fd[a] + F[a];
  }
  c.Sm = rho * mdot + c.u[0] * S.gr[0] + c.u[1] * S.gr[1] + c.u[2] * S.gr[2];
  c.uu = c.u[0] * c.u[0] + c.u[1] * c.u[1] + c.u[2] * c.u[2];
  c.uFt = c.u[0] * c.Ft[0] + c.u[1] * c.Ft[1] + c.u[2] * c.Ft[2];
  const float w0 = wgt(0);
  const float F0 = w0 * (c.Sm - 3.0f * c.uFt);
  c.p = (1.0f / 3.0f) / (1.0f - w0) *
        (snz + 0.5f * c.Sm + (tau_f - 0.5f) * F0 - 1.5f * w0 * rho * c.uu);
  c.rho = rho;
  c.ift = lbf::rcp(tau_f);
  c.pf = 1.0f - 0.5f * c.ift;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    c.j[a] = phi * c.u[a];
    c.dj[a] = c.j[a] - jprev[a];
  }
  c.pm = phi * m.divu;
  const float rhocp = rho * cp;
  c.Q = rhocp * T * mdot;
  c.ET = ph.Eref * T;
  c.cT = rhocp * T;
  c.ps = ph.src_tau_a ? (1.0f - 0.5f * c.inv_tau_a) : (1.0f - 0.5f * c.inv_tau_s);
}

// Flow collision (Sec. 3.1), in place.
__device__ __forceinline__ void collide3_f(const Coll3& c, float* fv) {
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const float cu = cx(i) * c.u[0] + cy(i) * c.u[1] + cz(i) * c.u[2];
    const float cF = cx(i) * c.rf[0] + cy(i) * c.rf[1] + cz(i) * c.rf[2];
    const float cFt = cx(i) * c.Ft[0] + cy(i) * c.Ft[1] + cz(i) * c.Ft[2];
    const float feq = 3.0f * c.p * (wgt(i) - (i == 0 ? 1.0f : 0.0f)) +
                      c.rho * wgt(i) * (3.0f * cu + 4.5f * cu * cu - 1.5f * c.uu);
    const float Fi = wgt(i) * (c.Sm + 3.0f * cF + 9.0f * cu * cFt - 3.0f * c.uFt);
    fv[i] = fv[i] - (fv[i] - feq) * c.ift + c.pf * Fi;
  }
}

// Phase-field collision (Sec. 3.2), in place; g_0 leaves as float-float
// (ghi, gv[0]).
__device__ __forceinline__ void collide3_g(const Phys& ph, const Mom& m, const Coll3& c,
                                           float* gv, float& ghi) {
  const float mu1 = wgt(1) * c.mu, mu7 = wgt(7) * c.mu;
  const float mrest = 6.0f * mu1 + 12.0f * mu7;
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const float cj = cx(i) * c.j[0] + cy(i) * c.j[1] + cz(i) * c.j[2];
    const float geq = (i == 0 ? m.dphi - mrest : (i <= 6 ? mu1 : mu7)) + 3.0f * wgt(i) * cj;
    const float Gi =
        wgt(i) * (3.0f * (cx(i) * c.dj[0] + cy(i) * c.dj[1] + cz(i) * c.dj[2]) + c.pm);
    gv[i] = gv[i] - (gv[i] - geq) * ph.inv_tau_g + ph.pg * Gi;
  }
  lbf::two_sum(m.ref_g, gv[0], ghi, gv[0]);
}

// Enthalpy collision, TRT (Sec. 3.3, eq22), in place, or the held
// substrate's equilibrium at T_substrate; h_0 leaves as float-float.
__device__ __forceinline__ void collide3_h(const Phys& ph, const Mom& m, const Coll3& c,
                                           float phi0, float ref_h, float* hv, float& hhi) {
  const float w0 = wgt(0);
  // rest term from the same rounded products as the moving ones, so that
  // the equilibria sum to rho H in FP32 without a systematic bias (the 2D
  // collision gives the reason)
  const float E1 = wgt(1) * c.ET, E7 = wgt(7) * c.ET;
  const float Erest = 6.0f * E1 + 12.0f * E7;
  float heq[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const float cu = cx(i) * c.u[0] + cy(i) * c.u[1] + cz(i) * c.u[2];
    heq[i] = (i == 0) ? m.dH - Erest - 1.5f * w0 * c.cT * c.uu
                      : (i <= 6 ? E1 : E7) +
                            wgt(i) * c.cT * (3.0f * cu + 4.5f * cu * cu - 1.5f * c.uu);
  }
  float hn[NQ];
#pragma unroll
  for (int i = 0; i < NQ; ++i) {
    const int jj = opp(i);
    const float ha = 0.5f * (hv[i] - hv[jj]), hs = 0.5f * (hv[i] + hv[jj]);
    const float ea = 0.5f * (heq[i] - heq[jj]), es = 0.5f * (heq[i] + heq[jj]);
    hn[i] = hv[i] - (ha - ea) * c.inv_tau_a - (hs - es) * c.inv_tau_s + c.ps * wgt(i) * c.Q;
  }
  if (ph.subfix && phi0 >= 0.5f) {
    const float Tw = ph.T_sub;
    const float rH = lbf::enthalpy_at(ph, Tw, m.Ksol, m.Kliq, m.chi);
    const float W1 = wgt(1) * ph.Eref * Tw, W7 = wgt(7) * ph.Eref * Tw;
#pragma unroll
    for (int i = 0; i < NQ; ++i)
      hn[i] = (i == 0) ? (rH - ref_h) - (6.0f * W1 + 12.0f * W7) : (i <= 6 ? W1 : W7);
  }
#pragma unroll
  for (int i = 1; i < NQ; ++i) hv[i] = hn[i];
  lbf::two_sum(ref_h, hn[0], hhi, hv[0]);
}

// The whole collision of one node, in place on fv, gv, hv (gv[0], hv[0] as
// deviations from the node's references).
__device__ __forceinline__ void collide3(const Phys& ph, const Mom& m, const Stencil3& S,
                                         float phi0, float cth, float lap_phi0,
                                         const float* jprev, float ref_h, float* fv, float* gv,
                                         float* hv, Post3& o) {
  Coll3 c;
  collide3_prepare(ph, m, S, phi0, cth, lap_phi0, jprev, fv, c);
  collide3_f(c, fv);
  collide3_g(ph, m, c, gv, o.ghi);
  collide3_h(ph, m, c, phi0, ref_h, hv, o.hhi);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    o.u[a] = c.u[a];
    o.j[a] = c.j[a];
  }
  o.p = c.p;
  o.Q = c.Q;
}

}  // namespace lbf3
