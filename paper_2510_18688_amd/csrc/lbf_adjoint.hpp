// Reverse-mode (adjoint) sweep of the coupled step.
//
// Forward map of step n: the state S^n = (D^n, L^n) holds the post-collision
// distributions D (27 planes, stored at the node that wrote them) and the
// lagged fields L = (f_s, Q, (phi u)_x, (phi u)_y, p) of the previous step.
// Step n pulls D^n (bounce-back, anti-bounce-back with the wall temperature),
// forms the node moments, the stencils of phi, f_s, rho and the lagged p,
// and collides into S^{n+1}.
//
// The adjoint of a step runs in two kernels:
//   k_adj_collide (one node per lane): gathers the adjoint of D^{n+1} at the
//     node through the transpose of step n+1's pull (a node's slot j was
//     read by node x + c_j, or by the node itself in direction opp(j) when the
//     link crosses a wall; anti-bounce-back flips the sign and adds the
//     wall-temperature derivative), recomputes the node's forward step and
//     runs the collision backwards to: the adjoints of the pulled
//     populations through the collision, of the eight stencil values, of the
//     lagged (phi u), and the d J / d cos(theta) contribution.  The moments are
//     reversed locally too, giving the node's local part of d J / d (sum g),
//     d J / d (sum h), d J / d f_s^prev and their Jacobian with respect to
//     the (not yet known) stencil contributions to phi, f_s and rho.
//   k_adj_gather (one node per lane): applies the transposed stencils (with
//     the same wrap / mirror-ghost neighbour map as the forward) to the
//     stencil adjoints and completes the moment reverse with the Jacobian.
// The adjoint of the pulled population j of a node is then its direct part
// plus d J / d (sum g) (g block) or d J / d (sum h) (h block), which the next
// k_adj_collide (of step n - 1) reads when it gathers through the pull.
//
// Non-smooth points take one-sided derivatives, with the conventions of the
// FP64 gradient oracle: a clamp passes the derivative on its closed interval,
// a maximum splits it evenly at a tie, the enthalpy-map branch and the
// mushy-zone test are those of the forward evaluation.
#pragma once
#include "lbf_step.hpp"

namespace lbf {

// adjoints of the node-local moment quantities
constexpr int NLOC = 11;
enum {
  AL_PHI = 0, AL_RHO, AL_FS, AL_C, AL_FSTOT, AL_MDOT, AL_T, AL_RHOH, AL_CHI, AL_KSOL, AL_KLIQ
};
// adjoints of the stencil values of a node
constexpr int NST = 8;
enum { AS_GPHX = 0, AS_GPHY, AS_LPHI, AS_LFS, AS_GRX, AS_GRY, AS_GPX, AS_GPY };
// adjoint of a time level's distributions: 27 direct parts, then
// d J / d (sum g) and d J / d (sum h) of the pulling node
constexpr int NADJ_D = 29;
enum { AD_SG = 27, AD_SH = 28 };
// adjoint of the lagged fields, planes in the LAG_FS .. LAG_P order
constexpr int NADJ_L = 5;
// moment-reverse Jacobian: local part of (sum g, sum h, f_s^prev) adjoints,
// then their derivatives with respect to the phi, f_s and rho adjoints
constexpr int NJAC = 12;

__device__ __forceinline__ float dzeta_ds(float C, float zs, float zl, float zg) {
  return zs - (C * zl + (1.0f - C) * zg);
}
__device__ __forceinline__ float dzeta_dC(float s, float zl, float zg) {
  return (1.0f - s) * (zl - zg);
}

// Reverse of moments(): adjoints of the moment quantities (loc) to the
// adjoints of sum g, sum h (also the lagged Q, at half weight) and f_s^prev.
// Linear in loc.
__device__ __forceinline__ void moments_reverse(const Phys& ph, const Mom& m, float phi0,
                                                float fs_prev, const float* loc, float& a_sg,
                                                float& a_sh, float& a_fsp) {
  float a_phi = loc[AL_PHI], a_rho = loc[AL_RHO], a_fs = loc[AL_FS], a_C = loc[AL_C];
  float a_fstot = loc[AL_FSTOT], a_mdot = loc[AL_MDOT], a_T = loc[AL_T];
  float a_rhoH = loc[AL_RHOH], a_chi = loc[AL_CHI], a_Ksol = loc[AL_KSOL];
  float a_Kliq = loc[AL_KLIQ];
  const float C = m.C;
  // rho = zeta(fstot, C)
  a_fstot += a_rho * dzeta_ds(C, ph.rho_s, ph.rho_l, ph.rho_g);
  a_C += a_rho * dzeta_dC(m.fstot, ph.rho_l, ph.rho_g);
  // phi = phihat / (1 - mdot / 2)
  const float iden = rcp(1.0f - 0.5f * m.mdot);
  float a_phihat = a_phi * iden;
  a_mdot += 0.5f * m.phi * iden * a_phi;
  // mdot = (1 - rho_s / rho_l)(fs - fs_prev)
  a_fs += ph.mdot_coef * a_mdot;
  a_fsp = -ph.mdot_coef * a_mdot;
  // fstot = min(1, phi0 + fs)
  if (phi0 + m.fs <= 1.0f) a_fs += a_fstot;
  // fs = chi (1 - fl)
  a_chi += (1.0f - m.fl) * a_fs;
  const float a_fl = -m.chi * a_fs;
  // enthalpy map on the branch the forward took
  float a_Es = 0.0f, a_El = 0.0f;
  if (m.sol) {
    const float iK = rcp(m.Ksol);
    a_rhoH += a_T * iK;
    a_Ksol -= m.T * iK * a_T;
  } else if (m.liq) {
    const float iK = rcp(m.Kliq);
    const float El = m.Kliq * ph.T_m + m.chi * ph.rho_l * ph.latent;
    a_rhoH += a_T * iK;
    a_El -= a_T * iK;
    a_Kliq -= (m.rhoH - El) * iK * iK * a_T;
  } else if (m.span > 0.0f) {
    const float is = rcp(m.span);
    a_rhoH += a_fl * is;
    a_Es += a_fl * (m.fl_m - 1.0f) * is;
    a_El -= a_fl * m.fl_m * is;
  }
  a_Ksol += ph.T_m * a_Es;
  a_Kliq += ph.T_m * a_El;
  a_chi += ph.rho_l * ph.latent * a_El;
  // Ksol = Zrho(s_sol, C) Zcp(s_sol, C), s_sol = min(1, phi0 + chi);
  // Kliq = Zrho(phi0, C) Zcp(phi0, C)
  {
    const float ss = fminf(1.0f, phi0 + m.chi);
    const float Zrs = zeta(ss, C, ph.rho_s, ph.rho_l, ph.rho_g);
    const float Zcs = zeta(ss, C, ph.cp_s, ph.cp_l, ph.cp_g);
    const float Zrl = zeta(phi0, C, ph.rho_s, ph.rho_l, ph.rho_g);
    const float Zcl = zeta(phi0, C, ph.cp_s, ph.cp_l, ph.cp_g);
    const float a_Zrs = Zcs * a_Ksol, a_Zcs = Zrs * a_Ksol;
    const float a_Zrl = Zcl * a_Kliq, a_Zcl = Zrl * a_Kliq;
    const float a_ss = a_Zrs * dzeta_ds(C, ph.rho_s, ph.rho_l, ph.rho_g) +
                       a_Zcs * dzeta_ds(C, ph.cp_s, ph.cp_l, ph.cp_g);
    a_C += a_Zrs * dzeta_dC(ss, ph.rho_l, ph.rho_g) + a_Zcs * dzeta_dC(ss, ph.cp_l, ph.cp_g) +
           a_Zrl * dzeta_dC(phi0, ph.rho_l, ph.rho_g) + a_Zcl * dzeta_dC(phi0, ph.cp_l, ph.cp_g);
    if (phi0 + m.chi <= 1.0f) a_chi += a_ss;
  }
  // rhoH = sum h + Q_prev / 2
  a_sh = a_rhoH;
  // chi = clamp(chi1, 0, 1 - phi0), chi1 = max(Cp, fs_prev) (latched) or Cp
  const float a_chi1 = (m.chi1 >= 0.0f && m.chi1 <= 1.0f - phi0) ? a_chi : 0.0f;
  float a_Cp = a_chi1;
  if (ph.latch) {
    if (m.Cp < fs_prev) {
      a_Cp = 0.0f;
      a_fsp += a_chi1;
    } else if (m.Cp == fs_prev) {
      a_Cp = 0.5f * a_chi1;
      a_fsp += 0.5f * a_chi1;
    }
  }
  // Cp = clamp((C - floor) / (1 - floor), 0, 1); C = clamp((1 - phi0 + phihat) / 2, 0, 1)
  if (m.Cpraw >= 0.0f && m.Cpraw <= 1.0f) a_C += a_Cp * ph.inv_pcm_span;
  if (m.Craw >= 0.0f && m.Craw <= 1.0f) a_phihat += 0.5f * a_C;
  a_sg = a_phihat;
}

// Reverse of collide_node<true> at one node.
//  fv, hv: the pulled flow and enthalpy populations (hv[0] the low part of
//    the float-float rest population, as the forward uses it);
//  af, ag, ah: on entry d J / d (post-collision populations); on return
//    d J / d (pulled populations) through the collision alone;
//  aL: d J / d (lagged outputs f_s, Q, (phi u)_x, (phi u)_y, p);
//  loc, st: adjoints of the moment quantities and stencil values used;
//  a_jxp, a_jyp: d J / d (lagged (phi u) read by the collision);
//  a_cth: d J / d cos(theta) of the node.
__device__ __forceinline__ void collide_reverse(const Phys& ph, const Mom& m, const Stencil& S,
                                                float phi0, float cth, float lap_phi0,
                                                const float* fv, const float* hv, float* af,
                                                float* ag, float* ah, const float* aL,
                                                float* loc, float* st, float& a_jxp,
                                                float& a_jyp, float& a_cth) {
  // ---------------- forward values
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
  const float fs = m.fs;
  const float mu_v = zeta(fstot, C, ph.mu_s, ph.mu_l, ph.mu_g);
  const float lam = zeta(fstot, C, ph.lam_s, ph.lam_l, ph.lam_g);
  const float cp = zeta(fstot, C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float inv_rho = rcp(rho);
  const float tau_f = 3.0f * mu_v * inv_rho + 0.5f;
  const float ia = rcp(lam * ph.three_over_Eref + 0.5f);
  const float is = 2.0f - ia;
  const float a = ph.a3, kk = ph.kap, cps = ph.cos_psi;
  const float mu = chem_pot(ph, phi, lphi, phi0, cth, lap_phi0, fs, lfs);
  const float Fx = mu * gphx, Fy = mu * gphy;
  float mx = 0, my = 0, snz = 0;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    mx += cx(i) * fv[i];
    my += cy(i) * fv[i];
    if (i) snz += fv[i];
  }
  const float usx = (mx + 0.5f * Fx) * inv_rho, usy = (my + 0.5f * Fy) * inv_rho;
  const float fdx = -fstot * usx, fdy = -fstot * usy;
  const float ux = usx + 0.5f * fdx, uy = usy + 0.5f * fdy;
  const float Sm = rho * mdot + ux * grx + uy * gry;
  const float Ftx = Fx - gpx + (1.0f / 3.0f) * grx, Fty = Fy - gpy + (1.0f / 3.0f) * gry;
  const float uu = ux * ux + uy * uy;
  const float uFt = ux * Ftx + uy * Fty;
  const float w0 = wgt(0);
  const float F0 = w0 * (Sm - 3.0f * uFt);
  const float Kp = (1.0f / 3.0f) / (1.0f - w0);
  const float p = Kp * (snz + 0.5f * Sm + (tau_f - 0.5f) * F0 - 1.5f * w0 * rho * uu);
  const float ift = rcp(tau_f);
  const float pf = 1.0f - 0.5f * ift;
  const float rfx = rho * fdx + Fx, rfy = rho * fdy + Fy;
  const float rhocp = rho * cp;
  const float ET = ph.Eref * T, cT = rhocp * T;
  const float Q = cT * mdot;
  const bool reset = ph.subfix && phi0 >= 0.5f;

  // ---------------- reverse
  float a_ux = 0, a_uy = 0, a_uu = 0, a_rho = 0, a_p = aL[LAG_P], a_phi = 0, a_mu = 0;
  float a_jx = aL[LAG_JX], a_jy = aL[LAG_JY], a_mdot = 0, a_T = 0, a_rhoH = 0;
  float a_Q = aL[LAG_Q], a_ia = 0, a_is = 0, a_rhocp = 0, a_chi = 0, a_Ksol = 0, a_Kliq = 0;
  float a_fs = aL[LAG_FS];

  // enthalpy populations
  if (reset) {
    // held node: every h* is the equilibrium at the held temperature; only
    // the rest population depends on the state, through rho H(T_held)
    const float Tw = ph.T_sub;
    const float a_rH = ah[0];
    if (Tw <= ph.T_m) {
      a_Ksol += a_rH * Tw;
    } else {
      a_Kliq += a_rH * Tw;
      a_chi += a_rH * ph.rho_l * ph.latent;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) ah[i] = 0.0f;
  } else {
    const float ps = ph.src_tau_a ? (1.0f - 0.5f * ia) : (1.0f - 0.5f * is);
    float heq[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float cu = cx(i) * ux + cy(i) * uy;
      // rest population relative to the node's reference, as in the forward
      heq[i] = (i == 0) ? m.dH - (1.0f - w0) * ET - 1.5f * w0 * cT * uu
                        : wgt(i) * (ET + cT * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
    }
    float a_e[9], ah_in[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      a_e[i] = 0.0f;
      ah_in[i] = 0.0f;
    }
    float a_ps = 0.0f;
    // h*_i = h_i - ia (h_i - h_j)/2 - is (h_i + h_j)/2 + ia (e_i - e_j)/2
    //        + is (e_i + e_j)/2 + ps w_i Q,  j = opp(i)
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const int j = opp(i);
      const float A = ah[i];
      ah_in[i] += A * (1.0f - 0.5f * ia - 0.5f * is);
      ah_in[j] += A * (0.5f * ia - 0.5f * is);
      a_e[i] += A * (0.5f * ia + 0.5f * is);
      a_e[j] += A * (0.5f * is - 0.5f * ia);
      a_ia -= 0.5f * A * ((hv[i] - hv[j]) - (heq[i] - heq[j]));
      a_is -= 0.5f * A * ((hv[i] + hv[j]) - (heq[i] + heq[j]));
      a_ps += A * wgt(i) * Q;
      a_Q += A * ps * wgt(i);
    }
    if (ph.src_tau_a) a_ia -= 0.5f * a_ps;
    else a_is -= 0.5f * a_ps;
    // e_0 = rhoH - ET + w0 (ET - 1.5 cT uu),  e_i = w_i (ET + cT P_i)
    float a_ET = (w0 - 1.0f) * a_e[0];
    float a_cT = -1.5f * w0 * uu * a_e[0];
    a_uu -= 1.5f * w0 * cT * a_e[0];
    a_rhoH += a_e[0];
#pragma unroll
    for (int i = 1; i < 9; ++i) {
      const float cu = cx(i) * ux + cy(i) * uy;
      const float P = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
      a_ET += wgt(i) * a_e[i];
      a_cT += wgt(i) * P * a_e[i];
      a_uu -= 1.5f * wgt(i) * cT * a_e[i];
      const float a_cu = wgt(i) * cT * (3.0f + 9.0f * cu) * a_e[i];
      a_ux += cx(i) * a_cu;
      a_uy += cy(i) * a_cu;
    }
    a_T += ph.Eref * a_ET + rhocp * a_cT;
    a_rhocp += T * a_cT;
#pragma unroll
    for (int i = 0; i < 9; ++i) ah[i] = ah_in[i];
  }
  // Q = rho cp T mdot
  a_rhocp += T * mdot * a_Q;
  a_T += rhocp * mdot * a_Q;
  a_mdot += cT * a_Q;
  // phase field: g*_i = g_i (1 - 1/tau_g) + geq_i / tau_g + pg G_i
  {
    const float igt = ph.inv_tau_g, pg = ph.pg;
    float sG = 0.0f;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const float A = ag[i];
      const float a_geq = igt * A, a_G = pg * A;
      ag[i] = (1.0f - igt) * A;
      if (i == 0) a_phi += a_geq;
      a_mu += (wgt(i) - (i == 0 ? 1.0f : 0.0f)) * a_geq;
      a_jx += 3.0f * wgt(i) * cx(i) * (a_geq + a_G);
      a_jy += 3.0f * wgt(i) * cy(i) * (a_geq + a_G);
      a_jxp -= 3.0f * wgt(i) * cx(i) * a_G;
      a_jyp -= 3.0f * wgt(i) * cy(i) * a_G;
      sG += wgt(i) * a_G;
    }
    a_phi += mdot * sG;
    a_mdot += phi * sG;
  }
  // j = phi u
  a_phi += ux * a_jx + uy * a_jy;
  a_ux += phi * a_jx;
  a_uy += phi * a_jy;
  // flow: f*_i = f_i (1 - 1/tau_f) + feq_i / tau_f + pf F_i
  float a_ift = 0.0f, a_Sm = 0.0f, a_rfx = 0.0f, a_rfy = 0.0f, a_uFt = 0.0f;
  float a_Ftx = 0.0f, a_Fty = 0.0f;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const float A = af[i];
    const float cu = cx(i) * ux + cy(i) * uy;
    const float cF = cx(i) * rfx + cy(i) * rfy;
    const float cFt = cx(i) * Ftx + cy(i) * Fty;
    const float P = 3.0f * cu + 4.5f * cu * cu - 1.5f * uu;
    const float feq = 3.0f * p * (wgt(i) - (i == 0 ? 1.0f : 0.0f)) + rho * wgt(i) * P;
    const float Fi = wgt(i) * (Sm + 3.0f * cF + 9.0f * cu * cFt - 3.0f * uFt);
    af[i] = (1.0f - ift) * A;
    const float a_feq = ift * A, a_F = pf * A;
    a_ift += A * (feq - fv[i]) - 0.5f * A * Fi;
    a_p += 3.0f * (wgt(i) - (i == 0 ? 1.0f : 0.0f)) * a_feq;
    a_rho += wgt(i) * P * a_feq;
    float a_cu = rho * wgt(i) * (3.0f + 9.0f * cu) * a_feq;
    a_uu -= 1.5f * rho * wgt(i) * a_feq;
    a_Sm += wgt(i) * a_F;
    a_rfx += 3.0f * wgt(i) * cx(i) * a_F;
    a_rfy += 3.0f * wgt(i) * cy(i) * a_F;
    a_cu += 9.0f * wgt(i) * cFt * a_F;
    const float a_cFt = 9.0f * wgt(i) * cu * a_F;
    a_Ftx += cx(i) * a_cFt;
    a_Fty += cy(i) * a_cFt;
    a_uFt -= 3.0f * wgt(i) * a_F;
    a_ux += cx(i) * a_cu;
    a_uy += cy(i) * a_cu;
  }
  // rf = rho fd + F
  float a_fdx = rho * a_rfx, a_fdy = rho * a_rfy;
  a_rho += fdx * a_rfx + fdy * a_rfy;
  float a_Fx = a_rfx, a_Fy = a_rfy;
  // p = Kp (snz + Sm/2 + (tau_f - 1/2) F0 - 1.5 w0 rho uu)
  const float a_snz = Kp * a_p;
  a_Sm += 0.5f * Kp * a_p;
  float a_tauf = Kp * F0 * a_p;
  const float a_F0 = Kp * (tau_f - 0.5f) * a_p;
  a_rho -= 1.5f * w0 * uu * Kp * a_p;
  a_uu -= 1.5f * w0 * rho * Kp * a_p;
  // F0 = w0 (Sm - 3 uFt)
  a_Sm += w0 * a_F0;
  a_uFt -= 3.0f * w0 * a_F0;
  // uFt = u . Ft, uu = u . u
  a_ux += Ftx * a_uFt + 2.0f * ux * a_uu;
  a_uy += Fty * a_uFt + 2.0f * uy * a_uu;
  a_Ftx += ux * a_uFt;
  a_Fty += uy * a_uFt;
  // Ft = F - grad p + grad rho / 3
  a_Fx += a_Ftx;
  a_Fy += a_Fty;
  const float a_gpx = -a_Ftx, a_gpy = -a_Fty;
  float a_grx = a_Ftx * (1.0f / 3.0f), a_gry = a_Fty * (1.0f / 3.0f);
  // Sm = rho mdot + u . grad rho
  a_rho += mdot * a_Sm;
  a_mdot += rho * a_Sm;
  a_ux += grx * a_Sm;
  a_uy += gry * a_Sm;
  a_grx += ux * a_Sm;
  a_gry += uy * a_Sm;
  // u = us + fd / 2, fd = -fstot us
  float a_usx = a_ux, a_usy = a_uy;
  a_fdx += 0.5f * a_ux;
  a_fdy += 0.5f * a_uy;
  float a_fstot = -usx * a_fdx - usy * a_fdy;
  a_usx -= fstot * a_fdx;
  a_usy -= fstot * a_fdy;
  // us = (m + F / 2) / rho
  const float a_mx = a_usx * inv_rho, a_my = a_usy * inv_rho;
  a_Fx += 0.5f * a_mx;
  a_Fy += 0.5f * a_my;
  a_rho -= (usx * a_usx + usy * a_usy) * inv_rho;
#pragma unroll
  for (int i = 0; i < 9; ++i) af[i] += cx(i) * a_mx + cy(i) * a_my + (i ? a_snz : 0.0f);
  // F = mu grad phi
  a_mu += gphx * a_Fx + gphy * a_Fy;
  const float a_gphx = mu * a_Fx, a_gphy = mu * a_Fy;
  // chemical potential (derivative of the free energy eq44)
  a_phi += a_mu * (a * (3.0f * phi * phi - 1.0f) + 3.0f * a * phi0 * phi0 +
                   6.0f * a * cth * phi0 * phi + 3.0f * a * fs * fs + 6.0f * a * cps * fs * phi);
  a_fs += a_mu * (6.0f * a * fs * phi + a * cps * (3.0f * phi * phi + 3.0f * fs * fs - 1.0f));
  const float a_lphi = -kk * a_mu, a_lfs = -kk * cps * a_mu;
  a_cth += a_mu * (a * phi0 * (3.0f * phi * phi + phi0 * phi0 - 1.0f) - kk * lap_phi0);
  // relaxation rates: 1/tau_f, 1/tau_a (1/tau_s = 2 - 1/tau_a)
  a_tauf -= ift * ift * a_ift;
  a_ia -= a_is;
  const float a_lam = -ia * ia * a_ia * ph.three_over_Eref;
  const float a_muv = 3.0f * inv_rho * a_tauf;
  a_rho -= 3.0f * mu_v * inv_rho * inv_rho * a_tauf;
  // rho cp
  a_rho += cp * a_rhocp;
  const float a_cp = rho * a_rhocp;
  // mixing rule of mu, lambda, C_p in (fstot, C)
  a_fstot += a_muv * dzeta_ds(C, ph.mu_s, ph.mu_l, ph.mu_g) +
             a_lam * dzeta_ds(C, ph.lam_s, ph.lam_l, ph.lam_g) +
             a_cp * dzeta_ds(C, ph.cp_s, ph.cp_l, ph.cp_g);
  const float a_C = a_muv * dzeta_dC(fstot, ph.mu_l, ph.mu_g) +
                    a_lam * dzeta_dC(fstot, ph.lam_l, ph.lam_g) +
                    a_cp * dzeta_dC(fstot, ph.cp_l, ph.cp_g);
  loc[AL_PHI] = a_phi;
  loc[AL_RHO] = a_rho;
  loc[AL_FS] = a_fs;
  loc[AL_C] = a_C;
  loc[AL_FSTOT] = a_fstot;
  loc[AL_MDOT] = a_mdot;
  loc[AL_T] = a_T;
  loc[AL_RHOH] = a_rhoH;
  loc[AL_CHI] = a_chi;
  loc[AL_KSOL] = a_Ksol;
  loc[AL_KLIQ] = a_Kliq;
  st[AS_GPHX] = a_gphx;
  st[AS_GPHY] = a_gphy;
  st[AS_LPHI] = a_lphi;
  st[AS_LFS] = a_lfs;
  st[AS_GRX] = a_grx;
  st[AS_GRY] = a_gry;
  st[AS_GPX] = a_gpx;
  st[AS_GPY] = a_gpy;
}

// Arguments of the adjoint of step n.
struct AdjStepArgs {
  Geo G;
  Phys ph;
  BufArgs F;          // forward state n (din, lin, stat, wallT, wstride)
  const float* mom;   // phi, f_s, rho of state n (3 planes)
  const float* lamD;  // NADJ_D planes, time level n + 1
  const float* lamL;  // NADJ_L planes, time level n + 1
  float* outD;        // NADJ_D planes, time level n
  float* outL;        // NADJ_L planes, time level n
  float* st;          // NST planes
  float* jac;         // NJAC planes
  double* gcth;       // nx * ny, accumulated
  double* gwall;      // 4 * wstride, accumulated
};

// Adjoint of the distributions a node wrote in step n (slots j of D^{n+1}),
// gathered through the transpose of step n + 1's pull.  Anti-bounce-back
// links add their wall-temperature derivative to gwall (each wall entry is
// reached from one node only).
__device__ __forceinline__ void gather_pull_adjoint(const Geo& G, const Phys& ph,
                                                    const float* __restrict__ lamD, int x, int y,
                                                    double* gwall, int wstride, float* af,
                                                    float* ag, float* ah) {
  const size_t P = (size_t)G.P;
  const int k = y * G.nx + x;
  // every lane requests the five values of each slot first (source node and
  // plane chosen per lane, no branch around the loads), so the 45 loads are
  // in flight together; the sums and the wall rules follow
  float vf[9], vg[9], vsg[9], vh[9], vsh[9];
  uint32_t wmask = 0u, ymask = 0u;
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    const int tx = pull_axis(x, -cx(j), G.nx, G.px), ty = pull_axis(y, -cy(j), G.ny, G.py);
    const bool wy = ty < 0, w = wy || tx < 0;
    wmask |= (uint32_t)w << j;
    ymask |= (uint32_t)wy << j;
    // across a wall the node pulls slot j back as population opp(j)
    const size_t r = w ? (size_t)k : (size_t)ty * G.nx + tx;
    const int pj = w ? opp(j) : j;
    vf[j] = lamD[pj * P + r];
    vg[j] = lamD[(9 + pj) * P + r];
    vsg[j] = lamD[AD_SG * P + r];
    vh[j] = lamD[(18 + pj) * P + r];
    vsh[j] = lamD[AD_SH * P + r];
  }
#pragma unroll
  for (int j = 0; j < 9; ++j) {
    af[j] = vf[j];
    ag[j] = vg[j] + vsg[j];
    const float A = vh[j] + vsh[j];
    ah[j] = A;
    if ((wmask >> j) & 1u) {
      const int i = opp(j);
      const int wall = ((ymask >> j) & 1u) ? (cy(i) > 0 ? 0 : 1) : (cx(i) > 0 ? 2 : 3);
      if ((G.tmask >> wall) & 1) {
        ah[j] = -A;
        gwall[wall * wstride + (wall < 2 ? x : y)] += 2.0 * (double)wgt(i) * (double)ph.Eref * A;
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_adj_collide(AdjStepArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.G.nx) return;
  const Geo& G = a.G;
  const Phys& ph = a.ph;
  const Bufs B = make_bufs(a.F, G);
  const size_t P = (size_t)G.P;
  const int k = y * G.nx + x;
  // forward recompute of the node
  NodeIn in;
  node_load(G, ph, B, x, y, in);
  Mom m;
  float s4[4];
  node_finish(ph, in, m, s4);
  FlowIn fl;
  flow_load(G, ph, B, x, y, fl);
  Stencil S;
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    const int xx = map_axis(x + cx(i), G.nx, G.px), yy = map_axis(y + cy(i), G.ny, G.py);
    const size_t kk = (size_t)yy * G.nx + xx;
    S.phi[i] = a.mom[kk];
    S.fs[i] = a.mom[P + kk];
    S.rho[i] = a.mom[2 * P + kk];
    S.p[i] = a.F.lin[LAG_P * P + kk];
  }
  // adjoint of what the node wrote
  float af[9], ag[9], ah[9], aL[NADJ_L];
  gather_pull_adjoint(G, ph, a.lamD, x, y, a.gwall, a.F.wstride, af, ag, ah);
#pragma unroll
  for (int j = 0; j < NADJ_L; ++j) aL[j] = a.lamL[j * P + k];
  float loc[NLOC], st[NST], ajx = 0.0f, ajy = 0.0f, acth = 0.0f;
  collide_reverse(ph, m, S, in.phi0, fl.cth, fl.lap0, fl.f, in.h, af, ag, ah, aL, loc, st, ajx,
                  ajy, acth);
#pragma unroll
  for (int i = 0; i < 9; ++i) {
    a.outD[i * P + k] = af[i];
    a.outD[(9 + i) * P + k] = ag[i];
    a.outD[(18 + i) * P + k] = ah[i];
  }
#pragma unroll
  for (int j = 0; j < NST; ++j) a.st[j * P + k] = st[j];
  a.outL[LAG_JX * P + k] = ajx;
  a.outL[LAG_JY * P + k] = ajy;
  // moment reverse: local part, then unit responses to phi, f_s and rho
  float jv[NJAC];
  moments_reverse(ph, m, in.phi0, in.fsp, loc, jv[0], jv[1], jv[2]);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float e[NLOC];
#pragma unroll
    for (int q = 0; q < NLOC; ++q) e[q] = 0.0f;
    e[c == 0 ? AL_PHI : (c == 1 ? AL_FS : AL_RHO)] = 1.0f;
    moments_reverse(ph, m, in.phi0, in.fsp, e, jv[3 + 3 * c], jv[4 + 3 * c], jv[5 + 3 * c]);
  }
#pragma unroll
  for (int q = 0; q < NJAC; ++q) a.jac[q * P + k] = jv[q];
  a.gcth[k] += (double)acth;
}

// Source nodes v (along one axis) whose neighbour v + c maps to t under the
// forward stencil's wrap / mirror-ghost rule; at most two.
__device__ __forceinline__ int stencil_sources(int t, int c, int n, int periodic, int* v) {
  int cnt = 0;
  int s = t - c;
  if (periodic) {
    if (s < 0) s += n;
    else if (s >= n) s -= n;
    v[cnt++] = s;
    return cnt;
  }
  if (s >= 0 && s < n) v[cnt++] = s;
  if (c == -1 && t == 0) v[cnt++] = 0;        // the ghost below row 0 mirrors row 0
  if (c == 1 && t == n - 1) v[cnt++] = n - 1; // the ghost above row n - 1 mirrors it
  return cnt;
}

struct AdjGatherArgs {
  Geo G;
  const float* st;
  const float* jac;
  float* outD;
  float* outL;
};

__global__ __launch_bounds__(256) void k_adj_gather(AdjGatherArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.G.nx) return;
  const Geo& G = a.G;
  const size_t P = (size_t)G.P;
  const int k = y * G.nx + x;
  const float* __restrict__ st = a.st;
  float dphi = 0.0f, dfs = 0.0f, drho = 0.0f, dp = 0.0f;
  // contribution of one source node s through link i
  auto add = [&](int i, size_t s) {
    const float w = wgt(i);
    dphi += 3.0f * w * (cx(i) * st[AS_GPHX * P + s] + cy(i) * st[AS_GPHY * P + s]) +
            6.0f * w * st[AS_LPHI * P + s];
    dfs += 6.0f * w * st[AS_LFS * P + s];
    drho += 3.0f * w * (cx(i) * st[AS_GRX * P + s] + cy(i) * st[AS_GRY * P + s]);
    dp += 3.0f * w * (cx(i) * st[AS_GPX * P + s] + cy(i) * st[AS_GPY * P + s]);
  };
  // first the first source of each link: one per link away from a wall,
  // requested by every lane (a valid node either way, the term dropped where
  // the link has none), so these loads are in flight together; then, in a
  // separate pass, the mirror-ghost sources that only boundary nodes have
  int vx[9][2], vy[9][2], nxs[9], nys[9];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    nxs[i] = stencil_sources(x, cx(i), G.nx, G.px, vx[i]);
    nys[i] = stencil_sources(y, cy(i), G.ny, G.py, vy[i]);
  }
  float t8[9][8];
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    const size_t s = (size_t)(nys[i] > 0 ? vy[i][0] : y) * G.nx + (nxs[i] > 0 ? vx[i][0] : x);
#pragma unroll
    for (int q = 0; q < 8; ++q) t8[i][q] = st[q * P + s];
  }
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (nxs[i] > 0 && nys[i] > 0) {
      const float w = wgt(i);
      dphi += 3.0f * w * (cx(i) * t8[i][AS_GPHX] + cy(i) * t8[i][AS_GPHY]) + 6.0f * w * t8[i][AS_LPHI];
      dfs += 6.0f * w * t8[i][AS_LFS];
      drho += 3.0f * w * (cx(i) * t8[i][AS_GRX] + cy(i) * t8[i][AS_GRY]);
      dp += 3.0f * w * (cx(i) * t8[i][AS_GPX] + cy(i) * t8[i][AS_GPY]);
    }
  }
#pragma unroll
  for (int i = 1; i < 9; ++i) {
    if (nxs[i] > 1 || nys[i] > 1) {
      for (int b = 0; b < nys[i]; ++b)
        for (int c = 0; c < nxs[i]; ++c)
          if (b > 0 || c > 0) add(i, (size_t)vy[i][b] * G.nx + vx[i][c]);
    }
  }
  // the node's own value in its Laplacians (weights of the moving links: 5/9)
  dphi -= 6.0f * (5.0f / 9.0f) * st[AS_LPHI * P + k];
  dfs -= 6.0f * (5.0f / 9.0f) * st[AS_LFS * P + k];
  float r[3];
#pragma unroll
  for (int q = 0; q < 3; ++q)
    r[q] = a.jac[q * P + k] + a.jac[(3 + q) * P + k] * dphi + a.jac[(6 + q) * P + k] * dfs +
           a.jac[(9 + q) * P + k] * drho;
  a.outD[AD_SG * P + k] = r[0];
  a.outD[AD_SH * P + k] = r[1];
  a.outL[LAG_FS * P + k] = r[2];
  a.outL[LAG_Q * P + k] = 0.5f * r[1];
  a.outL[LAG_P * P + k] = dp;
}

// Seed of the reverse sweep: d J / d (phi, T, f_s) of the final state's
// fields (NULL planes are zero) to the adjoint of that state.
struct AdjSeedArgs {
  Geo G;
  Phys ph;
  BufArgs F;          // final state
  const float* sphi;  // nx * ny or NULL
  const float* sT;
  const float* sfs;
  float* outD;
  float* outL;
};

__global__ __launch_bounds__(256) void k_adj_seed(AdjSeedArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.G.nx) return;
  const Geo& G = a.G;
  const Bufs B = make_bufs(a.F, G);
  const size_t P = (size_t)G.P;
  const int k = y * G.nx + x;
  NodeIn in;
  node_load(G, a.ph, B, x, y, in);
  Mom m;
  float s4[4];
  node_finish(a.ph, in, m, s4);
  float loc[NLOC];
#pragma unroll
  for (int q = 0; q < NLOC; ++q) loc[q] = 0.0f;
  loc[AL_PHI] = a.sphi ? a.sphi[k] : 0.0f;
  loc[AL_T] = a.sT ? a.sT[k] : 0.0f;
  loc[AL_FS] = a.sfs ? a.sfs[k] : 0.0f;
  float sg, sh, sfp;
  moments_reverse(a.ph, m, in.phi0, in.fsp, loc, sg, sh, sfp);
  for (int q = 0; q < 27; ++q) a.outD[q * P + k] = 0.0f;
  a.outD[AD_SG * P + k] = sg;
  a.outD[AD_SH * P + k] = sh;
  a.outL[LAG_FS * P + k] = sfp;
  a.outL[LAG_Q * P + k] = 0.5f * sh;
  a.outL[LAG_JX * P + k] = 0.0f;
  a.outL[LAG_JY * P + k] = 0.0f;
  a.outL[LAG_P * P + k] = 0.0f;
}

// Wettability term of the initial state: the initial g are equilibria
// phi delta_i0 + (w_i - delta_i0) mu(phi, cos theta) (fs = 0), so
// d J / d cos(theta) gains sum_i (w_i - delta_i0) lambda_g,i d mu / d cos(theta).
struct AdjInitArgs {
  Geo G;
  Phys ph;
  BufArgs F;          // initial state
  const float* lamD;  // time level 0
  double* gcth;
};

__global__ __launch_bounds__(256) void k_adj_init(AdjInitArgs a) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x, y = blockIdx.y;
  if (x >= a.G.nx) return;
  const Geo& G = a.G;
  const Phys& ph = a.ph;
  const Bufs B = make_bufs(a.F, G);
  const size_t P = (size_t)G.P;
  const int k = y * G.nx + x;
  NodeIn in;
  node_load(G, ph, B, x, y, in);
  float phi = in.ghi;
#pragma unroll
  for (int i = 0; i < 9; ++i) phi += in.g[i];
  const float phi0 = in.phi0;
  const float lap0 = ldp(B.stat, ST_LAP0, G.P, k);
  const float dmu = ph.a3 * phi0 * (3.0f * phi * phi + phi0 * phi0 - 1.0f) - ph.kap * lap0;
  // sum_i (w_i - delta_i0) = 0: the d J / d (sum g) part cancels
  float s = -a.lamD[9 * P + k];
#pragma unroll
  for (int i = 0; i < 9; ++i) s += wgt(i) * a.lamD[(9 + i) * P + k];
  a.gcth[k] += (double)s * (double)dmu;
}

}  // namespace lbf
