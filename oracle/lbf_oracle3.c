/*
 * FP64 CPU oracle of the coupled lattice Boltzmann freezing step on the
 * three-dimensional D3Q19 lattice (arXiv 2510.18688, Sec. 3: the same flow,
 * phase-field and enthalpy schemes with the nineteen-velocity set).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with the
 * HIP path, nor with the two-dimensional oracle.
 *
 * Full-lattice passes in IEEE double precision, in the order
 *   (1) node-local moments, enthalpy map, mass source, properties,
 *   (2) stencils, chemical potential, forces, velocity, pressure, the three
 *       collisions and the isothermal-region reset,
 *   (3) streaming with the wall rules.
 * State: post-streaming f_i, g_i, h_i (19 each) and the lagged f_s,
 * Q = rho C_p T mdot, phi u (3 components), p and u (3 components, for the
 * phase-field source of R54) of the previous step.
 * Node (x, y, z) is element (z ny + y) nx + x.  The readings of the
 * two-dimensional oracle apply unchanged; R49 and R50 are the 3D additions
 * (uniform temperature per Dirichlet face; wall precedence z, y, x).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D3Q19 (Sec. 3.1): c_0 = 0; c_1..c_6 along +-x, +-y, +-z; c_7..c_18 the
 * twelve face diagonals, in the printed order; w = 1/3, 1/18, 1/36. */
#define Q 19
static const int CX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int CY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int CZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};
static double W[Q];
static int OPP[Q];
#define CS2 (1.0 / 3.0)

static void lattice_init(void) {
  for (int i = 0; i < Q; ++i) {
    int n2 = CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i];
    W[i] = n2 == 0 ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
    for (int j = 0; j < Q; ++j)
      if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) OPP[i] = j;
  }
}

/* faces: x low, x high, y low, y high, z low, z high */
enum { FXL = 0, FXH, FYL, FYH, FZL, FZH };

typedef struct {
  int32_t nx, ny, nz, periodic[3];
  int32_t thermal_bc[6];      /* per face: 0 adiabatic, 1 Dirichlet */
  int32_t latch_fs, h_src_tau_a, substrate_fixed, pad_;
  double rho_l, rho_g, rho_s, mu_l, mu_g, mu_s, lam_l, lam_g, lam_s;
  double cp_l, cp_g, cp_s;
  double latent, T_m, sigma, eps, mobility, cos_psi, rho_ref, T_substrate;
  double pcm_floor;
  double wall_T[6];           /* temperature of each Dirichlet face (R49) */
  double grav[3];             /* body force G = rho g (R32) */
  double u_solid[3];          /* solid-phase velocity u_s of the drag */
  int32_t phi_src_mdot;       /* div u in the phase-field source and recovery: 0 the
                                 isotropic divergence of the previous step's velocity
                                 (R54), 1 the mass source mdot (R12) */
  int32_t pad2_;
} orc3_params;

typedef struct {
  orc3_params p;
  int n3[3];
  size_t n;
  double *f, *g, *h, *fc, *gc, *hc;            /* [Q][n] */
  double *fs_prev, *Q_prev, *jx_prev, *jy_prev, *jz_prev, *p_prev;
  double *fs_new, *Q_new, *jx_new, *jy_new, *jz_new, *p_new;
  double *phi0, *cth, *lap_phi0;
  double *phihat, *C, *chi, *rhoH, *T, *fs, *fstot, *mdot, *phi, *rho, *Ksol, *Kliq;
  double *ux, *uy, *uz, *pr, *mu;
  double *ux_lag, *uy_lag, *uz_lag, *ux_new, *uy_new, *uz_new; /* velocity, previous step (R54) */
  double *divu;                 /* div u of the phase-field source: R54 or R12 */
  double budget[4];
  long step;
} orc3_sim;

static inline double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}
static inline double zeta(double s, double C, double zs, double zl, double zg) {
  return s * zs + (1.0 - s) * (C * zl + (1.0 - C) * zg);
}
static inline double cp_ref(const orc3_params* p) {
  return 2.0 * p->cp_s * p->cp_l / (p->cp_s + p->cp_l);
}

/* Enthalpy map (Sec. 2, Hfl) for a node of phase-change fraction chi (R1). */
static void hmap(const orc3_params* p, double rhoH, double phi0, double C, double chi,
                 double* T, double* fl, double* Ksol_out, double* Kliq_out) {
  double s_sol = fmin(1.0, phi0 + chi);
  double Kliq = zeta(phi0, C, p->rho_s, p->rho_l, p->rho_g) *
                zeta(phi0, C, p->cp_s, p->cp_l, p->cp_g);
  double Ksol = zeta(s_sol, C, p->rho_s, p->rho_l, p->rho_g) *
                zeta(s_sol, C, p->cp_s, p->cp_l, p->cp_g);
  double Es = Ksol * p->T_m, El = Kliq * p->T_m + chi * p->rho_l * p->latent;
  if (rhoH < Es) {
    *fl = 0.0;
    *T = rhoH / Ksol;
  } else if (rhoH <= El) {
    *fl = (El > Es) ? (rhoH - Es) / (El - Es) : 1.0;
    *T = p->T_m;
  } else {
    *fl = 1.0;
    *T = p->T_m + (rhoH - El) / Kliq;
  }
  *Ksol_out = Ksol;
  *Kliq_out = Kliq;
}

static double enthalpy_at(const orc3_params* p, double Tw, double Ksol, double Kliq,
                          double chi) {
  if (Tw <= p->T_m) return Ksol * Tw;
  return Kliq * (Tw - p->T_m) + Kliq * p->T_m + chi * p->rho_l * p->latent;
}

/* Equilibria and forcing of Sec. 3.1-3.3 with three-component vectors. */
void orc3_feq(double p, double rho, const double* u, double* out) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    double s = W[i] * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2));
    out[i] = p / CS2 * (W[i] - (i == 0 ? 1.0 : 0.0)) + rho * s;
  }
}

void orc3_forcing(double S, const double* F, const double* rf, const double* Ft,
                  const double* u, double* out) {
  double uFt = u[0] * Ft[0] + u[1] * Ft[1] + u[2] * Ft[2];
  for (int i = 0; i < Q; ++i) {
    double cF = CX[i] * (F[0] + rf[0]) + CY[i] * (F[1] + rf[1]) + CZ[i] * (F[2] + rf[2]);
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    double cFt = CX[i] * Ft[0] + CY[i] * Ft[1] + CZ[i] * Ft[2];
    double t2 = (2.0 * cu * cFt - CS2 * 2.0 * uFt) / (2 * CS2 * CS2);
    out[i] = W[i] * (S + cF / CS2 + t2);
  }
}

void orc3_geq(double phi, double mu, const double* j, double* out) {
  for (int i = 0; i < Q; ++i) {
    double cj = CX[i] * j[0] + CY[i] * j[1] + CZ[i] * j[2];
    out[i] = (i == 0 ? phi : 0.0) + (W[i] - (i == 0 ? 1.0 : 0.0)) * mu + W[i] * cj / CS2;
  }
}

void orc3_heq(double rhoH, double T, double rhocp, double Eref, const double* u, double* out) {
  double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
  for (int i = 0; i < Q; ++i) {
    double cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
    if (i == 0)
      out[i] = rhoH - Eref * T + W[0] * (Eref * T - rhocp * T * uu / (2 * CS2));
    else
      out[i] = W[i] * (Eref * T + rhocp * T * (cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 * CS2)));
  }
}

/* lattice tables for the algebra checks */
void orc3_lattice(int* c /* 3 x Q */, double* w, int* opp) {
  lattice_init();
  for (int i = 0; i < Q; ++i) {
    c[i] = CX[i];
    c[Q + i] = CY[i];
    c[2 * Q + i] = CZ[i];
    w[i] = W[i];
    opp[i] = OPP[i];
  }
}

/* ------------------------------------------------------------ stencils */
static inline int nb_axis(int i, int n, int periodic) {
  if (i < 0) return periodic ? i + n : 0;       /* mirror ghost beyond a wall (R38) */
  if (i >= n) return periodic ? i - n : n - 1;
  return i;
}

static inline size_t idx(const orc3_sim* s, int x, int y, int z) {
  return ((size_t)z * s->n3[1] + y) * s->n3[0] + x;
}

/* Isotropic D3Q19 stencils (R15 with the 3D weights). */
static void grad_lap(const orc3_sim* s, const double* X, int x, int y, int z, double* g,
                     double* lap) {
  double sx = 0, sy = 0, sz = 0, sl = 0;
  double xc = X[idx(s, x, y, z)];
  for (int i = 1; i < Q; ++i) {
    int xx = nb_axis(x + CX[i], s->n3[0], s->p.periodic[0]);
    int yy = nb_axis(y + CY[i], s->n3[1], s->p.periodic[1]);
    int zz = nb_axis(z + CZ[i], s->n3[2], s->p.periodic[2]);
    double v = X[idx(s, xx, yy, zz)];
    sx += W[i] * CX[i] * v;
    sy += W[i] * CY[i] * v;
    sz += W[i] * CZ[i] * v;
    sl += W[i] * (v - xc);
  }
  if (g) {
    g[0] = sx / CS2;
    g[1] = sy / CS2;
    g[2] = sz / CS2;
  }
  if (lap) *lap = 2.0 * sl / CS2;
}

void orc3_stencil(int nx, int ny, int nz, const int* periodic, const double* X, double* gx,
                  double* gy, double* gz, double* lap) {
  orc3_sim s;
  memset(&s, 0, sizeof s);
  lattice_init();
  s.n3[0] = nx; s.n3[1] = ny; s.n3[2] = nz;
  for (int a = 0; a < 3; ++a) s.p.periodic[a] = periodic[a];
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(&s, x, y, z);
        double g[3];
        grad_lap(&s, X, x, y, z, g, &lap[k]);
        gx[k] = g[0]; gy[k] = g[1]; gz[k] = g[2];
      }
}

/* -------------------------------------------------------------- create */
static double* alloc0(size_t n) { return (double*)calloc(n, sizeof(double)); }

#define ONE_FIELDS(s)                                                                      \
  &s->fs_prev, &s->Q_prev, &s->jx_prev, &s->jy_prev, &s->jz_prev, &s->p_prev, &s->fs_new,  \
      &s->Q_new, &s->jx_new, &s->jy_new, &s->jz_new, &s->p_new, &s->phi0, &s->cth,          \
      &s->lap_phi0, &s->phihat, &s->C, &s->chi, &s->rhoH, &s->T, &s->fs, &s->fstot,         \
      &s->mdot, &s->phi, &s->rho, &s->Ksol, &s->Kliq, &s->ux, &s->uy, &s->uz, &s->pr, &s->mu, \
      &s->ux_lag, &s->uy_lag, &s->uz_lag, &s->ux_new, &s->uy_new, &s->uz_new, &s->divu

orc3_sim* orc3_create(const orc3_params* p) {
  if (p->nx <= 0 || p->ny <= 0 || p->nz <= 0) return NULL;
  lattice_init();
  orc3_sim* s = (orc3_sim*)calloc(1, sizeof(orc3_sim));
  s->p = *p;
  s->n3[0] = p->nx; s->n3[1] = p->ny; s->n3[2] = p->nz;
  s->n = (size_t)p->nx * p->ny * p->nz;
  double** big[] = {&s->f, &s->g, &s->h, &s->fc, &s->gc, &s->hc};
  for (size_t k = 0; k < 6; ++k) *big[k] = alloc0(Q * s->n);
  double** one[] = {ONE_FIELDS(s)};
  for (size_t k = 0; k < sizeof one / sizeof one[0]; ++k) *one[k] = alloc0(s->n);
  return s;
}

void orc3_destroy(orc3_sim* s) {
  if (!s) return;
  double** big[] = {&s->f, &s->g, &s->h, &s->fc, &s->gc, &s->hc};
  for (size_t k = 0; k < 6; ++k) free(*big[k]);
  double** one[] = {ONE_FIELDS(s)};
  for (size_t k = 0; k < sizeof one / sizeof one[0]; ++k) free(*one[k]);
  free(s);
}

void orc3_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

/* derivative of the free energy eq44 (Sec. 2) */
static double chem_pot(const orc3_params* p, double phi, double lap_phi, double phi0,
                       double cth, double lap_phi0, double fs, double lap_fs) {
  double a = 3.0 * p->sigma / p->eps, k = 3.0 * p->eps * p->sigma / 8.0;
  double m = a * phi * (phi * phi - 1.0) - k * lap_phi;
  m += 3.0 * a * phi0 * phi0 * phi + a * cth * phi0 * (3 * phi * phi + phi0 * phi0 - 1.0) -
       k * cth * lap_phi0;
  m += 3.0 * a * fs * fs * phi + a * p->cos_psi * fs * (3 * phi * phi + fs * fs - 1.0) -
       k * p->cos_psi * lap_fs;
  return m;
}

/* -------------------------------------------------------------- pass 1 */
static void pass1(orc3_sim* s) {
  const orc3_params* p = &s->p;
  const size_t n = s->n;
  const long nn = (long)n;
#pragma omp parallel for schedule(static)
  for (long kk = 0; kk < nn; ++kk) {
    size_t k = (size_t)kk;
    double sg = 0, sh = 0;
    for (int i = 0; i < Q; ++i) {
      sg += s->g[i * n + k];
      sh += s->h[i * n + k];
    }
    double phi0 = s->phi0[k];
    double C = clampd(0.5 * (1.0 - phi0 + sg), 0.0, 1.0);
    double Cp = clampd((C - p->pcm_floor) / (1.0 - p->pcm_floor), 0.0, 1.0);
    double chi = p->latch_fs ? fmax(Cp, s->fs_prev[k]) : Cp;
    chi = clampd(chi, 0.0, 1.0 - phi0);
    double rhoH = sh + 0.5 * s->Q_prev[k];
    double T, fl, Ksol, Kliq;
    hmap(p, rhoH, phi0, C, chi, &T, &fl, &Ksol, &Kliq);
    double fs = chi * (1.0 - fl);
    double fstot = fmin(1.0, phi0 + fs);
    double mdot = (1.0 - p->rho_s / p->rho_l) * (fs - s->fs_prev[k]);
    /* div u of the phase-field equation (Sec. 3.2): the model's mdot (R12), or
     * the divergence of the flow's own velocity of the previous step with the
     * isotropic stencil (R54) */
    double divu = mdot;
    if (!p->phi_src_mdot) {
      int x = (int)(k % (size_t)s->n3[0]);
      int y = (int)((k / (size_t)s->n3[0]) % (size_t)s->n3[1]);
      int z = (int)(k / ((size_t)s->n3[0] * s->n3[1]));
      double gx[3], gy[3], gz[3];
      grad_lap(s, s->ux_lag, x, y, z, gx, NULL);
      grad_lap(s, s->uy_lag, x, y, z, gy, NULL);
      grad_lap(s, s->uz_lag, x, y, z, gz, NULL);
      divu = gx[0] + gy[1] + gz[2];
    }
    s->divu[k] = divu;
    s->phihat[k] = sg; s->C[k] = C; s->chi[k] = chi; s->rhoH[k] = rhoH; s->T[k] = T;
    s->fs[k] = fs; s->fstot[k] = fstot; s->mdot[k] = mdot;
    s->phi[k] = sg / (1.0 - 0.5 * divu);
    s->Ksol[k] = Ksol; s->Kliq[k] = Kliq;
    s->rho[k] = zeta(fstot, C, p->rho_s, p->rho_l, p->rho_g);
  }
}

/* -------------------------------------------------------------- pass 2 */
static void pass2(orc3_sim* s, int collide) {
  const orc3_params* p = &s->p;
  const size_t n = s->n;
  const double Eref = p->rho_ref * cp_ref(p);
  const double tau_g = p->mobility / CS2 + 0.5;
  const int nz = s->n3[2], ny = s->n3[1], nx = s->n3[0];
  double* acc = (double*)calloc((size_t)nz * ny * 3, sizeof(double));
#pragma omp parallel for schedule(static) collapse(2)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      double a_heat = 0, a_phi = 0, a_reset = 0;
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, y, z);
        double phi = s->phi[k], rho = s->rho[k], C = s->C[k], fs = s->fs[k];
        double fstot = s->fstot[k], mdot = s->mdot[k], T = s->T[k];
        double mu_v = zeta(fstot, C, p->mu_s, p->mu_l, p->mu_g);
        double lam = zeta(fstot, C, p->lam_s, p->lam_l, p->lam_g);
        double cp = zeta(fstot, C, p->cp_s, p->cp_l, p->cp_g);
        double tau_f = mu_v / rho / CS2 + 0.5;
        double tau_a = lam / Eref / CS2 + 0.5;
        double tau_s = 1.0 / (2.0 - 1.0 / tau_a);
        double gph[3], gr[3], gp[3], lphi, lfs;
        grad_lap(s, s->phi, x, y, z, gph, &lphi);
        grad_lap(s, s->fs, x, y, z, NULL, &lfs);
        grad_lap(s, s->rho, x, y, z, gr, NULL);
        grad_lap(s, s->p_prev, x, y, z, gp, NULL);
        double mu = chem_pot(p, phi, lphi, s->phi0[k], s->cth[k], s->lap_phi0[k], fs, lfs);
        double F[3], m[3] = {0, 0, 0}, sum_nz = 0;
        for (int a = 0; a < 3; ++a) F[a] = mu * gph[a] + rho * p->grav[a];
        for (int i = 0; i < Q; ++i) {
          double fi = s->f[i * n + k];
          m[0] += CX[i] * fi;
          m[1] += CY[i] * fi;
          m[2] += CZ[i] * fi;
          if (i) sum_nz += fi;
        }
        double us[3], fd[3], u[3], Ft[3], rf[3];
        for (int a = 0; a < 3; ++a) {
          us[a] = (m[a] + 0.5 * F[a]) / rho;
          fd[a] = fstot * (p->u_solid[a] - us[a]);
          u[a] = us[a] + 0.5 * fd[a];
        }
        double S = rho * mdot + u[0] * gr[0] + u[1] * gr[1] + u[2] * gr[2];
        for (int a = 0; a < 3; ++a) {
          Ft[a] = F[a] - gp[a] + CS2 * gr[a];
          rf[a] = rho * fd[a];
        }
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double uFt = u[0] * Ft[0] + u[1] * Ft[1] + u[2] * Ft[2];
        double F0 = W[0] * (S - uFt / CS2);
        double s0 = W[0] * (-uu / (2 * CS2));
        double pr = CS2 / (1.0 - W[0]) * (sum_nz + 0.5 * S + (tau_f - 0.5) * F0 + rho * s0);
        s->ux[k] = u[0]; s->uy[k] = u[1]; s->uz[k] = u[2]; s->pr[k] = pr; s->mu[k] = mu;
        if (!collide) continue;
        double feq[Q], Fi[Q];
        orc3_feq(pr, rho, u, feq);
        orc3_forcing(S, F, rf, Ft, u, Fi);
        for (int i = 0; i < Q; ++i) {
          double fi = s->f[i * n + k];
          s->fc[i * n + k] = fi - (fi - feq[i]) / tau_f + (1.0 - 0.5 / tau_f) * Fi[i];
        }
        double j[3] = {phi * u[0], phi * u[1], phi * u[2]};
        double dj[3] = {j[0] - s->jx_prev[k], j[1] - s->jy_prev[k], j[2] - s->jz_prev[k]};
        double geq[Q];
        orc3_geq(phi, mu, j, geq);
        for (int i = 0; i < Q; ++i) {
          double Gi = W[i] * (CX[i] * dj[0] + CY[i] * dj[1] + CZ[i] * dj[2]) / CS2 +
                      W[i] * phi * s->divu[k];
          double gi = s->g[i * n + k];
          s->gc[i * n + k] = gi - (gi - geq[i]) / tau_g + (1.0 - 0.5 / tau_g) * Gi;
        }
        double rhocp = rho * cp;
        double heq[Q];
        orc3_heq(s->rhoH[k], T, rhocp, Eref, u, heq);
        double Qs = rhocp * T * mdot;
        double tau_src = p->h_src_tau_a ? tau_a : tau_s;
        double hsum = 0.0;
        for (int i = 0; i < Q; ++i) {
          int jj = OPP[i];
          double hi = s->h[i * n + k], hj = s->h[jj * n + k];
          double ha = 0.5 * (hi - hj), hs = 0.5 * (hi + hj);
          double ea = 0.5 * (heq[i] - heq[jj]), es = 0.5 * (heq[i] + heq[jj]);
          double v = hi - (ha - ea) / tau_a - (hs - es) / tau_s +
                     (1.0 - 0.5 / tau_src) * W[i] * Qs;
          s->hc[i * n + k] = v;
          hsum += v;
        }
        a_heat += 0.5 * s->Q_prev[k] / tau_s + (1.0 - 0.5 / tau_src) * Qs;
        a_phi += phi * s->divu[k];
        if (p->substrate_fixed && s->phi0[k] >= 0.5) {
          double Tw = p->T_substrate;
          double rH = enthalpy_at(p, Tw, s->Ksol[k], s->Kliq[k], s->chi[k]);
          double e[Q], zero[3] = {0, 0, 0}, es = 0.0;
          orc3_heq(rH, Tw, rhocp, Eref, zero, e);
          for (int i = 0; i < Q; ++i) {
            es += e[i];
            s->hc[i * n + k] = e[i];
          }
          a_reset += es - hsum;
        }
        s->fs_new[k] = fs; s->Q_new[k] = Qs;
        s->jx_new[k] = j[0]; s->jy_new[k] = j[1]; s->jz_new[k] = j[2];
        s->p_new[k] = pr;
        s->ux_new[k] = u[0]; s->uy_new[k] = u[1]; s->uz_new[k] = u[2];
      }
      size_t r = (size_t)z * ny + y;
      acc[3 * r] = a_heat; acc[3 * r + 1] = a_phi; acc[3 * r + 2] = a_reset;
    }
  if (collide) {
    double h = 0, ph = 0, rs = 0;
    for (size_t r = 0; r < (size_t)nz * ny; ++r) {
      h += acc[3 * r]; ph += acc[3 * r + 1]; rs += acc[3 * r + 2];
    }
    s->budget[0] = ph; s->budget[1] = h; s->budget[3] = rs;
  }
  free(acc);
}

/* ------------------------------------------------------------ stream */
/* X_i(x, t+1) = X_i*(x - c_i); beyond a wall (half-way, R17) f and g bounce
 * back, h bounces back (adiabatic) or is anti-bounced with
 * 2 w_i rho_ref C_p,ref T_w (Dirichlet).  A link leaving through several
 * walls takes the z wall, else the y wall, else the x wall (R50). */
static void stream(orc3_sim* s) {
  const orc3_params* p = &s->p;
  const size_t n = s->n;
  const double Eref = p->rho_ref * cp_ref(p);
  const int nz = s->n3[2], ny = s->n3[1], nx = s->n3[0];
  double* flux = (double*)calloc((size_t)nz * ny, sizeof(double));
#pragma omp parallel for schedule(static) collapse(2)
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y) {
      double fl = 0.0;
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, y, z);
        for (int i = 0; i < Q; ++i) {
          int src[3] = {x - CX[i], y - CY[i], z - CZ[i]};
          int wall = -1;
          for (int a = 2; a >= 0; --a) {
            if (src[a] < 0 || src[a] >= s->n3[a]) {
              if (p->periodic[a]) src[a] = (src[a] + s->n3[a]) % s->n3[a];
              else if (wall < 0) wall = 2 * a + (src[a] < 0 ? 0 : 1);
            }
          }
          if (wall < 0) {
            size_t sk = idx(s, src[0], src[1], src[2]);
            s->f[i * n + k] = s->fc[i * n + sk];
            s->g[i * n + k] = s->gc[i * n + sk];
            s->h[i * n + k] = s->hc[i * n + sk];
          } else {
            int j = OPP[i];
            s->f[i * n + k] = s->fc[j * n + k];
            s->g[i * n + k] = s->gc[j * n + k];
            if (p->thermal_bc[wall]) {
              double v = -s->hc[j * n + k] + 2.0 * W[i] * Eref * p->wall_T[wall];
              s->h[i * n + k] = v;
              fl += v - s->hc[j * n + k];
            } else {
              s->h[i * n + k] = s->hc[j * n + k];
            }
          }
        }
      }
      flux[(size_t)z * ny + y] = fl;
    }
  double tot = 0.0;
  for (size_t r = 0; r < (size_t)nz * ny; ++r) tot += flux[r];
  free(flux);
  s->budget[2] = tot;
}

static void swap_lagged(orc3_sim* s) {
  double* t;
#define SWAP(a, b) (t = a, a = b, b = t)
  SWAP(s->fs_prev, s->fs_new);
  SWAP(s->Q_prev, s->Q_new);
  SWAP(s->jx_prev, s->jx_new);
  SWAP(s->jy_prev, s->jy_new);
  SWAP(s->jz_prev, s->jz_new);
  SWAP(s->p_prev, s->p_new);
  SWAP(s->ux_lag, s->ux_new);
  SWAP(s->uy_lag, s->uy_new);
  SWAP(s->uz_lag, s->uz_new);
#undef SWAP
}

void orc3_step(orc3_sim* s, int nsteps) {
  for (int it = 0; it < nsteps; ++it) {
    pass1(s);
    pass2(s, 1);
    stream(s);
    swap_lagged(s);
    s->step++;
  }
}

/* ------------------------------------------------------------- init */
int orc3_init(orc3_sim* s, const double* phi0, const double* cth, const double* phi,
              const double* T0) {
  const orc3_params* p = &s->p;
  const size_t n = s->n;
  const double Eref = p->rho_ref * cp_ref(p);
  memcpy(s->phi0, phi0, n * sizeof(double));
  memcpy(s->cth, cth, n * sizeof(double));
  const int nz = s->n3[2], ny = s->n3[1], nx = s->n3[0];
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) grad_lap(s, s->phi0, x, y, z, NULL, &s->lap_phi0[idx(s, x, y, z)]);
  memset(s->f, 0, Q * n * sizeof(double));
  double** lag[] = {&s->fs_prev, &s->Q_prev, &s->jx_prev, &s->jy_prev, &s->jz_prev, &s->p_prev,
                    &s->ux_lag, &s->uy_lag, &s->uz_lag};   /* u = 0 initially (R29) */
  for (int a = 0; a < 9; ++a) memset(*lag[a], 0, n * sizeof(double));
  memcpy(s->phi, phi, n * sizeof(double));
  double zero[3] = {0, 0, 0};
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        size_t k = idx(s, x, y, z);
        double lphi;
        grad_lap(s, s->phi, x, y, z, NULL, &lphi);
        double mu = chem_pot(p, phi[k], lphi, phi0[k], cth[k], s->lap_phi0[k], 0.0, 0.0);
        double geq[Q], heq[Q];
        orc3_geq(phi[k], mu, zero, geq);
        double C = clampd(0.5 * (1.0 - phi0[k] + phi[k]), 0.0, 1.0);
        double Cp = clampd((C - p->pcm_floor) / (1.0 - p->pcm_floor), 0.0, 1.0);
        double chi = clampd(Cp, 0.0, 1.0 - phi0[k]);
        double Kliq = zeta(phi0[k], C, p->rho_s, p->rho_l, p->rho_g) *
                      zeta(phi0[k], C, p->cp_s, p->cp_l, p->cp_g);
        double rhoH = Kliq * (T0[k] - p->T_m) + Kliq * p->T_m + chi * p->rho_l * p->latent;
        orc3_heq(rhoH, T0[k], 0.0, Eref, zero, heq);
        for (int i = 0; i < Q; ++i) {
          s->g[i * n + k] = geq[i];
          s->h[i * n + k] = heq[i];
        }
      }
  memset(s->budget, 0, sizeof s->budget);
  s->step = 0;
  return 0;
}

/* fields: 0 phi, 1 T, 2 1 - f_s, 3 f_s, 4 u_x, 5 u_y, 6 u_z, 7 p, 8 rho H,
 * 9 mu_phi, 10 C, 11 chi, 12 rho, 13 sum g */
#define ORC3_NFIELDS 14
int orc3_nfields(void) { return ORC3_NFIELDS; }

void orc3_fields(orc3_sim* s, double* out) {
  pass1(s);
  pass2(s, 0);
  const size_t n = s->n;
  for (size_t k = 0; k < n; ++k) {
    out[0 * n + k] = s->phi[k];
    out[1 * n + k] = s->T[k];
    out[2 * n + k] = 1.0 - s->fs[k];
    out[3 * n + k] = s->fs[k];
    out[4 * n + k] = s->ux[k];
    out[5 * n + k] = s->uy[k];
    out[6 * n + k] = s->uz[k];
    out[7 * n + k] = s->pr[k];
    out[8 * n + k] = s->rhoH[k];
    out[9 * n + k] = s->mu[k];
    out[10 * n + k] = s->C[k];
    out[11 * n + k] = s->chi[k];
    out[12 * n + k] = s->rho[k];
    out[13 * n + k] = s->phihat[k];
  }
}

/* 0 sum g, 1 sum h, 2 sum f_s, 3 sum (chi - f_s), 4 max |u|, 5 non-finite,
 * 6..9 budget of the last step, 10 step */
void orc3_reduce(orc3_sim* s, double* out) {
  pass1(s);
  pass2(s, 0);
  const size_t n = s->n;
  double sg = 0, sh = 0, sfs = 0, sliq = 0, umax = 0, bad = 0;
  for (size_t k = 0; k < n; ++k) {
    for (int i = 0; i < Q; ++i) {
      sg += s->g[i * n + k];
      sh += s->h[i * n + k];
    }
    sfs += s->fs[k];
    sliq += s->chi[k] - s->fs[k];
    double um = sqrt(s->ux[k] * s->ux[k] + s->uy[k] * s->uy[k] + s->uz[k] * s->uz[k]);
    if (um > umax) umax = um;
    if (!isfinite(s->phi[k]) || !isfinite(s->T[k]) || !isfinite(um) || !isfinite(s->pr[k]))
      bad += 1;
  }
  out[0] = sg; out[1] = sh; out[2] = sfs; out[3] = sliq; out[4] = umax; out[5] = bad;
  out[6] = s->budget[0]; out[7] = s->budget[1]; out[8] = s->budget[2]; out[9] = s->budget[3];
  out[10] = (double)s->step;
}

long orc3_step_count(orc3_sim* s) { return s->step; }
