/*
 * FP64 CPU oracle of the coupled lattice Boltzmann freezing step
 * (Huang, Zhan, Chai, Huang, "A diffuse-interface method for the containerless
 * freezing of three-phase flows in complex geometries", arXiv 2510.18688).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
 * baseline of the benchmark may load this library.  It shares no code with the
 * HIP path: no headers, no helpers, no tables.
 *
 * It is a plain, slow, obviously-correct transcription of the method: every
 * node is visited in separate full-lattice passes, in the order
 *   (1) node-local moments, enthalpy map, mass source, properties,
 *   (2) stencils, chemical potential, forces, velocity, pressure, the three
 *       collisions and the isothermal-region reset,
 *   (3) streaming with the wall rules,
 * all in IEEE double precision.  The state is kept in the paper's notation:
 * post-streaming distributions f_i, g_i, h_i at time t, plus the lagged fields
 * that the implicit and time-derivative terms need (f_s, Q = rho C_p T mdot,
 * phi u and p of the previous step).
 *
 * Readings of the paper where it is silent or garbled are numbered R1..R55
 * and listed in the design notes; each is marked below where it applies.
 *
 * Parity unpinned: the phase-change fraction chi (R1-R3: which part of the
 * liquid may freeze, its latch by the previous ice fraction) and its floor
 * (R45) have no value printed by the paper to pin against; they are checked
 * only through the enthalpy-map identities, the exact budgets and the
 * three-phase Stefan problem (Table 1), where no gas is present.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- lattice */
/* D2Q9 velocities and weights (Sec. 3.1): c_0 = 0; c_1..c_4 axis-aligned,
 * counter-clockwise from +x; c_5..c_8 diagonals, counter-clockwise from (1,1);
 * w = 4/9, 1/9, 1/36. */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double W[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9,
                            1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};
#define CS2 (1.0 / 3.0)

/* ---------------------------------------------------------------- params */
typedef struct {
  int32_t nx, ny, periodic_x, periodic_y;
  int32_t thermal_bc[4];      /* bottom, top, left, right: 0 adiabatic, 1 Dirichlet */
  int32_t latch_fs;           /* R3 */
  int32_t h_src_tau_a;        /* R9 */
  int32_t substrate_fixed;    /* R21: phi0 >= 1/2 held at T_substrate */
  int32_t pad_;
  double rho_l, rho_g, rho_s, mu_l, mu_g, mu_s, lam_l, lam_g, lam_s;
  double cp_l, cp_g, cp_s;
  double latent, T_m, sigma, eps, mobility, cos_psi, rho_ref, T_substrate;
  double pcm_floor;           /* R45 */
  int32_t mrt;                /* 1: MRT flow collision (R53) */
  int32_t pad2_;
  int32_t phi_src_mdot;       /* div u in the phase-field source and recovery: 0 the
                                 discrete divergence of the previous step's velocity
                                 (R54), 1 the mass source mdot (R12) */
  int32_t pad3_;
  double s_b, s_q;            /* MRT rates: density, e and epsilon moments; energy flux
                                 (0: the BGK rate 1/tau_f) */
  double s_g;                 /* MRT rate of the phase-field moments above first order
                                 (0: the BGK rate 1/tau_g) */
  double grav[2];             /* body force G = rho g (R32) */
  double u_solid[2];          /* solid-phase velocity u_s of the drag */
} orc_params;

enum { WB = 0, WT = 1, WL = 2, WR = 3 };

typedef struct {
  orc_params p;
  int nx, ny;
  size_t n;
  double *f, *g, *h;            /* post-stream distributions [9][n] */
  double *fc, *gc, *hc;         /* post-collision distributions [9][n] */
  double *fs_prev, *Q_prev, *phiux_prev, *phiuy_prev, *p_prev;
  double *fs_new, *Q_new, *phiux_new, *phiuy_new, *p_new;
  double *phi0, *cth, *lap_phi0;
  double *thold;                /* per-node held temperature (NaN: free); used when
                                   held_per_node is set (O14 with a given region) */
  int held_per_node;
  double *wallT[4];
  /* pass-1 arrays */
  double *phihat, *C, *chi, *rhoH, *T, *fl, *fs, *fstot, *mdot, *phi, *rho, *Ksol, *Kliq;
  /* pass-2 diagnostics */
  double *ux, *uy, *pr, *mu;
  double *ux_lag, *uy_lag, *ux_new, *uy_new; /* velocity of the previous step (R54) */
  double *divu;                 /* div u of the phase-field source: R54 or R12 */
  double budget[4];             /* sum phi div u, heat source, wall flux, reset */
  long step;
  int store_f32;                /* conditioning probe: round the state to binary32 each step */
  double mrtM[81], mrtMinv[81]; /* MRT basis and its inverse (R53) */
} orc_sim;

/* --------------------------------------------------------- small helpers */
static inline double clampd(double v, double lo, double hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

/* Property mixing rule (Sec. 2, the linear rule for rho, mu, lambda, C_p):
 * zeta = s zeta_s + (1 - s) [C zeta_l + (1 - C) zeta_g],
 * with s the solid fraction (R2: ice plus pre-existing solid) and
 * C = (1 - phi0 + phi)/2 the liquid weight. */
static inline double zeta(double s, double C, double zs, double zl, double zg) {
  return s * zs + (1.0 - s) * (C * zl + (1.0 - C) * zg);
}

static inline double cp_ref(const orc_params* p) {
  /* Sec. 3.3: C_p,ref is the harmonic mean of the solid and liquid values. */
  return 2.0 * p->cp_s * p->cp_l / (p->cp_s + p->cp_l);
}

/* Enthalpy map (Sec. 2, eq. Hfl) with T_s = T_l = T_m (R26), generalised to a
 * node holding a phase-change fraction chi (R1): sensible capacities of the
 * node with its PCM all frozen (K_sol) and all liquid (K_liq); latent heat
 * chi rho_l L.  With chi = 1 and phi0 = 0 this is exactly Hfl.  Returns the
 * liquid fraction of the PCM and the temperature. */
static void hmap(const orc_params* p, double rhoH, double phi0, double C, double chi,
                 double* T, double* fl, double* Ksol_out, double* Kliq_out) {
  double s_liq = phi0;
  double s_sol = fmin(1.0, phi0 + chi);
  double Kliq = zeta(s_liq, C, p->rho_s, p->rho_l, p->rho_g) *
                zeta(s_liq, C, p->cp_s, p->cp_l, p->cp_g);
  double Ksol = zeta(s_sol, C, p->rho_s, p->rho_l, p->rho_g) *
                zeta(s_sol, C, p->cp_s, p->cp_l, p->cp_g);
  double Es = Ksol * p->T_m;
  double El = Kliq * p->T_m + chi * p->rho_l * p->latent;
  if (rhoH < Es) {
    *fl = 0.0;
    *T = rhoH / Ksol;
  } else if (rhoH <= El) {
    /* R34: an empty mushy interval (El == Es) counts as liquid */
    *fl = (El > Es) ? (rhoH - Es) / (El - Es) : 1.0;
    *T = p->T_m;
  } else {
    *fl = 1.0;
    *T = p->T_m + (rhoH - El) / Kliq;
  }
  if (Ksol_out) *Ksol_out = Ksol;
  if (Kliq_out) *Kliq_out = Kliq;
}

/* Enthalpy of a node held at temperature Tw: frozen at or below T_m, liquid
 * above (inverse of hmap on its solid and liquid branches; R21, R27). */
static double enthalpy_at(const orc_params* p, double Tw, double Ksol, double Kliq,
                          double chi) {
  if (Tw <= p->T_m) return Ksol * Tw;
  return Kliq * (Tw - p->T_m) + Kliq * p->T_m + chi * p->rho_l * p->latent;
}

/* Pressure-based flow equilibrium (Sec. 3.1):
 * f_i^eq = (p/c_s^2)(w_i - delta_i0) + rho s_i(u),
 * s_i(u) = w_i [c.u/c_s^2 + (c.u)^2/(2 c_s^4) - u.u/(2 c_s^2)]. */
void orc_feq(double p, double rho, double ux, double uy, double* out) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    double s = W[i] * (cu / CS2 + cu * cu / (2 * CS2 * CS2) - uu / (2 * CS2));
    out[i] = p / CS2 * (W[i] - (i == 0 ? 1.0 : 0.0)) + rho * s;
  }
}

/* Flow forcing (Sec. 3.1):
 * F_i = w_i [S + c.(F + rho f)/c_s^2 + (u Ft + Ft u):(c c - c_s^2 I)/(2 c_s^4)],
 * with the total force F, the solid drag rho f and Ft (R10). */
void orc_forcing(double S, double Fx, double Fy, double rfx, double rfy,
                 double Ftx, double Fty, double ux, double uy, double* out) {
  for (int i = 0; i < 9; ++i) {
    double cF = CX[i] * (Fx + rfx) + CY[i] * (Fy + rfy);
    double cu = CX[i] * ux + CY[i] * uy;
    double cFt = CX[i] * Ftx + CY[i] * Fty;
    /* (uFt + Ftu):(cc) = 2 (c.u)(c.Ft); (uFt + Ftu):I = 2 u.Ft */
    double t2 = (2.0 * cu * cFt - CS2 * 2.0 * (ux * Ftx + uy * Fty)) / (2 * CS2 * CS2);
    out[i] = W[i] * (S + cF / CS2 + t2);
  }
}

/* Phase-field equilibrium (Sec. 3.2), eta = 1 (R11):
 * g_0^eq = phi + (w_0 - 1) mu,  g_i^eq = w_i mu + w_i c_i.(phi u)/c_s^2. */
/* ------------------------------------------------------------ MRT (R53) */
/* Orthogonal moment basis of the D2Q9 lattice (Lallemand and Luo): density,
 * energy e, energy square epsilon, momentum j_x, energy flux q_x, j_y, q_y,
 * and the stresses p_xx, p_xy, as polynomials of the velocities. */
void orc_mrt_matrix(double* M /* 81, row-major: moment k, velocity i */) {
  for (int i = 0; i < 9; ++i) {
    double cx = CX[i], cy = CY[i], c2 = cx * cx + cy * cy;
    M[0 * 9 + i] = 1.0;
    M[1 * 9 + i] = -4.0 + 3.0 * c2;
    M[2 * 9 + i] = 4.0 - 10.5 * c2 + 4.5 * c2 * c2;
    M[3 * 9 + i] = cx;
    M[4 * 9 + i] = (-5.0 + 3.0 * c2) * cx;
    M[5 * 9 + i] = cy;
    M[6 * 9 + i] = (-5.0 + 3.0 * c2) * cy;
    M[7 * 9 + i] = cx * cx - cy * cy;
    M[8 * 9 + i] = cx * cy;
  }
}

/* Inverse of a 9 x 9 matrix by Gauss-Jordan elimination with partial
 * pivoting. */
void orc_invert9(const double* A, double* Ainv) {
  double a[9][18];
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 18; ++c) a[r][c] = c < 9 ? A[r * 9 + c] : (c - 9 == r ? 1.0 : 0.0);
  for (int col = 0; col < 9; ++col) {
    int piv = col;
    for (int r = col + 1; r < 9; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 18; ++c) {
        double t = a[col][c];
        a[col][c] = a[piv][c];
        a[piv][c] = t;
      }
    double d = a[col][col];
    for (int c = 0; c < 18; ++c) a[col][c] /= d;
    for (int r = 0; r < 9; ++r) {
      if (r == col) continue;
      double f = a[r][col];
      for (int c = 0; c < 18; ++c) a[r][c] -= f * a[col][c];
    }
  }
  for (int r = 0; r < 9; ++r)
    for (int c = 0; c < 9; ++c) Ainv[r * 9 + c] = a[r][c + 9];
}

/* Relaxation rates of the nine moments: momentum and stresses at 1/tau_f
 * (the viscosity); density, e and epsilon at one bulk rate s_b (the three
 * moments the rest population projects on, so its non-equilibrium part keeps
 * the BGK form with tau_f -> 1/s_b); the energy fluxes at s_q. */
static void mrt_rates(const orc_params* p, double tau_f, double* sr) {
  double sv = 1.0 / tau_f;
  double sb = p->s_b > 0 ? p->s_b : sv, sq = p->s_q > 0 ? p->s_q : sv;
  double r[9] = {sb, sb, sb, sv, sq, sv, sq, sv, sv};
  memcpy(sr, r, sizeof r);
}

/* Rest-population non-equilibrium implied by the forcing, f_0^neq =
 * [M^-1 (S^-1 - 1/2) M F]_0: (tau_f - 1/2) F_0 for BGK. */
static double mrt_f0neq(const double* M, const double* Minv, const double* sr, const double* Fi) {
  double v = 0.0;
  for (int k = 0; k < 9; ++k) {
    double Fm = 0.0;
    for (int i = 0; i < 9; ++i) Fm += M[k * 9 + i] * Fi[i];
    v += Minv[0 * 9 + k] * (1.0 / sr[k] - 0.5) * Fm;
  }
  return v;
}

/* Post-collision f = M^-1 [m - S (m - m^eq) + (I - S/2) M F]. */
static void mrt_collide(const double* M, const double* Minv, const double* sr, const double* f,
                        const double* feq, const double* Fi, double* out) {
  double ms[9];
  for (int k = 0; k < 9; ++k) {
    double m = 0, me = 0, Fm = 0;
    for (int i = 0; i < 9; ++i) {
      m += M[k * 9 + i] * f[i];
      me += M[k * 9 + i] * feq[i];
      Fm += M[k * 9 + i] * Fi[i];
    }
    ms[k] = m - sr[k] * (m - me) + (1.0 - 0.5 * sr[k]) * Fm;
  }
  for (int i = 0; i < 9; ++i) {
    double v = 0;
    for (int k = 0; k < 9; ++k) v += Minv[i * 9 + k] * ms[k];
    out[i] = v;
  }
}

void orc_geq(double phi, double mu, double phiux, double phiuy, double* out) {
  for (int i = 0; i < 9; ++i) {
    double cj = CX[i] * phiux + CY[i] * phiuy;
    out[i] = (i == 0 ? phi : 0.0) + (W[i] - (i == 0 ? 1.0 : 0.0)) * mu + W[i] * cj / CS2;
  }
}

/* Total-enthalpy equilibrium (Sec. 3.3) with the reference capacity in the
 * rest term of i = 0 (R4): sum_i h_i^eq = rho H exactly. */
void orc_heq(double rhoH, double T, double rhocp, double Eref, double ux, double uy,
             double* out) {
  double uu = ux * ux + uy * uy;
  for (int i = 0; i < 9; ++i) {
    double cu = CX[i] * ux + CY[i] * uy;
    if (i == 0)
      out[i] = rhoH - Eref * T + W[0] * (Eref * T - rhocp * T * uu / (2 * CS2));
    else
      out[i] = W[i] * (Eref * T +
                       rhocp * T * (cu / CS2 + (cu * cu - CS2 * uu) / (2 * CS2 * CS2)));
  }
}

/* Exported enthalpy map for the algebra checks. */
void orc_hmap(const orc_params* p, double rhoH, double phi0, double C, double chi,
              double* out /* T, fl, Ksol, Kliq */) {
  hmap(p, rhoH, phi0, C, chi, &out[0], &out[1], &out[2], &out[3]);
}

/* ------------------------------------------------------------ geometry */
/* Neighbour index for the stencils: periodic wrap, or the mirror ghost that
 * repeats the first interior node beyond a wall (R38). */
static inline int nb_axis(int i, int n, int periodic) {
  if (i < 0) return periodic ? i + n : 0;
  if (i >= n) return periodic ? i - n : n - 1;
  return i;
}

/* Isotropic D2Q9 stencils (R15):
 * grad X = (1/c_s^2) sum_i w_i c_i X(x + c_i),
 * lap  X = (2/c_s^2) sum_i w_i [X(x + c_i) - X(x)]. */
static void grad_lap(const orc_sim* s, const double* X, int x, int y, double* gx,
                     double* gy, double* lap) {
  double sx = 0, sy = 0, sl = 0;
  double xc = X[(size_t)y * s->nx + x];
  for (int i = 1; i < 9; ++i) {
    int xx = nb_axis(x + CX[i], s->nx, s->p.periodic_x);
    int yy = nb_axis(y + CY[i], s->ny, s->p.periodic_y);
    double v = X[(size_t)yy * s->nx + xx];
    sx += W[i] * CX[i] * v;
    sy += W[i] * CY[i] * v;
    sl += W[i] * (v - xc);
  }
  if (gx) *gx = sx / CS2;
  if (gy) *gy = sy / CS2;
  if (lap) *lap = 2.0 * sl / CS2;
}

/* Exported stencil on a user array (for the stencil checks). */
void orc_stencil(int nx, int ny, int periodic_x, int periodic_y, const double* X,
                 double* gx, double* gy, double* lap) {
  orc_sim s;
  memset(&s, 0, sizeof s);
  s.nx = nx; s.ny = ny; s.p.periodic_x = periodic_x; s.p.periodic_y = periodic_y;
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t k = (size_t)y * nx + x;
      grad_lap(&s, X, x, y, &gx[k], &gy[k], &lap[k]);
    }
}

/* --------------------------------------------------------------- create */
static double* alloc0(size_t n) { return (double*)calloc(n, sizeof(double)); }

orc_sim* orc_create(const orc_params* p) {
  if (p->nx <= 0 || p->ny <= 0) return NULL;
  orc_sim* s = (orc_sim*)calloc(1, sizeof(orc_sim));
  s->p = *p;
  s->nx = p->nx; s->ny = p->ny;
  s->n = (size_t)p->nx * p->ny;
  size_t n = s->n;
  s->f = alloc0(9 * n); s->g = alloc0(9 * n); s->h = alloc0(9 * n);
  s->fc = alloc0(9 * n); s->gc = alloc0(9 * n); s->hc = alloc0(9 * n);
  double** one[] = {&s->fs_prev, &s->Q_prev, &s->phiux_prev, &s->phiuy_prev, &s->p_prev,
                    &s->fs_new, &s->Q_new, &s->phiux_new, &s->phiuy_new, &s->p_new,
                    &s->phi0, &s->cth, &s->lap_phi0, &s->thold,
                    &s->phihat, &s->C, &s->chi, &s->rhoH, &s->T, &s->fl, &s->fs,
                    &s->fstot, &s->mdot, &s->phi, &s->rho, &s->Ksol, &s->Kliq,
                    &s->ux, &s->uy, &s->pr, &s->mu, &s->ux_lag, &s->uy_lag,
                    &s->ux_new, &s->uy_new, &s->divu};
  for (size_t k = 0; k < sizeof one / sizeof one[0]; ++k) *one[k] = alloc0(n);
  s->wallT[WB] = alloc0(p->nx); s->wallT[WT] = alloc0(p->nx);
  s->wallT[WL] = alloc0(p->ny); s->wallT[WR] = alloc0(p->ny);
  orc_mrt_matrix(s->mrtM);
  orc_invert9(s->mrtM, s->mrtMinv);
  return s;
}

void orc_destroy(orc_sim* s) {
  if (!s) return;
  double* all[] = {s->f, s->g, s->h, s->fc, s->gc, s->hc, s->fs_prev, s->Q_prev,
                   s->phiux_prev, s->phiuy_prev, s->p_prev, s->fs_new, s->Q_new,
                   s->phiux_new, s->phiuy_new, s->p_new, s->phi0, s->cth, s->lap_phi0,
                   s->thold, s->phihat, s->C, s->chi, s->rhoH, s->T, s->fl, s->fs, s->fstot,
                   s->mdot, s->phi, s->rho, s->Ksol, s->Kliq, s->ux, s->uy, s->pr,
                   s->mu, s->ux_lag, s->uy_lag, s->ux_new, s->uy_new, s->divu,
                   s->wallT[0], s->wallT[1], s->wallT[2], s->wallT[3]};
  for (size_t k = 0; k < sizeof all / sizeof all[0]; ++k) free(all[k]);
  free(s);
}

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------- chemical potential */
/* mu_phi = dF/dphi of the free energy eq44 (Sec. 2):
 *  (3 sigma/eps) phi (phi^2 - 1) - (3 eps sigma/8) lap phi
 *  + (9 sigma/eps) phi0^2 phi + (3 sigma cos th/eps) phi0 (3 phi^2 + phi0^2 - 1)
 *  - (3 eps sigma cos th/8) lap phi0
 *  + (9 sigma/eps) fs^2 phi + (3 sigma cos psi/eps) fs (3 phi^2 + fs^2 - 1)
 *  - (3 eps sigma cos psi/8) lap fs.
 * cos th is taken per node (R28); fs is the ice fraction (R2). */
static double chem_pot(const orc_params* p, double phi, double lap_phi, double phi0,
                       double cth, double lap_phi0, double fs, double lap_fs) {
  double a = 3.0 * p->sigma / p->eps, k = 3.0 * p->eps * p->sigma / 8.0;
  double m = a * phi * (phi * phi - 1.0) - k * lap_phi;
  m += 3.0 * a * phi0 * phi0 * phi + a * cth * phi0 * (3 * phi * phi + phi0 * phi0 - 1.0) -
       k * cth * lap_phi0;
  m += 3.0 * a * fs * fs * phi + a * p->cos_psi * fs * (3 * phi * phi + fs * fs - 1.0) -
       k * p->cos_psi * lap_fs;
  return m;
}

/* Exported for the pins: mu_phi of one node from its values and the three
 * Laplacians. */
double orc_chem_pot(const orc_params* p, double phi, double lap_phi, double phi0, double cth,
                    double lap_phi0, double fs, double lap_fs) {
  return chem_pot(p, phi, lap_phi, phi0, cth, lap_phi0, fs, lap_fs);
}

/* -------------------------------------------------------- pass 1 */
/* Node-local moments (O1-O6 of the design notes). */
static void pass1(orc_sim* s) {
  const orc_params* p = &s->p;
  const size_t n = s->n;
#pragma omp parallel for schedule(static)
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t k = (size_t)y * s->nx + x;
      double sg = 0, sh = 0;
      for (int i = 0; i < 9; ++i) {
        sg += s->g[i * n + k];
        sh += s->h[i * n + k];
      }
      double phi0 = s->phi0[k];
      /* liquid weight of the mixing rule (Sec. 2) from the raw zeroth moment */
      double C = clampd(0.5 * (1.0 - phi0 + sg), 0.0, 1.0);
      /* R1, R3, R45: phase-change fraction from the liquid weight above a
       * small floor, latched by the previous ice fraction */
      double Cp = clampd((C - p->pcm_floor) / (1.0 - p->pcm_floor), 0.0, 1.0);
      double chi = p->latch_fs ? fmax(Cp, s->fs_prev[k]) : Cp;
      chi = clampd(chi, 0.0, 1.0 - phi0);
      /* total enthalpy (Sec. 3.3) with the source lagged one step (R14) */
      double rhoH = sh + 0.5 * s->Q_prev[k];
      double T, fl, Ksol, Kliq;
      hmap(p, rhoH, phi0, C, chi, &T, &fl, &Ksol, &Kliq);
      double fs = chi * (1.0 - fl);
      double fstot = fmin(1.0, phi0 + fs); /* R2 */
      /* mass source mdot = (1 - rho_s/rho_l) d fs/dt (eq1), backward difference (R13) */
      double mdot = (1.0 - p->rho_s / p->rho_l) * (fs - s->fs_prev[k]);
      /* div u of the phase-field equation (Sec. 3.2): the model's mdot (R12),
       * or the divergence of the flow's own velocity, the previous step's,
       * with the isotropic stencil (R54) */
      double divu = mdot;
      if (!p->phi_src_mdot) {
        double gxx, gxy, gyx, gyy;
        grad_lap(s, s->ux_lag, x, y, &gxx, &gxy, NULL);
        grad_lap(s, s->uy_lag, x, y, &gyx, &gyy, NULL);
        divu = gxx + gyy;
      }
      /* phi = sum g + (dt/2) phi div u (Sec. 3.2) */
      double phi = sg / (1.0 - 0.5 * divu);
      s->divu[k] = divu;
      s->phihat[k] = sg; s->C[k] = C; s->chi[k] = chi; s->rhoH[k] = rhoH;
      s->T[k] = T; s->fl[k] = fl; s->fs[k] = fs; s->fstot[k] = fstot;
      s->mdot[k] = mdot; s->phi[k] = phi; s->Ksol[k] = Ksol; s->Kliq[k] = Kliq;
      s->rho[k] = zeta(fstot, C, p->rho_s, p->rho_l, p->rho_g);
    }
}

/* -------------------------------------------------------- pass 2 */
/* Stencils, chemical potential, forces, collisions (O7-O15).  With
 * collide == 0 only the diagnostics (u, p, mu) are produced. */
static void pass2(orc_sim* s, int collide) {
  const orc_params* p = &s->p;
  const size_t n = s->n;
  const double Eref = p->rho_ref * cp_ref(p);
  const double tau_g = p->mobility / CS2 + 0.5; /* Mbar = c_s^2 (tau_g - 1/2), R11 */
  double heat_src = 0.0, phi_src = 0.0, reset = 0.0;
  double* row_acc = (double*)calloc((size_t)s->ny * 3, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int y = 0; y < s->ny; ++y) {
    double acc_heat = 0, acc_phi = 0, acc_reset = 0;
    for (int x = 0; x < s->nx; ++x) {
      size_t k = (size_t)y * s->nx + x;
      double phi = s->phi[k], rho = s->rho[k], C = s->C[k], fs = s->fs[k];
      double fstot = s->fstot[k], mdot = s->mdot[k], T = s->T[k];
      /* properties and relaxation times (Sec. 3.1-3.3; R5, R6) */
      double mu_v = zeta(fstot, C, p->mu_s, p->mu_l, p->mu_g);
      double lam = zeta(fstot, C, p->lam_s, p->lam_l, p->lam_g);
      double cp = zeta(fstot, C, p->cp_s, p->cp_l, p->cp_g);
      double tau_f = mu_v / rho / CS2 + 0.5;
      double tau_a = lam / Eref / CS2 + 0.5;
      double tau_s = 1.0 / (2.0 - 1.0 / tau_a); /* 1/tau_s + 1/tau_a = 2 */
      /* stencils (R15, R38) */
      double gphx, gphy, lphi, lfs, grx, gry, gpx, gpy;
      grad_lap(s, s->phi, x, y, &gphx, &gphy, &lphi);
      grad_lap(s, s->fs, x, y, NULL, NULL, &lfs);
      grad_lap(s, s->rho, x, y, &grx, &gry, NULL);
      grad_lap(s, s->p_prev, x, y, &gpx, &gpy, NULL); /* lagged pressure (R14) */
      double mu = chem_pot(p, phi, lphi, s->phi0[k], s->cth[k], s->lap_phi0[k], fs, lfs);
      /* surface tension F_s = mu grad phi; no body force (R32) */
      /* total force F = F_s + G with G = rho g (R32) */
      double Fx = mu * gphx + rho * p->grav[0], Fy = mu * gphy + rho * p->grav[1];
      double mx = 0, my = 0, sum_nz = 0;
      for (int i = 0; i < 9; ++i) {
        double fi = s->f[i * n + k];
        mx += CX[i] * fi;
        my += CY[i] * fi;
        if (i) sum_nz += fi;
      }
      /* rho u* = sum c f + F/2; drag f = f_s (u_s - u*) with u_s = 0; u = u* + f/2
       * (Sec. 3.1), with the total solid fraction in the drag (R2) */
      double usx = (mx + 0.5 * Fx) / rho, usy = (my + 0.5 * Fy) / rho;
      double fdx = fstot * (p->u_solid[0] - usx), fdy = fstot * (p->u_solid[1] - usy);
      double ux = usx + 0.5 * fdx, uy = usy + 0.5 * fdy;
      double S = rho * mdot + ux * grx + uy * gry;
      double Ftx = Fx - gpx + CS2 * grx, Fty = Fy - gpy + CS2 * gry; /* R10 */
      double uu = ux * ux + uy * uy;
      double F0 = W[0] * (S - (ux * Ftx + uy * Fty) / CS2);
      double s0 = W[0] * (-uu / (2 * CS2));
      double Fi[9], sr[9];
      orc_forcing(S, Fx, Fy, rho * fdx, rho * fdy, Ftx, Fty, ux, uy, Fi);
      /* the rest population's non-equilibrium part: (tau_f - 1/2) F_0, or
       * its moment-space form under MRT (R53) */
      double f0neq = (tau_f - 0.5) * F0;
      if (p->mrt) {
        mrt_rates(p, tau_f, sr);
        f0neq = mrt_f0neq(s->mrtM, s->mrtMinv, sr, Fi);
      }
      double pr = CS2 / (1.0 - W[0]) * (sum_nz + 0.5 * S + f0neq + rho * s0);
      s->ux[k] = ux; s->uy[k] = uy; s->pr[k] = pr; s->mu[k] = mu;
      if (!collide) continue;
      s->ux_new[k] = ux;
      s->uy_new[k] = uy;
      /* flow collision (Sec. 3.1; MRT: R53) */
      double feq[9], fin[9];
      orc_feq(pr, rho, ux, uy, feq);
      for (int i = 0; i < 9; ++i) fin[i] = s->f[i * n + k];
      if (p->mrt) {
        double fo[9];
        mrt_collide(s->mrtM, s->mrtMinv, sr, fin, feq, Fi, fo);
        for (int i = 0; i < 9; ++i) s->fc[i * n + k] = fo[i];
      } else {
        for (int i = 0; i < 9; ++i)
          s->fc[i * n + k] = fin[i] - (fin[i] - feq[i]) / tau_f + (1.0 - 0.5 / tau_f) * Fi[i];
      }
      /* phase-field collision (Sec. 3.2): G_i = w_i c.d_t(phi u)/c_s^2 +
       * w_i phi div u, with a backward difference in time (R13) */
      double jx = phi * ux, jy = phi * uy;
      double geq[9];
      orc_geq(phi, mu, jx, jy, geq);
      double djx = jx - s->phiux_prev[k], djy = jy - s->phiuy_prev[k];
      double Gv[9], gin[9];
      for (int i = 0; i < 9; ++i) {
        Gv[i] = W[i] * (CX[i] * djx + CY[i] * djy) / CS2 + W[i] * phi * s->divu[k];
        gin[i] = s->g[i * n + k];
      }
      if (p->mrt) {
        /* MRT (R53): the zeroth and first moments at 1/tau_g (the mobility),
         * the moments above first order at s_g */
        double sv = 1.0 / tau_g, sg = p->s_g > 0 ? p->s_g : sv;
        double srg[9] = {sv, sg, sg, sv, sg, sv, sg, sg, sg}, go[9];
        mrt_collide(s->mrtM, s->mrtMinv, srg, gin, geq, Gv, go);
        for (int i = 0; i < 9; ++i) s->gc[i * n + k] = go[i];
      } else {
        for (int i = 0; i < 9; ++i)
          s->gc[i * n + k] = gin[i] - (gin[i] - geq[i]) / tau_g + (1.0 - 0.5 / tau_g) * Gv[i];
      }
      /* enthalpy TRT collision (Sec. 3.3, eq22; R7, R8, R9) */
      double rhocp = rho * cp;
      double heq[9];
      orc_heq(s->rhoH[k], T, rhocp, Eref, ux, uy, heq);
      double Q = rhocp * T * mdot;
      double tau_src = p->h_src_tau_a ? tau_a : tau_s;
      double hsum = 0.0;
      for (int i = 0; i < 9; ++i) {
        int j = OPP[i];
        double hi = s->h[i * n + k], hj = s->h[j * n + k];
        double ha = 0.5 * (hi - hj), hs = 0.5 * (hi + hj);
        double ea = 0.5 * (heq[i] - heq[j]), es = 0.5 * (heq[i] + heq[j]);
        double v = hi - (ha - ea) / tau_a - (hs - es) / tau_s +
                   (1.0 - 0.5 / tau_src) * W[i] * Q;
        s->hc[i * n + k] = v;
        hsum += v;
      }
      /* expected energy gain of the collision, from the TRT moment algebra:
       * sum h* - sum h = (1/tau_s) Q_prev/2 + (1 - 1/(2 tau_src)) Q */
      acc_heat += 0.5 * s->Q_prev[k] / tau_s + (1.0 - 0.5 / tau_src) * Q;
      acc_phi += phi * s->divu[k];
      /* isothermal region (O14): the nodes with phi0 >= 1/2 at T_substrate
       * (R21), or a region given node by node with its own temperatures */
      int held = s->held_per_node ? !isnan(s->thold[k])
                                  : (p->substrate_fixed && s->phi0[k] >= 0.5);
      if (held) {
        double Tw = s->held_per_node ? s->thold[k] : p->T_substrate;
        double rH = enthalpy_at(p, Tw, s->Ksol[k], s->Kliq[k], s->chi[k]);
        double e[9], es = 0.0;
        orc_heq(rH, Tw, rhocp, Eref, 0.0, 0.0, e);
        for (int i = 0; i < 9; ++i) {
          es += e[i];
          s->hc[i * n + k] = e[i];
        }
        acc_reset += es - hsum;
      }
      /* lagged fields for the next step */
      s->fs_new[k] = fs;
      s->Q_new[k] = Q;
      s->phiux_new[k] = jx;
      s->phiuy_new[k] = jy;
      s->p_new[k] = pr;
    }
    row_acc[3 * y + 0] = acc_heat;
    row_acc[3 * y + 1] = acc_phi;
    row_acc[3 * y + 2] = acc_reset;
  }
  for (int y = 0; y < s->ny; ++y) {
    heat_src += row_acc[3 * y + 0];
    phi_src += row_acc[3 * y + 1];
    reset += row_acc[3 * y + 2];
  }
  free(row_acc);
  if (collide) {
    s->budget[0] = phi_src;
    s->budget[1] = heat_src;
    s->budget[3] = reset;
  }
}

/* -------------------------------------------------------- streaming */
/* O16: X_i(x, t+1) = X_i*(x - c_i).  Beyond a wall (half-way, R17):
 * f and g bounce back; h bounces back on an adiabatic wall and is
 * anti-bounced with 2 w_i rho_ref C_p,ref T_w on a Dirichlet wall.  A link
 * that leaves through a y-wall is handled by that wall (R42). */
static void stream(orc_sim* s) {
  const orc_params* p = &s->p;
  const size_t n = s->n;
  const double Eref = p->rho_ref * cp_ref(p);
  double* row_flux = (double*)calloc((size_t)s->ny, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int y = 0; y < s->ny; ++y) {
    double flux = 0.0;
    for (int x = 0; x < s->nx; ++x) {
      size_t k = (size_t)y * s->nx + x;
      for (int i = 0; i < 9; ++i) {
        int sx = x - CX[i], sy = y - CY[i];
        int wall = -1;
        if (sy < 0 || sy >= s->ny) {
          if (p->periodic_y) sy = (sy + s->ny) % s->ny;
          else wall = sy < 0 ? WB : WT;
        }
        if (wall < 0 && (sx < 0 || sx >= s->nx)) {
          if (p->periodic_x) sx = (sx + s->nx) % s->nx;
          else wall = sx < 0 ? WL : WR;
        }
        if (wall < 0) {
          size_t src = (size_t)sy * s->nx + sx;
          s->f[i * n + k] = s->fc[i * n + src];
          s->g[i * n + k] = s->gc[i * n + src];
          s->h[i * n + k] = s->hc[i * n + src];
        } else {
          int j = OPP[i];
          s->f[i * n + k] = s->fc[j * n + k];
          s->g[i * n + k] = s->gc[j * n + k];
          if (p->thermal_bc[wall]) {
            double Tw = s->wallT[wall][(wall == WB || wall == WT) ? x : y];
            double v = -s->hc[j * n + k] + 2.0 * W[i] * Eref * Tw;
            s->h[i * n + k] = v;
            flux += v - s->hc[j * n + k];
          } else {
            s->h[i * n + k] = s->hc[j * n + k];
          }
        }
      }
    }
    row_flux[y] = flux;
  }
  double flux = 0.0;
  for (int y = 0; y < s->ny; ++y) flux += row_flux[y];
  free(row_flux);
  s->budget[2] = flux;
}

static void swap_lagged(orc_sim* s) {
  double* t;
  t = s->fs_prev; s->fs_prev = s->fs_new; s->fs_new = t;
  t = s->Q_prev; s->Q_prev = s->Q_new; s->Q_new = t;
  t = s->phiux_prev; s->phiux_prev = s->phiux_new; s->phiux_new = t;
  t = s->phiuy_prev; s->phiuy_prev = s->phiuy_new; s->phiuy_new = t;
  t = s->p_prev; s->p_prev = s->p_new; s->p_new = t;
  t = s->ux_lag; s->ux_lag = s->ux_new; s->ux_new = t;
  t = s->uy_lag; s->uy_lag = s->uy_new; s->uy_new = t;
}

/* Conditioning probe (off by default): with store_f32 set, the state is
 * rounded to IEEE binary32 after every step while all arithmetic stays in
 * binary64.  The divergence from the unrounded run measures how much any
 * binary32-storage implementation must differ from this oracle. */
static void round_state_f32(orc_sim* s) {
  double* arrs[] = {s->f, s->g, s->h};
  for (int a = 0; a < 3; ++a)
    for (size_t k = 0; k < 9 * s->n; ++k) arrs[a][k] = (double)(float)arrs[a][k];
  double* lag[] = {s->fs_prev, s->Q_prev, s->phiux_prev, s->phiuy_prev, s->p_prev,
                   s->ux_lag, s->uy_lag};
  for (int a = 0; a < 7; ++a)
    for (size_t k = 0; k < s->n; ++k) lag[a][k] = (double)(float)lag[a][k];
}

void orc_set_store_f32(orc_sim* s, int on) { s->store_f32 = on; }

void orc_step(orc_sim* s, int nsteps) {
  for (int it = 0; it < nsteps; ++it) {
    pass1(s);
    pass2(s, 1);
    stream(s);
    swap_lagged(s);
    if (s->store_f32) round_state_f32(s);
    s->step++;
  }
}

/* --------------------------------------------------------- init */
/* Geometry: phi0 and the per-node wettability cos(theta); the static
 * Laplacian of phi0 uses the same stencil as every other field. */
static void set_geometry(orc_sim* s, const double* phi0, const double* cth) {
  memcpy(s->phi0, phi0, s->n * sizeof(double));
  memcpy(s->cth, cth, s->n * sizeof(double));
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x)
      grad_lap(s, s->phi0, x, y, NULL, NULL, &s->lap_phi0[(size_t)y * s->nx + x]);
}

/* Wall temperature profiles: bottom and top indexed by x, left and right by y. */
void orc_set_wall_T(orc_sim* s, int wall, const double* Tw) {
  memcpy(s->wallT[wall], Tw, (size_t)((wall == WB || wall == WT) ? s->nx : s->ny) *
                                 sizeof(double));
}

/* Per-node isothermal region: T[k] is the held temperature of node k, NaN
 * where the node is free; T = NULL goes back to the substrate_fixed rule. */
void orc_set_isothermal(orc_sim* s, const double* T) {
  if (!T) {
    s->held_per_node = 0;
    return;
  }
  memcpy(s->thold, T, s->n * sizeof(double));
  s->held_per_node = 1;
}

void orc_set_cos_theta(orc_sim* s, const double* cth) { memcpy(s->cth, cth, s->n * sizeof(double)); }

/* Initial state: u = 0, p = 0 (R29), so f = 0; g = g^eq(phi, mu_phi, 0);
 * h = h^eq(rho H, T, 0) with the PCM liquid (R27); lagged fields zero. */
int orc_init(orc_sim* s, const double* phi0, const double* cth, const double* phi,
             const double* T0) {
  const orc_params* p = &s->p;
  const size_t n = s->n;
  const double Eref = p->rho_ref * cp_ref(p);
  set_geometry(s, phi0, cth);
  memset(s->f, 0, 9 * n * sizeof(double));
  memset(s->fs_prev, 0, n * sizeof(double));
  memset(s->Q_prev, 0, n * sizeof(double));
  memset(s->phiux_prev, 0, n * sizeof(double));
  memset(s->phiuy_prev, 0, n * sizeof(double));
  memset(s->p_prev, 0, n * sizeof(double));
  memset(s->ux_lag, 0, n * sizeof(double));   /* u = 0 initially (R29) */
  memset(s->uy_lag, 0, n * sizeof(double));
  memcpy(s->phi, phi, n * sizeof(double));
  for (size_t k = 0; k < n; ++k) s->fs[k] = 0.0;
  for (int y = 0; y < s->ny; ++y)
    for (int x = 0; x < s->nx; ++x) {
      size_t k = (size_t)y * s->nx + x;
      double lphi;
      grad_lap(s, s->phi, x, y, NULL, NULL, &lphi);
      double mu = chem_pot(p, phi[k], lphi, phi0[k], cth[k], s->lap_phi0[k], 0.0, 0.0);
      double geq[9], heq[9];
      orc_geq(phi[k], mu, 0.0, 0.0, geq);
      double C = clampd(0.5 * (1.0 - phi0[k] + phi[k]), 0.0, 1.0);
      double Cp = clampd((C - p->pcm_floor) / (1.0 - p->pcm_floor), 0.0, 1.0);
      double chi = clampd(Cp, 0.0, 1.0 - phi0[k]);
      double Kliq = zeta(phi0[k], C, p->rho_s, p->rho_l, p->rho_g) *
                    zeta(phi0[k], C, p->cp_s, p->cp_l, p->cp_g);
      double rhoH = Kliq * (T0[k] - p->T_m) + Kliq * p->T_m + chi * p->rho_l * p->latent;
      orc_heq(rhoH, T0[k], 0.0, Eref, 0.0, 0.0, heq);
      for (int i = 0; i < 9; ++i) {
        s->g[i * n + k] = geq[i];
        s->h[i * n + k] = heq[i];
      }
    }
  memset(s->budget, 0, sizeof s->budget);
  s->step = 0;
  return 0;
}

/* ------------------------------------------------------- read-out */
/* Fields of the state at the current time, as the next step would see them:
 * 0 phi, 1 T, 2 liquid fraction 1 - f_s (R37, R41), 3 f_s, 4 u_x, 5 u_y, 6 p,
 * 7 rho H, 8 mu_phi, 9 C, 10 chi, 11 rho, 12 sum g. */
#define ORC_NFIELDS 13
int orc_nfields(void) { return ORC_NFIELDS; }

void orc_fields(orc_sim* s, double* out) {
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
    out[6 * n + k] = s->pr[k];
    out[7 * n + k] = s->rhoH[k];
    out[8 * n + k] = s->mu[k];
    out[9 * n + k] = s->C[k];
    out[10 * n + k] = s->chi[k];
    out[11 * n + k] = s->rho[k];
    out[12 * n + k] = s->phihat[k];
  }
}

/* Global sums (a12): 0 sum sum g, 1 sum sum h, 2 sum f_s, 3 sum (chi - f_s),
 * 4 max |u|, 5 non-finite count, 6..9 budget of the last step (sum phi div u,
 * heat source, wall flux, isothermal reset), 10 step count. */
#define ORC_NRED 11
int orc_nred(void) { return ORC_NRED; }

void orc_reduce(orc_sim* s, double* out) {
  pass1(s);
  pass2(s, 0);
  const size_t n = s->n;
  double sg = 0, sh = 0, sfs = 0, sliq = 0, umax = 0, bad = 0;
  for (size_t k = 0; k < n; ++k) {
    for (int i = 0; i < 9; ++i) {
      sg += s->g[i * n + k];
      sh += s->h[i * n + k];
    }
    sfs += s->fs[k];
    sliq += s->chi[k] - s->fs[k];
    double um = sqrt(s->ux[k] * s->ux[k] + s->uy[k] * s->uy[k]);
    if (um > umax) umax = um;
    if (!isfinite(s->phi[k]) || !isfinite(s->T[k]) || !isfinite(um) || !isfinite(s->pr[k]))
      bad += 1;
  }
  out[0] = sg; out[1] = sh; out[2] = sfs; out[3] = sliq; out[4] = umax; out[5] = bad;
  out[6] = s->budget[0]; out[7] = s->budget[1]; out[8] = s->budget[2]; out[9] = s->budget[3];
  out[10] = (double)s->step;
}

/* Raw post-stream distributions and lagged fields (test access). */
void orc_get_state(orc_sim* s, double* f, double* g, double* h, double* lag /* 7n */) {
  const size_t n = s->n;
  memcpy(f, s->f, 9 * n * sizeof(double));
  memcpy(g, s->g, 9 * n * sizeof(double));
  memcpy(h, s->h, 9 * n * sizeof(double));
  memcpy(lag + 0 * n, s->fs_prev, n * sizeof(double));
  memcpy(lag + 1 * n, s->Q_prev, n * sizeof(double));
  memcpy(lag + 2 * n, s->phiux_prev, n * sizeof(double));
  memcpy(lag + 3 * n, s->phiuy_prev, n * sizeof(double));
  memcpy(lag + 4 * n, s->p_prev, n * sizeof(double));
  memcpy(lag + 5 * n, s->ux_lag, n * sizeof(double));
  memcpy(lag + 6 * n, s->uy_lag, n * sizeof(double));
}

void orc_set_state(orc_sim* s, const double* f, const double* g, const double* h,
                   const double* lag) {
  const size_t n = s->n;
  memcpy(s->f, f, 9 * n * sizeof(double));
  memcpy(s->g, g, 9 * n * sizeof(double));
  memcpy(s->h, h, 9 * n * sizeof(double));
  memcpy(s->fs_prev, lag + 0 * n, n * sizeof(double));
  memcpy(s->Q_prev, lag + 1 * n, n * sizeof(double));
  memcpy(s->phiux_prev, lag + 2 * n, n * sizeof(double));
  memcpy(s->phiuy_prev, lag + 3 * n, n * sizeof(double));
  memcpy(s->p_prev, lag + 4 * n, n * sizeof(double));
  memcpy(s->ux_lag, lag + 5 * n, n * sizeof(double));
  memcpy(s->uy_lag, lag + 6 * n, n * sizeof(double));
}

long orc_step_count(orc_sim* s) { return s->step; }
