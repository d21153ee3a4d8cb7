/*
 * liblbf — MI355X (gfx950) coupled lattice Boltzmann freezing step.
 *
 * The method is the diffuse-interface freezing model of Huang, Zhan, Chai and
 * Huang (arXiv 2510.18688): a pressure-based flow LB with surface tension, a
 * mass source and a solid drag (Sec. 3.1), a modified phase-field LB
 * (Sec. 3.2) and a total-enthalpy two-relaxation-time LB (Sec. 3.3, eq22)
 * coupled through the enthalpy map (Sec. 2, eq. Hfl), the mixing rule for
 * the properties (Sec. 2) and the chemical potential of the free energy eq44.
 * One call of lbf_step advances the coupled D2Q9 lattice by whole time steps.
 *
 * Conventions shared by every entry point:
 *  - A lattice has nx * ny nodes; node (x, y) of a 2D field is element
 *    y * nx + x (row-major, x fastest).  Walls sit half-way, at y = -1/2 and
 *    y = ny - 1/2 (and x = -1/2, x = nx - 1/2 when x is walled).
 *  - Float fields are IEEE binary32.  Host pointers are read or written
 *    synchronously; device pointers (on_device = 1) must be device memory
 *    valid on the stream the simulation was created with.
 *  - Every call returns LBF_OK (0) or a negative error code; the text of the
 *    last error of the calling thread is lbf_last_error().  No call throws.
 *  - Calls on one simulation are ordered on its HIP stream.  A simulation is
 *    used by one host thread at a time.
 */
#ifndef LBF_H
#define LBF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LBF_OK = 0,
  LBF_EINVAL = -1,    /* invalid argument or parameter set */
  LBF_EHIP = -2,      /* a HIP runtime call failed */
  LBF_ESTATE = -3,    /* call order: e.g. stepping before initialisation */
  LBF_EUNSTABLE = -4, /* non-finite values or |u| above the stability bound */
  LBF_ENOMEM = -5     /* workspace too small / allocation failed */
};

/* walls, in every per-wall array */
enum { LBF_WALL_BOTTOM = 0, LBF_WALL_TOP = 1, LBF_WALL_LEFT = 2, LBF_WALL_RIGHT = 3 };
enum { LBF_ADIABATIC = 0, LBF_DIRICHLET = 1 };

/* read-out fields of lbf_read_field, all at the current time level */
enum {
  LBF_FIELD_PHI = 0,    /* order parameter phi (Sec. 3.2 recovery) */
  LBF_FIELD_T = 1,      /* temperature (enthalpy map, Hfl) */
  LBF_FIELD_FL = 2,     /* liquid fraction 1 - f_s at node level */
  LBF_FIELD_FS = 3,     /* ice volume fraction f_s */
  LBF_FIELD_UX = 4,     /* velocity u (Sec. 3.1 recovery, drag included) */
  LBF_FIELD_UY = 5,
  LBF_FIELD_P = 6,      /* pressure (Sec. 3.1 recovery) */
  LBF_FIELD_RHOH = 7,   /* total enthalpy rho H */
  LBF_FIELD_MU = 8,     /* chemical potential mu_phi (eq44 derivative) */
  LBF_FIELD_C = 9,      /* liquid weight (1 - phi0 + phi_hat)/2, clamped */
  LBF_FIELD_CHI = 10,   /* phase-change fraction of the node */
  LBF_FIELD_RHO = 11,   /* density from the mixing rule */
  LBF_FIELD_PHIHAT = 12,/* zeroth moment sum_i g_i */
  LBF_NFIELDS = 13
};

/* entries of lbf_reduce's output (FP64, fixed-order reduction) */
enum {
  LBF_RED_SUM_G = 0,     /* sum over nodes and directions of g_i */
  LBF_RED_SUM_H = 1,     /* sum of h_i (total energy) */
  LBF_RED_SUM_FS = 2,    /* ice volume */
  LBF_RED_SUM_LIQ = 3,   /* liquid PCM volume sum (chi - f_s) */
  LBF_RED_UMAX = 4,      /* max |u| */
  LBF_RED_NONFINITE = 5, /* count of nodes with a non-finite phi, T, u or p */
  LBF_RED_SRC_PHI = 6,   /* last step: sum phi * mdot (phase-field source) */
  LBF_RED_SRC_HEAT = 7,  /* last step: heat source of the TRT collision */
  LBF_RED_WALL_FLUX = 8, /* last step: energy entering through Dirichlet walls */
  LBF_RED_RESET = 9,     /* last step: energy change of isothermal-region resets */
  LBF_RED_STEP = 10,     /* steps taken since initialisation */
  LBF_NRED = 11
};

/* Physical and lattice parameters (lattice units, dx = dt = 1).
 * Properties of the three phases enter the mixing rule of Sec. 2; the
 * relaxation times follow from them as in Sec. 3.1-3.3. */
typedef struct lbf_params {
  int32_t nx, ny;              /* lattice size, each >= 1 */
  int32_t periodic_x;          /* 1 periodic, 0 walls at x = -1/2, nx - 1/2 */
  int32_t periodic_y;          /* 1 periodic, 0 walls at y = -1/2, ny - 1/2 */
  int32_t thermal_bc[4];       /* per wall: LBF_ADIABATIC or LBF_DIRICHLET */
  int32_t latch_fs;            /* 1: PCM fraction latched by the previous ice fraction */
  int32_t h_src_tau_a;         /* 1: enthalpy source prefactor with tau_a, 0: tau_s */
  int32_t substrate_fixed;     /* 1: nodes with phi0 >= 1/2 held at T_substrate */
  int32_t plane_pad;           /* extra floats between consecutive planes of the
                                  workspace, a multiple of 64 in [0, 65536]: moves
                                  which HBM channels the planes of one step share
                                  (a tuning knob; results do not depend on it) */
  double rho_l, rho_g, rho_s;  /* densities */
  double mu_l, mu_g, mu_s;     /* dynamic viscosities */
  double lam_l, lam_g, lam_s;  /* thermal conductivities */
  double cp_l, cp_g, cp_s;     /* specific heats */
  double latent, T_m;          /* latent heat, melting temperature */
  double sigma, eps;           /* surface tension, interface width */
  double mobility;             /* Cahn-Hilliard mobility Mbar */
  double cos_psi;              /* cosine of the water-ice contact angle */
  double rho_ref;              /* reference density of the enthalpy LB */
  double T_substrate;          /* temperature of held solid nodes */
  double pcm_floor;            /* liquid weight below which a node holds no phase-change
                                  material, in [0, 1) (0.01 keeps gas fluctuations from
                                  freezing) */
  /* Flow and phase-field collisions (Sec. 3.1 and 3.2 use BGK and name MRT
   * as the extension): 0 BGK; 1 MRT in the orthogonal D2Q9 moment basis
   * (density, energy e, energy square epsilon, momentum j, energy flux q,
   * stresses p_xx, p_xy) with the source terms applied in moment space.  f:
   * j and the stresses at the viscous rate 1/tau_f, density, e and epsilon at
   * the bulk rate s_b, q at s_q.  g: the zeroth and first moments at 1/tau_g
   * (the mobility), the moments above first order at s_g.  A rate of 0
   * stands for the BGK rate (mrt = 1 with all three 0 is BGK).  Rates in
   * [0, 2).  The adjoint (lbf_tape_*) supports BGK only. */
  int32_t mrt;
  /* Stability check of lbf_step: with check_every = k > 0, every step that
   * starts at a time level divisible by k also forms the FP64 reduction of
   * the state it reads, and lbf_step returns LBF_EUNSTABLE right after that
   * step (which has run) when the state held a non-finite phi, T, u or p or
   * max |u| > 0.3.  Each check waits for the stream once.  0: no checks
   * (lbf_step stays fully asynchronous). */
  int32_t check_every;
  /* div u in the source phi div u of the phase-field equation and in the
   * recovery phi = sum g + phi div u / 2 (Sec. 3.2): 0 (default) the
   * isotropic divergence of the previous step's velocity, the flow's own
   * divergence, which keeps the bulk phi at its equilibrium value where the
   * discrete flow is not exactly divergence free: a drop freezing on a cold
   * wall, a drop dewetting a cylinder or a porous medium over thousands of
   * steps at a gas/liquid density ratio of 0.1 need it to stay stable; it
   * stores the previous step's velocity and phi in place of (phi u) (one
   * more lagged plane, 8 more bytes per node update).  1: the model's mass
   * source mdot of eq1 (sum phi changes by exactly sum phi mdot; stable only
   * over shorter runs).  The adjoint (lbf_tape_*) supports 1 only. */
  int32_t phi_src_mdot;
  /* Memory layout of the state (a tuning knob; results do not depend on it).
   * 0: plane-major, each plane's nx * ny nodes back to back.  1, 2, 4, 8, 16
   * or 32: row blocks of that many rows, each block holding its rows of every
   * distribution and lagged plane (and of every static plane) back to back,
   * so the planes one step touches at a time lie close together in HBM;
   * plane_pad then pads each block's planes.  The adjoint (lbf_tape_*)
   * supports 0 only.  Row blocks cap a lattice at about 29.8 M nodes. */
  int32_t row_block;
  double s_b, s_q, s_g;
  /* Body force G = rho * grav (a uniform acceleration acting on the local
   * density) and the solid-phase velocity u_s of the drag f_s (u_s - u*)
   * (Sec. 3.1); zero in the paper's droplet cases.  Finite.  The adjoint
   * supports zero values only. */
  double grav[2];
  double u_solid[2];
} lbf_params;

typedef struct lbf_sim lbf_sim;

/* Bytes of device workspace one simulation needs (distributions, lagged
 * fields, static fields, reduction scratch) for lattice nx x ny,
 * lbf_params.plane_pad and lbf_params.row_block, or 0 for invalid sizes,
 * pads or row blocks. */
size_t lbf_workspace_bytes(int32_t nx, int32_t ny, int32_t plane_pad, int32_t row_block);

/* Create a simulation on HIP stream `stream` (a hipStream_t, NULL for the
 * default stream).  `workspace` is caller-owned device memory of at least
 * lbf_workspace_bytes(nx, ny, plane_pad, row_block) bytes, 256-byte aligned, that must outlive the
 * simulation; with workspace == NULL the library allocates it with hipMalloc
 * and frees it in lbf_destroy.  Rejects with LBF_EINVAL: non-positive sizes,
 * non-positive densities, specific heats, viscosities or conductivities,
 * eps <= 0, mobility <= 0, a plane_pad outside its range, and rho_ref C_p,ref
 * larger than the smallest possible nodal heat capacity (the enthalpy scheme
 * is then unstable). */
int lbf_create(const lbf_params* params, void* stream, void* workspace, size_t workspace_bytes,
               lbf_sim** out);

/* Geometry: the diffuse solid label phi0 in [0, 1] (Sec. 2, Omega_0) and the
 * per-node cosine of the contact angle theta (eq44), nx * ny floats each.
 * The static Laplacian of phi0 is computed on the device. */
int lbf_set_geometry(lbf_sim* sim, const float* phi0, const float* cos_theta, int32_t on_device);

/* Isothermal region given node by node: every node whose mask byte is
 * nonzero is held at its own temperature T_hold[k] -- after each collision
 * its enthalpy populations are reset to the equilibrium, at rest, of the
 * enthalpy that the enthalpy map (Sec. 2, eq. Hfl) inverts to that
 * temperature (frozen phase-change material at or below T_m, liquid above).
 * This generalises the cold substrate of Sec. 4.4, which substrate_fixed
 * gives as the nodes with phi0 >= 1/2 at T_substrate, and replaces that rule
 * while it is set.  mask (nx * ny bytes) and T_hold (nx * ny floats) are
 * both host or both device memory; mask = NULL removes the per-node region
 * (substrate_fixed's rule applies again).  The region survives
 * lbf_set_geometry and lbf_init_fields.  The adjoint (lbf_tape_*) refuses a
 * simulation with a per-node region. */
int lbf_set_isothermal(lbf_sim* sim, const uint8_t* mask, const float* T_hold, int32_t on_device);

/* Temperature profile of one wall, used by its anti-bounce-back rule when the
 * wall is LBF_DIRICHLET: n = nx floats for bottom/top (indexed by x),
 * n = ny floats for left/right (indexed by y). */
int lbf_set_wall_temperature(lbf_sim* sim, int32_t wall, const float* Tw, int32_t n,
                             int32_t on_device);

/* Initial state from the order parameter phi and temperature T (nx * ny
 * each): u = 0, p = 0, phase-field and enthalpy distributions at
 * equilibrium, the phase-change material liquid.  Requires the geometry. */
int lbf_init_fields(lbf_sim* sim, const float* phi, const float* T, int32_t on_device);

/* Replace the state by an externally given one at time level `step`: the
 * post-streaming distributions (27 planes of nx * ny floats: f_0..f_8,
 * g_0..g_8, h_0..h_8, the populations each node holds at the start of a
 * step) and the lagged fields of the previous step (7 planes: f_s,
 * rho C_p T mdot, (phi u)_x, (phi u)_y, p, u_x, u_y).  Geometry and wall
 * temperatures must be set; they define the wall links that the state is
 * mapped through. */
int lbf_set_poststream_state(lbf_sim* sim, const float* dist, const float* lag, int64_t step,
                             int32_t on_device);

/* Advance nsteps coupled time steps (nsteps >= 0).  Asynchronous on the
 * simulation's stream, except for the stability checks that
 * lbf_params.check_every asks for: LBF_EUNSTABLE (message naming the time
 * level) when one fails; the steps up to and including the checking step
 * have then been taken and the simulation's step count says so. */
int lbf_step(lbf_sim* sim, int32_t nsteps);

/* Compute one read-out field (LBF_FIELD_*) of the current state into dst
 * (nx * ny floats, host or device). */
int lbf_read_field(lbf_sim* sim, int32_t field_id, float* dst, int32_t dst_on_device);

/* Compute every read-out field into dst (LBF_NFIELDS * nx * ny floats,
 * field-major). */
int lbf_read_fields(lbf_sim* sim, float* dst, int32_t dst_on_device);

/* FP64 global sums of the current state and the budget of the last step
 * (LBF_RED_*), written to host memory out[LBF_NRED].  Synchronises the
 * stream.  Returns LBF_EUNSTABLE (after filling out) if a node is
 * non-finite or max |u| exceeds 0.3. */
int lbf_reduce(lbf_sim* sim, double* out);

/* Column and row profiles of the current state, the reductions behind the
 * freezing observables: front height and final solid height (Sec. 4.2,
 * Table 1), drop height on a curved substrate (Sec. 4.4), radius and height
 * of the three-phase contact line (Fig. 6), solid fraction against the
 * Fourier number (Fig. 13).  FP64 sums of the FP32 fields in a fixed order
 * (deterministic).  col[LBF_NCOL * nx] (profile-major, indexed by x):
 *   LBF_COL_ICE      sum over y of the ice fraction f_s;
 *   LBF_COL_PCM      sum over y of the phase-change fraction chi (liquid and
 *                    ice of the phase-change material);
 *   LBF_COL_PCM_TOP  highest y at which chi crosses 1/2 from above (linear
 *                    interpolation between rows y and y + 1; ny - 1 when the
 *                    top row is at or above 1/2; -1 when no node is);
 *   LBF_COL_ICE_TOP  the same for f_s (the freezing front of the column).
 * row[LBF_NROW * ny] (indexed by y):
 *   LBF_ROW_ICE, LBF_ROW_PCM  sums over x of f_s and of chi;
 *   LBF_ROW_PCM_LEFT / _RIGHT the outermost 1/2-crossings of chi in the row:
 *                    the leftmost rise and the rightmost fall (linear
 *                    interpolation; the edge node itself when it is at or
 *                    above 1/2; -1 when no node is);
 *   LBF_ROW_ICE_LEFT / _RIGHT the same for f_s.
 * Rows and columns are ordered bottom to top and left to right whether or
 * not the axis is periodic.  dst_on_device selects device or host outputs;
 * synchronises the stream. */
enum { LBF_COL_ICE = 0, LBF_COL_PCM = 1, LBF_COL_PCM_TOP = 2, LBF_COL_ICE_TOP = 3, LBF_NCOL = 4 };
enum {
  LBF_ROW_ICE = 0, LBF_ROW_PCM = 1, LBF_ROW_PCM_LEFT = 2, LBF_ROW_PCM_RIGHT = 3,
  LBF_ROW_ICE_LEFT = 4, LBF_ROW_ICE_RIGHT = 5, LBF_NROW = 6
};
int lbf_profiles(lbf_sim* sim, double* col, double* row, int32_t dst_on_device);

/* Launch shape of the step kernel: threads per block along x (64, 128, 256,
 * 512) and rows per block along y (>= 1).  Defaults are chosen at creation. */
int lbf_set_tile(lbf_sim* sim, int32_t tile_x, int32_t tile_y);
int lbf_get_tile(const lbf_sim* sim, int32_t* tile_x, int32_t* tile_y);

/* Bytes of the checkpointable dynamic state and copy of it to / from `buf`
 * (device memory).  The buffer holds each plane's nx * ny values back to
 * back, so a state loads into any simulation of the same lattice size
 * whatever its plane_pad and row_block.  A loaded state continues
 * bit-identically. */
size_t lbf_state_bytes(const lbf_sim* sim);
int lbf_save_state(lbf_sim* sim, void* dst_device, size_t cap);
int lbf_load_state(lbf_sim* sim, const void* src_device, size_t bytes);

/* Average duration in milliseconds of the step kernel over the launches of
 * the last lbf_step call, from HIP events on the simulation's stream (0 if
 * timing is off).  lbf_set_timing(sim, 1) brackets each launch with events. */
int lbf_set_timing(lbf_sim* sim, int32_t on);
double lbf_last_step_kernel_ms(const lbf_sim* sim);

/* Measurement aid (no passage of the paper defines it): the HBM ceiling of
 * the step kernel's own access pattern.  Runs `launches` launches of a kernel
 * that, with the simulation's tile shape, tile order and row order, copies
 * every plane a step reads to the plane it writes (the 27 distributions and
 * the lagged planes in use) and reads the static planes the step reads, with
 * no arithmetic.  The copies go to the buffers the next step overwrites, so
 * the simulation's state is unchanged.  On success *ms_per_launch receives
 * the average launch duration (HIP events on the simulation's stream; the
 * call waits for them) and *bytes_per_launch the bytes one launch moves.
 * LBF_ESTATE before the state is set, LBF_EINVAL for launches < 1 or NULL
 * outputs. */
int lbf_copy_probe(lbf_sim* sim, int32_t launches, double* ms_per_launch,
                   double* bytes_per_launch);

const char* lbf_last_error(void);
void lbf_destroy(lbf_sim* sim);

/* ---- batches: many lattices advanced by one persistent launch per step ----
 * A batch groups n initialised simulations that share one HIP stream (the
 * simulations stay owned by the caller and must outlive the batch).  Each
 * step is one launch of a fixed grid (as many workgroups as fit on the device at once) that
 * walks the work list of every lattice's tiles; runs of 32 steps are
 * captured once in a HIP graph and replayed.  Every lattice is advanced
 * exactly as lbf_step would advance it (same arithmetic, bit-identical
 * states).  Budget tracking (the step budget entries of lbf_reduce) is not
 * kept for batched steps. */
typedef struct lbf_batch lbf_batch;

/* Rejects (LBF_EINVAL) empty batches, NULL or repeated simulations and
 * simulations on different streams; LBF_ESTATE if one is not initialised. */
int lbf_batch_create(lbf_sim* const* sims, int32_t n, lbf_batch** out);

/* Tile shape shared by every lattice of the batch (tile_x in {64, 128, 256},
 * 1 <= tile_y <= 256); the default is 128 x 32. */
int lbf_batch_set_tile(lbf_batch* batch, int32_t tile_x, int32_t tile_y);

/* Advance every lattice of the batch by nsteps (asynchronous unless timing
 * is on).  A simulation stepped on its own in between is picked up at its
 * current state; LBF_ESTATE if a simulation has lost its state since (new
 * geometry without lbf_init_fields or a loaded state). */
int lbf_batch_step(lbf_batch* batch, int32_t nsteps);

/* With timing on, lbf_batch_step brackets its launches with HIP events and
 * lbf_batch_last_step_ms returns the average milliseconds per step. */
int lbf_batch_set_timing(lbf_batch* batch, int32_t on);
double lbf_batch_last_step_ms(const lbf_batch* batch);

/* Number of (lattice, tile) work items of the current tile shape (0 before
 * the first step). */
int32_t lbf_batch_items(const lbf_batch* batch);

void lbf_batch_destroy(lbf_batch* batch);

/* ---- reverse-mode differentiation (adjoint with checkpoint recomputation) ----
 * A tape records a forward run of nsteps steps of one simulation and then
 * returns the exact gradient of a scalar J of the final state's phi, T and
 * f_s (the caller supplies dJ/dphi, dJ/dT, dJ/df_s per node) with respect to
 * the per-node cos(theta) of the wetting term (eq44) and the Dirichlet wall
 * temperatures of the anti-bounce-back rule.  This is the discrete adjoint
 * of the coupled step (an extension beyond the paper): each step is reversed
 * exactly, in FP32, with FP64 gradient accumulation; at non-smooth points
 * (clamps, the phase-change latch maximum, the enthalpy-map branches) it
 * takes the one-sided derivative of the branch the forward evaluated, a
 * clamp passing the derivative on its closed interval and a tie of the
 * maximum splitting it evenly.  When the recorded run starts from
 * lbf_init_fields (step 0), the dependence of the initial phase-field
 * equilibrium on cos(theta) is included; otherwise the starting state is
 * held fixed.  The wall temperatures and geometry must not change between
 * the forward run and the backward sweep. */
typedef struct lbf_tape lbf_tape;

/* Device bytes a tape allocates: ceil(nsteps / segment) stored states of
 * 34 planes, two buffers of `segment` recomputed states and their moments
 * (one segment is recomputed on a second stream while the other is
 * reversed), and the adjoint work planes, all with the simulation's plane
 * stride (its plane_pad; the tape needs row_block 0).  segment <= 0 selects
 * ceil(sqrt(nsteps)). */
size_t lbf_tape_bytes(int32_t nx, int32_t ny, int32_t plane_pad, int32_t nsteps,
                      int32_t segment);

/* Create a tape for `sim` (which must outlive it) recording nsteps >= 0
 * steps with a checkpoint every `segment` steps (<= 0: ceil(sqrt(nsteps))).
 * The tape owns its device memory (hipMalloc; LBF_ENOMEM on failure) and a
 * private non-blocking stream of default priority for the recomputation. */
int lbf_tape_create(lbf_sim* sim, int32_t nsteps, int32_t segment, lbf_tape** out);

/* The checkpoint interval in use. */
int lbf_tape_segment(const lbf_tape* tape);

/* Advance the simulation by the tape's nsteps, storing its state every
 * segment steps (asynchronous on the simulation's stream). */
int lbf_tape_forward(lbf_tape* tape);

/* Reverse sweep after lbf_tape_forward, with the simulation still at the
 * final state (LBF_ESTATE otherwise).  seed_phi, seed_T, seed_fs: dJ/d field
 * at every node of the final state (nx * ny floats each, host or device per
 * seeds_on_device; NULL means zero).  Outputs (host or device per
 * grads_on_device, FP64): grad_cos_theta[nx * ny] = dJ/dcos(theta) per node;
 * grad_wall_T[2 nx + 2 ny] = dJ/dT_w per wall node, bottom (nx, by x), top
 * (nx), left (ny, by y), right (ny); zero on adiabatic walls.  Each segment
 * is recomputed once from its checkpoint.  Synchronises the stream. */
int lbf_tape_backward(lbf_tape* tape, const float* seed_phi, const float* seed_T,
                      const float* seed_fs, int32_t seeds_on_device, double* grad_cos_theta,
                      double* grad_wall_T, int32_t grads_on_device);

void lbf_tape_destroy(lbf_tape* tape);

#ifdef __cplusplus
}
#endif
#endif
