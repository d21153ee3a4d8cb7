/*
 * liblbf, three-dimensional lattice: the coupled freezing step of
 * arXiv 2510.18688 on the D3Q19 lattice (Sec. 3.1 gives the nineteen
 * velocities and weights; the flow, phase-field and enthalpy schemes of
 * Sec. 3.1-3.3 are written for vectors of any dimension).
 *
 * Conventions as in lbf.h: a lattice has nx * ny * nz nodes; node (x, y, z)
 * of a 3D field is element (z * ny + y) * nx + x.  Faces, in every per-face
 * array: 0 x-low, 1 x-high, 2 y-low, 3 y-high, 4 z-low, 5 z-high; walls sit
 * half-way outside the first and last node.  Float fields are IEEE binary32;
 * every call returns LBF_OK or a negative LBF_* code with the message in
 * lbf_last_error(); calls are ordered on the simulation's HIP stream.
 *
 * Differences from the two-dimensional entry points: a Dirichlet face takes
 * one temperature (set in the parameters); a link that leaves through
 * several walls takes the z face, else the y face, else the x face; the step
 * budget entries of the reduction are not tracked.
 */
#ifndef LBF3_H
#define LBF3_H

#include <stddef.h>
#include <stdint.h>

#include "lbf.h"

#ifdef __cplusplus
extern "C" {
#endif

/* read-out fields of lbf3_read_fields, field-major */
enum {
  LBF3_FIELD_PHI = 0, LBF3_FIELD_T, LBF3_FIELD_FL, LBF3_FIELD_FS, LBF3_FIELD_UX,
  LBF3_FIELD_UY, LBF3_FIELD_UZ, LBF3_FIELD_P, LBF3_FIELD_RHOH, LBF3_FIELD_MU,
  LBF3_FIELD_C, LBF3_FIELD_CHI, LBF3_FIELD_RHO, LBF3_FIELD_PHIHAT, LBF3_NFIELDS
};

typedef struct lbf3_params {
  int32_t nx, ny, nz;          /* lattice size, each >= 1 */
  int32_t periodic[3];         /* per axis: 1 periodic, 0 walls */
  int32_t thermal_bc[6];       /* per face: LBF_ADIABATIC or LBF_DIRICHLET */
  int32_t latch_fs, h_src_tau_a, substrate_fixed;
  int32_t plane_pad;           /* extra floats between consecutive planes, a
                                  multiple of 64 in [0, 65536]; as in lbf_params
                                  (layout only, results do not depend on it) */
  double rho_l, rho_g, rho_s;
  double mu_l, mu_g, mu_s;
  double lam_l, lam_g, lam_s;
  double cp_l, cp_g, cp_s;
  double latent, T_m;
  double sigma, eps;
  double mobility;
  double cos_psi;
  double rho_ref;
  double T_substrate;
  double pcm_floor;
  double wall_T[6];            /* temperature of each Dirichlet face */
  double grav[3];              /* body force G = rho * grav, as in lbf_params */
  double u_solid[3];           /* solid-phase velocity of the drag */
  int32_t phi_src_mdot;        /* div u in the phase-field source and recovery, as
                                  in lbf_params: 0 (default) the isotropic divergence
                                  of the previous step's velocity (three more lagged
                                  planes and one plane from the moments pass), which
                                  the fracture set-up needs over its 20 000 steps;
                                  1 the mass source mdot of eq1 */
  int32_t row_block;           /* memory layout of the state (a tuning knob; results
                                  do not depend on it): 0 plane-major; 1, 2, 4, 8,
                                  16, 32 or 64 rows of nx nodes (row z ny + y) per
                                  block, each block holding its rows of every plane
                                  of the f, g, h, lagged and static arrays, so the
                                  planes one pass streams lie close together in HBM;
                                  plane_pad then pads each block's planes.  Row
                                  blocks cap a lattice at about 33 M nodes */
} lbf3_params;

typedef struct lbf3_sim lbf3_sim;

/* Device bytes of one simulation's workspace with lbf3_params.plane_pad and
 * lbf3_params.row_block, 0 for invalid sizes, pads or row blocks and for
 * lattices above the addressing limit of their layout. */
size_t lbf3_workspace_bytes(int32_t nx, int32_t ny, int32_t nz, int32_t plane_pad,
                            int32_t row_block);

/* Create on HIP stream `stream` (NULL: default stream); workspace as in
 * lbf_create (caller-owned, 256-byte aligned, or NULL for a library
 * allocation).  LBF_EINVAL for the parameter sets lbf_create rejects and
 * for lattices above the 56.5 M-node addressing limit. */
int lbf3_create(const lbf3_params* params, void* stream, void* workspace,
                size_t workspace_bytes, lbf3_sim** out);

/* phi0 and cos(theta), nx * ny * nz floats each; lap(phi0) is computed. */
int lbf3_set_geometry(lbf3_sim* sim, const float* phi0, const float* cos_theta,
                      int32_t on_device);

/* Initial state from phi and T (u = 0, p = 0, equilibria, PCM liquid). */
int lbf3_init_fields(lbf3_sim* sim, const float* phi, const float* T, int32_t on_device);

/* Advance nsteps steps (two kernels per step: moments, then the step). */
int lbf3_step(lbf3_sim* sim, int32_t nsteps);

/* Every read-out field (LBF3_NFIELDS * nx * ny * nz floats, field-major). */
int lbf3_read_fields(lbf3_sim* sim, float* dst, int32_t dst_on_device);

/* FP64 sums in lbf.h's LBF_RED_* order: sum g, sum h, sum f_s, sum of the
 * liquid PCM, max |u|, non-finite count; entries 6-9 (step budget) are 0;
 * step count.  Returns LBF_EUNSTABLE (after filling out) like lbf_reduce. */
int lbf3_reduce(lbf3_sim* sim, double* out);

/* Bytes of the checkpointable dynamic state (distributions, lagged fields,
 * step count) and its copy to / from `buf` (device memory, at least
 * lbf3_state_bytes).  The buffer holds each plane's nodes back to back, so a
 * state loads into any simulation of the same lattice size whatever its
 * plane_pad and row_block.  Loading needs the geometry set and a state of the same lattice
 * size (LBF_EINVAL otherwise); a loaded state continues bit-identically.
 * Synchronises the simulation's stream. */
size_t lbf3_state_bytes(const lbf3_sim* sim);
int lbf3_save_state(lbf3_sim* sim, void* dst_device, size_t cap);
int lbf3_load_state(lbf3_sim* sim, const void* src_device, size_t bytes);

/* Node order of the step kernel: strips of `rows` rows (default 16), each
 * walked slab by slab in z, so a node's z neighbours were read shortly
 * before (rows >= ny: the x-fastest order).  The same arithmetic per node:
 * the fields do not depend on it.  LBF_EINVAL for rows < 1. */
int lbf3_set_strip(lbf3_sim* sim, int32_t rows);

/* HIP-event timing of the step kernels: average milliseconds per step of
 * the last lbf3_step call (0 if timing is off). */
int lbf3_set_timing(lbf3_sim* sim, int32_t on);
double lbf3_last_step_ms(const lbf3_sim* sim);

void lbf3_destroy(lbf3_sim* sim);

#ifdef __cplusplus
}
#endif
#endif
