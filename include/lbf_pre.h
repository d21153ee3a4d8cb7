/*
 * liblbf, pre-processing: Cahn-Hilliard smoothing of a binary solid image
 * into the diffuse solid indicator phi0 (arXiv 2510.18688, Sec. 4.6: the
 * sandpack image is smoothed by a finite-time evolution of a standard
 * Cahn-Hilliard equation before the LB run; Sec. 2 gives the indicator's
 * interface profile 1/2 + 1/2 tanh(2 d / eps)).
 *
 * The equation is dc/dt = M lap(mu), mu = A (c^3 - c) - kappa lap(c), for
 * c = 2 s - 1 (s = 1 in the solid), stepped by explicit Euler steps of size
 * dt; phi0 = clamp((1 + c) / 2, 0, 1) at the end.  kappa = A eps^2 / 8 makes
 * the flat equilibrium c = tanh(2 d / eps).  lap is the lattice's isotropic
 * Laplacian 6 sum_i w_i (X(x + c_i) - X(x)): D2Q9 weights for a 2D image
 * (nz = 1), D3Q19 weights for a 3D one (Sec. 3.1); per axis a periodic wrap
 * or the mirror ghost (the first node repeated beyond a wall).  With either,
 * the sum of c is conserved.
 *
 * Layout: node (x, y, z) at (z * ny + y) * nx + x.  Returns LBF_OK or a
 * negative LBF_* code with the message in lbf_last_error().
 */
#ifndef LBF_PRE_H
#define LBF_PRE_H

#include <stddef.h>
#include <stdint.h>

#include "lbf.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbf_ch_params {
  int32_t nx, ny, nz;    /* image size; nz = 1 selects the 2D (D2Q9) stencil */
  int32_t periodic[3];   /* per axis (x, y, z): 1 periodic, 0 mirror walls */
  double A;              /* double-well height, >= 0 */
  double kappa;          /* gradient coefficient, >= 0 (A eps^2 / 8) */
  double mobility;       /* M >= 0 */
  double dt;             /* Euler step, > 0 */
} lbf_ch_params;

/* Device bytes of the workspace (two FP32 planes), 0 for invalid sizes
 * (a dimension below 1, or 2^31 nodes or more). */
size_t lbf_ch_workspace_bytes(int32_t nx, int32_t ny, int32_t nz);

/* Smooth the binary image `solid` (nx * ny * nz bytes, nonzero = solid) by
 * `iterations` Euler steps and write phi0 (nx * ny * nz floats).  `solid` and
 * `phi0` are host (*_on_device = 0, copied synchronously) or device memory.
 * `workspace`: caller-owned device memory of lbf_ch_workspace_bytes(), 256-byte
 * aligned, or NULL for a library allocation freed before return.  Ordered on
 * `stream` (NULL: the default stream); returns after the result is written
 * when either side is host memory.  LBF_EINVAL for bad sizes or coefficients
 * and for a step outside the explicit scheme's linear stability bound
 * dt M (16/3) (2 A + kappa 16/3) <= 2 (16/3 is the largest magnitude of the
 * lattice Laplacian's eigenvalues on both lattices). */
int lbf_ch_smooth(const lbf_ch_params* params, const uint8_t* solid, int32_t solid_on_device,
                  float* phi0, int32_t phi0_on_device, int32_t iterations, void* stream,
                  void* workspace, size_t workspace_bytes);

#ifdef __cplusplus
}
#endif
#endif
