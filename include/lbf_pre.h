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

/* Largest image (nx * ny * nz nodes) that lbf_ch_smooth_noalloc accepts:
 * 2^22 = 4 194 304 nodes (a 2048 x 2048 or 160^3 image). */
size_t lbf_ch_noalloc_max_nodes(void);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * smoothing as lbf_ch_smooth, with the same kernels and bit-identical
 * results, that calls no hipMalloc, hipFree or other allocating routine.
 * Its two planes of c live in a library-held device array of
 * 2 * lbf_ch_noalloc_max_nodes() floats (32 MiB), one per device, which each
 * device that the library runs on holds until the process ends; the array
 * of the current device (hipGetDevice) is used, so `stream` must belong to
 * that device.  `solid_dev` (nx * ny * nz bytes) and `phi0_dev`
 * (nx * ny * nz floats) are device memory owned by the caller.  Nothing in
 * the array needs to start at zero (the first kernel writes every node the
 * others read).  The call is ordered on `stream` (NULL: the default stream)
 * and returns without waiting for it.  Every call on one device shares that
 * device's array: calls that overlap on one device (on different streams, or
 * from several threads without ordering) race and must be serialised by the
 * caller.  LBF_EINVAL as for lbf_ch_smooth, for NULL buffers, and for images
 * of more than lbf_ch_noalloc_max_nodes() nodes; LBF_EHIP when the array's
 * device address cannot be obtained. */
int lbf_ch_smooth_noalloc(const lbf_ch_params* params, const uint8_t* solid_dev, float* phi0_dev,
                          int32_t iterations, void* stream);

#ifdef __cplusplus
}
#endif
#endif
