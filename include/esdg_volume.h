/*
 * esdg_volume.h -- C ABI of the volume-kernel cost comparison of Section 5.4 (Wu, Kubatko &
 * Chan, arXiv 2005.02516): the volume term of a traditional DG scheme against the
 * entropy-stable (flux-differencing) volume term, for random square matrices of size n as
 * in the paper, with the shallow-water fluxes of Section 2.8:
 *
 *   traditional     r[c][k][m] = sum_j Qx[m][j] f^x_c(u_kj) + Qy[m][j] f^y_c(u_kj)
 *   entropy-stable  r[c][k][m] = sum_j 2 (Qx[m][j] f^x_{S,c}(u_km, u_kj) + Qy[m][j] f^y_{S,c}(u_km, u_kj))
 *
 * f the physical flux, f_S the entropy-conservative two-point flux (arithmetic averages,
 * p = g {h}^2 - g {h^2} / 2).  Part of libesdg_swe; status codes from esdg_swe.h.
 */
#ifndef ESDG_VOLUME_H
#define ESDG_VOLUME_H

#include <stdint.h>

#include "esdg_swe.h"

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ESDG_VOLUME_TRADITIONAL = 0,    /* matrix-vector product with the flux at each node      */
  ESDG_VOLUME_ENTROPY_STABLE = 1  /* Hadamard product with the two-point flux, row sums    */
};

/* Evaluate one volume term for K elements of n nodes on the GPU, asynchronously on
 * hip_stream (a hipStream_t; NULL = the default stream).
 *   kind       ESDG_VOLUME_TRADITIONAL | ESDG_VOLUME_ENTROPY_STABLE
 *   precision  ESDG_FP64 | ESDG_FP32: the type of every array below
 *   QxT, QyT   device, [n][n]: the matrices transposed, QxT[j*n + m] = Qx[m][j]
 *   u          device, [3][K][n]: h, hu, hv at the nodes (h > 0)
 *   r          device, [3][K][n]: the result (must not overlap the inputs)
 *   n          nodes per element, 1 <= n <= 256;  K >= 1 elements;  g > 0
 * The caller owns every array.  Returns ESDG_EINVAL for a bad argument (nothing launched)
 * and ESDG_EDEVICE if the launch fails. */
esdg_status esdg_volume_kernel(int32_t kind, int32_t precision, const void *QxT, const void *QyT, const void *u,
                               void *r, int32_t n, int32_t K, double g, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* ESDG_VOLUME_H */
