/* Volume-kernel cost comparison of Section 5.4: plain C versions of the two volume terms
 * for the CPU side of the cost ratio.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of oracle/: only tests and bench.py load it.
 * Straightforward loops, FP64, one element after another, as a serial CPU code would
 * compute them (not tuned).  Definitions (u, r: [3][K][n]; Qx, Qy: [n][n] row-major):
 *   traditional     r[c][k][m] = sum_n Qx[m][n] f^x_c(u_kn) + Qy[m][n] f^y_c(u_kn)
 *   entropy-stable  r[c][k][m] = sum_n 2 (Qx[m][n] f^x_{S,c}(u_km, u_kn) + Qy[m][n] f^y_{S,c}(u_km, u_kn))
 * with the shallow-water physical flux and the entropy-conservative flux of Section 2.8. */
#include <stdlib.h>

void dg_volume_c(int n, int K, const double *Qx, const double *Qy, const double *u, double g, double *r) {
  const size_t plane = (size_t)K * n;
  double *f = (double *)malloc(sizeof(double) * 6 * (size_t)n);
  for (int k = 0; k < K; ++k) {
    const double *h = u + (size_t)k * n, *hu = h + plane, *hv = hu + plane;
    for (int j = 0; j < n; ++j) {         /* physical flux at every node */
      const double uu = hu[j] / h[j], vv = hv[j] / h[j], p = 0.5 * g * h[j] * h[j];
      f[6 * j + 0] = hu[j];
      f[6 * j + 1] = hu[j] * uu + p;
      f[6 * j + 2] = hu[j] * vv;
      f[6 * j + 3] = hv[j];
      f[6 * j + 4] = hv[j] * uu;
      f[6 * j + 5] = hv[j] * vv + p;
    }
    for (int m = 0; m < n; ++m) {
      double a0 = 0, a1 = 0, a2 = 0;
      for (int j = 0; j < n; ++j) {
        const double qx = Qx[(size_t)m * n + j], qy = Qy[(size_t)m * n + j];
        a0 += qx * f[6 * j + 0] + qy * f[6 * j + 3];
        a1 += qx * f[6 * j + 1] + qy * f[6 * j + 4];
        a2 += qx * f[6 * j + 2] + qy * f[6 * j + 5];
      }
      r[(size_t)k * n + m] = a0;
      r[plane + (size_t)k * n + m] = a1;
      r[2 * plane + (size_t)k * n + m] = a2;
    }
  }
  free(f);
}

void esdg_volume_c(int n, int K, const double *Qx, const double *Qy, const double *u, double g, double *r) {
  const size_t plane = (size_t)K * n;
  for (int k = 0; k < K; ++k) {
    const double *h = u + (size_t)k * n, *hu = h + plane, *hv = hu + plane;
    for (int m = 0; m < n; ++m) {
      const double um = hu[m] / h[m], vm = hv[m] / h[m];
      double a0 = 0, a1 = 0, a2 = 0;
      for (int j = 0; j < n; ++j) {
        const double uj = hu[j] / h[j], vj = hv[j] / h[j];
        const double havg = 0.5 * (h[m] + h[j]), h2avg = 0.5 * (h[m] * h[m] + h[j] * h[j]);
        const double huavg = 0.5 * (hu[m] + hu[j]), hvavg = 0.5 * (hv[m] + hv[j]);
        const double uavg = 0.5 * (um + uj), vavg = 0.5 * (vm + vj);
        const double p = g * havg * havg - 0.5 * g * h2avg;
        const double qx = Qx[(size_t)m * n + j], qy = Qy[(size_t)m * n + j];
        a0 += qx * huavg + qy * hvavg;
        a1 += qx * (huavg * uavg + p) + qy * (hvavg * uavg);
        a2 += qx * (huavg * vavg) + qy * (hvavg * vavg + p);
      }
      r[(size_t)k * n + m] = 2.0 * a0;
      r[plane + (size_t)k * n + m] = 2.0 * a1;
      r[2 * plane + (size_t)k * n + m] = 2.0 * a2;
    }
  }
}
