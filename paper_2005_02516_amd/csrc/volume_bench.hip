// Volume-kernel cost comparison of Section 5.4: the volume term of a traditional DG scheme
// (a matrix-vector product with the flux evaluated once per node) against the
// entropy-stable one (flux differencing: the Hadamard product of the matrix with the
// two-point entropy-conservative fluxes between every pair of nodes, summed along rows),
// for random square matrices of size n as in the paper, with the shallow-water fluxes of
// Section 2.8.  Both kernels share one structure, so their time ratio is the cost of the
// flux-differencing arithmetic:
//
//   * a workgroup takes `groups` row groups of n threads; group i owns kVolElems elements
//     and each thread one row m of those elements;
//   * the elements' node data are staged once in LDS (six values per node);
//   * each matrix entry is read once per thread from the transposed matrices (coalesced
//     across the rows of a group, shared by the groups through the L1) and applied to
//     kVolElems elements from registers.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "esdg_volume.h"

namespace esdg {

constexpr int kVolBlock = 256;
constexpr int kVolElems = 4;          // elements per thread (each matrix entry read once for 4)
constexpr int kVolNodeVals = 6;       // staged values per node

// Node data in LDS.  Traditional: the physical fluxes f^x (3) and f^y (3) at the node.
// Entropy-stable: h, hu, hv, u, v, h^2.
template <typename real, bool ESDG>
__device__ __forceinline__ void stage_node(real h, real hu, real hv, real g, real *s) {
  const real uu = hu / h, vv = hv / h;
  if constexpr (ESDG) {
    s[0] = h; s[1] = hu; s[2] = hv; s[3] = uu; s[4] = vv; s[5] = h * h;
  } else {
    const real p = real(0.5) * g * h * h;
    s[0] = hu; s[1] = hu * uu + p; s[2] = hu * vv;
    s[3] = hv; s[4] = hv * uu; s[5] = hv * vv + p;
  }
}

template <typename real, bool ESDG>
__global__ void __launch_bounds__(kVolBlock) volume_kernel(const real *__restrict__ QxT, const real *__restrict__ QyT,
                                                            const real *__restrict__ u, real *__restrict__ r, int n,
                                                            int K, int groups, real g) {
  extern __shared__ __align__(16) unsigned char vol_smem[];
  real *S = reinterpret_cast<real *>(vol_smem);
  const int epb = groups * kVolElems;
  const long long k0 = (long long)blockIdx.x * epb;
  const int ne = int(K - k0 < epb ? K - k0 : epb);
  const size_t plane = size_t(K) * n;
  for (int i = threadIdx.x; i < ne * n; i += blockDim.x) {
    const size_t o = size_t(k0) * n + i;
    stage_node<real, ESDG>(u[o], u[plane + o], u[2 * plane + o], g, S + size_t(i) * kVolNodeVals);
  }
  __syncthreads();
  const int gi = int(threadIdx.x) / n, m = int(threadIdx.x) - gi * n;
  const int e0 = gi * kVolElems;
  if (gi >= groups || e0 >= ne) return;
  const int nb = ne - e0 < kVolElems ? ne - e0 : kVolElems;
  real acc[kVolElems][3];
  real own[kVolElems][kVolNodeVals];
#pragma unroll
  for (int b = 0; b < kVolElems; ++b) {
    acc[b][0] = acc[b][1] = acc[b][2] = real(0);
#pragma unroll
    for (int v = 0; v < kVolNodeVals; ++v)
      own[b][v] = b < nb ? S[(size_t(e0 + b) * n + m) * kVolNodeVals + v] : real(1);
  }
  const real half_g = real(0.5) * g;
  for (int j = 0; j < n; ++j) {
    const real qx = QxT[size_t(j) * n + m], qy = QyT[size_t(j) * n + m];
#pragma unroll
    for (int b = 0; b < kVolElems; ++b) {
      if (b >= nb) break;
      const real *s = S + (size_t(e0 + b) * n + j) * kVolNodeVals;
      if constexpr (ESDG) {
        const real havg = real(0.5) * (own[b][0] + s[0]), h2avg = real(0.5) * (own[b][5] + s[5]);
        const real huavg = real(0.5) * (own[b][1] + s[1]), hvavg = real(0.5) * (own[b][2] + s[2]);
        const real uavg = real(0.5) * (own[b][3] + s[3]), vavg = real(0.5) * (own[b][4] + s[4]);
        const real p = g * havg * havg - half_g * h2avg;
        acc[b][0] += qx * huavg + qy * hvavg;
        acc[b][1] += qx * (huavg * uavg + p) + qy * (hvavg * uavg);
        acc[b][2] += qx * (huavg * vavg) + qy * (hvavg * vavg + p);
      } else {
        acc[b][0] += qx * s[0] + qy * s[3];
        acc[b][1] += qx * s[1] + qy * s[4];
        acc[b][2] += qx * s[2] + qy * s[5];
      }
    }
  }
#pragma unroll
  for (int b = 0; b < kVolElems; ++b) {
    if (b >= nb) break;
    const size_t o = size_t(k0 + e0 + b) * n + m;
    const real w = ESDG ? real(2) : real(1);
    r[o] = w * acc[b][0];
    r[plane + o] = w * acc[b][1];
    r[2 * plane + o] = w * acc[b][2];
  }
}

// Host launcher: kind 0 traditional, 1 entropy-stable; 1 <= n <= kVolBlock.
hipError_t launch_volume(int kind, bool fp64, const void *QxT, const void *QyT, const void *u, void *r, int n, int K,
                         double g, hipStream_t stream) {
  const int groups = kVolBlock / n;              // >= 1 for n <= kVolBlock
  const int epb = groups * kVolElems;
  const int grid = int((K + (long long)epb - 1) / epb);
  const size_t lds = size_t(epb) * n * kVolNodeVals * (fp64 ? 8 : 4);
  if (fp64) {
    if (kind)
      hipLaunchKernelGGL((volume_kernel<double, true>), dim3(grid), dim3(kVolBlock), lds, stream,
                         static_cast<const double *>(QxT), static_cast<const double *>(QyT),
                         static_cast<const double *>(u), static_cast<double *>(r), n, K, groups, g);
    else
      hipLaunchKernelGGL((volume_kernel<double, false>), dim3(grid), dim3(kVolBlock), lds, stream,
                         static_cast<const double *>(QxT), static_cast<const double *>(QyT),
                         static_cast<const double *>(u), static_cast<double *>(r), n, K, groups, g);
  } else {
    if (kind)
      hipLaunchKernelGGL((volume_kernel<float, true>), dim3(grid), dim3(kVolBlock), lds, stream,
                         static_cast<const float *>(QxT), static_cast<const float *>(QyT),
                         static_cast<const float *>(u), static_cast<float *>(r), n, K, groups, float(g));
    else
      hipLaunchKernelGGL((volume_kernel<float, false>), dim3(grid), dim3(kVolBlock), lds, stream,
                         static_cast<const float *>(QxT), static_cast<const float *>(QyT),
                         static_cast<const float *>(u), static_cast<float *>(r), n, K, groups, float(g));
  }
  return hipGetLastError();
}

}  // namespace esdg

extern "C" esdg_status esdg_volume_kernel(int32_t kind, int32_t precision, const void *QxT, const void *QyT,
                                          const void *u, void *r, int32_t n, int32_t K, double g, void *hip_stream) {
  if ((kind != ESDG_VOLUME_TRADITIONAL && kind != ESDG_VOLUME_ENTROPY_STABLE) ||
      (precision != ESDG_FP64 && precision != ESDG_FP32) || !QxT || !QyT || !u || !r || n < 1 ||
      n > esdg::kVolBlock || K < 1 || !(g > 0.0))
    return ESDG_EINVAL;
  const hipError_t e = esdg::launch_volume(kind, precision == ESDG_FP64, QxT, QyT, u, r, n, K, g,
                                           static_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? ESDG_OK : ESDG_EDEVICE;
}
