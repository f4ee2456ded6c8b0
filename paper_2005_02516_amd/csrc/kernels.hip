// HIP kernels (gfx950) for one RK stage of the modal ESDG shallow-water scheme.
//
// One workgroup processes a tile of consecutive elements of one instance.  Per tile:
//   1. node records of the entropy-projected state u~ (Section 2.5) and the J-scaled
//      metrics at the Nh hybridized nodes are staged in LDS;
//   2. flux differencing in skew form (Section 5.2, Step 4): for every row m and every
//      column n of the nonzero blocks of Q_skew = Q_h - Q_h^T (volume-volume and
//      volume-surface; the surface-surface block is zero and skipped), with the
//      element's physical operator built on the fly from averaged geometric factors
//      (Section 2.6) and the EC flux of Section 2.7.  The bathymetry source is folded
//      into the pair term as 1/2 g h_m (H_n - Href) Q_mn, exact because Q_h 1 = 0;
//   3. the interface flux f_S(u~+, u~) on face rows with the neighbour's values gathered
//      through mapP, the boundary half of the source, and the optional Lax-Friedrichs
//      penalty (Section 2.8);
//   4. lift: rhs = -(M_h^k)^{-1} V_h^T r_h (Section 2.7, stored inverses);
//   5. LSRK update (Section 4) and, fused, the entropy projection of the updated state
//      for the next stage (element-local), written to the other stage buffer.
// The launch boundary is the grid-wide barrier the neighbour gather needs.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device_types.hpp"

namespace esdg {

template <typename real>
__device__ inline bool bad_value(double h, double a, double b) {
  return !(h > 0.0) || !isfinite(h) || !isfinite(a) || !isfinite(b);
}

// Entropy projection of the element states held in sA ([3][ne][Np], modal) to the
// hybridized nodes, written to ut[3+1 planes] at out (Section 2.5):
//   u_q = V_q u_h; v_q = v(u_q) (FP64); v_h = Minv_k V_q^T diag(w J) v_q; v~ = V_h v_h;
//   u~ = u(v~) (FP64) stored as h~, v~2 (= u~), v~3 (= v~), H~ - Href.
template <typename real, int N>
__device__ void project_tile(const InstDesc &d, int k0, int ne, const real *sVh, real *sA, real *sB, real *sQ,
                             real *out, int32_t *flag) {
  constexpr int Np = dim_Np(N), Nq = dim_Nq(N), Nh = dim_Nh(N);
  const int K = d.K;
  const double g = d.g;
  const real *wJq = static_cast<const real *>(d.wJq);
  const real *Minv = static_cast<const real *>(d.Minv);
  const int tid = threadIdx.x, nth = blockDim.x;
  bool bad = false;
  for (int i = tid; i < ne * Nq; i += nth) {
    const int e = i / Nq, q = i - e * Nq, k = k0 + e;
    real u0 = 0, u1 = 0, u2 = 0;
#pragma unroll 4
    for (int j = 0; j < Np; ++j) {
      const real v = sVh[q * Np + j];
      u0 += v * sA[0 * ne * Np + e * Np + j];
      u1 += v * sA[1 * ne * Np + e * Np + j];
      u2 += v * sA[2 * ne * Np + e * Np + j];
    }
    const double h = u0, hu = u1, hv = u2;
    const double uu = hu / h, vv = hv / h;
    const double v1 = g * (h + d.bq[size_t(k) * Nq + q]) - 0.5 * (uu * uu + vv * vv);
    const double w = wJq[size_t(k) * Nq + q];
    sQ[0 * ne * Nq + i] = real(w * v1);
    sQ[1 * ne * Nq + i] = real(w * uu);
    sQ[2 * ne * Nq + i] = real(w * vv);
    bad |= bad_value<real>(h, hu, hv);
  }
  __syncthreads();
  for (int i = tid; i < ne * Np; i += nth) {
    const int e = i / Np, j = i - e * Np;
    real y0 = 0, y1 = 0, y2 = 0;
#pragma unroll 4
    for (int q = 0; q < Nq; ++q) {
      const real v = sVh[q * Np + j];
      y0 += v * sQ[0 * ne * Nq + e * Nq + q];
      y1 += v * sQ[1 * ne * Nq + e * Nq + q];
      y2 += v * sQ[2 * ne * Nq + e * Nq + q];
    }
    sB[0 * ne * Np + i] = y0;
    sB[1 * ne * Np + i] = y1;
    sB[2 * ne * Np + i] = y2;
  }
  __syncthreads();
  for (int i = tid; i < ne * Np; i += nth) {
    const int e = i / Np, row = i - e * Np, k = k0 + e;
    const real *Mi = Minv + (size_t(k) * Np + row) * Np;
    real v0 = 0, v1 = 0, v2 = 0;
#pragma unroll 4
    for (int j = 0; j < Np; ++j) {
      const real m = Mi[j];
      v0 += m * sB[0 * ne * Np + e * Np + j];
      v1 += m * sB[1 * ne * Np + e * Np + j];
      v2 += m * sB[2 * ne * Np + e * Np + j];
    }
    sA[0 * ne * Np + i] = v0;
    sA[1 * ne * Np + i] = v1;
    sA[2 * ne * Np + i] = v2;
  }
  __syncthreads();
  const size_t plane = size_t(K) * Nh;
  for (int i = tid; i < ne * Nh; i += nth) {
    const int e = i / Nh, n = i - e * Nh, k = k0 + e;
    real t0 = 0, t1 = 0, t2 = 0;
#pragma unroll 4
    for (int j = 0; j < Np; ++j) {
      const real v = sVh[n * Np + j];
      t0 += v * sA[0 * ne * Np + e * Np + j];
      t1 += v * sA[1 * ne * Np + e * Np + j];
      t2 += v * sA[2 * ne * Np + e * Np + j];
    }
    const double v1 = t0, v2 = t1, v3 = t2;
    const double H = (v1 + 0.5 * (v2 * v2 + v3 * v3)) / g;
    const double h = H - d.bh[size_t(k) * Nh + n];
    const size_t o = size_t(k) * Nh + n;
    out[0 * plane + o] = real(h);
    out[1 * plane + o] = real(v2);
    out[2 * plane + o] = real(v3);
    out[3 * plane + o] = real(H - d.Href);
    bad |= bad_value<real>(h, v2, v3);
  }
  if (bad) atomicOr(flag, 1);
}

// Flux differencing + interface flux + lift for one tile; then either write rhs or do
// the LSRK update and project the updated state.
template <typename real, int N>
__device__ void volume_tile(const StageArgs &a, const InstDesc &d, int k0, int ne, real *sm) {
  constexpr int Np = dim_Np(N), Nq = dim_Nq(N), Nfq = dim_Nfq(N), Nh = dim_Nh(N);
  const int K = d.K;
  const int tid = threadIdx.x, nth = blockDim.x;
  const real g = real(d.g);
  const real *sVh = sm;
  const real *sSr = sVh + Nh * Np;
  const real *sSs = sSr + Nq * Nh;
  const real *sF = sSs + Nq * Nh;
  real *sNode = sm + ref_words(N);
  real *sR = sNode + ne * Nh * kNodeRec;
  real *sA = sR + 3 * ne * Nh;
  real *sB = sA + 3 * ne * Np;
  const size_t plane = size_t(K) * Nh;
  const real *ut = static_cast<const real *>(d.ut[a.in_buf]);
  const real *geo = static_cast<const real *>(d.geo);

  for (int i = tid; i < ne * Nh; i += nth) {
    const int e = i / Nh, n = i - e * Nh;
    const size_t o = size_t(k0 + e) * Nh + n;
    const real h = ut[o], u = ut[plane + o], v = ut[2 * plane + o], dH = ut[3 * plane + o];
    real *rec = sNode + i * kNodeRec;
    rec[0] = real(0.5) * h * u;
    rec[1] = real(0.5) * h * v;
    rec[2] = real(0.5) * u;
    rec[3] = real(0.5) * v;
    rec[4] = real(0.5) * g * h;
    rec[5] = dH;
    rec[6] = geo[o];
    rec[7] = geo[plane + o];
    rec[8] = geo[2 * plane + o];
    rec[9] = geo[3 * plane + o];
    rec[10] = h;
  }
  __syncthreads();

  // volume rows: every column n != m (volume-volume and volume-surface blocks)
  for (int i = tid; i < ne * Nq; i += nth) {
    const int e = i / Nq, m = i - e * Nq;
    const real *rm = sNode + (e * Nh + m) * kNodeRec;
    const real hum = rm[0], hvm = rm[1], um = rm[2], vm = rm[3], ghm = rm[4];
    const real rxm = rm[6], sxm = rm[7], rym = rm[8], sym = rm[9];
    real acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll 2
    for (int n = 0; n < Nh; ++n) {
      if (n == m) continue;
      const real *rn = sNode + (e * Nh + n) * kNodeRec;
      const real Sr = sSr[m * Nh + n], Ss = sSs[m * Nh + n];
      const real Qx = (rxm + rn[6]) * Sr + (sxm + rn[7]) * Ss;
      const real Qy = (rym + rn[8]) * Sr + (sym + rn[9]) * Ss;
      const real c = Qx * (hum + rn[0]) + Qy * (hvm + rn[1]);
      const real t = ghm * rn[5];
      acc0 += c;
      acc1 += (um + rn[2]) * c + t * Qx;
      acc2 += (vm + rn[3]) * c + t * Qy;
    }
    sR[0 * ne * Nh + e * Nh + m] = acc0;
    sR[1 * ne * Nh + e * Nh + m] = acc1;
    sR[2 * ne * Nh + e * Nh + m] = acc2;
  }

  // face rows: volume columns (the surface-surface block is zero) + interface flux
  const int32_t *mapP = d.mapP;
  for (int i = tid; i < ne * Nfq; i += nth) {
    const int e = i / Nfq, f = i - e * Nfq, m = Nq + f, k = k0 + e;
    const real *rm = sNode + (e * Nh + m) * kNodeRec;
    const real hum = rm[0], hvm = rm[1], um = rm[2], vm = rm[3], ghm = rm[4];
    const real rxm = rm[6], sxm = rm[7], rym = rm[8], sym = rm[9];
    real acc0 = 0, acc1 = 0, acc2 = 0;
#pragma unroll 2
    for (int n = 0; n < Nq; ++n) {
      const real *rn = sNode + (e * Nh + n) * kNodeRec;
      const real Sr = -sSr[n * Nh + m], Ss = -sSs[n * Nh + m];
      const real Qx = (rxm + rn[6]) * Sr + (sxm + rn[7]) * Ss;
      const real Qy = (rym + rn[8]) * Sr + (sym + rn[9]) * Ss;
      const real c = Qx * (hum + rn[0]) + Qy * (hvm + rn[1]);
      const real t = ghm * rn[5];
      acc0 += c;
      acc1 += (um + rn[2]) * c + t * Qx;
      acc2 += (vm + rn[3]) * c + t * Qy;
    }
    // interface: W_f [ nJ . f_S(u~, u~+) + 1/2 g h (H+ - Href) nJ ] - LF
    const real wf = sF[f], nr = sF[Nfq + f], ns = sF[2 * Nfq + f];
    const real nJx = rxm * nr + sxm * ns, nJy = rym * nr + sym * ns;
    const real h = rm[10], u = real(2) * um, v = real(2) * vm, dH = rm[5];
    const real hu = real(2) * hum, hv = real(2) * hvm;
    const int32_t p = mapP[size_t(k) * Nfq + f];
    const real hP = ut[p], uP = ut[plane + p], vP = ut[2 * plane + p], dHP = ut[3 * plane + p];
    const real huP = hP * uP, hvP = hP * vP;
    const real hua = real(0.5) * (hu + huP), hva = real(0.5) * (hv + hvP);
    const real ua = real(0.5) * (u + uP), va = real(0.5) * (v + vP);
    const real pr = ghm * dHP;
    real f0 = nJx * hua + nJy * hva;
    real f1 = nJx * (hua * ua + pr) + nJy * hva * ua;
    real f2 = nJx * hua * va + nJy * (hva * va + pr);
    if (d.flux == 1) {
      const real sJ = sqrt(nJx * nJx + nJy * nJy);
      const real lm = fabs(u * nJx + v * nJy) + sqrt(g * h) * sJ;
      const real lp = fabs(uP * nJx + vP * nJy) + sqrt(g * hP) * sJ;
      const real c = real(0.5) * fmax(lm, lp);
      f0 -= c * (dHP - dH);
      f1 -= c * (huP - hu);
      f2 -= c * (hvP - hv);
    }
    sR[0 * ne * Nh + e * Nh + m] = acc0 + wf * f0;
    sR[1 * ne * Nh + e * Nh + m] = acc1 + wf * f1;
    sR[2 * ne * Nh + e * Nh + m] = acc2 + wf * f2;
  }
  __syncthreads();

  // lift: y = V_h^T r_h
  for (int i = tid; i < ne * Np; i += nth) {
    const int e = i / Np, j = i - e * Np;
    real y0 = 0, y1 = 0, y2 = 0;
#pragma unroll 4
    for (int n = 0; n < Nh; ++n) {
      const real v = sVh[n * Np + j];
      y0 += v * sR[0 * ne * Nh + e * Nh + n];
      y1 += v * sR[1 * ne * Nh + e * Nh + n];
      y2 += v * sR[2 * ne * Nh + e * Nh + n];
    }
    sB[0 * ne * Np + i] = y0;
    sB[1 * ne * Np + i] = y1;
    sB[2 * ne * Np + i] = y2;
  }
  __syncthreads();

  // rhs = -Minv y; then either store it or do the LSRK update
  const real *Minv = static_cast<const real *>(d.Minv);
  const size_t splane = size_t(K) * Np;
  real *uh = static_cast<real *>(d.uh);
  real *du = static_cast<real *>(d.du);
  real *rhs_out = static_cast<real *>(a.ext_rhs);
  const real ra = real(a.rk_a), rdt = real(d.dt), rb = real(a.rk_b);
  for (int i = tid; i < ne * Np; i += nth) {
    const int e = i / Np, row = i - e * Np, k = k0 + e;
    const real *Mi = Minv + (size_t(k) * Np + row) * Np;
    real r0 = 0, r1 = 0, r2 = 0;
#pragma unroll 4
    for (int j = 0; j < Np; ++j) {
      const real mm = Mi[j];
      r0 -= mm * sB[0 * ne * Np + e * Np + j];
      r1 -= mm * sB[1 * ne * Np + e * Np + j];
      r2 -= mm * sB[2 * ne * Np + e * Np + j];
    }
    const size_t o = size_t(k) * Np + row;
    if (a.mode == kRhs) {
      rhs_out[o] = r0;
      rhs_out[splane + o] = r1;
      rhs_out[2 * splane + o] = r2;
    } else {
      const real rr[3] = {r0, r1, r2};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const size_t oc = c * splane + o;
        const real dn = ra * du[oc] + rdt * rr[c];
        const real un = uh[oc] + rb * dn;
        du[oc] = dn;
        uh[oc] = un;
        sA[c * ne * Np + i] = un;
      }
    }
  }
  if (a.mode == kStage) {
    __syncthreads();
    project_tile<real, N>(d, k0, ne, sVh, sA, sB, sNode, static_cast<real *>(d.ut[a.out_buf]), a.flag);
  }
}

template <typename real, int N>
__device__ void process_tile(const StageArgs &a, const InstDesc &d, int k0, int ne, real *sm) {
  constexpr int words = ref_words(N);
  const real *ref = static_cast<const real *>(d.ref);
  for (int i = threadIdx.x; i < words; i += blockDim.x) sm[i] = ref[i];
  if (a.mode == kProject) {
    constexpr int Np = dim_Np(N), Nh = dim_Nh(N);
    real *sNode = sm + words;
    real *sA = sNode + ne * Nh * kNodeRec + 3 * ne * Nh;
    real *sB = sA + 3 * ne * Np;
    const real *src = static_cast<const real *>(a.ext_state ? a.ext_state : d.uh);
    const size_t splane = size_t(d.K) * Np;
    for (int i = threadIdx.x; i < 3 * ne * Np; i += blockDim.x) {
      const int c = i / (ne * Np), r = i - c * ne * Np;
      sA[i] = src[c * splane + size_t(k0) * Np + r];
    }
    __syncthreads();
    project_tile<real, N>(d, k0, ne, sm, sA, sB, sNode, static_cast<real *>(d.ut[a.out_buf]), a.flag);
  } else {
    __syncthreads();
    volume_tile<real, N>(a, d, k0, ne, sm);
  }
}

template <typename real>
__global__ void __launch_bounds__(kBlock, 4) stage_kernel(StageArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  real *sm = reinterpret_cast<real *>(smem_raw);
  for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
    const Tile tl = a.tiles[t];
    const InstDesc &d = a.desc[tl.inst];
    switch (d.N) {
      case 1: process_tile<real, 1>(a, d, tl.k0, tl.ne, sm); break;
      case 2: process_tile<real, 2>(a, d, tl.k0, tl.ne, sm); break;
      case 3: process_tile<real, 3>(a, d, tl.k0, tl.ne, sm); break;
      case 4: process_tile<real, 4>(a, d, tl.k0, tl.ne, sm); break;
      case 5: process_tile<real, 5>(a, d, tl.k0, tl.ne, sm); break;
      default: break;
    }
    __syncthreads();
  }
}

// FP64 diagnostics per tile: mass (3), entropy, entropy rate, sum |entropy-rate terms|.
template <typename real, int N>
__device__ void diag_tile(const InstDesc &d, int k0, int ne, double *acc) {
  constexpr int Np = dim_Np(N), Nq = dim_Nq(N);
  const real *ref = static_cast<const real *>(d.ref);   // Vh rows 0..Nq-1 are V_q
  const real *uh = static_cast<const real *>(d.uh);
  const real *rh = static_cast<const real *>(d.rhs_scratch);
  const real *wJq = static_cast<const real *>(d.wJq);
  const size_t splane = size_t(d.K) * Np;
  const double g = d.g;
  for (int i = threadIdx.x; i < ne * Nq; i += blockDim.x) {
    const int e = i / Nq, q = i - e * Nq, k = k0 + e;
    double u[3] = {0, 0, 0}, r[3] = {0, 0, 0};
    for (int j = 0; j < Np; ++j) {
      const double v = ref[q * Np + j];
      for (int c = 0; c < 3; ++c) {
        u[c] += v * double(uh[c * splane + size_t(k) * Np + j]);
        r[c] += v * double(rh[c * splane + size_t(k) * Np + j]);
      }
    }
    const double w = wJq[size_t(k) * Nq + q], b = d.bq[size_t(k) * Nq + q];
    const double h = u[0], uu = u[1] / h, vv = u[2] / h;
    acc[0] += w * u[0];
    acc[1] += w * u[1];
    acc[2] += w * u[2];
    acc[3] += w * (0.5 * h * (uu * uu + vv * vv) + 0.5 * g * h * h + g * h * b);
    const double t0 = w * (g * (h + b) - 0.5 * (uu * uu + vv * vv)) * r[0];
    const double t1 = w * uu * r[1], t2 = w * vv * r[2];
    acc[4] += t0 + t1 + t2;
    acc[5] += fabs(t0) + fabs(t1) + fabs(t2);
  }
}

template <typename real>
__global__ void __launch_bounds__(kBlock) diag_kernel(DiagArgs a) {
  __shared__ double red[kBlock][6];
  const int t = blockIdx.x;
  if (t >= a.ntiles) return;
  const Tile tl = a.tiles[t];
  const InstDesc &d = a.desc[tl.inst];
  double acc[6] = {0, 0, 0, 0, 0, 0};
  switch (d.N) {
    case 1: diag_tile<real, 1>(d, tl.k0, tl.ne, acc); break;
    case 2: diag_tile<real, 2>(d, tl.k0, tl.ne, acc); break;
    case 3: diag_tile<real, 3>(d, tl.k0, tl.ne, acc); break;
    case 4: diag_tile<real, 4>(d, tl.k0, tl.ne, acc); break;
    case 5: diag_tile<real, 5>(d, tl.k0, tl.ne, acc); break;
    default: break;
  }
  for (int c = 0; c < 6; ++c) red[threadIdx.x][c] = acc[c];
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (int(threadIdx.x) < s)
      for (int c = 0; c < 6; ++c) red[threadIdx.x][c] += red[threadIdx.x + s][c];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 6; ++c) a.partials[size_t(t) * 6 + c] = red[0][c];
}

// ---------------------------------------------------------------- host launchers

hipError_t set_stage_lds_limit(bool fp64, size_t lds_bytes) {
  const void *fn = fp64 ? reinterpret_cast<const void *>(&stage_kernel<double>)
                        : reinterpret_cast<const void *>(&stage_kernel<float>);
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
}

hipError_t launch_stage(bool fp64, const StageArgs &a, int grid, size_t lds_bytes, hipStream_t stream) {
  if (grid <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(stage_kernel<double>, dim3(grid), dim3(kBlock), lds_bytes, stream, a);
  else
    hipLaunchKernelGGL(stage_kernel<float>, dim3(grid), dim3(kBlock), lds_bytes, stream, a);
  return hipGetLastError();
}

hipError_t launch_diag(bool fp64, const DiagArgs &a, hipStream_t stream) {
  if (a.ntiles <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(diag_kernel<double>, dim3(a.ntiles), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(diag_kernel<float>, dim3(a.ntiles), dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

}  // namespace esdg
