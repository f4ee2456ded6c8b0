// HIP kernels (gfx950) for the RK stages of the modal ESDG shallow-water scheme.
//
// One workgroup processes a tile of consecutive elements of one instance:
//   0. every global array the tile needs (its entropy-projected values, the values its
//      face neighbours pushed into its slots, metric factors, state, RK register, the
//      static block of mass data, weights, bathymetry and push targets) is fetched into
//      LDS with asynchronous copies, so the global-memory latency is exposed once per tile;
//   1. node records at the Nh hybridized nodes are built in LDS;
//   2. flux differencing in skew form (Section 5.2, Step 4): every row m of every
//      nonzero block of Q_skew = Q_h - Q_h^T (volume-volume and volume-surface; the zero
//      surface-surface block is skipped), with the element's physical operator built on
//      the fly from averaged geometric factors (Section 2.7) and the EC flux of
//      Section 2.8; each thread owns R rows of one element so a column's node record is
//      read once for R rows.  The bathymetry source is folded in as
//      1/2 g h_m (H_n - Href) Q_mn (exact because Q_h 1 = 0);
//   3. interface flux f_S(u~+, u~), boundary half of the source and optional local
//      Lax-Friedrichs penalty (Section 2.8) on the face rows;
//   4. lift rhs = -(M_h^k)^{-1} V_h^T r_h, with the stored inverses (Section 2.8) or the
//      weight-adjusted inverse named after eq. (dgform);
//   5. LSRK update (Section 4), then, fused, the entropy projection of the updated state
//      (Section 2.6), written to the other stage buffer and pushed into the face slots of
//      the neighbours (or, on a reflective wall, Section 2.9, the mirror state into the
//      node's own slot).
// Between stages the face exchange needs every neighbour's projection: either the launch
// boundary (one launch per stage) or, in a multi-stage launch, per-tile progress counts
// that a tile waits on before it reads its neighbours' values.
//
// Depth is carried as the free-surface anomaly eta = h + b - Href (Href a per-instance
// constant), so the projection works on v1 - g Href and no quantity of size g H is
// rounded to the bulk precision; the conversions to h are done in double.
#include <hip/hip_runtime.h>
#include <algorithm>

#include <cmath>
#include <type_traits>

#include "device_types.hpp"

namespace esdg {

__device__ inline bool bad_value(double h, double a, double b) {
  return !(h > 0.0) || !isfinite(h) || !isfinite(a) || !isfinite(b);
}

// The wave's index in the workgroup, as a wave-uniform (scalar) value: loops over
// wave-sized chunks then keep their counters, bounds and LDS bases in scalar registers.
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6); }

// The thread index, read through an empty asm so that the compiler cannot hoist index
// arithmetic derived from it out of the stage loop of a multi-stage launch (hoisted, every
// phase's per-thread indices would stay live across all phases and spill).
__device__ __forceinline__ int phase_tid() {
  int t = int(threadIdx.x);
  asm volatile("" : "+v"(t));
  return t;
}

// Task i of a phase over (field c, element e, mode or node j) in [3][ne][M] order: c, the
// offset r = e M + j within field c's block, e and j.  The products take 24-bit multiplies
// and the division is unsigned by the constant M: 32-bit multiplies issue at a quarter of
// the vector-ALU rate, and these phases run their index arithmetic once per task.
template <int M>
struct FieldTask {
  int c, r, e, j;
  __device__ __forceinline__ FieldTask(int i, int nem) {     // nem = ne * M
    c = (i >= nem) + (i >= 2 * nem);
    r = i - __umul24(unsigned(c), unsigned(nem));
    e = int(unsigned(r) / unsigned(M));
    j = r - __umul24(unsigned(e), unsigned(M));
  }
};

// ---------------------------------------------------------------- matrix-core contractions
// C[M x NC] = A[M x KD] B[KD x NC], A and B read from LDS, on the matrix cores.  One wave
// per 16x16 output block; blocks are dealt to the workgroup's waves.  Lane layout of the
// 16x16xK instructions used: lane l holds A[row l%16][k in k-quad l/16], B[k in k-quad
// l/16][col l%16]; it receives D[row 4(l/16) + r][col l%16], r = 0..3, from the f32 and
// bf16 instructions, but D[row l/16 + 4r][col l%16] from v_mfma_f64_16x16x4_f64.
// Out-of-range rows, columns and k are zero.  Modes:
//   kMfmaNative: v_mfma_f32_16x16x4_f32 or v_mfma_f64_16x16x4_f64 (same rounding as the
//                VALU path up to summation order);
//   kMfmaBf16x3: each operand split x = hi + lo (hi = bf16(x), lo = bf16(x - hi)), product
//                hi_a hi_b + hi_a lo_b + lo_a hi_b by v_mfma_f32_16x16x16_bf16 with float
//                accumulation (relative error ~2^-16 per product).
enum ContractionMode : int { kValu = 0, kMfmaNative = 1, kMfmaBf16x3 = 2 };

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x4_t __attribute__((ext_vector_type(4)));

__device__ inline unsigned short bf16_rne(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);            // round to nearest even (finite inputs)
  return (unsigned short)(u >> 16);
}
__device__ inline float bf16_value(unsigned short h) { return __uint_as_float(unsigned(h) << 16); }

template <int MODE, typename real, class FA, class FB, class FC>
__device__ __forceinline__ void gemm_mfma(int M, int KD, int NC, FA a_at, FB b_at, FC c_store) {
  const int lane = threadIdx.x & 63, wave = wave_id(), nwaves = blockDim.x >> 6;
  const int mb = (M + 15) / 16, nb = (NC + 15) / 16;
  const int lrow = lane & 15, quad = lane >> 4;
#pragma unroll 1
  for (int blk = wave; blk < mb * nb; blk += nwaves) {
    const int bi = blk % mb, bj = blk / mb;
    const int row = bi * 16 + lrow, col = bj * 16 + lrow;
    if constexpr (MODE == kMfmaBf16x3) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 1
      for (int k0 = 0; k0 < KD; k0 += 16) {
        bf16x4_t ahi, alo, bhi, blo;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int k = k0 + 4 * quad + r;
          const float av = (row < M && k < KD) ? float(a_at(row, k)) : 0.f;
          const float bv = (col < NC && k < KD) ? float(b_at(k, col)) : 0.f;
          const unsigned short ah = bf16_rne(av), bh = bf16_rne(bv);
          ahi[r] = short(ah);
          alo[r] = short(bf16_rne(av - bf16_value(ah)));
          bhi[r] = short(bh);
          blo[r] = short(bf16_rne(bv - bf16_value(bh)));
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, bhi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ahi, blo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(alo, bhi, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = bi * 16 + 4 * quad + r;
        if (i < M && col < NC) c_store(i, col, real(acc[r]));
      }
    } else if constexpr (std::is_same<real, float>::value) {
      f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 2
      for (int k0 = 0; k0 < KD; k0 += 4) {
        const int k = k0 + quad;
        const float av = (row < M && k < KD) ? a_at(row, k) : 0.f;
        const float bv = (col < NC && k < KD) ? b_at(k, col) : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = bi * 16 + 4 * quad + r;
        if (i < M && col < NC) c_store(i, col, acc[r]);
      }
    } else {
      f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 2
      for (int k0 = 0; k0 < KD; k0 += 4) {
        const int k = k0 + quad;
        const double av = (row < M && k < KD) ? a_at(row, k) : 0.0;
        const double bv = (col < NC && k < KD) ? b_at(k, col) : 0.0;
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = bi * 16 + quad + 4 * r;      // f64 output rows are interleaved
        if (i < M && col < NC) c_store(i, col, acc[r]);
      }
    }
  }
}

// LDS carve-up of one tile (see lds_words()).
template <typename real, int N>
struct Lds {
  static constexpr int Np = dim_Np(N), Nq = dim_Nq(N), Nfq = dim_Nfq(N), Nh = dim_Nh(N);
  real *ref, *Vh, *ST, *FT, *wf, *nr, *ns;
  real *rec, *raw, *nb, *U, *DU, *Minv, *wJ, *bq, *bh;
  real *R, *T, *Q, *VH;
  int32_t *pp;
  // sm: the ref block (already loaded); tile: the tile region (after the largest ref block);
  // mw: reals of mass data per element (mass_words); P: column parts of the residual
  __device__ Lds(real *sm, real *tile, int E, int mw, int P) {
    ref = sm;
    Vh = ref;
    ST = Vh + Nh * Np;
    FT = ST + 2 * Nh * Nq;
    wf = FT + 2 * Nq * Nfq;
    nr = wf + Nfq;
    ns = nr + Nfq;
    rec = tile;
    raw = rec + E * rec_stride(N);
    nb = raw + E * raw_words(N, P);
    U = nb + 4 * E * Nfq;
    DU = U + 3 * E * Np;
    Minv = DU + 3 * E * Np;
    wJ = Minv + E * mw;          // Minv: [E][Np][Np], or w/J [E][Nq] (weight-adjusted)
    bq = wJ + E * Nq;
    bh = bq + E * Nq;
    pp = reinterpret_cast<int32_t *>(bh + E * Nh);
    // reuse: the residual, lift and projection temporaries live in the raw block (dead
    // after phase 1) and v'_h in the neighbour block (dead after the residual); the
    // node records and the state are left alone, so a resident tile keeps them
    R = raw;                      // the P partial residuals [P][3][E][Nh]
    T = raw + 3 * P * E * Nh;     // [3][E][Np]
    Q = raw;                      // [3][E][Nq] projection's weighted entropy variables
    VH = nb;                      // [3][E][Np] v'_h (3 Np <= 4 Nfq for N <= 5)
  }
};

// Default rows per thread of the residual phase (the build without tile-shape choice).
template <typename real, int N> struct RowsPerThread { static constexpr int value = 1; };
template <> struct RowsPerThread<float, 1> { static constexpr int value = 2; };
template <> struct RowsPerThread<float, 3> { static constexpr int value = 2; };
// Default column chunks of the residual phase: one at N = 5 (whose 512-thread workgroups
// have a task per row already), else two.
template <typename real, int N> struct DefaultParts { static constexpr int value = 2; };
template <> struct DefaultParts<float, 5> { static constexpr int value = 1; };
template <> struct DefaultParts<double, 5> { static constexpr int value = 1; };

// Tile shapes the residual phase is compiled for: R = 1 or 2 rows per thread (2 only in
// float, where R divides Nq and Nfq: two rows of double accumulators exceed the register
// budget of four waves per SIMD and spill) and P = 1..4 column parts.
template <typename real, int N>
__host__ __device__ constexpr bool shape_ok(int shape) {
  return shape_parts(shape) >= 1 && shape_parts(shape) <= 4 &&
         (shape_rows(shape) == 1 ||
          (shape_rows(shape) == 2 && sizeof(real) == 4 && dim_Nq(N) % 2 == 0 && dim_Nfq(N) % 2 == 0));
}

// Stage flags of a multi-stage launch whose tiles stay in LDS (StageArgs::resident).
constexpr int kResident = 1;       // the tile's records, metric factors, static block, state and
                                   // RK register stay in LDS between the stages of the launch
constexpr int kResMid = 2;         // not the first stage: only the neighbour values are fetched
constexpr int kResLast = 4;        // last stage: the state, RK register and u~ go to HBM

// Weight-adjusted inverse of the curved mass matrix (the implementation remark after eq.
// (dgform) in Section 2.8): (M_h^k)^{-1} y ~ M^{-1} M_{1/J} M^{-1} y with M_{1/J} =
// V_q^T W diag(1/J) V_q; the reference mass matrix M is the identity for the orthonormal
// basis with the degree-2N volume rule, so this is V_q^T diag(w/J) V_q y, two contractions
// with V_q (the first Nq rows of V_h) and the per-element weights w/J (held where the
// stored inverse would be).  First factor, one task per (field, element, volume node):
// S[c][e][q] = (w/J)[e][q] sum_j V_q[q][j] Y[c][e][j].
template <typename real, int N>
__device__ __forceinline__ void wadg_first(int ne, const Lds<real, N> &L, const real *Y, real *S) {
  constexpr int Np = dim_Np(N), Nq = dim_Nq(N);
  for (int i = phase_tid(); i < 3 * ne * Nq; i += blockDim.x) {
    const int c = (i >= ne * Nq) + (i >= 2 * ne * Nq), r = i - c * ne * Nq, e = r / Nq, q = r - e * Nq;
    const real *Yc = Y + c * ne * Np + e * Np;
    const real *Vq = L.Vh + q * Np;
    real a = 0, b = 0;
#pragma unroll 32
    for (int j = 0; j + 1 < Np; j += 2) {
      a += Vq[j] * Yc[j];
      b += Vq[j + 1] * Yc[j + 1];
    }
    if (Np & 1) a += Vq[Np - 1] * Yc[Np - 1];
    S[i] = L.Minv[e * Nq + q] * (a + b);
  }
}

// Second factor for one output mode: sum_q V_q[q][row] Sc[q].
template <typename real, int N>
__device__ __forceinline__ real wadg_second(const Lds<real, N> &L, const real *Sc, int row) {
  constexpr int Np = dim_Np(N), Nq = dim_Nq(N);
  real a = 0, b = 0;
#pragma unroll 32
  for (int q = 0; q + 1 < Nq; q += 2) {
    a += L.Vh[q * Np + row] * Sc[q];
    b += L.Vh[(q + 1) * Np + row] * Sc[q + 1];
  }
  if (Nq & 1) a += L.Vh[(Nq - 1) * Np + row] * Sc[Nq - 1];
  return a + b;
}

// Entropy projection of the tile states in L.U ([3][ne][Np]: eta, hu, hv) to the
// hybridized nodes (Section 2.6), written to out (tile-blocked [4][ne][Nh]: h~, u~, v~,
// H~ - Href) or, in a resident stage that is not the last, straight into the node records
// of the next stage (the same values the records phase would form from out):
//   q = V_q u_h; h = eta_q + (Href - b_q); v' = (g eta_q - |u|^2/2, u, v) = v(u_q) - (g Href, 0, 0)
//   (FP64); v'_h = Minv_k V_q^T diag(w J) v'_q (Minv_k the stored inverse, or the
//   weight-adjusted one); v~' = V_h v'_h;
//   H~ - Href = (v~1' + |v~23|^2/2)/g, h~ = (H~ - Href) + (Href - b~) (FP64).
// Subtracting the constant g Href is exact: the projection reproduces constants.  The rest
// depth Href - b comes from the static block, formed in double on the device from b (so in
// float it has the relative accuracy of the depth itself where the water is shallow).
template <typename real, int N, int CM, bool WADG>
__device__ __forceinline__ void project_tile(const InstDesc &d, int k0, int ne, Lds<real, N> &L, real *out,
                                             real *nbx_out, int32_t *flag, bool coherent, int res = 0) {
  const bool to_records = (res & kResident) && !(res & kResLast);
  constexpr bool mfma = CM != kValu;
  constexpr int Np = dim_Np(N), Nq = dim_Nq(N), Nh = dim_Nh(N), Nfq = dim_Nfq(N);
  const double g = d.g;
  const int tid = phase_tid(), nth = blockDim.x;
  const int nc = 3 * ne;                       // contraction columns: (field, element)
  real *Stage = L.R;                           // [3][ne][Nq] or [3][ne][Nh] staging (free here)
  bool bad = false;
  if constexpr (CM != kValu) {
    {                              // u_q = V_q u_h on the matrix cores
      gemm_mfma<CM, real>(Nq, Np, nc, [&](int i, int k) { return L.Vh[i * Np + k]; },
                  [&](int k, int c) { return L.U[c * Np + k]; },
                  [&](int i, int c, real v) { Stage[c * Nq + i] = v; });
      __syncthreads();
    }
  }
  for (int i = tid; i < ne * Nq; i += nth) {
    const int e = int(unsigned(i) / unsigned(Nq)), q = i - __umul24(unsigned(e), unsigned(Nq));
    real u0 = 0, u1 = 0, u2 = 0;
    if (mfma) {
      u0 = Stage[i];
      u1 = Stage[ne * Nq + i];
      u2 = Stage[2 * ne * Nq + i];
    } else {
      const real *Vq = L.Vh + __umul24(unsigned(q), unsigned(Np));
      const real *Ue = L.U + __umul24(unsigned(e), unsigned(Np));
#pragma unroll 32
      for (int j = 0; j < Np; ++j) {
        const real v = Vq[j];
        u0 += v * Ue[j];
        u1 += v * Ue[ne * Np + j];
        u2 += v * Ue[2 * ne * Np + j];
      }
    }
    const double eta = u0, hu = u1, hv = u2;
    const double h = eta + double(L.bq[i]);       // L.bq: rest depth Href - b
    const double rh = 1.0 / h, uu = hu * rh, vv = hv * rh;
    const double v1 = g * eta - 0.5 * (uu * uu + vv * vv);
    const double w = L.wJ[i];
    L.Q[0 * ne * Nq + i] = real(w * v1);
    L.Q[1 * ne * Nq + i] = real(w * uu);
    L.Q[2 * ne * Nq + i] = real(w * vv);
    bad |= bad_value(h, hu, hv);
  }
  __syncthreads();
  // y = V_q^T (w J v'): one task per (field, element, mode)
  if constexpr (CM != kValu) {
      gemm_mfma<CM, real>(Np, Nq, nc, [&](int i, int k) { return L.Vh[k * Np + i]; },
                  [&](int k, int c) { return L.Q[c * Nq + k]; },
                  [&](int i, int c, real v) { L.T[c * Np + i] = v; });
  }
  for (int i = tid; i < 3 * ne * Np && !mfma; i += nth) {
    const FieldTask<Np> k(i, ne * Np);
    const real *Qc = L.Q + __umul24(unsigned(k.c), unsigned(ne * Nq)) + __umul24(unsigned(k.e), unsigned(Nq));
    const real *Vj = L.Vh + k.j;
    real ya = 0, yb = 0;
#pragma unroll 32
    for (int q = 0; q + 1 < Nq; q += 2) {
      ya += Vj[q * Np] * Qc[q];
      yb += Vj[(q + 1) * Np] * Qc[q + 1];
    }
    if (Nq & 1) ya += Vj[(Nq - 1) * Np] * Qc[Nq - 1];
    L.T[i] = ya + yb;
  }
  __syncthreads();
  // v'_h = Minv_k y (weight-adjusted: the first factor into L.Q, dead once y is formed)
  if constexpr (WADG) {
    wadg_first<real, N>(ne, L, L.T, L.Q);
    __syncthreads();
  }
  for (int i = tid; i < 3 * ne * Np; i += nth) {
    const FieldTask<Np> k(i, ne * Np);
    if constexpr (WADG) {
      L.VH[i] = wadg_second<real, N>(L, L.Q + __umul24(unsigned(k.c), unsigned(ne * Nq)) +
                                            __umul24(unsigned(k.e), unsigned(Nq)), k.j);
    } else {
      const real *Mi = L.Minv + __umul24(unsigned(k.r), unsigned(Np));   // row (e, j) of Minv_e
      const real *Tc = L.T + (i - k.j);                                  // T[c][e][0..Np)
      real va = 0, vb = 0;
#pragma unroll 32
      for (int j = 0; j + 1 < Np; j += 2) {
        va += Mi[j] * Tc[j];
        vb += Mi[j + 1] * Tc[j + 1];
      }
      if (Np & 1) va += Mi[Np - 1] * Tc[Np - 1];
      L.VH[i] = va + vb;
    }
  }
  __syncthreads();
  if constexpr (CM != kValu) {
    {                              // v~ = V_h v_h on the matrix cores
      gemm_mfma<CM, real>(Nh, Np, nc, [&](int i, int k) { return L.Vh[i * Np + k]; },
                  [&](int k, int c) { return L.VH[c * Np + k]; },
                  [&](int i, int c, real v) { Stage[c * Nh + i] = v; });
      __syncthreads();
    }
  }
  for (int i = tid; i < ne * Nh; i += nth) {
    const int e = int(unsigned(i) / unsigned(Nh)), n = i - __umul24(unsigned(e), unsigned(Nh));
    real t0 = 0, t1 = 0, t2 = 0;
    if (mfma) {
      t0 = Stage[i];
      t1 = Stage[ne * Nh + i];
      t2 = Stage[2 * ne * Nh + i];
    } else {
      const real *Vn = L.Vh + __umul24(unsigned(n), unsigned(Np));
      const real *Ve = L.VH + __umul24(unsigned(e), unsigned(Np));
#pragma unroll 32
      for (int j = 0; j < Np; ++j) {
        const real v = Vn[j];
        t0 += v * Ve[j];
        t1 += v * Ve[ne * Np + j];
        t2 += v * Ve[2 * ne * Np + j];
      }
    }
    const double v1 = t0, v2 = t1, v3 = t2;
    const double dH = (v1 + 0.5 * (v2 * v2 + v3 * v3)) / g;
    const double h = dH + double(L.bh[i]);        // L.bh: rest depth Href - b
    if (to_records) {
      typedef real real4 __attribute__((ext_vector_type(4)));
      const real hr = real(h), ur = real(v2), vr = real(v3), gr = real(d.g);
      real4 *rec = reinterpret_cast<real4 *>(L.rec + __umul24(unsigned(e), unsigned(rec_stride(N))) + n * kNodeRec);
      rec[0] = real4{real(0.5) * hr * ur, real(0.5) * hr * vr, real(0.5) * ur, real(0.5) * vr};
      rec[2] = real4{real(0.5) * gr * hr, real(dH), hr, real(0)};
    } else {
      real *ot = out + size_t(k0) * 4 * Nh + unsigned(i);   // tile-blocked [4][ne][Nh]
      ot[0] = real(h);
      ot[ne * Nh] = real(v2);
      ot[2 * ne * Nh] = real(v3);
      ot[3 * ne * Nh] = real(dH);
    }
    if (n >= Nq) {                 // face node: also fill the neighbour's face slot
      const int f = n - Nq;
      const uint32_t tgt = uint32_t(L.pp[__umul24(unsigned(e), unsigned(Nfq)) + f]);
      real *slot = nbx_out + size_t(tgt & ~kPushWall) * 4;
      double pu = v2, pv = v3;     // the velocity the exterior side of the face sees
      if (tgt & kPushWall) {
        // reflective wall (Section 2.9): the exterior state is this node's own with the
        // normal velocity reversed, u+ = u - 2 (u . nJ) nJ / |nJ|^2, h+ = h (so H+ = H),
        // written into this node's own slot; nJ from the metric factors (tile-blocked, as
        // fetched) and the reference normal of the face
        const real *gm = static_cast<const real *>(d.geo) + size_t(k0) * 4 * Nh + unsigned(i);
        const double nr = double(L.nr[f]), ns = double(L.ns[f]);
        const double nx = double(gm[0]) * nr + double(gm[ne * Nh]) * ns;
        const double ny = double(gm[2 * ne * Nh]) * nr + double(gm[3 * ne * Nh]) * ns;
        const double c = 2.0 * (v2 * nx + v3 * ny) / (nx * nx + ny * ny);
        pu = v2 - c * nx;
        pv = v3 - c * ny;
      }
      if (coherent) {
        // multi-stage launches: device-coherent (sc1) 16-byte vector stores, since the
        // neighbour's workgroup may sit on another XCD, whose L2 does not see this one's.
        // The slot is 16-byte aligned; publish() waits for these stores (vmcnt) itself.
        // A vector store of more than 8 bytes reads its data registers after issue: a VALU
        // write to them must wait two cycles.  The compiler inserts that wait only for stores
        // it generates, not for these, so each statement carries its own s_nop (without it
        // the FP64 pair below had its first store's data overwritten by the second's address).
        if constexpr (sizeof(real) == 4) {
          typedef float f4 __attribute__((ext_vector_type(4)));
          const f4 val = {float(h), float(pu), float(pv), float(dH)};
          asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" ::"v"(slot), "v"(val) : "memory");
        } else {
          typedef double d2 __attribute__((ext_vector_type(2)));
          const d2 lo = {h, pu}, hi = {pv, dH};
          asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" ::"v"(slot), "v"(lo) : "memory");
          asm volatile("global_store_dwordx4 %0, %1, off sc1\n\ts_nop 1" ::"v"(slot + 2), "v"(hi) : "memory");
        }
      } else {
        typedef real real4 __attribute__((ext_vector_type(4)));
        const real4 val = {real(h), real(pu), real(pv), real(dH)};
        *reinterpret_cast<real4 *>(slot) = val;
      }
    }
    bad |= bad_value(h, v2, v3);
  }
  if (bad) atomicOr(flag, 1);
}

// Asynchronous global -> LDS copies (global_load_lds_dword): each lane moves one 32-bit
// word straight into LDS at (wave-uniform base) + 4 * lane, so a wave copies 64
// consecutive words per instruction without staging them in registers; completion is
// awaited once, with s_waitcnt vmcnt(0), before the tile's barrier.  (The 16-byte form,
// global_load_lds_dwordx4, measured slower for these tile fetches.)
typedef __attribute__((address_space(1))) const void *gptr_t;
typedef __attribute__((address_space(3))) void *lptr_t;

template <int CPOL = 0>
__device__ inline void async_copy_words(uint32_t *dst, const uint32_t *src, int nwords) {
  const int lane = threadIdx.x & 63, wave = wave_id(), nwaves = blockDim.x >> 6;
  for (int c = wave * 64; c < nwords; c += nwaves * 64) {
    if (c + lane < nwords)
      __builtin_amdgcn_global_load_lds((gptr_t)(src + c + lane), (lptr_t)(dst + c), 4, 0, CPOL);
  }
}
constexpr int kCpolAgent = 16;     // sc1: device-coherent access (other XCDs' stores visible)

// 32-bit words of a tile's static block staged through registers during a stage.
template <typename real>
__device__ __forceinline__ int stat_head(int nstat) {
  const int cap = StatRegs<real>::value * int(blockDim.x);
  return nstat < cap ? nstat : cap;
}

// Phase 0: fetch the tile's global data into LDS (all asynchronous; see above).
template <typename real, int N, bool WADG, bool MULTI>
__device__ __forceinline__ void fetch_tile(const StageArgs &a, const InstDesc &d, int k0, int ne, Lds<real, N> &L) {
  constexpr int Np = dim_Np(N), Nfq = dim_Nfq(N), Nh = dim_Nh(N);
  constexpr int W = sizeof(real) / 4;     // 32-bit words per value
  const size_t splane = size_t(d.K) * Np;
  auto words = [](const void *p) { return static_cast<const uint32_t *>(p); };
  auto lwords = [](real *p) { return reinterpret_cast<uint32_t *>(p); };
  // the multi-stage build runs RK stages only, on the instance buffers (see stage_tile)
  const int mode = MULTI ? int(kStage) : a.mode;
  const void *ext_ut = MULTI ? nullptr : a.ext_ut, *ext_state = MULTI ? nullptr : a.ext_state;
  const void *ext_nbx = MULTI ? nullptr : a.ext_nbx;
  if (mode != kProject) {
    // u~ and the metric factors are stored tile-blocked ([4][ne][Nh] per tile), one copy each
    const size_t base = size_t(k0) * 4 * Nh;
    const void *ut = ext_ut ? ext_ut : d.ut[a.in_buf];
    async_copy_words(lwords(L.raw), words(static_cast<const real *>(ut) + base), 4 * ne * Nh * W);
    async_copy_words(lwords(L.raw + 4 * ne * Nh), words(static_cast<const real *>(d.geo) + base), 4 * ne * Nh * W);
  }
  if (mode == kStage) {
    const real *uh = static_cast<const real *>(d.uh);
    const real *du = static_cast<const real *>(d.du);
    for (int c = 0; c < 3; ++c) {
      async_copy_words(lwords(L.U + c * ne * Np), words(uh + c * splane + size_t(k0) * Np), ne * Np * W);
      async_copy_words(lwords(L.DU + c * ne * Np), words(du + c * splane + size_t(k0) * Np), ne * Np * W);
    }
  } else if (mode == kProject) {
    const real *src = static_cast<const real *>(ext_state ? ext_state : d.uh);
    for (int c = 0; c < 3; ++c)
      async_copy_words(lwords(L.U + c * ne * Np), words(src + c * splane + size_t(k0) * Np), ne * Np * W);
  }
  {
    // static block (mass data, w J, b, push targets): contiguous in HBM and in LDS.  A
    // stage copies only the part beyond the first kStatRegs words per thread here; that head
    // goes through registers and lands in LDS after the residual (stage_tile).
    constexpr int SW = stat_words(N, WADG);
    const int nstat = ne * SW * W, head = mode == kProject ? 0 : stat_head<real>(nstat);
    async_copy_words(lwords(L.Minv) + head, words(static_cast<const real *>(d.stat) + size_t(k0) * SW) + head,
                     nstat - head);
  }
  if (mode != kProject) {          // neighbour values, pushed here by the neighbours' projections
    const void *nbx = ext_nbx ? ext_nbx : d.nbx[a.in_buf];
    const uint32_t *src = words(static_cast<const real *>(nbx) + size_t(k0) * Nfq * 4);
    if (MULTI && a.progress)       // multi-stage launch: written during this kernel, maybe on another XCD
      async_copy_words<kCpolAgent>(lwords(L.nb), src, ne * Nfq * 4 * W);
    else
      async_copy_words(lwords(L.nb), src, ne * Nfq * 4 * W);
  }
  __builtin_amdgcn_s_waitcnt(0);   // this wave's copies have landed in LDS
}

// Interface terms of face node f (Section 2.8) from its node record rm and the neighbour's
// values nbp (h, u, v, H - Href): W_f [ nJ . f_S(u~, u~+) + 1/2 g h (H+ - Href) nJ ] minus,
// for the LF flux, the penalty 1/2 lambda sJ (u~+ - u~).  One function for the pair loop's
// face rows and the separate interface pass, so both produce the same bits.
template <typename real>
__device__ __forceinline__ void interface_terms(const real *rm, const real *nbp, real wf, real nrf, real nsf, real g,
                                                int flux, real &t0, real &t1, real &t2) {
  typedef real real4 __attribute__((ext_vector_type(4)));
  const real4 s0 = *reinterpret_cast<const real4 *>(rm), s1 = *reinterpret_cast<const real4 *>(rm + 4);
  const real gh = rm[8], dH = rm[9], h = rm[10];
  const real nJx = s1.x * nrf + s1.y * nsf, nJy = s1.z * nrf + s1.w * nsf;
  const real uu = real(2) * s0.z, vv = real(2) * s0.w, huu = real(2) * s0.x, hvv = real(2) * s0.y;
  const real hP = nbp[0], uP = nbp[1], vP = nbp[2], dHP = nbp[3];
  const real huP = hP * uP, hvP = hP * vP;
  const real hua = real(0.5) * (huu + huP), hva = real(0.5) * (hvv + hvP);
  const real ua = real(0.5) * (uu + uP), va = real(0.5) * (vv + vP);
  const real pr = gh * dHP;
  real f0v = nJx * hua + nJy * hva;
  real f1v = nJx * (hua * ua + pr) + nJy * hva * ua;
  real f2v = nJx * hua * va + nJy * (hva * va + pr);
  if (flux == 1) {
    const real sJ = sqrt(nJx * nJx + nJy * nJy);
    const real lm = fabs(uu * nJx + vv * nJy) + sqrt(g * h) * sJ;
    const real lp = fabs(uP * nJx + vP * nJy) + sqrt(g * hP) * sJ;
    const real c = real(0.5) * fmax(lm, lp);
    f0v -= c * (dHP - dH);
    f1v -= c * (huP - huu);
    f2v -= c * (hvP - hvv);
  }
  t0 = wf * f0v;
  t1 = wf * f1v;
  t2 = wf * f2v;
}

// Residual rows (Section 2.8, flux differencing plus interface terms).  Row m accumulates,
// over its columns n, c = Qx {hu} + Qy {hv} (a0), u_n c and v_n c (b1, b2), and dH_n Qx,
// dH_n Qy (q1, q2); the row factors are applied once at the end:
//   sum_n ({u} c + gh_m dH_n Qx) = u_m a0 + b1 + gh_m q1   (halves folded into the records)
// Volume rows run over all Nh columns (the diagonal of the skew operator is zero), face rows
// over the Nq volume columns (the surface-surface block is zero).  This function is one
// task: rows m0 .. m0+R-1 (r0 .. r0+R-1 within their row set) of element e, over columns
// [n_lo, n_hi), with the operator table Stab (already offset to row r0) whose consecutive
// columns are ld2 reals apart; the sums go to chunk slot p of the residual block.
template <typename real, int N, int R, class LD, class LT>
__device__ __forceinline__ void row_sums(const InstDesc &d, int ne, int e, int r0, int m0, int p, bool face,
                                         int n_lo, int n_hi, const real *Stab, LD ld2, LT &L, bool iface) {
  constexpr int Nfq = dim_Nfq(N), Nh = dim_Nh(N);
  typedef real real4 __attribute__((ext_vector_type(4)));
  const real *rbase = L.rec + __umul24(unsigned(e), unsigned(rec_stride(N)));
  real hu[R], hv[R], u[R], v[R], gh[R], rx[R], sx[R], ry[R], sy[R], a0[R], a1[R], a2[R];
  real b1[R], b2[R], q1[R], q2[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const real *rm = rbase + (m0 + r) * kNodeRec;
    const real4 s0 = *reinterpret_cast<const real4 *>(rm), s1 = *reinterpret_cast<const real4 *>(rm + 4);
    hu[r] = s0.x; hv[r] = s0.y; u[r] = s0.z; v[r] = s0.w;
    rx[r] = s1.x; sx[r] = s1.y; ry[r] = s1.z; sy[r] = s1.w;
    gh[r] = rm[8];
    a0[r] = 0; b1[r] = 0; b2[r] = 0; q1[r] = 0; q2[r] = 0;
  }
#pragma unroll 2
  for (int n = n_lo; n < n_hi; ++n) {
    const real *rn = rbase + n * kNodeRec;
    const real4 c0 = *reinterpret_cast<const real4 *>(rn), c1 = *reinterpret_cast<const real4 *>(rn + 4);
    const real hun = c0.x, hvn = c0.y, un = c0.z, vn = c0.w, dHn = rn[9];
    const real rxn = c1.x, sxn = c1.y, ryn = c1.z, syn = c1.w;
    const real *S = Stab + n * ld2;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const real Sr = S[2 * r], Ss = S[2 * r + 1];
      const real Qx = (rx[r] + rxn) * Sr + (sx[r] + sxn) * Ss;
      const real Qy = (ry[r] + ryn) * Sr + (sy[r] + syn) * Ss;
      const real c = Qx * (hu[r] + hun) + Qy * (hv[r] + hvn);
      a0[r] += c;
      b1[r] += un * c;
      b2[r] += vn * c;
      q1[r] += dHn * Qx;
      q2[r] += dHn * Qy;
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    a1[r] = u[r] * a0[r] + b1[r] + gh[r] * q1[r];
    a2[r] = v[r] * a0[r] + b2[r] + gh[r] * q2[r];
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const int m = m0 + r;
    if (face && p == 0 && iface) {         // interface terms of face row m (else a later pass)
      const int f = r0 + r;
      real t0, t1, t2;
      interface_terms<real>(rbase + m * kNodeRec, L.nb + __umul24(unsigned(e), unsigned(Nfq * 4)) + f * 4, L.wf[f],
                            L.nr[f], L.ns[f], real(d.g), d.flux, t0, t1, t2);
      a0[r] = a0[r] + t0;
      a1[r] = a1[r] + t1;
      a2[r] = a2[r] + t2;
    }
    // partial sums of column chunk p
    real *Rp = L.R + __umul24(unsigned(p), unsigned(3 * ne * Nh)) + __umul24(unsigned(e), unsigned(Nh)) + m;
    Rp[0] = a0[r];
    Rp[ne * Nh] = a1[r];
    Rp[2 * ne * Nh] = a2[r];
  }
}

// Two task layouts for the residual rows.  Kinds with few hybrid nodes cut volume and face
// rows each into P chunks, and their tasks fill separate waves (volume tasks first), each
// row type with its own compile-time loop.  Kinds with many (wide_kind) cut both row
// types into chunks of one length (residual_chunk), so that volume and face tasks sharing
// a wave run about the same trip count through one loop; the chunk partials are then
// summed once (sum_partials) instead of in every lift task.
template <int D, int P> __host__ __device__ constexpr int face_chunks() {
  return wide_kind(D) ? residual_face_parts(D, P) : P;
}

template <typename real, int N, int R, int P, class LT>
__device__ __forceinline__ void residual_tile(const InstDesc &d, int ne, LT &L, bool iface) {
  constexpr int Nq = dim_Nq(N), Nfq = dim_Nfq(N), Nh = dim_Nh(N);
  constexpr int VB = Nq / R, FB = Nfq / R, PF = face_chunks<N, P>();
  static_assert(Nq % R == 0 && Nfq % R == 0, "R must divide Nq and Nfq");
  const int tid = phase_tid(), nth = blockDim.x;
  const int nv = ne * VB * P, ntask = nv + ne * FB * PF;
  // task splits in unsigned arithmetic by constants (see FieldTask)
  auto split = [](int t, unsigned parts, unsigned rows, int &p, int &e, int &b) {
    const unsigned rest = unsigned(t) / parts;
    p = t - __umul24(rest, parts);
    e = int(rest / rows);
    b = int(rest) - __umul24(unsigned(e), rows);
  };
  // chunk slowest: task t = (p ne + e) rows + b with per = ne rows tasks per chunk, P <= 4
  auto split_slow = [](int t, int per, unsigned rows, int &p, int &e, int &b) {
    p = (t >= per) + (t >= 2 * per) + (t >= 3 * per);
    const unsigned rest = unsigned(t - __umul24(unsigned(p), unsigned(per)));
    e = int(rest / rows);
    b = int(rest) - __umul24(unsigned(e), rows);
  };
  for (int t = tid; t < ntask; t += nth) {
    if constexpr (wide_kind(N)) {
      constexpr int C = residual_chunk(N, P);
      const bool face = t >= nv;
      int p, e, b;
      if (face) split(t - nv, PF, FB, p, e, b);
      else split(t, P, VB, p, e, b);
      const int ncol = face ? Nq : Nh, n_lo = __umul24(unsigned(p), unsigned(C)),
                n_hi = n_lo + C < ncol ? n_lo + C : ncol;
      const int r0 = b * R;
      row_sums<real, N, R>(d, ne, e, r0, face ? Nq + r0 : r0, p, face, n_lo, n_hi,
                           (face ? L.FT : L.ST) + 2 * r0, face ? 2 * Nfq : 2 * Nq, L, iface);
    } else {
      // column chunk slowest: a wave's lanes then share one column range (the node records
      // of its columns are read by several elements at once, the operator table's rows by
      // consecutive row blocks), where chunk-fastest lanes read columns Nh / P apart
      int p, e, b;
      if (t < nv) {
        split_slow(t, ne * VB, VB, p, e, b);
        const int r0 = b * R;
        row_sums<real, N, R>(d, ne, e, r0, r0, p, false, int(unsigned(p) * Nh / P), int(unsigned(p + 1) * Nh / P),
                             L.ST + 2 * r0, std::integral_constant<int, 2 * Nq>(), L, iface);
      } else {
        split_slow(t - nv, ne * FB, FB, p, e, b);
        const int r0 = b * R;
        row_sums<real, N, R>(d, ne, e, r0, Nq + r0, p, true, int(unsigned(p) * Nq / P), int(unsigned(p + 1) * Nq / P),
                             L.FT + 2 * r0, std::integral_constant<int, 2 * Nfq>(), L, iface);
      }
    }
  }
}

// The residual phase in the instance's tile shape (one of the shapes of shape_ok).
template <typename real, int N, class LT>
__device__ __forceinline__ void residual_shaped(const InstDesc &d, int ne, LT &L, bool iface, int shape) {
  switch (shape) {
    case make_shape(1, 1): residual_tile<real, N, 1, 1>(d, ne, L, iface); break;
    case make_shape(1, 2): residual_tile<real, N, 1, 2>(d, ne, L, iface); break;
    case make_shape(1, 3): residual_tile<real, N, 1, 3>(d, ne, L, iface); break;
    case make_shape(1, 4): residual_tile<real, N, 1, 4>(d, ne, L, iface); break;
    default:
      if constexpr (shape_ok<real, N>(make_shape(2, 1))) {
        switch (shape) {
          case make_shape(2, 1): residual_tile<real, N, 2, 1>(d, ne, L, iface); break;
          case make_shape(2, 2): residual_tile<real, N, 2, 2>(d, ne, L, iface); break;
          case make_shape(2, 3): residual_tile<real, N, 2, 3>(d, ne, L, iface); break;
          case make_shape(2, 4): residual_tile<real, N, 2, 4>(d, ne, L, iface); break;
          default: break;
        }
      }
      break;
  }
}

// Wide kinds: adds the chunk partial sums of every residual row into chunk 0's (P chunks
// for volume rows, face_chunks for face rows), once per (field, element, node), so that
// the lift reads one partial.
template <typename real, int N, int P, class LT>
__device__ __forceinline__ void sum_partials(int ne, LT &L) {
  constexpr int Nq = dim_Nq(N), Nh = dim_Nh(N), PF = face_chunks<N, P>();
  for (int i = phase_tid(); i < 3 * ne * Nh; i += blockDim.x) {
    const int n = int(unsigned(i) % unsigned(Nh));
    real r = L.R[i];
    if (n < Nq) {
#pragma unroll
      for (int p = 1; p < P; ++p) r += L.R[p * 3 * ne * Nh + i];
    } else {
#pragma unroll
      for (int p = 1; p < PF; ++p) r += L.R[p * 3 * ne * Nh + i];
    }
    L.R[i] = r;
  }
}

// Lift of the residual on the vector ALUs: T = V_h^T r_h, one task per (field, element,
// mode).  PS partial sums per row are added here (1 once sum_partials has run).
template <typename real, int N, int PS, class LT>
__device__ __forceinline__ void lift_valu(int ne, LT &L) {
  constexpr int Np = dim_Np(N), Nh = dim_Nh(N);
  for (int i = phase_tid(); i < 3 * ne * Np; i += blockDim.x) {
    const FieldTask<Np> k(i, ne * Np);
    const real *Rc = L.R + __umul24(unsigned(k.c), unsigned(ne * Nh)) + __umul24(unsigned(k.e), unsigned(Nh));
    const real *Vj = L.Vh + k.j;
    real ya = 0, yb = 0;
#pragma unroll 32
    for (int n = 0; n < Nh; ++n) {
      real rn = Rc[n];
#pragma unroll
      for (int p = 1; p < PS; ++p) rn += Rc[p * 3 * ne * Nh + n];
      if (n & 1) yb += Vj[n * Np] * rn; else ya += Vj[n * Np] * rn;
    }
    L.T[i] = ya + yb;
  }
}

// The residual's chunk partials reduced to what the lift reads: summed in place for wide
// kinds (then a barrier), left for the lift otherwise.
template <typename real, int N, int P, int CM, class LT>
__device__ __forceinline__ void lift_partials(int ne, LT &L) {
  constexpr int Np = dim_Np(N), Nh = dim_Nh(N);
  if constexpr (wide_kind(N) && P > 1) {
    sum_partials<real, N, P>(ne, L);
    __syncthreads();
  }
  constexpr int PS = wide_kind(N) ? 1 : P;
  if constexpr (CM != kValu) {
    gemm_mfma<CM, real>(Np, Nh, 3 * ne, [&](int i, int k) { return L.Vh[k * Np + i]; },
                        [&](int k, int c) {
                          real v = L.R[c * Nh + k];
                          for (int p = 1; p < PS; ++p) v += L.R[p * 3 * ne * Nh + c * Nh + k];
                          return v;
                        },
                        [&](int i, int c, real v) { L.T[c * Np + i] = v; });
  } else {
    lift_valu<real, N, PS>(ne, L);
  }
}

// Descriptors, tiles and tile ranges are written by the host before a launch and only
// read by kernels.  Reading them through the constant address space lets the compiler use
// scalar loads (lgkmcnt); as vector loads they would share vmcnt with the asynchronous
// LDS copies, and every descriptor field needed between two copies would wait for all
// copies issued before it.
template <typename T>
__device__ __forceinline__ const T &read_const(const T *p, int i) {
  return *(const T *)((const __attribute__((address_space(4))) T *)p + i);
}

// Multi-stage launches: before stage `target` of tile t, wait until every tile holding a
// face neighbour of t has published `target` completed stages (their projection has pushed
// t's neighbour values, and they have finished reading the slots t is about to fill).
// Wave 0 polls, one neighbour per lane, with device-coherent loads and a bounded spin; the
// barrier then releases the other waves.  The neighbour values themselves are read with
// device-coherent copies (fetch_tile), so no cache-wide invalidation is needed.  Returns
// false (for the whole workgroup) if a wait gave up.
__device__ __forceinline__ bool wait_neighbours(const StageArgs &a, int t, int target) {
  int ok = 1;
  if (threadIdx.x < 64) {
    const int b = read_const(a.nbr_off, t), e = read_const(a.nbr_off, t + 1);
    for (int j = b + int(threadIdx.x); j < e; j += 64) {
      const int u = read_const(a.nbr_idx, j);
      int spins = 0;
      while (__hip_atomic_load(a.progress + u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        if (++spins > a.spin_limit) { ok = 0; break; }
        __builtin_amdgcn_s_sleep(1);
      }
    }
  }
  return __syncthreads_and(ok) != 0;
}

// After a stage of tile t: every wave waits until its stores have completed (the pushed
// face values are device-coherent stores, so completion means visible to every XCD), then
// one thread publishes the tile's completed-stage count.  The tile's other outputs are read
// back only by this workgroup.
__device__ __forceinline__ void publish(const StageArgs &a, int t, int value) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(a.progress + t, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Phase 3: interface terms of the face rows (Section 2.8), added to the first column
// part of the residual: W_f [ nJ . f_S(u~, u~+) + 1/2 g h (H+ - Href) nJ ] - LF penalty,
// one task per (element, face node).  A separate pass so that a resident tile can run
// the whole pair loop before it waits for its neighbours' values.
template <typename real, int N, class LT>
__device__ __forceinline__ void interface_tile(const InstDesc &d, int ne, LT &L) {
  constexpr int Nq = dim_Nq(N), Nfq = dim_Nfq(N), Nh = dim_Nh(N);
  for (int i = phase_tid(); i < ne * Nfq; i += blockDim.x) {
    const int e = int(unsigned(i) / unsigned(Nfq)), f = i - __umul24(unsigned(e), unsigned(Nfq)), m = Nq + f;
    const int em = __umul24(unsigned(e), unsigned(Nh)) + m;
    real t0, t1, t2;
    interface_terms<real>(L.rec + __umul24(unsigned(e), unsigned(rec_stride(N))) + m * kNodeRec, L.nb + 4 * i, L.wf[f], L.nr[f],
                          L.ns[f], real(d.g), d.flux, t0, t1, t2);
    real *R0 = L.R + em;                  // column part 0 of the three fields
    R0[0] = R0[0] + t0;
    R0[ne * Nh] = R0[ne * Nh] + t1;
    R0[2 * ne * Nh] = R0[2 * ne * Nh] + t2;
  }
}

// SHAPES: the build that takes the residual's tile shape from the instance (every shape of
// shape_ok); without it, the default shape (RowsPerThread rows, DefaultParts column chunks),
// whose register allocation the other shapes' code does not affect.
template <typename real, int N, int CM, bool WADG, bool MULTI, bool SHAPES>
__device__ __forceinline__ bool stage_tile(const StageArgs &a, const InstDesc &d, int k0, int ne, real *sm, real *tile,
                                           int res = 0, int t = 0, int target = 0) {
  constexpr int Np = dim_Np(N), Nh = dim_Nh(N), Nfq = dim_Nfq(N);
  const int tid = phase_tid(), nth = blockDim.x;
  constexpr int Nq = dim_Nq(N);
  const int shape = SHAPES ? d.shape : make_shape(RowsPerThread<real, N>::value, DefaultParts<real, N>::value);
  const int P = SHAPES ? shape_parts(shape) : DefaultParts<real, N>::value;
  Lds<real, N> L(sm, tile, ne, mass_words(N, WADG), P);
  const real g = real(d.g);
  const bool mid = res & kResMid;                // resident tile after its first stage
  const bool keep = (res & kResident) && !(res & kResLast);   // state stays in LDS only
  // The multi-stage build runs only multi-stage launches (and their residency probe, which
  // returns before any tile): RK stages on the instance buffers.  Taking that as given here
  // compiles the projection-only and RHS paths and the external buffers out of it, whose
  // addresses would otherwise stay live in scalar registers (and spill) across the stage.
  const int mode = MULTI ? int(kStage) : a.mode;
  // a resident tile after its first stage has everything but the neighbour values in LDS;
  // it fetches those after the pair loop, once its neighbours have pushed them
  if (!mid) fetch_tile<real, N, WADG, MULTI>(a, d, k0, ne, L);
  // head of the static block: loaded into registers now, while the node records and the
  // residual run, and written to LDS before the barrier that ends the residual
  constexpr int W = sizeof(real) / 4;
  const int nstat = ne * stat_words(N, WADG) * W, head = stat_head<real>(nstat);
  constexpr int SR = StatRegs<real>::value;
  const uint32_t *sg = static_cast<const uint32_t *>(d.stat) + size_t(k0) * stat_words(N, WADG) * W;
  uint32_t sreg[SR];
  if (mode != kProject && !mid) {
#pragma unroll
    for (int j = 0; j < SR; ++j) {
      const int v = tid + j * nth;
      sreg[j] = v < head ? sg[v] : 0u;
    }
  }
  if (!MULTI && mode == kProject) {
    __syncthreads();
    project_tile<real, N, CM, WADG>(d, k0, ne, L, static_cast<real *>(a.ext_ut ? a.ext_ut : d.ut[a.out_buf]),
                              static_cast<real *>(a.ext_nbx ? a.ext_nbx : d.nbx[a.out_buf]), a.flag,
                              MULTI && a.progress != nullptr);
    return true;
  }
  // a resident tile after its first stage skips the fetch and the records: what its residual
  // reads (the node records) was written before the barrier of the previous stage's publish
  if (!mid) __syncthreads();
  // phase 1: node records from the fetched u~ and metric factors (a resident tile's
  // previous projection wrote them directly)
  for (int i = tid; i < ne * Nh && !mid; i += nth) {
    const real h = L.raw[i], u = L.raw[ne * Nh + i], v = L.raw[2 * ne * Nh + i], dH = L.raw[3 * ne * Nh + i];
    typedef real real4 __attribute__((ext_vector_type(4)));
    const int e = int(unsigned(i) / unsigned(Nh)), n = i - __umul24(unsigned(e), unsigned(Nh));
    real4 *rec = reinterpret_cast<real4 *>(L.rec + __umul24(unsigned(e), unsigned(rec_stride(N))) + n * kNodeRec);
    rec[0] = real4{real(0.5) * h * u, real(0.5) * h * v, real(0.5) * u, real(0.5) * v};
    rec[1] = real4{L.raw[4 * ne * Nh + i], L.raw[5 * ne * Nh + i], L.raw[6 * ne * Nh + i], L.raw[7 * ne * Nh + i]};
    rec[2] = real4{real(0.5) * g * h, dH, h, real(0)};
  }
  if (!mid) __syncthreads();
  if constexpr (SHAPES) residual_shaped<real, N>(d, ne, L, !mid, shape);
  else residual_tile<real, N, RowsPerThread<real, N>::value, DefaultParts<real, N>::value>(d, ne, L, !mid);
  if (!mid) {
    uint32_t *sl = reinterpret_cast<uint32_t *>(L.Minv);
#pragma unroll
    for (int j = 0; j < SR; ++j) {
      const int v = tid + j * nth;
      if (v < head) sl[v] = sreg[j];
    }
  } else {
    if (!wait_neighbours(a, t, target)) return false;
    // from here to its publish the tile is on its neighbours' critical path (their next
    // stage waits for its pushes), while the other workgroups on the CU that are still in
    // their pair loop have slack: raise this workgroup's wave priority until the publish
    __builtin_amdgcn_s_setprio(2);
    async_copy_words<kCpolAgent>(reinterpret_cast<uint32_t *>(L.nb),
                                 static_cast<const uint32_t *>(d.nbx[a.in_buf]) + size_t(k0) * Nfq * 4 * W,
                                 ne * Nfq * 4 * W);
    __builtin_amdgcn_s_waitcnt(0);
  }
  if (mid) {
    __syncthreads();
    interface_tile<real, N>(d, ne, L);
  }
  __syncthreads();
  // lift: y = V_h^T r_h (r_h = the sum of the chunk partials), one task per (field, element,
  // mode)
  if constexpr (SHAPES) {
    switch (P) {
      case 1: lift_partials<real, N, 1, CM>(ne, L); break;
      case 2: lift_partials<real, N, 2, CM>(ne, L); break;
      case 3: lift_partials<real, N, 3, CM>(ne, L); break;
      default: lift_partials<real, N, 4, CM>(ne, L); break;
    }
  } else {
    lift_partials<real, N, DefaultParts<real, N>::value, CM>(ne, L);
  }
  __syncthreads();
  // rhs = -Minv y; store it, or do the LSRK update
  const size_t splane = size_t(d.K) * Np;
  real *uh = static_cast<real *>(d.uh);
  real *du = static_cast<real *>(d.du);
  real *rhs_out = static_cast<real *>(MULTI ? nullptr : a.ext_rhs);
  const real ra = real(a.rk_a), rdt = real(d.dt), rb = real(a.rk_b);
  if constexpr (WADG) {            // first factor into the residual block (dead after the lift)
    wadg_first<real, N>(ne, L, L.T, L.R);
    __syncthreads();
  }
  // one task per (field, element, mode)
  for (int i = tid; i < 3 * ne * Np; i += nth) {
    const FieldTask<Np> k(i, ne * Np);
    real rr;
    if constexpr (WADG) {
      rr = -wadg_second<real, N>(L, L.R + __umul24(unsigned(k.c), unsigned(ne * Nq)) +
                                        __umul24(unsigned(k.e), unsigned(Nq)), k.j);
    } else {
      const real *Mi = L.Minv + __umul24(unsigned(k.r), unsigned(Np));   // row (e, j) of Minv_e
      const real *Tc = L.T + (i - k.j);                                  // T[c][e][0..Np)
      real ra0 = 0, ra1 = 0;
#pragma unroll 32
      for (int m = 0; m + 1 < Np; m += 2) {
        ra0 -= Mi[m] * Tc[m];
        ra1 -= Mi[m + 1] * Tc[m + 1];
      }
      if (Np & 1) ra0 -= Mi[Np - 1] * Tc[Np - 1];
      rr = ra0 + ra1;
    }
    // global index: field c's plane, the tile's first element, then r (zero-extended)
    const size_t o = size_t(unsigned(k.c)) * splane + size_t(k0) * Np + unsigned(k.r);
    if (mode == kRhs) {
      rhs_out[o] = rr;
    } else {
      const real dn = ra * L.DU[i] + rdt * rr;
      const real un = L.U[i] + rb * dn;
      if (!keep) {
        du[o] = dn;
        uh[o] = un;
      }
      L.DU[i] = dn;
      L.U[i] = un;
    }
  }
  if (mode == kStage) {
    __syncthreads();
    project_tile<real, N, CM, WADG>(d, k0, ne, L, static_cast<real *>(d.ut[a.out_buf]),
                              static_cast<real *>(d.nbx[a.out_buf]), a.flag, MULTI && a.progress != nullptr, res);
  }
  return true;
}



// Persistent stage kernel: block b walks a contiguous range of tiles.  Blocks are dealt
// to the XCDs round-robin, so block b's range is chosen as range number
// (b mod kXcds) * (gridDim / kXcds) + b / kXcds: each XCD owns a contiguous run of tiles.
// The reference-operator block stays in LDS and is reloaded only when the degree changes.
// With a.progress set, the launch runs a.nstages RK stages: each block takes its tiles
// through stage s before stage s + 1, and a tile starts a stage once its face neighbours'
// tiles have finished the previous one (see wait_neighbours), which the co-residency of
// all workgroups (cooperative launch) makes safe.  A wait that gives up sets flag bit 1
// and ends the workgroup; its neighbours' waits then give up in turn.
// V1: the build that also holds the variant-1 element kinds (N+2 points per direction and
// per face); launches whose instances are all of variant 0 use the build without them,
// whose register allocation those larger kinds do not affect.  SHAPES: see stage_tile
// (built with vector-ALU contractions and variant-0 kinds only).  KIND: a build for one
// variant-0 kind alone (vector-ALU contractions, default shapes), used when every instance
// is of that kind: its registers are allocated for that kind's code only (FP32 N=3: 95
// VGPRs and 86 scalar spills against 122 and 105 for the build of all kinds).
// Residency probe of a multi-stage grid (kProbe): every workgroup counts itself in and waits,
// with a bounded spin, until the whole grid has; a wait that gives up sets flag bit 2.  Run
// once at bind with the grid, workgroup size and LDS of the multi-stage launches: if every
// workgroup was resident at once, those launches go out as ordinary launches, else as
// cooperative ones.  The count is a word of the flag block of its own.
__device__ __forceinline__ void residency_probe(const StageArgs &a) {
  if (threadIdx.x == 0) {
    int32_t *count = a.flag + kProbeWord;
    __hip_atomic_fetch_add(count, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    int spins = 0;
    while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < int(gridDim.x)) {
      if (++spins > a.spin_limit) {
        atomicOr(a.flag, 4);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
}

template <typename real, int CM, bool WADG, bool MULTI, bool V1, bool SHAPES, int KIND = 0>
__global__ void __launch_bounds__(kBlockWide) __attribute__((amdgpu_waves_per_eu(4)))
stage_kernel(StageArgs a) {
  if (MULTI && a.mode == kProbe) {
    residency_probe(a);
    return;
  }
  extern __shared__ __align__(16) unsigned char smem_raw[];
  real *sm = reinterpret_cast<real *>(smem_raw);
  real *tile = sm + a.ref_words_max;
  const int G = int(gridDim.x);
  const int chunk = (int(blockIdx.x) % kXcds) * (G / kXcds) + int(blockIdx.x) / kXcds;
  const int t0 = a.ranges ? read_const(a.ranges, chunk) : int((long long)chunk * a.ntiles / G);
  const int t1 = a.ranges ? read_const(a.ranges, chunk + 1) : int((long long)(chunk + 1) * a.ntiles / G);
  // MULTI: the multi-stage instantiation; the per-stage one compiles without the waits,
  // resident tiles and device-coherent pushes (and keeps the registers they would cost)
  const bool multi = MULTI && a.progress != nullptr;
  // resident: the launch gives this workgroup at most one tile (cost-balanced ranges can
  // still give a workgroup two; that one then re-reads its tiles every stage)
  const bool resident = multi && a.resident && t1 - t0 <= 1;
  const int nst = multi ? a.nstages : 1;
  int loaded_N = 0;
  for (int s = 0; s < nst; ++s) {
    StageArgs as = a;
    if (multi) {
      as.mode = kStage;
      as.in_buf = (a.in_buf + s) & 1;
      as.out_buf = 1 - as.in_buf;
      as.rk_a = a.rk_a5[s % 5];
      as.rk_b = a.rk_b5[s % 5];
    }
    for (int t = t0; t < t1; ++t) {
      const int res = resident ? kResident | (s > 0 ? kResMid : 0) | (s == nst - 1 ? kResLast : 0) : 0;
      // non-resident tiles wait before the stage (they re-read their neighbours' values in
      // the fetch); resident ones inside it, after their pair loop
      if (multi && s > 0 && !(res & kResMid) && !wait_neighbours(a, t, a.stage0 + s)) {
        if (threadIdx.x == 0) atomicOr(a.flag, 2);
        return;
      }
      const Tile tl = read_const(a.tiles, t);
      const InstDesc &d = read_const(a.desc, tl.inst);
      if (d.N != loaded_N) {
        __syncthreads();
        const real *ref = static_cast<const real *>(d.ref);
        const int words = ref_words(d.N);
        for (int i = threadIdx.x; i < words; i += blockDim.x) sm[i] = ref[i];
        loaded_N = d.N;
      }
      bool ok = true;
#define ESDG_STAGE_CASE(D) \
  case D: ok = stage_tile<real, D, CM, WADG, MULTI, SHAPES>(as, d, tl.k0, tl.ne, sm, tile, res, t, a.stage0 + s); break;
      if constexpr (KIND != 0) {     // every tile is of this kind (the host's choice of kernel)
        switch (d.N) {
          ESDG_STAGE_CASE(KIND)
          default: break;
        }
      } else if constexpr (V1) {
        switch (d.N) {
          ESDG_STAGE_CASE(1) ESDG_STAGE_CASE(2) ESDG_STAGE_CASE(3) ESDG_STAGE_CASE(4) ESDG_STAGE_CASE(5)
          ESDG_STAGE_CASE(9) ESDG_STAGE_CASE(10) ESDG_STAGE_CASE(11) ESDG_STAGE_CASE(12) ESDG_STAGE_CASE(13)
          default: break;
        }
      } else {
        switch (d.N) {
          ESDG_STAGE_CASE(1) ESDG_STAGE_CASE(2) ESDG_STAGE_CASE(3) ESDG_STAGE_CASE(4) ESDG_STAGE_CASE(5)
          default: break;
        }
      }
#undef ESDG_STAGE_CASE
      if (!ok) {
        if (threadIdx.x == 0) atomicOr(a.flag, 2);
        return;
      }
      if (multi) {
        publish(a, t, a.stage0 + s + 1);
        __builtin_amdgcn_s_setprio(0);
      }
      else __syncthreads();
    }
  }
}

// FP64 diagnostics per tile: mass (3), entropy, entropy rate, sum |entropy-rate terms|.
// Everything but the state and the RHS (widened exactly from the bulk precision) is double:
// V_q, w J and the bathymetry come from double copies kept for the diagnostics.
template <typename real, int D>
__device__ void diag_tile(const InstDesc &d, int k0, int ne, double *acc) {
  constexpr int Np = dim_Np(D), Nq = dim_Nq(D), Nh = dim_Nh(D);
  const real *uh = static_cast<const real *>(d.uh);
  const real *rh = static_cast<const real *>(d.rhs_scratch);
  const double *wJq = static_cast<const double *>(d.wJq);
  const size_t splane = size_t(d.K) * Np;
  const double g = d.g;
  for (int i = threadIdx.x; i < ne * Nq; i += blockDim.x) {
    const int e = i / Nq, q = i - e * Nq, k = k0 + e;
    double u[3] = {0, 0, 0}, r[3] = {0, 0, 0};
    if constexpr (key_sbp(D)) {    // nodal state: the values at the volume nodes themselves
      for (int c = 0; c < 3; ++c) {
        u[c] = double(uh[c * splane + size_t(k) * Np + q]);
        r[c] = double(rh[c * splane + size_t(k) * Np + q]);
      }
    } else {
      for (int j = 0; j < Np; ++j) {
        const double v = d.Vqd[q * Np + j];
        for (int c = 0; c < 3; ++c) {
          u[c] += v * double(uh[c * splane + size_t(k) * Np + j]);
          r[c] += v * double(rh[c * splane + size_t(k) * Np + j]);
        }
      }
    }
    const double w = wJq[size_t(k) * Nq + q], b = d.bd[size_t(k) * Nh + q];
    const double h = u[0] + (d.Href - b), uu = u[1] / h, vv = u[2] / h;
    acc[0] += w * h;
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
  const Tile tl = read_const(a.tiles, t);
  const InstDesc &d = read_const(a.desc, tl.inst);
  double acc[6] = {0, 0, 0, 0, 0, 0};
  switch (d.N) {
#define ESDG_DIAG_CASE(D) \
  case D: diag_tile<real, D>(d, tl.k0, tl.ne, acc); break;
    ESDG_DIAG_CASE(1) ESDG_DIAG_CASE(2) ESDG_DIAG_CASE(3) ESDG_DIAG_CASE(4) ESDG_DIAG_CASE(5)
    ESDG_DIAG_CASE(9) ESDG_DIAG_CASE(10) ESDG_DIAG_CASE(11) ESDG_DIAG_CASE(12) ESDG_DIAG_CASE(13)
    ESDG_DIAG_CASE(17) ESDG_DIAG_CASE(18) ESDG_DIAG_CASE(19) ESDG_DIAG_CASE(20)
#undef ESDG_DIAG_CASE
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

// The rest depth Href - b of every tile of an instance, rounded once from double into the
// static block (Href changes at every set_state).  One workgroup per tile.
template <typename real>
__global__ void __launch_bounds__(kBlock) rest_depth_kernel(DiagArgs a) {
  const int t = blockIdx.x;
  if (t >= a.ntiles) return;
  const Tile tl = read_const(a.tiles, t);
  const InstDesc &d = read_const(a.desc, tl.inst);
  const int D = d.N, Nq = dim_Nq(D), Nh = dim_Nh(D), ne = tl.ne;
  const bool wadg = a.wadg != 0;
  real *st = static_cast<real *>(const_cast<void *>(d.stat)) + size_t(tl.k0) * stat_words(D, wadg);
  // modal kinds: Href - b at the volume nodes, then at the hybrid nodes, after the mass data
  // and w J; DG-SBP: at the volume nodes, after 1/(w J)
  real *dq = st + ne * (key_sbp(D) ? Nq : mass_words(D, wadg) + Nq);
  real *dh = dq + ne * Nq;
  for (int i = threadIdx.x; i < ne * Nq; i += blockDim.x) {
    const int e = i / Nq, q = i - e * Nq;
    dq[i] = real(d.Href - d.bd[size_t(tl.k0 + e) * Nh + q]);
  }
  if (!key_sbp(D))
    for (int i = threadIdx.x; i < ne * Nh; i += blockDim.x) {
      const int e = i / Nh, n = i - e * Nh;
      dh[i] = real(d.Href - d.bd[size_t(tl.k0 + e) * Nh + n]);
    }
}

// ---------------------------------------------------------------- DG-SBP (Section 3)
// The DG-SBP scheme with traditional SBP operators obtained from the hybridized ones
// (Section 3.2): Q_SBP = [I; I_f]^T Q_h [I; I_f] on a volume rule whose boundary nodes are
// the face nodes, diagonal mass matrix W J, nodal state at the volume nodes, no entropy
// projection.  Per element,
//   (W J) du/dt = -[I; I_f]^T r_h,
// where r_h is the hybridized residual of the modal kernel (skew form, zero block skipped,
// folded source, interface terms) evaluated with the face values taken from the volume
// nodes they coincide with: each face row is added to its volume node's row.

// LDS carve-up of one DG-SBP tile (see tile_words()).
template <typename real, int D>
struct LdsSbp {
  static constexpr int Nq = dim_Nq(D), Nfq = dim_Nfq(D), Nh = dim_Nh(D);
  real *ref, *ST, *FT, *wf, *nr, *ns, *fvol, *vface;
  real *rec, *R, *nb, *U, *DU, *iwJ, *dep, *geo;
  int32_t *pp;
  __device__ LdsSbp(real *sm, real *tile, int E) {
    ref = sm;
    ST = ref;
    FT = ST + 2 * Nh * Nq;
    wf = FT + 2 * Nq * Nfq;
    nr = wf + Nfq;
    ns = nr + Nfq;
    fvol = ns + Nfq;              // volume node of face node f (integer-valued reals)
    vface = fvol + Nfq;           // face node of volume node n, or -1
    rec = tile;
    R = rec + E * rec_stride(D);  // two column-part partials [2][3][E][Nh]
    nb = R + 6 * E * Nh;
    U = nb + 4 * E * Nfq;
    DU = U + 3 * E * Nq;
    iwJ = DU + 3 * E * Nq;        // static block: 1/(w J) | rest depth | metrics [4][E][Nq] | push targets
    dep = iwJ + E * Nq;
    geo = dep + E * Nq;
    pp = reinterpret_cast<int32_t *>(geo + 4 * E * Nq);
  }
};

// Face values (h, u, v, H - Href) of the tile's state, pushed into the neighbours' slots (a
// reflective wall node, Section 2.9, writes the mirror state into its own slot).
template <typename real, int D>
__device__ __forceinline__ void sbp_push(const InstDesc &d, int ne, LdsSbp<real, D> &L, real *nbx_out, int32_t *flag) {
  constexpr int Nq = dim_Nq(D), Nfq = dim_Nfq(D);
  bool bad = false;
  for (int i = phase_tid(); i < ne * Nfq; i += blockDim.x) {
    const int e = i / Nfq, f = i - e * Nfq, j = e * Nq + int(L.fvol[f]);
    const double eta = L.U[j], hu = L.U[ne * Nq + j], hv = L.U[2 * ne * Nq + j];
    const double h = eta + double(L.dep[j]);
    const double u = hu / h, v = hv / h;
    double pu = u, pv = v;
    const uint32_t tgt = uint32_t(L.pp[i]);
    if (tgt & kPushWall) {
      const double nr = double(L.nr[f]), ns = double(L.ns[f]);
      const double nx = double(L.geo[j]) * nr + double(L.geo[ne * Nq + j]) * ns;
      const double ny = double(L.geo[2 * ne * Nq + j]) * nr + double(L.geo[3 * ne * Nq + j]) * ns;
      const double c = 2.0 * (u * nx + v * ny) / (nx * nx + ny * ny);
      pu = u - c * nx;
      pv = v - c * ny;
    }
    typedef real real4 __attribute__((ext_vector_type(4)));
    const real4 val = {real(h), real(pu), real(pv), real(eta)};
    *reinterpret_cast<real4 *>(nbx_out + size_t(tgt & ~kPushWall) * 4) = val;
    bad |= bad_value(h, hu, hv);
  }
  if (bad) atomicOr(flag, 1);
}

template <typename real, int D>
__device__ __forceinline__ void sbp_tile(const StageArgs &a, const InstDesc &d, int k0, int ne, real *sm, real *tile) {
  constexpr int Nq = dim_Nq(D), Nfq = dim_Nfq(D), Nh = dim_Nh(D), SW = stat_words(D);
  constexpr int W = sizeof(real) / 4;
  LdsSbp<real, D> L(sm, tile, ne);
  const int tid = phase_tid(), nth = blockDim.x;
  const size_t splane = size_t(d.K) * Nq;
  auto words = [](const void *p) { return static_cast<const uint32_t *>(p); };
  auto lwords = [](real *p) { return reinterpret_cast<uint32_t *>(p); };
  {                                // fetch: state, RK register, static block, neighbour values
    const real *src = static_cast<const real *>(a.ext_state ? a.ext_state : d.uh);
    const real *du = static_cast<const real *>(d.du);
    for (int c = 0; c < 3; ++c) {
      async_copy_words(lwords(L.U + c * ne * Nq), words(src + c * splane + size_t(k0) * Nq), ne * Nq * W);
      if (a.mode == kStage)
        async_copy_words(lwords(L.DU + c * ne * Nq), words(du + c * splane + size_t(k0) * Nq), ne * Nq * W);
    }
    async_copy_words(lwords(L.iwJ), words(static_cast<const real *>(d.stat) + size_t(k0) * SW), ne * SW * W);
    if (a.mode != kProject) {
      const void *nbx = a.ext_nbx ? a.ext_nbx : d.nbx[a.in_buf];
      async_copy_words(lwords(L.nb), words(static_cast<const real *>(nbx) + size_t(k0) * Nfq * 4), ne * Nfq * 4 * W);
    }
    __builtin_amdgcn_s_waitcnt(0);
  }
  __syncthreads();
  real *nbx_out = static_cast<real *>(a.ext_nbx ? a.ext_nbx : d.nbx[a.out_buf]);
  if (a.mode == kProject) {
    sbp_push<real, D>(d, ne, L, nbx_out, a.flag);
    return;
  }
  // node records of the volume nodes, from the nodal state (h in double from eta and the
  // rest depth; H - Href is eta itself)
  const real g = real(d.g);
  bool bad = false;
  for (int i = tid; i < ne * Nq; i += nth) {
    const double eta = L.U[i], hu = L.U[ne * Nq + i], hv = L.U[2 * ne * Nq + i];
    const double h = eta + double(L.dep[i]);
    const double u = hu / h, v = hv / h;
    const int e = i / Nq, q = i - e * Nq;
    typedef real real4 __attribute__((ext_vector_type(4)));
    real4 *rec = reinterpret_cast<real4 *>(L.rec + e * rec_stride(D) + q * kNodeRec);
    rec[0] = real4{real(0.5 * hu), real(0.5 * hv), real(0.5 * u), real(0.5 * v)};
    rec[1] = real4{L.geo[i], L.geo[ne * Nq + i], L.geo[2 * ne * Nq + i], L.geo[3 * ne * Nq + i]};
    rec[2] = real4{real(0.5) * g * real(h), real(eta), real(h), real(0)};
    bad |= bad_value(h, hu, hv);
  }
  if (bad) atomicOr(a.flag, 1);
  __syncthreads();
  // the face nodes' records are those of the volume nodes they coincide with
  for (int i = tid; i < ne * Nfq * 3; i += nth) {
    const int quad = i % 3, ef = i / 3, e = ef / Nfq, f = ef - e * Nfq;
    typedef real real4 __attribute__((ext_vector_type(4)));
    const real4 *srcr = reinterpret_cast<const real4 *>(L.rec + e * rec_stride(D) + int(L.fvol[f]) * kNodeRec);
    reinterpret_cast<real4 *>(L.rec + e * rec_stride(D) + (Nq + f) * kNodeRec)[quad] = srcr[quad];
  }
  __syncthreads();
  residual_tile<real, D, 1, 2>(d, ne, L, true);
  __syncthreads();
  // du/dt = -(W J)^{-1} [I; I_f]^T r_h; store it, or do the LSRK update
  real *uh = static_cast<real *>(d.uh);
  real *du = static_cast<real *>(d.du);
  real *rhs_out = static_cast<real *>(a.ext_rhs);
  const real ra = real(a.rk_a), rdt = real(d.dt), rb = real(a.rk_b);
  for (int i = tid; i < 3 * ne * Nq; i += nth) {
    const int c = (i >= ne * Nq) + (i >= 2 * ne * Nq), j = i - c * ne * Nq, e = j / Nq, n = j - e * Nq;
    const real *R0 = L.R + c * ne * Nh + e * Nh, *R1 = R0 + 3 * ne * Nh;
    real r = R0[n] + R1[n];
    const int vf = int(L.vface[n]);
    if (vf >= 0) {                 // face rows have face_chunks<D, 2>() chunk partials
      r += R0[Nq + vf];
      if constexpr (face_chunks<D, 2>() > 1) r += R1[Nq + vf];
    }
    const real rr = -r * L.iwJ[j];
    const size_t o = size_t(c) * splane + size_t(k0) * Nq + j;
    if (a.mode == kRhs) {
      rhs_out[o] = rr;
    } else {
      const real dn = ra * L.DU[i] + rdt * rr;
      const real un = L.U[i] + rb * dn;
      du[o] = dn;
      uh[o] = un;
      L.U[i] = un;
    }
  }
  if (a.mode == kStage) {
    __syncthreads();
    sbp_push<real, D>(d, ne, L, nbx_out, a.flag);
  }
}

// One launch per RK stage (or per projection / RHS) for every DG-SBP tile; persistent,
// XCD-aligned chunks as in stage_kernel.
template <typename real>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
sbp_stage_kernel(StageArgs a) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  real *sm = reinterpret_cast<real *>(smem_raw);
  real *tile = sm + a.ref_words_max;
  const int G = int(gridDim.x);
  const int chunk = (int(blockIdx.x) % kXcds) * (G / kXcds) + int(blockIdx.x) / kXcds;
  const int t0 = a.ranges ? read_const(a.ranges, chunk) : int((long long)chunk * a.ntiles / G);
  const int t1 = a.ranges ? read_const(a.ranges, chunk + 1) : int((long long)(chunk + 1) * a.ntiles / G);
  int loaded = 0;
  for (int t = t0; t < t1; ++t) {
    const Tile tl = read_const(a.tiles, t);
    const InstDesc &d = read_const(a.desc, tl.inst);
    if (d.N != loaded) {
      __syncthreads();
      const real *ref = static_cast<const real *>(d.ref);
      const int words = ref_words(d.N);
      for (int i = threadIdx.x; i < words; i += blockDim.x) sm[i] = ref[i];
      loaded = d.N;
    }
    switch (d.N) {
#define ESDG_SBP_CASE(N) \
  case make_key(N, 2): sbp_tile<real, make_key(N, 2)>(a, d, tl.k0, tl.ne, sm, tile); break;
      ESDG_SBP_CASE(1) ESDG_SBP_CASE(2) ESDG_SBP_CASE(3) ESDG_SBP_CASE(4)
#undef ESDG_SBP_CASE
      default: break;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- instantiation units
// This file is compiled once per (precision, mass inverse) with ESDG_UNIT_REAL and
// ESDG_UNIT_WADG defined, instantiating the stage kernels of that combination only, and
// once with ESDG_UNIT_HOST for the DG-SBP, diagnostics and rest-depth kernels and the host
// launchers; the five objects compile in parallel.  Each unit exports the stage kernels of
// its combination by contraction mode and launch kind.
#define ESDG_CAT4(a, b, c, d) a##b##c##d
#define ESDG_UNIT_FN(R, W) ESDG_CAT4(stage_fn_unit_, R, _, W)
const void *stage_fn_unit_float_0(int cm, bool multi, bool v1, bool shapes, int kind);
const void *stage_fn_unit_float_1(int cm, bool multi, bool v1, bool shapes, int kind);
const void *stage_fn_unit_double_0(int cm, bool multi, bool v1, bool shapes, int kind);
const void *stage_fn_unit_double_1(int cm, bool multi, bool v1, bool shapes, int kind);

#if defined(ESDG_UNIT_REAL)
template <bool V1>
static const void *unit_fn(int cm, bool multi) {
  using real = ESDG_UNIT_REAL;
  constexpr bool W = ESDG_UNIT_WADG != 0;
  if constexpr (std::is_same<real, double>::value) {
    if (cm == kMfmaNative)
      return multi ? reinterpret_cast<const void *>(&stage_kernel<double, kMfmaNative, W, true, V1, false>)
                   : reinterpret_cast<const void *>(&stage_kernel<double, kMfmaNative, W, false, V1, false>);
    return multi ? reinterpret_cast<const void *>(&stage_kernel<double, kValu, W, true, V1, false>)
                 : reinterpret_cast<const void *>(&stage_kernel<double, kValu, W, false, V1, false>);
  } else {
    if (cm == kMfmaBf16x3)
      return multi ? reinterpret_cast<const void *>(&stage_kernel<float, kMfmaBf16x3, W, true, V1, false>)
                   : reinterpret_cast<const void *>(&stage_kernel<float, kMfmaBf16x3, W, false, V1, false>);
    if (cm == kMfmaNative)
      return multi ? reinterpret_cast<const void *>(&stage_kernel<float, kMfmaNative, W, true, V1, false>)
                   : reinterpret_cast<const void *>(&stage_kernel<float, kMfmaNative, W, false, V1, false>);
    return multi ? reinterpret_cast<const void *>(&stage_kernel<float, kValu, W, true, V1, false>)
                 : reinterpret_cast<const void *>(&stage_kernel<float, kValu, W, false, V1, false>);
  }
}
template <bool MULTI>
static const void *kind_fn(int kind) {
  using real = ESDG_UNIT_REAL;
  constexpr bool W = ESDG_UNIT_WADG != 0;
  switch (kind) {
    case 1: return reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, MULTI, false, false, 1>);
    case 2: return reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, MULTI, false, false, 2>);
    case 3: return reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, MULTI, false, false, 3>);
    case 4: return reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, MULTI, false, false, 4>);
    case 5: return reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, MULTI, false, false, 5>);
    default: return nullptr;
  }
}
const void *ESDG_UNIT_FN(ESDG_UNIT_REAL, ESDG_UNIT_WADG)(int cm, bool multi, bool v1, bool shapes, int kind) {
  using real = ESDG_UNIT_REAL;
  constexpr bool W = ESDG_UNIT_WADG != 0;
  // one variant-0 kind, vector-ALU contractions and its default shape: that kind's own build
  if (kind >= 1 && kind <= 5 && cm == kValu && !v1 && !shapes) return multi ? kind_fn<true>(kind) : kind_fn<false>(kind);
  if (shapes)                      // vector-ALU contractions, variant-0 kinds
    return multi ? reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, true, false, true>)
                 : reinterpret_cast<const void *>(&stage_kernel<real, kValu, W, false, false, true>);
  return v1 ? unit_fn<true>(cm, multi) : unit_fn<false>(cm, multi);
}
#endif

#if defined(ESDG_UNIT_HOST)
// ---------------------------------------------------------------- host launchers

// The stage kernel for a precision, contraction mode, mass inverse and launch kind (one
// launch per stage, or all stages of a step call in one multi-stage launch).  One launch
// per stage runs the per-stage instantiation, built without the waits, resident tiles and
// coherent pushes: its scalar registers spill far less (FP32 all kinds 36 against 102),
// and each reload of a spilled one is a vector instruction.  (FP32 once ran its
// multi-stage instantiation for single stages as well, measured faster then; with the
// single-kind builds and the current task layout the per-stage one is faster on one box:
// N=1..5 by 11, 7.5, 6.5, 2 and 2.3 %, the mixed-degree ensemble by 5 %.)
static const void *stage_fn(bool fp64, int cm, bool wadg, bool multi, bool v1, bool shapes, int kind) {
  if (fp64)
    return wadg ? stage_fn_unit_double_1(cm, multi, v1, shapes, kind) : stage_fn_unit_double_0(cm, multi, v1, shapes, kind);
  return wadg ? stage_fn_unit_float_1(cm, multi, v1, shapes, kind) : stage_fn_unit_float_0(cm, multi, v1, shapes, kind);
}

static const void *sbp_fn(bool fp64) {
  return fp64 ? reinterpret_cast<const void *>(&sbp_stage_kernel<double>)
              : reinterpret_cast<const void *>(&sbp_stage_kernel<float>);
}

// Workgroups of the stage kernel (the DG-SBP kernel with sbp) that stay resident on the
// whole device.
hipError_t stage_max_blocks(bool fp64, int cm, bool wadg, bool sbp, bool v1, bool shapes, int kind, size_t lds_bytes,
                            int block, int *out) {
  int dev = 0, ncu = 0, per_cu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // The occupancy query does not round the LDS request up to the allocation granule; a
  // workgroup count it reports can then fail to fit, and the persistent grid's surplus
  // blocks only start when others finish (for a multi-stage launch, which needs every
  // workgroup resident at once, their neighbours then wait for stages that cannot come).
  // So cap it with 1 KiB granules of the CU's LDS, counting the kernel's own static LDS
  // (the multi-stage build's workgroup reduction) on top of the dynamic request.  Both
  // launch kinds use the same grid: the smaller residency of the two builds.
  int lds_cu = 0;
  e = hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev);
  if (e != hipSuccess) return e;
  for (int multi = 0; multi < 2; ++multi) {
    const void *fn = sbp ? sbp_fn(fp64) : stage_fn(fp64, cm, wadg, multi != 0, v1, shapes, kind);
    int n = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, fn, block, lds_bytes);
    if (e != hipSuccess) return e;
    hipFuncAttributes fa{};
    e = hipFuncGetAttributes(&fa, fn);
    if (e != hipSuccess) return e;
    const size_t granule = 1024, total = lds_bytes + fa.sharedSizeBytes;
    const size_t need = (total + granule - 1) / granule * granule;
    if (need > 0 && lds_cu > 0) n = std::min<long long>(n, (long long)(size_t(lds_cu) / need));
    per_cu = multi ? std::min(per_cu, n) : n;
  }
  *out = ncu * (per_cu > 0 ? per_cu : 1);
  return hipSuccess;
}

hipError_t set_stage_lds_limit(bool fp64, int cm, bool wadg, bool sbp, bool v1, bool shapes, int kind,
                               size_t lds_bytes) {
  if (sbp) return hipFuncSetAttribute(sbp_fn(fp64), hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
  hipError_t e = hipFuncSetAttribute(stage_fn(fp64, cm, wadg, false, v1, shapes, kind),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_bytes));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(stage_fn(fp64, cm, wadg, true, v1, shapes, kind), hipFuncAttributeMaxDynamicSharedMemorySize,
                             int(lds_bytes));
}

// Persistent grid: at most max_blocks (what stays resident), at most one block per tile,
// always a whole number of XCD rounds (blocks whose range is empty just exit).
int stage_grid(int ntiles, int max_blocks);
int stage_grid(int ntiles, int max_blocks) {
  int g = ntiles < max_blocks ? ntiles : max_blocks;
  return ((g + kXcds - 1) / kXcds) * kXcds;
}

hipError_t launch_stage(bool fp64, bool sbp, const StageArgs &a, int max_blocks, size_t lds_bytes, int block,
                        hipStream_t stream) {
  if (a.ntiles <= 0) return hipSuccess;
  const int grid = stage_grid(a.ntiles, max_blocks);
  StageArgs arg = a;
  void *params[] = {&arg};
  return hipLaunchKernel(sbp ? sbp_fn(fp64) : stage_fn(fp64, a.contraction, a.wadg != 0, false, a.v1 != 0, a.shapes != 0, a.kind),
                         dim3(grid),
                         dim3(sbp ? kBlock : block), params, lds_bytes, stream);
}

// Multi-stage launch: every workgroup of the grid must be resident at once (tiles wait on
// their neighbours' progress), which the cooperative launch guarantees or refuses.
hipError_t launch_stage_fused(bool fp64, const StageArgs &a, int max_blocks, size_t lds_bytes, int block,
                              bool cooperative, hipStream_t stream) {
  if (a.ntiles <= 0) return hipSuccess;
  const int grid = stage_grid(a.ntiles, max_blocks);
  StageArgs arg = a;
  void *params[] = {&arg};
  const void *fn = stage_fn(fp64, a.contraction, a.wadg != 0, true, a.v1 != 0, a.shapes != 0, a.kind);
  if (cooperative) return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), params, lds_bytes, stream);
  return hipLaunchKernel(fn, dim3(grid), dim3(block), params, lds_bytes, stream);
}

hipError_t launch_diag(bool fp64, const DiagArgs &a, hipStream_t stream) {
  if (a.ntiles <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(diag_kernel<double>, dim3(a.ntiles), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(diag_kernel<float>, dim3(a.ntiles), dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

// Rest depth of the tiles a.tiles[0 .. a.ntiles) (one instance's) into their static blocks.
hipError_t launch_rest_depth(bool fp64, const DiagArgs &a, hipStream_t stream) {
  if (a.ntiles <= 0) return hipSuccess;
  if (fp64)
    hipLaunchKernelGGL(rest_depth_kernel<double>, dim3(a.ntiles), dim3(kBlock), 0, stream, a);
  else
    hipLaunchKernelGGL(rest_depth_kernel<float>, dim3(a.ntiles), dim3(kBlock), 0, stream, a);
  return hipGetLastError();
}

#endif  // ESDG_UNIT_HOST

}  // namespace esdg
