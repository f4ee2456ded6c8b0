// Types shared by the HIP kernels and the host runtime of the ESDG shallow-water library.
#pragma once

#include <cstddef>
#include <cstdint>

namespace esdg {

constexpr int kMaxN = 5;
constexpr int kBlock = 256;        // threads per workgroup (4 wave64s)
constexpr int kNodeRec = 12;       // per hybrid node in LDS: hu/2 hv/2 u/2 v/2 | rxJ sxJ ryJ syJ | gh/2 dH h -
                                   // (three aligned quads, so a column is read with two 16-byte loads)
constexpr int kXcds = 8;           // MI355X accelerator complex dies (each with its own L2)

// Push-target flag: the face node lies on a reflective wall (Section 2.9); its projection
// writes the mirror state into its own neighbour slot (the target's other bits).
constexpr uint32_t kPushWall = 0x80000000u;

__host__ __device__ constexpr int dim_Np(int N) { return (N + 1) * (N + 2) / 2; }
__host__ __device__ constexpr int dim_Nq(int N) { return (N + 1) * (N + 1); }
__host__ __device__ constexpr int dim_Nfq(int N) { return 3 * (N + 1); }
__host__ __device__ constexpr int dim_Nh(int N) { return dim_Nq(N) + dim_Nfq(N); }

// Relative cost of one element of degree N in a stage (flux-differencing and contraction
// flops), used to balance persistent workgroups over mixed-degree tile lists.
__host__ __device__ constexpr long long elem_cost(int N) {
  return 35LL * (dim_Nq(N) * (dim_Nq(N) - 1) / 2 + dim_Nq(N) * dim_Nfq(N)) +
         6LL * (2 * dim_Nq(N) * dim_Np(N) + 2 * dim_Np(N) * dim_Np(N) + 2 * dim_Nh(N) * dim_Np(N));
}

// Reference-operator block of degree N, stored contiguously in the bulk precision:
//   Vh [Nh][Np]
//   ST [Nh][Nq][2]  ST[n][m] = (S^r[m][n], S^s[m][n]) for volume rows m (column-major
//                   so one column's entries for consecutive rows are contiguous)
//   FT [Nq][Nfq][2] FT[n][f] = (-S^r[n][Nq+f], -S^s[n][Nq+f]): face row f, volume column n
//   wf [Nfq] | nr [Nfq] | ns [Nfq]
// where S^j = 1/2 (Qhat_h^j - Qhat_h^j^T) (its surface-surface block is zero).
__host__ __device__ constexpr int ref_words(int N) {
  return dim_Nh(N) * dim_Np(N) + 2 * dim_Nh(N) * dim_Nq(N) + 2 * dim_Nq(N) * dim_Nfq(N) + 3 * dim_Nfq(N);
}

// Reals per element of the mass-matrix data: the stored inverse (M_h^k)^{-1} [Np][Np], or,
// with the weight-adjusted inverse, the quadrature weights over J at the volume nodes [Nq].
__host__ __device__ constexpr int mass_words(int N, bool wadg) {
  return wadg ? dim_Nq(N) : dim_Np(N) * dim_Np(N);
}

// Words (of the bulk precision) of LDS one tile of E elements of degree N needs (the
// reference block is held separately, once per workgroup): node records [E][Nh][kNodeRec] | fetched u~ and metrics [8][E][Nh] |
// neighbour values [E][Nfq][4] | state, RK register [3][E][Np] each | mass data
// [E][mass_words] | w J [E][Nq] | b at volume nodes [E][Nq] | b at hybrid nodes [E][Nh] |
// push targets [E][Nfq] (int32, one word of the bulk precision each).
__host__ __device__ constexpr int tile_words(int N, int E, bool wadg = false) {
  return E * (dim_Nh(N) * kNodeRec + 8 * dim_Nh(N) + 4 * dim_Nfq(N) + 6 * dim_Np(N) +
                             mass_words(N, wadg) + 2 * dim_Nq(N) + dim_Nh(N) + dim_Nfq(N));
}

// Reals per element of the static per-tile block (see InstDesc::stat): the mass data, w J,
// b at the volume and at the hybrid nodes, and the face push targets (int32, one real-sized
// slot each).
__host__ __device__ constexpr int stat_words(int N, bool wadg = false) {
  return mass_words(N, wadg) + 2 * dim_Nq(N) + dim_Nh(N) + dim_Nfq(N);
}

// 32-bit words per thread of the static block that a stage stages through registers
// (issued after the tile's other copies have landed, stored to LDS after the residual),
// for float and for double tiles.
constexpr int kStatRegs = 8;
template <typename real> struct StatRegs { static constexpr int value = sizeof(real) == 4 ? kStatRegs : 4; };

// One instance as the kernels see it (device pointers into the bound workspace).
struct InstDesc {
  int32_t N, K, flux, pad0;
  double g, Href, dt, pad1;
  void *uh;            // [3][K][Np] modal state (eta = h + b - Href, hu, hv)
  void *du;            // [3][K][Np] LSRK register
  void *ut[3];         // entropy-projected h~, u~, v~, H~ - Href at the hybrid nodes, tile-blocked:
                       // the tile of elements k0..k0+ne-1 holds [4][ne][Nh] from real k0*4*Nh
                       // (two stage buffers + rhs scratch)
  void *nbx[3];        // [K][Nfq][4] the same four values at each face node's neighbour, written
                       // by the neighbour's projection (one per ut buffer)
  const void *geo;     // rxJ, sxJ, ryJ, syJ at the hybrid nodes, tile-blocked like ut
  const void *wJq;     // [K][Nq] w_q J (diagnostics)
  const void *bq;      // [K][Nq] bathymetry at volume nodes (diagnostics)
  const void *stat;    // static data in tile order: the tile of elements k0..k0+ne-1 holds, from
                       // real k0 * stat_words(N, wadg): the mass data [ne][mass_words] (Minv
                       // [Np][Np], or w/J at the volume nodes [Nq]) | w J [ne][Nq] | b [ne][Nq] |
                       // b [ne][Nh] | push targets [ne][Nfq] (int32 k'*Nfq + f' of the nbx slot
                       // that face node f fills, packed in the first ne*Nfq 32-bit words;
                       // kPushWall set on wall nodes, whose slot is their own)
  const void *ref;     // reference-operator block for this N
  void *rhs_scratch;   // [3][K][Np] used by the diagnostics
};

// A contiguous range of elements of one instance, processed by one workgroup.
struct Tile {
  int32_t inst, k0, ne, pad;
};

enum StageMode : int32_t {
  kProject = 0,   // state -> entropy-projected values (ut[out])
  kRhs = 1,       // ut[in] -> rhs (no update)
  kStage = 2      // ut[in] -> rhs -> LSRK update of uh, du -> project new uh to ut[out]
};

struct StageArgs {
  const InstDesc *desc;
  const Tile *tiles;
  int32_t ntiles;
  int32_t mode;
  int32_t ref_words_max;  // LDS words reserved for the reference block (largest degree)
  int32_t contraction;    // constant-matrix contractions: 0 VALU, 1 matrix cores in the bulk
                          // precision, 2 matrix cores with split-bf16 products
  int32_t wadg;           // 0: stored inverse mass matrices; 1: weight-adjusted inverse
  int32_t pad_w;
  const int32_t *ranges;  // optional [grid+1]: tile range of each block's chunk (cost-balanced);
                          // null means equal numbers of tiles per chunk
  int32_t in_buf, out_buf;
  double rk_a, rk_b;
  const void *ext_state;  // kProject: read this state instead of desc.uh (when non-null)
  void *ext_rhs;          // kRhs: write here
  void *ext_ut;           // kProject / kRhs: the projected values and the face slots of this
  void *ext_nbx;          // launch in these buffers instead of desc.ut / desc.nbx (when non-null;
                          // one instance per launch, layouts as desc.ut[b] and desc.nbx[b])
  int32_t *flag;          // bit 0: a non-physical value was seen; bit 1: a neighbour wait timed out
  // Multi-stage launch (progress != null; all workgroups co-resident): nstages kStage stages
  // starting at global stage index stage0, buffers alternating from in_buf, coefficients
  // rk_a5/rk_b5[stage mod 5].  Before a stage, a tile waits until every tile holding a face
  // neighbour has completed the previous one; after it, it publishes its count.
  int32_t *progress;      // [ntiles] stages completed by each tile (monotone over launches)
  const int32_t *nbr_off; // [ntiles + 1] CSR offsets into nbr_idx
  const int32_t *nbr_idx; // tiles (other than itself) holding a face neighbour of each tile
  int32_t stage0, nstages;
  int32_t spin_limit;     // polls of one neighbour count before the wait gives up
  int32_t resident;       // multi-stage launch with at most one tile per workgroup: the tile
                          // stays in LDS from its first stage to its last (see stage_tile)
  double rk_a5[5], rk_b5[5];
};

struct DiagArgs {
  const InstDesc *desc;
  const Tile *tiles;
  int32_t ntiles;
  int32_t pad;
  double *partials;       // [ntiles][6]
};

}  // namespace esdg
