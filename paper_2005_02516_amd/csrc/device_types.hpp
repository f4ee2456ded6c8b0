// Types shared by the HIP kernels and the host runtime of the ESDG shallow-water library.
#pragma once

#include <cstddef>
#include <cstdint>

namespace esdg {

constexpr int kMaxN = 5;
constexpr int kBlock = 256;        // threads per workgroup (4 wave64s)
constexpr int kBlockWide = 512;    // stage-kernel workgroups of launches whose kinds are all
                                   // wide (wide_kind): 8 wave64s sharing one reference block
constexpr int kNodeRec = 12;       // per hybrid node in LDS: hu/2 hv/2 u/2 v/2 | rxJ sxJ ryJ syJ | gh/2 dH h -
                                   // (three aligned quads, so a column is read with two 16-byte loads)
constexpr int kProbeWord = 16;     // int32 word of the flag block counting a residency probe
constexpr int kXcds = 8;           // MI355X accelerator complex dies (each with its own L2)

// Push-target flag: the face node lies on a reflective wall (Section 2.9); its projection
// writes the mirror state into its own neighbour slot (the target's other bits).
constexpr uint32_t kPushWall = 0x80000000u;

// Element kinds.  A key D = N | (variant << 3) names the degree N and the node sets the
// kernels are compiled for:
//   variant 0: volume rule of (N+1)^2 nodes (the Stroud collapsed rule, or a caller's rule of
//              at most that many nodes padded with zero-weight nodes), N+1 Gauss-Legendre
//              points per face;
//   variant 1: (N+2)^2 volume nodes (likewise), N+2 Gauss-Legendre points per face;
//   variant 2: the DG-SBP scheme of Section 3: a volume rule of sbp_nodes(N) nodes whose
//              boundary nodes are the N+1 Gauss-Legendre points of every face; the state is
//              the nodal values at the volume nodes.
// A plain degree N (variant 0) is its own key.
constexpr int kKeyShift = 3;
constexpr int kMaxKey = (2 << kKeyShift) | kMaxN;
__host__ __device__ constexpr int key_N(int D) { return D & ((1 << kKeyShift) - 1); }
__host__ __device__ constexpr int key_variant(int D) { return D >> kKeyShift; }
__host__ __device__ constexpr int make_key(int N, int variant) { return N | (variant << kKeyShift); }
__host__ __device__ constexpr bool key_sbp(int D) { return key_variant(D) == 2; }
// Nodes of the DG-SBP volume rules the kernels are compiled for (N = 1..4).
__host__ __device__ constexpr int sbp_nodes(int N) { return N == 1 ? 6 : N == 2 ? 10 : N == 3 ? 18 : N == 4 ? 22 : 0; }

__host__ __device__ constexpr int dim_modes(int D) { return (key_N(D) + 1) * (key_N(D) + 2) / 2; }
__host__ __device__ constexpr int dim_Nfp(int D) { return key_N(D) + 1 + (key_variant(D) == 1); }
__host__ __device__ constexpr int dim_Nq(int D) {
  return key_sbp(D) ? sbp_nodes(key_N(D)) : (key_N(D) + 1 + key_variant(D)) * (key_N(D) + 1 + key_variant(D));
}
// values per field and element of the state: modal coefficients, or nodal values (DG-SBP)
__host__ __device__ constexpr int dim_Np(int D) { return key_sbp(D) ? dim_Nq(D) : dim_modes(D); }
__host__ __device__ constexpr int dim_Nfq(int D) { return 3 * dim_Nfp(D); }
__host__ __device__ constexpr int dim_Nh(int D) { return dim_Nq(D) + dim_Nfq(D); }

// Operation count of one element of kind D in a stage: 35 FLOPs per unordered nonzero node
// pair of the flux differencing, and the projection and lift contractions.
__host__ __device__ constexpr long long elem_work(int D) {
  return 35LL * (dim_Nq(D) * (dim_Nq(D) - 1) / 2 + dim_Nq(D) * dim_Nfq(D)) +
         (key_sbp(D) ? 0LL
                     : 6LL * (2 * dim_Nq(D) * dim_Np(D) + 2 * dim_Np(D) * dim_Np(D) + 2 * dim_Nh(D) * dim_Np(D)));
}

// Relative cost of one element of kind D in a stage, for splitting the tiles of a
// mixed-degree launch into ranges of equal cost.  The operation count overstates the higher
// degrees (their phases keep more lanes busy), so the default-quadrature modal kinds take
// measured per-element stage times instead: single-degree meshes of 131072 elements, FP32,
// tuned tiles of 256-thread workgroups, relative to N=2 (0.87 ns) in hundredths; the other
// kinds scale their degree's figure by their operation count relative to it.
constexpr long long kStageCost[6] = {0, 46, 100, 182, 384, 724};
__host__ __device__ constexpr long long elem_cost(int D) {
  return kStageCost[key_N(D)] * elem_work(D) / elem_work(key_N(D));
}

// Reference-operator block of kind D, stored contiguously in the bulk precision:
//   Vh [Nh][Np]     (modal kinds only)
//   ST [Nh][Nq][2]  ST[n][m] = (S^r[m][n], S^s[m][n]) for volume rows m (column-major
//                   so one column's entries for consecutive rows are contiguous)
//   FT [Nq][Nfq][2] FT[n][f] = (-S^r[n][Nq+f], -S^s[n][Nq+f]): face row f, volume column n
//   wf [Nfq] | nr [Nfq] | ns [Nfq]
//   DG-SBP only: fvol [Nfq] (int32: the volume node at face node f) | vface [Nq] (int32:
//   the face node at volume node n, or -1)
// where S^j = 1/2 (Qhat_h^j - Qhat_h^j^T) (its surface-surface block is zero).
__host__ __device__ constexpr int ref_words(int D) {
  return (key_sbp(D) ? dim_Nfq(D) + dim_Nq(D) : dim_Nh(D) * dim_Np(D)) + 2 * dim_Nh(D) * dim_Nq(D) +
         2 * dim_Nq(D) * dim_Nfq(D) + 3 * dim_Nfq(D);
}

// Reals per element of the mass-matrix data: the stored inverse (M_h^k)^{-1} [Np][Np], or,
// with the weight-adjusted inverse, the quadrature weights over J at the volume nodes [Nq]
// (DG-SBP: the inverse of the diagonal mass matrix, 1/(w J) [Nq]).
__host__ __device__ constexpr int mass_words(int D, bool wadg) {
  return (wadg || key_sbp(D)) ? dim_Nq(D) : dim_Np(D) * dim_Np(D);
}

// Reals per element of the static per-tile block (see InstDesc::stat).  Modal kinds: the
// mass data, w J, the rest depth Href - b at the volume and at the hybrid nodes, and the
// face push targets (int32, one real-sized slot each).  DG-SBP: 1/(w J), the rest depth and
// the metric factors rxJ, sxJ, ryJ, syJ at the volume nodes, and the push targets.
__host__ __device__ constexpr int stat_words(int D, bool wadg = false) {
  return key_sbp(D) ? 6 * dim_Nq(D) + dim_Nfq(D)
                    : mass_words(D, wadg) + 2 * dim_Nq(D) + dim_Nh(D) + dim_Nfq(D);
}

// Tile shape of the residual phase: rows per thread R (it divides Nq and Nfq) and column
// parts P, packed as (R << 4) | P.  A task is (element, R rows, column part); the P partial
// sums of a row are added in the lift.
constexpr int kShapeDefault = 0;
__host__ __device__ constexpr int shape_rows(int shape) { return shape >> 4; }
__host__ __device__ constexpr int shape_parts(int shape) { return shape & 15; }
__host__ __device__ constexpr int make_shape(int R, int P) { return (R << 4) | P; }

// Kinds with many hybrid nodes (N=5, and N=4 with N+2 points): their reference block fills
// a quarter of a CU's LDS, so their launches run workgroups of kBlockWide threads (twice the
// elements sharing one copy of it), and their residual rows use balanced column chunks.
__host__ __device__ constexpr bool wide_kind(int D) { return !key_sbp(D) && dim_Nh(D) >= 50; }

// Balanced column chunks of the residual phase (the kinds with many hybrid nodes; see
// kernels.hip): volume rows (Nh columns) are cut into P chunks of residual_chunk columns
// (the last one shorter), and face rows (Nq columns) into chunks of the same length,
// residual_face_parts of them, so that every task runs about as many columns.
__host__ __device__ constexpr int residual_chunk(int D, int P) { return (dim_Nh(D) + P - 1) / P; }
__host__ __device__ constexpr int residual_face_parts(int D, int P) {
  return (dim_Nq(D) + residual_chunk(D, P) - 1) / residual_chunk(D, P);
}

// Reals per element of the block that holds the fetched u~ and metric factors [8][Nh]
// (dead after the node records) and then the P residual partials [P][3][Nh] and the lift's
// output [3][Np].
__host__ __device__ constexpr int raw_words(int D, int P) {
  return 8 * dim_Nh(D) > 3 * P * dim_Nh(D) + 3 * dim_Np(D) ? 8 * dim_Nh(D) : 3 * P * dim_Nh(D) + 3 * dim_Np(D);
}

// Reals of one element's node records in LDS: Nh records of kNodeRec, padded so that the
// stride is an odd multiple of 4 words.  The residual's lanes read the records of up to
// eight elements at one column at once; with such a stride their 16-byte reads fall on
// eight different groups of four banks (an even multiple, e.g. 336 at N=3, puts elements
// two apart on the same banks).
__host__ __device__ constexpr int rec_stride(int D) {
  return dim_Nh(D) * kNodeRec + (dim_Nh(D) % 2 == 0 ? 4 : 0);
}

// Words (of the bulk precision) of LDS one tile of E elements of kind D needs (the
// reference block is held separately, once per workgroup).  Modal kinds: node records
// [E][rec_stride] | raw block [E][raw_words] | neighbour values [E][Nfq][4] | state, RK
// register [3][E][Np] each | static block [E][stat_words].  DG-SBP: node records | two
// residual partials [2][3][E][Nh] | neighbour values | state, RK register [3][E][Nq] each |
// static block.
__host__ __device__ constexpr int tile_words(int D, int E, bool wadg = false, int P = 2) {
  return key_sbp(D) ? E * (rec_stride(D) + 6 * dim_Nh(D) + 4 * dim_Nfq(D) + 6 * dim_Nq(D) + stat_words(D))
                    : E * (rec_stride(D) + raw_words(D, P) + 4 * dim_Nfq(D) + 6 * dim_Np(D) +
                           stat_words(D, wadg));
}

// 32-bit words per thread of the static block that a stage stages through registers
// (issued after the tile's other copies have landed, stored to LDS after the residual),
// for float and for double tiles.
constexpr int kStatRegs = 8;
template <typename real> struct StatRegs { static constexpr int value = sizeof(real) == 4 ? kStatRegs : 4; };

// One instance as the kernels see it (device pointers into the bound workspace).
struct InstDesc {
  int32_t N, K, flux;   // N: the element kind D (degree | variant << kKeyShift)
  int32_t shape;        // tile shape of the residual phase, (R << 4) | P
  double g, Href, dt, pad1;
  void *uh;            // [3][K][Np] modal state (eta = h + b - Href, hu, hv)
  void *du;            // [3][K][Np] LSRK register
  void *ut[3];         // entropy-projected h~, u~, v~, H~ - Href at the hybrid nodes, tile-blocked:
                       // the tile of elements k0..k0+ne-1 holds [4][ne][Nh] from real k0*4*Nh
                       // (two stage buffers + rhs scratch)
  void *nbx[3];        // [K][Nfq][4] the same four values at each face node's neighbour, written
                       // by the neighbour's projection (one per ut buffer)
  const void *geo;     // rxJ, sxJ, ryJ, syJ at the hybrid nodes, tile-blocked like ut
  const void *wJq;     // [K][Nq] w_q J in double (diagnostics)
  const void *stat;    // static data in tile order: the tile of elements k0..k0+ne-1 holds, from
                       // real k0 * stat_words(N, wadg): the mass data [ne][mass_words] (Minv
                       // [Np][Np], or w/J at the volume nodes [Nq]) | w J [ne][Nq] | rest depth
                       // Href - b [ne][Nq] | Href - b [ne][Nh] | push targets [ne][Nfq] (int32
                       // k'*Nfq + f' of the nbx slot that face node f fills, packed in the first
                       // ne*Nfq 32-bit words; kPushWall set on wall nodes, whose slot is their
                       // own).  DG-SBP: 1/(w J) [ne][Nq] | Href - b [ne][Nq] | rxJ, sxJ, ryJ, syJ
                       // [4][ne][Nq] | push targets [ne][Nfq].  The rest depth is rewritten from
                       // bd (double) whenever Href changes, so a near-dry depth h = eta +
                       // (Href - b) keeps its relative accuracy in float.
  const void *ref;     // reference-operator block for this kind
  void *rhs_scratch;   // [3][K][Np] used by the diagnostics
  const double *bd;    // [K][Nh] bathymetry at the hybrid nodes in double (volume nodes first):
                       // the source of the rest depth Href - b written into the static block
  const double *Vqd;   // V_q [Nq][Np] in double (diagnostics; modal kinds)
};

// A contiguous range of elements of one instance, processed by one workgroup.
struct Tile {
  int32_t inst, k0, ne, pad;
};

enum StageMode : int32_t {
  kProject = 0,   // state -> entropy-projected values (ut[out])
  kRhs = 1,       // ut[in] -> rhs (no update)
  kStage = 2,     // ut[in] -> rhs -> LSRK update of uh, du -> project new uh to ut[out]
  kProbe = 3      // residency probe of a multi-stage grid (no tile work; see stage_kernel)
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
  int32_t v1;             // an instance is of a variant-1 kind (selects the stage-kernel build)
  int32_t shapes;         // an instance's tile shape is not the default (selects the build)
  int32_t kind;           // the element kind of every instance of a single-kind launch, which
                          // then runs the kernel built for that kind alone; 0 otherwise
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
  int32_t wadg;           // static-block layout of the modal kinds (weight-adjusted inverse)
  double *partials;       // [ntiles][6]
};

}  // namespace esdg
