// C-ABI runtime of the ESDG shallow-water library: planning (host FP64 setup), the
// device workspace layout, uploads, RK-stage launches, HIP-graph replay and diagnostics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "esdg_swe.h"
#include "device_types.hpp"
#include "host_setup.hpp"

namespace esdg {
hipError_t set_stage_lds_limit(bool fp64, int cm, bool wadg, bool sbp, bool v1, bool shapes, int kind,
                               size_t lds_bytes);
hipError_t launch_stage(bool fp64, bool sbp, const StageArgs &a, int max_blocks, size_t lds_bytes, int block,
                        hipStream_t stream);
hipError_t launch_stage_fused(bool fp64, const StageArgs &a, int max_blocks, size_t lds_bytes, int block,
                              bool cooperative, hipStream_t stream);
hipError_t stage_max_blocks(bool fp64, int cm, bool wadg, bool sbp, bool v1, bool shapes, int kind, size_t lds_bytes,
                            int block, int *out);
int stage_grid(int ntiles, int max_blocks);
hipError_t launch_diag(bool fp64, const DiagArgs &a, hipStream_t stream);
hipError_t launch_rest_depth(bool fp64, const DiagArgs &a, hipStream_t stream);
}  // namespace esdg

using namespace esdg;

namespace {

// Carpenter & Kennedy (1994) five-stage fourth-order 2N-storage coefficients.
const double kRkA[5] = {0.0, -567301805773.0 / 1357537059087.0, -2404267990393.0 / 2016746695238.0,
                        -3550918686646.0 / 2091501179385.0, -1275806237668.0 / 842570457699.0};
const double kRkB[5] = {1432997174477.0 / 9575080441904.0, 5161836677717.0 / 13612068292357.0,
                        1720146321549.0 / 2090206949498.0, 3134564353537.0 / 4481467310338.0,
                        2277821191437.0 / 14882151754819.0};

thread_local std::string g_init_error;

// Scratch of esdg_swe_rhs_noalloc (callers that cannot allocate device memory): a flag word,
// then the entropy-projected values and the face slots of the one instance it evaluates.
// Each device that loads the library holds its own copy until the process ends; host code
// uses only the device address returned by hipGetSymbolAddress (kept per device), never the
// array's name, which on the host is a stand-in and not a device address.
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr size_t kScratchHead = 256;       // flag word (int32), padded to the 256-byte alignment
}  // namespace

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch array (resolved once per device).
hipError_t scratch_address(void **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

// Bytes of scratch one no-allocation RHS evaluation of an instance needs.
size_t noalloc_bytes(int N, int K, size_t word) {
  const size_t ut = (size_t(4) * K * dim_Nh(N) * word + 255) & ~size_t(255);
  return kScratchHead + ut + size_t(4) * K * dim_Nfq(N) * word;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Default elements per workgroup of an element kind: as many as keep E*Nh <= 2 per thread
// and the tile's LDS <= 40 KiB per 256 threads (with the reference block, several
// workgroups stay resident per CU).
int default_epb(int D, size_t word, bool wadg, int P, int block) {
  int best = 1;
  for (int E = 1; E <= 64; E *= 2) {
    if (E * dim_Nh(D) > 2 * block) break;
    if (size_t(tile_words(D, E, wadg, P)) * word > size_t(40 * 1024) * block / kBlock) break;
    best = E;
  }
  return best;
}

// Default tile shape of the residual phase (kernels.hip: RowsPerThread, DefaultParts): two
// rows per thread in float at N = 1 and 3 of the default quadrature, else one; one column
// chunk at N = 5 of the default quadrature, else two.  (DG-SBP tiles use one row and two
// chunks always.)
int default_shape(int D, bool fp64) {
  const bool v0 = key_variant(D) == 0;
  const bool two = v0 && !fp64 && (key_N(D) == 1 || key_N(D) == 3);
  const bool one = v0 && key_N(D) == 5;
  return make_shape(two ? 2 : 1, one ? 1 : 2);
}

// A tile shape the stage kernel is compiled for (kernels.hip: shape_ok).
bool shape_valid(int D, bool fp64, int shape) {
  const int R = shape_rows(shape), P = shape_parts(shape);
  if (P < 1 || P > 4) return false;
  if (R == 1) return true;
  return R == 2 && !fp64 && dim_Nq(D) % 2 == 0 && dim_Nfq(D) % 2 == 0;
}

struct Offsets {
  size_t uh, du, ut[3], nbx[3], geo, wJq, bd, stat, rhs;
};

}  // namespace

struct esdg_swe {
  int n_inst = 0;
  esdg_swe_options opt{};
  bool fp64 = true;
  bool bf16x3 = false;
  int contraction = 0;             // 0 VALU, 1 matrix cores (bulk precision), 2 split-bf16
  bool wadg = false;               // weight-adjusted mass inverse instead of stored inverses
  bool sbp = false;                // DG-SBP scheme (every instance)
  bool v1 = false;                 // some instance is of a variant-1 kind (N+2 points)
  bool shapes = false;             // some kind's tile shape is not the default
  size_t word = 8;
  std::map<int, RefElem> refs;     // per element kind (degree | variant << 3)
  std::map<int, QuadRule> rules;   // the caller's volume rule of each kind (checked at init)
  std::vector<InstanceHost> host;
  std::vector<Offsets> off;
  std::map<int, size_t> ref_off, vqd_off;   // per kind: reference block, V_q in double
  size_t tiles_off = 0, desc_off = 0, flag_off = 0, partial_off = 0, ranges_off = 0;
  size_t progress_off = 0, nbr_off_off = 0, nbr_idx_off = 0;
  std::vector<int32_t> nbr_off, nbr_idx;   // tiles holding a face neighbour of each tile (CSR)
  long long stage_count = 0;       // global index of the next stage of a fused launch
  bool fused = false;
  bool balanced = false;           // mixed degrees: cost-balanced tile ranges uploaded
  size_t ws_bytes = 0;
  std::map<int, int> epb;          // elements per workgroup per element kind
  std::map<int, int> shape;        // tile shape of the residual phase per element kind
  size_t lds_bytes = 0;
  int block = kBlock;              // stage-kernel workgroup size (kBlockWide if every kind is wide)
  int kind = 0;                    // the one element kind of every instance (modal), else 0
  bool cooperative = true;         // multi-stage launches through hipLaunchCooperativeKernel (false
                                   // once the residency probe at bind saw the whole grid resident)
  int ref_max = 0;                 // LDS words reserved for the largest reference block
  int max_blocks = 0;              // resident workgroups of the stage kernel (set at bind)
  std::vector<Tile> tiles;
  std::vector<int> tile_begin, tile_count;
  std::vector<InstDesc> desc;
  // binding
  unsigned char *ws = nullptr;
  hipStream_t stream = nullptr;
  bool bound = false;
  std::vector<bool> state_set;
  int parity = 0;                  // which ut buffer holds the projection of the current state
  void *scratch_dev = nullptr;     // the bound device's scratch array (esdg_swe_rhs_noalloc)
  bool scratch_used = false;       // an esdg_swe_rhs_noalloc call may have set its flag word
  std::map<std::pair<int, int>, hipGraphExec_t> graphs;   // (steps, start parity) -> exec
  std::string err;

  ~esdg_swe() {
    // work still queued on the stream may be a replay of one of these graphs, or a
    // cooperative launch reading the workspace: let it finish before anything is released
    if (bound) (void)hipStreamSynchronize(stream);
    for (auto &kv : graphs) (void)hipGraphExecDestroy(kv.second);
  }
  template <typename T>
  T *dev(size_t o) const { return reinterpret_cast<T *>(ws + o); }
  esdg_status fail(esdg_status st, const std::string &m) {
    err = m;
    return st;
  }
  esdg_status hip_fail(hipError_t e, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(e);
    return ESDG_EDEVICE;
  }
};

namespace {

// Convert doubles to the bulk precision into a byte buffer.
std::vector<unsigned char> to_bulk(const std::vector<double> &v, bool fp64) {
  std::vector<unsigned char> out(v.size() * (fp64 ? 8 : 4));
  if (fp64) {
    std::memcpy(out.data(), v.data(), out.size());
  } else {
    float *f = reinterpret_cast<float *>(out.data());
    for (size_t i = 0; i < v.size(); ++i) f[i] = float(v[i]);
  }
  return out;
}

std::vector<double> ref_block(const RefElem &R) {
  std::vector<double> b;
  const bool sbp = key_sbp(R.key);
  b.reserve(ref_words(R.key));
  if (!sbp) b.insert(b.end(), R.Vh.a.begin(), R.Vh.a.end());
  for (int n = 0; n < R.Nh; ++n)
    for (int m = 0; m < R.Nq; ++m) {
      b.push_back(R.Sr(m, n));
      b.push_back(R.Ss(m, n));
    }
  for (int n = 0; n < R.Nq; ++n)
    for (int f = 0; f < R.Nfq; ++f) {
      b.push_back(-R.Sr(n, R.Nq + f));
      b.push_back(-R.Ss(n, R.Nq + f));
    }
  b.insert(b.end(), R.wf.begin(), R.wf.end());
  b.insert(b.end(), R.nr.begin(), R.nr.end());
  b.insert(b.end(), R.ns.begin(), R.ns.end());
  if (sbp) {                       // face <-> volume node maps, integer-valued
    for (int v : R.fvol) b.push_back(double(v));
    for (int v : R.vface) b.push_back(double(v));
  }
  return b;
}

esdg_status upload(esdg_swe *s, size_t off, const void *src, size_t bytes) {
  hipError_t e = hipMemcpyAsync(s->ws + off, src, bytes, hipMemcpyHostToDevice, s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "hipMemcpyAsync (upload)");
  return ESDG_OK;
}

esdg_status launch(esdg_swe *s, const StageArgs &a, int /*ntiles*/) {
  hipError_t e = launch_stage(s->fp64, s->sbp, a, s->max_blocks, s->lds_bytes, s->block, s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "stage kernel launch");
  return ESDG_OK;
}

StageArgs base_args(esdg_swe *s, int inst) {
  StageArgs a{};
  a.desc = s->dev<InstDesc>(s->desc_off);
  if (inst < 0) {
    a.tiles = s->dev<Tile>(s->tiles_off);
    a.ntiles = int(s->tiles.size());
    a.ranges = s->balanced ? s->dev<int32_t>(s->ranges_off) : nullptr;
  } else {
    a.tiles = s->dev<Tile>(s->tiles_off) + s->tile_begin[inst];
    a.ntiles = s->tile_count[inst];
  }
  a.flag = s->dev<int32_t>(s->flag_off);
  a.ref_words_max = s->ref_max;   // a multiple of 4: node records stay 16-byte aligned
  a.contraction = s->contraction;
  a.wadg = s->wadg ? 1 : 0;
  a.v1 = s->v1 ? 1 : 0;
  a.shapes = s->shapes ? 1 : 0;
  a.kind = s->kind;
  return a;
}

esdg_status check_flag(esdg_swe *s) {
  hipError_t e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "hipStreamSynchronize");
  int32_t flag = 0;
  e = hipMemcpy(&flag, s->dev<int32_t>(s->flag_off), sizeof flag, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return s->hip_fail(e, "hipMemcpy (flag)");
  if (s->scratch_used) {           // the no-allocation RHS reports into the scratch flag word
    int32_t f2 = 0;
    e = hipMemcpy(&f2, s->scratch_dev, sizeof f2, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return s->hip_fail(e, "hipMemcpy (scratch flag)");
    if (f2) {
      const int32_t zero = 0;
      e = hipMemcpy(s->scratch_dev, &zero, sizeof zero, hipMemcpyHostToDevice);
      if (e != hipSuccess) return s->hip_fail(e, "hipMemcpy (scratch flag reset)");
    }
    s->scratch_used = false;
    flag |= f2;
  }
  if (flag) {
    int32_t zero = 0;
    (void)hipMemcpy(s->dev<int32_t>(s->flag_off), &zero, sizeof zero, hipMemcpyHostToDevice);
    if (flag & 2) {
      // a fused launch gave up waiting: restart the stage counts from zero
      std::vector<int32_t> z(s->tiles.size(), 0);
      (void)hipMemcpy(s->dev<int32_t>(s->progress_off), z.data(), z.size() * sizeof(int32_t), hipMemcpyHostToDevice);
      s->stage_count = 0;
      return s->fail(ESDG_EDEVICE, "fused step: a tile's wait for its neighbours gave up; the state is undefined");
    }
    return s->fail(ESDG_ENONPHYS, "a kernel saw a non-finite value or a depth h~ <= 0");
  }
  return ESDG_OK;
}

// The state of instance inst from host coefficients of (h, hu, hv) (modal, or nodal for
// DG-SBP): reference level, eta = h + b - Href, RK register zero, rest depth, projection.
esdg_status set_modal(esdg_swe *s, int inst, const std::vector<double> &uh) {
  const InstanceHost &H = s->host[inst];
  const RefElem &R = s->refs.at(H.key);
  const bool sbp = key_sbp(H.key);
  const int Ns = dim_Np(H.key), Nq = R.Nq, Np = R.Np;
  const size_t n = size_t(3) * H.K * Ns;
  // reference level for the pressure term: mean of h + b over volume nodes
  double sum = 0.0, wsum = 0.0;
  for (int k = 0; k < H.K; ++k)
    for (int q = 0; q < Nq; ++q) {
      double hq = 0.0;
      if (sbp) hq = uh[size_t(k) * Ns + q];
      else
        for (int j = 0; j < Np; ++j) hq += R.Vh(q, j) * uh[size_t(k) * Ns + j];
      const double w = H.wJq[size_t(k) * Nq + q];
      sum += w * (hq + H.bq[size_t(k) * Nq + q]);
      wsum += w;
    }
  const double Href = sum / wsum;
  s->desc[inst].Href = Href;
  // internal depth: eta = h + b - Href (modal: the constant 1 is sqrt(2) phi_0)
  std::vector<double> w = uh;
  const double c0 = std::sqrt(2.0);
  for (int k = 0; k < H.K; ++k) {
    if (sbp) {
      for (int q = 0; q < Nq; ++q) w[size_t(k) * Ns + q] += H.bq[size_t(k) * Nq + q] - Href;
    } else {
      for (int j = 0; j < Np; ++j) w[size_t(k) * Ns + j] += H.bmodal[size_t(k) * Np + j];
      w[size_t(k) * Ns] -= Href * c0;
    }
  }
  auto bulk = to_bulk(w, s->fp64);
  esdg_status st = upload(s, s->off[inst].uh, bulk.data(), bulk.size());
  if (st) return st;
  hipError_t e = hipMemsetAsync(s->ws + s->off[inst].du, 0, n * s->word, s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "hipMemsetAsync (du)");
  st = upload(s, s->desc_off + inst * sizeof(InstDesc), &s->desc[inst], sizeof(InstDesc));
  if (st) return st;
  {                                // rest depth Href - b into the instance's static blocks
    DiagArgs da{};
    da.desc = s->dev<InstDesc>(s->desc_off);
    da.tiles = s->dev<Tile>(s->tiles_off) + s->tile_begin[inst];
    da.ntiles = s->tile_count[inst];
    da.wadg = s->wadg ? 1 : 0;
    e = launch_rest_depth(s->fp64, da, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "rest depth kernel launch");
  }
  StageArgs a = base_args(s, inst);
  a.mode = kProject;
  a.out_buf = s->parity;
  st = launch(s, a, a.ntiles);
  if (st) return st;
  s->state_set[inst] = true;
  return check_flag(s);
}

}  // namespace

extern "C" {

// Element kind and volume rule of one instance from its quadrature request (Section 2.1;
// Section 3.1 for DG-SBP).  Returns "" or an error message.
static std::string plan_quadrature(int N, const esdg_swe_quadrature *q, bool sbp, int *variant, QuadRule *rule,
                                   bool *custom) {
  const int vdeg = q && q->vol_degree ? q->vol_degree : (sbp ? 2 * N - 1 : 2 * N);
  const int fp = q && q->face_points ? q->face_points : N + 1;
  const int nq = q ? q->nq : 0;
  *custom = nq > 0;
  if (q && (q->vol_degree < 0 || q->face_points < 0 || q->nq < 0)) return "negative quadrature field";
  if (sbp) {
    if (N > 4) return "DG-SBP is compiled for N = 1..4";
    if (nq <= 0) return "DG-SBP needs the caller's volume rule (esdg_swe_quadrature.nq > 0)";
    if (fp != N + 1) return "DG-SBP uses N+1 Gauss-Legendre points per face";
    if (vdeg < 2 * N - 1) return "DG-SBP volume rule: vol_degree must be at least 2N-1";
    *variant = 2;
  } else {
    if (fp != N + 1 && fp != N + 2) return "face_points must be N+1 or N+2";
    if (vdeg < 2 * N) return "vol_degree must be at least 2N";
    int need = 0;                  // volume nodes
    if (nq > 0) need = nq;
    else {
      const int qd = (vdeg + 2) / 2;                    // ceil((vdeg + 1) / 2) points per direction
      if (qd > N + 2) return "vol_degree above 2N+3 (the Stroud rule is compiled for N+1 or N+2 points)";
      need = std::max(qd, N + 1) * std::max(qd, N + 1);
    }
    *variant = (need > (N + 1) * (N + 1) || fp == N + 2) ? 1 : 0;
    if (*variant == 1 && fp != N + 2) return "a volume rule of more than (N+1)^2 nodes needs face_points = N+2";
    if (need > (N + 2) * (N + 2)) return "a volume rule of more than (N+2)^2 nodes";
  }
  if (nq > 0) {
    if (!q->rq || !q->sq || !q->wq) return "null rule pointers";
    rule->r.assign(q->rq, q->rq + nq);
    rule->s.assign(q->sq, q->sq + nq);
    rule->w.assign(q->wq, q->wq + nq);
    std::string m = check_rule(*rule, vdeg);
    if (!m.empty()) return m;
  } else if (!sbp && *variant == 1) {
    // Stroud rule with N+2 points per direction (or N+1, padded) - built by build_ref
    const int qd = std::max((vdeg + 2) / 2, N + 1);
    if (qd == N + 1) {             // (N+1)^2 Stroud nodes in a variant-1 element: pad them
      RefElem tmp = build_ref(N, 0, nullptr, nullptr);
      rule->r = tmp.rq; rule->s = tmp.sq; rule->w = tmp.wq;
      *custom = true;
    }
  }
  return "";
}

esdg_status esdg_swe_init(int32_t n_inst, const esdg_swe_instance *inst, const esdg_swe_quadrature *quad,
                          const esdg_swe_options *opt, esdg_swe **out, size_t *workspace_bytes) {
  g_init_error.clear();
  if (!out || !workspace_bytes || !inst || !opt || n_inst < 1) {
    g_init_error = "esdg_swe_init: null argument or n_inst < 1";
    return ESDG_EINVAL;
  }
  *out = nullptr;
  if (opt->precision < ESDG_FP64 || opt->precision > ESDG_FP32_BF16X3 || opt->flux < 0 || opt->flux > 1 ||
      !(opt->g > 0.0) || opt->matrix_cores < 0 || opt->matrix_cores > 2 || opt->fused_steps < 0 ||
      opt->fused_steps > 2 || opt->mass_inverse < 0 || opt->mass_inverse > 1 || opt->scheme < 0 || opt->scheme > 1) {
    g_init_error = "esdg_swe_init: option out of range";
    return ESDG_EINVAL;
  }
  for (int N = 1; N <= kMaxN; ++N)
    if (opt->elems_per_block[N] < 0 || opt->elems_per_block[N] > 64) {
      g_init_error = "esdg_swe_init: elems_per_block out of range (0..64)";
      return ESDG_EINVAL;
    }
  std::unique_ptr<esdg_swe> s(new esdg_swe());
  s->n_inst = n_inst;
  s->opt = *opt;
  s->sbp = opt->scheme == ESDG_SCHEME_SBP;
  if (s->sbp && (opt->precision == ESDG_FP32_BF16X3 || opt->matrix_cores == 2 || opt->mass_inverse != 0)) {
    g_init_error = "esdg_swe_init: DG-SBP has no contractions and a diagonal mass matrix (precision FP64 or FP32, "
                   "matrix_cores 0/1, mass_inverse stored)";
    return ESDG_EINVAL;
  }
  if (s->sbp) s->opt.fused_steps = 0;
  s->fp64 = opt->precision == ESDG_FP64;
  s->bf16x3 = opt->precision == ESDG_FP32_BF16X3;
  s->contraction = s->sbp ? 0 : (s->bf16x3 ? 2 : (opt->matrix_cores == 2 ? 1 : 0));
  s->wadg = !s->sbp && opt->mass_inverse == ESDG_MASS_WEIGHT_ADJUSTED;
  s->word = s->fp64 ? 8 : 4;
  s->host.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const esdg_swe_instance &I = inst[i];
    if (I.N < 1 || I.N > kMaxN || I.K < 1 || !I.xg || !I.yg || !std::isfinite(I.Lx) || !std::isfinite(I.Ly)) {
      g_init_error = "esdg_swe_init: instance " + std::to_string(i) + ": bad N, K, pointers or periods";
      return ESDG_EINVAL;
    }
    int variant = 0;
    bool custom = false;
    QuadRule rule;
    std::string qm = plan_quadrature(I.N, quad ? &quad[i] : nullptr, s->sbp, &variant, &rule, &custom);
    if (!qm.empty()) {
      g_init_error = "esdg_swe_init: instance " + std::to_string(i) + ": " + qm;
      return ESDG_EINVAL;
    }
    const int key = make_key(I.N, variant);
    if (variant == 1) s->v1 = true;
    if (!s->refs.count(key)) {
      std::string m;
      s->refs[key] = build_ref(I.N, variant, custom ? &rule : nullptr, &m);
      if (m.empty()) m = check_ref(s->refs[key], 1e-12);
      if (!m.empty()) {
        g_init_error = "esdg_swe_init: instance " + std::to_string(i) + ": " + m;
        return ESDG_EINVAL;
      }
      if (custom) s->rules[key] = rule;
    } else {
      // instances of one kind share the reference block: their rules must be the same
      const bool had = s->rules.count(key) != 0;
      const bool same = had == custom && (!custom || (s->rules[key].r == rule.r && s->rules[key].s == rule.s &&
                                                      s->rules[key].w == rule.w));
      if (!same) {
        g_init_error = "esdg_swe_init: instance " + std::to_string(i) +
                       ": instances of one degree must use the same quadrature";
        return ESDG_EINVAL;
      }
    }
    std::string m = build_instance(s->refs[key], I.K, I.xg, I.yg, I.b, I.Lx, I.Ly, s->host[i], !s->wadg && !s->sbp);
    if (!m.empty()) {
      g_init_error = "instance " + std::to_string(i) + ": " + m;
      return ESDG_EMESH;
    }
    if (size_t(I.K) * dim_Nh(key) >= size_t(1) << 31) {
      g_init_error = "instance " + std::to_string(i) + ": K * Nh exceeds the 32-bit face index";
      return ESDG_EINVAL;
    }
  }
  // one modal kind for every instance: the stage kernel built for that kind alone
  if (s->refs.size() == 1 && !s->sbp) s->kind = s->refs.begin()->first;
  // workgroup size: kBlockWide when every kind is wide (its reference block is then shared
  // by twice the elements), else kBlock
  {
    bool all_wide = !s->refs.empty();
    for (auto &kv : s->refs) all_wide = all_wide && wide_kind(kv.first);
    s->block = all_wide ? kBlockWide : kBlock;
  }
  // elements per workgroup and LDS: the largest reference block + the largest tile
  size_t tile = 0;
  for (auto &kv : s->refs) {
    const int D = kv.first, N = key_N(D);
    int shape = opt->tile_shape[N] ? opt->tile_shape[N] : default_shape(D, s->fp64);
    if (s->sbp) shape = make_shape(1, 2);
    else if (!shape_valid(D, s->fp64, shape)) {
      g_init_error = "esdg_swe_init: tile_shape for N=" + std::to_string(N) +
                     " not compiled (rows 1, or 2 in float where they divide Nq and Nfq; parts 1..4)";
      return ESDG_EINVAL;
    }
    s->shape[D] = shape;
    if (!s->sbp && shape != default_shape(D, s->fp64)) s->shapes = true;
    const int P = shape_parts(shape);
    int E = opt->elems_per_block[N] ? opt->elems_per_block[N] : default_epb(D, s->word, s->wadg, P, s->block);
    s->epb[D] = E;
    s->ref_max = std::max(s->ref_max, ref_words(D));
    tile = std::max(tile, size_t(tile_words(D, E, s->wadg, P)));
  }
  if (s->shapes && (s->contraction != 0 || s->v1)) {
    g_init_error = "esdg_swe_init: tile shapes other than the default are compiled with vector-ALU contractions "
                   "and (N+1)-point quadrature only";
    return ESDG_EINVAL;
  }
  s->ref_max = (s->ref_max + 3) & ~3;
  size_t lds = (size_t(s->ref_max) + tile) * s->word;
  if (lds > 160 * 1024) {
    g_init_error = "esdg_swe_init: elems_per_block needs more than 160 KiB of LDS";
    return ESDG_EINVAL;
  }
  s->lds_bytes = lds;
  // tiles
  s->tile_begin.resize(n_inst);
  s->tile_count.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const int E = s->epb[s->host[i].key];
    s->tile_begin[i] = int(s->tiles.size());
    for (int k0 = 0; k0 < inst[i].K; k0 += E) s->tiles.push_back(Tile{i, k0, std::min(E, inst[i].K - k0), 0});
    s->tile_count[i] = int(s->tiles.size()) - s->tile_begin[i];
  }
  // tiles holding face neighbours of each tile (for fused multi-stage launches)
  s->nbr_off.assign(1, 0);
  for (int i = 0; i < n_inst; ++i) {
    const InstanceHost &H = s->host[i];
    const int Nh = dim_Nh(H.key), Nfq = dim_Nfq(H.key), E = s->epb[H.key];
    for (int t = s->tile_begin[i]; t < s->tile_begin[i] + s->tile_count[i]; ++t) {
      std::vector<int32_t> nb;
      for (int k = s->tiles[t].k0; k < s->tiles[t].k0 + s->tiles[t].ne; ++k)
        for (int f = 0; f < Nfq; ++f) {
          const int u = s->tile_begin[i] + H.mapP[size_t(k) * Nfq + f] / Nh / E;
          if (u != t) nb.push_back(u);
        }
      std::sort(nb.begin(), nb.end());
      nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
      s->nbr_idx.insert(s->nbr_idx.end(), nb.begin(), nb.end());
      s->nbr_off.push_back(int32_t(s->nbr_idx.size()));
    }
  }
  s->fused = s->opt.fused_steps != 0;   // mode 2 is resolved at bind, once the resident count is known
  // workspace layout
  size_t o = 0;
  auto take = [&](size_t bytes) {
    size_t r = o;
    o = align256(o + bytes);
    return r;
  };
  for (auto &kv : s->refs) {
    s->ref_off[kv.first] = take(size_t(ref_words(kv.first)) * s->word);
    s->vqd_off[kv.first] = take(size_t(kv.second.Nq) * kv.second.Np * sizeof(double));
  }
  s->off.resize(n_inst);
  for (int i = 0; i < n_inst; ++i) {
    const int D = s->host[i].key, K = inst[i].K;
    const size_t Np = dim_Np(D), Nq = dim_Nq(D), Nh = dim_Nh(D), Nfq = dim_Nfq(D), w = s->word;
    Offsets &f = s->off[i];
    f.uh = take(3 * K * Np * w);
    f.du = take(3 * K * Np * w);
    for (int b = 0; b < 3; ++b) f.ut[b] = s->sbp ? 0 : take(4 * K * Nh * w);
    for (int b = 0; b < 3; ++b) f.nbx[b] = take(4 * K * Nfq * w);
    f.geo = s->sbp ? 0 : take(4 * K * Nh * w);
    f.wJq = take(K * Nq * sizeof(double));
    f.bd = take(K * Nh * sizeof(double));
    f.stat = take(K * size_t(stat_words(D, s->wadg)) * w);
    f.rhs = take(3 * K * Np * w);
  }
  s->tiles_off = take(s->tiles.size() * sizeof(Tile));
  s->desc_off = take(n_inst * sizeof(InstDesc));
  s->flag_off = take(256);
  s->partial_off = take(s->tiles.size() * 6 * sizeof(double));
  s->ranges_off = take((s->tiles.size() + 16) * sizeof(int32_t));
  s->progress_off = take(s->tiles.size() * sizeof(int32_t));
  s->nbr_off_off = take(s->nbr_off.size() * sizeof(int32_t));
  s->nbr_idx_off = take(std::max<size_t>(s->nbr_idx.size(), 1) * sizeof(int32_t));
  s->ws_bytes = o;
  s->desc.resize(n_inst);
  s->state_set.assign(n_inst, false);
  *workspace_bytes = s->ws_bytes;
  *out = s.release();
  return ESDG_OK;
}

esdg_status esdg_swe_bind(esdg_swe *s, void *dev_workspace, size_t bytes, void *hip_stream) {
  if (!s || !dev_workspace) return s ? s->fail(ESDG_EINVAL, "bind: null workspace") : ESDG_EINVAL;
  if (bytes < s->ws_bytes) return s->fail(ESDG_ENOMEM, "bind: workspace smaller than esdg_swe_init asked for");
  if (reinterpret_cast<uintptr_t>(dev_workspace) % 256) return s->fail(ESDG_EINVAL, "bind: workspace not 256-byte aligned");
  s->ws = static_cast<unsigned char *>(dev_workspace);
  s->stream = static_cast<hipStream_t>(hip_stream);
  {
    hipError_t e = scratch_address(&s->scratch_dev);
    if (e != hipSuccess) return s->hip_fail(e, "hipGetSymbolAddress (scratch)");
  }
  if (s->lds_bytes > 64 * 1024) {
    hipError_t e = set_stage_lds_limit(s->fp64, s->contraction, s->wadg, s->sbp, s->v1, s->shapes, s->kind, s->lds_bytes);
    if (e != hipSuccess) return s->hip_fail(e, "hipFuncSetAttribute (LDS)");
  }
  {
    hipError_t e = stage_max_blocks(s->fp64, s->contraction, s->wadg, s->sbp, s->v1, s->shapes, s->kind, s->lds_bytes, s->block,
                                    &s->max_blocks);
    if (e != hipSuccess) return s->hip_fail(e, "hipOccupancyMaxActiveBlocksPerMultiprocessor");
    if (std::getenv("ESDG_SWE_VERBOSE")) {
      std::fprintf(stderr, "esdg_swe: %s, %d threads and LDS %zu B per workgroup, %d resident workgroups, %zu tiles;",
                   s->fp64 ? (s->contraction ? "fp64+mfma" : "fp64")
                           : (s->bf16x3 ? "fp32+bf16x3" : (s->contraction ? "fp32+mfma" : "fp32")), s->block, s->lds_bytes,
                   s->max_blocks, s->tiles.size());
      for (auto &kv : s->epb)
        std::fprintf(stderr, " N=%d%s: %d elements/tile", key_N(kv.first),
                     key_variant(kv.first) == 1 ? " (N+2 points)" : (key_sbp(kv.first) ? " (DG-SBP)" : ""), kv.second);
      std::fprintf(stderr, "\n");
    }
  }
  esdg_status st;
  // host staging buffers stay alive until the stream is synchronised below
  std::vector<std::vector<unsigned char>> keep;
  for (auto &kv : s->refs) {
    keep.push_back(to_bulk(ref_block(kv.second), s->fp64));
    if ((st = upload(s, s->ref_off[kv.first], keep.back().data(), keep.back().size()))) return st;
    // V_q in double for the diagnostics (the first Nq rows of V_h)
    const RefElem &R = kv.second;
    keep.push_back(std::vector<unsigned char>(size_t(R.Nq) * R.Np * sizeof(double)));
    std::memcpy(keep.back().data(), R.Vh.a.data(), keep.back().size());
    if ((st = upload(s, s->vqd_off[kv.first], keep.back().data(), keep.back().size()))) return st;
  }
  for (int i = 0; i < s->n_inst; ++i) {
    const InstanceHost &H = s->host[i];
    const Offsets &f = s->off[i];
    if (!s->sbp) {
      // metric factors in tile-blocked order: [4][ne][Nh] per tile, from k0 * 4 * Nh
      const size_t Nh = size_t(dim_Nh(H.key)), plane = size_t(H.K) * Nh;
      std::vector<double> g(H.geo.size());
      for (int t = s->tile_begin[i]; t < s->tile_begin[i] + s->tile_count[i]; ++t) {
        const size_t k0 = size_t(s->tiles[t].k0), ne = size_t(s->tiles[t].ne);
        for (size_t c = 0; c < 4; ++c)
          for (size_t j = 0; j < ne * Nh; ++j) g[k0 * 4 * Nh + c * ne * Nh + j] = H.geo[c * plane + k0 * Nh + j];
      }
      keep.push_back(to_bulk(g, s->fp64));
      if ((st = upload(s, f.geo, keep.back().data(), keep.back().size()))) return st;
    }
    // w J and the bathymetry at the hybrid nodes, in double (diagnostics, rest depth)
    if ((st = upload(s, f.wJq, H.wJq.data(), H.wJq.size() * sizeof(double)))) return st;
    if ((st = upload(s, f.bd, H.bh.data(), H.bh.size() * sizeof(double)))) return st;
    {
      // face node f of element k fills slot k' * Nfq + f' of the neighbour's face list
      const int D = H.key, Np = dim_Np(D), Nh = dim_Nh(D), Nq = dim_Nq(D), Nfq = dim_Nfq(D);
      std::vector<int32_t> push(H.mapP.size());
      for (size_t j = 0; j < push.size(); ++j) {
        const int32_t m = H.mapP[j], k2 = m / Nh;
        push[j] = k2 * Nfq + (m - k2 * Nh - Nq);
        if (H.wall[j]) push[j] = int32_t(uint32_t(push[j]) | kPushWall);   // own slot, mirrored
      }
      // inverse-permutation check: every slot is filled exactly once
      std::vector<char> hit(push.size(), 0);
      for (int32_t p0 : push) {
        const int32_t p = int32_t(uint32_t(p0) & ~kPushWall);
        if (p < 0 || size_t(p) >= push.size() || hit[p]) return s->fail(ESDG_EMESH, "face push map is not a permutation");
        hit[p] = 1;
      }
      // static blocks in tile order (the layout of the tile's LDS region from the mass data on);
      // the rest depth Href - b is written by the device at every set_state (here: -b)
      const size_t SW = size_t(stat_words(D, s->wadg)), word = s->word;
      std::vector<unsigned char> blk(size_t(H.K) * SW * word, 0);
      auto put = [&](size_t real_index, double v) {
        if (s->fp64) std::memcpy(&blk[real_index * 8], &v, 8);
        else { const float f32 = float(v); std::memcpy(&blk[real_index * 4], &f32, 4); }
      };
      for (int t = s->tile_begin[i]; t < s->tile_begin[i] + s->tile_count[i]; ++t) {
        const int k0 = s->tiles[t].k0, ne = s->tiles[t].ne;
        size_t o = size_t(k0) * SW;
        if (s->sbp) {              // 1/(w J) | -b | rxJ, sxJ, ryJ, syJ [4][ne][Nq] at the volume nodes
          const size_t plane = size_t(H.K) * Nh;
          for (int e = 0; e < ne; ++e)
            for (int q = 0; q < Nq; ++q) put(o++, 1.0 / H.wJq[size_t(k0 + e) * Nq + q]);
          for (int e = 0; e < ne; ++e)
            for (int q = 0; q < Nq; ++q) put(o++, -H.bq[size_t(k0 + e) * Nq + q]);
          for (int c = 0; c < 4; ++c)
            for (int e = 0; e < ne; ++e)
              for (int q = 0; q < Nq; ++q) put(o++, H.geo[c * plane + size_t(k0 + e) * Nh + q]);
        } else {
          if (s->wadg) {           // w/J at the volume nodes
            for (int e = 0; e < ne; ++e)
              for (int q = 0; q < Nq; ++q) put(o++, H.wOverJ[size_t(k0 + e) * Nq + q]);
          } else {                 // the stored inverse curved mass matrices
            for (int e = 0; e < ne; ++e)
              for (int j = 0; j < Np * Np; ++j) put(o++, H.Minv[size_t(k0 + e) * Np * Np + j]);
          }
          for (int e = 0; e < ne; ++e)
            for (int q = 0; q < Nq; ++q) put(o++, H.wJq[size_t(k0 + e) * Nq + q]);
          for (int e = 0; e < ne; ++e)
            for (int q = 0; q < Nq; ++q) put(o++, -H.bq[size_t(k0 + e) * Nq + q]);
          for (int e = 0; e < ne; ++e)
            for (int n = 0; n < Nh; ++n) put(o++, -H.bh[size_t(k0 + e) * Nh + n]);
        }
        std::memcpy(&blk[o * word], &push[size_t(k0) * Nfq], size_t(ne) * Nfq * 4);
      }
      keep.push_back(std::move(blk));
      if ((st = upload(s, f.stat, keep.back().data(), keep.back().size()))) return st;
    }
    InstDesc &d = s->desc[i];
    d.N = H.key;
    d.shape = s->shape[H.key];
    d.K = H.K;
    d.flux = s->opt.flux;
    d.g = s->opt.g;
    d.Href = 0.0;
    d.dt = 0.0;
    d.uh = s->ws + f.uh;
    d.du = s->ws + f.du;
    for (int b = 0; b < 3; ++b) d.ut[b] = s->sbp ? nullptr : s->ws + f.ut[b];
    for (int b = 0; b < 3; ++b) d.nbx[b] = s->ws + f.nbx[b];
    d.geo = s->sbp ? nullptr : s->ws + f.geo;
    d.wJq = s->ws + f.wJq;
    d.stat = s->ws + f.stat;
    d.ref = s->ws + s->ref_off[H.key];
    d.rhs_scratch = s->ws + f.rhs;
    d.bd = reinterpret_cast<const double *>(s->ws + f.bd);
    d.Vqd = reinterpret_cast<const double *>(s->ws + s->vqd_off[H.key]);
  }
  if ((st = upload(s, s->desc_off, s->desc.data(), s->desc.size() * sizeof(InstDesc)))) return st;
  if ((st = upload(s, s->tiles_off, s->tiles.data(), s->tiles.size() * sizeof(Tile)))) return st;
  if ((st = upload(s, s->nbr_off_off, s->nbr_off.data(), s->nbr_off.size() * sizeof(int32_t)))) return st;
  if (!s->nbr_idx.empty() && (st = upload(s, s->nbr_idx_off, s->nbr_idx.data(), s->nbr_idx.size() * sizeof(int32_t))))
    return st;
  keep.push_back(std::vector<unsigned char>(s->tiles.size() * sizeof(int32_t), 0));
  if ((st = upload(s, s->progress_off, keep.back().data(), keep.back().size()))) return st;
  s->stage_count = 0;
  if (s->opt.fused_steps == 2)
    s->fused = stage_grid(int(s->tiles.size()), s->max_blocks) >= int(s->tiles.size());
  if (s->fused) {
    int dev = 0, coop = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev);
    if (e != hipSuccess) return s->hip_fail(e, "hipDeviceGetAttribute (cooperative launch)");
    if (!coop && s->opt.fused_steps == 2) s->fused = false;   // automatic: fall back to per-stage launches
    else if (!coop) return s->fail(ESDG_EDEVICE, "fused_steps: the device does not support cooperative launches");
  }
  // mixed degrees: split the tile list into contiguous chunks of equal estimated cost
  std::vector<int32_t> ranges;
  if (s->refs.size() > 1) {
    const int G = stage_grid(int(s->tiles.size()), s->max_blocks);
    std::vector<long long> cum(s->tiles.size() + 1, 0);
    for (size_t t = 0; t < s->tiles.size(); ++t)
      cum[t + 1] = cum[t] + elem_cost(s->host[s->tiles[t].inst].key) * s->tiles[t].ne;
    ranges.resize(G + 1);
    size_t t = 0;
    for (int c = 0; c <= G; ++c) {
      const long long target = (long long)((__int128)cum.back() * c / G);
      while (t < s->tiles.size() && cum[t] < target) ++t;
      ranges[c] = int32_t(t);
    }
    ranges[G] = int32_t(s->tiles.size());
    if ((st = upload(s, s->ranges_off, ranges.data(), ranges.size() * sizeof(int32_t)))) return st;
    s->balanced = true;
  }
  hipError_t e = hipMemsetAsync(s->ws + s->flag_off, 0, 256, s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "hipMemsetAsync (flag)");
  e = hipStreamSynchronize(s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "hipStreamSynchronize (bind)");
  // Multi-stage launches need every workgroup of their grid resident at once.  The grid is
  // what the occupancy query (capped by LDS granules) says fits, so an ordinary launch of it
  // is normally resident, and it is cheaper than a cooperative one (about 5 % per stage at
  // config 2).  A probe launch with the same grid, workgroup size and LDS checks that here;
  // if any workgroup waited in vain the multi-stage launches stay cooperative.  (Their
  // neighbour waits are bounded either way: a grid that is not resident makes step fail.)
  s->cooperative = true;
  if (s->fused) {
    StageArgs a = base_args(s, -1);
    a.mode = kProbe;
    a.spin_limit = 1 << 17;
    e = launch_stage_fused(s->fp64, a, s->max_blocks, s->lds_bytes, s->block, false, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "residency probe");
    int32_t word[2] = {0, 0};
    e = hipMemcpy(&word[0], s->dev<int32_t>(s->flag_off), sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e == hipSuccess)
      e = hipMemcpy(&word[1], s->dev<int32_t>(s->flag_off) + kProbeWord, sizeof(int32_t), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return s->hip_fail(e, "hipMemcpy (residency probe)");
    s->cooperative = (word[0] & 4) != 0 || word[1] != stage_grid(int(s->tiles.size()), s->max_blocks);
    e = hipMemset(s->ws + s->flag_off, 0, 256);
    if (e != hipSuccess) return s->hip_fail(e, "hipMemset (flag)");
    if (std::getenv("ESDG_SWE_VERBOSE"))
      std::fprintf(stderr, "esdg_swe: multi-stage launches %s\n", s->cooperative ? "cooperative" : "ordinary");
  }
  s->bound = true;
  return ESDG_OK;
}

esdg_status esdg_swe_set_state(esdg_swe *s, int32_t inst, const double *u_nodes) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound) return s->fail(ESDG_ESTATE, "set_state before bind");
  if (inst < 0 || inst >= s->n_inst || !u_nodes) return s->fail(ESDG_EINVAL, "set_state: bad instance or null");
  const InstanceHost &H = s->host[inst];
  const RefElem &R = s->refs.at(H.key);
  const size_t plane = size_t(H.K) * R.Np;
  std::vector<double> uh(3 * plane);
  for (int c = 0; c < 3; ++c) nodes_to_modes(R, H.K, u_nodes + c * plane, uh.data() + c * plane);
  if (!key_sbp(H.key)) return set_modal(s, inst, uh);
  // DG-SBP: the interpolant's values at the volume nodes
  const size_t nplane = size_t(H.K) * R.Nq;
  std::vector<double> un(3 * nplane, 0.0);
  for (int c = 0; c < 3; ++c)
    for (int k = 0; k < H.K; ++k)
      for (int q = 0; q < R.Nq; ++q) {
        double v = 0.0;
        for (int j = 0; j < R.Np; ++j) v += R.Vh(q, j) * uh[c * plane + size_t(k) * R.Np + j];
        un[c * nplane + size_t(k) * R.Nq + q] = v;
      }
  return set_modal(s, inst, un);
}

esdg_status esdg_swe_set_state_modal(esdg_swe *s, int32_t inst, const double *uh) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound) return s->fail(ESDG_ESTATE, "set_state_modal before bind");
  if (inst < 0 || inst >= s->n_inst || !uh) return s->fail(ESDG_EINVAL, "set_state_modal: bad instance or null");
  const InstanceHost &H = s->host[inst];
  std::vector<double> v(uh, uh + size_t(3) * H.K * dim_Np(H.key));
  return set_modal(s, inst, v);
}

esdg_status esdg_swe_get_state(esdg_swe *s, int32_t inst, double *uh) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound || inst < 0 || inst >= s->n_inst || !uh) return s->fail(ESDG_EINVAL, "get_state: bad arguments");
  esdg_status st = check_flag(s);
  const InstanceHost &H = s->host[inst];
  const size_t n = size_t(3) * H.K * dim_Np(H.key);
  std::vector<unsigned char> buf(n * s->word);
  hipError_t e = hipMemcpy(buf.data(), s->ws + s->off[inst].uh, buf.size(), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return s->hip_fail(e, "hipMemcpy (get_state)");
  if (s->fp64)
    std::memcpy(uh, buf.data(), buf.size());
  else
    for (size_t i = 0; i < n; ++i) uh[i] = reinterpret_cast<const float *>(buf.data())[i];
  // eta -> h
  const int Np = dim_Np(H.key), Nq = dim_Nq(H.key);
  const double Href = s->desc[inst].Href, c0 = std::sqrt(2.0);
  for (int k = 0; k < H.K; ++k) {
    if (key_sbp(H.key)) {
      for (int q = 0; q < Nq; ++q) uh[size_t(k) * Np + q] -= H.bq[size_t(k) * Nq + q] - Href;
    } else {
      for (int j = 0; j < Np; ++j) uh[size_t(k) * Np + j] -= H.bmodal[size_t(k) * Np + j];
      uh[size_t(k) * Np] += Href * c0;
    }
  }
  return st;
}

esdg_status esdg_swe_state_device(esdg_swe *s, int32_t inst, void **uh_dev) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound || inst < 0 || inst >= s->n_inst || !uh_dev) return s->fail(ESDG_EINVAL, "state_device: bad arguments");
  *uh_dev = s->ws + s->off[inst].uh;
  return ESDG_OK;
}

esdg_status esdg_swe_rhs(esdg_swe *s, int32_t inst, const void *state_dev, void *rhs_dev) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound) return s->fail(ESDG_ESTATE, "rhs before bind");
  if (inst < 0 || inst >= s->n_inst || !state_dev || !rhs_dev) return s->fail(ESDG_EINVAL, "rhs: bad arguments");
  if (!s->state_set[inst]) return s->fail(ESDG_ESTATE, "rhs: set_state first (defines the pressure reference level)");
  const size_t bytes = size_t(3) * s->host[inst].K * dim_Np(s->host[inst].key) * s->word;
  const char *a0 = static_cast<const char *>(state_dev), *b0 = static_cast<const char *>(rhs_dev);
  if (a0 < b0 + bytes && b0 < a0 + bytes) return s->fail(ESDG_EINVAL, "rhs: state and rhs overlap");
  StageArgs a = base_args(s, inst);
  a.mode = kProject;
  a.ext_state = state_dev;
  a.out_buf = 2;
  esdg_status st = launch(s, a, a.ntiles);
  if (st) return st;
  a.mode = kRhs;
  a.in_buf = 2;
  a.ext_state = s->sbp ? state_dev : nullptr;   // DG-SBP forms its node records from the state
  a.ext_rhs = rhs_dev;
  return launch(s, a, a.ntiles);
}

esdg_status esdg_swe_rhs_noalloc(esdg_swe *s, int32_t inst, const void *state_dev, void *rhs_dev) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound) return s->fail(ESDG_ESTATE, "rhs_noalloc before bind");
  if (inst < 0 || inst >= s->n_inst || !state_dev || !rhs_dev) return s->fail(ESDG_EINVAL, "rhs_noalloc: bad arguments");
  if (!s->state_set[inst]) return s->fail(ESDG_ESTATE, "rhs_noalloc: set_state first (defines the pressure reference level)");
  const InstanceHost &H = s->host[inst];
  const size_t bytes = size_t(3) * H.K * dim_Np(H.key) * s->word;
  const char *a0 = static_cast<const char *>(state_dev), *b0 = static_cast<const char *>(rhs_dev);
  if (a0 < b0 + bytes && b0 < a0 + bytes) return s->fail(ESDG_EINVAL, "rhs_noalloc: state and rhs overlap");
  const size_t need = noalloc_bytes(H.key, H.K, s->word);
  if (need > kScratchBytes)
    return s->fail(ESDG_EINVAL, "rhs_noalloc: the instance needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                                    " the library holds per device (use esdg_swe_rhs)");
  unsigned char *base = static_cast<unsigned char *>(s->scratch_dev);
  StageArgs a = base_args(s, inst);
  a.flag = reinterpret_cast<int32_t *>(base);
  a.ext_ut = base + kScratchHead;
  a.ext_nbx = base + kScratchHead + ((size_t(4) * H.K * dim_Nh(H.key) * s->word + 255) & ~size_t(255));
  a.mode = kProject;
  a.ext_state = state_dev;
  s->scratch_used = true;
  esdg_status st = launch(s, a, a.ntiles);
  if (st) return st;
  a.mode = kRhs;
  a.ext_state = s->sbp ? state_dev : nullptr;
  a.ext_rhs = rhs_dev;
  return launch(s, a, a.ntiles);
}

static esdg_status run_steps_direct(esdg_swe *s, int nsteps) {
  for (int n = 0; n < nsteps; ++n)
    for (int st = 0; st < 5; ++st) {
      StageArgs a = base_args(s, -1);
      a.mode = kStage;
      a.in_buf = s->parity;
      a.out_buf = 1 - s->parity;
      a.rk_a = kRkA[st];
      a.rk_b = kRkB[st];
      esdg_status r = launch(s, a, a.ntiles);
      if (r) return r;
      s->parity = 1 - s->parity;
    }
  return ESDG_OK;
}

// All 5 * nsteps stages in one cooperative launch (see stage_kernel).  Stage counts are
// global and monotone; launches of at most 2^20 steps keep them well inside int32.
static esdg_status run_steps_fused(esdg_swe *s, int nsteps) {
  for (int done = 0; done < nsteps;) {
    const int n = std::min(nsteps - done, 1 << 20);
    if (s->stage_count + 5LL * n >= (1LL << 31) - 1) {
      std::vector<int32_t> z(s->tiles.size(), 0);
      hipError_t e = hipMemcpyAsync(s->dev<int32_t>(s->progress_off), z.data(), z.size() * sizeof(int32_t),
                                    hipMemcpyHostToDevice, s->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
      if (e != hipSuccess) return s->hip_fail(e, "reset of the stage counts");
      s->stage_count = 0;
    }
    StageArgs a = base_args(s, -1);
    a.mode = kStage;
    a.in_buf = s->parity;
    a.out_buf = 1 - s->parity;
    a.progress = s->dev<int32_t>(s->progress_off);
    a.nbr_off = s->dev<int32_t>(s->nbr_off_off);
    a.nbr_idx = s->dev<int32_t>(s->nbr_idx_off);
    a.stage0 = int32_t(s->stage_count);
    a.nstages = 5 * n;
    a.resident = stage_grid(a.ntiles, s->max_blocks) >= a.ntiles ? 1 : 0;   // one tile per workgroup
    a.spin_limit = 1 << 17;     // polls (each a device-coherent load): tens of ms, above any one stage
    for (int st = 0; st < 5; ++st) {
      a.rk_a5[st] = kRkA[st];
      a.rk_b5[st] = kRkB[st];
    }
    hipError_t e = launch_stage_fused(s->fp64, a, s->max_blocks, s->lds_bytes, s->block, s->cooperative, s->stream);
    if (e != hipSuccess) return s->hip_fail(e, "hipLaunchCooperativeKernel (fused steps)");
    s->stage_count += 5LL * n;
    if (n & 1) s->parity = 1 - s->parity;
    done += n;
  }
  return ESDG_OK;
}

esdg_status esdg_swe_step(esdg_swe *s, const double *dt, int32_t nsteps) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound) return s->fail(ESDG_ESTATE, "step before bind");
  if (!dt || nsteps < 0) return s->fail(ESDG_EINVAL, "step: null dt or negative nsteps");
  for (int i = 0; i < s->n_inst; ++i) {
    if (!s->state_set[i]) return s->fail(ESDG_ESTATE, "step: instance " + std::to_string(i) + " has no state");
    if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return s->fail(ESDG_EINVAL, "step: dt must be positive and finite");
  }
  bool changed = false;
  for (int i = 0; i < s->n_inst; ++i)
    if (s->desc[i].dt != dt[i]) {
      s->desc[i].dt = dt[i];
      changed = true;
    }
  if (changed) {
    esdg_status st = upload(s, s->desc_off, s->desc.data(), s->desc.size() * sizeof(InstDesc));
    if (st) return st;
  }
  if (nsteps == 0) return ESDG_OK;
  if (s->fused) return run_steps_fused(s, nsteps);
  if (!s->opt.use_graph || s->stream == nullptr) return run_steps_direct(s, nsteps);
  // graphs of an even number of steps keep the stage-buffer parity; replay them
  const int chunk = std::min(nsteps - nsteps % 2, 20);
  int done = 0;
  if (chunk >= 2) {
    auto key = std::make_pair(chunk, s->parity);
    hipGraphExec_t exec = nullptr;
    auto it = s->graphs.find(key);
    if (it == s->graphs.end()) {
      hipError_t e = hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return s->hip_fail(e, "hipStreamBeginCapture");
      const int p0 = s->parity;
      esdg_status st = run_steps_direct(s, chunk);
      hipGraph_t graph = nullptr;
      e = hipStreamEndCapture(s->stream, &graph);
      s->parity = p0;
      if (st) return st;
      if (e != hipSuccess) return s->hip_fail(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) return s->hip_fail(e, "hipGraphInstantiate");
      s->graphs[key] = exec;
    } else {
      exec = it->second;
    }
    while (nsteps - done >= chunk) {
      hipError_t e = hipGraphLaunch(exec, s->stream);
      if (e != hipSuccess) return s->hip_fail(e, "hipGraphLaunch");
      done += chunk;
    }
  }
  return run_steps_direct(s, nsteps - done);
}

esdg_status esdg_swe_diagnostics(esdg_swe *s, double *out) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound || !out) return s->fail(ESDG_EINVAL, "diagnostics: bad arguments");
  for (int i = 0; i < s->n_inst; ++i) {
    if (!s->state_set[i]) return s->fail(ESDG_ESTATE, "diagnostics: instance without state");
    esdg_status st = esdg_swe_rhs(s, i, s->ws + s->off[i].uh, s->ws + s->off[i].rhs);
    if (st) return st;
  }
  DiagArgs a{};
  a.desc = s->dev<InstDesc>(s->desc_off);
  a.tiles = s->dev<Tile>(s->tiles_off);
  a.ntiles = int(s->tiles.size());
  a.partials = s->dev<double>(s->partial_off);
  a.wadg = s->wadg ? 1 : 0;
  hipError_t e = launch_diag(s->fp64, a, s->stream);
  if (e != hipSuccess) return s->hip_fail(e, "diag kernel launch");
  esdg_status st = check_flag(s);
  std::vector<double> part(s->tiles.size() * 6);
  e = hipMemcpy(part.data(), s->dev<double>(s->partial_off), part.size() * 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return s->hip_fail(e, "hipMemcpy (diagnostics)");
  for (int i = 0; i < s->n_inst; ++i) {
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int t = s->tile_begin[i]; t < s->tile_begin[i] + s->tile_count[i]; ++t)
      for (int c = 0; c < 6; ++c) acc[c] += part[size_t(t) * 6 + c];
    for (int c = 0; c < 6; ++c) out[i * 6 + c] = acc[c];
  }
  return st;
}

esdg_status esdg_swe_sync(esdg_swe *s) {
  if (!s) return ESDG_EINVAL;
  if (!s->bound) return s->fail(ESDG_ESTATE, "sync before bind");
  return check_flag(s);
}

esdg_status esdg_swe_query(const esdg_swe *s, int32_t inst, int32_t *out6) {
  if (!s || !out6 || inst < 0 || inst >= s->n_inst) return ESDG_EINVAL;
  const int D = s->host[inst].key;
  out6[0] = key_N(D);
  out6[1] = s->host[inst].K;
  out6[2] = dim_Np(D);
  out6[3] = dim_Nq(D);             // volume nodes as compiled (a caller's rule zero-padded)
  out6[4] = dim_Nfq(D);
  out6[5] = dim_Nh(D);
  return ESDG_OK;
}

esdg_status esdg_swe_launch_info(const esdg_swe *s, int32_t *out4) {
  if (!s || !out4) return ESDG_EINVAL;
  if (!s->bound) return ESDG_ESTATE;
  const int ntiles = int(s->tiles.size());
  out4[0] = ntiles;
  out4[1] = s->max_blocks;
  out4[2] = int32_t(s->lds_bytes);
  out4[3] = !s->fused ? 0 : (stage_grid(ntiles, s->max_blocks) >= ntiles ? 2 : 1);
  return ESDG_OK;
}

esdg_status esdg_swe_reference_level(const esdg_swe *s, int32_t inst, double *Href) {
  if (!s || !Href || inst < 0 || inst >= s->n_inst) return ESDG_EINVAL;
  if (!s->state_set[inst]) return ESDG_ESTATE;
  *Href = s->desc[inst].Href;
  return ESDG_OK;
}

const char *esdg_swe_last_error(const esdg_swe *s) { return s ? s->err.c_str() : g_init_error.c_str(); }

void esdg_swe_destroy(esdg_swe *s) { delete s; }

}  // extern "C"
