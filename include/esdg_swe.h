/*
 * esdg_swe.h -- C ABI of the MI355X (gfx950) library that evaluates the modal
 * entropy-stable DG (ESDG) right-hand side of the 2D shallow water equations on
 * curved triangles and advances it with the five-stage low-storage RK4.
 *
 * Method: Wu, Kubatko & Chan, "High-order entropy stable discontinuous Galerkin
 * methods for the shallow water equations: curved triangular meshes and GPU
 * acceleration", arXiv 2005.02516.
 *
 *   rhs = -(M_h^k)^{-1} V_h^T r_h, where r_h is the hybridized-node residual of the
 *   semi-discrete form eq. (dgform) (Section 2.8): entropy projection (Section 2.6),
 *   flux differencing with the hybridized SBP operators and the entropy-conservative
 *   SWE flux on curved elements (Sections 2.3, 2.7, 2.8), bathymetry source, interface
 *   flux with optional local Lax-Friedrichs penalty (Section 2.8), and the
 *   per-element inverse curved mass matrix.  Time stepping: the 2N-storage
 *   Carpenter-Kennedy RK4(5) named in Section 4.
 *
 * Conventions shared with the caller (they fix coefficient-level results):
 *   - Reference triangle: counter-clockwise vertices v1=(-1,-1), v2=(1,-1), v3=(-1,1).
 *   - Modal basis: orthonormal Dubiner basis
 *       phi_ij(r,s) = sqrt(2) P~_i(a) P~_j^{(2i+1,0)}(b) (1-b)^i,
 *       a = 2(1+r)/(1-s) - 1, b = s, P~ orthonormal Jacobi polynomials,
 *     modes ordered "for i in 0..N: for j in 0..N-i".
 *   - Quadrature (Section 2.1 fixes only minimum degrees): by default the (N+1)^2-point
 *     Stroud collapsed rule (Gauss-Legendre x Gauss-Jacobi(1,0), exact to degree 2N+1) and
 *     N+1 Gauss-Legendre points per face; esdg_swe_quadrature selects another (below).
 *   - Geometry / sampling nodes: order-N equispaced nodes listed
 *       "for j in 0..N: for i in 0..N-j: (r,s) = (-1 + 2i/N, -1 + 2j/N)"
 *     (node 0 = v1, node N = v2, last node = v3).  Each element is the
 *     isoparametric degree-N map through its nodes.
 *   - Np = (N+1)(N+2)/2 (the number of modes), except for the DG-SBP scheme, whose state is
 *     nodal: Np = Nq there.  State layout everywhere: [3][K][Np], element-major planes, modes
 *     (or nodes) fastest.  Host-side states (set_state*, get_state) hold (h, hu, hv).  Device-side
 *     states (esdg_swe_state_device, esdg_swe_rhs) hold (eta, hu, hv) with the depth
 *     carried as the free-surface anomaly eta = h + b - Href, Href the instance's
 *     reference level (esdg_swe_reference_level): the modal coefficients of eta are those
 *     of h plus those of b minus Href*sqrt(2) on mode 0 (the constant 1 is sqrt(2) phi_00);
 *     for DG-SBP the nodal values of h plus those of b minus Href.  The time derivative of
 *     eta equals that of h.
 *
 * Ownership: the caller owns every host array passed in and may free it once the call
 * returns.  The caller owns the device workspace and the HIP stream given to
 * esdg_swe_bind and must keep both alive until esdg_swe_destroy.  The library never
 * allocates device memory: all its device arrays live in that workspace.
 *
 * Errors: every call returns an esdg_status; no C++ exception crosses this ABI.
 * esdg_swe_last_error returns a message for the last failing call on a handle (or, with
 * a NULL handle, for the last failing esdg_swe_init on this thread).
 *
 * Threading: a handle is not thread-safe; calls on one handle must be serialised.
 */
#ifndef ESDG_SWE_H
#define ESDG_SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct esdg_swe esdg_swe;

typedef enum {
  ESDG_OK = 0,
  ESDG_EINVAL = -1,     /* bad argument (null pointer, size, option out of range)         */
  ESDG_EMESH = -2,      /* mesh rejected: J <= 0, unmatched periodic face node, ...        */
  ESDG_ENOMEM = -3,     /* workspace smaller than esdg_swe_init asked for                  */
  ESDG_EDEVICE = -4,    /* a HIP runtime call failed (message names it)                    */
  ESDG_ENONPHYS = -5,   /* a kernel saw a non-finite value or a depth h~ <= 0              */
  ESDG_ESTATE = -6      /* call out of order (e.g. step before bind or before set_state)   */
} esdg_status;

/* arithmetic of the bulk path */
enum {
  ESDG_FP64 = 0,        /* everything in double precision                                  */
  ESDG_FP32 = 1,        /* state, operators, fluxes in float; the entropy <-> conservative
                           variable maps and the diagnostics in double                     */
  ESDG_FP32_BF16X3 = 2  /* as ESDG_FP32, with the projection and lift contractions done as
                           three bf16 products (hi*hi + hi*lo + lo*hi) accumulated in float */
};

/* interface flux (Section 2.8) */
enum {
  ESDG_FLUX_EC = 0,     /* entropy-conservative flux, no dissipation                        */
  ESDG_FLUX_LF = 1      /* plus local Lax-Friedrichs penalty on entropy-projected variables */
};

/* how the inverse curved mass matrices (M_h^k)^{-1} = (V_q^T W diag(J) V_q)^{-1} of Section
 * 2.7 are applied, in the entropy projection (Section 2.6) and in the lift (Section 2.8) */
enum {
  ESDG_MASS_STORED = 0,           /* precomputed per element and stored, Np x Np reals each   */
  ESDG_MASS_WEIGHT_ADJUSTED = 1   /* weight-adjusted inverse M^{-1} M_{1/J} M^{-1}, M_{1/J} =
                                     V_q^T W diag(1/J) V_q (the alternative the paper names
                                     after eq. (dgform), Section 2.8): only w/J at the Nq volume
                                     nodes is stored per element.  Exact where J is constant on
                                     the element, otherwise an approximation that agrees with
                                     the stored inverse to first order in the variation of J.
                                     Used in both places, the scheme keeps its entropy
                                     conservation (EC flux) and dissipation (LF).  The
                                     projected entropy variables are those of S - g Href h
                                     (Href: esdg_swe_reference_level), so a lake at rest at
                                     that level stays exactly at rest.  The mass reported by
                                     esdg_swe_diagnostics (the J-weighted integral of h) is then
                                     conserved only to the accuracy of the weight adjustment. */
};

/* scheme (esdg_swe_options.scheme) */
enum {
  ESDG_SCHEME_MODAL = 0,  /* modal ESDG with hybridized SBP operators (Section 2)              */
  ESDG_SCHEME_SBP = 1     /* DG-SBP with traditional SBP operators built from the hybridized
                             ones (Section 3.2): nodal state at the volume nodes of a rule whose
                             boundary nodes are the face nodes, diagonal mass matrix W J, no
                             entropy projection; per-stage launches only                       */
};

/* Quadrature of one instance (Section 2.1: volume rule exact to degree 2N, face rule to
 * degree 2N+1; Section 3.1 for DG-SBP: positive weights, volume rule exact to degree 2N-1
 * with the face nodes among its nodes).  Caller-owned, copied during init. */
typedef struct {
  int32_t vol_degree;     /* 0 = 2N (2N-1 for DG-SBP).  Stroud rule: the collapsed rule with
                             q = ceil((vol_degree + 1) / 2) points per direction, q = N+1 or
                             N+2 (vol_degree <= 2N+3).  Caller's rule: the degree it must be
                             exact to (>= 2N; >= 2N-1 for DG-SBP), checked at init          */
  int32_t face_points;    /* Gauss-Legendre points per face: 0 = N+1; N+1 or N+2 (DG-SBP: N+1) */
  int32_t nq;             /* 0 = Stroud rule; else the caller's volume rule of nq nodes:      */
  const double *rq, *sq;  /*   nodes on the reference triangle (closed)                       */
  const double *wq;       /*   positive weights (they sum to 2, the reference area)          */
} esdg_swe_quadrature;

/* The kernels are compiled for volume rules of (N+1)^2 nodes with N+1 face points, and of
 * (N+2)^2 nodes with N+2 face points; a rule with fewer nodes is padded with zero-weight
 * nodes (which leave every weighted operator unchanged), so a caller's rule may have up to
 * (N+2)^2 nodes, and more than (N+1)^2 only with face_points = N+2.  DG-SBP is compiled for
 * N = 1..4 with rules of exactly 6, 10, 18, 22 nodes. */

/* One independent shallow-water instance on a periodic box, or a domain closed (in one or
 * both directions) by reflective walls. */
typedef struct {
  int32_t N;            /* polynomial (and geometry) degree, 1..5                          */
  int32_t K;            /* number of triangles, >= 1                                        */
  const double *xg;     /* [K][Np] x of the equispaced geometry nodes (warped allowed)      */
  const double *yg;     /* [K][Np] y of the same nodes; each element counter-clockwise      */
  const double *b;      /* [K][Np] bathymetry sampled at the same nodes (C0 across faces for
                           the well-balanced property); NULL means b = 0                     */
  double Lx, Ly;        /* periods in x and y; a period <= 0 means the mesh is not periodic
                           in that direction.  Every face must match a face of another
                           element (shifted by a multiple of the period in each periodic
                           direction), except that, when some direction is not periodic, a
                           face no other face matches is a reflective wall (Section 2.9):
                           its exterior state is the interior one with the normal velocity
                           reversed, h+ = h, (u, v)+ = (u, v) - 2 ((u, v) . n) n            */
} esdg_swe_instance;

typedef struct {
  int32_t precision;        /* ESDG_FP64 | ESDG_FP32 | ESDG_FP32_BF16X3                      */
  int32_t flux;             /* ESDG_FLUX_EC | ESDG_FLUX_LF                                   */
  double g;                 /* gravitational constant, > 0                                    */
  int32_t use_graph;        /* nonzero: esdg_swe_step replays HIP graphs of its RK stages    */
  int32_t elems_per_block[6]; /* elements per workgroup for degree N = index (1..5); 0 = the
                                 library's default for that degree; index 0 unused            */
  int32_t matrix_cores;     /* projection/lift contractions with constant operators: 0 or 1 =
                               vector ALUs, 2 = matrix cores (MFMA) in the bulk precision;
                               ESDG_FP32_BF16X3 always uses the split-bf16 matrix-core path  */
  int32_t fused_steps;      /* how esdg_swe_step launches its RK stages: 0 = one launch per
                               stage (HIP graphs if use_graph); 1 = all stages of the call in
                               one launch whose workgroups are all resident (an ordinary
                               launch if a probe at bind saw the grid resident, else a
                               cooperative one), each element tile starting a stage once
                               the tiles of its face neighbours have finished the previous
                               one (no grid-wide barrier); when every workgroup holds at most
                               one tile, that tile also stays in LDS from the first stage to
                               the last; 2 = automatic: 1 when every workgroup holds at most
                               one tile, else 0.  With 1 (or 2 resolving to 1) bind fails with
                               ESDG_EDEVICE where cooperative launch is missing.  Results are
                               bitwise the same in every mode.                                */
  int32_t mass_inverse;     /* ESDG_MASS_STORED | ESDG_MASS_WEIGHT_ADJUSTED (modal scheme)     */
  int32_t tile_shape[6];    /* residual-phase tile shape per degree N = index (1..5), packed
                               (R << 4) | P: R rows per thread (1, or 2 in FP32 where 2 divides
                               Nq and Nfq), P column parts (1..4) whose partial sums the lift
                               adds; 0 = the library's default ((2 << 4) | 2 in FP32 at N = 1
                               and 3, else (1 << 4) | 2); another shape returns ESDG_EINVAL.
                               A shape other than the default needs matrix_cores 0 or 1 and
                               the (N+1)-point quadrature.  The shape changes the summation
                               order only.                                                   */
  int32_t scheme;           /* ESDG_SCHEME_MODAL | ESDG_SCHEME_SBP (every instance a caller's
                               DG-SBP rule; precision FP64 or FP32, flux EC or LF, walls
                               allowed; contractions, mass_inverse and fused_steps do not apply) */
} esdg_swe_options;

/* Plan a solver for n_inst independent instances (n_inst = 1 for a single run).  Builds,
 * on the host in double precision, the reference operators of each degree and quadrature,
 * the isoparametric geometry, the face connectivity (periodic, or reflective walls) and the
 * inverse curved mass matrices, or with ESDG_MASS_WEIGHT_ADJUSTED the weights w/J
 * (Sections 2.1-2.7, 2.9; Section 3 for DG-SBP).  quad is NULL (every instance the default
 * rules) or an array of n_inst entries; instances of one degree must use the same
 * quadrature.  Validates: 1 <= N <= 5 (1..4 for DG-SBP), the quadrature (a caller's rule:
 * positive weights, nodes in the triangle, exactness to the required degree, for DG-SBP the
 * face nodes among its nodes; ESDG_EINVAL otherwise), J > 0 at every quadrature node, every
 * face node matched (or on a wall).  On success *out is a new handle and *workspace_bytes
 * the device workspace size esdg_swe_bind needs.  No device call is made. */
esdg_status esdg_swe_init(int32_t n_inst, const esdg_swe_instance *inst, const esdg_swe_quadrature *quad,
                          const esdg_swe_options *opt, esdg_swe **out, size_t *workspace_bytes);

/* Attach a caller-owned device workspace (>= workspace_bytes, 256-byte aligned) and a
 * HIP stream (hipStream_t as void*, NULL = default stream), then upload the operators
 * and mesh data with asynchronous copies on that stream.  The handle keeps both.  With
 * fused_steps, bind also runs one residency probe of the multi-stage grid (every
 * workgroup counts itself in and waits, bounded, for the rest) and synchronises. */
esdg_status esdg_swe_bind(esdg_swe *s, void *dev_workspace, size_t bytes, void *hip_stream);

/* Set instance `inst`'s state from samples at its geometry nodes: u_nodes is host
 * [3][K][(N+1)(N+2)/2] (h, hu, hv).  The library interpolates to modal coefficients (DG-SBP:
 * evaluates that interpolant at the volume nodes), resets the RK register to zero, sets the
 * reference level and computes the entropy projection (DG-SBP: the face values) of the new
 * state.  Synchronous. */
esdg_status esdg_swe_set_state(esdg_swe *s, int32_t inst, const double *u_nodes);

/* As esdg_swe_set_state, from the state's own coefficients (host [3][K][Np] of h, hu, hv):
 * modal coefficients, or for DG-SBP the values at the rule's volume nodes. */
esdg_status esdg_swe_set_state_modal(esdg_swe *s, int32_t inst, const double *uh);

/* Copy instance `inst`'s state (modal, or nodal for DG-SBP) to the host as double [3][K][Np].  Synchronises the
 * stream; returns ESDG_ENONPHYS if any kernel since the last check flagged a bad state. */
esdg_status esdg_swe_get_state(esdg_swe *s, int32_t inst, double *uh);

/* Device pointer to instance `inst`'s modal state ([3][K][Np] (eta, hu, hv), float for the
 * FP32 modes, double for ESDG_FP64).  Valid until esdg_swe_destroy; reading it is ordered
 * by the bound stream. */
esdg_status esdg_swe_state_device(esdg_swe *s, int32_t inst, void **uh_dev);

/* rhs_dev = du_h/dt of eq. (dgform) evaluated at state_dev for instance `inst`: both are
 * device arrays [3][K][Np] in the library precision (float or double); state_dev holds
 * (eta, hu, hv) as esdg_swe_state_device does, rhs_dev receives d/dt of (h, hu, hv).  Asynchronous on
 * the bound stream; does not touch the instance's own state.  state_dev and rhs_dev must
 * not overlap. */
esdg_status esdg_swe_rhs(esdg_swe *s, int32_t inst, const void *state_dev, void *rhs_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): esdg_swe_rhs without the workspace's
 * RHS scratch.  Same arguments, kernels and results (bitwise) as esdg_swe_rhs; the
 * entropy-projected values and face slots of the evaluation, and its non-physical-state
 * flag, live in a scratch array the library holds per device (64 MiB, kept until the process
 * ends), and the call allocates nothing.  The instance needs
 *   256 + round_up(16 K Nh w, 256) + 16 K Nfq w   bytes of it (w = 4 for float, 8 for double;
 * N=3, K=8192: 5.3 MB in FP32); a larger one returns ESDG_EINVAL (use esdg_swe_rhs).
 * Asynchronous on the bound stream; a non-physical state is reported by the handle's next
 * synchronising call.  Every handle on a device shares that device's array, which keeps the
 * last call's contents: calls that overlap in time on one device (two streams, two handles,
 * two threads) race and give undefined results. */
esdg_status esdg_swe_rhs_noalloc(esdg_swe *s, int32_t inst, const void *state_dev, void *rhs_dev);

/* Advance every instance by nsteps LSRK4(5) steps (5 RHS evaluations each, Section 4).
 * dt is a host array with one time step per instance.  Asynchronous on the bound stream:
 * one kernel launch per RK stage for all instances together, replayed from HIP graphs
 * when use_graph is set, or one launch for all nsteps stages when fused_steps is set.  Non-physical states (ESDG_ENONPHYS) and a fused launch whose neighbour wait
 * gave up (ESDG_EDEVICE; the state is then undefined) are reported by the next
 * synchronising call (get_state, diagnostics, sync). */
esdg_status esdg_swe_step(esdg_swe *s, const double *dt, int32_t nsteps);

/* Per-instance FP64 diagnostics of the current state, out = host [n_inst][6]:
 *   mass of h, hu, hv (sum_k 1^T W J V_q u_h), total entropy sum w J S(u_q) (Section 2.4),
 *   entropy rate sum w J v(u_q).(V_q du/dt) (zero for the EC flux on periodic or
 *   wall-bounded meshes, <= 0 with LF), and the sum of the absolute values of the
 *   entropy-rate terms.
 * Synchronises the stream. */
esdg_status esdg_swe_diagnostics(esdg_swe *s, double *out);

/* Wait for the bound stream; ESDG_ENONPHYS if a kernel flagged a bad state since the
 * last check (the flag is then cleared). */
esdg_status esdg_swe_sync(esdg_swe *s);

/* Reference level Href of instance `inst` (the mean of h + b over the domain at the last
 * set_state; it defines eta = h + b - Href and the H - Href form of the pressure terms,
 * both exact rewritings because the operators annihilate constants).  ESDG_ESTATE before
 * the first set_state. */
esdg_status esdg_swe_reference_level(const esdg_swe *s, int32_t inst, double *Href);

/* Sizes of instance `inst`: out = {N, K, Np, Nq, Nfq, Nh} (Np the state values per field and
 * element; Nq the volume nodes the kernels use, a caller's rule counted with its padding). */
esdg_status esdg_swe_query(const esdg_swe *s, int32_t inst, int32_t *out6);

/* Launch plan (after bind): out = {element tiles, resident workgroups of the stage kernel,
 * LDS bytes per workgroup, step mode (0 = one launch per stage, 1 = one launch per step
 * call re-reading tiles every stage, 2 = one launch per step call with tiles resident in
 * LDS)}.  ESDG_ESTATE before bind. */
esdg_status esdg_swe_launch_info(const esdg_swe *s, int32_t *out4);

/* Message for the last failing call on s (s may be NULL: last failing init on this thread). */
const char *esdg_swe_last_error(const esdg_swe *s);

/* Wait for the work queued on the bound stream (a replay of the handle's HIP graphs or a
 * cooperative launch may still read the workspace), then release the handle's host
 * resources (HIP graphs included).  The workspace and stream remain the caller's and may be
 * freed once this returns.  NULL is ignored. */
void esdg_swe_destroy(esdg_swe *s);

#ifdef __cplusplus
}
#endif

#endif /* ESDG_SWE_H */
