// Host-side FP64 setup for the ESDG shallow-water library: reference element of degree
// N (basis, quadrature, hybridized SBP operators) and per-instance mesh data (isoparametric
// geometry, face connectivity with periodic partners or reflective walls, inverse curved
// mass matrices or the weights of their weight-adjusted form).  Nothing here is timed: it
// runs once in esdg_swe_init, before any device work.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace esdg {

inline int n_modes(int N) { return (N + 1) * (N + 2) / 2; }

// Row-major dense matrix of doubles.
struct Mat {
  int rows = 0, cols = 0;
  std::vector<double> a;
  Mat() = default;
  Mat(int r, int c) : rows(r), cols(c), a(size_t(r) * c, 0.0) {}
  double &operator()(int i, int j) { return a[size_t(i) * cols + j]; }
  double operator()(int i, int j) const { return a[size_t(i) * cols + j]; }
};

// A volume quadrature rule on the reference triangle given by the caller.
struct QuadRule {
  std::vector<double> r, s, w;
};

// Checks a caller's volume rule: positive weights, nodes in the closed reference triangle,
// and exactness for every monomial r^a s^b with a + b <= degree (against the closed-form
// integrals).  Returns "" or an error message.
std::string check_rule(const QuadRule &q, int degree);

// Reference element of one element kind (Sections 2.1-2.3; Section 3 for DG-SBP).
struct RefElem {
  int N = 0, Np = 0, Nq = 0, Nfp = 0, Nfq = 0, Nh = 0;
  int key = 0;                           // element kind (device_types.hpp): N | variant << 3
  int nrule = 0;                         // nodes of the volume rule before zero-weight padding
  std::vector<double> rq, sq, wq;        // volume rule (Nq nodes; zero-weight padding at the end)
  std::vector<double> rf, sf, wf;        // face rule, faces 1..3, Nfp Gauss points each
  std::vector<int> fvol, vface;          // DG-SBP: volume node of each face node, face node of
                                         // each volume node (-1 if none)
  std::vector<double> nr, ns;            // reference normals scaled by the face Jacobian
  Mat Vh, Vrh, Vsh;                      // basis and its r/s derivatives at the Nh hybrid nodes
  Mat Vgeo_inv;                          // equispaced node values -> modal coefficients
  // Volume rows (Nq x Nh) of S^j = 1/2 (Qh^j - Qh^j^T), j = r, s: the physical skew
  // operator of an element is sum_j (G_j[m] + G_j[n]) S^j[m, n].
  Mat Sr, Ss;
};

// Reference element of degree N and variant 0, 1 (modal; Stroud rule with N+1+variant
// points per direction, or the caller's rule padded with zero-weight nodes to the variant's
// node count) or 2 (DG-SBP; the caller's rule, whose boundary nodes must include the N+1
// Gauss-Legendre points of every face).  Returns "" or an error message in *err.
RefElem build_ref(int N, int variant, const QuadRule *rule, std::string *err);

// Per-instance host data produced from the caller's mesh (Section 2.7).
struct InstanceHost {
  int N = 0, K = 0, key = 0;
  double Lx = 0, Ly = 0;
  std::vector<double> geo;    // [4][K][Nh]: rxJ, sxJ, ryJ, syJ (J-scaled metric cofactors)
  std::vector<double> wJq;    // [K][Nq]: w_q * J at volume nodes
  std::vector<double> Minv;   // [K][Np][Np]: (V_q^T W diag(J) V_q)^{-1} (empty when not needed)
  std::vector<double> wOverJ; // [K][Nq]: w_q / J at volume nodes (weight-adjusted inverse)
  std::vector<double> bq;     // [K][Nq]: bathymetry at volume nodes
  std::vector<double> bh;     // [K][Nh]: bathymetry at hybrid nodes
  std::vector<double> bmodal; // [K][Np]: modal coefficients of the bathymetry
  std::vector<int32_t> mapP;  // [K][Nfq]: k' * Nh + Nq + f' of the matching neighbour node
                              // (the node itself on a reflective wall)
  std::vector<uint8_t> wall;  // [K][Nfq]: 1 on reflective wall faces (Section 2.9)
  long long nwall = 0;        // wall face nodes
  double Jmin = 0, Jmax = 0;
};

// Returns "" on success or an error message.  xg, yg, b are [K][Np] (b may be null).  With
// want_minv false the inverse curved mass matrices are not formed (weight-adjusted inverse).
std::string build_instance(const RefElem &ref, int K, const double *xg, const double *yg, const double *b,
                           double Lx, double Ly, InstanceHost &out, bool want_minv = true);

// Modal coefficients of the interpolant through equispaced-node samples: out[k][i].
void nodes_to_modes(const RefElem &ref, int K, const double *u_nodes, double *uh);

// Internal consistency checks of the reference operators (used by init): max errors of
// PqVq - I and of the SBP relation and the row sums.  Returns "" if all below tol.
std::string check_ref(const RefElem &ref, double tol);

}  // namespace esdg
