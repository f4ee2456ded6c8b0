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

// Reference element of degree N (Sections 2.1-2.3).
struct RefElem {
  int N = 0, Np = 0, Nq = 0, Nfp = 0, Nfq = 0, Nh = 0;
  std::vector<double> rq, sq, wq;        // volume rule (Stroud, (N+1)^2 points)
  std::vector<double> rf, sf, wf;        // face rule, faces 1..3, N+1 Gauss points each
  std::vector<double> nr, ns;            // reference normals scaled by the face Jacobian
  Mat Vh, Vrh, Vsh;                      // basis and its r/s derivatives at the Nh hybrid nodes
  Mat Vgeo_inv;                          // equispaced node values -> modal coefficients
  // Volume rows (Nq x Nh) of S^j = 1/2 (Qh^j - Qh^j^T), j = r, s: the physical skew
  // operator of an element is sum_j (G_j[m] + G_j[n]) S^j[m, n].
  Mat Sr, Ss;
};

RefElem build_ref(int N);

// Per-instance host data produced from the caller's mesh (Section 2.7).
struct InstanceHost {
  int N = 0, K = 0;
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
