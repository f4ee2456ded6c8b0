// Host-side FP64 setup: reference element, isoparametric geometry, face connectivity
// (periodic, or reflective walls) and inverse curved mass matrices.  See host_setup.hpp.
#include "host_setup.hpp"
#include "device_types.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <unordered_map>

namespace esdg {
namespace {

// Orthonormal Jacobi polynomials P~_0..P~_n at x for weight (1-x)^al (1+x)^be on [-1,1]
// (normalised three-term recurrence).
void jacobi_all(double x, double al, double be, int n, std::vector<double> &P) {
  P.assign(n + 1, 0.0);
  const double g0 = std::pow(2.0, al + be + 1) / (al + be + 1) * std::tgamma(al + 1) * std::tgamma(be + 1) /
                    std::tgamma(al + be + 1);
  P[0] = 1.0 / std::sqrt(g0);
  if (n == 0) return;
  const double g1 = (al + 1) * (be + 1) / (al + be + 3) * g0;
  P[1] = ((al + be + 2) * x / 2 + (al - be) / 2) / std::sqrt(g1);
  double aold = 2.0 / (2 + al + be) * std::sqrt((al + 1) * (be + 1) / (al + be + 3));
  for (int i = 1; i < n; ++i) {
    const double h1 = 2 * i + al + be;
    const double anew =
        2.0 / (h1 + 2) * std::sqrt((i + 1) * (i + 1 + al + be) * (i + 1 + al) * (i + 1 + be) / ((h1 + 1) * (h1 + 3)));
    const double bnew = -(al * al - be * be) / (h1 * (h1 + 2));
    P[i + 1] = ((x - bnew) * P[i] - aold * P[i - 1]) / anew;
    aold = anew;
  }
}

double jacobi(double x, double al, double be, int n) {
  std::vector<double> P;
  jacobi_all(x, al, be, n, P);
  return P[n];
}

double jacobi_d(double x, double al, double be, int n) {
  if (n == 0) return 0.0;
  return std::sqrt(n * (n + al + be + 1)) * jacobi(x, al + 1, be + 1, n - 1);
}

// Gauss-Jacobi rule: roots of P~_n by Newton's method with deflation, weights from the
// Christoffel numbers w_i = 1 / sum_{k<n} P~_k(x_i)^2.
void gauss_jacobi(int n, double al, double be, std::vector<double> &x, std::vector<double> &w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int k = 0; k < n; ++k) {
    double r = -std::cos((2.0 * k + 1.0) * pi / (2.0 * n));
    if (k > 0) r = 0.5 * (r + x[k - 1]);
    for (int it = 0; it < 200; ++it) {
      double s = 0.0;
      for (int j = 0; j < k; ++j) s += 1.0 / (r - x[j]);
      const double p = jacobi(r, al, be, n), dp = jacobi_d(r, al, be, n);
      const double delta = -p / (dp - s * p);
      r += delta;
      if (std::fabs(delta) < 1e-16) break;
    }
    x[k] = r;
  }
  for (int k = 0; k < n; ++k) {   // polish without deflation
    double r = x[k];
    for (int it = 0; it < 3; ++it) r -= jacobi(r, al, be, n) / jacobi_d(r, al, be, n);
    x[k] = r;
  }
  std::sort(x.begin(), x.end());
  for (int k = 0; k < n; ++k) {
    std::vector<double> P;
    jacobi_all(x[k], al, be, n - 1, P);
    double s = 0.0;
    for (int j = 0; j < n; ++j) s += P[j] * P[j];
    w[k] = 1.0 / s;
  }
}

// Orthonormal Dubiner basis and gradient at (r, s), modes "for i: for j <= N-i".
void dubiner(int N, double r, double s, double *phi, double *dr, double *ds) {
  const double a = (std::fabs(1.0 - s) > 1e-14) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  const double b = s;
  const double sq2 = std::sqrt(2.0);
  int m = 0;
  for (int i = 0; i <= N; ++i) {
    const double fa = jacobi(a, 0, 0, i), dfa = jacobi_d(a, 0, 0, i);
    const double omb_i = std::pow(1.0 - b, i);
    const double omb_im1 = (i > 0) ? std::pow(1.0 - b, i - 1) : 0.0;
    for (int j = 0; j <= N - i; ++j, ++m) {
      const double gb = jacobi(b, 2 * i + 1, 0, j), dgb = jacobi_d(b, 2 * i + 1, 0, j);
      phi[m] = sq2 * fa * gb * omb_i;
      if (dr) dr[m] = sq2 * 2.0 * dfa * gb * omb_im1;
      if (ds) ds[m] = sq2 * (dfa * (1.0 + a) * gb * omb_im1 + fa * (dgb * omb_i - i * gb * omb_im1));
    }
  }
}

Mat matmul(const Mat &A, const Mat &B) {
  Mat C(A.rows, B.cols);
  for (int i = 0; i < A.rows; ++i)
    for (int k = 0; k < A.cols; ++k) {
      const double aik = A(i, k);
      for (int j = 0; j < B.cols; ++j) C(i, j) += aik * B(k, j);
    }
  return C;
}

Mat transpose(const Mat &A) {
  Mat T(A.cols, A.rows);
  for (int i = 0; i < A.rows; ++i)
    for (int j = 0; j < A.cols; ++j) T(j, i) = A(i, j);
  return T;
}

// Inverse by Gauss-Jordan elimination with partial pivoting; false if singular.
bool invert(const Mat &A, Mat &Ainv) {
  const int n = A.rows;
  Mat W = A;
  Ainv = Mat(n, n);
  for (int i = 0; i < n; ++i) Ainv(i, i) = 1.0;
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(W(r, c)) > std::fabs(W(p, c))) p = r;
    if (std::fabs(W(p, c)) < 1e-300) return false;
    if (p != c)
      for (int j = 0; j < n; ++j) {
        std::swap(W(p, j), W(c, j));
        std::swap(Ainv(p, j), Ainv(c, j));
      }
    const double d = 1.0 / W(c, c);
    for (int j = 0; j < n; ++j) {
      W(c, j) *= d;
      Ainv(c, j) *= d;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = W(r, c);
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        W(r, j) -= f * W(c, j);
        Ainv(r, j) -= f * Ainv(c, j);
      }
    }
  }
  return true;
}

// Inverse of a symmetric positive definite matrix through its Cholesky factor L L^T.
bool spd_inverse(int n, const double *A, double *Ainv) {
  std::vector<double> L(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = A[j * n + j];
    for (int k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) return false;
    L[j * n + j] = std::sqrt(d);
    for (int i = j + 1; i < n; ++i) {
      double v = A[i * n + j];
      for (int k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  // Linv (lower triangular)
  std::vector<double> Li(size_t(n) * n, 0.0);
  for (int c = 0; c < n; ++c) {
    Li[c * n + c] = 1.0 / L[c * n + c];
    for (int i = c + 1; i < n; ++i) {
      double v = 0.0;
      for (int k = c; k < i; ++k) v -= L[i * n + k] * Li[k * n + c];
      Li[i * n + c] = v / L[i * n + i];
    }
  }
  // A^{-1} = Linv^T Linv
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      double v = 0.0;
      for (int k = std::max(i, j); k < n; ++k) v += Li[k * n + i] * Li[k * n + j];
      Ainv[i * n + j] = v;
    }
  return true;
}

}  // namespace

std::string check_rule(const QuadRule &q, int degree) {
  const size_t n = q.w.size();
  if (n == 0 || q.r.size() != n || q.s.size() != n) return "quadrature rule: empty, or r, s, w of different lengths";
  char buf[200];
  for (size_t i = 0; i < n; ++i) {
    if (!(q.w[i] > 0.0) || !std::isfinite(q.w[i])) {
      std::snprintf(buf, sizeof buf, "quadrature rule: weight %zu is %.3e (must be positive)", i, q.w[i]);
      return buf;
    }
    const double r = q.r[i], s = q.s[i];
    if (!(r >= -1.0 - 1e-12 && s >= -1.0 - 1e-12 && r + s <= 1e-12)) {
      std::snprintf(buf, sizeof buf, "quadrature rule: node %zu (%.6f, %.6f) outside the reference triangle", i, r, s);
      return buf;
    }
  }
  // int_T r^a s^b = int_{-1}^{1} s^b ((-s)^(a+1) - (-1)^(a+1)) / (a+1) ds
  auto pint = [](int p) { return (p % 2) ? 0.0 : 2.0 / (p + 1); };
  for (int d = 0; d <= degree; ++d)
    for (int a = 0; a <= d; ++a) {
      const int b = d - a;
      const double sg = (a + 1) % 2 ? -1.0 : 1.0;   // (-1)^(a+1)
      const double exact = sg * (pint(a + b + 1) - pint(b)) / (a + 1);
      double sum = 0.0, mag = 0.0;
      for (size_t i = 0; i < n; ++i) {
        const double t = q.w[i] * std::pow(q.r[i], a) * std::pow(q.s[i], b);
        sum += t;
        mag += std::fabs(t);
      }
      if (std::fabs(sum - exact) > 1e-12 * std::max(1.0, mag)) {
        std::snprintf(buf, sizeof buf, "quadrature rule: not exact for r^%d s^%d (degree %d required): %.6e vs %.6e",
                      a, b, degree, sum, exact);
        return buf;
      }
    }
  return "";
}

RefElem build_ref(int N, int variant, const QuadRule *rule, std::string *err) {
  RefElem R;
  const int D = make_key(N, variant);
  R.N = N;
  R.key = D;
  R.Np = n_modes(N);
  R.Nfp = dim_Nfp(D);
  R.Nq = dim_Nq(D);
  R.Nfq = dim_Nfq(D);
  R.Nh = R.Nq + R.Nfq;
  const int Np = R.Np, Nq = R.Nq, Nfq = R.Nfq, Nh = R.Nh, Nfp = R.Nfp;
  // volume rule: the caller's, or Gauss-Legendre in a times Gauss-Jacobi(1,0) in b, collapsed
  if (rule) {
    R.rq = rule->r; R.sq = rule->s; R.wq = rule->w;
  } else {
    std::vector<double> xa, wa, xb, wb;
    const int q = N + 1 + variant;
    gauss_jacobi(q, 0.0, 0.0, xa, wa);
    gauss_jacobi(q, 1.0, 0.0, xb, wb);
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) {
        R.rq.push_back((1.0 + xa[i]) * (1.0 - xb[j]) / 2.0 - 1.0);
        R.sq.push_back(xb[j]);
        R.wq.push_back(0.5 * wa[i] * wb[j]);
      }
  }
  R.nrule = int(R.wq.size());
  if (R.nrule > Nq || (variant == 2 && R.nrule != Nq)) {
    if (err) *err = "quadrature rule has " + std::to_string(R.nrule) + " nodes; this element kind takes " +
                    (variant == 2 ? "exactly " : "at most ") + std::to_string(Nq);
    return R;
  }
  // zero-weight padding (at the centroid): such a node has zero rows and columns in every
  // weighted operator, so it leaves the scheme unchanged
  while (int(R.wq.size()) < Nq) {
    R.rq.push_back(-1.0 / 3.0);
    R.sq.push_back(-1.0 / 3.0);
    R.wq.push_back(0.0);
  }
  // faces: s=-1 (v1->v2), r+s=0 (v2->v3), r=-1 (v3->v1), Nfp Gauss-Legendre points each
  std::vector<double> xf, wfl;
  gauss_jacobi(Nfp, 0.0, 0.0, xf, wfl);
  for (int f = 0; f < 3; ++f)
    for (int i = 0; i < Nfp; ++i) {
      const double t = xf[i];
      double r, s, nr_, ns_;
      if (f == 0) { r = t; s = -1.0; nr_ = 0.0; ns_ = -1.0; }
      else if (f == 1) { r = -t; s = t; nr_ = 1.0; ns_ = 1.0; }
      else { r = -1.0; s = -t; nr_ = -1.0; ns_ = 0.0; }
      R.rf.push_back(r); R.sf.push_back(s); R.wf.push_back(wfl[i]);
      R.nr.push_back(nr_); R.ns.push_back(ns_);
    }
  if (variant == 2) {              // DG-SBP: every face node is one of the volume nodes
    R.fvol.assign(Nfq, -1);
    R.vface.assign(Nq, -1);
    for (int f = 0; f < Nfq; ++f) {
      for (int q = 0; q < Nq; ++q)
        if (std::hypot(R.rq[q] - R.rf[f], R.sq[q] - R.sf[f]) < 1e-12) {
          R.fvol[f] = q;
          break;
        }
      if (R.fvol[f] < 0) {
        char buf[200];
        std::snprintf(buf, sizeof buf, "DG-SBP rule: face node (%.6f, %.6f) (Gauss-Legendre point %d of face %d) is "
                      "not a volume node", R.rf[f], R.sf[f], f % Nfp, f / Nfp);
        if (err) *err = buf;
        return R;
      }
      if (R.vface[R.fvol[f]] >= 0) {
        if (err) *err = "DG-SBP rule: two face nodes at one volume node";
        return R;
      }
      R.vface[R.fvol[f]] = f;
    }
  }
  // basis at hybrid nodes
  R.Vh = Mat(Nh, Np); R.Vrh = Mat(Nh, Np); R.Vsh = Mat(Nh, Np);
  for (int n = 0; n < Nh; ++n) {
    const double r = n < Nq ? R.rq[n] : R.rf[n - Nq];
    const double s = n < Nq ? R.sq[n] : R.sf[n - Nq];
    dubiner(N, r, s, &R.Vh.a[size_t(n) * Np], &R.Vrh.a[size_t(n) * Np], &R.Vsh.a[size_t(n) * Np]);
  }
  // equispaced Vandermonde
  Mat Vg(Np, Np);
  {
    int p = 0;
    for (int j = 0; j <= N; ++j)
      for (int i = 0; i <= N - j; ++i, ++p)
        dubiner(N, -1.0 + 2.0 * i / N, -1.0 + 2.0 * j / N, &Vg.a[size_t(p) * Np], nullptr, nullptr);
  }
  invert(Vg, R.Vgeo_inv);
  // Vq, Vf, Vr at volume nodes
  Mat Vq(Nq, Np), Vf(Nfq, Np), Vrq(Nq, Np), Vsq(Nq, Np);
  for (int q = 0; q < Nq; ++q)
    for (int i = 0; i < Np; ++i) {
      Vq(q, i) = R.Vh(q, i); Vrq(q, i) = R.Vrh(q, i); Vsq(q, i) = R.Vsh(q, i);
    }
  for (int f = 0; f < Nfq; ++f)
    for (int i = 0; i < Np; ++i) Vf(f, i) = R.Vh(Nq + f, i);
  // M, Pq = M^-1 Vq^T W (M is the identity for a rule exact to degree 2N; a DG-SBP rule of
  // degree 2N-1 gives another symmetric positive definite M)
  Mat VqTW = transpose(Vq);
  for (int i = 0; i < Np; ++i)
    for (int q = 0; q < Nq; ++q) VqTW(i, q) *= R.wq[q];
  Mat M = matmul(VqTW, Vq), Minv;
  if (!invert(M, Minv)) {
    if (err) *err = "quadrature rule: the mass matrix V_q^T W V_q is singular (too few nodes for degree " +
                    std::to_string(N) + ")";
    return R;
  }
  Mat Pq = matmul(Minv, VqTW);
  Mat E = matmul(Vf, Pq);
  Mat PqT = transpose(Pq);
  R.Sr = Mat(Nq, Nh);
  R.Ss = Mat(Nq, Nh);
  for (int dir = 0; dir < 2; ++dir) {
    const Mat &Vd = dir == 0 ? Vrq : Vsq;
    const std::vector<double> &nd = dir == 0 ? R.nr : R.ns;
    Mat Qhat = matmul(VqTW, Vd);                     // M D^j = V_q^T W (d_j phi)(x_q)
    Mat Q = matmul(matmul(PqT, Qhat), Pq);           // P_q^T Qhat P_q
    Mat &S = dir == 0 ? R.Sr : R.Ss;
    for (int m = 0; m < Nq; ++m) {
      for (int n = 0; n < Nq; ++n) S(m, n) = 0.5 * (Q(m, n) - Q(n, m));
      for (int f = 0; f < Nfq; ++f) S(m, Nq + f) = 0.5 * E(f, m) * R.wf[f] * nd[f];
    }
  }
  if (err) err->clear();
  return R;
}

std::string check_ref(const RefElem &R, double tol) {
  // sum_n S^j[m, n] over volume rows equals -1/2 of the zero-padded B row sum (zero);
  // for the full skew operator: Qh 1 = 0 and Qh + Qh^T = Bh imply S 1 = -1/2 Bh 1.
  // Volume rows have no B, so every volume row of S must sum to zero.
  double err = 0.0;
  for (int dir = 0; dir < 2; ++dir) {
    const Mat &S = dir == 0 ? R.Sr : R.Ss;
    for (int m = 0; m < R.Nq; ++m) {
      double s = 0.0;
      for (int n = 0; n < R.Nh; ++n) s += S(m, n);
      err = std::max(err, std::fabs(s));
    }
    // face rows: -sum_m S[m, Nq+f] must equal -1/2 wf n_f
    const std::vector<double> &nd = dir == 0 ? R.nr : R.ns;
    for (int f = 0; f < R.Nfq; ++f) {
      double s = 0.0;
      for (int m = 0; m < R.Nq; ++m) s -= S(m, R.Nq + f);
      err = std::max(err, std::fabs(s + 0.5 * R.wf[f] * nd[f]));
    }
  }
  double wsum = 0.0;
  for (double w : R.wq) wsum += w;
  err = std::max(err, std::fabs(wsum - 2.0));
  if (err > tol) {
    char buf[128];
    std::snprintf(buf, sizeof buf, "reference operator check failed for N=%d (err %.3e)", R.N, err);
    return buf;
  }
  return "";
}

void nodes_to_modes(const RefElem &R, int K, const double *u, double *uh) {
  const int Np = R.Np;
  for (int k = 0; k < K; ++k)
    for (int i = 0; i < Np; ++i) {
      double v = 0.0;
      for (int p = 0; p < Np; ++p) v += R.Vgeo_inv(i, p) * u[size_t(k) * Np + p];
      uh[size_t(k) * Np + i] = v;
    }
}

std::string build_instance(const RefElem &R, int K, const double *xg, const double *yg, const double *b, double Lx,
                           double Ly, InstanceHost &out, bool want_minv) {
  const int Np = R.Np, Nq = R.Nq, Nh = R.Nh, Nfp = R.Nfp, Nfq = R.Nfq;
  out.N = R.N; out.key = R.key; out.K = K; out.Lx = Lx; out.Ly = Ly;
  out.geo.assign(size_t(4) * K * Nh, 0.0);
  out.wJq.assign(size_t(K) * Nq, 0.0);
  if (want_minv) out.Minv.assign(size_t(K) * Np * Np, 0.0);
  else out.Minv.clear();
  out.wOverJ.assign(size_t(K) * Nq, 0.0);
  out.bq.assign(size_t(K) * Nq, 0.0);
  out.bh.assign(size_t(K) * Nh, 0.0);
  out.bmodal.assign(size_t(K) * Np, 0.0);
  out.mapP.assign(size_t(K) * Nfq, -1);
  std::vector<double> xh(size_t(K) * Nh), yh(size_t(K) * Nh);
  std::vector<double> xm(Np), ym(Np), bm(Np), Mh(size_t(Np) * Np);
  double Jmin = 1e300, Jmax = -1e300;
  char buf[256];
  for (int k = 0; k < K; ++k) {
    for (int i = 0; i < Np; ++i) {
      double sx = 0, sy = 0, sb = 0;
      for (int p = 0; p < Np; ++p) {
        const double c = R.Vgeo_inv(i, p);
        sx += c * xg[size_t(k) * Np + p];
        sy += c * yg[size_t(k) * Np + p];
        if (b) sb += c * b[size_t(k) * Np + p];
      }
      xm[i] = sx; ym[i] = sy; bm[i] = sb;
      out.bmodal[size_t(k) * Np + i] = sb;
    }
    std::vector<double> J(Nh);
    for (int n = 0; n < Nh; ++n) {
      double xr = 0, xs = 0, yr = 0, ys = 0, xx = 0, yy = 0, bb = 0;
      for (int i = 0; i < Np; ++i) {
        xr += R.Vrh(n, i) * xm[i]; xs += R.Vsh(n, i) * xm[i];
        yr += R.Vrh(n, i) * ym[i]; ys += R.Vsh(n, i) * ym[i];
        xx += R.Vh(n, i) * xm[i]; yy += R.Vh(n, i) * ym[i];
        bb += R.Vh(n, i) * bm[i];
      }
      const size_t o = size_t(k) * Nh + n, plane = size_t(K) * Nh;
      out.geo[0 * plane + o] = ys;
      out.geo[1 * plane + o] = -yr;
      out.geo[2 * plane + o] = -xs;
      out.geo[3 * plane + o] = xr;
      J[n] = xr * ys - xs * yr;
      xh[o] = xx; yh[o] = yy;
      out.bh[o] = bb;
      if (n < Nq) out.bq[size_t(k) * Nq + n] = bb;
    }
    for (int q = 0; q < Nq; ++q) {
      if (!(J[q] > 0.0)) {
        std::snprintf(buf, sizeof buf, "element %d: Jacobian %.3e <= 0 at volume node %d (clockwise or folded)", k,
                      J[q], q);
        return buf;
      }
      Jmin = std::min(Jmin, J[q]); Jmax = std::max(Jmax, J[q]);
      out.wJq[size_t(k) * Nq + q] = R.wq[q] * J[q];
      out.wOverJ[size_t(k) * Nq + q] = R.wq[q] / J[q];
    }
    if (!want_minv) continue;
    for (int i = 0; i < Np; ++i)
      for (int j = 0; j < Np; ++j) {
        double v = 0.0;
        for (int q = 0; q < Nq; ++q) v += R.Vh(q, i) * out.wJq[size_t(k) * Nq + q] * R.Vh(q, j);
        Mh[size_t(i) * Np + j] = v;
      }
    if (!spd_inverse(Np, Mh.data(), &out.Minv[size_t(k) * Np * Np])) {
      std::snprintf(buf, sizeof buf, "element %d: curved mass matrix not positive definite", k);
      return buf;
    }
  }
  out.Jmin = Jmin; out.Jmax = Jmax;

  // face matching through quantised face midpoints, wrapped in each periodic direction (a
  // period <= 0: none).  A face no other face matches is a reflective wall (Section 2.9)
  // when some direction is not periodic; on a fully periodic box it is a mesh error.
  const bool px = Lx > 0.0, py = Ly > 0.0;
  auto wrap = [](double v, double L) {
    if (!(L > 0.0)) return v;
    double w = std::fmod(v, L);
    if (w < 0) w += L;
    return w;
  };
  out.wall.assign(size_t(K) * Nfq, 0);
  out.nwall = 0;
  double hmin = 1e300;
  std::vector<double> mx(size_t(K) * 3), my(size_t(K) * 3);
  for (int k = 0; k < K; ++k)
    for (int f = 0; f < 3; ++f) {
      double sx = 0, sy = 0;
      for (int i = 0; i < Nfp; ++i) {
        const size_t o = size_t(k) * Nh + Nq + f * Nfp + i;
        sx += xh[o]; sy += yh[o];
      }
      mx[k * 3 + f] = wrap(sx / Nfp, Lx);
      my[k * 3 + f] = wrap(sy / Nfp, Ly);
      const size_t o0 = size_t(k) * Nh + Nq + f * Nfp, o1 = o0 + Nfp - 1;
      hmin = std::min(hmin, std::hypot(xh[o1] - xh[o0], yh[o1] - yh[o0]));
    }
  const double tol = 1e-8 * std::max(std::max(Lx, Ly), 0.0) + 1e-6 * hmin;
  const double cell = 4.0 * tol;
  const int64_t ncx = px ? std::max<int64_t>(1, int64_t(std::ceil(Lx / cell))) : 0;
  const int64_t ncy = py ? std::max<int64_t>(1, int64_t(std::ceil(Ly / cell))) : 0;
  const int64_t kOff = int64_t(1) << 30;     // non-periodic cell indices: offset, then packed
  auto cell_key = [&](int64_t cx, int64_t cy) {
    cx = px ? ((cx % ncx) + ncx) % ncx : cx + kOff;
    cy = py ? ((cy % ncy) + ncy) % ncy : cy + kOff;
    return cx * (int64_t(2) * kOff) + cy;
  };
  std::unordered_map<int64_t, std::vector<int>> grid;
  grid.reserve(size_t(K) * 3 * 2);
  for (int e = 0; e < 3 * K; ++e)
    grid[cell_key(int64_t(std::floor(mx[e] / cell)), int64_t(std::floor(my[e] / cell)))].push_back(e);
  auto pdist = [&](double x1, double y1, double x2, double y2) {
    double dx = x2 - x1, dy = y2 - y1;
    if (px) dx -= Lx * std::nearbyint(dx / Lx);
    if (py) dy -= Ly * std::nearbyint(dy / Ly);
    return std::hypot(dx, dy);
  };
  for (int e = 0; e < 3 * K; ++e) {
    const int64_t cx = int64_t(std::floor(mx[e] / cell)), cy = int64_t(std::floor(my[e] / cell));
    int partner = -1, count = 0;
    for (int64_t dx = -1; dx <= 1; ++dx)
      for (int64_t dy = -1; dy <= 1; ++dy) {
        auto it = grid.find(cell_key(cx + dx, cy + dy));
        if (it == grid.end()) continue;
        for (int e2 : it->second)
          if (e2 != e && pdist(mx[e], my[e], mx[e2], my[e2]) < tol) {
            if (e2 != partner) ++count;
            partner = e2;
          }
      }
    if (count == 0 && !(px && py)) {   // reflective wall: each node is its own exterior node
      const int k = e / 3, f = e % 3;
      for (int i = 0; i < Nfp; ++i) {
        out.mapP[size_t(k) * Nfq + f * Nfp + i] = int32_t(size_t(k) * Nh + Nq + f * Nfp + i);
        out.wall[size_t(k) * Nfq + f * Nfp + i] = 1;
      }
      out.nwall += Nfp;
      continue;
    }
    if (count != 1) {
      std::snprintf(buf, sizeof buf, "face %d of element %d has %d partners (need exactly 1%s)", e % 3, e / 3, count,
                    px && py ? " on a fully periodic box" : "");
      return buf;
    }
    const int k = e / 3, f = e % 3, k2 = partner / 3, f2 = partner % 3;
    for (int i = 0; i < Nfp; ++i) {
      const size_t o = size_t(k) * Nh + Nq + f * Nfp + i;
      int best = -1;
      double bd = 1e300;
      for (int j = 0; j < Nfp; ++j) {
        const size_t o2 = size_t(k2) * Nh + Nq + f2 * Nfp + j;
        const double d = pdist(xh[o], yh[o], xh[o2], yh[o2]);
        if (d < bd) { bd = d; best = j; }
      }
      if (bd > tol) {
        std::snprintf(buf, sizeof buf, "face node %d of face %d, element %d is unmatched (distance %.3e)", i, f, k, bd);
        return buf;
      }
      out.mapP[size_t(k) * Nfq + f * Nfp + i] = int32_t(size_t(k2) * Nh + Nq + f2 * Nfp + best);
    }
  }
  return "";
}

}  // namespace esdg
