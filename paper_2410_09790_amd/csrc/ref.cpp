// Reference-element data for the HDG-IMEX library: Gauss rules, the
// documented orthonormal bases and the reference matrices the kernels combine
// with per-cell affine geometry.
//
// Spaces (paper, Section "Discontinuous Galerkin spaces" and the trace space of
// Section "Hybridisation"): velocity [P_{k+1}]^2, pressure P_k, trace P_k.
// Bases (part of the data layout, see include/hdg.h):
//   cell  phi_ij = sqrt(2(2i+1)(i+j+1)) P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b),
//         r = 2xi-1, s = 2eta-1, a = 2(1+r)/(1-s)-1, b = s; i+j <= m ordered by
//         total degree, then i ascending;
//   facet mu_i(t) = sqrt(2i+1) P_i(2t-1).
// The paper fixes no quadrature; every polynomial integrand is integrated
// exactly and the facet rule (ceil((3k+4)/2) Gauss-Legendre points) also
// carries the non-polynomial upwind weight |Q*.n|.
#include <cmath>
#include <stdexcept>

#include "hdg_impl.h"

namespace hdg {

int dim_p(int m) { return (m + 1) * (m + 2) / 2; }

// Eigen-decomposition of a small symmetric matrix by cyclic Jacobi rotations.
static void sym_eig(int n, std::vector<double>& A, std::vector<double>& V) {
  V.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-32) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < n; ++r) {  // columns p, q
          double arp = A[r * n + p], arq = A[r * n + q];
          A[r * n + p] = c * arp - s * arq;
          A[r * n + q] = s * arp + c * arq;
        }
        for (int r = 0; r < n; ++r) {  // rows p, q
          double apr = A[p * n + r], aqr = A[q * n + r];
          A[p * n + r] = c * apr - s * aqr;
          A[q * n + r] = s * apr + c * aqr;
        }
        for (int r = 0; r < n; ++r) {
          double vrp = V[r * n + p], vrq = V[r * n + q];
          V[r * n + p] = c * vrp - s * vrq;
          V[r * n + q] = s * vrp + c * vrq;
        }
      }
    }
  }
}

void gauss_jacobi(int n, double al, double be, std::vector<double>& x, std::vector<double>& w) {
  // three-term recurrence of the monic orthogonal polynomials -> Jacobi matrix
  std::vector<double> A(n * n, 0.0), V;
  for (int j = 0; j < n; ++j) {
    double s = 2.0 * j + al + be;
    A[j * n + j] = (s == 0.0) ? (be - al) / (al + be + 2.0) : (be * be - al * al) / (s * (s + 2.0));
    if (j + 1 < n) {
      double jj = j + 1.0, s1 = 2.0 * jj + al + be;
      double b2 = 4.0 * jj * (jj + al) * (jj + be) * (jj + al + be) / (s1 * s1 * (s1 + 1.0) * (s1 - 1.0));
      A[j * n + j + 1] = A[(j + 1) * n + j] = std::sqrt(b2);
    }
  }
  sym_eig(n, A, V);
  double mu0 = std::pow(2.0, al + be + 1.0) * std::tgamma(al + 1.0) * std::tgamma(be + 1.0) / std::tgamma(al + be + 2.0);
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (A[order[j] * n + order[j]] < A[order[i] * n + order[i]]) std::swap(order[i], order[j]);
  x.resize(n);
  w.resize(n);
  for (int i = 0; i < n; ++i) {
    int e = order[i];
    x[i] = A[e * n + e];
    w[i] = mu0 * V[0 * n + e] * V[0 * n + e];
  }
  // the Legendre rule is symmetric: enforce it exactly so mirrored facet
  // points coincide bit for bit
  if (al == 0.0 && be == 0.0) {
    for (int i = 0; i < n / 2; ++i) {
      double xm = 0.5 * (x[n - 1 - i] - x[i]), wm = 0.5 * (w[i] + w[n - 1 - i]);
      x[i] = -xm; x[n - 1 - i] = xm; w[i] = w[n - 1 - i] = wm;
    }
    if (n % 2) x[n / 2] = 0.0;
  }
}

double jacobi_p(int n, double a, double b, double x) {
  if (n == 0) return 1.0;
  double p0 = 1.0, p1 = 0.5 * ((a + b + 2.0) * x + (a - b));
  for (int m = 2; m <= n; ++m) {
    double s = 2.0 * m + a + b;
    double c1 = 2.0 * m * (m + a + b) * (s - 2.0);
    double c2 = (s - 1.0) * (s * (s - 2.0) * x + a * a - b * b);
    double c3 = 2.0 * (m + a - 1.0) * (m + b - 1.0) * s;
    double p2 = (c2 * p1 - c3 * p0) / c1;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

double jacobi_dp(int n, double a, double b, double x) {
  if (n == 0) return 0.0;
  return 0.5 * (n + a + b + 1.0) * jacobi_p(n - 1, a + 1.0, b + 1.0, x);
}

void dubiner_eval(int m, double xi, double eta, double* v, double* dxi, double* deta) {
  double r = 2.0 * xi - 1.0, s = 2.0 * eta - 1.0;
  double a = (std::fabs(1.0 - s) > 1e-300) ? 2.0 * (1.0 + r) / (1.0 - s) - 1.0 : -1.0;
  double b = s, h = 0.5 * (1.0 - b);
  int col = 0;
  for (int d = 0; d <= m; ++d) {
    for (int i = 0; i <= d; ++i, ++col) {
      int j = d - i;
      double nrm = std::sqrt(2.0 * (2 * i + 1) * (i + j + 1));
      double Pa = jacobi_p(i, 0, 0, a), Pb = jacobi_p(j, 2 * i + 1, 0, b);
      double hi = std::pow(h, i);
      v[col] = nrm * Pa * hi * Pb;
      if (dxi) {
        double dPa = jacobi_dp(i, 0, 0, a), dPb = jacobi_dp(j, 2 * i + 1, 0, b);
        double him1 = i >= 1 ? std::pow(h, i - 1) : 0.0;
        dxi[col] = i >= 1 ? nrm * dPa * 2.0 * him1 * Pb : 0.0;
        double dg = (i >= 1 ? -0.5 * i * him1 * Pb : 0.0) + hi * dPb;
        deta[col] = nrm * ((i >= 1 ? dPa * (1.0 + a) * him1 * Pb : 0.0) + 2.0 * Pa * dg);
      }
    }
  }
}

double legendre01(int i, double t) { return std::sqrt(2.0 * i + 1.0) * jacobi_p(i, 0, 0, 2.0 * t - 1.0); }

static void invert(int n, std::vector<double> A, std::vector<double>& out) {
  out.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i) out[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (std::fabs(A[piv * n + c]) < 1e-14) throw std::runtime_error("singular reference matrix");
    for (int j = 0; j < n; ++j) {
      std::swap(A[c * n + j], A[piv * n + j]);
      std::swap(out[c * n + j], out[piv * n + j]);
    }
    double d = 1.0 / A[c * n + c];
    for (int j = 0; j < n; ++j) { A[c * n + j] *= d; out[c * n + j] *= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) { A[r * n + j] -= f * A[c * n + j]; out[r * n + j] -= f * out[c * n + j]; }
    }
  }
}

void build_reference(int k, RefTables& t) {
  if (k < 1 || k > kMaxDegree) throw std::runtime_error("degree out of range");
  t.k = k;
  t.ns = dim_p(k + 1);
  t.np = dim_p(k);
  t.nf = k + 1;
  t.nned = k * (k + 2);
  const int ns = t.ns, np = t.np, nf = t.nf;
  // collapsed cell rule, exact for total degree 3k+2
  int n1 = (3 * k + 4) / 2;  // ceil((3k+3)/2)
  std::vector<double> xa, wa, xb, wb;
  gauss_jacobi(n1, 0.0, 0.0, xa, wa);
  gauss_jacobi(n1, 1.0, 0.0, xb, wb);
  for (int i = 0; i < n1; ++i)
    for (int j = 0; j < n1; ++j) {
      t.cq_xi.push_back((1.0 + xa[i]) * (1.0 - xb[j]) / 4.0);
      t.cq_eta.push_back((1.0 + xb[j]) / 2.0);
      t.cq_w.push_back(wa[i] * wb[j] / 8.0);
    }
  t.nqc = (int)t.cq_w.size();
  // facet Gauss-Legendre rule on [0, 1]
  int nq = (3 * k + 5) / 2;  // ceil((3k+4)/2)
  std::vector<double> xl, wl;
  gauss_jacobi(nq, 0.0, 0.0, xl, wl);
  for (int i = 0; i < nq; ++i) { t.fq_s.push_back(0.5 * (xl[i] + 1.0)); t.fq_w.push_back(0.5 * wl[i]); }
  t.nqf = nq;

  std::vector<double> v(ns), dx(ns), dy(ns), vp(np), dpx(np), dpy(np);
  t.Bu.resize(t.nqc * ns); t.Gux.resize(t.nqc * ns); t.Guy.resize(t.nqc * ns);
  t.Bp.resize(t.nqc * np); t.Gpx.resize(t.nqc * np); t.Gpy.resize(t.nqc * np);
  for (int q = 0; q < t.nqc; ++q) {
    dubiner_eval(k + 1, t.cq_xi[q], t.cq_eta[q], v.data(), dx.data(), dy.data());
    dubiner_eval(k, t.cq_xi[q], t.cq_eta[q], vp.data(), dpx.data(), dpy.data());
    for (int s = 0; s < ns; ++s) { t.Bu[q * ns + s] = v[s]; t.Gux[q * ns + s] = dx[s]; t.Guy[q * ns + s] = dy[s]; }
    for (int s = 0; s < np; ++s) { t.Bp[q * np + s] = vp[s]; t.Gpx[q * np + s] = dpx[s]; t.Gpy[q * np + s] = dpy[s]; }
  }
  t.FBu.resize(3 * nq * ns); t.FGux.resize(3 * nq * ns); t.FGuy.resize(3 * nq * ns); t.FBp.resize(3 * nq * np);
  for (int f = 0; f < 3; ++f)
    for (int q = 0; q < nq; ++q) {
      double xi, eta;
      facet_point(f, t.fq_s[q], xi, eta);
      dubiner_eval(k + 1, xi, eta, v.data(), dx.data(), dy.data());
      dubiner_eval(k, xi, eta, vp.data(), nullptr, nullptr);
      for (int s = 0; s < ns; ++s) {
        t.FBu[(f * nq + q) * ns + s] = v[s];
        t.FGux[(f * nq + q) * ns + s] = dx[s];
        t.FGuy[(f * nq + q) * ns + s] = dy[s];
      }
      for (int s = 0; s < np; ++s) t.FBp[(f * nq + q) * np + s] = vp[s];
    }
  t.MU.resize(nq * nf);
  t.NUB.resize(nq * (k + 2));
  for (int q = 0; q < nq; ++q) {
    for (int m = 0; m < nf; ++m) t.MU[q * nf + m] = legendre01(m, t.fq_s[q]);
    for (int m = 0; m < k + 2; ++m) t.NUB[q * (k + 2) + m] = legendre01(m, t.fq_s[q]);
  }
  // trace of a velocity-degree function on local facet f as a polynomial of
  // degree k+1 in the facet parameter: its coefficients in the orthonormal
  // Legendre basis (exact: the facet rule integrates degree 2k+2)
  t.TRU.assign(3 * (k + 2) * ns, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int q = 0; q < nq; ++q)
      for (int m = 0; m < k + 2; ++m)
        for (int s = 0; s < ns; ++s)
          t.TRU[(f * (k + 2) + m) * ns + s] += t.fq_w[q] * t.NUB[q * (k + 2) + m] * t.FBu[(f * nq + q) * ns + s];
  // reference matrices
  t.Dx.assign(np * ns, 0.0); t.Dy.assign(np * ns, 0.0); t.Rx.assign(np * ns, 0.0); t.Ry.assign(np * ns, 0.0);
  for (int q = 0; q < t.nqc; ++q)
    for (int i = 0; i < np; ++i)
      for (int s = 0; s < ns; ++s) {
        double w = t.cq_w[q];
        t.Dx[i * ns + s] += w * t.Bp[q * np + i] * t.Gux[q * ns + s];
        t.Dy[i * ns + s] += w * t.Bp[q * np + i] * t.Guy[q * ns + s];
        t.Rx[i * ns + s] += w * t.Gpx[q * np + i] * t.Bu[q * ns + s];
        t.Ry[i * ns + s] += w * t.Gpy[q * np + i] * t.Bu[q * ns + s];
      }
  t.Chat.assign(3 * nf * ns, 0.0); t.That.assign(3 * np * np, 0.0); t.Ehat.assign(3 * nf * np, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int q = 0; q < nq; ++q) {
      double w = t.fq_w[q];
      for (int m = 0; m < nf; ++m) {
        for (int s = 0; s < ns; ++s) t.Chat[(f * nf + m) * ns + s] += w * t.MU[q * nf + m] * t.FBu[(f * nq + q) * ns + s];
        for (int i = 0; i < np; ++i) t.Ehat[(f * nf + m) * np + i] += w * t.MU[q * nf + m] * t.FBp[(f * nq + q) * np + i];
      }
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j)
          t.That[(f * np + i) * np + j] += w * t.FBp[(f * nq + q) * np + i] * t.FBp[(f * nq + q) * np + j];
    }
  const double* Da[2] = {t.Dx.data(), t.Dy.data()};
  t.CC.assign(9 * nf * nf, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int g = 0; g < 3; ++g)
      for (int m = 0; m < nf; ++m)
        for (int l = 0; l < nf; ++l) {
          double acc = 0.0;
          for (int s = 0; s < ns; ++s) acc += t.Chat[(f * nf + m) * ns + s] * t.Chat[(g * nf + l) * ns + s];
          t.CC[((f * 3 + g) * nf + m) * nf + l] = acc;
        }
  t.KDD.assign(4 * np * np, 0.0);
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          double acc = 0.0;
          for (int s = 0; s < ns; ++s) acc += Da[a][i * ns + s] * Da[b][j * ns + s];
          t.KDD[((a * 2 + b) * np + i) * np + j] = acc;
        }
  t.CD.assign(6 * nf * np, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int a = 0; a < 2; ++a)
      for (int m = 0; m < nf; ++m)
        for (int j = 0; j < np; ++j) {
          double acc = 0.0;
          for (int s = 0; s < ns; ++s) acc += t.Chat[(f * nf + m) * ns + s] * Da[a][j * ns + s];
          t.CD[((f * 2 + a) * nf + m) * np + j] = acc;
        }
  // reference Nedelec (first kind, degree k) basis: [P_{k-1}]^2 + x^perp P~_{k-1}
  t.NED.assign(t.nqc * t.nned * 2, 0.0);
  for (int q = 0; q < t.nqc; ++q) {
    double X = t.cq_xi[q], Y = t.cq_eta[q];
    int l = 0;
    for (int d = 0; d < k; ++d)
      for (int a = 0; a <= d; ++a) {
        double mval = std::pow(X, d - a) * std::pow(Y, a);
        t.NED[(q * t.nned + l) * 2 + 0] = mval; ++l;
        t.NED[(q * t.nned + l) * 2 + 1] = mval; ++l;
      }
    for (int a = 0; a < k; ++a) {
      double mval = std::pow(X, k - 1 - a) * std::pow(Y, a);
      t.NED[(q * t.nned + l) * 2 + 0] = -Y * mval;
      t.NED[(q * t.nned + l) * 2 + 1] = X * mval;
      ++l;
    }
  }
  // reference BDM moment matrix: rows = normal moments against P_{k+1} on the
  // three facets, then interior moments against the Nedelec basis; columns =
  // velocity coefficients (component-major)
  const int nu = 2 * ns, nm = k + 2;
  const double rn[3][2] = {{M_SQRT1_2, M_SQRT1_2}, {-1.0, 0.0}, {0.0, -1.0}};
  const double flen[3] = {M_SQRT2, 1.0, 1.0};
  std::vector<double> R(nu * nu, 0.0);
  for (int f = 0; f < 3; ++f)
    for (int m = 0; m < nm; ++m)
      for (int q = 0; q < nq; ++q)
        for (int b = 0; b < 2; ++b)
          for (int s = 0; s < ns; ++s)
            R[(f * nm + m) * nu + b * ns + s] += flen[f] * t.fq_w[q] * t.NUB[q * nm + m] * t.FBu[(f * nq + q) * ns + s] * rn[f][b];
  for (int l = 0; l < t.nned; ++l)
    for (int q = 0; q < t.nqc; ++q)
      for (int b = 0; b < 2; ++b)
        for (int s = 0; s < ns; ++s)
          R[(3 * nm + l) * nu + b * ns + s] += t.cq_w[q] * t.NED[(q * t.nned + l) * 2 + b] * t.Bu[q * ns + s];
  invert(nu, R, t.BDMinv);
}

}  // namespace hdg
