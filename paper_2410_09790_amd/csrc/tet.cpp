// Tetrahedral meshes and reference data of the three-dimensional HDG-IMEX
// path (the method is stated for d = 2 and 3: Sections "Discontinuous
// Galerkin spaces" and "Hybridisation"; velocity [P_{k+1}]^3, pressure P_k,
// trace P_k on triangles).
//
// Layout contract (see include/hdg.h):
// * local facet f of a cell is the triangle opposite local vertex f, with
//   local vertices LF[f] in ascending order;
// * facets are the distinct sorted vertex triples (lo, mid, hi), numbered in
//   lexicographic order; on facet F the point with facet coordinates (s, t)
//   is x_lo + s (x_mid - x_lo) + t (x_hi - x_lo), and the trace basis is a
//   function of (s, t), so both cells of a facet see the same trace function;
// * a cell sees its local facet f with one of six orientations: perm p lists
//   which local positions of LF[f] hold lo, mid and hi (PERM3[p]);
// * bases: monomials of the centred coordinates x' = (d + 1) x - 1, of total
//   degree <= m, by degree and then in descending lexicographic order of the
//   exponents, orthonormalised in that order (Gram-Schmidt, here classical
//   with one re-orthogonalisation) on the reference simplex; the facet bases
//   are orthonormal for twice the reference triangle's measure, so that on a
//   facet of area |F| the trace functions are orthogonal with norm^2 |F|.
// * rules: the collapsed (Duffy) Gauss rule on the reference tetrahedron
//   with ceil((3k+3)/2) points per direction (exact for degree 3k+2), and the
//   collapsed rule on the facet triangle with ceil((3k+4)/2) points per
//   direction (exact for 3k+3; it also carries the upwind weight |Q*.n|).
#include <algorithm>
#include <cmath>
#include <stdexcept>
#include <string>

#include "hdg_impl.h"

namespace hdg {

namespace {

// exponent tuples of total degree <= m in d variables: by degree, then
// descending lexicographic order
std::vector<std::array<int, 3>> exponents(int m, int d) {
  std::vector<std::array<int, 3>> out;
  for (int deg = 0; deg <= m; ++deg) {
    std::vector<std::array<int, 3>> lev;
    for (int a = deg; a >= 0; --a)
      for (int b = deg - a; b >= 0; --b) {
        const int c = deg - a - b;
        if (d == 2) {
          if (c == 0) lev.push_back({a, b, 0});
        } else {
          lev.push_back({a, b, c});
        }
      }
    // a descending, then b descending, then c descending: the generation order
    out.insert(out.end(), lev.begin(), lev.end());
  }
  return out;
}

struct Rule {
  std::vector<double> x, y, z, w;
};

// collapsed Gauss rule on the reference triangle (d = 2) or tetrahedron (d = 3)
Rule simplex_rule(int n, int d) {
  Rule r;
  std::vector<double> a, wa, b, wb, c, wc;
  gauss_jacobi(n, 0.0, 0.0, a, wa);
  gauss_jacobi(n, 1.0, 0.0, b, wb);
  if (d == 2) {
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        r.x.push_back((1.0 + a[i]) * (1.0 - b[j]) / 4.0);
        r.y.push_back((1.0 + b[j]) / 2.0);
        r.z.push_back(0.0);
        r.w.push_back(wa[i] * wb[j] / 8.0);
      }
    return r;
  }
  gauss_jacobi(n, 2.0, 0.0, c, wc);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int l = 0; l < n; ++l) {
        const double zeta = (1.0 + c[l]) / 2.0;
        const double eta = (1.0 + b[j]) / 2.0 * (1.0 - zeta);
        const double xi = (1.0 + a[i]) / 2.0 * (1.0 - eta - zeta);
        r.x.push_back(xi);
        r.y.push_back(eta);
        r.z.push_back(zeta);
        r.w.push_back(wa[i] * wb[j] * wc[l] / 64.0);
      }
  return r;
}

double ipow(double v, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= v;
  return r;
}

}  // namespace

// --------------------------------------------------------------- bases
OrthoSimplexBasis::OrthoSimplexBasis(int m_, int d_, double scale) : m(m_), d(d_) {
  exps = exponents(m, d);
  n = (int)exps.size();
  const Rule r = simplex_rule(m + 1, d);  // exact for degree 2m + 1
  const int nq = (int)r.w.size();
  // values of the monomials at the rule points, and coefficient vectors
  std::vector<double> V((size_t)n * nq), C((size_t)n * n, 0.0);
  std::vector<double> mono(n);
  for (int q = 0; q < nq; ++q) {
    eval_monomials(r.x[q], r.y[q], r.z[q], mono.data(), nullptr);
    for (int j = 0; j < n; ++j) V[(size_t)j * nq + q] = mono[j];
  }
  auto dot = [&](const double* u, const double* v) {
    double s = 0.0;
    for (int q = 0; q < nq; ++q) s += scale * r.w[q] * u[q] * v[q];
    return s;
  };
  for (int j = 0; j < n; ++j) {
    double* vj = &V[(size_t)j * nq];
    double* cj = &C[(size_t)j * n];
    cj[j] = 1.0;
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        const double* vi = &V[(size_t)i * nq];
        const double* ci = &C[(size_t)i * n];
        const double h = dot(vi, vj);
        for (int q = 0; q < nq; ++q) vj[q] -= h * vi[q];
        for (int l = 0; l < n; ++l) cj[l] -= h * ci[l];
      }
    const double nrm = std::sqrt(dot(vj, vj));
    for (int q = 0; q < nq; ++q) vj[q] /= nrm;
    for (int l = 0; l < n; ++l) cj[l] /= nrm;
  }
  coef = C;  // basis j = sum_l coef[j][l] monomial_l
}

void OrthoSimplexBasis::eval_monomials(double x, double y, double z, double* v, double (*dv)[3]) const {
  const double s = d + 1.0;
  const double X[3] = {s * x - 1.0, s * y - 1.0, s * z - 1.0};
  for (int j = 0; j < n; ++j) {
    const auto& e = exps[j];
    v[j] = ipow(X[0], e[0]) * ipow(X[1], e[1]) * ipow(X[2], e[2]);
    if (dv) {
      for (int a = 0; a < 3; ++a) {
        if (e[a] == 0) { dv[j][a] = 0.0; continue; }
        double t = s * e[a];
        for (int b = 0; b < 3; ++b) t *= ipow(X[b], e[b] - (b == a ? 1 : 0));
        dv[j][a] = t;
      }
    }
  }
}

void OrthoSimplexBasis::eval(double x, double y, double z, double* v, double* dx, double* dy, double* dz) const {
  std::vector<double> mono(n);
  std::vector<double> dm((size_t)3 * n);
  eval_monomials(x, y, z, mono.data(), reinterpret_cast<double(*)[3]>(dm.data()));
  for (int j = 0; j < n; ++j) {
    double a = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
    for (int l = 0; l < n; ++l) {
      const double c = coef[(size_t)j * n + l];
      a += c * mono[l];
      gx += c * dm[3 * l + 0];
      gy += c * dm[3 * l + 1];
      gz += c * dm[3 * l + 2];
    }
    v[j] = a;
    if (dx) dx[j] = gx;
    if (dy) dy[j] = gy;
    if (dz) dz[j] = gz;
  }
}

// ----------------------------------------------------- reference tables
int dim_p3(int m) { return (m + 1) * (m + 2) * (m + 3) / 6; }

// reference coordinates of local vertex v
static const double kRefVert[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

void facet_point3(int f, int p, double s, double t, double* xi) {
  const int* lf = LF3[f];
  const int lo = lf[PERM3[p][0]], mid = lf[PERM3[p][1]], hi = lf[PERM3[p][2]];
  for (int a = 0; a < 3; ++a)
    xi[a] = kRefVert[lo][a] + s * (kRefVert[mid][a] - kRefVert[lo][a]) + t * (kRefVert[hi][a] - kRefVert[lo][a]);
}

// facet coordinates, in the cell's own orientation of local facet f (perm 0),
// of the point with coordinates (s, t) in orientation p
static void local_facet_coords(int p, double s, double t, double& sl, double& tl) {
  double bary[3];  // weights of the local positions 0, 1, 2 of LF[f]
  bary[PERM3[p][0]] = 1.0 - s - t;
  bary[PERM3[p][1]] = s;
  bary[PERM3[p][2]] = t;
  sl = bary[1];
  tl = bary[2];
}

static void invert_dense(int n, std::vector<double> A, std::vector<double>& out) {
  out.assign((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) out[(size_t)i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[(size_t)r * n + c]) > std::fabs(A[(size_t)piv * n + c])) piv = r;
    if (std::fabs(A[(size_t)piv * n + c]) < 1e-13) throw std::runtime_error("singular reference BDM matrix");
    for (int j = 0; j < n; ++j) {
      std::swap(A[(size_t)c * n + j], A[(size_t)piv * n + j]);
      std::swap(out[(size_t)c * n + j], out[(size_t)piv * n + j]);
    }
    const double dd = 1.0 / A[(size_t)c * n + c];
    for (int j = 0; j < n; ++j) { A[(size_t)c * n + j] *= dd; out[(size_t)c * n + j] *= dd; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * n + c];
      if (f == 0.0) continue;
      for (int j = 0; j < n; ++j) {
        A[(size_t)r * n + j] -= f * A[(size_t)c * n + j];
        out[(size_t)r * n + j] -= f * out[(size_t)c * n + j];
      }
    }
  }
}

void build_reference3(int k, RefTables3& t) {
  if (k < 1 || k > kMaxDegree3) throw std::runtime_error("degree out of range for tetrahedra");
  t.k = k;
  t.ns = dim_p3(k + 1);
  t.np = dim_p3(k);
  t.nf = (k + 1) * (k + 2) / 2;
  t.nb = (k + 2) * (k + 3) / 2;
  t.nned = k * (k + 2) * (k + 3) / 2;
  const int ns = t.ns, np = t.np, nf = t.nf, nb = t.nb;
  const OrthoSimplexBasis bu(k + 1, 3), bp(k, 3), bmu(k, 2, 2.0), bnu(k + 1, 2, 2.0);
  const Rule rc = simplex_rule((3 * k + 4) / 2, 3);  // ceil((3k+3)/2)
  const Rule rf = simplex_rule((3 * k + 5) / 2, 2);  // ceil((3k+4)/2)
  t.nqc = (int)rc.w.size();
  t.nqf = (int)rf.w.size();
  const int nqc = t.nqc, nqf = t.nqf;
  t.cq_x = rc.x; t.cq_y = rc.y; t.cq_z = rc.z; t.cq_w = rc.w;
  t.fq_s = rf.x; t.fq_t = rf.y; t.fq_w = rf.w;

  std::vector<double> v(ns), gx(ns), gy(ns), gz(ns), vp(np), px(np), py(np), pz(np);
  t.Bu.assign((size_t)nqc * ns, 0.0);
  t.dBu.assign((size_t)3 * nqc * ns, 0.0);
  t.Bp.assign((size_t)nqc * np, 0.0);
  t.dBp.assign((size_t)3 * nqc * np, 0.0);
  for (int q = 0; q < nqc; ++q) {
    bu.eval(rc.x[q], rc.y[q], rc.z[q], v.data(), gx.data(), gy.data(), gz.data());
    bp.eval(rc.x[q], rc.y[q], rc.z[q], vp.data(), px.data(), py.data(), pz.data());
    for (int s = 0; s < ns; ++s) {
      t.Bu[(size_t)q * ns + s] = v[s];
      t.dBu[((size_t)0 * nqc + q) * ns + s] = gx[s];
      t.dBu[((size_t)1 * nqc + q) * ns + s] = gy[s];
      t.dBu[((size_t)2 * nqc + q) * ns + s] = gz[s];
    }
    for (int s = 0; s < np; ++s) {
      t.Bp[(size_t)q * np + s] = vp[s];
      t.dBp[((size_t)0 * nqc + q) * np + s] = px[s];
      t.dBp[((size_t)1 * nqc + q) * np + s] = py[s];
      t.dBp[((size_t)2 * nqc + q) * np + s] = pz[s];
    }
  }
  // facet tables per (local facet, orientation)
  t.FBu.assign((size_t)24 * nqf * ns, 0.0);
  t.FdBu.assign((size_t)24 * 3 * nqf * ns, 0.0);
  t.FBp.assign((size_t)24 * nqf * np, 0.0);
  t.NUL.assign((size_t)24 * nqf * nb, 0.0);
  std::vector<double> nuv(nb), muv(nf);
  for (int f = 0; f < 4; ++f)
    for (int p = 0; p < 6; ++p) {
      const int fp = f * 6 + p;
      for (int q = 0; q < nqf; ++q) {
        double xi[3];
        facet_point3(f, p, rf.x[q], rf.y[q], xi);
        bu.eval(xi[0], xi[1], xi[2], v.data(), gx.data(), gy.data(), gz.data());
        bp.eval(xi[0], xi[1], xi[2], vp.data(), nullptr, nullptr, nullptr);
        for (int s = 0; s < ns; ++s) {
          t.FBu[((size_t)fp * nqf + q) * ns + s] = v[s];
          t.FdBu[(((size_t)fp * 3 + 0) * nqf + q) * ns + s] = gx[s];
          t.FdBu[(((size_t)fp * 3 + 1) * nqf + q) * ns + s] = gy[s];
          t.FdBu[(((size_t)fp * 3 + 2) * nqf + q) * ns + s] = gz[s];
        }
        for (int s = 0; s < np; ++s) t.FBp[((size_t)fp * nqf + q) * np + s] = vp[s];
        double sl, tl;
        local_facet_coords(p, rf.x[q], rf.y[q], sl, tl);
        bnu.eval(sl, tl, 0.0, nuv.data(), nullptr, nullptr, nullptr);
        for (int m = 0; m < nb; ++m) t.NUL[((size_t)fp * nqf + q) * nb + m] = nuv[m];
      }
    }
  t.MU.assign((size_t)nqf * nf, 0.0);
  for (int q = 0; q < nqf; ++q) {
    bmu.eval(rf.x[q], rf.y[q], 0.0, muv.data(), nullptr, nullptr, nullptr);
    for (int m = 0; m < nf; ++m) t.MU[(size_t)q * nf + m] = muv[m];
  }
  // volume matrices
  t.D.assign((size_t)3 * np * ns, 0.0);
  t.R.assign((size_t)3 * np * ns, 0.0);
  for (int a = 0; a < 3; ++a)
    for (int q = 0; q < nqc; ++q)
      for (int i = 0; i < np; ++i)
        for (int s = 0; s < ns; ++s) {
          const double w = rc.w[q];
          t.D[((size_t)a * np + i) * ns + s] += w * t.Bp[(size_t)q * np + i] * t.dBu[((size_t)a * nqc + q) * ns + s];
          t.R[((size_t)a * np + i) * ns + s] += w * t.dBp[((size_t)a * nqc + q) * np + i] * t.Bu[(size_t)q * ns + s];
        }
  t.KDD.assign((size_t)9 * np * np, 0.0);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int i = 0; i < np; ++i)
        for (int j = 0; j < np; ++j) {
          double acc = 0.0;
          for (int s = 0; s < ns; ++s) acc += t.D[((size_t)a * np + i) * ns + s] * t.D[((size_t)b * np + j) * ns + s];
          t.KDD[(((size_t)a * 3 + b) * np + i) * np + j] = acc;
        }
  // facet matrices (twice the reference triangle's measure: a facet of area
  // |F| scales them by |F|)
  t.That.assign((size_t)4 * np * np, 0.0);
  t.Chat.assign((size_t)24 * nf * ns, 0.0);
  t.Ehat.assign((size_t)24 * nf * np, 0.0);
  for (int f = 0; f < 4; ++f)
    for (int p = 0; p < 6; ++p) {
      const int fp = f * 6 + p;
      for (int q = 0; q < nqf; ++q) {
        const double w = 2.0 * rf.w[q];
        for (int m = 0; m < nf; ++m) {
          const double mu = t.MU[(size_t)q * nf + m];
          for (int s = 0; s < ns; ++s) t.Chat[((size_t)fp * nf + m) * ns + s] += w * mu * t.FBu[((size_t)fp * nqf + q) * ns + s];
          for (int i = 0; i < np; ++i) t.Ehat[((size_t)fp * nf + m) * np + i] += w * mu * t.FBp[((size_t)fp * nqf + q) * np + i];
        }
        if (p == 0)
          for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j)
              t.That[((size_t)f * np + i) * np + j] +=
                  w * t.FBp[((size_t)fp * nqf + q) * np + i] * t.FBp[((size_t)fp * nqf + q) * np + j];
      }
    }
  t.CD.assign((size_t)24 * 3 * nf * np, 0.0);
  for (int fp = 0; fp < 24; ++fp)
    for (int a = 0; a < 3; ++a)
      for (int m = 0; m < nf; ++m)
        for (int j = 0; j < np; ++j) {
          double acc = 0.0;
          for (int s = 0; s < ns; ++s)
            acc += t.Chat[((size_t)fp * nf + m) * ns + s] * t.D[((size_t)a * np + j) * ns + s];
          t.CD[(((size_t)fp * 3 + a) * nf + m) * np + j] = acc;
        }
  // reference Nedelec (first kind, degree k): [P_{k-1}]^3 and xi x (m e_j)
  // for homogeneous monomials m of degree k-1, j = 0, 1, and j = 2 for m
  // free of zeta (the others are combinations: xi x (xi q) = 0)
  auto ned = [&](double x, double y, double z, std::vector<std::array<double, 3>>& out) {
    out.clear();
    const double X[3] = {x, y, z};
    for (int deg = 0; deg < k; ++deg)
      for (int a = deg; a >= 0; --a)
        for (int b = deg - a; b >= 0; --b) {
          const int c = deg - a - b;
          const double mv = ipow(x, a) * ipow(y, b) * ipow(z, c);
          for (int comp = 0; comp < 3; ++comp) {
            std::array<double, 3> u{0.0, 0.0, 0.0};
            u[comp] = mv;
            out.push_back(u);
          }
        }
    for (int a = k - 1; a >= 0; --a)
      for (int b = k - 1 - a; b >= 0; --b) {
        const int c = k - 1 - a - b;
        const double mv = ipow(x, a) * ipow(y, b) * ipow(z, c);
        for (int j = 0; j < 3; ++j) {
          if (j == 2 && c > 0) continue;
          double e[3] = {0.0, 0.0, 0.0};
          e[j] = mv;
          out.push_back({X[1] * e[2] - X[2] * e[1], X[2] * e[0] - X[0] * e[2], X[0] * e[1] - X[1] * e[0]});
        }
      }
  };
  const int nu = 3 * ns;
  t.NEDM.assign((size_t)t.nned * 3 * ns, 0.0);
  std::vector<std::array<double, 3>> nv;
  for (int q = 0; q < nqc; ++q) {
    ned(rc.x[q], rc.y[q], rc.z[q], nv);
    if ((int)nv.size() != t.nned) throw std::runtime_error("Nedelec basis size");
    for (int l = 0; l < t.nned; ++l)
      for (int b = 0; b < 3; ++b)
        for (int s = 0; s < ns; ++s) t.NEDM[((size_t)l * 3 + b) * ns + s] += rc.w[q] * nv[l][b] * t.Bu[(size_t)q * ns + s];
  }
  // reference BDM moment matrix: normal moments against P_{k+1} of each
  // local facet (cell orientation, perm 0), then the interior moments;
  // columns are the velocity coefficients (component-major)
  const double sq3 = std::sqrt(3.0);
  const double rn[4][3] = {{1.0 / sq3, 1.0 / sq3, 1.0 / sq3}, {-1.0, 0.0, 0.0}, {0.0, -1.0, 0.0}, {0.0, 0.0, -1.0}};
  const double rarea[4] = {0.5 * sq3, 0.5, 0.5, 0.5};
  std::vector<double> A((size_t)nu * nu, 0.0);
  for (int f = 0; f < 4; ++f) {
    const int fp = f * 6;
    for (int m = 0; m < nb; ++m)
      for (int q = 0; q < nqf; ++q) {
        const double w = 2.0 * rarea[f] * rf.w[q] * t.NUL[((size_t)fp * nqf + q) * nb + m];
        for (int b = 0; b < 3; ++b)
          for (int s = 0; s < ns; ++s)
            A[((size_t)f * nb + m) * nu + b * ns + s] += w * rn[f][b] * t.FBu[((size_t)fp * nqf + q) * ns + s];
      }
  }
  for (int l = 0; l < t.nned; ++l)
    for (int b = 0; b < 3; ++b)
      for (int s = 0; s < ns; ++s) A[((size_t)4 * nb + l) * nu + b * ns + s] = t.NEDM[((size_t)l * 3 + b) * ns + s];
  std::vector<double> inv;
  invert_dense(nu, A, inv);
  // stored transposed: lane i of a wave forms row i of the product, so
  // column-major storage makes the wave's loads of one column contiguous
  t.BDMinv.assign((size_t)nu * nu, 0.0);
  for (int i = 0; i < nu; ++i)
    for (int j = 0; j < nu; ++j) t.BDMinv[(size_t)j * nu + i] = inv[(size_t)i * nu + j];
}

// ------------------------------------------------------------------ mesh
std::string build_mesh3(int64_t nv, const double* coords, int64_t nc, const int32_t* cells, HostMesh& m) {
  if (nv < 4 || nc < 1 || !coords || !cells) return "empty mesh";
  if (nv > INT32_MAX / 2 || nc > INT32_MAX / 8) return "mesh too large for 32-bit indices";
  m.dim = 3;
  m.nfc = 4;
  m.nv = nv;
  m.nc = nc;
  m.nvt = nv;
  m.coords.assign(coords, coords + 3 * nv);
  m.cells.assign(cells, cells + 4 * nc);
  m.vtopo.resize(nv);
  for (int64_t v = 0; v < nv; ++v) m.vtopo[v] = (int32_t)v;
  for (int64_t i = 0; i < 4 * nc; ++i)
    if (cells[i] < 0 || cells[i] >= nv) return "cell vertex index out of range";
  struct Ent { int32_t v[3]; int32_t cell, f; };
  std::vector<Ent> ents(4 * nc);
  m.cf_flip.assign(4 * nc, 0);
  for (int64_t K = 0; K < nc; ++K)
    for (int f = 0; f < 4; ++f) {
      int32_t g[3];
      for (int i = 0; i < 3; ++i) g[i] = cells[4 * K + LF3[f][i]];
      if (g[0] == g[1] || g[0] == g[2] || g[1] == g[2]) return "degenerate cell";
      // positions of lo, mid, hi among the local positions 0, 1, 2
      int pos[3] = {0, 1, 2};
      std::sort(pos, pos + 3, [&](int a, int b) { return g[a] < g[b]; });
      int perm = -1;
      for (int p = 0; p < 6; ++p)
        if (PERM3[p][0] == pos[0] && PERM3[p][1] == pos[1] && PERM3[p][2] == pos[2]) perm = p;
      m.cf_flip[f * nc + K] = perm;
      ents[4 * K + f] = {{g[pos[0]], g[pos[1]], g[pos[2]]}, (int32_t)K, f};
    }
  auto less = [](const Ent& x, const Ent& y) {
    for (int i = 0; i < 3; ++i)
      if (x.v[i] != y.v[i]) return x.v[i] < y.v[i];
    return x.cell < y.cell;
  };
  std::sort(ents.begin(), ents.end(), less);
  auto same = [](const Ent& x, const Ent& y) { return x.v[0] == y.v[0] && x.v[1] == y.v[1] && x.v[2] == y.v[2]; };
  m.cf_facet.assign(4 * nc, -1);
  m.cf_nb.assign(4 * nc, -1);
  m.cf_nbf.assign(4 * nc, -1);
  m.facet_lo.clear(); m.facet_mid.clear(); m.facet_hi.clear();
  std::vector<int32_t> fcp, fcm, ffp, ffm;
  for (size_t i = 0; i < ents.size();) {
    size_t j = i + 1;
    while (j < ents.size() && same(ents[j], ents[i])) ++j;
    if (j - i > 2) return "non-manifold facet";
    const int32_t F = (int32_t)m.facet_lo.size();
    m.facet_lo.push_back(ents[i].v[0]);
    m.facet_mid.push_back(ents[i].v[1]);
    m.facet_hi.push_back(ents[i].v[2]);
    fcp.push_back(ents[i].cell); ffp.push_back(ents[i].f);
    m.cf_facet[ents[i].f * nc + ents[i].cell] = F;
    if (j - i == 2) {
      fcm.push_back(ents[i + 1].cell); ffm.push_back(ents[i + 1].f);
      m.cf_facet[ents[i + 1].f * nc + ents[i + 1].cell] = F;
      m.cf_nb[ents[i].f * nc + ents[i].cell] = ents[i + 1].cell;
      m.cf_nbf[ents[i].f * nc + ents[i].cell] = ents[i + 1].f;
      m.cf_nb[ents[i + 1].f * nc + ents[i + 1].cell] = ents[i].cell;
      m.cf_nbf[ents[i + 1].f * nc + ents[i + 1].cell] = ents[i].f;
    } else {
      fcm.push_back(-1); ffm.push_back(0);
    }
    i = j;
  }
  m.nF = (int64_t)m.facet_lo.size();
  m.fc_cell.resize(2 * m.nF); m.fc_f.resize(2 * m.nF);
  for (int64_t F = 0; F < m.nF; ++F) {
    m.fc_cell[F] = fcp[F]; m.fc_cell[m.nF + F] = fcm[F];
    m.fc_f[F] = ffp[F]; m.fc_f[m.nF + F] = ffm[F];
  }
  m.geo.assign((size_t)kGeo3 * nc, 0.0);
  auto G = [&](int fld, int64_t K) -> double& { return m.geo[(size_t)fld * nc + K]; };
  for (int64_t K = 0; K < nc; ++K) {
    double X[4][3];
    for (int i = 0; i < 4; ++i)
      for (int a = 0; a < 3; ++a) X[i][a] = coords[3 * cells[4 * K + i] + a];
    double J[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) J[a][b] = X[b + 1][a] - X[0][a];
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    if (!(det > 0.0)) return "cell " + std::to_string(K) + " is not positively oriented (det J <= 0)";
    double iJ[3][3];
    iJ[0][0] = c00 / det;
    iJ[1][0] = c01 / det;
    iJ[2][0] = c02 / det;
    iJ[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    iJ[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    iJ[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    iJ[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    iJ[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    iJ[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    G(E_DET, K) = det;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        G(E_IJ + 3 * a + b, K) = iJ[a][b];
        G(E_J + 3 * a + b, K) = J[a][b];
      }
    for (int f = 0; f < 4; ++f) {
      const double* A = X[LF3[f][0]];
      const double* B = X[LF3[f][1]];
      const double* C = X[LF3[f][2]];
      double u[3], w[3], nrm[3];
      for (int a = 0; a < 3; ++a) { u[a] = B[a] - A[a]; w[a] = C[a] - A[a]; }
      nrm[0] = u[1] * w[2] - u[2] * w[1];
      nrm[1] = u[2] * w[0] - u[0] * w[2];
      nrm[2] = u[0] * w[1] - u[1] * w[0];
      const double len = std::sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
      double out = 0.0;
      for (int a = 0; a < 3; ++a) out += nrm[a] * (A[a] - X[f][a]);
      const double sg = out < 0.0 ? -1.0 : 1.0;
      for (int a = 0; a < 3; ++a) G(E_N + 3 * f + a, K) = sg * nrm[a] / len;
      G(E_A + f, K) = 0.5 * len;
    }
  }
  for (int64_t F = 0; F < m.nF; ++F) {
    const int32_t Km = m.fc_cell[m.nF + F];
    if (Km < 0) continue;
    const double ap = G(E_A + m.fc_f[F], m.fc_cell[F]), am = G(E_A + m.fc_f[m.nF + F], Km);
    if (std::fabs(ap - am) > 1e-12 * ap) return "the two sides of facet " + std::to_string(F) + " differ in area";
  }
  return "";
}

void mesh_unit_cube(int n, double* coords, int32_t* cells) {
  const int64_t m = n + 1;
  for (int64_t l = 0; l < m; ++l)
    for (int64_t j = 0; j < m; ++j)
      for (int64_t i = 0; i < m; ++i) {
        const int64_t v = (l * m + j) * m + i;
        coords[3 * v + 0] = (double)i / n;
        coords[3 * v + 1] = (double)j / n;
        coords[3 * v + 2] = (double)l / n;
      }
  // the six permutations of the axes in lexicographic order
  static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int64_t l = 0; l < n; ++l)
    for (int64_t j = 0; j < n; ++j)
      for (int64_t i = 0; i < n; ++i) {
        const int64_t cube = (l * n + j) * n + i;
        for (int r = 0; r < 6; ++r) {
          int64_t p[3] = {i, j, l};
          int32_t* c = cells + 4 * (6 * cube + r);
          c[0] = (int32_t)((p[2] * m + p[1]) * m + p[0]);
          for (int s = 0; s < 3; ++s) {
            p[perms[r][s]] += 1;
            c[s + 1] = (int32_t)((p[2] * m + p[1]) * m + p[0]);
          }
          // a path simplex is positively oriented for an even permutation
          int inv = 0;
          for (int a = 0; a < 3; ++a)
            for (int b = a + 1; b < 3; ++b) inv += perms[r][a] > perms[r][b];
          if (inv % 2) std::swap(c[2], c[3]);
        }
      }
}

}  // namespace hdg
