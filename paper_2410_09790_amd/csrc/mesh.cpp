// Mesh topology, affine geometry and the algebraic multigrid setup for the
// P1 coarse space of the trace preconditioner.
//
// Facet numbering (part of the data layout): distinct vertex pairs (lo, hi),
// lo < hi, in lexicographic order; the trace parameter runs from lo to hi.
// On a periodic mesh the pairs are taken over classes of identified vertices
// (vertices with the same representative), numbered by the rank of the
// representative; geometry always uses each cell's own vertex coordinates.
// Local facet f of a cell is the edge opposite local vertex f, with local
// parameter running from local vertex FA[f] to FB[f].
//
// The coarse space of the non-nested multigrid (paper, Section "Solvers and
// preconditioners") is P1 on the same mesh.  Its operator is the Galerkin
// product P^T S P and is solved approximately by one smoothed-aggregation
// V-cycle (standard greedy aggregation, Jacobi-smoothed tentative
// prolongator, damped Jacobi smoothing, dense pseudo-inverse on the coarsest
// level); the paper uses PETSc's GAMG for this level.  On tetrahedra the
// tentative prolongator is used unsmoothed: smoothing it fills the Galerkin
// coarse operators of the three-dimensional P1 stencil far more than in 2D.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <string>

#include "hdg_impl.h"

namespace hdg {

std::string build_mesh(int64_t nv, const double* coords, int64_t nc, const int32_t* cells,
                       const int32_t* vertex_rep, HostMesh& m) {
  if (nv < 3 || nc < 1 || !coords || !cells) return "empty mesh";
  if (nv > INT32_MAX / 2 || nc > INT32_MAX / 4) return "mesh too large for 32-bit indices";
  m.nv = nv;
  m.nc = nc;
  m.coords.assign(coords, coords + 2 * nv);
  m.cells.assign(cells, cells + 3 * nc);
  for (int64_t i = 0; i < 3 * nc; ++i)
    if (cells[i] < 0 || cells[i] >= nv) return "cell vertex index out of range";
  // topological vertex ids: rank of each vertex's representative
  std::vector<int32_t> topo(nv);
  if (vertex_rep) {
    std::vector<int32_t> rank(nv, 0);
    for (int64_t v = 0; v < nv; ++v) {
      if (vertex_rep[v] < 0 || vertex_rep[v] >= nv) return "vertex_rep entry out of range";
      rank[vertex_rep[v]] = 1;
    }
    int32_t r = 0;
    for (int64_t v = 0; v < nv; ++v) {
      const int32_t used = rank[v];
      rank[v] = r;
      r += used;
    }
    for (int64_t v = 0; v < nv; ++v) topo[v] = rank[vertex_rep[v]];
    m.nvt = r;
  } else {
    std::iota(topo.begin(), topo.end(), 0);
    m.nvt = nv;
  }
  const int64_t nvt = m.nvt;
  m.vtopo = topo;
  struct Ent { int64_t key; int32_t cell, f; };
  std::vector<Ent> ents(3 * nc);
  m.cf_flip.assign(3 * nc, 0);
  for (int64_t K = 0; K < nc; ++K)
    for (int f = 0; f < 3; ++f) {
      int32_t a = topo[cells[3 * K + FA[f]]], b = topo[cells[3 * K + FB[f]]];
      if (a == b) return vertex_rep ? "a cell edge joins identified vertices" : "degenerate cell";
      int64_t lo = std::min(a, b), hi = std::max(a, b);
      ents[3 * K + f] = {lo * nvt + hi, (int32_t)K, f};
      m.cf_flip[f * nc + K] = a > b ? 1 : 0;
    }
  std::sort(ents.begin(), ents.end(), [](const Ent& x, const Ent& y) {
    return x.key < y.key || (x.key == y.key && x.cell < y.cell);
  });
  m.cf_facet.assign(3 * nc, -1);
  m.cf_nb.assign(3 * nc, -1);
  m.cf_nbf.assign(3 * nc, -1);
  m.facet_lo.clear(); m.facet_hi.clear(); m.fc_cell.clear(); m.fc_f.clear();
  std::vector<int32_t> fcp, fcm, ffp, ffm;
  for (size_t i = 0; i < ents.size();) {
    size_t j = i + 1;
    while (j < ents.size() && ents[j].key == ents[i].key) ++j;
    if (j - i > 2) return "non-manifold facet";
    int32_t F = (int32_t)m.facet_lo.size();
    m.facet_lo.push_back((int32_t)(ents[i].key / nvt));
    m.facet_hi.push_back((int32_t)(ents[i].key % nvt));
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
  m.geo.assign((size_t)kGeo * nc, 0.0);
  auto G = [&](int fld, int64_t K) -> double& { return m.geo[(size_t)fld * nc + K]; };
  for (int64_t K = 0; K < nc; ++K) {
    double x[3], y[3];
    for (int i = 0; i < 3; ++i) { x[i] = coords[2 * cells[3 * K + i]]; y[i] = coords[2 * cells[3 * K + i] + 1]; }
    double j00 = x[1] - x[0], j01 = x[2] - x[0], j10 = y[1] - y[0], j11 = y[2] - y[0];
    double det = j00 * j11 - j01 * j10;
    if (!(det > 0.0)) return "cell " + std::to_string(K) + " is not counter-clockwise (det J <= 0)";
    G(G_DET, K) = det;
    G(G_IJ00, K) = j11 / det; G(G_IJ01, K) = -j01 / det; G(G_IJ10, K) = -j10 / det; G(G_IJ11, K) = j00 / det;
    G(G_J00, K) = j00; G(G_J01, K) = j01; G(G_J10, K) = j10; G(G_J11, K) = j11;
    for (int f = 0; f < 3; ++f) {
      int a = FA[f], b = FB[f];
      double ex = x[b] - x[a], ey = y[b] - y[a], len = std::sqrt(ex * ex + ey * ey);
      double nx = ey / len, ny = -ex / len;
      if (nx * (x[a] - x[f]) + ny * (y[a] - y[f]) < 0) { nx = -nx; ny = -ny; }
      G(G_NX0 + 2 * f, K) = nx; G(G_NY0 + 2 * f, K) = ny; G(G_H0 + f, K) = len;
    }
  }
  // both sides of a facet (two placements of it on a periodic mesh) must match
  for (int64_t F = 0; F < m.nF; ++F) {
    const int32_t Km = m.fc_cell[m.nF + F];
    if (Km < 0) continue;
    const double hp = G(G_H0 + m.fc_f[F], m.fc_cell[F]), hm = G(G_H0 + m.fc_f[m.nF + F], Km);
    if (std::fabs(hp - hm) > 1e-12 * hp) return "the two sides of facet " + std::to_string(F) + " differ in length";
  }
  return "";
}

// ------------------------------------------------------------------ CSR
Csr csr_transpose(const Csr& A) {
  Csr T;
  T.nrows = A.ncols; T.ncols = A.nrows;
  T.ptr.assign(T.nrows + 1, 0);
  for (int32_t j : A.idx) T.ptr[j + 1]++;
  for (int64_t i = 0; i < T.nrows; ++i) T.ptr[i + 1] += T.ptr[i];
  T.idx.resize(A.idx.size()); T.val.resize(A.val.size());
  std::vector<int32_t> pos(T.ptr.begin(), T.ptr.end() - 1);
  for (int64_t i = 0; i < A.nrows; ++i)
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int32_t q = pos[A.idx[p]]++;
      T.idx[q] = (int32_t)i; T.val[q] = A.val[p];
    }
  return T;
}

Csr csr_multiply(const Csr& A, const Csr& B) {
  Csr C;
  C.nrows = A.nrows; C.ncols = B.ncols;
  C.ptr.assign(C.nrows + 1, 0);
  std::vector<int32_t> mark(B.ncols, -1);
  std::vector<double> acc(B.ncols, 0.0);
  std::vector<int32_t> cols;
  for (int64_t i = 0; i < A.nrows; ++i) {
    cols.clear();
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) {
      int32_t a = A.idx[p];
      double va = A.val[p];
      for (int32_t q = B.ptr[a]; q < B.ptr[a + 1]; ++q) {
        int32_t b = B.idx[q];
        if (mark[b] != (int32_t)i) { mark[b] = (int32_t)i; acc[b] = 0.0; cols.push_back(b); }
        acc[b] += va * B.val[q];
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t b : cols) { C.idx.push_back(b); C.val.push_back(acc[b]); }
    C.ptr[i + 1] = (int32_t)C.idx.size();
  }
  return C;
}

// ------------------------------------------------------------------ AMG
static std::vector<int32_t> aggregate(const Csr& A, int64_t& nagg) {
  const double theta = 0.08;
  int64_t n = A.nrows;
  std::vector<double> d(n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
      if (A.idx[p] == i) d[i] = std::fabs(A.val[p]);
  auto strong = [&](int64_t i, int32_t p) {
    int32_t j = A.idx[p];
    return j != i && std::fabs(A.val[p]) >= theta * std::sqrt(d[i] * d[j]);
  };
  std::vector<int32_t> agg(n, -1);
  nagg = 0;
  for (int64_t i = 0; i < n; ++i) {  // pass 1: seeds with a free neighbourhood
    if (agg[i] >= 0) continue;
    bool free_nb = true;
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1] && free_nb; ++p)
      if (strong(i, p) && agg[A.idx[p]] >= 0) free_nb = false;
    if (!free_nb) continue;
    agg[i] = (int32_t)nagg;
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
      if (strong(i, p)) agg[A.idx[p]] = (int32_t)nagg;
    ++nagg;
  }
  std::vector<int32_t> agg1 = agg;
  for (int64_t i = 0; i < n; ++i) {  // pass 2: join a neighbouring aggregate
    if (agg[i] >= 0) continue;
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
      if (strong(i, p) && agg1[A.idx[p]] >= 0) { agg[i] = agg1[A.idx[p]]; break; }
  }
  for (int64_t i = 0; i < n; ++i)  // pass 3: leftovers
    if (agg[i] < 0) agg[i] = (int32_t)nagg++;
  return agg;
}

static double spectral_radius_dinv_a(const Csr& A, const std::vector<double>& dinv) {
  int64_t n = A.nrows;
  std::vector<double> x(n), y(n);
  for (int64_t i = 0; i < n; ++i) x[i] = std::sin(0.37 * (double)i + 0.11) + 0.5 * std::cos(1.3 * (double)i);
  double rho = 1.0;
  for (int it = 0; it < 30; ++it) {
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      double acc = 0.0;
      for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) acc += A.val[p] * x[A.idx[p]];
      y[i] = dinv[i] * acc;
      nrm += y[i] * y[i];
    }
    nrm = std::sqrt(nrm);
    double xn = 0.0;
    for (double v : x) xn += v * v;
    rho = nrm / std::sqrt(xn);
    if (nrm == 0.0) break;
    for (int64_t i = 0; i < n; ++i) x[i] = y[i] / nrm;
  }
  return rho;
}

static void sym_pinv(int64_t n, const Csr& A, std::vector<double>& out) {
  std::vector<double> M(n * n, 0.0), V(n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p) M[i * n + A.idx[p]] = A.val[p];
  for (int64_t i = 0; i < n; ++i)  // symmetrise round-off
    for (int64_t j = i + 1; j < n; ++j) { double v = 0.5 * (M[i * n + j] + M[j * n + i]); M[i * n + j] = M[j * n + i] = v; }
  for (int64_t i = 0; i < n; ++i) V[i * n + i] = 1.0;
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int64_t p = 0; p < n; ++p) {
      diag += M[p * n + p] * M[p * n + p];
      for (int64_t q = p + 1; q < n; ++q) off += M[p * n + q] * M[p * n + q];
    }
    if (off <= 1e-30 * diag) break;
    for (int64_t p = 0; p < n; ++p)
      for (int64_t q = p + 1; q < n; ++q) {
        double apq = M[p * n + q];
        if (std::fabs(apq) < 1e-300) continue;
        double theta = (M[q * n + q] - M[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int64_t r = 0; r < n; ++r) {
          double a = M[r * n + p], b = M[r * n + q];
          M[r * n + p] = c * a - s * b; M[r * n + q] = s * a + c * b;
        }
        for (int64_t r = 0; r < n; ++r) {
          double a = M[p * n + r], b = M[q * n + r];
          M[p * n + r] = c * a - s * b; M[q * n + r] = s * a + c * b;
        }
        for (int64_t r = 0; r < n; ++r) {
          double a = V[r * n + p], b = V[r * n + q];
          V[r * n + p] = c * a - s * b; V[r * n + q] = s * a + c * b;
        }
      }
  }
  double lmax = 0.0;
  for (int64_t i = 0; i < n; ++i) lmax = std::max(lmax, std::fabs(M[i * n + i]));
  out.assign(n * n, 0.0);
  for (int64_t e = 0; e < n; ++e) {
    double lam = M[e * n + e];
    if (std::fabs(lam) <= 1e-10 * lmax) continue;  // drop the null space (constants)
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < n; ++j) out[i * n + j] += V[i * n + e] * V[j * n + e] / lam;
  }
}

void amg_setup(const Csr& A0, AmgHierarchy& h, int64_t coarsest, bool smooth) {
  h.levels.clear();
  Csr A = A0;
  while (A.nrows > coarsest) {
    AmgLevel L;
    L.A = A;
    int64_t n = A.nrows;
    L.dinv.assign(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
      for (int32_t p = A.ptr[i]; p < A.ptr[i + 1]; ++p)
        if (A.idx[p] == i && A.val[p] != 0.0) L.dinv[i] = 1.0 / A.val[p];
    double rho = spectral_radius_dinv_a(A, L.dinv);
    L.omega = 4.0 / (3.0 * rho);
    int64_t na = 0;
    std::vector<int32_t> agg = aggregate(A, na);
    if (na >= n) break;  // no coarsening possible
    std::vector<double> cnt(na, 0.0);
    for (int32_t a : agg) cnt[a] += 1.0;
    Csr T;
    T.nrows = n; T.ncols = na;
    T.ptr.resize(n + 1);
    for (int64_t i = 0; i <= n; ++i) T.ptr[i] = (int32_t)i;
    T.idx.assign(agg.begin(), agg.end());
    T.val.resize(n);
    for (int64_t i = 0; i < n; ++i) T.val[i] = 1.0 / std::sqrt(cnt[agg[i]]);
    Csr AT = smooth ? csr_multiply(A, T) : Csr{};  // P = T - omega D^{-1} A T (smooth), else P = T
    Csr P;
    P.nrows = n; P.ncols = na;
    P.ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < n && !smooth; ++i) {
      P.idx.push_back(agg[i]);
      P.val.push_back(T.val[i]);
      P.ptr[i + 1] = (int32_t)P.idx.size();
    }
    for (int64_t i = 0; i < n && smooth; ++i) {
      std::vector<std::pair<int32_t, double>> row;
      for (int32_t p = AT.ptr[i]; p < AT.ptr[i + 1]; ++p) row.push_back({AT.idx[p], -L.omega * L.dinv[i] * AT.val[p]});
      bool found = false;
      for (auto& e : row)
        if (e.first == agg[i]) { e.second += T.val[i]; found = true; }
      if (!found) row.push_back({agg[i], T.val[i]});
      std::sort(row.begin(), row.end());
      for (auto& e : row) { P.idx.push_back(e.first); P.val.push_back(e.second); }
      P.ptr[i + 1] = (int32_t)P.idx.size();
    }
    L.P = P;
    L.R = csr_transpose(P);
    A = csr_multiply(L.R, csr_multiply(A, P));
    h.levels.push_back(std::move(L));
  }
  h.ncoarse = A.nrows;
  sym_pinv(A.nrows, A, h.coarse_pinv);
}

}  // namespace hdg
