// Internal declarations of the HDG-IMEX library (host side).  Not part of
// the public C ABI; see include/hdg.h for that.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

namespace hdg {

constexpr int kMaxDegree = 4;  // pressure/trace degree k supported by the kernels

// ---------------------------------------------------------------- reference
// Gauss rule on [-1, 1] for the weight (1-x)^alpha (1+x)^beta (Golub-Welsch).
void gauss_jacobi(int n, double alpha, double beta, std::vector<double>& x, std::vector<double>& w);

// Jacobi polynomial P_n^{(a,b)}(x) and its derivative.
double jacobi_p(int n, double a, double b, double x);
double jacobi_dp(int n, double a, double b, double x);

int dim_p(int m);  // (m+1)(m+2)/2

// Orthonormal Dubiner basis of degree m on {xi, eta >= 0, xi + eta <= 1}:
// values and xi/eta derivatives at one point, written to v[dim_p(m)] etc.
void dubiner_eval(int m, double xi, double eta, double* v, double* dxi, double* deta);

// Orthonormal Legendre basis on [0, 1]: mu_i(t) = sqrt(2i+1) P_i(2t-1).
double legendre01(int i, double t);

// Reference tables for one degree k.  All matrices are row-major.
struct RefTables {
  int k, ns, np, nf, nqc, nqf, nned;
  std::vector<double> cq_xi, cq_eta, cq_w;       // cell rule (nqc), weights sum to 1/2
  std::vector<double> fq_s, fq_w;                // facet rule on [0,1] (nqf), weights sum to 1
  std::vector<double> Bu, Gux, Guy;              // [nqc][ns]  velocity-degree basis at cell points
  std::vector<double> Bp, Gpx, Gpy;              // [nqc][np]
  std::vector<double> FBu, FGux, FGuy;           // [3][nqf][ns] at local facet points
  std::vector<double> FBp;                       // [3][nqf][np]
  std::vector<double> MU;                        // [nqf][nf]   trace basis at s_q (local parameter)
  std::vector<double> NUB;                       // [nqf][k+2]  BDM facet-moment basis
  std::vector<double> TRU;                       // [3][k+2][ns] Legendre coefficients of the trace on facet f
  // reference matrices
  std::vector<double> Dx, Dy;                    // [np][ns]  int psi_i d_a phi_s
  std::vector<double> Rx, Ry;                    // [np][ns]  int d_a psi_i phi_s
  std::vector<double> Chat;                      // [3][nf][ns] int_0^1 mu_m phi_s(x_f(s)) ds
  std::vector<double> That;                      // [3][np][np]
  std::vector<double> Ehat;                      // [3][nf][np]
  std::vector<double> CC;                        // [3][3][nf][nf]  Chat_f Chat_g^T
  std::vector<double> KDD;                       // [2][2][np][np]  D_a D_b^T
  std::vector<double> CD;                        // [3][2][nf][np]  Chat_f D_a^T
  std::vector<double> BDMinv;                    // [2ns][2ns] inverse of the reference BDM moment matrix
  std::vector<double> NED;                       // [nqc][nned][2] reference Nedelec basis at cell points
};

void build_reference(int k, RefTables& t);

// local facet f runs from local vertex FA[f] to FB[f]
constexpr int FA[3] = {1, 0, 0};
constexpr int FB[3] = {2, 2, 1};
inline void facet_point(int f, double s, double& xi, double& eta) {
  if (f == 0) { xi = 1.0 - s; eta = s; }
  else if (f == 1) { xi = 0.0; eta = s; }
  else { xi = s; eta = 0.0; }
}

// ------------------------------------------------------- tetrahedra (d = 3)
constexpr int kMaxDegree3 = 2;  // pressure/trace degree k supported on tetrahedra
// local facet f: the triangle opposite local vertex f, local vertices ascending
constexpr int LF3[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
// orientation p of a local facet: the local positions (into LF3[f]) of the
// facet's lowest, middle and highest global vertex
constexpr int PERM3[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
int dim_p3(int m);  // (m+1)(m+2)(m+3)/6
// reference coordinates of the point (s, t) of local facet f seen in orientation p
void facet_point3(int f, int p, double s, double t, double* xi);

// Orthonormal basis of P_m on the reference triangle (d = 2) or tetrahedron
// (d = 3): the centred monomials ((d+1)x - 1)^a ... by degree, then in
// descending lexicographic order of the exponents, Gram-Schmidt
// orthonormalised for `scale` times the reference measure.
struct OrthoSimplexBasis {
  int m, d, n;
  std::vector<std::array<int, 3>> exps;
  std::vector<double> coef;  // [n][n]: function j = sum_l coef[j][l] monomial l
  OrthoSimplexBasis(int m, int d, double scale = 1.0);
  void eval_monomials(double x, double y, double z, double* v, double (*dv)[3]) const;
  void eval(double x, double y, double z, double* v, double* dx, double* dy, double* dz) const;
};

// Reference tables for one degree k on tetrahedra (row-major).  Facet tables
// are indexed by fp = 6 f + p (local facet f, orientation p) and evaluated at
// the facet rule's points in the facet's own coordinates (s, t).
struct RefTables3 {
  int k, ns, np, nf, nb, nned, nqc, nqf;
  std::vector<double> cq_x, cq_y, cq_z, cq_w;    // cell rule, weights sum to 1/6
  std::vector<double> fq_s, fq_t, fq_w;          // facet rule, weights sum to 1/2
  std::vector<double> Bu, dBu;                   // [nqc][ns], [3][nqc][ns]
  std::vector<double> Bp, dBp;                   // [nqc][np], [3][nqc][np]
  std::vector<double> FBu, FdBu, FBp;            // [24][nqf][ns], [24][3][nqf][ns], [24][nqf][np]
  std::vector<double> MU;                        // [nqf][nf] trace basis
  std::vector<double> NUL;                       // [24][nqf][nb] BDM facet-moment basis, cell orientation
  std::vector<double> D, R;                      // [3][np][ns]: int psi d_a phi, int d_a psi phi
  std::vector<double> KDD;                       // [3][3][np][np] = D_a D_b^T
  std::vector<double> That;                      // [4][np][np]  2 sum_q w psi psi on facet f
  std::vector<double> Chat, Ehat;                // [24][nf][ns], [24][nf][np]
  std::vector<double> CD;                        // [24][3][nf][np] = Chat D_a^T
  std::vector<double> NEDM;                      // [nned][3][ns] interior moments of the reference Nedelec basis
  std::vector<double> BDMinv;                    // [3ns][3ns] inverse of the reference BDM moment matrix, column-major
};
void build_reference3(int k, RefTables3& t);

// per-cell geometry of a tetrahedron, field-major [field][cell]
enum GeoField3 { E_DET = 0, E_IJ = 1, E_J = 10, E_N = 19, E_A = 31, kGeo3 = 35 };

// ------------------------------------------------------------------- mesh
struct HostMesh {
  int dim = 2, nfc = 3;             // spatial dimension, facets per cell
  int64_t nv = 0, nc = 0, nF = 0;
  int64_t nvt = 0;                  // topological vertices (classes of identified vertices)
  std::vector<int32_t> vtopo;       // [nv] topological id of each vertex
  std::vector<double> coords;       // [nv][2]
  std::vector<int32_t> cells;       // [nc][3]
  std::vector<int32_t> facet_lo, facet_hi;
  std::vector<int32_t> facet_mid;   // tetrahedra: the middle vertex of each facet
  std::vector<int32_t> cf_facet;    // [3][nc]
  std::vector<int32_t> cf_nb;       // [3][nc]  neighbour cell or -1
  std::vector<int32_t> cf_nbf;      // [3][nc]  neighbour's local facet
  std::vector<int32_t> cf_flip;     // [3][nc]  1 if the local parameter runs hi->lo
                                    // (tetrahedra: [4][nc] orientation p of the facet)
  std::vector<int32_t> fc_cell;     // [2][nF]  K+, K- (-1 on the boundary)
  std::vector<int32_t> fc_f;        // [2][nF]
  std::vector<double> geo;          // [kGeo][nc]
};
enum GeoField { G_DET = 0, G_IJ00, G_IJ01, G_IJ10, G_IJ11, G_NX0, G_NY0, G_NX1, G_NY1, G_NX2, G_NY2,
                G_H0, G_H1, G_H2, G_J00, G_J01, G_J10, G_J11, kGeo };

// tetrahedral mesh (coords [nv][3], cells [nc][4], positively oriented)
std::string build_mesh3(int64_t nv, const double* coords, int64_t nc, const int32_t* cells, HostMesh& m);
// Kuhn split of the unit cube: coords [(n+1)^3][3], cells [6 n^3][4]
void mesh_unit_cube(int n, double* coords, int32_t* cells);

// returns empty string on success, else an error message
std::string build_mesh(int64_t nv, const double* coords, int64_t nc, const int32_t* cells,
                       const int32_t* vertex_rep, HostMesh& m);

// ------------------------------------------------------------ AMG (host)
struct Csr {
  int64_t nrows = 0, ncols = 0;
  std::vector<int32_t> ptr, idx;
  std::vector<double> val;
};
struct AmgLevel {
  Csr A, P, R;
  std::vector<double> dinv;
  double omega = 0.0;
};
struct AmgHierarchy {
  std::vector<AmgLevel> levels;     // level l: A_l, P_l (l -> l+1 prolongation), R_l = P_l^T
  int64_t ncoarse = 0;
  std::vector<double> coarse_pinv;  // dense pseudo-inverse of the coarsest operator
};
void amg_setup(const Csr& A, AmgHierarchy& h, int64_t coarsest = 200, bool smooth = true);
Csr csr_transpose(const Csr& A);
Csr csr_multiply(const Csr& A, const Csr& B);

}  // namespace hdg
