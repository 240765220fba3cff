// Internal declarations of the HDG-IMEX library (host side).  Not part of
// the public C ABI; see include/hdg.h for that.
#pragma once

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

// ------------------------------------------------------------------- mesh
struct HostMesh {
  int64_t nv = 0, nc = 0, nF = 0;
  int64_t nvt = 0;                  // topological vertices (classes of identified vertices)
  std::vector<int32_t> vtopo;       // [nv] topological id of each vertex
  std::vector<double> coords;       // [nv][2]
  std::vector<int32_t> cells;       // [nc][3]
  std::vector<int32_t> facet_lo, facet_hi;
  std::vector<int32_t> cf_facet;    // [3][nc]
  std::vector<int32_t> cf_nb;       // [3][nc]  neighbour cell or -1
  std::vector<int32_t> cf_nbf;      // [3][nc]  neighbour's local facet
  std::vector<int32_t> cf_flip;     // [3][nc]  1 if the local parameter runs hi->lo
  std::vector<int32_t> fc_cell;     // [2][nF]  K+, K- (-1 on the boundary)
  std::vector<int32_t> fc_f;        // [2][nF]
  std::vector<double> geo;          // [kGeo][nc]
};
enum GeoField { G_DET = 0, G_IJ00, G_IJ01, G_IJ10, G_IJ11, G_NX0, G_NY0, G_NX1, G_NY1, G_NX2, G_NY2,
                G_H0, G_H1, G_H2, G_J00, G_J01, G_J10, G_J11, kGeo };

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
void amg_setup(const Csr& A, AmgHierarchy& h, int64_t coarsest = 200);
Csr csr_transpose(const Csr& A);
Csr csr_multiply(const Csr& A, const Csr& B);

}  // namespace hdg
