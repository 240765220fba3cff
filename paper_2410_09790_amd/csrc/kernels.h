// Device-side data views and kernel launchers of the HDG-IMEX library.
#pragma once

#include <hip/hip_runtime.h>

namespace hdg {

// per-cell geometry fields, stored field-major [field][cell]
enum DGeo { D_DET = 0, D_IJ00, D_IJ01, D_IJ10, D_IJ11, D_NX0, D_NY0, D_NX1, D_NY1, D_NX2, D_NY2,
            D_H0, D_H1, D_H2, D_J00, D_J01, D_J10, D_J11, kDGeo };

struct DMesh {
  int nc, nF;
  const double* geo;       // [kDGeo][nc]
  const int* cf_facet;     // [3][nc]
  const int* cf_nb;        // [3][nc]
  const int* cf_nbf;       // [3][nc]
  const int* cf_flip;      // [3][nc]
  const int* fc_cell;      // [2][nF]
  const int* fc_f;         // [2][nF]
};

// Reference tables live in the constant address space: every wave reads the
// same entry at the same time, so the loads become scalar (s_load) loads.
typedef const __attribute__((address_space(4))) double* cdptr;
struct DTab {
  cdptr Bu, Gux, Guy, Bp, Gpx, Gpy, cw;
  cdptr FBu, FGux, FGuy, FBp, fw, MU, NUB;
  cdptr Dx, Dy, Rx, Ry, Chat, That, Ehat, CC, KDD, CD, BDMinv, NED;
};

struct DCsr {
  int n;
  const int* ptr;
  const int* idx;
  const double* val;
};

constexpr int kBlock = 256;
constexpr int kIdrMax = 8;  // largest IDR(s) shadow-space dimension
struct IdrCoef {
  double v[kIdrMax];
};
constexpr int kRedBlocks = 1024;  // fixed grid for deterministic reductions

// launchers (k = degree); all enqueue on `st`
void launch_condense(int k, hipStream_t st, DMesh m, DTab t, double c, double tau, double* Pinv, double* SK);
void launch_assemble(int k, hipStream_t st, DMesh m, const double* SK, double* vals, int* cols, double* Dinv);
void launch_spmv(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* x, double* y);
void launch_residual(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* b,
                     const double* x, double* r);
void launch_jacobi_sweep(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* Dinv,
                         double omega, const double* b, const double* xin, double* xout);
void launch_blockdiag(int k, hipStream_t st, int nF, const double* Dinv, const double* x, double* y);
void launch_rhs_condense(int k, hipStream_t st, DMesh m, DTab t, double c, double tau, const double* Pinv,
                         const double* Fw, const double* Fpsi, double* ycell);
void launch_gather_rhs(int k, hipStream_t st, DMesh m, const double* ycell, const double* Fmu, double* g);
void launch_backsub(int k, hipStream_t st, DMesh m, DTab t, double c, double tau, const double* Pinv,
                    const double* Fw, const double* Fpsi, const double* lam, double* U, double* p, double* part);
void launch_prep_adv(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, double* adv);
// mode 0: out = x - (adt/det) f_im(x)          (mass-scaled Step I operator)
// mode 1: out = (r - det x + adt (f_im(x) + g(p, lam))) / det  (mass-scaled residual)
// mode 2: out = r - det x + adt (f_im(x) + g(p, lam))           (residual, dual vector)
void launch_apply(int k, hipStream_t st, int mode, DMesh m, DTab t, const double* adv, double alpha, double adt,
                  const double* x, const double* r, const double* p, const double* lam, double* out);
// Step I operator on structure-of-arrays vectors (2 threads per cell), with an
// optional fused reduction: dot 1 -> sum w.out; dot 2 -> sum out.x and sum out.out
// (second set of partials at part + apply_soa_blocks(nc))
template <typename TS, typename T>
void launch_apply_soa(int k, hipStream_t st, int dot, DMesh m, DTab t, const T* adv, double alpha, double adt,
                      const TS* x, const TS* w, TS* out, double* part);
int apply_soa_blocks(long nc);
template <typename T>
void launch_to_soa(int k, hipStream_t st, DMesh m, int inv_det, const double* x, T* y);
template <typename T>
void launch_to_aos(int k, hipStream_t st, DMesh m, const T* x, double* y);
void launch_div(int k, hipStream_t st, DMesh m, DTab t, const double* F, double scale, double* out);
void launch_bdm(int k, hipStream_t st, DMesh m, DTab t, const double* Q, double* Qs);
void launch_recon_rhs(int k, hipStream_t st, DMesh m, DTab t, const double* Q, double* out);
void launch_project(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* Q);
void launch_mass(int k, hipStream_t st, DMesh m, double s, const double* x, double* y);
void launch_shift_mean(int k, hipStream_t st, DMesh m, const double* mean, double* p, double* lam);

void launch_csr_spmv(hipStream_t st, DCsr A, const double* x, double* y, double beta);
void launch_csr_jacobi(hipStream_t st, DCsr A, const double* dinv, double omega, const double* b,
                       const double* xin, double* xout);
void launch_dense_mv(hipStream_t st, int n, const double* M, const double* x, double* y);

// reductions: partial sums into part[kRedBlocks], then out[0] = sum
void launch_dot(hipStream_t st, long n, const double* a, const double* b, double* part);
void launch_dot(hipStream_t st, long n, const float* a, const float* b, double* part);
void launch_dot_sub(hipStream_t st, long n, int stride, int off, const double* a, double* part);
void launch_finish(hipStream_t st, const double* part, int nparts, double* out);
void launch_finish_mean(hipStream_t st, const double* part, int nparts, double area, double* out);

// vectors: y = a*x + b*y with host scalars
void launch_axpby(hipStream_t st, long n, double a, const double* x, double b, double* y);
void launch_axpby(hipStream_t st, long n, double a, const float* x, double b, float* y);
void launch_copy(hipStream_t st, long n, const double* x, double* y);
void launch_copy(hipStream_t st, long n, const float* x, float* y);
void launch_fill(hipStream_t st, long n, double v, double* y);
void launch_fill(hipStream_t st, long n, double v, float* y);
void launch_convert(hipStream_t st, long n, const double* x, float* y);
void launch_project_const(hipStream_t st, int nF, int nf, const double* sum, double* g);

// Krylov helpers with device scalars
void launch_pcg_update(hipStream_t st, long n, const double* rz, const double* pq, const double* p, const double* q,
                       double* x, double* r, double* part_rr);
void launch_pcg_direction(hipStream_t st, long n, const double* rz_new, const double* rz_old, const double* z, double* p);
template <typename T>
void launch_bicg_p(hipStream_t st, long n, const double* sc, int it, const T* r, const T* v, T* p);
template <typename T>
void launch_bicg_s(hipStream_t st, long n, const double* sc, int it, const T* r, const T* v, T* s);
template <typename T>
void launch_bicg_xr(hipStream_t st, long n, const double* sc, int it, const T* p, const T* s, const T* t, T* x,
                    T* r, const T* rhat, double* part2);
void launch_dot2(hipStream_t st, long n, const double* a, const double* b, const double* c, double* part2);
void launch_finish2(hipStream_t st, const double* part2, double* out2);
void launch_finish_sets(hipStream_t st, const double* part, int np, int nsets, double* out);
void launch_idr_u(hipStream_t st, long n, int k, int s, IdrCoef c, double om, const double* r, const double* G,
                  double* U);
void launch_multidot(hipStream_t st, long n, int s, const double* P, const double* g, double* part, double* out);
void launch_idr_update(hipStream_t st, long n, int k, IdrCoef a, double beta, double* G, double* U, double* r,
                       double* x, double* part);
void launch_idr_reduce(hipStream_t st, long n, double om, const double* t, double* r, double* x, double* part);
void launch_random(hipStream_t st, long n, unsigned long long seed, double* y);

}  // namespace hdg
