// Device-side data views and kernel launchers of the HDG-IMEX library.
#pragma once

#include <hip/hip_runtime.h>

namespace hdg {

// per-cell geometry fields, stored field-major [field][cell]
enum DGeo { D_DET = 0, D_IJ00, D_IJ01, D_IJ10, D_IJ11, D_NX0, D_NY0, D_NX1, D_NY1, D_NX2, D_NY2,
            D_H0, D_H1, D_H2, D_J00, D_J01, D_J10, D_J11, kDGeo };

struct DMesh {
  int nc, nF;
  int dim;                 // 2: triangles; 3: tetrahedra (the launchers forward to launch3_*)
  const double* geo;       // [kDGeo][nc]
  const int* cf_facet;     // [3][nc]
  const int* cf_nb;        // [3][nc]
  const int* cf_nbf;       // [3][nc]
  const int* cf_flip;      // [3][nc]
  const int* cf_nbx;       // [3][nc] -1 on walls, else (nb << 3) | (nb's local facet << 1) | reversed
  const int* fc_cell;      // [2][nF]
  const int* fc_f;         // [2][nF]
};

// Tetrahedra (d = 3): per-cell geometry fields [field][cell] (det J, J^{-1}
// row-major, J row-major, the outward unit normals and areas of the four
// facets); the DMesh index arrays are [4][nc] and cf_flip holds each local
// facet's orientation p.
enum DGeo3 { E3_DET = 0, E3_IJ = 1, E3_J = 10, E3_N = 19, E3_A = 31, kDGeo3 = 35 };

// Reference tables on tetrahedra (global memory; facet tables are indexed by
// fp = 6 * local facet + orientation).
struct DTab3 {
  const double *Bu, *dBu, *Bp, *dBp, *cw;           // cell rule
  const double *FBu, *FdBu, *FBp, *fw, *MU, *NUL;   // facet rule
  const double *D, *R, *KDD, *That, *Chat, *Ehat, *CD, *NEDM, *BDMinv;
};

// Reference tables live in the constant address space: every wave reads the
// same entry at the same time, so the loads become scalar (s_load) loads.
typedef const __attribute__((address_space(4))) double* cdptr;
struct DTab {
  cdptr Bu, Gux, Guy, Bp, Gpx, Gpy, cw;
  cdptr FBu, FGux, FGuy, FBp, fw, MU, NUB, TRU;
  cdptr Dx, Dy, Rx, Ry, Chat, That, Ehat, CC, KDD, CD, BDMinv, NED;
  DTab3 t3;  // tetrahedra
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
// Grid of the BiCGStab vector kernels (k_bicg_s, k_bicg_xrp): every block
// finishes the inner products of the preceding operator launch itself, so
// fewer, fuller blocks read fewer partials in total; k_bicg_xrp leaves
// kVecBlocks partials of r.r.
constexpr int kVecBlocks = 512;

// Device scalars of one BiCGStab iteration (BS_STRIDE doubles per slot).
enum BiCGSlot {
  BS_RHO = 0,              // rho = rh.r of this iteration
  BS_RV, BS_ALPHA,         // after v = A p: rh.v, alpha
  BS_TS, BS_TT, BS_OMEGA,  // after t = A s: t.s, t.t, omega
  BS_BETA,                 // for the next direction
  BS_RR,                   // r.r after the updates (filled when the host checks)
  BS_FLAG,                 // 1 on a breakdown (zero divisor)
  BS_STRIDE = 16
};

// Trace-operator kernels are keyed by the facet block size and the number of
// blocks per row: tk = k on triangles (k+1, 5 blocks), tk = 10 + k on
// tetrahedra ((k+1)(k+2)/2, 7 blocks).
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
// scale * Gamma(psi, mu, Q, P, lam) as dual vectors: gpsi [nc][np] and gmu [nF][nf]
// (ycell: scratch of nc * 3 * nf doubles); P or lam may be null (zero)
void launch_gamma(int k, hipStream_t st, DMesh m, DTab t, double tau, double scale, const double* Q, const double* P,
                  const double* lam, double* gpsi, double* ycell, double* gmu);
void launch_prep_adv(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, double* adv);
// mode 0: out = x - (adt/det) f_im(x)          (mass-scaled Step I operator)
// mode 1: out = (r - det x + adt (f_im(x) + g(p, lam))) / det  (mass-scaled residual)
// mode 2: out = r - det x + adt (f_im(x) + g(p, lam))           (residual, dual vector)
void launch_apply(int k, hipStream_t st, int mode, DMesh m, DTab t, const double* adv, double alpha, double adt,
                  const double* x, const double* r, const double* p, const double* lam, double* out);
// Per-stage data of the Step I operator for advecting velocity Qs (AoS): the
// volume data V (FP32 when v32, else FP64) and the facet upwind weights beta
// (3*nq_facet entries, FP32 when b32, else FP64).  Triangles: V is the
// advecting field at the cell points (2*nq_cell entries per cell), both in
// tiles of 32 cells (arrays hold ceil(nc/32)*32 cells; entry j of cell e at
// ((e/32)*nj + j)*32 + e%32).  Tetrahedra: cell-major volume matrices
// [nc][ns][ns] and weights [nc][4][nq_facet].
void launch_step1_data(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, void* V, bool v32,
                       void* beta, bool b32);
// Launch shape of the Step I operator: threads per workgroup (64, 128 or
// 256; two threads per cell) and the workgroup-to-XCD order (1: each XCD
// takes a contiguous eighth of the cells, 0: hardware order).
struct Step1Launch {
  int block;
  int xcd;
};
// Step I operator on structure-of-arrays vectors (2 threads per cell):
// out = x - (adt/det) f_im(x), with partial sums (apply_soa_blocks(nc, block)
// per set): dot 0 none; dot 1 w.out; dot 2 out.x, out.out, w.x, w.out
// (dot 3: as dot 2 with the dots taken against sd instead of x: out.sd,
// out.out, w.sd, w.out; sd is ignored otherwise).  x32: FP32 vectors, beta
// and arithmetic (V FP32); else FP64 vectors, beta and arithmetic (V FP32
// when v32).  Inner products accumulate in FP64 either way.
void launch_apply_soa(int k, hipStream_t st, Step1Launch ln, int dot, DMesh m, DTab t, const void* V, bool v32,
                      const void* beta, double alpha, double adt, const void* x, const void* w, void* out,
                      double* part, const void* sd, bool x32);
int apply_soa_blocks(long nc, int block);
// BiCGStab pieces (slot sc of BS_STRIDE scalars):
//   v = A p: launch_apply_soa dot 1 with rh (np partials in part)
//   s = r - alpha v, alpha from those partials: launch_bicg_s
//   t = A s: launch_apply_soa dot 2 with rh (4 sets of np partials in part2)
//   x, r, p updates, omega and beta from part2, partials of r.r
//   (kVecBlocks of them) in part: launch_bicg_xrp
void launch_bicg_s(hipStream_t st, long n, int np, const double* part, double* sc, const void* r, const void* v,
                   void* s, bool x32);
void launch_bicg_xrp(hipStream_t st, long n, int np, const double* part2, double* sc, const void* s, const void* tv,
                     const void* v, const void* ph, const void* sh, void* x, void* r, void* p, double* part,
                     bool x32);
void launch_bicg_init(hipStream_t st, double* sc);  // zero a slot except BS_RHO
// Step I preconditioner: additive Schwarz over facet patches (two cells per
// interior facet) of the mass-scaled Step I operator, in Woodbury form (cell
// inverses and per-facet trace corrections).  launch_pc_build forms them for
// the Q* and adt of a stage (D: scratch of nc * nu * nu doubles; Binv:
// pc_entries(k, nc) FP16 entries); launch_pc_apply gives z = B r on
// structure-of-arrays vectors (X: scratch of pc_scratch(k, nc) entries of the vectors' type).
void launch_pc_build(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, double alpha,
                     double adt, double* D, void* Binv);
void launch_pc_apply(int k, hipStream_t st, DMesh m, const void* Binv, void* X, const void* r, void* z, bool x32);
long pc_entries(int k, long nc);
long pc_scratch(int k, long nc);
void launch_to_soa(int k, hipStream_t st, DMesh m, int inv_det, const double* x, void* y, bool x32);
void launch_to_aos(int k, hipStream_t st, DMesh m, const void* x, double* y, bool x32);
// Step I vectors in either type (x32: FP32): copy, fill, a x + b y, and FP64
// partials of a.b (b null: a.a) over kRedBlocks blocks for launch_finish
void launch_vcopy(hipStream_t st, long n, const void* x, void* y, bool x32);
void launch_vfill(hipStream_t st, long n, double v, void* y, bool x32);
void launch_vaxpby(hipStream_t st, long n, double a, const void* x, double b, void* y, bool x32);
void launch_vdot(hipStream_t st, long n, const void* a, const void* b, double* part, bool x32);
void launch_div(int k, hipStream_t st, DMesh m, DTab t, const double* F, double scale, double* out);
void launch_bdm(int k, hipStream_t st, DMesh m, DTab t, const double* Q, double* Qs);
// f_p data of the pressure reconstruction: (Q.grad)Q - fsc f, f at the cell
// and facet points (null: no forcing)
void launch_recon_rhs(int k, hipStream_t st, DMesh m, DTab t, const double* Q, const double* fcell,
                      const double* ffac, double fsc, double* out);
// forcing: dual vector of cell point values; wall data -<mu, n.f> of facet point values (interior 0 untouched)
void launch_point_dual(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* out);
void launch_wall_flux(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* out);
void launch_project(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* Q);
void launch_mass(int k, hipStream_t st, DMesh m, double s, const double* x, double* y);
void launch_shift_mean(int k, hipStream_t st, DMesh m, const double* mean, double* p, double* lam);

void launch_csr_spmv(hipStream_t st, DCsr A, const double* x, double* y, double beta);
void launch_csr_jacobi(hipStream_t st, DCsr A, const double* dinv, double omega, const double* b,
                       const double* xin, double* xout);
void launch_dense_mv(hipStream_t st, int n, const double* M, const double* x, double* y);

// reductions: partial sums into part[kRedBlocks], then out[0] = sum
void launch_dot(hipStream_t st, long n, const double* a, const double* b, double* part);
void launch_dot_sub(hipStream_t st, long n, int stride, int off, const double* a, double* part);
void launch_finish(hipStream_t st, const double* part, int nparts, double* out);
void launch_finish_mean(hipStream_t st, const double* part, int nparts, double area, double* out);

// vectors: y = a*x + b*y with host scalars
void launch_axpby(hipStream_t st, long n, double a, const double* x, double b, double* y);
void launch_copy(hipStream_t st, long n, const double* x, double* y);
void launch_fill(hipStream_t st, long n, double v, double* y);
void launch_project_const(hipStream_t st, int nF, int nf, const double* sum, double* g);
// facet-block-Jacobi PCG of a small trace system in one workgroup (one launch per solve);
// info[4]: iterations, squared projected residual, floor stop, converged
void launch_pcg_small(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* Dinv,
                      const double* g, double* x, double* r, double* z, double* p, double* q, int maxit, double tol2,
                      double floor2, int flat_blocks, double* info);
// passive tracer: CG_{k+1} projection pieces and the DG transport rate M^-1 a(., q, U)
void launch_cg_rhs(hipStream_t st, int N, const int* ptr, const int* inc, int ns, const double* T, DMesh m,
                   const double* Q, int comp, double* b);
void launch_cg_to_dg(hipStream_t st, long nc, int ns, const double* T, const int* l2g, const double* u, int comp,
                     double* U);
void launch_project_scalar(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* q);
void launch_tracer_rate(int k, hipStream_t st, DMesh m, DTab t, const double* U, const double* q, double* out);
// Qo[cell][pt][2], po[cell][pt] from the velocity / pressure bases at the points (either output may be null)
void launch_eval_points(hipStream_t st, long nc, int npts, int ns, int np, const double* BU, const double* BP,
                        const double* Q, const double* p, double* Qo, double* po);

// Krylov helpers with device scalars
void launch_pcg_update(hipStream_t st, long n, int nf, const double* rz, const double* pq, const double* p,
                       const double* q, double* x, double* r, double* part_rr);
// partials of r.r and sum r_0 over kRedBlocks blocks, the layout launch_pcg_update leaves
void launch_rr_partials(hipStream_t st, long n, int nf, const double* r, double* part);
// sum(part[0..n)) - sum(part[n..2n))^2 / nnull  (residual norm^2 without its null-vector part)
void launch_finish_proj(hipStream_t st, const double* part, int nparts, double nnull, double* out);
void launch_pcg_direction(hipStream_t st, long n, const double* rz_new, const double* rz_old, const double* z, double* p);
void launch_dot2(hipStream_t st, long n, const double* a, const double* b, const double* c, double* part2);
void launch_finish2(hipStream_t st, const double* part2, double* out2);
void launch_idr_u(hipStream_t st, long n, int k, int s, IdrCoef c, double om, const double* r, const double* G,
                  double* U);
void launch_multidot(hipStream_t st, long n, int s, const double* P, const double* g, double* part, double* out);
void launch_idr_update(hipStream_t st, long n, int k, IdrCoef a, double beta, double* G, double* U, double* r,
                       double* x, double* part);
void launch_idr_reduce(hipStream_t st, long n, double om, const double* t, double* r, double* x, double* part);
void launch_random(hipStream_t st, long n, unsigned long long seed, double* y);

// ------------------------------------------------------------ tetrahedra
// The same operations on tetrahedral meshes (k = 1, 2); vectors cell-major.
void launch3_condense(int k, hipStream_t st, DMesh m, DTab3 t, double c, double tau, double* Pinv, double* SK);
void launch3_assemble(int k, hipStream_t st, DMesh m, const double* SK, double* vals, int* cols, double* Dinv);
void launch3_rhs_condense(int k, hipStream_t st, DMesh m, DTab3 t, double c, double tau, const double* Pinv,
                          const double* Fw, const double* Fpsi, double* ycell);
// cellint: scratch of nc doubles; part: ceil(nc / kBlock) partial sums of int p
void launch3_backsub(int k, hipStream_t st, DMesh m, DTab3 t, double c, double tau, const double* Pinv,
                     const double* Fw, const double* Fpsi, const double* lam, double* U, double* p, double* cellint,
                     double* part);
void launch3_shift_mean(int k, hipStream_t st, DMesh m, const double* mean, double* p, double* lam);
// psi part into gpsi, mu part per (cell, local facet) into ycell (gathered by launch_gather_rhs)
void launch3_gamma(int k, hipStream_t st, DMesh m, DTab3 t, double tau, double scale, const double* Q, const double* P,
                   const double* lam, double* gpsi, double* ycell);
void launch3_mass(int k, hipStream_t st, DMesh m, double s, const double* x, double* y);
// per-stage Step I data: V [nc][ns][ns] (transposed: [cell][trial][test]), beta [nc][4][nq_facet]
// (f32: V and beta in FP32, the mixed-precision Step I data)
void launch3_prep(int k, hipStream_t st, DMesh m, DTab3 t, const double* Qs, double delta_up, void* V, void* beta,
                  bool f32);
// Step I operator (mode 0, with the dot variants of launch_apply_soa over
// nparts blocks) and residuals (modes 1, 2) as launch_apply describes them
// (x32: V, beta, x, w, sd, out and the arithmetic in FP32, mode 0 only)
void launch3_apply(int k, hipStream_t st, int mode, int dot, DMesh m, DTab3 t, const void* V, const void* beta,
                   double alpha, double adt, const void* x, const double* r, const double* p, const double* lam,
                   void* out, const void* w, const void* sd, double* part, int nparts, bool x32);
// out = in converted between FP64 and FP32 (n entries)
void launch3_convert(hipStream_t st, long n, const void* in, bool in32, void* out, bool out32);
void launch3_div(int k, hipStream_t st, DMesh m, DTab3 t, const double* F, double scale, double* out);
void launch3_bdm(int k, hipStream_t st, DMesh m, DTab3 t, const double* Q, double* Qs);
void launch3_recon_rhs(int k, hipStream_t st, DMesh m, DTab3 t, const double* Q, double* out);
// Step I preconditioner on tetrahedra (facet-patch additive Schwarz): built
// from the per-stage V and beta of launch3_prep (D: scratch of nc nu^2
// doubles; Binv: pc_entries3(k, nc) FP16 entries); z = B r on cell-major vectors
void launch3_pc_build(int k, hipStream_t st, DMesh m, DTab3 t, const double* V, const double* beta, double alpha,
                      double adt, double* D, void* Binv);
void launch3_pc_apply(int k, hipStream_t st, DMesh m, const void* Binv, const void* r, void* z, bool x32);
long pc_entries3(int k, long nc);
// velocity from values at the cell points [nc][nq_cell][3]
void launch3_project(int k, hipStream_t st, DMesh m, DTab3 t, const double* vals, double* Q);

}  // namespace hdg
