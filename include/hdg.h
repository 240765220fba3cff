/*
 * hdg.h - C ABI of the MI355X HDG-IMEX library (libhdg.so).
 *
 * The library advances the incompressible Euler equations with the
 * hybridised DG discretisation and IMEX Runge-Kutta time stepping of
 * Mueller, "A Higher-order Hybridisable Discontinuous Galerkin IMEX method
 * for the incompressible Euler equations" (arXiv:2410.09790):
 *   - problem: eqs. (incompressible_euler_momentum/constraint), n.Q = 0 on
 *     walls, or periodic identification (Section "Double-layer shear flow");
 *   - spaces: V_Q = [DG_{k+1}]^2, V_p = DG_k with int p = 0, V_trace = P_k on
 *     the facets (Section "Discontinuous Galerkin spaces", "Hybridisation");
 *   - one time step: Algorithm 1, each implicit stage solved by Algorithm 2
 *     (Chorin-split preconditioned Richardson iteration);
 *   - the hybridised mixed solve of Step II, of the final projection and of
 *     the pressure reconstruction: static condensation onto the trace,
 *     multigrid-preconditioned CG on the trace system, back-substitution
 *     (Section "Solvers and preconditioners").
 * Only two-dimensional triangle meshes are supported; the forcing f is zero
 * unless hdg_set_forcing supplies one.
 *
 * Data layout (all state and right-hand-side arrays):
 *   Q[cell][c*ns + s]  velocity, component c in {x, y}, ns = (k+2)(k+3)/2;
 *   p[cell][s]         pressure, s < (k+1)(k+2)/2;
 *   lam[facet][m]      trace, m < k+1.
 *   Cell basis: orthonormal Dubiner basis on the reference triangle
 *   {xi, eta >= 0, xi + eta <= 1}, mapped by x = v0 + (v1-v0) xi + (v2-v0) eta
 *   with (v0, v1, v2) the cell's vertices in the order given to hdg_create;
 *     phi_ij = sqrt(2(2i+1)(i+j+1)) P_i(a) ((1-b)/2)^i P_j^{(2i+1,0)}(b),
 *     r = 2xi-1, s = 2eta-1, a = 2(1+r)/(1-s)-1, b = s, ordered by total
 *     degree i+j, then by i ascending.
 *   Facets: the distinct vertex pairs (lo, hi), lo < hi, numbered in
 *   lexicographic order; facet basis mu_m(t) = sqrt(2m+1) P_m(2t-1) with t
 *   running from vertex lo (t=0) to vertex hi (t=1).  On a periodic mesh
 *   (hdg_create_periodic) lo and hi are topological vertex ids: the classes
 *   of identified vertices, numbered by the rank of their representative.
 *   A dual vector (a right-hand side F_w(w) = sum_i F_i w_i) uses the same
 *   index as the unknown it tests.
 *
 * Conventions:
 *   - Every compute entry point takes DEVICE pointers (e.g. the data_ptr() of
 *     a torch tensor on the context's device), enqueues its work on the
 *     context's HIP stream and returns after that work has completed.
 *   - Buffers passed in stay owned by the caller; the context owns every
 *     internal device allocation and frees it in hdg_destroy.
 *   - No exception crosses the ABI: every function returns an hdg_status;
 *     hdg_last_error() gives a message.  A context is used by one host
 *     thread at a time.
 */
#ifndef HDG_H
#define HDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HDG_OK = 0,
  HDG_ERR_INVALID_ARG = 1,   /* bad pointer, size or parameter */
  HDG_ERR_OUT_OF_MEMORY = 2, /* device allocation failed */
  HDG_ERR_DEVICE = 3,        /* a HIP call failed */
  HDG_ERR_NOT_CONVERGED = 4, /* a Krylov solve hit its iteration cap; the result is kept */
  HDG_ERR_BAD_STATE = 5,     /* e.g. hdg_advance before any state was set */
  HDG_ERR_UNSUPPORTED = 6    /* not available: degree > 4, k > 2 or forcing, tracer, periodic meshes on tetrahedra */
} hdg_status;

/* IMEX schemes (Appendix A): IMEX Euler as printed; ARS(2,2,2) and ARS(2,3,3)
 * of Ascher, Ruuth and Spiteri (cited, not printed); SSP3(4,3,3) as printed,
 * read through Algorithm 1 (stage 0 = Q^n, the unused first implicit column
 * dropped: s = 4, 3 implicit stages per step); SSP2(3,3,2) as printed with
 * an explicit stage 0 in front of its implicit first stage (s = 4, 3
 * implicit stages), since dropping its first implicit column would lose the
 * weight b^im_0 = 1/3. */
typedef enum {
  HDG_IMEX_EULER = 0,
  HDG_ARS222 = 1,
  HDG_ARS233 = 2,
  HDG_SSP2_332 = 3,
  HDG_SSP3_433 = 4
} hdg_imex_scheme;
typedef enum { HDG_TRACE_JACOBI_PCG = 0, HDG_TRACE_MG_PCG = 1 } hdg_trace_solver;
typedef enum { HDG_PRESSURE_RECONSTRUCT = 0, HDG_PRESSURE_FIRST_ORDER = 1 } hdg_pressure_update;
/* HDG_MIXED: the tentative-velocity solve (Algorithm 2, Step I) runs in
 * FP32: Krylov vectors, the per-stage volume data (the advecting field at the
 * cell points on triangles, the cell matrices on tetrahedra) and upwind
 * weights, and the operator's arithmetic; its inner products accumulate in FP64, and it
 * stops at max(rtol_velocity, 1e-6) (FP32 cannot go tighter).  Everything
 * else stays FP64: the Richardson residual of Algorithm 2 (eq. (f_impl) in
 * FP64), which refines each stage, the trace solves, the final projection
 * (in increment form) and the pressure reconstruction.  The Step I
 * preconditioner is the same FP16-stored Schwarz method in both modes. */
typedef enum { HDG_FP64 = 0, HDG_MIXED = 1 } hdg_precision;
/* Step II of Algorithm 2.  PRINTED (reading A): the mixed solve of eq.
 * (pressure_increment) with c = 1, psi-data -Div(psi, Qbar)/(a_ii dt) and
 * the update of Step III; its fixed point satisfies the stage momentum
 * equation but not the constraint Gamma(Q_i, p_i, lam_i) = 0 of eq.
 * (imex_implicit_solve_constraint), which only the final projection of
 * Algorithm 1 enforces.  STAGE_SOLVE (reading B): the mixed solve of the
 * stage operator itself (c = a_ii dt) with w-data (Qbar, w) and constraint
 * data -Gamma(psi, mu, Q, p, lam) of the iterate, whose solution is added to
 * the iterate: a fixed point solves eqs. (imex_implicit_solve) and
 * (imex_implicit_solve_constraint) exactly, and the iteration converges to
 * that monolithic stage solution as n_R grows. */
typedef enum { HDG_STEP2_PRINTED = 0, HDG_STEP2_STAGE_SOLVE = 1 } hdg_step2_reading;

typedef struct hdg_ctx hdg_ctx;
typedef struct hdg_batch hdg_batch;

/* Discretisation and solver parameters.  Paper values (Section "Setup"):
 * tau = alpha = delta_up = 1; the paper uses n_R = 2 Richardson iterations. */
typedef struct {
  int degree;            /* k: pressure and trace degree, velocity degree k+1; 1..4 */
  double tau;            /* HDG stabilisation, eq. (flux_hdg) */
  double alpha;          /* interior-penalty weight, eq. (f_impl) */
  double delta_up;       /* upwind weight, eq. (f_impl) */
  int imex;              /* hdg_imex_scheme */
  int n_richardson;      /* n_R of Algorithm 2 */
  int trace_solver;      /* hdg_trace_solver */
  double rtol_trace;     /* PCG: ||g - S lam||_2 <= rtol ||g||_2 (the residual's component along
                            the constant trace left out).  Round-off band: min(1e4 rtol, 1e-9)
                            relative.  A solve whose preconditioned residual r.z stalls (< 1 %
                            gain per four iterations for a quarter of the iterations spent, at
                            least 12) with the current |r| inside the band (the round-off floor
                            of an ill-conditioned S) also ends, counted as pcg_floor_stops in
                            hdg_get_info; so does, in the multigrid path, |r| setting no new 2 %
                            low over the same window inside the band.  The true residual g - S lam
                            of such a stop is recomputed (pcg_floor_true_residual_max) and must
                            lie in the band, else NOT_CONVERGED.  At max_it_trace: NOT_CONVERGED
                            unless the true residual is within min(1e2 rtol, band). */
  double rtol_velocity;  /* Step I: same criterion on the mass-scaled system; when BiCGStab's
                            recursive residual reaches it, the true residual is recomputed and
                            the solve continues from it unless it is within 10 rtol
                            (velocity_true_residual_max, velocity_true_residual_restarts) */
  int max_it_trace;
  int max_it_velocity;
  int pressure_update;   /* hdg_pressure_update */
  int idr_s;             /* Step I Krylov method: IDR(s) with this s (1..8), or 0 = BiCGStab */
  int precision;         /* hdg_precision */
  int use_graphs;        /* 1: the Krylov iteration blocks (PCG: 4 iterations, BiCGStab: 8)
                            are captured once as HIP graphs and replayed; 0: launched one by
                            one.  Results are the same.  Ignored while profiling is on. */
  int step1_block;       /* launch shape of the Step I operator: threads per workgroup, 64, 128
                            or 256 (two threads per cell).  The partial sums of the Krylov
                            inner products follow the workgroups, so results differ between
                            shapes in the last bits only; one shape always gives the same bits. */
  int step1_xcd;         /* 1: each of the eight XCDs (own L2) takes a contiguous eighth of the
                            cells; 0: the hardware's round-robin order of workgroups */
  int step1_precond;     /* Step I preconditioner (BiCGStab; ignored with idr_s > 0; right
                            preconditioning, so the
                            stopping residual is that of the unpreconditioned system): 1 =
                            additive Schwarz over facet patches (per interior facet, the block
                            of the operator on its two cells, formed per stage in FP64 and
                            stored in FP16, which changes the convergence, not the solution);
                            0 = none.  The patches contain the normal-continuous fields on
                            which the penalty term alpha h^-1 <[Q.n][w.n]> of eq. (f_impl)
                            vanishes, so the iteration count does not grow with that term's
                            weight adt/h^2 as it does for cell blocks.  On triangles the patch
                            inverses are held in Woodbury form (cell inverses and per-facet
                            trace-space corrections, the same operator); device memory per
                            cell: 8 nu^2 bytes of build scratch, 2 ((nu + 3m) nu + 3 nu m +
                            6 m^2) + 12 bytes of FP16 factors and (nu + 3m) vector entries of
                            apply scratch (nu = (k+2)(k+3), m = 2(k+2)).  On tetrahedra the
                            dense patch inverses: 8 nu^2 + 16 nu^2 bytes per cell
                            (nu = 3 dim P_{k+1}). */
  int step2_reading;     /* hdg_step2_reading */
  int step1_precond_lag; /* the Step I preconditioner is rebuilt when the stage's adt changes and
                            otherwise every this many stages (1, the default: every stage; its
                            Q* is then that of the stage).  A lagged preconditioner changes the
                            iteration count only, never the solution. */
  int dim;               /* 2: triangles (coords [nv][2], cells [nc][3]); 3: tetrahedra (coords
                            [nv][3], cells [nc][4], positively oriented, degree 1..2, FP64; the
                            method is stated for d = 2 and 3 in Sections "Discontinuous Galerkin
                            spaces" and "Hybridisation").  On tetrahedra: local facet f is the
                            triangle opposite local vertex f; facets are the sorted vertex triples
                            (lo, mid, hi) in lexicographic order with facet coordinates (s, t) at
                            x_lo + s (x_mid - x_lo) + t (x_hi - x_lo); bases are the centred
                            monomials ((d+1)x - 1)^a.. by degree and then descending exponents,
                            Gram-Schmidt orthonormalised on the reference cell (trace: for twice
                            the reference triangle's measure).  Not available on tetrahedra:
                            periodic meshes, forcing, the tracer and point evaluation. */
} hdg_params;

/* Fill p with the defaults: k=1, tau=alpha=delta_up=1, ARS(2,2,2), n_R=3,
 * MG-PCG, rtol 1e-12 for both solvers, caps 5000 / 20000, reconstruction,
 * BiCGStab for Step I with the facet-patch preconditioner, FP64, graph
 * replay on, Step I operator in workgroups of 256 threads in XCD order. */
void hdg_default_params(hdg_params* p);

/* Create a context on the current HIP device.  coords: host [nv][dim];
 * cells: host [nc][dim+1] vertex ids, positively oriented (det J > 0).  stream:
 * a hipStream_t (NULL = the null stream).  The mesh is copied.  Errors:
 * INVALID_ARG (bad mesh or parameters; message via hdg_last_error(NULL)),
 * UNSUPPORTED (degree), OUT_OF_MEMORY, DEVICE. */
int hdg_create(int64_t nv, const double* coords, int64_t nc, const int32_t* cells,
               const hdg_params* prm, void* stream, hdg_ctx** out);

/* Create a context on a periodic mesh (Section "Double-layer shear flow":
 * periodic boundary conditions in both directions).  vertex_rep: host [nv],
 * the vertex each vertex is identified with (itself if none); vertices with
 * the same representative are one topological vertex, so the cells on both
 * sides of a period share facets and every facet is interior.  Geometry uses
 * each cell's own coordinates, so a cell may reach across the period.  The
 * two placements of an identified facet must have the same length (else
 * INVALID_ARG), and no cell edge may join two identified vertices (a
 * periodic split-square mesh needs at least 3 x 3 squares).  vertex_rep =
 * NULL gives hdg_create.  Other arguments and errors as for hdg_create. */
int hdg_create_periodic(int64_t nv, const double* coords, int64_t nc, const int32_t* cells,
                        const int32_t* vertex_rep, const hdg_params* prm, void* stream, hdg_ctx** out);
void hdg_destroy(hdg_ctx* ctx);

/* Last error message of ctx, or of the last failed hdg_create in this
 * thread when ctx is NULL.  Never NULL. */
const char* hdg_last_error(const hdg_ctx* ctx);

/* Sizes, written to out[0..n-1] (n <= 8): ncells, nfacets, dim V_Q, dim
 * V_p, dim V_trace, number of cell quadrature points per cell, number of
 * vertices, degree. */
int hdg_sizes(const hdg_ctx* ctx, int64_t* out, int n);

/* Physical coordinates of the cell quadrature points, HOST buffer
 * [ncells][nq][2].  The caller evaluates the initial velocity there and
 * passes the values to hdg_set_velocity_from_points. */
int hdg_cell_points(const hdg_ctx* ctx, double* xy);

/* Physical coordinates of the facet quadrature points seen from each cell,
 * HOST buffer [ncells][3][nq_facet][2] (local facet f of a cell joins its
 * vertices (1,2), (0,2), (0,1) for f = 0, 1, 2; the number of facet points is
 * ceil((3k+4)/2)).  Used to pass a forcing to hdg_set_forcing. */
int hdg_facet_points(const hdg_ctx* ctx, double* xy);

/* Forcing f(x, t) = exp(-decay t) f0(x) of the momentum equation (eq.
 * f_expl, explicit in the IMEX stages; the form of the paper's Taylor-Green
 * forcing, eq. taylor_green_Q0_f).  cell_vals: f0 at the cell quadrature
 * points [ncells][nq][2], facet_vals: f0 at the facet points
 * [ncells][3][nq_facet][2], both DEVICE buffers, copied.  The forcing enters
 * the stage and final residuals (eqs. imex_residual, final_residual) and
 * the pressure reconstruction (f_p = -f + (Q.grad)Q, wall data -<mu, n.f>),
 * so set it before hdg_set_velocity_from_points.  cell_vals == NULL removes
 * the forcing. */
int hdg_set_forcing(hdg_ctx* ctx, const double* cell_vals, const double* facet_vals, double decay);

/* Time of the state (0 after hdg_create; hdg_advance adds dt per step).  It
 * only matters with a forcing. */
int hdg_set_time(hdg_ctx* ctx, double t);
double hdg_get_time(const hdg_ctx* ctx);

/* Initial state (the paper leaves it open): Q = cell-wise L2 projection of
 * the given point values [ncells][nq][2] with the cell rule; (p, lam) from
 * the pressure reconstruction of Q (with the forcing at the current time). */
int hdg_set_velocity_from_points(hdg_ctx* ctx, const double* qvals);

/* State exchange in the layout above (device pointers; get_state accepts
 * NULL for fields not wanted).  During a step in progress (see
 * hdg_advance_stages) get_state returns the state of the last completed
 * step; set_state, set_velocity_from_points and hdg_set_time abandon the
 * step in progress. */
int hdg_set_state(hdg_ctx* ctx, const double* Q, const double* p, const double* lam);
int hdg_get_state(const hdg_ctx* ctx, double* Q, double* p, double* lam);

/* Algorithm 1: nsteps IMEX-HDG steps of size dt from the current state.
 * BAD_STATE while a step started by hdg_advance_stages is unfinished. */
int hdg_advance(hdg_ctx* ctx, double dt, int nsteps);

/* Stage granularity of Algorithm 1 for schedulers that interleave jobs:
 * runs the next nstages implicit stages (each a full Algorithm 2 solve),
 * starting a step of size dt when none is in progress; the final projection
 * and the pressure reconstruction run right after the last stage of a step
 * (so a step of an s-stage scheme takes s - 1 stages).  Any chunking gives
 * results bit for bit equal to hdg_advance.  INVALID_ARG if a step is in
 * progress with another dt.  hdg_pending_stage: the next stage of the step
 * in progress (1..s-1), 0 if none, -1 for NULL. */
int hdg_advance_stages(hdg_ctx* ctx, double dt, int nstages);
int hdg_pending_stage(const hdg_ctx* ctx);

/* Passive tracer (Appendix "DG tracer advection"): a scalar q in DG_k
 * (layout and basis of the pressure, q[cell][s]) advected explicitly with
 * the IMEX scheme's explicit tableau by U = P_CG(Q_j), the L2 projection of
 * the stage velocities onto continuous CG_{k+1}; the transport form is
 * (q, div(chi U)) minus the upwind flux <q^up [[chi U.n]]> on interior
 * facets (walls carry no term, as printed), and the final update sums the
 * explicit weights b^ex_j over every stage j = 0..s-1 (printed from j = 1,
 * which would freeze q for IMEX Euler).  hdg_set_tracer: L2 projection of
 * the values at the cell points (device [ncells][nq_cell]; NULL switches
 * the tracer off); hdg_advance then transports it.  hdg_get_tracer: device
 * [ncells][n_p].  hdg_cg_project: U = P_CG(Q) in the layout of Q (device);
 * hdg_tracer_rate: out = M^-1 a(., q, P_CG(Q)) (device, tracer layout).
 * The CG space (a nodal basis on equispaced points, its mass matrix and
 * maps) is set up on first use; it is solved by Jacobi-PCG to a relative
 * residual of 1e-14. */
int hdg_set_tracer(hdg_ctx* ctx, const double* q_at_points);
int hdg_get_tracer(const hdg_ctx* ctx, double* q);
int hdg_cg_project(hdg_ctx* ctx, const double* Q, double* U);
int hdg_tracer_rate(hdg_ctx* ctx, const double* Q, const double* q, double* out);

/* Basis-free export: the velocity and pressure polynomials of every cell at
 * npts (1..1024) points given in reference coordinates (xi, eta) (host
 * [npts][2], the same for every cell; the cell map is the one of the data
 * layout; points outside the reference triangle extrapolate).  Q_out:
 * device [ncells][npts][2], p_out: device [ncells][npts]; either may be
 * NULL (not both).  Allocates a basis table of 8 * 1024 * (n_u/2 + n_p)
 * bytes on first use. */
int hdg_eval_points(hdg_ctx* ctx, const double* xy_ref, int npts, double* Q_out, double* p_out);

/* For callers that cannot allocate device memory (tight serving loops, code
 * that must not call hipMalloc): hdg_eval_points with the same arguments,
 * layout and results, but the basis table is staged in a static device array
 * of 288 KiB (1024 points at degree 4) that every device holds until the
 * process ends, so the call allocates nothing.  npts above 1024 gives
 * INVALID_ARG with a message.  All contexts on one device share that array:
 * calls that overlap on one device (contexts on different streams or host
 * threads) race and must be serialised by the caller. */
int hdg_eval_points_noalloc(hdg_ctx* ctx, const double* xy_ref, int npts, double* Q_out, double* p_out);

/* Host-side mesh of the square [0, length]^2 cut into n x n squares, each
 * split along a diagonal (the paper's test meshes): vertex (i, j) has id
 * j (n+1) + i at (i, j) length / n; square (i, j) gives the cells with ids
 * 2 (j n + i) and 2 (j n + i) + 1: (v00, v10, v11) and (v00, v11, v01) for
 * diagonal = 0 (the "/" diagonal), (v00, v10, v01) and (v10, v11, v01) for
 * diagonal = 1 ("\"), all counter-clockwise.  coords: [(n+1)^2][2], cells:
 * [2 n^2][3], vertex_rep: [(n+1)^2] or NULL when periodic = 0 (then the
 * identity); with periodic = 1 (n >= 3) the right and top vertices map to
 * their left and bottom copies (hdg_create_periodic). */
int hdg_mesh_square(int n, double length, int diagonal, int periodic, double* coords, int32_t* cells,
                    int32_t* vertex_rep);

/* Host-side mesh of the unit cube cut into n^3 cubes of six tetrahedra
 * (the Kuhn split, every tetrahedron of a cube contains its diagonal from
 * the corner nearest the origin; the three-dimensional workload, for the
 * method as stated for d = 3 in Section "Discontinuous Galerkin spaces"):
 * vertex (i, j, l) has id (l (n+1) + j)(n+1) + i at (i, j, l)/n; cube
 * (i, j, l) gives the cells 6 ((l n + j) n + i) + r, r = 0..5, one per
 * permutation (a, b, c) of the axes in lexicographic order, with vertices
 * corner, corner + e_a, corner + e_a + e_b, corner + (1, 1, 1) (all /n),
 * the last two swapped for an odd permutation so that det J > 0.
 * coords: [(n+1)^3][3], cells: [6 n^3][4] (caller-owned); 1 <= n <= 1024. */
int hdg_mesh_unit_cube(int n, double* coords, int32_t* cells);

/* One hybridised mixed solve (paper, Section "Solvers and preconditioners"):
 * find (U, p, lam) with
 *   (U, w) - c g(w, p, lam) = Fw(w),  Gamma(psi, mu, U, p, lam) = Fpsi(psi) + Fmu(mu)
 * for all (w, psi, mu); g and Gamma as in Section "Hybridisation".  The data
 * must satisfy Fpsi(1) = Fmu(1) (the component violating it is removed);
 * (p, lam) is normalised to int p = 0.  c > 0.  A null Fw, Fpsi or Fmu
 * stands for zero data. */
int hdg_solve_trace(hdg_ctx* ctx, double c, const double* Fw, const double* Fpsi,
                    const double* Fmu, double* U, double* p, double* lam);

/* y = S_c x for the condensed trace operator of hdg_solve_trace (a1). */
int hdg_trace_matvec(hdg_ctx* ctx, double c, const double* x, double* y);

/* Q* = P(Q), the H(div)-conforming (BDM) interpolant used as advecting
 * velocity (Section "Original fully-implicit DG method"): normal moments of
 * the facet average against P_{k+1}(F) (zero on walls) and interior moments
 * against the first-kind Nedelec space of degree k. */
int hdg_bdm_project(hdg_ctx* ctx, const double* Q, double* Qstar);

/* out = Div(psi, F) for all psi (dual vector in V_p): the weak divergence of
 * Section "Splitting method", central flux {F}.n on interior facets and
 * zero flux on walls. */
int hdg_weak_divergence(hdg_ctx* ctx, const double* F, double* out);

/* Algorithm 2, residual step: out(w) = r(w) - (Q, w) + adt (f_im(w, Q, Qstar)
 * + g(w, p, lam)), with f_im of eq. (f_impl). */
int hdg_momentum_residual(hdg_ctx* ctx, double adt, const double* r, const double* Qstar,
                          const double* Q, const double* p, const double* lam, double* out);

/* Algorithm 2, Step I: solve (Qbar, w) - adt f_im(w, Qbar, Qstar) = rhs(w). */
int hdg_tentative_velocity(hdg_ctx* ctx, double adt, const double* Qstar, const double* rhs,
                           double* Qbar);

/* The Step I preconditioner (step1_precond = 1) for the operator of
 * hdg_tentative_velocity in its mass-scaled form A = I - adt M^-1 f_im(., .;
 * Q*): z = sum over interior facets F of R_F^T A_F^{-1} R_F r, with A_F the
 * block of A on the unknowns of the two cells of F (couplings through other
 * facets dropped) and R_F the restriction to them.  r and z in the layout
 * of Q.  UNSUPPORTED when the context has the preconditioner off (also on a
 * mesh with a cell that touches no interior facet). */
int hdg_step1_precond(hdg_ctx* ctx, double adt, const double* Qstar, const double* r, double* z);

/* The constraint residual Gamma(psi, mu, Q, p, lam) of Section
 * "Hybridisation" (the second line of the hybridised system) as dual
 * vectors: Fpsi in the layout of p, Fmu in the layout of lam.  p or lam may
 * be NULL (zero). */
int hdg_constraint_residual(hdg_ctx* ctx, const double* Q, const double* p, const double* lam, double* Fpsi,
                            double* Fmu);

/* Pressure reconstruction (Section "Pressure reconstruction"): the mixed
 * problem with psi-data Div(psi, f_p), f_p = -f + (Q.grad_h)Q, and, with a
 * forcing set, the wall data -<mu n.f>, f taken at the context's time;
 * returns (p, lam) with int p = 0. */
int hdg_reconstruct_pressure(hdg_ctx* ctx, const double* Q, double* p, double* lam);

/* enable = N > 0: from now on time every N-th launch of each main kernel
 * class (Step I operator, residual, trace SpMV, smoother sweeps, AMG levels,
 * condensation, RHS condensation, back-substitution, BDM, weak divergence,
 * reconstruction data, Krylov vector updates) with HIP events on the context
 * stream; counters are reset.  hdg_get_info reports per class under
 * "kernels": all launches, the number timed and their summed milliseconds.
 * enable <= 0 stops timing. */
int hdg_profile(hdg_ctx* ctx, int enable);

/* JSON with sizes, iteration counts (totals since creation over every trace
 * and Step I solve, whether from hdg_advance or the single-step entry points,
 * and those of the last 16 solves), timings, the Step I launch shape, and the
 * device memory held (device_bytes) and the largest short-lived buffer
 * (device_transient_bytes, the condensation scratch of a trace-operator
 * build). */
int hdg_get_info(const hdg_ctx* ctx, char* buf, size_t cap);

/* ---------------------------------------------------------------- serving
 * Independent instances (many meshes, degrees, time steps) share one GPU.
 * For admission control, hdg_footprint_bytes estimates, on the host and
 * without touching the device, the device memory a context created from the
 * same arguments holds after its first hdg_advance(dt, .) (one trace
 * operator per distinct c of the scheme: the stage coefficients a_ii dt,
 * b^im_{s-1} dt and 1), plus the condensation scratch of an operator build.
 * It covers the forcing-free configuration; hdg_set_forcing adds
 * 8 (n_u + 2 nq_cell + 6 nq_facet) bytes per cell and 16 bytes per trace
 * unknown.  Mesh errors are
 * reported as by hdg_create (INVALID_ARG, message via hdg_last_error(NULL)). */
int hdg_footprint_bytes(int64_t nv, const double* coords, int64_t nc, const int32_t* cells,
                        const int32_t* vertex_rep, const hdg_params* prm, double dt, int64_t* bytes);

/* A batch is a non-owning view of n distinct contexts (none NULL); the
 * contexts must outlive it and must not be used elsewhere during
 * hdg_batch_advance.  hdg_batch_advance(b, dt[n], nsteps[n], status[n])
 * advances member i by nsteps[i] steps of dt[i], running the members on up
 * to 16 host threads: members on distinct HIP streams overlap on the
 * device, members sharing a stream are serialised by it.  Each member's
 * result is bit for bit that of a lone hdg_advance.  status (optional)
 * receives each member's hdg_status (details via hdg_last_error(member));
 * the return value is the first non-OK member status, else HDG_OK. */
int hdg_batch_create(int n, hdg_ctx* const* members, hdg_batch** out);
int hdg_batch_size(const hdg_batch* b);
int hdg_batch_advance(hdg_batch* b, const double* dt, const int* nsteps, int* status);
void hdg_batch_destroy(hdg_batch* b);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
