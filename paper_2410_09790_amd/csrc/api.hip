// C ABI, device memory management, Krylov solvers and the IMEX-HDG driver.
//
// Paper map:
//   Algorithm 1 (IMEX-HDG step)          -> Ctx::step
//   Algorithm 2 (Richardson, Steps I-III) -> Ctx::richardson
//   static condensation + trace solve     -> Ctx::solve_trace (a1, a7, a8, a9)
//   non-nested multigrid (P1 coarse space, facet-block smoother, AMG coarse
//   solve; Section "Solvers and preconditioners") -> Ctx::mg_apply
//   pressure reconstruction               -> Ctx::reconstruct
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <set>
#include <string>
#include <thread>
#include <vector>

#include "../../include/hdg.h"
#include "hdg_impl.h"
#include "kernels.h"

namespace hdg {

static thread_local std::string g_create_error;
constexpr int kMaxEvalPoints = 1024;

// Staging area of hdg_eval_points_noalloc: the velocity- and pressure-degree
// basis values at up to kMaxEvalPoints points for the largest degree
// (ns = 21 and np = 15 at k = 4), 288 KiB.  Every device the library runs on
// holds its own copy until the process ends; host code reaches it only
// through the address hipGetSymbolAddress gives on that device.
constexpr int kEvalScratchDoubles = kMaxEvalPoints * (21 + 15);
static __device__ __align__(256) double scratch[kEvalScratchDoubles];
static std::mutex g_scratch_mu;
static std::map<int, double*> g_scratch_ptr;  // device id -> that device's copy of scratch

// Address of the current device's copy of scratch, looked up once per device
// (the caller has made `device` current); nullptr if the lookup fails.
static double* scratch_address(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it != g_scratch_ptr.end()) return it->second;
  double* ptr = nullptr;
  if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  g_scratch_ptr[device] = ptr;
  return ptr;
}

struct HipError : std::runtime_error {
  explicit HipError(const std::string& s) : std::runtime_error(s) {}
};
struct OomError : std::runtime_error {
  explicit OomError(const std::string& s) : std::runtime_error(s) {}
};
struct ArgError : std::runtime_error {
  explicit ArgError(const std::string& s) : std::runtime_error(s) {}
};
struct SolverBreakdown : std::runtime_error {
  explicit SolverBreakdown(const std::string& s) : std::runtime_error(s) {}
};

#define HIPCHK(call)                                                                              \
  do {                                                                                            \
    hipError_t e_ = (call);                                                                       \
    if (e_ != hipSuccess) throw ::hdg::HipError(std::string(#call) + ": " + hipGetErrorString(e_));     \
  } while (0)
#define KCHK() HIPCHK(hipGetLastError())

static std::string sci(double v) {
  char b[32];
  std::snprintf(b, sizeof b, "%.3e", v);
  return b;
}

constexpr int kMaxStages = 4;
struct Tableau {
  int s;
  double Aex[kMaxStages][kMaxStages], bex[kMaxStages], Aim[kMaxStages][kMaxStages], bim[kMaxStages];
};

// explicit abscissa c_j = sum_l a^ex_jl
static double abscissa(const Tableau& t, int j) {
  double c = 0.0;
  for (int l = 0; l < t.s; ++l) c += t.Aex[j][l];
  return c;
}

static Tableau make_tableau(int which) {
  Tableau t{};
  if (which == HDG_IMEX_EULER) {
    t.s = 2;
    t.Aex[1][0] = 1.0; t.bex[0] = 1.0;
    t.Aim[1][1] = 1.0; t.bim[1] = 1.0;
  } else if (which == HDG_ARS222) {
    const double g = 1.0 - 1.0 / std::sqrt(2.0), d = 1.0 - 1.0 / (2.0 * g);
    t.s = 3;
    t.Aex[1][0] = g; t.Aex[2][0] = d; t.Aex[2][1] = 1.0 - d;
    t.bex[0] = d; t.bex[1] = 1.0 - d;
    t.Aim[1][1] = g; t.Aim[2][1] = 1.0 - g; t.Aim[2][2] = g;
    t.bim[1] = 1.0 - g; t.bim[2] = g;
  } else if (which == HDG_ARS233) {
    const double g = (3.0 + std::sqrt(3.0)) / 6.0;
    t.s = 3;
    t.Aex[1][0] = g; t.Aex[2][0] = g - 1.0; t.Aex[2][1] = 2.0 * (1.0 - g);
    t.bex[1] = 0.5; t.bex[2] = 0.5;
    t.Aim[1][1] = g; t.Aim[2][1] = 1.0 - 2.0 * g; t.Aim[2][2] = g;
    t.bim[1] = 0.5; t.bim[2] = 0.5;
  } else if (which == HDG_SSP2_332) {
    // SSP2(3,3,2) as printed (Appendix A) has an implicit first stage with
    // weight b^im_0 = 1/3.  Algorithm 1 fixes stage 0 to Q^n and never uses
    // the first implicit column, so the printed stages go after an explicit
    // stage 0 and all three are solved (rows/columns 1..3); the printed
    // abscissae are replaced by the row sums (0, 1/2, 1).
    const double h = 0.5, w = 1.0 / 3.0;
    t.s = 4;
    t.Aex[2][1] = h; t.Aex[3][1] = h; t.Aex[3][2] = h;
    t.bex[1] = t.bex[2] = t.bex[3] = w;
    t.Aim[1][1] = 0.25; t.Aim[2][2] = 0.25;
    t.Aim[3][1] = t.Aim[3][2] = t.Aim[3][3] = w;
    t.bim[1] = t.bim[2] = t.bim[3] = w;
  } else if (which == HDG_SSP3_433) {
    // SSP3(4,3,3) as printed, through Algorithm 1: stage 0 is Q^n and the
    // printed first implicit column (alpha, -alpha, 0, beta) is not used (its
    // weight b^im_0 is zero), so stages 1..3 are implicit with diagonal alpha.
    const double al = 0.24169426078821, bt = 0.06042356519705, et = 0.12915286960590;
    t.s = 4;
    t.Aex[2][1] = 1.0; t.Aex[3][1] = 0.25; t.Aex[3][2] = 0.25;
    t.bex[1] = t.bex[2] = 1.0 / 6.0; t.bex[3] = 2.0 / 3.0;
    t.Aim[1][1] = al; t.Aim[2][1] = 1.0 - al; t.Aim[2][2] = al;
    t.Aim[3][1] = et; t.Aim[3][2] = 0.5 - al - bt - et; t.Aim[3][3] = al;
    t.bim[1] = t.bim[2] = 1.0 / 6.0; t.bim[3] = 2.0 / 3.0;
  } else {
    throw ArgError("unknown IMEX scheme");
  }
  return t;
}

struct DevLevel {
  int n = 0;
  DCsr A{}, P{}, R{};
  double* dinv = nullptr;
  double omega = 0.0;
  double *b = nullptr, *x = nullptr, *x2 = nullptr, *r = nullptr;
};

struct TraceOp {
  double c = 0.0;
  double* Pinv = nullptr;
  double* vals = nullptr;
  int* cols = nullptr;
  double* Dinv = nullptr;
  bool mg = false;
  DCsr Pt{}, Rt{};
  std::vector<DevLevel> levels;
  int ncoarse = 0;
  double* coarse_pinv = nullptr;
  double *cb = nullptr, *cx = nullptr;  // coarsest rhs / solution
  hipGraphExec_t pcg_block = nullptr;    // captured block of PCG iterations
};

// Optional per-kernel-class timing with HIP events on the context stream:
// every `every`-th launch of a class is bracketed by two events (sampling
// keeps the cost of the event records out of the timed work).
enum KClass { KC_APPLY_OP = 0, KC_APPLY_RES, KC_TRACE_SPMV, KC_SMOOTH, KC_AMG, KC_CONDENSE, KC_RHS, KC_BACKSUB,
              KC_BDM, KC_DIV, KC_RECON, KC_VECTOR, KC_PC_APPLY, KC_PC_BUILD, kNumKClass };
static const char* kKClassName[kNumKClass] = {"apply_step1_operator", "apply_residual", "trace_spmv",
                                              "trace_jacobi_sweep", "amg_coarse", "condense_assemble",
                                              "rhs_condense", "backsub", "bdm", "weak_div", "recon_rhs",
                                              "krylov_vector", "step1_precond_apply", "step1_precond_build"};

struct Profiler {
  bool on = false;
  int every = 1;
  hipStream_t st = nullptr;
  std::vector<hipEvent_t> pool;
  struct Pending { int cls; hipEvent_t a, b; };
  std::vector<Pending> pending;
  double ms[kNumKClass] = {};   // summed over the timed launches
  long launches[kNumKClass] = {};
  long timed[kNumKClass] = {};
  bool sample(int cls) { return on && launches[cls]++ % every == 0; }
  hipEvent_t get() {
    if (pool.empty()) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) throw std::runtime_error("hipEventCreate failed");
      return e;
    }
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  void harvest() {  // after a stream synchronisation
    for (auto& p : pending) {
      float t = 0.f;
      if (hipEventElapsedTime(&t, p.a, p.b) == hipSuccess) ms[p.cls] += t;
      timed[p.cls] += 1;
      pool.push_back(p.a);
      pool.push_back(p.b);
    }
    pending.clear();
  }
  void reset() {
    for (int i = 0; i < kNumKClass; ++i) { ms[i] = 0.0; launches[i] = 0; timed[i] = 0; }
  }
  ~Profiler() {
    for (auto& p : pending) { (void)hipEventDestroy(p.a); (void)hipEventDestroy(p.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct Timed {
  Profiler& pr;
  int cls;
  hipEvent_t a = nullptr;
  Timed(Profiler& p, int c) : pr(p), cls(c) {
    if (pr.sample(cls)) { a = pr.get(); (void)hipEventRecord(a, pr.st); }
  }
  ~Timed() {
    if (a) {
      hipEvent_t b = pr.get();
      (void)hipEventRecord(b, pr.st);
      pr.pending.push_back({cls, a, b});
    }
  }
};

}  // namespace hdg

struct hdg_ctx {
  hdg::Profiler prof;
  hdg_params prm{};
  hdg::Step1Launch s1{256, 1};  // launch shape of the Step I operator (from prm)
  int k = 1;
  int dim = 2, nfc = 3;  // tetrahedra: 3, 4
  int tk = 1;            // key of the trace-operator kernels (k; 10 + k on tetrahedra)
  int slots = 5;         // facet blocks per trace-operator row (7 on tetrahedra)
  hipStream_t st = nullptr;
  hdg::HostMesh hm;
  hdg::RefTables rt;
  hdg::RefTables3 rt3;
  hdg::DMesh dm{};
  hdg::DTab dt{};
  int ns = 0, np = 0, nf = 0, nu = 0, nlam = 0, nqc = 0, nqf = 0;
  long nQ = 0, nP = 0, nT = 0;
  double area = 0.0;
  std::vector<void*> allocs;
  int device = 0;              // HIP device current at creation
  size_t dev_bytes = 0;        // device memory held (every dalloc)
  size_t dev_transient = 0;    // largest short-lived allocation (trace-operator assembly)
  std::map<double, std::unique_ptr<hdg::TraceOp>> ops;
  // work vectors
  double *ycell = nullptr, *g = nullptr, *part = nullptr, *part2 = nullptr, *scal = nullptr;
  double *pr = nullptr, *pz = nullptr, *pp = nullptr, *pq = nullptr, *t1 = nullptr, *t2 = nullptr, *t3 = nullptr;
  double *br = nullptr, *bt = nullptr;  // IDR(s) residual and work vector
  double* bsc = nullptr;                 // BiCGStab scalar slots
  double* kpart = nullptr;               // partials of t = A s (4 sets)
  double *adv = nullptr, *Qs = nullptr, *dr = nullptr, *Qbar = nullptr, *dQ = nullptr, *dp = nullptr, *dl = nullptr,
         *fpsi = nullptr, *Ut = nullptr;
  double* fmu = nullptr;  // trace data of a mixed solve (reading B of Step II)
  double *Q = nullptr, *p = nullptr, *lam = nullptr;
  double* stQ[hdg::kMaxStages] = {};
  double* stP[hdg::kMaxStages] = {};
  double* stL[hdg::kMaxStages] = {};
  double* stR[hdg::kMaxStages] = {};
  double* stMQ[hdg::kMaxStages] = {};
  static constexpr int kPinned = 512;
  double* h_pinned = nullptr;
  bool have_state = false;
  std::string err;
  // statistics
  std::vector<int> pcg_iters, bicg_iters;
  long total_pcg = 0, total_bicg = 0, n_trace_solves = 0, n_velocity_solves = 0, bicg_restarts = 0;
  long pcg_floor_stops = 0;  // trace solves ended at the round-off floor (within floor_band())
  double pcg_floor_true_max = 0.0;  // largest true relative residual |g - S x| / |g| of those solves
  double velocity_true_max = 0.0;   // largest true relative residual of a converged Step I solve
  long velocity_true_restarts = 0;  // Step I solves continued because the true residual was above 10 rtol
  static constexpr int kPcgFlatBlocks = 3;  // shortest stall window (blocks); it grows to a quarter of the iterations spent
  static constexpr long kSmallTrace = 24576;  // trace unknowns up to which Jacobi-PCG runs in one workgroup
  double* small_info = nullptr;
  int pcg_small(hdg::TraceOp& op, const double* gin, double gnorm, double* x);
  static constexpr double kPcgFloor = 1e4;
  static constexpr double kPcgFloorMax = 1e-9;
  // Relative round-off band of the trace solve: a solve may end above rtol
  // only with its residual inside this band.  It is kPcgFloor * rtol, but
  // never above kPcgFloorMax, so that a loose rtol does not widen it.
  double floor_band() const { return std::min(kPcgFloor * prm.rtol_trace, kPcgFloorMax); }
  double trace_true_residual(hdg::TraceOp& op, const double* gin, const double* x);
  // a solve ended at the round-off floor: its true residual must lie in the band
  void accept_floor(double true_rel, int its) {
    ++pcg_floor_stops;
    pcg_floor_true_max = std::max(pcg_floor_true_max, true_rel);
    if (true_rel > floor_band())
      cap_reached("PCG on the trace system: stalled after " + std::to_string(its) + " iterations with a true "
                  "relative residual of " + hdg::sci(true_rel) + ", above the round-off band " + hdg::sci(floor_band()));
  }
  double t_trace = 0.0, t_velocity = 0.0, t_other = 0.0;
  int max_pcg_bicg_seen = 0;
  bool not_converged = false;
  // an iteration cap was reached: the result is kept and flagged; the first
  // such event of a call is reported through hdg_last_error
  void cap_reached(const std::string& what) {
    if (!not_converged) err = what;
    not_converged = true;
  }

  template <class T>
  T* dalloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) throw hdg::OomError("hipMalloc of " + std::to_string(n * sizeof(T)) + " bytes failed");
    allocs.push_back(p);
    dev_bytes += n * sizeof(T);
    return static_cast<T*>(p);
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* d = dalloc<T>(v.size());
    HIPCHK(hipMemcpyAsync(d, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, st));
    return d;
  }
  void sync() {
    HIPCHK(hipStreamSynchronize(st));
    if (prof.on || !prof.pending.empty()) prof.harvest();
  }
  double read_scalar(const double* d) {
    HIPCHK(hipMemcpyAsync(h_pinned, d, sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    return h_pinned[0];
  }

  void setup();
  void setup_tri();
  void setup_tet();
  void setup_work();
  hdg::TraceOp& trace_op(double c);
  void build_mg(hdg::TraceOp& op);
  void precond(hdg::TraceOp& op, const double* r, double* z);
  void project_null(double* v);
  void mg_apply(hdg::TraceOp& op, const double* r, double* z);
  void vcycle(hdg::TraceOp& op, int l);
  int pcg(hdg::TraceOp& op, const double* g, double* x);
  static constexpr int kPcgBlock = 4;  // PCG iterations per captured block
  void pcg_block(hdg::TraceOp& op);
  double* px = nullptr;                // PCG iterate (fixed address for the captured block)
  void solve_trace(double c, const double* Fw, const double* Fpsi, const double* Fmu, double* U, double* p,
                   double* lam);
  // BiCGStab vectors, structure-of-arrays
  // structure-of-arrays Krylov vectors of the Step I solve, FP64 or, in the
  // mixed-precision mode (kx32), FP32
  struct KrylovBuf {
    void *b = nullptr, *x = nullptr, *r = nullptr, *rh = nullptr, *s = nullptr, *t = nullptr, *p = nullptr,
         *v = nullptr;
    void *ph = nullptr, *sh = nullptr;  // preconditioned directions (right preconditioning)
  };
  bool kx32 = false;  // FP32 Step I: vectors, volume data, upwind weights and arithmetic
  static constexpr double kMixedRtolFloor = 1e-6;
  KrylovBuf kd;
  // per-stage Step I data of the current Q*: the volume data (triangles: the
  // advecting field at the cell points; tetrahedra: the cell volume
  // matrices; FP32 in the mixed-precision mode) and facet upwind weights
  // (tiles of 32 cells) for the Step I operator, and the advection data of the
  // cell-major residual kernels (FP64 in both modes: the Richardson residual
  // is the accuracy reference)
  void* vk = nullptr;
  bool vk32 = false;
  void* vbeta = nullptr;  // upwind weights, FP32 when kx32
  void prepare_step1(const double* Qstar) {
    hdg::launch_prep_adv(k, st, dm, dt, Qstar, prm.delta_up, adv);
    hdg::launch_step1_data(k, st, dm, dt, Qstar, prm.delta_up, vk, vk32, vbeta, kx32);
    vk_qs = Qstar;
    ++vk_gen;
  }
  // Step I preconditioner (facet-patch additive Schwarz): built for the Q*
  // and adt of the current stage on the first solve that needs it
  const double* vk_qs = nullptr;  // Q* the Step I data were prepared for
  long vk_gen = 0, pc_gen = -1;   // generation of the Step I data / of the preconditioner
  double pc_adt = 0.0;
  bool pc_on = false;
  double* pcD = nullptr;          // cell blocks (FP64 scratch of the build)
  void* pcB = nullptr;            // patch inverses (FP16; in 2D the cell inverses and facet corrections)
  void* pcS = nullptr;            // 2D: first-pass results (A^{-1} r and the facet traces)
  long pc_builds = 0;
  void pc_prepare(double adt) {
    // rebuilt for a new adt, else when the stage data are step1_precond_lag generations newer
    if (!pc_on || (pc_adt == adt && pc_gen >= 0 && vk_gen - pc_gen < prm.step1_precond_lag)) return;
    hdg::Timed tm(prof, hdg::KC_PC_BUILD);
    if (dim == 3)  // from the stage's FP64 V and beta (prepare_step1, the residual kernels' copy)
      hdg::launch3_pc_build(k, st, dm, dt.t3, adv, adv + hm.nc * (long)ns * ns, prm.alpha, adt, pcD, pcB);
    else
      hdg::launch_pc_build(k, st, dm, dt, vk_qs, prm.delta_up, prm.alpha, adt, pcD, pcB);
    KCHK();
    pc_gen = vk_gen;
    pc_adt = adt;
    ++pc_builds;
  }
  void pc_apply(const void* r, void* z) {
    hdg::Timed tm(prof, hdg::KC_PC_APPLY);
    if (dim == 3) hdg::launch3_pc_apply(k, st, dm, pcB, r, z, kx32);
    else hdg::launch_pc_apply(k, st, dm, pcB, pcS, r, z, kx32);
  }
  int bicgstab(double adt, const double* b, double* x);
  static constexpr int kBicgBlock = 8;  // BiCGStab iterations per captured block
  void bicgstab_block(double adt);
  std::map<double, hipGraphExec_t> bicg_graphs;  // captured blocks per adt
  // Graph capture runs on a private stream (capture is not possible on the
  // legacy null stream a caller may pass); the graphs are launched on st.
  hipStream_t cap_st = nullptr;
  template <class Body>
  hipGraphExec_t capture(Body&& body);
  int idrs(double adt, const double* b, double* x);
  int velocity_solve(double adt, const double* b, double* x) {
    return prm.idr_s > 0 ? idrs(adt, b, x) : bicgstab(adt, b, x);
  }
  double *iP = nullptr, *iG = nullptr, *iU = nullptr, *ired = nullptr;
  void reconstruct(const double* Qin, double* pout, double* lout);
  // forcing f(x, t) = exp(-f_decay t) f0(x) (eq. f_expl): f0 as a dual vector,
  // at the cell and facet points, and its wall data; time of the state
  double time = 0.0, f_decay = 0.0;
  double *f_dual = nullptr, *f_cell = nullptr, *f_fac = nullptr, *f_wall = nullptr, *f_tmp = nullptr;
  bool forced = false;
  double f_scale(double tt) const { return std::exp(-f_decay * tt); }
  void richardson(double adt, const double* r, double* Q, double* p, double* lam);
  void step(double dt);
  // passive tracer (Appendix "DG tracer advection"): q in DG_k advected by
  // P_CG(Q_j) with the explicit tableau; the CG_{k+1} space is set up on
  // first use
  bool tracer_on = false;
  double *trq = nullptr, *trq_tmp = nullptr, *Ucg = nullptr;
  double* trR[hdg::kMaxStages] = {};
  struct Cg {
    bool ready = false;
    int N = 0;
    int *l2g = nullptr, *gptr = nullptr, *ginc = nullptr;
    double *T = nullptr, *dinv = nullptr, *b = nullptr, *u = nullptr, *r = nullptr, *z = nullptr, *p = nullptr,
           *w = nullptr, *sc = nullptr;
    hdg::DCsr M{};
    int last_its = 0;
  } cg;
  void cg_setup();
  void cg_project(const double* Qin, double* Uout);
  void tracer_alloc();
  void tracer_step(double dtv);
  int pend_stage = 0;     // next implicit stage of a step in progress (0: none)
  double* eval_tab = nullptr;  // basis values at hdg_eval_points' points
  double* eval_scratch = nullptr;        // this device's copy of scratch (hdg_eval_points_noalloc)
  std::vector<double> eval_host;         // host staging of the same values, sized at creation
  double pend_dt = 0.0;   // its time step
  void begin_step(double dt);
  void stage_once();
  void finish_step();
};

using namespace hdg;

void hdg_ctx::setup() {
  if (dim == 3) {
    ns = rt3.ns; np = rt3.np; nf = rt3.nf; nu = 3 * ns; nlam = 4 * nf; nqc = rt3.nqc; nqf = rt3.nqf;
    nfc = 4; tk = 10 + k; slots = 7;
  } else {
    ns = rt.ns; np = rt.np; nf = rt.nf; nu = 2 * ns; nlam = 3 * nf; nqc = rt.nqc; nqf = rt.nqf;
    nfc = 3; tk = k; slots = 5;
  }
  const long nc = hm.nc, nF = hm.nF;
  nQ = nc * nu; nP = nc * np; nT = nF * nf;
  area = 0.0;
  dm.dim = dim;
  if (dim == 3) {
    setup_tet();
  } else {
    for (long e = 0; e < nc; ++e) area += 0.5 * hm.geo[G_DET * nc + e];
    setup_tri();
  }
  setup_work();
}

// triangles: mesh and reference tables
void hdg_ctx::setup_tri() {
  const long nc = hm.nc;
  // mesh
  std::vector<double> geo((size_t)kDGeo * nc);
  const int map[kDGeo] = {G_DET, G_IJ00, G_IJ01, G_IJ10, G_IJ11, G_NX0, G_NY0, G_NX1, G_NY1, G_NX2, G_NY2,
                          G_H0, G_H1, G_H2, G_J00, G_J01, G_J10, G_J11};
  for (int f = 0; f < kDGeo; ++f)
    std::memcpy(&geo[(size_t)f * nc], &hm.geo[(size_t)map[f] * nc], nc * sizeof(double));
  dm.nc = (int)nc;
  dm.nF = (int)hm.nF;
  dm.geo = upload(geo);
  dm.cf_facet = upload(hm.cf_facet);
  dm.cf_nb = upload(hm.cf_nb);
  dm.cf_nbf = upload(hm.cf_nbf);
  dm.cf_flip = upload(hm.cf_flip);
  {
    // packed neighbour descriptor: one load gives the neighbour, its local
    // facet and whether the two local facet parametrisations run opposite
    std::vector<int32_t> nbx(3 * (size_t)nc, -1);
    for (int f = 0; f < 3; ++f)
      for (long e = 0; e < nc; ++e) {
        const int en = hm.cf_nb[f * nc + e];
        if (en < 0) continue;
        const int fn = hm.cf_nbf[f * nc + e];
        const int rev = hm.cf_flip[f * nc + e] != hm.cf_flip[(long)fn * nc + en];
        nbx[f * nc + e] = (en << 3) | (fn << 1) | rev;
      }
    dm.cf_nbx = upload(nbx);
  }
  dm.fc_cell = upload(hm.fc_cell);
  dm.fc_f = upload(hm.fc_f);
  // tables (constant address space on the device side)
  auto cu = [&](const std::vector<double>& v) { return (cdptr)upload(v); };
  dt.Bu = cu(rt.Bu); dt.Gux = cu(rt.Gux); dt.Guy = cu(rt.Guy);
  dt.Bp = cu(rt.Bp); dt.Gpx = cu(rt.Gpx); dt.Gpy = cu(rt.Gpy); dt.cw = cu(rt.cq_w);
  dt.FBu = cu(rt.FBu); dt.FGux = cu(rt.FGux); dt.FGuy = cu(rt.FGuy); dt.FBp = cu(rt.FBp);
  dt.fw = cu(rt.fq_w); dt.MU = cu(rt.MU); dt.NUB = cu(rt.NUB); dt.TRU = cu(rt.TRU);
  dt.Dx = cu(rt.Dx); dt.Dy = cu(rt.Dy); dt.Rx = cu(rt.Rx); dt.Ry = cu(rt.Ry);
  dt.Chat = cu(rt.Chat); dt.That = cu(rt.That); dt.Ehat = cu(rt.Ehat); dt.CC = cu(rt.CC);
  dt.KDD = cu(rt.KDD); dt.CD = cu(rt.CD); dt.BDMinv = cu(rt.BDMinv); dt.NED = cu(rt.NED);
}

// tetrahedra: mesh and reference tables (geometry fields in the device order)
void hdg_ctx::setup_tet() {
  const long nc = hm.nc;
  for (long e = 0; e < nc; ++e) area += hm.geo[E_DET * nc + e] / 6.0;
  static_assert((int)kGeo3 == (int)kDGeo3 && (int)E_N == (int)E3_N && (int)E_A == (int)E3_A, "geometry layout");
  dm.nc = (int)nc;
  dm.nF = (int)hm.nF;
  dm.geo = upload(hm.geo);
  dm.cf_facet = upload(hm.cf_facet);
  dm.cf_nb = upload(hm.cf_nb);
  dm.cf_nbf = upload(hm.cf_nbf);
  dm.cf_flip = upload(hm.cf_flip);
  dm.cf_nbx = nullptr;
  dm.fc_cell = upload(hm.fc_cell);
  dm.fc_f = upload(hm.fc_f);
  DTab3& t = dt.t3;
  t.Bu = upload(rt3.Bu); t.dBu = upload(rt3.dBu); t.Bp = upload(rt3.Bp); t.dBp = upload(rt3.dBp);
  t.cw = upload(rt3.cq_w);
  t.FBu = upload(rt3.FBu); t.FdBu = upload(rt3.FdBu); t.FBp = upload(rt3.FBp); t.fw = upload(rt3.fq_w);
  t.MU = upload(rt3.MU); t.NUL = upload(rt3.NUL);
  t.D = upload(rt3.D); t.R = upload(rt3.R); t.KDD = upload(rt3.KDD); t.That = upload(rt3.That);
  t.Chat = upload(rt3.Chat); t.Ehat = upload(rt3.Ehat); t.CD = upload(rt3.CD); t.NEDM = upload(rt3.NEDM);
  t.BDMinv = upload(rt3.BDMinv);
}

// work vectors (both cell shapes)
void hdg_ctx::setup_work() {
  const long nc = hm.nc;
  // work
  ycell = dalloc<double>(nc * nlam);
  g = dalloc<double>(nT);
  // (tetrahedra: the back-substitution also keeps nc cell integrals behind its partial sums)
  part = dalloc<double>(std::max<long>((long)kRedBlocks * kIdrMax, 4L * apply_soa_blocks(nc, s1.block) + 16) +
                        (dim == 3 ? nc : 0));
  part2 = dalloc<double>(2 * kRedBlocks);
  const int mt = prm.max_it_trace + 4, mv = prm.max_it_velocity + 4;
  scal = dalloc<double>(3 * mt + 16);
  bsc = dalloc<double>((long)BS_STRIDE * std::max(mv + 2, kBicgBlock + 2));
  kpart = dalloc<double>(4L * apply_soa_blocks(nc, s1.block) + 16);
  pr = dalloc<double>(nT); pz = dalloc<double>(nT); pp = dalloc<double>(nT); pq = dalloc<double>(nT);
  t1 = dalloc<double>(nT); t2 = dalloc<double>(nT); t3 = dalloc<double>(nT); px = dalloc<double>(nT);
  small_info = dalloc<double>(4);
  kx32 = prm.precision == HDG_MIXED;
  auto kvec = [&]() -> void* { return kx32 ? (void*)dalloc<float>(nQ) : (void*)dalloc<double>(nQ); };
  for (void** v : {&kd.b, &kd.x, &kd.r, &kd.rh, &kd.s, &kd.t, &kd.p, &kd.v}) *v = kvec();
  // the facet-patch preconditioner needs every cell on an interior facet
  // (else a cell would receive no correction)
  pc_on = prm.step1_precond == 1 && prm.idr_s == 0;
  for (long e = 0; pc_on && e < nc; ++e) {
    bool any = false;
    for (int f = 0; f < nfc; ++f) any = any || hm.cf_nb[f * nc + e] >= 0;
    pc_on = any;
  }
  if (pc_on) {
    kd.ph = kvec();
    kd.sh = kvec();
    pcD = dalloc<double>(nc * nu * nu);
    const long npc = dim == 3 ? pc_entries3(k, nc) : pc_entries(k, nc);
    pcB = dalloc<uint16_t>(npc);
    HIPCHK(hipMemsetAsync(pcB, 0, npc * sizeof(uint16_t), st));  // padding entries stay zero
    if (dim == 2) pcS = kx32 ? (void*)dalloc<float>(pc_scratch(k, nc)) : (void*)dalloc<double>(pc_scratch(k, nc));
  }
  const long nc32 = (nc + 31) / 32 * 32;
  vk32 = prm.precision == HDG_MIXED;
  // Step I volume data: tetrahedra, the cell matrices (ns x ns); triangles, the field at the cell points
  const long nvk = dim == 3 ? (long)ns * ns : 2L * nqc;
  vk = vk32 ? (void*)dalloc<float>(nvk * nc32) : (void*)dalloc<double>(nvk * nc32);
  vbeta = kx32 ? (void*)dalloc<float>((long)nfc * nqf * nc32) : (void*)dalloc<double>((long)nfc * nqf * nc32);
  br = dalloc<double>(nQ); bt = dalloc<double>(nQ);
  // residual-kernel advection data (tetrahedra: the cell volume matrices and the facet weights)
  adv = dalloc<double>(dim == 3 ? (long)nc * (ns * ns + 4 * nqf) : (long)nc * (2 * nqc + 3 * nqf));
  Qs = dalloc<double>(nQ); dr = dalloc<double>(nQ); Qbar = dalloc<double>(nQ); dQ = dalloc<double>(nQ);
  dp = dalloc<double>(nP); dl = dalloc<double>(nT); fpsi = dalloc<double>(nP); Ut = dalloc<double>(nQ);
  fmu = dalloc<double>(nT);
  Q = dalloc<double>(nQ); p = dalloc<double>(nP); lam = dalloc<double>(nT);
  for (int i = 0; i < make_tableau(prm.imex).s; ++i) {
    stQ[i] = dalloc<double>(nQ); stP[i] = dalloc<double>(nP); stL[i] = dalloc<double>(nT);
    stR[i] = dalloc<double>(nQ); stMQ[i] = dalloc<double>(nQ);
  }
  HIPCHK(hipHostMalloc((void**)&h_pinned, kPinned * sizeof(double), hipHostMallocDefault));
  prof.st = st;
  sync();
}

TraceOp& hdg_ctx::trace_op(double c) {
  auto it = ops.find(c);
  if (it != ops.end()) return *it->second;
  auto op = std::make_unique<TraceOp>();
  op->c = c;
  const long nc = hm.nc, nF = hm.nF;
  op->Pinv = dalloc<double>(nc * np * np);
  double* SK = nullptr;
  HIPCHK(hipMalloc(&SK, sizeof(double) * nc * nlam * nlam));
  dev_transient = std::max(dev_transient, sizeof(double) * nc * nlam * nlam);
  op->vals = dalloc<double>((long)slots * nF * nf * nf);
  op->cols = dalloc<int>((long)slots * nF);
  op->Dinv = dalloc<double>(nF * nf * nf);
  {
    Timed tm(prof, KC_CONDENSE);
    launch_condense(k, st, dm, dt, c, prm.tau, op->Pinv, SK);
    KCHK();
    launch_assemble(k, st, dm, SK, op->vals, op->cols, op->Dinv);
    KCHK();
  }
  sync();
  HIPCHK(hipFree(SK));
  if (prm.trace_solver == HDG_TRACE_MG_PCG) build_mg(*op);
  TraceOp& ref = *op;
  ops[c] = std::move(op);
  return ref;
}

// Galerkin P1 coarse operator and AMG hierarchy (host setup, device apply)
void hdg_ctx::build_mg(TraceOp& op) {
  const long nF = hm.nF;
  std::vector<double> vals((size_t)slots * nF * nf * nf);
  std::vector<int> cols((size_t)slots * nF);
  HIPCHK(hipMemcpyAsync(vals.data(), op.vals, vals.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(cols.data(), op.cols, cols.size() * sizeof(int), hipMemcpyDeviceToHost, st));
  sync();
  Csr S;
  S.nrows = S.ncols = nT;
  S.ptr.assign(nT + 1, 0);
  for (long F = 0; F < nF; ++F)
    for (int i = 0; i < nf; ++i) {
      const long row = F * nf + i;
      for (int s = 0; s < slots; ++s)
        for (int j = 0; j < nf; ++j) {
          double v = vals[((long)(s * nf + i) * nf + j) * nF + F];
          if (v == 0.0) continue;
          S.idx.push_back(cols[s * nF + F] * nf + j);
          S.val.push_back(v);
        }
      S.ptr[row + 1] = (int32_t)S.idx.size();
    }
  Csr Pt;
  Pt.nrows = nT;
  Pt.ncols = hm.nvt;
  Pt.ptr.assign(nT + 1, 0);
  if (dim == 3) {
    // the hat functions of the facet's three vertices (1 - s - t, s, t in the
    // facet's coordinates) projected onto the orthonormal trace basis
    double proj[3][64] = {};
    for (int q = 0; q < rt3.nqf; ++q) {
      const double sq = rt3.fq_s[q], tq = rt3.fq_t[q], w = 2.0 * rt3.fq_w[q];
      const double hat[3] = {1.0 - sq - tq, sq, tq};
      for (int v = 0; v < 3; ++v)
        for (int i = 0; i < nf; ++i) proj[v][i] += w * hat[v] * rt3.MU[(size_t)q * nf + i];
    }
    for (long F = 0; F < nF; ++F)
      for (int i = 0; i < nf; ++i) {
        const long row = F * nf + i;
        const int32_t vv[3] = {hm.facet_lo[F], hm.facet_mid[F], hm.facet_hi[F]};
        for (int v = 0; v < 3; ++v)
          if (std::fabs(proj[v][i]) > 1e-14) { Pt.idx.push_back(vv[v]); Pt.val.push_back(proj[v][i]); }
        Pt.ptr[row + 1] = (int32_t)Pt.idx.size();
      }
  } else {
    const double r3 = 0.5 / std::sqrt(3.0);
    for (long F = 0; F < nF; ++F)
      for (int i = 0; i < nf; ++i) {
        const long row = F * nf + i;
        if (i == 0) {  // mean of the linear function
          Pt.idx.push_back(hm.facet_lo[F]); Pt.val.push_back(0.5);
          Pt.idx.push_back(hm.facet_hi[F]); Pt.val.push_back(0.5);
        } else if (i == 1) {  // slope in the orthonormal Legendre basis
          Pt.idx.push_back(hm.facet_lo[F]); Pt.val.push_back(-r3);
          Pt.idx.push_back(hm.facet_hi[F]); Pt.val.push_back(r3);
        }
        Pt.ptr[row + 1] = (int32_t)Pt.idx.size();
      }
  }
  Csr Rt = csr_transpose(Pt);
  Csr Ac = csr_multiply(Rt, csr_multiply(S, Pt));
  AmgHierarchy h;
  amg_setup(Ac, h, 200, dim == 2);
  auto up = [&](const Csr& A) {
    DCsr d;
    d.n = (int)A.nrows;
    d.ptr = upload(A.ptr);
    d.idx = A.idx.empty() ? dalloc<int>(1) : upload(A.idx);
    d.val = A.val.empty() ? dalloc<double>(1) : upload(A.val);
    return d;
  };
  op.Pt = up(Pt);
  op.Rt = up(Rt);
  for (auto& L : h.levels) {
    DevLevel d;
    d.n = (int)L.A.nrows;
    d.A = up(L.A); d.P = up(L.P); d.R = up(L.R);
    d.dinv = upload(L.dinv);
    d.omega = L.omega;
    d.b = dalloc<double>(d.n); d.x = dalloc<double>(d.n); d.x2 = dalloc<double>(d.n); d.r = dalloc<double>(d.n);
    op.levels.push_back(d);
  }
  op.ncoarse = (int)h.ncoarse;
  op.coarse_pinv = upload(h.coarse_pinv);
  op.cb = dalloc<double>(op.ncoarse);
  op.cx = dalloc<double>(op.ncoarse);
  op.mg = true;
  sync();
}

void hdg_ctx::vcycle(TraceOp& op, int l) {
  // level l solves A_l x = b with b in levels[l].b (or op.cb on the coarsest level)
  if (l == (int)op.levels.size()) {
    launch_dense_mv(st, op.ncoarse, op.coarse_pinv, op.cb, op.cx);
    return;
  }
  DevLevel& L = op.levels[l];
  launch_csr_jacobi(st, L.A, L.dinv, L.omega, L.b, nullptr, L.x);
  launch_csr_jacobi(st, L.A, L.dinv, L.omega, L.b, L.x, L.x2);
  launch_csr_spmv(st, L.A, L.x2, L.r, 0.0);
  launch_axpby(st, L.n, 1.0, L.b, -1.0, L.r);
  const bool last = (l + 1 == (int)op.levels.size());
  double* bc = last ? op.cb : op.levels[l + 1].b;
  double* xc = last ? op.cx : op.levels[l + 1].x;
  launch_csr_spmv(st, L.R, L.r, bc, 0.0);
  vcycle(op, l + 1);
  // on the next level the result of vcycle is in its x (levels) or cx (coarsest)
  launch_csr_spmv(st, L.P, xc, L.x2, 1.0);
  launch_csr_jacobi(st, L.A, L.dinv, L.omega, L.b, L.x2, L.x);
  launch_csr_jacobi(st, L.A, L.dinv, L.omega, L.b, L.x, L.x2);
  launch_copy(st, L.n, L.x2, L.x);
}

// z = B r: two damped facet-block-Jacobi sweeps, P1 coarse correction, two sweeps
void hdg_ctx::mg_apply(TraceOp& op, const double* r, double* z) {
  const int nF = (int)hm.nF;
  const double om = 0.7;
  {
    Timed tm(prof, KC_SMOOTH);
    launch_jacobi_sweep(tk, st, nF, op.vals, op.cols, op.Dinv, om, r, nullptr, t1);
    launch_jacobi_sweep(tk, st, nF, op.vals, op.cols, op.Dinv, om, r, t1, t2);
    launch_residual(tk, st, nF, op.vals, op.cols, r, t2, t3);
  }
  double* b0 = op.levels.empty() ? op.cb : op.levels[0].b;
  double* x0 = op.levels.empty() ? op.cx : op.levels[0].x;
  {
    Timed tm(prof, KC_AMG);  // the whole coarse correction, transfers included
    launch_csr_spmv(st, op.Rt, t3, b0, 0.0);
    vcycle(op, 0);
    launch_csr_spmv(st, op.Pt, x0, t2, 1.0);
  }
  Timed tm(prof, KC_SMOOTH);
  launch_jacobi_sweep(tk, st, nF, op.vals, op.cols, op.Dinv, om, r, t2, t1);
  launch_jacobi_sweep(tk, st, nF, op.vals, op.cols, op.Dinv, om, r, t1, z);
}

// Remove from a trace vector its component along the null vector of the
// condensed operator (the constant trace: e_0 = 1 on every facet).
void hdg_ctx::project_null(double* v) {
  double* sum = scal + 3 * (prm.max_it_trace + 4);
  launch_dot_sub(st, hm.nF, nf, 0, v, part);
  launch_finish(st, part, kRedBlocks, sum);
  launch_project_const(st, (int)hm.nF, nf, sum, v);
}

// z = B r; the block-Jacobi parts of B do not preserve orthogonality to the
// null vector, so z is projected back: otherwise the iterate drifts along
// the null vector, its norm grows and the attainable residual with it.
void hdg_ctx::precond(TraceOp& op, const double* r, double* z) {
  if (op.mg) mg_apply(op, r, z);
  else launch_blockdiag(tk, st, (int)hm.nF, op.Dinv, r, z);
  project_null(z);
  KCHK();
}

// Records the launches body() issues on the context stream into a graph
// and instantiates it.  Nothing runs during capture.
template <class Body>
hipGraphExec_t hdg_ctx::capture(Body&& body) {
  if (!cap_st) HIPCHK(hipStreamCreateWithFlags(&cap_st, hipStreamNonBlocking));
  hipStream_t keep = st;
  hipGraph_t gr = nullptr;
  HIPCHK(hipStreamBeginCapture(cap_st, hipStreamCaptureModeThreadLocal));
  st = cap_st;
  try {
    body();
  } catch (...) {
    st = keep;
    if (hipStreamEndCapture(cap_st, &gr) == hipSuccess && gr) (void)hipGraphDestroy(gr);
    throw;
  }
  st = keep;
  HIPCHK(hipStreamEndCapture(cap_st, &gr));
  hipGraphExec_t exec = nullptr;
  const hipError_t e = hipGraphInstantiate(&exec, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  HIPCHK(e);
  return exec;
}

// Preconditioned CG on S x = g (g orthogonal to the constant trace), x0 = 0,
// in blocks of kPcgBlock iterations.  A block is the same sequence of
// launches every time (its scalars live in a ring that the block rotates
// first), so it is captured once per operator as a HIP graph and replayed;
// the host then reads the block's residual norms (a converged solve runs
// at most kPcgBlock - 1 extra iterations, which only improve x).  The norms
// leave out the residual's component along the null vector: S 1 vanishes
// only to round-off, so the recursive residual gathers a component of order
// eps |S| |x| along it that no search direction (projected, hence
// orthogonal to it) can remove; on smooth data it can exceed rtol |g|.  With
// kernel timing on, the block runs eagerly so that its launches are timed.
void hdg_ctx::pcg_block(TraceOp& op) {
  const long n = nT;
  const int nF = (int)hm.nF;
  double* rz = scal;  // ring: rz[0..kPcgBlock], pq[0..kPcgBlock), rr[0..kPcgBlock)
  double* pqv = scal + kPcgBlock + 1;
  double* rr = scal + 2 * kPcgBlock + 1;
  launch_copy(st, 1, rz + kPcgBlock, rz);
  for (int b = 0; b < kPcgBlock; ++b) {
    {
      Timed tm(prof, KC_TRACE_SPMV);
      launch_spmv(tk, st, nF, op.vals, op.cols, pp, pq);
    }
    launch_dot(st, n, pp, pq, part);
    launch_finish(st, part, kRedBlocks, pqv + b);
    launch_pcg_update(st, n, nf, rz + b, pqv + b, pp, pq, px, pr, part);
    launch_finish_proj(st, part, kRedBlocks, (double)hm.nF, rr + b);
    precond(op, pr, pz);
    launch_dot(st, n, pr, pz, part);
    launch_finish(st, part, kRedBlocks, rz + b + 1);
    launch_pcg_direction(st, n, rz + b + 1, rz + b, pz, pp);
  }
  KCHK();
}

int hdg_ctx::pcg(TraceOp& op, const double* gin, double* x) {
  static_assert(kPcgBlock <= kPinned, "pinned buffer holds a block of residuals");
  const long n = nT;
  const int maxit = prm.max_it_trace;
  double* rz = scal;
  // the squared residual norms of a block follow at scal + 2 * kPcgBlock + 1
  double* gsq = scal + 3 * kPcgBlock + 2;
  launch_fill(st, n, 0.0, px);
  launch_copy(st, n, gin, pr);
  launch_dot(st, n, pr, nullptr, part);
  launch_finish(st, part, kRedBlocks, gsq);
  const double gnorm = std::sqrt(read_scalar(gsq));
  if (gnorm == 0.0) {
    launch_fill(st, n, 0.0, x);
    return 0;
  }
  if (!op.mg && n <= kSmallTrace) return pcg_small(op, gin, gnorm, x);
  precond(op, pr, pz);
  launch_dot(st, n, pr, pz, part);
  launch_finish(st, part, kRedBlocks, rz + kPcgBlock);  // the block rotates it to rz[0]
  launch_copy(st, n, pz, pp);
  KCHK();
  const bool graphs = prm.use_graphs && !prof.on;
  if (graphs && !op.pcg_block) op.pcg_block = capture([&] { pcg_block(op); });
  double res = 0.0, best_rz = HUGE_VAL, best_r = HUGE_VAL;
  int it = 0, flat = 0, flat_r = 0;
  while (it < maxit) {
    if (graphs) HIPCHK(hipGraphLaunch(op.pcg_block, st));
    else pcg_block(op);
    // the block's scalars: rz[0..kPcgBlock], pq[0..kPcgBlock), rr[0..kPcgBlock)
    HIPCHK(hipMemcpyAsync(h_pinned, rz, (3 * kPcgBlock + 1) * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    const double* hrz = h_pinned;
    const double* hrr = h_pinned + 2 * kPcgBlock + 1;
    double low = HUGE_VAL, low_rz = HUGE_VAL;
    for (int b = 0; b < kPcgBlock; ++b) {
      res = std::sqrt(hrr[b]);
      if (!(res == res)) throw SolverBreakdown("PCG breakdown (NaN residual)");
      if (res <= prm.rtol_trace * gnorm) {
        launch_copy(st, n, px, x);
        return it + kPcgBlock;
      }
      low = std::min(low, res);
      low_rz = std::min(low_rz, std::fabs(hrz[b + 1]));
    }
    it += kPcgBlock;
    if (low < 0.98 * best_r) {
      best_r = low;
      flat_r = 0;
    } else {
      ++flat_r;
    }
    // Round-off floor: with rtol near eps times the condition number of S
    // (1e-12 against ~3e4 at 64 x 64, k = 3, c = 1, and more at higher k and
    // finer meshes) the recursion can stop improving above rtol on smooth
    // data.  Stalling is judged on r.z, the preconditioned residual norm:
    // r.z gaining less than 1 % (in norm) per block for a window of
    // max(kPcgFlatBlocks, it / 16) blocks (a quarter of the iterations
    // spent so far: a fast multigrid solve that stalls gives up after 12
    // iterations, a slow Jacobi solve with long plateaus waits longer), with
    // the current |r| within the round-off band (floor_band()), ends the
    // solve (counted) instead of running to the cap.  So does |r| itself
    // setting no new 2 % low for that window inside the band (a multigrid
    // solve whose r.z keeps wobbling to new lows while |r| sits at the
    // floor).  Either way the true residual is recomputed and must lie in
    // the band too.
    const int window = std::max(kPcgFlatBlocks, it / 16);
    // the iterate returned is the current one: its own residual must be in the band
    const bool in_band = res <= floor_band() * gnorm;
    if (low_rz < 0.98 * best_rz) {
      best_rz = low_rz;
      flat = 0;
    } else {
      ++flat;
    }
    if (in_band && (flat >= window || flat_r >= window)) {
      launch_copy(st, n, px, x);
      accept_floor(trace_true_residual(op, gin, px) / gnorm, it);
      return it;
    }
  }
  launch_copy(st, n, px, x);
  // at the cap: accepted only with a true residual within 1e2 rtol (a
  // residual that kept wobbling at its round-off floor just above rtol)
  const double tr = trace_true_residual(op, gin, px) / gnorm;
  if (tr <= std::min(1e2 * prm.rtol_trace, floor_band())) {
    accept_floor(tr, it);
    return it;
  }
  cap_reached("PCG on the trace system: " + std::to_string(it) + " iterations without reaching rtol_trace (relative residual " +
              sci(res / gnorm) + ")");
  return it;
}

// Small facet-block-Jacobi systems: the whole solve in one single-workgroup
// launch (launch and synchronisation latency, not bandwidth, bound the
// multi-launch iteration there).  Same stopping rules as pcg().
int hdg_ctx::pcg_small(TraceOp& op, const double* gin, double gnorm, double* x) {
  const double tol = prm.rtol_trace * gnorm, flo = floor_band() * gnorm;
  launch_pcg_small(tk, st, (int)hm.nF, op.vals, op.cols, op.Dinv, gin, px, pr, pz, pp, pq, prm.max_it_trace, tol * tol,
                   flo * flo, kPcgFlatBlocks, small_info);
  KCHK();
  HIPCHK(hipMemcpyAsync(h_pinned, small_info, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
  sync();
  const int its = (int)h_pinned[0];
  const double res = std::sqrt(h_pinned[1]);
  if (!(res == res)) throw SolverBreakdown("PCG breakdown (NaN residual)");
  launch_copy(st, nT, px, x);
  if (h_pinned[3] == 0.0) {
    const double tr = trace_true_residual(op, gin, px) / gnorm;
    if (h_pinned[2] != 0.0 || tr <= std::min(1e2 * prm.rtol_trace, floor_band())) {  // stalled in the band, or at the cap near rtol
      accept_floor(tr, its);
    } else {
      cap_reached("PCG on the trace system: " + std::to_string(its) + " iterations without reaching rtol_trace "
                  "(relative residual " + sci(res / gnorm) + ")");
    }
  }
  return its;
}

// |g - S x| without the component along the constant trace (the norm the
// trace solves stop on), recomputed from x rather than recursively updated
double hdg_ctx::trace_true_residual(TraceOp& op, const double* gin, const double* xv) {
  const double* scr = scal + 3 * (prm.max_it_trace + 4) + 2;
  launch_residual(tk, st, (int)hm.nF, op.vals, op.cols, gin, xv, t3);
  launch_rr_partials(st, nT, nf, t3, part);
  launch_finish_proj(st, part, kRedBlocks, (double)hm.nF, const_cast<double*>(scr));
  KCHK();
  return std::sqrt(read_scalar(scr));
}

void hdg_ctx::solve_trace(double c, const double* Fw, const double* Fpsi, const double* Fmu, double* U, double* pout,
                          double* lout) {
  auto t0 = std::chrono::steady_clock::now();
  TraceOp& op = trace_op(c);
  {
    Timed tm(prof, KC_RHS);
    launch_rhs_condense(k, st, dm, dt, c, prm.tau, op.Pinv, Fw, Fpsi, ycell);
    launch_gather_rhs(k, st, dm, ycell, Fmu, g);
  }
  // compatible right-hand side: no component along the null vector
  project_null(g);
  KCHK();
  const int its = pcg(op, g, lout);
  pcg_iters.push_back(its);
  total_pcg += its;
  ++n_trace_solves;
  const long nb = (hm.nc + kBlock - 1) / kBlock;
  {
    Timed tm(prof, KC_BACKSUB);
    launch_backsub(k, st, dm, dt, c, prm.tau, op.Pinv, Fw, Fpsi, lout, U, pout, part);
  }
  launch_finish_mean(st, part, (int)nb, area, scal + 3 * (prm.max_it_trace + 4) + 1);
  launch_shift_mean(k, st, dm, scal + 3 * (prm.max_it_trace + 4) + 1, pout, lout);
  KCHK();
  sync();
  t_trace += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// BiCGStab on the mass-scaled Step I operator  x - (adt/det) f_im(x) = b,
// in the vectors' type (FP64; in the mixed-precision mode FP32, stopped no
// tighter than kMixedRtolFloor and refined by the FP64 Richardson residual).  An iteration is four launches: v = A p
// (with partials of rh.v), s = r - alpha v (alpha finished there), t = A s
// (with partials of t.s, t.t, rh.s, rh.t), and the x, r, p updates (omega
// and beta finished there, partials of r.r).  Coefficients stay in device
// memory; the host reads a block's slots back after every kBicgBlock
// iterations: the residual r.r of the current iterate, NaNs and breakdown
// flags.  A breakdown (zero divisor) restarts from the current iterate with
// the true residual.
// One block of kBicgBlock iterations on the slot ring bsc[0..kBicgBlock]:
// the block first moves the opening slot (kBicgBlock) to slot 0, iteration
// b uses slot b and opens slot b + 1, and the block ends with r.r of its
// last iterate in slot kBicgBlock - 1.  The same launches every time, so
// the block is captured once per adt as a HIP graph and replayed.
void hdg_ctx::bicgstab_block(double adt) {
  KrylovBuf& B = kd;
  const long n = nQ;
  launch_copy(st, BS_STRIDE, bsc + (long)BS_STRIDE * kBicgBlock, bsc);
  // right preconditioning: the operator acts on ph = B p and sh = B s, the
  // residual stays that of the unpreconditioned system
  const void* ph = pc_on ? B.ph : B.p;
  const void* sh = pc_on ? B.sh : B.s;
  for (int b = 0; b < kBicgBlock; ++b) {
    double* sc = bsc + (long)BS_STRIDE * b;
    if (pc_on) pc_apply(B.p, B.ph);
    {
      Timed tm(prof, KC_APPLY_OP);
      launch_apply_soa(k, st, s1, 1, dm, dt, vk, vk32, vbeta, prm.alpha, adt, ph, B.rh, B.v, part, nullptr, kx32);
    }
    {
      Timed tm(prof, KC_VECTOR);
      launch_bicg_s(st, n, apply_soa_blocks(hm.nc, s1.block), part, sc, B.r, B.v, B.s, kx32);
    }
    if (pc_on) pc_apply(B.s, B.sh);
    {
      Timed tm(prof, KC_APPLY_OP);
      launch_apply_soa(k, st, s1, pc_on ? 3 : 2, dm, dt, vk, vk32, vbeta, prm.alpha, adt, sh, B.rh, B.t, kpart,
                       B.s, kx32);
    }
    {
      Timed tm(prof, KC_VECTOR);
      launch_bicg_xrp(st, n, apply_soa_blocks(hm.nc, s1.block), kpart, sc, B.s, B.t, B.v, ph, sh, B.x, B.r, B.p,
                      part, kx32);
    }
  }
  launch_finish(st, part, kVecBlocks, bsc + (long)BS_STRIDE * (kBicgBlock - 1) + BS_RR);
  KCHK();
}

int hdg_ctx::bicgstab(double adt, const double* b_aos, double* x_aos) {
  KrylovBuf& B = kd;
  static_assert(BS_STRIDE * kBicgBlock <= kPinned, "pinned buffer holds a block of slots");
  const long n = nQ;
  const int maxit = prm.max_it_velocity;
  // FP32 arithmetic cannot reach the tolerances of FP64: the mixed mode's
  // Step I stops no tighter than kMixedRtolFloor (the FP64 Richardson
  // residual of Algorithm 2 refines the stage)
  const double rtol = kx32 ? std::max(prm.rtol_velocity, kMixedRtolFloor) : prm.rtol_velocity;
  double* open = bsc + (long)BS_STRIDE * kBicgBlock;  // slot opening the next block
  launch_to_soa(k, st, dm, 0, b_aos, B.b, kx32);
  launch_vdot(st, n, B.b, nullptr, part, kx32);
  launch_finish(st, part, kRedBlocks, bsc);
  const double bnorm = std::sqrt(read_scalar(bsc));
  if (!(bnorm == bnorm)) throw SolverBreakdown("BiCGStab: non-finite right-hand side");
  if (bnorm == 0.0) {
    launch_fill(st, nQ, 0.0, x_aos);
    return 0;
  }
  pc_prepare(adt);
  const bool graphs = prm.use_graphs && !prof.on;
  hipGraphExec_t* exec = nullptr;
  if (graphs) {
    if (bicg_graphs.size() >= 16 && !bicg_graphs.count(adt)) {  // time step changes: drop the old ones
      for (auto& g : bicg_graphs)
        if (g.second) (void)hipGraphExecDestroy(g.second);
      bicg_graphs.clear();
    }
    exec = &bicg_graphs[adt];
  }
  launch_vfill(st, n, 0.0, B.x, kx32);
  int it = 0, restarts = 0;
  bool restart = true;
  while (true) {
    if (restart) {
      if (it == 0) {
        launch_vcopy(st, n, B.b, B.r, kx32);
      } else {  // true residual of the current iterate
        {
          Timed tm(prof, KC_APPLY_OP);
          launch_apply_soa(k, st, s1, 0, dm, dt, vk, vk32, vbeta, prm.alpha, adt, B.x, nullptr, B.t, nullptr,
                           nullptr, kx32);
        }
        launch_vcopy(st, n, B.b, B.r, kx32);
        launch_vaxpby(st, n, -1.0, B.t, 1.0, B.r, kx32);
        ++bicg_restarts;
        if (++restarts > 50) throw SolverBreakdown("BiCGStab: too many restarts");
      }
      launch_vcopy(st, n, B.r, B.p, kx32);
      launch_vcopy(st, n, B.r, B.rh, kx32);
      launch_bicg_init(st, open);
      launch_vdot(st, n, B.rh, nullptr, part, kx32);
      launch_finish(st, part, kRedBlocks, open + BS_RHO);
      KCHK();
      restart = false;
    }
    if (graphs) {
      if (!*exec) *exec = capture([&] { bicgstab_block(adt); });
      HIPCHK(hipGraphLaunch(*exec, st));
    } else {
      bicgstab_block(adt);
    }
    it += kBicgBlock;
    HIPCHK(hipMemcpyAsync(h_pinned, bsc, (size_t)BS_STRIDE * kBicgBlock * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    const double rr = h_pinned[BS_STRIDE * (kBicgBlock - 1) + BS_RR];
    if (!(rr == rr)) throw SolverBreakdown("BiCGStab breakdown (NaN residual); the result is invalid");
    if (std::sqrt(rr) <= rtol * bnorm) {
      // the recursive residual says converged: check the true one b - A x
      // (in B.r from here on); more than 10 rtol away continues from it
      {
        Timed tm(prof, KC_APPLY_OP);
        launch_apply_soa(k, st, s1, 0, dm, dt, vk, vk32, vbeta, prm.alpha, adt, B.x, nullptr, B.t, nullptr,
                         nullptr, kx32);
      }
      launch_vcopy(st, n, B.b, B.r, kx32);
      launch_vaxpby(st, n, -1.0, B.t, 1.0, B.r, kx32);
      double* tslot = bsc + (long)BS_STRIDE * (kBicgBlock + 1);
      launch_vdot(st, n, B.r, nullptr, part, kx32);
      launch_finish(st, part, kRedBlocks, tslot);
      const double tr = std::sqrt(read_scalar(tslot)) / bnorm;
      if (!(tr == tr)) throw SolverBreakdown("BiCGStab: non-finite true residual");
      velocity_true_max = std::max(velocity_true_max, tr);
      if (tr <= 10.0 * rtol) break;
      if (it >= maxit) {
        cap_reached("BiCGStab (Step I): " + std::to_string(it) + " iterations; true relative residual " + sci(tr) +
                    " above 10 rtol_velocity");
        break;
      }
      ++velocity_true_restarts;
      restart = true;
      continue;
    }
    if (it >= maxit) {
      cap_reached("BiCGStab (Step I): " + std::to_string(it) + " iterations without reaching rtol_velocity "
                  "(relative residual " + sci(std::sqrt(rr) / bnorm) + ", " +
                  std::to_string(restarts) + " restarts)");
      break;
    }
    bool flag = false;
    for (int b = 0; b < kBicgBlock; ++b) flag |= h_pinned[BS_STRIDE * b + BS_FLAG] != 0.0;
    if (flag) restart = true;
  }
  launch_to_aos(k, st, dm, B.x, x_aos, kx32);
  KCHK();
  return it;
}

// IDR(s) with bi-orthogonalisation on the mass-scaled Step I operator.  The
// shadow space is spanned by s counter-based random vectors, orthonormalised
// once.  Each inner step needs one operator application and one pass of s
// dot products; the small triangular systems are solved on the host.  The
// dimension-reduction step uses omega from the local minimal residual,
// enlarged when the angle between t and r is small (|cos| < 0.7).
int hdg_ctx::idrs(double adt, const double* b, double* x) {
  const long n = nQ;
  const int s = prm.idr_s;
  const int maxit = prm.max_it_velocity;
  if (!iP) {
    iP = dalloc<double>((long)s * n);
    iG = dalloc<double>((long)s * n);
    iU = dalloc<double>((long)s * n);
    ired = dalloc<double>(kIdrMax + 8);
    for (int j = 0; j < s; ++j) {  // modified Gram-Schmidt
      double* pj = iP + (long)j * n;
      launch_random(st, n, 0x5eedull + 7919ull * j, pj);
      for (int i = 0; i < j; ++i) {
        launch_dot(st, n, iP + (long)i * n, pj, part);
        launch_finish(st, part, kRedBlocks, ired);
        const double d = read_scalar(ired);
        launch_axpby(st, n, -d, iP + (long)i * n, 1.0, pj);
      }
      launch_dot(st, n, pj, nullptr, part);
      launch_finish(st, part, kRedBlocks, ired);
      const double nrm = std::sqrt(read_scalar(ired));
      launch_axpby(st, n, 0.0, pj, 1.0 / nrm, pj);
    }
    KCHK();
  }
  launch_fill(st, n, 0.0, x);
  launch_copy(st, n, b, br);
  launch_fill(st, (long)s * n, 0.0, iG);
  launch_fill(st, (long)s * n, 0.0, iU);
  launch_dot(st, n, br, nullptr, part);
  launch_finish(st, part, kRedBlocks, ired);
  const double bnorm = std::sqrt(read_scalar(ired));
  if (bnorm == 0.0) return 0;
  const double tol = prm.rtol_velocity * bnorm;
  double M[kIdrMax][kIdrMax] = {}, f[kIdrMax], m[kIdrMax];
  for (int i = 0; i < s; ++i) M[i][i] = 1.0;
  double om = 1.0, normr = bnorm;
  int it = 0;
  auto read_vec = [&](int cnt, double* out) {
    HIPCHK(hipMemcpyAsync(h_pinned, ired, cnt * sizeof(double), hipMemcpyDeviceToHost, st));
    sync();
    for (int i = 0; i < cnt; ++i) out[i] = h_pinned[i];
  };
  while (normr > tol && it < maxit) {
    launch_multidot(st, n, s, iP, br, part, ired);
    read_vec(s, f);
    for (int kk = 0; kk < s; ++kk) {
      IdrCoef c{};
      for (int i = kk; i < s; ++i) {  // M(kk:s, kk:s) c = f(kk:s), lower triangular
        double v = f[i];
        for (int j = kk; j < i; ++j) v -= M[i][j] * c.v[j - kk];
        c.v[i - kk] = v / M[i][i];
      }
      launch_idr_u(st, n, kk, s, c, om, br, iG, iU);
      {
        Timed tm(prof, KC_APPLY_OP);
        launch_apply(k, st, 0, dm, dt, adv, prm.alpha, adt, iU + (long)kk * n, nullptr, nullptr, nullptr,
                     iG + (long)kk * n);
      }
      launch_multidot(st, n, s, iP, iG + (long)kk * n, part, ired);
      read_vec(s, m);
      IdrCoef al{};
      for (int i = 0; i < kk; ++i) {  // bi-orthogonalise against P_0..P_{kk-1}
        double v = m[i];
        for (int j = 0; j < i; ++j) v -= M[i][j] * al.v[j];
        al.v[i] = v / M[i][i];
      }
      for (int i = kk; i < s; ++i) {
        double v = m[i];
        for (int j = 0; j < kk; ++j) v -= al.v[j] * M[i][j];
        M[i][kk] = v;
      }
      if (M[kk][kk] == 0.0) throw SolverBreakdown("IDR(s) breakdown (M_kk = 0)");
      const double beta = f[kk] / M[kk][kk];
      launch_idr_update(st, n, kk, al, beta, iG, iU, br, x, part);
      launch_finish(st, part, kRedBlocks, ired);
      KCHK();
      normr = std::sqrt(read_scalar(ired));
      if (!(normr == normr)) throw SolverBreakdown("IDR(s) breakdown (NaN residual)");
      ++it;
      if (normr <= tol || it >= maxit) break;
      for (int i = kk + 1; i < s; ++i) f[i] -= beta * M[i][kk];
    }
    if (normr <= tol || it >= maxit) break;
    {
      Timed tm(prof, KC_APPLY_OP);
      launch_apply(k, st, 0, dm, dt, adv, prm.alpha, adt, br, nullptr, nullptr, nullptr, bt);
    }
    launch_dot2(st, n, bt, br, bt, part2);
    launch_finish2(st, part2, ired);
    double tr_tt[2];
    read_vec(2, tr_tt);
    if (!(tr_tt[1] > 0.0)) throw SolverBreakdown("IDR(s) breakdown (t = 0)");
    om = tr_tt[0] / tr_tt[1];
    const double rho = std::fabs(tr_tt[0]) / (std::sqrt(tr_tt[1]) * normr);
    if (rho < 0.7) om *= 0.7 / rho;
    if (om == 0.0) throw SolverBreakdown("IDR(s) breakdown (omega = 0)");
    launch_idr_reduce(st, n, om, bt, br, x, part);
    launch_finish(st, part, kRedBlocks, ired);
    KCHK();
    normr = std::sqrt(read_scalar(ired));
    if (!(normr == normr)) throw SolverBreakdown("IDR(s) breakdown (NaN residual)");
    ++it;
  }
  if (normr > tol)
    cap_reached("IDR(s) (Step I): " + std::to_string(it) + " iterations without reaching rtol_velocity (relative "
                "residual " + std::to_string(normr / bnorm) + ")");
  return it;
}

// Pressure reconstruction at the current time (eq.
// (pressure_reconstruction_compact)): psi-data Div_c(psi, (Q.grad)Q - f) and,
// with forcing, wall data -<mu, n.f>.
void hdg_ctx::reconstruct(const double* Qin, double* pout, double* lout) {
  const double fs = forced ? f_scale(time) : 0.0;
  {
    Timed tm(prof, KC_RECON);
    launch_recon_rhs(k, st, dm, dt, Qin, forced ? f_cell : nullptr, forced ? f_fac : nullptr, fs, fpsi);
    if (forced) launch_axpby(st, nT, fs, f_wall, 0.0, f_tmp);
    KCHK();
  }
  solve_trace(1.0, nullptr, fpsi, forced ? f_tmp : nullptr, Ut, pout, lout);
}

// Algorithm 2 for one stage: (Q, p, lam) hold the iterate on entry and exit
void hdg_ctx::richardson(double adt, const double* r, double* Qv, double* pv, double* lv) {
  for (int it = 0; it < prm.n_richardson; ++it) {
    auto t0 = std::chrono::steady_clock::now();
    {
      Timed tm(prof, KC_APPLY_RES);
      launch_apply(k, st, 1, dm, dt, adv, prm.alpha, adt, Qv, r, pv, lv, dr);  // delta r / det
      KCHK();
    }
    const int its = velocity_solve(adt, dr, Qbar);  // Step I
    bicg_iters.push_back(its);
    total_bicg += its;
    ++n_velocity_solves;
    if (prm.step2_reading == HDG_STEP2_PRINTED) {
      Timed tm(prof, KC_DIV);
      launch_div(k, st, dm, dt, Qbar, -1.0 / adt, fpsi);  // Step II data
      KCHK();
    }
    sync();
    t_velocity += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (prm.step2_reading == HDG_STEP2_PRINTED) {
      solve_trace(1.0, nullptr, fpsi, nullptr, dQ, dp, dl);
      // Step III
      launch_axpby(st, nQ, 1.0, Qbar, 1.0, Qv);
      launch_axpby(st, nQ, adt, dQ, 1.0, Qv);
    } else {
      // reading B: the mixed solve of the stage operator H_adt with w-data
      // (Qbar, w) and the iterate's constraint residual -Gamma(Q, p, lam),
      // whose solution is added to the iterate
      launch_mass(k, st, dm, 1.0, Qbar, Ut);
      launch_gamma(k, st, dm, dt, prm.tau, -1.0, Qv, pv, lv, fpsi, ycell, fmu);
      KCHK();
      solve_trace(adt, Ut, fpsi, fmu, dQ, dp, dl);
      launch_axpby(st, nQ, 1.0, dQ, 1.0, Qv);
    }
    launch_axpby(st, nP, 1.0, dp, 1.0, pv);
    launch_axpby(st, nT, 1.0, dl, 1.0, lv);
    KCHK();
  }
}

// Algorithm 1
// One step of Algorithm 1 is begin_step, stages 1..s-1 and finish_step; the
// pieces keep their state in the stage arrays, so hdg_advance_stages can stop
// between stages.  Q, p, lam change only in finish_step.
void hdg_ctx::step(double dtv) {
  begin_step(dtv);
  while (pend_stage != 0) stage_once();
}

void hdg_ctx::begin_step(double dtv) {
  double* MQn = stMQ[0];
  launch_mass(k, st, dm, 1.0, Q, MQn);
  launch_copy(st, nQ, Q, stQ[0]);
  launch_copy(st, nP, p, stP[0]);
  launch_copy(st, nT, lam, stL[0]);
  pend_stage = 1;
  pend_dt = dtv;
}

// implicit stage pend_stage; after the last one, the final projection
void hdg_ctx::stage_once() {
  const Tableau tab = make_tableau(prm.imex);
  const int s = tab.s;
  const double dtv = pend_dt;
  const int i = pend_stage;
  double* MQn = stMQ[0];
  {
    // stage residual r_i, eq. (imex_residual)
    launch_copy(st, nQ, MQn, stR[i]);
    for (int j = 1; j < i; ++j) {
      const double w = tab.Aim[i][j] / tab.Aim[j][j];
      launch_axpby(st, nQ, w, stMQ[j], 1.0, stR[i]);
      launch_axpby(st, nQ, -w, stR[j], 1.0, stR[i]);
    }
    if (forced) {  // dt sum_{j<i} a^ex_ij f^ex(t + c_j dt)
      double w = 0.0;
      for (int j = 0; j < i; ++j) w += tab.Aex[i][j] * f_scale(time + abscissa(tab, j) * dtv);
      launch_axpby(st, nQ, dtv * w, f_dual, 1.0, stR[i]);
    }
    {
      Timed tm(prof, KC_BDM);
      launch_bdm(k, st, dm, dt, stQ[i - 1], Qs);
      prepare_step1(Qs);
    }
    launch_copy(st, nQ, stQ[i - 1], stQ[i]);
    launch_copy(st, nP, stP[i - 1], stP[i]);
    launch_copy(st, nT, stL[i - 1], stL[i]);
    KCHK();
    richardson(tab.Aim[i][i] * dtv, stR[i], stQ[i], stP[i], stL[i]);
    launch_mass(k, st, dm, 1.0, stQ[i], stMQ[i]);
  }
  if (++pend_stage == s) finish_step();
}

void hdg_ctx::finish_step() {
  const Tableau tab = make_tableau(prm.imex);
  const int s = tab.s;
  const double dtv = pend_dt;
  double* MQn = stMQ[0];
  pend_stage = 0;  // Q, p, lam (and the tracer) are overwritten from here on
  if (tracer_on) tracer_step(dtv);
  // final residual and projection
  double* rn = dr;
  launch_copy(st, nQ, MQn, rn);
  for (int i = 1; i < s; ++i) {
    const double w = tab.bim[i] / tab.Aim[i][i];
    launch_axpby(st, nQ, w, stMQ[i], 1.0, rn);
    launch_axpby(st, nQ, -w, stR[i], 1.0, rn);
  }
  if (forced) {  // dt sum_j b^ex_j f^ex(t + c_j dt), eq. (final_residual)
    double w = 0.0;
    for (int j = 0; j < s; ++j) w += tab.bex[j] * f_scale(time + abscissa(tab, j) * dtv);
    launch_axpby(st, nQ, dtv * w, f_dual, 1.0, rn);
  }
  KCHK();
  time += dtv;  // the final projection and the reconstruction belong to t^{n+1}
  // Final projection (Algorithm 1, eq. (final_update)) in increment form:
  // with Q^{n+1} = Q_{s-1} + dQ, H_c(Q^{n+1}, dp, dl) = (r^{n+1}, 0, 0) is
  // H_c(dQ, dp, dl) = (r^{n+1} - M Q_{s-1}, -Gamma(Q_{s-1}, 0, 0)), the same
  // system in exact arithmetic; the trace solve's error then scales with the
  // increment rather than with the state.
  launch_mass(k, st, dm, -1.0, stQ[s - 1], Ut);
  launch_axpby(st, nQ, 1.0, Ut, 1.0, rn);
  launch_gamma(k, st, dm, dt, prm.tau, -1.0, stQ[s - 1], nullptr, nullptr, fpsi, ycell, fmu);
  KCHK();
  solve_trace(dtv * tab.bim[s - 1], rn, fpsi, fmu, dQ, dp, dl);
  launch_copy(st, nQ, stQ[s - 1], Q);
  launch_axpby(st, nQ, 1.0, dQ, 1.0, Q);
  if (prm.pressure_update == HDG_PRESSURE_RECONSTRUCT) {
    reconstruct(Q, p, lam);
  } else {
    launch_copy(st, nP, stP[s - 1], p);
    launch_copy(st, nT, stL[s - 1], lam);
    launch_axpby(st, nP, 1.0, dp, 1.0, p);
    launch_axpby(st, nT, 1.0, dl, 1.0, lam);  // both terms have int p = 0 already
    KCHK();
  }
  sync();
}


// ------------------------------------------------------------------ tracer
// CG_{k+1}: nodal Lagrange basis on the equispaced points of the reference
// triangle (vertices, then the m-1 inner points of each local edge from its
// first to its second vertex, then the inner points), glued along the
// topological vertices and facets; inner edge points are numbered along the
// facet parameter (lower topological vertex first).
void hdg_ctx::cg_setup() {
  if (cg.ready) return;
  const int m = k + 1;
  const long nc = hm.nc, nF = hm.nF, nvt = hm.nvt;
  const int nint = (m - 1) * (m - 2) / 2;
  std::vector<double> px, py;
  const double V[3][2] = {{0.0, 0.0}, {1.0, 0.0}, {0.0, 1.0}};
  for (int v = 0; v < 3; ++v) { px.push_back(V[v][0]); py.push_back(V[v][1]); }
  for (int f = 0; f < 3; ++f)
    for (int r = 1; r < m; ++r) {
      px.push_back(V[FA[f]][0] + (V[FB[f]][0] - V[FA[f]][0]) * r / m);
      py.push_back(V[FA[f]][1] + (V[FB[f]][1] - V[FA[f]][1]) * r / m);
    }
  for (int j = 1; j < m; ++j)
    for (int i = 1; i < m - j; ++i) { px.push_back((double)i / m); py.push_back((double)j / m); }
  if ((int)px.size() != ns) throw std::runtime_error("CG node count mismatch");
  // T = Vn^-1, Vn[a][s] = phi_s(node a): Gauss-Jordan with partial pivoting
  std::vector<double> A((size_t)ns * ns), T((size_t)ns * ns, 0.0);
  for (int a = 0; a < ns; ++a) dubiner_eval(m, px[a], py[a], &A[(size_t)a * ns], nullptr, nullptr);
  for (int i = 0; i < ns; ++i) T[(size_t)i * ns + i] = 1.0;
  for (int c = 0; c < ns; ++c) {
    int piv = c;
    for (int r = c + 1; r < ns; ++r)
      if (std::fabs(A[(size_t)r * ns + c]) > std::fabs(A[(size_t)piv * ns + c])) piv = r;
    for (int j = 0; j < ns; ++j) {
      std::swap(A[(size_t)c * ns + j], A[(size_t)piv * ns + j]);
      std::swap(T[(size_t)c * ns + j], T[(size_t)piv * ns + j]);
    }
    const double d = A[(size_t)c * ns + c];
    for (int j = 0; j < ns; ++j) { A[(size_t)c * ns + j] /= d; T[(size_t)c * ns + j] /= d; }
    for (int r = 0; r < ns; ++r) {
      if (r == c) continue;
      const double f = A[(size_t)r * ns + c];
      if (f == 0.0) continue;
      for (int j = 0; j < ns; ++j) { A[(size_t)r * ns + j] -= f * A[(size_t)c * ns + j]; T[(size_t)r * ns + j] -= f * T[(size_t)c * ns + j]; }
    }
  }
  // T now holds Vn^-1 with rows indexed by s and columns by the node a
  const long N = nvt + nF * (m - 1) + nc * nint;
  if (N > INT32_MAX / 2) throw ArgError("CG space too large");
  std::vector<int32_t> l2g((size_t)nc * ns);
  for (long e = 0; e < nc; ++e) {
    int a = 0;
    for (int v = 0; v < 3; ++v) l2g[e * ns + a++] = hm.vtopo[hm.cells[3 * e + v]];
    for (int f = 0; f < 3; ++f) {
      const long F = hm.cf_facet[f * nc + e];
      const bool flip = hm.cf_flip[f * nc + e] != 0;
      for (int r = 0; r < m - 1; ++r) l2g[e * ns + a++] = (int32_t)(nvt + F * (m - 1) + (flip ? m - 2 - r : r));
    }
    for (int c = 0; c < nint; ++c) l2g[e * ns + a++] = (int32_t)(nvt + nF * (m - 1) + e * nint + c);
  }
  // mass matrix: M_K = det_K T^T T (the Dubiner mass is det_K I)
  std::vector<double> G((size_t)ns * ns, 0.0);
  for (int x = 0; x < ns; ++x)
    for (int y = 0; y < ns; ++y)
      for (int s = 0; s < ns; ++s) G[(size_t)x * ns + y] += T[(size_t)s * ns + x] * T[(size_t)s * ns + y];
  std::vector<std::pair<int64_t, double>> trip;
  trip.reserve((size_t)nc * ns * ns);
  for (long e = 0; e < nc; ++e) {
    const double det = hm.geo[(size_t)G_DET * nc + e];
    for (int x = 0; x < ns; ++x)
      for (int y = 0; y < ns; ++y)
        trip.push_back({(int64_t)l2g[e * ns + x] * N + l2g[e * ns + y], det * G[(size_t)x * ns + y]});
  }
  std::sort(trip.begin(), trip.end(), [](const auto& u, const auto& v) { return u.first < v.first; });
  Csr M;
  M.nrows = M.ncols = N;
  M.ptr.assign(N + 1, 0);
  for (size_t i = 0; i < trip.size();) {
    size_t j = i;
    double v = 0.0;
    while (j < trip.size() && trip[j].first == trip[i].first) v += trip[j++].second;
    const int64_t row = trip[i].first / N, col = trip[i].first % N;
    M.idx.push_back((int32_t)col);
    M.val.push_back(v);
    M.ptr[row + 1]++;
    i = j;
  }
  for (long r = 0; r < N; ++r) M.ptr[r + 1] += M.ptr[r];
  std::vector<double> dinv(N, 0.0);
  for (long r = 0; r < N; ++r)
    for (int32_t q = M.ptr[r]; q < M.ptr[r + 1]; ++q)
      if (M.idx[q] == r) dinv[r] = 1.0 / M.val[q];
  // incidences of each unknown, for the gathered right-hand side
  std::vector<int32_t> gptr(N + 1, 0), ginc((size_t)nc * ns);
  for (size_t i = 0; i < l2g.size(); ++i) gptr[l2g[i] + 1]++;
  for (long r = 0; r < N; ++r) gptr[r + 1] += gptr[r];
  {
    std::vector<int32_t> pos(gptr.begin(), gptr.end() - 1);
    for (size_t i = 0; i < l2g.size(); ++i) ginc[pos[l2g[i]]++] = (int32_t)i;
  }
  cg.N = (int)N;
  cg.l2g = upload(l2g);
  cg.gptr = upload(gptr);
  cg.ginc = upload(ginc);
  cg.T = upload(T);
  cg.M.n = (int)N;
  cg.M.ptr = upload(M.ptr);
  cg.M.idx = upload(M.idx);
  cg.M.val = upload(M.val);
  cg.dinv = upload(dinv);
  for (double** v : {&cg.b, &cg.u, &cg.r, &cg.z, &cg.p, &cg.w}) *v = dalloc<double>(N);
  cg.sc = dalloc<double>(4);
  sync();
  cg.ready = true;
}

// Uout = P_CG(Qin): per component, Jacobi-PCG on the CG mass matrix to a
// relative residual of 1e-14, then the nodal values back to Dubiner form.
void hdg_ctx::cg_project(const double* Qin, double* Uout) {
  cg_setup();
  const long N = cg.N;
  for (int comp = 0; comp < 2; ++comp) {
    launch_cg_rhs(st, cg.N, cg.gptr, cg.ginc, ns, cg.T, dm, Qin, comp, cg.b);
    launch_fill(st, N, 0.0, cg.u);
    launch_copy(st, N, cg.b, cg.r);
    launch_csr_jacobi(st, cg.M, cg.dinv, 1.0, cg.r, nullptr, cg.z);
    launch_copy(st, N, cg.z, cg.p);
    launch_dot(st, N, cg.b, nullptr, part);
    launch_finish(st, part, kRedBlocks, cg.sc);
    const double bn = std::sqrt(read_scalar(cg.sc));
    launch_dot(st, N, cg.r, cg.z, part);
    launch_finish(st, part, kRedBlocks, cg.sc);
    double rz = read_scalar(cg.sc);
    int it = 0;
    for (; bn > 0.0 && it < 1000; ++it) {
      launch_csr_spmv(st, cg.M, cg.p, cg.w, 0.0);
      launch_dot(st, N, cg.p, cg.w, part);
      launch_finish(st, part, kRedBlocks, cg.sc);
      const double pw = read_scalar(cg.sc);
      if (!(pw > 0.0)) break;
      const double alpha = rz / pw;
      launch_axpby(st, N, alpha, cg.p, 1.0, cg.u);
      launch_axpby(st, N, -alpha, cg.w, 1.0, cg.r);
      launch_dot(st, N, cg.r, nullptr, part);
      launch_finish(st, part, kRedBlocks, cg.sc);
      if (std::sqrt(read_scalar(cg.sc)) <= 1e-14 * bn) { ++it; break; }
      launch_csr_jacobi(st, cg.M, cg.dinv, 1.0, cg.r, nullptr, cg.z);
      launch_dot(st, N, cg.r, cg.z, part);
      launch_finish(st, part, kRedBlocks, cg.sc);
      const double rzn = read_scalar(cg.sc);
      launch_axpby(st, N, 1.0, cg.z, rzn / rz, cg.p);
      rz = rzn;
    }
    cg.last_its = it;
    launch_cg_to_dg(st, hm.nc, ns, cg.T, cg.l2g, cg.u, comp, Uout);
  }
  KCHK();
}

void hdg_ctx::tracer_alloc() {
  if (trq) return;
  trq = dalloc<double>(nP);
  trq_tmp = dalloc<double>(nP);
  Ucg = dalloc<double>(nQ);
  for (int i = 0; i < make_tableau(prm.imex).s; ++i) trR[i] = dalloc<double>(nP);
}

// eqs. (advection_update_stages), (advection_update_final): stage tracer
// values with the explicit tableau and the stage velocities Q_j of this step
void hdg_ctx::tracer_step(double dtv) {
  const Tableau tab = make_tableau(prm.imex);
  const int s = tab.s;
  for (int j = 0; j < s; ++j) {
    bool needed = tab.bex[j] != 0.0;
    for (int i = j + 1; i < s; ++i) needed = needed || tab.Aex[i][j] != 0.0;
    if (!needed) continue;
    launch_copy(st, nP, trq, trq_tmp);
    for (int i = 0; i < j; ++i)
      if (tab.Aex[j][i] != 0.0) launch_axpby(st, nP, dtv * tab.Aex[j][i], trR[i], 1.0, trq_tmp);
    cg_project(stQ[j], Ucg);
    launch_tracer_rate(k, st, dm, dt, Ucg, trq_tmp, trR[j]);
  }
  for (int j = 0; j < s; ++j)
    if (tab.bex[j] != 0.0) launch_axpby(st, nP, dtv * tab.bex[j], trR[j], 1.0, trq);
  KCHK();
}

// ======================================================================= ABI

// Device bytes a context holds after its first step, from the allocations
// made in setup(), per trace operator (one per distinct c: the stage
// coefficients a_ii dt, the final b^im_{s-1} dt and the reconstruction's
// c = 1) and by the multigrid hierarchy (P1 coarse operator and its
// aggregation levels, estimated as 2x the first level).  The transient
// condensation buffer of an operator build is reported separately.
static void estimate_footprint(const hdg::HostMesh& m, const hdg::RefTables& rt, const hdg_params& prm, double dtv,
                               int64_t* held, int64_t* transient) {
  const double nc = (double)m.nc, nF = (double)m.nF, nvt = (double)m.nvt;
  const double ns = rt.ns, np = rt.np, nf = rt.nf, nqc = rt.nqc, nqf = rt.nqf;
  const double nu = 2 * ns, nlam = 3 * nf, nc32 = std::ceil(nc / 32.0) * 32.0;
  const double nQ = nc * nu, nP = nc * np, nT = nF * nf;
  const Tableau tab = make_tableau(prm.imex);
  const double s = tab.s;
  const double blocks = (double)apply_soa_blocks((long)m.nc, prm.step1_block);
  double b = 0.0;
  // mesh (geometry, connectivity, packed neighbours) and reference tables
  b += 8.0 * kDGeo * nc + 4.0 * 5 * 3 * nc + 4.0 * 4 * nF;
  for (const std::vector<double>* v : {&rt.Bu, &rt.Gux, &rt.Guy, &rt.Bp, &rt.Gpx, &rt.Gpy, &rt.cq_w, &rt.FBu, &rt.FGux,
                                       &rt.FGuy, &rt.FBp, &rt.fq_w, &rt.MU, &rt.NUB, &rt.TRU, &rt.Dx, &rt.Dy, &rt.Rx, &rt.Ry,
                                       &rt.Chat, &rt.That, &rt.Ehat, &rt.CC, &rt.KDD, &rt.CD, &rt.BDMinv, &rt.NED})
    b += 8.0 * v->size();
  // work vectors: cell duals, trace vectors, Krylov and stage vectors
  b += 8.0 * (nc * nlam + nT * (12 + s) + nQ * (18 + 2 * s) + nP * (3 + s));
  const bool x32 = prm.precision == HDG_MIXED;  // the 8 Step I Krylov vectors in FP32
  if (x32) b -= 4.0 * 8 * nQ;
  b += 8.0 * ((double)kRedBlocks * kIdrMax + 2.0 * kRedBlocks + 3.0 * (prm.max_it_trace + 4) + 16 +
              (double)BS_STRIDE * std::max(prm.max_it_velocity + 6, 10) + 2 * (4 * blocks + 16));
  // Step I data: the field at the cell points, upwind weights, residual-kernel advection data
  b += 2 * nqc * nc32 * (x32 ? 4.0 : 8.0) + (x32 ? 4.0 : 8.0) * 3 * nqf * nc32 + 8.0 * nc * (2 * nqc + 3 * nqf);
  if (prm.idr_s > 0) b += 8.0 * (3.0 * prm.idr_s * nQ + kIdrMax + 8);
  // Step I preconditioner: two direction vectors, the cell blocks and the patch inverses
  if (prm.step1_precond == 1 && prm.idr_s == 0)
    b += (x32 ? 4.0 : 8.0) * 2 * nQ + 8.0 * nc * nu * nu + 2.0 * (double)pc_entries(rt.k, (long)m.nc) +
         (x32 ? 4.0 : 8.0) * (double)pc_scratch(rt.k, (long)m.nc);
  // trace operators
  std::set<double> cs = {1.0, tab.bim[tab.s - 1] * dtv};
  for (int i = 1; i < tab.s; ++i) cs.insert(tab.Aim[i][i] * dtv);
  double op = 8.0 * (nc * np * np + 5 * nF * nf * nf + nF * nf * nf) + 4.0 * 5 * nF;
  if (prm.trace_solver == HDG_TRACE_MG_PCG) {
    const double transfer = 2 * (4.0 * (nT + 1) + 12.0 * 4 * nF);        // P1 prolongation and restriction
    const double level0 = 12.0 * 9 * nvt + 4.0 * nvt + 2 * (12.0 * 3 * nvt + 4.0 * nvt) + 8.0 * 5 * nvt;
    double nco = nvt;  // coarsest level: aggregates of about six P1 vertices until at most 200 remain
    while (nco > 200) nco = std::ceil(nco / 6.0);
    op += transfer + 2.0 * level0 + 8.0 * nco * (nco + 2);
  }
  b += cs.size() * op;
  *held = (int64_t)(1.02 * b) + 65536;  // margin for the small buffers not itemised here
  *transient = (int64_t)(8.0 * nc * nlam * nlam);
}

#define API_BEGIN try {
#define API_END(ctxp)                                                   \
  }                                                                     \
  catch (const hdg::OomError& e) { (ctxp)->err = e.what(); return HDG_ERR_OUT_OF_MEMORY; } \
  catch (const hdg::ArgError& e) { (ctxp)->err = e.what(); return HDG_ERR_INVALID_ARG; }   \
  catch (const hdg::SolverBreakdown& e) { (ctxp)->err = e.what(); return HDG_ERR_NOT_CONVERGED; } \
  catch (const std::exception& e) { (ctxp)->err = e.what(); return HDG_ERR_DEVICE; }       \
  return (ctxp)->not_converged ? HDG_ERR_NOT_CONVERGED : HDG_OK;

extern "C" {

void hdg_default_params(hdg_params* p) {
  if (!p) return;
  p->degree = 1;
  p->tau = 1.0;
  p->alpha = 1.0;
  p->delta_up = 1.0;
  p->imex = HDG_ARS222;
  p->n_richardson = 3;
  p->trace_solver = HDG_TRACE_MG_PCG;
  p->rtol_trace = 1e-12;
  p->rtol_velocity = 1e-12;
  p->max_it_trace = 5000;
  p->max_it_velocity = 20000;
  p->pressure_update = HDG_PRESSURE_RECONSTRUCT;
  p->idr_s = 0;
  p->precision = HDG_FP64;
  p->use_graphs = 1;
  p->step1_block = 256;
  p->step1_xcd = 1;
  p->step1_precond = 1;
  p->step2_reading = HDG_STEP2_PRINTED;
  p->step1_precond_lag = 1;
  p->dim = 2;
}

int hdg_create(int64_t nv, const double* coords, int64_t nc, const int32_t* cells, const hdg_params* prm,
               void* stream, hdg_ctx** out) {
  return hdg_create_periodic(nv, coords, nc, cells, nullptr, prm, stream, out);
}

int hdg_create_periodic(int64_t nv, const double* coords, int64_t nc, const int32_t* cells,
                        const int32_t* vertex_rep, const hdg_params* prm, void* stream, hdg_ctx** out) {
  if (!out || !prm) { g_create_error = "null argument"; return HDG_ERR_INVALID_ARG; }
  *out = nullptr;
  if (prm->dim != 2 && prm->dim != 3) { g_create_error = "dim must be 2 or 3"; return HDG_ERR_INVALID_ARG; }
  if (prm->degree < 1 || prm->degree > (prm->dim == 3 ? kMaxDegree3 : kMaxDegree)) {
    g_create_error = prm->dim == 3 ? "degree must be in 1..2 on tetrahedra" : "degree must be in 1..4";
    return HDG_ERR_UNSUPPORTED;
  }
  if (prm->dim == 3 && vertex_rep) {
    g_create_error = "tetrahedra: no periodic meshes";
    return HDG_ERR_UNSUPPORTED;
  }
  if (prm->tau <= 0 || prm->alpha < 0 || prm->delta_up < 0 || prm->n_richardson < 1 || prm->max_it_trace < 1 ||
      prm->max_it_velocity < 1 || !(prm->rtol_trace > 0) || !(prm->rtol_velocity > 0) || prm->imex < 0 ||
      prm->imex > 4 || prm->trace_solver < 0 || prm->trace_solver > 1 || prm->pressure_update < 0 ||
      prm->pressure_update > 1 || prm->idr_s < 0 || prm->idr_s > kIdrMax ||
      prm->precision < 0 || prm->precision > 1 || prm->use_graphs < 0 || prm->use_graphs > 1 ||
      (prm->step1_block != 64 && prm->step1_block != 128 && prm->step1_block != 256) || prm->step1_xcd < 0 ||
      prm->step1_xcd > 1 || prm->step1_precond < 0 || prm->step1_precond > 1 || prm->step2_reading < 0 ||
      prm->step2_reading > 1 || prm->step1_precond_lag < 1) {
    g_create_error = "invalid parameter";
    return HDG_ERR_INVALID_ARG;
  }

  auto ctx = std::make_unique<hdg_ctx>();
  ctx->prm = *prm;
  ctx->s1 = {prm->step1_block, prm->step1_xcd};
  ctx->k = prm->degree;
  ctx->st = (hipStream_t)stream;
  ctx->dim = prm->dim;
  std::string e = prm->dim == 3 ? build_mesh3(nv, coords, nc, cells, ctx->hm)
                                : build_mesh(nv, coords, nc, cells, vertex_rep, ctx->hm);
  if (!e.empty()) { g_create_error = e; return HDG_ERR_INVALID_ARG; }
  if (hipGetDevice(&ctx->device) != hipSuccess) { g_create_error = "no HIP device"; return HDG_ERR_DEVICE; }
  try {
    if (prm->dim == 3) build_reference3(ctx->k, ctx->rt3);
    else build_reference(ctx->k, ctx->rt);
    ctx->setup();
    ctx->eval_scratch = scratch_address(ctx->device);
    ctx->eval_host.assign(kEvalScratchDoubles, 0.0);
  } catch (const OomError& ex) {
    g_create_error = ex.what();
    hdg_destroy(ctx.release());
    return HDG_ERR_OUT_OF_MEMORY;
  } catch (const std::exception& ex) {
    g_create_error = ex.what();
    hdg_destroy(ctx.release());
    return HDG_ERR_DEVICE;
  }
  *out = ctx.release();
  return HDG_OK;
}

void hdg_destroy(hdg_ctx* ctx) {
  if (!ctx) return;
  (void)hipStreamSynchronize(ctx->st);
  for (auto& kv : ctx->ops)
    if (kv.second->pcg_block) (void)hipGraphExecDestroy(kv.second->pcg_block);
  for (auto& g : ctx->bicg_graphs)
    if (g.second) (void)hipGraphExecDestroy(g.second);
  if (ctx->cap_st) (void)hipStreamDestroy(ctx->cap_st);
  for (void* p : ctx->allocs) (void)hipFree(p);
  if (ctx->h_pinned) (void)hipHostFree(ctx->h_pinned);
  delete ctx;
}

const char* hdg_last_error(const hdg_ctx* ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->err.c_str();
}

int hdg_sizes(const hdg_ctx* ctx, int64_t* out, int n) {
  if (!ctx || !out || n < 0 || n > 8) return HDG_ERR_INVALID_ARG;
  const int64_t v[8] = {ctx->hm.nc, ctx->hm.nF, ctx->nQ, ctx->nP, ctx->nT, ctx->nqc, ctx->hm.nv, ctx->k};
  for (int i = 0; i < n; ++i) out[i] = v[i];
  return HDG_OK;
}

int hdg_cell_points(const hdg_ctx* ctx, double* xy) {
  if (!ctx || !xy) return HDG_ERR_INVALID_ARG;
  const auto& m = ctx->hm;
  if (ctx->dim == 3) {
    const auto& t = ctx->rt3;
    for (int64_t e = 0; e < m.nc; ++e) {
      const double* v0 = &m.coords[3 * m.cells[4 * e]];
      for (int q = 0; q < t.nqc; ++q) {
        const double r[3] = {t.cq_x[q], t.cq_y[q], t.cq_z[q]};
        for (int a = 0; a < 3; ++a) {
          double x = v0[a];
          for (int b = 0; b < 3; ++b) x += m.geo[(size_t)(E_J + 3 * a + b) * m.nc + e] * r[b];
          xy[(e * t.nqc + q) * 3 + a] = x;
        }
      }
    }
    return HDG_OK;
  }
  const auto& t = ctx->rt;
  for (int64_t e = 0; e < m.nc; ++e) {
    const double* v0 = &m.coords[2 * m.cells[3 * e]];
    const double* v1 = &m.coords[2 * m.cells[3 * e + 1]];
    const double* v2 = &m.coords[2 * m.cells[3 * e + 2]];
    for (int q = 0; q < t.nqc; ++q) {
      const double a = t.cq_xi[q], b = t.cq_eta[q];
      xy[(e * t.nqc + q) * 2] = v0[0] + (v1[0] - v0[0]) * a + (v2[0] - v0[0]) * b;
      xy[(e * t.nqc + q) * 2 + 1] = v0[1] + (v1[1] - v0[1]) * a + (v2[1] - v0[1]) * b;
    }
  }
  return HDG_OK;
}

int hdg_facet_points(const hdg_ctx* ctx, double* xy) {
  if (!ctx || !xy) return HDG_ERR_INVALID_ARG;
  const auto& m = ctx->hm;
  if (ctx->dim == 3) {  // [nc][4][nq][3], facet f's points in the facet's own order
    const auto& t = ctx->rt3;
    for (int64_t e = 0; e < m.nc; ++e)
      for (int f = 0; f < 4; ++f) {
        const int64_t F = m.cf_facet[f * m.nc + e];
        const double* a = &m.coords[3 * m.facet_lo[F]];
        const double* b = &m.coords[3 * m.facet_mid[F]];
        const double* c = &m.coords[3 * m.facet_hi[F]];
        for (int q = 0; q < t.nqf; ++q)
          for (int d = 0; d < 3; ++d)
            xy[((e * 4 + f) * t.nqf + q) * 3 + d] = a[d] + t.fq_s[q] * (b[d] - a[d]) + t.fq_t[q] * (c[d] - a[d]);
      }
    return HDG_OK;
  }
  const auto& t = ctx->rt;
  for (int64_t e = 0; e < m.nc; ++e) {
    const double* v0 = &m.coords[2 * m.cells[3 * e]];
    const double* v1 = &m.coords[2 * m.cells[3 * e + 1]];
    const double* v2 = &m.coords[2 * m.cells[3 * e + 2]];
    for (int f = 0; f < 3; ++f)
      for (int q = 0; q < t.nqf; ++q) {
        double a, b;  // the reference point of the facet trace tables
        hdg::facet_point(f, t.fq_s[q], a, b);
        const int64_t i = ((e * 3 + f) * t.nqf + q) * 2;
        xy[i] = v0[0] + (v1[0] - v0[0]) * a + (v2[0] - v0[0]) * b;
        xy[i + 1] = v0[1] + (v1[1] - v0[1]) * a + (v2[1] - v0[1]) * b;
      }
  }
  return HDG_OK;
}

int hdg_set_forcing(hdg_ctx* ctx, const double* cell_vals, const double* facet_vals, double decay) {
  if (!ctx || (cell_vals && !facet_vals) || !(decay == decay)) return HDG_ERR_INVALID_ARG;
  if (ctx->dim == 3 && cell_vals) { ctx->err = "forcing is not available on tetrahedra"; return HDG_ERR_UNSUPPORTED; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  if (!cell_vals) {
    ctx->forced = false;
  } else {
    const long nc = ctx->hm.nc;
    if (!ctx->f_dual) {
      ctx->f_dual = ctx->dalloc<double>(ctx->nQ);
      ctx->f_cell = ctx->dalloc<double>(nc * ctx->nqc * 2);
      ctx->f_fac = ctx->dalloc<double>(nc * 3 * ctx->nqf * 2);
      ctx->f_wall = ctx->dalloc<double>(ctx->nT);
      ctx->f_tmp = ctx->dalloc<double>(ctx->nT);
    }
    HIPCHK(hipMemcpyAsync(ctx->f_cell, cell_vals, nc * ctx->nqc * 2 * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->st));
    HIPCHK(hipMemcpyAsync(ctx->f_fac, facet_vals, nc * 3 * ctx->nqf * 2 * sizeof(double), hipMemcpyDeviceToDevice,
                          ctx->st));
    launch_point_dual(ctx->k, ctx->st, ctx->dm, ctx->dt, ctx->f_cell, ctx->f_dual);
    launch_fill(ctx->st, ctx->nT, 0.0, ctx->f_wall);
    launch_wall_flux(ctx->k, ctx->st, ctx->dm, ctx->dt, ctx->f_fac, ctx->f_wall);
    KCHK();
    ctx->f_decay = decay;
    ctx->forced = true;
  }
  ctx->sync();
  API_END(ctx)
}

int hdg_set_time(hdg_ctx* ctx, double t) {
  if (!ctx || !(t == t)) return HDG_ERR_INVALID_ARG;
  ctx->time = t;
  ctx->pend_stage = 0;  // a step in progress is abandoned
  return HDG_OK;
}

double hdg_get_time(const hdg_ctx* ctx) { return ctx ? ctx->time : 0.0; }

int hdg_set_velocity_from_points(hdg_ctx* ctx, const double* qvals) {
  if (!ctx || !qvals) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  ctx->pend_stage = 0;  // a step in progress is abandoned
  API_BEGIN
  launch_project(ctx->k, ctx->st, ctx->dm, ctx->dt, qvals, ctx->Q);
  KCHK();
  ctx->reconstruct(ctx->Q, ctx->p, ctx->lam);
  ctx->have_state = true;
  API_END(ctx)
}

int hdg_set_state(hdg_ctx* ctx, const double* Qv, const double* pv, const double* lv) {
  if (!ctx || !Qv || !pv || !lv) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  ctx->pend_stage = 0;  // a step in progress is abandoned
  API_BEGIN
  launch_copy(ctx->st, ctx->nQ, Qv, ctx->Q);
  launch_copy(ctx->st, ctx->nP, pv, ctx->p);
  launch_copy(ctx->st, ctx->nT, lv, ctx->lam);
  KCHK();
  ctx->sync();
  ctx->have_state = true;
  API_END(ctx)
}

int hdg_get_state(const hdg_ctx* cctx, double* Qv, double* pv, double* lv) {
  hdg_ctx* ctx = const_cast<hdg_ctx*>(cctx);
  if (!ctx) return HDG_ERR_INVALID_ARG;
  if (!ctx->have_state) { ctx->err = "no state set"; return HDG_ERR_BAD_STATE; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  if (Qv) launch_copy(ctx->st, ctx->nQ, ctx->Q, Qv);
  if (pv) launch_copy(ctx->st, ctx->nP, ctx->p, pv);
  if (lv) launch_copy(ctx->st, ctx->nT, ctx->lam, lv);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_advance(hdg_ctx* ctx, double dtv, int nsteps) {
  if (!ctx || !(dtv > 0) || nsteps < 0) return HDG_ERR_INVALID_ARG;
  if (!ctx->have_state) { ctx->err = "no state set"; return HDG_ERR_BAD_STATE; }
  if (ctx->pend_stage != 0) {
    ctx->err = "a step is in progress (hdg_advance_stages): finish it first";
    return HDG_ERR_BAD_STATE;
  }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  try {
    for (int n = 0; n < nsteps; ++n) ctx->step(dtv);
  } catch (...) {
    ctx->pend_stage = 0;
    throw;
  }
  API_END(ctx)
}

int hdg_advance_stages(hdg_ctx* ctx, double dtv, int nstages) {
  if (!ctx || !(dtv > 0) || nstages < 0) return HDG_ERR_INVALID_ARG;
  if (!ctx->have_state) { ctx->err = "no state set"; return HDG_ERR_BAD_STATE; }
  if (ctx->pend_stage != 0 && dtv != ctx->pend_dt) {
    ctx->err = "the step in progress has another dt";
    return HDG_ERR_INVALID_ARG;
  }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  try {
    for (int n = 0; n < nstages; ++n) {
      if (ctx->pend_stage == 0) ctx->begin_step(dtv);
      ctx->stage_once();
    }
    ctx->sync();
  } catch (...) {
    ctx->pend_stage = 0;
    throw;
  }
  API_END(ctx)
}

int hdg_pending_stage(const hdg_ctx* ctx) { return ctx ? ctx->pend_stage : -1; }

int hdg_set_tracer(hdg_ctx* ctx, const double* qvals) {
  if (!ctx) return HDG_ERR_INVALID_ARG;
  if (ctx->dim == 3) { ctx->err = "hdg_set_tracer: triangles only"; return HDG_ERR_UNSUPPORTED; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  if (!qvals) {
    ctx->tracer_on = false;
  } else {
    ctx->tracer_alloc();
    launch_project_scalar(ctx->k, ctx->st, ctx->dm, ctx->dt, qvals, ctx->trq);
    KCHK();
    ctx->tracer_on = true;
  }
  ctx->sync();
  API_END(ctx)
}

int hdg_get_tracer(const hdg_ctx* cctx, double* q) {
  hdg_ctx* ctx = const_cast<hdg_ctx*>(cctx);
  if (!ctx || !q) return HDG_ERR_INVALID_ARG;
  if (!ctx->tracer_on) { ctx->err = "no tracer set"; return HDG_ERR_BAD_STATE; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  launch_copy(ctx->st, ctx->nP, ctx->trq, q);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_cg_project(hdg_ctx* ctx, const double* Qv, double* Ucg) {
  if (!ctx || !Qv || !Ucg) return HDG_ERR_INVALID_ARG;
  if (ctx->dim == 3) { ctx->err = "hdg_cg_project: triangles only"; return HDG_ERR_UNSUPPORTED; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->cg_project(Qv, Ucg);
  ctx->sync();
  API_END(ctx)
}

int hdg_tracer_rate(hdg_ctx* ctx, const double* Qv, const double* q, double* out) {
  if (!ctx || !Qv || !q || !out) return HDG_ERR_INVALID_ARG;
  if (ctx->dim == 3) { ctx->err = "hdg_tracer_rate: triangles only"; return HDG_ERR_UNSUPPORTED; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->tracer_alloc();
  ctx->cg_project(Qv, ctx->Ucg);
  launch_tracer_rate(ctx->k, ctx->st, ctx->dm, ctx->dt, ctx->Ucg, q, out);
  KCHK();
  ctx->sync();
  API_END(ctx)
}


int hdg_eval_points(hdg_ctx* ctx, const double* xy_ref, int npts, double* Qo, double* po) {
  if (!ctx || !xy_ref || npts < 1 || npts > kMaxEvalPoints || (!Qo && !po)) return HDG_ERR_INVALID_ARG;
  if (ctx->dim == 3) { ctx->err = "hdg_eval_points: triangles only"; return HDG_ERR_UNSUPPORTED; }
  if (!ctx->have_state) { ctx->err = "no state set"; return HDG_ERR_BAD_STATE; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  const int ns = ctx->ns, np = ctx->np;
  std::vector<double> bu((size_t)npts * ns), bp((size_t)npts * np);
  for (int q = 0; q < npts; ++q) {
    dubiner_eval(ctx->k + 1, xy_ref[2 * q], xy_ref[2 * q + 1], &bu[(size_t)q * ns], nullptr, nullptr);
    dubiner_eval(ctx->k, xy_ref[2 * q], xy_ref[2 * q + 1], &bp[(size_t)q * np], nullptr, nullptr);
  }
  if (!ctx->eval_tab) ctx->eval_tab = ctx->dalloc<double>((size_t)kMaxEvalPoints * (ns + np));
  HIPCHK(hipMemcpyAsync(ctx->eval_tab, bu.data(), bu.size() * sizeof(double), hipMemcpyHostToDevice, ctx->st));
  HIPCHK(hipMemcpyAsync(ctx->eval_tab + bu.size(), bp.data(), bp.size() * sizeof(double), hipMemcpyHostToDevice,
                        ctx->st));
  launch_eval_points(ctx->st, ctx->hm.nc, npts, ns, np, ctx->eval_tab, ctx->eval_tab + bu.size(), ctx->Q, ctx->p, Qo,
                     po);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

// hdg_eval_points with the basis table staged in the device's static scratch
// array instead of a buffer allocated on first use: no device allocation.
// Calls on one device share the array, so calls that overlap there race.
int hdg_eval_points_noalloc(hdg_ctx* ctx, const double* xy_ref, int npts, double* Qo, double* po) {
  if (!ctx || !xy_ref || npts < 1 || (!Qo && !po)) return HDG_ERR_INVALID_ARG;
  if (ctx->dim == 3) { ctx->err = "hdg_eval_points_noalloc: triangles only"; return HDG_ERR_UNSUPPORTED; }
  if (npts > kMaxEvalPoints) {
    ctx->err = "hdg_eval_points_noalloc: " + std::to_string(npts) + " points, more than the static staging area's " +
               std::to_string(kMaxEvalPoints);
    return HDG_ERR_INVALID_ARG;
  }
  if (!ctx->have_state) { ctx->err = "no state set"; return HDG_ERR_BAD_STATE; }
  if (!ctx->eval_scratch) {
    ctx->err = "hdg_eval_points_noalloc: the static staging area has no address on this device";
    return HDG_ERR_DEVICE;
  }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  const int ns = ctx->ns, np = ctx->np;
  if ((long)npts * (ns + np) > kEvalScratchDoubles) throw ArgError("staging area too small for this degree");
  double* bu = ctx->eval_host.data();
  double* bp = bu + (size_t)npts * ns;
  for (int q = 0; q < npts; ++q) {
    dubiner_eval(ctx->k + 1, xy_ref[2 * q], xy_ref[2 * q + 1], bu + (size_t)q * ns, nullptr, nullptr);
    dubiner_eval(ctx->k, xy_ref[2 * q], xy_ref[2 * q + 1], bp + (size_t)q * np, nullptr, nullptr);
  }
  double* d = ctx->eval_scratch;
  HIPCHK(hipMemcpyAsync(d, bu, sizeof(double) * (size_t)npts * (ns + np), hipMemcpyHostToDevice, ctx->st));
  launch_eval_points(ctx->st, ctx->hm.nc, npts, ns, np, d, d + (size_t)npts * ns, ctx->Q, ctx->p, Qo, po);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_mesh_square(int n, double length, int diagonal, int periodic, double* coords, int32_t* cells,
                    int32_t* vertex_rep) {
  if (n < 1 || !(length > 0) || !coords || !cells || (periodic && (!vertex_rep || n < 3)) || diagonal < 0 ||
      diagonal > 1)
    return HDG_ERR_INVALID_ARG;
  const int64_t m = n + 1;
  if ((int64_t)n * n * 2 > INT32_MAX / 3) return HDG_ERR_INVALID_ARG;
  for (int64_t j = 0; j < m; ++j)
    for (int64_t i = 0; i < m; ++i) {
      const int64_t v = j * m + i;
      coords[2 * v] = length * (double)i / n;
      coords[2 * v + 1] = length * (double)j / n;
      if (vertex_rep) vertex_rep[v] = periodic ? (int32_t)((j % n) * m + (i % n)) : (int32_t)v;
    }
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = 0; i < n; ++i) {
      const int32_t v00 = (int32_t)(j * m + i), v10 = v00 + 1, v01 = (int32_t)(v00 + m), v11 = v01 + 1;
      int32_t* c = cells + 6 * (j * n + i);
      if (diagonal == 0) {
        c[0] = v00; c[1] = v10; c[2] = v11;  // below the "/" diagonal
        c[3] = v00; c[4] = v11; c[5] = v01;  // above it
      } else {
        c[0] = v00; c[1] = v10; c[2] = v01;  // below the "\" diagonal
        c[3] = v10; c[4] = v11; c[5] = v01;  // above it
      }
    }
  return HDG_OK;
}

int hdg_mesh_unit_cube(int n, double* coords, int32_t* cells) {
  if (n < 1 || n > 1024 || !coords || !cells) return HDG_ERR_INVALID_ARG;
  hdg::mesh_unit_cube(n, coords, cells);
  return HDG_OK;
}

int hdg_solve_trace(hdg_ctx* ctx, double c, const double* Fw, const double* Fpsi, const double* Fmu, double* U,
                    double* pv, double* lv) {
  if (!ctx || !(c > 0) || !U || !pv || !lv) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->solve_trace(c, Fw, Fpsi, Fmu, U, pv, lv);
  API_END(ctx)
}

int hdg_trace_matvec(hdg_ctx* ctx, double c, const double* x, double* y) {
  if (!ctx || !(c > 0) || !x || !y) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  TraceOp& op = ctx->trace_op(c);
  {
    Timed tm(ctx->prof, KC_TRACE_SPMV);
    launch_spmv(ctx->tk, ctx->st, (int)ctx->hm.nF, op.vals, op.cols, x, y);
  }
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_bdm_project(hdg_ctx* ctx, const double* Qv, double* Qsv) {
  if (!ctx || !Qv || !Qsv) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  launch_bdm(ctx->k, ctx->st, ctx->dm, ctx->dt, Qv, Qsv);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_weak_divergence(hdg_ctx* ctx, const double* F, double* out) {
  if (!ctx || !F || !out) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  launch_div(ctx->k, ctx->st, ctx->dm, ctx->dt, F, 1.0, out);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_momentum_residual(hdg_ctx* ctx, double adt, const double* r, const double* Qsv, const double* Qv,
                          const double* pv, const double* lv, double* out) {
  if (!ctx || !r || !Qsv || !Qv || !pv || !lv || !out) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  launch_prep_adv(ctx->k, ctx->st, ctx->dm, ctx->dt, Qsv, ctx->prm.delta_up, ctx->adv);
  launch_apply(ctx->k, ctx->st, 2, ctx->dm, ctx->dt, ctx->adv, ctx->prm.alpha, adt, Qv, r, pv, lv, out);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_tentative_velocity(hdg_ctx* ctx, double adt, const double* Qsv, const double* rhs, double* Qbar) {
  if (!ctx || !Qsv || !rhs || !Qbar) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->prepare_step1(Qsv);
  // mass-scaled right-hand side rhs / det: the residual kernel with Q = p = lam = 0
  {
    launch_fill(ctx->st, ctx->nQ, 0.0, ctx->Ut);
    launch_fill(ctx->st, ctx->nP, 0.0, ctx->dp);
    launch_fill(ctx->st, ctx->nT, 0.0, ctx->dl);
    launch_apply(ctx->k, ctx->st, 1, ctx->dm, ctx->dt, ctx->adv, ctx->prm.alpha, adt, ctx->Ut, rhs, ctx->dp,
                 ctx->dl, ctx->dr);
  }
  KCHK();
  int its = ctx->velocity_solve(adt, ctx->dr, Qbar);
  ctx->bicg_iters.push_back(its);
  ctx->total_bicg += its;
  ++ctx->n_velocity_solves;
  ctx->sync();
  API_END(ctx)
}

int hdg_step1_precond(hdg_ctx* ctx, double adt, const double* Qsv, const double* r, double* z) {
  if (!ctx || !(adt > 0) || !Qsv || !r || !z) return HDG_ERR_INVALID_ARG;
  if (!ctx->pc_on) { ctx->err = "the Step I preconditioner is off for this context"; return HDG_ERR_UNSUPPORTED; }
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->prepare_step1(Qsv);
  ctx->pc_prepare(adt);
  launch_to_soa(ctx->k, ctx->st, ctx->dm, 0, r, ctx->kd.b, ctx->kx32);
  ctx->pc_apply(ctx->kd.b, ctx->kd.x);
  launch_to_aos(ctx->k, ctx->st, ctx->dm, ctx->kd.x, z, ctx->kx32);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_constraint_residual(hdg_ctx* ctx, const double* Qv, const double* pv, const double* lv, double* Fpsi,
                            double* Fmu) {
  if (!ctx || !Qv || !Fpsi || !Fmu) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  launch_gamma(ctx->k, ctx->st, ctx->dm, ctx->dt, ctx->prm.tau, 1.0, Qv, pv, lv, Fpsi, ctx->ycell, Fmu);
  KCHK();
  ctx->sync();
  API_END(ctx)
}

int hdg_reconstruct_pressure(hdg_ctx* ctx, const double* Qv, double* pv, double* lv) {
  if (!ctx || !Qv || !pv || !lv) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->reconstruct(Qv, pv, lv);
  API_END(ctx)
}

int hdg_profile(hdg_ctx* ctx, int enable) {
  if (!ctx) return HDG_ERR_INVALID_ARG;
  ctx->not_converged = false;
  ctx->err.clear();
  API_BEGIN
  ctx->sync();
  ctx->prof.reset();
  ctx->prof.on = enable > 0;
  ctx->prof.every = enable > 0 ? enable : 1;
  API_END(ctx)
}

int hdg_get_info(const hdg_ctx* ctx, char* buf, size_t cap) {
  if (!ctx || !buf || cap == 0) return HDG_ERR_INVALID_ARG;
  auto last = [](const std::vector<int>& v, size_t n) {
    std::string s = "[";
    size_t st = v.size() > n ? v.size() - n : 0;
    for (size_t i = st; i < v.size(); ++i) s += (i > st ? "," : "") + std::to_string(v[i]);
    return s + "]";
  };
  size_t amg_levels = 0;  // aggregation levels below the P1 coarse space (largest over the trace operators)
  for (const auto& kv : ctx->ops) amg_levels = std::max(amg_levels, kv.second->levels.size());
  std::string s = "{\"ncells\":" + std::to_string(ctx->hm.nc) + ",\"nfacets\":" + std::to_string(ctx->hm.nF) +
                  ",\"amg_levels\":" + std::to_string(amg_levels) +
                  ",\"degree\":" + std::to_string(ctx->k) + ",\"n_trace_dofs\":" + std::to_string(ctx->nT) +
                  ",\"trace_solves\":" + std::to_string(ctx->n_trace_solves) +
                  ",\"pcg_iterations_total\":" + std::to_string(ctx->total_pcg) +
                  ",\"velocity_solves\":" + std::to_string(ctx->n_velocity_solves) +
                  ",\"velocity_iterations_total\":" + std::to_string(ctx->total_bicg) +
                  ",\"bicgstab_restarts\":" + std::to_string(ctx->bicg_restarts) +
                  ",\"pcg_floor_stops\":" + std::to_string(ctx->pcg_floor_stops) +
                  ",\"pcg_floor_band\":" + hdg::sci(ctx->floor_band()) +
                  ",\"pcg_floor_true_residual_max\":" + hdg::sci(ctx->pcg_floor_true_max) +
                  ",\"velocity_true_residual_max\":" + hdg::sci(ctx->velocity_true_max) +
                  ",\"velocity_true_residual_restarts\":" + std::to_string(ctx->velocity_true_restarts) +
                  ",\"device_bytes\":" + std::to_string(ctx->dev_bytes) +
                  ",\"pending_stage\":" + std::to_string(ctx->pend_stage) +
                  ",\"step1_block\":" + std::to_string(ctx->s1.block) +
                  ",\"step1_xcd\":" + std::to_string(ctx->s1.xcd) +
                  ",\"step1_precond\":" + std::to_string(ctx->pc_on ? 1 : 0) +
                  ",\"step2_reading\":" + std::to_string(ctx->prm.step2_reading) +
                  ",\"step1_precond_builds\":" + std::to_string(ctx->pc_builds) +
                  ",\"device_transient_bytes\":" + std::to_string(ctx->dev_transient) +
                  ",\"pcg_iterations_last\":" + last(ctx->pcg_iters, 16) +
                  ",\"velocity_iterations_last\":" + last(ctx->bicg_iters, 16) +
                  ",\"seconds_trace\":" + std::to_string(ctx->t_trace) +
                  ",\"seconds_velocity\":" + std::to_string(ctx->t_velocity) + ",\"kernels\":{";
  for (int i = 0; i < kNumKClass; ++i) {
    s += std::string(i ? "," : "") + "\"" + kKClassName[i] + "\":{\"launches\":" +
         std::to_string(ctx->prof.launches[i]) + ",\"timed\":" + std::to_string(ctx->prof.timed[i]) +
         ",\"ms\":" + std::to_string(ctx->prof.ms[i]) + "}";
  }
  s += "}}";
  std::snprintf(buf, cap, "%s", s.c_str());
  return s.size() < cap ? HDG_OK : HDG_ERR_INVALID_ARG;
}


int hdg_footprint_bytes(int64_t nv, const double* coords, int64_t nc, const int32_t* cells, const int32_t* vertex_rep,
                        const hdg_params* prm, double dt, int64_t* bytes) {
  if (!prm || !bytes || !(dt > 0)) { g_create_error = "null argument or dt <= 0"; return HDG_ERR_INVALID_ARG; }
  if (prm->dim != 2) { g_create_error = "footprint estimate: triangles only"; return HDG_ERR_UNSUPPORTED; }
  if (prm->degree < 1 || prm->degree > kMaxDegree) { g_create_error = "degree must be in 1..4"; return HDG_ERR_UNSUPPORTED; }
  if (prm->imex < 0 || prm->imex > 4 ||
      (prm->step1_block != 64 && prm->step1_block != 128 && prm->step1_block != 256)) {
    g_create_error = "invalid parameter";
    return HDG_ERR_INVALID_ARG;
  }
  try {
    hdg::HostMesh m;
    std::string e = build_mesh(nv, coords, nc, cells, vertex_rep, m);
    if (!e.empty()) { g_create_error = e; return HDG_ERR_INVALID_ARG; }
    hdg::RefTables rt;
    build_reference(prm->degree, rt);
    int64_t held = 0, transient = 0;
    estimate_footprint(m, rt, *prm, dt, &held, &transient);
    *bytes = held + transient;
  } catch (const std::exception& ex) {
    g_create_error = ex.what();
    return HDG_ERR_INVALID_ARG;
  }
  return HDG_OK;
}

}  // extern "C"

// A batch is a non-owning list of distinct contexts.  Advancing it runs
// every member's hdg_advance on a pool of host threads (at most 16, one
// member at a time per thread), so members on distinct streams overlap on
// the device; each member's arithmetic is exactly that of a lone call.
struct hdg_batch {
  std::vector<hdg_ctx*> members;
};

extern "C" {

int hdg_batch_create(int n, hdg_ctx* const* members, hdg_batch** out) {
  if (!out || n < 1 || !members) { g_create_error = "null argument or empty batch"; return HDG_ERR_INVALID_ARG; }
  *out = nullptr;
  std::set<hdg_ctx*> seen;
  for (int i = 0; i < n; ++i) {
    if (!members[i] || !seen.insert(members[i]).second) {
      g_create_error = "batch members must be distinct, non-null contexts";
      return HDG_ERR_INVALID_ARG;
    }
  }
  auto b = new (std::nothrow) hdg_batch;
  if (!b) { g_create_error = "out of host memory"; return HDG_ERR_OUT_OF_MEMORY; }
  b->members.assign(members, members + n);
  *out = b;
  return HDG_OK;
}

int hdg_batch_size(const hdg_batch* b) { return b ? (int)b->members.size() : 0; }

int hdg_batch_advance(hdg_batch* b, const double* dt, const int* nsteps, int* status) {
  if (!b || !dt || !nsteps) return HDG_ERR_INVALID_ARG;
  const int n = (int)b->members.size();
  std::vector<int> st(n, HDG_OK);
  std::atomic<int> next{0};
  auto work = [&] {
    for (int i = next.fetch_add(1); i < n; i = next.fetch_add(1)) {
      hdg_ctx* c = b->members[i];
      if (hipSetDevice(c->device) != hipSuccess) {
        c->err = "hipSetDevice failed";
        st[i] = HDG_ERR_DEVICE;
        continue;
      }
      st[i] = hdg_advance(c, dt[i], nsteps[i]);
    }
  };
  const int nthreads = std::min(n, 16);
  std::vector<std::thread> pool;
  try {
    for (int t = 1; t < nthreads; ++t) pool.emplace_back(work);
  } catch (const std::exception&) {
    // fewer threads: the calling thread and those started share the members
  }
  work();
  for (auto& t : pool) t.join();
  int worst = HDG_OK;
  for (int i = 0; i < n; ++i) {
    if (status) status[i] = st[i];
    if (worst == HDG_OK && st[i] != HDG_OK) worst = st[i];
  }
  return worst;
}

void hdg_batch_destroy(hdg_batch* b) { delete b; }

}  // extern "C"
