// gfx950 kernels of the tentative-velocity solve (Algorithm 2, Step I): the
// per-stage cell data of the Step I form f_im(., .; Q*) of eq. (f_impl), the
// mass-scaled operator on structure-of-arrays vectors and the BiCGStab
// vector kernels.
#include <hip/hip_runtime.h>

#include <stdexcept>

#include "device_common.h"

namespace hdg {

// Value held by the other lane of an adjacent lane pair (2i <-> 2i+1), via a
// DPP quad permutation [1,0,3,2]: a VALU operation, so unlike a bpermute it
// does not wait on outstanding scalar loads.  Both lanes of a pair must be
// active.
__device__ __forceinline__ double pair_swap(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), 0xB1, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), 0xB1, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float pair_swap(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
}

// Per-cell data of the Step I operator are stored in tiles of 32 cells
// (one wave of the two-threads-per-cell kernels): entry j of cell e sits at
// ((e/32)*nj + j)*32 + e%32.  A wave then reads 256 contiguous bytes per
// entry and one contiguous block overall, which keeps the number of DRAM
// streams small.  Arrays hold ceil(nc/32)*32 cells.
__device__ __forceinline__ long tile_idx(long e, int j, int nj) { return ((e >> 5) * nj + j) * 32 + (e & 31); }

typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));

// Per-cell advecting field of the Step I volume term at the cell points,
// for the Q* of a stage.  The volume term -(Q*.grad x, w) of eq. (f_impl)
// is, on every velocity component alike,
//   -sum_q w_q phi_s(q) (Q*(q) . grad phi_s'(q)) det J
//     = sum_q phi_s(q) (A_q . grad_ref phi_s'(q)),  A_q = -w_q det J^{-1} Q*(q)
// (grad = J^{-T} grad_ref), so the operator evaluates it at the NQC cell
// points from A_q (2 numbers per point) instead of streaming an NS x NS
// matrix per cell.  Entry 2q + d of cell e in tiles of 32 cells; TV is the
// storage type (FP32 in the mixed-precision mode).  One thread per cell.
template <int K, typename TV>
__global__ void __launch_bounds__(kBlock) k_step1_field(DMesh m, DTab t, const double* __restrict__ Qs,
                                                        TV* __restrict__ A) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nc = m.nc;
  if (e >= nc) return;
  double q[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) q[i] = Qs[e * NU + i];
  const double det = m.geo[D_DET * nc + e];
  const double i00 = det * m.geo[D_IJ00 * nc + e], i01 = det * m.geo[D_IJ01 * nc + e];
  const double i10 = det * m.geo[D_IJ10 * nc + e], i11 = det * m.geo[D_IJ11 * nc + e];
  for (int qq = 0; qq < NQC; ++qq) {
    double qx = 0.0, qy = 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      qx += t.Bu[qq * NS + i] * q[i];
      qy += t.Bu[qq * NS + i] * q[NS + i];
    }
    const double w = -t.cw[qq];
    A[tile_idx(e, 2 * qq, 2 * NQC)] = (TV)(w * (i00 * qx + i01 * qy));
    A[tile_idx(e, 2 * qq + 1, 2 * NQC)] = (TV)(w * (i10 * qx + i11 * qy));
  }
}

// Upwind weights of the Step I facet term at the facet points, for the Q*
// of a stage: beta = w_q h (Q*.n/2 - delta_up |Q*.n|) on interior facets,
// 0 on walls, entry f*NQF + q in tiles, stored as TB (the operator's
// arithmetic type).  One thread per (cell, facet).
template <int K, typename TB>
__global__ void __launch_bounds__(kBlock) k_step1_beta(DMesh m, DTab t, const double* __restrict__ Qs,
                                                       double delta_up, TB* __restrict__ beta) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQF = D::NQF;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nc = m.nc;
  if (tid >= 3 * nc) return;
  const int e = (int)(tid % nc), f = (int)(tid / nc);
  const bool inner = m.cf_nb[f * nc + e] >= 0;
  const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
  const double h = m.geo[(D_H0 + f) * nc + e];
  for (int qq = 0; qq < NQF; ++qq) {
    double vx = 0.0, vy = 0.0;
    for (int s = 0; s < NS; ++s) {
      const double b = t.FBu[(f * NQF + qq) * NS + s];
      vx += b * Qs[(long)e * NU + s];
      vy += b * Qs[(long)e * NU + NS + s];
    }
    const double qn = vx * nx + vy * ny;
    beta[tile_idx(e, f * NQF + qq, 3 * NQF)] = (TB)(inner ? t.fw[qq] * h * (0.5 * qn - delta_up * fabs(qn)) : 0.0);
  }
}

// The Step I form f_im(w, x; Q*) of eq. (f_impl) for one cell e and one
// velocity component c on structure-of-arrays data x[(c*NS + s)*nc + e]:
// the volume term at the cell points from the per-stage field A_q
// (k_step1_field), and per facet the upwinded advective jump term
// beta(q) [[x]] (beta = w_q h (Q*.n/2 - delta_up |Q*.n|) at the facet
// points, precomputed per stage in tiles, entry f*NQF + q, zero on walls)
// and the normal-jump penalty alpha ([[x]].n)(w.n).  Two threads per cell
// (lanes 2i, 2i+1, one per component) exchange their components of the jump
// with pair_swap.  y receives the result in reference scaling (the caller
// multiplies by adt/det).  The neighbour's input value at structure-of-arrays
// index idx is nb(idx); sFBu is the facet trace table staged in LDS.  TC is
// the arithmetic type (FP64, or FP32 in the mixed-precision mode), TV the
// storage type of the field.  The reference tables are indexed by loop
// counters only, the same on every lane: scalar loads.
template <int K, typename TV, typename TC, typename NbVal>
__device__ __forceinline__ void step1_core(const DMesh& m, const DTab& t, const TC* sFBu,
                                           const TV* __restrict__ A, const TC* __restrict__ beta, long nc,
                                           int e, int c, TC alpha, const TC (&xv)[Dims<K>::NS],
                                           TC (&y)[Dims<K>::NS], const NbVal& nb) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NQF = D::NQF, NQC = D::NQC;
  // volume: the reference gradient of x at each cell point, dotted with A_q,
  // tested against phi_s.  A is read once per application: non-temporal
  // loads keep it from evicting the velocity vectors (read again by the
  // neighbouring cells) from the caches.
#pragma unroll
  for (int s = 0; s < NS; ++s) y[s] = 0;
#pragma unroll 2
  for (int qq = 0; qq < NQC; ++qq) {
    const TC a0 = (TC)__builtin_nontemporal_load(&A[tile_idx(e, 2 * qq, 2 * NQC)]);
    const TC a1 = (TC)__builtin_nontemporal_load(&A[tile_idx(e, 2 * qq + 1, 2 * NQC)]);
    TC gx = 0, gy = 0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      gx += (TC)t.Gux[qq * NS + s] * xv[s];
      gy += (TC)t.Guy[qq * NS + s] * xv[s];
    }
    const TC tq = a0 * gx + a1 * gy;
#pragma unroll
    for (int s = 0; s < NS; ++s) y[s] += (TC)t.Bu[qq * NS + s] * tq;
  }
  int nbx[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) nbx[f] = m.cf_nbx[f * nc + e];
#pragma unroll 1
  for (int f = 0; f < 3; ++f) {
    const int en = nbx[f] >= 0 ? nbx[f] >> 3 : -1;
    const int fn = nbx[f] >= 0 ? (nbx[f] >> 1) & 3 : 0;
    const int rev = nbx[f] >= 0 ? nbx[f] & 1 : 0;
    const TC nx = (TC)m.geo[(D_NX0 + 2 * f) * nc + e], ny = (TC)m.geo[(D_NY0 + 2 * f) * nc + e];
    const TC ncomp = c ? ny : nx;
    TC xn[NS], bq[NQF];
#pragma unroll
    for (int qq = 0; qq < NQF; ++qq) bq[qq] = __builtin_nontemporal_load(&beta[tile_idx(e, f * NQF + qq, 3 * NQF)]);
    if (en >= 0) {
#pragma unroll
      for (int s = 0; s < NS; ++s) xn[s] = nb((long)(c * NS + s) * nc + en);
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) xn[s] = 0;
    }
#pragma unroll
    for (int qq = 0; qq < NQF; ++qq) {
      const int qn = rev ? NQF - 1 - qq : qq;
      TC j = 0, jn = 0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        j += (TC)t.FBu[(f * NQF + qq) * NS + s] * xv[s];
        jn += sFBu[(fn * NQF + qn) * NS + s] * xn[s];
      }
      j -= jn;
      const TC jo = pair_swap(j);
      const TC jdotn = c ? (jo * nx + j * ny) : (j * nx + jo * ny);
      const TC con = bq[qq] * j - alpha * (TC)t.fw[qq] * jdotn * ncomp;
#pragma unroll
      for (int s = 0; s < NS; ++s) y[s] += (TC)t.FBu[(f * NQF + qq) * NS + s] * con;
    }
  }
}

// Waves per SIMD the Step I operator kernels are compiled for (bounds their
// registers, and with them how many loads the compiler keeps in flight).
#ifndef HDG_STEP1_WAVES
#define HDG_STEP1_WAVES 2
#endif
constexpr int kStep1Waves = HDG_STEP1_WAVES;

// Workgroups are dealt to the eight XCDs in turn (workgroup i to XCD i % 8),
// and each XCD has its own L2.  The Step I operator reads the input vector
// at neighbour cells, which sit a few workgroups away; renumbering so that
// each XCD takes one contiguous eighth of the cells keeps those reads in the
// same L2.  A bijection of [0, gridDim.x) onto itself.
__device__ __forceinline__ int xcd_block() {
  const int nb = gridDim.x, b = blockIdx.x;
  const int q = nb >> 3, r = nb & 7, x = b & 7, j = b >> 3;
  return x < r ? x * (q + 1) + j : r * (q + 1) + (x - r) * q + j;
}

// Stage the facet trace table in LDS: the neighbour's table row is indexed
// by the neighbour's local facet and orientation, which differ between lanes.
template <int K, typename TC>
__device__ __forceinline__ void stage_fbu(const DTab& t, TC* sFBu) {
  constexpr int N = 3 * Dims<K>::NQF * Dims<K>::NS;
  for (int i = threadIdx.x; i < N; i += blockDim.x) sFBu[i] = (TC)t.FBu[i];
  __syncthreads();
}

// out = x - (adt/det) f_im(., x; Q*): the mass-scaled Step I operator on
// structure-of-arrays vectors (two threads per cell), with per-block
// partial sums (nb = gridDim.x sets of partials at part + i*nb):
//   DOT 0: none;  DOT 1: w.out;  DOT 2: out.x, out.out, w.x, w.out;
//   DOT 3: out.sd, out.out, w.sd, w.out (sd: the unpreconditioned vector
//   whose preconditioned image is x).
// In BiCGStab, DOT 1 gives rh.v for v = A p and DOT 2 gives t.s, t.t, rh.s,
// rh.t for t = A s.  BS threads per workgroup (64, 128 or 256); xcd = 1 deals
// the cells to the XCDs in contiguous eighths (xcd_block), 0 keeps the
// hardware order.  TX: the vectors' type and the arithmetic type (FP64, or
// FP32 in the mixed-precision mode); the inner products accumulate in FP64.
template <int K, int DOT, typename TV, int BS, typename TX>
__global__ void __launch_bounds__(BS, kStep1Waves) k_apply_soa(DMesh m, DTab t, const TV* __restrict__ A,
                                                               const TX* __restrict__ beta, double alpha,
                                                               double adt, const TX* __restrict__ x,
                                                               const TX* __restrict__ w,
                                                               const TX* __restrict__ sd,
                                                               TX* __restrict__ out,
                                                               double* __restrict__ part, int xcd) {
  using D = Dims<K>;
  constexpr int NS = D::NS;
  __shared__ TX sFBu[3 * D::NQF * NS];
  stage_fbu<K, TX>(t, sFBu);
  const int blk = xcd ? xcd_block() : (int)blockIdx.x;
  const long tid = (long)blk * BS + threadIdx.x;
  const long nc = m.nc;
  const int e = (int)(tid >> 1), c = (int)(tid & 1);
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  if (e < nc) {
    TX xv[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) xv[s] = x[(long)(c * NS + s) * nc + e];
    step1_core<K, TV, TX>(m, t, sFBu, A, beta, nc, e, c, (TX)alpha, xv, y, [&](long i) { return x[i]; });
    const TX sc = (TX)(adt / m.geo[D_DET * nc + e]);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const long idx = (long)(c * NS + s) * nc + e;
      const TX ot = xv[s] - sc * y[s];
      out[idx] = ot;
      const double o = ot;
      if (DOT == 1) d0 += (double)w[idx] * o;
      if (DOT >= 2) {
        const double wv = w[idx];
        const double sv = DOT == 3 ? (double)sd[idx] : (double)xv[s];
        d0 += o * sv;
        d1 += o * o;
        d2 += wv * sv;
        d3 += wv * o;
      }
    }
  }
  if (DOT >= 1) {
    d0 = block_sum_n<BS>(d0);
    if (threadIdx.x == 0) part[blk] = d0;
  }
  if (DOT >= 2) {
    const int nb = gridDim.x;
    d1 = block_sum_n<BS>(d1);
    d2 = block_sum_n<BS>(d2);
    d3 = block_sum_n<BS>(d3);
    if (threadIdx.x == 0) {
      part[nb + blk] = d1;
      part[2 * nb + blk] = d2;
      part[3 * nb + blk] = d3;
    }
  }
}

// Sum of np partials in a fixed order, returned to every thread of the block.
__device__ __forceinline__ double sum_partials(const double* __restrict__ part, int np) {
  __shared__ double r;
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) r = v;
  __syncthreads();
  return r;
}

// BiCGStab on the mass-scaled Step I operator A.  Per iteration, with the
// scalars of the iteration in the slot sc (layout BiCGSlot):
//   v = A p                 k_apply_soa<DOT 1>: partials of rh.v
//   s = r - alpha v         k_bicg_s: every block finishes rh.v itself
//                           (alpha = rho / rh.v), block 0 records it
//   t = A s                 k_apply_soa<DOT 2>: partials of t.s, t.t, rh.s, rh.t
//   x += alpha p + omega s, r = s - omega t, p = r + beta (p - omega v)
//                           k_bicg_xrp: every block finishes the four sums
//                           (omega, beta), block 0 records them and opens the
//                           next slot; partials of r.r
// Both vector kernels run on a fixed grid of kVecBlocks blocks, so the
// redundant finishes read few partials in total.
// Vectors of type TX (FP64, or FP32 in the mixed-precision mode) accessed as
// pairs (n is even: 2 ns entries per cell and component pair); the
// coefficients are FP64 and so are the inner-product partials.
template <typename TX> struct VPair2;
template <> struct VPair2<double> { using T = f64x2; };
template <> struct VPair2<float> { using T = f32x2; };
template <typename TX>
__global__ void __launch_bounds__(kBlock) k_bicg_s(long n, int np, const double* __restrict__ part,
                                                   double* __restrict__ sc, const TX* __restrict__ R,
                                                   const TX* __restrict__ Vv, TX* __restrict__ S) {
  using T2 = typename VPair2<TX>::T;
  const double rv = sum_partials(part, np);
  const bool ok = rv != 0.0 && rv == rv;
  const double al = ok ? sc[BS_RHO] / rv : 0.0;
  const long n2 = n >> 1;
  const T2* R2 = reinterpret_cast<const T2*>(R);
  const T2* V2 = reinterpret_cast<const T2*>(Vv);
  T2* S2 = reinterpret_cast<T2*>(S);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
    const T2 r = R2[i], v = V2[i];
    T2 o;
    o.x = (TX)((double)r.x - al * (double)v.x);
    o.y = (TX)((double)r.y - al * (double)v.y);
    S2[i] = o;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[BS_RV] = rv;
    sc[BS_ALPHA] = al;
    if (!ok) sc[BS_FLAG] = 1.0;
  }
}

template <typename TX>
__global__ void __launch_bounds__(kBlock) k_bicg_xrp(long n, int np, const double* __restrict__ part2,
                                                     double* __restrict__ sc, const TX* __restrict__ S,
                                                     const TX* __restrict__ Tv, const TX* __restrict__ Vv,
                                                     const TX* __restrict__ PH, const TX* __restrict__ SH,
                                                     TX* __restrict__ X, TX* __restrict__ R,
                                                     TX* __restrict__ P, double* __restrict__ part) {
  using T2 = typename VPair2<TX>::T;
  // omega = t.s / t.t, rho_next = rh.s - omega rh.t (= rh.r_next),
  // beta = (rho_next / rho)(alpha / omega)
  const double ts = sum_partials(part2, np);
  const double tt = sum_partials(part2 + np, np);
  const double rs = sum_partials(part2 + 2 * np, np);
  const double rt = sum_partials(part2 + 3 * np, np);
  const double al = sc[BS_ALPHA], rho = sc[BS_RHO];
  const bool okw = tt > 0.0 && ts != 0.0 && ts == ts;
  const double om = okw ? ts / tt : 0.0;
  const double rho_next = rs - om * rt;
  const bool okb = okw && rho != 0.0 && rho_next == rho_next;
  const double be = okb ? (rho_next / rho) * (al / om) : 0.0;
  double rr = 0.0;
  const long n2 = n >> 1;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
    const T2 p = reinterpret_cast<const T2*>(P)[i], s = reinterpret_cast<const T2*>(S)[i];
    const T2 t = reinterpret_cast<const T2*>(Tv)[i], v = reinterpret_cast<const T2*>(Vv)[i];
    // the iterate moves along the preconditioned directions (PH = P, SH = S without a preconditioner)
    const T2 ph = reinterpret_cast<const T2*>(PH)[i], sh = reinterpret_cast<const T2*>(SH)[i];
    T2 x = reinterpret_cast<const T2*>(X)[i];
    x.x = (TX)((double)x.x + (al * (double)ph.x + om * (double)sh.x));
    x.y = (TX)((double)x.y + (al * (double)ph.y + om * (double)sh.y));
    reinterpret_cast<T2*>(X)[i] = x;
    T2 r;
    r.x = (TX)((double)s.x - om * (double)t.x);
    r.y = (TX)((double)s.y - om * (double)t.y);
    reinterpret_cast<T2*>(R)[i] = r;
    rr += (double)r.x * (double)r.x + (double)r.y * (double)r.y;
    T2 pn;
    pn.x = (TX)((double)r.x + be * ((double)p.x - om * (double)v.x));
    pn.y = (TX)((double)r.y + be * ((double)p.y - om * (double)v.y));
    reinterpret_cast<T2*>(P)[i] = pn;
  }
  rr = block_sum(rr);
  if (threadIdx.x == 0) part[blockIdx.x] = rr;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[BS_TS] = ts;
    sc[BS_TT] = tt;
    sc[BS_OMEGA] = om;
    sc[BS_BETA] = be;
    if (!okb) sc[BS_FLAG] = 1.0;
    sc[BS_STRIDE + BS_RHO] = rho_next;
    sc[BS_STRIDE + BS_FLAG] = 0.0;
  }
}

// Slot 0 of a (re)start: no previous coefficients; rho is set by the caller.
__global__ void k_bicg_init(double* __restrict__ sc) {
  if (threadIdx.x < BS_STRIDE && threadIdx.x != BS_RHO) sc[threadIdx.x] = 0.0;
}

// AoS [cell][2 ns] <-> SoA [(c ns + s) nc + cell]; inv_det = 1 also divides by det J
template <int K, typename TX>
__global__ void k_to_soa(DMesh m, int inv_det, const double* __restrict__ x, TX* __restrict__ y) {
  constexpr int NU = Dims<K>::NU;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long)m.nc * NU) return;
  const long e = tid % m.nc, i = tid / m.nc;
  const double sc = inv_det ? 1.0 / m.geo[D_DET * (long)m.nc + e] : 1.0;
  y[tid] = (TX)(sc * x[e * NU + i]);
}
template <int K, typename TX>
__global__ void k_to_aos(DMesh m, const TX* __restrict__ x, double* __restrict__ y) {
  constexpr int NU = Dims<K>::NU;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long)m.nc * NU) return;
  const long e = tid / NU, i = tid % NU;
  y[tid] = (double)x[i * m.nc + e];
}

// Generic vector pieces of the Step I solve in either vector type: y = x,
// y = v, y = a x + b y, and FP64 partial sums of a.b (b null: a.a) over
// kRedBlocks blocks.
template <typename TX>
__global__ void k_vcopy(long n, const TX* __restrict__ x, TX* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
template <typename TX>
__global__ void k_vfill(long n, double v, TX* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (TX)v;
}
template <typename TX>
__global__ void k_vaxpby(long n, double a, const TX* __restrict__ x, double b, TX* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (TX)(a * (double)x[i] + b * (double)y[i]);
}
template <typename TX>
__global__ void __launch_bounds__(kBlock) k_vdot(long n, const TX* __restrict__ a, const TX* __restrict__ b,
                                                 double* __restrict__ part) {
  double v = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v += (double)a[i] * (double)(b ? b[i] : a[i]);
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// ======================================================= Step I preconditioner
// Additive Schwarz over facet patches, B r = sum_F R_F^T A_F^{-1} R_F r: for
// every interior facet F with cells K+ and K-, A_F is the block of the
// mass-scaled Step I operator on the 2 NU unknowns of the two cells (both
// cell blocks and their coupling through F; couplings through the other
// facets are left out).  The interior-penalty term alpha h^-1 <[Q.n][w.n]> of
// eq. (f_impl) carries the factor adt/h^2 against the mass term, and it
// vanishes exactly on fields whose normal component is continuous.  Those
// fields are spanned by functions that live on one cell or on the two cells
// of one facet, so every patch holds its share of them and the
// preconditioned operator stays well conditioned however strong the penalty
// is; single-cell blocks (block Jacobi) hold no such function across a
// facet and lose that property.
//
// Woodbury form.  Within a patch the two cells are coupled only through
// their traces on F, and the trace of a velocity-degree function is a
// polynomial of degree k+1 in the facet parameter.  With L_f the map from a
// cell's coefficients to the orthonormal Legendre coefficients of its trace
// on local facet f (nm = k+2 per component, m = 2 nm in all, in the cell's
// own facet parameter; the reference table TRU), the patch block is
//   A_F = Bd + U^T Kf U,  Bd = diag(A_+, A_-),  U = diag(L_{f+}, L_{f-}),
// where A_e is the whole own-cell block of the operator and Kf (2m x 2m) the
// facet quadrature of the two coupling blocks (zero diagonal blocks).  Then
//   A_F^{-1} = Bd^{-1} - Bd^{-1} U^T M_F U Bd^{-1},  M_F = (I + Kf U Bd^{-1} U^T)^{-1} Kf,
// an exact identity, so this is the same preconditioner as the dense patch
// inverses.  Per cell, with R_f the rotation of the trace components into
// the (normal, tangent) frame of facet f,
//   z_e = n_int(e) A_e^{-1} r_e - sum_f H_f W_f [G_f r_e ; G_{f'} r_{n(f)}],
//   G_f = R_f L_f A_e^{-1},  H_f = A_e^{-1} L_f^T R_f^T,
// W_f the m rows of M_F that belong to e, rotated on both sides (own trace
// columns first, the neighbour's in its own frame).  The rotation is what
// makes FP16 storage safe: M_F grows like adt/h^2 in its normal-normal block
// only, the normal traces of A_e^{-1} r are smaller by the same factor, and
// in x/y components those small normal traces would be differences of O(1)
// numbers that FP16 cannot resolve.  In the facet frame every stored number
// keeps its own relative precision.  The products G_f, H_f are stored, not
// formed from A_e^{-1} in the apply: formed from the FP16 inverse, the
// normal traces carry its rounding of the O(1) entries, and at a 256 x 256
// mesh's penalty the solves took 18 % more iterations.
//
// Storage (FP16, in tiles of 32 cells; thread g of a cell's G = 6 threads
// reads one contiguous run of quads, lane = cell % 32 fastest, zero padded):
// * pass 1, rows [g RG1, (g+1) RG1) of the stacked [A_e^{-1}; G_0; G_1; G_2]
//   (NU + 3m rows of NU entries);
// * W: thread g = 2 f + h holds the nm rows of W_f of frame component h
//   (normal, tangent), each of 2m entries;
// * H: rows [g RG, (g+1) RG) of [H_0 H_1 H_2] (NU rows of 3m entries);
// * one FP32 scale per (cell, facet), a power of two: W is stored divided by
//   it, so that its largest entry is at most 2^14 whatever the mesh size and
//   time step.
// At k = 3: 1,800 + 600 + 900 entries per cell against 3 x 1,800 for the
// dense rows.  Slots of wall facets are never written or read.
using pc_t = _Float16;
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
__device__ __forceinline__ pc_t pc_store(double v) {
  const double lim = 65504.0;  // largest finite FP16
  return (pc_t)(v > lim ? lim : (v < -lim ? -lim : v));
}
template <int K>
struct PcWood {
  static constexpr int NU = Dims<K>::NU, NS = Dims<K>::NS, NM = K + 2;
  static constexpr int M = 2 * NM;                 // trace coefficients of one cell on one facet
  static constexpr int G = 6;                      // threads per cell in the apply (3 facets x 2)
  static constexpr int R1 = NU + 3 * M;            // rows of the pass-1 matrix
  static constexpr int RG1 = (R1 + G - 1) / G;     // pass-1 rows per thread
  static constexpr int NQ1 = (RG1 * NU + 3) / 4;   // pass-1 quads per thread
  static constexpr int NQW = NM * NM;              // W quads per thread: nm rows of 2m = 4 nm entries
  static constexpr int RG = (NU + G - 1) / G;      // H rows per thread
  static constexpr int NQH = (RG * 3 * M + 3) / 4; // H quads per thread
  __host__ __device__ static long w_off(long nc32) { return nc32 * G * NQ1 * 4; }
  __host__ __device__ static long h_off(long nc32) { return w_off(nc32) + nc32 * G * NQW * 4; }
  __host__ __device__ static long scale_off(long nc32) { return h_off(nc32) + nc32 * G * NQH * 4; }
  __host__ __device__ static long entries(long nc32) { return scale_off(nc32) + 2 * 3 * nc32; }
  __device__ static long q(long e, int g, int nq, int i) { return (((e >> 5) * G + g) * (long)nq + i) * 32 + (e & 31); }
};
// Rotation of facet f of cell e: row 0 the outward normal n, row 1 the tangent (-n_y, n_x).
__device__ __forceinline__ void facet_frame(const DMesh& m, long e, int f, double R[2][2]) {
  const long nc = m.nc;
  const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
  R[0][0] = nx; R[0][1] = ny;
  R[1][0] = -ny; R[1][1] = nx;
}

// Own-cell block of the mass-scaled Step I operator, row i = (c, s) of cell
// e: D[e][i][j] = delta_ij - (adt/det) (volume term + the own-side facet
// terms of all three facets), FP64, row-major per cell.  The same terms, in
// the same form, as step1_core with the neighbour's values set to zero.  One
// thread per (cell, row).
template <int K>
__global__ void __launch_bounds__(kBlock) k_pc_cellblock(DMesh m, DTab t, const double* __restrict__ Qs,
                                                         double delta_up, double alpha, double adt,
                                                         double* __restrict__ D) {
  using Dm = Dims<K>;
  constexpr int NS = Dm::NS, NU = Dm::NU, NQC = Dm::NQC, NQF = Dm::NQF;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nc = m.nc;
  if (tid >= nc * NU) return;
  const int e = (int)(tid % nc), i = (int)(tid / nc);
  const int c = i / NS, s = i % NS;
  // vc: the terms acting on component c alone (volume, upwind), indexed by
  // s'; pen: the normal-jump penalty, indexed by (c', s')
  double q[NU], vc[NS], pen[NU];
#pragma unroll
  for (int a = 0; a < NU; ++a) { q[a] = Qs[(long)e * NU + a]; pen[a] = 0.0; }
#pragma unroll
  for (int a = 0; a < NS; ++a) vc[a] = 0.0;
  const double det = m.geo[D_DET * nc + e];
  const double i00 = det * m.geo[D_IJ00 * nc + e], i01 = det * m.geo[D_IJ01 * nc + e];
  const double i10 = det * m.geo[D_IJ10 * nc + e], i11 = det * m.geo[D_IJ11 * nc + e];
  // volume: -(phi_s, Q*.grad phi_s') det J
  for (int qq = 0; qq < NQC; ++qq) {
    double qx = 0.0, qy = 0.0;
#pragma unroll
    for (int a = 0; a < NS; ++a) { qx += t.Bu[qq * NS + a] * q[a]; qy += t.Bu[qq * NS + a] * q[NS + a]; }
    const double w = -t.cw[qq] * t.Bu[qq * NS + s];
    const double a0 = w * (i00 * qx + i01 * qy), a1 = w * (i10 * qx + i11 * qy);
#pragma unroll
    for (int a = 0; a < NS; ++a) vc[a] += a0 * t.Gux[qq * NS + a] + a1 * t.Guy[qq * NS + a];
  }
  // own side of each facet: phi_s phi_s' (beta delta_cc' - alpha w_q n_c n_c')
#pragma unroll 1
  for (int f = 0; f < 3; ++f) {
    const bool inner = m.cf_nbx[f * nc + e] >= 0;
    const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
    const double h = m.geo[(D_H0 + f) * nc + e];
    const double ncomp = c ? ny : nx;
    for (int qq = 0; qq < NQF; ++qq) {
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        const double b = t.FBu[(f * NQF + qq) * NS + a];
        vx += b * q[a];
        vy += b * q[NS + a];
      }
      const double qn = vx * nx + vy * ny;
      const double beta = inner ? t.fw[qq] * h * (0.5 * qn - delta_up * fabs(qn)) : 0.0;
      const double ps = t.FBu[(f * NQF + qq) * NS + s];
      const double pw = alpha * t.fw[qq] * ncomp;
#pragma unroll
      for (int a = 0; a < NS; ++a) {
        const double b = ps * t.FBu[(f * NQF + qq) * NS + a];
        vc[a] += b * beta;
        pen[a] -= b * pw * nx;
        pen[NS + a] -= b * pw * ny;
      }
    }
  }
  const double sc = adt / det;
#pragma unroll
  for (int j = 0; j < NU; ++j) {
    const double own = j < NS ? (c == 0 ? vc[j % NS] : 0.0) : (c == 1 ? vc[j % NS] : 0.0);
    D[((long)e * NU + i) * NU + j] = (i == j ? 1.0 : 0.0) - sc * (own + pen[j]);
  }
}

// In-place inverse of each cell block (FP64, kept for the facet pass), and
// its FP16 products in the apply layout: A_e^{-1}, G_f and H_f.  Gauss-Jordan
// elimination without pivoting (the symmetric part of the block is positive
// definite, as for the patches), one thread per column holding it in
// registers, the pivot column and row through LDS (two buffers each, one
// barrier per pivot); then the inverse goes through LDS once more so that
// thread j can read row j for H.  NC lanes per cell, 64 / NC cells per
// workgroup.
template <int K>
struct PcInvShape {
  static constexpr int NC = Dims<K>::NU <= 32 ? 32 : 64;
  static constexpr int CPB = 64 / NC;
};
template <int K>
__global__ void __launch_bounds__(64) k_pc_cellinv(DMesh m, DTab t, double* __restrict__ D, pc_t* __restrict__ P) {
  using W = PcWood<K>;
  constexpr int NU = W::NU, NS = W::NS, NM = W::NM, M = W::M, RG1 = W::RG1, NQ1 = W::NQ1, RG = W::RG,
                NQH = W::NQH, NC = PcInvShape<K>::NC, CPB = PcInvShape<K>::CPB;
  const long nc = m.nc, nc32 = (nc + 31) / 32 * 32;
  __shared__ double scol[2][CPB][NU], srow[2][CPB][NC];
  __shared__ double sinv[CPB][NU][NU + 1];
  const int slot = threadIdx.x / NC, j = threadIdx.x % NC;
  const long e = (long)blockIdx.x * CPB + slot;
  const long ec = e < nc ? e : nc - 1;  // a spare slot inverts a copy of the last cell
  const int jc = j < NU ? j : 0;        // idle lanes carry a copy of column 0
  double col[NU];
#pragma unroll
  for (int r = 0; r < NU; ++r) col[r] = D[(ec * NU + r) * NU + jc];
#pragma unroll 1
  for (int p = 0; p < NU; ++p) {
    double* cp = scol[p & 1][slot];
    double* rp = srow[p & 1][slot];
    if (j == p) {
#pragma unroll
      for (int r = 0; r < NU; ++r) cp[r] = col[r];
    }
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < NU; ++r) v = r == p ? col[r] : v;
    rp[j] = v;
    __syncthreads();
    // branch-free update: the pivot column in registers, one select per row
    double cpv[NU];
#pragma unroll
    for (int r = 0; r < NU; ++r) cpv[r] = cp[r];
    const double d = 1.0 / cp[p];
    const bool piv = j == p;
    const double a = piv ? d : rp[j] * d;
#pragma unroll
    for (int r = 0; r < NU; ++r) col[r] = r == p ? a : (piv ? 0.0 : col[r]) - cpv[r] * a;
  }
  if (j < NU) {
#pragma unroll
    for (int r = 0; r < NU; ++r) sinv[slot][r][j] = col[r];
  }
  __syncthreads();
  if (e >= nc || j >= NU) return;
  auto put1 = [&](int row, double v) {  // entry (row, j) of the pass-1 matrix
    const int flat = (row % RG1) * NU + j;
    P[4 * W::q(e, row / RG1, NQ1, flat >> 2) + (flat & 3)] = pc_store(v);
  };
#pragma unroll
  for (int r = 0; r < NU; ++r) {
    D[(e * NU + r) * NU + j] = col[r];
    put1(r, col[r]);
  }
  pc_t* PH = P + W::h_off(nc32);
#pragma unroll 1
  for (int f = 0; f < 3; ++f) {
    double R[2][2];
    facet_frame(m, e, f, R);
    for (int mm = 0; mm < NM; ++mm) {
      // column j of L_f A^{-1} (both components), then rotated: G_f[:, j]
      double lx = 0.0, ly = 0.0, hx = 0.0, hy = 0.0;
      for (int s = 0; s < NS; ++s) {
        const double l = t.TRU[(f * NM + mm) * NS + s];
        lx += l * col[s];
        ly += l * col[NS + s];
        hx += l * sinv[slot][j][s];  // row j of A^{-1} L_f^T
        hy += l * sinv[slot][j][NS + s];
      }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        put1(NU + f * M + h * NM + mm, R[h][0] * lx + R[h][1] * ly);
        const int flat = (j % RG) * 3 * M + f * M + h * NM + mm;
        PH[4 * W::q(e, j / RG, NQH, flat >> 2) + (flat & 3)] = pc_store(R[h][0] * hx + R[h][1] * hy);
      }
    }
  }
}

// One wave per interior facet: T_side = A_side^{-1} L^T from the two cell
// inverses (read from global memory, each row once), S_side = L T_side, the
// coupling Kf from the facet rule (the same terms as the patch entries:
// upwind weight on the own component, normal-jump penalty on both, scaled by
// adt / det of the row cell), then [I + Kf S | Kf] reduced by Gauss-Jordan
// elimination with partial pivoting (I + Kf S need not be diagonally
// dominant; the pivot row found by a wave reduction, the first of equal
// magnitudes), and each cell's rows of M_F, rotated into the facet frames,
// stored with their scale.  Wall facets return at once.
template <int K>
__global__ void __launch_bounds__(64) k_pc_facet(DMesh m, DTab t, const double* __restrict__ Qs, double delta_up,
                                                 double alpha, double adt, const double* __restrict__ Ai,
                                                 pc_t* __restrict__ P) {
  using Dm = Dims<K>;
  using W = PcWood<K>;
  constexpr int NS = Dm::NS, NU = Dm::NU, NQF = Dm::NQF, NM = W::NM, M = W::M, M2 = 2 * M, NQW = W::NQW;
  const int F = blockIdx.x;
  const long nc = m.nc, nc32 = (nc + 31) / 32 * 32;
  const int Km = m.fc_cell[m.nF + F];
  if (Km < 0) return;  // uniform over the workgroup
  const int Kp = m.fc_cell[F];
  const int fp = m.fc_f[F], fm = m.fc_f[m.nF + F];
  const int rev = (m.cf_nbx[fp * nc + Kp] & 1);
  auto cell = [&](int side) { return side ? Km : Kp; };
  auto lf = [&](int side) { return side ? fm : fp; };
  __shared__ double sT[2][NU][M];
  __shared__ double sS[2][M][M];
  __shared__ double sa[M2][2 * M2 + 1];
  __shared__ double sw[M][M2];
  __shared__ double sbeta[2][NQF], scp[M2];
  const int tid = threadIdx.x;
  static_assert(M2 <= 64, "one lane per row of the facet system");
  if (tid < 2 * NQF) {  // upwind weights of both sides at their own facet points
    const int side = tid / NQF, qq = tid % NQF;
    const int e = cell(side), f = lf(side);
    const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
    const double hf = m.geo[(D_H0 + f) * nc + e];
    double vx = 0.0, vy = 0.0;
    for (int a = 0; a < NS; ++a) {
      const double b = t.FBu[(f * NQF + qq) * NS + a];
      vx += b * Qs[(long)e * NU + a];
      vy += b * Qs[(long)e * NU + NS + a];
    }
    const double qn = vx * nx + vy * ny;
    sbeta[side][qq] = t.fw[qq] * hf * (0.5 * qn - delta_up * fabs(qn));
  }
  // T = A^{-1} L^T (rows (c, s), columns (c', m')): lane x holds row i of
  // one side's inverse, component c2, and forms its NM entries
  for (int x = tid; x < 2 * NU * 2; x += 64) {
    const int side = x / (NU * 2), i = (x / 2) % NU, c2 = x % 2, f = lf(side);
    const double* arow = Ai + ((long)cell(side) * NU + i) * NU + c2 * NS;
    double a[NS];
#pragma unroll
    for (int s2 = 0; s2 < NS; ++s2) a[s2] = arow[s2];
#pragma unroll
    for (int m2 = 0; m2 < NM; ++m2) {
      double v = 0.0;
#pragma unroll
      for (int s2 = 0; s2 < NS; ++s2) v += a[s2] * t.TRU[(f * NM + m2) * NS + s2];
      sT[side][i][c2 * NM + m2] = v;
    }
  }
  // Kf into the right half of the augmented matrix
  for (int x = tid; x < M2 * M2; x += 64) {
    const int r = x / M2, jj = x % M2, a = r / M, b = jj / M;
    double v = 0.0;
    if (a != b) {
      const int e = cell(a), f = lf(a);
      const int c = (r % M) / NM, mr = (r % M) % NM, c2 = (jj % M) / NM, mc = (jj % M) % NM;
      const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
      const double nn = (c ? ny : nx) * (c2 ? ny : nx);
      for (int qq = 0; qq < NQF; ++qq) {
        const double coef = (c == c2 ? sbeta[a][qq] : 0.0) - alpha * t.fw[qq] * nn;
        v += t.NUB[qq * NM + mr] * t.NUB[(rev ? NQF - 1 - qq : qq) * NM + mc] * coef;
      }
      v *= adt / m.geo[D_DET * nc + e];
    }
    sa[r][M2 + jj] = v;
  }
  __syncthreads();
  // S = L T
  for (int x = tid; x < 2 * M * M; x += 64) {
    const int side = x / (M * M), r = (x / M) % M, cm = x % M;
    const int c = r / NM, mr = r % NM, f = lf(side);
    double v = 0.0;
    for (int s = 0; s < NS; ++s) v += t.TRU[(f * NM + mr) * NS + s] * sT[side][c * NS + s][cm];
    sS[side][r][cm] = v;
  }
  __syncthreads();
  // left half: I + Kf S (S block diagonal, Kf off-diagonal)
  for (int x = tid; x < M2 * M2; x += 64) {
    const int r = x / M2, jj = x % M2, a = r / M, b = jj / M;
    double v = r == jj ? 1.0 : 0.0;
    if (a != b)
      for (int i = 0; i < M; ++i) v += sa[r][M2 + b * M + i] * sS[b][i][jj % M];
    sa[r][jj] = v;
  }
  __syncthreads();
#pragma unroll 1
  for (int p = 0; p < M2; ++p) {
    // pivot row: the largest |sa[r][p]| over r >= p, the first of equal ones
    double bv = tid >= p && tid < M2 ? fabs(sa[tid][p]) : -1.0;
    int pv = tid;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double ov = __shfl_xor(bv, o, 64);
      const int oi = __shfl_xor(pv, o, 64);
      if (ov > bv || (ov == bv && oi < pv)) { bv = ov; pv = oi; }
    }
    if (pv != p)
      for (int j = tid; j < 2 * M2; j += 64) {
        const double v = sa[p][j];
        sa[p][j] = sa[pv][j];
        sa[pv][j] = v;
      }
    __syncthreads();
    for (int r = tid; r < M2; r += 64) scp[r] = sa[r][p];
    __syncthreads();
    const double d = 1.0 / scp[p];
    for (int j = tid; j < 2 * M2; j += 64) {
      const double rowp = sa[p][j] * d;
      for (int r = 0; r < M2; ++r) sa[r][j] = r == p ? rowp : sa[r][j] - scp[r] * rowp;
    }
    __syncthreads();
  }
  // M_F = right half.  Side a keeps rows [a M, (a+1) M), its own columns
  // first; rows and columns rotated by the frame of the side they belong to.
  float* scale = reinterpret_cast<float*>(P + W::scale_off(nc32));
  pc_t* PW = P + W::w_off(nc32);
#pragma unroll 1
  for (int a = 0; a < 2; ++a) {
    double Ra[2][2], Rb[2][2];
    facet_frame(m, cell(a), lf(a), Ra);
    facet_frame(m, cell(1 - a), lf(1 - a), Rb);
    double mx = 0.0;
    for (int x = tid; x < M * M2; x += 64) {
      const int r = x / M2, j = x % M2;
      const int h = r / NM, mr = r % NM, own = j < M, h2 = (j % M) / NM, mc = (j % M) % NM;
      const int b = own ? a : 1 - a;
      double v = 0.0;
      for (int c = 0; c < 2; ++c)
        for (int c2 = 0; c2 < 2; ++c2)
          v += Ra[h][c] * sa[a * M + c * NM + mr][M2 + b * M + c2 * NM + mc] * (own ? Ra[h2][c2] : Rb[h2][c2]);
      sw[r][j] = v;
      mx = fmax(mx, fabs(v));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    __syncthreads();
    const double sc = mx > 0.0 ? ldexp(1.0, ilogb(mx) - 13) : 1.0;  // max |W| / sc < 2^14
    const long e = cell(a);
    const int f = lf(a);
    if (tid == 0) scale[f * nc32 + e] = (float)sc;
    for (int x = tid; x < M * M2; x += 64) {
      const int r = x / M2, j = x % M2;
      const int h = r / NM, mr = r % NM, flat = mr * M2 + j;
      PW[4 * W::q(e, 2 * f + h, NQW, flat >> 2) + (flat & 3)] = pc_store(sw[r][j] / sc);
    }
    __syncthreads();
  }
}

// z = B r, first pass: the stacked rows [A_e^{-1}; G_0; G_1; G_2] applied to
// r_e, G threads per cell, thread g the rows [g RG1, (g+1) RG1): into X
// the NU entries of s = A_e^{-1} r_e, then the 3m rotated traces.  X is
// structure-of-arrays, row i of cell e at i * nc + e.  Both passes compute
// in the type of the Krylov vectors: in FP32 the preconditioner's rounding
// would change with its input at the 1e-7 level, and BiCGStab, which
// assumes a fixed preconditioner, slows down on the way to 1e-10.
template <int K, typename TX>
__global__ void __launch_bounds__(kBlock) k_pc_pass1(long nc, const pc_t* __restrict__ P, const TX* __restrict__ r,
                                                     TX* __restrict__ X) {
  using W = PcWood<K>;
  constexpr int NU = W::NU, G = W::G, RG1 = W::RG1, NQ1 = W::NQ1, R1 = W::R1;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tile = tid / (G * 32);
  const int rem = (int)(tid % (G * 32));
  const int g = rem >> 5;
  const long e = tile * 32 + (rem & 31);
  if (e >= nc) return;
  TX rv[NU], acc[RG1];
#pragma unroll
  for (int a = 0; a < NU; ++a) rv[a] = r[(long)a * nc + e];
#pragma unroll
  for (int a = 0; a < RG1; ++a) acc[a] = 0;
  const f16x4* A4 = reinterpret_cast<const f16x4*>(P);
#pragma unroll
  for (int q = 0; q < NQ1; ++q) {
    const f16x4 b = __builtin_nontemporal_load(&A4[W::q(e, g, NQ1, q)]);
    const TX bv[4] = {(TX)b.x, (TX)b.y, (TX)b.z, (TX)b.w};
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int flat = 4 * q + u;
      if (flat < RG1 * NU) acc[flat / NU] += bv[u] * rv[flat % NU];
    }
  }
#pragma unroll
  for (int a = 0; a < RG1; ++a)
    if (g * RG1 + a < R1) X[(long)(g * RG1 + a) * nc + e] = acc[a];
}

// Second pass, one workgroup per tile of 32 cells (G half-wave groups):
// thread g = 2 f + h applies the frame-component-h rows of W_f to the own
// and the neighbour's rotated traces on facet f (LDS exchange), then thread
// g writes its rows of n_int s - sum_f H_f c_f.
template <int K, typename TX>
__global__ void __launch_bounds__(PcWood<K>::G * 32) k_pc_pass2(DMesh m, const pc_t* __restrict__ P,
                                                                const TX* __restrict__ X, TX* __restrict__ z) {
  using W = PcWood<K>;
  constexpr int NU = W::NU, NM = W::NM, M = W::M, RG = W::RG, NQW = W::NQW, NQH = W::NQH;
  const long nc = m.nc, nc32 = (nc + 31) / 32 * 32;
  const int lane = threadIdx.x & 31, g = threadIdx.x >> 5;
  const long e = (long)blockIdx.x * 32 + lane;
  const long ec = e < nc ? e : nc - 1;
  const int f = g >> 1, h = g & 1;
  __shared__ TX sC[3][M][32];
  {
    const int nbx = m.cf_nbx[f * nc + ec];
    TX cc[NM];
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) cc[mm] = 0;
    if (nbx >= 0) {
      const long x = nbx >> 3;
      const int fx = (nbx >> 1) & 3;
      TX tau[2 * M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        tau[j] = X[(long)(NU + f * M + j) * nc + ec];
        tau[M + j] = X[(long)(NU + fx * M + j) * nc + x];
      }
      const f16x4* W4 = reinterpret_cast<const f16x4*>(P + W::w_off(nc32));
#pragma unroll
      for (int q = 0; q < NQW; ++q) {
        const f16x4 b = __builtin_nontemporal_load(&W4[W::q(ec, g, NQW, q)]);
        const TX bv[4] = {(TX)b.x, (TX)b.y, (TX)b.z, (TX)b.w};
#pragma unroll
        for (int v = 0; v < 4; ++v) cc[(4 * q + v) / (2 * M)] += bv[v] * tau[(4 * q + v) % (2 * M)];
      }
      const TX sc = reinterpret_cast<const float*>(P + W::scale_off(nc32))[f * nc32 + ec];
#pragma unroll
      for (int mm = 0; mm < NM; ++mm) cc[mm] *= sc;
    }
#pragma unroll
    for (int mm = 0; mm < NM; ++mm) sC[f][h * NM + mm][lane] = cc[mm];
  }
  __syncthreads();
  if (e >= nc) return;
  TX c[3 * M], acc[RG];
#pragma unroll
  for (int j = 0; j < 3 * M; ++j) c[j] = sC[j / M][j % M][lane];
#pragma unroll
  for (int a = 0; a < RG; ++a) acc[a] = 0;
  const f16x4* H4 = reinterpret_cast<const f16x4*>(P + W::h_off(nc32));
#pragma unroll
  for (int q = 0; q < NQH; ++q) {
    const f16x4 b = __builtin_nontemporal_load(&H4[W::q(e, g, NQH, q)]);
    const TX bv[4] = {(TX)b.x, (TX)b.y, (TX)b.z, (TX)b.w};
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int flat = 4 * q + v;
      if (flat < RG * 3 * M) acc[flat / (3 * M)] += bv[v] * c[flat % (3 * M)];
    }
  }
  const TX nint = (TX)((m.cf_nbx[e] >= 0) + (m.cf_nbx[nc + e] >= 0) + (m.cf_nbx[2 * nc + e] >= 0));
#pragma unroll
  for (int a = 0; a < RG; ++a) {
    const int row = g * RG + a;
    if (row < NU) z[(long)row * nc + e] = nint * X[(long)row * nc + e] - acc[a];
  }
}

// ============================================================== launchers
void launch_step1_data(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, void* V, bool v32,
                       void* beta, bool b32) {
  if (m.dim == 3) {  // tetrahedra: cell-major V [nc][ns][ns] and beta [nc][4][nq_facet], one type for both
    if (v32 != b32) throw std::invalid_argument("launch_step1_data: V and beta of one type on tetrahedra");
    return launch3_prep(k, st, m, t.t3, Qs, delta_up, V, beta, v32);
  }
  const int nb = nblocks((long)m.nc);
  if (v32) {
    HDG_DISPATCH(k, (k_step1_field<KK, float><<<nb, kBlock, 0, st>>>(m, t, Qs, (float*)V)));
  } else {
    HDG_DISPATCH(k, (k_step1_field<KK, double><<<nb, kBlock, 0, st>>>(m, t, Qs, (double*)V)));
  }
  if (b32) {
    HDG_DISPATCH(k, (k_step1_beta<KK, float><<<nblocks(3L * m.nc), kBlock, 0, st>>>(m, t, Qs, delta_up, (float*)beta)));
  } else {
    HDG_DISPATCH(k, (k_step1_beta<KK, double><<<nblocks(3L * m.nc), kBlock, 0, st>>>(m, t, Qs, delta_up,
                                                                                    (double*)beta)));
  }
}
template <int DOT, typename TV, typename TX, int BS>
static void apply_soa_bs(int k, hipStream_t st, DMesh m, DTab t, const TV* V, const TX* beta, double alpha,
                         double adt, const TX* x, const TX* w, const TX* sd, TX* out, double* part, int xcd) {
  const int nb = apply_soa_blocks(m.nc, BS);
  HDG_DISPATCH(k, (k_apply_soa<KK, DOT, TV, BS, TX><<<nb, BS, 0, st>>>(m, t, V, beta, alpha, adt, x, w, sd, out,
                                                                       part, xcd)));
}
template <int DOT, typename TV, typename TX>
static void apply_soa_d(int k, hipStream_t st, Step1Launch ln, DMesh m, DTab t, const TV* V, const TX* beta,
                        double alpha, double adt, const TX* x, const TX* w, const TX* sd, TX* out, double* part) {
  switch (ln.block) {
    case 64: apply_soa_bs<DOT, TV, TX, 64>(k, st, m, t, V, beta, alpha, adt, x, w, sd, out, part, ln.xcd); break;
    case 128: apply_soa_bs<DOT, TV, TX, 128>(k, st, m, t, V, beta, alpha, adt, x, w, sd, out, part, ln.xcd); break;
    default: apply_soa_bs<DOT, TV, TX, 256>(k, st, m, t, V, beta, alpha, adt, x, w, sd, out, part, ln.xcd); break;
  }
}
template <typename TV, typename TX>
static void apply_soa_t(int k, hipStream_t st, Step1Launch ln, int dot, DMesh m, DTab t, const TV* V, const TX* beta,
                        double alpha, double adt, const TX* x, const TX* w, const TX* sd, TX* out, double* part) {
  if (dot == 0) apply_soa_d<0, TV, TX>(k, st, ln, m, t, V, beta, alpha, adt, x, w, sd, out, part);
  else if (dot == 1) apply_soa_d<1, TV, TX>(k, st, ln, m, t, V, beta, alpha, adt, x, w, sd, out, part);
  else if (dot == 2) apply_soa_d<2, TV, TX>(k, st, ln, m, t, V, beta, alpha, adt, x, w, sd, out, part);
  else apply_soa_d<3, TV, TX>(k, st, ln, m, t, V, beta, alpha, adt, x, w, sd, out, part);
}
void launch_apply_soa(int k, hipStream_t st, Step1Launch ln, int dot, DMesh m, DTab t, const void* V, bool v32,
                      const void* beta, double alpha, double adt, const void* x, const void* w, void* out,
                      double* part, const void* sd, bool x32) {
  if (m.dim == 3) {
    if (v32 != x32) throw std::invalid_argument("launch_apply_soa: V and the vectors of one type on tetrahedra");
    return launch3_apply(k, st, 0, dot, m, t.t3, V, beta, alpha, adt, x, nullptr, nullptr, nullptr, out, w, sd,
                         part, apply_soa_blocks(m.nc, ln.block), x32);
  }
  if (x32) {  // FP32 vectors and arithmetic (the field is FP32 too)
    apply_soa_t(k, st, ln, dot, m, t, (const float*)V, (const float*)beta, alpha, adt, (const float*)x,
                (const float*)w, (const float*)sd, (float*)out, part);
  } else if (v32) {
    apply_soa_t(k, st, ln, dot, m, t, (const float*)V, (const double*)beta, alpha, adt, (const double*)x,
                (const double*)w, (const double*)sd, (double*)out, part);
  } else {
    apply_soa_t(k, st, ln, dot, m, t, (const double*)V, (const double*)beta, alpha, adt, (const double*)x,
                (const double*)w, (const double*)sd, (double*)out, part);
  }
}
int apply_soa_blocks(long nc, int block) { return (int)((2L * nc + block - 1) / block); }
void launch_bicg_s(hipStream_t st, long n, int np, const double* part, double* sc, const void* r, const void* v,
                   void* s, bool x32) {
  if (x32) k_bicg_s<float><<<kVecBlocks, kBlock, 0, st>>>(n, np, part, sc, (const float*)r, (const float*)v, (float*)s);
  else k_bicg_s<double><<<kVecBlocks, kBlock, 0, st>>>(n, np, part, sc, (const double*)r, (const double*)v, (double*)s);
}
void launch_bicg_xrp(hipStream_t st, long n, int np, const double* part2, double* sc, const void* s, const void* tv,
                     const void* v, const void* ph, const void* sh, void* x, void* r, void* p, double* part,
                     bool x32) {
  if (x32) {
    k_bicg_xrp<float><<<kVecBlocks, kBlock, 0, st>>>(n, np, part2, sc, (const float*)s, (const float*)tv,
                                                     (const float*)v, (const float*)ph, (const float*)sh, (float*)x,
                                                     (float*)r, (float*)p, part);
  } else {
    k_bicg_xrp<double><<<kVecBlocks, kBlock, 0, st>>>(n, np, part2, sc, (const double*)s, (const double*)tv,
                                                      (const double*)v, (const double*)ph, (const double*)sh,
                                                      (double*)x, (double*)r, (double*)p, part);
  }
}
void launch_bicg_init(hipStream_t st, double* sc) { k_bicg_init<<<1, 64, 0, st>>>(sc); }
void launch_to_soa(int k, hipStream_t st, DMesh m, int inv_det, const double* x, void* y, bool x32) {
  if (m.dim == 3) {  // tetrahedra: the Step I vectors stay cell-major (FP32 in the mixed mode)
    if (inv_det) throw std::invalid_argument("launch_to_soa: inv_det is not available on tetrahedra");
    const long n = (long)m.nc * 3 * (k + 2) * (k + 3) * (k + 4) / 6;
    if (x32) return launch3_convert(st, n, x, false, y, true);
    return launch_vcopy(st, n, x, y, false);
  }
  const int nb = nblocks((long)m.nc * (k + 2) * (k + 3));
  if (x32) { HDG_DISPATCH(k, (k_to_soa<KK, float><<<nb, kBlock, 0, st>>>(m, inv_det, x, (float*)y))); }
  else { HDG_DISPATCH(k, (k_to_soa<KK, double><<<nb, kBlock, 0, st>>>(m, inv_det, x, (double*)y))); }
}
void launch_to_aos(int k, hipStream_t st, DMesh m, const void* x, double* y, bool x32) {
  if (m.dim == 3) {
    const long n = (long)m.nc * 3 * (k + 2) * (k + 3) * (k + 4) / 6;
    if (x32) return launch3_convert(st, n, x, true, y, false);
    return launch_copy(st, n, (const double*)x, y);
  }
  const int nb = nblocks((long)m.nc * (k + 2) * (k + 3));
  if (x32) { HDG_DISPATCH(k, (k_to_aos<KK, float><<<nb, kBlock, 0, st>>>(m, (const float*)x, y))); }
  else { HDG_DISPATCH(k, (k_to_aos<KK, double><<<nb, kBlock, 0, st>>>(m, (const double*)x, y))); }
}
void launch_vcopy(hipStream_t st, long n, const void* x, void* y, bool x32) {
  if (x32) k_vcopy<float><<<nblocks(n), kBlock, 0, st>>>(n, (const float*)x, (float*)y);
  else k_vcopy<double><<<nblocks(n), kBlock, 0, st>>>(n, (const double*)x, (double*)y);
}
void launch_vfill(hipStream_t st, long n, double v, void* y, bool x32) {
  if (x32) k_vfill<float><<<nblocks(n), kBlock, 0, st>>>(n, v, (float*)y);
  else k_vfill<double><<<nblocks(n), kBlock, 0, st>>>(n, v, (double*)y);
}
void launch_vaxpby(hipStream_t st, long n, double a, const void* x, double b, void* y, bool x32) {
  if (x32) k_vaxpby<float><<<nblocks(n), kBlock, 0, st>>>(n, a, (const float*)x, b, (float*)y);
  else k_vaxpby<double><<<nblocks(n), kBlock, 0, st>>>(n, a, (const double*)x, b, (double*)y);
}
void launch_vdot(hipStream_t st, long n, const void* a, const void* b, double* part, bool x32) {
  if (x32) k_vdot<float><<<kRedBlocks, kBlock, 0, st>>>(n, (const float*)a, (const float*)b, part);
  else k_vdot<double><<<kRedBlocks, kBlock, 0, st>>>(n, (const double*)a, (const double*)b, part);
}
// Facet-patch preconditioner of the Step I operator for the Q* and adt of a
// stage, in Woodbury form: cell blocks (D, FP64 scratch of nc*NU*NU doubles,
// left holding their inverses), then the FP16 cell inverses and facet
// corrections (Binv, pc_entries(k, nc) FP16 entries).
void launch_pc_build(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, double alpha,
                     double adt, double* D, void* Binv) {
  HDG_DISPATCH(k, (k_pc_cellblock<KK><<<nblocks((long)m.nc * Dims<KK>::NU), kBlock, 0, st>>>(m, t, Qs, delta_up,
                                                                                              alpha, adt, D)));
  HDG_DISPATCH(k, (k_pc_cellinv<KK><<<(m.nc + PcInvShape<KK>::CPB - 1) / PcInvShape<KK>::CPB, 64, 0, st>>>(
                      m, t, D, (pc_t*)Binv)));
  HDG_DISPATCH(k, (k_pc_facet<KK><<<m.nF, 64, 0, st>>>(m, t, Qs, delta_up, alpha, adt, D, (pc_t*)Binv)));
}
// z = B r: the first pass into the scratch X (pc_scratch(k, nc) entries
// of the vectors' type), then the trace correction
void launch_pc_apply(int k, hipStream_t st, DMesh m, const void* Binv, void* X, const void* r, void* z, bool x32) {
  const long nc32 = ((long)m.nc + 31) / 32 * 32;
  const int nb1 = nblocks(nc32 * 6), nb2 = (int)(nc32 / 32);
  if (x32) {
    HDG_DISPATCH(k, (k_pc_pass1<KK, float><<<nb1, kBlock, 0, st>>>(m.nc, (const pc_t*)Binv, (const float*)r,
                                                                    (float*)X)));
    HDG_DISPATCH(k, (k_pc_pass2<KK, float><<<nb2, PcWood<KK>::G * 32, 0, st>>>(m, (const pc_t*)Binv, (const float*)X,
                                                                                (float*)z)));
  } else {
    HDG_DISPATCH(k, (k_pc_pass1<KK, double><<<nb1, kBlock, 0, st>>>(m.nc, (const pc_t*)Binv, (const double*)r,
                                                                     (double*)X)));
    HDG_DISPATCH(k, (k_pc_pass2<KK, double><<<nb2, PcWood<KK>::G * 32, 0, st>>>(m, (const pc_t*)Binv,
                                                                                 (const double*)X, (double*)z)));
  }
}
long pc_scratch(int k, long nc) {
  HDG_DISPATCH(k, return nc * PcWood<KK>::R1);
  return 0;
}
long pc_entries(int k, long nc) {
  const long nc32 = (nc + 31) / 32 * 32;
  HDG_DISPATCH(k, return PcWood<KK>::entries(nc32));
  return 0;
}
}  // namespace hdg
