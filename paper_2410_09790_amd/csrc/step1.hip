// gfx950 kernels of the tentative-velocity solve (Algorithm 2, Step I): the
// per-stage cell data of the Step I form f_im(., .; Q*) of eq. (f_impl), the
// mass-scaled operator on structure-of-arrays vectors and the BiCGStab
// vector kernels.
#include <hip/hip_runtime.h>

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

// Per-cell data of the Step I operator are stored in tiles of 32 cells
// (one wave of the two-threads-per-cell kernels): entry j of cell e sits at
// ((e/32)*nj + j)*32 + e%32.  A wave then reads 256 contiguous bytes per
// entry and one contiguous block overall, which keeps the number of DRAM
// streams small.  Arrays hold ceil(nc/32)*32 cells.
__device__ __forceinline__ long tile_idx(long e, int j, int nj) { return ((e >> 5) * nj + j) * 32 + (e & 31); }

// The cell matrices are stored as pairs of adjacent row entries, so that one
// load per lane brings two of them (16 bytes in FP64, 8 in FP32): row s of
// cell e holds NP2 = floor(NS/2) pairs, pair pi of row s at
// pair(e, s, pi) in units of pairs, in tiles of 32 cells; when NS is odd the
// last entry of every row follows all pairs, at tail(nc) + tile_idx(e, s, NS)
// in units of entries.  The array holds ceil(nc/32)*32*NS*NS entries either way.
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename TV> struct Pair2;
template <> struct Pair2<float> { using T = f32x2; };
template <> struct Pair2<double> { using T = f64x2; };
template <int K>
struct VPairs {
  static constexpr int NS = Dims<K>::NS;
  static constexpr int NP2 = NS / 2;
  __device__ static long pair(long e, int s, int pi) { return ((e >> 5) * (long)(NS * NP2) + s * NP2 + pi) * 32 + (e & 31); }
  __device__ static long tail(long nc) { return ((nc + 31) >> 5) * 32 * (long)NS * (2 * NP2); }
};

// Per-cell volume matrix of the Step I form, for the Q* of a stage:
//   V[s][s'] = -sum_q w_q phi_s(q) (Q*(q) . grad phi_s'(q)) det J
// (the volume term -(Q*.grad x, w) of eq. (f_impl) acts on each velocity
// component alike), entry s*NS + s' in tiles.  TV is the storage type: FP64,
// or FP32 in the mixed-precision mode (the operator still computes in FP64).
// One thread per (cell, row s).
template <int K, typename TV>
__global__ void __launch_bounds__(kBlock) k_step1_matrix(DMesh m, DTab t, const double* __restrict__ Qs,
                                                         TV* __restrict__ V) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nc = m.nc;
  if (tid >= nc * NS) return;
  const int e = (int)(tid % nc), s = (int)(tid / nc);
  double q[NU], row[NS];
#pragma unroll
  for (int i = 0; i < NU; ++i) q[i] = Qs[(long)e * NU + i];
#pragma unroll
  for (int i = 0; i < NS; ++i) row[i] = 0.0;
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
    const double w = -t.cw[qq] * t.Bu[qq * NS + s];
    const double a0 = w * (i00 * qx + i01 * qy), a1 = w * (i10 * qx + i11 * qy);
#pragma unroll
    for (int i = 0; i < NS; ++i) row[i] += a0 * t.Gux[qq * NS + i] + a1 * t.Guy[qq * NS + i];
  }
  using TV2 = typename Pair2<TV>::T;
  TV2* V2 = reinterpret_cast<TV2*>(V);
#pragma unroll
  for (int pi = 0; pi < VPairs<K>::NP2; ++pi) {
    TV2 v;
    v.x = (TV)row[2 * pi];
    v.y = (TV)row[2 * pi + 1];
    V2[VPairs<K>::pair(e, s, pi)] = v;
  }
  if constexpr (NS & 1) V[VPairs<K>::tail(nc) + tile_idx(e, s, NS)] = (TV)row[NS - 1];
}

// Upwind weights of the Step I facet term at the facet points, for the Q*
// of a stage: beta = w_q h (Q*.n/2 - delta_up |Q*.n|) on interior facets,
// 0 on walls, entry f*NQF + q in tiles.  One thread per (cell, facet).
template <int K>
__global__ void __launch_bounds__(kBlock) k_step1_beta(DMesh m, DTab t, const double* __restrict__ Qs,
                                                       double delta_up, double* __restrict__ beta) {
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
    beta[tile_idx(e, f * NQF + qq, 3 * NQF)] = inner ? t.fw[qq] * h * (0.5 * qn - delta_up * fabs(qn)) : 0.0;
  }
}

// The Step I form f_im(w, x; Q*) of eq. (f_impl) for one cell e and one
// velocity component c on structure-of-arrays data x[(c*NS + s)*nc + e]:
// the volume term through the cell matrix V, and per facet the upwinded
// advective jump term beta(q) [[x]] (beta = w_q h (Q*.n/2 - delta_up
// |Q*.n|) at the facet points, precomputed per stage in tiles, entry
// f*NQF + q, zero on walls) and the normal-jump penalty
// alpha ([[x]].n)(w.n).  Two threads per cell (lanes 2i, 2i+1, one per
// component) exchange their components of the jump with pair_swap.  y
// receives the result in reference scaling (the caller multiplies by
// adt/det).  The neighbour's input value at structure-of-arrays index idx
// is nb(idx); sFBu is the facet trace table staged in LDS.
template <int K, typename TV, typename NbVal>
__device__ __forceinline__ void step1_core(const DMesh& m, const DTab& t, const double* sFBu,
                                           const TV* __restrict__ V, const double* __restrict__ beta, long nc,
                                           int e, int c, double alpha, const double (&xv)[Dims<K>::NS],
                                           double (&y)[Dims<K>::NS], const NbVal& nb) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NQF = D::NQF;
  // volume: the two lanes of a cell split the rows of V (lane c takes rows
  // 2r + c) and apply them to both components, so that every lane loads
  // distinct entries; the partner's results come back through pair_swap.
  // V and the upwind weights are read once per application: non-temporal
  // loads keep them from evicting the velocity vectors (read again by the
  // neighbouring cells) from the caches.
  {
    using TV2 = typename Pair2<TV>::T;
    const long vtail = VPairs<K>::tail(nc);
    double xo[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) xo[i] = pair_swap(xv[i]);
#pragma unroll
    for (int r = 0; r < (NS + 1) / 2; ++r) {
      const int s = 2 * r + c < NS ? 2 * r + c : NS - 1;
      double am = 0.0, ao = 0.0;
      const TV2* V2 = reinterpret_cast<const TV2*>(V);
#pragma unroll
      for (int pi = 0; pi < VPairs<K>::NP2; ++pi) {
        const TV2 v = __builtin_nontemporal_load(&V2[VPairs<K>::pair(e, s, pi)]);
        am += (double)v.x * xv[2 * pi];
        ao += (double)v.x * xo[2 * pi];
        am += (double)v.y * xv[2 * pi + 1];
        ao += (double)v.y * xo[2 * pi + 1];
      }
      if constexpr (NS & 1) {
        const double v = (double)__builtin_nontemporal_load(&V[vtail + tile_idx(e, s, NS)]);
        am += v * xv[NS - 1];
        ao += v * xo[NS - 1];
      }
      const double recv = pair_swap(ao);
      if (2 * r + 1 < NS) {
        y[2 * r] = c ? recv : am;
        y[2 * r + 1] = c ? am : recv;
      } else {
        y[2 * r] = c ? recv : am;
      }
    }
  }
  int nbx[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) nbx[f] = m.cf_nbx[f * nc + e];
#pragma unroll 1
  for (int f = 0; f < 3; ++f) {
    const int en = nbx[f] >= 0 ? nbx[f] >> 3 : -1;
    const int fn = nbx[f] >= 0 ? (nbx[f] >> 1) & 3 : 0;
    const int rev = nbx[f] >= 0 ? nbx[f] & 1 : 0;
    const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
    const double ncomp = c ? ny : nx;
    double xn[NS], bq[NQF];
#pragma unroll
    for (int qq = 0; qq < NQF; ++qq) bq[qq] = __builtin_nontemporal_load(&beta[tile_idx(e, f * NQF + qq, 3 * NQF)]);
    if (en >= 0) {
#pragma unroll
      for (int s = 0; s < NS; ++s) xn[s] = nb((long)(c * NS + s) * nc + en);
    } else {
#pragma unroll
      for (int s = 0; s < NS; ++s) xn[s] = 0.0;
    }
#pragma unroll
    for (int qq = 0; qq < NQF; ++qq) {
      const int qn = rev ? NQF - 1 - qq : qq;
      double j = 0.0, jn = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        j += t.FBu[(f * NQF + qq) * NS + s] * xv[s];
        jn += sFBu[(fn * NQF + qn) * NS + s] * xn[s];
      }
      j -= jn;
      const double jo = pair_swap(j);
      const double jdotn = c ? (jo * nx + j * ny) : (j * nx + jo * ny);
      const double con = bq[qq] * j - alpha * t.fw[qq] * jdotn * ncomp;
#pragma unroll
      for (int s = 0; s < NS; ++s) y[s] += t.FBu[(f * NQF + qq) * NS + s] * con;
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
template <int K>
__device__ __forceinline__ void stage_fbu(const DTab& t, double* sFBu) {
  constexpr int N = 3 * Dims<K>::NQF * Dims<K>::NS;
  for (int i = threadIdx.x; i < N; i += blockDim.x) sFBu[i] = t.FBu[i];
  __syncthreads();
}

// out = x - (adt/det) f_im(., x; Q*): the mass-scaled Step I operator on
// structure-of-arrays vectors (two threads per cell), with per-block
// partial sums (nb = gridDim.x sets of partials at part + i*nb):
//   DOT 0: none;  DOT 1: w.out;  DOT 2: out.x, out.out, w.x, w.out.
// In BiCGStab, DOT 1 gives rh.v for v = A p and DOT 2 gives t.s, t.t, rh.s,
// rh.t for t = A s.  BS threads per workgroup (64, 128 or 256); xcd = 1 deals
// the cells to the XCDs in contiguous eighths (xcd_block), 0 keeps the
// hardware order.
template <int K, int DOT, typename TV, int BS>
__global__ void __launch_bounds__(BS, kStep1Waves) k_apply_soa(DMesh m, DTab t, const TV* __restrict__ V,
                                                               const double* __restrict__ beta, double alpha,
                                                               double adt, const double* __restrict__ x,
                                                               const double* __restrict__ w,
                                                               double* __restrict__ out,
                                                               double* __restrict__ part, int xcd) {
  using D = Dims<K>;
  constexpr int NS = D::NS;
  __shared__ double sFBu[3 * D::NQF * NS];
  stage_fbu<K>(t, sFBu);
  const int blk = xcd ? xcd_block() : (int)blockIdx.x;
  const long tid = (long)blk * BS + threadIdx.x;
  const long nc = m.nc;
  const int e = (int)(tid >> 1), c = (int)(tid & 1);
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  if (e < nc) {
    double xv[NS], y[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) xv[s] = x[(long)(c * NS + s) * nc + e];
    step1_core<K, TV>(m, t, sFBu, V, beta, nc, e, c, alpha, xv, y, [&](long i) { return x[i]; });
    const double sc = adt / m.geo[D_DET * nc + e];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const long idx = (long)(c * NS + s) * nc + e;
      const double o = xv[s] - sc * y[s];
      out[idx] = o;
      if (DOT == 1) d0 += w[idx] * o;
      if (DOT == 2) {
        const double wv = w[idx];
        d0 += o * xv[s];
        d1 += o * o;
        d2 += wv * xv[s];
        d3 += wv * o;
      }
    }
  }
  if (DOT >= 1) {
    d0 = block_sum_n<BS>(d0);
    if (threadIdx.x == 0) part[blk] = d0;
  }
  if (DOT == 2) {
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
__global__ void __launch_bounds__(kBlock) k_bicg_s(long n, int np, const double* __restrict__ part,
                                                   double* __restrict__ sc, const double* __restrict__ R,
                                                   const double* __restrict__ Vv, double* __restrict__ S) {
  const double rv = sum_partials(part, np);
  const bool ok = rv != 0.0 && rv == rv;
  const double al = ok ? sc[BS_RHO] / rv : 0.0;
  // n is even (2 ns doubles per cell and component pair): 16-byte accesses
  const long n2 = n >> 1;
  const double2* R2 = reinterpret_cast<const double2*>(R);
  const double2* V2 = reinterpret_cast<const double2*>(Vv);
  double2* S2 = reinterpret_cast<double2*>(S);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
    const double2 r = R2[i], v = V2[i];
    S2[i] = make_double2(r.x - al * v.x, r.y - al * v.y);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[BS_RV] = rv;
    sc[BS_ALPHA] = al;
    if (!ok) sc[BS_FLAG] = 1.0;
  }
}

__global__ void __launch_bounds__(kBlock) k_bicg_xrp(long n, int np, const double* __restrict__ part2,
                                                     double* __restrict__ sc, const double* __restrict__ S,
                                                     const double* __restrict__ Tv, const double* __restrict__ Vv,
                                                     double* __restrict__ X, double* __restrict__ R,
                                                     double* __restrict__ P, double* __restrict__ part) {
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
  const long n2 = n >> 1;  // n is even: 16-byte accesses
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
    const double2 p = reinterpret_cast<const double2*>(P)[i], s = reinterpret_cast<const double2*>(S)[i];
    const double2 t = reinterpret_cast<const double2*>(Tv)[i], v = reinterpret_cast<const double2*>(Vv)[i];
    double2 x = reinterpret_cast<const double2*>(X)[i];
    x.x += al * p.x + om * s.x;
    x.y += al * p.y + om * s.y;
    reinterpret_cast<double2*>(X)[i] = x;
    const double2 r = make_double2(s.x - om * t.x, s.y - om * t.y);
    reinterpret_cast<double2*>(R)[i] = r;
    rr += r.x * r.x + r.y * r.y;
    reinterpret_cast<double2*>(P)[i] = make_double2(r.x + be * (p.x - om * v.x), r.y + be * (p.y - om * v.y));
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
template <int K>
__global__ void k_to_soa(DMesh m, int inv_det, const double* __restrict__ x, double* __restrict__ y) {
  constexpr int NU = Dims<K>::NU;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long)m.nc * NU) return;
  const long e = tid % m.nc, i = tid / m.nc;
  const double sc = inv_det ? 1.0 / m.geo[D_DET * (long)m.nc + e] : 1.0;
  y[tid] = sc * x[e * NU + i];
}
template <int K>
__global__ void k_to_aos(DMesh m, const double* __restrict__ x, double* __restrict__ y) {
  constexpr int NU = Dims<K>::NU;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long)m.nc * NU) return;
  const long e = tid / NU, i = tid % NU;
  y[tid] = x[i * m.nc + e];
}

// ============================================================== launchers
void launch_step1_matrix(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, void* V, bool v32,
                         double* beta) {
  const int nb = nblocks((long)m.nc * (k + 2) * (k + 3) / 2);
  if (v32) {
    HDG_DISPATCH(k, (k_step1_matrix<KK, float><<<nb, kBlock, 0, st>>>(m, t, Qs, (float*)V)));
  } else {
    HDG_DISPATCH(k, (k_step1_matrix<KK, double><<<nb, kBlock, 0, st>>>(m, t, Qs, (double*)V)));
  }
  HDG_DISPATCH(k, (k_step1_beta<KK><<<nblocks(3L * m.nc), kBlock, 0, st>>>(m, t, Qs, delta_up, beta)));
}
template <int DOT, typename TV, int BS>
static void apply_soa_bs(int k, hipStream_t st, DMesh m, DTab t, const TV* V, const double* beta, double alpha,
                         double adt, const double* x, const double* w, double* out, double* part, int xcd) {
  const int nb = apply_soa_blocks(m.nc, BS);
  HDG_DISPATCH(k, (k_apply_soa<KK, DOT, TV, BS><<<nb, BS, 0, st>>>(m, t, V, beta, alpha, adt, x, w, out, part, xcd)));
}
template <int DOT, typename TV>
static void apply_soa_d(int k, hipStream_t st, Step1Launch ln, DMesh m, DTab t, const TV* V, const double* beta,
                        double alpha, double adt, const double* x, const double* w, double* out, double* part) {
  switch (ln.block) {
    case 64: apply_soa_bs<DOT, TV, 64>(k, st, m, t, V, beta, alpha, adt, x, w, out, part, ln.xcd); break;
    case 128: apply_soa_bs<DOT, TV, 128>(k, st, m, t, V, beta, alpha, adt, x, w, out, part, ln.xcd); break;
    default: apply_soa_bs<DOT, TV, 256>(k, st, m, t, V, beta, alpha, adt, x, w, out, part, ln.xcd); break;
  }
}
template <typename TV>
static void apply_soa_t(int k, hipStream_t st, Step1Launch ln, int dot, DMesh m, DTab t, const TV* V,
                        const double* beta, double alpha, double adt, const double* x, const double* w, double* out,
                        double* part) {
  if (dot == 0) apply_soa_d<0, TV>(k, st, ln, m, t, V, beta, alpha, adt, x, w, out, part);
  else if (dot == 1) apply_soa_d<1, TV>(k, st, ln, m, t, V, beta, alpha, adt, x, w, out, part);
  else apply_soa_d<2, TV>(k, st, ln, m, t, V, beta, alpha, adt, x, w, out, part);
}
void launch_apply_soa(int k, hipStream_t st, Step1Launch ln, int dot, DMesh m, DTab t, const void* V, bool v32,
                      const double* beta, double alpha, double adt, const double* x, const double* w, double* out,
                      double* part) {
  if (v32) apply_soa_t(k, st, ln, dot, m, t, (const float*)V, beta, alpha, adt, x, w, out, part);
  else apply_soa_t(k, st, ln, dot, m, t, (const double*)V, beta, alpha, adt, x, w, out, part);
}
int apply_soa_blocks(long nc, int block) { return (int)((2L * nc + block - 1) / block); }
void launch_bicg_s(hipStream_t st, long n, int np, const double* part, double* sc, const double* r, const double* v,
                   double* s) {
  k_bicg_s<<<kVecBlocks, kBlock, 0, st>>>(n, np, part, sc, r, v, s);
}
void launch_bicg_xrp(hipStream_t st, long n, int np, const double* part2, double* sc, const double* s,
                     const double* tv, const double* v, double* x, double* r, double* p, double* part) {
  k_bicg_xrp<<<kVecBlocks, kBlock, 0, st>>>(n, np, part2, sc, s, tv, v, x, r, p, part);
}
void launch_bicg_init(hipStream_t st, double* sc) { k_bicg_init<<<1, 64, 0, st>>>(sc); }
void launch_to_soa(int k, hipStream_t st, DMesh m, int inv_det, const double* x, double* y) {
  HDG_DISPATCH(k, (k_to_soa<KK><<<nblocks((long)m.nc * Dims<KK>::NU), kBlock, 0, st>>>(m, inv_det, x, y)));
}
void launch_to_aos(int k, hipStream_t st, DMesh m, const double* x, double* y) {
  HDG_DISPATCH(k, (k_to_aos<KK><<<nblocks((long)m.nc * Dims<KK>::NU), kBlock, 0, st>>>(m, x, y)));
}
}  // namespace hdg
