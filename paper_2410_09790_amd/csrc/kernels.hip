// gfx950 kernels of the HDG-IMEX library.
//
// One thread per cell (or per facet) for the element kernels: every wave
// walks the same reference-table entries at the same time, so table reads are
// uniform (broadcast) and per-cell data are laid out field-major [field][cell]
// so that a wave's loads of one field are contiguous.  Templated on the degree
// k so that every loop over basis functions and quadrature points unrolls.
// All reductions use a fixed grid and a fixed summation order, so results are
// bitwise reproducible run to run.
#include <hip/hip_runtime.h>

#include "device_common.h"
#include "kernels.h"

namespace hdg {

// Facet block size and blocks per row of the trace operator, keyed by tk
// (k on triangles, 10 + k on tetrahedra).
template <int TK>
struct TraceDims {
  static constexpr int NF = TK < 10 ? TK + 1 : (TK - 9) * (TK - 8) / 2;
  static constexpr int SL = TK < 10 ? 5 : 7;
};

#define TRACE_DISPATCH(tk, CALL)     \
  switch (tk) {                      \
    case 1: { constexpr int KK = 1; CALL; } break; \
    case 2: { constexpr int KK = 2; CALL; } break; \
    case 3: { constexpr int KK = 3; CALL; } break; \
    case 4: { constexpr int KK = 4; CALL; } break; \
    case 11: { constexpr int KK = 11; CALL; } break; \
    case 12: { constexpr int KK = 12; CALL; } break; \
    default: break;                  \
  }

#define TET_TRACE_DISPATCH(tk, CALL) \
  switch (tk) {                      \
    case 11: { constexpr int KK = 11; CALL; } break; \
    case 12: { constexpr int KK = 12; CALL; } break; \
    default: break;                  \
  }

static inline int trace_key(int k, const DMesh& m) { return m.dim == 3 ? 10 + k : k; }

// ===================================================================== a1
// Local condensation.  With the orthonormal basis the velocity mass matrix is
// det*I, so the cell problem [[M, -c D^T], [D, T]] reduces to the pressure
// Schur complement P = T + (c/det) D D^T, and the trace operator of the cell
// is S_K = F + (c/det) C C^T - G P^{-1} G^T with G = E + (c/det) C D^T.
// D, C, E, T are linear combinations of reference matrices with geometric
// weights, and so are the products D D^T, C C^T, C D^T.
template <int K>
__global__ void __launch_bounds__(kBlock) k_condense(DMesh m, DTab t, double c, double tau, double* __restrict__ Pinv,
                                                     double* __restrict__ SK) {
  using D = Dims<K>;
  constexpr int NP = D::NP, NF = D::NF, NL = D::NLAM;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const CellGeo g = load_geo(m, e);
  int flip[3];
#pragma unroll
  for (int f = 0; f < 3; ++f) flip[f] = m.cf_flip[f * m.nc + e];
  double Gm[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) Gm[a][b] = g.ij[a][0] * g.ij[b][0] + g.ij[a][1] * g.ij[b][1];
  double L[NP][NP];
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double v = tau * (g.h[0] * t.That[(0 * NP + i) * NP + j] + g.h[1] * t.That[(1 * NP + i) * NP + j] +
                        g.h[2] * t.That[(2 * NP + i) * NP + j]);
      double dd = 0.0;
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) dd += Gm[a][b] * t.KDD[((a * 2 + b) * NP + i) * NP + j];
      L[i][j] = v + c * g.det * dd;
    }
  // Cholesky (lower), in place
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    double d = L[j][j];
#pragma unroll
    for (int q = 0; q < j; ++q) d -= L[j][q] * L[j][q];
    d = sqrt(d);
    L[j][j] = d;
    double inv = 1.0 / d;
#pragma unroll
    for (int i = j + 1; i < NP; ++i) {
      double v = L[i][j];
#pragma unroll
      for (int q = 0; q < j; ++q) v -= L[i][q] * L[j][q];
      L[i][j] = v * inv;
    }
  }
  // Linv (lower) by forward substitution, stored in the upper triangle of a new array
  double Li[NP][NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      if (i < j) { Li[i][j] = 0.0; continue; }
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int q = j; q < i; ++q) v -= L[i][q] * Li[q][j];
      Li[i][j] = v / L[i][i];
    }
  }
  // P^{-1} = Linv^T Linv
#pragma unroll
  for (int i = 0; i < NP; ++i)
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double v = 0.0;
#pragma unroll
      for (int q = (i > j ? i : j); q < NP; ++q) v += Li[q][i] * Li[q][j];
      Pinv[(i * NP + j) * (long)m.nc + e] = v;
    }
  // W = Linv G^T  (NP x NL)
  double W[NP][NL];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    double nu[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) nu[a] = g.n[f][0] * g.ij[a][0] + g.n[f][1] * g.ij[a][1];
#pragma unroll
    for (int mm = 0; mm < NF; ++mm) {
      const double sc = g.h[f] * sgn(flip[f], mm);
      double Grow[NP];
#pragma unroll
      for (int j = 0; j < NP; ++j)
        Grow[j] = sc * (tau * t.Ehat[(f * NF + mm) * NP + j] + c * (nu[0] * t.CD[((f * 2 + 0) * NF + mm) * NP + j] +
                                                                    nu[1] * t.CD[((f * 2 + 1) * NF + mm) * NP + j]));
#pragma unroll
      for (int i = 0; i < NP; ++i) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j <= i; ++j) v += Li[i][j] * Grow[j];
        W[i][f * NF + mm] = v;
      }
    }
  }
  const double cod = c / g.det;
#pragma unroll
  for (int f = 0; f < 3; ++f)
#pragma unroll
    for (int mm = 0; mm < NF; ++mm)
#pragma unroll
      for (int gg = 0; gg < 3; ++gg)
#pragma unroll
        for (int l = 0; l < NF; ++l) {
          const int r = f * NF + mm, s = gg * NF + l;
          double v = (r == s) ? tau * g.h[f] : 0.0;
          const double nn = g.n[f][0] * g.n[gg][0] + g.n[f][1] * g.n[gg][1];
          v += cod * g.h[f] * g.h[gg] * sgn(flip[f], mm) * sgn(flip[gg], l) * nn * t.CC[((f * 3 + gg) * NF + mm) * NF + l];
          double ww = 0.0;
#pragma unroll
          for (int i = 0; i < NP; ++i) ww += W[i][r] * W[i][s];
          SK[(r * NL + s) * (long)m.nc + e] = v - ww;
        }
}

// Facet-block ELL assembly of S = sum_K S_K, one thread per facet (no atomics).
// Slot 0: the facet itself; slots 1-2: the other facets of K+; slots 3-4: of K-.
template <int K>
__global__ void __launch_bounds__(kBlock) k_assemble(DMesh m, const double* __restrict__ SK, double* __restrict__ vals,
                                                     int* __restrict__ cols, double* __restrict__ Dinv) {
  using D = Dims<K>;
  constexpr int NF = D::NF, NL = D::NLAM;
  const int F = blockIdx.x * blockDim.x + threadIdx.x;
  const int nF = m.nF;
  if (F >= nF) return;
  const long nc = m.nc;
  const int Kp = m.fc_cell[F], fp = m.fc_f[F], Km = m.fc_cell[nF + F], fm = m.fc_f[nF + F];
  auto put = [&](int slot, int col, int cell, int fr, int fcol, bool add) {
    if (!add) cols[slot * nF + F] = col;
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        double v = cell >= 0 ? SK[((fr * NF + i) * NL + fcol * NF + j) * nc + cell] : 0.0;
        long idx = ((long)(slot * NF + i) * NF + j) * nF + F;
        vals[idx] = add ? vals[idx] + v : v;
      }
  };
  put(0, F, Kp, fp, fp, false);
  if (Km >= 0) put(0, F, Km, fm, fm, true);
#pragma unroll
  for (int o = 1; o <= 2; ++o) {
    const int gq = (fp + o) % 3;
    put(o, m.cf_facet[gq * nc + Kp], Kp, fp, gq, false);
  }
#pragma unroll
  for (int o = 1; o <= 2; ++o) {
    if (Km >= 0) {
      const int gq = (fm + o) % 3;
      put(2 + o, m.cf_facet[gq * nc + Km], Km, fm, gq, false);
    } else {
      put(2 + o, F, -1, 0, 0, false);
    }
  }
  // inverse of the diagonal block (SPD), Gauss-Jordan without pivoting
  double A[NF][NF], B[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      A[i][j] = vals[((long)(0 * NF + i) * NF + j) * nF + F];
      B[i][j] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int cidx = 0; cidx < NF; ++cidx) {
    double d = 1.0 / A[cidx][cidx];
#pragma unroll
    for (int j = 0; j < NF; ++j) { A[cidx][j] *= d; B[cidx][j] *= d; }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      if (r == cidx) continue;
      double f = A[r][cidx];
#pragma unroll
      for (int j = 0; j < NF; ++j) { A[r][j] -= f * A[cidx][j]; B[r][j] -= f * B[cidx][j]; }
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) Dinv[(long)(i * NF + j) * nF + F] = B[i][j];
}

// ===================================================================== a8
// Trace SpMV, one thread per facet and all NF rows of its block row: the five
// blocks of a facet row are stored slot-major, then row, then column, with
// the facet index fastest, so every value load is coalesced across the
// wavefront, and each thread writes its NF results as one contiguous run.
template <int K>
__global__ void __launch_bounds__(kBlock) k_spmv(int nF, const double* __restrict__ vals, const int* __restrict__ cols,
                                                 const double* __restrict__ x, const double* __restrict__ b,
                                                 double* __restrict__ y) {
  constexpr int NF = K + 1;
  const int F = blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= nF) return;
  double acc[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) acc[i] = 0.0;
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    const int col = cols[s * nF + F];
    double xc[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) xc[j] = x[(long)col * NF + j];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) acc[i] += vals[((long)(s * NF + i) * NF + j) * nF + F] * xc[j];
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) y[(long)F * NF + i] = b ? b[(long)F * NF + i] - acc[i] : acc[i];
}

// The same product on tetrahedra (tk = 10 + k: (k+1)(k+2)/2 unknowns per
// facet, 7 blocks per row).  A facet row holds 7 x 36 values at k = 2, too
// many for one thread's registers, so a workgroup takes 64 facets and each
// of its NF waves one row of their blocks: every value load is coalesced
// across the wave (facet index fastest).  The column ids and the x entries
// the 64 rows touch are gathered once per workgroup into LDS (the NF waves
// would otherwise each gather them again), and the NF results of a facet are
// staged in LDS so that y is written in contiguous runs.
template <int TK>
struct TetRowsShape {
  static constexpr int NF = TraceDims<TK>::NF, SL = TraceDims<TK>::SL, NT = 64 * NF;
};
// gathers cols and x of facets F0 .. F0 + 63 into sc[s][f], sx[s][j][f]
template <int TK>
__device__ __forceinline__ void tet_gather(int nF, long F0, const int* __restrict__ cols,
                                           const double* __restrict__ x, int (&sc)[TraceDims<TK>::SL][64],
                                           double (&sx)[TraceDims<TK>::SL][TraceDims<TK>::NF][64]) {
  constexpr int NF = TraceDims<TK>::NF, SL = TraceDims<TK>::SL, NT = TetRowsShape<TK>::NT;
  for (int idx = threadIdx.x; idx < SL * 64; idx += NT) {
    const int sl = idx / 64, fl = idx % 64;
    sc[sl][fl] = F0 + fl < nF ? cols[sl * (long)nF + F0 + fl] : 0;
  }
  __syncthreads();
  for (int idx = threadIdx.x; idx < SL * 64 * NF; idx += NT) {
    const int sl = idx / (64 * NF), rem = idx % (64 * NF), fl = rem / NF, jj = rem % NF;
    sx[sl][jj][fl] = x[(long)sc[sl][fl] * NF + jj];  // consecutive threads: one facet's entries
  }
  __syncthreads();
}
template <int TK>
__global__ void __launch_bounds__(TetRowsShape<TK>::NT) k_spmv_tet(int nF, const double* __restrict__ vals,
                                                                 const int* __restrict__ cols,
                                                                 const double* __restrict__ x,
                                                                 const double* __restrict__ b,
                                                                 double* __restrict__ y) {
  constexpr int NF = TraceDims<TK>::NF, SL = TraceDims<TK>::SL;
  __shared__ int sc[SL][64];
  __shared__ double sx[SL][NF][64];
  __shared__ double sy[NF][64];
  const int lane = threadIdx.x & 63, i = threadIdx.x >> 6;
  const long F0 = (long)blockIdx.x * 64;
  const long F = F0 + lane;
  tet_gather<TK>(nF, F0, cols, x, sc, sx);
  if (F < nF) {
    double acc = 0.0;
#pragma unroll
    for (int sl = 0; sl < SL; ++sl) {
      const double* v = vals + ((long)(sl * NF + i) * NF) * nF + F;
#pragma unroll
      for (int jj = 0; jj < NF; ++jj) acc += v[(long)jj * nF] * sx[sl][jj][lane];
    }
    sy[i][lane] = b ? b[F * NF + i] - acc : acc;
  }
  __syncthreads();
  const long idx = F0 * NF + threadIdx.x;  // contiguous run of this block's outputs
  if (idx < (long)nF * NF) y[idx] = sy[threadIdx.x % NF][threadIdx.x / NF];
}

// damped block-Jacobi sweep on tetrahedra, the same arrangement:
// xout = xin + omega Dinv (b - S xin) (xin == nullptr: xin = 0)
template <int TK>
__global__ void __launch_bounds__(TetRowsShape<TK>::NT) k_jacobi_tet(int nF, const double* __restrict__ vals,
                                                                   const int* __restrict__ cols,
                                                                   const double* __restrict__ Dinv, double omega,
                                                                   const double* __restrict__ b,
                                                                   const double* __restrict__ xin,
                                                                   double* __restrict__ xout) {
  constexpr int NF = TraceDims<TK>::NF, SL = TraceDims<TK>::SL;
  __shared__ int sc[SL][64];
  __shared__ double sx[SL][NF][64];
  __shared__ double sr[NF][64], sz[NF][64];
  const int lane = threadIdx.x & 63, i = threadIdx.x >> 6;
  const long F0 = (long)blockIdx.x * 64;
  const long F = F0 + lane;
  if (xin) tet_gather<TK>(nF, F0, cols, xin, sc, sx);  // xin is uniform: every thread takes the same branch
  if (F < nF) {
    double acc = 0.0;
    if (xin) {
#pragma unroll
      for (int sl = 0; sl < SL; ++sl) {
        const double* v = vals + ((long)(sl * NF + i) * NF) * nF + F;
#pragma unroll
        for (int jj = 0; jj < NF; ++jj) acc += v[(long)jj * nF] * sx[sl][jj][lane];
      }
    }
    sr[i][lane] = b[F * NF + i] - acc;
  }
  __syncthreads();
  if (F < nF) {
    double z = 0.0;
#pragma unroll
    for (int jj = 0; jj < NF; ++jj) z += Dinv[(long)(i * NF + jj) * nF + F] * sr[jj][lane];
    sz[i][lane] = z;
  }
  __syncthreads();
  const long idx = F0 * NF + threadIdx.x;
  if (idx < (long)nF * NF) {
    const int fl = threadIdx.x / NF, ii = threadIdx.x % NF;
    xout[idx] = (xin ? xin[idx] : 0.0) + omega * sz[ii][fl];
  }
}

// damped block-Jacobi sweep: xout = xin + omega Dinv (b - S xin); xin == nullptr means xin = 0
template <int K>
__global__ void __launch_bounds__(kBlock) k_jacobi(int nF, const double* __restrict__ vals, const int* __restrict__ cols,
                                                   const double* __restrict__ Dinv, double omega,
                                                   const double* __restrict__ b, const double* __restrict__ xin,
                                                   double* __restrict__ xout) {
  constexpr int NF = TraceDims<K>::NF, SL = TraceDims<K>::SL;
  (void)SL;
  const int F = blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= nF) return;
  double r[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) r[i] = b[(long)F * NF + i];
  if (xin) {
#pragma unroll
    for (int s = 0; s < SL; ++s) {
      const int col = cols[s * nF + F];
      double xc[NF];
#pragma unroll
      for (int j = 0; j < NF; ++j) xc[j] = xin[(long)col * NF + j];
#pragma unroll
      for (int i = 0; i < NF; ++i)
#pragma unroll
        for (int j = 0; j < NF; ++j) r[i] -= vals[((long)(s * NF + i) * NF + j) * nF + F] * xc[j];
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j) v += Dinv[(long)(i * NF + j) * nF + F] * r[j];
    xout[(long)F * NF + i] = (xin ? xin[(long)F * NF + i] : 0.0) + omega * v;
  }
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_blockdiag(int nF, const double* __restrict__ Dinv,
                                                      const double* __restrict__ x, double* __restrict__ y) {
  constexpr int NF = TraceDims<K>::NF, SL = TraceDims<K>::SL;
  (void)SL;
  const int F = blockIdx.x * blockDim.x + threadIdx.x;
  if (F >= nF) return;
  double xv[NF];
#pragma unroll
  for (int j = 0; j < NF; ++j) xv[j] = x[(long)F * NF + j];
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NF; ++j) v += Dinv[(long)(i * NF + j) * nF + F] * xv[j];
    y[(long)F * NF + i] = v;
  }
}

// ================================================================ a7, a9
// helpers shared by the condensation right-hand side and back-substitution:
// u_a[s] = sum_c iJ[a][c] F[c][s];  (D F)_i = det sum_a sum_s Dhat_a[i][s] u_a[s]
template <int K>
__device__ __forceinline__ void pressure_solve(const DTab& t, const CellGeo& g, double c, const double* Pinv, long nc,
                                               int e, const double (&fw)[Dims<K>::NU], const double (&fpsi)[Dims<K>::NP],
                                               double (&p)[Dims<K>::NP]) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NP = D::NP;
  double b[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double u0 = g.ij[0][0] * fw[s] + g.ij[0][1] * fw[NS + s];
      const double u1 = g.ij[1][0] * fw[s] + g.ij[1][1] * fw[NS + s];
      v += t.Dx[i * NS + s] * u0 + t.Dy[i * NS + s] * u1;
    }
    b[i] = fpsi[i] - v;  // f_psi - D f_w / det
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) v += Pinv[(i * NP + j) * nc + e] * b[j];
    p[i] = v;
  }
  (void)c;
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_rhs_condense(DMesh m, DTab t, double c, double tau,
                                                         const double* __restrict__ Pinv, const double* __restrict__ Fw,
                                                         const double* __restrict__ Fpsi, double* __restrict__ ycell) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double fw[NU], fpsi[NP], p[NP];
#pragma unroll
  for (int i = 0; i < NU; ++i) fw[i] = Fw ? Fw[(long)e * NU + i] : 0.0;
#pragma unroll
  for (int i = 0; i < NP; ++i) fpsi[i] = Fpsi ? Fpsi[(long)e * NP + i] : 0.0;
  pressure_solve<K>(t, g, c, Pinv, nc, e, fw, fpsi, p);
  const double idet = 1.0 / g.det;
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int flip = m.cf_flip[f * nc + e];
    double nu[2];
#pragma unroll
    for (int a = 0; a < 2; ++a) nu[a] = g.n[f][0] * g.ij[a][0] + g.n[f][1] * g.ij[a][1];
#pragma unroll
    for (int mm = 0; mm < NF; ++mm) {
      double cf = 0.0;  // (C f_w) / (h sigma)
#pragma unroll
      for (int s = 0; s < NS; ++s) cf += t.Chat[(f * NF + mm) * NS + s] * (g.n[f][0] * fw[s] + g.n[f][1] * fw[NS + s]);
      double gp = 0.0;  // (G p) / (h sigma)
#pragma unroll
      for (int j = 0; j < NP; ++j)
        gp += (tau * t.Ehat[(f * NF + mm) * NP + j] +
               c * (nu[0] * t.CD[((f * 2 + 0) * NF + mm) * NP + j] + nu[1] * t.CD[((f * 2 + 1) * NF + mm) * NP + j])) *
              p[j];
      ycell[(long)(f * NF + mm) * nc + e] = g.h[f] * sgn(flip, mm) * (cf * idet + gp);
    }
  }
}

// g_F = sum over the cells of F of their condensed contributions - F_mu
template <int K>
__global__ void __launch_bounds__(kBlock) k_gather_rhs(DMesh m, const double* __restrict__ ycell,
                                                       const double* __restrict__ Fmu, double* __restrict__ gout) {
  constexpr int NF = TraceDims<K>::NF, SL = TraceDims<K>::SL;
  (void)SL;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int nF = m.nF;
  if (tid >= (long)nF * NF) return;
  const int F = (int)(tid / NF), mm = (int)(tid % NF);
  const long nc = m.nc;
  const int Kp = m.fc_cell[F], fp = m.fc_f[F], Km = m.fc_cell[nF + F], fm = m.fc_f[nF + F];
  double v = ycell[(long)(fp * NF + mm) * nc + Kp];
  if (Km >= 0) v += ycell[(long)(fm * NF + mm) * nc + Km];
  if (Fmu) v -= Fmu[tid];
  gout[tid] = v;
}

template <int K>
__global__ void __launch_bounds__(kBlock) k_backsub(DMesh m, DTab t, double c, double tau,
                                                    const double* __restrict__ Pinv, const double* __restrict__ Fw,
                                                    const double* __restrict__ Fpsi, const double* __restrict__ lam,
                                                    double* __restrict__ U, double* __restrict__ P,
                                                    double* __restrict__ part) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double pint = 0.0;
  if (e < m.nc) {
    const long nc = m.nc;
    const CellGeo g = load_geo(m, e);
    double fw[NU], fpsi[NP], p[NP];
#pragma unroll
    for (int i = 0; i < NU; ++i) fw[i] = Fw ? Fw[(long)e * NU + i] : 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) fpsi[i] = Fpsi ? Fpsi[(long)e * NP + i] : 0.0;
    // f_w -= c C^T lam;  f_psi += E^T lam
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const int F = m.cf_facet[f * nc + e];
      const int flip = m.cf_flip[f * nc + e];
      double l[NF];
#pragma unroll
      for (int mm = 0; mm < NF; ++mm) l[mm] = sgn(flip, mm) * lam[(long)F * NF + mm] * g.h[f];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        double v = 0.0;
#pragma unroll
        for (int mm = 0; mm < NF; ++mm) v += t.Chat[(f * NF + mm) * NS + s] * l[mm];
        fw[s] -= c * g.n[f][0] * v;
        fw[NS + s] -= c * g.n[f][1] * v;
      }
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        double v = 0.0;
#pragma unroll
        for (int mm = 0; mm < NF; ++mm) v += t.Ehat[(f * NF + mm) * NP + j] * l[mm];
        fpsi[j] += tau * v;
      }
    }
    pressure_solve<K>(t, g, c, Pinv, nc, e, fw, fpsi, p);
    const double idet = 1.0 / g.det;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double d0 = 0.0, d1 = 0.0;  // sum_i Dhat_a[i][s] p_i
#pragma unroll
      for (int i = 0; i < NP; ++i) { d0 += t.Dx[i * NS + s] * p[i]; d1 += t.Dy[i * NS + s] * p[i]; }
#pragma unroll
      for (int cc = 0; cc < 2; ++cc)
        U[(long)e * NU + cc * NS + s] = fw[cc * NS + s] * idet + c * (g.ij[0][cc] * d0 + g.ij[1][cc] * d1);
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) P[(long)e * NP + i] = p[i];
    pint = g.det * p[0] * 0.70710678118654752440;  // int_K p = det p_0 int phi_0, int phi_0 = 1/sqrt(2)
  }
  if (part) {
    double s = block_sum(pint);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
  }
}

// shift (p, lam) by -mean: p_0 -= mean/sqrt(2) (phi_0 = sqrt 2), lam_0 -= mean (mu_0 = 1)
template <int K>
__global__ void k_shift_mean(DMesh m, const double* __restrict__ mean, double* __restrict__ p, double* __restrict__ lam) {
  constexpr int NP = Dims<K>::NP, NF = K + 1;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double mv = mean[0];
  if (tid < m.nc) p[tid * NP] -= mv * 0.70710678118654752440;
  if (tid < m.nF && lam) lam[tid * NF] -= mv;
}

// Constraint residual Gamma(psi, mu, Q, p, lam) of Section "Hybridisation"
// (the second line of the hybridised system) as dual vectors, times scale:
//   psi part, per cell:  (psi, div Q)_K + <tau (p - lam), psi>_dK
//   mu part, per (cell, local facet): <Q.n_K + tau (p - lam), mu>_F from
//   this cell's side, written to ycell in the layout k_gather_rhs sums over
//   the facet's cells.
// With the reference blocks: D Q + T p - E^T lam and C Q + E p - F lam.
// P or lam may be null (zero).
template <int K>
__global__ void __launch_bounds__(kBlock) k_gamma(DMesh m, DTab t, double tau, double scale,
                                                  const double* __restrict__ Q, const double* __restrict__ P,
                                                  const double* __restrict__ lam, double* __restrict__ gpsi,
                                                  double* __restrict__ ycell) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double q[NU], p[NP], ps[NP];
#pragma unroll
  for (int i = 0; i < NU; ++i) q[i] = Q[(long)e * NU + i];
#pragma unroll
  for (int i = 0; i < NP; ++i) p[i] = P ? P[(long)e * NP + i] : 0.0;
  // (psi_i, div Q)_K = det sum_s (Dhat_x[i][s] u0_s + Dhat_y[i][s] u1_s), u_a = sum_c iJ[a][c] Q_c
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double u0 = g.ij[0][0] * q[s] + g.ij[0][1] * q[NS + s];
      const double u1 = g.ij[1][0] * q[s] + g.ij[1][1] * q[NS + s];
      v += t.Dx[i * NS + s] * u0 + t.Dy[i * NS + s] * u1;
    }
    ps[i] = g.det * v;
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int F = m.cf_facet[f * nc + e];
    const int flip = m.cf_flip[f * nc + e];
    const double h = g.h[f];
    double l[NF];
#pragma unroll
    for (int mm = 0; mm < NF; ++mm) l[mm] = lam ? lam[(long)F * NF + mm] : 0.0;
    // psi part: tau h (That p - Ehat^T sgn lam)
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) v += t.That[(f * NP + i) * NP + j] * p[j];
#pragma unroll
      for (int mm = 0; mm < NF; ++mm) v -= t.Ehat[(f * NF + mm) * NP + i] * sgn(flip, mm) * l[mm];
      ps[i] += tau * h * v;
    }
    // mu part from this side: h sgn (Chat (Q.n) + tau Ehat p) - tau h lam
#pragma unroll
    for (int mm = 0; mm < NF; ++mm) {
      double cq = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) cq += t.Chat[(f * NF + mm) * NS + s] * (g.n[f][0] * q[s] + g.n[f][1] * q[NS + s]);
      double ep = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) ep += t.Ehat[(f * NF + mm) * NP + j] * p[j];
      ycell[(long)(f * NF + mm) * nc + e] = scale * (h * sgn(flip, mm) * (cq + tau * ep) - tau * h * l[mm]);
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) gpsi[(long)e * NP + i] = scale * ps[i];
}

// ================================================================ a4, a5
// Per-stage advection data from Q*: weighted reference-direction velocities
// at the cell points and the facet weights (1/2 qn - delta |qn|) w h at the
// facet points (own side; qn = Q*.n is single-valued for the BDM field).
template <int K>
__global__ void __launch_bounds__(kBlock) k_prep_adv(DMesh m, DTab t, const double* __restrict__ Qs, double delta_up,
                                                     double* __restrict__ adv) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC, NQF = D::NQF;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double q[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) q[i] = Qs[(long)e * NU + i];
  for (int qq = 0; qq < NQC; ++qq) {
    double vx = 0.0, vy = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) { const double b = t.Bu[qq * NS + s]; vx += b * q[s]; vy += b * q[NS + s]; }
    const double w = t.cw[qq] * g.det;
    adv[(long)(0 * NQC + qq) * nc + e] = w * (g.ij[0][0] * vx + g.ij[0][1] * vy);
    adv[(long)(1 * NQC + qq) * nc + e] = w * (g.ij[1][0] * vx + g.ij[1][1] * vy);
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const bool inner = m.cf_nb[f * nc + e] >= 0;
    for (int qq = 0; qq < NQF; ++qq) {
      double vx = 0.0, vy = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) { const double b = t.FBu[(f * NQF + qq) * NS + s]; vx += b * q[s]; vy += b * q[NS + s]; }
      const double qn = vx * g.n[f][0] + vy * g.n[f][1];
      adv[(long)(2 * NQC + f * NQF + qq) * nc + e] = inner ? t.fw[qq] * g.h[f] * (0.5 * qn - delta_up * fabs(qn)) : 0.0;
    }
  }
}

// f_im applied matrix-free (eq. f_impl), cell by cell; each interior facet
// term is evaluated from both of its cells, so no scatter is needed.
template <int K, int MODE>
__global__ void __launch_bounds__(kBlock) k_apply(DMesh m, DTab t, const double* __restrict__ adv, double alpha,
                                                  double adt, const double* __restrict__ x, const double* __restrict__ r,
                                                  const double* __restrict__ pp, const double* __restrict__ lam,
                                                  double* __restrict__ out) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC, NQF = D::NQF, NP = D::NP, NF = D::NF;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double xv[NU], y[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) { xv[i] = x[(long)e * NU + i]; y[i] = 0.0; }
  // volume: -(w . (Q* . grad) x)
  for (int qq = 0; qq < NQC; ++qq) {
    const double a0 = adv[(long)(0 * NQC + qq) * nc + e], a1 = adv[(long)(1 * NQC + qq) * nc + e];
    double v[2];
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) {
      double dx = 0.0, dy = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) { dx += t.Gux[qq * NS + s] * xv[cc * NS + s]; dy += t.Guy[qq * NS + s] * xv[cc * NS + s]; }
      v[cc] = a0 * dx + a1 * dy;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double b = t.Bu[qq * NS + s];
      y[s] -= b * v[0];
      y[NS + s] -= b * v[1];
    }
  }
  // facets: central + upwind (weight beta) and interior penalty
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int nb = m.cf_nb[f * nc + e];
    double xn[NU];
    int fn = 0, rev = 0;
    if (nb >= 0) {
      fn = m.cf_nbf[f * nc + e];
      rev = m.cf_flip[f * nc + e] != m.cf_flip[fn * nc + nb];
#pragma unroll
      for (int i = 0; i < NU; ++i) xn[i] = x[(long)nb * NU + i];
    } else {
#pragma unroll
      for (int i = 0; i < NU; ++i) xn[i] = 0.0;
    }
    for (int qq = 0; qq < NQF; ++qq) {
      const int qn = rev ? NQF - 1 - qq : qq;
      double jx = 0.0, jy = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double b = t.FBu[(f * NQF + qq) * NS + s];
        jx += b * xv[s];
        jy += b * xv[NS + s];
      }
      if (nb >= 0) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
          const double b = t.FBu[(fn * NQF + qn) * NS + s];
          jx -= b * xn[s];
          jy -= b * xn[NS + s];
        }
      }
      const double beta = adv[(long)(2 * NQC + f * NQF + qq) * nc + e];
      const double pen = alpha * t.fw[qq] * (jx * g.n[f][0] + jy * g.n[f][1]);
      const double cx = beta * jx - pen * g.n[f][0];
      const double cy = beta * jy - pen * g.n[f][1];
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double b = t.FBu[(f * NQF + qq) * NS + s];
        y[s] += b * cx;
        y[NS + s] += b * cy;
      }
    }
  }
  if (MODE == 0) {
    const double sc = adt / g.det;
#pragma unroll
    for (int i = 0; i < NU; ++i) out[(long)e * NU + i] = xv[i] - sc * y[i];
    return;
  }
  // g(w, p, lam) = (p, div w) - <lam, w.n>
  double pv[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) pv[i] = pp[(long)e * NP + i];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double d0 = 0.0, d1 = 0.0;
#pragma unroll
    for (int i = 0; i < NP; ++i) { d0 += t.Dx[i * NS + s] * pv[i]; d1 += t.Dy[i * NS + s] * pv[i]; }
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) y[cc * NS + s] += g.det * (g.ij[0][cc] * d0 + g.ij[1][cc] * d1);
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int F = m.cf_facet[f * nc + e];
    const int flip = m.cf_flip[f * nc + e];
    double l[NF];
#pragma unroll
    for (int mm = 0; mm < NF; ++mm) l[mm] = sgn(flip, mm) * lam[(long)F * NF + mm] * g.h[f];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double v = 0.0;
#pragma unroll
      for (int mm = 0; mm < NF; ++mm) v += t.Chat[(f * NF + mm) * NS + s] * l[mm];
      y[s] -= g.n[f][0] * v;
      y[NS + s] -= g.n[f][1] * v;
    }
  }
  const double sc = (MODE == 1) ? 1.0 / g.det : 1.0;
#pragma unroll
  for (int i = 0; i < NU; ++i) out[(long)e * NU + i] = sc * (r[(long)e * NU + i] - g.det * xv[i] + adt * y[i]);
}

// ===================================================================== a6
// Div(psi, F) = sum_K [ -(grad psi, F)_K + <psi {F}.n_K>_dK ], {F}.n = 0 on walls
template <int K>
__global__ void __launch_bounds__(kBlock) k_div(DMesh m, DTab t, const double* __restrict__ F, double scale,
                                                double* __restrict__ out) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NP = D::NP, NQF = D::NQF;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double fv[NU], o[NP];
#pragma unroll
  for (int i = 0; i < NU; ++i) fv[i] = F[(long)e * NU + i];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    double v = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double u0 = g.ij[0][0] * fv[s] + g.ij[0][1] * fv[NS + s];
      const double u1 = g.ij[1][0] * fv[s] + g.ij[1][1] * fv[NS + s];
      v += t.Rx[i * NS + s] * u0 + t.Ry[i * NS + s] * u1;
    }
    o[i] = -g.det * v;
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int nb = m.cf_nb[f * nc + e];
    if (nb < 0) continue;
    const int fn = m.cf_nbf[f * nc + e];
    const int rev = m.cf_flip[f * nc + e] != m.cf_flip[fn * nc + nb];
    double xn[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) xn[i] = F[(long)nb * NU + i];
    for (int qq = 0; qq < NQF; ++qq) {
      const int qn = rev ? NQF - 1 - qq : qq;
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double b = t.FBu[(f * NQF + qq) * NS + s], bn = t.FBu[(fn * NQF + qn) * NS + s];
        ax += b * fv[s] + bn * xn[s];
        ay += b * fv[NS + s] + bn * xn[NS + s];
      }
      const double flux = 0.5 * t.fw[qq] * g.h[f] * (ax * g.n[f][0] + ay * g.n[f][1]);
#pragma unroll
      for (int i = 0; i < NP; ++i) o[i] += t.FBp[(f * NQF + qq) * NP + i] * flux;
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) out[(long)e * NP + i] = scale * o[i];
}

// ===================================================================== a3
// BDM interpolant through the reference element: the physical moments equal
// the reference moments of the contravariant Piola pull-back, so
// Qhat* = R^{-1} m and Q* = J Qhat* / det.
template <int K>
__global__ void __launch_bounds__(kBlock) k_bdm(DMesh m, DTab t, const double* __restrict__ Q, double* __restrict__ Qs) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC, NQF = D::NQF, NNED = D::NNED, NM = D::NM;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double qv[NU], mom[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) { qv[i] = Q[(long)e * NU + i]; mom[i] = 0.0; }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int nb = m.cf_nb[f * nc + e];
    if (nb < 0) continue;  // wall: zero normal moments
    const int fn = m.cf_nbf[f * nc + e];
    const int rev = m.cf_flip[f * nc + e] != m.cf_flip[fn * nc + nb];
    double xn[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) xn[i] = Q[(long)nb * NU + i];
    for (int qq = 0; qq < NQF; ++qq) {
      const int qn = rev ? NQF - 1 - qq : qq;
      double ax = 0.0, ay = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double b = t.FBu[(f * NQF + qq) * NS + s], bn = t.FBu[(fn * NQF + qn) * NS + s];
        ax += b * qv[s] + bn * xn[s];
        ay += b * qv[NS + s] + bn * xn[NS + s];
      }
      const double flux = 0.5 * t.fw[qq] * g.h[f] * (ax * g.n[f][0] + ay * g.n[f][1]);
#pragma unroll
      for (int j = 0; j < NM; ++j) mom[f * NM + j] += t.NUB[qq * NM + j] * flux;
    }
  }
  for (int qq = 0; qq < NQC; ++qq) {
    double vx = 0.0, vy = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) { const double b = t.Bu[qq * NS + s]; vx += b * qv[s]; vy += b * qv[NS + s]; }
    // reference components of the covariant pull-back: (J^{-T} vhat) . Q = vhat . (J^{-1} Q)
    const double w = t.cw[qq] * g.det;
    const double r0 = w * (g.ij[0][0] * vx + g.ij[0][1] * vy);
    const double r1 = w * (g.ij[1][0] * vx + g.ij[1][1] * vy);
#pragma unroll
    for (int l = 0; l < NNED; ++l) mom[3 * NM + l] += t.NED[(qq * NNED + l) * 2 + 0] * r0 + t.NED[(qq * NNED + l) * 2 + 1] * r1;
  }
  double qh[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NU; ++j) v += t.BDMinv[i * NU + j] * mom[j];
    qh[i] = v;
  }
  const double idet = 1.0 / g.det;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    Qs[(long)e * NU + s] = idet * (g.J[0][0] * qh[s] + g.J[0][1] * qh[NS + s]);
    Qs[(long)e * NU + NS + s] = idet * (g.J[1][0] * qh[s] + g.J[1][1] * qh[NS + s]);
  }
}

// ==================================================================== a12
// psi-data of the pressure reconstruction: Div(psi, f_p), f_p = (Q.grad_h)Q
template <int K>
__global__ void __launch_bounds__(kBlock) k_recon_rhs(DMesh m, DTab t, const double* __restrict__ Q,
                                                      const double* __restrict__ fcell,
                                                      const double* __restrict__ ffac, double fsc,
                                                      double* __restrict__ out) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NP = D::NP, NQC = D::NQC, NQF = D::NQF;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double qv[NU], o[NP];
#pragma unroll
  for (int i = 0; i < NU; ++i) qv[i] = Q[(long)e * NU + i];
#pragma unroll
  for (int i = 0; i < NP; ++i) o[i] = 0.0;
  auto conv = [&](cdptr B, cdptr Gx, cdptr Gy, const double* qc, const double (&ij)[2][2],
                  double& fx, double& fy) {
    double vx = 0.0, vy = 0.0, d[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      vx += B[s] * qc[s]; vy += B[s] * qc[NS + s];
      d[0][0] += Gx[s] * qc[s]; d[0][1] += Gy[s] * qc[s];
      d[1][0] += Gx[s] * qc[NS + s]; d[1][1] += Gy[s] * qc[NS + s];
    }
    // physical derivative d_dd Q_c = sum_a iJ[a][dd] dref_a Q_c
    const double gxx = ij[0][0] * d[0][0] + ij[1][0] * d[0][1], gxy = ij[0][1] * d[0][0] + ij[1][1] * d[0][1];
    const double gyx = ij[0][0] * d[1][0] + ij[1][0] * d[1][1], gyy = ij[0][1] * d[1][0] + ij[1][1] * d[1][1];
    fx = vx * gxx + vy * gxy;
    fy = vx * gyx + vy * gyy;
  };
  for (int qq = 0; qq < NQC; ++qq) {
    double fx, fy;
    conv(t.Bu + qq * NS, t.Gux + qq * NS, t.Guy + qq * NS, qv, g.ij, fx, fy);
    if (fcell) {  // f_p = (Q.grad)Q - f
      fx -= fsc * fcell[((long)e * NQC + qq) * 2];
      fy -= fsc * fcell[((long)e * NQC + qq) * 2 + 1];
    }
    const double w = t.cw[qq] * g.det;
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const double gx = g.ij[0][0] * t.Gpx[qq * NP + i] + g.ij[1][0] * t.Gpy[qq * NP + i];
      const double gy = g.ij[0][1] * t.Gpx[qq * NP + i] + g.ij[1][1] * t.Gpy[qq * NP + i];
      o[i] -= w * (gx * fx + gy * fy);
    }
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int nb = m.cf_nb[f * nc + e];
    if (nb < 0) continue;
    const int fn = m.cf_nbf[f * nc + e];
    const int rev = m.cf_flip[f * nc + e] != m.cf_flip[fn * nc + nb];
    double xn[NU];
#pragma unroll
    for (int i = 0; i < NU; ++i) xn[i] = Q[(long)nb * NU + i];
    double ijn[2][2];
    ijn[0][0] = m.geo[D_IJ00 * nc + nb]; ijn[0][1] = m.geo[D_IJ01 * nc + nb];
    ijn[1][0] = m.geo[D_IJ10 * nc + nb]; ijn[1][1] = m.geo[D_IJ11 * nc + nb];
    for (int qq = 0; qq < NQF; ++qq) {
      const int qn = rev ? NQF - 1 - qq : qq;
      double fx, fy, gx, gy;
      conv(t.FBu + (f * NQF + qq) * NS, t.FGux + (f * NQF + qq) * NS, t.FGuy + (f * NQF + qq) * NS, qv, g.ij, fx, fy);
      conv(t.FBu + (fn * NQF + qn) * NS, t.FGux + (fn * NQF + qn) * NS, t.FGuy + (fn * NQF + qn) * NS, xn, ijn, gx, gy);
      if (ffac) {  // f is continuous: the same point value on both sides
        const long fi = (((long)e * 3 + f) * NQF + qq) * 2;
        fx -= fsc * ffac[fi]; gx -= fsc * ffac[fi];
        fy -= fsc * ffac[fi + 1]; gy -= fsc * ffac[fi + 1];
      }
      const double flux = 0.5 * t.fw[qq] * g.h[f] * ((fx + gx) * g.n[f][0] + (fy + gy) * g.n[f][1]);
#pragma unroll
      for (int i = 0; i < NP; ++i) o[i] += t.FBp[(f * NQF + qq) * NP + i] * flux;
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) out[(long)e * NP + i] = o[i];
}

// L2 projection of point values [cell][q][2] (orthonormal basis: M = det I)
template <int K>
__global__ void __launch_bounds__(kBlock) k_project(DMesh m, DTab t, const double* __restrict__ vals,
                                                    double* __restrict__ Q) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  double o[NU];
#pragma unroll
  for (int i = 0; i < NU; ++i) o[i] = 0.0;
  for (int qq = 0; qq < NQC; ++qq) {
    const double vx = vals[((long)e * NQC + qq) * 2], vy = vals[((long)e * NQC + qq) * 2 + 1];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double b = t.cw[qq] * t.Bu[qq * NS + s];
      o[s] += b * vx;
      o[NS + s] += b * vy;
    }
  }
#pragma unroll
  for (int i = 0; i < NU; ++i) Q[(long)e * NU + i] = o[i];
}

template <int K>
__global__ void k_mass(DMesh m, double s, const double* __restrict__ x, double* __restrict__ y) {
  constexpr int NU = Dims<K>::NU;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long)m.nc * NU) return;
  const int e = (int)(tid / NU);
  y[tid] = s * m.geo[D_DET * (long)m.nc + e] * x[tid];
}

// ====================================================== forcing (eq. f_expl)
// Dual vector (f, w) of a field given at the cell quadrature points
// (vals[(e*NQC + q)*2 + c]), AoS [cell][c*NS + s].
template <int K>
__global__ void k_point_dual(DMesh m, DTab t, const double* __restrict__ vals, double* __restrict__ out) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long)m.nc * NU) return;
  const long e = tid / NU;
  const int i = (int)(tid % NU), c = i / NS, s = i % NS;
  double acc = 0.0;
  for (int q = 0; q < NQC; ++q) acc += t.cw[q] * t.Bu[q * NS + s] * vals[(e * NQC + q) * 2 + c];
  out[tid] = m.geo[D_DET * (long)m.nc + e] * acc;
}

// Wall data of the pressure reconstruction for a field f given at the facet
// points (vals[((e*3 + f)*NQF + q)*2 + c], the cell's local parametrisation):
// out(mu) = -<mu, n.f> on wall facets, 0 on interior facets.  One thread per
// (cell, local facet).
template <int K>
__global__ void k_wall_flux(DMesh m, DTab t, const double* __restrict__ vals, double* __restrict__ out) {
  using D = Dims<K>;
  constexpr int NF = D::NF, NQF = D::NQF;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nc = m.nc;
  if (tid >= 3 * nc) return;
  const long e = tid % nc;
  const int f = (int)(tid / nc);
  if (m.cf_nb[f * nc + e] >= 0) return;
  const int F = m.cf_facet[f * nc + e], flip = m.cf_flip[f * nc + e];
  const double nx = m.geo[(D_NX0 + 2 * f) * nc + e], ny = m.geo[(D_NY0 + 2 * f) * nc + e];
  const double h = m.geo[(D_H0 + f) * nc + e];
  for (int mm = 0; mm < NF; ++mm) {
    double acc = 0.0;
    for (int q = 0; q < NQF; ++q) {
      const long vi = ((e * 3 + f) * NQF + q) * 2;
      acc += t.fw[q] * t.MU[q * NF + mm] * (nx * vals[vi] + ny * vals[vi + 1]);
    }
    out[(long)F * NF + mm] = -sgn(flip, mm) * h * acc;
  }
}

// ================================================================ generic
__global__ void k_csr_spmv(DCsr A, const double* __restrict__ x, double* __restrict__ y, double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double acc = 0.0;
  for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) acc += A.val[p] * x[A.idx[p]];
  y[i] = (beta != 0.0 ? beta * y[i] : 0.0) + acc;
}

__global__ void k_csr_jacobi(DCsr A, const double* __restrict__ dinv, double omega, const double* __restrict__ b,
                             const double* __restrict__ xin, double* __restrict__ xout) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= A.n) return;
  double r = b[i];
  if (xin) {
    for (int p = A.ptr[i]; p < A.ptr[i + 1]; ++p) r -= A.val[p] * xin[A.idx[p]];
    xout[i] = xin[i] + omega * dinv[i] * r;
  } else {
    xout[i] = omega * dinv[i] * r;
  }
}

__global__ void k_dense_mv(int n, const double* __restrict__ M, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int j = 0; j < n; ++j) acc += M[(long)i * n + j] * x[j];
  y[i] = acc;
}

__global__ void __launch_bounds__(kBlock) k_dot(long n, const double* __restrict__ a, const double* __restrict__ b,
                                                double* __restrict__ part) {
  double v = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v += a[i] * (b ? b[i] : a[i]);
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

// sum of a[j*stride + off]
__global__ void __launch_bounds__(kBlock) k_dot_sub(long n, int stride, int off, const double* __restrict__ a,
                                                    double* __restrict__ part) {
  double v = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    v += a[i * stride + off];
  v = block_sum(v);
  if (threadIdx.x == 0) part[blockIdx.x] = v;
}

__global__ void __launch_bounds__(kBlock) k_dot2(long n, const double* __restrict__ a, const double* __restrict__ b,
                                                 const double* __restrict__ c, double* __restrict__ part2) {
  double v = 0.0, w = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    v += a[i] * b[i];
    w += a[i] * c[i];
  }
  v = block_sum(v);
  w = block_sum(w);
  if (threadIdx.x == 0) { part2[blockIdx.x] = v; part2[kRedBlocks + blockIdx.x] = w; }
}

__global__ void __launch_bounds__(kBlock) k_finish(const double* __restrict__ part, int np, double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[0] = v;
}

__global__ void __launch_bounds__(kBlock) k_finish_mean(const double* __restrict__ part, int np, double area,
                                                        double* __restrict__ out) {
  double v = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) v += part[i];
  v = block_sum(v);
  if (threadIdx.x == 0) out[0] = v / area;
}

// out[j] = sum_{i < np} part[j * np + i] for j < nsets

__global__ void __launch_bounds__(kBlock) k_finish2(const double* __restrict__ part2, double* __restrict__ out2) {
  double v = 0.0, w = 0.0;
  for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) { v += part2[i]; w += part2[kRedBlocks + i]; }
  v = block_sum(v);
  w = block_sum(w);
  if (threadIdx.x == 0) { out2[0] = v; out2[1] = w; }
}

__global__ void k_axpby(long n, double a, const double* __restrict__ x, double b, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + (b != 0.0 ? b * y[i] : 0.0);
}
__global__ void k_copy(long n, const double* __restrict__ x, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = x[i];
}
__global__ void k_fill(long n, double v, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = v;
}
// remove the constant-trace component: g_F,0 -= sum / nF
__global__ void k_project_const(int nF, int nf, const double* __restrict__ sum, double* __restrict__ g) {
  const int F = blockIdx.x * blockDim.x + threadIdx.x;
  if (F < nF) g[(long)F * nf] -= sum[0] / (double)nF;
}

// Also returns, per block, the partial sums of the residual's coefficients
// along the trace null vector (coefficient 0 of every facet, stride nf):
// round-off of S along that vector accumulates there, and the convergence
// test leaves it out.
__global__ void __launch_bounds__(kBlock) k_pcg_update(long n, int nf, const double* __restrict__ rz,
                                                       const double* __restrict__ pq, const double* __restrict__ p,
                                                       const double* __restrict__ q, double* __restrict__ x,
                                                       double* __restrict__ r, double* __restrict__ part) {
  // a vanished p.q (converged to an exact zero residual) leaves x and r as they are
  const double alpha = pq[0] != 0.0 ? rz[0] / pq[0] : 0.0;
  double v = 0.0, s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * p[i];
    const double ri = r[i] - alpha * q[i];
    r[i] = ri;
    v += ri * ri;
    if (i % nf == 0) s += ri;
  }
  v = block_sum(v);
  s = block_sum(s);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v;
    part[gridDim.x + blockIdx.x] = s;
  }
}

// Partial sums of r.r and of the constant-trace coefficients r_0 (the layout
// k_pcg_update leaves for k_finish_proj), for a residual formed outside PCG.
__global__ void __launch_bounds__(kBlock) k_rr_partials(long n, int nf, const double* __restrict__ r,
                                                        double* __restrict__ part) {
  double v = 0.0, s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double ri = r[i];
    v += ri * ri;
    if (i % nf == 0) s += ri;
  }
  v = block_sum(v);
  s = block_sum(s);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = v;
    part[gridDim.x + blockIdx.x] = s;
  }
}

// out = sum(part[0..np)) - sum(part[np..2np))^2 / nnull: the squared norm of
// the residual with its null-vector component removed (|v|^2 = nnull)
__global__ void __launch_bounds__(kBlock) k_finish_proj(const double* __restrict__ part, int np, double nnull,
                                                        double* __restrict__ out) {
  double v = 0.0, s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    v += part[i];
    s += part[np + i];
  }
  v = block_sum(v);
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = fmax(v - s * s / nnull, 0.0);
}

__global__ void k_pcg_direction(long n, const double* __restrict__ rzn, const double* __restrict__ rzo,
                                const double* __restrict__ z, double* __restrict__ p) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + (rzo[0] != 0.0 ? rzn[0] / rzo[0] : 0.0) * p[i];
}

// ----------------------------------------------------------------- IDR(s)
// U_k = om r + sum_{i=k}^{s-1} c_i (U_i - om G_i)   (G, U stored column-major, n per column)
__global__ void k_idr_u(long n, int k, int s, IdrCoef c, double om, const double* __restrict__ r,
                        const double* __restrict__ G, double* __restrict__ U) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = om * r[i];
  for (int j = k; j < s; ++j) v += c.v[j - k] * (U[(long)j * n + i] - om * G[(long)j * n + i]);
  U[(long)k * n + i] = v;
}

// partial sums of P_j . g for j < s: part[j * kRedBlocks + block]
__global__ void __launch_bounds__(kBlock) k_multidot(long n, int s, const double* __restrict__ P,
                                                     const double* __restrict__ g, double* __restrict__ part) {
  double acc[kIdrMax];
#pragma unroll
  for (int j = 0; j < kIdrMax; ++j) acc[j] = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double gi = g[i];
#pragma unroll
    for (int j = 0; j < kIdrMax; ++j)
      if (j < s) acc[j] += P[(long)j * n + i] * gi;
  }
#pragma unroll
  for (int j = 0; j < kIdrMax; ++j) {
    if (j >= s) break;
    const double v = block_sum(acc[j]);
    if (threadIdx.x == 0) part[j * kRedBlocks + blockIdx.x] = v;
  }
}

__global__ void __launch_bounds__(kBlock) k_finish_multi(const double* __restrict__ part, int s, double* __restrict__ out) {
  for (int j = 0; j < s; ++j) {
    double v = 0.0;
    for (int i = threadIdx.x; i < kRedBlocks; i += blockDim.x) v += part[j * kRedBlocks + i];
    v = block_sum(v);
    if (threadIdx.x == 0) out[j] = v;
  }
}

// G_k -= sum_{i<k} a_i G_i; U_k -= sum_{i<k} a_i U_i; r -= beta G_k; x += beta U_k; partial |r|^2
__global__ void __launch_bounds__(kBlock) k_idr_update(long n, int k, IdrCoef a, double beta, double* __restrict__ G,
                                                       double* __restrict__ U, double* __restrict__ r,
                                                       double* __restrict__ x, double* __restrict__ part) {
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double g = G[(long)k * n + i], u = U[(long)k * n + i];
    for (int j = 0; j < k; ++j) {
      g -= a.v[j] * G[(long)j * n + i];
      u -= a.v[j] * U[(long)j * n + i];
    }
    G[(long)k * n + i] = g;
    U[(long)k * n + i] = u;
    const double ri = r[i] - beta * g;
    r[i] = ri;
    x[i] += beta * u;
    acc += ri * ri;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// x += om r; r -= om t; partial |r|^2
__global__ void __launch_bounds__(kBlock) k_idr_reduce(long n, double om, const double* __restrict__ t,
                                                       double* __restrict__ r, double* __restrict__ x,
                                                       double* __restrict__ part) {
  double acc = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double ri = r[i];
    x[i] += om * ri;
    const double rn = ri - om * t[i];
    r[i] = rn;
    acc += rn * rn;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = acc;
}

// counter-based pseudo-random shadow vectors in (-1, 1) (splitmix64 finaliser)
__global__ void k_random(long n, unsigned long long seed, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = seed + 0x9E3779B97F4A7C15ull * (unsigned long long)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  y[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
}

// ============================================================== launchers

void launch_condense(int k, hipStream_t st, DMesh m, DTab t, double c, double tau, double* Pinv, double* SK) {
  if (m.dim == 3) return launch3_condense(k, st, m, t.t3, c, tau, Pinv, SK);
  HDG_DISPATCH(k, (k_condense<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, c, tau, Pinv, SK)));
}
void launch_assemble(int k, hipStream_t st, DMesh m, const double* SK, double* vals, int* cols, double* Dinv) {
  if (m.dim == 3) return launch3_assemble(k, st, m, SK, vals, cols, Dinv);
  HDG_DISPATCH(k, (k_assemble<KK><<<nblocks(m.nF), kBlock, 0, st>>>(m, SK, vals, cols, Dinv)));
}
void launch_spmv(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* x, double* y) {
  if (k > 10) TET_TRACE_DISPATCH(k, (k_spmv_tet<KK><<<(nF + 63) / 64, TetRowsShape<KK>::NT, 0, st>>>(
                                            nF, vals, cols, x, nullptr, y)))
  else HDG_DISPATCH(k, (k_spmv<KK><<<nblocks(nF), kBlock, 0, st>>>(nF, vals, cols, x, nullptr, y)));
}
void launch_residual(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* b,
                     const double* x, double* r) {
  if (k > 10) TET_TRACE_DISPATCH(k, (k_spmv_tet<KK><<<(nF + 63) / 64, TetRowsShape<KK>::NT, 0, st>>>(
                                            nF, vals, cols, x, b, r)))
  else HDG_DISPATCH(k, (k_spmv<KK><<<nblocks(nF), kBlock, 0, st>>>(nF, vals, cols, x, b, r)));
}
void launch_jacobi_sweep(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* Dinv,
                         double omega, const double* b, const double* xin, double* xout) {
  if (k > 10) TET_TRACE_DISPATCH(k, (k_jacobi_tet<KK><<<(nF + 63) / 64, TetRowsShape<KK>::NT, 0, st>>>(
                                            nF, vals, cols, Dinv, omega, b, xin, xout)))
  else TRACE_DISPATCH(k, (k_jacobi<KK><<<nblocks(nF), kBlock, 0, st>>>(nF, vals, cols, Dinv, omega, b, xin, xout)));
}
void launch_blockdiag(int k, hipStream_t st, int nF, const double* Dinv, const double* x, double* y) {
  TRACE_DISPATCH(k, (k_blockdiag<KK><<<nblocks(nF), kBlock, 0, st>>>(nF, Dinv, x, y)));
}
void launch_rhs_condense(int k, hipStream_t st, DMesh m, DTab t, double c, double tau, const double* Pinv,
                         const double* Fw, const double* Fpsi, double* ycell) {
  if (m.dim == 3) return launch3_rhs_condense(k, st, m, t.t3, c, tau, Pinv, Fw, Fpsi, ycell);
  HDG_DISPATCH(k, (k_rhs_condense<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, c, tau, Pinv, Fw, Fpsi, ycell)));
}
void launch_gather_rhs(int k, hipStream_t st, DMesh m, const double* ycell, const double* Fmu, double* g) {
  TRACE_DISPATCH(trace_key(k, m), (k_gather_rhs<KK><<<nblocks((long)m.nF * TraceDims<KK>::NF), kBlock, 0, st>>>(
                                        m, ycell, Fmu, g)));
}
void launch_backsub(int k, hipStream_t st, DMesh m, DTab t, double c, double tau, const double* Pinv,
                    const double* Fw, const double* Fpsi, const double* lam, double* U, double* p, double* part) {
  // tetrahedra: the per-cell integrals of p go behind the partial sums in part
  if (m.dim == 3) return launch3_backsub(k, st, m, t.t3, c, tau, Pinv, Fw, Fpsi, lam, U, p, part + nblocks(m.nc), part);
  // one partial sum per block: part holds ceil(nc / kBlock) entries
  HDG_DISPATCH(k, (k_backsub<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, c, tau, Pinv, Fw, Fpsi, lam, U, p, part)));
}
void launch_gamma(int k, hipStream_t st, DMesh m, DTab t, double tau, double scale, const double* Q, const double* P,
                  const double* lam, double* gpsi, double* ycell, double* gmu) {
  if (m.dim == 3) launch3_gamma(k, st, m, t.t3, tau, scale, Q, P, lam, gpsi, ycell);
  else HDG_DISPATCH(k, (k_gamma<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, tau, scale, Q, P, lam, gpsi, ycell)));
  launch_gather_rhs(k, st, m, ycell, nullptr, gmu);
}
void launch_prep_adv(int k, hipStream_t st, DMesh m, DTab t, const double* Qs, double delta_up, double* adv) {
  if (m.dim == 3) {  // adv: V [nc][ns][ns], then beta [nc][4][nq_facet]
    const long ns = (k + 2) * (k + 3) * (k + 4) / 6;
    return launch3_prep(k, st, m, t.t3, Qs, delta_up, adv, adv + (long)m.nc * ns * ns, false);
  }
  HDG_DISPATCH(k, (k_prep_adv<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, Qs, delta_up, adv)));
}
void launch_apply(int k, hipStream_t st, int mode, DMesh m, DTab t, const double* adv, double alpha, double adt,
                  const double* x, const double* r, const double* p, const double* lam, double* out) {
  if (m.dim == 3) {
    const long ns = (k + 2) * (k + 3) * (k + 4) / 6;
    return launch3_apply(k, st, mode, 0, m, t.t3, adv, adv + (long)m.nc * ns * ns, alpha, adt, x, r, p, lam, out,
                         nullptr, nullptr, nullptr, 0, false);
  }
  if (mode == 0) {
    HDG_DISPATCH(k, (k_apply<KK, 0><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, adv, alpha, adt, x, r, p, lam, out)));
  } else if (mode == 1) {
    HDG_DISPATCH(k, (k_apply<KK, 1><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, adv, alpha, adt, x, r, p, lam, out)));
  } else {
    HDG_DISPATCH(k, (k_apply<KK, 2><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, adv, alpha, adt, x, r, p, lam, out)));
  }
}
void launch_div(int k, hipStream_t st, DMesh m, DTab t, const double* F, double scale, double* out) {
  if (m.dim == 3) return launch3_div(k, st, m, t.t3, F, scale, out);
  HDG_DISPATCH(k, (k_div<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, F, scale, out)));
}
void launch_bdm(int k, hipStream_t st, DMesh m, DTab t, const double* Q, double* Qs) {
  if (m.dim == 3) return launch3_bdm(k, st, m, t.t3, Q, Qs);
  HDG_DISPATCH(k, (k_bdm<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, Q, Qs)));
}
void launch_recon_rhs(int k, hipStream_t st, DMesh m, DTab t, const double* Q, const double* fcell,
                      const double* ffac, double fsc, double* out) {
  if (m.dim == 3) return launch3_recon_rhs(k, st, m, t.t3, Q, out);  // no forcing on tetrahedra
  HDG_DISPATCH(k, (k_recon_rhs<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, Q, fcell, ffac, fsc, out)));
}
void launch_point_dual(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* out) {
  HDG_DISPATCH(k, (k_point_dual<KK><<<nblocks((long)m.nc * Dims<KK>::NU), kBlock, 0, st>>>(m, t, vals, out)));
}
void launch_wall_flux(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* out) {
  HDG_DISPATCH(k, (k_wall_flux<KK><<<nblocks(3L * m.nc), kBlock, 0, st>>>(m, t, vals, out)));
}
// ===================================================================== tracer
// Passive tracer (Appendix "DG tracer advection"): q in DG_k (the pressure
// basis), advected by U = P_CG(Q), the L2 projection of the velocity onto
// continuous CG_{k+1}.  The CG space is nodal Lagrange on equispaced points;
// T maps a cell's nodal values to its Dubiner coefficients (L_a =
// sum_s T[s][a] phi_s), l2g its nodes to global CG unknowns.

// b[d] = (L_d, Q_comp): sum over the (cell, node) incidences of unknown d of
// det * sum_s T[s][a] Q[cell][comp][s] (the Dubiner mass is det * I).
__global__ void k_cg_rhs(int N, const int* __restrict__ ptr, const int* __restrict__ inc, int ns,
                         const double* __restrict__ T, const double* __restrict__ geo, int nc,
                         const double* __restrict__ Q, int comp, double* __restrict__ b) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= N) return;
  double acc = 0.0;
  for (int p = ptr[d]; p < ptr[d + 1]; ++p) {
    const int e = inc[p] / ns, a = inc[p] - e * ns;
    const double* Qe = Q + ((long)e * 2 + comp) * ns;
    double v = 0.0;
    for (int s = 0; s < ns; ++s) v += T[s * ns + a] * Qe[s];
    acc += geo[D_DET * (long)nc + e] * v;
  }
  b[d] = acc;
}

// U[cell][comp][s] = sum_a T[s][a] u[l2g[cell][a]]
__global__ void k_cg_to_dg(long nc, int ns, const double* __restrict__ T, const int* __restrict__ l2g,
                           const double* __restrict__ u, int comp, double* __restrict__ U) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc * ns) return;
  const long e = i / ns;
  const int s = (int)(i - e * ns);
  double v = 0.0;
  for (int a = 0; a < ns; ++a) v += T[s * ns + a] * u[l2g[e * ns + a]];
  U[(e * 2 + comp) * ns + s] = v;
}

// L2 projection of point values onto the tracer space (orthonormal basis:
// coefficient s = sum_q w_q phi_s(x_q) v_q)
template <int K>
__global__ void __launch_bounds__(kBlock) k_project_scalar(DMesh m, DTab t, const double* __restrict__ vals,
                                                           double* __restrict__ q) {
  using D = Dims<K>;
  constexpr int NP = D::NP, NQC = D::NQC;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  double o[NP];
#pragma unroll
  for (int i = 0; i < NP; ++i) o[i] = 0.0;
  for (int qq = 0; qq < NQC; ++qq) {
    const double v = t.cw[qq] * vals[(long)e * NQC + qq];
#pragma unroll
    for (int s = 0; s < NP; ++s) o[s] += t.Bp[qq * NP + s] * v;
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) q[(long)e * NP + i] = o[i];
}

// out = M^-1 a(., q, U): volume (q, div(chi U)) and, on interior facets,
// -<q^up [[chi U.n]]> with q^up from the side U.n points away from.
template <int K>
__global__ void __launch_bounds__(kBlock) k_tracer_rate(DMesh m, DTab t, const double* __restrict__ U,
                                                        const double* __restrict__ q, double* __restrict__ out) {
  using D = Dims<K>;
  constexpr int NS = D::NS, NP = D::NP, NQC = D::NQC, NQF = D::NQF;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m.nc) return;
  const long nc = m.nc;
  const CellGeo g = load_geo(m, e);
  double uc[2 * NS], qv[NP], o[NP];
#pragma unroll
  for (int i = 0; i < 2 * NS; ++i) uc[i] = U[(long)e * 2 * NS + i];
#pragma unroll
  for (int i = 0; i < NP; ++i) {
    qv[i] = q[(long)e * NP + i];
    o[i] = 0.0;
  }
  for (int qq = 0; qq < NQC; ++qq) {
    double ux = 0.0, uy = 0.0, dxx = 0.0, dxe = 0.0, dyx = 0.0, dye = 0.0, qval = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const double b = t.Bu[qq * NS + s], gx = t.Gux[qq * NS + s], gy = t.Guy[qq * NS + s];
      ux += b * uc[s];
      uy += b * uc[NS + s];
      dxx += gx * uc[s];       // d Ux / d xi
      dxe += gy * uc[s];       // d Ux / d eta
      dyx += gx * uc[NS + s];  // d Uy / d xi
      dye += gy * uc[NS + s];
    }
#pragma unroll
    for (int s = 0; s < NP; ++s) qval += t.Bp[qq * NP + s] * qv[s];
    // physical derivative d/dx_d = sum_a d/dxi_a ij[a][d]
    const double div = g.ij[0][0] * dxx + g.ij[1][0] * dxe + g.ij[0][1] * dyx + g.ij[1][1] * dye;
    const double a0 = g.ij[0][0] * ux + g.ij[0][1] * uy;  // sum_d ij[0][d] U_d
    const double a1 = g.ij[1][0] * ux + g.ij[1][1] * uy;
    const double w = t.cw[qq] * g.det * qval;
#pragma unroll
    for (int i = 0; i < NP; ++i)
      o[i] += w * (t.Gpx[qq * NP + i] * a0 + t.Gpy[qq * NP + i] * a1 + t.Bp[qq * NP + i] * div);
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int nb = m.cf_nb[f * nc + e];
    if (nb < 0) continue;  // walls carry no term
    const int fn = m.cf_nbf[f * nc + e];
    const int rev = m.cf_flip[f * nc + e] != m.cf_flip[fn * nc + nb];
    double qn[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) qn[i] = q[(long)nb * NP + i];
    for (int qq = 0; qq < NQF; ++qq) {
      const int qm = rev ? NQF - 1 - qq : qq;
      double ux = 0.0, uy = 0.0, qo = 0.0, qb = 0.0;
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const double b = t.FBu[(f * NQF + qq) * NS + s];
        ux += b * uc[s];
        uy += b * uc[NS + s];
      }
#pragma unroll
      for (int s = 0; s < NP; ++s) {
        qo += t.FBp[(f * NQF + qq) * NP + s] * qv[s];
        qb += t.FBp[(fn * NQF + qm) * NP + s] * qn[s];
      }
      const double un = ux * g.n[f][0] + uy * g.n[f][1];
      const double flux = t.fw[qq] * g.h[f] * un * (un >= 0.0 ? qo : qb);
#pragma unroll
      for (int i = 0; i < NP; ++i) o[i] -= t.FBp[(f * NQF + qq) * NP + i] * flux;
    }
  }
#pragma unroll
  for (int i = 0; i < NP; ++i) out[(long)e * NP + i] = o[i] / g.det;
}

void launch_cg_rhs(hipStream_t st, int N, const int* ptr, const int* inc, int ns, const double* T, DMesh m,
                   const double* Q, int comp, double* b) {
  k_cg_rhs<<<nblocks(N), kBlock, 0, st>>>(N, ptr, inc, ns, T, m.geo, m.nc, Q, comp, b);
}
void launch_cg_to_dg(hipStream_t st, long nc, int ns, const double* T, const int* l2g, const double* u, int comp,
                     double* U) {
  k_cg_to_dg<<<nblocks(nc * ns), kBlock, 0, st>>>(nc, ns, T, l2g, u, comp, U);
}
void launch_project_scalar(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* q) {
  HDG_DISPATCH(k, (k_project_scalar<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, vals, q)));
}
void launch_tracer_rate(int k, hipStream_t st, DMesh m, DTab t, const double* U, const double* q, double* out) {
  HDG_DISPATCH(k, (k_tracer_rate<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, U, q, out)));
}


// ------------------------------------------------------------------ small PCG
// Facet-block-Jacobi PCG on a small trace system in one workgroup: every
// iteration (S p, the updates, the block-Jacobi preconditioner with the
// null-vector projection, the new direction) runs between workgroup
// barriers, so a solve is one launch instead of a dozen per iteration.  The
// arithmetic is that of the multi-launch path (projected residual norm, the
// same round-off-floor stop); only the summation order of the inner
// products differs.  info: iterations, final squared residual (null
// component removed), floor stop, converged.  Workgroup size 512: fewer
// waves make each barrier cheaper (on 1600 unknowns a solve took 3.9 ms
// against 4.8 ms with 1024 threads and 4.0 ms with 256; on 9408 unknowns,
// vectors in global memory, 27.9 against 31.6 ms with 1024).
constexpr int kSmallBlock = 512;

// No barrier follows the final reads of sh: a caller alternates two scratch
// areas between consecutive reductions, so the barrier inside the next
// reduction orders those reads before sh is written again.
template <int BS>
__device__ __forceinline__ void small_reduce(double* v, int nv, double* sh) {
  // sh: shared scratch of nv * (BS / 64) doubles; all threads get the sums
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int c = 0; c < nv; ++c) {
    double x = v[c];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_down(x, o, 64);
    if (lane == 0) sh[c * (BS / 64) + w] = x;
  }
  __syncthreads();
  for (int c = 0; c < nv; ++c) {
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < BS / 64; ++i) s += sh[c * (BS / 64) + i];
    v[c] = s;
  }
}

// Up to kSmallLds unknowns the work vectors r, z, p, q live in LDS
// (4 x 1920 doubles = 60 KiB); beyond that in global memory.  With REG (one
// facet per thread at most, degree 1) each thread also keeps its facet's
// neighbour list and preconditioner block in registers for the whole solve,
// so that no load of an iteration waits on another global load (the operator
// values are still loaded every iteration, independently: kept in registers
// too they would spill); the arithmetic is the same.
constexpr int kSmallLds = 1920;

template <int K, bool LDS, bool REG, int BS>
__global__ void __launch_bounds__(BS) k_pcg_small(int nF, const double* __restrict__ vals,
                                                           const int* __restrict__ cols, const double* __restrict__ Dinv,
                                                           const double* __restrict__ g, double* __restrict__ x,
                                                           double* __restrict__ rg, double* __restrict__ zg,
                                                           double* __restrict__ pg, double* __restrict__ qg, int maxit,
                                                           double tol2, double floor2, int flat_blocks,
                                                           double* __restrict__ info) {
  constexpr int NF = TraceDims<K>::NF, SL = TraceDims<K>::SL;
  // reduction scratch: shq for p.q, shr for the four sums of the update pass
  // (alternating areas; see small_reduce)
  __shared__ double shq[BS / 64], shr[4 * (BS / 64)];
  __shared__ double sv[LDS ? 4 : 1][LDS ? kSmallLds : 1];
  double* r = LDS ? sv[0] : rg;
  double* z = LDS ? sv[1] : zg;
  double* p = LDS ? sv[2] : pg;
  double* q = LDS ? sv[3] : qg;
  const int tid = threadIdx.x;
  const double nnull = (double)nF;
  static_assert(!REG || (K == 1 && LDS), "register caching is for degree 1 with LDS vectors");
  constexpr int NR = REG ? NF : 1;
  double rD[NR][NR];
  int rc[REG ? SL : 1];
  if constexpr (REG) {
    const int F = tid < nF ? tid : 0;
#pragma unroll
    for (int s = 0; s < SL; ++s) rc[s] = cols[s * nF + F];
#pragma unroll
    for (int i = 0; i < NF; ++i)
#pragma unroll
      for (int j = 0; j < NF; ++j) rD[i][j] = Dinv[(long)(i * NF + j) * nF + F];
  }
  // Every pass below maps a thread to whole facets, so q, r and z of a facet
  // are written and read by the same thread and only p (read across facets
  // by S p) needs a barrier between passes.
  // z_F = Dinv_F r_F; red = (r.r, sum r_0, r.z, sum z_0)
  auto precond_facet = [&](int F, double* red) {
    double rv[NF];
#pragma unroll
    for (int j = 0; j < NF; ++j) rv[j] = r[F * NF + j];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < NF; ++j) {
        if constexpr (REG) v += rD[i][j] * rv[j];
        else v += Dinv[(long)(i * NF + j) * nF + F] * rv[j];
      }
      z[F * NF + i] = v;
      red[0] += rv[i] * rv[i];
      red[2] += rv[i] * v;
    }
    red[1] += rv[0];
    red[3] += z[F * NF];
  };
  double red[4] = {0.0, 0.0, 0.0, 0.0};
  for (int F = tid; F < nF; F += BS) {
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      x[(long)F * NF + i] = 0.0;
      r[F * NF + i] = g[(long)F * NF + i];
    }
    precond_facet(F, red);
  }
  small_reduce<BS>(red, 4, shr);
  double mean = red[3] / nnull;
  double rz = red[2] - mean * red[1];
  for (int F = tid; F < nF; F += BS)
#pragma unroll
    for (int i = 0; i < NF; ++i) p[F * NF + i] = z[F * NF + i] - (i == 0 ? mean : 0.0);
  __syncthreads();
  double rr = 0.0, best_rz = 1e300, low = 1e300;
  int it = 0, flat = 0, conv = 0, floor_stop = 0;
  while (it < maxit) {
    // q = S p and p.q
    double pq = 0.0;
    for (int F = tid; F < nF; F += BS) {
      double pc[SL][NF];
#pragma unroll
      for (int s = 0; s < SL; ++s) {
        const int col = REG ? rc[REG ? s : 0] : cols[s * nF + F];
#pragma unroll
        for (int j = 0; j < NF; ++j) pc[s][j] = p[col * NF + j];
      }
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < SL; ++s)
#pragma unroll
          for (int j = 0; j < NF; ++j) acc += vals[((long)(s * NF + i) * NF + j) * nF + F] * pc[s][j];
        q[F * NF + i] = acc;
        pq += p[F * NF + i] * acc;
      }
    }
    small_reduce<BS>(&pq, 1, shq);
    const double alpha = pq != 0.0 ? rz / pq : 0.0;
    // x, r updates and the preconditioner, facet by facet
    red[0] = red[1] = red[2] = red[3] = 0.0;
    for (int F = tid; F < nF; F += BS) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        x[(long)F * NF + i] += alpha * p[F * NF + i];
        r[F * NF + i] -= alpha * q[F * NF + i];
      }
      precond_facet(F, red);
    }
    small_reduce<BS>(red, 4, shr);
    rr = fmax(red[0] - red[1] * red[1] / nnull, 0.0);
    ++it;
    if (rr <= tol2) { conv = 1; break; }
    mean = red[3] / nnull;
    const double rzn = red[2] - mean * red[1];
    low = fmin(low, fabs(rzn));
    if (it % 4 == 0) {  // blocks of four iterations, as the multi-launch path checks
      // stalls judged on r.z (1 % per block in norm), accepted with the current |r| within the floor
      if (low < 0.98 * best_rz) { best_rz = low; flat = 0; }
      else if (++flat >= max(flat_blocks, it / 16) && rr <= floor2) { floor_stop = 1; break; }
      low = 1e300;
    }
    const double beta = rz != 0.0 ? rzn / rz : 0.0;
    rz = rzn;
    for (int F = tid; F < nF; F += BS)
#pragma unroll
      for (int i = 0; i < NF; ++i) p[F * NF + i] = z[F * NF + i] - (i == 0 ? mean : 0.0) + beta * p[F * NF + i];
    __syncthreads();
  }
  if (tid == 0) {
    info[0] = it;
    info[1] = rr;
    info[2] = floor_stop;
    info[3] = conv;
  }
}

void launch_pcg_small(int k, hipStream_t st, int nF, const double* vals, const int* cols, const double* Dinv,
                      const double* g, double* x, double* r, double* z, double* p, double* q, int maxit, double tol2,
                      double floor2, int flat_blocks, double* info) {
  constexpr int BS = kSmallBlock;
  const int nf = k < 10 ? k + 1 : (k - 9) * (k - 8) / 2;  // k is the trace key here
  if ((long)nF * nf <= kSmallLds) {
    if (k == 1 && nF <= BS) {
      k_pcg_small<1, true, true, BS><<<1, BS, 0, st>>>(nF, vals, cols, Dinv, g, x, r, z, p, q, maxit, tol2, floor2,
                                                       flat_blocks, info);
    } else {
      TRACE_DISPATCH(k, (k_pcg_small<KK, true, false, BS><<<1, BS, 0, st>>>(nF, vals, cols, Dinv, g, x, r, z, p, q,
                                                                           maxit, tol2, floor2, flat_blocks, info)));
    }
  } else {
    TRACE_DISPATCH(k, (k_pcg_small<KK, false, false, BS><<<1, BS, 0, st>>>(nF, vals, cols, Dinv, g, x, r, z, p, q,
                                                                          maxit, tol2, floor2, flat_blocks, info)));
  }
}

void launch_project(int k, hipStream_t st, DMesh m, DTab t, const double* vals, double* Q) {
  if (m.dim == 3) return launch3_project(k, st, m, t.t3, vals, Q);
  HDG_DISPATCH(k, (k_project<KK><<<nblocks(m.nc), kBlock, 0, st>>>(m, t, vals, Q)));
}
void launch_mass(int k, hipStream_t st, DMesh m, double s, const double* x, double* y) {
  if (m.dim == 3) return launch3_mass(k, st, m, s, x, y);
  HDG_DISPATCH(k, (k_mass<KK><<<nblocks((long)m.nc * Dims<KK>::NU), kBlock, 0, st>>>(m, s, x, y)));
}
void launch_shift_mean(int k, hipStream_t st, DMesh m, const double* mean, double* p, double* lam) {
  if (m.dim == 3) return launch3_shift_mean(k, st, m, mean, p, lam);
  const long n = m.nc > m.nF ? m.nc : m.nF;
  HDG_DISPATCH(k, (k_shift_mean<KK><<<nblocks(n), kBlock, 0, st>>>(m, mean, p, lam)));
}
void launch_csr_spmv(hipStream_t st, DCsr A, const double* x, double* y, double beta) {
  k_csr_spmv<<<nblocks(A.n), kBlock, 0, st>>>(A, x, y, beta);
}
void launch_csr_jacobi(hipStream_t st, DCsr A, const double* dinv, double omega, const double* b, const double* xin,
                       double* xout) {
  k_csr_jacobi<<<nblocks(A.n), kBlock, 0, st>>>(A, dinv, omega, b, xin, xout);
}
void launch_dense_mv(hipStream_t st, int n, const double* M, const double* x, double* y) {
  k_dense_mv<<<nblocks(n), kBlock, 0, st>>>(n, M, x, y);
}
void launch_dot(hipStream_t st, long n, const double* a, const double* b, double* part) {
  k_dot<<<kRedBlocks, kBlock, 0, st>>>(n, a, b, part);
}
void launch_dot_sub(hipStream_t st, long n, int stride, int off, const double* a, double* part) {
  k_dot_sub<<<kRedBlocks, kBlock, 0, st>>>(n, stride, off, a, part);
}
void launch_finish(hipStream_t st, const double* part, int nparts, double* out) {
  k_finish<<<1, kBlock, 0, st>>>(part, nparts, out);
}
void launch_finish_mean(hipStream_t st, const double* part, int nparts, double area, double* out) {
  k_finish_mean<<<1, kBlock, 0, st>>>(part, nparts, area, out);
}
void launch_axpby(hipStream_t st, long n, double a, const double* x, double b, double* y) {
  k_axpby<<<nblocks(n), kBlock, 0, st>>>(n, a, x, b, y);
}
void launch_copy(hipStream_t st, long n, const double* x, double* y) {
  k_copy<<<nblocks(n), kBlock, 0, st>>>(n, x, y);
}
void launch_fill(hipStream_t st, long n, double v, double* y) { k_fill<<<nblocks(n), kBlock, 0, st>>>(n, v, y); }
// Point values of the cell polynomials: thread per (cell, point); BU, BP are
// the velocity and pressure bases at the points ([npts][ns], [npts][np]).
__global__ void k_eval_points(long nc, int npts, int ns, int np, const double* __restrict__ BU,
                              const double* __restrict__ BP, const double* __restrict__ Q,
                              const double* __restrict__ p, double* __restrict__ Qo, double* __restrict__ po) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nc * npts) return;
  const long e = i / npts;
  const int q = (int)(i - e * npts);
  if (Qo) {
    const double* Qe = Q + e * 2 * ns;
    double ux = 0.0, uy = 0.0;
    for (int s = 0; s < ns; ++s) {
      const double b = BU[q * ns + s];
      ux += b * Qe[s];
      uy += b * Qe[ns + s];
    }
    Qo[2 * i] = ux;
    Qo[2 * i + 1] = uy;
  }
  if (po) {
    const double* pe = p + e * np;
    double v = 0.0;
    for (int s = 0; s < np; ++s) v += BP[q * np + s] * pe[s];
    po[i] = v;
  }
}

void launch_eval_points(hipStream_t st, long nc, int npts, int ns, int np, const double* BU, const double* BP,
                        const double* Q, const double* p, double* Qo, double* po) {
  const long n = nc * npts;
  k_eval_points<<<(int)((n + kBlock - 1) / kBlock), kBlock, 0, st>>>(nc, npts, ns, np, BU, BP, Q, p, Qo, po);
}

void launch_project_const(hipStream_t st, int nF, int nf, const double* sum, double* g) {
  k_project_const<<<nblocks(nF), kBlock, 0, st>>>(nF, nf, sum, g);
}
void launch_pcg_update(hipStream_t st, long n, int nf, const double* rz, const double* pq, const double* p,
                       const double* q, double* x, double* r, double* part_rr) {
  k_pcg_update<<<kRedBlocks, kBlock, 0, st>>>(n, nf, rz, pq, p, q, x, r, part_rr);
}
void launch_rr_partials(hipStream_t st, long n, int nf, const double* r, double* part) {
  k_rr_partials<<<kRedBlocks, kBlock, 0, st>>>(n, nf, r, part);
}
void launch_finish_proj(hipStream_t st, const double* part, int nparts, double nnull, double* out) {
  k_finish_proj<<<1, kBlock, 0, st>>>(part, nparts, nnull, out);
}
void launch_pcg_direction(hipStream_t st, long n, const double* rzn, const double* rzo, const double* z, double* p) {
  k_pcg_direction<<<nblocks(n), kBlock, 0, st>>>(n, rzn, rzo, z, p);
}
void launch_dot2(hipStream_t st, long n, const double* a, const double* b, const double* c, double* part2) {
  k_dot2<<<kRedBlocks, kBlock, 0, st>>>(n, a, b, c, part2);
}
void launch_finish2(hipStream_t st, const double* part2, double* out2) { k_finish2<<<1, kBlock, 0, st>>>(part2, out2); }
void launch_idr_u(hipStream_t st, long n, int k, int s, IdrCoef c, double om, const double* r, const double* G,
                  double* U) {
  k_idr_u<<<nblocks(n), kBlock, 0, st>>>(n, k, s, c, om, r, G, U);
}
void launch_multidot(hipStream_t st, long n, int s, const double* P, const double* g, double* part, double* out) {
  k_multidot<<<kRedBlocks, kBlock, 0, st>>>(n, s, P, g, part);
  k_finish_multi<<<1, kBlock, 0, st>>>(part, s, out);
}
void launch_idr_update(hipStream_t st, long n, int k, IdrCoef a, double beta, double* G, double* U, double* r,
                       double* x, double* part) {
  k_idr_update<<<kRedBlocks, kBlock, 0, st>>>(n, k, a, beta, G, U, r, x, part);
}
void launch_idr_reduce(hipStream_t st, long n, double om, const double* t, double* r, double* x, double* part) {
  k_idr_reduce<<<kRedBlocks, kBlock, 0, st>>>(n, om, t, r, x, part);
}
void launch_random(hipStream_t st, long n, unsigned long long seed, double* y) {
  k_random<<<nblocks(n), kBlock, 0, st>>>(n, seed, y);
}

}  // namespace hdg
