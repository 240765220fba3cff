// gfx950 kernels of the HDG-IMEX library on tetrahedra (d = 3).
//
// The forms are those of the triangle kernels (Section 2 of the paper: the
// mass, f_im of eq. (f_impl), g and Gamma of Section "Hybridisation", the
// weak divergence, the BDM interpolant), with velocity [P_{k+1}]^3, pressure
// P_k and trace P_k on triangles.  A cell's local problems are small dense
// matrices (60 velocity, 10 pressure and 24 trace unknowns at k = 2), so one
// 64-lane wavefront works on one cell: the lanes split the rows or entries
// of a local matrix and the cell's data are staged in LDS.  Reference tables
// are read through the L2; their facet tables are indexed by the local facet
// and its orientation (fp = 6 f + p), the same for every lane of the wave.
// Vectors are cell-major ([cell][component][basis]), as in the triangle path.
// All reductions use a fixed grid and order (bitwise reproducible).
#include <hip/hip_runtime.h>

#include <stdexcept>

#include "device_common.h"
#include "kernels.h"

namespace hdg {

template <int K>
struct Dims3 {
  static constexpr int NS = (K + 2) * (K + 3) * (K + 4) / 6;
  static constexpr int NP = (K + 1) * (K + 2) * (K + 3) / 6;
  static constexpr int NF = (K + 1) * (K + 2) / 2;
  static constexpr int NB = (K + 2) * (K + 3) / 2;
  static constexpr int NNED = K * (K + 2) * (K + 3) / 2;
  static constexpr int NU = 3 * NS;
  static constexpr int NL = 4 * NF;
  static constexpr int NQ1 = (3 * K + 4) / 2;
  static constexpr int NQC = NQ1 * NQ1 * NQ1;
  static constexpr int NQF1 = (3 * K + 5) / 2;
  static constexpr int NQF = NQF1 * NQF1;
};

constexpr int kW3 = 64;  // lanes per cell
typedef double f64x4_3 __attribute__((ext_vector_type(4)));  // accumulator of v_mfma_f64_16x16x4f64

struct Geo3 {
  double det, ij[3][3], n[4][3], a[4];
};

__device__ __forceinline__ Geo3 load_geo3(const DMesh& m, int e) {
  Geo3 g;
  const double* G = m.geo;
  const long nc = m.nc;
  g.det = G[(long)E3_DET * nc + e];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) g.ij[a][b] = G[(long)(E3_IJ + 3 * a + b) * nc + e];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
#pragma unroll
    for (int c = 0; c < 3; ++c) g.n[f][c] = G[(long)(E3_N + 3 * f + c) * nc + e];
    g.a[f] = G[(long)(E3_A + f) * nc + e];
  }
  return g;
}

__device__ __forceinline__ void load_j3(const DMesh& m, int e, double (&J)[3][3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) J[a][b] = m.geo[(long)(E3_J + 3 * a + b) * m.nc + e];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Gauss-Jordan inverse of an SPD n x n matrix held in LDS as [n][2n]
// (A | I) by one wave (a 64-thread workgroup): the lanes split the entries
// of each elimination step; col holds the step's multipliers.
template <int N>
__device__ void wave_invert(double (&A)[N][2 * N], double (&col)[N]) {
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < N; ++c) {
    __syncthreads();
    const double piv = 1.0 / A[c][c];
    for (int r = lane; r < N; r += 64) col[r] = A[r][c];
    __syncthreads();
    for (int j = lane; j < 2 * N; j += 64) A[c][j] *= piv;
    __syncthreads();
    for (int idx = lane; idx < N * 2 * N; idx += 64) {
      const int r = idx / (2 * N), j = idx % (2 * N);
      if (r != c) A[r][j] -= col[r] * A[c][j];
    }
  }
  __syncthreads();
}

// ===================================================================== a1
// Local condensation.  With orthonormal reference bases the velocity mass is
// det I, so the cell problem reduces to the pressure Schur complement
//   P = tau sum_f |F_f| That_f + c det sum_ab (iJ iJ^T)_ab KDD_ab,
// and the cell's trace operator is
//   S_K = tau |F| I + (c/det) Gl^T Gl - W^T P^{-1} W,
//   W[i][(f,m)] = -|F_f| (c sum_a nu_fa CD[fp][a][m][i] + tau Ehat[fp][m][i]),
//   nu_fa = sum_c iJ[a][c] n_f[c],  (Gl^T Gl) = |F_f||F_g| (n_f.n_g) Chat_f Chat_g^T.
template <int K>
__global__ void __launch_bounds__(kW3) k3_condense(DMesh m, DTab3 t, double c, double tau, double* __restrict__ Pinv,
                                                   double* __restrict__ SK) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NL = D::NL;
  const int e = blockIdx.x;
  const int lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  int fpv[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) fpv[f] = 6 * f + m.cf_flip[f * nc + e];
  __shared__ double A[NP][2 * NP];
  __shared__ double colb[NP];
  __shared__ double W[NP][NL];
  __shared__ double Y[NP][NL];
  double Gm[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) Gm[a][b] = g.ij[a][0] * g.ij[b][0] + g.ij[a][1] * g.ij[b][1] + g.ij[a][2] * g.ij[b][2];
  for (int idx = lane; idx < NP * NP; idx += kW3) {
    const int i = idx / NP, j = idx % NP;
    double v = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) v += g.a[f] * t.That[(f * NP + i) * NP + j];
    double dd = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) dd += Gm[a][b] * t.KDD[((a * 3 + b) * NP + i) * NP + j];
    A[i][j] = tau * v + c * g.det * dd;
    A[i][NP + j] = (i == j) ? 1.0 : 0.0;
  }
  wave_invert<NP>(A, colb);
  for (int idx = lane; idx < NP * NP; idx += kW3) {
    const int i = idx / NP, j = idx % NP;
    Pinv[(long)(i * NP + j) * nc + e] = A[i][NP + j];
  }
  for (int idx = lane; idx < NP * NL; idx += kW3) {
    const int i = idx / NL, r = idx % NL, f = r / NF, mm = r % NF;
    const int fp = fpv[f];
    double nu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) nu[a] = g.ij[a][0] * g.n[f][0] + g.ij[a][1] * g.n[f][1] + g.ij[a][2] * g.n[f][2];
    double v = tau * t.Ehat[(fp * NF + mm) * NP + i];
#pragma unroll
    for (int a = 0; a < 3; ++a) v += c * nu[a] * t.CD[((fp * 3 + a) * NF + mm) * NP + i];
    W[i][r] = -g.a[f] * v;
  }
  __syncthreads();
  // Y = P^{-1} W and W^T Y on the FP64 matrix cores (v_mfma_f64_16x16x4f64:
  // lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16] and holds
  // D[4 v + l / 16][l % 16] in its accumulator double v), zero-padded to
  // tiles of 16 rows and columns and steps of 4 in the contracted index.
  constexpr int NLT = (NL + 15) / 16, NKP = (NP + 3) / 4;
  static_assert(NP <= 16, "one row tile of P^{-1}");
  const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
  for (int tj = 0; tj < NLT; ++tj) {
    const int col = 16 * tj + lc;
    f64x4_3 y = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int kk = 0; kk < NKP; ++kk) {
      const int kq = 4 * kk + lr;
      const double a = (lc < NP && kq < NP) ? A[lc][NP + kq] : 0.0;
      const double b = (kq < NP && col < NL) ? W[kq][col] : 0.0;
      y = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, y, 0, 0, 0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v)
      if (4 * v + lr < NP && col < NL) Y[4 * v + lr][col] = y[v];
  }
  __syncthreads();
  const double cod = c / g.det;
#pragma unroll
  for (int ti = 0; ti < NLT; ++ti)
#pragma unroll
    for (int tj = 0; tj < NLT; ++tj) {
      f64x4_3 ww = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < NKP; ++kk) {
        const int kq = 4 * kk + lr;
        const double a = (kq < NP && 16 * ti + lc < NL) ? W[kq][16 * ti + lc] : 0.0;  // W^T
        const double b = (kq < NP && 16 * tj + lc < NL) ? Y[kq][16 * tj + lc] : 0.0;
        ww = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, ww, 0, 0, 0);
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * ti + 4 * v + lr, s = 16 * tj + lc;
        if (r >= NL || s >= NL) continue;
        const int f = r / NF, mm = r % NF, gg = s / NF, l = s % NF;
        const double* cf = t.Chat + (long)(fpv[f] * NF + mm) * NS;
        const double* cg = t.Chat + (long)(fpv[gg] * NF + l) * NS;
        double cc = 0.0;
#pragma unroll
        for (int q = 0; q < NS; ++q) cc += cf[q] * cg[q];
        const double nn = g.n[f][0] * g.n[gg][0] + g.n[f][1] * g.n[gg][1] + g.n[f][2] * g.n[gg][2];
        double x = (r == s) ? tau * g.a[f] : 0.0;
        x += cod * g.a[f] * g.a[gg] * nn * cc;
        SK[(long)(r * NL + s) * nc + e] = x - ww[v];
      }
    }
}

// Facet-block ELL assembly of S = sum_K S_K, one thread per facet (no
// atomics).  Slot 0: the facet itself; slots 1-3: the other facets of K+ in
// local order; slots 4-6: those of K- (column F with zero blocks on walls).
template <int K>
__global__ void __launch_bounds__(kBlock) k3_assemble(DMesh m, const double* __restrict__ SK,
                                                      double* __restrict__ vals, int* __restrict__ cols,
                                                      double* __restrict__ Dinv) {
  using D = Dims3<K>;
  constexpr int NF = D::NF, NL = D::NL;
  const int F = blockIdx.x * blockDim.x + threadIdx.x;
  const int nF = m.nF;
  if (F >= nF) return;
  const long nc = m.nc;
  const int Kp = m.fc_cell[F], fp = m.fc_f[F], Km = m.fc_cell[nF + F], fm = m.fc_f[nF + F];
  auto put = [&](int slot, int col, int cell, int fr, int fcol, bool add) {
    if (!add) cols[slot * nF + F] = col;
    for (int i = 0; i < NF; ++i)
      for (int j = 0; j < NF; ++j) {
        const double v = cell >= 0 ? SK[(long)((fr * NF + i) * NL + fcol * NF + j) * nc + cell] : 0.0;
        const long idx = ((long)(slot * NF + i) * NF + j) * nF + F;
        vals[idx] = add ? vals[idx] + v : v;
      }
  };
  put(0, F, Kp, fp, fp, false);
  if (Km >= 0) put(0, F, Km, fm, fm, true);
  for (int o = 1; o <= 3; ++o) {
    const int gq = (fp + o) & 3;
    put(o, m.cf_facet[gq * nc + Kp], Kp, fp, gq, false);
  }
  for (int o = 1; o <= 3; ++o) {
    if (Km >= 0) {
      const int gq = (fm + o) & 3;
      put(3 + o, m.cf_facet[gq * nc + Km], Km, fm, gq, false);
    } else {
      put(3 + o, F, -1, 0, 0, false);
    }
  }
  double A[NF][NF], B[NF][NF];
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) {
      A[i][j] = vals[((long)i * NF + j) * nF + F];
      B[i][j] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int cidx = 0; cidx < NF; ++cidx) {
    const double dd = 1.0 / A[cidx][cidx];
#pragma unroll
    for (int j = 0; j < NF; ++j) { A[cidx][j] *= dd; B[cidx][j] *= dd; }
#pragma unroll
    for (int r = 0; r < NF; ++r) {
      if (r == cidx) continue;
      const double f = A[r][cidx];
#pragma unroll
      for (int j = 0; j < NF; ++j) { A[r][j] -= f * A[cidx][j]; B[r][j] -= f * B[cidx][j]; }
    }
  }
#pragma unroll
  for (int i = 0; i < NF; ++i)
#pragma unroll
    for (int j = 0; j < NF; ++j) Dinv[(long)(i * NF + j) * nF + F] = B[i][j];
}

// ================================================================ a7, a9
// Cell data of the condensed right-hand side and the back-substitution.
// (Gp^T F)_i = det sum_a sum_s D_a[i][s] (sum_c iJ[a][c] F_c[s]).
template <int K>
__device__ __forceinline__ void stage_vel(const double* __restrict__ src, int e, double* dst) {
  constexpr int NU = Dims3<K>::NU;
  const int lane = threadIdx.x;
  for (int i = lane; i < NU; i += kW3) dst[i] = src ? src[(long)e * NU + i] : 0.0;
}

// p = P^{-1} (fpsi - Gp^T fw / det) with fw, fpsi in LDS, p to LDS
template <int K>
__device__ __forceinline__ void pressure_solve3(const DTab3& t, const Geo3& g, const double* Pinv, long nc, int e,
                                                const double* fw, const double* fpsi, double* b, double* p) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP;
  const int lane = threadIdx.x;
  for (int i = lane; i < NP; i += kW3) {
    double v = 0.0;
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double u = g.ij[a][0] * fw[s] + g.ij[a][1] * fw[NS + s] + g.ij[a][2] * fw[2 * NS + s];
        v += t.D[(a * NP + i) * NS + s] * u;
      }
    }
    b[i] = fpsi[i] - v;  // f_psi - (Gp^T f_w) / det
  }
  __syncthreads();
  for (int i = lane; i < NP; i += kW3) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) v += Pinv[(long)(i * NP + j) * nc + e] * b[j];
    p[i] = v;
  }
  __syncthreads();
}

// y[(f,m)] = -(Gl^T Fw)[(f,m)] / det - (W^T p0)[(f,m)],  p0 = P^{-1}(Fpsi - Gp^T Fw / det)
template <int K>
__global__ void __launch_bounds__(kW3) k3_rhs_condense(DMesh m, DTab3 t, double c, double tau,
                                                       const double* __restrict__ Pinv, const double* __restrict__ Fw,
                                                       const double* __restrict__ Fpsi, double* __restrict__ ycell) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU, NL = D::NL;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double fw[NU], fpsi[NP], b[NP], p[NP];
  stage_vel<K>(Fw, e, fw);
  for (int i = lane; i < NP; i += kW3) fpsi[i] = Fpsi ? Fpsi[(long)e * NP + i] : 0.0;
  __syncthreads();
  pressure_solve3<K>(t, g, Pinv, nc, e, fw, fpsi, b, p);
  for (int r = lane; r < NL; r += kW3) {
    const int f = r / NF, mm = r % NF;
    const int fp = 6 * f + m.cf_flip[f * nc + e];
    double cf = 0.0;  // (Chat n.fw)
    for (int s = 0; s < NS; ++s)
      cf += t.Chat[(fp * NF + mm) * NS + s] * (g.n[f][0] * fw[s] + g.n[f][1] * fw[NS + s] + g.n[f][2] * fw[2 * NS + s]);
    double nu[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) nu[a] = g.ij[a][0] * g.n[f][0] + g.ij[a][1] * g.n[f][1] + g.ij[a][2] * g.n[f][2];
    double wp = 0.0;  // -(W^T p) / |F|
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      double v = tau * t.Ehat[(fp * NF + mm) * NP + j];
#pragma unroll
      for (int a = 0; a < 3; ++a) v += c * nu[a] * t.CD[((fp * 3 + a) * NF + mm) * NP + j];
      wp += v * p[j];
    }
    ycell[(long)r * nc + e] = g.a[f] * (cf / g.det + wp);
  }
}

// x = A^{-1}(f - B lam):  fw' = Fw + c Gl lam,  fpsi' = Fpsi - Tpl lam,
// p = P^{-1}(fpsi' - Gp^T fw' / det),  U = (fw' + c Gp p) / det
template <int K>
__global__ void __launch_bounds__(kW3) k3_backsub(DMesh m, DTab3 t, double c, double tau,
                                                  const double* __restrict__ Pinv, const double* __restrict__ Fw,
                                                  const double* __restrict__ Fpsi, const double* __restrict__ lam,
                                                  double* __restrict__ U, double* __restrict__ P,
                                                  double* __restrict__ cellint) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU, NL = D::NL;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double fw[NU], fpsi[NP], b[NP], p[NP], l[NL];
  __shared__ int fps[4];
  if (lane < 4) fps[lane] = 6 * lane + m.cf_flip[lane * nc + e];
  for (int r = lane; r < NL; r += kW3) {
    const int f = r / NF, mm = r % NF;
    l[r] = lam[(long)m.cf_facet[f * nc + e] * NF + mm];
  }
  __syncthreads();
  for (int i = lane; i < NU; i += kW3) {
    const int cc = i / NS, s = i % NS;
    double v = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double a = 0.0;
#pragma unroll
      for (int mm = 0; mm < NF; ++mm) a += t.Chat[(fps[f] * NF + mm) * NS + s] * l[f * NF + mm];
      v += g.a[f] * g.n[f][cc] * a;
    }
    fw[i] = (Fw ? Fw[(long)e * NU + i] : 0.0) - c * v;
  }
  for (int i = lane; i < NP; i += kW3) {
    double v = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double a = 0.0;
#pragma unroll
      for (int mm = 0; mm < NF; ++mm) a += t.Ehat[(fps[f] * NF + mm) * NP + i] * l[f * NF + mm];
      v += g.a[f] * a;
    }
    fpsi[i] = (Fpsi ? Fpsi[(long)e * NP + i] : 0.0) + tau * v;
  }
  __syncthreads();
  pressure_solve3<K>(t, g, Pinv, nc, e, fw, fpsi, b, p);
  const double idet = 1.0 / g.det;
  for (int i = lane; i < NU; i += kW3) {
    const int cc = i / NS, s = i % NS;
    double v = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) d += t.D[(a * NP + j) * NS + s] * p[j];
      v += g.ij[a][cc] * d;
    }
    U[(long)e * NU + i] = fw[i] * idet + c * v;
  }
  for (int i = lane; i < NP; i += kW3) P[(long)e * NP + i] = p[i];
  // int_K p = det p_0 int phi_0, phi_0 = sqrt(6) on the reference cell of volume 1/6
  if (lane == 0 && cellint) cellint[e] = g.det * p[0] * 0.40824829046386301637;
}

// partial sums of the per-cell pressure integrals over kBlock cells
__global__ void __launch_bounds__(kBlock) k3_sum_cells(long nc, const double* __restrict__ v, double* __restrict__ part) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double s = block_sum(e < nc ? v[e] : 0.0);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// shift (p, lam) by -mean: p_0 -= mean / sqrt(6), lam_0 -= mean (mu_0 = 1)
template <int K>
__global__ void k3_shift_mean(DMesh m, const double* __restrict__ mean, double* __restrict__ p,
                              double* __restrict__ lam) {
  constexpr int NP = Dims3<K>::NP, NF = Dims3<K>::NF;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const double mv = mean[0];
  if (tid < m.nc) p[tid * NP] -= mv * 0.40824829046386301637;
  if (tid < m.nF && lam) lam[tid * NF] -= mv;
}

// Gamma(psi, mu, Q, P, lam) times scale: psi part per cell
//   Gp^T Q + Tpp P + Tpl lam,
// mu part per (cell, local facet) into ycell:
//   |F| (Chat n.Q + tau Ehat P - tau lam)
template <int K>
__global__ void __launch_bounds__(kW3) k3_gamma(DMesh m, DTab3 t, double tau, double scale,
                                                const double* __restrict__ Q, const double* __restrict__ Pv,
                                                const double* __restrict__ lam, double* __restrict__ gpsi,
                                                double* __restrict__ ycell) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU, NL = D::NL;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double q[NU], p[NP], l[NL];
  __shared__ int fps[4];
  if (lane < 4) fps[lane] = 6 * lane + m.cf_flip[lane * nc + e];
  stage_vel<K>(Q, e, q);
  for (int i = lane; i < NP; i += kW3) p[i] = Pv ? Pv[(long)e * NP + i] : 0.0;
  for (int r = lane; r < NL; r += kW3) {
    const int f = r / NF, mm = r % NF;
    l[r] = lam ? lam[(long)m.cf_facet[f * nc + e] * NF + mm] : 0.0;
  }
  __syncthreads();
  for (int i = lane; i < NP; i += kW3) {
    double v = 0.0;
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double u = g.ij[a][0] * q[s] + g.ij[a][1] * q[NS + s] + g.ij[a][2] * q[2 * NS + s];
        v += t.D[(a * NP + i) * NS + s] * u;
      }
    }
    double tp = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double a = 0.0;
#pragma unroll
      for (int j = 0; j < NP; ++j) a += t.That[(f * NP + i) * NP + j] * p[j];
#pragma unroll
      for (int mm = 0; mm < NF; ++mm) a -= t.Ehat[(fps[f] * NF + mm) * NP + i] * l[f * NF + mm];
      tp += g.a[f] * a;
    }
    gpsi[(long)e * NP + i] = scale * (g.det * v + tau * tp);
  }
  for (int r = lane; r < NL; r += kW3) {
    const int f = r / NF, mm = r % NF;
    const int fp = fps[f];
    double cq = 0.0;
    for (int s = 0; s < NS; ++s)
      cq += t.Chat[(fp * NF + mm) * NS + s] * (g.n[f][0] * q[s] + g.n[f][1] * q[NS + s] + g.n[f][2] * q[2 * NS + s]);
    double ep = 0.0;
#pragma unroll
    for (int j = 0; j < NP; ++j) ep += t.Ehat[(fp * NF + mm) * NP + j] * p[j];
    ycell[(long)r * nc + e] = scale * g.a[f] * (cq + tau * ep - tau * l[r]);
  }
}

template <int K>
__global__ void k3_mass(DMesh m, double s, const double* __restrict__ x, double* __restrict__ y) {
  constexpr int NU = Dims3<K>::NU;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)m.nc * NU) return;
  y[i] = s * m.geo[(long)E3_DET * m.nc + i / NU] * x[i];
}

// ================================================================ a4, a5
// Per-stage Step I data of the advecting velocity Q* (cell-major):
//   V[e][j][i] = -sum_q det w_q phi_i (Q*.grad phi_j)   (the volume term of
//   f_im, the same for every velocity component; stored with the test index
//   i fastest, so that the lanes of the operator read it coalesced), and
//   beta[e][f][q] = |F| 2 w_q (qn/2 - delta |qn|),  qn = {Q*}.n_K at the
//   facet point (0 on walls, where f_im has the penalty term only).
template <int K, typename TO>
__global__ void __launch_bounds__(kW3) k3_prep(DMesh m, DTab3 t, const double* __restrict__ Qs, double delta_up,
                                               TO* __restrict__ V, TO* __restrict__ beta) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC, NQF = D::NQF;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double q[NU], qn[NU], a[3][NQC];  // a: Q* in reference directions at the cell points
  __shared__ double Mq[NQC][NS];                // (a . grad_ref) phi_j at the cell points
  stage_vel<K>(Qs, e, q);
  __syncthreads();
  for (int iq = lane; iq < NQC; iq += kW3) {
    double u[3] = {0.0, 0.0, 0.0};
    for (int s = 0; s < NS; ++s) {
      const double b = t.Bu[iq * NS + s];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) u[cc] += b * q[cc * NS + s];
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) a[r][iq] = g.det * t.cw[iq] * (g.ij[r][0] * u[0] + g.ij[r][1] * u[1] + g.ij[r][2] * u[2]);
  }
  __syncthreads();
  for (int idx = lane; idx < NQC * NS; idx += kW3) {
    const int iq = idx / NS, j = idx % NS;
    Mq[iq][j] = a[0][iq] * t.dBu[(0 * NQC + iq) * NS + j] + a[1][iq] * t.dBu[(1 * NQC + iq) * NS + j] +
                a[2][iq] * t.dBu[(2 * NQC + iq) * NS + j];
  }
  __syncthreads();
  // V = Bu^T Mq (NS x NS, contracted over the NQC cell points) on the FP64
  // matrix cores: tiles of 16 x 16 zero-padded, steps of 4 points; lane l
  // supplies A[l % 16][l / 16], B[l / 16][l % 16] and holds D[4 v + l / 16][l % 16]
  {
    constexpr int NST = (NS + 15) / 16, NKQ = (NQC + 3) / 4;
    const int lr = lane >> 4, lc = lane & 15;
#pragma unroll
    for (int ti = 0; ti < NST; ++ti)
#pragma unroll
      for (int tj = 0; tj < NST; ++tj) {
        f64x4_3 acc = {0.0, 0.0, 0.0, 0.0};
        const int ia = 16 * ti + lc, jb = 16 * tj + lc;
#pragma unroll 4
        for (int kk = 0; kk < NKQ; ++kk) {
          const int kq = 4 * kk + lr;
          const double av = (kq < NQC && ia < NS) ? t.Bu[kq * NS + ia] : 0.0;
          const double bv = (kq < NQC && jb < NS) ? Mq[kq][jb] : 0.0;
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * ti + 4 * v + lr, j = 16 * tj + lc;
          if (i < NS && j < NS) V[((long)e * NS + j) * NS + i] = (TO)(-acc[v]);  // stored transposed: V[e][j][i]
        }
      }
  }
  for (int f = 0; f < 4; ++f) {
    const int en = m.cf_nb[f * nc + e];
    __syncthreads();
    if (en >= 0) {
      for (int i = lane; i < NU; i += kW3) qn[i] = Qs[(long)en * NU + i];
    }
    __syncthreads();
    const int fp = 6 * f + m.cf_flip[f * nc + e];
    const int fpn = en >= 0 ? 6 * m.cf_nbf[f * nc + e] + m.cf_flip[m.cf_nbf[f * nc + e] * nc + en] : 0;
    for (int iq = lane; iq < NQF; iq += kW3) {
      double w = 0.0;
      if (en >= 0) {
        double u = 0.0;
        for (int s = 0; s < NS; ++s) {
          const double b0 = t.FBu[(fp * NQF + iq) * NS + s], b1 = t.FBu[(fpn * NQF + iq) * NS + s];
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) u += g.n[f][cc] * (b0 * q[cc * NS + s] + b1 * qn[cc * NS + s]);
        }
        const double qv = 0.5 * u;
        w = g.a[f] * 2.0 * t.fw[iq] * (0.5 * qv - delta_up * fabs(qv));
      }
      beta[((long)e * 4 + f) * NQF + iq] = (TO)w;
    }
  }
}

// Step I operator / residual on cell-major vectors, one wave per cell:
//   F = f_im(x) = V x (per component, V stored transposed) + sum over facets and facet points of
//       phi_i [beta (x_K - x_N) - alpha 2 w_q n (n.(x_K - x_N))]   (x_N = 0 on walls)
//   MODE 0: out = x - (adt/det) F
//   MODE 1: out = (r - det x + adt (F + g(p, lam))) / det
//   MODE 2: out = r - det x + adt (F + g(p, lam))
// DOT (MODE 0): partial inner products per block as the structure-of-arrays
// operator leaves them (dot 1: w.out; dot 2: out.x, out.out, w.x, w.out;
// dot 3: out.sd, out.out, w.sd, w.out), nparts blocks per set.  Blocks of
// WPB waves walk the cells with a stride of the grid.  TX: the type of V,
// beta, the vectors and the arithmetic (float in the mixed-precision mode,
// MODE 0 only); the inner products accumulate in FP64 either way.
// The facet-point tables of the 24 (local facet, orientation) point sets are
// copied into LDS once per workgroup: every cell reads about 200 of their
// rows, and from the 96 KB tables in L2 those reads bound the kernel (1.74 ms
// per launch at 32^3, k = 2, against 0.22 ms for its HBM bytes).  The table
// rows are padded by one entry against LDS bank conflicts; the table takes
// 100.8 KB at k = 2, which leaves room for the per-cell buffers of 12 waves.
template <int K>
struct Apply3Shape {
  static constexpr int WPB = 12;               // waves (cells in flight) per workgroup
  static constexpr int TS = Dims3<K>::NS + 1;  // padded table row
};
template <int K, int MODE, int DOT, typename TX = double>
__global__ void __launch_bounds__(Apply3Shape<K>::WPB * 64) k3_apply(DMesh m, DTab3 t, const TX* __restrict__ V,
                                                const TX* __restrict__ beta, double alpha, double adt,
                                                const TX* __restrict__ x, const double* __restrict__ r,
                                                const double* __restrict__ pv, const double* __restrict__ lam,
                                                TX* __restrict__ out, const TX* __restrict__ w,
                                                const TX* __restrict__ sd, double* __restrict__ part) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NF = D::NF, NU = D::NU, NQF = D::NQF;
  constexpr int WPB = Apply3Shape<K>::WPB, TS = Apply3Shape<K>::TS;
  static_assert(NU <= 64, "one lane per cell unknown");
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const long nc = m.nc;
  static_assert(MODE == 0 || sizeof(TX) == sizeof(double), "the residual modes are FP64");
  __shared__ double tab[24][NQF][TS];
  __shared__ TX xs[WPB][5][NU];
  __shared__ TX phi[WPB][4][NQF][3];
  __shared__ double red[WPB][4];
  for (int i = threadIdx.x; i < 24 * NQF * NS; i += WPB * 64) tab[i / (NQF * NS)][(i / NS) % NQF][i % NS] = t.FBu[i];
  double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
  const long stride = (long)gridDim.x * WPB;
  // every wave of a block runs the same number of rounds (the barriers)
  for (long base = (long)blockIdx.x * WPB; base < nc; base += stride) {
    // the cell index is the same on every lane of the wave: keep it (and all
    // per-cell scalars loaded with it) in scalar registers
    const long e = (long)__builtin_amdgcn_readfirstlane((int)(base + wv));
    const bool act = e < nc;
    const long ec = act ? e : base;  // an inactive wave reads a valid cell and writes nothing
    TX(&X)[5][NU] = xs[wv];
    TX(&PH)[4][NQF][3] = phi[wv];
    int nb[4], fps[4], fpn[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      nb[f] = m.cf_nb[f * nc + ec];
      fps[f] = 6 * f + m.cf_flip[f * nc + ec];
      const int fn = m.cf_nbf[f * nc + ec];
      fpn[f] = nb[f] >= 0 ? 6 * fn + m.cf_flip[fn * nc + nb[f]] : 0;
    }
    {  // the cell's and its neighbours' unknowns, all five loads in flight together
      TX xv[5];
      xv[0] = lane < NU ? x[ec * NU + lane] : (TX)0;
#pragma unroll
      for (int f = 0; f < 4; ++f) xv[1 + f] = (lane < NU && nb[f] >= 0) ? x[(long)nb[f] * NU + lane] : (TX)0;
      if (lane < NU) {
#pragma unroll
        for (int v = 0; v < 5; ++v) X[v][lane] = xv[v];
      }
    }
    double nrm[4][3];
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) nrm[f][cc] = m.geo[(long)(E3_N + 3 * f + cc) * nc + ec];
    __syncthreads();
    for (int idx = lane; idx < 4 * NQF; idx += 64) {
      const int f = idx / NQF, iq = idx % NQF;
      TX du[3];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) du[cc] = (TX)0;
      const double* b0 = tab[fps[f]][iq];
#pragma unroll 4
      for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) du[cc] += (TX)b0[s] * X[0][cc * NS + s];
      }
      if (nb[f] >= 0) {
        const double* b1 = tab[fpn[f]][iq];
#pragma unroll 4
        for (int s = 0; s < NS; ++s) {
#pragma unroll
          for (int cc = 0; cc < 3; ++cc) du[cc] -= (TX)b1[s] * X[1 + f][cc * NS + s];
        }
      }
      const TX bq = beta[(ec * 4 + f) * NQF + iq];
      const TX pen = (TX)(alpha * 2.0 * t.fw[iq]);
      const TX dn = (TX)nrm[f][0] * du[0] + (TX)nrm[f][1] * du[1] + (TX)nrm[f][2] * du[2];
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) PH[f][iq][cc] = bq * du[cc] - pen * (TX)nrm[f][cc] * dn;
    }
    __syncthreads();
    const double det = m.geo[(long)E3_DET * nc + ec];
    for (int i = act ? lane : NU; i < NU; i += 64) {
      const int cc = i / NS, s = i % NS;
      TX F = (TX)0;
      const TX* vr = V + e * NS * NS + s;
#pragma unroll 4
      for (int j = 0; j < NS; ++j) F += vr[j * NS] * X[0][cc * NS + j];
#pragma unroll
      for (int f = 0; f < 4; ++f) {
#pragma unroll 5
        for (int iq = 0; iq < NQF; ++iq) F += (TX)tab[fps[f]][iq][s] * PH[f][iq][cc];
      }
      const long gi = e * NU + i;
      TX o;
      if constexpr (MODE == 0) {
        o = X[0][i] - (TX)(adt / det) * F;
        if constexpr (DOT == 1) {
          d0 += (double)w[gi] * (double)o;
        } else if constexpr (DOT == 2 || DOT == 3) {
          const double xr = DOT == 2 ? (double)X[0][i] : (double)sd[gi];
          const double od = (double)o, wd = (double)w[gi];
          d0 += od * xr;
          d1 += od * od;
          d2 += wd * xr;
          d3 += wd * od;
        }
      } else {
        // g(p, lam) = Gp p + Gl lam
        double gpl = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          double dd = 0.0;
#pragma unroll
          for (int j = 0; j < NP; ++j) dd += t.D[(a * NP + j) * NS + s] * pv[e * NP + j];
          gpl += det * m.geo[(long)(E3_IJ + 3 * a + cc) * nc + e] * dd;
        }
#pragma unroll
        for (int f = 0; f < 4; ++f) {
          const long Ff = m.cf_facet[f * nc + e];
          double a = 0.0;
#pragma unroll
          for (int mm = 0; mm < NF; ++mm) a += t.Chat[(fps[f] * NF + mm) * NS + s] * lam[Ff * NF + mm];
          gpl -= m.geo[(long)(E3_A + f) * nc + e] * nrm[f][cc] * a;
        }
        o = r[gi] - det * X[0][i] + adt * (F + gpl);
        if constexpr (MODE == 1) o /= det;
      }
      out[gi] = o;
    }
    __syncthreads();
  }
  if constexpr (MODE == 0 && DOT > 0) {
    d0 = wave_sum(d0);
    if constexpr (DOT >= 2) { d1 = wave_sum(d1); d2 = wave_sum(d2); d3 = wave_sum(d3); }
    if (lane == 0) { red[wv][0] = d0; red[wv][1] = d1; red[wv][2] = d2; red[wv][3] = d3; }
    __syncthreads();
    if (threadIdx.x == 0) {
      const int nb = gridDim.x, blk = blockIdx.x;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
#pragma unroll
      for (int i = 0; i < WPB; ++i) { s0 += red[i][0]; s1 += red[i][1]; s2 += red[i][2]; s3 += red[i][3]; }
      part[blk] = s0;
      if constexpr (DOT >= 2) { part[nb + blk] = s1; part[2 * nb + blk] = s2; part[3 * nb + blk] = s3; }
    }
  }
}

// Weak divergence Div(psi, F) times scale (central flux, walls excluded):
//   -det sum_a sum_c iJ[a][c] (R_a F_c)_i + sum_f |F_f| 2 sum_q w_q psi_i {F}.n_K
template <int K>
__global__ void __launch_bounds__(kW3) k3_div(DMesh m, DTab3 t, const double* __restrict__ Fv, double scale,
                                              double* __restrict__ out) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NU = D::NU, NQF = D::NQF;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double X[5][NU];
  __shared__ double fl[4][NQF];
  int nb[4], fps[4], fpn[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    nb[f] = m.cf_nb[f * nc + e];
    fps[f] = 6 * f + m.cf_flip[f * nc + e];
    const int fn = m.cf_nbf[f * nc + e];
    fpn[f] = nb[f] >= 0 ? 6 * fn + m.cf_flip[fn * nc + nb[f]] : 0;
  }
  for (int i = lane; i < NU; i += kW3) X[0][i] = Fv[(long)e * NU + i];
#pragma unroll
  for (int f = 0; f < 4; ++f)
    if (nb[f] >= 0)
      for (int i = lane; i < NU; i += kW3) X[1 + f][i] = Fv[(long)nb[f] * NU + i];
  __syncthreads();
  for (int idx = lane; idx < 4 * NQF; idx += kW3) {
    const int f = idx / NQF, iq = idx % NQF;
    double v = 0.0;
    if (nb[f] >= 0) {
      const double* b0 = t.FBu + (long)(fps[f] * NQF + iq) * NS;
      const double* b1 = t.FBu + (long)(fpn[f] * NQF + iq) * NS;
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) v += g.n[f][cc] * (b0[s] * X[0][cc * NS + s] + b1[s] * X[1 + f][cc * NS + s]);
      v *= 0.5 * g.a[f] * 2.0 * t.fw[iq];
    }
    fl[f][iq] = v;
  }
  __syncthreads();
  for (int i = lane; i < NP; i += kW3) {
    double vol = 0.0;
    for (int s = 0; s < NS; ++s) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double u = g.ij[a][0] * X[0][s] + g.ij[a][1] * X[0][NS + s] + g.ij[a][2] * X[0][2 * NS + s];
        vol += t.R[(a * NP + i) * NS + s] * u;
      }
    }
    double fac = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f)
      for (int iq = 0; iq < NQF; ++iq) fac += t.FBp[(fps[f] * NQF + iq) * NP + i] * fl[f][iq];
    out[(long)e * NP + i] = scale * (-g.det * vol + fac);
  }
}

// BDM interpolant by the contravariant Piola map: the reference moments of
// Qhat = det J^{-1} Q* are the physical ones (facet moments of {Q}.n against
// P_{k+1} of each facet, zero on walls; interior moments of Q against the
// first-kind Nedelec space, invariant under the covariant map), so
// Qhat* = BDMinv rhs and Q* = J Qhat* / det.
template <int K>
__global__ void __launch_bounds__(kW3) k3_bdm(DMesh m, DTab3 t, const double* __restrict__ Q, double* __restrict__ Qs) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NU = D::NU, NQF = D::NQF, NB = D::NB, NNED = D::NNED;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double X[5][NU];
  __shared__ double fl[4][NQF];
  __shared__ double rhs[NU], qh[NU];
  int nb[4], fps[4], fpn[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    nb[f] = m.cf_nb[f * nc + e];
    fps[f] = 6 * f + m.cf_flip[f * nc + e];
    const int fn = m.cf_nbf[f * nc + e];
    fpn[f] = nb[f] >= 0 ? 6 * fn + m.cf_flip[fn * nc + nb[f]] : 0;
  }
  for (int i = lane; i < NU; i += kW3) X[0][i] = Q[(long)e * NU + i];
#pragma unroll
  for (int f = 0; f < 4; ++f)
    if (nb[f] >= 0)
      for (int i = lane; i < NU; i += kW3) X[1 + f][i] = Q[(long)nb[f] * NU + i];
  __syncthreads();
  for (int idx = lane; idx < 4 * NQF; idx += kW3) {
    const int f = idx / NQF, iq = idx % NQF;
    double v = 0.0;
    if (nb[f] >= 0) {
      const double* b0 = t.FBu + (long)(fps[f] * NQF + iq) * NS;
      const double* b1 = t.FBu + (long)(fpn[f] * NQF + iq) * NS;
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) v += g.n[f][cc] * (b0[s] * X[0][cc * NS + s] + b1[s] * X[1 + f][cc * NS + s]);
      v *= 0.5 * g.a[f] * 2.0 * t.fw[iq];
    }
    fl[f][iq] = v;
  }
  __syncthreads();
  for (int r = lane; r < NU; r += kW3) {
    double v = 0.0;
    if (r < 4 * NB) {
      const int f = r / NB, mm = r % NB;
      for (int iq = 0; iq < NQF; ++iq) v += t.NUL[(fps[f] * NQF + iq) * NB + mm] * fl[f][iq];
    } else {
      const int l = r - 4 * NB;
      // (Q, J^{-T} vhat)_K = det sum_b sum_c iJ[b][c] (NEDM_b Q_c)
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
          const double u = g.ij[b][0] * X[0][s] + g.ij[b][1] * X[0][NS + s] + g.ij[b][2] * X[0][2 * NS + s];
          v += t.NEDM[(l * 3 + b) * NS + s] * u;
        }
      v *= g.det;
    }
    rhs[r] = v;
  }
  __syncthreads();
  (void)NNED;
  for (int i = lane; i < NU; i += kW3) {
    double v = 0.0;
    for (int j = 0; j < NU; ++j) v += t.BDMinv[(long)j * NU + i] * rhs[j];  // column-major: coalesced
    qh[i] = v;
  }
  __syncthreads();
  double J[3][3];
  load_j3(m, e, J);
  for (int i = lane; i < NU; i += kW3) {
    const int cc = i / NS, s = i % NS;
    Qs[(long)e * NU + i] = (J[cc][0] * qh[s] + J[cc][1] * qh[NS + s] + J[cc][2] * qh[2 * NS + s]) / g.det;
  }
}

// f_p data of the pressure reconstruction: Div(psi, (Q.grad)Q) with the
// broken gradient at the cell points and at both sides' facet points.
template <int K>
__global__ void __launch_bounds__(kW3) k3_recon_rhs(DMesh m, DTab3 t, const double* __restrict__ Q,
                                                    double* __restrict__ out) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NP = D::NP, NU = D::NU, NQC = D::NQC, NQF = D::NQF;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double X[5][NU];
  __shared__ double fl[4][NQF];
  __shared__ double cv[3][NQC];  // det w_q (Q.grad)Q at the cell points
  int nb[4], fps[4], fpn[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    nb[f] = m.cf_nb[f * nc + e];
    fps[f] = 6 * f + m.cf_flip[f * nc + e];
    const int fn = m.cf_nbf[f * nc + e];
    fpn[f] = nb[f] >= 0 ? 6 * fn + m.cf_flip[fn * nc + nb[f]] : 0;
  }
  for (int i = lane; i < NU; i += kW3) X[0][i] = Q[(long)e * NU + i];
#pragma unroll
  for (int f = 0; f < 4; ++f)
    if (nb[f] >= 0)
      for (int i = lane; i < NU; i += kW3) X[1 + f][i] = Q[(long)nb[f] * NU + i];
  __syncthreads();
  // (Q.grad)Q of cell `which` at a point with basis values b and reference gradients db[a]
  auto conv = [&](const double* Xc, const double* b, const double* db0, const double* db1, const double* db2,
                  long dstride, const double (&ij)[3][3], double (&o)[3]) {
    double u[3] = {0.0, 0.0, 0.0}, gr[3][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    for (int s = 0; s < NS; ++s) {
      const double d[3] = {db0[s * dstride], db1[s * dstride], db2[s * dstride]};
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const double qv = Xc[cc * NS + s];
        u[cc] += b[s * dstride] * qv;
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[cc][a] += d[a] * qv;  // d/d xi_a
      }
    }
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) {
      double v = 0.0;
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        const double dxq = gr[cc][0] * ij[0][x] + gr[cc][1] * ij[1][x] + gr[cc][2] * ij[2][x];
        v += u[x] * dxq;
      }
      o[cc] = v;
    }
  };
  for (int iq = lane; iq < NQC; iq += kW3) {
    double o[3];
    conv(X[0], t.Bu + (long)iq * NS, t.dBu + (long)iq * NS, t.dBu + (long)(NQC + iq) * NS,
         t.dBu + (long)(2 * NQC + iq) * NS, 1, g.ij, o);
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) cv[cc][iq] = g.det * t.cw[iq] * o[cc];
  }
  for (int idx = lane; idx < 4 * NQF; idx += kW3) {
    const int f = idx / NQF, iq = idx % NQF;
    double v = 0.0;
    if (nb[f] >= 0) {
      double o0[3], o1[3], ijn[3][3];
      conv(X[0], t.FBu + (long)(fps[f] * NQF + iq) * NS, t.FdBu + (long)((fps[f] * 3 + 0) * NQF + iq) * NS,
           t.FdBu + (long)((fps[f] * 3 + 1) * NQF + iq) * NS, t.FdBu + (long)((fps[f] * 3 + 2) * NQF + iq) * NS, 1,
           g.ij, o0);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) ijn[a][b] = m.geo[(long)(E3_IJ + 3 * a + b) * nc + nb[f]];
      conv(X[1 + f], t.FBu + (long)(fpn[f] * NQF + iq) * NS, t.FdBu + (long)((fpn[f] * 3 + 0) * NQF + iq) * NS,
           t.FdBu + (long)((fpn[f] * 3 + 1) * NQF + iq) * NS, t.FdBu + (long)((fpn[f] * 3 + 2) * NQF + iq) * NS, 1,
           ijn, o1);
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) v += g.n[f][cc] * 0.5 * (o0[cc] + o1[cc]);
      v *= g.a[f] * 2.0 * t.fw[iq];
    }
    fl[f][iq] = v;
  }
  __syncthreads();
  for (int i = lane; i < NP; i += kW3) {
    double vol = 0.0;
    for (int iq = 0; iq < NQC; ++iq) {
      double gp = 0.0;
#pragma unroll
      for (int x = 0; x < 3; ++x) {
        const double dpx = t.dBp[(0 * NQC + iq) * NP + i] * g.ij[0][x] + t.dBp[(1 * NQC + iq) * NP + i] * g.ij[1][x] +
                           t.dBp[(2 * NQC + iq) * NP + i] * g.ij[2][x];
        gp += dpx * cv[x][iq];
      }
      vol += gp;
    }
    double fac = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f)
      for (int iq = 0; iq < NQF; ++iq) fac += t.FBp[(fps[f] * NQF + iq) * NP + i] * fl[f][iq];
    out[(long)e * NP + i] = -vol + fac;
  }
}

// velocity coefficients from values at the cell points [nc][NQC][3]:
// coef[c][s] = sum_q w_q phi_s(q) v_c(q) (orthonormal reference basis)
template <int K>
__global__ void __launch_bounds__(kW3) k3_project(DMesh m, DTab3 t, const double* __restrict__ vals,
                                                  double* __restrict__ Q) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NU = D::NU, NQC = D::NQC;
  const int e = blockIdx.x, lane = threadIdx.x;
  for (int i = lane; i < NU; i += kW3) {
    const int cc = i / NS, s = i % NS;
    double v = 0.0;
    for (int iq = 0; iq < NQC; ++iq) v += t.cw[iq] * t.Bu[iq * NS + s] * vals[((long)e * NQC + iq) * 3 + cc];
    Q[(long)e * NU + i] = v;
  }
}

// ================================================= Step I preconditioner
// Additive Schwarz over facet patches, as on triangles: per interior facet F
// with cells K+ and K-, A_F is the restriction of the mass-scaled Step I
// operator to the 2 NU unknowns of the two cells, and z = B r sums, for each
// cell, its rows of A_F^{-1} applied to (r_K, r_neighbour) over the cell's
// interior facets.  The patches contain the fields whose normal component
// is continuous across F, on which the penalty term of eq. (f_impl)
// vanishes, so the iteration count does not grow with that term's weight.
// Storage: per (cell, local facet), NU rows of 2 NU FP16 entries (own
// columns first), as quads of 4 in tiles of 32 cells (cell fastest).
using pc3_t = _Float16;
typedef _Float16 f16x4_3 __attribute__((ext_vector_type(4)));
template <int K>
struct PcLayout3 {
  static constexpr int NU = Dims3<K>::NU, NQ = 2 * NU / 4;
  __device__ static long quad(long e, int f, int i, int jq) {
    return ((((e >> 5) * 4 + f) * (long)NU + i) * NQ + jq) * 32 + (e & 31);
  }
};
__device__ __forceinline__ pc3_t pc3_store(double v) {
  const double lim = 65504.0;  // largest finite FP16
  return (pc3_t)(v > lim ? lim : (v < -lim ? -lim : v));
}

// Own-cell block D_K = I - (adt/det) (volume term + own-side facet terms of
// the four facets), FP64 [cell][row][col], rows and columns (c, s).  One
// wave per cell; from the per-stage V (transposed) and beta of k3_prep:
//   D[(c,s)][(c',s')] = delta - (adt/det) (delta_cc' (V_ss' + Mb_ss')
//                        - alpha sum_f n_fc n_fc' Mp_f,ss'),
//   Mb = sum_f sum_q beta_fq phi_s phi_s',  Mp_f = sum_q 2 w_q phi_s phi_s'.
template <int K>
__global__ void __launch_bounds__(kW3) k3_pc_cellblock(DMesh m, DTab3 t, const double* __restrict__ V,
                                                       const double* __restrict__ beta, double alpha, double adt,
                                                       double* __restrict__ Dout) {
  using D = Dims3<K>;
  constexpr int NS = D::NS, NU = D::NU, NQF = D::NQF;
  const int e = blockIdx.x, lane = threadIdx.x;
  const long nc = m.nc;
  const Geo3 g = load_geo3(m, e);
  __shared__ double mb[NS * NS], mp[4][NS * NS];
  int fps[4];
#pragma unroll
  for (int f = 0; f < 4; ++f) fps[f] = 6 * f + m.cf_flip[f * nc + e];
  for (int idx = lane; idx < NS * NS; idx += kW3) {
    const int s = idx / NS, s2 = idx % NS;
    double b = 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      double pm = 0.0;
      const double* tb = t.FBu + (long)fps[f] * NQF * NS;
      for (int q = 0; q < NQF; ++q) {
        const double pp = tb[q * NS + s] * tb[q * NS + s2];
        b += beta[((long)e * 4 + f) * NQF + q] * pp;
        pm += 2.0 * t.fw[q] * pp;
      }
      mp[f][idx] = pm;
    }
    mb[idx] = b + V[((long)e * NS + s2) * NS + s];  // V stored [trial][test]
  }
  __syncthreads();
  const double sc = adt / g.det;
  for (int idx = lane; idx < NU * NU; idx += kW3) {
    const int i = idx / NU, j = idx % NU;
    const int c = i / NS, s = i % NS, c2 = j / NS, s2 = j % NS;
    double v = c == c2 ? mb[s * NS + s2] : 0.0;
#pragma unroll
    for (int f = 0; f < 4; ++f) v -= alpha * g.n[f][c] * g.n[f][c2] * mp[f][s * NS + s2];
    Dout[(long)e * NU * NU + idx] = (i == j ? 1.0 : 0.0) - sc * v;
  }
}

// Patch inversion on the FP64 matrix cores.  v_mfma_f64_16x16x4f64 forms
// D = A B + C for a 16 x 4 A, a 4 x 16 B and a 16 x 16 C: lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16] and holds D[4 v + l / 16][l % 16]
// in its four accumulator doubles v (rows interleaved over the four lane
// groups; measured on gfx950).  The patch block (N = 2 NU, padded with
// the identity to NT tiles of 16) stays in registers as accumulator tiles,
// wave w holding tile row w.
template <int K>
struct PcPatchShape3 {
  static constexpr int NU = Dims3<K>::NU, N = 2 * NU;
  static constexpr int NT = (N + 15) / 16;  // tiles per row and column, and waves per workgroup
  static constexpr int NB = N / 4;          // pivot blocks of four
  static_assert(NB * 4 == N, "four-row pivot blocks");
  static constexpr int NTH = NT * 64;
};

// One workgroup per facet: A_F assembled from the two cell blocks and the
// coupling through F,
//   C[(c,s) of row cell][(c',s') of column cell] =
//     (adt/det_row) sum_q phi_s phi'_s' (beta_row,q delta_cc' - alpha 2 w_q n_c n_c'),
// (both cells see the facet's points in the facet's own order), inverted by
// block Gauss-Jordan elimination without pivoting (the symmetric part of A_F
// is positive definite, as on triangles) on pivot blocks P of four rows:
// with E = A[:, P] - I[:, P] (so E_P = A_PP - I), R = A_PP^{-1} A[P, :] except
// R[:, P] = A_PP^{-1}, and A[:, P] replaced by I[:, P], one step is the
// rank-4 update A <- A - E R, which leaves the in-place inverse's rows P and
// columns P where Gauss-Jordan puts them.  Each step is one matrix-core
// product per tile; the wave holding rows P inverts the 4 x 4 block and
// writes R to LDS (double-buffered: one barrier per step).  Each cell's rows
// of the inverse are stored in FP16 (own columns first).  Wall facets return
// at once.
template <int K>
__global__ void __launch_bounds__(PcPatchShape3<K>::NTH) __attribute__((amdgpu_waves_per_eu(4)))
k3_pc_patch(DMesh m, DTab3 t,
                                                                     const double* __restrict__ beta, double alpha,
                                                                     double adt, const double* __restrict__ Dc,
                                                                     pc3_t* __restrict__ Binv) {
  using Dm = Dims3<K>;
  using Sh = PcPatchShape3<K>;
  constexpr int NS = Dm::NS, NU = Dm::NU, NQF = Dm::NQF, N = Sh::N, NT = Sh::NT, NTH = Sh::NTH;
  const int F = blockIdx.x;
  const long nc = m.nc;
  const int Km = m.fc_cell[m.nF + F];
  if (Km < 0) return;  // wall facet (uniform over the workgroup)
  const int Kp = m.fc_cell[F];
  const int fp = m.fc_f[F], fm = m.fc_f[m.nF + F];
  auto cell = [&](int side) { return side ? Km : Kp; };
  auto lf = [&](int side) { return side ? fm : fp; };
  const int tp = 6 * fp + m.cf_flip[fp * nc + Kp], tm = 6 * fm + m.cf_flip[fm * nc + Km];
  auto tab = [&](int side) { return side ? tm : tp; };
  // the facet's data of both sides, then the three NS x NS facet matrices
  //   Mb_side[s][s'] = sum_q beta_side,q phi^side_s phi^other_s',
  //   Mw[s][s'] = sum_q 2 w_q phi^+_s phi^-_s'
  // (every quantity the coupling blocks need, computed once per patch)
  __shared__ double tb[2][NQF][NS], bq[2][NQF], w2[NQF];
  __shared__ double Mb[2][NS][NS], Mw[NS][NS];
  __shared__ double sR[2][4][NT * 16];
  for (int idx = threadIdx.x; idx < 2 * NQF * NS; idx += NTH) {
    const int side = idx / (NQF * NS), rem = idx % (NQF * NS);
    tb[side][rem / NS][rem % NS] = t.FBu[(long)tab(side) * NQF * NS + rem];
  }
  for (int idx = threadIdx.x; idx < 2 * NQF; idx += NTH) {
    const int side = idx / NQF, q = idx % NQF;
    bq[side][q] = beta[((long)cell(side) * 4 + lf(side)) * NQF + q];
  }
  for (int q = threadIdx.x; q < NQF; q += NTH) w2[q] = 2.0 * t.fw[q];
  __syncthreads();
  for (int idx = threadIdx.x; idx < 3 * NS * NS; idx += NTH) {
    const int which = idx / (NS * NS), s = (idx / NS) % NS, s2 = idx % NS;
    double v = 0.0;
    if (which < 2) {
      for (int q = 0; q < NQF; ++q) v += bq[which][q] * tb[which][q][s] * tb[1 - which][q][s2];
      Mb[which][s][s2] = v;
    } else {
      for (int q = 0; q < NQF; ++q) v += w2[q] * tb[0][q][s] * tb[1][q][s2];
      Mw[s][s2] = v;
    }
  }
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l >> 4, lc = l & 15;  // accumulator rows 16 w + 4 v + lr, columns 16 J + lc
  // the row cell's facet normal and adt / det, both sides, loaded once
  double nrm[2][3], sc[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
#pragma unroll
    for (int c3 = 0; c3 < 3; ++c3) nrm[side][c3] = m.geo[(long)(E3_N + 3 * lf(side) + c3) * nc + cell(side)];
    sc[side] = adt / m.geo[(long)E3_DET * nc + cell(side)];
  }
  f64x4_3 acc[NT];
#pragma unroll
  for (int J = 0; J < NT; ++J)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + 4 * v + lr, col = 16 * J + lc;
      double x;
      if (row >= N || col >= N) {
        x = row == col ? 1.0 : 0.0;
      } else {
        const int rs = row / NU, cs = col / NU, rr = row % NU, jj = col % NU;
        if (rs == cs) {
          x = Dc[((long)cell(rs) * NU + rr) * NU + jj];
        } else {  // coupling block: row cell rs, column cell 1 - rs
          const int cr = rr / NS, sr = rr % NS, cj = jj / NS, s2 = jj % NS;
          // selects, not indexing: a per-lane index into a register array would go to scratch
          const double n0 = rs ? nrm[1][0] : nrm[0][0], n1 = rs ? nrm[1][1] : nrm[0][1],
                       n2 = rs ? nrm[1][2] : nrm[0][2];
          const double nr = cr == 0 ? n0 : (cr == 1 ? n1 : n2), nj = cj == 0 ? n0 : (cj == 1 ? n1 : n2);
          const double mw = rs == 0 ? Mw[sr][s2] : Mw[s2][sr];
          x = (rs ? sc[1] : sc[0]) * ((cr == cj ? Mb[rs][sr][s2] : 0.0) - alpha * nr * nj * mw);
        }
      }
      acc[J][v] = x;
    }
#pragma unroll 1
  for (int p = 0; p < Sh::NB; ++p) {
    const int P0 = 4 * p, Tp = P0 >> 4, q0 = P0 & 15;  // rows and columns P0..P0+3: tile Tp, local q0..q0+3
    // this wave's tiles of the pivot columns (tile column Tp, a uniform choice)
    f64x4_3 ct = acc[0];
#pragma unroll
    for (int J = 1; J < NT; ++J) ct = J == Tp ? acc[J] : ct;
    // A operand: E[16 w + lc][lr] = A[16 w + lc][P0 + lr] - delta, held by
    // lane 16 (lc % 4) + q0 + lr of this wave in accumulator v = lc / 4
    double e;
    {
      const int src = 16 * (lc & 3) + q0 + lr;
      const double e0 = __shfl(ct[0], src), e1 = __shfl(ct[1], src), e2 = __shfl(ct[2], src),
                   e3 = __shfl(ct[3], src);
      const int v = lc >> 2;
      e = v == 0 ? e0 : (v == 1 ? e1 : (v == 2 ? e2 : e3));
      if (w == Tp && lc == q0 + lr) e -= 1.0;
    }
    double* R = &sR[p & 1][0][0];
    if (w == Tp) {  // the wave holding rows P: the 4 x 4 pivot block, its inverse, then R
      // row P0 + i of column 16 J + c sits in lane 16 i + c, accumulator g0
      const int g0 = q0 >> 2;
      const double cg = g0 == 0 ? ct[0] : (g0 == 1 ? ct[1] : (g0 == 2 ? ct[2] : ct[3]));
      double d[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) d[i][j] = __shfl(cg, 16 * i + q0 + j);
#pragma unroll
      for (int q = 0; q < 4; ++q) {  // in-place Gauss-Jordan of the 4 x 4 block
        const double r = 1.0 / d[q][q];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[q][j] = j == q ? r : d[q][j] * r;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          if (i == q) continue;
          const double a = d[i][q];
#pragma unroll
          for (int j = 0; j < 4; ++j) d[i][j] = j == q ? -a * r : d[i][j] - a * d[q][j];
        }
      }
      // lane (lr, lc) forms R[lr][16 J + lc] from the four pivot rows of its column
      const double di0 = lr == 0 ? d[0][0] : (lr == 1 ? d[1][0] : (lr == 2 ? d[2][0] : d[3][0]));
      const double di1 = lr == 0 ? d[0][1] : (lr == 1 ? d[1][1] : (lr == 2 ? d[2][1] : d[3][1]));
      const double di2 = lr == 0 ? d[0][2] : (lr == 1 ? d[1][2] : (lr == 2 ? d[2][2] : d[3][2]));
      const double di3 = lr == 0 ? d[0][3] : (lr == 1 ? d[1][3] : (lr == 2 ? d[2][3] : d[3][3]));
#pragma unroll
      for (int J = 0; J < NT; ++J) {
        const double aJ = g0 == 0 ? acc[J][0] : (g0 == 1 ? acc[J][1] : (g0 == 2 ? acc[J][2] : acc[J][3]));
        double v = di0 * __shfl(aJ, lc) + di1 * __shfl(aJ, 16 + lc) + di2 * __shfl(aJ, 32 + lc) +
                   di3 * __shfl(aJ, 48 + lc);
        if (J == Tp && lc >= q0 && lc < q0 + 4) {
          const int jp = lc - q0;
          v = jp == 0 ? di0 : (jp == 1 ? di1 : (jp == 2 ? di2 : di3));
        }
        R[lr * NT * 16 + 16 * J + lc] = v;
      }
    }
    // columns P become I[:, P]
#pragma unroll
    for (int J = 0; J < NT; ++J) {
      if (J == Tp && lc >= q0 && lc < q0 + 4) {
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[J][v] = (w == Tp && 4 * v + lr == lc) ? 1.0 : 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int J = 0; J < NT; ++J)
      acc[J] = __builtin_amdgcn_mfma_f64_16x16x4f64(-e, R[lr * NT * 16 + 16 * J + lc], acc[J], 0, 0, 0);
  }
  // rows of one side each: for K+ the column order is (own, neighbour); for
  // K- its own columns are those of side 1
#pragma unroll
  for (int J = 0; J < NT; ++J)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 16 * w + 4 * v + lr, col = 16 * J + lc;
      if (row < N && col < N) {
        const int side = row / NU;
        const int jb = side == 0 ? col : (col >= NU ? col - NU : col + NU);
        Binv[4 * PcLayout3<K>::quad(cell(side), lf(side), row % NU, jb >> 2) + (jb & 3)] = pc3_store(acc[J][v]);
      }
    }
}

// z = B r on cell-major vectors: thread (cell e, row group g) sums over the
// cell's interior facets its rows of A_F^{-1} applied to (r_e, r_neighbour).
template <int K>
struct PcApplyShape3 {
  static constexpr int NU = Dims3<K>::NU;
  static constexpr int G = K == 1 ? 3 : 6;  // row groups per cell
  static constexpr int RG = NU / G;
  static_assert(RG * G == NU, "rows split evenly");
};
template <int K, typename TX>
__global__ void __launch_bounds__(kBlock) k3_pc_apply(DMesh m, const pc3_t* __restrict__ Binv,
                                                      const TX* __restrict__ r, TX* __restrict__ z) {
  using Sh = PcApplyShape3<K>;
  constexpr int NU = Dims3<K>::NU, NQ = PcLayout3<K>::NQ, G = Sh::G, RG = Sh::RG;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long nc = m.nc;
  const long tile = tid / (G * 32);
  const int rem = (int)(tid % (G * 32));
  const int g = rem >> 5;
  const long e = tile * 32 + (rem & 31);
  if (e >= nc) return;
  double acc[RG];
#pragma unroll
  for (int a = 0; a < RG; ++a) acc[a] = 0.0;
  const f16x4_3* B4 = reinterpret_cast<const f16x4_3*>(Binv);
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    const long en = m.cf_nb[f * nc + e];
    if (en < 0) continue;
    const TX* ro = r + e * NU;
    const TX* rn = r + en * NU;
#pragma unroll 1
    for (int jq = 0; jq < NQ; ++jq) {
      // column 4 jq + u: own entries first, then the neighbour's (a quad may
      // straddle the two when NU is not a multiple of 4)
      double xv[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jx = 4 * jq + u;
        xv[u] = (double)*(jx < NU ? ro + jx : rn + (jx - NU));
      }
      const double x0 = xv[0], x1 = xv[1], x2 = xv[2], x3 = xv[3];
#pragma unroll
      for (int a = 0; a < RG; ++a) {
        const f16x4_3 b = __builtin_nontemporal_load(&B4[PcLayout3<K>::quad(e, f, g * RG + a, jq)]);
        acc[a] += (double)b.x * x0 + (double)b.y * x1 + (double)b.z * x2 + (double)b.w * x3;
      }
    }
  }
#pragma unroll
  for (int a = 0; a < RG; ++a) z[e * NU + g * RG + a] = (TX)acc[a];
}

long pc_entries3(int k, long nc) {
  const long nu = 3L * (k + 2) * (k + 3) * (k + 4) / 6;
  return (nc + 31) / 32 * 32 * 4 * nu * 2 * nu;
}

template <typename TI, typename TO>
__global__ void k3_convert(long n, const TI* __restrict__ in, TO* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = (TO)in[i];
}

// ============================================================== launchers
#define HDG3_DISPATCH(k, CALL)     \
  switch (k) {                     \
    case 1: { constexpr int KK = 1; CALL; } break; \
    case 2: { constexpr int KK = 2; CALL; } break; \
    default: break;                \
  }

void launch3_condense(int k, hipStream_t st, DMesh m, DTab3 t, double c, double tau, double* Pinv, double* SK) {
  HDG3_DISPATCH(k, (k3_condense<KK><<<m.nc, kW3, 0, st>>>(m, t, c, tau, Pinv, SK)));
}
void launch3_assemble(int k, hipStream_t st, DMesh m, const double* SK, double* vals, int* cols, double* Dinv) {
  HDG3_DISPATCH(k, (k3_assemble<KK><<<nblocks(m.nF), kBlock, 0, st>>>(m, SK, vals, cols, Dinv)));
}
void launch3_rhs_condense(int k, hipStream_t st, DMesh m, DTab3 t, double c, double tau, const double* Pinv,
                          const double* Fw, const double* Fpsi, double* ycell) {
  HDG3_DISPATCH(k, (k3_rhs_condense<KK><<<m.nc, kW3, 0, st>>>(m, t, c, tau, Pinv, Fw, Fpsi, ycell)));
}
void launch3_backsub(int k, hipStream_t st, DMesh m, DTab3 t, double c, double tau, const double* Pinv,
                     const double* Fw, const double* Fpsi, const double* lam, double* U, double* p, double* cellint,
                     double* part) {
  HDG3_DISPATCH(k, (k3_backsub<KK><<<m.nc, kW3, 0, st>>>(m, t, c, tau, Pinv, Fw, Fpsi, lam, U, p, cellint)));
  k3_sum_cells<<<nblocks(m.nc), kBlock, 0, st>>>(m.nc, cellint, part);
}
void launch3_shift_mean(int k, hipStream_t st, DMesh m, const double* mean, double* p, double* lam) {
  const long n = m.nc > m.nF ? m.nc : m.nF;
  HDG3_DISPATCH(k, (k3_shift_mean<KK><<<nblocks(n), kBlock, 0, st>>>(m, mean, p, lam)));
}
void launch3_gamma(int k, hipStream_t st, DMesh m, DTab3 t, double tau, double scale, const double* Q, const double* P,
                   const double* lam, double* gpsi, double* ycell) {
  HDG3_DISPATCH(k, (k3_gamma<KK><<<m.nc, kW3, 0, st>>>(m, t, tau, scale, Q, P, lam, gpsi, ycell)));
}
void launch3_mass(int k, hipStream_t st, DMesh m, double s, const double* x, double* y) {
  HDG3_DISPATCH(k, (k3_mass<KK><<<nblocks((long)m.nc * Dims3<KK>::NU), kBlock, 0, st>>>(m, s, x, y)));
}
void launch3_prep(int k, hipStream_t st, DMesh m, DTab3 t, const double* Qs, double delta_up, void* V, void* beta,
                  bool f32) {
  if (f32) HDG3_DISPATCH(k, (k3_prep<KK, float><<<m.nc, kW3, 0, st>>>(m, t, Qs, delta_up, (float*)V, (float*)beta)))
  else HDG3_DISPATCH(k, (k3_prep<KK, double><<<m.nc, kW3, 0, st>>>(m, t, Qs, delta_up, (double*)V, (double*)beta)));
}
int apply3_blocks(long nc) { return (int)((nc + 3) / 4 < 4096 ? (nc + 3) / 4 : 4096); }
void launch3_apply(int k, hipStream_t st, int mode, int dot, DMesh m, DTab3 t, const void* V, const void* beta,
                   double alpha, double adt, const void* x, const double* r, const double* p, const double* lam,
                   void* out, const void* w, const void* sd, double* part, int nparts, bool x32) {
  const int nb = nparts > 0 ? nparts : apply3_blocks(m.nc);
  using D = const double*;
  using F = const float*;
  if (x32) {
    if (mode != 0) throw std::invalid_argument("launch3_apply: the residual modes are FP64");
#define K3F(DT) HDG3_DISPATCH(k, (k3_apply<KK, 0, DT, float><<<nb, Apply3Shape<KK>::WPB * 64, 0, st>>>(m, t, (F)V, \
                                  (F)beta, alpha, adt, \
                                  (F)x, r, p, lam, (float*)out, (F)w, (F)sd, part)))
    switch (dot) { case 0: K3F(0); break; case 1: K3F(1); break; case 2: K3F(2); break; default: K3F(3); break; }
#undef K3F
    return;
  }
#define K3D(MD, DT) HDG3_DISPATCH(k, (k3_apply<KK, MD, DT, double><<<nb, Apply3Shape<KK>::WPB * 64, 0, st>>>(m, t, \
                                      (D)V, (D)beta, alpha, \
                                      adt, (D)x, r, p, lam, (double*)out, (D)w, (D)sd, part)))
  if (mode == 0) {
    switch (dot) { case 0: K3D(0, 0); break; case 1: K3D(0, 1); break; case 2: K3D(0, 2); break; default: K3D(0, 3); break; }
  } else if (mode == 1) {
    K3D(1, 0);
  } else {
    K3D(2, 0);
  }
#undef K3D
}
void launch3_convert(hipStream_t st, long n, const void* in, bool in32, void* out, bool out32) {
  if (in32 == out32) throw std::invalid_argument("launch3_convert: same types");
  if (in32) k3_convert<float, double><<<nblocks(n), kBlock, 0, st>>>(n, (const float*)in, (double*)out);
  else k3_convert<double, float><<<nblocks(n), kBlock, 0, st>>>(n, (const double*)in, (float*)out);
}
void launch3_div(int k, hipStream_t st, DMesh m, DTab3 t, const double* F, double scale, double* out) {
  HDG3_DISPATCH(k, (k3_div<KK><<<m.nc, kW3, 0, st>>>(m, t, F, scale, out)));
}
void launch3_bdm(int k, hipStream_t st, DMesh m, DTab3 t, const double* Q, double* Qs) {
  HDG3_DISPATCH(k, (k3_bdm<KK><<<m.nc, kW3, 0, st>>>(m, t, Q, Qs)));
}
void launch3_recon_rhs(int k, hipStream_t st, DMesh m, DTab3 t, const double* Q, double* out) {
  HDG3_DISPATCH(k, (k3_recon_rhs<KK><<<m.nc, kW3, 0, st>>>(m, t, Q, out)));
}
void launch3_pc_build(int k, hipStream_t st, DMesh m, DTab3 t, const double* V, const double* beta, double alpha,
                      double adt, double* D, void* Binv) {
  HDG3_DISPATCH(k, (k3_pc_cellblock<KK><<<m.nc, kW3, 0, st>>>(m, t, V, beta, alpha, adt, D)));
  HDG3_DISPATCH(k, (k3_pc_patch<KK><<<m.nF, PcPatchShape3<KK>::NTH, 0, st>>>(m, t, beta, alpha, adt, D,
                                                                             (pc3_t*)Binv)));
}
void launch3_pc_apply(int k, hipStream_t st, DMesh m, const void* Binv, const void* r, void* z, bool x32) {
  const long nc32 = (m.nc + 31) / 32 * 32;
  if (x32) HDG3_DISPATCH(k, (k3_pc_apply<KK, float><<<nblocks(nc32 * PcApplyShape3<KK>::G), kBlock, 0, st>>>(
                                m, (const pc3_t*)Binv, (const float*)r, (float*)z)))
  else HDG3_DISPATCH(k, (k3_pc_apply<KK, double><<<nblocks(nc32 * PcApplyShape3<KK>::G), kBlock, 0, st>>>(
                            m, (const pc3_t*)Binv, (const double*)r, (double*)z)));
}
void launch3_project(int k, hipStream_t st, DMesh m, DTab3 t, const double* vals, double* Q) {
  HDG3_DISPATCH(k, (k3_project<KK><<<m.nc, kW3, 0, st>>>(m, t, vals, Q)));
}

}  // namespace hdg
