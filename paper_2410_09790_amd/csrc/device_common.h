// Device-side helpers shared by the kernel sources of the HDG-IMEX library:
// degree-dependent sizes, per-cell geometry, block reductions and the
// launch-time dispatch over the degree k.
#pragma once

#include <hip/hip_runtime.h>

#include "kernels.h"

namespace hdg {

template <int K>
struct Dims {
  static constexpr int NS = (K + 2) * (K + 3) / 2;
  static constexpr int NP = (K + 1) * (K + 2) / 2;
  static constexpr int NF = K + 1;
  static constexpr int NU = 2 * NS;
  static constexpr int NLAM = 3 * NF;
  static constexpr int NQ1 = (3 * K + 4) / 2;
  static constexpr int NQC = NQ1 * NQ1;
  static constexpr int NQF = (3 * K + 5) / 2;
  static constexpr int NNED = K * (K + 2);
  static constexpr int NM = K + 2;
};

struct CellGeo {
  double det, ij[2][2], J[2][2], n[3][2], h[3];
};

__device__ __forceinline__ CellGeo load_geo(const DMesh& m, int e) {
  CellGeo g;
  const double* G = m.geo;
  const int nc = m.nc;
  g.det = G[D_DET * nc + e];
  g.ij[0][0] = G[D_IJ00 * nc + e]; g.ij[0][1] = G[D_IJ01 * nc + e];
  g.ij[1][0] = G[D_IJ10 * nc + e]; g.ij[1][1] = G[D_IJ11 * nc + e];
  g.J[0][0] = G[D_J00 * nc + e]; g.J[0][1] = G[D_J01 * nc + e];
  g.J[1][0] = G[D_J10 * nc + e]; g.J[1][1] = G[D_J11 * nc + e];
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    g.n[f][0] = G[(D_NX0 + 2 * f) * nc + e];
    g.n[f][1] = G[(D_NY0 + 2 * f) * nc + e];
    g.h[f] = G[(D_H0 + f) * nc + e];
  }
  return g;
}

__device__ __forceinline__ double sgn(int flip, int m) { return (flip && (m & 1)) ? -1.0 : 1.0; }

template <int BS>
__device__ __forceinline__ double block_sum_n(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  if constexpr (BS == 64) {
    return v;  // one wavefront: lane 0 holds the sum
  } else {
    __shared__ double s[BS / 64];
    int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) s[w] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int i = 0; i < BS / 64; ++i) r += s[i];
    }
    return r;
  }
}
__device__ __forceinline__ double block_sum(double v) { return block_sum_n<kBlock>(v); }

static inline int nblocks(long n) { return (int)((n + kBlock - 1) / kBlock); }


#define HDG_DISPATCH(k, CALL)       \
  switch (k) {                      \
    case 1: { constexpr int KK = 1; CALL; } break; \
    case 2: { constexpr int KK = 2; CALL; } break; \
    case 3: { constexpr int KK = 3; CALL; } break; \
    case 4: { constexpr int KK = 4; CALL; } break; \
    default: break;                 \
  }

}  // namespace hdg
