// Virial observation rows of L-hat K_NM, FP64.
//
// A configuration's virial stress is a sum of partial derivatives of its local
// energies (Sec. "Theory": targets are totals of local energies or of their
// derivatives; Sec. "Theory" eq. GP_L: sigma_virial regularises such rows).
// For a homogeneous strain eps acting on the pair displacement vectors
// r_p -> (I + eps) r_p, the derivative of the local energy of atom i is
// sum over its pairs of r_p,alpha dE_i/dr_j(p),beta, so row (c, alpha, beta),
// column m is
//   K_V[(c, alpha, beta), m] = - sum_{p in c} r[p][alpha] S[src(p)][m] (J[p][beta] . x_m)
// with S = delta^2 zeta (d_i . x_m)^(zeta-1) of the pair's source atom.
//
// Work decomposition: a block owns one configuration and 64 sparse-point
// columns; its four waves take the configuration's pairs 16 at a time (wave w
// the chunks w, w + 4, ...), contract the three Jacobian rows of each pair
// with the columns' x_m on the FP64 matrix core, and accumulate the nine
// weighted sums in registers.  One cross-lane and cross-wave reduction in a
// fixed order ends the block, so results do not depend on scheduling.
#include "launch.h"
#include "mma_f64.h"

namespace gapk {

namespace {

template <typename TJ>
__global__ __launch_bounds__(256) void k_virial_rows(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const double* __restrict__ X,
    int64_t ldx, int64_t M, const double* __restrict__ S, int64_t ldS,
    const int64_t* __restrict__ cfg_ptr, const int64_t* __restrict__ pair_ptr,
    const int32_t* __restrict__ pair_src, const double* __restrict__ pair_r, int64_t n_atoms,
    int64_t n_pairs, double* __restrict__ K, int64_t ldk) {
  __shared__ double red[4][9][64];
  const int64_t c = blockIdx.y;
  const int64_t colbase = (int64_t)blockIdx.x * 64;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t a0 = min(max(cfg_ptr[c], (int64_t)0), n_atoms);
  const int64_t a1 = min(max(cfg_ptr[c + 1], a0), n_atoms);
  const int64_t p_lo = min(max(pair_ptr[a0], (int64_t)0), n_pairs);
  const int64_t p_hi = min(max(pair_ptr[a1], p_lo), n_pairs);

  FragRowK<double> fb[4];
  int64_t colr[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    colr[u] = colbase + u * 16 + idx;
    fb[u] = FragRowK<double>{X + (colr[u] < M ? colr[u] : 0) * ldx, D, colr[u] < M};
  }
  double acc[9][4];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[q][u] = 0.0;

  for (int64_t p0 = p_lo + 16 * wave; p0 < p_hi; p0 += 64) {
    const int64_t p = p0 + idx;
    const bool pv = p < p_hi;
    const TJ* jr = jac + (pv ? p : 0) * 3 * ldj;
    const FragRowK<TJ> fa[3] = {FragRowK<TJ>{jr, D, pv}, FragRowK<TJ>{jr + ldj, D, pv},
                                FragRowK<TJ>{jr + 2 * ldj, D, pv}};
    d4v G[3][4];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int u = 0; u < 4; ++u) G[b][u] = zero4();
    for (int64_t k0 = 0; k0 < D; k0 += 16) {
      double a[3][4], bx[4][4];
#pragma unroll
      for (int b = 0; b < 3; ++b) fa[b].frag(k0, g, a[b]);
#pragma unroll
      for (int u = 0; u < 4; ++u) fb[u].frag(k0, g, bx[u]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int u = 0; u < 4; ++u) G[b][u] = mfma_f64(a[b][s], bx[u][s], G[b][u]);
    }
    // C layout: lane holds pairs p0 + g + 4 r of each tile's column idx
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t pr = p0 + g + 4 * r;
      if (pr >= p_hi) continue;
      const int32_t src = pair_src[pr];
      if (src < 0 || src >= n_atoms) continue;
      const double rv[3] = {pair_r[3 * pr], pair_r[3 * pr + 1], pair_r[3 * pr + 2]};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double sv = colr[u] < M ? S[(int64_t)src * ldS + colr[u]] : 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int b = 0; b < 3; ++b) acc[3 * al + b][u] += rv[al] * sv * G[b][u][r];
      }
    }
  }
  // sum the four lane groups (pair rows), then the waves
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      acc[q][u] += __shfl_xor(acc[q][u], 16);
      acc[q][u] += __shfl_xor(acc[q][u], 32);
    }
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
      for (int u = 0; u < 4; ++u) red[wave][q][u * 16 + idx] = acc[q][u];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int64_t col = colbase + threadIdx.x;
    if (col < M) {
#pragma unroll
      for (int q = 0; q < 9; ++q) {
        const double t = red[0][q][threadIdx.x] + red[1][q][threadIdx.x] +
                         red[2][q][threadIdx.x] + red[3][q][threadIdx.x];
        K[(9 * c + q) + col * ldk] = -t;
      }
    }
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void virial_rows_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* X,
                     int64_t ldx, int64_t M, const double* S, int64_t ldS, const int64_t* cfg_ptr,
                     int64_t n_cfg, const int64_t* pair_ptr, const int32_t* pair_src,
                     const double* pair_r, int64_t n_atoms, int64_t n_pairs, double* K,
                     int64_t ldk, hipStream_t st) {
  if (n_cfg <= 0 || M <= 0) return;
  dim3 grid(cdiv(M, 64), (unsigned)n_cfg);
  if (jac_f32)
    hipLaunchKernelGGL(k_virial_rows<float>, grid, dim3(256), 0, st,
                       reinterpret_cast<const float*>(jac), ldj, D, X, ldx, M, S, ldS, cfg_ptr,
                       pair_ptr, pair_src, pair_r, n_atoms, n_pairs, K, ldk);
  else
    hipLaunchKernelGGL(k_virial_rows<double>, grid, dim3(256), 0, st,
                       reinterpret_cast<const double*>(jac), ldj, D, X, ldx, M, S, ldS, cfg_ptr,
                       pair_ptr, pair_src, pair_r, n_atoms, n_pairs, K, ldk);
}

}  // namespace gapk
