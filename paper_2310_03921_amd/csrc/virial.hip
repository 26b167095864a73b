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
// columns; its eight waves are four pair streams x two 32-column halves.  A
// stream takes the configuration's pairs 16 at a time (stream s the chunks s,
// s + 4, ...), contracts the three Jacobian rows of each pair with its columns'
// x_m on the FP64 matrix core (whole 16-deep steps load unconditionally, the
// next step's fragments ahead of the current step's matrix work; one guarded
// step covers a D that is not a multiple of 16), and accumulates the nine
// weighted sums in registers.  One cross-lane and cross-wave reduction in a
// fixed order ends the block, so results do not depend on scheduling.
#include "launch.h"
#include "mma_f64.h"

namespace gapk {

namespace {

constexpr int kVU = 2;  // 16-column tiles per wave; a wave pair covers the block's 64 columns
template <typename TJ>
__global__ __launch_bounds__(512) void k_virial_rows(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const double* __restrict__ X,
    int64_t ldx, int64_t M, const double* __restrict__ S, int64_t ldS,
    const int64_t* __restrict__ cfg_ptr, const int64_t* __restrict__ pair_ptr,
    const int32_t* __restrict__ pair_src, const double* __restrict__ pair_r, int64_t n_atoms,
    int64_t n_pairs, double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_cfg) {
  __shared__ double red[4][9][64];
  int64_t c, ct;
  if (!xcd_group_tile(n_cfg, n_ct, c, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int stream = wave >> 1;  // pair chunks stream, stream + 4, ...
  const int64_t colbase = ct * 64 + (wave & 1) * 16 * kVU;
  const int64_t a0 = min(max(cfg_ptr[c], (int64_t)0), n_atoms);
  const int64_t a1 = min(max(cfg_ptr[c + 1], a0), n_atoms);
  const int64_t p_lo = min(max(pair_ptr[a0], (int64_t)0), n_pairs);
  const int64_t p_hi = min(max(pair_ptr[a1], p_lo), n_pairs);

  FragRowK<double> fb[kVU];
  const double* xr[kVU];
  int64_t colr[kVU];
#pragma unroll
  for (int u = 0; u < kVU; ++u) {
    colr[u] = colbase + u * 16 + idx;
    fb[u] = FragRowK<double>{X + (colr[u] < M ? colr[u] : 0) * ldx, D, colr[u] < M};
    xr[u] = X + min(colr[u], M - 1) * ldx + 4 * g;  // columns past M are never stored
  }
  double acc[9][kVU];
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int u = 0; u < kVU; ++u) acc[q][u] = 0.0;
  const int64_t kfull = D & ~int64_t(15);  // whole 16-deep steps

  for (int64_t p0 = p_lo + 16 * stream; p0 < p_hi; p0 += 64) {
    // pairs past the configuration read its last pair's rows (never accumulated)
    const int64_t p = min(p0 + idx, p_hi - 1);
    const TJ* jr = jac + p * 3 * ldj + 4 * g;
    d4v G[3][kVU];
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int u = 0; u < kVU; ++u) G[b][u] = zero4();
    // whole 16-deep steps with unconditional loads, the next step's fragments
    // loaded before this step's matrix work; then one guarded tail step
    double a[2][3][4], bx[2][kVU][4];
    auto load = [&](int64_t k0, int st) {
#pragma unroll
      for (int b = 0; b < 3; ++b) load4u(jr + b * ldj + k0, a[st][b]);
#pragma unroll
      for (int u = 0; u < kVU; ++u) load4u(xr[u] + k0, bx[st][u]);
    };
    auto step = [&](int st) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
          for (int u = 0; u < kVU; ++u) G[b][u] = mfma_f64(a[st][b][s4], bx[st][u][s4], G[b][u]);
    };
    int64_t k0 = 0;
    if (kfull > 0) load(0, 0);
    for (; k0 + 32 <= kfull; k0 += 32) {
      load(k0 + 16, 1);
      step(0);
      if (k0 + 32 < kfull) load(k0 + 32, 0);
      step(1);
    }
    if (k0 < kfull) {  // an odd number of whole steps: the last one is loaded in set 0
      step(0);
      k0 += 16;
    }
    if (k0 < D) {
      const TJ* jt = jac + p * 3 * ldj;
#pragma unroll
      for (int b = 0; b < 3; ++b) FragRowK<TJ>{jt + b * ldj, D, true}.frag(k0, g, a[0][b]);
#pragma unroll
      for (int u = 0; u < kVU; ++u) fb[u].frag(k0, g, bx[0][u]);
      step(0);
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
      for (int u = 0; u < kVU; ++u) {
        const double sv = colr[u] < M ? S[(int64_t)src * ldS + colr[u]] : 0.0;
#pragma unroll
        for (int al = 0; al < 3; ++al)
#pragma unroll
          for (int b = 0; b < 3; ++b) acc[3 * al + b][u] += rv[al] * sv * G[b][u][r];
      }
    }
  }
  // sum the four lane groups (pair rows), then the four pair streams
#pragma unroll
  for (int q = 0; q < 9; ++q)
#pragma unroll
    for (int u = 0; u < kVU; ++u) {
      acc[q][u] += __shfl_xor(acc[q][u], 16);
      acc[q][u] += __shfl_xor(acc[q][u], 32);
    }
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < 9; ++q)
#pragma unroll
      for (int u = 0; u < kVU; ++u) red[stream][q][(wave & 1) * 16 * kVU + u * 16 + idx] = acc[q][u];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int64_t col = ct * 64 + threadIdx.x;
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

// Unconditional 4-wide loads of a Jacobian row segment (32-byte aligned).
GAP_DEV void ldj4(const double* p, double out[4]) {
  const d4v v = *reinterpret_cast<const d4v*>(p);
  out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
}
GAP_DEV void ldj4(const float* p, double out[4]) {
  const f4v v = *reinterpret_cast<const f4v*>(p);
  out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
}

// The same rows for D % 4 == 0 and D <= 256 with the block's 64 columns of X
// resident in LDS for its lifetime, stored in the matrix core's operand order
// (as in the force-row kernel): twelve waves, wave w taking Jacobian component
// beta = w % 3 of pair stream w / 3, so three waves share a SIMD.  Every load
// in the pair loop reads a valid address (pairs past the configuration read
// its last pair, k blocks past D the row's last four elements against zero
// rows of X) and invalid data are cancelled by zero weights; the next k
// block's (or the next chunk's first) Jacobian fragment is loaded before the
// current block's matrix work.
constexpr int kVW = 12;
constexpr int kVNC = 4;      // 16-column tiles per block
constexpr int kVMaxKb = 16;  // D <= 256
template <typename TJ>
__global__ __launch_bounds__(64 * kVW) void k_virial_rows_lds(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const double* __restrict__ X,
    int64_t ldx, int64_t M, const double* __restrict__ S, int64_t ldS,
    const int64_t* __restrict__ cfg_ptr, const int64_t* __restrict__ pair_ptr,
    const int32_t* __restrict__ pair_src, const double* __restrict__ pair_r, int64_t n_atoms,
    int64_t n_pairs, double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_cfg, int nkb) {
  extern __shared__ double xs[];  // [nkb][kVNC][2 halves][64 lanes][2]
  __shared__ double red[4][9][64];
  int64_t c, ct;
  if (!xcd_group_tile(n_cfg, n_ct, c, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int beta = wave % 3, stream = wave / 3;
  const int64_t colbase = ct * (16 * kVNC);
  for (int e = threadIdx.x; e < nkb * kVNC * 64; e += 64 * kVW) {
    const int kb = e / (kVNC * 64), rem = e % (kVNC * 64);
    const int u = rem / 64, ln = rem % 64;
    const int64_t col = colbase + 4 * (ln & 15) + u;  // lane idx of tile u: column 4 idx + u
    double v[4];
    if (col < M)
      load4(X + col * ldx, (int64_t)kb * 16 + 4 * (ln >> 4), D, v);
    else
      zero_frag(v);
    const d2v lo = {v[0], v[1]}, hi = {v[2], v[3]};
    double* t = xs + (size_t)(e >> 6) * 256 + 2 * (e & 63);
    *reinterpret_cast<d2v*>(t) = lo;
    *reinterpret_cast<d2v*>(t + 128) = hi;
  }
  __syncthreads();

  const int64_t a0 = min(max(cfg_ptr[c], (int64_t)0), n_atoms);
  const int64_t a1 = min(max(cfg_ptr[c + 1], a0), n_atoms);
  const int64_t p_lo = min(max(pair_ptr[a0], (int64_t)0), n_pairs);
  const int64_t p_hi = min(max(pair_ptr[a1], p_lo), n_pairs);
  const int64_t kmax4 = D - 4;
  double cm[kVNC];
#pragma unroll
  for (int u = 0; u < kVNC; ++u) cm[u] = colbase + 4 * idx + u < M ? 1.0 : 0.0;
  const int64_t scol = min(colbase + 4 * idx, ldS - 4);
  double acc[3][kVNC];
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int u = 0; u < kVNC; ++u) acc[al][u] = 0.0;
  const d2v* xb = reinterpret_cast<const d2v*>(xs) + lane;
  auto xfrag = [&](int tile) -> d4v {
    const d2v lo = xb[tile * 128], hi = xb[tile * 128 + 64];
    const d4v f = {lo[0], lo[1], hi[0], hi[1]};
    return f;
  };
  if (p_lo < p_hi && p_lo + 16 * stream < p_hi) {
    auto row_of = [&](int64_t p0) -> const TJ* {
      return jac + min(p0 + idx, p_hi - 1) * 3 * ldj + beta * ldj;
    };
    int64_t p0 = p_lo + 16 * stream;
    const TJ* jr = row_of(p0);
    double fa[4], fb[4];
    ldj4(jr + min((int64_t)4 * g, kmax4), fa);
    for (; p0 < p_hi; p0 += 64) {
      const int64_t pn = p0 + 64;
      const TJ* jn = row_of(pn < p_hi ? pn : p0);
      d4v G[kVNC];
#pragma unroll
      for (int u = 0; u < kVNC; ++u) G[u] = zero4();
      for (int kb = 0; kb < nkb; kb += 2) {  // nkb is even
        ldj4(jr + min((int64_t)(kb + 1) * 16 + 4 * g, kmax4), fb);
        {
          d4v b[kVNC];
#pragma unroll
          for (int u = 0; u < kVNC; ++u) b[u] = xfrag(kb * kVNC + u);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int u = 0; u < kVNC; ++u) G[u] = mfma_f64(fa[s4], b[u][s4], G[u]);
        }
        const bool more = kb + 2 < nkb;
        const TJ* jp = more ? jr + (int64_t)(kb + 2) * 16 : jn;
        ldj4(jp + min((int64_t)4 * g, kmax4 - (more ? (int64_t)(kb + 2) * 16 : 0)), fa);
        {
          d4v b[kVNC];
#pragma unroll
          for (int u = 0; u < kVNC; ++u) b[u] = xfrag((kb + 1) * kVNC + u);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int u = 0; u < kVNC; ++u) G[u] = mfma_f64(fb[s4], b[u][s4], G[u]);
        }
      }
      // C layout: lane holds pairs p0 + g + 4 r of its four columns
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t pr = p0 + g + 4 * r;
        const int64_t pc = min(pr, p_hi - 1);
        const int32_t src = pair_src[pc];
        const double ok = (pr < p_hi && src >= 0 && src < n_atoms) ? 1.0 : 0.0;
        const int64_t sr = min(max((int64_t)src, (int64_t)0), n_atoms - 1);
        const d4v sv = *reinterpret_cast<const d4v*>(S + sr * ldS + scol);
        const double rv[3] = {ok * pair_r[3 * pc], ok * pair_r[3 * pc + 1],
                              ok * pair_r[3 * pc + 2]};
#pragma unroll
        for (int u = 0; u < kVNC; ++u) {
          const double w = sv[u] * cm[u] * G[u][r];
#pragma unroll
          for (int al = 0; al < 3; ++al) acc[al][u] += rv[al] * w;
        }
      }
      jr = jn;
    }
  }
  // sum the four lane groups (pair rows), then the four pair streams of each beta
#pragma unroll
  for (int al = 0; al < 3; ++al)
#pragma unroll
    for (int u = 0; u < kVNC; ++u) {
      acc[al][u] += __shfl_xor(acc[al][u], 16);
      acc[al][u] += __shfl_xor(acc[al][u], 32);
    }
  if (g == 0) {
#pragma unroll
    for (int al = 0; al < 3; ++al)
#pragma unroll
      for (int u = 0; u < kVNC; ++u) red[stream][3 * al + beta][4 * idx + u] = acc[al][u];
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

}  // namespace

void virial_rows_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* X,
                     int64_t ldx, int64_t M, const double* S, int64_t ldS, const int64_t* cfg_ptr,
                     int64_t n_cfg, const int64_t* pair_ptr, const int32_t* pair_src,
                     const double* pair_r, int64_t n_atoms, int64_t n_pairs, double* K,
                     int64_t ldk, hipStream_t st) {
  if (n_cfg <= 0 || M <= 0) return;
  // the column tiles of a configuration stay on one XCD (its pairs' Jacobian
  // rows are then read from HBM once, into that XCD's L2); configurations are
  // dealt to the XCDs in turn
  const int64_t n_ct = (M + 63) / 64;
  dim3 grid(xcd_group_tile_blocks(n_cfg, n_ct));
  if (D % 4 == 0 && D >= 4 && D <= 16 * kVMaxKb && ldS % 4 == 0 && ldS >= 4) {
    const int nkb = 2 * (int)((D + 31) / 32);  // even, 16-deep blocks
    const size_t lds = (size_t)nkb * kVNC * 64 * 4 * sizeof(double);
    static bool attr = false;
    if (!attr) {
      const int mx = (int)((size_t)kVMaxKb * kVNC * 64 * 4 * sizeof(double));
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_virial_rows_lds<float>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx);
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_virial_rows_lds<double>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, mx);
      attr = true;
    }
    if (jac_f32)
      hipLaunchKernelGGL(k_virial_rows_lds<float>, grid, dim3(64 * kVW), lds, st,
                         reinterpret_cast<const float*>(jac), ldj, D, X, ldx, M, S, ldS, cfg_ptr,
                         pair_ptr, pair_src, pair_r, n_atoms, n_pairs, K, ldk, n_ct, n_cfg, nkb);
    else
      hipLaunchKernelGGL(k_virial_rows_lds<double>, grid, dim3(64 * kVW), lds, st,
                         reinterpret_cast<const double*>(jac), ldj, D, X, ldx, M, S, ldS, cfg_ptr,
                         pair_ptr, pair_src, pair_r, n_atoms, n_pairs, K, ldk, n_ct, n_cfg, nkb);
    return;
  }
  if (jac_f32)
    hipLaunchKernelGGL(k_virial_rows<float>, grid, dim3(512), 0, st,
                       reinterpret_cast<const float*>(jac), ldj, D, X, ldx, M, S, ldS, cfg_ptr,
                       pair_ptr, pair_src, pair_r, n_atoms, n_pairs, K, ldk, n_ct, n_cfg);
  else
    hipLaunchKernelGGL(k_virial_rows<double>, grid, dim3(512), 0, st,
                       reinterpret_cast<const double*>(jac), ldj, D, X, ldx, M, S, ldS, cfg_ptr,
                       pair_ptr, pair_src, pair_r, n_atoms, n_pairs, K, ldk, n_ct, n_cfg);
}

}  // namespace gapk
