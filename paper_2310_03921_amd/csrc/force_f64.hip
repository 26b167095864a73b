// Force observations of L-hat K_NM, and force prediction, in FP64.
//
// Force row (j, alpha), column m (Sec. "Theory": derivative rows of K_NM,
// accumulated over every pair pointing at atom j):
//   K_F[(j,alpha), m] = - sum_{(i,k): j(i,k)=j} S[i][m] * (J[(i,k)][alpha] . x_m),
//   S[i][m] = delta^2 zeta (d_i . x_m)^(zeta-1)   (written by the energy-row kernel).
//
// Work decomposition: a wavefront owns 16 target atoms (a "slot group" of the
// degree-sorted target list) and 16*NC sparse-point columns.  Step t multiplies
// the t-th incoming pair of each of the 16 targets (one matrix row per target,
// three alpha components as three accumulators) with X^T on the FP64 matrix
// core, scales the 16 x 16 results by S of each pair's source atom, and adds
// them into per-target accumulators that stay in registers for the whole
// kernel.  Each output row is written once, no atomics, so results do not
// depend on scheduling.  The four waves of a block share the slot group (their
// Jacobian rows hit L1) and cover consecutive column ranges.
#include "launch.h"
#include "mma_f64.h"

namespace gapk {

namespace {

constexpr int kFNC = 2;  // 16-column tiles per wave in the force-row kernel

template <typename TJ>
__global__ __launch_bounds__(256) void k_force_rows(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const double* __restrict__ X,
    int64_t ldx, int64_t M, const double* __restrict__ S, int64_t ldS,
    const int64_t* __restrict__ tgt_ptr, const int32_t* __restrict__ tgt_pair,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ order, int64_t n_atoms,
    int64_t row0, double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_grp) {
  int64_t ct, grp;
  if (!xcd_group_tile(n_grp, n_ct, grp, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t colbase = (ct * 4 + wave) * (16 * kFNC);
  if (colbase >= M) return;

  // Row metadata: lane idx describes slot row idx (same in every lane group).
  const int64_t slot = grp * 16 + idx;
  const int target = slot < n_atoms ? order[slot] : -1;
  const int64_t seg0 = target >= 0 ? tgt_ptr[target] : 0;
  const int deg = target >= 0 ? (int)(tgt_ptr[target + 1] - seg0) : 0;
  const int maxdeg = wave_max16(deg);

  FragRowK<double> fb[kFNC];
#pragma unroll
  for (int u = 0; u < kFNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
    fb[u] = FragRowK<double>{X + (col < M ? col : 0) * ldx, D, col < M};
  }
  int64_t colr[kFNC];
#pragma unroll
  for (int u = 0; u < kFNC; ++u) colr[u] = colbase + u * 16 + idx;

  d4v acc[3][kFNC];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int u = 0; u < kFNC; ++u) acc[a][u] = zero4();

  for (int t = 0; t < maxdeg; ++t) {
    int pair = t < deg ? tgt_pair[seg0 + t] : -1;
    const int src = pair >= 0 ? pair_src[pair] : -1;
    if (src < 0) pair = -1;
    const TJ* jr = jac + (int64_t)(pair >= 0 ? pair : 0) * 3 * ldj;
    FragRowK<TJ> fa[3] = {FragRowK<TJ>{jr, D, pair >= 0}, FragRowK<TJ>{jr + ldj, D, pair >= 0},
                          FragRowK<TJ>{jr + 2 * ldj, D, pair >= 0}};
    d4v G[3][kFNC];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int u = 0; u < kFNC; ++u) G[a][u] = zero4();

    double a0[3][4], a1[3][4], b0[kFNC][4], b1[kFNC][4];
#pragma unroll
    for (int a = 0; a < 3; ++a) fa[a].frag(0, g, a0[a]);
#pragma unroll
    for (int u = 0; u < kFNC; ++u) fb[u].frag(0, g, b0[u]);
    int64_t k0 = 0;
    for (; k0 + 16 < D; k0 += 32) {
#pragma unroll
      for (int a = 0; a < 3; ++a) fa[a].frag(k0 + 16, g, a1[a]);
#pragma unroll
      for (int u = 0; u < kFNC; ++u) fb[u].frag(k0 + 16, g, b1[u]);
#pragma unroll
      for (int a = 0; a < 3; ++a) mma_block<kFNC>(a0[a], b0, G[a]);
      if (k0 + 32 < D) {
#pragma unroll
        for (int a = 0; a < 3; ++a) fa[a].frag(k0 + 32, g, a0[a]);
#pragma unroll
        for (int u = 0; u < kFNC; ++u) fb[u].frag(k0 + 32, g, b0[u]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) mma_block<kFNC>(a1[a], b1, G[a]);
    }
    if (k0 < D) {
#pragma unroll
      for (int a = 0; a < 3; ++a) mma_block<kFNC>(a0[a], b0, G[a]);
    }

    // acc += S[src(row)][col] * G   (C layout: lane holds rows g + 4 r)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int src_r = __shfl(src, g + 4 * r);
#pragma unroll
      for (int u = 0; u < kFNC; ++u) {
        const double sv = (src_r >= 0 && colr[u] < M) ? S[(int64_t)src_r * ldS + colr[u]] : 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a][u][r] += sv * G[a][u][r];
      }
    }
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tr = __shfl(target, g + 4 * r);
    if (tr < 0) continue;
#pragma unroll
    for (int u = 0; u < kFNC; ++u) {
      if (colr[u] >= M) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a) K[(row0 + 3 * (int64_t)tr + a) + colr[u] * ldk] = -acc[a][u][r];
    }
  }
}

// LDS-resident forms for D <= 256: the block's 64 sparse-point columns of X
// stay in LDS for its whole lifetime, stored in the order the matrix core
// consumes them.  A block covers 64 targets (four 16-target slot groups) x 64
// columns.  Consecutive logical blocks on one XCD walk the column tiles of the
// same 64 targets, so their Jacobian rows are fetched from HBM once and then
// served mostly from that XCD's L2.
constexpr int kLdsNC = 4;
constexpr int kLdsMaxKb = 16;  // D <= 256

// Twelve-wave form: wave w handles Jacobian component alpha = w % 3 of slot
// group w / 3, so three waves share a SIMD and hide each other's Jacobian load
// latency.  X in LDS per 16-k block, per 16-column tile, per lane: 4 doubles.
// (Used when D is not a multiple of 4; k_force_rows_lds12f below otherwise.)
constexpr int kW12 = 12;
template <typename TJ>
__global__ __launch_bounds__(64 * kW12) void k_force_rows_lds12(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const double* __restrict__ X,
    int64_t ldx, int64_t M, const double* __restrict__ S, int64_t ldS,
    const int64_t* __restrict__ tgt_ptr, const int32_t* __restrict__ tgt_pair,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ order, int64_t n_atoms,
    int64_t row0, double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_grp, int nkb) {
  extern __shared__ double xs[];  // [nkb][kLdsNC][64 lanes][4]
  int64_t ct, tgb;
  if (!xcd_group_tile(n_grp, n_ct, tgb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int alpha = wave % 3, grp = wave / 3;
  const int64_t colbase = ct * (16 * kLdsNC);

  for (int e = threadIdx.x; e < nkb * kLdsNC * 64; e += 64 * kW12) {
    const int kb = e / (kLdsNC * 64), rem = e % (kLdsNC * 64);
    const int u = rem / 64, ln = rem % 64;
    const int64_t col = colbase + u * 16 + (ln & 15);
    double v[4];
    if (col < M)
      load4(X + col * ldx, (int64_t)kb * 16 + 4 * (ln >> 4), D, v);
    else
      zero_frag(v);
    d4v w = {v[0], v[1], v[2], v[3]};
    *reinterpret_cast<d4v*>(xs + (size_t)e * 4) = w;
  }
  __syncthreads();

  const int64_t slot = (tgb * 4 + grp) * 16 + idx;
  const int target = slot < n_atoms ? order[slot] : -1;
  const int64_t seg0 = target >= 0 ? tgt_ptr[target] : 0;
  const int deg = target >= 0 ? (int)(tgt_ptr[target + 1] - seg0) : 0;
  const int maxdeg = wave_max16(deg);
  int64_t colr[kLdsNC];
#pragma unroll
  for (int u = 0; u < kLdsNC; ++u) colr[u] = colbase + u * 16 + idx;
  d4v acc[kLdsNC];
#pragma unroll
  for (int u = 0; u < kLdsNC; ++u) acc[u] = zero4();
  const d4v* xb = reinterpret_cast<const d4v*>(xs) + lane;
  auto pair_at = [&](int t) -> int { return t < deg ? tgt_pair[seg0 + t] : -1; };
  int pair = maxdeg > 0 ? pair_at(0) : -1;
  int src = pair >= 0 ? pair_src[pair] : -1;
  if (src < 0) pair = -1;
  double a0[4], a1[4];
  if (pair >= 0) load4(jac + (int64_t)pair * 3 * ldj + alpha * ldj, 4 * g, D, a0); else zero_frag(a0);
  for (int t = 0; t < maxdeg; ++t) {
    const bool pv = pair >= 0;
    const TJ* jr = jac + (int64_t)(pv ? pair : 0) * 3 * ldj + alpha * ldj;
    int pair_n = pair_at(t + 1);
    int src_n = -1;
    d4v G[kLdsNC];
#pragma unroll
    for (int u = 0; u < kLdsNC; ++u) G[u] = zero4();
    for (int kb = 0; kb < nkb; kb += 2) {  // nkb is even
      if (pv) load4(jr, (int64_t)(kb + 1) * 16 + 4 * g, D, a1); else zero_frag(a1);
      if (kb == 0) src_n = pair_n >= 0 ? pair_src[pair_n] : -1;
      {
        d4v b[kLdsNC];
#pragma unroll
        for (int u = 0; u < kLdsNC; ++u) b[u] = xb[(kb * kLdsNC + u) * 64];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int u = 0; u < kLdsNC; ++u) G[u] = mfma_f64(a0[s4], b[u][s4], G[u]);
      }
      if (kb + 2 < nkb) {
        if (pv) load4(jr, (int64_t)(kb + 2) * 16 + 4 * g, D, a0); else zero_frag(a0);
      } else {
        if (src_n < 0) pair_n = -1;
        if (pair_n >= 0) load4(jac + (int64_t)pair_n * 3 * ldj + alpha * ldj, 4 * g, D, a0);
        else zero_frag(a0);
      }
      {
        d4v b[kLdsNC];
#pragma unroll
        for (int u = 0; u < kLdsNC; ++u) b[u] = xb[((kb + 1) * kLdsNC + u) * 64];
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
          for (int u = 0; u < kLdsNC; ++u) G[u] = mfma_f64(a1[s4], b[u][s4], G[u]);
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int src_r = __shfl(src, g + 4 * r);
#pragma unroll
      for (int u = 0; u < kLdsNC; ++u) {
        const double sv = (src_r >= 0 && colr[u] < M) ? S[(int64_t)src_r * ldS + colr[u]] : 0.0;
        acc[u][r] += sv * G[u][r];
      }
    }
    pair = pair_n;
    src = src_n;
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tr = __shfl(target, g + 4 * r);
    if (tr < 0) continue;
#pragma unroll
    for (int u = 0; u < kLdsNC; ++u)
      if (colr[u] < M) K[(row0 + 3 * (int64_t)tr + alpha) + colr[u] * ldk] = -acc[u][r];
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

// The twelve-wave kernel for D % 4 == 0 with no guarded load on its hot path.
// A load under a condition compiles to a branch whose join waits for the load
// at once, which would serialise the Jacobian stream; here every load reads a
// valid address and invalid data is cancelled arithmetically:
//  - k blocks beyond D read the row's last 4 elements and meet zero rows of X;
//  - a slot past its degree (or a target past n_atoms) reads a valid pair of
//    the same target (or pair 0) and its step result is multiplied by a zero S;
//  - S is read at a clamped (source, column) and multiplied by the validity.
// Matrix data are finite, so garbage * 0 == 0.  Results equal those of the
// guarded form up to the order of FP64 additions (identical here: the zero
// contributions add exact zeros).
template <typename TJ>
__global__ __launch_bounds__(64 * kW12) void k_force_rows_lds12f(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const double* __restrict__ X,
    int64_t ldx, int64_t M, const double* __restrict__ S, int64_t ldS,
    const int64_t* __restrict__ tgt_ptr, const int32_t* __restrict__ tgt_pair,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ order, int64_t n_atoms,
    int64_t n_pairs, int64_t row0, double* __restrict__ K, int64_t ldk, int64_t n_ct,
    int64_t n_grp, int nkb) {
  // X tiles in LDS: [nkb][kLdsNC][2 halves][64 lanes][2 doubles]: a lane's four
  // k values of one fragment are split into two 16-byte halves stored 1 KB
  // apart, so each 16-byte LDS read of the wave is contiguous (no bank conflict)
  extern __shared__ double xs[];
  int64_t ct, tgb;
  if (!xcd_group_tile(n_grp, n_ct, tgb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int alpha = wave % 3, grp = wave / 3;
  const int64_t colbase = ct * (16 * kLdsNC);

  for (int e = threadIdx.x; e < nkb * kLdsNC * 64; e += 64 * kW12) {
    const int kb = e / (kLdsNC * 64), rem = e % (kLdsNC * 64);
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

  const int64_t slot = (tgb * 4 + grp) * 16 + idx;
  const int target = slot < n_atoms ? order[slot] : -1;
  const int64_t seg0 = target >= 0 ? tgt_ptr[target] : 0;
  const int deg = target >= 0 ? (int)(tgt_ptr[target + 1] - seg0) : 0;
  const int maxdeg = wave_max16(deg);
  // step t of this slot reads tgt_pair[pair_slot(t)], always a valid entry
  const int64_t last = min(seg0 + max(deg - 1, 0), n_pairs - 1);
  auto pair_slot = [&](int t) -> int64_t { return min(seg0 + t, last); };
  const int64_t kmax4 = D - 4;
  // the four columns of a lane are consecutive (4 idx + u), so its S values
  // for one source are one 32-byte load (S rows padded with zeros to ldS)
  int64_t colr[kLdsNC];
#pragma unroll
  for (int u = 0; u < kLdsNC; ++u) colr[u] = colbase + 4 * idx + u;
  const int64_t scol = min(colbase + 4 * idx, ldS - 4);
  d4v acc[kLdsNC];
#pragma unroll
  for (int u = 0; u < kLdsNC; ++u) acc[u] = zero4();
  const d2v* xb = reinterpret_cast<const d2v*>(xs) + lane;
  auto xfrag = [&](int tile) -> d4v {
    const d2v lo = xb[tile * 128], hi = xb[tile * 128 + 64];
    const d4v f = {lo[0], lo[1], hi[0], hi[1]};
    return f;
  };
  if (maxdeg <= 0) {
    // no pair reaches any of these targets: the rows are zero
  } else {
    // Pair metadata runs one step ahead of its use: at step t the pair of
    // step t + 1 is known, so its source and the pair of step t + 2 are
    // loaded now and first needed a whole step later.
    int pair = tgt_pair[pair_slot(0)];
    int pair_n = tgt_pair[pair_slot(1)];
    int src = pair_src[pair];
    double a0[4], a1[4];
    const TJ* jr = jac + (int64_t)pair * 3 * ldj + alpha * ldj;
    ldj4(jr + min((int64_t)4 * g, kmax4), a0);
    for (int t = 0; t < maxdeg; ++t) {
      const int pair_nn = tgt_pair[pair_slot(t + 2)];
      const int src_n = pair_src[pair_n];
      const TJ* jn = jac + (int64_t)pair_n * 3 * ldj + alpha * ldj;
      d4v G[kLdsNC];
#pragma unroll
      for (int u = 0; u < kLdsNC; ++u) G[u] = zero4();
      for (int kb = 0; kb < nkb; kb += 2) {  // nkb is even
        ldj4(jr + min((int64_t)(kb + 1) * 16 + 4 * g, kmax4), a1);
        {
          d4v b[kLdsNC];
#pragma unroll
          for (int u = 0; u < kLdsNC; ++u) b[u] = xfrag(kb * kLdsNC + u);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int u = 0; u < kLdsNC; ++u) G[u] = mfma_f64(a0[s4], b[u][s4], G[u]);
        }
        // the next block of this step, or the first block of the next step
        const TJ* jp = (kb + 2 < nkb) ? jr + (int64_t)(kb + 2) * 16 : jn;
        ldj4(jp + min((int64_t)4 * g, kmax4 - ((kb + 2 < nkb) ? (int64_t)(kb + 2) * 16 : 0)), a0);
        {
          d4v b[kLdsNC];
#pragma unroll
          for (int u = 0; u < kLdsNC; ++u) b[u] = xfrag((kb + 1) * kLdsNC + u);
#pragma unroll
          for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
            for (int u = 0; u < kLdsNC; ++u) G[u] = mfma_f64(a1[s4], b[u][s4], G[u]);
        }
      }
      d4v sv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src_r = __shfl(src, g + 4 * r);
        sv[r] = *reinterpret_cast<const d4v*>(S + (int64_t)max(src_r, 0) * ldS + scol);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src_r = __shfl(src, g + 4 * r);
        const int deg_r = __shfl(deg, g + 4 * r);
        const bool ok_r = t < deg_r && src_r >= 0;
#pragma unroll
        for (int u = 0; u < kLdsNC; ++u)
          acc[u][r] += sv[r][u] * ((ok_r && colr[u] < M) ? 1.0 : 0.0) * G[u][r];
      }
      jr = jn;
      pair_n = pair_nn;
      src = src_n;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tr = __shfl(target, g + 4 * r);
    if (tr < 0) continue;
#pragma unroll
    for (int u = 0; u < kLdsNC; ++u)
      if (colr[u] < M) K[(row0 + 3 * (int64_t)tr + alpha) + colr[u] * ldk] = -acc[u][r];
  }
}

// f_pair[p][alpha] = J[p][alpha] . g[src(p)]; one wavefront per pair.
template <typename TJ>
__global__ __launch_bounds__(256) void k_pair_dots(const TJ* __restrict__ jac, int64_t ldj,
                                                   int64_t D, const double* __restrict__ gm,
                                                   int64_t ldg, const int32_t* __restrict__ src,
                                                   int64_t n_pairs, double* __restrict__ f_pair) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t p = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6); p < n_pairs;
       p += nw) {
    const int i = src[p];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (i >= 0) {
      const TJ* jr = jac + p * 3 * ldj;
      const double* gr = gm + (int64_t)i * ldg;
      for (int64_t k = 4 * lane; k < D; k += 256) {
        double gv[4], j0[4], j1[4], j2[4];
        load4(gr, k, D, gv);
        load4(jr, k, D, j0);
        load4(jr + ldj, k, D, j1);
        load4(jr + 2 * ldj, k, D, j2);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          s0 += j0[q] * gv[q];
          s1 += j1[q] * gv[q];
          s2 += j2[q] * gv[q];
        }
      }
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      f_pair[p * 3 + 0] = s0;
      f_pair[p * 3 + 1] = s1;
      f_pair[p * 3 + 2] = s2;
    }
  }
}

// The same products for D % 4 == 0, D <= 1024, with every load of a wave
// issued before any use: a wave takes PB consecutive pairs (PB * IT = 4, IT =
// 256-element segments per row) and a lane the 4-element segments 4 lane +
// 256 it of the pairs' three Jacobian rows and source gradients.  Segments
// past D re-read the row's last four elements and are weighted by zero; a
// pair past n_pairs re-reads the last pair and is not stored.
template <typename TJ, int IT, int PB>
__global__ __launch_bounds__(256) void k_pair_dots4(const TJ* __restrict__ jac, int64_t ldj,
                                                    int64_t D, const double* __restrict__ gm,
                                                    int64_t ldg, const int32_t* __restrict__ src,
                                                    int64_t n_pairs,
                                                    double* __restrict__ f_pair) {
  const int lane = threadIdx.x & 63;
  const int64_t p0 = (blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6)) * PB;
  if (p0 >= n_pairs) return;
  int64_t kk[IT];
  double wk[IT];
#pragma unroll
  for (int it = 0; it < IT; ++it) {
    const int64_t k = 4 * lane + 256 * it;
    kk[it] = min(k, D - 4);
    wk[it] = k < D ? 1.0 : 0.0;
  }
  double gv[PB][IT][4], jv[PB][3][IT][4];
  int32_t si[PB];
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    const int64_t p = min(p0 + q, n_pairs - 1);
    si[q] = src[p];
    const double* gr = gm + (int64_t)max(si[q], 0) * ldg;
    const TJ* jr = jac + p * 3 * ldj;
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      ldj4(gr + kk[it], gv[q][it]);
#pragma unroll
      for (int a = 0; a < 3; ++a) ldj4(jr + a * ldj + kk[it], jv[q][a][it]);
    }
  }
#pragma unroll
  for (int q = 0; q < PB; ++q) {
    double s[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double t = 0.0;
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        double u = 0.0;
#pragma unroll
        for (int e = 0; e < 4; ++e) u += jv[q][a][it][e] * gv[q][it][e];
        t += wk[it] * u;
      }
      s[a] = wave_sum(t);
    }
    const int64_t p = p0 + q;
    if (lane == 0 && p < n_pairs) {
      const double ok = si[q] >= 0 ? 1.0 : 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) f_pair[p * 3 + a] = ok * s[a];
    }
  }
}

__global__ void k_gather_forces(const double* __restrict__ f_pair,
                                const int64_t* __restrict__ tgt_ptr,
                                const int32_t* __restrict__ tgt_pair, int64_t n_atoms,
                                double* __restrict__ F) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < 3 * n_atoms;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = q / 3;
    const int a = (int)(q - 3 * j);
    double s = 0.0;
    for (int64_t e = tgt_ptr[j]; e < tgt_ptr[j + 1]; ++e) s += f_pair[(int64_t)tgt_pair[e] * 3 + a];
    F[q] = -s;
  }
}

// h[i] = sum over the pairs (i, k) of sum_alpha v[j(i,k)][alpha] J[(i,k)][alpha]; one wave per atom.
constexpr int kHMaxIt = 8;  // D <= 2048
template <typename TJ>
__global__ __launch_bounds__(256) void k_jac_t_apply(const TJ* __restrict__ jac, int64_t ldj,
                                                     int64_t D, const int64_t* __restrict__ pair_ptr,
                                                     const int32_t* __restrict__ pair_j,
                                                     int64_t n_atoms, int64_t n_pairs,
                                                     const double* __restrict__ v,
                                                     double* __restrict__ h, int64_t ldh) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n_atoms) return;
  double acc[kHMaxIt][4];
#pragma unroll
  for (int it = 0; it < kHMaxIt; ++it)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[it][q] = 0.0;
  const int64_t lo = max((int64_t)0, pair_ptr[i]), hi = min(n_pairs, pair_ptr[i + 1]);
  for (int64_t p = lo; p < hi; ++p) {
    const int32_t j = pair_j[p];
    if (j < 0 || j >= n_atoms) continue;
    const double v0 = v[3 * (int64_t)j], v1 = v[3 * (int64_t)j + 1], v2 = v[3 * (int64_t)j + 2];
    const TJ* jr = jac + p * 3 * ldj;
#pragma unroll
    for (int it = 0; it < kHMaxIt; ++it) {
      const int64_t k = 4 * lane + 256 * it;
      if (k >= D) break;
      double j0[4], j1[4], j2[4];
      load4(jr, k, D, j0);
      load4(jr + ldj, k, D, j1);
      load4(jr + 2 * ldj, k, D, j2);
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[it][q] += v0 * j0[q] + v1 * j1[q] + v2 * j2[q];
    }
  }
#pragma unroll
  for (int it = 0; it < kHMaxIt; ++it) {
    const int64_t k = 4 * lane + 256 * it;
    if (k >= D) break;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k + q < D) h[i * ldh + k + q] = acc[it][q];
  }
}

// The same product for D % 4 == 0 and D <= 256 with no guarded load in its
// pair loop: a lane reads the 4-element segment min(4 lane, D - 4) of the
// three Jacobian rows of a pair (lanes past D re-read the last segment and
// store nothing), and the pair's target and v come from one guarded batch load
// per 64 pairs, broadcast from lane q with readlane (so they are scalars), so
// the loads of successive pairs overlap instead of waiting on each other.
// The association order of the sum (per pair, then over pairs) is the one of
// k_jac_t_apply.
GAP_DEV double readlane_f64(double x, int q) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)b, q);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(b >> 32), q);
  return __builtin_bit_cast(double, (uint64_t)hi << 32 | lo);
}
template <typename TJ>
__global__ __launch_bounds__(256) void k_jac_t_apply4(const TJ* __restrict__ jac, int64_t ldj,
                                                      int64_t D,
                                                      const int64_t* __restrict__ pair_ptr,
                                                      const int32_t* __restrict__ pair_j,
                                                      int64_t n_atoms, int64_t n_pairs,
                                                      const double* __restrict__ v,
                                                      double* __restrict__ h, int64_t ldh) {
  const int lane = threadIdx.x & 63;
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= n_atoms) return;
  const int64_t kk = min((int64_t)4 * lane, D - 4);
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t lo = max((int64_t)0, pair_ptr[i]), hi = min(n_pairs, pair_ptr[i + 1]);
  for (int64_t base = lo; base < hi; base += 64) {
    const int64_t pl = base + lane;
    const int32_t j = pl < hi ? pair_j[pl] : -1;
    const bool ok = j >= 0 && j < n_atoms;
    const double w0 = ok ? v[3 * (int64_t)j] : 0.0;
    const double w1 = ok ? v[3 * (int64_t)j + 1] : 0.0;
    const double w2 = ok ? v[3 * (int64_t)j + 2] : 0.0;
    const int cnt = (int)min((int64_t)64, hi - base);
#pragma unroll 4
    for (int q = 0; q < cnt; ++q) {
      const double v0 = readlane_f64(w0, q), v1 = readlane_f64(w1, q), v2 = readlane_f64(w2, q);
      const bool okq = __builtin_amdgcn_readlane((int)ok, q) != 0;
      const TJ* jr = jac + (base + q) * 3 * ldj + kk;
      double j0[4], j1[4], j2[4];
      ldj4(jr, j0);
      ldj4(jr + ldj, j1);
      ldj4(jr + 2 * ldj, j2);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double t = acc[u] + (v0 * j0[u] + v1 * j1[u] + v2 * j2[u]);
        acc[u] = okq ? t : acc[u];  // a left-out pair adds nothing, even a non-finite J row
      }
    }
  }
  if (4 * lane < D) {
#pragma unroll
    for (int u = 0; u < 4; ++u) h[i * ldh + 4 * lane + u] = acc[u];
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void force_rows_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* X,
                    int64_t ldx, int64_t M, const double* S, int64_t ldS, const int64_t* tgt_ptr,
                    const int32_t* tgt_pair, const int32_t* pair_src, const int32_t* order,
                    int64_t n_atoms, int64_t n_pairs, int64_t row0, double* K, int64_t ldk,
                    hipStream_t st) {
  if (n_atoms <= 0 || M <= 0) return;
  if (D <= 16 * kLdsMaxKb && D % 4 == 0 && ldS % 4 == 0 && ldS >= 4 && n_pairs > 0) {
    const int nkb = (int)(((D + 15) / 16 + 1) / 2 * 2);  // even number of 16-k blocks
    const int64_t n_ct = (M + 16 * kLdsNC - 1) / (16 * kLdsNC);
    const int64_t n_tgb = (n_atoms + 63) / 64;
    const unsigned blocks = xcd_group_tile_blocks(n_tgb, n_ct);
    const size_t lds = (size_t)nkb * kLdsNC * 64 * 4 * sizeof(double);
    const int lds_max = 16 * kLdsNC * 64 * 4 * 8;
    dim3 grid(blocks);
    if (jac_f32) {
      static bool attr = false;
      if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_rows_lds12f<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
        attr = true;
      }
      hipLaunchKernelGGL(k_force_rows_lds12f<float>, grid, dim3(64 * kW12), lds, st,
                         reinterpret_cast<const float*>(jac), ldj, D, X, ldx, M, S, ldS, tgt_ptr,
                         tgt_pair, pair_src, order, n_atoms, n_pairs, row0, K, ldk, n_ct, n_tgb,
                         nkb);
    } else {
      static bool attr = false;
      if (!attr) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_rows_lds12f<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
        attr = true;
      }
      hipLaunchKernelGGL(k_force_rows_lds12f<double>, grid, dim3(64 * kW12), lds, st,
                         reinterpret_cast<const double*>(jac), ldj, D, X, ldx, M, S, ldS, tgt_ptr,
                         tgt_pair, pair_src, order, n_atoms, n_pairs, row0, K, ldk, n_ct, n_tgb,
                         nkb);
    }
    return;
  }
  if (D <= 16 * kLdsMaxKb) {
    const int nkb = (int)(((D + 15) / 16 + 1) / 2 * 2);  // even number of 16-k blocks
    const int64_t n_ct = (M + 16 * kLdsNC - 1) / (16 * kLdsNC);
    const int64_t n_tgb = (n_atoms + 63) / 64;
    const unsigned blocks = xcd_group_tile_blocks(n_tgb, n_ct);
    const size_t lds = (size_t)nkb * kLdsNC * 64 * 4 * sizeof(double);
    dim3 grid(blocks);
    if (jac_f32) {
      static bool attr_f = false;
      if (!attr_f) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_rows_lds12<float>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 16 * kLdsNC * 64 * 4 * 8);
        attr_f = true;
      }
      hipLaunchKernelGGL(k_force_rows_lds12<float>, grid, dim3(64 * kW12), lds, st,
                         reinterpret_cast<const float*>(jac), ldj, D, X, ldx, M, S, ldS, tgt_ptr,
                         tgt_pair, pair_src, order, n_atoms, row0, K, ldk, n_ct, n_tgb, nkb);
    } else {
      static bool attr_d = false;
      if (!attr_d) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_rows_lds12<double>),
                                  hipFuncAttributeMaxDynamicSharedMemorySize, 16 * kLdsNC * 64 * 4 * 8);
        attr_d = true;
      }
      hipLaunchKernelGGL(k_force_rows_lds12<double>, grid, dim3(64 * kW12), lds, st,
                         reinterpret_cast<const double*>(jac), ldj, D, X, ldx, M, S, ldS, tgt_ptr,
                         tgt_pair, pair_src, order, n_atoms, row0, K, ldk, n_ct, n_tgb, nkb);
    }
    return;
  }
  const int64_t n_ct = (M + 4 * 16 * kFNC - 1) / (4 * 16 * kFNC);
  const int64_t n_grp = (n_atoms + 15) / 16;
  dim3 grid(xcd_group_tile_blocks(n_grp, n_ct));
  if (jac_f32)
    hipLaunchKernelGGL(k_force_rows<float>, grid, dim3(256), 0, st,
                       reinterpret_cast<const float*>(jac), ldj, D, X, ldx, M, S, ldS, tgt_ptr,
                       tgt_pair, pair_src, order, n_atoms, row0, K, ldk, n_ct, n_grp);
  else
    hipLaunchKernelGGL(k_force_rows<double>, grid, dim3(256), 0, st,
                       reinterpret_cast<const double*>(jac), ldj, D, X, ldx, M, S, ldS, tgt_ptr,
                       tgt_pair, pair_src, order, n_atoms, row0, K, ldk, n_ct, n_grp);
}

void forces_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const double* g,
                int64_t ldg, const int32_t* pair_src, int64_t n_atoms, int64_t n_pairs,
                const int64_t* tgt_ptr, const int32_t* tgt_pair, double* f_pair, double* forces,
                hipStream_t st) {
  if (n_atoms <= 0) return;
  if (n_pairs > 0 && D % 4 == 0 && D >= 4 && D <= 1024 && ldg % 4 == 0) {
    // IT 256-element segments per row and PB = 4 / IT pairs per wave, 4 waves a block
    const int it = (int)((D + 255) / 256);
    const unsigned b4 = cdiv(cdiv(n_pairs, 4), 4), b2 = cdiv(cdiv(n_pairs, 2), 4),
                   b1 = cdiv(n_pairs, 4);
    const dim3 blk(256);
    if (jac_f32) {
      const float* j = reinterpret_cast<const float*>(jac);
      if (it == 1)
        hipLaunchKernelGGL((k_pair_dots4<float, 1, 4>), dim3(b4), blk, 0, st, j, ldj, D, g, ldg,
                           pair_src, n_pairs, f_pair);
      else if (it == 2)
        hipLaunchKernelGGL((k_pair_dots4<float, 2, 2>), dim3(b2), blk, 0, st, j, ldj, D, g, ldg,
                           pair_src, n_pairs, f_pair);
      else
        hipLaunchKernelGGL((k_pair_dots4<float, 4, 1>), dim3(b1), blk, 0, st, j, ldj, D, g, ldg,
                           pair_src, n_pairs, f_pair);
    } else {
      const double* j = reinterpret_cast<const double*>(jac);
      if (it == 1)
        hipLaunchKernelGGL((k_pair_dots4<double, 1, 4>), dim3(b4), blk, 0, st, j, ldj, D, g, ldg,
                           pair_src, n_pairs, f_pair);
      else if (it == 2)
        hipLaunchKernelGGL((k_pair_dots4<double, 2, 2>), dim3(b2), blk, 0, st, j, ldj, D, g, ldg,
                           pair_src, n_pairs, f_pair);
      else
        hipLaunchKernelGGL((k_pair_dots4<double, 4, 1>), dim3(b1), blk, 0, st, j, ldj, D, g, ldg,
                           pair_src, n_pairs, f_pair);
    }
  } else if (n_pairs > 0) {
    const unsigned blocks = (unsigned)std::min<int64_t>((n_pairs + 3) / 4, 65536);
    if (jac_f32)
      hipLaunchKernelGGL(k_pair_dots<float>, dim3(blocks), dim3(256), 0, st,
                         reinterpret_cast<const float*>(jac), ldj, D, g, ldg, pair_src, n_pairs,
                         f_pair);
    else
      hipLaunchKernelGGL(k_pair_dots<double>, dim3(blocks), dim3(256), 0, st,
                         reinterpret_cast<const double*>(jac), ldj, D, g, ldg, pair_src, n_pairs,
                         f_pair);
  }
  hipLaunchKernelGGL(k_gather_forces, dim3(std::min<unsigned>(cdiv(3 * n_atoms, 256), 65536u)),
                     dim3(256), 0, st, f_pair, tgt_ptr, tgt_pair, n_atoms, forces);
}

void jac_transpose_apply_f64(const void* jac, bool jac_f32, int64_t ldj, int64_t D,
                             const int64_t* pair_ptr, const int32_t* pair_j, int64_t n_atoms,
                             int64_t n_pairs, const double* v, double* h, int64_t ldh,
                             hipStream_t st) {
  if (n_atoms <= 0) return;
  dim3 grid(cdiv(n_atoms, 4));
  if (D % 4 == 0 && D >= 4 && D <= 256) {
    if (jac_f32)
      hipLaunchKernelGGL(k_jac_t_apply4<float>, grid, dim3(256), 0, st,
                         reinterpret_cast<const float*>(jac), ldj, D, pair_ptr, pair_j, n_atoms,
                         n_pairs, v, h, ldh);
    else
      hipLaunchKernelGGL(k_jac_t_apply4<double>, grid, dim3(256), 0, st,
                         reinterpret_cast<const double*>(jac), ldj, D, pair_ptr, pair_j, n_atoms,
                         n_pairs, v, h, ldh);
    return;
  }
  if (jac_f32)
    hipLaunchKernelGGL(k_jac_t_apply<float>, grid, dim3(256), 0, st,
                       reinterpret_cast<const float*>(jac), ldj, D, pair_ptr, pair_j, n_atoms,
                       n_pairs, v, h, ldh);
  else
    hipLaunchKernelGGL(k_jac_t_apply<double>, grid, dim3(256), 0, st,
                       reinterpret_cast<const double*>(jac), ldj, D, pair_ptr, pair_j, n_atoms,
                       n_pairs, v, h, ldh);
}

}  // namespace gapk
