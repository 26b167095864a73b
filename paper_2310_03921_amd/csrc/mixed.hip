// Split-BF16 (BF16x3) forms of the descriptor and Jacobian contractions:
// the same outputs as the FP64 kernels (energy rows + kernel-gradient scale,
// force rows, predict P-stage, W X and W^T D), with every D . x and J . x
// product formed on the BF16 matrix cores from hi/lo halves (see mma_bf16.h).
// Kernel scales, pair accumulation and outputs stay in FP64 except the
// per-target accumulation of force rows, which is FP32 (relative 1e-7,
// below the split error).
#include <algorithm>

#include "launch.h"
#include "mma_bf16.h"

namespace gapk {

namespace {

constexpr int kNCb = 4;  // 16-column tiles per wave in the dense BF16x3 kernels

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// ------------------------------------------------------------------ split ----
// X [M][ldx] FP64 -> Xh/Xl [M][ldp] (ldp = D rounded up to 32, zero padded)
// and, when Xth is given, the transposed halves Xth/Xtl [D][ldm] (ldm = M rounded to 32).
__global__ void k_split_x(const double* __restrict__ X, int64_t ldx, int64_t M, int64_t D,
                          __bf16* __restrict__ Xh, __bf16* __restrict__ Xl, int64_t ldp,
                          __bf16* __restrict__ Xth, __bf16* __restrict__ Xtl, int64_t ldm) {
  const int64_t rows = std::max(M, (int64_t)0);
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * ldp;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t m = e / ldp, k = e - m * ldp;
    const float x = (k < D) ? (float)X[m * ldx + k] : 0.f;
    const __bf16 h = (__bf16)x;
    const __bf16 l = (__bf16)(x - (float)h);
    Xh[e] = h;
    Xl[e] = l;
    if (Xth && k < D) {
      Xth[k * ldm + m] = h;
      Xtl[k * ldm + m] = l;
    }
  }
}

__global__ void k_zero_bf16(__bf16* __restrict__ p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (__bf16)0.0f;
}

// --------------------------------------------------------- energy rows ----
// K_E[c][m] = sum over the atoms i of configuration c of delta^2 (d_i . x_m)^zeta
// and the kernel-gradient scale S[i][m] = delta^2 zeta (d_i . x_m)^(zeta-1)
// (FP32), from split-BF16 products.  A block covers one configuration and 256
// columns (wave w: columns 64 w .. + 63, four tiles); a wave takes the
// configuration's atoms 32 at a time (two 16-row fragments that share every X
// fragment), and the next 32-entry block's descriptor entries and X halves
// are loaded while the current block's products run.  Loads in the loop are
// unconditional: rows past the configuration re-read its last atom and
// columns past M re-read column M - 1 (neither is stored); entries past D
// meet the zero padding of the X halves, and the last, partial block of a
// descriptor row takes a guarded load.
template <typename TD>
__global__ __launch_bounds__(256) void k_energy_rows_b3(
    const TD* __restrict__ desc, int64_t ldd, const int64_t* __restrict__ cfg_ptr,
    const __bf16* __restrict__ Xh, const __bf16* __restrict__ Xl, int64_t ldp, int64_t M,
    int64_t D, int zeta, double delta, double* __restrict__ K, int64_t ldk,
    float* __restrict__ S, int64_t ldS, int64_t n_atoms,
    const int32_t* __restrict__ species, int32_t zsel) {
  const int64_t c = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t colbase = (int64_t)blockIdx.x * 256 + wave * 64;
  if (colbase >= M) return;
  const int64_t a0 = max((int64_t)0, min(cfg_ptr[c], n_atoms));
  const int64_t a1 = max(a0, min(cfg_ptr[c + 1], n_atoms));
  const __bf16* xh[kNCb];
  const __bf16* xl[kNCb];
#pragma unroll
  for (int u = 0; u < kNCb; ++u) {
    const int64_t col = min(colbase + u * 16 + idx, M - 1);
    xh[u] = Xh + col * ldp + 8 * g;
    xl[u] = Xl + col * ldp + 8 * g;
  }
  const int64_t nkb = (D + 31) / 32, nfull = D / 32;
  const double d2 = delta * delta, d2z = d2 * zeta;
  double e[kNCb];
#pragma unroll
  for (int u = 0; u < kNCb; ++u) e[u] = 0.0;
  for (int64_t a = a0; a < a1; a += 32) {
    const TD* rowp[2];
    double on_lane[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t row = min(a + 16 * h + idx, a1 - 1);
      rowp[h] = desc + row * ldd + 8 * g;
      // species mask of a per-species block (see the FP64 kernel)
      on_lane[h] = (species == nullptr || species[row] == zsel) ? 1.0 : 0.0;
    }
    auto load_a = [&](int64_t kb, float (&dst)[2][8]) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (kb < nfull)
          load8f_full(rowp[h], kb * 32, dst[h]);
        else
          load8f(rowp[h] - 8 * g, kb * 32 + 8 * g, D, dst[h]);
      }
    };
    auto load_b = [&](int64_t kb, bf8v (&h_)[kNCb], bf8v (&l_)[kNCb]) {
#pragma unroll
      for (int u = 0; u < kNCb; ++u) {
        h_[u] = *reinterpret_cast<const bf8v*>(xh[u] + kb * 32);
        l_[u] = *reinterpret_cast<const bf8v*>(xl[u] + kb * 32);
      }
    };
    f4v acc[2][kNCb];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < kNCb; ++u) acc[h][u] = zero4f();
    float ra[2][8];
    bf8v bh[kNCb], bl[kNCb];
    load_a(0, ra);
    load_b(0, bh, bl);
    for (int64_t kb = 0; kb < nkb; ++kb) {
      bf8v ah[2], al[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) split8(ra[h], ah[h], al[h]);
      bf8v ch[kNCb], cl[kNCb];
#pragma unroll
      for (int u = 0; u < kNCb; ++u) {
        ch[u] = bh[u];
        cl[u] = bl[u];
      }
      const int64_t kn = min(kb + 1, nkb - 1);
      load_a(kn, ra);
      load_b(kn, bh, bl);
#pragma unroll
      for (int u = 0; u < kNCb; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          acc[h][u] = mfma_bf16(ah[h], ch[u], acc[h][u]);
          acc[h][u] = mfma_bf16(ah[h], cl[u], acc[h][u]);
          acc[h][u] = mfma_bf16(al[h], ch[u], acc[h][u]);
        }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int u = 0; u < kNCb; ++u) {
        const int64_t col = colbase + u * 16 + idx;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t rr = a + 16 * h + 4 * g + r;
          const double on = __shfl(on_lane[h], 4 * g + r);
          if (rr < a1) {
            const double p = acc[h][u][r];
            const double pz1 = on * ipow(p, zeta - 1);
            e[u] += d2 * pz1 * p;
            if (col < ldS) S[rr * ldS + col] = (col < M) ? (float)(d2z * pz1) : 0.f;
          }
        }
      }
  }
#pragma unroll
  for (int u = 0; u < kNCb; ++u) {
    double v = e[u];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    const int64_t col = colbase + u * 16 + idx;
    if (g == 0 && col < M) K[c + col * ldk] = v;
  }
}

// ------------------------------------------------------------ force rows ----
// As the FP64 LDS kernel: a block covers 64 targets (four slot groups of 16,
// one per wave) x 16*NCF columns; the split halves of its X columns sit in
// LDS in matrix-core order (per 32-k block, per column tile, per lane: 8 hi
// then 8 lo), so each B fragment pair is one 32-byte LDS read.  Jacobian rows
// are split in registers.  Descriptors longer than one LDS chunk (256
// entries) are taken chunk by chunk: a force row is linear in the pair
// products J . x_m, so every chunk adds S * (J[chunk] . X[chunk]) of every
// pair into the same per-target accumulators.
constexpr int kNCF = 8;       // 128 columns per block
constexpr int kMaxKb32 = 8;   // 256 descriptor entries per LDS chunk

struct SplitPair {
  bf8v h, l;
};

template <typename TJ, int NC>
__global__ __launch_bounds__(256) void k_force_rows_b3(
    const TJ* __restrict__ jac, int64_t ldj, int64_t D, const __bf16* __restrict__ Xh,
    const __bf16* __restrict__ Xl, int64_t ldp, int64_t M, const float* __restrict__ S,
    int64_t ldS, const int64_t* __restrict__ tgt_ptr, const int32_t* __restrict__ tgt_pair,
    const int32_t* __restrict__ pair_src, const int32_t* __restrict__ order, int64_t n_atoms,
    int64_t row0, double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_grp,
    int nkb_all) {
  extern __shared__ SplitPair xs2[];  // [min(nkb_all, kMaxKb32)][NC][64]
  int64_t ct, tgb;
  if (!xcd_group_tile(n_grp, n_ct, tgb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t colbase = ct * (16 * NC);

  const int64_t slot = (tgb * 4 + wave) * 16 + idx;
  const int target = slot < n_atoms ? order[slot] : -1;
  const int64_t seg0 = target >= 0 ? tgt_ptr[target] : 0;
  const int deg = target >= 0 ? (int)(tgt_ptr[target + 1] - seg0) : 0;
  const int maxdeg = wave_max16(deg);
  int64_t colr[NC];
#pragma unroll
  for (int u = 0; u < NC; ++u) colr[u] = colbase + u * 16 + idx;

  f4v acc[3][NC];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int u = 0; u < NC; ++u) acc[a][u] = zero4f();

  const SplitPair* xb = xs2 + lane;
  for (int kc0 = 0; kc0 < nkb_all; kc0 += kMaxKb32) {
  const int nkb = min(kMaxKb32, nkb_all - kc0);
  __syncthreads();  // the previous chunk's products are done with the LDS
  for (int e = threadIdx.x; e < nkb * NC * 64; e += 256) {
    const int kb = e / (NC * 64), rem = e % (NC * 64);
    const int u = rem / 64, ln = rem % 64;
    const int64_t col = colbase + u * 16 + (ln & 15);
    SplitPair sp;
    if (col < M) {
      const int64_t k = (int64_t)(kc0 + kb) * 32 + 8 * (ln >> 4);
      sp.h = *reinterpret_cast<const bf8v*>(Xh + col * ldp + k);
      sp.l = *reinterpret_cast<const bf8v*>(Xl + col * ldp + k);
    } else {
      zero_split(sp.h, sp.l);
    }
    xs2[e] = sp;
  }
  __syncthreads();
  const int64_t k_base = (int64_t)kc0 * 32;
  const int nfull = (int)min((int64_t)nkb, (D - k_base) / 32);  // whole 32-blocks inside D
  for (int t = 0; t < maxdeg; ++t) {
    int pair = t < deg ? tgt_pair[seg0 + t] : -1;
    const int src = pair >= 0 ? pair_src[pair] : -1;
    if (src < 0) pair = -1;
    const bool pv = pair >= 0;
    const TJ* jr = jac + (int64_t)(pv ? pair : 0) * 3 * ldj;
    f4v G[3][NC];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int u = 0; u < NC; ++u) G[a][u] = zero4f();
    float nx[3][8];
    // An absent pair reads pair 0's rows (valid memory, finite values) and is
    // weighted by S = 0 below.  Blocks of 32 entries inside D load with no
    // bound; only the block that D ends in takes the bounded load.
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (nfull > 0)
        load8f_full(jr + a * ldj, k_base + 8 * g, nx[a]);
      else
        load8f(jr + a * ldj, k_base + 8 * g, D, nx[a]);
    }
    for (int kb = 0; kb < nkb; ++kb) {
      bf8v ah[3], al[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) split8(nx[a], ah[a], al[a]);
      if (kb + 1 < nkb) {
        const int64_t kn = k_base + (int64_t)(kb + 1) * 32 + 8 * g;
        if (kb + 1 < nfull) {
#pragma unroll
          for (int a = 0; a < 3; ++a) load8f_full(jr + a * ldj, kn, nx[a]);
        } else {
#pragma unroll
          for (int a = 0; a < 3; ++a) load8f(jr + a * ldj, kn, D, nx[a]);
        }
      }
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const SplitPair b = xb[(kb * NC + u) * 64];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          G[a][u] = mfma_bf16(ah[a], b.h, G[a][u]);
          G[a][u] = mfma_bf16(ah[a], b.l, G[a][u]);
          G[a][u] = mfma_bf16(al[a], b.h, G[a][u]);
        }
      }
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int src_r = __shfl(src, 4 * g + r);
#pragma unroll
      for (int u = 0; u < NC; ++u) {
        const float sv = (src_r >= 0 && colr[u] < M) ? S[(int64_t)src_r * ldS + colr[u]] : 0.f;
#pragma unroll
        for (int a = 0; a < 3; ++a) acc[a][u][r] += sv * G[a][u][r];
      }
    }
  }
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tr = __shfl(target, 4 * g + r);
    if (tr < 0) continue;
#pragma unroll
    for (int u = 0; u < NC; ++u) {
      if (colr[u] >= M) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        K[(row0 + 3 * (int64_t)tr + a) + colr[u] * ldk] = -(double)acc[a][u][r];
    }
  }
}

// BF16x3 force rows for D % 4 == 0 (any length): four waves, each holding 16
// targets (a slot group) for all three components and 128 columns; the split
// X halves of the block's columns are staged through LDS 256 descriptor
// entries at a time (a force row is linear in J . x, so each chunk adds
// S * (J[chunk] . X[chunk]) of every pair into the same per-target
// accumulators).  Every B fragment read from LDS feeds nine matrix-core
// products (three components x three split products), which keeps the LDS
// traffic well below its bandwidth.  The hot loop holds no guarded load (a
// guarded load compiles to a branch whose join waits for it at once):
//  - Jacobian blocks are two 4-wide loads clamped to the row's last four
//    entries; entries past D meet zero-padded X halves;
//  - a slot past its degree re-reads its target's last pair (or pair 0 past
//    n_atoms) and its products are cancelled by a zero weight;
//  - the next step's pair index, source and first Jacobian block, and this
//    step's S values (one 32-byte row segment per source: lane idx of tile u
//    owns column 8 idx + u), are loaded a step or a block ahead of their use.
constexpr int kNCW = 8;  // 16-column tiles per wave and per block: 128 columns

template <typename TJ>
GAP_DEV void jblock8(const TJ* __restrict__ row, int64_t k, int64_t kmax4, float out[8]) {
  const int64_t o0 = min(k, kmax4), o1 = min(k + 4, kmax4);
  if constexpr (sizeof(TJ) == 4) {
    const f4v v0 = *reinterpret_cast<const f4v*>(row + o0);
    const f4v v1 = *reinterpret_cast<const f4v*>(row + o1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      out[s] = v0[s];
      out[4 + s] = v1[s];
    }
  } else {
    const d4v v0 = *reinterpret_cast<const d4v*>(row + o0);
    const d4v v1 = *reinterpret_cast<const d4v*>(row + o1);
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      out[s] = (float)v0[s];
      out[4 + s] = (float)v1[s];
    }
  }
}

// Jacobian source of the wide kernel: FP32 / FP64 rows [3 n_pairs][ld], eight
// entries per lane loaded as two clamped 4-wide loads and split in registers.
// (Rows split once up front and streamed as hi / lo halves ran slower here,
// 6.7 s against 5.1 s on the 576k-atom fit.)
template <typename TJ>
struct JRows {
  const TJ* base;
  int64_t ld, kmax4;
  struct Frag {
    float x[8];
  };
  GAP_DEV int64_t row(int pair) const { return (int64_t)pair * 3 * ld; }
  GAP_DEV void load(int64_t r, int a, int64_t k, Frag& f) const {
    jblock8(base + r + a * ld, k, kmax4, f.x);
  }
  GAP_DEV void ops(const Frag& f, bf8v& h, bf8v& l) const { split8(f.x, h, l); }
};
template <class JS>
__global__ __launch_bounds__(256, 1) void k_force_rows_b3w(
    JS js, int64_t D, const __bf16* __restrict__ Xh, const __bf16* __restrict__ Xl, int64_t ldp,
    int64_t M, const float* __restrict__ S, int64_t ldS, const int64_t* __restrict__ tgt_ptr,
    const int32_t* __restrict__ tgt_pair, const int32_t* __restrict__ pair_src,
    const int32_t* __restrict__ order, int64_t n_atoms, int64_t n_pairs, int64_t row0,
    double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_grp, int nkb_all) {
  // X halves of one chunk: [kb][tile u][hi | lo][64 lanes] of 16 bytes, so each
  // 16-byte LDS read of the wave is contiguous (no bank conflict)
  extern __shared__ bf8v xw[];
  int64_t ct, tgb;
  if (!xcd_group_tile(n_grp, n_ct, tgb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t colbase = ct * (16 * kNCW);
  const int64_t cl0 = colbase + kNCW * idx;     // column of tile u: cl0 + u
  const int64_t scol = min(cl0, ldS - kNCW);    // clamped (valid) S offset
  float colok[kNCW];
#pragma unroll
  for (int u = 0; u < kNCW; ++u) colok[u] = (cl0 + u < M) ? 1.f : 0.f;

  const int64_t slot = (tgb * 4 + wave) * 16 + idx;
  const int target = slot < n_atoms ? order[slot] : -1;
  const int64_t seg0 = target >= 0 ? tgt_ptr[target] : 0;
  const int deg = target >= 0 ? (int)(tgt_ptr[target + 1] - seg0) : 0;
  const int maxdeg = wave_max16(deg);
  const int64_t last = min(seg0 + max(deg - 1, 0), n_pairs - 1);
  auto pair_slot = [&](int t) -> int64_t { return min(seg0 + t, last); };

  f4v acc[3][kNCW];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int u = 0; u < kNCW; ++u) acc[a][u] = zero4f();
  const bf8v* xb = xw + lane;

  for (int kc0 = 0; kc0 < nkb_all; kc0 += kMaxKb32) {
    const int nkb = min(kMaxKb32, nkb_all - kc0);
    __syncthreads();  // the previous chunk's products are done with the LDS
    for (int e = threadIdx.x; e < nkb * kNCW * 64; e += 256) {
      const int kb = e / (kNCW * 64), rem = e % (kNCW * 64);
      const int u = rem / 64, ln = rem % 64;
      const int64_t col = colbase + kNCW * (ln & 15) + u;
      bf8v h, l;
      if (col < M) {
        const int64_t k = (int64_t)(kc0 + kb) * 32 + 8 * (ln >> 4);
        h = *reinterpret_cast<const bf8v*>(Xh + col * ldp + k);
        l = *reinterpret_cast<const bf8v*>(Xl + col * ldp + k);
      } else {
        zero_split(h, l);
      }
      bf8v* t = xw + (size_t)(e >> 6) * 128 + (e & 63);
      t[0] = h;
      t[64] = l;
    }
    __syncthreads();
    if (maxdeg <= 0) continue;
    const int64_t kb0 = (int64_t)kc0 * 32 + 8 * g;  // this lane's first k in the chunk
    // pair metadata one step ahead of its use
    int pair = tgt_pair[pair_slot(0)];
    int pair_n = tgt_pair[pair_slot(1)];
    int src = pair_src[pair];
    int64_t jr = js.row(pair);
    typename JS::Frag nx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) js.load(jr, a, kb0, nx[a]);
    for (int t = 0; t < maxdeg; ++t) {
      const int64_t jn = js.row(pair_n);
      int pair_nn = 0, src_n = 0;
      f4v s_lo[4], s_hi[4];
      f4v G[3][kNCW];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int u = 0; u < kNCW; ++u) G[a][u] = zero4f();
      for (int kb = 0; kb < nkb; ++kb) {
        bf8v ah[3], al[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) js.ops(nx[a], ah[a], al[a]);
        // the next block of this step, or the first block of the next step
        const bool more = kb + 1 < nkb;
        const int64_t rn = more ? jr : jn;
        const int64_t kn = more ? kb0 + (int64_t)(kb + 1) * 32 : kb0;
#pragma unroll
        for (int a = 0; a < 3; ++a) js.load(rn, a, kn, nx[a]);
        if (kb == 0) {
          // S of this step's sources (rows 4 g + r of the output tile), used
          // after the last block, and the pair metadata of the steps ahead:
          // issued behind the first block's Jacobian prefetch, so that the wait
          // for that prefetch (every load before it completes first) does not
          // wait for them as well
          pair_nn = tgt_pair[pair_slot(t + 2)];
          src_n = pair_src[pair_n];
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int src_r = __shfl(src, 4 * g + r);
            const float* sp = S + (int64_t)max(src_r, 0) * ldS + scol;
            s_lo[r] = *reinterpret_cast<const f4v*>(sp);
            s_hi[r] = *reinterpret_cast<const f4v*>(sp + 4);
          }
        }
        __builtin_amdgcn_sched_barrier(0);  // issue these loads before the products
        // X halves one tile ahead of their products, so that each tile's LDS
        // reads are in flight under the previous tile's nine products
        const bf8v* xk = xb + (size_t)kb * kNCW * 128;
        bf8v bh = xk[0], bl = xk[64];
#pragma unroll
        for (int u = 0; u < kNCW; ++u) {
          bf8v nh = bh, nl = bl;
          if (u + 1 < kNCW) {
            nh = xk[(u + 1) * 128];
            nl = xk[(u + 1) * 128 + 64];
          }
#pragma unroll
          for (int a = 0; a < 3; ++a) {
            G[a][u] = mfma_bf16(ah[a], bh, G[a][u]);
            G[a][u] = mfma_bf16(ah[a], bl, G[a][u]);
            G[a][u] = mfma_bf16(al[a], bh, G[a][u]);
          }
          bh = nh;
          bl = nl;
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src_r = __shfl(src, 4 * g + r);
        const int deg_r = __shfl(deg, 4 * g + r);
        const float ok = (t < deg_r && src_r >= 0) ? 1.f : 0.f;
#pragma unroll
        for (int u = 0; u < kNCW; ++u) {
          const float sv = (u < 4 ? s_lo[r][u & 3] : s_hi[r][u & 3]) * (ok * colok[u]);
#pragma unroll
          for (int a = 0; a < 3; ++a) acc[a][u][r] += sv * G[a][u][r];
        }
      }
      jr = jn;
      pair_n = pair_nn;
      src = src_n;
    }
  }

#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tr = __shfl(target, 4 * g + r);
    if (tr < 0) continue;
#pragma unroll
    for (int u = 0; u < kNCW; ++u) {
      if (cl0 + u >= M) continue;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        K[(row0 + 3 * (int64_t)tr + a) + (cl0 + u) * ldk] = -(double)acc[a][u][r];
    }
  }
}

template <class JS>
void launch_b3w(JS js, int64_t D, const __bf16* Xh, const __bf16* Xl, int64_t ldp, int64_t M,
                const float* S, int64_t ldS, const int64_t* tgt_ptr, const int32_t* tgt_pair,
                const int32_t* pair_src, const int32_t* order, int64_t n_atoms, int64_t n_pairs,
                int64_t row0, double* K, int64_t ldk, hipStream_t st) {
  const int nkb = (int)(ldp / 32);
  const int64_t n_tgb = (n_atoms + 63) / 64;
  const int64_t n_ct = (M + 16 * kNCW - 1) / (16 * kNCW);
  const unsigned blocks = xcd_group_tile_blocks(n_tgb, n_ct);
  const size_t lds = (size_t)std::min(nkb, kMaxKb32) * kNCW * 128 * sizeof(bf8v);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_force_rows_b3w<JS>),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((size_t)kMaxKb32 * kNCW * 128 * sizeof(bf8v)));
    attr = true;
  }
  hipLaunchKernelGGL((k_force_rows_b3w<JS>), dim3(blocks), dim3(256), lds, st, js, D, Xh, Xl, ldp,
                     M, S, ldS, tgt_ptr, tgt_pair, pair_src, order, n_atoms, n_pairs, row0, K, ldk,
                     n_ct, n_tgb, nkb);
}

// Jacobian rows split once into hi/lo halves, [n_pairs][3][ldp] each (ldp = D
// rounded up to 32, zero padded), so the force-row kernel streams 4 bytes per
// element and does no splitting in its inner loop.
template <typename TJ>
__global__ void k_split_j(const TJ* __restrict__ J, int64_t ldj, int64_t rows, int64_t D,
                          __bf16* __restrict__ Jh, __bf16* __restrict__ Jl, int64_t ldp) {
  const int64_t per_row = ldp / 8;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * per_row;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / per_row, k = (e - r * per_row) * 8;
    float x[8];
    load8f(J + r * ldj, k, D, x);
    bf8v h, l;
    split8(x, h, l);
    *reinterpret_cast<bf8v*>(Jh + r * ldp + k) = h;
    *reinterpret_cast<bf8v*>(Jl + r * ldp + k) = l;
  }
}

// Twelve-wave BF16x3 force rows on pre-split Jacobians: wave w handles
// component alpha = w % 3 of slot group w / 3 (16 targets), 128 columns whose
// split X halves sit in LDS in matrix-core order.  Pair metadata, the next
// pair's first Jacobian block and the S values of the current step are
// fetched ahead, as in the FP64 form.
template <int NKB>
__global__ __launch_bounds__(768) void k_force_rows_b3s(
    const __bf16* __restrict__ Jh, const __bf16* __restrict__ Jl, int64_t ldp, int64_t D,
    const __bf16* __restrict__ Xh, const __bf16* __restrict__ Xl, int64_t M,
    const float* __restrict__ S, int64_t ldS, const int64_t* __restrict__ tgt_ptr,
    const int32_t* __restrict__ tgt_pair, const int32_t* __restrict__ pair_src,
    const int32_t* __restrict__ order, int64_t n_atoms, int64_t n_pairs, int64_t row0,
    double* __restrict__ K, int64_t ldk, int64_t n_ct, int64_t n_grp) {
  constexpr int nkb = NKB;  // 32-deep k blocks (compile time: straight-line, exact waits)
  // No guarded load on the hot path (a guarded load compiles to a branch whose
  // join waits for it at once): every load reads a valid address, and invalid
  // steps are cancelled by a zero S factor.  A slot past its degree (or a
  // target past n_atoms) re-reads a valid pair of its target (or pair 0); the
  // split Jacobian rows are zero-padded to ldp, so no k clamp is needed.  Lane
  // idx of column tile u owns column 8 idx + u, so a lane's eight S values for
  // one source are 32 contiguous bytes (S rows zero-padded to ldS).
  // X halves in LDS: [nkb][kNCF][hi | lo][64 lanes] of 16 bytes, so each 16-byte
  // LDS read of the wave is contiguous (no bank conflict)
  extern __shared__ SplitPair xs3[];
  int64_t ct, tgb;
  if (!xcd_group_tile(n_grp, n_ct, tgb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int alpha = wave % 3, grp = wave / 3;
  const int64_t colbase = ct * (16 * kNCF);
  for (int e = threadIdx.x; e < nkb * kNCF * 64; e += 768) {
    const int kb = e / (kNCF * 64), rem = e % (kNCF * 64);
    const int u = rem / 64, ln = rem % 64;
    const int64_t col = colbase + kNCF * (ln & 15) + u;
    SplitPair sp;
    if (col < M) {
      const int64_t k = (int64_t)kb * 32 + 8 * (ln >> 4);
      sp.h = *reinterpret_cast<const bf8v*>(Xh + col * ldp + k);
      sp.l = *reinterpret_cast<const bf8v*>(Xl + col * ldp + k);
    } else {
      zero_split(sp.h, sp.l);
    }
    bf8v* t = reinterpret_cast<bf8v*>(xs3) + (size_t)(e >> 6) * 128 + (e & 63);
    t[0] = sp.h;
    t[64] = sp.l;
  }
  __syncthreads();
  const int64_t slot = (tgb * 4 + grp) * 16 + idx;
  const int target = slot < n_atoms ? order[slot] : -1;
  const int64_t seg0 = target >= 0 ? tgt_ptr[target] : 0;
  const int deg = target >= 0 ? (int)(tgt_ptr[target + 1] - seg0) : 0;
  const int maxdeg = wave_max16(deg);
  const int64_t last = min(seg0 + max(deg - 1, 0), n_pairs - 1);
  auto pair_slot = [&](int t) -> int64_t { return min(seg0 + t, last); };
  auto rowoff = [&](int p) -> int64_t { return ((int64_t)p * 3 + alpha) * ldp + 8 * g; };
  const int64_t cl0 = colbase + kNCF * idx;           // first column of this lane
  const int64_t scol = min(cl0, ldS - kNCF);          // clamped (valid) S offset
  f4v acc[kNCF];
#pragma unroll
  for (int u = 0; u < kNCF; ++u) acc[u] = zero4f();
  const bf8v* xb = reinterpret_cast<const bf8v*>(xs3) + lane;
  if (maxdeg > 0) {
    // pair metadata one step ahead of its use
    int pair = tgt_pair[pair_slot(0)];
    int pair_n = tgt_pair[pair_slot(1)];
    int src = pair_src[pair];
    int64_t ro = rowoff(pair);
    bf8v ah = *reinterpret_cast<const bf8v*>(Jh + ro);
    bf8v al = *reinterpret_cast<const bf8v*>(Jl + ro);
    for (int t = 0; t < maxdeg; ++t) {
      const int pair_nn = tgt_pair[pair_slot(t + 2)];
      const int src_n = pair_src[pair_n];
      const int64_t ro_n = rowoff(pair_n);
      // S of this step's sources (rows 4 g + r of the output tile)
      f4v s_lo[4], s_hi[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src_r = __shfl(src, 4 * g + r);
        const float* sp = S + (int64_t)max(src_r, 0) * ldS + scol;
        s_lo[r] = *reinterpret_cast<const f4v*>(sp);
        s_hi[r] = *reinterpret_cast<const f4v*>(sp + 4);
      }
      f4v G[kNCF];
#pragma unroll
      for (int u = 0; u < kNCF; ++u) G[u] = zero4f();
#pragma unroll 1
      for (int kb = 0; kb < nkb; ++kb) {
        const int64_t nro = (kb + 1 < nkb) ? ro + (int64_t)(kb + 1) * 32 : ro_n;
        const bf8v nh = *reinterpret_cast<const bf8v*>(Jh + nro);
        const bf8v nl = *reinterpret_cast<const bf8v*>(Jl + nro);
#pragma unroll
        for (int u = 0; u < kNCF; ++u) {
          const bf8v bh = xb[(kb * kNCF + u) * 128], bl = xb[(kb * kNCF + u) * 128 + 64];
          G[u] = mfma_bf16(ah, bh, G[u]);
          G[u] = mfma_bf16(ah, bl, G[u]);
          G[u] = mfma_bf16(al, bh, G[u]);
        }
        ah = nh;
        al = nl;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int src_r = __shfl(src, 4 * g + r);
        const int deg_r = __shfl(deg, 4 * g + r);
        const float ok = (t < deg_r && src_r >= 0) ? 1.f : 0.f;
#pragma unroll
        for (int u = 0; u < kNCF; ++u) {
          const float sv = (u < 4 ? s_lo[r][u & 3] : s_hi[r][u & 3]) *
                           ((cl0 + u < M) ? ok : 0.f);
          acc[u][r] += sv * G[u][r];
        }
      }
      ro = ro_n;
      pair_n = pair_nn;
      src = src_n;
    }
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int tr = __shfl(target, 4 * g + r);
    if (tr < 0) continue;
#pragma unroll
    for (int u = 0; u < kNCF; ++u)
      if (cl0 + u < M) K[(row0 + 3 * (int64_t)tr + alpha) + (cl0 + u) * ldk] = -(double)acc[u][r];
  }
}

template <typename T>
inline const T* tp(const void* p) {
  return reinterpret_cast<const T*>(p);
}

}  // namespace

int64_t split_ld(int64_t n) { return (n + 31) / 32 * 32; }

void split_x_bf16(const double* X, int64_t ldx, int64_t M, int64_t D, __bf16* Xh, __bf16* Xl,
                  __bf16* Xth, __bf16* Xtl, hipStream_t st) {
  const int64_t ldp = split_ld(D), ldm = split_ld(M);
  if (Xth) {
    const int64_t nt = D * ldm;
    const unsigned gz = std::max(1u, std::min(cdiv(nt, 256), 65536u));
    hipLaunchKernelGGL(k_zero_bf16, dim3(gz), dim3(256), 0, st, Xth, nt);
    hipLaunchKernelGGL(k_zero_bf16, dim3(gz), dim3(256), 0, st, Xtl, nt);
  }
  const unsigned g = std::max(1u, std::min(cdiv(M * ldp, 256), 65536u));
  hipLaunchKernelGGL(k_split_x, dim3(g), dim3(256), 0, st, X, ldx, M, D, Xh, Xl, ldp, Xth, Xtl,
                     ldm);
}

void energy_rows_bf16x3(const void* desc, bool desc_f32, int64_t ldd, const int64_t* cfg_ptr,
                        int64_t n_cfg, int64_t n_atoms, const __bf16* Xh, const __bf16* Xl,
                        int64_t M, int64_t D, int zeta, double delta, double* K, int64_t ldk,
                        float* S, int64_t ldS, hipStream_t st, const int32_t* species,
                        int32_t zsel) {
  if (n_cfg <= 0 || M <= 0) return;
  const int64_t ldp = split_ld(D);
  dim3 grid(cdiv(M, 256), (unsigned)n_cfg);
  if (desc_f32)
    hipLaunchKernelGGL(k_energy_rows_b3<float>, grid, dim3(256), 0, st, tp<float>(desc), ldd,
                       cfg_ptr, Xh, Xl, ldp, M, D, zeta, delta, K, ldk, S, ldS, n_atoms, species,
                       zsel);
  else
    hipLaunchKernelGGL(k_energy_rows_b3<double>, grid, dim3(256), 0, st, tp<double>(desc), ldd,
                       cfg_ptr, Xh, Xl, ldp, M, D, zeta, delta, K, ldk, S, ldS, n_atoms, species,
                       zsel);
}

void force_rows_bf16x3(const void* jac, bool jac_f32, int64_t ldj, int64_t D, const __bf16* Xh,
                       const __bf16* Xl, int64_t M, const float* S, int64_t ldS,
                       const int64_t* tgt_ptr, const int32_t* tgt_pair, const int32_t* pair_src,
                       const int32_t* order, int64_t n_atoms, int64_t n_pairs, int64_t row0,
                       double* K, int64_t ldk, hipStream_t st) {
  if (n_atoms <= 0 || M <= 0) return;
  const int64_t ldp = split_ld(D);
  const int64_t n_tgb = (n_atoms + 63) / 64;
  const int nkb = (int)(ldp / 32);
  if (D % 4 == 0 && D >= 4 && n_pairs > 0 && ldj % 4 == 0 && ldS % 8 == 0 && ldS >= 8) {
    if (jac_f32)
      launch_b3w(JRows<float>{tp<float>(jac), ldj, D - 4}, D, Xh, Xl, ldp, M, S, ldS, tgt_ptr,
                 tgt_pair, pair_src, order, n_atoms, n_pairs, row0, K, ldk, st);
    else
      launch_b3w(JRows<double>{tp<double>(jac), ldj, D - 4}, D, Xh, Xl, ldp, M, S, ldS, tgt_ptr,
                 tgt_pair, pair_src, order, n_atoms, n_pairs, row0, K, ldk, st);
    return;
  }
  // Up to 256 descriptor entries: 128 columns per block.  Longer descriptors:
  // 64 columns per block (half the accumulators), so that two waves share a
  // SIMD and cover each other's Jacobian loads.
  const int nc = nkb <= kMaxKb32 ? 8 : 4;
  const int64_t n_ct = (M + 16 * nc - 1) / (16 * nc);
  const unsigned blocks = xcd_group_tile_blocks(n_tgb, n_ct);
  const size_t lds = (size_t)std::min(nkb, kMaxKb32) * nc * 64 * sizeof(SplitPair);
  const int lds_max = (int)((size_t)kMaxKb32 * nc * 64 * sizeof(SplitPair));
  auto prep = [&](const void* kern, bool& done) {
    if (!done) {
      (void)hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max);
      done = true;
    }
  };
  static bool f8 = false, f4 = false, d8 = false, d4 = false;
  if (jac_f32 && nc == 8) {
    prep(reinterpret_cast<const void*>(&k_force_rows_b3<float, 8>), f8);
    hipLaunchKernelGGL((k_force_rows_b3<float, 8>), dim3(blocks), dim3(256), lds, st,
                       tp<float>(jac), ldj, D, Xh, Xl, ldp, M, S, ldS, tgt_ptr, tgt_pair,
                       pair_src, order, n_atoms, row0, K, ldk, n_ct, n_tgb, nkb);
  } else if (jac_f32) {
    prep(reinterpret_cast<const void*>(&k_force_rows_b3<float, 4>), f4);
    hipLaunchKernelGGL((k_force_rows_b3<float, 4>), dim3(blocks), dim3(256), lds, st,
                       tp<float>(jac), ldj, D, Xh, Xl, ldp, M, S, ldS, tgt_ptr, tgt_pair,
                       pair_src, order, n_atoms, row0, K, ldk, n_ct, n_tgb, nkb);
  } else if (nc == 8) {
    prep(reinterpret_cast<const void*>(&k_force_rows_b3<double, 8>), d8);
    hipLaunchKernelGGL((k_force_rows_b3<double, 8>), dim3(blocks), dim3(256), lds, st,
                       tp<double>(jac), ldj, D, Xh, Xl, ldp, M, S, ldS, tgt_ptr, tgt_pair,
                       pair_src, order, n_atoms, row0, K, ldk, n_ct, n_tgb, nkb);
  } else {
    prep(reinterpret_cast<const void*>(&k_force_rows_b3<double, 4>), d4);
    hipLaunchKernelGGL((k_force_rows_b3<double, 4>), dim3(blocks), dim3(256), lds, st,
                       tp<double>(jac), ldj, D, Xh, Xl, ldp, M, S, ldS, tgt_ptr, tgt_pair,
                       pair_src, order, n_atoms, row0, K, ldk, n_ct, n_tgb, nkb);
  }
}

void split_j_bf16(const void* jac, bool jac_f32, int64_t ldj, int64_t n_pairs, int64_t D,
                  __bf16* Jh, __bf16* Jl, hipStream_t st) {
  split_rows_bf16(jac, jac_f32, ldj, 3 * n_pairs, D, Jh, Jl, st);
}

void split_rows_bf16(const void* jac, bool jac_f32, int64_t ldj, int64_t rows, int64_t D,
                     __bf16* Jh, __bf16* Jl, hipStream_t st) {
  if (rows <= 0) return;
  const int64_t ldp = split_ld(D);
  const unsigned g = std::max(1u, std::min(cdiv(rows * (ldp / 8), 256), 65536u));
  if (jac_f32)
    hipLaunchKernelGGL(k_split_j<float>, dim3(g), dim3(256), 0, st, tp<float>(jac), ldj, rows, D,
                       Jh, Jl, ldp);
  else
    hipLaunchKernelGGL(k_split_j<double>, dim3(g), dim3(256), 0, st, tp<double>(jac), ldj, rows, D,
                       Jh, Jl, ldp);
}

bool force_rows_bf16x3_split(const __bf16* Jh, const __bf16* Jl, int64_t D, const __bf16* Xh,
                             const __bf16* Xl, int64_t M, const float* S, int64_t ldS,
                             const int64_t* tgt_ptr, const int32_t* tgt_pair,
                             const int32_t* pair_src, const int32_t* order, int64_t n_atoms,
                             int64_t n_pairs, int64_t row0, double* K, int64_t ldk,
                             hipStream_t st) {
  if (n_atoms <= 0 || M <= 0) return true;
  if (D > 32 * kMaxKb32 || n_pairs <= 0 || ldS % 8 != 0 || ldS < 8) return false;
  const int64_t ldp = split_ld(D);
  const int nkb = (int)(ldp / 32);
  const int64_t n_tgb = (n_atoms + 63) / 64;
  const int64_t n_ct = (M + 16 * kNCF - 1) / (16 * kNCF);
  const unsigned blocks = xcd_group_tile_blocks(n_tgb, n_ct);
  const size_t lds = (size_t)nkb * kNCF * 64 * sizeof(SplitPair);
  auto launch = [&](auto kern) {
    static bool attr[kMaxKb32 + 1] = {};
    if (!attr[nkb]) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)((size_t)kMaxKb32 * kNCF * 64 * sizeof(SplitPair)));
      attr[nkb] = true;
    }
    hipLaunchKernelGGL(kern, dim3(blocks), dim3(768), lds, st, Jh, Jl, ldp, D, Xh,
                       Xl, M, S, ldS, tgt_ptr, tgt_pair, pair_src, order, n_atoms, n_pairs, row0,
                       K, ldk, n_ct, n_tgb);
  };
  switch (nkb) {
    case 1: launch(k_force_rows_b3s<1>); break;
    case 2: launch(k_force_rows_b3s<2>); break;
    case 3: launch(k_force_rows_b3s<3>); break;
    case 4: launch(k_force_rows_b3s<4>); break;
    case 5: launch(k_force_rows_b3s<5>); break;
    case 6: launch(k_force_rows_b3s<6>); break;
    case 7: launch(k_force_rows_b3s<7>); break;
    case 8: launch(k_force_rows_b3s<8>); break;
    default: return false;
  }
  return true;
}




}  // namespace gapk
