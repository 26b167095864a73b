// Tiled BF16x3 GEMM for the predict and backward contractions (eq. epsilon and
// its derivatives): C[i][j] = sum_k A[i][k] B[j][k], both operands K-contiguous,
// every value split hi = bf16(fp32(x)), lo = bf16(fp32(x) - hi) while it is
// staged into LDS, products hi*hi + hi*lo + lo*hi on the BF16 matrix cores with
// FP32 accumulation (see mma_bf16.h).
//
// A block computes a 256 x 256 tile of C with eight waves (64 x 128 each: four
// A and eight B fragments, thirty-two accumulators), over 32-deep k blocks
// whose split A and B halves are double-buffered in LDS in matrix-core operand
// order (128 KB); the next k block is loaded into registers while the current
// one feeds the matrix cores.  A 256-wide tile moves 64 bytes of operands per
// 768 BF16 flop (12,288 per k block and thread pair), so at the matrix cores'
// rate the operand stream from L2 stays near 15 TB/s for the whole chip; a
// 128-wide tile would need twice that.
//
// Epilogues:
//   kPlain   C (FP64, row-major), or a split-K partial C + z * zstride;
//   kPEnergy P-stage of predict: P = D X^T, e_part[ct][i] = sum over the
//            columns of column tile ct of c_m k(p_im), W[i][m] = delta^2 zeta c_m p^(zeta-1)
//            (FP32, the forward W, whose product with X is the descriptor gradient);
//   kPBack   P-stage of the backward: dc_part[rt][m] = sum over the rows of row tile rt of
//            g_e[i] k(p_im), W[i][m] = g_e[i] delta^2 zeta c_m p^(zeta-1) (FP32).
// An operand may also be a column view (ColOp: element (r, k) at p[k ld + r]),
// which the backward's d_X = W^T D uses for both W and the descriptors, so that
// neither is transposed in memory.
#include <algorithm>
#include <type_traits>

#include "launch.h"
#include "mma_bf16.h"

namespace gapk {

namespace {

constexpr int kGT = 256;            // tile rows and columns
constexpr int kGThreads = 512;      // eight waves: 4 (64-row quarters) x 2 (128-column halves)
constexpr int kGStage = kGT * 32;   // elements of one operand per k block
constexpr int kGStageV = kGStage / 8 * 2;   // 16-byte LDS entries of one split block
constexpr int kGLds = 4 * kGStageV * 16;   // dynamic LDS bytes of a block (128 KB)
constexpr int kGRowStep = kGThreads / 4;   // rows between a thread's two staged rows
constexpr int kPlain = 0, kPEnergy = 1, kPBack = 2;

inline unsigned cdiv_u(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Staging of a 256 x 32 operand block.  The next block's loads are issued
// before the current block's products and their registers are read only when
// the block is written to LDS after them, so the products never wait for
// memory: a load fetches raw values from a clamped, valid address, and what
// lies outside the operand (rows past its end, k past the slice end) is
// replaced by zeros, by selection, only when the block is staged, where the
// values are also converted to FP32 and split into 16-byte hi / lo halves at
// [tile][hi | lo][lane] (lane = row % 16 + 16 group).
template <typename TOp>
struct Stage;

// Thread t of a row operand stages row 16 (t / 64) + t % 16 (+ 128 h) and k
// group (t / 16) % 4: the 64 lanes of a wave then write 64 consecutive
// 16-byte LDS entries, where four lanes of one row with consecutive k groups
// would meet in the same banks four at a time.
GAP_DEV int stage_row(int t) { return 16 * (t >> 6) + (t & 15); }
GAP_DEV int stage_grp(int t) { return (t >> 4) & 3; }

// Rows (element (r, k) at p[r ld + k], ld a multiple of 4): thread t holds rows
// stage_row(t) + 128 h, entries k0 + 8 stage_grp(t) .. + 7, as two 4-wide loads whose
// start is clamped to the last 4-group that holds entries below K.
template <typename T>
struct Stage<const T*> {
  T v[2][8];
  GAP_DEV void load(const T* __restrict__ p, int64_t ld, int64_t rows, int64_t K, int64_t r0,
                    int64_t k0) {
    const int t = threadIdx.x, grp = stage_grp(t);
    const int64_t k4 = (K - 1) & ~(int64_t)3;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const T* row = p + min(r0 + stage_row(t) + kGRowStep * h, rows - 1) * ld;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int64_t kk = min(k0 + 8 * grp + 4 * q, k4);
        if constexpr (sizeof(T) == 4) {
          const f4v x = *reinterpret_cast<const f4v*>(row + kk);
#pragma unroll
          for (int e = 0; e < 4; ++e) v[h][4 * q + e] = x[e];
        } else {
          const d4v x = *reinterpret_cast<const d4v*>(row + kk);
#pragma unroll
          for (int e = 0; e < 4; ++e) v[h][4 * q + e] = x[e];
        }
      }
    }
  }
  GAP_DEV void store(int64_t rows, int64_t K, int64_t r0, int64_t k0,
                     bf8v* __restrict__ dst) const {
    const int t = threadIdx.x, grp = stage_grp(t);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = stage_row(t) + kGRowStep * h;
      const bool rok = r0 + r < rows;
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (rok && k0 + 8 * grp + e < K) ? (float)v[h][e] : 0.f;
      bf8v hi, lo;
      split8(x, hi, lo);
      bf8v* d = dst + (r >> 4) * 128 + (r & 15) + 16 * grp;
      d[0] = hi;
      d[64] = lo;
    }
  }
};

// Pre-split operand rows: hi and lo halves [rows][ld], ld a multiple of 32,
// zero padded along k; 16-byte loads of both halves, no split.
struct SplitRows {
  const __bf16* hi;
  const __bf16* lo;
};
template <>
struct Stage<SplitRows> {
  bf8v hi[2], lo[2];
  GAP_DEV void load(const SplitRows& s, int64_t ld, int64_t rows, int64_t K, int64_t r0,
                    int64_t k0) {
    const int t = threadIdx.x, grp = stage_grp(t);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t off = min(r0 + stage_row(t) + kGRowStep * h, rows - 1) * ld + k0 + 8 * grp;
      hi[h] = *reinterpret_cast<const bf8v*>(s.hi + off);
      lo[h] = *reinterpret_cast<const bf8v*>(s.lo + off);
    }
  }
  GAP_DEV void store(int64_t rows, int64_t K, int64_t r0, int64_t k0,
                     bf8v* __restrict__ dst) const {
    const int t = threadIdx.x, grp = stage_grp(t);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = stage_row(t) + kGRowStep * h;
      bf8v a = hi[h], b = lo[h];
      if (r0 + r >= rows) zero_split(a, b);
      bf8v* d = dst + (r >> 4) * 128 + (r & 15) + 16 * grp;
      d[0] = a;
      d[64] = b;
    }
  }
};

// Column view of a row-major matrix: element (r, k) at p[k * ld + r].  Thread t
// holds rows (t & 127) + 128 h and k group 8 (t >> 7) .. + 7, one load per k,
// so that for a given k a wave's lanes read 64 consecutive r (whole 256-byte
// runs for FP32); the block lands in the same LDS places as a row operand's.
template <typename T>
struct ColOp {
  const T* p;
};
template <typename T>
struct Stage<ColOp<T>> {
  T v[2][8];
  GAP_DEV void load(const ColOp<T>& op, int64_t ld, int64_t rows, int64_t K, int64_t r0,
                    int64_t k0) {
    const int t = threadIdx.x, grp = t >> 7;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t rc = min(r0 + (t & 127) + kGRowStep * h, rows - 1);
#pragma unroll
      for (int e = 0; e < 8; ++e) v[h][e] = op.p[min(k0 + 8 * grp + e, K - 1) * ld + rc];
    }
  }
  GAP_DEV void store(int64_t rows, int64_t K, int64_t r0, int64_t k0,
                     bf8v* __restrict__ dst) const {
    const int t = threadIdx.x, grp = t >> 7;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int r = (t & 127) + kGRowStep * h;
      const bool rok = r0 + r < rows;
      float x[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) x[e] = (rok && k0 + 8 * grp + e < K) ? (float)v[h][e] : 0.f;
      bf8v hi, lo;
      split8(x, hi, lo);
      bf8v* d = dst + (r >> 4) * 128 + (r & 15) + 16 * grp;
      d[0] = hi;
      d[64] = lo;
    }
  }
};

struct EpiArgs {
  int zeta;
  double delta;
  const double* c;      // [n_b] coefficients (P-stages)
  const double* g_e;    // [n_a] upstream gradient (backward P-stage)
  float* W;             // [n_a][ldw]
  int64_t ldw;
  double* e_part;       // [column tiles][n_a]
  double* dc_part;      // [row tiles][n_b]
  double* C;            // plain: [n_a][ldc] (+ z * zstride)
  int64_t ldc;
  int64_t zstride;
};

template <typename TA, typename TB, int EPI>
__global__ __launch_bounds__(kGThreads, 1) void k_gemm_b3(TA A, int64_t lda, int64_t n_a, TB B,
                                                          int64_t ldb, int64_t n_b, int64_t K,
                                                          int64_t k_per_z, EpiArgs ep) {
  // split operand blocks, double-buffered: [A | B][buf][8 tiles x (hi | lo) x 64 lanes]
  extern __shared__ bf8v smem[];
  auto sA = [&](int buf) { return smem + buf * kGStageV; };
  auto sB = [&](int buf) { return smem + (2 + buf) * kGStageV; };
  __shared__ double red[4][kGT];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wr = wave & 3, wc = wave >> 2;   // 64-row quarter and 128-column half of the tile
  // tiles dealt by row tile: all column tiles of a row tile run on one XCD,
  // where they share the row tile's A rows in L2
  int64_t rt, ct;
  if (!xcd_group_tile((n_a + kGT - 1) / kGT, (n_b + kGT - 1) / kGT, rt, ct)) return;
  const int64_t i0 = rt * kGT, j0 = ct * kGT;
  const int64_t kz0 = (int64_t)blockIdx.y * k_per_z;
  const int64_t kz1 = min(K, kz0 + k_per_z);
  const int nkb = (int)((kz1 - kz0 + 31) / 32);

  f4v acc[4][8];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 8; ++b) acc[a][b] = zero4f();

  Stage<TA> sa;
  Stage<TB> sb;
  if (nkb > 0) {
    sa.load(A, lda, n_a, kz1, i0, kz0);
    sb.load(B, ldb, n_b, kz1, j0, kz0);
    sa.store(n_a, kz1, i0, kz0, sA(0));
    sb.store(n_b, kz1, j0, kz0, sB(0));
  }
  __syncthreads();
  for (int kb = 0; kb < nkb; ++kb) {
    const int buf = kb & 1;
    const bool more = kb + 1 < nkb;
    const int64_t kn = kz0 + (int64_t)(kb + 1) * 32;
    if (more) {
      sa.load(A, lda, n_a, kz1, i0, kn);
      sb.load(B, ldb, n_b, kz1, j0, kn);
    }
    __builtin_amdgcn_sched_barrier(0);
    const bf8v* xa = sA(buf) + lane + wr * 4 * 128;
    const bf8v* xb = sB(buf) + lane + wc * 8 * 128;
    bf8v ah[4], al[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      ah[a] = xa[a * 128];
      al[a] = xa[a * 128 + 64];
    }
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bf8v bh = xb[b * 128], bl = xb[b * 128 + 64];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        acc[a][b] = mfma_bf16(ah[a], bh, acc[a][b]);
        acc[a][b] = mfma_bf16(ah[a], bl, acc[a][b]);
        acc[a][b] = mfma_bf16(al[a], bh, acc[a][b]);
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (more) {
      sa.store(n_a, kz1, i0, kn, sA(buf ^ 1));
      sb.store(n_b, kz1, j0, kn, sB(buf ^ 1));
    }
    __syncthreads();
  }

  // C[4 g + r][idx] of fragment (a, b): row i0 + 64 wr + 16 a + 4 g + r,
  // column j0 + 128 wc + 16 b + idx
  if constexpr (EPI == kPlain) {
    double* C = ep.C + blockIdx.y * ep.zstride;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 64 * wr + 16 * a + 4 * g + r;
        if (i >= n_a) continue;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int64_t j = j0 + 128 * wc + 16 * b + idx;
          if (j < n_b) C[i * ep.ldc + j] = (double)acc[a][b][r];
        }
      }
  } else {
    // The element-wise arithmetic runs in FP32: p is an FP32 accumulation of the
    // split products and W is stored in FP32, so FP64 here would only cost
    // VALU time while the matrix cores idle; each lane's partial sums over
    // its own entries are FP32, and everything past them (lanes, halves,
    // tiles) is summed in FP64.
    const float d2 = (float)(ep.delta * ep.delta);
    const int zm1 = ep.zeta - 1;
    float cf[8], cw[8];   // c_m and delta^2 zeta c_m of this lane's columns
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const int64_t j = j0 + 128 * wc + 16 * b + idx;
      const double cj = j < n_b ? ep.c[j] : 0.0;
      cf[b] = (float)cj;
      cw[b] = (float)(ep.delta * ep.delta * ep.zeta * cj);
    }
    // g_e of the wave's 64 rows, one per lane, loaded ahead of every W store
    // (the stores could alias g_e as far as the compiler knows, and a load
    // issued behind them would wait for all of them to complete); row
    // 16 a + 4 g + r of the quarter is read from its lane by a shuffle
    float ge_lane = 1.f;
    if (EPI == kPBack && i0 + 64 * wr + lane < n_a) ge_lane = (float)ep.g_e[i0 + 64 * wr + lane];
    double rowsum[4][4];   // kPEnergy: [a][r] partial row sums over this lane's columns
    float colsum[8];       // kPBack: [b] partial column sums over this lane's rows
#pragma unroll
    for (int b = 0; b < 8; ++b) colsum[b] = 0.f;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      // p^(zeta-1) of the 32 entries of fragment row a: one walk over the
      // exponent's bits serves all of them
      float pw[8][4], x[8][4];
#pragma unroll
      for (int b = 0; b < 8; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          pw[b][r] = 1.f;
          x[b][r] = acc[a][b][r];
        }
      for (int e = zm1; e > 0; e >>= 1) {
        if (e & 1) {
#pragma unroll
          for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) pw[b][r] *= x[b][r];
        }
        if (e > 1) {
#pragma unroll
          for (int b = 0; b < 8; ++b)
#pragma unroll
            for (int r = 0; r < 4; ++r) x[b][r] *= x[b][r];
        }
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 64 * wr + 16 * a + 4 * g + r;
        const bool iv = i < n_a;
        float* wrow = ep.W + (iv ? i : 0) * ep.ldw + j0 + 128 * wc + idx;
        const float ge = EPI == kPBack ? __shfl(ge_lane, 16 * a + 4 * g + r) : 1.f;
        float rs = 0.f;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const float pz1 = pw[b][r];
          const float kv = d2 * pz1 * acc[a][b][r];
          if (iv && j0 + 128 * wc + 16 * b + idx < n_b) {
            if (EPI == kPEnergy) rs += cf[b] * kv;
            if (EPI == kPBack) colsum[b] += ge * kv;
            wrow[16 * b] = ge * cw[b] * pz1;
          }
        }
        rowsum[a][r] = rs;
      }
    }
    if constexpr (EPI == kPEnergy) {
      // row sums over the 16 columns of each fragment (lanes idx), then the
      // two column halves of the tile in a fixed order
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
          for (int o = 1; o < 16; o <<= 1) rowsum[a][r] += __shfl_xor(rowsum[a][r], o);
        }
      if (wc == 1 && idx == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) red[wr][16 * a + 4 * g + r] = rowsum[a][r];
      }
      __syncthreads();
      if (wc == 0 && idx == 0) {
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 64 * wr + 16 * a + 4 * g + r;
            if (i < n_a)
              ep.e_part[ct * n_a + i] = rowsum[a][r] + red[wr][16 * a + 4 * g + r];
          }
      }
    } else {
      // column sums over the 16 rows of each fragment (lanes g, r), then the
      // four row quarters in a fixed order
      double cs[8];
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        cs[b] = colsum[b];
        cs[b] += __shfl_xor(cs[b], 16);
        cs[b] += __shfl_xor(cs[b], 32);
      }
      if (g == 0) {
#pragma unroll
        for (int b = 0; b < 8; ++b) red[wr][128 * wc + 16 * b + idx] = cs[b];
      }
      __syncthreads();
      if (wr == 0 && g == 0) {
#pragma unroll
        for (int b = 0; b < 8; ++b) {
          const int sl = 128 * wc + 16 * b + idx;
          const int64_t j = j0 + sl;
          if (j < n_b)
            ep.dc_part[rt * n_b + j] = ((red[0][sl] + red[1][sl]) + red[2][sl]) + red[3][sl];
        }
      }
    }
  }
}

// out[j] = sum over z of part[z][j] (fixed order)
__global__ void k_sum_parts(const double* __restrict__ part, int64_t nz, int64_t n,
                            int64_t stride, double* __restrict__ out, int64_t rows,
                            int64_t ldo, int64_t cols) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < rows * cols;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / cols, j = e - i * cols;
    double s = 0.0;
    for (int64_t z = 0; z < nz; ++z) s += part[z * stride + i * cols + j];
    out[i * ldo + j] = s;
  }
}

template <typename TA, typename TB, int EPI>
void launch_gemm(TA A, int64_t lda, int64_t n_a, TB B, int64_t ldb, int64_t n_b, int64_t K,
                 int nz, const EpiArgs& ep, hipStream_t st) {
  const int64_t kpz = ((K + nz - 1) / nz + 31) / 32 * 32;
  const dim3 grid(xcd_group_tile_blocks(cdiv_u(n_a, kGT), cdiv_u(n_b, kGT)),
                  (unsigned)cdiv_u(K, kpz));
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_gemm_b3<TA, TB, EPI>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, kGLds);
    attr = true;
  }
  hipLaunchKernelGGL((k_gemm_b3<TA, TB, EPI>), grid, dim3(kGThreads), kGLds, st, A, lda, n_a, B,
                     ldb, n_b, K, kpz, ep);
}

}  // namespace

int64_t gemm_b3_col_blocks(int64_t n_b) { return (n_b + kGT - 1) / kGT; }
int64_t gemm_b3_row_blocks(int64_t n_a) { return (n_a + kGT - 1) / kGT; }

void pstage_b3t(int mode, const void* desc, bool desc_f32, int64_t ldd, int64_t n,
                const __bf16* Xh, const __bf16* Xl, int64_t M, int64_t D, int zeta,
                double delta, const double* c, const double* g_e, float* W, int64_t ldw,
                double* e_part, double* dc_part, hipStream_t st) {
  if (n <= 0 || M <= 0) return;
  EpiArgs ep{};
  ep.zeta = zeta;
  ep.delta = delta;
  ep.c = c;
  ep.g_e = g_e;
  ep.W = W;
  ep.ldw = ldw;
  ep.e_part = e_part;
  ep.dc_part = dc_part;
  // X is taken pre-split (rows [M][split_ld(D)], hi and lo halves)
  const SplitRows xs{Xh, Xl};
  const int64_t ldp = split_ld(D);
  if (mode == 0) {
    if (desc_f32)
      launch_gemm<const float*, SplitRows, kPEnergy>(static_cast<const float*>(desc), ldd, n, xs,
                                                     ldp, M, D, 1, ep, st);
    else
      launch_gemm<const double*, SplitRows, kPEnergy>(static_cast<const double*>(desc), ldd, n,
                                                      xs, ldp, M, D, 1, ep, st);
  } else {
    if (desc_f32)
      launch_gemm<const float*, SplitRows, kPBack>(static_cast<const float*>(desc), ldd, n, xs,
                                                   ldp, M, D, 1, ep, st);
    else
      launch_gemm<const double*, SplitRows, kPBack>(static_cast<const double*>(desc), ldd, n, xs,
                                                    ldp, M, D, 1, ep, st);
  }
}

void gemm_b3_wx(const float* W, int64_t ldw, int64_t n, int64_t M, const __bf16* Xth,
                const __bf16* Xtl, int64_t D, double* out, int64_t ldo, hipStream_t st) {
  if (n <= 0 || D <= 0) return;
  EpiArgs ep{};
  ep.C = out;
  ep.ldc = ldo;
  launch_gemm<const float*, SplitRows, kPlain>(W, ldw, n, SplitRows{Xth, Xtl}, split_ld(M), D, M,
                                               1, ep, st);
}

void gemm_b3_wtd(const float* W, int64_t ldw, int64_t M, int64_t n, const void* desc,
                 bool desc_f32, int64_t ldd, int64_t D, double* part, int nz, double* out,
                 int64_t ldo, hipStream_t st) {
  if (M <= 0 || D <= 0) return;
  EpiArgs ep{};
  ep.C = part;
  ep.ldc = D;
  ep.zstride = M * D;
  // out[m][d] = sum_i W[i][m] desc[i][d]: both operands are column views (k = i)
  if (desc_f32)
    launch_gemm<ColOp<float>, ColOp<float>, kPlain>(ColOp<float>{W}, ldw, M,
                                                    ColOp<float>{static_cast<const float*>(desc)},
                                                    ldd, D, n, nz, ep, st);
  else
    launch_gemm<ColOp<float>, ColOp<double>, kPlain>(
        ColOp<float>{W}, ldw, M, ColOp<double>{static_cast<const double*>(desc)}, ldd, D, n, nz, ep,
        st);
  const unsigned g = std::max(1u, std::min(cdiv_u(M * D, 256), 65536u));
  hipLaunchKernelGGL(k_sum_parts, dim3(g), dim3(256), 0, st, part, (int64_t)nz, M * D, M * D, out,
                     M, ldo, D);
}

void sum_parts_f64(const double* part, int64_t nz, int64_t stride, double* out, int64_t rows,
                   int64_t ldo, int64_t cols, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return;
  const unsigned g = std::max(1u, std::min(cdiv_u(rows * cols, 256), 65536u));
  hipLaunchKernelGGL(k_sum_parts, dim3(g), dim3(256), 0, st, part, nz, rows * cols, stride, out,
                     rows, ldo, cols);
}

}  // namespace gapk
