// FP64 linear algebra of the stable least-squares route (Sec. "Theory"):
//   A = [Sigma^-1/2 L-hat K_NM ; U_MM],  b = [Sigma^-1/2 y ; 0],
//   K_MM + jitter I = U^T U (Cholesky), A = QR (Householder), c = R^-1 Q^T b,
// plus the pieces of FP64 iterative refinement (semi-normal equations).
//
// Householder QR, right-looking and blocked (compact WY, Q = I - V T V^T):
//   panel: one launch per column; every launch applies the previous reflector
//          to the rest of the panel and, in the same pass over the rows,
//          accumulates the norm and dot products that define the next
//          reflector; the last block to finish reduces the per-block partial
//          sums in a fixed order (no atomics on data, deterministic).
//   trailing update: W = V^T C (split over row slabs on FP64 MFMA, then a
//          fixed-order reduction), T from the Gram V^T V and tau, and
//          C -= V (T^T W) on FP64 MFMA.  b rides along as the last column.
#include <algorithm>

#include "launch.h"
#include "mma_f64.h"

namespace gapk {

namespace {

constexpr int kQrNB = 64;      // outer block width (compact-WY trailing update)
constexpr int kTrsvMaxBlocks = 256;  // multi-block triangular solve: n <= 64 * 256
constexpr int kPanelW = 32;    // inner panel width (column-by-column factorisation)
constexpr int kCholNB = 64;    // Cholesky block
constexpr int kPanelMaxGrid = 256;
// Workspace counter words: [0] the column kernels' counter, [kPanelBar ..
// kPanelBar + 8 * 16) the cooperative panel's eight arrival counters.
constexpr int kPanelBar = 64;
constexpr int kCounterWords = 256;

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

// Values exchanged between blocks of one launch (which may run on different
// XCDs with separate L2 caches) are written and read with relaxed device-scope
// atomics, which bypass the non-coherent caches, and ordered with s_waitcnt.
// No device-scope fence is used: on this part such a fence writes back and
// invalidates a whole L2.
GAP_DEV double vload(const double* p) {
  const uint64_t bits = __hip_atomic_load(reinterpret_cast<const uint64_t*>(p), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
  return __builtin_bit_cast(double, bits);
}
GAP_DEV void xstore(double* p, double v) {
  __hip_atomic_store(reinterpret_cast<uint64_t*>(p), __builtin_bit_cast(uint64_t, v),
                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until every memory operation this wave issued has completed.
GAP_DEV void wait_mem() { __builtin_amdgcn_s_waitcnt(0); }

// ----------------------------------------------------------- scale/stack ----
// rows r < n_rows: A[r][0:M] /= sigma_r, A[r][M] = y_r / sigma_r
__global__ void k_scale_rows(double* __restrict__ A, int64_t ld, int64_t n_rows, int64_t M,
                             const double* __restrict__ y, const double* __restrict__ sigma) {
  const int64_t col = blockIdx.y;
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n_rows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const double w = 1.0 / sigma[r];
    A[r + col * ld] = (col < M) ? A[r + col * ld] * w : y[r] * w;
  }
}

// rows n_rows + i (i < M): U = L^T (row i of U is column i of L), b = 0
__global__ void k_stack_u(double* __restrict__ A, int64_t ld, int64_t n_rows, int64_t M,
                          const double* __restrict__ L, int64_t ldl) {
  const int64_t col = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M;
       i += (int64_t)gridDim.x * blockDim.x)
    A[(n_rows + i) + col * ld] = (col < M && col >= i) ? L[col + i * ldl] : 0.0;
}

// -------------------------------------------------------------- Cholesky ----
__global__ void k_chol_init(double* __restrict__ Lw, int64_t ldl, int64_t M, double jitter,
                            const double* __restrict__ Kmm, int64_t ldk) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M;
       i += (int64_t)gridDim.x * blockDim.x)
    Lw[i + j * ldl] = Kmm[i + j * ldk] + (i == j ? jitter : 0.0);
}

// Diagonal block (nbj <= 64) by one wave, left-looking: lane r holds row r of
// the block in registers.  For column c, lane c publishes the finished part of
// its row (L[c][0:c]) to LDS; every lane forms the dot product of its row with
// it (broadcast reads), lane c's residual gives the pivot by a lane shuffle,
// and lanes below divide.  The column loop is unrolled so that every register
// index is a compile-time constant.
__global__ __launch_bounds__(64) void k_chol_diag(double* __restrict__ Lw, int64_t ldl, int64_t j0,
                                                  int nbj, int* dev_err) {
  __shared__ double rowc[kCholNB];
  const int l = threadIdx.x;
  double row[kCholNB];
#pragma unroll
  for (int c = 0; c < kCholNB; ++c)
    row[c] = (l < nbj && c < nbj) ? Lw[(j0 + l) + (j0 + c) * ldl] : 0.0;
  bool bad = false;
#pragma unroll
  for (int c = 0; c < kCholNB; ++c) {
    if (c < nbj) {
      if (l == c) {
#pragma unroll
        for (int q = 0; q < c; ++q) rowc[q] = row[q];
      }
      __syncthreads();
      double dot = 0.0;
#pragma unroll
      for (int q = 0; q < c; ++q) dot += row[q] * rowc[q];
      const double res = row[c] - dot;
      double p = __shfl(res, c);
      if (!(p > 0.0) || !isfinite(p)) {
        bad = true;
        p = 1.0;
      }
      const double d = sqrt(p);
      if (l == c) row[c] = d;
      else if (l > c) row[c] = res / d;
      __syncthreads();
    }
  }
  if (bad && l == 0) atomicOr(dev_err, GAP_DEVERR_NOT_PD);
#pragma unroll
  for (int c = 0; c < kCholNB; ++c)
    if (c < nbj && l < nbj && l >= c) Lw[(j0 + l) + (j0 + c) * ldl] = row[c];
}

// Rows below the diagonal block: L[r, j0:j0+nbj] = A[r, j0:j0+nbj] L_dd^-T.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ Lw, int64_t ldl, int64_t M,
                                                    int64_t j0, int nbj) {
  __shared__ double s[kCholNB][kCholNB + 1];
  for (int e = threadIdx.x; e < nbj * nbj; e += 256) {
    const int r = e % nbj, c = e / nbj;
    s[r][c] = (r >= c) ? Lw[(j0 + r) + (j0 + c) * ldl] : 0.0;
  }
  __syncthreads();
  const int64_t r = j0 + nbj + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= M) return;
  double x[kCholNB];
#pragma unroll
  for (int c = 0; c < kCholNB; ++c) {
    if (c < nbj) {
      double v = Lw[r + (j0 + c) * ldl];
#pragma unroll
      for (int q = 0; q < c; ++q) v -= x[q] * s[c][q];
      x[c] = v / s[c][c];
      Lw[r + (j0 + c) * ldl] = x[c];
    } else {
      x[c] = 0.0;
    }
  }
}

// C[r][c] -= sum_k P[r][k] P[c][k] on the lower trailing block (r >= c).
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ Lw, int64_t ldl,
                                                     int64_t M, int64_t j0, int nbj) {
  const int64_t t0 = j0 + nbj;
  const int64_t cbase = t0 + (int64_t)blockIdx.x * 64;  // columns (MFMA rows)
  const int64_t rbase = t0 + (int64_t)blockIdx.y * 64;  // rows (MFMA columns)
  if (rbase + 63 < cbase) return;                        // tile strictly above the diagonal
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t c = cbase + wave * 16 + idx;
  FragColK<double> fa{Lw + (c < M ? c : 0) + j0 * ldl, ldl, nbj, c < M};
  FragColK<double> fb[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = rbase + u * 16 + idx;
    fb[u] = FragColK<double>{Lw + (r < M ? r : 0) + j0 * ldl, ldl, nbj, r < M};
  }
  d4v acc[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) acc[u] = zero4();
  wave_mma<4>(fa, fb, nbj, g, acc);
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = rbase + u * 16 + idx;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t cc = cbase + wave * 16 + g + 4 * q;
      if (r < M && cc < M && r >= cc) Lw[r + cc * ldl] -= acc[u][q];
    }
  }
}

// ------------------------------------------------------------------- QR ----
// Column state of the current inner panel, per column: tau, beta, scale,
// tw[kPanelW] where tw[j] = tau * (v^T a_j) for the panel columns j to its right.
constexpr int kCS = kPanelW + 3;

__global__ __launch_bounds__(256) void k_qr_col(double* __restrict__ A, int64_t ld, int64_t m,
                                                int64_t j0, int pw, int64_t k,
                                                double* __restrict__ colstate,
                                                double* __restrict__ red,
                                                unsigned int* __restrict__ counter,
                                                double* __restrict__ tau_all) {
  __shared__ double s_tw[kPanelW];
  __shared__ double s_red[4][kPanelW];
  __shared__ double s_tot[kPanelW];
  __shared__ int s_last;
  __shared__ double s_par[2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t pend = j0 + pw;
  const bool has_prev = k > j0;
  const bool has_next = k < pend;
  const int64_t prev = k - 1;
  double beta_p = 0.0, scale_p = 0.0;
  if (has_prev) {
    const double* cs = colstate + (prev - j0) * kCS;
    beta_p = cs[1];
    scale_p = cs[2];
    for (int j = threadIdx.x; j < kPanelW; j += 256) s_tw[j] = cs[3 + j];
  }
  __syncthreads();
  const int ncnt = has_next ? (int)(pend - k) : 0;  // sigma, then d_{k+1} .. d_{pend-1}
  double part[kPanelW];
#pragma unroll
  for (int jj = 0; jj < kPanelW; ++jj) part[jj] = 0.0;

  const int64_t r_lo = has_prev ? prev : k;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // Columns touched this pass: jb .. pend-1 (jb = prev when a reflector is applied).
  const int64_t jb = has_prev ? prev : k;
  const int nc = (int)(pend - jb);
  for (int64_t r = r_lo + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < m; r += stride) {
    // all loads of the row first (independent, issued together), then compute, then store
    double a[kPanelW + 1];
    double* rp = A + jb * ld + r;  // column offsets jj * ld are uniform across the wave
#pragma unroll
    for (int jj = 0; jj <= kPanelW; ++jj) a[jj] = (jj < nc) ? rp[jj * ld] : 0.0;
    const bool acc_row = has_next && r > k;
    int o = 0;  // offset of column k in a[]
    if (has_prev) {
      double v;
      if (r == prev) {
        v = 1.0;
        a[0] = beta_p;
      } else {
        v = a[0] * scale_p;
        a[0] = v;
      }
#pragma unroll
      for (int jj = 1; jj <= kPanelW; ++jj)
        if (jj < nc) a[jj] -= s_tw[jb + jj - j0] * v;
      o = 1;
    }
    if (acc_row) {
      const double ak = has_prev ? a[1] : a[0];
      part[0] += ak * ak;
#pragma unroll
      for (int jj = 1; jj < kPanelW; ++jj)
        if (jj < ncnt) part[jj] += ak * (has_prev ? a[jj + 1] : a[jj]);
    }
    if (has_prev) {
      if (r == k) {  // the next pivot row is read by the last block of this launch
#pragma unroll
        for (int jj = 0; jj <= kPanelW; ++jj)
          if (jj < nc) xstore(rp + jj * ld, a[jj]);
      } else {
#pragma unroll
        for (int jj = 0; jj <= kPanelW; ++jj)
          if (jj < nc) rp[jj * ld] = a[jj];
      }
    }
    (void)o;
  }
  if (!has_next) return;

  // block partial sums -> red[v * gridDim.x + block]
#pragma unroll
  for (int v = 0; v < kPanelW; ++v) {
    if (v < ncnt) {
      const double s = wave_sum(part[v]);
      if (lane == 0) s_red[wave][v] = s;
    }
  }
  __syncthreads();
  const int G = gridDim.x;
  for (int v = threadIdx.x; v < ncnt; v += 256)
    xstore(red + (int64_t)v * G + blockIdx.x,
           ((s_red[0][v] + s_red[1][v]) + s_red[2][v]) + s_red[3][v]);
  wait_mem();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned t =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_last = (t == (unsigned)G - 1u);
  }
  __syncthreads();
  if (!s_last) return;
  // Fixed-order reduction of the per-block partials: thread t sums blocks
  // t, t + 256, ... (loads issued together), then a wave and block tree.
  double tot[kPanelW];
#pragma unroll
  for (int v = 0; v < kPanelW; ++v) tot[v] = 0.0;
  for (int b = threadIdx.x; b < G; b += 256) {
#pragma unroll
    for (int v = 0; v < kPanelW; ++v)
      if (v < ncnt) tot[v] += vload(red + (int64_t)v * G + b);
  }
#pragma unroll
  for (int v = 0; v < kPanelW; ++v) {
    if (v < ncnt) {
      const double s = wave_sum(tot[v]);
      if (lane == 0) s_red[wave][v] = s;
    }
  }
  __syncthreads();
  for (int v = threadIdx.x; v < ncnt; v += 256)
    s_tot[v] = ((s_red[0][v] + s_red[1][v]) + s_red[2][v]) + s_red[3][v];
  __syncthreads();
  double* cs = colstate + (k - j0) * kCS;
  if (threadIdx.x == 0) {
    const double alpha = vload(A + k + k * ld);
    const double xnorm = sqrt(s_tot[0]);
    double tau = 0.0, beta = alpha, scale = 0.0;
    if (xnorm > 0.0) {
      beta = -copysign(hypot(alpha, xnorm), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    cs[0] = tau;
    cs[1] = beta;
    cs[2] = scale;
    tau_all[k] = tau;
    s_par[0] = tau;
    s_par[1] = scale;
    __hip_atomic_store(counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  for (int jj = 1 + threadIdx.x; jj < ncnt; jj += 256) {
    const int64_t j = k + jj;
    const double w = vload(A + k + j * ld) + s_par[1] * s_tot[jj];
    cs[3 + (j - j0)] = s_par[0] * w;
  }
}

// ------------------------------------------------ register-resident panel ----
// Householder factorisation of an inner panel of width <= kRRW with the whole
// panel held in registers across a cooperative grid: thread t of block b owns
// the panel rows i0 + (b * 512 + t) + q * (grid * 512), q < kRRQ.  Every column
// step applies the previous reflector to the thread's rows, forms per-block
// partial sums of the next column's norm and dot products, publishes them, and
// waits at a grid barrier; every block then reduces all partials in the same
// fixed order, so all blocks derive identical reflector parameters without a
// second barrier.  Partials alternate between two buffers so a block that is
// one step ahead never overwrites values a slower block is still reading.
static_assert(kPanelMaxGrid <= 256, "the panel reduction reads at most 4 partials per lane");
constexpr int kRRW = 16;    // panel width
constexpr int kRRQ = 4;     // rows per thread
constexpr int kRRT = 512;   // threads per block
static_assert(kRRW == 16, "the panel's wave reduction is a 16-value butterfly");

GAP_DEV void grid_barrier(unsigned int* arrive, unsigned int target, int* dev_err) {
  wait_mem();  // this wave's cross-block stores (device-scope atomics) have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(arrive, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t spins = 0;
    // Bounded wait: a barrier that does not complete within ~0.2 s sets the
    // error bit, and every later barrier returns at once once the bit is set,
    // so a failed co-residency assumption costs one timeout, never a hang.
    while (__hip_atomic_load(arrive, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
      if (__hip_atomic_load(dev_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & GAP_DEVERR_SYNC)
        break;
      __builtin_amdgcn_s_sleep(2);
      if (++spins > (1ull << 22)) {
        atomicOr(dev_err, GAP_DEVERR_SYNC);
        break;
      }
    }
  }
  __syncthreads();
}

// Grid barrier on eight arrival counters, one per XCD slot of the block index
// (64 bytes apart), instead of one: the atomic adds of a few hundred blocks on a
// single address serialise at the memory-side atomic unit.  `round` counts the
// barriers completed including this one; counter x has seen round * n_x arrivals
// (n_x = blocks with index = x mod 8) when all blocks have arrived.  One wave
// polls all eight counters with one load per lane.  The counters are zeroed
// before the launch.
constexpr int kBarStride = 16;  // uints between arrival counters
GAP_DEV void grid_barrier_x8(unsigned int* arrive, unsigned int round, int* dev_err) {
  wait_mem();  // this wave's cross-block stores (device-scope atomics) have completed
  __syncthreads();
  if (threadIdx.x < 64) {
    const unsigned G = gridDim.x;
    if (threadIdx.x == 0)
      __hip_atomic_fetch_add(arrive + (blockIdx.x & 7) * kBarStride, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    const unsigned x = threadIdx.x & 7;
    const unsigned target = round * (G > x ? (G - x + 7) / 8 : 0u);
    uint64_t spins = 0;
    // Bounded wait, as in grid_barrier: a timeout sets the error bit, and a
    // set bit (checked every 64 polls) ends every later wait at once.
    for (;;) {
      const unsigned c =
          __hip_atomic_load(arrive + x * kBarStride, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
      if (__all(c >= target)) break;
      if ((spins & 63) == 63 &&
          (__hip_atomic_load(dev_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
           GAP_DEVERR_SYNC))
        break;
      __builtin_amdgcn_s_sleep(1);
      if (++spins > (1ull << 22)) {
        if (threadIdx.x == 0) atomicOr(dev_err, GAP_DEVERR_SYNC);
        break;
      }
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(kRRT) void k_qr_panel_rr(double* __restrict__ A, int64_t ld,
                                                      int64_t m, int64_t i0, int pw,
                                                      double* __restrict__ red,
                                                      double* __restrict__ piv,
                                                      unsigned int* __restrict__ arrive,
                                                      double* __restrict__ tau_all,
                                                      int* __restrict__ dev_err) {
  __shared__ double s_wred[kRRT / 64][kRRW];
  __shared__ double s_tot[kRRW];
  __shared__ double s_tw[kRRW];
  __shared__ double s_par[3];  // tau, beta, scale of the reflector just formed
  __shared__ double s_pv[kRRW];  // the pivot row of the current column
  const int G = gridDim.x;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)G * kRRT;
  int64_t lrow[kRRQ];  // local row index (row - i0), or -1
  double a[kRRQ][kRRW];
#pragma unroll
  for (int q = 0; q < kRRQ; ++q) {
    const int64_t lr = (int64_t)blockIdx.x * kRRT + threadIdx.x + q * stride;
    lrow[q] = (i0 + lr < m) ? lr : -1;
#pragma unroll
    for (int j = 0; j < kRRW; ++j)
      a[q][j] = (lrow[q] >= 0 && j < pw) ? A[(i0 + lr) + (i0 + j) * ld] : 0.0;
  }
  double beta_p = 0.0, scale_p = 0.0;
  for (int k = 0; k <= pw; ++k) {
    // 1. apply reflector k-1 to rows >= k-1.  Register arrays are indexed by
    //    absolute column only (selects against k), never by a k-relative
    //    index, which would force them out of registers.  tw[j] is zero for
    //    j <= k-1, and v is zero on rows above the reflector, so the update
    //    needs no condition.
    if (k > 0) {
      double tw[kRRW];
#pragma unroll
      for (int j = 0; j < kRRW; ++j) tw[j] = s_tw[j];
#pragma unroll
      for (int q = 0; q < kRRQ; ++q) {
        const bool at = lrow[q] == k - 1, below = lrow[q] > k - 1;
        double ak1 = 0.0;
#pragma unroll
        for (int j = 0; j < kRRW; ++j) ak1 = (j == k - 1) ? a[q][j] : ak1;
        const double v = at ? 1.0 : (below ? ak1 * scale_p : 0.0);
        const double nk1 = at ? beta_p : (below ? v : ak1);
#pragma unroll
        for (int j = 0; j < kRRW; ++j) {
          a[q][j] = (j == k - 1) ? nk1 : a[q][j];
          a[q][j] -= tw[j] * v;
        }
      }
    }
    if (k == pw) break;
    // 2. partial sums for column k over rows > k, by absolute column:
    //    part[k] = sum a_k^2, part[j] = sum a_k a_j (j > k); pivot row published
    double part[kRRW];
#pragma unroll
    for (int j = 0; j < kRRW; ++j) part[j] = 0.0;
#pragma unroll
    for (int q = 0; q < kRRQ; ++q) {
      double ak = 0.0;
#pragma unroll
      for (int j = 0; j < kRRW; ++j) ak = (j == k) ? a[q][j] : ak;
      ak = (lrow[q] > k) ? ak : 0.0;
      // columns j < k are summed too (no select per register) and never used
#pragma unroll
      for (int j = 0; j < kRRW; ++j) part[j] += ak * a[q][j];
      if (lrow[q] == k) {
        double* pv = piv + (k & 1) * kRRW;
#pragma unroll
        for (int j = 0; j < kRRW; ++j) xstore(pv + j, a[q][j]);
      }
    }
    // wave sums of the 16 partials by a halving butterfly (17 lane exchanges
    // instead of 16 separate 6-step reductions): lane l ends with the total of
    // column 8 b5 + 4 b4 + 2 b3 + b2 of its lane bits
    {
      double t8[8], t4[4], t2[2], t1;
      const bool u5 = lane & 32, u4 = lane & 16, u3 = lane & 8, u2 = lane & 4;
#pragma unroll
      for (int i = 0; i < 8; ++i)
        t8[i] = (u5 ? part[i + 8] : part[i]) + __shfl_xor(u5 ? part[i] : part[i + 8], 32);
#pragma unroll
      for (int i = 0; i < 4; ++i)
        t4[i] = (u4 ? t8[i + 4] : t8[i]) + __shfl_xor(u4 ? t8[i] : t8[i + 4], 16);
#pragma unroll
      for (int i = 0; i < 2; ++i)
        t2[i] = (u3 ? t4[i + 2] : t4[i]) + __shfl_xor(u3 ? t4[i] : t4[i + 2], 8);
      t1 = (u2 ? t2[1] : t2[0]) + __shfl_xor(u2 ? t2[0] : t2[1], 4);
      t1 += __shfl_xor(t1, 2);
      t1 += __shfl_xor(t1, 1);
      const int jj = (u5 ? 8 : 0) + (u4 ? 4 : 0) + (u3 ? 2 : 0) + (u2 ? 1 : 0);
      if ((lane & 3) == 0 && jj >= k && jj < pw) s_wred[wave][jj - k] = t1;
    }
    const int ncnt = pw - k;
    __syncthreads();
    double* rb = red + (size_t)(k & 1) * kRRW * G;
    if (threadIdx.x < ncnt) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kRRT / 64; ++w) s += s_wred[w][threadIdx.x];
      xstore(rb + (int64_t)threadIdx.x * G + blockIdx.x, s);
    }
    grid_barrier_x8(arrive, (unsigned)(k + 1), dev_err);
    // the pivot row, read together with the partials below (one round trip)
    const double* pv = piv + (k & 1) * kRRW;
    if (threadIdx.x < kRRW) s_pv[threadIdx.x] = vload(pv + threadIdx.x);
    // 3. every block reduces all partials in the same order.  A wave reads the
    //    G <= 256 partials of its two columns (wave, wave + 8) with all eight
    //    loads in flight together (clamped addresses, out-of-range ones scaled
    //    by zero), so the reads cost one memory round trip, not one per load.
    if (wave < ncnt) {
      const int v0 = wave, v1 = min(wave + kRRT / 64, ncnt - 1);
      double x0[4], x1[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int b = min(lane + 64 * i, G - 1);
        x0[i] = vload(rb + (int64_t)v0 * G + b);
        x1[i] = vload(rb + (int64_t)v1 * G + b);
      }
      double s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double w = (lane + 64 * i < G) ? 1.0 : 0.0;
        s0 += w * x0[i];
        s1 += w * x1[i];
      }
      s0 = wave_sum(s0);
      s1 = wave_sum(s1);
      if (lane == 0) {
        s_tot[v0] = s0;
        if (wave + kRRT / 64 < ncnt) s_tot[wave + kRRT / 64] = s1;
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const double alpha = s_pv[k];
      const double xnorm = sqrt(s_tot[0]);
      double tau = 0.0, beta = alpha, scale = 0.0;
      if (xnorm > 0.0) {
        beta = -copysign(hypot(alpha, xnorm), alpha);
        tau = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      s_par[0] = tau;
      s_par[1] = beta;
      s_par[2] = scale;
      if (blockIdx.x == 0) tau_all[i0 + k] = tau;
    }
    __syncthreads();
    if (threadIdx.x < kRRW) {
      const int j = threadIdx.x;
      s_tw[j] = (j > k && j < pw) ? s_par[0] * (s_pv[j] + s_par[2] * s_tot[j - k]) : 0.0;
    }
    beta_p = s_par[1];
    scale_p = s_par[2];
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kRRQ; ++q) {
    if (lrow[q] < 0) continue;
#pragma unroll
    for (int j = 0; j < kRRW; ++j)
      if (j < pw) A[(i0 + lrow[q]) + (i0 + j) * ld] = a[q][j];
  }
}

__global__ void k_sum_slabs(const double* __restrict__ part, int64_t nslab, int64_t n,
                            double* __restrict__ W) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t q = 0; q < nslab; ++q) s += part[q * n + e];
    W[e] = s;
  }
}

// sum_{q0 <= q < q1} a(q) b(q) with four independent partial sums, so that the
// LDS reads of four terms are in flight together (a single running sum waits
// for each read in turn)
template <class FA, class FB>
GAP_DEV double dot4(int q0, int q1, FA a, FB b) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int q = q0;
  for (; q + 3 < q1; q += 4) {
    s0 += a(q) * b(q);
    s1 += a(q + 1) * b(q + 1);
    s2 += a(q + 2) * b(q + 2);
    s3 += a(q + 3) * b(q + 3);
  }
  for (; q < q1; ++q) s0 += a(q) * b(q);
  return (s0 + s1) + (s2 + s3);
}

// T (pw x pw upper, row-major ld kQrNB): T_ii = tau_i, T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i]
__global__ __launch_bounds__(256) void k_qr_larft(const double* __restrict__ W, int64_t nct, int pw,
                                                  const double* __restrict__ tau,
                                                  double* __restrict__ T) {
  __shared__ double sT[kQrNB][kQrNB + 1];
  __shared__ double sG[kQrNB][kQrNB + 1];
  __shared__ double sTau[kQrNB];  // staged once: a load per column would cost a round trip each
  if (threadIdx.x < kQrNB) sTau[threadIdx.x] = (int)threadIdx.x < pw ? tau[threadIdx.x] : 0.0;
  for (int e = threadIdx.x; e < kQrNB * kQrNB; e += 256) {
    const int l = e / kQrNB, i = e % kQrNB;
    sG[l][i] = (l < pw && i < pw) ? W[(int64_t)l * nct + i] : 0.0;
    sT[l][i] = 0.0;
  }
  __syncthreads();
  for (int i = 0; i < pw; ++i) {
    const double ti = sTau[i];
    double z = 0.0;
    const int l = threadIdx.x;
    if (l < i) z = dot4(l, i, [&](int q) { return sT[l][q]; }, [&](int q) { return sG[q][i]; });
    __syncthreads();
    if (l < i) sT[l][i] = -ti * z;
    if (l == i) sT[i][i] = ti;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kQrNB * kQrNB; e += 256) T[e] = sT[e / kQrNB][e % kQrNB];
}

// Wt[kk][c'] = sum_{l <= kk} T[l][kk] W[l][c']  for c' in [pw, nct)
// Wt[kk][cp] = -(T^T W)[kk][cp] for cp in [pw, nct) (negated: the update adds V Wt)
__global__ void k_qr_tw(const double* __restrict__ W, int64_t nct, int pw,
                        const double* __restrict__ T, double* __restrict__ Wt) {
  const int64_t ntr = nct - pw;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)pw * ntr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int kk = (int)(e / ntr);
    const int64_t cp = pw + (e - (int64_t)kk * ntr);
    double s = 0.0;
    for (int l = 0; l <= kk; ++l) s += T[l * kQrNB + kk] * W[(int64_t)l * nct + cp];
    Wt[(int64_t)kk * nct + cp] = -s;
  }
}

// T and Wt = -T^T W of a narrow reflector block (pw <= 16, nct <= 64) in one
// wave: the same sums in the same order as k_qr_larft followed by k_qr_tw, in
// one launch instead of two.  W's pw rows and tau are staged in LDS first with
// all loads in flight at once; the rest works from LDS with a one-wave barrier
// per column.
__global__ __launch_bounds__(64) void k_qr_larft_tw16(const double* __restrict__ W, int64_t nct,
                                                      int pw, const double* __restrict__ tau,
                                                      double* __restrict__ T,
                                                      double* __restrict__ Wt) {
  __shared__ double sW[16][65];
  __shared__ double sT[16][17];
  __shared__ double sTau[16];
  const int l = threadIdx.x;
#pragma unroll
  for (int r = 0; r < 16; ++r)
    sW[r][l] = (r < pw && l < nct) ? W[(int64_t)r * nct + l] : 0.0;
  if (l < 16) sTau[l] = l < pw ? tau[l] : 0.0;
  for (int e = l; e < 256; e += 64) sT[e / 16][e % 16] = 0.0;
  __syncthreads();
  for (int i = 0; i < pw; ++i) {
    const double ti = sTau[i];
    double z = 0.0;
    if (l < i) z = dot4(l, i, [&](int q) { return sT[l][q]; }, [&](int q) { return sW[q][i]; });
    __syncthreads();
    if (l < i) sT[l][i] = -ti * z;
    if (l == i) sT[i][i] = ti;
    __syncthreads();
  }
  for (int e = l; e < pw * pw; e += 64) T[(e / pw) * kQrNB + e % pw] = sT[e / pw][e % pw];
  const int ntr = (int)(nct - pw);
  for (int e = l; e < pw * ntr; e += 64) {
    const int kk = e / ntr, cp = pw + (e - kk * ntr);
    const double acc =
        dot4(0, kk + 1, [&](int q) { return sT[q][kk]; }, [&](int q) { return sW[q][cp]; });
    Wt[(int64_t)kk * nct + cp] = -acc;
  }
}

// Trailing update, persistent over a 128-row block of C: the block stages
// V^T for its rows once in LDS (with the unit lower trapezoid applied), then
// walks the 64-wide column tiles of C.  W' = -(T^T W) tiles are double-buffered
// in LDS and the next C tile is prefetched into registers while the current
// one runs on the matrix cores; accumulators start as the C tile, so each C
// element is read and written once.  Eight waves: 2 (column halves) x 4 (row
// quarters), each a 32 x 32 block of (C column, C row) = (matrix-core row, col).
constexpr int kUR = 128;  // rows of C per block
constexpr int kUC = 64;   // columns per tile
template <int KW>
__global__ __launch_bounds__(512) void k_qr_upd(double* __restrict__ A, int64_t ld, int64_t m,
                                                int64_t j0, int pw, int64_t c_end, int64_t nct,
                                                const double* __restrict__ Wt) {
  // padded row strides: the four lane groups of a fragment read (rows kk .. kk+3)
  // fall on different banks
  __shared__ double sV[KW][kUR + 8];
  __shared__ double sW[2][KW][kUC + 8];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wc = wave & 1, wr = wave >> 1;
  const int64_t r0 = j0 + (int64_t)blockIdx.x * kUR;
  const int64_t cbeg = j0 + pw;
  const int ntile = (int)((c_end - cbeg + kUC - 1) / kUC);
  if (r0 - j0 >= KW && r0 + kUR <= m) {
    // below the unit triangle and inside the matrix: all loads issued at once
    // (rows kk >= pw read row pw - 1 and are zeroed after), not one guarded
    // load after another
    constexpr int kN = KW * kUR / 512;
    double tmp[kN];
#pragma unroll
    for (int t = 0; t < kN; ++t) {
      const int e = threadIdx.x + t * 512, kk = e / kUR, x = e % kUR;
      tmp[t] = A[(r0 + x) + (j0 + min(kk, pw - 1)) * ld];
    }
#pragma unroll
    for (int t = 0; t < kN; ++t) {
      const int e = threadIdx.x + t * 512, kk = e / kUR, x = e % kUR;
      sV[kk][x] = kk < pw ? tmp[t] : 0.0;
    }
  } else {
    for (int e = threadIdx.x; e < KW * kUR; e += 512) {
      const int kk = e / kUR, x = e % kUR;
      const int64_t r = r0 + x;
      double v = 0.0;
      if (kk < pw && r < m) {
        const int64_t rr = r - j0;
        v = (rr == kk) ? 1.0 : (rr > kk ? A[r + (j0 + kk) * ld] : 0.0);
      }
      sV[kk][x] = v;
    }
  }
  // W' tile in registers first (8 values per thread), written to LDS later
  double wreg[KW * kUC / 512];
  auto load_w = [&](int tile) {
#pragma unroll
    for (int t = 0; t < KW * kUC / 512; ++t) {
      // clamped, unconditional: rows kk >= pw meet zero rows of sV, columns
      // beyond c_end only feed outputs that are never stored
      const int e = threadIdx.x + t * 512;
      const int kk = min(e / kUC, pw - 1), x = e % kUC;
      const int64_t c = min(cbeg + (int64_t)min(tile, ntile - 1) * kUC + x, c_end - 1);
      wreg[t] = Wt[(int64_t)kk * nct + (c - j0)];
    }
  };
  auto store_w = [&](int buf) {
#pragma unroll
    for (int t = 0; t < KW * kUC / 512; ++t) {
      const int e = threadIdx.x + t * 512;
      sW[buf][e / kUC][e % kUC] = wreg[t];
    }
  };
  auto load_c = [&](int tile, d4v (&dst)[2][2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t rc = min(r0 + wr * 32 + j * 16 + idx, m - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t c = cbeg + (int64_t)tile * kUC + wc * 32 + i * 16 + g + 4 * q;
          dst[i][j][q] = A[rc + min(c, c_end - 1) * ld];
        }
      }
  };
  d4v acc[2][2], nxt[2][2];
  load_w(0);
  load_c(0, acc);
  store_w(0);
  __syncthreads();
  int buf = 0;
  for (int tile = 0; tile < ntile; ++tile) {
    const bool more = tile + 1 < ntile;
    if (more) {
      load_w(tile + 1);
      load_c(tile + 1, nxt);
    }
#pragma unroll
    for (int k0 = 0; k0 < KW; k0 += 4) {  // rows of sV at and beyond pw are zero
      const int kk = k0 + g;
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sW[buf][kk][wc * 32 + i * 16 + idx];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sV[kk][wr * 32 + j * 16 + idx];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t r = r0 + wr * 32 + j * 16 + idx;
        if (r >= m) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t c = cbeg + (int64_t)tile * kUC + wc * 32 + i * 16 + g + 4 * q;
          if (c < c_end) A[r + c * ld] = acc[i][j][q];
        }
      }
    if (more) store_w(buf ^ 1);
    lds_barrier();
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = nxt[i][j];
    buf ^= 1;
  }
}

// Buffer resources with a base in scalar registers: an access is that base
// plus a 32-bit per-lane offset plus a scalar offset, so a kernel that walks
// many columns of the column-major matrix keeps one offset register instead of
// a 64-bit address per column.  An access at or beyond the resource's size
// reads zero (a store is dropped).
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
GAP_DEV __amdgpu_buffer_rsrc_t uniform_rsrc(const double* p, uint32_t bytes) {
  const uint64_t x = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)((uint64_t)hi << 32 | lo), 0, (int)bytes,
                                           0x00020000);
}
GAP_DEV double buf_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
GAP_DEV void buf_st(double x, __amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, voff, soff, 0);
}

// W = V^T C over row slabs, staged through LDS: a block owns one slab and a
// 128-wide column tile (relative to the panel start; columns < pw are the
// panel's own V columns, giving the Gram V^T V).  32-row chunks of V and C are
// double-buffered in LDS (register prefetch of the next chunk while the
// current one runs on the matrix cores).  Consecutive logical blocks on an XCD
// share the slab, so its V rows come from that XCD's L2.  Eight waves:
// 2 (V-column halves) x 4 (C-column quarters), 32 x 32 outputs each.
constexpr int kVC = 128;  // C columns per block
constexpr int kVK = 32;   // rows per chunk
__global__ __launch_bounds__(512) void k_qr_vtc2(const double* __restrict__ A, int64_t ld,
                                                 int64_t m, int64_t j0, int pw, int64_t nct,
                                                 int64_t slab, int64_t n_ct, int64_t total,
                                                 int64_t per_xcd, double* __restrict__ part) {
  // row strides padded (73 and 137 doubles) so that neither the row-wise stash
  // (consecutive threads -> consecutive rows) nor the fragment reads conflict
  __shared__ double sV[2][kVK][kQrNB + 9];
  __shared__ double sC[2][kVK][kVC + 9];
  const int64_t logical = xcd_logical_block(per_xcd);
  if (logical >= total) return;
  const int64_t s = logical / n_ct, ct = logical % n_ct;
  const int64_t r0 = j0 + s * slab, r1 = std::min(m, r0 + slab);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wv = wave & 1, wq = wave >> 1;
  const int64_t c0 = ct * kVC;  // first column (relative to j0) of the tile
  // per-thread slice of a chunk: V 4 elements, C 8 elements (rows fastest);
  // two register sets so chunk k+2 is in flight while chunk k+1 lands in LDS
  double rv[2][4], rc[2][8];
  auto fetch = [&](int64_t rk, int set) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = threadIdx.x + t * 512;
      const int x = e / kVK, kk = e % kVK;
      const int64_t r = rk + kk;
      double v = 0.0;
      if (x < pw && r < r1) {
        const int64_t rr = r - j0;
        v = (rr == x) ? 1.0 : (rr > x ? A[r + (j0 + x) * ld] : 0.0);
      }
      rv[set][t] = v;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = threadIdx.x + t * 512;
      const int x = e / kVK, kk = e % kVK;
      const int64_t r = rk + kk;
      const int64_t cp = c0 + x;
      double v = 0.0;
      if (cp < nct && r < r1) {
        if (cp < pw) {
          const int64_t rr = r - j0;
          v = (rr == cp) ? 1.0 : (rr > cp ? A[r + (j0 + cp) * ld] : 0.0);
        } else {
          v = A[r + (j0 + cp) * ld];
        }
      }
      rc[set][t] = v;
    }
  };
  auto stash = [&](int buf, int set) {
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int e = threadIdx.x + t * 512;
      sV[buf][e % kVK][e / kVK] = rv[set][t];
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int e = threadIdx.x + t * 512;
      sC[buf][e % kVK][e / kVK] = rc[set][t];
    }
  };
  d4v acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = zero4();
  auto compute = [&](int buf) {
#pragma unroll
    for (int k0 = 0; k0 < kVK; k0 += 4) {
      const int kk = k0 + g;
      double a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) a[i] = sV[buf][kk][wv * 32 + i * 16 + idx];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sC[buf][kk][wq * 32 + j * 16 + idx];
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
  };
  // chunk c covers rows r0 + c * kVK; chunk c lives in LDS buffer c & 1 and,
  // before that, in register set c & 1
  const int64_t nch = (r1 - r0 + kVK - 1) / kVK;
  fetch(r0, 0);
  if (nch > 1) fetch(r0 + kVK, 1);
  stash(0, 0);
  __syncthreads();
  for (int64_t c = 0; c < nch; c += 2) {
    // even chunk c in LDS buffer 0; chunk c+1 in register set 1
    if (c + 2 < nch) fetch(r0 + (c + 2) * kVK, 0);
    compute(0);
    if (c + 1 < nch) stash(1, 1);
    lds_barrier();
    if (c + 1 >= nch) break;
    if (c + 3 < nch) fetch(r0 + (c + 3) * kVK, 1);
    compute(1);
    if (c + 2 < nch) stash(0, 0);
    lds_barrier();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t cp = c0 + wq * 32 + j * 16 + idx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ii = wv * 32 + i * 16 + g + 4 * q;
        if (ii < pw && cp < nct) part[(s * pw + ii) * nct + cp] = acc[i][j][q];
      }
    }
}

// W = V^T C for a narrow reflector block (pw <= 16) and a narrow C (nct <= 64
// columns, the panel's own columns first): the update inside a 64-column block
// after each 16-wide panel.  This is a memory-bound pass over m x nct doubles,
// so it has no LDS staging: wave u of a block owns C columns [16 u, 16 u + 16)
// and all 16 V columns, reads 4 consecutive rows of its columns per lane
// (32-byte loads, K-permuted so lane group g holds rows 4 g .. 4 g + 3 of a
// 16-row chunk), and keeps two chunks in flight.  Slabs are short (kNarrowSlab
// rows) so that many blocks stream at once; chunks clear of the V triangle and
// of the slab end load with no condition.
constexpr int kNarrowSlab = 512;
__global__ __launch_bounds__(256) void k_qr_vtc_narrow(const double* __restrict__ A, int64_t ld,
                                                       int64_t m, int64_t j0, int pw, int64_t nct,
                                                       double* __restrict__ part) {
  const int64_t s = blockIdx.x;
  const int64_t r0 = j0 + s * kNarrowSlab, r1 = std::min(m, r0 + kNarrowSlab);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t cp = (int64_t)wave * 16 + idx;  // this lane's C column (relative to j0)
  if ((int64_t)wave * 16 >= nct) return;
  const double* vcol = A + (j0 + min(idx, pw - 1)) * ld;
  const double* ccol = A + (j0 + min(cp, nct - 1)) * ld;
  d4v acc = zero4();
  auto chunk = [&](int64_t rk, double (&va)[4], double (&cb)[4]) {
    const int64_t r = rk + 4 * g;
    if (rk - j0 >= 16 && rk + 16 <= r1) {  // uniform over the wave
      const d4v v = *reinterpret_cast<const d4v*>(vcol + r);
      const d4v c = *reinterpret_cast<const d4v*>(ccol + r);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        va[q] = v[q];
        cb[q] = c[q];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t rq = r + q, rr = rq - j0;
        const bool in = rq < r1;
        const double v = in ? vcol[rq] : 0.0;
        const double c = in ? ccol[rq] : 0.0;
        va[q] = (!in || idx >= pw) ? 0.0 : (rr == idx ? 1.0 : (rr > idx ? v : 0.0));
        cb[q] = (!in || cp >= nct) ? 0.0
                                   : (cp < pw ? (rr == cp ? 1.0 : (rr > cp ? c : 0.0)) : c);
      }
    }
  };
  const int64_t nch = (r1 - r0 + 15) / 16;
  double va0[4], cb0[4], va1[4], cb1[4];
  if (nch > 0) chunk(r0, va0, cb0);
  if (nch > 1) chunk(r0 + 16, va1, cb1);
  for (int64_t c = 0; c < nch; c += 2) {
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = mfma_f64(va0[q], cb0[q], acc);
    if (c + 2 < nch) chunk(r0 + (c + 2) * 16, va0, cb0);
    if (c + 1 >= nch) break;
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = mfma_f64(va1[q], cb1[q], acc);
    if (c + 3 < nch) chunk(r0 + (c + 3) * 16, va1, cb1);
  }
  // D layout: lane (g, idx) holds W[V column g + 4 q][C column idx of the tile]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int ii = g + 4 * q;
    if (ii < pw && cp < nct) part[(s * pw + ii) * nct + cp] = acc[q];
  }
}

// ---------------------------------------------- outer (128-wide) WY update ----
// The same two products as above for a reflector block up to kQrOB = 128 wide:
// one pass over the trailing columns per 128 reflectors halves the HBM traffic
// of the 64-wide update, and each C element then carries 256 flops per 16 bytes
// moved, enough to keep the FP64 matrix cores ahead of memory.
constexpr int kQrOB = 128;

// W = V^T C over row slabs with V up to 128 wide.  Eight waves: 2 (64-column
// halves of V) x 4 (32-column quarters of the 128-column C tile).
template <bool BUF>
__global__ __launch_bounds__(512) void k_qr_vtc3(const double* __restrict__ A, int64_t ld,
                                                 int64_t m, int64_t j0, int pw, int64_t nct,
                                                 int64_t slab, int64_t n_ct, int64_t total,
                                                 int64_t per_xcd, double* __restrict__ part) {
  __shared__ double sV[2][kVK][kQrOB + 9];
  __shared__ double sC[2][kVK][kVC + 9];
  const int64_t logical = xcd_logical_block(per_xcd);
  if (logical >= total) return;
  const int64_t s = logical / n_ct, ct = logical % n_ct;
  const int64_t r0 = j0 + s * slab, r1 = std::min(m, r0 + slab);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wv = wave & 1, wq = wave >> 1;
  const int64_t c0 = ct * kVC;
  // each thread stages one row (kk) of a chunk and the columns x0 + 16 t
  const int kk_t = threadIdx.x & (kVK - 1), x0 = threadIdx.x / kVK;
  double rv[8], rc[8], rv2[8], rc2[8];
  // Two fetch forms.  Interior chunks (every row inside the slab and below the
  // V triangle) load from clamped addresses with no condition at all: V
  // columns >= pw only feed W rows >= pw and C columns >= nct only feed W
  // columns >= nct, none of which are stored.  A guarded load compiles to a
  // branch that waits for the load on the spot, so guards are kept to the few
  // edge chunks (the V triangle at the top of the first slab, a partial last
  // chunk), which use the masked form.
  auto fetch_fast = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    const double* rowp = A + (rk + kk_t);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      rv[t] = rowp[(j0 + min(x0 + 16 * t, pw - 1)) * ld];
      rc[t] = rowp[(j0 + min(c0 + x0 + 16 * t, nct - 1)) * ld];
    }
  };
  auto fetch_masked = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    const int64_t r = rk + kk_t;
    const bool rin = r < r1;
    const int64_t rr = r - j0;
    const double* rowp = A + (rin ? r : 0);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int x = x0 + 16 * t;
      double v = 0.0;
      if (rin && x < pw) v = (rr == x) ? 1.0 : (rr > x ? rowp[(j0 + x) * ld] : 0.0);
      rv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t cp = c0 + x0 + 16 * t;
      double v = 0.0;
      if (rin && cp < nct) {
        if (cp >= pw)
          v = rowp[(j0 + cp) * ld];
        else
          v = (rr == cp) ? 1.0 : (rr > cp ? rowp[(j0 + cp) * ld] : 0.0);
      }
      rc[t] = v;
    }
  };
  // The interior form through buffer resources based at the chunk's first row
  // of the first V column and of the tile's first C column: the thread's row
  // and column x0 are its offset, each t adds 16 columns as a scalar offset,
  // and columns past pw (V) or nct (C) lie outside the resources and read zero.
  const uint32_t xoff = (uint32_t)(((int64_t)x0 * ld + kk_t) * 8);
  const uint32_t vbytes = (uint32_t)((int64_t)pw * ld * 8);
  const uint32_t cbytes = (uint32_t)(std::min<int64_t>(nct - c0, kVC) * ld * 8);
  auto fetch_buf = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    const auto rsv = uniform_rsrc(A + j0 * ld + rk, vbytes);
    const auto rsc = uniform_rsrc(A + (j0 + c0) * ld + rk, cbytes);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      rv[t] = buf_ld(rsv, xoff, (uint32_t)(16 * t * ld * 8));
      rc[t] = buf_ld(rsc, xoff, (uint32_t)(16 * t * ld * 8));
    }
  };
  auto fetch = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    if (rk - j0 >= pw && rk + kVK <= r1) {
      if (BUF)
        fetch_buf(rk, rv, rc);
      else
        fetch_fast(rk, rv, rc);
    } else {
      fetch_masked(rk, rv, rc);
    }
  };
  auto stash = [&](int buf, const double (&rv)[8], const double (&rc)[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      sV[buf][kk_t][x0 + 16 * t] = rv[t];
      sC[buf][kk_t][x0 + 16 * t] = rc[t];
    }
  };
  d4v acc[4][2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = zero4();
  auto compute = [&](int buf, int k_lo, int k_hi) {
#pragma unroll
    for (int k0 = k_lo; k0 < k_hi; k0 += 4) {
      const int kk = k0 + g;
      double a[4], b[2];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sV[buf][kk][wv * 64 + i * 16 + idx];
#pragma unroll
      for (int j = 0; j < 2; ++j) b[j] = sC[buf][kk][wq * 32 + j * 16 + idx];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
  };
  // Chunks that meet the unit triangle of V (first slab) or end past the
  // matrix take the masked fetch one at a time; the interior ones run a
  // pipeline: chunk c is fetched into a register set two chunks ahead and
  // written to LDS buffer c & 1 in the middle of chunk c - 1's products (that
  // buffer was last read by chunk c - 2, before the previous barrier), so the
  // LDS writes overlap matrix-core work and the loads have a chunk and a half
  // to arrive.  The pipeline is straight-line code (fetches past the last
  // interior chunk re-read it, and its extra LDS write is never read), which
  // lets every wait for a fetch count the newer fetches still in flight.
  const int64_t nfull = (r1 - r0) / kVK;
  const int64_t c_lo = std::min<int64_t>(nfull, r0 - j0 >= pw ? 0 : (pw - (r0 - j0) + kVK - 1) / kVK);
  const int64_t c_hi = nfull;
  auto single = [&](int64_t c) {
    fetch_masked(r0 + c * kVK, rv, rc);
    lds_barrier();
    stash(0, rv, rc);
    lds_barrier();
    compute(0, 0, kVK);
  };
  for (int64_t c = 0; c < c_lo; ++c) single(c);
  if (c_hi > c_lo) {
    auto fetch_i = [&](int64_t c, double (&rv_)[8], double (&rc_)[8]) {
      const int64_t rk = r0 + std::min(c, c_hi - 1) * kVK;
      if (BUF)
        fetch_buf(rk, rv_, rc_);
      else
        fetch_fast(rk, rv_, rc_);
    };
    lds_barrier();
    fetch_i(c_lo, rv, rc);
    stash(0, rv, rc);
    fetch_i(c_lo + 1, rv2, rc2);
    lds_barrier();
    auto step = [&](int64_t c, double (&rnext)[8], double (&cnext)[8], double (&rfar)[8],
                    double (&cfar)[8]) {
      const int buf = (int)((c - c_lo) & 1);
      fetch_i(c + 2, rfar, cfar);
      compute(buf, 0, kVK / 2);
      stash(buf ^ 1, rnext, cnext);
      compute(buf, kVK / 2, kVK);
      lds_barrier();
    };
    int64_t c = c_lo;
    for (; c + 1 < c_hi; c += 2) {
      step(c, rv2, rc2, rv, rc);      // chunk c + 1 is in set 2, chunk c + 2 goes to set 1
      step(c + 1, rv, rc, rv2, rc2);  // chunk c + 2 is in set 1, chunk c + 3 goes to set 2
    }
    if (c < c_hi) step(c, rv2, rc2, rv, rc);
  }
  if (c_hi * kVK < r1 - r0) {
    lds_barrier();
    single(c_hi);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int64_t cp = c0 + wq * 32 + j * 16 + idx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ii = wv * 64 + i * 16 + g + 4 * q;
        if (ii < pw && cp < nct) part[(s * pw + ii) * nct + cp] = acc[i][j][q];
      }
    }
}

// The same product with four waves per block (each a 64 x 64 block of W) and
// 16-row chunks, so that the LDS of a block is 70 KB and two blocks share a
// compute unit: the two waves on a SIMD then belong to different blocks and
// are not held in step by one barrier, so one block's LDS writes and barrier
// overlap the other block's matrix-core products.
constexpr int kV5K = 16;
template <bool BUF>
__global__ __launch_bounds__(256, 2) void k_qr_vtc5(const double* __restrict__ A, int64_t ld,
                                                 int64_t m, int64_t j0, int pw, int64_t nct,
                                                 int64_t slab, int64_t n_ct, int64_t total,
                                                 int64_t per_xcd, double* __restrict__ part) {
  constexpr int kVK = kV5K;
  __shared__ double sV[2][kVK][kQrOB + 9];
  __shared__ double sC[2][kVK][kVC + 9];
  const int64_t logical = xcd_logical_block(per_xcd);
  if (logical >= total) return;
  const int64_t s = logical / n_ct, ct = logical % n_ct;
  const int64_t r0 = j0 + s * slab, r1 = std::min(m, r0 + slab);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wv = wave & 1, wq = wave >> 1;
  const int64_t c0 = ct * kVC;
  // each thread stages one row (kk) of a chunk and the columns x0 + 16 t
  const int kk_t = threadIdx.x & (kVK - 1), x0 = threadIdx.x / kVK;  // x0 < 16
  double rv[8], rc[8], rv2[8], rc2[8];
  // Two fetch forms.  Interior chunks (every row inside the slab and below the
  // V triangle) load from clamped addresses with no condition at all: V
  // columns >= pw only feed W rows >= pw and C columns >= nct only feed W
  // columns >= nct, none of which are stored.  A guarded load compiles to a
  // branch that waits for the load on the spot, so guards are kept to the few
  // edge chunks (the V triangle at the top of the first slab, a partial last
  // chunk), which use the masked form.
  auto fetch_fast = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    const double* rowp = A + (rk + kk_t);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      rv[t] = rowp[(j0 + min(x0 + 16 * t, pw - 1)) * ld];
      rc[t] = rowp[(j0 + min(c0 + x0 + 16 * t, nct - 1)) * ld];
    }
  };
  auto fetch_masked = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    const int64_t r = rk + kk_t;
    const bool rin = r < r1;
    const int64_t rr = r - j0;
    const double* rowp = A + (rin ? r : 0);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int x = x0 + 16 * t;
      double v = 0.0;
      if (rin && x < pw) v = (rr == x) ? 1.0 : (rr > x ? rowp[(j0 + x) * ld] : 0.0);
      rv[t] = v;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int64_t cp = c0 + x0 + 16 * t;
      double v = 0.0;
      if (rin && cp < nct) {
        if (cp >= pw)
          v = rowp[(j0 + cp) * ld];
        else
          v = (rr == cp) ? 1.0 : (rr > cp ? rowp[(j0 + cp) * ld] : 0.0);
      }
      rc[t] = v;
    }
  };
  // The interior form through buffer resources based at the chunk's first row
  // of the first V column and of the tile's first C column: the thread's row
  // and column x0 are its offset, each t adds 16 columns as a scalar offset,
  // and columns past pw (V) or nct (C) lie outside the resources and read zero.
  const uint32_t xoff = (uint32_t)(((int64_t)x0 * ld + kk_t) * 8);
  const uint32_t vbytes = (uint32_t)((int64_t)pw * ld * 8);
  const uint32_t cbytes = (uint32_t)(std::min<int64_t>(nct - c0, kVC) * ld * 8);
  auto fetch_buf = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    const auto rsv = uniform_rsrc(A + j0 * ld + rk, vbytes);
    const auto rsc = uniform_rsrc(A + (j0 + c0) * ld + rk, cbytes);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      rv[t] = buf_ld(rsv, xoff, (uint32_t)(16 * t * ld * 8));
      rc[t] = buf_ld(rsc, xoff, (uint32_t)(16 * t * ld * 8));
    }
  };
  auto fetch = [&](int64_t rk, double (&rv)[8], double (&rc)[8]) {
    if (rk - j0 >= pw && rk + kVK <= r1) {
      if (BUF)
        fetch_buf(rk, rv, rc);
      else
        fetch_fast(rk, rv, rc);
    } else {
      fetch_masked(rk, rv, rc);
    }
  };
  auto stash = [&](int buf, const double (&rv)[8], const double (&rc)[8]) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      sV[buf][kk_t][x0 + 16 * t] = rv[t];
      sC[buf][kk_t][x0 + 16 * t] = rc[t];
    }
  };
  d4v acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = zero4();
  auto compute = [&](int buf, int k_lo, int k_hi) {
#pragma unroll
    for (int k0 = k_lo; k0 < k_hi; k0 += 4) {
      const int kk = k0 + g;
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = sV[buf][kk][wv * 64 + i * 16 + idx];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = sC[buf][kk][wq * 64 + j * 16 + idx];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
  };
  // Chunks that meet the unit triangle of V (first slab) or end past the
  // matrix take the masked fetch one at a time; the interior ones run a
  // pipeline: chunk c is fetched into a register set two chunks ahead and
  // written to LDS buffer c & 1 in the middle of chunk c - 1's products (that
  // buffer was last read by chunk c - 2, before the previous barrier), so the
  // LDS writes overlap matrix-core work and the loads have a chunk and a half
  // to arrive.  The pipeline is straight-line code (fetches past the last
  // interior chunk re-read it, and its extra LDS write is never read), which
  // lets every wait for a fetch count the newer fetches still in flight.
  const int64_t nfull = (r1 - r0) / kVK;
  const int64_t c_lo = std::min<int64_t>(nfull, r0 - j0 >= pw ? 0 : (pw - (r0 - j0) + kVK - 1) / kVK);
  const int64_t c_hi = nfull;
  auto single = [&](int64_t c) {
    fetch_masked(r0 + c * kVK, rv, rc);
    lds_barrier();
    stash(0, rv, rc);
    lds_barrier();
    compute(0, 0, kVK);
  };
  for (int64_t c = 0; c < c_lo; ++c) single(c);
  if (c_hi > c_lo) {
    auto fetch_i = [&](int64_t c, double (&rv_)[8], double (&rc_)[8]) {
      const int64_t rk = r0 + std::min(c, c_hi - 1) * kVK;
      if (BUF)
        fetch_buf(rk, rv_, rc_);
      else
        fetch_fast(rk, rv_, rc_);
    };
    lds_barrier();
    fetch_i(c_lo, rv, rc);
    stash(0, rv, rc);
    fetch_i(c_lo + 1, rv2, rc2);
    lds_barrier();
    auto step = [&](int64_t c, double (&rnext)[8], double (&cnext)[8], double (&rfar)[8],
                    double (&cfar)[8]) {
      const int buf = (int)((c - c_lo) & 1);
      fetch_i(c + 2, rfar, cfar);
      compute(buf, 0, kVK / 2);
      stash(buf ^ 1, rnext, cnext);
      compute(buf, kVK / 2, kVK);
      lds_barrier();
    };
    int64_t c = c_lo;
    for (; c + 1 < c_hi; c += 2) {
      step(c, rv2, rc2, rv, rc);      // chunk c + 1 is in set 2, chunk c + 2 goes to set 1
      step(c + 1, rv, rc, rv2, rc2);  // chunk c + 2 is in set 1, chunk c + 3 goes to set 2
    }
    if (c < c_hi) step(c, rv2, rc2, rv, rc);
  }
  if (c_hi * kVK < r1 - r0) {
    lds_barrier();
    single(c_hi);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t cp = c0 + wq * 64 + j * 16 + idx;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ii = wv * 64 + i * 16 + g + 4 * q;
        if (ii < pw && cp < nct) part[(s * pw + ii) * nct + cp] = acc[i][j][q];
      }
    }
}

// T (pw x pw upper triangular, ld kQrOB) of a reflector block from the Gram
// G = V^T V held in the first pw columns of W (row l at W + l * nct), in two
// steps.  The diagonal 64 x 64 blocks come from the column recursion
// T[0:i, i] = -tau_i T[0:i, 0:i] G[0:i, i], T[i][i] = tau_i, one block per half
// (k_qr_larft_half); the coupling block is T12 = -T11 G12 T22 (k_qr_tcouple),
// since for H = H1 H2 with H_k = I - V_k T_k V_k^T the product is
// I - [V1 V2] [[T1, -T1 V1^T V2 T2], [0, T2]] [V1 V2]^T.
__global__ __launch_bounds__(256) void k_qr_larft_half(const double* __restrict__ W,
                                                       int64_t nct, int pw,
                                                       const double* __restrict__ tau,
                                                       double* __restrict__ T) {
  __shared__ double sT[kQrNB][kQrNB + 1];
  __shared__ double sG[kQrNB][kQrNB + 1];
  const int o = blockIdx.x * kQrNB;
  const int w = min(kQrNB, pw - o);
  if (w <= 0) return;
  __shared__ double sTau[kQrNB];  // staged once: a load per column would cost a round trip each
  if (threadIdx.x < kQrNB) sTau[threadIdx.x] = (int)threadIdx.x < w ? tau[o + threadIdx.x] : 0.0;
  for (int e = threadIdx.x; e < kQrNB * kQrNB; e += 256) {
    const int l = e / kQrNB, i = e % kQrNB;
    sG[l][i] = (l < w && i < w) ? W[(int64_t)(o + l) * nct + (o + i)] : 0.0;
    sT[l][i] = 0.0;
  }
  __syncthreads();
  const int l = threadIdx.x;
  for (int i = 0; i < w; ++i) {
    double z = 0.0;
    if (l < i) z = dot4(l, i, [&](int q) { return sT[l][q]; }, [&](int q) { return sG[q][i]; });
    __syncthreads();
    const double ti = sTau[i];
    if (l < i) sT[l][i] = -ti * z;
    if (l == i) sT[i][i] = ti;
    __syncthreads();
  }
  for (int e = threadIdx.x; e < kQrNB * kQrNB; e += 256) {
    const int r = e / kQrNB, c = e % kQrNB;
    T[(int64_t)(o + r) * kQrOB + (o + c)] = sT[r][c];
    if (blockIdx.x == 1) T[(int64_t)(o + r) * kQrOB + c] = 0.0;  // lower-left block
  }
}

__global__ __launch_bounds__(256) void k_qr_tcouple(const double* __restrict__ W, int64_t nct,
                                                    int pw, double* __restrict__ T) {
  __shared__ double sA[kQrNB][kQrNB + 1];  // T11, then X = G12 T22
  __shared__ double sB[kQrNB][kQrNB + 1];  // G12
  __shared__ double sC[kQrNB][kQrNB + 1];  // T22
  const int w2 = pw - kQrNB;  // width of the second half (> 0)
  for (int e = threadIdx.x; e < kQrNB * kQrNB; e += 256) {
    const int r = e / kQrNB, c = e % kQrNB;
    sB[r][c] = (c < w2) ? W[(int64_t)r * nct + (kQrNB + c)] : 0.0;
    sC[r][c] = (r < w2 && c < w2) ? T[(int64_t)(kQrNB + r) * kQrOB + (kQrNB + c)] : 0.0;
  }
  __syncthreads();
  // X = G12 T22 (T22 upper triangular)
  double x[16];
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + u * 256, r = e / kQrNB, c = e % kQrNB;
    x[u] = dot4(0, c + 1, [&](int q) { return sB[r][q]; }, [&](int q) { return sC[q][c]; });
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + u * 256;
    sB[e / kQrNB][e % kQrNB] = x[u];  // sB now holds X
    sA[e / kQrNB][e % kQrNB] = T[(int64_t)(e / kQrNB) * kQrOB + (e % kQrNB)];
  }
  __syncthreads();
  // T12 = -T11 X (T11 upper triangular)
  for (int u = 0; u < 16; ++u) {
    const int e = threadIdx.x + u * 256, r = e / kQrNB, c = e % kQrNB;
    const double acc =
        dot4(r, kQrNB, [&](int q) { return sA[r][q]; }, [&](int q) { return sB[q][c]; });
    T[(int64_t)r * kQrOB + (kQrNB + c)] = -acc;
  }
}

// Wn[kk][cp] = -sum_{l <= kk} T[l][kk] W[l][cp] for cp in [pw, nct)  (T with ld ldt):
// the negated W' = T^T W, so the update kernel adds V Wn to C without a negation
// on the freshly loaded value (which would wait for the load at once)
__global__ void k_qr_tw_ld(const double* __restrict__ W, int64_t nct, int pw,
                           const double* __restrict__ T, int ldt, double* __restrict__ Wt) {
  const int64_t ntr = nct - pw;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < (int64_t)pw * ntr;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int kk = (int)(e / ntr);
    const int64_t cp = pw + (e - (int64_t)kk * ntr);
    double s = 0.0;
    for (int l = 0; l <= kk; ++l) s += T[l * ldt + kk] * W[(int64_t)l * nct + cp];
    Wt[(int64_t)kk * nct + cp] = -s;
  }
}

// C -= V W' for a reflector block up to 128 wide, persistent over a 128-row
// block of C: V^T for the rows is staged once in LDS (unit lower trapezoid
// applied, zero rows beyond pw).  A W' = T^T W tile (128 x 64) is loaded into
// registers one tile ahead, together with the next C tile (16 + 16 values per
// thread), and moves through a two-deep LDS ring in 16-deep k chunks, so no
// global load is waited on inside a tile.  Accumulators start as the C tile.
// Eight waves: 2 (column halves) x 4 (row quarters), each a 32 x 32 block of
// (C column, C row) = (matrix-core row, column).
constexpr int kU3R = 128;
constexpr int kU3C = 64;
constexpr int kU3K = kQrOB / 16;  // k chunks per tile
__global__ __launch_bounds__(512) void k_qr_upd3(double* __restrict__ A, int64_t ld, int64_t m,
                                                 int64_t j0, int pw, int64_t c_end, int64_t nct,
                                                 const double* __restrict__ Wn) {
  __shared__ double sV[kQrOB][kU3R + 8];
  __shared__ double sW[2][16][kU3C + 4];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wc = wave & 1, wr = wave >> 1;
  const int64_t r0 = j0 + (int64_t)blockIdx.x * kU3R;
  const int64_t cbeg = j0 + pw;
  const int ntile = (int)((c_end - cbeg + kU3C - 1) / kU3C);
  // All kU3K chunks are always run (rows of sV beyond pw are zero): only the
  // last outer block is narrower than kQrOB, and its trailing part is the
  // right-hand side alone.  A compile-time chunk count keeps the choice of the
  // next chunk's source free of selects that would wait on the prefetch.
  for (int e = threadIdx.x; e < kQrOB * kU3R; e += 512) {
    const int kk = e / kU3R, x = e % kU3R;
    const int64_t r = r0 + x;
    double v = 0.0;
    if (kk < pw && r < m) {
      const int64_t rr = r - j0;
      v = (rr == kk) ? 1.0 : (rr > kk ? A[r + (j0 + kk) * ld] : 0.0);
    }
    sV[kk][x] = v;
  }
  // -W' tile (Wn): thread t holds, for chunk kc, elements t and t + 512 of the
  // 16 x 64 chunk (row e / 64, column e % 64)
  auto load_w = [&](int tile, double (&dst)[kU3K][2]) {
#pragma unroll
    for (int kc = 0; kc < kU3K; ++kc)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        // Unconditional load from a clamped (valid) address: a guarded load
        // becomes a branch whose join waits for every load in flight.  No mask
        // is needed: a clamped k row meets a zero row of sV, a clamped column
        // only feeds outputs that are never stored, and a tile beyond the last
        // is never used.
        const int e = threadIdx.x + h * 512;
        const int kk = min(kc * 16 + e / kU3C, pw - 1);  // rows >= pw meet zero rows of sV
        const int64_t c = min(cbeg + (int64_t)min(tile, ntile - 1) * kU3C + (e % kU3C), c_end - 1);
        dst[kc][h] = Wn[(int64_t)kk * nct + (c - j0)];
      }
  };
  auto store_w = [&](int buf, const double (&src)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int e = threadIdx.x + h * 512;
      sW[buf][e / kU3C][e % kU3C] = src[h];
    }
  };
  auto load_c = [&](int tile, d4v (&dst)[2][2]) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // clamped, unconditional (rows or columns outside C are never stored)
        const int64_t rc = min(r0 + wr * 32 + j * 16 + idx, m - 1);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t c =
              cbeg + (int64_t)min(tile, ntile - 1) * kU3C + wc * 32 + i * 16 + g + 4 * q;
          dst[i][j][q] = A[rc + min(c, c_end - 1) * ld];
        }
      }
  };
  d4v acc[2][2], nxt[2][2];
  double wcur[kU3K][2], wnxt[kU3K][2];
  load_c(0, acc);
  load_w(0, wcur);
  store_w(0, wcur[0]);
  __syncthreads();
  int buf = 0;
  for (int tile = 0; tile < ntile; ++tile) {
    load_c(tile + 1, nxt);
    load_w(tile + 1, wnxt);
#pragma unroll
    for (int kc = 0; kc < kU3K; ++kc) {
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) {
        const int kr = 4 * s4 + g;
        const int kk = kc * 16 + kr;
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = sW[buf][kr][wc * 32 + i * 16 + idx];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = sV[kk][wr * 32 + j * 16 + idx];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
      }
      // the next chunk: of this tile, or the first of the next tile
      if (kc + 1 < kU3K)
        store_w(buf ^ 1, wcur[kc + 1 < kU3K ? kc + 1 : 0]);
      else
        store_w(buf ^ 1, wnxt[0]);
      lds_barrier();
      buf ^= 1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int64_t r = r0 + wr * 32 + j * 16 + idx;
        if (r >= m) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t c = cbeg + (int64_t)tile * kU3C + wc * 32 + i * 16 + g + 4 * q;
          if (c < c_end) A[r + c * ld] = acc[i][j][q];
        }
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[i][j] = nxt[i][j];
#pragma unroll
    for (int kc = 0; kc < kU3K; ++kc) {
      wcur[kc][0] = wnxt[kc][0];
      wcur[kc][1] = wnxt[kc][1];
    }
  }
}

// C -= V W' for a full 128-wide reflector block, one barrier per 64-column
// tile.  Each of the eight waves owns 16 rows of the block's 128 and keeps
// their V (128 deep) in registers for the whole kernel; -W' (Wn) is the only
// shared operand and goes through LDS one whole 128 x 64 tile at a time,
// double-buffered: the next tile's Wn and C are fetched into registers at the
// start of a tile and Wn is written to the free LDS buffer at its end.  A
// wave's block is 16 rows x 64 columns (four matrix-core tiles sharing the V
// operand).  Odd Wn rows are stored with their 16-column halves swapped so that
// the lane groups reading rows 4t + g and 4t + g + 1 meet different banks.
//
// The memory traffic of a tile is issued between its matrix-core products, not
// around them: the two waves of a SIMD run in step (one barrier per tile), so
// work issued before or after the products leaves the matrix pipe idle.  For
// that the previous tile's result is stored during the next tile (from a copy,
// out), with buffer stores whose out-of-range offset drops the lanes that
// must not write, so no store sits in a branch.
//
// Every global access is a wave-uniform base (scalar registers) plus a 32-bit
// per-lane byte offset, and no column is clamped: the last tile is shifted left
// to end at c_end (it needs c_end - cbeg >= 64) and stores only the columns the
// previous tile did not.  Per-access 64-bit addresses would take 64 registers.
constexpr int kU5R = 128;  // rows per block (8 waves x 16)
constexpr int kU5C = 64;   // columns per tile
constexpr uint32_t kDropOffset = 0x80000000u;  // beyond any buffer this kernel makes
__global__ __launch_bounds__(512) void k_qr_upd5(double* __restrict__ A, int64_t ld, int64_t m,
                                                 int64_t j0, int64_t c_end, int64_t nct,
                                                 const double* __restrict__ Wn) {
  __shared__ double sW[2][kQrOB][kU5C];
  const int lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t r0 = j0 + (int64_t)blockIdx.x * kU5R;
  const int64_t rw = r0 + wave * 16 + idx;  // this lane's C row
  const int64_t cbeg = j0 + kQrOB;
  const int ntile = (int)((c_end - cbeg + kU5C - 1) / kU5C);
  // V(rw, k) for k = 4 t + g
  double v[kQrOB / 4];
  {
    const int64_t rr = rw - j0;
#pragma unroll
    for (int t = 0; t < kQrOB / 4; ++t) {
      const int k = 4 * t + g;
      double x = 0.0;
      if (rw < m) x = (rr == k) ? 1.0 : (rr > k ? A[rw + (j0 + k) * ld] : 0.0);
      v[t] = x;
    }
  }
  // first column of a tile (the last one shifted to end at c_end)
  auto tile_col = [&](int tile) { return min(cbeg + (int64_t)tile * kU5C, c_end - kU5C); };
  // Wn tile: thread (wave, lane) holds rows wave + 8 h (h = 0..15), column lane
  const uint32_t woff = (uint32_t)lane * 8u;
  const uint32_t wbytes = (uint32_t)(kQrOB * nct * 8);
  auto load_w = [&](int tile, double (&dst)[kQrOB / 8]) {
    const auto rs = uniform_rsrc(Wn + (tile_col(min(tile, ntile - 1)) - j0) + (int64_t)wave * nct,
                                 wbytes);
#pragma unroll
    for (int h = 0; h < kQrOB / 8; ++h) dst[h] = buf_ld(rs, woff, (uint32_t)(8 * h * nct * 8));
  };
  auto store_w = [&](int buf, const double (&src)[kQrOB / 8]) {
#pragma unroll
    for (int h = 0; h < kQrOB / 8; ++h) {
      const int k = wave + 8 * h;
      sW[buf][k][lane ^ ((k & 1) << 4)] = src[h];
    }
  };
  // C element (rw, c0 + 16 i + 4 q + g): base column pointer uniform, the row
  // and the lane group's column in the offset (rows past m read row m - 1)
  const uint32_t coff = (uint32_t)((min(rw, m - 1) - r0 + g * ld) * 8);
  const uint32_t cbytes = (uint32_t)(kU5C * ld * 8);  // a tile's extent from its base
  // C (rows r0.., a tile's 64 columns) as four 16-column groups i: lane holds
  // (rw, c0 + 16 i + 4 q + g) in q; reads of rows past m read row m - 1
  auto load_ci = [&](int tile, int i, d4v& dst) {
    const auto rs = uniform_rsrc(A + r0 + tile_col(min(tile, ntile - 1)) * ld, cbytes);
#pragma unroll
    for (int q = 0; q < 4; ++q) dst[q] = buf_ld(rs, coff, (uint32_t)((16 * i + 4 * q) * ld * 8));
  };
  // Stores of a tile through a buffer resource based at its first column: a
  // lane that must not write (row past m, or a column the shifted last tile
  // shares with the previous one) gets an offset past the buffer's end, which
  // the hardware drops.  Tile -1 (before the first) stores nothing.
  auto store_ci = [&](int tile, int i, const d4v& src) {
    const int64_t c0 = tile_col(max(tile, 0));
    const int shift = tile < 0 ? kU5C : (int)(cbeg + (int64_t)tile * kU5C - c0);
    const auto rs = uniform_rsrc(A + r0 + c0 * ld, cbytes);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool ok = rw < m && 16 * i + 4 * q + g >= shift;
      buf_st(src[q], rs, ok ? coff : kDropOffset, (uint32_t)((16 * i + 4 * q) * ld * 8));
    }
  };
  // a lane reads Wn row 4 t + g, columns 16 i + idx; odd rows are half-swapped
  const int sw = (g & 1) << 4;
  auto products = [&](d4v (&acc)[4], int t0, int t1, const double* wb) {
#pragma unroll
    for (int t = t0; t < t1; ++t) {
      double a[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = wb[t * 4 * kU5C + ((i * 16) ^ sw)];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] = mfma_f64(a[i], v[t], acc[i]);
    }
  };
  d4v acc[4], nxt[4];
  double wst[kQrOB / 8];
#pragma unroll
  for (int i = 0; i < 4; ++i) load_ci(0, i, acc[i]);
  load_w(0, wst);
  store_w(0, wst);
  // nothing of the prologue may be left in flight at the loop head: a pending
  // load there would make the wait at the head of every tile wait for the
  // previous tile's accesses as well
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  int buf = 0;
#pragma clang loop unroll(disable)
  for (int tile = 0; tile < ntile; ++tile) {
    load_w(tile + 1, wst);
#pragma unroll
    for (int i = 0; i < 4; ++i) load_ci(tile + 1, i, nxt[i]);
    products(acc, 0, kQrOB / 4, &sW[buf][g][idx]);
    store_w(buf ^ 1, wst);
#pragma unroll
    for (int i = 0; i < 4; ++i) store_ci(tile, i, acc[i]);
    lds_barrier();
    buf ^= 1;
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = nxt[i];
  }
}

// ------------------------------------------------------- triangular solves ----
// One workgroup of 16 waves solves R x = z (TRANS = false, back substitution) or
// R^T x = z (TRANS = true, forward substitution), R upper triangular, col-major (ld).
// Blocks of 64 unknowns: the 64 x 64 diagonal block is staged in LDS and solved by
// wave 0 (one unknown per lane, the solved value broadcast by a lane shuffle); the
// off-diagonal part is a GEMV over all 16 waves.  x lives in LDS (n doubles).
// A zero or non-finite diagonal entry sets GAP_DEVERR_RANK (if dev_err).
template <bool TRANS>
GAP_DEV void trsv_blk_lds(const double* __restrict__ R, int64_t ld, int64_t n, double* xs,
                          double (&T)[64][65], int* dev_err) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t nb = (n + 63) / 64;
  for (int64_t b = 0; b < nb; ++b) {
    const int64_t blk = TRANS ? b : nb - 1 - b;
    const int64_t j0 = blk * 64;
    const int w = (int)min((int64_t)64, n - j0);
    __syncthreads();
    for (int e = tid; e < 64 * 64; e += 1024) {
      const int r = e & 63, c = e >> 6;
      T[r][c] = (r < w && c < w && r <= c) ? R[(j0 + r) + (j0 + c) * ld] : 0.0;
    }
    if (TRANS) {
      // x_j -= sum_{i < j0} R[i][j] x_i for the block's columns (left-looking)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int cj = wave * 4 + q;
        if (cj < w) {
          const double* col = R + (j0 + cj) * ld;
          double s = 0.0;
          for (int64_t i = lane; i < j0; i += 64) s += col[i] * xs[i];
          s = wave_sum(s);
          if (lane == 0) xs[j0 + cj] -= s;
        }
      }
    }
    __syncthreads();
    if (wave == 0) {
      double t = lane < w ? xs[j0 + lane] : 0.0;
      bool bad = false;
      if (TRANS) {
        for (int c = 0; c < w; ++c) {
          const double d = T[c][c];
          bad |= (d == 0.0 || !isfinite(d));
          const double xc = __shfl(t, c) / d;
          if (lane == c) t = xc;
          else if (lane > c) t -= T[c][lane] * xc;
        }
      } else {
        for (int c = w - 1; c >= 0; --c) {
          const double d = T[c][c];
          bad |= (d == 0.0 || !isfinite(d));
          const double xc = __shfl(t, c) / d;
          if (lane == c) t = xc;
          else if (lane < c) t -= T[lane][c] * xc;
        }
      }
      if (lane < w) xs[j0 + lane] = t;
      if (bad && lane == 0 && dev_err) atomicOr(dev_err, GAP_DEVERR_RANK);
    }
    __syncthreads();
    if (!TRANS) {
      // x_i -= sum_{c in block} R[i][c] x_c for i < j0 (right-looking)
      for (int64_t i = tid; i < j0; i += 1024) {
        double s = 0.0;
#pragma unroll 8
        for (int c = 0; c < w; ++c) s += R[i + (j0 + c) * ld] * xs[j0 + c];
        xs[i] -= s;
      }
    }
  }
  __syncthreads();
}

template <bool TRANS>
__global__ __launch_bounds__(1024) void k_trsv_blk(const double* __restrict__ R, int64_t ld,
                                                   int64_t n, const double* z, double* x,
                                                   int* dev_err) {
  extern __shared__ double xs[];
  __shared__ double T[64][65];
  for (int64_t i = threadIdx.x; i < n; i += 1024) xs[i] = z[i];
  trsv_blk_lds<TRANS>(R, ld, n, xs, T, dev_err);
  for (int64_t i = threadIdx.x; i < n; i += 1024) x[i] = xs[i];
}

// Inverse of an upper-triangular R (col-major, ld), one column per workgroup:
// block c solves R y = e_c, which only involves the leading (c+1) x (c+1)
// block, and writes y as row-major Y (Y[i * ldy + c] = (R^-1)[i][c], zero
// below the diagonal).
__global__ __launch_bounds__(1024) void k_trinv_upper(const double* __restrict__ R, int64_t ld,
                                                      int64_t n, double* __restrict__ Y,
                                                      int64_t ldy, int* dev_err) {
  extern __shared__ double xs[];
  __shared__ double T[64][65];
  const int64_t c = blockIdx.x;
  for (int64_t i = threadIdx.x; i <= c; i += 1024) xs[i] = (i == c) ? 1.0 : 0.0;
  trsv_blk_lds<false>(R, ld, c + 1, xs, T, dev_err);
  for (int64_t i = threadIdx.x; i < n; i += 1024) Y[i * ldy + c] = (i <= c) ? xs[i] : 0.0;
}

// var[i] += sign * sum_j Z[i][j]^2 (row-major Z, one wave per row); with
// init, var[i] starts at delta^2 (d_i . d_i)^zeta instead.
template <typename TD>
__global__ __launch_bounds__(256) void k_var_rows(const double* __restrict__ Z, int64_t ldz,
                                                  int64_t n, int64_t m, double sign,
                                                  const TD* __restrict__ desc, int64_t ldd,
                                                  int64_t D, int zeta, double delta, int init,
                                                  double* __restrict__ var) {
  const int64_t i = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t j = lane; j < m; j += 64) {
    const double z = Z[i * ldz + j];
    s += z * z;
  }
  s = wave_sum(s);
  double kii = 0.0;
  if (init == 1) {
    double t = 0.0;
    for (int64_t k = lane; k < D; k += 64) {
      const double d = (double)desc[i * ldd + k];
      t += d * d;
    }
    t = wave_sum(t);
    double p = 1.0;
    for (int q = 0; q < zeta; ++q) p *= t;
    kii = delta * delta * p;
  }
  if (lane == 0) var[i] = (init ? kii : var[i]) + sign * s;
}

// Descriptors as FP64 rows [n][ldo] with zero row padding (columns D .. ldo - 1).
template <typename TD>
__global__ void k_desc_f64(const TD* __restrict__ desc, int64_t ldd, int64_t n, int64_t D,
                           double* __restrict__ out, int64_t ldo) {
  const int64_t i = blockIdx.y;
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < ldo;
       k += (int64_t)gridDim.x * blockDim.x)
    out[i * ldo + k] = k < D ? (double)desc[i * ldd + k] : 0.0;
}

// CUR selection keys, padded to n_pad (a power of two) with -inf / index n_pad:
// key_i = l_i (u NULL) or log(u_i) / l_i (weighted sampling without replacement).
__global__ void k_cur_keys(const double* __restrict__ lev, const double* __restrict__ u,
                           int64_t n, int64_t n_pad, double* __restrict__ key,
                           int32_t* __restrict__ idx) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_pad;
       i += (int64_t)gridDim.x * blockDim.x) {
    double k = -HUGE_VAL;
    if (i < n) {
      const double l = lev[i];
      k = u ? (l > 0.0 ? log(u[i]) / l : -HUGE_VAL) : l;
      if (!(k == k)) k = -HUGE_VAL;  // NaN sorts last
    }
    key[i] = k;
    idx[i] = (int32_t)i;
  }
}

// One compare-exchange stage of a bitonic sort into decreasing key, ties by
// increasing index (a total order, so the result is unique).
__global__ void k_bitonic(double* __restrict__ key, int32_t* __restrict__ idx, int64_t n_pad,
                          int64_t j, int64_t k) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_pad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i ^ j;
    if (l <= i) continue;
    const double ki = key[i], kl = key[l];
    const int32_t ii = idx[i], il = idx[l];
    const bool i_first = ki > kl || (ki == kl && ii < il);  // i precedes l in the final order
    const bool down = (i & k) == 0;                          // this run is sorted in final order
    if (down != i_first) {
      key[i] = kl;
      key[l] = ki;
      idx[i] = il;
      idx[l] = ii;
    }
  }
}

// Multi-block form of the same solves: block t owns the 64 unknowns of column
// block b (b = t for the forward solve with R^T, b = nb - 1 - t for back
// substitution), so every block it depends on has a smaller index and was
// dispatched earlier; the launch is cooperative, so all blocks are resident.
// A block folds in each dependency block c as soon as c publishes its 64
// values (flag[c] == epoch): a 64 x 64 product with the R tile, spread over
// 4 waves.  Then wave 0 solves the diagonal block (staged in LDS), and the
// block publishes its values with device-scope stores before its flag
// (cross-XCD exchange without an L2-flushing fence).  Waits are bounded and
// set GAP_DEVERR_SYNC on expiry, after which every wait returns at once.
template <bool TRANS>
__global__ __launch_bounds__(256) void k_trsv_coop(const double* __restrict__ R, int64_t ld,
                                                   int64_t n, const double* z, double* x,
                                                   unsigned int* __restrict__ flag,
                                                   unsigned int epoch, int* dev_err) {
  __shared__ double T[64][65];
  __shared__ double part[4][64];
  __shared__ double xd[64];
  const int nb = (int)((n + 63) / 64);
  const int b = TRANS ? (int)blockIdx.x : nb - 1 - (int)blockIdx.x;
  const int64_t j0 = (int64_t)b * 64;
  const int w = (int)min((int64_t)64, n - j0);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int r = e & 63, c = e >> 6;
    T[r][c] = (r < w && c < w && r <= c) ? R[(j0 + r) + (j0 + c) * ld] : 0.0;
  }
  double acc = 0.0;
  const int ndep = TRANS ? b : nb - 1 - b;
  for (int d = 0; d < ndep; ++d) {
    const int c = TRANS ? d : nb - 1 - d;  // in the order the dependencies complete
    const int64_t c0 = (int64_t)c * 64;
    if (tid == 0) {
      uint64_t spins = 0;
      while (__hip_atomic_load(flag + c, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != epoch) {
        if (dev_err && (__hip_atomic_load(dev_err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) &
                        GAP_DEVERR_SYNC))
          break;
        __builtin_amdgcn_s_sleep(1);
        if (++spins > (1ull << 22)) {
          if (dev_err) atomicOr(dev_err, GAP_DEVERR_SYNC);
          break;
        }
      }
    }
    __syncthreads();
    if (tid < 64) xd[tid] = (c0 + tid < n) ? vload(x + c0 + tid) : 0.0;
    __syncthreads();
    if (lane < w) {
      if (TRANS) {
        // unknown j0 + lane needs sum_i R[c0 + i][j0 + lane] y[c0 + i]
        const double* col = R + (j0 + lane) * ld + c0;
#pragma unroll 4
        for (int i = wave * 16; i < wave * 16 + 16; ++i) acc += col[i] * xd[i];
      } else {
        // unknown j0 + lane needs sum_j R[j0 + lane][c0 + j] x[c0 + j]
        // columns past n (the last block) are clamped in range; xd is zero there
        const double* row = R + (j0 + lane);
#pragma unroll 4
        for (int jj = wave * 16; jj < wave * 16 + 16; ++jj)
          acc += row[min(c0 + jj, n - 1) * ld] * xd[jj];
      }
    }
  }
  part[wave][lane] = acc;
  __syncthreads();
  if (wave == 0) {
    double t = lane < w ? z[j0 + lane] - (((part[0][lane] + part[1][lane]) + part[2][lane]) +
                                          part[3][lane])
                        : 0.0;
    bool bad = false;
    if (TRANS) {
      for (int c = 0; c < w; ++c) {
        const double dg = T[c][c];
        bad |= (dg == 0.0 || !isfinite(dg));
        const double xc = __shfl(t, c) / dg;
        if (lane == c) t = xc;
        else if (lane > c) t -= T[c][lane] * xc;
      }
    } else {
      for (int c = w - 1; c >= 0; --c) {
        const double dg = T[c][c];
        bad |= (dg == 0.0 || !isfinite(dg));
        const double xc = __shfl(t, c) / dg;
        if (lane == c) t = xc;
        else if (lane < c) t -= T[lane][c] * xc;
      }
    }
    if (lane < w) xstore(x + j0 + lane, t);
    if (bad && lane == 0 && dev_err) atomicOr(dev_err, GAP_DEVERR_RANK);
    wait_mem();
    if (lane == 0) __hip_atomic_store(flag + b, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
}

__global__ __launch_bounds__(1024) void k_rdiag_minmax(const double* __restrict__ R, int64_t ld,
                                                       int64_t n, double* __restrict__ rd) {
  __shared__ double smin[16], smax[16];
  double lo = INFINITY, hi = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
    const double a = fabs(R[i + i * ld]);
    lo = fmin(lo, a);
    hi = fmax(hi, a);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
  }
  if ((threadIdx.x & 63) == 0) {
    smin[threadIdx.x >> 6] = lo;
    smax[threadIdx.x >> 6] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      lo = fmin(lo, smin[w]);
      hi = fmax(hi, smax[w]);
    }
    lo = fmin(lo, smin[0]);
    hi = fmax(hi, smax[0]);
    rd[0] = lo;
    rd[1] = hi;
  }
}

// ------------------------------------------------------------ refinement ----
// r_top[r] = (y_r - kc_r) / sigma_r;  r_bot[i] = -(U c)_i = -sum_{j >= i} L[j][i] c_j
__global__ void k_residual_top(const double* __restrict__ y, const double* __restrict__ sigma,
                               const double* __restrict__ kc, int64_t n, double* __restrict__ r) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    r[i] = (y[i] - kc[i]) / sigma[i];
}

__global__ __launch_bounds__(256) void k_residual_bot(const double* __restrict__ L, int64_t ldl,
                                                      int64_t M, const double* __restrict__ c,
                                                      double* __restrict__ rb) {
  const int64_t i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= M) return;
  double s = 0.0;
  for (int64_t j = i + lane; j < M; j += 64) s += L[j + i * ldl] * c[j];
  s = wave_sum(s);
  if (lane == 0) rb[i] = -s;
}

// g[m] += sum_{i <= m} U[i][m] r_bot[i] = sum_{i <= m} L[m][i] r_bot[i]
// 64 rows per block, 16 waves splitting i; partial sums combined in LDS in a fixed order.
__global__ __launch_bounds__(1024) void k_add_ut_r(const double* __restrict__ L, int64_t ldl,
                                                   int64_t M, const double* __restrict__ rb,
                                                   double* __restrict__ g) {
  __shared__ double part[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t mm = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (mm < M)
    for (int64_t i = wave; i <= mm; i += 16) s += L[mm + i * ldl] * rb[i];
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && mm < M) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += part[w][lane];
    g[mm] += t;
  }
}

__global__ void k_div(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                      double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = a[i] / b[i];
}

__global__ void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_axpy(int64_t n, double a, const double* __restrict__ x, double* __restrict__ y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] += a * x[i];
}

// out[0] += sum_i x_i^2 (one workgroup; fixed summation order)
__global__ __launch_bounds__(1024) void k_sumsq_add(const double* __restrict__ x, int64_t n,
                                                    double* __restrict__ out) {
  __shared__ double sp[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i] * x[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sp[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sp[w];
    *out += t;
  }
}

__global__ __launch_bounds__(1024) void k_norm2(const double* __restrict__ x, int64_t n,
                                                double* __restrict__ out) {
  __shared__ double sp[16];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += blockDim.x) s += x[i] * x[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) sp[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += sp[w];
    *out = sqrt(t);
  }
}

// Streamed-fit state after a fold: the top M + 1 rows of columns [0, M) keep
// R (upper triangle); what the QR left below the diagonal there (Householder
// vectors, and row M) is cleared.  With zero_corner (the initial state) row M
// of column M is cleared too.
__global__ void k_fold_tidy(double* __restrict__ T, int64_t ld, int64_t M, int zero_corner) {
  const int64_t col = blockIdx.y;
  const int64_t r0 = col < M ? col + 1 : (zero_corner ? M : M + 1);
  for (int64_t r = r0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r <= M;
       r += (int64_t)gridDim.x * blockDim.x)
    T[r + col * ld] = 0.0;
}

__global__ void k_expand_cfg(const double* __restrict__ v, const int32_t* __restrict__ atom_cfg,
                             int64_t n, double* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = atom_cfg[i];
    out[i] = c >= 0 ? v[c] : 0.0;
  }
}

__global__ void k_fill_u32(unsigned int* __restrict__ p, int64_t n, unsigned int v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

inline unsigned g256(int64_t n) { return std::max(1u, std::min(cdiv(n, 256), 65536u)); }

}  // namespace

void scale_rows(double* A, int64_t ld, int64_t n_rows, int64_t M, const double* y,
                const double* sigma, hipStream_t st) {
  if (n_rows <= 0) return;
  dim3 grid(std::min(cdiv(n_rows, 256), 4096u), (unsigned)(M + 1));
  hipLaunchKernelGGL(k_scale_rows, grid, dim3(256), 0, st, A, ld, n_rows, M, y, sigma);
}

void stack_u(double* A, int64_t ld, int64_t n_rows, int64_t M, const double* L, int64_t ldl,
             hipStream_t st) {
  dim3 grid(cdiv(M, 256), (unsigned)(M + 1));
  hipLaunchKernelGGL(k_stack_u, grid, dim3(256), 0, st, A, ld, n_rows, M, L, ldl);
}

void cholesky_lower(double* Lw, int64_t ldl, int64_t M, double jitter, const double* Kmm,
                    int64_t ldk, int* dev_err, hipStream_t st) {
  hipLaunchKernelGGL(k_chol_init, dim3(cdiv(M, 256), (unsigned)M), dim3(256), 0, st, Lw, ldl, M,
                     jitter, Kmm, ldk);
  for (int64_t j0 = 0; j0 < M; j0 += kCholNB) {
    const int nbj = (int)std::min<int64_t>(kCholNB, M - j0);
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(64), 0, st, Lw, ldl, j0, nbj, dev_err);
    const int64_t rest = M - j0 - nbj;
    if (rest <= 0) break;
    hipLaunchKernelGGL(k_chol_panel, dim3(cdiv(rest, 256)), dim3(256), 0, st, Lw, ldl, M, j0, nbj);
    hipLaunchKernelGGL(k_chol_update, dim3(cdiv(rest, 64), cdiv(rest, 64)), dim3(256), 0, st, Lw,
                       ldl, M, j0, nbj);
  }
}

static int64_t qr_slab_rows(int64_t m) {
  // slabs of >= 2048 rows (a multiple of 32), at most 256 of them
  int64_t s = (m + 255) / 256;
  s = std::max<int64_t>(s, 2048);
  return (s + 31) / 32 * 32;
}

// Elements of the split-K partials buffer: those of the 128-wide updates, or
// of the 16- and 64-wide ones over short slabs (at most 64 reflectors x 128
// columns).  Both the workspace size and its binding use this one count.
static int64_t qr_part_elems(int64_t m, int64_t n) {
  const int64_t ncols = n + 1;
  const int64_t nslab = (m + qr_slab_rows(m) - 1) / qr_slab_rows(m);
  return std::max(nslab * kQrOB * ncols,
                  ((m + kNarrowSlab - 1) / kNarrowSlab + 1) * (int64_t)kQrNB * 2 * kQrNB);
}

size_t qr_workspace_bytes(int64_t m, int64_t n) {
  const int64_t ncols = n + 1;
  size_t d = 0;
  d += (size_t)qr_part_elems(m, n);           // part
  d += (size_t)kQrOB * ncols * 2;            // W, Wt
  d += (size_t)kQrOB * kQrOB;                // T
  d += (size_t)kQrNB * kCS;                  // colstate
  d += (size_t)kQrNB * kPanelMaxGrid;        // red
  d += (size_t)n + 8;                        // tau
  return d * sizeof(double) + sizeof(unsigned int) * (kCounterWords + kTrsvMaxBlocks);  // counters, flags
}

void qr_bind_workspace(void* base, int64_t m, int64_t n, QrWork* w) {
  const int64_t ncols = n + 1;
  double* p = reinterpret_cast<double*>(base);
  w->part = p;
  w->part_elems = qr_part_elems(m, n);
  p += w->part_elems;
  w->W = p;
  p += kQrOB * ncols;
  w->Wt = p;
  p += kQrOB * ncols;
  w->T = p;
  p += kQrOB * kQrOB;
  w->colstate = p;
  p += kQrNB * kCS;
  w->red = p;
  p += kQrNB * kPanelMaxGrid;
  w->tau = p;
  p += n + 8;
  w->counter = reinterpret_cast<unsigned int*>(p);
  w->flags = w->counter + kCounterWords;
}

// Compact-WY update of columns [c0, c_end) with the pw reflectors stored in
// columns [j0, j0 + pw): W = V^T A[j0:m, j0:c_end) (Gram V^T V included),
// T from the Gram and tau, then A[j0:m, c0:c_end) -= V (T^T W).
static void qr_wy_update(double* A, int64_t ld, int64_t m, int64_t j0, int pw, int64_t c_end,
                         int64_t slab, QrWork* w, hipStream_t st) {
  const int64_t nct = c_end - j0;
  if (nct <= pw) return;
  if (pw <= 16 && nct <= 64) {
    const int64_t nslab = (m - j0 + kNarrowSlab - 1) / kNarrowSlab;
    hipLaunchKernelGGL(k_qr_vtc_narrow, dim3((unsigned)nslab), dim3(256), 0, st, A, ld, m, j0, pw,
                       nct, w->part);
    // many slabs, few outputs: 16 waves per 64 outputs split the slab sum
    reduce_rows_f64(w->part, nslab, (int64_t)pw * nct, w->W, st);
    hipLaunchKernelGGL(k_qr_larft_tw16, dim3(1), dim3(64), 0, st, w->W, nct, pw, w->tau + j0,
                       w->T, w->Wt);
    hipLaunchKernelGGL(k_qr_upd<16>, dim3(cdiv(m - j0, kUR)), dim3(512), 0, st, A, ld, m, j0,
                       pw, c_end, nct, w->Wt);
    return;
  } else {
    // Short slabs: a 64-wide update has one column tile, so the slabs alone
    // must give enough blocks to fill the device; the many partials are summed
    // by the multi-block row reduction.
    (void)slab;
    const int64_t nslab = (m - j0 + kNarrowSlab - 1) / kNarrowSlab;
    const int64_t n_ct = (nct + kVC - 1) / kVC;
    const int64_t total = nslab * n_ct, per_xcd = (total + 7) / 8;
    hipLaunchKernelGGL(k_qr_vtc2, dim3((unsigned)(8 * per_xcd)), dim3(512), 0, st, A, ld, m, j0,
                       pw, nct, (int64_t)kNarrowSlab, n_ct, total, per_xcd, w->part);
    reduce_rows_f64(w->part, nslab, (int64_t)pw * nct, w->W, st);
  }
  hipLaunchKernelGGL(k_qr_larft, dim3(1), dim3(256), 0, st, w->W, nct, pw, w->tau + j0, w->T);
  hipLaunchKernelGGL(k_qr_tw, dim3(g256(pw * (nct - pw))), dim3(256), 0, st, w->W, nct, pw, w->T,
                     w->Wt);
  hipLaunchKernelGGL(k_qr_upd<kQrNB>, dim3(cdiv(m - j0, kUR)), dim3(512), 0, st, A, ld, m, j0, pw, c_end,
                     nct, w->Wt);
}

// The same update for an outer block of up to kQrOB reflectors.
static void qr_wy_update_ob(double* A, int64_t ld, int64_t m, int64_t j0, int pw, int64_t c_end,
                            int64_t slab, QrWork* w, hipStream_t st) {
  const int64_t nct = c_end - j0;
  if (nct <= pw) return;
  const int64_t nslab = (m - j0 + slab - 1) / slab;
  const int64_t n_ct = (nct + kVC - 1) / kVC;
  const int64_t total = nslab * n_ct, per_xcd = (total + 7) / 8;
  // buffer offsets reach 128 columns of the matrix
  if ((int64_t)kVC * ld * 8 < ((int64_t)1 << 31))
    hipLaunchKernelGGL(k_qr_vtc5<true>, dim3((unsigned)(8 * per_xcd)), dim3(256), 0, st, A, ld,
                       m, j0, pw, nct, slab, n_ct, total, per_xcd, w->part);
  else
    hipLaunchKernelGGL(k_qr_vtc3<false>, dim3((unsigned)(8 * per_xcd)), dim3(512), 0, st, A, ld,
                       m, j0, pw, nct, slab, n_ct, total, per_xcd, w->part);
  hipLaunchKernelGGL(k_sum_slabs, dim3(g256(pw * nct)), dim3(256), 0, st, w->part, nslab,
                     (int64_t)pw * nct, w->W);
  hipLaunchKernelGGL(k_qr_larft_half, dim3(2), dim3(256), 0, st, w->W, nct, pw, w->tau + j0,
                     w->T);
  if (pw > kQrNB)
    hipLaunchKernelGGL(k_qr_tcouple, dim3(1), dim3(256), 0, st, w->W, nct, pw, w->T);
  hipLaunchKernelGGL(k_qr_tw_ld, dim3(g256(pw * (nct - pw))), dim3(256), 0, st, w->W, nct, pw,
                     w->T, kQrOB, w->Wt);
  // the barrier-light kernel needs a full block, a full tile of trailing
  // columns and a 64-column tile of C within 31-bit offsets
  if (pw == kQrOB && nct - pw >= kU5C && ld < (int64_t)(1 << 22))
    hipLaunchKernelGGL(k_qr_upd5, dim3(cdiv(m - j0, kU5R)), dim3(512), 0, st, A, ld, m, j0,
                       c_end, nct, w->Wt);
  else
    hipLaunchKernelGGL(k_qr_upd3, dim3(cdiv(m - j0, kU3R)), dim3(512), 0, st, A, ld, m, j0, pw,
                       c_end, nct, w->Wt);
}

// Number of k_qr_panel_rr blocks that are co-resident on the current device (0 if unknown).
static int rr_capacity() {
  static int cap = -1;
  if (cap < 0) {
    cap = 0;
    int dev = 0, nb = 0;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_qr_panel_rr, kRRT, 0) == hipSuccess &&
        nb > 0)
      cap = std::min(nb * p.multiProcessorCount, kPanelMaxGrid);
  }
  return cap;
}

void qr_factor(double* A, int64_t ld, int64_t m, int64_t ncols, int64_t n, QrWork* w,
               hipStream_t st, int* dev_err, Timer* tm) {
  Timer dummy;
  if (!tm) tm = &dummy;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, w->counter);
  const int64_t slab = qr_slab_rows(m);
  const int cap = rr_capacity();
  // Three levels: 16-wide register-resident panels inside 64-wide blocks
  // (compact-WY updates within the block), 64-wide blocks inside 128-wide outer
  // blocks (one 64-wide update of the outer block's second half), and one
  // 128-wide update of the trailing matrix per outer block.
  for (int64_t o0 = 0; o0 < n; o0 += kQrOB) {
    const int ow = (int)std::min<int64_t>(kQrOB, n - o0);
    for (int64_t j0 = o0; j0 < o0 + ow; j0 += kQrNB) {
      const int bw = (int)std::min<int64_t>(kQrNB, o0 + ow - j0);
      int64_t i0 = j0;
      while (i0 < j0 + bw) {
        const int64_t rows = m - i0;
        // as few blocks as hold the panel: every column costs one grid barrier
        // and a reduction over the blocks' partials, both growing with the grid
        const int64_t G_rr = std::min<int64_t>(cap, (rows + kRRT * kRRQ - 1) / (kRRT * kRRQ));
        const bool rr = cap > 0 && rows <= G_rr * kRRT * kRRQ;
        const int pw = (int)std::min<int64_t>(rr ? kRRW : kPanelW, j0 + bw - i0);
        tm->begin(TM_QR_PANEL);
        bool done = false;
        if (rr) {
          hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, w->counter + kPanelBar,
                             (int64_t)8 * kBarStride, 0u);
          int64_t ld_ = ld, m_ = m, i0_ = i0;
          int pw_ = pw;
          double* A_ = A;
          double* red_ = w->red;
          double* piv_ = w->T;  // the T scratch is free while a panel is factored
          unsigned int* arr_ = w->counter + kPanelBar;
          double* tau_ = w->tau;
          int* err_ = dev_err;
          void* args[] = {&A_, &ld_, &m_, &i0_, &pw_, &red_, &piv_, &arr_, &tau_, &err_};
          done = hipLaunchCooperativeKernel(reinterpret_cast<const void*>(&k_qr_panel_rr),
                                            dim3((unsigned)G_rr), dim3(kRRT), args, 0,
                                            st) == hipSuccess;
          if (!done) (void)hipGetLastError();
        }
        if (!done) {
          for (int64_t k = i0; k <= i0 + pw; ++k) {
            const int64_t r_lo = (k > i0) ? k - 1 : k;
            const int64_t rr_rows = m - r_lo;
            const unsigned G = std::max(1u, std::min(cdiv(rr_rows, 512), (unsigned)kPanelMaxGrid));
            hipLaunchKernelGGL(k_qr_col, dim3(G), dim3(256), 0, st, A, ld, m, i0, pw, k,
                               w->colstate, w->red, w->counter, w->tau);
          }
        }
        // rest of the 64-wide block with this inner panel's reflectors
        qr_wy_update(A, ld, m, i0, pw, j0 + bw, slab, w, st);
        tm->end(TM_QR_PANEL);
        i0 += pw;
      }
      if (j0 + bw >= o0 + ow) continue;
      // rest of the outer block with this 64-wide block's reflectors
      tm->begin(TM_QR_UPDATE);
      qr_wy_update(A, ld, m, j0, bw, o0 + ow, slab, w, st);
      tm->end(TM_QR_UPDATE);
    }
    if (o0 + ow >= ncols) continue;
    tm->begin(TM_QR_UPDATE);
    qr_wy_update_ob(A, ld, m, o0, ow, ncols, slab, w, st);
    tm->end(TM_QR_UPDATE);
  }
}

// One triangular solve: the multi-block kernel when flags are given and it can
// be launched cooperatively, else the one-workgroup kernel.  x may alias z only
// for the one-workgroup form (it reads z into LDS first); the multi-block form
// reads z[j] only in the block that writes x[j], before it writes it.
static void trsv(bool trans, const double* A, int64_t ld, int64_t n, const double* z, double* x,
                 unsigned int* flags, int* dev_err, hipStream_t st) {
  const int nb = (int)((n + 63) / 64);
  if (flags && nb <= kTrsvMaxBlocks) {
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, st, flags, (int64_t)nb, 0u);
    unsigned int ep = 1;
    const double* A_ = A;
    int64_t ld_ = ld, n_ = n;
    const double* z_ = z;
    double* x_ = x;
    unsigned int* f_ = flags;
    int* e_ = dev_err;
    void* args[] = {&A_, &ld_, &n_, &z_, &x_, &f_, &ep, &e_};
    const void* kern = trans ? reinterpret_cast<const void*>(&k_trsv_coop<true>)
                             : reinterpret_cast<const void*>(&k_trsv_coop<false>);
    if (hipLaunchCooperativeKernel(kern, dim3((unsigned)nb), dim3(256), args, 0, st) ==
        hipSuccess)
      return;
    (void)hipGetLastError();
  }
  if (trans)
    hipLaunchKernelGGL(k_trsv_blk<true>, dim3(1), dim3(1024), (size_t)n * sizeof(double), st, A,
                       ld, n, z, x, dev_err);
  else
    hipLaunchKernelGGL(k_trsv_blk<false>, dim3(1), dim3(1024), (size_t)n * sizeof(double), st, A,
                       ld, n, z, x, dev_err);
}

void back_substitute(const double* A, int64_t ld, int64_t n, const double* z, double* x,
                     double* rd, int* dev_err, hipStream_t st, unsigned int* flags) {
  hipLaunchKernelGGL(k_rdiag_minmax, dim3(1), dim3(1024), 0, st, A, ld, n, rd);
  trsv(false, A, ld, n, z, x, flags, dev_err, st);
}

void seminormal_solve(const double* A, int64_t ld, int64_t n, double* x, hipStream_t st,
                      unsigned int* flags, double* tmp, int* dev_err) {
  // R^T y = x, then R x = y; the multi-block form needs y apart from x
  if (flags && tmp) {
    trsv(true, A, ld, n, x, tmp, flags, dev_err, st);
    trsv(false, A, ld, n, tmp, x, flags, dev_err, st);
  } else {
    trsv(true, A, ld, n, x, x, nullptr, nullptr, st);
    trsv(false, A, ld, n, x, x, nullptr, nullptr, st);
  }
}

void residual_top(const double* y, const double* sigma, const double* kc, int64_t n_rows,
                  double* r_top, hipStream_t st) {
  if (n_rows <= 0) return;
  hipLaunchKernelGGL(k_residual_top, dim3(g256(n_rows)), dim3(256), 0, st, y, sigma, kc, n_rows,
                     r_top);
}

void residual_bot(const double* L, int64_t ldl, int64_t M, const double* c, double* r_bot,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_residual_bot, dim3(cdiv(M, 4)), dim3(256), 0, st, L, ldl, M, c, r_bot);
}

void add_ut_r(const double* L, int64_t ldl, int64_t M, const double* r_bot, double* g,
              hipStream_t st) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_add_ut_r, dim3(cdiv(M, 64)), dim3(1024), 0, st, L, ldl, M, r_bot, g);
}

void div_sigma(const double* r_top, const double* sigma, int64_t n, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_div, dim3(g256(n)), dim3(256), 0, st, r_top, sigma, n, v);
}

void fill_f64(double* p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_fill_f64, dim3(g256(n)), dim3(256), 0, st, p, n, v);
}

void axpy_f64(int64_t n, double a, const double* x, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_axpy, dim3(g256(n)), dim3(256), 0, st, n, a, x, y);
}

void norm2_f64(const double* x, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_norm2, dim3(1), dim3(1024), 0, st, x, n, out);
}

void sumsq_add_f64(const double* x, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sumsq_add, dim3(1), dim3(1024), 0, st, x, n, out);
}

void trinv_upper(const double* R, int64_t ld, int64_t n, double* Y, int64_t ldy, int* dev_err,
                 hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_trinv_upper, dim3((unsigned)n), dim3(1024), (size_t)n * sizeof(double), st,
                     R, ld, n, Y, ldy, dev_err);
}

void var_rows(const double* Z, int64_t ldz, int64_t n, int64_t m, double sign, const void* desc,
              bool desc_f32, int64_t ldd, int64_t D, int zeta, double delta, int init,
              double* var, hipStream_t st) {
  if (n <= 0) return;
  dim3 grid(cdiv(n, 4));
  if (desc_f32)
    hipLaunchKernelGGL(k_var_rows<float>, grid, dim3(256), 0, st, Z, ldz, n, m, sign,
                       reinterpret_cast<const float*>(desc), ldd, D, zeta, delta, init, var);
  else
    hipLaunchKernelGGL(k_var_rows<double>, grid, dim3(256), 0, st, Z, ldz, n, m, sign,
                       reinterpret_cast<const double*>(desc), ldd, D, zeta, delta, init, var);
}

void desc_f64(const void* desc, bool desc_f32, int64_t ldd, int64_t n, int64_t D, double* out,
              int64_t ldo, hipStream_t st) {
  if (n <= 0) return;
  dim3 grid(cdiv(ldo, 256), (unsigned)n);
  if (desc_f32)
    hipLaunchKernelGGL(k_desc_f64<float>, grid, dim3(256), 0, st,
                       reinterpret_cast<const float*>(desc), ldd, n, D, out, ldo);
  else
    hipLaunchKernelGGL(k_desc_f64<double>, grid, dim3(256), 0, st,
                       reinterpret_cast<const double*>(desc), ldd, n, D, out, ldo);
}

int64_t cur_pad(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

void cur_select_sort(const double* lev, const double* u, int64_t n, double* key, int32_t* idx,
                     hipStream_t st) {
  const int64_t n_pad = cur_pad(n);
  const unsigned grid = std::max(1u, std::min(cdiv(n_pad, 256), 65536u));
  hipLaunchKernelGGL(k_cur_keys, dim3(grid), dim3(256), 0, st, lev, u, n, n_pad, key, idx);
  for (int64_t k = 2; k <= n_pad; k <<= 1)
    for (int64_t j = k >> 1; j > 0; j >>= 1)
      hipLaunchKernelGGL(k_bitonic, dim3(grid), dim3(256), 0, st, key, idx, n_pad, j, k);
}

void fold_tidy(double* T, int64_t ld, int64_t M, bool zero_corner, hipStream_t st) {
  // column M has rows > M only below the state, so it needs no clearing unless
  // the corner itself is reset
  dim3 grid(cdiv(M + 1, 256), (unsigned)(M + 1));
  hipLaunchKernelGGL(k_fold_tidy, grid, dim3(256), 0, st, T, ld, M, zero_corner ? 1 : 0);
}

void expand_cfg(const double* v, const int32_t* atom_cfg, int64_t n_atoms, double* out,
                hipStream_t st) {
  hipLaunchKernelGGL(k_expand_cfg, dim3(g256(n_atoms)), dim3(256), 0, st, v, atom_cfg, n_atoms,
                     out);
}

}  // namespace gapk
