// Dense FP64 contractions of the polynomial dot-product kernel on gfx950 MFMA:
//   K_MM = delta^2 (X X^T)^zeta                         (covariance of sparse points)
//   energy rows of L-hat K_NM and the kernel-gradient scale S used by force rows
//   predict / backward P-stage (P = D X^T recomputed, never stored)
//   the two follow-up GEMMs W X and W^T D.
// Polynomial dot-product kernel: Sec. "Regression"; energy rows: eq. 1 summed
// by L-hat over a configuration (Sec. "Theory"); predict: eq. epsilon.
#include <algorithm>

#include "launch.h"
#include "mma_f64.h"

namespace gapk {

namespace {

constexpr int kNC = 4;  // 16-column tiles per wave

template <typename T>
inline const T* tptr(const void* p) {
  return reinterpret_cast<const T*>(p);
}

// ---------------------------------------------------------------- K_MM ----
// Block (bi, bj) with bi <= bj computes the 64 x 64 tile of X X^T; every value
// with row <= col is written to (row, col) and (col, row), so K_MM is exactly
// symmetric whatever the summation order inside the matrix core.
__global__ __launch_bounds__(256) void k_kmm(const double* __restrict__ X, int64_t ldx, int64_t M,
                                             int64_t D, int zeta, double delta,
                                             double* __restrict__ K, int64_t ldk) {
  const int bi = blockIdx.y, bj = blockIdx.x;
  if (bi > bj) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t row = (int64_t)bi * 64 + wave * 16 + idx;
  FragRowK<double> fa{X + (row < M ? row : 0) * ldx, D, row < M};
  FragRowK<double> fb[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = (int64_t)bj * 64 + u * 16 + idx;
    fb[u] = FragRowK<double>{X + (col < M ? col : 0) * ldx, D, col < M};
  }
  d4v acc[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) acc[u] = zero4();
  wave_mma<kNC>(fa, fb, D, g, acc);
  const double d2 = delta * delta;
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = (int64_t)bj * 64 + u * 16 + idx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = (int64_t)bi * 64 + wave * 16 + g + 4 * r;
      if (rr < M && col < M && rr <= col) {
        const double v = d2 * ipow(acc[u][r], zeta);
        K[rr + col * ldk] = v;
        K[col + rr * ldk] = v;
      }
    }
  }
}

// ----------------------------------------------------- local-property rows ----
// Row r is atom i = idx[r] (i = r without an index list): K[r][m] = delta^2 (d_i . x_m)^zeta.  Block (column
// tile, row tile) of 64 x 64; each wave 16 rows (gathered descriptor rows) x
// 64 columns.  An index outside [0, n_atoms) gives a zero row and raises the
// index flag.
template <typename TD>
__global__ __launch_bounds__(256) void k_local_rows(const TD* __restrict__ desc, int64_t ldd,
                                                    int64_t n_atoms,
                                                    const int32_t* __restrict__ idx_list,
                                                    int64_t n_local, const double* __restrict__ X,
                                                    int64_t ldx, int64_t M, int64_t D, int zeta,
                                                    double delta, double* __restrict__ K,
                                                    int64_t ldk, int* __restrict__ dev_err,
                                                    int row_major) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = (int64_t)blockIdx.y * 64 + wave * 16;
  const int64_t row = rowbase + idx;
  const int64_t atom = row < n_local ? (idx_list ? (int64_t)idx_list[row] : row) : -1;
  const bool ok = atom >= 0 && atom < n_atoms;
  if (row < n_local && !ok && g == 0 && blockIdx.x == 0) atomicOr(dev_err, GAP_DEVERR_INDEX);
  FragRowK<TD> fa{desc + (ok ? atom : 0) * ldd, D, ok};
  FragRowK<double> fb[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = (int64_t)blockIdx.x * 64 + u * 16 + idx;
    fb[u] = FragRowK<double>{X + (col < M ? col : 0) * ldx, D, col < M};
  }
  d4v acc[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) acc[u] = zero4();
  wave_mma<kNC>(fa, fb, D, g, acc);
  const double d2 = delta * delta;
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = (int64_t)blockIdx.x * 64 + u * 16 + idx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rowbase + g + 4 * r;
      // (the contraction reads a clamped row for an invalid index; the row is zeroed here)
      const bool rok = __shfl(ok ? 1 : 0, g + 4 * r) != 0;
      const double v = (rok && col < M) ? d2 * ipow(acc[u][r], zeta) : 0.0;
      if (row_major) {  // [n_local][ldk], row padding (columns M .. ldk - 1) written as zero
        if (rr < n_local && col < ldk) K[rr * ldk + col] = v;
      } else if (rr < n_local && col < M) {
        K[rr + col * ldk] = v;
      }
    }
  }
}

// --------------------------------------------------------- energy rows ----
// Block (column tile ct, configuration c): the four waves own disjoint 64-column
// ranges and walk the configuration's atoms 16 at a time.
template <typename TD>
__global__ __launch_bounds__(256) void k_energy_rows(const TD* __restrict__ desc, int64_t ldd,
                                                     const int64_t* __restrict__ cfg_ptr,
                                                     const double* __restrict__ X, int64_t ldx,
                                                     int64_t M, int64_t D, int zeta, double delta,
                                                     double* __restrict__ K, int64_t ldk,
                                                     double* __restrict__ S, int64_t ldS,
                                                     int64_t n_atoms,
                                                     const int32_t* __restrict__ species,
                                                     int32_t zsel) {
  const int64_t c = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t colbase = (int64_t)blockIdx.x * 256 + wave * 64;
  if (colbase >= M) return;
  // clamp to [0, n_atoms] so malformed cfg_ptr data cannot address outside desc / S
  const int64_t a0 = max((int64_t)0, min(cfg_ptr[c], n_atoms));
  const int64_t a1 = max(a0, min(cfg_ptr[c + 1], n_atoms));
  FragRowK<double> fb[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
    fb[u] = FragRowK<double>{X + (col < M ? col : 0) * ldx, D, col < M};
  }
  const double d2 = delta * delta, d2z = d2 * zeta;
  double e[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) e[u] = 0.0;
  for (int64_t a = a0; a < a1; a += 16) {
    const int64_t row = a + idx;
    FragRowK<TD> fa{desc + (row < a1 ? row : a0) * ldd, D, row < a1};
    // species mask of a per-species block: atoms of other species are no
    // centre of this block's local energies (kernel value and S zero)
    const double on_lane =
        (species == nullptr || species[row < a1 ? row : a0] == zsel) ? 1.0 : 0.0;
    d4v acc[kNC];
#pragma unroll
    for (int u = 0; u < kNC; ++u) acc[u] = zero4();
    wave_mma<kNC>(fa, fb, D, g, acc);
#pragma unroll
    for (int u = 0; u < kNC; ++u) {
      const int64_t col = colbase + u * 16 + idx;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = a + g + 4 * r;
        const double on = __shfl(on_lane, g + 4 * r);
        if (rr < a1) {
          const double p = acc[u][r];
          const double pz1 = on * ipow(p, zeta - 1);
          e[u] += d2 * pz1 * p;
          if (col < ldS) S[rr * ldS + col] = (col < M) ? d2z * pz1 : 0.0;  // zero row padding
        }
      }
    }
  }
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    double v = e[u];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    const int64_t col = colbase + u * 16 + idx;
    if (g == 0 && col < M) K[c + col * ldk] = v;
  }
}

// ------------------------------------------------------------- P-stage ----
// Block = 64 rows (16 per wave); loops over all columns 64 at a time.
template <typename TD>
__global__ __launch_bounds__(256) void k_pstage(int mode, const TD* __restrict__ desc, int64_t ldd,
                                                int64_t n, const double* __restrict__ X,
                                                int64_t ldx, int64_t M, int64_t D, int zeta,
                                                double delta, const double* __restrict__ cc,
                                                const double* __restrict__ g_e,
                                                const double* __restrict__ H, int64_t ldh,
                                                double* __restrict__ W, int64_t ldw,
                                                double* __restrict__ e_atom,
                                                double* __restrict__ dc_part,
                                                const double* __restrict__ Sx, int64_t ldsx) {
  __shared__ double colsum[4][64];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t row = rowbase + idx;
  const bool rvalid = row < n;
  FragRowK<TD> fa{desc + (rvalid ? row : 0) * ldd, D, rvalid && mode != 3};
  FragRowK<double> fh{H ? H + (rvalid ? row : 0) * ldh : nullptr, D, rvalid && H != nullptr};
  const double d2 = delta * delta, d2z = d2 * zeta;
  double ge[4];
  bool rv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t rr = rowbase + g + 4 * r;
    rv[r] = rr < n;
    ge[r] = ((mode == 1 || mode == 2) && rv[r]) ? g_e[rr] : 0.0;
  }
  double esum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t col0 = 0; col0 < M; col0 += 16 * kNC) {
    FragRowK<double> fb[kNC];
#pragma unroll
    for (int u = 0; u < kNC; ++u) {
      const int64_t col = col0 + u * 16 + idx;
      fb[u] = FragRowK<double>{X + (col < M ? col : 0) * ldx, D, col < M};
    }
    d4v acc[kNC], accq[kNC];
#pragma unroll
    for (int u = 0; u < kNC; ++u) {
      acc[u] = zero4();
      accq[u] = zero4();
    }
    if (mode == 2)
      wave_mma2<kNC>(fa, fh, fb, D, g, acc, accq);
    else if (mode == 3)
      wave_mma<kNC>(fh, fb, D, g, accq);
    else
      wave_mma<kNC>(fa, fb, D, g, acc);
#pragma unroll
    for (int u = 0; u < kNC; ++u) {
      const int64_t col = col0 + u * 16 + idx;
      const bool cvalid = col < M;
      const double cm = (cvalid && cc) ? cc[col] : 0.0;
      double csum = 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t rr = rowbase + g + 4 * r;
        if (rv[r] && !cvalid && W && mode < 2 && col < ldw) W[rr * ldw + col] = 0.0;  // row padding
        if (!rv[r] || !cvalid) continue;
        if (mode == 3) {
          csum -= Sx[rr * ldsx + col] * accq[u][r];
          continue;
        }
        const double p = acc[u][r];
        const double pz1 = ipow(p, zeta - 1);
        const double kval = d2 * pz1 * p;
        if (mode == 0) {
          esum[r] += cm * kval;
          if (W) W[rr * ldw + col] = d2z * cm * pz1;
        } else if (mode == 1) {
          csum += ge[r] * kval;
          if (W) W[rr * ldw + col] = ge[r] * d2z * cm * pz1;
        } else {
          csum += ge[r] * kval - d2z * pz1 * accq[u][r];
        }
      }
      if (mode != 0) {
        csum += __shfl_xor(csum, 16);
        csum += __shfl_xor(csum, 32);
        if (g == 0) colsum[wave][u * 16 + idx] = csum;
      }
    }
    if (mode != 0) {
      __syncthreads();
      if (threadIdx.x < 64) {
        const int64_t col = col0 + threadIdx.x;
        if (col < M)
          dc_part[(int64_t)blockIdx.x * M + col] =
              ((colsum[0][threadIdx.x] + colsum[1][threadIdx.x]) + colsum[2][threadIdx.x]) +
              colsum[3][threadIdx.x];
      }
      __syncthreads();
    }
  }
  if (mode == 0 && e_atom) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      double v = esum[r];
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) v += __shfl_xor(v, o);
      const int64_t rr = rowbase + g + 4 * r;
      if (idx == 0 && rr < n) e_atom[rr] = v;
    }
  }
}

// Column sums of the refinement residual's force part, column-stationary:
//   dc_part[rg][m] = -sum over atoms i of row group rg of S[i][m] (h_i . x_m).
// A block keeps 64 columns of X in LDS for its lifetime (as the force-row
// kernel does) and streams the atom rows of its row group: each of its 12
// waves takes 16 rows per step, multiplies them with the X tile on the FP64
// matrix cores, scales by S and accumulates per-lane column sums in registers;
// one cross-wave reduction at the end writes the block's 64 sums.  Consecutive
// logical blocks on an XCD walk the column tiles of one row group, so its h
// rows are read from HBM about once.  Hot loads are unconditional: rows past n
// read a clamped valid row (masked out by a zero factor), k blocks past D meet
// zero rows of X; S rows are zero-padded to ldS (a multiple of 4).
constexpr int kRcW = 12;       // waves per block
constexpr int kRcMaxKb = 16;   // D <= 256
__global__ __launch_bounds__(64 * kRcW) void k_resid_colsum(
    const double* __restrict__ H, int64_t ldh, int64_t n, int64_t D,
    const double* __restrict__ X, int64_t ldx, int64_t M, const double* __restrict__ S,
    int64_t ldS, int64_t rows_per_group, int64_t n_ct, int64_t total, int64_t per_xcd,
    int nkb, double* __restrict__ dc_part) {
  extern __shared__ double xs[];  // [nkb][4 tiles][2 halves][64 lanes][2]
  __shared__ double red[kRcW][64];
  const int64_t logical = xcd_logical_block(per_xcd);
  if (logical >= total) return;
  const int64_t ct = logical % n_ct, rg = logical / n_ct;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t colbase = ct * 64;
  for (int e = threadIdx.x; e < nkb * 4 * 64; e += 64 * kRcW) {
    const int kb = e / 256, u = (e / 64) & 3, ln = e & 63;
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
  const d2v* xb = reinterpret_cast<const d2v*>(xs) + lane;
  auto xfrag = [&](int tile) -> d4v {
    const d2v lo = xb[tile * 128], hi = xb[tile * 128 + 64];
    const d4v f = {lo[0], lo[1], hi[0], hi[1]};
    return f;
  };
  const int64_t r_lo = rg * rows_per_group, r_hi = min(n, r_lo + rows_per_group);
  const int64_t kmax4 = ((D + 3) & ~int64_t(3)) - 4;  // last aligned 4-block inside ldh
  const int64_t scol = min(colbase + 4 * idx, ldS - 4);
  double csum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t rb = r_lo + wave * 16; rb < r_hi; rb += 16 * kRcW) {
    const double* hrow = H + min(rb + idx, n - 1) * ldh;
    // S of the step's output rows (rows rb + g + 4 r), used after the matrix work
    d4v sv[4];
#pragma unroll
    for (int r = 0; r < 4; ++r)
      sv[r] = *reinterpret_cast<const d4v*>(S + min(rb + g + 4 * r, n - 1) * ldS + scol);
    d4v G[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) G[u] = zero4();
    double a0[4], a1[4];
    load4u(hrow + min((int64_t)4 * g, kmax4), a0);
    for (int kb = 0; kb < nkb; ++kb) {
      load4u(hrow + min((int64_t)(kb + 1) * 16 + 4 * g, kmax4), a1);
      d4v b[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) b[u] = xfrag(kb * 4 + u);
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4)
#pragma unroll
        for (int u = 0; u < 4; ++u) G[u] = mfma_f64(a0[s4], b[u][s4], G[u]);
#pragma unroll
      for (int s4 = 0; s4 < 4; ++s4) a0[s4] = a1[s4];
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double ok = (rb + g + 4 * r < r_hi) ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < 4; ++u) csum[u] += sv[r][u] * ok * G[u][r];
    }
  }
  // sum the four row sub-groups (lane groups), then the waves
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    csum[u] += __shfl_xor(csum[u], 16);
    csum[u] += __shfl_xor(csum[u], 32);
  }
  if (g == 0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) red[wave][4 * idx + u] = csum[u];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRcW; ++w) t += red[w][threadIdx.x];
    const int64_t col = colbase + threadIdx.x;
    if (col < M) dc_part[rg * M + col] = -t;
  }
}

// A row of W with every element k scaled by cs[k] (cs: any alignment, length kmax).
struct FragRowKScaled {
  const double* row;
  const double* cs;
  int64_t kmax;
  bool valid;
  GAP_DEV void frag(int64_t k0, int g, double out[4]) const {
    if (!valid) {
      zero_frag(out);
      return;
    }
    const int64_t k = k0 + 4 * g;
    load4(row, k, kmax, out);
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] *= (k + s < kmax) ? cs[k + s] : 0.0;
  }
  struct Raw {
    double w[4], c[4];
  };
  GAP_DEV void fast(int64_t k0, int g, Raw& r) const {
    const int64_t k = k0 + 4 * g;
    load4u(row + k, r.w);
#pragma unroll
    for (int s = 0; s < 4; ++s) r.c[s] = cs[k + s];
  }
  GAP_DEV void cook(const Raw& r, double out[4]) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = r.w[s] * r.c[s];
  }
};

// ------------------------------------------------------- out = W X (row-major)
// With cs non-null, W is used with its columns scaled: out = (W diag(cs)) X.
__global__ __launch_bounds__(256) void k_gemm_wx_cs(const double* __restrict__ W, int64_t ldw,
                                                    int64_t n, int64_t M,
                                                    const double* __restrict__ cs,
                                                    const double* __restrict__ X, int64_t ldx,
                                                    int64_t D, double* __restrict__ out,
                                                    int64_t ldo) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t row = rowbase + idx;
  const int64_t colbase = (int64_t)blockIdx.y * 64;
  FragRowKScaled fa{W + (row < n ? row : 0) * ldw, cs, M, row < n};
  FragColK<double> fb[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
    fb[u] = FragColK<double>{X + (col < D ? col : 0), ldx, M, col < D};
  }
  d4v acc[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) acc[u] = zero4();
  wave_mma<kNC>(fa, fb, M, g, acc);
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rowbase + g + 4 * r;
      if (rr < n && col < D) out[rr * ldo + col] = acc[u][r];
    }
  }
}

// Raw buffer resources for the staged loads of the W X and P-stage kernels.
GAP_DEV __amdgpu_buffer_rsrc_t wx_rsrc(const double* p, uint32_t bytes) {
  const uint64_t x = reinterpret_cast<uint64_t>(p);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(x >> 32));
  return __builtin_amdgcn_make_buffer_rsrc((void*)((uint64_t)hi << 32 | lo), 0, (int)bytes,
                                           0x00020000);
}
// A load through a raw buffer resource: vector offsets at or past its size
// read zero (every offset that may leave the range is kept in the vector part).
GAP_DEV double wx_ld(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}

// out = (W diag(cs)) X (CS false: cs unused) with four-wave blocks, three of
// them per compute unit: a block covers 64 rows and 128 columns (wave w: rows
// 16 w .. + 15, eight column tiles), the contraction runs over 16-wide chunks
// of k staged in LDS (16 KB per buffer, double-buffered), and the three
// blocks on a compute unit are not held in step by one barrier, so each
// block's staging and barrier wait are covered by the others' products.
// Within a chunk, lane group g holds W[row][kc + 4 g + q] (one 32-byte load)
// and product q takes k = kc + 4 g + q, so the staged X follows the same
// order: element (k = kc + 4 g + q, column 16 u + idx) sits at
// [(q / 2) * 8 + u][16 g + idx][q % 2].  The column groups of a row block run
// on one XCD (xcd_group_tile), where they share the W rows in L2.  Loads in
// the loop are unconditional: rows past n and k past ldw - 4 read clamped
// valid addresses, the staged X is zero for k >= M and for columns >= D.
constexpr int kQxK = 16;                  // k per chunk
constexpr int kQxBuf = kQxK * 128;        // doubles per staged chunk
constexpr int kQxPer = kQxBuf / 256;      // staged elements per thread
constexpr size_t kQxLds = 2 * kQxBuf * sizeof(double);
template <bool CS>
__global__ __launch_bounds__(256, 3) void k_gemm_wx_q(
    const double* __restrict__ W, int64_t ldw, int64_t n, int64_t M,
    const double* __restrict__ cs, const double* __restrict__ X, int64_t ldx, int64_t D,
    double* __restrict__ out, int64_t ldo, int64_t n_ct) {
  __shared__ __attribute__((aligned(16))) double xs[2 * kQxBuf];
  int64_t rb, ct;
  if (!xcd_group_tile((n + 63) / 64, n_ct, rb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = rb * 64 + wave * 16;
  const double* wrow = W + min(rowbase + idx, n - 1) * ldw;
  const int64_t nch = (M + kQxK - 1) / kQxK;
  const int64_t cg = ct * 128;

  // staging: thread t moves elements e = t + 256 it: k offset kl = t / 128 + 2 it
  // (the same in a wave), column d = t % 128
  const int kl0 = __builtin_amdgcn_readfirstlane(threadIdx.x >> 7), d = threadIdx.x & 127;
  const auto xr = wx_rsrc(X, (uint32_t)(M * ldx * 8));
  const uint32_t xoff0 = cg + d < D ? (uint32_t)((kl0 * ldx + cg + d) * 8) : 0x80000000u;
  const uint32_t xstep = (uint32_t)(2 * ldx * 8);
  auto soff = [&](int it) {
    const int kl = kl0 + 2 * it, gq = kl >> 2, q = kl & 3;
    return ((q >> 1) * 8 + (d >> 4)) * 128 + (gq * 16 + (d & 15)) * 2 + (q & 1);
  };
  auto fetch = [&](int64_t c, double v[kQxPer], double sc[kQxPer]) {
    const uint32_t base = (uint32_t)(c * kQxK * ldx * 8);
#pragma unroll
    for (int it = 0; it < kQxPer; ++it) {
      v[it] = wx_ld(xr, xoff0 + base + it * xstep, 0);
      sc[it] = CS ? cs[min(c * kQxK + kl0 + 2 * it, M - 1)] : 1.0;
    }
  };
  auto stage = [&](double* dst, const double v[kQxPer], const double sc[kQxPer]) {
#pragma unroll
    for (int it = 0; it < kQxPer; ++it) dst[soff(it)] = CS ? v[it] * sc[it] : v[it];
  };
  auto afrag = [&](int64_t c, double a[4]) {
    load4u(wrow + min(c * kQxK + 4 * g, ldw - 4), a);
  };

  double sv[kQxPer], cv[kQxPer], a_cur[4], a_nxt[4];
  fetch(0, sv, cv);
  afrag(0, a_cur);
  stage(xs, sv, cv);
  __syncthreads();
  d4v acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = zero4();
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t cn = min(c + 1, nch - 1);
    fetch(cn, sv, cv);
    afrag(cn, a_nxt);
    __builtin_amdgcn_sched_barrier(0);
    const d2v* xb = reinterpret_cast<const d2v*>(xs + (c & 1) * kQxBuf) + lane;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      d2v b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = xb[(h * 8 + u) * 64];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = mfma_f64(a_cur[2 * h + j], b[u][j], acc[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
    stage(xs + ((c + 1) & 1) * kQxBuf, sv, cv);
    lds_barrier();
#pragma unroll
    for (int q = 0; q < 4; ++q) a_cur[q] = a_nxt[q];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t col = cg + (int64_t)u * 16 + idx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rowbase + g + 4 * r;
      if (rr < n && col < D) out[rr * ldo + col] = acc[u][r];
    }
  }
}

// P-stage of predict (MODE 0) and backward (MODE 1) for D % 4 == 0, in the
// layout of k_gemm_wx_q: four-wave blocks, three per compute unit, each
// covering 64 rows and a group of 128 sparse-point columns (wave w: rows
// 16 w .. + 15, eight column tiles); the contraction over D runs in 16-wide
// chunks whose X rows are staged in LDS (double-buffered, in the matrix core's
// operand order), each wave reads its 16 descriptor rows straight from memory,
// and the column groups of a row block run on one XCD.  Loads in the loop are
// unconditional: rows past n, columns past M and k past D read clamped valid
// addresses and are cancelled by zero factors when staged (X) or by the zero X
// rows (descriptors).  The epilogue is the one of k_pstage: p = d_i . x_m,
// W[i][m] (MODE 0: delta^2 zeta c_m p^(zeta-1); MODE 1: the same times g_e[i],
// zero row padding), and
// MODE 0: per-row energy partials of the column group in e_part[group][i];
// MODE 1: dc_part[row block][m] = sum over the block's 64 rows of
//   g_e[i] delta^2 p^zeta;
// MODE 3 (rows d_i = h_i, the refinement's column sums of the force rows, which
// carry a minus sign): dc_part[row block][m] = - sum over the block's rows of
// Sx[i][m] p_im, with no kernel and no W.
// Column sums are taken per wave (16 rows), then over the four waves in order.
template <typename TD, int MODE>
__global__ __launch_bounds__(256, 3) void k_pstage_q(
    const TD* __restrict__ desc, int64_t ldd, int64_t n, const double* __restrict__ X,
    int64_t ldx, int64_t M, int64_t D, int zeta, double delta, const double* __restrict__ cc,
    const double* __restrict__ g_e, double* __restrict__ W, int64_t ldw,
    double* __restrict__ e_part, double* __restrict__ dc_part, const double* __restrict__ Sx,
    int64_t ldsx, int64_t n_ct) {
  __shared__ __attribute__((aligned(16))) double xs[2 * kQxBuf];
  __shared__ double red[4][128];
  int64_t rb, ct;
  if (!xcd_group_tile((n + 63) / 64, n_ct, rb, ct)) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = rb * 64 + wave * 16;
  const int64_t cg = ct * 128;
  const TD* drow = desc + min(rowbase + idx, n - 1) * ldd;
  const int64_t nch = (D + kQxK - 1) / kQxK;

  // staging: thread t moves the 4-entry groups gi = t + 256 it (it < 2) of the
  // chunk: sparse point m = cg + gi / 4, entries k = 16 c + 4 (gi % 4) .. + 3,
  // which land as (k = 16 c + 4 g + q, column 16 u + idx) at
  // [(q / 2) * 8 + u][16 g + idx][q % 2]
  const double* xrow[2];
  double xok[2];
  int soff[2], dqv[2];
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int gi = threadIdx.x + 256 * it, ml = gi >> 2, dq = gi & 3;
    const int64_t m = cg + ml;
    xrow[it] = X + min(m, M - 1) * ldx;
    xok[it] = m < M ? 1.0 : 0.0;
    dqv[it] = dq;
    soff[it] = (ml >> 4) * 128 + (dq * 16 + (ml & 15)) * 2;
  }
  auto fetch = [&](int64_t c, d4v v[2]) {
#pragma unroll
    for (int it = 0; it < 2; ++it)
      v[it] = *reinterpret_cast<const d4v*>(xrow[it] + min(c * kQxK + 4 * dqv[it], D - 4));
  };
  auto stage = [&](int64_t c, double* dst, const d4v v[2]) {
#pragma unroll
    for (int it = 0; it < 2; ++it) {
      const double f = (c * kQxK + 4 * dqv[it] < D) ? xok[it] : 0.0;
      const d2v lo = {f * v[it][0], f * v[it][1]}, hi = {f * v[it][2], f * v[it][3]};
      *reinterpret_cast<d2v*>(dst + soff[it]) = lo;
      *reinterpret_cast<d2v*>(dst + soff[it] + 8 * 128) = hi;
    }
  };
  auto afrag = [&](int64_t c, double a[4]) {
    load4u(drow + min(c * kQxK + 4 * g, D - 4), a);
  };

  d4v sv[2];
  double a_cur[4], a_nxt[4];
  fetch(0, sv);
  afrag(0, a_cur);
  stage(0, xs, sv);
  __syncthreads();
  d4v acc[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) acc[u] = zero4();
  for (int64_t c = 0; c < nch; ++c) {
    const int64_t cn = min(c + 1, nch - 1);
    fetch(cn, sv);
    afrag(cn, a_nxt);
    __builtin_amdgcn_sched_barrier(0);
    const d2v* xb = reinterpret_cast<const d2v*>(xs + (c & 1) * kQxBuf) + lane;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      d2v b[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) b[u] = xb[(h * 8 + u) * 64];
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int u = 0; u < 8; ++u) acc[u] = mfma_f64(a_cur[2 * h + j], b[u][j], acc[u]);
    }
    __builtin_amdgcn_sched_barrier(0);
    stage(cn, xs + ((c + 1) & 1) * kQxBuf, sv);
    lds_barrier();
#pragma unroll
    for (int q = 0; q < 4; ++q) a_cur[q] = a_nxt[q];
  }

  const double d2 = delta * delta, d2z = d2 * zeta;
  double ge[4], esum[4] = {0.0, 0.0, 0.0, 0.0};
  bool rv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int64_t rr = rowbase + g + 4 * r;
    rv[r] = rr < n;
    ge[r] = (MODE == 1 && rv[r]) ? g_e[rr] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int64_t col = cg + u * 16 + idx;
    const bool cvalid = col < M;
    const double cm = (MODE != 3 && cvalid) ? cc[col] : 0.0;
    double csum = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rowbase + g + 4 * r;
      if (!rv[r]) continue;
      if (!cvalid) {
        if (W && col < ldw) W[rr * ldw + col] = 0.0;  // row padding
        continue;
      }
      const double p = acc[u][r];
      if (MODE == 3) {
        csum -= Sx[rr * ldsx + col] * p;
        continue;
      }
      const double pz1 = ipow(p, zeta - 1);
      const double kval = d2 * pz1 * p;
      if (MODE == 0) {
        esum[r] += cm * kval;
        if (W) W[rr * ldw + col] = d2z * cm * pz1;
      } else {
        csum += ge[r] * kval;
        if (W) W[rr * ldw + col] = ge[r] * d2z * cm * pz1;
      }
    }
    if (MODE != 0) {
      csum += __shfl_xor(csum, 16);
      csum += __shfl_xor(csum, 32);
      if (g == 0) red[wave][u * 16 + idx] = csum;
    }
  }
  if (MODE == 0) {
    // row sums over the wave's 128 columns
#pragma unroll
    for (int r = 0; r < 4; ++r) {
#pragma unroll
      for (int o = 1; o < 16; o <<= 1) esum[r] += __shfl_xor(esum[r], o);
      const int64_t rr = rowbase + g + 4 * r;
      if (idx == 0 && e_part && rr < n) e_part[ct * n + rr] = esum[r];
    }
  } else {
    __syncthreads();
    if (threadIdx.x < 128) {
      const int64_t col = cg + threadIdx.x;
      if (col < M)
        dc_part[rb * M + col] =
            ((red[0][threadIdx.x] + red[1][threadIdx.x]) + red[2][threadIdx.x]) +
            red[3][threadIdx.x];
    }
  }
}

// e[i] = sum over the column groups g of part[g][i], in group order
__global__ void k_sum_groups(const double* __restrict__ part, int64_t ng, int64_t n,
                             double* __restrict__ e) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int64_t q = 0; q < ng; ++q) s += part[q * n + i];
    e[i] = s;
  }
}

// y[i] = sum_k A[i + k * lda] x[k]  (column-major GEMV): 64 rows per block, 16 waves
// splitting k, partial sums combined in LDS in a fixed order.
__global__ __launch_bounds__(1024) void k_gemv_cm(const double* __restrict__ A, int64_t lda,
                                                  int64_t rows, int64_t cols,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y) {
  __shared__ double part[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (i < rows)
    for (int64_t k = wave; k < cols; k += 16) s += A[i + k * lda] * x[k];
  part[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && i < rows) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += part[w][lane];
    y[i] = t;
  }
}

// y[k] += sum_i A[i + k * lda] x[i]  (transposed GEMV, one wave per column)
__global__ void k_gemvt_cm_add(const double* __restrict__ A, int64_t lda, int64_t rows,
                               int64_t cols, const double* __restrict__ x, double* __restrict__ y) {
  const int64_t k = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (k >= cols) return;
  double s = 0.0;
  for (int64_t i = lane; i < rows; i += 64) s += A[i + k * lda] * x[i];
  s = wave_sum(s);
  if (lane == 0) y[k] += s;
}

// ------------------------------------------------------- out = W X (row-major)
__global__ __launch_bounds__(256) void k_gemm_wx(const double* __restrict__ W, int64_t ldw,
                                                 int64_t n, int64_t M,
                                                 const double* __restrict__ X, int64_t ldx,
                                                 int64_t D, double* __restrict__ out,
                                                 int64_t ldo) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = (int64_t)blockIdx.x * 64 + wave * 16;
  const int64_t row = rowbase + idx;
  const int64_t colbase = (int64_t)blockIdx.y * 64;
  FragRowK<double> fa{W + (row < n ? row : 0) * ldw, M, row < n};
  FragColK<double> fb[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
    fb[u] = FragColK<double>{X + (col < D ? col : 0), ldx, M, col < D};
  }
  d4v acc[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) acc[u] = zero4();
  wave_mma<kNC>(fa, fb, M, g, acc);
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rowbase + g + 4 * r;
      if (rr < n && col < D) out[rr * ldo + col] = acc[u][r];
    }
  }
}

// ------------------------------------------------------ out = W^T desc ----
template <typename TD>
__global__ __launch_bounds__(256) void k_gemm_wtd(const double* __restrict__ W, int64_t ldw,
                                                  int64_t n, int64_t M,
                                                  const TD* __restrict__ desc, int64_t ldd,
                                                  int64_t D, double* __restrict__ out,
                                                  int64_t ldo) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, g = lane >> 4, idx = lane & 15;
  const int64_t rowbase = (int64_t)blockIdx.x * 64 + wave * 16;  // sparse point m
  const int64_t row = rowbase + idx;
  const int64_t colbase = (int64_t)blockIdx.y * 64;                 // descriptor component
  FragColK<double> fa{W + (row < M ? row : 0), ldw, n, row < M};
  FragColK<TD> fb[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
    fb[u] = FragColK<TD>{desc + (col < D ? col : 0), ldd, n, col < D};
  }
  d4v acc[kNC];
#pragma unroll
  for (int u = 0; u < kNC; ++u) acc[u] = zero4();
  wave_mma<kNC>(fa, fb, n, g, acc);
#pragma unroll
  for (int u = 0; u < kNC; ++u) {
    const int64_t col = colbase + u * 16 + idx;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t rr = rowbase + g + 4 * r;
      if (rr < M && col < D) out[rr * ldo + col] = acc[u][r];
    }
  }
}

// out[m] = sum_p part[p * M + m]: 64 columns per block, 16 waves splitting p, partial
// sums combined in LDS in a fixed order.
__global__ __launch_bounds__(1024) void k_reduce_rows(const double* __restrict__ part,
                                                      int64_t nparts, int64_t M,
                                                      double* __restrict__ out) {
  __shared__ double ps[16][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t m = (int64_t)blockIdx.x * 64 + lane;
  double s = 0.0;
  if (m < M)
    for (int64_t p = wave; p < nparts; p += 16) s += part[p * M + m];
  ps[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && m < M) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < 16; ++w) t += ps[w][lane];
    out[m] = t;
  }
}

__global__ void k_segment_sum(const double* __restrict__ v, const int64_t* __restrict__ ptr,
                              int64_t nseg, int64_t n, double* __restrict__ out) {
  const int64_t c = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= nseg) return;
  const int64_t lo = max((int64_t)0, min(ptr[c], n)), hi = max(lo, min(ptr[c + 1], n));
  double s = 0.0;
  for (int64_t i = lo + lane; i < hi; i += 64) s += v[i];
  s = wave_sum(s);
  if (lane == 0) out[c] = s;
}

__global__ void k_copy_rows(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                            int64_t ldd, int64_t n, int64_t D) {
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < n * D;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e / D, j = e - i * D;
    dst[i * ldd + j] = src[i * lds + j];
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

}  // namespace

void copy_rows_f64(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n, int64_t D,
                   hipStream_t st) {
  if (n <= 0 || D <= 0) return;
  const unsigned g = (unsigned)std::min<int64_t>((n * D + 255) / 256, 65536);
  hipLaunchKernelGGL(k_copy_rows, dim3(g), dim3(256), 0, st, src, lds, dst, ldd, n, D);
}

void kmm_f64(const double* X, int64_t ldx, int64_t M, int64_t D, int zeta, double delta,
             double* K, int64_t ldk, hipStream_t st) {
  if (M <= 0) return;
  const unsigned nt = cdiv(M, 64);
  hipLaunchKernelGGL(k_kmm, dim3(nt, nt), dim3(256), 0, st, X, ldx, M, D, zeta, delta, K, ldk);
}

void energy_rows_f64(const void* desc, bool desc_f32, int64_t ldd, const int64_t* cfg_ptr,
                     int64_t n_cfg, int64_t n_atoms, const double* X, int64_t ldx, int64_t M,
                     int64_t D, int zeta, double delta, double* K, int64_t ldk, double* S,
                     int64_t ldS, hipStream_t st, const int32_t* species, int32_t zsel) {
  if (n_cfg <= 0 || M <= 0) return;
  dim3 grid(cdiv(M, 256), (unsigned)n_cfg);
  if (desc_f32)
    hipLaunchKernelGGL(k_energy_rows<float>, grid, dim3(256), 0, st, tptr<float>(desc), ldd,
                       cfg_ptr, X, ldx, M, D, zeta, delta, K, ldk, S, ldS, n_atoms, species,
                       zsel);
  else
    hipLaunchKernelGGL(k_energy_rows<double>, grid, dim3(256), 0, st, tptr<double>(desc), ldd,
                       cfg_ptr, X, ldx, M, D, zeta, delta, K, ldk, S, ldS, n_atoms, species,
                       zsel);
}

void local_rows_f64(const void* desc, bool desc_f32, int64_t ldd, int64_t n_atoms,
                    const int32_t* atom_idx, int64_t n_local, const double* X, int64_t ldx,
                    int64_t M, int64_t D, int zeta, double delta, double* K, int64_t ldk,
                    int* dev_err, hipStream_t st, bool row_major) {
  if (n_local <= 0 || M <= 0) return;
  dim3 grid(cdiv(row_major ? ldk : M, 64), cdiv(n_local, 64));
  if (desc_f32)
    hipLaunchKernelGGL(k_local_rows<float>, grid, dim3(256), 0, st, tptr<float>(desc), ldd,
                       n_atoms, atom_idx, n_local, X, ldx, M, D, zeta, delta, K, ldk, dev_err,
                       row_major ? 1 : 0);
  else
    hipLaunchKernelGGL(k_local_rows<double>, grid, dim3(256), 0, st, tptr<double>(desc), ldd,
                       n_atoms, atom_idx, n_local, X, ldx, M, D, zeta, delta, K, ldk, dev_err,
                       row_major ? 1 : 0);
}

int64_t pstage_row_blocks(int64_t n) { return (n + 63) / 64; }

int64_t pstage_groups(int64_t M) { return (M + 127) / 128; }

void pstage_f64(int mode, const void* desc, bool desc_f32, int64_t ldd, int64_t n,
                const double* X, int64_t ldx, int64_t M, int64_t D, int zeta, double delta,
                const double* c, const double* g_e, const double* H, int64_t ldh, double* W,
                int64_t ldw, double* e_atom, double* dc_part, hipStream_t st,
                const double* Sx, int64_t ldsx, double* e_part) {
  if (n <= 0 || M <= 0) return;
  // LDS-staged form: energies (mode 0) go through per-column-group partials
  // (mode 3 takes the rows h_i of H as its descriptors)
  const void* arows = mode == 3 ? static_cast<const void*>(H) : desc;
  const int64_t lda = mode == 3 ? ldh : ldd;
  const bool lds_ok = D % 4 == 0 && D >= 4 && lda % 4 == 0 && ldx % 4 == 0 && arows &&
                      (reinterpret_cast<uintptr_t>(arows) & 31) == 0 &&
                      (reinterpret_cast<uintptr_t>(X) & 31) == 0 &&
                      ((mode == 0 && c && (!e_atom || e_part)) || (mode == 1 && c && g_e) ||
                       (mode == 3 && Sx));
  if (lds_ok) {
    const int64_t ng = pstage_groups(M);
    const dim3 grid(xcd_group_tile_blocks(pstage_row_blocks(n), ng)), blk(256);
    double* ep = e_atom ? e_part : nullptr;
    if (mode == 3) {
      hipLaunchKernelGGL((k_pstage_q<double, 3>), grid, blk, 0, st, H, ldh, n, X, ldx, M, D,
                         zeta, delta, nullptr, nullptr, nullptr, 0, nullptr, dc_part, Sx, ldsx,
                         ng);
      return;
    }
    if (desc_f32) {
      if (mode == 0)
        hipLaunchKernelGGL((k_pstage_q<float, 0>), grid, blk, 0, st, tptr<float>(desc), ldd, n,
                           X, ldx, M, D, zeta, delta, c, g_e, W, ldw, ep, dc_part, nullptr, 0,
                           ng);
      else
        hipLaunchKernelGGL((k_pstage_q<float, 1>), grid, blk, 0, st, tptr<float>(desc), ldd, n,
                           X, ldx, M, D, zeta, delta, c, g_e, W, ldw, ep, dc_part, nullptr, 0,
                           ng);
    } else {
      if (mode == 0)
        hipLaunchKernelGGL((k_pstage_q<double, 0>), grid, blk, 0, st, tptr<double>(desc), ldd,
                           n, X, ldx, M, D, zeta, delta, c, g_e, W, ldw, ep, dc_part, nullptr, 0,
                           ng);
      else
        hipLaunchKernelGGL((k_pstage_q<double, 1>), grid, blk, 0, st, tptr<double>(desc), ldd,
                           n, X, ldx, M, D, zeta, delta, c, g_e, W, ldw, ep, dc_part, nullptr, 0,
                           ng);
    }
    if (mode == 0 && e_atom)
      hipLaunchKernelGGL(k_sum_groups, dim3(std::max(1u, std::min(cdiv(n, 256), 65536u))),
                         dim3(256), 0, st, e_part, ng, n, e_atom);
    return;
  }
  dim3 grid((unsigned)pstage_row_blocks(n));
  if (desc_f32)
    hipLaunchKernelGGL(k_pstage<float>, grid, dim3(256), 0, st, mode, tptr<float>(desc), ldd, n,
                       X, ldx, M, D, zeta, delta, c, g_e, H, ldh, W, ldw, e_atom, dc_part, Sx,
                       ldsx);
  else
    hipLaunchKernelGGL(k_pstage<double>, grid, dim3(256), 0, st, mode, tptr<double>(desc), ldd,
                       n, X, ldx, M, D, zeta, delta, c, g_e, H, ldh, W, ldw, e_atom, dc_part, Sx,
                       ldsx);
}

// The LDS-staged form needs W rows of whole 32-byte groups (ldw % 4 == 0, W
// 32-byte aligned) and X under 2 GB; the general form takes any layout.
inline bool wx_lds_ok(const double* W, int64_t ldw, int64_t M, int64_t ldx,
                      int64_t D) {
  // offsets into X, including a dropped column's, stay below 2^31
  return D > 0 && M > 0 && ldw >= 4 && ldw % 4 == 0 && D <= (int64_t)128 * 65535 &&
         (reinterpret_cast<uintptr_t>(W) & 31) == 0 && (M + 2 * kQxK) * ldx * 8 < (1ll << 31);
}

void gemm_wx_f64(const double* W, int64_t ldw, int64_t n, int64_t M, const double* X,
                 int64_t ldx, int64_t D, double* out, int64_t ldo, hipStream_t st) {
  if (n <= 0 || D <= 0) return;
  if (wx_lds_ok(W, ldw, M, ldx, D)) {
    const int64_t n_ct = cdiv(D, 128);
    hipLaunchKernelGGL(k_gemm_wx_q<false>, dim3(xcd_group_tile_blocks(cdiv(n, 64), n_ct)),
                       dim3(256), 0, st, W, ldw, n, M, nullptr, X, ldx, D, out, ldo, n_ct);
    return;
  }
  hipLaunchKernelGGL(k_gemm_wx, dim3(cdiv(n, 64), cdiv(D, 64)), dim3(256), 0, st, W, ldw, n, M,
                     X, ldx, D, out, ldo);
}

int64_t resid_colsum_groups(int64_t n, int64_t M) {
  const int64_t n_ct = (M + 63) / 64;
  // about three blocks per CU over the whole grid, at least one row step each
  const int64_t want = std::max<int64_t>(1, (768 + n_ct - 1) / n_ct);
  return std::max<int64_t>(1, std::min<int64_t>(want, (n + 16 * kRcW - 1) / (16 * kRcW)));
}

bool resid_colsum_f64(const double* H, int64_t ldh, int64_t n, int64_t D, const double* X,
                      int64_t ldx, int64_t M, const double* S, int64_t ldS, double* dc_part,
                      hipStream_t st) {
  if (n <= 0 || M <= 0) return true;
  if (D > 16 * kRcMaxKb || D % 4 != 0 || ldS % 4 != 0 || ldS < 4 || ldh % 4 != 0 || D < 4)
    return false;  // (D % 4: the row padding of H is not written, so it is never read)
  const int nkb = (int)((D + 15) / 16);
  const int64_t n_ct = (M + 63) / 64;
  const int64_t n_rg = resid_colsum_groups(n, M);
  const int64_t rows = (n + n_rg - 1) / n_rg;
  const int64_t total = n_ct * n_rg, per_xcd = (total + 7) / 8;
  const size_t lds = (size_t)nkb * 4 * 64 * 4 * sizeof(double);
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_resid_colsum),
                              hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)((size_t)kRcMaxKb * 4 * 64 * 4 * sizeof(double)));
    attr = true;
  }
  hipLaunchKernelGGL(k_resid_colsum, dim3((unsigned)(8 * per_xcd)), dim3(64 * kRcW), lds, st, H,
                     ldh, n, D, X, ldx, M, S, ldS, rows, n_ct, total, per_xcd, nkb, dc_part);
  return true;
}

void gemm_wx_scaled_f64(const double* W, int64_t ldw, int64_t n, int64_t M, const double* cs,
                        const double* X, int64_t ldx, int64_t D, double* out, int64_t ldo,
                        hipStream_t st) {
  if (n <= 0 || D <= 0) return;
  if (wx_lds_ok(W, ldw, M, ldx, D)) {
    const int64_t n_ct = cdiv(D, 128);
    hipLaunchKernelGGL(k_gemm_wx_q<true>, dim3(xcd_group_tile_blocks(cdiv(n, 64), n_ct)),
                       dim3(256), 0, st, W, ldw, n, M, cs, X, ldx, D, out, ldo, n_ct);
    return;
  }
  hipLaunchKernelGGL(k_gemm_wx_cs, dim3(cdiv(n, 64), cdiv(D, 64)), dim3(256), 0, st, W, ldw, n, M,
                     cs, X, ldx, D, out, ldo);
}

void gemv_cm_f64(const double* A, int64_t lda, int64_t rows, int64_t cols, const double* x,
                 double* y, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(k_gemv_cm, dim3(cdiv(rows, 64)), dim3(1024), 0, st, A, lda, rows, cols, x,
                     y);
}

void gemvt_cm_add_f64(const double* A, int64_t lda, int64_t rows, int64_t cols, const double* x,
                      double* y, hipStream_t st) {
  if (cols <= 0) return;
  hipLaunchKernelGGL(k_gemvt_cm_add, dim3(cdiv(cols, 4)), dim3(256), 0, st, A, lda, rows, cols, x,
                     y);
}

void gemm_wtd_f64(const double* W, int64_t ldw, int64_t n, int64_t M, const void* desc,
                  bool desc_f32, int64_t ldd, int64_t D, double* out, int64_t ldo,
                  hipStream_t st) {
  if (M <= 0 || D <= 0) return;
  dim3 grid(cdiv(M, 64), cdiv(D, 64));
  if (desc_f32)
    hipLaunchKernelGGL(k_gemm_wtd<float>, grid, dim3(256), 0, st, W, ldw, n, M,
                       tptr<float>(desc), ldd, D, out, ldo);
  else
    hipLaunchKernelGGL(k_gemm_wtd<double>, grid, dim3(256), 0, st, W, ldw, n, M,
                       tptr<double>(desc), ldd, D, out, ldo);
}

void reduce_rows_f64(const double* part, int64_t nparts, int64_t M, double* out,
                     hipStream_t st) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_reduce_rows, dim3(cdiv(M, 64)), dim3(1024), 0, st, part, nparts, M, out);
}

namespace {
// e_cfg[c] = sum_{i in c} (d_i . g_i) / zeta: configuration energies from the
// descriptor gradients g_i = d eps_i / d d_i (eps is homogeneous of degree zeta
// in d, so d . d eps / d d = zeta eps).  One block per configuration, fixed
// reduction order.
template <typename TD>
__global__ __launch_bounds__(256) void k_cfg_energy_from_grad(
    const TD* __restrict__ desc, int64_t ldd, const double* __restrict__ g, int64_t ldg,
    const int64_t* __restrict__ cfg_ptr, int64_t n, int64_t D, double inv_zeta,
    double* __restrict__ out) {
  __shared__ double red[256];
  const int64_t c = blockIdx.x;
  const int64_t a0 = max((int64_t)0, min(cfg_ptr[c], n));
  const int64_t a1 = max(a0, min(cfg_ptr[c + 1], n));
  double s = 0.0;
  for (int64_t i = a0; i < a1; ++i)
    for (int64_t k = threadIdx.x; k < D; k += 256) s += (double)desc[i * ldd + k] * g[i * ldg + k];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = red[0] * inv_zeta;
}

// H[i] -= (v[c(i)] / zeta) d_i for the atoms i of every configuration c: folds
// the energy rows' share of A^T v into the force rows' column sums
// (k(d_i, x_m) = S_im (d_i . x_m) / zeta).  One block per configuration.
template <typename TD>
__global__ __launch_bounds__(256) void k_sub_cfg_desc(double* __restrict__ H, int64_t ldh,
                                                      const TD* __restrict__ desc, int64_t ldd,
                                                      const double* __restrict__ v,
                                                      const int64_t* __restrict__ cfg_ptr,
                                                      int64_t n, int64_t D, double inv_zeta) {
  const int64_t c = blockIdx.x;
  const int64_t a0 = max((int64_t)0, min(cfg_ptr[c], n));
  const int64_t a1 = max(a0, min(cfg_ptr[c + 1], n));
  const double f = v[c] * inv_zeta;
  for (int64_t e = threadIdx.x; e < (a1 - a0) * D; e += 256) {
    const int64_t i = a0 + e / D, k = e % D;
    H[i * ldh + k] -= f * (double)desc[i * ldd + k];
  }
}

// Rows of atoms whose species is not zsel: local energy and W row set to zero
// (a per-species GP predicts only the local energies of its own species).
__global__ void k_mask_species_rows(const int32_t* __restrict__ species, int32_t zsel, int64_t n,
                                    double* __restrict__ e_atom, double* __restrict__ W,
                                    float* __restrict__ W32, int64_t ldw) {
  const int64_t i = blockIdx.x;
  if (i >= n || species[i] == zsel) return;
  if (e_atom && threadIdx.x == 0) e_atom[i] = 0.0;
  if (W)
    for (int64_t m = threadIdx.x; m < ldw; m += blockDim.x) W[i * ldw + m] = 0.0;
  if (W32)
    for (int64_t m = threadIdx.x; m < ldw; m += blockDim.x) W32[i * ldw + m] = 0.f;
}
}  // namespace

void cfg_energy_from_grad(const void* desc, bool desc_f32, int64_t ldd, const double* g,
                          int64_t ldg, const int64_t* cfg_ptr, int64_t n_cfg, int64_t n, int64_t D,
                          int zeta, double* out, hipStream_t st) {
  if (n_cfg <= 0) return;
  if (desc_f32)
    hipLaunchKernelGGL(k_cfg_energy_from_grad<float>, dim3((unsigned)n_cfg), dim3(256), 0, st,
                       tptr<float>(desc), ldd, g, ldg, cfg_ptr, n, D, 1.0 / zeta, out);
  else
    hipLaunchKernelGGL(k_cfg_energy_from_grad<double>, dim3((unsigned)n_cfg), dim3(256), 0, st,
                       tptr<double>(desc), ldd, g, ldg, cfg_ptr, n, D, 1.0 / zeta, out);
}

void sub_cfg_desc(double* H, int64_t ldh, const void* desc, bool desc_f32, int64_t ldd,
                  const double* v, const int64_t* cfg_ptr, int64_t n_cfg, int64_t n, int64_t D,
                  int zeta, hipStream_t st) {
  if (n_cfg <= 0 || n <= 0) return;
  if (desc_f32)
    hipLaunchKernelGGL(k_sub_cfg_desc<float>, dim3((unsigned)n_cfg), dim3(256), 0, st, H, ldh,
                       tptr<float>(desc), ldd, v, cfg_ptr, n, D, 1.0 / zeta);
  else
    hipLaunchKernelGGL(k_sub_cfg_desc<double>, dim3((unsigned)n_cfg), dim3(256), 0, st, H, ldh,
                       tptr<double>(desc), ldd, v, cfg_ptr, n, D, 1.0 / zeta);
}

void mask_species_rows(const int32_t* species, int32_t zsel, int64_t n, double* e_atom, double* W,
                       int64_t ldw, hipStream_t st, float* W32) {
  if (n <= 0 || (!e_atom && !W && !W32)) return;
  hipLaunchKernelGGL(k_mask_species_rows, dim3((unsigned)n), dim3(256), 0, st, species, zsel, n,
                     e_atom, W, W32, ldw);
}

void segment_sum_f64(const double* e_atom, const int64_t* cfg_ptr, int64_t n_cfg, int64_t n,
                     double* e_cfg, hipStream_t st) {
  if (n_cfg <= 0) return;
  hipLaunchKernelGGL(k_segment_sum, dim3(cdiv(n_cfg, 4)), dim3(256), 0, st, e_atom, cfg_ptr,
                     n_cfg, n, e_cfg);
}

}  // namespace gapk
