// Wavefront-level FP64 MFMA tiles: one wave computes a 16 x (16*NC) block of
// A * B with the 16x16x4 FP64 matrix instruction, operands streamed from
// global memory (L1/L2) with one block of 16 k values prefetched ahead.
#pragma once

#include "common.h"

// Operand source for the wave's 16 rows (A) or one 16-column tile (B).
// frag(k0, g, out): the four values this lane feeds at steps s = 0..3 of the
// k-block starting at k0, i.e. element (idx, k0 + 4 g + s) of the operand,
// where idx is the lane's row (A) or column (B).

// fast(k0, g, out): the same values for a k-block that lies wholly inside
// [0, kmax), read with no condition at all.  An operand row or column outside
// the matrix keeps a pointer to a valid row (callers clamp it) and yields
// finite values that only reach outputs the caller never stores.  A guarded
// load compiles to a branch whose join waits for the load at once, which would
// defeat the prefetch of the next block.

// Element (idx, k) at row[k]: contiguous along k (one vector load per block).
template <typename T>
struct FragRowK {
  const T* row;
  int64_t kmax;
  bool valid;
  GAP_DEV void frag(int64_t k0, int g, double out[4]) const {
    if (valid)
      load4(row, k0 + 4 * g, kmax, out);
    else
      zero_frag(out);
  }
  GAP_DEV void fast(int64_t k0, int g, double out[4]) const { load4u(row + k0 + 4 * g, out); }
};

// Element (idx, k) at col[k * ld]: contiguous along idx (coalesced across lanes).
template <typename T>
struct FragColK {
  const T* col;
  int64_t ld;
  int64_t kmax;
  bool valid;
  GAP_DEV void frag(int64_t k0, int g, double out[4]) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int64_t k = k0 + 4 * g + s;
      out[s] = (valid && k < kmax) ? (double)col[k * ld] : 0.0;
    }
  }
  GAP_DEV void fast(int64_t k0, int g, double out[4]) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = (double)col[(k0 + 4 * g + s) * ld];
  }
};

template <int NC>
GAP_DEV void mma_block(const double a[4], const double b[NC][4], d4v (&acc)[NC]) {
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int u = 0; u < NC; ++u) acc[u] = mfma_f64(a[s], b[u][s], acc[u]);
}

// acc[u] += A(16 x K) * B_u(K x 16) over k in [0, K).  Whole 16-deep blocks
// use the unconditional fast() loads with one block prefetched ahead; a
// ragged last block uses the guarded frag().
template <int NC, class FA, class FB>
GAP_DEV void wave_mma(const FA& fa, const FB (&fb)[NC], int64_t K, int g, d4v (&acc)[NC]) {
  const int64_t Kf = K & ~int64_t(15);
  double a0[4], a1[4], b0[NC][4], b1[NC][4];
  if (Kf > 0) {
    fa.fast(0, g, a0);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].fast(0, g, b0[u]);
#pragma unroll 2
    for (int64_t k0 = 0; k0 < Kf; k0 += 16) {
      const int64_t kn = min(k0 + 16, Kf - 16);  // the last prefetch re-reads a valid block
      fa.fast(kn, g, a1);
#pragma unroll
      for (int u = 0; u < NC; ++u) fb[u].fast(kn, g, b1[u]);
      mma_block<NC>(a0, b0, acc);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        a0[s] = a1[s];
#pragma unroll
        for (int u = 0; u < NC; ++u) b0[u][s] = b1[u][s];
      }
    }
  }
  if (Kf < K) {
    fa.frag(Kf, g, a0);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].frag(Kf, g, b0[u]);
    mma_block<NC>(a0, b0, acc);
  }
}

// Two A operands against the same B tiles: acc0 += A0 B, acc1 += A1 B.
template <int NC, class FA0, class FA1, class FB>
GAP_DEV void wave_mma2(const FA0& fa0, const FA1& fa1, const FB (&fb)[NC], int64_t K, int g,
                       d4v (&acc0)[NC], d4v (&acc1)[NC]) {
  const int64_t Kf = K & ~int64_t(15);
  for (int64_t k0 = 0; k0 < Kf; k0 += 16) {
    double a0[4], a1[4], b[NC][4];
    fa0.fast(k0, g, a0);
    fa1.fast(k0, g, a1);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].fast(k0, g, b[u]);
    mma_block<NC>(a0, b, acc0);
    mma_block<NC>(a1, b, acc1);
  }
  if (Kf < K) {
    double a0[4], a1[4], b[NC][4];
    fa0.frag(Kf, g, a0);
    fa1.frag(Kf, g, a1);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].frag(Kf, g, b[u]);
    mma_block<NC>(a0, b, acc0);
    mma_block<NC>(a1, b, acc1);
  }
}
