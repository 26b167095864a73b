// Wavefront-level FP64 MFMA tiles: one wave computes a 16 x (16*NC) block of
// A * B with the 16x16x4 FP64 matrix instruction, operands streamed from
// global memory (L1/L2) with one block of 16 k values prefetched ahead.
#pragma once

#include "common.h"

// Operand source for the wave's 16 rows (A) or one 16-column tile (B).
// frag(k0, g, out): the four values this lane feeds at steps s = 0..3 of the
// k-block starting at k0, i.e. element (idx, k0 + 4 g + s) of the operand,
// where idx is the lane's row (A) or column (B).

// fast(k0, g, raw) then cook(raw, out): the same values for a k-block that lies
// wholly inside [0, kmax), read with no condition at all into raw registers
// and turned into FP64 operands (converted, scaled) only when they are used,
// one block later: a load whose value is converted or selected as soon as it
// arrives (a guarded load, whose branch join waits for it, too) would make the
// wave wait for the prefetch before the current block's products.  An operand
// row or column outside the matrix keeps a pointer to a valid row (callers
// clamp it) and yields finite values that only reach outputs the caller never
// stores.

template <typename T>
struct Raw4 {
  T v[4];
};

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
  using Raw = Raw4<T>;
  GAP_DEV void fast(int64_t k0, int g, Raw& r) const {
    if constexpr (sizeof(T) == 4) {
      const f4v v = *reinterpret_cast<const f4v*>(row + k0 + 4 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s) r.v[s] = v[s];
    } else {
      const d4v v = *reinterpret_cast<const d4v*>(row + k0 + 4 * g);
#pragma unroll
      for (int s = 0; s < 4; ++s) r.v[s] = v[s];
    }
  }
  GAP_DEV void cook(const Raw& r, double out[4]) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = (double)r.v[s];
  }
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
  using Raw = Raw4<T>;
  GAP_DEV void fast(int64_t k0, int g, Raw& r) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) r.v[s] = col[(k0 + 4 * g + s) * ld];
  }
  GAP_DEV void cook(const Raw& r, double out[4]) const {
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = (double)r.v[s];
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
// use the unconditional fast() loads, one block ahead, into two register sets
// used in turn (the next block lands in the set the current products do not
// read, so nothing is copied between them); a ragged last block uses the
// guarded frag().
template <int NC, class FA, class FB>
GAP_DEV void wave_mma(const FA& fa, const FB (&fb)[NC], int64_t K, int g, d4v (&acc)[NC]) {
  const int64_t Kf = K & ~int64_t(15);
  if (Kf > 0) {
    typename FA::Raw ra[2];
    typename FB::Raw rb[2][NC];
    fa.fast(0, g, ra[0]);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].fast(0, g, rb[0][u]);
    auto step = [&](int64_t k0, const int cur) {
      const int64_t kn = min(k0 + 16, Kf - 16);  // the last prefetch re-reads a valid block
      fa.fast(kn, g, ra[cur ^ 1]);
#pragma unroll
      for (int u = 0; u < NC; ++u) fb[u].fast(kn, g, rb[cur ^ 1][u]);
      double a[4], b[NC][4];
      fa.cook(ra[cur], a);
#pragma unroll
      for (int u = 0; u < NC; ++u) fb[u].cook(rb[cur][u], b[u]);
      mma_block<NC>(a, b, acc);
    };
    int64_t k0 = 0;
    for (; k0 + 16 < Kf; k0 += 32) {
      step(k0, 0);
      step(k0 + 16, 1);
    }
    if (k0 < Kf) step(k0, 0);
  }
  if (Kf < K) {
    double a0[4], b0[NC][4];
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
    typename FA0::Raw r0;
    typename FA1::Raw r1;
    typename FB::Raw rb[NC];
    fa0.fast(k0, g, r0);
    fa1.fast(k0, g, r1);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].fast(k0, g, rb[u]);
    double a0[4], a1[4], b[NC][4];
    fa0.cook(r0, a0);
    fa1.cook(r1, a1);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].cook(rb[u], b[u]);
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
