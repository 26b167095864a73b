// Split-BF16 ("BF16x3") contractions on the gfx950 BF16 matrix cores.
//
// A value x is rounded to FP32 (round to nearest even), then split into
//   hi = bf16(x),  lo = bf16(x - hi)
// (both round to nearest even).  A product x*y is formed as
//   hi_x*hi_y + hi_x*lo_y + lo_x*hi_y
// with FP32 accumulation in the matrix core; lo*lo (relative size ~2^-16) is
// dropped.  This keeps ~16 significant bits per operand and FP32 accumulation.
//
// v_mfma_f32_16x16x32_bf16: D(16x16, f32) = A(16x32) B(32x16) + C.
// Lane l (group g = l / 16, idx = l % 16) feeds A[idx][8 g + e] and
// B[8 g + e][idx] for e = 0..7, and holds D[4 g + r][idx] for r = 0..3
// (layout checked on gfx950 with an in-bounds probe).
#pragma once

#include "common.h"

typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef float f8v __attribute__((ext_vector_type(8)));

GAP_DEV f4v mfma_bf16(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

GAP_DEV f4v zero4f() { f4v z = {0.f, 0.f, 0.f, 0.f}; return z; }

typedef __bf16 bf2v __attribute__((ext_vector_type(2)));
typedef float f2v __attribute__((ext_vector_type(2)));
typedef uint32_t u4v __attribute__((ext_vector_type(4)));

// Pairs of values are rounded together (one packed conversion, round to
// nearest even, per pair for hi and per pair for lo); hi is widened back to
// FP32 by placing its 16 bits at the top of a word, so x - hi is exact.
GAP_DEV void split8(const float x[8], bf8v& hi, bf8v& lo) {
  u4v hp, lp;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const f2v v = {x[2 * q], x[2 * q + 1]};
    const uint32_t hb = __builtin_bit_cast(uint32_t, __builtin_convertvector(v, bf2v));
    const float h0 = __builtin_bit_cast(float, hb << 16);
    const float h1 = __builtin_bit_cast(float, hb & 0xffff0000u);
    const f2v r = {x[2 * q] - h0, x[2 * q + 1] - h1};
    hp[q] = hb;
    lp[q] = __builtin_bit_cast(uint32_t, __builtin_convertvector(r, bf2v));
  }
  hi = __builtin_bit_cast(bf8v, hp);
  lo = __builtin_bit_cast(bf8v, lp);
}

GAP_DEV void zero_split(bf8v& hi, bf8v& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    hi[e] = (__bf16)0.0f;
    lo[e] = (__bf16)0.0f;
  }
}

// Eight consecutive elements row[k .. k+7] as FP32 (zero at or beyond kmax);
// k % 8 == 0 and the row storage extends to k + 3 whenever k < kmax
// (leading dimensions are multiples of 4), so reads use 4-wide vectors.
GAP_DEV void load8f(const double* __restrict__ row, int64_t k, int64_t kmax, float out[8]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t kk = k + 4 * h;
    if (kk < kmax) {
      d4v v = *reinterpret_cast<const d4v*>(row + kk);
#pragma unroll
      for (int s = 0; s < 4; ++s) out[4 * h + s] = (kk + s < kmax) ? (float)v[s] : 0.f;
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) out[4 * h + s] = 0.f;
    }
  }
}

GAP_DEV void load8f(const float* __restrict__ row, int64_t k, int64_t kmax, float out[8]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int64_t kk = k + 4 * h;
    if (kk < kmax) {
      f4v v = *reinterpret_cast<const f4v*>(row + kk);
#pragma unroll
      for (int s = 0; s < 4; ++s) out[4 * h + s] = (kk + s < kmax) ? v[s] : 0.f;
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) out[4 * h + s] = 0.f;
    }
  }
}

// The same eight entries where all of row[k .. k+7] lie inside the row: no
// bound, so the loads carry no branch.
GAP_DEV void load8f_full(const float* __restrict__ row, int64_t k, float out[8]) {
  const f4v v0 = *reinterpret_cast<const f4v*>(row + k);
  const f4v v1 = *reinterpret_cast<const f4v*>(row + k + 4);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    out[s] = v0[s];
    out[4 + s] = v1[s];
  }
}

GAP_DEV void load8f_full(const double* __restrict__ row, int64_t k, float out[8]) {
  const d4v v0 = *reinterpret_cast<const d4v*>(row + k);
  const d4v v1 = *reinterpret_cast<const d4v*>(row + k + 4);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    out[s] = (float)v0[s];
    out[4 + s] = (float)v1[s];
  }
}

// Element (idx, k) at row[k]: contiguous along k, split on the fly.
template <typename T>
struct Frag32Row {
  const T* row;
  int64_t kmax;
  bool valid;
  GAP_DEV void frag(int64_t k0, int g, bf8v& hi, bf8v& lo) const {
    if (!valid) {
      zero_split(hi, lo);
      return;
    }
    float x[8];
    load8f(row, k0 + 8 * g, kmax, x);
    split8(x, hi, lo);
  }
};

// Pre-split rows: hi/lo arrays padded with zeros to a multiple of 32 along k.
struct Frag32Split {
  const __bf16* hi;
  const __bf16* lo;
  bool valid;
  GAP_DEV void frag(int64_t k0, int g, bf8v& h, bf8v& l) const {
    if (!valid) {
      zero_split(h, l);
      return;
    }
    h = *reinterpret_cast<const bf8v*>(hi + k0 + 8 * g);
    l = *reinterpret_cast<const bf8v*>(lo + k0 + 8 * g);
  }
};

template <int NC>
GAP_DEV void mma3_block(const bf8v& ah, const bf8v& al, const bf8v (&bh)[NC], const bf8v (&bl)[NC],
                        f4v (&acc)[NC]) {
#pragma unroll
  for (int u = 0; u < NC; ++u) {
    acc[u] = mfma_bf16(ah, bh[u], acc[u]);
    acc[u] = mfma_bf16(ah, bl[u], acc[u]);
    acc[u] = mfma_bf16(al, bh[u], acc[u]);
  }
}

// acc[u] += A(16 x K) B_u(K x 16) in BF16x3 over k in [0, K) (K padded to 32 by zeros).
template <int NC, class FA, class FB>
GAP_DEV void wave_mma_bf16x3(const FA& fa, const FB (&fb)[NC], int64_t K, int g, f4v (&acc)[NC]) {
  for (int64_t k0 = 0; k0 < K; k0 += 32) {
    bf8v ah, al, bh[NC], bl[NC];
    fa.frag(k0, g, ah, al);
#pragma unroll
    for (int u = 0; u < NC; ++u) fb[u].frag(k0, g, bh[u], bl[u]);
    mma3_block<NC>(ah, al, bh, bl, acc);
  }
}
