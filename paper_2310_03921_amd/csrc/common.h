// Device-side building blocks shared by the gfx950 kernels of libgap.
//
// FP64 matrix cores: v_mfma_f64_16x16x4_f64 computes D = A(16x4) B(4x16) + C.
// Operand layout of one 64-lane wavefront (lane l, group g = l / 16, idx = l % 16):
//   A: lane holds A[idx][g]        B: lane holds B[g][idx]
//   C/D: lane holds D[g + 4 r][idx] for r = 0..3 (four doubles, rows interleaved
//        across the lane groups; checked on gfx950 with an in-bounds probe)
// Contraction order is free, so over a block of 16 k values the kernels let
// lane group g own k = k0 + 4 g + s for MFMA step s = 0..3.  A lane then
// reads four consecutive k of one row (one 32-byte load) when the operand is
// contiguous along k, or one element per step, coalesced across the 16 lanes
// of its group, when the operand is contiguous along the other index.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

#define GAP_DEV __device__ __forceinline__

GAP_DEV d4v mfma_f64(double a, double b, d4v c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

GAP_DEV d4v zero4() { d4v z = {0.0, 0.0, 0.0, 0.0}; return z; }

// x^n for a small integer n >= 0 by repeated squaring (the dot-product kernel
// exponent is an integer; p may be negative).
GAP_DEV double ipow(double x, int n) {
  double r = 1.0;
  double b = x;
  while (n > 0) {
    if (n & 1) r *= b;
    b *= b;
    n >>= 1;
  }
  return r;
}

// Four consecutive elements row[k .. k+3] (k % 4 == 0) as doubles, elements
// at or beyond kmax set to zero.  The row's storage must extend to k + 3
// whenever k < kmax (leading dimensions are multiples of 4).
GAP_DEV void load4(const double* __restrict__ row, int64_t k, int64_t kmax, double out[4]) {
  if (k + 3 < kmax) {
    d4v v = *reinterpret_cast<const d4v*>(row + k);
    out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
  } else if (k < kmax) {
    d4v v = *reinterpret_cast<const d4v*>(row + k);
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = (k + s < kmax) ? v[s] : 0.0;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = 0.0;
  }
}

GAP_DEV void load4(const float* __restrict__ row, int64_t k, int64_t kmax, double out[4]) {
  if (k < kmax) {
    f4v v = *reinterpret_cast<const f4v*>(row + k);
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = (k + s < kmax) ? (double)v[s] : 0.0;
  } else {
#pragma unroll
    for (int s = 0; s < 4; ++s) out[s] = 0.0;
  }
}

// Unconditional 4-wide load (32-byte aligned for double, 16-byte for float).
GAP_DEV void load4u(const double* p, double out[4]) {
  const d4v v = *reinterpret_cast<const d4v*>(p);
  out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
}
GAP_DEV void load4u(const float* p, double out[4]) {
  const f4v v = *reinterpret_cast<const f4v*>(p);
  out[0] = v[0]; out[1] = v[1]; out[2] = v[2]; out[3] = v[3];
}

GAP_DEV void zero_frag(double out[4]) {
#pragma unroll
  for (int s = 0; s < 4; ++s) out[s] = 0.0;
}

// Block-to-tile mapping that keeps consecutive logical tiles on one XCD.
// Workgroups are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8);
// logical = (b % 8) * per_xcd + b / 8 makes the blocks an XCD runs back to
// back consecutive logical tiles, so tiles that share operands share that
// XCD's L2.  The grid must be 8 * per_xcd; logical >= total exits.
GAP_DEV int64_t xcd_logical_block(int64_t per_xcd) {
  const int64_t b = blockIdx.x;
  return (b & 7) * per_xcd + (b >> 3);
}

// (group, column tile) of this block, for kernels whose groups come in order of
// decreasing work (targets sorted by degree).  All column tiles of a group run
// on one XCD, where they share the group's rows in that XCD's L2, and the
// groups are dealt to the eight XCDs in turn, so every XCD receives the same
// mix of heavy and light groups (contiguous group ranges per XCD would leave
// the XCD with the heaviest groups running long after the others are done).
// The grid has xcd_group_tile_blocks(n_grp, n_ct) blocks.
GAP_DEV bool xcd_group_tile(int64_t n_grp, int64_t n_ct, int64_t& grp, int64_t& ct) {
  const int64_t b = blockIdx.x, j = b >> 3;
  grp = (j / n_ct) * 8 + (b & 7);
  ct = j % n_ct;
  return grp < n_grp;
}
inline unsigned xcd_group_tile_blocks(int64_t n_grp, int64_t n_ct) {
  return (unsigned)(((n_grp + 7) / 8) * 8 * n_ct);
}

// Workgroup barrier that orders LDS only: workgroup-scope fences restricted to
// the local address space (the compiler may not move LDS accesses across them,
// and the hardware waits only for this wave's LDS operations, lgkmcnt = 0),
// leaving global loads and stores in flight, unlike __syncthreads(), whose
// fences drain every outstanding memory access.
GAP_DEV void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

GAP_DEV double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
}

GAP_DEV int wave_max16(int v) {
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) v = max(v, __shfl_xor(v, o));
  return v;
}

