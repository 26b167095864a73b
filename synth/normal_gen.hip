// Counter-based normal deviates on the GPU for the synthetic inputs that do not
// fit in device memory (the Jacobians of the largest fit are regenerated, one
// batch of configurations at a time, whenever a pass needs them).
//
// Generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11) -- ten rounds of two 32x32 -> 64-bit
// multiplies with the published multipliers and Weyl key increments --
// followed by the Box-Muller transform (one pair of uniforms -> two normals).
// Element e of a stream keyed (seed, tag) comes from group g = e / 4: counter
// (g mod 2^32, g / 2^32, 0, 0), key (seed mod 2^32, tag); its four words give
// u1 = (w0 + 1) 2^-32, v1 = w1 2^-32, u2 = (w2 + 1) 2^-32, v2 = w3 2^-32 and
//   z0 = sqrt(-2 ln u1) cos(2 pi v1), z1 = sqrt(-2 ln u1) sin(2 pi v1),
//   z2, z3 likewise from (u2, v2),
// so any element range can be regenerated alone.  This file holds no part of
// the GAP method: it only draws inputs.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

struct W4 {
  uint32_t w0, w1, w2, w3;
};

__device__ __forceinline__ W4 philox4x32_10(W4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(kM0, c.w0), lo0 = kM0 * c.w0;
    const uint32_t hi1 = __umulhi(kM1, c.w2), lo1 = kM1 * c.w2;
    c = W4{hi1 ^ c.w1 ^ k0, lo1, hi0 ^ c.w3 ^ k1, lo0};
    k0 += kW0;
    k1 += kW1;
  }
  return c;
}

__device__ __forceinline__ W4 group_words(uint64_t g, uint32_t k0, uint32_t k1) {
  return philox4x32_10(W4{(uint32_t)g, (uint32_t)(g >> 32), 0u, 0u}, k0, k1);
}

// Box-Muller on one pair of words; the angle is taken in revolutions, the
// native argument of the hardware sine and cosine.
__device__ __forceinline__ void box_muller(uint32_t a, uint32_t b, float& z0, float& z1) {
  constexpr float k2m32 = 2.3283064365386963e-10f;  // 2^-32
  const float u = ((float)a + 1.0f) * k2m32;          // (0, 1]
  const float v = (float)b * k2m32;                   // [0, 1)
  const float r = sqrtf(-2.0f * logf(u));
  z0 = r * __builtin_amdgcn_cosf(v);
  z1 = r * __builtin_amdgcn_sinf(v);
}

__global__ void k_philox_words(uint32_t k0, uint32_t k1, uint64_t g0, int64_t n_groups,
                               uint32_t* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_groups;
       i += (int64_t)gridDim.x * blockDim.x) {
    const W4 w = group_words(g0 + (uint64_t)i, k0, k1);
    out[4 * i + 0] = w.w0;
    out[4 * i + 1] = w.w1;
    out[4 * i + 2] = w.w2;
    out[4 * i + 3] = w.w3;
  }
}

// rows x D block of the stream starting at element e0 (row r, column d is
// element e0 + r D + d), times `scale`, into out[r * ld + d].  Fast path: rows
// whose groups never straddle a row (e0 % 4 == 0, D % 4 == 0) with one
// 16-byte store per group.
__global__ void k_normal_rows_vec(uint32_t k0, uint32_t k1, uint64_t e0, int64_t rows, int64_t D,
                                  int64_t ld, float scale, float* __restrict__ out) {
  const int64_t gpr = D / 4, n = rows * gpr;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = i / gpr, q = i - r * gpr;
    const W4 w = group_words(e0 / 4 + (uint64_t)i, k0, k1);
    float4 z;
    box_muller(w.w0, w.w1, z.x, z.y);
    box_muller(w.w2, w.w3, z.z, z.w);
    z.x *= scale;
    z.y *= scale;
    z.z *= scale;
    z.w *= scale;
    *reinterpret_cast<float4*>(out + r * ld + 4 * q) = z;
  }
}

__global__ void k_normal_rows(uint32_t k0, uint32_t k1, uint64_t e0, int64_t rows, int64_t D,
                              int64_t ld, float scale, float* __restrict__ out) {
  const int64_t n = rows * D;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t e = e0 + (uint64_t)i;
    const W4 w = group_words(e / 4, k0, k1);
    float z[4];
    box_muller(w.w0, w.w1, z[0], z[1]);
    box_muller(w.w2, w.w3, z[2], z[3]);
    const int64_t r = i / D, d = i - r * D;
    out[r * ld + d] = scale * z[e & 3];
  }
}

unsigned grid_of(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

}  // namespace

extern "C" {

// Raw Philox4x32-10 words of groups g0 .. g0 + n_groups - 1 (four words each).
int synth_philox_words(void* stream, uint32_t key0, uint32_t key1, uint64_t g0, int64_t n_groups,
                       uint32_t* out) {
  if (n_groups < 0 || (n_groups > 0 && !out)) return -1;
  if (n_groups == 0) return 0;
  hipLaunchKernelGGL(k_philox_words, dim3(grid_of(n_groups)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(stream), key0, key1, g0, n_groups, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// scale * N(0, 1) deviates of stream (seed, tag), elements e0 .. e0 + rows D - 1,
// as a row-major rows x D FP32 array of leading dimension ld >= D (out 16-byte
// aligned; padding columns are not written).
int synth_normal_rows_f32(void* stream, uint64_t seed, uint32_t tag, uint64_t e0, int64_t rows,
                          int64_t D, int64_t ld, float scale, float* out) {
  if (rows < 0 || D < 1 || ld < D || (rows > 0 && !out)) return -1;
  if (rows == 0) return 0;
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  const uint32_t k0 = (uint32_t)seed, k1 = tag;
  const bool vec = e0 % 4 == 0 && D % 4 == 0 && ld % 4 == 0 &&
                   (reinterpret_cast<uintptr_t>(out) & 15u) == 0;
  if (vec)
    hipLaunchKernelGGL(k_normal_rows_vec, dim3(grid_of(rows * (D / 4))), dim3(256), 0, st, k0, k1,
                       e0, rows, D, ld, scale, out);
  else
    hipLaunchKernelGGL(k_normal_rows, dim3(grid_of(rows * D)), dim3(256), 0, st, k0, k1, e0, rows,
                       D, ld, scale, out);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
