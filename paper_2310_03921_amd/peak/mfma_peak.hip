// Matrix-core throughput probe: the measured denominators of the roofline
// fractions (FP64 and BF16 dense MFMA peaks of the device it runs on).
// Every wave issues a long stream of independent matrix-core products (eight
// accumulators, no memory traffic in the loop), so the rate is the matrix
// cores' own.  Not part of the GAP path; the benchmark calls it once.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

constexpr int kAcc = 8;

__global__ __launch_bounds__(256) void k_peak_f64(int64_t iters, double seed, double* out) {
  d4v acc[kAcc];
#pragma unroll
  for (int u = 0; u < kAcc; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
  const double a = seed * (1 + (threadIdx.x & 3)), b = seed * (1 + (threadIdx.x >> 6));
  // iters is a multiple of 16; the 16-fold unrolled body keeps the
  // accumulators in place across the loop (no copies between iterations)
  for (int64_t it = 0; it < iters; it += 16) {
#pragma unroll
    for (int rep = 0; rep < 16; ++rep)
#pragma unroll
      for (int u = 0; u < kAcc; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[u], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kAcc; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_bf16(int64_t iters, float seed, double* out) {
  f4v acc[kAcc];
#pragma unroll
  for (int u = 0; u < kAcc; ++u) acc[u] = f4v{0.f, 0.f, 0.f, 0.f};
  bf8v a, b;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    a[e] = (__bf16)(seed * (e + 1));
    b[e] = (__bf16)(seed * (8 - e));
  }
  for (int64_t it = 0; it < iters; it += 16) {
#pragma unroll
    for (int rep = 0; rep < 16; ++rep)
#pragma unroll
      for (int u = 0; u < kAcc; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[u], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int u = 0; u < kAcc; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

// The same streams with operands that change from product to product: four
// register sets of per-lane pseudo-random values (BF16 in [-2, 2), FP64 with
// full-width mantissas), cycled so that consecutive products read different
// bits.  The matrix cores draw more power on such data than on the constant
// operands above, and the clock the chip holds drops with it.
__device__ uint32_t mix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}
__device__ float unit_rand(uint32_t s) {
  return ((mix32(s) >> 8) * (1.0f / 16777216.0f) - 0.5f) * 4.0f;
}

__global__ __launch_bounds__(256) void k_peak_bf16_var(int64_t iters, double* out) {
  f4v acc[kAcc];
#pragma unroll
  for (int u = 0; u < kAcc; ++u) acc[u] = f4v{0.f, 0.f, 0.f, 0.f};
  bf8v a[4], b[4];
  const uint32_t base = (blockIdx.x * 256 + threadIdx.x) * 64;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      a[v][e] = (__bf16)unit_rand(base + 16 * v + e);
      b[v][e] = (__bf16)unit_rand(base + 16 * v + 8 + e + 977);
    }
  for (int64_t it = 0; it < iters; it += 16) {
#pragma unroll
    for (int rep = 0; rep < 16; ++rep)
#pragma unroll
      for (int u = 0; u < kAcc; ++u)
        acc[u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[(rep + u) & 3], b[(3 * rep + u) & 3],
                                                         acc[u], 0, 0, 0);
  }
  float s = 0.f;
#pragma unroll
  for (int u = 0; u < kAcc; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

__global__ __launch_bounds__(256) void k_peak_f64_var(int64_t iters, double* out) {
  d4v acc[kAcc];
#pragma unroll
  for (int u = 0; u < kAcc; ++u) acc[u] = d4v{0.0, 0.0, 0.0, 0.0};
  double a[4], b[4];
  const uint32_t base = (blockIdx.x * 256 + threadIdx.x) * 64;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    a[v] = (double)unit_rand(base + v) * (1.0 + 2.3e-10 * mix32(base + v + 5));
    b[v] = (double)unit_rand(base + v + 99) * (1.0 + 2.3e-10 * mix32(base + v + 7));
  }
  for (int64_t it = 0; it < iters; it += 16) {
#pragma unroll
    for (int rep = 0; rep < 16; ++rep)
#pragma unroll
      for (int u = 0; u < kAcc; ++u)
        acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[(rep + u) & 3], b[(3 * rep + u) & 3],
                                                      acc[u], 0, 0, 0);
  }
  double s = 0.0;
#pragma unroll
  for (int u = 0; u < kAcc; ++u) s += acc[u][0] + acc[u][1] + acc[u][2] + acc[u][3];
  out[blockIdx.x * 256 + threadIdx.x] = s;
}

}  // namespace

extern "C" {

// kind 0: FP64 (v_mfma_f64_16x16x4f64, 2048 flop per wave instruction);
// kind 1: BF16 (v_mfma_f32_16x16x32_bf16, 16384 flop); kinds 2 and 3: the BF16
// and FP64 streams on pseudo-random operands that change every product.  `blocks` workgroups of
// four waves each run `iters` x 8 products (iters a multiple of 16).  Returns the elapsed milliseconds
// (HIP events on `stream`) and the flops performed.  out: device scratch of
// blocks * 256 doubles.
int gap_peak_mfma(void* stream, int kind, int64_t iters, int blocks, double* out, double* ms,
                  double* flops) {
  if (blocks < 1 || iters < 16 || iters % 16 != 0 || !out || !ms || !flops || kind < 0 ||
      kind > 3)
    return -1;
  const hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -2;
  hipEventRecord(e0, st);
  if (kind == 0)
    hipLaunchKernelGGL(k_peak_f64, dim3(blocks), dim3(256), 0, st, iters, 1e-3, out);
  else if (kind == 1)
    hipLaunchKernelGGL(k_peak_bf16, dim3(blocks), dim3(256), 0, st, iters, 1e-3f, out);
  else if (kind == 2)
    hipLaunchKernelGGL(k_peak_bf16_var, dim3(blocks), dim3(256), 0, st, iters, out);
  else
    hipLaunchKernelGGL(k_peak_f64_var, dim3(blocks), dim3(256), 0, st, iters, out);
  hipEventRecord(e1, st);
  const bool ok = hipEventSynchronize(e1) == hipSuccess;
  float t = 0.f;
  hipEventElapsedTime(&t, e0, e1);
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!ok || hipGetLastError() != hipSuccess) return -2;
  *ms = t;
  *flops = (double)blocks * 4 * (double)iters * kAcc * (kind == 0 || kind == 3 ? 2048.0 : 16384.0);
  return 0;
}

}  // extern "C"
