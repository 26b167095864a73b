// Two-body (distance) descriptor with the squared-exponential kernel, FP64.
//
// Sec. "Descriptors based on interatomic distances": the pair distance r is
// the descriptor and the kernel is multiplied by the cosine cutoff function
// f_cut of each distance; Sec. "Regression": k_SE(x, x') = exp(-(x - x')^2 /
// (2 theta^2)) for a one-dimensional descriptor.  A directed pair p = (i, k)
// of the neighbour list, with displacement r_p = pair_r[p] (r_j - r_i) and
// r = |r_p|, is one descriptor instance carrying half of the bond energy (a
// full neighbour list holds each bond twice):
//   k(r, x_m) = delta^2 fc(r) fc(x_m) exp(-(r - x_m)^2 / (2 theta^2))
//   energy row c:        sum_{p in c} k(r_p, x_m) / 2
//   force row (a, alpha): - d/dr_a,alpha of that sum
//     = sum_{p: i(p) = a} k'(r_p) rhat_p,alpha / 2 - sum_{p: j(p) = a} k'(r_p) rhat_p,alpha / 2
// with k' = dk/dr.  The work per pair is a handful of flops per sparse
// point (no contraction over a descriptor dimension), so these are plain
// vector kernels: lanes over sparse points, loops over pairs.
#include <algorithm>

#include "common.h"
#include "launch.h"

namespace gapk {

namespace {

struct Se2b {
  double d2, inv2t2, rc, w;
};

GAP_DEV double fcut(double r, const Se2b& k) {
  if (r >= k.rc) return 0.0;
  if (r < k.rc - k.w) return 1.0;
  return 0.5 * (cos(M_PI * (r - k.rc + k.w) / k.w) + 1.0);
}
GAP_DEV double dfcut(double r, const Se2b& k) {
  if (r >= k.rc || r < k.rc - k.w) return 0.0;
  return -0.5 * M_PI / k.w * sin(M_PI * (r - k.rc + k.w) / k.w);
}

// k and dk/dr of one pair (fr = fc(r), dfr = fc'(r)) with sparse point x (fx = fc(x))
GAP_DEV void kse(double r, double fr, double dfr, double x, double fx, const Se2b& k, double& v,
                 double& dv) {
  const double t = r - x;
  const double e = k.d2 * fx * exp(-t * t * k.inv2t2);
  v = fr * e;
  dv = e * (dfr - fr * 2.0 * t * k.inv2t2);
}

// Pair geometry: r, fc(r), fc'(r) and the unit vector (zero for r = 0).
GAP_DEV void pair_geom(const double* __restrict__ pair_r, int64_t p, const Se2b& k, double& r,
                       double& fr, double& dfr, double u[3]) {
  const double a = pair_r[3 * p], b = pair_r[3 * p + 1], c = pair_r[3 * p + 2];
  r = sqrt(a * a + b * b + c * c);
  fr = fcut(r, k);
  dfr = dfcut(r, k);
  const double inv = r > 0.0 ? 1.0 / r : 0.0;
  u[0] = a * inv;
  u[1] = b * inv;
  u[2] = c * inv;
}

// Energy rows: block (column tile of 64, configuration); lane m of each wave,
// waves split the configuration's pairs, fixed-order reduction over the waves.
__global__ __launch_bounds__(256) void k_2b_energy(const double* __restrict__ pair_r,
                                                    const int64_t* __restrict__ cfg_ptr,
                                                    const int64_t* __restrict__ pair_ptr,
                                                    int64_t n_atoms, int64_t n_pairs,
                                                    const double* __restrict__ x, int64_t M,
                                                    Se2b k, double* __restrict__ K, int64_t ldk) {
  __shared__ double red[4][64];
  const int64_t c = blockIdx.y;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 64 + lane;
  const double xm = m < M ? x[m] : 0.0;
  const double fx = fcut(xm, k);
  const int64_t a0 = min(max(cfg_ptr[c], (int64_t)0), n_atoms);
  const int64_t a1 = min(max(cfg_ptr[c + 1], a0), n_atoms);
  const int64_t p0 = min(max(pair_ptr[a0], (int64_t)0), n_pairs);
  const int64_t p1 = min(max(pair_ptr[a1], p0), n_pairs);
  double s = 0.0;
  for (int64_t p = p0 + wave; p < p1; p += 4) {
    double r, fr, dfr, u[3], v, dv;
    pair_geom(pair_r, p, k, r, fr, dfr, u);
    kse(r, fr, dfr, xm, fx, k, v, dv);
    s += v;
  }
  red[wave][lane] = s;
  __syncthreads();
  if (wave == 0 && m < M)
    K[c + m * ldk] = 0.5 * (red[0][lane] + red[1][lane] + red[2][lane] + red[3][lane]);
}

// Force rows: one wave per atom a, lane m; the atom's own pairs (a as i) and
// the pairs pointing at it (a as j, through the target-major view).
__global__ __launch_bounds__(256) void k_2b_force(
    const double* __restrict__ pair_r, const int64_t* __restrict__ pair_ptr,
    const int64_t* __restrict__ tgt_ptr, const int32_t* __restrict__ tgt_pair, int64_t n_atoms,
    int64_t n_pairs, const double* __restrict__ x, int64_t M, Se2b k, int64_t row0,
    double* __restrict__ K, int64_t ldk) {
  const int64_t a = blockIdx.y * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t m = (int64_t)blockIdx.x * 64 + lane;
  if (a >= n_atoms) return;
  const double xm = m < M ? x[m] : 0.0;
  const double fx = fcut(xm, k);
  double f[3] = {0.0, 0.0, 0.0};
  const int64_t s0 = min(max(pair_ptr[a], (int64_t)0), n_pairs);
  const int64_t s1 = min(max(pair_ptr[a + 1], s0), n_pairs);
  for (int64_t p = s0; p < s1; ++p) {
    double r, fr, dfr, u[3], v, dv;
    pair_geom(pair_r, p, k, r, fr, dfr, u);
    kse(r, fr, dfr, xm, fx, k, v, dv);
#pragma unroll
    for (int al = 0; al < 3; ++al) f[al] += 0.5 * dv * u[al];
  }
  for (int64_t e = tgt_ptr[a]; e < tgt_ptr[a + 1]; ++e) {
    const int64_t p = tgt_pair[e];
    double r, fr, dfr, u[3], v, dv;
    pair_geom(pair_r, p, k, r, fr, dfr, u);
    kse(r, fr, dfr, xm, fx, k, v, dv);
#pragma unroll
    for (int al = 0; al < 3; ++al) f[al] -= 0.5 * dv * u[al];
  }
  if (m < M) {
#pragma unroll
    for (int al = 0; al < 3; ++al) K[(row0 + 3 * a + al) + m * ldk] = f[al];
  }
}

// K_MM of the sparse distances, written in an order-free form (the product of
// the two cutoffs and the square of the difference are symmetric in i, j), so
// the matrix is exactly symmetric.
__global__ void k_2b_kmm(const double* __restrict__ x, int64_t M, Se2b k, double* __restrict__ K,
                         int64_t ldk) {
  const int64_t j = blockIdx.y;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < M;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double t = x[i] - x[j];
    K[i + j * ldk] = k.d2 * (fcut(x[i], k) * fcut(x[j], k)) * exp(-(t * t) * k.inv2t2);
  }
}

// Per-pair terms of a prediction: e_p = sum_m c_m k(r_p, x_m) / 2 and
// g_p = sum_m c_m k'(r_p, x_m) / 2 (one thread per pair, sparse points in order).
__global__ void k_2b_pair_terms(const double* __restrict__ pair_r, int64_t n_pairs,
                                const double* __restrict__ x, const double* __restrict__ c,
                                int64_t M, Se2b k, double* __restrict__ ep,
                                double* __restrict__ gp) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    double r, fr, dfr, u[3];
    pair_geom(pair_r, p, k, r, fr, dfr, u);
    double se = 0.0, sg = 0.0;
    for (int64_t m = 0; m < M; ++m) {
      double v, dv;
      kse(r, fr, dfr, x[m], fcut(x[m], k), k, v, dv);
      se += c[m] * v;
      sg += c[m] * dv;
    }
    ep[p] = 0.5 * se;
    gp[p] = 0.5 * sg;
  }
}

// e_cfg[c] = sum of e_p over the configuration's pairs (one wave per configuration)
__global__ void k_2b_cfg_energy(const double* __restrict__ ep, const int64_t* __restrict__ cfg_ptr,
                                const int64_t* __restrict__ pair_ptr, int64_t n_cfg,
                                int64_t n_atoms, int64_t n_pairs, double* __restrict__ e_cfg) {
  const int64_t c = blockIdx.x * (int64_t)(blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (c >= n_cfg) return;
  const int64_t a0 = min(max(cfg_ptr[c], (int64_t)0), n_atoms);
  const int64_t a1 = min(max(cfg_ptr[c + 1], a0), n_atoms);
  const int64_t p0 = min(max(pair_ptr[a0], (int64_t)0), n_pairs);
  const int64_t p1 = min(max(pair_ptr[a1], p0), n_pairs);
  double s = 0.0;
  for (int64_t p = p0 + lane; p < p1; p += 64) s += ep[p];
  s = wave_sum(s);
  if (lane == 0) e_cfg[c] = s;
}

// F_a = sum_{p: i(p) = a} g_p rhat_p - sum_{p: j(p) = a} g_p rhat_p (thread per atom)
__global__ void k_2b_forces(const double* __restrict__ gp, const double* __restrict__ pair_r,
                            const int64_t* __restrict__ pair_ptr,
                            const int64_t* __restrict__ tgt_ptr,
                            const int32_t* __restrict__ tgt_pair, int64_t n_atoms,
                            int64_t n_pairs, double* __restrict__ F) {
  for (int64_t a = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; a < n_atoms;
       a += (int64_t)gridDim.x * blockDim.x) {
    double f[3] = {0.0, 0.0, 0.0};
    const int64_t s0 = min(max(pair_ptr[a], (int64_t)0), n_pairs);
    const int64_t s1 = min(max(pair_ptr[a + 1], s0), n_pairs);
    for (int64_t p = s0; p < s1; ++p) {
      const double a0 = pair_r[3 * p], a1 = pair_r[3 * p + 1], a2 = pair_r[3 * p + 2];
      const double r = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
      const double s = r > 0.0 ? gp[p] / r : 0.0;
      f[0] += s * a0;
      f[1] += s * a1;
      f[2] += s * a2;
    }
    for (int64_t e = tgt_ptr[a]; e < tgt_ptr[a + 1]; ++e) {
      const int64_t p = tgt_pair[e];
      const double a0 = pair_r[3 * p], a1 = pair_r[3 * p + 1], a2 = pair_r[3 * p + 2];
      const double r = sqrt(a0 * a0 + a1 * a1 + a2 * a2);
      const double s = r > 0.0 ? gp[p] / r : 0.0;
      f[0] -= s * a0;
      f[1] -= s * a1;
      f[2] -= s * a2;
    }
#pragma unroll
    for (int al = 0; al < 3; ++al) F[3 * a + al] = f[al];
  }
}

inline unsigned cdiv(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }

Se2b make_k(double delta, double theta, double r_cut, double width) {
  return Se2b{delta * delta, 1.0 / (2.0 * theta * theta), r_cut, width};
}

}  // namespace

void se2b_rows_f64(const double* pair_r, const int64_t* cfg_ptr, int64_t n_cfg,
                   const int64_t* pair_ptr, const int64_t* tgt_ptr, const int32_t* tgt_pair,
                   int64_t n_atoms, int64_t n_pairs, const double* x, int64_t M, double delta,
                   double theta, double r_cut, double width, double* K, int64_t ldk,
                   hipStream_t st) {
  if (M <= 0) return;
  const Se2b k = make_k(delta, theta, r_cut, width);
  if (n_cfg > 0)
    hipLaunchKernelGGL(k_2b_energy, dim3(cdiv(M, 64), (unsigned)n_cfg), dim3(256), 0, st, pair_r,
                       cfg_ptr, pair_ptr, n_atoms, n_pairs, x, M, k, K, ldk);
  if (n_atoms > 0)
    hipLaunchKernelGGL(k_2b_force, dim3(cdiv(M, 64), cdiv(n_atoms, 4)), dim3(256), 0, st, pair_r,
                       pair_ptr, tgt_ptr, tgt_pair, n_atoms, n_pairs, x, M, k, n_cfg, K, ldk);
}

void se2b_kmm_f64(const double* x, int64_t M, double delta, double theta, double r_cut,
                  double width, double* K, int64_t ldk, hipStream_t st) {
  if (M <= 0) return;
  hipLaunchKernelGGL(k_2b_kmm, dim3(cdiv(M, 256), (unsigned)M), dim3(256), 0, st, x, M,
                     make_k(delta, theta, r_cut, width), K, ldk);
}

void se2b_predict_f64(const double* pair_r, const int64_t* cfg_ptr, int64_t n_cfg,
                      const int64_t* pair_ptr, const int64_t* tgt_ptr, const int32_t* tgt_pair,
                      int64_t n_atoms, int64_t n_pairs, const double* x, const double* c,
                      int64_t M, double delta, double theta, double r_cut, double width,
                      double* ep, double* gp, double* e_cfg, double* forces, hipStream_t st) {
  const Se2b k = make_k(delta, theta, r_cut, width);
  if (n_pairs > 0)
    hipLaunchKernelGGL(k_2b_pair_terms, dim3(std::min(cdiv(n_pairs, 256), 65536u)), dim3(256), 0,
                       st, pair_r, n_pairs, x, c, M, k, ep, gp);
  if (e_cfg && n_cfg > 0)
    hipLaunchKernelGGL(k_2b_cfg_energy, dim3(cdiv(n_cfg, 4)), dim3(256), 0, st, ep, cfg_ptr,
                       pair_ptr, n_cfg, n_atoms, n_pairs, e_cfg);
  if (forces && n_atoms > 0)
    hipLaunchKernelGGL(k_2b_forces, dim3(std::min(cdiv(n_atoms, 256), 65536u)), dim3(256), 0, st,
                       gp, pair_r, pair_ptr, tgt_ptr, tgt_pair, n_atoms, n_pairs, forces);
}

}  // namespace gapk
