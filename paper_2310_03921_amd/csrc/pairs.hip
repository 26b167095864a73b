// Pair-list transposition for the L-hat accumulation of force observations.
//
// The descriptor derivatives come as a source-major pair list (atom i, slot k)
// pointing at atoms j(i,k).  A force observation on atom j sums over every pair
// pointing at j (Sec. "Theory", operator L-hat), so the force-row and force
// kernels walk a target-major view.  The view is built by a counting sort:
// per-target counts (integer atomics), an exclusive scan, placement with
// per-target cursors, and a per-target insertion sort that restores increasing
// pair order, so the result does not depend on atomic ordering.
//
// Targets are also ordered by decreasing in-degree: the force-row kernel
// processes 16 targets per wavefront, one incoming pair of each per step, and
// grouping targets of similar degree keeps those steps nearly all useful.
// Within one degree the order is increasing atom index, so the 16 targets of
// a wavefront usually come from one or two neighbouring configurations and
// their incoming pairs' Jacobian rows lie close together in memory.
#include "common.h"
#include "launch.h"

namespace gapk {

namespace {

constexpr int kDegBuckets = 1024;

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_count_targets(const int32_t* __restrict__ pair_j, int64_t n_pairs,
                                int64_t n_atoms, int32_t* __restrict__ cnt, int* dev_err) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = pair_j[p];
    if (j < 0 || j >= n_atoms) {
      atomicOr(dev_err, GAP_DEVERR_INDEX);
      continue;
    }
    atomicAdd(&cnt[j], 1);
  }
}

// Exclusive scan of n int32 counts into n+1 int64 offsets; one block of 1024.
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t* __restrict__ cnt, int64_t n,
                                                      int64_t* __restrict__ ptr) {
  __shared__ int64_t part[1024];
  const int t = threadIdx.x;
  const int64_t chunk = (n + 1023) / 1024;
  const int64_t lo = min(n, t * chunk), hi = min(n, lo + chunk);
  int64_t s = 0;
  for (int64_t i = lo; i < hi; ++i) s += cnt[i];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int64_t v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - s;
  for (int64_t i = lo; i < hi; ++i) {
    ptr[i] = run;
    run += cnt[i];
  }
  if (t == 1023) ptr[n] = part[1023];
}

__global__ void k_place_pairs(const int32_t* __restrict__ pair_j, int64_t n_pairs, int64_t n_atoms,
                              const int64_t* __restrict__ tgt_ptr, int32_t* __restrict__ cursor,
                              int32_t* __restrict__ tgt_pair) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n_pairs;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int32_t j = pair_j[p];
    if (j < 0 || j >= n_atoms) continue;
    const int32_t pos = atomicAdd(&cursor[j], 1);
    tgt_pair[tgt_ptr[j] + pos] = (int32_t)p;
  }
}

__global__ void k_sort_segments(const int64_t* __restrict__ tgt_ptr, int64_t n_atoms,
                                int32_t* __restrict__ tgt_pair) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_atoms;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = tgt_ptr[j], hi = tgt_ptr[j + 1];
    for (int64_t a = lo + 1; a < hi; ++a) {
      const int32_t v = tgt_pair[a];
      int64_t b = a - 1;
      while (b >= lo && tgt_pair[b] > v) {
        tgt_pair[b + 1] = tgt_pair[b];
        --b;
      }
      tgt_pair[b + 1] = v;
    }
  }
}

__global__ void k_pair_src(const int64_t* __restrict__ pair_ptr, int64_t n_atoms, int64_t n_pairs,
                           int32_t* __restrict__ src, int* dev_err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n_atoms;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = pair_ptr[i], hi = pair_ptr[i + 1];
    if (lo < 0 || hi > n_pairs || hi < lo) {
      atomicOr(dev_err, GAP_DEVERR_INDEX);
      lo = max((int64_t)0, min(lo, n_pairs));
      hi = max(lo, min(hi, n_pairs));
    }
    for (int64_t p = lo; p < hi; ++p) src[p] = (int32_t)i;
  }
}

__global__ void k_degree_hist(const int64_t* __restrict__ tgt_ptr, int64_t n_atoms,
                              int32_t* __restrict__ hist) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n_atoms;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = tgt_ptr[j + 1] - tgt_ptr[j];
    atomicAdd(&hist[d < kDegBuckets ? d : kDegBuckets - 1], 1);
  }
}

// Turn the degree histogram into start offsets for decreasing degree.
__global__ __launch_bounds__(kDegBuckets) void k_degree_offsets(int32_t* __restrict__ hist) {
  __shared__ int32_t s[kDegBuckets];
  const int t = threadIdx.x;
  const int b = kDegBuckets - 1 - t;  // position t holds bucket b (decreasing degree)
  s[t] = hist[b];
  __syncthreads();
  for (int off = 1; off < kDegBuckets; off <<= 1) {
    int32_t v = (t >= off) ? s[t - off] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  hist[b] = s[t] - hist[b];
}

// Stable placement: one workgroup, thread b owns degree bucket b and walks the
// atoms in index order, a chunk of kDegBuckets degrees at a time staged in
// LDS.  Waves whose 64 buckets are all empty only help with the staging.
__global__ __launch_bounds__(kDegBuckets) void k_degree_place(const int64_t* __restrict__ tgt_ptr,
                                                              int64_t n_atoms,
                                                              const int32_t* __restrict__ off,
                                                              int32_t* __restrict__ order) {
  __shared__ int16_t deg[kDegBuckets];
  const int b = threadIdx.x;
  int32_t pos = off[b];
  const int32_t end = b > 0 ? off[b - 1] : (int32_t)n_atoms;  // buckets laid out decreasing
  const bool busy = __any(pos < end);
  for (int64_t base = 0; base < n_atoms; base += kDegBuckets) {
    const int64_t j = base + b;
    int d = -1;
    if (j < n_atoms) d = (int)min(tgt_ptr[j + 1] - tgt_ptr[j], (int64_t)kDegBuckets - 1);
    deg[b] = (int16_t)d;
    __syncthreads();
    if (busy) {
      const int n = (int)min((int64_t)kDegBuckets, n_atoms - base);
      const int4* d8 = reinterpret_cast<const int4*>(deg);
      for (int i8 = 0; i8 < (n + 7) / 8; ++i8) {
        const int4 v = d8[i8];  // eight degrees (entries past n hold -1)
        const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          const int dq = (int16_t)(w[q >> 1] >> (16 * (q & 1)));
          if (dq == b) order[pos++] = (int32_t)(base + 8 * i8 + q);
        }
      }
    }
    __syncthreads();
  }
}

__global__ void k_atom_cfg(const int64_t* __restrict__ cfg_ptr, int64_t n_cfg, int64_t n_atoms,
                           int32_t* __restrict__ atom_cfg) {
  for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < n_cfg;
       c += (int64_t)gridDim.x * blockDim.x) {
    const int64_t lo = max((int64_t)0, cfg_ptr[c]), hi = min(n_atoms, cfg_ptr[c + 1]);
    for (int64_t i = lo; i < hi; ++i) atom_cfg[i] = (int32_t)c;
  }
}

inline unsigned grid_for(int64_t n, int block = 256) {
  int64_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  if (g > 65536) g = 65536;
  return (unsigned)g;
}

}  // namespace

void pair_transpose(const int64_t* pair_ptr, const int32_t* pair_j, int64_t n_atoms,
                    int64_t n_pairs, int64_t* tgt_ptr, int32_t* tgt_pair, int32_t* pair_src,
                    int32_t* order, int32_t* scratch, int* dev_err, hipStream_t st) {
  int32_t* cnt = scratch;                   // n_atoms
  int32_t* hist = scratch + n_atoms;        // kDegBuckets
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_atoms + kDegBuckets)), dim3(256), 0, st, cnt,
                     n_atoms + kDegBuckets, 0);
  if (n_pairs > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_pairs)), dim3(256), 0, st, pair_src, n_pairs,
                       -1);
    // entries past the last valid target's segment (pairs dropped for an
    // out-of-range target) hold pair 0, a valid index for readers that clamp
    // a slot to the end of the list
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_pairs)), dim3(256), 0, st, tgt_pair, n_pairs, 0);
    hipLaunchKernelGGL(k_count_targets, dim3(grid_for(n_pairs)), dim3(256), 0, st, pair_j, n_pairs,
                       n_atoms, cnt, dev_err);
  }
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, st, cnt, n_atoms, tgt_ptr);
  if (n_pairs > 0) {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_atoms)), dim3(256), 0, st, cnt, n_atoms, 0);
    hipLaunchKernelGGL(k_place_pairs, dim3(grid_for(n_pairs)), dim3(256), 0, st, pair_j, n_pairs,
                       n_atoms, tgt_ptr, cnt, tgt_pair);
    hipLaunchKernelGGL(k_sort_segments, dim3(grid_for(n_atoms)), dim3(256), 0, st, tgt_ptr,
                       n_atoms, tgt_pair);
    hipLaunchKernelGGL(k_pair_src, dim3(grid_for(n_atoms)), dim3(256), 0, st, pair_ptr, n_atoms,
                       n_pairs, pair_src, dev_err);
  }
  if (order != nullptr && n_atoms > 0) {
    hipLaunchKernelGGL(k_degree_hist, dim3(grid_for(n_atoms)), dim3(256), 0, st, tgt_ptr, n_atoms,
                       hist);
    hipLaunchKernelGGL(k_degree_offsets, dim3(1), dim3(kDegBuckets), 0, st, hist);
    hipLaunchKernelGGL(k_degree_place, dim3(1), dim3(kDegBuckets), 0, st, tgt_ptr, n_atoms, hist,
                       order);
  }
}

void atom_config(const int64_t* cfg_ptr, int64_t n_cfg, int64_t n_atoms, int32_t* atom_cfg,
                 hipStream_t st) {
  if (n_atoms > 0)
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n_atoms)), dim3(256), 0, st, atom_cfg, n_atoms,
                       -1);
  if (n_cfg <= 0) return;
  hipLaunchKernelGGL(k_atom_cfg, dim3(grid_for(n_cfg)), dim3(256), 0, st, cfg_ptr, n_cfg, n_atoms,
                     atom_cfg);
}

}  // namespace gapk
