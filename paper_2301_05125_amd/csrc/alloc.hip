// alloc.hip - integer ray-budget allocation and the ray-offset scan.
//
// The paper fixes the number of samples per frame (the chain count, Sec. 3.3)
// and lets its guide decide where they go. Here the guide is the per-probe
// score s_i and the split is exact integer arithmetic:
//   w_i = s_i shifted so that max w lies in [2^31, 2^32) (all zero: w = 2^31),
//   e_i(lambda) = min(n_max - n_min, floor(lambda * w_i / 2^32)),
//   lambda* = the largest lambda in [0, 2^31] with sum_i e_i <= B - P n_min,
//   the remainder R goes one ray each to the lowest-index probes with
//   e_i(lambda*+1) > e_i(lambda*), and n_i = n_min + e_i + bonus_i.
// lambda* is found by four 256-way interval searches: each pass evaluates
// the monotone sum at 255 candidates in parallel (one candidate per thread,
// the block's weights staged in LDS) and accumulates per-candidate integer
// sums with atomics; every block of the next pass replays the narrowing from
// those sums, so no grid-wide synchronisation is needed. The top-up ranks and
// the exclusive scan of n_i then take three passes: per-block sums, a scan
// over the blocks in one workgroup, and per-block local scans.
#include "adgi_internal.hpp"

namespace adgi {

__device__ __forceinline__ uint32_t weight_of(uint64_t s, uint64_t maxs) {
  if (maxs == 0) return 1u << 31;
  int bits = 64 - __clzll((long long)maxs);
  return bits <= 32 ? (uint32_t)(s << (32 - bits)) : (uint32_t)(s >> (bits - 32));
}

__device__ __forceinline__ uint32_t extra_rays(uint32_t lambda, uint32_t w, uint32_t E) {
  return min(E, __umulhi(lambda, w));
}

// Interval [lo, hi] containing lambda* after `passes` narrowing passes,
// replayed by all kAllocCandidates threads of a block together: candidate m of
// a pass is kept when it lies in the interval and its sum fits the budget,
// and since the sums grow with m the kept candidates are m = 1..m_best, so
// m_best is their count.
__device__ void replay_interval(const uint64_t* sums, int passes, int64_t Bp, uint32_t& lo, uint32_t& hi) {
  lo = 0u;
  hi = 1u << 31;
  const int m = (int)threadIdx.x;
  for (int p = 0; p < passes; ++p) {
    const uint32_t step = (uint32_t)(((uint64_t)hi - lo + 1 + kAllocCandidates - 1) / kAllocCandidates);
    const uint64_t c = (uint64_t)lo + (uint64_t)m * step;
    const bool keep = m >= 1 && m < kAllocCandidates && c <= hi && (int64_t)sums[(p * kAllocCandidates + m) * kLamLine] <= Bp;
    const int m_best = __syncthreads_count(keep);
    const uint64_t nlo = (uint64_t)lo + (uint64_t)m_best * step;
    const uint64_t nxt = nlo + step;
    const uint32_t nhi = (m_best + 1 < kAllocCandidates && nxt <= hi) ? (uint32_t)(nxt - 1) : hi;
    lo = (uint32_t)nlo;
    hi = nhi;
  }
}

__global__ void alloc_max_kernel(VolumeView v) {
  if (!v.fp->adaptive) return;
  __shared__ uint64_t red[4];
  uint64_t m = 0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < v.P; i += gridDim.x * blockDim.x)
    m = max(m, (uint64_t)v.score[i]);
  for (int off = 32; off > 0; off >>= 1) m = max(m, (uint64_t)__shfl_xor((unsigned long long)m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = max(m, red[w]);
    atomicMax((unsigned long long*)&v.stats->max_score, (unsigned long long)m);
  }
}

// One 256-way pass: block b covers probes [b*256, b*256+256).
__global__ __launch_bounds__(256) void lambda_pass_kernel(VolumeView v, int pass) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive) return;
  __shared__ uint32_t w_s[256];
  const int64_t Bp = fp.budget - (int64_t)v.P * fp.n_min;
  const uint32_t E = (uint32_t)(fp.n_max - fp.n_min);
  uint32_t lo, hi;
  replay_interval(v.lam_sums, pass, Bp, lo, hi);
  const uint64_t maxs = v.stats->max_score;
  const int i = blockIdx.x * 256 + threadIdx.x;
  w_s[threadIdx.x] = i < v.P ? weight_of((uint64_t)v.score[i], maxs) : 0u;
  __syncthreads();
  const uint32_t step = (uint32_t)(((uint64_t)hi - lo + 1 + kAllocCandidates - 1) / kAllocCandidates);
  const int m = threadIdx.x;
  if (m == 0) return;
  uint64_t c = (uint64_t)lo + (uint64_t)m * step;
  if (c > hi) return;
  const uint32_t lam = (uint32_t)c;
  uint32_t sum = 0;
  const int cnt = min(256, v.P - blockIdx.x * 256);
  for (int k = 0; k < cnt; ++k) sum += extra_rays(lam, w_s[k], E);
  // each candidate's sum on a cache line of its own: the blocks' atomics on
  // neighbouring candidates do not queue on one line
  if (sum) atomicAdd((unsigned long long*)&v.lam_sums[(pass * kAllocCandidates + m) * kLamLine], (unsigned long long)sum);
}

// Block-wide exclusive scan (blockDim multiple of 64, <= 1024).
__device__ int64_t block_exclusive_scan(int64_t x, int64_t* sm, int64_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int64_t v = x;
  for (int off = 1; off < 64; off <<= 1) {
    int64_t y = __shfl_up(v, off);
    if (lane >= off) v += y;
  }
  __syncthreads();
  if (lane == 63) sm[wave] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t acc = 0;
    for (int k = 0; k < nw; ++k) {
      int64_t t = sm[k];
      sm[k] = acc;
      acc += t;
    }
    sm[nw] = acc;
  }
  __syncthreads();
  total = sm[nw];
  return v - x + sm[wave];
}

// Blend work order: probes sorted by their number of 64-ray chunks, most
// first, so that the longest per-probe blends start first. Bucket b holds the
// probes with min(max(ceil(n/64), 1), 32) = 32 - b chunks (a probe without
// rays, possible in chain frames, joins the one-chunk bucket). Counting happens with the
// allocation; order_scatter_kernel then places every probe. The order inside a
// bucket depends on timing, which does not matter: every probe's blend is
// independent of the others.
__device__ __forceinline__ int order_bucket(int n) {
  const int c = min(max((n + 63) >> 6, 1), kOrderBuckets);
  return kOrderBuckets - c;
}

__device__ void count_buckets(const VolumeView& v, bool valid, int n, uint32_t* hist) {
  if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0u;
  __syncthreads();
  if (valid) atomicAdd(&hist[order_bucket(n)], 1u);
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && hist[threadIdx.x])
    atomicAdd(&v.stats->bucket_count[threadIdx.x], hist[threadIdx.x]);
}

__global__ __launch_bounds__(256) void order_scatter_kernel(VolumeView v) {
  __shared__ uint32_t start[kOrderBuckets], hist[kOrderBuckets], base[kOrderBuckets];
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int b = 0; b < kOrderBuckets; ++b) {
      start[b] = acc;
      acc += v.stats->bucket_count[b];
    }
  }
  if (threadIdx.x < kOrderBuckets) hist[threadIdx.x] = 0u;
  __syncthreads();
  int b = 0;
  uint32_t local = 0;
  if (i < v.P) {
    b = order_bucket(v.n[i]);
    local = atomicAdd(&hist[b], 1u);
  }
  __syncthreads();
  if (threadIdx.x < kOrderBuckets && hist[threadIdx.x])
    base[threadIdx.x] = atomicAdd(&v.stats->bucket_cursor[threadIdx.x], hist[threadIdx.x]);
  __syncthreads();
  if (i < v.P) v.order[start[b] + base[b] + local] = i;
}

// Finalize in three parallel steps over blocks of 256 probes:
//   F1 per block: e_i(lambda*), top-up eligibility, block sums;
//   F2 one workgroup: R, exclusive rank bases and ray offsets of the blocks;
//   F3 per block: local scans -> bonus_i, n_i and ray offsets.
__global__ __launch_bounds__(256) void alloc_blocks_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive) return;
  __shared__ int64_t red_e[4];
  __shared__ uint32_t red_el[4];
  const int64_t Bp = fp.budget - (int64_t)v.P * fp.n_min;
  const uint32_t E = (uint32_t)(fp.n_max - fp.n_min);
  uint32_t lam, hi;
  replay_interval(v.lam_sums, kAllocPasses, Bp, lam, hi);
  const int i = blockIdx.x * 256 + threadIdx.x;
  int64_t e0 = 0;
  uint32_t el = 0;
  if (i < v.P) {
    const uint32_t w = weight_of((uint64_t)v.score[i], v.stats->max_score);
    const uint32_t a = extra_rays(lam, w, E), b = extra_rays(lam + 1u, w, E);
    e0 = a;
    el = b > a ? 1u : 0u;
  }
  for (int o = 32; o > 0; o >>= 1) {
    e0 += __shfl_xor(e0, o);
    el += __shfl_xor(el, o);
  }
  if ((threadIdx.x & 63) == 0) {
    red_e[threadIdx.x >> 6] = e0;
    red_el[threadIdx.x >> 6] = el;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    v.blk_e[blockIdx.x] = red_e[0] + red_e[1] + red_e[2] + red_e[3];
    v.blk_el[blockIdx.x] = red_el[0] + red_el[1] + red_el[2] + red_el[3];
    if (blockIdx.x == 0) v.stats->lambda = lam;
  }
}

__global__ __launch_bounds__(1024) void alloc_scan_blocks_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive) return;
  __shared__ int64_t sm[17];
  const int nb = (v.P + 255) / 256;
  const int64_t Bp = fp.budget - (int64_t)v.P * fp.n_min;
  // total extras -> remainder R
  int64_t part = 0;
  for (int b = threadIdx.x; b < nb; b += blockDim.x) part += v.blk_e[b];
  int64_t tot_e;
  block_exclusive_scan(part, sm, tot_e);
  const int64_t R = Bp - tot_e;
  // exclusive scans over blocks, in tiles of blockDim with a running carry
  int64_t carry_rank = 0, carry_off = 0;
  for (int t0 = 0; t0 < nb; t0 += blockDim.x) {
    const int b = t0 + threadIdx.x;
    int64_t el = 0, nsum = 0;
    if (b < nb) el = v.blk_el[b];
    int64_t tot;
    int64_t rank = carry_rank + block_exclusive_scan(el, sm, tot);
    if (b < nb) {
      const int cnt = min(256, v.P - b * 256);
      int64_t bonus = R - rank;
      bonus = bonus < 0 ? 0 : (bonus > el ? el : bonus);
      nsum = (int64_t)cnt * fp.n_min + v.blk_e[b] + bonus;
    }
    carry_rank += tot;
    int64_t tot_n;
    int64_t off = carry_off + block_exclusive_scan(nsum, sm, tot_n);
    carry_off += tot_n;
    if (b < nb) {
      v.blk_rank[b] = (uint32_t)rank;
      v.blk_off[b] = (uint32_t)off;
    }
  }
  if (threadIdx.x == 0) {
    v.stats->remainder = R;
    v.offsets[v.P] = (uint32_t)carry_off;
    v.stats->budget_used = (uint64_t)carry_off;
    v.stats->n_min_seen = 0x7fffffff;
    v.stats->n_max_seen = 0;
  }
}

__global__ __launch_bounds__(256) void alloc_write_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive) return;
  __shared__ int64_t sm[17];
  __shared__ uint32_t hist[kOrderBuckets];
  const uint32_t E = (uint32_t)(fp.n_max - fp.n_min);
  const uint32_t lam = v.stats->lambda;
  const int64_t R = v.stats->remainder;
  const int b = blockIdx.x, i = b * 256 + threadIdx.x;
  uint32_t e0 = 0, el = 0;
  if (i < v.P) {
    const uint32_t w = weight_of((uint64_t)v.score[i], v.stats->max_score);
    e0 = extra_rays(lam, w, E);
    el = extra_rays(lam + 1u, w, E) > e0 ? 1u : 0u;
  }
  int64_t tot;
  const int64_t rank = (int64_t)v.blk_rank[b] + block_exclusive_scan((int64_t)el, sm, tot);
  const int n = fp.n_min + (int)e0 + ((el && rank < R) ? 1 : 0);
  const int64_t off = (int64_t)v.blk_off[b] + block_exclusive_scan(i < v.P ? (int64_t)n : 0, sm, tot);
  int nmin = 0x7fffffff, nmax = 0;
  if (i < v.P) {
    v.n[i] = n;
    v.offsets[i] = (uint32_t)off;
    nmin = nmax = n;
    // the 64-ray trace batches that start among this probe's rays
    for (int64_t r = (off + 63) & ~(int64_t)63; r < off + n; r += 64) v.batch_probe[r >> 6] = (uint32_t)i;
  }
  count_buckets(v, i < v.P, n, hist);
  // block minimum and maximum, then one atomic each per block (a per-wave
  // atomic on these two words serialises about a thousand times per frame)
  __shared__ int red_min[4], red_max[4];
  for (int o = 32; o > 0; o >>= 1) {
    nmin = min(nmin, __shfl_xor(nmin, o));
    nmax = max(nmax, __shfl_xor(nmax, o));
  }
  if ((threadIdx.x & 63) == 0) {
    red_min[threadIdx.x >> 6] = nmin;
    red_max[threadIdx.x >> 6] = nmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 1; k < 4; ++k) {
      nmin = min(nmin, red_min[k]);
      nmax = max(nmax, red_max[k]);
    }
    atomicMin(&v.stats->n_min_seen, nmin);
    atomicMax(&v.stats->n_max_seen, nmax);
  }
}

__global__ void uniform_offsets_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (fp.adaptive) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const uint32_t n = (uint32_t)fp.n_uniform;
  if (i < v.P) v.n[i] = (int)n;
  if (i <= v.P) v.offsets[i] = (uint32_t)i * n;
  if (i == 0) {
    v.stats->bucket_count[order_bucket((int)n)] = (uint32_t)v.P;
    v.stats->n_min_seen = (int)n;
    v.stats->n_max_seen = (int)n;
    v.stats->budget_used = (uint64_t)v.P * n;
  }
}

hipError_t launch_alloc(const VolumeView& v, hipStream_t s) {
  int g = (v.P + 255) / 256;
  hipLaunchKernelGGL(alloc_max_kernel, dim3(g < 1024 ? g : 1024), dim3(256), 0, s, v);
  for (int p = 0; p < kAllocPasses; ++p)
    hipLaunchKernelGGL(lambda_pass_kernel, dim3(g), dim3(256), 0, s, v, p);
  hipLaunchKernelGGL(alloc_blocks_kernel, dim3(g), dim3(256), 0, s, v);
  hipLaunchKernelGGL(alloc_scan_blocks_kernel, dim3(1), dim3(1024), 0, s, v);
  hipLaunchKernelGGL(alloc_write_kernel, dim3(g), dim3(256), 0, s, v);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(g), dim3(256), 0, s, v);
  return hipGetLastError();
}

// Blend order for lists whose counts v.n are already set (chain samples).
__global__ __launch_bounds__(256) void order_count_kernel(VolumeView v) {
  __shared__ uint32_t hist[kOrderBuckets];
  const int i = blockIdx.x * 256 + threadIdx.x;
  count_buckets(v, i < v.P, i < v.P ? v.n[i] : 0, hist);
  if (i == 0) v.stats->budget_used = v.offsets[v.P];
}

hipError_t launch_blend_order(const VolumeView& v, hipStream_t s) {
  hipLaunchKernelGGL(order_count_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  hipLaunchKernelGGL(order_scatter_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_uniform_offsets(const VolumeView& v, hipStream_t s) {
  hipLaunchKernelGGL(uniform_offsets_kernel, dim3((v.P + 1 + 255) / 256), dim3(256), 0, s, v);
  hipLaunchKernelGGL(order_scatter_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  return hipGetLastError();
}

}  // namespace adgi
