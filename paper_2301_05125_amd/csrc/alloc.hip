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
// those sums, so no grid-wide synchronisation is needed. A single workgroup
// then derives e_i, the top-up ranks and the exclusive scan of n_i.
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

// Interval [lo, hi] containing lambda* after `passes` narrowing passes.
__device__ void replay_interval(const FrameStats* st, int passes, int64_t Bp, uint32_t& lo,
                                uint32_t& hi) {
  lo = 0u;
  hi = 1u << 31;
  for (int p = 0; p < passes; ++p) {
    uint32_t step = (uint32_t)(((uint64_t)hi - lo + 1 + kAllocCandidates - 1) / kAllocCandidates);
    int m_best = 0;
    for (int m = 1; m < kAllocCandidates; ++m) {
      uint64_t c = (uint64_t)lo + (uint64_t)m * step;
      if (c > hi) break;
      if ((int64_t)st->sums[p][m] <= Bp) m_best = m;
      else break;
    }
    uint64_t nlo = (uint64_t)lo + (uint64_t)m_best * step;
    uint64_t nxt = nlo + step;
    uint32_t nhi = (m_best + 1 < kAllocCandidates && nxt <= hi) ? (uint32_t)(nxt - 1) : hi;
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
  __shared__ uint32_t iv[2];
  const int64_t Bp = fp.budget - (int64_t)v.P * fp.n_min;
  const uint32_t E = (uint32_t)(fp.n_max - fp.n_min);
  if (threadIdx.x == 0) {
    uint32_t lo, hi;
    replay_interval(v.stats, pass, Bp, lo, hi);
    iv[0] = lo;
    iv[1] = hi;
  }
  const uint64_t maxs = v.stats->max_score;
  const int i = blockIdx.x * 256 + threadIdx.x;
  w_s[threadIdx.x] = i < v.P ? weight_of((uint64_t)v.score[i], maxs) : 0u;
  __syncthreads();
  const uint32_t lo = iv[0], hi = iv[1];
  const uint32_t step = (uint32_t)(((uint64_t)hi - lo + 1 + kAllocCandidates - 1) / kAllocCandidates);
  const int m = threadIdx.x;
  if (m == 0) return;
  uint64_t c = (uint64_t)lo + (uint64_t)m * step;
  if (c > hi) return;
  const uint32_t lam = (uint32_t)c;
  uint32_t sum = 0;
  const int cnt = min(256, v.P - blockIdx.x * 256);
  for (int k = 0; k < cnt; ++k) sum += extra_rays(lam, w_s[k], E);
  if (sum) atomicAdd((unsigned long long*)&v.stats->sums[pass][m], (unsigned long long)sum);
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

__global__ __launch_bounds__(1024) void alloc_finalize_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive) return;
  __shared__ int64_t sm[17];
  __shared__ int32_t mm[2][16];
  const int P = v.P;
  const int64_t Bp = fp.budget - (int64_t)P * fp.n_min;
  const uint32_t E = (uint32_t)(fp.n_max - fp.n_min);
  uint32_t lam, hi;
  replay_interval(v.stats, kAllocPasses, Bp, lam, hi);
  const uint64_t maxs = v.stats->max_score;
  const int per = (P + blockDim.x - 1) / blockDim.x;
  const int b = threadIdx.x * per, e = min(P, b + per);
  int64_t se = 0, sel = 0;
  for (int i = b; i < e; ++i) {
    uint32_t w = weight_of((uint64_t)v.score[i], maxs);
    uint32_t e0 = extra_rays(lam, w, E), e1 = extra_rays(lam + 1u, w, E);
    se += e0;
    sel += e1 > e0;
  }
  int64_t tot_e;
  block_exclusive_scan(se, sm, tot_e);
  int64_t tot_el;
  int64_t rank = block_exclusive_scan(sel, sm, tot_el);
  const int64_t R = Bp - tot_e;
  int64_t nsum = 0;
  for (int i = b; i < e; ++i) {
    uint32_t w = weight_of((uint64_t)v.score[i], maxs);
    uint32_t e0 = extra_rays(lam, w, E), e1 = extra_rays(lam + 1u, w, E);
    int bonus = 0;
    if (e1 > e0) {
      bonus = rank < R ? 1 : 0;
      ++rank;
    }
    int n = fp.n_min + (int)e0 + bonus;
    v.n[i] = n;
    nsum += n;
  }
  int64_t total;
  int64_t off = block_exclusive_scan(nsum, sm, total);
  int nmin = 0x7fffffff, nmax = 0;
  for (int i = b; i < e; ++i) {
    v.offsets[i] = (uint32_t)off;
    int n = v.n[i];
    off += n;
    nmin = min(nmin, n);
    nmax = max(nmax, n);
  }
  for (int o = 32; o > 0; o >>= 1) {
    nmin = min(nmin, __shfl_xor(nmin, o));
    nmax = max(nmax, __shfl_xor(nmax, o));
  }
  if ((threadIdx.x & 63) == 0) {
    mm[0][threadIdx.x >> 6] = nmin;
    mm[1][threadIdx.x >> 6] = nmax;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) {
      nmin = min(nmin, mm[0][w]);
      nmax = max(nmax, mm[1][w]);
    }
    v.offsets[P] = (uint32_t)total;
    v.stats->lambda = lam;
    v.stats->n_min_seen = nmin;
    v.stats->n_max_seen = nmax;
    v.stats->budget_used = (uint64_t)total;
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
  hipLaunchKernelGGL(alloc_finalize_kernel, dim3(1), dim3(1024), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_uniform_offsets(const VolumeView& v, hipStream_t s) {
  hipLaunchKernelGGL(uniform_offsets_kernel, dim3((v.P + 1 + 255) / 256), dim3(256), 0, s, v);
  return hipGetLastError();
}

}  // namespace adgi
