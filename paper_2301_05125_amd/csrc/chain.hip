// chain.hip - the static Metropolis chains (Sec. 3.2, Alg. MarkovChainMT with
// Alg. MetropolisStep; Sec. 4.7) and the grouping of their samples by probe.
//
// A chain's state is x = (p, uv): p in the box spanned by the probe centres,
// uv the octahedral coordinates of a direction. Its target is
// h = exp(min(g/f, 1)) f with f = Qv/1024, the 10-bit f_v code of the current
// frame's pilot in the octant of the direction at the nearest probe, and g the
// luminance of that probe's irradiance averaged over the 2x2 texels (one
// level coarser) whose cell holds uv, as the previous frame left it. Each
// frame a chain takes `steps` random-walk steps from where it stopped: normal
// proposals (Box-Muller from counter-based uniforms), rejection outside the
// domain, acceptance when the current density is 0 or u7 h(x) <= h(x'); steps
// after the first burn_in + 1 emit the state (nearest probe, uv) as a sample.
// Samples are then sorted by probe (stable, so a probe's samples stay in
// chain-major order) and the per-probe counts scanned into ranges, so the
// trace and the blend see per-probe sample lists like the budgeted path's
// per-probe rays.
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstring>

#include <rocprim/rocprim.hpp>

#include "adgi_internal.hpp"

namespace adgi {

template <bool HALF>
__device__ __forceinline__ float load_texel(const void* base, size_t i) {
  if (HALF) return __half2float(((const __half*)base)[i]);
  return ((const float*)base)[i];
}

// g of every (probe, coarse cell): the luminance of the mean of the cell's
// 2x2 interior irradiance texels, once per chain frame, so that the chains'
// dependent look-ups hit a table of P (r/2)^2 floats (2.4 MB for 65,536
// probes with 6x6 interiors) instead of the texels.
template <bool HALF>
__global__ void chain_lum_kernel(VolumeView v, const void* irr) {
  const int m = (v.irr_res - 2) / 2, cells = m * m, gi = v.irr_res;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= v.P * cells) return;
  const int pr = idx / cells, cell = idx - pr * cells, cy = cell / m, cx = cell - cy * m;
  const size_t tile = (size_t)pr * gi * gi * 3;
  float rgb[3] = {0.f, 0.f, 0.f};
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const size_t t = tile + (size_t)((2 * cy + b + 1) * gi + 2 * cx + a + 1) * 3;
      rgb[0] += load_texel<HALF>(irr, t);
      rgb[1] += load_texel<HALF>(irr, t + 1);
      rgb[2] += load_texel<HALF>(irr, t + 2);
    }
  v.chain_lum[idx] = fmaf(0.0722f, rgb[2] * 0.25f, fmaf(0.7152f, rgb[1] * 0.25f, 0.2126f * (rgb[0] * 0.25f)));
}

// The target in two halves: target_fetch issues the two look-ups (f_v code
// and g) for a point, target_value finishes h once they have arrived, so that
// independent work can run while they are in flight.
struct TargetFetch {
  uint32_t probe;
  uint32_t code;
  float lum;
};

__device__ __forceinline__ TargetFetch target_fetch(const VolumeView& v, const uint16_t* __restrict__ qv,
                                                    const float* x) {
  const float o[3] = {v.ox, v.oy, v.oz}, s[3] = {v.sx, v.sy, v.sz};
  const int dims[3] = {v.dx, v.dy, v.dz};
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float f = dims[a] > 1 ? (x[a] - o[a]) / s[a] : 0.0f;
    int i = (int)floorf(f + 0.5f);
    idx[a] = min(max(i, 0), dims[a] - 1);
  }
  TargetFetch t;
  const uint32_t pr = (uint32_t)(idx[0] + v.dx * (idx[1] + v.dy * idx[2]));
  t.probe = pr;
  // octant from the signs of the decoded direction (O1 inverse)
  const float u = x[3], w = x[4];
  const bool lower = 1.0f - fabsf(u) - fabsf(w) < 0.0f;
  const int k = (u < 0.0f ? 1 : 0) | (w < 0.0f ? 2 : 0) | (lower ? 4 : 0);
  t.code = qv[8 * pr + k];
  const int m = (v.irr_res - 2) / 2;
  const int cx = min(max((int)floorf((u + 1.0f) * 0.5f * (float)m), 0), m - 1);
  const int cy = min(max((int)floorf((w + 1.0f) * 0.5f * (float)m), 0), m - 1);
  t.lum = v.chain_lum[(size_t)pr * m * m + cy * m + cx];
  return t;
}

__device__ __forceinline__ float target_value(const TargetFetch& t) {
  const float f = (float)t.code * (1.0f / 1024.0f);
  if (f <= 0.0f) return 0.0f;
  return expf(fminf(t.lum / f, 1.0f)) * f;
}

__device__ __forceinline__ float chain_h(const VolumeView& v, const uint16_t* __restrict__ qv, const float* x,
                                         uint32_t& probe) {
  const TargetFetch t = target_fetch(v, qv, x);
  probe = t.probe;
  return target_value(t);
}

__device__ __forceinline__ bool chain_in_domain(const VolumeView& v, const float* x) {
  const float lo[3] = {v.ox, v.oy, v.oz};
  const float hi[3] = {fmaf((float)(v.dx - 1), v.sx, v.ox), fmaf((float)(v.dy - 1), v.sy, v.oy),
                       fmaf((float)(v.dz - 1), v.sz, v.oz)};
  bool in = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) in = in && x[a] >= lo[a] && x[a] <= hi[a];
  return in && x[3] >= -1.0f && x[3] <= 1.0f && x[4] >= -1.0f && x[4] <= 1.0f;
}

// One chain step's random numbers: Box-Muller pairs (u1,u2), (u3,u4), (u5,u6)
// give g[0..5] (g[5] unused), u7 the acceptance uniform.
struct StepRand {
  float g[5];
  float eps;
};

__device__ __forceinline__ StepRand step_rand(const FrameParams& fp, uint32_t c, uint32_t i) {
  const uint64_t key = stream_key(fp.seed, kTagChain, c, (uint32_t)fp.frame, i);
  StepRand r;
  float g[6];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const float u1 = uniform24(key, (uint64_t)(2 * q + 1)), u2 = uniform24(key, (uint64_t)(2 * q + 2));
    const float rr = sqrtf(-2.0f * logf(1.0f - u1));
    float sn, cs;
    sincosf(kTwoPi * u2, &sn, &cs);
    g[2 * q] = rr * cs;
    g[2 * q + 1] = rr * sn;
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) r.g[a] = g[a];
  r.eps = uniform24(key, 7);
  return r;
}

// Proposal x' = x + (sigma_pos spacing, sigma_dir) * g, the same FP32
// operations in every variant.
__device__ __forceinline__ void propose(const FrameParams& fp, const float* x, const float* g, float* xp) {
#pragma unroll
  for (int a = 0; a < 3; ++a) xp[a] = fmaf(fp.chain_sp[a], g[a], x[a]);
  xp[3] = fmaf(fp.chain_sd, g[3], x[3]);
  xp[4] = fmaf(fp.chain_sd, g[4], x[4]);
}

__device__ __forceinline__ void chain_start(const VolumeView& v, const FrameParams& fp, int c, float* x) {
  if (fp.chain_init) {
    const uint64_t key = stream_key(fp.seed, kTagChainInit, (uint32_t)c, 0, 0);
    const float ext[3] = {(float)(v.dx - 1) * v.sx, (float)(v.dy - 1) * v.sy, (float)(v.dz - 1) * v.sz};
    const float lo[3] = {v.ox, v.oy, v.oz};
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmaf(uniform24(key, (uint64_t)(a + 1)), ext[a], lo[a]);
    x[3] = fmaf(2.0f, uniform24(key, 4), -1.0f);
    x[4] = fmaf(2.0f, uniform24(key, 5), -1.0f);
  } else {
    const float* st = v.chain_state + 8 * (size_t)c;
#pragma unroll
    for (int a = 0; a < 5; ++a) x[a] = st[a];
  }
}

// Step i of chain c leaves state (x, probe): record it, count it.
__device__ __forceinline__ void emit(const VolumeView& v, const FrameParams& fp, int c, int i, bool acc,
                                     const float* x, uint32_t pr) {
  const int M = fp.chain_steps, K = fp.chain_burn_in, S = M - K - 1;
  if (fp.debug) v.dbg_accept[(size_t)c * M + i] = acc ? 1 : 0;
  if (i > K) {
    const size_t s = (size_t)c * S + (size_t)(i - K - 1);
    v.smp_probe_raw[s] = pr;
    v.smp_uv_raw[s] = make_float2(x[3], x[4]);
    atomicAdd(&v.n[pr], 1);
  }
}

// One thread per chain, one step after the other.
__global__ void chain_kernel(VolumeView v) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const FrameParams& fp = *v.fp;
  if (c >= fp.chains) return;
  const uint16_t* qv = v.qv[fp.frame & 1];
  float x[5];
  chain_start(v, fp, c, x);
  uint32_t pr = 0;
  float y = chain_in_domain(v, x) ? chain_h(v, qv, x, pr) : 0.0f;
  const int M = fp.chain_steps;
  StepRand r = step_rand(fp, (uint32_t)c, 0u);
  for (int i = 0; i < M; ++i) {
    float xp[5];
    propose(fp, x, r.g, xp);
    const bool in = chain_in_domain(v, xp);
    TargetFetch t = {pr, 0u, 0.0f};
    if (in) t = target_fetch(v, qv, xp);
    // the next step's randomness while the look-ups are in flight
    StepRand next = {};
    if (i + 1 < M) next = step_rand(fp, (uint32_t)c, (uint32_t)(i + 1));
    const uint32_t prp = t.probe;
    const float yp = in ? target_value(t) : 0.0f;
    const bool acc = in && (y <= 0.0f || r.eps * y <= yp);
    if (acc) {
#pragma unroll
      for (int a = 0; a < 5; ++a) x[a] = xp[a];
      y = yp;
      pr = prp;
    }
    emit(v, fp, c, i, acc, x, pr);
    r = next;
  }
  float* st = v.chain_state + 8 * (size_t)c;
#pragma unroll
  for (int a = 0; a < 5; ++a) st[a] = x[a];
}

// Prefetching Metropolis (Brockwell, "Parallel Markov chain Monte Carlo
// simulation by pre-fetching", 2006): a group of G = 2^D lanes advances one
// chain D steps per round. Node n < G - 1 of a heap-ordered tree (children
// 2n+1 = reject, 2n+2 = accept) sits at depth d = floor(log2(n+1)); the bits
// of n+1 below its leading one are the accept/reject decisions of the round's
// first d steps. Lane n builds the state those decisions leave (the same fma
// sequence as one step at a time), proposes step d from it and evaluates the
// target there, so the D dependent target look-ups of the round overlap. The
// group then walks the tree from the root with the acceptance rule: the same
// proposals, targets and decisions as chain_kernel, bit for bit.
template <int D>
__global__ __launch_bounds__(256) void chain_prefetch_kernel(VolumeView v) {
  constexpr int G = 1 << D;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int base = lane & ~(G - 1);  // first lane of this chain's group
  const int node = lane & (G - 1);
  const int c = tid / G;
  const FrameParams& fp = *v.fp;
  const bool live = c < fp.chains;   // uniform over the group; dead groups still shuffle
  const uint16_t* qv = v.qv[fp.frame & 1];
  float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  uint32_t pr = 0;
  float y = 0.0f;
  if (live) {
    chain_start(v, fp, c, x);
    if (chain_in_domain(v, x)) y = chain_h(v, qv, x, pr);
  }
  const int d = 31 - __clz(node + 1);  // this lane's depth (node G-1 is idle)
  const int M = fp.chain_steps;
  // randomness of step i0 + node, computed by the first D lanes
  StepRand mine = {};
  if (live && node < min(D, M)) mine = step_rand(fp, (uint32_t)c, (uint32_t)node);
  for (int i0 = 0; i0 < M; i0 += D) {
    const int steps = min(D, M - i0);
    float g[D][5], eps[D];
#pragma unroll
    for (int s = 0; s < D; ++s) {
#pragma unroll
      for (int a = 0; a < 5; ++a) g[s][a] = __shfl(mine.g[a], base + s, 64);
      eps[s] = __shfl(mine.eps, base + s, 64);
    }
    // the state the path to this node leaves, and the proposal of step d
    float cur[5], xp[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) cur[a] = x[a];
#pragma unroll
    for (int s = 0; s < D - 1; ++s) {
      if (s < d && (((node + 1) >> (d - 1 - s)) & 1)) {
        float t[5];
        propose(fp, cur, g[s], t);
#pragma unroll
        for (int a = 0; a < 5; ++a) cur[a] = t[a];
      }
    }
    float gd[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) gd[a] = g[0][a];
#pragma unroll
    for (int s = 1; s < D; ++s)
      if (s == d) {
#pragma unroll
        for (int a = 0; a < 5; ++a) gd[a] = g[s][a];
      }
    propose(fp, cur, gd, xp);
    bool in = false;
    TargetFetch t = {0u, 0u, 0.0f};
    if (live && node < G - 1 && d < steps) {
      in = chain_in_domain(v, xp);
      if (in) t = target_fetch(v, qv, xp);
    }
    // the next round's randomness while the look-ups are in flight
    StepRand next = {};
    if (live && node < min(D, M - i0 - D)) next = step_rand(fp, (uint32_t)c, (uint32_t)(i0 + D + node));
    const float h = in ? target_value(t) : 0.0f;
    const uint32_t prp = t.probe;
    // walk the tree
    int n = 0;
#pragma unroll
    for (int s = 0; s < D; ++s) {
      if (s < steps) {
        const int src = base + n;
        const bool in_n = __shfl((int)in, src, 64) != 0;
        const float h_n = __shfl(h, src, 64);
        const bool acc = in_n && (y <= 0.0f || eps[s] * y <= h_n);
        if (acc) {
#pragma unroll
          for (int a = 0; a < 5; ++a) x[a] = __shfl(xp[a], src, 64);
          pr = (uint32_t)__shfl((int)prp, src, 64);
          y = h_n;
        }
        if (live && node == 0) emit(v, fp, c, i0 + s, acc, x, pr);
        n = 2 * n + 1 + (acc ? 1 : 0);
      }
    }
    mine = next;
  }
  if (live && node == 0) {
    float* st = v.chain_state + 8 * (size_t)c;
#pragma unroll
    for (int a = 0; a < 5; ++a) st[a] = x[a];
  }
}

// Per-probe sample counts start at zero (the chain kernels count with atomics).
__global__ void chain_clear_kernel(VolumeView v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < v.P) v.n[i] = 0;
  if (i == 0) v.offsets[0] = 0u;
}

static int probe_key_bits(int P) {
  int bits = 1;
  while ((1ll << bits) < (long long)P) ++bits;
  return bits;
}

// Onesweep above one block of keys: the merge-sort path rocprim takes by
// default below 2^20 keys launches about twice as many kernels here.
using SortConfig = rocprim::radix_sort_config<rocprim::default_config, rocprim::default_config,
                                              rocprim::default_config, 0>;

static size_t sort_bytes_for(uint32_t samples, int P) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs<SortConfig>(nullptr, bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint64_t*)nullptr,
                                  (uint64_t*)nullptr, (size_t)samples, 0, probe_key_bits(P), (hipStream_t)0);
  return bytes;
}

static size_t scan_bytes_for(int P) {
  size_t bytes = 0;
  (void)rocprim::inclusive_scan(nullptr, bytes, (const uint32_t*)nullptr, (uint32_t*)nullptr, (size_t)P,
                                rocprim::plus<uint32_t>(), (hipStream_t)0);
  return bytes;
}

// The sort may pick another algorithm for fewer keys: the workspace covers
// every power of two up to max_samples, max_samples itself and the count scan.
size_t chain_sort_temp_bytes(uint32_t max_samples, int P) {
  size_t bytes = std::max(sort_bytes_for(max_samples, P), scan_bytes_for(P));
  for (uint64_t n = 1; n < max_samples; n <<= 1) bytes = std::max(bytes, sort_bytes_for((uint32_t)n, P));
  return bytes;
}

size_t chain_sort_needed_bytes(uint32_t samples, int P) {
  return std::max(sort_bytes_for(samples, P), scan_bytes_for(P));
}

int chain_lanes_auto(int chains) {
  // measured on the 65,536-probe box field: 16 lanes up to 16k chains, 4 at
  // 64k (the rounds' extra target evaluations then cost more than the latency
  // they hide); about four waves per SIMD of a 256-CU chip
  const long long want = 262144;
  if ((long long)chains * 16 <= want) return 16;
  if ((long long)chains * 8 <= want) return 8;
  if ((long long)chains * 4 <= want) return 4;
  return 1;
}

static hipError_t launch_chain_kernel(const VolumeView& v, int chains, int lanes, hipStream_t s) {
  const long long threads = (long long)chains * lanes;
  const dim3 grid((unsigned)((threads + 255) / 256));
  switch (lanes) {
    case 1:
      hipLaunchKernelGGL(chain_kernel, dim3((chains + 127) / 128), dim3(128), 0, s, v);
      break;
    case 4:
      hipLaunchKernelGGL((chain_prefetch_kernel<2>), grid, dim3(256), 0, s, v);
      break;
    case 8:
      hipLaunchKernelGGL((chain_prefetch_kernel<3>), grid, dim3(256), 0, s, v);
      break;
    case 16:
      hipLaunchKernelGGL((chain_prefetch_kernel<4>), grid, dim3(256), 0, s, v);
      break;
    case 32:
      hipLaunchKernelGGL((chain_prefetch_kernel<5>), grid, dim3(256), 0, s, v);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_chains(const VolumeView& v, bool fp16, const void* irr, int chains, int lanes, uint32_t samples,
                         void* sort_temp, size_t sort_temp_bytes, hipStream_t s) {
  hipLaunchKernelGGL(chain_clear_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  const int m = (v.irr_res - 2) / 2;
  const long long cells = (long long)v.P * m * m;
  if (fp16)
    hipLaunchKernelGGL(chain_lum_kernel<true>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, v, irr);
  else
    hipLaunchKernelGGL(chain_lum_kernel<false>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, v, irr);
  hipError_t e = launch_chain_kernel(v, chains, lanes, s);
  if (e != hipSuccess) return e;
  // stable LSD radix sort of (probe, uv) by probe: a probe's samples stay in
  // chain-major order
  size_t tb = sort_temp_bytes;
  e = rocprim::radix_sort_pairs<SortConfig>(sort_temp, tb, v.smp_probe_raw, v.smp_probe, (uint64_t*)v.smp_uv_raw,
                                (uint64_t*)v.smp_uv, (size_t)samples, 0, probe_key_bits(v.P), s);
  if (e != hipSuccess) return e;
  tb = sort_temp_bytes;
  e = rocprim::inclusive_scan(sort_temp, tb, (const uint32_t*)v.n, v.offsets + 1, (size_t)v.P,
                              rocprim::plus<uint32_t>(), s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace adgi
