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
// chain-major order) and each probe's range found, so the trace and the
// blend see per-probe sample lists like the budgeted path's per-probe rays.
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

template <bool HALF>
__device__ float chain_h(const VolumeView& v, const uint16_t* __restrict__ qv, const void* irr,
                         const float* x, uint32_t& probe) {
  const float o[3] = {v.ox, v.oy, v.oz}, s[3] = {v.sx, v.sy, v.sz};
  const int dims[3] = {v.dx, v.dy, v.dz};
  int idx[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float f = dims[a] > 1 ? (x[a] - o[a]) / s[a] : 0.0f;
    int i = (int)floorf(f + 0.5f);
    idx[a] = min(max(i, 0), dims[a] - 1);
  }
  const uint32_t pr = (uint32_t)(idx[0] + v.dx * (idx[1] + v.dy * idx[2]));
  probe = pr;
  // octant from the signs of the decoded direction (O1 inverse)
  const float u = x[3], w = x[4];
  const bool lower = 1.0f - fabsf(u) - fabsf(w) < 0.0f;
  const int k = (u < 0.0f ? 1 : 0) | (w < 0.0f ? 2 : 0) | (lower ? 4 : 0);
  const float f = (float)qv[8 * pr + k] * (1.0f / 1024.0f);
  if (f <= 0.0f) return 0.0f;
  const int r = v.irr_res - 2, m = r / 2, gi = v.irr_res;
  const int cx = min(max((int)floorf((u + 1.0f) * 0.5f * (float)m), 0), m - 1);
  const int cy = min(max((int)floorf((w + 1.0f) * 0.5f * (float)m), 0), m - 1);
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
  const float lum = 0.2126f * (rgb[0] * 0.25f) + 0.7152f * (rgb[1] * 0.25f) + 0.0722f * (rgb[2] * 0.25f);
  return expf(fminf(lum / f, 1.0f)) * f;
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

template <bool HALF>
__global__ void chain_kernel(VolumeView v, const void* irr) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const FrameParams& fp = *v.fp;
  if (c >= fp.chains) return;
  const uint16_t* qv = v.qv[fp.frame & 1];
  float* st = v.chain_state + 8 * (size_t)c;
  float x[5];
  if (fp.chain_init) {
    const uint64_t key = stream_key(fp.seed, kTagChainInit, (uint32_t)c, 0, 0);
    const float ext[3] = {(float)(v.dx - 1) * v.sx, (float)(v.dy - 1) * v.sy, (float)(v.dz - 1) * v.sz};
    const float lo[3] = {v.ox, v.oy, v.oz};
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmaf(uniform24(key, (uint64_t)(a + 1)), ext[a], lo[a]);
    x[3] = fmaf(2.0f, uniform24(key, 4), -1.0f);
    x[4] = fmaf(2.0f, uniform24(key, 5), -1.0f);
  } else {
#pragma unroll
    for (int a = 0; a < 5; ++a) x[a] = st[a];
  }
  uint32_t pr = 0;
  float y = chain_in_domain(v, x) ? chain_h<HALF>(v, qv, irr, x, pr) : 0.0f;
  const int M = fp.chain_steps, K = fp.chain_burn_in, S = M - K - 1;
  for (int i = 0; i < M; ++i) {
    const uint64_t key = stream_key(fp.seed, kTagChain, (uint32_t)c, (uint32_t)fp.frame, (uint32_t)i);
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
    const float eps = uniform24(key, 7);
    float xp[5];
#pragma unroll
    for (int a = 0; a < 3; ++a) xp[a] = fmaf(fp.chain_sp[a], g[a], x[a]);
    xp[3] = fmaf(fp.chain_sd, g[3], x[3]);
    xp[4] = fmaf(fp.chain_sd, g[4], x[4]);
    const bool in = chain_in_domain(v, xp);
    uint32_t prp = pr;
    const float yp = in ? chain_h<HALF>(v, qv, irr, xp, prp) : 0.0f;
    const bool acc = in && (y <= 0.0f || eps * y <= yp);
    if (acc) {
#pragma unroll
      for (int a = 0; a < 5; ++a) x[a] = xp[a];
      y = yp;
      pr = prp;
    }
    if (fp.debug) v.dbg_accept[(size_t)c * M + i] = acc ? 1 : 0;
    if (i > K) {
      const size_t s = (size_t)c * S + (size_t)(i - K - 1);
      v.smp_probe_raw[s] = pr;
      v.smp_uv_raw[s] = make_float2(x[3], x[4]);
    }
  }
#pragma unroll
  for (int a = 0; a < 5; ++a) st[a] = x[a];
}

__global__ void chain_iota_kernel(uint32_t* idx, uint32_t count) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) idx[k] = k;
}

// Sorted samples: uv gathered; probe ranges by binary search on the sorted
// probe keys; n and offsets of the budgeted path reused as per-probe sample
// counts and ranges.
__global__ void chain_ranges_kernel(VolumeView v, const uint32_t* __restrict__ raw_index, uint32_t count) {
  const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < count) v.smp_uv[k] = v.smp_uv_raw[raw_index[k]];
  if ((int)k <= v.P) {
    uint32_t lo = 0, hi = count;  // first sorted position with probe >= k
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (v.smp_probe[mid] < k) lo = mid + 1;
      else hi = mid;
    }
    v.offsets[k] = lo;
  }
}

__global__ void chain_counts_kernel(VolumeView v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < v.P) v.n[i] = (int32_t)(v.offsets[i + 1] - v.offsets[i]);
  if (i == 0) {
    v.stats->budget_used = v.offsets[v.P];
  }
}

static int probe_key_bits(int P) {
  int bits = 1;
  while ((1ll << bits) < (long long)P) ++bits;
  return bits;
}

static size_t sort_bytes_for(uint32_t samples, int P) {
  size_t bytes = 0;
  (void)rocprim::radix_sort_pairs(nullptr, bytes, (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                                  (uint32_t*)nullptr, (size_t)samples, 0, probe_key_bits(P), (hipStream_t)0);
  return bytes;
}

// The sort may pick another algorithm for fewer keys: the workspace covers
// every power of two up to max_samples and max_samples itself.
size_t chain_sort_temp_bytes(uint32_t max_samples, int P) {
  size_t bytes = sort_bytes_for(max_samples, P);
  for (uint64_t n = 1; n < max_samples; n <<= 1) bytes = std::max(bytes, sort_bytes_for((uint32_t)n, P));
  return bytes;
}

size_t chain_sort_needed_bytes(uint32_t samples, int P) { return sort_bytes_for(samples, P); }

hipError_t launch_chains(const VolumeView& v, bool fp16, const void* irr, int chains, uint32_t samples,
                         void* sort_temp, size_t sort_temp_bytes, hipStream_t s) {
  if (fp16)
    hipLaunchKernelGGL(chain_kernel<true>, dim3((chains + 127) / 128), dim3(128), 0, s, v, irr);
  else
    hipLaunchKernelGGL(chain_kernel<false>, dim3((chains + 127) / 128), dim3(128), 0, s, v, irr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (samples > 0) {
    hipLaunchKernelGGL(chain_iota_kernel, dim3((samples + 255) / 256), dim3(256), 0, s, v.smp_index, samples);
    // stable LSD radix sort: (raw probe, raw index) -> (sorted probe, raw index)
    size_t tb = sort_temp_bytes;
    e = rocprim::radix_sort_pairs(sort_temp, tb, v.smp_probe_raw, v.smp_probe, v.smp_index, v.smp_order,
                                  (size_t)samples, 0, probe_key_bits(v.P), s);
    if (e != hipSuccess) return e;
  }
  const uint32_t n = std::max<uint32_t>(samples, (uint32_t)v.P + 1);
  hipLaunchKernelGGL(chain_ranges_kernel, dim3((n + 255) / 256), dim3(256), 0, s, v, v.smp_order, samples);
  hipLaunchKernelGGL(chain_counts_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  return hipGetLastError();
}

}  // namespace adgi
