// chain.hip - the Metropolis chains of chain frames (Sec. 3.2-3.3, Alg.
// MarkovChainMT with Alg. MetropolisStep): the static chain (Sec. 4.8), the
// dynamic chain on 3x3x3 virtual proxies (Sec. 4.9), and the grouping of the
// static samples and dynamic rays by probe.
//
// A chain's state is x = (p, uv): p in the box spanned by the probe centres,
// uv the octahedral coordinates of a direction. Each frame a chain takes
// `steps` random-walk steps from where it stopped: normal proposals
// (Box-Muller from counter-based uniforms), rejection outside the domain,
// acceptance when the current density is 0 or u7 h(x) <= h(x'); steps after
// the first burn_in + 1 emit the state.
//   static:  h = exp(min(g/f, 1)) f with f = Qv/1024, the 10-bit f_v code of
//            this frame's pilot in the octant of the direction at the
//            nearest probe, and g the luminance of that probe's irradiance
//            averaged over the 2x2 texels (one level coarser) whose cell
//            holds uv, as the previous frame left it. A state emits a
//            sample (nearest probe, uv); the samples are sorted by probe
//            (stable: a probe's samples stay in chain-major order) and the
//            per-probe counts scanned into ranges.
//   dynamic: h = F[proxy of the nearest probe][octant of uv], F the max of
//            f_d = Qv (Cv + mu Cr) over the proxy's probes (alpha = 0). A
//            state with h > 0 marks its (proxy, octant); every probe of a
//            marked proxy then traces the octant's texel-centre rays.
#include <hip/hip_fp16.h>

#include <algorithm>
#include <cstring>


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

__device__ __forceinline__ uint32_t nearest_probe(const VolumeView& v, const float* x, int idx[3]) {
  const float o[3] = {v.ox, v.oy, v.oz}, s[3] = {v.sx, v.sy, v.sz};
  const int dims[3] = {v.dx, v.dy, v.dz};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float f = dims[a] > 1 ? (x[a] - o[a]) / s[a] : 0.0f;
    int i = (int)floorf(f + 0.5f);
    idx[a] = min(max(i, 0), dims[a] - 1);
  }
  return (uint32_t)(idx[0] + v.dx * (idx[1] + v.dy * idx[2]));
}

// octant of the direction with octahedral coordinates (u, w): the signs of
// the decoded direction
__device__ __forceinline__ int uv_octant(float u, float w) {
  const bool lower = 1.0f - fabsf(u) - fabsf(w) < 0.0f;
  return (u < 0.0f ? 1 : 0) | (w < 0.0f ? 2 : 0) | (lower ? 4 : 0);
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

// A target in two halves: fetch issues the look-ups for a point, value
// finishes h once they have arrived, so that independent work can run while
// they are in flight. cell: the nearest probe (static) or proxy * 8 + octant
// (dynamic).
struct TargetFetch {
  uint32_t cell;
  uint32_t code;
  float lum;
};

struct StaticChain {
  const VolumeView& v;
  const FrameParams& fp;
  const uint16_t* qv;
  __device__ StaticChain(const VolumeView& v_, const FrameParams& fp_)
      : v(v_), fp(fp_), qv(v_.qv[fp_.frame & 1]) {}
  __device__ int chains() const { return fp.chains; }
  __device__ int steps() const { return fp.chain_steps; }
  __device__ int burn_in() const { return fp.chain_burn_in; }
  __device__ bool init() const { return fp.chain_init != 0; }
  __device__ const float* sp() const { return fp.chain_sp; }
  __device__ float sd() const { return fp.chain_sd; }
  __device__ float* state() const { return v.chain_state; }
  __device__ uint8_t* accept() const { return v.dbg_accept; }
  static constexpr uint64_t kTagStep = kTagChain, kTagInit = kTagChainInit;
  __device__ TargetFetch fetch(const float* x) const {
    int idx[3];
    TargetFetch t;
    const uint32_t pr = nearest_probe(v, x, idx);
    t.cell = pr;
    const float u = x[3], w = x[4];
    t.code = qv[8 * pr + uv_octant(u, w)];
    const int m = (v.irr_res - 2) / 2;
    const int cx = min(max((int)floorf((u + 1.0f) * 0.5f * (float)m), 0), m - 1);
    const int cy = min(max((int)floorf((w + 1.0f) * 0.5f * (float)m), 0), m - 1);
    t.lum = v.chain_lum[(size_t)pr * m * m + cy * m + cx];
    return t;
  }
  __device__ static float value(const TargetFetch& t) {
    const float f = (float)t.code * (1.0f / 1024.0f);
    if (f <= 0.0f) return 0.0f;
    return expf(fminf(t.lum / f, 1.0f)) * f;
  }
  // step i of chain c left (x, cell, h): record the sample, count it
  __device__ void emit(int c, int i, const float* x, uint32_t cell, float h) const {
    (void)h;
    const int S = fp.chain_steps - fp.chain_burn_in - 1;
    const size_t s = (size_t)c * S + (size_t)(i - fp.chain_burn_in - 1);
    v.smp_probe_raw[s] = cell;
    v.smp_uv_raw[s] = make_float2(x[3], x[4]);
    atomicAdd(&v.n[cell], 1);
  }
};

struct DynamicChain {
  const VolumeView& v;
  const FrameParams& fp;
  __device__ DynamicChain(const VolumeView& v_, const FrameParams& fp_) : v(v_), fp(fp_) {}
  __device__ int chains() const { return fp.dyn_chains; }
  __device__ int steps() const { return fp.dyn_steps; }
  __device__ int burn_in() const { return fp.dyn_burn_in; }
  __device__ bool init() const { return fp.dyn_init != 0; }
  __device__ const float* sp() const { return fp.dyn_sp; }
  __device__ float sd() const { return fp.dyn_sd; }
  __device__ float* state() const { return v.dyn_state; }
  __device__ uint8_t* accept() const { return v.dbg_dyn_accept; }
  static constexpr uint64_t kTagStep = kTagDynChain, kTagInit = kTagDynChainInit;
  __device__ TargetFetch fetch(const float* x) const {
    int idx[3];
    (void)nearest_probe(v, x, idx);
    const uint32_t q = (uint32_t)(idx[0] / 3 + v.pdx * (idx[1] / 3 + v.pdy * (idx[2] / 3)));
    TargetFetch t;
    t.cell = 8 * q + (uint32_t)uv_octant(x[3], x[4]);
    t.code = 0u;
    t.lum = v.dyn_F[t.cell];
    return t;
  }
  __device__ static float value(const TargetFetch& t) { return t.lum; }
  // a state with h > 0 marks its (proxy, octant): every mark is the same byte
  __device__ void emit(int c, int i, const float* x, uint32_t cell, float h) const {
    (void)c;
    (void)i;
    (void)x;
    if (h > 0.0f) v.dyn_mark[cell] = 1;
  }
};

// One chain step's random numbers: Box-Muller pairs (u1,u2), (u3,u4), (u5,u6)
// give g[0..5] (g[5] unused), u7 the acceptance uniform.
struct StepRand {
  float g[5];
  float eps;
};

__device__ __forceinline__ StepRand step_rand(const FrameParams& fp, uint64_t tag, uint32_t c, uint32_t i) {
  const uint64_t key = stream_key(fp.seed, tag, c, (uint32_t)fp.frame, i);
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

// Proposal x' = x + (step per axis, uv step) * g, the same FP32 operations in
// every variant.
__device__ __forceinline__ void propose(const float* sp, float sd, const float* x, const float* g, float* xp) {
#pragma unroll
  for (int a = 0; a < 3; ++a) xp[a] = fmaf(sp[a], g[a], x[a]);
  xp[3] = fmaf(sd, g[3], x[3]);
  xp[4] = fmaf(sd, g[4], x[4]);
}

template <class T>
__device__ __forceinline__ void chain_start(const VolumeView& v, const FrameParams& fp, const T& t, int c,
                                            float* x) {
  if (t.init()) {
    const uint64_t key = stream_key(fp.seed, T::kTagInit, (uint32_t)c, 0, 0);
    const float ext[3] = {(float)(v.dx - 1) * v.sx, (float)(v.dy - 1) * v.sy, (float)(v.dz - 1) * v.sz};
    const float lo[3] = {v.ox, v.oy, v.oz};
#pragma unroll
    for (int a = 0; a < 3; ++a) x[a] = fmaf(uniform24(key, (uint64_t)(a + 1)), ext[a], lo[a]);
    x[3] = fmaf(2.0f, uniform24(key, 4), -1.0f);
    x[4] = fmaf(2.0f, uniform24(key, 5), -1.0f);
  } else {
    const float* st = t.state() + 8 * (size_t)c;
#pragma unroll
    for (int a = 0; a < 5; ++a) x[a] = st[a];
  }
}

// One thread per chain, one step after the other.
template <class T>
__global__ void chain_kernel(VolumeView v) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const FrameParams& fp = *v.fp;
  const T t(v, fp);
  if (c >= t.chains()) return;
  float x[5];
  chain_start(v, fp, t, c, x);
  uint32_t cell = 0;
  float y = 0.0f;
  if (chain_in_domain(v, x)) {
    const TargetFetch f = t.fetch(x);
    cell = f.cell;
    y = T::value(f);
  }
  const int M = t.steps(), K = t.burn_in();
  StepRand r = step_rand(fp, T::kTagStep, (uint32_t)c, 0u);
  for (int i = 0; i < M; ++i) {
    float xp[5];
    propose(t.sp(), t.sd(), x, r.g, xp);
    const bool in = chain_in_domain(v, xp);
    TargetFetch f = {cell, 0u, 0.0f};
    if (in) f = t.fetch(xp);
    // the next step's randomness while the look-ups are in flight
    StepRand next = {};
    if (i + 1 < M) next = step_rand(fp, T::kTagStep, (uint32_t)c, (uint32_t)(i + 1));
    const float yp = in ? T::value(f) : 0.0f;
    const bool acc = in && (y <= 0.0f || r.eps * y <= yp);
    if (acc) {
#pragma unroll
      for (int a = 0; a < 5; ++a) x[a] = xp[a];
      y = yp;
      cell = f.cell;
    }
    if (fp.debug) t.accept()[(size_t)c * M + i] = acc ? 1 : 0;
    if (i > K) t.emit(c, i, x, cell, y);
    r = next;
  }
  float* st = t.state() + 8 * (size_t)c;
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
template <int D, class T>
__global__ __launch_bounds__(256) void chain_prefetch_kernel(VolumeView v) {
  constexpr int G = 1 << D;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & 63;
  const int base = lane & ~(G - 1);  // first lane of this chain's group
  const int node = lane & (G - 1);
  const int c = tid / G;
  const FrameParams& fp = *v.fp;
  const T t(v, fp);
  const bool live = c < t.chains();   // uniform over the group; dead groups still shuffle
  float x[5] = {0.f, 0.f, 0.f, 0.f, 0.f};
  uint32_t cell = 0;
  float y = 0.0f;
  if (live) {
    chain_start(v, fp, t, c, x);
    if (chain_in_domain(v, x)) {
      const TargetFetch f = t.fetch(x);
      cell = f.cell;
      y = T::value(f);
    }
  }
  const int d = 31 - __clz(node + 1);  // this lane's depth (node G-1 is idle)
  const int M = t.steps(), K = t.burn_in();
  // randomness of step i0 + node, computed by the first D lanes
  StepRand mine = {};
  if (live && node < min(D, M)) mine = step_rand(fp, T::kTagStep, (uint32_t)c, (uint32_t)node);
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
        float tmp[5];
        propose(t.sp(), t.sd(), cur, g[s], tmp);
#pragma unroll
        for (int a = 0; a < 5; ++a) cur[a] = tmp[a];
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
    propose(t.sp(), t.sd(), cur, gd, xp);
    bool in = false;
    TargetFetch f = {0u, 0u, 0.0f};
    if (live && node < G - 1 && d < steps) {
      in = chain_in_domain(v, xp);
      if (in) f = t.fetch(xp);
    }
    // the next round's randomness while the look-ups are in flight
    StepRand next = {};
    if (live && node < min(D, M - i0 - D))
      next = step_rand(fp, T::kTagStep, (uint32_t)c, (uint32_t)(i0 + D + node));
    const float h = in ? T::value(f) : 0.0f;
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
          cell = (uint32_t)__shfl((int)f.cell, src, 64);
          y = h_n;
        }
        if (live && node == 0) {
          if (fp.debug) t.accept()[(size_t)c * M + i0 + s] = acc ? 1 : 0;
          if (i0 + s > K) t.emit(c, i0 + s, x, cell, y);
        }
        n = 2 * n + 1 + (acc ? 1 : 0);
      }
    }
    mine = next;
  }
  if (live && node == 0) {
    float* st = t.state() + 8 * (size_t)c;
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

// F of every (proxy, octant): the max over the proxy's probes of
// f_d = Qv (Cv + mu Cr), from the pilot codes of the last odd frame and the
// box sums in box_a; marks cleared.
__global__ void dyn_proxy_kernel(VolumeView v) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int Pp = v.pdx * v.pdy * v.pdz;
  if (e >= 8 * Pp) return;
  const int q = e >> 3, k = e & 7;
  const int X = q % v.pdx, Y = (q / v.pdx) % v.pdy, Z = q / (v.pdx * v.pdy);
  const int64_t mu = v.fp->mu;
  int64_t best = 0;
  for (int z = 3 * Z; z < min(3 * Z + 3, v.dz); ++z)
    for (int y = 3 * Y; y < min(3 * Y + 3, v.dy); ++y)
      for (int x = 3 * X; x < min(3 * X + 3, v.dx); ++x) {
        const int i = x + v.dx * (y + v.dy * z);
        const int2 c = v.box_a[8 * i + k];
        const int64_t fd = (int64_t)v.qv[1][8 * i + k] * ((int64_t)c.x + mu * (int64_t)c.y);
        best = max(best, fd);
      }
  v.dyn_F[e] = (float)best;
  v.dyn_mark[e] = 0;
}

// Dynamic rays of every probe: the texel-centre rays of the marked octants of
// its proxy; dyn_off[0] = 0 (the scan fills the rest).
__global__ void dyn_count_kernel(VolumeView v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) v.dyn_off[0] = 0u;
  if (i >= v.P) return;
  const int x = i % v.dx, y = (i / v.dx) % v.dy, z = i / (v.dx * v.dy);
  const int q = x / 3 + v.pdx * (y / 3 + v.pdy * (z / 3));
  const DynTables& tb = *v.dyn_tab;
  uint32_t n = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (v.dyn_mark[8 * q + k])
      n += (uint32_t)(tb.start_i[k + 1] - tb.start_i[k]) + (uint32_t)(tb.start_d[k + 1] - tb.start_d[k]);
  v.dyn_n[i] = n;
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

template <class T>
static hipError_t launch_chain_kernel(const VolumeView& v, int chains, int lanes, hipStream_t s) {
  const long long threads = (long long)chains * lanes;
  const dim3 grid((unsigned)((threads + 255) / 256));
  switch (lanes) {
    case 1:
      hipLaunchKernelGGL(chain_kernel<T>, dim3((chains + 127) / 128), dim3(128), 0, s, v);
      break;
    case 4:
      hipLaunchKernelGGL((chain_prefetch_kernel<2, T>), grid, dim3(256), 0, s, v);
      break;
    case 8:
      hipLaunchKernelGGL((chain_prefetch_kernel<3, T>), grid, dim3(256), 0, s, v);
      break;
    case 16:
      hipLaunchKernelGGL((chain_prefetch_kernel<4, T>), grid, dim3(256), 0, s, v);
      break;
    case 32:
      hipLaunchKernelGGL((chain_prefetch_kernel<5, T>), grid, dim3(256), 0, s, v);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_chains(const VolumeView& v, bool fp16, const void* irr, int chains, int lanes, uint32_t samples,
                         void* sort_temp, uint32_t sample_cap, hipStream_t s) {
  hipLaunchKernelGGL(chain_clear_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  const int m = (v.irr_res - 2) / 2;
  const long long cells = (long long)v.P * m * m;
  if (fp16)
    hipLaunchKernelGGL(chain_lum_kernel<true>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, v, irr);
  else
    hipLaunchKernelGGL(chain_lum_kernel<false>, dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, s, v, irr);
  hipError_t e = launch_chain_kernel<StaticChain>(v, chains, lanes, s);
  if (e != hipSuccess) return e;
  // stable sort of (probe, uv) by probe: a probe's samples stay in
  // chain-major order; then the per-probe offsets
  e = launch_sample_sort(v, samples, sample_cap, sort_temp, s);
  if (e != hipSuccess) return e;
  return launch_offsets_scan((const uint32_t*)v.n, v.P, v.offsets, sample_cap, sort_temp, s);
}

hipError_t launch_dyn_chains(const VolumeView& v, int chains, int lanes, void* scan_temp, uint32_t sample_cap,
                             hipStream_t s) {
  const int Pp = v.pdx * v.pdy * v.pdz;
  hipLaunchKernelGGL(dyn_proxy_kernel, dim3((8 * Pp + 255) / 256), dim3(256), 0, s, v);
  hipError_t e = launch_chain_kernel<DynamicChain>(v, chains, lanes, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(dyn_count_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, v);
  return launch_offsets_scan((const uint32_t*)v.dyn_n, v.P, v.dyn_off, sample_cap, scan_temp, s);
}

}  // namespace adgi
