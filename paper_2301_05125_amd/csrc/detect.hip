// detect.hip - per-frame setup and change detection -> per-probe scores.
//
// On the second frame of each pair (odd t) the pilot codes of this frame and
// the previous one give the temporal gradient d = |Q_t - Q_{t-1}| of probe
// visibility and radiance (eq. tempGradVis, eq. tempGradIrr), the temporal
// trigger T <- max(d, T - ceil(1023/theta)) turns a change into a linearly
// decaying signal (Sec. 4.1.4), and an unnormalised 5x5x5 box sum over
// probes, zero padded, spreads it in space (the spatial convolution of
// Sec. 4.1.4-4.1.5; the directional part is per probe a constant and is
// dropped). The score sum_k Qv (Cv + mu Cr) is the dynamic composition
// f_v (f_dv + mu f_dr) of eq. priorDynamic, summed over the eight octants.
// Everything after the 10-bit codes is integer arithmetic, so the result is
// exact. The box sum is separable: three 5-tap passes along x, y and z.
#include "adgi_internal.hpp"

namespace adgi {

__global__ void frame_begin_kernel(VolumeView v) {
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  FrameStats* st = v.stats;
  if (tid < kAllocPasses * kAllocCandidates) v.lam_sums[(size_t)tid * kLamLine] = 0ull;
  if (tid < kOrderBuckets) {
    st->bucket_count[tid] = 0u;
    st->bucket_cursor[tid] = 0u;
  }
  if (tid == 0) {
    st->shadow_rays = 0ull;
    st->max_score = 0ull;
    st->lambda = 0u;
    st->n_min_seen = 0;
    st->n_max_seen = 0;
    st->budget_used = 0ull;
    st->node_tests = 0ull;
    st->tri_tests = 0ull;
    st->shade_node_tests = 0ull;
    st->shade_tri_tests = 0ull;
    st->box_tests = 0ull;
    st->shade_box_tests = 0ull;
    st->remainder = 0;
  }
  if (v.fp->frame == 0 && tid < v.P) v.score[tid] = 0;
}

__global__ void trigger_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive || (fp.frame & 1) == 0) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8 * v.P) return;
  const int delta = (1023 + fp.theta - 1) / fp.theta;
  int dv = abs((int)v.qv[1][e] - (int)v.qv[0][e]);
  int dr = abs((int)v.qr[1][e] - (int)v.qr[0][e]);
  int2 t = v.trig[e];
  t.x = max(dv, t.x - delta);
  t.y = max(dr, t.y - delta);
  v.trig[e] = t;
}

// 5-tap sum along one grid axis; element e = probe * 8 + octant. The axis is
// given by its probe-index divisor (1, dx, dx*dy) and extent (dx, dy, dz), so
// the kernel is straight-line code: the coordinate along the axis is
// (i / div) % D and neighbours are 8 * div elements apart.
__global__ void box_pass_kernel(VolumeView v, const int2* __restrict__ src, int2* __restrict__ dst,
                                int div, int D, int force) {
  const FrameParams& fp = *v.fp;
  if (!force && (!fp.adaptive || (fp.frame & 1) == 0)) return;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= 8 * v.P) return;
  const int i = e >> 3;
  const int c = (i / div) % D;
  const int stride = 8 * div;
  int sx = 0, sy = 0;
#pragma unroll
  for (int o = -2; o <= 2; ++o) {
    const int cc = c + o;
    if (cc >= 0 && cc < D) {
      const int2 t = src[e + o * stride];
      sx += t.x;
      sy += t.y;
    }
  }
  dst[e] = make_int2(sx, sy);
}

__global__ void score_kernel(VolumeView v) {
  const FrameParams& fp = *v.fp;
  if (!fp.adaptive || (fp.frame & 1) == 0) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= v.P) return;
  const int64_t mu = fp.mu;
  int64_t s = 0;
  for (int k = 0; k < 8; ++k) {
    int2 c = v.box_b[8 * i + k];
    s += (int64_t)v.qv[1][8 * i + k] * ((int64_t)c.x + mu * (int64_t)c.y);
  }
  v.score[i] = s;
}

hipError_t launch_frame_begin(const VolumeView& v, hipStream_t s) {
  int n = v.P > 4 * kAllocCandidates ? v.P : 4 * kAllocCandidates;
  hipLaunchKernelGGL(frame_begin_kernel, dim3((n + 255) / 256), dim3(256), 0, s, v);
  return hipGetLastError();
}

hipError_t launch_box_sums(const VolumeView& v, hipStream_t s) {
  const int n = 8 * v.P, g = (n + 255) / 256;
  hipLaunchKernelGGL(box_pass_kernel, dim3(g), dim3(256), 0, s, v, (const int2*)v.trig, v.box_a, 1, v.dx, 1);
  hipLaunchKernelGGL(box_pass_kernel, dim3(g), dim3(256), 0, s, v, (const int2*)v.box_a, v.box_b, v.dx,
                     v.dy, 1);
  hipLaunchKernelGGL(box_pass_kernel, dim3(g), dim3(256), 0, s, v, (const int2*)v.box_b, v.box_a,
                     v.dx * v.dy, v.dz, 1);
  return hipGetLastError();
}

hipError_t launch_detect(const VolumeView& v, hipStream_t s) {
  const int n = 8 * v.P, g = (n + 255) / 256;
  hipLaunchKernelGGL(trigger_kernel, dim3(g), dim3(256), 0, s, v);
  // box sum: trig -> a (x) -> b (y) -> a (z); the score reads a
  hipLaunchKernelGGL(box_pass_kernel, dim3(g), dim3(256), 0, s, v, (const int2*)v.trig, v.box_a, 1, v.dx, 0);
  hipLaunchKernelGGL(box_pass_kernel, dim3(g), dim3(256), 0, s, v, (const int2*)v.box_a, v.box_b, v.dx,
                     v.dy, 0);
  hipLaunchKernelGGL(box_pass_kernel, dim3(g), dim3(256), 0, s, v, (const int2*)v.box_b, v.box_a,
                     v.dx * v.dy, v.dz, 0);
  VolumeView w = v;
  w.box_b = v.box_a;  // score reads the z-pass output
  hipLaunchKernelGGL(score_kernel, dim3((v.P + 255) / 256), dim3(256), 0, s, w);
  return hipGetLastError();
}

}  // namespace adgi
