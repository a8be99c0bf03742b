// refit.hip - device BVH refit after vertex motion (same topology).
//
// 1. Rebuild every triangle record (v0, e1, e2) from the current positions.
// 2. Refit the boxes level by level from the deepest internal nodes to the
//    root: a node's child slot gets the (padded) bounds of its leaf
//    triangles, or the union of the internal child's two slots, which the
//    previous level finished. A level with many nodes gets a launch of its
//    own; a run of consecutive small levels (the thin bottom of the tree, the
//    top) runs in one workgroup with a barrier between levels. Kernel
//    boundaries and barriers order the levels, so no cross-workgroup atomics
//    or cache maintenance are needed.
#include "adgi_internal.hpp"

namespace adgi {

__global__ void refit_tris_kernel(RefitView r) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= r.num_tris) return;
  const int t = r.tri_order[s];
  const float* v0 = r.positions + 3 * (size_t)r.indices[3 * t];
  const float* v1 = r.positions + 3 * (size_t)r.indices[3 * t + 1];
  const float* v2 = r.positions + 3 * (size_t)r.indices[3 * t + 2];
  float4 a = make_float4(v0[0], v0[1], v0[2], __int_as_float(t));
  r.tris[3 * (size_t)s] = a;
  r.tris[3 * (size_t)s + 1] = make_float4(v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2], 0.f);
  r.tris[3 * (size_t)s + 2] = make_float4(v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2], 0.f);
}

__device__ __forceinline__ void write_slot(float4* node, int side, const float* lo, const float* hi) {
  float* f = (float*)node;
  const int b = side ? 6 : 0;
  f[b + 0] = lo[0];
  f[b + 1] = lo[1];
  f[b + 2] = lo[2];
  f[b + 3] = hi[0];
  f[b + 4] = hi[1];
  f[b + 5] = hi[2];
}

__device__ __forceinline__ void refit_node(const RefitView& r, int g) {
  const int* meta = (const int*)(r.nodes + 4 * (size_t)g + 3);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int c = meta[side];
    float lo[3], hi[3];
    if (c < 0) {
      const int code = ~c;
      const int first = code >> kLeafShift, count_t = (code & (kLeafMaxTris - 1)) + 1;
      lo[0] = lo[1] = lo[2] = INFINITY;
      hi[0] = hi[1] = hi[2] = -INFINITY;
      for (int k = 0; k < count_t; ++k) {
        const int t = r.tri_order[first + k];
        for (int v = 0; v < 3; ++v) {
          const float* p = r.positions + 3 * (size_t)r.indices[3 * t + v];
          for (int a = 0; a < 3; ++a) {
            lo[a] = fminf(lo[a], p[a]);
            hi[a] = fmaxf(hi[a], p[a]);
          }
        }
      }
      for (int a = 0; a < 3; ++a) {
        lo[a] = pad_lo(lo[a], r.pad_abs);
        hi[a] = pad_hi(hi[a], r.pad_abs);
      }
    } else {
      // union of the child's two (already padded) slots
      const float* f = (const float*)(r.nodes + 4 * (size_t)c);
      for (int a = 0; a < 3; ++a) {
        lo[a] = fminf(f[a], f[6 + a]);
        hi[a] = fmaxf(f[3 + a], f[9 + a]);
      }
    }
    write_slot(r.nodes + 4 * (size_t)g, side, lo, hi);
  }
}

__global__ void refit_level_kernel(RefitView r, const int32_t* __restrict__ nodes_of_level, int count) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) refit_node(r, nodes_of_level[q]);
}

// Consecutive levels of at most kRefitSmall nodes, deepest first: level k
// holds level_nodes[lo[k], hi[k]).
constexpr int kRefitSmall = 1024;
constexpr int kRefitRunMax = 64;
struct RefitRun {
  int n;
  int lo[kRefitRunMax], hi[kRefitRunMax];
};

__global__ __launch_bounds__(kRefitSmall) void refit_run_kernel(RefitView r, RefitRun run) {
  for (int k = 0; k < run.n; ++k) {
    for (int q = run.lo[k] + (int)threadIdx.x; q < run.hi[k]; q += (int)blockDim.x)
      refit_node(r, r.level_nodes[q]);
    __syncthreads();
  }
}

hipError_t launch_refit(const RefitView& r, const std::vector<int32_t>& level_offsets, hipStream_t s) {
  if (r.num_tris == 0) return hipSuccess;
  hipLaunchKernelGGL(refit_tris_kernel, dim3((r.num_tris + 255) / 256), dim3(256), 0, s, r);
  RefitRun run;
  run.n = 0;
  auto flush = [&]() {
    if (run.n > 0) hipLaunchKernelGGL(refit_run_kernel, dim3(1), dim3(kRefitSmall), 0, s, r, run);
    run.n = 0;
  };
  for (int d = (int)level_offsets.size() - 2; d >= 0; --d) {
    const int b = level_offsets[d], cnt = level_offsets[d + 1] - b;
    if (cnt <= 0) continue;
    if (cnt <= kRefitSmall) {
      if (run.n == kRefitRunMax) flush();
      run.lo[run.n] = b;
      run.hi[run.n] = b + cnt;
      ++run.n;
      continue;
    }
    flush();
    hipLaunchKernelGGL(refit_level_kernel, dim3((cnt + 255) / 256), dim3(256), 0, s, r,
                       r.level_nodes + b, cnt);
  }
  flush();
  return hipGetLastError();
}

// BVH4 child slot k of node n copies BVH2 child slot src = 2g + side.
__global__ void bvh4_gather_kernel(float4* __restrict__ nodes4, const int32_t* __restrict__ src,
                                   int num_slots, const float4* __restrict__ nodes2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= num_slots) return;
  const int ref = src[q];
  if (ref < 0) return;
  const float* b = (const float*)(nodes2 + 4 * (size_t)(ref >> 1)) + 6 * (ref & 1);
  float* f = (float*)(nodes4 + 8 * (size_t)(q >> 2));
  const int k = q & 3;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    f[4 * a + k] = b[a];
    f[12 + 4 * a + k] = b[3 + a];
  }
}

hipError_t launch_bvh4_gather(float4* nodes4, const int32_t* src, int num_nodes4, const float4* nodes2,
                              hipStream_t s) {
  const int slots = 4 * num_nodes4;
  if (slots <= 0) return hipSuccess;
  hipLaunchKernelGGL(bvh4_gather_kernel, dim3((slots + 255) / 256), dim3(256), 0, s, nodes4, src, slots,
                     nodes2);
  return hipGetLastError();
}

}  // namespace adgi
