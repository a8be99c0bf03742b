// refit.hip - device BVH refit after vertex motion (same topology).
//
// 1. Rebuild every triangle record (v0, e1, e2) from the current positions.
// 2. One thread per leaf child slot computes its leaf's box from the vertex
//    positions, writes it (padded) into the parent node, and climbs: at each
//    node an acquire/release arrival counter lets the second arriving child
//    merge both child boxes into the grandparent's slot, so every node is
//    finished exactly once without a launch per level.
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

__global__ void refit_clear_kernel(RefitView r) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < r.num_nodes) r.arrive[k] = 0u;
}

__device__ __forceinline__ void write_slot(float4* node, int side, const float* lo, const float* hi) {
  float* f = (float*)node;
  if (side == 0) {
    f[0] = lo[0];
    f[1] = lo[1];
    f[2] = lo[2];
    f[3] = hi[0];
    f[4] = hi[1];
    f[5] = hi[2];
  } else {
    f[6] = lo[0];
    f[7] = lo[1];
    f[8] = lo[2];
    f[9] = hi[0];
    f[10] = hi[1];
    f[11] = hi[2];
  }
}

__global__ void refit_nodes_kernel(RefitView r) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= r.num_leaf_slots) return;
  const int slot = r.leaf_slots[q];
  int node = slot >> 1;
  const int side = slot & 1;
  const int* meta = (const int*)(r.nodes + 4 * (size_t)node + 3);
  const int code = ~meta[side];
  const int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < count; ++k) {
    const int t = r.tri_order[first + k];
    for (int c = 0; c < 3; ++c) {
      const float* p = r.positions + 3 * (size_t)r.indices[3 * t + c];
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
  write_slot(r.nodes + 4 * (size_t)node, side, lo, hi);
  for (;;) {
    uint32_t prev = __hip_atomic_fetch_add(&r.arrive[node], 1u, __ATOMIC_ACQ_REL,
                                           __HIP_MEMORY_SCOPE_AGENT);
    if (prev == 0u) return;  // the sibling finishes this node
    const int* m = (const int*)(r.nodes + 4 * (size_t)node + 3);
    const int parent = m[2], pside = m[3];
    if (parent < 0) return;
    const float* f = (const float*)(r.nodes + 4 * (size_t)node);
    float blo[3], bhi[3];
    for (int a = 0; a < 3; ++a) {
      blo[a] = fminf(f[a], f[6 + a]);
      bhi[a] = fmaxf(f[3 + a], f[9 + a]);
    }
    write_slot(r.nodes + 4 * (size_t)parent, pside, blo, bhi);
    node = parent;
  }
}

hipError_t launch_refit(const RefitView& r, hipStream_t s) {
  if (r.num_tris > 0)
    hipLaunchKernelGGL(refit_tris_kernel, dim3((r.num_tris + 255) / 256), dim3(256), 0, s, r);
  hipLaunchKernelGGL(refit_clear_kernel, dim3((r.num_nodes + 255) / 256), dim3(256), 0, s, r);
  if (r.num_leaf_slots > 0)
    hipLaunchKernelGGL(refit_nodes_kernel, dim3((r.num_leaf_slots + 255) / 256), dim3(256), 0, s, r);
  return hipGetLastError();
}

}  // namespace adgi
