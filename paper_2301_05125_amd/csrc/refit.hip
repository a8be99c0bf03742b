// refit.hip - device BVH refit after vertex motion (same topology).
//
// 1. Every triangle record (v0, e1, e2) and triangle box with a vertex in
//    the moved range is rebuilt from the current positions (a thread per
//    triangle slot), then every leaf child slot holding such a triangle gets
//    the (padded) union of its leaf's triangle boxes (a thread per leaf slot;
//    a leaf's triangles are contiguous). The least and greatest vertex index
//    of every triangle slot and leaf slot, set once per build, rule out the
//    others without reading their triangles.
// 2. The internal child slots, from the deepest internal nodes to the root:
//    the union of the child's two slots, which a deeper level finished. The
//    levels below a cut depth run in one launch, one workgroup per subtree
//    rooted at the cut, level after level with a barrier between them (a
//    subtree only reads its own nodes); the levels above the cut follow, runs
//    of small levels in one workgroup, a large level in a launch of its own.
//    Kernel boundaries and barriers order the levels, so no cross-workgroup
//    atomics or cache maintenance are needed.
#include "adgi_internal.hpp"

#include <algorithm>
#include <climits>
#include <cstring>

namespace adgi {

// Record of triangle slot s (original triangle t): (v0, t), e1, e2.
__device__ __forceinline__ void write_tri(const RefitView& r, int s, int t, const float* v0, const float* v1,
                                          const float* v2) {
  r.tris[3 * (size_t)s] = make_float4(v0[0], v0[1], v0[2], __int_as_float(t));
  r.tris[3 * (size_t)s + 1] = make_float4(v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2], 0.f);
  r.tris[3 * (size_t)s + 2] = make_float4(v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2], 0.f);
}

// Whether [lo, hi] (a slot's vertex indices lie in it) meets the moved range
// [vb, ve); when it does not, no vertex of the slot moved.
__device__ __forceinline__ bool range_meets(int2 vr, int vb, int ve) { return vr.y >= vb && vr.x < ve; }

// Record of triangle slot s and its box (min xyz, max xyz of its vertices),
// for the triangles with a vertex in this refit's range; the others did not
// move, and their records and boxes from an earlier refit or the build stand.
// The slot's vertex-index range, read in slot order, rules out most of them
// before the triangle's own indices are gathered.
__global__ void refit_tris_kernel(RefitView r) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= r.num_tris) return;
  const int vb = r.range[0], ve = r.range[1];
  if (!range_meets(r.slot_vrange[s], vb, ve)) return;
  const int t = r.tri_order[s];
  const int i0 = r.indices[3 * t], i1 = r.indices[3 * t + 1], i2 = r.indices[3 * t + 2];
  if (!((i0 >= vb && i0 < ve) || (i1 >= vb && i1 < ve) || (i2 >= vb && i2 < ve))) return;
  const float* p[3] = {r.positions + 3 * (size_t)i0, r.positions + 3 * (size_t)i1, r.positions + 3 * (size_t)i2};
  write_tri(r, s, t, p[0], p[1], p[2]);
  float* b = r.tri_box + 6 * (size_t)s;
  for (int a = 0; a < 3; ++a) {
    b[a] = fminf(fminf(p[0][a], p[1][a]), p[2][a]);
    b[3 + a] = fmaxf(fmaxf(p[0][a], p[1][a]), p[2][a]);
  }
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

// Bounds of a leaf child slot (padded): the union of its triangles' boxes,
// which refit_tris_kernel left in tri_box (a leaf's slots are contiguous).
__device__ __forceinline__ void refit_leaf_slot(const RefitView& r, int g, int side) {
  const int* meta = (const int*)(r.nodes + 4 * (size_t)g + 3);
  const int code = ~meta[side];
  const int first = code >> kLeafShift, count_t = (code & (kLeafMaxTris - 1)) + 1;
  float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int k = 0; k < count_t; ++k) {
    const float* b = r.tri_box + 6 * (size_t)(first + k);
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(lo[a], b[a]);
      hi[a] = fmaxf(hi[a], b[3 + a]);
    }
  }
  for (int a = 0; a < 3; ++a) {
    lo[a] = pad_lo(lo[a], r.pad_abs);
    hi[a] = pad_hi(hi[a], r.pad_abs);
  }
  write_slot(r.nodes + 4 * (size_t)g, side, lo, hi);
}

// Internal child slots of node g: the union of the child's two (already
// padded) slots. Leaf slots are done beforehand by refit_leaves_kernel.
__device__ __forceinline__ void refit_node(const RefitView& r, int g) {
  const int* meta = (const int*)(r.nodes + 4 * (size_t)g + 3);
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int c = meta[side];
    if (c < 0) continue;
    const float* f = (const float*)(r.nodes + 4 * (size_t)c);
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = fminf(f[a], f[6 + a]);
      hi[a] = fmaxf(f[3 + a], f[9 + a]);
    }
    write_slot(r.nodes + 4 * (size_t)g, side, lo, hi);
  }
}

// Every leaf child slot (entry 2g + side of leaf_slots) with a triangle that
// has a vertex in the moved range, all independent; the others keep their
// bounds, which their unchanged triangle boxes would give again.
__global__ void refit_leaves_kernel(RefitView r) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < r.num_leaf_slots && range_meets(r.leaf_vrange[q], r.range[0], r.range[1])) {
    const int e = r.leaf_slots[q];
    refit_leaf_slot(r, e >> 1, e & 1);
  }
}

__global__ void slot_vrange_kernel(RefitView r) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= r.num_tris) return;
  const int t = r.tri_order[s];
  const int i0 = r.indices[3 * t], i1 = r.indices[3 * t + 1], i2 = r.indices[3 * t + 2];
  r.slot_vrange[s] = make_int2(min(min(i0, i1), i2), max(max(i0, i1), i2));
}

__global__ void leaf_vrange_kernel(RefitView r) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= r.num_leaf_slots) return;
  const int e = r.leaf_slots[q];
  const int* meta = (const int*)(r.nodes + 4 * (size_t)(e >> 1) + 3);
  const int code = ~meta[e & 1];
  const int first = code >> kLeafShift, count_t = (code & (kLeafMaxTris - 1)) + 1;
  int2 vr = make_int2(INT_MAX, -1);
  for (int k = 0; k < count_t; ++k) {
    const int2 t = r.slot_vrange[first + k];
    vr.x = min(vr.x, t.x);
    vr.y = max(vr.y, t.y);
  }
  r.leaf_vrange[q] = vr;
}

hipError_t launch_refit_ranges(const RefitView& r, hipStream_t s) {
  if (r.num_tris == 0) return hipSuccess;
  hipLaunchKernelGGL(slot_vrange_kernel, dim3((r.num_tris + 255) / 256), dim3(256), 0, s, r);
  if (r.num_leaf_slots > 0)
    hipLaunchKernelGGL(leaf_vrange_kernel, dim3((r.num_leaf_slots + 255) / 256), dim3(256), 0, s, r);
  return hipGetLastError();
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

// One workgroup per subtree rooted at depth r.cut: its nodes of every deeper
// level, deepest first.
__global__ __launch_bounds__(256) void refit_deep_kernel(RefitView r) {
  const int sub = blockIdx.x, stride = r.subtrees + 1;
  for (int k = r.deep_levels - 1; k >= 0; --k) {
    const int lo = r.tab[k * stride + sub], hi = r.tab[k * stride + sub + 1];
    for (int q = lo + (int)threadIdx.x; q < hi; q += (int)blockDim.x) refit_node(r, r.level_nodes[q]);
    __syncthreads();
  }
}

// Cut depth: levels 0..kRefitCut-1 (at most 2^d nodes each) stay above it.
constexpr int kRefitCut = 10;

void plan_refit(const BvhHost& bvh, RefitPlan& p) {
  p.level_nodes = bvh.level_nodes;
  p.level_offsets = bvh.level_offsets;
  p.leaf_slots.clear();
  for (size_t g = 0; g < bvh.nodes.size() / 4; ++g)
    for (int side = 0; side < 2; ++side) {
      int c;
      std::memcpy(&c, side ? &bvh.nodes[4 * g + 3].y : &bvh.nodes[4 * g + 3].x, 4);
      if (c < 0) p.leaf_slots.push_back((int32_t)(2 * g + side));
    }
  p.tab.clear();
  p.cut = p.subtrees = p.deep_levels = 0;
  const int levels = (int)bvh.level_offsets.size() - 1;
  if (levels <= kRefitCut) return;
  const int cut = kRefitCut;
  const int S = bvh.level_offsets[cut + 1] - bvh.level_offsets[cut];
  if (S <= 0) return;
  const size_t nn = bvh.nodes.size() / 4;
  std::vector<int32_t> sub(nn, -1);
  for (int s = 0; s < S; ++s) sub[bvh.level_nodes[bvh.level_offsets[cut] + s]] = s;
  for (int d = cut + 1; d < levels; ++d)
    for (int q = bvh.level_offsets[d]; q < bvh.level_offsets[d + 1]; ++q) {
      const int g = bvh.level_nodes[q];
      int par;
      std::memcpy(&par, &bvh.nodes[4 * (size_t)g + 3].z, 4);
      sub[g] = sub[par];
    }
  p.cut = cut;
  p.subtrees = S;
  p.deep_levels = levels - cut;
  p.tab.assign((size_t)p.deep_levels * (S + 1), 0);
  for (int d = cut; d < levels; ++d) {
    const int b = bvh.level_offsets[d], e = bvh.level_offsets[d + 1];
    std::stable_sort(p.level_nodes.begin() + b, p.level_nodes.begin() + e,
                     [&](int32_t x, int32_t y) { return sub[x] < sub[y]; });
    int32_t* t = &p.tab[(size_t)(d - cut) * (S + 1)];
    int q = b;
    for (int s = 0; s <= S; ++s) {
      while (q < e && sub[p.level_nodes[q]] < s) ++q;
      t[s] = q;
    }
  }
}

hipError_t launch_refit(const RefitView& r, const std::vector<int32_t>& level_offsets, hipStream_t s) {
  if (r.num_tris == 0) return hipSuccess;
  hipLaunchKernelGGL(refit_tris_kernel, dim3((r.num_tris + 255) / 256), dim3(256), 0, s, r);
  if (level_offsets.size() < 2) return hipGetLastError();  // no internal node
  if (r.num_leaf_slots > 0)
    hipLaunchKernelGGL(refit_leaves_kernel, dim3((r.num_leaf_slots + 255) / 256), dim3(256), 0, s, r);
  if (r.subtrees > 0) hipLaunchKernelGGL(refit_deep_kernel, dim3(r.subtrees), dim3(256), 0, s, r);
  RefitRun run;
  run.n = 0;
  auto flush = [&]() {
    if (run.n > 0) hipLaunchKernelGGL(refit_run_kernel, dim3(1), dim3(kRefitSmall), 0, s, r, run);
    run.n = 0;
  };
  const int top = r.subtrees > 0 ? r.cut : (int)level_offsets.size() - 1;
  for (int d = top - 1; d >= 0; --d) {
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
