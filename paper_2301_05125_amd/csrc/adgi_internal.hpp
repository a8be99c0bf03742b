// adgi_internal.hpp - kernel launchers and host-side helpers of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/adgi.h"
#include "adgi_device.hpp"
#include "adgi_layout.hpp"

namespace adgi {

// trace.hip
size_t trace_lds_bytes(int block);
// w4: traverse the BVH4 (v.nodes4) instead of the BVH2. chain: the two rays of
// each chain sample (probe rays otherwise).
hipError_t launch_trace(const VolumeView& v, hipStream_t s, bool pilot, bool persistent, int block,
                        int grid, int shade_grid, bool count = false, bool w4 = false, bool chain = false,
                        hipEvent_t between = nullptr);

// chain.hip: one frame of `chains` Metropolis chains, then their samples
// sorted by probe (v.smp_probe / v.smp_uv, v.offsets / v.n as per-probe
// sample ranges). samples = chains * (steps - burn_in - 1). lanes: 1 (one
// thread per chain) or 4 / 8 / 16 (prefetching groups); chain_lanes_auto
// picks one from the chain count.
int chain_lanes_auto(int chains);
// alloc.hip: blend order (most 64-entry chunks first) from counts already in v.n
hipError_t launch_blend_order(const VolumeView& v, hipStream_t s);
hipError_t launch_chains(const VolumeView& v, bool fp16, const void* irr, int chains, int lanes, uint32_t samples,
                         void* sort_temp, uint32_t sample_cap, hipStream_t s);
// chain.hip: F per (proxy, octant) from f_d (needs the box sums in box_a),
// one frame of the dynamic chains (marks), per-probe dynamic ray counts and
// their scan into v.dyn_off.
hipError_t launch_dyn_chains(const VolumeView& v, int chains, int lanes, void* scan_temp, uint32_t sample_cap,
                             hipStream_t s);
// sort.hip: the chain samples (v.smp_probe_raw / v.smp_uv_raw, S of them)
// sorted by probe, stably, into v.smp_probe / v.smp_uv; exclusive scan of P
// counts into offsets[0..P] (offsets[P] the total). Both use a workspace of
// sort_temp_bytes(cap, P) bytes for up to cap samples.
size_t sort_temp_bytes(uint32_t cap, int P);
hipError_t launch_sample_sort(const VolumeView& v, uint32_t S, uint32_t cap, void* temp, hipStream_t s);
hipError_t launch_offsets_scan(const uint32_t* counts, int P, uint32_t* offsets, uint32_t cap, void* temp,
                               hipStream_t s);
// detect.hip: the three 5-tap passes of the box sum into box_a, whatever the
// frame (the dynamic chains read them on even frames too)
hipError_t launch_box_sums(const VolumeView& v, hipStream_t s);

// query.hip: irradiance at count points (device [count][3] points, normals,
// out) from the bordered tiles
hipError_t launch_query(const VolumeView& v, bool fp16, const void* irr, const void* dep, const float* pts,
                        const float* nrm, float* out, int64_t count, hipStream_t s);

// detect.hip: trigger update and the separable 5x5x5 box sum -> scores
hipError_t launch_frame_begin(const VolumeView& v, hipStream_t s);
hipError_t launch_detect(const VolumeView& v, hipStream_t s);

// alloc.hip: integer budget split and exclusive scan
hipError_t launch_alloc(const VolumeView& v, hipStream_t s);
hipError_t launch_uniform_offsets(const VolumeView& v, hipStream_t s);

// blend.hip: per-probe texel update and border fold
struct BlendIO {
  const void* irr_in;
  const void* dep_in;
  const uint8_t* irr_n_in;
  const uint8_t* dep_n_in;
  void* irr_out;
  void* dep_out;
  uint8_t* irr_n_out;
  uint8_t* dep_n_out;
};
// Packed round trip of n device values through channel 0..3 (R/G 9 bits, B 8
// bits, tau 13 bits, tau^2 13 bits); dec/up: the decode table and its
// rounding bits (kPkDecSize floats, then kPkUpWords words).
hipError_t launch_pack_channel(const float* x, int64_t n, int channel, const float* dec, const uint32_t* up,
                               uint32_t* codes, float* decoded, hipStream_t s);
// Once per volume before its first blend (ADGI_PACKED raises the packed
// kernel's dynamic LDS limit).
hipError_t blend_prepare(int irr_res, int dep_res, int storage);
// chunk = 0 selects the wave-per-probe kernel (tile sizes 8/16 and 16/16) with
// `grid` workgroups walking the allocation's probe order; otherwise one
// workgroup per probe with `chunk` rays staged per step.
// storage: ADGI_FP32, ADGI_FP16 or ADGI_PACKED (wave kernel only; packed:
// `grid` workgroups of 16 waves, one per CU)
// chain: the lists are chain samples (wave kernel; not with ADGI_PACKED)
// gather: DDGI's cosine-weighted gather instead of the per-sample update
// (wave kernel; not with ADGI_PACKED or chain frames)
hipError_t launch_blend(const VolumeView& v, const BlendIO& io, hipStream_t s, int storage, int chunk,
                        int grid = 0, bool chain = false, bool gather = false);
bool blend_wave_supported(const VolumeView& v);
size_t blend_lds_bytes(const VolumeView& v, int chunk);

// refit.hip
struct RefitView {
  const float* positions;      // [V][3]
  const int32_t* indices;      // [T][3]
  const int32_t* tri_order;    // slot -> original triangle
  float4* tris;                // [T][3]
  float4* nodes;               // [N][4]
  const int32_t* level_nodes;  // node indices grouped by depth (RefitPlan order)
  int32_t num_tris;
  int32_t num_nodes;
  float pad_abs;
  const int32_t* tab;          // RefitPlan::tab on the device
  int32_t cut, subtrees, deep_levels;
  const int32_t* leaf_slots;   // RefitPlan::leaf_slots on the device
  int32_t num_leaf_slots;
  float* tri_box;              // [T][6] each triangle slot's box, kept from refit to refit
  const int32_t* range;        // [2] on the device: the vertex range this refit moves
  int2* slot_vrange;           // [T] least and greatest vertex index of each triangle slot
  int2* leaf_vrange;           // [num_leaf_slots] the same over each leaf slot's triangles
};
// Refit plan of a BVH2: the internal nodes at depth >= cut are grouped, in
// every level, by their ancestor at depth `cut` (one subtree per workgroup,
// all its levels in one launch); the levels above are refit separately.
// tab[(d - cut) * (subtrees + 1) + s] is where subtree s starts in level d's
// part of level_nodes (s = subtrees: the level's end). cut = 0: no deep part.
struct RefitPlan {
  int32_t cut = 0, subtrees = 0, deep_levels = 0;
  std::vector<int32_t> level_nodes;
  std::vector<int32_t> level_offsets;  // size levels + 1
  std::vector<int32_t> tab;
  std::vector<int32_t> leaf_slots;     // 2g + side of every child slot that holds a leaf
};
// level_offsets[d] .. level_offsets[d+1] index level_nodes for depth d
hipError_t launch_refit(const RefitView& r, const std::vector<int32_t>& level_offsets, hipStream_t s);
// The vertex-index ranges of the triangle and leaf slots, once per build
// (indices and tri_order uploaded, in stream order).
hipError_t launch_refit_ranges(const RefitView& r, hipStream_t s);
// Copy refitted BVH2 child boxes into the BVH4 nodes (one thread per slot).
hipError_t launch_bvh4_gather(float4* nodes4, const int32_t* src, int num_nodes4, const float4* nodes2,
                              hipStream_t s);

// bvh_build.cpp: binned SAH on the host
struct BvhHost {
  std::vector<float4> nodes;       // 4 per node
  std::vector<float4> tris;        // 3 per triangle slot
  std::vector<int32_t> tri_order;  // slot -> original triangle
  std::vector<int32_t> level_nodes;   // internal nodes grouped by depth (root first)
  std::vector<int32_t> level_offsets; // size depth+1
  int32_t depth = 0;
  int32_t num_big = 0;             // slots [0, num_big): large triangles outside the tree
};
bool build_bvh(const float* positions, int32_t nv, const int32_t* indices, int32_t nt, float pad_abs,
               BvhHost& out, const char** err);
void plan_refit(const BvhHost& bvh, RefitPlan& plan);
// BVH4 collapse of a BVH2 (node layout in adgi_layout.hpp), nodes in
// depth-first order. src[4n+k] = 2*g + side names the BVH2 child slot that
// child k of node n copies (-1: empty), so a refit of the BVH2 is carried over
// by a gather. max_stack is the worst-case traversal stack depth.
struct Bvh4Host {
  std::vector<float4> nodes;   // 8 per node
  std::vector<int32_t> src;    // 4 per node
  int32_t max_stack = 0;
};
void collapse_bvh4(const BvhHost& b2, Bvh4Host& out);

// volume.hip: a REBUILD split into its host build and the device install, so
// a caller that keeps scenes on the host (the server) builds each BVH once.
// Arrays a REBUILD uploads besides the vertex positions, in the order of
// their offsets inside a pinned scene image.
enum PinPart { kPinIdx, kPinOrder, kPinTris, kPinLevels, kPinTab, kPinLeaf, kPinNodes, kPinAlbedo, kPinNodes4,
               kPinSrc4, kPinParts };
struct BuiltScene {
  BvhHost bvh;
  Bvh4Host bvh4;
  RefitPlan plan;
  bool fits4 = false;
  float pad_abs = 0.f;
  double build_ms = 0.0;
  // Optional pinned host copy of the uploaded arrays (pin_scene; released
  // by unpin_scene, not by the destructor). With it a REBUILD from this
  // scene enqueues its uploads on the volume's scene stream and returns
  // before they finish; the image must then outlive every volume it fed.
  uint8_t* pinned = nullptr;
  size_t pin_off[kPinParts] = {}, pin_len[kPinParts] = {};
};
bool build_scene(const adgi_volume_desc& d, const adgi_scene_desc* sc, BuiltScene& out, const char** err);
// Pinned image of `b` for the scene `sc` it was built from; false when the
// pinned allocation fails (the scene then uploads synchronously).
bool pin_scene(BuiltScene& b, const adgi_scene_desc* sc);
void unpin_scene(BuiltScene& b);
// adgi_update_scene with an optional prebuilt BVH for a REBUILD (same checks).
adgi_status update_scene_impl(adgi_volume* vol, const adgi_scene_desc* sc, const BuiltScene* prebuilt);
// adgi_restore_state; with `async` the copies are enqueued on the volume's
// stream, so `src` must stay unchanged until that stream has passed them.
adgi_status restore_state_impl(adgi_volume* vol, const void* src, size_t bytes, bool async);
// adgi_save_state; with `async` the copies are enqueued on the volume's
// stream behind its queued frames, and `dst` holds the snapshot only once
// that stream has passed them.
adgi_status save_state_impl(adgi_volume* vol, void* dst, size_t bytes, bool async);
hipStream_t volume_stream(adgi_volume* vol);
// Runs the volume's later work on `lane` (its scene work too), or on its own
// streams again when lane is NULL. Work queued on the volume's own streams
// is ordered before the lane's; the caller guarantees that the volume's work
// on a lane it leaves is complete, and returns the volume to its own streams
// before destroying it or the lane.
adgi_status bind_streams(adgi_volume* vol, hipStream_t lane);
// True once nothing is queued on the volume's own streams (creation fills,
// scene uploads, state copies), so binding it to a lane adds no wait there.
bool volume_settled(adgi_volume* vol);
// Conservative box padding (builder and refit): a few ulps of the coordinate
// plus an absolute term tied to the scene's coordinate scale, so that FP32
// slab tests from any ray origin in the scene never cull a box a hit lies in.
__host__ __device__ __forceinline__ float pad_lo(float x, float pad_abs) {
  return x - (fabsf(x) * 4.8e-7f + pad_abs);
}
__host__ __device__ __forceinline__ float pad_hi(float x, float pad_abs) {
  return x + (fabsf(x) * 4.8e-7f + pad_abs);
}

}  // namespace adgi
