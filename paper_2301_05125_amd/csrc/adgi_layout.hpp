// adgi_layout.hpp - device data layout shared by the host runtime and kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace adgi {

constexpr uint64_t kTagRotation = 0x524F54ull;  // "ROT"
constexpr uint64_t kTagPilot = 0x50494Cull;     // "PIL"
constexpr uint64_t kTagChain = 0x4D4353ull;     // "MCS": one Metropolis step
constexpr uint64_t kTagChainInit = 0x4D4349ull; // "MCI": a chain's first state
constexpr uint64_t kTagDynChain = 0x4D4453ull;  // "MDS": one dynamic-chain step
constexpr uint64_t kTagDynChainInit = 0x4D4449ull; // "MDI": a dynamic chain's first state
constexpr int kChainMaxSteps = 256;
constexpr int kDynTexels = 196;                  // interior texels of a map, at most (14 x 14)
constexpr int kMaxLights = 8;
constexpr int kPairsPerBatch = 64 * kMaxLights;  // shadow pairs of one 64-ray batch, at most
constexpr int kPairScanPer = 1024;               // batches per block of the pair-count scan
constexpr int kAllocCandidates = 256;           // per k-ary search pass (m = 1..255)
constexpr int kAllocPasses = 4;                 // 2^31+1 -> 1 in four 256-ary steps
constexpr int kLamLine = 16;                    // lambda-pass sums: one per 128-byte line (uint64 stride)
constexpr int kStackLds = 7;                    // traversal stack entries kept in LDS
constexpr int kOrderBuckets = 32;               // blend order: 64-ray chunks per probe, capped
constexpr int kStackMax = 64;                   // BVH depth bound enforced by the builder
constexpr int kPkDecIrr9 = 0, kPkDecIrr8 = 512, kPkDecTau = 768, kPkDecTau2 = 768 + 8192;
constexpr int kPkDecSize = 768 + 2 * 8192;      // decoded values of all packed codes
constexpr int kPkUpWords = (kPkDecSize + 31) / 32;  // one bit per code: decoded value rounded up
constexpr float kShadowOffset = 1e-4f;          // shadow origin offset, units of s
constexpr float kShadowShorten = 1e-6f;         // relative shortening of shadow rays

// BVH2 node: the boxes of both children live in the parent (64 bytes).
//   f[0] = (L.lo.x, L.lo.y, L.lo.z, L.hi.x)
//   f[1] = (L.hi.y, L.hi.z, R.lo.x, R.lo.y)
//   f[2] = (R.lo.z, R.hi.x, R.hi.y, R.hi.z)
//   f[3] = (left, right, parent, side-in-parent) as int bits
// A child c >= 0 is an internal node; c < 0 is a leaf with
// ~c = (first triangle slot << 4) | (count - 1), count in 1..16.
// Node 0 is the root and is always internal.
constexpr int kLeafShift = 4;
constexpr int kLeafMaxTris = 16;

// BVH4 node (128 bytes), derived from the BVH2 by pulling grandchildren up
// into their parent (up to four children per node), child boxes as SoA:
//   f[0] = lo.x[4], f[1] = lo.y[4], f[2] = lo.z[4],
//   f[3] = hi.x[4], f[4] = hi.y[4], f[5] = hi.z[4],
//   f[6] = child[4] as int bits (same codes as BVH2; kEmptyChild = unused),
//   f[7] = unused.
// Every child box is a copy of a BVH2 child slot, so padding is unchanged.
constexpr int kEmptyChild = (int)0x80000000;

// Triangle record in leaf order (48 bytes): (v0, id bits), (e1, 0), (e2, 0).

struct SceneParams {
  float lpos[kMaxLights][4];
  float lint[kMaxLights][4];
  float sky[4];
  int32_t num_lights;
  int32_t num_tris;
  int32_t num_nodes;
  int32_t num_big;    // triangle slots [0, num_big) are tested by every ray before the tree
  // vertices the current refit moves: the refit rebuilds the records and
  // boxes of the triangles that touch [refit_vb, refit_ve) only
  int32_t refit_vb, refit_ve;
};

struct FrameParams {
  float R[12];        // row-major rotation (9 used)
  uint64_t seed;
  int64_t budget;
  int32_t frame;
  int32_t adaptive;
  int32_t n_min, n_max, n_uniform;
  int32_t mu, theta;
  float beta;
  int32_t debug;
  // chain frames (adaptive == 2)
  int32_t chains, chain_steps, chain_burn_in, chain_init;
  float chain_sp[3];          // position step per axis (sigma_pos * spacing)
  float chain_sd;             // octahedral uv step
  // dynamic chains on the 3x3x3 proxies (dyn_chains = 0: none)
  int32_t dyn_chains, dyn_steps, dyn_burn_in, dyn_init;
  float dyn_sp[3];
  float dyn_sd;
  float dyn_one_minus_h;      // 1 - h_dyn: the dynamic updates' step floor
  int32_t pilot_reuse;        // this frame's pilot samples also update the caches
  int32_t pad[2];
};

// Texel-centre ray tables (dynamic updates): the interior texels of the
// irradiance (i) and depth (d) maps in octant order, each octant's start, and
// each texel's octant and rank within its octant.
struct DynTables {
  uint16_t ord_i[kDynTexels], ord_d[kDynTexels];
  uint16_t rank_i[kDynTexels], rank_d[kDynTexels];
  uint8_t oct_i[kDynTexels], oct_d[kDynTexels];
  uint16_t start_i[9], start_d[9];
};

struct FrameStats {
  uint32_t pair_batches;    // 64-ray batches of the last trace pass
  uint32_t pair_total;      // shadow pairs of the last trace pass
  uint64_t shadow_rays;
  uint64_t max_score;
  uint32_t lambda;
  int32_t n_min_seen, n_max_seen;
  int32_t pad;
  uint64_t budget_used;
  uint64_t node_tests;      // work-counting traversal only
  uint64_t tri_tests;
  uint64_t shade_node_tests; // the shading kernel's part of the two above
  uint64_t shade_tri_tests;
  uint64_t box_tests;        // child boxes tested (BVH4: non-empty slots only)
  uint64_t shade_box_tests;
  int64_t remainder;        // R = B' - sum e_i(lambda*)
  uint32_t bucket_count[kOrderBuckets];   // probes per ray-chunk bucket
  uint32_t bucket_cursor[kOrderBuckets];  // scatter cursors
};

// Everything a kernel needs, passed by value.
struct VolumeView {
  // grid
  float ox, oy, oz;
  float sx, sy, sz;
  int32_t dx, dy, dz;
  int32_t P;
  float s_diag;
  int32_t irr_res, dep_res;
  float one_minus_h;
  float tau_max;
  // scene
  const float4* nodes;
  const float4* nodes4;       // BVH4 (null when the collapse does not fit the stack)
  const float4* tris;
  const float4* albedo;       // by original triangle index
  const SceneParams* scene;
  const FrameParams* fp;
  FrameStats* stats;
  // detection
  uint16_t* qv[2];            // [P*8] pilot visibility codes, slot = frame & 1
  uint16_t* qr[2];            // [P*8] pilot radiance codes
  int2* trig;                 // [P*8] (Tv, Tr)
  int2* box_a;                // [P*8] box-sum scratch
  int2* box_b;
  int64_t* score;             // [P]
  // allocation
  int32_t* n;                 // [P]
  uint32_t* offsets;          // [P+1]
  int64_t* blk_e;             // [ceil(P/256)] per-block sum of e_i(lambda*)
  uint32_t* blk_el;           // per-block count of probes eligible for the top-up
  uint32_t* blk_rank;         // per-block exclusive rank base among eligible probes
  uint32_t* blk_off;          // per-block exclusive ray offset
  int32_t* order;             // [P] blend order: most 64-ray chunks first
  // chain frames: state [C][8] = (p.xyz, u, v, -, -, -); samples in chain
  // order (probe, uv) and grouped by probe (sorted)
  float* chain_state;
  uint32_t* smp_probe_raw;
  float2* smp_uv_raw;
  uint32_t* smp_probe;        // sorted
  float2* smp_uv;             // sorted
  float* chain_lum;           // [P][(irr_res-2)/2]^2 g of each coarse cell
  // dynamic chains: state [C][8], F and marks per (proxy, octant), per-probe
  // dynamic ray counts and offsets (after the 2S sample rays)
  float* dyn_state;
  float* dyn_F;               // [Pp*8]
  uint8_t* dyn_mark;          // [Pp*8]
  uint32_t* dyn_n;            // [P]
  uint32_t* dyn_off;          // [P+1]
  const DynTables* dyn_tab;
  uint8_t* dbg_dyn_accept;    // [C][steps] (debug)
  int32_t pdx, pdy, pdz;      // proxy grid
  uint8_t* dbg_accept;        // [C][steps] (debug)
  const float* pk_dec;        // packed storage: decoded value of every code
  const uint32_t* pk_up;      // packed storage: bit k set if pk_dec[k] >= the exact value
                              // [irr 9-bit 512 | irr 8-bit 256 | tau 8192 | tau^2 8192]
  // trace / blend
  float4* rec;                // [max_rays] radiance RGB, t
  float4* pilot_rec;          // [8P] pilot radiance RGB, t (pilot reuse frames)
  uint32_t* pilot_bins;       // [8P] pilot irradiance texel | depth texel << 16
  int32_t* dbg_ptri;          // [8P] pilot closest triangle (debug)
  uint8_t* dbg_pshadow;       // [8P] pilot shadow bits (debug)
  uint32_t* batch_probe;      // [max_rays / 64] budgeted frames: the probe of ray 64 b
  uint64_t* lam_sums;         // [kAllocPasses][kAllocCandidates] candidate sums, kLamLine apart
  uint32_t* ray_bins;         // [max_rays] probe rays: interior irradiance texel
                              // | interior depth texel << 16 of the direction
  // lit hits waiting for their shadow rays (the pilot and probe passes of a
  // frame use them one after the other), by ray index: hit point and t, unit
  // normal and original triangle index, and a word (pending shadow rays << 8
  // | visible lights); per batch of 64 rays, its (lane | light << 6) pairs,
  // light-major, their number, and its offset in the frame's pair list
  float4* hit_pos;            // [hit_cap]
  float4* hit_nrm;            // [hit_cap]
  uint32_t* hit_vis;          // [hit_cap]
  uint32_t* hit_dst;          // [hit_cap] probe rays: index of the ray a slot traces
  // coherent order of a probe's rays (null: natural order): slot k of a probe
  // with n <= ray_perm_max rays traces ray ray_perm[n (n - 1) / 2 + k]
  const uint16_t* ray_perm;
  int32_t ray_perm_max;
  uint16_t* pairs;            // [ceil(hit_cap/64)][kPairsPerBatch]
  uint32_t* pair_cnt;         // [ceil(hit_cap/64)]
  uint32_t* pair_off;         // [ceil(hit_cap/64) + 1] exclusive scan of pair_cnt
  uint32_t* pair_blk;         // [ceil(hit_cap/64)/kPairScanPer + 1] scan block totals
  uint32_t hit_cap;           // max(max_rays, 8 P)
  uint32_t batch_rays;        // rays per wave batch of a trace pass: 64, or 32 .. 1 for small pilot passes
  int32_t* dbg_tri;           // [max_rays] or null
  uint8_t* dbg_shadow;
  uint16_t* dbg_ibin;
  uint16_t* dbg_dbin;
  uint32_t max_rays;
};

}  // namespace adgi
