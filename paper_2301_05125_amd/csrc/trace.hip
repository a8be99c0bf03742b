// trace.hip - probe-ray and pilot-ray traversal, direct light and shadow rays.
//
// One kernel template serves both ray sources:
//   KIND_PRIMARY: ray r of probe i is the j-th point of a rotated spherical
//     Fibonacci set of n_i directions (r = offsets[i] + j); output one 16-byte
//     record (radiance RGB, hit distance) per ray.
//   KIND_CHAIN:   rays 2k and 2k+1 belong to chain sample k (probes' samples
//     grouped by probe): along d(uv_k) from the sample's probe, shaded, and
//     along -d, distance only (the visibility ray of Sec. 4.8); with dynamic
//     chains, a probe with a dynamic component (score > 0) traces them
//     through the centres of the irradiance texel of d and the depth texel
//     of -d, and rays 2S + dyn_off[i] + j are probe i's dynamic rays: for
//     each marked octant of its proxy, ascending, a shaded ray through the
//     centre of each irradiance texel of the octant, then a distance-only
//     ray through the centre of each depth texel of the octant (Sec. 4.9);
//   KIND_PILOT:   ray r = 8i + k is the pilot of octant k (Sec. 4.1, 4.4);
//     output the 10-bit codes of f_v = exp(-2t/s) (eq. ProbeVis) and
//     f_r = min(lum, beta)/beta (Sec. 4.1.3).
// Rays are handed out 64 at a time to waves from a global counter (persistent
// work-stealing launch) or one per thread (plain launch). Traversal is a
// while-while loop over the BVH2 or its 4-wide collapse, with a short per-lane
// stack in LDS (deeper entries in private memory); a few very large triangles
// sit outside the tree and every ray tests them first. Shadow rays of a
// wave's front-face hits are compacted with ballot/prefix into a wave-local
// LDS queue and traced by all 64 lanes together.
#include "adgi_internal.hpp"

namespace adgi {

enum { KIND_PRIMARY = 0, KIND_PILOT = 1, KIND_CHAIN = 2 };

// Per-lane traversal stack of (node, entry distance of its box): the first
// kStackLds entries in the wave's LDS region (entry k of lane l at 8-byte
// word 64k + l, so a wave's pushes at one depth hit consecutive words), deeper
// entries in private memory. The LDS pointer is typed as LDS so the compiler
// emits ds_ instructions rather than generic (flat) accesses. A closest-hit
// traversal drops popped entries whose box starts beyond the current best
// hit: the box test would reject them (and their children, whose boxes lie
// inside theirs) with the same comparison.
typedef __attribute__((address_space(3))) uint64_t lds_u64;

struct Stack {
  lds_u64* lds;   // this lane's entry 0; an entry is (t bits << 32) | node
  int sp;
  uint64_t deep[kStackMax - kStackLds];
  __device__ __forceinline__ void push(int node, float t) {
    const uint64_t e = ((uint64_t)__float_as_uint(t) << 32) | (uint32_t)node;
    if (sp < kStackLds) {
      lds[sp << 6] = e;
    } else {
      deep[sp - kStackLds] = e;
    }
    ++sp;
  }
  __device__ __forceinline__ uint64_t pop() {
    --sp;
    uint64_t e;
    if (sp < kStackLds) {
      e = lds[sp << 6];
    } else {
      e = deep[sp - kStackLds];
    }
    return e;
  }
  __device__ __forceinline__ int pop_node() { return (int)(uint32_t)pop(); }
  // Next entry whose box may hold a hit at t <= tmax; false when none is left.
  __device__ __forceinline__ bool pop_live(float tmax, int& node) {
    while (sp > 0) {
      const uint64_t e = pop();
      if (__uint_as_float((uint32_t)(e >> 32)) <= tmax) {
        node = (int)(uint32_t)e;
        return true;
      }
    }
    return false;
  }
};

struct NodeData {
  float4 a, b, c;
  int left, right;
};

__device__ __forceinline__ NodeData fetch_node(const float4* __restrict__ nodes, int idx) {
  NodeData n;
  const float4* src = nodes + 4 * (size_t)idx;
  n.a = src[0];
  n.b = src[1];
  n.c = src[2];
  float4 d = src[3];
  n.left = __float_as_int(d.x);
  n.right = __float_as_int(d.y);
  return n;
}

// Work counters of the counting variant (node visits = box-pair tests).
struct Work {
  uint32_t nodes = 0, tris = 0;
};

// The large triangles kept outside the tree (slots [0, num_big)): closest
// hit over them, or whether any of them blocks (0, tmax].
__device__ __forceinline__ void closest_big(const VolumeView& v, const Ray& ray, float& t_best, int& id_best,
                                            int& slot_best, bool& front_best) {
  const int nb = v.scene->num_big;
  for (int k = 0; k < nb; ++k) {
    const float4* tp = v.tris + 3 * (size_t)k;
    float4 a = tp[0], b = tp[1], c = tp[2];
    float t;
    bool fr;
    if (tri_hit(ray, a, b, c, 0.0f, t_best, t, fr)) {
      int id = __float_as_int(a.w);
      if (t < t_best || id < id_best) {
        t_best = t;
        id_best = id;
        slot_best = k;
        front_best = fr;
      }
    }
  }
}

__device__ __forceinline__ bool any_big(const VolumeView& v, const Ray& ray, float tmax) {
  const int nb = v.scene->num_big;
  for (int k = 0; k < nb; ++k) {
    const float4* tp = v.tris + 3 * (size_t)k;
    float t;
    bool fr;
    if (tri_hit(ray, tp[0], tp[1], tp[2], 0.0f, tmax, t, fr)) return true;
  }
  return false;
}

// Closest hit: smallest t in (0, inf); equal t resolves to the lowest
// original triangle index. Returns the triangle slot or -1.
template <bool COUNT>
__device__ int closest_hit(const VolumeView& v, const Ray& ray,
                           Stack& st, float& t_best, bool& front_best, int& id_best, Work& w) {
  t_best = INFINITY;
  id_best = 0x7fffffff;
  int slot_best = -1;
  front_best = false;
  closest_big(v, ray, t_best, id_best, slot_best, front_best);
  if (COUNT) w.tris += v.scene->num_big;
  st.sp = 0;
  int node = 0;
  for (;;) {
    while (node >= 0) {
      NodeData nd = fetch_node(v.nodes, node);
      if (COUNT) ++w.nodes;
      float tl, tr;
      bool hl = box_hit(ray, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, 0.0f, t_best, tl);
      bool hr = box_hit(ray, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, 0.0f, t_best, tr);
      if (hl && hr) {
        bool lf = tl <= tr;
        st.push(lf ? nd.right : nd.left, lf ? tr : tl);
        node = lf ? nd.left : nd.right;
      } else if (hl) {
        node = nd.left;
      } else if (hr) {
        node = nd.right;
      } else {
        if (!st.pop_live(t_best, node)) return slot_best;
      }
    }
    int code = ~node;
    int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
    if (COUNT) w.tris += count;
    for (int k = 0; k < count; ++k) {
      const float4* tp = v.tris + 3 * (size_t)(first + k);
      float4 a = tp[0], b = tp[1], c = tp[2];
      float t;
      bool fr;
      if (tri_hit(ray, a, b, c, 0.0f, t_best, t, fr)) {
        int id = __float_as_int(a.w);
        if (t < t_best || id < id_best) {
          t_best = t;
          id_best = id;
          slot_best = first + k;
          front_best = fr;
        }
      }
    }
    if (!st.pop_live(t_best, node)) return slot_best;
  }
}

// Any hit on (0, tmax].
template <bool COUNT>
__device__ bool any_hit(const VolumeView& v, const Ray& ray,
                        float tmax, Stack& st, Work& w) {
  if (COUNT) w.tris += v.scene->num_big;
  if (any_big(v, ray, tmax)) return true;
  st.sp = 0;
  int node = 0;
  for (;;) {
    while (node >= 0) {
      NodeData nd = fetch_node(v.nodes, node);
      if (COUNT) ++w.nodes;
      float tl, tr;
      bool hl = box_hit(ray, nd.a.x, nd.a.y, nd.a.z, nd.a.w, nd.b.x, nd.b.y, 0.0f, tmax, tl);
      bool hr = box_hit(ray, nd.b.z, nd.b.w, nd.c.x, nd.c.y, nd.c.z, nd.c.w, 0.0f, tmax, tr);
      if (hl && hr) {
        bool lf = tl <= tr;
        st.push(lf ? nd.right : nd.left, lf ? tr : tl);
        node = lf ? nd.left : nd.right;
      } else if (hl) {
        node = nd.left;
      } else if (hr) {
        node = nd.right;
      } else {
        if (st.sp == 0) return false;
        node = st.pop_node();
      }
    }
    int code = ~node;
    int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
    for (int k = 0; k < count; ++k) {
      const float4* tp = v.tris + 3 * (size_t)(first + k);
      float t;
      bool fr;
      if (COUNT) ++w.tris;
      if (tri_hit(ray, tp[0], tp[1], tp[2], 0.0f, tmax, t, fr)) return true;
    }
    if (st.sp == 0) return false;
    node = st.pop_node();
  }
}

// ---- BVH4 traversal
// Tests the four child boxes of node `idx` on (0, lim]. Returns the number of
// boxes hit; the nearest child goes to `next`, the others are pushed farthest
// first (so they pop nearest first). Empty slots never count as hits.
__device__ __forceinline__ void order2(float& ka, int& ca, float& kb, int& cb) {
  const bool sw = kb < ka;
  const float k = sw ? kb : ka;
  const int c = sw ? cb : ca;
  kb = sw ? ka : kb;
  cb = sw ? ca : cb;
  ka = k;
  ca = c;
}

__device__ __forceinline__ int node4_step(const float4* __restrict__ nodes4, int idx, const Ray& ray,
                                          float lim, Stack& st, int& next) {
  const float4* src = nodes4 + 8 * (size_t)idx;
  const float4 lx = src[0], ly = src[1], lz = src[2], hx = src[3], hy = src[4], hz = src[5], cf = src[6];
  int c0 = __float_as_int(cf.x), c1 = __float_as_int(cf.y), c2 = __float_as_int(cf.z),
      c3 = __float_as_int(cf.w);
  float t0, t1, t2, t3;
  const bool h0 = box_hit(ray, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, 0.0f, lim, t0) && c0 != kEmptyChild;
  const bool h1 = box_hit(ray, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, 0.0f, lim, t1) && c1 != kEmptyChild;
  const bool h2 = box_hit(ray, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, 0.0f, lim, t2) && c2 != kEmptyChild;
  const bool h3 = box_hit(ray, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, 0.0f, lim, t3) && c3 != kEmptyChild;
  // hits sort before misses: finite keys for hits, +inf for misses
  float k0 = h0 ? fminf(t0, 3.0e38f) : INFINITY, k1 = h1 ? fminf(t1, 3.0e38f) : INFINITY;
  float k2 = h2 ? fminf(t2, 3.0e38f) : INFINITY, k3 = h3 ? fminf(t3, 3.0e38f) : INFINITY;
  order2(k0, c0, k1, c1);
  order2(k2, c2, k3, c3);
  order2(k0, c0, k2, c2);
  order2(k1, c1, k3, c3);
  order2(k1, c1, k2, c2);
  const int nh = (int)h0 + (int)h1 + (int)h2 + (int)h3;
  if (nh >= 4) st.push(c3, k3);
  if (nh >= 3) st.push(c2, k2);
  if (nh >= 2) st.push(c1, k1);
  next = c0;
  return nh;
}

template <bool COUNT>
__device__ int closest_hit4(const VolumeView& v, const Ray& ray, Stack& st, float& t_best, bool& front_best,
                            int& id_best, Work& w) {
  t_best = INFINITY;
  id_best = 0x7fffffff;
  int slot_best = -1;
  front_best = false;
  closest_big(v, ray, t_best, id_best, slot_best, front_best);
  if (COUNT) w.tris += v.scene->num_big;
  st.sp = 0;
  int node = 0;
  for (;;) {
    while (node >= 0) {
      if (COUNT) ++w.nodes;
      int next;
      if (node4_step(v.nodes4, node, ray, t_best, st, next) > 0) {
        node = next;
      } else {
        if (!st.pop_live(t_best, node)) return slot_best;
      }
    }
    int code = ~node;
    int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
    if (COUNT) w.tris += count;
    for (int k = 0; k < count; ++k) {
      const float4* tp = v.tris + 3 * (size_t)(first + k);
      float4 a = tp[0], b = tp[1], c = tp[2];
      float t;
      bool fr;
      if (tri_hit(ray, a, b, c, 0.0f, t_best, t, fr)) {
        int id = __float_as_int(a.w);
        if (t < t_best || id < id_best) {
          t_best = t;
          id_best = id;
          slot_best = first + k;
          front_best = fr;
        }
      }
    }
    if (!st.pop_live(t_best, node)) return slot_best;
  }
}

template <bool COUNT>
__device__ bool any_hit4(const VolumeView& v, const Ray& ray, float tmax, Stack& st, Work& w) {
  if (COUNT) w.tris += v.scene->num_big;
  if (any_big(v, ray, tmax)) return true;
  st.sp = 0;
  int node = 0;
  for (;;) {
    while (node >= 0) {
      if (COUNT) ++w.nodes;
      int next;
      if (node4_step(v.nodes4, node, ray, tmax, st, next) > 0) {
        node = next;
      } else {
        if (st.sp == 0) return false;
        node = st.pop_node();
      }
    }
    int code = ~node;
    int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
    for (int k = 0; k < count; ++k) {
      const float4* tp = v.tris + 3 * (size_t)(first + k);
      float t;
      bool fr;
      if (COUNT) ++w.tris;
      if (tri_hit(ray, tp[0], tp[1], tp[2], 0.0f, tmax, t, fr)) return true;
    }
    if (st.sp == 0) return false;
    node = st.pop_node();
  }
}

// First probe i with offsets[i+1] > r (offsets ascending, offsets[0] = 0).
__device__ __forceinline__ int probe_of_ray(const uint32_t* __restrict__ off, int P, uint32_t r) {
  int lo = 0, hi = P - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ float3 probe_position(const VolumeView& v, int i) {
  int x = i % v.dx, y = (i / v.dx) % v.dy, z = i / (v.dx * v.dy);
  return make_float3(fmaf((float)x, v.sx, v.ox), fmaf((float)y, v.sy, v.oy),
                     fmaf((float)z, v.sz, v.oz));
}

template <int KIND, bool COUNT, bool W4>
__device__ void trace_wave(const VolumeView& v, Stack& st,
                           uint16_t* queue, uint32_t* vis, uint32_t base, uint32_t total) {
  const FrameParams& fp = *v.fp;
  const SceneParams& sc = *v.scene;
  const uint32_t lane = lane_id();
  const uint32_t r = base + lane;
  const bool active = r < total;

  // ---- ray generation
  float3 o = make_float3(0.f, 0.f, 0.f), d = make_float3(0.f, 0.f, 1.f);
  bool shade = true;  // chain frames: false for distance-only rays
  if (active) {
    if (KIND == KIND_PRIMARY) {
      int i = probe_of_ray(v.offsets, v.P, r);
      uint32_t b = v.offsets[i], n = v.offsets[i + 1] - b;
      o = probe_position(v, i);
      d = sf_direction(r - b, n, fp.R);
    } else if (KIND == KIND_CHAIN) {
      const uint32_t S2 = 2u * v.offsets[v.P];
      if (r < S2) {
        const uint32_t k = r >> 1;
        const int i = (int)v.smp_probe[k];
        o = probe_position(v, i);
        d = oct_decode_dir(v.smp_uv[k]);
        if (r & 1u) d = make_float3(-d.x, -d.y, -d.z);
        if (fp.dyn_chains > 0 && v.score[i] > 0) {  // through the texel centre
          const int R = (r & 1u) ? v.dep_res - 2 : v.irr_res - 2;
          d = texel_centre_dir(oct_bin(oct_encode(d), R), R);
        }
        shade = !(r & 1u);
      } else {
        const uint32_t rr = r - S2;
        const int i = probe_of_ray(v.dyn_off, v.P, rr);
        uint32_t j = rr - v.dyn_off[i];
        o = probe_position(v, i);
        const int x = i % v.dx, y = (i / v.dx) % v.dy, z = i / (v.dx * v.dy);
        const uint8_t* mk = v.dyn_mark + 8 * (x / 3 + v.pdx * (y / 3 + v.pdy * (z / 3)));
        const DynTables& tb = *v.dyn_tab;
        for (int oc = 0; oc < 8; ++oc) {
          if (!mk[oc]) continue;
          const uint32_t ni = tb.start_i[oc + 1] - tb.start_i[oc], nd = tb.start_d[oc + 1] - tb.start_d[oc];
          if (j < ni) {
            d = texel_centre_dir(tb.ord_i[tb.start_i[oc] + j], v.irr_res - 2);
            shade = true;
            break;
          }
          j -= ni;
          if (j < nd) {
            d = texel_centre_dir(tb.ord_d[tb.start_d[oc] + j], v.dep_res - 2);
            shade = false;
            break;
          }
          j -= nd;
        }
      }
    } else {
      uint32_t i = r >> 3, k = r & 7;
      o = probe_position(v, (int)i);
      d = pilot_direction(fp.seed, i, k, (uint32_t)fp.frame >> 1);
    }
  }

  // ---- closest hit
  float t = INFINITY;
  bool front = false;
  int id = -1, slot = -1;
  Work w;
  if (active && sc.num_tris > 0) {
    Ray ray = make_ray(o, d);
    slot = W4 ? closest_hit4<COUNT>(v, ray, st, t, front, id, w)
              : closest_hit<COUNT>(v, ray, st, t, front, id, w);
    if (slot < 0) {
      id = -1;
      t = INFINITY;
    }
  }

  // ---- direct light at front-face hits, shadow rays compacted per wave
  const bool lit_hit = active && slot >= 0 && front && (KIND != KIND_CHAIN || shade);
  float3 x = make_float3(0.f, 0.f, 0.f), nrm = make_float3(0.f, 0.f, 0.f);
  if (lit_hit) {
    const float4* tp = v.tris + 3 * (size_t)slot;
    float4 b = tp[1], c = tp[2];
    float nx = b.y * c.z - b.z * c.y, ny = b.z * c.x - b.x * c.z, nz = b.x * c.y - b.y * c.x;
    float inv = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
    nrm = make_float3(nx * inv, ny * inv, nz * inv);
    x = make_float3(fmaf(t, d.x, o.x), fmaf(t, d.y, o.y), fmaf(t, d.z, o.z));
  }
  const int nl = sc.num_lights;
  uint32_t qtotal = 0;
  for (int l = 0; l < nl; ++l) {
    bool need = false;
    if (lit_hit) {
      float lx = sc.lpos[l][0] - x.x, ly = sc.lpos[l][1] - x.y, lz = sc.lpos[l][2] - x.z;
      need = nrm.x * lx + nrm.y * ly + nrm.z * lz > 0.0f;
    }
    uint64_t mask = ballot(need);
    if (need) queue[qtotal + lanes_below(mask)] = (uint16_t)(lane | (l << 6));
    qtotal += (uint32_t)__popcll(mask);
  }
  vis[lane] = 0u;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const float off_len = kShadowOffset * v.s_diag;
  for (uint32_t qb = 0; qb < qtotal; qb += 64) {
    uint32_t q = qb + lane;
    bool has = q < qtotal;
    uint32_t e = has ? queue[q] : 0u;
    int src = (int)(e & 63u), l = (int)(e >> 6);
    float sx = __shfl(x.x, src), sy = __shfl(x.y, src), sz = __shfl(x.z, src);
    float mx = __shfl(nrm.x, src), my = __shfl(nrm.y, src), mz = __shfl(nrm.z, src);
    if (has) {
      float3 so = make_float3(fmaf(off_len, mx, sx), fmaf(off_len, my, sy), fmaf(off_len, mz, sz));
      float gx = sc.lpos[l][0] - so.x, gy = sc.lpos[l][1] - so.y, gz = sc.lpos[l][2] - so.z;
      float len = sqrtf(gx * gx + gy * gy + gz * gz);
      float il = 1.0f / len;
      Ray sray = make_ray(so, make_float3(gx * il, gy * il, gz * il));
      const float smax = len * (1.0f - kShadowShorten);
      bool blocked = W4 ? any_hit4<COUNT>(v, sray, smax, st, w) : any_hit<COUNT>(v, sray, smax, st, w);
      if (!blocked) atomicOr(&vis[src], 1u << l);
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t bits = vis[lane];
  if (COUNT) {
    uint32_t n = w.nodes, tt = w.tris;
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
      n += __shfl_xor(n, o2);
      tt += __shfl_xor(tt, o2);
    }
    if (lane == 0) {
      atomicAdd((unsigned long long*)&v.stats->node_tests, (unsigned long long)n);
      atomicAdd((unsigned long long*)&v.stats->tri_tests, (unsigned long long)tt);
    }
  }
  if (lane == 0 && qtotal > 0) atomicAdd((unsigned long long*)&v.stats->shadow_rays, (unsigned long long)qtotal);

  float3 L = make_float3(0.f, 0.f, 0.f);
  if (active && slot < 0) {
    L = make_float3(sc.sky[0], sc.sky[1], sc.sky[2]);
  } else if (lit_hit) {
    float er = 0.f, eg = 0.f, eb = 0.f;
    for (int l = 0; l < nl; ++l) {
      if (!((bits >> l) & 1u)) continue;
      float lx = sc.lpos[l][0] - x.x, ly = sc.lpos[l][1] - x.y, lz = sc.lpos[l][2] - x.z;
      float d2 = lx * lx + ly * ly + lz * lz;
      float cs = (nrm.x * lx + nrm.y * ly + nrm.z * lz) / sqrtf(d2);
      float w = fmaxf(cs, 0.0f) / d2;
      er = fmaf(sc.lint[l][0], w, er);
      eg = fmaf(sc.lint[l][1], w, eg);
      eb = fmaf(sc.lint[l][2], w, eb);
    }
    float4 rho = v.albedo[id];
    const float inv_pi = 0.318309886183790671538f;
    L = make_float3(rho.x * inv_pi * er, rho.y * inv_pi * eg, rho.z * inv_pi * eb);
  }

  // ---- outputs
  if (!active) return;
  if (KIND != KIND_PILOT) {
    v.rec[r] = make_float4(L.x, L.y, L.z, t);
    if (fp.debug) {
      v.dbg_tri[r] = id;
      v.dbg_shadow[r] = (uint8_t)bits;
    }
  } else {
    int qv = 0;
    if (t < INFINITY) qv = min(1023, (int)floorf(1024.0f * expf(-2.0f * t / v.s_diag)));
    float lum = 0.2126f * L.x + 0.7152f * L.y + 0.0722f * L.z;
    int qr = min(1023, (int)floorf(1024.0f * (fminf(lum, fp.beta) / fp.beta)));
    int slot_q = fp.frame & 1;
    v.qv[slot_q][r] = (uint16_t)qv;
    v.qr[slot_q][r] = (uint16_t)max(qr, 0);
  }
}

// Eight waves per SIMD (64 VGPRs): traversal is bound by memory latency, so
// occupancy pays for the few registers the compiler then keeps in scratch.
template <int KIND, bool COUNT, bool W4>
__global__ __attribute__((amdgpu_waves_per_eu(8, 8))) void trace_kernel(VolumeView v, int persistent) {
  extern __shared__ uint64_t smem[];
  uint64_t* stack_base = (uint64_t*)smem;                         // kStackLds * blockDim
  uint16_t* queues = (uint16_t*)(stack_base + kStackLds * blockDim.x);  // waves * 64 * kMaxLights
  const int nwaves = blockDim.x >> 6;
  uint32_t* vis_all = (uint32_t*)(queues + nwaves * 64 * kMaxLights);   // waves * 64
  const int wave = threadIdx.x >> 6;
  Stack st;
  st.lds = (lds_u64*)stack_base + wave * (64 * kStackLds) + lane_id();
  st.sp = 0;
  uint16_t* queue = queues + wave * 64 * kMaxLights;
  uint32_t* vis = vis_all + wave * 64;
  const uint32_t total = KIND == KIND_PRIMARY ? v.offsets[v.P]
                         : KIND == KIND_CHAIN ? 2u * v.offsets[v.P] + (v.fp->dyn_chains > 0 ? v.dyn_off[v.P] : 0u)
                                              : 8u * (uint32_t)v.P;
  if (persistent) {
    uint32_t* counter = KIND == KIND_PILOT ? &v.stats->pilot_counter : &v.stats->ray_counter;
    for (;;) {
      uint32_t base = 0;
      if (lane_id() == 0) base = atomicAdd(counter, 64u);
      base = __shfl(base, 0);
      if (base >= total) break;
      trace_wave<KIND, COUNT, W4>(v, st, queue, vis, base, total);
    }
  } else {
    uint32_t base = (blockIdx.x * blockDim.x) + (uint32_t)wave * 64u;
    if (base < total) trace_wave<KIND, COUNT, W4>(v, st, queue, vis, base, total);
  }
}

size_t trace_lds_bytes(int block) {
  return (size_t)kStackLds * block * 8 + (size_t)(block / 64) * 64 * kMaxLights * 2 + (size_t)(block / 64) * 64 * 4;
}

template <bool W4>
static void launch_trace_w(const VolumeView& v, hipStream_t s, bool pilot, int pers, int block, int grid,
                           bool count, bool chain) {
  const size_t lds = trace_lds_bytes(block);
  if (chain && count)
    hipLaunchKernelGGL((trace_kernel<KIND_CHAIN, true, W4>), dim3(grid), dim3(block), lds, s, v, pers);
  else if (chain)
    hipLaunchKernelGGL((trace_kernel<KIND_CHAIN, false, W4>), dim3(grid), dim3(block), lds, s, v, pers);
  else if (pilot && count)
    hipLaunchKernelGGL((trace_kernel<KIND_PILOT, true, W4>), dim3(grid), dim3(block), lds, s, v, pers);
  else if (pilot)
    hipLaunchKernelGGL((trace_kernel<KIND_PILOT, false, W4>), dim3(grid), dim3(block), lds, s, v, pers);
  else if (count)
    hipLaunchKernelGGL((trace_kernel<KIND_PRIMARY, true, W4>), dim3(grid), dim3(block), lds, s, v, pers);
  else
    hipLaunchKernelGGL((trace_kernel<KIND_PRIMARY, false, W4>), dim3(grid), dim3(block), lds, s, v, pers);
}

hipError_t launch_trace(const VolumeView& v, hipStream_t s, bool pilot, bool persistent, int block, int grid,
                        bool count, bool w4, bool chain) {
  if (w4)
    launch_trace_w<true>(v, s, pilot, persistent ? 1 : 0, block, grid, count, chain);
  else
    launch_trace_w<false>(v, s, pilot, persistent ? 1 : 0, block, grid, count, chain);
  return hipGetLastError();
}

}  // namespace adgi
