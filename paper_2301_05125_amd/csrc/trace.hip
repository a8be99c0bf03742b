// trace.hip - probe-ray and pilot-ray traversal, direct light and shadow rays.
//
// One pair of kernels serves every ray source:
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
// The closest-hit kernel finds every ray's hit and writes the final output
// of misses and unlit hits; a lit front-face hit keeps its hit data at its
// ray index and lists one (ray, light) pair per light on its front side. The
// shading kernel traces those pairs' shadow rays in full 64-lane batches and
// writes the lit rays' output. Work goes to waves by fixed batch index (grid
// stride when persistent): no wave waits on a counter shared by the whole
// grid, which costs more here than the traversal it would balance.
// Traversal is a while-while loop over the BVH2 or its 4-wide collapse, with
// a short per-lane stack in LDS (deeper entries in private memory); a few
// very large triangles sit outside the tree and every ray tests them first.
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

// The deeper entries sit in an array of the kernel's own (private memory)
// and the struct holds a pointer to it, so sp stays in a register: with the
// array as a member the whole struct, sp included, lived in private memory
// and every push stored sp there.
struct Stack {
  lds_u64* lds;   // this lane's entry 0; an entry is (t bits << 32) | node
  int sp;
  uint64_t* deep;
  static __device__ __forceinline__ uint64_t entry(int node, float t) {
    return ((uint64_t)__float_as_uint(t) << 32) | (uint32_t)node;
  }
  __device__ __forceinline__ void push(int node, float t) { push_entry(entry(node, t)); }
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
  // The hit children after the nearest of a 4-wide visit, sorted near to far
  // (e1 <= e2 <= e3 by distance), nh hits in all (2..4): pushed farthest
  // first, so they pop nearest first. While three more entries fit in LDS,
  // the three slots above sp are written whatever nh is (a slot above the new
  // top holds nothing live), with no branch per entry.
  __device__ __forceinline__ void push_after_nearest(int nh, uint64_t e1, uint64_t e2, uint64_t e3) {
    if (sp + 3 <= kStackLds) {
      lds_u64* p = lds + (sp << 6);
      p[0] = nh >= 4 ? e3 : nh == 3 ? e2 : e1;
      p[64] = nh >= 4 ? e2 : e1;
      p[128] = e1;
      sp += nh - 1;
    } else {
      if (nh >= 4) push_entry(e3);
      if (nh >= 3) push_entry(e2);
      push_entry(e1);
    }
  }
  __device__ __forceinline__ void push_entry(uint64_t e) {
    if (sp < kStackLds) {
      lds[sp << 6] = e;
    } else {
      deep[sp - kStackLds] = e;
    }
    ++sp;
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
  uint32_t boxes = 0;  // child boxes tested: two per BVH2 visit, the non-empty slots of a BVH4 visit
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
      if (COUNT) {
        ++w.nodes;
        w.boxes += 2u;
      }
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

// Any hit on (0, tmax]: a while-while traversal with wave-wide loop exits
// (the node phase runs until no lane needs another node, then the lanes
// holding a leaf test its triangles).
template <bool COUNT>
__device__ bool any_hit(const VolumeView& v, const Ray& ray,
                        float tmax, Stack& st, Work& w) {
  if (COUNT) w.tris += v.scene->num_big;
  const bool big = any_big(v, ray, tmax);
  st.sp = 0;
  int node = 0;
  bool more = !big, hit = big;
  for (;;) {
    for (;;) {
      if (more && node >= 0) {
        NodeData nd = fetch_node(v.nodes, node);
        if (COUNT) {
          ++w.nodes;
          w.boxes += 2u;
        }
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
          more = st.sp > 0;
          if (more) node = st.pop_node();
        }
      }
      if (ballot(more && node >= 0) == 0ull) break;
    }
    if (more) {
      const int code = ~node;
      const int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
      for (int k = 0; k < count && !hit; ++k) {
        const float4* tp = v.tris + 3 * (size_t)(first + k);
        float t;
        bool fr;
        if (COUNT) ++w.tris;
        hit = tri_hit(ray, tp[0], tp[1], tp[2], 0.0f, tmax, t, fr);
      }
      more = !hit && st.sp > 0;
      if (more) node = st.pop_node();
    }
    if (ballot(more) == 0ull) break;
  }
  return hit;
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

template <bool COUNT>
__device__ __forceinline__ int node4_step(const float4* __restrict__ nodes4, int idx, const Ray& ray,
                                          float lim, Stack& st, int& next, Work& w) {
  const float4* src = nodes4 + 8 * (size_t)idx;
  const float4 lx = src[0], ly = src[1], lz = src[2], hx = src[3], hy = src[4], hz = src[5], cf = src[6];
  int c0 = __float_as_int(cf.x), c1 = __float_as_int(cf.y), c2 = __float_as_int(cf.z),
      c3 = __float_as_int(cf.w);
  if (COUNT) {
    ++w.nodes;
    w.boxes += (uint32_t)(c0 != kEmptyChild) + (uint32_t)(c1 != kEmptyChild) + (uint32_t)(c2 != kEmptyChild) +
               (uint32_t)(c3 != kEmptyChild);
  }
  float t0, t1, t2, t3;
  const bool h0 = box_hit(ray, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, 0.0f, lim, t0) && c0 != kEmptyChild;
  const bool h1 = box_hit(ray, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, 0.0f, lim, t1) && c1 != kEmptyChild;
  const bool h2 = box_hit(ray, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, 0.0f, lim, t2) && c2 != kEmptyChild;
  const bool h3 = box_hit(ray, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, 0.0f, lim, t3) && c3 != kEmptyChild;
  // hits sort before misses: a hit's entry distance is finite (padded bounds
  // are finite and |1/d| <= 1e20), a miss keys +inf
  float k0 = h0 ? t0 : INFINITY, k1 = h1 ? t1 : INFINITY;
  float k2 = h2 ? t2 : INFINITY, k3 = h3 ? t3 : INFINITY;
  order2(k0, c0, k1, c1);
  order2(k2, c2, k3, c3);
  order2(k0, c0, k2, c2);
  order2(k1, c1, k3, c3);
  order2(k1, c1, k2, c2);
  const int nh = (int)h0 + (int)h1 + (int)h2 + (int)h3;
  if (nh >= 2) st.push_after_nearest(nh, Stack::entry(c1, k1), Stack::entry(c2, k2), Stack::entry(c3, k3));
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
      int next;
      if (node4_step<COUNT>(v.nodes4, node, ray, t_best, st, next, w) > 0) {
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
  const bool big = any_big(v, ray, tmax);
  st.sp = 0;
  // while-while with wave-wide loop exits: the node phase runs until no lane
  // needs another node (each lane then holds a leaf or is done), then the
  // lanes holding a leaf test its triangles
  int node = 0;
  bool more = !big, hit = big;
  for (;;) {
    for (;;) {
      if (more && node >= 0) {
        int next;
        if (node4_step<COUNT>(v.nodes4, node, ray, tmax, st, next, w) > 0) {
          node = next;
        } else {
          more = st.sp > 0;
          if (more) node = st.pop_node();
        }
      }
      if (ballot(more && node >= 0) == 0ull) break;
    }
    if (more) {
      const int code = ~node;
      const int first = code >> kLeafShift, count = (code & (kLeafMaxTris - 1)) + 1;
      for (int k = 0; k < count && !hit; ++k) {
        const float4* tp = v.tris + 3 * (size_t)(first + k);
        float t;
        bool fr;
        if (COUNT) ++w.tris;
        hit = tri_hit(ray, tp[0], tp[1], tp[2], 0.0f, tmax, t, fr);
      }
      more = !hit && st.sp > 0;
      if (more) node = st.pop_node();
    }
    if (ballot(more) == 0ull) break;
  }
  return hit;
}


// First probe i in [lo, hi] with offsets[i+1] > r (offsets ascending,
// offsets[0] = 0; the answer lies in the window).
__device__ __forceinline__ int probe_in(const uint32_t* __restrict__ off, int lo, int hi, uint32_t r) {
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= r) lo = mid;
    else hi = mid - 1;
  }
  return lo;
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

// ---- ray sources
template <int KIND>
__device__ __forceinline__ uint32_t ray_total(const VolumeView& v) {
  return KIND == KIND_PRIMARY ? v.offsets[v.P]
         : KIND == KIND_CHAIN ? 2u * v.offsets[v.P] + (v.fp->dyn_chains > 0 ? v.dyn_off[v.P] : 0u)
                              : 8u * (uint32_t)v.P;
}

// Origin and direction of ray r; `shade` is false for the distance-only rays
// of chain frames. Probe rays: i0 is the probe of a ray at most 63 before r
// (every probe has at least one ray, so r's probe is within i0 + 63).
// dst: where the ray's outputs go (probe rays: the index of the ray that the
// slot traces under the coherent order, else r itself).
template <int KIND>
__device__ __forceinline__ void gen_ray(const VolumeView& v, uint32_t r, int i0, float3& o, float3& d,
                                        bool& shade, uint32_t& dst) {
  const FrameParams& fp = *v.fp;
  shade = true;
  dst = r;
  if (KIND == KIND_PRIMARY) {
    int i = probe_in(v.offsets, i0, min(i0 + 63, v.P - 1), r);
    uint32_t b = v.offsets[i], n = v.offsets[i + 1] - b;
    o = probe_position(v, i);
    uint32_t j = r - b;
    if (v.ray_perm && n <= (uint32_t)v.ray_perm_max) j = v.ray_perm[(size_t)n * (n - 1u) / 2u + j];
    dst = b + j;
    d = sf_direction(sf_point_of_ray(j, n), n, fp.R);
  } else if (KIND == KIND_CHAIN) {
    const uint32_t S2 = 2u * v.offsets[v.P];
    d = make_float3(0.f, 0.f, 1.f);
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

// Final output of ray r: the record (radiance, t) of probe and chain rays, the
// 10-bit codes of f_v = exp(-2t/s) (eq. ProbeVis) and f_r = min(lum, beta)/beta
// (Sec. 4.1.3) of pilots.
template <int KIND>
__device__ __forceinline__ void emit_ray(const VolumeView& v, uint32_t r, float3 L, float t, int id,
                                         uint32_t bits) {
  const FrameParams& fp = *v.fp;
  if (KIND != KIND_PILOT) {
    v.rec[r] = make_float4(L.x, L.y, L.z, t);
    if (fp.debug) {
      v.dbg_tri[r] = id;
      v.dbg_shadow[r] = (uint8_t)bits;
    }
  } else {
    if (fp.pilot_reuse) v.pilot_rec[r] = make_float4(L.x, L.y, L.z, t);
    if (fp.debug) {
      v.dbg_ptri[r] = id;
      v.dbg_pshadow[r] = (uint8_t)bits;
    }
    int qv = 0;
    if (t < INFINITY) qv = min(1023, (int)floorf(1024.0f * expf(-2.0f * t / v.s_diag)));
    float lum = 0.2126f * L.x + 0.7152f * L.y + 0.0722f * L.z;
    int qr = min(1023, (int)floorf(1024.0f * (fminf(lum, fp.beta) / fp.beta)));
    int slot_q = fp.frame & 1;
    v.qv[slot_q][r] = (uint16_t)qv;
    v.qr[slot_q][r] = (uint16_t)max(qr, 0);
  }
}

// Lights on the front side of a hit at x with normal n, one bit each.
__device__ __forceinline__ uint32_t lights_facing(const SceneParams& sc, float3 x, float3 n) {
  uint32_t m = 0u;
  for (int l = 0; l < sc.num_lights; ++l) {
    const float lx = sc.lpos[l][0] - x.x, ly = sc.lpos[l][1] - x.y, lz = sc.lpos[l][2] - x.z;
    if (n.x * lx + n.y * ly + n.z * lz > 0.0f) m |= 1u << l;
  }
  return m;
}

// Adds the work counters of the wave's lanes to the frame statistics (the
// shading kernel's also to its own pair); `shadow`, the wave's shadow pairs,
// is the same in every lane.
template <bool COUNT, bool SHADE>
__device__ __forceinline__ void flush_stats(const VolumeView& v, const Work& w, uint32_t shadow) {
  uint32_t n = COUNT ? w.nodes : 0u, tt = COUNT ? w.tris : 0u, bx = COUNT ? w.boxes : 0u;
  const uint32_t s = shadow;
  if (COUNT) {
    for (int o2 = 32; o2 > 0; o2 >>= 1) {
      n += __shfl_xor(n, o2);
      tt += __shfl_xor(tt, o2);
      bx += __shfl_xor(bx, o2);
    }
  }
  if (lane_id() == 0) {
    if (COUNT) {
      atomicAdd((unsigned long long*)&v.stats->node_tests, (unsigned long long)n);
      atomicAdd((unsigned long long*)&v.stats->tri_tests, (unsigned long long)tt);
      atomicAdd((unsigned long long*)&v.stats->box_tests, (unsigned long long)bx);
      if (SHADE) {
        atomicAdd((unsigned long long*)&v.stats->shade_node_tests, (unsigned long long)n);
        atomicAdd((unsigned long long*)&v.stats->shade_tri_tests, (unsigned long long)tt);
        atomicAdd((unsigned long long*)&v.stats->shade_box_tests, (unsigned long long)bx);
      }
    }
    if (s > 0) atomicAdd((unsigned long long*)&v.stats->shadow_rays, (unsigned long long)s);
  }
}

// One lane's ray of a batch after its closest hit: x and n the hit point and
// unit face normal, need the lights on the front side of a lit hit (0 for a
// miss, a back face, a distance-only ray or a hit no light faces).
struct BatchHit {
  bool active;
  uint32_t dst;
  float3 x, n;
  float t;
  int id, slot;
  uint32_t need;
};

template <int KIND, bool COUNT, bool W4>
__device__ __forceinline__ BatchHit closest_of_batch(const VolumeView& v, Stack& st, uint32_t b, uint32_t total,
                                                     Work& w) {
  const SceneParams& sc = *v.scene;
  const uint32_t lane = lane_id(), br = v.batch_rays;
  const uint32_t r = b * br + lane;
  BatchHit h;
  h.active = lane < br && r < total;
  float3 o = make_float3(0.f, 0.f, 0.f), d = make_float3(0.f, 0.f, 1.f);
  bool shade = true;
  h.dst = r;
  // probe of the batch's first ray (the same in every lane): budgeted frames
  // list it per 64-ray batch with the allocation, uniform ones divide
  int i0 = 0;
  if (KIND == KIND_PRIMARY)
    i0 = v.fp->adaptive ? (int)v.batch_probe[b] : (int)(b * br / (uint32_t)v.fp->n_uniform);
  if (h.active) gen_ray<KIND>(v, r, i0, o, d, shade, h.dst);
  if (KIND == KIND_PILOT && h.active && v.fp->pilot_reuse) {
    const float2 uv = oct_encode(d);
    v.pilot_bins[r] = oct_bin(uv, v.irr_res - 2) | (oct_bin(uv, v.dep_res - 2) << 16);
  }
  if (KIND == KIND_PRIMARY && h.active) {
    // the interior irradiance and depth texels the ray's direction falls in,
    // for the blend (one 4-byte word per ray instead of regenerating the
    // direction there)
    const float2 uv = oct_encode(d);
    const uint32_t bI = oct_bin(uv, v.irr_res - 2), bD = oct_bin(uv, v.dep_res - 2);
    v.ray_bins[h.dst] = bI | (bD << 16);
    if (v.fp->debug) {
      v.dbg_ibin[h.dst] = (uint16_t)bI;
      v.dbg_dbin[h.dst] = (uint16_t)bD;
    }
  }
  h.t = INFINITY;
  bool front = false;
  h.id = -1;
  h.slot = -1;
  if (h.active && sc.num_tris > 0) {
    Ray ray = make_ray(o, d);
    h.slot = W4 ? closest_hit4<COUNT>(v, ray, st, h.t, front, h.id, w)
                : closest_hit<COUNT>(v, ray, st, h.t, front, h.id, w);
    if (h.slot < 0) {
      h.id = -1;
      h.t = INFINITY;
    }
  }
  h.need = 0u;
  h.x = h.n = make_float3(0.f, 0.f, 0.f);
  if (h.active && h.slot >= 0 && front && shade) {
    const float4* tp = v.tris + 3 * (size_t)h.slot;
    const float4 tb = tp[1], tc = tp[2];
    const float nx = tb.y * tc.z - tb.z * tc.y, ny = tb.z * tc.x - tb.x * tc.z, nz = tb.x * tc.y - tb.y * tc.x;
    const float inv = 1.0f / sqrtf(nx * nx + ny * ny + nz * nz);
    h.n = make_float3(nx * inv, ny * inv, nz * inv);
    h.x = make_float3(fmaf(h.t, d.x, o.x), fmaf(h.t, d.y, o.y), fmaf(h.t, d.z, o.z));
    h.need = lights_facing(sc, h.x, h.n);
  }
  return h;
}

// The final output of a ray with no shadow ray to wait for: the sky for a
// miss, black for any hit.
template <int KIND>
__device__ __forceinline__ void emit_unshadowed(const VolumeView& v, const BatchHit& h) {
  const SceneParams& sc = *v.scene;
  const float3 L = h.slot < 0 ? make_float3(sc.sky[0], sc.sky[1], sc.sky[2]) : make_float3(0.f, 0.f, 0.f);
  emit_ray<KIND>(v, h.dst, L, h.t, h.id, 0u);
}

// ---- closest-hit kernel
// A wave owns a batch of consecutive rays (batch b = rays [B b, B b + B),
// B = v.batch_rays = 64; the fused pilot pass below takes fewer when the pass
// is too small to fill the launch's waves); a persistent launch walks the
// batches with a grid stride, so no wave ever waits on a shared counter.
// Every ray finds its closest hit. A miss, a back face, a distance-only ray
// or a lit hit with no light on its front side is final and is written at
// once; a lit hit with lights on its front side keeps its hit point, t,
// normal and triangle at its own index, its pending shadow-ray count in its
// visibility word, and puts one (lane, light) pair per such light into the
// batch's pair segment, all pairs of light 0 first, then light 1, and so on
// (neighbouring shadow rays mostly share a light).
template <int KIND, bool COUNT, bool W4>
__device__ __forceinline__ void hit_batch(const VolumeView& v, Stack& st, uint32_t b, uint32_t total, Work& w,
                                          uint32_t& shadow) {
  const SceneParams& sc = *v.scene;
  const uint32_t lane = lane_id();
  const uint32_t r = b * v.batch_rays + lane;
  const BatchHit h = closest_of_batch<KIND, COUNT, W4>(v, st, b, total, w);
  if (h.need) {
    v.hit_pos[r] = make_float4(h.x.x, h.x.y, h.x.z, h.t);
    v.hit_nrm[r] = make_float4(h.n.x, h.n.y, h.n.z, __int_as_float(h.id));
    v.hit_vis[r] = (uint32_t)__popc(h.need) << 8;
    if (KIND == KIND_PRIMARY) v.hit_dst[r] = h.dst;
  }
  uint16_t* seg = v.pairs + (size_t)b * kPairsPerBatch;
  uint32_t n = 0u;
  for (int l = 0; l < sc.num_lights; ++l) {
    const bool p = (h.need >> l) & 1u;
    const uint64_t m = ballot(p);
    if (p) seg[n + lanes_below(m)] = (uint16_t)(lane | ((uint32_t)l << 6));
    n += (uint32_t)__popcll(m);
  }
  if (lane == 0) v.pair_cnt[b] = n;
  shadow += n;
  if (h.active && !h.need) {
    emit_unshadowed<KIND>(v, h);
  } else if (h.active && v.fp->debug) {
    if (KIND == KIND_PILOT) v.dbg_ptri[h.dst] = h.id;
    else v.dbg_tri[h.dst] = h.id;
  }
}

template <int KIND, bool COUNT, bool W4>
__global__ __attribute__((amdgpu_waves_per_eu(8, 8))) void trace_hit_kernel(VolumeView v, int persistent) {
  extern __shared__ uint64_t smem[];
  const int wave = threadIdx.x >> 6;
  uint64_t deep[kStackMax - kStackLds];
  Stack st;
  st.lds = (lds_u64*)smem + wave * (64 * kStackLds) + lane_id();
  st.sp = 0;
  st.deep = deep;
  const uint32_t total = ray_total<KIND>(v);
  const uint32_t nbatch = (total + v.batch_rays - 1u) / v.batch_rays;
  const uint32_t waves = blockDim.x >> 6;
  const uint32_t first = blockIdx.x * waves + (uint32_t)wave;
  const uint32_t stride = persistent ? gridDim.x * waves : nbatch;
  if (first == 0 && lane_id() == 0) v.stats->pair_batches = nbatch;
  Work w;
  uint32_t shadow = 0u;
  for (uint32_t b = first; b < nbatch; b += stride) hit_batch<KIND, COUNT, W4>(v, st, b, total, w, shadow);
  flush_stats<COUNT, false>(v, w, shadow);
}

// ---- exclusive scan of the batches' pair counts -> pair_off[0..nbatch]
// Three launches over the buffer's batch capacity (counts past the frame's
// batches read as zero): a block-local scan of kScanPer batches per block
// with the block totals, a scan of the block totals (one block), and the
// block offsets added in.
constexpr int kScanThreads = 256, kScanItems = kPairScanPer / kScanThreads, kScanPer = kPairScanPer;

__device__ __forceinline__ uint32_t block_scan_u32(uint32_t x, uint32_t* sm, uint32_t& total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  uint32_t s = x;
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(s, (unsigned)off);
    if (lane >= off) s += y;
  }
  if (lane == 63) sm[wave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0u;
    for (int k = 0; k < nw; ++k) {
      const uint32_t tk = sm[k];
      sm[k] = acc;
      acc += tk;
    }
    sm[nw] = acc;
  }
  __syncthreads();
  total = sm[nw];
  const uint32_t out = s - x + sm[wave];
  __syncthreads();
  return out;
}

__global__ __launch_bounds__(kScanThreads) void pair_scan_local_kernel(VolumeView v) {
  __shared__ uint32_t sm[kScanThreads / 64 + 1];
  const uint32_t nb = v.stats->pair_batches;
  const uint32_t b0 = blockIdx.x * (uint32_t)kScanPer + threadIdx.x * (uint32_t)kScanItems;
  uint32_t c[kScanItems], sum = 0u;
  for (int k = 0; k < kScanItems; ++k) {
    c[k] = b0 + k < nb ? v.pair_cnt[b0 + k] : 0u;
    sum += c[k];
  }
  uint32_t total;
  uint32_t acc = block_scan_u32(sum, sm, total);
  for (int k = 0; k < kScanItems; ++k) {
    if (b0 + k <= nb) v.pair_off[b0 + k] = acc;
    acc += c[k];
  }
  if (threadIdx.x == 0) v.pair_blk[blockIdx.x] = total;
}

__global__ __launch_bounds__(1024) void pair_scan_blocks_kernel(VolumeView v) {
  __shared__ uint32_t sm[1024 / 64 + 1];
  const uint32_t nblk = v.stats->pair_batches / (uint32_t)kScanPer + 1u;
  uint32_t carry = 0u;
  for (uint32_t base = 0; base < nblk; base += 1024u) {
    const uint32_t k = base + threadIdx.x;
    const uint32_t x = k < nblk ? v.pair_blk[k] : 0u;
    uint32_t total;
    const uint32_t e = block_scan_u32(x, sm, total);
    if (k < nblk) v.pair_blk[k] = carry + e;
    carry += total;
  }
  if (threadIdx.x == 0) v.stats->pair_total = carry;
}

__global__ __launch_bounds__(kScanThreads) void pair_scan_add_kernel(VolumeView v) {
  const uint32_t nb = v.stats->pair_batches;
  const uint32_t b = blockIdx.x * kScanThreads + threadIdx.x;
  if (b <= nb) v.pair_off[b] += v.pair_blk[b / (uint32_t)kScanPer];
}

// The same scan in one workgroup (used while the buffers hold at most
// kScanSingleMax batches): thread k scans a contiguous chunk of the counts.
// At 2^17 batches it took 0.2 ms more than the three launches (each thread
// walks 128 counts twice), so it serves small volumes only.
constexpr uint32_t kScanSingleMax = 1024u * 16u;

__global__ __launch_bounds__(1024) void pair_scan_single_kernel(VolumeView v) {
  __shared__ uint32_t sm[1024 / 64 + 1];
  const uint32_t nb = v.stats->pair_batches;
  const uint32_t chunk = (nb + 1023u) / 1024u;
  const uint32_t b0 = threadIdx.x * chunk, b1 = min(b0 + chunk, nb);
  uint32_t sum = 0u;
  for (uint32_t b = b0; b < b1; ++b) sum += v.pair_cnt[b];
  uint32_t total;
  uint32_t acc = block_scan_u32(sum, sm, total);
  for (uint32_t b = b0; b < b1; ++b) {
    const uint32_t c = v.pair_cnt[b];
    v.pair_off[b] = acc;
    acc += c;
  }
  if (threadIdx.x == 0) {
    v.pair_off[nb] = total;
    v.stats->pair_total = total;
  }
}

// Whether light l is blocked from the hit point pos (normal nrm): any hit on
// the segment from pos offset along the normal to the light, shortened.
template <bool COUNT, bool W4>
__device__ __forceinline__ bool shadow_blocked(const VolumeView& v, const SceneParams& sc, float4 pos, float4 nrm,
                                               uint32_t l, Stack& st, Work& w) {
  const float off_len = kShadowOffset * v.s_diag;
  const float3 so = make_float3(fmaf(off_len, nrm.x, pos.x), fmaf(off_len, nrm.y, pos.y),
                                fmaf(off_len, nrm.z, pos.z));
  const float gx = sc.lpos[l][0] - so.x, gy = sc.lpos[l][1] - so.y, gz = sc.lpos[l][2] - so.z;
  const float len = sqrtf(gx * gx + gy * gy + gz * gz);
  const float il = 1.0f / len;
  const Ray sray = make_ray(so, make_float3(gx * il, gy * il, gz * il));
  const float smax = len * (1.0f - kShadowShorten);
  return W4 ? any_hit4<COUNT>(v, sray, smax, st, w) : any_hit<COUNT>(v, sray, smax, st, w);
}

// Radiance leaving a lit hit (Lambertian, albedo of triangle id): rho/pi
// times the sum over the visible lights `bits` of I_l cos / d^2, the lights
// taken in index order.
__device__ __forceinline__ float3 lit_radiance(const VolumeView& v, const SceneParams& sc, float4 pos, float4 nrm,
                                               int id, uint32_t bits) {
  float er = 0.f, eg = 0.f, eb = 0.f;
  for (int k = 0; k < sc.num_lights; ++k) {
    if (!((bits >> k) & 1u)) continue;
    const float lx = sc.lpos[k][0] - pos.x, ly = sc.lpos[k][1] - pos.y, lz = sc.lpos[k][2] - pos.z;
    const float d2 = lx * lx + ly * ly + lz * lz;
    const float cs = (nrm.x * lx + nrm.y * ly + nrm.z * lz) / sqrtf(d2);
    const float wl = fmaxf(cs, 0.0f) / d2;
    er = fmaf(sc.lint[k][0], wl, er);
    eg = fmaf(sc.lint[k][1], wl, eg);
    eb = fmaf(sc.lint[k][2], wl, eb);
  }
  const float4 rho = v.albedo[id];
  const float inv_pi = 0.318309886183790671538f;
  return make_float3(rho.x * inv_pi * er, rho.y * inv_pi * eg, rho.z * inv_pi * eb);
}

// ---- shadow and shading kernel
// Wave-batch q takes pairs [64q, 64q + 64) of the frame's pair list (the
// batches' segments end to end): lane p finds its batch by binary search in
// pair_off, traces the shadow ray of its (ray, light) pair from the hit point
// offset along the normal towards the light (any hit on the shortened
// segment), and adds its light's bit (if unblocked) and -1 to the ray's
// pending count in one atomic on the ray's own word. The lane that retires
// the ray's last shadow ray shades it: rho/pi times the sum over its visible
// lights of I_l cos / d^2, the lights taken in index order.
template <int KIND, bool COUNT, bool W4>
__device__ __forceinline__ void shade_batch(const VolumeView& v, Stack& st, uint32_t q, uint32_t T, uint32_t nb,
                                            Work& w) {
  const SceneParams& sc = *v.scene;
  const uint32_t p = q * 64u + lane_id();
  if (p >= T) return;
  uint32_t lo = 0u, hi = nb - 1u;  // last batch with pair_off[b] <= p
  while (lo < hi) {
    const uint32_t mid = (lo + hi + 1u) >> 1;
    if (v.pair_off[mid] <= p) lo = mid;
    else hi = mid - 1u;
  }
  const uint32_t b = lo;
  const uint32_t e = v.pairs[(size_t)b * kPairsPerBatch + (p - v.pair_off[b])];
  const uint32_t r = b * v.batch_rays + (e & 63u), l = e >> 6;
  const float4 pos = v.hit_pos[r], nrm = v.hit_nrm[r];
  const bool blocked = shadow_blocked<COUNT, W4>(v, sc, pos, nrm, l, st, w);
  const uint32_t mine = blocked ? 0u : 1u << l;
  const uint32_t old = atomicAdd(&v.hit_vis[r], mine - 256u);
  if ((old >> 8) != 1u) return;
  const uint32_t bits = (old & 0xffu) | mine;
  const int id = __float_as_int(nrm.w);
  emit_ray<KIND>(v, KIND == KIND_PRIMARY ? v.hit_dst[r] : r, lit_radiance(v, sc, pos, nrm, id, bits), pos.w, id,
                 bits);
}

template <int KIND, bool COUNT, bool W4>
__global__ __attribute__((amdgpu_waves_per_eu(8, 8))) void trace_shade_kernel(VolumeView v) {
  extern __shared__ uint64_t smem[];
  const int wave = threadIdx.x >> 6;
  const uint32_t waves = blockDim.x >> 6;
  uint64_t deep[kStackMax - kStackLds];
  Stack st;
  st.lds = (lds_u64*)smem + wave * (64 * kStackLds) + lane_id();
  st.sp = 0;
  st.deep = deep;
  const uint32_t T = v.stats->pair_total, nb = v.stats->pair_batches;
  const uint32_t nq = (T + 63u) / 64u;
  Work w;
  for (uint32_t q = blockIdx.x * waves + (uint32_t)wave; q < nq; q += gridDim.x * waves)
    shade_batch<KIND, COUNT, W4>(v, st, q, T, nb, w);
  flush_stats<COUNT, true>(v, w, 0u);
}

// ---- fused pilot kernel
// Pilot passes are small (8 rays per probe) and their waves end unevenly, so
// a wave traces a batch's shadow rays itself, right after the batch's
// closest hits, with no pair list in global memory, no scan and no second
// launch. The batch's (ray, light) pairs go to the wave's LDS in the order
// the two-kernel form lists them (all pairs of light 0 in lane order, then
// light 1, ...); pair k is traced by lane k mod 64 in round k / 64 and ORs
// its light's bit into its ray's LDS visibility word when unblocked. A ray's
// outputs are those of the two-kernel form: the same hit, the same shadow
// rays, the same light order in its radiance sum. One wave per workgroup;
// its LDS holds the traversal stack, then the pair list (64 kMaxLights
// 16-bit entries), then the 64 visibility words.
constexpr size_t kPilotLdsWave = (size_t)kStackLds * 64 * 8 + 64 * kMaxLights * 2 + 64 * 4;

typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) uint32_t lds_u32;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KIND, bool COUNT, bool W4>
__device__ __forceinline__ void fused_batch(const VolumeView& v, Stack& st, lds_u16* pairs, lds_u32* vis, uint32_t b,
                                            uint32_t total, Work& w, Work& ws, uint32_t& shadow) {
  const SceneParams& sc = *v.scene;
  const uint32_t lane = lane_id(), r0 = b * v.batch_rays;
  uint32_t need, dst;
  {
    const BatchHit h = closest_of_batch<KIND, COUNT, W4>(v, st, b, total, w);
    need = h.need;
    dst = h.dst;
    if (need) {
      v.hit_pos[r0 + lane] = make_float4(h.x.x, h.x.y, h.x.z, h.t);
      v.hit_nrm[r0 + lane] = make_float4(h.n.x, h.n.y, h.n.z, __int_as_float(h.id));
    } else if (h.active) {
      emit_unshadowed<KIND>(v, h);
    }
  }
  vis[lane] = 0u;
  uint32_t n = 0u;
  for (int l = 0; l < sc.num_lights; ++l) {
    const bool p = (need >> l) & 1u;
    const uint64_t m = ballot(p);
    if (p) pairs[n + lanes_below(m)] = (uint16_t)(lane | ((uint32_t)l << 6));
    n += (uint32_t)__popcll(m);
  }
  shadow += n;
  wave_sync();
  for (uint32_t k = lane; k < n; k += 64u) {
    const uint32_t e = pairs[k];
    const uint32_t r = r0 + (e & 63u), l = e >> 6;
    if (!shadow_blocked<COUNT, W4>(v, sc, v.hit_pos[r], v.hit_nrm[r], l, st, ws)) atomicOr((uint32_t*)&vis[e & 63u], 1u << l);
  }
  wave_sync();
  const uint32_t bits = vis[lane];
  wave_sync();  // the next batch rewrites the pair list and the words
  if (!need) return;
  const uint32_t r = r0 + lane;
  const float4 pos = v.hit_pos[r], nrm = v.hit_nrm[r];
  const int id = __float_as_int(nrm.w);
  emit_ray<KIND>(v, dst, lit_radiance(v, sc, pos, nrm, id, bits), pos.w, id, bits);
}

template <int KIND, bool COUNT, bool W4>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(8, 8))) void trace_fused_kernel(VolumeView v,
                                                                                                  int persistent) {
  extern __shared__ uint64_t smem[];
  uint64_t deep[kStackMax - kStackLds];
  Stack st;
  st.lds = (lds_u64*)smem + lane_id();
  st.sp = 0;
  st.deep = deep;
  lds_u16* pairs = (lds_u16*)((lds_u64*)smem + 64 * kStackLds);
  lds_u32* vis = (lds_u32*)(pairs + 64 * kMaxLights);
  const uint32_t total = ray_total<KIND>(v);
  const uint32_t nbatch = (total + v.batch_rays - 1u) / v.batch_rays;
  const uint32_t stride = persistent ? gridDim.x : nbatch;
  Work w, ws;
  uint32_t shadow = 0u;
  for (uint32_t b = blockIdx.x; b < nbatch; b += stride)
    fused_batch<KIND, COUNT, W4>(v, st, pairs, vis, b, total, w, ws, shadow);
  flush_stats<COUNT, false>(v, w, shadow);
  flush_stats<COUNT, true>(v, ws, 0u);
}

size_t trace_lds_bytes(int block) { return (size_t)kStackLds * block * 8; }

template <int KIND, bool COUNT, bool W4>
static hipError_t launch_kind(const VolumeView& v, hipStream_t s, int pers, int block, int grid, int shade_grid,
                              hipEvent_t between) {
  const size_t lds = trace_lds_bytes(block);
  hipLaunchKernelGGL((trace_hit_kernel<KIND, COUNT, W4>), dim3(grid), dim3(block), lds, s, v, pers);
  if (between) {
    const hipError_t e = hipEventRecord(between, s);
    if (e != hipSuccess) return e;
  }
  const uint32_t cap_batches = (v.hit_cap + 63u) / 64u;
  if (cap_batches <= kScanSingleMax) {
    hipLaunchKernelGGL(pair_scan_single_kernel, dim3(1), dim3(1024), 0, s, v);
  } else {
    const uint32_t scan_blocks = cap_batches / (uint32_t)kScanPer + 1u;
    hipLaunchKernelGGL(pair_scan_local_kernel, dim3(scan_blocks), dim3(kScanThreads), 0, s, v);
    hipLaunchKernelGGL(pair_scan_blocks_kernel, dim3(1), dim3(1024), 0, s, v);
    hipLaunchKernelGGL(pair_scan_add_kernel, dim3((cap_batches + kScanThreads) / kScanThreads),
                       dim3(kScanThreads), 0, s, v);
  }
  hipLaunchKernelGGL((trace_shade_kernel<KIND, COUNT, W4>), dim3(shade_grid), dim3(block), lds, s, v);
  return hipGetLastError();
}

template <bool W4>
static hipError_t launch_trace_w(const VolumeView& v, hipStream_t s, bool pilot, int pers, int block, int grid,
                                 int shade_grid, bool count, bool chain, hipEvent_t between) {
  if (chain && count) return launch_kind<KIND_CHAIN, true, W4>(v, s, pers, block, grid, shade_grid, between);
  if (chain) return launch_kind<KIND_CHAIN, false, W4>(v, s, pers, block, grid, shade_grid, between);
  if (pilot) {  // one wave per workgroup, as many waves as the closest-hit launch would have
    const dim3 waves((unsigned)grid * (unsigned)(block / 64));
    if (count) hipLaunchKernelGGL((trace_fused_kernel<KIND_PILOT, true, W4>), waves, dim3(64), kPilotLdsWave, s, v, pers);
    else hipLaunchKernelGGL((trace_fused_kernel<KIND_PILOT, false, W4>), waves, dim3(64), kPilotLdsWave, s, v, pers);
    return hipGetLastError();
  }
  if (count) return launch_kind<KIND_PRIMARY, true, W4>(v, s, pers, block, grid, shade_grid, between);
  return launch_kind<KIND_PRIMARY, false, W4>(v, s, pers, block, grid, shade_grid, between);
}

// grid: blocks of the closest-hit kernel (persistent: the resident grid;
// otherwise enough for every ray). The shading kernel always runs a resident
// grid of `waves_per_cu` waves per CU over the frame's pair list. `between`,
// when given, is recorded after the closest-hit kernel.
hipError_t launch_trace(const VolumeView& v, hipStream_t s, bool pilot, bool persistent, int block, int grid,
                        int shade_grid, bool count, bool w4, bool chain, hipEvent_t between) {
  if (w4) return launch_trace_w<true>(v, s, pilot, persistent ? 1 : 0, block, grid, shade_grid, count, chain, between);
  return launch_trace_w<false>(v, s, pilot, persistent ? 1 : 0, block, grid, shade_grid, count, chain, between);
}

}  // namespace adgi
