// bvh_build.cpp - binned-SAH BVH2 builder (host) for the traversal kernels,
// and its collapse into a 4-wide BVH.
//
// Top-down build with 16 centroid bins per axis and the surface-area cost
// C = 2 + (A_L N_L + A_R N_R) / A (a traversal step costs about two triangle
// tests); leaves hold at most 8 triangles (16 when the depth bound forces
// it). Below depth 40 nodes are split at the object median so the tree never
// exceeds the traversal stack bound. Up to 8 triangles whose box covers at
// least 1/16 of the scene box's area are kept out of the tree (every ray
// tests them first). The output layout stores the first 1024 internal nodes
// breadth-first (the top of the tree is a prefix of the array) and every
// remaining subtree depth-first (children near their parents).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <vector>

#include "adgi_internal.hpp"

namespace adgi {

namespace {

struct Box {
  float lo[3], hi[3];
  void reset() {
    for (int a = 0; a < 3; ++a) {
      lo[a] = INFINITY;
      hi[a] = -INFINITY;
    }
  }
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  double area() const {
    double e[3];
    for (int a = 0; a < 3; ++a) e[a] = std::max(0.0, (double)hi[a] - (double)lo[a]);
    return 2.0 * (e[0] * e[1] + e[1] * e[2] + e[2] * e[0]);
  }
};

struct BNode {
  Box box;
  int left = -1, right = -1;  // build-node indices; -1 for a leaf
  int start = 0, count = 0;
  int depth = 0;
};

constexpr int kBins = 16;
constexpr int kLeafTarget = 8;
constexpr int kMedianDepth = 40;
constexpr double kBigFraction = 1.0 / 16;  // of the scene box's surface area
constexpr int32_t kMaxBigTris = 8;
// SAH cost of one traversal step relative to one triangle test: a node visit
// (two slab tests, stack work) costs about two triangle tests here.
constexpr double kTraversalCost = 2.0;

}  // namespace

bool build_bvh(const float* pos, int32_t nv, const int32_t* idx, int32_t nt, float pad_abs,
               BvhHost& out, const char** err) {
  out.nodes.clear();
  out.tris.clear();
  out.tri_order.clear();
  out.level_nodes.clear();
  out.level_offsets.clear();
  out.depth = 0;
  out.num_big = 0;
  if (nt == 0) {
    // a root whose children are never entered (the kernels skip traversal)
    out.nodes.assign(4, make_float4(0.f, 0.f, 0.f, 0.f));
    float4 lk;
    int neg = ~0;
    std::memcpy(&lk.x, &neg, 4);
    std::memcpy(&lk.y, &neg, 4);
    int par = -1, side = 0;
    std::memcpy(&lk.z, &par, 4);
    std::memcpy(&lk.w, &side, 4);
    out.nodes[3] = lk;
    out.depth = 1;
    return true;
  }
  std::vector<Box> tb(nt);
  std::vector<float> cen(3 * (size_t)nt);
  for (int32_t t = 0; t < nt; ++t) {
    tb[t].reset();
    for (int c = 0; c < 3; ++c) {
      int32_t v = idx[3 * t + c];
      if (v < 0 || v >= nv) {
        *err = "triangle index out of range";
        return false;
      }
      tb[t].grow(pos + 3 * (size_t)v);
    }
    for (int a = 0; a < 3; ++a) cen[3 * (size_t)t + a] = 0.5f * (tb[t].lo[a] + tb[t].hi[a]);
  }
  std::vector<int32_t> ord(nt);
  for (int32_t t = 0; t < nt; ++t) ord[t] = t;

  // Triangles whose box is a large fraction of the scene box (a ground
  // plane, a wall) would inflate every node on their leaf's path to nearly
  // the scene's size, so every ray would descend that whole path. They go to
  // a short list in slots [0, num_big) that rays test before the tree.
  int32_t nbig = 0;
  {
    Box all;
    all.reset();
    for (int32_t t = 0; t < nt; ++t) all.grow(tb[t]);
    const double a_all = all.area();
    std::vector<int32_t> big;
    for (int32_t t = 0; t < nt; ++t)
      if (tb[t].area() >= kBigFraction * a_all) big.push_back(t);
    std::stable_sort(big.begin(), big.end(),
                     [&](int32_t x, int32_t y) { return tb[x].area() > tb[y].area(); });
    nbig = std::min<int32_t>({(int32_t)big.size(), kMaxBigTris, nt - 1});
    std::vector<char> is_big(nt, 0);
    for (int32_t k = 0; k < nbig; ++k) is_big[big[k]] = 1;
    int32_t w = 0;
    for (int32_t k = 0; k < nbig; ++k) ord[w++] = big[k];
    for (int32_t t = 0; t < nt; ++t)
      if (!is_big[t]) ord[w++] = t;
  }
  out.num_big = nbig;

  std::vector<BNode> bn;
  bn.reserve(2 * (size_t)nt / 2 + 8);
  bn.push_back(BNode());
  bn[0].start = nbig;
  bn[0].count = nt - nbig;
  std::vector<int> work{0};
  int max_depth = 0;
  while (!work.empty()) {
    int ni = work.back();
    work.pop_back();
    BNode nd = bn[ni];
    nd.box.reset();
    Box cb;
    cb.reset();
    for (int i = nd.start; i < nd.start + nd.count; ++i) {
      nd.box.grow(tb[ord[i]]);
      cb.grow(&cen[3 * (size_t)ord[i]]);
    }
    max_depth = std::max(max_depth, nd.depth);
    bool make_leaf = nd.count <= 2;
    int split = -1;
    if (!make_leaf) {
      int axis = -1, bin_split = -1;
      double best = INFINITY;
      if (nd.depth < kMedianDepth) {
        for (int a = 0; a < 3; ++a) {
          float ext = cb.hi[a] - cb.lo[a];
          if (!(ext > 0.f)) continue;
          Box bb[kBins];
          int bc[kBins] = {0};
          for (int b = 0; b < kBins; ++b) bb[b].reset();
          float k = kBins / ext;
          for (int i = nd.start; i < nd.start + nd.count; ++i) {
            int t = ord[i];
            int b = std::min(kBins - 1, (int)((cen[3 * (size_t)t + a] - cb.lo[a]) * k));
            bb[b].grow(tb[t]);
            bc[b]++;
          }
          Box rb[kBins];
          int rc[kBins];
          Box acc;
          acc.reset();
          int cnt = 0;
          for (int b = kBins - 1; b >= 0; --b) {
            acc.grow(bb[b]);
            cnt += bc[b];
            rb[b] = acc;
            rc[b] = cnt;
          }
          acc.reset();
          cnt = 0;
          for (int b = 0; b < kBins - 1; ++b) {
            acc.grow(bb[b]);
            cnt += bc[b];
            if (cnt == 0 || rc[b + 1] == 0) continue;
            double c = acc.area() * cnt + rb[b + 1].area() * rc[b + 1];
            if (c < best) {
              best = c;
              axis = a;
              bin_split = b;
            }
          }
        }
      }
      double parent_area = std::max(nd.box.area(), 1e-30);
      double split_cost = kTraversalCost + best / parent_area;
      if (axis >= 0 && !(nd.count <= kLeafTarget && split_cost >= (double)nd.count)) {
        float ext = cb.hi[axis] - cb.lo[axis];
        float k = kBins / ext;
        auto mid = std::partition(ord.begin() + nd.start, ord.begin() + nd.start + nd.count,
                                  [&](int32_t t) {
                                    int b = std::min(kBins - 1,
                                                     (int)((cen[3 * (size_t)t + axis] - cb.lo[axis]) * k));
                                    return b <= bin_split;
                                  });
        split = (int)(mid - ord.begin());
        if (split == nd.start || split == nd.start + nd.count) split = -1;
      } else if (axis >= 0) {
        make_leaf = true;
      }
      if (!make_leaf && split < 0) {
        if (nd.count <= kLeafTarget) {
          make_leaf = true;
        } else {
          // object median along the widest centroid extent
          int a = 0;
          for (int q = 1; q < 3; ++q)
            if (cb.hi[q] - cb.lo[q] > cb.hi[a] - cb.lo[a]) a = q;
          split = nd.start + nd.count / 2;
          std::nth_element(ord.begin() + nd.start, ord.begin() + split,
                           ord.begin() + nd.start + nd.count, [&](int32_t x, int32_t y) {
                             float cx = cen[3 * (size_t)x + a], cy = cen[3 * (size_t)y + a];
                             return cx < cy || (cx == cy && x < y);
                           });
        }
      }
    }
    if (make_leaf && nd.count > kLeafMaxTris) {
      make_leaf = false;
      split = nd.start + nd.count / 2;
    }
    if (make_leaf) {
      bn[ni] = nd;
      continue;
    }
    BNode L, R;
    L.start = nd.start;
    L.count = split - nd.start;
    R.start = split;
    R.count = nd.start + nd.count - split;
    L.depth = R.depth = nd.depth + 1;
    nd.left = (int)bn.size();
    nd.right = nd.left + 1;
    bn[ni] = nd;
    bn.push_back(L);
    bn.push_back(R);
    work.push_back(nd.left);
    work.push_back(nd.right);
  }
  // leaf boxes were computed when popped; make sure every node has its box
  out.depth = max_depth + 1;
  if (out.depth > kStackMax - 2) {
    *err = "BVH deeper than the traversal stack bound";
    return false;
  }

  // ---- layout: BFS for the first 1024 internal nodes, then DFS subtrees
  const size_t kTop = 1024;
  std::vector<int> gpu_of(bn.size(), -1), order;
  bool root_leaf = bn[0].left < 0;
  if (!root_leaf) {
    std::deque<int> q{0};
    while (!q.empty() && order.size() < kTop) {
      int n = q.front();
      q.pop_front();
      gpu_of[n] = (int)order.size();
      order.push_back(n);
      if (bn[n].left >= 0 && bn[bn[n].left].left >= 0) q.push_back(bn[n].left);
      if (bn[n].right >= 0 && bn[bn[n].right].left >= 0) q.push_back(bn[n].right);
    }
    std::vector<int> st;
    for (int r : q) {
      st.push_back(r);
      while (!st.empty()) {
        int n = st.back();
        st.pop_back();
        gpu_of[n] = (int)order.size();
        order.push_back(n);
        if (bn[bn[n].right].left >= 0) st.push_back(bn[n].right);
        if (bn[bn[n].left].left >= 0) st.push_back(bn[n].left);
      }
    }
  } else {
    order.push_back(0);
    gpu_of[0] = 0;
  }

  out.tri_order = ord;
  out.tris.resize(3 * (size_t)nt);
  for (int32_t s = 0; s < nt; ++s) {
    int32_t t = ord[s];
    const float* v0 = pos + 3 * (size_t)idx[3 * t];
    const float* v1 = pos + 3 * (size_t)idx[3 * t + 1];
    const float* v2 = pos + 3 * (size_t)idx[3 * t + 2];
    float4 a, b, c;
    a.x = v0[0];
    a.y = v0[1];
    a.z = v0[2];
    std::memcpy(&a.w, &t, 4);
    b = make_float4(v1[0] - v0[0], v1[1] - v0[1], v1[2] - v0[2], 0.f);
    c = make_float4(v2[0] - v0[0], v2[1] - v0[1], v2[2] - v0[2], 0.f);
    out.tris[3 * (size_t)s] = a;
    out.tris[3 * (size_t)s + 1] = b;
    out.tris[3 * (size_t)s + 2] = c;
  }

  auto child_code = [&](int c) -> int {
    if (bn[c].left >= 0) return gpu_of[c];
    return ~((bn[c].start << kLeafShift) | (bn[c].count - 1));
  };
  auto put = [&](float4* f, int side, const Box& b) {
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = pad_lo(b.lo[a], pad_abs);
      hi[a] = pad_hi(b.hi[a], pad_abs);
    }
    if (side == 0) {
      f[0].x = lo[0];
      f[0].y = lo[1];
      f[0].z = lo[2];
      f[0].w = hi[0];
      f[1].x = hi[1];
      f[1].y = hi[2];
    } else {
      f[1].z = lo[0];
      f[1].w = lo[1];
      f[2].x = lo[2];
      f[2].y = hi[0];
      f[2].z = hi[1];
      f[2].w = hi[2];
    }
  };
  out.nodes.assign(4 * order.size(), make_float4(0.f, 0.f, 0.f, 0.f));
  for (size_t g = 0; g < order.size(); ++g) {
    int n = order[g];
    float4* f = &out.nodes[4 * g];
    int lc, rc, par = -1, side = 0;
    if (root_leaf) {
      // root leaf: both sides point at the same leaf
      lc = rc = ~((bn[0].start << kLeafShift) | (bn[0].count - 1));
      put(f, 0, bn[0].box);
      put(f, 1, bn[0].box);
    } else {
      lc = child_code(bn[n].left);
      rc = child_code(bn[n].right);
      put(f, 0, bn[bn[n].left].box);
      put(f, 1, bn[bn[n].right].box);
    }
    std::memcpy(&f[3].x, &lc, 4);
    std::memcpy(&f[3].y, &rc, 4);
    std::memcpy(&f[3].z, &par, 4);
    std::memcpy(&f[3].w, &side, 4);
  }
  // internal nodes grouped by depth, for the level-by-level refit
  {
    std::vector<std::vector<int32_t>> lv;
    for (size_t g = 0; g < order.size(); ++g) {
      int d = bn[order[g]].depth;
      if ((int)lv.size() <= d) lv.resize(d + 1);
      lv[d].push_back((int32_t)g);
    }
    out.level_offsets.push_back(0);
    for (auto& l : lv) {
      out.level_nodes.insert(out.level_nodes.end(), l.begin(), l.end());
      out.level_offsets.push_back((int32_t)out.level_nodes.size());
    }
  }
  // parent links
  for (size_t g = 0; g < order.size(); ++g) {
    int lc, rc;
    std::memcpy(&lc, &out.nodes[4 * g + 3].x, 4);
    std::memcpy(&rc, &out.nodes[4 * g + 3].y, 4);
    int gi = (int)g;
    if (lc >= 0) {
      std::memcpy(&out.nodes[4 * (size_t)lc + 3].z, &gi, 4);
      int s0 = 0;
      std::memcpy(&out.nodes[4 * (size_t)lc + 3].w, &s0, 4);
    }
    if (rc >= 0 && !(root_leaf)) {
      std::memcpy(&out.nodes[4 * (size_t)rc + 3].z, &gi, 4);
      int s1 = 1;
      std::memcpy(&out.nodes[4 * (size_t)rc + 3].w, &s1, 4);
    }
  }
  return true;
}

void collapse_bvh4(const BvhHost& b2, Bvh4Host& out) {
  out.nodes.clear();
  out.src.clear();
  out.max_stack = 0;
  const float* f2 = (const float*)b2.nodes.data();
  auto code_of = [&](int ref) {
    int c;
    std::memcpy(&c, f2 + 16 * (size_t)(ref >> 1) + 12 + (ref & 1), 4);
    return c;
  };
  auto area_of = [&](int ref) {
    const float* b = f2 + 16 * (size_t)(ref >> 1) + 6 * (ref & 1);
    float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
    return dx * dy + dy * dz + dz * dx;
  };
  // explicit DFS: a node's children are emitted (depth first) before its
  // next sibling; `patch` is where the parent stores the child's index
  struct Item {
    int g2, acc, patch;
  };
  std::vector<Item> todo{{0, 0, -1}};
  while (!todo.empty()) {
    Item it = todo.back();
    todo.pop_back();
    const int me = (int)(out.nodes.size() / 8);
    if (it.patch >= 0) std::memcpy((float*)out.nodes.data() + it.patch, &me, 4);
    int refs[4] = {2 * it.g2, 2 * it.g2 + 1, -1, -1};
    int nch = 2;
    while (nch < 4) {
      int best = -1;
      float best_a = -1.f;
      for (int k = 0; k < nch; ++k)
        if (code_of(refs[k]) >= 0 && area_of(refs[k]) > best_a) {
          best_a = area_of(refs[k]);
          best = k;
        }
      if (best < 0) break;
      const int c = code_of(refs[best]);
      refs[best] = 2 * c;
      refs[nch++] = 2 * c + 1;
    }
    const int acc = it.acc + nch - 1;
    out.max_stack = std::max(out.max_stack, acc);
    out.nodes.resize(8 * (size_t)(me + 1), make_float4(0.f, 0.f, 0.f, 0.f));
    out.src.resize(4 * (size_t)(me + 1), -1);
    float* f = (float*)&out.nodes[8 * (size_t)me];
    std::vector<Item> kids;
    for (int k = 0; k < 4; ++k) {
      int child = kEmptyChild;
      if (k < nch) {
        const float* b = f2 + 16 * (size_t)(refs[k] >> 1) + 6 * (refs[k] & 1);
        for (int a = 0; a < 3; ++a) {
          f[4 * a + k] = b[a];
          f[12 + 4 * a + k] = b[3 + a];
        }
        out.src[4 * (size_t)me + k] = refs[k];
        child = code_of(refs[k]);
        if (child >= 0) kids.push_back({child, acc, 8 * me * 4 + 24 + k});
      }
      std::memcpy(f + 24 + k, &child, 4);
    }
    // first child on top of the work stack, so it directly follows its parent
    for (auto k = kids.rbegin(); k != kids.rend(); ++k) todo.push_back(*k);
  }
}

}  // namespace adgi
