// bvh.cpp -- host construction of the 4-wide BVH used by the transport kernels.
//
// The paper does not describe its acceleration structure; this one is built
// for gfx950: a binned surface-area-heuristic binary tree (Wald, "On fast
// construction of SAH-based bounding volume hierarchies", 2007) collapsed to
// 4-wide nodes whose child boxes fill one 128-byte cache line, laid out
// breadth-first so that the top levels are a prefix of the node array and can
// be staged in LDS with one contiguous copy.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>

#include "xp_internal.h"

namespace xp {
namespace {

struct Box {
  float lo[3], hi[3];
  Box() {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::numeric_limits<float>::infinity();
      hi[k] = -std::numeric_limits<float>::infinity();
    }
  }
  void grow(const float* p) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  double area() const {
    if (!(hi[0] >= lo[0])) return 0.0;
    const double dx = double(hi[0]) - lo[0], dy = double(hi[1]) - lo[1], dz = double(hi[2]) - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct Node2 {
  Box box;
  int32_t left = -1, right = -1;  // inner: children
  int32_t first = 0, count = 0;   // leaf: range in the permutation
};

}  // namespace

bool build_bvh4(const float* vtx, const int32_t* tri, int64_t nt, const int32_t* mat_in,
                const int32_t* mat_out, const int32_t* surface, const int32_t* sensor,
                int max_leaf, int bins, BvhResult& out, std::string& err) {
  if (nt <= 0) {
    err = "empty mesh";
    return false;
  }
  if (nt >= kMaxLeafFirst) {
    err = "mesh has 2^28 or more triangles";
    return false;
  }
  if (max_leaf < 1 || max_leaf > 8) {
    err = "max_leaf_size must be 1..8";
    return false;
  }
  std::vector<Box> tb(nt);
  std::vector<float> cen(3 * nt);
  for (int64_t i = 0; i < nt; ++i) {
    for (int j = 0; j < 3; ++j) tb[i].grow(vtx + 3 * int64_t(tri[3 * i + j]));
    for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5f * (tb[i].lo[k] + tb[i].hi[k]);
  }
  std::vector<int32_t> perm(nt);
  for (int64_t i = 0; i < nt; ++i) perm[i] = int32_t(i);

  // ---- binned SAH binary tree ----
  std::vector<Node2> n2;
  n2.reserve(2 * size_t(nt) / std::max(1, max_leaf) + 16);
  n2.emplace_back();
  struct Work { int32_t node, first, count; };
  std::vector<Work> work{{0, 0, int32_t(nt)}};
  std::vector<Box> bin_box(bins);
  std::vector<int32_t> bin_cnt(bins);
  std::vector<double> right_cost(bins);
  while (!work.empty()) {
    const Work w = work.back();
    work.pop_back();
    Box box, cb;
    for (int32_t i = w.first; i < w.first + w.count; ++i) {
      box.grow(tb[perm[i]]);
      cb.grow(&cen[3 * size_t(perm[i])]);
    }
    n2[w.node].box = box;
    auto make_leaf = [&]() {
      n2[w.node].first = w.first;
      n2[w.node].count = w.count;
    };
    if (w.count <= 1) {
      make_leaf();
      continue;
    }
    // best split over the three axes
    double best_cost = std::numeric_limits<double>::infinity();
    int best_axis = -1, best_split = -1;
    const double parent_area = std::max(box.area(), 1e-30);
    for (int axis = 0; axis < 3; ++axis) {
      const float ext = cb.hi[axis] - cb.lo[axis];
      if (!(ext > 0.0f)) continue;
      const double scale = double(bins) / ext;
      std::fill(bin_cnt.begin(), bin_cnt.end(), 0);
      for (auto& b : bin_box) b = Box();
      for (int32_t i = w.first; i < w.first + w.count; ++i) {
        const int32_t t = perm[i];
        int b = int((cen[3 * size_t(t) + axis] - cb.lo[axis]) * scale);
        b = std::min(std::max(b, 0), bins - 1);
        bin_cnt[b] += 1;
        bin_box[b].grow(tb[t]);
      }
      Box acc;
      int32_t cnt = 0;
      for (int b = bins - 1; b > 0; --b) {
        acc.grow(bin_box[b]);
        cnt += bin_cnt[b];
        right_cost[b] = acc.area() * cnt;
      }
      acc = Box();
      cnt = 0;
      for (int b = 0; b < bins - 1; ++b) {
        acc.grow(bin_box[b]);
        cnt += bin_cnt[b];
        if (cnt == 0 || cnt == w.count) continue;
        const double c = 1.0 + (acc.area() * cnt + right_cost[b + 1]) / parent_area;
        if (c < best_cost) {
          best_cost = c;
          best_axis = axis;
          best_split = b + 1;
        }
      }
    }
    if (w.count <= max_leaf && best_cost >= double(w.count)) {
      make_leaf();
      continue;
    }
    int32_t mid;
    if (best_axis >= 0) {
      const float ext = cb.hi[best_axis] - cb.lo[best_axis];
      const double scale = double(bins) / ext;
      auto it = std::partition(perm.begin() + w.first, perm.begin() + w.first + w.count,
                               [&](int32_t t) {
                                 int b = int((cen[3 * size_t(t) + best_axis] - cb.lo[best_axis]) * scale);
                                 b = std::min(std::max(b, 0), bins - 1);
                                 return b < best_split;
                               });
      mid = int32_t(it - perm.begin());
    } else {
      mid = w.first + w.count / 2;  // coincident centroids: split the list in half
    }
    if (mid <= w.first || mid >= w.first + w.count) mid = w.first + w.count / 2;
    const int32_t l = int32_t(n2.size());
    n2.emplace_back();
    n2.emplace_back();
    n2[w.node].left = l;
    n2[w.node].right = l + 1;
    work.push_back({l + 1, mid, w.first + w.count - mid});
    work.push_back({l, w.first, mid - w.first});
  }

  // ---- collapse to 4-wide nodes, breadth-first ----
  auto is_leaf = [&](int32_t i) { return n2[i].left < 0; };
  out.nodes.clear();
  out.level_end.clear();
  struct Item { int32_t n2, slot, level; };
  std::deque<Item> q;
  out.nodes.emplace_back();
  q.push_back({0, 0, 0});
  int32_t depth = 0;
  std::vector<int32_t> level_of;
  level_of.push_back(0);
  while (!q.empty()) {
    const Item it = q.front();
    q.pop_front();
    int32_t kids[4];
    int nk = 0;
    if (is_leaf(it.n2)) {
      kids[nk++] = it.n2;
    } else {
      kids[nk++] = n2[it.n2].left;
      kids[nk++] = n2[it.n2].right;
      while (nk < 4) {
        int pick = -1;
        double area = -1.0;
        for (int k = 0; k < nk; ++k)
          if (!is_leaf(kids[k]) && n2[kids[k]].box.area() > area) {
            area = n2[kids[k]].box.area();
            pick = k;
          }
        if (pick < 0) break;
        const int32_t x = kids[pick];
        kids[pick] = n2[x].left;
        kids[nk++] = n2[x].right;
      }
    }
    Node4 node;
    for (int k = 0; k < 4; ++k) {
      if (k >= nk) {
        node.lox[k] = node.loy[k] = node.loz[k] = 0.0f;
        node.hix[k] = node.hiy[k] = node.hiz[k] = 0.0f;
        node.child[k] = kEmptyChild;
        node.reserved[k] = 0;
        continue;
      }
      const Node2& c = n2[kids[k]];
      // pad each box so that the kernel's slab test never drops a triangle the
      // exact triangle test would hit: 2^-20 relative plus 1e-7 m absolute
      float lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        const float pad = (std::fabs(c.box.lo[d]) + std::fabs(c.box.hi[d])) * 9.5367432e-7f + 1e-7f;
        lo[d] = c.box.lo[d] - pad;
        hi[d] = c.box.hi[d] + pad;
      }
      node.lox[k] = lo[0]; node.loy[k] = lo[1]; node.loz[k] = lo[2];
      node.hix[k] = hi[0]; node.hiy[k] = hi[1]; node.hiz[k] = hi[2];
      node.reserved[k] = 0;
      if (is_leaf(kids[k])) {
        node.child[k] = ~((c.first << 3) | (c.count - 1));
      } else {
        const int32_t slot = int32_t(out.nodes.size());
        out.nodes.emplace_back();
        level_of.push_back(it.level + 1);
        depth = std::max(depth, it.level + 1);
        node.child[k] = slot;
        q.push_back({kids[k], slot, it.level + 1});
      }
    }
    out.nodes[it.slot] = node;
  }
  out.depth = depth;
  out.level_end.assign(depth + 1, 0);
  for (size_t i = 0; i < level_of.size(); ++i) out.level_end[level_of[i]] = int32_t(i) + 1;
  for (int l = 1; l <= depth; ++l) out.level_end[l] = std::max(out.level_end[l], out.level_end[l - 1]);

  // worst-case stack of the traversal: a visit pushes at most (children - 1)
  // of its own children (one is followed or postponed) plus the partly tested
  // leaf the lane may still hold; need(node) = children + max need(inner child)
  std::vector<int32_t> need(out.nodes.size(), 0);
  for (int64_t i = int64_t(out.nodes.size()) - 1; i >= 0; --i) {
    const Node4& nd = out.nodes[i];
    int kids = 0, sub = 0;
    for (int k = 0; k < 4; ++k) {
      if (nd.child[k] == kEmptyChild) continue;
      ++kids;
      if (nd.child[k] >= 0) sub = std::max(sub, need[nd.child[k]]);
    }
    need[i] = kids + sub;
  }
  out.max_stack = need[0] + 1;

  // ---- triangle records in leaf order, three rotated copies ----
  out.tris.resize(3 * nt);
  for (int64_t i = 0; i < nt; ++i) {
    const int32_t t = perm[i];
    const float* p0 = vtx + 3 * int64_t(tri[3 * int64_t(t)]);
    const float* p1 = vtx + 3 * int64_t(tri[3 * int64_t(t) + 1]);
    const float* p2 = vtx + 3 * int64_t(tri[3 * int64_t(t) + 2]);
    const uint32_t packed = uint32_t(mat_in[t]) | (uint32_t(mat_out[t]) << 8) |
                            (uint32_t(surface[t] + 1) << 16);
    const int32_t sens = sensor[t];
    for (int kz = 0; kz < 3; ++kz) {
      TriRec r;
      for (int k = 0; k < 3; ++k) {
        const int src = (kz + 1 + k) % 3;  // k = 0, 1, 2 -> kx, ky, kz
        r.a[k] = p0[src];
        r.b[k] = p1[src];
        r.c[k] = p2[src];
      }
      std::memcpy(&r.a[3], &t, 4);
      std::memcpy(&r.b[3], &packed, 4);
      std::memcpy(&r.c[3], &sens, 4);
      out.tris[((kz + 1) % 3) * nt + i] = r;
    }
  }
  return true;
}

}  // namespace xp
