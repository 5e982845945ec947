// bvh.cpp -- host construction of the 4-wide BVH used by the transport kernels.
//
// The paper does not describe its acceleration structure; this one is built
// for gfx950: a binned surface-area-heuristic binary tree (Wald, "On fast
// construction of SAH-based bounding volume hierarchies", 2007) collapsed to
// 4-wide nodes whose child boxes fill one 128-byte cache line, laid out
// breadth-first so that the top levels are a prefix of the node array and can
// be staged in LDS with one contiguous copy.
//
// Before the build, triangles whose bounding box is much larger than the
// triangle itself (long slivers, such as the wedges of a disk triangulated as
// a fan from its centre) are pre-split into several references with tighter
// boxes (early split clipping: Ernst and Woop, "Early split clipping for
// bounding volume hierarchies", 2007; the worst boxes first, under a budget of
// extra references, in the spirit of Karras and Aila, "Fast parallel
// construction of high-quality bounding volume hierarchies", 2013).  Every
// reference stores the whole triangle and its id, so the closest hit, and with
// it every result, is the same with or without splitting.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <limits>
#include <queue>

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

// ---- reference pre-splitting ----

constexpr int kMaxSplitDepth = 10;    // at most 2^10 pieces per triangle
constexpr double kSplitWasteRatio = 2.0;  // split while box area > ratio * ideal area

float round_down(double x) {
  float f = float(x);
  return double(f) > x ? std::nextafter(f, -std::numeric_limits<float>::infinity()) : f;
}
float round_up(double x) {
  float f = float(x);
  return double(f) < x ? std::nextafter(f, std::numeric_limits<float>::infinity()) : f;
}

struct Poly {
  static constexpr int kCap = 3 + 2 * 6;
  int n = 0;
  bool overflow = false;  // a clip would have exceeded kCap vertices
  double v[kCap][3];      // a triangle clipped by at most six planes (one vertex each)
};

// Clip a convex polygon to {x[axis] <= c} (keep_below) or {x[axis] >= c}.
// Each plane adds at most one vertex to a convex polygon; should rounding make
// an edge list cross the plane more often, the result is marked as overflowed
// rather than written past its capacity.
Poly clip(const Poly& in, int axis, double c, bool keep_below) {
  Poly out;
  out.overflow = in.overflow;
  for (int i = 0; i < in.n; ++i) {
    if (out.n + 2 > Poly::kCap) {
      out.overflow = true;
      return out;
    }
    const double* p = in.v[i];
    const double* q = in.v[(i + 1) % in.n];
    const double dp = keep_below ? c - p[axis] : p[axis] - c;
    const double dq = keep_below ? c - q[axis] : q[axis] - c;
    if (dp >= 0.0) std::memcpy(out.v[out.n++], p, sizeof(out.v[0]));
    if ((dp > 0.0 && dq < 0.0) || (dp < 0.0 && dq > 0.0)) {
      const double s = dp / (dp - dq);
      double* r = out.v[out.n++];
      for (int k = 0; k < 3; ++k) r[k] = p[k] + s * (q[k] - p[k]);
      r[axis] = c;
    }
  }
  return out;
}

struct Piece {
  double cell_lo[3], cell_hi[3];  // the region of the triangle this reference covers
  float lo[3], hi[3];             // its bounds, rounded outward
  double waste;                   // box area above the ideal one
  int32_t tri, depth;
  bool operator<(const Piece& o) const { return waste < o.waste; }
};

// The part of triangle t inside the cell, its outward-rounded bounds and its
// wasted box area: a planar piece of area A and unit normal n needs a box of
// area at least 2 A (|nx| + |ny| + |nz|).  Returns false for an empty piece.
bool make_piece(const double tri[3][3], const double n_l1, Piece& pc) {
  Poly poly;
  poly.n = 3;
  for (int j = 0; j < 3; ++j)
    for (int k = 0; k < 3; ++k) poly.v[j][k] = tri[j][k];
  for (int k = 0; k < 3 && poly.n > 0 && !poly.overflow; ++k) {
    if (std::isfinite(pc.cell_lo[k])) poly = clip(poly, k, pc.cell_lo[k], false);
    if (poly.n > 0 && std::isfinite(pc.cell_hi[k])) poly = clip(poly, k, pc.cell_hi[k], true);
  }
  if (poly.overflow) {
    // conservative piece: the triangle's box within the cell, never split further
    for (int k = 0; k < 3; ++k) {
      double lo = std::min(std::min(tri[0][k], tri[1][k]), tri[2][k]);
      double hi = std::max(std::max(tri[0][k], tri[1][k]), tri[2][k]);
      if (std::isfinite(pc.cell_lo[k])) lo = std::max(lo, pc.cell_lo[k]);
      if (std::isfinite(pc.cell_hi[k])) hi = std::min(hi, pc.cell_hi[k]);
      if (lo > hi) return false;
      pc.lo[k] = round_down(lo);
      pc.hi[k] = round_up(hi);
    }
    pc.waste = 0.0;
    return true;
  }
  if (poly.n < 3) return false;
  double lo[3], hi[3];
  for (int k = 0; k < 3; ++k) lo[k] = hi[k] = poly.v[0][k];
  for (int i = 1; i < poly.n; ++i)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], poly.v[i][k]);
      hi[k] = std::max(hi[k], poly.v[i][k]);
    }
  double cx = 0.0, cy = 0.0, cz = 0.0;  // polygon area from the fan of cross products
  for (int i = 1; i + 1 < poly.n; ++i) {
    const double* a = poly.v[0];
    const double* b = poly.v[i];
    const double* c = poly.v[i + 1];
    const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    cx += u[1] * w[2] - u[2] * w[1];
    cy += u[2] * w[0] - u[0] * w[2];
    cz += u[0] * w[1] - u[1] * w[0];
  }
  const double area = 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
  for (int k = 0; k < 3; ++k) {
    pc.lo[k] = round_down(lo[k]);
    pc.hi[k] = round_up(hi[k]);
  }
  const double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
  const double box_area = 2.0 * (dx * dy + dy * dz + dz * dx);
  const double ideal = 2.0 * area * n_l1;
  pc.waste = box_area > kSplitWasteRatio * ideal ? box_area - ideal : 0.0;
  return true;
}

struct Node2 {
  Box box;
  int32_t left = -1, right = -1;  // inner: children
  int32_t first = 0, count = 0;   // leaf: range in the permutation
};

}  // namespace

bool build_bvh4(const float* vtx, const int32_t* tri, int64_t nt, const int32_t* mat_in,
                const int32_t* mat_out, const int32_t* surface, const int32_t* sensor,
                int max_leaf, int bins, double split_budget, BvhResult& out, std::string& err) {
  if (nt <= 0) {
    err = "empty mesh";
    return false;
  }
  if (nt >= kMaxReferences) {
    err = "mesh has 2^24 or more triangles";
    return false;
  }
  if (max_leaf < 1 || max_leaf > 8) {
    err = "max_leaf_size must be 1..8";
    return false;
  }
  // ---- references: whole triangles, or pieces of the worst-fitting ones ----
  std::vector<Box> tb;
  std::vector<int32_t> ref_tri;
  const int64_t budget = std::min<int64_t>(int64_t(split_budget * double(nt)),
                                           kMaxReferences - 1 - nt);
  {
    std::priority_queue<Piece> heap;
    std::vector<Piece> done;
    std::vector<double> n_l1(nt, 0.0);
    auto corners = [&](int32_t t, double p[3][3]) {
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k) p[j][k] = vtx[3 * int64_t(tri[3 * int64_t(t) + j]) + k];
    };
    tb.reserve(size_t(nt) + size_t(std::max<int64_t>(budget, 0)));
    ref_tri.reserve(tb.capacity());
    for (int64_t i = 0; i < nt; ++i) {
      Box b;
      for (int j = 0; j < 3; ++j) b.grow(vtx + 3 * int64_t(tri[3 * i + j]));
      if (budget <= 0) {
        tb.push_back(b);
        ref_tri.push_back(int32_t(i));
        continue;
      }
      double p[3][3];
      corners(int32_t(i), p);
      const double u[3] = {p[1][0] - p[0][0], p[1][1] - p[0][1], p[1][2] - p[0][2]};
      const double w[3] = {p[2][0] - p[0][0], p[2][1] - p[0][1], p[2][2] - p[0][2]};
      const double c[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2],
                           u[0] * w[1] - u[1] * w[0]};
      const double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
      Piece pc;
      for (int k = 0; k < 3; ++k) {
        pc.cell_lo[k] = -std::numeric_limits<double>::infinity();
        pc.cell_hi[k] = std::numeric_limits<double>::infinity();
      }
      pc.tri = int32_t(i);
      pc.depth = 0;
      if (len > 0.0) n_l1[i] = (std::fabs(c[0]) + std::fabs(c[1]) + std::fabs(c[2])) / len;
      if (len > 0.0 && make_piece(p, n_l1[i], pc) && pc.waste > 0.0) {
        heap.push(pc);
      } else {  // degenerate or well fitting: the whole triangle
        tb.push_back(b);
        ref_tri.push_back(int32_t(i));
      }
    }
    int64_t extra = 0;
    while (!heap.empty()) {
      Piece pc = heap.top();
      heap.pop();
      if (extra >= budget || pc.depth >= kMaxSplitDepth || pc.waste <= 0.0) {
        done.push_back(pc);
        continue;
      }
      // halve the piece's bounds along their longest axis
      int axis = 0;
      for (int k = 1; k < 3; ++k)
        if (double(pc.hi[k]) - pc.lo[k] > double(pc.hi[axis]) - pc.lo[axis]) axis = k;
      const double mid = 0.5 * (double(pc.lo[axis]) + double(pc.hi[axis]));
      double p[3][3];
      corners(pc.tri, p);
      Piece kid[2] = {pc, pc};
      kid[0].cell_hi[axis] = std::min(pc.cell_hi[axis], mid);
      kid[1].cell_lo[axis] = std::max(pc.cell_lo[axis], mid);
      int made = 0;
      for (Piece& k : kid) {
        k.depth = pc.depth + 1;
        if (make_piece(p, n_l1[pc.tri], k)) {
          heap.push(k);
          ++made;
        }
      }
      if (made == 0) {  // cannot happen for a non-empty piece; keep it whole
        done.push_back(pc);
        continue;
      }
      extra += made - 1;
    }
    for (const Piece& pc : done) {
      Box b;
      for (int k = 0; k < 3; ++k) {
        b.lo[k] = pc.lo[k];
        b.hi[k] = pc.hi[k];
      }
      tb.push_back(b);
      ref_tri.push_back(pc.tri);
    }
  }
  const int64_t nr = int64_t(tb.size());
  if (nr >= kMaxReferences) {
    err = "too many triangle references";
    return false;
  }
  std::vector<float> cen(3 * nr);
  for (int64_t i = 0; i < nr; ++i)
    for (int k = 0; k < 3; ++k) cen[3 * i + k] = 0.5f * (tb[i].lo[k] + tb[i].hi[k]);
  std::vector<int32_t> perm(nr);
  for (int64_t i = 0; i < nr; ++i) perm[i] = int32_t(i);

  // ---- binned SAH binary tree ----
  std::vector<Node2> n2;
  n2.reserve(2 * size_t(nr) / std::max(1, max_leaf) + 16);
  n2.emplace_back();
  struct Work { int32_t node, first, count; };
  std::vector<Work> work{{0, 0, int32_t(nr)}};
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
      if (k >= nk) {  // an inverted box: every slab test misses it
        node.lox[k] = node.loy[k] = node.loz[k] = std::numeric_limits<float>::infinity();
        node.hix[k] = node.hiy[k] = node.hiz[k] = -std::numeric_limits<float>::infinity();
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

  // ---- triangle records in leaf order (one per reference), three rotated copies ----
  out.n_refs = nr;
  out.tris.resize(3 * nr);
  for (int64_t i = 0; i < nr; ++i) {
    const int32_t t = ref_tri[perm[i]];
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
      out.tris[((kz + 1) % 3) * nr + i] = r;
    }
  }
  return true;
}

}  // namespace xp
