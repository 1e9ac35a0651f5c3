// Host construction of the walk geometry: scene frame, binned-SAH binary
// tree, collapse to 4-wide nodes, breadth-first node order and leaf-order
// triangle records.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <limits>

#include "msk_internal.h"

namespace msk {
namespace {

struct Box {
  float lo[3], hi[3];
  void reset() {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::numeric_limits<float>::infinity();
      hi[k] = -std::numeric_limits<float>::infinity();
    }
  }
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  double area() const {
    double d[3];
    for (int k = 0; k < 3; ++k) d[k] = std::max(0.0, (double)hi[k] - (double)lo[k]);
    return 2.0 * (d[0] * d[1] + d[1] * d[2] + d[2] * d[0]);
  }
};

struct BNode {  // binary node
  Box box;
  int32_t left = -1, right = -1;  // children (inner)
  int32_t first = 0, count = 0;   // leaf range in the triangle order
};

struct Builder {
  const std::vector<Box>& tb;
  const std::vector<float>& cen;  // n x 3 centroids
  std::vector<int32_t>& order;
  std::vector<BNode> nodes;
  int leaf_size;

  Builder(const std::vector<Box>& tb_, const std::vector<float>& cen_, std::vector<int32_t>& order_, int leaf)
      : tb(tb_), cen(cen_), order(order_), leaf_size(leaf) {}

  int32_t make_leaf(int32_t first, int32_t count, const Box& b) {
    BNode n;
    n.box = b;
    n.first = first;
    n.count = count;
    nodes.push_back(n);
    return (int32_t)nodes.size() - 1;
  }

  // Iterative build with an explicit work stack.
  void build(int32_t n) {
    struct Item { int32_t first, count, parent; bool is_left; };
    std::vector<Item> stack;
    stack.push_back({0, n, -1, false});
    constexpr int kBins = 16;
    while (!stack.empty()) {
      Item it = stack.back();
      stack.pop_back();
      Box b, cb;
      b.reset();
      cb.reset();
      for (int32_t i = it.first; i < it.first + it.count; ++i) {
        int32_t t = order[i];
        b.grow(tb[t]);
        for (int k = 0; k < 3; ++k) {
          cb.lo[k] = std::min(cb.lo[k], cen[3 * t + k]);
          cb.hi[k] = std::max(cb.hi[k], cen[3 * t + k]);
        }
      }
      int32_t id;
      bool split = it.count > leaf_size;
      int best_axis = -1, best_bin = -1;
      double best_cost = std::numeric_limits<double>::infinity();
      if (split) {
        for (int ax = 0; ax < 3; ++ax) {
          double ext = (double)cb.hi[ax] - (double)cb.lo[ax];
          if (!(ext > 0)) continue;
          Box bins[kBins];
          int32_t cnt[kBins] = {0};
          for (auto& x : bins) x.reset();
          double scale = kBins / ext;
          for (int32_t i = it.first; i < it.first + it.count; ++i) {
            int32_t t = order[i];
            int bi = std::min(kBins - 1, (int)((cen[3 * t + ax] - cb.lo[ax]) * scale));
            cnt[bi]++;
            bins[bi].grow(tb[t]);
          }
          Box lb[kBins];
          int32_t lc[kBins];
          Box acc;
          acc.reset();
          int32_t c = 0;
          for (int i = 0; i < kBins; ++i) {
            acc.grow(bins[i]);
            c += cnt[i];
            lb[i] = acc;
            lc[i] = c;
          }
          acc.reset();
          c = 0;
          for (int i = kBins - 1; i > 0; --i) {
            acc.grow(bins[i]);
            c += cnt[i];
            if (lc[i - 1] == 0 || c == 0) continue;
            double cost = lb[i - 1].area() * lc[i - 1] + acc.area() * c;
            if (cost < best_cost) {
              best_cost = cost;
              best_axis = ax;
              best_bin = i;
            }
          }
        }
      }
      int32_t mid = -1;
      if (split && best_axis >= 0) {
        double ext = (double)cb.hi[best_axis] - (double)cb.lo[best_axis];
        double scale = kBins / ext;
        auto part = std::partition(order.begin() + it.first, order.begin() + it.first + it.count, [&](int32_t t) {
          int bi = std::min(kBins - 1, (int)((cen[3 * t + best_axis] - cb.lo[best_axis]) * scale));
          return bi < best_bin;
        });
        mid = (int32_t)(part - order.begin());
        if (mid == it.first || mid == it.first + it.count) mid = -1;
      }
      if (split && mid < 0) {  // coincident centroids: split the range in half
        mid = it.first + it.count / 2;
      }
      if (!split) {
        id = make_leaf(it.first, it.count, b);
      } else {
        BNode nd;
        nd.box = b;
        nodes.push_back(nd);
        id = (int32_t)nodes.size() - 1;
        stack.push_back({mid, it.first + it.count - mid, id, false});
        stack.push_back({it.first, mid - it.first, id, true});
      }
      if (it.parent >= 0) {
        if (it.is_left) nodes[it.parent].left = id;
        else nodes[it.parent].right = id;
      }
    }
  }
};

}  // namespace

std::string build_bvh_boxes(const std::vector<Box3f>& boxes, const std::vector<float>& cen, int leaf_size,
                            std::vector<Node4>& nodes_out, std::vector<int32_t>& leaf_order, int& depth) {
  if (boxes.empty()) return "no elements";
  if (leaf_size < 1 || leaf_size > 8) return "leaf_size must be in 1..8";
  std::vector<Box> tb(boxes.size());
  for (size_t i = 0; i < boxes.size(); ++i)
    for (int k = 0; k < 3; ++k) {
      tb[i].lo[k] = boxes[i].lo[k];
      tb[i].hi[k] = boxes[i].hi[k];
    }
  const int64_t nf = (int64_t)tb.size();
  std::vector<int32_t> order((size_t)nf);
  for (int64_t i = 0; i < nf; ++i) order[i] = (int32_t)i;
  Builder bld(tb, cen, order, leaf_size);
  bld.nodes.reserve((size_t)(2 * nf / std::max(1, leaf_size) + 8));
  bld.build((int32_t)nf);
  const std::vector<BNode>& bn = bld.nodes;

  // Collapse to 4-wide nodes, breadth first. Each wide node gathers up to
  // four binary descendants by repeatedly opening the largest inner child.
  struct WItem { int32_t bin; int32_t depth; };
  std::vector<WItem> queue;
  nodes_out.clear();
  std::vector<int32_t> wide_of;  // queue index == wide node index
  queue.push_back({0, 1});
  size_t head = 0;
  int maxdepth = 0;
  std::vector<int32_t> leaf_first, leaf_count;
  // leaf order assigned in BFS order of leaves
  leaf_order.clear();
  leaf_order.reserve((size_t)nf);
  while (head < queue.size()) {
    WItem it = queue[head++];
    maxdepth = std::max(maxdepth, it.depth);
    Node4 w;
    for (int k = 0; k < 4; ++k) {
      w.lox[k] = w.loy[k] = w.loz[k] = INFINITY;
      w.hix[k] = w.hiy[k] = w.hiz[k] = -INFINITY;
      w.child[k] = INT32_MIN;
      w.count[k] = 0;
    }
    int32_t kids[4];
    int nk = 0;
    const BNode& root = bn[it.bin];
    if (root.left < 0) {
      kids[nk++] = it.bin;  // whole tree is a single leaf
    } else {
      kids[nk++] = root.left;
      kids[nk++] = root.right;
      while (nk < 4) {
        int best = -1;
        double ba = -1;
        for (int k = 0; k < nk; ++k)
          if (bn[kids[k]].left >= 0 && bn[kids[k]].box.area() > ba) {
            ba = bn[kids[k]].box.area();
            best = k;
          }
        if (best < 0) break;
        int32_t b = kids[best];
        kids[best] = bn[b].left;
        kids[nk++] = bn[b].right;
      }
    }
    for (int k = 0; k < nk; ++k) {
      const BNode& c = bn[kids[k]];
      w.lox[k] = c.box.lo[0]; w.loy[k] = c.box.lo[1]; w.loz[k] = c.box.lo[2];
      w.hix[k] = c.box.hi[0]; w.hiy[k] = c.box.hi[1]; w.hiz[k] = c.box.hi[2];
      if (c.left < 0) {
        int32_t first = (int32_t)leaf_order.size();
        for (int32_t i = c.first; i < c.first + c.count; ++i) leaf_order.push_back(order[i]);
        w.child[k] = -first - 1;
        w.count[k] = c.count;
      } else {
        w.child[k] = (int32_t)queue.size();
        queue.push_back({kids[k], it.depth + 1});
      }
    }
    nodes_out.push_back(w);
  }
  depth = maxdepth;
  if (leaf_order.size() != tb.size()) return "internal error: element count mismatch";
  // traversal stack: at most 3 pending siblings per level (with margin)
  if (3 * maxdepth + 5 > kStackDepth) return "BVH too deep for the traversal stack";
  return "";
}

std::string build_bvh_host(const float* V, int64_t nv, const int32_t* F, int64_t nf, int leaf_size, HostBvh& out) {
  if (nv < 3 || nf < 1) return "mesh needs at least 3 vertices and 1 triangle";
  // the walk kernel packs a triangle slot and a lane into one 32-bit word
  if (nf >= (int64_t)1 << 26) return "too many triangles (a mesh holds at most 2^26 - 1)";
  if (leaf_size < 1 || leaf_size > 8) return "leaf_size must be in 1..8";
  out.leaf_size = leaf_size;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) {
      double x = V[3 * i + k];
      if (!std::isfinite(x)) return "vertex coordinates must be finite";
      lo[k] = std::min(lo[k], x);
      hi[k] = std::max(hi[k], x);
    }
  for (int k = 0; k < 3; ++k) out.centre[k] = 0.5 * (lo[k] + hi[k]);
  double r2 = 0;
  for (int64_t i = 0; i < nv; ++i) {
    double d0 = V[3 * i] - out.centre[0], d1 = V[3 * i + 1] - out.centre[1], d2 = V[3 * i + 2] - out.centre[2];
    r2 = std::max(r2, d0 * d0 + d1 * d1 + d2 * d2);
  }
  out.radius = (1.0 + std::ldexp(1.0, -20)) * std::sqrt(r2);
  std::vector<float> Vr((size_t)nv * 3);
  for (int64_t i = 0; i < nv; ++i)
    for (int k = 0; k < 3; ++k) Vr[3 * i + k] = (float)((double)V[3 * i + k] - out.centre[k]);

  std::vector<Box3f> tb((size_t)nf);
  std::vector<float> cen((size_t)nf * 3);
  double area = 0;
  for (int64_t t = 0; t < nf; ++t) {
    for (int k = 0; k < 3; ++k) {
      tb[t].lo[k] = std::numeric_limits<float>::infinity();
      tb[t].hi[k] = -std::numeric_limits<float>::infinity();
    }
    double c[3] = {0, 0, 0}, P[3][3];
    for (int j = 0; j < 3; ++j) {
      int64_t v = F[3 * t + j];
      if (v < 0 || v >= nv) return "face index out of range";
      for (int k = 0; k < 3; ++k) {
        float x = Vr[3 * v + k];
        tb[t].lo[k] = std::min(tb[t].lo[k], x);
        tb[t].hi[k] = std::max(tb[t].hi[k], x);
        c[k] += x;
        P[j][k] = V[3 * v + k];
      }
    }
    for (int k = 0; k < 3; ++k) cen[3 * t + k] = (float)(c[k] / 3.0);
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = P[1][k] - P[0][k];
      e2[k] = P[2][k] - P[0][k];
    }
    double cx = e1[1] * e2[2] - e1[2] * e2[1], cy = e1[2] * e2[0] - e1[0] * e2[2], cz = e1[0] * e2[1] - e1[1] * e2[0];
    area += 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
  }
  if (!(area > 0)) return "mesh has zero total area";
  out.area = area;

  std::vector<int32_t> leaf_order;
  std::string err = build_bvh_boxes(tb, cen, leaf_size, out.nodes, leaf_order, out.depth);
  if (!err.empty()) return err;
  std::vector<TriRec> tris(leaf_order.size());
  out.slot_of_tri.assign((size_t)nf, -1);
  for (size_t slot = 0; slot < leaf_order.size(); ++slot) {
    const int32_t t = leaf_order[slot];
    TriRec r;
    const int32_t* f = F + 3 * (int64_t)t;
    r.a = make_float4(Vr[3 * f[0]], Vr[3 * f[0] + 1], Vr[3 * f[0] + 2], 0.f);
    r.b = make_float4(Vr[3 * f[1]], Vr[3 * f[1] + 1], Vr[3 * f[1] + 2], 0.f);
    r.c = make_float4(Vr[3 * f[2]], Vr[3 * f[2] + 1], Vr[3 * f[2] + 2], 0.f);
    int32_t ti = t;
    std::memcpy(&r.a.w, &ti, 4);
    out.slot_of_tri[t] = (int32_t)slot;
    tris[slot] = r;
  }
  out.tris.swap(tris);
  if ((int64_t)out.tris.size() != nf) return "internal error: triangle count mismatch";
  return "";
}

}  // namespace msk
