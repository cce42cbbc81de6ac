// Host-side binned-SAH BVH builder for one mesh in its body frame.
//
// Visibility of a facet (single-bounce reading of the bidirectional ray tracing of
// Section 2.2) needs "any triangle blocks this segment" queries for every facet and
// chirp. Meshes are rigid, so each is indexed once at load time in its body frame
// and rays are moved into that frame per instance and chirp.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

#include "rsim_internal.h"

namespace rsim {

struct BuildPrim {
  float lo[3], hi[3], c[3];
  int32_t id;
};

struct Box {
  float lo[3] = {std::numeric_limits<float>::infinity(), std::numeric_limits<float>::infinity(),
                 std::numeric_limits<float>::infinity()};
  float hi[3] = {-std::numeric_limits<float>::infinity(), -std::numeric_limits<float>::infinity(),
                 -std::numeric_limits<float>::infinity()};
  void grow(const float *l, const float *h) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], l[k]);
      hi[k] = std::max(hi[k], h[k]);
    }
  }
  void grow_pt(const float *p) { grow(p, p); }
  bool empty() const { return !(lo[0] <= hi[0]); }
  double area() const {
    if (empty()) return 0.0;
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct Builder {
  std::vector<BuildPrim> prims;
  std::vector<BvhNode> nodes;
  std::vector<int32_t> order;
  int max_depth = 0;

  static int32_t leaf_ref(int64_t first, int64_t count) {
    return -(1 + static_cast<int32_t>((first << 4) | count));
  }

  Box bounds(int64_t b, int64_t e) const {
    Box bx;
    for (int64_t i = b; i < e; ++i) bx.grow(prims[i].lo, prims[i].hi);
    return bx;
  }

  int32_t make_leaf(int64_t b, int64_t e) {
    int64_t first = static_cast<int64_t>(order.size());
    for (int64_t i = b; i < e; ++i) order.push_back(prims[i].id);
    return leaf_ref(first, e - b);
  }

  // Builds the subtree over prims[b, e), returns its child ref; box = its bounds.
  int32_t build(int64_t b, int64_t e, int depth, Box &box) {
    box = bounds(b, e);
    max_depth = std::max(max_depth, depth);
    const int64_t n = e - b;
    if (n <= kLeafMax) return make_leaf(b, e);
    Box cb;
    for (int64_t i = b; i < e; ++i) cb.grow_pt(prims[i].c);
    constexpr int kBins = 16;
    double best_cost = std::numeric_limits<double>::infinity();
    int best_axis = -1, best_split = -1;
    for (int ax = 0; ax < 3; ++ax) {
      float ext = cb.hi[ax] - cb.lo[ax];
      if (!(ext > 0.0f)) continue;
      Box bin_box[kBins];
      int64_t bin_n[kBins] = {0};
      for (int64_t i = b; i < e; ++i) {
        int k = static_cast<int>(kBins * ((prims[i].c[ax] - cb.lo[ax]) / ext));
        k = std::min(std::max(k, 0), kBins - 1);
        bin_n[k]++;
        bin_box[k].grow(prims[i].lo, prims[i].hi);
      }
      double right_area[kBins];
      int64_t right_n[kBins];
      Box acc;
      int64_t cnt = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bin_box[k].lo, bin_box[k].hi);
        cnt += bin_n[k];
        right_area[k] = acc.area();
        right_n[k] = cnt;
      }
      Box lacc;
      int64_t lcnt = 0;
      for (int k = 1; k < kBins; ++k) {
        lacc.grow(bin_box[k - 1].lo, bin_box[k - 1].hi);
        lcnt += bin_n[k - 1];
        if (lcnt == 0 || right_n[k] == 0) continue;
        double cost = lacc.area() * lcnt + right_area[k] * right_n[k];
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = ax;
          best_split = k;
        }
      }
    }
    int64_t mid;
    if (best_axis >= 0 && depth < 32) {  // median splits below keep depth <= 32 + 26
      float ext = cb.hi[best_axis] - cb.lo[best_axis];
      auto it = std::partition(prims.begin() + b, prims.begin() + e, [&](const BuildPrim &p) {
        int k = static_cast<int>(kBins * ((p.c[best_axis] - cb.lo[best_axis]) / ext));
        k = std::min(std::max(k, 0), kBins - 1);
        return k < best_split;
      });
      mid = it - prims.begin();
    } else {
      mid = b;  // fall through to the median split below
    }
    if (mid <= b || mid >= e) {
      // median split on the widest centroid axis (degenerate or deep subtrees)
      int ax = 0;
      float ext = -1.0f;
      for (int k = 0; k < 3; ++k)
        if (cb.hi[k] - cb.lo[k] > ext) {
          ext = cb.hi[k] - cb.lo[k];
          ax = k;
        }
      mid = b + n / 2;
      std::nth_element(prims.begin() + b, prims.begin() + mid, prims.begin() + e,
                       [ax](const BuildPrim &p, const BuildPrim &q) { return p.c[ax] < q.c[ax]; });
    }
    int32_t me = static_cast<int32_t>(nodes.size());
    nodes.emplace_back();
    Box lb, rb;
    int32_t l = build(b, mid, depth + 1, lb);
    int32_t r = build(mid, e, depth + 1, rb);
    BvhNode &nd = nodes[me];
    std::memset(&nd, 0, sizeof(nd));
    for (int k = 0; k < 3; ++k) {
      nd.lo0[k] = lb.lo[k];
      nd.hi0[k] = lb.hi[k];
      nd.lo1[k] = rb.lo[k];
      nd.hi1[k] = rb.hi[k];
    }
    nd.c0 = l;
    nd.c1 = r;
    return me;
  }
};

// Inflate a box so FP32 slab tests stay conservative (a box that is slightly too
// large costs time, never a missed occluder).
static void inflate(float *lo, float *hi) {
  for (int k = 0; k < 3; ++k) {
    if (!(lo[k] <= hi[k])) continue;
    float pad = 1e-5f * (std::fabs(lo[k]) + std::fabs(hi[k]) + (hi[k] - lo[k])) + 1e-6f;
    lo[k] -= pad;
    hi[k] += pad;
  }
}

// Four-wide node `n4` from binary node n: its children are the two children of each inner
// binary child (with the boxes that child holds) or the binary child itself when it is a
// leaf; inner ones are collapsed in turn. Returns the four-wide index; *depth the deepest
// four-wide level below (root level 0).
static int32_t collapse(const std::vector<BvhNode> &bin, int32_t n, int level,
                        std::vector<BvhNode4> &out, int *depth) {
  *depth = std::max(*depth, level);
  const int32_t me = static_cast<int32_t>(out.size());
  out.emplace_back();
  BvhNode4 nd;
  std::memset(&nd, 0, sizeof(nd));
  int ne = 0;
  auto put = [&](int32_t ref, const float *lo, const float *hi) {
    for (int k = 0; k < 3; ++k) {
      nd.lo[k][ne] = lo[k];
      nd.hi[k][ne] = hi[k];
    }
    nd.c[ne++] = ref;
  };
  const BvhNode &b = bin[n];
  for (int side = 0; side < 2; ++side) {
    const int32_t ref = side ? b.c1 : b.c0;
    if (ref >= 0) {
      const BvhNode &g = bin[ref];
      put(g.c0, g.lo0, g.hi0);
      put(g.c1, g.lo1, g.hi1);
    } else {
      put(ref, side ? b.lo1 : b.lo0, side ? b.hi1 : b.hi0);
    }
  }
  for (; ne < 4; ++ne) {  // empty slots: never entered
    for (int k = 0; k < 3; ++k) {
      nd.lo[k][ne] = 1.0f;
      nd.hi[k][ne] = -1.0f;
    }
    nd.c[ne] = Builder::leaf_ref(0, 0);
  }
  for (int i = 0; i < 4; ++i)
    if (nd.c[i] >= 0) nd.c[i] = collapse(bin, nd.c[i], level + 1, out, depth);
  out[me] = nd;
  return me;
}

// Builds the four-wide nodes (root = node 0) and leaf triangles (3 float4 each).
// Degenerate (zero-area) triangles are left out: they never block. Returns the depth of the
// four-wide tree (root 0), or -1 if no triangle has area.
int build_bvh(const float *verts, const int32_t *tris, int64_t n_tris,
              std::vector<BvhNode4> &nodes_out, std::vector<float> &leaf_out) {
  Builder bd;
  bd.prims.reserve(n_tris);
  for (int64_t t = 0; t < n_tris; ++t) {
    const float *a = verts + 3 * tris[3 * t + 0];
    const float *b = verts + 3 * tris[3 * t + 1];
    const float *c = verts + 3 * tris[3 * t + 2];
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
      e1[k] = double(b[k]) - a[k];
      e2[k] = double(c[k]) - a[k];
    }
    double nx = e1[1] * e2[2] - e1[2] * e2[1];
    double ny = e1[2] * e2[0] - e1[0] * e2[2];
    double nz = e1[0] * e2[1] - e1[1] * e2[0];
    if (nx == 0.0 && ny == 0.0 && nz == 0.0) continue;
    BuildPrim p;
    for (int k = 0; k < 3; ++k) {
      p.lo[k] = std::min(a[k], std::min(b[k], c[k]));
      p.hi[k] = std::max(a[k], std::max(b[k], c[k]));
      p.c[k] = (a[k] + b[k] + c[k]) / 3.0f;
    }
    p.id = static_cast<int32_t>(t);
    bd.prims.push_back(p);
  }
  nodes_out.clear();
  leaf_out.clear();
  if (bd.prims.empty()) return -1;
  const int64_t np = static_cast<int64_t>(bd.prims.size());
  bd.order.reserve(np);
  bd.nodes.reserve(2 * np / kLeafMax + 2);
  if (np <= kLeafMax) {
    // root with one leaf child and one empty child
    bd.nodes.emplace_back();
    Box lb;
    int32_t l = bd.build(0, np, 1, lb);
    BvhNode &nd = bd.nodes[0];
    std::memset(&nd, 0, sizeof(nd));
    for (int k = 0; k < 3; ++k) {
      nd.lo0[k] = lb.lo[k];
      nd.hi0[k] = lb.hi[k];
      nd.lo1[k] = 1.0f;   // empty box: lo > hi never hits
      nd.hi1[k] = -1.0f;
    }
    nd.c0 = l;
    nd.c1 = Builder::leaf_ref(0, 0);
  } else {
    Box root;
    bd.build(0, np, 0, root);
  }
  for (auto &nd : bd.nodes) {
    inflate(nd.lo0, nd.hi0);
    inflate(nd.lo1, nd.hi1);
  }
  nodes_out.reserve(bd.nodes.size() / 2 + 1);
  int depth4 = 0;
  collapse(bd.nodes, 0, 0, nodes_out, &depth4);
  leaf_out.resize(bd.order.size() * 12);
  for (size_t i = 0; i < bd.order.size(); ++i) {
    int32_t t = bd.order[i];
    const float *a = verts + 3 * tris[3 * t + 0];
    const float *b = verts + 3 * tris[3 * t + 1];
    const float *c = verts + 3 * tris[3 * t + 2];
    float *o = leaf_out.data() + 12 * i;
    o[0] = a[0]; o[1] = a[1]; o[2] = a[2];
    o[3] = b[0] - a[0]; o[4] = b[1] - a[1]; o[5] = b[2] - a[2];
    o[6] = c[0] - a[0]; o[7] = c[1] - a[1]; o[8] = c[2] - a[2];
    std::memcpy(&o[9], &t, sizeof(int32_t));
    o[10] = 0.0f;
    o[11] = 0.0f;
  }
  return depth4;
}

}  // namespace rsim
