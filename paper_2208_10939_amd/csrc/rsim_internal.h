// Internal definitions shared by the host runtime and the gfx950 kernels of librsim.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rsim {

constexpr double kC0 = 299792458.0;  // speed of light, m/s
constexpr double kPi = 3.14159265358979323846;

// Segment-parameter window of a shadow ray [kTEps, 1 - kTEps]: an occluder counts
// only strictly between the facet centroid and the antenna phase centre.
constexpr float kTEps = 1e-6f;

constexpr int kMaxElements = 128;  // Tx + Rx elements
constexpr int kBvhStack = 96;      // traversal stack entries at most (3 per 4-wide level)
constexpr int kBvhMaxDepth = 60;   // binary levels at most (the builder caps them at 58)
constexpr int kLeafMax = 4;        // triangles per leaf (encoding allows 15)

// Two-wide BVH node: both child boxes live in the parent so one 64-byte fetch tests
// two boxes. Child ref >= 0: inner node index; < 0: leaf, -(1 + (first << 4 | count)).
struct alignas(16) BvhNode {
  float lo0[3], hi0[3];
  float lo1[3], hi1[3];
  int32_t c0, c1;
  int32_t pad0, pad1;
};
static_assert(sizeof(BvhNode) == 64, "node size");

// Four-wide node, the traversal's format (the binary tree collapsed: a node's children are
// its binary grandchildren, or a binary child that is a leaf): one 128-byte fetch tests four
// boxes, and a root-to-leaf chain of dependent fetches is half as long. Boxes as structure
// of arrays; unused slots hold an empty box (lo > hi) and an empty leaf.
struct alignas(16) BvhNode4 {
  float lo[3][4], hi[3][4];  // [axis][child]
  int32_t c[4];              // as BvhNode: >= 0 inner node, < 0 leaf
  int32_t pad[4];
};
static_assert(sizeof(BvhNode4) == 128, "node size");

// Leaf triangle in BVH order as three float4: (v0.xyz, e1.x) (e1.yz, e2.xy)
// (e2.z, id bits, 0, 0) with e1 = v1 - v0, e2 = v2 - v0 and id the mesh-local index.

// One rigid instance of a mesh in a scene (device copy).
struct DevInstance {
  double rot[9];   // row-major body -> world
  double pos0[3];  // world position of the body origin at t = 0
  double vel[3];   // world velocity
  double box_lo[3], box_hi[3];  // world box of rot * body box (add pos0 + vel t)
  const float *verts;           // [V][3] body frame
  const int32_t *tris;          // [F][3]
  const BvhNode4 *nodes;        // four-wide BVH, root = node 0
  const float4 *leaf;           // [n_leaf_tris * 3]
  int64_t facet_base;           // scene-global index of this instance's triangle 0
  int32_t n_tris;
  int32_t has_bvh;              // 0 if the mesh has no non-degenerate triangle
  int32_t in_plane;             // 1: lies in the reflecting ground plane (never blocks legs ending on it)
  int32_t flat;                 // 1: horizontal (world vertex heights within 2e-6 m), no vertical motion
  double flat_lo, flat_hi;      // lowest and highest world vertex height of a flat instance
};

// A value read-only for the rest of the kernel, at a wave-uniform address: loaded through
// the constant address space so that it lands in scalar registers (the compiler cannot
// otherwise prove that stores or atomics elsewhere in the kernel leave it unchanged).
template <typename T>
__device__ inline T load_uniform(const T *p) {
  static_assert(sizeof(T) % 4 == 0, "whole dwords");
  using CInt = const __attribute__((address_space(4))) int32_t;
  CInt *q = (CInt *)p;
  int32_t w[sizeof(T) / 4];
#pragma unroll
  for (int k = 0; k < static_cast<int>(sizeof(T) / 4); ++k) w[k] = q[k];
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

// Radar constants passed by value.
struct RadarConst {
  double f0, slope, fs, df, tc;  // df = slope / fs
  double tx_c[3], rx_c[3];       // phase centres (element means)
  int32_t M, N, P, Q;
  int32_t intra;   // 1: propagation delay at each sample time within the chirp
  int32_t bounce;  // 1: visibility also of the ground-reflected paths (four mask sets)
  double z_ground; // height of the reflecting ground plane
};

// Per-scene device view used by the visibility, compaction and echo kernels.
struct DevScene {
  const DevInstance *inst;
  int32_t n_inst;
  int32_t n_points;
  int64_t n_facets;
  int64_t mask_words;        // per chirp
  const double *pt_pos0;     // [n_points][3]
  const double *pt_vel;      // [n_points][3]
  const double *pt_amp;      // [n_points][2]
  uint32_t *mask;            // [N][mask_words]
  int32_t *vis_idx;          // [N][n_facets] compacted lit facets per chirp
  int32_t *vis_cnt;          // [N]
  void *echo;                // [O][N][M] complex
  int32_t stack_depth;       // traversal stack entries per thread (> deepest BVH level)
  // facet-to-facet double bounce (db_on = 1): per (end k, chirp n, facet A) the facet B
  // that A's reflected ray connects to or -1, the connected A per (k, n) in ascending
  // order and their counts; N = db_n chirps; gamma of the reflection
  int32_t db_on;
  const int32_t *db_b;       // [2][N][n_facets]
  const int32_t *db_idx;     // [2][N][n_facets]
  const int32_t *db_cnt;     // [2][N]
  double db_gamma_re, db_gamma_im;
  int32_t db_n, db_pad;
};

// Facet-sum entries of chirp n: its lit facets, the points, then (double bounce) the
// connections launched from the Tx side and from the Rx side.
__device__ inline int32_t entry_total(const DevScene &sc, int n) {
  int32_t e = sc.vis_cnt[n] + sc.n_points;
  if (sc.db_on) e += sc.db_cnt[n] + sc.db_cnt[sc.db_n + n];
  return e;
}

}  // namespace rsim
