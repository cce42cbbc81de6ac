// Lit-facet mask per chirp and its compaction into per-chirp facet lists.
//
// Single-bounce reading of bidirectional analytic ray tracing (Section 2.2): a
// forward ray from the transmitter and a backward ray from the receiver meet on the
// same facet. Facet f is lit at chirp n when it faces both phase centres and
// neither segment centroid -> phase centre is blocked by another triangle. The
// geometry is that of chirp start t_n (stop-and-hop, eq. (12) per chirp).
//
// Layout: a workgroup per (32 or more facets, up to 64 chirps), lane = chirp. The facing test
// runs in FP64 on world coordinates; the two shadow rays run in FP32 in each
// candidate instance's body frame, starting at the facet centroid (close to the
// occluders, so the FP32 Moller-Trumbore test keeps its precision). Each thread
// owns a column of an LDS stack (stride = block size, conflict-free) as deep as the
// scene's deepest BVH, which sets how many waves share a CU.
#include <algorithm>

#include "rsim_internal.h"
#include "rsim_launch.h"

namespace rsim {

namespace {

constexpr int kVisThreads = 256;
constexpr int kVisFilterFacets = 32;  // facets per workgroup with 64 chirps per group
constexpr int kVisBitWords = 4 * 64;  // LDS bit words: path types x chirps x mask words

__device__ inline int find_instance(const DevInstance *inst, int n_inst, int64_t f) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (inst[mid].facet_base <= f)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ inline bool box_hit(const float *lo, const float *hi, float ox, float oy, float oz,
                               float ix, float iy, float iz, float pad = 0.0f) {
  float tx0 = (lo[0] - pad - ox) * ix, tx1 = (hi[0] + pad - ox) * ix;
  float ty0 = (lo[1] - pad - oy) * iy, ty1 = (hi[1] + pad - oy) * iy;
  float tz0 = (lo[2] - pad - oz) * iz, tz1 = (hi[2] + pad - oz) * iz;
  float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
  float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), 1.0f));
  return tn <= tf;
}

// Any triangle of the leaf hit by o + t d, t in [kTEps, 1 - kTEps] (closed test)?
__device__ inline bool leaf_hit(const float4 *leaf, int32_t ref, float ox, float oy, float oz,
                                float dx, float dy, float dz, int32_t skip) {
  uint32_t code = static_cast<uint32_t>(-ref - 1);
  uint32_t first = code >> 4, count = code & 15u;
  for (uint32_t k = 0; k < count; ++k) {
    const float4 a = leaf[3 * (first + k) + 0];
    const float4 b = leaf[3 * (first + k) + 1];
    const float4 c = leaf[3 * (first + k) + 2];
    if (__float_as_int(c.y) == skip) continue;
    // v0 = a.xyz, e1 = (a.w, b.x, b.y), e2 = (b.z, b.w, c.x)
    float e1x = a.w, e1y = b.x, e1z = b.y;
    float e2x = b.z, e2y = b.w, e2z = c.x;
    float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    float det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0f) continue;
    float inv = 1.0f / det;
    float sx = ox - a.x, sy = oy - a.y, sz = oz - a.z;
    float u = (sx * px + sy * py + sz * pz) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) continue;
    float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    float v = (dx * qx + dy * qy + dz * qz) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) continue;
    float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
    if (t >= kTEps && t <= 1.0f - kTEps) return true;
  }
  return false;
}

__device__ inline float safe_inv(float d) {
  const float tiny = 1e-30f;
  return 1.0f / (fabsf(d) > tiny ? d : copysignf(tiny, d));
}

// Any-hit traversal of one four-wide BLAS for the body-frame segment o -> o + d: leaves
// are tested when their box is hit, the first hit inner child is entered next and the other
// hit inner children (at most three per level) wait on the stack.
__device__ bool blas_occluded(const BvhNode4 *nodes, const float4 *leaf, float ox, float oy,
                              float oz, float dx, float dy, float dz, int32_t skip,
                              int32_t *stack, int stride) {
  const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const BvhNode4 nd = nodes[node];
    int32_t next = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float lo[3] = {nd.lo[0][i], nd.lo[1][i], nd.lo[2][i]};
      const float hi[3] = {nd.hi[0][i], nd.hi[1][i], nd.hi[2][i]};
      if (!box_hit(lo, hi, ox, oy, oz, ix, iy, iz)) continue;
      const int32_t c = nd.c[i];
      if (c < 0) {
        if (leaf_hit(leaf, c, ox, oy, oz, dx, dy, dz, skip)) return true;
      } else if (next >= 0) {
        stack[sp * stride] = c;  // <= 3 per level: stack_depth = 3 (depth + 1)
        ++sp;
      } else {
        next = c;
      }
    }
    if (next < 0) {
      if (sp == 0) return false;
      --sp;
      next = stack[sp * stride];
    }
    node = next;
  }
}

// A flat (horizontal) instance cannot block the segment c -> s: c lies no lower than its
// lowest vertex and at most 0.5e-6 m below its highest, and s lies at least 1 m above c,
// so for t >= kTEps the segment runs at least 0.5e-6 m above every vertex (a ground facet's
// rays towards the array leave the road grid's BVH untouched).
__device__ inline bool flat_below(const DevInstance &I, const double c[3], double s_z) {
  return I.flat && c[2] >= I.flat_lo && I.flat_hi - c[2] <= 0.5e-6 && s_z - c[2] >= 1.0;
}

// Is the world segment c -> s blocked by any triangle of the scene at time t
// (triangle `self_local` of instance `self_inst` excluded)?
__device__ bool segment_blocked(const DevScene &sc, double t, const double c[3],
                                const double s[3], int self_inst, int32_t self_local,
                                int32_t *stack, int stride, bool skip_plane = false,
                                uint64_t cand = ~uint64_t(0)) {
  double d[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
  // reciprocals once per segment (the boxes are padded, so the rounding of a product
  // instead of a quotient cannot turn a hit box into a miss)
  const double id[3] = {d[0] != 0.0 ? 1.0 / d[0] : 0.0, d[1] != 0.0 ? 1.0 / d[1] : 0.0,
                        d[2] != 0.0 ? 1.0 / d[2] : 0.0};
  for (int j = 0; j < sc.n_inst; ++j) {
    if (j < 64 && !((cand >> j) & 1u)) continue;  // no segment of the wave meets its box
    const DevInstance &I = sc.inst[j];
    if (!I.has_bvh) continue;
    if (skip_plane && I.in_plane) continue;  // the road surface under a reflected leg
    if (flat_below(I, c, s[2])) continue;
    double p[3] = {I.pos0[0] + I.vel[0] * t, I.pos0[1] + I.vel[1] * t, I.pos0[2] + I.vel[2] * t};
    // world-space slab test against the instance box (FP64, conservative box)
    double tn = 0.0, tf = 1.0;
    bool miss = false;
    for (int k = 0; k < 3; ++k) {
      double lo = I.box_lo[k] + p[k], hi = I.box_hi[k] + p[k];
      if (d[k] == 0.0) {
        if (c[k] < lo || c[k] > hi) miss = true;
        continue;
      }
      double a = (lo - c[k]) * id[k], b = (hi - c[k]) * id[k];
      tn = fmax(tn, fmin(a, b));
      tf = fmin(tf, fmax(a, b));
    }
    if (miss || tn > tf) continue;
    // body frame: x_body = R^T (x - p)
    const double *R = I.rot;
    double q0 = c[0] - p[0], q1 = c[1] - p[1], q2 = c[2] - p[2];
    float ox = static_cast<float>(R[0] * q0 + R[3] * q1 + R[6] * q2);
    float oy = static_cast<float>(R[1] * q0 + R[4] * q1 + R[7] * q2);
    float oz = static_cast<float>(R[2] * q0 + R[5] * q1 + R[8] * q2);
    float dx = static_cast<float>(R[0] * d[0] + R[3] * d[1] + R[6] * d[2]);
    float dy = static_cast<float>(R[1] * d[0] + R[4] * d[1] + R[7] * d[2]);
    float dz = static_cast<float>(R[2] * d[0] + R[5] * d[1] + R[8] * d[2]);
    int32_t skip = (j == self_inst) ? self_local : -1;
    if (blas_occluded(I.nodes, I.leaf, ox, oy, oz, dx, dy, dz, skip, stack, stride)) return true;
  }
  return false;
}

// Any triangle of the leaf hit by o + t d1 or o + t d2, t in [kTEps, 1 - kTEps]?
__device__ inline bool leaf_hit2(const float4 *leaf, int32_t ref, float ox, float oy, float oz,
                                 const float d[2][3], int32_t skip) {
  uint32_t code = static_cast<uint32_t>(-ref - 1);
  uint32_t first = code >> 4, count = code & 15u;
  for (uint32_t k = 0; k < count; ++k) {
    const float4 a = leaf[3 * (first + k) + 0];
    const float4 b = leaf[3 * (first + k) + 1];
    const float4 c = leaf[3 * (first + k) + 2];
    if (__float_as_int(c.y) == skip) continue;
    const float e1x = a.w, e1y = b.x, e1z = b.y;
    const float e2x = b.z, e2y = b.w, e2z = c.x;
    const float sx = ox - a.x, sy = oy - a.y, sz = oz - a.z;
    const float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const float dx = d[r][0], dy = d[r][1], dz = d[r][2];
      const float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
      const float det = e1x * px + e1y * py + e1z * pz;
      if (det == 0.0f) continue;
      const float inv = 1.0f / det;
      const float u = (sx * px + sy * py + sz * pz) * inv;
      if (!(u >= 0.0f && u <= 1.0f)) continue;
      const float v = (dx * qx + dy * qy + dz * qz) * inv;
      if (!(v >= 0.0f && u + v <= 1.0f)) continue;
      const float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
      if (t >= kTEps && t <= 1.0f - kTEps) return true;
    }
  }
  return false;
}

// Any-hit traversal of one BLAS for the two body-frame segments o -> o + d1 and
// o -> o + d2 together, so the two nearly parallel shadow rays of a facet share every
// node fetch. A node is entered when the first segment meets its box grown by
// |d1 - d2| on every side: the points of the two segments at the same parameter are at
// most that far apart, so this enters every node either segment meets (and a few more);
// the leaf tests are exact for both segments.
__device__ bool blas_occluded2(const BvhNode4 *nodes, const float4 *leaf, float ox, float oy,
                               float oz, const float d[2][3], int32_t skip, int32_t *stack,
                               int stride) {
  const float ix = safe_inv(d[0][0]), iy = safe_inv(d[0][1]), iz = safe_inv(d[0][2]);
  const float ex = d[0][0] - d[1][0], ey = d[0][1] - d[1][1], ez = d[0][2] - d[1][2];
  // |d1 - d2| rounded up (FP32 sqrt is correctly rounded; the factor covers the rest)
  const float pad = __builtin_sqrtf(ex * ex + ey * ey + ez * ez) * 1.0001f + 1e-7f;
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const BvhNode4 nd = nodes[node];
    int32_t next = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float lo[3] = {nd.lo[0][i], nd.lo[1][i], nd.lo[2][i]};
      const float hi[3] = {nd.hi[0][i], nd.hi[1][i], nd.hi[2][i]};
      if (!box_hit(lo, hi, ox, oy, oz, ix, iy, iz, pad)) continue;
      const int32_t c = nd.c[i];
      if (c < 0) {
        if (leaf_hit2(leaf, c, ox, oy, oz, d, skip)) return true;
      } else if (next >= 0) {
        stack[sp * stride] = c;  // <= 3 per level: stack_depth = 3 (depth + 1)
        ++sp;
      } else {
        next = c;
      }
    }
    if (next < 0) {
      if (sp == 0) return false;
      --sp;
      next = stack[sp * stride];
    }
    node = next;
  }
}

// Is either world segment c -> s1 or c -> s2 blocked by a triangle of the scene at time t
// (triangle `self_local` of instance `self_inst` excluded)? Same decisions as two calls
// of segment_blocked joined by "or".
__device__ bool pair_blocked(const DevScene &sc, double t, const double c[3], const double s1[3],
                             const double s2[3], int self_inst, int32_t self_local,
                             int32_t *stack, int stride, uint64_t cand) {
  const double dw[2][3] = {{s1[0] - c[0], s1[1] - c[1], s1[2] - c[2]},
                           {s2[0] - c[0], s2[1] - c[1], s2[2] - c[2]}};
  double idw[2][3];  // reciprocals once per segment, as in segment_blocked
  for (int r = 0; r < 2; ++r)
    for (int k = 0; k < 3; ++k) idw[r][k] = dw[r][k] != 0.0 ? 1.0 / dw[r][k] : 0.0;
  for (int j = 0; j < sc.n_inst; ++j) {
    if (j < 64 && !((cand >> j) & 1u)) continue;  // no segment of the wave meets its box
    const DevInstance &I = sc.inst[j];
    if (!I.has_bvh) continue;
    if (flat_below(I, c, s1[2]) && flat_below(I, c, s2[2])) continue;
    double p[3] = {I.pos0[0] + I.vel[0] * t, I.pos0[1] + I.vel[1] * t, I.pos0[2] + I.vel[2] * t};
    // world-space slab test of each segment against the instance box (FP64)
    bool any = false;
    for (int r = 0; r < 2; ++r) {
      double tn = 0.0, tf = 1.0;
      bool miss = false;
      for (int k = 0; k < 3; ++k) {
        double lo = I.box_lo[k] + p[k], hi = I.box_hi[k] + p[k];
        if (dw[r][k] == 0.0) {
          if (c[k] < lo || c[k] > hi) miss = true;
          continue;
        }
        double a = (lo - c[k]) * idw[r][k], b = (hi - c[k]) * idw[r][k];
        tn = fmax(tn, fmin(a, b));
        tf = fmin(tf, fmax(a, b));
      }
      any = any || !(miss || tn > tf);
    }
    if (!any) continue;
    // body frame: x_body = R^T (x - p)
    const double *R = I.rot;
    double q0 = c[0] - p[0], q1 = c[1] - p[1], q2 = c[2] - p[2];
    float ox = static_cast<float>(R[0] * q0 + R[3] * q1 + R[6] * q2);
    float oy = static_cast<float>(R[1] * q0 + R[4] * q1 + R[7] * q2);
    float oz = static_cast<float>(R[2] * q0 + R[5] * q1 + R[8] * q2);
    float d[2][3];
    for (int r = 0; r < 2; ++r) {
      d[r][0] = static_cast<float>(R[0] * dw[r][0] + R[3] * dw[r][1] + R[6] * dw[r][2]);
      d[r][1] = static_cast<float>(R[1] * dw[r][0] + R[4] * dw[r][1] + R[7] * dw[r][2]);
      d[r][2] = static_cast<float>(R[2] * dw[r][0] + R[5] * dw[r][1] + R[8] * dw[r][2]);
    }
    int32_t skip = (j == self_inst) ? self_local : -1;
    if (blas_occluded2(I.nodes, I.leaf, ox, oy, oz, d, skip, stack, stride)) return true;
  }
  return false;
}

// Does the segment a -> b meet the box [lo, hi] (FP64 slab test, closed)?
__device__ inline bool seg_box(const double a[3], const double b[3], const double lo[3],
                               const double hi[3]) {
  double tn = 0.0, tf = 1.0;
  for (int k = 0; k < 3; ++k) {
    const double d = b[k] - a[k];
    if (d == 0.0) {
      if (a[k] < lo[k] || a[k] > hi[k]) return false;
      continue;
    }
    const double u = (lo[k] - a[k]) / d, w = (hi[k] - a[k]) / d;
    tn = fmax(tn, fmin(u, w));
    tf = fmin(tf, fmax(u, w));
  }
  return tn <= tf;
}

// World box of instance I swept over the times [ta, tb] and grown by g[k] on each side.
__device__ inline void swept_box(const DevInstance &I, double ta, double tb, const double g[3],
                                 double lo[3], double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    const double pa = I.pos0[k] + I.vel[k] * ta, pb = I.pos0[k] + I.vel[k] * tb;
    lo[k] = I.box_lo[k] + fmin(pa, pb) - g[k];
    hi[k] = I.box_hi[k] + fmax(pa, pb) + g[k];
  }
}

// Instances (bit j for instance j < 64) whose box some segment c(t) -> T or c(t) -> R of
// the wave may meet, c(t) the centroid of facet f (the wave's one facet) at the chirp times
// t of chirps n_a .. n_b. Lane j tests instance j: the segments from the centroid at the
// middle time, against the box swept over the chirps' times and grown by the centroid's
// sweep about its middle position (the point at parameter s of c(t) -> S differs from that
// of c_m -> S by (1 - s)(c(t) - c_m)) and by 1e-6 m against rounding. A superset of the
// instances the per-chirp FP64 box test admits, so the decisions are those without it;
// instances from 64 on are not filtered.
__device__ uint64_t wave_candidates(const DevScene &sc, const RadarConst &rc, int64_t f, int n_a,
                                    int n_b) {
  const int lane = threadIdx.x & 63;
  const double ta = n_a * rc.tc, tb = n_b * rc.tc, tm = 0.5 * (ta + tb);
  const DevInstance &F = sc.inst[find_instance(sc.inst, sc.n_inst, f)];
  const int32_t lt = static_cast<int32_t>(f - F.facet_base);
  double b[3] = {0.0, 0.0, 0.0};
  for (int v = 0; v < 3; ++v) {
    const int32_t vi = F.tris[3 * lt + v];
    for (int k = 0; k < 3; ++k) b[k] += F.verts[3 * vi + k];
  }
  double cm[3], hw[3];
  for (int k = 0; k < 3; ++k) {
    cm[k] = (F.rot[3 * k + 0] * b[0] + F.rot[3 * k + 1] * b[1] + F.rot[3 * k + 2] * b[2]) / 3.0 +
            (F.pos0[k] + F.vel[k] * tm);
    hw[k] = fabs(F.vel[k]) * (0.5 * (tb - ta)) + 1e-6;
  }
  bool cand = false;
  if (lane < sc.n_inst) {
    const DevInstance &I = sc.inst[lane];
    double lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      const double pa = I.pos0[k] + I.vel[k] * ta, pb = I.pos0[k] + I.vel[k] * tb;
      lo[k] = I.box_lo[k] + fmin(pa, pb) - hw[k];
      hi[k] = I.box_hi[k] + fmax(pa, pb) + hw[k];
    }
    for (int r = 0; r < 2; ++r) {
      const double *S = r ? rc.rx_c : rc.tx_c;
      double tn = 0.0, tf = 1.0;
      bool miss = false;
      for (int k = 0; k < 3; ++k) {
        const double d = S[k] - cm[k];
        if (d == 0.0) {
          if (cm[k] < lo[k] || cm[k] > hi[k]) miss = true;
          continue;
        }
        const double a = (lo[k] - cm[k]) / d, e = (hi[k] - cm[k]) / d;
        tn = fmax(tn, fmin(a, e));
        tf = fmin(tf, fmax(a, e));
      }
      cand = cand || !(miss || tn > tf);
    }
  }
  return __ballot(cand);
}

// One side (phase centre E, facing value fe = n . (E - c)) of a facet: *direct when it
// faces E and centroid -> E is clear; *reflected when the centroid lies above the ground
// plane, the facet faces the image E' and both legs centroid -> S -> E are clear, S the
// specular point (the road surface is skipped for these legs).
__device__ void reflected_sides(const DevScene &sc, const RadarConst &rc, double t,
                                const double c[3], const double n[3], const double E[3], double fe,
                                int ii, int32_t lt, int32_t *stk, int stride, bool *direct,
                                bool *refl) {
  *direct = fe > 0.0 && !segment_blocked(sc, t, c, E, ii, lt, stk, stride);
  *refl = false;
  if (!(c[2] > rc.z_ground)) return;
  const double ez = 2.0 * rc.z_ground - E[2];  // image height
  const double fi = n[0] * (E[0] - c[0]) + n[1] * (E[1] - c[1]) + n[2] * (ez - c[2]);
  if (!(fi > 0.0)) return;
  const double a = (c[2] - rc.z_ground) / (c[2] - ez);
  const double S[3] = {c[0] + a * (E[0] - c[0]), c[1] + a * (E[1] - c[1]), rc.z_ground};
  *refl = !segment_blocked(sc, t, c, S, ii, lt, stk, stride, true) &&
          !segment_blocked(sc, t, S, E, -1, -1, stk, stride, true);
}

}  // namespace

namespace {

// Lit decisions of facet f at chirp n: the single path (lit[0]) or, with the ground bounce,
// the four path types (transmit side k & 1, receive side k >> 1).
__device__ void facet_lit(const DevScene &sc, const RadarConst &rc, int64_t f, int n,
                          int32_t *stk, int stride, uint64_t cand, bool lit[4]) {
  lit[0] = lit[1] = lit[2] = lit[3] = false;
  const double t = n * rc.tc;
  const int ii = find_instance(sc.inst, sc.n_inst, f);
  const DevInstance &I = sc.inst[ii];
  const int32_t lt = static_cast<int32_t>(f - I.facet_base);
  double x[3][3];
  for (int v = 0; v < 3; ++v) {
    const int32_t vi = I.tris[3 * lt + v];
    const double b0 = I.verts[3 * vi + 0], b1 = I.verts[3 * vi + 1], b2 = I.verts[3 * vi + 2];
    for (int k = 0; k < 3; ++k)
      x[v][k] = I.rot[3 * k + 0] * b0 + I.rot[3 * k + 1] * b1 + I.rot[3 * k + 2] * b2 +
                (I.pos0[k] + I.vel[k] * t);
  }
  double c[3], e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = (x[0][k] + x[1][k] + x[2][k]) / 3.0;
    e1[k] = x[1][k] - x[0][k];
    e2[k] = x[2][k] - x[0][k];
  }
  const double nx = e1[1] * e2[2] - e1[2] * e2[1];
  const double ny = e1[2] * e2[0] - e1[0] * e2[2];
  const double nz = e1[0] * e2[1] - e1[1] * e2[0];
  const bool nonzero = (nx != 0.0 || ny != 0.0 || nz != 0.0);
  const double ft = nx * (rc.tx_c[0] - c[0]) + ny * (rc.tx_c[1] - c[1]) + nz * (rc.tx_c[2] - c[2]);
  const double fr = nx * (rc.rx_c[0] - c[0]) + ny * (rc.rx_c[1] - c[1]) + nz * (rc.rx_c[2] - c[2]);
  if (!rc.bounce) {
    if (nonzero && ft > 0.0 && fr > 0.0)
      lit[0] = !pair_blocked(sc, t, c, rc.tx_c, rc.rx_c, ii, lt, stk, stride, cand);
  } else if (nonzero) {
    const double nv[3] = {nx, ny, nz};
    bool dt, it, dr, ir;
    reflected_sides(sc, rc, t, c, nv, rc.tx_c, ft, ii, lt, stk, stride, &dt, &it);
    reflected_sides(sc, rc, t, c, nv, rc.rx_c, fr, ii, lt, stk, stride, &dr, &ir);
    lit[0] = dt && dr;
    lit[1] = it && dr;
    lit[2] = dt && ir;
    lit[3] = it && ir;
  }
}

}  // namespace

// A workgroup covers kVisFacetsPer facets (whole mask words) and `cw` consecutive chirps
// (a power of two up to 64); lane = chirp within the group, so the lanes of a wave trace
// nearly the same rays of one facet at neighbouring chirps and follow nearly one BVH path
// (mapping lanes to neighbouring facets instead makes every wave walk the union of 64
// different paths). Decisions are gathered as bits in LDS and written as whole words.
__global__ void __launch_bounds__(kVisThreads) __attribute__((amdgpu_waves_per_eu(4, 8))) vis_kernel(DevScene sc, RadarConst rc, int cw,
                                                        int facets_per_block, int n_begin,
                                                        int n_end) {
  extern __shared__ int32_t vis_lds[];
  __shared__ uint64_t cand_lds[kVisFilterFacets];
  const int words = facets_per_block >> 5;
  const int types = rc.bounce ? 4 : 1;
  uint32_t *bits = reinterpret_cast<uint32_t *>(vis_lds);  // [types][cw][words]
  int32_t *stk = vis_lds + kVisBitWords + threadIdx.x;      // column per thread
  for (int k = threadIdx.x; k < types * cw * words; k += blockDim.x) bits[k] = 0u;
  __syncthreads();
  const int nl = threadIdx.x % cw;
  const int n = n_begin + static_cast<int>(blockIdx.y) * cw + nl;
  const int64_t f0 = static_cast<int64_t>(blockIdx.x) * facets_per_block;
  // With 64 chirps per group (a wave per facet) and the single path, the instances each
  // facet's segments may meet are found first, one wave per facet in turn, into LDS.
  const bool filter = cw == 64 && !rc.bounce && facets_per_block <= kVisFilterFacets;
  if (filter) {
    const int n_a = n_begin + static_cast<int>(blockIdx.y) * cw;
    const int n_b = min(n_end, n_a + cw) - 1;
    for (int fl = threadIdx.x >> 6; fl < facets_per_block; fl += blockDim.x >> 6) {
      const int64_t f = f0 + fl;
      if (f >= sc.n_facets) break;  // wave-uniform
      const uint64_t m = wave_candidates(sc, rc, f, n_a, n_b);
      if ((threadIdx.x & 63) == 0) cand_lds[fl] = m;
    }
    __syncthreads();
  }
  for (int fl = threadIdx.x / cw; fl < facets_per_block; fl += blockDim.x / cw) {
    const int64_t f = f0 + fl;
    if (f >= sc.n_facets || n >= n_end) continue;
    const uint64_t cand = filter ? cand_lds[fl] : ~uint64_t(0);
    bool lit[4];
    facet_lit(sc, rc, f, n, stk, blockDim.x, cand, lit);
    for (int k = 0; k < types; ++k)
      if (lit[k]) atomicOr(&bits[(k * cw + nl) * words + (fl >> 5)], 1u << (fl & 31));
  }
  __syncthreads();
  for (int e = threadIdx.x; e < types * cw * words; e += blockDim.x) {
    const int w = e % words, r = e / words;  // r = k * cw + chirp within the group
    const int k = r / cw, nn = n_begin + static_cast<int>(blockIdx.y) * cw + (r % cw);
    const int64_t word = static_cast<int64_t>(blockIdx.x) * words + w;
    if (nn < n_end && word < sc.mask_words)
      sc.mask[(static_cast<int64_t>(k) * rc.N + nn) * sc.mask_words + word] = bits[e];
  }
}

// Per-chirp compaction of the mask into ascending facet indices (deterministic).
__global__ void __launch_bounds__(1024) compact_kernel(DevScene sc, int n_begin) {
  __shared__ int32_t s_scan[1024];
  const int n = n_begin + static_cast<int>(blockIdx.x);
  const uint32_t *row = sc.mask + static_cast<int64_t>(n) * sc.mask_words;
  const int64_t per = (sc.mask_words + blockDim.x - 1) / blockDim.x;
  const int64_t w0 = static_cast<int64_t>(threadIdx.x) * per;
  const int64_t w1 = min(sc.mask_words, w0 + per);
  const uint32_t tail_bits = static_cast<uint32_t>(sc.n_facets & 31);
  int32_t cnt = 0;
  for (int64_t w = w0; w < w1; ++w) {
    uint32_t b = row[w];
    if (w == sc.mask_words - 1 && tail_bits) b &= (1u << tail_bits) - 1u;
    cnt += __popc(b);
  }
  s_scan[threadIdx.x] = cnt;
  __syncthreads();
  for (int off = 1; off < static_cast<int>(blockDim.x); off <<= 1) {
    int32_t v = (threadIdx.x >= static_cast<unsigned>(off)) ? s_scan[threadIdx.x - off] : 0;
    __syncthreads();
    s_scan[threadIdx.x] += v;
    __syncthreads();
  }
  int32_t pos = s_scan[threadIdx.x] - cnt;
  int32_t *out = sc.vis_idx + static_cast<int64_t>(n) * sc.n_facets;
  for (int64_t w = w0; w < w1; ++w) {
    uint32_t b = row[w];
    if (w == sc.mask_words - 1 && tail_bits) b &= (1u << tail_bits) - 1u;
    while (b) {
      const int bit = __ffs(b) - 1;
      out[pos++] = static_cast<int32_t>(w * 32 + bit);
      b &= b - 1u;
    }
  }
  if (threadIdx.x == blockDim.x - 1) sc.vis_cnt[n] = s_scan[threadIdx.x];
}

// ---- facet-to-facet double bounce: connections ----------------------------------------

namespace {

// Slab test of the body-frame ray o + t d against a box for t in [0, t_end].
__device__ inline bool box_hit_t(const float *lo, const float *hi, float ox, float oy, float oz,
                                 float ix, float iy, float iz, float t_end) {
  float tx0 = (lo[0] - ox) * ix, tx1 = (hi[0] - ox) * ix;
  float ty0 = (lo[1] - oy) * iy, ty1 = (hi[1] - oy) * iy;
  float tz0 = (lo[2] - oz) * iz, tz1 = (hi[2] - oz) * iz;
  float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
  float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fminf(fmaxf(tz0, tz1), t_end));
  return tn <= tf;
}

// Nearer hits of the leaf's triangles by o + t d, t in (t_min, t_best) (closed test):
// shrinks t_best and records the triangle id.
__device__ inline void leaf_closest(const float4 *leaf, int32_t ref, float ox, float oy, float oz,
                                    float dx, float dy, float dz, int32_t skip, float t_min,
                                    float &t_best, int32_t &id) {
  uint32_t code = static_cast<uint32_t>(-ref - 1);
  uint32_t first = code >> 4, count = code & 15u;
  for (uint32_t k = 0; k < count; ++k) {
    const float4 a = leaf[3 * (first + k) + 0];
    const float4 b = leaf[3 * (first + k) + 1];
    const float4 c = leaf[3 * (first + k) + 2];
    const int32_t tid = __float_as_int(c.y);
    if (tid == skip) continue;
    float e1x = a.w, e1y = b.x, e1z = b.y;
    float e2x = b.z, e2y = b.w, e2z = c.x;
    float px = dy * e2z - dz * e2y, py = dz * e2x - dx * e2z, pz = dx * e2y - dy * e2x;
    float det = e1x * px + e1y * py + e1z * pz;
    if (det == 0.0f) continue;
    float inv = 1.0f / det;
    float sx = ox - a.x, sy = oy - a.y, sz = oz - a.z;
    float u = (sx * px + sy * py + sz * pz) * inv;
    if (!(u >= 0.0f && u <= 1.0f)) continue;
    float qx = sy * e1z - sz * e1y, qy = sz * e1x - sx * e1z, qz = sx * e1y - sy * e1x;
    float v = (dx * qx + dy * qy + dz * qz) * inv;
    if (!(v >= 0.0f && u + v <= 1.0f)) continue;
    float t = (e2x * qx + e2y * qy + e2z * qz) * inv;
    if (t > t_min && t < t_best) {
      t_best = t;
      id = tid;
    }
  }
}

// Closest-hit traversal of one four-wide BLAS (body frame; the same stack discipline as
// blas_occluded: at most three pending children per level).
__device__ void blas_closest(const BvhNode4 *nodes, const float4 *leaf, float ox, float oy,
                             float oz, float dx, float dy, float dz, int32_t skip, float t_min,
                             float &t_best, int32_t &id, int32_t *stack, int stride) {
  const float ix = safe_inv(dx), iy = safe_inv(dy), iz = safe_inv(dz);
  int sp = 0;
  int32_t node = 0;
  while (true) {
    const BvhNode4 nd = nodes[node];
    int32_t next = -1;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float lo[3] = {nd.lo[0][i], nd.lo[1][i], nd.lo[2][i]};
      const float hi[3] = {nd.hi[0][i], nd.hi[1][i], nd.hi[2][i]};
      if (!box_hit_t(lo, hi, ox, oy, oz, ix, iy, iz, t_best)) continue;
      const int32_t c = nd.c[i];
      if (c < 0) {
        leaf_closest(leaf, c, ox, oy, oz, dx, dy, dz, skip, t_min, t_best, id);
      } else if (next >= 0) {
        stack[sp * stride] = c;
        ++sp;
      } else {
        next = c;
      }
    }
    if (next < 0) {
      if (sp == 0) return;
      --sp;
      next = stack[sp * stride];
    }
    node = next;
  }
}

__device__ inline void world_vertices(const DevInstance &I, int64_t lt, double t, double x[3][3]) {
  for (int v = 0; v < 3; ++v) {
    const int32_t vi = I.tris[3 * lt + v];
    const double b0 = I.verts[3 * vi + 0], b1 = I.verts[3 * vi + 1], b2 = I.verts[3 * vi + 2];
    for (int k = 0; k < 3; ++k)
      x[v][k] = I.rot[3 * k + 0] * b0 + I.rot[3 * k + 1] * b1 + I.rot[3 * k + 2] * b2 +
                (I.pos0[k] + I.vel[k] * t);
  }
}

// Unit normal (CCW) and centroid of a world triangle; false for zero area.
__device__ inline bool tri_frame(const double x[3][3], double c[3], double n[3]) {
  double e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    c[k] = (x[0][k] + x[1][k] + x[2][k]) / 3.0;
    e1[k] = x[1][k] - x[0][k];
    e2[k] = x[2][k] - x[0][k];
  }
  n[0] = e1[1] * e2[2] - e1[2] * e2[1];
  n[1] = e1[2] * e2[0] - e1[0] * e2[2];
  n[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double a = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
  if (!(a > 0.0)) return false;
  for (int k = 0; k < 3; ++k) n[k] /= a;
  return true;
}

__device__ inline double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// The pair search's instance filter for facet f (the wave's one facet) at chirps n_a .. n_b:
// for each launching end k, the instances (bit j for instance j < 64) that the shadow
// segment c(t) -> E (out[2 k]) or the specular segment c(t) -> c(t) + ray_len r(t)
// (out[2 k + 1]) of some chirp may meet. Lane j tests instance j with the segments at the
// middle time against its box swept over the chirps' times and grown: by the centroid's
// sweep per axis for the shadow segment (as in visibility); for the specular one by
// |delta| (1 + 2 ray_len / (|E - c_m| - |delta|)), |delta| the centroid's largest
// displacement from its middle position (the unit vector towards E turns by at most
// 2 |delta| / (|E - c_m| - |delta|), and the mirror in A's plane, fixed under translation,
// keeps that), plus 1e-6 m against rounding. Supersets of what the per-chirp FP64 box
// tests admit; all instances where that bound does not apply.
__device__ void db_wave_candidates(const DevScene &sc, const RadarConst &rc, int64_t f, int n_a,
                                   int n_b, double ray_len, uint64_t out[4]) {
  const int lane = threadIdx.x & 63;
  const double ta = n_a * rc.tc, tb = n_b * rc.tc, tm = 0.5 * (ta + tb);
  const DevInstance &A = sc.inst[find_instance(sc.inst, sc.n_inst, f)];
  double x[3][3], c[3], na[3];
  world_vertices(A, f - A.facet_base, tm, x);
  const bool ok = tri_frame(x, c, na);
  double hw[3], sweep = 0.0;
  for (int k = 0; k < 3; ++k) {
    const double dk = fabs(A.vel[k]) * (0.5 * (tb - ta));
    hw[k] = dk + 1e-6;
    sweep += dk * dk;
  }
  sweep = sqrt(sweep);
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double *E = k ? rc.rx_c : rc.tx_c;
    double de[3] = {E[0] - c[0], E[1] - c[1], E[2] - c[2]};
    const double ld = sqrt(dot3(de, de));
    bool all = !ok || !(ld - sweep > 0.0);
    double end[3], gr[3];
    if (!all) {
      double r[3];
      for (int q = 0; q < 3; ++q) r[q] = -de[q] / ld;
      const double rn = dot3(r, na);
      for (int q = 0; q < 3; ++q) {
        r[q] -= 2.0 * rn * na[q];
        end[q] = c[q] + ray_len * r[q];
      }
      const double g = sweep * (1.0 + 2.0 * ray_len / (ld - sweep)) + 1e-6;
      gr[0] = gr[1] = gr[2] = g;
    }
    bool ce = true, cr = true;
    if (lane < sc.n_inst && !all) {
      const DevInstance &I = sc.inst[lane];
      double lo[3], hi[3];
      swept_box(I, ta, tb, hw, lo, hi);
      ce = seg_box(c, E, lo, hi);
      swept_box(I, ta, tb, gr, lo, hi);
      cr = seg_box(c, end, lo, hi);
    }
    out[2 * k] = __ballot(ce);
    out[2 * k + 1] = __ballot(cr);
  }
}

// Facet B that the ray launched from end k (0: Tx phase centre, 1: Rx) reflected off facet A
// (scene index f) connects to at chirp n, or -1 (Section 2.2; the rules of the oracle's
// facet-to-facet double bounce): A faces the launching centre E and sees it; the specular
// ray from A's centroid first hits B (FP32 traversal over a segment of ray_len metres); B
// faces the image E' of E in A's plane and the other centre O, and the segment from the
// hit point to O is clear; the central projection from E' of A's vertices onto B's plane
// lies ahead of E' (parameters above 1/2) and within 1.5 r_lim of its centroid. Reads
// the chirp's lit mask (computed before, single path).
__device__ int32_t db_connect(const DevScene &sc, const RadarConst &rc, int64_t f, int n, int k,
                              double ray_len, double r_lim, int32_t *stk, int stride,
                              uint64_t cand_e, uint64_t cand_r) {
  const double t = n * rc.tc;
  const double *E = k ? rc.rx_c : rc.tx_c;
  const double *O = k ? rc.tx_c : rc.rx_c;
  const int ia = find_instance(sc.inst, sc.n_inst, f);
  const DevInstance &IA = sc.inst[ia];
  const int32_t la = static_cast<int32_t>(f - IA.facet_base);
  double xa[3][3], ca[3], na[3];
  world_vertices(IA, la, t, xa);
  if (!tri_frame(xa, ca, na)) return -1;
  double de[3] = {E[0] - ca[0], E[1] - ca[1], E[2] - ca[2]};
  const double fe = dot3(na, de);
  if (!(fe > 0.0)) return -1;
  // A lit facet (single path, this chirp's mask) faces both centres with both segments from
  // its centroid clear, the one to E among them: its test is not repeated
  const bool lit = (sc.mask[static_cast<int64_t>(n) * sc.mask_words + (f >> 5)] >> (f & 31)) & 1u;
  if (!lit && segment_blocked(sc, t, ca, E, ia, la, stk, stride, false, cand_e)) return -1;
  // specular direction of d = (c_A - E) / |c_A - E|
  const double ld = sqrt(dot3(de, de));
  double r[3];
  for (int q = 0; q < 3; ++q) r[q] = -de[q] / ld;
  const double rn = dot3(r, na);
  for (int q = 0; q < 3; ++q) r[q] -= 2.0 * rn * na[q];
  // first hit over all instances (A excluded), t as a fraction of ray_len
  float t_best = 1.0f;
  int32_t id_best = -1, inst_best = -1;
  const double ir[3] = {r[0] != 0.0 ? 1.0 / (r[0] * ray_len) : 0.0,
                        r[1] != 0.0 ? 1.0 / (r[1] * ray_len) : 0.0,
                        r[2] != 0.0 ? 1.0 / (r[2] * ray_len) : 0.0};
  const float t_min = static_cast<float>(1e-6 / ray_len);
  for (int j = 0; j < sc.n_inst; ++j) {
    if (j < 64 && !((cand_r >> j) & 1u)) continue;  // no specular segment of the wave meets it
    const DevInstance &I = sc.inst[j];
    if (!I.has_bvh) continue;
    double p[3] = {I.pos0[0] + I.vel[0] * t, I.pos0[1] + I.vel[1] * t, I.pos0[2] + I.vel[2] * t};
    double tn = 0.0, tf = static_cast<double>(t_best);
    bool miss = false;
    for (int q = 0; q < 3; ++q) {
      const double lo = I.box_lo[q] + p[q], hi = I.box_hi[q] + p[q];
      if (r[q] == 0.0) {
        if (ca[q] < lo || ca[q] > hi) miss = true;
        continue;
      }
      const double a = (lo - ca[q]) * ir[q], b = (hi - ca[q]) * ir[q];
      tn = fmax(tn, fmin(a, b));
      tf = fmin(tf, fmax(a, b));
    }
    if (miss || tn > tf) continue;
    const double *R = I.rot;
    const double q0 = ca[0] - p[0], q1 = ca[1] - p[1], q2 = ca[2] - p[2];
    const float ox = static_cast<float>(R[0] * q0 + R[3] * q1 + R[6] * q2);
    const float oy = static_cast<float>(R[1] * q0 + R[4] * q1 + R[7] * q2);
    const float oz = static_cast<float>(R[2] * q0 + R[5] * q1 + R[8] * q2);
    const double d0 = r[0] * ray_len, d1 = r[1] * ray_len, d2 = r[2] * ray_len;
    const float dx = static_cast<float>(R[0] * d0 + R[3] * d1 + R[6] * d2);
    const float dy = static_cast<float>(R[1] * d0 + R[4] * d1 + R[7] * d2);
    const float dz = static_cast<float>(R[2] * d0 + R[5] * d1 + R[8] * d2);
    int32_t id = -1;
    blas_closest(I.nodes, I.leaf, ox, oy, oz, dx, dy, dz, j == ia ? la : -1, t_min, t_best, id,
                 stk, stride);
    if (id >= 0) {
      id_best = id;
      inst_best = j;
    }
  }
  if (id_best < 0) return -1;
  const DevInstance &IB = sc.inst[inst_best];
  double xb[3][3], cb[3], nb[3];
  world_vertices(IB, id_best, t, xb);
  if (!tri_frame(xb, cb, nb)) return -1;
  const double th = static_cast<double>(t_best) * ray_len;
  const double h[3] = {ca[0] + th * r[0], ca[1] + th * r[1], ca[2] + th * r[2]};
  double ei[3];
  for (int q = 0; q < 3; ++q) ei[q] = E[q] - 2.0 * fe * na[q];
  const double f1 = nb[0] * (ei[0] - h[0]) + nb[1] * (ei[1] - h[1]) + nb[2] * (ei[2] - h[2]);
  const double f2 = nb[0] * (O[0] - h[0]) + nb[1] * (O[1] - h[1]) + nb[2] * (O[2] - h[2]);
  if (!(f1 > 0.0) || !(f2 > 0.0)) return -1;
  if (segment_blocked(sc, t, h, O, inst_best, id_best, stk, stride)) return -1;
  // footprint of A's tube on B's plane
  const double num = nb[0] * (cb[0] - ei[0]) + nb[1] * (cb[1] - ei[1]) + nb[2] * (cb[2] - ei[2]);
  double fp[3][3], cf[3] = {0.0, 0.0, 0.0};
  for (int v = 0; v < 3; ++v) {
    double dv[3] = {xa[v][0] - ei[0], xa[v][1] - ei[1], xa[v][2] - ei[2]};
    const double den = dot3(nb, dv);
    const double sv = num / den;
    if (!(sv > 0.5) || !isfinite(sv)) return -1;
    for (int q = 0; q < 3; ++q) {
      fp[v][q] = ei[q] + sv * dv[q];
      cf[q] += fp[v][q] / 3.0;
    }
  }
  const double lim2 = 2.25 * r_lim * r_lim;
  for (int v = 0; v < 3; ++v) {
    const double a = fp[v][0] - cf[0], b = fp[v][1] - cf[1], c = fp[v][2] - cf[2];
    if (!(a * a + b * b + c * c <= lim2)) return -1;
  }
  return static_cast<int32_t>(IB.facet_base + id_best);
}

}  // namespace

// Connections of every facet at chirps n_begin .. n_begin + n_chirps - 1, both launching
// ends: pair_b[(k N + n) F + f]. Workgroups as in vis_kernel (lane = chirp).
__global__ void __launch_bounds__(kVisThreads) dbounce_kernel(DevScene sc, RadarConst rc, int cw,
                                                            int facets_per_block, int n_begin,
                                                            int n_end, double ray_len,
                                                            double r_lim, int32_t *pair_b) {
  extern __shared__ int32_t db_lds[];
  __shared__ uint64_t cand_lds[kVisFilterFacets][4];
  int32_t *stk = db_lds + threadIdx.x;  // column per thread
  const int nl = threadIdx.x % cw;
  const int n = n_begin + static_cast<int>(blockIdx.y) * cw + nl;
  const int64_t f0 = static_cast<int64_t>(blockIdx.x) * facets_per_block;
  // with 64 chirps per group (a wave per facet) each facet's instances are filtered first
  const bool filter = cw == 64 && facets_per_block <= kVisFilterFacets;
  if (filter) {
    const int n_a = n_begin + static_cast<int>(blockIdx.y) * cw;
    const int n_b = min(n_end, n_a + cw) - 1;
    for (int fl = threadIdx.x >> 6; fl < facets_per_block; fl += blockDim.x >> 6) {
      const int64_t f = f0 + fl;
      if (f >= sc.n_facets) break;  // wave-uniform
      uint64_t m[4];
      db_wave_candidates(sc, rc, f, n_a, n_b, ray_len, m);
      if ((threadIdx.x & 63) == 0)
        for (int q = 0; q < 4; ++q) cand_lds[fl][q] = m[q];
    }
    __syncthreads();
  }
  for (int fl = threadIdx.x / cw; fl < facets_per_block; fl += blockDim.x / cw) {
    const int64_t f = f0 + fl;
    if (f >= sc.n_facets || n >= n_end) continue;
    for (int k = 0; k < 2; ++k) {
      const uint64_t ce = filter ? cand_lds[fl][2 * k] : ~uint64_t(0);
      const uint64_t cr = filter ? cand_lds[fl][2 * k + 1] : ~uint64_t(0);
      pair_b[(static_cast<int64_t>(k) * rc.N + n) * sc.n_facets + f] =
          db_connect(sc, rc, f, n, k, ray_len, r_lim, stk, blockDim.x, ce, cr);
    }
  }
}

// Per (end, chirp): the connected facets in ascending order and their count (deterministic).
// The row is read in tiles of one element per thread (coalesced); ballots and the waves'
// counts in LDS (two sets, alternating per tile, so one barrier per tile) place each
// connected facet.
__global__ void __launch_bounds__(1024) db_compact_kernel(const int32_t *pair_b, int64_t F,
                                                          int32_t *idx, int32_t *cnt) {
  __shared__ int32_t s_w[2][16];
  const int64_t row = blockIdx.x;  // k N + n
  const int32_t *b = pair_b + row * F;
  int32_t *out = idx + row * F;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  int32_t base = 0;
  int par = 0;
  for (int64_t t0 = 0; t0 < F; t0 += blockDim.x, par ^= 1) {
    const int64_t i = t0 + threadIdx.x;
    const int32_t v = i < F ? b[i] : -1;
    const bool on = v >= 0 && v < F;  // others: no connection
    const uint64_t m = __ballot(on);
    if (lane == 0) s_w[par][wv] = __popcll(m);
    __syncthreads();
    int32_t before = 0, total = 0;
    for (int w = 0; w < nw; ++w) {
      const int32_t c = s_w[par][w];
      before += w < wv ? c : 0;
      total += c;
    }
    if (on) out[base + before + __popcll(m & ((uint64_t(1) << lane) - 1))] = static_cast<int32_t>(i);
    base += total;
  }
  if (threadIdx.x == 0) cnt[row] = base;
}

hipError_t launch_dbounce(const DevScene &sc, const RadarConst &rc, double ray_len, double r_lim,
                          int32_t *pair_b, int32_t *idx, int32_t *cnt, hipStream_t s) {
  if (rc.N <= 0) return hipSuccess;
  if (sc.n_facets > 0 && ray_len > 0.0) {
    int cw = 1;
    while (cw < rc.N && cw < 64) cw <<= 1;
    const int fpb = std::max(32, kVisThreads / cw);
    dim3 grid(static_cast<unsigned>((sc.n_facets + fpb - 1) / fpb),
              static_cast<unsigned>((rc.N + cw - 1) / cw));
    const size_t lds = sizeof(int32_t) * static_cast<size_t>(sc.stack_depth) * kVisThreads;
    hipLaunchKernelGGL(dbounce_kernel, grid, dim3(kVisThreads), lds, s, sc, rc, cw, fpb, 0,
                       rc.N, ray_len, r_lim, pair_b);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(db_compact_kernel, dim3(static_cast<unsigned>(2 * rc.N)), dim3(1024), 0, s,
                     pair_b, sc.n_facets, idx, cnt);
  return hipGetLastError();
}

hipError_t launch_visibility(const DevScene &sc, const RadarConst &rc, int n_begin, int n_chirps,
                             hipStream_t s) {
  if (sc.n_facets == 0 || n_chirps <= 0) return hipSuccess;
  if (n_begin < 0 || n_begin + n_chirps > rc.N) return hipErrorInvalidValue;
  int cw = 1;  // chirps per group: the smallest power of two >= the count, at most 64
  while (cw < n_chirps && cw < 64) cw <<= 1;
  // facets per workgroup: whole 32-bit mask words, every thread busy for cw >= 8
  const int fpb = std::max(32, kVisThreads / cw);
  dim3 grid(static_cast<unsigned>((sc.n_facets + fpb - 1) / fpb),
            static_cast<unsigned>((n_chirps + cw - 1) / cw));
  // bit words: types x max(cw, 8) <= 4 x 64
  const size_t lds = sizeof(int32_t) * (kVisBitWords + static_cast<size_t>(sc.stack_depth) * kVisThreads);
  hipLaunchKernelGGL(vis_kernel, grid, dim3(kVisThreads), lds, s, sc, rc, cw, fpb, n_begin,
                     n_begin + n_chirps);
  return hipGetLastError();
}

hipError_t launch_compact(const DevScene &sc, int n_begin, int n_chirps, hipStream_t s) {
  if (n_chirps <= 0) return hipSuccess;
  hipLaunchKernelGGL(compact_kernel, dim3(n_chirps), dim3(1024), 0, s, sc, n_begin);
  return hipGetLastError();
}

}  // namespace rsim
