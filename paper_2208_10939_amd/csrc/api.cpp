// Host runtime and C ABI of librsim (see include/rsim.h for the contract).
//
// The context owns device copies of meshes (vertices, triangles, BVH), per-scene
// instance tables and work buffers (lit-facet lists per chirp), twiddle tables and
// timing events. Every launch goes to the caller's stream; nothing here blocks
// unless the call is documented as synchronous.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/rsim.h"
#include "rsim_internal.h"
#include "rsim_launch.h"

using namespace rsim;

namespace {

thread_local std::string g_thread_error;

constexpr int kStages = 10;
// stages 8 and 9 sum their own event pairs: the NUFFT spread kernel (one pair per launch)
// and the NUFFT adjoint's gather kernels (one pair per chunk)
constexpr int kKernelStage0 = 8;

struct MeshRec {
  std::vector<float> verts;
  std::vector<int32_t> tris;
  double box_lo[3], box_hi[3];  // body bounding box
  double r_max = 0.0;           // largest vertex-to-centroid distance of any triangle
  int depth = -1;
  int64_t n_nodes = 0, n_leaf = 0;
  void *d_verts = nullptr, *d_tris = nullptr, *d_nodes = nullptr, *d_leaf = nullptr;
  // vertex -> incident (triangle * 3 + corner), for the gradient gather
  int32_t *d_csr_off = nullptr, *d_csr_ent = nullptr;
};

struct InstRec {
  int32_t mesh;
  double rot[9], pos0[3], vel[3];
};

struct SceneRec {
  std::vector<InstRec> inst;
  std::vector<double> pt_pos, pt_vel, pt_amp;
  int64_t n_facets = 0;
  // device copies (rebuilt when dirty)
  bool dirty = true;
  DevInstance *d_inst = nullptr;
  double *d_pt = nullptr;  // pos [n][3], vel [n][3], amp [n][2]
  // work buffers sized for (N, F)
  int32_t buf_N = -1;
  int32_t buf_types = 0;  // path types the mask buffer holds (1, or 4 with the ground bounce)
  uint32_t *d_mask = nullptr;
  int32_t *d_vis_idx = nullptr;
  int32_t *d_vis_cnt = nullptr;
  // double bounce: connections [2][N][F], connected facets [2][N][F], counts [2][N]
  int32_t db_N = -1;
  int32_t *d_db = nullptr;
};

struct TunedShape {
  int mb, ft;
  int kernel;  // RSIM_KERNEL_VECTOR, _MATRIX or _NUFFT (0: not tuned: vector units)
};

// Device-side tables of one batched call: scene views and the longest-first work
// queue of (scene, chirp, sample tile, channel tile) items.
struct BatchTables {
  DevScene *d_scenes = nullptr;
  int4 *d_items = nullptr;
  int32_t *d_queue = nullptr;
  NuUnit *d_units = nullptr;  // NUFFT: (scene, chirp) units of every chunk, longest first
  size_t scenes_cap = 0, items_cap = 0, units_cap = 0;
  int32_t n_items = 0;
  // key of the uploaded contents
  std::vector<int32_t> ids;
  void *echo = nullptr;
  uint32_t *mask = nullptr;
  uint64_t version = 0;
  int mb = 0;
  int precision = -1;
};

struct GraphCache {
  bool valid = false;
  std::vector<int32_t> ids;
  void *echo = nullptr;
  uint32_t *mask = nullptr;
  rsim_opts opts{};
  uint64_t version = 0;
  hipGraphExec_t exec = nullptr;
  hipGraph_t graph = nullptr;
  BatchTables tables;  // the graph replays kernels reading these
};

}  // namespace

struct rsim_ctx {
  int device = -1;
  bool host_only = true;
  std::string err;
  uint64_t mem_limit = 0, mem_used = 0;
  std::map<void *, size_t> allocs;
  std::vector<MeshRec> meshes;
  std::vector<SceneRec> scenes;
  bool have_wf = false, have_arr = false;
  rsim_waveform wf{};
  std::vector<double> tx, rx;
  double *d_elem = nullptr;
  uint64_t version = 1;  // bumped on any change that invalidates cached graphs
  std::map<std::pair<int, int>, void *> twiddles;  // (L, precision) -> table
  void *d_scratch = nullptr;
  size_t scratch_bytes = 0;
  hipEvent_t ev0[kStages] = {}, ev1[kStages] = {};
  bool stage_ran[kStages] = {};
  std::vector<hipEvent_t> kern_ev[2];  // event pairs of stages 8 and 9 (grow-only pools)
  int kern_used[2] = {0, 0};           // pairs recorded since the timing reset
  bool timing_pending = false;
  hipStream_t capture_stream = nullptr;
  int cu_count = 0;
  size_t max_lds = 0;
  std::map<std::tuple<int, int, int>, TunedShape> tuned;  // (M, O, precision) -> shape
  int32_t bwd_kernel = RSIM_KERNEL_AUTO;  // facet-sum kernel of rsim_backward
  int32_t bwd_intra = 0;  // rsim_backward differentiates the delay within the chirp
  // velocity sums of that adjoint: per (chirp, lit facet, slot) [4] and per facet [N][F][3]
  void *adj_pv = nullptr, *adj_gxv = nullptr;
  size_t adj_pv_bytes = 0, adj_gxv_bytes = 0;
  // double-bounce adjoint: the connections' per-facet chirp sums [2][F][9] FP64
  void *adj_dbsum = nullptr;
  size_t adj_dbsum_bytes = 0;
  // adjoint work buffers
  float *adj_partial = nullptr, *adj_gxw = nullptr;
  double *adj_vpart = nullptr, *adj_gsum = nullptr;  // gsum: [2][F][9] (plain, t_n-weighted)
  // NUFFT facet sum work buffer (records, keys, order, cell counts, grids) and the layout
  // its count and grid regions were last cleared for
  unsigned long long *d_census = nullptr;  // NUFFT record census [kNuCensusSlots][4]
  bool census_ready = false;                // the last census call ran the NUFFT
  void *nu_buf = nullptr;
  size_t nu_buf_bytes = 0;
  void *adj_gscaled = nullptr;  // echo gradient times conj(gamma) (ground-bounce adjoint)
  size_t adj_gscaled_bytes = 0;
  void *nu_adj_buf = nullptr;  // work buffers of the NUFFT adjoint (grow-only)
  size_t nu_adj_bytes = 0;
  int32_t nu_chunk_max = 0;    // chirps per NUFFT chunk at most (0: as many as fit)
  std::array<int64_t, 6> nu_layout{};
  size_t adj_partial_n = 0, adj_gxw_n = 0, adj_vpart_n = 0, adj_gsum_n = 0;
  BatchTables batch;  // persistent launches outside graphs
  GraphCache graph;
  // detection and noise work buffers (grow only)
  void *det_P = nullptr, *det_mask = nullptr, *det_noise = nullptr, *det_list = nullptr;
  size_t det_P_n = 0, det_mask_n = 0, det_noise_n = 0, det_list_n = 0;
  int32_t *det_nodes = nullptr;             // node position, CSR offsets, channels
  size_t det_nodes_n = 0;
  std::vector<int32_t> det_nodes_host;      // uploaded contents
  double *noise_part = nullptr;
  size_t noise_part_n = 0;
  // ground plane of the reflected paths (rsim_set_ground)
  bool ground = false;
  double z_ground = 0.0, gamma_re = -1.0, gamma_im = 0.0;
  double *d_elem_img = nullptr;  // [3][E][3]: elements of path types 1..3 (images)
  uint64_t elem_img_version = 0;
  // facet-to-facet double bounce (rsim_set_double_bounce)
  bool dbounce = false;
  double db_gamma_re = -1.0, db_gamma_im = 0.0;
  // this device's copy of the allocation-free entry point's work array (never freed)
  void *static_scratch = nullptr;
};

namespace {

int32_t fail(rsim_ctx *ctx, int32_t code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx)
    ctx->err = buf;
  else
    g_thread_error = buf;
  return code;
}

#define HIP_TRY(ctx, expr)                                                                 \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess)                                                                  \
      return fail(ctx, RSIM_EDEVICE, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                     \
  } while (0)

int32_t dev_alloc(rsim_ctx *ctx, void **p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return RSIM_OK;
  if (ctx->mem_limit && ctx->mem_used + bytes > ctx->mem_limit)
    return fail(ctx, RSIM_ENOMEM, "allocation of %zu bytes exceeds the memory limit (%llu used of %llu)",
                bytes, (unsigned long long)ctx->mem_used, (unsigned long long)ctx->mem_limit);
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(ctx, RSIM_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
  }
  ctx->mem_used += bytes;
  ctx->allocs[*p] = bytes;
  return RSIM_OK;
}

void dev_free(rsim_ctx *ctx, void *p) {
  if (!p) return;
  auto it = ctx->allocs.find(p);
  if (it != ctx->allocs.end()) {
    ctx->mem_used -= it->second;
    ctx->allocs.erase(it);
  }
  (void)hipFree(p);
}

// Grow-only device buffer: reallocates (contents lost) when fewer than `bytes` are held.
int32_t grow_bytes(rsim_ctx *ctx, void **p, size_t *cap, size_t bytes) {
  if (*cap >= bytes && *p) return RSIM_OK;
  dev_free(ctx, *p);
  *p = nullptr;
  *cap = 0;
  int32_t rc = dev_alloc(ctx, p, std::max<size_t>(bytes, 64));
  if (!rc) *cap = std::max<size_t>(bytes, 64);
  return rc;
}

template <typename T>
int32_t upload(rsim_ctx *ctx, T **dst, const T *src, size_t count) {
  void *p = nullptr;
  int32_t rc = dev_alloc(ctx, &p, sizeof(T) * count);
  if (rc) return rc;
  if (count) {
    hipError_t e = hipMemcpy(p, src, sizeof(T) * count, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
      dev_free(ctx, p);
      return fail(ctx, RSIM_EDEVICE, "hipMemcpy failed: %s", hipGetErrorString(e));
    }
  }
  *dst = static_cast<T *>(p);
  return RSIM_OK;
}

bool finite_all(const double *p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

// FFT lengths of the range and Doppler transforms: 2^a 3^b in 2..4096
bool fft_size_ok(int v) {
  if (v < 2 || v > 4096) return false;
  while (v % 2 == 0) v /= 2;
  while (v % 3 == 0) v /= 3;
  return v == 1;
}

int32_t need_device(rsim_ctx *ctx) {
  if (ctx->host_only) return fail(ctx, RSIM_EDEVICE, "host-only context: no device calls");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  return RSIM_OK;
}

RadarConst radar_const(const rsim_ctx *ctx) {
  RadarConst rc{};
  rc.f0 = ctx->wf.f0_hz;
  rc.slope = ctx->wf.slope_hz_per_s;
  rc.fs = ctx->wf.fs_hz;
  rc.df = ctx->wf.slope_hz_per_s / ctx->wf.fs_hz;
  rc.tc = ctx->wf.chirp_period_s;
  rc.M = ctx->wf.n_samples;
  rc.N = ctx->wf.n_chirps;
  rc.P = static_cast<int32_t>(ctx->tx.size() / 3);
  rc.Q = static_cast<int32_t>(ctx->rx.size() / 3);
  rc.bounce = ctx->ground ? 1 : 0;
  rc.z_ground = ctx->z_ground;
  for (int k = 0; k < 3; ++k) {
    double st = 0, sr = 0;
    for (int p = 0; p < rc.P; ++p) st += ctx->tx[3 * p + k];
    for (int q = 0; q < rc.Q; ++q) sr += ctx->rx[3 * q + k];
    rc.tx_c[k] = st / rc.P;
    rc.rx_c[k] = sr / rc.Q;
  }
  return rc;
}

// Largest |2 pi slope d_p e_q| over any facet position (triangle inequality bound).
double cross_term_bound(const rsim_ctx *ctx, const RadarConst &rc) {
  double mt = 0, mr = 0;
  for (int p = 0; p < rc.P; ++p) {
    double d = 0;
    for (int k = 0; k < 3; ++k) d += (ctx->tx[3 * p + k] - rc.tx_c[k]) * (ctx->tx[3 * p + k] - rc.tx_c[k]);
    mt = std::max(mt, std::sqrt(d));
  }
  for (int q = 0; q < rc.Q; ++q) {
    double d = 0;
    for (int k = 0; k < 3; ++k) d += (ctx->rx[3 * q + k] - rc.rx_c[k]) * (ctx->rx[3 * q + k] - rc.rx_c[k]);
    mr = std::max(mr, std::sqrt(d));
  }
  return 2.0 * kPi * std::fabs(rc.slope) * mt * mr / (kC0 * kC0);
}

int32_t ensure_scene_device(rsim_ctx *ctx, SceneRec &sc) {
  const int N = ctx->wf.n_chirps;
  if (sc.dirty) {
    dev_free(ctx, sc.d_inst);
    dev_free(ctx, sc.d_pt);
    sc.d_inst = nullptr;
    sc.d_pt = nullptr;
    std::vector<DevInstance> di(sc.inst.size());
    int64_t base = 0;
    for (size_t i = 0; i < sc.inst.size(); ++i) {
      const InstRec &r = sc.inst[i];
      const MeshRec &m = ctx->meshes[r.mesh];
      DevInstance &d = di[i];
      std::memcpy(d.rot, r.rot, sizeof(d.rot));
      std::memcpy(d.pos0, r.pos0, sizeof(d.pos0));
      std::memcpy(d.vel, r.vel, sizeof(d.vel));
      // world box of rot * body box, padded for the FP32 traversal inside it
      for (int k = 0; k < 3; ++k) {
        double lo = 0, hi = 0;
        for (int j = 0; j < 3; ++j) {
          double a = r.rot[3 * k + j] * m.box_lo[j], b = r.rot[3 * k + j] * m.box_hi[j];
          lo += std::min(a, b);
          hi += std::max(a, b);
        }
        double pad = 1e-6 * (std::fabs(lo) + std::fabs(hi)) + 1e-6;
        d.box_lo[k] = lo - pad;
        d.box_hi[k] = hi + pad;
      }
      d.verts = static_cast<const float *>(m.d_verts);
      d.tris = static_cast<const int32_t *>(m.d_tris);
      d.nodes = static_cast<const BvhNode4 *>(m.d_nodes);
      d.leaf = static_cast<const float4 *>(m.d_leaf);
      d.facet_base = base;
      d.n_tris = static_cast<int32_t>(m.tris.size() / 3);
      d.has_bvh = m.depth >= 0 ? 1 : 0;
      // in the ground plane: every world vertex within 1e-6 m of it at t = 0, and no
      // vertical motion
      bool flat = !m.verts.empty() && r.vel[2] == 0.0;
      for (size_t v = 0; flat && v < m.verts.size() / 3; ++v) {
        const double z = r.rot[6] * m.verts[3 * v] + r.rot[7] * m.verts[3 * v + 1] +
                         r.rot[8] * m.verts[3 * v + 2] + r.pos0[2];
        flat = std::fabs(z - ctx->z_ground) <= 1e-6;
      }
      d.in_plane = flat ? 1 : 0;
      // horizontal at any height: the vertex height range, when no wider than 2e-6 m
      double zlo = 0.0, zhi = 0.0;
      for (size_t v = 0; v < m.verts.size() / 3; ++v) {
        const double z = r.rot[6] * m.verts[3 * v] + r.rot[7] * m.verts[3 * v + 1] +
                         r.rot[8] * m.verts[3 * v + 2] + r.pos0[2];
        zlo = v ? std::min(zlo, z) : z;
        zhi = v ? std::max(zhi, z) : z;
      }
      d.flat = (!m.verts.empty() && r.vel[2] == 0.0 && zhi - zlo <= 2e-6) ? 1 : 0;
      d.flat_lo = zlo;
      d.flat_hi = zhi;
      base += d.n_tris;
    }
    sc.n_facets = base;
    int32_t rc = upload(ctx, &sc.d_inst, di.data(), di.size());
    if (rc) return rc;
    const size_t np = sc.pt_amp.size() / 2;
    if (np) {
      std::vector<double> pts;
      pts.insert(pts.end(), sc.pt_pos.begin(), sc.pt_pos.end());
      pts.insert(pts.end(), sc.pt_vel.begin(), sc.pt_vel.end());
      pts.insert(pts.end(), sc.pt_amp.begin(), sc.pt_amp.end());
      rc = upload(ctx, &sc.d_pt, pts.data(), pts.size());
      if (rc) return rc;
    }
    sc.dirty = false;
    sc.buf_N = -1;
  }
  const int types = ctx->ground ? 4 : 1;
  if (sc.buf_N != N || sc.buf_types != types) {
    dev_free(ctx, sc.d_mask);
    dev_free(ctx, sc.d_vis_idx);
    dev_free(ctx, sc.d_vis_cnt);
    sc.d_mask = nullptr;
    sc.d_vis_idx = nullptr;
    sc.d_vis_cnt = nullptr;
    const int64_t words = (sc.n_facets + 31) / 32;
    int32_t rc;
    if ((rc = dev_alloc(ctx, reinterpret_cast<void **>(&sc.d_mask),
                        sizeof(uint32_t) * std::max<int64_t>(1, words) * N * types)))
      return rc;
    if ((rc = dev_alloc(ctx, reinterpret_cast<void **>(&sc.d_vis_idx),
                        sizeof(int32_t) * std::max<int64_t>(1, sc.n_facets) * N)))
      return rc;
    if ((rc = dev_alloc(ctx, reinterpret_cast<void **>(&sc.d_vis_cnt), sizeof(int32_t) * N))) return rc;
    sc.buf_N = N;
    sc.buf_types = types;
  }
  if (ctx->dbounce && sc.db_N != N) {
    dev_free(ctx, sc.d_db);
    sc.d_db = nullptr;
    sc.db_N = -1;
    const size_t words = 4 * static_cast<size_t>(N) * std::max<int64_t>(1, sc.n_facets) + 2 * N;
    int32_t rc;
    if ((rc = dev_alloc(ctx, reinterpret_cast<void **>(&sc.d_db), sizeof(int32_t) * words)))
      return rc;
    sc.db_N = N;
  }
  return RSIM_OK;
}

DevScene dev_scene(const SceneRec &sc, uint32_t *mask, void *echo) {
  DevScene d{};
  d.inst = sc.d_inst;
  d.n_inst = static_cast<int32_t>(sc.inst.size());
  d.n_points = static_cast<int32_t>(sc.pt_amp.size() / 2);
  d.n_facets = sc.n_facets;
  d.mask_words = (sc.n_facets + 31) / 32;
  const size_t np = d.n_points;
  d.pt_pos0 = sc.d_pt;
  d.pt_vel = sc.d_pt ? sc.d_pt + 3 * np : nullptr;
  d.pt_amp = sc.d_pt ? sc.d_pt + 6 * np : nullptr;
  d.mask = mask;
  d.vis_idx = sc.d_vis_idx;
  d.vis_cnt = sc.d_vis_cnt;
  d.echo = echo;
  return d;
}

TunedShape pick_shape(const rsim_ctx *ctx, int precision, const rsim_opts &o) {
  const int M = ctx->wf.n_samples;
  const int O = static_cast<int>(ctx->tx.size() / 3 * ctx->rx.size() / 3);
  // defaults from a tile sweep on MI355X (c2 workload); rsim_autotune refines them
  TunedShape s = precision ? TunedShape{16, 8, 0} : TunedShape{64, 16, 0};
  auto it = ctx->tuned.find(std::make_tuple(M, O, precision));
  if (it != ctx->tuned.end()) s = it->second;
  if (o.tile_m) s.mb = o.tile_m;
  if (o.tile_f) s.ft = o.tile_f;
  return s;
}

EchoShape echo_shape(const rsim_ctx *ctx, const RadarConst &rc, int mb, int max_threads = 512,
                     int max_blocks = 1 << 30) {
  EchoShape sh{};
  sh.O = rc.P * rc.Q;
  sh.E = rc.P + rc.Q;
  sh.O_w = std::min(sh.O, 256);
  sh.o_tiles = (sh.O + sh.O_w - 1) / sh.O_w;
  const int blocks_needed = (rc.M + mb - 1) / mb;
  sh.B_w = std::max(1, std::min({blocks_needed, max_threads / sh.O_w, max_blocks}));
  sh.M_t = sh.B_w * mb;
  sh.m_tiles = (rc.M + sh.M_t - 1) / sh.M_t;
  sh.n_compute = (sh.O_w * sh.B_w + 63) / 64 * 64;
  sh.two_pi_slope = 2.0 * kPi * rc.slope;
  return sh;
}

// Shape of the forward facet sum: at most kMaxComputeThreads accumulating threads (plus
// the staging waves), and as many sample blocks as fit the LDS double buffer.
EchoShape forward_shape(const rsim_ctx *ctx, const RadarConst &rc, int precision, int mb, int ft) {
  EchoShape sh = echo_shape(ctx, rc, mb, kMaxComputeThreads);
  while (sh.B_w > 1 && echo_smem_bytes(precision, mb, ft, sh) > ctx->max_lds)
    sh = echo_shape(ctx, rc, mb, kMaxComputeThreads, sh.B_w - 1);
  return sh;
}

// Largest cross-term phase the matrix-core sum may drop: each term then carries a relative
// error below 1e-5, an order of magnitude under the FP32 sum's tolerance.
constexpr double kMatrixCrossLimit = 1e-5;

// Why the matrix-core facet sum cannot run for this array and precision (nullptr: it can).
const char *matrix_ineligible(const rsim_ctx *ctx, const RadarConst &rc, int precision) {
  int pt = 0, qt = 0;
  if (precision != RSIM_FP32_PHASE64) return "the matrix-core facet sum is FP32 only";
  if (!mfma_variant(rc.P, rc.Q, &pt, &qt)) return "the matrix-core facet sum needs P <= 12, Q <= 16";
  if (cross_term_bound(ctx, rc) > kMatrixCrossLimit)
    return "array aperture too large to drop the Tx-Rx cross term on the matrix cores";
  return nullptr;
}

// Shape of the matrix-core facet sum: all O channels and 128 samples per workgroup.
EchoShape matrix_shape(const RadarConst &rc) {
  EchoShape sh{};
  sh.O = rc.P * rc.Q;
  sh.E = rc.P + rc.Q;
  sh.O_w = sh.O;
  sh.o_tiles = 1;
  sh.M_t = mfma_tile_samples();
  sh.B_w = 1;
  sh.m_tiles = (rc.M + sh.M_t - 1) / sh.M_t;
  sh.n_compute = 512;
  sh.two_pi_slope = 2.0 * kPi * rc.slope;
  int pt = 1, qt = 1;
  mfma_variant(rc.P, rc.Q, &pt, &qt);
  sh.slots_tx = 4 * pt;
  sh.slots = 4 * (pt + qt);
  return sh;
}

// NUFFT facet sum: grid length and work-buffer budget.
constexpr int kNuMaxGrid = 2048;
// NUFFT work buffer cap (chirps per launch): up to 48 GiB, within half the device memory
// free at the call and within the context's memory limit. A whole frame per launch keeps
// the per-chirp kernels (sort: one workgroup per chirp) filling the device.
constexpr size_t kNuRecBudgetMax = size_t(48) << 30;

size_t nufft_budget(const rsim_ctx *ctx, size_t held) {
  size_t free_b = 0, total_b = 0;
  size_t b = kNuRecBudgetMax;
  if (hipMemGetInfo(&free_b, &total_b) == hipSuccess) b = std::min(b, (free_b + held) / 2);
  if (ctx->mem_limit)
    b = std::min(b, ctx->mem_limit > ctx->mem_used - held ? ctx->mem_limit - (ctx->mem_used - held) : 0);
  return std::max<size_t>(b, size_t(256) << 20);
}

int smooth_at_least(int n) {  // smallest 2^a 3^b >= n
  int best = 1 << 30;
  for (int64_t p3 = 1; p3 < (int64_t(1) << 31); p3 *= 3)
    for (int64_t v = p3; v < (int64_t(1) << 31); v *= 2)
      if (v >= n) {
        best = std::min<int64_t>(best, v);
        break;
      }
  return best;
}

double scenes_rmax(const rsim_ctx *ctx, const std::vector<int32_t> &ids) {
  double r = 0.0;
  for (int32_t id : ids)
    for (const InstRec &i : ctx->scenes[id].inst) r = std::max(r, ctx->meshes[i.mesh].r_max);
  return r;
}

double scenes_vmax(const rsim_ctx *ctx, const std::vector<int32_t> &ids) {
  double v = 0.0;
  for (int32_t id : ids) {
    const SceneRec &sc = ctx->scenes[id];
    for (const InstRec &i : sc.inst)
      v = std::max(v, std::sqrt(i.vel[0] * i.vel[0] + i.vel[1] * i.vel[1] + i.vel[2] * i.vel[2]));
    for (size_t k = 0; k + 2 < sc.pt_vel.size(); k += 3)
      v = std::max(v, std::sqrt(sc.pt_vel[k] * sc.pt_vel[k] + sc.pt_vel[k + 1] * sc.pt_vel[k + 1] +
                                sc.pt_vel[k + 2] * sc.pt_vel[k + 2]));
  }
  return v;
}

// Grid, channel reach and FFT grouping shared by the NUFFT forward and adjoint (nullptr:
// fine; else why not).
const char *nufft_common(const rsim_ctx *ctx, const RadarConst &rc, const rsim_opts &o,
                         double v_max, NuShape *ns) {
  if (o.precision != RSIM_FP32_PHASE64) return "the NUFFT facet sum is FP32 only";
  const int ng = smooth_at_least(2 * rc.M);
  if (ng > kNuMaxGrid) return "the NUFFT facet sum needs 2M <= 2048";
  if (ng < 32) return "the NUFFT facet sum needs M >= 16";
  const double kappa = rc.df * ng / kC0;
  // every channel's grid position lies within chan_d cells of the phase-centre path's
  double et = 0.0, er = 0.0;
  for (int p = 0; p < rc.P; ++p) {
    double d = 0.0;
    for (int k = 0; k < 3; ++k) d += (ctx->tx[3 * p + k] - rc.tx_c[k]) * (ctx->tx[3 * p + k] - rc.tx_c[k]);
    et = std::max(et, std::sqrt(d));
  }
  for (int q = 0; q < rc.Q; ++q) {
    double d = 0.0;
    for (int k = 0; k < 3; ++k) d += (ctx->rx[3 * q + k] - rc.rx_c[k]) * (ctx->rx[3 * q + k] - rc.rx_c[k]);
    er = std::max(er, std::sqrt(d));
  }
  // with the delay within the chirp a channel's source also moves by its Doppler shift
  // (A + B M) n_g, at most n_g (f0 + M df) 2 v_max / (c fs) cells, relative to the
  // record's by twice that
  // within one wave of the spread (channels 64 g .. 64 g + 63) a channel lies within
  // kappa (|a_t - a_t0| + |a_r - a_r0|) cells of the wave's first (triangle inequality on
  // the two path lengths), plus rounding
  const int O = rc.P * rc.Q;
  double wd = 0.0;
  for (int o0 = 0; o0 < O; o0 += 64) {
    const int p0 = o0 / rc.Q, q0 = o0 % rc.Q;
    for (int o = o0; o < std::min(O, o0 + 64); ++o) {
      const int p = o / rc.Q, q = o % rc.Q;
      double dt = 0.0, dr = 0.0;
      for (int k = 0; k < 3; ++k) {
        const double a = ctx->tx[3 * p + k] - ctx->tx[3 * p0 + k];
        const double b = ctx->rx[3 * q + k] - ctx->rx[3 * q0 + k];
        dt += a * a;
        dr += b * b;
      }
      wd = std::max(wd, std::sqrt(dt) + std::sqrt(dr));
    }
  }
  double chan_d = kappa * (et + er);
  double wave_d = kappa * wd + 1e-3;
  if (o.intra_chirp) {
    const double dop = 2.0 * ng * (rc.f0 + rc.M * rc.df) * 2.0 * v_max / (kC0 * rc.fs);
    chan_d += dop;
    wave_d += dop;
  }
  NuShape s{};
  s.ng = ng;
  s.ld = ng + 1;
  s.fc = rc.f0 + (rc.M / 2) * rc.df;
  s.kc = 2.0 * kPi * s.fc / kC0;
  s.cells_per_s = rc.df * ng;
  s.kappa = kappa;
  s.sigma = kNuSigma;
  s.chan_d = chan_d;
  s.wave_d = wave_d;
  s.spread_groups = (O + 63) / 64;
  s.n0 = 0;
  s.n_chirps = rc.N;
  *ns = s;
  return nullptr;
}

// Channels per FFT workgroup: two workgroups per CU where the LDS allows (extra_lds:
// bytes beyond the two row buffers).
void nufft_fft_groups(const rsim_ctx *ctx, const RadarConst &rc, NuShape &s, size_t extra_lds) {
  s.cb = 0;
  for (int cb = 16; cb >= 1 && !s.cb; --cb) {
    NuShape t = s;
    t.cb = cb;
    if (nufft_smem_bytes(t) + extra_lds <= ctx->max_lds / 2) s.cb = cb;
  }
  if (!s.cb) s.cb = 1;
  const int O = rc.P * rc.Q;
  s.cb = std::min(s.cb, O);
  s.groups = (O + s.cb - 1) / s.cb;
}

// Why the NUFFT forward cannot run (nullptr: it can, and *ns holds its shape for facets
// within r_max of their centroids, without the chirp chunk, record stride and run bound):
// every source of a record lies within off_max = 2 r_max kappa cells of the record's
// path position and every channel within chan_d of the phase-centre path, and a run's
// window of kNuSlots cells must hold both sides of that reach and at least one cell.
const char *nufft_ineligible(const rsim_ctx *ctx, const RadarConst &rc, const rsim_opts &o,
                             double r_max, double v_max, NuShape *ns) {
  NuShape s{};
  if (const char *why = nufft_common(ctx, rc, o, v_max, &s)) return why;
  // a double-bounce footprint reaches 1.5 times the largest facet radius
  s.off_max = (ctx->dbounce ? 3.0 : 2.0) * r_max * s.kappa;
  s.b0 = static_cast<int32_t>(std::ceil(s.chan_d + s.off_max + 0.5 * kNuWidth));
  s.kspan = kNuSlots - 2 - 2 * s.b0;
  if (nufft_cells_per_source(s) == 0)
    return "array aperture too wide for the NUFFT spread (channels of one 64-channel group "
           "more than 4 grid cells apart)";
  if (s.kspan < 0)
    return "facets or array aperture too wide for the NUFFT window: node offsets (2 r_max "
           "df n_g / c) plus channel offsets exceed 9 grid cells";
  *ns = s;
  return nullptr;
}

// Why the NUFFT adjoint cannot run for facets within r_max of their centroids; *ns: its
// shape. Its gather reads each source's own cells from a staged grid row, so no run window
// bounds the node or channel offsets; they must stay within half the grid (a source's
// cells then lie within half a grid of its record's cell, which the gather's periodic
// indexing assumes).
const char *nufft_adj_ineligible(const rsim_ctx *ctx, const RadarConst &rc, double r_max,
                                 NuShape *ns) {
  rsim_opts o{};
  o.precision = RSIM_FP32_PHASE64;
  NuShape s{};
  if (const char *why = nufft_common(ctx, rc, o, 0.0, &s)) return why;
  if (2.0 * r_max * s.kappa + s.chan_d + 0.5 * kNuWidth + 2.0 >= 0.5 * s.ng)
    return "facets too large for the NUFFT adjoint: node offsets (2 r_max df n_g / c) plus "
           "channel offsets reach half the grid";
  nufft_fft_groups(ctx, rc, s, 0);
  *ns = s;
  return nullptr;
}

// Records per spread run: enough runs to fill the device several times over at the
// expected ~40% lit facets, 256 .. 1024.
int nufft_run_len(const rsim_ctx *ctx, int64_t stride, int n_chirps) {
  const double recs = 0.4 * static_cast<double>(stride) * n_chirps;
  const double want = recs / (32.0 * std::max(1, ctx->cu_count));
  int L = 256;
  while (L < 1024 && 2.0 * L <= want) L *= 2;
  return L;
}

// Runs of a chirp: every run but those cut by a gap of more than kspan cells (at most
// n_g / (kspan + 1) + 1 of them) and the last holds run_len records.
int32_t nufft_max_runs(const NuShape &ns, int64_t stride) {
  const int64_t full = stride / ns.run_len;
  return static_cast<int32_t>(full + (ns.ng + ns.kspan) / (ns.kspan + 1) + 2);
}

// Kernel, tiles and shape of one rsim_synthesize call.
struct SumPlan {
  bool matrix = false;
  bool nufft = false;
  TunedShape ts{};
  EchoShape sh{};
  NuShape ns{};         // NUFFT: shape; n_chirps = chirps per launch
  NuBuffers nb{};       // NUFFT: work buffers
  std::vector<NuShape> nu_scene;  // NUFFT: per scene of the call (reach, runs, stride)
  // NUFFT batched (persistent) calls: the units and the chunks of one launch each
  // (first unit, units, largest record stride, largest run bound)
  std::vector<NuUnit> nu_units;
  std::vector<std::array<int64_t, 4>> nu_chunks;
  const void *tw = nullptr;  // NUFFT: twiddles of the grid length
  // double bounce, per scene: metres a reflected ray is followed; largest facet radius
  std::vector<double> db_ray_len, db_r_lim;
  int batch_key = 0;  // tile key of the persistent work tables (0 for the matrix cores)
};

SumPlan plan_sum(const rsim_ctx *ctx, const RadarConst &rc, const rsim_opts &o, double r_max,
                 double v_max) {
  SumPlan pl;
  pl.ts = pick_shape(ctx, o.precision, o);
  const bool eligible = matrix_ineligible(ctx, rc, o.precision) == nullptr;
  NuShape ns{};
  const bool nu_ok = nufft_ineligible(ctx, rc, o, r_max, v_max, &ns) == nullptr;
  if (o.kernel == RSIM_KERNEL_NUFFT || ctx->dbounce ||
      (o.kernel == RSIM_KERNEL_AUTO && nu_ok && pl.ts.kernel == RSIM_KERNEL_NUFFT &&
       !o.tile_m && !o.tile_f)) {
    pl.nufft = true;
    pl.ns = ns;
    pl.sh = echo_shape(ctx, rc, 64);
    pl.batch_key = -1;
    return pl;
  }
  if (o.kernel == RSIM_KERNEL_MATRIX)
    pl.matrix = true;
  else if (o.kernel == RSIM_KERNEL_AUTO)  // the autotuned choice; vector units by default
    pl.matrix = eligible && pl.ts.kernel == RSIM_KERNEL_MATRIX && !o.tile_m && !o.tile_f;
  if (pl.matrix) {
    pl.sh = matrix_shape(rc);
    pl.batch_key = 0;
  } else {
    pl.sh = forward_shape(ctx, rc, o.precision, pl.ts.mb, pl.ts.ft);
    pl.batch_key = pl.ts.mb;
  }
  return pl;
}

void *twiddles(rsim_ctx *ctx, int L, int precision, int32_t *status) {
  auto key = std::make_pair(L, precision);
  auto it = ctx->twiddles.find(key);
  if (it != ctx->twiddles.end()) return it->second;
  const int full = std::max(1, L);
  void *p = nullptr;
  if (precision) {
    std::vector<double> t(2 * full);
    for (int i = 0; i < full; ++i) {
      t[2 * i] = std::cos(2.0 * kPi * i / L);
      t[2 * i + 1] = -std::sin(2.0 * kPi * i / L);
    }
    double *d = nullptr;
    *status = upload(ctx, &d, t.data(), t.size());
    p = d;
  } else {
    std::vector<float> t(2 * full);
    for (int i = 0; i < full; ++i) {
      t[2 * i] = static_cast<float>(std::cos(2.0 * kPi * i / L));
      t[2 * i + 1] = static_cast<float>(-std::sin(2.0 * kPi * i / L));
    }
    float *d = nullptr;
    *status = upload(ctx, &d, t.data(), t.size());
    p = d;
  }
  if (*status) return nullptr;
  ctx->twiddles[key] = p;
  return p;
}

int32_t scratch(rsim_ctx *ctx, size_t bytes, void **out) {
  if (ctx->scratch_bytes < bytes) {
    dev_free(ctx, ctx->d_scratch);
    ctx->d_scratch = nullptr;
    ctx->scratch_bytes = 0;
    int32_t rc = dev_alloc(ctx, &ctx->d_scratch, bytes);
    if (rc) return rc;
    ctx->scratch_bytes = bytes;
  }
  *out = ctx->d_scratch;
  return RSIM_OK;
}

void stage_begin(rsim_ctx *ctx, bool on, int k, hipStream_t s) {
  if (!on) return;
  (void)hipEventRecord(ctx->ev0[k], s);
  ctx->stage_ran[k] = true;
}
void stage_end(rsim_ctx *ctx, bool on, int k, hipStream_t s) {
  if (on) (void)hipEventRecord(ctx->ev1[k], s);
}
// Next event pair of kernel stage k (8 or 9) for this call's timing; nullptr without
// timing or when an event cannot be created.
const hipEvent_t *kernel_events(rsim_ctx *ctx, bool on, int k) {
  if (!on) return nullptr;
  std::vector<hipEvent_t> &pool = ctx->kern_ev[k - kKernelStage0];
  int &used = ctx->kern_used[k - kKernelStage0];
  while (static_cast<int>(pool.size()) < 2 * (used + 1)) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    pool.push_back(e);
  }
  ctx->stage_ran[k] = true;
  return &pool[2 * used++];
}

void timing_reset(rsim_ctx *ctx, bool on) {
  if (!on) return;
  for (int k = 0; k < kStages; ++k) ctx->stage_ran[k] = false;
  ctx->kern_used[0] = ctx->kern_used[1] = 0;
  ctx->timing_pending = true;
}

int32_t check_scene(rsim_ctx *ctx, int32_t scene_id) {
  if (scene_id < 0 || scene_id >= static_cast<int32_t>(ctx->scenes.size()))
    return fail(ctx, RSIM_EINVAL, "unknown scene id %d", scene_id);
  return RSIM_OK;
}

// Bounding box, BVH and vertex -> (triangle, corner) index of a mesh, uploaded to the
// device (first = true: fresh mesh; false: vertices changed, triangles unchanged).
int32_t index_mesh(rsim_ctx *ctx, MeshRec &m, bool first_time) {
  const int64_t n_tris = static_cast<int64_t>(m.tris.size() / 3);
  const int64_t n_verts = static_cast<int64_t>(m.verts.size() / 3);
  for (int k = 0; k < 3; ++k) {
    m.box_lo[k] = 0;
    m.box_hi[k] = 0;
  }
  bool first = true;
  for (int64_t t = 0; t < 3 * n_tris; ++t) {
    const float *v = &m.verts[3 * static_cast<int64_t>(m.tris[t])];
    for (int k = 0; k < 3; ++k) {
      if (first || v[k] < m.box_lo[k]) m.box_lo[k] = v[k];
      if (first || v[k] > m.box_hi[k]) m.box_hi[k] = v[k];
    }
    first = false;
  }
  m.r_max = 0.0;
  for (int64_t t = 0; t < n_tris; ++t) {
    double x[3][3], c[3] = {0.0, 0.0, 0.0};
    for (int v = 0; v < 3; ++v)
      for (int k = 0; k < 3; ++k) {
        x[v][k] = m.verts[3 * static_cast<int64_t>(m.tris[3 * t + v]) + k];
        c[k] += x[v][k] / 3.0;
      }
    for (int v = 0; v < 3; ++v) {
      double d = 0.0;
      for (int k = 0; k < 3; ++k) d += (x[v][k] - c[k]) * (x[v][k] - c[k]);
      m.r_max = std::max(m.r_max, std::sqrt(d));
    }
  }
  std::vector<BvhNode4> nodes;
  std::vector<float> leaf;
  m.depth = build_bvh(m.verts.data(), m.tris.data(), n_tris, nodes, leaf);
  if (3 * (m.depth + 1) > kBvhStack)
    return fail(ctx, RSIM_ERANGE, "BVH depth %d needs more than %d stack entries", m.depth,
                kBvhStack);
  m.n_nodes = static_cast<int64_t>(nodes.size());
  m.n_leaf = static_cast<int64_t>(leaf.size() / 12);
  if (ctx->host_only) return RSIM_OK;
  int32_t rc = need_device(ctx);
  if (rc) return rc;
  dev_free(ctx, m.d_verts);
  dev_free(ctx, m.d_nodes);
  dev_free(ctx, m.d_leaf);
  m.d_verts = m.d_nodes = m.d_leaf = nullptr;
  float *dv = nullptr;
  BvhNode4 *dn = nullptr;
  float *dl = nullptr;
  if ((rc = upload(ctx, &dv, m.verts.data(), m.verts.size()))) return rc;
  if ((rc = upload(ctx, &dn, nodes.data(), nodes.size()))) return rc;
  if ((rc = upload(ctx, &dl, leaf.data(), leaf.size()))) return rc;
  m.d_verts = dv;
  m.d_nodes = dn;
  m.d_leaf = dl;
  if (first_time) {
    int32_t *dt = nullptr;
    if ((rc = upload(ctx, &dt, m.tris.data(), m.tris.size()))) return rc;
    m.d_tris = dt;
    // counting sort of corners by vertex
    std::vector<int32_t> off(n_verts + 1, 0), ent(3 * n_tris);
    for (int64_t t = 0; t < 3 * n_tris; ++t) off[m.tris[t] + 1]++;
    for (int64_t v = 0; v < n_verts; ++v) off[v + 1] += off[v];
    std::vector<int32_t> pos(off.begin(), off.end() - 1);
    for (int64_t t = 0; t < 3 * n_tris; ++t) ent[pos[m.tris[t]]++] = static_cast<int32_t>(t);
    if ((rc = upload(ctx, &m.d_csr_off, off.data(), off.size()))) return rc;
    if ((rc = upload(ctx, &m.d_csr_ent, ent.data(), ent.size()))) return rc;
  }
  return RSIM_OK;
}

int32_t check_radar(rsim_ctx *ctx) {
  if (!ctx->have_wf) return fail(ctx, RSIM_ESTATE, "waveform not set");
  if (!ctx->have_arr) return fail(ctx, RSIM_ESTATE, "array not set");
  return RSIM_OK;
}

std::vector<DevScene> scene_views(rsim_ctx *ctx, const std::vector<int32_t> &ids, void *echo,
                                  uint32_t *vis_mask, int precision, const EchoShape &sh) {
  const RadarConst rc = radar_const(ctx);
  const size_t csize = precision ? 16 : 8;
  const int64_t cube = static_cast<int64_t>(sh.O) * rc.N * rc.M;
  std::vector<DevScene> ds(ids.size());
  int64_t mask_off = 0;
  for (size_t i = 0; i < ids.size(); ++i) {
    SceneRec &sc = ctx->scenes[ids[i]];
    uint32_t *mask = vis_mask ? vis_mask + mask_off : sc.d_mask;
    mask_off += static_cast<int64_t>(ctx->ground ? 4 : 1) * rc.N * ((sc.n_facets + 31) / 32);
    ds[i] = dev_scene(sc, mask, static_cast<char *>(echo) + i * cube * csize);
    if (ctx->dbounce && sc.d_db) {
      // the connection table follows the scene's mask words in a caller's mask buffer
      const int64_t plane = 2 * static_cast<int64_t>(rc.N) * std::max<int64_t>(1, sc.n_facets);
      ds[i].db_on = 1;
      ds[i].db_b = sc.d_db;
      if (vis_mask) {
        ds[i].db_b = reinterpret_cast<const int32_t *>(vis_mask + mask_off);
        mask_off += 2 * static_cast<int64_t>(rc.N) * sc.n_facets;
      }
      ds[i].db_idx = sc.d_db + plane;
      ds[i].db_cnt = sc.d_db + 2 * plane;
      ds[i].db_gamma_re = ctx->db_gamma_re;
      ds[i].db_gamma_im = ctx->db_gamma_im;
      ds[i].db_n = rc.N;
    }
    // a traversal keeps at most three pending nodes per level of its four-wide BVH
    int depth = 0;
    for (const InstRec &r : sc.inst) depth = std::max(depth, ctx->meshes[r.mesh].depth);
    ds[i].stack_depth = 3 * (depth + 1);
  }
  return ds;
}

// Upload (synchronously, after draining `s`) the tables of a persistent launch unless the
// same tables are already resident.
int32_t prepare_batch(rsim_ctx *ctx, BatchTables &bt, const std::vector<int32_t> &ids,
                      const std::vector<DevScene> &ds, void *echo, uint32_t *vis_mask,
                      int precision, int mb, const EchoShape &sh, hipStream_t s) {
  const RadarConst rc = radar_const(ctx);
  if (bt.d_items && bt.ids == ids && bt.echo == echo && bt.mask == vis_mask &&
      bt.version == ctx->version && bt.mb == mb && bt.precision == precision)
    return RSIM_OK;
  std::vector<int> order(ds.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return ds[a].n_facets + ds[a].n_points > ds[b].n_facets + ds[b].n_points;
  });
  std::vector<int4> items;
  items.reserve(order.size() * rc.N * sh.m_tiles * sh.o_tiles);
  for (int si : order)
    for (int n = 0; n < rc.N; ++n)
      for (int mt = 0; mt < sh.m_tiles; ++mt)
        for (int ot = 0; ot < sh.o_tiles; ++ot) items.push_back(make_int4(si, n, mt, ot));
  HIP_TRY(ctx, hipStreamSynchronize(s));  // a previous launch may still read the tables
  if (bt.scenes_cap < ds.size()) {
    dev_free(ctx, bt.d_scenes);
    bt.d_scenes = nullptr;
    bt.scenes_cap = 0;
    int32_t r = dev_alloc(ctx, reinterpret_cast<void **>(&bt.d_scenes), sizeof(DevScene) * ds.size());
    if (r) return r;
    bt.scenes_cap = ds.size();
  }
  if (bt.items_cap < items.size()) {
    dev_free(ctx, bt.d_items);
    bt.d_items = nullptr;
    bt.items_cap = 0;
    int32_t r = dev_alloc(ctx, reinterpret_cast<void **>(&bt.d_items), sizeof(int4) * items.size());
    if (r) return r;
    bt.items_cap = items.size();
  }
  if (!bt.d_queue) {
    int32_t r = dev_alloc(ctx, reinterpret_cast<void **>(&bt.d_queue), 64);
    if (r) return r;
  }
  HIP_TRY(ctx, hipMemcpy(bt.d_scenes, ds.data(), sizeof(DevScene) * ds.size(), hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(bt.d_items, items.data(), sizeof(int4) * items.size(), hipMemcpyHostToDevice));
  bt.n_items = static_cast<int32_t>(items.size());
  bt.ids = ids;
  bt.echo = echo;
  bt.mask = vis_mask;
  bt.version = ctx->version;
  bt.mb = mb;
  bt.precision = precision;
  return RSIM_OK;
}

// Upload (synchronously, after draining `s`) the scene and unit tables of a batched NUFFT
// call unless the same tables are already resident.
int32_t prepare_nufft_batch(rsim_ctx *ctx, BatchTables &bt, const std::vector<int32_t> &ids,
                            const std::vector<DevScene> &ds, void *echo, uint32_t *vis_mask,
                            const SumPlan &pl, hipStream_t s) {
  if (bt.d_units && bt.ids == ids && bt.echo == echo && bt.mask == vis_mask &&
      bt.version == ctx->version && bt.mb == -1 && bt.precision == 0 &&
      bt.n_items == static_cast<int32_t>(pl.nu_units.size()))
    return RSIM_OK;
  HIP_TRY(ctx, hipStreamSynchronize(s));  // a previous launch may still read the tables
  auto grow = [&](void **p, size_t *cap, size_t need) -> int32_t {
    if (*cap >= need && *p) return RSIM_OK;
    dev_free(ctx, *p);
    *p = nullptr;
    *cap = 0;
    int32_t r = dev_alloc(ctx, p, need);
    if (!r) *cap = need;
    return r;
  };
  size_t scap = bt.scenes_cap * sizeof(DevScene), ucap = bt.units_cap * sizeof(NuUnit);
  int32_t r;
  if ((r = grow(reinterpret_cast<void **>(&bt.d_scenes), &scap, sizeof(DevScene) * ds.size())))
    return r;
  bt.scenes_cap = scap / sizeof(DevScene);
  if ((r = grow(reinterpret_cast<void **>(&bt.d_units), &ucap,
                sizeof(NuUnit) * std::max<size_t>(1, pl.nu_units.size()))))
    return r;
  bt.units_cap = ucap / sizeof(NuUnit);
  HIP_TRY(ctx, hipMemcpy(bt.d_scenes, ds.data(), sizeof(DevScene) * ds.size(), hipMemcpyHostToDevice));
  HIP_TRY(ctx, hipMemcpy(bt.d_units, pl.nu_units.data(), sizeof(NuUnit) * pl.nu_units.size(),
                         hipMemcpyHostToDevice));
  bt.n_items = static_cast<int32_t>(pl.nu_units.size());
  bt.ids = ids;
  bt.echo = echo;
  bt.mask = vis_mask;
  bt.version = ctx->version;
  bt.mb = -1;
  bt.precision = 0;
  return RSIM_OK;
}

// Enqueue visibility + compaction + facet sum (kernels only; capturable).
int32_t enqueue_synthesis(rsim_ctx *ctx, const std::vector<DevScene> &ds, const BatchTables *bt,
                          hipStream_t s, const rsim_opts &o, bool timing, const SumPlan &pl) {
  RadarConst rc = radar_const(ctx);
  rc.intra = o.intra_chirp ? 1 : 0;
  const int precision = o.precision;
  const TunedShape ts = pl.ts;
  if (pl.nufft && pl.nb.census)
    HIP_TRY(ctx, launch_fill_zero(reinterpret_cast<float *>(pl.nb.census), 8 * kNuCensusSlots, s));
  const EchoShape sh = pl.sh;
  auto sum_plain = [&](const DevScene &d, const RadarConst &r, const double *elem,
                       const EchoShape &shk) {
    return pl.matrix ? launch_echo_mfma(d, r, elem, shk, s)
                     : launch_echo_plain(precision, ts.mb, ts.ft, d, r, elem, shk, s);
  };
  if (o.mask_mode == RSIM_MASK_COMPUTE) {
    stage_begin(ctx, timing, 0, s);
    for (auto &d : ds) HIP_TRY(ctx, launch_visibility(d, rc, 0, rc.N, s));
    stage_end(ctx, timing, 0, s);
  }
  if (!ctx->ground) {
    stage_begin(ctx, timing, 1, s);
    for (auto &d : ds) HIP_TRY(ctx, launch_compact(d, 0, rc.N, s));
    for (size_t i = 0; i < ds.size() && ctx->dbounce; ++i) {
      // facet-to-facet connections (computed, or given with the mask), then their lists
      const DevScene &d = ds[i];
      const int64_t plane = 2 * static_cast<int64_t>(rc.N) * std::max<int64_t>(1, d.n_facets);
      int32_t *work = const_cast<int32_t *>(d.db_idx) - plane;
      HIP_TRY(ctx, launch_dbounce(d, rc, o.mask_mode == RSIM_MASK_COMPUTE ? pl.db_ray_len[i] : 0.0,
                                  pl.db_r_lim[i], const_cast<int32_t *>(d.db_b), work + plane,
                                  work + 2 * plane, s));
    }
    stage_end(ctx, timing, 1, s);
    stage_begin(ctx, timing, 2, s);
    if (pl.nufft && bt) {
      // batched: one launch per stage over each chunk of (scene, chirp) units
      for (const auto &ch : pl.nu_chunks) {
        NuShape ns = pl.ns;
        ns.n_chirps = static_cast<int32_t>(ch[1]);
        ns.rec_stride = ch[2];
        ns.max_runs = static_cast<int32_t>(ch[3]);
        const NuBatch batch{bt->d_scenes, bt->d_units + ch[0]};
        HIP_TRY(ctx, launch_nufft(ds[0], rc, ctx->d_elem, ns, pl.nb, pl.tw, s, batch,
                                  kernel_events(ctx, timing, kKernelStage0)));
      }
    } else if (pl.nufft) {
      // per scene, in chirp chunks that fit the record buffer
      for (size_t i = 0; i < ds.size(); ++i) {
        NuShape ns = pl.nu_scene[i];
        for (int n0 = 0; n0 < rc.N; n0 += pl.ns.n_chirps) {
          ns.n0 = n0;
          ns.n_chirps = std::min(pl.ns.n_chirps, rc.N - n0);
          HIP_TRY(ctx, launch_nufft(ds[i], rc, ctx->d_elem, ns, pl.nb, pl.tw, s, NuBatch{},
                                    kernel_events(ctx, timing, kKernelStage0)));
        }
      }
    } else if (bt && pl.matrix) {
      int per_cu = 0;
      HIP_TRY(ctx, mfma_occupancy(rc.P, rc.Q, sh, &per_cu));
      const int groups = std::max(1, per_cu) * ctx->cu_count;
      HIP_TRY(ctx, launch_echo_mfma_persistent(bt->d_scenes, bt->d_items, bt->n_items, bt->d_queue,
                                               rc, ctx->d_elem, sh, groups, s));
    } else if (bt) {
      int per_cu = 0;
      HIP_TRY(ctx, echo_occupancy(precision, ts.mb, ts.ft, sh, &per_cu));
      const int groups = std::max(1, per_cu) * ctx->cu_count;
      HIP_TRY(ctx, launch_echo_persistent(precision, ts.mb, ts.ft, bt->d_scenes, bt->d_items,
                                          bt->n_items, bt->d_queue, rc, ctx->d_elem, sh, groups, s));
    } else {
      for (auto &d : ds) HIP_TRY(ctx, sum_plain(d, rc, ctx->d_elem, sh));
    }
    stage_end(ctx, timing, 2, s);
    return RSIM_OK;
  }
  // ground bounce: the four path types in turn, each its own mask set, elements
  // (images for the reflected sides) and factor gamma per bounce, summed into the echo
  const int E = rc.P + rc.Q;
  stage_begin(ctx, timing, 2, s);
  for (int k = 0; k < 4; ++k) {
    RadarConst rk = rc;
    if (k & 1) rk.tx_c[2] = 2.0 * ctx->z_ground - rc.tx_c[2];
    if (k >> 1) rk.rx_c[2] = 2.0 * ctx->z_ground - rc.rx_c[2];
    const double *elem = k ? ctx->d_elem_img + static_cast<size_t>(k - 1) * 3 * E : ctx->d_elem;
    EchoShape sk = sh;
    sk.accumulate = k ? 1 : 0;
    double gr = 1.0, gi = 0.0;
    for (int b = 0; b < ((k & 1) + (k >> 1)); ++b) {
      const double t = gr * ctx->gamma_re - gi * ctx->gamma_im;
      gi = gr * ctx->gamma_im + gi * ctx->gamma_re;
      gr = t;
    }
    sk.gamma_re = gr;
    sk.gamma_im = gi;
    for (size_t i = 0; i < ds.size(); ++i) {
      DevScene dk = ds[i];
      dk.mask = ds[i].mask + static_cast<int64_t>(k) * rc.N * ds[i].mask_words;
      HIP_TRY(ctx, launch_compact(dk, 0, rc.N, s));
      if (pl.nufft) {
        NuShape ns = pl.nu_scene[i];
        ns.accumulate = sk.accumulate;
        ns.gamma_re = sk.gamma_re;
        ns.gamma_im = sk.gamma_im;
        for (int n0 = 0; n0 < rc.N; n0 += pl.ns.n_chirps) {
          ns.n0 = n0;
          ns.n_chirps = std::min(pl.ns.n_chirps, rc.N - n0);
          HIP_TRY(ctx, launch_nufft(dk, rk, elem, ns, pl.nb, pl.tw, s));
        }
      } else {
        HIP_TRY(ctx, sum_plain(dk, rk, elem, sk));
      }
    }
  }
  stage_end(ctx, timing, 2, s);
  return RSIM_OK;
}

// Element positions of path types 1..3 (Tx images; Rx images; both) on the device.
int32_t ensure_elem_images(rsim_ctx *ctx) {
  if (ctx->d_elem_img && ctx->elem_img_version == ctx->version) return RSIM_OK;
  const size_t E = (ctx->tx.size() + ctx->rx.size()) / 3;
  std::vector<double> e(3 * 3 * E);
  for (int k = 1; k < 4; ++k) {
    double *dst = e.data() + (k - 1) * 3 * E;
    size_t j = 0;
    for (size_t p = 0; p < ctx->tx.size() / 3; ++p, ++j) {
      dst[3 * j] = ctx->tx[3 * p];
      dst[3 * j + 1] = ctx->tx[3 * p + 1];
      dst[3 * j + 2] = (k & 1) ? 2.0 * ctx->z_ground - ctx->tx[3 * p + 2] : ctx->tx[3 * p + 2];
    }
    for (size_t q = 0; q < ctx->rx.size() / 3; ++q, ++j) {
      dst[3 * j] = ctx->rx[3 * q];
      dst[3 * j + 1] = ctx->rx[3 * q + 1];
      dst[3 * j + 2] = (k >> 1) ? 2.0 * ctx->z_ground - ctx->rx[3 * q + 2] : ctx->rx[3 * q + 2];
    }
  }
  dev_free(ctx, ctx->d_elem_img);
  ctx->d_elem_img = nullptr;
  int32_t rc = upload(ctx, &ctx->d_elem_img, e.data(), e.size());
  if (rc) return rc;
  ctx->elem_img_version = ctx->version;
  return RSIM_OK;
}

}  // namespace

extern "C" {

int32_t rsim_abi_version(void) { return RSIM_ABI_VERSION; }

int32_t rsim_create(int32_t hip_device, rsim_ctx **out) {
  if (!out) return fail(nullptr, RSIM_EINVAL, "rsim_create: out is NULL");
  *out = nullptr;
  std::unique_ptr<rsim_ctx> ctx(new rsim_ctx());
  if (hip_device == -1) {
    ctx->host_only = true;
    *out = ctx.release();
    return RSIM_OK;
  }
  if (hip_device < 0) return fail(nullptr, RSIM_EINVAL, "rsim_create: bad device %d", hip_device);
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0)
    return fail(nullptr, RSIM_EDEVICE, "rsim_create: no HIP device (%s)",
                e != hipSuccess ? hipGetErrorString(e) : "count = 0");
  if (hip_device >= count)
    return fail(nullptr, RSIM_EDEVICE, "rsim_create: device %d of %d", hip_device, count);
  if ((e = hipSetDevice(hip_device)) != hipSuccess)
    return fail(nullptr, RSIM_EDEVICE, "hipSetDevice: %s", hipGetErrorString(e));
  hipDeviceProp_t prop;
  if ((e = hipGetDeviceProperties(&prop, hip_device)) != hipSuccess)
    return fail(nullptr, RSIM_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  ctx->device = hip_device;
  ctx->host_only = false;
  ctx->cu_count = prop.multiProcessorCount;
  ctx->max_lds = prop.sharedMemPerBlock;
  for (int k = 0; k < kStages; ++k) {
    if (hipEventCreate(&ctx->ev0[k]) != hipSuccess || hipEventCreate(&ctx->ev1[k]) != hipSuccess)
      return fail(nullptr, RSIM_EDEVICE, "hipEventCreate failed");
  }
  if ((e = hipStreamCreateWithFlags(&ctx->capture_stream, hipStreamNonBlocking)) != hipSuccess)
    return fail(nullptr, RSIM_EDEVICE, "hipStreamCreate: %s", hipGetErrorString(e));
  if ((e = static_scratch_address(hip_device, &ctx->static_scratch)) != hipSuccess)
    return fail(nullptr, RSIM_EDEVICE, "hipGetSymbolAddress of the static work array: %s",
                hipGetErrorString(e));
  *out = ctx.release();
  return RSIM_OK;
}

void rsim_destroy(rsim_ctx *ctx) {
  if (!ctx) return;
  if (!ctx->host_only) {
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    if (ctx->graph.exec) (void)hipGraphExecDestroy(ctx->graph.exec);
    if (ctx->graph.graph) (void)hipGraphDestroy(ctx->graph.graph);
    for (auto &kv : ctx->allocs) (void)hipFree(kv.first);
    for (int k = 0; k < kStages; ++k) {
      if (ctx->ev0[k]) (void)hipEventDestroy(ctx->ev0[k]);
      if (ctx->ev1[k]) (void)hipEventDestroy(ctx->ev1[k]);
    }
    for (auto &pool : ctx->kern_ev)
      for (hipEvent_t e : pool) (void)hipEventDestroy(e);
    if (ctx->capture_stream) (void)hipStreamDestroy(ctx->capture_stream);
  }
  delete ctx;
}

const char *rsim_last_error(const rsim_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_thread_error.c_str();
}

int32_t rsim_set_mem_limit(rsim_ctx *ctx, uint64_t bytes) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  ctx->mem_limit = bytes;
  return RSIM_OK;
}

int32_t rsim_load_mesh(rsim_ctx *ctx, const float *verts_xyz, int64_t n_verts, const int32_t *tris,
                       int64_t n_tris, int32_t *mesh_id) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!mesh_id || n_verts < 0 || n_tris < 0 || (n_verts && !verts_xyz) || (n_tris && !tris))
    return fail(ctx, RSIM_EINVAL, "rsim_load_mesh: bad pointer or count");
  if (n_tris > (int64_t(1) << 26) || n_verts > (int64_t(1) << 31) - 1)
    return fail(ctx, RSIM_ERANGE, "rsim_load_mesh: %lld triangles exceed 2^26", (long long)n_tris);
  for (int64_t i = 0; i < 3 * n_verts; ++i)
    if (!std::isfinite(verts_xyz[i]))
      return fail(ctx, RSIM_EINVAL, "rsim_load_mesh: vertex coordinate %lld is not finite", (long long)i);
  for (int64_t i = 0; i < 3 * n_tris; ++i)
    if (tris[i] < 0 || tris[i] >= n_verts)
      return fail(ctx, RSIM_EINVAL, "rsim_load_mesh: triangle index %lld = %d out of range", (long long)i, tris[i]);
  MeshRec m;
  m.verts.assign(verts_xyz, verts_xyz + 3 * n_verts);
  m.tris.assign(tris, tris + 3 * n_tris);
  int32_t rc = index_mesh(ctx, m, true);
  if (rc) return rc;
  ctx->meshes.push_back(std::move(m));
  *mesh_id = static_cast<int32_t>(ctx->meshes.size() - 1);
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_update_mesh(rsim_ctx *ctx, int32_t mesh_id, const float *verts_xyz, int64_t n_verts) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (mesh_id < 0 || mesh_id >= static_cast<int32_t>(ctx->meshes.size()))
    return fail(ctx, RSIM_EINVAL, "unknown mesh id %d", mesh_id);
  MeshRec &m = ctx->meshes[mesh_id];
  if (!verts_xyz || n_verts != static_cast<int64_t>(m.verts.size() / 3))
    return fail(ctx, RSIM_EINVAL, "rsim_update_mesh: need %lld vertices",
                (long long)(m.verts.size() / 3));
  for (int64_t i = 0; i < 3 * n_verts; ++i)
    if (!std::isfinite(verts_xyz[i]))
      return fail(ctx, RSIM_EINVAL, "rsim_update_mesh: vertex coordinate %lld is not finite", (long long)i);
  if (!ctx->host_only) {
    int32_t rc = need_device(ctx);
    if (rc) return rc;
    HIP_TRY(ctx, hipDeviceSynchronize());  // kernels may still read the old copies
  }
  m.verts.assign(verts_xyz, verts_xyz + 3 * n_verts);
  int32_t rc = index_mesh(ctx, m, false);
  if (rc) return rc;
  for (auto &sc : ctx->scenes) sc.dirty = true;  // instance tables hold mesh pointers
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_set_instance_motion(rsim_ctx *ctx, int32_t scene_id, int32_t inst_id,
                                 const double pos0[3], const double vel[3]) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  int32_t rc = check_scene(ctx, scene_id);
  if (rc) return rc;
  SceneRec &sc = ctx->scenes[scene_id];
  if (inst_id < 0 || inst_id >= static_cast<int32_t>(sc.inst.size()))
    return fail(ctx, RSIM_EINVAL, "unknown instance id %d", inst_id);
  if (!pos0 || !vel || !finite_all(pos0, 3) || !finite_all(vel, 3))
    return fail(ctx, RSIM_EINVAL, "rsim_set_instance_motion: bad position or velocity");
  if (!ctx->host_only) {
    if ((rc = need_device(ctx))) return rc;
    HIP_TRY(ctx, hipDeviceSynchronize());
  }
  std::memcpy(sc.inst[inst_id].pos0, pos0, sizeof(double) * 3);
  std::memcpy(sc.inst[inst_id].vel, vel, sizeof(double) * 3);
  sc.dirty = true;
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_create_scene(rsim_ctx *ctx, int32_t *scene_id) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!scene_id) return fail(ctx, RSIM_EINVAL, "scene_id is NULL");
  ctx->scenes.emplace_back();
  *scene_id = static_cast<int32_t>(ctx->scenes.size() - 1);
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_add_instance(rsim_ctx *ctx, int32_t scene_id, int32_t mesh_id, const double rot[9],
                          const double pos0[3], const double vel[3], int32_t *inst_id) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  int32_t rc = check_scene(ctx, scene_id);
  if (rc) return rc;
  if (mesh_id < 0 || mesh_id >= static_cast<int32_t>(ctx->meshes.size()))
    return fail(ctx, RSIM_EINVAL, "unknown mesh id %d", mesh_id);
  if (!rot || !pos0 || !vel) return fail(ctx, RSIM_EINVAL, "rsim_add_instance: NULL argument");
  if (!finite_all(rot, 9) || !finite_all(pos0, 3) || !finite_all(vel, 3))
    return fail(ctx, RSIM_EINVAL, "rsim_add_instance: non-finite pose");
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double d = 0;
      for (int k = 0; k < 3; ++k) d += rot[3 * k + i] * rot[3 * k + j];
      if (std::fabs(d - (i == j ? 1.0 : 0.0)) > 1e-6)
        return fail(ctx, RSIM_EINVAL, "rsim_add_instance: rotation is not orthonormal");
    }
  SceneRec &sc = ctx->scenes[scene_id];
  if (sc.inst.size() >= 4096) return fail(ctx, RSIM_ERANGE, "more than 4096 instances");
  InstRec r;
  r.mesh = mesh_id;
  std::memcpy(r.rot, rot, sizeof(r.rot));
  std::memcpy(r.pos0, pos0, sizeof(r.pos0));
  std::memcpy(r.vel, vel, sizeof(r.vel));
  sc.inst.push_back(r);
  sc.n_facets += static_cast<int64_t>(ctx->meshes[mesh_id].tris.size() / 3);
  if (sc.n_facets > (int64_t(1) << 30)) return fail(ctx, RSIM_ERANGE, "scene exceeds 2^30 facets");
  sc.dirty = true;
  ctx->version++;
  if (inst_id) *inst_id = static_cast<int32_t>(sc.inst.size() - 1);
  return RSIM_OK;
}

int32_t rsim_add_points(rsim_ctx *ctx, int32_t scene_id, const double *pos0, const double *vel,
                        const double *amp_re_im, int64_t n) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  int32_t rc = check_scene(ctx, scene_id);
  if (rc) return rc;
  if (n < 0 || (n && (!pos0 || !vel || !amp_re_im)))
    return fail(ctx, RSIM_EINVAL, "rsim_add_points: bad pointer or count");
  if (!finite_all(pos0, 3 * n) || !finite_all(vel, 3 * n) || !finite_all(amp_re_im, 2 * n))
    return fail(ctx, RSIM_EINVAL, "rsim_add_points: non-finite input");
  SceneRec &sc = ctx->scenes[scene_id];
  if (sc.pt_amp.size() / 2 + n > (1 << 24)) return fail(ctx, RSIM_ERANGE, "too many points");
  sc.pt_pos.insert(sc.pt_pos.end(), pos0, pos0 + 3 * n);
  sc.pt_vel.insert(sc.pt_vel.end(), vel, vel + 3 * n);
  sc.pt_amp.insert(sc.pt_amp.end(), amp_re_im, amp_re_im + 2 * n);
  sc.dirty = true;
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_scene_info(rsim_ctx *ctx, int32_t scene_id, int64_t *n_facets, int64_t *mask_words) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  int32_t rc = check_scene(ctx, scene_id);
  if (rc) return rc;
  const SceneRec &sc = ctx->scenes[scene_id];
  if (n_facets) *n_facets = sc.n_facets;
  if (mask_words) *mask_words = (sc.n_facets + 31) / 32;
  return RSIM_OK;
}

int32_t rsim_set_waveform(rsim_ctx *ctx, const rsim_waveform *wf) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!wf) return fail(ctx, RSIM_EINVAL, "waveform is NULL");
  const double v[4] = {wf->f0_hz, wf->slope_hz_per_s, wf->fs_hz, wf->chirp_period_s};
  if (!finite_all(v, 4) || wf->f0_hz <= 0 || wf->fs_hz <= 0 || wf->chirp_period_s <= 0 ||
      wf->slope_hz_per_s == 0)
    return fail(ctx, RSIM_EINVAL, "rsim_set_waveform: f0, fs, chirp period must be > 0, slope != 0");
  if (wf->n_samples < 1 || wf->n_samples > 4096 || wf->n_chirps < 1 || wf->n_chirps > 4096)
    return fail(ctx, RSIM_ERANGE, "rsim_set_waveform: M and N must be in 1..4096");
  ctx->wf = *wf;
  ctx->have_wf = true;
  for (auto &sc : ctx->scenes) sc.buf_N = sc.buf_N == wf->n_chirps ? sc.buf_N : -1;
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_set_array(rsim_ctx *ctx, const double *tx_xyz, int32_t n_tx, const double *rx_xyz,
                       int32_t n_rx) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!tx_xyz || !rx_xyz) return fail(ctx, RSIM_EINVAL, "rsim_set_array: NULL positions");
  if (n_tx < 1 || n_tx > 64 || n_rx < 1 || n_rx > 64)
    return fail(ctx, RSIM_ERANGE, "rsim_set_array: 1..64 Tx and 1..64 Rx elements");
  if (!finite_all(tx_xyz, 3 * n_tx) || !finite_all(rx_xyz, 3 * n_rx))
    return fail(ctx, RSIM_EINVAL, "rsim_set_array: non-finite position");
  if (ctx->ground) {
    for (int32_t k = 0; k < n_tx; ++k)
      if (!(tx_xyz[3 * k + 2] > ctx->z_ground))
        return fail(ctx, RSIM_ERANGE, "rsim_set_array: elements must lie above the ground plane");
    for (int32_t k = 0; k < n_rx; ++k)
      if (!(rx_xyz[3 * k + 2] > ctx->z_ground))
        return fail(ctx, RSIM_ERANGE, "rsim_set_array: elements must lie above the ground plane");
  }
  ctx->tx.assign(tx_xyz, tx_xyz + 3 * n_tx);
  ctx->rx.assign(rx_xyz, rx_xyz + 3 * n_rx);
  if (!ctx->host_only) {
    int32_t rc = need_device(ctx);
    if (rc) return rc;
    dev_free(ctx, ctx->d_elem);
    ctx->d_elem = nullptr;
    std::vector<double> e(ctx->tx);
    e.insert(e.end(), ctx->rx.begin(), ctx->rx.end());
    if ((rc = upload(ctx, &ctx->d_elem, e.data(), e.size()))) return rc;
  }
  ctx->have_arr = true;
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_set_ground(rsim_ctx *ctx, int32_t enable, double z_ground, double gamma_re,
                        double gamma_im) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if ((enable != 0 && enable != 1) || !std::isfinite(z_ground) || !std::isfinite(gamma_re) ||
      !std::isfinite(gamma_im))
    return fail(ctx, RSIM_EINVAL, "rsim_set_ground: enable 0/1 and finite plane and gamma");
  if (enable && ctx->have_arr) {
    for (size_t k = 2; k < ctx->tx.size(); k += 3)
      if (!(ctx->tx[k] > z_ground))
        return fail(ctx, RSIM_ERANGE, "rsim_set_ground: array elements must lie above the plane");
    for (size_t k = 2; k < ctx->rx.size(); k += 3)
      if (!(ctx->rx[k] > z_ground))
        return fail(ctx, RSIM_ERANGE, "rsim_set_ground: array elements must lie above the plane");
  }
  ctx->ground = enable != 0;
  ctx->z_ground = z_ground;
  ctx->gamma_re = gamma_re;
  ctx->gamma_im = gamma_im;
  for (SceneRec &sc : ctx->scenes) sc.dirty = true;  // instance in-plane flags
  ctx->version++;
  return RSIM_OK;
}

int32_t rsim_set_double_bounce(rsim_ctx *ctx, int32_t enable, double gamma_re,
                               double gamma_im) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if ((enable != 0 && enable != 1) || !std::isfinite(gamma_re) || !std::isfinite(gamma_im))
    return fail(ctx, RSIM_EINVAL, "rsim_set_double_bounce: enable 0/1 and a finite gamma");
  ctx->dbounce = enable != 0;
  ctx->db_gamma_re = gamma_re;
  ctx->db_gamma_im = gamma_im;
  ctx->version++;  // captured graphs hold the old entries
  return RSIM_OK;
}

int32_t rsim_set_nufft_chunk(rsim_ctx *ctx, int32_t max_chirps) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (max_chirps < 0)
    return fail(ctx, RSIM_EINVAL, "rsim_set_nufft_chunk: max_chirps %d < 0", max_chirps);
  ctx->nu_chunk_max = max_chirps;
  return RSIM_OK;
}

int32_t rsim_set_backward_kernel(rsim_ctx *ctx, int32_t kernel) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (kernel < RSIM_KERNEL_AUTO || kernel > RSIM_KERNEL_NUFFT)
    return fail(ctx, RSIM_EINVAL, "rsim_set_backward_kernel: unknown kernel %d", kernel);
  ctx->bwd_kernel = kernel;
  return RSIM_OK;
}

int32_t rsim_set_backward_intra_chirp(rsim_ctx *ctx, int32_t enable) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (enable != 0 && enable != 1)
    return fail(ctx, RSIM_EINVAL, "rsim_set_backward_intra_chirp: enable must be 0 or 1");
  ctx->bwd_intra = enable;
  return RSIM_OK;
}

int32_t rsim_synthesize(rsim_ctx *ctx, const int32_t *scene_ids, int32_t n_scenes, void *echo,
                        uint32_t *vis_mask, void *hip_stream, const rsim_opts *opts) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  rsim_opts o{};
  if (opts) o = *opts;
  if (!scene_ids || n_scenes < 1 || !echo)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: need scene ids and an echo buffer");
  if (o.precision != RSIM_FP32_PHASE64 && o.precision != RSIM_FP64)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: unknown precision %d", o.precision);
  if (o.mask_mode != RSIM_MASK_COMPUTE && o.mask_mode != RSIM_MASK_INPUT)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: unknown mask mode %d", o.mask_mode);
  if (o.mask_mode == RSIM_MASK_INPUT && !vis_mask)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: RSIM_MASK_INPUT needs vis_mask");
  if (o.intra_chirp != 0 && o.intra_chirp != 1)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: intra_chirp must be 0 or 1");
  if (o.intra_chirp && o.precision == RSIM_FP64)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: the intra-chirp delay is implemented in the "
                "FP32 sum only");
  if (o.kernel < RSIM_KERNEL_AUTO || o.kernel > RSIM_KERNEL_NUFFT)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: unknown kernel %d", o.kernel);
  if (o.kernel == RSIM_KERNEL_MATRIX && o.precision != RSIM_FP32_PHASE64)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: the matrix-core facet sum is FP32 only");
  if (o.kernel == RSIM_KERNEL_NUFFT && o.precision != RSIM_FP32_PHASE64)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: the NUFFT facet sum is FP32 only");
  if (ctx->ground && o.persistent)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: the ground bounce runs with plain launches "
                "(persistent = 0)");
  if (o.census && o.use_graph)
    return fail(ctx, RSIM_EINVAL, "rsim_synthesize: census is not taken under a captured graph");
  if (ctx->dbounce) {
    if (o.precision != RSIM_FP32_PHASE64 || o.kernel == RSIM_KERNEL_VECTOR ||
        o.kernel == RSIM_KERNEL_MATRIX)
      return fail(ctx, RSIM_EINVAL, "rsim_synthesize: the facet-to-facet double bounce is "
                  "implemented in the NUFFT facet sum only (FP32, kernel AUTO or NUFFT)");
    if (o.intra_chirp || o.persistent || ctx->ground)
      return fail(ctx, RSIM_EINVAL, "rsim_synthesize: the facet-to-facet double bounce runs "
                  "stop-and-hop, with plain launches and without the ground plane");
  }
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  std::vector<int32_t> ids(scene_ids, scene_ids + n_scenes);
  for (int32_t id : ids)
    if ((rc = check_scene(ctx, id))) return rc;
  const RadarConst rcn = radar_const(ctx);
  const double eps = cross_term_bound(ctx, rcn);
  // cross-term factor exp(j eps): first order in the FP32 sum (error eps^2/2 below
  // FP32 rounding for eps <= 3e-4), fourth order in the FP64 sum (eps <= 1e-3)
  const double eps_limit = o.precision == RSIM_FP64 ? 1e-3 : 3e-4;
  if (eps > eps_limit)
    return fail(ctx, RSIM_ERANGE,
                "array aperture too large: |2 pi slope d_p e_q| may reach %.3g rad (limit %.1g)",
                eps, eps_limit);
  if (o.kernel == RSIM_KERNEL_MATRIX) {
    if (const char *why = matrix_ineligible(ctx, rcn, o.precision))
      return fail(ctx, RSIM_ERANGE, "rsim_synthesize: %s", why);
  }
  const double r_max = scenes_rmax(ctx, ids), v_max = scenes_vmax(ctx, ids);
  if (o.kernel == RSIM_KERNEL_NUFFT || ctx->dbounce) {
    NuShape tmp{};
    if (const char *why = nufft_ineligible(ctx, rcn, o, r_max, v_max, &tmp))
      return fail(ctx, RSIM_ERANGE, "rsim_synthesize: %s", why);
  }
  SumPlan pl = plan_sum(ctx, rcn, o, r_max, v_max);
  if (ctx->dbounce) {
    // per scene: a reflected ray is followed across the scene's extent over the frame
    // (the union of its instances' world boxes at the first and last chirp); the
    // footprint limit is its largest facet radius
    const double T = (rcn.N - 1) * rcn.tc;
    for (int32_t id : ids) {
      double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
      for (const InstRec &r : ctx->scenes[id].inst) {
        const MeshRec &m = ctx->meshes[r.mesh];
        for (int corner = 0; corner < 8; ++corner) {
          const double b[3] = {(corner & 1) ? m.box_hi[0] : m.box_lo[0],
                               (corner & 2) ? m.box_hi[1] : m.box_lo[1],
                               (corner & 4) ? m.box_hi[2] : m.box_lo[2]};
          for (int q = 0; q < 3; ++q) {
            const double x = r.rot[3 * q] * b[0] + r.rot[3 * q + 1] * b[1] + r.rot[3 * q + 2] * b[2] +
                             r.pos0[q];
            for (const double tt : {0.0, T}) {
              lo[q] = std::min(lo[q], x + r.vel[q] * tt);
              hi[q] = std::max(hi[q], x + r.vel[q] * tt);
            }
          }
        }
      }
      double diag = 0.0;
      for (int q = 0; q < 3; ++q) diag += hi[q] > lo[q] ? (hi[q] - lo[q]) * (hi[q] - lo[q]) : 0.0;
      pl.db_ray_len.push_back(std::sqrt(diag) + 1.0);
      pl.db_r_lim.push_back(scenes_rmax(ctx, {id}));
    }
  }
  const TunedShape ts = pl.ts;
  if (!pl.matrix && !pl.nufft && !echo_variant_exists(o.precision, ts.mb, ts.ft))
    return fail(ctx, RSIM_EINVAL, "no facet-sum variant with tile_m=%d tile_f=%d", ts.mb, ts.ft);
  if ((rc = need_device(ctx))) return rc;
  if (pl.nufft) {
    // twiddles of the grid length and the record buffer (both before any capture);
    // a reallocated buffer invalidates captured graphs
    pl.tw = twiddles(ctx, pl.ns.ng, 0, &rc);
    if (rc) return rc;
    // reach, run length and run bound per scene (from its own meshes); the buffers hold
    // the largest scene
    int64_t stride = 1;
    int32_t max_runs = 1;
    const size_t rec_b = nufft_record_bytes(o.intra_chirp != 0);
    pl.nu_scene.clear();
    for (int32_t id : ids) {
      // eligible, since the call's largest r_max is
      NuShape si{};
      (void)nufft_ineligible(ctx, rcn, o, scenes_rmax(ctx, {id}), v_max, &si);
      si.rec_stride = std::max<int64_t>(
          1, ctx->scenes[id].n_facets * (ctx->dbounce ? 3 : 1) +
                 static_cast<int64_t>(ctx->scenes[id].pt_amp.size() / 2));
      si.run_len = nufft_run_len(ctx, si.rec_stride, rcn.N);
      si.max_runs = nufft_max_runs(si, si.rec_stride);
      stride = std::max(stride, si.rec_stride);
      max_runs = std::max(max_runs, si.max_runs);
      pl.nu_scene.push_back(si);
    }
    const int64_t O = static_cast<int64_t>(rcn.P) * rcn.Q;
    // the layout only grows while channels, grid and record size stay: calls on
    // smaller scenes reuse it, so captured graphs stay valid
    (void)0;
    nufft_fft_groups(ctx, rcn, pl.ns, sizeof(int32_t) * max_runs);
    for (NuShape &si : pl.nu_scene) {
      si.cb = pl.ns.cb;
      si.groups = pl.ns.groups;
    }
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const size_t run_b = sizeof(int4) + static_cast<size_t>(O) * kNuSlots * sizeof(float2);
    // work-buffer extents: records (and keys, positions), runs and units per launch
    int64_t ext_rec = 0, ext_run = 0, chunk = 0;
    const size_t budget = nufft_budget(ctx, ctx->nu_buf_bytes);
    pl.nu_units.clear();
    pl.nu_chunks.clear();
    if (o.persistent) {
      // batched: (scene, chirp) units, the scenes with the most records first, cut into
      // launches of at most the work-buffer budget and 65535 units
      std::vector<int> order(ids.size());
      for (size_t i = 0; i < order.size(); ++i) order[i] = static_cast<int>(i);
      std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return pl.nu_scene[a].rec_stride > pl.nu_scene[c].rec_stride;
      });
      int64_t u0 = 0, rec = 0, run = 0, big_s = 0, big_r = 0;
      auto close = [&]() {
        const int64_t n_u = static_cast<int64_t>(pl.nu_units.size()) - u0;
        if (n_u <= 0) return;
        pl.nu_chunks.push_back({u0, n_u, big_s, big_r});
        ext_rec = std::max(ext_rec, rec);
        ext_run = std::max(ext_run, run);
        chunk = std::max(chunk, n_u);
        u0 = static_cast<int64_t>(pl.nu_units.size());
        rec = run = big_s = big_r = 0;
      };
      for (int i : order) {
        const NuShape &si = pl.nu_scene[i];
        const size_t unit_b = si.rec_stride * (rec_b + 8) + si.max_runs * run_b + 4;
        for (int n = 0; n < rcn.N; ++n) {
          const size_t used = rec * (rec_b + 8) + run * run_b +
                              4 * (static_cast<size_t>(pl.nu_units.size()) - u0);
          if (static_cast<int64_t>(pl.nu_units.size()) > u0 &&
              (used + unit_b > budget ||
               static_cast<int64_t>(pl.nu_units.size()) - u0 >= 65535))
            close();
          NuUnit un{};
          un.scene = i;
          un.n = n;
          un.rec_base = rec;
          un.rec_stride = si.rec_stride;
          un.run_base = run;
          un.max_runs = si.max_runs;
          un.run_len = si.run_len;
          un.b0 = si.b0;
          un.kspan = si.kspan;
          pl.nu_units.push_back(un);
          rec += si.rec_stride;
          run += si.max_runs;
          big_s = std::max(big_s, si.rec_stride);
          big_r = std::max<int64_t>(big_r, si.max_runs);
        }
      }
      close();
    } else {
      const size_t per_chirp = stride * (rec_b + 8) + max_runs * run_b + 4;
      chunk = std::max<int64_t>(1, std::min<int64_t>(rcn.N, budget / per_chirp));
      if (ctx->nu_chunk_max > 0) chunk = std::min<int64_t>(chunk, ctx->nu_chunk_max);
      ext_rec = chunk * stride;
      ext_run = chunk * max_runs;
    }
    const size_t off_pos = al(ext_rec * 4);
    const size_t off_srec = off_pos + al(ext_rec * 4);
    const size_t off_runs = off_srec + al(ext_rec * rec_b);
    const size_t off_nruns = off_runs + al(ext_run * sizeof(int4));
    const size_t off_part = off_nruns + al(chunk * 4);
    const size_t total = off_part + ext_run * static_cast<size_t>(O) * kNuSlots * sizeof(float2);
    const std::array<int64_t, 6> layout{ext_rec, chunk, O, pl.ns.ng, static_cast<int64_t>(rec_b),
                                        ext_run};
    if (ctx->nu_buf_bytes < total) {
      HIP_TRY(ctx, hipDeviceSynchronize());  // earlier launches may still use the buffer
      dev_free(ctx, ctx->nu_buf);
      ctx->nu_buf = nullptr;
      ctx->nu_buf_bytes = 0;
      ctx->nu_layout = {};
      if ((rc = dev_alloc(ctx, &ctx->nu_buf, total))) return rc;
      ctx->nu_buf_bytes = total;
    }
    if (layout != ctx->nu_layout) {
      ctx->nu_layout = layout;
      ctx->version++;  // captured graphs hold the old layout
    }
    char *b = static_cast<char *>(ctx->nu_buf);
    pl.nb = NuBuffers{reinterpret_cast<int32_t *>(b), reinterpret_cast<int32_t *>(b + off_pos),
                      b + off_srec, reinterpret_cast<float2 *>(b + off_part), rec_b, nullptr,
                      reinterpret_cast<int4 *>(b + off_runs), reinterpret_cast<int32_t *>(b + off_nruns)};
    if (o.census) {
      if (!ctx->d_census) {
        void *p = nullptr;
        if ((rc = dev_alloc(ctx, &p, sizeof(unsigned long long) * 4 * kNuCensusSlots))) return rc;
        ctx->d_census = static_cast<unsigned long long *>(p);
      }
      pl.nb.census = ctx->d_census;
    }
    pl.ns.n_chirps = static_cast<int32_t>(chunk);
    pl.ns.max_runs = max_runs;
    if (nufft_sort_smem_bytes(pl.ns) > ctx->max_lds)
      return fail(ctx, RSIM_ERANGE, "NUFFT sort needs %zu bytes of LDS (max %zu)",
                  nufft_sort_smem_bytes(pl.ns), ctx->max_lds);
  }
  const EchoShape sh = pl.sh;
  const size_t lds = pl.nufft    ? nufft_fft_smem_bytes(pl.ns)
                     : pl.matrix ? mfma_smem_bytes(sh)
                                 : echo_smem_bytes(o.precision, ts.mb, ts.ft, sh);
  if (lds > ctx->max_lds)
    return fail(ctx, RSIM_ERANGE, "facet-sum tile needs %zu bytes of LDS (max %zu)", lds,
                ctx->max_lds);
  for (int32_t id : ids)
    if ((rc = ensure_scene_device(ctx, ctx->scenes[id]))) return rc;
  if (ctx->ground && (rc = ensure_elem_images(ctx))) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool timing = o.timing != 0;
  timing_reset(ctx, timing);
  const std::vector<DevScene> ds = scene_views(ctx, ids, echo, vis_mask, o.precision, sh);
  if (o.use_graph) {
    // Capture once per (scenes, buffers, options, scene/radar version); replay after.
    GraphCache &g = ctx->graph;
    const bool hit = g.valid && g.ids == ids && g.echo == echo && g.mask == vis_mask &&
                     g.version == ctx->version && std::memcmp(&g.opts, &o, sizeof(o)) == 0;
    if (!hit) {
      HIP_TRY(ctx, hipStreamSynchronize(s));  // an older replay may still be running
      if (g.exec) (void)hipGraphExecDestroy(g.exec);
      if (g.graph) (void)hipGraphDestroy(g.graph);
      g.exec = nullptr;
      g.graph = nullptr;
      g.valid = false;
      if (o.persistent && pl.nufft &&
          (rc = prepare_nufft_batch(ctx, g.tables, ids, ds, echo, vis_mask, pl, s)))
        return rc;
      if (o.persistent && !pl.nufft &&
          (rc = prepare_batch(ctx, g.tables, ids, ds, echo, vis_mask, o.precision, pl.batch_key,
                              sh, s)))
        return rc;
      HIP_TRY(ctx, hipStreamBeginCapture(ctx->capture_stream, hipStreamCaptureModeRelaxed));
      int32_t rc2 = enqueue_synthesis(ctx, ds, o.persistent ? &g.tables : nullptr,
                                      ctx->capture_stream, o, false, pl);
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamEndCapture(ctx->capture_stream, &graph);
      if (rc2) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc2;
      }
      if (e != hipSuccess) return fail(ctx, RSIM_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
      e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return fail(ctx, RSIM_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
      }
      g.graph = graph;
      g.valid = true;
      g.ids = ids;
      g.echo = echo;
      g.mask = vis_mask;
      g.version = ctx->version;
      g.opts = o;
    }
    stage_begin(ctx, timing, 2, s);
    HIP_TRY(ctx, hipGraphLaunch(g.exec, s));
    stage_end(ctx, timing, 2, s);
    return RSIM_OK;
  }
  if (o.persistent && pl.nufft &&
      (rc = prepare_nufft_batch(ctx, ctx->batch, ids, ds, echo, vis_mask, pl, s)))
    return rc;
  if (o.persistent && !pl.nufft &&
      (rc = prepare_batch(ctx, ctx->batch, ids, ds, echo, vis_mask, o.precision, pl.batch_key, sh,
                          s)))
    return rc;
  if (o.census) ctx->census_ready = false;
  if ((rc = enqueue_synthesis(ctx, ds, o.persistent ? &ctx->batch : nullptr, s, o, timing, pl)))
    return rc;
  if (o.census) ctx->census_ready = pl.nufft;
  return RSIM_OK;
}

// NUFFT adjoint of one scene's facet sum into ctx->adj_partial (one slot per chirp and lit
// facet), then the shared chain rule into ctx->adj_gxw. Work buffers per chunk of chirps:
// records and adjoint records [chunk][facet records] in entry order, the two class lists,
// their cells and the lists ordered by cell [chunk][2][facet records], grids [chunk][O][n_g].
static int32_t enqueue_nufft_adjoint(rsim_ctx *ctx, const DevScene &d_in, const RadarConst &rcn,
                                     const double *elem, NuShape ns, const void *grad_echo,
                                     bool accumulate, hipStream_t s, double *dbsum = nullptr,
                                     double *dbtsum = nullptr) {
  DevScene d = d_in;
  d.n_points = 0;  // points carry no parameters
  const int64_t F = d.n_facets, N = rcn.N, O = static_cast<int64_t>(rcn.P) * rcn.Q;
  const int64_t E = rcn.P + rcn.Q;
  const bool db = d.db_on != 0;
  // entries per chirp: the lit facets, then (double bounce) up to 2 F connections
  const int64_t stride = std::max<int64_t>(1, db ? 3 * F : F);
  const int64_t db_stride = db ? std::max<int64_t>(1, 2 * F) : 0;
  const int64_t ncls = db ? 4 : 2;
  const size_t rec_b = nufft_record_bytes(false), der_b = nufft_der_bytes();
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t per_chirp = stride * (rec_b + der_b + 12 * ncls) + 4 * ncls + O * ns.ng * 8 +
                           db_stride * (kAdjSlotFloats + E) * 4;
  int64_t chunk = std::max<int64_t>(
      1, std::min<int64_t>(N, nufft_budget(ctx, ctx->nu_adj_bytes) / per_chirp));
  if (ctx->nu_chunk_max > 0) chunk = std::min<int64_t>(chunk, ctx->nu_chunk_max);
  const size_t off_srec = 0;
  const size_t off_sder = off_srec + al(chunk * stride * rec_b);
  const size_t off_lists = off_sder + al(chunk * stride * der_b);
  const size_t off_cells = off_lists + al(chunk * ncls * stride * 4);
  const size_t off_order = off_cells + al(chunk * ncls * stride * 4);
  const size_t off_counts = off_order + al(chunk * ncls * stride * 4);
  const size_t off_grid = off_counts + al(chunk * ncls * 4);
  const size_t off_pdb = off_grid + al(chunk * O * ns.ng * 8);
  const size_t off_eldb = off_pdb + al(chunk * db_stride * kAdjSlotFloats * 4);
  const size_t total = off_eldb + chunk * db_stride * E * 4;
  int32_t rc = RSIM_OK;
  if (ctx->nu_adj_bytes < total) {
    HIP_TRY(ctx, hipDeviceSynchronize());  // earlier launches may still use the buffer
    dev_free(ctx, ctx->nu_adj_buf);
    ctx->nu_adj_buf = nullptr;
    ctx->nu_adj_bytes = 0;
    if ((rc = dev_alloc(ctx, &ctx->nu_adj_buf, total))) return rc;
    ctx->nu_adj_bytes = total;
  }
  char *b = static_cast<char *>(ctx->nu_adj_buf);
  NuBuffers nb{};
  nb.key = reinterpret_cast<int32_t *>(b + off_lists);
  nb.pos = reinterpret_cast<int32_t *>(b + off_cells);
  nb.order = reinterpret_cast<int32_t *>(b + off_order);
  nb.srec = b + off_srec;
  nb.grid = reinterpret_cast<float2 *>(b + off_grid);
  nb.rec_bytes = rec_b;
  nb.sder = b + off_sder;
  nb.n_runs = reinterpret_cast<int32_t *>(b + off_counts);
  if (db) {
    nb.part_db = reinterpret_cast<float *>(b + off_pdb);
    nb.el_db = reinterpret_cast<float *>(b + off_eldb);
    nb.db_stride = db_stride;
  }
  void *tw = twiddles(ctx, ns.ng, 0, &rc);
  if (rc) return rc;
  // every lit (chirp, facet) slot of adj_partial is written by the preparation (zero-area
  // facets) or a gather, and facet_grad reads lit slots only: no clearing
  ns.rec_stride = stride;
  for (int64_t n0 = 0; n0 < N; n0 += chunk) {
    ns.n0 = static_cast<int32_t>(n0);
    ns.n_chirps = static_cast<int32_t>(std::min<int64_t>(chunk, N - n0));
    HIP_TRY(ctx, launch_nufft_adjoint(d, rcn, elem, ns, nb, tw, grad_echo,
                                      ctx->adj_partial, s,
                                      kernel_events(ctx, ctx->timing_pending, kKernelStage0 + 1),
                                      dbsum, dbtsum));
  }
  EchoShape sh{};
  sh.O = static_cast<int32_t>(O);
  sh.o_tiles = 1;
  sh.m_tiles = 1;
  sh.accumulate = accumulate ? 1 : 0;
  if (!accumulate) HIP_TRY(ctx, launch_fill_zero(ctx->adj_gxw, N * F * 9, s));
  HIP_TRY(ctx, launch_adjoint_finish(d, rcn, sh, ctx->adj_partial, ctx->adj_gxw, s));
  return RSIM_OK;
}

int32_t rsim_backward(rsim_ctx *ctx, int32_t scene_id, const void *grad_echo,
                      const uint32_t *vis_mask, float *const *grad_verts, int32_t n_meshes,
                      double *grad_vel, void *hip_stream) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!grad_echo || !vis_mask || n_meshes < 0 || (n_meshes && !grad_verts))
    return fail(ctx, RSIM_EINVAL, "rsim_backward: need grad_echo, vis_mask and grad buffers");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  if ((rc = check_scene(ctx, scene_id))) return rc;
  if (ctx->dbounce) {
    // the connections' chain rule runs in the NUFFT adjoint, stop-and-hop
    if (ctx->ground || ctx->bwd_intra)
      return fail(ctx, RSIM_EINVAL, "rsim_backward: the facet-to-facet double bounce runs "
                  "stop-and-hop and without the ground plane");
    if (ctx->bwd_kernel == RSIM_KERNEL_VECTOR || ctx->bwd_kernel == RSIM_KERNEL_MATRIX)
      return fail(ctx, RSIM_EINVAL, "rsim_backward: the facet-to-facet double bounce is "
                  "differentiated by the NUFFT adjoint (backward kernel AUTO or NUFFT)");
    if ((ctx->tx.size() + ctx->rx.size()) / 3 > static_cast<size_t>(kNuDbMaxElems))
      return fail(ctx, RSIM_ERANGE, "rsim_backward: the double-bounce adjoint keeps one LDS "
                  "column per element: at most %d Tx + Rx elements", kNuDbMaxElems);
  }
  if (ctx->bwd_intra &&
      (ctx->bwd_kernel == RSIM_KERNEL_MATRIX || ctx->bwd_kernel == RSIM_KERNEL_NUFFT))
    return fail(ctx, RSIM_EINVAL, "rsim_backward: the adjoint with the delay within the chirp "
                "runs on the vector units (backward kernel AUTO or VECTOR)");
  RadarConst rcn = radar_const(ctx);
  rcn.intra = ctx->bwd_intra;
  if (cross_term_bound(ctx, rcn) > 3e-4)
    return fail(ctx, RSIM_ERANGE, "rsim_backward: array aperture too large for the FP32 sum");
  // the NUFFT adjoint when asked for, and with AUTO where eligible; else the matrix cores
  // when the array allows them (unless the vector units are asked for, or the delay within
  // the chirp, which only the vector-unit adjoint takes)
  NuShape nsb{};
  bool nufft = false;
  if (!ctx->bwd_intra &&
      (ctx->bwd_kernel == RSIM_KERNEL_NUFFT || ctx->bwd_kernel == RSIM_KERNEL_AUTO)) {
    const char *nwhy = nufft_adj_ineligible(ctx, rcn, scenes_rmax(ctx, {scene_id}), &nsb);
    if (nwhy && (ctx->bwd_kernel == RSIM_KERNEL_NUFFT || ctx->dbounce))
      return fail(ctx, RSIM_ERANGE, "rsim_backward: %s", nwhy);
    nufft = !nwhy;
  }
  if ((rc = need_device(ctx))) return rc;
  SceneRec &sc = ctx->scenes[scene_id];
  if ((rc = ensure_scene_device(ctx, sc))) return rc;
  const char *why = matrix_ineligible(ctx, rcn, RSIM_FP32_PHASE64);
  if (ctx->bwd_kernel == RSIM_KERNEL_MATRIX && why)
    return fail(ctx, RSIM_ERANGE, "rsim_backward: %s", why);
  const bool matrix = !nufft && !why && !ctx->bwd_intra && ctx->bwd_kernel != RSIM_KERNEL_VECTOR &&
                      adjoint_mfma_smem_bytes(rcn.P, rcn.Q, rcn.P + rcn.Q) <= ctx->max_lds;
  EchoShape sh{};
  if (nufft) {
    sh.O = rcn.P * rcn.Q;
    sh.o_tiles = 1;
    sh.m_tiles = 1;  // one adjoint slot per (chirp, lit facet)
  } else if (matrix) {
    sh.O = rcn.P * rcn.Q;
    sh.E = rcn.P + rcn.Q;
    sh.O_w = sh.O;
    sh.o_tiles = 1;
    sh.B_w = 1;
    sh.M_t = adjoint_mfma_tile_m();
    sh.m_tiles = (rcn.M + sh.M_t - 1) / sh.M_t;
    sh.n_compute = 256;
    sh.two_pi_slope = 2.0 * kPi * rcn.slope;
  } else {
    const bool intra = ctx->bwd_intra != 0;
    sh = echo_shape(ctx, rcn, adjoint_tile_m(), kMaxComputeThreads);
    while (sh.B_w > 1 && adjoint_smem_bytes(sh, intra) > ctx->max_lds)
      sh = echo_shape(ctx, rcn, adjoint_tile_m(), kMaxComputeThreads, sh.B_w - 1);
    if (adjoint_smem_bytes(sh, intra) > ctx->max_lds)
      return fail(ctx, RSIM_ERANGE, "adjoint tile needs %zu bytes of LDS",
                  adjoint_smem_bytes(sh, intra));
  }
  const int64_t F = sc.n_facets, N = rcn.N;
  size_t vmax = 1;
  for (const InstRec &r : sc.inst) vmax = std::max(vmax, ctx->meshes[r.mesh].verts.size() / 3);
  auto grow_f = [&](float *&p, size_t &cap, size_t need) -> int32_t {
    if (cap >= need) return RSIM_OK;
    dev_free(ctx, p);
    p = nullptr;
    cap = 0;
    int32_t r = dev_alloc(ctx, reinterpret_cast<void **>(&p), sizeof(float) * need);
    if (!r) cap = need;
    return r;
  };
  if ((rc = grow_f(ctx->adj_partial, ctx->adj_partial_n,
                   std::max<size_t>(1, adjoint_partial_floats(sh, N, F)))))
    return rc;
  if ((rc = grow_f(ctx->adj_gxw, ctx->adj_gxw_n, std::max<size_t>(1, N * F * 9)))) return rc;
  float *pv = nullptr, *gxv = nullptr;
  if (ctx->bwd_intra) {
    const size_t pv_b = sizeof(float) * 4 * std::max<size_t>(1, adjoint_partial_floats(sh, N, F) / kAdjSlotFloats);
    const size_t gxv_b = sizeof(float) * 3 * std::max<int64_t>(1, N * F);
    if ((rc = grow_bytes(ctx, &ctx->adj_pv, &ctx->adj_pv_bytes, pv_b))) return rc;
    if ((rc = grow_bytes(ctx, &ctx->adj_gxv, &ctx->adj_gxv_bytes, gxv_b))) return rc;
    pv = static_cast<float *>(ctx->adj_pv);
    gxv = static_cast<float *>(ctx->adj_gxv);
  }
  if (ctx->adj_gsum_n < static_cast<size_t>(2 * 9 * std::max<int64_t>(1, F))) {
    dev_free(ctx, ctx->adj_gsum);
    ctx->adj_gsum = nullptr;
    ctx->adj_gsum_n = 0;
    const size_t need = 2 * 9 * static_cast<size_t>(std::max<int64_t>(1, F));
    if ((rc = dev_alloc(ctx, reinterpret_cast<void **>(&ctx->adj_gsum), sizeof(double) * need)))
      return rc;
    ctx->adj_gsum_n = need;
  }
  if (ctx->adj_vpart_n < 3 * vmax) {
    dev_free(ctx, ctx->adj_vpart);
    ctx->adj_vpart = nullptr;
    ctx->adj_vpart_n = 0;
    if ((rc = dev_alloc(ctx, reinterpret_cast<void **>(&ctx->adj_vpart), sizeof(double) * 3 * vmax)))
      return rc;
    ctx->adj_vpart_n = 3 * vmax;
  }
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  DevScene d = dev_scene(sc, const_cast<uint32_t *>(vis_mask), nullptr);
  double *dbsum = nullptr, *dbtsum = nullptr;
  if (ctx->dbounce) {
    // the connection table follows the mask words in the caller's buffer; its lists are
    // rebuilt here, and the connections' chain rule adds into per-facet FP64 sums
    if (!sc.d_db) return fail(ctx, RSIM_ESTATE, "rsim_backward: no connection table");
    const int64_t plane = 2 * static_cast<int64_t>(rcn.N) * std::max<int64_t>(1, sc.n_facets);
    d.db_on = 1;
    d.db_b = reinterpret_cast<const int32_t *>(vis_mask + static_cast<int64_t>(rcn.N) * d.mask_words);
    d.db_idx = sc.d_db + plane;
    d.db_cnt = sc.d_db + 2 * plane;
    d.db_gamma_re = ctx->db_gamma_re;
    d.db_gamma_im = ctx->db_gamma_im;
    d.db_n = rcn.N;
    const size_t need = sizeof(double) * 2 * 9 * static_cast<size_t>(std::max<int64_t>(1, F));
    if ((rc = grow_bytes(ctx, &ctx->adj_dbsum, &ctx->adj_dbsum_bytes, need))) return rc;
    dbsum = static_cast<double *>(ctx->adj_dbsum);
    dbtsum = dbsum + 9 * std::max<int64_t>(1, F);
    HIP_TRY(ctx, launch_fill_zero(reinterpret_cast<float *>(dbsum), 2 * 2 * 9 * std::max<int64_t>(1, F), s));
  }
  const bool timing = ctx->timing_pending;
  // With the ground plane the forward added four path types (their own masks, mirrored
  // elements and gamma per bounce); the adjoint runs each with the echo gradient times
  // conj(gamma^bounces) and adds their world-vertex gradients in path-type order.
  const int types = ctx->ground ? 4 : 1;
  const int E = rcn.P + rcn.Q;
  if (ctx->ground) {
    if ((rc = ensure_elem_images(ctx))) return rc;
    const size_t cube = static_cast<size_t>(rcn.P) * rcn.Q * rcn.N * rcn.M * 8;
    if (ctx->adj_gscaled_bytes < cube) {
      dev_free(ctx, ctx->adj_gscaled);
      ctx->adj_gscaled = nullptr;
      ctx->adj_gscaled_bytes = 0;
      if ((rc = dev_alloc(ctx, &ctx->adj_gscaled, cube))) return rc;
      ctx->adj_gscaled_bytes = cube;
    }
  }
  stage_begin(ctx, timing, 5, s);
  for (int k = 0; k < types; ++k) {
    DevScene dk = d;
    dk.mask = d.mask + static_cast<int64_t>(k) * rcn.N * d.mask_words;
    HIP_TRY(ctx, launch_compact(dk, 0, rcn.N, s));
    if (dk.db_on) {
      const int64_t plane = 2 * static_cast<int64_t>(rcn.N) * std::max<int64_t>(1, dk.n_facets);
      int32_t *work = const_cast<int32_t *>(dk.db_idx) - plane;
      HIP_TRY(ctx, launch_dbounce(dk, rcn, 0.0, scenes_rmax(ctx, {scene_id}),
                                  const_cast<int32_t *>(dk.db_b), work + plane, work + 2 * plane,
                                  s));
    }
    RadarConst rk = rcn;
    if (k & 1) rk.tx_c[2] = 2.0 * ctx->z_ground - rcn.tx_c[2];
    if (k >> 1) rk.rx_c[2] = 2.0 * ctx->z_ground - rcn.rx_c[2];
    const double *elem = k ? ctx->d_elem_img + static_cast<size_t>(k - 1) * 3 * E : ctx->d_elem;
    const void *gk = grad_echo;
    if (k) {
      double gr = 1.0, gi = 0.0;
      for (int b = 0; b < ((k & 1) + (k >> 1)); ++b) {
        const double t = gr * ctx->gamma_re - gi * ctx->gamma_im;
        gi = gr * ctx->gamma_im + gi * ctx->gamma_re;
        gr = t;
      }
      const int64_t n = static_cast<int64_t>(rcn.P) * rcn.Q * rcn.N * rcn.M;
      HIP_TRY(ctx, launch_scale_conj(grad_echo, ctx->adj_gscaled, n, gr, gi, s));
      gk = ctx->adj_gscaled;
    }
    EchoShape sk = sh;
    sk.accumulate = k ? 1 : 0;
    if (nufft) {
      if ((rc = enqueue_nufft_adjoint(ctx, dk, rk, elem, nsb, gk, k > 0, s, dbsum, dbtsum)))
        return rc;
    } else if (matrix)
      HIP_TRY(ctx, launch_adjoint_mfma(dk, rk, elem, sk, gk, ctx->adj_partial, ctx->adj_gxw, s));
    else
      HIP_TRY(ctx, launch_adjoint(dk, rk, elem, sk, gk, ctx->adj_partial, ctx->adj_gxw, s, pv, gxv));
  }
  stage_end(ctx, timing, 5, s);
  stage_begin(ctx, timing, 7, s);
  double *gsum = ctx->adj_gsum, *gtsum = ctx->adj_gsum + 9 * F;
  HIP_TRY(ctx, launch_facet_chirp_sum(ctx->adj_gxw, gxv, F, rcn.N, rcn.tc, gsum, gtsum, s,
                                      dbsum));
  for (size_t i = 0; i < sc.inst.size(); ++i) {
    const InstRec &r = sc.inst[i];
    const MeshRec &m = ctx->meshes[r.mesh];
    float *gv = (r.mesh < n_meshes) ? grad_verts[r.mesh] : nullptr;
    const double *rot_dev = reinterpret_cast<const double *>(
        reinterpret_cast<const char *>(sc.d_inst) + i * sizeof(DevInstance) + offsetof(DevInstance, rot));
    // without grad_vel the velocity sum lands in vpart[0..2], after vpart has been read
    double *vel_out = grad_vel ? grad_vel + 3 * i : ctx->adj_vpart;
    const int64_t base = [&] {
      int64_t b = 0;
      for (size_t k = 0; k < i; ++k) b += static_cast<int64_t>(ctx->meshes[sc.inst[k].mesh].tris.size() / 3);
      return b;
    }();
    HIP_TRY(ctx, launch_vertex_gather(gsum, gtsum, rot_dev, base, m.d_csr_off, m.d_csr_ent,
                                      static_cast<int32_t>(m.verts.size() / 3), gv,
                                      ctx->adj_vpart, vel_out, s));
  }
  stage_end(ctx, timing, 7, s);
  return RSIM_OK;
}

int32_t rsim_rdm_backward(rsim_ctx *ctx, const float *grad_rdm, const void *y, int32_t n_cubes,
                          void *grad_echo, void *hip_stream) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!grad_rdm || !y || !grad_echo || n_cubes < 1)
    return fail(ctx, RSIM_EINVAL, "rsim_rdm_backward: need grad_rdm, y, grad_echo, n_cubes >= 1");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  const int M = ctx->wf.n_samples, N = ctx->wf.n_chirps;
  if (!fft_size_ok(M) || !fft_size_ok(N))
    return fail(ctx, RSIM_ERANGE, "rsim_rdm_backward: M and N must be 2^a 3^b in 2..4096");
  if ((rc = need_device(ctx))) return rc;
  const int64_t O = static_cast<int64_t>(ctx->tx.size() / 3) * (ctx->rx.size() / 3);
  const int64_t planes = O * n_cubes;
  void *Z = nullptr;
  if ((rc = scratch(ctx, 8 * planes * N * M, &Z))) return rc;
  void *twM = twiddles(ctx, M, 0, &rc);
  if (rc) return rc;
  void *twN = twiddles(ctx, N, 0, &rc);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool timing = ctx->timing_pending;
  stage_begin(ctx, timing, 6, s);
  HIP_TRY(ctx, launch_doppler_fft(0, y, Z, nullptr, planes, N, M, 2, twN, s, grad_rdm));
  HIP_TRY(ctx, launch_range_fft(0, Z, grad_echo, planes * N, M, 0, twM, s));
  stage_end(ctx, timing, 6, s);
  return RSIM_OK;
}

int32_t rsim_form_rdm(rsim_ctx *ctx, const void *echo, int32_t n_cubes, void *rdm, void *y_opt,
                      void *hip_stream, const rsim_opts *opts) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  rsim_opts o{};
  if (opts) o = *opts;
  if (!echo || n_cubes < 1 || (!rdm && !y_opt))
    return fail(ctx, RSIM_EINVAL, "rsim_form_rdm: need echo, n_cubes >= 1 and an output");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  const int M = ctx->wf.n_samples, N = ctx->wf.n_chirps;
  if (!fft_size_ok(M) || !fft_size_ok(N))
    return fail(ctx, RSIM_ERANGE, "rsim_form_rdm: M=%d and N=%d must be 2^a 3^b in 2..4096", M, N);
  if ((rc = need_device(ctx))) return rc;
  const int precision = o.precision ? 1 : 0;
  const size_t csize = precision ? 16 : 8;
  const int64_t O = static_cast<int64_t>(ctx->tx.size() / 3) * (ctx->rx.size() / 3);
  const int64_t planes = O * n_cubes;
  const size_t need_lds = 2 * csize * (std::max(M, N) + 32);
  if (need_lds > ctx->max_lds) return fail(ctx, RSIM_ERANGE, "FFT length exceeds LDS");
  void *X = nullptr;
  if ((rc = scratch(ctx, csize * planes * N * M, &X))) return rc;
  void *twM = twiddles(ctx, M, precision, &rc);
  if (rc) return rc;
  void *twN = twiddles(ctx, N, precision, &rc);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool timing = o.timing != 0;
  if (timing && !ctx->timing_pending) timing_reset(ctx, true);
  stage_begin(ctx, timing, 3, s);
  HIP_TRY(ctx, launch_range_fft(precision, echo, X, planes * N, M, 1, twM, s));
  stage_end(ctx, timing, 3, s);
  stage_begin(ctx, timing, 4, s);
  HIP_TRY(ctx, launch_doppler_fft(precision, X, y_opt, rdm, planes, N, M, 0, twN, s));
  stage_end(ctx, timing, 4, s);
  return RSIM_OK;
}

int32_t rsim_form_rdm_noalloc(rsim_ctx *ctx, const void *echo, int32_t n_cubes, void *rdm,
                              void *y_opt, void *hip_stream, const rsim_opts *opts) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  rsim_opts o{};
  if (opts) o = *opts;
  if (!echo || n_cubes < 1 || (!rdm && !y_opt))
    return fail(ctx, RSIM_EINVAL, "rsim_form_rdm_noalloc: need echo, n_cubes >= 1 and an output");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  const int M = ctx->wf.n_samples, N = ctx->wf.n_chirps;
  if (!fft_size_ok(M) || !fft_size_ok(N))
    return fail(ctx, RSIM_ERANGE, "rsim_form_rdm_noalloc: M=%d and N=%d must be 2^a 3^b in 2..4096",
                M, N);
  if ((rc = need_device(ctx))) return rc;
  if (!ctx->static_scratch)
    return fail(ctx, RSIM_EDEVICE, "rsim_form_rdm_noalloc: no static work array on this device");
  const int precision = o.precision ? 1 : 0;
  const size_t csize = precision ? 16 : 8;
  const size_t need_lds = 2 * csize * (std::max(M, N) + 32);
  if (need_lds > ctx->max_lds) return fail(ctx, RSIM_ERANGE, "FFT length exceeds LDS");
  // layout of the static array: twiddles of M, twiddles of N, then X of g planes
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t tw_bytes = al(csize * M) + al(csize * N);
  const size_t plane = csize * static_cast<size_t>(N) * M;
  if (tw_bytes + plane > kStaticScratchBytes)
    return fail(ctx, RSIM_ERANGE,
                "rsim_form_rdm_noalloc: one %d x %d plane (%zu bytes) and its twiddles exceed the "
                "static work array (%zu bytes)", N, M, plane, kStaticScratchBytes);
  const int64_t O = static_cast<int64_t>(ctx->tx.size() / 3) * (ctx->rx.size() / 3);
  const int64_t planes = O * n_cubes;
  const int64_t group = static_cast<int64_t>((kStaticScratchBytes - tw_bytes) / plane);
  char *base = static_cast<char *>(ctx->static_scratch);
  void *twM = base, *twN = base + al(csize * M);
  void *X = base + tw_bytes;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const bool timing = o.timing != 0;
  if (timing && !ctx->timing_pending) timing_reset(ctx, true);
  HIP_TRY(ctx, launch_twiddle_fill(twM, M, precision, s));
  HIP_TRY(ctx, launch_twiddle_fill(twN, N, precision, s));
  stage_begin(ctx, timing, 3, s);
  for (int64_t p0 = 0; p0 < planes; p0 += group) {
    const int64_t g = std::min(group, planes - p0);
    const size_t off = static_cast<size_t>(p0) * N * M;
    HIP_TRY(ctx, launch_range_fft(precision, static_cast<const char *>(echo) + off * csize, X,
                                  g * N, M, 1, twM, s));
    HIP_TRY(ctx, launch_doppler_fft(precision, X,
                                    y_opt ? static_cast<char *>(y_opt) + off * csize : nullptr,
                                    rdm ? static_cast<char *>(rdm) + off * (csize / 2) : nullptr,
                                    g, N, M, 0, twN, s));
  }
  stage_end(ctx, timing, 3, s);
  return RSIM_OK;
}

int32_t rsim_rdm_adjoint(rsim_ctx *ctx, const void *grad_y, int32_t n_cubes, void *grad_echo,
                         void *hip_stream) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!grad_y || !grad_echo || n_cubes < 1)
    return fail(ctx, RSIM_EINVAL, "rsim_rdm_adjoint: need grad_y, grad_echo and n_cubes >= 1");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  const int M = ctx->wf.n_samples, N = ctx->wf.n_chirps;
  if (!fft_size_ok(M) || !fft_size_ok(N))
    return fail(ctx, RSIM_ERANGE, "rsim_rdm_adjoint: M and N must be 2^a 3^b in 2..4096");
  if ((rc = need_device(ctx))) return rc;
  const int64_t O = static_cast<int64_t>(ctx->tx.size() / 3) * (ctx->rx.size() / 3);
  const int64_t planes = O * n_cubes;
  void *Z = nullptr;
  if ((rc = scratch(ctx, 8 * planes * N * M, &Z))) return rc;
  void *twM = twiddles(ctx, M, 0, &rc);
  if (rc) return rc;
  void *twN = twiddles(ctx, N, 0, &rc);
  if (rc) return rc;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  // G_H = FFT_m(FFT_n(conj(unshift_n(G_Y)))) for X = FFT_m(conj H), Y = shift FFT_n(X)
  HIP_TRY(ctx, launch_doppler_fft(0, grad_y, Z, nullptr, planes, N, M, 1, twN, s));
  HIP_TRY(ctx, launch_range_fft(0, Z, grad_echo, planes * N, M, 0, twM, s));
  return RSIM_OK;
}

int32_t rsim_last_census(rsim_ctx *ctx, int64_t counts[4]) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!counts) return fail(ctx, RSIM_EINVAL, "rsim_last_census: counts is NULL");
  if (ctx->host_only) return fail(ctx, RSIM_EDEVICE, "host-only context");
  if (!ctx->census_ready)
    return fail(ctx, RSIM_ESTATE, "rsim_last_census: no NUFFT facet sum ran with census set");
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  HIP_TRY(ctx, hipDeviceSynchronize());
  std::vector<unsigned long long> h(4 * kNuCensusSlots);
  HIP_TRY(ctx, hipMemcpy(h.data(), ctx->d_census, sizeof(unsigned long long) * h.size(),
                         hipMemcpyDeviceToHost));
  for (int k = 0; k < 4; ++k) {
    counts[k] = 0;
    for (int r = 0; r < kNuCensusSlots; ++r) counts[k] += static_cast<int64_t>(h[4 * r + k]);
  }
  return RSIM_OK;
}

int32_t rsim_last_timings(rsim_ctx *ctx, float *ms, int32_t n_stages) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!ms || n_stages < 1 || n_stages > kStages)
    return fail(ctx, RSIM_EINVAL, "rsim_last_timings: n_stages must be 1..%d", kStages);
  if (ctx->host_only) return fail(ctx, RSIM_EDEVICE, "host-only context");
  for (int k = 0; k < n_stages; ++k) {
    ms[k] = 0.0f;
    if (!ctx->stage_ran[k]) continue;
    if (k >= kKernelStage0) {
      const std::vector<hipEvent_t> &pool = ctx->kern_ev[k - kKernelStage0];
      for (int i = 0; i < ctx->kern_used[k - kKernelStage0]; ++i) {
        HIP_TRY(ctx, hipEventSynchronize(pool[2 * i + 1]));
        float v = 0.0f;
        HIP_TRY(ctx, hipEventElapsedTime(&v, pool[2 * i], pool[2 * i + 1]));
        ms[k] += v;
      }
      continue;
    }
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev1[k]));
    float v = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&v, ctx->ev0[k], ctx->ev1[k]));
    ms[k] = v;
  }
  ctx->timing_pending = false;
  return RSIM_OK;
}

int32_t rsim_detect(rsim_ctx *ctx, const float *rdm, const void *y, int32_t n_cubes,
                    const rsim_cfar_opts *opts, uint8_t *det_mask, float *noise_map,
                    rsim_point *points, int32_t *n_points, void *hip_stream) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!rdm || !y || !opts || !points || !n_points || n_cubes < 1)
    return fail(ctx, RSIM_EINVAL, "rsim_detect: need rdm, y, opts, points, n_points, n_cubes >= 1");
  const rsim_cfar_opts o = *opts;
  if (o.guard_doppler < 0 || o.guard_range < 0 || o.train_doppler < 0 || o.train_range < 0 ||
      o.train_doppler + o.train_range < 1 || !(o.scale > 0.0f) || !std::isfinite(o.scale) ||
      o.max_points < 1 || o.na_x < 0 || o.na_z < 0)
    return fail(ctx, RSIM_EINVAL, "rsim_detect: bad CFAR settings");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  const int M = ctx->wf.n_samples, N = ctx->wf.n_chirps;
  const int hd = o.guard_doppler + o.train_doppler, hr = o.guard_range + o.train_range;
  if (2 * hd + 1 > N || 2 * hr + 1 > M)
    return fail(ctx, RSIM_ERANGE, "rsim_detect: CFAR window %dx%d exceeds the %dx%d map",
                2 * hd + 1, 2 * hr + 1, N, M);
  // virtual elements tx_p + rx_q on the half-wavelength grid of the x-z plane
  const double df = ctx->wf.slope_hz_per_s / ctx->wf.fs_hz;
  const double lam_c = kC0 / (ctx->wf.f0_hz + 0.5 * M * df);
  const double d = 0.5 * lam_c;
  const int P = static_cast<int>(ctx->tx.size() / 3), Q = static_cast<int>(ctx->rx.size() / 3);
  const int O = P * Q;
  std::vector<double> vx(O), vy(O), vz(O);
  for (int p = 0; p < P; ++p)
    for (int q = 0; q < Q; ++q) {
      vx[p * Q + q] = ctx->tx[3 * p + 0] + ctx->rx[3 * q + 0];
      vy[p * Q + q] = ctx->tx[3 * p + 1] + ctx->rx[3 * q + 1];
      vz[p * Q + q] = ctx->tx[3 * p + 2] + ctx->rx[3 * q + 2];
    }
  const double x0 = *std::min_element(vx.begin(), vx.end());
  const double z0 = *std::min_element(vz.begin(), vz.end());
  const double y_lo = *std::min_element(vy.begin(), vy.end());
  const double y_hi = *std::max_element(vy.begin(), vy.end());
  if (y_hi - y_lo > 1e-9)
    return fail(ctx, RSIM_ERANGE, "rsim_detect: virtual elements are not in one x-z plane");
  std::vector<int> ix(O), iz(O);
  int nx = 0, nz = 0;
  for (int k = 0; k < O; ++k) {
    const double gx = (vx[k] - x0) / d, gz = (vz[k] - z0) / d;
    ix[k] = static_cast<int>(std::lround(gx));
    iz[k] = static_cast<int>(std::lround(gz));
    if (std::fabs(gx - ix[k]) > 1e-6 || std::fabs(gz - iz[k]) > 1e-6)
      return fail(ctx, RSIM_ERANGE, "rsim_detect: virtual elements are not on a half-wavelength grid");
    nx = std::max(nx, ix[k] + 1);
    nz = std::max(nz, iz[k] + 1);
  }
  auto smallest_fft = [](int n) {
    int best = 1 << 30;
    for (long p2 = 1; p2 < 4L * n + 4; p2 *= 2)
      for (long p = p2; p < 4L * n + 4; p *= 3)
        if (p >= n && p < best) best = static_cast<int>(p);
    return best;
  };
  const int na_x = o.na_x ? o.na_x : smallest_fft(2 * nx);
  const int na_z = o.na_z ? o.na_z : (nz == 1 ? 1 : smallest_fft(2 * nz));
  if (!fft_size_ok(na_x) || na_x < nx || (na_z != 1 && !fft_size_ok(na_z)) || na_z < nz)
    return fail(ctx, RSIM_ERANGE, "rsim_detect: angle lengths %dx%d must be 2^a 3^b covering the "
                "%dx%d virtual grid", na_x, na_z, nx, nz);
  if ((rc = need_device(ctx))) return rc;
  if (cfar_smem_bytes(o.guard_doppler, o.guard_range, o.train_doppler, o.train_range) > ctx->max_lds)
    return fail(ctx, RSIM_ERANGE, "rsim_detect: CFAR window too large for LDS");
  if (angle_smem_bytes(na_x, na_z) + 4096 > ctx->max_lds)
    return fail(ctx, RSIM_ERANGE, "rsim_detect: angle grid %dx%d too large for LDS", na_x, na_z);
  // grid nodes in ascending position, each with its channels in channel order
  std::vector<int> order(O);
  for (int k = 0; k < O; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return iz[a] * na_x + ix[a] < iz[b] * na_x + ix[b];
  });
  std::vector<int32_t> pos, off, ch;
  for (int k = 0; k < O; ++k) {
    const int g = iz[order[k]] * na_x + ix[order[k]];
    if (pos.empty() || pos.back() != g) {
      pos.push_back(g);
      off.push_back(k);
    }
    ch.push_back(order[k]);
  }
  off.push_back(O);
  const int n_nodes = static_cast<int>(pos.size());
  std::vector<int32_t> tables;
  tables.insert(tables.end(), pos.begin(), pos.end());
  tables.insert(tables.end(), off.begin(), off.end());
  tables.insert(tables.end(), ch.begin(), ch.end());
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  if (tables != ctx->det_nodes_host) {
    HIP_TRY(ctx, hipStreamSynchronize(s));  // an earlier call may still read the tables
    void *pn = ctx->det_nodes;
    if ((rc = grow_bytes(ctx, &pn, &ctx->det_nodes_n, sizeof(int32_t) * tables.size()))) return rc;
    ctx->det_nodes = static_cast<int32_t *>(pn);
    HIP_TRY(ctx, hipMemcpy(ctx->det_nodes, tables.data(), sizeof(int32_t) * tables.size(),
                           hipMemcpyHostToDevice));
    ctx->det_nodes_host = tables;
  }
  const int64_t cells = static_cast<int64_t>(n_cubes) * N * M;
  if ((rc = grow_bytes(ctx, &ctx->det_P, &ctx->det_P_n, sizeof(float) * cells))) return rc;
  if (!det_mask) {
    if ((rc = grow_bytes(ctx, &ctx->det_mask, &ctx->det_mask_n, cells))) return rc;
    det_mask = static_cast<uint8_t *>(ctx->det_mask);
  }
  if (!noise_map) {
    if ((rc = grow_bytes(ctx, &ctx->det_noise, &ctx->det_noise_n, sizeof(float) * cells))) return rc;
    noise_map = static_cast<float *>(ctx->det_noise);
  }
  if ((rc = grow_bytes(ctx, &ctx->det_list, &ctx->det_list_n,
                       sizeof(int32_t) * static_cast<size_t>(n_cubes) * o.max_points)))
    return rc;
  void *tw_x = twiddles(ctx, na_x, 0, &rc);
  if (rc) return rc;
  void *tw_z = na_z > 1 ? twiddles(ctx, na_z, 0, &rc) : tw_x;
  if (rc) return rc;
  double c_ref[3];
  for (int k = 0; k < 3; ++k) {
    double a = 0.0, b = 0.0;
    for (int p = 0; p < P; ++p) a += ctx->tx[3 * p + k];
    for (int q = 0; q < Q; ++q) b += ctx->rx[3 * q + k];
    c_ref[k] = 0.5 * (a / P + b / Q);
  }
  const double range_res = kC0 / (2.0 * M * df);
  const double vel_res = lam_c / (2.0 * N * ctx->wf.chirp_period_s);
  const int32_t *nodes = ctx->det_nodes;
  HIP_TRY(ctx, launch_detect(rdm, y, n_cubes, O, N, M, o.guard_doppler, o.guard_range,
                             o.train_doppler, o.train_range, o.scale, na_x, na_z, o.max_points,
                             range_res, vel_res, c_ref, nodes, nodes + n_nodes,
                             nodes + 2 * n_nodes + 1, n_nodes, tw_x, tw_z,
                             static_cast<float *>(ctx->det_P), det_mask, noise_map,
                             static_cast<int32_t *>(ctx->det_list), n_points, points, s));
  return RSIM_OK;
}

int32_t rsim_add_noise(rsim_ctx *ctx, void *echo, int32_t n_cubes, double snr_db, uint64_t seed,
                       void *hip_stream, const rsim_opts *opts) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!echo || n_cubes < 1 || !std::isfinite(snr_db))
    return fail(ctx, RSIM_EINVAL, "rsim_add_noise: need echo, n_cubes >= 1 and a finite SNR");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  if ((rc = need_device(ctx))) return rc;
  const int precision = (opts && opts->precision) ? 1 : 0;
  const int64_t n = static_cast<int64_t>(ctx->tx.size() / 3) * (ctx->rx.size() / 3) *
                    ctx->wf.n_chirps * ctx->wf.n_samples;
  void *part = ctx->noise_part;
  const size_t need = sizeof(double) * static_cast<size_t>(n_cubes) * (noise_partials_per_cube() + 1);
  if ((rc = grow_bytes(ctx, &part, &ctx->noise_part_n, need))) return rc;
  ctx->noise_part = static_cast<double *>(part);
  double *scale = ctx->noise_part + static_cast<size_t>(n_cubes) * noise_partials_per_cube();
  HIP_TRY(ctx, launch_add_noise(precision, echo, n, n_cubes, snr_db, seed, ctx->noise_part, scale,
                                static_cast<hipStream_t>(hip_stream)));
  return RSIM_OK;
}

int32_t rsim_autotune(rsim_ctx *ctx, const int32_t *scene_ids, int32_t n_scenes,
                      const char *cache_json_path) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  if (!scene_ids || n_scenes < 1) return fail(ctx, RSIM_EINVAL, "rsim_autotune: no scenes");
  if (ctx->dbounce)
    return fail(ctx, RSIM_ESTATE, "rsim_autotune: with the double bounce the facet sum is the "
                "NUFFT; disable it (rsim_set_double_bounce) to time the kernels");
  int32_t rc = check_radar(ctx);
  if (rc) return rc;
  if ((rc = need_device(ctx))) return rc;
  const RadarConst rcn = radar_const(ctx);
  const int O = rcn.P * rcn.Q;
  const int64_t cube = static_cast<int64_t>(O) * rcn.N * rcn.M;
  void *echo = nullptr;
  if ((rc = dev_alloc(ctx, &echo, 8 * cube * n_scenes))) return rc;
  // the NUFFT where the scenes allow it (mb = -1), the matrix cores where the array allows
  // them (mb = 0), then the vector-unit tiles
  struct Cand { int mb, ft; };
  std::vector<Cand> cands;
  {
    rsim_opts probe{};
    NuShape ns{};
    const std::vector<int32_t> ids(scene_ids, scene_ids + n_scenes);
    for (int32_t id : ids)
      if ((rc = check_scene(ctx, id))) {
        dev_free(ctx, echo);
        return rc;
      }
    if (!nufft_ineligible(ctx, rcn, probe, scenes_rmax(ctx, ids), scenes_vmax(ctx, ids), &ns))
      cands.push_back({-1, 0});
  }
  if (!matrix_ineligible(ctx, rcn, RSIM_FP32_PHASE64)) cands.push_back({0, 0});
  for (const Cand c : {Cand{64, 16}, Cand{32, 16}, Cand{64, 8}, Cand{32, 8}, Cand{16, 16}})
    cands.push_back(c);
  // each candidate runs once (cold); one within 1.5x of the best so far runs once more
  // and keeps the faster of its two facet-sum times
  float best = 1e30f;
  TunedShape best_s{32, 16, RSIM_KERNEL_VECTOR};
  float best_vec = 1e30f;
  hipStream_t s = ctx->capture_stream;
  for (const Cand &c : cands) {
    rsim_opts o{};
    o.timing = 1;
    if (c.mb > 0) {
      o.tile_m = c.mb;
      o.tile_f = c.ft;
      o.kernel = RSIM_KERNEL_VECTOR;
      const EchoShape sh = forward_shape(ctx, rcn, 0, c.mb, c.ft);
      if (echo_smem_bytes(0, c.mb, c.ft, sh) > ctx->max_lds) continue;
    } else if (c.mb == 0) {
      o.kernel = RSIM_KERNEL_MATRIX;
      if (mfma_smem_bytes(matrix_shape(rcn)) > ctx->max_lds) continue;
    } else {
      o.kernel = RSIM_KERNEL_NUFFT;
    }
    float t = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      if ((rc = rsim_synthesize(ctx, scene_ids, n_scenes, echo, nullptr, s, &o))) {
        dev_free(ctx, echo);
        return rc;
      }
      float ms[kStages];
      if ((rc = rsim_last_timings(ctx, ms, kStages))) {
        dev_free(ctx, echo);
        return rc;
      }
      t = std::min(t, ms[2]);
      if (t > 1.5f * std::min(best, c.mb > 0 ? best_vec : best)) break;
    }
    if (c.mb > 0 && t < best_vec) {
      best_vec = t;
      best_s.mb = c.mb;  // the best vector tiles, kept for opts.kernel = VECTOR
      best_s.ft = c.ft;
    }
    if (t < best) {
      best = t;
      best_s.kernel = c.mb > 0 ? RSIM_KERNEL_VECTOR
                      : c.mb == 0 ? RSIM_KERNEL_MATRIX : RSIM_KERNEL_NUFFT;
    }
  }
  dev_free(ctx, echo);
  ctx->tuned[std::make_tuple(rcn.M, O, 0)] = best_s;
  ctx->version++;
  if (cache_json_path) {
    std::ofstream f(cache_json_path, std::ios::app);
    if (!f) return fail(ctx, RSIM_EINVAL, "cannot open %s", cache_json_path);
    f << "{\"arch\": \"gfx950\", \"M\": " << rcn.M << ", \"O\": " << O
      << ", \"precision\": \"fp32\", \"kernel\": \""
      << (best_s.kernel == RSIM_KERNEL_MATRIX  ? "matrix"
          : best_s.kernel == RSIM_KERNEL_NUFFT ? "nufft"
                                               : "vector")
      << "\", \"tile_m\": " << best_s.mb << ", \"tile_f\": " << best_s.ft
      << ", \"facet_sum_ms\": " << best << "}\n";
  }
  return RSIM_OK;
}

int32_t rsim_sync(rsim_ctx *ctx, void *hip_stream) {
  if (!ctx) return fail(nullptr, RSIM_EINVAL, "ctx is NULL");
  int32_t rc = need_device(ctx);
  if (rc) return rc;
  HIP_TRY(ctx, hipStreamSynchronize(static_cast<hipStream_t>(hip_stream)));
  return RSIM_OK;
}

}  // extern "C"
