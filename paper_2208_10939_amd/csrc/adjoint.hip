// Adjoint of the coherent facet sum: dL/d(vertex positions) and dL/d(instance
// velocity) for a real loss L, given g = dL/dRe(H) + j dL/dIm(H) (Sections 2.2, 3.2;
// eqs. (7), (9)-(13) as in the forward kernel). The lit-facet mask is held fixed and
// every chirp is recomputed rather than stored.
//
// For one facet f at chirp n, the forward term is T = G(m) z_o(m) with
//   G(m)   = j o A Phi(k_m b) / (2 pi),   z_o(m) = exp(-j 2 pi psi) / (R_p R_q),
//   psi    = f_m tau - slope tau^2 / 2,   tau = (R_p + R_q) / c,
// so with w = conj(g) z and y = G w (summed over channels o and samples m):
//   dL/do     = sum Re(y) / o,            dL/dA = sum Re(y) / A,
//   dL/db_i   = sum Re(D_i w),  D_i = j o A k_m dPhi/da_i / (2 pi),
//   dL/dR_p   = sum_q,m [ (2 pi / c)(f_m - slope tau) Im y - Re y / R_p ]  (same for R_q).
// The adjoint facet-sum kernel forms these sums (20 VALU ops per evaluation) and
// reduces them over its channels with wave shuffles in a fixed order; a second
// kernel applies the FP64 chain rule from (o, A, b, centroid) to the three world
// vertices; a third gathers per-vertex gradients through a vertex -> (triangle,
// corner) index, rotates them to the body frame and sums t_n-weighted gradients into
// the velocity gradient. No floating-point atomics: results are deterministic.
//
// With the delay taken at the sample times (eq. (12) at t_n + m / fs; amplitude, facet
// integral and lit set at t_n), the forward's element phasors run along the chord of
// each block of MB samples and the phase-centre path's curvature rides in G; the adjoint
// stages the same. The centroid then moves with the facet's velocity within the chirp,
// so the velocity gradient gains sum_m (m / fs) dL/dc|_phase(m): per channel
//   -(2 pi / c) / fs * sum_m m (f_0 - slope tau + m df) Im y_m * (e_p + e_q)
// (e the unit vectors centroid -> element); its phase derivative takes the delay and the
// unit vectors at t_n (they move by v m / fs, a relative change below 1e-6 here).
#include <algorithm>

#include "adjoint_common.h"

namespace rsim {

namespace {


// LDS layout of the adjoint facet sum: shared tables, per-staging-wave geometry, the
// per-wave channel sums of two tiles, and two tile buffers.
template <int MB, int FT>
struct AdjLayout {
  size_t elem, geo, glin, red, buf[2], GD, U, rat, off, er, tau, total;
  int waves;      // accumulating waves
  int rat_b;      // element ratios per element: one, or one per block (delay within the chirp)
  int red_vals;   // per-wave sums per facet: kAdjVals, or kAdjRedIntra with the chirp delay

  __host__ __device__ AdjLayout(const EchoShape &sh, bool intra) {
    auto up = [](size_t b) { return (b + 15) & ~size_t(15); };
    waves = sh.n_compute / 64;
    rat_b = intra ? sh.B_w : 1;
    red_vals = intra ? kAdjRedIntra : kAdjVals;
    size_t b = 0;
    elem = b;
    b = up(b + sizeof(double) * 3 * sh.E);
    geo = b;
    b = up(b + sizeof(Geo) * FT);
    glin = b;
    b = up(b + sizeof(GLin) * FT);
    red = b;  // [2][FT][waves][red_vals]
    b = up(b + sizeof(float) * 2 * FT * waves * red_vals);
    size_t t = 0;
    GD = t;  // [FT][M_t][2] float4: (G, D0), (D1, D2)
    t += sizeof(float4) * FT * 2 * sh.M_t;
    U = t;  // [FT][E][B_w]
    t += sizeof(float2) * FT * sh.E * sh.B_w;
    rat = t;  // [FT][E][rat_b]
    t += sizeof(float2) * FT * sh.E * rat_b;
    er = t;  // [FT][E]: unit vector centroid -> element (xyz), 1 / R (w)
    t += sizeof(float4) * FT * sh.E;
    off = t;  // [FT][E]
    t += sizeof(float) * FT * sh.E;
    tau = t;  // [FT][E]
    t = up(t + sizeof(float) * FT * sh.E);
    buf[0] = b;
    buf[1] = b + t;
    total = b + 2 * t;
  }
};

struct AdjTile {
  float4 *GD;
  float2 *U, *rat;
  float4 *er;
  float *off, *tau;
};

template <int MB, int FT>
struct AdjSmem {
  double *elem;
  Geo *geo;
  GLin *glin;
  float *red;
  unsigned char *buf0;
  size_t stride, oGD, oU, orat, oer, ooff, otau;
  int waves, rat_b, red_vals;

  __device__ void carve(unsigned char *base, const EchoShape &sh, bool intra) {
    const AdjLayout<MB, FT> L(sh, intra);
    elem = reinterpret_cast<double *>(base + L.elem);
    geo = reinterpret_cast<Geo *>(base + L.geo);
    glin = reinterpret_cast<GLin *>(base + L.glin);
    red = reinterpret_cast<float *>(base + L.red);
    buf0 = base + L.buf[0];
    stride = L.buf[1] - L.buf[0];
    oGD = L.GD;
    oU = L.U;
    orat = L.rat;
    oer = L.er;
    ooff = L.off;
    otau = L.tau;
    waves = L.waves;
    rat_b = L.rat_b;
    red_vals = L.red_vals;
  }
  __device__ AdjTile tile(int k) const {
    unsigned char *t = buf0 + static_cast<size_t>(k) * stride;
    return {reinterpret_cast<float4 *>(t + oGD), reinterpret_cast<float2 *>(t + oU),
            reinterpret_cast<float2 *>(t + orat), reinterpret_cast<float4 *>(t + oer),
            reinterpret_cast<float *>(t + ooff), reinterpret_cast<float *>(t + otau)};
  }
  __device__ float *red_buf(int k) const { return red + static_cast<size_t>(k) * FT * waves * red_vals; }
};

// Orders a wave's own LDS writes before its later LDS reads by other lanes.
__device__ inline void wave_lds_sync_adj() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Staging of one tile (lit entries t0 .. t0 + nf - 1 of chirp n) by the staging waves.
template <int MB, int FT>
__device__ void adj_stage_tile(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                               const AdjSmem<MB, FT> &sm, const AdjTile &tl, int n, int32_t cnt,
                               int32_t t0, int nf, int m_tile0, int st) {
  const int P = rc.P, E = sh.E;
  const double slope = rc.slope;
  // each staging wave takes half of the tile's facets through all steps
  constexpr int kHalf = FT / 2;
  static_assert(FT % 2 == 0 && kHalf <= 64, "two staging waves split the tile");
  const int lane = st & 63, i0 = (st >> 6) * kHalf;
  Geo *geo = sm.geo;
  GLin *glin = sm.glin;
  for (int i = i0 + lane; i < i0 + kHalf && lane < kHalf; i += 64) {
    if (i < nf)
      entry_geometry(sc, rc, n, cnt, t0 + i, geo[i]);
    else
      geo[i].valid = 0;
    make_glin(geo[i], rc, m_tile0, glin[i]);
    if (rc.intra && geo[i].valid) glin[i].quad = static_cast<float>(chord_curvature(geo[i], rc, m_tile0, MB));
  }
  wave_lds_sync_adj();
  for (int task = lane; task < kHalf * E; task += 64) {
    const int i = i0 + task / E, e = task % E;
    const Geo g = lds_copy(geo[i]);  // one batch of LDS reads
    float2 *Ue = tl.U + (i * E + e) * sh.B_w;
    float2 *re = tl.rat + (i * E + e) * sm.rat_b;
    if (!g.valid) {
      for (int bb = 0; bb < sh.B_w; ++bb) Ue[bb] = make_float2(0.0f, 0.0f);
      for (int bb = 0; bb < sm.rat_b; ++bb) re[bb] = make_float2(1.0f, 0.0f);
      tl.off[i * E + e] = 0.0f;
      tl.er[i * E + e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      tl.tau[i * E + e] = 0.0f;
      continue;
    }
    const double dx = sm.elem[3 * e + 0] - g.c[0];
    const double dy = sm.elem[3 * e + 1] - g.c[1];
    const double dz = sm.elem[3 * e + 2] - g.c[2];
    const double Rn = sqrt(dx * dx + dy * dy + dz * dz);
    const double inv_rd = 1.0 / Rn;
    const double tau = Rn * (1.0 / kC0);
    // Tx element: reference delay of its own side tref_t, of the other side tref_r
    const bool tx = e < P;
    const double t_self = tx ? g.tref_t : g.tref_r, t_other = tx ? g.tref_r : g.tref_t;
    const double d = tau - t_self;
    double psi0 = rc.f0 * tau - 0.5 * slope * tau * tau - slope * t_other * d -
                  0.5 * slope * g.tref_t * g.tref_r;
    const double offv = tx ? sh.two_pi_slope * d : d;
    psi0 -= floor(psi0);
    double delta = rc.df * tau;
    delta -= floor(delta);
    const float inv_r = static_cast<float>(inv_rd);
    if (!rc.intra) {
      for (int bb = 0; bb < sh.B_w; ++bb)
        Ue[bb] = phasor_m2pi<float>(psi0 + static_cast<double>(m_tile0 + bb * MB) * delta, inv_r);
      re[0] = phasor_m2pi<float>(delta, 1.0f);
    } else {
      // as the forward: exact FP64 phases at both ends of each block, joined by the chord
      for (int bb = 0; bb < sh.B_w; ++bb) {
        const int ma = m_tile0 + bb * MB;
        const double pa = element_phase(g, rc, sm.elem + 3 * e, tx, ma);
        const double pb = element_phase(g, rc, sm.elem + 3 * e, tx, ma + MB);
        Ue[bb] = phasor_m2pi<float>(pa - floor(pa), inv_r);
        re[bb] = phasor_m2pi<float>((pb - pa) * (1.0 / MB), 1.0f);
      }
    }
    tl.off[i * E + e] = static_cast<float>(offv);
    tl.er[i * E + e] = make_float4(static_cast<float>(dx * inv_rd), static_cast<float>(dy * inv_rd),
                                   static_cast<float>(dz * inv_rd), inv_r);
    tl.tau[i * E + e] = static_cast<float>(tau);
  }
  // G and its node derivatives, one facet at a time: its record is read from LDS into
  // registers once (in one batch), not field by field inside the branches
  for (int ii = 0; ii < kHalf; ++ii) {
    const int i = i0 + ii;
    const GLin q = lds_copy(glin[i]);
    for (int j = lane; j < sh.M_t; j += 64) {
      float2 gv, dv[3];
      g_lin_grad(q, j, gv, dv);
      if (rc.intra) {
        // the forward's curvature factor exp(-j 2 pi q jj (jj - MB)) to first order, on G
        // and on its node derivatives alike
        const int jj = j % MB;
        const float x = 6.283185307179586f * q.quad * static_cast<float>(jj * (jj - MB));
        gv = make_float2(fmaf(gv.y, x, gv.x), fmaf(-gv.x, x, gv.y));
#pragma unroll
        for (int k = 0; k < 3; ++k) dv[k] = make_float2(fmaf(dv[k].y, x, dv[k].x), fmaf(-dv[k].x, x, dv[k].y));
      }
      float4 *dst = tl.GD + (static_cast<int64_t>(i) * sh.M_t + j) * 2;
      dst[0] = make_float4(gv.x, gv.y, dv[0].x, dv[0].y);
      dst[1] = make_float4(dv[1].x, dv[1].y, dv[2].x, dv[2].y);
    }
  }
}

// Sums of a finished tile's per-wave channel sums (fixed wave order) into the
// per-(chirp, facet, tile) partials, by the staging waves.
// With the delay within the chirp, the three velocity sums go to partial_v [slot][4].
template <int MB, int FT>
__device__ void adj_flush(const AdjSmem<MB, FT> &sm, const float *red, float *partial,
                          float *partial_v, int64_t F, const EchoShape &sh, int n, int mt, int ot,
                          int32_t t0, int nf, int st) {
  const int nv = partial_v ? 10 : 7;
  for (int task = st; task < nf * nv; task += kStagingThreads) {
    const int i = task / nv, k = task % nv;
    float s = 0.0f;
    for (int wv = 0; wv < sm.waves; ++wv) s += red[(i * sm.waves + wv) * sm.red_vals + k];
    const int64_t slot = ((static_cast<int64_t>(n) * F + t0 + i) * sh.m_tiles + mt) * sh.o_tiles + ot;
    if (k < 7)
      partial[slot * kAdjVals + k] = s;
    else
      partial_v[slot * 4 + (k - 7)] = s;
  }
}

// One workgroup per (chirp, sample tile, channel tile): accumulating waves (thread (o, b)
// holds conj(g) for MB samples of channel o in registers) and two staging waves, with
// double-buffered tiles of FT lit facets as in the forward kernel. Both branches pass
// the same barriers: one per tile and a final one.
// INTRA: the delay within the chirp (rc.intra), with the velocity sums into partial_v.
template <int MB, int FT, bool INTRA>
__global__ void __launch_bounds__(512) adjoint_echo_kernel(DevScene sc, RadarConst rc,
                                                           const double *elem, AdjShape ash,
                                                           const float2 *grad_echo,
                                                           float *partial, float *partial_v) {
  extern __shared__ __align__(16) unsigned char adj_smem[];
  const EchoShape &sh = ash.sh;
  AdjSmem<MB, FT> sm;
  sm.carve(adj_smem, sh, INTRA);
  const int tid = threadIdx.x;
  for (int i = tid; i < 3 * sh.E; i += blockDim.x) sm.elem[i] = elem[i];
  __syncthreads();
  const int per_chirp = sh.m_tiles * sh.o_tiles;
  const int n = blockIdx.x / per_chirp;
  const int mt = (blockIdx.x % per_chirp) / sh.o_tiles;
  const int ot = blockIdx.x % sh.o_tiles;
  const int m_tile0 = mt * sh.M_t;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t n_tiles = (cnt + FT - 1) / FT;

  if (tid >= sh.n_compute) {
    const int st = tid - sh.n_compute;
    if (n_tiles > 0) adj_stage_tile<MB, FT>(sc, rc, sh, sm, sm.tile(0), n, cnt, 0, min(FT, cnt), m_tile0, st);
    for (int32_t k = 0; k < n_tiles; ++k) {
      __syncthreads();
      if (k > 0)
        adj_flush<MB, FT>(sm, sm.red_buf((k - 1) & 1), partial, partial_v, ash.F, sh, n, mt, ot,
                          (k - 1) * FT, min(FT, cnt - (k - 1) * FT), st);
      const int32_t t1 = (k + 1) * FT;
      if (t1 < cnt)
        adj_stage_tile<MB, FT>(sc, rc, sh, sm, sm.tile((k & 1) ^ 1), n, cnt, t1, min(FT, cnt - t1),
                               m_tile0, st);
    }
    __syncthreads();
    if (n_tiles > 0)
      adj_flush<MB, FT>(sm, sm.red_buf((n_tiles - 1) & 1), partial, partial_v, ash.F, sh, n, mt,
                        ot, (n_tiles - 1) * FT, min(FT, cnt - (n_tiles - 1) * FT), st);
    return;
  }

  const int P = rc.P, Q = rc.Q, E = sh.E;
  const int ol = tid % sh.O_w, b = tid / sh.O_w;
  const int o = ot * sh.O_w + ol;
  const bool o_ok = b < sh.B_w && o < sh.O;
  const int p = o_ok ? o / Q : 0, q = o_ok ? o % Q : 0;
  const int m_base = m_tile0 + b * MB;
  const double slope = rc.slope;
  const float kf0 = static_cast<float>(2.0 * kPi / kC0);
  const int wv = tid >> 6;

  // conj(g) for this thread's samples
  float2 gq[MB];
  {
    const float2 *gsrc = grad_echo + (static_cast<int64_t>(o_ok ? o : 0) * rc.N + n) * rc.M;
#pragma unroll
    for (int j = 0; j < MB; ++j) {
      const bool in = o_ok && (m_base + j < rc.M);
      const float2 v = in ? gsrc[m_base + j] : make_float2(0.0f, 0.0f);
      gq[j] = make_float2(v.x, -v.y);
    }
  }

  for (int32_t kt = 0; kt < n_tiles; ++kt) {
    __syncthreads();
    const AdjTile tl = sm.tile(kt & 1);
    float *red = sm.red_buf(kt & 1);
    const int nf = min(FT, cnt - kt * FT);
    for (int i = 0; i < nf; ++i) {
      constexpr int NV = INTRA ? 10 : 7;
      float v[NV];
#pragma unroll
      for (int k = 0; k < NV; ++k) v[k] = 0.0f;
      if (o_ok) {
        const float2 up = tl.U[(i * E + p) * sh.B_w + b];
        const float2 uq = tl.U[(i * E + P + q) * sh.B_w + b];
        const int rb = INTRA ? b : 0;
        const float2 rp = tl.rat[(i * E + p) * sm.rat_b + rb];
        const float2 rq = tl.rat[(i * E + P + q) * sm.rat_b + rb];
        const float eps = tl.off[i * E + p] * tl.off[i * E + P + q];
        float2 z = make_float2(fma_r(up.x, uq.x, -up.y * uq.y), fma_r(up.x, uq.y, up.y * uq.x));
        z = make_float2(fma_r(-eps, z.y, z.x), fma_r(eps, z.x, z.y));
        const float2 r = make_float2(fma_r(rp.x, rq.x, -rp.y * rq.y), fma_r(rp.x, rq.y, rp.y * rq.x));
        // per sample: (G, D0) and (D1, D2) as two 16-byte LDS reads, a block ahead
        const float4 *gd = tl.GD + (static_cast<int64_t>(i) * sh.M_t + b * MB) * 2;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, s3 = 0.0f, a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
        constexpr int kB = 2;
        float4 ca[2 * kB], cb[2 * kB];
#pragma unroll
        for (int u = 0; u < 2 * kB; ++u) ca[u] = gd[u];
#pragma unroll
        for (int j0 = 0; j0 < MB; j0 += kB) {
          if (j0 + kB < MB) {
#pragma unroll
            for (int u = 0; u < 2 * kB; ++u) cb[u] = gd[2 * (j0 + kB) + u];
          }
#pragma unroll
          for (int jj = 0; jj < kB; ++jj) {
            const int j = j0 + jj;
            const float4 g0 = ca[2 * jj], g1 = ca[2 * jj + 1];  // (G, D0), (D1, D2)
            const float2 w = make_float2(fma_r(gq[j].x, z.x, -gq[j].y * z.y),
                                         fma_r(gq[j].x, z.y, gq[j].y * z.x));
            // Re y straight into its sum (two FMAs); Im y is kept for the two sums it feeds
            s0 = fma_r(g0.x, w.x, fma_r(-g0.y, w.y, s0));
            const float yy = fma_r(g0.x, w.y, g0.y * w.x);
            s1 += yy;
            s2 = fma_r(static_cast<float>(j), yy, s2);
            if constexpr (INTRA) s3 = fma_r(static_cast<float>(j * j), yy, s3);
            a0 = fma_r(g0.z, w.x, fma_r(-g0.w, w.y, a0));
            a1 = fma_r(g1.x, w.x, fma_r(-g1.y, w.y, a1));
            a2 = fma_r(g1.z, w.x, fma_r(-g1.w, w.y, a2));
            const float zx = fma_r(z.x, r.x, -z.y * r.y);
            z.y = fma_r(z.x, r.y, z.y * r.x);
            z.x = zx;
          }
#pragma unroll
          for (int u = 0; u < 2 * kB; ++u) ca[u] = cb[u];
        }
        // sum_m m Im(y) (and m^2 Im(y)) with m counted from the block start; shift to
        // absolute m
        const float mb = static_cast<float>(m_base);
        if constexpr (INTRA) s3 = fma_r(mb * mb, s1, fma_r(2.0f * mb, s2, s3));
        s2 = fma_r(mb, s1, s2);
        // dL/dR_p and dL/dR_q of this channel, then onto the centroid: dR/dc = -e_hat
        const float tpq = tl.tau[i * E + p] + tl.tau[i * E + P + q];
        const float f0mu = static_cast<float>(rc.f0 - slope * static_cast<double>(tpq));
        const float kap = kf0 * (f0mu * s1 + static_cast<float>(rc.df) * s2);
        const float4 ep = tl.er[i * E + p], eq = tl.er[i * E + P + q];
        const float cp = kap - s0 * ep.w, cq = kap - s0 * eq.w;
        v[0] = -(cp * ep.x + cq * eq.x);
        v[1] = -(cp * ep.y + cq * eq.y);
        v[2] = -(cp * ep.z + cq * eq.z);
        v[3] = s0;
        v[4] = a0;
        v[5] = a1;
        v[6] = a2;
        if constexpr (INTRA) {
          // the velocity's share through the phase at the sample times
          const float kv = -kf0 * static_cast<float>(1.0 / rc.fs) *
                           (f0mu * s2 + static_cast<float>(rc.df) * s3);
          v[7] = kv * (ep.x + eq.x);
          v[8] = kv * (ep.y + eq.y);
          v[9] = kv * (ep.z + eq.z);
        }
      }
      // every lane of the (whole) wave takes part: DPP reads all lanes
#pragma unroll
      for (int k = 0; k < NV; ++k) {
        const float s = wave_sum(v[k]);
        if ((tid & 63) == 0) red[(i * sm.waves + wv) * sm.red_vals + k] = s;
      }
    }
  }
  __syncthreads();
}

// Per lit (chirp, facet): sum the partials and apply the chain rule to the three
// world vertices (FP64). Writes gxw[(n F + f) * 9 + 3 corner + axis]; with partial_v, the
// velocity's sums over samples into gxv[(n F + f) * 3 + axis].
__global__ void __launch_bounds__(256) facet_grad_kernel(DevScene sc, RadarConst rc,
                                                         AdjShape ash, const float *partial,
                                                         float *gxw, const float *partial_v,
                                                         float *gxv) {
  const int n = blockIdx.y;
  const int32_t item = blockIdx.x * blockDim.x + threadIdx.x;
  if (item >= sc.vis_cnt[n]) return;
  const EchoShape &sh = ash.sh;
  const int nslots = sh.m_tiles * sh.o_tiles;
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  const float *src = partial + (static_cast<int64_t>(n) * ash.F + item) * nslots * kAdjVals;
  for (int s = 0; s < nslots; ++s)
    for (int k = 0; k < 7; ++k) acc[k] += src[s * kAdjVals + k];
  const int64_t f = sc.vis_idx[static_cast<int64_t>(n) * sc.n_facets + item];
  if (partial_v) {
    double vs[3] = {0.0, 0.0, 0.0};
    const float *pv = partial_v + (static_cast<int64_t>(n) * ash.F + item) * nslots * 4;
    for (int s = 0; s < nslots; ++s)
      for (int k = 0; k < 3; ++k) vs[k] += pv[s * 4 + k];
    float *ov = gxv + (static_cast<int64_t>(n) * sc.n_facets + f) * 3;
    for (int k = 0; k < 3; ++k) {
      const float g = static_cast<float>(vs[k]);
      ov[k] = sh.accumulate ? ov[k] + g : g;
    }
  }
  const int ii = find_inst(sc.inst, sc.n_inst, f);
  const DevInstance &I = sc.inst[ii];
  const int64_t lt = f - I.facet_base;
  const double t = n * rc.tc;
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
  double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                 e1[0] * e2[1] - e1[1] * e2[0]};
  const double nl = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
  double nh[3] = {N[0] / nl, N[1] / nl, N[2] / nl};
  double dT[3], dR[3];
  for (int k = 0; k < 3; ++k) {
    dT[k] = rc.tx_c[k] - c[k];
    dR[k] = rc.rx_c[k] - c[k];
  }
  const double rt = sqrt(dT[0] * dT[0] + dT[1] * dT[1] + dT[2] * dT[2]);
  const double rr = sqrt(dR[0] * dR[0] + dR[1] * dR[1] + dR[2] * dR[2]);
  double ut[3], ur[3], w[3];
  for (int k = 0; k < 3; ++k) {
    ut[k] = dT[k] / rt;
    ur[k] = dR[k] / rr;
    w[k] = ut[k] + ur[k];
  }
  const double obl = 0.5 * (nh[0] * w[0] + nh[1] * w[1] + nh[2] * w[2]);
  const double area = 0.5 * nl;
  const double S = acc[3];
  const double go = S / obl, gA = S / area;
  const double gb[3] = {acc[4], acc[5], acc[6]};
  double gx[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
  double gc[3] = {acc[0], acc[1], acc[2]};  // through the element distances
  // beta_i = w . (x_i - c)
  double gw[3] = {0, 0, 0};
  for (int v = 0; v < 3; ++v)
    for (int k = 0; k < 3; ++k) {
      gx[v][k] += gb[v] * w[k];
      gc[k] -= gb[v] * w[k];
      gw[k] += gb[v] * (x[v][k] - c[k]);
    }
  // o = n . w / 2
  for (int k = 0; k < 3; ++k) gw[k] += 0.5 * go * nh[k];
  double gn[3] = {0.5 * go * w[0], 0.5 * go * w[1], 0.5 * go * w[2]};
  // w = dT/|dT| + dR/|dR|, dT = T - c, dR = R - c
  const double wt = gw[0] * ut[0] + gw[1] * ut[1] + gw[2] * ut[2];
  const double wr = gw[0] * ur[0] + gw[1] * ur[1] + gw[2] * ur[2];
  for (int k = 0; k < 3; ++k) {
    gc[k] -= (gw[k] - wt * ut[k]) / rt;
    gc[k] -= (gw[k] - wr * ur[k]) / rr;
  }
  // n = N / |N| and A = |N| / 2
  const double nn = gn[0] * nh[0] + gn[1] * nh[1] + gn[2] * nh[2];
  double gN[3];
  for (int k = 0; k < 3; ++k) gN[k] = (gn[k] - nn * nh[k]) / nl + 0.5 * gA * nh[k];
  // N = e1 x e2
  const double ge1[3] = {e2[1] * gN[2] - e2[2] * gN[1], e2[2] * gN[0] - e2[0] * gN[2],
                         e2[0] * gN[1] - e2[1] * gN[0]};
  const double ge2[3] = {gN[1] * e1[2] - gN[2] * e1[1], gN[2] * e1[0] - gN[0] * e1[2],
                         gN[0] * e1[1] - gN[1] * e1[0]};
  for (int k = 0; k < 3; ++k) {
    gx[1][k] += ge1[k];
    gx[2][k] += ge2[k];
    gx[0][k] -= ge1[k] + ge2[k];
    for (int v = 0; v < 3; ++v) gx[v][k] += gc[k] / 3.0;
  }
  float *out = gxw + (static_cast<int64_t>(n) * sc.n_facets + f) * 9;
  for (int v = 0; v < 3; ++v)
    for (int k = 0; k < 3; ++k) {
      const float g = static_cast<float>(gx[v][k]);
      out[3 * v + k] = sh.accumulate ? out[3 * v + k] + g : g;  // accumulate: further path types
    }
}

// out = conj(gamma) in: the echo gradient of a path type whose echo was added times gamma.
__global__ void scale_conj_kernel(const float2 *in, float2 *out, int64_t n, float gr, float gi) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const float2 v = in[i];
    out[i] = make_float2(gr * v.x + gi * v.y, gr * v.y - gi * v.x);
  }
}

__global__ void fill_zero_kernel(float *p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0f;
}

// Per facet and component: the sum over chirps of the world-vertex gradients and of t_n
// times them (FP64, chirp order): gsum[f * 9 + c], gtsum[f * 9 + c]. Consecutive threads
// read consecutive components of one chirp's row. gxv (or null): the velocity's sums over
// the samples of each chirp [N][F][3], a third of which joins the t_n-weighted sum of each
// corner (the vertex gather adds the three corners back up for the velocity).
__global__ void __launch_bounds__(256) facet_chirp_sum_kernel(const float *gxw, const float *gxv,
                                                              int64_t n_facets, int N, double tc,
                                                              double *gsum, double *gtsum,
                                                              const double *dbsum) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= n_facets * 9) return;
  const int64_t f = idx / 9;
  const int axis = static_cast<int>(idx % 3);
  double g = 0.0, gt = 0.0;
  for (int n = 0; n < N; ++n) {
    const double v = gxw[static_cast<int64_t>(n) * n_facets * 9 + idx];
    g += v;
    gt += (n * tc) * v;
    if (gxv) gt += gxv[(static_cast<int64_t>(n) * n_facets + f) * 3 + axis] * (1.0 / 3.0);
  }
  if (dbsum) {  // the double-bounce connections' sums over chirps (plain, t_n-weighted)
    g += dbsum[idx];
    gt += dbsum[n_facets * 9 + idx];
  }
  gsum[idx] = g;
  gtsum[idx] = gt;
}

// One instance: per body vertex, gather over incident (triangle, corner) the chirp-summed
// world gradients, rotate to the body frame and accumulate into gv; vpart[v] = sum over
// chirps of t_n (world gradient of v at chirp n) for the velocity gradient.
__global__ void __launch_bounds__(256) vertex_gather_kernel(
    const double *gsum, const double *gtsum, const double *rot, int64_t facet_base,
    const int32_t *csr_off, const int32_t *csr_ent, int32_t n_verts, float *gv, double *vpart) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_verts) return;
  double g[3] = {0, 0, 0}, gt[3] = {0, 0, 0};
  const int32_t b = csr_off[v], e = csr_off[v + 1];
  for (int32_t k = b; k < e; ++k) {
    const int32_t ent = csr_ent[k];  // triangle * 3 + corner
    const int64_t o = (facet_base + ent / 3) * 9 + 3 * (ent % 3);
    for (int c = 0; c < 3; ++c) {
      g[c] += gsum[o + c];
      gt[c] += gtsum[o + c];
    }
  }
  // body gradient = R^T (world gradient)
  for (int k = 0; k < 3; ++k) {
    const double body = rot[0 * 3 + k] * g[0] + rot[1 * 3 + k] * g[1] + rot[2 * 3 + k] * g[2];
    if (gv) gv[3 * v + k] += static_cast<float>(body);
    vpart[3 * v + k] = gt[k];
  }
}

// Fixed-order sum of vpart over the vertices of one instance -> grad_vel[inst].
__global__ void __launch_bounds__(256) velocity_reduce_kernel(const double *vpart, int32_t n_verts,
                                                              double *out3) {
  __shared__ double s[3][256];
  double a[3] = {0, 0, 0};
  for (int32_t v = threadIdx.x; v < n_verts; v += blockDim.x)
    for (int k = 0; k < 3; ++k) a[k] += vpart[3 * v + k];
  for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < static_cast<unsigned>(w))
      for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) out3[k] = s[k][0];
}

}  // namespace

constexpr int kAdjMB = 64;
constexpr int kAdjFT = 8;

size_t adjoint_partial_floats(const EchoShape &sh, int64_t N, int64_t F) {
  return static_cast<size_t>(N) * F * sh.m_tiles * sh.o_tiles * kAdjVals;
}

int adjoint_tile_m() { return kAdjMB; }

size_t adjoint_smem_bytes(const EchoShape &sh, bool intra) {
  return AdjLayout<kAdjMB, kAdjFT>(sh, intra).total;
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_adjoint_finish(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                                 const float *partial, float *gxw, hipStream_t s,
                                 const float *partial_v, float *gxv) {
  if (sc.n_facets == 0) return hipGetLastError();
  if ((partial_v == nullptr) != (gxv == nullptr)) return hipErrorInvalidValue;
  AdjShape ash{sh, static_cast<int32_t>(sc.n_facets), 0};
  dim3 g2(static_cast<unsigned>((sc.n_facets + 255) / 256), rc.N);
  hipLaunchKernelGGL(facet_grad_kernel, g2, dim3(256), 0, s, sc, rc, ash, partial, gxw, partial_v,
                     gxv);
  return hipGetLastError();
}

hipError_t launch_adjoint(const DevScene &sc, const RadarConst &rc, const double *elem,
                          const EchoShape &sh, const void *grad_echo, float *partial, float *gxw,
                          hipStream_t s, float *partial_v, float *gxv) {
  AdjShape ash{sh, static_cast<int32_t>(sc.n_facets), 0};
  const int threads = sh.n_compute + kStagingThreads;
  const bool intra = rc.intra != 0;
  if (intra != (partial_v != nullptr) || (partial_v == nullptr) != (gxv == nullptr))
    return hipErrorInvalidValue;
  hipError_t e =
      sh.accumulate ? hipSuccess : launch_fill_zero(gxw, static_cast<int64_t>(rc.N) * sc.n_facets * 9, s);
  if (e == hipSuccess && intra && !sh.accumulate)
    e = launch_fill_zero(gxv, static_cast<int64_t>(rc.N) * sc.n_facets * 3, s);
  if (e != hipSuccess || sc.n_facets == 0) return e;
  const unsigned grid = static_cast<unsigned>(rc.N) * sh.m_tiles * sh.o_tiles;
  if (intra)
    hipLaunchKernelGGL((adjoint_echo_kernel<kAdjMB, kAdjFT, true>), dim3(grid), dim3(threads),
                       adjoint_smem_bytes(sh, true), s, sc, rc, elem, ash,
                       static_cast<const float2 *>(grad_echo), partial, partial_v);
  else
    hipLaunchKernelGGL((adjoint_echo_kernel<kAdjMB, kAdjFT, false>), dim3(grid), dim3(threads),
                       adjoint_smem_bytes(sh, false), s, sc, rc, elem, ash,
                       static_cast<const float2 *>(grad_echo), partial, nullptr);
  return launch_adjoint_finish(sc, rc, sh, partial, gxw, s, partial_v, gxv);
}

hipError_t launch_scale_conj(const void *in, void *out, int64_t n, double gr, double gi,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(scale_conj_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     static_cast<const float2 *>(in), static_cast<float2 *>(out), n,
                     static_cast<float>(gr), static_cast<float>(gi));
  return hipGetLastError();
}

hipError_t launch_facet_chirp_sum(const float *gxw, const float *gxv, int64_t n_facets, int N,
                                  double tc, double *gsum, double *gtsum, hipStream_t s,
                                  const double *dbsum) {
  if (n_facets > 0) {
    const int64_t n = n_facets * 9;
    hipLaunchKernelGGL(facet_chirp_sum_kernel, dim3(static_cast<unsigned>((n + 255) / 256)),
                       dim3(256), 0, s, gxw, gxv, n_facets, N, tc, gsum, gtsum, dbsum);
  }
  return hipGetLastError();
}

hipError_t launch_vertex_gather(const double *gsum, const double *gtsum, const double *rot_dev,
                                int64_t facet_base, const int32_t *csr_off, const int32_t *csr_ent,
                                int32_t n_verts, float *gv, double *vpart, double *vel_out,
                                hipStream_t s) {
  if (n_verts > 0) {
    hipLaunchKernelGGL(vertex_gather_kernel, dim3((n_verts + 255) / 256), dim3(256), 0, s, gsum,
                       gtsum, rot_dev, facet_base, csr_off, csr_ent, n_verts, gv, vpart);
  }
  hipLaunchKernelGGL(velocity_reduce_kernel, dim3(1), dim3(256), 0, s, vpart, n_verts, vel_out);
  return hipGetLastError();
}

}  // namespace rsim
