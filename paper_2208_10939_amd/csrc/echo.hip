// Coherent facet sum: the echo frequency response H[o, n, m] (Sections 2.2, 3.2;
// eqs. (7), (9)-(13)) for every lit facet of chirp n, frequency sample m and
// virtual channel o = p Q + q:
//
//   H[o,n,m] = sum_f G_f(m) U_fp(m) U_fq(m) exp(+j 2 pi slope d_p e_q)
//   G_f(m)   = j o_f A_f Phi(k_m b_f) / (2 pi)          (closed-form facet integral)
//   U_fe(m)  = exp(-j 2 pi psi_e(m)) / R_e,  psi_e(m) = psi_e(0) + m df tau_e
//
// which regroups f_m tau - slope tau^2 / 2 (tau = tau_p + tau_q) exactly into a Tx
// part, an Rx part and the cross term slope d_p e_q, where d_p, e_q are the element
// delays relative to the phase-centre delays (|2 pi slope d_p e_q| is ~1e-5 rad for
// the arrays here; it is applied as a short Taylor polynomial, exact to rounding).
//
// Work split (one item = chirp n x sample tile x channel tile): a workgroup holds
// n_compute accumulating threads, thread (o, b) keeping MB consecutive samples of one
// channel in registers, and two staging waves. The lit facets are taken in tiles of FT;
// while the accumulating threads sum tile k from one LDS buffer, the staging waves fill
// the other with tile k + 1, in FP64: facet geometry, element distances, phases reduced
// to turns (the only FP64 arithmetic of the sum); then G_f(m) for the tile's samples and
// each element's phasor at every block start. One workgroup barrier per tile hands the
// buffers over. Block starts are re-seeded from FP64 phases, so a phasor recurrence
// never runs more than MB steps.
#include "echo_common.h"

namespace rsim {

template <typename R, int MB, int FT>
struct EchoLayout {
  using C = typename Cx<R>::T;
  static constexpr bool kRotated = sizeof(R) == 4;  // FP32 keeps G (-j)^m as well
  size_t elem, geo, glin, buf[2], G, G1, U, rat, off, total;

  __host__ __device__ explicit EchoLayout(const EchoShape &sh) {
    auto up = [](size_t b) { return (b + 15) & ~size_t(15); };
    size_t b = 0;
    elem = b;
    b = up(b + sizeof(double) * 3 * sh.E);
    geo = b;  // [FT]
    b = up(b + sizeof(Geo) * FT);
    glin = b;  // [FT], FP32 path
    b = up(b + (kRotated ? sizeof(GLin) * FT : 0));
    // offsets inside one tile buffer
    size_t t = 0;
    G = t;
    t += sizeof(C) * FT * sh.M_t;
    G1 = t;
    t += kRotated ? sizeof(C) * FT * sh.M_t : 0;
    U = t;
    t += sizeof(C) * FT * sh.E * sh.B_w;
    rat = t;
    t += sizeof(C) * FT * sh.E * sh.B_w;
    off = t;
    t = up(t + sizeof(R) * FT * sh.E);
    buf[0] = b;
    buf[1] = b + t;
    // the output staging reuses the tile buffers: O_w x min(MB, 16) values
    const size_t out_stage = sizeof(C) * sh.O_w * ((MB < 16) ? MB : 16);
    total = b + (2 * t > out_stage ? 2 * t : out_stage);
  }
};

template <typename R, int MB, int FT>
struct EchoTile {
  using C = typename Cx<R>::T;
  C *G;    // [FT][M_t]
  C *G1;   // [FT][M_t]: G (-j)^(m mod 4), for quarter-turn-rotated recurrences (FP32)
  C *U;    // [B_w][FT][E]
  C *rat;  // [B_w][FT][E]: per-sample phasor step of each block
  R *off;  // [FT][E]
};

template <typename R, int MB, int FT>
struct EchoSmem {
  using C = typename Cx<R>::T;
  double *elem;  // [E][3]
  Geo *geo;      // [FT]: entry i written and read by the staging wave that owns it
  GLin *glin;    // [FT]: the same, FP32 path
  unsigned char *buf0;
  size_t buf_stride, oG, oG1, oU, orat, ooff;

  __device__ void carve(unsigned char *base, const EchoShape &sh) {
    const EchoLayout<R, MB, FT> L(sh);
    elem = reinterpret_cast<double *>(base + L.elem);
    geo = reinterpret_cast<Geo *>(base + L.geo);
    glin = reinterpret_cast<GLin *>(base + L.glin);
    buf0 = base + L.buf[0];
    buf_stride = L.buf[1] - L.buf[0];
    oG = L.G;
    oG1 = L.G1;
    oU = L.U;
    orat = L.rat;
    ooff = L.off;
  }
  // tile buffer k (0 or 1), by address arithmetic so no array of pointers is indexed
  __device__ EchoTile<R, MB, FT> tile(int k) const {
    unsigned char *t = buf0 + static_cast<size_t>(k) * buf_stride;
    return {reinterpret_cast<C *>(t + oG), reinterpret_cast<C *>(t + oG1),
            reinterpret_cast<C *>(t + oU), reinterpret_cast<C *>(t + orat),
            reinterpret_cast<R *>(t + ooff)};
  }
};

// Orders a wave's own LDS writes before its later LDS reads by other lanes.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// Staging of one tile (entries t0 .. t0 + nf - 1 of chirp n) by the staging waves,
// st = staging thread index in [0, kStagingThreads).
template <typename R, int MB, int FT>
__device__ void stage_tile(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                           const EchoSmem<R, MB, FT> &sm, const EchoTile<R, MB, FT> &tl, int n,
                           int32_t cnt, int32_t t0, int nf, int m_tile0, int st) {
  using C = typename Cx<R>::T;
  const int P = rc.P, E = sh.E;
  const double slope = rc.slope;
  // Each staging wave takes half of the tile's entries through all three steps, so the
  // geometry it reads back was written by itself and needs no workgroup barrier.
  constexpr int kHalf = FT / 2;
  static_assert(FT % 2 == 0 && kHalf <= 64, "two staging waves split the tile");
  const int lane = st & 63, i0 = (st >> 6) * kHalf;
  Geo *geo = sm.geo;
  GLin *glin = sm.glin;
  // A: facet / point geometry (FP64)
  for (int i = i0 + lane; i < i0 + kHalf && lane < kHalf; i += 64) {
    if (i < nf)
      entry_geometry(sc, rc, n, cnt, t0 + i, geo[i]);
    else
      geo[i].valid = 0;
    if constexpr (EchoLayout<R, MB, FT>::kRotated) {
      make_glin(geo[i], rc, m_tile0, glin[i]);
      if (rc.intra && geo[i].valid) glin[i].quad = static_cast<float>(chord_curvature(geo[i], rc, m_tile0, MB));
    }
  }
  wave_lds_sync();
  // B1: per element distance, phases in FP64 reduced to turns
  for (int task = lane; task < kHalf * E; task += 64) {
    const int i = i0 + task / E, e = task % E;
    const Geo g = lds_copy(geo[i]);  // one batch of LDS reads
    // block-major [B_w][FT][E]: the lanes of a wave (consecutive channels) then read
    // consecutive Rx elements of one block
    C *Ue = tl.U + i * E + e;
    C *re = tl.rat + i * E + e;
    const int bstride = FT * E;
    if (!g.valid) {
      for (int bb = 0; bb < sh.B_w; ++bb) {
        Ue[bb * bstride] = {R(0), R(0)};
        re[bb * bstride] = {R(1), R(0)};
      }
      tl.off[i * E + e] = R(0);
      continue;
    }
    const double dx = sm.elem[3 * e + 0] - g.c[0];
    const double dy = sm.elem[3 * e + 1] - g.c[1];
    const double dz = sm.elem[3 * e + 2] - g.c[2];
    const double Rn = sqrt(dx * dx + dy * dy + dz * dz);
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
    R inv_r;
    if constexpr (sizeof(R) == 4)
      inv_r = __builtin_amdgcn_rcpf(static_cast<float>(Rn));  // amplitude only: 1 ulp
    else
      inv_r = 1.0 / Rn;
    if (!rc.intra) {
      const C step = phasor_m2pi<R>(delta, R(1));
      for (int bb = 0; bb < sh.B_w; ++bb) {
        const double m0 = static_cast<double>(m_tile0 + bb * MB);
        Ue[bb * bstride] = phasor_m2pi<R>(psi0 + m0 * delta, inv_r);
        re[bb * bstride] = step;
      }
    } else {
      // delay at each sample time t_n + m / fs: exact FP64 phases at both ends of each
      // block; the block runs along their chord (the curvature goes into G)
      for (int bb = 0; bb < sh.B_w; ++bb) {
        const int ma = m_tile0 + bb * MB;
        const double pa = element_phase(g, rc, sm.elem + 3 * e, e < P, ma);
        const double pb = element_phase(g, rc, sm.elem + 3 * e, e < P, ma + MB);
        Ue[bb * bstride] = phasor_m2pi<R>(pa - floor(pa), inv_r);
        re[bb * bstride] = phasor_m2pi<R>((pb - pa) * (1.0 / MB), R(1));
      }
    }
    tl.off[i * E + e] = static_cast<R>(offv);
  }
  // B2: G_f(m) for the tile's samples, one entry at a time: its record is read from LDS
  // into registers once (in one batch), not field by field inside the branches
  for (int ii = 0; ii < kHalf; ++ii) {
    const int i = i0 + ii;
    GLin q{};
    Geo g{};
    if constexpr (EchoLayout<R, MB, FT>::kRotated)
      q = lds_copy(glin[i]);
    else
      g = lds_copy(geo[i]);
    for (int j = lane; j < sh.M_t; j += 64) {
      C val = {R(0), R(0)};
      if constexpr (EchoLayout<R, MB, FT>::kRotated) {
        val = g_lin(q, j);
        if (rc.intra) {
          // deviation of the phase from its chord over the block:
          // exp(-j 2 pi q jj (jj - MB)) to first order (|2 pi q jj (jj - MB)| <= ~2e-4 rad)
          const int jj = j % MB;
          const float x = 6.283185307179586f * q.quad * static_cast<float>(jj * (jj - MB));
          val = {fma_r(val.y, x, val.x), fma_r(-val.x, x, val.y)};
        }
      } else {
        if (g.valid) {
          const double fm = rc.f0 + static_cast<double>(m_tile0 + j) * rc.df;
          const double s = fm / kC0;  // turns per metre
          const C ph = phi_turns<R>(s * g.beta[0], s * g.beta[1], s * g.beta[2]);
          const R ar = static_cast<R>(g.amp_re), ai = static_cast<R>(g.amp_im);
          val = {ar * ph.x - ai * ph.y, ar * ph.y + ai * ph.x};
        }
      }
      tl.G[i * sh.M_t + j] = val;
      if constexpr (EchoLayout<R, MB, FT>::kRotated) {
        // (-j)^(j mod 4): block starts are multiples of 4 samples
        C v1;
        switch (j & 3) {
          case 0: v1 = val; break;
          case 1: v1 = {val.y, -val.x}; break;
          case 2: v1 = {-val.x, -val.y}; break;
          default: v1 = {-val.y, val.x}; break;
        }
        tl.G1[i * sh.M_t + j] = v1;
      }
    }
  }
}

// Accumulation of one staged tile of nf entries into a thread's MB samples. Per sample:
// one complex multiply-accumulate (4 FMA) and one phasor step. G is read from LDS in
// blocks of 8 samples, double-buffered in registers; the next facet's element phasors
// are prefetched.
template <typename R, int MB, int FT>
__device__ inline void sum_tile(const RadarConst &rc, const EchoShape &sh,
                                const EchoTile<R, MB, FT> &tl, int nf, int p, int q, int b,
                                typename Cx<R>::T (&acc)[MB]) {
  using C = typename Cx<R>::T;
  const int P = rc.P, E = sh.E;
  const int iu_p = b * FT * E + p, iu_q = b * FT * E + P + q;
  const int stride_u = E;
  C up = tl.U[iu_p], uq = tl.U[iu_q];
  C rp = tl.rat[iu_p], rq = tl.rat[iu_q];
  R op = tl.off[p], oq = tl.off[P + q];
  for (int i = 0; i < nf; ++i) {
    const R eps = op * oq;
    C z = {fma_r(up.x, uq.x, -up.y * uq.y), fma_r(up.x, uq.y, up.y * uq.x)};
    if constexpr (sizeof(R) == 8) {
      // exp(j eps) to fourth order (|eps| <= 1e-3 is enforced on the host)
      const R e2 = eps * eps;
      const C ce = {R(1) - e2 * (R(0.5) - e2 * R(1.0 / 24.0)), eps * (R(1) - e2 * R(1.0 / 6.0))};
      z = {z.x * ce.x - z.y * ce.y, z.x * ce.y + z.y * ce.x};
    } else {
      // exp(j eps) ~ 1 + j eps: the host keeps |eps| <= 3e-4, so eps^2 / 2 stays
      // below FP32 rounding
      z = {fma_r(-eps, z.y, z.x), fma_r(eps, z.x, z.y)};
    }
    const C r = {fma_r(rp.x, rq.x, -rp.y * rq.y), fma_r(rp.x, rq.y, rp.y * rq.x)};
    // FP32: advance the phasor with the three-term recurrence
    //   z_{m+1} = 2 cos(t) z_m - z_{m-1}   (2 FMA instead of a complex multiply),
    // whose error grows like 1/|sin t|. When |sin t| < |cos t| the ramp is rotated by a
    // quarter turn per sample (r -> j r, so |sin| >= 0.707) and the lane reads G
    // pre-rotated by (-j)^m instead, which undoes it exactly.
    bool quarter = false;
    C zn = z;
    R c2 = R(0);
    if constexpr (sizeof(R) == 4) {
      quarter = fabsf(r.y) < fabsf(r.x);
      const C rk = quarter ? C{-r.y, r.x} : r;
      c2 = R(2) * rk.x;
      zn = {fma_r(z.x, rk.x, -z.y * rk.y), fma_r(z.x, rk.y, z.y * rk.x)};
    }
    if (i + 1 < nf) {
      up = tl.U[(i + 1) * stride_u + iu_p];
      uq = tl.U[(i + 1) * stride_u + iu_q];
      rp = tl.rat[(i + 1) * stride_u + iu_p];
      rq = tl.rat[(i + 1) * stride_u + iu_q];
      op = tl.off[(i + 1) * E + p];
      oq = tl.off[(i + 1) * E + P + q];
    }
    const C *Gi = (quarter ? tl.G1 : tl.G) + i * sh.M_t + b * MB;
    constexpr int kBlk = (MB < 8) ? MB : 8;
    C ga[kBlk], gb[kBlk];
#pragma unroll
    for (int j = 0; j < kBlk; ++j) ga[j] = Gi[j];
#pragma unroll
    for (int j0 = 0; j0 < MB; j0 += kBlk) {
      if (j0 + kBlk < MB) {
#pragma unroll
        for (int j = 0; j < kBlk; ++j) gb[j] = Gi[j0 + kBlk + j];
      }
#pragma unroll
      for (int j = 0; j < kBlk; ++j) {
        const C g = ga[j];
        C &a = acc[j0 + j];
        a.x = fma_r(g.x, z.x, a.x);
        a.x = fma_r(-g.y, z.y, a.x);
        a.y = fma_r(g.x, z.y, a.y);
        a.y = fma_r(g.y, z.x, a.y);
        if constexpr (sizeof(R) == 4) {
          const C zz = {fma_r(c2, zn.x, -z.x), fma_r(c2, zn.y, -z.y)};
          z = zn;
          zn = zz;
        } else {
          const R zx = fma_r(z.x, r.x, -z.y * r.y);
          z.y = fma_r(z.x, r.y, z.y * r.x);
          z.x = zx;
        }
      }
#pragma unroll
      for (int j = 0; j < kBlk; ++j) ga[j] = gb[j];
    }
  }
}

// One work item. The staging waves and the accumulating waves run separate branches
// (whole waves each, so the accumulators are not live in the staging code); both pass
// the same sequence of workgroup barriers: one per tile, then two per output chunk.
// The tile count depends only on the chirp's lit count.
// Output of one work item in chunks of kOut samples: the accumulating threads park kOut
// values each in LDS, then consecutive lanes write consecutive samples of one channel
// row, so a wave writes whole 128-byte runs instead of one 8-byte value per row.
template <typename R, int MB>
__device__ inline void store_chunk(const RadarConst &rc, const EchoShape &sh,
                                   const typename Cx<R>::T *stage, typename Cx<R>::T *echo_out,
                                   int n, int ot, int m0) {
  using C = typename Cx<R>::T;
  constexpr int kOut = (MB < 16) ? MB : 16;
  for (int e = threadIdx.x; e < sh.O_w * kOut; e += blockDim.x) {
    const int oo = ot * sh.O_w + e / kOut;
    const int m = m0 + e % kOut;
    if (oo < sh.O && m < rc.M) {
      C *dst = echo_out + (static_cast<int64_t>(oo) * rc.N + n) * rc.M + m;
      if (!sh.accumulate) {
        *dst = stage[e];
      } else {
        // a further path type of the same echo: dst += gamma x value
        const C v = stage[e], d = *dst;
        const R gr = static_cast<R>(sh.gamma_re), gi = static_cast<R>(sh.gamma_im);
        *dst = {d.x + (gr * v.x - gi * v.y), d.y + (gr * v.y + gi * v.x)};
      }
    }
  }
}

// One work item (chirp n, sample tile mt, channel tile ot), split in its two roles. The
// staging waves and the accumulating waves pass the same barriers: one per tile, then
// two per output chunk.
template <typename R, int MB, int FT>
__device__ void echo_stage_item(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                                EchoSmem<R, MB, FT> &sm, int n, int mt, int ot, int st) {
  using C = typename Cx<R>::T;
  constexpr int kOut = (MB < 16) ? MB : 16;
  const int m_tile0 = mt * sh.M_t;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t total = cnt + sc.n_points;
  const int32_t n_tiles = (total + FT - 1) / FT;
  const C *stage = sm.tile(0).G;  // output staging: the layout reserves O_w x kOut values here
  C *echo_out = static_cast<C *>(sc.echo);
  if (n_tiles > 0)
    stage_tile<R, MB, FT>(sc, rc, sh, sm, sm.tile(0), n, cnt, 0, min(FT, total), m_tile0, st);
  for (int32_t k = 0; k < n_tiles; ++k) {
    // tile k is staged in buffer k & 1; buffer (k + 1) & 1 was consumed in step k - 1
    __syncthreads();
    const int32_t t1 = (k + 1) * FT;
    if (t1 < total)
      stage_tile<R, MB, FT>(sc, rc, sh, sm, sm.tile((k & 1) ^ 1), n, cnt, t1,
                            min(FT, total - t1), m_tile0, st);
  }
  for (int bb = 0; bb < sh.B_w; ++bb) {
    for (int jc = 0; jc < MB; jc += kOut) {
      __syncthreads();
      __syncthreads();
      store_chunk<R, MB>(rc, sh, stage, echo_out, n, ot, m_tile0 + bb * MB + jc);
    }
  }
}

template <typename R, int MB, int FT>
__device__ void echo_compute_item(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                                  EchoSmem<R, MB, FT> &sm, int n, int mt, int ot) {
  using C = typename Cx<R>::T;
  constexpr int kOut = (MB < 16) ? MB : 16;
  const int tid = threadIdx.x;
  const int m_tile0 = mt * sh.M_t;
  const int32_t total = sc.vis_cnt[n] + sc.n_points;
  const int32_t n_tiles = (total + FT - 1) / FT;
  C *stage = sm.tile(0).G;
  C *echo_out = static_cast<C *>(sc.echo);
  const int Q = rc.Q;
  const int ol = tid % sh.O_w;
  const int b = tid / sh.O_w;
  const int o = ot * sh.O_w + ol;
  const bool o_ok = b < sh.B_w && o < sh.O;
  const int p = o_ok ? o / Q : 0;
  const int q = o_ok ? o % Q : 0;
  C acc[MB];
#pragma unroll
  for (int j = 0; j < MB; ++j) acc[j] = {R(0), R(0)};
  for (int32_t k = 0; k < n_tiles; ++k) {
    __syncthreads();
    if (o_ok) sum_tile<R, MB, FT>(rc, sh, sm.tile(k & 1), min(FT, total - k * FT), p, q, b, acc);
  }
  for (int bb = 0; bb < sh.B_w; ++bb) {
#pragma unroll
    for (int jc = 0; jc < MB; jc += kOut) {
      __syncthreads();
      if (b == bb) {
#pragma unroll
        for (int j = 0; j < kOut; ++j) stage[ol * kOut + j] = acc[jc + j];
      }
      __syncthreads();
      store_chunk<R, MB>(rc, sh, stage, echo_out, n, ot, m_tile0 + bb * MB + jc);
    }
  }
}

template <typename R, int MB, int FT>
__global__ void __launch_bounds__(512) echo_kernel(DevScene sc, RadarConst rc, const double *elem,
                                                   EchoShape sh) {
  extern __shared__ __align__(16) unsigned char echo_smem[];
  EchoSmem<R, MB, FT> sm;
  sm.carve(echo_smem, sh);
  for (int i = threadIdx.x; i < 3 * sh.E; i += blockDim.x) sm.elem[i] = elem[i];
  __syncthreads();
  const int per_chirp = sh.m_tiles * sh.o_tiles;
  const int n = blockIdx.x / per_chirp;
  const int r = blockIdx.x % per_chirp;
  if (threadIdx.x >= sh.n_compute)
    echo_stage_item<R, MB, FT>(sc, rc, sh, sm, n, r / sh.o_tiles, r % sh.o_tiles,
                               threadIdx.x - sh.n_compute);
  else
    echo_compute_item<R, MB, FT>(sc, rc, sh, sm, n, r / sh.o_tiles, r % sh.o_tiles);
}

// Persistent form: a grid sized to the machine drains a queue of work items
// (scene, chirp, sample tile, channel tile), ordered longest-first by the host.
template <typename R, int MB, int FT>
__global__ void __launch_bounds__(512) echo_persistent_kernel(const DevScene *scenes,
                                                              const int4 *items, int32_t n_items,
                                                              int32_t *queue, RadarConst rc,
                                                              const double *elem, EchoShape sh) {
  extern __shared__ __align__(16) unsigned char echo_smem[];
  __shared__ int32_t s_item;
  EchoSmem<R, MB, FT> sm;
  sm.carve(echo_smem, sh);
  for (int i = threadIdx.x; i < 3 * sh.E; i += blockDim.x) sm.elem[i] = elem[i];
  // each role runs its own loop (so that neither holds the other's values); both pass the
  // same barriers per item
  if (threadIdx.x >= sh.n_compute) {
    const int st = threadIdx.x - sh.n_compute;
    while (true) {
      __syncthreads();
      if (st == 0) s_item = atomicAdd(queue, 1);
      __syncthreads();
      const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
      if (it >= n_items) break;  // every workgroup reaches this once the queue is drained
      const int4 w = items[it];
      echo_stage_item<R, MB, FT>(scenes[w.x], rc, sh, sm, w.y, w.z, w.w, st);
    }
  } else {
    while (true) {
      __syncthreads();
      __syncthreads();
      const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
      if (it >= n_items) break;
      const int4 w = items[it];
      echo_compute_item<R, MB, FT>(scenes[w.x], rc, sh, sm, w.y, w.z, w.w);
    }
  }
}

__global__ void reset_counter_kernel(int32_t *q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

template <typename R, int MB, int FT>
static size_t smem_bytes(const EchoShape &sh) {
  return EchoLayout<R, MB, FT>(sh).total;
}

// Host-side dispatch over the compiled (precision, MB, FT) variants.
struct EchoLaunch {
  int precision;  // 0 fp32, 1 fp64
  int mb, ft;
};

template <typename R, int MB, int FT>
static hipError_t launch_plain_t(const DevScene &sc, const RadarConst &rc, const double *elem,
                                 const EchoShape &sh, hipStream_t s) {
  const size_t lds = smem_bytes<R, MB, FT>(sh);
  const int threads = sh.n_compute + kStagingThreads;
  const unsigned grid = static_cast<unsigned>(rc.N) * sh.m_tiles * sh.o_tiles;
  hipLaunchKernelGGL((echo_kernel<R, MB, FT>), dim3(grid), dim3(threads), lds, s, sc, rc, elem, sh);
  return hipGetLastError();
}

template <typename R, int MB, int FT>
static hipError_t launch_persistent_t(const DevScene *scenes, const int4 *items, int32_t n_items,
                                      int32_t *queue, const RadarConst &rc, const double *elem,
                                      const EchoShape &sh, int n_groups, hipStream_t s) {
  const size_t lds = smem_bytes<R, MB, FT>(sh);
  const int threads = sh.n_compute + kStagingThreads;
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, s, queue);
  hipLaunchKernelGGL((echo_persistent_kernel<R, MB, FT>), dim3(n_groups), dim3(threads), lds, s,
                     scenes, items, n_items, queue, rc, elem, sh);
  return hipGetLastError();
}

template <typename R, int MB, int FT>
static hipError_t occupancy_t(const EchoShape &sh, int *groups_per_cu) {
  const size_t lds = smem_bytes<R, MB, FT>(sh);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(
      groups_per_cu, reinterpret_cast<const void *>(echo_persistent_kernel<R, MB, FT>),
      sh.n_compute + kStagingThreads, lds);
}

#define RSIM_ECHO_VARIANTS(X) \
  X(float, 16, 16)            \
  X(float, 32, 8)             \
  X(float, 32, 16)            \
  X(float, 64, 8)             \
  X(float, 64, 16)            \
  X(double, 8, 8)             \
  X(double, 16, 8)

#define RSIM_PREC_OF(R) (sizeof(R) == 8 ? 1 : 0)

hipError_t launch_echo_plain(int precision, int mb, int ft, const DevScene &sc, const RadarConst &rc,
                             const double *elem, const EchoShape &sh, hipStream_t s) {
#define X(R, MB, FT)                                              \
  if (precision == RSIM_PREC_OF(R) && mb == MB && ft == FT)       \
    return launch_plain_t<R, MB, FT>(sc, rc, elem, sh, s);
  RSIM_ECHO_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_echo_persistent(int precision, int mb, int ft, const DevScene *scenes,
                                  const int4 *items, int32_t n_items, int32_t *queue,
                                  const RadarConst &rc, const double *elem, const EchoShape &sh,
                                  int n_groups, hipStream_t s) {
#define X(R, MB, FT)                                                                    \
  if (precision == RSIM_PREC_OF(R) && mb == MB && ft == FT)                             \
    return launch_persistent_t<R, MB, FT>(scenes, items, n_items, queue, rc, elem, sh, \
                                          n_groups, s);
  RSIM_ECHO_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t echo_occupancy(int precision, int mb, int ft, const EchoShape &sh, int *groups_per_cu) {
#define X(R, MB, FT)                                        \
  if (precision == RSIM_PREC_OF(R) && mb == MB && ft == FT) \
    return occupancy_t<R, MB, FT>(sh, groups_per_cu);
  RSIM_ECHO_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

bool echo_variant_exists(int precision, int mb, int ft) {
#define X(R, MB, FT) \
  if (precision == RSIM_PREC_OF(R) && mb == MB && ft == FT) return true;
  RSIM_ECHO_VARIANTS(X)
#undef X
  return false;
}

size_t echo_smem_bytes(int precision, int mb, int ft, const EchoShape &sh) {
#define X(R, MB, FT) \
  if (precision == RSIM_PREC_OF(R) && mb == MB && ft == FT) return smem_bytes<R, MB, FT>(sh);
  RSIM_ECHO_VARIANTS(X)
#undef X
  return 0;
}

}  // namespace rsim
