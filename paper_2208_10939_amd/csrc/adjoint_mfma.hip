// Adjoint of the facet sum on the matrix cores (FP32): the separable Tx x Rx form of the
// forward sum (Sections 2.2 and 3.2; eqs. (7), (9)-(13)), differentiated as in the
// vector-unit adjoint, with the Tx-Rx cross term dropped (the host takes this kernel only
// where its bound is below 1e-5 rad).
//
// With conj(g)[p, q, m] the conjugated loss gradient of channel (p, q), A_p(m) and B_q(m)
// the Tx and Rx element phasors (1/R included) of a facet and G, D_k its facet integral
// and node derivatives, the forward term of channel (p, q) is y_pq = G conj(g_pq) A_p B_q
// (w_pq = conj(g_pq) A_p B_q). Everything the chain rule needs is a sum over channels of
// per-channel sums, and those reduce to two contractions per sample:
//   X_p = sum_q conj(g)[p, q] B_q  (y_p = G A_p X_p = sum_q y_pq),
//   Y_q = sum_p conj(g)[p, q] A_p  (y'_q = G B_q Y_q = sum_p y_pq),
//   W   = sum_p A_p X_p = sum_pq w_pq.
// Per sample m (absolute index), per facet:
//   grad_c -= sum_p e_p [(K_p + k0 df m) Im y_p - Re y_p / R_p]
//           + sum_q e_q [(K_q + k0 df m) Im y'_q - Re y'_q / R_q],
//   sum Re y += Re(G W),  t_k += Re(D_k W),
// with e the unit vector centroid -> element, k0 = 2 pi / c and K_e = k0 (f0 - slope
// (tau_e + tau_ref of the other side)): the per-channel delay sum tau_p + tau_q of the
// vector-unit adjoint taken with the other side at its reference delay (a relative change
// of slope |tau_q - tau_ref| / f0 ~ 1e-7).
//
// Layout: a workgroup covers one chirp and 64 samples: eight accumulating waves (wave w:
// samples 8w .. 8w+7, two per SIMD) and four staging waves; conj(g) of the tile sits in
// LDS for the whole item. Tiles of eight lit facets, double-buffered. Per tile, MFMA block
// b = (sample s = b mod 8, facet group b / 8) of a wave: lane (b, l) takes facet
// 4 (b / 8) + l at sample s. Its 4 PT Tx and 4 QT Rx phasors are the MFMA B operands,
// conj(g) rows (X) or columns (Y) the A operands read from LDS, so that after the K loop
// lane (b, l) holds X_p (or Y_q) of its facet at its sample.
#include "adjoint_common.h"

namespace rsim {

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kAmWaves = 8;                 // accumulating waves, 8 samples each
constexpr int kAmBlk = 8;                   // samples per wave
constexpr int kAmTile = kAmWaves * kAmBlk;  // samples per workgroup
constexpr int kAmFT = 8;                    // facets per tile: two groups of four columns
constexpr int kAmStaging = 4;               // staging waves, two facets each
constexpr int kAmThreads = (kAmWaves + kAmStaging) * 64;
constexpr double kAmMid = 31.5;             // tile centre, where staged phases are taken

// LDS: elem | conj(g) [w][4PT][row] (row = 8 (4QT) + 8 float2: each p row starts 16 banks
// after the previous one, so the four rows or columns a read touches fall in distinct
// banks) | red [2][FT][waves][kAdjVals] | two tile buffers.
template <int PT, int QT>
struct AmLayout {
  static constexpr int kRow = kAmBlk * 4 * QT + 8;  // float2 per p row
  static constexpr int kSlots = 4 * (PT + QT);
  size_t elem, gc, red, buf[2], geo, glin, EP, EC, KC, GD, total;
  __host__ __device__ explicit AmLayout(int E) {
    auto up = [](size_t b) { return (b + 15) & ~size_t(15); };
    size_t b = 0;
    elem = b;
    b = up(b + sizeof(double) * 3 * E);
    gc = b;
    b = up(b + sizeof(float2) * kAmWaves * 4 * PT * kRow);
    red = b;
    b = up(b + sizeof(float) * 2 * kAmFT * kAmWaves * kAdjVals);
    size_t t = 0;
    geo = t;
    t = up(t + sizeof(Geo) * kAmFT);
    glin = t;
    t = up(t + sizeof(GLin) * kAmFT);
    EP = t;  // [FT][slots] float2: phase at the tile centre, step (turns)
    t = up(t + sizeof(float2) * kAmFT * kSlots);
    EC = t;  // [FT][slots] float4: unit vector centroid -> element, 1 / R
    t = up(t + sizeof(float4) * kAmFT * kSlots);
    KC = t;  // [FT][slots] float: k0 (f0 - slope (tau_e + tau_ref,other))
    t = up(t + sizeof(float) * kAmFT * kSlots);
    GD = t;  // [FT][kAmTile][2] float4: (G, D0), (D1, D2)
    t = up(t + sizeof(float4) * kAmFT * kAmTile * 2);
    buf[0] = b;
    buf[1] = b + t;
    total = b + 2 * t;
  }
};

template <int PT, int QT>
struct AmSmem {
  double *elem;
  float2 *gc;
  float *red;
  unsigned char *buf0;
  size_t stride, ogeo, oglin, oEP, oEC, oKC, oGD;
  __device__ void carve(unsigned char *base, int E) {
    const AmLayout<PT, QT> L(E);
    elem = reinterpret_cast<double *>(base + L.elem);
    gc = reinterpret_cast<float2 *>(base + L.gc);
    red = reinterpret_cast<float *>(base + L.red);
    buf0 = base + L.buf[0];
    stride = L.buf[1] - L.buf[0];
    ogeo = L.geo;
    oglin = L.glin;
    oEP = L.EP;
    oEC = L.EC;
    oKC = L.KC;
    oGD = L.GD;
  }
  __device__ unsigned char *b(int k) const { return buf0 + static_cast<size_t>(k) * stride; }
  __device__ Geo *geo(int k) const { return reinterpret_cast<Geo *>(b(k) + ogeo); }
  __device__ GLin *glin(int k) const { return reinterpret_cast<GLin *>(b(k) + oglin); }
  __device__ float2 *EP(int k) const { return reinterpret_cast<float2 *>(b(k) + oEP); }
  __device__ float4 *EC(int k) const { return reinterpret_cast<float4 *>(b(k) + oEC); }
  __device__ float *KC(int k) const { return reinterpret_cast<float *>(b(k) + oKC); }
  __device__ float4 *GD(int k) const { return reinterpret_cast<float4 *>(b(k) + oGD); }
  __device__ float *red_buf(int k) const { return red + static_cast<size_t>(k) * kAmFT * kAmWaves * kAdjVals; }
};

__device__ inline float am_centred(double t) { return static_cast<float>(t - rint(t)); }

// Staging of tile entries t0 .. t0 + nf - 1 of chirp n into buffer k: staging wave sw
// takes facets 2 sw and 2 sw + 1 through geometry, element data and G, D_k. Padding slots
// (and absent facets) get zeros, so that every phasor built from them is zero.
template <int PT, int QT>
__device__ void am_stage(const DevScene &sc, const RadarConst &rc, const AmSmem<PT, QT> &sm, int k,
                         int n, int32_t cnt, int32_t t0, int nf, int m_tile0, int st) {
  constexpr int kSlots = 4 * (PT + QT);
  constexpr int kPer = kAmFT / kAmStaging;  // facets per staging wave
  static_assert(kPer * kSlots <= 64, "one pass over a wave's element slots");
  const int lane = st & 63, i0 = (st >> 6) * kPer;
  const int P = rc.P, Q = rc.Q;
  Geo *geo = sm.geo(k);
  GLin *glin = sm.glin(k);
  if (lane < kPer) {
    const int i = i0 + lane;
    if (i < nf)
      entry_geometry(sc, rc, n, cnt, t0 + i, geo[i]);
    else
      geo[i].valid = 0;
    make_glin(geo[i], rc, m_tile0, glin[i]);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
  float2 *EP = sm.EP(k);
  float4 *EC = sm.EC(k);
  float *KC = sm.KC(k);
  const double slope = rc.slope;
  const double k0 = 2.0 * kPi / kC0;
  if (lane < kPer * kSlots) {
    const int i = i0 + lane / kSlots, slot = lane % kSlots;
    const Geo g = lds_copy(geo[i]);
    const bool tx = slot < 4 * PT;
    const int e = tx ? slot : P + (slot - 4 * PT);  // element of the slot
    const bool real = tx ? (slot < P) : (slot - 4 * PT < Q);
    if (!g.valid || !real) {
      EP[i * kSlots + slot] = make_float2(0.0f, 0.0f);
      EC[i * kSlots + slot] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      KC[i * kSlots + slot] = 0.0f;
    } else {
      const double dx = sm.elem[3 * e + 0] - g.c[0];
      const double dy = sm.elem[3 * e + 1] - g.c[1];
      const double dz = sm.elem[3 * e + 2] - g.c[2];
      const double Rn = sqrt(dx * dx + dy * dy + dz * dz);
      const double inv = 1.0 / Rn;
      const double tau = Rn * (1.0 / kC0);
      const double t_self = tx ? g.tref_t : g.tref_r, t_other = tx ? g.tref_r : g.tref_t;
      double psi0 = rc.f0 * tau - 0.5 * slope * tau * tau - slope * t_other * (tau - t_self) -
                    0.5 * slope * g.tref_t * g.tref_r;
      psi0 -= floor(psi0);
      double delta = rc.df * tau;
      delta -= floor(delta);
      const double mc = static_cast<double>(m_tile0) + kAmMid;
      EP[i * kSlots + slot] = make_float2(am_centred(psi0 + mc * delta), am_centred(delta));
      EC[i * kSlots + slot] = make_float4(static_cast<float>(dx * inv), static_cast<float>(dy * inv),
                                          static_cast<float>(dz * inv), static_cast<float>(inv));
      KC[i * kSlots + slot] = static_cast<float>(k0 * (rc.f0 - slope * (tau + t_other)));
    }
  }
  float4 *GD = sm.GD(k);
  for (int t = lane; t < kPer * kAmTile; t += 64) {
    const int i = i0 + t / kAmTile, j = t % kAmTile;
    const GLin q = lds_copy(glin[i]);
    float2 gv, dv[3];
    g_lin_grad(q, j, gv, dv);
    GD[(i * kAmTile + j) * 2 + 0] = make_float4(gv.x, gv.y, dv[0].x, dv[0].y);
    GD[(i * kAmTile + j) * 2 + 1] = make_float4(dv[1].x, dv[1].y, dv[2].x, dv[2].y);
  }
}

// Sum of a finished tile's per-wave sums (fixed wave order) into the per-(chirp, facet,
// sample tile) partials, by the staging waves.
__device__ inline void am_flush(const float *red, float *partial, int64_t F, int m_tiles, int n,
                                int mt, int32_t t0, int nf, int st) {
  for (int task = st; task < nf * 7; task += kAmStaging * 64) {
    const int i = task / 7, k = task % 7;
    float s = 0.0f;
    for (int wv = 0; wv < kAmWaves; ++wv) s += red[(i * kAmWaves + wv) * kAdjVals + k];
    const int64_t slot = (static_cast<int64_t>(n) * F + t0 + i) * m_tiles + mt;
    partial[slot * kAdjVals + k] = s;
  }
}

// exp(-j 2 pi (phi_c + s step)) / R at s samples from the tile centre (|s| <= 31.5: FP32
// rounding of the phase <= 1e-6 turns, well inside the adjoint's tolerance)
__device__ inline float2 am_phasor(float2 ep, float s, float ir) {
  const float t = fmaf(s, ep.y, ep.x);
  return make_float2(__builtin_amdgcn_cosf(t) * ir, -__builtin_amdgcn_sinf(t) * ir);
}

// Sum over the 8 lanes 4 (s + 8 fg) + l (s = 0..7) that share the facet (fg, l); every
// lane gets its group's sum.
// (ds_swizzle in bit-mask mode, lane ^ m within 32-lane halves: no address registers)
template <int kXor>
__device__ inline float swz_xor(float v) {
  constexpr int kPattern = 0x1F | (kXor << 10);  // and 0x1F, or 0, xor kXor
  return __builtin_bit_cast(float,
                            __builtin_amdgcn_ds_swizzle(__builtin_bit_cast(int, v), kPattern));
}

__device__ inline float sum_over_samples(float v) {
  v += swz_xor<4>(v);
  v += swz_xor<8>(v);
  v += swz_xor<16>(v);
  return v;
}

template <int PT, int QT>
__global__ void __launch_bounds__(kAmThreads) adjoint_mfma_kernel(DevScene sc, RadarConst rc,
                                                                  const double *elem, AdjShape ash,
                                                                  const float2 *grad_echo,
                                                                  float *partial) {
  using L = AmLayout<PT, QT>;
  constexpr int kSlots = L::kSlots;
  constexpr int kRow = L::kRow;
  extern __shared__ __align__(16) unsigned char am_smem[];
  const EchoShape &sh = ash.sh;
  AmSmem<PT, QT> sm;
  sm.carve(am_smem, sh.E);
  const int tid = threadIdx.x;
  const int n = blockIdx.x / sh.m_tiles, mt = blockIdx.x % sh.m_tiles;
  const int m_tile0 = mt * kAmTile;
  const int P = rc.P, Q = rc.Q, M = rc.M, N = rc.N;
  for (int i = tid; i < 3 * sh.E; i += blockDim.x) sm.elem[i] = elem[i];
  // conj(g) of this chirp and sample tile: [w][p][q][s] (padding rows, columns and samples
  // beyond M are zero)
  for (int idx = tid; idx < kAmWaves * 4 * PT * kRow; idx += blockDim.x) {
    const int w = idx / (4 * PT * kRow), rem = idx % (4 * PT * kRow);
    const int p = rem / kRow, c = rem % kRow;
    const int q = c / kAmBlk, s = c % kAmBlk;
    const int m = m_tile0 + w * kAmBlk + s;
    float2 v = make_float2(0.0f, 0.0f);
    if (p < P && q < Q && c < kAmBlk * 4 * QT && m < M) {
      const float2 gv = grad_echo[(static_cast<int64_t>(p * Q + q) * N + n) * M + m];
      v = make_float2(gv.x, -gv.y);
    }
    sm.gc[idx] = v;
  }
  __syncthreads();
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t n_tiles = (cnt + kAmFT - 1) / kAmFT;
  constexpr int nc = kAmWaves * 64;

  if (tid >= nc) {
    const int st = tid - nc;
    if (n_tiles > 0) am_stage<PT, QT>(sc, rc, sm, 0, n, cnt, 0, min(kAmFT, cnt), m_tile0, st);
    for (int32_t k = 0; k < n_tiles; ++k) {
      __syncthreads();
      if (k > 0)
        am_flush(sm.red_buf((k - 1) & 1), partial, ash.F, sh.m_tiles, n, mt, (k - 1) * kAmFT,
                 min(kAmFT, cnt - (k - 1) * kAmFT), st);
      const int32_t t1 = (k + 1) * kAmFT;
      if (t1 < cnt)
        am_stage<PT, QT>(sc, rc, sm, (k & 1) ^ 1, n, cnt, t1, min(kAmFT, cnt - t1), m_tile0, st);
    }
    __syncthreads();
    if (n_tiles > 0)
      am_flush(sm.red_buf((n_tiles - 1) & 1), partial, ash.F, sh.m_tiles, n, mt,
               (n_tiles - 1) * kAmFT, min(kAmFT, cnt - (n_tiles - 1) * kAmFT), st);
    return;
  }

  const float kdf = static_cast<float>(2.0 * kPi / kC0 * rc.df);
  for (int32_t kt = 0; kt < n_tiles; ++kt) {
    __syncthreads();
    // The lane's indices and addresses are formed here, per tile, from a thread id passed
    // through an empty asm: hoisted out of the loop they would be held (and spilled)
    // across it at three waves per SIMD.
    int lt = tid;
    asm volatile("" : "+v"(lt));
    const int w = lt >> 6, lane = lt & 63;
    const int blk = lane >> 2, l = lane & 3;  // MFMA block; row / column within it
    const int s = blk % kAmBlk, fi = 4 * (blk / kAmBlk) + l;  // sample in the wave; facet
    const int mw = w * kAmBlk + s;                            // sample in the tile
    const float sf = static_cast<float>(mw) - static_cast<float>(kAmMid);
    const float mabs = static_cast<float>(m_tile0 + mw);
    const float2 *gcw = sm.gc + static_cast<size_t>(w) * 4 * PT * kRow;
    const int buf = kt & 1;
    const float2 *EP = sm.EP(buf) + fi * kSlots;
    const float4 *EC = sm.EC(buf) + fi * kSlots;
    const float *KC = sm.KC(buf) + fi * kSlots;
    // phasors of this lane's facet at its sample: Tx slots 0 .. 4PT-1, Rx slots after
    // Phases in this order (scheduling barriers between them, and every four elements
    // inside, bound what the compiler keeps live at three waves per SIMD): Rx phasors, the
    // X contraction, Tx phasors, the Tx-side sums, the Y contraction, the Rx-side sums.
    float ar[4 * PT], ai[4 * PT], br[4 * QT], bi[4 * QT];
#pragma unroll
    for (int q = 0; q < 4 * QT; ++q) {
      const float2 t = am_phasor(EP[4 * PT + q], sf, EC[4 * PT + q].w);
      br[q] = t.x;
      bi[q] = t.y;
      if (q % 4 == 3) __builtin_amdgcn_sched_barrier(0);
    }
    const float kmf = kdf * mabs;
    float v[7] = {0, 0, 0, 0, 0, 0, 0};
    float wr = 0.0f, wi = 0.0f;
    float4 g0, g1;  // (G, D0), (D1, D2) of this facet and sample
    {
      // X_p = sum_q conj(g)[p, q] B_q: A operand conj(g)[4a + l, q] (row l of block b, at
      // the block's sample); lane (b, l) register r of tile a then holds X[4a + r] of its facet
      v4f xr[PT], xi[PT];
#pragma unroll
      for (int a = 0; a < PT; ++a) {
        xr[a] = v4f{0.f, 0.f, 0.f, 0.f};
        xi[a] = v4f{0.f, 0.f, 0.f, 0.f};
      }
      // conj(g) operands one step ahead of the MFMAs that use them (LDS latency)
      float2 gn[PT];
#pragma unroll
      for (int a = 0; a < PT; ++a) gn[a] = gcw[(4 * a + l) * kRow + s];
#pragma unroll
      for (int q = 0; q < 4 * QT; ++q) {
        const float nb = -bi[q];
        float2 g[PT];
#pragma unroll
        for (int a = 0; a < PT; ++a) {
          g[a] = gn[a];
          if (q + 1 < 4 * QT) gn[a] = gcw[(4 * a + l) * kRow + (q + 1) * kAmBlk + s];
        }
        // four passes over the tiles, so that no MFMA waits on the one just before it
#pragma unroll
        for (int a = 0; a < PT; ++a)
          xr[a] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[a].x, br[q], xr[a], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < PT; ++a)
          xi[a] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[a].x, bi[q], xi[a], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < PT; ++a)
          xi[a] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[a].y, br[q], xi[a], 0, 0, 0);
#pragma unroll
        for (int a = 0; a < PT; ++a)
          xr[a] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[a].y, nb, xr[a], 0, 0, 0);
        // bounds how far ahead the operand reads are hoisted (register pressure)
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int p = 0; p < 4 * PT; ++p) {
        const float2 t = am_phasor(EP[p], sf, EC[p].w);
        ar[p] = t.x;
        ai[p] = t.y;
        if (p % 4 == 3) __builtin_amdgcn_sched_barrier(0);
      }
      const float4 *gd = sm.GD(buf) + (fi * kAmTile + mw) * 2;
      g0 = gd[0];
      g1 = gd[1];
#pragma unroll
      for (int a = 0; a < PT; ++a)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int p = 4 * a + r;
          // A_p X_p, then y_p = G A_p X_p
          const float tr = ar[p] * xr[a][r] - ai[p] * xi[a][r];
          const float ti = ar[p] * xi[a][r] + ai[p] * xr[a][r];
          wr += tr;
          wi += ti;
          const float yre = g0.x * tr - g0.y * ti, yim = g0.x * ti + g0.y * tr;
          const float4 e = EC[p];
          const float c = fmaf(KC[p] + kmf, yim, -yre * e.w);
          v[0] = fmaf(-c, e.x, v[0]);
          v[1] = fmaf(-c, e.y, v[1]);
          v[2] = fmaf(-c, e.z, v[2]);
          if (r == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }
    {
      // Y_q = sum_p conj(g)[p, q] A_p: A operand conj(g)[p, 4b + l] (row l of the block)
      v4f yr[QT], yi[QT];
#pragma unroll
      for (int b = 0; b < QT; ++b) {
        yr[b] = v4f{0.f, 0.f, 0.f, 0.f};
        yi[b] = v4f{0.f, 0.f, 0.f, 0.f};
      }
      float2 gn[QT];
#pragma unroll
      for (int b = 0; b < QT; ++b) gn[b] = gcw[(4 * b + l) * kAmBlk + s];
#pragma unroll
      for (int p = 0; p < 4 * PT; ++p) {
        const float na = -ai[p];
        float2 g[QT];
#pragma unroll
        for (int b = 0; b < QT; ++b) {
          g[b] = gn[b];
          if (p + 1 < 4 * PT) gn[b] = gcw[(p + 1) * kRow + (4 * b + l) * kAmBlk + s];
        }
#pragma unroll
        for (int b = 0; b < QT; ++b)
          yr[b] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[b].x, ar[p], yr[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < QT; ++b)
          yi[b] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[b].x, ai[p], yi[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < QT; ++b)
          yi[b] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[b].y, ar[p], yi[b], 0, 0, 0);
#pragma unroll
        for (int b = 0; b < QT; ++b)
          yr[b] = __builtin_amdgcn_mfma_f32_4x4x1f32(g[b].y, na, yr[b], 0, 0, 0);
        __builtin_amdgcn_sched_barrier(0);
      }
#pragma unroll
      for (int b = 0; b < QT; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int q = 4 * b + r;
          const float tr = br[q] * yr[b][r] - bi[q] * yi[b][r];
          const float ti = br[q] * yi[b][r] + bi[q] * yr[b][r];
          const float yre = g0.x * tr - g0.y * ti, yim = g0.x * ti + g0.y * tr;
          const float4 e = EC[4 * PT + q];
          const float c = fmaf(KC[4 * PT + q] + kmf, yim, -yre * e.w);
          v[0] = fmaf(-c, e.x, v[0]);
          v[1] = fmaf(-c, e.y, v[1]);
          v[2] = fmaf(-c, e.z, v[2]);
          if (r == 3) __builtin_amdgcn_sched_barrier(0);
        }
    }
    v[3] = g0.x * wr - g0.y * wi;  // Re(G W)
    v[4] = g0.z * wr - g0.w * wi;  // Re(D_k W)
    v[5] = g1.x * wr - g1.y * wi;
    v[6] = g1.z * wr - g1.w * wi;
    // sums over the wave's 8 samples (every lane takes part); the lanes of sample 0 record them
    float *red = sm.red_buf(buf);
#pragma unroll
    for (int k = 0; k < 7; ++k) {
      const float tot = sum_over_samples(v[k]);
      if (s == 0) red[(fi * kAmWaves + w) * kAdjVals + k] = tot;
    }
  }
  __syncthreads();
}

}  // namespace

#define RSIM_AM_VARIANTS(X) \
  X(1, 1)                   \
  X(1, 4)                   \
  X(2, 2)                   \
  X(3, 4)

int adjoint_mfma_tile_m() { return kAmTile; }

size_t adjoint_mfma_smem_bytes(int P, int Q, int E) {
  int pt = 0, qt = 0;
  if (!mfma_variant(P, Q, &pt, &qt)) return 0;
#define X(PT, QT) \
  if (pt == PT && qt == QT) return AmLayout<PT, QT>(E).total;
  RSIM_AM_VARIANTS(X)
#undef X
  return 0;
}

hipError_t launch_adjoint_mfma(const DevScene &sc, const RadarConst &rc, const double *elem,
                               const EchoShape &sh, const void *grad_echo, float *partial,
                               float *gxw, hipStream_t s) {
  int pt = 0, qt = 0;
  if (!mfma_variant(rc.P, rc.Q, &pt, &qt) || sh.o_tiles != 1 ||
      sh.m_tiles != (rc.M + kAmTile - 1) / kAmTile)
    return hipErrorInvalidValue;
  AdjShape ash{sh, static_cast<int32_t>(sc.n_facets), 0};
  const hipError_t e =
      sh.accumulate ? hipSuccess : launch_fill_zero(gxw, static_cast<int64_t>(rc.N) * sc.n_facets * 9, s);
  if (e != hipSuccess || sc.n_facets == 0) return e;
  const unsigned grid = static_cast<unsigned>(rc.N) * sh.m_tiles;
  const size_t lds = adjoint_mfma_smem_bytes(rc.P, rc.Q, sh.E);
#define X(PT, QT)                                                                         \
  if (pt == PT && qt == QT)                                                               \
    hipLaunchKernelGGL((adjoint_mfma_kernel<PT, QT>), dim3(grid), dim3(kAmThreads), lds, s, \
                       sc, rc, elem, ash, static_cast<const float2 *>(grad_echo), partial);
  RSIM_AM_VARIANTS(X)
#undef X
  const hipError_t e2 = hipGetLastError();
  if (e2 != hipSuccess) return e2;
  return launch_adjoint_finish(sc, rc, sh, partial, gxw, s);
}

}  // namespace rsim
