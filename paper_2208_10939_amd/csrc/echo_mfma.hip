// Facet sum on the matrix cores (FP32): the separable Tx x Rx form of the coherent sum
// of Sections 2.2 and 3.2 (eqs. (7), (9)-(13)).
//
// With the exact split of the phase into a Tx part psi_p(m), an Rx part psi_q(m) and the
// cross term slope d_p e_q used by the VALU kernel, the echo is
//   H[p, q, m] = sum_f A_fp(m) B_fq(m) exp(j 2 pi slope d_p e_q),
//   A_fp(m) = G_f(m) exp(-j 2 pi psi_p(m)) / R_p,   B_fq(m) = exp(-j 2 pi psi_q(m)) / R_q.
// Dropping the cross term (the host bounds |2 pi slope d_p e_q| and takes this kernel
// only below 1e-5 rad, i.e. a relative error below 1e-5 per term) leaves, for every
// sample m, a complex (P x F) (F x Q) contraction over the lit facets: matrix-core work.
//
// Layout: v_mfma_f32_4x4x1f32 computes 16 independent 4x4 outer products per wave
// (block k = lanes 4k..4k+3: A lane 4k+i is row i, B lane 4k+j is column j, result
// register i of lane 4k+j is element (i, j)). Here block k = sample m_w + k, rows = 4 Tx
// elements of a Tx tile, columns = 4 Rx elements of an Rx tile. Per facet a lane
// evaluates its PT Tx and QT Rx element phasors at its sample (one FMA on an FP32 phase
// taken at the block centre after an FP64 reduction, hardware sine/cosine), multiplies
// the Tx ones by G_f(m), and the wave issues 4 MFMAs per (Tx tile, Rx tile) for the
// complex product:
//   Re += Ar Br + (-Ai) Bi,  Im += Ai Br + Ar Bi.
// A workgroup covers one chirp and 128 samples with eight accumulating waves (16 samples
// each) and four staging waves (one per SIMD) that fill double-buffered LDS tiles of FT
// facets (FP64 geometry, element phases per block, G(m)), as in the VALU kernel. MFMAs
// and vector instructions of one wave are issued in separate groups: interleaved, they
// cost extra issue cycles on this GPU.
#include "echo_common.h"

namespace rsim {

typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMfmaWaves = 8;          // accumulating waves, 16 samples each
constexpr int kMfmaTile = 16 * kMfmaWaves;  // samples per workgroup
constexpr int kMfmaBlk = 16;           // samples per phase block (one wave)
constexpr double kBlkMid = 7.5;        // block centre, where the staged phase is taken
constexpr int kMfmaStagingWaves = 4;  // one per SIMD, beside two accumulating waves
constexpr int kMfmaThreads = (kMfmaWaves + kMfmaStagingWaves) * 64;

template <int FT>
struct MfmaLayout {
  size_t elem, geo, glin, buf[2], G, EP, IR, total;
  __host__ __device__ explicit MfmaLayout(const EchoShape &sh) {
    auto up = [](size_t b) { return (b + 15) & ~size_t(15); };
    size_t b = 0;
    elem = b;
    b = up(b + sizeof(double) * 3 * sh.E);
    geo = b;
    b = up(b + sizeof(Geo) * FT);
    glin = b;
    b = up(b + sizeof(GLin) * FT);
    size_t t = 0;
    G = t;  // [FT][kMfmaTile] float2
    t += sizeof(float2) * FT * kMfmaTile;
    EP = t;  // [kMfmaWaves][FT][slots] float2: (phase at the block centre, step) in turns
    t += sizeof(float2) * kMfmaWaves * FT * sh.slots;
    IR = t;  // [FT][slots] float: 1 / R
    t = up(t + sizeof(float) * FT * sh.slots);
    buf[0] = b;
    buf[1] = b + t;
    total = b + 2 * t;
  }
};

template <int FT>
struct MfmaSmem {
  double *elem;
  Geo *geo;
  GLin *glin;
  unsigned char *buf0;
  size_t stride, oG, oEP, oIR;
  __device__ void carve(unsigned char *base, const EchoShape &sh) {
    const MfmaLayout<FT> L(sh);
    elem = reinterpret_cast<double *>(base + L.elem);
    geo = reinterpret_cast<Geo *>(base + L.geo);
    glin = reinterpret_cast<GLin *>(base + L.glin);
    buf0 = base + L.buf[0];
    stride = L.buf[1] - L.buf[0];
    oG = L.G;
    oEP = L.EP;
    oIR = L.IR;
  }
  __device__ float2 *G(int k) const { return reinterpret_cast<float2 *>(buf0 + k * stride + oG); }
  __device__ float2 *EP(int k) const { return reinterpret_cast<float2 *>(buf0 + k * stride + oEP); }
  __device__ float *IR(int k) const { return reinterpret_cast<float *>(buf0 + k * stride + oIR); }
};

__device__ inline void mfma_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ inline float centred(double t) { return static_cast<float>(t - rint(t)); }

// Staging of one tile (entries t0 .. t0 + nf - 1 of chirp n) into buffer k; each of the
// staging waves takes its share of the entries through all steps. Element e has slot e
// (Tx) or slots_tx + e - P (Rx) in a facet's row of sh.slots; the padding slots are
// never written (they feed only product rows and columns that are never stored).
template <int FT>
__device__ void mfma_stage(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                           const MfmaSmem<FT> &sm, int k, int n, int32_t cnt, int32_t t0, int nf,
                           int m_tile0, int st) {
  constexpr int kHalf = FT / kMfmaStagingWaves;  // entries per staging wave
  static_assert(FT % kMfmaStagingWaves == 0 && kHalf <= 64, "staging waves split the tile");
  const int P = rc.P, E = sh.E;
  const int lane = st & 63, i0 = (st >> 6) * kHalf;
  const double slope = rc.slope;
  float2 *G = sm.G(k);
  float2 *EP = sm.EP(k);
  float *IR = sm.IR(k);
  for (int i = i0 + lane; i < i0 + kHalf && lane < kHalf; i += 64) {
    if (i < nf)
      entry_geometry(sc, rc, n, cnt, t0 + i, sm.geo[i]);
    else
      sm.geo[i].valid = 0;
    make_glin(sm.geo[i], rc, m_tile0, sm.glin[i]);
    if (rc.intra && sm.geo[i].valid)
      sm.glin[i].quad = static_cast<float>(chord_curvature(sm.geo[i], rc, m_tile0, kMfmaBlk));
  }
  mfma_lds_sync();
  // element phases per 16-sample block: FP64, reduced to turns, then FP32
  for (int task = lane; task < kHalf * E; task += 64) {
    const int i = i0 + task / E, e = task % E;
    const int slot = e < P ? e : sh.slots_tx + (e - P);  // Tx slots, then Rx slots
    const int S = sh.slots;
    const Geo g = lds_copy(sm.geo[i]);  // one batch of LDS reads
    if (!g.valid) {
      for (int b = 0; b < kMfmaWaves; ++b) EP[(b * FT + i) * S + slot] = make_float2(0.0f, 0.0f);
      IR[i * S + slot] = 0.0f;
      continue;
    }
    const double dx = sm.elem[3 * e + 0] - g.c[0];
    const double dy = sm.elem[3 * e + 1] - g.c[1];
    const double dz = sm.elem[3 * e + 2] - g.c[2];
    const double Rn = sqrt(dx * dx + dy * dy + dz * dz);
    IR[i * S + slot] = __builtin_amdgcn_rcpf(static_cast<float>(Rn));  // amplitude only: 1 ulp
    if (!rc.intra) {
      const double tau = Rn * (1.0 / kC0);
      // Tx element: reference delay of its own side tref_t, of the other side tref_r
      const bool tx = e < P;
      const double t_self = tx ? g.tref_t : g.tref_r, t_other = tx ? g.tref_r : g.tref_t;
      double psi0 = rc.f0 * tau - 0.5 * slope * tau * tau - slope * t_other * (tau - t_self) -
                    0.5 * slope * g.tref_t * g.tref_r;
      psi0 -= floor(psi0);
      double delta = rc.df * tau;
      delta -= floor(delta);
      const float dstep = centred(delta);
      for (int b = 0; b < kMfmaWaves; ++b) {
        const double m0 = static_cast<double>(m_tile0 + b * kMfmaBlk);
        EP[(b * FT + i) * S + slot] = make_float2(centred(psi0 + (m0 + kBlkMid) * delta), dstep);
      }
    } else {
      for (int b = 0; b < kMfmaWaves; ++b) {
        const int ma = m_tile0 + b * kMfmaBlk;
        const double pa = element_phase(g, rc, sm.elem + 3 * e, e < P, ma);
        const double pb = element_phase(g, rc, sm.elem + 3 * e, e < P, ma + kMfmaBlk);
        const double step = (pb - pa) * (1.0 / kMfmaBlk);
        EP[(b * FT + i) * S + slot] = make_float2(centred(pa + kBlkMid * step), centred(step));
      }
    }
  }
  // G_f(m) for the tile's samples: one facet at a time, its coefficients read from LDS
  // into registers once (in one batch) rather than field by field inside the branches
  static_assert(kMfmaTile % 64 == 0, "whole waves per facet");
  for (int ii = 0; ii < kHalf; ++ii) {
    const int i = i0 + ii;
    const GLin q = lds_copy(sm.glin[i]);
    for (int j = lane; j < kMfmaTile; j += 64) {
      float2 val = g_lin(q, j);
      if (rc.intra) {
        const int jj = j % kMfmaBlk;
        const float x = 6.283185307179586f * q.quad * static_cast<float>(jj * (jj - kMfmaBlk));
        val = make_float2(fmaf(val.y, x, val.x), fmaf(-val.x, x, val.y));
      }
      G[i * kMfmaTile + j] = val;
    }
  }
}

// exp(-j 2 pi (phi0 + s step)) * ir
// exp(-j 2 pi (phi_c + s step)) / R for a sample s - 7.5 samples from the block centre
// (|t| <= 4.25 turns: the hardware sine and cosine take it unreduced, and its FP32
// rounding stays below 2.4e-7 turns)
__device__ inline float2 elem_phasor(float2 ep, float s, float ir) {
  const float t = fmaf(s, ep.y, ep.x);
  return make_float2(__builtin_amdgcn_cosf(t) * ir, -__builtin_amdgcn_sinf(t) * ir);
}

// LDS values behind the operands of one facet for this lane (sample mj, slot l of each
// group of four): G at its sample, and (phase, step) and 1 / R of its Tx slots 4a + l and
// Rx slots 4 PT + 4b + l. Padding slots hold whatever the LDS holds; they reach only
// products that are never stored.
template <int PT, int QT>
struct MfmaRaw {
  float2 g, et[PT], er[QT];
  float it[PT], ir[QT];
};

template <int PT, int QT>
__device__ inline void mfma_load(const float2 *G, const float2 *EP, const float *IR, int i, int mj,
                                 int l, MfmaRaw<PT, QT> &r) {
  constexpr int kSlots = 4 * (PT + QT);
  r.g = G[i * kMfmaTile + mj];
  const float2 *ep = EP + i * kSlots + l;
  const float *ir = IR + i * kSlots + l;
#pragma unroll
  for (int a = 0; a < PT; ++a) {
    r.et[a] = ep[4 * a];
    r.it[a] = ir[4 * a];
  }
#pragma unroll
  for (int b = 0; b < QT; ++b) {
    r.er[b] = ep[4 * (PT + b)];
    r.ir[b] = ir[4 * (PT + b)];
  }
}

// Operands A = G T_p / R_p (Tx) and B = T_q / R_q (Rx) at sample offset sf in the block.
template <int PT, int QT>
__device__ inline void mfma_form(const MfmaRaw<PT, QT> &r, float sf, float (&ar)[PT],
                                 float (&ai)[PT], float (&br)[QT], float (&bi)[QT]) {
#pragma unroll
  for (int a = 0; a < PT; ++a) {
    const float2 t = elem_phasor(r.et[a], sf, r.it[a]);
    ar[a] = r.g.x * t.x - r.g.y * t.y;
    ai[a] = r.g.x * t.y + r.g.y * t.x;
  }
#pragma unroll
  for (int b = 0; b < QT; ++b) {
    const float2 t = elem_phasor(r.er[b], sf, r.ir[b]);
    br[b] = t.x;
    bi[b] = t.y;
  }
}

// Complex rank-1 update of every (Tx tile, Rx tile) pair in four passes, so that
// consecutive MFMAs are independent: Re += Ar Br - Ai Bi, Im += Ai Br + Ar Bi.
template <int PT, int QT>
__device__ inline void mfma_accumulate(v4f (&acr)[PT][QT], v4f (&aci)[PT][QT],
                                       const float (&ar)[PT], const float (&ai)[PT],
                                       const float (&br)[QT], const float (&bi)[QT]) {
  float nai[PT];
#pragma unroll
  for (int a = 0; a < PT; ++a) nai[a] = -ai[a];
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b)
      acr[a][b] = __builtin_amdgcn_mfma_f32_4x4x1f32(ar[a], br[b], acr[a][b], 0, 0, 0);
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b)
      aci[a][b] = __builtin_amdgcn_mfma_f32_4x4x1f32(ai[a], br[b], aci[a][b], 0, 0, 0);
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b)
      aci[a][b] = __builtin_amdgcn_mfma_f32_4x4x1f32(ar[a], bi[b], aci[a][b], 0, 0, 0);
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b)
      acr[a][b] = __builtin_amdgcn_mfma_f32_4x4x1f32(nai[a], bi[b], acr[a][b], 0, 0, 0);
}

// One work item (chirp n, sample tile mt), split in its two roles. The staging waves and
// the accumulating waves pass the same barriers: one per tile and a final one.
template <int FT>
__device__ void mfma_stage_item(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                                const MfmaSmem<FT> &sm, int n, int mt, int st) {
  const int m_tile0 = mt * kMfmaTile;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t total = cnt + sc.n_points;
  const int32_t n_tiles = (total + FT - 1) / FT;
  if (n_tiles > 0) mfma_stage<FT>(sc, rc, sh, sm, 0, n, cnt, 0, min(FT, total), m_tile0, st);
  for (int32_t k = 0; k < n_tiles; ++k) {
    __syncthreads();
    const int32_t t1 = (k + 1) * FT;
    if (t1 < total)
      mfma_stage<FT>(sc, rc, sh, sm, (k & 1) ^ 1, n, cnt, t1, min(FT, total - t1), m_tile0, st);
  }
  __syncthreads();
}

template <int PT, int QT, int FT>
__device__ void mfma_compute_item(const DevScene &sc, const RadarConst &rc, const EchoShape &sh,
                                  const MfmaSmem<FT> &sm, int n, int mt) {
  const int tid = threadIdx.x;
  const int m_tile0 = mt * kMfmaTile;
  const int32_t total = sc.vis_cnt[n] + sc.n_points;
  const int32_t n_tiles = (total + FT - 1) / FT;
  const int P = rc.P, Q = rc.Q;
  const int w = tid >> 6, lane = tid & 63;
  const int s = lane >> 2, l = lane & 3;  // block (sample) and row/column within it
  const int mj = w * kMfmaBlk + s;        // sample within the tile
  const float sf = static_cast<float>(s) - static_cast<float>(kBlkMid);  // from the block centre
  v4f acr[PT][QT], aci[PT][QT];
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int b = 0; b < QT; ++b) {
      acr[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
      aci[a][b] = v4f{0.f, 0.f, 0.f, 0.f};
    }
  for (int32_t k = 0; k < n_tiles; ++k) {
    __syncthreads();
    const int buf = k & 1;
    const float2 *G = sm.G(buf);
    const float2 *EP = sm.EP(buf) + w * FT * (4 * (PT + QT));
    const float *IR = sm.IR(buf);
    const int nf = min(FT, total - k * FT);  // >= 1
    // Software pipeline: the LDS reads of facet i + 1 are in flight while the MFMAs of
    // facet i run; its operands are formed after them. Scheduling barriers keep the
    // MFMAs in one group and the vector work in another (interleaving the two within a
    // wave costs issue cycles on this hardware).
    float ar[PT], ai[PT], br[QT], bi[QT];
    MfmaRaw<PT, QT> raw;
    mfma_load<PT, QT>(G, EP, IR, 0, mj, l, raw);
    mfma_form<PT, QT>(raw, sf, ar, ai, br, bi);
    for (int i = 1; i < nf; ++i) {
      mfma_load<PT, QT>(G, EP, IR, i, mj, l, raw);
      __builtin_amdgcn_sched_barrier(0);
      mfma_accumulate<PT, QT>(acr, aci, ar, ai, br, bi);
      __builtin_amdgcn_sched_barrier(0);
      mfma_form<PT, QT>(raw, sf, ar, ai, br, bi);
    }
    mfma_accumulate<PT, QT>(acr, aci, ar, ai, br, bi);
  }
  __syncthreads();  // every wave done with the tile buffers (the next item reuses them)
  // lane (s, l), register r of tile pair (a, b): p = 4a + r, q = 4b + l, sample mj
  const int m = m_tile0 + mj;
  if (m >= rc.M) return;
  // The channel stride and sizes pass through an empty asm so that the output addresses
  // are formed here, per item, instead of being hoisted out of the persistent loop and
  // held (spilled) across it.
  int64_t S = static_cast<int64_t>(rc.N) * rc.M;
  int Pv = P, Qv = Q;
  asm volatile("" : "+s"(S), "+s"(Pv), "+s"(Qv));
  float2 *base = static_cast<float2 *>(sc.echo) + (l * S + static_cast<int64_t>(n) * rc.M + m);
  const float gr = static_cast<float>(sh.gamma_re), gi = static_cast<float>(sh.gamma_im);
#pragma unroll
  for (int a = 0; a < PT; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int p = 4 * a + r;
      if (p >= Pv) continue;
      float2 *row = base + static_cast<int64_t>(p) * Qv * S;
#pragma unroll
      for (int b = 0; b < QT; ++b) {
        if (4 * b + l >= Qv) continue;
        float2 *dst = row + static_cast<int64_t>(4 * b) * S;
        const float vr = acr[a][b][r], vi = aci[a][b][r];
        if (!sh.accumulate) {
          *dst = make_float2(vr, vi);
        } else {
          const float2 d = *dst;
          *dst = make_float2(d.x + (gr * vr - gi * vi), d.y + (gr * vi + gi * vr));
        }
      }
    }
}

template <int PT, int QT, int FT>
__global__ void __launch_bounds__(kMfmaThreads) echo_mfma_kernel(DevScene sc, RadarConst rc,
                                                        const double *elem, EchoShape sh) {
  extern __shared__ __align__(16) unsigned char mfma_smem[];
  MfmaSmem<FT> sm;
  sm.carve(mfma_smem, sh);
  for (int i = threadIdx.x; i < 3 * sh.E; i += blockDim.x) sm.elem[i] = elem[i];
  __syncthreads();
  const int n = blockIdx.x / sh.m_tiles, mt = blockIdx.x % sh.m_tiles;
  constexpr int nc = kMfmaWaves * 64;
  if (threadIdx.x >= nc)
    mfma_stage_item<FT>(sc, rc, sh, sm, n, mt, threadIdx.x - nc);
  else
    mfma_compute_item<PT, QT, FT>(sc, rc, sh, sm, n, mt);
}

// Persistent form over a longest-first queue of (scene, chirp, sample tile) items. Each
// role runs its own loop (so that neither holds the other's values); both pass the same
// barriers per item.
template <int PT, int QT, int FT>
__global__ void __launch_bounds__(kMfmaThreads) echo_mfma_persistent_kernel(
    const DevScene *scenes, const int4 *items, int32_t n_items, int32_t *queue, RadarConst rc,
    const double *elem, EchoShape sh) {
  extern __shared__ __align__(16) unsigned char mfma_smem[];
  __shared__ int32_t s_item;
  MfmaSmem<FT> sm;
  sm.carve(mfma_smem, sh);
  for (int i = threadIdx.x; i < 3 * sh.E; i += blockDim.x) sm.elem[i] = elem[i];
  constexpr int nc = kMfmaWaves * 64;
  if (threadIdx.x >= nc) {
    const int st = threadIdx.x - nc;
    while (true) {
      __syncthreads();
      if (st == 0) s_item = atomicAdd(queue, 1);
      __syncthreads();
      const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
      if (it >= n_items) break;  // every workgroup reaches this once the queue is drained
      const int4 wk = items[it];
      mfma_stage_item<FT>(scenes[wk.x], rc, sh, sm, wk.y, wk.z, st);
    }
  } else {
    while (true) {
      __syncthreads();
      __syncthreads();
      const int32_t it = __builtin_amdgcn_readfirstlane(s_item);
      if (it >= n_items) break;
      const int4 wk = items[it];
      mfma_compute_item<PT, QT, FT>(scenes[wk.x], rc, sh, sm, wk.y, wk.z);
    }
  }
}

__global__ void mfma_reset_counter_kernel(int32_t *q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

constexpr int kMfmaFT = 16;

#define RSIM_MFMA_VARIANTS(X) \
  X(1, 1)                     \
  X(1, 4)                     \
  X(2, 2)                     \
  X(3, 4)

bool mfma_variant(int P, int Q, int *pt, int *qt) {
  const int a = (P + 3) / 4, b = (Q + 3) / 4;
#define X(PT, QT)                   \
  if (a <= PT && b <= QT) {         \
    *pt = PT;                       \
    *qt = QT;                       \
    return true;                    \
  }
  RSIM_MFMA_VARIANTS(X)
#undef X
  return false;
}

size_t mfma_smem_bytes(const EchoShape &sh) { return MfmaLayout<kMfmaFT>(sh).total; }

int mfma_tile_samples() { return kMfmaTile; }

hipError_t launch_echo_mfma(const DevScene &sc, const RadarConst &rc, const double *elem,
                            const EchoShape &sh, hipStream_t s) {
  int pt = 0, qt = 0;
  if (!mfma_variant(rc.P, rc.Q, &pt, &qt)) return hipErrorInvalidValue;
  if (sh.slots_tx != 4 * pt || sh.slots != 4 * (pt + qt)) return hipErrorInvalidValue;
  const unsigned grid = static_cast<unsigned>(rc.N) * sh.m_tiles;
  const size_t lds = mfma_smem_bytes(sh);
  const int threads = kMfmaThreads;
#define X(PT, QT)                                                                            \
  if (pt == PT && qt == QT) {                                                                \
    hipLaunchKernelGGL((echo_mfma_kernel<PT, QT, kMfmaFT>), dim3(grid), dim3(threads), lds, s, \
                       sc, rc, elem, sh);                                                    \
    return hipGetLastError();                                                                \
  }
  RSIM_MFMA_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t launch_echo_mfma_persistent(const DevScene *scenes, const int4 *items, int32_t n_items,
                                       int32_t *queue, const RadarConst &rc, const double *elem,
                                       const EchoShape &sh, int n_groups, hipStream_t s) {
  int pt = 0, qt = 0;
  if (!mfma_variant(rc.P, rc.Q, &pt, &qt)) return hipErrorInvalidValue;
  if (sh.slots_tx != 4 * pt || sh.slots != 4 * (pt + qt)) return hipErrorInvalidValue;
  const size_t lds = mfma_smem_bytes(sh);
  const int threads = kMfmaThreads;
  hipLaunchKernelGGL(mfma_reset_counter_kernel, dim3(1), dim3(64), 0, s, queue);
#define X(PT, QT)                                                                           \
  if (pt == PT && qt == QT) {                                                               \
    hipLaunchKernelGGL((echo_mfma_persistent_kernel<PT, QT, kMfmaFT>), dim3(n_groups),       \
                       dim3(threads), lds, s, scenes, items, n_items, queue, rc, elem, sh); \
    return hipGetLastError();                                                               \
  }
  RSIM_MFMA_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

hipError_t mfma_occupancy(int P, int Q, const EchoShape &sh, int *groups_per_cu) {
  int pt = 0, qt = 0;
  if (!mfma_variant(P, Q, &pt, &qt)) return hipErrorInvalidValue;
  if (sh.slots_tx != 4 * pt || sh.slots != 4 * (pt + qt)) return hipErrorInvalidValue;
  const size_t lds = mfma_smem_bytes(sh);
  const int threads = kMfmaThreads;
#define X(PT, QT)                                                                       \
  if (pt == PT && qt == QT)                                                             \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(                                \
        groups_per_cu,                                                                  \
        reinterpret_cast<const void *>(echo_mfma_persistent_kernel<PT, QT, kMfmaFT>),   \
        threads, lds);
  RSIM_MFMA_VARIANTS(X)
#undef X
  return hipErrorInvalidValue;
}

}  // namespace rsim
