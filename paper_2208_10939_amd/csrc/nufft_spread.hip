// NUFFT facet sum, the spread: each run of cell-sorted records (one lit facet, point or
// double-bounce connection of one chirp each) adds its Gaussian grid sources, for every
// channel, into a register window of kNuSlots grid cells, written out once per run (see
// nufft.hip for the transform it belongs to and the kernels around it).
#include <hip/hip_runtime.h>

#include "nufft_common.h"
#include "rsim_internal.h"
#include "rsim_launch.h"

namespace rsim {

namespace {

// Gaussian (from cell S0 on: g_{s+1} = g_s rho_s, rho_{s+1} = rho_s exp(-1/s^2)) times the
// weight cw at the NCELL cells S0 .. S0 + NCELL - 1 of the window (cells past the window's
// end are dropped at compile time; the runs keep every source inside).
template <int S0, int NCELL>
__device__ __forceinline__ void point_cells(float2 (&acc)[kNuSlots], float2 cw, float gw,
                                            float rho, float q_ratio) {
  // the weights are formed here, in the block: hoisted ahead of the chain of blocks (they
  // are the same in every block) they would hold NCELL registers more across it
  asm volatile("" : "+v"(gw), "+v"(rho));
#pragma unroll
  for (int j = 0; j < NCELL; ++j) {
    if (S0 + j < kNuSlots) {
      acc[S0 + j].x = fmaf(gw, cw.x, acc[S0 + j].x);
      acc[S0 + j].y = fmaf(gw, cw.y, acc[S0 + j].y);
      gw *= rho;
      rho *= q_ratio;
    }
  }
}

// Gaussian times the polynomial sum_k c_k (s - pos)^k at the cells S0 .. S0 + NCELL - 1.
template <int S0, int NCELL, int NC>
__device__ __forceinline__ void poly_cells(float2 (&acc)[kNuSlots], const float2 (&c)[NC],
                                           float u0, float gw, float rho, float q_ratio) {
  asm volatile("" : "+v"(u0), "+v"(gw), "+v"(rho));  // formed in the block, as above
#pragma unroll
  for (int j = 0; j < NCELL; ++j) {
    if (S0 + j < kNuSlots) {
      const float xx = u0 + static_cast<float>(j);
      float pr = c[NC - 1].x, pi = c[NC - 1].y;
#pragma unroll
      for (int k = NC - 2; k >= 0; --k) {
        pr = fmaf(pr, xx, c[k].x);
        pi = fmaf(pi, xx, c[k].y);
      }
      acc[S0 + j].x = fmaf(gw, pr, acc[S0 + j].x);
      acc[S0 + j].y = fmaf(gw, pi, acc[S0 + j].y);
      gw *= rho;
      rho *= q_ratio;
    }
  }
}

// Gaussian times c0 + c2 (s - pos)^2 (no linear term: a point source under the delay
// within the chirp) at the cells S0 .. S0 + NCELL - 1.
template <int S0, int NCELL>
__device__ __forceinline__ void even2_cells(float2 (&acc)[kNuSlots], float2 c0, float2 c2,
                                            float u0, float gw, float rho, float q_ratio) {
  asm volatile("" : "+v"(u0), "+v"(gw), "+v"(rho));  // formed in the block, as above
#pragma unroll
  for (int j = 0; j < NCELL; ++j) {
    if (S0 + j < kNuSlots) {
      const float xx = u0 + static_cast<float>(j);
      const float x2 = xx * xx;
      const float pr = fmaf(c2.x, x2, c0.x), pi = fmaf(c2.y, x2, c0.y);
      acc[S0 + j].x = fmaf(gw, pr, acc[S0 + j].x);
      acc[S0 + j].y = fmaf(gw, pi, acc[S0 + j].y);
      gw *= rho;
      rho *= q_ratio;
    }
  }
}

// The window cell s_lo (wave-uniform) selects one straight-line block of NCELL cells. A
// source covers NCELL or fewer cells (its count is floor(2 reach) or one more, NCELL at
// least the larger), so a block may reach up to four cells past the last the runs
// guarantee inside the window; those are dropped (their Gaussian weights are below
// psi(W/2) for every channel). The blocks sit behind a chain of independent scalar bit
// tests rather than a switch: every block then updates the window registers in place,
// where the merge of a switch's cases costs register copies of the untouched cells.
// First cell of a source's block: the lowest cell within `reach` of the source's
// position for the wave's first channel, clamped to the blocks the chain holds (the
// runs keep every channel's cells inside the window, so a clamp never drops one of them).
// lo_lanes holds the unclamped cell of the record's source at s[3 j] in lane j (j < 3).
__device__ __forceinline__ int block_start(int lo_lanes, int j) {
  const int s = __builtin_amdgcn_readlane(lo_lanes, j);
  return s < 0 ? 0 : s > 22 ? 22 : s;
}

#define RSIM_NU_CASES(X) \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) \
  X(16) X(17) X(18) X(19) X(20) X(21) X(22)

template <int NCELL>
__device__ __forceinline__ void spread_point(float2 (&acc)[kNuSlots], float2 cw, float pos,
                                             int s_lo, float nc, float q_ratio) {
  const float u0 = static_cast<float>(s_lo) - pos;
  const float gw = __builtin_amdgcn_exp2f(nc * u0 * u0);
  const float rho = __builtin_amdgcn_exp2f(nc * fmaf(2.0f, u0, 1.0f));
  const uint32_t bit = static_cast<uint32_t>(s_lo) < 32u ? 1u << s_lo : 0u;  // none: no cell
#define RSIM_NU_POINT(S) \
  if (bit & (1u << S)) point_cells<S, NCELL>(acc, cw, gw, rho, q_ratio);
  RSIM_NU_CASES(RSIM_NU_POINT)
#undef RSIM_NU_POINT
}

template <int NCELL>
__device__ __forceinline__ void spread_even2(float2 (&acc)[kNuSlots], float2 c0, float2 c2,
                                             float pos, int s_lo, float nc, float q_ratio) {
  const float u0 = static_cast<float>(s_lo) - pos;
  const float gw = __builtin_amdgcn_exp2f(nc * u0 * u0);
  const float rho = __builtin_amdgcn_exp2f(nc * fmaf(2.0f, u0, 1.0f));
  const uint32_t bit = static_cast<uint32_t>(s_lo) < 32u ? 1u << s_lo : 0u;  // none: no cell
#define RSIM_NU_EVEN2(S) \
  if (bit & (1u << S)) even2_cells<S, NCELL>(acc, c0, c2, u0, gw, rho, q_ratio);
  RSIM_NU_CASES(RSIM_NU_EVEN2)
#undef RSIM_NU_EVEN2
}

template <int NCELL, int NC>
__device__ __forceinline__ void spread_poly(float2 (&acc)[kNuSlots], const float2 (&c)[NC],
                                            float pos, int s_lo, float nc, float q_ratio) {
  const float u0 = static_cast<float>(s_lo) - pos;
  const float gw = __builtin_amdgcn_exp2f(nc * u0 * u0);
  const float rho = __builtin_amdgcn_exp2f(nc * fmaf(2.0f, u0, 1.0f));
  const uint32_t bit = static_cast<uint32_t>(s_lo) < 32u ? 1u << s_lo : 0u;  // none: no cell
#define RSIM_NU_POLY(S) \
  if (bit & (1u << S)) poly_cells<S, NCELL, NC>(acc, c, u0, gw, rho, q_ratio);
  RSIM_NU_CASES(RSIM_NU_POLY)
#undef RSIM_NU_POLY
}

// (1 - j 2 pi B m'^2) on the modes is F + j eps F'' on the grid (F = psi P): coefficient
// k of the result is c_k + j eps (c_{k-2} / s^4 - (2k + 1) c_k / s^2 + (k+1)(k+2) c_{k+2}).
template <int NI, int NO>
__device__ __forceinline__ void intra_coeffs(const float2 (&c)[NI], float2 (&o)[NO], float eps,
                                             float inv_s2) {
  const float inv_s4 = inv_s2 * inv_s2;
#pragma unroll
  for (int k = 0; k < NO; ++k) {
    const float2 ck = k < NI ? c[k] : make_float2(0.0f, 0.0f);
    const float2 cm2 = (k >= 2 && k - 2 < NI) ? c[k - 2] : make_float2(0.0f, 0.0f);
    const float2 cp2 = (k + 2 < NI) ? c[k + 2] : make_float2(0.0f, 0.0f);
    const float wk = -(2.0f * k + 1.0f) * inv_s2;
    const float wp = static_cast<float>((k + 1) * (k + 2));
    const float dx = cm2.x * inv_s4 + wk * ck.x + wp * cp2.x;
    const float dy = cm2.y * inv_s4 + wk * ck.y + wp * cp2.y;
    o[k] = {ck.x - eps * dy, ck.y + eps * dx};
  }
}

}  // namespace

// One workgroup per (chirp, run) and up to four 64-channel groups (blockIdx.z counts
// further groups); lane = channel. The run's records (read once per wave through scalar
// loads, the next one in flight while the current one is spread) add their sources into a
// register window of kNuSlots cells starting at the run's base cell; the window is written
// to part[chirp][run][channel][kNuSlots]. The kernel waits mostly on latencies (record
// loads, transcendental results, the branch chain), so occupancy pays: the stop-and-hop
// form is held to five waves per SIMD (96 registers), the other to four.
template <bool INTRA, int NCELL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(INTRA ? 4 : 5, 8)))
nufft_spread_kernel(
    DevScene sc0, RadarConst rc, NuShape ns, const double *elem,
    const NuRecF<INTRA> *__restrict__ sorted, const int4 *__restrict__ runs,
    const int32_t *__restrict__ n_runs, float2 *__restrict__ part, NuBatch bt) {
  const int nl = blockIdx.y;
  const int run = blockIdx.x;
  if (run >= load_uniform(n_runs + nl)) return;  // whole workgroup
  const NuWork w = nu_work(sc0, ns, bt, nl);
  const int grp = static_cast<int>(blockIdx.z) * 4 + static_cast<int>(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int O = rc.P * rc.Q;
  if (grp * 64 >= O) return;  // whole wave
  const int4 rr = load_uniform(runs + w.run + run);
  const int o = grp * 64 + lane;
  const bool on = o < O;
  // this lane's element offsets from the phase centres
  double at[3], ar[3];
  float aat, aar, atf[3], arf[3];
  {
    const int oc = on ? o : grp * 64;  // idle lanes: the wave's first channel
    const int p = oc / rc.Q, q = oc - p * rc.Q;
    double st = 0.0, sr = 0.0;
    for (int k = 0; k < 3; ++k) {
      at[k] = elem[3 * p + k] - rc.tx_c[k];
      ar[k] = elem[3 * (rc.P + q) + k] - rc.rx_c[k];
      st += at[k] * at[k];
      sr += ar[k] * ar[k];
    }
    aat = static_cast<float>(st);
    aar = static_cast<float>(sr);
    for (int k = 0; k < 3; ++k) {
      atf[k] = static_cast<float>(at[k]);
      arf[k] = static_cast<float>(ar[k]);
    }
  }
  const float inv_c0 = static_cast<float>(1.0 / kC0), inv_fs = static_cast<float>(1.0 / rc.fs);
  const float df_fs = static_cast<float>(rc.df / rc.fs);
  const float half_m = 0.5f * rc.M, quarter_m2 = 0.25f * rc.M * rc.M, m_f = static_cast<float>(rc.M);
  const float ngf = static_cast<float>(ns.ng);
  const float eps_scale = static_cast<float>(static_cast<double>(ns.ng) * ns.ng / (2.0 * kPi));
  const float inv_s2 = static_cast<float>(1.0 / (ns.sigma * ns.sigma));
  const NuRecF<INTRA> *srec = sorted + w.rec;
  const float nc = static_cast<float>(-1.4426950408889634 / (2.0 * ns.sigma * ns.sigma));
  const float q_ratio = __builtin_amdgcn_exp2f(2.0f * nc);  // exp(-1 / s^2)
  const float kappa = static_cast<float>(ns.kappa);
  const float g2 = static_cast<float>(0.5 * rc.slope / (kC0 * kC0));
  const float reach = static_cast<float>(ns.wave_d) + 0.5f * kNuWidth;
  float2 acc[kNuSlots];
#pragma unroll
  for (int s = 0; s < kNuSlots; ++s) acc[s] = {0.0f, 0.0f};
  NuRecF<INTRA> nxt = load_uniform(srec + rr.x);
  for (int i = rr.x; i < rr.y; ++i) {
    const NuRecF<INTRA> r = nxt;
    nxt = load_uniform(srec + (i + 1 < rr.y ? i + 1 : i));
    if (r.kind == 0) continue;  // wave-uniform
    // position of the phase-centre path in the window
    const float rel_c = static_cast<float>(r.cell - rr.z) + r.frac;
    // this channel's path difference dL = -(s_t + s_r) + e_t + e_r, amplitude, phase
    // and grid position
    const double st = r.ut[0] * at[0] + r.ut[1] * at[1] + r.ut[2] * at[2];
    const double sr = r.ur[0] * ar[0] + r.ur[1] * ar[1] + r.ur[2] * ar[2];
    const double ps = (st + sr) * r.g1;  // turns, up to ~25
    const float pr = static_cast<float>(ps - rint(ps));
    const float sft = static_cast<float>(st), sfr = static_cast<float>(sr);
    const float ht = fmaf(-sft, sft, aat), hr = fmaf(-sfr, sfr, aar);
    const float rdt = __builtin_amdgcn_rcpf(fmaf(-2.0f, sft, 2.0f * r.rt));
    const float rdr = __builtin_amdgcn_rcpf(fmaf(-2.0f, sfr, 2.0f * r.rr));
    const float qt = ht * rdt, qr = hr * rdr;
    const float et = qt * fmaf(-qt, rdt, 1.0f), er = qr * fmaf(-qr, rdr, 1.0f);
    const float dRt = et - sft, dRr = er - sfr;
    const float dL = dRt + dRr;
    float t = (r.t0 - pr) + fmaf(static_cast<float>(r.g1), et + er, -g2 * dL * dL);
    float xr = fmaf(kappa, dL, rel_c);
    float eps = 0.0f;  // B n_g^2 / (2 pi): weight of F'' for the B m'^2 term
    if constexpr (INTRA) {
      // this channel's tau' (first order in the sample time), its Doppler shift relative
      // to the record's and the constant phase A M/2 + B M^2/4
      const float vat = r.ext[0] * atf[0] + r.ext[1] * atf[1] + r.ext[2] * atf[2];
      const float var = r.ext[0] * arf[0] + r.ext[1] * arf[1] + r.ext[2] * arf[2];
      const float rdt_dot = fmaf(r.rt, r.ext[3], -vat) * __builtin_amdgcn_rcpf(r.rt + dRt);
      const float rdr_dot = fmaf(r.rr, r.ext[4], -var) * __builtin_amdgcn_rcpf(r.rr + dRr);
      const float tdot = (rdt_dot + rdr_dot) * inv_c0;
      const float fmt = static_cast<float>(r.g1 * kC0 - (rc.M / 2) * rc.df);
      const float A = fmt * tdot * inv_fs, B = df_fs * tdot;
      t += fmaf(A, half_m, B * quarter_m2);
      xr += fmaf(B, m_f, A) * ngf - r.ext[5];
      eps = B * eps_scale;
    }
    t -= rintf(t);
    // the wave's first channel: every channel of the wave lies within wave_d cells of it
    const float x0 = __builtin_bit_cast(
        float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, xr)));
    const float amp = __builtin_amdgcn_rcpf((r.rt + dRt) * (r.rr + dRr));
    const float qx = __builtin_amdgcn_cosf(t) * amp, qy = -__builtin_amdgcn_sinf(t) * amp;
    const int n_pts = r.kind == 1 ? 3 : r.kind == 2 ? 1 : 0;
    // the block starts of the record's sources at s[0], s[3], s[6], one per lane (lanes 0,
    // 1, 2) in one pass instead of one wave-wide pass each
    const float off_l = lane == 0 ? r.s[0] : lane == 1 ? r.s[3] : r.s[6];
    const int lo_lanes = static_cast<int>(ceilf((x0 - off_l) - reach));
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      if (j < n_pts) {
        const float off = r.s[3 * j];
        const float2 cw = {qx * r.s[3 * j + 1] - qy * r.s[3 * j + 2],
                           qx * r.s[3 * j + 2] + qy * r.s[3 * j + 1]};
        // cells some channel reaches: |s - (x_o - off)| <= W/2 with |x_o - x0| <= wave_d,
        // NCELL of them from s_lo
        const int s_lo = block_start(lo_lanes, j);
        if constexpr (INTRA) {
          // (1 - j 2 pi B m'^2) on a point's modes: cw (1 - j eps / s^2) + j eps cw / s^4 x^2
          // (intra_coeffs of one coefficient; its linear term is zero)
          const float e2 = eps * inv_s2, e4 = e2 * inv_s2;
          const float2 c0 = {fmaf(e2, cw.y, cw.x), fmaf(-e2, cw.x, cw.y)};
          const float2 c2 = {-e4 * cw.y, e4 * cw.x};
          spread_even2<NCELL>(acc, c0, c2, xr - off, s_lo, nc, q_ratio);
        } else {
          spread_point<NCELL>(acc, cw, xr - off, s_lo, nc, q_ratio);
        }
      }
    }
    if (r.kind >= 2) {
      const float off = r.s[3];
      float2 cq[3];
#pragma unroll
      for (int k = 0; k < 3; ++k)
        cq[k] = {qx * r.s[4 + 2 * k] - qy * r.s[5 + 2 * k], qx * r.s[5 + 2 * k] + qy * r.s[4 + 2 * k]};
      const int s_lo = block_start(lo_lanes, 1);
      if constexpr (INTRA) {
        float2 c5[5];
        intra_coeffs(cq, c5, eps, inv_s2);
        spread_poly<NCELL>(acc, c5, xr - off, s_lo, nc, q_ratio);
      } else {
        spread_poly<NCELL>(acc, cq, xr - off, s_lo, nc, q_ratio);
      }
    }
  }
  if (!on) return;
  float4 *dst = reinterpret_cast<float4 *>(
      part + ((w.run + run) * O + o) * kNuSlots);
#pragma unroll
  for (int s = 0; s < kNuSlots / 2; ++s)
    dst[s] = make_float4(acc[2 * s].x, acc[2 * s].y, acc[2 * s + 1].x, acc[2 * s + 1].y);
}

namespace {

template <bool INTRA>
hipError_t launch_spread_t(const DevScene &sc, const RadarConst &rc, const NuShape &ns,
                           const double *elem, const NuRecF<INTRA> *recs, const int4 *runs,
                           const int32_t *n_runs, float2 *part, const NuBatch &bt, dim3 grid,
                           dim3 blk, int ncell, hipStream_t s) {
  switch (ncell) {
    case 14:
      hipLaunchKernelGGL((nufft_spread_kernel<INTRA, 14>), grid, blk, 0, s, sc, rc, ns, elem,
                         recs, runs, n_runs, part, bt);
      break;
    case 16:
      hipLaunchKernelGGL((nufft_spread_kernel<INTRA, 16>), grid, blk, 0, s, sc, rc, ns, elem,
                         recs, runs, n_runs, part, bt);
      break;
    case 20:
      hipLaunchKernelGGL((nufft_spread_kernel<INTRA, 20>), grid, blk, 0, s, sc, rc, ns, elem,
                         recs, runs, n_runs, part, bt);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_nufft_spread(const DevScene &sc, const RadarConst &rc, const NuShape &ns,
                               const double *elem, const void *srec, const int4 *runs,
                               const int32_t *n_runs, float2 *part, const NuBatch &bt,
                               hipStream_t s) {
  const int O = rc.P * rc.Q;
  const int groups = (O + 63) / 64;
  const int per_block = groups < 4 ? groups : 4;
  dim3 sgrid(static_cast<unsigned>(ns.max_runs), static_cast<unsigned>(ns.n_chirps),
             static_cast<unsigned>((groups + 3) / 4));
  const dim3 blk(64 * per_block);
  const int ncell = nufft_cells_per_source(ns);
  if (rc.intra)
    return launch_spread_t<true>(sc, rc, ns, elem, static_cast<const NuRecF<true> *>(srec), runs,
                                 n_runs, part, bt, sgrid, blk, ncell, s);
  return launch_spread_t<false>(sc, rc, ns, elem, static_cast<const NuRecF<false> *>(srec), runs,
                                n_runs, part, bt, sgrid, blk, ncell, s);
}

}  // namespace rsim
