// Shared pieces of the two adjoint facet-sum kernels (vector units and matrix cores):
// the per-facet sums they produce and the facet integral with its node derivatives.
#ifndef RSIM_ADJOINT_COMMON_H
#define RSIM_ADJOINT_COMMON_H

#include "echo_common.h"

namespace rsim {

constexpr int kAdjVals = 8;  // grad_c (3), sum Re y, t0, t1, t2, pad
// per-wave sums of the vector-unit adjoint with the delay within the chirp: the seven
// above, then the velocity's sum over samples (3), padding
constexpr int kAdjRedIntra = 12;

// sinc(u) and sinc'(u) = (cos u - sinc u) / u at u = x0 + j x_i (rad), t = u / (2 pi)
// (turns, centred at j = 0). Series below |u| = 0.3.
__device__ inline float sinc_d_lin(float x0, float x_i, float t0, float t_i, float jf,
                                   float *sinc_out) {
  const float u = fmaf(jf, x_i, x0);
  if (fabsf(u) < kSincSeries) {
    const float u2 = u * u;
    *sinc_out = sinc_series(u2);
    return u * fmaf(u2, fmaf(u2, fmaf(u2, 1.0f / 45360.0f, -1.0f / 840.0f), 1.0f / 30.0f),
                    -1.0f / 3.0f);
  }
  float t = fmaf(jf, t_i, t0);
  t -= rintf(t);
  const float r = __builtin_amdgcn_rcpf(u);
  const float sc = __builtin_amdgcn_sinf(t) * r;
  *sinc_out = sc;
  return (__builtin_amdgcn_cosf(t) - sc) * r;
}

// G(m) = amp Phi and D_k(m) = amp k_m dPhi/da_k (k = triangle vertex; a_k = k_m b_k) at
// sample m_tile0 + j, from the linear-phase coefficients of the forward facet integral.
// Sinc form: with F(x, y) = -j exp(j (x + y) / 2) sinc((y - x) / 2),
//   Phi = (F(a_l, a_j) - F(a_l, a_i)) / (a_j - a_i),
//   dPhi/da_l = (F_x(a_l, a_j) - F_x(a_l, a_i)) / (a_j - a_i),
//   dPhi/da_j = (F_y(a_l, a_j) - Phi) / (a_j - a_i),  dPhi/da_i = (Phi - F_y(a_l, a_i)) / (a_j - a_i),
//   F_x = K (-sinc'/2 + j sinc/2),  F_y = K (sinc'/2 + j sinc/2),  K = -j exp(j (x + y) / 2).
// Series form about the mean (Sec. 3.2): Phi_0 = sum_n j^n h_n(b) / (n+2)!,
//   dPhi_0/db_k = sum_n j^(n+1) h_n(b, b_k) / (n+3)!, both turned by exp(j mean).
__device__ inline void g_lin_grad(const GLin &q, int j, float2 &G, float2 D[3]) {
  if (!q.valid) {
    G = D[0] = D[1] = D[2] = make_float2(0.0f, 0.0f);
    return;
  }
  const float jf = static_cast<float>(j);
  float2 p0, d[3];
  if (fmaf(jf, q.gap_i, q.gap) < static_cast<float>(kSeriesGap)) {
    const float bk[3] = {fmaf(jf, q.b0_i, q.b0), fmaf(jf, q.b1_i, q.b1), fmaf(jf, q.b2_i, q.b2)};
    const float e1 = bk[0] + bk[1] + bk[2];
    const float e2 = bk[0] * bk[1] + bk[0] * bk[2] + bk[1] * bk[2];
    const float e3 = bk[0] * bk[1] * bk[2];
    float h[9];
    h[0] = 1.0f;
    float hm1 = 1.0f, hm2 = 0.0f, hm3 = 0.0f;
#pragma unroll
    for (int n = 1; n < 9; ++n) {
      const float hn = e1 * hm1 - e2 * hm2 + e3 * hm3;
      hm3 = hm2;
      hm2 = hm1;
      hm1 = hn;
      h[n] = hn;
    }
    float re = 0.0f, im = 0.0f, inv_fact = 0.5f;  // 1 / (n+2)!
#pragma unroll
    for (int n = 0; n <= 8; ++n) {
      if (n > 0) inv_fact *= 1.0f / static_cast<float>(n + 2);
      const float term = h[n] * inv_fact;
      switch (n & 3) {
        case 0: re += term; break;
        case 1: im += term; break;
        case 2: re -= term; break;
        default: im -= term; break;
      }
    }
    p0 = make_float2(re, im);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      float h4 = 1.0f, dre = 0.0f, dim = 0.0f, inv3 = 1.0f / 6.0f;  // 1 / (n+3)!
#pragma unroll
      for (int n = 0; n <= 7; ++n) {
        if (n > 0) {
          h4 = fmaf(bk[k], h4, h[n]);
          inv3 *= 1.0f / static_cast<float>(n + 3);
        }
        const float term = h4 * inv3;
        switch ((n + 1) & 3) {  // j^(n+1)
          case 0: dre += term; break;
          case 1: dim += term; break;
          case 2: dre -= term; break;
          default: dim -= term; break;
        }
      }
      d[k] = make_float2(dre, dim);
    }
    float t = fmaf(jf, q.mp_i, q.mp);
    t -= rintf(t);
    const float ms = __builtin_amdgcn_sinf(t), mc = __builtin_amdgcn_cosf(t);
    p0 = make_float2(p0.x * mc - p0.y * ms, p0.x * ms + p0.y * mc);
#pragma unroll
    for (int k = 0; k < 3; ++k)
      d[k] = make_float2(d[k].x * mc - d[k].y * ms, d[k].x * ms + d[k].y * mc);
  } else {
    float t1 = fmaf(jf, q.p1_i, q.p1);
    t1 -= rintf(t1);
    float t2 = fmaf(jf, q.p2_i, q.p2);
    t2 -= rintf(t2);
    const float sn1 = __builtin_amdgcn_sinf(t1), cs1 = __builtin_amdgcn_cosf(t1);
    const float sn2 = __builtin_amdgcn_sinf(t2), cs2 = __builtin_amdgcn_cosf(t2);
    float sc1, sc2;
    const float sd1 = sinc_d_lin(q.x1, q.x1_i, q.t1, q.t1_i, jf, &sc1);
    const float sd2 = sinc_d_lin(q.x2, q.x2_i, q.t2, q.t2_i, jf, &sc2);
    const float inv = __builtin_amdgcn_rcpf(fmaf(jf, q.w_i, q.w));
    // K = (sn, -cs); F = K sinc; F_x = K (-sd/2 + j sc/2); F_y = K (sd/2 + j sc/2)
    const float2 F1 = make_float2(sn1 * sc1, -cs1 * sc1), F2 = make_float2(sn2 * sc2, -cs2 * sc2);
    const float2 F1x = make_float2(0.5f * (cs1 * sc1 - sn1 * sd1), 0.5f * (sn1 * sc1 + cs1 * sd1));
    const float2 F2x = make_float2(0.5f * (cs2 * sc2 - sn2 * sd2), 0.5f * (sn2 * sc2 + cs2 * sd2));
    const float2 F1y = make_float2(0.5f * (cs1 * sc1 + sn1 * sd1), 0.5f * (sn1 * sc1 - cs1 * sd1));
    const float2 F2y = make_float2(0.5f * (cs2 * sc2 + sn2 * sd2), 0.5f * (sn2 * sc2 - cs2 * sd2));
    p0 = make_float2((F1.x - F2.x) * inv, (F1.y - F2.y) * inv);
    const float2 dl = make_float2((F1x.x - F2x.x) * inv, (F1x.y - F2x.y) * inv);
    const float2 dj = make_float2((F1y.x - p0.x) * inv, (F1y.y - p0.y) * inv);
    const float2 di = make_float2((p0.x - F2y.x) * inv, (p0.y - F2y.y) * inv);
    // scatter to vertex order
#pragma unroll
    for (int k = 0; k < 3; ++k) d[k] = (k == q.nl) ? dl : ((k == q.nj) ? dj : di);
  }
  const float km = fmaf(jf, q.k_i, q.k);
  G = make_float2(q.ar * p0.x - q.ai * p0.y, q.ar * p0.y + q.ai * p0.x);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    D[k] = make_float2(km * (q.ar * d[k].x - q.ai * d[k].y), km * (q.ar * d[k].y + q.ai * d[k].x));
}

// Sum over the 64 lanes of a wave: DPP moves inside each 16-lane row (no LDS round
// trips), then the four row sums read out with readlane (the DPP row-broadcast
// controls do not exist on this GPU generation). Fixed order: deterministic.
template <int kCtrl, int kRowMask>
__device__ inline float dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, kRowMask, 0xF,
                                            false);
  return v + __builtin_bit_cast(float, t);
}

// DPP reads the registers of inactive lanes as they are: every caller runs it with the
// whole wave active.
__device__ inline float wave_sum(float v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]: quad sums
  v = dpp_add<0x141, 0xF>(v);  // row_half_mirror: 8-lane sums
  v = dpp_add<0x140, 0xF>(v);  // row_mirror: 16-lane (row) sums in every lane
  const int iv = __builtin_bit_cast(int, v);
  const float r0 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 0));
  const float r1 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 16));
  const float r2 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 32));
  const float r3 = __builtin_bit_cast(float, __builtin_amdgcn_readlane(iv, 48));
  return (r0 + r1) + (r2 + r3);
}

struct AdjShape {
  EchoShape sh;
  int32_t F;  // facets of the scene (capacity of a chirp's lit list)
  int32_t pad;
};

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s);

}  // namespace rsim

#endif
