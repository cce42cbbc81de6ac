// Device helpers shared by the facet-sum kernel and its adjoint: complex types,
// the closed-form facet integral Phi and the FP64 facet/point geometry.
#pragma once

#include "rsim_internal.h"
#include "rsim_launch.h"

namespace rsim {

template <typename R>
struct Cx;
template <>
struct Cx<float> {
  using T = float2;
};
template <>
struct Cx<double> {
  using T = double2;
};

template <typename R>
struct EchoTraits;
template <>
struct EchoTraits<float> {
  static constexpr int kSeriesTerms = 8;
};
template <>
struct EchoTraits<double> {
  static constexpr int kSeriesTerms = 16;
};
constexpr double kSeriesGap = 0.5;  // radians: series below, divided-difference form above

struct alignas(16) Geo {
  double c[3];        // centroid (world) at t_n
  double tref_t, tref_r;
  double beta[3];     // w . (x_i - c), metres
  double amp_re, amp_im;  // G = amp * Phi
  double vel[3];      // world velocity of the facet or point
  int32_t valid, pad;
};

// A copy of an LDS record in registers, read as whole 16-byte words in one batch.
template <typename T>
__device__ inline T lds_copy(const T &src) {
  static_assert(sizeof(T) % 16 == 0 && alignof(T) >= 16, "16-byte records");
  constexpr int kWords = sizeof(T) / 16;
  float4 w[kWords];
  const float4 *p = reinterpret_cast<const float4 *>(&src);
#pragma unroll
  for (int k = 0; k < kWords; ++k) w[k] = p[k];
  T out;
  __builtin_memcpy(&out, w, sizeof(T));
  return out;
}

__device__ inline float fma_r(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ inline double fma_r(double a, double b, double c) { return __builtin_fma(a, b, c); }

// sin(pi x), cos(pi x) for |x| <= 1 (every caller reduces first). The FP32 version uses
// the hardware transcendental unit, which takes revolutions; its error on this range
// was measured at <= 1.3e-7 absolute on MI355X (ocml sincospif: 5e-8).
__device__ inline void sincospi_t(float x, float *s, float *c) {
  const float r = 0.5f * x;
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}
__device__ inline void sincospi_t(double x, double *s, double *c) { sincospi(x, s, c); }

// exp(-j 2 pi turns) * scale, with the FP64 phase reduced before the conversion.
template <typename R>
__device__ inline typename Cx<R>::T phasor_m2pi(double turns, R scale) {
  const double r = turns - rint(turns);
  R s, c;
  sincospi_t(static_cast<R>(2.0 * r), &s, &c);
  return {c * scale, -s * scale};
}

// First divided difference of -exp(jx) at nodes given in turns X, Y:
// -j exp(j pi (X + Y)) sinc(pi (Y - X)).
template <typename R>
__device__ inline typename Cx<R>::T first_dd(double X, double Y) {
  const double S = X + Y;
  const double D = Y - X;
  R cs, sn;
  sincospi_t(static_cast<R>(S - 2.0 * rint(0.5 * S)), &sn, &cs);
  R sc = R(1);
  if (D != 0.0) {
    R s_d, c_d;
    sincospi_t(static_cast<R>(D - 2.0 * rint(0.5 * D)), &s_d, &c_d);
    sc = s_d / static_cast<R>(kPi * D);
  }
  return {sn * sc, -cs * sc};
}

// Phi(a0, a1, a2): second divided difference of -exp(jx); nodes in turns (a = 2 pi A).
template <typename R>
__device__ typename Cx<R>::T phi_turns(double A0, double A1, double A2) {
  using C = typename Cx<R>::T;
  const double mean = (A0 + A1 + A2) / 3.0;
  const double B0 = A0 - mean, B1 = A1 - mean, B2 = A2 - mean;
  const double g12 = fabs(B1 - B2), g02 = fabs(B0 - B2), g01 = fabs(B0 - B1);
  double Bl, Bi, Bj, gmax;
  if (g12 >= g02 && g12 >= g01) {
    Bl = B0; Bi = B1; Bj = B2; gmax = g12;
  } else if (g02 >= g01) {
    Bl = B1; Bi = B0; Bj = B2; gmax = g02;
  } else {
    Bl = B2; Bi = B0; Bj = B1; gmax = g01;
  }
  C phi0;
  if (2.0 * kPi * gmax < kSeriesGap) {
    // Taylor series about the mean: sum_n j^n h_n(b) / (n+2)!, h_n by the
    // recurrence h_n = e1 h_{n-1} - e2 h_{n-2} + e3 h_{n-3}.
    const R b0 = static_cast<R>(2.0 * kPi * B0);
    const R b1 = static_cast<R>(2.0 * kPi * B1);
    const R b2 = static_cast<R>(2.0 * kPi * B2);
    const R e1 = b0 + b1 + b2, e2 = b0 * b1 + b0 * b2 + b1 * b2, e3 = b0 * b1 * b2;
    R hm3 = 0, hm2 = 0, hm1 = 1;  // h_{n-3}, h_{n-2}, h_{n-1} with h_0 = 1
    R re = R(0.5), im = 0;        // n = 0 term: 1/2!
    R inv_fact = R(0.5);
    for (int n = 1; n <= EchoTraits<R>::kSeriesTerms; ++n) {
      const R h = e1 * hm1 - e2 * hm2 + e3 * hm3;
      hm3 = hm2;
      hm2 = hm1;
      hm1 = h;
      inv_fact = inv_fact / static_cast<R>(n + 2);
      const R term = h * inv_fact;
      switch (n & 3) {  // j^n
        case 0: re += term; break;
        case 1: im += term; break;
        case 2: re -= term; break;
        default: im -= term; break;
      }
    }
    phi0 = {re, im};
  } else {
    const C fj = first_dd<R>(Bl, Bj);
    const C fi = first_dd<R>(Bl, Bi);
    const R inv = static_cast<R>(1.0 / (2.0 * kPi * (Bj - Bi)));
    phi0 = {(fj.x - fi.x) * inv, (fj.y - fi.y) * inv};
  }
  // shift back by the mean: Phi(a) = exp(j mean) Phi(a - mean)
  R ms, mc;
  const double mr = mean - rint(mean);
  sincospi_t(static_cast<R>(2.0 * mr), &ms, &mc);
  return {phi0.x * mc - phi0.y * ms, phi0.x * ms + phi0.y * mc};
}

// FP32 path: the facet integral G_f(m) over one sample tile, with every phase reduced
// in FP64 at the tile's first sample and advanced linearly in FP32 from there (the
// spatial frequency s_m = f_m / c is linear in m, and so is every argument of Phi).
// Nodes l, i, j as in phi_turns: (i, j) spans the widest gap. With nodes taken about
// the centroid, the divided-difference form reads
//   Phi = (f_j - f_i) / (2 pi s (b_j - b_i)),
//   f_k = -j exp(j pi s (b_l + b_k)) sinc(pi s (b_k - b_l)),
// and below the series gap the Taylor series about the mean applies as in phi_turns.
struct alignas(16) GLin {
  float gap, gap_i;          // rad: 2 pi s g_max (series below kSeriesGap)
  float p1, p1_i, p2, p2_i;  // turns: s (b_l + b_j) / 2, s (b_l + b_i) / 2
  float t1, t1_i, t2, t2_i;  // turns: s (b_j - b_l) / 2, s (b_i - b_l) / 2
  float x1, x1_i, x2, x2_i;  // rad: pi s (b_j - b_l), pi s (b_i - b_l)
  float w, w_i;              // rad: 2 pi s (b_j - b_i)
  float b0, b0_i, b1, b1_i, b2, b2_i;  // rad: 2 pi s (b_k - mean)
  float mp, mp_i;            // turns: s mean
  float ar, ai;              // G = (ar + j ai) Phi
  float k, k_i;              // rad per metre: 2 pi s (k_m of the wavenumber)
  float quad;                // turns per sample^2 of the delay's motion within a chirp
  int32_t valid;
  int32_t nl, ni, nj;  // vertex index of node l, i, j
};

__device__ inline float centred_turns(double t) { return static_cast<float>(t - rint(t)); }

// Coefficients for samples m = m_tile0 + j of the facet with geometry g.
__device__ inline void make_glin(const Geo &g, const RadarConst &rc, int m_tile0, GLin &q) {
  q.valid = g.valid;
  if (!g.valid) return;
  const double inv_c = 1.0 / kC0;
  const double s0 = (rc.f0 + static_cast<double>(m_tile0) * rc.df) * inv_c;
  const double ds = rc.df * inv_c;
  const double mean = (g.beta[0] + g.beta[1] + g.beta[2]) * (1.0 / 3.0);
  const double B0 = g.beta[0] - mean, B1 = g.beta[1] - mean, B2 = g.beta[2] - mean;
  const double g12 = fabs(B1 - B2), g02 = fabs(B0 - B2), g01 = fabs(B0 - B1);
  double bl, bi, bj, gmax;
  if (g12 >= g02 && g12 >= g01) {
    bl = B0; bi = B1; bj = B2; gmax = g12;
    q.nl = 0; q.ni = 1; q.nj = 2;
  } else if (g02 >= g01) {
    bl = B1; bi = B0; bj = B2; gmax = g02;
    q.nl = 1; q.ni = 0; q.nj = 2;
  } else {
    bl = B2; bi = B0; bj = B1; gmax = g01;
    q.nl = 2; q.ni = 0; q.nj = 1;
  }
  const double two_pi = 2.0 * kPi;
  q.gap = static_cast<float>(two_pi * s0 * gmax);
  q.gap_i = static_cast<float>(two_pi * ds * gmax);
  // the sinc form on absolute nodes b + mean, so no separate mean phase
  const double S1 = 0.5 * (bl + bj) + mean, S2 = 0.5 * (bl + bi) + mean;
  q.p1 = centred_turns(s0 * S1);
  q.p1_i = static_cast<float>(ds * S1);
  q.p2 = centred_turns(s0 * S2);
  q.p2_i = static_cast<float>(ds * S2);
  const double d1 = bj - bl, d2 = bi - bl;
  q.t1 = centred_turns(0.5 * s0 * d1);
  q.t1_i = static_cast<float>(0.5 * ds * d1);
  q.t2 = centred_turns(0.5 * s0 * d2);
  q.t2_i = static_cast<float>(0.5 * ds * d2);
  q.x1 = static_cast<float>(kPi * s0 * d1);
  q.x1_i = static_cast<float>(kPi * ds * d1);
  q.x2 = static_cast<float>(kPi * s0 * d2);
  q.x2_i = static_cast<float>(kPi * ds * d2);
  q.w = static_cast<float>(two_pi * s0 * (bj - bi));
  q.w_i = static_cast<float>(two_pi * ds * (bj - bi));
  q.b0 = static_cast<float>(two_pi * s0 * B0);
  q.b0_i = static_cast<float>(two_pi * ds * B0);
  q.b1 = static_cast<float>(two_pi * s0 * B1);
  q.b1_i = static_cast<float>(two_pi * ds * B1);
  q.b2 = static_cast<float>(two_pi * s0 * B2);
  q.b2_i = static_cast<float>(two_pi * ds * B2);
  q.mp = centred_turns(s0 * mean);
  q.mp_i = static_cast<float>(ds * mean);
  q.ar = static_cast<float>(g.amp_re);
  q.ai = static_cast<float>(g.amp_im);
  q.k = static_cast<float>(two_pi * s0);
  q.k_i = static_cast<float>(two_pi * ds);
  q.quad = 0.0f;
}

// sin(x) / x for x = x0 + j x_i (rad), t = t0 + j t_i = x / (2 pi) (turns, centred at
// j = 0). Below |x| = 0.3 the even series to x^8 (truncation < x^10 / 4e7); above, the
// hardware sine (absolute error ~1.3e-7) over x, relative error <= 4.4e-7.
constexpr float kSincSeries = 0.3f;

__device__ inline float sinc_series(float x2) {
  return fmaf(x2, fmaf(x2, fmaf(x2, fmaf(x2, 1.0f / 362880.0f, -1.0f / 5040.0f), 1.0f / 120.0f),
                       -1.0f / 6.0f), 1.0f);
}

__device__ inline float sinc_lin(float x0, float x_i, float t0, float t_i, float jf) {
  const float x = fmaf(jf, x_i, x0);
  if (fabsf(x) < kSincSeries) return sinc_series(x * x);
  float t = fmaf(jf, t_i, t0);
  t -= rintf(t);
  return __builtin_amdgcn_sinf(t) * __builtin_amdgcn_rcpf(x);
}

// G_f(m_tile0 + j)
__device__ inline float2 g_lin(const GLin &q, int j) {
  if (!q.valid) return {0.0f, 0.0f};
  const float jf = static_cast<float>(j);
  float2 phi;
  if (fmaf(jf, q.gap_i, q.gap) < static_cast<float>(kSeriesGap)) {
    const float b0 = fmaf(jf, q.b0_i, q.b0), b1 = fmaf(jf, q.b1_i, q.b1),
                b2 = fmaf(jf, q.b2_i, q.b2);
    const float e1 = b0 + b1 + b2, e2 = b0 * b1 + b0 * b2 + b1 * b2, e3 = b0 * b1 * b2;
    float hm3 = 0.0f, hm2 = 0.0f, hm1 = 1.0f;
    float re = 0.5f, im = 0.0f, inv_fact = 0.5f;
#pragma unroll
    for (int n = 1; n <= EchoTraits<float>::kSeriesTerms; ++n) {
      const float h = e1 * hm1 - e2 * hm2 + e3 * hm3;
      hm3 = hm2;
      hm2 = hm1;
      hm1 = h;
      inv_fact = inv_fact / static_cast<float>(n + 2);
      const float term = h * inv_fact;
      switch (n & 3) {
        case 0: re += term; break;
        case 1: im += term; break;
        case 2: re -= term; break;
        default: im -= term; break;
      }
    }
    float t = fmaf(jf, q.mp_i, q.mp);
    t -= rintf(t);
    const float ms = __builtin_amdgcn_sinf(t), mc = __builtin_amdgcn_cosf(t);
    phi = {re * mc - im * ms, re * ms + im * mc};
  } else {
    float t1 = fmaf(jf, q.p1_i, q.p1);
    t1 -= rintf(t1);
    float t2 = fmaf(jf, q.p2_i, q.p2);
    t2 -= rintf(t2);
    const float sc1 = sinc_lin(q.x1, q.x1_i, q.t1, q.t1_i, jf);
    const float sc2 = sinc_lin(q.x2, q.x2_i, q.t2, q.t2_i, jf);
    const float inv = __builtin_amdgcn_rcpf(fmaf(jf, q.w_i, q.w));
    // f_k = -j exp(j 2 pi t_k) sinc_k = (sin, -cos) sinc_k
    const float s1 = __builtin_amdgcn_sinf(t1) * sc1, c1 = __builtin_amdgcn_cosf(t1) * sc1;
    const float s2 = __builtin_amdgcn_sinf(t2) * sc2, c2 = __builtin_amdgcn_cosf(t2) * sc2;
    phi = {(s1 - s2) * inv, (c2 - c1) * inv};
  }
  return {q.ar * phi.x - q.ai * phi.y, q.ar * phi.y + q.ai * phi.x};
}

// Delay of element `el` from the facet centroid moved to sample time t_n + m / fs.
__device__ inline double moving_delay(const Geo &g, const double *el, double t) {
  const double dx = el[0] - (g.c[0] + g.vel[0] * t);
  const double dy = el[1] - (g.c[1] + g.vel[1] * t);
  const double dz = el[2] - (g.c[2] + g.vel[2] * t);
  return sqrt(dx * dx + dy * dy + dz * dz) * (1.0 / kC0);
}

// Element part of the phase (turns, unreduced) at sample m with the delay taken at the
// sample time: f_m tau - slope tau^2 / 2 - slope tau_ref,other (tau - tau_ref,self)
// - slope tau_ref,t tau_ref,r / 2, the same split as the stop-and-hop phases.
__device__ inline double element_phase(const Geo &g, const RadarConst &rc, const double *el,
                                       bool tx, int m) {
  const double tau = moving_delay(g, el, m / rc.fs);
  const double fm = rc.f0 + m * rc.df;
  const double d = tau - (tx ? g.tref_t : g.tref_r);
  return fm * tau - 0.5 * rc.slope * tau * tau - rc.slope * (tx ? g.tref_r : g.tref_t) * d -
         0.5 * rc.slope * g.tref_t * g.tref_r;
}

// Quadratic coefficient (turns per sample^2) of the phase-centre path's phase
// f_m tau - slope tau^2 / 2 with the delay at the sample time, from a second difference
// over one block: the phase leaves the chord of a block by q j (j - MB).
__device__ inline double chord_curvature(const Geo &g, const RadarConst &rc, int m0, int mb) {
  const int h = mb / 2;
  double ph[3];
  for (int k = 0; k < 3; ++k) {
    const int m = m0 + k * h;
    const double t = m / rc.fs;
    const double tau = moving_delay(g, rc.tx_c, t) + moving_delay(g, rc.rx_c, t);
    ph[k] = (rc.f0 + m * rc.df) * tau - 0.5 * rc.slope * tau * tau;
  }
  return (ph[2] - 2.0 * ph[1] + ph[0]) / (2.0 * h * h);
}

__device__ inline int find_inst(const DevInstance *inst, int n_inst, int64_t f) {
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

// FP64 geometry of work entry `item` of chirp n (lit facet, or point after them).
__device__ void entry_geometry(const DevScene &sc, const RadarConst &rc, int n, int32_t cnt,
                               int32_t item, Geo &g) {
  const double t = n * rc.tc;
  const double inv_c = 1.0 / kC0;
  double c[3];
  if (item < cnt) {
    const int64_t f = sc.vis_idx[static_cast<int64_t>(n) * sc.n_facets + item];
    const int ii = find_inst(sc.inst, sc.n_inst, f);
    const DevInstance &I = sc.inst[ii];
    const int64_t lt = f - I.facet_base;
    double x[3][3];
    for (int v = 0; v < 3; ++v) {
      const int32_t vi = I.tris[3 * lt + v];
      const double b0 = I.verts[3 * vi + 0], b1 = I.verts[3 * vi + 1], b2 = I.verts[3 * vi + 2];
      for (int k = 0; k < 3; ++k)
        x[v][k] = I.rot[3 * k + 0] * b0 + I.rot[3 * k + 1] * b1 + I.rot[3 * k + 2] * b2 +
                  (I.pos0[k] + I.vel[k] * t);
    }
    double e1[3], e2[3];
    for (int k = 0; k < 3; ++k) {
      c[k] = (x[0][k] + x[1][k] + x[2][k]) * (1.0 / 3.0);
      e1[k] = x[1][k] - x[0][k];
      e2[k] = x[2][k] - x[0][k];
    }
    double nv[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                    e1[0] * e2[1] - e1[1] * e2[0]};
    const double two_area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
    double ut[3], ur[3];
    for (int k = 0; k < 3; ++k) {
      ut[k] = rc.tx_c[k] - c[k];
      ur[k] = rc.rx_c[k] - c[k];
    }
    const double rt = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
    const double rr = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
    const double irt = 1.0 / rt, irr = 1.0 / rr;
    double w[3];
    for (int k = 0; k < 3; ++k) w[k] = ut[k] * irt + ur[k] * irr;
    // o = n . w / 2 with n = nv / |nv|; G = j o A Phi / (2 pi), A = |nv| / 2, so
    // o A = (nv . w) / 4 and no division by the area is needed
    const double nw = nv[0] * w[0] + nv[1] * w[1] + nv[2] * w[2];
    for (int v = 0; v < 3; ++v)
      g.beta[v] = w[0] * (x[v][0] - c[0]) + w[1] * (x[v][1] - c[1]) + w[2] * (x[v][2] - c[2]);
    g.amp_re = 0.0;
    g.amp_im = two_area > 0.0 ? nw * (0.25 / (2.0 * kPi)) : 0.0;
    g.tref_t = rt * inv_c;
    g.tref_r = rr * inv_c;
    for (int k = 0; k < 3; ++k) g.vel[k] = I.vel[k];
    g.valid = two_area > 0.0;
  } else {
    const int32_t k = item - cnt;
    for (int d = 0; d < 3; ++d) c[d] = sc.pt_pos0[3 * k + d] + sc.pt_vel[3 * k + d] * t;
    double ut[3], ur[3];
    for (int d = 0; d < 3; ++d) {
      ut[d] = rc.tx_c[d] - c[d];
      ur[d] = rc.rx_c[d] - c[d];
    }
    g.tref_t = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]) * inv_c;
    g.tref_r = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]) * inv_c;
    g.beta[0] = g.beta[1] = g.beta[2] = 0.0;
    // Phi(0,0,0) = 1/2, so G = s / (4 pi) with amp = s / (2 pi)
    g.amp_re = sc.pt_amp[2 * k + 0] / (2.0 * kPi);
    g.amp_im = sc.pt_amp[2 * k + 1] / (2.0 * kPi);
    for (int d = 0; d < 3; ++d) g.vel[d] = sc.pt_vel[3 * k + d];
    g.valid = 1;
  }
  g.c[0] = c[0];
  g.c[1] = c[1];
  g.c[2] = c[2];
}

}  // namespace rsim
