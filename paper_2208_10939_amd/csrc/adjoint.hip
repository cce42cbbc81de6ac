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
// The adjoint facet-sum kernel forms these sums (21 VALU ops per evaluation) and
// reduces them over its channels with wave shuffles in a fixed order; a second
// kernel applies the FP64 chain rule from (o, A, b, centroid) to the three world
// vertices; a third gathers per-vertex gradients through a vertex -> (triangle,
// corner) index, rotates them to the body frame and sums t_n-weighted gradients into
// the velocity gradient. No floating-point atomics: results are deterministic.
#include "echo_common.h"

namespace rsim {

namespace {

constexpr int kAdjVals = 8;  // grad_c (3), sum Re y, t0, t1, t2, pad

// sinc(u) = sin u / u and its derivative (cos u - sinc u) / u at u = pi D, D in turns
// (FP64, reduced before the FP32 trigonometry).
__device__ inline float sinc_d(double D, float *sinc_out) {
  const float u = static_cast<float>(kPi * D);
  const float au = fabsf(u);
  if (au < 0.05f) {
    const float u2 = u * u;
    *sinc_out = 1.0f - u2 * (1.0f / 6.0f) + u2 * u2 * (1.0f / 120.0f);
    return u * (-1.0f / 3.0f + u2 * (1.0f / 30.0f - u2 * (1.0f / 840.0f)));
  }
  float s, c;
  sincospi_t(static_cast<float>(D - 2.0 * rint(0.5 * D)), &s, &c);
  const float sc = s / u;
  *sinc_out = sc;
  return (c - sc) / u;
}

// Phi(a0,a1,a2) and dPhi/da_i (a in radians, given in turns A), FP32 results.
__device__ void phi_grad_turns(double A0, double A1, double A2, float2 *phi, float2 dphi[3]) {
  const double mean = (A0 + A1 + A2) / 3.0;
  const double B[3] = {A0 - mean, A1 - mean, A2 - mean};
  const double g12 = fabs(B[1] - B[2]), g02 = fabs(B[0] - B[2]), g01 = fabs(B[0] - B[1]);
  int l, i, j;
  double gmax;
  if (g12 >= g02 && g12 >= g01) {
    l = 0; i = 1; j = 2; gmax = g12;
  } else if (g02 >= g01) {
    l = 1; i = 0; j = 2; gmax = g02;
  } else {
    l = 2; i = 0; j = 1; gmax = g01;
  }
  float2 p0, d[3];
  if (2.0 * kPi * gmax < kSeriesGap) {
    // Phi_0 = sum_n j^n h_n(b)/(n+2)!,  dPhi_0/db_k = sum_n j^{n+1} h_n(b, b_k)/(n+3)!
    const float b0 = static_cast<float>(2.0 * kPi * B[0]);
    const float b1 = static_cast<float>(2.0 * kPi * B[1]);
    const float b2 = static_cast<float>(2.0 * kPi * B[2]);
    const float bk[3] = {b0, b1, b2};
    const float e1 = b0 + b1 + b2, e2 = b0 * b1 + b0 * b2 + b1 * b2, e3 = b0 * b1 * b2;
    float h[10];
    h[0] = 1.0f;
    float hm1 = 1.0f, hm2 = 0.0f, hm3 = 0.0f;
    for (int n = 1; n < 10; ++n) {
      const float hn = e1 * hm1 - e2 * hm2 + e3 * hm3;
      hm3 = hm2;
      hm2 = hm1;
      hm1 = hn;
      h[n] = hn;
    }
    float re = 0.0f, im = 0.0f, fact = 2.0f;  // (n+2)!
    for (int n = 0; n <= 8; ++n) {
      if (n > 0) fact *= static_cast<float>(n + 2);
      const float term = h[n] / fact;
      switch (n & 3) {
        case 0: re += term; break;
        case 1: im += term; break;
        case 2: re -= term; break;
        default: im -= term; break;
      }
    }
    p0 = make_float2(re, im);
    for (int k = 0; k < 3; ++k) {
      float h4 = 1.0f, dre = 0.0f, dim = 0.0f, f3 = 6.0f;  // (n+3)!
      for (int n = 0; n <= 7; ++n) {
        if (n > 0) {
          h4 = h[n] + bk[k] * h4;
          f3 *= static_cast<float>(n + 3);
        }
        const float term = h4 / f3;
        switch ((n + 1) & 3) {  // j^{n+1}
          case 0: dre += term; break;
          case 1: dim += term; break;
          case 2: dre -= term; break;
          default: dim -= term; break;
        }
      }
      d[k] = make_float2(dre, dim);
    }
  } else {
    // divided-difference form: Phi_0 = (F(b_l, b_j) - F(b_l, b_i)) / (b_j - b_i),
    // F(x, y) = -j exp(j (x+y)/2) sinc((y-x)/2)
    float2 F[2], Fx[2], Fy[2];
    const int other[2] = {j, i};
    for (int k = 0; k < 2; ++k) {
      const double X = B[l], Y = B[other[k]];
      const double S = X + Y;
      float cs, sn;
      sincospi_t(static_cast<float>(S - 2.0 * rint(0.5 * S)), &sn, &cs);
      float sc;
      const float scd = sinc_d(Y - X, &sc);
      // K = -j exp(js) = (sn, -cs)
      F[k] = make_float2(sn * sc, -cs * sc);
      // dF/dx = K (-sinc'/2 + j sinc/2),  dF/dy = K (sinc'/2 + j sinc/2)
      const float ax = -0.5f * scd, bx = 0.5f * sc;
      const float ay = 0.5f * scd, by = 0.5f * sc;
      Fx[k] = make_float2(sn * ax + cs * bx, sn * bx - cs * ax);
      Fy[k] = make_float2(sn * ay + cs * by, sn * by - cs * ay);
    }
    const float inv = static_cast<float>(1.0 / (2.0 * kPi * (B[j] - B[i])));
    p0 = make_float2((F[0].x - F[1].x) * inv, (F[0].y - F[1].y) * inv);
    d[l] = make_float2((Fx[0].x - Fx[1].x) * inv, (Fx[0].y - Fx[1].y) * inv);
    d[j] = make_float2((Fy[0].x - p0.x) * inv, (Fy[0].y - p0.y) * inv);
    d[i] = make_float2((p0.x - Fy[1].x) * inv, (p0.y - Fy[1].y) * inv);
  }
  float ms, mc;
  sincospi_t(static_cast<float>(2.0 * (mean - rint(mean))), &ms, &mc);
  *phi = make_float2(p0.x * mc - p0.y * ms, p0.x * ms + p0.y * mc);
  for (int k = 0; k < 3; ++k)
    dphi[k] = make_float2(d[k].x * mc - d[k].y * ms, d[k].x * ms + d[k].y * mc);
}

struct AdjShape {
  EchoShape sh;
  int32_t F;  // facets of the scene (capacity of a chirp's lit list)
  int32_t pad;
};

template <int MB, int FT>
struct AdjSmem {
  double *elem;  // [E][3]
  Geo *geo;      // [FT]
  float4 *GD;    // [FT][M_t][2]: (G, D0), (D1, D2)
  float2 *U;     // [FT][E][B_w]
  float2 *rat;   // [FT][E]
  float *off;    // [FT][E]
  float4 *er;    // [FT][E]: unit vector centroid -> element (xyz), 1 / R (w)
  float *tau;    // [FT][E]
  float *red;    // [FT][waves][kAdjVals]

  __device__ void carve(unsigned char *base, const EchoShape &sh, int waves) {
    size_t b = 0;
    auto take = [&](size_t bytes) {
      b = (b + 15) & ~size_t(15);
      unsigned char *p = base + b;
      b += bytes;
      return p;
    };
    elem = reinterpret_cast<double *>(take(sizeof(double) * 3 * sh.E));
    geo = reinterpret_cast<Geo *>(take(sizeof(Geo) * FT));
    GD = reinterpret_cast<float4 *>(take(sizeof(float4) * FT * 2 * sh.M_t));
    U = reinterpret_cast<float2 *>(take(sizeof(float2) * FT * sh.E * sh.B_w));
    rat = reinterpret_cast<float2 *>(take(sizeof(float2) * FT * sh.E));
    off = reinterpret_cast<float *>(take(sizeof(float) * FT * sh.E));
    er = reinterpret_cast<float4 *>(take(sizeof(float4) * FT * sh.E));
    tau = reinterpret_cast<float *>(take(sizeof(float) * FT * sh.E));
    red = reinterpret_cast<float *>(take(sizeof(float) * FT * waves * kAdjVals));
  }
  static size_t bytes(const EchoShape &sh, int waves) {
    size_t b = 0;
    auto take = [&](size_t bytes) {
      b = (b + 15) & ~size_t(15);
      b += bytes;
    };
    take(sizeof(double) * 3 * sh.E);
    take(sizeof(Geo) * FT);
    take(sizeof(float4) * FT * 2 * sh.M_t);
    take(sizeof(float2) * FT * sh.E * sh.B_w);
    take(sizeof(float2) * FT * sh.E);
    take(sizeof(float) * FT * sh.E);
    take(sizeof(float4) * FT * sh.E);
    take(sizeof(float) * FT * sh.E);
    take(sizeof(float) * FT * waves * kAdjVals);
    return b;
  }
};

// Sum over the 64 lanes of a wave: DPP moves inside each 16-lane row (no LDS round
// trips), then the four row sums read out with readlane (the DPP row-broadcast
// controls do not exist on this GPU generation). Fixed order: deterministic.
template <int kCtrl, int kRowMask>
__device__ inline float dpp_add(float v) {
  const int t = __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, kRowMask, 0xF,
                                            false);
  return v + __builtin_bit_cast(float, t);
}

// DPP reads the registers of inactive lanes as they are, so it is used only when the
// workgroup is made of whole waves; partial waves take the permute path.
__device__ inline float wave_sum_partial(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

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

template <int MB, int FT>
__global__ void __launch_bounds__(512) adjoint_echo_kernel(DevScene sc, RadarConst rc,
                                                           const double *elem, AdjShape ash,
                                                           const float2 *grad_echo,
                                                           float *partial) {
  extern __shared__ __align__(16) unsigned char adj_smem[];
  const EchoShape &sh = ash.sh;
  const int waves = (blockDim.x + 63) / 64;
  const bool whole_waves = (blockDim.x & 63) == 0;
  AdjSmem<MB, FT> sm;
  sm.carve(adj_smem, sh, waves);
  const int tid = threadIdx.x, nthr = blockDim.x;
  for (int i = tid; i < 3 * sh.E; i += nthr) sm.elem[i] = elem[i];
  const int per_chirp = sh.m_tiles * sh.o_tiles;
  const int n = blockIdx.x / per_chirp;
  const int mt = (blockIdx.x % per_chirp) / sh.o_tiles;
  const int ot = blockIdx.x % sh.o_tiles;
  const int P = rc.P, Q = rc.Q, E = sh.E;
  const int ol = tid % sh.O_w, b = tid / sh.O_w;
  const int o = ot * sh.O_w + ol;
  const bool o_ok = o < sh.O;
  const int p = o_ok ? o / Q : 0, q = o_ok ? o % Q : 0;
  const int m_tile0 = mt * sh.M_t;
  const int m_base = m_tile0 + b * MB;
  const int32_t cnt = sc.vis_cnt[n];
  const double slope = rc.slope;
  const float kf0 = static_cast<float>(2.0 * kPi / kC0);

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

  for (int32_t t0 = 0; t0 < cnt; t0 += FT) {
    const int nf = min(FT, cnt - t0);
    __syncthreads();
    for (int i = tid; i < FT; i += nthr) {
      if (i < nf)
        entry_geometry(sc, rc, n, cnt, t0 + i, sm.geo[i]);
      else
        sm.geo[i].valid = 0;
    }
    __syncthreads();
    for (int task = tid; task < FT * E; task += nthr) {
      const int i = task / E, e = task % E;
      const Geo &g = sm.geo[i];
      float2 *Ue = sm.U + (i * E + e) * sh.B_w;
      if (!g.valid) {
        for (int bb = 0; bb < sh.B_w; ++bb) Ue[bb] = make_float2(0.0f, 0.0f);
        sm.rat[i * E + e] = make_float2(1.0f, 0.0f);
        sm.off[i * E + e] = 0.0f;
        sm.er[i * E + e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        sm.tau[i * E + e] = 0.0f;
        continue;
      }
      const double dx = sm.elem[3 * e + 0] - g.c[0];
      const double dy = sm.elem[3 * e + 1] - g.c[1];
      const double dz = sm.elem[3 * e + 2] - g.c[2];
      const double Rn = sqrt(dx * dx + dy * dy + dz * dz);
      const double tau = Rn / kC0;
      double psi0, offv;
      if (e < P) {
        const double d = tau - g.tref_t;
        psi0 = rc.f0 * tau - 0.5 * slope * tau * tau - slope * g.tref_r * d -
               0.5 * slope * g.tref_t * g.tref_r;
        offv = sh.two_pi_slope * d;
      } else {
        const double d = tau - g.tref_r;
        psi0 = rc.f0 * tau - 0.5 * slope * tau * tau - slope * g.tref_t * d -
               0.5 * slope * g.tref_t * g.tref_r;
        offv = d;
      }
      psi0 -= floor(psi0);
      double delta = rc.df * tau;
      delta -= floor(delta);
      const float inv_r = static_cast<float>(1.0 / Rn);
      for (int bb = 0; bb < sh.B_w; ++bb)
        Ue[bb] = phasor_m2pi<float>(psi0 + static_cast<double>(m_tile0 + bb * MB) * delta, inv_r);
      sm.rat[i * E + e] = phasor_m2pi<float>(delta, 1.0f);
      sm.off[i * E + e] = static_cast<float>(offv);
      sm.er[i * E + e] = make_float4(static_cast<float>(dx / Rn), static_cast<float>(dy / Rn),
                                     static_cast<float>(dz / Rn), inv_r);
      sm.tau[i * E + e] = static_cast<float>(tau);
    }
    for (int task = tid; task < FT * sh.M_t; task += nthr) {
      const int i = task / sh.M_t, j = task % sh.M_t;
      const Geo &g = sm.geo[i];
      float2 gv = make_float2(0.0f, 0.0f), dv[3] = {gv, gv, gv};
      if (g.valid) {
        const double fm = rc.f0 + static_cast<double>(m_tile0 + j) * rc.df;
        const double s = fm / kC0;
        float2 ph, dph[3];
        phi_grad_turns(s * g.beta[0], s * g.beta[1], s * g.beta[2], &ph, dph);
        const float ar = static_cast<float>(g.amp_re), ai = static_cast<float>(g.amp_im);
        gv = make_float2(ar * ph.x - ai * ph.y, ar * ph.y + ai * ph.x);
        const float km = static_cast<float>(2.0 * kPi * s);
        for (int k = 0; k < 3; ++k)
          dv[k] = make_float2(km * (ar * dph[k].x - ai * dph[k].y),
                              km * (ar * dph[k].y + ai * dph[k].x));
      }
      float4 *dst = sm.GD + (static_cast<int64_t>(i) * sh.M_t + j) * 2;
      dst[0] = make_float4(gv.x, gv.y, dv[0].x, dv[0].y);
      dst[1] = make_float4(dv[1].x, dv[1].y, dv[2].x, dv[2].y);
    }
    __syncthreads();
    for (int i = 0; i < nf; ++i) {
      float v[kAdjVals] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (o_ok) {
        const float2 up = sm.U[(i * E + p) * sh.B_w + b];
        const float2 uq = sm.U[(i * E + P + q) * sh.B_w + b];
        const float2 rp = sm.rat[i * E + p], rq = sm.rat[i * E + P + q];
        const float eps = sm.off[i * E + p] * sm.off[i * E + P + q];
        float2 z = make_float2(up.x * uq.x - up.y * uq.y, up.x * uq.y + up.y * uq.x);
        z = make_float2(z.x - eps * z.y, z.y + eps * z.x);
        const float2 r = make_float2(rp.x * rq.x - rp.y * rq.y, rp.x * rq.y + rp.y * rq.x);
        // per sample: (G, D0) and (D1, D2) as two 16-byte LDS reads, a block ahead
        const float4 *gd = sm.GD + (static_cast<int64_t>(i) * sh.M_t + b * MB) * 2;
        float s0 = 0.0f, s1 = 0.0f, s2 = 0.0f, a0 = 0.0f, a1 = 0.0f, a2 = 0.0f;
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
            const float yx = fma_r(g0.x, w.x, -g0.y * w.y);
            const float yy = fma_r(g0.x, w.y, g0.y * w.x);
            s0 += yx;
            s1 += yy;
            s2 = fma_r(static_cast<float>(m_base + j), yy, s2);
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
        // dL/dR_p and dL/dR_q of this channel, then onto the centroid: dR/dc = -e_hat
        const float tpq = sm.tau[i * E + p] + sm.tau[i * E + P + q];
        const float f0mu = static_cast<float>(rc.f0 - slope * static_cast<double>(tpq));
        const float kap = kf0 * (f0mu * s1 + static_cast<float>(rc.df) * s2);
        const float4 ep = sm.er[i * E + p], eq = sm.er[i * E + P + q];
        const float cp = kap - s0 * ep.w, cq = kap - s0 * eq.w;
        v[0] = -(cp * ep.x + cq * eq.x);
        v[1] = -(cp * ep.y + cq * eq.y);
        v[2] = -(cp * ep.z + cq * eq.z);
        v[3] = s0;
        v[4] = a0;
        v[5] = a1;
        v[6] = a2;
      }
      const int wv = tid >> 6;
#pragma unroll
      for (int k = 0; k < 7; ++k) {
        const float s = whole_waves ? wave_sum(v[k]) : wave_sum_partial(v[k]);
        if ((tid & 63) == 0) sm.red[(i * waves + wv) * kAdjVals + k] = s;
      }
    }
    __syncthreads();
    for (int task = tid; task < nf * 7; task += nthr) {
      const int i = task / 7, k = task % 7;
      float s = 0.0f;
      for (int wv = 0; wv < waves; ++wv) s += sm.red[(i * waves + wv) * kAdjVals + k];
      const int64_t slot = ((static_cast<int64_t>(n) * ash.F + t0 + i) * sh.m_tiles + mt) * sh.o_tiles + ot;
      partial[slot * kAdjVals + k] = s;
    }
  }
}

// Per lit (chirp, facet): sum the partials and apply the chain rule to the three
// world vertices (FP64). Writes gxw[(n F + f) * 9 + 3 corner + axis].
__global__ void __launch_bounds__(256) facet_grad_kernel(DevScene sc, RadarConst rc,
                                                         AdjShape ash, const float *partial,
                                                         float *gxw) {
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
    for (int k = 0; k < 3; ++k) out[3 * v + k] = static_cast<float>(gx[v][k]);
}

__global__ void fill_zero_kernel(float *p, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0.0f;
}

// One instance: per body vertex, gather sum over chirps and incident (triangle,
// corner) of the world gradients, rotate to the body frame and accumulate into gv;
// vpart[v] = sum_n t_n (world gradient of v at chirp n) for the velocity gradient.
__global__ void __launch_bounds__(256) vertex_gather_kernel(
    const float *gxw, int64_t n_facets, int N, double tc, const double *rot,
    int64_t facet_base, const int32_t *csr_off, const int32_t *csr_ent, int32_t n_verts,
    float *gv, double *vpart) {
  const int32_t v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_verts) return;
  double g[3] = {0, 0, 0}, gt[3] = {0, 0, 0};
  const int32_t b = csr_off[v], e = csr_off[v + 1];
  for (int n = 0; n < N; ++n) {
    double gn[3] = {0, 0, 0};
    for (int32_t k = b; k < e; ++k) {
      const int32_t ent = csr_ent[k];  // triangle * 3 + corner
      const float *src = gxw + (static_cast<int64_t>(n) * n_facets + facet_base + ent / 3) * 9 +
                         3 * (ent % 3);
      gn[0] += src[0];
      gn[1] += src[1];
      gn[2] += src[2];
    }
    const double tn = n * tc;
    for (int k = 0; k < 3; ++k) {
      g[k] += gn[k];
      gt[k] += tn * gn[k];
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

constexpr int kAdjMB = 32;
constexpr int kAdjFT = 16;

size_t adjoint_partial_floats(const EchoShape &sh, int64_t N, int64_t F) {
  return static_cast<size_t>(N) * F * sh.m_tiles * sh.o_tiles * kAdjVals;
}

int adjoint_tile_m() { return kAdjMB; }

size_t adjoint_smem_bytes(const EchoShape &sh) {
  const int waves = (sh.O_w * sh.B_w + 63) / 64;
  return AdjSmem<kAdjMB, kAdjFT>::bytes(sh, waves);
}

hipError_t launch_adjoint(const DevScene &sc, const RadarConst &rc, const double *elem,
                          const EchoShape &sh, const void *grad_echo, float *partial, float *gxw,
                          hipStream_t s) {
  AdjShape ash{sh, static_cast<int32_t>(sc.n_facets), 0};
  const int threads = sh.O_w * sh.B_w;
  const int64_t gx_n = static_cast<int64_t>(rc.N) * sc.n_facets * 9;
  hipLaunchKernelGGL(fill_zero_kernel, dim3(1024), dim3(256), 0, s, gxw, gx_n);
  if (sc.n_facets == 0) return hipGetLastError();
  const unsigned grid = static_cast<unsigned>(rc.N) * sh.m_tiles * sh.o_tiles;
  hipLaunchKernelGGL((adjoint_echo_kernel<kAdjMB, kAdjFT>), dim3(grid), dim3(threads),
                     adjoint_smem_bytes(sh), s, sc, rc, elem, ash,
                     static_cast<const float2 *>(grad_echo), partial);
  dim3 g2(static_cast<unsigned>((sc.n_facets + 255) / 256), rc.N);
  hipLaunchKernelGGL(facet_grad_kernel, g2, dim3(256), 0, s, sc, rc, ash, partial, gxw);
  return hipGetLastError();
}

hipError_t launch_vertex_gather(const float *gxw, int64_t n_facets, int N, double tc,
                                const double *rot_dev, int64_t facet_base, const int32_t *csr_off,
                                const int32_t *csr_ent, int32_t n_verts, float *gv, double *vpart,
                                double *vel_out, hipStream_t s) {
  if (n_verts > 0) {
    hipLaunchKernelGGL(vertex_gather_kernel, dim3((n_verts + 255) / 256), dim3(256), 0, s, gxw,
                       n_facets, N, tc, rot_dev, facet_base, csr_off, csr_ent, n_verts, gv, vpart);
  }
  hipLaunchKernelGGL(velocity_reduce_kernel, dim3(1), dim3(256), 0, s, vpart, n_verts, vel_out);
  return hipGetLastError();
}

}  // namespace rsim
