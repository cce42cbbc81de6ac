// Facet sum as a type-1 non-uniform FFT over the sample index (stop-and-hop, FP32 with
// FP64 geometry and phases). Same result as the direct sum of Sections 2.2 and 3.2,
// eqs. (7)-(13), within the spread kernel's error.
//
// With the closed-form facet integral written as a divided difference, the term of a
// lit facet (or point) for channel (p, q) at sample m = m' + M/2 is
//   T(m) = -amp / (R_t R_r k_m^2) exp(-j 2 pi (f_c tau - mu tau^2 / 2))
//          DD2_beta[ exp(j k_c beta) exp(-j m' dk (L - beta)) ](beta_0, beta_1, beta_2),
// with L = R_t + R_r, tau = L / c, f_c = f0 + (M/2) df, k = 2 pi f / c, dk = 2 pi df / c
// and DD2 the second divided difference over the facet's node offsets beta_v. For every
// channel the sum over facets is therefore a type-1 transform of sources at path lengths
// L - beta onto the modes m'. Each source set is spread onto a periodic grid of n_g >= 2M
// cells with a Gaussian psi(x) = exp(-x^2 / (2 s^2)); the grid position of path length L
// is x = kappa L with kappa = df n_g / c cells per metre. Expanding psi(l - x_L + kappa
// beta) in beta turns the facet's spread into
//   Q(p, q) psi(l - x_L) sum_k b_k (l - x_L)^k,
//   b_k = -amp / (k_c^2 s^k) sum_{r >= k} D_r (-kappa / s)^r / r! He_{r,k},
//   D_r = DD2[beta^r exp(j k_c beta)] (Leibniz rule over the stable divided
//         differences of exp(j k_c beta); He_{r,k} the coefficients of He_r(y)),
// where only Q = exp(-j 2 pi (f_c tau - mu tau^2/2)) / (R_t R_r) and x_L depend on the
// channel. A forward FFT of each channel's grid then gives
//   H(m' + M/2) = U(m') k_c^2 / (k_m^2 psi_hat(2 pi m' / n_g)),
//   psi_hat(w) = s sqrt(2 pi) exp(-s^2 w^2 / 2).
//
// Channel (p, q) differs from the phase-centre path (centres t_c, r_c of the Tx and Rx
// elements) only through dL = (R_tp - R_tc) + (R_rq - R_rc), a few centimetres. With
// u the unit vector from t_c to the centroid, a = t_p - t_c and s = u.a, exactly
//   R_tp - R_tc = -s + e,   e (2 R_tc - 2 s + e) = |a|^2 - s^2 =: h,
// so e = h / D (1 - h / D^2 + ...) with D = 2 R_tc - 2 s (the next term is below
// e (h / D^2)^2). s is formed in FP64 and its phase g1 s reduced in FP64; e and the rest
// in FP32. The phase-centre path itself (delay, reduced phase, grid cell) is FP64, once
// per entry:
//   f_c tau - mu tau^2 / 2 = [same at tau_c] + dL g1 - mu dL^2 / (2 c^2),
//   g1 = (f_c - mu tau_c) / c.
//
// Five kernels per chunk of chirps:
//   key     per (chirp, lit facet or point): grid cell of the phase-centre path;
//   count   per chirp: counting sort by cell in LDS, giving each entry its position in
//           cell order (order within a cell is that of the LDS counter, so sums are
//           reproducible to FP32 rounding only);
//   prep    per entry: b_k and the phase-centre path (FP64 work, stored as FP32
//           offsets, reduced phase and grid cell), written at the sorted position;
//   spread  one wave per (chirp, 64 channels, run of kNuSeg sorted records): each lane
//           (channel) accumulates a window of kNuSlots cells in registers, with Gaussian
//           weights from a product recurrence, and adds it to the global grid
//           [chirp][channel][n_g] only when the sorted positions leave the window (and at
//           the end of the run);
//   fft     per (chirp, group of channels): grid rows into LDS (rows zeroed behind),
//           in-LDS Stockham FFT, deconvolution, echo samples.
#include <type_traits>

#include "adjoint_common.h"
#include "echo_common.h"
#include "fft_common.h"

namespace rsim {

constexpr int kNuFftThreads = 512;
constexpr int kNuMaxOrder = 10;
constexpr int kNuSeg = 256;    // sorted records per spread wave
constexpr int kNuSlots = 20;   // register window of grid cells per lane
constexpr int kNuSpreadThreads = 256;
constexpr int kNuGatherRecs = 256;  // records (lanes) per adjoint gather workgroup
constexpr int kXcds = 8;            // accelerator complex dies: workgroups go round-robin

template <int R>
struct alignas(16) NuRec {
  double ut[3], ur[3];  // unit vectors from t_c and r_c to the centroid c at t_n
  double g1;            // (f_c - mu tau_c) / c: turns per metre of dL
  float rt, rr;         // |c - t_c|, |c - r_c|
  float t0;             // f_c tau_c - mu tau_c^2 / 2 reduced to [-1/2, 1/2] turns
  float frac;           // grid position of the phase-centre path minus `cell`
  int32_t cell;         // its grid cell (0 .. n_g - 1)
  int32_t valid;
  float2 b[R];          // polynomial coefficients in grid cells (see the header comment)
};
// with the delay within the chirp: velocity, its components along ut and ur, and the
// phase-centre path's Doppler shift of the source (cells; included in cell and frac)
template <int R>
struct alignas(16) NuRecIntra : NuRec<R> {
  float v[3];
  float vut, vur;
  float dxc;
};
template <int R, bool INTRA>
using NuRecT = typename std::conditional<INTRA, NuRecIntra<R>, NuRec<R>>::type;
static_assert(sizeof(NuRec<5>) == 128 && sizeof(NuRec<7>) == 144 && sizeof(NuRec<10>) == 160,
              "record size");
// (the derived record reuses the base's tail padding: float2 is not plain old data)
static_assert(sizeof(NuRecIntra<5>) == 144 && sizeof(NuRecIntra<7>) == 160 &&
                  sizeof(NuRecIntra<10>) == 192,
              "record size");

// Adjoint record: derivatives of the Taylor coefficients and of the source position with
// respect to the facet's three node offsets, and the facet's index in the lit list.
template <int R>
struct alignas(16) NuDer {
  float2 db[3][R];  // d b_k / d beta_v (per metre)
  float dx[3];      // d x / d beta_v (cells per metre; nonzero for sub-triangles)
  int32_t item;
};
static_assert(sizeof(NuDer<5>) == 144 && sizeof(NuDer<7>) == 192 && sizeof(NuDer<10>) == 256,
              "adjoint record size");
static_assert(kAdjVals == kAdjSlotFloats, "adjoint slot layout");
constexpr double kNuDerStep = 1e-6;  // metres: central differences of b_k in beta (FP64)

size_t nufft_der_bytes(int order) {
  return order <= 5 ? sizeof(NuDer<5>) : order <= 7 ? sizeof(NuDer<7>) : sizeof(NuDer<10>);
}

template <bool INTRA>
static size_t record_bytes_t(int order) {
  return order <= 5 ? sizeof(NuRecT<5, INTRA>)
                    : order <= 7 ? sizeof(NuRecT<7, INTRA>) : sizeof(NuRecT<10, INTRA>);
}
size_t nufft_record_bytes(int order, bool intra) {
  return intra ? record_bytes_t<true>(order) : record_bytes_t<false>(order);
}
int nufft_window_cells() { return kNuSlots; }
int nufft_run_length() { return kNuSeg; }

// Probabilists' Hermite polynomials He_r(y) = sum_k kHe.c[r][k] y^k, from
// He_{r+1} = y He_r - r He_{r-1}.
struct HermiteTable {
  double c[kNuMaxOrder][kNuMaxOrder];
};
constexpr HermiteTable make_hermite() {
  HermiteTable t{};
  t.c[0][0] = 1.0;
  t.c[1][1] = 1.0;
  for (int r = 1; r + 1 < kNuMaxOrder; ++r)
    for (int k = 0; k < kNuMaxOrder; ++k)
      t.c[r + 1][k] = (k ? t.c[r][k - 1] : 0.0) - r * t.c[r - 1][k];
  return t;
}
constexpr HermiteTable kHe = make_hermite();

__device__ inline int wrap_cell(int64_t c, int ng) {
  const int64_t r = c % ng;
  return static_cast<int>(r < 0 ? r + ng : r);
}

// Grid position and cell (0 .. n_g - 1) of a source on the phase-centre path of an entry,
// shifted by the node offset bc of a sub-triangle's centroid (x = kappa (L - bc)), and the
// two distances of that path; FP64.
// With the delay taken at each sample time (rc.intra), the path's delay grows by
// tau' m / fs over the chirp (tau' = d tau / dt, first order; the second-order term is
// below 1e-7 of a turn here), which adds A m + B m^2 turns to its phase with
// A = (f0 - mu tau) tau' / fs and B = df tau' / fs. With m = m' + M/2 that is a constant
// phase A M/2 + B M^2/4, a shift of the source by (A + B M) n_g cells, and B m'^2.
__device__ inline double doppler_cells(const Geo &g, const RadarConst &rc, const NuShape &ns,
                                       double Rt, double Rr, double tau) {
  if (!rc.intra) return 0.0;
  double vt = 0.0, vr = 0.0;
  for (int k = 0; k < 3; ++k) {
    vt += g.vel[k] * (g.c[k] - rc.tx_c[k]);
    vr += g.vel[k] * (g.c[k] - rc.rx_c[k]);
  }
  const double tdot = (vt / Rt + vr / Rr) * (1.0 / kC0);
  const double A = (rc.f0 - rc.slope * tau) * tdot / rc.fs, B = rc.df * tdot / rc.fs;
  return (A + B * rc.M) * ns.ng;
}

__device__ inline void centre_cell(const Geo &g, const RadarConst &rc, const NuShape &ns,
                                   double bc, double *x_out, int *cell_out, double *Rt,
                                   double *Rr, double *dxc) {
  double dt = 0.0, dr = 0.0;
  for (int k = 0; k < 3; ++k) {
    dt += (g.c[k] - rc.tx_c[k]) * (g.c[k] - rc.tx_c[k]);
    dr += (g.c[k] - rc.rx_c[k]) * (g.c[k] - rc.rx_c[k]);
  }
  *Rt = sqrt(dt);
  *Rr = sqrt(dr);
  const double tau = (*Rt + *Rr) * (1.0 / kC0);
  *dxc = doppler_cells(g, rc, ns, *Rt, *Rr, tau);
  const double x = tau * ns.cells_per_s - ns.kappa * bc + *dxc;
  *x_out = x;
  *cell_out = wrap_cell(static_cast<int64_t>(floor(x)), ns.ng);
}

// Record `rec` of a chirp with `cnt` lit facets: facet records first (4^split per lit
// facet), then one per point. Returns the entry (lit facet or point) and the sub-triangle.
__device__ inline int32_t record_entry(int32_t rec, int32_t cnt, int split, int *sub) {
  const int32_t subs = 1 << (2 * split);
  if (rec < cnt * subs) {
    *sub = rec & (subs - 1);
    return rec >> (2 * split);
  }
  *sub = -1;  // a point: not split
  return cnt + (rec - cnt * subs);
}

// Node offsets of sub-triangle `sub` (base-4 digits, most significant first; each digit
// picks one of the four midpoint sub-triangles) of a facet with node offsets beta about its
// centroid: offsets are linear in position, so a midpoint's is the mean of its ends.
// Returns the offset of the sub-triangle's centroid; out[] = its nodes about that centroid.
__device__ inline double sub_nodes(const double beta[3], int sub, int split, double out[3]) {
  double p0 = beta[0], p1 = beta[1], p2 = beta[2];
  for (int l = split - 1; l >= 0; --l) {
    const int d = (sub >> (2 * l)) & 3;
    const double m01 = 0.5 * (p0 + p1), m12 = 0.5 * (p1 + p2), m20 = 0.5 * (p2 + p0);
    if (d == 0) {
      p1 = m01;
      p2 = m20;
    } else if (d == 1) {
      p0 = m01;
      p2 = m12;
    } else if (d == 2) {
      p0 = m20;
      p1 = m12;
    } else {
      p0 = m01;
      p1 = m12;
      p2 = m20;
    }
  }
  const double c = (p0 + p1 + p2) * (1.0 / 3.0);
  out[0] = p0 - c;
  out[1] = p1 - c;
  out[2] = p2 - c;
  return c;
}

// Taylor coefficients b_k (FP64) of one record: the facet with node offsets beta_f about
// its centroid, or its sub-triangle `sub` (own nodes about the sub-centroid, 4^-split of the
// area, the factor exp(j k_c bc)). Returns bc, the sub-centroid's offset (0 unsplit).
template <int R>
__device__ double taylor_coeffs(const Geo &g, const double beta_f[3], int sub,
                                const NuShape &ns, double br[R], double bi[R]) {
  double beta[3] = {beta_f[0], beta_f[1], beta_f[2]};
  double bc = 0.0;
  double amp_re = g.amp_re, amp_im = g.amp_im;
  if (sub >= 0 && ns.split > 0) {
    bc = sub_nodes(beta_f, sub, ns.split, beta);
    const double scale = 1.0 / static_cast<double>(1 << (2 * ns.split));
    double sb, cb;
    const double tb = ns.fc / kC0 * bc;
    sincospi_t(2.0 * (tb - rint(tb)), &sb, &cb);
    const double ar = amp_re * scale, ai = amp_im * scale;
    amp_re = ar * cb - ai * sb;
    amp_im = ar * sb + ai * cb;
  }
#pragma unroll
  for (int k = 0; k < R; ++k) br[k] = bi[k] = 0.0;
  if (!g.valid) return bc;
  const double turns_per_m = ns.fc / kC0;  // k_c / (2 pi)
  const double A0 = turns_per_m * beta[0], A1 = turns_per_m * beta[1],
               A2 = turns_per_m * beta[2];
  // divided differences of exp(j k_c beta) over beta, divided by k_c^2:
  // [b0,b1,b2] = -Phi, [b1,b2] = -F[a1,a2] / k_c, [b2] = exp(j k_c b2) / k_c^2
  // (Phi and F the second and first divided differences of -exp(jx) at a = k_c beta)
  const double2 phi = phi_turns<double>(A0, A1, A2);
  const double2 f12 = first_dd<double>(A1, A2);
  const double ik = 1.0 / ns.kc;
  double s2, c2;
  sincospi_t(2.0 * (A2 - rint(A2)), &s2, &c2);
  const double g2r = -phi.x, g2i = -phi.y;
  const double g1r = -f12.x * ik, g1i = -f12.y * ik;
  const double g0r = c2 * ik * ik, g0i = s2 * ik * ik;
  const double b0 = beta[0], b1 = beta[1], b2 = beta[2];
  const double e1 = b0 + b1 + b2, e2 = b0 * b1 + b0 * b2 + b1 * b2, e3 = b0 * b1 * b2;
  // a_r = D_r (-kappa / s)^r / r!, D_r = b0^r [b0,b1,b2] + h_{r-1}(b0,b1) [b1,b2]
  //                                      + h_{r-2}(b0,b1,b2) [b2]
  double ar[R], ai[R];
  double p0 = 1.0;                       // b0^r
  double q1m = 0.0, q1 = 0.0;            // h_{r-2}(b0,b1), h_{r-1}(b0,b1)
  double t3 = 0.0, t2 = 0.0, t1 = 0.0;   // h_{r-4}, h_{r-3}, h_{r-2} of (b0,b1,b2)
  double scale = 1.0;                    // (-kappa / s)^r / r!
  const double step = -ns.kappa / ns.sigma;
#pragma unroll
  for (int r = 0; r < R; ++r) {
    if (r >= 1) {
      p0 *= b0;
      const double qn = (r == 1) ? 1.0 : (b0 + b1) * q1 - b0 * b1 * q1m;
      q1m = q1;
      q1 = qn;
      scale *= step / r;
    }
    if (r >= 2) {
      const double tn = (r == 2) ? 1.0 : e1 * t1 - e2 * t2 + e3 * t3;
      t3 = t2;
      t2 = t1;
      t1 = tn;
    }
    const double dr = p0 * g2r + q1 * g1r + t1 * g0r;
    const double di = p0 * g2i + q1 * g1i + t1 * g0i;
    ar[r] = dr * scale;
    ai[r] = di * scale;
  }
  // b_k = -amp / s^k sum_{r >= k} a_r He_{r,k}
  double is_k = 1.0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    double sr = 0.0, si = 0.0;
#pragma unroll
    for (int r = k; r < R; ++r) {
      sr += ar[r] * kHe.c[r][k];
      si += ai[r] * kHe.c[r][k];
    }
    sr *= is_k;
    si *= is_k;
    is_k /= ns.sigma;
    br[k] = -(amp_re * sr - amp_im * si);
    bi[k] = -(amp_re * si + amp_im * sr);
  }
  return bc;
}

// The phase-centre path of a record (FP64): unit vectors, distances, reduced phase, the
// source's grid cell and fraction (the same cell as the key pass).
template <int R>
__device__ void path_fields(const Geo &g, const RadarConst &rc, const NuShape &ns, double bc,
                            NuRec<R> &out, double *Rt, double *Rr, double *dxc) {
  double x;
  int cell;
  centre_cell(g, rc, ns, bc, &x, &cell, Rt, Rr, dxc);
  for (int k = 0; k < 3; ++k) {
    out.ut[k] = (g.c[k] - rc.tx_c[k]) / *Rt;
    out.ur[k] = (g.c[k] - rc.rx_c[k]) / *Rr;
  }
  const double tau = (*Rt + *Rr) * (1.0 / kC0);
  const double turns = ns.fc * tau - 0.5 * rc.slope * tau * tau;
  out.rt = static_cast<float>(*Rt);
  out.rr = static_cast<float>(*Rr);
  out.t0 = static_cast<float>(turns - rint(turns));
  out.g1 = (ns.fc - rc.slope * tau) * (1.0 / kC0);
  out.frac = static_cast<float>(x - floor(x));
  out.cell = cell;
}

template <int R, bool INTRA>
__global__ void __launch_bounds__(256) nufft_prep_kernel(DevScene sc, RadarConst rc, NuShape ns,
                                                        NuBuffers nb) {
  const int nl = blockIdx.y;
  const int n = ns.n0 + nl;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t item = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (item >= (cnt << (2 * ns.split)) + sc.n_points) return;
  int sub;
  const int32_t entry = record_entry(item, cnt, ns.split, &sub);
  Geo g;
  entry_geometry(sc, rc, n, cnt, entry, g);
  NuRecT<R, INTRA> out;
  out.valid = g.valid;
  double br[R], bi[R];
  const double bc = taylor_coeffs<R>(g, g.beta, sub, ns, br, bi);
#pragma unroll
  for (int k = 0; k < R; ++k) out.b[k] = {static_cast<float>(br[k]), static_cast<float>(bi[k])};
  double Rt, Rr, dxc;
  path_fields(g, rc, ns, bc, out, &Rt, &Rr, &dxc);
  if constexpr (INTRA) {
    double vut = 0.0, vur = 0.0;
    for (int k = 0; k < 3; ++k) {
      out.v[k] = static_cast<float>(g.vel[k]);
      vut += g.vel[k] * (g.c[k] - rc.tx_c[k]) / Rt;
      vur += g.vel[k] * (g.c[k] - rc.rx_c[k]) / Rr;
    }
    out.vut = static_cast<float>(vut);
    out.vur = static_cast<float>(vur);
    out.dxc = static_cast<float>(dxc);
  }
  const int64_t row = static_cast<int64_t>(nl) * ns.rec_stride;
  static_cast<NuRecT<R, INTRA> *>(nb.srec)[row + nb.pos[row + item]] = out;
}

__global__ void __launch_bounds__(256) nufft_key_kernel(DevScene sc, RadarConst rc, NuShape ns,
                                                       NuBuffers nb) {
  const int nl = blockIdx.y;
  const int n = ns.n0 + nl;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t item = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (item >= (cnt << (2 * ns.split)) + sc.n_points) return;
  int sub;
  const int32_t entry = record_entry(item, cnt, ns.split, &sub);
  Geo g;
  entry_geometry(sc, rc, n, cnt, entry, g);
  double nodes[3], bc = 0.0;
  if (sub >= 0 && ns.split > 0) bc = sub_nodes(g.beta, sub, ns.split, nodes);
  double x, Rt, Rr, dxc;
  int cell;
  centre_cell(g, rc, ns, bc, &x, &cell, &Rt, &Rr, &dxc);
  nb.key[static_cast<int64_t>(nl) * ns.rec_stride + item] = cell;
}

// Per chirp: LDS counts per cell (the counter's old value is the rank within the cell),
// exclusive scan, then position = cell offset + rank.
__global__ void __launch_bounds__(1024) nufft_count_kernel(DevScene sc, NuShape ns, NuBuffers nb) {
  __shared__ int32_t s_cnt[2048];
  __shared__ int32_t s_part[1024];
  const int nl = blockIdx.x;
  const int n = ns.n0 + nl;
  const int64_t row = static_cast<int64_t>(nl) * ns.rec_stride;
  const int32_t *key = nb.key + row;
  int32_t *pos = nb.pos + row;
  const int32_t n_ent = (sc.vis_cnt[n] << (2 * ns.split)) + sc.n_points;
  __shared__ int32_t s_lo, s_hi;
  for (int c = threadIdx.x; c < 2048; c += blockDim.x) s_cnt[c] = 0;
  if (threadIdx.x == 0) {
    s_lo = ns.ng;
    s_hi = -1;
  }
  __syncthreads();
  for (int32_t e = threadIdx.x; e < n_ent; e += blockDim.x) pos[e] = atomicAdd(&s_cnt[key[e]], 1);
  __syncthreads();
  // occupied cells, widened by every cell a window flush can reach (channel offsets, the
  // Gaussian's half width and the fraction): the grid is zero outside; a wrapping interval
  // becomes the whole row
  {
    const int c0 = 2 * threadIdx.x;
    if (c0 < ns.ng && s_cnt[c0]) { atomicMin(&s_lo, c0); atomicMax(&s_hi, c0); }
    if (c0 + 1 < ns.ng && s_cnt[c0 + 1]) { atomicMin(&s_lo, c0 + 1); atomicMax(&s_hi, c0 + 1); }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int m = static_cast<int>(ceil(ns.chan_d)) + kNuWidth / 2 + 2;
    int lo = s_lo - m, hi = s_hi + m;
    if (s_hi < 0) {
      lo = 0;
      hi = -1;
    } else if (lo < 0 || hi >= ns.ng) {
      lo = 0;
      hi = ns.ng - 1;
    }
    nb.range[nl] = make_int2(lo, hi);
  }
  __syncthreads();
  // exclusive scan, two cells per thread (n_g <= 2048)
  const int c0 = 2 * threadIdx.x;
  const int32_t h0 = s_cnt[c0], h1 = s_cnt[c0 + 1];
  s_part[threadIdx.x] = h0 + h1;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const int32_t v = threadIdx.x >= static_cast<unsigned>(off) ? s_part[threadIdx.x - off] : 0;
    __syncthreads();
    s_part[threadIdx.x] += v;
    __syncthreads();
  }
  const int32_t base = s_part[threadIdx.x] - h0 - h1;
  s_cnt[c0] = base;
  s_cnt[c0 + 1] = base + h0;
  __syncthreads();
  for (int32_t e = threadIdx.x; e < n_ent; e += blockDim.x) pos[e] += s_cnt[key[e]];
}

template <int R, bool INTRA>
__global__ void __launch_bounds__(kNuSpreadThreads) nufft_spread_kernel(
    DevScene sc, RadarConst rc, NuShape ns, const double *elem,
    const NuRecT<R, INTRA> *__restrict__ sorted, float2 *__restrict__ grids) {
  const int wave = __builtin_amdgcn_readfirstlane(
      static_cast<int>(blockIdx.x) * (kNuSpreadThreads / 64) + static_cast<int>(threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  // item = (chirp, channel group, run); the runs of a chirp are consecutive
  const int runs = ns.runs;
  const int per_chirp = ns.spread_groups * runs;
  const int nl = wave / per_chirp;
  if (nl >= ns.n_chirps) return;
  const int rem = wave - nl * per_chirp;
  const int grp = rem / runs;
  const int run = rem - grp * runs;
  const int n = ns.n0 + nl;
  const int32_t n_ent = (sc.vis_cnt[n] << (2 * ns.split)) + sc.n_points;
  const int e_begin = run * kNuSeg;
  if (e_begin >= n_ent) return;
  const int e_end = min(n_ent, e_begin + kNuSeg);
  const int ng = ns.ng;
  const int O = rc.P * rc.Q;
  const int o = grp * 64 + lane;
  const bool on = o < O;
  // this lane's element offsets from the phase centres
  double at[3], ar[3];
  float aat, aar, atf[3], arf[3];
  {
    const int oc = on ? o : 0;
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
  const float inv_s4 = inv_s2 * inv_s2;
  const NuRecT<R, INTRA> *srec = sorted + static_cast<int64_t>(nl) * ns.rec_stride;
  float2 *grid = grids + (static_cast<int64_t>(nl) * O + (on ? o : 0)) * ng;
  const float nc = static_cast<float>(-1.4426950408889634 / (2.0 * ns.sigma * ns.sigma));
  const float q_ratio = __builtin_amdgcn_exp2f(2.0f * nc);  // exp(-1 / s^2)
  const float kappa = static_cast<float>(ns.kappa);
  const float g2 = static_cast<float>(0.5 * rc.slope / (kC0 * kC0));
  const float d = static_cast<float>(ns.chan_d);
  const int b0 = static_cast<int>(ceilf(d + 0.5f * kNuWidth));  // key offset after a rebase
  const float rel_hi = static_cast<float>(kNuSlots - 1) - d - 0.5f * kNuWidth;
  float2 acc[kNuSlots];
#pragma unroll
  for (int s = 0; s < kNuSlots; ++s) acc[s] = {0.0f, 0.0f};
  // windows: the records that fit one placement of the register window, then a flush;
  // invalid records carry zero coefficients and need no test
  int i = e_begin;
  NuRecT<R, INTRA> nxt = load_uniform(srec + i);
  while (i < e_end) {
    const int base = nxt.cell - b0;  // wave-uniform
    int used_lo = kNuSlots, used_hi = -1;
    const int first = i;
    for (; i < e_end; ++i) {
      const NuRecT<R, INTRA> r = nxt;
      // window position of the phase-centre path (wrapped cell difference + fraction);
      // the record that placed the window always fits it (chan_d <= 2.5 cells), and is
      // taken regardless so that every window makes progress
      int rk = r.cell - base;
      if (rk > ng / 2) rk -= ng;
      if (rk < -ng / 2) rk += ng;
      const float rel_c = static_cast<float>(rk) + r.frac;
      if (i > first && (rel_c < d + 0.5f * kNuWidth || rel_c > rel_hi)) break;
      if (i + 1 < e_end) nxt = load_uniform(srec + i + 1);
      // cells some channel reaches: |s - x_o| <= W/2 with |x_o - rel_c| <= d
      const int s_lo =
          __builtin_amdgcn_readfirstlane(static_cast<int>(ceilf(rel_c - d - 0.5f * kNuWidth)));
      const int s_hi =
          __builtin_amdgcn_readfirstlane(static_cast<int>(floorf(rel_c + d + 0.5f * kNuWidth)));
      used_lo = min(used_lo, s_lo);
      used_hi = max(used_hi, s_hi);
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
        const float vat = r.v[0] * atf[0] + r.v[1] * atf[1] + r.v[2] * atf[2];
        const float var = r.v[0] * arf[0] + r.v[1] * arf[1] + r.v[2] * arf[2];
        const float rdt_dot = fmaf(r.rt, r.vut, -vat) * __builtin_amdgcn_rcpf(r.rt + dRt);
        const float rdr_dot = fmaf(r.rr, r.vur, -var) * __builtin_amdgcn_rcpf(r.rr + dRr);
        const float tdot = (rdt_dot + rdr_dot) * inv_c0;
        const float fmt = static_cast<float>(r.g1 * kC0 - (rc.M / 2) * rc.df);
        const float A = fmt * tdot * inv_fs, B = df_fs * tdot;
        t += fmaf(A, half_m, B * quarter_m2);
        xr += fmaf(B, m_f, A) * ngf - r.dxc;
        eps = B * eps_scale;
      }
      t -= rintf(t);
      const float amp = __builtin_amdgcn_rcpf((r.rt + dRt) * (r.rr + dRr));
      const float qx = __builtin_amdgcn_cosf(t) * amp, qy = -__builtin_amdgcn_sinf(t) * amp;
      constexpr int NC = INTRA ? R + 2 : R;  // the B m'^2 term raises the degree by two
      float2 cq[NC];
#pragma unroll
      for (int k = 0; k < R; ++k)
        cq[k] = {qx * r.b[k].x - qy * r.b[k].y, qx * r.b[k].y + qy * r.b[k].x};
      if (INTRA) {
        // (1 - j 2 pi B m'^2) on the modes is F + j eps F'' on the grid, F = psi P, with
        // F'' = psi (P'' - (2u / s^2) P' + (u^2 / s^4 - 1 / s^2) P): coefficient k of the
        // result is c_k + j eps (c_{k-2} / s^4 - (2k + 1) c_k / s^2 + (k + 1)(k + 2) c_{k+2})
        float2 c[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) {
          const float2 ck = k < R ? cq[k] : make_float2(0.0f, 0.0f);
          const float2 cm2 = (k >= 2 && k - 2 < R) ? cq[k - 2] : make_float2(0.0f, 0.0f);
          const float2 cp2 = (k + 2 < R) ? cq[k + 2] : make_float2(0.0f, 0.0f);
          const float wk = -(2.0f * k + 1.0f) * inv_s2;
          const float wp = static_cast<float>((k + 1) * (k + 2));
          const float dx = cm2.x * inv_s4 + wk * ck.x + wp * cp2.x;
          const float dy = cm2.y * inv_s4 + wk * ck.y + wp * cp2.y;
          c[k] = {ck.x - eps * dy, ck.y + eps * dx};
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) cq[k] = c[k];
      }
      // Gaussian weights from s_lo on: g_{s+1} = g_s rho_s, rho_{s+1} = rho_s exp(-1/s^2)
      const float u0 = static_cast<float>(s_lo) - xr;
      float gw = __builtin_amdgcn_exp2f(nc * u0 * u0);
      float rho = __builtin_amdgcn_exp2f(nc * fmaf(2.0f, u0, 1.0f));
#pragma unroll
      for (int s = 0; s < kNuSlots; ++s) {
        if (s >= s_lo && s <= s_hi) {
          const float xx = static_cast<float>(s) - xr;
          float pr2 = cq[NC - 1].x, pi2 = cq[NC - 1].y;
#pragma unroll
          for (int k = NC - 2; k >= 0; --k) {
            pr2 = fmaf(pr2, xx, cq[k].x);
            pi2 = fmaf(pi2, xx, cq[k].y);
          }
          acc[s].x = fmaf(gw, pr2, acc[s].x);
          acc[s].y = fmaf(gw, pi2, acc[s].y);
          gw *= rho;
          rho *= q_ratio;
        }
      }
    }
    // add the window to the grid row and clear it
#pragma unroll
    for (int s = 0; s < kNuSlots; ++s) {
      if (s >= used_lo && s <= used_hi) {
        if (on) {
          // base + s lies in [-ng, 2 ng) (n_g >= 32 > the window)
          int cell = base + s;
          cell += (cell < 0) ? ng : 0;
          cell -= (cell >= ng) ? ng : 0;
          atomicAdd(&grid[cell].x, acc[s].x);
          atomicAdd(&grid[cell].y, acc[s].y);
        }
        acc[s] = {0.0f, 0.0f};
      }
    }
  }
}

// Per (chirp, group of cb channels): grid rows into LDS (zeroed behind for the next
// call), forward FFT of all cb rows together (ping-pong buffers of cb rows), deconvolution
// and the k_c^2 / k_m^2 factor on the M kept modes.
__global__ void __launch_bounds__(kNuFftThreads) nufft_fft_kernel(DevScene sc, RadarConst rc,
                                                                NuShape ns, NuBuffers nb,
                                                                const float2 *tw, bool ranged) {
  extern __shared__ float2 nu_smem[];
  const int nl = blockIdx.x / ns.groups;
  const int grp = blockIdx.x - nl * ns.groups;
  const int n = ns.n0 + nl;
  const int ld = ns.ld, ng = ns.ng, cb = ns.cb;
  const int O = rc.P * rc.Q;
  float2 *lgrid = nu_smem;            // [cb][ld]
  float2 *work = nu_smem + cb * ld;   // [cb][ld]
  // only the chirp's occupied cells are read (and zeroed behind); none without records
  const int2 rg = ranged ? nb.range[nl] : make_int2(0, -1);
  for (int c = 0; c < cb; ++c) {
    const int o = grp * cb + c;
    float2 *src = nb.grid + (static_cast<int64_t>(nl) * O + o) * ng;
    for (int l = threadIdx.x; l < ng; l += blockDim.x) {
      float2 v = {0.0f, 0.0f};
      if (o < O && l >= rg.x && l <= rg.y) {
        v = src[l];
        src[l] = {0.0f, 0.0f};
      }
      lgrid[c * ld + l] = v;
    }
  }
  __syncthreads();
  const int M = rc.M;
  const float s = static_cast<float>(ns.sigma);
  const float hs2 = 0.5f * s * s;
  const float inv_norm = static_cast<float>(1.0 / (ns.sigma * 2.5066282746310002));
  const float w_per_mode = static_cast<float>(2.0 * kPi / ng);
  float2 *echo = static_cast<float2 *>(sc.echo);
  const float2 *res = stockham(lgrid, work, ng, cb, ld, tw);
  for (int idx = threadIdx.x; idx < cb * M; idx += blockDim.x) {
    const int sq = idx / M;
    const int m = idx - sq * M;
    const int oo = grp * cb + sq;
    if (oo >= O) continue;
    const int mp = m - M / 2;
    const float2 u = res[sq * ld + (mp < 0 ? mp + ng : mp)];
    const float w = w_per_mode * static_cast<float>(mp);
    const float fr = static_cast<float>(ns.fc / (rc.f0 + m * rc.df));
    const float corr = fr * fr * inv_norm * __expf(hs2 * w * w);
    float2 *dst = echo + (static_cast<int64_t>(oo) * rc.N + n) * M + m;
    if (ns.accumulate) {  // a reflected path type: add gamma x its echo
      const float gr = static_cast<float>(ns.gamma_re) * corr;
      const float gi = static_cast<float>(ns.gamma_im) * corr;
      const float2 h = *dst;
      *dst = {h.x + gr * u.x - gi * u.y, h.y + gr * u.y + gi * u.x};
    } else {
      *dst = {u.x * corr, u.y * corr};
    }
  }
}


// ---- adjoint (type-2 transform): the loss gradient G = dL/dRe H + j dL/dIm H of the
// kept modes goes through the transpose of the deconvolution and FFT onto each channel's
// grid, and every record then gathers Gaussian-weighted moments of that grid instead of
// spreading onto it. With y = sum_m conj(G) H of one (record, channel),
//   y = Q sum_k b_k mu_k,  mu_k = sum_l g(l) psi(l - x) (l - x)^k,
//   dy/dx = Q sum_k b_k (mu_{k+1} / s^2 - k mu_{k-1}),
// and the seven per-(facet, chirp) sums of the direct adjoint follow: dL/dc through the
// element distances (the channel's delay and 1 / (R_t R_r)), sum Re y, and dL/dbeta_v
// through b_k (and the sub-triangle's source position).

// Adjoint preparation: the forward record plus d b_k / d beta_v by central differences in
// FP64 (step kNuDerStep: truncation ~ (k_c h)^2 / 6 ~ 5e-7, rounding ~ 1e-10 relative).
template <int R>
__global__ void __launch_bounds__(256) nufft_adj_prep_kernel(DevScene sc, RadarConst rc,
                                                            NuShape ns, NuBuffers nb) {
  const int nl = blockIdx.y;
  const int n = ns.n0 + nl;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t item = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (item >= (cnt << (2 * ns.split))) return;
  int sub;
  const int32_t entry = record_entry(item, cnt, ns.split, &sub);
  Geo g;
  entry_geometry(sc, rc, n, cnt, entry, g);
  NuRec<R> out;
  out.valid = g.valid;
  NuDer<R> der;
  der.item = entry;
  double bc = 0.0;
  double dbr[3][R], dbi[3][R], dbc[3] = {0.0, 0.0, 0.0};
  const double h2 = 0.5 / kNuDerStep;
#pragma unroll
  for (int e = 0; e < 7; ++e) {  // the facet's offsets, then each one moved by +h and -h
    double bt[3] = {g.beta[0], g.beta[1], g.beta[2]};
    const int v = (e - 1) >> 1;
    const double sgn = ((e - 1) & 1) ? -1.0 : 1.0;
    if (e > 0) bt[v] += sgn * kNuDerStep;
    double cr[R], ci[R];
    const double c = taylor_coeffs<R>(g, bt, sub, ns, cr, ci);
    if (e == 0) {
      bc = c;
#pragma unroll
      for (int k = 0; k < R; ++k) out.b[k] = {static_cast<float>(cr[k]), static_cast<float>(ci[k])};
    } else if (sgn > 0.0) {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        dbr[v][k] = cr[k];
        dbi[v][k] = ci[k];
      }
      dbc[v] = c;
    } else {
#pragma unroll
      for (int k = 0; k < R; ++k) {
        der.db[v][k] = {static_cast<float>((dbr[v][k] - cr[k]) * h2),
                        static_cast<float>((dbi[v][k] - ci[k]) * h2)};
      }
      der.dx[v] = static_cast<float>(-ns.kappa * (dbc[v] - c) * h2);
    }
  }
  double Rt, Rr, dxc;
  path_fields(g, rc, ns, bc, out, &Rt, &Rr, &dxc);
  const int64_t at = static_cast<int64_t>(nl) * ns.rec_stride + item;  // entry order
  static_cast<NuRec<R> *>(nb.srec)[at] = out;
  static_cast<NuDer<R> *>(nb.sder)[at] = der;
}

// Per (chirp, group of cb channels): the transpose of nufft_fft_kernel. conj(G) of the kept
// modes times the same deconvolution factor, placed at mode m' mod n_g and transformed with
// the same sign, gives grid rows g(l) with sum_m conj(G(m)) H(m) = sum_l S(l) g(l) for the
// spread S of the forward transform.
__global__ void __launch_bounds__(kNuFftThreads) nufft_adj_fft_kernel(
    DevScene sc, RadarConst rc, NuShape ns, NuBuffers nb, const float2 *tw,
    const float2 *grad_echo) {
  extern __shared__ float2 nu_smem[];
  const int nl = blockIdx.x / ns.groups;
  const int grp = blockIdx.x - nl * ns.groups;
  const int n = ns.n0 + nl;
  const int ld = ns.ld, ng = ns.ng, cb = ns.cb;
  const int O = rc.P * rc.Q;
  float2 *lgrid = nu_smem;            // [cb][ld]
  float2 *work = nu_smem + cb * ld;   // [cb][ld]
  for (int i = threadIdx.x; i < cb * ng; i += blockDim.x) {
    const int c = i / ng, l = i - c * ng;
    lgrid[c * ld + l] = {0.0f, 0.0f};
  }
  __syncthreads();
  const int M = rc.M;
  const float s = static_cast<float>(ns.sigma);
  const float hs2 = 0.5f * s * s;
  const float inv_norm = static_cast<float>(1.0 / (ns.sigma * 2.5066282746310002));
  const float w_per_mode = static_cast<float>(2.0 * kPi / ng);
  for (int idx = threadIdx.x; idx < cb * M; idx += blockDim.x) {
    const int sq = idx / M;
    const int m = idx - sq * M;
    const int oo = grp * cb + sq;
    if (oo >= O) continue;
    const int mp = m - M / 2;
    const float w = w_per_mode * static_cast<float>(mp);
    const float fr = static_cast<float>(ns.fc / (rc.f0 + m * rc.df));
    const float corr = fr * fr * inv_norm * __expf(hs2 * w * w);
    const float2 G = grad_echo[(static_cast<int64_t>(oo) * rc.N + n) * M + m];
    lgrid[sq * ld + (mp < 0 ? mp + ng : mp)] = {G.x * corr, -G.y * corr};
  }
  __syncthreads();
  const float2 *res = stockham(lgrid, work, ng, cb, ld, tw);
  for (int i = threadIdx.x; i < cb * ng; i += blockDim.x) {
    const int c = i / ng, l = i - c * ng;
    const int o = grp * cb + c;
    if (o < O) nb.grid[(static_cast<int64_t>(nl) * O + o) * ng + l] = res[c * ld + l];
  }
}

// One lane per (chirp, record), a workgroup per (chirp, kNuGatherRecs records in entry
// order), looping over the channels: each channel's grid row of the chirp is staged in LDS
// and every lane forms the moments mu_0 .. mu_R of its own 13 cells about its own position
// (|l - x| <= kNuWidth / 2, the spread's truncation), then adds this channel's share of the
// seven per-facet sums in registers: Re y, Re dy/dx and Q mu_k (for dL/dbeta_v, applied once
// per record with d b_k / d beta_v) and dL/dc through the channel's distances. One atomic add
// per value and record into partial[chirp][lit facet][kAdjVals] (sub-triangles of a facet
// add into the same slot). Blocks are ordered so that those of one chirp share an XCD (and
// its L2, which holds the chirp's grids).
template <int R>
__global__ void __launch_bounds__(kNuGatherRecs) nufft_gather_kernel(
    DevScene sc, RadarConst rc, NuShape ns, const double *elem, const NuRec<R> *__restrict__ recs,
    const NuDer<R> *__restrict__ ders, const float2 *__restrict__ grids, float *partial,
    int blocks_per_chirp) {
  extern __shared__ float2 nu_row[];  // [n_g]
  const int per_xcd = (gridDim.x + kXcds - 1) / kXcds;  // gridDim.x is a multiple of kXcds
  const int logical = static_cast<int>(blockIdx.x % kXcds) * per_xcd + static_cast<int>(blockIdx.x / kXcds);
  const int nl = logical / blocks_per_chirp;
  if (nl >= ns.n_chirps) return;  // padding blocks (whole workgroup, before any barrier)
  const int rb = logical - nl * blocks_per_chirp;
  const int n = ns.n0 + nl;
  const int32_t n_ent = sc.vis_cnt[n] << (2 * ns.split);
  if (rb * kNuGatherRecs >= n_ent) return;  // whole workgroup
  const int32_t e = rb * kNuGatherRecs + static_cast<int32_t>(threadIdx.x);
  const bool live = e < n_ent;
  const int ng = ns.ng;
  const int O = rc.P * rc.Q;
  const int64_t rec_at = static_cast<int64_t>(nl) * ns.rec_stride + (live ? e : 0);
  const NuRec<R> r = recs[rec_at];
  const bool on = live && r.valid;
  float2 b[R];
#pragma unroll
  for (int k = 0; k < R; ++k) b[k] = on ? r.b[k] : make_float2(0.0f, 0.0f);
  const float utf[3] = {static_cast<float>(r.ut[0]), static_cast<float>(r.ut[1]),
                        static_cast<float>(r.ut[2])};
  const float urf[3] = {static_cast<float>(r.ur[0]), static_cast<float>(r.ur[1]),
                        static_cast<float>(r.ur[2])};
  // positions relative to the record's cell (small numbers: FP32 keeps ~1e-6 cells)
  const float nc = static_cast<float>(-1.4426950408889634 / (2.0 * ns.sigma * ns.sigma));
  const float q_ratio = __builtin_amdgcn_exp2f(2.0f * nc);  // exp(-1 / s^2)
  const float inv_s2 = static_cast<float>(1.0 / (ns.sigma * ns.sigma));
  const float kappa = static_cast<float>(ns.kappa);
  const float g2 = static_cast<float>(0.5 * rc.slope / (kC0 * kC0));
  const float two_pi = static_cast<float>(2.0 * kPi);
  const float g1f = static_cast<float>(r.g1);
  const float half_w = 0.5f * kNuWidth;
  float acc_c[3] = {0.0f, 0.0f, 0.0f}, acc_s = 0.0f, acc_yx = 0.0f;
  float acc_mr[R], acc_mi[R];
#pragma unroll
  for (int k = 0; k < R; ++k) acc_mr[k] = acc_mi[k] = 0.0f;
  const float2 *grow = grids + static_cast<int64_t>(nl) * O * ng;
  for (int o = 0; o < O; ++o) {
    __syncthreads();  // the previous channel's row is no longer read
    for (int l = threadIdx.x; l < ng; l += blockDim.x) nu_row[l] = grow[static_cast<int64_t>(o) * ng + l];
    __syncthreads();
    // this channel's element offsets from the phase centres (wave-uniform)
    const int p = o / rc.Q, q = o - p * rc.Q;
    double at[3], ar[3];
    double st2 = 0.0, sr2 = 0.0;
    for (int k = 0; k < 3; ++k) {
      at[k] = elem[3 * p + k] - rc.tx_c[k];
      ar[k] = elem[3 * (rc.P + q) + k] - rc.rx_c[k];
      st2 += at[k] * at[k];
      sr2 += ar[k] * ar[k];
    }
    const float aat = static_cast<float>(st2), aar = static_cast<float>(sr2);
    // the channel's path (as in the spread)
    const double st = r.ut[0] * at[0] + r.ut[1] * at[1] + r.ut[2] * at[2];
    const double sr = r.ur[0] * ar[0] + r.ur[1] * ar[1] + r.ur[2] * ar[2];
    const double ps = (st + sr) * r.g1;
    const float pr = static_cast<float>(ps - rint(ps));
    const float sft = static_cast<float>(st), sfr = static_cast<float>(sr);
    const float ht = fmaf(-sft, sft, aat), hr = fmaf(-sfr, sfr, aar);
    const float rdt = __builtin_amdgcn_rcpf(fmaf(-2.0f, sft, 2.0f * r.rt));
    const float rdr = __builtin_amdgcn_rcpf(fmaf(-2.0f, sfr, 2.0f * r.rr));
    const float qt = ht * rdt, qr = hr * rdr;
    const float et = qt * fmaf(-qt, rdt, 1.0f), er = qr * fmaf(-qr, rdr, 1.0f);
    const float dRt = et - sft, dRr = er - sfr;
    const float dL = dRt + dRr;
    float t = (r.t0 - pr) + fmaf(g1f, et + er, -g2 * dL * dL);
    t -= rintf(t);
    const float x = fmaf(kappa, dL, r.frac);  // grid position minus the record's cell
    const float Rtp = r.rt + dRt, Rrq = r.rr + dRr;
    const float irt = __builtin_amdgcn_rcpf(Rtp), irr = __builtin_amdgcn_rcpf(Rrq);
    const float amp = irt * irr;
    const float qx = __builtin_amdgcn_cosf(t) * amp, qy = -__builtin_amdgcn_sinf(t) * amp;
    // moments of the grid row about x over the cells |l - x| <= W / 2 (13 cells from
    // ceil(x - W / 2); a 13th cell past x + W / 2 carries a weight below 4e-7)
    const float s0 = ceilf(x - half_w);
    int cell = (r.cell + static_cast<int>(s0)) % ng;  // r.cell + s0 lies in (-ng, 2 ng)
    cell += (cell < 0) ? ng : 0;
    const float u0 = s0 - x;
    float gw = __builtin_amdgcn_exp2f(nc * u0 * u0);
    float rho = __builtin_amdgcn_exp2f(nc * fmaf(2.0f, u0, 1.0f));
    float2 mu[R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) mu[k] = {0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j <= kNuWidth; ++j) {
      const float2 gv = nu_row[cell];
      cell = (cell + 1 == ng) ? 0 : cell + 1;
      const float u = u0 + static_cast<float>(j);
      const float wr = gw * gv.x, wi = gw * gv.y;
      mu[0].x += wr;
      mu[0].y += wi;
      float up = 1.0f;
#pragma unroll
      for (int k = 1; k <= R; ++k) {
        up *= u;
        mu[k].x = fmaf(wr, up, mu[k].x);
        mu[k].y = fmaf(wi, up, mu[k].y);
      }
      gw *= rho;
      rho *= q_ratio;
    }
    // Q mu_k; y and dy/dx
    float2 qm[R + 1];
#pragma unroll
    for (int k = 0; k <= R; ++k) qm[k] = {qx * mu[k].x - qy * mu[k].y, qx * mu[k].y + qy * mu[k].x};
    float yr = 0.0f, yi = 0.0f, yxr = 0.0f;
#pragma unroll
    for (int k = 0; k < R; ++k) {
      yr += b[k].x * qm[k].x - b[k].y * qm[k].y;
      yi += b[k].x * qm[k].y + b[k].y * qm[k].x;
      float nr = qm[k + 1].x * inv_s2, ni = qm[k + 1].y * inv_s2;
      if (k > 0) {
        nr = fmaf(-static_cast<float>(k), qm[k - 1].x, nr);
        ni = fmaf(-static_cast<float>(k), qm[k - 1].y, ni);
      }
      yxr += b[k].x * nr - b[k].y * ni;
      acc_mr[k] += qm[k].x;
      acc_mi[k] += qm[k].y;
    }
    acc_s += yr;
    acc_yx += yxr;
    // dL/dc through the element distances: d Re y / dR = K Im y + kappa Re(dy/dx) - Re y / R
    // (K = 2 pi (f_c - mu tau) / c of this channel), with dR_tp / dc = -e_p
    const float K = two_pi * fmaf(-2.0f * g2, dL, g1f);
    const float A = fmaf(K, yi, kappa * yxr);
    const float ct = A - yr * irt, cr = A - yr * irr;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ep = (static_cast<float>(at[k]) - r.rt * utf[k]) * irt;
      const float eq = (static_cast<float>(ar[k]) - r.rr * urf[k]) * irr;
      acc_c[k] -= ct * ep + cr * eq;
    }
  }
  if (!on) return;
  // dL/dbeta_v = Re sum_k (d b_k / d beta_v) sum_o Q mu_k + (dx / dbeta_v) sum_o Re(dy/dx)
  const NuDer<R> dv = ders[rec_at];
  float tv[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    float a = dv.dx[v] * acc_yx;
#pragma unroll
    for (int k = 0; k < R; ++k) a += dv.db[v][k].x * acc_mr[k] - dv.db[v][k].y * acc_mi[k];
    tv[v] = a;
  }
  float *slot = partial + (static_cast<int64_t>(n) * sc.n_facets + dv.item) * kAdjVals;
  const float vals[kAdjVals - 1] = {acc_c[0], acc_c[1], acc_c[2], acc_s, tv[0], tv[1], tv[2]};
#pragma unroll
  for (int k = 0; k < kAdjVals - 1; ++k) atomicAdd(&slot[k], vals[k]);
}

size_t nufft_smem_bytes(const NuShape &ns) {
  return sizeof(float2) * static_cast<size_t>(2 * ns.cb) * ns.ld;
}

template <int R>
hipError_t launch_nufft_t(const DevScene &sc, const RadarConst &rc, const double *elem,
                          const NuShape &ns, const NuBuffers &nb, const void *tw, hipStream_t s) {
  if (ns.n_chirps <= 0) return hipSuccess;
  const int64_t items = (sc.n_facets << (2 * ns.split)) + sc.n_points;
  if ((rc.intra ? sizeof(NuRecT<R, true>) : sizeof(NuRecT<R, false>)) > nb.rec_bytes)
    return hipErrorInvalidValue;
  if (items > 0) {
    dim3 grid(static_cast<unsigned>((items + 255) / 256), static_cast<unsigned>(ns.n_chirps));
    hipLaunchKernelGGL(nufft_key_kernel, grid, dim3(256), 0, s, sc, rc, ns, nb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nufft_count_kernel, dim3(ns.n_chirps), dim3(1024), 0, s, sc, ns, nb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    const int64_t waves = static_cast<int64_t>(ns.n_chirps) * ns.spread_groups * ns.runs;
    const int64_t blocks = (waves + kNuSpreadThreads / 64 - 1) / (kNuSpreadThreads / 64);
    if (rc.intra) {
      hipLaunchKernelGGL((nufft_prep_kernel<R, true>), grid, dim3(256), 0, s, sc, rc, ns, nb);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL((nufft_spread_kernel<R, true>), dim3(static_cast<unsigned>(blocks)),
                         dim3(kNuSpreadThreads), 0, s, sc, rc, ns, elem,
                         static_cast<const NuRecT<R, true> *>(nb.srec), nb.grid);
    } else {
      hipLaunchKernelGGL((nufft_prep_kernel<R, false>), grid, dim3(256), 0, s, sc, rc, ns, nb);
      if ((e = hipGetLastError()) != hipSuccess) return e;
      hipLaunchKernelGGL((nufft_spread_kernel<R, false>), dim3(static_cast<unsigned>(blocks)),
                         dim3(kNuSpreadThreads), 0, s, sc, rc, ns, elem,
                         static_cast<const NuRecT<R, false> *>(nb.srec), nb.grid);
    }
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(nufft_fft_kernel, dim3(static_cast<unsigned>(ns.n_chirps * ns.groups)),
                     dim3(kNuFftThreads), nufft_smem_bytes(ns), s, sc, rc, ns, nb,
                     static_cast<const float2 *>(tw), items > 0);
  return hipGetLastError();
}

hipError_t launch_nufft(const DevScene &sc, const RadarConst &rc, const double *elem,
                        const NuShape &ns, const NuBuffers &nb, const void *tw, hipStream_t s) {
  if (ns.order == 5) return launch_nufft_t<5>(sc, rc, elem, ns, nb, tw, s);
  if (ns.order == 7) return launch_nufft_t<7>(sc, rc, elem, ns, nb, tw, s);
  if (ns.order == 10) return launch_nufft_t<10>(sc, rc, elem, ns, nb, tw, s);
  return hipErrorInvalidValue;
}


template <int R>
hipError_t launch_nufft_adjoint_t(const DevScene &sc, const RadarConst &rc, const double *elem,
                                  const NuShape &ns, const NuBuffers &nb, const void *tw,
                                  const void *grad_echo, float *partial, hipStream_t s) {
  if (ns.n_chirps <= 0) return hipSuccess;
  if (sizeof(NuRec<R>) > nb.rec_bytes || !nb.sder || sc.n_points != 0 || rc.intra)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(nufft_adj_fft_kernel, dim3(static_cast<unsigned>(ns.n_chirps * ns.groups)),
                     dim3(kNuFftThreads), nufft_smem_bytes(ns), s, sc, rc, ns, nb,
                     static_cast<const float2 *>(tw), static_cast<const float2 *>(grad_echo));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t items = sc.n_facets << (2 * ns.split);
  if (items == 0) return hipSuccess;
  dim3 grid(static_cast<unsigned>((items + 255) / 256), static_cast<unsigned>(ns.n_chirps));
  hipLaunchKernelGGL((nufft_adj_prep_kernel<R>), grid, dim3(256), 0, s, sc, rc, ns, nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int bpc = static_cast<int>((items + kNuGatherRecs - 1) / kNuGatherRecs);
  const int64_t blocks = (static_cast<int64_t>(ns.n_chirps) * bpc + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL((nufft_gather_kernel<R>), dim3(static_cast<unsigned>(blocks)),
                     dim3(kNuGatherRecs), sizeof(float2) * ns.ng, s, sc, rc, ns, elem,
                     static_cast<const NuRec<R> *>(nb.srec), static_cast<const NuDer<R> *>(nb.sder),
                     static_cast<const float2 *>(nb.grid), partial, bpc);
  return hipGetLastError();
}

hipError_t launch_nufft_adjoint(const DevScene &sc, const RadarConst &rc, const double *elem,
                                const NuShape &ns, const NuBuffers &nb, const void *tw,
                                const void *grad_echo, float *partial, hipStream_t s) {
  if (ns.order == 5) return launch_nufft_adjoint_t<5>(sc, rc, elem, ns, nb, tw, grad_echo, partial, s);
  if (ns.order == 7) return launch_nufft_adjoint_t<7>(sc, rc, elem, ns, nb, tw, grad_echo, partial, s);
  if (ns.order == 10) return launch_nufft_adjoint_t<10>(sc, rc, elem, ns, nb, tw, grad_echo, partial, s);
  return hipErrorInvalidValue;
}

}  // namespace rsim
