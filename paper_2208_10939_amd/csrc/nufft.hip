// Facet sum as a type-1 non-uniform FFT over the sample index (FP32 with FP64 geometry and
// phases). Same result as the direct sum of Sections 2.2 and 3.2, eqs. (7)-(13), within
// the spread's error (~1e-6 relative).
//
// With the closed-form facet integral written as a divided difference, the term of a
// lit facet (or point) for channel (p, q) at sample m = m' + M/2 is
//   T(m) = -amp / (R_t R_r k_m^2) exp(-j 2 pi (f_c tau - mu tau^2 / 2))
//          DD2_beta[ exp(j k_c beta) exp(-j m' dk (L - beta)) ](beta_0, beta_1, beta_2),
// with L = R_t + R_r, tau = L / c, f_c = f0 + (M/2) df, k = 2 pi f / c, dk = 2 pi df / c
// and DD2 the second divided difference over the facet's node offsets beta_v. For every
// channel the sum over facets is therefore a type-1 transform of sources at path lengths
// L - beta onto the modes m'. Each is spread onto a periodic grid of n_g >= 2M cells with
// a Gaussian psi(x) = exp(-x^2 / (2 s^2)); the grid position of path length L is
// x = kappa L with kappa = df n_g / c cells per metre, and the facet's spread is
//   Q(p, q) F(l - x_L),  F(u) = (-amp / k_c^2) DD2_beta[ exp(j k_c beta) psi(u + kappa beta) ],
// where only Q = exp(-j 2 pi (f_c tau - mu tau^2/2)) / (R_t R_r) and x_L depend on the
// channel. A forward FFT of each channel's grid then gives
//   H(m' + M/2) = U(m') k_c^2 / (k_m^2 psi_hat(2 pi m' / n_g)),
//   psi_hat(w) = s sqrt(2 pi) exp(-s^2 w^2 / 2).
//
// F is written as at most three grid sources, chosen by the gaps between the nodes
// a_v = k_c beta_v (radians; threshold kNuGapMin):
//   all gaps wide: the vertex form of the divided difference, three Gaussians at
//     -kappa beta_v with weights exp(j k_c beta_v) / prod_{w != v} (beta_v - beta_w);
//   one close pair (beta_0, beta_1) and a far node beta_2: from
//     DD2 = h(beta_2) / ((beta_2 - beta_1)(beta_2 - beta_0))
//           - [h(beta_1) / (beta_2 - beta_1) + DD1 h(beta_0, beta_1)] / (beta_2 - beta_0),
//     a Gaussian at the far node and a Gaussian-weighted quadratic about the pair's
//     midpoint mu (psi expanded in kappa (beta - mu), three terms, with DD1 of
//     (beta - mu)^r exp(j k_c beta) in closed form);
//   all gaps narrow (the facet spans under kNuGapMin / k_c along its direction of
//     incidence, e.g. near the specular direction, and points): psi expanded about the
//     centroid, three terms, with D_r = DD2[beta^r exp(j k_c beta)] by the Leibniz rule
//     over the stable divided differences of exp(j k_c beta).
// No source needs splitting: the weights stay bounded because every divided difference
// is taken over nodes at least kNuGapMin apart or expanded.
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
// Entries of a chirp: its lit facets, the point scatterers and, with the facet-to-facet
// double bounce, one footprint per connection (nufft_entry). Five kernels per chunk of
// chirps, all in a fixed order of operations, so that a call gives the same bits every
// time and whatever other scenes share it:
//   key     per (chirp, entry): grid cell of the phase-centre path;
//   sort    per chirp: a stable counting sort by cell (entries keep their order within a
//           cell), and the chirp's runs: consecutive sorted records, run_len of them unless
//           the next record's cell is more than kspan past the run's first, so that every
//           source of a run lands in one window of kNuSlots cells;
//   prep    per entry: the sources and the phase-centre path (FP64 work, stored as FP32
//           offsets, weights, reduced phase and grid cell), written at the sorted position;
//   spread  (nufft_spread.hip) one workgroup per (chirp, run), one wave per 64 channels:
//           each lane accumulates the run's sources in a register window of kNuSlots
//           cells and writes it out once (no atomics);
//   fft     per (chirp, group of channels): every grid cell summed from the windows that
//           cover it in run order, in-LDS Stockham FFT, deconvolution, echo samples.
#include <type_traits>

#include "adjoint_common.h"
#include "echo_common.h"
#include "fft_common.h"
#include "nufft_common.h"

namespace rsim {

constexpr int kNuFftThreads = 512;
constexpr int kNuMaxOrder = 4;  // Hermite table rows (three Taylor terms are used)
constexpr int kNuSortThreads = 1024;  // 16 waves: each ranks one sixteenth of a chirp's entries
constexpr int kNuSortWaves = kNuSortThreads / 64;
constexpr int kNuGatherRecs = 256;  // records (lanes) per adjoint gather workgroup
constexpr int kNuRedBatch = 8;      // run windows read together by a cell sum of the FFT kernel
constexpr int kNuGatherStage = 4096;  // grid cells staged in LDS by a gather workgroup (32 KB)
static_assert(kNuGatherStage >= 2048 + 12, "a whole row fits the gather's staging");
constexpr int kXcds = 8;            // accelerator complex dies: workgroups go round-robin
constexpr double kNuGapMin = 2.0;   // radians of k_c beta between nodes of a divided difference


size_t nufft_record_bytes(bool intra) {
  return intra ? sizeof(NuRecF<true>) : sizeof(NuRecF<false>);
}

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

// Grid position and cell (0 .. n_g - 1) of a source on the phase-centre path of an entry,
// shifted by the node offset bc of a sub-triangle's centroid (x = kappa (L - bc)), and the
// two distances of that path; FP64.
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

// Taylor coefficients b_k (FP64) of psi expanded about the centroid for a facet with node
// offsets beta about it; b_k includes the common factor -amp / k_c^2.
template <int R>
__device__ void taylor_coeffs(const Geo &g, const double beta[3], const NuShape &ns,
                              double br[R], double bi[R]) {
  const double amp_re = g.amp_re, amp_im = g.amp_im;
#pragma unroll
  for (int k = 0; k < R; ++k) br[k] = bi[k] = 0.0;
  if (!g.valid) return;
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
}

// The phase-centre path of a record (FP64): unit vectors, distances, reduced phase, the
// source's grid cell and fraction (the same cell as the key pass).
template <typename Rec>
__device__ void path_fields(const Geo &g, const RadarConst &rc, const NuShape &ns, double bc,
                            Rec &out, double *Rt, double *Rr, double *dxc) {
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

// (x + j y) exp(j 2 pi T) for T in turns (FP64)
__device__ inline double2 rot_turns(double x, double y, double T) {
  double s, c;
  sincospi(2.0 * (T - rint(T)), &s, &c);
  return make_double2(x * c - y * s, x * s + y * c);
}

// Source form of one lit facet or point (see the header comment): kind 1, 2 or 3 (0 for a
// zero-area facet); for kind 2, *far = the node away from the close pair.
__device__ inline int nufft_classify(const Geo &g, const NuShape &ns, int *far) {
  *far = 0;
  if (!g.valid) return 0;
  const double tpm = ns.fc / kC0;  // turns of k_c beta per metre
  const double *b = g.beta;
  const double gap = kNuGapMin / (2.0 * kPi);  // turns
  // gap opposite node v: between the other two
  const double d0 = fabs(b[1] - b[2]) * tpm, d1 = fabs(b[0] - b[2]) * tpm,
               d2 = fabs(b[0] - b[1]) * tpm;
  const int narrow = (d0 < gap) + (d1 < gap) + (d2 < gap);
  if (narrow == 0) return 1;
  if (narrow == 1) {
    *far = d0 < gap ? 0 : d1 < gap ? 1 : 2;
    return 2;
  }
  return 3;
}

// The grid sources of a facet of the given kind with node offsets beta (FP64): fills
// s[10]. Weights and coefficients include the common factor -amp / k_c^2.
__device__ void nufft_fill(const Geo &g, const double beta[3], const NuShape &ns, int kind,
                           int far, double s[10]) {
#pragma unroll
  for (int k = 0; k < 10; ++k) s[k] = 0.0;
  if (kind == 0) return;
  const double tpm = ns.fc / kC0;
  const double ik2 = 1.0 / (ns.kc * ns.kc);
  const double cr = -g.amp_re * ik2, ci = -g.amp_im * ik2;
  const double *b = beta;
  const double kappa = ns.kappa;
  if (kind == 1) {
    for (int v = 0; v < 3; ++v) {
      const int a = v == 0 ? 1 : 0, c = v == 2 ? 1 : 2;
      const double den = (b[v] - b[a]) * (b[v] - b[c]);
      const double2 w = rot_turns(cr / den, ci / den, tpm * b[v]);
      s[3 * v] = kappa * b[v];
      s[3 * v + 1] = w.x;
      s[3 * v + 2] = w.y;
    }
    return;
  }
  if (kind == 2) {
    // the close pair (p0, p1) = the two nodes other than the far node p2, in index order
    // (picked by selects: an index known only at run time would move the geometry to
    // scratch memory)
    const double B0 = far == 0 ? b[1] : b[0];
    const double B1 = far == 2 ? b[1] : b[2];
    const double B2 = far == 0 ? b[0] : far == 1 ? b[1] : b[2];
    const double d21 = B2 - B1, d20 = B2 - B0;
    const double2 wA = rot_turns(cr / (d21 * d20), ci / (d21 * d20), tpm * B2);
    s[0] = kappa * B2;
    s[1] = wA.x;
    s[2] = wA.y;
    // about mu = (B0 + B1) / 2 with delta = -h, +h at the pair:
    // V_r = -exp(j k_c h) h^r / (d21 d20) - DD1[delta^r exp(j k_c delta)](-h, h) / d20
    // with DD1 = j k_c sinc(k_c h), cos(k_c h), j h sin(k_c h) for r = 0, 1, 2
    const double mu = 0.5 * (B0 + B1), h = 0.5 * (B1 - B0);
    double sh, ch;
    sincospi(2.0 * tpm * h, &sh, &ch);  // |k_c h| < kNuGapMin / 2
    const double kh = ns.kc * h;
    const double snc = fabs(kh) < 1e-4 ? 1.0 - kh * kh * (1.0 / 6.0) : sh / kh;
    const double i12 = 1.0 / (d21 * d20), i0 = 1.0 / d20;
    double vr[3], vi[3];
    vr[0] = -ch * i12;
    vi[0] = -sh * i12 - ns.kc * snc * i0;
    vr[1] = -ch * h * i12 - ch * i0;
    vi[1] = -sh * h * i12;
    vr[2] = -ch * h * h * i12;
    vi[2] = -sh * h * h * i12 - h * sh * i0;
    // a_r = exp(j k_c mu) (-kappa / s)^r / r! V_r; c0 = a0 - a2, c1 = a1 / s, c2 = a2 / s^2
    const double st = -kappa / ns.sigma;
    const double sc[3] = {1.0, st, 0.5 * st * st};
    double ar[3], ai[3];
    for (int r = 0; r < 3; ++r) {
      const double2 v = rot_turns(vr[r] * sc[r], vi[r] * sc[r], tpm * mu);
      ar[r] = v.x * cr - v.y * ci;  // times -amp / k_c^2
      ai[r] = v.x * ci + v.y * cr;
    }
    const double is = 1.0 / ns.sigma;
    s[3] = kappa * mu;
    s[4] = ar[0] - ar[2];
    s[5] = ai[0] - ai[2];
    s[6] = ar[1] * is;
    s[7] = ai[1] * is;
    s[8] = ar[2] * is * is;
    s[9] = ai[2] * is * is;
    return;
  }
  double br[3], bi[3];
  taylor_coeffs<3>(g, beta, ns, br, bi);
  s[3] = 0.0;
  for (int k = 0; k < 3; ++k) {
    s[4 + 2 * k] = br[k];
    s[5 + 2 * k] = bi[k];
  }
}

// The grid sources of one lit facet or point: fills s[10] (FP32) and returns the kind.
__device__ int nufft_sources(const Geo &g, const NuShape &ns, float s[10]) {
  int far;
  const int kind = nufft_classify(g, ns, &far);
  double sd[10];
  nufft_fill(g, g.beta, ns, kind, far, sd);
#pragma unroll
  for (int k = 0; k < 10; ++k) s[k] = static_cast<float>(sd[k]);
  return kind;
}


// Connection j (0-based among chirp n's connections, both launching ends) of the
// facet-to-facet double bounce: its launching end k (0 Tx, 1 Rx), facet A it reflects off
// and facet B it meets.
__device__ inline void db_connection(const DevScene &sc, int n, int32_t j, int *k, int64_t *fa,
                                     int64_t *fb) {
  *k = 0;
  const int32_t c0 = sc.db_cnt[n];
  if (j >= c0) {
    *k = 1;
    j -= c0;
  }
  const int64_t row = (static_cast<int64_t>(*k) * sc.db_n + n) * sc.n_facets;
  *fa = sc.db_idx[row + j];
  *fb = sc.db_b[row + *fa];
}

// World vertices of scene facet f at time t (FP64).
__device__ inline void facet_world(const DevScene &sc, int64_t f, double t, double x[3][3]) {
  const DevInstance &I = sc.inst[find_inst(sc.inst, sc.n_inst, f)];
  const int64_t lt = f - I.facet_base;
  for (int v = 0; v < 3; ++v) {
    const int32_t vi = I.tris[3 * lt + v];
    const double b0 = I.verts[3 * vi + 0], b1 = I.verts[3 * vi + 1], b2 = I.verts[3 * vi + 2];
    for (int q = 0; q < 3; ++q)
      x[v][q] = I.rot[3 * q + 0] * b0 + I.rot[3 * q + 1] * b1 + I.rot[3 * q + 2] * b2 +
                (I.pos0[q] + I.vel[q] * t);
  }
}

// Centroid c and unit normal of a world triangle.
__device__ inline void unit_normal(const double x[3][3], double nrm[3], double c[3]) {
  double e1[3], e2[3];
  for (int q = 0; q < 3; ++q) {
    c[q] = (x[0][q] + x[1][q] + x[2][q]) * (1.0 / 3.0);
    e1[q] = x[1][q] - x[0][q];
    e2[q] = x[2][q] - x[0][q];
  }
  nrm[0] = e1[1] * e2[2] - e1[2] * e2[1];
  nrm[1] = e1[2] * e2[0] - e1[0] * e2[2];
  nrm[2] = e1[0] * e2[1] - e1[1] * e2[0];
  const double a = sqrt(nrm[0] * nrm[0] + nrm[1] * nrm[1] + nrm[2] * nrm[2]);
  for (int q = 0; q < 3; ++q) nrm[q] /= a;
}

// The footprint of a connection launched from end k (0: E is the Tx phase centre, 1: the
// Rx one) from world triangles xa (A) and xb (B) and the launching and other phase
// centres E and O: the image ei of E in A's plane, A's unit normal na, the
// footprint x (central projection from ei of A's vertices onto B's plane, ordered to B's
// normal) as the facet of g (centroid, node offsets along w = unit vectors to ei and O,
// amplitude gamma / 2 times j o A / (2 pi), reference delays), and the footprint's
// centroid in c (also g.c). Shared by the forward entry and the adjoint's chain rule.
__device__ inline void db_footprint(const double xa[3][3], const double xb[3][3],
                                    const double E[3], const double O[3], int k,
                                    double gamma_re, double gamma_im, Geo &g, double ei[3],
                                    double na[3], double x[3][3], double *xo_out = nullptr) {
  double ca[3], nb[3], cb[3];
  unit_normal(xa, na, ca);
  unit_normal(xb, nb, cb);
  const double fe = na[0] * (E[0] - ca[0]) + na[1] * (E[1] - ca[1]) + na[2] * (E[2] - ca[2]);
  for (int q = 0; q < 3; ++q) ei[q] = E[q] - 2.0 * fe * na[q];
  const double num = nb[0] * (cb[0] - ei[0]) + nb[1] * (cb[1] - ei[1]) + nb[2] * (cb[2] - ei[2]);
  for (int v = 0; v < 3; ++v) {
    const double d0 = xa[v][0] - ei[0], d1 = xa[v][1] - ei[1], d2 = xa[v][2] - ei[2];
    const double sv = num / (nb[0] * d0 + nb[1] * d1 + nb[2] * d2);
    x[v][0] = ei[0] + sv * d0;
    x[v][1] = ei[1] + sv * d1;
    x[v][2] = ei[2] + sv * d2;
  }
  double c[3], e1[3], e2[3];
  for (int q = 0; q < 3; ++q) {
    c[q] = (x[0][q] + x[1][q] + x[2][q]) * (1.0 / 3.0);
    e1[q] = x[1][q] - x[0][q];
    e2[q] = x[2][q] - x[0][q];
  }
  double nv[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2],
                  e1[0] * e2[1] - e1[1] * e2[0]};
  if (nv[0] * nb[0] + nv[1] * nb[1] + nv[2] * nb[2] < 0.0) {
    // ordered to B's normal: swapping two vertices flips the winding
    for (int q = 0; q < 3; ++q) {
      const double tmp = x[1][q];
      x[1][q] = x[2][q];
      x[2][q] = tmp;
      nv[q] = -nv[q];
    }
  }
  const double two_area = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  // the path's Tx-side and Rx-side centres: the image on the launching side
  double ut[3], ur[3];
  for (int q = 0; q < 3; ++q) {
    ut[q] = (k ? O[q] : ei[q]) - c[q];
    ur[q] = (k ? ei[q] : O[q]) - c[q];
  }
  const double rt = sqrt(ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2]);
  const double rr = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
  double w[3];
  for (int q = 0; q < 3; ++q) w[q] = ut[q] / rt + ur[q] / rr;
  const double nw = nv[0] * w[0] + nv[1] * w[1] + nv[2] * w[2];
  for (int v = 0; v < 3; ++v)
    g.beta[v] = w[0] * (x[v][0] - c[0]) + w[1] * (x[v][1] - c[1]) + w[2] * (x[v][2] - c[2]);
  // j (o A / (2 pi)) times gamma / 2
  const double xo = two_area > 0.0 ? nw * (0.25 / (2.0 * kPi)) : 0.0;
  if (xo_out) *xo_out = xo;
  g.amp_re = -0.5 * xo * gamma_im;
  g.amp_im = 0.5 * xo * gamma_re;
  g.tref_t = rt / kC0;
  g.tref_r = rr / kC0;
  for (int q = 0; q < 3; ++q) {
    g.vel[q] = 0.0;
    g.c[q] = c[q];
  }
  g.valid = two_area > 0.0;
  g.pad = 0;
}

// Geometry of facet-sum entry `item` of chirp n and the phase centres its path starts
// from: a lit facet or a point (entry_geometry, rc_e = rc, *side = -1), or a facet-to-facet
// double-bounce connection (A, B) launched from end *side (0 Tx, 1 Rx): the footprint of
// A's reflected tube on B's plane (db_footprint) as the facet, that end's phase centre
// replaced by its image E' in rc_e, gamma / 2 in the amplitude (the connection is one of
// the two evaluations of its path), and A's unit normal in refl: the mirror that maps that
// end's channel offsets to the image elements' (distances from image elements are those of
// the folded path).
__device__ void nufft_entry(const DevScene &sc, const RadarConst &rc, int n, int32_t cnt,
                            int32_t item, Geo &g, RadarConst &rc_e, double refl[3], int *side) {
  rc_e = rc;
  refl[0] = refl[1] = refl[2] = 0.0;
  *side = -1;
  const int32_t base = cnt + sc.n_points;
  if (!sc.db_on || item < base) {
    entry_geometry(sc, rc, n, cnt, item, g);
    return;
  }
  int k;
  int64_t fa, fb;
  db_connection(sc, n, item - base, &k, &fa, &fb);
  const double t = n * rc.tc;
  double xa[3][3], xb[3][3], x[3][3], ei[3], na[3];
  facet_world(sc, fa, t, xa);
  facet_world(sc, fb, t, xb);
  // the launching and other centres by value (selects, not a pointer chosen at run time,
  // which would move the centres to scratch memory)
  double E[3], O[3];
  for (int q = 0; q < 3; ++q) {
    E[q] = k ? rc.rx_c[q] : rc.tx_c[q];
    O[q] = k ? rc.tx_c[q] : rc.rx_c[q];
  }
  db_footprint(xa, xb, E, O, k, sc.db_gamma_re, sc.db_gamma_im, g, ei, na, x);
  for (int q = 0; q < 3; ++q) {
    rc_e.tx_c[q] = k == 0 ? ei[q] : rc.tx_c[q];
    rc_e.rx_c[q] = k == 1 ? ei[q] : rc.rx_c[q];
    refl[q] = na[q];
  }
  *side = k;
}

// u minus twice its component along the unit normal nrm (a mirror image of the direction)
__device__ __forceinline__ void mirror_dir(double (&u)[3], const double nrm[3]) {
  const double un = u[0] * nrm[0] + u[1] * nrm[1] + u[2] * nrm[2];
  for (int q = 0; q < 3; ++q) u[q] -= 2.0 * un * nrm[q];
}

template <bool INTRA>
__global__ void __launch_bounds__(256) nufft_prep_kernel(DevScene sc0, RadarConst rc, NuShape ns,
                                                        NuBuffers nb, NuBatch bt) {
  const NuWork w = nu_work(sc0, ns, bt, blockIdx.y);
  const DevScene &sc = *w.sc;
  const int n = w.n;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t item = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  const int32_t total = entry_total(sc, n);
  if (nb.census) {
    // wave counts of each form, added into one of kNuCensusSlots rows
    int kind = -1;
    if (item < total) {
      Geo g;
      RadarConst rc_e;
      double refl[3];
      int side;
      nufft_entry(sc, rc, n, cnt, item, g, rc_e, refl, &side);
      int far;
      kind = nufft_classify(g, ns, &far);
    }
    const int row = static_cast<int>((blockIdx.y * gridDim.x + blockIdx.x) * (blockDim.x >> 6) +
                                     (threadIdx.x >> 6)) % kNuCensusSlots;
    for (int k = 0; k < 4; ++k) {
      const unsigned long long m = __ballot(kind == k);
      if ((threadIdx.x & 63) == 0 && m)
        atomicAdd(nb.census + 4 * row + k, static_cast<unsigned long long>(__popcll(m)));
    }
  }
  if (item >= total) return;
  Geo g;
  RadarConst rc_e;
  double refl[3];
  int side;
  nufft_entry(sc, rc, n, cnt, item, g, rc_e, refl, &side);
  NuRecF<INTRA> out;
  out.kind = nufft_sources(g, ns, out.s);
  double Rt, Rr, dxc;
  path_fields(g, rc_e, ns, 0.0, out, &Rt, &Rr, &dxc);
  // the launching end's channel offsets act through its mirrored direction (each side
  // named by a constant: a pointer chosen at run time would move the record to scratch)
  if (side == 0) mirror_dir(out.ut, refl);
  if (side == 1) mirror_dir(out.ur, refl);
  if constexpr (INTRA) {
    double vut = 0.0, vur = 0.0;
    for (int k = 0; k < 3; ++k) {
      out.ext[k] = static_cast<float>(g.vel[k]);
      vut += g.vel[k] * (g.c[k] - rc.tx_c[k]) / Rt;
      vur += g.vel[k] * (g.c[k] - rc.rx_c[k]) / Rr;
    }
    out.ext[3] = static_cast<float>(vut);
    out.ext[4] = static_cast<float>(vur);
    out.ext[5] = static_cast<float>(dxc);
  } else {
    out.ext[0] = out.ext[1] = 0.0f;
  }
  static_cast<NuRecF<INTRA> *>(nb.srec)[w.rec + nb.pos[w.rec + item]] = out;
}

__global__ void __launch_bounds__(256) nufft_key_kernel(DevScene sc0, RadarConst rc, NuShape ns,
                                                       NuBuffers nb, NuBatch bt) {
  const NuWork w = nu_work(sc0, ns, bt, blockIdx.y);
  const DevScene &sc = *w.sc;
  const int n = w.n;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t item = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (item >= entry_total(sc, n)) return;
  Geo g;
  RadarConst rc_e;
  double refl[3];
  int side;
  nufft_entry(sc, rc, n, cnt, item, g, rc_e, refl, &side);
  double x, Rt, Rr, dxc;
  int cell;
  centre_cell(g, rc_e, ns, 0.0, &x, &cell, &Rt, &Rr, &dxc);
  nb.key[w.rec + item] = cell;
}

// Lane `lane`'s key k (0 <= k < 2^nbits; valid: the lane holds an entry) among the keys of
// its wave: how many earlier lanes hold k, and how many lanes in all. The lanes holding
// the same key are found bit by bit from one ballot per key bit (a wave-uniform mask of
// the lanes with that bit set, or its complement): a fixed amount of work per 64 entries,
// where a loop over the distinct keys would wait on a shuffle and an LDS round trip for
// each.
__device__ inline void chunk_rank(int32_t k, bool valid, int nbits, int lane, int *before,
                                  int *total) {
  uint64_t eq = __ballot(valid);
  for (int b = 0; b < nbits; ++b) {
    const uint64_t m = __ballot(valid && ((k >> b) & 1));
    eq &= ((k >> b) & 1) ? m : ~m;
  }
  *before = __popcll(eq & ((uint64_t(1) << lane) - 1));
  *total = __popcll(eq);
}

// Per chirp: stable counting sort of the entries by cell, and the chirp's runs.
// Wave w takes the w-th sixteenth of the entries (in entry order), 64 at a time: it counts
// its cells in its own LDS row (the first lane of each cell in a chunk adds the chunk's
// count), the rows become per-wave starting positions (cell offset plus the counts of
// earlier waves), and each wave then ranks its entries 64 at a time: start of the cell
// plus the earlier lanes of the chunk with that cell (chunk_rank). Runs are cut by one
// lane over the occupied cells.
__global__ void __launch_bounds__(kNuSortThreads) nufft_sort_kernel(DevScene sc0, NuShape ns,
                                                                   NuBuffers nb, NuBatch bt) {
  extern __shared__ int32_t sort_smem[];
  const int ng = ns.ng;
  int32_t *cnt = sort_smem;                           // [kNuSortWaves][ng]
  int32_t *cbase = sort_smem + kNuSortWaves * ng;     // [ng + 1]: first record of each cell
  int32_t *part = cbase + ng + 1;                     // [kNuSortThreads]
  const int nl = blockIdx.x;
  const NuWork wk = nu_work(sc0, ns, bt, nl);
  const DevScene &sc = *wk.sc;
  const int n = wk.n;
  const int32_t *key = nb.key + wk.rec;
  int32_t *pos = nb.pos + wk.rec;
  const int32_t n_ent = entry_total(sc, n);
  const int tid = static_cast<int>(threadIdx.x);
  const int w = tid >> 6, lane = tid & 63;
  int nbits = 1;
  while ((1 << nbits) < ng) ++nbits;  // cells are below 2^nbits
  const int32_t seg = ((n_ent + kNuSortWaves - 1) / kNuSortWaves + 63) & ~63;
  const int32_t e0 = min(n_ent, w * seg), e1 = min(n_ent, e0 + seg);
  for (int i = tid; i < kNuSortWaves * ng; i += kNuSortThreads) cnt[i] = 0;
  __syncthreads();
  for (int32_t chunk = e0; chunk < e1; chunk += 64) {
    const int32_t e = chunk + lane;
    const bool valid = e < e1;
    const int32_t k = valid ? key[e] : 0;
    int before, total;
    chunk_rank(k, valid, nbits, lane, &before, &total);
    if (valid && before == 0) cnt[w * ng + k] += total;  // one lane per cell: no race
  }
  __syncthreads();
  // totals of two cells per thread (n_g <= 2048), exclusive scan over cells, then each
  // wave's starting position per cell
  const int c0 = 2 * tid;
  int32_t t0 = 0, t1 = 0;
  if (c0 < ng)
    for (int v = 0; v < kNuSortWaves; ++v) t0 += cnt[v * ng + c0];
  if (c0 + 1 < ng)
    for (int v = 0; v < kNuSortWaves; ++v) t1 += cnt[v * ng + c0 + 1];
  part[tid] = t0 + t1;
  __syncthreads();
  for (int off = 1; off < kNuSortThreads; off <<= 1) {
    const int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const int32_t base0 = part[tid] - t0 - t1;
  if (c0 < ng) {
    cbase[c0] = base0;
    int32_t at = base0;
    for (int v = 0; v < kNuSortWaves; ++v) {
      const int32_t k = cnt[v * ng + c0];
      cnt[v * ng + c0] = at;
      at += k;
    }
  }
  if (c0 + 1 < ng) {
    cbase[c0 + 1] = base0 + t0;
    int32_t at = base0 + t0;
    for (int v = 0; v < kNuSortWaves; ++v) {
      const int32_t k = cnt[v * ng + c0 + 1];
      cnt[v * ng + c0 + 1] = at;
      at += k;
    }
  }
  if (tid == 0) cbase[ng] = n_ent;
  __syncthreads();
  // runs: cut by one lane over the occupied cells (reads cbase only)
  if (tid == 0) {
    int4 *runs = nb.runs + wk.run;
    int nr = 0;
    int open_cell = 0, open_rb = 0, open_n = 0;
    auto emit = [&](int rb, int re, int base) {
      if (nr < wk.max_runs) runs[nr] = make_int4(rb, re, base, 0);
      ++nr;
    };
    for (int c = 0; c < ng; ++c) {
      int h = cbase[c + 1] - cbase[c];
      if (!h) continue;
      int rb = cbase[c];
      if (open_n > 0 && c - open_cell > wk.kspan) {
        emit(open_rb, open_rb + open_n, open_cell - wk.b0);
        open_n = 0;
      }
      while (h > 0) {
        if (open_n == 0) {
          open_cell = c;
          open_rb = rb;
        }
        const int take = min(h, wk.run_len - open_n);
        open_n += take;
        h -= take;
        rb += take;
        if (open_n == wk.run_len) {
          emit(open_rb, open_rb + open_n, open_cell - wk.b0);
          open_n = 0;
        }
      }
    }
    if (open_n > 0) emit(open_rb, open_rb + open_n, open_cell - wk.b0);
    nb.n_runs[nl] = min(nr, wk.max_runs);
  }
  // stable ranks: start of the cell for this wave plus the earlier lanes of the chunk
  for (int32_t chunk = e0; chunk < e1; chunk += 64) {
    const int32_t e = chunk + lane;
    const bool valid = e < e1;
    const int32_t k = valid ? key[e] : 0;
    int before, total;
    chunk_rank(k, valid, nbits, lane, &before, &total);
    if (valid) {
      // one LDS read by every lane of the wave, then one write by the first lane of each
      // cell (in that order: a wave's LDS instructions run in program order)
      const int32_t start = cnt[w * ng + k];
      pos[e] = start + before;
      if (before == 0) cnt[w * ng + k] = start + total;
    }
  }
}

// First index in the sorted bases[0 .. n) with bases[i] >= v.
__device__ inline int lower_bound_lds(const int32_t *bases, int n, int v) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bases[mid] < v)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// Per (chirp, group of cb channels): each grid cell l summed from the run windows that
// cover it (at l, l - n_g or l + n_g on the periodic grid; in order of the runs' base
// cells, which is the run order), forward FFT of all cb rows together (ping-pong buffers),
// deconvolution and the k_c^2 / k_m^2 factor on the M kept modes.
__global__ void __launch_bounds__(kNuFftThreads) nufft_fft_kernel(DevScene sc0, RadarConst rc,
                                                                NuShape ns, NuBuffers nb,
                                                                const float2 *tw, NuBatch bt) {
  extern __shared__ float2 nu_smem[];
  const int nl = blockIdx.x / ns.groups;
  const int grp = blockIdx.x - nl * ns.groups;
  const NuWork wk = nu_work(sc0, ns, bt, nl);
  const DevScene &sc = *wk.sc;
  const int n = wk.n;
  const int ld = ns.ld, ng = ns.ng, cb = ns.cb;
  const int O = rc.P * rc.Q;
  float2 *lgrid = nu_smem;            // [cb][ld]
  float2 *work = nu_smem + cb * ld;   // [cb][ld]
  int32_t *bases = reinterpret_cast<int32_t *>(work + cb * ld);  // [max_runs]
  const int nr = nb.n_runs[nl];
  const int4 *runs = nb.runs + wk.run;
  for (int r = threadIdx.x; r < nr; r += blockDim.x) bases[r] = runs[r].z;
  __syncthreads();
  const float2 *part = nb.grid + wk.run * O * kNuSlots;
  for (int l = threadIdx.x; l < ng; l += blockDim.x) {
    int lo[3], hi[3];
#pragma unroll
    for (int im = 0; im < 3; ++im) {
      const int P = l + (im - 1) * ng;
      lo[im] = lower_bound_lds(bases, nr, P - kNuSlots + 1);
      hi[im] = lower_bound_lds(bases, nr, P + 1);
    }
    for (int c = 0; c < cb; ++c) {
      const int o = grp * cb + c;
      float2 v = {0.0f, 0.0f};
      if (o < O) {
#pragma unroll
        for (int im = 0; im < 3; ++im) {
          const int P = l + (im - 1) * ng;
          // kNuRedBatch windows' loads in flight together, then added in run order (the
          // loads are independent; only the sum is ordered)
          for (int r0 = lo[im]; r0 < hi[im]; r0 += kNuRedBatch) {
            float2 p[kNuRedBatch];
#pragma unroll
            for (int k = 0; k < kNuRedBatch; ++k) {
              const int r = r0 + k;
              if (r < hi[im])
                p[k] = part[(static_cast<int64_t>(r) * O + o) * kNuSlots + (P - bases[r])];
            }
#pragma unroll
            for (int k = 0; k < kNuRedBatch; ++k) {
              if (r0 + k < hi[im]) {
                v.x += p[k].x;
                v.y += p[k].y;
              }
            }
          }
        }
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
// grid g(l), and every record then gathers Gaussian-weighted moments of that grid at its
// sources instead of spreading onto it. With y = sum_m conj(G) H of one (record, channel)
// and the source positions x_s = x - off_s (x the channel's path position),
//   y = Q sum_s sum_k c_sk mu_sk,  mu_sk = sum_l g(l) psi(l - x_s) (l - x_s)^k,
//   dy/dx_s = Q sum_k c_sk (mu_s,k+1 / s^2 - k mu_s,k-1)
// (a point has c_s0 = its weight only), and the seven per-(facet, chirp) sums of the direct
// adjoint follow: dL/dc through the element distances (the channel's delay and
// 1 / (R_t R_r); every source moves with x), sum Re y, and
//   dL/dbeta_v = Re sum_sk (d c_sk / d beta_v) sum_o Q mu_sk
//                - Re sum_s (d off_s / d beta_v) sum_o dy/dx_s,
// one record per lit facet, so every per-facet slot is written once (no atomics).

// Adjoint record: d s[j] / d beta_v of the forward record's sources and the facet's
// index in the lit list.
struct alignas(16) NuDerF {
  float ds[3][10];
  int32_t item;
  int32_t pad;
};
static_assert(sizeof(NuDerF) == 128, "adjoint record size");
static_assert(kAdjVals == kAdjSlotFloats, "adjoint slot layout");
constexpr double kNuDerStep = 1e-6;  // metres: central differences of the sources in beta

size_t nufft_der_bytes() { return sizeof(NuDerF); }

// Adjoint preparation, one thread per (chirp, lit facet): the forward record and the
// derivatives of its sources in FP64 with the source form held (closed form for three
// points; central differences for the others, step kNuDerStep: every form is analytic in
// the node offsets, truncation ~ (k_c h)^2 / 6 ~ 5e-7, rounding ~ 1e-10 relative), both in
// entry order; the facet's
// entry is appended to its chirp's list of three-point records (class 0) or of the others
// (class 1), so that a gather wave meets one kind of record, with the record's cell beside
// it (nb.pos). A zero-area facet gets a zero slot here and no list entry.
__global__ void __launch_bounds__(256) nufft_adj_prep_kernel(DevScene sc, RadarConst rc,
                                                            NuShape ns, NuBuffers nb,
                                                            float *partial) {
  const int nl = blockIdx.y;
  const int n = ns.n0 + nl;
  const int32_t cnt = sc.vis_cnt[n];
  const int32_t item = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  const bool live = item < entry_total(sc, n);
  const bool conn = item >= cnt;  // a double-bounce connection (the adjoint has no points)
  const int ncls = sc.db_on ? 4 : 2;  // class lists per chirp: facets, then connections
  int kind = 0, cell = 0;
  if (live) {
    Geo g;
    RadarConst rc_e;
    double refl[3];
    int side;
    nufft_entry(sc, rc, n, cnt, item, g, rc_e, refl, &side);
    int far;
    kind = nufft_classify(g, ns, &far);
    NuRecF<false> out;
    double sd[10];
    nufft_fill(g, g.beta, ns, kind, far, sd);
#pragma unroll
    for (int k = 0; k < 10; ++k) out.s[k] = static_cast<float>(sd[k]);
    out.kind = kind;
    out.ext[0] = out.ext[1] = 0.0f;
    double Rt, Rr, dxc;
    path_fields(g, rc_e, ns, 0.0, out, &Rt, &Rr, &dxc);
    // a connection's launching end acts through its mirrored direction, as in the forward
    if (side == 0) mirror_dir(out.ut, refl);
    if (side == 1) mirror_dir(out.ur, refl);
    cell = out.cell;
    const int64_t at = static_cast<int64_t>(nl) * ns.rec_stride + item;  // entry order
    static_cast<NuRecF<false> *>(nb.srec)[at] = out;
    // derivatives stored row by row (a local record indexed by the loop's v would sit in
    // scratch)
    NuDerF *der = static_cast<NuDerF *>(nb.sder) + at;
    der->item = item;
    der->pad = 0;
    if (kind == 1) {
      // three points: s[3v] = kappa beta_v and w_v = C exp(j k_c beta_v) / prod_{u != v}
      // (beta_v - beta_u) (s[3v + 1], s[3v + 2]) have closed-form derivatives:
      // dw_v/dbeta_v = w_v (j k_c - sum_{u != v} 1 / (beta_v - beta_u)),
      // dw_v/dbeta_u = w_v / (beta_v - beta_u)
      const double kc = 2.0 * kPi * ns.fc / kC0;
      const double *b = g.beta;
      for (int u = 0; u < 3; ++u) {
        double d[10];
        d[9] = 0.0;
        for (int v = 0; v < 3; ++v) {
          const double wr = sd[3 * v + 1], wi = sd[3 * v + 2];
          d[3 * v] = u == v ? ns.kappa : 0.0;
          if (u == v) {
            const int a = v == 0 ? 1 : 0, c = v == 2 ? 1 : 2;
            const double fr = -(1.0 / (b[v] - b[a]) + 1.0 / (b[v] - b[c]));
            d[3 * v + 1] = wr * fr - wi * kc;
            d[3 * v + 2] = wr * kc + wi * fr;
          } else {
            const double f = 1.0 / (b[v] - b[u]);
            d[3 * v + 1] = wr * f;
            d[3 * v + 2] = wi * f;
          }
        }
#pragma unroll
        for (int k = 0; k < 10; ++k) der->ds[u][k] = static_cast<float>(d[k]);
      }
    } else {
      const double h2 = 0.5 / kNuDerStep;
      for (int v = 0; v < 3; ++v) {
        double bp[3] = {g.beta[0], g.beta[1], g.beta[2]}, bm[3] = {g.beta[0], g.beta[1], g.beta[2]};
        bp[v] += kNuDerStep;
        bm[v] -= kNuDerStep;
        double sp[10], sm[10];
        nufft_fill(g, bp, ns, kind, far, sp);
        nufft_fill(g, bm, ns, kind, far, sm);
#pragma unroll
        for (int k = 0; k < 10; ++k) der->ds[v][k] = static_cast<float>((sp[k] - sm[k]) * h2);
      }
    }
    if (kind == 0) {
      float *slot = conn ? nb.part_db + (static_cast<int64_t>(nl) * nb.db_stride + item - cnt) *
                                            kAdjVals
                         : partial + (static_cast<int64_t>(n) * sc.n_facets + item) * kAdjVals;
#pragma unroll
      for (int k = 0; k < kAdjVals; ++k) slot[k] = 0.0f;
    }
  }
  // wave-aggregated appends to the class lists: three-point facets, other facets, then
  // (with the double bounce) three-point connections, other connections
  const int lane = threadIdx.x & 63;
  for (int c = 0; c < ncls; ++c) {
    const bool mine = live && kind != 0 && (kind == 1) == ((c & 1) == 0) && conn == (c >= 2);
    const uint64_t m = __ballot(mine);
    if (!m) continue;
    const int leader = __ffsll(static_cast<unsigned long long>(m)) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(&nb.n_runs[ncls * nl + c], __popcll(m));
    base = __shfl(base, leader);
    if (mine) {
      const int64_t at = static_cast<int64_t>(ncls * nl + c) * ns.rec_stride + base +
                         __popcll(m & ((uint64_t(1) << lane) - 1));
      nb.key[at] = item;
      nb.pos[at] = cell;
    }
  }
}

// Chain rule of one facet-to-facet connection (chirp n, connection j) to the world vertices
// of its facets A and B: its adjoint sums (dL/dbeta_v of the footprint's node offsets, the
// sum of Re y = dL/d ln(amplitude)) and per-element sums dL/dR_e of the distances from the
// channel elements (the launching side's mirrored in A's plane) to the footprint's
// centroid give
//   dL/dtheta = sum_e (dL/dR_e) dR_e/dtheta + sum_v (dL/dbeta_v) dbeta_v/dtheta
//               + (sum Re y) d ln(o A)/dtheta
// for each of the 18 vertex coordinates theta. With u_e the unit vector from the centroid
// c to element e and a_e = e - E, the element image E' + M a_e (M = I - 2 n n^T, n A's unit
// normal) moves by dE' - 2 (dn (n . a_e) + n (dn . a_e)), so the distance term's change is
//   -S . dc + S_L . dE' - 2 V . dn,   S = sum_e (dL/dR_e) u_e,  S_L the same over the
//   launching side,  V = sum over that side of (dL/dR_e) ((n . a_e) u_e + (u_e . n) a_e),
// formed once; the derivatives of the FP64 footprint construction (db_footprint: c, E', n,
// the node offsets and o A) are taken by central differences (step kDbStep). The gradients
// are added with FP64 atomics into the per-facet chirp sums (plain and t_n-weighted, [F][9]
// each), so their last bits depend on the order in which connections meeting the same
// facet arrive.
constexpr double kDbStep = 1e-6;  // metres

__global__ void __launch_bounds__(128) nufft_db_grad_kernel(DevScene sc, RadarConst rc,
                                                           NuShape ns, NuBuffers nb,
                                                           const double *elem, double *dbsum,
                                                           double *dbtsum) {
  const int nl = blockIdx.y;
  const int n = ns.n0 + nl;
  const int32_t j = static_cast<int32_t>(blockIdx.x * blockDim.x + threadIdx.x);
  if (j >= sc.db_cnt[n] + sc.db_cnt[sc.db_n + n]) return;
  const int32_t cnt = sc.vis_cnt[n];
  const auto *rec = static_cast<const NuRecF<false> *>(nb.srec) +
                    static_cast<int64_t>(nl) * ns.rec_stride + cnt + j;
  if (rec->kind == 0) return;  // zero-area footprint: no echo
  const int64_t slot = static_cast<int64_t>(nl) * nb.db_stride + j;
  const float *sums = nb.part_db + slot * kAdjVals;
  const int P = rc.P, Q = rc.Q, E = P + Q;
  const float *del = nb.el_db + slot * E;
  int k;
  int64_t fa, fb;
  db_connection(sc, n, j, &k, &fa, &fb);
  const double t = n * rc.tc;
  double xw[2][3][3];
  facet_world(sc, fa, t, xw[0]);
  facet_world(sc, fb, t, xw[1]);
  // the launching and other centres by value (selects: no run-time pointer into rc)
  double Ec[3], Oc[3];
  for (int q = 0; q < 3; ++q) {
    Ec[q] = k ? rc.rx_c[q] : rc.tx_c[q];
    Oc[q] = k ? rc.tx_c[q] : rc.rx_c[q];
  }
  const double S = sums[3];
  const double gb[3] = {sums[4], sums[5], sums[6]};
  // the element sums at the connection's geometry
  double sa[3] = {0.0, 0.0, 0.0}, sl[3] = {0.0, 0.0, 0.0}, vv[3] = {0.0, 0.0, 0.0};
  {
    Geo g0;
    double ei[3], na[3], x[3][3], xo;
    db_footprint(xw[0], xw[1], Ec, Oc, k, 1.0, 0.0, g0, ei, na, x, &xo);
    for (int e = 0; e < E; ++e) {
      const bool launching = (e < P) == (k == 0);
      const double de = static_cast<double>(del[e]);
      double a[3], pe[3];
      for (int q = 0; q < 3; ++q) a[q] = elem[3 * e + q] - Ec[q];
      const double an = a[0] * na[0] + a[1] * na[1] + a[2] * na[2];
      for (int q = 0; q < 3; ++q)
        pe[q] = launching ? ei[q] + a[q] - 2.0 * an * na[q] : elem[3 * e + q];
      double u[3] = {pe[0] - g0.c[0], pe[1] - g0.c[1], pe[2] - g0.c[2]};
      const double r = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
      for (int q = 0; q < 3; ++q) u[q] /= r;
      const double un = u[0] * na[0] + u[1] * na[1] + u[2] * na[2];
      for (int q = 0; q < 3; ++q) {
        sa[q] += de * u[q];
        sl[q] += launching ? de * u[q] : 0.0;
        vv[q] += launching ? de * (an * u[q] + un * a[q]) : 0.0;
      }
    }
  }
  // L's first-order change for a geometry: node offsets, amplitude and the element term
  auto lin = [&](const double (&xq)[2][3][3]) {
    Geo g;
    double ei[3], na[3], x[3][3], xo;
    db_footprint(xq[0], xq[1], Ec, Oc, k, 1.0, 0.0, g, ei, na, x, &xo);
    double v = gb[0] * g.beta[0] + gb[1] * g.beta[1] + gb[2] * g.beta[2] + S * log(fabs(xo));
    for (int q = 0; q < 3; ++q) v += -sa[q] * g.c[q] + sl[q] * ei[q] - 2.0 * vv[q] * na[q];
    return v;
  };
  // coordinate cc of facet w moved by dh (selects: no run-time index into the arrays)
  auto lin_at = [&](int w, int cc, double dh) {
    double xq[2][3][3];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
      for (int v = 0; v < 3; ++v)
#pragma unroll
        for (int q = 0; q < 3; ++q) xq[u][v][q] = xw[u][v][q] + ((u == w && 3 * v + q == cc) ? dh : 0.0);
    return lin(xq);
  };
  const double h2 = 0.5 / kDbStep;
  for (int w = 0; w < 2; ++w) {
    const int64_t f = w ? fb : fa;
    for (int cc = 0; cc < 9; ++cc) {
      const double gr = (lin_at(w, cc, kDbStep) - lin_at(w, cc, -kDbStep)) * h2;
      atomicAdd(dbsum + f * 9 + cc, gr);
      atomicAdd(dbtsum + f * 9 + cc, t * gr);
    }
  }
}

// Per (chirp, class): the class list reordered by the records' cells (a counting sort; the
// order within a cell is whatever the LDS atomics give, which no result depends on: every
// record's sums stay in its own lane), so that the lanes of a gather wave read neighbouring
// cells of the staged row instead of all of its banks.
__global__ void __launch_bounds__(kNuSortThreads) nufft_adj_sort_kernel(NuShape ns,
                                                                       NuBuffers nb) {
  extern __shared__ int32_t sort_smem[];
  const int ng = ns.ng;
  int32_t *cnt = sort_smem;        // [ng]
  int32_t *part = sort_smem + ng;  // [kNuSortThreads]
  const int64_t lo = static_cast<int64_t>(blockIdx.x) * ns.rec_stride;  // blockIdx = 2 nl + c
  const int32_t count = nb.n_runs[blockIdx.x];
  const int32_t *items = nb.key + lo, *cells = nb.pos + lo;
  const int tid = static_cast<int>(threadIdx.x);
  for (int i = tid; i < ng; i += kNuSortThreads) cnt[i] = 0;
  __syncthreads();
  for (int32_t e = tid; e < count; e += kNuSortThreads) atomicAdd(&cnt[cells[e]], 1);
  __syncthreads();
  const int c0 = 2 * tid;
  const int32_t t0 = c0 < ng ? cnt[c0] : 0, t1 = c0 + 1 < ng ? cnt[c0 + 1] : 0;
  part[tid] = t0 + t1;
  __syncthreads();
  for (int off = 1; off < kNuSortThreads; off <<= 1) {
    const int32_t v = tid >= off ? part[tid - off] : 0;
    __syncthreads();
    part[tid] += v;
    __syncthreads();
  }
  const int32_t base0 = part[tid] - t0 - t1;
  if (c0 < ng) cnt[c0] = base0;
  if (c0 + 1 < ng) cnt[c0 + 1] = base0 + t0;
  __syncthreads();
  for (int32_t e = tid; e < count; e += kNuSortThreads)
    nb.order[lo + atomicAdd(&cnt[cells[e]], 1)] = items[e];
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

__global__ void __launch_bounds__(256) fill_zero_i32_kernel(int32_t *p, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0;
}

// Gaussian-weighted moments mu_k = sum_l g(l) psi(l - x) (l - x)^k, k < K, of a grid row
// over the kNuWidth + 1 cells from the first within W/2 of x = rc0 + xs. With wrap the row
// holds n_g + kNuWidth cells (its first kNuWidth repeated at the end) and the first cell is
// taken modulo n_g; without, the row is a stretch of the grid staged from cell 0 of rc0's
// frame and holds every cell asked for. Either way the reads are fixed offsets from one
// base. With l - x = c + j' (c = s0 + W/2 - xs in (-1, 0],
// j' = j - W/2 in [-W/2, W/2]) the sums T_m = sum g psi j'^m come first, the powers of j'
// being constants of the unrolled loop, and mu_k = sum_m binom(k, m) c^(k - m) T_m (|c| < 1:
// no cancellation).
template <int K>
__device__ __forceinline__ void row_moments(const float2 *row, int ng, bool wrap, int rc0,
                                            float xs, float nc, float q_ratio,
                                            float2 (&mu)[K]) {
  static_assert(K == 2 || K == 4, "moment counts used");
  const float s0 = ceilf(xs - 0.5f * kNuWidth);
  // with wrap in (-ng / 2, 3 ng / 2): the host keeps node and channel offsets within half
  // the grid
  int cell = rc0 + static_cast<int>(s0);
  cell -= (wrap && cell >= ng) ? ng : 0;
  cell += (wrap && cell < 0) ? ng : 0;
  const float2 *rp = row + cell;
  const float u0 = s0 - xs;
  float gw = __builtin_amdgcn_exp2f(nc * u0 * u0);
  float rho = __builtin_amdgcn_exp2f(nc * fmaf(2.0f, u0, 1.0f));
  float2 T[K];
#pragma unroll
  for (int k = 0; k < K; ++k) T[k] = {0.0f, 0.0f};
#pragma unroll
  for (int j = 0; j <= kNuWidth; ++j) {
    const float2 v = rp[j];
    constexpr int h = kNuWidth / 2;
    T[0].x = fmaf(gw, v.x, T[0].x);
    T[0].y = fmaf(gw, v.y, T[0].y);
    if (j != h) {
      const float jp = static_cast<float>(j - h);
      float pw = jp;
#pragma unroll
      for (int m = 1; m < K; ++m) {
        const float gm = gw * pw;
        T[m].x = fmaf(gm, v.x, T[m].x);
        T[m].y = fmaf(gm, v.y, T[m].y);
        pw *= jp;
      }
    }
    gw *= rho;
    rho *= q_ratio;
  }
  const float c = u0 + 0.5f * kNuWidth;
  mu[0] = T[0];
  mu[1] = {fmaf(c, T[0].x, T[1].x), fmaf(c, T[0].y, T[1].y)};
  if constexpr (K == 4) {
    const float c2 = c * c, c3 = c2 * c;
    mu[2] = {fmaf(c2, T[0].x, fmaf(2.0f * c, T[1].x, T[2].x)),
             fmaf(c2, T[0].y, fmaf(2.0f * c, T[1].y, T[2].y))};
    mu[3] = {fmaf(c3, T[0].x, fmaf(3.0f * c2, T[1].x, fmaf(3.0f * c, T[2].x, T[3].x))),
             fmaf(c3, T[0].y, fmaf(3.0f * c2, T[1].y, fmaf(3.0f * c, T[2].y, T[3].y)))};
  }
}

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}

// One lane per (chirp, record of one class), a workgroup per (chirp, class, kNuGatherRecs
// entries of the list ordered by cell), looping over the channels: each channel's grid
// cells that the workgroup's sources reach are staged in LDS (the records of a workgroup
// lie within a few cells of each other, so this is a short stretch of the row; the whole
// row when the stretch would be longer) and every lane forms the moments at its own
// sources, then adds this channel's
// share of the per-facet sums in registers: Re y, dL/dc through the channel's distances,
// and per source parameter sum_o Q mu (weights, coefficients) and sum_o dy/dx_s (offsets).
// Class 0: three points (kind 1); class 1: a point (zero weight for kind 3) and a
// quadratic. Blocks are ordered so that those of one chirp share an XCD (and its L2, which
// holds the chirp's grids).
template <int CLS>
__global__ void __launch_bounds__(kNuGatherRecs) nufft_gather_kernel(
    DevScene sc, RadarConst rc, NuShape ns, const double *elem,
    const NuRecF<false> *__restrict__ recs, const NuDerF *__restrict__ ders,
    const int32_t *__restrict__ lists, const int32_t *__restrict__ counts,
    const float2 *__restrict__ grids, float *partial, int blocks_per_chirp, float *part_db,
    float *el_db, int64_t nb_db_stride) {
  extern __shared__ float2 nu_row[];  // [kNuGatherStage]: rows of consecutive channels,
                                      // each the row and its first cells again, or the
                                      // stretch [lo, lo + span) the sources reach
  __shared__ int32_t reach[3];        // lowest and one past the highest cell reached; 1 if
                                      // some bound lies outside [-n_g, 2 n_g]
  const int per_xcd = (gridDim.x + kXcds - 1) / kXcds;  // gridDim.x is a multiple of kXcds
  const int logical = static_cast<int>(blockIdx.x % kXcds) * per_xcd + static_cast<int>(blockIdx.x / kXcds);
  const int nl = logical / blocks_per_chirp;
  if (nl >= ns.n_chirps) return;  // padding blocks (whole workgroup, before any barrier)
  const int rb = logical - nl * blocks_per_chirp;
  const int n = ns.n0 + nl;
  const int ncls = sc.db_on ? 4 : 2;
  const int32_t count = counts[ncls * nl + CLS];
  if (rb * kNuGatherRecs >= count) return;  // whole workgroup
  const int32_t idx = rb * kNuGatherRecs + static_cast<int32_t>(threadIdx.x);
  const bool on = idx < count;
  const int32_t item =
      on ? lists[static_cast<int64_t>(ncls * nl + CLS) * ns.rec_stride + idx] : 0;
  const int ng = ns.ng;
  const int O = rc.P * rc.Q;
  const int64_t rec_at = static_cast<int64_t>(nl) * ns.rec_stride + item;
  const NuRecF<false> r = recs[on ? rec_at : static_cast<int64_t>(nl) * ns.rec_stride];
  // sources: classes 0 and 2: points j = 0..2 at s[3j]; classes 1 and 3: a point at s[0]
  // and the quadratic at s[3]. Classes 2 and 3 are double-bounce connections: they also
  // sum dL/dR over the channels of each element (for the chain rule through the image
  // elements and the footprint).
  constexpr int SRC = CLS & 1;
  constexpr bool DB = CLS >= 2;
  constexpr int NP = SRC == 0 ? 3 : 1;
  float offp[NP];
  float2 wp[NP];
#pragma unroll
  for (int j = 0; j < NP; ++j) {
    offp[j] = r.s[3 * j];
    wp[j] = on ? make_float2(r.s[3 * j + 1], r.s[3 * j + 2]) : make_float2(0.0f, 0.0f);
  }
  float offq = 0.0f;
  float2 cq[3] = {{0.0f, 0.0f}, {0.0f, 0.0f}, {0.0f, 0.0f}};
  if (SRC == 1) {
    offq = r.s[3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
      cq[k] = on ? make_float2(r.s[4 + 2 * k], r.s[5 + 2 * k]) : make_float2(0.0f, 0.0f);
  }
  const float utf[3] = {static_cast<float>(r.ut[0]), static_cast<float>(r.ut[1]),
                        static_cast<float>(r.ut[2])};
  const float urf[3] = {static_cast<float>(r.ur[0]), static_cast<float>(r.ur[1]),
                        static_cast<float>(r.ur[2])};
  const float nc = static_cast<float>(-1.4426950408889634 / (2.0 * ns.sigma * ns.sigma));
  const float q_ratio = __builtin_amdgcn_exp2f(2.0f * nc);  // exp(-1 / s^2)
  const float inv_s2 = static_cast<float>(1.0 / (ns.sigma * ns.sigma));
  const float kappa = static_cast<float>(ns.kappa);
  const float g2 = static_cast<float>(0.5 * rc.slope / (kC0 * kC0));
  const float two_pi = static_cast<float>(2.0 * kPi);
  const float g1f = static_cast<float>(r.g1);
  float acc_c[3] = {0.0f, 0.0f, 0.0f}, acc_s = 0.0f;
  float2 aw[NP], ax[NP], ac[3], axq = {0.0f, 0.0f};
#pragma unroll
  for (int j = 0; j < NP; ++j) aw[j] = ax[j] = {0.0f, 0.0f};
#pragma unroll
  for (int k = 0; k < 3; ++k) ac[k] = {0.0f, 0.0f};
  const float2 *grow = grids + static_cast<int64_t>(nl) * O * ng;
  // connections: dL/dR per element, one LDS column per lane ([P + Q][kNuGatherRecs] after
  // the staging area)
  float *el_acc = reinterpret_cast<float *>(nu_row + kNuGatherStage);
  if (DB)
    for (int e = 0; e < rc.P + rc.Q; ++e) el_acc[e * kNuGatherRecs + threadIdx.x] = 0.0f;
  // cells the lane's sources reach over every channel: a source at x - off with
  // |x| <= chan_d + 1 cell reads W + 1 cells from ceil(x - off - W/2)
  {
    float mn = -offp[0], mx = -offp[0];
#pragma unroll
    for (int j = 1; j < NP; ++j) {
      mn = fminf(mn, -offp[j]);
      mx = fmaxf(mx, -offp[j]);
    }
    if (SRC == 1) {
      mn = fminf(mn, -offq);
      mx = fmaxf(mx, -offq);
    }
    const float cd = static_cast<float>(ns.chan_d);
    if (threadIdx.x == 0) {
      reach[0] = INT32_MAX;
      reach[1] = INT32_MIN;
      reach[2] = 0;
    }
    __syncthreads();
    const float lo_f = static_cast<float>(r.cell) + floorf(mn - cd - 0.5f * kNuWidth - 1.0f);
    const float hi_f = static_cast<float>(r.cell) + ceilf(mx + cd + 0.5f * kNuWidth + 2.0f);
    if (on) {
      if (lo_f >= -static_cast<float>(ng) && hi_f <= 2.0f * ng) {
        atomicMin(&reach[0], static_cast<int32_t>(lo_f));
        atomicMax(&reach[1], static_cast<int32_t>(hi_f));
      } else {
        atomicOr(&reach[2], 1);
      }
    }
    __syncthreads();
  }
  // workgroup-uniform values, held in scalar registers
  const int32_t lo = __builtin_amdgcn_readfirstlane(reach[0]);
  const int64_t span = static_cast<int64_t>(__builtin_amdgcn_readfirstlane(reach[1])) - lo;
  // the whole row when a source reaches far or the stretch would be as long; else the
  // stretch [lo, lo + span) (lo >= -n_g, lo + span <= 2 n_g)
  const bool wrap = __builtin_amdgcn_readfirstlane(reach[2]) != 0 || span > ng + kNuWidth;
  const int rc0 = wrap ? r.cell : r.cell - lo;
  const int n_stage = wrap ? ng + kNuWidth : static_cast<int>(span);
  const int s_base = wrap ? 0 : (lo % ng + ng) % ng;  // grid cell of the first staged one
  // as many channels' rows per staging (and barrier pair) as kNuGatherStage cells hold
  const int per_stage = max(1, min(O, kNuGatherStage / n_stage));
  for (int o0 = 0; o0 < O; o0 += per_stage) {
  const int nch = min(per_stage, O - o0);
  __syncthreads();  // the previous channels' rows are no longer read
  for (int i = threadIdx.x; i < nch * n_stage; i += blockDim.x) {
    const int ch = i / n_stage, l = i - ch * n_stage;
    int c = s_base + l;  // < 2 n_g + kNuWidth
    c -= (c >= ng) ? ng : 0;
    c -= (c >= ng) ? ng : 0;
    nu_row[i] = grow[static_cast<int64_t>(o0 + ch) * ng + c];
  }
  __syncthreads();
  for (int o = o0; o < o0 + nch; ++o) {
    const float2 *row = nu_row + (o - o0) * n_stage;
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
    const float2 Q = {__builtin_amdgcn_cosf(t) * amp, -__builtin_amdgcn_sinf(t) * amp};
    // y / Q and (dy/dx) / Q over the sources; per-parameter sums
    float2 y = {0.0f, 0.0f}, yx = {0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      float2 mu[2];
      row_moments<2>(row, ng, wrap, rc0, x - offp[j], nc, q_ratio, mu);
      const float2 ys = cmul(wp[j], mu[0]);
      const float2 yxs = cmul(wp[j], make_float2(mu[1].x * inv_s2, mu[1].y * inv_s2));
      y.x += ys.x;
      y.y += ys.y;
      yx.x += yxs.x;
      yx.y += yxs.y;
      const float2 qm = cmul(Q, mu[0]), qx = cmul(Q, yxs);
      aw[j].x += qm.x;
      aw[j].y += qm.y;
      ax[j].x += qx.x;
      ax[j].y += qx.y;
    }
    if (SRC == 1) {
      float2 mu[4];
      row_moments<4>(row, ng, wrap, rc0, x - offq, nc, q_ratio, mu);
      float2 yp = {0.0f, 0.0f}, yxp = {0.0f, 0.0f};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float2 a = cmul(cq[k], mu[k]);
        yp.x += a.x;
        yp.y += a.y;
        float2 d = {mu[k + 1].x * inv_s2, mu[k + 1].y * inv_s2};
        if (k > 0) {
          d.x = fmaf(-static_cast<float>(k), mu[k - 1].x, d.x);
          d.y = fmaf(-static_cast<float>(k), mu[k - 1].y, d.y);
        }
        const float2 b = cmul(cq[k], d);
        yxp.x += b.x;
        yxp.y += b.y;
        const float2 qm = cmul(Q, mu[k]);
        ac[k].x += qm.x;
        ac[k].y += qm.y;
      }
      y.x += yp.x;
      y.y += yp.y;
      yx.x += yxp.x;
      yx.y += yxp.y;
      const float2 qx = cmul(Q, yxp);
      axq.x += qx.x;
      axq.y += qx.y;
    }
    const float2 Y = cmul(Q, y), YX = cmul(Q, yx);
    acc_s += Y.x;
    // dL/dc through the element distances: d Re y / dR = K Im y + kappa Re(dy/dx) - Re y / R
    // (K = 2 pi (f_c - mu tau) / c of this channel), with dR_tp / dc = -e_p
    const float K = two_pi * fmaf(-2.0f * g2, dL, g1f);
    const float A = fmaf(K, Y.y, kappa * YX.x);
    const float ct = A - Y.x * irt, cr = A - Y.x * irr;
    if (DB) {
      el_acc[p * kNuGatherRecs + threadIdx.x] += ct;
      el_acc[(rc.P + q) * kNuGatherRecs + threadIdx.x] += cr;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float ep = (static_cast<float>(at[k]) - r.rt * utf[k]) * irt;
      const float eq = (static_cast<float>(ar[k]) - r.rr * urf[k]) * irr;
      acc_c[k] -= ct * ep + cr * eq;
    }
  }
  }
  if (!on) return;
  // dL/dbeta_v = Re sum (d param / d beta_v) (its sum) - Re sum (d off / d beta_v) sum dy/dx
  const NuDerF dv = ders[rec_at];
  float tv[3];
#pragma unroll
  for (int v = 0; v < 3; ++v) {
    float a = 0.0f;
#pragma unroll
    for (int j = 0; j < NP; ++j) {
      a += aw[j].x * dv.ds[v][3 * j + 1] - aw[j].y * dv.ds[v][3 * j + 2];
      a -= ax[j].x * dv.ds[v][3 * j];
    }
    if (SRC == 1) {
#pragma unroll
      for (int k = 0; k < 3; ++k) a += ac[k].x * dv.ds[v][4 + 2 * k] - ac[k].y * dv.ds[v][5 + 2 * k];
      a -= axq.x * dv.ds[v][3];
    }
    tv[v] = a;
  }
  const int64_t dslot = static_cast<int64_t>(nl) * nb_db_stride + (dv.item - sc.vis_cnt[n]);
  float *slot = DB ? part_db + dslot * kAdjVals
                   : partial + (static_cast<int64_t>(n) * sc.n_facets + dv.item) * kAdjVals;
  if (DB)
    for (int e = 0; e < rc.P + rc.Q; ++e)
      el_db[dslot * (rc.P + rc.Q) + e] = el_acc[e * kNuGatherRecs + threadIdx.x];
  const float vals[kAdjVals] = {acc_c[0], acc_c[1], acc_c[2], acc_s, tv[0], tv[1], tv[2], 0.0f};
#pragma unroll
  for (int k = 0; k < kAdjVals; ++k) slot[k] = vals[k];
}

size_t nufft_smem_bytes(const NuShape &ns) {
  return sizeof(float2) * static_cast<size_t>(2 * ns.cb) * ns.ld;
}
size_t nufft_fft_smem_bytes(const NuShape &ns) {
  return nufft_smem_bytes(ns) + sizeof(int32_t) * static_cast<size_t>(ns.max_runs);
}
// Cells a source covers over all channels of a wave: the integers within W/2 + wave_d of
// its position for the wave's first channel, rounded up to a compiled block length (14,
// 16 or 20; 0 beyond).
int nufft_cells_per_source(const NuShape &ns) {
  const int need = static_cast<int>(std::floor(2.0 * (ns.wave_d + 0.5 * kNuWidth))) + 1;
  return need <= 14 ? 14 : need <= 16 ? 16 : need <= 20 ? 20 : 0;
}

size_t nufft_sort_smem_bytes(const NuShape &ns) {
  return sizeof(int32_t) * (static_cast<size_t>(kNuSortWaves) * ns.ng + ns.ng + 1 + kNuSortThreads);
}

template <bool INTRA>
static hipError_t launch_nufft_t(const DevScene &sc, const RadarConst &rc, const double *elem,
                                 const NuShape &ns, const NuBuffers &nb, const void *tw,
                                 hipStream_t s, const NuBatch &bt, const hipEvent_t *ev) {
  const int64_t items = bt.units ? ns.rec_stride
                                 : sc.n_facets + sc.n_points + (sc.db_on ? 2 * sc.n_facets : 0);
  if (items > 0) {
    dim3 grid(static_cast<unsigned>((items + 255) / 256), static_cast<unsigned>(ns.n_chirps));
    hipLaunchKernelGGL(nufft_key_kernel, grid, dim3(256), 0, s, sc, rc, ns, nb, bt);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(nufft_sort_kernel, dim3(ns.n_chirps), dim3(kNuSortThreads),
                       nufft_sort_smem_bytes(ns), s, sc, ns, nb, bt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((nufft_prep_kernel<INTRA>), grid, dim3(256), 0, s, sc, rc, ns, nb, bt);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
    if ((e = launch_nufft_spread(sc, rc, ns, elem, nb.srec, nb.runs, nb.n_runs, nb.grid, bt, s)) !=
        hipSuccess)
      return e;
    if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  } else {
    // no entries (no facet or point): no runs, so the FFT kernel transforms empty grids
    hipLaunchKernelGGL(fill_zero_i32_kernel, dim3(1), dim3(256), 0, s, nb.n_runs, ns.n_chirps);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(nufft_fft_kernel, dim3(static_cast<unsigned>(ns.n_chirps * ns.groups)),
                     dim3(kNuFftThreads), nufft_fft_smem_bytes(ns), s, sc, rc, ns, nb,
                     static_cast<const float2 *>(tw), bt);
  return hipGetLastError();
}

hipError_t launch_nufft(const DevScene &sc, const RadarConst &rc, const double *elem,
                        const NuShape &ns, const NuBuffers &nb, const void *tw, hipStream_t s,
                        const NuBatch &bt, const hipEvent_t *ev) {
  if (ns.n_chirps <= 0) return hipSuccess;
  if (nufft_record_bytes(rc.intra != 0) > nb.rec_bytes || !nb.runs || !nb.n_runs || !nb.key ||
      !nb.pos || ns.ng > 2 * kNuSortThreads || ns.max_runs < 1 || (bt.units && !bt.scenes))
    return hipErrorInvalidValue;
  return rc.intra ? launch_nufft_t<true>(sc, rc, elem, ns, nb, tw, s, bt, ev)
                  : launch_nufft_t<false>(sc, rc, elem, ns, nb, tw, s, bt, ev);
}

hipError_t launch_nufft_adjoint(const DevScene &sc, const RadarConst &rc, const double *elem,
                                const NuShape &ns, const NuBuffers &nb, const void *tw,
                                const void *grad_echo, float *partial, hipStream_t s,
                                const hipEvent_t *ev, double *dbsum, double *dbtsum) {
  if (ns.n_chirps <= 0) return hipSuccess;
  if (sizeof(NuRecF<false>) > nb.rec_bytes || !nb.sder || !nb.key || !nb.pos || !nb.order ||
      !nb.n_runs || sc.n_points != 0 || rc.intra || ns.ng > 2 * kNuSortThreads)
    return hipErrorInvalidValue;
  if (sc.db_on && (!nb.part_db || !nb.el_db || nb.db_stride < 2 * sc.n_facets || !dbsum ||
                   !dbtsum || ns.rec_stride < 3 * sc.n_facets || rc.P + rc.Q > kNuDbMaxElems))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(nufft_adj_fft_kernel, dim3(static_cast<unsigned>(ns.n_chirps * ns.groups)),
                     dim3(kNuFftThreads), nufft_smem_bytes(ns), s, sc, rc, ns, nb,
                     static_cast<const float2 *>(tw), static_cast<const float2 *>(grad_echo));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t items = sc.n_facets * (sc.db_on ? 3 : 1);  // facets, then connections
  if (sc.n_facets == 0) return hipSuccess;
  const int ncls = sc.db_on ? 4 : 2;
  hipLaunchKernelGGL(fill_zero_i32_kernel, dim3(1), dim3(256), 0, s, nb.n_runs, ncls * ns.n_chirps);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dim3 grid(static_cast<unsigned>((items + 255) / 256), static_cast<unsigned>(ns.n_chirps));
  hipLaunchKernelGGL(nufft_adj_prep_kernel, grid, dim3(256), 0, s, sc, rc, ns, nb, partial);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(nufft_adj_sort_kernel, dim3(static_cast<unsigned>(ncls * ns.n_chirps)),
                     dim3(kNuSortThreads), sizeof(int32_t) * (ns.ng + kNuSortThreads), s, ns, nb);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int bpc = static_cast<int>((items + kNuGatherRecs - 1) / kNuGatherRecs);
  const int64_t blocks = (static_cast<int64_t>(ns.n_chirps) * bpc + kXcds - 1) / kXcds * kXcds;
  const auto *recs = static_cast<const NuRecF<false> *>(nb.srec);
  const auto *ders = static_cast<const NuDerF *>(nb.sder);
  const auto *grids = static_cast<const float2 *>(nb.grid);
  const size_t lds = sizeof(float2) * kNuGatherStage;
  const size_t lds_db = lds + sizeof(float) * (rc.P + rc.Q) * kNuGatherRecs;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  hipLaunchKernelGGL((nufft_gather_kernel<0>), dim3(static_cast<unsigned>(blocks)),
                     dim3(kNuGatherRecs), lds, s, sc, rc, ns, elem, recs, ders, nb.order,
                     nb.n_runs, grids, partial, bpc, nb.part_db, nb.el_db, nb.db_stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL((nufft_gather_kernel<1>), dim3(static_cast<unsigned>(blocks)),
                     dim3(kNuGatherRecs), lds, s, sc, rc, ns, elem, recs, ders, nb.order,
                     nb.n_runs, grids, partial, bpc, nb.part_db, nb.el_db, nb.db_stride);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (sc.db_on) {
    hipLaunchKernelGGL((nufft_gather_kernel<2>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kNuGatherRecs), lds_db, s, sc, rc, ns, elem, recs, ders, nb.order,
                       nb.n_runs, grids, partial, bpc, nb.part_db, nb.el_db, nb.db_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL((nufft_gather_kernel<3>), dim3(static_cast<unsigned>(blocks)),
                       dim3(kNuGatherRecs), lds_db, s, sc, rc, ns, elem, recs, ders, nb.order,
                       nb.n_runs, grids, partial, bpc, nb.part_db, nb.el_db, nb.db_stride);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  if (sc.db_on) {
    dim3 g2(static_cast<unsigned>((2 * sc.n_facets + 127) / 128),
            static_cast<unsigned>(ns.n_chirps));
    hipLaunchKernelGGL(nufft_db_grad_kernel, g2, dim3(128), 0, s, sc, rc, ns, nb, elem, dbsum,
                       dbtsum);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rsim
