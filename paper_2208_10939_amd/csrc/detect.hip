// Detection stage after the RDM (Section 3.3): channel integration, cell-averaging
// CFAR, the 2-D angle FFT over the virtual array (eq. (6)) and the point cloud; and
// additive white Gaussian noise at a set SNR (Section 3.2).
//
// All of it is small next to the facet sum: the integrated map and the CFAR are
// HBM/LDS bound (one pass over the cube, then LDS tiles with a periodic halo), the
// angle transform runs one workgroup per detected cell.
#include "fft_common.h"
#include "rsim.h"

namespace rsim {

// P[c][r] = sum_o rdm[c][o][r] over the O channels, in channel order.
__global__ void __launch_bounds__(256) integrate_kernel(const float *rdm, float *P, int O,
                                                        int64_t NM, int64_t cubes) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cubes * NM) return;
  const int64_t c = idx / NM, r = idx - c * NM;
  const float *src = rdm + c * O * NM + r;
  float s = 0.0f;
  for (int o = 0; o < O; ++o) s += src[o * NM];
  P[idx] = s;
}

constexpr int kCfarTileN = 16, kCfarTileM = 64;

// CA-CFAR over one tile of kCfarTileN x kCfarTileM cells of one cube. The tile and its
// periodic halo (hd = guard + train rows, hr = guard + train bins each side) go to LDS;
// row sums of the full window width and of its two side strips (outside the guard
// columns) are formed first, then the training sum of each cell as the full-width row
// sums of the rows outside the guard band plus the side-strip sums of the rows inside
// it. No subtraction, so a strong cell under test cannot cancel against its ring.
__global__ void __launch_bounds__(256) cfar_kernel(const float *P, int N, int M, int gd, int gr,
                                                   int td, int tr, float scale, float inv_k,
                                                   int tiles_n, int tiles_m, uint8_t *det,
                                                   float *noise) {
  extern __shared__ __align__(16) unsigned char cfar_smem[];
  const int hd = gd + td, hr = gr + tr;
  const int rows = kCfarTileN + 2 * hd, cols = kCfarTileM + 2 * hr;
  float *tile = reinterpret_cast<float *>(cfar_smem);  // [rows][cols]
  float *rs_full = tile + rows * cols;                   // [rows][kCfarTileM]
  float *rs_side = rs_full + rows * kCfarTileM;          // [rows][kCfarTileM]
  const int per_cube = tiles_n * tiles_m;
  const int64_t c = blockIdx.x / per_cube;
  const int t = blockIdx.x % per_cube;
  const int n0 = (t / tiles_m) * kCfarTileN, m0 = (t % tiles_m) * kCfarTileM;
  const float *src = P + c * static_cast<int64_t>(N) * M;
  for (int i = threadIdx.x; i < rows * cols; i += blockDim.x) {
    const int r = i / cols, q = i - r * cols;
    const int n = ((n0 - hd + r) % N + N) % N;
    const int m = ((m0 - hr + q) % M + M) % M;
    tile[i] = src[static_cast<int64_t>(n) * M + m];
  }
  __syncthreads();
  for (int i = threadIdx.x; i < rows * kCfarTileM; i += blockDim.x) {
    const int r = i / kCfarTileM, q = i - r * kCfarTileM;
    const float *row = tile + r * cols + q;  // window columns q .. q + 2 hr
    float left = 0.0f, right = 0.0f, mid = 0.0f;
    for (int k = 0; k < tr; ++k) {
      left += row[k];
      right += row[2 * hr - k];
    }
    for (int k = tr; k <= 2 * hr - tr; ++k) mid += row[k];
    rs_side[i] = left + right;
    rs_full[i] = (left + right) + mid;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kCfarTileN * kCfarTileM; i += blockDim.x) {
    const int r = i / kCfarTileM, q = i - r * kCfarTileM;
    const int n = n0 + r, m = m0 + q;
    if (n >= N || m >= M) continue;
    float train = 0.0f;
    for (int k = 0; k < td; ++k) train += rs_full[(r + k) * kCfarTileM + q];
    for (int k = td; k <= 2 * hd - td; ++k) train += rs_side[(r + k) * kCfarTileM + q];
    for (int k = 2 * hd - td + 1; k <= 2 * hd; ++k) train += rs_full[(r + k) * kCfarTileM + q];
    const float nz = train * inv_k;
    const float cut = tile[(r + hd) * cols + q + hr];
    const int64_t g = c * static_cast<int64_t>(N) * M + static_cast<int64_t>(n) * M + m;
    det[g] = cut > scale * nz ? 1 : 0;
    noise[g] = nz;
  }
}

// Row-major list of the detected cells of one cube (first max_points), and the count.
__global__ void __launch_bounds__(1024) det_list_kernel(const uint8_t *det, int64_t NM,
                                                        int max_points, int32_t *list,
                                                        int32_t *count) {
  __shared__ int32_t wave_tot[16];
  __shared__ int32_t s_base;
  const int64_t c = blockIdx.x;
  const uint8_t *d = det + c * NM;
  int32_t *out = list + c * max_points;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int waves = blockDim.x >> 6;
  if (threadIdx.x == 0) s_base = 0;
  __syncthreads();
  for (int64_t k0 = 0; k0 < NM; k0 += blockDim.x) {
    const int64_t k = k0 + threadIdx.x;
    const bool f = k < NM && d[k] != 0;
    const uint64_t bal = __ballot(f);
    const int before = __popcll(bal & ((1ull << lane) - 1ull));
    if (lane == 0) wave_tot[wv] = __popcll(bal);
    __syncthreads();
    int off = s_base;
    for (int w = 0; w < wv; ++w) off += wave_tot[w];
    if (f && off + before < max_points) out[off + before] = static_cast<int32_t>(k);
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < waves; ++w) tot += wave_tot[w];
      s_base += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) count[c] = s_base;
}

struct AngleParams {
  int O, N, M, na_x, na_z, n_nodes, max_points;
  int pad;
  double range_res, vel_res;
  double c_ref[3];
};

// One workgroup per listed cell: the channels of Y at that cell averaged onto their
// grid nodes (node_off/node_ch: channels of each node, in channel order), a 2-D FFT
// (rows along x, then a transpose and the columns along z), and the first maximum of
// |A|^2 in row-major (z, x) order.
__global__ void __launch_bounds__(256) angle_kernel(const float2 *y, const float *P,
                                                    const float *noise, const int32_t *list,
                                                    const int32_t *count, const int32_t *node_pos,
                                                    const int32_t *node_off,
                                                    const int32_t *node_ch, const float2 *tw_x,
                                                    const float2 *tw_z, AngleParams ap,
                                                    rsim_point *points) {
  extern __shared__ __align__(16) unsigned char ang_smem[];
  __shared__ float s_val[256];
  __shared__ int32_t s_idx[256];
  const int64_t c = blockIdx.x / ap.max_points;
  const int slot = blockIdx.x % ap.max_points;
  const int32_t cnt = min(count[c], ap.max_points);
  if (slot >= cnt) return;  // whole workgroup leaves before any barrier
  const int L = ap.na_x * ap.na_z;
  float2 *a = reinterpret_cast<float2 *>(ang_smem);
  float2 *b = a + L;
  const int64_t NM = static_cast<int64_t>(ap.N) * ap.M;
  const int32_t cell = list[c * ap.max_points + slot];
  for (int i = threadIdx.x; i < L; i += blockDim.x) a[i] = make_float2(0.0f, 0.0f);
  __syncthreads();
  const float2 *yc = y + c * ap.O * NM + cell;
  for (int k = threadIdx.x; k < ap.n_nodes; k += blockDim.x) {
    float sx = 0.0f, sy = 0.0f;
    const int e0 = node_off[k], e1 = node_off[k + 1];
    for (int e = e0; e < e1; ++e) {
      const float2 v = yc[static_cast<int64_t>(node_ch[e]) * NM];
      sx += v.x;
      sy += v.y;
    }
    const float inv = 1.0f / static_cast<float>(e1 - e0);
    a[node_pos[k]] = make_float2(sx * inv, sy * inv);
  }
  __syncthreads();
  float2 *r1 = stockham<float2>(a, b, ap.na_x, ap.na_z, ap.na_x, tw_x);  // rows along x
  float2 *t = (r1 == a) ? b : a;
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    const int kz = i / ap.na_x, kx = i - kz * ap.na_x;
    t[kx * ap.na_z + kz] = r1[i];
  }
  __syncthreads();
  float2 *r2 = t;
  if (ap.na_z > 1) r2 = stockham<float2>(t, r1, ap.na_z, ap.na_x, ap.na_z, tw_z);
  // first maximum in row-major (kz, kx) order
  float best = -1.0f;
  int32_t bidx = 0x7fffffff;
  for (int i = threadIdx.x; i < L; i += blockDim.x) {
    const int kz = i / ap.na_x, kx = i - kz * ap.na_x;
    const float2 v = r2[kx * ap.na_z + kz];
    const float p = v.x * v.x + v.y * v.y;
    if (p > best) {  // i grows within a thread, so ties keep the first index
      best = p;
      bidx = i;
    }
  }
  s_val[threadIdx.x] = best;
  s_idx[threadIdx.x] = bidx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < static_cast<unsigned>(s)) {
      const float v2 = s_val[threadIdx.x + s];
      const int32_t i2 = s_idx[threadIdx.x + s];
      if (v2 > s_val[threadIdx.x] || (v2 == s_val[threadIdx.x] && i2 < s_idx[threadIdx.x])) {
        s_val[threadIdx.x] = v2;
        s_idx[threadIdx.x] = i2;
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int flat = s_idx[0];
    const int kz = flat / ap.na_x, kx = flat - kz * ap.na_x;
    const int skx = kx >= (ap.na_x + 1) / 2 ? kx - ap.na_x : kx;
    const int skz = kz >= (ap.na_z + 1) / 2 ? kz - ap.na_z : kz;
    const double u = -2.0 * skx / ap.na_x;
    const double w = ap.na_z > 1 ? -2.0 * skz / ap.na_z : 0.0;
    const int n = cell / ap.M, m = cell - n * ap.M;
    const double R = m * ap.range_res;
    const double dy = sqrt(fmax(0.0, 1.0 - u * u - w * w));
    rsim_point pt;
    pt.row = n;
    pt.bin = m;
    pt.power = P[c * NM + cell];
    pt.noise = noise[c * NM + cell];
    pt.range_m = static_cast<float>(R);
    pt.velocity_mps = static_cast<float>((n - ap.N / 2) * ap.vel_res);
    pt.u = static_cast<float>(u);
    pt.w = static_cast<float>(w);
    pt.x = static_cast<float>(ap.c_ref[0] + R * u);
    pt.y = static_cast<float>(ap.c_ref[1] + R * dy);
    pt.z = static_cast<float>(ap.c_ref[2] + R * w);
    pt.angle_power = s_val[0];
    pt.kx = skx;
    pt.kz = skz;
    pt.reserved[0] = pt.reserved[1] = 0;
    points[c * ap.max_points + slot] = pt;
  }
}

// ---- white Gaussian noise --------------------------------------------------------------

// Philox4x32 with 10 rounds (Salmon et al., SC 2011): round multipliers 0xD2511F53 and
// 0xCD9E8D57, key increments 0x9E3779B9 and 0xBB67AE85.
__device__ inline uint4 philox4x32_10(uint4 x, uint2 k) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k.x += 0x9E3779B9u;
      k.y += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, x.x), lo0 = 0xD2511F53u * x.x;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, x.z), lo1 = 0xCD9E8D57u * x.z;
    x = make_uint4(hi1 ^ x.y ^ k.x, lo1, hi0 ^ x.w ^ k.y, lo0);
  }
  return x;
}

constexpr int kPowerBlocks = 256;

// Per cube: partial sums of |H|^2 in FP64 over kPowerBlocks fixed slices.
template <typename C>
__global__ void __launch_bounds__(256) power_partial_kernel(const C *h, int64_t n, double *part) {
  __shared__ double s[256];
  const int64_t c = blockIdx.y;
  const int b = blockIdx.x;
  const int64_t chunk = (n + kPowerBlocks - 1) / kPowerBlocks;
  const int64_t lo = b * chunk, hi = min(n, lo + chunk);
  const C *src = h + c * n;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const double x = src[i].x, y = src[i].y;
    acc += x * x + y * y;
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < static_cast<unsigned>(w)) s[threadIdx.x] += s[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[c * kPowerBlocks + b] = s[0];
}

// Per cube: the per-part noise standard deviation sqrt(mean |H|^2 / snr / 2).
__global__ void noise_scale_kernel(const double *part, int64_t n, int64_t cubes, double inv_snr,
                                   double *scale) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= cubes) return;
  double s = 0.0;
  for (int b = 0; b < kPowerBlocks; ++b) s += part[c * kPowerBlocks + b];
  scale[c] = sqrt(0.5 * (s / static_cast<double>(n)) * inv_snr);
}

template <typename C>
__global__ void __launch_bounds__(256) add_noise_kernel(C *h, int64_t n, int64_t cubes,
                                                        const double *scale, uint2 key) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= cubes * n) return;
  const int64_t c = idx / n, i = idx - c * n;
  const uint4 x = philox4x32_10(make_uint4(static_cast<uint32_t>(i), static_cast<uint32_t>(i >> 32),
                                           static_cast<uint32_t>(c), 0u), key);
  const double u1 = (static_cast<double>(x.x) + 0.5) * 0x1p-32;
  const double u2 = (static_cast<double>(x.y) + 0.5) * 0x1p-32;
  const double r = sqrt(-2.0 * log(u1)) * scale[c];
  double sn, cs;
  sincospi(2.0 * u2, &sn, &cs);
  C v = h[idx];
  v.x += r * cs;
  v.y += r * sn;
  h[idx] = v;
}

// ---- host launches -----------------------------------------------------------------------

size_t cfar_smem_bytes(int gd, int gr, int td, int tr) {
  const int hd = gd + td, hr = gr + tr;
  const size_t rows = kCfarTileN + 2 * hd;
  return sizeof(float) * (rows * (kCfarTileM + 2 * hr) + 2 * rows * kCfarTileM);
}

size_t angle_smem_bytes(int na_x, int na_z) {
  return 2 * sizeof(float2) * static_cast<size_t>(na_x) * na_z;
}

hipError_t launch_detect(const float *rdm, const void *y, int64_t cubes, int O, int N, int M,
                         int gd, int gr, int td, int tr, float scale, int na_x, int na_z,
                         int max_points, double range_res, double vel_res, const double *c_ref,
                         const int32_t *node_pos, const int32_t *node_off,
                         const int32_t *node_ch, int n_nodes, const void *tw_x, const void *tw_z,
                         float *P, uint8_t *det, float *noise, int32_t *list, int32_t *count,
                         void *points, hipStream_t s) {
  const int64_t NM = static_cast<int64_t>(N) * M;
  hipLaunchKernelGGL(integrate_kernel, dim3(static_cast<unsigned>((cubes * NM + 255) / 256)),
                     dim3(256), 0, s, rdm, P, O, NM, cubes);
  const int tiles_n = (N + kCfarTileN - 1) / kCfarTileN, tiles_m = (M + kCfarTileM - 1) / kCfarTileM;
  const int K = (2 * (gd + td) + 1) * (2 * (gr + tr) + 1) - (2 * gd + 1) * (2 * gr + 1);
  hipLaunchKernelGGL(cfar_kernel, dim3(static_cast<unsigned>(cubes * tiles_n * tiles_m)), dim3(256),
                     cfar_smem_bytes(gd, gr, td, tr), s, P, N, M, gd, gr, td, tr, scale,
                     1.0f / static_cast<float>(K), tiles_n, tiles_m, det, noise);
  hipLaunchKernelGGL(det_list_kernel, dim3(static_cast<unsigned>(cubes)), dim3(1024), 0, s, det, NM,
                     max_points, list, count);
  AngleParams ap{O, N, M, na_x, na_z, n_nodes, max_points, 0, range_res, vel_res,
                 {c_ref[0], c_ref[1], c_ref[2]}};
  hipLaunchKernelGGL(angle_kernel, dim3(static_cast<unsigned>(cubes * max_points)), dim3(256),
                     angle_smem_bytes(na_x, na_z), s, static_cast<const float2 *>(y), P, noise,
                     list, count, node_pos, node_off, node_ch, static_cast<const float2 *>(tw_x),
                     static_cast<const float2 *>(tw_z), ap, static_cast<rsim_point *>(points));
  return hipGetLastError();
}

hipError_t launch_add_noise(int precision, void *echo, int64_t n, int64_t cubes, double snr_db,
                            uint64_t seed, double *part, double *scale, hipStream_t s) {
  const double inv_snr = pow(10.0, -snr_db / 10.0);
  const uint2 key = make_uint2(static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  const dim3 pg(kPowerBlocks, static_cast<unsigned>(cubes));
  const unsigned grid = static_cast<unsigned>((cubes * n + 255) / 256);
  if (precision) {
    hipLaunchKernelGGL(power_partial_kernel<double2>, pg, dim3(256), 0, s,
                       static_cast<const double2 *>(echo), n, part);
    hipLaunchKernelGGL(noise_scale_kernel, dim3(static_cast<unsigned>((cubes + 63) / 64)), dim3(64),
                       0, s, part, n, cubes, inv_snr, scale);
    hipLaunchKernelGGL(add_noise_kernel<double2>, dim3(grid), dim3(256), 0, s,
                       static_cast<double2 *>(echo), n, cubes, scale, key);
  } else {
    hipLaunchKernelGGL(power_partial_kernel<float2>, pg, dim3(256), 0, s,
                       static_cast<const float2 *>(echo), n, part);
    hipLaunchKernelGGL(noise_scale_kernel, dim3(static_cast<unsigned>((cubes + 63) / 64)), dim3(64),
                       0, s, part, n, cubes, inv_snr, scale);
    hipLaunchKernelGGL(add_noise_kernel<float2>, dim3(grid), dim3(256), 0, s,
                       static_cast<float2 *>(echo), n, cubes, scale, key);
  }
  return hipGetLastError();
}

int noise_partials_per_cube() { return kPowerBlocks; }

}  // namespace rsim
