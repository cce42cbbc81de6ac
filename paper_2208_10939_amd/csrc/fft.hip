// Range and Doppler transforms (Section 3.3; eqs. (4), (5), (10)-(11)).
//
// The beat signal is x = conj(H) (eq. (13) under stretch processing); the range
// transform X = FFT_m(x) is the paper's inverse transform of the frequency-domain
// echo, up to conjugation and the factor M. The Doppler transform Y = FFT_n(X) puts
// zero Doppler in row N/2; the RDM is |Y|^2. Unnormalised, no window.
//
// Both are HBM-bound: each workgroup loads a block of rows (range) or a tile of
// columns (Doppler, coalesced along the range axis) into LDS, runs a mixed radix-4/2/3
// Stockham FFT there and writes the result once. Twiddles come from an FP64-
// accurate table, tw[i] = exp(-j 2 pi i / L), i < L.
#include "fft_common.h"

namespace rsim {

// Rows of length M: out[row] = FFT(conj_in ? conj(in[row]) : in[row]).
template <typename R>
__global__ void __launch_bounds__(256) range_fft_kernel(const typename Cx2<R>::T *in,
                                                        typename Cx2<R>::T *out, int64_t rows,
                                                        int M, int rows_per_wg, int conj_in,
                                                        const typename Cx2<R>::T *tw) {
  using C = typename Cx2<R>::T;
  extern __shared__ __align__(16) unsigned char fft_smem[];
  C *a = reinterpret_cast<C *>(fft_smem);
  C *b = a + rows_per_wg * M;
  const int64_t row0 = static_cast<int64_t>(blockIdx.x) * rows_per_wg;
  const int nrow = static_cast<int>(min<int64_t>(rows_per_wg, rows - row0));
  const C *src = in + row0 * M;
  for (int i = threadIdx.x; i < nrow * M; i += blockDim.x) {
    C v = src[i];
    if (conj_in) v.y = -v.y;
    a[i] = v;
  }
  __syncthreads();
  C *res = stockham<C>(a, b, M, nrow, M, tw);
  C *dst = out + row0 * M;
  for (int i = threadIdx.x; i < nrow * M; i += blockDim.x) dst[i] = res[i];
}

// Columns of length N (stride M) of each channel's [N][M] plane.
// mode 0 (forward): Y = shift_n(FFT_n(X)), row l holding Doppler index l - floor(N/2) for
//   even and odd N alike; writes rdm = |Y|^2 and y_out if given.
// mode 1 (adjoint input side): Z = FFT_n(conj(unshift_n(G))) written to y_out.
// mode 2 (RDM backward): as mode 1 with G = 2 (dL/dP) Y formed on the fly from
//   gp = dL/dP (rdm-shaped) and in = Y, since P = |Y|^2.
template <typename R>
__global__ void __launch_bounds__(256) doppler_fft_kernel(const typename Cx2<R>::T *in,
                                                          typename Cx2<R>::T *y_out, R *rdm,
                                                          int64_t planes, int N, int M, int kt,
                                                          int mode, const typename Cx2<R>::T *tw,
                                                          const R *gp) {
  using C = typename Cx2<R>::T;
  extern __shared__ __align__(16) unsigned char fft_smem[];
  const int ld = N + 1;
  C *a = reinterpret_cast<C *>(fft_smem);
  C *b = a + kt * ld;
  const int tiles = (M + kt - 1) / kt;
  const int64_t plane = blockIdx.x / tiles;
  const int k0 = (blockIdx.x % tiles) * kt;
  const int ncol = min(kt, M - k0);
  const C *src = in + plane * static_cast<int64_t>(N) * M;
  const int hN = N >> 1;
  for (int idx = threadIdx.x; idx < N * kt; idx += blockDim.x) {
    const int n = idx / kt, c = idx - n * kt;
    if (c >= ncol) continue;
    if (mode == 0) {
      a[c * ld + n] = src[static_cast<int64_t>(n) * M + k0 + c];
    } else {
      // row l of G holds Doppler index l' = l - floor(N/2); place it at l' mod N, conjugated
      const int lp = (n + N - hN) % N;
      const int64_t gi = static_cast<int64_t>(n) * M + k0 + c;
      C v = src[gi];
      if (mode == 2) {
        const R s = R(2) * gp[plane * static_cast<int64_t>(N) * M + gi];
        v.x *= s;
        v.y *= s;
      }
      v.y = -v.y;
      a[c * ld + lp] = v;
    }
  }
  __syncthreads();
  C *res = stockham<C>(a, b, N, kt, ld, tw);
  const int64_t base = plane * static_cast<int64_t>(N) * M;
  for (int idx = threadIdx.x; idx < N * kt; idx += blockDim.x) {
    const int l = idx / kt, c = idx - l * kt;
    if (c >= ncol) continue;
    const int64_t g = base + static_cast<int64_t>(l) * M + k0 + c;
    if (mode == 0) {
      const C v = res[c * ld + (l + N - hN) % N];  // row l <- index l - floor(N/2)
      if (rdm) rdm[g] = v.x * v.x + v.y * v.y;
      if (y_out) y_out[g] = v;
    } else {
      y_out[g] = res[c * ld + l];
    }
  }
}

template <typename R>
static hipError_t launch_range_t(const void *in, void *out, int64_t rows, int M, int conj_in,
                                 const void *tw, hipStream_t s) {
  using C = typename Cx2<R>::T;
  const int budget = (sizeof(R) == 4) ? 2048 : 1024;  // points per workgroup (2 buffers in LDS)
  const int rpw = max(1, budget / M);
  const unsigned grid = static_cast<unsigned>((rows + rpw - 1) / rpw);
  const size_t lds = 2 * sizeof(C) * rpw * M;
  hipLaunchKernelGGL(range_fft_kernel<R>, dim3(grid), dim3(256), lds, s,
                     static_cast<const C *>(in), static_cast<C *>(out), rows, M, rpw, conj_in,
                     static_cast<const C *>(tw));
  return hipGetLastError();
}

template <typename R>
static hipError_t launch_doppler_t(const void *in, void *y_out, void *rdm, int64_t planes, int N,
                                   int M, int mode, const void *tw, hipStream_t s,
                                   const void *gp) {
  using C = typename Cx2<R>::T;
  const int budget = (sizeof(R) == 4) ? 2048 : 1024;
  int kt = max(1, min(32, budget / N));
  kt = min(kt, M);
  const int tiles = (M + kt - 1) / kt;
  const unsigned grid = static_cast<unsigned>(planes * tiles);
  const size_t lds = 2 * sizeof(C) * kt * (N + 1);
  hipLaunchKernelGGL(doppler_fft_kernel<R>, dim3(grid), dim3(256), lds, s,
                     static_cast<const C *>(in), static_cast<C *>(y_out), static_cast<R *>(rdm),
                     planes, N, M, kt, mode, static_cast<const C *>(tw),
                     static_cast<const R *>(gp));
  return hipGetLastError();
}

hipError_t launch_range_fft(int precision, const void *in, void *out, int64_t rows, int M,
                            int conj_in, const void *tw, hipStream_t s) {
  return precision ? launch_range_t<double>(in, out, rows, M, conj_in, tw, s)
                   : launch_range_t<float>(in, out, rows, M, conj_in, tw, s);
}

hipError_t launch_doppler_fft(int precision, const void *in, void *y_out, void *rdm,
                              int64_t planes, int N, int M, int mode, const void *tw,
                              hipStream_t s, const void *gp) {
  return precision ? launch_doppler_t<double>(in, y_out, rdm, planes, N, M, mode, tw, s, gp)
                   : launch_doppler_t<float>(in, y_out, rdm, planes, N, M, mode, tw, s, gp);
}

}  // namespace rsim
