// In-LDS mixed radix-4/2/3 Stockham FFT shared by the range/Doppler transforms and the
// angle transform of the detection stage.
#pragma once

#include "rsim_internal.h"
#include "rsim_launch.h"

namespace rsim {

template <typename R>
struct Cx2;
template <>
struct Cx2<float> {
  using T = float2;
};
template <>
struct Cx2<double> {
  using T = double2;
};

// In-LDS Stockham autosort FFT over nseq sequences of length L = 2^a 3^b (radix-4 passes
// while two factors of 2 remain, a radix-2 pass for an odd one, then radix-3 passes: fewer
// passes, so fewer barriers and LDS round trips); sequence s starts at s * ld. Pass with
// radix R after
// sub-transforms of length ns: butterfly j < L/R takes x_i = a[j + i L/R], twiddles
// them by exp(-j 2 pi i k / (ns R)) with k = j mod ns, and writes the R-point DFT to
// b[(j / ns) ns R + k + i ns], so the output stays in natural order. tw holds
// exp(-j 2 pi t / L) for t < L. Returns the buffer (a or b) holding the result.
template <typename C>
__device__ C *stockham(C *a, C *b, int L, int nseq, int ld, const C *tw) {
  using R = decltype(C{}.x);
  int twos = 0, rest = L;
  while ((rest & 1) == 0) {
    rest >>= 1;
    ++twos;
  }
  int ns = 1;
  while (ns < L) {
    const int radix = (twos >= 2) ? 4 : (twos == 1) ? 2 : 3;
    twos -= (radix == 4) ? 2 : (radix == 2) ? 1 : 0;
    const int span = L / radix;
    const int tstep = L / (ns * radix);  // twiddle index step per unit of i * k
    for (int idx = threadIdx.x; idx < nseq * span; idx += blockDim.x) {
      const int s = idx / span;
      const int j = idx - s * span;
      const int k = j % ns;
      const int o = s * ld + (j / ns) * ns * radix + k;
      const C *src = a + s * ld + j;
      if (radix == 4) {
        const C x0 = src[0];
        const C y1 = src[span], y2 = src[2 * span], y3 = src[3 * span];
        const C w1 = tw[k * tstep], w2 = tw[2 * k * tstep], w3 = tw[3 * k * tstep];
        const C x1 = {w1.x * y1.x - w1.y * y1.y, w1.x * y1.y + w1.y * y1.x};
        const C x2 = {w2.x * y2.x - w2.y * y2.y, w2.x * y2.y + w2.y * y2.x};
        const C x3 = {w3.x * y3.x - w3.y * y3.y, w3.x * y3.y + w3.y * y3.x};
        // X_q = sum_i x_i exp(-j 2 pi i q / 4): X0,2 = (x0 + x2) +/- (x1 + x3),
        // X1,3 = (x0 - x2) -/+ j (x1 - x3)
        const C s02 = {x0.x + x2.x, x0.y + x2.y}, d02 = {x0.x - x2.x, x0.y - x2.y};
        const C s13 = {x1.x + x3.x, x1.y + x3.y}, d13 = {x1.x - x3.x, x1.y - x3.y};
        b[o] = {s02.x + s13.x, s02.y + s13.y};
        b[o + ns] = {d02.x + d13.y, d02.y - d13.x};
        b[o + 2 * ns] = {s02.x - s13.x, s02.y - s13.y};
        b[o + 3 * ns] = {d02.x - d13.y, d02.y + d13.x};
      } else if (radix == 2) {
        const C x0 = src[0];
        const C x1 = src[span];
        const C w = tw[k * tstep];
        const C t = {w.x * x1.x - w.y * x1.y, w.x * x1.y + w.y * x1.x};
        b[o] = {x0.x + t.x, x0.y + t.y};
        b[o + ns] = {x0.x - t.x, x0.y - t.y};
      } else {
        const C x0 = src[0];
        const C y1 = src[span], y2 = src[2 * span];
        const C w1 = tw[k * tstep], w2 = tw[2 * k * tstep];
        const C x1 = {w1.x * y1.x - w1.y * y1.y, w1.x * y1.y + w1.y * y1.x};
        const C x2 = {w2.x * y2.x - w2.y * y2.y, w2.x * y2.y + w2.y * y2.x};
        // X0 = x0 + x1 + x2; X1,2 = x0 - (x1 + x2)/2 -/+ j (sqrt(3)/2)(x1 - x2)
        const R h = R(0.86602540378443864676);
        const C t1 = {x1.x + x2.x, x1.y + x2.y};
        const C t2 = {x0.x - R(0.5) * t1.x, x0.y - R(0.5) * t1.y};
        const C t3 = {h * (x1.y - x2.y), -h * (x1.x - x2.x)};  // -j h (x1 - x2)
        b[o] = {x0.x + t1.x, x0.y + t1.y};
        b[o + ns] = {t2.x + t3.x, t2.y + t3.y};
        b[o + 2 * ns] = {t2.x - t3.x, t2.y - t3.y};
      }
    }
    __syncthreads();
    C *tmp = a;
    a = b;
    b = tmp;
    ns *= radix;
  }
  return a;
}

}  // namespace rsim
