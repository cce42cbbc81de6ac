// Work memory of the allocation-free range-Doppler entry point (rsim_form_rdm_noalloc).
//
// The buffer is a file-scope device array: every GPU the library runs on holds one copy of
// kStaticScratchBytes from the time the code object is loaded until the process ends, and
// every call on that GPU shares it. Host code never passes the array's name to a kernel (in
// host code it names a host-side stand-in, not device memory): the device address of each
// GPU's copy is looked up once per device with hipGetSymbolAddress (with that device
// current) and only that address is used. Contents persist between calls; the entry point
// rewrites everything it reads (twiddles, then each group of planes) before reading it, so
// nothing needs clearing. Two calls that overlap on one GPU (other streams, other host
// threads, other contexts) share the same memory and race.
#include <hip/hip_runtime.h>

#include <mutex>

#include "rsim_internal.h"
#include "rsim_launch.h"

namespace rsim {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
}  // namespace

hipError_t static_scratch_address(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    if (!ptr) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = ptr;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// tw[i] = exp(-j 2 pi i / L), i < L, from FP64 sincospi (cast to the table's type).
template <typename C>
__global__ void __launch_bounds__(256) twiddle_fill_kernel(C *tw, int L) {
  const int i = static_cast<int>(blockIdx.x * blockDim.x + threadIdx.x);
  if (i >= L) return;
  double s, c;
  sincospi(2.0 * static_cast<double>(i) / static_cast<double>(L), &s, &c);
  using R = decltype(C{}.x);
  tw[i] = C{static_cast<R>(c), static_cast<R>(-s)};
}

hipError_t launch_twiddle_fill(void *tw, int L, int precision, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((L + 255) / 256);
  if (precision)
    hipLaunchKernelGGL(twiddle_fill_kernel<double2>, dim3(grid), dim3(256), 0, s,
                       static_cast<double2 *>(tw), L);
  else
    hipLaunchKernelGGL(twiddle_fill_kernel<float2>, dim3(grid), dim3(256), 0, s,
                       static_cast<float2 *>(tw), L);
  return hipGetLastError();
}

}  // namespace rsim
