// Allocation-free variant of the twist overlap (Sec. III; App. B form
// z = sum_a c_a^2 u_a) for callers that cannot allocate device memory.
//
// mbl_twist_expect keeps its per-workgroup partial sums in a per-basis scratch
// workspace that the library allocates on first use. This variant runs the
// same kernels (the phase-bucket partial sums, then the fixed-order reduce)
// with the partial sums and the reduced values in a file-scope static device
// array instead, so the call performs no device allocation. Its size bounds
// one call to kNoAllocVecs vectors.
//
// Each GPU holds its own copy of the array until the process ends. Host code
// never passes the array's name to a kernel: the name is a host-side stand-in,
// not a device address. The device address is looked up once per device with
// hipGetSymbolAddress (first call on that device, with the device current) and
// kept in g_scratch_ptr. Calls that overlap on one GPU share the array and race.
// Nothing in it needs to start at zero: every partial is written before it is
// read.
#include "mbl_internal.h"

#include <cmath>
#include <mutex>

namespace mbl {

constexpr int kNoAllocVecs = 32;
// partials of one pass: (vector, workgroup, {Re, Im}); then the reduced values
constexpr size_t kNoAllocPartials = (size_t)kNoAllocVecs * kMaxPartials * 2;
constexpr size_t kNoAllocDoubles = kNoAllocPartials + 2 * kNoAllocVecs;

static __device__ __align__(256) double scratch[kNoAllocDoubles];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static double* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's copy of the scratch array.
static mbl_status scratch_of_current_device(int device, double** out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr) {
      set_error(std::string("hipGetSymbolAddress of the static scratch array: ") +
                hipGetErrorString(e));
      return MBL_ERR_HIP;
    }
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return MBL_OK;
}

}  // namespace mbl

using namespace mbl;

extern "C" mbl_status mbl_twist_expect_noalloc(mbl_basis b, const double* psi_dev, int64_t ld,
                                               int nvec, double* z_host, void* stream) {
  clear_error();
  MBL_ARG(b && psi_dev && z_host, "NULL argument");
  MBL_ARG(ld >= b->n, "need ld >= n");
  MBL_ARG(nvec >= 1, "need nvec >= 1");
  MBL_ARG(nvec <= kNoAllocVecs,
          "nvec exceeds the 32 vectors the static scratch of mbl_twist_expect_noalloc holds "
          "(use mbl_twist_expect, or call once per 32 vectors)");
  int device = -1;
  MBL_HIP(hipGetDevice(&device));
  MBL_ARG(device >= 0 && device < kMaxDevices, "device index out of range");
  MBL_ARG(device == b->device, "the basis was built on another device than the current one");
  double* sc = nullptr;
  MBL_TRY(scratch_of_current_device(device, &sc));
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // phase table u_m = exp(i pi m / L), m = 0 .. 2L-1 (host stack arrays)
  const int L = b->L;
  double ct[2 * kMaxL], st[2 * kMaxL];
  const double pi = 3.14159265358979323846;
  for (int m = 0; m < 2 * L; ++m) {
    ct[m] = std::cos(pi * m / L);
    st[m] = std::sin(pi * m / L);
  }
  int G = 0;
  MBL_HIP(launch_twist(b, psi_dev, ld, nvec, ct, st, sc, &G, s));
  if ((size_t)G * nvec * 2 > kNoAllocPartials) {
    // launch_twist keeps G * nvec <= 32 * kMaxPartials; this cannot happen
    set_error("internal: twist partials exceed the static scratch");
    return MBL_ERR_ARG;
  }
  double* red = sc + kNoAllocPartials;
  for (int t = 0; t < nvec; ++t)
    MBL_HIP(launch_reduce(sc + (size_t)t * G * 2, G, 2, 2, red + 2 * t, s));
  MBL_HIP(hipMemcpyAsync(z_host, red, sizeof(double) * 2 * nvec, hipMemcpyDeviceToHost, s));
  MBL_HIP(hipStreamSynchronize(s));
  return MBL_OK;
}
