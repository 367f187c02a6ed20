// Cubic product entry point that allocates nothing (bmm_cubic_noalloc).
//
// bmm_gf2 / bmm_boolean transpose B into a library-owned device buffer that
// grows with hipMalloc.  This variant runs the same transpose and leaf kernels
// with that buffer taken from a fixed, file-scope device array instead, so a
// caller that must not allocate (code under HIP graph capture, serving loops,
// harnesses that forbid hipMalloc) can still pass B untransposed.  Each device
// that runs it holds its own copy of the array until the process ends.
//
// In host code `scratch` names a host-side stand-in, not device memory: the
// device address is looked up once per device with hipGetSymbolAddress (with
// that device current) and only that address is ever handed to a kernel.
#include <mutex>

#include "../../include/bmm.h"
#include "bmm_internal.h"

namespace bmm {
namespace {

constexpr size_t kNoallocScratchBytes = (size_t)BMM_NOALLOC_SCRATCH_BYTES;
static_assert(kNoallocScratchBytes % 256 == 0, "scratch size must keep 256-byte alignment");

__device__ __align__(256) uint64_t scratch[kNoallocScratchBytes / 8];

constexpr int kMaxDevices = 64;
std::once_flag g_once[kMaxDevices];
void* g_ptr[kMaxDevices];
hipError_t g_err[kMaxDevices];

// The device address of `scratch` on the current device (looked up on the
// first call per device).  Returns a bmm status.
int scratch_ptr(void** out) {
  int dev = 0;
  const hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(BMM_E_DEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(BMM_E_UNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::call_once(g_once[dev], [dev] {
    void* p = nullptr;
    g_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    g_ptr[dev] = g_err[dev] == hipSuccess ? p : nullptr;
  });
  if (g_err[dev] != hipSuccess || !g_ptr[dev])
    return set_error(BMM_E_DEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                     hipGetErrorString(g_err[dev]));
  *out = g_ptr[dev];
  return BMM_OK;
}

}  // namespace
}  // namespace bmm

extern "C" int bmm_cubic_noalloc(int semiring, const uint64_t* A, int64_t lda,
                                 const uint64_t* B, int64_t ldb, uint64_t* C, int64_t ldc,
                                 int64_t m, int64_t k, int64_t n, const bmm_options* opt,
                                 void* hip_stream) {
  using namespace bmm;
  if (semiring != BMM_GF2 && semiring != BMM_BOOLEAN)
    return set_error(BMM_E_INVAL, "unknown semiring %d", semiring);
  if (opt && (opt->flags & BMM_FLAG_HOST_OPERANDS))
    return set_error(BMM_E_UNSUPPORTED, "host operands stream through HBM buffers that "
                     "the library allocates: use bmm_ooc");
  const BtScratch bt{kNoallocScratchBytes, &scratch_ptr};
  return cubic_product(semiring, A, lda, B, ldb, C, ldc, m, k, n, opt, hip_stream, &bt);
}
