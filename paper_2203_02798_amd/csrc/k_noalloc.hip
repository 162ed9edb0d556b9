// sketch_qr_noalloc: sketch_qr with its scratch in a file-scope device array
// instead of a caller workspace, for callers that cannot allocate device
// memory.  The array is one per GPU (each device holds its own copy until the
// process ends); host code reaches it only through the device address that
// hipGetSymbolAddress returns for the current device, resolved once per
// device on the first call there.
#include <map>
#include <mutex>

#include "internal.hpp"

namespace psk {
namespace {

__device__ __align__(256) unsigned char scratch[PSK_NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;  // device -> address of its `scratch`

// the device address of this device's scratch array (the current device's)
int scratch_address(void **out) {
  int dev = 0;
  PSK_HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(dev);
  if (it == g_scratch_ptr.end()) {
    void *p = nullptr;
    PSK_HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PSK_EDEVICE, "hipGetSymbolAddress returned no address for the scratch");
    it = g_scratch_ptr.emplace(dev, p).first;
  }
  *out = it->second;
  return 0;
}

}  // namespace
}  // namespace psk

using namespace psk;

extern "C" int sketch_qr_noalloc(const double *C, int64_t m, int64_t d, double *R, double *Rinv,
                                 void *stream) {
  if (d < 1 || m < d) return fail(PSK_EINVAL, "sketch_qr_noalloc needs m >= d >= 1");
  if (!C || !R || !Rinv) return fail(PSK_EINVAL, "C, R and Rinv must be non-NULL");
  Arena plan;
  int rc = sketch_qr_impl(nullptr, m, d, nullptr, nullptr, plan, nullptr);
  if (rc) return rc;
  if (plan.peak > PSK_NOALLOC_SCRATCH_BYTES)
    return fail(PSK_EUNSUPPORTED,
                "sketch_qr_noalloc: this m x d needs more scratch than PSK_NOALLOC_SCRATCH_BYTES");
  void *base = nullptr;
  if ((rc = scratch_address(&base))) return rc;
  Arena ws = Arena::over(base, PSK_NOALLOC_SCRATCH_BYTES);
  return sketch_qr_impl(C, m, d, R, Rinv, ws, reinterpret_cast<hipStream_t>(stream));
}
