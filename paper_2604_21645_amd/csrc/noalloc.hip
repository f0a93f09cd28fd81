// Encode without a caller workspace: the scratch memory of mipq_pq_encode
// (packed centroid operands, squared-error partials) lives in a fixed device
// array of the library, one copy per GPU, so the call allocates nothing.
//
// In host code the array's name is only a stand-in for the symbol; its device
// address is taken once per device with hipGetSymbolAddress (with that device
// current) and kept in g_scratch_ptr, which is what the kernels receive.
#include <mutex>

#include "mipq_internal.h"

namespace mipq {
namespace {

constexpr size_t kNoallocBytes = MIPQ_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kNoallocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this GPU's scratch array (looked up on first use)
int scratch_for_current_device(void** out) {
  int dev = 0;
  MIPQ_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(MIPQ_EUNSUPPORTED, "device index %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    MIPQ_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(MIPQ_EHIP, "hipGetSymbolAddress returned no address for the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MIPQ_OK;
}

}  // namespace
}  // namespace mipq

using namespace mipq;

extern "C" {

int mipq_pq_encode_noalloc(const float* x, int64_t n, int d, int m, int ks, const float* codebook, int precision,
                           int flags, uint8_t* codes, float* min_dist, double* sse_rmse, int64_t* rescored,
                           void* stream) {
  if (n < 0 || n > MIPQ_NOALLOC_MAX_N)
    return fail(MIPQ_EINVAL, "pq_encode_noalloc: n=%lld outside [0, %lld]", (long long)n,
                (long long)MIPQ_NOALLOC_MAX_N);
  if (flags & MIPQ_CHECK_FINITE)
    return fail(MIPQ_EINVAL, "pq_encode_noalloc: MIPQ_CHECK_FINITE copies to the host; use mipq_pq_encode");
  const size_t need = mipq_pq_encode_workspace_size(n, d, m, ks, precision);
  if (need == 0) {   // invalid shape or precision: the full call reports why
    return mipq_pq_encode(x, n, d, m, ks, codebook, precision, flags, codes, min_dist, sse_rmse, rescored, nullptr,
                          0, stream);
  }
  if (need > kNoallocBytes)
    return fail(MIPQ_ENOMEM, "pq_encode_noalloc: needs %zu bytes of scratch, the fixed array holds %zu", need,
                kNoallocBytes);
  void* ws = nullptr;
  int rc;
  if ((rc = scratch_for_current_device(&ws))) return rc;
  return mipq_pq_encode(x, n, d, m, ks, codebook, precision, flags, codes, min_dist, sse_rmse, rescored, ws,
                        kNoallocBytes, stream);
}

}  // extern "C"
