// gp_kmatvec_noalloc: the product of gp_kmatvec for callers that cannot allocate device memory.
//
// The workspace is a file-scope device array of kNoAllocBytes.  Host code never passes the
// array's name to a kernel or a copy (in host code it is only a stand-in symbol): its device
// address is looked up once per device with hipGetSymbolAddress, with that device current, and
// that address is what the product kernels receive as their workspace.
#include <map>
#include <mutex>

#include "gpk.h"
#include "pass.h"

namespace gpk {

gp_status fail(gp_status st, const char *fmt, ...);
void clear_error();
gp_status hip_fail(hipError_t e, const char *where);
gp_status kmatvec_run(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                      int32_t r, const void *V, int64_t ldv, const double *col_shift, void *out,
                      int64_t ldo, void *ws, size_t ws_bytes, hipStream_t stream, size_t cap,
                      bool dry);

namespace {

constexpr size_t kNoAllocBytes = (size_t)64 << 20;

__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_mu;
std::map<int, void *> g_scratch;  // device ordinal -> device address of `scratch`

// Device address of this device's copy of `scratch`, looked up on the first call per device.
gp_status scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  std::lock_guard<std::mutex> lock(g_mu);
  auto it = g_scratch.find(dev);
  if (it == g_scratch.end()) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(GP_ERR_HIP, "hipGetSymbolAddress(scratch) returned NULL");
    it = g_scratch.emplace(dev, p).first;
  }
  *out = it->second;
  return GP_OK;
}

}  // namespace
}  // namespace gpk

using namespace gpk;

extern "C" {

gp_status gp_kmatvec_noalloc(const gp_kernel *k, int64_t n, const void *X, const double *theta,
                             int32_t r, const void *V, int64_t ldv, const double *col_shift,
                             void *out, int64_t ldo, hipStream_t stream) {
  clear_error();
  // every argument check, the fit in the array included, before the first HIP call
  gp_status st = kmatvec_run(k, n, X, theta, r, V, ldv, col_shift, out, ldo, nullptr, 0, stream,
                             kNoAllocBytes, true);
  if (st != GP_OK || n == 0 || r == 0) return st;
  void *ws = nullptr;
  st = scratch_address(&ws);
  if (st != GP_OK) return st;
  return kmatvec_run(k, n, X, theta, r, V, ldv, col_shift, out, ldo, ws, kNoAllocBytes, stream,
                     kNoAllocBytes, false);
}

}  // extern "C"
