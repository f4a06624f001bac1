// fs_decode_noalloc: the decode of fs_decode with its workspace in a fixed
// device array of the library instead of caller memory, for callers that
// cannot allocate (code under stream capture, tight request loops, harnesses
// that forbid allocation calls).
//
// `scratch` is one file-scope device array; every GPU the library runs on
// holds its own copy until the process ends.  Its name is not a device address
// in host code: the address of this device's copy comes from
// hipGetSymbolAddress, taken once per device with that device current and
// kept in scratch_ptr[], and only that pointer is handed to kernels.  The
// decode kernels initialise every workspace byte they read, so nothing has to
// be cleared between calls; calls that overlap on one device share the array
// and race.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "fs_internal.h"

namespace fs {
namespace {

constexpr size_t kScratchBytes = size_t(16) << 20;
constexpr int kMaxDevices = 64;

__device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex scratch_mu;
void *scratch_ptr[kMaxDevices] = {};

fs_status scratch_for_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(FS_ERR_HIP, "fs_decode_noalloc: no current device");
  std::lock_guard<std::mutex> lock(scratch_mu);
  if (!scratch_ptr[dev]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      return fail(FS_ERR_HIP, std::string("fs_decode_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return FS_OK;
}

}  // namespace
}  // namespace fs

using namespace fs;

extern "C" {

fs_status fs_decode_noalloc(const fs_graph *g, const void *c, const uint8_t *erased, uint32_t maxit, void *x,
                            uint8_t *recovered, int32_t *status, uint64_t t, hipStream_t stream) {
  clear_error();
  size_t need = 0;
  const fs_status sz = fs_workspace_size(g, FS_OP_DECODE, t, 0, &need);
  if (sz != FS_OK) return sz;
  if (need > kScratchBytes)
    return fail(FS_ERR_WORKSPACE, "fs_decode_noalloc: this graph's decode needs " + std::to_string(need) +
                                      " bytes of workspace, above the fixed " + std::to_string(kScratchBytes) +
                                      "; use fs_decode with a caller workspace");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(FS_ERR_HIP, "fs_decode_noalloc: hipGetDevice failed");
  if (g->device >= 0 && g->device != dev)
    return fail(FS_ERR_INVALID, "fs_decode_noalloc: the graph lives on another device than the current one");
  void *ws = nullptr;
  const fs_status st = scratch_for_current_device(&ws);
  if (st != FS_OK) return st;
  return fs_decode(g, c, erased, maxit, x, recovered, status, t, ws, kScratchBytes, stream);
}

}  // extern "C"
