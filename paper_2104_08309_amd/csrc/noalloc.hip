// pft_forward_3d_noalloc: the 3D forward with no device allocation in the call.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation). The call's
// temporaries -- the mesh centre, the per-face records and the per-split
// partial sums -- live in `scratch`, a file-scope device array of fixed size:
// each GPU the library runs on holds its own copy until the process ends, at
// the address hipGetSymbolAddress reports with that GPU current. That address
// is looked up once per device (at the device's first call) and kept; host code
// passes only that address on, never the array's name (which, in host code, is
// a host-side stand-in and not a device address). Every call on one GPU shares
// that GPU's array, so calls that overlap on one GPU (other streams, other host
// threads) race; calls in one stream are ordered. Nothing needs to start at
// zero: each call writes every byte it reads before reading it.
#include <map>
#include <mutex>

#include "pft_internal.h"

namespace pft {
namespace {

constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;  // 64 MiB per GPU

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;  // device ordinal -> address of that device's `scratch`

}  // namespace
}  // namespace pft

static __device__ __align__(256) unsigned char scratch[pft::kNoAllocScratchBytes];

namespace pft {
namespace {

// Address of the current device's copy of `scratch` (looked up at its first use on that device).
pft_status scratch_for_current_device(void** p) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(PFT_EHIP, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_addr.find(dev);
  if (it != g_scratch_addr.end()) {
    *p = it->second;
    return PFT_OK;
  }
  void* addr = nullptr;
  e = hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || addr == nullptr) return set_error(PFT_EHIP, "hipGetSymbolAddress(scratch) failed");
  g_scratch_addr[dev] = addr;
  *p = addr;
  return PFT_OK;
}

}  // namespace
}  // namespace pft

extern "C" pft_status pft_forward_3d_noalloc(const void* verts, pft_dtype vdtype, int64_t nv, const int32_t* tris,
                                             int64_t nf, const void* q, pft_dtype qdtype, int64_t nq, pft_mode mode,
                                             void* out, void* intensity, void* stream) {
  return pft::forward3d_noalloc(pft::scratch_for_current_device, pft::kNoAllocScratchBytes, verts, vdtype, nv, tris,
                                nf, q, qdtype, nq, mode, out, intensity, stream);
}
