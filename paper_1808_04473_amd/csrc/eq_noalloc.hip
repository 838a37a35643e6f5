// eq_pd_noalloc: the partially decentralised L-MMSE call (Section II-C,
// Section III-A) for callers that cannot allocate device memory.  Its only
// scratch buffer, the queue of systems routed to the FP64 re-solve (two
// counters in a 256-byte header, then one int32 per system), lives in a
// file-scope device array instead of a caller workspace.
#include <mutex>

#include "eq_common.h"

static_assert(EQ_NOALLOC_SCRATCH_BYTES % 256 == 0, "whole 256-byte blocks");

// One copy per GPU, at its own device address; kernels get that address
// (scratch_ptr), never this name, which in host code is a host-side stand-in.
static __device__ __align__(256) unsigned char scratch[EQ_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
hipError_t scratch_ptr(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[dev] = p;
  }
  *out = g_scratch[dev];
  return hipSuccess;
}

}  // namespace

extern "C" eq_status eq_pd_noalloc(const eq_problem *p, const eq_c32 *H, const eq_c32 *y, eq_c32 *z,
                                   float *sigma2, int32_t *info, void *stream) {
  const eq_status st = dbpeq::forward_validate(p, false, H, y, nullptr, z, sigma2, info);
  if (st != EQ_OK || p->W == 0) return st;
  if (p->W > EQ_NOALLOC_MAX_W || dbpeq::forward_ws_bytes(p) > (size_t)EQ_NOALLOC_SCRATCH_BYTES)
    return EQ_ENOTSUP;
  void *ws = nullptr;
  if (scratch_ptr(&ws) != hipSuccess) return EQ_EHIP;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  // the array keeps whatever the last call on this GPU left: clear the queue
  // counters (a fill kernel, so that the call can be captured into a graph)
  if (dbpeq::launch_zero_i32(reinterpret_cast<int32_t *>(ws), 64, s) != hipSuccess) return EQ_EHIP;
  return dbpeq::forward_launch(p, false, H, y, nullptr, z, sigma2, info, ws, s);
}
