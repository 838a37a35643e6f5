// Read-bandwidth probe: the practical HBM read ceiling of the device the
// equaliser runs on.  Not part of the equaliser; bench.py reports the
// equaliser's bandwidth against it.
#include <hip/hip_runtime.h>

namespace dbpeq {

namespace {

constexpr int kChunk8 = 8192;              // 8-byte elements per wave: 64 KiB of consecutive bytes
constexpr int kSteps = kChunk8 / 64;       // load instructions per wave
constexpr int kDepth = 16;                 // loads in flight per wave (8 KiB)

// One wave reads one 64 KiB chunk with 8-byte nontemporal loads, 16 in
// flight; every load instruction reads 512 consecutive bytes and the wave's
// instructions follow each other through the chunk (the access pattern of
// the equaliser's streams).  Elements past n8 read as zero.  The sum is
// stored only if it equals a value that finite data cannot give, which keeps
// the loads live.
__global__ __launch_bounds__(64) void eq_probe_read_kernel(const float2 *p, size_t n8, float *sink) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v *q = reinterpret_cast<const f2v *>(p);
  const size_t base = (size_t)blockIdx.x * kChunk8 + threadIdx.x;
  auto ld = [&](int step) -> f2v {
    const size_t i = base + (size_t)step * 64;
    return i < n8 ? __builtin_nontemporal_load(q + i) : f2v{0.f, 0.f};
  };
  f2v buf[kDepth];
#pragma unroll
  for (int d = 0; d < kDepth; ++d) buf[d] = ld(d);
  float acc = 0.f;
  for (int s = 0; s < kSteps; s += kDepth) {
#pragma unroll
    for (int d = 0; d < kDepth; ++d) {
      acc += buf[d].x + buf[d].y;
      if (s + d + kDepth < kSteps) buf[d] = ld(s + d + kDepth);
    }
  }
  if (acc == -1.2345e38f) sink[0] = acc;
}

}  // namespace

hipError_t launch_probe_read(const void *buf, size_t bytes, float *sink, hipStream_t s) {
  const size_t n8 = bytes / 8;
  const size_t grid = (n8 + kChunk8 - 1) / kChunk8;
  hipLaunchKernelGGL(eq_probe_read_kernel, dim3((unsigned)grid), dim3(64), 0, s,
                     reinterpret_cast<const float2 *>(buf), n8, sink);
  return hipGetLastError();
}

}  // namespace dbpeq
