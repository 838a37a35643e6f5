// Read-bandwidth probe: the practical HBM read ceiling of the device the
// equaliser runs on, measured with 16-byte nontemporal loads.  Not part of
// the equaliser; bench.py reports the equaliser's bandwidth against it.
#include <hip/hip_runtime.h>

namespace dbpeq {

namespace {

constexpr int kProbeBlock = 256;
constexpr int kProbeGrid = 8192;
constexpr int kProbeUnroll = 4;

// Grid-stride read of n16 16-byte chunks; the chunks of one unrolled step are
// one grid stride apart, so every load instruction of a wave reads 1 KiB of
// consecutive bytes.  The sum is stored only if it equals a value that finite
// data cannot give, which keeps the loads live.
__global__ __launch_bounds__(kProbeBlock) void eq_probe_read_kernel(const float4 *p, size_t n16, float *sink) {
  typedef float f4v __attribute__((ext_vector_type(4)));
  const f4v *q = reinterpret_cast<const f4v *>(p);
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  float acc = 0.f;
  size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (kProbeUnroll - 1) * stride < n16; i += kProbeUnroll * stride) {
    f4v v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(q + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc += v[u].x + v[u].y + v[u].z + v[u].w;
  }
  for (; i < n16; i += stride) {
    const f4v v = q[i];
    acc += v.x + v.y + v.z + v.w;
  }
  if (acc == -1.2345e38f) sink[0] = acc;
}

}  // namespace

hipError_t launch_probe_read(const void *buf, size_t bytes, float *sink, hipStream_t s) {
  hipLaunchKernelGGL(eq_probe_read_kernel, dim3(kProbeGrid), dim3(kProbeBlock), 0, s,
                     reinterpret_cast<const float4 *>(buf), bytes / 16, sink);
  return hipGetLastError();
}

}  // namespace dbpeq
