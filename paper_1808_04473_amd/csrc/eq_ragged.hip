// Persistent kernel for ragged batches.  Each wave takes work items from an
// atomic queue head until the queue is empty (every wave reaches the exit).
// Items are cost-sorted on the host (largest first), so the tail of the
// launch is made of the cheapest systems.  The per-item work is the same
// fused Gram + solve + fusion as the uniform kernels, with every system's
// shape, N0 and cluster offsets read from the descriptor table.
#include "eq_ragged.h"
#include "eq_round.h"

namespace dbpeq {

template <int UT, int PREC>
__device__ __forceinline__ void ragged_pd(const RaggedArgs &a, const RTask &task, Smem<UT> &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
  const int n = task.count;
  const int U = task.U;
  auto sysk = [&](int s) { return a.order[task.first + s]; };
  auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    const RSys &d = a.sys[sysk(s)];
    Hw = a.Hpool + d.h_off;
    yw = a.ypool + d.y_off;
    r0 = 0;
    r1 = d.B;
  };
  gram_stream<UT, PREC, refines(PREC) ? kLoadKeep : kLoadLast>(n, U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
    store_gram<UT, PREC>(sm.A[s], acc, a.sys[sysk(s)].rho);
    if (lane < UT) sm.M[s][lane] = mf;
  });
  for (int s = n; s < NSYS; ++s) {
    store_identity<UT>(sm.A[s]);
    if (lane < UT) sm.M[s][lane] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const bool live = sme < n;
  LocalSolve<UT> r;
  local_solve<UT>(r, sm, sme, i, U);
  if constexpr (refines(PREC))
    refine_round<UT>(r, sm, n, U, [&](int s) { return a.sys[sysk(s)].rho; }, seg, live);
  const float kappa = r.norm1 * gsum<UT>(i < U ? r.d : 0.f);
  const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
  if (live) {
    const int k = sysk(sme);
    const RSys &d = a.sys[k];
    const float nanv = __int_as_float(0x7fc00000);
    if (i < U) {
      a.zpool[d.z_off + i] = r.bad ? make_float2(nanv, nanv) : r.z;
      if (a.s2pool) a.s2pool[d.z_off + i] = r.bad ? nanv : d.n0 * r.d;
    }
    if (i == 0) {
      if (a.info) a.info[k] = (r.bad ? -1 : r.fail) | (routed ? EQ_INFO_FP64 : 0);
      if (routed) {
        const int pos = atomicAdd(a.fb_count, 1);
        if (pos >= 0 && pos < a.nsys) a.fb_list[pos] = k;
      }
    }
  }
}

template <int UT, int PREC>
__device__ __forceinline__ void ragged_fd(const RaggedArgs &a, const RTask &task, Smem<UT> &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
  const int k = a.order[task.first];
  const RSys d = a.sys[k];
  const int U = d.U, C = d.C;
  const float nanv = __int_as_float(0x7fc00000);
  float sw = 0.f, szx = 0.f, szy = 0.f;
  int worst = 0;  // group-uniform first failure code of this lane's clusters
  bool routed_any = false, bad_any = false;
  for (int base = 0; base < C; base += NSYS) {
    const int n = min(NSYS, C - base);
    auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
      Hw = a.Hpool + d.h_off;
      yw = a.ypool + d.y_off;
      r0 = a.offs[d.off_first + base + s];
      r1 = a.offs[d.off_first + base + s + 1];
    };
    gram_stream<UT, PREC, refines(PREC) ? kLoadKeep : kLoadLast>(n, U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
      store_gram<UT, PREC>(sm.A[s], acc, d.rho);
      if (lane < UT) sm.M[s][lane] = mf;
    });
    for (int s = n; s < NSYS; ++s) {
      store_identity<UT>(sm.A[s]);
      if (lane < UT) sm.M[s][lane] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    const bool live = sme < n;
    LocalSolve<UT> r;
    local_solve<UT>(r, sm, sme, i, U);
    if constexpr (refines(PREC))
      refine_round<UT>(r, sm, n, U, [&](int) { return d.rho; }, seg, live);
    const float kappa = r.norm1 * gsum<UT>(i < U ? r.d : 0.f);
    const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
    if (live) {
      routed_any |= routed;
      bad_any |= r.bad;
      if (!worst) worst = r.bad ? -1 : r.fail;
    }
    __syncthreads();
    sm.F[sme][i] = live ? (r.bad ? make_float4(nanv, nanv, nanv, 1.f)
                                 : make_float4(r.z.x, r.z.y, d.n0 * r.d, 1.f))
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    if (lane < UT && i < U) {
      for (int s = 0; s < n; ++s) {
        const float4 v = sm.F[s][i];
        const float p = 1.0f / v.z;
        sw += p;
        szx += p * v.x;
        szy += p * v.y;
      }
    }
    __syncthreads();
  }
  // combine the per-group flags of the system
  const unsigned long long rm = __ballot(routed_any);
  const unsigned long long bm = __ballot(bad_any);
  if (lane < U) {
    const float inv = 1.0f / sw;
    a.zpool[d.z_off + lane] = make_float2(szx * inv, szy * inv);
    if (a.s2pool) a.s2pool[d.z_off + lane] = inv;
  }
  // first failure code over the groups, in group order
  int code = 0;
  for (int g = 0; g < NSYS; ++g) {
    const int cg = __shfl(worst, g * UT);
    if (!code) code = cg;
  }
  if (lane == 0) {
    const bool routed = rm != 0ull && bm == 0ull;
    if (a.info) a.info[k] = code | (routed ? EQ_INFO_FP64 : 0);
    if (routed) {
      const int pos = atomicAdd(a.fb_count, 1);
      if (pos >= 0 && pos < a.nsys) a.fb_list[pos] = k;
    }
  }
}

// Holds both the UT = 16 and the UT = 32 paths: 2 waves per SIMD (256 VGPRs)
// for the one-pass forms; the refining forms need more than 256.
template <int PREC, bool FD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(refines(PREC) ? 1 : 2, 8))) void eq_ragged_kernel(const RaggedArgs a) {
  __shared__ union {
    Smem<16> s16;
    Smem<32> s32;
  } sm;
  const int lane = lane_id();
  while (true) {
    int t = 0;
    if (lane == 0) t = atomicAdd(a.counter, 1);
    t = __shfl(t, 0);
    if (t >= a.ntasks) break;
    const RTask task = a.tasks[t];
    if (task.ut == 16) {
      if constexpr (FD) ragged_fd<16, PREC>(a, task, sm.s16);
      else ragged_pd<16, PREC>(a, task, sm.s16);
    } else {
      if constexpr (FD) ragged_fd<32, PREC>(a, task, sm.s32);
      else ragged_pd<32, PREC>(a, task, sm.s32);
    }
    __syncthreads();
  }
}

hipError_t launch_ragged(const RaggedArgs &a, bool fd, int prec, int grid, hipStream_t s) {
  const dim3 g(grid), b(64);
#define EQ_RAGGED_LAUNCH(P)                                                        \
  if (fd) hipLaunchKernelGGL((eq_ragged_kernel<P, true>), g, b, 0, s, a);         \
  else hipLaunchKernelGGL((eq_ragged_kernel<P, false>), g, b, 0, s, a);
  switch (prec) {
    case PREC_FP32: EQ_RAGGED_LAUNCH(PREC_FP32) break;
    case PREC_BF16:  // PD only (the plan refuses FD with the single-BF16 Gram)
      if (fd) return hipErrorInvalidValue;
      hipLaunchKernelGGL((eq_ragged_kernel<PREC_BF16, false>), g, b, 0, s, a);
      break;
    case PREC_BF16X3: EQ_RAGGED_LAUNCH(PREC_BF16X3) break;
    default: EQ_RAGGED_LAUNCH(PREC_BF16X3_NR) break;
  }
#undef EQ_RAGGED_LAUNCH
  return hipGetLastError();
}

}  // namespace dbpeq
