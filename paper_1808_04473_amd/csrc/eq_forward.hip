// Forward kernels: fused Gram + matched filter + fusion + L-MMSE solve.
//
// PD (Section II-C, Section III-A): a wave equalises NSYS subcarriers.  The
// adder tree of eq. (fullMRC) is the MFMA accumulator itself: the row blocks
// of all clusters are accumulated into one G and one y^MRC, so the per-cluster
// statistics are summed on chip and never leave the wave.
//
// FD (Section II-D, Section IV): a wave equalises all clusters of `spw`
// subcarriers, NSYS local systems per round; after each round the local
// estimates and variances go through LDS to the lanes that hold the fusion
// sums of eq. (fusionrule) with the weights of Lemma 1 (eq. (opt_fusion)).
//
// The precision forms differ only in the Gram product (FP32 MFMA, BF16 MFMA,
// or three BF16 MFMA products of split operands) and, for the BF16 forms, one
// refinement step z += A^{-1} (H^H (y - H z) - rho z) with the FP32 residual.
// Systems whose condition estimate ||A||_1 * trace(A^{-1}) exceeds
// EQ_COND_LIMIT, or whose pivot failed, are queued for an FP64 re-solve.
#include "eq_round.h"

#ifndef EQ_WAVES_PER_EU
#define EQ_WAVES_PER_EU 4
#endif
#ifndef EQ_PD_PER32
#define EQ_PD_PER32 1
#endif

namespace dbpeq {

// Queue subcarrier w for the FP64 re-solve (one lane calls this).
__device__ __forceinline__ void enqueue_fp64(const FwdArgs &a, int w) {
  const int pos = atomicAdd(a.fb_count, 1);
  if (pos >= 0 && pos < a.W) a.fb_list[pos] = w;  // capacity W
}

// PD systems per work item.  A 32-lane group streams 32 KiB..1 MiB per
// system, so one system per item keeps the work items short enough to fill
// the device several times over (two per item left most of it idle during
// the last generation of workgroups).
template <int UT, int PREC>
constexpr int pd_per() {
  return UT == 32 ? EQ_PD_PER32 : (refines(PREC) ? 2 : 64 / UT);
}

// Occupancy target.  UT = 16: 4 waves per SIMD (128 VGPRs) for the
// one-pass forms; 3 (168 VGPRs) for the refining forms, which hold a factor
// across the residual pass, and for FD with the split-BF16 Gram, whose
// operand splits spill at 128.  UT = 32: 2 (256 VGPRs); the factor and the
// inverse columns alone take 129.
template <int UT, int PREC, bool FD>
constexpr int waves_target() {
  if (UT == 32) return 2;
  return (refines(PREC) || (FD && PREC == PREC_BF16X3_NR)) ? 3 : EQ_WAVES_PER_EU;
}

template <int UT, int PREC, class SM>
__device__ __forceinline__ void pd_task(const FwdArgs &a, int w0, int nvalid, SM &sm) {
  const int lane = lane_id();
  const int sme = lane / UT;
  const int i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    const size_t w = (size_t)w0 + s;
    Hw = a.H + w * HB;
    yw = a.y + w * a.B;
    r0 = 0;
    r1 = a.B;
  };

  // ---- Gram + matched filter of the round's subcarriers (all clusters
  //      accumulate into one G and one y^MRC: the adder tree of eq. (fullMRC))
  gram_stream<UT, PREC, refines(PREC) ? kLoadKeep : kLoadLast>(nvalid, a.U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
    store_gram<UT, PREC>(sm.A[s], acc, a.rho, a.U);
    if (lane < UT) sm.M[s][lane] = mf;
  });
  for (int s = nvalid; s < SM::NS; ++s) {
    store_identity<UT>(sm.A[s]);
    if (lane < UT) sm.M[s][lane] = make_float2(0.f, 0.f);
  }
  __syncthreads();

  // ---- factor and solve: group sme, row/column i
  const int w = w0 + sme;
  const bool live = sme < nvalid;
  LocalSolve<UT> r;
  local_solve<UT>(r, sm, slot_of<SM>(sme), i, a.U);
  if constexpr (refines(PREC)) refine_round<UT>(r, sm, nvalid, a.U, [&](int) { return a.rho; }, seg, live);

  const float kappa = r.norm1 * gsum<UT>(i < a.U ? r.d : 0.f);
  const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
  if (live) {
    if (i < a.U) {
      const float nanv = __int_as_float(0x7fc00000);
      const float s2 = a.n0 * r.d, k = unbias_factor(s2, a.ub);
      a.z[(size_t)w * a.U + i] = r.bad ? make_float2(nanv, nanv) : make_float2(r.z.x * k, r.z.y * k);
      if (a.s2) a.s2[(size_t)w * a.U + i] = r.bad ? nanv : s2 * k;
    }
    if (i == 0) {
      if (a.info) a.info[w] = (r.bad ? -1 : r.fail) | (routed ? EQ_INFO_FP64 : 0);
      if (routed) enqueue_fp64(a, w);
    }
  }
}

template <int UT, int PREC, class SM>
__device__ __forceinline__ void fd_task(const FwdArgs &a, int w0, int nsub, SM &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT;
  const int i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int C = a.C;
  // clusters of the subcarriers of this task
  const int ntot = nsub * C;
  const bool user_nu = a.nu != nullptr;
  const float nanv = __int_as_float(0x7fc00000);

  // fusion sums held by lane (wl = lane / UT, u = lane % UT)
  const int wlf = lane / UT;
  float sw = 0.f, szx = 0.f, szy = 0.f, sv = 0.f;
  if (lane < NSYS) sm.routed[lane] = 0;

  for (int base = 0; base < ntot; base += NSYS) {
    const int nvalid = min(NSYS, ntot - base);
    auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
      const int idx = base + s;
      const int wl = idx / C, c = idx - wl * C;
      const size_t w = (size_t)(w0 + wl);
      Hw = a.H + w * HB;
      yw = a.y + w * a.B;
      r0 = a.off[c];
      r1 = a.off[c + 1];
    };
    // ---- local Gram + MRC of the clusters of this round
    gram_stream<UT, PREC, refines(PREC) ? kLoadKeep : kLoadLast>(nvalid, a.U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
      store_gram<UT, PREC>(sm.A[s], acc, a.rho, a.U);
      if (lane < UT) sm.M[s][lane] = mf;
    });
    for (int s = nvalid; s < NSYS; ++s) {
      store_identity<UT>(sm.A[s]);
      if (lane < UT) sm.M[s][lane] = make_float2(0.f, 0.f);
    }
    __syncthreads();

    // ---- local L-MMSE of cluster (wl, c) by group sme
    const int idx = base + sme;
    const int wl = idx / C, c = idx - wl * C;
    const int w = w0 + wl;
    const bool live = sme < nvalid;
    LocalSolve<UT> r;
    local_solve<UT, 1>(r, sm, sme, i, a.U);
    if constexpr (refines(PREC)) refine_round<UT>(r, sm, nvalid, a.U, [&](int) { return a.rho; }, seg, live);

    const float kappa = r.norm1 * gsum<UT>(i < a.U ? r.d : 0.f);
    const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
    if (live && i == 0) {
      if (a.info) a.info[(size_t)w * C + c] = (r.bad ? -1 : r.fail) | (routed ? EQ_INFO_FP64 : 0);
      if (routed) sm.routed[wl] = 1;
    }
    // local estimate and variance (scaled to unit gain for the unbiased L-MMSE)
    const float k = unbias_factor(a.n0 * r.d, a.ub);
    const float s2c = a.n0 * r.d * k;
    __syncthreads();
    sm.F[sme][i] = live ? (r.bad ? make_float4(nanv, nanv, nanv, 1.f) : make_float4(r.z.x * k, r.z.y * k, s2c, 1.f))
                        : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();

    // ---- fusion: lane (wlf, u) adds the clusters of its subcarrier, in c order
    if (wlf < nsub && i < a.U) {
      for (int s = 0; s < nvalid; ++s) {
        const int idx3 = base + s;
        if (idx3 / C != wlf) continue;
        const float4 v = sm.F[s][i];
        if (user_nu) {
          const int c3 = idx3 - wlf * C;
          const float nu = a.nu[((size_t)(w0 + wlf) * C + c3) * a.U + i];
          szx += nu * v.x;
          szy += nu * v.y;
          sv += nu * nu * v.z;
        } else {
          const float p = 1.0f / v.z;
          sw += p;
          szx += p * v.x;
          szy += p * v.y;
        }
      }
    }
    __syncthreads();
  }

  const int w = w0 + wlf;
  if (wlf < nsub) {
    if (i < a.U) {
      float2 zo;
      float so;
      if (user_nu) {
        zo = make_float2(szx, szy);
        so = sv;
      } else {
        const float inv = 1.0f / sw;
        zo = make_float2(szx * inv, szy * inv);
        so = inv;
      }
      a.z[(size_t)w * a.U + i] = zo;
      if (a.s2) a.s2[(size_t)w * a.U + i] = so;
    }
    if (i == 0 && sm.routed[wlf]) enqueue_fp64(a, w);
  }
}

// Systems per work item: a round of subcarriers (PD) or `spw` subcarriers
// with all their clusters (FD).
template <int UT, int PREC, bool FD>
__host__ __device__ constexpr int task_size(int spw) {
  return FD ? spw : pd_per<UT, PREC>();
}

// One wave per workgroup.  Workgroup b of G takes the contiguous share
// [b W / G, (b+1) W / G) of the systems, in work items of up to task_size
// systems (with G = ceil(W / task_size), one work item each).
template <int UT, int PREC, bool FD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(waves_target<UT, PREC, FD>(), 8))) void eq_forward_kernel(const FwdArgs a) {
  // PD work items of fewer systems than lane groups need fewer matrix slots
  __shared__ Smem<UT, FD ? 64 / UT : (pd_per<UT, PREC>() < 64 / UT ? pd_per<UT, PREC>() : 64 / UT)> sm;
  const int per = task_size<UT, PREC, FD>(a.spw);
  const int lo = (int)((long long)blockIdx.x * a.W / gridDim.x);
  const int hi = (int)((long long)(blockIdx.x + 1) * a.W / gridDim.x);
  for (int w = lo; w < hi; w += per) {
    const int n = min(per, hi - w);
    if constexpr (FD)
      fd_task<UT, PREC>(a, w, n, sm);
    else
      pd_task<UT, PREC>(a, w, n, sm);
  }
}

__global__ void zero_i32_kernel(int32_t *p, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) p[t] = 0;
}

hipError_t launch_zero_i32(int32_t *p, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_i32_kernel, dim3((n + 63) / 64), dim3(64), 0, s, p, n);
  return hipGetLastError();
}

template <int UT, int PREC, bool FD>
static hipError_t launch_one(const FwdArgs &a, hipStream_t s) {
  // one work item per workgroup: the hardware dispatcher refills a freed slot
  // at once (a one-generation grid with equal shares per workgroup measured
  // slower: its partial rounds add solves)
  const int per = task_size<UT, PREC, FD>(a.spw);
  const int grid = (a.W + per - 1) / per;
  hipLaunchKernelGGL((eq_forward_kernel<UT, PREC, FD>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int UT, bool FD>
static hipError_t launch_prec(const FwdArgs &a, int prec, hipStream_t s) {
  switch (prec) {
    case PREC_FP32: return launch_one<UT, PREC_FP32, FD>(a, s);
    case PREC_BF16:  // PD only (eq_fd refuses the single-BF16 Gram)
      if constexpr (FD) return hipErrorInvalidValue;
      else return launch_one<UT, PREC_BF16, FD>(a, s);
    case PREC_BF16X3: return launch_one<UT, PREC_BF16X3, FD>(a, s);
    default: return launch_one<UT, PREC_BF16X3_NR, FD>(a, s);
  }
}

hipError_t launch_forward(const FwdArgs &a, bool fd, int prec, hipStream_t s) {
  const int UT = ut_for(a.U);
  if (UT == 16) return fd ? launch_prec<16, true>(a, prec, s) : launch_prec<16, false>(a, prec, s);
  return fd ? launch_prec<32, true>(a, prec, s) : launch_prec<32, false>(a, prec, s);
}

}  // namespace dbpeq
