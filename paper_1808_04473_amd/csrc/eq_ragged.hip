// Persistent kernel for ragged batches.  Each wave takes work items from its
// queue's atomic head (eight queues, the items dealt round-robin) until that
// queue is empty; every wave reaches the exit.  Items are cost-sorted on the
// host (largest first), so the tail of the launch is made of the cheapest
// ones.  The per-item work is the fused Gram +
// solve (+ fusion) of the uniform kernels, with every system's shape, N0 and
// cluster offsets read from the descriptor table.  Three kinds of item:
//
//  * PD group: a round of up to 64/UT whole systems of equal U, streamed one
//    after the other and solved together;
//  * PD piece: a row range of a large system.  Its partial Gram and matched
//    filter (the raw MFMA accumulators) go to a partial slot; the wave that
//    finishes the system's last piece sums the slots in piece order, then
//    factors and solves it.  A large system therefore streams at the speed of
//    several waves, on any CUs, with no wave waiting for another;
//  * FD round: up to 64/UT clusters of equal U (of one system or several),
//    each solved locally; every cluster's fusion terms go to its slot and the
//    lane group that finishes a system's last cluster sums its C slots in
//    cluster order and writes the fused estimate.
//
// The hand-over uses the device-scope arrival counter of each system.  The
// slots are written and read with device-scope accesses (stores written
// through to the device coherence point, loads that do not hit a stale L2
// line of another XCD); a writer waits until its slot stores are complete
// before its increment.  An agent-scope release fence would do the same by
// writing back the whole L2 of the XCD, on every item.  Sums run in a fixed
// order, so results do not depend on which wave finishes.
#include "eq_ragged.h"
#include "eq_round.h"

namespace dbpeq {

template <int UT>
constexpr int acc_regs() {
  return UT == 16 ? 4 : 16;
}

// Device-scope store / load of one slot word.
template <class T>
__device__ __forceinline__ void st_dev(T *p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T>
__device__ __forceinline__ T ld_dev(const T *p) {
  return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Waits until this wave's stores are complete (written through), before the
// arrival increment that publishes them.
__device__ __forceinline__ void stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Solve and outputs of a PD round whose n systems (sysk(s), s < n) have their
// G + rho I and matched filters in sm.A / sm.M; seg re-streams them for the
// refinement step.
template <int UT, int PREC, class SysK, class Seg>
__device__ __forceinline__ void pd_solve_round(const RaggedArgs &a, Smem<UT> &sm, int n, int U, SysK sysk,
                                               Seg seg) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
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
__device__ __forceinline__ void pd_group(const RaggedArgs &a, const RTask &task, Smem<UT> &sm) {
  const int lane = lane_id();
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
  pd_solve_round<UT, PREC>(a, sm, n, U, sysk, seg);
}

template <int UT, int PREC>
__device__ __forceinline__ void pd_piece(const RaggedArgs &a, const RTask &task, Smem<UT> &sm) {
  constexpr int R = acc_regs<UT>();
  constexpr bool II = PREC != PREC_FP32;  // the FP32 Gram keeps two accumulator arrays
  const int lane = lane_id();
  const int k = task.first;
  const int U = task.U;
  const RSys &d = a.sys[k];
  const int np = d.npieces;
  float *slot = a.part + (size_t)(d.slot0 + task.piece) * kPartStride;
  auto seg_piece = [&](int, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    Hw = a.Hpool + d.h_off;
    yw = a.ypool + d.y_off;
    r0 = task.r0;
    r1 = task.r1;
  };
  gram_stream<UT, PREC, kLoadLast>(1, U, seg_piece, [&](int, const Acc<UT> &acc, float2 mf) {
#pragma unroll
    for (int r = 0; r < R; ++r) {
      st_dev(slot + r * 64 + lane, (float)acc.rr[r]);
      st_dev(slot + (R + r) * 64 + lane, (float)acc.ri[r]);
      if constexpr (II) st_dev(slot + (2 * R + r) * 64 + lane, (float)acc.ii[r]);
    }
    st_dev(slot + 3 * R * 64 + lane, mf.x);
    st_dev(slot + (3 * R + 1) * 64 + lane, mf.y);
  });
  stores_done();
  int old = 0;
  if (lane == 0) old = atomicAdd(a.arrive + k, 1);
  old = __shfl(old, 0);
  if (old != np - 1) return;
  // every piece has arrived: the counter starts the next execution at zero
  if (lane == 0) a.arrive[k] = 0;
  // the last piece: sum every piece's slot in piece order, then solve alone
  Acc<UT> acc;
  acc_zero<UT>(acc);
  float2 mf = make_float2(0.f, 0.f);
  for (int p = 0; p < np; ++p) {
    const float *q = a.part + (size_t)(d.slot0 + p) * kPartStride;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      acc.rr[r] += ld_dev(q + r * 64 + lane);
      acc.ri[r] += ld_dev(q + (R + r) * 64 + lane);
      if constexpr (II) acc.ii[r] += ld_dev(q + (2 * R + r) * 64 + lane);
    }
    mf.x += ld_dev(q + 3 * R * 64 + lane);
    mf.y += ld_dev(q + (3 * R + 1) * 64 + lane);
  }
  store_gram<UT, PREC>(sm.A[0], acc, d.rho);
  if (lane < UT) sm.M[0][lane] = mf;
  auto seg_whole = [&](int, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    Hw = a.Hpool + d.h_off;
    yw = a.ypool + d.y_off;
    r0 = 0;
    r1 = d.B;
  };
  pd_solve_round<UT, PREC>(a, sm, 1, U, [&](int) { return k; }, seg_whole);
}

template <int UT, int PREC>
__device__ __forceinline__ void fd_round(const RaggedArgs &a, const RTask &task, Smem<UT> &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
  const int n = task.count;
  const int U = task.U;
  const float nanv = __int_as_float(0x7fc00000);
  auto gcl = [&](int s) { return a.order[task.first + s]; };
  auto sysk = [&](int s) { return a.cl_sys[gcl(s)]; };
  auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    const int gc = gcl(s);
    const RSys &d = a.sys[a.cl_sys[gc]];
    const int c = gc - d.cl0;
    Hw = a.Hpool + d.h_off;
    yw = a.ypool + d.y_off;
    r0 = a.offs[d.off_first + c];
    r1 = a.offs[d.off_first + c + 1];
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
  local_solve<UT, 3>(r, sm, sme, i, U);
  if constexpr (refines(PREC))
    refine_round<UT>(r, sm, n, U, [&](int s) { return a.sys[sysk(s)].rho; }, seg, live);
  const float kappa = r.norm1 * gsum<UT>(i < U ? r.d : 0.f);
  const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
  // this group's cluster: its fusion terms and failure code to its slot
  const int gc = live ? gcl(sme) : 0;
  const int k = live ? a.cl_sys[gc] : 0;
  if (live) {
    const float n0 = a.sys[k].n0;
    if (i < U) {
      float3 f = make_float3(nanv, nanv, nanv);
      if (!r.bad) {
        const float p = 1.0f / (n0 * r.d);
        f = make_float3(p, p * r.z.x, p * r.z.y);
      }
      float *q = a.fpart + ((size_t)gc * kFusionStride + i) * 4;
      st_dev(q, f.x);
      st_dev(q + 1, f.y);
      st_dev(q + 2, f.z);
    }
    if (i == 0) {
      st_dev(a.fcode + 2 * gc, r.bad ? -1 : r.fail);
      st_dev(a.fcode + 2 * gc + 1, routed ? 1 : 0);
    }
  }
  stores_done();
  int old = -1;
  if (live && i == 0) old = atomicAdd(a.arrive + k, 1);
  old = __shfl(old, sme * UT);
  const bool fin = live && old == a.sys[k].C - 1;
  if (__ballot(fin) == 0ull) return;
  // every cluster has arrived: the counter starts the next execution at zero
  if (fin && i == 0) a.arrive[k] = 0;
  // groups that finished their system's last cluster fuse its C clusters in
  // cluster order
  if (fin) {
    const RSys &d = a.sys[k];
    float sw = 0.f, szx = 0.f, szy = 0.f;
    int first_code = 0;
    bool any_routed = false, any_bad = false;
    for (int c = 0; c < d.C; ++c) {
      if (i < U) {
        const float *q = a.fpart + ((size_t)(d.cl0 + c) * kFusionStride + i) * 4;
        sw += ld_dev(q);
        szx += ld_dev(q + 1);
        szy += ld_dev(q + 2);
      }
      const int code = ld_dev(a.fcode + 2 * (d.cl0 + c));
      const int rt = ld_dev(a.fcode + 2 * (d.cl0 + c) + 1);
      if (code != 0 && first_code == 0) first_code = code;
      any_routed |= rt != 0;
      any_bad |= code == -1;
    }
    if (i < U) {
      const float inv = 1.0f / sw;
      a.zpool[d.z_off + i] = make_float2(szx * inv, szy * inv);
      if (a.s2pool) a.s2pool[d.z_off + i] = inv;
    }
    if (i == 0) {
      const bool routed_sys = any_routed && !any_bad;
      if (a.info) a.info[k] = first_code | (routed_sys ? EQ_INFO_FP64 : 0);
      if (routed_sys) {
        const int pos = atomicAdd(a.fb_count, 1);
        if (pos >= 0 && pos < a.nsys) a.fb_list[pos] = k;
      }
    }
  }
}

template <int PREC, bool FD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(refines(PREC) ? 1 : 2, 8))) void eq_ragged_kernel(
    const RaggedArgs a) {
  __shared__ union {
    Smem<16> s16;
    Smem<32> s32;
  } sm;
  const int lane = lane_id();
  const int q = (int)(blockIdx.x % kQueues);
  int32_t *head = a.counter + q * kQueueStride;
  while (true) {
    int t = 0;
    if (lane == 0) t = atomicAdd(head, 1);
    t = q + kQueues * __shfl(t, 0);
    if (t >= a.ntasks) break;
    const RTask task = a.tasks[t];
    if constexpr (FD) {
      if (task.ut == 16)
        fd_round<16, PREC>(a, task, sm.s16);
      else
        fd_round<32, PREC>(a, task, sm.s32);
    } else if (task.kind == kItemPiece) {
      if (task.ut == 16)
        pd_piece<16, PREC>(a, task, sm.s16);
      else
        pd_piece<32, PREC>(a, task, sm.s32);
    } else {
      if (task.ut == 16)
        pd_group<16, PREC>(a, task, sm.s16);
      else
        pd_group<32, PREC>(a, task, sm.s32);
    }
    __syncthreads();
  }
}

hipError_t launch_ragged(const RaggedArgs &a, bool fd, int prec, int grid, hipStream_t s) {
  const dim3 g(grid), b(64);
#define EQ_RAGGED_LAUNCH(P)                                                \
  if (fd) hipLaunchKernelGGL((eq_ragged_kernel<P, true>), g, b, 0, s, a); \
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
