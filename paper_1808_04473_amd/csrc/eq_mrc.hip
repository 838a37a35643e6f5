// MRC equalisation (Section III-A; Section IV-A for FD): the same fused
// Gram + matched-filter pass as the L-MMSE kernels, then, per user u,
//   z_u = y^MRC_u / G_uu,
//   sigma2_u = N0 / G_uu + E_s sum_{k != u} |G_uk|^2 / G_uu^2,
// which is the diagonal of D^{-1} G D^{-H} N0 + (D^{-1} G - I)(D^{-1} G - I)^H E_s
// with D = diag(G) (the diagonal of D^{-1} G is one).  No factorisation, so
// no condition check and no FP64 re-solve.  FD applies it to every
// cluster's statistics and fuses as the L-MMSE kernel does.
#include "eq_round.h"

namespace dbpeq {

struct MrcOut {
  float2 z;
  float s2;
  int fail;  // 0, or u + 1 for the first user of the group with G_uu <= 0
  bool bad;  // non-finite statistics
};

// Lane i of group `slot` (row i of the slot's G, y^MRC_i).
template <int UT, class SM>
__device__ __forceinline__ MrcOut mrc_local(SM &sm, int slot, int i, int U, float n0, float es) {
  float2 gii = make_float2(0.f, 0.f);
  float off = 0.f;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < UT; ++k) {
    const float2 g = lds_el<UT>(sm.A[slot], i, k);
    bad |= !finite2(g);
    if (k == i) gii = g;
    else off = fmaf(g.x, g.x, fmaf(g.y, g.y, off));
  }
  const float2 m = sm.M[slot][i];
  bad |= !finite2(m);
  MrcOut o;
  o.bad = gany<UT>(bad);
  const bool pos = gii.x > 0.f;
  // first user of the group with a non-positive diagonal entry
  const unsigned long long nm = __ballot(i < U && !pos);
  const int base = (lane_id() / UT) * UT;
  const unsigned long long gm = (UT == 64 ? ~0ull : ((1ull << UT) - 1ull)) << base;
  const unsigned long long fm = nm & gm;
  o.fail = fm ? __builtin_ctzll(fm) - base + 1 : 0;
  const float inv = 1.0f / gii.x;
  o.z = make_float2(m.x * inv, m.y * inv);
  o.s2 = n0 * inv + es * off * inv * inv;
  return o;
}

template <int UT, int PREC>
__device__ __forceinline__ void mrc_pd_task(const FwdArgs &a, int w0, int nvalid, Smem<UT> &sm) {
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    const size_t w = (size_t)w0 + s;
    Hw = a.H + w * HB;
    yw = a.y + w * a.B;
    r0 = 0;
    r1 = a.B;
  };
  gram_stream<UT, PREC, kLoadLast>(nvalid, a.U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
    store_gram<UT, PREC>(sm.A[s], acc, 0.f);
    if (lane < UT) sm.M[s][lane] = mf;
  });
  __syncthreads();
  const MrcOut o = mrc_local<UT>(sm, g, i, a.U, a.n0, a.es);
  if (g >= nvalid) return;
  const int w = w0 + g;
  const float nanv = __int_as_float(0x7fc00000);
  const bool out_nan = o.bad || o.fail;
  if (i < a.U) {
    a.z[(size_t)w * a.U + i] = out_nan ? make_float2(nanv, nanv) : o.z;
    if (a.s2) a.s2[(size_t)w * a.U + i] = out_nan ? nanv : o.s2;
  }
  if (i == 0 && a.info) a.info[w] = o.bad ? -1 : o.fail;
}

template <int UT, int PREC>
__device__ __forceinline__ void mrc_fd_task(const FwdArgs &a, int w, Smem<UT> &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int C = a.C;
  const bool user_nu = a.nu != nullptr;
  const float nanv = __int_as_float(0x7fc00000);
  float sw = 0.f, szx = 0.f, szy = 0.f, sv = 0.f;
  for (int base = 0; base < C; base += NSYS) {
    const int nvalid = min(NSYS, C - base);
    auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
      Hw = a.H + (size_t)w * HB;
      yw = a.y + (size_t)w * a.B;
      r0 = a.off[base + s];
      r1 = a.off[base + s + 1];
    };
    gram_stream<UT, PREC, kLoadLast>(nvalid, a.U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
      store_gram<UT, PREC>(sm.A[s], acc, 0.f);
      if (lane < UT) sm.M[s][lane] = mf;
    });
    __syncthreads();
    const int c = base + g;
    const bool live = g < nvalid;
    const MrcOut o = mrc_local<UT>(sm, g, i, a.U, a.n0, a.es);
    if (live && i == 0 && a.info) a.info[(size_t)w * C + c] = o.bad ? -1 : o.fail;
    const bool out_nan = o.bad || o.fail;
    sm.F[g][i] = live ? (out_nan ? make_float4(nanv, nanv, nanv, 1.f) : make_float4(o.z.x, o.z.y, o.s2, 1.f))
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // lanes of group 0 fuse user i over the round's clusters, in cluster order
    if (g == 0 && i < a.U) {
      for (int s = 0; s < nvalid; ++s) {
        const float4 v = sm.F[s][i];
        if (user_nu) {
          const float nu = a.nu[((size_t)w * C + base + s) * a.U + i];
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
  if (g == 0 && i < a.U) {
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
}

// One wave per workgroup: NSYS subcarriers per work item (PD) or one
// subcarrier with all its clusters (FD).  MRC holds no factor, so the
// one-pass register target of the L-MMSE kernels applies.
template <int UT, int PREC, bool FD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(UT == 16 ? 4 : 2, 8))) void eq_mrc_kernel(const FwdArgs a) {
  __shared__ Smem<UT> sm;
  if constexpr (FD) {
    mrc_fd_task<UT, PREC>(a, blockIdx.x, sm);
  } else {
    const int w0 = blockIdx.x * (64 / UT);
    mrc_pd_task<UT, PREC>(a, w0, min(64 / UT, a.W - w0), sm);
  }
}

template <int UT, int PREC, bool FD>
static hipError_t launch_mrc_one(const FwdArgs &a, hipStream_t s) {
  const int per = FD ? 1 : 64 / UT;
  const int grid = (a.W + per - 1) / per;
  hipLaunchKernelGGL((eq_mrc_kernel<UT, PREC, FD>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int UT, bool FD>
static hipError_t launch_mrc_prec(const FwdArgs &a, int prec, hipStream_t s) {
  return prec == PREC_FP32 ? launch_mrc_one<UT, PREC_FP32, FD>(a, s) : launch_mrc_one<UT, PREC_BF16X3_NR, FD>(a, s);
}

hipError_t launch_mrc(const FwdArgs &a, bool fd, int prec, hipStream_t s) {
  if (prec != PREC_FP32 && prec != PREC_BF16X3_NR) return hipErrorInvalidValue;
  const int UT = ut_for(a.U);
  if (UT == 16) return fd ? launch_mrc_prec<16, true>(a, prec, s) : launch_mrc_prec<16, false>(a, prec, s);
  return fd ? launch_mrc_prec<32, true>(a, prec, s) : launch_mrc_prec<32, false>(a, prec, s);
}

}  // namespace dbpeq
