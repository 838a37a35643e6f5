// LAMA-PD and LAMA-FD (Algorithm 1; Section IV with the normalisation of the
// proof of Lemma 2).  The same fused Gram + matched-filter pass as the
// L-MMSE kernels (G stored unshifted), then every lane group iterates on
// its system's statistics held in registers:
//     z = y^MRC + (I - G) s + v,   tau = N0 + beta phi
//     s' = F(z, tau),   phi' = <G(z, tau)>,   v' = beta phi' / tau (z - s)
// Lane i keeps row i of G (conjugated, so that the DPP-broadcast product
// that forms X^H t in the L-MMSE solve gives (G s)_i here), and s_i, v_i.
// The posterior mean and variance of a square-QAM point factor into those of
// two PAM coordinates (the prior is a product of uniform PAMs and the CN(0,
// tau) likelihood a product of N(0, tau/2) ones).
//
// FD runs the iteration in every cluster on G_c / w_c, y_c^MRC / w_c with
// noise N0 / w_c and system ratio beta / w_c (w_c = B_c / B), then fuses the
// local estimates with Lemma 1's weights built from N0/w_c + (beta/w_c) phi_c.
#include "eq_lama.h"

namespace dbpeq {

struct LamaOut {
  float2 z;
  float s2;
  bool bad;
};

// Algorithm 1 for the system in `slot` (lane i: row i of G, y^MRC_i), with
// the statistics scaled by `scale`, noise n0 and system ratio beta.
template <int UT, int M, class SM>
__device__ __forceinline__ LamaOut lama_local(SM &sm, int slot, int i, int U, float scale, float n0, float beta,
                                              float es, int t_max) {
  Factor<UT> f;  // f.x[k] = conj(G_ik) * scale
  bool bad = false;
#pragma unroll
  for (int k = 0; k < UT; ++k) {
    const float2 g = lds_el<UT>(sm.A[slot], i, k);
    bad |= !finite2(g);
    f.x[k] = make_float2(g.x * scale, -g.y * scale);
  }
  float2 m = sm.M[slot][i];
  bad |= !finite2(m);
  m = make_float2(m.x * scale, m.y * scale);
  LamaOut o;
  o.bad = gany<UT>(bad);
  lama_iterate<UT, M>(f, m, i, U, n0, beta, es, t_max, o.z, o.s2);
  return o;
}

template <int UT, int PREC, int M>
__device__ __forceinline__ void lama_pd_task(const FwdArgs &a, int w0, int nvalid, Smem<UT> &sm) {
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
  for (int s = nvalid; s < 64 / UT; ++s) {
    store_identity<UT>(sm.A[s]);
    if (lane < UT) sm.M[s][lane] = make_float2(0.f, 0.f);
  }
  __syncthreads();
  const float beta = (float)a.U / (float)a.B;
  const LamaOut o = lama_local<UT, M>(sm, g, i, a.U, 1.0f, a.n0, beta, a.es, a.lama_t);
  if (g >= nvalid) return;
  const int w = w0 + g;
  const float nanv = __int_as_float(0x7fc00000);
  if (i < a.U) {
    a.z[(size_t)w * a.U + i] = o.bad ? make_float2(nanv, nanv) : o.z;
    if (a.s2) a.s2[(size_t)w * a.U + i] = o.bad ? nanv : o.s2;
  }
  if (i == 0 && a.info) a.info[w] = o.bad ? -1 : 0;
}

template <int UT, int PREC, int M>
__device__ __forceinline__ void lama_fd_task(const FwdArgs &a, int w, Smem<UT> &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int C = a.C;
  const bool user_nu = a.nu != nullptr;
  const float nanv = __int_as_float(0x7fc00000);
  const float beta = (float)a.U / (float)a.B;
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
    for (int s = nvalid; s < NSYS; ++s) {
      store_identity<UT>(sm.A[s]);
      if (lane < UT) sm.M[s][lane] = make_float2(0.f, 0.f);
    }
    __syncthreads();
    const int c = base + g;
    const bool live = g < nvalid;
    // w_c of this lane group's cluster (1 for groups past the round)
    const float wc = live ? (float)(a.off[c + 1] - a.off[c]) / (float)a.B : 1.0f;
    const float iw = 1.0f / wc;
    const LamaOut o = lama_local<UT, M>(sm, g, i, a.U, iw, a.n0 * iw, beta * iw, a.es, a.lama_t);
    if (live && i == 0 && a.info) a.info[(size_t)w * C + c] = o.bad ? -1 : 0;
    sm.F[g][i] = live ? (o.bad ? make_float4(nanv, nanv, nanv, 1.f) : make_float4(o.z.x, o.z.y, o.s2, 1.f))
                      : make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
    // lanes of group 0 fuse user i over the round's clusters, in cluster order
    if (g == 0 && i < a.U) {
      for (int s = 0; s < nvalid; ++s) {
        const float4 vv = sm.F[s][i];
        if (user_nu) {
          const float nu = a.nu[((size_t)w * C + base + s) * a.U + i];
          szx += nu * vv.x;
          szy += nu * vv.y;
          sv += nu * nu * vv.z;
        } else {
          const float p = 1.0f / vv.z;
          sw += p;
          szx += p * vv.x;
          szy += p * vv.y;
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
// subcarrier with all its clusters (FD).  3 waves per SIMD at UT = 16: the
// row of G, the iterates and the denoiser's level terms spill at 4.
template <int UT, int PREC, bool FD, int M>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(UT == 16 ? 3 : 2, 8))) void eq_lama_kernel(const FwdArgs a) {
  __shared__ Smem<UT> sm;
  if constexpr (FD) {
    lama_fd_task<UT, PREC, M>(a, blockIdx.x, sm);
  } else {
    const int w0 = blockIdx.x * (64 / UT);
    lama_pd_task<UT, PREC, M>(a, w0, min(64 / UT, a.W - w0), sm);
  }
}

template <int UT, int PREC, bool FD, int M>
static hipError_t launch_lama_one(const FwdArgs &a, hipStream_t s) {
  const int per = FD ? 1 : 64 / UT;
  const int grid = (a.W + per - 1) / per;
  hipLaunchKernelGGL((eq_lama_kernel<UT, PREC, FD, M>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int UT, int PREC, bool FD>
static hipError_t launch_lama_m(const FwdArgs &a, hipStream_t s) {
  switch (a.lama_m) {
    case 2: return launch_lama_one<UT, PREC, FD, 2>(a, s);
    case 4: return launch_lama_one<UT, PREC, FD, 4>(a, s);
    case 8: return launch_lama_one<UT, PREC, FD, 8>(a, s);
    default: return hipErrorInvalidValue;
  }
}

template <int UT, bool FD>
static hipError_t launch_lama_prec(const FwdArgs &a, int prec, hipStream_t s) {
  return prec == PREC_FP32 ? launch_lama_m<UT, PREC_FP32, FD>(a, s) : launch_lama_m<UT, PREC_BF16X3_NR, FD>(a, s);
}

hipError_t launch_lama(const FwdArgs &a, bool fd, int prec, hipStream_t s) {
  if (prec != PREC_FP32 && prec != PREC_BF16X3_NR) return hipErrorInvalidValue;
  const int UT = ut_for(a.U);
  if (UT == 16) return fd ? launch_lama_prec<16, true>(a, prec, s) : launch_lama_prec<16, false>(a, prec, s);
  return fd ? launch_lama_prec<32, true>(a, prec, s) : launch_lama_prec<32, false>(a, prec, s);
}

}  // namespace dbpeq
