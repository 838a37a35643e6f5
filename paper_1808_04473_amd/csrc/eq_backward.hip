// Hand-written adjoint of the PD and FD L-MMSE equalisers (the paper gives
// the forward maps only; the derivation is in dbpeq.h and the FP64 oracle).
//
// For one system with A = G + rho I, z = A^{-1} y^MRC, d = diag(A^{-1}),
// upstream gradients gz (complex, of z) and gs (real, of sigma2 = N0 d):
//   lambda = A^{-1} gz,  Q = A^{-1} diag(gs) A^{-1},
//   grad_H = (y - H z) lambda^H - H lambda z^H - 2 N0 H Q,   grad_y = H lambda,
//   grad_N0 = -Re(z^H lambda)/E_s + sum_u gs_u d_u - N0 tr(Q)/E_s.
// PD treats each subcarrier as one system.  FD first recomputes every local
// estimate of a subcarrier (pass A), forms the fusion-rule gradients
// (optimal weights nu = p/S, p = 1/sigma2_c, depend on sigma2_c), then
// differentiates each cluster (pass B).  A wave recomputes the factor of its
// systems from H (nothing is stored by the forward call) and streams the rows
// of H once more to write grad_H and grad_y.
#include "eq_round.h"

namespace dbpeq {

template <int UT>
struct BSmem {
  static constexpr int NSYS = 64 / UT;
  Smem<UT> r;
  float2 L[NSYS][UT];   // lambda of each system of the round
  float4 FB[NSYS][UT];  // FD: (S, sum_c nu_c g_nu_c) per (subcarrier, user)
};

// Gradient of one round of systems.  Lane (sme, i) holds the upstream
// gradients gzc, gsc of user i of system sme and its factorisation r.
// Streams the systems' rows to write grad_H / grad_y; returns this lane's
// share of grad_N0.
template <int UT, class Seg>
__device__ __forceinline__ float round_backward(const BwdArgs &a, BSmem<UT> &sm, LocalSolve<UT> &r,
                                                int nvalid, Seg seg, float2 gzc, float gsc) {
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
  const int col = lane % UT;
  const int U = a.U;
  const float inv_es = 1.0f / a.es;

  // lambda = A^{-1} gz
  const float2 lam = solve<UT>(r.f, i, gzc);
  const bool use_q = __ballot(gsc != 0.f) != 0ull;

  float gn0 = -(r.z.x * lam.x + r.z.y * lam.y) * inv_es + gsc * r.d;

  __syncthreads();  // the matrix slots are reused for Q below
  if (use_q) {
    // column i of A^{-1} = X^H X: ainv[k] = sum_m conj(X_mk) X_mi (X = L^{-1},
    // lane k holds column k), one m at a time over all k: X_mk is the DPP
    // broadcast of lane k fused into the FMACs, and the UT sums are
    // independent
    float2 ainv[UT];
#pragma unroll
    for (int k = 0; k < UT; ++k) ainv[k] = make_float2(0.f, 0.f);
    sfor<UT>([&](auto M) {
      constexpr int m = M;
      const BSrc bx = bsrc<UT>(r.f.x[m].x), by = bsrc<UT>(r.f.x[m].y);
      sfor<UT>([&](auto K) {
        constexpr int k = K;
        // conj(X_mk) X_mi
        fmac_rowbcast<k % 16, false, k == 0 ? 4 : 0>(ainv[k].x, bpick<k>(bx), r.f.x[m].x);
        fmac_rowbcast<k % 16, false, k == 0 ? 4 : 0>(ainv[k].y, bpick<k>(bx), r.f.x[m].y);
      });
      sfor<UT>([&](auto K) {
        constexpr int k = K;
        fmac_rowbcast<k % 16, false, k == 0 ? 4 : 0>(ainv[k].x, bpick<k>(by), r.f.x[m].y);
        fmac_rowbcast<k % 16, true, 0>(ainv[k].y, bpick<k>(by), r.f.x[m].x);
      });
      step_fence();
    });
    // column i of Q: Q_ki = sum_u A^{-1}_ku gs_u A^{-1}_ui, A^{-1}_ku from lane u
    float2 q[UT];
#pragma unroll
    for (int k = 0; k < UT; ++k) q[k] = make_float2(0.f, 0.f);
    float tr = 0.f;
#pragma unroll
    for (int k = 0; k < UT; ++k) tr += ainv[k].x * ainv[k].x + ainv[k].y * ainv[k].y;
    gn0 -= a.n0 * gsc * tr * inv_es;  // tr(Q) = sum_u gs_u sum_k |A^{-1}_ku|^2
    float dep = 0.f;
    sfor<UT>([&](auto Uu) {
      constexpr int u = Uu;
      const float gsu = gbcast<UT, u>(gsc);
      const float2 w = make_float2(ainv[u].x * gsu, ainv[u].y * gsu);  // gs_u A^{-1}_ui
      // q[k] += A^{-1}_ku w with A^{-1}_ku = ainv[k] of lane u
      if constexpr (UT == 16) {
        // ainv[k] itself is the DPP source (not written here)
        sfor<UT>([&](auto K) {
          constexpr int k = K;
          fmac_rowbcast<u, false, u == 0 && k == 0 ? 4 : 0>(q[k].x, ainv[k].x, w.x);
          fmac_rowbcast<u, false, 0>(q[k].y, ainv[k].x, w.y);
          fmac_rowbcast<u, true, 0>(q[k].x, ainv[k].y, w.y);
          fmac_rowbcast<u, false, 0>(q[k].y, ainv[k].y, w.x);
        });
      } else {
        // a swap per source and lane: broadcasts from registers, each step tied
        // to the previous one so that they are not all hoisted
        sfor<UT>([&](auto K) {
          constexpr int k = K;
          float2 src = ainv[k];
          asm volatile("" : "+v"(src.x), "+v"(src.y) : "v"(dep));
          const float2 aku = gbcast2<UT, u>(src);
          q[k].x += aku.x * w.x - aku.y * w.y;
          q[k].y += aku.x * w.y + aku.y * w.x;
        });
        dep = q[UT - 1].x;
      }
      step_fence();
    });
#pragma unroll
    for (int k = 0; k < UT; ++k) lds_el<UT>(sm.r.A[sme], k, i) = q[k];
  }
  sm.r.M[sme][i] = r.z;
  sm.L[sme][i] = lam;
  __syncthreads();

  // ---- stream the rows again: grad_H and grad_y
  if (nvalid > 0) {
    const int g = lane / UT;
    float2 zc = sm.r.M[0][col], lc = sm.L[0][col];
    float2 qc[UT];
    if (use_q) {
#pragma unroll
      for (int k = 0; k < UT; ++k) qc[k] = lds_el<UT>(sm.r.A[0], k, col);
    }
    stream_blocks<UT, kLoadLast>(
        nvalid, U, seg,
        [&](const Slot &b) {
          float2 *gHw = a.gH ? a.gH + (b.Hw - a.H) : nullptr;
          float2 *gyw = a.gy ? a.gy + (b.yw - a.y) : nullptr;
          sfor<8>([&](auto E) {
            constexpr int e = E;
            const float2 h = slot_h<UT>(b, e, U);
            const float hzx = gsum<UT>(h.x * zc.x - h.y * zc.y);
            const float hzy = gsum<UT>(h.x * zc.y + h.y * zc.x);
            const float hlx = gsum<UT>(h.x * lc.x - h.y * lc.y);
            const float hly = gsum<UT>(h.x * lc.y + h.y * lc.x);
            const float2 yv = slot_y<UT, e>(b);
            const float rx = yv.x - hzx, ry = yv.y - hzy;
            // (y - Hz)_row conj(lambda_col) - (H lambda)_row conj(z_col)
            float gx = rx * lc.x + ry * lc.y - (hlx * zc.x + hly * zc.y);
            float gy = ry * lc.x - rx * lc.y - (hly * zc.x - hlx * zc.y);
            if (use_q) {
              // (H Q)_{row,col} = sum_k H[row][k] Q[k][col]: H[row][k] is the DPP
              // row broadcast of lane k, fused into the FMACs; two partial sums
              // per component for independent chains
              const BSrc bx = bsrc<UT>(h.x), by = bsrc<UT>(h.y);
              float q[4] = {0.f, 0.f, 0.f, 0.f};
              sfor<UT>([&](auto K) {
                constexpr int k = K;
                constexpr int p = 2 * (k & 1);
                fmac_rowbcast<k % 16, false, k == 0 ? 4 : 0>(q[p], bpick<k>(bx), qc[k].x);
                fmac_rowbcast<k % 16, false, 0>(q[p + 1], bpick<k>(bx), qc[k].y);
                fmac_rowbcast<k % 16, true, k == 0 ? 4 : 0>(q[p], bpick<k>(by), qc[k].y);
                fmac_rowbcast<k % 16, false, 0>(q[p + 1], bpick<k>(by), qc[k].x);
              });
              gx -= 2.f * a.n0 * (q[0] + q[2]);
              gy -= 2.f * a.n0 * (q[1] + q[3]);
            }
            const int row = b.rb + slot_row(e, g);
            if (row < b.r1) {
              if (gHw && col < U) gHw[(size_t)row * U + col] = make_float2(gx, gy);
              if (gyw && col == 0) gyw[row] = make_float2(hlx, hly);
            }
          });
        },
        [&](int s) {
          if (s + 1 < nvalid) {
            zc = sm.r.M[s + 1][col];
            lc = sm.L[s + 1][col];
            if (use_q) {
#pragma unroll
              for (int k = 0; k < UT; ++k) qc[k] = lds_el<UT>(sm.r.A[s + 1], k, col);
            }
          }
        });
  }
  __syncthreads();
  return (sme < nvalid && i < U) ? gn0 : 0.f;
}

template <int UT, class Seg>
__device__ __forceinline__ void gram_round(const BwdArgs &a, BSmem<UT> &sm, int nvalid,
                                           const Seg &seg) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  gram_stream<UT, PREC_FP32, kLoadKeep>(nvalid, a.U, seg, [&](int s, const Acc<UT> &acc, float2 mf) {
    store_gram<UT, PREC_FP32>(sm.r.A[s], acc, a.rho);
    if (lane < UT) sm.r.M[s][lane] = mf;
  });
  for (int s = nvalid; s < NSYS; ++s) {
    store_identity<UT>(sm.r.A[s]);
    if (lane < UT) sm.r.M[s][lane] = make_float2(0.f, 0.f);
  }
  __syncthreads();
}

template <int UT>
__device__ __forceinline__ float pd_backward_task(const BwdArgs &a, int task, BSmem<UT> &sm) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int nvalid = min(NSYS, a.W - task * NSYS);
  auto seg = [&](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
    const size_t w = (size_t)task * NSYS + s;
    Hw = a.H + w * HB;
    yw = a.y + w * a.B;
    r0 = 0;
    r1 = a.B;
  };
  gram_round<UT>(a, sm, nvalid, seg);
  LocalSolve<UT> r;
  local_solve<UT>(r, sm.r, sme, i, a.U);
  const bool live = sme < nvalid && i < a.U;
  const size_t w = (size_t)task * NSYS + sme;
  float2 gzc = make_float2(0.f, 0.f);
  float gsc = 0.f;
  if (live) {
    if (a.gz) gzc = a.gz[w * a.U + i];
    if (a.gs) gsc = a.gs[w * a.U + i];
  }
  return round_backward<UT>(a, sm, r, nvalid, seg, gzc, gsc);
}

template <int UT>
__device__ __forceinline__ float fd_backward_task(const BwdArgs &a, int task, BSmem<UT> &sm,
                                                  float4 *__restrict__ fwd) {
  constexpr int NSYS = 64 / UT;
  const int lane = lane_id();
  const int sme = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int C = a.C, U = a.U;
  const int w0 = task * a.spw;
  const int nsub = min(a.spw, a.W - w0);
  const int ntot = nsub * C;
  const bool optimal = a.nu == nullptr;
  float gn0 = 0.f;

  auto make_seg = [&](int base) {
    return [&a, base, C, w0, HB](int s, const float2 *&Hw, const float2 *&yw, int &r0, int &r1) {
      const int idx = base + s;
      const int wl = idx / C, c = idx - wl * C;
      const size_t w = (size_t)(w0 + wl);
      Hw = a.H + w * HB;
      yw = a.y + w * a.B;
      r0 = a.off[c];
      r1 = a.off[c + 1];
    };
  };

  // ---- pass A: local estimates and variances of every cluster
  if (optimal) {
    for (int base = 0; base < ntot; base += NSYS) {
      const int nvalid = min(NSYS, ntot - base);
      gram_round<UT>(a, sm, nvalid, make_seg(base));
      LocalSolve<UT> r;
      local_solve<UT>(r, sm.r, sme, i, U);
      const int idx = base + sme;
      if (sme < nvalid && i < U) {
        const int wl = idx / C, c = idx - wl * C;
        fwd[((size_t)(w0 + wl) * C + c) * U + i] = make_float4(r.z.x, r.z.y, a.n0 * r.d, 0.f);
      }
      __syncthreads();
    }
    __threadfence_block();
    __syncthreads();
    // fusion sums: S = sum_c p_c and sum_c nu_c g_nu_c for lane (wl, u)
    const int wl = lane / UT;
    if (wl < nsub && i < U) {
      const size_t w = (size_t)(w0 + wl);
      const float2 gz = a.gz ? a.gz[w * U + i] : make_float2(0.f, 0.f);
      const float gs = a.gs ? a.gs[w * U + i] : 0.f;
      float S = 0.f;
      for (int c = 0; c < C; ++c) S += 1.0f / fwd[(w * C + c) * U + i].z;
      float sng = 0.f;
      for (int c = 0; c < C; ++c) {
        const float4 v = fwd[(w * C + c) * U + i];
        const float nu = (1.0f / v.z) / S;
        const float gnu = gz.x * v.x + gz.y * v.y + 2.f * gs * nu * v.z;
        sng += nu * gnu;
      }
      sm.FB[wl][i] = make_float4(S, sng, 0.f, 0.f);
    }
    __syncthreads();
  }

  // ---- pass B: each cluster's adjoint with the fusion-rule upstream gradients
  for (int base = 0; base < ntot; base += NSYS) {
    const int nvalid = min(NSYS, ntot - base);
    auto seg = make_seg(base);
    gram_round<UT>(a, sm, nvalid, seg);
    LocalSolve<UT> r;
    local_solve<UT>(r, sm.r, sme, i, U);
    const int idx = base + sme;
    const int wl = idx / C, c = idx - wl * C;
    const size_t w = (size_t)(w0 + wl);
    float2 gzc = make_float2(0.f, 0.f);
    float gsc = 0.f;
    if (sme < nvalid && i < U) {
      const float2 gz = a.gz ? a.gz[w * U + i] : make_float2(0.f, 0.f);
      const float gs = a.gs ? a.gs[w * U + i] : 0.f;
      const float s2c = a.n0 * r.d;
      // partial w.r.t. the weight with the weights held fixed
      float nu, gnu;
      if (optimal) {
        const float4 fb = sm.FB[wl][i];
        const float p = 1.0f / s2c;
        nu = p / fb.x;
        gnu = gz.x * r.z.x + gz.y * r.z.y + 2.f * gs * nu * s2c;
        const float gp = (gnu - fb.y) / fb.x;
        gsc = gs * nu * nu - p * p * gp;
      } else {
        nu = a.nu[(w * C + c) * U + i];
        gnu = gz.x * r.z.x + gz.y * r.z.y + 2.f * gs * nu * s2c;
        gsc = gs * nu * nu;
        if (a.gnu) a.gnu[(w * C + c) * U + i] = gnu;
      }
      gzc = make_float2(nu * gz.x, nu * gz.y);
    }
    gn0 += round_backward<UT>(a, sm, r, nvalid, seg, gzc, gsc);
  }
  return gn0;
}

// 3 waves per SIMD at UT = 16 (168 VGPRs), 2 at UT = 32.
template <int UT, bool FD>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(UT == 16 ? 3 : 2, 8))) void eq_backward_kernel(const BwdArgs a, float4 *fwd) {
  __shared__ BSmem<UT> sm;
  float g = FD ? fd_backward_task<UT>(a, blockIdx.x, sm, fwd) : pd_backward_task<UT>(a, blockIdx.x, sm);
  // wave sum of the grad_N0 shares
  g = row16_sum(g);
  g += __shfl_xor(g, 16);
  g += __shfl_xor(g, 32);
  if (lane_id() == 0) a.gn0_part[blockIdx.x] = g;
}

// Deterministic sum of the per-wave shares into the grad_N0 scalar.
__global__ __launch_bounds__(256) void sum_parts_kernel(const float *__restrict__ part, int n, float *out) {
  __shared__ float red[256];
  float s = 0.f;
  for (int t = threadIdx.x; t < n; t += 256) s += part[t];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

int backward_tasks(int W, int U, int C, bool fd, int *spw) {
  const int UT = ut_for(U);
  const int nsys = 64 / UT;
  *spw = fd_spw(UT, C);
  return fd ? (W + *spw - 1) / *spw : (W + nsys - 1) / nsys;
}

hipError_t launch_backward(const BwdArgs &a, bool fd, int ntasks, hipStream_t s) {
  const int UT = ut_for(a.U);
  float4 *fwd = reinterpret_cast<float4 *>(a.gn0_part + ((ntasks + 63) / 64) * 64);
  const dim3 grid(ntasks), block(64);
  if (UT == 16) {
    if (fd) hipLaunchKernelGGL((eq_backward_kernel<16, true>), grid, block, 0, s, a, fwd);
    else hipLaunchKernelGGL((eq_backward_kernel<16, false>), grid, block, 0, s, a, fwd);
  } else {
    if (fd) hipLaunchKernelGGL((eq_backward_kernel<32, true>), grid, block, 0, s, a, fwd);
    else hipLaunchKernelGGL((eq_backward_kernel<32, false>), grid, block, 0, s, a, fwd);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.gn0) {
    hipLaunchKernelGGL(sum_parts_kernel, dim3(1), dim3(256), 0, s, a.gn0_part, ntasks, a.gn0);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace dbpeq
