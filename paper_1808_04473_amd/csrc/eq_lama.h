// LAMA iteration (Algorithm 1) on statistics held in registers, shared by
// the single-vector kernels (eq_lama.hip) and the several-vector ones
// (eq_symbols.hip).
#pragma once
#include "eq_round.h"

namespace dbpeq {

// Posterior mean and E|s|^2 of one PAM coordinate with levels
// (2k - (M - 1)) * lvl, k = 0..M-1, observed as x in N(0, tau/2) noise.
template <int M>
__device__ __forceinline__ void pam_posterior(float x, float inv_tau, float lvl, float &mean, float &second) {
  float d[M];
  float dmin = 3.0e38f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const float a = (float)(2 * k - (M - 1)) * lvl;
    d[k] = (x - a) * (x - a) * inv_tau;
    dmin = fminf(dmin, d[k]);
  }
  float sw = 0.f, sa = 0.f, sa2 = 0.f;
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const float a = (float)(2 * k - (M - 1)) * lvl;
    const float w = __expf(dmin - d[k]);
    sw += w;
    sa = fmaf(w, a, sa);
    sa2 = fmaf(w, a * a, sa2);
  }
  const float inv = 1.0f / sw;
  mean = sa * inv;
  second = sa2 * inv;
}

// t_max iterations of Algorithm 1 for lane i of a group whose f.x[k] holds
// conj(G_ik) (so that apply_xh gives (G s)_i) and m = y^MRC_i, with noise n0
// and system ratio beta over U users of a square QAM with M levels per
// coordinate and energy es.  Returns z of the last iteration in z and its
// variance N0 + beta phi in tau.
template <int UT, int M>
__device__ __forceinline__ void lama_iterate(const Factor<UT> &f, float2 m, int i, int U, float n0, float beta,
                                             float es, int t_max, float2 &z, float &tau) {
  const float lvl = sqrtf(3.0f * es / (2.0f * (float)(M * M - 1)));
  const float inv_u = 1.0f / (float)U;
  float2 s = make_float2(0.f, 0.f), v = make_float2(0.f, 0.f);
  float phi = es;
  z = m;
  tau = n0 + beta * es;
  for (int t = 0; t < t_max; ++t) {
    const float2 gs = apply_xh<UT>(f, s);
    z = make_float2(m.x + s.x - gs.x + v.x, m.y + s.y - gs.y + v.y);
    tau = n0 + beta * phi;
    const float inv_tau = 1.0f / tau;
    float mr, qr, mi, qi;
    pam_posterior<M>(z.x, inv_tau, lvl, mr, qr);
    pam_posterior<M>(z.y, inv_tau, lvl, mi, qi);
    const float g = (qr - mr * mr) + (qi - mi * mi);
    const float phi_new = gsum<UT>(i < U ? g : 0.f) * inv_u;
    const float c = beta * phi_new * inv_tau;
    v = make_float2(c * (z.x - s.x), c * (z.y - s.y));
    s = i < U ? make_float2(mr, mi) : make_float2(0.f, 0.f);
    phi = phi_new;
  }
}

}  // namespace dbpeq
