// Per-wave round state shared by the forward and backward kernels: the LDS
// staging of a round of NSYS = 64/UT small systems and the per-group
// factorisation of one system.
#pragma once
#include "eq_device.h"

namespace dbpeq {

// NS matrix slots (one per system of a round by default; fewer when the
// work items hold fewer systems than there are lane groups, which leaves
// room for more waves per CU).
template <int UT, int NSLOT = 64 / UT>
struct Smem {
  static constexpr int NSYS = 64 / UT;
  static constexpr int NS = NSLOT;
  float2 A[NS][UT][UT];  // swizzled rows (lds_el)
  float2 M[NS][UT];
  float4 F[NS][UT];
  int routed[NSYS];
};

// LDS slot of lane group g: groups beyond the slots alias the last one (they
// then solve a copy of that system, and write nothing).
template <class SM>
__device__ __forceinline__ int slot_of(int g) {
  return g < SM::NS ? g : SM::NS - 1;
}

// Loads row i of system `sme` from LDS and factorises / solves it.
template <int UT>
struct LocalSolve {
  Factor<UT> f;
  float2 z;
  float d;
  float norm1;
  int fail;
  bool bad;
};

// PAD (factor_solve): leave out the steps of the factorisation and inverse
// that only touch padded users, for at most 24 users in a 32-lane group
// (PAD & 1) or 8 in a 16-lane group (PAD & 2); the FD forms, which solve one
// system per cluster, use it (PD measured no faster).
template <int UT, int PAD = 0, class SM>
__device__ __forceinline__ void local_solve(LocalSolve<UT> &r, SM &sm, int sme, int i, int U) {
  float rowsum = 0.f;
#pragma unroll
  for (int k = 0; k < UT; ++k) {
    r.f.a[k] = lds_el<UT>(sm.A[sme], i, k);
    rowsum = abs_row_acc(rowsum, r.f.a[k]);
  }
  const float2 m = sm.M[sme][i];
  r.bad = gany<UT>(!isfinite(abs_row_acc(rowsum, m)));
  r.norm1 = gmax<UT>(i < U ? rowsum * (1.f / kRowScale) : 0.f);
  // with fewer slots than groups (PD items of one 32-lane system) the freed
  // registers raise occupancy, so the inverse reads L from LDS there
  // with a slot per system, the 32 x 32 forms run their two block products
  // on MFMA through the slots (read above, free until the solve ends)
  float2 *split = nullptr;
  if constexpr (UT == 32 && SM::NS == SM::NSYS) split = &sm.A[0][0][0];
  r.z = factor_solve<UT, PAD>(r.f, i, m, r.fail, SM::NS < SM::NSYS ? sm.A[sme] : nullptr, split, U);
  r.d = inv_diag<UT>(r.f);
}

// One refinement step for the systems of a round: every group's z goes to
// LDS, the residual pass streams the systems' rows again and each group
// solves A dz = H^H (y - H z) - rho z as dz = X^H (X r) with X = L^{-1}
// (A^{-1} = X^H X): the columns of X are parked in LDS during the pass,
// t = X r is read back along rows of X and dz = X^H t uses the reloaded
// columns, so the factor L is dead once the inverse is formed.
template <int UT, class SM, class Rho, class Seg>
__device__ __forceinline__ void refine_round(LocalSolve<UT> &r, SM &sm, int nvalid, int U,
                                             Rho rhof, Seg seg, bool live) {
  const int lane = lane_id();
  const int sme = slot_of<SM>(lane / UT), i = lane % UT;
  __syncthreads();
  sm.M[sme][i] = r.z;
  // row u of the slot holds column u of X: lds_el(A, u, k) = X_ku
#pragma unroll
  for (int k = 0; k < UT; ++k) lds_el<UT>(sm.A[sme], i, k) = r.f.x[k];
  __syncthreads();
  residual_stream<UT>(
      nvalid, U, seg, [&](int s) { return sm.M[s][lane % UT]; },
      [&](int s, float2 n) {
        const float2 zc = sm.M[s][lane % UT];
        const float rho = rhof(s);
        if (lane < UT) sm.F[s][lane] = make_float4(n.x - rho * zc.x, n.y - rho * zc.y, 0.f, 0.f);
      });
  __syncthreads();
  asm volatile("" ::: "memory");  // reload the parked columns instead of keeping them live
  // t_j = sum_u X_ju r_u at lane j
  float tx = 0.f, ty = 0.f;
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const float2 x = lds_el<UT>(sm.A[sme], u, i);
    const float4 rv = sm.F[sme][u];
    tx = fmaf(x.x, rv.x, fmaf(-x.y, rv.y, tx));
    ty = fmaf(x.x, rv.y, fmaf(x.y, rv.x, ty));
  }
#pragma unroll
  for (int k = 0; k < UT; ++k) r.f.x[k] = lds_el<UT>(sm.A[sme], i, k);
  const float2 dz = apply_xh<UT>(r.f, make_float2(tx, ty));
  if (live) {
    r.z.x += dz.x;
    r.z.y += dz.y;
  }
}

}  // namespace dbpeq
