// FP64 re-solve of the systems queued by the forward kernels.
//
// The queue holds subcarriers (or ragged systems) for which some local (FD)
// or fused (PD) matrix A = G + rho I had a condition estimate above
// EQ_COND_LIMIT or a failed FP32 pivot.  One 64-lane workgroup recomputes
// such a system from the complex64 inputs with FP64 arithmetic: Gram and MRC
// (Section II-C), the Cholesky factor, z = A^{-1} y^MRC, d = diag(A^{-1}) and,
// for FD, the fusion of eq. (fusionrule) with the weights of Lemma 1.  It is
// rare and simple: a plain LDS-resident algorithm, no tiling.
#include "eq_ragged.h"

namespace dbpeq {

struct Dc {
  double x, y;
};

__device__ __forceinline__ Dc dmulc(Dc a, Dc b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ Dc dmul(Dc a, Dc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// Receive vectors per re-solve pass (the widest symbol tile).
constexpr int kF64Sym = 32;

struct F64Smem {
  Dc L[EQ_MAX_U][EQ_MAX_U + 1];
  Dc X[EQ_MAX_U][EQ_MAX_U + 1];  // X[j][u] = (L^{-1})_ju
  Dc m[EQ_MAX_U];
  Dc t[EQ_MAX_U];
  Dc Z[kF64Sym][EQ_MAX_U];       // estimates (FD: weighted sums) per vector
  int fail;
};

// Re-solves one system for nsym <= kF64Sym receive vectors (vector s at
// yw + s * ys, its estimate at zw + s * zs).  Clusters c = 0..nclus-1 own rows
// off(c)..off(c+1)-1 (PD passes one cluster covering every row); nu_w = [C][U]
// user weights or nullptr; on_info(c, fail) reports each cluster's FP64 pivot
// status.
template <class Off, class Info>
__device__ void fp64_system(F64Smem &sm, const float2 *__restrict__ Hw, const float2 *__restrict__ yw,
                            int U, int nclus, Off off, double n0, double rho, double ub, bool fd,
                            const float *nu_w, float2 *zw, float *s2w, Info on_info,
                            int nsym, size_t ys, size_t zs) {
  const int tid = threadIdx.x;
  double sw = 0.0, sv = 0.0;
  bool any_bad = false;
  for (int c = 0; c < nclus; ++c) {
    const int r0 = off(c), r1 = off(c + 1);
    // Gram (lower triangle) + rho I
    for (int p = tid; p < U * U; p += 64) {
      const int i = p / U, j = p % U;
      if (j > i) continue;
      Dc acc = {0.0, 0.0};
      for (int b = r0; b < r1; ++b) {
        const float2 hi = Hw[(size_t)b * U + i], hj = Hw[(size_t)b * U + j];
        acc.x += (double)hi.x * hj.x + (double)hi.y * hj.y;
        acc.y += (double)hi.x * hj.y - (double)hi.y * hj.x;
      }
      if (i == j) acc.x += rho;
      sm.L[i][j] = acc;
    }
    if (tid == 0) sm.fail = 0;
    __syncthreads();
    // Cholesky A = L L^H, column by column, lower triangle in place
    for (int j = 0; j < U; ++j) {
      if (tid == 0) {
        double s = sm.L[j][j].x;
        for (int k = 0; k < j; ++k) s -= sm.L[j][k].x * sm.L[j][k].x + sm.L[j][k].y * sm.L[j][k].y;
        if (!(s > 0.0) && sm.fail == 0) sm.fail = j + 1;
        sm.L[j][j] = {sqrt(s), 0.0};
      }
      __syncthreads();
      for (int i = j + 1 + tid; i < U; i += 64) {
        Dc s = sm.L[i][j];
        for (int k = 0; k < j; ++k) {
          const Dc p = dmulc(sm.L[i][k], sm.L[j][k]);
          s.x -= p.x;
          s.y -= p.y;
        }
        sm.L[i][j] = {s.x / sm.L[j][j].x, s.y / sm.L[j][j].x};
      }
      __syncthreads();
    }
    // the columns of L^{-1} (thread u)
    if (tid < U) {
      const int u = tid;
      for (int j = 0; j < U; ++j) {
        Dc s = {j == u ? 1.0 : 0.0, 0.0};
        for (int k = u; k < j; ++k) {
          const Dc p = dmul(sm.L[j][k], sm.X[k][u]);
          s.x -= p.x;
          s.y -= p.y;
        }
        sm.X[j][u] = j < u ? Dc{0.0, 0.0} : Dc{s.x / sm.L[j][j].x, s.y / sm.L[j][j].x};
      }
    }
    __syncthreads();
    // error variance and fusion weight of user u (estimate and variance
    // divided by the gain 1 - sigma2 ub: the unbiased L-MMSE, 1 at ub = 0)
    double wgt = 1.0, kub = 1.0;
    if (tid < U) {
      const int u = tid;
      double d = 0.0;
      for (int j = u; j < U; ++j) d += sm.X[j][u].x * sm.X[j][u].x + sm.X[j][u].y * sm.X[j][u].y;
      kub = 1.0 / (1.0 - n0 * d * ub);
      const double s2 = n0 * d * kub;
      if (fd) {
        if (nu_w) {
          wgt = nu_w[(size_t)c * U + u];
          sv += wgt * wgt * s2;
        } else {
          wgt = 1.0 / s2;
          sw += wgt;
        }
      } else {
        sv = s2;
      }
      if (sm.fail) any_bad = true;
    }
    for (int s = 0; s < nsym; ++s) {
      const float2 *ysv = yw + (size_t)s * ys;
      // MRC of vector s
      if (tid < U) {
        Dc acc = {0.0, 0.0};
        for (int b = r0; b < r1; ++b) {
          const float2 h = Hw[(size_t)b * U + tid], yv = ysv[b];
          acc.x += (double)h.x * yv.x + (double)h.y * yv.y;
          acc.y += (double)h.x * yv.y - (double)h.y * yv.x;
        }
        sm.m[tid] = acc;
      }
      __syncthreads();
      // t = L^{-1} m (thread 0)
      if (tid == 0) {
        for (int i = 0; i < U; ++i) {
          Dc t = sm.m[i];
          for (int k = 0; k < i; ++k) {
            const Dc p = dmul(sm.L[i][k], sm.t[k]);
            t.x -= p.x;
            t.y -= p.y;
          }
          sm.t[i] = {t.x / sm.L[i][i].x, t.y / sm.L[i][i].x};
        }
      }
      __syncthreads();
      // z_u = sum_j conj(X_ju) t_j, weighted and summed over the clusters (FD)
      if (tid < U) {
        const int u = tid;
        Dc z = {0.0, 0.0};
        for (int j = u; j < U; ++j) {
          z.x += sm.X[j][u].x * sm.t[j].x + sm.X[j][u].y * sm.t[j].y;
          z.y += sm.X[j][u].x * sm.t[j].y - sm.X[j][u].y * sm.t[j].x;
        }
        z.x *= kub;
        z.y *= kub;
        if (fd) {
          const Dc prev = c == 0 ? Dc{0.0, 0.0} : sm.Z[s][u];
          sm.Z[s][u] = {prev.x + wgt * z.x, prev.y + wgt * z.y};
        } else {
          sm.Z[s][u] = z;
        }
      }
      __syncthreads();
    }
    if (tid == 0) on_info(c, sm.fail);
    __syncthreads();
  }
  if (tid < U) {
    const double nanv = __longlong_as_double(0x7ff8000000000000ll);
    const bool norm = fd && !nu_w;
    for (int s = 0; s < nsym; ++s) {
      double zx = sm.Z[s][tid].x, zy = sm.Z[s][tid].y;
      if (norm) {
        zx /= sw;
        zy /= sw;
      }
      if (any_bad) zx = zy = nanv;
      zw[(size_t)s * zs + tid] = make_float2((float)zx, (float)zy);
    }
    double so = norm ? 1.0 / sw : sv;
    if (any_bad) so = nanv;
    if (s2w) s2w[tid] = (float)so;
  }
  __syncthreads();
}

// The queue (a.fb_count, a.fb_list) is filled by the forward kernel.  Blocks
// 0 .. min(n, grid) - 1 take entries; the last of them to finish sets the
// count and its own completion counter back to zero (every block that takes
// entries has read the count by then; the others find nothing to do whether
// they read it before or after), so every call leaves the workspace as the
// next one expects it, and a call that routed nothing does no atomics.
template <bool FD>
__global__ __launch_bounds__(64) void eq_fp64_kernel(const FwdArgs a) {
  __shared__ F64Smem sm;
  const int n = min(*a.fb_count, a.W);
  if ((int)blockIdx.x >= n) return;
  // ZF is the L-MMSE solve with rho = 0
  const double rho = a.eqz == EQZ_ZF ? 0.0 : (double)a.n0 / (double)a.es;
  const size_t HB = (size_t)a.B * a.U;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int w = a.fb_list[q];
    if (w < 0 || w >= a.W) continue;
    auto off = [&](int c) { return FD ? (int)a.off[c] : (c == 0 ? 0 : a.B); };
    auto info = [&](int c, int fail) {
      if (!a.info) return;
      const size_t ii = FD ? (size_t)w * a.C + c : (size_t)w;
      a.info[ii] = fail | (a.info[ii] & EQ_INFO_FP64);
    };
    fp64_system(sm, a.H + (size_t)w * HB, a.y + (size_t)w * a.ysw, a.U, FD ? a.C : 1, off,
                (double)a.n0, rho, (double)a.ub, FD, a.nu ? a.nu + (size_t)w * a.C * a.U : nullptr,
                a.z + (size_t)w * a.zsw, a.s2 ? a.s2 + (size_t)w * a.U : nullptr, info, a.nsym,
                (size_t)a.B, (size_t)a.U);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // every block read the count before it arrives here
    if (atomicAdd(a.fb_done, 1) == min(n, (int)gridDim.x) - 1) {
      *a.fb_count = 0;
      *a.fb_done = 0;
    }
  }
}

// The ragged form runs after the persistent launch, so it also clears that
// launch's queue heads for the next execution; its own count is cleared as
// in eq_fp64_kernel.
template <bool FD>
__global__ __launch_bounds__(64) void eq_fp64_ragged_kernel(const RaggedArgs a) {
  __shared__ F64Smem sm;
  if (blockIdx.x == 0 && threadIdx.x < kQueues) a.counter[threadIdx.x * kQueueStride] = 0;
  const int n = min(*a.fb_count, a.nsys);
  if ((int)blockIdx.x >= n) return;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int k = a.fb_list[q];
    if (k < 0 || k >= a.nsys) continue;
    const RSys d = a.sys[k];
    auto off = [&](int c) { return FD ? a.offs[d.off_first + c] : (c == 0 ? 0 : d.B); };
    int worst = 0;
    auto info = [&](int c, int fail) {
      if (fail && !worst) worst = fail;
    };
    fp64_system(sm, a.Hpool + d.h_off, a.ypool + d.y_off, d.U, FD ? d.C : 1, off, (double)d.n0,
                (double)d.n0 / (double)a.es, 0.0, FD, nullptr, a.zpool + d.z_off,
                a.s2pool ? a.s2pool + d.z_off : nullptr, info, 1, 0, 0);
    if (threadIdx.x == 0 && a.info) a.info[k] = worst | EQ_INFO_FP64;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    // every block read the count before it arrives here
    if (atomicAdd(a.fb_done, 1) == min(n, (int)gridDim.x) - 1) {
      *a.fb_count = 0;
      *a.fb_done = 0;
    }
  }
}

hipError_t launch_fp64_resolve(const FwdArgs &a, bool fd, hipStream_t s) {
  const int grid = a.W < 512 ? (a.W > 0 ? a.W : 1) : 512;
  if (fd)
    hipLaunchKernelGGL((eq_fp64_kernel<true>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((eq_fp64_kernel<false>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fp64_ragged(const RaggedArgs &a, bool fd, hipStream_t s) {
  const int grid = a.nsys < 512 ? (a.nsys > 0 ? a.nsys : 1) : 512;
  if (fd)
    hipLaunchKernelGGL((eq_fp64_ragged_kernel<true>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((eq_fp64_ragged_kernel<false>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

}  // namespace dbpeq
