// FP64 re-solve of the subcarriers queued by the forward kernels.
//
// The queue holds subcarriers for which some local (FD) or fused (PD) matrix
// A = G + rho I had a condition estimate above EQ_COND_LIMIT or a failed FP32
// pivot.  One 64-lane workgroup recomputes such a subcarrier from the
// complex64 inputs with FP64 arithmetic: Gram and MRC (Section II-C), the
// Cholesky factor, z = A^{-1} y^MRC, d = diag(A^{-1}) and, for FD, the fusion
// of eq. (fusionrule) with the weights of Lemma 1.  It is rare and simple:
// a plain LDS-resident algorithm, no tiling.
#include "eq_common.h"

namespace dbpeq {

struct Dc { double x, y; };

__device__ __forceinline__ Dc dmulc(Dc a, Dc b) {  // a * conj(b)
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ Dc dmul(Dc a, Dc b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

template <bool FD>
__global__ __launch_bounds__(64) void eq_fp64_kernel(const FwdArgs a) {
  __shared__ Dc L[EQ_MAX_U][EQ_MAX_U + 1];
  __shared__ Dc X[EQ_MAX_U][EQ_MAX_U + 1];  // X[j][u] = (L^{-1})_ju
  __shared__ Dc m[EQ_MAX_U];
  __shared__ Dc t[EQ_MAX_U];
  __shared__ int fail;
  const int tid = threadIdx.x;
  const int U = a.U;
  const int n = *a.fb_count;
  const double rho = (double)a.n0 / (double)a.es;
  const size_t HB = (size_t)a.B * U;
  for (int q = blockIdx.x; q < n; q += gridDim.x) {
    const int w = a.fb_list[q];
    const float2 *Hw = a.H + (size_t)w * HB;
    const float2 *yw = a.y + (size_t)w * a.B;
    const int nsys = FD ? a.C : 1;
    // fusion sums of thread u
    double sw = 0.0, szx = 0.0, szy = 0.0, sv = 0.0;
    bool any_bad = false;
    for (int c = 0; c < nsys; ++c) {
      const int r0 = FD ? a.off[c] : 0;
      const int r1 = FD ? a.off[c + 1] : a.B;
      // Gram (lower triangle) and MRC
      for (int p = tid; p < U * U; p += 64) {
        const int i = p / U, j = p % U;
        if (j > i) continue;
        Dc acc = {0.0, 0.0};
        for (int b = r0; b < r1; ++b) {
          const float2 hi = Hw[(size_t)b * U + i], hj = Hw[(size_t)b * U + j];
          // conj(H_bi) H_bj
          acc.x += (double)hi.x * hj.x + (double)hi.y * hj.y;
          acc.y += (double)hi.x * hj.y - (double)hi.y * hj.x;
        }
        if (i == j) acc.x += rho;
        L[i][j] = acc;
      }
      if (tid < U) {
        Dc acc = {0.0, 0.0};
        for (int b = r0; b < r1; ++b) {
          const float2 h = Hw[(size_t)b * U + tid], yv = yw[b];
          acc.x += (double)h.x * yv.x + (double)h.y * yv.y;
          acc.y += (double)h.x * yv.y - (double)h.y * yv.x;
        }
        m[tid] = acc;
      }
      if (tid == 0) fail = 0;
      __syncthreads();
      // Cholesky, column by column (A = L L^H, lower triangle in place)
      for (int j = 0; j < U; ++j) {
        if (tid == 0) {
          double s = L[j][j].x;
          for (int k = 0; k < j; ++k) s -= L[j][k].x * L[j][k].x + L[j][k].y * L[j][k].y;
          if (!(s > 0.0) && fail == 0) fail = j + 1;
          L[j][j] = {sqrt(s), 0.0};
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < U; i += 64) {
          Dc s = L[i][j];
          for (int k = 0; k < j; ++k) {
            const Dc p = dmulc(L[i][k], L[j][k]);
            s.x -= p.x;
            s.y -= p.y;
          }
          L[i][j] = {s.x / L[j][j].x, s.y / L[j][j].x};
        }
        __syncthreads();
      }
      // forward substitution t = L^{-1} m (thread 0) and columns of L^{-1} (thread u)
      if (tid == 0) {
        for (int i = 0; i < U; ++i) {
          Dc s = m[i];
          for (int k = 0; k < i; ++k) {
            const Dc p = dmul(L[i][k], t[k]);
            s.x -= p.x;
            s.y -= p.y;
          }
          t[i] = {s.x / L[i][i].x, s.y / L[i][i].x};
        }
      }
      if (tid < U) {
        const int u = tid;
        for (int j = 0; j < U; ++j) {
          Dc s = {j == u ? 1.0 : 0.0, 0.0};
          for (int k = u; k < j; ++k) {
            const Dc p = dmul(L[j][k], X[k][u]);
            s.x -= p.x;
            s.y -= p.y;
          }
          X[j][u] = j < u ? Dc{0.0, 0.0} : Dc{s.x / L[j][j].x, s.y / L[j][j].x};
        }
      }
      __syncthreads();
      if (tid < U) {
        const int u = tid;
        double d = 0.0;
        Dc z = {0.0, 0.0};
        for (int j = u; j < U; ++j) {
          d += X[j][u].x * X[j][u].x + X[j][u].y * X[j][u].y;
          // conj(X_ju) t_j
          z.x += X[j][u].x * t[j].x + X[j][u].y * t[j].y;
          z.y += X[j][u].x * t[j].y - X[j][u].y * t[j].x;
        }
        const double s2 = (double)a.n0 * d;
        if (FD) {
          if (a.nu) {
            const double nu = a.nu[((size_t)w * a.C + c) * U + u];
            szx += nu * z.x;
            szy += nu * z.y;
            sv += nu * nu * s2;
          } else {
            const double p = 1.0 / s2;
            sw += p;
            szx += p * z.x;
            szy += p * z.y;
          }
        } else {
          szx = z.x;
          szy = z.y;
          sv = s2;
        }
        if (fail) any_bad = true;
      }
      if (tid == 0 && a.info) {
        const size_t ii = FD ? (size_t)w * a.C + c : (size_t)w;
        const int prev = a.info[ii];
        a.info[ii] = fail | (prev & EQ_INFO_FP64);
      }
      __syncthreads();
    }
    if (tid < U) {
      double zx, zy, so;
      if (FD && !a.nu) {
        zx = szx / sw;
        zy = szy / sw;
        so = 1.0 / sw;
      } else {
        zx = szx;
        zy = szy;
        so = sv;
      }
      if (any_bad) {
        zx = zy = so = __longlong_as_double(0x7ff8000000000000ll);
      }
      a.z[(size_t)w * U + tid] = make_float2((float)zx, (float)zy);
      if (a.s2) a.s2[(size_t)w * U + tid] = (float)so;
    }
    __syncthreads();
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

}  // namespace dbpeq
