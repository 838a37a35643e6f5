// C ABI of libdbpeq.so: host-side validation and dispatch.  Every argument is
// checked before the first HIP call, so invalid calls have no device effects.
#include <math.h>
#include <string.h>

#include <mutex>
#include <vector>

#include "eq_common.h"

using namespace dbpeq;

namespace {

// Measurement aid (eq_kernel_timer_*): pairs of events recorded around the
// main kernel of the forward calls while the timer is on.
struct KernelTimer {
  std::mutex mu;
  std::vector<hipEvent_t> ev;  // 2 per pair, created by eq_kernel_timer_start
  size_t used = 0;             // pairs handed out
  bool on = false;
};

KernelTimer &kernel_timer() {
  static KernelTimer t;
  return t;
}

// The next free pair, or two null events when the timer is off or full.
void timer_pair(hipEvent_t &e0, hipEvent_t &e1) {
  e0 = e1 = nullptr;
  KernelTimer &t = kernel_timer();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.on || 2 * (t.used + 1) > t.ev.size()) return;
  e0 = t.ev[2 * t.used];
  e1 = t.ev[2 * t.used + 1];
  ++t.used;
}

constexpr size_t kWsHeader = 256;

bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

eq_status check_problem(const eq_problem *p) {
  if (!p) return EQ_EINVAL;
  if (p->W < 0 || p->B < 1 || p->U < 1 || p->C < 1) return EQ_EINVAL;
  if (p->B > EQ_MAX_B || p->C > EQ_MAX_C) return EQ_ENOTSUP;
  if (p->C > p->B) return EQ_EINVAL;
  if (p->U > EQ_MAX_U) return EQ_ENOTSUP;
  if (!p->cluster_off) return EQ_EINVAL;
  if (p->cluster_off[0] != 0 || p->cluster_off[p->C] != p->B) return EQ_EINVAL;
  for (int c = 0; c < p->C; ++c)
    if (p->cluster_off[c + 1] <= p->cluster_off[c]) return EQ_EINVAL;
  if (!isfinite(p->n0) || !(p->n0 > 0.f)) return EQ_EINVAL;
  if (!isfinite(p->es) || !(p->es > 0.f)) return EQ_EINVAL;
  if (p->precision < EQ_FP32 || p->precision > EQ_BF16X3) return EQ_EINVAL;
  if (p->equalizer < EQ_LMMSE || p->equalizer > EQ_LMMSE_UNBIASED) return EQ_EINVAL;
  // MRC has no factor to refine; the unbiased L-MMSE gain comes from diag(A^{-1}),
  // which a refinement step does not improve
  if ((p->equalizer == EQ_MRC || p->equalizer == EQ_LMMSE_UNBIASED) && p->precision != EQ_FP32 &&
      p->precision != EQ_BF16X3)
    return EQ_ENOTSUP;
  const float rho = p->n0 / p->es;
  if (!isfinite(rho) || !(rho > 0.f)) return EQ_EINVAL;
  return EQ_OK;
}

size_t ws_bytes_for(const eq_problem *p) {
  const size_t list = (size_t)(p->W > 0 ? p->W : 1) * sizeof(int32_t);
  return kWsHeader + ((list + 255) / 256) * 256;
}

void fill_fwd(FwdArgs &a, const eq_problem *p) {
  memset(&a, 0, sizeof(a));
  a.W = p->W;
  a.B = p->B;
  a.U = p->U;
  a.C = p->C;
  a.n0 = p->n0;
  a.es = p->es;
  // ZF is the L-MMSE solve with rho = 0; MRC stores G without a shift; the
  // unbiased L-MMSE divides the L-MMSE outputs by their gain
  const bool lmmse = p->equalizer == EQ_LMMSE || p->equalizer == EQ_LMMSE_UNBIASED;
  a.rho = lmmse ? p->n0 / p->es : 0.f;
  a.ub = p->equalizer == EQ_LMMSE_UNBIASED ? 1.0f / p->es : 0.f;
  a.eqz = p->equalizer;
  for (int c = 0; c <= p->C; ++c) a.off[c] = (uint16_t)p->cluster_off[c];
  a.spw = fd_spw(ut_for(p->U), p->C);
  a.nsym = 1;
  a.ysw = p->B;
  a.zsw = p->U;
}

}  // namespace

namespace dbpeq {

eq_status forward_validate(const eq_problem *p, bool fd, const eq_c32 *H, const eq_c32 *y, const float *nu,
                           const eq_c32 *z, const float *s2, const int32_t *info) {
  eq_status st = check_problem(p);
  if (st != EQ_OK) return st;
  // FD fuses with weights from diag(A_c^{-1}) of the local Grams; a refinement
  // step corrects z_c but not that diagonal, which the single-BF16 Gram leaves
  // about 1e-3 off (the split-BF16 form EQ_BF16X3_REFINE is the FD form)
  if (fd && p->precision == EQ_BF16_REFINE) return EQ_ENOTSUP;
  if (p->W == 0) return EQ_OK;
  if (!H || !y || !z) return EQ_EINVAL;
  if (!aligned(H, 8) || !aligned(y, 8) || !aligned(z, 8)) return EQ_EINVAL;
  if ((s2 && !aligned(s2, 4)) || (info && !aligned(info, 4)) || (nu && !aligned(nu, 4))) return EQ_EINVAL;
  return EQ_OK;
}

size_t forward_ws_bytes(const eq_problem *p) { return ws_bytes_for(p); }

// Launches of a validated forward call with a workspace of at least
// forward_ws_bytes(p) bytes whose first kWsHeader bytes are zero.
eq_status forward_launch(const eq_problem *p, bool fd, const eq_c32 *H, const eq_c32 *y, const float *nu,
                         eq_c32 *z, float *s2, int32_t *info, void *ws, hipStream_t s) {
  if (p->W == 0) return EQ_OK;
  FwdArgs a;
  fill_fwd(a, p);
  a.H = reinterpret_cast<const float2 *>(H);
  a.y = reinterpret_cast<const float2 *>(y);
  a.nu = fd ? nu : nullptr;
  a.z = reinterpret_cast<float2 *>(z);
  a.s2 = s2;
  a.info = info;
  a.fb_count = reinterpret_cast<int32_t *>(ws);
  a.fb_done = a.fb_count + 1;
  a.fb_list = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(ws) + kWsHeader);
  hipEvent_t e0, e1;
  timer_pair(e0, e1);
  if (e0 && hipEventRecord(e0, s) != hipSuccess) return EQ_EHIP;
  if (p->equalizer == EQ_MRC) {
    const int prec = p->precision == EQ_FP32 ? PREC_FP32 : PREC_BF16X3_NR;
    if (launch_mrc(a, fd, prec, s) != hipSuccess) return EQ_EHIP;
    return e1 && hipEventRecord(e1, s) != hipSuccess ? EQ_EHIP : EQ_OK;
  }
  if (launch_forward(a, fd, p->precision, s) != hipSuccess) return EQ_EHIP;
  if (e1 && hipEventRecord(e1, s) != hipSuccess) return EQ_EHIP;
  if (launch_fp64_resolve(a, fd, s) != hipSuccess) return EQ_EHIP;
  return EQ_OK;
}

}  // namespace dbpeq

namespace {

eq_status forward(const eq_problem *p, bool fd, const eq_c32 *H, const eq_c32 *y, const float *nu,
                  eq_c32 *z, float *s2, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  eq_status st = forward_validate(p, fd, H, y, nu, z, s2, info);
  if (st != EQ_OK || p->W == 0) return st;
  if (!ws || ws_bytes < ws_bytes_for(p) || !aligned(ws, 4)) return EQ_EWORKSPACE;
  // the workspace starts zero-filled and the re-solve kernel leaves it so
  return forward_launch(p, fd, H, y, nu, z, s2, info, ws, reinterpret_cast<hipStream_t>(stream));
}

// Several receive vectors per channel matrix: Y [W][nsym][B], Z [W][nsym][U].
// Tiles of up to symbol_tile(U) vectors per launch pair (equaliser + FP64
// re-solve); every tile re-reads H.
eq_status forward_sym(const eq_problem *p, bool fd, int32_t nsym, const eq_c32 *H, const eq_c32 *Y,
                      const float *nu, eq_c32 *Z, float *s2, int32_t *info, void *ws, size_t ws_bytes,
                      void *stream) {
  eq_status st = check_problem(p);
  if (st != EQ_OK) return st;
  if (nsym < 1) return EQ_EINVAL;
  if (nsym > EQ_MAX_SYM) return EQ_ENOTSUP;
  if (p->precision != EQ_FP32 && p->precision != EQ_BF16X3) return EQ_ENOTSUP;
  if (p->W == 0) return EQ_OK;
  if (!H || !Y || !Z) return EQ_EINVAL;
  if (!aligned(H, 8) || !aligned(Y, 8) || !aligned(Z, 8)) return EQ_EINVAL;
  if ((s2 && !aligned(s2, 4)) || (info && !aligned(info, 4)) || (nu && !aligned(nu, 4))) return EQ_EINVAL;
  if (!ws || ws_bytes < ws_bytes_for(p) || !aligned(ws, 4)) return EQ_EWORKSPACE;
  FwdArgs a;
  fill_fwd(a, p);
  a.H = reinterpret_cast<const float2 *>(H);
  a.nu = fd ? nu : nullptr;
  a.s2 = s2;
  a.info = info;
  a.fb_count = reinterpret_cast<int32_t *>(ws);
  a.fb_done = a.fb_count + 1;
  a.fb_list = reinterpret_cast<int32_t *>(reinterpret_cast<char *>(ws) + kWsHeader);
  a.ysw = (int64_t)nsym * p->B;
  a.zsw = (int64_t)nsym * p->U;
  const int tile = symbol_tile(p->U);
  const int prec = p->precision == EQ_FP32 ? PREC_FP32 : PREC_BF16X3_NR;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int s0 = 0; s0 < nsym; s0 += tile) {
    a.nsym = nsym - s0 < tile ? nsym - s0 : tile;
    a.y = reinterpret_cast<const float2 *>(Y) + (size_t)s0 * p->B;
    a.z = reinterpret_cast<float2 *>(Z) + (size_t)s0 * p->U;
    if (launch_symbols(a, fd, prec, s) != hipSuccess) return EQ_EHIP;
    if (launch_fp64_resolve(a, fd, s) != hipSuccess) return EQ_EHIP;
  }
  return EQ_OK;
}

eq_status forward_lama(const eq_problem *p, bool fd, int32_t t_max, int32_t qam_order, const eq_c32 *H,
                       const eq_c32 *y, const float *nu, eq_c32 *z, float *s2, int32_t *info, void *stream) {
  if (!p) return EQ_EINVAL;
  eq_problem q = *p;
  q.equalizer = EQ_LMMSE;  // not used by LAMA
  eq_status st = check_problem(&q);
  if (st != EQ_OK) return st;
  if (t_max < 1 || t_max > EQ_MAX_LAMA_ITER) return EQ_EINVAL;
  if (qam_order != 4 && qam_order != 16 && qam_order != 64) return EQ_EINVAL;
  if (p->precision != EQ_FP32 && p->precision != EQ_BF16X3) return EQ_ENOTSUP;
  if (p->W == 0) return EQ_OK;
  if (!H || !y || !z) return EQ_EINVAL;
  if (!aligned(H, 8) || !aligned(y, 8) || !aligned(z, 8)) return EQ_EINVAL;
  if ((s2 && !aligned(s2, 4)) || (info && !aligned(info, 4)) || (nu && !aligned(nu, 4))) return EQ_EINVAL;
  FwdArgs a;
  fill_fwd(a, &q);
  a.rho = 0.f;
  a.H = reinterpret_cast<const float2 *>(H);
  a.y = reinterpret_cast<const float2 *>(y);
  a.nu = fd ? nu : nullptr;
  a.z = reinterpret_cast<float2 *>(z);
  a.s2 = s2;
  a.info = info;
  a.lama_t = t_max;
  a.lama_m = qam_order == 4 ? 2 : (qam_order == 16 ? 4 : 8);
  const int prec = p->precision == EQ_FP32 ? PREC_FP32 : PREC_BF16X3_NR;
  return launch_lama(a, fd, prec, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? EQ_OK : EQ_EHIP;
}

// LAMA over several receive vectors: Y [W][nsym][B], Z and sigma2
// [W][nsym][U]; tiles of up to symbol_tile(U) vectors, each reading H once.
eq_status forward_lama_sym(const eq_problem *p, bool fd, int32_t nsym, int32_t t_max, int32_t qam_order,
                           const eq_c32 *H, const eq_c32 *Y, const float *nu, eq_c32 *Z, float *s2, int32_t *info,
                           void *stream) {
  if (!p) return EQ_EINVAL;
  eq_problem q = *p;
  q.equalizer = EQ_LMMSE;  // not used by LAMA
  eq_status st = check_problem(&q);
  if (st != EQ_OK) return st;
  if (nsym < 1) return EQ_EINVAL;
  if (nsym > EQ_MAX_SYM) return EQ_ENOTSUP;
  if (t_max < 1 || t_max > EQ_MAX_LAMA_ITER) return EQ_EINVAL;
  if (qam_order != 4 && qam_order != 16 && qam_order != 64) return EQ_EINVAL;
  if (p->precision != EQ_FP32 && p->precision != EQ_BF16X3) return EQ_ENOTSUP;
  if (p->W == 0) return EQ_OK;
  if (!H || !Y || !Z) return EQ_EINVAL;
  if (!aligned(H, 8) || !aligned(Y, 8) || !aligned(Z, 8)) return EQ_EINVAL;
  if ((s2 && !aligned(s2, 4)) || (info && !aligned(info, 4)) || (nu && !aligned(nu, 4))) return EQ_EINVAL;
  FwdArgs a;
  fill_fwd(a, &q);
  a.rho = 0.f;
  a.H = reinterpret_cast<const float2 *>(H);
  a.nu = fd ? nu : nullptr;
  a.info = info;
  a.lama_t = t_max;
  a.lama_m = qam_order == 4 ? 2 : (qam_order == 16 ? 4 : 8);
  a.ysw = (int64_t)nsym * p->B;
  a.zsw = (int64_t)nsym * p->U;
  const int tile = symbol_tile(p->U);
  const int prec = p->precision == EQ_FP32 ? PREC_FP32 : PREC_BF16X3_NR;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  for (int s0 = 0; s0 < nsym; s0 += tile) {
    a.nsym = nsym - s0 < tile ? nsym - s0 : tile;
    a.y = reinterpret_cast<const float2 *>(Y) + (size_t)s0 * p->B;
    a.z = reinterpret_cast<float2 *>(Z) + (size_t)s0 * p->U;
    a.s2 = s2 ? s2 + (size_t)s0 * p->U : nullptr;
    if (launch_symbols_lama(a, fd, prec, s) != hipSuccess) return EQ_EHIP;
  }
  return EQ_OK;
}

size_t bwd_ws_bytes(const eq_problem *p) {
  int spw;
  const int nt = backward_tasks(p->W > 0 ? p->W : 1, p->U, p->C, true, &spw);
  const int nt_pd = backward_tasks(p->W > 0 ? p->W : 1, p->U, p->C, false, &spw);
  const size_t parts = (size_t)(((nt > nt_pd ? nt : nt_pd) + 63) / 64) * 64 * sizeof(float);
  const size_t fwd = (size_t)(p->W > 0 ? p->W : 1) * p->C * p->U * 16;
  return parts + fwd;
}

eq_status backward(const eq_problem *p, bool fd, const eq_c32 *H, const eq_c32 *y, const float *nu,
                   const eq_c32 *gz, const float *gs, eq_c32 *gH, eq_c32 *gy, float *gn0, float *gnu,
                   void *ws, size_t ws_bytes, void *stream) {
  eq_status st = check_problem(p);
  if (st != EQ_OK) return st;
  if (p->equalizer != EQ_LMMSE) return EQ_ENOTSUP;
  if (!fd && (nu || gnu)) return EQ_EINVAL;
  if (fd && gnu && !nu) return EQ_EINVAL;
  if (p->W == 0) return EQ_OK;
  if (!H || !y) return EQ_EINVAL;
  if (!aligned(H, 8) || !aligned(y, 8) || (gz && !aligned(gz, 8)) || (gH && !aligned(gH, 8)) ||
      (gy && !aligned(gy, 8)))
    return EQ_EINVAL;
  if ((gs && !aligned(gs, 4)) || (gn0 && !aligned(gn0, 4)) || (nu && !aligned(nu, 4)) ||
      (gnu && !aligned(gnu, 4)))
    return EQ_EINVAL;
  if (!ws || ws_bytes < bwd_ws_bytes(p) || !aligned(ws, 256)) return EQ_EWORKSPACE;
  BwdArgs a;
  memset(&a, 0, sizeof(a));
  a.W = p->W;
  a.B = p->B;
  a.U = p->U;
  a.C = p->C;
  a.n0 = p->n0;
  a.es = p->es;
  a.rho = p->n0 / p->es;
  for (int c = 0; c <= p->C; ++c) a.off[c] = (uint16_t)p->cluster_off[c];
  const int ntasks = backward_tasks(p->W, p->U, p->C, fd, &a.spw);
  a.H = reinterpret_cast<const float2 *>(H);
  a.y = reinterpret_cast<const float2 *>(y);
  a.nu = nu;
  a.gz = reinterpret_cast<const float2 *>(gz);
  a.gs = gs;
  a.gH = reinterpret_cast<float2 *>(gH);
  a.gy = reinterpret_cast<float2 *>(gy);
  a.gnu = gnu;
  a.gn0_part = reinterpret_cast<float *>(ws);
  a.gn0 = gn0;
  if (launch_backward(a, fd, ntasks, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return EQ_EHIP;
  return EQ_OK;
}

}  // namespace

extern "C" {

size_t eq_backward_workspace_size(const eq_problem *p) {
  if (check_problem(p) != EQ_OK || p->equalizer != EQ_LMMSE) return 0;
  return bwd_ws_bytes(p);
}

eq_status eq_pd_backward(const eq_problem *p, const eq_c32 *H, const eq_c32 *y, const eq_c32 *gz,
                         const float *gs, eq_c32 *gH, eq_c32 *gy, float *gn0, void *ws, size_t ws_bytes,
                         void *stream) {
  return backward(p, false, H, y, nullptr, gz, gs, gH, gy, gn0, nullptr, ws, ws_bytes, stream);
}

eq_status eq_fd_backward(const eq_problem *p, const eq_c32 *H, const eq_c32 *y, const float *nu,
                         const eq_c32 *gz, const float *gs, eq_c32 *gH, eq_c32 *gy, float *gn0,
                         float *gnu, void *ws, size_t ws_bytes, void *stream) {
  return backward(p, true, H, y, nu, gz, gs, gH, gy, gn0, gnu, ws, ws_bytes, stream);
}


int32_t eq_abi_version(void) { return EQ_ABI_VERSION; }

eq_status eq_probe_read(const void *buf, size_t bytes, float *sink, void *stream) {
  if (bytes == 0) return EQ_OK;
  if (!buf || !sink || !aligned(buf, 16) || !aligned(sink, 4) || bytes % 16 != 0) return EQ_EINVAL;
  if (launch_probe_read(buf, bytes, sink, reinterpret_cast<hipStream_t>(stream)) != hipSuccess) return EQ_EHIP;
  return EQ_OK;
}

eq_status eq_kernel_timer_start(int32_t capacity) {
  if (capacity < 1 || capacity > EQ_KERNEL_TIMER_MAX) return EQ_EINVAL;
  KernelTimer &t = kernel_timer();
  std::lock_guard<std::mutex> g(t.mu);
  if (t.on) return EQ_EINVAL;
  t.ev.assign(2 * (size_t)capacity, nullptr);
  for (hipEvent_t &e : t.ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      for (hipEvent_t x : t.ev)
        if (x) (void)hipEventDestroy(x);
      t.ev.clear();
      return EQ_EHIP;
    }
  }
  t.used = 0;
  t.on = true;
  return EQ_OK;
}

eq_status eq_kernel_timer_stop(int32_t *count, double *total_ms) {
  KernelTimer &t = kernel_timer();
  std::lock_guard<std::mutex> g(t.mu);
  if (!t.on) return EQ_EINVAL;
  t.on = false;
  double sum = 0.0;
  bool ok = true;
  for (size_t k = 0; k < t.used && ok; ++k) {
    float ms = 0.f;
    ok = hipEventSynchronize(t.ev[2 * k + 1]) == hipSuccess &&
         hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess;
    sum += ms;
  }
  for (hipEvent_t e : t.ev)
    if (e) ok &= hipEventDestroy(e) == hipSuccess;
  if (count) *count = (int32_t)t.used;
  if (total_ms) *total_ms = sum;
  t.ev.clear();
  t.used = 0;
  return ok ? EQ_OK : EQ_EHIP;
}

const char *eq_status_string(eq_status s) {
  switch (s) {
    case EQ_OK: return "ok";
    case EQ_EINVAL: return "invalid argument";
    case EQ_ENOTSUP: return "unsupported problem size";
    case EQ_EHIP: return "HIP runtime error";
    case EQ_EWORKSPACE: return "workspace missing or too small";
    case EQ_ENOMEM: return "device allocation failed";
  }
  return "unknown status";
}

size_t eq_workspace_size(const eq_problem *p) {
  if (check_problem(p) != EQ_OK) return 0;
  return ws_bytes_for(p);
}

eq_status eq_pd(const eq_problem *p, const eq_c32 *H, const eq_c32 *y, eq_c32 *z, float *sigma2,
                int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  return forward(p, false, H, y, nullptr, z, sigma2, info, ws, ws_bytes, stream);
}

eq_status eq_fd(const eq_problem *p, const eq_c32 *H, const eq_c32 *y, const float *nu, eq_c32 *z,
                float *sigma2, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  return forward(p, true, H, y, nu, z, sigma2, info, ws, ws_bytes, stream);
}

eq_status eq_pd_lama(const eq_problem *p, int32_t t_max, int32_t qam_order, const eq_c32 *H, const eq_c32 *y,
                     eq_c32 *z, float *sigma2, int32_t *info, void *stream) {
  if (!p) return EQ_EINVAL;
  return forward_lama(p, false, t_max, qam_order, H, y, nullptr, z, sigma2, info, stream);
}

eq_status eq_fd_lama(const eq_problem *p, int32_t t_max, int32_t qam_order, const eq_c32 *H, const eq_c32 *y,
                     const float *nu, eq_c32 *z, float *sigma2, int32_t *info, void *stream) {
  if (!p) return EQ_EINVAL;
  return forward_lama(p, true, t_max, qam_order, H, y, nu, z, sigma2, info, stream);
}

eq_status eq_pd_lama_sym(const eq_problem *p, int32_t nsym, int32_t t_max, int32_t qam_order, const eq_c32 *H,
                         const eq_c32 *Y, eq_c32 *Z, float *sigma2, int32_t *info, void *stream) {
  return forward_lama_sym(p, false, nsym, t_max, qam_order, H, Y, nullptr, Z, sigma2, info, stream);
}

eq_status eq_fd_lama_sym(const eq_problem *p, int32_t nsym, int32_t t_max, int32_t qam_order, const eq_c32 *H,
                         const eq_c32 *Y, const float *nu, eq_c32 *Z, float *sigma2, int32_t *info,
                         void *stream) {
  return forward_lama_sym(p, true, nsym, t_max, qam_order, H, Y, nu, Z, sigma2, info, stream);
}

eq_status eq_pd_sym(const eq_problem *p, int32_t nsym, const eq_c32 *H, const eq_c32 *Y, eq_c32 *Z,
                    float *sigma2, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  return forward_sym(p, false, nsym, H, Y, nullptr, Z, sigma2, info, ws, ws_bytes, stream);
}

eq_status eq_fd_sym(const eq_problem *p, int32_t nsym, const eq_c32 *H, const eq_c32 *Y, const float *nu,
                    eq_c32 *Z, float *sigma2, int32_t *info, void *ws, size_t ws_bytes, void *stream) {
  return forward_sym(p, true, nsym, H, Y, nu, Z, sigma2, info, ws, ws_bytes, stream);
}

}  // extern "C"
