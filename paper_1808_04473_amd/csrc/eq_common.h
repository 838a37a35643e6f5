// Internal definitions shared by the host launcher code and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dbpeq.h"

namespace dbpeq {

enum Prec { PREC_FP32 = 0, PREC_BF16 = 1, PREC_BF16X3 = 2, PREC_BF16X3_NR = 3 };

// Equaliser of the forward calls (the eq_equalizer values).
enum Eqz { EQZ_LMMSE = 0, EQZ_ZF = 1, EQZ_MRC = 2, EQZ_LMMSE_UB = 3 };

// Forms that run the refinement step with the FP32 residual y - H z.
constexpr bool refines(int prec) { return prec == PREC_BF16 || prec == PREC_BF16X3; }

// Forward launch arguments (passed by value; the cluster table lives in the
// kernel-argument segment, so no device-side copy of the host partition is
// needed and the launch can be captured into a graph).
struct FwdArgs {
  const float2 *H;
  const float2 *y;
  const float *nu;      // [W][C][U] or nullptr (optimal weights)
  float2 *z;
  float *s2;            // may be nullptr
  int32_t *info;        // may be nullptr
  int32_t *fb_count;    // FP64 re-solve queue (workspace): length,
  int32_t *fb_done;     // blocks of the re-solve kernel that finished,
  int32_t *fb_list;     // queued systems
  int32_t W, B, U, C;
  float n0, rho, es;
  float ub;             // 1/E_s for the unbiased L-MMSE, else 0: the outputs are
                        // divided by the gain 1 - sigma2 * ub (exactly 1 at ub = 0)
  int32_t spw;          // FD: subcarriers per wave
  // receive vectors: nsym per channel matrix in this launch (1 for the
  // single-vector entry points), y + w*ysw is the first of subcarrier w,
  // z + w*zsw its first estimate; vectors of one subcarrier are B (y) and
  // U (z) elements apart
  int32_t nsym;
  int64_t ysw, zsw;
  int32_t eqz;          // Eqz; ZF runs the L-MMSE kernels with rho = 0
  int32_t lama_t;       // LAMA: iterations T_max
  int32_t lama_m;       // LAMA: levels per coordinate of the square QAM (2, 4, 8)
  uint16_t off[EQ_MAX_C + 1];
};

// Backward launch arguments.
struct BwdArgs {
  const float2 *H;
  const float2 *y;
  const float *nu;
  const float2 *gz;     // may be nullptr
  const float *gs;      // may be nullptr
  float2 *gH;           // may be nullptr
  float2 *gy;           // may be nullptr
  float *gnu;           // may be nullptr
  float *gn0_part;      // [tasks] partial sums (workspace)
  float *gn0;           // final scalar (may be nullptr)
  int32_t W, B, U, C;
  float n0, rho, es;
  int32_t spw;
  uint16_t off[EQ_MAX_C + 1];
};

// Host launchers (defined in the .hip files).
hipError_t launch_forward(const FwdArgs &a, bool fd, int prec, hipStream_t s);
hipError_t launch_fp64_resolve(const FwdArgs &a, bool fd, hipStream_t s);
hipError_t launch_zero_i32(int32_t *p, int n, hipStream_t s);
hipError_t launch_probe_read(const void *buf, size_t bytes, float *sink, hipStream_t s);
// several receive vectors per channel matrix: a.nsym <= symbol_tile(a.U)
hipError_t launch_symbols(const FwdArgs &a, bool fd, int prec, hipStream_t s);
int symbol_tile(int U);
// MRC (no factorisation): FP32 or split-BF16 Gram
hipError_t launch_mrc(const FwdArgs &a, bool fd, int prec, hipStream_t s);
// LAMA (Algorithm 1): FP32 or split-BF16 Gram; one receive vector, or a tile
// of a.nsym <= symbol_tile(a.U) vectors per channel matrix
hipError_t launch_lama(const FwdArgs &a, bool fd, int prec, hipStream_t s);
hipError_t launch_symbols_lama(const FwdArgs &a, bool fd, int prec, hipStream_t s);

hipError_t launch_backward(const BwdArgs &a, bool fd, int ntasks, hipStream_t s);

// Forward calls (eq_abi.cpp), split for the entry point with a library-owned
// workspace: argument checks (no HIP call), workspace bytes, and the launches
// (the workspace's first 256 bytes must be zero).
eq_status forward_validate(const eq_problem *p, bool fd, const eq_c32 *H, const eq_c32 *y, const float *nu,
                           const eq_c32 *z, const float *s2, const int32_t *info);
size_t forward_ws_bytes(const eq_problem *p);
eq_status forward_launch(const eq_problem *p, bool fd, const eq_c32 *H, const eq_c32 *y, const float *nu,
                         eq_c32 *z, float *s2, int32_t *info, void *ws, hipStream_t s);
int backward_tasks(int W, int U, int C, bool fd, int *spw);

inline int ut_for(int U) { return U <= 16 ? 16 : 32; }
inline int fd_spw(int UT, int C) {
  const int nsys = 64 / UT;
  return C >= nsys ? 1 : nsys / C;
}

}  // namespace dbpeq
