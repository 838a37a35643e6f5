// Ragged batches: thousands of independent systems of uneven (B, U, C) in one
// persistent launch driven by a device-side descriptor table.
#pragma once
#include "eq_common.h"

namespace dbpeq {

// One system of a ragged batch (device copy of eq_sys, plus derived fields).
struct RSys {
  int64_t h_off, y_off, z_off;
  int32_t B, U, C, off_first;  // off_first: index of its first cluster offset in offs[]
  float n0, rho;
  int32_t ut, pad;
};

// A work item: `count` systems order[first .. first+count-1] of one U (PD),
// or one system (FD).
struct RTask {
  int32_t first, count, ut, U;
};

struct RaggedArgs {
  const float2 *Hpool;
  const float2 *ypool;
  float2 *zpool;
  float *s2pool;
  int32_t *info;        // [nsys] or nullptr
  const RSys *sys;
  const int32_t *offs;  // cluster row offsets, C+1 per system
  const RTask *tasks;
  const int32_t *order;
  int32_t *counter;     // work-queue head (reset before every launch)
  int32_t *fb_count;    // FP64 re-solve queue
  int32_t *fb_list;
  int32_t nsys, ntasks;
  float es;
};

hipError_t launch_ragged(const RaggedArgs &a, bool fd, int prec, int grid, hipStream_t s);
hipError_t launch_fp64_ragged(const RaggedArgs &a, bool fd, hipStream_t s);

}  // namespace dbpeq
