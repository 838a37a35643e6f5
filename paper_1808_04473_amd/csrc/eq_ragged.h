// Ragged batches: thousands of independent systems of uneven (B, U, C), in
// one persistent launch driven by a device-side descriptor table.
#pragma once
#include "eq_common.h"

namespace dbpeq {

// One system of a ragged batch (device copy of eq_sys, plus derived fields).
struct RSys {
  int64_t h_off, y_off, z_off;
  int32_t B, U, C, off_first;  // off_first: index of its first cluster offset in offs[]
  float n0, rho;
  int32_t ut;       // padded user count (16 or 32)
  int32_t npieces;  // PD: row pieces (1 = the system is solved whole, inside a group item)
  int32_t slot0;    // PD: partial slot of its first piece
  int32_t cl0;      // FD: global index of its first cluster (clusters are numbered system by system)
};

// Work items.  A wave takes one item at a time from the queue.
enum : int32_t {
  kItemGroup = 0,  // PD: `count` whole systems of equal U, order[first ..]
  kItemPiece = 1,  // PD: rows [r0, r1) of system `first`, piece `piece` of its npieces
  kItemRound = 2,  // FD: `count` clusters of equal U (of any systems), global cluster indices order[first ..]
};

struct RTask {
  int32_t kind, ut, U, first;
  int32_t count, r0, r1, piece;
};

// The items are dealt round-robin to kQueues queues (item t to queue
// t % kQueues); workgroup b drains queue b % kQueues.  One queue head per
// 128-byte line: a single head serialises every fetch of the launch on one
// address.
constexpr int kQueues = 8;
constexpr int kQueueStride = 32;

// Floats per PD partial slot: the three accumulator arrays and the matched
// filter, per lane, for the widest tile (UT = 32: 16 accumulator registers).
constexpr int kPartRegs = 3 * 16 + 2;
constexpr int kPartStride = kPartRegs * 64;
// FD fusion terms per cluster: (1/sigma2, z.re/sigma2, z.im/sigma2, -) for up
// to 32 users.
constexpr int kFusionStride = 32;

struct RaggedArgs {
  const float2 *Hpool;
  const float2 *ypool;
  float2 *zpool;
  float *s2pool;
  int32_t *info;        // [nsys] or nullptr
  const RSys *sys;
  const int32_t *offs;  // cluster row offsets, C+1 per system
  const RTask *tasks;
  const int32_t *order;   // systems of group items, then clusters of round items
  const int32_t *cl_sys;  // system of each global cluster (FD)
  // An execution leaves these at zero for the next one: each system's
  // finisher resets its arrival counter, and the FP64 launch that follows the
  // persistent one clears the queue heads and then its own queue.
  int32_t *counter;       // work-queue heads, kQueueStride apart
  int32_t *fb_count;      // FP64 re-solve queue
  int32_t *fb_done;       // FP64 blocks done
  int32_t *fb_list;
  int32_t *arrive;        // per system: pieces (PD) or clusters (FD) finished
  float *part;            // PD partial accumulators, kPartStride floats per slot
  float *fpart;           // FD fusion terms, kFusionStride x 4 floats per cluster
  int32_t *fcode;         // FD per cluster: failure code, routed to FP64
  int32_t nsys, ntasks;
  float es;
};

hipError_t launch_ragged(const RaggedArgs &a, bool fd, int prec, int grid, hipStream_t s);
hipError_t launch_fp64_ragged(const RaggedArgs &a, bool fd, hipStream_t s);

}  // namespace dbpeq
