// Device building blocks of the equaliser kernels (gfx950, wave64).
//
// Work decomposition.  A wave owns a "round" of NSYS = 64/UT small systems
// (UT = 16 or 32 is the padded user count).  Two layouts are used:
//
//  * streaming layout (Gram + matched filter): lane l covers column
//    col = l % UT of H and row offset g = l / UT.  One load step reads
//    RPS = 64/UT consecutive rows of H (RPS*U*8 contiguous bytes) with one
//    8-byte load per lane.  The loaded value is at the same time the A and B
//    operand of an MFMA whose K index runs over rows, so H_c^H H_c needs no
//    LDS staging: FP32 MFMA consumes one load step per instruction
//    (16x16x4 / 32x32x2), BF16 MFMA eight (16x16x32 / 32x32x16).
//
//  * solve layout: lane l works on system s = l / UT, row / column
//    i = l % UT.  The Cholesky factor is held by rows (lane i owns row i of
//    L), the inverse factor X = L^{-1} by columns (lane u owns column u), so
//    diag(A^{-1})_u = sum_j |X_ju|^2 and z = X^H (L^{-1} m) need no
//    cross-lane reduction.  Values move between lanes of a group by
//    broadcasting one lane: a DPP row broadcast, after a v_permlane16_swap
//    for 32-lane groups, fused into the FMAC that consumes it.
#pragma once
#include <utility>

#include "eq_common.h"

namespace dbpeq {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

// ---------------------------------------------------------------- compile-time loops
template <int... Is, class F>
__device__ __forceinline__ void sfor_impl(std::integer_sequence<int, Is...>, F &&f) {
  (f(std::integral_constant<int, Is>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void sfor(F &&f) {
  sfor_impl(std::make_integer_sequence<int, N>{}, f);
}

// Lane index within the wave.  Opaque to the optimiser: otherwise every
// lane-dependent value (masks, offsets, selects) is computed once and kept
// live across the whole kernel, which costs tens of registers; recomputing
// it is one VALU instruction.
__device__ __forceinline__ int lane_id() {
  int l = threadIdx.x & 63;
  asm volatile("" : "+v"(l));
  return l;
}

// ---------------------------------------------------------------- cross-lane primitives
// DPP controls (GCN/CDNA data-parallel primitives).
constexpr int DPP_QUAD_XOR1 = 0xB1;      // quad_perm [1,0,3,2]
constexpr int DPP_QUAD_XOR2 = 0x4E;      // quad_perm [2,3,0,1]
constexpr int DPP_ROW_MIRROR = 0x140;    // lane i <-> 15 - i inside a row of 16
constexpr int DPP_ROW_HMIRROR = 0x141;   // lane i <-> 7 - i inside half rows
constexpr int DPP_ROW_NEWBCAST = 0x150;  // + k: lane k of each row to the whole row

// Every control used here reads a valid lane, so the bound_ctrl / old value
// never matter; this form lets the compiler fold the DPP into the add (or
// other VOP2 instruction) that consumes it.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

// Broadcast source of a value v for groups of UT lanes.  A group of 16 lanes
// is one DPP row, so lane K of it is DPP row_newbcast:K of v itself.  A group
// of 32 lanes spans two rows: v_permlane16_swap(v, v) yields `lo`, in which
// the group's first row fills both of its rows, and `hi`, with the second
// row; lane K of the group is then row_newbcast:(K % 16) of lo (K < 16) or
// hi.  One swap serves every K, so a step that broadcasts the same register
// from many lanes pays for it once.
struct BSrc {
  float lo, hi;
};
template <int UT>
__device__ __forceinline__ BSrc bsrc(float v) {
  if constexpr (UT == 16) {
    return {v, v};
  } else {
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return {__uint_as_float(r[0]), __uint_as_float(r[1])};
  }
}
template <int K>
__device__ __forceinline__ float bpick(const BSrc &b) {
  return K < 16 ? b.lo : b.hi;
}

// Value of lane K of this lane's group of UT lanes.
template <int UT, int K>
__device__ __forceinline__ float gbcast(float v) {
  return dpp<DPP_ROW_NEWBCAST + K % 16>(bpick<K>(bsrc<UT>(v)));
}
template <int UT, int K>
__device__ __forceinline__ float2 gbcast2(float2 v) {
  return make_float2(gbcast<UT, K>(v.x), gbcast<UT, K>(v.y));
}

// acc += (NEG ? -1 : 1) * src[lane K of this lane's DPP row] * b: one VOP2
// FMAC whose src0 comes through a DPP row broadcast (src is a BSrc half, so
// that K = group lane % 16).  Written as inline assembly because the
// compiler folds DPP movs into adds but not into FMACs.  The hardware needs
// two wait states between a VALU write of the DPP source and the read (five
// after a VALU write of EXEC); the compiler does not see the DPP operand of
// inline assembly, so NOP = 4 puts an s_nop 4 at the head of each group of
// these instructions, whose sources are written before the group and not
// inside it.  The build checks the generated assembly for these hazards.
#define EQ_FMAC_ROWBCAST(PRE, NEGS)                                                          \
  asm volatile(PRE "v_fmac_f32_dpp %0, " NEGS "%1, %2 row_newbcast:%3 row_mask:0xf bank_mask:0xf" \
               : "+v"(acc)                                                                     \
               : "v"(src), "v"(b), "n"(K))
template <int K, bool NEG, int NOP>
__device__ __forceinline__ void fmac_rowbcast(float &acc, float src, float b) {
  static_assert(NOP == 0 || NOP == 4, "wait states");
  if constexpr (NEG && NOP == 4) EQ_FMAC_ROWBCAST("s_nop 4\n\t", "-");
  else if constexpr (NEG) EQ_FMAC_ROWBCAST("", "-");
  else if constexpr (NOP == 4) EQ_FMAC_ROWBCAST("s_nop 4\n\t", "");
  else EQ_FMAC_ROWBCAST("", "");
}
#undef EQ_FMAC_ROWBCAST

// Sum over the 16 lanes of a DPP row; every lane receives the sum.
__device__ __forceinline__ float row16_sum(float v) {
  v += dpp<DPP_QUAD_XOR1>(v);
  v += dpp<DPP_QUAD_XOR2>(v);
  v += dpp<DPP_ROW_HMIRROR>(v);
  v += dpp<DPP_ROW_MIRROR>(v);
  return v;
}

// Sum / max / any over an aligned group of UT lanes; all lanes get the result.
template <int UT>
__device__ __forceinline__ float gsum(float v) {
  v = row16_sum(v);
  if constexpr (UT == 32) {
    // the two row sums of the 32-lane group, each replicated over the group
    const BSrc r = bsrc<32>(v);
    v = r.lo + r.hi;
  }
  return v;
}
template <int UT>
__device__ __forceinline__ float gmax(float v) {
  v = fmaxf(v, __shfl_xor(v, 1));
  v = fmaxf(v, __shfl_xor(v, 2));
  v = fmaxf(v, __shfl_xor(v, 4));
  v = fmaxf(v, __shfl_xor(v, 8));
  if constexpr (UT == 32) v = fmaxf(v, __shfl_xor(v, 16));
  return v;
}
template <int UT>
__device__ __forceinline__ bool gany(bool p) {
  const unsigned long long m = __ballot(p);
  const int s = lane_id() / UT;
  const unsigned long long gm = (UT == 64) ? ~0ull : ((1ull << UT) - 1ull) << (s * UT);
  return (m & gm) != 0ull;
}

// Sum over the 64/UT lanes that share a column in the streaming layout.
template <int UT>
__device__ __forceinline__ float colsum(float v) {
  if constexpr (UT == 16) v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// ---------------------------------------------------------------- MFMA wrappers
template <int UT> struct Acc;
template <> struct Acc<16> { f4 rr, ri, ii; };
template <> struct Acc<32> { f16v rr, ri, ii; };

__device__ __forceinline__ f4 mma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f16v mma32(float a, float b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mma16(bf8 a, bf8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f16v mma16(bf8 a, bf8 b, f16v c) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

// Position (i, j) of accumulator register r in lane l.
template <int UT>
__device__ __forceinline__ void acc_pos(int l, int r, int &i, int &j) {
  if constexpr (UT == 16) {
    i = 4 * (l >> 4) + r;
    j = l & 15;
  } else {
    i = 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    j = l & 31;
  }
}

template <int UT>
__device__ __forceinline__ void acc_zero(Acc<UT> &a) {
  constexpr int NR = UT == 16 ? 4 : 16;
#pragma unroll
  for (int r = 0; r < NR; ++r) { a.rr[r] = 0.f; a.ri[r] = 0.f; a.ii[r] = 0.f; }
}

// ---------------------------------------------------------------- row-block streaming
// One block = 8 load steps = 8 * (64/UT) rows of one system, in the
// streaming layout: lane l holds H[rb + e*RPS + g][col] (col = l % UT,
// g = l / UT, e = 0..7).  y is loaded once per row (lane j < RPB holds
// y[rb + j]) and handed to the lanes of a row by a lane shuffle: a per-lane
// copy would cost eight vector-memory instructions for 256 bytes.
struct Blk8 {
  float2 h[8];
};

struct Slot {
  float2 h[8];
  float2 yl;
  const float2 *Hw;
  const float2 *yw;
  int s, rb, r1;  // s: system index within its task
  int tk;         // task the system belongs to
  int g;          // row group of this lane (lane / UT)
  bool last;
};

// One system of a stream: rows [r0, r1) of Hw / yw, identified by (tk, s).
struct SysRef {
  const float2 *Hw;
  const float2 *yw;
  int r0, r1, tk, s;
};

// Loads go through buffer resources that cover exactly the system's rows
// [r0, r1): the hardware returns zero for any offset outside the range, so
// rows past r1 and padded columns (col >= U, given an offset that is always
// out of range) need neither clamping nor masking, and the address of each
// load is one integer add.  No load sits behind a divergent branch, so the
// compiler can wait for one block while the next blocks are in flight.
constexpr int kBufFlags = 0x00020000;  // raw 32-bit buffer, gfx9 format bits
constexpr unsigned kOutOfRange = 0x80000000u;

// Cache policy of a stream's loads: the last read of these bytes uses the
// nontemporal policy (they are not kept in L2 / Infinity Cache); a read that
// a later pass of the same wave repeats uses the default policy.
constexpr int kLoadKeep = 0;
constexpr int kLoadLast = 2;  // NT

template <int AUX>
__device__ __forceinline__ float2 buf_ld2(__amdgpu_buffer_rsrc_t r, unsigned off) {
  typedef float f2v __attribute__((ext_vector_type(2)));
  const f2v v = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, AUX));
  return make_float2(v.x, v.y);
}

// Row of load step e of group g (lane / UT) within a row block: each group
// holds 8 consecutive rows, so that y of those rows sits in the group's own
// DPP row (lanes 0..7 of it) and reaches the other lanes by row broadcast.
__device__ __forceinline__ int slot_row(int e, int g) { return 8 * g + e; }

// Per-lane byte offsets of the streaming layout (constant over a stream).
template <int UT>
struct LaneOff {
  unsigned h;  // (8 g U + col) * 8, or out of range for padded columns
  unsigned y;  // (8 g + c) * 8 for lanes c = lane % 16 < 8, else out of range
  int g;       // row group lane / UT
};

template <int UT>
__device__ __forceinline__ LaneOff<UT> lane_offsets(int U) {
  const int lane = lane_id();
  const int col = lane % UT, g = lane / UT, c = lane % 16;
  LaneOff<UT> o;
  o.h = col < U ? (unsigned)((slot_row(0, g) * U + col) * 8) : kOutOfRange;
  o.y = c < 8 ? (unsigned)(slot_row(c, g) * 8) : kOutOfRange;
  o.g = g;
  return o;
}

// Loads the row block at rb of rows [r0, r1).  live = false gives the
// descriptors zero length: every load is then out of range and returns zero
// without a memory access (the same instructions, no traffic).
template <int UT, int AUX>
__device__ __forceinline__ void load_slot(Slot &b, const LaneOff<UT> &lo, const float2 *__restrict__ Hw,
                                          const float2 *__restrict__ yw, int U, int rb, int r0,
                                          int r1, bool live) {
  const int nrow = live ? r1 - r0 : 0;
  const __amdgpu_buffer_rsrc_t rh =
      __builtin_amdgcn_make_buffer_rsrc((void *)(Hw + (size_t)r0 * U), (short)0, nrow * U * 8, kBufFlags);
  const __amdgpu_buffer_rsrc_t ry =
      __builtin_amdgcn_make_buffer_rsrc((void *)(yw + r0), (short)0, nrow * 8, kBufFlags);
  const unsigned rowb = (unsigned)((rb - r0) * U * 8);
  const unsigned step = (unsigned)(U * 8);
#pragma unroll
  for (int e = 0; e < 8; ++e) b.h[e] = buf_ld2<AUX>(rh, lo.h + rowb + e * step);
  b.yl = buf_ld2<AUX>(ry, lo.y + (unsigned)((rb - r0) * 8));
  b.g = lo.g;
  b.Hw = Hw;
  b.yw = yw;
  b.rb = rb;
  b.r1 = r1;
}

// H[rb + slot_row(e, g)][col] of this lane (zero outside the system).
template <int UT>
__device__ __forceinline__ float2 slot_h(const Slot &b, int e, int) {
  return b.h[e];
}

// y[rb + slot_row(E, g)] of this lane's row in load step E (zero past the
// end): lane E of the DPP row holds it.
template <int UT, int E>
__device__ __forceinline__ float2 slot_y(const Slot &b) {
  return make_float2(dpp<DPP_ROW_NEWBCAST + E>(b.yl.x), dpp<DPP_ROW_NEWBCAST + E>(b.yl.y));
}

// Three-slot ring over row blocks: issue(slot) starts the loads of the next
// block (returning false once the stream is exhausted, after issuing the
// same loads against empty descriptors), body(slot) consumes a block and
// done(slot) follows the last block of each system.  Two blocks are in
// flight while one is consumed (a fourth slot measured no faster at either
// group width, and spills in the refining forms).  sched_barrier keeps each
// block's loads where they are issued: the scheduler must not sink them into
// (or hoist the consumer above) the previous block's arithmetic.
template <class SlotT, class Issue, class Body, class Done>
__device__ __forceinline__ void stream_ring3(Issue &issue, Body &body, Done &done) {
  SlotT sa, sb, sc;
  issue(sa);
  bool vb = issue(sb);
  while (true) {
    const bool vc = issue(sc);
    __builtin_amdgcn_sched_barrier(0);
    body(sa);
    if (sa.last) done(sa);
    if (!vb) break;
    const bool va = issue(sa);
    __builtin_amdgcn_sched_barrier(0);
    body(sb);
    if (sb.last) done(sb);
    if (!vc) break;
    vb = issue(sb);
    __builtin_amdgcn_sched_barrier(0);
    body(sc);
    if (sc.last) done(sc);
    if (!va) break;
  }
}

// Streams the row blocks of a sequence of systems produced by gen (a
// functor bool(SysRef &) returning false at the end of the sequence).
template <int UT, int AUX, class Gen, class Body, class Done>
__device__ __forceinline__ void stream_gen(int U, Gen &gen, Body body, Done done) {
  constexpr int RPB = 8 * (64 / UT);
  SysRef cur;
  if (!gen(cur)) return;
  int crb = cur.r0;
  bool more = true;
  const LaneOff<UT> lo = lane_offsets<UT>(U);
  // Every issue executes the same loads: an exhausted stream issues them
  // against empty descriptors (no memory access) so that the number of loads
  // in flight is the same on every path and the compiler can wait for one
  // block at a time.
  auto issue = [&](Slot &sl) -> bool {
    const bool valid = more;
    load_slot<UT, AUX>(sl, lo, cur.Hw, cur.yw, U, crb, cur.r0, cur.r1, valid);
    sl.s = cur.s;
    sl.tk = cur.tk;
    sl.last = crb + RPB >= cur.r1;
    if (valid) {
      if (crb + RPB < cur.r1) {
        crb += RPB;
      } else {
        SysRef nx;
        if (gen(nx)) {
          cur = nx;
          crb = cur.r0;
        } else {
          more = false;
        }
      }
    }
    return valid;
  };
  stream_ring3<Slot>(issue, body, done);
}

// Fixed list of systems 0..ns-1 described by seg(s, Hw, yw, r0, r1);
// done(s) follows the last block of system s.
template <int UT, int AUX, class Seg, class Body, class Done>
__device__ __forceinline__ void stream_blocks(int ns, int U, Seg seg, Body body, Done done) {
  int next = 0;
  auto gen = [&](SysRef &r) -> bool {
    if (next >= ns) return false;
    seg(next, r.Hw, r.yw, r.r0, r.r1);
    r.tk = 0;
    r.s = next++;
    return true;
  };
  stream_gen<UT, AUX>(U, gen, body, [&](const Slot &sl) { done(sl.s); });
}

// ---------------------------------------------------------------- Gram + matched filter
// acc += real split of the block's H^H H: rr = Hr^T Hr, ri = Hr^T Hi,
// ii = Hi^T Hi in the BF16 forms; in FP32, two products only, rr = P =
// (Hr + Hi)^T (Hr + Hi) = Hr^T Hr + Hi^T Hi + ri + ri^T and ri (Re G needs
// only the sum of the two squares, store_gram takes ri + ri^T back out).
// (mfx, mfy) += partial of sum conj(H[row][col]) y[row].
template <int UT, int PREC>
__device__ __forceinline__ void gram_blk(const Slot &sl, int U, Acc<UT> &acc, float &mfx, float &mfy) {
  Blk8 b;
#pragma unroll
  for (int e = 0; e < 8; ++e) b.h[e] = slot_h<UT>(sl, e, U);
  if constexpr (PREC == PREC_FP32) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float sum = b.h[e].x + b.h[e].y;
      acc.rr = mma32(sum, sum, acc.rr);
      acc.ri = mma32(b.h[e].x, b.h[e].y, acc.ri);
    }
  } else if constexpr (PREC == PREC_BF16) {
    bf8 re, im;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      re[e] = (__bf16)b.h[e].x;
      im[e] = (__bf16)b.h[e].y;
    }
    acc.rr = mma16(re, re, acc.rr);
    acc.ri = mma16(re, im, acc.ri);
    acc.ii = mma16(im, im, acc.ii);
  } else {
    bf8 rh, rl, ih, il;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      rh[e] = (__bf16)b.h[e].x;
      rl[e] = (__bf16)(b.h[e].x - (float)rh[e]);
      ih[e] = (__bf16)b.h[e].y;
      il[e] = (__bf16)(b.h[e].y - (float)ih[e]);
    }
    acc.rr = mma16(rh, rl, acc.rr);
    acc.rr = mma16(rl, rh, acc.rr);
    acc.rr = mma16(rh, rh, acc.rr);
    acc.ri = mma16(rh, il, acc.ri);
    acc.ri = mma16(rl, ih, acc.ri);
    acc.ri = mma16(rh, ih, acc.ri);
    acc.ii = mma16(ih, il, acc.ii);
    acc.ii = mma16(il, ih, acc.ii);
    acc.ii = mma16(ih, ih, acc.ii);
  }
  // conj(h) * y as FMACs whose y operand is the DPP row broadcast of the
  // lane that loaded it
  sfor<8>([&](auto E) {
    constexpr int e = E;
    fmac_rowbcast<e, false, e == 0 ? 4 : 0>(mfx, sl.yl.x, b.h[e].x);
    fmac_rowbcast<e, false, 0>(mfy, sl.yl.y, b.h[e].x);
    fmac_rowbcast<e, false, 0>(mfx, sl.yl.y, b.h[e].y);
    fmac_rowbcast<e, true, 0>(mfy, sl.yl.x, b.h[e].y);
  });
}

// Gram + matched filter of systems 0..ns-1; done(s, acc, mf) receives each
// system's accumulators and its matched filter (reduced over a column).
// AUX is the loads' cache policy (kLoadLast unless a later pass re-reads H).
template <int UT, int PREC, int AUX, class Seg, class Done>
__device__ __forceinline__ void gram_stream(int ns, int U, Seg seg, Done done) {
  Acc<UT> acc;
  acc_zero<UT>(acc);
  float mfx = 0.f, mfy = 0.f;
  stream_blocks<UT, AUX>(
      ns, U, seg, [&](const Slot &b) { gram_blk<UT, PREC>(b, U, acc, mfx, mfy); },
      [&](int s) {
        done(s, acc, make_float2(colsum<UT>(mfx), colsum<UT>(mfy)));
        acc_zero<UT>(acc);
        mfx = 0.f;
        mfy = 0.f;
      });
}

// Residual pass of the refinement step: for system s (zcf(s) gives z[col]
// of that system) accumulates n = H^H (y - H z) and calls done(s, n) with
// n[col] valid in every lane.
template <int UT, class Seg, class Zc, class Done>
__device__ __forceinline__ void residual_stream(int ns, int U, Seg seg, Zc zcf, Done done) {
  float nx = 0.f, ny = 0.f;
  float2 zc = zcf(0);
  stream_blocks<UT, kLoadLast>(
      ns, U, seg,
      [&](const Slot &b) {
        sfor<8>([&](auto E) {
          constexpr int e = E;
          const float2 h = slot_h<UT>(b, e, U);
          // (H z)_row = sum over the UT lanes of this row of h * z
          const float px = gsum<UT>(h.x * zc.x - h.y * zc.y);
          const float py = gsum<UT>(h.x * zc.y + h.y * zc.x);
          const float2 yv = slot_y<UT, e>(b);
          const float rx = yv.x - px;
          const float ry = yv.y - py;
          nx = fmaf(h.x, rx, nx);
          nx = fmaf(h.y, ry, nx);
          ny = fmaf(h.x, ry, ny);
          ny = fmaf(-h.y, rx, ny);
        });
      },
      [&](int s) {
        done(s, make_float2(colsum<UT>(nx), colsum<UT>(ny)));
        nx = 0.f;
        ny = 0.f;
        if (s + 1 < ns) zc = zcf(s + 1);
      });
}

// Element (i, k) of a UT x UT matrix in LDS.  Rows are not padded: column k
// of row i is stored at k ^ i, so that the lanes of a group that read one
// row, or one column, touch UT different banks.
template <int UT>
__device__ __forceinline__ float2 &lds_el(float2 (*As)[UT], int i, int k) {
  return As[i][k ^ i];
}

// Writes G + rho I of one system from the MFMA accumulators into LDS
// (full Hermitian matrix, swizzled rows):
//   Re G = Hr^T Hr + Hi^T Hi,   Im G[i][j] = (Hr^T Hi)[i][j] - (Hr^T Hi)[j][i],
// with Re G = P - ri - ri^T for the FP32 accumulators (see gram_blk).
// Rows and columns of padded users (i >= U) are zero; their diagonal gets 1
// instead of rho, so that the matrix stays positive definite when rho = 0
// (ZF).  That block is decoupled from the users' block, whose factor and
// solves it leaves unchanged.
template <int UT, int PREC>
__device__ __forceinline__ void store_gram(float2 (*As)[UT], const Acc<UT> &acc, float rho, int U = UT) {
  constexpr int NR = UT == 16 ? 4 : 16;
  const int lane = lane_id();
  sfor<NR>([&](auto R) {
    constexpr int r = R;
    int i, j;
    acc_pos<UT>(lane, r, i, j);
    lds_el<UT>(As, i, j) = make_float2(0.f, acc.ri[r]);
  });
  __syncthreads();
  float im[NR], re[NR];
  sfor<NR>([&](auto R) {
    constexpr int r = R;
    int i, j;
    acc_pos<UT>(lane, r, i, j);
    const float rij = lds_el<UT>(As, j, i).y;  // (Hr^T Hi)[j][i]
    im[r] = acc.ri[r] - rij;
    re[r] = PREC == PREC_FP32 ? acc.rr[r] - acc.ri[r] - rij : acc.rr[r] + acc.ii[r];
  });
  __syncthreads();
  sfor<NR>([&](auto R) {
    constexpr int r = R;
    int i, j;
    acc_pos<UT>(lane, r, i, j);
    lds_el<UT>(As, i, j) = make_float2(re[r] + (i == j ? (i < U ? rho : 1.f) : 0.f), im[r]);
  });
}

template <int UT>
__device__ __forceinline__ void store_identity(float2 (*As)[UT]) {
  for (int idx = lane_id(); idx < UT * UT; idx += 64) {
    const int i = idx / UT, j = idx % UT;
    lds_el<UT>(As, i, j) = make_float2(i == j ? 1.f : 0.f, 0.f);
  }
}

// ---------------------------------------------------------------- factor / solves
// Keeps the scheduler from hoisting the broadcasts of later pivot steps above
// the current one (which would keep hundreds of values live at once).
__device__ __forceinline__ void step_fence() { __builtin_amdgcn_sched_barrier(0); }

// Hides a register's value from common-subexpression elimination: the
// inverse broadcasts the same (lane, register) pairs as the factorisation,
// and reusing those would keep every broadcast of the factorisation live.
__device__ __forceinline__ void opaque(float2 &v) { asm volatile("" : "+v"(v.x), "+v"(v.y)); }

// The same for a lane index: each phase of the solve compares it with the
// step number, and sharing those lane masks between phases would keep dozens
// of 64-bit masks live in scalar registers.
__device__ __forceinline__ int opaque_idx(int i) {
  asm volatile("" : "+v"(i));
  return i;
}

template <int UT>
struct Factor {
  float2 a[UT];   // row i of L (entries j <= i), lane i of the group
  float2 x[UT];   // column i of X = L^{-1}
  float dinv;     // 1 / L_ii of this lane's row
};

// Step j of the right-looking Cholesky A = L L^H of the row held by each
// lane: column j of L, then the update of the trailing columns j < k < KEND.
template <int UT, int J, int KEND>
__device__ __forceinline__ void chol_step(Factor<UT> &f, int i, int &fail) {
  constexpr int j = J;
  const float ajj = gbcast<UT, j>(f.a[j].x);
  if (!(ajj > 0.f) && fail == 0) fail = j + 1;
  // hardware reciprocal square root (about 1 ulp): 1/L_jj and L_jj = a_jj / sqrt(a_jj)
  const float inv = __builtin_amdgcn_rsqf(ajj);
  const float ljj = ajj * inv;
  if (i == j) f.dinv = inv;
  float2 lij = make_float2(f.a[j].x * inv, f.a[j].y * inv);
  if (i == j) lij = make_float2(ljj, 0.f);
  if (i < j) lij = make_float2(0.f, 0.f);
  f.a[j] = lij;
  const float2 lm = (i > j) ? lij : make_float2(0.f, 0.f);
  // a_ik -= l_ij * conj(l_kj), with l_kj broadcast from lane k: the real
  // part of l_kj for every k, then the imaginary part, so that no
  // instruction reads an accumulator its predecessor wrote
  const BSrc bx = bsrc<UT>(lij.x), by = bsrc<UT>(lij.y);
  sfor<UT>([&](auto K) {
    constexpr int k = K;
    if constexpr (k > j && k < KEND) {
      fmac_rowbcast<k % 16, true, k == j + 1 ? 4 : 0>(f.a[k].x, bpick<k>(bx), lm.x);
      fmac_rowbcast<k % 16, true, 0>(f.a[k].y, bpick<k>(bx), lm.y);
    }
  });
  sfor<UT>([&](auto K) {
    constexpr int k = K;
    if constexpr (k > j && k < KEND) {
      fmac_rowbcast<k % 16, true, k == j + 1 ? 4 : 0>(f.a[k].x, bpick<k>(by), lm.y);
      fmac_rowbcast<k % 16, false, 0>(f.a[k].y, bpick<k>(by), lm.x);
    }
  });
  step_fence();
}

// Right-looking Cholesky A = L L^H of the row held by each lane.
// Returns 0, or j+1 for the first pivot j that is not positive (or NaN).
template <int UT>
__device__ __forceinline__ int cholesky(Factor<UT> &f, int i) {
  i = opaque_idx(i);
  int fail = 0;
  sfor<UT>([&](auto J) { chol_step<UT, J, UT>(f, i, fail); });
  return fail;
}

// Lane u computes column u of X = L^{-1}:
//   X_ju = (delta_ju - sum_{k<j} L_jk X_ku) / L_jj,
// right-looking: once X_ju is final, every later row i subtracts L_ij X_ju
// (L_ij broadcast from lane i), so each step has UT - 1 - j independent
// accumulators instead of one long chain.  inv_step is step j, with the
// update restricted to the rows j < i < IEND.
template <int UT, int J, int IEND>
__device__ __forceinline__ void inv_step(Factor<UT> &f) {
  constexpr int j = J;
  const float invj = gbcast<UT, j>(f.dinv);
  f.x[j] = make_float2(f.x[j].x * invj, f.x[j].y * invj);
  // x_i -= L_ij x_j: real part of L_ij for every i, then the imaginary part
  const BSrc bx = bsrc<UT>(f.a[j].x), by = bsrc<UT>(f.a[j].y);
  sfor<UT>([&](auto I) {
    constexpr int i = I;
    if constexpr (i > j && i < IEND) {
      fmac_rowbcast<i % 16, true, i == j + 1 ? 4 : 0>(f.x[i].x, bpick<i>(bx), f.x[j].x);
      fmac_rowbcast<i % 16, true, 0>(f.x[i].y, bpick<i>(bx), f.x[j].y);
    }
  });
  sfor<UT>([&](auto I) {
    constexpr int i = I;
    if constexpr (i > j && i < IEND) {
      fmac_rowbcast<i % 16, false, i == j + 1 ? 4 : 0>(f.x[i].x, bpick<i>(by), f.x[j].y);
      fmac_rowbcast<i % 16, true, 0>(f.x[i].y, bpick<i>(by), f.x[j].x);
    }
  });
  step_fence();
}

template <int UT>
__device__ __forceinline__ void inverse_columns(Factor<UT> &f, int u) {
  u = opaque_idx(u);
#pragma unroll
  for (int j = 0; j < UT; ++j) f.x[j] = make_float2(u == j ? 1.f : 0.f, 0.f);
  sfor<UT>([&](auto J) { inv_step<UT, J, UT>(f); });
}

// The factorisation and inverse of a system whose rows KE..UT-1 are padding
// (users past U: identity rows of A, so identity rows of L and X): the first
// KE steps, with the updates restricted to the first KE rows and columns.
template <int UT, int KE>
__device__ __forceinline__ int cholesky_pad(Factor<UT> &f, int i) {
  i = opaque_idx(i);
  int fail = 0;
  sfor<KE>([&](auto J) { chol_step<UT, J, KE>(f, i, fail); });
  if (i >= KE) f.dinv = 1.f;
  return fail;
}

template <int UT, int KE>
__device__ __forceinline__ void inverse_columns_pad(Factor<UT> &f, int u) {
  u = opaque_idx(u);
#pragma unroll
  for (int j = 0; j < UT; ++j) f.x[j] = make_float2(u == j ? 1.f : 0.f, 0.f);
  sfor<KE>([&](auto J) { inv_step<UT, J, KE>(f); });
}

// ---- 32 x 32: the two 16 x 16 x 16 products of the blocked forms on MFMA
// With A = [A11 A12; A21 A22] in 16 x 16 blocks, the Cholesky factor is
// L11 = chol(A11), L21 = A21 L11^{-H}, L22 = chol(A22 - L21 L21^H), and the
// inverse X = L^{-1} has X11 = L11^{-1}, X22 = L22^{-1}, X21 = -X22 (L21 X11).
// The first 16 steps of the factorisation and of the inverse run on their
// own block only; the Schur complement A22 - L21 L21^H and -L21 X11 are
// complex products on 16x16x4 FP32 MFMA, staged through the LDS matrix slot
// of each system of the wave (free while the solve runs), and the last 16
// steps are the usual ones.  This moves 2,048 of the DPP FMACs of a round
// onto the matrix cores.  Each slot holds three 16 x 16 matrices with a row
// stride of 17 elements (a column read touches 16 distinct bank pairs):
// L21 at 0, A22 / S then X11 at kSplitM, -L21 X11 at kSplitY.
constexpr int kSplitStride = 17;
constexpr int kSplitM = 16 * kSplitStride;
constexpr int kSplitY = 32 * kSplitStride;

// C (16 x 16, MFMA D layout) += sign(A) * A B over K = 16 for complex A, B
// given per lane as A[lr][4 kc + lg] and B[4 kc + lg][lr] (lr = lane % 16,
// lg = lane / 16): the four real products of the complex one.
template <class GetA, class GetB>
__device__ __forceinline__ void cmma16(f4 &re, f4 &im, GetA ga, GetB gb, bool neg) {
#pragma unroll
  for (int kc = 0; kc < 4; ++kc) {
    const float2 p = ga(kc), q = gb(kc);
    const float s = neg ? -1.f : 1.f;
    re = mma32(s * p.x, q.x, re);
    re = mma32(-s * p.y, q.y, re);
    im = mma32(s * p.x, q.y, im);
    im = mma32(s * p.y, q.x, im);
  }
}

// Schur complement of the 32 x 32 systems of the wave: lanes 16..31 of each
// group (rows 16..31) hold L21 in a[0..15] and A22 in a[16..31] on entry and
// S = A22 - L21 L21^H in a[16..31] on return.  base: the wave's LDS slots.
__device__ __forceinline__ void schur32_mfma(Factor<32> &f, int gi, float2 *base) {
  const int lane = lane_id();
  float2 *W = base + (lane / 32) * 1024;
  if (gi >= 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      W[(gi - 16) * kSplitStride + k] = f.a[k];
      W[kSplitM + (gi - 16) * kSplitStride + k] = f.a[16 + k];
    }
  }
  __syncthreads();
  const int lr = lane % 16, lg = lane / 16;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    float2 *Ws = base + s * 1024;
    f4 re, im;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float2 v = Ws[kSplitM + (4 * lg + r) * kSplitStride + lr];
      re[r] = v.x;
      im[r] = v.y;
    }
    // (L21 L21^H)[i][j] = sum_k L21[i][k] conj(L21[j][k]): both operands are
    // the element (lr, 4 kc + lg) of L21
    auto ga = [&](int kc) { return Ws[lr * kSplitStride + 4 * kc + lg]; };
    auto gb = [&](int kc) {
      const float2 v = Ws[lr * kSplitStride + 4 * kc + lg];
      return make_float2(v.x, -v.y);
    };
    cmma16(re, im, ga, gb, true);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ws[kSplitM + (4 * lg + r) * kSplitStride + lr] = make_float2(re[r], im[r]);
  }
  __syncthreads();
  if (gi >= 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) f.a[16 + k] = W[kSplitM + (gi - 16) * kSplitStride + k];
  }
}

__device__ __forceinline__ int cholesky32_split(Factor<32> &f, int i, float2 *base) {
  i = opaque_idx(i);
  int fail = 0;
  sfor<16>([&](auto J) { chol_step<32, J, 16>(f, i, fail); });
  schur32_mfma(f, i, base);
  sfor<16>([&](auto J) {
    constexpr int j = J;
    chol_step<32, j + 16, 32>(f, i, fail);
  });
  return fail;
}

// X = L^{-1} by columns (lane u = column u), with rows 16..31 of the columns
// u < 16 set to -L21 X11 on MFMA between the two halves.  L21 is still in
// each slot from cholesky32_split.
__device__ __forceinline__ void inverse32_split(Factor<32> &f, int u, float2 *base) {
  u = opaque_idx(u);
#pragma unroll
  for (int j = 0; j < 32; ++j) f.x[j] = make_float2(u == j ? 1.f : 0.f, 0.f);
  sfor<16>([&](auto J) { inv_step<32, J, 16>(f); });
  const int lane = lane_id();
  float2 *W = base + (lane / 32) * 1024;
  if (u < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) W[kSplitM + k * kSplitStride + u] = f.x[k];
  }
  __syncthreads();
  const int lr = lane % 16, lg = lane / 16;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    float2 *Ws = base + s * 1024;
    f4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
    auto ga = [&](int kc) { return Ws[lr * kSplitStride + 4 * kc + lg]; };
    auto gb = [&](int kc) { return Ws[kSplitM + (4 * kc + lg) * kSplitStride + lr]; };
    cmma16(re, im, ga, gb, true);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ws[kSplitY + (4 * lg + r) * kSplitStride + lr] = make_float2(re[r], im[r]);
  }
  __syncthreads();
  if (u < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) f.x[16 + k] = W[kSplitY + k * kSplitStride + u];
  }
  sfor<16>([&](auto J) {
    constexpr int j = J;
    inv_step<32, j + 16, 32>(f);
  });
}

// The same two forms in halves, for callers whose U may leave padded users
// in a 32-lane group (the FD forms): the first 16 steps with the block
// products, then steps 16 .. KE-1 with the updates restricted to the first KE
// rows and columns.  For KE = 24 the rows 24..31 must be padding: users past
// U, whose rows of A are the identity (zero Gram entries, 1 on the diagonal),
// so their rows of L and X are the identity too and the 8 steps left out
// would only scale them by 1.  cholesky32_split and inverse32_split keep their
// own copies of the first halves: built from these pieces, the PD kernels
// (which never take the short form) ran 1-2% slower.
__device__ __forceinline__ int cholesky32_first(Factor<32> &f, int i, float2 *base) {
  i = opaque_idx(i);
  int fail = 0;
  sfor<16>([&](auto J) { chol_step<32, J, 16>(f, i, fail); });
  schur32_mfma(f, i, base);
  return fail;
}

template <int KE>
__device__ __forceinline__ void cholesky32_second(Factor<32> &f, int i, int &fail) {
  i = opaque_idx(i);
  sfor<KE - 16>([&](auto J) {
    constexpr int j = J;
    chol_step<32, j + 16, KE>(f, i, fail);
  });
  if constexpr (KE < 32) {
    if (i >= KE) f.dinv = 1.f;
  }
}

__device__ __forceinline__ void inverse32_first(Factor<32> &f, int u, float2 *base) {
  u = opaque_idx(u);
#pragma unroll
  for (int j = 0; j < 32; ++j) f.x[j] = make_float2(u == j ? 1.f : 0.f, 0.f);
  sfor<16>([&](auto J) { inv_step<32, J, 16>(f); });
  const int lane = lane_id();
  float2 *W = base + (lane / 32) * 1024;
  if (u < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) W[kSplitM + k * kSplitStride + u] = f.x[k];
  }
  __syncthreads();
  const int lr = lane % 16, lg = lane / 16;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    float2 *Ws = base + s * 1024;
    f4 re = {0.f, 0.f, 0.f, 0.f}, im = {0.f, 0.f, 0.f, 0.f};
    auto ga = [&](int kc) { return Ws[lr * kSplitStride + 4 * kc + lg]; };
    auto gb = [&](int kc) { return Ws[kSplitM + (4 * kc + lg) * kSplitStride + lr]; };
    cmma16(re, im, ga, gb, true);
#pragma unroll
    for (int r = 0; r < 4; ++r) Ws[kSplitY + (4 * lg + r) * kSplitStride + lr] = make_float2(re[r], im[r]);
  }
  __syncthreads();
  if (u < 16) {
#pragma unroll
    for (int k = 0; k < 16; ++k) f.x[16 + k] = W[kSplitY + k * kSplitStride + u];
  }
}

template <int KE>
__device__ __forceinline__ void inverse32_second(Factor<32> &f) {
  sfor<KE - 16>([&](auto J) {
    constexpr int j = J;
    inv_step<32, j + 16, KE>(f);
  });
}

// The same inverse with L read from LDS instead of registers: Ls holds L
// (row i written by lane i) with 1 / L_jj on the diagonal, and every lane of
// a group reads the same element (an LDS broadcast).  The rows of L in
// registers are dead once they are stored, which is what the 32-lane groups
// need: there L and L^{-1} together take 128 VGPRs.
template <int UT>
__device__ __forceinline__ void inverse_columns_lds(Factor<UT> &f, int u, float2 (*Ls)[UT]) {
  u = opaque_idx(u);
#pragma unroll
  for (int j = 0; j < UT; ++j) f.x[j] = make_float2(u == j ? 1.f : 0.f, 0.f);
  sfor<UT>([&](auto J) {
    constexpr int j = J;
    const float invj = lds_el<UT>(Ls, j, j).x;
    f.x[j] = make_float2(f.x[j].x * invj, f.x[j].y * invj);
    // x_i -= L_ij x_j
    sfor<UT>([&](auto I) {
      constexpr int i = I;
      if constexpr (i > j) {
        const float2 l = lds_el<UT>(Ls, i, j);
        f.x[i].x = fmaf(-l.x, f.x[j].x, fmaf(l.y, f.x[j].y, f.x[i].x));
        f.x[i].y = fmaf(-l.x, f.x[j].y, fmaf(-l.y, f.x[j].x, f.x[i].y));
      }
    });
    step_fence();
  });
}

// t = L^{-1} b by forward substitution; lane i holds b_i on entry, t_i on exit.
template <int UT>
__device__ __forceinline__ float2 fwd_subst(const Factor<UT> &f, int i, float2 b) {
  i = opaque_idx(i);
  float2 t = b;
  sfor<UT>([&](auto J) {
    constexpr int j = J;
    if (i == j) { t.x *= f.dinv; t.y *= f.dinv; }
    const float2 tj = gbcast2<UT, j>(t);
    if (i > j) {
      t.x -= f.a[j].x * tj.x - f.a[j].y * tj.y;
      t.y -= f.a[j].x * tj.y + f.a[j].y * tj.x;
    }
  });
  return t;
}

// (X^H t)_u = sum_j conj(X_ju) t_j for lane u; t_j is the DPP row broadcast
// of lane j, fused into the FMACs (t does not change here, so one group).
template <int UT>
__device__ __forceinline__ float2 apply_xh(const Factor<UT> &f, float2 t) {
  const BSrc bx = bsrc<UT>(t.x), by = bsrc<UT>(t.y);
  float r[4] = {0.f, 0.f, 0.f, 0.f};
  sfor<UT>([&](auto J) {
    constexpr int j = J;
    constexpr int p = 2 * (j & 1);
    // the first reader of each source carries the wait states
    fmac_rowbcast<j % 16, false, j == 0 ? 4 : 0>(r[p], bpick<j>(bx), f.x[j].x);
    fmac_rowbcast<j % 16, false, j == 0 ? 4 : 0>(r[p + 1], bpick<j>(by), f.x[j].x);
    fmac_rowbcast<j % 16, false, 0>(r[p], bpick<j>(by), f.x[j].y);
    fmac_rowbcast<j % 16, true, 0>(r[p + 1], bpick<j>(bx), f.x[j].y);
  });
  return make_float2(r[0] + r[2], r[1] + r[3]);
}

// Factorises A (rows in f.a) and solves A z = m: returns z_u at lane u,
// fills f.x (columns of L^{-1}) and sets `fail` (0 or first bad pivot + 1).
// The forward substitution runs before the inverse so the two independent
// chains are not interleaved by the compiler.
//
// Ls (optional) is the LDS matrix slot the system was loaded from: with it,
// 32-lane groups store L there and form the inverse from LDS.
//
// PAD: U (wave-uniform) may leave padded users; the 32 x 32 forms (PAD & 1)
// then leave out the last 8 steps for at most 24 users, the 16 x 16 forms
// (PAD & 2) the last 8 for at most 8 users.
template <int UT, int PAD = 0>
__device__ __forceinline__ float2 factor_solve(Factor<UT> &f, int i, float2 m, int &fail,
                                               float2 (*Ls)[UT] = nullptr, float2 *split = nullptr,
                                               int U = UT) {
  if constexpr (UT == 16 && (PAD & 2)) {
    if (__builtin_amdgcn_readfirstlane(U) <= 8) {
      fail = cholesky_pad<UT, 8>(f, i);
      const float2 t = fwd_subst<UT>(f, i, m);
      asm volatile("" : "+v"(f.a[0].x) : "v"(t.x), "v"(t.y));
      inverse_columns_pad<UT, 8>(f, i);
      return apply_xh<UT>(f, t);
    }
  }
  if constexpr (UT == 32 && (PAD & 1)) {
    if (split) {
      const bool u24 = __builtin_amdgcn_readfirstlane(U) <= 24;
      fail = cholesky32_first(f, i, split);
      if (u24)
        cholesky32_second<24>(f, i, fail);
      else
        cholesky32_second<32>(f, i, fail);
      const float2 t = fwd_subst<UT>(f, i, m);
      asm volatile("" : "+v"(f.a[0].x) : "v"(t.x), "v"(t.y));
      inverse32_first(f, i, split);
      if (u24)
        inverse32_second<24>(f);
      else
        inverse32_second<32>(f);
      return apply_xh<UT>(f, t);
    }
  }
  if constexpr (UT == 32) {
    if (split) {
      // the wave's systems each own an LDS matrix slot (split: the first)
      fail = cholesky32_split(f, i, split);
      const float2 t = fwd_subst<UT>(f, i, m);
      asm volatile("" : "+v"(f.a[0].x) : "v"(t.x), "v"(t.y));
      inverse32_split(f, i, split);
      return apply_xh<UT>(f, t);
    }
  }
  fail = cholesky<UT>(f, i);
  const float2 t = fwd_subst<UT>(f, i, m);
  asm volatile("" : "+v"(f.a[0].x) : "v"(t.x), "v"(t.y));
  if (UT == 32 && Ls) {
    // row i of L, with 1 / L_ii on the diagonal
#pragma unroll
    for (int k = 0; k < UT; ++k) lds_el<UT>(Ls, i, k) = k == i ? make_float2(f.dinv, 0.f) : f.a[k];
    __syncthreads();
    inverse_columns_lds<UT>(f, i, Ls);
  } else {
    inverse_columns<UT>(f, i);
  }
  return apply_xh<UT>(f, t);
}

// Factorises A (rows in f.a) and forms the columns of X = L^{-1} in f.x,
// for systems whose right-hand sides come later (several per factor).
// Returns 0 or the first bad pivot + 1.  With Ls (32-lane groups) L is
// stored there and the inverse is formed from LDS, as in factor_solve.
template <int UT>
__device__ __forceinline__ int factor_inverse(Factor<UT> &f, int i, float2 (*Ls)[UT] = nullptr,
                                              float2 *split = nullptr) {
  if constexpr (UT == 32) {
    if (split) {
      // the wave's systems each own an LDS matrix slot (split: the first)
      const int fail = cholesky32_split(f, i, split);
      inverse32_split(f, i, split);
      return fail;
    }
  }
  const int fail = cholesky<UT>(f, i);
  if (UT == 32 && Ls) {
#pragma unroll
    for (int k = 0; k < UT; ++k) lds_el<UT>(Ls, i, k) = k == i ? make_float2(f.dinv, 0.f) : f.a[k];
    __syncthreads();
    inverse_columns_lds<UT>(f, i, Ls);
  } else {
    inverse_columns<UT>(f, i);
  }
  return fail;
}

// A^{-1} b for lane-distributed b (lane i holds b_i); result at lane u.
template <int UT>
__device__ __forceinline__ float2 solve(const Factor<UT> &f, int i, float2 b) {
  return apply_xh<UT>(f, fwd_subst<UT>(f, i, b));
}

// [A^{-1}]_uu for lane u.
template <int UT>
__device__ __forceinline__ float inv_diag(const Factor<UT> &f) {
  float d = 0.f;
#pragma unroll
  for (int j = 0; j < UT; ++j) d += f.x[j].x * f.x[j].x + f.x[j].y * f.x[j].y;
  return d;
}

__device__ __forceinline__ bool finite2(float2 v) { return isfinite(v.x) && isfinite(v.y); }

// Row sums for the condition estimate and the finiteness test of a system:
// (|Re| + |Im|) of each entry, scaled by 2^-32 so that no row of finite
// entries overflows.  The scaled sum is finite exactly when every entry is,
// and 2^32 times it bounds the row's sum of moduli from above (by at most
// sqrt 2).  Two FMAs per entry, against a square root and two compares.
constexpr float kRowScale = 0x1p-32f;
__device__ __forceinline__ float abs_row_acc(float acc, float2 v) {
  return fmaf(fabsf(v.y), kRowScale, fmaf(fabsf(v.x), kRowScale, acc));
}

// Unbiased L-MMSE: the L-MMSE estimate of user u has gain
// mu_u = [(G + rho I)^{-1} G]_uu = 1 - rho d_u = 1 - sigma2_u / E_s; returns
// 1 / mu_u for ub = 1/E_s, and exactly 1 for ub = 0 (biased L-MMSE, ZF).
__device__ __forceinline__ float unbias_factor(float s2, float ub) { return 1.0f / (1.0f - s2 * ub); }

}  // namespace dbpeq
