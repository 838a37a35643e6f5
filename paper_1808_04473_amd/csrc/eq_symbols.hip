// Several receive vectors per channel matrix (Section VI-B).
//
// The OFDM symbols of one coherence interval share the channel, so the Gram
// matrix of a subcarrier (PD) or cluster (FD) and its factor are formed once
// and applied to every symbol; only the matched filter is formed per symbol.
// The matched filters of a tile of up to UT symbols, H_c^H [y_1 .. y_S], are a
// second MFMA product in the same pass over H: lane (g, j) of the streaming
// layout loads rows 8g .. 8g+7 of receive vector j, which is the B operand
// for the same K (row) index as the lane's H value is for the Gram.  H and
// the receive vectors are each read from HBM once per tile.
//
// After the pass a lane group factors its system and forms X = L^{-1}.
// With 16 users the estimates of all symbols, Z = X^H (X M), are two
// complex 16 x 16 x 16 products on FP32 MFMA per system; with 32 users each
// lane group computes, per symbol, t = X m_s (rows of X read back from LDS)
// and z_s = X^H t (columns of X in registers).  FD weights every cluster's
// estimates with the weights of Lemma 1 (or given ones), which do not depend
// on the symbol, and sums them over the clusters in cluster order.
//
// LAMA (Algorithm 1) runs on the same pass, the iteration once per vector
// with the system's Gram row held in registers (eq_symbols_lama_kernel).
//
// Forms: FP32 MFMA (the matched filter as three real products), and
// split-BF16 MFMA (three products per real product) without refinement; the refining forms are not offered for several
// symbols.  Ill-conditioned systems go to the FP64 re-solve queue as in the
// single-vector kernels; the re-solve recomputes every symbol of the tile.
#include "eq_lama.h"

namespace dbpeq {

// ---------------------------------------------------------------- streaming
// One row block: H as in the single-vector stream, and rows 8g .. 8g+7 of
// receive vector j = lane % UT of the tile.
struct SymSlot {
  float2 h[8];
  float2 y[8];
  int s;
  int nv;  // rows of this lane's group, from its first, inside the system
  bool last;
};

template <int UT>
struct SymLaneOff {
  unsigned h;  // as LaneOff::h
  unsigned y;  // (j B + 8 g) * 8 for symbols j < nsym, else out of range
  int g;
};

template <int UT>
__device__ __forceinline__ SymLaneOff<UT> sym_lane_offsets(int U, int B, int nsym) {
  const int lane = lane_id();
  const int col = lane % UT, g = lane / UT;
  SymLaneOff<UT> o;
  o.h = col < U ? (unsigned)((slot_row(0, g) * U + col) * 8) : kOutOfRange;
  o.y = col < nsym ? (unsigned)(((unsigned)col * (unsigned)B + (unsigned)slot_row(0, g)) * 8u) : kOutOfRange;
  o.g = g;
  return o;
}

// Loads the row block at rb of rows [r0, r1) of H (row stride U) and of the
// tile's receive vectors (vector stride B, Yw = vector 0 of the tile).  The Y
// descriptor spans from row r0 of the first vector to row r1 of the last one:
// rows past r1 of the other vectors are in range and are masked by nv when
// the block is consumed.
template <int UT>
__device__ __forceinline__ void load_sym_slot(SymSlot &b, const SymLaneOff<UT> &lo, const float2 *__restrict__ Hw,
                                              const float2 *__restrict__ Yw, int U, int B, int nsym, int rb,
                                              int r0, int r1, bool live) {
  const int nrow = live ? r1 - r0 : 0;
  const int ylen = live ? ((nsym - 1) * B + (r1 - r0)) * 8 : 0;
  const __amdgpu_buffer_rsrc_t rh =
      __builtin_amdgcn_make_buffer_rsrc((void *)(Hw + (size_t)r0 * U), (short)0, nrow * U * 8, kBufFlags);
  const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc((void *)(Yw + r0), (short)0, ylen, kBufFlags);
  const unsigned rowb = (unsigned)((rb - r0) * U * 8);
  const unsigned step = (unsigned)(U * 8);
#pragma unroll
  for (int e = 0; e < 8; ++e) b.h[e] = buf_ld2<kLoadLast>(rh, lo.h + rowb + e * step);
  // one 8-byte load per row: a load is then either wholly inside the
  // descriptor's range or wholly outside it.  The eight loads of a lane read
  // one 64-byte span, so consecutive loads share cache lines: these use the
  // default policy (with the nontemporal one the lines were fetched from
  // HBM again, 22-28% more bytes than the algorithm reads).
  const unsigned yb = lo.y + (unsigned)((rb - r0) * 8);
#pragma unroll
  for (int e = 0; e < 8; ++e) b.y[e] = buf_ld2<kLoadKeep>(ry, yb + 8u * e);
  b.nv = r1 - (rb + slot_row(0, lo.g));
}

// Matched-filter accumulators, element (u, j) at the position acc_pos gives
// for (i, j).  FP32 forms the complex product H^H Y with three real MFMA
// products (Gauss):
//   k1 = (Hr - Hi)^T Yr,  k2 = Hr^T (Yi - Yr),  k3 = Hi^T (Yr + Yi),
//   Re M = Hr^T Yr + Hi^T Yi = k1 + k3,   Im M = Hr^T Yi - Hi^T Yr = k1 + k2;
// the split-BF16 form accumulates Re M in k1 and Im M in k2 directly.
template <int UT> struct MAcc;
template <> struct MAcc<16> { f4 k1, k2, k3; };
template <> struct MAcc<32> { f16v k1, k2, k3; };

template <int UT>
__device__ __forceinline__ void macc_zero(MAcc<UT> &m) {
  constexpr int NR = UT == 16 ? 4 : 16;
#pragma unroll
  for (int r = 0; r < NR; ++r) { m.k1[r] = 0.f; m.k2[r] = 0.f; m.k3[r] = 0.f; }
}

template <int PREC, int UT>
__device__ __forceinline__ float2 macc_value(const MAcc<UT> &m, int r) {
  if constexpr (PREC == PREC_FP32) return make_float2(m.k1[r] + m.k3[r], m.k1[r] + m.k2[r]);
  else return make_float2(m.k1[r], m.k2[r]);
}

// acc += the block's Gram products (as gram_blk: P and ri in FP32, the
// split products otherwise); m += H^H Y of the block.
template <int UT, int PREC>
__device__ __forceinline__ void gram_mf_blk(const SymSlot &sl, Acc<UT> &acc, MAcc<UT> &m) {
  float2 y[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) y[e] = e < sl.nv ? sl.y[e] : make_float2(0.f, 0.f);
  if constexpr (PREC == PREC_FP32) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 h = sl.h[e];
      const float sum = h.x + h.y;
      acc.rr = mma32(sum, sum, acc.rr);
      m.k1 = mma32(h.x - h.y, y[e].x, m.k1);
      acc.ri = mma32(h.x, h.y, acc.ri);
      m.k2 = mma32(h.x, y[e].y - y[e].x, m.k2);
      m.k3 = mma32(h.y, y[e].x + y[e].y, m.k3);
    }
  } else {
    static_assert(PREC == PREC_BF16X3_NR, "one-pass forms only");
    bf8 rh, rl, ih, il, yrh, yrl, yih, yil, nrh, nrl;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const float2 h = sl.h[e];
      rh[e] = (__bf16)h.x;
      rl[e] = (__bf16)(h.x - (float)rh[e]);
      ih[e] = (__bf16)h.y;
      il[e] = (__bf16)(h.y - (float)ih[e]);
      yrh[e] = (__bf16)y[e].x;
      yrl[e] = (__bf16)(y[e].x - (float)yrh[e]);
      yih[e] = (__bf16)y[e].y;
      yil[e] = (__bf16)(y[e].y - (float)yih[e]);
      // round-to-nearest-even is symmetric: the split of -yr is the negated split
      nrh[e] = -yrh[e];
      nrl[e] = -yrl[e];
    }
    acc.rr = mma16(rh, rl, acc.rr);
    m.k1 = mma16(rh, yrl, m.k1);
    acc.ri = mma16(rh, il, acc.ri);
    m.k2 = mma16(rh, yil, m.k2);
    acc.ii = mma16(ih, il, acc.ii);
    m.k1 = mma16(rl, yrh, m.k1);
    acc.rr = mma16(rl, rh, acc.rr);
    m.k2 = mma16(rl, yih, m.k2);
    acc.ri = mma16(rl, ih, acc.ri);
    m.k1 = mma16(rh, yrh, m.k1);
    acc.ii = mma16(il, ih, acc.ii);
    m.k2 = mma16(rh, yih, m.k2);
    acc.rr = mma16(rh, rh, acc.rr);
    m.k1 = mma16(ih, yil, m.k1);
    acc.ri = mma16(rh, ih, acc.ri);
    m.k2 = mma16(ih, nrl, m.k2);
    acc.ii = mma16(ih, ih, acc.ii);
    m.k1 = mma16(il, yih, m.k1);
    m.k2 = mma16(il, nrh, m.k2);
    m.k1 = mma16(ih, yih, m.k1);
    m.k2 = mma16(ih, nrh, m.k2);
  }
}

// Gram + matched filters of systems 0..ns-1 (seg(s, Hw, Yw, r0, r1) as in
// stream_blocks, Yw = vector 0 of the tile); done(s, acc, m) follows the last
// block of system s while the next blocks' loads are in flight.
template <int UT, int PREC, class Seg, class Done>
__device__ __forceinline__ void gram_mf_stream(int ns, int U, int B, int nsym, Seg seg, Done done) {
  constexpr int RPB = 8 * (64 / UT);
  Acc<UT> acc;
  acc_zero<UT>(acc);
  MAcc<UT> m;
  macc_zero<UT>(m);
  const SymLaneOff<UT> lo = sym_lane_offsets<UT>(U, B, nsym);
  SysRef cur;
  seg(0, cur.Hw, cur.yw, cur.r0, cur.r1);
  cur.s = 0;
  int next = 1;
  int crb = cur.r0;
  bool more = true;
  auto issue = [&](SymSlot &sl) -> bool {
    const bool valid = more;
    load_sym_slot<UT>(sl, lo, cur.Hw, cur.yw, U, B, nsym, crb, cur.r0, cur.r1, valid);
    sl.s = cur.s;
    sl.last = crb + RPB >= cur.r1;
    if (valid) {
      if (crb + RPB < cur.r1) {
        crb += RPB;
      } else if (next < ns) {
        seg(next, cur.Hw, cur.yw, cur.r0, cur.r1);
        cur.s = next++;
        crb = cur.r0;
      } else {
        more = false;
      }
    }
    return valid;
  };
  auto body = [&](const SymSlot &b) { gram_mf_blk<UT, PREC>(b, acc, m); };
  auto fin = [&](const SymSlot &b) {
    done(b.s, acc, m);
    acc_zero<UT>(acc);
    macc_zero<UT>(m);
  };
  stream_ring3<SymSlot>(issue, body, fin);
}

// ---------------------------------------------------------------- LDS staging
// NS matrix slots: A (G + rho I, then X), the matched filters of the tile
// (rows = symbols, padded by two entries so the MFMA-layout stores hit
// distinct banks, slots offset by 8 banks so the groups' broadcast reads do
// too), and per-group fusion terms (FD).
template <int UT, int NSLOT>
struct SymSmem {
  static constexpr int NSYS = 64 / UT;
  static constexpr int NS = NSLOT;
  static constexpr int MROW = UT + 2;
  static constexpr int MSLOT = UT * MROW + 4;
  float2 A[NS][UT][UT];
  float2 Mv[NS * MSLOT];
  float2 F[NS][UT];
  __device__ __forceinline__ float2 &m(int slot, int s, int u) { return Mv[slot * MSLOT + s * MROW + u]; }
};

template <int UT, int PREC, class SM>
__device__ __forceinline__ void store_msym(SM &sm, int slot, const MAcc<UT> &m) {
  constexpr int NR = UT == 16 ? 4 : 16;
  const int lane = lane_id();
  sfor<NR>([&](auto R) {
    constexpr int r = R;
    int i, j;
    acc_pos<UT>(lane, r, i, j);
    sm.m(slot, j, i) = macc_value<PREC>(m, r);
  });
}

// ---------------------------------------------------------------- solve
template <int UT>
struct SymSolve {
  Factor<UT> f;
  float2 xr[UT];  // row i of X (lane i; 32-lane groups only)
  float d;        // [A^{-1}]_ii
  float norm1;
  int fail;
  bool bad;
};

// Loads row i of the slot's A, factors it, forms X = L^{-1} (columns in
// f.x) and parks X in the slot (row u holds column u); 32-lane groups then
// read row i of X back.
template <int UT, class SM>
__device__ __forceinline__ void sym_factor(SymSolve<UT> &r, SM &sm, int slot, int i, int U) {
  float rowsum = 0.f;
#pragma unroll
  for (int k = 0; k < UT; ++k) {
    r.f.a[k] = lds_el<UT>(sm.A[slot], i, k);
    rowsum = abs_row_acc(rowsum, r.f.a[k]);
  }
  r.bad = gany<UT>(!isfinite(rowsum));
  r.norm1 = gmax<UT>(i < U ? rowsum * (1.f / kRowScale) : 0.f);
  // with a slot per system, the 32 x 32 factor and inverse run their two
  // block products on MFMA through the slots (read above, free until X is
  // parked)
  float2 *split = nullptr;
  if constexpr (UT == 32 && SM::NS == SM::NSYS) split = &sm.A[0][0][0];
  r.fail = factor_inverse<UT>(r.f, i, SM::NS < SM::NSYS ? sm.A[slot] : nullptr, split);
  r.d = inv_diag<UT>(r.f);
  __syncthreads();
  // row u of the slot holds column u of X: lds_el(A, u, k) = X_ku
#pragma unroll
  for (int k = 0; k < UT; ++k) lds_el<UT>(sm.A[slot], i, k) = r.f.x[k];
  __syncthreads();
  if constexpr (UT == 32) {
#pragma unroll
    for (int u = 0; u < UT; ++u) r.xr[u] = lds_el<UT>(sm.A[slot], u, i);
  }
}

// 16 x 16 systems: Z = X^H (X M) for the slot's system and the tile's
// symbols on FP32 MFMA (16x16x4), the whole wave on one system.  Each complex
// product takes three real products (Gauss).  X comes from the slot (row u
// holds column u of X), M from its matched-filter rows, which T = X M then
// replaces.  On return lane (kk, c) = (lane / 16, lane % 16) holds
// Z[4 kk + r][c] in (zr[r], zi[r]), r = 0..3: four users of symbol c.
template <class SM>
__device__ __forceinline__ void sym_mfma16(SM &sm, int slot, f4 &zr, f4 &zi) {
  const int lane = lane_id();
  const int kk = lane >> 4, c = lane & 15;
  f4 k1, k2, k3;
#pragma unroll
  for (int r = 0; r < 4; ++r) { k1[r] = 0.f; k2[r] = 0.f; k3[r] = 0.f; }
  // T = X M: operand A[c][u] = X_cu, B[u][c] = M[u][c] (u = 4q + kk);
  //   Re T = k1 - k3, Im T = k1 + k2 with k1 = (Xr + Xi) Mr,
  //   k2 = Xr (Mi - Mr), k3 = Xi (Mr + Mi)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int u = 4 * q + kk;
    const float2 x = lds_el<16>(sm.A[slot], u, c);
    const float2 mv = sm.m(slot, c, u);
    k1 = mma32(x.x + x.y, mv.x, k1);
    k2 = mma32(x.x, mv.y - mv.x, k2);
    k3 = mma32(x.y, mv.x + mv.y, k3);
  }
  // T replaces M (the wave's LDS accesses are performed in order, so every
  // read of M above precedes these writes)
#pragma unroll
  for (int r = 0; r < 4; ++r) sm.m(slot, c, 4 * kk + r) = make_float2(k1[r] - k3[r], k1[r] + k2[r]);
  __syncthreads();
#pragma unroll
  for (int r = 0; r < 4; ++r) { k1[r] = 0.f; k2[r] = 0.f; k3[r] = 0.f; }
  // Z = X^H T: operand A[c][i] = conj(X_ic), B[i][c] = T[i][c] (i = 4q + kk);
  //   Re Z = k1 + k3, Im Z = k1 + k2 with k1 = (Xr - Xi) Tr,
  //   k2 = Xr (Ti - Tr), k3 = Xi (Tr + Ti)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int i = 4 * q + kk;
    const float2 x = lds_el<16>(sm.A[slot], c, i);
    const float2 tv = sm.m(slot, c, i);
    k1 = mma32(x.x - x.y, tv.x, k1);
    k2 = mma32(x.x, tv.y - tv.x, k2);
    k3 = mma32(x.y, tv.x + tv.y, k3);
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    zr[r] = k1[r] + k3[r];
    zi[r] = k1[r] + k2[r];
  }
}

// z_s = X^H (X m_s) at lane i for the matched filter m_s of the slot.
template <int UT, class SM>
__device__ __forceinline__ float2 sym_apply(const SymSolve<UT> &r, SM &sm, int slot, int s) {
  float tx = 0.f, ty = 0.f;
#pragma unroll
  for (int u = 0; u < UT; ++u) {
    const float2 mv = sm.m(slot, s, u);
    tx = fmaf(r.xr[u].x, mv.x, fmaf(-r.xr[u].y, mv.y, tx));
    ty = fmaf(r.xr[u].x, mv.y, fmaf(r.xr[u].y, mv.x, ty));
  }
  return apply_xh<UT>(r.f, make_float2(tx, ty));
}

// MRC (Section III-A) on the slot's G (stored unshifted): lane i gets
// 1 / G_ii and sigma2_i = N0 / G_ii + E_s sum_{k != i} |G_ik|^2 / G_ii^2;
// fail = u + 1 for the group's first user with G_uu <= 0.
struct SymMrc {
  float inv_gii;
  float s2;
  int fail;
  bool bad;
};

template <int UT, class SM>
__device__ __forceinline__ SymMrc sym_mrc_row(SM &sm, int slot, int i, int U, float n0, float es) {
  float gii = 0.f, off = 0.f;
  bool bad = false;
#pragma unroll
  for (int k = 0; k < UT; ++k) {
    const float2 g = lds_el<UT>(sm.A[slot], i, k);
    bad |= !finite2(g);
    if (k == i) gii = g.x;
    else off = fmaf(g.x, g.x, fmaf(g.y, g.y, off));
  }
  SymMrc o;
  o.bad = gany<UT>(bad);
  const int base = (lane_id() / UT) * UT;
  const unsigned long long gm = ((UT == 64 ? ~0ull : ((1ull << UT) - 1ull)) << base);
  const unsigned long long fm = __ballot(i < U && !(gii > 0.f)) & gm;
  o.fail = fm ? __builtin_ctzll(fm) - base + 1 : 0;
  o.inv_gii = 1.0f / gii;
  o.s2 = n0 * o.inv_gii + es * off * o.inv_gii * o.inv_gii;
  return o;
}

__device__ __forceinline__ void enqueue_fp64_sym(const FwdArgs &a, int w) {
  const int pos = atomicAdd(a.fb_count, 1);
  if (pos >= 0 && pos < a.W) a.fb_list[pos] = w;  // capacity W
}

// PD: systems w0 .. w0+nvalid-1, one per lane group.
template <int UT, int PREC, bool MRC, class SM>
__device__ __forceinline__ void pd_sym_task(const FwdArgs &a, int w0, int nvalid, SM &sm) {
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  auto seg = [&](int s, const float2 *&Hw, const float2 *&Yw, int &r0, int &r1) {
    const size_t w = (size_t)w0 + s;
    Hw = a.H + w * HB;
    Yw = a.y + w * (size_t)a.ysw;
    r0 = 0;
    r1 = a.B;
  };
  gram_mf_stream<UT, PREC>(nvalid, a.U, a.B, a.nsym, seg, [&](int s, const Acc<UT> &acc, const MAcc<UT> &m) {
    store_gram<UT, PREC>(sm.A[s], acc, a.rho, a.U);
    store_msym<UT, PREC>(sm, s, m);
  });
  for (int s = nvalid; s < SM::NS; ++s) store_identity<UT>(sm.A[s]);
  __syncthreads();

  const int slot = slot_of<SM>(g);
  const bool live = g < nvalid;
  if constexpr (MRC) {
    const SymMrc o = sym_mrc_row<UT>(sm, slot, i, a.U, a.n0, a.es);
    const bool out_nan = o.bad || o.fail;
    const float nanv = __int_as_float(0x7fc00000);
    const int w = w0 + g;
    if (live && i < a.U) {
      float2 *zw = a.z + (size_t)w * a.zsw;
      for (int s = 0; s < a.nsym; ++s) {
        const float2 mv = sm.m(slot, s, i);
        zw[(size_t)s * a.U + i] = out_nan ? make_float2(nanv, nanv) : make_float2(mv.x * o.inv_gii, mv.y * o.inv_gii);
      }
      if (a.s2) a.s2[(size_t)w * a.U + i] = out_nan ? nanv : o.s2;
    }
    if (live && i == 0 && a.info) a.info[w] = o.bad ? -1 : o.fail;
    return;
  }
  SymSolve<UT> r;
  sym_factor<UT>(r, sm, slot, i, a.U);
  const float kappa = r.norm1 * gsum<UT>(i < a.U ? r.d : 0.f);
  const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
  const int w = w0 + g;
  const float nanv = __int_as_float(0x7fc00000);
  // gain factor of user i (1 unless the unbiased L-MMSE)
  const float ku = unbias_factor(a.n0 * r.d, a.ub);
  if constexpr (UT == 16) {
    // one system at a time on MFMA; slot q holds system w0 + q.  Lane
    // (kk, c) writes users 4 kk + r, whose factors it reads from F (the
    // barrier inside the first product orders these writes before the reads)
    sm.F[g][i] = make_float2(ku, 0.f);
    const unsigned long long badm = __ballot(r.bad);
    const int kk = lane >> 4, c = lane & 15;
    for (int q = 0; q < nvalid; ++q) {
      f4 zr, zi;
      sym_mfma16(sm, q, zr, zi);
      const bool bq = (badm >> (16 * q)) & 1ull;
      float2 *zw = a.z + (size_t)(w0 + q) * a.zsw + (size_t)c * a.U;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int u = 4 * kk + rr;
        const float kq = sm.F[q][u].x;
        if (c < a.nsym && u < a.U) zw[u] = bq ? make_float2(nanv, nanv) : make_float2(zr[rr] * kq, zi[rr] * kq);
      }
    }
  } else {
    float2 *zw = a.z + (size_t)w * a.zsw;
    for (int s = 0; s < a.nsym; ++s) {
      const float2 z = sym_apply<UT>(r, sm, slot, s);
      if (live && i < a.U) zw[(size_t)s * a.U + i] = r.bad ? make_float2(nanv, nanv) : make_float2(z.x * ku, z.y * ku);
    }
  }
  if (live) {
    if (i < a.U && a.s2) a.s2[(size_t)w * a.U + i] = r.bad ? nanv : a.n0 * r.d * ku;
    if (i == 0) {
      if (a.info) a.info[w] = (r.bad ? -1 : r.fail) | (routed ? EQ_INFO_FP64 : 0);
      if (routed) enqueue_fp64_sym(a, w);
    }
  }
}

// FD: all clusters of subcarrier w, NSYS local systems per round.  The
// fusion sums (eq. (fusionrule)) run over the clusters in cluster order.
// MRC (no factor) fuses m_s / G_uu with the 32-lane layout's LDS fusion at
// every width.
// 16-lane groups: Z of each cluster comes from MFMA in accumulator layout,
// and lane (kk, c) keeps the sums of users 4 kk + r of symbol c.  32-lane
// groups: lane (q, u) = (lane / UT, lane % UT) keeps the sums of user u for
// the symbols q, q + NSYS, q + 2 NSYS, ...
template <int UT, int PREC, bool MRC, class SM>
__device__ __forceinline__ void fd_sym_task(const FwdArgs &a, int w, SM &sm) {
  constexpr int NSYS = 64 / UT;
  constexpr int KS = UT == 16 ? 4 : UT / NSYS;  // sums per lane
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int C = a.C;
  const bool user_nu = a.nu != nullptr;
  const float nanv = __int_as_float(0x7fc00000);
  // F[g][i] = (weight of cluster g's estimate of user i, its term of tk):
  // tk sums the weights (optimal fusion: the fused variance is 1 / tk) or,
  // with given weights, nu^2 sigma2_c (the fused variance itself)
  float2 zf[KS];
  float tk[UT == 16 ? 4 : 1];
#pragma unroll
  for (int k = 0; k < KS; ++k) zf[k] = make_float2(0.f, 0.f);
#pragma unroll
  for (int k = 0; k < (UT == 16 ? 4 : 1); ++k) tk[k] = 0.f;
  bool routed_any = false;
  // MRC keeps the sums in the (lane / UT, lane % UT) layout at every width
  constexpr bool mrc = MRC;
  // fusion of the round's weighted estimates (rows of the slots' matched
  // filters) and weights (F) by lane (g, i): symbols g, g + NSYS, ...
  auto valu_fuse = [&](int nvalid) {
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int s = g + NSYS * k;
      if (s < a.nsym) {
        for (int q = 0; q < nvalid; ++q) {
          const float2 v = sm.m(q, s, i);
          zf[k].x += v.x;
          zf[k].y += v.y;
        }
      }
    }
    for (int q = 0; q < nvalid; ++q) tk[0] += sm.F[q][i].y;
  };

  for (int base = 0; base < C; base += NSYS) {
    const int nvalid = min(NSYS, C - base);
    auto seg = [&](int s, const float2 *&Hw, const float2 *&Yw, int &r0, int &r1) {
      Hw = a.H + (size_t)w * HB;
      Yw = a.y + (size_t)w * a.ysw;
      r0 = a.off[base + s];
      r1 = a.off[base + s + 1];
    };
    gram_mf_stream<UT, PREC>(nvalid, a.U, a.B, a.nsym, seg, [&](int s, const Acc<UT> &acc, const MAcc<UT> &m) {
      store_gram<UT, PREC>(sm.A[s], acc, a.rho, a.U);
      store_msym<UT, PREC>(sm, s, m);
    });
    for (int s = nvalid; s < NSYS; ++s) store_identity<UT>(sm.A[s]);
    __syncthreads();

    const int c = base + g;
    const bool live = g < nvalid;
    if constexpr (MRC) {
      const SymMrc o = sym_mrc_row<UT>(sm, g, i, a.U, a.n0, a.es);
      if (live && i == 0 && a.info) a.info[(size_t)w * C + c] = o.bad ? -1 : o.fail;
      const bool out_nan = o.bad || o.fail;
      float p = 0.f;
      if (live && i < a.U) p = user_nu ? a.nu[((size_t)w * C + c) * a.U + i] : 1.0f / o.s2;
      const float q = p * o.inv_gii;
      for (int s = 0; s < a.nsym; ++s) {
        const float2 mv = sm.m(g, s, i);
        sm.m(g, s, i) = out_nan ? make_float2(nanv, nanv) : make_float2(q * mv.x, q * mv.y);
      }
      sm.F[g][i] = out_nan ? make_float2(nanv, nanv) : make_float2(p, user_nu ? p * p * o.s2 : p);
      __syncthreads();
      valu_fuse(nvalid);
      __syncthreads();
      continue;
    }
    SymSolve<UT> r;
    sym_factor<UT>(r, sm, g, i, a.U);
    const float kappa = r.norm1 * gsum<UT>(i < a.U ? r.d : 0.f);
    const bool routed = live && !r.bad && (r.fail != 0 || !(kappa <= EQ_COND_LIMIT));
    if (live && i == 0 && a.info) a.info[(size_t)w * C + c] = (r.bad ? -1 : r.fail) | (routed ? EQ_INFO_FP64 : 0);
    routed_any |= __ballot(routed) != 0ull;
    // local variance (of the estimate scaled to unit gain for the unbiased
    // L-MMSE: estimate and variance times ku) and fusion weight p; the
    // estimate's weight is p ku
    const float ku = unbias_factor(a.n0 * r.d, a.ub);
    const float s2c = a.n0 * r.d * ku;
    float p = 0.f;
    if (live && i < a.U) p = user_nu ? a.nu[((size_t)w * C + c) * a.U + i] : 1.0f / s2c;
    const float pz = p * ku;
    const float2 fterm = r.bad ? make_float2(nanv, nanv) : make_float2(pz, user_nu ? p * p * s2c : p);
    if constexpr (UT == 16) {
      sm.F[g][i] = fterm;
      __syncthreads();
      const int kk = lane >> 4;
      for (int q = 0; q < nvalid; ++q) {
        f4 zr, zi;
        sym_mfma16(sm, q, zr, zi);
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const float2 fv = sm.F[q][4 * kk + rr];
          zf[rr].x += fv.x * zr[rr];
          zf[rr].y += fv.x * zi[rr];
          tk[rr] += fv.y;
        }
      }
    } else {
      // weighted estimates replace the group's matched filters, row by row
      // (each row is read by the whole group before its lane i overwrites it)
      for (int s = 0; s < a.nsym; ++s) {
        const float2 z = sym_apply<UT>(r, sm, g, s);
        sm.m(g, s, i) = r.bad ? make_float2(nanv, nanv) : make_float2(pz * z.x, pz * z.y);
      }
      sm.F[g][i] = fterm;
      __syncthreads();
      valu_fuse(nvalid);
    }
    __syncthreads();
  }

  float2 *zw = a.z + (size_t)w * a.zsw;
  bool mfma_layout = false;
  if constexpr (UT == 16) mfma_layout = !mrc;
  if (mfma_layout) {
    const int kk = lane >> 4, cs = lane & 15;
#pragma unroll
    for (int rr = 0; rr < 4; ++rr) {
      const int u = 4 * kk + rr;
      const float inv = 1.0f / tk[rr];
      if (cs < a.nsym && u < a.U)
        zw[(size_t)cs * a.U + u] = user_nu ? zf[rr] : make_float2(zf[rr].x * inv, zf[rr].y * inv);
      if (cs == 0 && u < a.U && a.s2) a.s2[(size_t)w * a.U + u] = user_nu ? tk[rr] : inv;
    }
  } else if (i < a.U) {
    const float inv = 1.0f / tk[0];
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int s = g + NSYS * k;
      if (s < a.nsym) zw[(size_t)s * a.U + i] = user_nu ? zf[k] : make_float2(zf[k].x * inv, zf[k].y * inv);
    }
    if (g == 0 && a.s2) a.s2[(size_t)w * a.U + i] = user_nu ? tk[0] : inv;
  }
  if (lane == 0 && routed_any) enqueue_fp64_sym(a, w);
}

// ---------------------------------------------------------------- LAMA
// LAMA (Algorithm 1) for every receive vector of the tile: one Gram per
// subcarrier (PD) or cluster (FD), the iteration per vector.  LAMA's
// variance N0 + beta phi depends on the vector, so sigma2 is [W][S][U] here.

// Lane i of group g: f.x = conj(row i of the slot's G) * scale.
template <int UT, class SM>
__device__ __forceinline__ bool lama_load_row(Factor<UT> &f, SM &sm, int slot, int i, float scale) {
  bool bad = false;
#pragma unroll
  for (int k = 0; k < UT; ++k) {
    const float2 g = lds_el<UT>(sm.A[slot], i, k);
    bad |= !finite2(g);
    f.x[k] = make_float2(g.x * scale, -g.y * scale);
  }
  return gany<UT>(bad);
}

template <int UT, int PREC, int M, class SM>
__device__ __forceinline__ void pd_sym_lama_task(const FwdArgs &a, int w0, int nvalid, SM &sm) {
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  auto seg = [&](int s, const float2 *&Hw, const float2 *&Yw, int &r0, int &r1) {
    const size_t w = (size_t)w0 + s;
    Hw = a.H + w * HB;
    Yw = a.y + w * (size_t)a.ysw;
    r0 = 0;
    r1 = a.B;
  };
  gram_mf_stream<UT, PREC>(nvalid, a.U, a.B, a.nsym, seg, [&](int s, const Acc<UT> &acc, const MAcc<UT> &m) {
    store_gram<UT, PREC>(sm.A[s], acc, 0.f, a.U);
    store_msym<UT, PREC>(sm, s, m);
  });
  for (int s = nvalid; s < SM::NS; ++s) store_identity<UT>(sm.A[s]);
  __syncthreads();
  const int slot = slot_of<SM>(g);
  const bool live = g < nvalid;
  const int w = w0 + g;
  Factor<UT> f;
  const bool bad = lama_load_row<UT>(f, sm, slot, i, 1.0f);
  const float beta = (float)a.U / (float)a.B;
  const float nanv = __int_as_float(0x7fc00000);
  const size_t ob = (size_t)w * a.zsw;
  for (int s = 0; s < a.nsym; ++s) {
    float2 z;
    float tau;
    lama_iterate<UT, M>(f, sm.m(slot, s, i), i, a.U, a.n0, beta, a.es, a.lama_t, z, tau);
    if (live && i < a.U) {
      a.z[ob + (size_t)s * a.U + i] = bad ? make_float2(nanv, nanv) : z;
      if (a.s2) a.s2[ob + (size_t)s * a.U + i] = bad ? nanv : tau;
    }
  }
  if (live && i == 0 && a.info) a.info[w] = bad ? -1 : 0;
}

// FD: rounds of NSYS clusters.  After a cluster's iteration for vector s,
// lane (g, i) leaves nu z in the slot's matched-filter row s and (nu,
// nu^2 sigma2_c) in row s of the slot's (no longer needed) G; fusion lane
// (g, i) then sums user i of the vectors g, g + NSYS, ... over the clusters.
template <int UT, int PREC, int M, class SM>
__device__ __forceinline__ void fd_sym_lama_task(const FwdArgs &a, int w, SM &sm) {
  constexpr int NSYS = 64 / UT;
  constexpr int KS = UT / NSYS;
  const int lane = lane_id();
  const int g = lane / UT, i = lane % UT;
  const size_t HB = (size_t)a.B * a.U;
  const int C = a.C;
  const bool user_nu = a.nu != nullptr;
  const float nanv = __int_as_float(0x7fc00000);
  const float beta = (float)a.U / (float)a.B;
  float2 zf[KS];
  float swk[KS], svk[KS];
#pragma unroll
  for (int k = 0; k < KS; ++k) {
    zf[k] = make_float2(0.f, 0.f);
    swk[k] = 0.f;
    svk[k] = 0.f;
  }
  for (int base = 0; base < C; base += NSYS) {
    const int nvalid = min(NSYS, C - base);
    auto seg = [&](int s, const float2 *&Hw, const float2 *&Yw, int &r0, int &r1) {
      Hw = a.H + (size_t)w * HB;
      Yw = a.y + (size_t)w * a.ysw;
      r0 = a.off[base + s];
      r1 = a.off[base + s + 1];
    };
    gram_mf_stream<UT, PREC>(nvalid, a.U, a.B, a.nsym, seg, [&](int s, const Acc<UT> &acc, const MAcc<UT> &m) {
      store_gram<UT, PREC>(sm.A[s], acc, 0.f, a.U);
      store_msym<UT, PREC>(sm, s, m);
    });
    for (int s = nvalid; s < NSYS; ++s) store_identity<UT>(sm.A[s]);
    __syncthreads();
    const int c = base + g;
    const bool live = g < nvalid;
    const float wc = live ? (float)(a.off[c + 1] - a.off[c]) / (float)a.B : 1.0f;
    const float iw = 1.0f / wc;
    Factor<UT> f;
    const bool bad = lama_load_row<UT>(f, sm, g, i, iw);
    if (live && i == 0 && a.info) a.info[(size_t)w * C + c] = bad ? -1 : 0;
    float nu = 0.f;
    if (user_nu && live && i < a.U) nu = a.nu[((size_t)w * C + c) * a.U + i];
    __syncthreads();  // every row of G is in registers: the slots' G rows are free
    for (int s = 0; s < a.nsym; ++s) {
      const float2 mv = sm.m(g, s, i);
      float2 z;
      float tau;
      lama_iterate<UT, M>(f, make_float2(mv.x * iw, mv.y * iw), i, a.U, a.n0 * iw, beta * iw, a.es, a.lama_t, z, tau);
      const float p = (live && i < a.U) ? (user_nu ? nu : 1.0f / tau) : 0.f;
      sm.m(g, s, i) = bad ? make_float2(nanv, nanv) : make_float2(p * z.x, p * z.y);
      lds_el<UT>(sm.A[g], s, i) = bad ? make_float2(nanv, nanv) : make_float2(p, p * p * tau);
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int s = g + NSYS * k;
      if (s < a.nsym) {
        for (int q = 0; q < nvalid; ++q) {
          const float2 v = sm.m(q, s, i);
          const float2 pw = lds_el<UT>(sm.A[q], s, i);
          zf[k].x += v.x;
          zf[k].y += v.y;
          swk[k] += pw.x;
          svk[k] += pw.y;
        }
      }
    }
    __syncthreads();
  }
  if (i < a.U) {
    const size_t ob = (size_t)w * a.zsw;
#pragma unroll
    for (int k = 0; k < KS; ++k) {
      const int s = g + NSYS * k;
      if (s < a.nsym) {
        const float inv = 1.0f / swk[k];
        a.z[ob + (size_t)s * a.U + i] = user_nu ? zf[k] : make_float2(zf[k].x * inv, zf[k].y * inv);
        if (a.s2) a.s2[ob + (size_t)s * a.U + i] = user_nu ? svk[k] : inv;
      }
    }
  }
}

// PD systems per work item.
template <int UT>
constexpr int sym_pd_per() {
  return UT == 32 ? 1 : 4;
}

// One wave per workgroup, one work item per workgroup.  The LDS staging
// (about 17 KB UT = 16, 17 KB PD / 35 KB FD at UT = 32) bounds occupancy to
// two waves per SIMD or fewer, which the register target matches.
template <int UT, int PREC, bool FD, bool MRC>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void eq_symbols_kernel(const FwdArgs a) {
  __shared__ SymSmem<UT, FD ? 64 / UT : sym_pd_per<UT>()> sm;
  if constexpr (FD) {
    fd_sym_task<UT, PREC, MRC>(a, blockIdx.x, sm);
  } else {
    const int w0 = blockIdx.x * sym_pd_per<UT>();
    pd_sym_task<UT, PREC, MRC>(a, w0, min(sym_pd_per<UT>(), a.W - w0), sm);
  }
}

template <int UT, int PREC, bool FD>
static hipError_t launch_sym_one(const FwdArgs &a, hipStream_t s) {
  const int per = FD ? 1 : sym_pd_per<UT>();
  const int grid = (a.W + per - 1) / per;
  if (a.eqz == EQZ_MRC)
    hipLaunchKernelGGL((eq_symbols_kernel<UT, PREC, FD, true>), dim3(grid), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((eq_symbols_kernel<UT, PREC, FD, false>), dim3(grid), dim3(64), 0, s, a);
  return hipGetLastError();
}

template <int UT, bool FD>
static hipError_t launch_sym_prec(const FwdArgs &a, int prec, hipStream_t s) {
  return prec == PREC_FP32 ? launch_sym_one<UT, PREC_FP32, FD>(a, s) : launch_sym_one<UT, PREC_BF16X3_NR, FD>(a, s);
}

template <int UT, int PREC, bool FD, int M>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2, 8))) void eq_symbols_lama_kernel(const FwdArgs a) {
  __shared__ SymSmem<UT, FD ? 64 / UT : sym_pd_per<UT>()> sm;
  if constexpr (FD) {
    fd_sym_lama_task<UT, PREC, M>(a, blockIdx.x, sm);
  } else {
    const int w0 = blockIdx.x * sym_pd_per<UT>();
    pd_sym_lama_task<UT, PREC, M>(a, w0, min(sym_pd_per<UT>(), a.W - w0), sm);
  }
}

template <int UT, int PREC, bool FD>
static hipError_t launch_sym_lama_one(const FwdArgs &a, hipStream_t s) {
  const int per = FD ? 1 : sym_pd_per<UT>();
  const dim3 grid((a.W + per - 1) / per), block(64);
  switch (a.lama_m) {
    case 2: hipLaunchKernelGGL((eq_symbols_lama_kernel<UT, PREC, FD, 2>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((eq_symbols_lama_kernel<UT, PREC, FD, 4>), grid, block, 0, s, a); break;
    case 8: hipLaunchKernelGGL((eq_symbols_lama_kernel<UT, PREC, FD, 8>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int UT, bool FD>
static hipError_t launch_sym_lama_prec(const FwdArgs &a, int prec, hipStream_t s) {
  return prec == PREC_FP32 ? launch_sym_lama_one<UT, PREC_FP32, FD>(a, s)
                           : launch_sym_lama_one<UT, PREC_BF16X3_NR, FD>(a, s);
}

hipError_t launch_symbols_lama(const FwdArgs &a, bool fd, int prec, hipStream_t s) {
  if (prec != PREC_FP32 && prec != PREC_BF16X3_NR) return hipErrorInvalidValue;
  if (a.nsym < 1 || a.nsym > symbol_tile(a.U)) return hipErrorInvalidValue;
  const int UT = ut_for(a.U);
  if (UT == 16) return fd ? launch_sym_lama_prec<16, true>(a, prec, s) : launch_sym_lama_prec<16, false>(a, prec, s);
  return fd ? launch_sym_lama_prec<32, true>(a, prec, s) : launch_sym_lama_prec<32, false>(a, prec, s);
}

int symbol_tile(int U) { return ut_for(U); }

hipError_t launch_symbols(const FwdArgs &a, bool fd, int prec, hipStream_t s) {
  if (prec != PREC_FP32 && prec != PREC_BF16X3_NR) return hipErrorInvalidValue;
  if (a.nsym < 1 || a.nsym > symbol_tile(a.U)) return hipErrorInvalidValue;
  const int UT = ut_for(a.U);
  if (UT == 16) return fd ? launch_sym_prec<16, true>(a, prec, s) : launch_sym_prec<16, false>(a, prec, s);
  return fd ? launch_sym_prec<32, true>(a, prec, s) : launch_sym_prec<32, false>(a, prec, s);
}

}  // namespace dbpeq
