/*
 * dbpeq.h -- C ABI of libdbpeq.so: decentralized feedforward L-MMSE
 * equalisation for the massive MU-MIMO uplink on AMD Instinct MI355X (gfx950).
 *
 * Problem (Section II-A, eq. (iorelation)): y = H s0 + n with H in C^{B x U}
 * perfectly known, n ~ CN(0, N0 I), symbols of energy E_s (eq. (prior)).  The
 * B antenna rows are split into C contiguous clusters (Section II-B,
 * eq. (perclusterInOutrelation)).  Every call processes W independent systems
 * ("subcarriers") that share (B, U, partition, N0).
 *
 * Memory layout (all DEVICE pointers, owned by the caller, complex values
 * interleaved re/im as in torch.complex64, row-major, no padding):
 *   H      [W][B][U]   eq_c32     system matrices; cluster c owns rows
 *                                 cluster_off[c] .. cluster_off[c+1]-1
 *   y      [W][B]      eq_c32     receive vectors
 *   z      [W][U]      eq_c32     equalised estimate (output)
 *   sigma2 [W][U]      float      post-equalisation error variance (output)
 *   nu     [W][C][U]   float      FD fusion weights (input, optional)
 *   info   PD: [W], FD: [W][C]    int32 status per system / cluster (output)
 *
 * Error behaviour.  Arguments are validated on the host before any HIP call;
 * on failure a call returns EQ_EINVAL (or EQ_ENOTSUP / EQ_EWORKSPACE) and has
 * no device side effects.  Calls are asynchronous and stream-ordered
 * (`stream` is a hipStream_t, NULL = the null stream).  Numerical trouble is
 * reported per system in `info`:
 *     0            success
 *     k > 0        leading minor k of (G + rho I) not positive definite even
 *                  after the FP64 re-solve (MRC: G_kk <= 0 for user k-1);
 *                  that system's outputs are NaN
 *    -1            a non-finite value in the system's H or y; outputs NaN
 *   | EQ_INFO_FP64 (bit 30) the system (PD) or cluster (FD) had an estimated
 *                  condition number above EQ_COND_LIMIT or a failed FP32/BF16
 *                  pivot, and its subcarrier was re-solved in FP64 on the GPU
 *                  (informational, not an error).
 * No exceptions and no global mutable state cross the ABI (except the plans,
 * their tuning cache and the device array of eq_pd_noalloc); concurrent calls
 * on different streams are safe when they use different workspaces.
 */
#ifndef DBPEQ_H
#define DBPEQ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EQ_ABI_VERSION 3
#define EQ_MAX_U 32          /* users per system */
#define EQ_MAX_B 65535       /* antennas per system */
#define EQ_MAX_C 1024        /* clusters per system */
#define EQ_MAX_SYM 1024      /* receive vectors per channel matrix (eq_*_sym) */
#define EQ_MAX_LAMA_ITER 64  /* LAMA iterations T_max */
#define EQ_INFO_FP64 (1 << 30)
#define EQ_COND_LIMIT 1.0e4f

typedef struct { float re, im; } eq_c32;   /* == one torch.complex64 element */

typedef enum {
  EQ_OK = 0,
  EQ_EINVAL = -1,      /* invalid argument (shape, pointer, partition, N0 ...) */
  EQ_ENOTSUP = -2,     /* valid but unsupported (U > EQ_MAX_U, ...)            */
  EQ_EHIP = -3,        /* a HIP runtime call failed                             */
  EQ_EWORKSPACE = -4,  /* workspace missing or smaller than eq_workspace_size   */
  EQ_ENOMEM = -5       /* plan creation could not allocate device memory        */
} eq_status;

typedef enum {
  /* Gram + matched filter in FP32 (Gram on FP32 MFMA), FP32 solves. */
  EQ_FP32 = 0,
  /* Gram on BF16 MFMA with FP32 accumulation, FP32 matched filter and solves,
     then one refinement step with the FP32 residual y - H z.  PD only: FD
     (eq_fd and FD plans) returns EQ_ENOTSUP, because its fusion weights come
     from the diagonal of the inverse of G_c + rho I, which the refinement
     step does not correct and the single-BF16 Gram leaves about 1e-3 off; FD uses
     EQ_BF16X3_REFINE, whose split-BF16 Gram gives them to FP32 accuracy. */
  EQ_BF16_REFINE = 1,
  /* As EQ_BF16_REFINE with each operand split into a BF16 high and low part
     (three BF16 products hi*hi + hi*lo + lo*hi per Gram term). */
  EQ_BF16X3_REFINE = 2,
  /* Split-BF16 Gram on BF16 MFMA with FP32 accumulation, FP32 matched filter
     and solves, no refinement pass: the Gram is accurate to a few 1e-6
     relative, which meets the FP32 error bound without a second read of H. */
  EQ_BF16X3 = 3
} eq_precision;

/* Equaliser of the forward calls (Section III-A; each FD cluster applies it
   to its own statistics, Section IV-A):
     EQ_LMMSE  z = (G + rho I)^{-1} y^MRC,  sigma2 = N0 diag((G + rho I)^{-1})
     EQ_ZF     z = G^{-1} y^MRC,            sigma2 = N0 diag(G^{-1})
               (needs B >= U for PD and every B_c >= U for FD; otherwise G is
               singular: the system fails an FP32 pivot or the condition
               check and is re-solved in FP64, and its outputs are NaN with
               the pivot in info where the FP64 factorisation fails as well)
     EQ_MRC    z = diag(G)^{-1} y^MRC,
               sigma2_u = N0 / G_uu + E_s sum_{k != u} |G_uk|^2 / G_uu^2
               (the diagonal of the Section III-A MRC variance); no
               factorisation and no FP64 re-solve; EQ_FP32 or EQ_BF16X3 only.
     EQ_LMMSE_UNBIASED
               the L-MMSE estimate scaled to unit gain (the paper defines
               only the biased one): user u's gain in the L-MMSE estimate is
               mu_u = [(G + rho I)^{-1} G]_uu = 1 - sigma2_u / E_s, and the
               outputs are z_u / mu_u and sigma2_u / mu_u (sigma2 of
               EQ_LMMSE), so that E_s / sigma2 is the unbiased SINR.  FD
               scales every cluster's estimate before the fusion, whose
               weights then come from the scaled variances.  EQ_FP32 or
               EQ_BF16X3 only: the refinement step improves z, not the
               diagonal of the inverse that gives mu.  A user with no
               channel energy in the system (FD: in one cluster) has
               mu_u = 0; its outputs (FD: the fused ones) are then not
               finite, and info reports no failure for it.
   The multi-vector calls take every equaliser; the backward calls and the
   ragged plans are L-MMSE only. */
typedef enum { EQ_LMMSE = 0, EQ_ZF = 1, EQ_MRC = 2, EQ_LMMSE_UNBIASED = 3 } eq_equalizer;

/* Shared description of a batch of W systems. */
typedef struct {
  int32_t W;                  /* systems in the batch, >= 0 (0 = no-op)          */
  int32_t B;                  /* BS antennas, 1..EQ_MAX_B                        */
  int32_t U;                  /* single-antenna users, 1..EQ_MAX_U               */
  int32_t C;                  /* clusters, 1..min(B, EQ_MAX_C)                   */
  const int32_t *cluster_off; /* HOST array of C+1 offsets,
                                 0 = off[0] < off[1] < ... < off[C] = B          */
  float n0;                   /* noise variance per complex entry, finite, > 0   */
  float es;                   /* symbol energy E_s, finite, > 0 (normally 1)     */
  int32_t precision;          /* an eq_precision value                            */
  int32_t equalizer;          /* an eq_equalizer value (0 = L-MMSE)              */
} eq_problem;

/* Bytes of device workspace the forward calls need for this problem (the
   queue of systems routed to the FP64 re-solve).  The caller allocates it
   and fills it with zeros once, before its first use; every call leaves it
   zero-filled again, so calls that share a workspace must be ordered on one
   stream.  The library never allocates device memory in eq_pd / eq_fd. */
size_t eq_workspace_size(const eq_problem *p);

/* Partially decentralised L-MMSE (Section II-C; Section III-A).
   Each cluster forms G_c = H_c^H H_c and y_c^MRC = H_c^H y_c; the adder tree
   sums them (eq. (fullMRC)); the centralised unit returns
   z = (G + rho I)^{-1} y^MRC with rho = N0/E_s and its error variance
   sigma2 = N0 diag((G + rho I)^{-1}), which is the Section III-A variance
   evaluated at rho = N0/E_s.  sigma2 and info may be NULL. */
eq_status eq_pd(const eq_problem *p, const eq_c32 *H, const eq_c32 *y,
                eq_c32 *z, float *sigma2, int32_t *info,
                void *workspace, size_t workspace_bytes, void *stream);

/* Fully decentralised L-MMSE (Section II-D; Section IV).
   Each cluster equalises locally, z_c = (G_c + rho I)^{-1} y_c^MRC and
   sigma2_c = N0 diag((G_c + rho I)^{-1}); the fusion tree returns
   z_u = sum_c nu_{c,u} z_{c,u} (eq. (fusionrule)).  With nu == NULL the
   weights are the optimal ones of Lemma 1 (eq. (opt_fusion)) and
   sigma2_u = (sum_c 1/sigma2_{c,u})^{-1} (Theorem 3); with user weights
   nu [W][C][U] they are used as given and sigma2_u = sum_c nu^2 sigma2_{c,u}.
   sigma2 and info (size [W][C]) may be NULL. */
eq_status eq_fd(const eq_problem *p, const eq_c32 *H, const eq_c32 *y,
                const float *nu, eq_c32 *z, float *sigma2, int32_t *info,
                void *workspace, size_t workspace_bytes, void *stream);

/* eq_pd without a caller workspace, for callers that cannot allocate device
   memory: code under HIP graph capture, tight serving loops, harnesses that
   forbid hipMalloc.  Arguments, results and error behaviour are those of
   eq_pd without the workspace.  The FP64 re-solve queue lives instead in a
   library-owned device array of EQ_NOALLOC_SCRATCH_BYTES bytes on each GPU
   the call runs on, held until the process ends; W above EQ_NOALLOC_MAX_W
   returns EQ_ENOTSUP before any HIP call.  The call allocates nothing: it
   clears the queue's counters with a fill kernel on `stream`, then launches
   eq_pd's kernels.  All calls on one GPU share that GPU's array, so calls
   that overlap on one GPU (other streams, other host threads) race: the
   caller orders them.  The first call on a device looks up the array's
   device address (hipGetSymbolAddress) with that device current, so make
   it outside graph capture; `stream` must belong to the current device. */
#define EQ_NOALLOC_MAX_W 262144
#define EQ_NOALLOC_SCRATCH_BYTES (256 + 4 * EQ_NOALLOC_MAX_W)
eq_status eq_pd_noalloc(const eq_problem *p, const eq_c32 *H, const eq_c32 *y,
                        eq_c32 *z, float *sigma2, int32_t *info, void *stream);

/* Several receive vectors per channel matrix (Section VI-B): the OFDM
   symbols of one coherence interval share H, so the Gram matrices, their
   factors and sigma2 are formed once per subcarrier and applied to all nsym
   receive vectors; only the matched filters are formed per vector.
   Y [W][nsym][B] (receive vector s of subcarrier w at Y + (w*nsym + s)*B),
   Z [W][nsym][U] likewise; sigma2 [W][U] and info ([W] for PD, [W][C] for
   FD) as for eq_pd / eq_fd, which these equal vector by vector (nsym = 1 is
   the single-vector problem).  nsym in 1..EQ_MAX_SYM; the vectors are
   processed in tiles of 16 (U <= 16) or 32 (U > 16), and each tile reads H
   once.  Precision EQ_FP32 or EQ_BF16X3 (the refining forms return
   EQ_ENOTSUP).  Same workspace as eq_pd / eq_fd. */
eq_status eq_pd_sym(const eq_problem *p, int32_t nsym, const eq_c32 *H,
                    const eq_c32 *Y, eq_c32 *Z, float *sigma2, int32_t *info,
                    void *workspace, size_t workspace_bytes, void *stream);
eq_status eq_fd_sym(const eq_problem *p, int32_t nsym, const eq_c32 *H,
                    const eq_c32 *Y, const float *nu, eq_c32 *Z, float *sigma2,
                    int32_t *info, void *workspace, size_t workspace_bytes,
                    void *stream);

/* LAMA-PD (Algorithm 1, Section III-C): on the PD statistics (G, y^MRC),
   starting from s = E[S] = 0, phi = E_s, v = 0, t_max iterations of
       z = y^MRC + (I - G) s + v,  tau = N0 + beta phi,  beta = U / B,
       s' = F(z, tau),  phi' = <G(z, tau)>,  v' = beta phi' / tau (z - s),
   with F, G the posterior mean and variance of eq. (F) for a square QAM of
   qam_order points (4, 16 or 64) and energy E_s.  Returns z of the last
   iteration and sigma2 = N0 + beta phi of that iteration (equal for every
   user of a system).  t_max in 1..EQ_MAX_LAMA_ITER; precision EQ_FP32 or
   EQ_BF16X3; the equalizer field is not used.  info: 0, or -1 for
   non-finite statistics (outputs NaN).  No workspace. */
eq_status eq_pd_lama(const eq_problem *p, int32_t t_max, int32_t qam_order,
                     const eq_c32 *H, const eq_c32 *y, eq_c32 *z, float *sigma2,
                     int32_t *info, void *stream);

/* LAMA-FD (Section IV): every cluster runs Algorithm 1 on its statistics
   normalised by 1/sqrt(w_c), w_c = B_c / B (proof of Lemma 2): G_c / w_c,
   y_c^MRC / w_c, noise N0 / w_c, system ratio beta / w_c; the local
   estimates are fused as in eq_fd with the variances
   sigma2_c = N0 / w_c + (beta / w_c) phi_c (or with nu [W][C][U]).
   info [W][C]. */
eq_status eq_fd_lama(const eq_problem *p, int32_t t_max, int32_t qam_order,
                     const eq_c32 *H, const eq_c32 *y, const float *nu, eq_c32 *z,
                     float *sigma2, int32_t *info, void *stream);

/* LAMA-PD / LAMA-FD over several receive vectors per channel matrix
   (Section VI-B runs LAMA over N_sc x N_sym vectors with the Gram formed once
   per subcarrier): Y [W][nsym][B], Z [W][nsym][U] as for eq_pd_sym, and
   sigma2 [W][nsym][U], since LAMA's variance N0 + beta phi depends on the
   vector.  Each vector gets what eq_pd_lama / eq_fd_lama give for it alone;
   arguments and info as there. */
eq_status eq_pd_lama_sym(const eq_problem *p, int32_t nsym, int32_t t_max,
                         int32_t qam_order, const eq_c32 *H, const eq_c32 *Y,
                         eq_c32 *Z, float *sigma2, int32_t *info, void *stream);
eq_status eq_fd_lama_sym(const eq_problem *p, int32_t nsym, int32_t t_max,
                         int32_t qam_order, const eq_c32 *H, const eq_c32 *Y,
                         const float *nu, eq_c32 *Z, float *sigma2,
                         int32_t *info, void *stream);

/* Bytes of device workspace the backward calls need. */
size_t eq_backward_workspace_size(const eq_problem *p);

/* Adjoint of eq_pd (not in the paper; derived from its forward map).  Given
   upstream gradients gz [W][U] (complex, d/dRe + i d/dIm, may be NULL = 0)
   and gs [W][U] (of sigma2, may be NULL = 0), writes
     gH [W][B][U] = (y - H z) lambda^H - H lambda z^H - 2 N0 H Q,
     gy [W][B]    = H lambda,
     gn0 (one device float) = sum_w [ -Re(z^H lambda)/E_s + sum_u gs_u d_u - N0 tr(Q)/E_s ],
   with lambda = A^{-1} gz, Q = A^{-1} diag(gs) A^{-1}, d = diag(A^{-1}),
   A = G + rho I, all recomputed from H, y (FP32; `precision` is ignored).
   gH, gy, gn0 may each be NULL to skip that output. */
eq_status eq_pd_backward(const eq_problem *p, const eq_c32 *H, const eq_c32 *y,
                         const eq_c32 *gz, const float *gs,
                         eq_c32 *gH, eq_c32 *gy, float *gn0,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Adjoint of eq_fd.  The per-cluster maps are differentiated as in
   eq_pd_backward with upstream gradients g_{z_c} = nu_c * gz and g_{sigma2_c}
   from the fusion rule; with optimal weights the dependence of nu on sigma2_c
   is included.  gnu [W][C][U] (may be NULL) receives dL/dnu when nu is given
   (it must be NULL when nu is NULL). */
eq_status eq_fd_backward(const eq_problem *p, const eq_c32 *H, const eq_c32 *y,
                         const float *nu, const eq_c32 *gz, const float *gs,
                         eq_c32 *gH, eq_c32 *gy, float *gn0, float *gnu,
                         void *workspace, size_t workspace_bytes, void *stream);

/* ---- Ragged batches: thousands of independent systems of uneven shape ---- */

/* One system of a ragged batch.  Offsets are in ELEMENTS of the pools given
   to eq_plan_execute: H at Hpool + h_off ([B][U] row-major), y at ypool + y_off
   ([B]), z / sigma2 at zpool / s2pool + z_off ([U]).  Its C cluster sizes are
   cluster_sizes[clus_first .. clus_first + C - 1] (they must sum to B). */
typedef struct {
  int64_t h_off, y_off, z_off;
  int32_t B, U, C, clus_first;
  float n0;
  int32_t _reserved;
} eq_sys;

typedef struct eq_plan eq_plan;

/* Validates the descriptors and builds the plan's work items, all run by
   one persistent launch: PD rounds of up to 64/UT whole systems of equal U
   (UT = 16 or 32, the tile class), PD row pieces of the systems longer than
   the class's piece rows (each piece's partial Gram goes to a plan-owned
   slot; the last piece of a system sums them in piece order and solves), FD
   rounds of up to 64/UT clusters of equal U (each cluster's fusion terms go
   to a slot; the last cluster of a system fuses them in cluster order).
   Results do not depend on the launch shape beyond the rounding of those
   sums.  The launch shape (waves per CU; piece rows per class) comes from
   the autotune cache (`tune_cache_path`, NULL = the DBPEQ_TUNE_CACHE
   environment variable, else no cache), whose entries are keyed by device,
   mode, precision and, for the piece rows, tile class, so that any batch of
   the same classes reuses them.  fd selects FD (1) or PD (0).  The plan owns
   its device memory (descriptor table, items, slots); EQ_ENOMEM if it cannot
   be allocated. */
eq_status eq_plan_create(eq_plan **out, const eq_sys *host_desc, int32_t nsys,
                         const int32_t *host_cluster_sizes, int32_t n_cluster_sizes,
                         int32_t fd, int32_t precision, float es,
                         const char *tune_cache_path);

/* Equalises every system of the plan: z, sigma2 (may be NULL) and info
   ([nsys], may be NULL).  The first call on a plan autotunes what the cache
   has no entry for (timing the launch on these pools, which it overwrites
   as a normal call would) and captures the launch into a hipGraph; later
   calls with the same pools replay the graph.  Stream-ordered, except that
   a call with other pools first waits on the host for the plan's previous
   launch to finish before it replaces the graph.  Calls on one plan share
   its queue counters and slots (each call leaves them as the next expects),
   so calls on different streams must be ordered by the caller. */
eq_status eq_plan_execute(eq_plan *plan, const eq_c32 *Hpool, const eq_c32 *ypool,
                          eq_c32 *zpool, float *s2pool, int32_t *info, void *stream);

/* Launch shape of the plan, per tile class k (EQ_PLAN_CLASSES of them: the
   padded user count 16, 32), in out_shape[5k .. 5k+4] (out_shape holds
   5 * EQ_PLAN_CLASSES entries, may be NULL): systems of the class, work
   items, PD row pieces (FD: clusters), PD piece rows (0 = systems are not
   cut; always 0 for FD and the refining forms), persistent waves of the
   launch.  *out_tasks (may be NULL) = work items of all classes. */
#define EQ_PLAN_CLASSES 2
eq_status eq_plan_describe(const eq_plan *plan, int32_t *out_shape, int32_t *out_tasks);

/* Waits on the host for the plan's last launch, then frees the plan and
   every device buffer, stream and graph it holds (a null plan is a no-op).
   The plan is gone on return either way; EQ_EHIP reports that one of the
   releases failed. */
eq_status eq_plan_destroy(eq_plan *plan);

/* Measurement aid, not part of the equaliser: the device time of the main
   kernel of the forward calls.  eq_kernel_timer_start creates `capacity`
   pairs of HIP events (1 .. EQ_KERNEL_TIMER_MAX; EQ_EINVAL if the timer is
   already on).  Until eq_kernel_timer_stop, each eq_pd / eq_fd /
   eq_pd_noalloc call (any equaliser) records one pair on its stream, around
   its Gram + solve (+ fusion) launch and without the FP64 re-solve launch,
   while pairs remain; the calls allocate nothing for it.  eq_kernel_timer_stop
   waits for the recorded events, writes the number of recorded pairs and the
   sum of their elapsed times (ms), and destroys the events (EQ_EINVAL if the
   timer is off).  Not for calls under stream capture, and start / stop must
   not overlap forward calls made on other host threads. */
#define EQ_KERNEL_TIMER_MAX 65536
eq_status eq_kernel_timer_start(int32_t capacity);
eq_status eq_kernel_timer_stop(int32_t *count, double *total_ms);

const char *eq_status_string(eq_status s);
int32_t eq_abi_version(void);

/* Measurement aid, not part of the equaliser: reads the `bytes` bytes (a
   multiple of 16; device pointer aligned to 16) at `buf` once, one wave per
   64 KiB of consecutive bytes with 8-byte nontemporal loads (the access
   pattern of the equaliser's streams), and may write one float to the
   device pointer `sink`.  bytes / (time of the call on `stream`) is the
   practical HBM read ceiling against which the equaliser's streams are
   compared.  bytes == 0 is a no-op; bad arguments give EQ_EINVAL. */
eq_status eq_probe_read(const void *buf, size_t bytes, float *sink, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* DBPEQ_H */
