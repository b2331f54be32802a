/*
 * lrx.h -- C ABI of liblrx: batched low-rank updates (LRU) of determinants
 * and Pfaffians for many Markov-chain walkers on one MI355X (gfx950) GPU.
 *
 * Method: Chen & Roth, "lrux: Fast low-rank updates of determinants and
 * Pfaffians in JAX", arXiv 2602.05255.  Section references below are to that
 * paper (Sec. II = determinant, Sec. III = Pfaffian, Appendix A = Pfaffian
 * definition, properties and gradient).
 *
 * Conventions that hold for every entry point
 * -------------------------------------------
 * - Pointers named in a signature are DEVICE pointers unless the comment says
 *   "host".  The caller owns all memory: the library never allocates or frees
 *   device memory, and keeps no per-call state besides the caller's
 *   lrx_state (a host struct).
 * - `stream` is a hipStream_t (NULL = the legacy default stream).  Every call
 *   only enqueues work on it and returns without synchronising.  Calls on
 *   distinct states are thread-safe; calls on one state must be ordered by
 *   the caller (one stream).
 * - Return codes are synchronous and come from host-side validation (shape,
 *   dtype, null pointers, slot bookkeeping) or from a failed kernel launch:
 *   LRX_OK (0) or one of the LRX_E* codes.  Numerical trouble is reported per
 *   walker in st->flags (device, uint32 [W]) and never as a return code.
 * - Dense matrices are row-major, batch-contiguous ([W][rows][cols]).
 *   Complex data are interleaved (re, im) pairs of the element's real type.
 *   Complex means transpose, never conjugate transpose (Sec. II-III use the
 *   plain transpose throughout).
 * - Index base is 0.
 *
 * Per-walker state (device buffers sized by lrx_state_sizes)
 * ----------------------------------------------------------
 * inv   : DET: M = A^-T, i.e. A^-1 stored column-major, so column i of A^-1
 *         (the one a row-i update needs) is the contiguous row i of M.
 *         PF : M = A^-1 row-major, kept exactly skew-symmetric.
 *         Bulk dtype, [W][n][n].  With delay K > 0 it holds A_0^-1 of the
 *         current delay window (Sec. II.C / III.C).  LRX_LAYOUT_PACKED: the
 *         upper tiles only (see LRX_LAYOUT_* below).
 * fa    : delayed factors a_t (DET Eq. det_a, PF Eq. pf_a), stored as columns:
 *         [W][K*KA][n] with KA = k_max (DET) or 2*k_max (PF); K is the slot
 *         capacity: the delay, or 2 (FUSED) / 1 (PACKED with delay 0).
 * fb    : DET: b_t (Eq. det_b) as rows, [W][n][K*k_max];
 *         PF : R_t^-1 (2k x 2k), [W][K][2k_max][2k_max].
 * stash : per-walker scratch written by propose and read by accept
 *         (ratio, the gathered columns of A^-1, R^-1, small products).
 * logabs: double [W], log|det A| (or log|pf A|) tracked through the ratios.
 * phase : real states: double [W] (+1/-1); complex: complex double [W].
 * flags : uint32 [W], LRX_FLAG_* bits; a flagged walker's accept is a no-op
 *         until the next init/refresh clears the flags.
 * work  : init/refresh workspace (FP64 / complex128 copies of the matrices).
 */
#ifndef LRX_H
#define LRX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LRX_VERSION 2

/* Return codes. */
enum {
    LRX_OK = 0,
    LRX_EINVAL = 1,        /* null pointer, bad mode or negative size           */
    LRX_EUNSUPPORTED = 2,  /* dtype/kind/rank combination not provided          */
    LRX_ESHAPE = 3,        /* n, W, k_max or K out of range                     */
    LRX_ENEEDFLUSH = 4,    /* accept with slot == K: flush_delayed first        */
    LRX_EODD = 5,          /* Pfaffian state with odd n (pf is 0 by definition) */
    LRX_EHIP = 6,          /* a HIP launch or runtime call failed               */
    LRX_EKIND = 7          /* DET entry point on a PF state or vice versa       */
};

/* Kinds and bulk dtypes. */
enum { LRX_DET = 0, LRX_PF = 1 };
enum { LRX_F32 = 0, LRX_F64 = 1, LRX_C64 = 2, LRX_C128 = 3 };

/* Per-walker flag bits (device, st->flags). */
enum {
    LRX_FLAG_SINGULAR_R = 1u,  /* det R = 0 / pf R = 0 or non-finite: update impossible (Sec. II.A) */
    LRX_FLAG_NONFINITE = 2u,   /* non-finite ratio                                                  */
    LRX_FLAG_SINGULAR_A = 4u,  /* init/refresh met an exactly singular matrix                        */
    LRX_FLAG_BADINDEX = 8u     /* a row/column/site index outside its range (clamped, step skipped)  */
};

/* Limits. */
#define LRX_MAX_N 1024
#define LRX_MAX_KMAX_DET 8
#define LRX_MAX_KMAX_PF 4      /* k_max > 1: plain states (delay 0) for the general updates */
#define LRX_MAX_DELAY 64

/* Metropolis modes for lrx_metropolis. */
enum {
    LRX_MH_UNIFORMS = 0,  /* accept iff u01[w] < min(1, |r|^2)                      */
    LRX_MH_DEVICE_RNG = 1,/* same rule, u from a counter-based generator (seed, ctr) */
    LRX_MH_FORCE = 2,     /* accept every unflagged walker with a finite nonzero r    */
    LRX_MH_MASK = 3       /* lrx_det_window only: accept[] holds the caller's decision */
};

/*
 * Storage layouts and update schemes (lrx_shape.layout).
 *
 * LRX_LAYOUT_FULL  : inv holds the whole n x n matrix; plain (delay 0) or
 *                    delayed (delay K) updates as described above.
 * LRX_LAYOUT_FUSED : PF, delay 0, k_max 1.  The plain update of Eq. pf_inv
 *                    (k = 1) with a delay of one accepted step fused into the
 *                    next pass: the state holds M0 and at most one pending
 *                    rank-2 update (a, R^-1) per walker (the delayed form of
 *                    Eq. pf_delayed_Ainv with one slot), and an accepted step
 *                    makes ONE pass over M0 that adds the pending update to
 *                    every row (exactly skew, from the ordered index pair),
 *                    writes the row back and takes its dot with the new x in
 *                    the same pass.  HBM per accepted step: 2 n^2 elements
 *                    instead of 3 n^2.
 * LRX_LAYOUT_PACKED: PF, k_max 1, inv holding only the tiles on and above the
 *                    diagonal (skewness of A^-1, Sec. III.A): 64 x 64 row-major
 *                    tiles (I <= J) of the n x n matrix, tile (I, J) at tile
 *                    index I*nt - I*(I-1)/2 + (J - I), nt = ceil(n / 64),
 *                    element (r, c) of the tile at r * 64 + c; entries past n
 *                    are zero; diagonal tiles hold the whole (exactly skew)
 *                    64 x 64 block.  Delay 0: the fused update above on the
 *                    tiles, about n^2 elements per accepted step (read and write
 *                    of one triangle).  Delay K > 0: the delayed update of
 *                    Sec. III.C with A_0^-1 x formed from the tiles (n^2 / 2
 *                    elements read per step) and a flush that reads and writes
 *                    the stored tiles only (half the output of the full flush).
 * For FUSED states and PACKED states with delay 0, st->slot is 0 (nothing
 * pending) or 1 (slot 0 may hold each walker's pending update; a walker that
 * rejected keeps its own); accept sets it to 1, flush_delayed applies the
 * pending updates and sets it to 0.  PACKED states with a delay count slots as
 * LRX_LAYOUT_FULL ones do.  Refresh needs st->slot == 0 (LRX_ENEEDFLUSH
 * otherwise).  The low-rank, gradient and general-update entry points take
 * LRX_LAYOUT_FULL states only (LRX_EUNSUPPORTED).  lrx_pf_read_inverse returns
 * A^-1 for every layout.
 */
enum { LRX_LAYOUT_FULL = 0, LRX_LAYOUT_FUSED = 1, LRX_LAYOUT_PACKED = 2 };
#define LRX_PACK_TILE 64

/* Largest number of size classes in one lrx_det_window call. */
#define LRX_MAX_CLASSES 8

typedef struct lrx_shape {
    int32_t kind;     /* LRX_DET or LRX_PF                                    */
    int32_t dtype;    /* bulk dtype of inv/fa/fb and of the update vectors   */
    int32_t walkers;  /* W >= 1                                               */
    int32_t n;        /* matrix dimension, 1..LRX_MAX_N (PF: even)            */
    int32_t k_max;    /* largest rank per step (DET 1, 2, 4, 8; PF 1, 2, 4)    */
    int32_t delay;    /* K: 0 = plain update every step, else 1..LRX_MAX_DELAY */
    int32_t layout;   /* LRX_LAYOUT_*: storage and update scheme (PF only for
                         anything but LRX_LAYOUT_FULL)                        */
} lrx_shape;

typedef struct lrx_sizes {     /* bytes; every buffer 256-byte aligned by the caller */
    size_t inv, fa, fb, stash, logabs, phase, flags, work;
    size_t stash_stride;       /* bytes of stash per walker                   */
} lrx_sizes;

typedef struct lrx_state {
    lrx_shape shape;
    int32_t slot;     /* delay slot tau in [0, K] (the paper's current_delay,
                         Sec. II.C): accept_update writes slot `slot` and
                         increments it; flush_delayed resets it to 0.  Uniform
                         across the batch.                                     */
    int32_t reserved;
    void *inv, *fa, *fb, *stash;
    double *logabs;
    void *phase;
    uint32_t *flags;
    void *work;
} lrx_state;

/* Library version (LRX_VERSION). */
int lrx_version(void);

/* Static text for a return code (host). */
const char *lrx_strerror(int code);

/*
 * Buffer sizes for a shape (host only; no GPU needed).
 *   shape: host; out: host.  Returns LRX_ESHAPE / LRX_EUNSUPPORTED / LRX_EODD
 *   for shapes the library does not handle.
 */
int lrx_state_sizes(const lrx_shape *shape, lrx_sizes *out);

/* Host-side validation of a filled state (shape, non-null buffers, slot range). */
int lrx_validate(const lrx_state *st);

/* ------------------------------------------------------------------------ */
/* Slater determinants (Sec. II)                                            */
/* ------------------------------------------------------------------------ */

/*
 * Build A_0 and factorise it from scratch in FP64 (real states) or complex128
 * (complex states): Gauss-Jordan inversion with partial pivoting, log|det A|
 * and phase from the pivots.  Writes inv (cast to the bulk dtype), logabs,
 * phase; clears flags; sets st->slot = 0 (delay slots are always rewritten
 * before they are read, so they need no clearing).
 *   phi : [sites][n] orbital matrix (FP64 or complex128), row s = orbital
 *         values at site s.  A[w][i][:] = phi[occ[w][i]][:] (rows are electron
 *         labels).  If occ is NULL, phi is instead a dense batch [W][n][n] and
 *         A[w] = phi[w].
 *   occ : int32 [W][n] occupied site of each electron, or NULL.
 * An exactly singular A_0 sets LRX_FLAG_SINGULAR_A for that walker.
 */
int lrx_det_init_inverse(lrx_state *st, const void *phi, int32_t sites,
                         const int32_t *occ, void *stream);

/*
 * Periodic refresh (bounds the drift of reduced-precision bulk updates,
 * Sec. II.A stability remark).  Same factorisation as init_inverse on the
 * current occupancy.  Pending delayed factors must have been flushed
 * (st->slot == 0, else LRX_ENEEDFLUSH).
 *   report: double [W][2] or NULL.  report[w][0] = ||M_lru - M_new||_F /
 *           ||M_new||_F (inverse drift); report[w][1] = |log|det|_lru -
 *           log|det|_new| + |phase_lru - phase_new| (log-determinant drift).
 */
int lrx_det_refresh(lrx_state *st, const void *phi, int32_t sites,
                    const int32_t *occ, double *report, void *stream);

/*
 * Build the update vectors of one hop step (Sec. II.B rank-1 / rank-k row
 * updates): electron elec[w][c] moves from site s = occ[w][elec[w][c]] to the
 * empty site s' = empty[w][slot[w][c]], c < k[w], and
 *   u[w][c][:] = phi[s'][:] - phi[s][:]   (computed in FP64/complex128, stored in
 *                                          the bulk dtype; zero rows for c >= k[w]).
 * The row-update form is A_t = A_{t-1} + v u^T with v the one-hot selector of
 * rows elec[w][:k].
 *   phi: [sites][n] FP64/complex128; occ: int32 [W][n]; empty: int32 [W][n_empty];
 *   k: int32 [W] in 1..k_max; elec, slot: int32 [W][k_max]; u: bulk [W][k_max][n].
 */
int lrx_det_build_hop(const lrx_state *st, const void *phi, int32_t sites,
                      const int32_t *occ, const int32_t *empty, int32_t n_empty,
                      const int32_t *k, const int32_t *elec, const int32_t *slot,
                      void *u, void *stream);

/*
 * Ratio of a proposed rank-k row update (Sec. II.A Eqs. det_ratio, det_R;
 * delayed form Sec. II.C):
 *   C = A_{tau-1}^-1[:, rows]  = (rows of M0) - sum_t a_t (b_t[rows, :])^T
 *   R = I_k + u^T C,  r = det R   (k x k LU with partial pivoting).
 * Stashes C, R^-1 and r for accept_update; writes ratio (double [W] for real
 * states, complex double [W] for complex).  Reads no n x n data: the cost is
 * O(n k + tau n k) per walker.  Entries c >= k[w] of rows/u are ignored.
 *   k: int32 [W]; rows: int32 [W][k_max] distinct electron labels (the one-hot
 *   v of Sec. II.B); u: bulk [W][k_max][n].
 * det R == 0 or non-finite sets LRX_FLAG_SINGULAR_R / LRX_FLAG_NONFINITE.
 */
int lrx_det_propose_ratio(lrx_state *st, const int32_t *k, const int32_t *rows,
                          const void *u, void *ratio, void *stream);

/*
 * Apply the proposal to walkers with accept[w] != 0 (and no flag set);
 * logabs += log|r|, phase *= r/|r|.
 *   K == 0: Sherman-Morrison/Woodbury, Eq. det_inv, in one pass over the rows
 *           of M: M[q,:] -= (R^-1 (M[q,:] u)) . C^T.
 *   K  > 0: writes slot tau = st->slot: a_tau = C and
 *           b_tau = (M_{tau-1} u) R^-T  (Eqs. det_a, det_b and the a_tau/b_tau
 *           recurrences of Sec. II.C); rejected walkers get a zero slot.
 *           Then st->slot += 1.  Returns LRX_ENEEDFLUSH if st->slot == K.
 * Must follow lrx_det_propose_ratio with the same k/rows/u.
 *   accept: uint8 [W], in/out.  Walkers whose update is impossible (flagged,
 *           or a zero / non-finite ratio, Sec. II.A) are skipped and their
 *           accept byte is cleared, so a following lrx_hop_commit leaves
 *           their occupancy unchanged.
 */
int lrx_det_accept_update(lrx_state *st, const int32_t *k, const int32_t *rows,
                          const void *u, uint8_t *accept, void *stream);

/*
 * lrx_det_build_hop followed by lrx_det_propose_ratio in one launch: the hop
 * vectors u = phi[s'] - phi[s] are built inside the ratio kernel (and written
 * to u for the accept that follows).  Arguments as for the two calls; rows are
 * the electron labels elec.
 */
int lrx_det_propose_hop(lrx_state *st, const void *phi, int32_t sites,
                        const int32_t *occ, const int32_t *empty, int32_t n_empty,
                        const int32_t *k, const int32_t *elec, const int32_t *slot,
                        void *u, void *ratio, void *stream);

/*
 * lrx_metropolis, lrx_det_accept_update and lrx_hop_commit in one launch:
 * every block of a walker takes the same Metropolis decision from the stashed
 * ratio (mode LRX_MH_UNIFORMS with u01, LRX_MH_DEVICE_RNG with seed/counter,
 * or LRX_MH_FORCE), applies the update, and one block commits the occupancy.
 *   accept: uint8 [W] out (the decision actually applied).
 */
int lrx_det_accept_hop(lrx_state *st, const int32_t *k, const int32_t *elec,
                       const int32_t *slot, const void *u, int32_t mode,
                       const double *u01, uint64_t seed, uint64_t counter,
                       uint8_t *accept, int32_t *occ, int32_t *empty,
                       int32_t n_empty, void *stream);

/*
 * Flush the delay window (Eq. delayed_Ainv): M0 -= sum_{t<tau} b_t a_t^T as one
 * batched MFMA GEMM with inner dimension tau*k_max, then zero the slots and
 * set st->slot = 0.  A no-op when st->slot == 0 or K == 0.
 */
int lrx_det_flush_delayed(lrx_state *st, void *stream);

/* ------------------------------------------------------------------------ */
/* Uneven batches: one launch for a window of delayed steps                  */
/* ------------------------------------------------------------------------ */

/* Largest number of steps in one lrx_det_window call. */
#define LRX_MAX_WINDOW_STEPS 256

/* One size class of an uneven batch (all walkers of a class share n). */
typedef struct lrx_window_class {
    lrx_state *state;       /* DET state of the class: real bulk dtype, delay K >= 1;
                               st->slot is advanced by the call                     */
    const void *table;      /* device phi [sites][n], FP64                           */
    int32_t sites;
    int32_t n_empty;
    int32_t *occ, *empty;   /* device int32 [W][n], [W][n_empty]; updated on accept  */
    const int32_t *k;       /* device int32 [steps][W]: rank of each proposal        */
    const int32_t *elec;    /* device int32 [steps][W][k_max]: electrons moved       */
    const int32_t *slot;    /* device int32 [steps][W][k_max]: indices into empty    */
    const double *u01;      /* device [steps][W] uniforms (LRX_MH_UNIFORMS) or NULL  */
    void *u;                /* device bulk [W][k_max][n]: update vectors (scratch)   */
    void *ratio;            /* device double [steps][W]: ratio of every proposal     */
    uint8_t *accept;        /* device uint8 [steps][W]: decision applied (in and out
                               for LRX_MH_MASK, out otherwise)                       */
} lrx_window_class;

/* Device workspace bytes of lrx_det_window (host only): its work counter, 256-byte rounded. */
int lrx_window_work_bytes(const lrx_window_class *classes, int32_t n_classes, size_t *out);

/*
 * Advance every walker of every class by `steps` Markov-chain steps in one
 * persistent launch: per walker and step, the hop vectors u = phi[s'] - phi[s]
 * (Sec. II.B), the ratio r = det(I + u^T C) of the delayed form (Eqs. det_R,
 * det_ratio and the C recurrence of Sec. II.C), the decision (`mode`, as for
 * lrx_metropolis, or LRX_MH_MASK), the slot write a_tau = C,
 * b_tau = (M_{tau-1} u) R^-T (Eqs. det_a, det_b), the occupancy commit, and
 * whenever a class's slot reaches K the flush M0 -= sum_t b_t a_t^T
 * (Eq. delayed_Ainv) of that walker.  Results equal the sequence of per-step
 * calls (propose_hop, accept_hop, flush_delayed) up to rounding.
 * Walkers are handed out heaviest first (classes by n descending) from a work
 * counter in `work` to `grid` persistent work-groups; a work-group keeps its
 * walker for the whole window (its flush runs as 64-column MFMA strips).
 *   work: device workspace of lrx_window_work_bytes bytes (cleared by the call;
 *         calls sharing a workspace must not overlap);
 *   grid: work-groups of the persistent launch (a few per compute unit);
 *   seed, counter: generator key and step-0 counter (LRX_MH_DEVICE_RNG); the
 *   key's walker index is the walker's position in the class list (class 0
 *   first), and step t uses counter + t.
 * All classes must share the bulk dtype (FP32 or FP64) and k_max; steps is
 * 1..LRX_MAX_WINDOW_STEPS.  The refresh of each class stays a separate
 * lrx_det_refresh call.
 */
int lrx_det_window(lrx_window_class *classes, int32_t n_classes, int32_t steps,
                   int32_t mode, uint64_t seed, uint64_t counter,
                   void *work, size_t work_bytes, int32_t grid, void *stream);

/* 32-bit words of the library's own window workspace (lrx_det_window_noalloc). */
#define LRX_NOALLOC_SCRATCH_WORDS 64

/*
 * lrx_det_window for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same launch, with its work counter held by the library in a device array of
 * its own (LRX_NOALLOC_SCRATCH_WORDS 32-bit words, 256 bytes, on every GPU the
 * library runs on, kept until the process ends) instead of a caller
 * workspace; the launch needs no more than that at any batch size.  It calls
 * no allocation routine; the array's device address is looked up once per
 * device on the first call made with that device current.  The call clears
 * the counter before the launch (with a fill kernel, so it can be recorded in
 * a HIP graph), so consecutive calls need nothing in between; calls that
 * overlap on one GPU (different streams, or threads, without ordering) share
 * the array and race.  Arguments and errors as for lrx_det_window.
 */
int lrx_det_window_noalloc(lrx_window_class *classes, int32_t n_classes, int32_t steps,
                           int32_t mode, uint64_t seed, uint64_t counter, int32_t grid,
                           void *stream);

/* ------------------------------------------------------------------------ */
/* Tuning table                                                             */
/* ------------------------------------------------------------------------ */

/* Launch parameters of one (bulk dtype, n, k_max) size class. */
typedef struct lrx_tune {
    int32_t delay;          /* delay K (window length between flushes, Sec. II.C)        */
    int32_t rows_per_block; /* rows of M per work-group of the per-step accept kernels
                               (0: the library's heuristic; the accept launches use a
                               stored value >= 16)                                        */
    int32_t wgs_per_cu;     /* persistent work-groups per compute unit (0: not stored)   */
    int32_t window;         /* schedule: 1 = the persistent lrx_det_window launch,
                               0 = per-step launches (propose_hop / accept_hop / flush)   */
    int32_t tuned;          /* out: 1 = stored by lrx_autotune_store, 0 = default        */
    int32_t reserved;
} lrx_tune;

/*
 * Record measured launch parameters for a size class in the library's
 * process-wide table (host only, thread-safe; a later store replaces an
 * earlier one).  The table lives in host memory for the life of the process.
 * Returns LRX_ESHAPE / LRX_EINVAL for a bad key or values (delay 1..LRX_MAX_DELAY
 * with delay * k_max <= 256, rows_per_block >= 16 or 0, wgs_per_cu 0..16,
 * window 0 or 1).  The per-step accept launches of the library read
 * rows_per_block from this table.
 */
int lrx_autotune_store(int32_t dtype, int32_t n, int32_t k_max, const lrx_tune *t);

/*
 * Launch parameters for a size class (host only): the stored entry if there is
 * one (out->tuned = 1), otherwise the byte-model default (out->tuned = 0): the
 * delay K that minimises the bytes per step of the delayed form, the power of
 * two nearest sqrt(2 n / kbar) with kbar = (k_max + 1) / 2 (Sec. II.C moves
 * n^2 + n kbar tau bytes per accept and 2 n^2 per flush), the library's
 * accept heuristic (rows_per_block 0), two work-groups per compute unit, and
 * the persistent window below n = 512 (per-step launches from n = 512 on).
 */
int lrx_autotune_lookup(int32_t dtype, int32_t n, int32_t k_max, lrx_tune *out);

/* ------------------------------------------------------------------------ */
/* Low-rank log-determinant and its adjoint                                  */
/* ------------------------------------------------------------------------ */

/*
 * log det M_w for M_w = A_w + B_w C_w^T, with A_w^-T the state's inverse used
 * as it stands: flushed (st->slot == 0) or in the delayed form of Sec. II.C,
 * A^-T = M0 - sum_{t < slot} b_t a_t^T (Eq. delayed_Ainv), whose slot terms
 * enter P and Q through O(n slot r) products without flushing (the state is
 * the checkpoint of the forward pass; it must not change before the backward).
 * By the matrix determinant lemma (Sec. II.A with dense u = C, v = B):
 *   log det M = log det A + log det R,  R = I_r + C^T P,  P = A^-1 B,
 * computed in one pass over M0 per walker.
 *   r: rank, 1..8.  B, C: bulk [W][n][r].  P, Q (= A^-T C): bulk [W][n][r] out;
 *   Rinv: bulk [W][r][r] out; logabs: double [W] out; phase: wide [W] out
 *   (zero phase and -inf logabs when R is singular).
 * LRX_ENEEDFLUSH when the delay window is full (st->slot == K).
 */
int lrx_det_lowrank_fwd(const lrx_state *st, int32_t r, const void *B, const void *C,
                        void *P, void *Q, void *Rinv, double *logabs, void *phase,
                        void *stream);

/* Workspace bytes of lrx_det_lowrank_bwd for a shape (host only; covers any slot). */
int lrx_det_lowrank_work_bytes(const lrx_shape *shape, int32_t r, int32_t sites, size_t *out);

/*
 * Adjoint of lrx_det_lowrank_fwd (same state, same st->slot).  g: wide [W], the
 * cotangent of log det M_w in torch's convention (gradients of a real loss are
 * returned conjugate-weighted).  With M^-T = A^-T - Q R^-T P^T (Woodbury,
 * Eq. det_inv):
 *   dB   = g conj(M^-T C) = g conj(Q R^-T)          bulk [W][n][r]
 *   dC   = g conj(M^-1 B) = g conj(P R^-1)          bulk [W][n][r]
 *   dphi[s][:] = sum over (w, i) with occ[w][i] = s of g_w conj(M_w^-T[i][:])
 *                                                   bulk [sites][n] (overwritten)
 * (the gradient with respect to the orbital matrix through A_w = phi[occ_w]).
 * The first term of dphi is gathered site by site from M0; the low-rank terms
 * (Q R^-T P^T and, in the delayed form, the slot terms b_t a_t^T) form one dense
 * product on MFMA with inner dimension W (r + slot k_max).  Every sum runs in a
 * fixed order, so the results are bitwise reproducible.
 *   occ: int32 [W][n] distinct sites in 0..sites-1;
 *   work: device workspace of lrx_det_lowrank_work_bytes bytes.
 */
int lrx_det_lowrank_bwd(const lrx_state *st, int32_t r, const int32_t *occ, int32_t sites,
                        const void *P, const void *Q, const void *Rinv, const void *g,
                        void *dphi, void *dB, void *dC, void *work, size_t work_bytes,
                        void *stream);

/* ------------------------------------------------------------------------ */
/* Pfaffians (Sec. III)                                                     */
/* ------------------------------------------------------------------------ */

/*
 * Build A_0[w][i][j] = f[occ[w][i]][occ[w][j]] (or the dense skew batch f
 * [W][n][n] when occ is NULL) and factorise from scratch in FP64/complex128:
 * Parlett-Reid elimination for log|pf| and phase (Appendix A), the inverse
 * from the same factorisation (A = Pi U^T D U Pi^T with D of 2x2 blocks, so
 * A^-1 = Pi U^-1 D^-1 U^-T Pi^T), then M = (X - X^T)/2 so that M is exactly
 * skew.  A zero pivot (pf = 0) flags the walker SINGULAR_A and leaves M = 0.
 * n must be even.  The workspace grows by two n x n matrices per walker over
 * the determinant's (lrx_state_sizes).
 *   f: [sites][sites] skew pairing matrix (FP64 or complex128).
 */
int lrx_pf_init_inverse(lrx_state *st, const void *f, int32_t sites,
                        const int32_t *occ, void *stream);

/* Refresh of a Pfaffian state; report as for lrx_det_refresh. */
int lrx_pf_refresh(lrx_state *st, const void *f, int32_t sites,
                   const int32_t *occ, double *report, void *stream);

/*
 * Update vector of a single-electron hop in the Pfaffian state (Sec. III.B,
 * "update of 1 row and 1 column", Eq. pf_rank2): electron i = elec[w][0]
 * moves from s = occ[w][i] to s' = empty[w][slot[w][0]];
 *   x[w][j] = f[s'][occ[w][j]] - f[s][occ[w][j]]  (j != i),  x[w][i] = 0,
 * so that A_t = A_{t-1} - u J u^T with u = (x, e_i).  k must be 1.
 *   x: bulk [W][n].
 */
int lrx_pf_build_hop(const lrx_state *st, const void *f, int32_t sites,
                     const int32_t *occ, const int32_t *empty, int32_t n_empty,
                     const int32_t *k, const int32_t *elec, const int32_t *slot,
                     void *x, void *stream);

/*
 * Pfaffian ratio of u = (x, e_i) (Eqs. pf_ratio, pf_R with k = 1, pf J = 1):
 *   col = A_{tau-1}^-1[:, i] = -M0[i, :]^T + sum_t a_t R_t^-1 a_t[i, :]^T
 *   r   = R_12 = 1 + x . col.
 * (R_11 = x^T A^-1 x vanishes because M is exactly skew.)  Stashes col, r and
 * a_t^T x.  cols: int32 [W][k_max] (the one-hot e_i); x: bulk [W][n].
 */
int lrx_pf_propose_ratio(lrx_state *st, const int32_t *k, const int32_t *cols,
                         const void *x, void *ratio, void *stream);

/*
 * Apply accepted Pfaffian hops.
 *   K == 0: Eq. pf_inv with k = 1: a_x = M x (one pass), then
 *           M += (col a_x^T - a_x col^T) / r (second pass), exactly skew.
 *   K  > 0: slot tau: a_tau = [M_{tau-1} x, col], R_tau^-1 = [[0,-1/r],[1/r,0]]
 *           (Eq. pf_a and the a_tau recurrence of Sec. III.C, with u_tau in
 *           its first term).  Then st->slot += 1.
 * accept is in/out as for lrx_det_accept_update.
 */
int lrx_pf_accept_update(lrx_state *st, const int32_t *k, const int32_t *cols,
                         const void *x, uint8_t *accept, void *stream);

/*
 * lrx_pf_build_hop followed by lrx_pf_propose_ratio in one launch: the hop
 * vector x (Sec. III.B, Eq. pf_rank2: x_j = f[s'][occ_j] - f[s][occ_j] for
 * j != i, x_i = 0) is built inside the ratio kernel and written to x for the
 * accept that follows.  Arguments as for the two calls; cols are the electron
 * labels.
 */
int lrx_pf_propose_hop(lrx_state *st, const void *f, int32_t sites,
                       const int32_t *occ, const int32_t *empty, int32_t n_empty,
                       const int32_t *k, const int32_t *cols, const int32_t *slot,
                       void *x, void *ratio, void *stream);

/*
 * lrx_metropolis, lrx_pf_accept_update and lrx_hop_commit in one launch
 * sequence: every block of the row pass takes the same Metropolis decision
 * from the stashed ratio (mode LRX_MH_UNIFORMS with u01, LRX_MH_DEVICE_RNG
 * with seed/counter, or LRX_MH_FORCE), applies the update of
 * lrx_pf_accept_update, and one block commits the occupancy (the swap of
 * occ[w][cols[w]] and empty[w][slot[w]] for an accepted walker).
 *   slot: int32 [W][k_max] index into empty of the target site (device);
 *   accept: uint8 [W] out (the decision actually applied).
 * Errors as for lrx_pf_accept_update; LRX_EINVAL also for an unknown mode or
 * LRX_MH_UNIFORMS without u01, LRX_ESHAPE for n_empty < 1.
 */
int lrx_pf_accept_hop(lrx_state *st, const int32_t *k, const int32_t *cols,
                      const int32_t *slot, const void *x, int32_t mode,
                      const double *u01, uint64_t seed, uint64_t counter,
                      uint8_t *accept, int32_t *occ, int32_t *empty,
                      int32_t n_empty, void *stream);

/*
 * Flush (Eq. pf_delayed_Ainv): M0 += sum_t a_t R_t^-1 a_t^T on MFMA, computing
 * only tiles on and above the diagonal and writing the lower triangle as the
 * exact negative transpose, so M0 stays exactly skew.  Zeroes the slots and
 * sets st->slot = 0.
 */
int lrx_pf_flush_delayed(lrx_state *st, void *stream);

/*
 * A^-1 of every walker of a Pfaffian state in any layout, as the state stands:
 * M0 (unpacked for LRX_LAYOUT_PACKED) plus the live delayed or pending slots,
 * sum_t a_t R_t^-1 a_t^T (Eq. pf_delayed_Ainv), without changing the state.
 * Entry (q, j) is computed on the ordered pair and negated below the diagonal,
 * so the output is exactly skew.
 *   out: device, bulk dtype [W][n][n] row-major (caller-owned, written whole).
 * Errors: LRX_EINVAL (null out), LRX_EKIND (DET state).
 */
int lrx_pf_read_inverse(const lrx_state *st, void *out, void *stream);

/*
 * log pf M_w for M_w = A_w - U_w J U_w^T (Sec. III.A: the general low-rank
 * update of a skew matrix, J the 2k x 2k skew identity) with A_w^-1 the
 * Pfaffian state's inverse as it stands (flushed or in the delayed form
 * A^-1 = M0 + sum_t a_t R_t^-1 a_t^T, Eq. pf_delayed_Ainv):
 *   log pf M = log pf A + log pf R - log pf J,  R = J + U^T P,  P = A^-1 U
 * (Eqs. pf_ratio, pf_R; pf J = (-1)^(k(k-1)/2)); R is made exactly skew and its
 * Pfaffian taken by Parlett-Reid.
 *   r: columns of U (= 2k), even, 2..8.  U: bulk [W][n][r].  P: bulk [W][n][r]
 *   out; Rinv: bulk [W][r][r] out; logabs: double [W]; phase: wide [W] out.
 */
int lrx_pf_lowrank_fwd(const lrx_state *st, int32_t r, const void *U, void *P, void *Rinv,
                       double *logabs, void *phase, void *stream);

/* Workspace bytes of lrx_pf_lowrank_bwd for a shape (host only). */
int lrx_pf_lowrank_work_bytes(const lrx_shape *shape, int32_t r, int32_t sites, size_t *out);

/*
 * Adjoint of lrx_pf_lowrank_fwd.  With d log pf M / dM_ij = (1/2) (M^-1)_ji
 * (Appendix A, Eq. pf_grad) and M^-1 = A^-1 + P R^-1 P^T (Eq. pf_inv):
 *   dU = g conj(P R^-1)                              bulk [W][n][r]
 *   dF[a][b] = -(1/2) sum over walkers w with sites a = occ[w][i], b = occ[w][j]
 *              of g_w conj(M_w^-1[i][j])              bulk [sites][sites] (overwritten)
 * (the gradient with respect to the pairing matrix through A_w = F[occ_w][:, occ_w]).
 * Fixed summation order (bitwise reproducible).
 */
int lrx_pf_lowrank_bwd(const lrx_state *st, int32_t r, const int32_t *occ, int32_t sites,
                       const void *P, const void *Rinv, const void *g, void *dF, void *dU,
                       void *work, size_t work_bytes, void *stream);

/*
 * Gradient of log pf A for a flushed Pfaffian state (the standalone pf /
 * slogpf operation: lrx_pf_init_inverse of a dense skew batch, then this):
 *   dA[w][i][j] = g_w conj((1/2) (A_w^-1)_ji)   (Appendix A, Eq. pf_grad)
 *   g: wide [W] cotangent of log pf; dA: bulk [W][n][n] out.
 */
int lrx_pf_grad(const lrx_state *st, const void *g, void *dA, void *stream);

/* ------------------------------------------------------------------------ */
/* General low-rank updates (plain form: states with delay 0)               */
/* ------------------------------------------------------------------------ */

/*
 * Ratio of a general determinant update A_1 = A_0 + v u^T given as the mixed
 * dense / one-hot tuples of Sec. II.B ("Matrix updates"):
 *   u = [xu_0 .. xu_{kr-1} | e_{eu_0} .. e_{eu_{kc-1}}],
 *   v = [e_{ev_0} .. e_{ev_{kr-1}} | xv_0 .. xv_{kc-1}],
 * so row ev_c of A gains xu_c (c < kr) and column eu_e gains xv_e (e < kc): rank-kr
 * row updates (kc = 0), rank-kc column updates (kr = 0), or both at once
 * (simultaneous row + column update; a row and column that cross add both at the
 * crossing).  r = det(I_k + u^T A^-1 v), k = kr + kc <= k_max (Eqs. det_ratio,
 * det_R).  A dense v column costs one pass over the inverse (A^-1 xv); one-hot
 * entries cost O(n).  Stashes A^-1 v and R^-1 for the accept.
 *   ev: int32 [W][kr]; xu: bulk [W][kr][n]; eu: int32 [W][kc]; xv: bulk [W][kc][n];
 *   ratio: wide [W] out.  The same kr and kc for every walker.
 * States with delay > 0: LRX_EUNSUPPORTED.  An index out of range sets
 * LRX_FLAG_BADINDEX and a zero ratio.
 */
int lrx_det_propose_general(lrx_state *st, int32_t kr, const int32_t *ev, const void *xu,
                            int32_t kc, const int32_t *eu, const void *xv, void *ratio,
                            void *stream);

/*
 * Apply a general determinant update to the walkers with accept[w] != 0 (Woodbury,
 * Eq. det_inv): A_1^-T = A^-T - (A^-T u) R^-T (A^-1 v)^T in one pass over the rows
 * of the stored A^-T; logabs += log|r|, phase *= r/|r|.  Same arguments as the
 * propose; accept in/out as for lrx_det_accept_update.
 */
int lrx_det_accept_general(lrx_state *st, int32_t kr, const int32_t *ev, const void *xu,
                           int32_t kc, const int32_t *eu, const void *xv, uint8_t *accept,
                           void *stream);

/*
 * Ratio of a general Pfaffian update of k rows and k columns (Sec. III.B,
 * "update of 2 rows and 2 columns" and its k-fold form): A_1 = A_0 - u J u^T with
 *   u = [x_0 .. x_{k-1} | e_{cols_0} .. e_{cols_{k-1}}],  J the 2k x 2k skew identity,
 * r = pf(R) / pf(J), R = J + u^T A^-1 u (Eqs. pf_ratio, pf_R), 1 <= k <= k_max <= 4.
 * The dense-dense entries x_c^T A^-1 x_d need one pass over the inverse
 * (A^-1 x); R is made exactly skew and its Pfaffian taken by Parlett-Reid.
 *   cols: int32 [W][k]; x: bulk [W][k][n]; ratio: wide [W] out.
 */
int lrx_pf_propose_general(lrx_state *st, int32_t k, const int32_t *cols, const void *x,
                           void *ratio, void *stream);

/*
 * Apply a general Pfaffian update (Eq. pf_inv): A_1^-1 = A^-1 + Z R^-1 Z^T with
 * Z = A^-1 u, computed entry by entry from the ordered index pair so the inverse
 * stays exactly skew.  Same arguments as the propose.
 */
int lrx_pf_accept_general(lrx_state *st, int32_t k, const int32_t *cols, const void *x,
                          uint8_t *accept, void *stream);

/* ------------------------------------------------------------------------ */
/* Markov-chain helpers                                                     */
/* ------------------------------------------------------------------------ */

/*
 * Accept decisions from ratios (the chain's acceptance rule; the paper gives
 * none, the library uses Metropolis on |r|^2).
 *   ratio: as written by *_propose_ratio; u01: double [W] (mode
 *   LRX_MH_UNIFORMS) or NULL; seed/counter: Philox-4x32-10 key and counter
 *   (mode LRX_MH_DEVICE_RNG); accept: uint8 [W] out.  Flagged walkers, zero
 *   and non-finite ratios are always rejected.
 */
int lrx_metropolis(const lrx_state *st, const void *ratio, const double *u01,
                   uint64_t seed, uint64_t counter, int32_t mode,
                   uint8_t *accept, void *stream);

/*
 * Occupancy bookkeeping after a step: for accepted walkers and c < k[w],
 * swap occ[w][elec[w][c]] with empty[w][slot[w][c]].
 */
int lrx_hop_commit(int32_t walkers, int32_t n, int32_t n_empty, int32_t k_max,
                   const int32_t *k, const int32_t *elec, const int32_t *slot,
                   const uint8_t *accept, int32_t *occ, int32_t *empty,
                   void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LRX_H */
