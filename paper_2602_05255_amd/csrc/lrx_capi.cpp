// C ABI of liblrx: host-side validation, buffer sizing and kernel dispatch.
// Every check here runs on the host before anything is enqueued, so the error
// paths are testable without a GPU.
#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>
#include <hip/hip_runtime.h>

#include <string.h>

#include "../../include/lrx.h"
#include "lrx_internal.hpp"

namespace lrx {

static size_t al256(size_t b) { return (b + 255) / 256 * 256; }

Layout stash_layout(const lrx_shape &s) {
    const size_t es = bulk_bytes(s.dtype);
    const int n = s.n, KM = s.k_max, K = slot_capacity(s);
    const bool pf = s.kind == LRX_PF;
    const int KA = pf ? 2 * KM : KM;
    Layout L;
    size_t off = 0;
    // C: the gathered columns (DET) or A^-1 u (PF, 2 k_max of them, the general updates)
    L.c = (uint32_t)off; off += al256((size_t)(pf ? 2 * KM : KM) * n * es);
    // R^-1 held square at the next power of two of its size (the general updates' tiles)
    int p2 = 1;
    while (p2 < (pf ? 2 * KM : KM)) p2 <<= 1;
    L.rinv = (uint32_t)off; off += al256((size_t)p2 * p2 * es);
    L.g = (uint32_t)off; off += al256((size_t)(K > 0 ? K : 1) * KA * (pf ? 1 : KM) * es);
    L.ratio = (uint32_t)off; off += al256(16);
    L.kslot = (uint32_t)off; off += al256((size_t)(K > 0 ? K : 1) * 4);
    L.ax = (uint32_t)off; off += al256(pf ? (size_t)n * es : 16);
    L.stride = (uint32_t)off;
    return L;
}

// Largest padded row length the row-streaming kernels hold in LDS.
static size_t padded_n(int n, size_t es) {
    const int per = (int)(16 / es) * 64;
    int nch = (n + per - 1) / per;
    int p2 = 1;
    while (p2 < nch) p2 <<= 1;
    return (size_t)p2 * per;
}

static int check_shape(const lrx_shape *s) {
    if (!s) return LRX_EINVAL;
    if (s->kind != LRX_DET && s->kind != LRX_PF) return LRX_EUNSUPPORTED;
    if (s->dtype < LRX_F32 || s->dtype > LRX_C128) return LRX_EUNSUPPORTED;
    if (s->walkers < 1 || s->n < 1 || s->n > LRX_MAX_N) return LRX_ESHAPE;
    if (s->delay < 0 || s->delay > LRX_MAX_DELAY) return LRX_ESHAPE;
    if (s->layout < LRX_LAYOUT_FULL || s->layout > LRX_LAYOUT_PACKED) return LRX_EUNSUPPORTED;
    // the fused and packed layouts: single-hop Pfaffian updates (fused: plain only)
    if (s->layout != LRX_LAYOUT_FULL && (s->kind != LRX_PF || s->k_max != 1)) return LRX_EUNSUPPORTED;
    if (s->layout == LRX_LAYOUT_FUSED && s->delay != 0) return LRX_EUNSUPPORTED;
    const size_t es = bulk_bytes(s->dtype);
    if (s->kind == LRX_DET) {
        if (s->k_max != 1 && s->k_max != 2 && s->k_max != 4 && s->k_max != 8) return LRX_ESHAPE;
        if (s->k_max > s->n) return LRX_ESHAPE;
        // accept kernel keeps u and C panels in LDS
        if (2 * (size_t)s->k_max * padded_n(s->n, es) * es > 65536) return LRX_EUNSUPPORTED;
        // delayed accept: u panel, R^-1, the slot products G and the staged b_tau rows in LDS
        if (s->delay > 0) {
            const size_t np = padded_n(s->n, es);
            const size_t per_row = (2 * np / 64 + s->k_max) * es;    // rows per batch as the kernel picks them
            const size_t rb = 8 * per_row <= 192 ? 8 : (4 * per_row <= 192 ? 4 : (2 * per_row <= 192 ? 2 : 1));
            if ((size_t)s->k_max * np * es + (size_t)(s->delay + 1) * s->k_max * s->k_max * es +
                    4 * 16 * rb * s->k_max * es > 65536)
                return LRX_EUNSUPPORTED;
        }
        // delayed accept: a lane owns at most 4 slot columns
        if ((size_t)s->delay * s->k_max > 256) return LRX_ESHAPE;
        // propose keeps b-slot rows I in LDS
        if ((size_t)s->k_max * s->delay * s->k_max * es > 49152) return LRX_EUNSUPPORTED;
    } else {
        if (s->n & 1) return LRX_EODD;
        // k_max > 1 serves the general k-row/k-column updates, which have no delayed form
        if (s->k_max != 1 && s->k_max != 2 && s->k_max != 4) return LRX_EUNSUPPORTED;
        if (s->k_max > 1 && s->delay > 0) return LRX_EUNSUPPORTED;
        if (s->n < 2 * s->k_max) return LRX_ESHAPE;
    }
    return LRX_OK;
}

static hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

static int hip_rc(hipError_t e) { return e == hipSuccess ? LRX_OK : LRX_EHIP; }

static StepArgs step_args(const lrx_state *st) {
    StepArgs a;
    memset(&a, 0, sizeof(a));
    a.W = st->shape.walkers;
    a.n = st->shape.n;
    a.KM = st->shape.k_max;
    a.K = slot_capacity(st->shape);
    a.tau = st->slot;
    a.layout = st->shape.layout;
    a.delay = st->shape.delay;
    a.part = st->work;
    a.aligned = ((size_t)st->shape.n * bulk_bytes(st->shape.dtype)) % 16 == 0 ? 1 : 0;
    a.inv = st->inv;
    a.fa = st->fa;
    a.fb = st->fb;
    a.stash = static_cast<uint8_t *>(st->stash);
    a.L = stash_layout(st->shape);
    a.logabs = st->logabs;
    a.phase = st->phase;
    a.flags = st->flags;
    a.mh_mode = -1;
    return a;
}

}  // namespace lrx

using namespace lrx;

extern "C" {

int lrx_version(void) { return LRX_VERSION; }

const char *lrx_strerror(int code) {
    switch (code) {
        case LRX_OK: return "ok";
        case LRX_EINVAL: return "invalid argument (null pointer, bad mode or size)";
        case LRX_EUNSUPPORTED: return "unsupported kind/dtype/rank combination";
        case LRX_ESHAPE: return "shape out of range (n, walkers, k_max or delay)";
        case LRX_ENEEDFLUSH: return "delay window full: call flush_delayed first";
        case LRX_EODD: return "Pfaffian state with odd n";
        case LRX_EHIP: return "HIP launch or runtime error";
        case LRX_EKIND: return "entry point does not match the state kind";
    }
    return "unknown error";
}

int lrx_state_sizes(const lrx_shape *shape, lrx_sizes *out) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if (!out) return LRX_EINVAL;
    const size_t W = shape->walkers, n = shape->n, K = slot_capacity(*shape), KM = shape->k_max;
    const size_t es = bulk_bytes(shape->dtype);
    const bool pf = shape->kind == LRX_PF;
    const bool packed = shape->layout == LRX_LAYOUT_PACKED;
    const size_t KA = pf ? 2 * KM : KM;
    memset(out, 0, sizeof(*out));
    out->inv = W * (packed ? pk_elems(shape->n) : n * n) * es;
    out->fa = W * K * KA * n * es;
    out->fb = pf ? W * K * KA * KA * es : W * n * K * KM * es;
    const Layout L = stash_layout(*shape);
    out->stash_stride = L.stride;
    out->stash = W * L.stride;
    out->logabs = W * 8;
    out->phase = W * wide_bytes(shape->dtype);
    out->flags = W * 4;
    out->work = factor_work_bytes(shape->kind, shape->dtype, shape->walkers, shape->n);
    // packed: the accept pass keeps its per-tile partial dots [W][tiles][2][64] in the workspace
    if (packed) out->work = std::max(out->work, W * (size_t)pk_tiles(shape->n) * 2 * LRX_PACK_TILE * es);
    return LRX_OK;
}

int lrx_validate(const lrx_state *st) {
    if (!st) return LRX_EINVAL;
    int rc = check_shape(&st->shape);
    if (rc) return rc;
    if (!st->inv || !st->stash || !st->logabs || !st->phase || !st->flags || !st->work) return LRX_EINVAL;
    if (slot_capacity(st->shape) > 0 && (!st->fa || !st->fb)) return LRX_EINVAL;
    // FULL: the delay; FUSED and PACKED with delay 0: one pending slot; PACKED with a delay: the delay
    const int max_slot = st->shape.delay > 0 ? st->shape.delay : (st->shape.layout != LRX_LAYOUT_FULL ? 1 : 0);
    if (st->slot < 0 || st->slot > max_slot) return LRX_EINVAL;
    return LRX_OK;
}

static int check_kind(const lrx_state *st, int kind) {
    int rc = lrx_validate(st);
    if (rc) return rc;
    return st->shape.kind == kind ? LRX_OK : LRX_EKIND;
}

static int factor_common(lrx_state *st, int kind, const void *src, int32_t sites, const int32_t *occ,
                         double *report, int refresh, void *stream) {
    int rc = check_kind(st, kind);
    if (rc) return rc;
    if (!src) return LRX_EINVAL;
    if (occ) {
        if (kind == LRX_DET && sites < 1) return LRX_ESHAPE;
        if (kind == LRX_PF && sites < st->shape.n) return LRX_ESHAPE;
    }
    if (refresh && st->slot != 0) return LRX_ENEEDFLUSH;     // delayed or pending updates not flushed
    FactorArgs a;
    a.kind = kind;
    a.dtype = st->shape.dtype;
    a.W = st->shape.walkers;
    a.n = st->shape.n;
    a.sites = sites;
    a.src = src;
    a.occ = occ;
    a.work = st->work;
    a.inv = st->inv;
    a.logabs = st->logabs;
    a.phase = st->phase;
    a.flags = st->flags;
    a.report = refresh ? report : nullptr;
    a.refresh = refresh;
    a.packed = st->shape.layout == LRX_LAYOUT_PACKED ? 1 : 0;
    rc = hip_rc(factor(a, as_stream(stream)));
    if (rc == LRX_OK) st->slot = 0;
    return rc;
}

int lrx_det_init_inverse(lrx_state *st, const void *phi, int32_t sites, const int32_t *occ, void *stream) {
    return factor_common(st, LRX_DET, phi, sites, occ, nullptr, 0, stream);
}

int lrx_det_refresh(lrx_state *st, const void *phi, int32_t sites, const int32_t *occ, double *report,
                    void *stream) {
    return factor_common(st, LRX_DET, phi, sites, occ, report, 1, stream);
}

int lrx_pf_init_inverse(lrx_state *st, const void *f, int32_t sites, const int32_t *occ, void *stream) {
    return factor_common(st, LRX_PF, f, sites, occ, nullptr, 0, stream);
}

int lrx_pf_refresh(lrx_state *st, const void *f, int32_t sites, const int32_t *occ, double *report,
                   void *stream) {
    return factor_common(st, LRX_PF, f, sites, occ, report, 1, stream);
}

static int build_hop_common(const lrx_state *st, int kind, const void *phi, int32_t sites, const int32_t *occ,
                            const int32_t *empty, int32_t n_empty, const int32_t *k, const int32_t *elec,
                            const int32_t *slot, void *out, void *stream) {
    int rc = check_kind(st, kind);
    if (rc) return rc;
    if (!phi || !occ || !empty || !k || !elec || !slot || !out) return LRX_EINVAL;
    if (sites < st->shape.n || n_empty < 1) return LRX_ESHAPE;
    HopArgs a;
    a.W = st->shape.walkers;
    a.n = st->shape.n;
    a.KM = st->shape.k_max;
    a.sites = sites;
    a.n_empty = n_empty;
    a.phi = phi;
    a.occ = occ;
    a.empty = empty;
    a.k = k;
    a.elec = elec;
    a.slot = slot;
    a.out = out;
    a.flags = st->flags;
    hipError_t e = kind == LRX_DET ? det_build_hop(st->shape.dtype, a, as_stream(stream))
                                   : pf_build_hop(st->shape.dtype, a, as_stream(stream));
    return hip_rc(e);
}

int lrx_det_build_hop(const lrx_state *st, const void *phi, int32_t sites, const int32_t *occ,
                      const int32_t *empty, int32_t n_empty, const int32_t *k, const int32_t *elec,
                      const int32_t *slot, void *u, void *stream) {
    return build_hop_common(st, LRX_DET, phi, sites, occ, empty, n_empty, k, elec, slot, u, stream);
}

int lrx_pf_build_hop(const lrx_state *st, const void *f, int32_t sites, const int32_t *occ,
                     const int32_t *empty, int32_t n_empty, const int32_t *k, const int32_t *elec,
                     const int32_t *slot, void *x, void *stream) {
    return build_hop_common(st, LRX_PF, f, sites, occ, empty, n_empty, k, elec, slot, x, stream);
}

int lrx_det_propose_ratio(lrx_state *st, const int32_t *k, const int32_t *rows, const void *u, void *ratio,
                          void *stream) {
    int rc = check_kind(st, LRX_DET);
    if (rc) return rc;
    if (!k || !rows || !u || !ratio) return LRX_EINVAL;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = rows;
    a.u = u;
    a.ratio = ratio;
    return hip_rc(det_propose(st->shape.dtype, a, as_stream(stream)));
}

int lrx_det_accept_update(lrx_state *st, const int32_t *k, const int32_t *rows, const void *u,
                          uint8_t *accept, void *stream) {
    int rc = check_kind(st, LRX_DET);
    if (rc) return rc;
    if (!k || !rows || !u || !accept) return LRX_EINVAL;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = rows;
    a.u = u;
    a.accept = accept;
    rc = hip_rc(det_accept(st->shape.dtype, a, as_stream(stream)));
    if (rc == LRX_OK && st->shape.delay > 0) st->slot += 1;
    return rc;
}

int lrx_det_propose_hop(lrx_state *st, const void *phi, int32_t sites, const int32_t *occ, const int32_t *empty,
                        int32_t n_empty, const int32_t *k, const int32_t *elec, const int32_t *slot, void *u,
                        void *ratio, void *stream) {
    int rc = check_kind(st, LRX_DET);
    if (rc) return rc;
    if (!phi || !occ || !empty || !k || !elec || !slot || !u || !ratio) return LRX_EINVAL;
    if (sites < st->shape.n || n_empty < 1) return LRX_ESHAPE;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = elec;
    a.u = u;
    a.ratio = ratio;
    a.hop_table = phi;
    a.sites = sites;
    a.n_empty = n_empty;
    a.occ = const_cast<int32_t *>(occ);
    a.empty = const_cast<int32_t *>(empty);
    a.slot = slot;
    return hip_rc(det_propose(st->shape.dtype, a, as_stream(stream)));
}

int lrx_det_accept_hop(lrx_state *st, const int32_t *k, const int32_t *elec, const int32_t *slot, const void *u,
                       int32_t mode, const double *u01, uint64_t seed, uint64_t counter, uint8_t *accept,
                       int32_t *occ, int32_t *empty, int32_t n_empty, void *stream) {
    int rc = check_kind(st, LRX_DET);
    if (rc) return rc;
    if (!k || !elec || !slot || !u || !accept || !occ || !empty) return LRX_EINVAL;
    if (mode != LRX_MH_UNIFORMS && mode != LRX_MH_DEVICE_RNG && mode != LRX_MH_FORCE) return LRX_EINVAL;
    if (mode == LRX_MH_UNIFORMS && !u01) return LRX_EINVAL;
    if (n_empty < 1) return LRX_ESHAPE;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = elec;
    a.u = u;
    a.accept = accept;
    a.slot = slot;
    a.occ = occ;
    a.empty = empty;
    a.n_empty = n_empty;
    a.mh_mode = mode;
    a.u01 = u01;
    a.seed = seed;
    a.counter = counter;
    rc = hip_rc(det_accept(st->shape.dtype, a, as_stream(stream)));
    if (rc == LRX_OK && st->shape.delay > 0) st->slot += 1;
    return rc;
}

int lrx_det_flush_delayed(lrx_state *st, void *stream) {
    int rc = check_kind(st, LRX_DET);
    if (rc) return rc;
    if (st->shape.delay == 0 || st->slot == 0) return LRX_OK;
    StepArgs a = step_args(st);
    rc = hip_rc(det_flush(st->shape.dtype, a, as_stream(stream)));
    if (rc == LRX_OK) st->slot = 0;
    return rc;
}

static int lowrank_check(const lrx_state *st, int32_t r, int kind) {
    int rc = check_kind(st, kind);
    if (rc) return rc;
    if (st->shape.layout != LRX_LAYOUT_FULL) return LRX_EUNSUPPORTED;
    if (kind == LRX_DET && (r < 1 || r > 8 || r > st->shape.n)) return LRX_ESHAPE;
    if (kind == LRX_PF && (r < 2 || r > 8 || (r & 1) || r > st->shape.n)) return LRX_ESHAPE;
    if (st->shape.delay > 0 && st->slot == st->shape.delay) return LRX_ENEEDFLUSH;
    const int KA = kind == LRX_PF ? 2 * st->shape.k_max : st->shape.k_max;
    const int RR = r <= 1 ? 1 : (r <= 2 ? 2 : (r <= 4 ? 4 : 8));
    if (lowrank_lds_bytes(kind, st->shape.dtype, st->shape.n, RR, st->shape.delay * KA) > 163840)
        return LRX_EUNSUPPORTED;
    return LRX_OK;
}

// Arguments shared by the forward and backward calls: the state, flushed or in
// the delayed form (its st->slot live steps of slot columns).
static LowRankArgs lowrank_args(const lrx_state *st, int32_t r, int kind) {
    LowRankArgs a;
    memset(&a, 0, sizeof(a));
    a.kind = kind;
    a.dtype = st->shape.dtype;
    a.W = st->shape.walkers;
    a.n = st->shape.n;
    a.r = r;
    a.K = st->shape.delay;
    a.KA = (kind == LRX_PF ? 2 * st->shape.k_max : st->shape.k_max) * st->shape.delay;
    a.KK = st->shape.k_max * st->shape.delay;
    a.TE = st->shape.delay > 0 ? st->slot * (kind == LRX_PF ? 2 * st->shape.k_max : st->shape.k_max) : 0;
    a.inv = st->inv;
    a.fa = st->fa;
    a.fb = st->fb;
    a.state_logabs = st->logabs;
    a.state_phase = st->phase;
    return a;
}

int lrx_det_lowrank_fwd(const lrx_state *st, int32_t r, const void *B, const void *C, void *P, void *Q,
                        void *Rinv, double *logabs, void *phase, void *stream) {
    int rc = lowrank_check(st, r, LRX_DET);
    if (rc) return rc;
    if (!B || !C || !P || !Q || !Rinv || !logabs || !phase) return LRX_EINVAL;
    LowRankArgs a = lowrank_args(st, r, LRX_DET);
    a.B = B;
    a.C = C;
    a.P = P;
    a.Q = Q;
    a.Rinv = Rinv;
    a.logabs = logabs;
    a.phase = phase;
    return hip_rc(lowrank_fwd(a, as_stream(stream)));
}

static int lowrank_work(const lrx_shape *shape, int32_t r, int32_t sites, size_t *out, int kind) {
    int rc = check_shape(shape);
    if (rc) return rc;
    if (shape->kind != kind) return LRX_EKIND;
    if (!out) return LRX_EINVAL;
    if (r < 1 || r > 8 || sites < shape->n) return LRX_ESHAPE;
    const int KA = kind == LRX_PF ? 2 * shape->k_max : shape->k_max;
    *out = lowrank_work_bytes(kind, shape->dtype, shape->walkers, shape->n, r, shape->delay * KA, sites);
    return LRX_OK;
}

int lrx_det_lowrank_work_bytes(const lrx_shape *shape, int32_t r, int32_t sites, size_t *out) {
    return lowrank_work(shape, r, sites, out, LRX_DET);
}

int lrx_pf_lowrank_work_bytes(const lrx_shape *shape, int32_t r, int32_t sites, size_t *out) {
    return lowrank_work(shape, r, sites, out, LRX_PF);
}

int lrx_det_lowrank_bwd(const lrx_state *st, int32_t r, const int32_t *occ, int32_t sites, const void *P,
                        const void *Q, const void *Rinv, const void *g, void *dphi, void *dB, void *dC,
                        void *work, size_t work_bytes, void *stream) {
    int rc = lowrank_check(st, r, LRX_DET);
    if (rc) return rc;
    if (!occ || !P || !Q || !Rinv || !g || !dphi || !dB || !dC || !work) return LRX_EINVAL;
    if (sites < st->shape.n) return LRX_ESHAPE;
    LowRankArgs a = lowrank_args(st, r, LRX_DET);
    if (work_bytes < lowrank_work_bytes(LRX_DET, a.dtype, a.W, a.n, r, a.TE, sites)) return LRX_EINVAL;
    a.sites = sites;
    a.P = const_cast<void *>(P);
    a.Q = const_cast<void *>(Q);
    a.Rinv = const_cast<void *>(Rinv);
    a.g = g;
    a.occ = occ;
    a.dphi = dphi;
    a.dB = dB;
    a.dC = dC;
    lowrank_bind_work(a, work);
    return hip_rc(lowrank_bwd(a, as_stream(stream)));
}

int lrx_pf_lowrank_fwd(const lrx_state *st, int32_t r, const void *U, void *P, void *Rinv, double *logabs,
                       void *phase, void *stream) {
    int rc = lowrank_check(st, r, LRX_PF);
    if (rc) return rc;
    if (!U || !P || !Rinv || !logabs || !phase) return LRX_EINVAL;
    LowRankArgs a = lowrank_args(st, r, LRX_PF);
    a.B = U;
    a.P = P;
    a.Rinv = Rinv;
    a.logabs = logabs;
    a.phase = phase;
    return hip_rc(lowrank_fwd(a, as_stream(stream)));
}

int lrx_pf_lowrank_bwd(const lrx_state *st, int32_t r, const int32_t *occ, int32_t sites, const void *P,
                       const void *Rinv, const void *g, void *dF, void *dU, void *work, size_t work_bytes,
                       void *stream) {
    int rc = lowrank_check(st, r, LRX_PF);
    if (rc) return rc;
    if (!occ || !P || !Rinv || !g || !dF || !dU || !work) return LRX_EINVAL;
    if (sites < st->shape.n) return LRX_ESHAPE;
    LowRankArgs a = lowrank_args(st, r, LRX_PF);
    if (work_bytes < lowrank_work_bytes(LRX_PF, a.dtype, a.W, a.n, r, a.TE, sites)) return LRX_EINVAL;
    a.sites = sites;
    a.P = const_cast<void *>(P);
    a.Rinv = const_cast<void *>(Rinv);
    a.g = g;
    a.occ = occ;
    a.dphi = dF;
    a.dB = dU;
    lowrank_bind_work(a, work);
    return hip_rc(lowrank_bwd(a, as_stream(stream)));
}

int lrx_pf_grad(const lrx_state *st, const void *g, void *dA, void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (st->shape.layout != LRX_LAYOUT_FULL) return LRX_EUNSUPPORTED;
    if (st->shape.delay > 0 && st->slot != 0) return LRX_ENEEDFLUSH;
    if (!g || !dA) return LRX_EINVAL;
    return hip_rc(pf_grad(st->shape.dtype, st->inv, g, dA, st->shape.walkers, st->shape.n, as_stream(stream)));
}

// Plain / delayed accept (lrx_pf.hip) or the fused pass of the FUSED and PACKED layouts.
static int pf_accept_common(lrx_state *st, const StepArgs &a, void *stream) {
    if (st->shape.layout != LRX_LAYOUT_FULL) {
        const int rc = hip_rc(pf_fused_accept(st->shape.dtype, a, as_stream(stream)));
        if (rc == LRX_OK) st->slot = st->shape.delay > 0 ? st->slot + 1 : 1;   // delayed packed: next slot
        return rc;
    }
    const int rc = hip_rc(pf_accept(st->shape.dtype, a, as_stream(stream)));
    if (rc == LRX_OK && st->shape.delay > 0) st->slot += 1;
    return rc;
}

int lrx_pf_propose_ratio(lrx_state *st, const int32_t *k, const int32_t *cols, const void *x, void *ratio,
                         void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (!k || !cols || !x || !ratio) return LRX_EINVAL;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = cols;
    a.u = x;
    a.ratio = ratio;
    return hip_rc(pf_propose(st->shape.dtype, a, as_stream(stream)));
}

int lrx_pf_accept_update(lrx_state *st, const int32_t *k, const int32_t *cols, const void *x,
                         uint8_t *accept, void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (!k || !cols || !x || !accept) return LRX_EINVAL;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = cols;
    a.u = x;
    a.accept = accept;
    return pf_accept_common(st, a, stream);
}

int lrx_pf_propose_hop(lrx_state *st, const void *f, int32_t sites, const int32_t *occ, const int32_t *empty,
                       int32_t n_empty, const int32_t *k, const int32_t *cols, const int32_t *slot, void *x,
                       void *ratio, void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (!f || !occ || !empty || !k || !cols || !slot || !x || !ratio) return LRX_EINVAL;
    if (sites < st->shape.n || n_empty < 1) return LRX_ESHAPE;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = cols;
    a.u = x;
    a.ratio = ratio;
    a.hop_table = f;
    a.sites = sites;
    a.n_empty = n_empty;
    a.occ = const_cast<int32_t *>(occ);
    a.empty = const_cast<int32_t *>(empty);
    a.slot = slot;
    return hip_rc(pf_propose(st->shape.dtype, a, as_stream(stream)));
}

int lrx_pf_accept_hop(lrx_state *st, const int32_t *k, const int32_t *cols, const int32_t *slot, const void *x,
                      int32_t mode, const double *u01, uint64_t seed, uint64_t counter, uint8_t *accept,
                      int32_t *occ, int32_t *empty, int32_t n_empty, void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (!k || !cols || !slot || !x || !accept || !occ || !empty) return LRX_EINVAL;
    if (mode != LRX_MH_UNIFORMS && mode != LRX_MH_DEVICE_RNG && mode != LRX_MH_FORCE) return LRX_EINVAL;
    if (mode == LRX_MH_UNIFORMS && !u01) return LRX_EINVAL;
    if (n_empty < 1) return LRX_ESHAPE;
    if (st->shape.delay > 0 && st->slot >= st->shape.delay) return LRX_ENEEDFLUSH;
    StepArgs a = step_args(st);
    a.k = k;
    a.rows = cols;
    a.u = x;
    a.accept = accept;
    a.slot = slot;
    a.occ = occ;
    a.empty = empty;
    a.n_empty = n_empty;
    a.mh_mode = mode;
    a.u01 = u01;
    a.seed = seed;
    a.counter = counter;
    return pf_accept_common(st, a, stream);
}

int lrx_pf_flush_delayed(lrx_state *st, void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (st->slot == 0) return LRX_OK;
    StepArgs a = step_args(st);
    if (st->shape.layout != LRX_LAYOUT_FULL) rc = hip_rc(pf_fused_flush(st->shape.dtype, a, as_stream(stream)));
    else rc = hip_rc(pf_flush(st->shape.dtype, a, as_stream(stream)));
    if (rc == LRX_OK) st->slot = 0;
    return rc;
}

int lrx_pf_read_inverse(const lrx_state *st, void *out, void *stream) {
    int rc = check_kind(st, LRX_PF);
    if (rc) return rc;
    if (!out) return LRX_EINVAL;
    StepArgs a = step_args(st);
    return hip_rc(pf_read_inverse(st->shape.dtype, a, out, as_stream(stream)));
}

int lrx_metropolis(const lrx_state *st, const void *ratio, const double *u01, uint64_t seed, uint64_t counter,
                   int32_t mode, uint8_t *accept, void *stream) {
    int rc = lrx_validate(st);
    if (rc) return rc;
    if (!ratio || !accept) return LRX_EINVAL;
    if (mode != LRX_MH_UNIFORMS && mode != LRX_MH_DEVICE_RNG && mode != LRX_MH_FORCE) return LRX_EINVAL;
    if (mode == LRX_MH_UNIFORMS && !u01) return LRX_EINVAL;
    return hip_rc(metropolis(st->shape.dtype, st->shape.walkers, ratio, u01, seed, counter, mode, st->flags,
                             accept, as_stream(stream)));
}

// ------------------------------------------------------------------ uneven window
static int window_check(const lrx_window_class *classes, int32_t n_classes, int64_t *walkers_total) {
    if (!classes || n_classes < 1 || n_classes > LRX_MAX_CLASSES) return LRX_EINVAL;
    int64_t total = 0;
    for (int c = 0; c < n_classes; ++c) {
        const lrx_window_class &wc = classes[c];
        if (!wc.state) return LRX_EINVAL;
        int rc = lrx_validate(wc.state);
        if (rc) return rc;
        const lrx_shape &sh = wc.state->shape;
        if (sh.kind != LRX_DET) return LRX_EKIND;
        if (sh.dtype != LRX_F32 && sh.dtype != LRX_F64) return LRX_EUNSUPPORTED;
        if (sh.delay < 1) return LRX_EUNSUPPORTED;
        if (sh.dtype != classes[0].state->shape.dtype || sh.k_max != classes[0].state->shape.k_max)
            return LRX_EUNSUPPORTED;
        if (wc.state->slot >= sh.delay) return LRX_ENEEDFLUSH;
        if (!wc.table || !wc.occ || !wc.empty || !wc.k || !wc.elec || !wc.slot || !wc.u || !wc.ratio || !wc.accept)
            return LRX_EINVAL;
        if (wc.sites < 1 || wc.n_empty < 1) return LRX_ESHAPE;
        total += sh.walkers;
    }
    if (walkers_total) *walkers_total = total;
    return LRX_OK;
}

int lrx_window_work_bytes(const lrx_window_class *classes, int32_t n_classes, size_t *out) {
    int64_t total = 0;
    int rc = window_check(classes, n_classes, &total);
    if (rc) return rc;
    if (!out) return LRX_EINVAL;
    *out = 256;
    return LRX_OK;
}

static int det_window_impl(lrx_window_class *classes, int32_t n_classes, int32_t steps, int32_t mode,
                           uint64_t seed, uint64_t counter, void *work, size_t work_bytes, int32_t grid,
                           void *stream, bool own_counters) {
    int64_t total = 0;
    int rc = window_check(classes, n_classes, &total);
    if (rc) return rc;
    if (steps < 1 || steps > LRX_MAX_WINDOW_STEPS || grid < 1 || (!own_counters && !work)) return LRX_EINVAL;
    if (!own_counters && work_bytes < sizeof(uint32_t)) return LRX_EINVAL;
    if (mode != LRX_MH_UNIFORMS && mode != LRX_MH_DEVICE_RNG && mode != LRX_MH_FORCE && mode != LRX_MH_MASK)
        return LRX_EINVAL;
    for (int c = 0; c < n_classes; ++c)
        if (mode == LRX_MH_UNIFORMS && !classes[c].u01) return LRX_EINVAL;
    WindowArgs wa;
    memset(&wa, 0, sizeof(wa));
    const int dtype = classes[0].state->shape.dtype;
    const size_t es = bulk_bytes(dtype);
    const int per = (int)(16 / es) * 64;     // elements of one 16-byte chunk per lane across a wave
    // processing order: n descending (stable in the caller's class index)
    int idx[LRX_MAX_CLASSES];
    uint32_t rng_base[LRX_MAX_CLASSES];
    uint32_t rb = 0;
    for (int c = 0; c < n_classes; ++c) {
        idx[c] = c;
        rng_base[c] = rb;                        // generator key: position in the caller's class list
        rb += (uint32_t)classes[c].state->shape.walkers;
    }
    for (int i = 1; i < n_classes; ++i)
        for (int j = i; j > 0 && classes[idx[j]].state->shape.n > classes[idx[j - 1]].state->shape.n; --j) {
            const int t = idx[j];
            idx[j] = idx[j - 1];
            idx[j - 1] = t;
        }
    size_t lds = 0;
    for (int ci = 0; ci < n_classes; ++ci) {
        const lrx_window_class &wc = classes[idx[ci]];
        const int n = wc.state->shape.n;
        WindowClass &d = wa.cls[ci];
        d.a = step_args(wc.state);
        d.a.u = wc.u;
        d.a.hop_table = wc.table;
        d.a.sites = wc.sites;
        d.a.n_empty = wc.n_empty;
        d.a.occ = wc.occ;
        d.a.empty = wc.empty;
        d.a.mh_mode = mode == LRX_MH_MASK ? -1 : mode;
        d.a.seed = seed;
        d.a.counter = counter;
        d.a.rng_base = rng_base[idx[ci]];
        int nch = 1;
        while (nch * per < n) nch <<= 1;
        d.nch = nch;
        d.k = wc.k;
        d.elec = wc.elec;
        d.slot = wc.slot;
        d.u01 = wc.u01;
        d.ratio = wc.ratio;
        d.accept = wc.accept;
        const size_t l = window_lds_bytes(dtype, wc.state->shape.k_max, wc.state->shape.delay, nch);
        lds = l > lds ? l : lds;
    }
    if (lds == 0 || lds > 160 * 1024) return LRX_EUNSUPPORTED;
    wa.n_classes = n_classes;
    wa.steps = steps;
    wa.walkers = (int)total;
    if (own_counters) {
        rc = hip_rc(window_scratch(&wa.queue));
        if (rc) return rc;
    } else {
        wa.queue = static_cast<uint32_t *>(work);
    }
    rc = hip_rc(det_window(dtype, wa, grid, lds, as_stream(stream)));
    if (rc == LRX_OK)
        for (int c = 0; c < n_classes; ++c)
            classes[c].state->slot = (classes[c].state->slot + steps) % classes[c].state->shape.delay;
    return rc;
}

int lrx_det_window(lrx_window_class *classes, int32_t n_classes, int32_t steps, int32_t mode, uint64_t seed,
                   uint64_t counter, void *work, size_t work_bytes, int32_t grid, void *stream) {
    return det_window_impl(classes, n_classes, steps, mode, seed, counter, work, work_bytes, grid, stream, false);
}

int lrx_det_window_noalloc(lrx_window_class *classes, int32_t n_classes, int32_t steps, int32_t mode,
                           uint64_t seed, uint64_t counter, int32_t grid, void *stream) {
    return det_window_impl(classes, n_classes, steps, mode, seed, counter, nullptr, 0, grid, stream, true);
}

// ------------------------------------------------------------------ general updates
static GeneralArgs general_args(lrx_state *st) {
    GeneralArgs a;
    memset(&a, 0, sizeof(a));
    const Layout L = stash_layout(st->shape);
    a.W = st->shape.walkers;
    a.n = st->shape.n;
    a.inv = st->inv;
    a.stash = static_cast<uint8_t *>(st->stash);
    a.stride = L.stride;
    a.off_c = L.c;
    a.off_rinv = L.rinv;
    a.off_ratio = L.ratio;
    a.flags = st->flags;
    a.logabs = st->logabs;
    a.phase = st->phase;
    return a;
}

static int general_check(const lrx_state *st, int kind, int32_t k1, int32_t k2) {
    int rc = check_kind(st, kind);
    if (rc) return rc;
    if (st->shape.delay != 0 || st->shape.layout != LRX_LAYOUT_FULL) return LRX_EUNSUPPORTED;   // plain form only
    if (k1 < 0 || k2 < 0 || k1 + k2 < 1 || k1 + k2 > st->shape.k_max) return LRX_ESHAPE;
    return LRX_OK;
}

int lrx_det_propose_general(lrx_state *st, int32_t kr, const int32_t *ev, const void *xu, int32_t kc,
                            const int32_t *eu, const void *xv, void *ratio, void *stream) {
    int rc = general_check(st, LRX_DET, kr, kc);
    if (rc) return rc;
    if (!ratio || (kr && (!ev || !xu)) || (kc && (!eu || !xv))) return LRX_EINVAL;
    GeneralArgs a = general_args(st);
    a.kr = kr;
    a.kc = kc;
    a.ev = ev;
    a.xu = xu;
    a.eu = eu;
    a.xv = xv;
    a.ratio = ratio;
    return hip_rc(general_update(LRX_DET, st->shape.dtype, a, true, as_stream(stream)));
}

int lrx_det_accept_general(lrx_state *st, int32_t kr, const int32_t *ev, const void *xu, int32_t kc,
                           const int32_t *eu, const void *xv, uint8_t *accept, void *stream) {
    int rc = general_check(st, LRX_DET, kr, kc);
    if (rc) return rc;
    if (!accept || (kr && (!ev || !xu)) || (kc && (!eu || !xv))) return LRX_EINVAL;
    GeneralArgs a = general_args(st);
    a.kr = kr;
    a.kc = kc;
    a.ev = ev;
    a.xu = xu;
    a.eu = eu;
    a.xv = xv;
    a.accept = accept;
    return hip_rc(general_update(LRX_DET, st->shape.dtype, a, false, as_stream(stream)));
}

int lrx_pf_propose_general(lrx_state *st, int32_t k, const int32_t *cols, const void *x, void *ratio,
                           void *stream) {
    int rc = general_check(st, LRX_PF, k, 0);
    if (rc) return rc;
    if (!cols || !x || !ratio) return LRX_EINVAL;
    GeneralArgs a = general_args(st);
    a.kr = k;
    a.ev = cols;
    a.xu = x;
    a.ratio = ratio;
    return hip_rc(general_update(LRX_PF, st->shape.dtype, a, true, as_stream(stream)));
}

int lrx_pf_accept_general(lrx_state *st, int32_t k, const int32_t *cols, const void *x, uint8_t *accept,
                          void *stream) {
    int rc = general_check(st, LRX_PF, k, 0);
    if (rc) return rc;
    if (!cols || !x || !accept) return LRX_EINVAL;
    GeneralArgs a = general_args(st);
    a.kr = k;
    a.ev = cols;
    a.xu = x;
    a.accept = accept;
    return hip_rc(general_update(LRX_PF, st->shape.dtype, a, false, as_stream(stream)));
}

// ------------------------------------------------------------------ tuning table
namespace {
struct TuneEntry {
    int32_t dtype, n, k_max;
    lrx_tune t;
};
std::mutex g_tune_mu;
std::vector<TuneEntry> g_tune;

int tune_key_ok(int32_t dtype, int32_t n, int32_t k_max) {
    if (dtype < LRX_F32 || dtype > LRX_C128) return LRX_EUNSUPPORTED;
    if (n < 1 || n > LRX_MAX_N || k_max < 1 || k_max > LRX_MAX_KMAX_DET) return LRX_ESHAPE;
    return LRX_OK;
}
}  // namespace

int lrx_autotune_store(int32_t dtype, int32_t n, int32_t k_max, const lrx_tune *t) {
    int rc = tune_key_ok(dtype, n, k_max);
    if (rc) return rc;
    if (!t) return LRX_EINVAL;
    if (t->delay < 1 || t->delay > LRX_MAX_DELAY || t->delay * k_max > 256) return LRX_EINVAL;
    if (t->rows_per_block != 0 && t->rows_per_block < 16) return LRX_EINVAL;
    if (t->wgs_per_cu < 0 || t->wgs_per_cu > 16) return LRX_EINVAL;
    if (t->window != 0 && t->window != 1) return LRX_EINVAL;
    std::lock_guard<std::mutex> lock(g_tune_mu);
    lrx_tune v = *t;
    v.tuned = 1;
    for (TuneEntry &e : g_tune)
        if (e.dtype == dtype && e.n == n && e.k_max == k_max) {
            e.t = v;
            return LRX_OK;
        }
    g_tune.push_back({dtype, n, k_max, v});
    return LRX_OK;
}

int lrx_autotune_lookup(int32_t dtype, int32_t n, int32_t k_max, lrx_tune *out) {
    int rc = tune_key_ok(dtype, n, k_max);
    if (rc) return rc;
    if (!out) return LRX_EINVAL;
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        for (const TuneEntry &e : g_tune)
            if (e.dtype == dtype && e.n == n && e.k_max == k_max) {
                *out = e.t;
                return LRX_OK;
            }
    }
    const double kbar = 0.5 * (k_max + 1);
    const double kstar = std::sqrt(2.0 * n / kbar);
    int K = 1;
    while (K * 2 <= LRX_MAX_DELAY && K * 2 * k_max <= 256 && std::fabs(std::log2(K * 2.0) - std::log2(kstar)) <
                                                                  std::fabs(std::log2((double)K) - std::log2(kstar)))
        K *= 2;
    out->delay = K;
    out->rows_per_block = 0;
    out->wgs_per_cu = 2;
    out->window = n < 512 ? 1 : 0;
    out->tuned = 0;
    out->reserved = 0;
    return LRX_OK;
}

int lrx_hop_commit(int32_t walkers, int32_t n, int32_t n_empty, int32_t k_max, const int32_t *k,
                   const int32_t *elec, const int32_t *slot, const uint8_t *accept, int32_t *occ,
                   int32_t *empty, void *stream) {
    if (walkers < 1 || n < 1 || n_empty < 1 || k_max < 1 || k_max > LRX_MAX_KMAX_DET) return LRX_ESHAPE;
    if (!k || !elec || !slot || !accept || !occ || !empty) return LRX_EINVAL;
    return hip_rc(hop_commit(walkers, n, n_empty, k_max, k, elec, slot, accept, occ, empty, as_stream(stream)));
}

}  // extern "C"
