// Private interface between the C-ABI layer (lrx_capi.cpp) and the kernel
// translation units.  Host code only; no torch types anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/lrx.h"

namespace lrx {

struct Layout {                 // byte offsets in one walker's stash
    uint32_t c, rinv, g, ratio, kslot, ax, stride;
};

// Element sizes.
inline size_t bulk_bytes(int dtype) {
    switch (dtype) {
        case LRX_F32: return 4;
        case LRX_F64: return 8;
        case LRX_C64: return 8;
        case LRX_C128: return 16;
    }
    return 0;
}
inline bool is_complex(int dtype) { return dtype == LRX_C64 || dtype == LRX_C128; }
inline size_t wide_bytes(int dtype) { return is_complex(dtype) ? 16 : 8; }

Layout stash_layout(const lrx_shape &s);

// Common argument block for the per-step kernels.
struct StepArgs {
    int W, n, KM, K, tau;
    int aligned;            // rows of inv start on 16-byte boundaries
    void *inv, *fa, *fb;
    uint8_t *stash;
    Layout L;
    const int32_t *k, *rows;
    const void *u;
    uint8_t *accept;
    double *logabs;
    void *phase;
    uint32_t *flags;
    void *ratio;
    // Optional fusions.  propose: build the hop vectors in the same launch
    // (hop_table != NULL: u = table[s'] - table[s], written to u).  accept:
    // take the Metropolis decision and commit the occupancy in the same
    // launch (mh_mode >= 0; otherwise `accept` holds the caller's decision).
    const void *hop_table;
    int sites, n_empty;
    int32_t *occ, *empty;
    const int32_t *slot;
    int mh_mode;
    const double *u01;
    uint64_t seed, counter;
    uint32_t rng_base;      // added to the walker index in the device generator's key
    int layout;             // LRX_LAYOUT_* (PF): FULL, FUSED (one pending update), PACKED
    int delay;              // the shape's delay K (K above is the slot capacity)
    void *part;             // PACKED: per-tile partial dots [W][tiles][2][64] (the init workspace)
};

struct HopArgs {
    int W, n, KM, sites, n_empty;
    const void *phi;         // wide dtype
    const int32_t *occ, *empty, *k, *elec, *slot;
    void *out;               // bulk dtype
    uint32_t *flags;
};

// Determinant kernels (lrx_det.hip, one object per bulk dtype).
#define LRX_DECL_DET(sfx)                                                    \
    hipError_t det_build_hop_##sfx(const HopArgs &a, hipStream_t s);        \
    hipError_t det_propose_##sfx(const StepArgs &a, hipStream_t s);         \
    hipError_t det_accept_##sfx(const StepArgs &a, hipStream_t s);
LRX_DECL_DET(f32)
LRX_DECL_DET(f64)
LRX_DECL_DET(c64)
LRX_DECL_DET(c128)
#undef LRX_DECL_DET

#define LRX_DISPATCH(fn, dtype, ...)                                         \
    switch (dtype) {                                                         \
        case LRX_F32: return fn##_f32(__VA_ARGS__);                          \
        case LRX_F64: return fn##_f64(__VA_ARGS__);                          \
        case LRX_C64: return fn##_c64(__VA_ARGS__);                          \
        case LRX_C128: return fn##_c128(__VA_ARGS__);                        \
    }                                                                        \
    return hipErrorInvalidValue;

inline hipError_t det_build_hop(int dtype, const HopArgs &a, hipStream_t s) { LRX_DISPATCH(det_build_hop, dtype, a, s) }
inline hipError_t det_propose(int dtype, const StepArgs &a, hipStream_t s) { LRX_DISPATCH(det_propose, dtype, a, s) }
inline hipError_t det_accept(int dtype, const StepArgs &a, hipStream_t s) { LRX_DISPATCH(det_accept, dtype, a, s) }

// Pfaffian kernels (lrx_pf.hip).
hipError_t pf_build_hop(int dtype, const HopArgs &a, hipStream_t s);
hipError_t pf_propose(int dtype, const StepArgs &a, hipStream_t s);
hipError_t pf_accept(int dtype, const StepArgs &a, hipStream_t s);

// Flush GEMMs (lrx_flush.hip).
hipError_t det_flush(int dtype, const StepArgs &a, hipStream_t s);
hipError_t pf_flush(int dtype, const StepArgs &a, hipStream_t s);

// Delayed-by-one fused plain Pfaffian update, full or packed storage (lrx_pf_fused.hip).
hipError_t pf_fused_accept(int dtype, const StepArgs &a, hipStream_t s);
hipError_t pf_fused_flush(int dtype, const StepArgs &a, hipStream_t s);
hipError_t pf_read_inverse(int dtype, const StepArgs &a, void *out, hipStream_t s);

// Packed skew storage: upper 64 x 64 tiles (I <= J) per walker.
inline int pk_tiles(int n) {
    const int nt = (n + LRX_PACK_TILE - 1) / LRX_PACK_TILE;
    return nt * (nt + 1) / 2;
}
inline size_t pk_elems(int n) { return (size_t)pk_tiles(n) * LRX_PACK_TILE * LRX_PACK_TILE; }
// Slots the state's fa / fb hold: the delay, or the pending slot(s) of the fused layouts.
inline int slot_capacity(const lrx_shape &s) {
    if (s.layout == LRX_LAYOUT_FUSED) return 2;
    if (s.layout == LRX_LAYOUT_PACKED) return s.delay > 0 ? s.delay : 1;
    return s.delay;
}

// Chain helpers (lrx_det.hip).
hipError_t metropolis(int dtype, int W, const void *ratio, const double *u01,
                      uint64_t seed, uint64_t counter, int mode,
                      const uint32_t *flags, uint8_t *accept, hipStream_t s);
hipError_t hop_commit(int W, int n, int n_empty, int KM, const int32_t *k,
                      const int32_t *elec, const int32_t *slot,
                      const uint8_t *accept, int32_t *occ, int32_t *empty,
                      hipStream_t s);

// Persistent window over an uneven batch (lrx_window.hip).
constexpr int kMaxClasses = 8;
struct WindowClass {
    StepArgs a;              // step-0 arguments; a.tau = slot at the window start
    int nch;                 // 16-byte row chunks per lane, rounded to a power of two
    const int32_t *k, *elec, *slot;   // draws [steps][W], [steps][W][KM]
    const double *u01;       // [steps][W] (uniforms mode) or NULL
    void *ratio;             // wide [steps][W]
    uint8_t *accept;         // [steps][W]
};
struct WindowArgs {
    WindowClass cls[kMaxClasses];   // in processing order: n descending
    int n_classes, steps, walkers;
    uint32_t *queue;         // work counter (cleared by the launch)
};
size_t window_lds_bytes(int dtype, int KM, int K, int nch_max);
// Device address, on the current device, of the library's own window work
// counter (LRX_NOALLOC_SCRATCH_WORDS words), looked up once per device.
hipError_t window_scratch(uint32_t **out);
hipError_t det_window(int dtype, const WindowArgs &a, int grid, size_t lds, hipStream_t s);

// General low-rank updates in the plain form (lrx_general.hip).
struct GeneralArgs {
    int W, n, kr, kc;               // DET: kr dense-row / kc dense-column tuples; PF: kr = k
    void *inv;
    uint8_t *stash;
    uint32_t stride, off_c, off_rinv, off_ratio;
    const int32_t *ev, *eu;         // DET: ev [W][kr] rows, eu [W][kc] columns; PF: ev [W][k]
    const void *xu, *xv;            // DET: xu [W][kr][n], xv [W][kc][n]; PF: xu = x [W][k][n]
    void *ratio;                    // wide [W]
    uint8_t *accept;
    uint32_t *flags;
    double *logabs;
    void *phase;
};
hipError_t general_update(int kind, int dtype, const GeneralArgs &a, bool propose, hipStream_t s);

// Init / refresh (lrx_factor.hip).
struct FactorArgs {
    int kind, dtype, W, n, sites;
    const void *src;          // phi / f (wide) or dense batch
    const int32_t *occ;       // NULL -> dense batch
    void *work;               // workspace (see factor_work_bytes)
    void *inv;                // bulk out
    double *logabs;
    void *phase;
    uint32_t *flags;
    double *report;           // refresh report [W][2] or NULL
    int refresh;              // 1 -> compare with the current state
    int packed;               // PF: inv in packed skew storage (LRX_LAYOUT_PACKED)
};
size_t factor_work_bytes(int kind, int dtype, int W, int n);
hipError_t factor(const FactorArgs &a, hipStream_t s);

// Low-rank log-determinant / log-Pfaffian and adjoints (lrx_adjoint.hip).
struct LowRankArgs {
    int kind, dtype, W, n, r, sites; // r: rank of B C^T (DET) or columns of U (PF, even)
    int TE, KK, KA, K;               // live slot columns of the delayed form (0: flushed), fb row
                                     // stride (DET), fa columns per walker, delay K
    const void *inv, *fa, *fb;       // state: M0 (DET A^-T, PF A^-1), slot panels
    const void *B, *C;               // DET: bulk [W][n][r]; PF: B = U [W][n][r]
    void *P, *Q, *Rinv;              // bulk [W][n][r], [W][n][r] (DET), [W][r][r]
    double *logabs;                  // out: log|det M| / log|pf M|
    void *phase;                     // out: wide
    const double *state_logabs;      // log|det A| / log|pf A|
    const void *state_phase;         // wide
    const void *g;                   // wide [W] cotangent
    const int32_t *occ;              // [W][n]
    void *dphi, *dB, *dC;            // DET: dPhi [sites][n], dB, dC; PF: dF [sites][sites], dU (dB)
    // workspace
    int *pos;                        // [W][sites] electron on each site (-1: empty)
    void *E, *F, *part, *Y;
    int ksplit;
};
size_t lowrank_lds_bytes(int kind, int dtype, int n, int RR, int TE);
size_t lowrank_work_bytes(int kind, int dtype, int W, int n, int r, int TE, int sites);
void lowrank_bind_work(LowRankArgs &a, void *work);
hipError_t lowrank_fwd(const LowRankArgs &a, hipStream_t s);
hipError_t lowrank_bwd(const LowRankArgs &a, hipStream_t s);
hipError_t pf_grad(int dtype, const void *M, const void *g, void *dA, int W, int n, hipStream_t s);

}  // namespace lrx
