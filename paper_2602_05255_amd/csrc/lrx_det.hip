// Slater-determinant low-rank update kernels (Sec. II of the paper).
//
// State layout: M = A^-T row-major (A^-1 column-major), so the columns of A^-1
// that a row update touches are contiguous rows of M and the Sherman-Morrison
// update is a single streaming pass over the rows of M.
//
//   build_hop : u_c = Phi[s'_c] - Phi[s_c]                         (Sec. II.B)
//   propose   : C = A_{tau-1}^-1[:, I], R = I + u^T C, r = det R   (Eqs. det_ratio, det_R)
//   accept K=0: M[q,:] -= (R^-1 (M[q,:] u)) C^T                     (Eq. det_inv)
//   accept K>0: a_tau = C, b_tau = (M_{tau-1} u) R^-T              (Eqs. det_a, det_b, Sec. II.C)
//
// All kernels are HBM-streaming; MFMA is used only by the delayed flush.
#include "lrx_det_impl.hpp"

namespace {

using namespace lrxdet;
using lrx::StepArgs;
using lrx::HopArgs;

template <class T> constexpr int dtype_code();
template <> constexpr int dtype_code<float>() { return LRX_F32; }
template <> constexpr int dtype_code<double>() { return LRX_F64; }
template <> constexpr int dtype_code<cf32>() { return LRX_C64; }
template <> constexpr int dtype_code<cf64>() { return LRX_C128; }

// ------------------------------------------------------------------ launchers
template <class T> hipError_t build_hop_t(const HopArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(det_build_hop_kernel<T>, dim3(a.W), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

// Dynamic LDS a propose work-group may take: the per-wave partials of G grow
// with the live slot columns (FP64, k_max = 8, K = 32 needs about 83 KB at four
// waves), so beyond 64 KB the kernel's limit is raised first.
constexpr size_t kProposeLdsMax = 160 * 1024 - 4096;

template <class T, int KM, int NW, int NI> hipError_t propose_t(const StepArgs &a, hipStream_t s) {
    const size_t lds = propose_lds_bytes<T, KM, NW>(a.tau);
    if (lds > kProposeLdsMax) return hipErrorInvalidValue;
    if (lds > 65536) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&det_propose_kernel<T, KM, NW, NI>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((det_propose_kernel<T, KM, NW, NI>), dim3(a.W), dim3(64 * NW), lds, s, a);
    return hipGetLastError();
}

// One wave per walker for n <= 64; otherwise four waves, each thread owning
// NI = ceil(n / 256) entries of the columns.
template <class T, int KM> hipError_t propose_n(const StepArgs &a, hipStream_t s) {
    if (a.n <= 64) return propose_t<T, KM, 1, 1>(a, s);
    const int ni4 = (a.n + 255) / 256;
    if (ni4 <= 1) return propose_t<T, KM, 4, 1>(a, s);
    if constexpr (KM * sizeof(T) <= 64) {   // larger panels imply n <= 256 (LDS rule of the C ABI)
        if (ni4 <= 2) return propose_t<T, KM, 4, 2>(a, s);
        return propose_t<T, KM, 4, 4>(a, s);   // n <= LRX_MAX_N = 1024
    }
    return hipErrorInvalidValue;
}

template <class T> hipError_t propose_k(const StepArgs &a, hipStream_t s) {
    switch (a.KM) {
        case 1: return propose_n<T, 1>(a, s);
        case 2: return propose_n<T, 2>(a, s);
        case 4: return propose_n<T, 4>(a, s);
        case 8: return propose_n<T, 8>(a, s);
    }
    return hipErrorInvalidValue;
}

template <class T, int KM, int NEL, bool D> hipError_t accept_t(const StepArgs &a, hipStream_t s) {
    // u and C panels must fit the 64 KiB the C ABI allows (lrx_state_sizes rejects larger shapes)
    if constexpr (2 * KM * NEL * LRX_WAVE * sizeof(T) > 65536) {
        return hipErrorInvalidValue;
    } else {
    constexpr int RB = rows_per_batch<T, NEL, KM>();
    // Rows per block: a height stored in the tuning table for this size class, else
    // long-lived blocks (set-up amortised over at least 128 rows) with still about
    // eight blocks per compute unit.
    const int n = a.n;
    int rpb = kWaves * RB;
    long long blocks = (long long)a.W * ((n + rpb - 1) / rpb);
    while (rpb < n && (blocks > 8 * 256 || rpb < 128)) {
        rpb *= 2;
        blocks = (long long)a.W * ((n + rpb - 1) / rpb);
    }
    lrx_tune tuned;
    if (lrx_autotune_lookup(dtype_code<T>(), n, KM, &tuned) == LRX_OK && tuned.tuned && tuned.rows_per_block >= 16)
        rpb = tuned.rows_per_block < n ? tuned.rows_per_block : n;
    const int bpw = (n + rpb - 1) / rpb;
    const size_t lds = accept_lds_bytes<T, KM, NEL, D, RB>(a.K);
    const dim3 grid((unsigned)(a.W * bpw)), block(kThreads);
    if (!D || a.K * KM <= LRX_WAVE)   // one slot column per lane
        hipLaunchKernelGGL((det_accept_kernel<T, KM, NEL, RB, 1, D>), grid, block, lds, s, a, rpb, bpw);
    else
        hipLaunchKernelGGL((det_accept_kernel<T, KM, NEL, RB, 4, D>), grid, block, lds, s, a, rpb, bpw);
    return hipGetLastError();
    }
}

template <class T, int KM, bool D> hipError_t accept_n(const StepArgs &a, hipStream_t s) {
    constexpr int V = vec16<T>();
    const int per_chunk = V * LRX_WAVE;
    const int nch = (a.n + per_chunk - 1) / per_chunk;   // n <= LRX_MAX_N = 1024
    if (nch <= 1) return accept_t<T, KM, V, D>(a, s);
    if (nch <= 2) return accept_t<T, KM, 2 * V, D>(a, s);
    if (nch <= 4) return accept_t<T, KM, 4 * V, D>(a, s);
    if constexpr (V <= 2) { if (nch <= 8) return accept_t<T, KM, 8 * V, D>(a, s); }
    if constexpr (V == 1) { if (nch <= 16) return accept_t<T, KM, 16, D>(a, s); }
    return hipErrorInvalidValue;
}

template <class T, bool D> hipError_t accept_k(const StepArgs &a, hipStream_t s) {
    switch (a.KM) {
        case 1: return accept_n<T, 1, D>(a, s);
        case 2: return accept_n<T, 2, D>(a, s);
        case 4: return accept_n<T, 4, D>(a, s);
        case 8: return accept_n<T, 8, D>(a, s);
    }
    return hipErrorInvalidValue;
}

template <class T> hipError_t accept_d(const StepArgs &a, hipStream_t s) {
    return a.K > 0 ? accept_k<T, true>(a, s) : accept_k<T, false>(a, s);
}

}  // namespace

// One object per bulk dtype (LRX_DT = 0..3, set by the build), so the four
// instantiation sets compile in parallel.  Metropolis and occupancy commit are
// dtype independent and live in the LRX_DT = 0 object.
#if !defined(LRX_DT)
#error "compile lrx_det.hip with -DLRX_DT=0..3"
#endif
#if LRX_DT == 0
using TT = float;
#define LRX_SFX(x) x##_f32
#elif LRX_DT == 1
using TT = double;
#define LRX_SFX(x) x##_f64
#elif LRX_DT == 2
using TT = cf32;
#define LRX_SFX(x) x##_c64
#else
using TT = cf64;
#define LRX_SFX(x) x##_c128
#endif

namespace lrx {

hipError_t LRX_SFX(det_build_hop)(const HopArgs &a, hipStream_t s) { return build_hop_t<TT>(a, s); }
hipError_t LRX_SFX(det_propose)(const StepArgs &a, hipStream_t s) { return propose_k<TT>(a, s); }
hipError_t LRX_SFX(det_accept)(const StepArgs &a, hipStream_t s) { return accept_d<TT>(a, s); }

#if LRX_DT == 0
hipError_t metropolis(int dtype, int W, const void *ratio, const double *u01, uint64_t seed,
                      uint64_t counter, int mode, const uint32_t *flags, uint8_t *accept, hipStream_t s) {
    dim3 grid((W + 255) / 256), block(256);
    if (is_complex(dtype))
        hipLaunchKernelGGL(metropolis_kernel<cf64>, grid, block, 0, s, W, static_cast<const cf64 *>(ratio),
                           u01, seed, counter, mode, flags, accept);
    else
        hipLaunchKernelGGL(metropolis_kernel<double>, grid, block, 0, s, W, static_cast<const double *>(ratio),
                           u01, seed, counter, mode, flags, accept);
    return hipGetLastError();
}

hipError_t hop_commit(int W, int n, int n_empty, int KM, const int32_t *k, const int32_t *elec,
                      const int32_t *slot, const uint8_t *accept, int32_t *occ, int32_t *empty,
                      hipStream_t s) {
    hipLaunchKernelGGL(hop_commit_kernel, dim3((W + 255) / 256), dim3(256), 0, s, W, n, n_empty, KM, k, elec,
                       slot, accept, occ, empty);
    return hipGetLastError();
}
#endif

}  // namespace lrx
