// Delayed-update flush: a batched GEMM with a tiny inner dimension on MFMA.
//
//   DET (Eq. delayed_Ainv):     M0 -= B A^T,  B = [b_1 .. b_tau] rows  (fb, [n][K*KM])
//                                              A = [a_1 .. a_tau] cols  (fa, [K*KM][n])
//   PF  (Eq. pf_delayed_Ainv):  M0 += sum_t (a_t R_t^-1) a_t^T,  fa = [2K][n], fb = R_t^-1 [K][2][2]
//
// Work-group = 4 waves; each wave owns 16 rows x 64 columns of a 64 x 64
// output tile as four 16x16 MFMA blocks (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32,
// one 16x4 A and one 4x16 B fragment per lane-step).  Complex products use four
// real MFMAs.  The accumulator starts from the M0 tile, so M0 is read and
// written exactly once.  Blocks of one walker are kept on one XCD.
//
// DET: the contraction runs over the live slot columns only (columns c < k_t
// of each accepted step t); rejected steps and rank padding are skipped.
//
// PF: only tiles on or above the diagonal are computed; every upper entry is
// written together with its exact negative at the transposed position, so M0
// stays exactly skew-symmetric (and the diagonal stays exactly zero).
#include "lrx_flush_impl.hpp"

namespace {

using namespace lrxfl;
using lrx::StepArgs;

// ------------------------------------------------------------------ DET
// Complex data: one 64 x 64 tile per work-group (det_flush_tile).
template <class T>
__global__ __launch_bounds__(256) void det_flush_kernel(StepArgs a, int tiles_per_dim) {
    __shared__ __align__(16) unsigned char s_mem[FlushLds<T>::bytes];
    __shared__ int s_live[LRX_MAX_DELAY * LRX_MAX_KMAX_DET];
    __shared__ int s_nl;
    const int n = a.n, KK = a.K * a.KM;
    const int tiles = tiles_per_dim * tiles_per_dim;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / tiles;
    if (w >= a.W) return;
    const int tile = lb - w * tiles;
    const int ti = tile / tiles_per_dim, tj = tile - ti * tiles_per_dim;
    const int *kslot = reinterpret_cast<const int *>(a.stash + (size_t)w * a.L.stride + a.L.kslot);
    const int nl = det_live_columns(kslot, a.tau, a.KM, s_live, &s_nl);
    T *s_b = reinterpret_cast<T *>(s_mem);
    T *s_a = s_b + 64 * FlushLds<T>::SB;
    det_flush_tile<T>(static_cast<T *>(a.inv) + (size_t)w * n * n, static_cast<const T *>(a.fa) + (size_t)w * KK * n,
                      static_cast<const T *>(a.fb) + (size_t)w * n * KK, n, KK, s_live, nl, ti * 64, tj * 64, s_b,
                      s_a);
}

// Real data: one 64-column strip per work-group (det_flush_strip).
template <class T>
__global__ __launch_bounds__(256, 2) void det_flush_strip_kernel(StepArgs a, int tpd) {
    __shared__ __align__(16) T s_a[FlushStripLds<T>::kA];
    __shared__ int s_live[LRX_MAX_DELAY * LRX_MAX_KMAX_DET];
    __shared__ int s_nl;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / tpd;
    if (w >= a.W) return;
    det_flush_strip<T>(a, w, (int)(lb - w * tpd), tpd, s_a, s_live, &s_nl);
}

// ------------------------------------------------------------------ PF
// KAC: the slot width 2 k_max when known at compile time (2: single hops, the
// only width a delayed Pfaffian state has), 0 for a runtime width.  Offsets
// are 32-bit from the walker's base pointers (n^2 and K 2k_max n fit).
template <class T, int KAC>
__global__ __launch_bounds__(256) void pf_flush_kernel(StepArgs a, int tiles_per_dim) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    const int n = a.n, KA = KAC > 0 ? KAC : 2 * a.KM, TE = a.tau * KA;
    const int pairs = tiles_per_dim * (tiles_per_dim + 1) / 2;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / pairs;
    if (w >= a.W) return;
    int p = lb - w * pairs;
    // Map the pair index to (ti <= tj), row-major over the upper triangle.
    int ti = 0;
    while (p >= tiles_per_dim - ti) { p -= tiles_per_dim - ti; ++ti; }
    const int tj = ti + p;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int qa = ti * 64 + wv * 16 + (lane & 15);
    const int kq = lane >> 4;
    const int j0 = tj * 64;
    const uint32_t un = (uint32_t)n;

    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * (size_t)a.K * KA * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * (size_t)a.K * KA * KA;

    A4 re[4], im[4];
    const int rbase = ti * 64 + wv * 16;
    uint32_t jc[4];
    bool jin[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
        jin[jb] = j < n;
        jc[jb] = (uint32_t)min(j, n - 1);
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            const T x = M[(uint32_t)min(q, n - 1) * un + jc[jb]];
            const T v = (q < n && j < n && q < j) ? x : zero<T>();
            re[jb][r] = re_(v);
            im[jb][r] = im_(v);
        }
    }
    // Four 4-deep steps per batch, every load of the batch issued before its
    // MFMAs; loads come from clamped addresses and are masked by selects.
    const uint32_t qc = (uint32_t)min(qa, n - 1);
    const bool qin = qa < n;
    for (int te0 = 0; te0 < TE; te0 += 16) {
        T at[4], bv[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int te = te0 + 4 * u + kq;
            const bool tin = te < TE;
            const int tc = min(te, TE - 1);
            const int t = tc / KA, sp = tc - t * KA;
            // Atilde[q][te] = sum_s a_t[q][s] R_t^-1[s][te mod KA]
            T x = zero<T>();
#pragma unroll
            for (int s = 0; s < (KAC > 0 ? KAC : 1); ++s)
                x = fmac(fa[(uint32_t)(t * KA + s) * un + qc], rinv[(uint32_t)(t * KA * KA + s * KA + sp)], x);
            if constexpr (KAC == 0)
                for (int s = 1; s < KA; ++s)
                    x = fmac(fa[(uint32_t)(t * KA + s) * un + qc], rinv[(uint32_t)(t * KA * KA + s * KA + sp)], x);
            at[u] = (tin && qin) ? x : zero<T>();
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const T y = fa[(uint32_t)tc * un + jc[jb]];
                bv[u][jb] = (tin && jin[jb]) ? y : zero<T>();
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) mac<T>(at[u], bv[u][jb], re[jb], im[jb]);
    }
    // Upper entries in place; the mirrored ones (-v at (j, q)) as one store of
    // the lane's four consecutive rows q when the acc layout gives them
    // (single precision: rows 4 (lane / 16) + r) and the tile is off-diagonal.
    const bool offd = ti != tj;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
        if constexpr (sizeof(R) == 4) {
            const int q0 = rbase + acc_row<R>(lane, 0);
            if (offd && j < n && q0 + 3 < n) {
                struct alignas(4 * sizeof(T)) Q4 { T v[4]; } m4;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    M[(uint32_t)(q0 + r) * un + (uint32_t)j] = make_<T>(re[jb][r], im[jb][r]);
                    m4.v[r] = make_<T>(-re[jb][r], -im[jb][r]);
                }
                const uint32_t mo = (uint32_t)j * un + (uint32_t)q0;
                if (mo % 4 == 0) {
                    *reinterpret_cast<Q4 *>(M + mo) = m4;
                } else {
#pragma unroll
                    for (int r = 0; r < 4; ++r) M[mo + r] = m4.v[r];
                }
                continue;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            if (q >= n || j >= n) continue;
            if (q < j) {
                T v = make_<T>(re[jb][r], im[jb][r]);
                M[(uint32_t)q * un + (uint32_t)j] = v;
                M[(uint32_t)j * un + (uint32_t)q] = make_<T>(-re[jb][r], -im[jb][r]);
            } else if (q == j) {
                M[(uint32_t)q * un + (uint32_t)j] = zero<T>();
            }
        }
    }
}

template <class T> hipError_t det_flush_t(const StepArgs &a, hipStream_t s) {
    const int tpd = (a.n + 63) / 64;
    if constexpr (Real<T>::cplx) {
        hipLaunchKernelGGL(det_flush_kernel<T>, dim3((unsigned)(a.W * tpd * tpd)), dim3(256), 0, s, a, tpd);
    } else {
        hipLaunchKernelGGL(det_flush_strip_kernel<T>, dim3((unsigned)(a.W * tpd)), dim3(256), 0, s, a, tpd);
    }
    return hipGetLastError();
}

template <class T> hipError_t pf_flush_t(const StepArgs &a, hipStream_t s) {
    const int tpd = (a.n + 63) / 64;
    const int pairs = tpd * (tpd + 1) / 2;
    if (a.KM == 1)
        hipLaunchKernelGGL((pf_flush_kernel<T, 2>), dim3((unsigned)(a.W * pairs)), dim3(256), 0, s, a, tpd);
    else
        hipLaunchKernelGGL((pf_flush_kernel<T, 0>), dim3((unsigned)(a.W * pairs)), dim3(256), 0, s, a, tpd);
    return hipGetLastError();
}

}  // namespace

namespace lrx {

hipError_t det_flush(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return det_flush_t<float>(a, s);
        case LRX_F64: return det_flush_t<double>(a, s);
        case LRX_C64: return det_flush_t<cf32>(a, s);
        case LRX_C128: return det_flush_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t pf_flush(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return pf_flush_t<float>(a, s);
        case LRX_F64: return pf_flush_t<double>(a, s);
        case LRX_C64: return pf_flush_t<cf32>(a, s);
        case LRX_C128: return pf_flush_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
