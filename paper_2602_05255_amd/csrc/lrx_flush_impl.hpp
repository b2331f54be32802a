// MFMA helpers and the determinant flush tile, shared by the flush kernels
// (lrx_flush.hip) and the persistent window kernel (lrx_window.hip).
#pragma once

#include "lrx_common.hpp"
#include "lrx_internal.hpp"

// Internal linkage: every translation unit that includes this gets its own copy.
namespace {
namespace lrxfl {

using lrx::StepArgs;

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <class R> struct Acc;
template <> struct Acc<float> { using type = f4; };
template <> struct Acc<double> { using type = d4; };

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Output row of accumulator register r in a lane (column = lane % 16).
// v_mfma_f32_16x16x4f32: row 4 * (lane / 16) + r;
// v_mfma_f64_16x16x4f64: row 4 * r + lane / 16 (measured on gfx950).
template <class R> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) { return 4 * (lane >> 4) + r; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) { return 4 * r + (lane >> 4); }

template <class T> __device__ __forceinline__ typename Real<T>::type re_(T v);
template <> __device__ __forceinline__ float re_<float>(float v) { return v; }
template <> __device__ __forceinline__ double re_<double>(double v) { return v; }
template <> __device__ __forceinline__ float re_<cf32>(cf32 v) { return v.x; }
template <> __device__ __forceinline__ double re_<cf64>(cf64 v) { return v.x; }
template <class T> __device__ __forceinline__ typename Real<T>::type im_(T v);
template <> __device__ __forceinline__ float im_<float>(float) { return 0.f; }
template <> __device__ __forceinline__ double im_<double>(double) { return 0.0; }
template <> __device__ __forceinline__ float im_<cf32>(cf32 v) { return v.y; }
template <> __device__ __forceinline__ double im_<cf64>(cf64 v) { return v.y; }
template <class T> __device__ __forceinline__ T make_(typename Real<T>::type r, typename Real<T>::type i);
template <> __device__ __forceinline__ float make_<float>(float r, float) { return r; }
template <> __device__ __forceinline__ double make_<double>(double r, double) { return r; }
template <> __device__ __forceinline__ cf32 make_<cf32>(float r, float i) { return {r, i}; }
template <> __device__ __forceinline__ cf64 make_<cf64>(double r, double i) { return {r, i}; }

// acc += a * b over one 4-deep inner step (complex: four real products).
template <class T>
__device__ __forceinline__ void mac(T a, T b, typename Acc<typename Real<T>::type>::type &re,
                                    typename Acc<typename Real<T>::type>::type &im) {
    re = mfma(re_(a), re_(b), re);
    if constexpr (Real<T>::cplx) {
        re = mfma(-im_(a), im_(b), re);
        im = mfma(re_(a), im_(b), im);
        im = mfma(im_(a), re_(b), im);
    }
}

// ------------------------------------------------------------------ DET
// Live slot columns: slot t holds k_t = kslot[t] columns t*KM + c (c < k_t);
// rejected steps (k_t = 0) and the zero padding beyond k_t contribute nothing
// to M0 -= B A^T, so the flush contracts over the live columns only.  The
// first wave builds the list, one lane per slot (tau <= 64): an inclusive
// scan of the k_t gives each slot its place.  All threads of the block call
// this; s_live must hold tau*KM ints.
template <int D> __device__ __forceinline__ int scan_up(int s, int t) {
    if constexpr (D < LRX_WAVE) {
        const int o = __shfl_up(s, D, LRX_WAVE);
        return scan_up<D * 2>(t >= D ? s + o : s, t);
    } else {
        return s;
    }
}
__device__ __forceinline__ int det_live_columns(const int *kslot, int tau, int KM, int *s_live, int *s_n) {
    if (threadIdx.x < LRX_WAVE) {
        const int t = threadIdx.x;
        const int kt = t < tau ? min(max(kslot[max(min(t, tau - 1), 0)], 0), KM) : 0;
        const int incl = scan_up<1>(kt, t);
        for (int c = 0; c < kt; ++c) s_live[incl - kt + c] = t * KM + c;
        if (t == LRX_WAVE - 1) *s_n = incl;
    }
    __syncthreads();
    return *s_n;
}

// LDS staging for one 64 x 64 tile: b rows x 256 bytes of live columns, and
// the matching a columns over 64 entries; rows padded by one element.
template <class T> struct FlushLds {
    static constexpr int kChunk = 256 / (int)sizeof(T);
    static constexpr int SB = kChunk + 1;
    static constexpr int SA = 64 + 1;
    static constexpr size_t bytes = sizeof(T) * ((size_t)64 * SB + (size_t)kChunk * SA);
};

// One 64 x 64 tile (rows q0.., columns j0..) of M0 -= B A^T over the live
// columns.  Work-group = 4 waves; wave wv owns rows q0 + 16 wv .. + 15 as four
// 16x16 MFMA blocks.  The accumulator starts from the M0 tile, so M0 is read
// and written once.  Every thread of the block must call this.
template <class T>
__device__ __forceinline__ void det_flush_tile(T *M, const T *fa, const T *fb, int n, int KK, const int *s_live,
                                               int nl, int q0, int j0, T *s_b, T *s_a) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    constexpr int V = vec16<T>();
    constexpr int kChunk = FlushLds<T>::kChunk;
    constexpr int SB = FlushLds<T>::SB;
    constexpr int SA = FlushLds<T>::SA;
    if (nl == 0) return;                      // nothing accepted since the last flush
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int kq = lane >> 4;                 // inner index within a 4-deep step

    A4 re[4], im[4];
    const int rbase = q0 + wv * 16;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            T v = (q < n && j < n) ? M[(size_t)q * n + j] : zero<T>();
            re[jb][r] = re_(v);
            im[jb][r] = im_(v);
        }
    }
    const bool vec_a = (n % V) == 0;
    for (int c0 = 0; c0 < nl; c0 += kChunk) {
        const int cw = min(kChunk, nl - c0);
        __syncthreads();
        // b panel: 64 rows x cw live columns (gathered from the rows of fb)
        for (int idx = tid; idx < 64 * kChunk; idx += 256) {
            const int r = idx / kChunk, t = idx - r * kChunk;
            const int q = q0 + r;
            s_b[r * SB + t] = (q < n && t < cw) ? fb[(size_t)q * KK + s_live[c0 + t]] : zero<T>();
        }
        // a panel: cw live columns x 64 (contiguous in fa)
        for (int idx = tid; idx < kChunk * (64 / V); idx += 256) {
            const int t = idx / (64 / V), jv = (idx - t * (64 / V)) * V;
            const int j = j0 + jv;
            T tmp[V];
            if (t < cw && vec_a && j + V <= n) {
                ld16<T>(fa + (size_t)s_live[c0 + t] * n + j, tmp);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    tmp[v] = (t < cw && j + v < n) ? fa[(size_t)s_live[c0 + t] * n + j + v] : zero<T>();
            }
#pragma unroll
            for (int v = 0; v < V; ++v) s_a[t * SA + jv + v] = tmp[v];
        }
        __syncthreads();
        for (int t0 = 0; t0 < cw; t0 += 4) {
            T bv = s_b[(wv * 16 + (lane & 15)) * SB + t0 + kq];
            bv = make_<T>(-re_(bv), -im_(bv));      // acc += (-b) a^T accumulates M0 - B A^T
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const T av = s_a[(t0 + kq) * SA + jb * 16 + (lane & 15)];
                mac<T>(bv, av, re[jb], im[jb]);
            }
        }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            if (q < n && j < n) M[(size_t)q * n + j] = make_<T>(re[jb][r], im[jb][r]);
        }
    }
}

// Real data: a work-group owns a 64-column strip of one walker and walks its
// 64-row tiles.  The strip's a panel (live columns x 64) is staged in LDS once
// and serves every row tile; the b values are read straight into the MFMA
// operand registers.  The next tile's M block is in flight while the current
// tile is on the matrix cores, and its b values while the current tile is
// stored.  Live columns are taken in
// chunks of 64 (one chunk unless tau * k_max exceeds 64).
template <class T> struct FlushStripLds {
    static constexpr int kA = 64 * (64 + 1);     // a panel: 64 live columns x 64 entries, padded rows
};

// Strip `strip` (columns 64 strip ..) of walker w; every thread of the
// 256-thread work-group calls it.  s_a: FlushStripLds<T>::kA elements; s_live:
// tau * k_max ints; s_nl: one int.
template <class T>
__device__ __forceinline__ void det_flush_strip(const StepArgs &a, int w, int strip, int tpd, T *s_a, int *s_live,
                                                int *s_nl) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    constexpr int KCH = 64;                  // live columns per chunk
    constexpr int SA = 64 + 1;               // padded LDS row stride of the a panel
    constexpr int NS = KCH / 4;              // 4-deep MFMA steps per chunk
    constexpr int V = vec16<T>();
    const int n = a.n, KK = a.K * a.KM;
    const int j0 = strip * 64;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, kq = lane >> 4, lc = lane & 15;
    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * KK * n;
    const T *fb = static_cast<const T *>(a.fb) + (size_t)w * n * KK;
    int col[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) col[jb] = min(j0 + jb * 16 + lc, n - 1);
    struct Buf { T m[4][4]; };
    // M block of row tile rt (clamped to the last one, so that the load
    // counts stay exact), from 32-bit element offsets off the walker's base
    auto issue_m = [&](int rt, Buf &B) {
        const int rbase = min(rt, tpd - 1) * 64 + wv * 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint32_t ro = (uint32_t)min(rbase + acc_row<R>(lane, r), n - 1) * (uint32_t)n;
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) B.m[jb][r] = M[ro + (uint32_t)col[jb]];
        }
    };
    Buf b0, b1;
    issue_m(0, b0);                          // in flight while the live list and a panel are built
    const int *kslot = reinterpret_cast<const int *>(a.stash + (size_t)w * a.L.stride + a.L.kslot);
    const int nl = det_live_columns(kslot, a.tau, a.KM, s_live, s_nl);
    if (nl == 0) return;                     // nothing accepted since the last flush
    const bool vec_a = (n % V) == 0;
    for (int c0 = 0; c0 < nl; c0 += KCH) {
        const int cw = min(KCH, nl - c0);
        const int ns = (cw + 3) / 4;
        if (c0 > 0) __syncthreads();
        for (int idx = tid; idx < KCH * (64 / V); idx += 256) {
            const int t = idx / (64 / V), jv = (idx - t * (64 / V)) * V;
            const int j = j0 + jv;
            const T *src = fa + (size_t)s_live[c0 + min(t, cw - 1)] * n;
            T tmp[V];
            if (vec_a && j + V <= n) {
                ld16<T>(src + j, tmp);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) tmp[v] = src[min(j + v, n - 1)];
            }
#pragma unroll
            for (int v = 0; v < V; ++v) s_a[t * SA + jv + v] = (t < cw && j + v < n) ? tmp[v] : zero<T>();
        }
        __syncthreads();
        // Loads from clamped addresses, nothing selected until the values are used.
        auto load_b = [&](int rt, T (&bb)[NS]) {
            const int rbase = min(rt, tpd - 1) * 64 + wv * 16;
            const uint32_t bo = (uint32_t)min(rbase + lc, n - 1) * (uint32_t)KK;
#pragma unroll
            for (int s = 0; s < NS; ++s) bb[s] = fb[bo + (uint32_t)s_live[c0 + min(4 * s + kq, cw - 1)]];
        };
        // MFMAs of tile rt, then the b values of tile rt + 1 (issued before the
        // stores), then the stores.
        T bcur[NS];
        auto consume = [&](int rt, Buf &B) {
            const int rbase = rt * 64 + wv * 16;
            A4 acc[4];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb)
#pragma unroll
                for (int r = 0; r < 4; ++r) acc[jb][r] = B.m[jb][r];
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                if (s >= ns) break;
                const int k = 4 * s + kq;
                const T bv = k < cw ? -bcur[s] : zero<T>();      // acc += (-b) a^T: M0 - B A^T
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) acc[jb] = mfma(bv, s_a[k * SA + jb * 16 + lc], acc[jb]);
            }
            load_b(rt + 1, bcur);
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const int j = j0 + jb * 16 + lc;
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q = rbase + acc_row<R>(lane, r);
                    if (q < n && j < n) M[(uint32_t)q * (uint32_t)n + (uint32_t)j] = acc[jb][r];
                }
            }
        };
        if (c0 > 0) issue_m(0, b0);          // a later chunk re-reads the updated M
        load_b(0, bcur);
        for (int rt = 0; rt < tpd; rt += 2) {
            issue_m(rt + 1, b1);
            consume(rt, b0);
            if (rt + 1 >= tpd) break;
            issue_m(rt + 2, b0);
            consume(rt + 1, b1);
        }
    }
}

}  // namespace lrxfl
}  // namespace
