// MFMA helpers and the determinant flush tile, shared by the flush kernels
// (lrx_flush.hip) and the persistent window kernel (lrx_window.hip).
#pragma once

#include "lrx_common.hpp"
#include "lrx_internal.hpp"

// Internal linkage: every translation unit that includes this gets its own copy.
namespace {
namespace lrxfl {

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

}  // namespace lrxfl
}  // namespace
