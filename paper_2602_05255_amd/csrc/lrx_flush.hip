// Delayed-update flush: a batched GEMM with a tiny inner dimension on MFMA.
//
//   DET (Eq. delayed_Ainv):     M0 -= B A^T,  B = [b_1 .. b_tau] rows  (fb, [n][K*KM])
//                                              A = [a_1 .. a_tau] cols  (fa, [K*KM][n])
//   PF  (Eq. pf_delayed_Ainv):  M0 += sum_t (a_t R_t^-1) a_t^T,  fa = [2K][n], fb = R_t^-1 [K][2][2]
//
// Work-group = 4 waves = a 64 x 64 output tile; each wave owns 16 rows x 64
// columns as four 16x16 MFMA blocks (v_mfma_f64_16x16x4f64 / v_mfma_f32_16x16x4f32,
// one 16x4 A and one 4x16 B fragment per lane-step).  Complex products use four
// real MFMAs.  The accumulator starts from the M0 tile, so M0 is read and
// written exactly once.  Blocks of one walker are kept on one XCD.
//
// PF: only tiles on or above the diagonal are computed; every upper entry is
// written together with its exact negative at the transposed position, so M0
// stays exactly skew-symmetric (and the diagonal stays exactly zero).
#include "lrx_common.hpp"
#include "lrx_internal.hpp"

namespace {

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
// Panels are staged in LDS in chunks of 256 bytes of slot columns per row
// (32 KiB of LDS per work-group for every dtype) with coalesced 16-byte loads;
// rows are padded by one element to spread the fragment reads over the banks.
template <class T>
__global__ __launch_bounds__(256) void det_flush_kernel(StepArgs a, int tiles_per_dim) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    constexpr int V = vec16<T>();
    constexpr int kChunk = 256 / (int)sizeof(T);
    constexpr int SB = kChunk + 1;        // padded stride of the b panel rows
    constexpr int SA = 64 + 1;            // padded stride of the a panel rows
    __shared__ T s_b[64 * SB];            // b rows q0..q0+63, slot columns of the chunk
    __shared__ T s_a[kChunk * SA];        // a columns (slot te) over j0..j0+63
    const int n = a.n, KM = a.KM, KK = a.K * KM, TE = a.tau * KM;
    const int tiles = tiles_per_dim * tiles_per_dim;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / tiles;
    if (w >= a.W) return;
    const int tile = lb - w * tiles;
    const int ti = tile / tiles_per_dim, tj = tile - ti * tiles_per_dim;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int q0 = ti * 64, j0 = tj * 64;
    const int kq = lane >> 4;                 // inner index within a 4-deep step

    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * KK * n;
    const T *fb = static_cast<const T *>(a.fb) + (size_t)w * n * KK;

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
    const bool vec_b = (KK % V) == 0;         // b rows start on 16-byte boundaries
    const bool vec_a = (n % V) == 0;
    for (int c0 = 0; c0 < TE; c0 += kChunk) {
        const int cw = min(kChunk, TE - c0);
        __syncthreads();
        // b panel: 64 rows x cw slot columns (row-contiguous in fb)
        for (int idx = tid; idx < 64 * (kChunk / V); idx += 256) {
            const int r = idx / (kChunk / V), cv = (idx - r * (kChunk / V)) * V;
            const int q = q0 + r;
            T tmp[V];
            if (q < n && vec_b && cv + V <= cw) {
                ld16<T>(fb + (size_t)q * KK + c0 + cv, tmp);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) tmp[v] = (q < n && cv + v < cw) ? fb[(size_t)q * KK + c0 + cv + v] : zero<T>();
            }
#pragma unroll
            for (int v = 0; v < V; ++v) s_b[r * SB + cv + v] = tmp[v];
        }
        // a panel: cw slot columns x 64 (column-contiguous in fa)
        for (int idx = tid; idx < kChunk * (64 / V); idx += 256) {
            const int t = idx / (64 / V), jv = (idx - t * (64 / V)) * V;
            const int j = j0 + jv;
            T tmp[V];
            if (t < cw && vec_a && j + V <= n) {
                ld16<T>(fa + (size_t)(c0 + t) * n + j, tmp);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) tmp[v] = (t < cw && j + v < n) ? fa[(size_t)(c0 + t) * n + j + v] : zero<T>();
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

// ------------------------------------------------------------------ PF
template <class T>
__global__ __launch_bounds__(256) void pf_flush_kernel(StepArgs a, int tiles_per_dim) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    const int n = a.n, KM = a.KM, KA = 2 * KM, TE = a.tau * KA;
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

    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * (size_t)a.K * KA * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * (size_t)a.K * KA * KA;

    A4 re[4], im[4];
    const int rbase = ti * 64 + wv * 16;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            T v = (q < n && j < n && q < j) ? M[(size_t)q * n + j] : zero<T>();
            re[jb][r] = re_(v);
            im[jb][r] = im_(v);
        }
    }
    for (int te0 = 0; te0 < TE; te0 += 4) {
        const int te = te0 + kq;
        const bool tin = te < TE;
        // Atilde[q][te] = sum_s a_t[q][s] R_t^-1[s][te mod KA]
        T at = zero<T>();
        if (tin && qa < n) {
            const int t = te / KA, sp = te - t * KA;
            for (int s = 0; s < KA; ++s)
                at = fmac(fa[(size_t)(t * KA + s) * n + qa], rinv[(size_t)t * KA * KA + s * KA + sp], at);
        }
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int j = j0 + jb * 16 + (lane & 15);
            T av = (tin && j < n) ? fa[(size_t)te * n + j] : zero<T>();
            mac<T>(at, av, re[jb], im[jb]);
        }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int j = j0 + jb * 16 + (lane & 15);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            if (q >= n || j >= n) continue;
            if (q < j) {
                T v = make_<T>(re[jb][r], im[jb][r]);
                M[(size_t)q * n + j] = v;
                M[(size_t)j * n + q] = make_<T>(-re[jb][r], -im[jb][r]);
            } else if (q == j) {
                M[(size_t)q * n + j] = zero<T>();
            }
        }
    }
}

template <class T> hipError_t det_flush_t(const StepArgs &a, hipStream_t s) {
    const int tpd = (a.n + 63) / 64;
    hipLaunchKernelGGL(det_flush_kernel<T>, dim3((unsigned)(a.W * tpd * tpd)), dim3(256), 0, s, a, tpd);
    return hipGetLastError();
}

template <class T> hipError_t pf_flush_t(const StepArgs &a, hipStream_t s) {
    const int tpd = (a.n + 63) / 64;
    const int pairs = tpd * (tpd + 1) / 2;
    hipLaunchKernelGGL(pf_flush_kernel<T>, dim3((unsigned)(a.W * pairs)), dim3(256), 0, s, a, tpd);
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
