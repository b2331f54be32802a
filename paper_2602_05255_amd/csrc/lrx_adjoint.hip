// Low-rank log-determinant and its hand-written adjoint.
//
// M_w = A_w + B_w C_w^T, A_w = Phi[occ_w] (rows = electron labels), A_w^-T in
// the state.  By the matrix determinant lemma (Sec. II.A, with dense u, v):
//   log det M = log det A + log det R,  R = I_r + C^T P,  P = A^-1 B.
// Gradients (holomorphic; torch passes the cotangent g of log det M and
// expects conj-weighted results):
//   d/dM log det M = M^-T = A^-T - Q R^-T P^T,   Q = A^-T C   (Woodbury, Eq. det_inv)
//   dB = g conj(M^-T C) = g conj(Q R^-T),  dC = g conj(M^-1 B) = g conj(P R^-1)
//   dPhi[s] = sum_{w, i: occ_w[i] = s} g_w conj(M_w^-T[i, :])
//           = sum g_w conj(A_w^-T[i, :])  -  E F,
//   E[s][w r + c] = g_w conj(Q_w[i][c]),  F[w r + c][j] = conj((P_w R_w^-1)[j][c]).
// The first term is a site-major gather (every state row read once); the
// second is a dense GEMM with inner dimension W r on MFMA (split over K with
// atomic accumulation), so the n x n cotangent of a sample is never stored.
#include "lrx_common.hpp"
#include "lrx_internal.hpp"

namespace {

using lrx::LowRankArgs;

constexpr int kT = 256;
constexpr int kWaves = kT / LRX_WAVE;

__device__ __forceinline__ float conjv(float a) { return a; }
__device__ __forceinline__ double conjv(double a) { return a; }
__device__ __forceinline__ cf32 conjv(cf32 a) { return {a.x, -a.y}; }
__device__ __forceinline__ cf64 conjv(cf64 a) { return {a.x, -a.y}; }

// ------------------------------------------------------------------ forward
// One work-group per walker.  Each wave streams rows i = wv, wv + 4, ... of
// M = A^-T (lane owns NEL columns j):  Q[i][c] = M[i,:] . C[:, c] (wave
// reduction), P[j][c] += M[i][j] B[i][c] (per-lane accumulation, summed over
// the waves through LDS at the end).
template <class T, int RR, int NEL>
__global__ __launch_bounds__(kT) void lowrank_fwd_kernel(LowRankArgs a) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = blockIdx.x, n = a.n, r = a.r;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int npad = NCH * V * 64;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    const T *B = static_cast<const T *>(a.B) + (size_t)w * n * r;
    const T *C = static_cast<const T *>(a.C) + (size_t)w * n * r;
    T *P = static_cast<T *>(a.P) + (size_t)w * n * r;
    T *Q = static_cast<T *>(a.Q) + (size_t)w * n * r;
    T *s_c = reinterpret_cast<T *>(smem);            // C, [RR][npad]
    T *s_p = s_c + (size_t)RR * npad;                // P accumulation, [RR][npad]
    T *s_r = s_p + (size_t)RR * npad;                // R, [RR][RR]
    for (int idx = tid; idx < RR * npad; idx += kT) {
        const int c = idx / npad, j = idx - c * npad;
        s_c[idx] = (c < r && j < n) ? C[(size_t)j * r + c] : zero<T>();
        s_p[idx] = zero<T>();
    }
    __syncthreads();
    T pacc[NEL][RR];
#pragma unroll
    for (int e = 0; e < NEL; ++e)
#pragma unroll
        for (int c = 0; c < RR; ++c) pacc[e][c] = zero<T>();
    const bool vec_ok = (n % V) == 0;
    for (int i = wv; i < n; i += kWaves) {
        const T *row = M + (size_t)i * n;
        T x[NEL];
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int j0 = ch * V * 64 + lane * V;
            T tmp[V];
            if (vec_ok && j0 + V <= n) ld16<T>(row + j0, tmp);
            else {
#pragma unroll
                for (int v = 0; v < V; ++v) tmp[v] = (j0 + v < n) ? row[j0 + v] : zero<T>();
            }
#pragma unroll
            for (int v = 0; v < V; ++v) x[ch * V + v] = tmp[v];
        }
        T q[RR], bi[RR];
#pragma unroll
        for (int c = 0; c < RR; ++c) {
            q[c] = zero<T>();
            bi[c] = (c < r) ? B[(size_t)i * r + c] : zero<T>();
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
#pragma unroll
            for (int c = 0; c < RR; ++c) {
                T cv[V];
                ld16<T>(s_c + (size_t)c * npad + ch * V * 64 + lane * V, cv);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    q[c] = fmac(x[ch * V + v], cv[v], q[c]);
                    pacc[ch * V + v][c] = fmac(x[ch * V + v], bi[c], pacc[ch * V + v][c]);
                }
            }
        }
        const T qt = wave_sum_multi<T, RR>(q);     // lane c (< RR): Q[i][c]
        if (lane < r) Q[(size_t)i * r + lane] = qt;
    }
    // P = sum over the waves of their accumulators, one wave at a time.
    for (int q = 0; q < kWaves; ++q) {
        if (wv == q) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int j = ch * V * 64 + lane * V + v;
#pragma unroll
                    for (int c = 0; c < RR; ++c) s_p[c * npad + j] = s_p[c * npad + j] + pacc[ch * V + v][c];
                }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < n * r; idx += kT) {
        const int j = idx / r, c = idx - j * r;
        P[idx] = s_p[c * npad + j];
    }
    // R = I + C^T P (RR x RR dots of length n)
    if (tid < RR * RR) {
        const int c = tid / RR, d = tid - c * RR;
        T s = (c == d) ? one<T>() : zero<T>();
        if (c < r && d < r)
            for (int j = 0; j < n; ++j) s = fmac(s_c[c * npad + j], s_p[d * npad + j], s);
        s_r[tid] = s;
    }
    __syncthreads();
    if (tid == 0) {
        T rm[RR * RR], ri[RR * RR];
        for (int q = 0; q < RR * RR; ++q) { rm[q] = s_r[q]; ri[q] = zero<T>(); }
        Wd det;
        bool sing;
        small_lu_det_inv<T, RR>(rm, r, ri, det, sing);
        T *Ri = static_cast<T *>(a.Rinv) + (size_t)w * r * r;
        for (int c = 0; c < r; ++c)
            for (int d = 0; d < r; ++d) Ri[c * r + d] = ri[c * RR + d];
        double la = a.state_logabs[w];
        Wd ph = static_cast<const Wd *>(a.state_phase)[w];
        if (sing || is_zero(det) || !finite_v(det)) {
            a.logabs[w] = -INFINITY;
            static_cast<Wd *>(a.phase)[w] = zero<Wd>();
        } else {
            accum_logphase(det, &la, &ph);
            a.logabs[w] = la;
            static_cast<Wd *>(a.phase)[w] = ph;
        }
    }
}

// ------------------------------------------------------------------ backward
// Per row j of walker w: Y = P R^-1, Z = Q R^-T; dC = g conj(Y), dB = g conj(Z),
// F[w r + c][j] = conj(Y[j][c]).
template <class T, int RR>
__global__ __launch_bounds__(kT) void lowrank_small_kernel(LowRankArgs a, int bpw) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x / bpw, jb = blockIdx.x - w * bpw;
    const int n = a.n, r = a.r;
    const int j = jb * kT + threadIdx.x;
    __shared__ T s_ri[RR * RR];
    const T *Ri = static_cast<const T *>(a.Rinv) + (size_t)w * r * r;
    if (threadIdx.x < RR * RR) {
        const int c = threadIdx.x / RR, d = threadIdx.x - c * RR;
        s_ri[threadIdx.x] = (c < r && d < r) ? Ri[c * r + d] : zero<T>();
    }
    __syncthreads();
    if (j >= n) return;
    const T g = conv<T>(static_cast<const Wd *>(a.g)[w]);
    const T *P = static_cast<const T *>(a.P) + (size_t)w * n * r;
    const T *Q = static_cast<const T *>(a.Q) + (size_t)w * n * r;
    T pj[RR], qj[RR];
#pragma unroll
    for (int c = 0; c < RR; ++c) {
        pj[c] = (c < r) ? P[(size_t)j * r + c] : zero<T>();
        qj[c] = (c < r) ? Q[(size_t)j * r + c] : zero<T>();
    }
    T *dB = static_cast<T *>(a.dB) + (size_t)w * n * r;
    T *dC = static_cast<T *>(a.dC) + (size_t)w * n * r;
    T *F = static_cast<T *>(a.F);
#pragma unroll
    for (int c = 0; c < RR; ++c) {
        if (c >= r) continue;
        T y = zero<T>(), z = zero<T>();
#pragma unroll
        for (int d = 0; d < RR; ++d) {
            y = fmac(pj[d], s_ri[d * RR + c], y);     // (P R^-1)[j][c]
            z = fmac(qj[d], s_ri[c * RR + d], z);     // (Q R^-T)[j][c]
        }
        dC[(size_t)j * r + c] = g * conjv(y);
        dB[(size_t)j * r + c] = g * conjv(z);
        F[((size_t)w * r + c) * n + j] = conjv(y);
    }
}

__global__ void fill_int_kernel(int *p, size_t count, int v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

template <class T>
__global__ void fill_zero_kernel(T *p, size_t count) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x)
        p[i] = zero<T>();
}

// Site -> (walker, electron) lists: count, scan, fill.  The fill order (and so
// the summation order of the gather) depends on atomic scheduling, as does the
// split-K GEMM: the backward is reproducible to rounding, not bitwise.
__global__ void csr_count_kernel(LowRankArgs a) {
    const size_t total = (size_t)a.W * a.n;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int s = a.occ[idx];
        if (s >= 0 && s < a.sites) atomicAdd(a.csr_start + s, 1);
    }
}

__global__ __launch_bounds__(1024) void csr_scan_kernel(LowRankArgs a) {
    // exclusive scan of csr_start[0..sites) into csr_start, total in csr_start[sites]; copy to cursor
    __shared__ int s_part[1024];
    const int S = a.sites, t = threadIdx.x;
    const int per = (S + 1023) / 1024;
    int sum = 0;
    for (int q = 0; q < per; ++q) {
        const int s = t * per + q;
        if (s < S) sum += a.csr_start[s];
    }
    s_part[t] = sum;
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int q = 0; q < 1024; ++q) { const int v = s_part[q]; s_part[q] = run; run += v; }
        a.csr_start[S] = run;
    }
    __syncthreads();
    int run = s_part[t];
    for (int q = 0; q < per; ++q) {
        const int s = t * per + q;
        if (s < S) {
            const int v = a.csr_start[s];
            a.csr_start[s] = run;
            a.csr_cursor[s] = run;
            run += v;
        }
    }
}

__global__ void csr_fill_kernel(LowRankArgs a) {
    const size_t total = (size_t)a.W * a.n;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int s = a.occ[idx];
        if (s >= 0 && s < a.sites) a.csr_list[atomicAdd(a.csr_cursor + s, 1)] = (int)idx;
    }
}

// dPhi[s][j] = sum_{(w,i) in list(s)} g_w conj(A_w^-T[i][j]);  E[s][w r + c] = g_w conj(Q_w[i][c]).
template <class T>
__global__ __launch_bounds__(kT) void lowrank_gather_kernel(LowRankArgs a, int col_blocks) {
    using Wd = typename Wide<T>::type;
    const int s = blockIdx.x / col_blocks, cb = blockIdx.x - s * col_blocks;
    const int n = a.n, r = a.r;
    const int j = cb * kT + threadIdx.x;
    const int b = a.csr_start[s], e = a.csr_start[s + 1];
    const T *Minv = static_cast<const T *>(a.inv);
    const Wd *g = static_cast<const Wd *>(a.g);
    T acc = zero<T>();
    for (int q = b; q < e; ++q) {
        const int idx = a.csr_list[q];
        const int w = idx / n, i = idx - w * n;
        const T gw = conv<T>(g[w]);
        if (j < n) acc = fmac(gw, conjv(Minv[((size_t)w * n + i) * n + j]), acc);
        if (cb == 0 && threadIdx.x < r) {
            const T *Q = static_cast<const T *>(a.Q) + (size_t)w * n * r;
            static_cast<T *>(a.E)[(size_t)s * a.W * r + (size_t)w * r + threadIdx.x] = gw * conjv(Q[(size_t)i * r + threadIdx.x]);
        }
    }
    if (j < n) static_cast<T *>(a.dphi)[(size_t)s * n + j] = acc;
}

// dPhi -= E F : rows = sites, cols = n, inner = W r, split over K; 64 x 64 tiles,
// MFMA fragments from LDS-staged chunks (as in the delayed flush).
typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
template <class R> struct Acc;
template <> struct Acc<float> { using type = f4; };
template <> struct Acc<double> { using type = d4; };
__device__ __forceinline__ f4 mfma(float x, float y, f4 c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0); }
__device__ __forceinline__ d4 mfma(double x, double y, d4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0); }
template <class R> __device__ __forceinline__ int acc_row(int lane, int q);
template <> __device__ __forceinline__ int acc_row<float>(int lane, int q) { return 4 * (lane >> 4) + q; }
template <> __device__ __forceinline__ int acc_row<double>(int lane, int q) { return 4 * q + (lane >> 4); }
__device__ __forceinline__ float re_(float v) { return v; }
__device__ __forceinline__ double re_(double v) { return v; }
__device__ __forceinline__ float re_(cf32 v) { return v.x; }
__device__ __forceinline__ double re_(cf64 v) { return v.x; }
__device__ __forceinline__ float im_(float) { return 0.f; }
__device__ __forceinline__ double im_(double) { return 0.0; }
__device__ __forceinline__ float im_(cf32 v) { return v.y; }
__device__ __forceinline__ double im_(cf64 v) { return v.y; }

template <class T>
__global__ __launch_bounds__(256) void lowrank_gemm_kernel(LowRankArgs a, int tiles_c, int ksplit) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    constexpr int KC = 256 / (int)sizeof(T);
    constexpr int SE = KC + 1, SF = 64 + 1;
    __shared__ T s_e[64 * SE];
    __shared__ T s_f[KC * SF];
    const int rows = a.sites, cols = a.n, KI = a.W * a.r;
    const int tiles_r = (rows + 63) / 64;
    const int t = blockIdx.x / ksplit, ks = blockIdx.x - t * ksplit;
    const int ti = t / tiles_c, tj = t - ti * tiles_c;
    if (ti >= tiles_r) return;
    const int kper = ((KI + ksplit - 1) / ksplit + KC - 1) / KC * KC;
    const int k0 = ks * kper, k1 = min(KI, k0 + kper);
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6, kq = lane >> 4;
    const T *E = static_cast<const T *>(a.E);
    const T *F = static_cast<const T *>(a.F);
    A4 re[4], im[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int q = 0; q < 4; ++q) { re[jb][q] = 0; im[jb][q] = 0; }
    for (int c0 = k0; c0 < k1; c0 += KC) {
        const int cw = min(KC, k1 - c0);
        __syncthreads();
        for (int idx = tid; idx < 64 * KC; idx += 256) {
            const int rr = idx / KC, cc = idx - rr * KC, row = ti * 64 + rr;
            s_e[rr * SE + cc] = (row < rows && cc < cw) ? E[(size_t)row * KI + c0 + cc] : zero<T>();
        }
        for (int idx = tid; idx < KC * 64; idx += 256) {
            const int kk = idx / 64, jj = idx - kk * 64, col = tj * 64 + jj;
            s_f[kk * SF + jj] = (kk < cw && col < cols) ? F[(size_t)(c0 + kk) * cols + col] : zero<T>();
        }
        __syncthreads();
        for (int t0 = 0; t0 < cw; t0 += 4) {
            const T ev = s_e[(wv * 16 + (lane & 15)) * SE + t0 + kq];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const T fv = s_f[(t0 + kq) * SF + jb * 16 + (lane & 15)];
                re[jb] = mfma(re_(ev), re_(fv), re[jb]);
                if constexpr (Real<T>::cplx) {
                    re[jb] = mfma(-im_(ev), im_(fv), re[jb]);
                    im[jb] = mfma(re_(ev), im_(fv), im[jb]);
                    im[jb] = mfma(im_(ev), re_(fv), im[jb]);
                }
            }
        }
    }
    R *out = reinterpret_cast<R *>(a.dphi);
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int col = tj * 64 + jb * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = ti * 64 + wv * 16 + acc_row<R>(lane, q);
            if (row < rows && col < cols) {
                if constexpr (Real<T>::cplx) {
                    atomicAdd(out + 2 * ((size_t)row * cols + col), -re[jb][q]);
                    atomicAdd(out + 2 * ((size_t)row * cols + col) + 1, -im[jb][q]);
                } else {
                    atomicAdd(out + (size_t)row * cols + col, -re[jb][q]);
                }
            }
        }
    }
}

template <class T, int RR> hipError_t fwd_r(const LowRankArgs &a, hipStream_t s) {
    constexpr int V = vec16<T>();
    const int nch = (a.n + V * 64 - 1) / (V * 64);
    auto launch = [&](auto nel_tag) {
        constexpr int NEL = decltype(nel_tag)::value;
        const int npad = (NEL / V) * V * 64;
        const size_t lds = sizeof(T) * (2 * (size_t)RR * npad + RR * RR);
        hipLaunchKernelGGL((lowrank_fwd_kernel<T, RR, NEL>), dim3(a.W), dim3(kT), lds, s, a);
        return hipGetLastError();
    };
    if (nch <= 1) return launch(std::integral_constant<int, V>{});
    if (nch <= 2) return launch(std::integral_constant<int, 2 * V>{});
    if (nch <= 4) return launch(std::integral_constant<int, 4 * V>{});
    if constexpr (V <= 2) { if (nch <= 8) return launch(std::integral_constant<int, 8 * V>{}); }
    return hipErrorInvalidValue;
}

template <class T> hipError_t fwd_t(const LowRankArgs &a, hipStream_t s) {
    if (a.r <= 1) return fwd_r<T, 1>(a, s);
    if (a.r <= 2) return fwd_r<T, 2>(a, s);
    if (a.r <= 4) return fwd_r<T, 4>(a, s);
    return fwd_r<T, 8>(a, s);
}

template <class T> hipError_t bwd_t(const LowRankArgs &a, hipStream_t s) {
    const int bpw = (a.n + kT - 1) / kT;
    if (a.r <= 1) hipLaunchKernelGGL((lowrank_small_kernel<T, 1>), dim3(a.W * bpw), dim3(kT), 0, s, a, bpw);
    else if (a.r <= 2) hipLaunchKernelGGL((lowrank_small_kernel<T, 2>), dim3(a.W * bpw), dim3(kT), 0, s, a, bpw);
    else if (a.r <= 4) hipLaunchKernelGGL((lowrank_small_kernel<T, 4>), dim3(a.W * bpw), dim3(kT), 0, s, a, bpw);
    else hipLaunchKernelGGL((lowrank_small_kernel<T, 8>), dim3(a.W * bpw), dim3(kT), 0, s, a, bpw);
    const size_t e_count = (size_t)a.sites * a.W * a.r;
    hipLaunchKernelGGL(fill_zero_kernel<T>, dim3(1024), dim3(256), 0, s, static_cast<T *>(a.E), e_count);
    hipLaunchKernelGGL(fill_int_kernel, dim3(64), dim3(256), 0, s, a.csr_start, (size_t)a.sites + 1, 0);
    hipLaunchKernelGGL(csr_count_kernel, dim3(512), dim3(256), 0, s, a);
    hipLaunchKernelGGL(csr_scan_kernel, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(csr_fill_kernel, dim3(512), dim3(256), 0, s, a);
    const int col_blocks = (a.n + kT - 1) / kT;
    hipLaunchKernelGGL(lowrank_gather_kernel<T>, dim3(a.sites * col_blocks), dim3(kT), 0, s, a, col_blocks);
    const int tiles_r = (a.sites + 63) / 64, tiles_c = (a.n + 63) / 64;
    const int KI = a.W * a.r;
    int ksplit = 1;
    while (tiles_r * tiles_c * ksplit < 1024 && KI / (ksplit * 2) >= 256) ksplit *= 2;
    hipLaunchKernelGGL(lowrank_gemm_kernel<T>, dim3(tiles_r * tiles_c * ksplit), dim3(256), 0, s, a, tiles_c, ksplit);
    return hipGetLastError();
}

}  // namespace

namespace lrx {

size_t lowrank_work_bytes(int dtype, int W, int n, int r, int sites) {
    const size_t es = bulk_bytes(dtype);
    size_t off = 0;
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    off += al(sizeof(int) * ((size_t)sites + 1));        // csr_start
    off += al(sizeof(int) * (size_t)sites);              // csr_cursor
    off += al(sizeof(int) * (size_t)W * n);              // csr_list
    off += al(es * (size_t)sites * W * r);               // E
    off += al(es * (size_t)W * r * n);                   // F
    return off;
}

void lowrank_bind_work(LowRankArgs &a, void *work) {
    const size_t es = bulk_bytes(a.dtype);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    uint8_t *p = static_cast<uint8_t *>(work);
    a.csr_start = reinterpret_cast<int *>(p); p += al(sizeof(int) * ((size_t)a.sites + 1));
    a.csr_cursor = reinterpret_cast<int *>(p); p += al(sizeof(int) * (size_t)a.sites);
    a.csr_list = reinterpret_cast<int *>(p); p += al(sizeof(int) * (size_t)a.W * a.n);
    a.E = p; p += al(es * (size_t)a.sites * a.W * a.r);
    a.F = p;
}

hipError_t lowrank_fwd(const LowRankArgs &a, hipStream_t s) {
    switch (a.dtype) {
        case LRX_F32: return fwd_t<float>(a, s);
        case LRX_F64: return fwd_t<double>(a, s);
        case LRX_C64: return fwd_t<cf32>(a, s);
        case LRX_C128: return fwd_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t lowrank_bwd(const LowRankArgs &a, hipStream_t s) {
    switch (a.dtype) {
        case LRX_F32: return bwd_t<float>(a, s);
        case LRX_F64: return bwd_t<double>(a, s);
        case LRX_C64: return bwd_t<cf32>(a, s);
        case LRX_C128: return bwd_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
