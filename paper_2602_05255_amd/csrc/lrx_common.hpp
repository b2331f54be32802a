// Shared device helpers for the lrx kernels (gfx950, wave64).
//
// Scalar types: float, double, cf32, cf64 (interleaved complex).  Complex
// arithmetic is written out so that the same template code serves all four
// bulk dtypes; products are never conjugated (the method uses plain
// transposes for complex matrices).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <math.h>

#include "../../include/lrx.h"

#define LRX_WAVE 64

struct cf32 { float x, y; };
struct cf64 { double x, y; };

template <class T> struct Real;
template <> struct Real<float> { using type = float; static constexpr bool cplx = false; };
template <> struct Real<double> { using type = double; static constexpr bool cplx = false; };
template <> struct Real<cf32> { using type = float; static constexpr bool cplx = true; };
template <> struct Real<cf64> { using type = double; static constexpr bool cplx = true; };

// Wide ("FP64 or complex128") type used by init/refresh and for ratios.
template <class T> struct Wide;
template <> struct Wide<float> { using type = double; };
template <> struct Wide<double> { using type = double; };
template <> struct Wide<cf32> { using type = cf64; };
template <> struct Wide<cf64> { using type = cf64; };

// ---------------------------------------------------------------- arithmetic
__host__ __device__ inline cf32 operator+(cf32 a, cf32 b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cf32 operator-(cf32 a, cf32 b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cf32 operator-(cf32 a) { return {-a.x, -a.y}; }
__host__ __device__ inline cf32 operator*(cf32 a, cf32 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__host__ __device__ inline cf64 operator+(cf64 a, cf64 b) { return {a.x + b.x, a.y + b.y}; }
__host__ __device__ inline cf64 operator-(cf64 a, cf64 b) { return {a.x - b.x, a.y - b.y}; }
__host__ __device__ inline cf64 operator-(cf64 a) { return {-a.x, -a.y}; }
__host__ __device__ inline cf64 operator*(cf64 a, cf64 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

template <class T> __device__ __forceinline__ T zero() { return T{}; }
template <class T> __device__ __forceinline__ T one();
template <> __device__ __forceinline__ float one<float>() { return 1.0f; }
template <> __device__ __forceinline__ double one<double>() { return 1.0; }
template <> __device__ __forceinline__ cf32 one<cf32>() { return {1.0f, 0.0f}; }
template <> __device__ __forceinline__ cf64 one<cf64>() { return {1.0, 0.0}; }

// a*b + c
__device__ __forceinline__ float fmac(float a, float b, float c) { return fmaf(a, b, c); }
__device__ __forceinline__ double fmac(double a, double b, double c) { return fma(a, b, c); }
__device__ __forceinline__ cf32 fmac(cf32 a, cf32 b, cf32 c) {
    return {fmaf(a.x, b.x, fmaf(-a.y, b.y, c.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, c.y))};
}
__device__ __forceinline__ cf64 fmac(cf64 a, cf64 b, cf64 c) {
    return {fma(a.x, b.x, fma(-a.y, b.y, c.x)), fma(a.x, b.y, fma(a.y, b.x, c.y))};
}
// c - a*b
__device__ __forceinline__ float fmsc(float a, float b, float c) { return fmaf(-a, b, c); }
__device__ __forceinline__ double fmsc(double a, double b, double c) { return fma(-a, b, c); }
__device__ __forceinline__ cf32 fmsc(cf32 a, cf32 b, cf32 c) { return fmac(-a, b, c); }
__device__ __forceinline__ cf64 fmsc(cf64 a, cf64 b, cf64 c) { return fmac(-a, b, c); }

__device__ __forceinline__ double absv(float a) { return fabs((double)a); }
__device__ __forceinline__ double absv(double a) { return fabs(a); }
__device__ __forceinline__ double absv(cf32 a) { return hypot((double)a.x, (double)a.y); }
__device__ __forceinline__ double absv(cf64 a) { return hypot(a.x, a.y); }

__device__ __forceinline__ bool finite_v(float a) { return isfinite(a); }
__device__ __forceinline__ bool finite_v(double a) { return isfinite(a); }
__device__ __forceinline__ bool finite_v(cf32 a) { return isfinite(a.x) && isfinite(a.y); }
__device__ __forceinline__ bool finite_v(cf64 a) { return isfinite(a.x) && isfinite(a.y); }

__device__ __forceinline__ bool is_zero(float a) { return a == 0.0f; }
__device__ __forceinline__ bool is_zero(double a) { return a == 0.0; }
__device__ __forceinline__ bool is_zero(cf32 a) { return a.x == 0.0f && a.y == 0.0f; }
__device__ __forceinline__ bool is_zero(cf64 a) { return a.x == 0.0 && a.y == 0.0; }

// Division a / b.
__device__ __forceinline__ float divv(float a, float b) { return a / b; }
__device__ __forceinline__ double divv(double a, double b) { return a / b; }
__device__ __forceinline__ cf64 divv(cf64 a, cf64 b) {
    // Smith's algorithm (avoids overflow in |b|^2).
    if (fabs(b.x) >= fabs(b.y)) {
        double r = b.y / b.x, d = b.x + b.y * r;
        return {(a.x + a.y * r) / d, (a.y - a.x * r) / d};
    }
    double r = b.x / b.y, d = b.x * r + b.y;
    return {(a.x * r + a.y) / d, (a.y * r - a.x) / d};
}
__device__ __forceinline__ cf32 divv(cf32 a, cf32 b) {
    cf64 q = divv(cf64{a.x, a.y}, cf64{b.x, b.y});
    return {(float)q.x, (float)q.y};
}

// Conversions between precisions (same complexness).
template <class D, class S> __device__ __forceinline__ D conv(S s);
template <> __device__ __forceinline__ float conv<float, double>(double s) { return (float)s; }
template <> __device__ __forceinline__ double conv<double, double>(double s) { return s; }
template <> __device__ __forceinline__ double conv<double, float>(float s) { return (double)s; }
template <> __device__ __forceinline__ float conv<float, float>(float s) { return s; }
template <> __device__ __forceinline__ cf32 conv<cf32, cf64>(cf64 s) { return {(float)s.x, (float)s.y}; }
template <> __device__ __forceinline__ cf64 conv<cf64, cf64>(cf64 s) { return s; }
template <> __device__ __forceinline__ cf64 conv<cf64, cf32>(cf32 s) { return {(double)s.x, (double)s.y}; }
template <> __device__ __forceinline__ cf32 conv<cf32, cf32>(cf32 s) { return s; }

// ---------------------------------------------------------------- reductions
// Exchange with lane ^ m, m a power of two that is a compile-time constant once
// the caller's loops are unrolled: DPP quad permutes for 1 and 2 and the row
// rotate by 8 for 8 (a rotation by half of a 16-lane row is the xor), the
// ds_swizzle bit mode (and 0x1f, xor m) for 4 and 16, and ds_bpermute across
// the two 32-lane halves for 32.
__device__ __forceinline__ int xshfl_i32(int v, int m) {
    switch (m) {
        case 1: return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
        case 2: return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
        case 4: return __builtin_amdgcn_ds_swizzle(v, 0x101F);
        case 8: return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);  // row_ror:8
        case 16: return __builtin_amdgcn_ds_swizzle(v, 0x401F);
        default: return __builtin_amdgcn_ds_bpermute((((int)threadIdx.x & (LRX_WAVE - 1)) ^ m) << 2, v);
    }
}
__device__ __forceinline__ float shfl_xor_v(float v, int m) { return __int_as_float(xshfl_i32(__float_as_int(v), m)); }
__device__ __forceinline__ double shfl_xor_v(double v, int m) {
    const long long b = __double_as_longlong(v);
    const int lo = xshfl_i32((int)(b & 0xffffffffll), m), hi = xshfl_i32((int)(b >> 32), m);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ cf32 shfl_xor_v(cf32 v, int m) { return {shfl_xor_v(v.x, m), shfl_xor_v(v.y, m)}; }
__device__ __forceinline__ cf64 shfl_xor_v(cf64 v, int m) { return {shfl_xor_v(v.x, m), shfl_xor_v(v.y, m)}; }

// The exchange distances below are template parameters (compile-time
// recursion): a loop whose counter halves or doubles is not unrolled by the
// compiler, and a rolled loop turns the value arrays into runtime-indexed
// registers (one select per element per access).

// Butterfly rounds lane ^ M, ..., lane ^ 32 on one value; every lane gets the sum.
template <int M, class T> __device__ __forceinline__ T wave_fold(T r) {
    if constexpr (M < LRX_WAVE) return wave_fold<M * 2>(r + shfl_xor_v(r, M));
    else return r;
}

// Sum over the 64 lanes of a wave; every lane receives the total.
template <class T> __device__ __forceinline__ T wave_sum(T v) { return wave_fold<1>(v); }

// One halving round of wave_sum_multi: exchange with lane ^ H, keep the upper
// half of the live values on lanes with bit H set.
template <int H, class T, int NV> __device__ __forceinline__ void wave_halve(T (&v)[NV], int lane) {
    if constexpr (H >= 1) {
        const bool up = (lane & H) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            T send = up ? v[i] : v[i + H];
            T keep = up ? v[i + H] : v[i];
            v[i] = keep + shfl_xor_v(send, H);
        }
        wave_halve<H / 2>(v, lane);
    }
}

// Reduce NV values per lane across the wave with a butterfly that halves the
// live values each round: the round exchanging with lane ^ h keeps the upper
// half of the live values on lanes with bit h set, so after log2(NV) rounds
// lane l holds a partial of value (l mod NV); the remaining rounds finish the
// sum.  Returns the total of value (lane mod NV) on every lane.  NV must be a
// power of two <= 64.  Cost: NV - 1 + 6 - log2(NV) exchanges instead of 6 NV.
template <class T, int NV> __device__ __forceinline__ T wave_sum_multi(T (&v)[NV]) {
    const int lane = threadIdx.x & (LRX_WAVE - 1);
    wave_halve<NV / 2>(v, lane);
    return wave_fold<NV>(v[0]);
}

// Shuffle from an arbitrary lane (src taken modulo the wave size).
__device__ __forceinline__ float shfl_any(float v, int src) { return __shfl(v, src, LRX_WAVE); }
__device__ __forceinline__ double shfl_any(double v, int src) { return __shfl(v, src, LRX_WAVE); }
__device__ __forceinline__ cf32 shfl_any(cf32 v, int src) { return {__shfl(v.x, src, LRX_WAVE), __shfl(v.y, src, LRX_WAVE)}; }
__device__ __forceinline__ cf64 shfl_any(cf64 v, int src) { return {__shfl(v.x, src, LRX_WAVE), __shfl(v.y, src, LRX_WAVE)}; }

// ---------------------------------------------------------------- wave LU
// LU with partial pivoting (largest modulus, lowest row on ties) of a KM x KM
// matrix spread over the first KM*KM lanes of a wave: lane l holds entry
// (l / KM, l % KM).  Every lane of the wave calls it.  The row operations are
// applied to the identity alongside (b = L^-1 P), then U X = b is solved by
// back substitution, so on return lane l holds entry (l / KM, l % KM) of the
// inverse.  det (wide type) and singular (a zero pivot; the inverse is then
// undefined) are the same on every lane.  All indices are compile-time or
// wave-uniform, so nothing goes to scratch memory.
template <class T, int KM>
__device__ __forceinline__ void wave_lu_det_inv(T a, T &inv, typename Wide<T>::type &det, bool &singular) {
    using W = typename Wide<T>::type;
    const int lane = threadIdx.x & (LRX_WAVE - 1);
    const int i = lane / KM, c = lane % KM;
    T b = (i == c) ? one<T>() : zero<T>();
    W d = one<W>();
    bool sing = false;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        int p = j;
        double best = absv(shfl_any(a, j * KM + j));
#pragma unroll
        for (int ii = j + 1; ii < KM; ++ii) {
            const double v = absv(shfl_any(a, ii * KM + j));
            if (v > best) { best = v; p = ii; }
        }
        if (p != j) {
            const T aj = shfl_any(a, j * KM + c), ap = shfl_any(a, p * KM + c);
            const T bj = shfl_any(b, j * KM + c), bp = shfl_any(b, p * KM + c);
            if (i == j) { a = ap; b = bp; } else if (i == p) { a = aj; b = bj; }
            d = -d;
        }
        const T piv = shfl_any(a, j * KM + j);
        d = d * conv<W>(piv);
        if (is_zero(piv)) { sing = true; continue; }
        const T l = divv(shfl_any(a, i * KM + j), piv);
        const T ajc = shfl_any(a, j * KM + c), bjc = shfl_any(b, j * KM + c);
        if (i > j) { a = fmsc(l, ajc, a); b = fmsc(l, bjc, b); }
    }
    T x = b;
#pragma unroll
    for (int ii = KM - 1; ii >= 0; --ii) {
        const T uii = shfl_any(a, ii * KM + ii);
        if (i == ii) x = divv(x, uii);
        const T xr = shfl_any(x, ii * KM + c);
        const T uc = shfl_any(a, i * KM + ii);
        if (i < ii) x = fmsc(uc, xr, x);
    }
    inv = x;
    det = d;
    singular = sing;
}

// ---------------------------------------------------------------- small LU
// In-place LU with partial pivoting of a k x k matrix held by one thread
// (row-major, stride KM).  Returns det(R) in the wide type, writes R^-1 into
// inv (stride KM).  singular = true when a pivot is exactly zero.
template <class T, int KM>
__device__ void small_lu_det_inv(T (&r)[KM * KM], int k, T (&inv)[KM * KM],
                                 typename Wide<T>::type &det, bool &singular) {
    using W = typename Wide<T>::type;
    int piv[KM];
    W d = one<W>();
    singular = false;
    for (int j = 0; j < k; ++j) {
        int p = j;
        double best = absv(r[j * KM + j]);
        for (int i = j + 1; i < k; ++i) {
            double a = absv(r[i * KM + j]);
            if (a > best) { best = a; p = i; }
        }
        piv[j] = p;
        if (p != j) {
            for (int c = 0; c < k; ++c) { T t = r[j * KM + c]; r[j * KM + c] = r[p * KM + c]; r[p * KM + c] = t; }
            d = -d;
        }
        T dj = r[j * KM + j];
        d = d * conv<W>(dj);
        if (is_zero(dj)) { singular = true; continue; }
        for (int i = j + 1; i < k; ++i) {
            T l = divv(r[i * KM + j], dj);
            r[i * KM + j] = l;
            for (int c = j + 1; c < k; ++c) r[i * KM + c] = fmsc(l, r[j * KM + c], r[i * KM + c]);
        }
    }
    det = d;
    if (singular) return;
    // Columns of the inverse: solve L U x = P e_c.
    for (int c = 0; c < k; ++c) {
        T col[KM];
        for (int i = 0; i < k; ++i) col[i] = (i == c) ? one<T>() : zero<T>();
        for (int j = 0; j < k; ++j) { int p = piv[j]; if (p != j) { T t = col[j]; col[j] = col[p]; col[p] = t; } }
        for (int i = 0; i < k; ++i) {
            T s = col[i];
            for (int j = 0; j < i; ++j) s = fmsc(r[i * KM + j], col[j], s);
            col[i] = s;
        }
        for (int i = k - 1; i >= 0; --i) {
            T s = col[i];
            for (int j = i + 1; j < k; ++j) s = fmsc(r[i * KM + j], col[j], s);
            col[i] = divv(s, r[i * KM + i]);
        }
        for (int i = 0; i < k; ++i) inv[i * KM + c] = col[i];
    }
}

// Pfaffian of a small skew matrix held by one thread (m x m, stride N, m even),
// by Parlett-Reid elimination in pairs (Appendix A): for columns j = 0, 2, ...
// bring the largest |a[i][j]|, i > j, to row and column j + 1 (a swap flips the
// sign), multiply by the pivot a[j][j+1], and remove the pair with the rank-2
// skew update a[p][q] += w_p c_q - c_p w_q (c = a[j][q] / pivot, w = a[j+1][q]).
template <class T, int N>
__device__ void small_pf(T (&a)[N * N], int m, typename Wide<T>::type &pf) {
    using W = typename Wide<T>::type;
    W acc = one<W>();
    for (int j = 0; j + 1 < m; j += 2) {
        int p = j + 1;
        double best = absv(a[(j + 1) * N + j]);
        for (int i = j + 2; i < m; ++i) {
            const double v = absv(a[i * N + j]);
            if (v > best) { best = v; p = i; }
        }
        if (p != j + 1) {
            for (int c = 0; c < m; ++c) { T t = a[(j + 1) * N + c]; a[(j + 1) * N + c] = a[p * N + c]; a[p * N + c] = t; }
            for (int r = 0; r < m; ++r) { T t = a[r * N + j + 1]; a[r * N + j + 1] = a[r * N + p]; a[r * N + p] = t; }
            acc = -acc;
        }
        const T piv = a[j * N + j + 1];
        if (is_zero(piv)) { pf = zero<W>(); return; }
        acc = acc * conv<W>(piv);
        for (int q = j + 2; q < m; ++q) {
            const T cq = divv(a[j * N + q], piv), wq = a[(j + 1) * N + q];
            for (int pp = j + 2; pp < m; ++pp) {
                const T cp = divv(a[j * N + pp], piv), wp = a[(j + 1) * N + pp];
                a[pp * N + q] = fmsc(cp, wq, fmac(wp, cq, a[pp * N + q]));
            }
        }
    }
    pf = acc;
}

// ---------------------------------------------------------------- log|r|, phase
__device__ __forceinline__ void accum_logphase(double r, double *logabs, double *phase) {
    *logabs += log(fabs(r));
    if (r < 0) *phase = -*phase;
}
__device__ __forceinline__ void accum_logphase(cf64 r, double *logabs, cf64 *phase) {
    double m = hypot(r.x, r.y);
    *logabs += log(m);
    cf64 u = {r.x / m, r.y / m};
    *phase = (*phase) * u;
}

// ---------------------------------------------------------------- XCD mapping
// Work-groups are dispatched round-robin over the 8 XCDs of the MI355X
// (block b runs on XCD b % 8).  Remap so that consecutive logical blocks --
// the row blocks of one walker -- land on the same XCD and share its L2.
__device__ __forceinline__ uint32_t xcd_remap(uint32_t b, uint32_t nblocks) {
    const uint32_t nx = 8;
    uint32_t per = nblocks / nx;
    if (per == 0 || b >= per * nx) return b;   // ragged tail keeps its own order
    return (b % nx) * per + (b / nx);
}

// ---------------------------------------------------------------- packed skew storage
// The 64 x 64 tiles on and above the diagonal (I <= J) of an n x n skew matrix,
// tile (I, J) at index I*nt - I*(I-1)/2 + (J - I) (nt = ceil(n / 64)), each
// row-major.  pk_offset needs r / 64 <= c / 64.
__device__ __forceinline__ size_t pk_offset(int nt, int r, int c) {
    const int I = r >> 6, J = c >> 6;
    return ((size_t)(I * nt - I * (I - 1) / 2 + (J - I)) << 12) + (size_t)((r & 63) << 6) + (size_t)(c & 63);
}
__device__ __forceinline__ size_t lrx_pk_elems_dev(int n) {
    const int nt = (n + 63) >> 6;
    return (size_t)(nt * (nt + 1) / 2) << 12;
}

// ---------------------------------------------------------------- 16-byte IO
template <class T> constexpr int vec16() { return (int)(16 / sizeof(T)); }

template <class T>
__device__ __forceinline__ void ld16(const T *p, T (&o)[vec16<T>()]) {
    uint4 raw = *reinterpret_cast<const uint4 *>(p);
    __builtin_memcpy(&o[0], &raw, 16);
}
// Non-temporal variant: the data is read once (streamed), no reuse to keep.
template <class T>
__device__ __forceinline__ void ld16_nt(const T *p, T (&o)[vec16<T>()]) {
    typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
    const u32x4 raw = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
    __builtin_memcpy(&o[0], &raw, 16);
}
template <class T>
__device__ __forceinline__ void st16(T *p, const T (&o)[vec16<T>()]) {
    uint4 raw;
    __builtin_memcpy(&raw, &o[0], 16);
    *reinterpret_cast<uint4 *>(p) = raw;
}

// ---------------------------------------------------------------- RNG
// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter (c0..c3), key
// (k0, k1), ten rounds of two 32x32->64 multiplies with a Weyl key schedule.
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)M0 * c[0];
        uint64_t p1 = (uint64_t)M1 * c[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
}

// Uniform double in [0, 1) with 53 random bits for walker w at step counter ctr.
__device__ __forceinline__ double philox_uniform(uint64_t seed, uint64_t ctr, uint32_t w) {
    uint32_t c[4] = {w, (uint32_t)ctr, (uint32_t)(ctr >> 32), 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t bits = ((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6);
    return (double)bits * 0x1.0p-53;
}

__device__ __forceinline__ double abs2_wide(double r) { return r * r; }
__device__ __forceinline__ double abs2_wide(cf64 r) { return r.x * r.x + r.y * r.y; }

// Metropolis rule on |r|^2 (zero / non-finite ratios and flagged walkers rejected).
template <class Wd>
__device__ __forceinline__ uint8_t mh_decide(Wd r, uint32_t flags, int mode, double u01, uint64_t seed,
                                             uint64_t ctr, uint32_t w) {
    const double p = abs2_wide(r);
    if (flags != 0 || !isfinite(p) || !(p > 0.0)) return 0;
    if (mode == LRX_MH_FORCE) return 1;
    const double uu = mode == LRX_MH_UNIFORMS ? u01 : philox_uniform(seed, ctr, w);
    return uu < fmin(1.0, p) ? 1 : 0;
}
