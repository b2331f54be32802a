// General low-rank updates in the plain form (no delay).
//
// DET (Sec. II.B, "Matrix updates"): A_1 = A_0 + v u^T with the mixed tuples
//   u = [xu_0 .. xu_{kr-1} | e_{eu_0} .. e_{eu_{kc-1}}],
//   v = [e_{ev_0} .. e_{ev_{kr-1}} | xv_0 .. xv_{kc-1}],
// i.e. row ev_c gains xu_c (c < kr) and column eu_e gains xv_e (e < kc): row
// updates (kc = 0), column updates (kr = 0) and simultaneous row + column
// updates.  With M = A^-T (the state's layout):
//   X = A^-1 v = [M[ev_c, :]^T | M^T xv_e]                       (n x k)
//   R = I_k + u^T X,   r = det R                                  (Eqs. det_ratio, det_R)
//   M_1 = M - (M u) R^-T X^T                                      (Eq. det_inv, transposed)
// so the propose reads rows ev of M and, for dense v columns, streams M once
// (M^T xv); the accept is one pass over the rows q of M: (M u)[q] from the row
// itself (dots with xu, the entries at eu), z = R^-1 (M u)[q], M[q,:] -= z . X^T.
//
// PF (Sec. III.B, "update of k rows and k columns"): A_1 = A_0 - u J u^T with
//   u = [x_0 .. x_{k-1} | e_{i_0} .. e_{i_{k-1}}],  J the 2k x 2k skew identity.
// With M = A^-1 (exactly skew):
//   Z = A^-1 u = [M x_c | -M[i_c, :]^T]                           (Eq. pf_a)
//   R = J + u^T Z (made exactly skew),  r = pf(R) / pf(J)         (Eqs. pf_ratio, pf_R)
//   M_1 = M + Z R^-1 Z^T                                          (Eq. pf_inv)
// The dense-dense entries x_c^T M x_d need M x (one row-streaming GEMV).  The
// update keeps M exactly skew: entry (q, j) is computed from the ordered pair
// (min(q, j), max(q, j)) and negated below the diagonal.
#include "lrx_common.hpp"
#include "lrx_internal.hpp"

namespace {

using lrx::GeneralArgs;

constexpr int kT = 256;
constexpr int kW = kT / LRX_WAVE;

__device__ __forceinline__ float half_(float v) { return 0.5f * v; }
__device__ __forceinline__ double half_(double v) { return 0.5 * v; }
__device__ __forceinline__ cf32 half_(cf32 v) { return {0.5f * v.x, 0.5f * v.y}; }
__device__ __forceinline__ cf64 half_(cf64 v) { return {0.5 * v.x, 0.5 * v.y}; }

// ------------------------------------------------------------------ DET propose
// One work-group per walker.  X is written to the stash (C region, [k][n]).
template <class T, int KM>
__global__ __launch_bounds__(kT) void det_general_propose_kernel(GeneralArgs a) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x, n = a.n, kr = a.kr, kc = a.kc, k = kr + kc;
    const int tid = threadIdx.x;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    uint8_t *st = a.stash + (size_t)w * a.stride;
    T *X = reinterpret_cast<T *>(st + a.off_c);
    T *Rinv = reinterpret_cast<T *>(st + a.off_rinv);
    Wd *ratio_st = reinterpret_cast<Wd *>(st + a.off_ratio);
    const T *xu = static_cast<const T *>(a.xu) + (size_t)w * kr * n;
    const T *xv = static_cast<const T *>(a.xv) + (size_t)w * kc * n;
    __shared__ int s_ev[KM], s_eu[KM], s_bad;
    __shared__ T s_r[KM * KM];
    if (tid == 0) s_bad = 0;
    __syncthreads();
    if (tid < kr) {
        const int e = a.ev[w * kr + tid];
        if (e < 0 || e >= n) atomicOr(&s_bad, 1);
        s_ev[tid] = min(max(e, 0), n - 1);
    }
    if (tid < kc) {
        const int e = a.eu[w * kc + tid];
        if (e < 0 || e >= n) atomicOr(&s_bad, 1);
        s_eu[tid] = min(max(e, 0), n - 1);
    }
    __syncthreads();
    // X[c][:] = M[ev_c, :] (c < kr);  X[kr + e][j] = sum_i xv_e[i] M[i][j] (thread per column j)
    for (int j = tid; j < n; j += kT) {
        for (int c = 0; c < kr; ++c) X[(size_t)c * n + j] = M[(size_t)s_ev[c] * n + j];
        T acc[KM];
#pragma unroll
        for (int e = 0; e < KM; ++e) acc[e] = zero<T>();
        if (kc > 0) {
            for (int i = 0; i < n; ++i) {
                const T m = M[(size_t)i * n + j];
#pragma unroll
                for (int e = 0; e < KM; ++e)
                    if (e < kc) acc[e] = fmac(xv[(size_t)e * n + i], m, acc[e]);
            }
        }
        for (int e = 0; e < kc; ++e) X[(size_t)(kr + e) * n + j] = acc[e];
    }
    __syncthreads();
    // R[c][d] = delta_cd + u_c^T X_d:  c < kr: xu_c . X_d;  c = kr + e: X_d[eu_e]
    if (tid < k * k) {
        const int c = tid / k, d = tid - c * k;
        T s = (c == d) ? one<T>() : zero<T>();
        const T *xd = X + (size_t)d * n;
        if (c < kr) {
            const T *xc = xu + (size_t)c * n;
            T p0 = zero<T>(), p1 = zero<T>();
            int j = 0;
            for (; j + 1 < n; j += 2) { p0 = fmac(xc[j], xd[j], p0); p1 = fmac(xc[j + 1], xd[j + 1], p1); }
            if (j < n) p0 = fmac(xc[j], xd[j], p0);
            s = s + (p0 + p1);
        } else {
            s = s + xd[s_eu[c - kr]];
        }
        s_r[c * KM + d] = s;
    }
    __syncthreads();
    if (tid == 0) {
        T rm[KM * KM], ri[KM * KM];
        for (int q = 0; q < KM * KM; ++q) { rm[q] = zero<T>(); ri[q] = zero<T>(); }
        for (int c = 0; c < k; ++c)
            for (int d = 0; d < k; ++d) rm[c * KM + d] = s_r[c * KM + d];
        Wd det;
        bool sing;
        small_lu_det_inv<T, KM>(rm, k, ri, det, sing);
        for (int c = 0; c < KM; ++c)
            for (int d = 0; d < KM; ++d) Rinv[c * KM + d] = (c < k && d < k && !sing) ? ri[c * KM + d] : zero<T>();
        if (s_bad) {
            det = zero<Wd>();
            atomicOr(a.flags + w, LRX_FLAG_BADINDEX);
        }
        static_cast<Wd *>(a.ratio)[w] = det;
        *ratio_st = (sing || s_bad || is_zero(det) || !finite_v(det)) ? zero<Wd>() : det;
        if (!finite_v(det)) atomicOr(a.flags + w, LRX_FLAG_NONFINITE);
    }
}

// ------------------------------------------------------------------ DET accept
// Work-groups own row blocks of one walker; a wave takes one row at a time.
template <class T, int KM>
__global__ __launch_bounds__(kT) void det_general_accept_kernel(GeneralArgs a, int rows_per_block, int bpw) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x / bpw, rb = blockIdx.x - w * bpw;
    const int n = a.n, kr = a.kr, kc = a.kc, k = kr + kc;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    uint8_t *st = a.stash + (size_t)w * a.stride;
    const T *X = reinterpret_cast<const T *>(st + a.off_c);
    const T *Rinv = reinterpret_cast<const T *>(st + a.off_rinv);
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.off_ratio);
    const bool take = a.accept[w] != 0 && a.flags[w] == 0 && !is_zero(ratio);
    if (!take) {
        if (rb == 0 && tid == 0 && a.accept[w]) a.accept[w] = 0;
        return;
    }
    if (rb == 0 && tid == 0) accum_logphase(ratio, a.logabs + w, static_cast<Wd *>(a.phase) + w);
    const T *xu = static_cast<const T *>(a.xu) + (size_t)w * kr * n;
    __shared__ T s_ri[KM * KM];
    __shared__ int s_eu[KM];
    if (tid < KM * KM) s_ri[tid] = Rinv[tid];
    if (tid < kc) s_eu[tid] = min(max(a.eu[w * kc + tid], 0), n - 1);
    __syncthreads();
    const int q0 = rb * rows_per_block, q1 = min(n, q0 + rows_per_block);
    for (int q = q0 + wv; q < q1; q += kW) {
        T *row = M + (size_t)q * n;
        // y_c = (M u)[q][c]: dots with the dense xu_c, entries M[q][eu_e]
        T y[KM];
#pragma unroll
        for (int c = 0; c < KM; ++c) y[c] = zero<T>();
        for (int j = lane; j < n; j += LRX_WAVE) {
            const T m = row[j];
#pragma unroll
            for (int c = 0; c < KM; ++c)
                if (c < kr) y[c] = fmac(m, xu[(size_t)c * n + j], y[c]);
        }
#pragma unroll
        for (int c = 0; c < KM; ++c) {
            y[c] = wave_sum(y[c]);
            if (c >= kr && c < k) y[c] = row[s_eu[c - kr]];
        }
        // z = R^-1 y
        T z[KM];
#pragma unroll
        for (int d = 0; d < KM; ++d) {
            T s = zero<T>();
#pragma unroll
            for (int c = 0; c < KM; ++c)
                if (c < k) s = fmac(s_ri[d * KM + c], y[c], s);
            z[d] = s;
        }
        // every lane has read the row before any lane writes it
        __builtin_amdgcn_wave_barrier();
        for (int j = lane; j < n; j += LRX_WAVE) {
            T m = row[j];
#pragma unroll
            for (int d = 0; d < KM; ++d)
                if (d < k) m = fmsc(z[d], X[(size_t)d * n + j], m);
            row[j] = m;
        }
    }
}

// ------------------------------------------------------------------ PF propose
// One work-group per walker.  Z (stash C region, [2k][n]): Z[c][i] = M[i,:] . x_c
// (row dots, one wave per row), Z[k + c][i] = -M[i_c][i].
template <class T, int KP>
__global__ __launch_bounds__(kT) void pf_general_propose_kernel(GeneralArgs a) {
    using Wd = typename Wide<T>::type;
    constexpr int NR = 2 * KP;
    const int w = blockIdx.x, n = a.n, k = a.kr, m2 = 2 * k;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    uint8_t *st = a.stash + (size_t)w * a.stride;
    T *Z = reinterpret_cast<T *>(st + a.off_c);
    T *Rinv = reinterpret_cast<T *>(st + a.off_rinv);
    Wd *ratio_st = reinterpret_cast<Wd *>(st + a.off_ratio);
    const T *x = static_cast<const T *>(a.xu) + (size_t)w * k * n;
    __shared__ int s_i[KP], s_bad;
    __shared__ T s_r[NR * NR];
    if (tid == 0) s_bad = 0;
    __syncthreads();
    if (tid < k) {
        const int e = a.ev[w * k + tid];
        if (e < 0 || e >= n) atomicOr(&s_bad, 1);
        s_i[tid] = min(max(e, 0), n - 1);
    }
    __syncthreads();
    for (int i = wv; i < n; i += kW) {
        const T *row = M + (size_t)i * n;
        T p[KP];
#pragma unroll
        for (int c = 0; c < KP; ++c) p[c] = zero<T>();
        for (int j = lane; j < n; j += LRX_WAVE) {
            const T mv = row[j];
#pragma unroll
            for (int c = 0; c < KP; ++c)
                if (c < k) p[c] = fmac(mv, x[(size_t)c * n + j], p[c]);
        }
#pragma unroll
        for (int c = 0; c < KP; ++c) p[c] = wave_sum(p[c]);
        if (lane == 0)
            for (int c = 0; c < k; ++c) Z[(size_t)c * n + i] = p[c];
    }
    for (int idx = tid; idx < k * n; idx += kT) {
        const int c = idx / n, i = idx - c * n;
        Z[(size_t)(k + c) * n + i] = -M[(size_t)s_i[c] * n + i];
    }
    __syncthreads();
    // R = J + u^T Z: row a < k (dense x_a): x_a . Z_b; row k + c (one-hot i_c): Z_b[i_c]
    if (tid < m2 * m2) {
        const int r = tid / m2, b = tid - r * m2;
        T s = zero<T>();
        const T *zb = Z + (size_t)b * n;
        if (r < k) {
            const T *xa = x + (size_t)r * n;
            for (int j = 0; j < n; ++j) s = fmac(xa[j], zb[j], s);
        } else {
            s = zb[s_i[r - k]];
        }
        const T jv = (b == r + k && r < k) ? one<T>() : ((r == b + k && b < k) ? -one<T>() : zero<T>());
        s_r[r * NR + b] = jv + s;
    }
    __syncthreads();
    if (tid == 0) {
        T rp[NR * NR], rm[NR * NR], ri[NR * NR];
        for (int q = 0; q < NR * NR; ++q) { rp[q] = zero<T>(); ri[q] = zero<T>(); }
        for (int r = 0; r < m2; ++r)
            for (int b = 0; b < m2; ++b) {
                // exactly skew: (R - R^T) / 2
                rp[r * NR + b] = half_(s_r[r * NR + b] - s_r[b * NR + r]);
            }
        for (int q = 0; q < NR * NR; ++q) rm[q] = rp[q];
        Wd pf;
        small_pf<T, NR>(rp, m2, pf);
        if (((k * (k - 1)) / 2) & 1) pf = -pf;     // pf J = (-1)^(k(k-1)/2)
        Wd dd;
        bool sing;
        small_lu_det_inv<T, NR>(rm, m2, ri, dd, sing);
        for (int r = 0; r < NR; ++r)
            for (int b = 0; b < NR; ++b) {
                T v = zero<T>();
                if (r < m2 && b < m2 && !sing) v = half_(ri[r * NR + b] - ri[b * NR + r]);
                Rinv[r * NR + b] = v;
            }
        if (s_bad) {
            pf = zero<Wd>();
            atomicOr(a.flags + w, LRX_FLAG_BADINDEX);
        }
        static_cast<Wd *>(a.ratio)[w] = pf;
        *ratio_st = (sing || s_bad || is_zero(pf) || !finite_v(pf)) ? zero<Wd>() : pf;
        if (!finite_v(pf)) atomicOr(a.flags + w, LRX_FLAG_NONFINITE);
    }
}

// ------------------------------------------------------------------ PF accept
// M[q][j] += g(lo, hi) for q < j, -g(lo, hi) for q > j, with lo = min(q, j), hi = max(q, j):
//   g(lo, hi) = sum_{a < b} Rinv[a][b] (Z[a][lo] Z[b][hi] - Z[b][lo] Z[a][hi]).
template <class T, int KP>
__global__ __launch_bounds__(kT) void pf_general_accept_kernel(GeneralArgs a, int rows_per_block, int bpw) {
    using Wd = typename Wide<T>::type;
    constexpr int NR = 2 * KP;
    const int w = blockIdx.x / bpw, rb = blockIdx.x - w * bpw;
    const int n = a.n, m2 = 2 * a.kr;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    uint8_t *st = a.stash + (size_t)w * a.stride;
    const T *Z = reinterpret_cast<const T *>(st + a.off_c);
    const T *Rinv = reinterpret_cast<const T *>(st + a.off_rinv);
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.off_ratio);
    const bool take = a.accept[w] != 0 && a.flags[w] == 0 && !is_zero(ratio);
    if (!take) {
        if (rb == 0 && tid == 0 && a.accept[w]) a.accept[w] = 0;
        return;
    }
    if (rb == 0 && tid == 0) accum_logphase(ratio, a.logabs + w, static_cast<Wd *>(a.phase) + w);
    __shared__ T s_ri[NR * NR];
    if (tid < NR * NR) s_ri[tid] = Rinv[tid];
    __syncthreads();
    const int q0 = rb * rows_per_block, q1 = min(n, q0 + rows_per_block);
    for (int q = q0 + wv; q < q1; q += kW) {
        T zq[NR];
#pragma unroll
        for (int c = 0; c < NR; ++c) zq[c] = c < m2 ? Z[(size_t)c * n + q] : zero<T>();
        T *row = M + (size_t)q * n;
        for (int j = lane; j < n; j += LRX_WAVE) {
            if (j == q) continue;           // the diagonal stays exactly zero
            const bool up = q < j;
            T zj[NR];
#pragma unroll
            for (int c = 0; c < NR; ++c) zj[c] = c < m2 ? Z[(size_t)c * n + j] : zero<T>();
            T g = zero<T>();
#pragma unroll
            for (int aa = 0; aa < NR; ++aa)
#pragma unroll
                for (int bb = aa + 1; bb < NR; ++bb) {
                    if (bb >= m2) continue;
                    const T lo_a = up ? zq[aa] : zj[aa], lo_b = up ? zq[bb] : zj[bb];
                    const T hi_a = up ? zj[aa] : zq[aa], hi_b = up ? zj[bb] : zq[bb];
                    g = g + s_ri[aa * NR + bb] * (lo_a * hi_b - lo_b * hi_a);
                }
            row[j] = row[j] + (up ? g : -g);
        }
    }
}

template <class T, int KM> hipError_t det_general_t(const GeneralArgs &a, bool propose, hipStream_t s) {
    if (propose) {
        hipLaunchKernelGGL((det_general_propose_kernel<T, KM>), dim3(a.W), dim3(kT), 0, s, a);
    } else {
        const int rpb = a.n < 128 ? a.n : 128, bpw = (a.n + rpb - 1) / rpb;
        hipLaunchKernelGGL((det_general_accept_kernel<T, KM>), dim3(a.W * bpw), dim3(kT), 0, s, a, rpb, bpw);
    }
    return hipGetLastError();
}

template <class T> hipError_t det_general_k(const GeneralArgs &a, bool propose, hipStream_t s) {
    const int k = a.kr + a.kc;
    if (k <= 2) return det_general_t<T, 2>(a, propose, s);
    if (k <= 4) return det_general_t<T, 4>(a, propose, s);
    return det_general_t<T, 8>(a, propose, s);
}

template <class T, int KP> hipError_t pf_general_t(const GeneralArgs &a, bool propose, hipStream_t s) {
    if (propose) {
        hipLaunchKernelGGL((pf_general_propose_kernel<T, KP>), dim3(a.W), dim3(kT), 0, s, a);
    } else {
        const int rpb = a.n < 128 ? a.n : 128, bpw = (a.n + rpb - 1) / rpb;
        hipLaunchKernelGGL((pf_general_accept_kernel<T, KP>), dim3(a.W * bpw), dim3(kT), 0, s, a, rpb, bpw);
    }
    return hipGetLastError();
}

template <class T> hipError_t pf_general_k(const GeneralArgs &a, bool propose, hipStream_t s) {
    if (a.kr <= 1) return pf_general_t<T, 1>(a, propose, s);
    if (a.kr <= 2) return pf_general_t<T, 2>(a, propose, s);
    return pf_general_t<T, 4>(a, propose, s);
}

}  // namespace

namespace lrx {

hipError_t general_update(int kind, int dtype, const GeneralArgs &a, bool propose, hipStream_t s) {
    if (kind == LRX_DET) {
        switch (dtype) {
            case LRX_F32: return det_general_k<float>(a, propose, s);
            case LRX_F64: return det_general_k<double>(a, propose, s);
            case LRX_C64: return det_general_k<cf32>(a, propose, s);
            case LRX_C128: return det_general_k<cf64>(a, propose, s);
        }
    } else {
        switch (dtype) {
            case LRX_F32: return pf_general_k<float>(a, propose, s);
            case LRX_F64: return pf_general_k<double>(a, propose, s);
            case LRX_C64: return pf_general_k<cf32>(a, propose, s);
            case LRX_C128: return pf_general_k<cf64>(a, propose, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
