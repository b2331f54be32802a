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
#include "lrx_common.hpp"
#include "lrx_internal.hpp"

namespace {

using lrx::StepArgs;
using lrx::HopArgs;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / LRX_WAVE;

__device__ __forceinline__ void flag_or(uint32_t *flags, int w, uint32_t bit) {
    atomicOr(flags + w, bit);
}

// ------------------------------------------------------------------ build hop
template <class T>
__global__ __launch_bounds__(kThreads) void det_build_hop_kernel(HopArgs a) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x;
    const int n = a.n, KM = a.KM;
    const Wd *phi = static_cast<const Wd *>(a.phi);
    T *u = static_cast<T *>(a.out) + (size_t)w * KM * n;
    int kw = a.k[w];
    bool bad = kw < 1 || kw > KM;
    __shared__ int s_src[LRX_MAX_KMAX_DET], s_dst[LRX_MAX_KMAX_DET];
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = bad ? 1 : 0;
    __syncthreads();
    if (threadIdx.x < KM) {
        const int c = threadIdx.x;
        int e = a.elec[w * KM + c], sl = a.slot[w * KM + c];
        int src = 0, dst = 0;
        if (!bad && c < kw) {
            if (e < 0 || e >= n || sl < 0 || sl >= a.n_empty) atomicOr(&s_bad, 1);
            else {
                src = a.occ[(size_t)w * n + e];
                dst = a.empty[(size_t)w * a.n_empty + sl];
                if (src < 0 || src >= a.sites || dst < 0 || dst >= a.sites) { atomicOr(&s_bad, 1); src = dst = 0; }
            }
        }
        s_src[c] = src;
        s_dst[c] = dst;
    }
    __syncthreads();
    const bool fail = s_bad != 0;
    if (fail && threadIdx.x == 0) flag_or(a.flags, w, LRX_FLAG_BADINDEX);
    if (fail) kw = 0;
    for (int c = 0; c < KM; ++c) {
        const Wd *ps = phi + (size_t)s_src[c] * n;
        const Wd *pd = phi + (size_t)s_dst[c] * n;
        for (int j = threadIdx.x; j < n; j += kThreads)
            u[(size_t)c * n + j] = (c < kw) ? conv<T>(pd[j] - ps[j]) : zero<T>();
    }
}

// ------------------------------------------------------------------ propose
// One work-group per walker.  Cost O(n k + tau n k) per walker: rows I of M0,
// the a-slots (only their live columns) and b-slot rows I.
template <class T, int KM>
__global__ __launch_bounds__(kThreads) void det_propose_kernel(StepArgs a) {
    using Wd = typename Wide<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & (LRX_WAVE - 1), wv = tid / LRX_WAVE;
    const int n = a.n, tau = a.tau, KK = a.K * KM, TE = tau * KM;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    const T *u = static_cast<const T *>(a.u) + (size_t)w * KM * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * KK * n;
    const T *fb = static_cast<const T *>(a.fb) + (size_t)w * n * KK;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    T *C = reinterpret_cast<T *>(st + a.L.c);
    T *G = reinterpret_cast<T *>(st + a.L.g);
    T *Rinv = reinterpret_cast<T *>(st + a.L.rinv);
    Wd *ratio_st = reinterpret_cast<Wd *>(st + a.L.ratio);
    const int *kslot = reinterpret_cast<const int *>(st + a.L.kslot);

    T *s_fbI = reinterpret_cast<T *>(smem);                 // [KM][TE]
    T *s_red = s_fbI + (size_t)KM * TE;                     // [kWaves][KM*KM]
    __shared__ int s_rows[KM];
    __shared__ int s_k;
    __shared__ int s_bad;

    if (tid == 0) {
        int kw = a.k[w];
        int bad = (kw < 1 || kw > KM);
        s_k = bad ? 1 : kw;
        s_bad = bad;
    }
    __syncthreads();
    const int k = s_k;
    if (tid < KM) {
        int r = a.rows[w * KM + tid];
        if (tid < k && (r < 0 || r >= n)) { atomicOr(&s_bad, 1); r = 0; }
        s_rows[tid] = (tid < k) ? r : 0;
    }
    __syncthreads();
    // b-slot rows I (only needed for the delayed form).
    for (int idx = tid; idx < KM * TE; idx += kThreads) {
        int c = idx / TE, te = idx - c * TE;
        s_fbI[idx] = (c < k) ? fb[(size_t)s_rows[c] * KK + te] : zero<T>();
    }
    __syncthreads();

    // C[c][i] = M0[I_c][i] - sum_{t<tau, e<k_t} a_t[i][e] b_t[I_c][e]
    for (int i = tid; i < n; i += kThreads) {
        T cv[KM];
#pragma unroll
        for (int c = 0; c < KM; ++c) cv[c] = (c < k) ? M[(size_t)s_rows[c] * n + i] : zero<T>();
        for (int t = 0; t < tau; ++t) {
            const int kt = min(max(kslot[t], 0), KM);
            for (int e = 0; e < kt; ++e) {
                const int te = t * KM + e;
                const T av = fa[(size_t)te * n + i];
#pragma unroll
                for (int c = 0; c < KM; ++c)
                    if (c < k) cv[c] = fmsc(av, s_fbI[c * TE + te], cv[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < KM; ++c) C[(size_t)c * n + i] = cv[c];
    }
    __threadfence_block();
    __syncthreads();

    // R[c][d] = delta_cd + sum_i u[c][i] C[d][i]
    for (int c = 0; c < k; ++c) {
        T p[KM];
#pragma unroll
        for (int d = 0; d < KM; ++d) p[d] = zero<T>();
        for (int i = tid; i < n; i += kThreads) {
            const T uc = u[(size_t)c * n + i];
#pragma unroll
            for (int d = 0; d < KM; ++d) p[d] = fmac(uc, C[(size_t)d * n + i], p[d]);
        }
        T tot = wave_sum_multi<T, KM>(p);
        if (lane < KM) s_red[wv * KM * KM + c * KM + lane] = tot;
    }

    // G[te][c] = a_te . u_c  (te < tau*KM), used by the delayed accept.
    if (a.K > 0) {
        for (int te = wv; te < TE; te += kWaves) {
            const int t = te / KM, e = te - t * KM;
            const bool live = e < min(max(kslot[t], 0), KM);
            T p[KM];
#pragma unroll
            for (int c = 0; c < KM; ++c) p[c] = zero<T>();
            if (live) {
                for (int i = lane; i < n; i += LRX_WAVE) {
                    const T av = fa[(size_t)te * n + i];
#pragma unroll
                    for (int c = 0; c < KM; ++c)
                        if (c < k) p[c] = fmac(av, u[(size_t)c * n + i], p[c]);
                }
            }
            T tot = wave_sum_multi<T, KM>(p);
            if (lane < KM) G[(size_t)te * KM + lane] = (live && lane < k) ? tot : zero<T>();
        }
    }
    __syncthreads();

    if (tid == 0) {
        T r[KM * KM], ri[KM * KM];
        for (int c = 0; c < KM; ++c)
            for (int d = 0; d < KM; ++d) {
                T s = (c == d) ? one<T>() : zero<T>();
                if (c < k && d < k)
                    for (int q = 0; q < kWaves; ++q) s = s + s_red[q * KM * KM + c * KM + d];
                r[c * KM + d] = s;
                ri[c * KM + d] = zero<T>();
            }
        Wd det;
        bool sing;
        small_lu_det_inv<T, KM>(r, k, ri, det, sing);
        for (int c = 0; c < KM * KM; ++c) Rinv[c] = ri[c];
        if (s_bad) det = zero<Wd>();
        *ratio_st = det;
        static_cast<Wd *>(a.ratio)[w] = det;
        uint32_t f = 0;
        if (s_bad) f |= LRX_FLAG_BADINDEX;
        if (!finite_v(det)) f |= LRX_FLAG_NONFINITE;
        if (sing || is_zero(det) || !finite_v(det)) f |= LRX_FLAG_SINGULAR_R;
        // SINGULAR_R / NONFINITE describe only this proposal: they are kept in
        // the stash copy of the ratio (zero => accept is a no-op) rather than
        // in the sticky walker flags.  Bad indices are sticky.
        if (f & LRX_FLAG_BADINDEX) flag_or(a.flags, w, LRX_FLAG_BADINDEX);
        if (f & (LRX_FLAG_SINGULAR_R | LRX_FLAG_NONFINITE)) *ratio_st = zero<Wd>();
    }
}

// ------------------------------------------------------------------ accept
// Row-streaming pass.  A work-group handles `rows_per_block` rows of one
// walker; each wave takes RB rows at a time, each lane holding NEL elements of
// every row (16-byte vectors, coalesced).  u and C live in LDS, shared by all
// rows of the block.
//
// DELAYED = false: Sherman-Morrison/Woodbury in place (Eq. det_inv).
// DELAYED = true : b_tau rows and a_tau columns written to slot tau (Sec. II.C).
template <class T, int KM, int NEL, int RB, bool DELAYED>
__global__ __launch_bounds__(kThreads) void det_accept_kernel(StepArgs a, int rows_per_block, int blocks_per_walker) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;                 // 16-byte chunks per lane per row
    constexpr int NV = RB * KM;                  // reduced values per row batch
    constexpr int MG = 4;                        // max slot columns per lane (TE <= 256)
    extern __shared__ __align__(16) unsigned char smem[];

    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / blocks_per_walker;
    const int rb = lb - w * blocks_per_walker;
    if (w >= a.W) return;
    const int tid = threadIdx.x, lane = tid & (LRX_WAVE - 1), wv = tid / LRX_WAVE;
    const int n = a.n, KK = a.K * KM, tau = a.tau, TE = tau * KM;
    const int q0 = rb * rows_per_block;
    const int q1 = min(n, q0 + rows_per_block);

    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    const T *u = static_cast<const T *>(a.u) + (size_t)w * KM * n;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    const T *C = reinterpret_cast<const T *>(st + a.L.c);
    const T *G = reinterpret_cast<const T *>(st + a.L.g);
    const T *Rinv = reinterpret_cast<const T *>(st + a.L.rinv);
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.L.ratio);
    int *kslot = reinterpret_cast<int *>(st + a.L.kslot);
    T *fa = DELAYED ? static_cast<T *>(a.fa) + (size_t)w * KK * n : nullptr;
    T *fb = DELAYED ? static_cast<T *>(a.fb) + (size_t)w * n * KK : nullptr;

    int k = a.k[w];
    k = (k < 1 || k > KM) ? 1 : k;
    const bool take = a.accept[w] != 0 && a.flags[w] == 0 && !is_zero(ratio);

    if (!take) {
        if (rb == 0 && tid == 0 && a.accept[w]) a.accept[w] = 0;   // skipped: no occupancy commit
        if (DELAYED) {   // a rejected walker's slot contributes nothing
            for (int idx = tid; idx < KM * (q1 - q0); idx += kThreads) {
                int c = idx / (q1 - q0), q = q0 + idx - c * (q1 - q0);
                fa[(size_t)(tau * KM + c) * n + q] = zero<T>();
                fb[(size_t)q * KK + tau * KM + c] = zero<T>();
            }
            if (rb == 0 && tid == 0) kslot[tau] = 0;
        }
        return;
    }
    if (rb == 0 && tid == 0) {
        accum_logphase(ratio, a.logabs + w, static_cast<Wd *>(a.phase) + w);
        if (DELAYED) kslot[tau] = k;
    }

    const int npad = NCH * V * LRX_WAVE;        // padded row length held in LDS
    T *s_u = reinterpret_cast<T *>(smem);       // [KM][npad]
    T *s_c = s_u + (size_t)KM * npad;           // [KM][npad]
    T *s_ri = s_c + (size_t)KM * npad;          // [KM*KM]
    T *s_w = s_ri + KM * KM;                    // [kWaves][NV]
    for (int idx = tid; idx < KM * npad; idx += kThreads) {
        int c = idx / npad, j = idx - c * npad;
        bool ok = c < k && j < n;
        s_u[idx] = ok ? u[(size_t)c * n + j] : zero<T>();
        s_c[idx] = ok ? C[(size_t)c * n + j] : zero<T>();
    }
    if (tid < KM * KM) s_ri[tid] = Rinv[tid];
    if (DELAYED) {   // a_tau = C, written for this block's rows
        for (int idx = tid; idx < KM * (q1 - q0); idx += kThreads) {
            int c = idx / (q1 - q0), q = q0 + idx - c * (q1 - q0);
            fa[(size_t)(tau * KM + c) * n + q] = (c < k) ? C[(size_t)c * n + q] : zero<T>();
        }
    }
    // Slot products G[te][c] for the slot columns this lane owns (te = lane + 64 m).
    T g[MG][KM];
    if (DELAYED) {
#pragma unroll
        for (int m = 0; m < MG; ++m)
#pragma unroll
            for (int c = 0; c < KM; ++c) {
                int te = lane + m * LRX_WAVE;
                g[m][c] = (te < TE) ? G[(size_t)te * KM + c] : zero<T>();
            }
    }
    __syncthreads();

    const bool vec_ok = a.aligned != 0;
    for (int qb = q0 + wv * RB; qb < q1; qb += kWaves * RB) {
        T x[RB][NEL];
        // Load RB rows.
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int q = qb + r;
            const T *row = M + (size_t)q * n;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int j0 = ch * V * LRX_WAVE + lane * V;
                T tmp[V];
                if (q < q1 && vec_ok && j0 + V <= n) {
                    ld16<T>(row + j0, tmp);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) tmp[v] = (q < q1 && j0 + v < n) ? row[j0 + v] : zero<T>();
                }
#pragma unroll
                for (int v = 0; v < V; ++v) x[r][ch * V + v] = tmp[v];
            }
        }
        // w[r][c] = M[q_r,:] . u_c  (minus the delayed-slot correction)
        T p[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) p[i] = zero<T>();
#pragma unroll
        for (int c = 0; c < KM; ++c) {
            if (c < k) {
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    T uv[V];
                    ld16<T>(s_u + (size_t)c * npad + ch * V * LRX_WAVE + lane * V, uv);
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int v = 0; v < V; ++v) p[r * KM + c] = fmac(x[r][ch * V + v], uv[v], p[r * KM + c]);
                }
            }
        }
        if (DELAYED) {
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int q = qb + r;
                if (q >= q1) continue;
#pragma unroll
                for (int m = 0; m < MG; ++m) {
                    const int te = lane + m * LRX_WAVE;
                    if (te < TE) {
                        const T bv = fb[(size_t)q * KK + te];
#pragma unroll
                        for (int c = 0; c < KM; ++c) p[r * KM + c] = fmsc(bv, g[m][c], p[r * KM + c]);
                    }
                }
            }
        }
        T tot = wave_sum_multi<T, NV>(p);
        if (lane < NV) s_w[wv * NV + lane] = tot;
        __builtin_amdgcn_wave_barrier();
        // z[r] = R^-1 w[r]
        T z[RB][KM];
#pragma unroll
        for (int r = 0; r < RB; ++r)
#pragma unroll
            for (int c = 0; c < KM; ++c) {
                T s = zero<T>();
#pragma unroll
                for (int d = 0; d < KM; ++d)
                    if (c < k && d < k) s = fmac(s_ri[c * KM + d], s_w[wv * NV + r * KM + d], s);
                z[r][c] = s;
            }
        __builtin_amdgcn_wave_barrier();
        if (!DELAYED) {
            // M[q,:] -= sum_c z[c] C[:, c]^T
#pragma unroll
            for (int c = 0; c < KM; ++c) {
                if (c < k) {
#pragma unroll
                    for (int ch = 0; ch < NCH; ++ch) {
                        T cv[V];
                        ld16<T>(s_c + (size_t)c * npad + ch * V * LRX_WAVE + lane * V, cv);
#pragma unroll
                        for (int r = 0; r < RB; ++r)
#pragma unroll
                            for (int v = 0; v < V; ++v) x[r][ch * V + v] = fmsc(z[r][c], cv[v], x[r][ch * V + v]);
                    }
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int q = qb + r;
                if (q >= q1) continue;
                T *row = M + (size_t)q * n;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int j0 = ch * V * LRX_WAVE + lane * V;
                    T tmp[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) tmp[v] = x[r][ch * V + v];
                    if (vec_ok && j0 + V <= n) {
                        st16<T>(row + j0, tmp);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) if (j0 + v < n) row[j0 + v] = tmp[v];
                    }
                }
            }
        } else {
            // b_tau[q][c] = z[c]
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int q = qb + r;
                if (q < q1) {
#pragma unroll
                    for (int c = 0; c < KM; ++c)
                        if (lane == c) fb[(size_t)q * KK + tau * KM + c] = z[r][c];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ Metropolis
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

__device__ __forceinline__ double abs2_wide(double r) { return r * r; }
__device__ __forceinline__ double abs2_wide(cf64 r) { return r.x * r.x + r.y * r.y; }

template <class Wd>
__global__ void metropolis_kernel(int W, const Wd *ratio, const double *u01, uint64_t seed,
                                  uint64_t counter, int mode, const uint32_t *flags, uint8_t *accept) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    const Wd r = ratio[w];
    const double p = abs2_wide(r);
    bool ok = flags[w] == 0 && isfinite(p) && p > 0.0;
    uint8_t acc = 0;
    if (ok) {
        if (mode == LRX_MH_FORCE) {
            acc = 1;
        } else {
            double uu;
            if (mode == LRX_MH_UNIFORMS) {
                uu = u01[w];
            } else {
                uint32_t c[4] = {(uint32_t)w, (uint32_t)counter, (uint32_t)(counter >> 32), 0u};
                philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
                uint64_t bits = ((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6);  // 53 bits
                uu = (double)bits * 0x1.0p-53;
            }
            acc = uu < fmin(1.0, p) ? 1 : 0;
        }
    }
    accept[w] = acc;
}

__global__ void hop_commit_kernel(int W, int n, int n_empty, int KM, const int32_t *k, const int32_t *elec,
                                  const int32_t *slot, const uint8_t *accept, int32_t *occ, int32_t *empty) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W || !accept[w]) return;
    int kw = k[w];
    if (kw < 1 || kw > KM) return;
    for (int c = 0; c < kw; ++c) {
        int e = elec[w * KM + c], s = slot[w * KM + c];
        if (e < 0 || e >= n || s < 0 || s >= n_empty) continue;
        int32_t *po = occ + (size_t)w * n + e;
        int32_t *pe = empty + (size_t)w * n_empty + s;
        int32_t t = *po;
        *po = *pe;
        *pe = t;
    }
}

// ------------------------------------------------------------------ launchers
template <class T> hipError_t build_hop_t(const HopArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(det_build_hop_kernel<T>, dim3(a.W), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <class T, int KM> hipError_t propose_t(const StepArgs &a, hipStream_t s) {
    const int TE = a.tau * KM;
    size_t lds = sizeof(T) * ((size_t)KM * TE + (size_t)kWaves * KM * KM);
    hipLaunchKernelGGL((det_propose_kernel<T, KM>), dim3(a.W), dim3(kThreads), lds, s, a);
    return hipGetLastError();
}

template <class T> hipError_t propose_k(const StepArgs &a, hipStream_t s) {
    switch (a.KM) {
        case 1: return propose_t<T, 1>(a, s);
        case 2: return propose_t<T, 2>(a, s);
        case 4: return propose_t<T, 4>(a, s);
        case 8: return propose_t<T, 8>(a, s);
    }
    return hipErrorInvalidValue;
}

// Rows held per wave batch: the RB x NEL row values plus the RB x KM partial
// dot products stay within ~96 VGPRs.
template <class T, int NEL, int KM> constexpr int rows_per_batch() {
    constexpr int per_row = (NEL + KM) * (int)sizeof(T);
    return 8 * per_row <= 384 ? 8 : (4 * per_row <= 384 ? 4 : (2 * per_row <= 384 ? 2 : 1));
}

template <class T, int KM, int NEL, bool D> hipError_t accept_t(const StepArgs &a, hipStream_t s) {
    constexpr int RB = rows_per_batch<T, NEL, KM>();
    // Rows per block: enough blocks to fill 256 CUs several times over.
    const int n = a.n;
    int rpb = kWaves * RB;
    long long blocks = (long long)a.W * ((n + rpb - 1) / rpb);
    while (rpb < n && blocks > 8 * 256 * 4) {
        rpb *= 2;
        blocks = (long long)a.W * ((n + rpb - 1) / rpb);
    }
    const int bpw = (n + rpb - 1) / rpb;
    const int npad = (NEL / vec16<T>()) * vec16<T>() * LRX_WAVE;
    size_t lds = sizeof(T) * ((size_t)2 * KM * npad + KM * KM + (size_t)kWaves * RB * KM);
    hipLaunchKernelGGL((det_accept_kernel<T, KM, NEL, RB, D>), dim3((unsigned)(a.W * bpw)), dim3(kThreads),
                       lds, s, a, rpb, bpw);
    return hipGetLastError();
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

namespace lrx {

hipError_t det_build_hop(int dtype, const HopArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return build_hop_t<float>(a, s);
        case LRX_F64: return build_hop_t<double>(a, s);
        case LRX_C64: return build_hop_t<cf32>(a, s);
        case LRX_C128: return build_hop_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t det_propose(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return propose_k<float>(a, s);
        case LRX_F64: return propose_k<double>(a, s);
        case LRX_C64: return propose_k<cf32>(a, s);
        case LRX_C128: return propose_k<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t det_accept(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return accept_d<float>(a, s);
        case LRX_F64: return accept_d<double>(a, s);
        case LRX_C64: return accept_d<cf32>(a, s);
        case LRX_C128: return accept_d<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

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

}  // namespace lrx
