// Determinant step kernels as per-walker device functions, shared by the
// per-step launches (lrx_det.hip) and the persistent window kernel
// (lrx_window.hip).  See lrx_det.hip for the method notes.
#pragma once

#include "lrx_common.hpp"
#include "lrx_internal.hpp"

// Internal linkage: every translation unit that includes this gets its own copy.
namespace {
namespace lrxdet {

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
// One work-group per walker; thread t owns rows i = t + 256 ii of the columns.
// Cost O(n k + tau n k) per walker: rows I of M0, the live columns of the
// a-slots (read once), b-slot rows I and u.
//   C[c][i]  = M0[I_c][i] - sum_{live te} a_te[i] b_te[I_c]     (A_{tau-1}^-1[:, I])
//   G[te][c] = a_te . u_c   (reduced in groups with the multi-value butterfly)
//   R        = I + u^T C,   r = det R
// With a hop table the update vectors u = Phi[s'] - Phi[s] are built here too.
template <class T> constexpr int prop_nv() { return sizeof(T) <= 4 ? 32 : (sizeof(T) == 8 ? 16 : 8); }

// NW waves per walker (one work-group); each thread owns NI entries i = t + 64 NW ii.
// tid is the thread's index in the work-group (passed in so that a caller
// looping over steps can keep the derived addresses from living across steps).
// With NW = 1 every reduction stays inside the wave and no block barrier sits on
// the critical path.
template <class T, int KM, int NW, int NI>
__device__ __forceinline__ void det_propose_walker(const StepArgs &a, int w, unsigned char *smem, int tid) {
    using Wd = typename Wide<T>::type;
    constexpr int NT = 64 * NW;
    constexpr int NVG = prop_nv<T>() >= KM ? prop_nv<T>() : KM;   // values per group reduction
    constexpr int GS0 = NVG / KM;
    constexpr int GS = (GS0 * NI <= 32) ? GS0 : (32 / NI > 0 ? 32 / NI : 1);   // slot columns per group
    const int lane = tid & (LRX_WAVE - 1), wv = tid / LRX_WAVE;
    const int n = a.n, tau = a.tau, KK = a.K * KM, TE = tau * KM;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    T *u = const_cast<T *>(static_cast<const T *>(a.u)) + (size_t)w * KM * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * KK * n;
    const T *fb = static_cast<const T *>(a.fb) + (size_t)w * n * KK;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    T *C = reinterpret_cast<T *>(st + a.L.c);
    T *G = reinterpret_cast<T *>(st + a.L.g);
    T *Rinv = reinterpret_cast<T *>(st + a.L.rinv);
    Wd *ratio_st = reinterpret_cast<Wd *>(st + a.L.ratio);
    const int *kslot = reinterpret_cast<const int *>(st + a.L.kslot);

    const int TP = TE + 1;                                  // b-slot rows I, plus a zero column at TE
    T *s_fbI = reinterpret_cast<T *>(smem);                 // [KM][TP]
    T *s_red = s_fbI + (size_t)KM * TP;                     // [NW][64]
    T *s_gpart = s_red + NW * 64;                           // [NW][TE * KM] per-wave partial G (NW > 1)
    int *s_live = reinterpret_cast<int *>(s_gpart + (NW > 1 ? (size_t)NW * TE * KM : 0));   // [TE]
    int *s_ks = s_live + TE;                                   // [tau]
    __shared__ int s_rows[KM], s_src[KM], s_dst[KM];
    __shared__ int s_k, s_bad, s_nl;

    const bool fused = a.hop_table != nullptr;
    for (int t = tid; t < tau; t += NT) s_ks[t] = min(max(kslot[t], 0), KM);
    if (tid < KM) {
        int kw = a.k[w];
        const int bad = (kw < 1 || kw > KM);
        kw = bad ? 1 : kw;
        int r = a.rows[w * KM + tid];
        int src = 0, dst = 0, b = bad;
        if (tid < kw) {
            if (r < 0 || r >= n) { b = 1; r = 0; }
            if (fused) {
                const int sl = a.slot[w * KM + tid];
                if (sl < 0 || sl >= a.n_empty) {
                    b = 1;
                } else {
                    src = a.occ[(size_t)w * n + r];
                    dst = a.empty[(size_t)w * a.n_empty + sl];
                    if (src < 0 || src >= a.sites || dst < 0 || dst >= a.sites) { b = 1; src = dst = 0; }
                }
            }
        }
        s_rows[tid] = (tid < kw) ? r : 0;
        s_src[tid] = src;
        s_dst[tid] = dst;
        if (tid == 0) { s_k = kw; s_bad = 0; }
        __builtin_amdgcn_wave_barrier();
        if (b) atomicOr(&s_bad, 1);
    }
    if constexpr (NW == 1)
        for (int idx = tid; idx < TE * KM; idx += NT) G[idx] = zero<T>();
    __syncthreads();
    if (tid == 0) {
        int nl = 0;
        for (int t = 0; t < tau; ++t)
            for (int e = 0; e < s_ks[t]; ++e) s_live[nl++] = t * KM + e;
        s_nl = nl;
    }
    const int k = s_k;
    const bool bad = s_bad != 0;
    for (int idx = tid; idx < KM * TP; idx += NT) {
        int c = idx / TP, te = idx - c * TP;
        s_fbI[idx] = (c < k && te < TE) ? fb[(size_t)s_rows[c] * KK + te] : zero<T>();
    }

    // Loads from clamped, always valid addresses, then select: loads under
    // divergent branches would be serialised by the compiler's waits.
    T uv[NI][KM], cv[NI][KM];
    const Wd *tab = static_cast<const Wd *>(a.hop_table);
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
        const int i = tid + ii * NT;
        const bool valid = i < n;
        const int ic = valid ? i : n - 1;
#pragma unroll
        for (int c = 0; c < KM; ++c) {
            const bool live = valid && c < k;
            T uu;
            if (fused) {
                const Wd d = tab[(size_t)s_dst[c] * n + ic], sv = tab[(size_t)s_src[c] * n + ic];
                uu = (live && !bad) ? conv<T>(d - sv) : zero<T>();
            } else {
                const T uraw = u[(size_t)c * n + ic];
                uu = live ? uraw : zero<T>();
            }
            const T craw = M[(size_t)s_rows[c] * n + ic];
            if (fused && valid) u[(size_t)c * n + i] = uu;
            uv[ii][c] = uu;
            cv[ii][c] = live ? craw : zero<T>();
        }
    }
    __syncthreads();
    // Live slot columns in groups of GS: the loads of the next group are in
    // flight while the current one is reduced (unconditional loads from clamped
    // addresses; a padded entry multiplies the zero column TE of s_fbI and its
    // G partial is dropped).  Each wave reduces G over its own part of i and
    // keeps the partial in LDS, so the loop has no block barrier.
    const int nl = s_nl;
    auto load_grp = [&](int g0, T (&av)[GS][NI]) {
#pragma unroll
        for (int gi = 0; gi < GS; ++gi) {
            const int te = (g0 + gi < nl) ? s_live[g0 + gi] : 0;
#pragma unroll
            for (int ii = 0; ii < NI; ++ii) av[gi][ii] = fa[(size_t)te * n + min(tid + ii * NT, n - 1)];
        }
    };
    auto do_grp = [&](int g0, T (&av)[GS][NI]) {
        T gp[GS * KM];
#pragma unroll
        for (int q = 0; q < GS * KM; ++q) gp[q] = zero<T>();
#pragma unroll
        for (int gi = 0; gi < GS; ++gi) {
            const int te = (g0 + gi < nl) ? s_live[g0 + gi] : TE;
#pragma unroll
            for (int ii = 0; ii < NI; ++ii)
#pragma unroll
                for (int c = 0; c < KM; ++c) {
                    cv[ii][c] = fmsc(av[gi][ii], s_fbI[c * TP + te], cv[ii][c]);
                    gp[gi * KM + c] = fmac(av[gi][ii], uv[ii][c], gp[gi * KM + c]);
                }
        }
        const T tot = wave_sum_multi<T, GS * KM>(gp);      // lane l: value l (gi = l / KM, c = l % KM)
        if (lane < GS * KM && g0 + lane / KM < nl) {
            const int c = lane % KM;
            const int idx = s_live[g0 + lane / KM] * KM + c;
            if constexpr (NW == 1) G[idx] = (c < k) ? tot : zero<T>();
            else s_gpart[(size_t)wv * TE * KM + idx] = tot;
        }
    };
    {
        T a0[GS][NI], a1[GS][NI];
        int g0 = 0;
        if (nl > 0) load_grp(0, a0);
        while (g0 < nl) {
            load_grp(g0 + GS, a1);
            do_grp(g0, a0);
            g0 += GS;
            if (g0 >= nl) break;
            load_grp(g0 + GS, a0);
            do_grp(g0, a1);
            g0 += GS;
        }
    }
    if constexpr (NW > 1) {   // G = sum of the wave partials; dead slot columns and ranks >= k are zero
        __syncthreads();
        for (int idx = tid; idx < TE * KM; idx += NT) {
            const int te = idx / KM, c = idx - te * KM;
            const bool live = (te % KM) < s_ks[te / KM] && c < k;
            T sum = zero<T>();
#pragma unroll
            for (int q = 0; q < NW; ++q) sum = sum + s_gpart[(size_t)q * TE * KM + idx];
            G[idx] = live ? sum : zero<T>();
        }
    }
    // C (stash, and slot a_tau = C of the delayed form, Eq. det_a; a rejected
    // step leaves it dead), and R[c][d] = delta_cd + sum_i u[c][i] C[d][i]
    // (one KM-value reduction per row c of R)
    T *fa_tau = (a.K > 0) ? static_cast<T *>(a.fa) + ((size_t)w * KK + (size_t)tau * KM) * n : nullptr;
#pragma unroll
    for (int ii = 0; ii < NI; ++ii) {
        const int i = tid + ii * NT;
        if (i < n) {
#pragma unroll
            for (int c = 0; c < KM; ++c) {
                C[(size_t)c * n + i] = cv[ii][c];
                if (fa_tau) fa_tau[(size_t)c * n + i] = cv[ii][c];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < KM; ++c) {
        T rp[KM];
#pragma unroll
        for (int d = 0; d < KM; ++d) {
            rp[d] = zero<T>();
#pragma unroll
            for (int ii = 0; ii < NI; ++ii) rp[d] = fmac(uv[ii][c], cv[ii][d], rp[d]);
        }
        const T rt = wave_sum_multi<T, KM>(rp);
        if (lane < KM) s_red[wv * 64 + c * KM + lane] = rt;
    }
    __syncthreads();

    if (wv == 0) {   // R on the first KM*KM lanes of wave 0 (identity beyond the rank), LU across the wave
        const int c = lane / KM, d = lane % KM;
        T rv = zero<T>();
        if (lane < KM * KM) {
            rv = (c == d) ? one<T>() : zero<T>();
            if (c < k && d < k)
                for (int q = 0; q < NW; ++q) rv = rv + s_red[q * 64 + lane];
        }
        T iv;
        Wd det;
        bool sing;
        wave_lu_det_inv<T, KM>(rv, iv, det, sing);
        if (lane < KM * KM) Rinv[lane] = (c < k && d < k) ? iv : zero<T>();
        if (lane == 0) {
            if (bad) det = zero<Wd>();
            *ratio_st = det;
            static_cast<Wd *>(a.ratio)[w] = det;
            // A zero or non-finite ratio makes the update impossible (Sec. II.A): the
            // stash copy is zeroed so accept skips the walker.  Bad indices are sticky.
            if (bad) atomicOr(a.flags + w, LRX_FLAG_BADINDEX);
            if (sing || is_zero(det) || !finite_v(det)) *ratio_st = zero<Wd>();
        }
    }
}

template <class T, int KM, int NW> size_t propose_lds_bytes(int tau) {
    const size_t TE = (size_t)tau * KM;
    return sizeof(T) * (KM * (TE + 1) + (size_t)NW * 64 + (NW > 1 ? (size_t)NW * TE * KM : 0)) +
           sizeof(int) * (TE + (size_t)tau);
}

template <class T, int KM, int NW, int NI>
__global__ __launch_bounds__(64 * NW) void det_propose_kernel(StepArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    det_propose_walker<T, KM, NW, NI>(a, blockIdx.x, smem, threadIdx.x);
}

// ------------------------------------------------------------------ accept
// Row-streaming pass.  A work-group handles `rows_per_block` rows of one
// walker; each wave takes RB rows at a time, each lane holding NEL elements of
// every row (16-byte vectors, coalesced).  u and C live in LDS, shared by all
// rows of the block.  The row loop is specialised on KC, the walker's rank
// rounded up to a power of two: the padded columns of u and C are zero and the
// padded rows/columns of R^-1 are zero, so padding is exact.
//
// Per row batch: dots p[r][c] = M[q_r,:] . u_c (minus the slot correction),
// one multi-value butterfly reduction (lane l then holds w[r][c] with
// l = r*KC + c), z[r][c] = sum_d R^-1[c][d] w[r][d] on that lane, then
//   DELAYED = false: M[q_r,:] -= sum_c z[r][c] C[:, c]^T  (Eq. det_inv)
//   DELAYED = true : b_tau[q_r][c] = z[r][c]               (Eq. det_b)
template <class T>
__device__ __forceinline__ T lane_bcast(T v, int src) {     // src: wave-uniform
    static_assert(sizeof(T) % 4 == 0, "");
    constexpr int NW = sizeof(T) / 4;
    int w[NW];
    __builtin_memcpy(w, &v, sizeof(T));
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = __builtin_amdgcn_readlane(w[i], src);
    T o;
    __builtin_memcpy(&o, w, sizeof(T));
    return o;
}

template <class T>
struct AcceptCtx {
    T *M, *fa, *fb;
    const T *s_g;           // slot products G[te][c] staged in LDS (delayed update)
    const T *s_u, *s_c, *s_ri;
    T *s_z;                 // per-wave staging of b_tau values (delayed update), kZB batches
    int n, KK, tau, TE, q0, q1, npad, wv, lane;
    bool vec_ok;
};

// Batches of b_tau values a wave stages in LDS before writing them out: on
// this hardware stores share the in-order counter with loads, so a store in
// every batch would make the next batch's prefetched loads wait for it.
constexpr int kZB = 16;

template <class T, int KC, int KM, int NEL, int RB, int MG, bool DELAYED, int PD, bool VEC>
__device__ __forceinline__ void accept_rows(const AcceptCtx<T> &c) {
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;
    constexpr int NV = RB * KC;
    // u is held in registers when its KC x NEL slice is small; else read from LDS per row.
    constexpr bool UREG = KC * NEL * sizeof(T) <= 128;
    const int lane = c.lane;
    const int my_r = (lane % NV) / KC, my_c = lane % KC;
    T rrow[KC];
#pragma unroll
    for (int d = 0; d < KC; ++d) rrow[d] = c.s_ri[my_c * KM + d];
    T ureg[UREG ? KC : 1][UREG ? NEL : 1];
    if constexpr (UREG) {
#pragma unroll
        for (int cc = 0; cc < KC; ++cc)
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                T uv[V];
                ld16<T>(c.s_u + (size_t)cc * c.npad + ch * V * LRX_WAVE + lane * V, uv);
#pragma unroll
                for (int v = 0; v < V; ++v) ureg[cc][ch * V + v] = uv[v];
            }
    }
    const int n = c.n;
    // Software pipeline: the rows of the next PD (1..3) batches, with the
    // slot-row values b_t[q][te] they need, are in flight while the current
    // batch is reduced.
    // Loads are unconditional, from clamped (always valid) addresses, and
    // nothing is selected right after them: a load under a divergent branch,
    // or a select on its result, makes the compiler wait for it on the spot,
    // which would serialise the pipeline.  Out-of-range values are harmless:
    // u is zero beyond n (LDS panel padding) and G is zero beyond the live
    // slot columns, so they add nothing; rows past q1 are computed on a copy
    // of row q1-1 and never stored.  VEC: rows are 16-byte aligned and n is a
    // multiple of the vector width.
    auto load_rows = [&](int qb, T (&x)[RB][NEL], T (&bq)[RB][MG]) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int q = min(qb + r, c.q1 - 1);
            const T *row = c.M + (size_t)q * n;
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int j0 = ch * V * LRX_WAVE + lane * V;
                if constexpr (VEC) {
                    T tmp[V];
                    ld16_nt<T>(row + (j0 < n ? j0 : 0), tmp);
#pragma unroll
                    for (int v = 0; v < V; ++v) x[r][ch * V + v] = tmp[v];
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) x[r][ch * V + v] = row[min(j0 + v, n - 1)];
                }
            }
#pragma unroll
            for (int m = 0; m < MG; ++m) {
                const int te = lane + m * LRX_WAVE;
                bq[r][m] = (DELAYED && c.TE > m * LRX_WAVE) ? c.fb[(size_t)q * c.KK + min(te, c.TE - 1)] : zero<T>();
            }
        }
    };
    const int qstep = kWaves * RB;
    int nzb = 0;                                 // staged batches of b_tau values
    // One batch: dots with u, slot correction, reduction, z, then the store.
    // The batch registers are used in place (no copies between ring buffers:
    // moving a register with a load still in flight would wait for it).
    auto process = [&](int qb, T (&x)[RB][NEL], T (&bv)[RB][MG]) {
        T p[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) p[i] = zero<T>();
#pragma unroll
        for (int cc = 0; cc < KC; ++cc) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                T uv[V];
                if constexpr (UREG) {
#pragma unroll
                    for (int v = 0; v < V; ++v) uv[v] = ureg[cc][ch * V + v];
                } else {
                    ld16<T>(c.s_u + (size_t)cc * c.npad + ch * V * LRX_WAVE + lane * V, uv);
                }
#pragma unroll
                for (int r = 0; r < RB; ++r)
#pragma unroll
                    for (int v = 0; v < V; ++v) p[r * KC + cc] = fmac(x[r][ch * V + v], uv[v], p[r * KC + cc]);
            }
        }
        if (DELAYED) {
            // - sum_t b_t[q][:] (a_t^T u): this lane owns slot columns te = lane + 64 m
#pragma unroll
            for (int m = 0; m < MG; ++m) {
                if (m * LRX_WAVE < c.TE) {
                    // slot products G[te][c] (= a_te . u_c) of the column this lane owns
                    const int te = lane + m * LRX_WAVE;
                    T g[KC];
#pragma unroll
                    for (int cc = 0; cc < KC; ++cc) g[cc] = te < c.TE ? c.s_g[te * KM + cc] : zero<T>();
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int cc = 0; cc < KC; ++cc) p[r * KC + cc] = fmsc(bv[r][m], g[cc], p[r * KC + cc]);
                }
            }
        }
        const T w = wave_sum_multi<T, NV>(p);     // lane l: w[r][c], l mod NV = r*KC + c
        // w[r][d] sits in lane r*KC + d: read it as a wave-uniform value.
        T z = zero<T>();
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            T zr = zero<T>();
#pragma unroll
            for (int d = 0; d < KC; ++d) zr = fmac(rrow[d], lane_bcast(w, r * KC + d), zr);
            z = (my_r == r) ? zr : z;
        }
        if (DELAYED) {
            if (lane < NV) c.s_z[(size_t)c.wv * kZB * NV + nzb * NV + lane] = z;
        } else {
#pragma unroll
            for (int cc = 0; cc < KC; ++cc) {
                T zr[RB];
#pragma unroll
                for (int r = 0; r < RB; ++r) zr[r] = lane_bcast(z, r * KC + cc);
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    T cv[V];
                    ld16<T>(c.s_c + (size_t)cc * c.npad + ch * V * LRX_WAVE + lane * V, cv);
#pragma unroll
                    for (int r = 0; r < RB; ++r)
#pragma unroll
                        for (int v = 0; v < V; ++v) x[r][ch * V + v] = fmsc(zr[r], cv[v], x[r][ch * V + v]);
                }
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int q = qb + r;
                if (q >= c.q1) continue;
                T *row = c.M + (size_t)q * n;
#pragma unroll
                for (int ch = 0; ch < NCH; ++ch) {
                    const int j0 = ch * V * LRX_WAVE + lane * V;
                    T tmp[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) tmp[v] = x[r][ch * V + v];
                    if (c.vec_ok && j0 + V <= n) {
                        st16<T>(row + j0, tmp);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) if (j0 + v < n) row[j0 + v] = tmp[v];
                    }
                }
            }
        }
    };
    // Ring of PD + 1 batches, unrolled so that each buffer keeps its name:
    // consume buffer j, then refill it with the batch PD + 1 steps ahead.
    constexpr int S = PD + 1;
    T x0[RB][NEL], x1[RB][NEL], x2[RB][NEL], x3[RB][NEL];
    T b0[RB][MG], b1[RB][MG], b2[RB][MG], b3[RB][MG];
    int qb = c.q0 + c.wv * RB;
    load_rows(qb, x0, b0);
    if constexpr (S > 1) load_rows(qb + qstep, x1, b1);
    if constexpr (S > 2) load_rows(qb + 2 * qstep, x2, b2);
    if constexpr (S > 3) load_rows(qb + 3 * qstep, x3, b3);
    // b_tau rows of the staged batches go out together (the wave's own LDS
    // region: no block barrier; LDS operations of one wave stay in order).
    auto flush_z = [&]() {
        if constexpr (DELAYED) {
            const int q00 = qb - nzb * qstep;     // first row of the staged batches
            for (int idx = lane; idx < nzb * NV; idx += LRX_WAVE) {
                const int j = idx / NV, v = idx - j * NV;
                const int q = q00 + j * qstep + v / KC;
                if (q < c.q1) c.fb[(size_t)q * c.KK + c.tau * KM + v % KC] = c.s_z[(size_t)c.wv * kZB * NV + idx];
            }
        }
        nzb = 0;
    };
    auto stage = [&](T (&x)[RB][NEL], T (&bq)[RB][MG]) -> bool {
        if (qb >= c.q1) return false;
        process(qb, x, bq);
        load_rows(qb + S * qstep, x, bq);   // clamped past the end
        qb += qstep;
        if (DELAYED && ++nzb == kZB) flush_z();
        return true;
    };
    for (;;) {
        if (!stage(x0, b0)) break;
        if constexpr (S > 1) { if (!stage(x1, b1)) break; }
        if constexpr (S > 2) { if (!stage(x2, b2)) break; }
        if constexpr (S > 3) { if (!stage(x3, b3)) break; }
    }
    if (DELAYED && nzb > 0) flush_z();
}

// Rows [q0, q1) of walker w; rb == 0 marks the block that also does the
// per-walker bookkeeping (log|det|, phase, slot rank, decision, commit).
template <class T, int KM, int NEL, int RB, int MG, bool DELAYED, int PD = 1>
__device__ __forceinline__ void det_accept_rows_block(const StepArgs &a, int w, int rb, int q0, int q1,
                                                      unsigned char *smem, int tid) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;
    const int lane = tid & (LRX_WAVE - 1), wv = tid / LRX_WAVE;
    const int n = a.n, KK = a.K * KM, tau = a.tau, TE = tau * KM;

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
    const uint32_t fl = a.flags[w];
    uint8_t acc;
    if (a.mh_mode >= 0) {   // fused Metropolis decision (identical in every block of the walker)
        acc = mh_decide<Wd>(ratio, fl, a.mh_mode, a.mh_mode == LRX_MH_UNIFORMS ? a.u01[w] : 0.0, a.seed,
                            a.counter, (uint32_t)w + a.rng_base);
    } else {
        acc = a.accept[w];
    }
    const bool take = acc != 0 && fl == 0 && !is_zero(ratio);
    const int kc = k == 1 ? 1 : (k <= 2 ? 2 : (k <= 4 ? 4 : 8));
    if (rb == 0 && tid == 0) {
        if (a.mh_mode >= 0 || (!take && acc)) a.accept[w] = take ? 1 : 0;   // skipped: no occupancy commit
        if (take && a.occ) {   // fused occupancy commit
            for (int c = 0; c < k; ++c) {
                const int e = a.rows[w * KM + c], sl = a.slot[w * KM + c];
                if (e < 0 || e >= n || sl < 0 || sl >= a.n_empty) continue;
                int32_t *po = a.occ + (size_t)w * n + e;
                int32_t *pe = a.empty + (size_t)w * a.n_empty + sl;
                const int32_t t = *po;
                *po = *pe;
                *pe = t;
            }
        }
    }

    if (!take) {
        // A rejected walker's slot contributes nothing: its rank is 0, so the
        // propose and the flush skip its a-columns, and its b-columns are zero
        // for the slot correction of the following accepts.
        if (DELAYED) {
            for (int idx = tid; idx < KM * (q1 - q0); idx += kThreads) {
                int c = idx / (q1 - q0), q = q0 + idx - c * (q1 - q0);
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

    // Staging: every load is issued (unrolled, from clamped addresses) before
    // the first one is consumed, so the set-up costs one memory latency.
    constexpr int NPAD = NCH * V * LRX_WAVE;    // padded row length held in LDS
    const int npad = NPAD;
    T *s_u = reinterpret_cast<T *>(smem);                   // [KM][npad]
    T *s_c = DELAYED ? s_u : s_u + (size_t)KM * npad;       // [KM][npad], plain update only
    T *s_ri = s_c + (size_t)KM * npad;                      // [KM*KM]
    T *s_g = s_ri + KM * KM;                                // [TE][KM], delayed update only
    T *s_z = s_g + (DELAYED ? (size_t)TE * KM : 0);         // [kWaves][kZB * RB * KM], delayed update only
    constexpr int UIT = (KM * NPAD + kThreads - 1) / kThreads;
    constexpr int GIT = DELAYED ? KM : 1;     // TE * KM <= 256 KM (the C ABI keeps K * KM <= 256)
    T ub[UIT], cb[DELAYED ? 1 : UIT];
#pragma unroll
    for (int it = 0; it < UIT; ++it) {
        const int idx = tid + it * kThreads;
        const int c = min(idx / NPAD, KM - 1), j = min(idx % NPAD, n - 1);
        ub[it] = u[(size_t)c * n + j];
        if constexpr (!DELAYED) cb[it] = C[(size_t)c * n + j];
    }
    const T rv = Rinv[tid < KM * KM ? tid : 0];
    T gb[GIT];
    const int TEK = TE * KM;
#pragma unroll
    for (int it = 0; it < GIT; ++it) {
        const int idx = tid + it * kThreads;
        gb[it] = (DELAYED && it * kThreads < TEK) ? G[min(idx, TEK - 1)] : zero<T>();
    }
#pragma unroll
    for (int it = 0; it < UIT; ++it) {
        const int idx = tid + it * kThreads;
        if (idx < kc * NPAD) {
            const int c = idx / NPAD, j = idx % NPAD;
            const bool ok = c < k && j < n;
            s_u[idx] = ok ? ub[it] : zero<T>();
            if constexpr (!DELAYED) s_c[idx] = ok ? cb[it] : zero<T>();
        }
    }
    if (tid < KM * KM) {
        const int c = tid / KM, d = tid - c * KM;
        s_ri[tid] = (c < k && d < k) ? rv : zero<T>();
    }
#pragma unroll
    for (int it = 0; it < GIT; ++it) {
        const int idx = tid + it * kThreads;
        if (DELAYED && idx < TEK) s_g[idx] = gb[it];
    }
    if (DELAYED && kc < KM) {   // b_tau columns beyond kc are zero (a_tau is written by the propose)
        for (int idx = tid; idx < (KM - kc) * (q1 - q0); idx += kThreads) {
            const int c = kc + idx / (q1 - q0), q = q0 + idx % (q1 - q0);
            fb[(size_t)q * KK + tau * KM + c] = zero<T>();
        }
    }
    __syncthreads();

    AcceptCtx<T> ctx{M, fa, fb, s_g, s_u, s_c, s_ri, s_z, n, KK, tau, TE, q0, q1, npad, wv, lane, a.aligned != 0};
    if (ctx.vec_ok) {
        if (kc == 1) {
            accept_rows<T, 1, KM, NEL, RB, MG, DELAYED, PD, true>(ctx);
        } else if (kc == 2) {
            if constexpr (KM >= 2) accept_rows<T, 2, KM, NEL, RB, MG, DELAYED, PD, true>(ctx);
        } else if (kc == 4) {
            if constexpr (KM >= 4) accept_rows<T, 4, KM, NEL, RB, MG, DELAYED, PD, true>(ctx);
        } else {
            if constexpr (KM >= 8) accept_rows<T, 8, KM, NEL, RB, MG, DELAYED, PD, true>(ctx);
        }
    } else {
        if (kc == 1) {
            accept_rows<T, 1, KM, NEL, RB, MG, DELAYED, PD, false>(ctx);
        } else if (kc == 2) {
            if constexpr (KM >= 2) accept_rows<T, 2, KM, NEL, RB, MG, DELAYED, PD, false>(ctx);
        } else if (kc == 4) {
            if constexpr (KM >= 4) accept_rows<T, 4, KM, NEL, RB, MG, DELAYED, PD, false>(ctx);
        } else {
            if constexpr (KM >= 8) accept_rows<T, 8, KM, NEL, RB, MG, DELAYED, PD, false>(ctx);
        }
    }
}

template <class T, int KM, int NEL, int RB, int MG, bool DELAYED>
__global__ __launch_bounds__(kThreads) void det_accept_kernel(StepArgs a, int rows_per_block, int blocks_per_walker) {
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / blocks_per_walker;
    const int rb = lb - w * blocks_per_walker;
    if (w >= a.W) return;
    const int q0 = rb * rows_per_block;
    det_accept_rows_block<T, KM, NEL, RB, MG, DELAYED>(a, w, rb, q0, min(a.n, q0 + rows_per_block), smem, threadIdx.x);
}

// ------------------------------------------------------------------ Metropolis
template <class Wd>
__global__ void metropolis_kernel(int W, const Wd *ratio, const double *u01, uint64_t seed,
                                  uint64_t counter, int mode, const uint32_t *flags, uint8_t *accept) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= W) return;
    accept[w] = mh_decide<Wd>(ratio[w], flags[w], mode, mode == LRX_MH_UNIFORMS ? u01[w] : 0.0, seed, counter,
                              (uint32_t)w);
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

// Dynamic LDS of det_accept_rows_block: u (and C for the plain update) panels
// padded to whole 16-byte chunks per lane, R^-1, and the slot products G.
template <class T, int KM, int NEL, bool DELAYED, int RB = 8> size_t accept_lds_bytes(int K) {
    constexpr size_t npad = (size_t)(NEL / vec16<T>()) * vec16<T>() * LRX_WAVE;
    return sizeof(T) * ((DELAYED ? 1 : 2) * KM * npad + KM * KM +
                        (DELAYED ? (size_t)K * KM * KM + (size_t)kWaves * kZB * RB * KM : 0));
}

// Rows per wave batch: the RB x NEL row values of PD + 1 batches plus the
// RB x KM partial dot products stay within a small register budget (batches
// of one or two rows measured fastest: occupancy matters more than batch size).
template <class T, int NEL, int KM, int PD = 1> constexpr int rows_per_batch() {
    constexpr int per_row = ((PD + 1) * NEL + KM) * (int)sizeof(T);
    constexpr int budget = 192 + (PD - 1) * 128;
    return 8 * per_row <= budget ? 8 : (4 * per_row <= budget ? 4 : (2 * per_row <= budget ? 2 : 1));
}

}  // namespace lrxdet
}  // namespace
