// Pfaffian low-rank update kernels (Sec. III of the paper), single-electron
// hops: u = (x, e_i) with x_i = 0 (Eq. pf_rank2), a rank-2 skew update
// A_t = A_{t-1} - u J u^T.
//
// State: M = A^-1 row-major, exactly skew-symmetric.
//   propose   : col = A_{tau-1}^-1[:, i] = -M0[i,:]^T + sum_t a_t R_t^-1 a_t[i,:]^T,
//               r = pf R / pf J = R_12 = 1 + x . col          (Eqs. pf_ratio, pf_R)
//   accept K=0: a_x = M x (pass 1); M += (col a_x^T - a_x col^T)/r (pass 2)   (Eq. pf_inv, k = 1)
//   accept K>0: a_tau = [A_{tau-1}^-1 x, col], R_tau^-1 = [[0,-1/r],[1/r,0]] (Eq. pf_a, Sec. III.C)
//   (the fused and packed layouts' accept is in lrx_pf_fused.hip; their propose is this one,
//   with one pending slot and, packed, M0 read from the upper tiles)
//
// Exact skew symmetry of the plain update: entry (q, j) is computed from the
// ordered pair (min, max) and negated when q > j, so (j, q) receives exactly
// the negative of (q, j) whatever FMA contraction the compiler applies.
#include "lrx_common.hpp"
#include "lrx_internal.hpp"

namespace {

using lrx::StepArgs;
using lrx::HopArgs;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / LRX_WAVE;
constexpr int KA = 2;    // columns of u per hop (k = 1)

// ------------------------------------------------------------------ build hop
// x[j] = f[s'][occ_j] - f[s][occ_j] (j != i), x[i] = 0.
template <class T>
__global__ __launch_bounds__(kThreads) void pf_build_hop_kernel(HopArgs a) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x, n = a.n, KM = a.KM;
    const Wd *f = static_cast<const Wd *>(a.phi);
    T *x = static_cast<T *>(a.out) + (size_t)w * n;
    __shared__ int s_i, s_src, s_dst, s_bad;
    if (threadIdx.x == 0) {
        int kw = a.k[w];
        int e = a.elec[w * KM], sl = a.slot[w * KM];
        int bad = (kw != 1) || e < 0 || e >= n || sl < 0 || sl >= a.n_empty;
        int src = 0, dst = 0;
        if (!bad) {
            src = a.occ[(size_t)w * n + e];
            dst = a.empty[(size_t)w * a.n_empty + sl];
            if (src < 0 || src >= a.sites || dst < 0 || dst >= a.sites) bad = 1;
        }
        s_i = bad ? -1 : e;
        s_src = bad ? 0 : src;
        s_dst = bad ? 0 : dst;
        s_bad = bad;
        if (bad) atomicOr(a.flags + w, LRX_FLAG_BADINDEX);
    }
    __syncthreads();
    const Wd *fs = f + (size_t)s_src * a.sites;
    const Wd *fd = f + (size_t)s_dst * a.sites;
    const int32_t *occ = a.occ + (size_t)w * n;
    for (int j = threadIdx.x; j < n; j += kThreads) {
        T v = zero<T>();
        if (!s_bad && j != s_i) {
            const int oj = occ[j];
            if (oj >= 0 && oj < a.sites) v = conv<T>(fd[oj] - fs[oj]);
        }
        x[j] = v;
    }
}

// ------------------------------------------------------------------ propose
// Slot columns per unrolled round of loads in the column pass of the propose.
constexpr int kPfPropRound = 16;
// The propose runs one work-group of 8 waves per walker.  Where the columns
// fit in fewer threads, the column pass splits the slot columns over groups of
// threads whose partial sums meet in LDS; the slot correction spreads the
// slots over the 8 waves.  Larger work-groups shorten the chain of dependent
// loads further but are harder to place beside the other sub-batches' kernels.
constexpr int kPropThreads = 512;
constexpr int kPropWaves = kPropThreads / LRX_WAVE;

// Columns of the column pass covered at once (whole waves, at most the
// work-group); kPropThreads / pf_prop_cols(n) thread groups share the slots.
__host__ __device__ constexpr int pf_prop_cols(int n) {
    return n <= 64 ? 64 : ((n + 63) / 64 * 64 < kPropThreads ? (n + 63) / 64 * 64 : kPropThreads);
}

// One round of the column pass: c += sum_j fa[r*R + j][q] s_m[r*R + j] over a
// round of kPfPropRound slot columns (clamped addresses; s_m is zero-padded).
template <class T>
__device__ __forceinline__ T pf_prop_round(const T *fa, const T *s_m, int n, int TE, int r, int q, T c) {
    T fv[kPfPropRound];
#pragma unroll
    for (int j = 0; j < kPfPropRound; ++j) fv[j] = fa[(size_t)min(r * kPfPropRound + j, TE - 1) * n + q];
#pragma unroll
    for (int j = 0; j < kPfPropRound; ++j) c = fmac(fv[j], s_m[r * kPfPropRound + j], c);
    return c;
}

// col_q = A0^-1[q][i] = -A0^-1[i][q], from dense or packed skew storage.
template <class T, bool PK>
__device__ __forceinline__ T pf_prop_m(const T *M, int n, int nt, int i, int q) {
    if constexpr (PK) return (i >> 6) <= (q >> 6) ? -M[pk_offset(nt, i, q)] : M[pk_offset(nt, q, i)];
    else return -M[(size_t)i * n + q];
}

// PK: M0 in packed skew storage (upper 64 x 64 tiles, LRX_LAYOUT_PACKED).
template <class T, bool PK>
__global__ __launch_bounds__(kPropThreads) void pf_propose_kernel(StepArgs a) {
    using Wd = typename Wide<T>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = blockIdx.x, n = a.n, tau = a.tau, TE = tau * KA;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * (PK ? lrx_pk_elems_dev(n) : (size_t)n * n);
    const int nt = (n + 63) >> 6;
    const T *x = static_cast<const T *>(a.u) + (size_t)w * n;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * a.K * KA * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * a.K * KA * KA;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    T *col = reinterpret_cast<T *>(st + a.L.c);
    T *h = reinterpret_cast<T *>(st + a.L.g);
    Wd *ratio_st = reinterpret_cast<Wd *>(st + a.L.ratio);

    // Loads go out in unrolled rounds from clamped addresses; the LDS operands
    // they meet are zero-padded to whole rounds, so padded terms add nothing.
    const int TEp = (TE + kPfPropRound - 1) / kPfPropRound * kPfPropRound;
    const int npx = (n + 8 * 64 - 1) / (8 * 64) * (8 * 64);
    const int QW = pf_prop_cols(n), S = kPropThreads / QW;
    T *s_m = reinterpret_cast<T *>(smem);      // [TEp] R_t^-1 a_t[i,:]^T
    T *s_red = s_m + TEp;                      // [kPropWaves]
    T *s_x = s_red + kPropWaves;               // [npx] x
    T *s_part = s_x + npx;                     // [(S - 1) * QW] column partial sums
    // With a hop table the hop vector is built here, x[j] = f[s'][occ_j] -
    // f[s][occ_j] (j != i), and written to x for the accept that follows.
    const bool fused = a.hop_table != nullptr;
    __shared__ int s_i, s_bad, s_src, s_dst;
    if (tid == 0) {
        int i = a.rows[w * a.KM];
        int bad = (a.k[w] != 1) || i < 0 || i >= n;
        int src = 0, dst = 0;
        if (fused && !bad) {
            const int sl = a.slot[w * a.KM];
            if (sl < 0 || sl >= a.n_empty) {
                bad = 1;
            } else {
                src = a.occ[(size_t)w * n + i];
                dst = a.empty[(size_t)w * a.n_empty + sl];
                if (src < 0 || src >= a.sites || dst < 0 || dst >= a.sites) bad = 1;
            }
        }
        s_i = bad ? 0 : i;
        s_bad = bad;
        s_src = bad ? 0 : src;
        s_dst = bad ? 0 : dst;
    }
    __syncthreads();
    const int i = s_i;
    if (fused) {
        const Wd *tab = static_cast<const Wd *>(a.hop_table);
        const Wd *fs = tab + (size_t)s_src * a.sites, *fd = tab + (size_t)s_dst * a.sites;
        const int32_t *occ = a.occ + (size_t)w * n;
        T *xw = const_cast<T *>(x);
        for (int j = tid; j < npx; j += kPropThreads) {
            T v = zero<T>();
            if (j < n && !s_bad && j != i) {
                const int oj = occ[j];
                if (oj >= 0 && oj < a.sites) v = conv<T>(fd[oj] - fs[oj]);
            }
            if (j < n) xw[j] = v;
            s_x[j] = v;
        }
    } else {
        for (int j = tid; j < npx; j += kPropThreads) {
            T v = zero<T>();
            if (j < n) v = x[j];
            s_x[j] = v;
        }
    }
    for (int te = tid; te < TEp; te += kPropThreads) {
        const int t = te / KA, s = te - t * KA;
        T v = zero<T>();
        if (te < TE)
            for (int sp = 0; sp < KA; ++sp) v = fmac(rinv[(size_t)t * KA * KA + s * KA + sp], fa[(size_t)(t * KA + sp) * n + i], v);
        s_m[te] = v;
    }
    __syncthreads();
    // col_q = -A0^-1[i][q] + sum_te fa[te][q] s_m[te]; ratio - 1 = x . col.
    T part = zero<T>();
    const int nr = TEp / kPfPropRound;
    if (S == 1) {
        for (int q = tid; q < n; q += kPropThreads) {
            T c = pf_prop_m<T, PK>(M, n, nt, i, q);
            for (int r = 0; r < nr; ++r) c = pf_prop_round(fa, s_m, n, TE, r, q, c);
            col[q] = c;
            part = fmac(s_x[q], c, part);
        }
    } else {
        // Thread group g takes the rounds r = g, g + S, ... of column q.
        const int g = tid / QW, q = tid - g * QW, qc = min(q, n - 1);
        T c = zero<T>();
        if (n > 0 && g < S) {
            if (g == 0) c = pf_prop_m<T, PK>(M, n, nt, i, qc);
            for (int r = g; r < nr; r += S) c = pf_prop_round(fa, s_m, n, TE, r, qc, c);
            if (g > 0) s_part[(g - 1) * QW + q] = c;
        }
        __syncthreads();
        if (g == 0 && q < n) {
            for (int gp = 1; gp < S; ++gp) c = c + s_part[(gp - 1) * QW + q];
            col[q] = c;
            part = fmac(s_x[q], c, part);
        }
    }
    part = wave_sum(part);
    if (lane == 0) s_red[wv] = part;
    // h_t = R_t^-1 (a_t^T x): the slot correction of A_{tau-1}^-1 x.
    if (a.K > 0) {
        for (int t = wv; t < tau; t += kPropWaves) {
            T g[KA];
#pragma unroll
            for (int s = 0; s < KA; ++s) g[s] = zero<T>();
            for (int q0 = 0; q0 < n; q0 += 8 * 64) {
                T fv[8][KA];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const int q = min(q0 + j * 64 + lane, n - 1);
#pragma unroll
                    for (int s = 0; s < KA; ++s) fv[j][s] = fa[(size_t)(t * KA + s) * n + q];
                }
#pragma unroll
                for (int j = 0; j < 8; ++j)
#pragma unroll
                    for (int s = 0; s < KA; ++s) g[s] = fmac(fv[j][s], s_x[q0 + j * 64 + lane], g[s]);
            }
#pragma unroll
            for (int s = 0; s < KA; ++s) g[s] = wave_sum(g[s]);
            if (lane < KA) {
                T v = zero<T>();
#pragma unroll
                for (int sp = 0; sp < KA; ++sp)
                    v = fmac(rinv[(size_t)t * KA * KA + lane * KA + sp], g[sp], v);
                h[t * KA + lane] = v;
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        T tot = one<T>();
        for (int q = 0; q < kPropWaves; ++q) tot = tot + s_red[q];
        Wd r = conv<Wd>(tot);
        if (s_bad) r = zero<Wd>();
        static_cast<Wd *>(a.ratio)[w] = r;
        *ratio_st = (s_bad || is_zero(r) || !finite_v(r)) ? zero<Wd>() : r;
        if (s_bad) atomicOr(a.flags + w, LRX_FLAG_BADINDEX);
    }
}

// Slot columns covered by one round of slot-correction loads of a wave in
// pf_rowdot_kernel with RB rows per batch (8 per lane); the staged h is padded
// to a multiple of it.
template <int RB> constexpr int pf_slot_round() { return 8 * (64 / RB); }

// Value select (a conditional on two named complex values would select their
// addresses and push them to scratch memory).
template <class T> __device__ __forceinline__ T pick(bool c, T a, T b) { return c ? a : b; }

// ------------------------------------------------------------------ row dots
// ax[q] = M[q,:] . x (+ sum_te fa[te][q] h[te] in the delayed form).
// DELAYED: writes slot tau = [ax, col] and R_tau^-1; else stores ax in the stash.
template <class T, int NEL, int RB, bool DELAYED>
__global__ __launch_bounds__(kThreads) void pf_rowdot_kernel(StepArgs a, int rows_per_block, int bpw) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / bpw, rb = lb - w * bpw;
    if (w >= a.W) return;
    const int n = a.n, tau = a.tau, TE = tau * KA;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int q0 = rb * rows_per_block, q1 = min(n, q0 + rows_per_block);
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    const T *x = static_cast<const T *>(a.u) + (size_t)w * n;
    T *fa = static_cast<T *>(a.fa) + (size_t)w * a.K * KA * n;
    T *rinv = static_cast<T *>(a.fb) + (size_t)w * a.K * KA * KA;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    const T *col = reinterpret_cast<const T *>(st + a.L.c);
    const T *h = reinterpret_cast<const T *>(st + a.L.g);
    T *ax = reinterpret_cast<T *>(st + a.L.ax);
    int *kslot = reinterpret_cast<int *>(st + a.L.kslot);
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.L.ratio);
    const uint32_t fl = a.flags[w];
    uint8_t acc;
    if (a.mh_mode >= 0) {   // fused Metropolis decision (identical in every block of the walker)
        acc = mh_decide<Wd>(ratio, fl, a.mh_mode, a.mh_mode == LRX_MH_UNIFORMS ? a.u01[w] : 0.0, a.seed,
                            a.counter, (uint32_t)w + a.rng_base);
    } else {
        acc = a.accept[w];
    }
    const bool take = acc != 0 && fl == 0 && !is_zero(ratio);
    if (rb == 0 && tid == 0) {
        if (a.mh_mode >= 0 || (!take && acc)) a.accept[w] = take ? 1 : 0;   // skipped: no occupancy commit
        if (take && a.occ) {   // fused occupancy commit of the hop
            int kw = a.k[w];
            kw = (kw < 1 || kw > a.KM) ? 0 : kw;
            for (int c = 0; c < kw; ++c) {
                const int e = a.rows[w * a.KM + c], sl = a.slot[w * a.KM + c];
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
        if (DELAYED) {
            for (int q = q0 + tid; q < q1; q += kThreads) {
                fa[(size_t)(tau * KA) * n + q] = zero<T>();
                fa[(size_t)(tau * KA + 1) * n + q] = zero<T>();
            }
            if (rb == 0 && tid < KA * KA) rinv[(size_t)tau * KA * KA + tid] = zero<T>();
            if (rb == 0 && tid == 0) kslot[tau] = 0;
        }
        return;
    }
    if (DELAYED && rb == 0) {
        if (tid == 0) {
            accum_logphase(ratio, a.logabs + w, static_cast<Wd *>(a.phase) + w);
            kslot[tau] = 1;
        }
        if (tid < KA * KA) {
            // R = [[0, r], [-r, 0]]  ->  R^-1 = [[0, -1/r], [1/r, 0]]
            const Wd ir = divv(one<Wd>(), ratio);
            T v = zero<T>();
            if (tid == 1) v = conv<T>(-ir);
            if (tid == 2) v = conv<T>(ir);
            rinv[(size_t)tau * KA * KA + tid] = v;
        }
    }
    const int npad = NCH * V * 64;
    T *s_x = reinterpret_cast<T *>(smem);        // [npad]
    // Slot correction sum_te fa[te][q] h[te] of the batch's rows, spread over
    // the wave: lane l takes row l mod RB and the slot columns te = l / RB
    // (mod 64 / RB), CU of them per round of loads.  Its loads go out with the
    // batch's row loads and its partial joins the row's dot partial before the
    // one reduction.  h is staged in LDS padded with zeros to whole rounds, so
    // a padded column (its fa load clamped to a live one) adds nothing.
    constexpr int NSL = 64 / RB;
    constexpr int CU = pf_slot_round<RB>() / NSL;
    const int TEp = DELAYED ? (TE + pf_slot_round<RB>() - 1) / pf_slot_round<RB>() * pf_slot_round<RB>() : 0;
    T *s_h = s_x + npad;                         // [TEp], delayed form only
    for (int j = tid; j < npad; j += kThreads) s_x[j] = j < n ? x[j] : zero<T>();
    for (int te = tid; te < TEp; te += kThreads) {
        T v = zero<T>();
        if (te < TE) v = h[te];
        s_h[te] = v;
    }
    __syncthreads();
    const bool vec_ok = a.aligned != 0;
    const int cr = lane % RB, csl = lane / RB;
    for (int qb = q0 + wv * RB; qb < q1; qb += kWaves * RB) {
        T p[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) p[r] = zero<T>();
        if (DELAYED) {
            const int qc = min(qb + cr, q1 - 1);     // rows past q1 are never stored
            T corr = zero<T>();
            for (int t0 = 0; t0 < TE; t0 += CU * NSL) {
                T fv[CU], hv[CU];
#pragma unroll
                for (int j = 0; j < CU; ++j) {
                    const int te = t0 + csl + j * NSL;
                    fv[j] = fa[(size_t)min(te, TE - 1) * n + qc];
                    hv[j] = s_h[te];
                }
#pragma unroll
                for (int j = 0; j < CU; ++j) corr = fmac(fv[j], hv[j], corr);
            }
#pragma unroll
            for (int r = 0; r < RB; ++r) p[r] = pick(cr == r, corr, p[r]);
        }
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int j0 = ch * V * 64 + lane * V;
            T xv[V];
            ld16<T>(s_x + j0, xv);
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int q = qb + r;
                const T *row = M + (size_t)q * n;
                T tmp[V];
                if (q < q1 && vec_ok && j0 + V <= n) {
                    ld16_nt<T>(row + j0, tmp);   // streamed once per step
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) tmp[v] = (q < q1 && j0 + v < n) ? row[j0 + v] : zero<T>();
                }
#pragma unroll
                for (int v = 0; v < V; ++v) p[r] = fmac(tmp[v], xv[v], p[r]);
            }
        }
        const T tot = wave_sum_multi<T, RB>(p);
        // lane r (< RB) holds the dot of row qb + r, slot correction included
        if (lane < RB) {
            const int q = qb + lane;
            if (q < q1) {
                if (DELAYED) {
                    fa[(size_t)(tau * KA) * n + q] = tot;
                    fa[(size_t)(tau * KA + 1) * n + q] = col[q];
                } else {
                    ax[q] = tot;
                }
            }
        }
    }
}

// ------------------------------------------------------------------ plain pass 2
// M[q][j] += (col_q ax_j - ax_q col_j)/r, computed on the ordered pair.
template <class T, int NEL, int RB>
__global__ __launch_bounds__(kThreads) void pf_update_kernel(StepArgs a, int rows_per_block, int bpw) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / bpw, rb = lb - w * bpw;
    if (w >= a.W) return;
    const int n = a.n;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int q0 = rb * rows_per_block, q1 = min(n, q0 + rows_per_block);
    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    const T *col = reinterpret_cast<const T *>(st + a.L.c);
    const T *ax = reinterpret_cast<const T *>(st + a.L.ax);
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.L.ratio);
    const bool take = a.accept[w] != 0 && a.flags[w] == 0 && !is_zero(ratio);
    if (!take) return;
    if (rb == 0 && tid == 0) accum_logphase(ratio, a.logabs + w, static_cast<Wd *>(a.phase) + w);
    const T ir = conv<T>(divv(one<Wd>(), ratio));
    const int npad = NCH * V * 64;
    T *s_c = reinterpret_cast<T *>(smem);
    T *s_a = s_c + npad;
    for (int j = tid; j < npad; j += kThreads) {
        s_c[j] = j < n ? col[j] : zero<T>();
        s_a[j] = j < n ? ax[j] : zero<T>();
    }
    __syncthreads();
    const bool vec_ok = a.aligned != 0;
    for (int qb = q0 + wv * RB; qb < q1; qb += kWaves * RB) {
#pragma unroll
        for (int r = 0; r < RB; ++r) {
            const int q = qb + r;
            if (q >= q1) continue;
            T *row = M + (size_t)q * n;
            const T cq = s_c[q], aq = s_a[q];
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch) {
                const int j0 = ch * V * 64 + lane * V;
                T tmp[V], cj[V], aj[V];
                ld16<T>(s_c + j0, cj);
                ld16<T>(s_a + j0, aj);
                const bool full = vec_ok && j0 + V <= n;
                if (full) ld16<T>(row + j0, tmp);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) tmp[v] = (j0 + v < n) ? row[j0 + v] : zero<T>();
                }
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int j = j0 + v;
                    const bool up = q < j;
                    const T c_lo = up ? cq : cj[v], a_lo = up ? aq : aj[v];
                    const T c_hi = up ? cj[v] : cq, a_hi = up ? aj[v] : aq;
                    const T g = (c_lo * a_hi - a_lo * c_hi) * ir;
                    T d = up ? g : -g;
                    if (q == j) d = zero<T>();
                    tmp[v] = tmp[v] + d;
                }
                if (full) st16<T>(row + j0, tmp);
                else {
#pragma unroll
                    for (int v = 0; v < V; ++v) if (j0 + v < n) row[j0 + v] = tmp[v];
                }
            }
        }
    }
}

// ------------------------------------------------------------------ launchers
template <class T> hipError_t build_hop_t(const HopArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(pf_build_hop_kernel<T>, dim3(a.W), dim3(kThreads), 0, s, a);
    return hipGetLastError();
}

template <class T> hipError_t propose_t(const StepArgs &a, hipStream_t s) {
    const size_t tep = ((size_t)a.tau * KA + kPfPropRound - 1) / kPfPropRound * kPfPropRound;
    const size_t npx = ((size_t)a.n + 8 * 64 - 1) / (8 * 64) * (8 * 64);
    const size_t qw = pf_prop_cols(a.n);
    size_t lds = sizeof(T) * (tep + kPropWaves + npx + (kPropThreads / qw - 1) * qw);
    if (a.layout == LRX_LAYOUT_PACKED)
        hipLaunchKernelGGL((pf_propose_kernel<T, true>), dim3(a.W), dim3(kPropThreads), lds, s, a);
    else
        hipLaunchKernelGGL((pf_propose_kernel<T, false>), dim3(a.W), dim3(kPropThreads), lds, s, a);
    return hipGetLastError();
}

template <class T, int NEL> constexpr int pf_rb() {
    constexpr int per_row = NEL * (int)sizeof(T);
    return 8 * per_row <= 512 ? 8 : (4 * per_row <= 512 ? 4 : (2 * per_row <= 512 ? 2 : 1));
}

inline void block_shape(int W, int n, int rows_min, int &rpb, int &bpw) {
    rpb = rows_min;
    long long blocks = (long long)W * ((n + rpb - 1) / rpb);
    while (rpb < n && blocks > 8 * 256 * 4) {
        rpb *= 2;
        blocks = (long long)W * ((n + rpb - 1) / rpb);
    }
    bpw = (n + rpb - 1) / rpb;
}

template <class T, int NEL> hipError_t accept_nel(const StepArgs &a, hipStream_t s) {
    constexpr int RB = pf_rb<T, NEL>();
    constexpr int V = vec16<T>();
    const int npad = (NEL / V) * V * 64;
    int rpb, bpw;
    // at least two row batches per wave: the block's set-up (x and h staged
    // in LDS) is shared by twice the rows, and half as many blocks queue up
    block_shape(a.W, a.n, 2 * kWaves * RB, rpb, bpw);
    const dim3 grid((unsigned)(a.W * bpw));
    const size_t lds1 = sizeof(T) * ((size_t)npad + ((size_t)a.tau * KA + pf_slot_round<RB>() - 1) / pf_slot_round<RB>() * pf_slot_round<RB>());
    if (a.K > 0) {
        hipLaunchKernelGGL((pf_rowdot_kernel<T, NEL, RB, true>), grid, dim3(kThreads), lds1, s, a, rpb, bpw);
        return hipGetLastError();
    }
    hipLaunchKernelGGL((pf_rowdot_kernel<T, NEL, RB, false>), grid, dim3(kThreads), lds1, s, a, rpb, bpw);
    const size_t lds2 = sizeof(T) * 2 * (size_t)npad;
    hipLaunchKernelGGL((pf_update_kernel<T, NEL, RB>), grid, dim3(kThreads), lds2, s, a, rpb, bpw);
    return hipGetLastError();
}

template <class T> hipError_t accept_t(const StepArgs &a, hipStream_t s) {
    constexpr int V = vec16<T>();
    const int nch = (a.n + V * 64 - 1) / (V * 64);
    if (nch <= 1) return accept_nel<T, V>(a, s);
    if (nch <= 2) return accept_nel<T, 2 * V>(a, s);
    if (nch <= 4) return accept_nel<T, 4 * V>(a, s);
    if constexpr (V <= 2) { if (nch <= 8) return accept_nel<T, 8 * V>(a, s); }
    if constexpr (V == 1) { if (nch <= 16) return accept_nel<T, 16>(a, s); }
    return hipErrorInvalidValue;
}

}  // namespace

namespace lrx {

hipError_t pf_build_hop(int dtype, const HopArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return build_hop_t<float>(a, s);
        case LRX_F64: return build_hop_t<double>(a, s);
        case LRX_C64: return build_hop_t<cf32>(a, s);
        case LRX_C128: return build_hop_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t pf_propose(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return propose_t<float>(a, s);
        case LRX_F64: return propose_t<double>(a, s);
        case LRX_C64: return propose_t<cf32>(a, s);
        case LRX_C128: return propose_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t pf_accept(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return accept_t<float>(a, s);
        case LRX_F64: return accept_t<double>(a, s);
        case LRX_C64: return accept_t<cf32>(a, s);
        case LRX_C128: return accept_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
