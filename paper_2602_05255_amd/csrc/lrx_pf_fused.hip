// Plain Pfaffian hop update with a delay of one accepted step (Eq. pf_inv, k = 1),
// on full or packed skew storage, and the read-out of A^-1 for every layout.
//
// State (LRX_LAYOUT_FUSED / LRX_LAYOUT_PACKED): M0 plus at most one pending
// rank-2 update per walker, kept as slot 0 of the delayed form of
// Eq. pf_delayed_Ainv: a = [A^-1 x, col], R^-1 = [[0, -1/r], [1/r, 0]], so that
//   A^-1 = M0 + a R^-1 a^T,  entry (q, j) += (col_q ax_j - ax_q col_j) / r.
// The propose (lrx_pf.hip) reads col_i of A^-1 through that form.  An accepted
// step makes one pass over M0: every entry takes the pending update (computed
// on the ordered index pair and negated below the diagonal, so M0 stays exactly
// skew), is written back, and the new ax = (M0 + pending) x is formed from the
// same values.  The step's own update then becomes the new pending one.  HBM per
// accepted step: read + write of M0 (2 n^2 elements, full storage) instead of
// the three passes of the plain update (A^-1 x, then read + write).
//
// Packed storage holds the 64 x 64 tiles on and above the diagonal only.  The
// pass is one work-group per tile; A^-1 x needs both triangles, so a tile
// (I, J), I < J, adds its row dots to ax over rows I and its negated column dots
// (A^-1[j][q] = -A^-1[q][j]) over rows J.  These per-tile partials go to the
// workspace and are summed in a fixed order by the commit kernel.
#include "lrx_common.hpp"
#include "lrx_internal.hpp"
#include "lrx_flush_impl.hpp"

namespace {

using lrx::StepArgs;

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / LRX_WAVE;
constexpr int KA = 2;                   // columns of a per pending update (k = 1)
constexpr int TS = LRX_PACK_TILE;       // packed tile edge

// Metropolis decision (fused mode) or the caller's, identical in every block of
// a walker; the walker's first block records it and commits the occupancy.
template <class Wd>
__device__ __forceinline__ bool pf_take(const StepArgs &a, int w, bool first, int tid, const uint8_t *st) {
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.L.ratio);
    const uint32_t fl = a.flags[w];
    uint8_t acc;
    if (a.mh_mode >= 0)
        acc = mh_decide<Wd>(ratio, fl, a.mh_mode, a.mh_mode == LRX_MH_UNIFORMS ? a.u01[w] : 0.0, a.seed, a.counter,
                            (uint32_t)w + a.rng_base);
    else
        acc = a.accept[w];
    const bool take = acc != 0 && fl == 0 && !is_zero(ratio);
    if (first && tid == 0) {
        if (a.mh_mode >= 0 || (!take && acc)) a.accept[w] = take ? 1 : 0;   // skipped: no occupancy commit
        if (take && a.occ) {
            const int e = a.rows[w * a.KM], sl = a.slot[w * a.KM];
            if (a.k[w] == 1 && e >= 0 && e < a.n && sl >= 0 && sl < a.n_empty) {
                int32_t *po = a.occ + (size_t)w * a.n + e;
                int32_t *pe = a.empty + (size_t)w * a.n_empty + sl;
                const int32_t t = *po;
                *po = *pe;
                *pe = t;
            }
        }
    }
    return take;
}

// Pending entry (q, j) from the ordered pair: (c_lo p_hi - p_lo c_hi) / r,
// negated below the diagonal, zero on it.
template <class T>
__device__ __forceinline__ T pend_entry(bool up, bool diag, T cq, T pq, T cj, T pj, T ir) {
    const T c_lo = up ? cq : cj, p_lo = up ? pq : pj;
    const T c_hi = up ? cj : cq, p_hi = up ? pj : pq;
    const T g = (c_lo * p_hi - p_lo * c_hi) * ir;
    return diag ? zero<T>() : (up ? g : -g);
}

// ------------------------------------------------------------------ full storage pass
// Rows [q0, q1) of walker w; each wave takes RB rows at a time, a lane holding
// NEL entries of each (16-byte vectors).  Slot 1 column 0 receives ax; the
// commit kernel moves it to slot 0 once every block of the walker has read the
// old pending vectors.
template <class T, int NEL, int RB>
__global__ __launch_bounds__(kThreads) void pf_fused_rows_kernel(StepArgs a, int rows_per_block, int bpw) {
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
    const T *x = static_cast<const T *>(a.u) + (size_t)w * n;
    T *fa = static_cast<T *>(a.fa) + (size_t)w * a.K * KA * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * a.K * KA * KA;
    const uint8_t *st = a.stash + (size_t)w * a.L.stride;
    const int *kslot = reinterpret_cast<const int *>(st + a.L.kslot);
    if (!pf_take<Wd>(a, w, rb == 0, tid, st)) return;
    const bool pend = a.tau > 0 && kslot[0] != 0;
    const T ir = pend ? rinv[2] : zero<T>();          // R^-1[1][0] = 1/r
    const int npad = NCH * V * 64;
    T *s_x = reinterpret_cast<T *>(smem);             // [npad] x
    T *s_p = s_x + npad;                              // [npad] pending ax
    T *s_c = s_p + npad;                              // [npad] pending col
    for (int j = tid; j < npad; j += kThreads) {
        const bool in = j < n;
        s_x[j] = in ? x[j] : zero<T>();
        s_p[j] = (pend && in) ? fa[j] : zero<T>();
        s_c[j] = (pend && in) ? fa[n + j] : zero<T>();
    }
    __syncthreads();
    const bool vec_ok = a.aligned != 0;
    T *ax_new = fa + (size_t)KA * n;                  // slot 1, column 0
    for (int qb = q0 + wv * RB; qb < q1; qb += kWaves * RB) {
        T p[RB];
#pragma unroll
        for (int r = 0; r < RB; ++r) p[r] = zero<T>();
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch) {
            const int j0 = ch * V * 64 + lane * V;
            T xv[V], pj[V], cj[V];
            ld16<T>(s_x + j0, xv);
            ld16<T>(s_p + j0, pj);
            ld16<T>(s_c + j0, cj);
            const bool full = vec_ok && j0 + V <= n;
#pragma unroll
            for (int r = 0; r < RB; ++r) {
                const int q = qb + r;
                if (q >= q1) continue;                 // wave-uniform
                T *row = M + (size_t)q * n;
                T tmp[V];
                if (full) {
                    ld16<T>(row + j0, tmp);
                } else {
#pragma unroll
                    for (int v = 0; v < V; ++v) tmp[v] = (j0 + v < n) ? row[j0 + v] : zero<T>();
                }
                if (pend) {                            // walker-uniform
                    const T pq = s_p[q], cq = s_c[q];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        const int j = j0 + v;
                        tmp[v] = tmp[v] + pend_entry<T>(q < j, q == j, cq, pq, cj[v], pj[v], ir);
                    }
                    if (full) {
                        st16<T>(row + j0, tmp);
                    } else {
#pragma unroll
                        for (int v = 0; v < V; ++v) if (j0 + v < n) row[j0 + v] = tmp[v];
                    }
                }
#pragma unroll
                for (int v = 0; v < V; ++v) p[r] = fmac(tmp[v], xv[v], p[r]);
            }
        }
        const T tot = wave_sum_multi<T, RB>(p);
        if (lane < RB) {
            const int q = qb + lane;
            if (q < q1) ax_new[q] = tot;
        }
    }
}

// ------------------------------------------------------------------ packed storage pass
// One work-group per tile (I <= J) of walker w.  MODE 0 (fused accept): decision,
// pending update, write-back and the tile's partial dots of A^-1 x; MODE 2 (delayed
// accept, Sec. III.C): decision and the partial dots of A_0^-1 x, M0 untouched.
// Thread t holds row t / 4 and 16 consecutive columns.
template <class T, int MODE>
__global__ __launch_bounds__(kThreads) void pf_pk_tile_kernel(StepArgs a, int nt, int ntiles) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NE = 16;                            // entries per thread
    constexpr int SP = TS + 1;                        // padded LDS row of the staged tile
    __shared__ T s_v[6][TS];                          // pending ax, col and x at rows I and J
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / ntiles, t = lb - w * ntiles;
    if (w >= a.W) return;
    int I = 0, p = t;
    while (p >= nt - I) { p -= nt - I; ++I; }
    const int J = I + p;
    const int n = a.n, tid = threadIdx.x;
    T *P = static_cast<T *>(a.inv) + ((size_t)w * ntiles + t) * TS * TS;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * a.K * KA * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * a.K * KA * KA;
    const uint8_t *st = a.stash + (size_t)w * a.L.stride;
    const int *kslot = reinterpret_cast<const int *>(st + a.L.kslot);
    if (!pf_take<Wd>(a, w, t == 0, tid, st)) return;
    const bool pend = MODE == 0 && a.tau > 0 && kslot[0] != 0;
    const T ir = pend ? rinv[2] : zero<T>();
    if (tid < 2 * TS) {
        const int side = tid / TS, rr = tid - side * TS;
        const int q = (side ? J : I) * TS + rr;
        const bool in = q < n;
        s_v[side * 3 + 0][rr] = (pend && in) ? fa[q] : zero<T>();
        s_v[side * 3 + 1][rr] = (pend && in) ? fa[n + q] : zero<T>();
        s_v[side * 3 + 2][rr] = in ? static_cast<const T *>(a.u)[(size_t)w * n + q] : zero<T>();
    }
    __syncthreads();
    const int r = tid >> 2, c0 = (tid & 3) * NE;
    const int q = I * TS + r;
    T v[NE];
    T *prow = P + (size_t)r * TS + c0;
#pragma unroll
    for (int e = 0; e < NE; e += V) {
        T tmp[V];
        ld16<T>(prow + e, tmp);
#pragma unroll
        for (int u = 0; u < V; ++u) v[e + u] = tmp[u];
    }
    if (pend) {
        const T pq = s_v[0][r], cq = s_v[1][r];
#pragma unroll
        for (int e = 0; e < NE; ++e) {
            const int c = c0 + e, j = J * TS + c;
            if (q < n && j < n)
                v[e] = v[e] + pend_entry<T>(I < J || r < c, I == J && r == c, cq, pq, s_v[4][c], s_v[3][c], ir);
        }
#pragma unroll
        for (int e = 0; e < NE; e += V) {
            T tmp[V];
#pragma unroll
            for (int u = 0; u < V; ++u) tmp[u] = v[e + u];
            st16<T>(prow + e, tmp);
        }
    }
    {
        T *part = static_cast<T *>(a.part) + ((size_t)w * ntiles + t) * 2 * TS;
        // row dots over the tile's columns (rows I of A^-1 x)
        T rp = zero<T>();
#pragma unroll
        for (int e = 0; e < NE; ++e) rp = fmac(v[e], s_v[5][c0 + e], rp);
        rp = rp + shfl_xor_v(rp, 1);
        rp = rp + shfl_xor_v(rp, 2);
        if ((tid & 3) == 0) part[r] = rp;
        if (I < J) {
            // column dots (rows J of A^-1 x): A^-1[j][q] = -tile[q][j]
            T *s_t = reinterpret_cast<T *>(smem);     // [TS][SP] staged tile, then [4][TS] partials
#pragma unroll
            for (int e = 0; e < NE; ++e) s_t[r * SP + c0 + e] = v[e];
            __syncthreads();
            const int c = tid & (TS - 1), qt = tid / TS;
            T cp = zero<T>();
#pragma unroll 4
            for (int rr = qt * 16; rr < qt * 16 + 16; ++rr) cp = fmac(s_t[rr * SP + c], s_v[2][rr], cp);
            __syncthreads();
            s_t[qt * TS + c] = cp;
            __syncthreads();
            if (tid < TS) part[TS + tid] = -(s_t[tid] + s_t[TS + tid] + s_t[2 * TS + tid] + s_t[3 * TS + tid]);
        }
    }
}

// ------------------------------------------------------------------ commit
// Fused form (DELAYED = false): a taken walker's new update (ax, col, 1/r)
// becomes its pending slot 0; a walker that was not taken keeps its pending
// update, and at st->slot == 0 its slot 0 is cleared instead.
// Delayed packed form (DELAYED = true, Eq. pf_a): slot tau of a taken walker
// receives a_tau = [A_{tau-1}^-1 x, col] with A_{tau-1}^-1 x = A_0^-1 x (the
// tiles' partial dots) + sum_te a_te h_te (h = R^-1 a^T x, from the propose),
// and R_tau^-1; a rejected walker's slot tau is zeroed.  Either way log|pf| and
// the phase take the ratio of a taken walker.
template <class T, bool PACKED, bool DELAYED = false>
__global__ __launch_bounds__(kThreads) void pf_fused_commit_kernel(StepArgs a, int nt, int ntiles) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x, n = a.n, tid = threadIdx.x;
    uint8_t *st = a.stash + (size_t)w * a.L.stride;
    int *kslot = reinterpret_cast<int *>(st + a.L.kslot);
    const T *col = reinterpret_cast<const T *>(st + a.L.c);
    const T *h = reinterpret_cast<const T *>(st + a.L.g);
    const Wd ratio = *reinterpret_cast<const Wd *>(st + a.L.ratio);
    T *fa = static_cast<T *>(a.fa) + (size_t)w * a.K * KA * n;
    T *rinv = static_cast<T *>(a.fb) + (size_t)w * a.K * KA * KA;
    const int slot = DELAYED ? a.tau : 0, TE = DELAYED ? a.tau * KA : 0;
    T *fs = fa + (size_t)slot * KA * n;               // the slot written by this step
    T *rs = rinv + (size_t)slot * KA * KA;
    const bool take = a.accept[w] != 0 && a.flags[w] == 0 && !is_zero(ratio);
    if (!take) {
        if (DELAYED || a.tau == 0) {
            for (int q = tid; q < KA * n; q += kThreads) fs[q] = zero<T>();
            if (tid < KA * KA) rs[tid] = zero<T>();
            if (tid == 0) kslot[slot] = 0;
        }
        return;
    }
    const T *part = PACKED ? static_cast<const T *>(a.part) + (size_t)w * ntiles * 2 * TS : nullptr;
    for (int q = tid; q < n; q += kThreads) {
        T ax = zero<T>();
        if constexpr (PACKED) {
            const int I = q / TS, rr = q - I * TS;
            for (int Jt = 0; Jt < I; ++Jt)               // tiles (Jt, I) above: negated column dots
                ax = ax + part[(size_t)(Jt * nt - Jt * (Jt - 1) / 2 + (I - Jt)) * 2 * TS + TS + rr];
            const int base = I * nt - I * (I - 1) / 2;
            for (int Jt = I; Jt < nt; ++Jt)              // tiles (I, Jt): row dots
                ax = ax + part[(size_t)(base + Jt - I) * 2 * TS + rr];
        } else {
            ax = fa[(size_t)KA * n + q];
        }
        for (int te = 0; te < TE; ++te) ax = fmac(fa[(size_t)te * n + q], h[te], ax);   // delayed: slot correction
        fs[q] = ax;
        fs[n + q] = col[q];
    }
    if (tid == 0) {
        const T irt = conv<T>(divv(one<Wd>(), ratio));
        rs[0] = zero<T>();
        rs[1] = -irt;
        rs[2] = irt;
        rs[3] = zero<T>();
        kslot[slot] = 1;
        accum_logphase(ratio, a.logabs + w, static_cast<Wd *>(a.phase) + w);
    }
}

// ------------------------------------------------------------------ packed flush
// Upper tiles of M0 += sum_{t < tau} a_t R_t^-1 a_t^T (Eq. pf_delayed_Ainv) on the
// matrix cores: one work-group per stored tile, each wave 16 rows x 64 columns,
// Atilde[q][te] = sum_s a_t[q][s] R_t^-1[s][te mod KA] formed per 4-deep step.
// Only the stored tiles are read and written (half the output of the full-storage
// flush); a diagonal tile's lower half is written as the exact negative of its
// upper half.  Dead slots hold zeros.
template <class T>
__global__ __launch_bounds__(kThreads) void pf_pk_flush_kernel(StepArgs a, int nt, int ntiles) {
    using R = typename Real<T>::type;
    using A4 = typename lrxfl::Acc<R>::type;
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / ntiles, t = lb - w * ntiles;
    if (w >= a.W) return;
    int I = 0, p = t;
    while (p >= nt - I) { p -= nt - I; ++I; }
    const int J = I + p;
    const int n = a.n, TE = a.tau * KA;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, lc = lane & 15, kq = lane >> 4;
    T *P = static_cast<T *>(a.inv) + ((size_t)w * ntiles + t) * TS * TS;
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * a.K * KA * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * a.K * KA * KA;
    const bool diag = I == J;
    A4 re[4], im[4];
    const int rl0 = wv * 16;                          // local row base of this wave
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int cl = jb * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rl = rl0 + lrxfl::acc_row<R>(lane, r);
            const T v = (!diag || rl < cl) ? P[rl * TS + cl] : zero<T>();
            re[jb][r] = lrxfl::re_(v);
            im[jb][r] = lrxfl::im_(v);
        }
    }
    const int qa = I * TS + rl0 + lc;                 // this lane's A-operand row
    for (int te0 = 0; te0 < TE; te0 += 4) {
        const int te = te0 + kq;
        T at = zero<T>();
        if (te < TE && qa < n) {
            const int ts = te / KA, sp = te - ts * KA;
            for (int s2 = 0; s2 < KA; ++s2)
                at = fmac(fa[(size_t)(ts * KA + s2) * n + qa], rinv[(size_t)ts * KA * KA + s2 * KA + sp], at);
        }
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const int j = J * TS + jb * 16 + lc;
            const T av = (te < TE && j < n) ? fa[(size_t)te * n + j] : zero<T>();
            lrxfl::mac<T>(at, av, re[jb], im[jb]);
        }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int cl = jb * 16 + lc, j = J * TS + cl;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int rl = rl0 + lrxfl::acc_row<R>(lane, r), q = I * TS + rl;
            if (q >= n || j >= n) continue;           // entries past n stay zero
            const T v = lrxfl::make_<T>(re[jb][r], im[jb][r]);
            if (!diag) {
                P[rl * TS + cl] = v;
            } else if (rl < cl) {
                P[rl * TS + cl] = v;
                P[cl * TS + rl] = lrxfl::make_<T>(-re[jb][r], -im[jb][r]);
            } else if (rl == cl) {
                P[rl * TS + cl] = zero<T>();
            }
        }
    }
}

// ------------------------------------------------------------------ read-out
// out[q][j] = M0[q][j] + sum_{t < tau} sum_{s,s'} a_t[q][s] R_t^-1[s][s'] a_t[j][s'],
// computed on the ordered pair (lo, hi) and negated below the diagonal.  Dead
// slots hold zeros.  One work-group per 64 x 64 output tile.
template <class T>
__global__ __launch_bounds__(kThreads) void pf_read_inverse_kernel(StepArgs a, T *out, int ntd) {
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int per = ntd * ntd;
    const int w = lb / per, tt = lb - w * per;
    if (w >= a.W) return;
    const int TI = tt / ntd, TJ = tt - TI * ntd;
    const int n = a.n, tid = threadIdx.x, KAw = 2 * a.KM, TE = a.tau * KAw;
    const bool packed = a.layout == LRX_LAYOUT_PACKED;
    const int nt = (n + TS - 1) / TS;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * (packed ? lrx_pk_elems_dev(n) : (size_t)n * n);
    const T *fa = static_cast<const T *>(a.fa) + (size_t)w * a.K * KAw * n;
    const T *rinv = static_cast<const T *>(a.fb) + (size_t)w * a.K * KAw * KAw;
    T *o = out + (size_t)w * n * n;
    const int r = tid >> 2, c0 = (tid & 3) * 16;
    const int q = TI * TS + r;
    if (q >= n) return;
    for (int e = 0; e < 16; ++e) {
        const int j = TJ * TS + c0 + e;
        if (j >= n) break;
        const int lo = min(q, j), hi = max(q, j);
        T v = packed ? M[pk_offset(nt, lo, hi)] : M[(size_t)lo * n + hi];
        for (int t = 0; t < TE; t += KAw)
            for (int s = 0; s < KAw; ++s) {
                T h = zero<T>();
                for (int s2 = 0; s2 < KAw; ++s2)
                    h = fmac(rinv[(size_t)(t / KAw) * KAw * KAw + s * KAw + s2], fa[(size_t)(t + s2) * n + hi], h);
                v = fmac(fa[(size_t)(t + s) * n + lo], h, v);
            }
        o[(size_t)q * n + j] = q < j ? v : (q > j ? -v : zero<T>());
    }
}

// ------------------------------------------------------------------ launchers
template <class T, int NEL> constexpr int fused_rb() {
    constexpr int per_row = NEL * (int)sizeof(T);
    return 8 * per_row <= 512 ? 8 : (4 * per_row <= 512 ? 4 : (2 * per_row <= 512 ? 2 : 1));
}

template <class T, int NEL> hipError_t fused_rows(const StepArgs &a, hipStream_t s) {
    constexpr int RB = fused_rb<T, NEL>();
    constexpr int V = vec16<T>();
    const int npad = (NEL / V) * V * 64;
    // rows per block: at least two row batches per wave, at most ~8 blocks per CU
    int rpb = 2 * kWaves * RB;
    long long blocks = (long long)a.W * ((a.n + rpb - 1) / rpb);
    while (rpb < a.n && blocks > 8 * 256 * 4) {
        rpb *= 2;
        blocks = (long long)a.W * ((a.n + rpb - 1) / rpb);
    }
    const int bpw = (a.n + rpb - 1) / rpb;
    hipLaunchKernelGGL((pf_fused_rows_kernel<T, NEL, RB>), dim3((unsigned)(a.W * bpw)), dim3(kThreads),
                       sizeof(T) * 3 * (size_t)npad, s, a, rpb, bpw);
    return hipGetLastError();
}

template <class T> hipError_t fused_accept_t(const StepArgs &a, hipStream_t s) {
    hipError_t e = hipSuccess;
    const int nt = (a.n + TS - 1) / TS, ntiles = nt * (nt + 1) / 2;
    if (a.layout == LRX_LAYOUT_PACKED) {
        const size_t lds = sizeof(T) * (size_t)TS * (TS + 1);
        const dim3 grid((unsigned)(a.W * ntiles));
        if (a.delay > 0) {   // delayed form on packed storage: A_0^-1 x from the tiles, then slot tau
            hipLaunchKernelGGL((pf_pk_tile_kernel<T, 2>), grid, dim3(kThreads), lds, s, a, nt, ntiles);
            if ((e = hipGetLastError()) != hipSuccess) return e;
            hipLaunchKernelGGL((pf_fused_commit_kernel<T, true, true>), dim3((unsigned)a.W), dim3(kThreads), 0, s, a,
                               nt, ntiles);
            return hipGetLastError();
        }
        hipLaunchKernelGGL((pf_pk_tile_kernel<T, 0>), grid, dim3(kThreads), lds, s, a, nt, ntiles);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL((pf_fused_commit_kernel<T, true>), dim3((unsigned)a.W), dim3(kThreads), 0, s, a, nt, ntiles);
        return hipGetLastError();
    }
    constexpr int V = vec16<T>();
    const int nch = (a.n + V * 64 - 1) / (V * 64);
    if (nch <= 1) e = fused_rows<T, V>(a, s);
    else if (nch <= 2) e = fused_rows<T, 2 * V>(a, s);
    else if (nch <= 4) e = fused_rows<T, 4 * V>(a, s);
    else if constexpr (V <= 2) {
        if (nch <= 8) e = fused_rows<T, 8 * V>(a, s);
        else if constexpr (V == 1) { if (nch <= 16) e = fused_rows<T, 16>(a, s); else return hipErrorInvalidValue; }
        else return hipErrorInvalidValue;
    } else {
        return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((pf_fused_commit_kernel<T, false>), dim3((unsigned)a.W), dim3(kThreads), 0, s, a, nt, ntiles);
    return hipGetLastError();
}

template <class T> hipError_t packed_flush_t(const StepArgs &a, hipStream_t s) {
    const int nt = (a.n + TS - 1) / TS, ntiles = nt * (nt + 1) / 2;
    hipLaunchKernelGGL(pf_pk_flush_kernel<T>, dim3((unsigned)(a.W * ntiles)), dim3(kThreads), 0, s, a, nt, ntiles);
    return hipGetLastError();
}

template <class T> hipError_t read_inverse_t(const StepArgs &a, void *out, hipStream_t s) {
    const int ntd = (a.n + TS - 1) / TS;
    hipLaunchKernelGGL(pf_read_inverse_kernel<T>, dim3((unsigned)(a.W * ntd * ntd)), dim3(kThreads), 0, s, a,
                       static_cast<T *>(out), ntd);
    return hipGetLastError();
}

}  // namespace

namespace lrx {

hipError_t pf_fused_accept(int dtype, const StepArgs &a, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return fused_accept_t<float>(a, s);
        case LRX_F64: return fused_accept_t<double>(a, s);
        case LRX_C64: return fused_accept_t<cf32>(a, s);
        case LRX_C128: return fused_accept_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t pf_fused_flush(int dtype, const StepArgs &a, hipStream_t s) {
    if (a.layout != LRX_LAYOUT_PACKED) return pf_flush(dtype, a, s);   // slot form, full storage
    switch (dtype) {
        case LRX_F32: return packed_flush_t<float>(a, s);
        case LRX_F64: return packed_flush_t<double>(a, s);
        case LRX_C64: return packed_flush_t<cf32>(a, s);
        case LRX_C128: return packed_flush_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

hipError_t pf_read_inverse(int dtype, const StepArgs &a, void *out, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return read_inverse_t<float>(a, out, s);
        case LRX_F64: return read_inverse_t<double>(a, out, s);
        case LRX_C64: return read_inverse_t<cf32>(a, out, s);
        case LRX_C128: return read_inverse_t<cf64>(a, out, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
