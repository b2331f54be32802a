// Initialisation and periodic refresh: from-scratch factorisation in FP64 /
// complex128 (the paper advises double precision for the stored inverse and
// the determinant, Sec. I and the stability remark of Sec. II.A).
//
//   DET: B = A^T is inverted by blocked Gauss-Jordan elimination with partial
//        pivoting, giving M = B^-1 = A^-T directly in the state layout;
//        log|det A| and its phase come from the pivots.
//   PF : log|pf A| and phase by Parlett-Reid elimination (a congruence that
//        brings the largest entry of the leading column next to the diagonal,
//        pf(B A B^T) = det(B) pf(A), then the block Schur step of Appendix A,
//        Eq. pf_block, which splits off a 2x2 block whose Pfaffian is its (0,1)
//        entry); A^-1 from the same factorisation, A = Pi U^T D U Pi^T, as
//        Pi U^-1 D^-1 U^-T Pi^T, then M = (X - X^T)/2.
//
// Two-level blocked Gauss-Jordan (all in the workspace X, row-major).  The
// columns are taken in outer panels of up to 64; inside an outer panel, blocks
// of 4 CPT columns (the whole outer panel for real data up to n = 512) are
// eliminated one at a time and their transform is applied to the other
// columns of the outer panel only.  The outer panel's columns then hold
// Zt + E_P, with I + Zt E_P^T the composite transform of the whole outer
// panel, and every remaining column gets it in one MFMA GEMM of inner
// dimension 64 (gj_outer_kernel).  Per block:
//   block kernel : in-place Gauss-Jordan of the n x nb block in registers
//                  with partial pivoting; the block columns become Z + E_P,
//                  I + Z E_P^T the transform that turns the block into
//                  identity columns (Z also stored when other columns of the
//                  outer panel remain).
//   update kernel: the other columns of the outer panel: swap rows, then
//                  X += Z X[P rows].
//   final kernel : undo the row pivoting as a column permutation, cast to the
//                  bulk dtype, and (refresh) measure the drift of the old state.
#include <algorithm>

#include "lrx_common.hpp"
#include "lrx_flush_impl.hpp"
#include "lrx_internal.hpp"

namespace {

using namespace lrxfl;

using lrx::FactorArgs;

constexpr int kT = 256;
constexpr size_t kAlign = 256;
inline size_t al(size_t b) { return (b + kAlign - 1) / kAlign * kAlign; }

struct DetAcc {          // per-walker accumulators in the workspace
    double logabs;       // LU (Gauss-Jordan) log|det|
    double pad0;
    double ph[2];        // LU phase (re, im)
    double pf_logabs;    // Parlett-Reid log|pf|
    double pad1;
    double pf_ph[2];     // Parlett-Reid phase
    double dsq, nsq;     // refresh drift sums
    int singular;        // LU met a zero pivot
    int pf_zero;         // Parlett-Reid met a zero pivot
};

struct WorkLayout {
    size_t x, x2, x3, z, piv, src, perm, orig, ia, acc, stride;
};

// Columns per lane of the register-resident block kernel: the block is 4 CPT
// wide (64 real / 32 complex up to n = 512; 32 real / 8 complex up to
// n = 1024, where 16 waves share the register file).
template <class Wd> int block_cpt(int n) {
    if (sizeof(Wd) == 8) return n <= 512 ? 16 : 8;
    return n <= 512 ? 8 : 2;
}

// PF only: x2, the second matrix the Parlett-Reid panels alternate with; x3,
// the columns of L; orig, the original index of every position; ia, 1 / alpha
// of every pair.
inline WorkLayout work_layout(int n, size_t ws, bool pf) {
    WorkLayout L;
    size_t off = 0;
    const size_t mat = al((size_t)n * n * ws);
    L.x = off; off += mat;
    L.x2 = off; off += pf ? mat : 0;
    L.x3 = off; off += pf ? mat : 0;
    L.z = off; off += al((size_t)n * 32 * ws);
    L.piv = off; off += al((size_t)n * 4);
    L.src = off; off += al((size_t)n * 4);
    L.perm = off; off += al((size_t)n * 4);
    L.orig = off; off += pf ? al((size_t)n * 4) : 0;
    L.ia = off; off += pf ? al((size_t)n * ws) : 0;
    L.acc = off; off += al(sizeof(DetAcc));
    L.stride = off;
    return L;
}

struct FA {              // device-side argument block
    int kind, W, n, sites, nb;
    const void *src;
    const int32_t *occ;
    uint8_t *work;
    WorkLayout L;
    void *inv;
    double *logabs;
    void *phase;
    uint32_t *flags;
    double *report;
    int refresh;
    int packed;
};

template <class Wd> __device__ __forceinline__ Wd *wX(const FA &a, int w) {
    return reinterpret_cast<Wd *>(a.work + (size_t)w * a.L.stride + a.L.x);
}
template <class Wd> __device__ __forceinline__ Wd *wZ(const FA &a, int w) {
    return reinterpret_cast<Wd *>(a.work + (size_t)w * a.L.stride + a.L.z);
}
__device__ __forceinline__ int *wPiv(const FA &a, int w) {
    return reinterpret_cast<int *>(a.work + (size_t)w * a.L.stride + a.L.piv);
}
__device__ __forceinline__ int *wSrc(const FA &a, int w) {
    return reinterpret_cast<int *>(a.work + (size_t)w * a.L.stride + a.L.src);
}
// Row source of every position after the current outer panel's swaps so far
// (written by the block kernels, read by the outer update).
__device__ __forceinline__ int *wPerm(const FA &a, int w) {
    return reinterpret_cast<int *>(a.work + (size_t)w * a.L.stride + a.L.perm);
}
__device__ __forceinline__ int *wOrig(const FA &a, int w) {
    return reinterpret_cast<int *>(a.work + (size_t)w * a.L.stride + a.L.orig);
}
template <class Wd> __device__ __forceinline__ Wd *wIa(const FA &a, int w) {
    return reinterpret_cast<Wd *>(a.work + (size_t)w * a.L.stride + a.L.ia);
}
__device__ __forceinline__ DetAcc *wAcc(const FA &a, int w) {
    return reinterpret_cast<DetAcc *>(a.work + (size_t)w * a.L.stride + a.L.acc);
}

__device__ __forceinline__ void set_ph(double *p, double v) { p[0] = v; p[1] = 0.0; }
__device__ __forceinline__ void set_ph(double *p, cf64 v) { p[0] = v.x; p[1] = v.y; }
template <class Wd> __device__ __forceinline__ Wd get_ph(const double *p);
template <> __device__ __forceinline__ double get_ph<double>(const double *p) { return p[0]; }
template <> __device__ __forceinline__ cf64 get_ph<cf64>(const double *p) { return {p[0], p[1]}; }
__device__ __forceinline__ double unit(double v) { return v < 0 ? -1.0 : 1.0; }
__device__ __forceinline__ cf64 unit(cf64 v) { double m = hypot(v.x, v.y); return {v.x / m, v.y / m}; }
__device__ __forceinline__ double absdiff(double a, double b) { return fabs(a - b); }
__device__ __forceinline__ double absdiff(cf64 a, cf64 b) { return hypot(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double abs2(double a) { return a * a; }
__device__ __forceinline__ double half_of(double a) { return 0.5 * a; }
__device__ __forceinline__ cf64 half_of(cf64 a) { return {0.5 * a.x, 0.5 * a.y}; }
__device__ __forceinline__ double abs2(cf64 a) { return a.x * a.x + a.y * a.y; }

// ------------------------------------------------------------------ load
// X <- A^T (DET) or A (PF).  A[i][j]: DET phi[occ[i]][j] (or dense src[w][i][j]);
// PF f[occ[i]][occ[j]] (or dense).  32x32 tiles transposed through LDS.
template <class Wd>
__global__ __launch_bounds__(kT) void load_kernel(FA a, int tiles) {
    __shared__ Wd tile[32][33];
    const int n = a.n;
    const int w = blockIdx.x / (tiles * tiles);
    const int t = blockIdx.x - w * tiles * tiles;
    const int ti = t / tiles, tj = t - ti * tiles;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const Wd *src = static_cast<const Wd *>(a.src);
    Wd *X = wX<Wd>(a, w);
    const int32_t *occ = a.occ ? a.occ + (size_t)w * n : nullptr;
    // Tile of A: rows ti*32.., columns tj*32..
    for (int r = ty; r < 32; r += 8) {
        const int i = ti * 32 + r, j = tj * 32 + tx;
        Wd v = zero<Wd>();
        if (i < n && j < n) {
            // Out-of-range sites give a zero row (the walker is then flagged singular).
            if (a.kind == LRX_DET) {
                if (!occ) v = src[((size_t)w * n + i) * n + j];
                else if (occ[i] >= 0 && occ[i] < a.sites) v = src[(size_t)occ[i] * n + j];
            } else {
                if (!occ) v = src[((size_t)w * n + i) * n + j];
                else if (occ[i] >= 0 && occ[i] < a.sites && occ[j] >= 0 && occ[j] < a.sites)
                    v = src[(size_t)occ[i] * a.sites + occ[j]];
            }
        }
        tile[r][tx] = v;
    }
    __syncthreads();
    if (a.kind == LRX_DET) {   // X[j][i] = A[i][j]
        for (int r = ty; r < 32; r += 8) {
            const int j = tj * 32 + r, i = ti * 32 + tx;
            if (i < n && j < n) X[(size_t)j * n + i] = tile[tx][r];
        }
    } else {
        for (int r = ty; r < 32; r += 8) {
            const int i = ti * 32 + r, j = tj * 32 + tx;
            if (i < n && j < n) X[(size_t)i * n + j] = tile[r][tx];
        }
    }
}

template <class Wd>
__global__ void init_acc_kernel(FA a) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= a.W) return;
    DetAcc *d = wAcc(a, w);
    d->logabs = 0.0;
    d->ph[0] = 1.0; d->ph[1] = 0.0;
    d->pf_logabs = 0.0;
    d->pf_ph[0] = 1.0; d->pf_ph[1] = 0.0;
    d->dsq = 0.0; d->nsq = 0.0;
    d->singular = 0; d->pf_zero = 0;
}

// Block-wide argmax of a key with ties to the lowest index (NT threads).
// Returns the index on every thread (-1 when the block saw no candidate).  One
// barrier: every thread reduces the per-wave results itself; the caller must
// pass another barrier before calling again (s_val / s_idx are reused).
template <int M>
__device__ __forceinline__ void argmax_pair(double &val, int &idx) {
    const double ov = shfl_xor_v(val, M);                 // DPP / swizzle exchanges (xshfl_i32)
    const int oi = xshfl_i32(idx, M);
    const bool take = (oi >= 0) && (idx < 0 || ov > val || (ov == val && oi < idx));
    val = take ? ov : val;
    idx = take ? oi : idx;
}
template <int NT>
__device__ int block_argmax(double val, int idx, double *s_val, int *s_idx) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    argmax_pair<32>(val, idx);
    argmax_pair<16>(val, idx);
    argmax_pair<8>(val, idx);
    argmax_pair<4>(val, idx);
    argmax_pair<2>(val, idx);
    argmax_pair<1>(val, idx);
    if (lane == 0) { s_val[wv] = val; s_idx[wv] = idx; }
    __syncthreads();
    double bv = s_val[0];
    int bi = s_idx[0];
#pragma unroll
    for (int q = 1; q < NT / 64; ++q) {
        const double ov = s_val[q];
        const int oi = s_idx[q];
        const bool take = oi >= 0 && (bi < 0 || ov > bv || (ov == bv && oi < bi));
        bv = take ? ov : bv;
        bi = take ? oi : bi;
    }
    return bi;
}

// ------------------------------------------------------------------ Parlett-Reid
// Per matrix, on the workspace copy X of A (PF only), in the every-other-column
// form: for j = 0, 2, ...: pivot p = argmax_{i>j} |A[j][i]| (|A[i][j]| by
// skewness), swap index j+1 <-> p (rows and columns, sign flip), alpha =
// A[j][j+1] (the Pfaffian gains the factor alpha), then the skew rank-2 update
// A[r][s] += w_r c_s - c_r w_s (r, s >= j+2) with c = A[j][j+2:] / alpha and
// w = A[j+1][j+2:]  (Appendix A: pf(B A B^T) = det(B) pf(A), and the block
// Schur step of Eq. pf_block).
//
// Blocked in panels of P pairs, two launches per panel:
//   panel kernel: one work-group per matrix takes the panel's pairs one after
//                 the other.  Their rank-2 updates stay pending as vectors
//                 (c_t, w_t) in LDS, and the two rows a pair needs (its pivot
//                 row j+1 and the next pair's row j+2) are rebuilt from X plus
//                 the pending terms.  Swaps are not applied to X: a logical ->
//                 physical index map (the identity at the panel's start) is
//                 permuted instead, with the pending vectors and the current
//                 row, so a pair costs one gather of two rows of X, LDS work
//                 and three barriers.
//   trail kernel: the panel's trailing matrix, one upper 64 x 64 tile per
//                 work-group over all matrices: X'[r][s] = X[pm r][pm s] +
//                 sum_t w_t[r] c_t[s] - c_t[r] w_t[s], an MFMA GEMM of inner
//                 dimension 2P started from the gathered tile, written out of
//                 place to the second workspace matrix in logical order (the
//                 lower triangle is read as the negated transpose, pr_stored).
// The upper half of X is read and written once per panel, by the whole GPU.
// Each panel's P is the largest count (at most 16) whose 2P pending vectors,
// current row and index map fit in one work-group's LDS; they span only the
// panel's n - j0 logical indices, so later panels take more pairs.  The panel
// also records, for the
// inverse, the columns of L, 1/alpha and the original index of every
// position (see the PF inverse below).
constexpr int kPrMaxPairs = 16;          // the workspace Z holds 2 x 16 pending rows
constexpr int kPrThreads = 512;

// Pivot key: |x| for real, |x|^2 for complex (same order, no square root).
__device__ __forceinline__ double pivkey(double v) { return fabs(v); }
__device__ __forceinline__ double pivkey(cf64 v) { return v.x * v.x + v.y * v.y; }
__device__ __forceinline__ double recip(double v) { return 1.0 / v; }
__device__ __forceinline__ cf64 recip(cf64 v) { return divv(one<cf64>(), v); }

template <class Wd> __device__ __forceinline__ Wd *pr_buf(const FA &a, int w, int b) {
    return reinterpret_cast<Wd *>(a.work + (size_t)w * a.L.stride + (b ? a.L.x2 : a.L.x));
}

// Entry (r, c) of a trailing matrix whose update started at index `base`: the
// trail kernel stores the 64 x 64 tiles on and above the diagonal of the
// tiling that starts at base (diagonal tiles whole), so an entry below them is
// the negated transposed one.  The loaded A holds both triangles, which base 0
// reads the same way.
template <class Wd>
__device__ __forceinline__ Wd pr_stored(const Wd *X, int n, int base, int r, int c) {
    const bool up = ((r - base) >> 6) <= ((c - base) >> 6);
    const Wd v = X[up ? (size_t)r * n + c : (size_t)c * n + r];
    return up ? v : -v;
}

// LDS of a panel over m = n - j0 logical indices with P pairs, and the most
// pairs (up to kPrMaxPairs) that fit a budget.
template <class Wd> size_t pr_lds(int n, int P) {
    return sizeof(Wd) * ((size_t)2 * P * n + n) + sizeof(int) * (size_t)n;
}
template <class Wd> int pr_pairs(int n, size_t budget) {
    const size_t fixed = sizeof(Wd) * (size_t)n + sizeof(int) * (size_t)n;
    const size_t per = sizeof(Wd) * (size_t)2 * n;
    const size_t p = budget > fixed ? (budget - fixed) / per : 0;
    return (int)std::min<size_t>(std::max<size_t>(p, 1), kPrMaxPairs);
}

template <class Wd>
__global__ __launch_bounds__(kPrThreads) void pr_panel_kernel(FA a, int j0, int P, int cur) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_val[kPrThreads / 64];
    __shared__ int s_idx[kPrThreads / 64];
    __shared__ Wd s_ia[kPrMaxPairs];                    // 1 / alpha of the panel's pairs
    __shared__ Wd s_al[kPrMaxPairs];                    // alpha of the panel's pairs
    __shared__ int s_sw[kPrMaxPairs];                   // the pair swapped (sign flip)
    const int w = blockIdx.x, n = a.n, tid = threadIdx.x;
    // LDS arrays over the panel's logical indices j0 .. n-1, entry e at e - j0
    const int L = n - j0;
    Wd *s_c = reinterpret_cast<Wd *>(smem);             // [P][L] pending c_t
    Wd *s_w = s_c + (size_t)P * L;                      // [P][L] pending w_t
    Wd *s_rj = s_w + (size_t)P * L;                     // [L]    row j of the current matrix
    int *s_pm = reinterpret_cast<int *>(s_rj + L);      // [L]    logical -> physical index in X
    DetAcc *d = wAcc(a, w);
    const Wd *X = pr_buf<Wd>(a, w, cur);
    Wd *Cg = wZ<Wd>(a, w);                              // [kPrMaxPairs][n], for the trail kernel
    Wd *Wg = Cg + (size_t)kPrMaxPairs * n;
    double la = 0.0;
    Wd ph = one<Wd>();
    if (j0 > 0) {
        if (d->pf_zero) return;
        la = d->pf_logabs;
        ph = get_ph<Wd>(d->pf_ph);
    } else if (n & 1) {                                 // odd order: pf = 0
        if (tid == 0) { d->pf_zero = 1; d->pf_logabs = -INFINITY; set_ph(d->pf_ph, zero<Wd>()); }
        for (int e = tid; e < n; e += kPrThreads) wSrc(a, w)[e] = e;
        return;
    }
    for (int e = j0 + tid; e < n; e += kPrThreads) {
        s_pm[e - j0] = e;
        s_rj[e - j0] = X[(size_t)j0 * n + e];
    }
    __syncthreads();
    const int pairs = min(P, (n - j0) / 2);
    bool zero_pf = false;
    for (int t = 0; t < pairs; ++t) {
        const int j = j0 + 2 * t, q = j + 1;
        // row j takes the previous pair's term (the others are in already),
        // then the pivot search over its entries > j
        const Wd *lc = s_c + (size_t)(t > 0 ? t - 1 : 0) * L;
        const Wd *lw = s_w + (size_t)(t > 0 ? t - 1 : 0) * L;
        const Wd cl = t > 0 ? lc[j - j0] : zero<Wd>(), wl = t > 0 ? lw[j - j0] : zero<Wd>();
        double bv = -1.0;
        int bi = -1;
        for (int e = q + tid; e < n; e += kPrThreads) {
            Wd v = s_rj[e - j0];
            if (t > 0) v = v + (wl * lc[e - j0] - cl * lw[e - j0]);
            s_rj[e - j0] = v;
            const double kv = pivkey(v);
            if (bi < 0 || kv > bv) { bv = kv; bi = e; }
        }
        const int p = block_argmax<kPrThreads>(bv, bi, s_val, s_idx);
        if (p != q) {
            // swap index q <-> p in the map, the current row and the pending vectors
            if (tid == 0) {
                const int ti = s_pm[q - j0];
                s_pm[q - j0] = s_pm[p - j0];
                s_pm[p - j0] = ti;
                const Wd tv = s_rj[q - j0];
                s_rj[q - j0] = s_rj[p - j0];
                s_rj[p - j0] = tv;
            }
            if (tid < t) {
                Wd *c = s_c + (size_t)tid * L, *wv = s_w + (size_t)tid * L;
                const int qo = q - j0, po = p - j0;
                Wd tv = c[qo]; c[qo] = c[po]; c[po] = tv;
                tv = wv[qo]; wv[qo] = wv[po]; wv[po] = tv;
            }
        }
        __syncthreads();
        const Wd alpha = s_rj[q - j0];
        if (is_zero(alpha)) { zero_pf = true; break; }
        // log|pf| and the phase take alpha and the swap sign at the panel's end,
        // off the pair chain
        const Wd inva = recip(alpha);
        if (tid == 0) { s_ia[t] = inva; s_al[t] = alpha; s_sw[t] = p != q; }
        // the new pending pair (c = row j / alpha, w = row q) and row j+2 up
        // to this pair's term, on entries > q
        const bool more = t + 1 < pairs;
        const int j2 = more ? j + 2 : q;
        const int p1 = s_pm[q - j0], p2 = s_pm[j2 - j0];
        Wd *ct = s_c + (size_t)t * L, *wt = s_w + (size_t)t * L;
        for (int e = q + 1 + tid; e < n; e += kPrThreads) {
            const int pe = s_pm[e - j0];
            Wd wv = pr_stored<Wd>(X, n, j0, p1, pe);
            Wd rv = more ? pr_stored<Wd>(X, n, j0, p2, pe) : zero<Wd>();
            for (int u = 0; u < t; ++u) {
                const Wd *cu = s_c + (size_t)u * L, *wu = s_w + (size_t)u * L;
                const Wd ce = cu[e - j0], we = wu[e - j0];
                wv = wv + (wu[q - j0] * ce - cu[q - j0] * we);
                if (more) rv = rv + (wu[j2 - j0] * ce - cu[j2 - j0] * we);
            }
            const Wd c = s_rj[e - j0] * inva;
            ct[e - j0] = c;
            wt[e - j0] = wv;
            if (more) s_rj[e - j0] = rv;
        }
        __syncthreads();
    }
    __shared__ double s_lg[kPrMaxPairs];
    __shared__ Wd s_un[kPrMaxPairs];
    if (!zero_pf && tid < pairs) {                      // the pairs' factors in parallel ...
        s_lg[tid] = log(absv(s_al[tid]));
        s_un[tid] = unit(s_al[tid]);
    }
    __syncthreads();
    if (tid == 0) {                                     // ... accumulated in pair order
        if (!zero_pf) {
            for (int t = 0; t < pairs; ++t) {
                la += s_lg[t];
                if (s_sw[t]) ph = -ph;
                ph = ph * s_un[t];
            }
        }
        d->pf_zero = zero_pf ? 1 : 0;
        d->pf_logabs = zero_pf ? -INFINITY : la;
        set_ph(d->pf_ph, zero_pf ? zero<Wd>() : ph);
    }
    // the map and the pending vectors as the last swap left them, on the
    // entries the trail kernel reads
    int *pm = wPerm(a, w);
    int *src = wSrc(a, w);
    for (int e = j0 + tid; e < n; e += kPrThreads) pm[e] = s_pm[e - j0];
    if (zero_pf) {                                      // no inverse: identity column order
        for (int e = tid; e < n; e += kPrThreads) src[e] = e;
        return;
    }
    const int j1 = j0 + 2 * pairs;
    for (int t = 0; t < pairs; ++t) {
        for (int e = j1 + tid; e < n; e += kPrThreads) {
            Cg[(size_t)t * n + e] = s_c[(size_t)t * L + e - j0];
            Wg[(size_t)t * n + e] = s_w[(size_t)t * L + e - j0];
        }
    }
    // For the inverse (A = Pi U^T D U Pi^T, U = L^T): the original index of
    // every position at the panel's end, orig_b(e) = orig_{b-1}(pm e), and
    // the panel's rows of U (columns of L: -w_t / alpha_t and c_t below the
    // pair), scattered by it, so that later panels' swaps need not touch them.
    int *orig = wOrig(a, w);
    Wd *LT = reinterpret_cast<Wd *>(a.work + (size_t)w * a.L.stride + a.L.x3);
    int o[2];                                           // n <= 2 kPrThreads
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = j0 + tid + u * kPrThreads;
        o[u] = e < n ? (j0 > 0 ? orig[s_pm[e - j0]] : s_pm[e - j0]) : 0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const int e = j0 + tid + u * kPrThreads;
        if (e < n) orig[e] = o[u];
    }
    for (int t = 0; t < pairs; ++t) {
        const Wd iat = s_ia[t];
        Wd *l0 = LT + (size_t)(j0 + 2 * t) * n, *l1 = l0 + n;
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int e = j0 + tid + u * kPrThreads;
            if (e < n && e > j0 + 2 * t + 1) {
                l0[o[u]] = -(s_w[(size_t)t * L + e - j0] * iat);
                l1[o[u]] = s_c[(size_t)t * L + e - j0];
            }
        }
    }
    if (tid < pairs) wIa<Wd>(a, w)[j0 / 2 + tid] = s_ia[tid];
    if (j1 == n) {                                      // last panel: src = orig^-1
        __syncthreads();
        for (int e = tid; e < n; e += kPrThreads) src[orig[e]] = e;
    }
}

// The trailing matrix of the panel that ended at j1 (T pairs): 64 x 64 tile
// (I, J), I <= J, of X' = X[pm][pm] + P Q^T with P = [w_t, -c_t], Q = [c_t,
// w_t]; wave wv owns 16 rows of the tile as four 16x16 MFMA blocks.  X' is
// skew like X, so only the upper tiles are computed and stored (a diagonal
// tile whole); readers take an entry below them as the negated transposed one
// (pr_stored), the lower triangle is never written.  Rows and columns beyond n
// are clamped on load and dropped on store.
template <class Wd>
__global__ __launch_bounds__(kT) void pr_trail_kernel(FA a, int j1, int T, int cur, int nt) {
    using R = typename Real<Wd>::type;
    using A4 = typename Acc<R>::type;
    const int per = nt * (nt + 1) / 2;
    const int w = blockIdx.x / per;
    int tile = blockIdx.x - w * per, ti = 0;
    while (tile >= nt - ti) { tile -= nt - ti; ++ti; }
    const int tj = ti + tile;
    if (wAcc(a, w)->pf_zero) return;
    const int n = a.n;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kq = lane >> 4, lc = lane & 15;
    const Wd *X = pr_buf<Wd>(a, w, cur);
    Wd *Y = pr_buf<Wd>(a, w, cur ^ 1);
    const Wd *Cp = wZ<Wd>(a, w);
    const Wd *Wp = Cp + (size_t)kPrMaxPairs * n;
    const int *pm = wPerm(a, w);
    const int r0 = j1 + ti * 64, s0 = j1 + tj * 64;
    const int rbase = r0 + wv * 16, K2 = 2 * T;
    int pcol[4], prow[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) pcol[jb] = pm[min(s0 + jb * 16 + lc, n - 1)];
#pragma unroll
    for (int r = 0; r < 4; ++r) prow[r] = pm[min(rbase + acc_row<R>(lane, r), n - 1)];
    A4 re[4], im[4];
    const int base = j1 - 2 * T;                        // where the previous trail update started
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const Wd v = pr_stored<Wd>(X, n, base, prow[r], pcol[jb]);
            re[jb][r] = re_(v);
            im[jb][r] = im_(v);
        }
    }
    const int ra = min(rbase + lc, n - 1);
    for (int k0 = 0; k0 < K2; k0 += 4) {
        const int k = k0 + kq;
        const bool kin = k < K2;
        const int t = kin ? (k < T ? k : k - T) : 0;
        const Wd *pa = (k < T ? Wp : Cp) + (size_t)t * n;
        const Wd *qb = (k < T ? Cp : Wp) + (size_t)t * n;
        Wd av = pa[ra];
        av = !kin ? zero<Wd>() : (k < T ? av : -av);
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) {
            const Wd bv = kin ? qb[min(s0 + jb * 16 + lc, n - 1)] : zero<Wd>();
            mac<Wd>(av, bv, re[jb], im[jb]);
        }
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int sc = s0 + jb * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            if (q < n && sc < n) Y[(size_t)q * n + sc] = make_<Wd>(re[jb][r], im[jb][r]);
        }
    }
}

// ------------------------------------------------------------------ PF inverse
// From the Parlett-Reid factorisation itself: with the final order of the
// positions Pi (orig) and B = Pi^T A Pi = U^T D U, U = L^T unit upper
// triangular with identity 2x2 diagonal blocks and D the 2x2 blocks
// [[0, alpha_t], [-alpha_t, 0]],
//   A^-1 = Pi V D^-1 V^T Pi^T,   V = U^-1,
// so B^-1 = sum_t (V[:, 2t+1] V[:, 2t]^T - V[:, 2t] V[:, 2t+1]^T) / alpha_t
// (D^-1 has the blocks [[0, -1/alpha], [1/alpha, 0]]).  Four steps, all on
// 64 x 64 tiles:
//   U assembly : row c of U from the stored columns of L, gathered through
//                Pi (they were scattered by original index);
//   V diagonal : V_II = U_II^-1 by back substitution in LDS;
//   V rows     : block rows I = nt-2 .. 0, all J > I at once:
//                V_IJ = -V_II sum_{K=I+1..J} U_IK V_KJ (two MFMA products);
//   product    : upper tiles of B^-1 = P Q^T with P[i][2t] = V[i][2t+1] /
//                alpha_t, P[i][2t+1] = -V[i][2t] / alpha_t, Q = V, over the
//                columns m >= the tile's column start (V is upper triangular),
//                written to row Pi(i) of X, and negated at the mirror.
// The final kernel then reads X with the column source Pi^-1 and stores
// (X' - X'^T) / 2.  About n^3 / 3 complex multiply-adds against n^3 for a
// Gauss-Jordan inverse, in MFMA products over many work-groups.
template <class Wd> __device__ __forceinline__ Wd *pr_buf3(const FA &a, int w) {
    return reinterpret_cast<Wd *>(a.work + (size_t)w * a.L.stride + a.L.x3);
}

// U (into X): four rows per work-group, one per wave.
template <class Wd>
__global__ __launch_bounds__(kT) void pr_uasm_kernel(FA a, int bpw) {
    const int w = blockIdx.x / bpw;
    const int c = (blockIdx.x - w * bpw) * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63, n = a.n;
    if (c >= n || wAcc(a, w)->pf_zero) return;
    const Wd *lt = pr_buf3<Wd>(a, w) + (size_t)c * n;
    const int *pi = wOrig(a, w);
    Wd *u = wX<Wd>(a, w) + (size_t)c * n;
    const int lo = c | 1;
    for (int f = lane; f < n; f += 64) u[f] = f > lo ? lt[pi[f]] : (f == c ? one<Wd>() : zero<Wd>());
}

// V_II = U_II^-1 (into x2), tile I of walker w.  Past n the tile is taken as
// the identity.  A lane quad solves one column by back substitution, each
// lane taking every fourth term of a dot product; the tile is written whole
// (zeros below the diagonal).
template <class Wd> constexpr int vd_stride() { return 65; }
template <class Wd> size_t vdiag_lds() { return sizeof(Wd) * (size_t)2 * 64 * vd_stride<Wd>(); }
template <class Wd>
__global__ __launch_bounds__(kT) void pr_vdiag_kernel(FA a, int nt) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int S = vd_stride<Wd>();
    Wd *sU = reinterpret_cast<Wd *>(smem), *sV = sU + 64 * S;
    const int w = blockIdx.x / nt, I = blockIdx.x - w * nt, n = a.n, r0 = I * 64;
    if (wAcc(a, w)->pf_zero) return;
    const Wd *U = wX<Wd>(a, w);
    Wd *V = pr_buf<Wd>(a, w, 1);
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kT) {
        const int i = idx >> 6, k = idx & 63, gi = r0 + i, gk = r0 + k;
        sU[i * S + k] = (gi < n && gk < n) ? U[(size_t)gi * n + gk] : (i == k ? one<Wd>() : zero<Wd>());
    }
    __syncthreads();
    {
        // column j = 4 waves x 16 quads; the quad's lane 0 stores each entry,
        // which its wave reads back in the next step (LDS order within a wave)
        const int j = threadIdx.x >> 2, part = threadIdx.x & 3;
        for (int i = 63; i >= 0; --i) {
            Wd acc = zero<Wd>();
            for (int k = i + 1 + part; k <= j; k += 4) acc = acc + sU[i * S + k] * sV[k * S + j];
            acc = acc + shfl_xor_v(acc, 1);
            acc = acc + shfl_xor_v(acc, 2);
            if (part == 0) sV[i * S + j] = i == j ? one<Wd>() : (i > j ? zero<Wd>() : -acc);
        }
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kT) {
        const int i = idx >> 6, k = idx & 63, gi = r0 + i, gk = r0 + k;
        if (gi < n && gk < n) V[(size_t)gi * n + gk] = sV[i * S + k];
    }
}

// Block row I of V, tile J = I + 1 + (block index mod (nt - 1 - I)).  The
// first product sum_K U_IK V_KJ is staged in LDS as the B operand of the
// second, V_II times it.
template <class Wd> size_t vrow_lds() { return sizeof(Wd) * (size_t)64 * 65; }
template <class Wd>
__global__ __launch_bounds__(kT) void pr_vrow_kernel(FA a, int I, int nt) {
    using R = typename Real<Wd>::type;
    using A4 = typename Acc<R>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int S = 65;
    Wd *sT = reinterpret_cast<Wd *>(smem);
    const int per = nt - 1 - I;
    const int w = blockIdx.x / per, J = I + 1 + (blockIdx.x - w * per), n = a.n;
    if (wAcc(a, w)->pf_zero) return;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kq = lane >> 4, lc = lane & 15;
    const Wd *U = wX<Wd>(a, w);
    Wd *V = pr_buf<Wd>(a, w, 1);
    const int r0 = I * 64, s0 = J * 64, rbase = r0 + wv * 16;
    const int ra = min(rbase + lc, n - 1);
    int col[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) col[jb] = min(s0 + jb * 16 + lc, n - 1);
    A4 re[4], im[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) { re[jb] = A4{}; im[jb] = A4{}; }
    // four 4-deep steps per batch, every load of the batch issued before its
    // MFMAs (unconditional loads from clamped addresses)
    const int kend = min((J + 1) * 64, n);
    for (int k0 = r0 + 64; k0 < kend; k0 += 16) {
        Wd av[4], bv[4][4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int k = k0 + 4 * u + kq;
            const int kc = min(k, n - 1);
            const Wd x = U[(size_t)ra * n + kc];
            av[u] = k < kend ? x : zero<Wd>();
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) {
                const Wd y = V[(size_t)kc * n + col[jb]];
                bv[u][jb] = k < kend ? y : zero<Wd>();
            }
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) mac<Wd>(av[u], bv[u][jb], re[jb], im[jb]);
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r)
            sT[(wv * 16 + acc_row<R>(lane, r)) * S + jb * 16 + lc] = make_<Wd>(re[jb][r], im[jb][r]);
    __syncthreads();
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) { re[jb] = A4{}; im[jb] = A4{}; }
    for (int k0 = 0; k0 < 64; k0 += 4) {
        const int k = k0 + kq;
        const Wd av = r0 + k < n ? V[(size_t)ra * n + r0 + k] : zero<Wd>();
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) mac<Wd>(av, sT[k * S + jb * 16 + lc], re[jb], im[jb]);
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int sc = s0 + jb * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            if (q < n && sc < n) V[(size_t)q * n + sc] = -make_<Wd>(re[jb][r], im[jb][r]);
        }
    }
}

// Upper tile (I, J) of B^-1 into X at the rows Pi(i), mirrored; a walker
// with pf = 0 gets zeros in identity order.  A diagonal tile writes each
// entry above its diagonal with the negated mirror and zeros on the diagonal,
// so X holds an exactly skew matrix (rows permuted).
template <class Wd>
__global__ __launch_bounds__(kT) void pr_inv_kernel(FA a, int nt) {
    using R = typename Real<Wd>::type;
    using A4 = typename Acc<R>::type;
    const int per = nt * (nt + 1) / 2;
    const int w = blockIdx.x / per;
    int tile = blockIdx.x - w * per, ti = 0;
    while (tile >= nt - ti) { tile -= nt - ti; ++ti; }
    const int tj = ti + tile, n = a.n;
    const bool zero_pf = wAcc(a, w)->pf_zero != 0;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, kq = lane >> 4, lc = lane & 15;
    const Wd *V = pr_buf<Wd>(a, w, 1);
    const Wd *ia = wIa<Wd>(a, w);
    const int *pi = wOrig(a, w);
    Wd *X = wX<Wd>(a, w);
    const int r0 = ti * 64, s0 = tj * 64, rbase = r0 + wv * 16;
    A4 re[4], im[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) { re[jb] = A4{}; im[jb] = A4{}; }
    if (!zero_pf) {
        const int ra = min(rbase + lc, n - 1);
        int col[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb) col[jb] = min(s0 + jb * 16 + lc, n - 1);
        // Batches of four 4-deep steps, software pipelined over two register
        // sets: the next batch's loads (clamped addresses) are in flight
        // while the current one goes through the matrix cores.
        auto load = [&](int m0, Wd (&xa)[4], Wd (&ya)[4], Wd (&bb)[4][4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int mc = min(m0 + 4 * u + kq, n - 1);
                xa[u] = V[(size_t)ra * n + (mc ^ 1)];
                ya[u] = ia[mc >> 1];
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) bb[u][jb] = V[(size_t)col[jb] * n + mc];
            }
        };
        auto comp = [&](int m0, const Wd (&xa)[4], const Wd (&ya)[4], const Wd (&bb)[4][4]) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int m = m0 + 4 * u + kq;
                const Wd x = xa[u] * ya[u];
                const Wd av = m < n ? (m & 1 ? -x : x) : zero<Wd>();
#pragma unroll
                for (int jb = 0; jb < 4; ++jb) mac<Wd>(av, bb[u][jb], re[jb], im[jb]);
            }
        };
        Wd x0[4], y0[4], b0[4][4], x1[4], y1[4], b1[4][4];
        int m0 = s0;
        load(m0, x0, y0, b0);
        while (m0 < n) {
            load(m0 + 16, x1, y1, b1);
            comp(m0, x0, y0, b0);
            m0 += 16;
            if (m0 >= n) break;
            load(m0 + 16, x0, y0, b0);
            comp(m0, x1, y1, b1);
            m0 += 16;
        }
    }
    const bool diag = ti == tj;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int sc = s0 + jb * 16 + lc;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = rbase + acc_row<R>(lane, r);
            if (q < n && sc < n && (!diag || q <= sc)) {
                const Wd v = (q == sc) ? zero<Wd>() : make_<Wd>(re[jb][r], im[jb][r]);
                X[(size_t)(zero_pf ? q : pi[q]) * n + sc] = v;
                if (q != sc) X[(size_t)(zero_pf ? sc : pi[sc]) * n + q] = -v;
            }
        }
    }
}

// ------------------------------------------------------------------ GJ block
// In-place Gauss-Jordan elimination of the column block [j0, j0 + nbw) of X
// (the rows at positions >= j0 not yet used are the pivot candidates), with
// the whole n x nbw block in registers.  Column c: pivot row p (largest |x|),
// pi = x[p][c]; every other row r takes x[r] -= (x[r][c] / pi) x[p] and stores
// -x[r][c] / pi in column c, row p becomes x[p] / pi with 1 / pi in column c.
// After nbw columns the block holds the transform's columns Zt + E_P of the
// elimination, the rows written in their pivoted positions (explicit swaps and
// implicit pivoting give the same numbers up to that row order).  The division
// of a pivot row by pi is deferred to the write-out: the elimination is linear
// in each row, so the row is carried unscaled (1 in column c) with its factor
// 1 / pi kept beside it.
//
// Layout: wave wv, lane l holds rows wv*64 + 4 (l/4) + {0..3} and the columns
// q*CPT .. q*CPT + CPT-1 of the block, q = l % 4, so a row lives in one lane
// quad.  One barrier per column: the quad holding each wave's best candidate
// posts that row to the wave's LDS slot, lane 0 the key, row, position, pivot
// value and its reciprocal (two sets of slots, alternating); after the
// barrier every wave picks the winner over the waves and reads the pivot-row
// segment of its lane's quarter back as broadcasts.  The next column is
// updated first and sent round its quads before the rest of the update.  A
// zero column (singular block) turns the update into x += 0 * u.
template <class Wd, int CPT> constexpr int blk_qse() { return CPT + (int)(16 / sizeof(Wd)); }
template <class Wd, int CPT> size_t blk_lds(int nw) {
    return (size_t)2 * nw * (16 * blk_qse<Wd, CPT>() * sizeof(Wd) + 2 * sizeof(double) + 2 * sizeof(Wd)) +
           (size_t)4 * CPT * (sizeof(Wd) + sizeof(int));
}

__device__ __forceinline__ double bperm(double v, int addr) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_ds_bpermute(addr, (int)(b & 0xffffffffll));
    const int hi = __builtin_amdgcn_ds_bpermute(addr, (int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ cf64 bperm(cf64 v, int addr) { return {bperm(v.x, addr), bperm(v.y, addr)}; }
template <int CTRL> __device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double readlane_d(double v, int l) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ cf64 readlane_d(cf64 v, int l) { return {readlane_d(v.x, l), readlane_d(v.y, l)}; }
__device__ __forceinline__ double rfl_double(double v) { return readlane_d(v, __builtin_amdgcn_readfirstlane(0)); }
template <class Wd> __device__ __forceinline__ Wd sel(bool c, Wd a, Wd b) { return c ? a : b; }

// State of one block elimination, shared by its column steps.
template <class Wd, int CPT, int MAXT> struct BlkState {
    static constexpr int QSE = blk_qse<Wd, CPT>();   // quarter stride (elements): 16 bytes of bank padding
    static constexpr int RS = 4 * QSE;               // slot row stride
    static constexpr int MAXW = MAXT / 64;
    Wd x[4][CPT];
    Wd rsc[4];       // 1 / pi of the rows that have been pivots, 1 otherwise
    Wd v[4];         // the current column's values of the quad's rows
    int pos[4];
    unsigned elig;
    bool sing;
    int NW, j0, nbw, tid, lane, wv, q, gq, rbase, cq;
    Wd *slots;       // [2][NW][4 rows][RS]
    double *keys;    // [2][NW]
    int2 *rowpos;    // [2][NW]
    Wd *pvinv;       // [2][NW][2]
    Wd *s_pv;        // [4 CPT] pivot values
    int *s_piv;      // [4 CPT] swap partners
};

// Post the wave's best candidate for the current column (slot set PAR), then
// the barrier.
template <int PAR, class Wd, int CPT, int MAXT>
__device__ __forceinline__ void blk_post(BlkState<Wd, CPT, MAXT> &S) {
    using St = BlkState<Wd, CPT, MAXT>;
    constexpr int RS = St::RS;
    const int NW = S.NW, lane = S.lane, wv = S.wv;
    double bk = -1.0;
    int bi = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const double kv = ((S.elig >> i) & 1u) ? pivkey(S.v[i]) : -1.0;
        const bool tk = kv > bk;
        bk = tk ? kv : bk;
        bi = tk ? i : bi;
    }
    // the four lanes of a quad agree; rotate over the quads of each 16-lane row, then the rows
    double m = fmax(bk, dpp_d<0x124>(bk));   // row_ror:4
    m = fmax(m, dpp_d<0x128>(m));            // row_ror:8
    m = fmax(fmax(readlane_d(m, 0), readlane_d(m, 16)), fmax(readlane_d(m, 32), readlane_d(m, 48)));
    const unsigned long long bal = __ballot(bk == m);
    const int wl = __builtin_ctzll(bal);
    const int wbi = __builtin_amdgcn_readlane(bi, wl);
    // (values, not lvalues: a select of addresses would keep the state in memory)
    const int pb = sel(wbi == 0, S.pos[0], sel(wbi == 1, S.pos[1], sel(wbi == 2, S.pos[2], S.pos[3])));
    const Wd vb = sel(wbi == 0, S.v[0], sel(wbi == 1, S.v[1], sel(wbi == 2, S.v[2], S.v[3])));
    const int wpos = __builtin_amdgcn_readlane(pb, wl);
    const Wd pv = readlane_d(vb, wl);
    Wd *slot = S.slots + (size_t)(PAR * NW + wv) * 4 * RS + S.q * St::QSE;
    if (S.gq == (wl >> 2)) {
        // the winner row only; the distinct empty asm statement ending each
        // case keeps the compiler from merging the four store sequences into
        // one with selected operands
        switch (wbi) {
            case 0:
#pragma unroll
                for (int k = 0; k < CPT; ++k) slot[k] = S.x[0][k];
                asm volatile("; post row 0");
                break;
            case 1:
#pragma unroll
                for (int k = 0; k < CPT; ++k) slot[RS + k] = S.x[1][k];
                asm volatile("; post row 1");
                break;
            case 2:
#pragma unroll
                for (int k = 0; k < CPT; ++k) slot[2 * RS + k] = S.x[2][k];
                asm volatile("; post row 2");
                break;
            default:
#pragma unroll
                for (int k = 0; k < CPT; ++k) slot[3 * RS + k] = S.x[3][k];
                asm volatile("; post row 3");
                break;
        }
    }
    if (lane == 0) {
        S.keys[PAR * NW + wv] = m;
        S.rowpos[PAR * NW + wv] = make_int2(wv * 64 + (wl & ~3) + wbi, wpos);
        S.pvinv[2 * (PAR * NW + wv)] = pv;
        S.pvinv[2 * (PAR * NW + wv) + 1] = m > 0.0 ? recip(pv) : zero<Wd>();
    }
    __syncthreads();
}

// Finish column c = cq * CPT + KK (KK a compile-time constant, so x[.][KK]
// stays in registers): winner over the waves, update, bookkeeping; leaves the
// next column's values in S.v.
template <int KK, class Wd, int CPT, int MAXT>
__device__ __forceinline__ void blk_finish(BlkState<Wd, CPT, MAXT> &S) {
    using St = BlkState<Wd, CPT, MAXT>;
    constexpr int PAR = KK & 1;      // = c & 1 (CPT is even)
    constexpr int NK = KK + 1 < CPT ? KK + 1 : 0;
    const int c = S.cq * CPT + KK;
    const int NW = S.NW, q = S.q, rbase = S.rbase;
    // winner over the waves: largest key, lowest wave on ties
    double bkey = S.keys[PAR * NW];
    int wb = 0;
#pragma unroll
    for (int u = 1; u < St::MAXW; ++u) {
        const double o = S.keys[PAR * NW + min(u, NW - 1)];
        const bool tk = u < NW && o > bkey;
        bkey = tk ? o : bkey;
        wb = tk ? u : wb;
    }
    wb = __builtin_amdgcn_readfirstlane(wb);
    bkey = rfl_double(bkey);
    const int2 rpv = S.rowpos[PAR * NW + wb];
    const int p = __builtin_amdgcn_readfirstlane(rpv.x);
    const int ppos = __builtin_amdgcn_readfirstlane(rpv.y);
    const Wd pv = S.pvinv[2 * (PAR * NW + wb)];
    const Wd inv = S.pvinv[2 * (PAR * NW + wb) + 1];
    const bool sg = !(bkey > 0.0);
    const Wd *ur = S.slots + (size_t)(PAR * NW + wb) * 4 * St::RS + (p & 3) * St::RS + q * St::QSE;
    Wd u[CPT];
#pragma unroll
    for (int k = 0; k < CPT; ++k) u[k] = ur[k];
    // g = -x[c] / pi; the pivot row is left as it is (unscaled)
    Wd g[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) g[i] = sel(rbase + i == p, zero<Wd>(), -(S.v[i] * inv));
    // next column first, and round the quads
    const int nsrc = ((S.lane & ~3) | (KK + 1 < CPT ? S.cq : S.cq + 1)) << 2;
    Wd vn[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        S.x[i][NK] = fmac(g[i], u[NK], S.x[i][NK]);
        vn[i] = bperm(S.x[i][NK], nsrc);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int k = 0; k < CPT; ++k)
            if (k != NK) S.x[i][k] = fmac(g[i], u[k], S.x[i][k]);
    // column c: -x[c] / pi (1 on the unscaled pivot row); positions: the pivot
    // row moves to t, the row at t to the pivot's old place
    const int t = S.j0 + c;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const bool isp = rbase + i == p && !sg;
        if (q == S.cq && !sg) S.x[i][KK] = sel(isp, one<Wd>(), g[i]);
        S.rsc[i] = sel(isp, inv, S.rsc[i]);
        const bool at_t = S.pos[i] == t;
        const bool clr = sg ? at_t : isp;
        S.pos[i] = isp ? t : ((!sg && at_t) ? ppos : S.pos[i]);
        S.elig = clr ? (S.elig & ~(1u << i)) : S.elig;
        S.v[i] = vn[i];
    }
    S.sing = S.sing || sg;
    if (S.tid == 0) { S.s_piv[c] = sg ? t : ppos; S.s_pv[c] = sg ? zero<Wd>() : pv; }
}

template <int KK, class Wd, int CPT, int MAXT>
__device__ __forceinline__ void blk_run(BlkState<Wd, CPT, MAXT> &S) {
    if constexpr (KK < CPT) {
        const int c = S.cq * CPT + KK;
        if (c < S.nbw) {
            blk_finish<KK>(S);
            if (c + 1 < S.nbw) blk_post<(KK + 1) & 1>(S);
            blk_run<KK + 1>(S);
        }
    }
}

template <class Wd, int CPT, int MAXT>
__global__ __launch_bounds__(MAXT) void gj_block_kernel(FA a, int j0, int nbw, int write_z, int o0) {
    using St = BlkState<Wd, CPT, MAXT>;
    extern __shared__ __align__(16) unsigned char smem[];
    St S;
    S.NW = blockDim.x >> 6;
    const int w = blockIdx.x, n = a.n;
    S.j0 = j0;
    S.nbw = nbw;
    S.tid = threadIdx.x;
    S.lane = S.tid & 63;
    S.wv = __builtin_amdgcn_readfirstlane(S.tid >> 6);
    S.q = S.lane & 3;
    S.gq = S.lane >> 2;
    S.rbase = S.wv * 64 + S.gq * 4;
    const int q = S.q, rbase = S.rbase, NW = S.NW;
    Wd *X = wX<Wd>(a, w);
    S.slots = reinterpret_cast<Wd *>(smem);
    S.keys = reinterpret_cast<double *>(S.slots + (size_t)2 * NW * 4 * St::RS);
    S.rowpos = reinterpret_cast<int2 *>(S.keys + 2 * NW);
    S.pvinv = reinterpret_cast<Wd *>(S.rowpos + 2 * NW);
    S.s_pv = S.pvinv + 4 * NW;
    S.s_piv = reinterpret_cast<int *>(S.s_pv + 4 * CPT);
    S.elig = 0;
    S.sing = false;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int r = rbase + i;
        S.pos[i] = r;
        S.rsc[i] = one<Wd>();
        const bool ok = r < n;
        if (ok && r >= j0) S.elig |= 1u << i;
        const Wd *row = X + (size_t)min(r, n - 1) * n + j0;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int cc = q * CPT + k;
            const Wd xv = row[min(cc, nbw - 1)];
            S.x[i][k] = (ok && cc < nbw) ? xv : zero<Wd>();
        }
    }
    S.cq = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) S.v[i] = bperm(S.x[i][0], (S.lane & ~3) << 2);
    blk_post<0>(S);
    for (int cq = 0; cq < 4; ++cq) {
        S.cq = cq;
        blk_run<0>(S);
    }
    // the outer panel's row sources: position pos[i] now holds what position
    // rbase + i held, whose source is the identity at the panel's first block
    int *gperm = wPerm(a, w);
    int src4[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        src4[i] = j0 == o0 ? rbase + i : gperm[min(rbase + i, n - 1)];
        asm volatile("" ::"v"(src4[i]));              // the read has completed before any thread writes
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (rbase + i < n) gperm[S.pos[i]] = src4[i];
    Wd *Z = wZ<Wd>(a, w);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (rbase + i >= n) continue;
        Wd *row = X + (size_t)S.pos[i] * n + j0;
        Wd *zr = Z + (size_t)S.pos[i] * nbw;
#pragma unroll
        for (int k = 0; k < CPT; ++k) {
            const int cc = q * CPT + k;
            const Wd xv = S.x[i][k] * S.rsc[i];
            if (cc < nbw) row[cc] = xv;
            if (write_z && cc < nbw) zr[cc] = xv - ((S.pos[i] == j0 + cc) ? one<Wd>() : zero<Wd>());
        }
    }
    if (S.wv == 0) {
        const int lane = S.lane;
        double la = 0.0;
        if (lane < nbw) {
            const Wd pv = S.s_pv[lane];
            if (!is_zero(pv)) la = log(absv(pv));
            wPiv(a, w)[j0 + lane] = S.s_piv[lane];
        }
        la = wave_sum(la);
        if (lane == 0) {
            Wd ph = one<Wd>();
            for (int c = 0; c < nbw; ++c) {
                const Wd pv = S.s_pv[c];
                if (!is_zero(pv)) ph = ph * unit(pv);
                if (S.s_piv[c] != j0 + c) ph = -ph;
            }
            DetAcc *d = wAcc(a, w);
            if (S.sing) d->singular = 1;
            d->logabs += la;
            set_ph(d->ph, get_ph<Wd>(d->ph) * ph);
        }
    }
}

// ------------------------------------------------------------------ GJ update
// Columns [c_lo, c_hi) outside the block: X_new[i] = X_old[pi(i)] + Z[i] . X_old[pi(P)].
// A work-group owns 64 of those columns for all rows, in 64-row chunks; each
// wave takes 16 rows of a chunk as four 16x16 MFMA blocks over the block's nb
// columns (zero-padded to NB).  Rows moved by the pivoting (at most 2 nb) and
// the pivot rows X_old[pi(P)] are staged in LDS first, so every other row is
// read and written in place.
template <class Wd> constexpr int upd_zs(int NB) { return NB + 1; }   // padded LDS stride of the Z rows
template <class Wd, int NB> size_t upd_lds(int n, int nb) {
    return (((size_t)(2 * n + 1 + 2 * nb) * 4 + 15) / 16) * 16 +
           sizeof(Wd) * ((size_t)NB * 64 + (size_t)2 * nb * 64 + (size_t)64 * upd_zs<Wd>(NB));
}

template <class Wd, int NB>
__global__ __launch_bounds__(kT) void gj_update_kernel(FA a, int j0, int nb, int ncb, int c_lo, int c_hi) {
    using R = typename Real<Wd>::type;
    using A4 = typename Acc<R>::type;
    constexpr int ZS = upd_zs<Wd>(NB);
    constexpr int NS = (NB + 3) / 4;                                   // 4-deep MFMA steps
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / ncb, cb = lb - w * ncb;
    if (w >= a.W) return;
    const int n = a.n, others = (c_hi - c_lo) - nb;
    const int tid = threadIdx.x, lane = tid & 63, kq = lane >> 4, lc = lane & 15;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    Wd *X = wX<Wd>(a, w);
    const Wd *Z = wZ<Wd>(a, w);
    const int *piv = wPiv(a, w);
    int *perm = reinterpret_cast<int *>(smem);                         // [n]
    int *sslot = perm + n;                                             // [n]
    int *s_cnt = sslot + n;                                            // [1]
    int *s_mrow = s_cnt + 1;                                           // [2 nb] moved rows, by slot
    Wd *sXP = reinterpret_cast<Wd *>(smem + (((2 * n + 1 + 2 * nb) * 4 + 15) / 16) * 16);   // [NB][64]
    Wd *sS = sXP + (size_t)NB * 64;                                    // [2 nb][64]
    Wd *sZ = sS + (size_t)2 * nb * 64;                                 // [64][ZS]
    __shared__ int s_pv[64];
    if (tid < nb) s_pv[tid] = piv[j0 + tid];                           // all pivots fetched at once
    for (int i = tid; i < n; i += kT) { perm[i] = i; sslot[i] = -1; }
    if (tid == 0) *s_cnt = 0;
    __syncthreads();
    if (tid == 0) {
        for (int c = 0; c < nb; ++c) {
            const int r = j0 + c, p = s_pv[c];
            const int t = perm[r]; perm[r] = perm[p]; perm[p] = t;
        }
    }
    __syncthreads();
    for (int i = j0 + tid; i < n; i += kT)
        if (perm[i] != i) {
            const int sl = atomicAdd(s_cnt, 1);
            sslot[i] = sl;
            s_mrow[sl] = i;
        }
    __syncthreads();
    // the column this lane stages (one per lane), and the four it computes
    auto colof = [&](int cc) {
        const int ci = min(cb * 64 + cc, others - 1);                  // clamped: dead columns load, never store
        return c_lo + ci < j0 ? c_lo + ci : c_lo + ci + nb;           // columns [c_lo, c_hi) minus the block
    };
    const int scol = colof(lane);
    // pivot rows and moved rows, from the pre-update matrix; every load of a
    // wave is issued before the first store
    {
        constexpr int PW = (NB + kT / 64 - 1) / (kT / 64), MW = (2 * NB + kT / 64 - 1) / (kT / 64);
        const int cnt = *s_cnt;
        Wd pv[PW], mv[MW];
#pragma unroll
        for (int u = 0; u < PW; ++u) pv[u] = X[(size_t)perm[j0 + min(wv + u * (kT / 64), nb - 1)] * n + scol];
#pragma unroll
        for (int u = 0; u < MW; ++u) {
            const int sl = min(wv + u * (kT / 64), max(cnt - 1, 0));
            mv[u] = X[(size_t)perm[cnt > 0 ? s_mrow[sl] : 0] * n + scol];
        }
#pragma unroll
        for (int u = 0; u < PW; ++u) {
            const int c = wv + u * (kT / 64);
            if (c < NB) sXP[c * 64 + lane] = c < nb ? pv[u] : zero<Wd>();
        }
#pragma unroll
        for (int u = 0; u < MW; ++u) {
            const int sl = wv + u * (kT / 64);
            if (sl < cnt) sS[sl * 64 + lane] = mv[u];
        }
    }
    int col[4];
    bool live[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        col[jb] = colof(jb * 16 + lc);
        live[jb] = cb * 64 + jb * 16 + lc < others;
    }
    for (int i0 = 0; i0 < n; i0 += 64) {
        const int rbase = i0 + wv * 16;
        // the rows this lane holds in the MFMA accumulators, loaded before the
        // Z rows are staged (moved rows are replaced by their staged copies)
        Wd xv[4][4];
        int sl[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q = min(rbase + acc_row<R>(lane, r), n - 1);
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) xv[jb][r] = X[(size_t)q * n + col[jb]];
            sl[r] = sslot[q];
        }
        __syncthreads();
        for (int idx = tid; idx < 64 * NB; idx += kT) {
            const int r = idx / NB, c = idx - r * NB;
            const Wd zv = Z[(size_t)min(i0 + r, n - 1) * nb + min(c, nb - 1)];
            sZ[r * ZS + c] = c < nb ? zv : zero<Wd>();
        }
        __syncthreads();
        A4 re[4], im[4];
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Wd v = sl[r] >= 0 ? sS[sl[r] * 64 + jb * 16 + lc] : xv[jb][r];
                re[jb][r] = re_(v);
                im[jb][r] = im_(v);
            }
#pragma unroll
        for (int st = 0; st < NS; ++st) {
            const int k = 4 * st + kq;
            const Wd zv = sZ[(wv * 16 + lc) * ZS + k];
#pragma unroll
            for (int jb = 0; jb < 4; ++jb) mac<Wd>(zv, sXP[k * 64 + jb * 16 + lc], re[jb], im[jb]);
        }
#pragma unroll
        for (int jb = 0; jb < 4; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int q = rbase + acc_row<R>(lane, r);
                if (live[jb] && q < n) X[(size_t)q * n + col[jb]] = make_<Wd>(re[jb][r], im[jb][r]);
            }
    }
}

// ------------------------------------------------------------------ GJ outer update
// After the last block of the outer panel [j0, j0 + nbo), its columns hold
// Zt + E_P; with pi the row swaps piv[j0 .. j0+nbo) in order (their composite,
// the source row of every position, written by the block kernels), every
// column outside the outer panel becomes
//   X_new[i] = X_old[pi(i)] + Zt[i] . X_old[pi(P)],   P = rows j0 .. j0+nbo-1,
// an MFMA GEMM (v_mfma_f64_16x16x4f64; four real products per complex one)
// with inner dimension nbo.  Two facts keep it a plain streaming GEMM:
//  * Zt[i] is the panel row X[i][j0..] except on P, where the identity comes
//    off; there X_old[pi(i)] is the pivot row itself and cancels it, so
//    X_new[i] = X[i][j0..] . X_old[pi(P)] on P (no initial value) and
//    X_new[i] = X_old[pi(i)] + X[i][j0..] . X_old[pi(P)] elsewhere;
//  * rows moved by pi outside P only ever come from positions in P, so all
//    other row blocks are done first (reading those positions still unchanged)
//    and the block of P last.  Only the pivot rows X_old[pi(P)] are staged.
// A work-group (4 waves) owns CB columns of one walker and walks 64-row
// blocks (16 rows per wave), loading the next block while the current one is
// on the matrix cores.  Loads are unconditional from clamped addresses
// (rows past n and columns past the batch are computed and not stored).
// Columns per work-group: every work-group of a walker re-reads the whole Zt
// panel, so wider groups cut that re-read traffic; 64 real columns from
// n = 512 on, where a walker still has at least 7 groups.
template <class Wd> constexpr int outer_cb_max() { return sizeof(Wd) == 8 ? 64 : 16; }
template <class Wd> int outer_cb(int n) { return sizeof(Wd) == 8 ? (n >= 512 ? 64 : 32) : 16; }
template <class Wd> size_t outer_lds(int n, int cb) {
    return (((size_t)n * 4 + 15) / 16) * 16 + (size_t)64 * (cb + 1) * sizeof(Wd);
}

template <class Wd, int CB>
__global__ __launch_bounds__(kT) void gj_outer_kernel(FA a, int j0, int nbo, int ncb) {
    using R = typename Real<Wd>::type;
    using A4 = typename Acc<R>::type;
    constexpr int NTL = CB / 16;          // 16-column MFMA tiles per wave
    constexpr int SP = CB + 1;            // padded LDS row stride
    constexpr int NK = 64 / 4;            // 4-deep MFMA steps over the (zero-padded) outer panel
    extern __shared__ __align__(16) unsigned char smem[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / ncb, cb = lb - w * ncb;
    if (w >= a.W) return;
    const int n = a.n, others = n - nbo;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    Wd *X = wX<Wd>(a, w);
        int *perm = reinterpret_cast<int *>(smem);                                   // [n]
    Wd *sXP = reinterpret_cast<Wd *>(smem + (((size_t)n * 4 + 15) / 16) * 16);    // [64][SP]: X_old[pi(j0+c)]
    const int *gperm = wPerm(a, w);                   // row sources, from the block kernels
    for (int i = tid; i < n; i += kT) perm[i] = gperm[i];
    __syncthreads();
    const int ci0 = cb * CB;
    auto colof = [&](int jj) {
        const int ci = min(ci0 + jj, others - 1);
        return ci < j0 ? ci : ci + nbo;
    };
    for (int idx = tid; idx < 64 * CB; idx += kT) {
        const int c = idx / CB, jj = idx - c * CB;
        const Wd v = X[(size_t)perm[j0 + min(c, nbo - 1)] * n + colof(jj)];
        sXP[c * SP + jj] = (c < nbo && ci0 + jj < others) ? v : zero<Wd>();
    }
    __syncthreads();
    const int kq = lane >> 4, lc = lane & 15;
    int col[NTL];
#pragma unroll
    for (int jt = 0; jt < NTL; ++jt) col[jt] = colof(jt * 16 + lc);
    const int nblk = (n + 63) / 64, pblk = j0 / 64;

    struct Buf { Wd x[NTL][4]; Wd z[NK]; };
    // block index t = 0 .. nblk-1: the other blocks in order, the P block last
    auto blk_of = [&](int t) { return t < nblk - 1 ? (t < pblk ? t : t + 1) : pblk; };
    // The four row sources of the block are read from LDS once, and the row
    // loads are unconditional (the P block reads valid rows and selects zero),
    // so all of a block's loads issue back to back.
    auto issue = [&](int t, Buf &b) {
        const int blk = blk_of(t);
        const int rbase = blk * 64 + wv * 16;
        const bool pb = blk == pblk;
        uint32_t ro[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) ro[r] = (uint32_t)perm[min(rbase + acc_row<R>(lane, r), n - 1)] * (uint32_t)n;
#pragma unroll
        for (int jt = 0; jt < NTL; ++jt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const Wd v = X[ro[r] + (uint32_t)col[jt]];
                b.x[jt][r] = pb ? zero<Wd>() : v;
            }
        const uint32_t zo = (uint32_t)min(rbase + lc, n - 1) * (uint32_t)n;
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) b.z[kk] = X[zo + (uint32_t)min(j0 + kk * 4 + kq, n - 1)];
    };
    auto consume = [&](int t, Buf &b) {
        const int blk = blk_of(t);
        const int rbase = blk * 64 + wv * 16;
        A4 re[NTL], im[NTL];
#pragma unroll
        for (int jt = 0; jt < NTL; ++jt)
#pragma unroll
            for (int r = 0; r < 4; ++r) { re[jt][r] = re_(b.x[jt][r]); im[jt][r] = im_(b.x[jt][r]); }
#pragma unroll
        for (int kk = 0; kk < NK; ++kk) {
            const int k = kk * 4 + kq;
#pragma unroll
            for (int jt = 0; jt < NTL; ++jt) mac<Wd>(b.z[kk], sXP[k * SP + jt * 16 + lc], re[jt], im[jt]);
        }
#pragma unroll
        for (int jt = 0; jt < NTL; ++jt) {
            if (ci0 + jt * 16 + lc >= others) continue;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int i = rbase + acc_row<R>(lane, r);
                if (i < n) X[(size_t)i * n + col[jt]] = make_<Wd>(re[jt][r], im[jt][r]);
            }
        }
    };
    // Every block except P first (they read the P positions, still unchanged),
    // then a barrier, then P.
    const int nA = nblk - 1;
    Buf b0, b1;
    if (nA > 0) issue(0, b0);
    for (int t = 0; t < nA; t += 2) {
        if (t + 1 < nA) issue(t + 1, b1);
        consume(t, b0);
        if (t + 1 >= nA) break;
        if (t + 2 < nA) issue(t + 2, b0);
        consume(t + 1, b1);
    }
    __syncthreads();
    issue(nA, b0);
    consume(nA, b0);
}

// Column source of the final permutation: X (PB)^-1 -> B^-1 = X P, applied as
// column swaps in reverse pivot order (done in LDS by one thread per walker).
__global__ __launch_bounds__(kT) void src_perm_kernel(FA a) {
    extern __shared__ int s_src[];
    const int w = blockIdx.x, n = a.n;
    int *src = wSrc(a, w);
    const int *piv = wPiv(a, w);
    int *s_piv = s_src + n;
    for (int c = threadIdx.x; c < n; c += kT) { s_src[c] = c; s_piv[c] = piv[c]; }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int kx = n - 1; kx >= 0; --kx) {
            const int p = s_piv[kx];
            const int t = s_src[kx]; s_src[kx] = s_src[p]; s_src[p] = t;
        }
    }
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kT) src[c] = s_src[c];
}

// ------------------------------------------------------------------ final
// DET: M[i][c] = X[i][src[c]], cast to the bulk dtype; refresh: drift sums.
template <class T, class Wd>
__global__ __launch_bounds__(kT) void final_det_kernel(FA a, int rows_per_block, int bpw) {
    __shared__ double s_d[kT / 64], s_nrm[kT / 64];
    extern __shared__ int s_src[];
    const uint32_t lb = xcd_remap(blockIdx.x, gridDim.x);
    const int w = lb / bpw, rb = lb - w * bpw;
    if (w >= a.W) return;
    const int n = a.n;
    const Wd *X = wX<Wd>(a, w);
    const int *gsrc = wSrc(a, w);
    for (int c = threadIdx.x; c < n; c += kT) s_src[c] = gsrc[c];
    __syncthreads();
    const int *src = s_src;
    T *M = static_cast<T *>(a.inv) + (size_t)w * n * n;
    double dsq = 0.0, nsq = 0.0;
    const int q0 = rb * rows_per_block, q1 = min(n, q0 + rows_per_block);
    for (int i = q0; i < q1; ++i) {
        for (int c = threadIdx.x; c < n; c += kT) {
            const Wd v = X[(size_t)i * n + src[c]];
            if (a.report) {
                const Wd o = conv<Wd>(M[(size_t)i * n + c]);
                dsq += abs2(o - v);
                nsq += abs2(v);
            }
            M[(size_t)i * n + c] = conv<T>(v);
        }
    }
    if (a.report) {
        dsq = wave_sum(dsq);
        nsq = wave_sum(nsq);
        if ((threadIdx.x & 63) == 0) { s_d[threadIdx.x >> 6] = dsq; s_nrm[threadIdx.x >> 6] = nsq; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double t0 = 0, t1 = 0;
            for (int q = 0; q < kT / 64; ++q) { t0 += s_d[q]; t1 += s_nrm[q]; }
            DetAcc *d = wAcc(a, w);
            atomicAdd(&d->dsq, t0);
            atomicAdd(&d->nsq, t1);
        }
    }
}

// PF: M = A^-1 = X', X'[i][j] = X[i][src[j]]: the inverse kernel left the rows
// in place and X exactly skew, so only the columns are gathered here.  One
// wave per row: the row is read coalesced into LDS and gathered from there,
// and M is written row by row (the packed layout keeps the tiles at or above
// the row's diagonal tile).  The drift report weighs an entry of a strictly
// upper packed tile twice, for its unstored mirror.
template <class T, class Wd>
__global__ __launch_bounds__(kT) void final_pf_kernel(FA a, int groups) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ double s_d[kT / 64], s_nrm[kT / 64];
    constexpr int RW = kT / 64;                   // rows per work-group
    const int n = a.n;
    const int w = blockIdx.x / groups;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int i = (blockIdx.x - w * groups) * RW + wv;
    const Wd *X = wX<Wd>(a, w);
    const int *src = wSrc(a, w);
    Wd *s_row = reinterpret_cast<Wd *>(smem) + (size_t)wv * n;
    if (i < n)
        for (int c = lane; c < n; c += 64) s_row[c] = X[(size_t)i * n + c];
    __syncthreads();
    const int nt = (n + 63) >> 6;
    T *M = static_cast<T *>(a.inv) + (size_t)w * (a.packed ? lrx_pk_elems_dev(n) : (size_t)n * n);
    double dsq = 0.0, nsq = 0.0;
    if (i < n) {
        const int ti = i >> 6;
        for (int j = lane; j < n; j += 64) {
            const int tj = j >> 6;
            if (a.packed && tj < ti) continue;
            const int sj = min(max(src[j], 0), n - 1);
            const Wd h = (j == i) ? zero<Wd>() : s_row[sj];
            T *dst = a.packed ? M + pk_offset(nt, i, j) : M + (size_t)i * n + j;
            if (a.report) {
                const double wgt = (a.packed && tj > ti) ? 2.0 : 1.0;
                dsq += wgt * abs2(conv<Wd>(*dst) - h);
                nsq += wgt * abs2(h);
            }
            *dst = conv<T>(h);
        }
    }
    if (a.report) {
        dsq = wave_sum(dsq);
        nsq = wave_sum(nsq);
        if (lane == 0) { s_d[wv] = dsq; s_nrm[wv] = nsq; }
        __syncthreads();
        if (threadIdx.x == 0) {
            double s0 = 0, s1 = 0;
            for (int q = 0; q < RW; ++q) { s0 += s_d[q]; s1 += s_nrm[q]; }
            DetAcc *d = wAcc(a, w);
            atomicAdd(&d->dsq, s0);
            atomicAdd(&d->nsq, s1);
        }
    }
}

// Packed storage: zero the entries of the last tile row / column that lie past n
// (the packed pass reads whole tiles; nothing else writes there).
template <class T>
__global__ __launch_bounds__(kT) void pk_zero_tail_kernel(FA a, int nt) {
    const int w = blockIdx.x / nt, I = blockIdx.x - w * nt, n = a.n;
    T *M = static_cast<T *>(a.inv) + (size_t)w * lrx_pk_elems_dev(n);
    for (int idx = threadIdx.x; idx < 64 * 64; idx += kT) {
        const int r = I * 64 + (idx >> 6), c = (nt - 1) * 64 + (idx & 63);   // tile (I, nt - 1)
        if (r >= n || c >= n) M[pk_offset(nt, r, c)] = zero<T>();
    }
}

template <class Wd>
__global__ void finish_kernel(FA a) {
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= a.W) return;
    const DetAcc *d = wAcc(a, w);
    Wd *phase = static_cast<Wd *>(a.phase);
    double la;
    Wd ph;
    bool bad;
    if (a.kind == LRX_DET) {
        bad = d->singular != 0;
        la = bad ? -INFINITY : d->logabs;
        ph = bad ? zero<Wd>() : get_ph<Wd>(d->ph);
    } else {
        bad = d->singular != 0 || d->pf_zero != 0;
        la = d->pf_zero ? -INFINITY : d->pf_logabs;
        ph = d->pf_zero ? zero<Wd>() : get_ph<Wd>(d->pf_ph);
    }
    if (a.report) {
        const double oldla = a.logabs[w];
        const Wd oldph = phase[w];
        a.report[2 * w] = d->nsq > 0 ? sqrt(d->dsq / d->nsq) : 0.0;
        a.report[2 * w + 1] = fabs(oldla - la) + absdiff(oldph, ph);
    }
    a.logabs[w] = la;
    phase[w] = ph;
    a.flags[w] = bad ? LRX_FLAG_SINGULAR_A : 0u;
}

template <class Wd>
hipError_t launch_outer(const FA &fa, int j0, int nbo, hipStream_t s) {
    const int others = fa.n - nbo;
    if (others <= 0) return hipSuccess;
    const int cb = outer_cb<Wd>(fa.n);
    const int ncb = (others + cb - 1) / cb;
    const size_t lds = outer_lds<Wd>(fa.n, cb);
    if (cb == 64) {
        if constexpr (outer_cb_max<Wd>() >= 64)
            hipLaunchKernelGGL((gj_outer_kernel<Wd, 64>), dim3((unsigned)(fa.W * ncb)), dim3(kT), lds, s, fa, j0, nbo,
                               ncb);
    } else if (cb == 32) {
        if constexpr (outer_cb_max<Wd>() >= 32)
            hipLaunchKernelGGL((gj_outer_kernel<Wd, 32>), dim3((unsigned)(fa.W * ncb)), dim3(kT), lds, s, fa, j0, nbo,
                               ncb);
    } else {
        hipLaunchKernelGGL((gj_outer_kernel<Wd, 16>), dim3((unsigned)(fa.W * ncb)), dim3(kT), lds, s, fa, j0, nbo, ncb);
    }
    return hipGetLastError();
}

template <class Wd>
hipError_t launch_update(const FA &fa, int j0, int nb, int c_lo, int c_hi, hipStream_t s) {
    const int others = (c_hi - c_lo) - nb;
    if (others <= 0) return hipSuccess;
    const int ncb = (others + 63) / 64;
    const dim3 grid((unsigned)(fa.W * ncb)), block(kT);
    switch (fa.nb) {
        case 32: hipLaunchKernelGGL((gj_update_kernel<Wd, 32>), grid, block, (upd_lds<Wd, 32>(fa.n, nb)), s, fa, j0, nb, ncb, c_lo, c_hi); break;
        case 16: hipLaunchKernelGGL((gj_update_kernel<Wd, 16>), grid, block, (upd_lds<Wd, 16>(fa.n, nb)), s, fa, j0, nb, ncb, c_lo, c_hi); break;
        case 8: hipLaunchKernelGGL((gj_update_kernel<Wd, 8>), grid, block, (upd_lds<Wd, 8>(fa.n, nb)), s, fa, j0, nb, ncb, c_lo, c_hi); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <class Wd>
hipError_t launch_block(const FA &fa, int j0, int nbw, int write_z, int o0, hipStream_t s) {
    const int nw = (fa.n + 63) / 64;
    const dim3 grid((unsigned)fa.W), block((unsigned)(64 * nw));
    constexpr int CW = sizeof(Wd) == 8 ? 16 : 8;     // n <= 512
    constexpr int CN = sizeof(Wd) == 8 ? 8 : 2;      // n <= 1024
    if (block_cpt<Wd>(fa.n) == CW) {
        const size_t lds = blk_lds<Wd, CW>(nw);
        if (nw <= 4) hipLaunchKernelGGL((gj_block_kernel<Wd, CW, 256>), grid, block, lds, s, fa, j0, nbw, write_z, o0);
        else hipLaunchKernelGGL((gj_block_kernel<Wd, CW, 512>), grid, block, lds, s, fa, j0, nbw, write_z, o0);
    } else {
        const size_t lds = blk_lds<Wd, CN>(nw);
        hipLaunchKernelGGL((gj_block_kernel<Wd, CN, 1024>), grid, block, lds, s, fa, j0, nbw, write_z, o0);
    }
    return hipGetLastError();
}

template <class Wd>
hipError_t launch_pr(const FA &fa, hipStream_t s) {
    const int n = fa.n;
    int dev = 0, lds_max = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) return e;
    // the kernel's static arrays and a margin stay out of the budget; a panel
    // starting at j0 keeps n - j0 entries per pending vector, so the later
    // panels take more pairs
    const size_t budget = lds_max > 2048 ? (size_t)lds_max - 2048 : 0;
    if (pr_lds<Wd>(n, pr_pairs<Wd>(n, budget)) > 65536) {
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(&pr_panel_kernel<Wd>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, (int)budget);
        if (e != hipSuccess) return e;
    }
    const dim3 grid((unsigned)fa.W), block(kPrThreads);
    if (n & 1) {                                        // records pf = 0
        const int P = pr_pairs<Wd>(n, budget);
        hipLaunchKernelGGL(pr_panel_kernel<Wd>, grid, block, pr_lds<Wd>(n, P), s, fa, 0, P, 0);
        return hipGetLastError();
    }
    int cur = 0;
    for (int j0 = 0, P = 0; j0 < n; j0 += 2 * P) {
        P = pr_pairs<Wd>(n - j0, budget);
        hipLaunchKernelGGL(pr_panel_kernel<Wd>, grid, block, pr_lds<Wd>(n - j0, P), s, fa, j0, P, cur);
        const int j1 = j0 + 2 * P;
        if (j1 < n) {
            const int nt = (n - j1 + 63) / 64;
            hipLaunchKernelGGL(pr_trail_kernel<Wd>, dim3((unsigned)(fa.W * nt * (nt + 1) / 2)), dim3(kT), 0, s, fa, j1,
                               P, cur, nt);
            cur ^= 1;
        }
    }
    return hipGetLastError();
}

template <class Wd>
hipError_t launch_pf_inverse(const FA &fa, hipStream_t s) {
    const int n = fa.n, W = fa.W, nt = (n + 63) / 64;
    hipError_t e;
    const size_t ld = vdiag_lds<Wd>(), lr = vrow_lds<Wd>();
    if (ld > 65536 && (e = hipFuncSetAttribute(reinterpret_cast<const void *>(&pr_vdiag_kernel<Wd>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)ld)) != hipSuccess)
        return e;
    if (lr > 65536 && (e = hipFuncSetAttribute(reinterpret_cast<const void *>(&pr_vrow_kernel<Wd>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lr)) != hipSuccess)
        return e;
    const int bpw = (n + 3) / 4;
    hipLaunchKernelGGL(pr_uasm_kernel<Wd>, dim3((unsigned)(W * bpw)), dim3(kT), 0, s, fa, bpw);
    hipLaunchKernelGGL(pr_vdiag_kernel<Wd>, dim3((unsigned)(W * nt)), dim3(kT), ld, s, fa, nt);
    for (int I = nt - 2; I >= 0; --I)
        hipLaunchKernelGGL(pr_vrow_kernel<Wd>, dim3((unsigned)(W * (nt - 1 - I))), dim3(kT), lr, s, fa, I, nt);
    hipLaunchKernelGGL(pr_inv_kernel<Wd>, dim3((unsigned)(W * nt * (nt + 1) / 2)), dim3(kT), 0, s, fa, nt);
    return hipGetLastError();
}

template <class T>
hipError_t factor_t(const FactorArgs &in, hipStream_t s) {
    using Wd = typename Wide<T>::type;
    FA a;
    a.kind = in.kind; a.W = in.W; a.n = in.n; a.sites = in.sites;
    a.src = in.src; a.occ = in.occ;
    a.work = static_cast<uint8_t *>(in.work);
    a.L = work_layout(in.n, sizeof(Wd), in.kind == LRX_PF);
    a.inv = in.inv; a.logabs = in.logabs; a.phase = in.phase; a.flags = in.flags;
    a.report = in.report; a.refresh = in.refresh; a.packed = in.packed;
    const int n = in.n, W = in.W;
    const int tiles = (n + 31) / 32;
    hipError_t e;
    hipLaunchKernelGGL(init_acc_kernel<Wd>, dim3((W + 255) / 256), dim3(256), 0, s, a);
    if (a.kind == LRX_PF) {
        hipLaunchKernelGGL(load_kernel<Wd>, dim3((unsigned)(W * tiles * tiles)), dim3(kT), 0, s, a, tiles);
        if ((e = launch_pr<Wd>(a, s)) != hipSuccess) return e;
        if ((e = launch_pf_inverse<Wd>(a, s)) != hipSuccess) return e;
        const int groups = (n + kT / 64 - 1) / (kT / 64);
        const size_t flds = (size_t)(kT / 64) * n * sizeof(Wd);   // one row per wave (64 KB at n = 1024, complex128)
        if (flds > 60 * 1024 &&
            (e = hipFuncSetAttribute(reinterpret_cast<const void *>(&final_pf_kernel<T, Wd>),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)flds)) != hipSuccess)
            return e;
        hipLaunchKernelGGL((final_pf_kernel<T, Wd>), dim3((unsigned)(W * groups)), dim3(kT), flds, s, a, groups);
        if (a.packed && (n & 63)) {
            const int nt = (n + 63) / 64;
            hipLaunchKernelGGL(pk_zero_tail_kernel<T>, dim3((unsigned)(W * nt)), dim3(kT), 0, s, a, nt);
        }
        hipLaunchKernelGGL(finish_kernel<Wd>, dim3((W + 255) / 256), dim3(256), 0, s, a);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(load_kernel<Wd>, dim3((unsigned)(W * tiles * tiles)), dim3(kT), 0, s, a, tiles);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    constexpr int kOuter = 64;
    const int pwb = 4 * block_cpt<Wd>(n);
    a.nb = pwb;
    for (int o0 = 0; o0 < n; o0 += kOuter) {
        const int nbo = min(kOuter, n - o0);
        for (int j0 = o0; j0 < o0 + nbo; j0 += pwb) {
            const int nbw = min(pwb, o0 + nbo - j0);
            e = launch_block<Wd>(a, j0, nbw, nbw < nbo ? 1 : 0, o0, s);
            if (e != hipSuccess) return e;
            e = launch_update<Wd>(a, j0, nbw, o0, o0 + nbo, s);
            if (e != hipSuccess) return e;
        }
        e = launch_outer<Wd>(a, o0, nbo, s);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(src_perm_kernel, dim3(W), dim3(kT), sizeof(int) * 2 * (size_t)n, s, a);
    const int rpb = 8;
    const int bpw = (n + rpb - 1) / rpb;
    hipLaunchKernelGGL((final_det_kernel<T, Wd>), dim3((unsigned)(W * bpw)), dim3(kT), sizeof(int) * (size_t)n, s,
                       a, rpb, bpw);
    hipLaunchKernelGGL(finish_kernel<Wd>, dim3((W + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

namespace lrx {

size_t factor_work_bytes(int kind, int dtype, int W, int n) {
    return (size_t)W * work_layout(n, wide_bytes(dtype), kind == LRX_PF).stride;
}

hipError_t factor(const FactorArgs &a, hipStream_t s) {
    switch (a.dtype) {
        case LRX_F32: return factor_t<float>(a, s);
        case LRX_F64: return factor_t<double>(a, s);
        case LRX_C64: return factor_t<cf32>(a, s);
        case LRX_C128: return factor_t<cf64>(a, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
