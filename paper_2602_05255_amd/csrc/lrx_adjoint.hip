// Low-rank log-determinant / log-Pfaffian of a walker state and the
// hand-written adjoints.
//
// DET.  M_w = A_w + B_w C_w^T, A_w = Phi[occ_w] (rows = electron labels).  By
// the matrix determinant lemma (Sec. II.A, with dense u, v):
//   log det M = log det A + log det R,  R = I_r + C^T P,  P = A^-1 B.
// The state holds A^-T, flushed (M0) or in the delayed form of Sec. II.C
//   A^-T = M0 - Fb Fa^T,  Fb[i][te] = b_te[i],  Fa[j][te] = a_te[j]  (Eq. delayed_Ainv),
// so P = M0^T B - Fa (Fb^T B) and Q = A^-T C = M0 C - Fb (Fa^T C): the slot
// terms cost O(n tau r) and the state is used as it stands (no flush).
// Gradients (holomorphic; torch passes the cotangent g and expects
// conj-weighted results):
//   d/dM log det M = M^-T = A^-T - Q R^-T P^T   (Woodbury, Eq. det_inv)
//   dB = g conj(M^-T C) = g conj(Q R^-T),  dC = g conj(M^-1 B) = g conj(P R^-1)
//   dPhi[s] = sum_{w, i: occ_w[i] = s} g_w conj(M_w^-T[i, :])
//           = sum g_w conj(M0_w[i, :])  -  E F,
//   E[s][w RT + c] = g_w conj(Q_w[i][c])        (c < r)
//                    g_w conj(b_te,w[i])         (c = r + te, delayed form)
//   F[w RT + c][j] = conj((P_w R_w^-1)[j][c])   (c < r)
//                    conj(a_te,w[j])             (c = r + te).
//
// PF.  M_w = A_w - U_w J U_w^T with A_w = F[occ_w][:, occ_w] skew and U_w an
// n x 2k dense matrix (Eqs. pf_ratio, pf_R):
//   log pf M = log pf A + log pf R - log pf J,  R = J + U^T P,  P = A^-1 U,
// with A^-1 = M0 + Fa Rb Fa^T in the delayed form (Eq. pf_delayed_Ainv, Rb the
// block diagonal of the R_t^-1).  Gradients: d log pf M / dM_ij = (1/2) (M^-1)_ji
// (Appendix A, Eq. pf_grad), M^-1 = A^-1 + P R^-1 P^T (Eq. pf_inv), and
//   d log pf M / dU = -M^-1 U J = P R^-1          (from M^-1 U = P R^-1 J)
//   dF[a][b] = -(1/2) sum_{w: a, b occupied} g_w conj(M_w^-1[pos_w(a)][pos_w(b)]).
//
// Every reduction runs in a fixed order: the site sums walk the walkers in
// index order through a per-walker position map (no atomics), and the E F
// product is split over its inner dimension into partial sums that are added in
// split order, so the gradients are bitwise reproducible.
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

template <class T> __device__ __forceinline__ T scale_(T a, double s);
template <> __device__ __forceinline__ float scale_<float>(float a, double s) { return a * (float)s; }
template <> __device__ __forceinline__ double scale_<double>(double a, double s) { return a * s; }
template <> __device__ __forceinline__ cf32 scale_<cf32>(cf32 a, double s) { return {a.x * (float)s, a.y * (float)s}; }
template <> __device__ __forceinline__ cf64 scale_<cf64>(cf64 a, double s) { return {a.x * s, a.y * s}; }

// ------------------------------------------------------------------ forward
// One work-group per walker, rows of M0 streamed by the waves (lane owns NEL
// columns j).  Before the stream: the slot products YC = Fa^T C and
// ZB = Fb^T B (DET) or WU = Rb Fa^T U (PF) of the delayed form.
//   DET: Q[i][c] = M0[i,:] . C[:,c] - sum_te Fb[i][te] YC[te][c] (one wave
//        reduction per row), P[j][c] = sum_i M0[i][j] B[i][c] (per-lane
//        accumulation) - sum_te Fa[j][te] ZB[te][c]; R = I + C^T P.
//   PF : P[i][c] = M0[i,:] . U[:,c] + sum_te Fa[i][te] WU[te][c]; R = J + U^T P,
//        made exactly skew.
template <class T, int RR, int NEL, bool PF>
__global__ __launch_bounds__(kT) void lowrank_fwd_kernel(LowRankArgs a) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NCH = NEL / V;
    extern __shared__ __align__(16) unsigned char smem[];
    const int w = blockIdx.x, n = a.n, r = a.r, TE = a.TE;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int npad = NCH * V * 64;
    const T *M = static_cast<const T *>(a.inv) + (size_t)w * n * n;
    const T *B = static_cast<const T *>(a.B) + (size_t)w * n * r;     // PF: U
    const T *C = PF ? B : static_cast<const T *>(a.C) + (size_t)w * n * r;
    const T *fa = TE ? static_cast<const T *>(a.fa) + (size_t)w * a.KA * n : nullptr;
    T *P = static_cast<T *>(a.P) + (size_t)w * n * r;
    T *Q = PF ? nullptr : static_cast<T *>(a.Q) + (size_t)w * n * r;
    T *s_c = reinterpret_cast<T *>(smem);            // C (PF: U), [RR][npad]
    T *s_p = s_c + (size_t)RR * npad;                // P accumulation (DET), [RR][npad]
    T *s_r = s_p + (PF ? 0 : (size_t)RR * npad);     // R partials [kWaves][RR][RR], then R (PF)
    T *s_y = s_r + (size_t)(kWaves + 1) * RR * RR;   // YC (DET) or WU (PF), [TE][RR]
    T *s_z = s_y + (size_t)TE * RR;                  // ZB (DET), [TE][RR]
    for (int idx = tid; idx < RR * npad; idx += kT) {
        const int c = idx / npad, j = idx - c * npad;
        s_c[idx] = (c < r && j < n) ? C[(size_t)j * r + c] : zero<T>();
        if constexpr (!PF) s_p[idx] = zero<T>();
    }
    __syncthreads();
    // slot products, one slot column per thread (TE <= 256)
    if (tid < TE) {
        const int te = tid;
        T y[RR], z[RR];
#pragma unroll
        for (int c = 0; c < RR; ++c) { y[c] = zero<T>(); z[c] = zero<T>(); }
        const T *arow = fa + (size_t)te * n;
#pragma unroll 4
        for (int j = 0; j < n; ++j) {
            const T av = arow[j];
#pragma unroll
            for (int c = 0; c < RR; ++c) y[c] = fmac(av, s_c[c * npad + j], y[c]);
            if constexpr (!PF) {
                const T bv = static_cast<const T *>(a.fb)[((size_t)w * n + j) * a.KK + te];
#pragma unroll
                for (int c = 0; c < RR; ++c) z[c] = fmac(bv, B[(size_t)j * r + min(c, r - 1)], z[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < RR; ++c) {
            s_y[te * RR + c] = (c < r) ? y[c] : zero<T>();
            if constexpr (!PF) s_z[te * RR + c] = (c < r) ? z[c] : zero<T>();
        }
    }
    __syncthreads();
    if constexpr (PF) {
        // WU[2t + e][c] = sum_e' Rt^-1[e][e'] (Fa^T U)[2t + e'][c]  (R_t^-1 = fb[t], 2 x 2)
        T wu[RR];
        const int te = tid;
        if (te < TE) {
            const T *rt = static_cast<const T *>(a.fb) + ((size_t)w * a.K + te / 2) * 4;
            const int e = te & 1, t0 = te & ~1;
#pragma unroll
            for (int c = 0; c < RR; ++c)
                wu[c] = fmac(rt[e * 2 + 0], s_y[t0 * RR + c], rt[e * 2 + 1] * s_y[(t0 + 1) * RR + c]);
        }
        __syncthreads();
        if (te < TE) {
#pragma unroll
            for (int c = 0; c < RR; ++c) s_y[te * RR + c] = wu[c];
        }
        __syncthreads();
    }
    T pacc[PF ? 1 : NEL][RR];
    if constexpr (!PF) {
#pragma unroll
        for (int e = 0; e < NEL; ++e)
#pragma unroll
            for (int c = 0; c < RR; ++c) pacc[e][c] = zero<T>();
    }
    T racc = zero<T>();                              // PF: lane (c, d) of R partial
    const int rc_ = lane / RR, rd_ = lane % RR;
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
            bi[c] = (!PF && c < r) ? B[(size_t)i * r + c] : zero<T>();
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
                    if constexpr (!PF) pacc[ch * V + v][c] = fmac(x[ch * V + v], bi[c], pacc[ch * V + v][c]);
                }
            }
        }
        // slot term of row i, spread over the lanes (lane owns slot columns te = lane + 64 m)
        for (int te = lane; te < TE; te += 64) {
            if constexpr (PF) {
                const T av = fa[(size_t)te * n + i];                 // Fa[i][te]
#pragma unroll
                for (int c = 0; c < RR; ++c) q[c] = fmac(av, s_y[te * RR + c], q[c]);
            } else {
                const T bv = static_cast<const T *>(a.fb)[((size_t)w * n + i) * a.KK + te];   // Fb[i][te]
#pragma unroll
                for (int c = 0; c < RR; ++c) q[c] = fmsc(bv, s_y[te * RR + c], q[c]);
            }
        }
        const T qt = wave_sum_multi<T, RR>(q);     // lane c (mod RR): row i, column c
        if constexpr (PF) {
            if (lane < r) P[(size_t)i * r + lane] = qt;
            // R[c][d] += U[i][c] P[i][d] on lane c * RR + d
            const T pd = shfl_any(qt, rd_);
            if (lane < RR * RR) racc = fmac(s_c[rc_ * npad + i], pd, racc);
        } else {
            if (lane < r) Q[(size_t)i * r + lane] = qt;
        }
    }
    if constexpr (!PF) {
        // P = sum over the waves of their accumulators, one wave at a time, minus Fa ZB.
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
        for (int j = tid; j < n; j += kT) {
            T pj[RR];
#pragma unroll
            for (int c = 0; c < RR; ++c) pj[c] = s_p[c * npad + j];
            for (int te = 0; te < TE; ++te) {
                const T av = fa[(size_t)te * n + j];
#pragma unroll
                for (int c = 0; c < RR; ++c) pj[c] = fmsc(av, s_z[te * RR + c], pj[c]);
            }
#pragma unroll
            for (int c = 0; c < RR; ++c) s_p[c * npad + j] = pj[c];
        }
        __syncthreads();
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
    } else {
        if (lane < RR * RR) s_r[wv * RR * RR + lane] = racc;
        __syncthreads();
        if (tid < RR * RR) {      // R = J + U^T P, exactly skew: (R - R^T) / 2 of the sum
            const int c = tid / RR, d = tid - c * RR;
            T s = zero<T>(), st = zero<T>();
            for (int q = 0; q < kWaves; ++q) { s = s + s_r[q * RR * RR + tid]; st = st + s_r[q * RR * RR + d * RR + c]; }
            const int h = r / 2;
            T jv = zero<T>();
            if (c < r && d < r) jv = (d == c + h && c < h) ? one<T>() : ((c == d + h && d < h) ? -one<T>() : zero<T>());
            s_r[kWaves * RR * RR + tid] = (c < r && d < r) ? jv + scale_<T>(s - st, 0.5) : zero<T>();
        }
    }
    __syncthreads();
    if (tid == 0) {
        T rm[RR * RR], ri[RR * RR];
        const T *src = PF ? s_r + kWaves * RR * RR : s_r;
        for (int q = 0; q < RR * RR; ++q) { rm[q] = src[q]; ri[q] = zero<T>(); }
        Wd val;
        bool sing = false;
        if constexpr (PF) {
            T rp[RR * RR];
            for (int q = 0; q < RR * RR; ++q) rp[q] = rm[q];
            small_pf<T, RR>(rp, r, val);
            // pf J = (-1)^(k (k - 1) / 2) for the 2k x 2k skew identity (k = r / 2)
            const int k = r / 2;
            if (((k * (k - 1)) / 2) & 1) val = -val;
            Wd dd;
            bool s2;
            small_lu_det_inv<T, RR>(rm, r, ri, dd, s2);
            sing = s2;
        } else {
            small_lu_det_inv<T, RR>(rm, r, ri, val, sing);
        }
        T *Ri = static_cast<T *>(a.Rinv) + (size_t)w * r * r;
        for (int c = 0; c < r; ++c)
            for (int d = 0; d < r; ++d) Ri[c * r + d] = ri[c * RR + d];
        double la = a.state_logabs[w];
        Wd ph = static_cast<const Wd *>(a.state_phase)[w];
        if (sing || is_zero(val) || !finite_v(val)) {
            a.logabs[w] = -INFINITY;
            static_cast<Wd *>(a.phase)[w] = zero<Wd>();
        } else {
            accum_logphase(val, &la, &ph);
            a.logabs[w] = la;
            static_cast<Wd *>(a.phase)[w] = ph;
        }
    }
}

// ------------------------------------------------------------------ backward
// Per row j of walker w:
//   DET: Y = P R^-1, Z = Q R^-T; dC = g conj(Y), dB = g conj(Z);
//        F[w RT + c][j] = conj(Y[j][c]), F[w RT + r + te][j] = conj(a_te[j]).
//   PF : Y = P R^-1; dU = g conj(Y); Y kept (in dB's place) for the E panel.
template <class T, int RR, bool PF>
__global__ __launch_bounds__(kT) void lowrank_small_kernel(LowRankArgs a, int bpw) {
    using Wd = typename Wide<T>::type;
    const int w = blockIdx.x / bpw, jb = blockIdx.x - w * bpw;
    const int n = a.n, r = a.r, RT = a.r + a.TE;
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
    T pj[RR], qj[RR];
#pragma unroll
    for (int c = 0; c < RR; ++c) {
        pj[c] = (c < r) ? P[(size_t)j * r + c] : zero<T>();
        qj[c] = (!PF && c < r) ? static_cast<const T *>(a.Q)[(size_t)w * n * r + (size_t)j * r + c] : zero<T>();
    }
    T *dB = static_cast<T *>(a.dB) + (size_t)w * n * r;
    T *dC = PF ? nullptr : static_cast<T *>(a.dC) + (size_t)w * n * r;
    T *Yk = PF ? static_cast<T *>(a.Y) + (size_t)w * n * r : nullptr;
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
        if constexpr (PF) {
            dB[(size_t)j * r + c] = g * conjv(y);     // dU
            Yk[(size_t)j * r + c] = y;
        } else {
            dC[(size_t)j * r + c] = g * conjv(y);
            dB[(size_t)j * r + c] = g * conjv(z);
            F[((size_t)w * RT + c) * n + j] = conjv(y);
        }
    }
    if constexpr (!PF) {
        const T *fa = static_cast<const T *>(a.fa) + (size_t)w * a.KA * n;
        for (int te = 0; te < a.TE; ++te) F[((size_t)w * RT + r + te) * n + j] = conjv(fa[(size_t)te * n + j]);
    }
}

__global__ void fill_int_kernel(int *p, size_t count, int v) {
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// pos[w][s] = i for occ[w][i] = s (every other entry -1).
__global__ void pos_scatter_kernel(LowRankArgs a) {
    const size_t total = (size_t)a.W * a.n;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int w = (int)(idx / a.n), i = (int)(idx - (size_t)w * a.n);
        const int s = a.occ[idx];
        if (s >= 0 && s < a.sites) a.pos[(size_t)w * a.sites + s] = i;
    }
}

// E[s][w RT + c] for one site s per work-group (zero where walker w leaves s empty).
//   DET: g conj(Q[i][c]) | g conj(b_te[i]);   PF: g conj(Y[i][c]) | g conj((Fa Rb)[i][te]).
template <class T, bool PF>
__global__ __launch_bounds__(kT) void lowrank_e_kernel(LowRankArgs a) {
    using Wd = typename Wide<T>::type;
    const int s = blockIdx.x, n = a.n, r = a.r, RT = a.r + a.TE;
    T *E = static_cast<T *>(a.E) + (size_t)s * a.W * RT;
    for (int idx = threadIdx.x; idx < a.W * RT; idx += kT) {
        const int w = idx / RT, c = idx - w * RT;
        const int i = a.pos[(size_t)w * a.sites + s];
        T v = zero<T>();
        if (i >= 0) {
            const T g = conv<T>(static_cast<const Wd *>(a.g)[w]);
            if (c < r) {
                const T *src = static_cast<const T *>(PF ? a.Y : a.Q) + (size_t)w * n * r;
                v = g * conjv(src[(size_t)i * r + c]);
            } else if constexpr (PF) {
                const int te = c - r, t0 = te & ~1, e = te & 1;
                const T *fa = static_cast<const T *>(a.fa) + (size_t)w * a.KA * n;
                const T *rt = static_cast<const T *>(a.fb) + ((size_t)w * a.K + te / 2) * 4;
                // (Fa Rb)[i][t0 + e] = sum_e' Fa[i][t0 + e'] Rt^-1[e'][e]
                const T far = fmac(fa[(size_t)t0 * n + i], rt[e], fa[(size_t)(t0 + 1) * n + i] * rt[2 + e]);
                v = g * conjv(far);
            } else {
                v = g * conjv(static_cast<const T *>(a.fb)[((size_t)w * n + i) * a.KK + (c - r)]);
            }
        }
        E[idx] = v;
    }
}

// PF: F[w RT + c][b] = conj(P[pos_w(b)][c]) | conj(a_te[pos_w(b)])  (zero where b is empty).
template <class T>
__global__ __launch_bounds__(kT) void pf_f_kernel(LowRankArgs a) {
    const int w = blockIdx.y, RT = a.r + a.TE, n = a.n, r = a.r;
    const int b = blockIdx.x * kT + threadIdx.x;
    if (b >= a.sites) return;
    const int i = a.pos[(size_t)w * a.sites + b];
    T *F = static_cast<T *>(a.F);
    const T *P = static_cast<const T *>(a.P) + (size_t)w * n * r;
    const T *fa = a.TE ? static_cast<const T *>(a.fa) + (size_t)w * a.KA * n : nullptr;
    for (int c = 0; c < RT; ++c) {
        T v = zero<T>();
        if (i >= 0) v = conjv(c < r ? P[(size_t)i * r + c] : fa[(size_t)(c - r) * n + i]);
        F[((size_t)w * RT + c) * a.sites + b] = v;
    }
}

// DET: out[s][j] = sum_w (in index order) [pos_w(s) >= 0] g_w conj(M0_w[pos_w(s)][j]).
template <class T>
__global__ __launch_bounds__(kT) void det_gather_kernel(LowRankArgs a, int col_blocks) {
    using Wd = typename Wide<T>::type;
    const int s = blockIdx.x / col_blocks, cb = blockIdx.x - s * col_blocks;
    const int n = a.n;
    const int j = cb * kT + threadIdx.x;
    const T *Minv = static_cast<const T *>(a.inv);
    const Wd *g = static_cast<const Wd *>(a.g);
    T acc = zero<T>();
    for (int w = 0; w < a.W; ++w) {
        const int i = __builtin_amdgcn_readfirstlane(a.pos[(size_t)w * a.sites + s]);
        if (i < 0) continue;
        if (j < n) acc = fmac(conv<T>(g[w]), conjv(Minv[((size_t)w * n + i) * n + j]), acc);
    }
    if (j < n) static_cast<T *>(a.dphi)[(size_t)s * n + j] = acc;
}

// PF: out[a][b] = sum_w (in index order) [pos_w(a), pos_w(b) >= 0] g_w conj(M0_w[pos_w(a)][pos_w(b)])
// over 64 x 64 tiles of the site x site output; thread: column b, rows a = a0 + 4 m + wave.
template <class T>
__global__ __launch_bounds__(kT) void pf_gather_kernel(LowRankArgs a, int tiles) {
    using Wd = typename Wide<T>::type;
    const int ta = blockIdx.x / tiles, tb = blockIdx.x - ta * tiles;
    const int S = a.sites, n = a.n;
    const int lb = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int b = tb * 64 + lb;
    __shared__ int s_pa[64];
    T acc[16];
#pragma unroll
    for (int m = 0; m < 16; ++m) acc[m] = zero<T>();
    const T *Minv = static_cast<const T *>(a.inv);
    const Wd *g = static_cast<const Wd *>(a.g);
    for (int w = 0; w < a.W; ++w) {
        __syncthreads();
        if (threadIdx.x < 64) {
            const int aa = ta * 64 + threadIdx.x;
            s_pa[threadIdx.x] = aa < S ? a.pos[(size_t)w * S + aa] : -1;
        }
        __syncthreads();
        const int pb = b < S ? a.pos[(size_t)w * S + b] : -1;
        if (pb < 0) continue;
        const T gw = conv<T>(g[w]);
        const T *Mw = Minv + (size_t)w * n * n;
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int pa = s_pa[4 * m + wv];
            if (pa >= 0) acc[m] = fmac(gw, conjv(Mw[(size_t)pa * n + pb]), acc[m]);
        }
    }
    if (b < S) {
        T *out = static_cast<T *>(a.dphi);
#pragma unroll
        for (int m = 0; m < 16; ++m) {
            const int aa = ta * 64 + 4 * m + wv;
            if (aa < S) out[(size_t)aa * S + b] = acc[m];
        }
    }
}

// Partial products part[ks][s][j] = sum_{k in split ks} E[s][k] F[k][j] (rows = sites,
// cols = n (DET) or sites (PF), inner = W RT): 64 x 64 tiles, MFMA fragments from
// LDS-staged chunks.  Each split is summed in a fixed order.
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
__global__ __launch_bounds__(256) void lowrank_gemm_kernel(LowRankArgs a, int cols, int tiles_c, int ksplit) {
    using R = typename Real<T>::type;
    using A4 = typename Acc<R>::type;
    constexpr int KC = 256 / (int)sizeof(T);
    constexpr int SE = KC + 1, SF = 64 + 1;
    __shared__ T s_e[64 * SE];
    __shared__ T s_f[KC * SF];
    const int rows = a.sites, KI = a.W * (a.r + a.TE);
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
    T *part = static_cast<T *>(a.part) + (size_t)ks * rows * cols;
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
        const int col = tj * 64 + jb * 16 + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = ti * 64 + wv * 16 + acc_row<R>(lane, q);
            if (row < rows && col < cols) {
                T v;
                if constexpr (Real<T>::cplx) v = T{re[jb][q], im[jb][q]};
                else v = re[jb][q];
                part[(size_t)row * cols + col] = v;
            }
        }
    }
}

// out = alpha (out + sign sum_ks part[ks]), the splits added in order.
template <class T>
__global__ void lowrank_combine_kernel(LowRankArgs a, size_t count, int ksplit, double alpha, double sign) {
    T *out = static_cast<T *>(a.dphi);
    const T *part = static_cast<const T *>(a.part);
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        T s = zero<T>();
        for (int k = 0; k < ksplit; ++k) s = s + part[(size_t)k * count + i];
        out[i] = scale_<T>(out[i] + scale_<T>(s, sign), alpha);
    }
}

// Gradient of log pf of a flushed Pfaffian state: dA[w][i][j] = g_w conj((1/2) M_w[j][i])
// (Appendix A, Eq. pf_grad, M = A^-1).
template <class T>
__global__ void pf_grad_kernel(const T *M, const void *g, T *dA, int W, int n) {
    using Wd = typename Wide<T>::type;
    const size_t total = (size_t)W * n * n;
    for (size_t idx = blockIdx.x * (size_t)blockDim.x + threadIdx.x; idx < total; idx += (size_t)gridDim.x * blockDim.x) {
        const int w = (int)(idx / ((size_t)n * n));
        const size_t rem = idx - (size_t)w * n * n;
        const int i = (int)(rem / n), j = (int)(rem - (size_t)i * n);
        const T gw = conv<T>(static_cast<const Wd *>(g)[w]);
        dA[idx] = gw * conjv(scale_<T>(M[(size_t)w * n * n + (size_t)j * n + i], 0.5));
    }
}

template <class T, int RR, bool PF> hipError_t fwd_r(const LowRankArgs &a, hipStream_t s) {
    constexpr int V = vec16<T>();
    const int nch = (a.n + V * 64 - 1) / (V * 64);
    auto launch = [&](auto nel_tag) {
        constexpr int NEL = decltype(nel_tag)::value;
        const size_t lds = lrx::lowrank_lds_bytes(a.kind, a.dtype, a.n, RR, a.TE);
        if (lds > 65536) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&lowrank_fwd_kernel<T, RR, NEL, PF>),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL((lowrank_fwd_kernel<T, RR, NEL, PF>), dim3(a.W), dim3(kT), lds, s, a);
        return hipGetLastError();
    };
    if (nch <= 1) return launch(std::integral_constant<int, V>{});
    if (nch <= 2) return launch(std::integral_constant<int, 2 * V>{});
    if (nch <= 4) return launch(std::integral_constant<int, 4 * V>{});
    if constexpr (V <= 2) { if (nch <= 8) return launch(std::integral_constant<int, 8 * V>{}); }
    return hipErrorInvalidValue;
}

template <class T> hipError_t fwd_t(const LowRankArgs &a, hipStream_t s) {
    if (a.kind == LRX_PF) {
        if (a.r <= 2) return fwd_r<T, 2, true>(a, s);
        if (a.r <= 4) return fwd_r<T, 4, true>(a, s);
        return fwd_r<T, 8, true>(a, s);
    }
    if (a.r <= 1) return fwd_r<T, 1, false>(a, s);
    if (a.r <= 2) return fwd_r<T, 2, false>(a, s);
    if (a.r <= 4) return fwd_r<T, 4, false>(a, s);
    return fwd_r<T, 8, false>(a, s);
}

template <class T, bool PF> void small_launch(const LowRankArgs &a, hipStream_t s) {
    const int bpw = (a.n + kT - 1) / kT;
    const dim3 grid(a.W * bpw), block(kT);
    if (a.r <= 1) hipLaunchKernelGGL((lowrank_small_kernel<T, 1, PF>), grid, block, 0, s, a, bpw);
    else if (a.r <= 2) hipLaunchKernelGGL((lowrank_small_kernel<T, 2, PF>), grid, block, 0, s, a, bpw);
    else if (a.r <= 4) hipLaunchKernelGGL((lowrank_small_kernel<T, 4, PF>), grid, block, 0, s, a, bpw);
    else hipLaunchKernelGGL((lowrank_small_kernel<T, 8, PF>), grid, block, 0, s, a, bpw);
}

template <class T> hipError_t bwd_t(const LowRankArgs &a, hipStream_t s) {
    const bool pf = a.kind == LRX_PF;
    if (pf) small_launch<T, true>(a, s);
    else small_launch<T, false>(a, s);
    hipLaunchKernelGGL(fill_int_kernel, dim3(256), dim3(256), 0, s, a.pos, (size_t)a.W * a.sites, -1);
    hipLaunchKernelGGL(pos_scatter_kernel, dim3(512), dim3(256), 0, s, a);
    if (pf) hipLaunchKernelGGL((lowrank_e_kernel<T, true>), dim3(a.sites), dim3(kT), 0, s, a);
    else hipLaunchKernelGGL((lowrank_e_kernel<T, false>), dim3(a.sites), dim3(kT), 0, s, a);
    const int cols = pf ? a.sites : a.n;
    if (pf) {
        hipLaunchKernelGGL(pf_f_kernel<T>, dim3((a.sites + kT - 1) / kT, a.W), dim3(kT), 0, s, a);
        const int tiles = (a.sites + 63) / 64;
        hipLaunchKernelGGL(pf_gather_kernel<T>, dim3(tiles * tiles), dim3(kT), 0, s, a, tiles);
    } else {
        const int col_blocks = (a.n + kT - 1) / kT;
        hipLaunchKernelGGL(det_gather_kernel<T>, dim3(a.sites * col_blocks), dim3(kT), 0, s, a, col_blocks);
    }
    const int tiles_r = (a.sites + 63) / 64, tiles_c = (cols + 63) / 64;
    hipLaunchKernelGGL(lowrank_gemm_kernel<T>, dim3(tiles_r * tiles_c * a.ksplit), dim3(256), 0, s, a, cols, tiles_c,
                       a.ksplit);
    const size_t count = (size_t)a.sites * cols;
    hipLaunchKernelGGL(lowrank_combine_kernel<T>, dim3(1024), dim3(256), 0, s, a, count, a.ksplit,
                       pf ? -0.5 : 1.0, pf ? 1.0 : -1.0);
    return hipGetLastError();
}

}  // namespace

namespace lrx {

// Inner-dimension splits of the E F product: enough tiles to cover the chip,
// every split at least 256 deep.
int lowrank_ksplit(int kind, int W, int n, int r, int TE, int sites) {
    const int cols = kind == LRX_PF ? sites : n;
    const int tiles = ((sites + 63) / 64) * ((cols + 63) / 64);
    const int KI = W * (r + TE);
    int ks = 1;
    while (tiles * ks < 512 && KI / (ks * 2) >= 256 && ks < 16) ks *= 2;
    return ks;
}

size_t lowrank_lds_bytes(int kind, int dtype, int n, int RR, int TE) {
    const size_t es = bulk_bytes(dtype);
    const int per = (int)(16 / es) * 64;
    int nch = (n + per - 1) / per, p2 = 1;
    while (p2 < nch) p2 <<= 1;
    const size_t npad = (size_t)p2 * per;
    const bool pf = kind == LRX_PF;
    return es * ((pf ? 1 : 2) * (size_t)RR * npad + (size_t)(kWaves + 1) * RR * RR + (pf ? 1 : 2) * (size_t)TE * RR);
}

size_t lowrank_work_bytes(int kind, int dtype, int W, int n, int r, int TE, int sites) {
    const size_t es = bulk_bytes(dtype);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const int RT = r + TE;
    const int cols = kind == LRX_PF ? sites : n;
    const int ks = lowrank_ksplit(kind, W, n, r, TE, sites);
    size_t off = 0;
    off += al(sizeof(int) * (size_t)W * sites);          // pos
    off += al(es * (size_t)sites * W * RT);              // E
    off += al(es * (size_t)W * RT * cols);               // F
    off += al(es * (size_t)ks * sites * cols);           // partial products
    if (kind == LRX_PF) off += al(es * (size_t)W * n * r);   // Y = P R^-1
    return off;
}

void lowrank_bind_work(LowRankArgs &a, void *work) {
    const size_t es = bulk_bytes(a.dtype);
    auto al = [](size_t b) { return (b + 255) / 256 * 256; };
    const int RT = a.r + a.TE;
    const int cols = a.kind == LRX_PF ? a.sites : a.n;
    a.ksplit = lowrank_ksplit(a.kind, a.W, a.n, a.r, a.TE, a.sites);
    uint8_t *p = static_cast<uint8_t *>(work);
    a.pos = reinterpret_cast<int *>(p); p += al(sizeof(int) * (size_t)a.W * a.sites);
    a.E = p; p += al(es * (size_t)a.sites * a.W * RT);
    a.F = p; p += al(es * (size_t)a.W * RT * cols);
    a.part = p; p += al(es * (size_t)a.ksplit * a.sites * cols);
    a.Y = a.kind == LRX_PF ? p : nullptr;
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

hipError_t pf_grad(int dtype, const void *M, const void *g, void *dA, int W, int n, hipStream_t s) {
    const dim3 grid(1024), block(256);
    switch (dtype) {
        case LRX_F32: hipLaunchKernelGGL(pf_grad_kernel<float>, grid, block, 0, s, static_cast<const float *>(M), g,
                                         static_cast<float *>(dA), W, n); break;
        case LRX_F64: hipLaunchKernelGGL(pf_grad_kernel<double>, grid, block, 0, s, static_cast<const double *>(M), g,
                                         static_cast<double *>(dA), W, n); break;
        case LRX_C64: hipLaunchKernelGGL(pf_grad_kernel<cf32>, grid, block, 0, s, static_cast<const cf32 *>(M), g,
                                         static_cast<cf32 *>(dA), W, n); break;
        case LRX_C128: hipLaunchKernelGGL(pf_grad_kernel<cf64>, grid, block, 0, s, static_cast<const cf64 *>(M), g,
                                          static_cast<cf64 *>(dA), W, n); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace lrx
