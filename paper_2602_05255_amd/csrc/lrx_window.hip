// Persistent window kernel: one launch advances every walker of an uneven
// batch (several size classes n, one state per class) by `steps` delayed
// steps (Sec. II.C), flushing each walker's slots into M0 whenever its window
// fills (Eq. delayed_Ainv).
//
// Work items are whole walkers, handed out heaviest first (classes by n
// descending, a longest-processing-time order) from a device counter, so the
// large classes start early and the small ones fill the tail.  A work-group of
// four waves keeps one walker for the whole window: propose -> decision ->
// delayed accept -> commit, step after step, with only work-group barriers
// between the phases (the slot data written by one step is read by the next
// inside the same work-group, so no data crosses compute units), and the
// walker's flush runs as 64-column strips in the same work-group.  The size
// class picks the row-chunk specialisation of the step functions shared with
// the per-step kernels.
#include <mutex>

#include "lrx_det_impl.hpp"
#include "lrx_flush_impl.hpp"

namespace {

using namespace lrxdet;
using namespace lrxfl;
using lrx::StepArgs;
using lrx::WindowArgs;
using lrx::WindowClass;

constexpr int kWindowThreads = 256;   // det_propose_walker with NW = 4 and the accept rows share it

// The walker's flush M0 -= B A^T (Eq. delayed_Ainv), strip after strip.
template <class T>
__device__ __forceinline__ void window_flush(const StepArgs &a, int w, int tau, unsigned char *smem) {
    StepArgs f = a;
    f.tau = tau;
    T *s_a = reinterpret_cast<T *>(smem);
    int *s_live = reinterpret_cast<int *>(s_a + FlushStripLds<T>::kA);
    const int tpd = (a.n + 63) / 64;
    for (int strip = 0; strip < tpd; ++strip) {
        __syncthreads();
        det_flush_strip<T>(f, w, strip, tpd, s_a, s_live, s_live + a.K * a.KM);
    }
    __syncthreads();
}

template <class T, int KM, int NCH>
__device__ __forceinline__ void window_walker(const WindowClass &wc, int steps, int w, unsigned char *smem) {
    using Wd = typename Wide<T>::type;
    constexpr int V = vec16<T>();
    constexpr int NEL = NCH * V;
    constexpr int NI = (NCH * V / 4) > 1 ? NCH * V / 4 : 1;   // entries per thread of a 256-wide column
    constexpr int RB = rows_per_batch<T, NEL, KM>();
    StepArgs a = wc.a;
    const int W = a.W, K = a.K;
    int tau = a.tau;
    for (int t = 0; t < steps; ++t) {
        a.tau = tau;
        a.k = wc.k + (size_t)t * W;
        a.rows = wc.elec + (size_t)t * W * KM;
        a.slot = wc.slot + (size_t)t * W * KM;
        a.u01 = wc.u01 ? wc.u01 + (size_t)t * W : nullptr;
        a.ratio = static_cast<Wd *>(wc.ratio) + (size_t)t * W;
        a.accept = wc.accept + (size_t)t * W;
        a.counter = wc.a.counter + (uint64_t)t;
        // The thread index is made opaque once per step so that the compiler
        // recomputes the per-thread addresses of each phase instead of keeping
        // them all live across the whole window.
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        det_propose_walker<T, KM, 4, NI>(a, w, smem, tid);
        __syncthreads();
        tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        det_accept_rows_block<T, KM, NEL, RB, 4, true>(a, w, 0, 0, a.n, smem, tid);
        __syncthreads();
        if (++tau == K) {
            window_flush<T>(a, w, K, smem);
            tau = 0;
        }
    }
}

template <class T, int KM>
__global__ __launch_bounds__(kWindowThreads, 2) void det_window_kernel(WindowArgs wa) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int s_item;
    constexpr int V = vec16<T>();
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(wa.queue, 1u);
        __syncthreads();
        // The item is block-uniform: keep it (and everything addressed through it) in scalar registers.
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= wa.walkers) break;     // every work-group leaves once the list is drained
        // classes are in processing order (n descending): walker = position within its class
        int c = 0, w = item;
        while (w >= wa.cls[c].a.W) { w -= wa.cls[c].a.W; ++c; }
        c = __builtin_amdgcn_readfirstlane(c);
        w = __builtin_amdgcn_readfirstlane(w);
        const WindowClass &wc = wa.cls[c];
        switch (wc.nch) {
            case 1: window_walker<T, KM, 1>(wc, wa.steps, w, smem); break;
            case 2: window_walker<T, KM, 2>(wc, wa.steps, w, smem); break;
            case 4: window_walker<T, KM, 4>(wc, wa.steps, w, smem); break;
            case 8: if constexpr (V <= 2) window_walker<T, KM, 8>(wc, wa.steps, w, smem); break;
            default: break;
        }
    }
}

__global__ void window_reset_kernel(uint32_t *queue) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *queue = 0u;
}

template <class T, int KM> size_t window_lds_t(int K, int nch_max) {
    constexpr int V = vec16<T>();
    const size_t npad = (size_t)nch_max * V * LRX_WAVE;
    const size_t acc = sizeof(T) * (KM * npad + KM * KM + (size_t)K * KM * KM + (size_t)kWaves * kZB * 8 * KM);
    const size_t prop = propose_lds_bytes<T, KM, 4>(K);
    const size_t fl = sizeof(T) * FlushStripLds<T>::kA + sizeof(int) * ((size_t)K * KM + 1);
    return acc > prop ? (acc > fl ? acc : fl) : (prop > fl ? prop : fl);
}

template <class T, int KM> hipError_t window_t(const WindowArgs &a, int grid, size_t lds, hipStream_t s) {
    if (lds > 65536) {
        hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&det_window_kernel<T, KM>),
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(window_reset_kernel, dim3(1), dim3(64), 0, s, a.queue);
    hipLaunchKernelGGL((det_window_kernel<T, KM>), dim3((unsigned)grid), dim3(kWindowThreads), lds, s, a);
    return hipGetLastError();
}

template <class T> hipError_t window_k(const WindowArgs &a, int grid, size_t lds, hipStream_t s) {
    switch (a.cls[0].a.KM) {
        case 1: return window_t<T, 1>(a, grid, lds, s);
        case 2: return window_t<T, 2>(a, grid, lds, s);
        case 4: return window_t<T, 4>(a, grid, lds, s);
        case 8: return window_t<T, 8>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

template <class T> size_t window_lds_k(int KM, int K, int nch_max) {
    switch (KM) {
        case 1: return window_lds_t<T, 1>(K, nch_max);
        case 2: return window_lds_t<T, 2>(K, nch_max);
        case 4: return window_lds_t<T, 4>(K, nch_max);
        case 8: return window_lds_t<T, 8>(K, nch_max);
    }
    return 0;
}

// The work counter of lrx_det_window_noalloc, held by the library on every
// device it runs on (until the process ends).  Host code never passes
// `scratch` itself: its device address comes from hipGetSymbolAddress, once per
// device.
static __device__ __align__(256) uint32_t scratch[LRX_NOALLOC_SCRATCH_WORDS];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t *g_scratch_ptr[kMaxDevices];

}  // namespace

namespace lrx {

hipError_t window_scratch(uint32_t **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[dev] = static_cast<uint32_t *>(p);
    }
    *out = g_scratch_ptr[dev];
    return hipSuccess;
}

size_t window_lds_bytes(int dtype, int KM, int K, int nch_max) {
    switch (dtype) {
        case LRX_F32: return window_lds_k<float>(KM, K, nch_max);
        case LRX_F64: return window_lds_k<double>(KM, K, nch_max);
    }
    return 0;
}

hipError_t det_window(int dtype, const WindowArgs &a, int grid, size_t lds, hipStream_t s) {
    switch (dtype) {
        case LRX_F32: return window_k<float>(a, grid, lds, s);
        case LRX_F64: return window_k<double>(a, grid, lds, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace lrx
