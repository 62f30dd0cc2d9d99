// fill_learned.hip -- the one-axis fill with a learned find-bin index over an
// edge array too large for LDS, unit weights, 16-bit LDS counters: the
// variable-bin fill the benchmark times (arXiv:2401.13310 Sec. 3.1 find bin,
// weight increment and statistics; Sec. 3.2 two-stage accumulation).
//
// The general fill body issues about 60 vector instructions per event here.
// This kernel is the same computation laid out for the common case:
//   - the LDS window of 16-bit counters starts at LDS offset 0, so a counter's
//     word address is a shift of its bin;
//   - the learned index gives a one-bin interval for most events (the bin is
//     known without reading an edge); the coordinates of the others (two or
//     more candidates) go to a per-thread list in global memory and are
//     resolved after the workgroup's last batch, with the edge reads from
//     L2/HBM.  The event loop therefore issues no edge loads at all: loads of
//     a wave complete in issue order, so an edge load behind the next batch's
//     loads would wait for them.  The next batch is requested first thing in
//     every iteration;
//   - flow events and bins outside the window take the shared spill path (LDS
//     hot-bin cache, then global atomics);
//   - in-range events are counted as all events less the flow events (which
//     take the spill path anyway), x and x^2 summed per thread.
// When a workgroup's list is full the remaining candidates are searched in the
// loop (correct, slower; adversarial inputs only).
#include "fill_body.h"

namespace hg {

constexpr int kLeanU = 8;   // events per thread and iteration

// Segment and local feature of x, exactly as training computes them (FEAT 0:
// key feature of an axis of positive values, 1: key feature, 2: linear).
template <int FEAT>
__device__ __forceinline__ void lean_seg(double x, const AxisDev &ax, uint32_t kadd, int32_t &s, float &z)
{
    if (FEAT == 0)
        key_seg((uint32_t)((uint64_t)__double_as_longlong(x) >> 32) + kadd, ax, s, z);
    else if (FEAT == 1)
        key_seg(order_key32(x) - ax.key0, ax, s, z);
    else
        linear_seg(x, ax, s, z);
}

// Adds one event to bin g: the 16-bit window counter when g is in the window,
// else the spill path.
__device__ __forceinline__ void lean_add(const FillArgs &A, char *smem, uint32_t *win, int32_t g)
{
    const uint32_t l = (uint32_t)(g - A.win_lo);
    if (l < (uint32_t)A.win_len)
        lds_add_u32(&win[l >> 1], 1u << ((l & 1u) << 4));
    else
        spill<false>(A, smem, g, 1.0);
}

// The bin of an in-range x known to lie in [lo, hi] (global bins; lo > hi:
// the model gave no bound, the whole axis), found by binary search over the
// edges, then added.
__device__ __forceinline__ void lean_search_add(const FillArgs &A, char *smem, uint32_t *win, double x,
                                                int32_t lo, int32_t hi)
{
    if (lo > hi) {
        lo = 1;
        hi = A.ax[0].nbins;
    }
    search_one(x, A.ax[0].edges, A.ax[0].nbins, lo, hi);
    lean_add(A, smem, win, lo);
}

template <int FEAT>
__global__ void __launch_bounds__(kMaxThreads) fill_learned_kernel(const FillArgs A)
{
    constexpr int U = kLeanU;
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const AxisDev &ax = A.ax[0];
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;

    if (start == 0 && tid == 0 && A.entries)
        gl_add_u64(A.entries, (uint64_t)A.n);
    // LDS: the window at 0, then the model, the statistics partials, the
    // rare-list counter and the hot-bin cache (offsets from the host)
    uint32_t *win = reinterpret_cast<uint32_t *>(smem);
    const ModelSeg *model = reinterpret_cast<const ModelSeg *>(smem + ax.lds_model);
    // the list of a workgroup holds tcap coordinates per thread, thread t's
    // k-th at [k * threads + t]; a thread's count stays in a register
    {
        // the model, with the window's first bin subtracted from its offsets
        ModelSeg *dst = reinterpret_cast<ModelSeg *>(smem + ax.lds_model);
        for (int i = tid; i < ax.nseg; i += nthr) {
            ModelSeg ms = ax.model[i];
            ms.ai = (int32_t)((uint32_t)ms.ai - (uint32_t)A.win_lo);
            dst[i] = ms;
        }
        const int words = (A.win_len + 1) >> 1;
        for (int i = tid; i < words; i += nthr)
            win[i] = 0u;
    }
    cache_init<false>(A, smem);
    __syncthreads();

    const uint32_t kadd = 0x80000000u - ax.key0;
    double *rare = reinterpret_cast<double *>(A.rare + (int64_t)blockIdx.x * A.rare_cap);
    const uint32_t tcap = 2u * (uint32_t)A.rare_cap / (uint32_t)nthr;
    const uint32_t len = (uint32_t)(end > start ? end - start : 0);
    const uint32_t step = (uint32_t)nthr * U;
    __amdgpu_buffer_rsrc_t xb[1] = {column_rsrc(static_cast<const double *>(A.coords[0]) + start,
                                                len * (uint32_t)sizeof(double))};
    const __amdgpu_buffer_rsrc_t wb = column_rsrc(A.coords[0], 0u);
    double cx[U][1], cw[U];
    if (len > 0)
        load_batch<1, double, false, U>(xb, wb, 0, cx, cw);

    double sx = 0.0, sxx = 0.0;
    uint32_t nok = 0, nflow = 0;   // events of this thread, and those out of range
    uint32_t tcount = 0;           // coordinates this thread has listed
    int it = 0;
    // full batches need no per-event range check; the block's partial last
    // batch runs the same body with one
    auto iteration = [&](uint32_t base, auto full_t) {
        constexpr bool FULL = decltype(full_t)::value;
        double x[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            x[j] = cx[j][0];
        // the next batch first: no later load of this wave waits behind it
        load_batch<1, double, false, U>(xb, wb, base + step, cx, cw);
        __builtin_amdgcn_sched_barrier(0);

        int32_t s[U];
        float z[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            lean_seg<FEAT>(x[j], ax, kadd, s[j], z[j]);
        ModelSeg m[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            m[j] = model[s[j]];
        __builtin_amdgcn_sched_barrier(0);

        // each event is finished before the next one is looked at, so no
        // per-event masks stay live across the batch.  Bins are in window
        // coordinates (the staged model's offsets have the window start
        // subtracted).
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool ok = FULL || base + (uint32_t)j * nthr + tid < len;
            // for an in-range x, y stays within the segment's bins: the
            // conversions cannot overflow (an infinite width saturates and
            // is caught as an empty interval)
            const float y = model_eval(m[j], z[j]);
            const int32_t a = (int32_t)((uint32_t)m[j].ai + (uint32_t)(int32_t)__builtin_ceilf(y));
            const int32_t b =
                (int32_t)((uint32_t)m[j].ai + (uint32_t)(int32_t)__builtin_floorf(y + half_hi(m[j].cw)));
            const bool under = x[j] < ax.xmin;
            const bool in = !under && x[j] < ax.xmax;   // false for NaN
            const bool inw = (uint32_t)a < (uint32_t)A.win_len;
            const bool one = a == b;
            if (ok && in && one && inw)
                lds_add_u32(&win[(uint32_t)a >> 1], 1u << (((uint32_t)a & 1u) << 4));
            // statistics sums of in-range events
            const double xm = ok && in ? x[j] : 0.0;
            sx += xm;
            sxx = __builtin_fma(xm, xm, sxx);
            // flow events and bins outside the window: the spill path
            const bool sp = ok && (!in || (one && !inw));
            if (__builtin_amdgcn_ballot_w64(sp)) {
                if (sp) {
                    nflow += in ? 0u : 1u;
                    spill<false>(A, smem, in ? a + A.win_lo : (under ? 0 : ax.nbins + 1), 1.0);
                }
            }
            // several candidate bins: the coordinate goes to this thread's
            // list (the interval is evaluated again when it is resolved)
            if (ok && in && !one) {
                if (tcount < tcap)
                    rare[tcount * (uint32_t)nthr + tid] = x[j];
                else
                    lean_search_add(A, smem, win, x[j], a + A.win_lo, b + A.win_lo);   // list full
                ++tcount;
            }
        }
        nok += FULL ? (uint32_t)U : 0u;
        if (!FULL) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                nok += base + (uint32_t)j * nthr + tid < len ? 1u : 0u;
        }
        if (++it == A.epoch_iters) {
            it = 0;
            __syncthreads();
            drain_u16(win, (A.win_len + 1) >> 1, A.win_lo, A.cnt);
            __syncthreads();
        }
    };
    uint32_t base = 0;
    for (; base + step <= len; base += step)
        iteration(base, std::true_type{});
    for (; base < len; base += step)
        iteration(base, std::false_type{});

    // resolve the listed events: counters drained first, so the at most
    // rare_cap (<= kU16EpochEvents) increments cannot overflow them.  Eight
    // coordinates per thread at a time, their first edge reads issued
    // together.
    __syncthreads();
    drain_u16(win, (A.win_len + 1) >> 1, A.win_lo, A.cnt);
    __syncthreads();
    {
        constexpr int R = 8;
        const uint32_t mine = tcount < tcap ? tcount : tcap;
        for (uint32_t k0 = 0; k0 < mine; k0 += R) {
            double xv[R], ev[R];
            int32_t lo[R], hi[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const bool valid = k0 + j < mine;
                xv[j] = valid ? rare[(k0 + j) * (uint32_t)nthr + tid] : 0.0;
                int32_t sj;
                float zj;
                lean_seg<FEAT>(xv[j], ax, kadd, sj, zj);
                const ModelSeg mj = model[sj];
                const float y = model_eval(mj, zj);
                lo[j] = (int32_t)((uint32_t)mj.ai + (uint32_t)(int32_t)__builtin_ceilf(y)) + A.win_lo;
                hi[j] = (int32_t)((uint32_t)mj.ai + (uint32_t)(int32_t)__builtin_floorf(y + half_hi(mj.cw))) +
                        A.win_lo;
                if (!valid) {
                    lo[j] = 1;
                    hi[j] = 1;
                } else if (lo[j] > hi[j]) {   // no bound from the model: the whole axis
                    lo[j] = 1;
                    hi[j] = ax.nbins;
                }
            }
            first_step_loads<R>(ax.edges, ax.nbins, lo, hi, ev);
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (lo[j] < hi[j]) {
                    const int32_t mid = (lo[j] + hi[j] + 1) >> 1;
                    if (!(xv[j] < ev[j]))
                        lo[j] = mid;
                    else
                        hi[j] = mid - 1;
                }
            }
#pragma unroll
            for (int j = 0; j < R; ++j) {
                if (k0 + j < mine) {
                    search_one(xv[j], ax.edges, ax.nbins, lo[j], hi[j]);
                    lean_add(A, smem, win, lo[j]);
                }
            }
        }
    }

    const double nin = (double)(nok - nflow);
    double st[4] = {nin, nin, sx, sxx};
    __syncthreads();
    reduce_stats<4>(st, reinterpret_cast<double *>(smem + A.lds_red), A.stats);
    merge_window<ACC_U16>(win, A, blockIdx.x, gridDim.x);
    cache_flush<false>(A, smem);
}

bool learned_lean_supported(int dims, bool f32, bool weighted, int acc, const AxisDev *ax)
{
    return dims == 1 && !f32 && !weighted && acc == ACC_U16 && ax[0].kind == AX_LEARNED &&
           ax[0].lds_edges < 0;
}

hipError_t launch_fill_learned(int threads, int blocks, size_t lds, const FillArgs &a, hipStream_t s)
{
    const AxisDev &ax = a.ax[0];
    const int feat = ax.feature == FEAT_LINEAR ? 2 : (ax.keypos ? 0 : 1);
    const void *k = feat == 0 ? reinterpret_cast<const void *>(fill_learned_kernel<0>)
                  : feat == 1 ? reinterpret_cast<const void *>(fill_learned_kernel<1>)
                              : reinterpret_cast<const void *>(fill_learned_kernel<2>);
    allow_big_lds_ptr(k);
    if (feat == 0)
        hipLaunchKernelGGL(fill_learned_kernel<0>, dim3(blocks), dim3(threads), lds, s, a);
    else if (feat == 1)
        hipLaunchKernelGGL(fill_learned_kernel<1>, dim3(blocks), dim3(threads), lds, s, a);
    else
        hipLaunchKernelGGL(fill_learned_kernel<2>, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

}  // namespace hg
