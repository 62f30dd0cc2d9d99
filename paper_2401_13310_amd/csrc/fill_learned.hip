// fill_learned.hip -- the one-axis fill with a learned find-bin index over an
// edge array too large for LDS, unit weights, 16-bit LDS counters: the
// variable-bin fill the benchmark times (arXiv:2401.13310 Sec. 3.1 find bin,
// weight increment and statistics; Sec. 3.2 two-stage accumulation).
//
// The general fill body spends about 60 vector instructions per event here.
// This kernel is the same computation laid out for the common case, with
// few branches:
//   - the LDS window of 16-bit counters starts at LDS address 0, so a
//     counter's address is twice its bin;
//   - the learned index gives an interval of one or two bins for nearly every
//     event (three or more only for models with wide segments, a kernel
//     variant of its own).  A two-bin interval is decided by one edge: every
//     lane issues one edge read per event, from the edge array in L2/HBM for
//     a two-bin interval and of a +inf stored after the last edge otherwise,
//     so no lane branches on it.  The edge reads of a batch are issued after
//     the loads of the next batch (loads of a wave complete in issue order,
//     and the next batch is needed first in any case), then the batch's
//     counters are added once they arrive;
//   - flow events, bins outside the window and (in the wide variant) intervals
//     of three or more bins take the shared spill path (LDS hot-bin cache,
//     then global atomics) or an exact search, under a branch the wave skips
//     when none of its lanes needs it;
//   - in-range events are counted as all events less the flow events, x and
//     x^2 summed per thread.
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

// Adds v to the 16-bit window counter at LDS byte address ta (even): the
// 32-bit word at ta & ~3, shifted by 16 for the upper half.  The kernel has
// no static LDS, so the window (at offset 0 of the dynamic LDS) starts at LDS
// address 0.  The shift is the hardware's, which takes the amount modulo 32
// ((8 ta) mod 32 is 16 for the upper half, 0 for the lower).
__device__ __forceinline__ void window_add(uint32_t ta, uint32_t v)
{
    uint32_t inc;
    asm("v_lshlrev_b32 %0, %1, %2" : "=v"(inc) : "v"(ta << 3), "v"(v));
    __hip_atomic_fetch_add(reinterpret_cast<__attribute__((address_space(3))) uint32_t *>((size_t)(ta & ~3u)), inc,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
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

// Markers in place of twice a window bin (which stays far from them, the
// histogram having fewer than 2^28 bins): the event is out of range, or its
// interval holds more than two bins.  Adding 2 keeps them apart.
constexpr uint32_t kMarkOut = 0x80000000u;
constexpr uint32_t kMarkWide = 0x80000010u;

// WIDE: the index may give intervals of three or more bins (some segment's
// width is 2 or more); else every interval holds one or two.
template <int FEAT, bool WIDE>
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
    // LDS: the window at 0, then the model, the statistics partials and the
    // hot-bin cache (offsets from the host)
    uint32_t *win = reinterpret_cast<uint32_t *>(smem);
    const ModelSeg *model = reinterpret_cast<const ModelSeg *>(smem + ax.lds_model);
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
    // the edges and, after e[nbins], the +inf the lanes without a choice read
    const __amdgpu_buffer_rsrc_t eb = column_rsrc(ax.edges, (uint32_t)(ax.nbins + 2) * (uint32_t)sizeof(double));
    const uint32_t inf_off = (uint32_t)(ax.nbins + 1) * (uint32_t)sizeof(double);
    const uint32_t wlo8 = (uint32_t)A.win_lo * (uint32_t)sizeof(double);
    const uint32_t len = (uint32_t)(end > start ? end - start : 0);
    const uint32_t step = (uint32_t)nthr * U;
    // A batch's loads go through a descriptor based at the batch and sized to
    // what is left of the block's range (lanes past it read zero), so the
    // per-lane offsets stay the same from batch to batch: the descriptor is
    // advanced with scalar arithmetic and no load address is recomputed.
    const double *col = static_cast<const double *>(A.coords[0]) + start;
    uint32_t loff[U];
#pragma unroll
    for (int j = 0; j < U; ++j)
        loff[j] = ((uint32_t)j * (uint32_t)nthr + (uint32_t)tid) * (uint32_t)sizeof(double);
    double cx[U];
    auto load_at = [&](uint32_t b) {
        const uint32_t left = b < len ? (len - b) * (uint32_t)sizeof(double) : 0u;
        const __amdgpu_buffer_rsrc_t r = column_rsrc(col + b, left);
#pragma unroll
        for (int j = 0; j < U; ++j)
            cx[j] = buffer_load_nt<double>(r, loff[j]);
    };
    if (len > 0)
        load_at(0);

    double sx = 0.0, sxx = 0.0;
    uint32_t nok = 0, nflow = 0;   // events of this thread, and those out of range
    const uint32_t wlen2 = 2u * (uint32_t)A.win_len;
    int it = 0;
    // full batches need no per-event range check; the block's partial last
    // batch runs the same body with one
    auto iteration = [&](uint32_t base, auto full_t) {
        constexpr bool FULL = decltype(full_t)::value;
        double x[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            x[j] = cx[j];
        // the next batch first: loads complete in issue order, so the edge
        // reads below wait for it in any case
        load_at(base + step);
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

        // The interval [a, b] of the index.  t[j] is twice the lower bin a in
        // window coordinates (the staged model's offsets have the window
        // start subtracted), the byte address of its counter, or a marker.
        // A two-bin interval is decided by one edge, e[a] in global bins:
        // below it the event is in a, else in a + 1; the other lanes read
        // +inf and stay in a.
        uint32_t t[U];
        double e[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool ok = FULL || base + (uint32_t)j * nthr + tid < len;
            // for an in-range x, y stays within the segment's bins: the
            // conversions cannot overflow (an infinite width gives NaN or
            // infinite differences, hence the wide marker)
            const float y = model_eval(m[j], z[j]);
            const bool in = ok && !(x[j] < ax.xmin) && x[j] < ax.xmax;   // false for NaN
            uint32_t tj;
            bool two;   // the interval holds two bins
            if (WIDE) {
                const float fa = __builtin_ceilf(y);
                const float d = __builtin_floorf(y + half_hi(m[j].cw)) - fa;   // bins in the interval - 1
                tj = ((uint32_t)m[j].ai + (uint32_t)(int32_t)fa) << 1;
                t[j] = !in ? kMarkOut : d <= 1.0f ? tj : kMarkWide;
                two = d == 1.0f;
            } else {
                // widths below 2: the ends are integers near y, ceil(y) taken
                // as -floor(-y); only the lower one is converted, the two are
                // compared as floats (exact for integers of this size)
                const float na = __builtin_floorf(-y);
                const float b = __builtin_floorf(y + half_hi(m[j].cw));
                tj = ((uint32_t)m[j].ai - (uint32_t)(int32_t)na) << 1;
                t[j] = in ? tj : kMarkOut;
                two = b != -na;
            }
            const uint32_t eo = in && two ? 4u * tj + wlo8 : inf_off;
            e[j] = buffer_load_nt<double>(eb, eo);
        }
        nok += FULL ? (uint32_t)U : 0u;
        if (!FULL) {
#pragma unroll
            for (int j = 0; j < U; ++j)
                nok += base + (uint32_t)j * nthr + tid < len ? 1u : 0u;
        }

        // Each event's bin: in the window, its 16-bit counter; else the spill
        // path, which also takes flow events and searches the wide intervals.
#pragma unroll
        for (int j = 0; j < U; ++j) {
            // the statistics sums of in-range events are added under the
            // same branches as their counters
            const uint32_t b2 = t[j] + (x[j] < e[j] ? 0u : 2u);
            const bool fast = b2 < wlen2;
            if (fast) {
                window_add(b2, 1u);
                sx += x[j];
                sxx = __builtin_fma(x[j], x[j], sxx);
            } else if (FULL || base + (uint32_t)j * nthr + tid < len) {
                if ((b2 & ~31u) != kMarkOut) {        // in range, outside the window
                    spill<false>(A, smem, ((int32_t)b2 >> 1) + A.win_lo, 1.0);
                    sx += x[j];
                    sxx = __builtin_fma(x[j], x[j], sxx);
                } else if (WIDE && b2 >= kMarkWide) {   // three or more candidate bins
                    lean_search_add(A, smem, win, x[j], 1, 0);
                    sx += x[j];
                    sxx = __builtin_fma(x[j], x[j], sxx);
                } else {                                // flow
                    ++nflow;
                    spill<false>(A, smem, x[j] < ax.xmin ? 0 : ax.nbins + 1, 1.0);
                }
            }
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
           ax[0].lds_edges < 0 && ax[0].nbins < (1 << 28);
}

hipError_t launch_fill_learned(int threads, int blocks, size_t lds, bool wide, const FillArgs &a, hipStream_t s)
{
    const AxisDev &ax = a.ax[0];
    const int feat = ax.feature == FEAT_LINEAR ? 2 : (ax.keypos ? 0 : 1);
    auto go = [&](auto kernel) {
        allow_big_lds_ptr(reinterpret_cast<const void *>(kernel));
        hipLaunchKernelGGL(kernel, dim3(blocks), dim3(threads), lds, s, a);
    };
    if (wide)
        feat == 0 ? go(fill_learned_kernel<0, true>) : feat == 1 ? go(fill_learned_kernel<1, true>)
                                                                 : go(fill_learned_kernel<2, true>);
    else
        feat == 0 ? go(fill_learned_kernel<0, false>) : feat == 1 ? go(fill_learned_kernel<1, false>)
                                                                  : go(fill_learned_kernel<2, false>);
    return hipGetLastError();
}

}  // namespace hg
