// fill_body.h -- the body of a histogram fill (find bin, accumulate,
// statistics, merge) shared by the fill kernel (one range per workgroup) and
// the persistent batch kernel (one range per tile).  See fill.hip.
#pragma once

#include "device_common.h"
#include "kernels.h"

#include <type_traits>

namespace hg {

// 32-bit words of the LDS window arrays.
__device__ __forceinline__ int window_words(int acc, int win_len, int copies)
{
    if (acc == ACC_U32)
        return win_len * copies;
    if (acc == ACC_PCOUNT)
        return win_len;
    if (acc == ACC_U16)
        return (win_len + 1) >> 1;
    return win_len * copies * 4;   // F64: 2 doubles, F32C: 4 floats per bin and copy
}

// Moves the high nibble of every 16-bit counter to the global counts, so each
// counter is left <= 0x0FFF and can take kU16EpochEvents more increments.
// The window (16-byte aligned) is read four words at a time, four such reads
// per thread issued together; the rare words with a high nibble set are then
// drained one by one.
__device__ __forceinline__ void drain_word(uint32_t *win, int i, uint32_t v, int32_t win_lo, uint64_t *cnt)
{
    const uint32_t m = v & 0xF000F000u;
    if (m) {
        win[i] = v - m;
        const int64_t g0 = (int64_t)win_lo + 2 * (int64_t)i;
        if (m & 0xFFFFu)
            gl_add_u64(&cnt[g0], m & 0xFFFFu);
        if (m >> 16)
            gl_add_u64(&cnt[g0 + 1], m >> 16);
    }
}

__device__ __forceinline__ void drain_u16(uint32_t *win, int words, int32_t win_lo, uint64_t *cnt)
{
    int done = 0;
    if ((reinterpret_cast<uintptr_t>(win) & 15u) == 0) {
        const int quads = words >> 2;
        const uint4 *w4 = reinterpret_cast<const uint4 *>(win);
        constexpr int R = 4;
        for (int q0 = threadIdx.x; q0 < quads; q0 += R * blockDim.x) {
            uint4 v[R];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const int q = q0 + k * (int)blockDim.x;
                v[k] = q < quads ? w4[q] : make_uint4(0u, 0u, 0u, 0u);
            }
            uint32_t any = 0;
#pragma unroll
            for (int k = 0; k < R; ++k)
                any |= v[k].x | v[k].y | v[k].z | v[k].w;
            if (any & 0xF000F000u) {
#pragma unroll
                for (int k = 0; k < R; ++k) {
                    const int q = q0 + k * (int)blockDim.x;
                    if (q < quads) {
                        drain_word(win, 4 * q, v[k].x, win_lo, cnt);
                        drain_word(win, 4 * q + 1, v[k].y, win_lo, cnt);
                        drain_word(win, 4 * q + 2, v[k].z, win_lo, cnt);
                        drain_word(win, 4 * q + 3, v[k].w, win_lo, cnt);
                    }
                }
            }
        }
        done = 4 * quads;
    }
    for (int i = done + (int)threadIdx.x; i < words; i += blockDim.x)
        drain_word(win, i, win[i], win_lo, cnt);
}

// LDS window -> global histogram (atomics) or -> staging slot `col`; for
// PCOUNT, column `col` of the `cols`-column bucket-major count table.
template <int ACC>
__device__ __forceinline__ void merge_window(uint32_t *win, const FillArgs &A, int col, int cols)
{
    const int W = A.win_len;
    const int C = A.copies;
    if (ACC == ACC_PCOUNT) {
        for (int j = threadIdx.x; j < W; j += blockDim.x) {
            const uint32_t c = win[j];
            A.part_table[(int64_t)j * cols + col] = c;
            if (c)
                __hip_atomic_fetch_add(&A.part_totals[j], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else if (ACC == ACC_U32) {
        if (A.merge == MERGE_STAGE) {
            uint32_t *st = static_cast<uint32_t *>(A.stage) + (int64_t)col * A.stage_stride;
            for (int l = threadIdx.x; l < W; l += blockDim.x) {
                uint32_t c = 0;
                for (int r = 0; r < C; ++r)
                    c += win[l * C + r];
                st[l] = c;
            }
        } else {
            for (int l = threadIdx.x; l < W; l += blockDim.x) {
                uint32_t c = 0;
                for (int r = 0; r < C; ++r)
                    c += win[l * C + r];
                if (c)
                    gl_add_u64(&A.cnt[A.win_lo + l], c);
            }
        }
    } else if (ACC == ACC_U16) {
        const int words = (W + 1) >> 1;
        if (A.merge == MERGE_STAGE) {
            // the slot holds one byte per bin, bin 4i + k in byte k of word i;
            // a counter above 255 stages 255 and adds the rest to the
            // histogram itself (the bins past the window stage zeros)
            uint32_t *st = static_cast<uint32_t *>(A.stage) + (int64_t)col * A.stage_stride;
            const int swords = (W + 3) >> 2;
            for (int i = threadIdx.x; i < swords; i += blockDim.x) {
                const uint32_t v0 = win[2 * i];
                const uint32_t v1 = 2 * i + 1 < words ? win[2 * i + 1] : 0u;
                uint32_t c[4] = {v0 & 0xFFFFu, v0 >> 16, v1 & 0xFFFFu, v1 >> 16};
                if ((v0 | v1) & 0xFF00FF00u) {
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        if (c[k] > 255u) {
                            gl_add_u64(&A.cnt[A.win_lo + 4 * (int64_t)i + k], c[k] - 255u);
                            c[k] = 255u;
                        }
                }
                st[i] = c[0] | (c[1] << 8) | (c[2] << 16) | (c[3] << 24);
            }
        } else {
            for (int i = threadIdx.x; i < words; i += blockDim.x) {
                const uint32_t v = win[i];
                const int64_t g0 = (int64_t)A.win_lo + 2 * (int64_t)i;
                if (v & 0xFFFFu)
                    gl_add_u64(&A.cnt[g0], v & 0xFFFFu);
                if (v >> 16)
                    gl_add_u64(&A.cnt[g0 + 1], v >> 16);
            }
        }
    } else {
        // F64: [sumw][sumw2] each W*C doubles; F32C: [(sw, cw)][(sw2, cw2)] each
        // W*C pairs of floats (sum in the low word, compensation in the high)
        const int n1 = W * C;
        for (int l = threadIdx.x; l < W; l += blockDim.x) {
            double s = 0.0, s2 = 0.0;
            if (ACC == ACC_F64) {
                const double *d = reinterpret_cast<const double *>(win);
                for (int r = 0; r < C; ++r) {
                    s += d[l * C + r];
                    s2 += d[n1 + l * C + r];
                }
            } else {
                const uint64_t *q = reinterpret_cast<const uint64_t *>(win);
                for (int r = 0; r < C; ++r) {
                    const uint64_t a = q[l * C + r], b = q[n1 + l * C + r];
                    s += (double)__uint_as_float((uint32_t)a) + (double)__uint_as_float((uint32_t)(a >> 32));
                    s2 += (double)__uint_as_float((uint32_t)b) + (double)__uint_as_float((uint32_t)(b >> 32));
                }
            }
            if (A.merge == MERGE_STAGE) {
                double *st = static_cast<double *>(A.stage) + (int64_t)col * 2 * A.stage_stride;
                st[l] = s;
                st[A.stage_stride + l] = s2;
            } else if (s != 0.0 || s2 != 0.0) {
                gl_add_f64(&A.sumw[A.win_lo + l], s);
                gl_add_f64(&A.sumw2[A.win_lo + l], s2);
            }
        }
    }
}

// Update of a bin outside the LDS window: first a small LDS cache of hot
// bins (flow bins, spikes), open addressing with one probe, slots claimed
// with compare-and-swap; otherwise a global atomic.  Many workgroups hitting
// one global address serialize in L2, so a hot bin outside the window would
// otherwise cost far more than its share.
template <bool W>
__device__ __forceinline__ void spill(const FillArgs &A, char *smem, int32_t g, double w)
{
    // keeps the global update inside the histogram whatever the bin
    g = __builtin_elementwise_min(__builtin_elementwise_max(g, 0), A.total_bins - 1);
    if (A.lds_cache >= 0) {
        uint32_t *keys = reinterpret_cast<uint32_t *>(smem + A.lds_cache);
        const uint32_t h = ((uint32_t)g * 2654435761u) >> 16 & (uint32_t)(A.cache_slots - 1);
        uint32_t k = keys[h];
        if (k == kCacheEmpty) {
            uint32_t expected = kCacheEmpty;
            __hip_atomic_compare_exchange_strong(&keys[h], &expected, (uint32_t)g, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            k = expected == kCacheEmpty ? (uint32_t)g : expected;
        }
        if (k == (uint32_t)g) {
            if (W) {
                double *v = reinterpret_cast<double *>(keys + A.cache_slots);
                lds_add_f64(&v[2 * h], w);
                lds_add_f64(&v[2 * h + 1], w * w);
            } else {
                lds_add_u32(&keys[A.cache_slots + h], 1u);
            }
            return;
        }
    }
    if (W) {
        gl_add_f64(&A.sumw[g], w);
        gl_add_f64(&A.sumw2[g], w * w);
    } else {
        gl_add_u64(&A.cnt[g], 1ull);
    }
}

template <bool W>
__device__ __forceinline__ void cache_init(const FillArgs &A, char *smem)
{
    if (A.lds_cache < 0)
        return;
    uint32_t *keys = reinterpret_cast<uint32_t *>(smem + A.lds_cache);
    const int vwords = A.cache_slots * (W ? 4 : 1);
    for (int i = threadIdx.x; i < A.cache_slots; i += blockDim.x)
        keys[i] = kCacheEmpty;
    for (int i = threadIdx.x; i < vwords; i += blockDim.x)
        keys[A.cache_slots + i] = 0u;
}

template <bool W>
__device__ __forceinline__ void cache_flush(const FillArgs &A, char *smem)
{
    if (A.lds_cache < 0)
        return;
    const uint32_t *keys = reinterpret_cast<const uint32_t *>(smem + A.lds_cache);
    for (int i = threadIdx.x; i < A.cache_slots; i += blockDim.x) {
        const uint32_t k = keys[i];
        if (k == kCacheEmpty)
            continue;
        if (W) {
            const double *v = reinterpret_cast<const double *>(keys + A.cache_slots);
            gl_add_f64(&A.sumw[k], v[2 * i]);
            gl_add_f64(&A.sumw2[k], v[2 * i + 1]);
        } else {
            gl_add_u64(&A.cnt[k], keys[A.cache_slots + i]);
        }
    }
}

// Coalesced streaming loads of U events per thread: event base + j*blockDim +
// tid of the block's range, through buffer descriptors over the block's
// columns.  A descriptor covers exactly the block's len events, so loads past
// the end return 0 without touching memory (process_batch skips those
// events); every load is issued unconditionally, so the waits for loads issued
// before these stay exact.  Non-temporal, so the event stream does not evict
// edges and models.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t column_rsrc(const void *p, uint32_t bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T>
__device__ __forceinline__ T buffer_load_nt(__amdgpu_buffer_rsrc_t r, uint32_t off)
{
    constexpr int kNonTemporal = 2;
    if constexpr (sizeof(T) == 8)
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, kNonTemporal));
    else
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, kNonTemporal));
}

template <int D, typename T, bool W, int U>
__device__ __forceinline__ void load_batch(const __amdgpu_buffer_rsrc_t (&rx)[D],
                                           __amdgpu_buffer_rsrc_t rw, uint32_t base,
                                           T (&x)[U][D], T (&w)[U])
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const uint32_t off = (base + (uint32_t)j * blockDim.x + threadIdx.x) * (uint32_t)sizeof(T);
#pragma unroll
        for (int a = 0; a < D; ++a)
            x[j][a] = buffer_load_nt<T>(rx[a], off);
        w[j] = W ? buffer_load_nt<T>(rw, off) : T(0);
    }
}

// Find bin, statistics and accumulation for the U loaded events of a thread
// (events at offsets >= len are skipped; FULL: none is).  `prefetch` issues the loads of the
// next batch: first thing when no search reads HBM, else once the searches are
// done, so that they never wait for the next batch.  Unit weights count their in-range events in
// `nin` (the w and w^2 statistics) instead of adding 1.0 twice.  Events
// outside the LDS window are handled after the batch's LDS adds, in a branch
// the wave skips when none of its lanes has one.
template <int D, typename T, int ACC, bool W, int U, int KS, bool FULL, bool ST, typename Prefetch>
__device__ __forceinline__ void process_batch(const FillArgs &A, char *smem, uint32_t *win,
                                              const T (&cx)[U][D], const T (&cw)[U],
                                              uint32_t base, uint32_t len, int cp,
                                              double (&st)[NStats<D>::v], uint32_t &nin,
                                              int32_t *gb, Prefetch &&prefetch)
{
    constexpr int KIND = kind_of_set<KS>();
    constexpr bool early = KIND == AX_UNIFORM || KS == KS_STAGED;
    constexpr int ES = (KS == KS_LEARNED1 || KS == KS_BSEARCH1) ? EDGES_HBM : EDGES_ANY;
    // Loads complete in issue order, so the next batch is requested where no
    // later wait is for a load issued before it: first when every search
    // reads LDS (or there is none), else after the searches, whose HBM edge
    // loads would otherwise wait for it.  The scheduling barriers keep the
    // loads where they are written.
    if (early) {
        prefetch();
        __builtin_amdgcn_sched_barrier(0);
    }
    const uint32_t wlen = (uint32_t)A.win_len;
    double x[D][U];
    int32_t b[D][U];
    bool inr[D][U];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int j = 0; j < U; ++j)
            x[a][j] = (double)cx[j][a];
    if constexpr (KS == KS_STAGED) {
#pragma unroll
        for (int a = 0; a < D; ++a)
            axis_bins_staged<U, (D > 1)>(x[a], A.ax[a], smem, b[a], inr[a]);
    } else {
        int32_t lo[D][U], hi[D][U];
        double ev[D][U];
#pragma unroll
        for (int a = 0; a < D; ++a)
            axis_bins_begin<U, KIND, ES>(x[a], A.ax[a], smem, lo[a], hi[a], ev[a], inr[a]);
#pragma unroll
        for (int a = 0; a < D; ++a)
            axis_bins_finish<U, KIND, ES>(x[a], A.ax[a], smem, lo[a], hi[a], ev[a], b[a]);
        if (!early) {
            __builtin_amdgcn_sched_barrier(0);
            prefetch();
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    float wfv[U], w2v[U], e2v[U];
    uint32_t fidx[U];
    bool fin[U];
    int32_t gv[U];
    bool out[U];
    bool any_out = false;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        fin[j] = false;
        const bool ok = FULL || base + (uint32_t)j * blockDim.x + threadIdx.x < len;
        int32_t g = 0;
        bool inside = true;
        double xe[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xe[a] = x[a][j];
            inside = inside && inr[a][j];
            g += (a == 0) ? b[a][j] : b[a][j] * A.ax[a].stride;
        }
        gv[j] = g;
        const double w = W ? (double)cw[j] : 1.0;
        // statistics of in-range events: excluded events add exact zeros
        // (their coordinates and weight are masked, so no inf or NaN enters)
        const bool take = ok && inside;
        if (ST) {
            double xm[D];
#pragma unroll
            for (int a = 0; a < D; ++a)
                xm[a] = take ? xe[a] : 0.0;
            if (W) {
                stats_add<D>(st, xm, take ? w : 0.0);
            } else {
                stats_add_unit<D>(st, xm);
                nin += take ? 1u : 0u;
            }
        }
        const uint32_t l = (uint32_t)(g - A.win_lo);
        const bool inw = l < wlen;
        out[j] = ACC != ACC_PCOUNT && ok && !inw;
        any_out = any_out || out[j];
        if (ACC == ACC_PCOUNT) {
            if (ok) {
                gb[base + (uint32_t)j * blockDim.x + threadIdx.x] = g;
                lds_add_u32(&win[(uint32_t)g >> A.part_shift], 1u);
            }
        } else if (ok && inw) {
            if (ACC == ACC_U32) {
                lds_add_u32(&win[__umul24(l, (uint32_t)A.copies) + cp], 1u);
            } else if (ACC == ACC_U16) {
                lds_add_u32(&win[l >> 1], 1u << ((l & 1u) << 4));
            } else if (ACC == ACC_F64) {
                double *s = reinterpret_cast<double *>(win);
                const uint32_t idx = __umul24(l, (uint32_t)A.copies) + cp;
                lds_add_f64(&s[idx], w);
                lds_add_f64(&s[wlen * A.copies + idx], w * w);
            } else {
                const float wf = (float)cw[j];
                const float w2 = wf * wf;
                wfv[j] = wf;
                w2v[j] = w2;
                e2v[j] = __builtin_fmaf(wf, wf, -w2);   // exact: wf*wf = w2 + e2
                fidx[j] = __umul24(l, (uint32_t)A.copies) + cp;
                fin[j] = true;
            }
        }
    }
    if (ACC == ACC_F32C) {
        // each (sum, compensation) pair is updated as one 64-bit word: the
        // reads of the whole batch are issued first, then one compare-and-swap
        // per pair, repeated only when another lane changed the pair in between
        uint64_t *q = reinterpret_cast<uint64_t *>(win);
        const uint32_t n1 = wlen * A.copies;
        uint64_t old1[U], old2[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (fin[j]) {
                old1[j] = q[fidx[j]];
                old2[j] = q[n1 + fidx[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (fin[j]) {
                lds_add_compensated(&q[fidx[j]], old1[j], wfv[j], 0.0f);
                lds_add_compensated(&q[n1 + fidx[j]], old2[j], w2v[j], e2v[j]);
            }
        }
    }
    if (any_out) {
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (out[j])
                spill<W>(A, smem, gv[j], W ? (double)cw[j] : 1.0);
    }
}

// The whole fill of the events [start, end) of A by one workgroup: stage the
// learned models, zero the LDS window, the pipelined loop over the events,
// then the statistics and the merge of the window (into staging slot or
// count-table column `col` of `cols`).  The fill kernel runs it once per
// block; the batch kernel once per tile.  ST false leaves the statistics to
// separate reduction kernels (the launch-shape study).
template <int D, typename T, int ACC, bool W, int U, int KS, bool ST = true>
__device__ __forceinline__ void fill_range(const FillArgs &A, char *smem, int64_t start, int64_t end,
                                           int col, int cols)
{
    constexpr int NS = NStats<D>::v;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;

    // the fill's entry count, once per fill (the range that starts at event 0)
    if (start == 0 && tid == 0 && A.entries)
        gl_add_u64(A.entries, (uint64_t)A.n);
    stage_axes<D>(A.ax, smem);
    uint32_t *win = reinterpret_cast<uint32_t *>(smem + A.lds_win);
    const int words = window_words(ACC, A.win_len, A.copies);
    for (int i = tid; i < words; i += nthr)
        win[i] = 0u;
    cache_init<W>(A, smem);
    __syncthreads();

    double st[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        st[k] = 0.0;
    uint32_t nin = 0;   // unit weights: in-range events (w and w^2 statistics)

    const int cp = (ACC == ACC_U16) ? 0 : tid % A.copies;
    int it = 0;

    // Software pipeline: the loads of the next U events per thread are in
    // flight while the current ones are binned and accumulated (the last
    // iteration reloads the block's last event, unused).
    const uint32_t len = (uint32_t)(end > start ? end - start : 0);
    const uint32_t step = (uint32_t)nthr * U;
    // the plan keeps a block's range under 2^32 bytes
    const uint32_t bytes = len * (uint32_t)sizeof(T);
    __amdgpu_buffer_rsrc_t xb[D];
#pragma unroll
    for (int a = 0; a < D; ++a)
        xb[a] = column_rsrc(static_cast<const T *>(A.coords[a]) + start, bytes);
    const __amdgpu_buffer_rsrc_t wb =
        column_rsrc(W ? static_cast<const T *>(A.w) + start : static_cast<const T *>(A.coords[0]), W ? bytes : 0u);
    int32_t *gb = ACC == ACC_PCOUNT ? A.gbins + start : nullptr;
    T cx[U][D], cw[U];
    if (len > 0)
        load_batch<D, T, W, U>(xb, wb, 0, cx, cw);
    // full batches first, with no per-event range check, then the block's
    // partial last batch (if any) in a loop of its own
    auto iteration = [&](uint32_t base, auto full) {
        T nx[U][D], nw[U];
        process_batch<D, T, ACC, W, U, KS, decltype(full)::value, ST>(
            A, smem, win, cx, cw, base, len, cp, st, nin, gb,
            [&] { load_batch<D, T, W, U>(xb, wb, base + step, nx, nw); });
        if (ACC == ACC_U16 && ++it == A.epoch_iters) {
            it = 0;
            __syncthreads();
            drain_u16(win, words, A.win_lo, A.cnt);
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
#pragma unroll
            for (int a = 0; a < D; ++a)
                cx[j][a] = nx[j][a];
            cw[j] = nw[j];
        }
    };
    uint32_t base = 0;
    for (; base + step <= len; base += step)
        iteration(base, std::true_type{});
    for (; base < len; base += step)
        iteration(base, std::false_type{});
    if (!W) {
        st[0] = (double)nin;
        st[1] = (double)nin;
    }
    __syncthreads();
    if (ST)
        reduce_stats<NS>(st, reinterpret_cast<double *>(smem), A.stats);
    merge_window<ACC>(win, A, col, cols);
    cache_flush<W>(A, smem);
}

}  // namespace hg
