// plan.hip -- choosing how a fill is launched, and the autotuner.
//
// A plan fixes the accumulation strategy (LDS window, global atomics, or bin
// tiles), the LDS accumulator, the number of workgroups and LDS copies, the
// window of bins held in LDS and the merge.  The heuristic picks from the
// histogram shape and the gfx950 LDS budget; hist_tune replaces it with the
// fastest candidate measured on a sample (the launch-shape sensitivity the
// paper reports for its reductions in Sec. 4.3 is why the shape is measured
// rather than fixed).
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <tuple>
#include <vector>

namespace hg {

int unroll_of(const hist_s *h, bool f32, bool weighted, int acc)
{
    return fill_unroll(h->dims, f32, weighted, acc, kind_set(h->dims, h->ax));
}

int lds_axis_layout(int dims, AxisDev *ax, int off)
{
    const uint32_t staged = staged_edges_mask(dims, ax);
    for (int d = 0; d < dims; ++d) {
        if (ax[d].kind == AX_LEARNED) {
            ax[d].lds_model = off;
            off += ax[d].nseg * (int)sizeof(ModelSeg);
            off = (off + 15) & ~15;
        } else {
            ax[d].lds_model = -1;
        }
        if (staged & (1u << d)) {
            ax[d].lds_edges = off;
            off = (off + (ax[d].nbins + 1) * (int)sizeof(double) + 15) & ~15;
        } else {
            ax[d].lds_edges = -1;
        }
    }
    return off;
}

int apply_model_offsets(const hist_s *h, FillArgs &a)
{
    return lds_axis_layout(h->dims, a.ax, kRedBytes);
}

size_t stage_bytes_for(const Plan &p)
{
    return (size_t)p.blocks * (size_t)stage_stride_for(p) *
           (p.acc == ACC_U32 || p.acc == ACC_U16 ? 4 : 16);
}

int64_t stage_stride_for(const Plan &p)
{
    return stage_stride_of(p.acc, p.win_len);
}

int64_t stage_stride_of(int acc, int64_t win_len)
{
    if (acc == ACC_U16)   // one byte per bin, slots in whole 128-byte lines
        return ((win_len + 3) / 4 + 31) / 32 * 32;
    return win_len;
}

int64_t tiled_chunk(const hist_s *h)
{
    (void)h;
    return (int64_t)1 << 24;
}

int64_t part_chunk(const hist_s *h)
{
    (void)h;
    return (int64_t)1 << 25;
}

// Bucket widths 2^b a PART plan can use: the bucket's bins must fit LDS in the
// accumulate pass (4 or 16 bytes a bin), its offsets 16 bits (b <= 16), and the
// per-bucket counters of the count and scatter passes must fit LDS after the
// statistics and models.
void part_bits_range(const hist_s *h, bool weighted, int lds_base, int &lo, int &hi)
{
    const int per_bin = weighted ? 16 : 4;
    hi = 0;
    while (hi < 16 && ((int64_t)per_bin << (hi + 1)) <= h->lds_max)
        ++hi;
    const int64_t max_buckets = (h->lds_max - lds_base) / 4;
    lo = 6;
    while (lo <= hi && ((h->T + ((int64_t)1 << lo) - 1) >> lo) > max_buckets)
        ++lo;
}

static int window_bytes(int acc, int64_t len, int copies)
{
    if (acc == ACC_U16)
        return (int)(((len + 1) / 2) * 4);
    return (int)(len * copies * acc_bytes(acc));
}

Plan plan_from_choice(const hist_s *h, int64_t n, hist_dtype dtype, bool weighted,
                      const PlanChoice &c)
{
    Plan p;
    const bool f32 = dtype == HIST_F32;
    FillArgs probe;
    std::memset(&probe, 0, sizeof(probe));
    for (int d = 0; d < kMaxDims; ++d)
        probe.ax[d] = h->ax[d];
    const int base = apply_model_offsets(h, probe);
    const int avail = h->lds_max - base;
    p.lds_base = base;
    p.threads = c.threads > 0 ? c.threads : 1024;

    int acc;
    if (weighted)
        acc = (f32 && (h->flags & HIST_F_ACC_F32C)) ? ACC_F32C : ACC_F64;
    else
        acc = (h->T * 4 <= avail) ? ACC_U32 : ACC_U16;
    const int64_t cap = acc == ACC_U16 ? (int64_t)(avail / 4) * 2 : avail / acc_bytes(acc);

    int plo = 0, phi = -1;
    part_bits_range(h, weighted, base, plo, phi);
    int strategy = c.strategy;
    if (strategy == HIST_STRAT_AUTO) {
        if (h->T <= cap) {
            strategy = HIST_STRAT_LDS;
        } else if (2 * cap >= h->T) {
            strategy = HIST_STRAT_LDS;   // a window over most bins, the rest global
        } else {
            const int64_t tiles = (h->T + cap - 1) / cap;
            strategy = tiles <= 2 ? HIST_STRAT_TILED
                                  : (plo <= phi ? HIST_STRAT_PART : HIST_STRAT_GLOBAL);
        }
    }
    if (strategy == HIST_STRAT_PART && plo > phi)
        strategy = HIST_STRAT_GLOBAL;   // too many bins to partition by LDS-sized ranges
    p.strategy = strategy;

    if (strategy == HIST_STRAT_PART) {
        p.acc = weighted ? ACC_F64 : ACC_U32;
        // about one accumulate chunk of events per bucket: fewer, wider buckets
        // would merge several chunks with atomics over wide bin ranges, more,
        // narrower ones would scatter the events into shorter runs
        int b = c.bucket_bits;
        if (b <= 0) {
            const double per_chunk = (double)h->T * (double)kPartChunk / (double)std::max<int64_t>(n, 1);
            b = (int)std::ceil(std::log2(std::max(per_chunk, 2.0)));
        }
        b = std::min(std::max(b, plo), phi);
        p.bucket_bits = b;
        p.win_len = 1 << b;
        p.copies = 1;
        p.merge = MERGE_ATOMIC;
        const int64_t nb = (h->T + p.win_len - 1) >> b;
        p.lds = base + (int)(nb * 4);
        p.blocks = c.blocks > 0 ? c.blocks : h->num_cu * 2;
        return p;
    }

    if (strategy == HIST_STRAT_GLOBAL) {
        p.acc = weighted ? ACC_F64 : ACC_U32;
        p.win_len = 0;
        p.copies = 1;
        p.merge = MERGE_ATOMIC;
        p.lds = base;
    } else if (strategy == HIST_STRAT_TILED) {
        p.acc = weighted ? ACC_F64 : (h->T * 4 <= avail ? ACC_U32 : ACC_U16);
        const int64_t tcap = p.acc == ACC_U16 ? (int64_t)(avail / 4) * 2 : avail / acc_bytes(p.acc);
        p.win_len = (int32_t)std::min<int64_t>(tcap, h->T);
        p.copies = 1;
        p.merge = MERGE_ATOMIC;
        p.lds = base + window_bytes(p.acc, p.win_len, 1);
        p.epoch_iters = std::max(1, kU16EpochEvents / (p.threads * kTileUnroll));
        const int64_t tiles = (h->T + p.win_len - 1) / p.win_len;
        int bx = (int)std::max<int64_t>(1, (int64_t)h->num_cu * 2 / tiles);
        if (c.blocks > 0)
            bx = c.blocks;
        p.blocks = bx;
        return p;
    } else {
        p.acc = acc;
        int64_t lo = 0, len = h->T;
        if (h->T > cap) {
            // events outside the window: keep a small LDS cache of hot bins
            constexpr int kSlots = 256;
            p.lds_cache = base;
            p.cache_slots = kSlots;
            p.lds_base = (base + cache_bytes(kSlots, weighted) + 15) & ~15;
            const int avail2 = h->lds_max - p.lds_base;
            const int64_t cap2 = acc == ACC_U16 ? (int64_t)(avail2 / 4) * 2 : avail2 / acc_bytes(acc);
            len = cap2;
            lo = c.win_lo >= 0 ? c.win_lo : 0;
            if (lo + len > h->T)
                lo = h->T - len;
        }
        p.win_lo = (int32_t)lo;
        p.win_len = (int32_t)len;
        int copies = 1;
        if (acc != ACC_U16) {
            if (c.copies > 0) {
                copies = c.copies;
            } else {
                const int64_t fit = avail / std::max<int64_t>(1, len * acc_bytes(acc));
                // every copy is zeroed and merged once per workgroup: keep at
                // least about 4 events per bin and copy (at two workgroups
                // per CU), or a small fill spends its time on the copies
                const int64_t per_wg = n / std::max<int64_t>(1, (int64_t)h->num_cu * 2);
                const int64_t useful = std::max<int64_t>(1, per_wg / std::max<int64_t>(1, 4 * len));
                copies = (int)std::min<int64_t>(std::min<int64_t>(64, fit), std::max<int64_t>(1, useful));
            }
            while (copies > 1 && window_bytes(acc, len, copies) > h->lds_max - p.lds_base)
                --copies;
        }
        p.copies = copies;
        p.lds = p.lds_base + window_bytes(acc, len, copies);
    }

    int U = unroll_of(h, f32, weighted, p.acc);
    if ((c.unroll > 0 || c.stats_ept > 0) &&
        (p.strategy == HIST_STRAT_LDS || p.strategy == HIST_STRAT_GLOBAL)) {
        const int ks = kind_set(h->dims, h->ax);
        int u = c.unroll;
        if (u <= 0)   // separate statistics at the heuristic count (or the next variant below)
            for (u = 8; u > 1 && u > U; u >>= 1) {
            }
        if (fill_shape_supported(h->dims, f32, p.acc, weighted, ks, u)) {
            U = u;
            p.shape = true;
            p.stats_ept = c.stats_ept;
        }
    }
    p.unroll = U;
    const int64_t step = (int64_t)p.threads * U;
    int bpc = c.blocks_per_cu > 0 ? c.blocks_per_cu : (p.lds > h->lds_max / 2 ? 1 : 2);
    if (p.lds * bpc > h->lds_max)
        bpc = std::max(1, h->lds_max / std::max(1, p.lds));
    int64_t G = c.blocks > 0 ? c.blocks : (int64_t)h->num_cu * bpc;
    const int64_t need = (n + step - 1) / step;
    if (G > need)
        G = need;
    // a block addresses its events with 32-bit byte offsets
    constexpr int64_t kMaxBlockEvents = (int64_t)1 << 28;
    if (G < (n + kMaxBlockEvents - 1) / kMaxBlockEvents)
        G = (n + kMaxBlockEvents - 1) / kMaxBlockEvents;
    if (G < 1)
        G = 1;
    int64_t per = (n + G - 1) / G;
    per = (per + step - 1) / step * step;
    G = (n + per - 1) / per;
    if (G < 1)
        G = 1;
    p.blocks = (int)G;
    p.per_block = per;
    p.epoch_iters = std::max(1, kU16EpochEvents / (int)step);
    if (p.strategy == HIST_STRAT_LDS) {
        if (c.merge >= 0)
            p.merge = c.merge;
        else
            p.merge = (double)G * window_bytes(p.acc, p.win_len, 1) > 8.0e6 ? MERGE_STAGE
                                                                             : MERGE_ATOMIC;
    }
    return p;
}

// ------------------------------------------------------- tuned-plan cache --

namespace {
struct ShapeKey {
    int dims;
    int64_t T;
    int kinds;
    int weighted, f32;
    uint32_t flags;
    bool operator<(const ShapeKey &o) const
    {
        return std::tie(dims, T, kinds, weighted, f32, flags) <
               std::tie(o.dims, o.T, o.kinds, o.weighted, o.f32, o.flags);
    }
};
std::mutex g_cache_mu;
std::map<ShapeKey, PlanChoice> g_cache;

ShapeKey shape_key(const hist_s *h, bool weighted, bool f32)
{
    int kinds = 0;
    for (int d = 0; d < h->dims; ++d)
        kinds = kinds * 3 + h->ax[d].kind;
    return ShapeKey{h->dims, h->T, kinds, weighted ? 1 : 0, f32 ? 1 : 0, h->flags};
}
}  // namespace

bool tuned_choice(const hist_s *h, bool weighted, bool f32, PlanChoice &out)
{
    auto it = h->tuned.find(std::make_tuple(weighted ? 1 : 0, f32 ? 1 : 0, 0));
    if (it != h->tuned.end()) {
        out = it->second;
        return true;
    }
    std::lock_guard<std::mutex> lock(g_cache_mu);
    auto jt = g_cache.find(shape_key(h, weighted, f32));
    if (jt == g_cache.end())
        return false;
    out = jt->second;
    return true;
}

Plan make_plan(const hist_s *h, int64_t n, hist_dtype dtype, bool weighted)
{
    PlanChoice c = h->forced;
    if (c.strategy == HIST_STRAT_AUTO) {
        auto it = h->tuned.find(std::make_tuple(weighted ? 1 : 0, dtype == HIST_F32 ? 1 : 0, 0));
        if (it != h->tuned.end()) {
            c = it->second;
        } else {
            std::lock_guard<std::mutex> lock(g_cache_mu);
            auto jt = g_cache.find(shape_key(h, weighted, dtype == HIST_F32));
            if (jt != g_cache.end())
                c = jt->second;
        }
        // a shape fixed by hist_set_shape or hist_set_threads applies over
        // a tuned choice
        if (h->forced.threads > 0)
            c.threads = h->forced.threads;
        if (h->forced.unroll > 0)
            c.unroll = h->forced.unroll;
        if (h->forced.stats_ept > 0)
            c.stats_ept = h->forced.stats_ept;
    }
    return plan_from_choice(h, n, dtype, weighted, c);
}

}  // namespace hg

using namespace hg;

extern "C" hist_status hist_set_strategy(hist_t *h, int strategy, int blocks, int subhists)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_set_strategy: NULL handle");
    if (strategy < HIST_STRAT_AUTO || strategy > HIST_STRAT_PART)
        return set_error(HIST_EINVAL, "hist_set_strategy: unknown strategy %d", strategy);
    if (blocks < 0 || subhists < 0 || subhists > 64)
        return set_error(HIST_EINVAL, "hist_set_strategy: blocks >= 0, 0 <= subhists <= 64");
    PlanChoice c;
    c.strategy = strategy;
    c.blocks = blocks;
    c.copies = subhists;
    c.merge = h->forced.merge;
    c.win_lo = h->forced.win_lo;
    c.threads = h->forced.threads;
    c.bucket_bits = h->forced.bucket_bits;
    c.unroll = h->forced.unroll;
    c.stats_ept = h->forced.stats_ept;
    h->forced = c;
    return HIST_OK;
}

extern "C" hist_status hist_set_shape(hist_t *h, int unroll, int stats_ept)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_set_shape: NULL handle");
    if (unroll != 0 && unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8)
        return set_error(HIST_EINVAL, "hist_set_shape: unroll must be 0, 1, 2, 4 or 8");
    if (stats_ept != 0 && stats_ept != 1 && stats_ept != 4 && stats_ept != 16)
        return set_error(HIST_EINVAL, "hist_set_shape: stats_ept must be 0, 1, 4 or 16");
    h->forced.unroll = unroll;
    h->forced.stats_ept = stats_ept;
    return HIST_OK;
}

extern "C" hist_status hist_plan_shape(hist_t *h, int64_t n, hist_dtype dtype, int weighted,
                                       int *unroll, int *stats_ept, int *threads)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_plan_shape: NULL handle");
    const Plan p = make_plan(h, n < 1 ? 1 : n, dtype, weighted != 0);
    if (unroll)
        *unroll = p.unroll;
    if (stats_ept)
        *stats_ept = p.stats_ept;
    if (threads)
        *threads = p.threads;
    return HIST_OK;
}

extern "C" hist_status hist_set_threads(hist_t *h, int threads)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_set_threads: NULL handle");
    if (threads != 0 && threads != 256 && threads != 512 && threads != 1024)
        return set_error(HIST_EINVAL, "hist_set_threads: 0, 256, 512 or 1024");
    h->forced.threads = threads;
    return HIST_OK;
}

extern "C" hist_status hist_plan_info(hist_t *h, int64_t n, hist_dtype dtype, int weighted,
                                      int *strategy, int *blocks, int *subhists,
                                      int64_t *window_lo, int64_t *window_len, int *accumulator)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_plan_info: NULL handle");
    if (n < 1)
        n = 1;
    Plan p = make_plan(h, n, dtype, weighted != 0);
    if (strategy)
        *strategy = p.strategy;
    if (blocks)
        *blocks = p.blocks;
    if (subhists)
        *subhists = p.copies;
    if (window_lo)
        *window_lo = p.win_lo;
    if (window_len)
        *window_len = p.win_len;
    if (accumulator)
        *accumulator = p.acc;
    return HIST_OK;
}

// Extra control used by tests and the benchmark: merge mode (-1 auto) and LDS
// window start (-1 auto) for later fills.
extern "C" hist_status hist_set_window(hist_t *h, int64_t window_lo, int merge)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_set_window: NULL handle");
    if (window_lo < -1 || window_lo >= h->T || merge < -1 || merge > MERGE_STAGE)
        return set_error(HIST_EINVAL, "hist_set_window: bad window or merge");
    h->forced.win_lo = window_lo;
    h->forced.merge = merge;
    return HIST_OK;
}

// ------------------------------------------------------------- autotuner --

namespace {

// The histogram's device state: counts, sums, and the statistics with the
// entry count behind them (kMaxStats + 2 words).
struct Saved {
    uint64_t *cnt = nullptr;
    double *sumw = nullptr, *sumw2 = nullptr, *stats = nullptr;
};
constexpr size_t kStatsWords = kMaxStats + 2;

hist_status save_state(hist_s *h, Saved &sv, hipStream_t s)
{
    const size_t T = (size_t)h->T;
    if (hipMalloc(&sv.cnt, T * 8) != hipSuccess || hipMalloc(&sv.sumw, T * 8) != hipSuccess ||
        hipMalloc(&sv.sumw2, T * 8) != hipSuccess || hipMalloc(&sv.stats, 8 * kStatsWords) != hipSuccess)
        return set_error(HIST_ENOMEM, "hist_tune: cannot save the histogram");
    if (hipMemcpyAsync(sv.cnt, h->d_cnt, T * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sv.sumw, h->d_sumw, T * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sv.sumw2, h->d_sumw2, T * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(sv.stats, h->d_stats, 8 * kStatsWords, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return set_error(HIST_EDEVICE, "hist_tune: save copy failed");
    return HIST_OK;
}

hist_status restore_state(hist_s *h, Saved &sv, hipStream_t s)
{
    const size_t T = (size_t)h->T;
    hist_status st = HIST_OK;
    if (sv.cnt && (hipMemcpyAsync(h->d_cnt, sv.cnt, T * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                   hipMemcpyAsync(h->d_sumw, sv.sumw, T * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                   hipMemcpyAsync(h->d_sumw2, sv.sumw2, T * 8, hipMemcpyDeviceToDevice, s) != hipSuccess ||
                   hipMemcpyAsync(h->d_stats, sv.stats, 8 * kStatsWords, hipMemcpyDeviceToDevice, s) != hipSuccess))
        st = set_error(HIST_EDEVICE, "hist_tune: restore copy failed");
    (void)hipStreamSynchronize(s);
    (void)hipFree(sv.cnt);
    (void)hipFree(sv.sumw);
    (void)hipFree(sv.sumw2);
    (void)hipFree(sv.stats);
    return st;
}

// Window of `len` bins with the largest sample mass.
int64_t best_window(const std::vector<int32_t> &bins, int64_t T, int64_t len)
{
    std::vector<int64_t> cnt((size_t)T, 0);
    for (int32_t g : bins)
        if (g >= 0 && g < T)
            cnt[(size_t)g]++;
    int64_t run = 0;
    for (int64_t g = 0; g < len && g < T; ++g)
        run += cnt[(size_t)g];
    int64_t best = run, at = 0;
    for (int64_t g = len; g < T; ++g) {
        run += cnt[(size_t)g] - cnt[(size_t)(g - len)];
        if (run > best) {
            best = run;
            at = g - len + 1;
        }
    }
    return at;
}

}  // namespace

extern "C" hist_status hist_tune(hist_t *h, const void *const *coords, const void *weights,
                                 int64_t n, hist_dtype dtype, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_tune: NULL handle");
    if (n <= 0 || !coords)
        return set_error(HIST_EINVAL, "hist_tune: need a non-empty sample");
    for (int d = 0; d < h->dims; ++d)
        if (!coords[d])
            return set_error(HIST_EINVAL, "hist_tune: coordinate %d is NULL", d);
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return set_error(HIST_ECAPTURE, "hist_tune: stream is capturing");
    const bool weighted = weights != nullptr;
    const bool f32 = dtype == HIST_F32;

    // window with the largest mass in the sample (only matters when T exceeds LDS)
    PlanChoice auto_c;
    Plan p0 = plan_from_choice(h, n, dtype, weighted, auto_c);
    int64_t win_lo = 0;
    const int64_t cap_len = p0.strategy == HIST_STRAT_LDS ? p0.win_len : 0;
    if (cap_len > 0 && cap_len < h->T) {
        int32_t *d_bins = nullptr;
        if (hipMalloc(&d_bins, (size_t)n * 4) != hipSuccess)
            return set_error(HIST_ENOMEM, "hist_tune: sample bins");
        hist_status st = hist_findbin(h, coords, n, dtype, d_bins, stream);
        std::vector<int32_t> bins((size_t)n);
        if (st == HIST_OK &&
            (hipMemcpyAsync(bins.data(), d_bins, (size_t)n * 4, hipMemcpyDeviceToHost, s) != hipSuccess ||
             hipStreamSynchronize(s) != hipSuccess))
            st = set_error(HIST_EDEVICE, "hist_tune: sample bins copy");
        (void)hipFree(d_bins);
        if (st != HIST_OK)
            return st;
        win_lo = best_window(bins, h->T, cap_len);
    }

    // candidates.  The learned one-axis kernel keeps 1024-thread workgroups:
    // with 512 it is 12% slower on a 5e7-event fill, yet samples of 2^22 and
    // 2^24 events at times ranked 512 first.
    const bool lean0 = p0.strategy == HIST_STRAT_LDS &&
                       learned_lean_supported(h->dims, f32, weighted, p0.acc, h->ax);
    std::vector<PlanChoice> cands;
    for (int strat : {HIST_STRAT_LDS, HIST_STRAT_GLOBAL, HIST_STRAT_TILED, HIST_STRAT_PART}) {
        if ((strat == HIST_STRAT_TILED || strat == HIST_STRAT_PART) && p0.acc != ACC_U16 &&
            h->T * 16 <= h->lds_max)
            continue;
        if (strat == HIST_STRAT_PART) {
            // the bucket width follows the fill size (see plan_from_choice),
            // which a sample would not represent
            PlanChoice c;
            c.strategy = strat;
            cands.push_back(c);
            continue;
        }
        if (strat == HIST_STRAT_LDS) {
            for (int thr : {512, 1024}) {
                if (lean0 && thr != 1024)
                    continue;
                for (int bpc : {1, 2}) {
                    for (int merge : {MERGE_ATOMIC, MERGE_STAGE}) {
                        PlanChoice c;
                        c.strategy = strat;
                        c.blocks_per_cu = bpc;
                        c.merge = merge;
                        c.win_lo = win_lo;
                        c.threads = thr;
                        cands.push_back(c);
                    }
                }
            }
        } else {
            PlanChoice c;
            c.strategy = strat;
            cands.push_back(c);
        }
    }

    Saved sv;
    hist_status st = save_state(h, sv, s);
    if (st != HIST_OK) {
        restore_state(h, sv, s);
        return st;
    }
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    // the heuristic plan goes first; another candidate replaces it only when
    // it is clearly faster, so that near-ties do not flip between runs
    PlanChoice heur = auto_c;
    heur.strategy = p0.strategy;
    heur.win_lo = win_lo;
    cands.insert(cands.begin(), heur);
    // Best of five timed runs after a warm-up; false when the plan differs
    // from the choice (the strategy does not apply) or fails.
    auto time_choice = [&](const PlanChoice &c, float &out) -> bool {
        Plan p = plan_from_choice(h, n, dtype, weighted, c);
        if (p.strategy != c.strategy)
            return false;
        hist_status rs = run_plan(h, p, coords, weights, n, dtype, s);   // warm-up (and allocations)
        if (rs != HIST_OK) {
            if (std::getenv("HIST_LOG"))
                fprintf(stderr, "hist_tune: candidate strategy %d bucket_bits %d failed: %s\n",
                        c.strategy, c.bucket_bits, hist_last_error());
            return false;
        }
        float tmin = 1e30f;
        for (int r = 0; r < 5 && rs == HIST_OK; ++r) {
            (void)hipEventRecord(e0, s);
            rs = run_plan(h, p, coords, weights, n, dtype, s);
            (void)hipEventRecord(e1, s);
            (void)hipEventSynchronize(e1);
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tmin = std::min(tmin, ms);
        }
        out = tmin;
        return rs == HIST_OK;
    };
    // the heuristic plan goes first; another candidate replaces it only when
    // it is clearly faster, so that near-ties do not flip between runs
    float best_ms = 1e30f, heur_ms = 1e30f;
    PlanChoice best = heur;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        float ms;
        if (!time_choice(cands[ci], ms))
            continue;
        if (ci == 0)
            heur_ms = ms;
        if (ms < best_ms) {
            best_ms = ms;
            best = cands[ci];
        }
    }
    if (heur_ms <= best_ms * 1.05f) {
        best = heur;
        best_ms = heur_ms;
    }
    // Refinement of the chosen LDS or global plan, one knob at a time: the
    // interleaved copies of a small window (1 .. 64), then the events per
    // thread (1, 2, 4, 8 where a variant exists).  A change is kept only when
    // it is at least 3% faster.
    const Plan pb = plan_from_choice(h, n, dtype, weighted, best);
    if (pb.strategy == HIST_STRAT_LDS && (pb.acc == ACC_U32 || pb.acc == ACC_F64) &&
        pb.win_len == h->T) {
        PlanChoice base = best;
        for (int r : {1, 2, 4, 8, 16, 32, 64}) {
            PlanChoice c = base;
            c.copies = r;
            if (plan_from_choice(h, n, dtype, weighted, c).copies != r)
                continue;
            float ms;
            if (time_choice(c, ms) && ms < best_ms * 0.97f) {
                best_ms = ms;
                best = c;
            }
        }
    }
    // The events per thread of the general kernels.  A plan that runs the
    // learned one-axis kernel keeps it: that kernel stages its model in every
    // workgroup, a fixed cost that weighs more on a sample than on a full
    // fill, so a sample can rank a general shape ahead of it that is slower
    // at full size.
    const bool lean = pb.strategy == HIST_STRAT_LDS && !pb.shape && pb.unroll == 8 &&
                      learned_lean_supported(h->dims, f32, weighted, pb.acc, h->ax);
    if ((pb.strategy == HIST_STRAT_LDS || pb.strategy == HIST_STRAT_GLOBAL) && !lean) {
        PlanChoice base = best;
        for (int u : {1, 2, 4, 8}) {
            PlanChoice c = base;
            c.unroll = u;
            const Plan pu = plan_from_choice(h, n, dtype, weighted, c);
            if (!pu.shape || pu.unroll != u)
                continue;
            float ms;
            if (time_choice(c, ms) && ms < best_ms * 0.97f) {
                best_ms = ms;
                best = c;
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    st = restore_state(h, sv, s);
    h->tuned[std::make_tuple(weighted ? 1 : 0, f32 ? 1 : 0, 0)] = best;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        g_cache[shape_key(h, weighted, f32)] = best;
    }
    if (std::getenv("HIST_LOG"))
        fprintf(stderr, "hist_tune: T=%lld n=%lld -> strategy %d bpc %d merge %d win_lo %lld "
                        "bucket_bits %d copies %d unroll %d (%.3f ms)\n",
                (long long)h->T, (long long)n, best.strategy, best.blocks_per_cu, best.merge,
                (long long)best.win_lo, best.bucket_bits, best.copies, best.unroll, best_ms);
    return st;
}
