// hist_api.hip -- host side of the C ABI declared in include/hist.h.
//
// A hist_t is the GPU histogram object of arXiv:2401.13310 Sec. 3.2: it owns
// the device allocations (bin sums, statistics, edges, learned models,
// scratch), takes bulks of events through hist_fill (Sec. 3.1 steps 1-3 in one
// pass), keeps adding to the same sums across bulks (Sec. 3.3), and copies the
// result back only when it is read.
#include "../../include/hist.h"
#include "kernels.h"
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <mutex>
#include <string>
#include <vector>

using namespace hg;

// ---------------------------------------------------------------- errors ----

static thread_local std::string g_err;

hist_status hg::set_error(hist_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

static hist_status hip_fail(hipError_t e, const char *what)
{
    (void)hipGetLastError();
    return set_error(HIST_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIPCHK(expr, what)                        \
    do {                                          \
        hipError_t e_ = (expr);                   \
        if (e_ != hipSuccess)                     \
            return hip_fail(e_, what);            \
    } while (0)

extern "C" const char *hist_strerror(hist_status s)
{
    switch (s) {
    case HIST_OK: return "ok";
    case HIST_EINVAL: return "invalid argument";
    case HIST_ENOMEM: return "out of memory";
    case HIST_EDEVICE: return "device error";
    case HIST_ECAPTURE: return "not allowed during stream capture";
    case HIST_ENOTSUP: return "not supported";
    }
    return "unknown status";
}

extern "C" const char *hist_last_error(void) { return g_err.c_str(); }
extern "C" const char *hist_version(void) { return "histgpu 0.1 gfx950"; }

// ------------------------------------------------------------ helpers ------

uint64_t hg::host_order_key(double x)
{
    x = x + 0.0;
    uint64_t k;
    std::memcpy(&k, &x, sizeof(k));
    return (k >> 63) ? ~k : (k | 0x8000000000000000ull);
}

static bool is_capturing(hipStream_t s)
{
    hipStreamCaptureStatus st = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &st) != hipSuccess) {
        (void)hipGetLastError();   // leave no stale error for the next launch check
        return false;
    }
    return st != hipStreamCaptureStatusNone;
}

template <typename T>
static hipError_t dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0)
        return hipSuccess;
    return hipMalloc(reinterpret_cast<void **>(p), count * sizeof(T));
}

static void dfree(void *p)
{
    if (p && hipFree(p) != hipSuccess)
        (void)hipGetLastError();
}

static void free_handle(hist_s *h)
{
    if (!h)
        return;
    for (int a = 0; a < kMaxDims; ++a) {
        dfree(h->d_edges[a]);
        dfree(h->d_model[a]);
    }
    dfree(h->d_cnt);
    dfree(h->d_sumw);
    dfree(h->d_sumw2);
    dfree(h->d_stats);
    dfree(h->d_stage);
    dfree(h->d_gbins);
    dfree(h->d_part);
    for (hipEvent_t e : h->ev_pool)
        (void)hipEventDestroy(e);
    host_streamer_destroy(h->host);
    delete h;
}

hist_status hg::zero_state(hist_s *h, hipStream_t s)
{
    HIPCHK(launch_zero_u64(h->d_cnt, h->T, s), "zero counts");
    HIPCHK(launch_zero_f64(h->d_sumw, h->T, s), "zero sumw");
    HIPCHK(launch_zero_f64(h->d_sumw2, h->T, s), "zero sumw2");
    // statistics and the entry counter (its zero bit pattern) in one launch
    HIPCHK(launch_zero_f64(h->d_stats, kMaxStats + 2, s), "zero stats");
    return HIST_OK;
}

// ----------------------------------------------------------- lifecycle -----

extern "C" hist_status hist_create(int dims, const hist_axis *axes, uint32_t flags, hist_t **out)
{
    if (!out)
        return set_error(HIST_EINVAL, "hist_create: out is NULL");
    *out = nullptr;
    if (dims < 1 || dims > kMaxDims)
        return set_error(HIST_EINVAL, "hist_create: dims must be 1..3 (got %d)", dims);
    if (!axes)
        return set_error(HIST_EINVAL, "hist_create: axes is NULL");
    if (flags & ~(uint32_t)(HIST_F_ACC_F32C | HIST_F_LEARNED | HIST_F_NO_ALLOC))
        return set_error(HIST_EINVAL, "hist_create: unknown flags 0x%x", flags);
    int64_t T = 1;
    for (int a = 0; a < dims; ++a) {
        const hist_axis &ax = axes[a];
        if (ax.nbins < 1)
            return set_error(HIST_EINVAL, "hist_create: axis %d: nbins must be >= 1", a);
        if (ax.nbins > 0x7FFFFFFD)
            return set_error(HIST_EINVAL, "hist_create: axis %d: nbins too large", a);
        if (ax.edges) {
            for (int32_t i = 0; i <= ax.nbins; ++i) {
                if (!std::isfinite(ax.edges[i]))
                    return set_error(HIST_EINVAL, "hist_create: axis %d: edge %d not finite", a, i);
                if (i > 0 && !(ax.edges[i - 1] < ax.edges[i]))
                    return set_error(HIST_EINVAL,
                                     "hist_create: axis %d: edges not strictly increasing at %d", a, i);
            }
        } else {
            if (!std::isfinite(ax.xmin) || !std::isfinite(ax.xmax) || !(ax.xmin < ax.xmax))
                return set_error(HIST_EINVAL, "hist_create: axis %d: need finite xmin < xmax", a);
            if (!std::isfinite(ax.xmax - ax.xmin))
                return set_error(HIST_EINVAL, "hist_create: axis %d: xmax - xmin overflows", a);
        }
        T *= (int64_t)ax.nbins + 2;
        if (T > 0x7FFFFFFFll)
            return set_error(HIST_EINVAL, "hist_create: total bins exceed 2^31-1");
    }

    hist_s *h = new (std::nothrow) hist_s();
    if (!h)
        return set_error(HIST_ENOMEM, "hist_create: host allocation");
    h->dims = dims;
    h->flags = flags;
    h->T = T;
    h->S = 2 + 2 * dims + dims * (dims - 1) / 2;
    (void)hipGetDevice(&h->device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, h->device) != hipSuccess) {
        free_handle(h);
        return set_error(HIST_EDEVICE, "hist_create: no HIP device");
    }
    h->num_cu = prop.multiProcessorCount;
    h->lds_max = (int)prop.sharedMemPerBlock;
    if (h->lds_max > 163840)
        h->lds_max = 163840;

    int32_t stride = 1;
    for (int a = 0; a < dims; ++a) {
        const hist_axis &ax = axes[a];
        AxisDev &d = h->ax[a];
        std::memset(&d, 0, sizeof(d));
        d.nbins = ax.nbins;
        d.nbins_d = (double)ax.nbins;
        d.lds_model = -1;
        d.lds_edges = -1;
        d.stride = stride;
        stride *= ax.nbins + 2;
        if (ax.edges) {
            h->variable[a] = true;
            h->edges_host[a].assign(ax.edges, ax.edges + ax.nbins + 1);
            d.kind = AX_BSEARCH;
            d.xmin = ax.edges[0];
            d.xmax = ax.edges[ax.nbins];
            // the edges, then +inf (a learned fill's lanes that need no edge
            // read it)
            const double inf = std::numeric_limits<double>::infinity();
            hipError_t e = dalloc(&h->d_edges[a], (size_t)ax.nbins + 2);
            if (e == hipSuccess)
                e = hipMemcpy(h->d_edges[a], ax.edges, sizeof(double) * (ax.nbins + 1),
                              hipMemcpyHostToDevice);
            if (e == hipSuccess)
                e = hipMemcpy(h->d_edges[a] + ax.nbins + 1, &inf, sizeof(double), hipMemcpyHostToDevice);
            if (e != hipSuccess) {
                free_handle(h);
                return set_error(e == hipErrorOutOfMemory ? HIST_ENOMEM : HIST_EDEVICE,
                                 "hist_create: edges: %s", hipGetErrorString(e));
            }
            d.edges = h->d_edges[a];
        } else {
            d.kind = AX_UNIFORM;
            d.xmin = ax.xmin;
            d.xmax = ax.xmax;
            d.width = ax.xmax - ax.xmin;
            d.guess = d.nbins_d / d.width;
            d.margin = 1e-15 * ((double)ax.nbins + 1.0);
        }
    }
    hipError_t e = dalloc(&h->d_cnt, (size_t)T);
    if (e == hipSuccess)
        e = dalloc(&h->d_sumw, (size_t)T);
    if (e == hipSuccess)
        e = dalloc(&h->d_sumw2, (size_t)T);
    if (e == hipSuccess)
        e = dalloc(&h->d_stats, (size_t)kMaxStats + 2);   // statistics, then the entry count
    if (e == hipSuccess)
        h->d_entries = reinterpret_cast<uint64_t *>(h->d_stats + kMaxStats + 1);
    if (e != hipSuccess) {
        free_handle(h);
        return set_error(e == hipErrorOutOfMemory ? HIST_ENOMEM : HIST_EDEVICE,
                         "hist_create: bins: %s", hipGetErrorString(e));
    }
    hist_status st = zero_state(h, nullptr);
    if (st == HIST_OK && hipDeviceSynchronize() != hipSuccess)
        st = set_error(HIST_EDEVICE, "hist_create: synchronize failed");
    if (st != HIST_OK) {
        free_handle(h);
        return st;
    }
    if (flags & HIST_F_LEARNED) {
        for (int a = 0; a < dims; ++a) {
            if (!h->variable[a])
                continue;
            st = hist_train_index(h, a, nullptr);
            if (st != HIST_OK) {
                free_handle(h);
                return st;
            }
        }
    }
    *out = h;
    return HIST_OK;
}

extern "C" hist_status hist_destroy(hist_t *h)
{
    if (!h)
        return HIST_OK;
    const int users = h->users.load();
    if (users > 0)
        return set_error(HIST_EINVAL, "hist_destroy: the handle is a member of %d live batch(es) or "
                                      "multi-fill set(s); destroy those first", users);
    (void)hipDeviceSynchronize();
    free_handle(h);
    return HIST_OK;
}

extern "C" int64_t hist_nbins_total(const hist_t *h) { return h ? h->T : -1; }
extern "C" int hist_nstats(const hist_t *h) { return h ? h->S : -1; }

// ---------------------------------------------------------------- scratch --

// A fill may grow its scratch only outside capture and only for handles
// created without HIST_F_NO_ALLOC; hist_reserve always may.
static hist_status may_grow(hist_s *h, hipStream_t s, bool reserving, const char *what)
{
    if (!reserving && (h->flags & HIST_F_NO_ALLOC))
        return set_error(HIST_ENOMEM, "hist_fill: the %s this plan needs exceeds what "
                                      "hist_reserve set aside (HIST_F_NO_ALLOC handle)", what);
    if (is_capturing(s))
        return set_error(HIST_ECAPTURE, "hist_fill: the %s this plan needs is not allocated; "
                                        "call hist_reserve (or fill once) before capturing", what);
    return HIST_OK;
}

hist_status hg::ensure_stage(hist_s *h, size_t bytes, hipStream_t s, bool reserving)
{
    if (h->stage_bytes >= bytes)
        return HIST_OK;
    hist_status g = may_grow(h, s, reserving, "staging buffer");
    if (g != HIST_OK)
        return g;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
        return set_error(HIST_ENOMEM, "staging buffer of %zu bytes: %s", bytes, hipGetErrorString(e));
    if (h->d_stage) {
        HIPCHK(hipStreamSynchronize(s), "synchronize before freeing scratch");
        dfree(h->d_stage);
    }
    h->d_stage = p;
    h->stage_bytes = bytes;
    return HIST_OK;
}

hist_status hg::ensure_gbins(hist_s *h, int64_t count, hipStream_t s, bool reserving)
{
    if (h->gbins_cap >= count)
        return HIST_OK;
    hist_status g = may_grow(h, s, reserving, "bin scratch");
    if (g != HIST_OK)
        return g;
    int32_t *p = nullptr;
    hipError_t e = dalloc(&p, (size_t)count);
    if (e != hipSuccess)
        return set_error(HIST_ENOMEM, "tile scratch: %s", hipGetErrorString(e));
    if (h->d_gbins) {
        HIPCHK(hipStreamSynchronize(s), "synchronize before freeing scratch");
        dfree(h->d_gbins);
    }
    h->d_gbins = p;
    h->gbins_cap = count;
    return HIST_OK;
}

static hist_status ensure_part(hist_s *h, size_t bytes, hipStream_t s, bool reserving = false)
{
    if (h->part_bytes >= bytes)
        return HIST_OK;
    hist_status g = may_grow(h, s, reserving, "partition scratch");
    if (g != HIST_OK)
        return g;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess)
        return set_error(HIST_ENOMEM, "partition scratch of %zu bytes: %s", bytes,
                         hipGetErrorString(e));
    if (h->d_part) {
        HIPCHK(hipStreamSynchronize(s), "synchronize before freeing scratch");
        dfree(h->d_part);
    }
    h->d_part = p;
    h->part_bytes = bytes;
    h->part_zero_at = nullptr;
    return HIST_OK;
}

// Scratch layout of the partitioned strategy for chunks of at most mmax
// events: the count table, four (nbuckets + 1)-word arrays, the in-bucket
// offsets and (weighted) the weights in bucket order.
struct PartLayout {
    int nb;
    size_t table_b, start_b, off_b, w_b;
    size_t total() const { return table_b + start_b + off_b + w_b; }
};

static PartLayout part_layout(const hist_s *h, const Plan &p, int64_t mmax, bool weighted)
{
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    PartLayout L;
    L.nb = (int)((h->T + ((int64_t)1 << p.bucket_bits) - 1) >> p.bucket_bits);
    L.table_b = up((size_t)L.nb * p.blocks * 4);
    L.start_b = 4 * up((size_t)(L.nb + 1) * 4);
    L.off_b = up((size_t)mmax * 2);
    L.w_b = weighted ? up((size_t)mmax * 8) : 0;
    return L;
}

// The four passes of the partitioned strategy over chunks of at most
// part_chunk events (see partition.hip).
static size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// The learned one-axis kernel: one binary64 axis with a trained index whose
// edges stay in HBM, unit weights, 16-bit LDS window, the heuristic shape.
static bool use_learned_lean(const hist_s *h, const Plan &p, bool f32, bool weighted)
{
    return p.strategy == HIST_STRAT_LDS && !p.shape && p.unroll == 8 &&
           learned_lean_supported(h->dims, f32, weighted, p.acc, h->ax);
}

// Its LDS layout: the window at 0, the model, the statistics partials, the
// hot-bin cache; the window gives up bins (a few, from its top) if the LDS
// would be exceeded.  Returns the LDS bytes, 0 if no window fits.
static int lean_layout(const hist_s *h, const Plan &p, FillArgs &a)
{
    auto a16 = [](int64_t x) { return (x + 15) & ~(int64_t)15; };
    const int64_t model_b = (int64_t)h->ax[0].nseg * (int64_t)sizeof(ModelSeg);
    const int64_t cache_b = p.lds_cache >= 0 ? cache_bytes(p.cache_slots, false) : 0;
    int64_t wl = p.win_len, total = 0;
    for (;;) {
        total = a16(((wl + 1) / 2) * 4) + a16(model_b) + kRedBytes + cache_b;
        if (total <= h->lds_max)
            break;
        wl -= 64;
        if (wl < 64)
            return 0;
    }
    const int64_t win_b = a16(((wl + 1) / 2) * 4);
    a.win_len = (int32_t)wl;
    a.lds_win = 0;
    a.ax[0].lds_model = (int32_t)win_b;
    a.lds_red = (int32_t)(win_b + a16(model_b));
    a.lds_cache = p.lds_cache >= 0 ? a.lds_red + kRedBytes : -1;
    return (int)total;
}

// Events per chunk of a partitioned fill whose scratch (bin array plus
// partition tables) must fit `bytes`: the largest power of two up to the
// usual chunk that fits, 0 if none of at least 2^12 does.
static int64_t fixed_part_chunk(const hist_s *h, const Plan &p, bool weighted, size_t bytes)
{
    for (int64_t m = part_chunk(h); m >= ((int64_t)1 << 12); m >>= 1)
        if (up256((size_t)m * 4) + part_layout(h, p, m, weighted).total() <= bytes)
            return m;
    return 0;
}

static hist_status run_part(hist_s *h, const Plan &p, FillArgs a, const void *const *coords,
                            const void *w, int64_t n, bool f32, hipStream_t s, const FixedScratch *fx)
{
    const bool weighted = w != nullptr;
    const int64_t cap = fx ? fixed_part_chunk(h, p, weighted, fx->bytes) : part_chunk(h);
    if (cap <= 0)
        return set_error(HIST_ENOMEM, "hist_fill_static: the partition tables of this histogram "
                                      "exceed the %zu-byte scratch", fx->bytes);
    const int64_t mmax = n < cap ? n : cap;
    const int b = p.bucket_bits;
    const PartLayout L = part_layout(h, p, mmax, weighted);
    const int nb = L.nb;
    const int G = p.blocks;
    const size_t table_b = L.table_b, start_b = L.start_b, off_b = L.off_b;
    char *base;
    int32_t *gbins;
    if (fx) {
        gbins = reinterpret_cast<int32_t *>(fx->base);
        base = fx->base + up256((size_t)mmax * 4);
    } else {
        hist_status st = ensure_gbins(h, mmax, s);
        if (st != HIST_OK)
            return st;
        st = ensure_part(h, L.total(), s);
        if (st != HIST_OK)
            return st;
        base = static_cast<char *>(h->d_part);
        gbins = h->d_gbins;
    }
    PartArgs P;
    std::memset(&P, 0, sizeof(P));
    P.table = reinterpret_cast<uint32_t *>(base);
    P.bucket_start = reinterpret_cast<uint32_t *>(base + table_b);
    P.chunk_start = reinterpret_cast<uint32_t *>(base + table_b + start_b / 4);
    P.totals = reinterpret_cast<uint32_t *>(base + table_b + 2 * (start_b / 4));
    P.cursor = reinterpret_cast<uint32_t *>(base + table_b + 3 * (start_b / 4));
    P.rec_off = reinterpret_cast<uint16_t *>(base + table_b + start_b);
    P.rec_w = weighted ? reinterpret_cast<double *>(base + table_b + start_b + off_b) : nullptr;
    P.T = h->T;
    P.nbuckets = nb;
    P.bshift = b;
    P.lds_buckets = p.lds_base;
    a.gbins = gbins;
    const size_t esz = f32 ? 4 : 8;
    const size_t acc_lds = (size_t)(weighted ? 16 : 4) << b;
    const int t0 = h->timing ? timing_event(h) : -1;
    if (t0 >= 0)
        HIPCHK(hipEventRecord(h->ev_pool[t0], s), "timing event");
    for (int64_t off = 0; off < n; off += cap) {
        const int64_t m = (n - off) < cap ? (n - off) : cap;
        FillArgs c = a;
        for (int d = 0; d < h->dims; ++d)
            c.coords[d] = static_cast<const char *>(coords[d]) + off * esz;
        c.w = w ? static_cast<const char *>(w) + off * esz : nullptr;
        c.n = m;
        const int64_t step = (int64_t)p.threads * unroll_of(h, f32, weighted, ACC_PCOUNT);
        int64_t per = (m + G - 1) / G;
        per = (per + step - 1) / step * step;
        const int g = (int)((m + per - 1) / per);
        c.per_block = per;
        // count pass: the fill kernel in its partition-count mode
        c.win_lo = 0;
        c.win_len = nb;
        c.copies = 1;
        c.lds_win = p.lds_base;
        c.part_table = P.table;
        c.part_totals = P.totals;
        c.part_shift = b;
        // a fill that ran its scatter pass left these totals zero (never
        // assumed of fixed scratch, which other fills share)
        const bool clean = !fx && h->part_zero_at == P.totals && nb <= h->part_zero_n;
        h->part_zero_at = nullptr;
        if (!clean)
            HIPCHK(launch_zero_u32(P.totals, nb, s), "partition totals reset");
        HIPCHK(launch_fill(h->dims, f32, ACC_PCOUNT, weighted, p.threads, g, (size_t)p.lds, c, s),
               "partition count launch");
        HIPCHK(launch_part_scan(P, s), "partition scan launch");
        HIPCHK(launch_part_scatter(f32, weighted, kMaxThreads, g, (size_t)part_scatter_lds(nb, weighted),
                                   c, P, s),
               "partition scatter launch");
        if (!fx) {
            h->part_zero_at = P.totals;
            h->part_zero_n = nb;
        }
        // every bucket has at most ceil(records / kPartChunk) chunks
        const int chunks_max = nb + (int)((m + kPartChunk - 1) / kPartChunk);
        HIPCHK(launch_part_accum(weighted, 1024, chunks_max, acc_lds, c, P, s),
               "partition accumulate launch");
    }
    const int t1 = h->timing ? timing_event(h) : -1;
    if (t0 >= 0 && t1 >= 0) {
        HIPCHK(hipEventRecord(h->ev_pool[t1], s), "timing event");
        h->ev_fill.emplace_back(t0, t1);
    }
    return HIST_OK;
}

// ---------------------------------------------------------- kernel timing --

int hg::timing_event(hist_s *h)
{
    if (h->ev_next >= (int)h->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess)
            return -1;
        h->ev_pool.push_back(e);
    }
    return h->ev_next++;
}

extern "C" hist_status hist_timing(hist_t *h, int enable)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_timing: NULL handle");
    h->timing = enable != 0;
    h->ev_fill.clear();
    h->ev_merge.clear();
    h->ev_next = 0;
    return HIST_OK;
}

extern "C" hist_status hist_timing_read(hist_t *h, double *fill_ms, double *merge_ms,
                                        int64_t *launches)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_timing_read: NULL handle");
    double f = 0.0, m = 0.0;
    for (auto &pr : h->ev_fill) {
        if (pr.first < 0 || pr.second < 0)
            continue;
        HIPCHK(hipEventSynchronize(h->ev_pool[pr.second]), "timing synchronize");
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev_pool[pr.first], h->ev_pool[pr.second]), "elapsed");
        f += ms;
    }
    for (auto &pr : h->ev_merge) {
        if (pr.first < 0 || pr.second < 0)
            continue;
        HIPCHK(hipEventSynchronize(h->ev_pool[pr.second]), "timing synchronize");
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, h->ev_pool[pr.first], h->ev_pool[pr.second]), "elapsed");
        m += ms;
    }
    if (fill_ms)
        *fill_ms = f;
    if (merge_ms)
        *merge_ms = m;
    if (launches)
        *launches = (int64_t)h->ev_fill.size();
    h->ev_fill.clear();
    h->ev_merge.clear();
    h->ev_next = 0;
    return HIST_OK;
}

// ----------------------------------------------------------------- fill ----

static hist_status check_coords(const hist_s *h, const void *const *coords, int64_t n,
                                const char *who)
{
    if (n < 0)
        return set_error(HIST_EINVAL, "%s: n < 0", who);
    if (n == 0)
        return HIST_OK;
    if (!coords)
        return set_error(HIST_EINVAL, "%s: coords is NULL", who);
    for (int a = 0; a < h->dims; ++a)
        if (!coords[a])
            return set_error(HIST_EINVAL, "%s: coordinate %d is NULL", who, a);
    return HIST_OK;
}

FillArgs hg::base_args(const hist_s *h, const void *const *coords, const void *w, int64_t n)
{
    FillArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int d = 0; d < kMaxDims; ++d) {
        a.ax[d] = h->ax[d];
        a.coords[d] = d < h->dims ? coords[d] : nullptr;
    }
    a.w = w;
    a.n = n;
    a.copies = 1;
    a.total_bins = (int32_t)h->T;
    a.lds_cache = -1;
    a.cache_slots = 0;
    a.cnt = h->d_cnt;
    a.sumw = h->d_sumw;
    a.sumw2 = h->d_sumw2;
    a.stats = h->d_stats;
    a.entries = h->d_entries;
    a.stage = h->d_stage;
    return a;
}

hist_status hg::run_plan(hist_s *h, const Plan &p, const void *const *coords, const void *w,
                         int64_t n, hist_dtype dtype, hipStream_t s, const FixedScratch *fx)
{
    // launches are checked with hipGetLastError: start from a clean state, so
    // an error left by an unrelated runtime call is not reported as ours
    (void)hipGetLastError();
    const bool f32 = dtype == HIST_F32;
    const bool weighted = w != nullptr;
    FillArgs a = base_args(h, coords, w, n);
    apply_model_offsets(h, a);
    if (p.strategy == HIST_STRAT_PART)
        return run_part(h, p, a, coords, w, n, f32, s, fx);
    if (p.strategy == HIST_STRAT_TILED) {
        // fixed scratch holds the bin array of a chunk of bytes/4 events
        int64_t cap = tiled_chunk(h);
        if (fx)
            while (cap > 1 && (size_t)cap * 4 > fx->bytes)
                cap >>= 1;
        int32_t *gbins;
        if (fx) {
            gbins = reinterpret_cast<int32_t *>(fx->base);
        } else {
            hist_status st = ensure_gbins(h, n < cap ? n : cap, s);
            if (st != HIST_OK)
                return st;
            gbins = h->d_gbins;
        }
        a.gbins = gbins;
        const size_t esz = f32 ? 4 : 8;
        const int t0 = h->timing ? timing_event(h) : -1;
        if (t0 >= 0)
            HIPCHK(hipEventRecord(h->ev_pool[t0], s), "timing event");
        for (int64_t off = 0; off < n; off += cap) {
            const int64_t m = (n - off) < cap ? (n - off) : cap;
            FillArgs c = a;
            for (int d = 0; d < h->dims; ++d)
                c.coords[d] = static_cast<const char *>(coords[d]) + off * esz;
            c.w = w ? static_cast<const char *>(w) + off * esz : nullptr;
            c.n = m;
            int bb = (int)((m + p.threads - 1) / p.threads);
            const int bmax = h->num_cu * 4;
            if (bb > bmax)
                bb = bmax;
            if (bb < 1)
                bb = 1;
            HIPCHK(launch_tiled_bins(h->dims, f32, weighted, p.threads, bb, (size_t)p.lds_base, c, s),
                   "tiled bins launch");
            TileArgs t;
            std::memset(&t, 0, sizeof(t));
            t.gbins = gbins;
            t.w = c.w;
            t.n = m;
            t.tile_len = p.win_len;
            t.T = (int32_t)h->T;
            t.copies = p.copies;
            t.lds_win = p.lds_base;
            t.epoch_iters = p.epoch_iters;
            t.cnt = h->d_cnt;
            t.sumw = h->d_sumw;
            t.sumw2 = h->d_sumw2;
            const int tiles = (int)((h->T + p.win_len - 1) / p.win_len);
            int bx = p.blocks;
            const int64_t step = (int64_t)p.threads * 4;
            int64_t per = (m + bx - 1) / bx;
            per = (per + step - 1) / step * step;
            bx = (int)((m + per - 1) / per);
            if (bx < 1)
                bx = 1;
            t.per_block = per;
            HIPCHK(launch_tile(p.acc, f32, p.threads, bx, tiles, (size_t)p.lds, t, s), "tile launch");
        }
        const int t1 = h->timing ? timing_event(h) : -1;
        if (t0 >= 0 && t1 >= 0) {
            HIPCHK(hipEventRecord(h->ev_pool[t1], s), "timing event");
            h->ev_fill.emplace_back(t0, t1);
        }
        return HIST_OK;
    }
    a.win_lo = p.win_lo;
    a.win_len = p.win_len;
    a.copies = p.copies;
    a.merge = p.merge;
    a.lds_win = p.lds_base;
    a.lds_cache = p.lds_cache;
    a.cache_slots = p.cache_slots;
    a.epoch_iters = p.epoch_iters;
    a.per_block = p.per_block;
    const bool lean = use_learned_lean(h, p, f32, weighted);
    const int lean_lds = lean ? lean_layout(h, p, a) : 0;
    if (lean && lean_lds <= 0)
        return set_error(HIST_EINVAL, "hist_fill: no LDS layout for the learned kernel");
    if (p.merge == MERGE_STAGE) {
        const size_t stage_b = stage_bytes_for(p);
        char *base = nullptr;
        if (fx) {
            if (stage_b > fx->bytes)
                return set_error(HIST_ENOMEM, "hist_fill_static: the staging slots of this plan (%zu "
                                              "bytes) exceed the %zu-byte scratch",
                                 stage_b, fx->bytes);
            base = fx->base;
        } else {
            hist_status st = ensure_stage(h, stage_b, s);
            if (st != HIST_OK)
                return st;
            base = static_cast<char *>(h->d_stage);
        }
        a.stage = base;
        a.stage_stride = stage_stride_of(p.acc, a.win_len);
    }
    const int t0 = h->timing ? timing_event(h) : -1;
    if (t0 >= 0)
        HIPCHK(hipEventRecord(h->ev_pool[t0], s), "timing event");
    if (p.shape) {
        HIPCHK(launch_fill_shape(p.acc, weighted, kind_set(h->dims, a.ax), p.unroll, p.stats_ept == 0,
                                 p.threads, p.blocks, (size_t)p.lds, a, s),
               "fill launch");
        if (p.stats_ept > 0)
            HIPCHK(launch_stats_separate(weighted, p.stats_ept, h->num_cu, a, s), "statistics launch");
    } else if (lean) {
        HIPCHK(launch_fill_learned(p.threads, p.blocks, (size_t)lean_lds, !h->index_narrow[0], a, s),
               "fill launch");
    } else {
        HIPCHK(launch_fill(h->dims, f32, p.acc, weighted, p.threads, p.blocks, (size_t)p.lds, a, s),
               "fill launch");
    }
    const int t1 = h->timing ? timing_event(h) : -1;
    if (t1 >= 0) {
        HIPCHK(hipEventRecord(h->ev_pool[t1], s), "timing event");
        h->ev_fill.emplace_back(t0, t1);
    }
    if (p.merge == MERGE_STAGE) {
        HIPCHK(launch_stage_reduce(p.acc, p.blocks, a, s), "stage reduce launch");
        const int t2 = h->timing ? timing_event(h) : -1;
        if (t2 >= 0) {
            HIPCHK(hipEventRecord(h->ev_pool[t2], s), "timing event");
            h->ev_merge.emplace_back(t1, t2);
        }
    }
    return HIST_OK;
}

extern "C" hist_status hist_fill(hist_t *h, const void *const *coords, const void *weights,
                                 int64_t n, hist_dtype dtype, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_fill: NULL handle");
    if (dtype != HIST_F64 && dtype != HIST_F32)
        return set_error(HIST_EINVAL, "hist_fill: unknown dtype %d", (int)dtype);
    hist_status st = check_coords(h, coords, n, "hist_fill");
    if (st != HIST_OK || n == 0)
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    Plan p = make_plan(h, n, dtype, weights != nullptr);
    return run_plan(h, p, coords, weights, n, dtype, s);
}

// ------------------------------------------------ fills that allocate nothing --

// Scratch of hist_fill_static: one region per device (every GPU the library
// runs on holds its copy until the process ends), shared by every call on
// that device.  In host code `scratch` names a host-side stand-in; kernels get
// the device address that hipGetSymbolAddress returns for the current device.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {
constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxStaticDevices] = {};
}  // namespace

// Device address of the current device's scratch, looked up once per device.
static hist_status static_scratch(FixedScratch &fx)
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return hip_fail(hipGetLastError(), "hist_fill_static: current device");
    if (dev < 0 || dev >= kMaxStaticDevices)
        return set_error(HIST_ENOTSUP, "hist_fill_static: device %d beyond %d", dev, kMaxStaticDevices);
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                            "hist_fill_static: scratch address");
        g_static_ptr[dev] = ptr;
    }
    fx.base = static_cast<char *>(g_static_ptr[dev]);
    fx.bytes = kStaticScratchBytes;
    return HIST_OK;
}

extern "C" hist_status hist_fill_static(hist_t *h, const void *const *coords, const void *weights,
                                        int64_t n, hist_dtype dtype, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_fill_static: NULL handle");
    if (dtype != HIST_F64 && dtype != HIST_F32)
        return set_error(HIST_EINVAL, "hist_fill_static: unknown dtype %d", (int)dtype);
    hist_status st = check_coords(h, coords, n, "hist_fill_static");
    if (st != HIST_OK || n == 0)
        return st;
    FixedScratch fx;
    st = static_scratch(fx);
    if (st != HIST_OK)
        return st;
    const Plan p = make_plan(h, n, dtype, weights != nullptr);
    return run_plan(h, p, coords, weights, n, dtype, static_cast<hipStream_t>(stream), &fx);
}

extern "C" int64_t hist_static_scratch_bytes(void) { return (int64_t)kStaticScratchBytes; }

extern "C" hist_status hist_reserve(hist_t *h, int64_t n_max, hist_dtype dtype, int weighted,
                                    void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_reserve: NULL handle");
    if (n_max < 0 || (dtype != HIST_F64 && dtype != HIST_F32))
        return set_error(HIST_EINVAL, "hist_reserve: need n_max >= 0 and a known dtype");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (is_capturing(s))
        return set_error(HIST_ECAPTURE, "hist_reserve: stream is capturing");
    if (n_max == 0)
        return HIST_OK;
    hist_status st = reserve_scratch(h, n_max, dtype, weighted != 0, s);
    if (st == HIST_OK && hipStreamSynchronize(s) != hipSuccess)
        st = hip_fail(hipGetLastError(), "hist_reserve: synchronize");
    return st;
}

hist_status hg::reserve_scratch(hist_s *h, int64_t n_max, hist_dtype dtype, bool weighted,
                                hipStream_t s)
{
    // Under one plan choice the scratch a fill needs grows with n (more
    // workgroups up to the plan's grid, longer chunks, more buckets), so the
    // plan of n_max events bounds every smaller fill.
    const Plan p = make_plan(h, n_max, dtype, weighted);
    hist_status st = HIST_OK;
    if (p.strategy == HIST_STRAT_LDS && p.merge == MERGE_STAGE)
        st = ensure_stage(h, stage_bytes_for(p), s, true);
    if (st == HIST_OK && p.strategy == HIST_STRAT_TILED)
        st = ensure_gbins(h, std::min<int64_t>(n_max, tiled_chunk(h)), s, true);
    if (st == HIST_OK && p.strategy == HIST_STRAT_PART) {
        const int64_t mmax = std::min<int64_t>(n_max, part_chunk(h));
        st = ensure_gbins(h, mmax, s, true);
        if (st == HIST_OK)
            st = ensure_part(h, part_layout(h, p, mmax, weighted).total(), s, true);
    }
    return st;
}

extern "C" hist_status hist_findbin(hist_t *h, const void *const *coords, int64_t n,
                                    hist_dtype dtype, int32_t *bins_dev, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_findbin: NULL handle");
    if (dtype != HIST_F64 && dtype != HIST_F32)
        return set_error(HIST_EINVAL, "hist_findbin: unknown dtype %d", (int)dtype);
    hist_status st = check_coords(h, coords, n, "hist_findbin");
    if (st != HIST_OK || n == 0)
        return st;
    if (!bins_dev)
        return set_error(HIST_EINVAL, "hist_findbin: bins_dev is NULL");
    FillArgs a = base_args(h, coords, nullptr, n);
    const int lds = apply_model_offsets(h, a);
    int blocks = (int)((n + 255) / 256);
    if (blocks > h->num_cu * 8)
        blocks = h->num_cu * 8;
    HIPCHK(launch_findbin(h->dims, dtype == HIST_F32, 256, blocks, (size_t)lds, a, bins_dev,
                          static_cast<hipStream_t>(stream)),
           "findbin launch");
    return HIST_OK;
}

// -------------------------------------------------------------- reading ----

extern "C" hist_status hist_stats(hist_t *h, double *out, int cap, int *count, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_stats: NULL handle");
    if (count)
        *count = h->S;
    if (!out || cap < h->S)
        return set_error(HIST_EINVAL, "hist_stats: need room for %d values", h->S);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (is_capturing(s))
        return set_error(HIST_ECAPTURE, "hist_stats: stream is capturing");
    HIPCHK(hipMemcpyAsync(out, h->d_stats, sizeof(double) * h->S, hipMemcpyDeviceToHost, s),
           "stats copy");
    HIPCHK(hipStreamSynchronize(s), "stats synchronize");
    return HIST_OK;
}

extern "C" hist_status hist_read(hist_t *h, double *sumw, double *sumw2, int64_t *entries,
                                 void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_read: NULL handle");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (is_capturing(s))
        return set_error(HIST_ECAPTURE, "hist_read: stream is capturing");
    if (sumw || sumw2) {
        std::vector<uint64_t> cnt((size_t)h->T);
        HIPCHK(hipMemcpyAsync(cnt.data(), h->d_cnt, sizeof(uint64_t) * h->T,
                              hipMemcpyDeviceToHost, s),
               "count copy");
        if (sumw)
            HIPCHK(hipMemcpyAsync(sumw, h->d_sumw, sizeof(double) * h->T, hipMemcpyDeviceToHost, s),
                   "sumw copy");
        if (sumw2)
            HIPCHK(hipMemcpyAsync(sumw2, h->d_sumw2, sizeof(double) * h->T,
                                  hipMemcpyDeviceToHost, s),
                   "sumw2 copy");
        HIPCHK(hipStreamSynchronize(s), "read synchronize");
        // unit-weight fills count events exactly; each counts w = w^2 = 1
        for (int64_t g = 0; g < h->T; ++g) {
            const double c = (double)cnt[(size_t)g];
            if (sumw)
                sumw[g] += c;
            if (sumw2)
                sumw2[g] += c;
        }
    } else {
        HIPCHK(hipStreamSynchronize(s), "read synchronize");
    }
    if (entries) {
        uint64_t e = 0;
        HIPCHK(hipMemcpyAsync(&e, h->d_entries, sizeof(e), hipMemcpyDeviceToHost, s), "entries copy");
        HIPCHK(hipStreamSynchronize(s), "entries synchronize");
        *entries = (int64_t)e;
    }
    return HIST_OK;
}

extern "C" hist_status hist_reset(hist_t *h, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_reset: NULL handle");
    return zero_state(h, static_cast<hipStream_t>(stream));
}

// ------------------------------------------------------- learned index ----

static int default_segments(int32_t nbins)
{
    int s = nbins / 8;
    if (s < 4)
        s = 4;
    if (s > kMaxSegments)
        s = kMaxSegments;
    return s;
}

// Key feature: the top 32 bits of the order key, cut into segments of
// 2^(20-q) units, i.e. 2^q segments per binade (power of two) of |x|, aligned
// so that every binade boundary -- where the key is not linear in x -- is a
// segment boundary.  The scale 2^(q-20) is a power of two, so t is exact.
// Picks the largest q whose segment count fits kMaxSegments.
static uint32_t host_order_key32(double x)
{
    return (uint32_t)(host_order_key(x) >> 32);
}

static void key_segments(double e0, double en, AxisDev &ax)
{
    const uint32_t k0 = host_order_key32(e0), k1 = host_order_key32(en);
    for (int q = 20; q >= -11; --q) {
        const int sh = 20 - q;   // log2 of the segment width in key units, <= 31
        const uint32_t mask = sh >= 32 ? 0xFFFFFFFFu : ((1u << sh) - 1u);
        const uint32_t k0a = k0 & ~mask;
        const uint64_t count = (uint64_t)((k1 - k0a) >> sh) + 1;
        if (count <= (uint64_t)kMaxSegments || q == -11) {
            ax.key0 = k0a;
            ax.kshift = sh;
            ax.kmask = mask;
            ax.zscale = std::ldexp(1.0f, -sh);
            ax.nseg = (int)std::min<uint64_t>(count, (uint64_t)kMaxSegments);
            ax.keypos = e0 > 0.0 ? 1 : 0;
            return;
        }
    }
}

extern "C" hist_status hist_train_index(hist_t *h, int axis, void *stream)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_train_index: NULL handle");
    if (axis < 0 || axis >= h->dims || !h->variable[axis])
        return set_error(HIST_EINVAL, "hist_train_index: axis %d is not a variable axis", axis);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (is_capturing(s))
        return set_error(HIST_ECAPTURE, "hist_train_index: stream is capturing");
    const int32_t n = h->ax[axis].nbins;
    const double e0 = h->edges_host[axis][0];
    const double en = h->edges_host[axis][(size_t)n];
    AxisDev keyax = h->ax[axis];
    key_segments(e0, en, keyax);
    int nseg_f[2] = {keyax.nseg, default_segments(n)};
    const int nseg = std::max(nseg_f[0], nseg_f[1]);

    int32_t *d_seg = nullptr;
    ModelSeg *d_model[2] = {nullptr, nullptr};
    double *d_diag = nullptr;
    hipError_t e = dalloc(&d_seg, (size_t)n + 1);
    if (e == hipSuccess)
        e = dalloc(&d_model[0], (size_t)nseg);
    if (e == hipSuccess)
        e = dalloc(&d_model[1], (size_t)nseg);
    if (e == hipSuccess)
        e = dalloc(&d_diag, (size_t)nseg * 2);
    AxisDev cand[2];
    double score[2] = {INFINITY, INFINITY}, maxw[2] = {0, 0}, meanw[2] = {0, 0};
    bool narrow[2] = {false, false};
    std::vector<double> diag((size_t)nseg * 2);
    for (int f = 0; f < 2 && e == hipSuccess; ++f) {
        AxisDev ax = f == 0 ? keyax : h->ax[axis];
        ax.kind = AX_LEARNED;
        ax.nseg = nseg_f[f];
        ax.feature = f == 0 ? FEAT_KEY : FEAT_LINEAR;
        ax.lds_model = -1;
        ax.lds_edges = -1;
        ax.x0 = e0;
        if (f == 1) {
            const double fmax = en - e0;
            ax.fscale = (std::isfinite(fmax) && fmax > 0) ? (double)ax.nseg / fmax : 0.0;
        }
        ax.model = d_model[f];
        cand[f] = ax;
        e = launch_seg_of_edges(ax, d_seg, s);
        if (e == hipSuccess)
            e = launch_fit_segments(ax, d_seg, d_model[f], d_diag, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(diag.data(), d_diag, sizeof(double) * 2 * ax.nseg,
                               hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess)
            break;
        // edge-weighted mean candidate-interval width
        double num = 0, den = 0, mx = 0, sm = 0, mxe = 0;
        for (int i = 0; i < ax.nseg; ++i) {
            const double wdt = diag[2 * i], cnt = diag[2 * i + 1] + 1.0;
            num += wdt * cnt;
            den += cnt;
            sm += wdt;
            mx = wdt > mx ? wdt : mx;
            mxe = cnt > mxe ? cnt : mxe;
        }
        // at most two candidate bins for every x: widths below 2 with room
        // for the rounding of y + w (y stays within about the segment's bins,
        // below 2^16, where an FP32 ulp is at most 2^-8)
        narrow[f] = mx < 1.99 && mxe < 65536.0;
        score[f] = den > 0 ? num / den : INFINITY;
        maxw[f] = mx;
        meanw[f] = sm / ax.nseg;
    }
    if (e != hipSuccess) {
        dfree(d_seg);
        dfree(d_model[0]);
        dfree(d_model[1]);
        dfree(d_diag);
        return hip_fail(e, "hist_train_index");
    }
    const int best = score[1] < score[0] ? 1 : 0;
    dfree(h->d_model[axis]);
    h->d_model[axis] = d_model[best];
    dfree(d_model[1 - best]);
    dfree(d_seg);
    dfree(d_diag);
    AxisDev &ax = h->ax[axis];
    ax = cand[best];
    ax.model = h->d_model[axis];
    h->trained[axis] = true;
    h->index_feature[axis] = best;
    h->index_mean_window[axis] = score[best];
    h->index_max_window[axis] = maxw[best];
    h->index_narrow[axis] = narrow[best];
    (void)meanw;
    return HIST_OK;
}

extern "C" hist_status hist_set_search(hist_t *h, int axis, hist_search mode)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_set_search: NULL handle");
    if (axis < 0 || axis >= h->dims || !h->variable[axis])
        return set_error(HIST_EINVAL, "hist_set_search: axis %d is not a variable axis", axis);
    if (mode == HIST_SEARCH_LEARNED) {
        if (!h->trained[axis])
            return set_error(HIST_EINVAL, "hist_set_search: axis %d has no trained index", axis);
        h->ax[axis].kind = AX_LEARNED;
    } else if (mode == HIST_SEARCH_BINARY) {
        h->ax[axis].kind = AX_BSEARCH;
    } else {
        return set_error(HIST_EINVAL, "hist_set_search: unknown mode %d", (int)mode);
    }
    return HIST_OK;
}

extern "C" hist_status hist_index_info(hist_t *h, int axis, int *segments, int *feature,
                                       double *mean_window, double *max_window)
{
    if (!h)
        return set_error(HIST_EINVAL, "hist_index_info: NULL handle");
    if (axis < 0 || axis >= h->dims || !h->trained[axis])
        return set_error(HIST_EINVAL, "hist_index_info: axis %d has no trained index", axis);
    if (segments)
        *segments = h->ax[axis].nseg;
    if (feature)
        *feature = h->index_feature[axis];
    if (mean_window)
        *mean_window = h->index_mean_window[axis];
    if (max_window)
        *max_window = h->index_max_window[axis];
    return HIST_OK;
}
