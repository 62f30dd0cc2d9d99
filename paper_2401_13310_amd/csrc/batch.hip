// batch.hip -- many histograms filled by one persistent launch, replayed from
// a HIP graph.
//
// The paper leaves several histograms per event loop to future work
// (arXiv:2401.13310 Sec. 6) and finds that small kernels and launch overhead
// dominate its single-histogram GPU path (Sec. 6).  Here every member of a
// batch (its own dims, axes, event count and weights) is cut into tiles of
// events; one persistent grid takes tiles from an atomic queue in decreasing
// size order.  For each tile a workgroup privatizes the member's bins in LDS
// when they fit (else it uses global atomics), finds bins and accumulates as
// the single-histogram kernel does (Sec. 3.1 steps 1-3), and merges its LDS
// copy and statistics with atomics -- tiles of one member run concurrently on
// several CUs.  The last workgroup to finish resets the queue, so the graph
// holds a single kernel node and replays need no memset.
#include "fill_body.h"
#include "part_common.h"
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

namespace hg {

// Member accumulation beyond the LDS accumulators of kernels.h.
constexpr int kAccGlobal = -1;   // global atomics (histograms too large for LDS, few events)
constexpr int kAccPart = -2;     // partitioned: count tiles here, then scan, scatter, accumulate

struct MemberDev {
    AxisDev ax[kMaxDims];
    const void *coords[kMaxDims];
    const void *w;
    int64_t n;
    uint64_t *cnt;
    double *sumw, *sumw2, *stats;
    int32_t dims, f32, acc;       // acc: ACC_U32 / ACC_F64, kAccGlobal or kAccPart
    int32_t win_len, copies, pad;
    // kAccPart members: scratch owned by the batch (partition.hip's layout)
    int32_t *gbins;               // [n] global bin of every event
    uint16_t *rec_off;            // [n] in-bucket offsets in bucket order
    double *rec_w;                // [n] weights in bucket order (weighted members)
    uint32_t *table;              // [nbuckets * ntiles]
    uint32_t *totals;             // [nbuckets] (in the batch's totals array)
    uint32_t *cursor;             // [nbuckets]
    uint32_t *bucket_start;       // [nbuckets + 1]
    uint32_t *chunk_start;        // [nbuckets + 1]
    int64_t T;
    int32_t nbuckets, bshift, ntiles, pad2;
};

struct TileDev {
    int64_t start;
    int32_t len;
    int32_t member;
    int32_t ptile;                // kAccPart members: index of the tile within the member
    int32_t pad;
};

struct ChunkDev {
    int32_t member;
    int32_t chunk;                // accumulate chunk of the member (may be past its last)
};

// A member's fill variant: dims, input type, accumulation (unit-weight LDS
// counts, binary64 LDS sums, or the partition count pass with or without
// weights) and axis kinds.
enum BatchAcc : int32_t { BA_U32 = 0, BA_F64 = 1, BA_PCOUNT = 2, BA_PCOUNT_W = 3 };

__host__ __device__ constexpr int batch_variant(int dims, bool f32, int bacc, int ks)
{
    return (((dims - 1) * 2 + (f32 ? 1 : 0)) * 4 + bacc) * 8 + ks;
}

// The member's fill arguments are read through the constant address space:
// the pointer is wave-uniform, so every field is a scalar load that the
// compiler may hoist out of the event loop (through a generic pointer they
// would be per-lane flat loads, re-read each iteration).
using ConstFillArgs = __attribute__((address_space(4))) const FillArgs;

// Events per thread and iteration of a tile: the tile function is called,
// not inlined, and the registers the call convention reserves leave the
// multi-axis bodies less room than in the single-histogram kernel.
__host__ __device__ constexpr int batch_unroll(int D, bool f32, bool W, int ACC, int KS)
{
    // (a count tile runs at the batch kernel's occupancy, like a window tile)
    const int u = fill_unroll(D, f32, W, ACC == ACC_PCOUNT ? (W ? ACC_F64 : ACC_U32) : ACC, KS);
    const int cap = D == 2 && W && !f32 ? 3 : u;
    return u < cap ? u : cap;
}

// One tile of one member: the fill body specialized for the member's variant.
// Not inlined, so the persistent kernel stays small and each variant compiles
// on its own; the call costs nothing next to a tile of tens of thousands of
// events.
template <int D, typename T, int ACC, bool W, int KS>
__device__ __attribute__((noinline)) void batch_tile(ConstFillArgs *A, int64_t start, int64_t end,
                                                     int col, int cols)
{
    extern __shared__ __align__(16) char smem[];
    fill_range<D, T, ACC, W, batch_unroll(D, sizeof(T) == 4, W, ACC, KS), KS>(*(const FillArgs *)A, smem,
                                                                             start, end, col, cols);
}

template <int D, typename T, int KS>
__device__ __forceinline__ void batch_tile_acc(int bacc, ConstFillArgs *A, int64_t start, int64_t end,
                                               int col, int cols)
{
    switch (bacc) {
    case BA_U32: batch_tile<D, T, ACC_U32, false, KS>(A, start, end, col, cols); break;
    case BA_F64: batch_tile<D, T, ACC_F64, true, KS>(A, start, end, col, cols); break;
    case BA_PCOUNT: batch_tile<D, T, ACC_PCOUNT, false, KS>(A, start, end, col, cols); break;
    default: batch_tile<D, T, ACC_PCOUNT, true, KS>(A, start, end, col, cols); break;
    }
}

template <int D, typename T>
__device__ __forceinline__ void batch_tile_ks(int bacc, int ks, ConstFillArgs *A, int64_t start,
                                              int64_t end, int col, int cols)
{
    if (ks == KS_UNIFORM) {
        batch_tile_acc<D, T, KS_UNIFORM>(bacc, A, start, end, col, cols);
    } else if (ks == KS_STAGED) {
        batch_tile_acc<D, T, KS_STAGED>(bacc, A, start, end, col, cols);
    } else if constexpr (D == 1) {
        if (ks == KS_LEARNED1)
            batch_tile_acc<D, T, KS_LEARNED1>(bacc, A, start, end, col, cols);
        else
            batch_tile_acc<D, T, KS_BSEARCH1>(bacc, A, start, end, col, cols);
    } else {
        batch_tile_acc<D, T, KS_MIXED>(bacc, A, start, end, col, cols);
    }
}

__global__ void __launch_bounds__(kMaxThreads)
batch_kernel(const MemberDev *__restrict__ members, const FillArgs *__restrict__ fargs,
             const int32_t *__restrict__ variants, const TileDev *__restrict__ tiles, int ntiles,
             uint32_t *queue)
{
    __shared__ int s_tile;
    const int tid = threadIdx.x;
    for (;;) {
        if (tid == 0)
            s_tile = (int)__hip_atomic_fetch_add(&queue[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        const int t = __builtin_amdgcn_readfirstlane(s_tile);
        __syncthreads();
        if (t >= ntiles)
            break;
        const TileDev tile = tiles[t];
        const int m = __builtin_amdgcn_readfirstlane(tile.member);
        const int v = __builtin_amdgcn_readfirstlane(variants[m]);
        ConstFillArgs *A = (ConstFillArgs *)(fargs + m);
        const int ks = v & 7, bacc = (v >> 3) & 3, dt = v >> 5;
        const int col = tile.ptile, cols = members[m].ntiles;
        const int64_t start = tile.start, end = tile.start + tile.len;
        switch (dt) {
        case 0: batch_tile_ks<1, double>(bacc, ks, A, start, end, col, cols); break;
        case 1: batch_tile_ks<1, float>(bacc, ks, A, start, end, col, cols); break;
        case 2: batch_tile_ks<2, double>(bacc, ks, A, start, end, col, cols); break;
        case 3: batch_tile_ks<2, float>(bacc, ks, A, start, end, col, cols); break;
        case 4: batch_tile_ks<3, double>(bacc, ks, A, start, end, col, cols); break;
        default: batch_tile_ks<3, float>(bacc, ks, A, start, end, col, cols); break;
        }
        __syncthreads();   // the tile's window merge is done before the next tile zeroes it
    }
    // Every workgroup has drawn past the last tile before it counts itself
    // done, so the last one can reset the queue for the next launch.
    if (tid == 0) {
        const uint32_t d = __hip_atomic_fetch_add(&queue[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (d == gridDim.x - 1) {
            __hip_atomic_store(&queue[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&queue[1], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

// Scan, scatter and accumulate passes over the kAccPart members of a batch
// (one workgroup per member, per member tile, per member bucket).  Members are
// read through the constant address space, so their pointers are known to be
// global (global, not flat, loads and stores).
using ConstMember = __attribute__((address_space(4))) const MemberDev;
__global__ void __launch_bounds__(1024)
batch_part_scan_kernel(const MemberDev *__restrict__ members, const int32_t *__restrict__ part_members)
{
    ConstMember &M = *(ConstMember *)(members + part_members[blockIdx.x]);
    part_scan(M.totals, M.bucket_start, M.chunk_start, M.cursor, M.nbuckets, kBatchPartChunk);
}

__global__ void __launch_bounds__(kMaxThreads)
batch_part_scatter_kernel(const MemberDev *__restrict__ members, const TileDev *__restrict__ ptiles,
                          uint32_t *totals, int ntotals)
{
    extern __shared__ __align__(16) char smem[];
    // the scan has read every member's bucket totals: clear them for the next
    // replay's count tiles (the batch starts with them zero)
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j < ntotals; j += blockDim.x)
            totals[j] = 0u;
    const TileDev tile = ptiles[blockIdx.x];
    ConstMember &M = *(ConstMember *)(members + tile.member);
    const int64_t end = tile.start + tile.len;
    if (!M.w)
        part_scatter<double, false>(M.gbins, nullptr, tile.start, end, M.table, M.cursor, M.ntiles,
                                    tile.ptile, M.nbuckets, M.bshift, M.rec_off, M.rec_w, smem);
    else if (M.f32)
        part_scatter<float, true>(M.gbins, static_cast<const float *>(M.w), tile.start, end, M.table,
                                  M.cursor, M.ntiles, tile.ptile, M.nbuckets, M.bshift, M.rec_off,
                                  M.rec_w, smem);
    else
        part_scatter<double, true>(M.gbins, static_cast<const double *>(M.w), tile.start, end,
                                   M.table, M.cursor, M.ntiles, tile.ptile, M.nbuckets, M.bshift,
                                   M.rec_off, M.rec_w, smem);
}

__global__ void __launch_bounds__(1024)
batch_part_accum_kernel(const MemberDev *__restrict__ members, const ChunkDev *__restrict__ chunks)
{
    extern __shared__ __align__(16) char smem[];
    const ChunkDev ck = chunks[blockIdx.x];
    ConstMember &M = *(ConstMember *)(members + ck.member);
    if (M.w)
        part_accum_chunk<true>(ck.chunk, M.bucket_start, M.chunk_start, M.nbuckets, M.bshift, M.T,
                               M.rec_off, M.rec_w, M.cnt, M.sumw, M.sumw2, smem, kBatchPartChunk);
    else
        part_accum_chunk<false>(ck.chunk, M.bucket_start, M.chunk_start, M.nbuckets, M.bshift, M.T,
                                M.rec_off, M.rec_w, M.cnt, M.sumw, M.sumw2, smem, kBatchPartChunk);
}

__global__ void zero_u32_kernel(uint32_t *p, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x)
        p[i] = 0u;
}

}  // namespace hg

using namespace hg;

struct hist_batch_s {
    int k = 0;
    std::vector<hist_t *> hs;
    std::vector<int64_t> n;
    MemberDev *d_members = nullptr;
    FillArgs *d_fargs = nullptr;
    int32_t *d_variants = nullptr;
    TileDev *d_tiles = nullptr;
    uint32_t *d_queue = nullptr;
    int ntiles = 0;
    int blocks = 1, threads = 1024;
    int lds = 0, lds_win = 0;
    // partitioned members
    int npart = 0, nptiles = 0, nchunks = 0;
    int32_t *d_part_members = nullptr;
    TileDev *d_ptiles = nullptr;
    ChunkDev *d_chunks = nullptr;
    void *d_part = nullptr;
    uint32_t *d_totals = nullptr;                 // bucket totals of every partitioned member
    int64_t ntotals = 0;
    int scatter_lds = 0, accum_lds = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

static void batch_free(hist_batch_s *b)
{
    if (!b)
        return;
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    if (b->cap_stream)
        (void)hipStreamDestroy(b->cap_stream);
    if (b->d_members)
        (void)hipFree(b->d_members);
    if (b->d_fargs)
        (void)hipFree(b->d_fargs);
    if (b->d_variants)
        (void)hipFree(b->d_variants);
    if (b->d_tiles)
        (void)hipFree(b->d_tiles);
    if (b->d_queue)
        (void)hipFree(b->d_queue);
    if (b->d_part_members)
        (void)hipFree(b->d_part_members);
    if (b->d_ptiles)
        (void)hipFree(b->d_ptiles);
    if (b->d_chunks)
        (void)hipFree(b->d_chunks);
    if (b->d_part)
        (void)hipFree(b->d_part);
    if (b->d_totals)
        (void)hipFree(b->d_totals);
    delete b;
}

static hipError_t batch_enqueue(hist_batch_s *b, hipStream_t s)
{
    hipLaunchKernelGGL(batch_kernel, dim3(b->blocks), dim3(b->threads), (size_t)b->lds, s,
                       b->d_members, b->d_fargs, b->d_variants, b->d_tiles, b->ntiles, b->d_queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || b->npart == 0)
        return e;
    hipLaunchKernelGGL(batch_part_scan_kernel, dim3(b->npart), dim3(1024), 0, s, b->d_members,
                       b->d_part_members);
    hipLaunchKernelGGL(batch_part_scatter_kernel, dim3(b->nptiles), dim3(1024), (size_t)b->scatter_lds,
                       s, b->d_members, b->d_ptiles, b->d_totals, (int)b->ntotals);
    hipLaunchKernelGGL(batch_part_accum_kernel, dim3(b->nchunks), dim3(1024), (size_t)b->accum_lds,
                       s, b->d_members, b->d_chunks);
    return hipGetLastError();
}

extern "C" hist_status hist_batch_create(int k, hist_t *const *hs, const hist_fill_desc *descs,
                                         hist_batch_t **out, void *stream)
{
    if (!out)
        return set_error(HIST_EINVAL, "hist_batch_create: out is NULL");
    *out = nullptr;
    if (k < 1 || !hs || !descs)
        return set_error(HIST_EINVAL, "hist_batch_create: need k >= 1 handles and descriptors");
    for (int i = 0; i < k; ++i) {
        if (!hs[i])
            return set_error(HIST_EINVAL, "hist_batch_create: handle %d is NULL", i);
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i])
                return set_error(HIST_EINVAL, "hist_batch_create: handle %d repeats %d", i, j);
        const hist_fill_desc &d = descs[i];
        if (d.n < 0 || (d.dtype != HIST_F64 && d.dtype != HIST_F32))
            return set_error(HIST_EINVAL, "hist_batch_create: member %d: bad n or dtype", i);
        if (d.n > 0x7FFFFFFFll * 64)
            return set_error(HIST_EINVAL, "hist_batch_create: member %d: too many events", i);
        for (int a = 0; a < hs[i]->dims && d.n > 0; ++a)
            if (!d.coords[a])
                return set_error(HIST_EINVAL, "hist_batch_create: member %d: coordinate %d is NULL", i, a);
    }
    hipStream_t s = static_cast<hipStream_t>(stream);
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
        return set_error(HIST_ECAPTURE, "hist_batch_create: stream is capturing");

    hist_batch_s *b = new (std::nothrow) hist_batch_s();
    if (!b)
        return set_error(HIST_ENOMEM, "hist_batch_create: host allocation");
    b->k = k;
    b->hs.assign(hs, hs + k);
    const hist_s *h0 = hs[0];

    // LDS budget: statistics partials, then the largest set of staged models,
    // then the window of bins
    int axes_end = kRedBytes;
    for (int i = 0; i < k; ++i) {
        AxisDev ax[kMaxDims];
        std::memcpy(ax, hs[i]->ax, sizeof(ax));
        axes_end = std::max(axes_end, lds_axis_layout(hs[i]->dims, ax, kRedBytes));
    }
    b->lds_win = (axes_end + 15) & ~15;
    const int avail = h0->lds_max - b->lds_win - 64;   // room for the kernel's static LDS

    std::vector<MemberDev> mem((size_t)k);
    std::vector<FillArgs> fargs((size_t)k);
    std::vector<int32_t> variants((size_t)k);
    std::vector<TileDev> tiles, ptiles;
    std::vector<int32_t> part_members;
    std::vector<ChunkDev> chunks;
    std::vector<size_t> part_off((size_t)k, 0);   // scratch offsets of kAccPart members
    std::vector<int64_t> tot_off((size_t)k, 0);   // offsets in the totals array
    size_t part_bytes = 0;
    auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
    // Tile sizes: a tile runs on one workgroup, so members whose events are
    // latency-bound (searches, global atomics) need many tiles to spread over
    // the CUs; LDS members get enough events per tile to amortize the zeroing
    // and merging of their window.
    constexpr int64_t kPartTile = 65536;          // events per count / scatter tile
    constexpr int64_t kPartMinEvents = 4096;      // fewer events: global atomics
    // more events: global atomics too -- a partitioned member's slots, bucket
    // starts and cursors are 32-bit words over all of its events (a single
    // fill splits such inputs into chunks of the same size instead)
    constexpr int64_t kPartMaxEvents = (int64_t)1 << 25;
    int max_window_bytes = 0;
    for (int i = 0; i < k; ++i) {
        hist_s *h = hs[i];
        const hist_fill_desc &d = descs[i];
        MemberDev &m = mem[(size_t)i];
        std::memset(&m, 0, sizeof(m));
        for (int a = 0; a < kMaxDims; ++a) {
            m.ax[a] = h->ax[a];
            m.coords[a] = a < h->dims ? d.coords[a] : nullptr;
        }
        lds_axis_layout(h->dims, m.ax, kRedBytes);
        m.w = d.weights;
        m.n = d.n;
        m.cnt = h->d_cnt;
        m.sumw = h->d_sumw;
        m.sumw2 = h->d_sumw2;
        m.stats = h->d_stats;
        m.dims = h->dims;
        m.f32 = d.dtype == HIST_F32 ? 1 : 0;
        const int bytes = d.weights ? 16 : 4;
        m.T = h->T;
        m.copies = 1;
        // bucket width of a partitioned member: the bucket fits LDS in the
        // accumulate pass, the bucket counters fit the window room
        int pbits = d.weights ? 12 : 13;
        while (pbits < 16 && ((h->T + ((int64_t)1 << pbits) - 1) >> pbits) * 4 > avail)
            ++pbits;
        const int64_t pnb = (h->T + ((int64_t)1 << pbits) - 1) >> pbits;
        const bool part_ok = ((int64_t)bytes << pbits) <= h0->lds_max && pnb * 4 <= avail;
        // the member's fill arguments: every tile runs the fill body on them
        FillArgs &fa = fargs[(size_t)i];
        std::memset(&fa, 0, sizeof(fa));
        for (int a = 0; a < kMaxDims; ++a) {
            fa.ax[a] = m.ax[a];
            fa.coords[a] = m.coords[a];
        }
        fa.w = d.weights;
        fa.n = d.n;
        fa.cnt = m.cnt;
        fa.sumw = m.sumw;
        fa.sumw2 = m.sumw2;
        fa.stats = m.stats;
        fa.entries = h->d_entries;
        fa.lds_win = b->lds_win;
        fa.lds_cache = -1;
        fa.total_bins = (int32_t)h->T;
        fa.merge = MERGE_ATOMIC;
        fa.epoch_iters = 1;
        fa.copies = 1;
        const int ks = kind_set(h->dims, h->ax);
        int bacc = d.weights ? BA_F64 : BA_U32;
        // a plan hist_tune chose for this handle's shape decides between LDS,
        // partitioned and global accumulation, and the LDS copies
        PlanChoice tc;
        const bool tuned = tuned_choice(h, d.weights != nullptr, d.dtype == HIST_F32, tc);
        const bool tuned_global = tuned && tc.strategy == HIST_STRAT_GLOBAL;
        const bool tuned_part = tuned && tc.strategy == HIST_STRAT_PART;
        if (h->T * bytes <= avail && !tuned_global && !tuned_part) {
            m.acc = d.weights ? ACC_F64 : ACC_U32;
            m.win_len = (int32_t)h->T;
            // interleaved copies for small histograms, within 32 KB so the
            // per-tile zeroing and merge stay small next to the tile
            const int64_t fit = std::min<int64_t>(avail, 32768) / (h->T * bytes);
            m.copies = (int32_t)std::min<int64_t>(64, std::max<int64_t>(1, fit));
            if (tuned && tc.copies > 0)
                m.copies = (int32_t)std::min<int64_t>(std::max<int64_t>(1, avail / (h->T * bytes)),
                                                      tc.copies);
            fa.win_len = m.win_len;
            fa.copies = m.copies;
            max_window_bytes = std::max(max_window_bytes, (int)(h->T * bytes * m.copies));
        } else if (part_ok && d.n >= kPartMinEvents && d.n <= kPartMaxEvents && !tuned_global) {
            bacc = d.weights ? BA_PCOUNT_W : BA_PCOUNT;
            m.acc = kAccPart;
            m.bshift = pbits;
            m.nbuckets = (int32_t)pnb;
            m.ntiles = (int32_t)((d.n + kPartTile - 1) / kPartTile);
            max_window_bytes = std::max(max_window_bytes, (int)(pnb * 4));
            b->scatter_lds = std::max(b->scatter_lds, part_scatter_lds((int)pnb, d.weights != nullptr));
            b->accum_lds = std::max(b->accum_lds, bytes << pbits);
            part_off[(size_t)i] = part_bytes;
            part_bytes += up((size_t)d.n * 4) + up((size_t)d.n * 2) +
                          (d.weights ? up((size_t)d.n * 8) : 0) +
                          up((size_t)pnb * m.ntiles * 4) + 3 * up((size_t)(pnb + 1) * 4);
            tot_off[(size_t)i] = b->ntotals;
            b->ntotals += pnb;
            part_members.push_back(i);
            // every bucket has at most ceil(records / kBatchPartChunk) chunks
            const int64_t cmax = pnb + (d.n + kBatchPartChunk - 1) / kBatchPartChunk;
            for (int64_t t = 0; t < cmax; ++t)
                chunks.push_back(ChunkDev{i, (int32_t)t});
            fa.win_len = m.nbuckets;
            fa.part_shift = m.bshift;
        } else {
            m.acc = kAccGlobal;
            m.win_len = 0;
        }
        variants[(size_t)i] = batch_variant(h->dims, d.dtype == HIST_F32, bacc, ks);
        b->n.push_back(d.n);
        if (m.acc == kAccPart) {
            for (int32_t t = 0; t < m.ntiles; ++t) {
                const int64_t s0 = (int64_t)t * kPartTile;
                const int64_t s1 = std::min<int64_t>(d.n, s0 + kPartTile);
                const TileDev td{s0, (int32_t)(s1 - s0), i, t, 0};
                tiles.push_back(td);
                ptiles.push_back(td);
            }
            continue;
        }
        // tiles: LDS members get enough events per tile to amortize the
        // zeroing and merging of their window
        const int64_t tile_len =
            m.acc >= 0 ? std::max<int64_t>(65536, 8 * (int64_t)m.win_len * m.copies) : 16384;
        const int64_t nt = (d.n + tile_len - 1) / tile_len;
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t s0 = d.n * t / nt, s1 = d.n * (t + 1) / nt;
            if (s1 > s0)
                tiles.push_back(TileDev{s0, (int32_t)(s1 - s0), i, 0, 0});
        }
    }
    b->npart = (int)part_members.size();
    b->nptiles = (int)ptiles.size();
    b->nchunks = (int)chunks.size();
    std::stable_sort(tiles.begin(), tiles.end(),
                     [](const TileDev &x, const TileDev &y) { return x.len > y.len; });
    b->ntiles = (int)tiles.size();
    b->lds = b->lds_win + max_window_bytes;
    b->threads = 1024;
    const int bpc = b->lds * 2 <= h0->lds_max ? 2 : 1;
    b->blocks = std::max(1, std::min(h0->num_cu * bpc, std::max(1, b->ntiles)));

    hipError_t e = hipSuccess;
    if (b->npart > 0) {
        e = hipMalloc(&b->d_part, part_bytes);
        if (e == hipSuccess)
            e = hipMalloc(&b->d_totals, sizeof(uint32_t) * (size_t)b->ntotals);
        if (e == hipSuccess)
            e = hipMemset(b->d_totals, 0, sizeof(uint32_t) * (size_t)b->ntotals);
        if (e == hipSuccess)
            e = hipMalloc(&b->d_part_members, sizeof(int32_t) * part_members.size());
        if (e == hipSuccess)
            e = hipMalloc(&b->d_ptiles, sizeof(TileDev) * ptiles.size());
        if (e == hipSuccess)
            e = hipMalloc(&b->d_chunks, sizeof(ChunkDev) * chunks.size());
        if (e == hipSuccess)
            e = hipMemcpy(b->d_part_members, part_members.data(), sizeof(int32_t) * part_members.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_ptiles, ptiles.data(), sizeof(TileDev) * ptiles.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess)
            e = hipMemcpy(b->d_chunks, chunks.data(), sizeof(ChunkDev) * chunks.size(),
                          hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            for (int i : part_members) {
                MemberDev &m = mem[(size_t)i];
                const size_t nn = (size_t)m.n;
                char *q = static_cast<char *>(b->d_part) + part_off[(size_t)i];
                m.gbins = reinterpret_cast<int32_t *>(q);
                q += up(nn * 4);
                m.rec_off = reinterpret_cast<uint16_t *>(q);
                q += up(nn * 2);
                if (m.w) {
                    m.rec_w = reinterpret_cast<double *>(q);
                    q += up(nn * 8);
                }
                m.table = reinterpret_cast<uint32_t *>(q);
                q += up((size_t)m.nbuckets * m.ntiles * 4);
                m.bucket_start = reinterpret_cast<uint32_t *>(q);
                q += up((size_t)(m.nbuckets + 1) * 4);
                m.chunk_start = reinterpret_cast<uint32_t *>(q);
                q += up((size_t)(m.nbuckets + 1) * 4);
                m.cursor = reinterpret_cast<uint32_t *>(q);
                m.totals = b->d_totals + tot_off[(size_t)i];
                fargs[(size_t)i].gbins = m.gbins;
                fargs[(size_t)i].part_table = m.table;
                fargs[(size_t)i].part_totals = m.totals;
            }
        }
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(batch_part_scatter_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, h0->lds_max);
        if (e == hipSuccess)
            e = hipFuncSetAttribute(reinterpret_cast<const void *>(batch_part_accum_kernel),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, h0->lds_max);
    }
    if (e == hipSuccess)
        e = hipMalloc(&b->d_members, sizeof(MemberDev) * (size_t)k);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_fargs, sizeof(FillArgs) * (size_t)k);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_variants, sizeof(int32_t) * (size_t)k);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_fargs, fargs.data(), sizeof(FillArgs) * (size_t)k, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMemcpy(b->d_variants, variants.data(), sizeof(int32_t) * (size_t)k, hipMemcpyHostToDevice);
    if (e == hipSuccess)
        e = hipMalloc(&b->d_tiles, sizeof(TileDev) * std::max<size_t>(1, tiles.size()));
    if (e == hipSuccess)
        e = hipMalloc(&b->d_queue, 2 * sizeof(uint32_t));
    if (e == hipSuccess)
        e = hipMemcpy(b->d_members, mem.data(), sizeof(MemberDev) * (size_t)k, hipMemcpyHostToDevice);
    if (e == hipSuccess && !tiles.empty())
        e = hipMemcpy(b->d_tiles, tiles.data(), sizeof(TileDev) * tiles.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, b->d_queue, 2);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipStreamSynchronize(s);
    if (e == hipSuccess)
        e = hipFuncSetAttribute(reinterpret_cast<const void *>(batch_kernel),
                                hipFuncAttributeMaxDynamicSharedMemorySize, h0->lds_max - 64);
    // capture one launch into a graph on a private stream
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = batch_enqueue(b, b->cap_stream);
        e = hipStreamEndCapture(b->cap_stream, &b->graph);
        if (le != hipSuccess)
            e = le;
    }
    if (e == hipSuccess)
        e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        batch_free(b);
        return set_error(e == hipErrorOutOfMemory ? HIST_ENOMEM : HIST_EDEVICE,
                         "hist_batch_create: %s", hipGetErrorString(e));
    }
    for (hist_t *h : b->hs)
        ++h->users;
    *out = b;
    return HIST_OK;
}

extern "C" hist_status hist_batch_launch(hist_batch_t *b, void *stream)
{
    if (!b)
        return set_error(HIST_EINVAL, "hist_batch_launch: NULL batch");
    if (b->ntiles > 0) {
        hipError_t e = hipGraphLaunch(b->exec, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(HIST_EDEVICE, "hist_batch_launch: %s", hipGetErrorString(e));
        }
    }
    return HIST_OK;
}

extern "C" hist_status hist_batch_launch_eager(hist_batch_t *b, void *stream)
{
    if (!b)
        return set_error(HIST_EINVAL, "hist_batch_launch_eager: NULL batch");
    if (b->ntiles > 0) {
        hipError_t e = batch_enqueue(b, static_cast<hipStream_t>(stream));
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return set_error(HIST_EDEVICE, "hist_batch_launch_eager: %s", hipGetErrorString(e));
        }
    }
    return HIST_OK;
}

extern "C" hist_status hist_batch_destroy(hist_batch_t *b)
{
    if (!b)
        return HIST_OK;
    (void)hipDeviceSynchronize();
    for (hist_t *h : b->hs)
        --h->users;
    batch_free(b);
    return HIST_OK;
}
