// kernels.h -- launch interface between the host library and the gfx950
// kernels of the histogram library.
#pragma once

#include "hist_internal.h"

namespace hg {

// LDS accumulators for the window of bins a block privatizes.
enum Acc : int32_t {
    ACC_U32 = 0,   // unit weights: 32-bit counters, `copies` interleaved copies
    ACC_U16 = 1,   // unit weights: 16-bit counters packed in pairs, drained by
                   // periodic scans so they provably never overflow
    ACC_F64 = 2,   // weights: binary64 sum and sum of squares, `copies` copies
    ACC_F32C = 3,  // FP32 weights: FP32 sums with TwoSum compensation terms
    ACC_PCOUNT = 4 // count pass of the partitioned strategy: global bins to
                   // scratch and per-bucket event counts (win_len buckets)
};

enum Merge : int32_t { MERGE_ATOMIC = 0, MERGE_STAGE = 1 };

// Out-of-window hot-bin cache: keys (u32) then values (u32 counts, or binary64
// sum and sum of squares per entry).
constexpr uint32_t kCacheEmpty = 0xFFFFFFFFu;
__host__ __device__ inline int cache_bytes(int slots, bool weighted)
{
    return slots * 4 + slots * (weighted ? 16 : 4);
}

// Bytes one bin needs in LDS for one copy.
__host__ __device__ inline int acc_bytes(int acc)
{
    return acc == ACC_U32 ? 4 : acc == ACC_U16 ? 2 : 16;
}

// Largest number of events one block may add between two drains of the
// 16-bit counters: a drain leaves every counter <= 0x0FFF, so 61440 more
// increments reach at most 0xFFFF.
constexpr int kU16EpochEvents = 61440;
constexpr int kRedBytes = 16 * kMaxStats * 8;      // per-wave statistics partials
constexpr int kMaxThreads = 1024;
constexpr int kTileUnroll = 4;

// Events each thread loads per loop iteration of the fill kernel.
// Sized so the double-buffered batch fits the 128 VGPRs a 1024-thread
// workgroup allows without spilling; kernels that dispatch on the axis kinds
// at run time (KS_MIXED, KS_STAGED) carry every kind's code and get fewer
// events.
// The partition count pass keeps only bucket counters in LDS, so two
// 1024-thread workgroups share a CU when a thread stays within 64 VGPRs
// (8 waves per SIMD): fewer events per thread, twice the waves to hide
// latency with.
constexpr int kCountWavesPerSimd = 8;

__host__ __device__ constexpr int fill_unroll(int D, bool f32, bool weighted, int acc, int ks)
{
    const bool w64 = weighted && !f32;
    if (acc == ACC_PCOUNT && ks == KS_UNIFORM)
        return D == 1 ? (w64 ? 2 : 4) : (D == 2 ? (w64 ? 1 : 2) : 1);
    if (ks == KS_MIXED)
        return (D == 2 && acc != ACC_F32C) ? 2 : 1;
    if (ks == KS_STAGED)
        return acc == ACC_F32C ? 2 : (D == 1 ? (weighted ? 4 : 6) : (D == 2 ? (weighted ? 3 : 4) : 2));
    if (acc == ACC_F32C)
        return 4;
    if (D == 1)
        return w64 ? 4 : 8;
    if (D == 2)
        return 4;
    return 2;
}

// Kernel specialization for the axis kinds of a fill.
__host__ __device__ inline int kind_set(int dims, const AxisDev *ax)
{
    bool all_uniform = true;
    for (int d = 0; d < dims; ++d)
        all_uniform = all_uniform && ax[d].kind == AX_UNIFORM;
    if (all_uniform)
        return KS_UNIFORM;
    const uint32_t staged = staged_edges_mask(dims, ax);
    bool all_staged = true;
    for (int d = 0; d < dims; ++d)
        all_staged = all_staged && (ax[d].kind == AX_UNIFORM || (staged & (1u << d)));
    if (all_staged)
        return KS_STAGED;
    if (dims == 1)
        return ax[0].kind == AX_LEARNED ? KS_LEARNED1 : KS_BSEARCH1;
    return KS_MIXED;
}

struct FillArgs {
    AxisDev ax[kMaxDims];
    const void *coords[kMaxDims];
    const void *w;            // nullptr: unit weights
    int64_t n;
    int64_t per_block;        // events per block, multiple of threads * unroll
    int32_t win_lo;           // first global bin held in LDS
    int32_t win_len;          // bins held in LDS (0: every event uses global atomics)
    int32_t copies;           // interleaved LDS copies (U32, F64, F32C)
    int32_t merge;            // Merge
    int32_t lds_win;          // byte offset of the window arrays in LDS
    int32_t epoch_iters;      // U16: loop iterations between drains
    int32_t lds_cache;        // byte offset of the out-of-window hot-bin cache, -1: none
    int32_t cache_slots;      // entries of that cache (power of two)
    uint64_t *cnt;            // [T] unit-weight counts
    double *sumw, *sumw2;     // [T] weighted sums
    double *stats;            // [S]
    uint64_t *entries;        // entry count: the workgroup that starts at event 0 adds n
    void *stage;              // staging, one slot of stage_stride units per block
    int64_t stage_stride;     // units per block: u32 words (U32; U16: four 8-bit bins a word) or bins (F64/F32C)
    int32_t *gbins;           // TILED pass 1 / PCOUNT: global bin of every event
    uint32_t *part_table;     // PCOUNT: bucket-major counts table[bucket * gridDim.x + block]
    uint32_t *part_totals;    // PCOUNT: events per bucket (added to with atomics)
    int32_t part_shift;       // PCOUNT: log2 of the bucket width
    int32_t total_bins;       // T (global bins of the histogram)
    int32_t lds_red;          // learned one-axis kernel: statistics partials
};

struct TileArgs {
    const int32_t *gbins;
    const void *w;            // nullptr: unit weights
    int64_t n;
    int64_t per_block;
    int32_t tile_len;         // bins per tile
    int32_t T;                // total bins
    int32_t copies;
    int32_t lds_win;
    int32_t epoch_iters;
    uint64_t *cnt;
    double *sumw, *sumw2;
};

// The partitioned strategy: events are counted per bucket (a range of
// 2^bshift consecutive global bins) per workgroup, the counts are scanned into
// slots, and the events are written in bucket order as in-bucket offsets.
struct PartArgs {
    uint32_t *table;          // [nbuckets * G] counts per (bucket, workgroup)
    uint32_t *totals;         // [nbuckets] events per bucket
    uint32_t *cursor;         // [nbuckets] next free slot of every bucket (scatter pass)
    uint32_t *bucket_start;   // [nbuckets + 1] first slot of every bucket, then the total
    uint32_t *chunk_start;    // [nbuckets + 1] first accumulate chunk of every bucket, then the count
    uint16_t *rec_off;        // [m] bin offset within the bucket, in bucket order
    double *rec_w;            // [m] weights in bucket order (weighted fills)
    int64_t T;                // total bins
    int32_t nbuckets;
    int32_t bshift;           // log2 of the bucket width, <= 16
    int32_t lds_buckets;      // byte offset of the per-bucket counters in LDS
    int32_t pad;
};

// Records one accumulate workgroup of the partitioned strategy takes: a bucket
// with more records is split into chunks of this many, each added in its own
// LDS copy and merged with coalesced atomics.
constexpr uint32_t kPartChunk = 65536;
// A batch's members share the accumulate launch with every other member, so
// shorter chunks balance it better (its buckets do not depend on the chunk).
constexpr uint32_t kBatchPartChunk = 32768;

// Events a scatter sub-tile sorts in LDS: longer sub-tiles give longer runs
// per bucket in the records (fewer partly written lines), bounded by the LDS
// that staging a weighted record takes.
__host__ __device__ constexpr int scatter_tile(bool weighted) { return weighted ? 4096 : 8192; }
constexpr int kScatterStagedBuckets = 2048;   // more buckets: direct scatter

// LDS bytes of the scatter pass for nbuckets buckets.
__host__ __device__ inline int part_scatter_lds(int nbuckets, bool weighted)
{
    if (nbuckets > kScatterStagedBuckets)
        return nbuckets * 4;
    return 3 * nbuckets * 4 + 64 + scatter_tile(weighted) * (weighted ? 12 : 4) + 8;
}

// Raises a kernel's dynamic LDS limit to the whole 160 KB (once per kernel).
void allow_big_lds_ptr(const void *kernel);

// Launchers (return the launch status).
hipError_t launch_fill(int dims, bool f32, int acc, bool weighted, int threads, int blocks,
                       size_t lds, const FillArgs &a, hipStream_t s);
hipError_t launch_stage_reduce(int acc, int blocks_used, const FillArgs &a, hipStream_t s);
// Launch-shape variants (fill_shape.hip): events per thread 1, 2, 4, 8 and
// statistics fused or left to separate reduction kernels.
bool fill_shape_supported(int dims, bool f32, int acc, bool weighted, int ks, int unroll);
hipError_t launch_fill_shape(int acc, bool weighted, int ks, int unroll, bool fused_stats,
                             int threads, int blocks, size_t lds, const FillArgs &a, hipStream_t s);
hipError_t launch_stats_separate(bool weighted, int ept, int num_cu, const FillArgs &a, hipStream_t s);
// The learned one-axis kernel (fill_learned.hip): unit weights, 16-bit
// window, edges in HBM.  Its LDS: the window at 0, the model, the statistics
// partials and list count, the hot-bin cache.
bool learned_lean_supported(int dims, bool f32, bool weighted, int acc, const AxisDev *ax);
// wide: the index may give intervals of three or more bins
hipError_t launch_fill_learned(int threads, int blocks, size_t lds, bool wide, const FillArgs &a, hipStream_t s);
hipError_t launch_findbin(int dims, bool f32, int threads, int blocks, size_t lds,
                          const FillArgs &a, int32_t *out, hipStream_t s);
hipError_t launch_tiled_bins(int dims, bool f32, bool weighted, int threads, int blocks,
                             size_t lds, const FillArgs &a, hipStream_t s);
hipError_t launch_tile(int acc, bool f32, int threads, int blocks_x, int tiles, size_t lds,
                       const TileArgs &t, hipStream_t s);
hipError_t launch_part_scan(const PartArgs &p, hipStream_t s);
hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s);
hipError_t launch_part_scatter(bool f32, bool weighted, int threads, int blocks, size_t lds,
                               const FillArgs &a, const PartArgs &p, hipStream_t s);
hipError_t launch_part_accum(bool weighted, int threads, int blocks, size_t lds,
                             const FillArgs &a, const PartArgs &p, hipStream_t s);
hipError_t launch_zero_u64(uint64_t *p, int64_t n, hipStream_t s);
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s);
hipError_t launch_add_u64_to_f64(double *dst, const uint64_t *src, int64_t n, hipStream_t s);

// Learned index training (learned.hip).
hipError_t launch_seg_of_edges(const AxisDev &ax, int32_t *seg, hipStream_t s);
hipError_t launch_fit_segments(const AxisDev &ax, const int32_t *seg, ModelSeg *model,
                               double *diag, hipStream_t s);

}  // namespace hg
