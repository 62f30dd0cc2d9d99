// part_common.h -- workgroup-level pieces of the partitioned strategy (see
// partition.hip), shared by single fills and batches.
//
// A histogram of T bins is cut into buckets of 2^bshift consecutive global
// bins.  G workgroups (or tiles) each own a contiguous range of events; the
// count pass leaves, in a bucket-major table, how many events of each range
// fall in each bucket.
#pragma once

#include "device_common.h"
#include "kernels.h"

namespace hg {

// Exclusive prefix sum over `total` values (one workgroup of 1024 threads):
// get(i) reads value i, put(i, prefix) stores its exclusive prefix; returns
// the sum of all values to every thread.  Each thread takes a contiguous run,
// the run sums are scanned in LDS (Hillis-Steele), then each thread rewrites
// its run.
// The run values are read kRunBatch at a time with independent loads, so a
// thread's reads overlap instead of paying one memory latency each.
constexpr int kRunBatch = 16;

template <typename Get, typename Put>
__device__ __forceinline__ uint32_t block_exclusive_scan(int64_t total, Get &&get, Put &&put)
{
    __shared__ uint32_t part[2][1024];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int64_t per = (total + nthr - 1) / nthr;
    const int64_t b0 = (int64_t)tid * per < total ? (int64_t)tid * per : total;
    const int64_t b1 = b0 + per < total ? b0 + per : total;
    uint32_t s = 0;
    for (int64_t i0 = b0; i0 < b1; i0 += kRunBatch) {
        uint32_t v[kRunBatch];
#pragma unroll
        for (int r = 0; r < kRunBatch; ++r)
            v[r] = get(i0 + r < b1 ? i0 + r : b1 - 1);
#pragma unroll
        for (int r = 0; r < kRunBatch; ++r)
            s += i0 + r < b1 ? v[r] : 0u;
    }
    __syncthreads();   // earlier users of `part` are done
    part[0][tid] = s;
    __syncthreads();
    int cur = 0;
    for (int off = 1; off < nthr; off <<= 1) {
        const uint32_t v = part[cur][tid] + (tid >= off ? part[cur][tid - off] : 0u);
        part[cur ^ 1][tid] = v;
        cur ^= 1;
        __syncthreads();
    }
    uint32_t run = part[cur][tid] - s;   // exclusive prefix of this thread's run
    for (int64_t i0 = b0; i0 < b1; i0 += kRunBatch) {
        uint32_t v[kRunBatch];
#pragma unroll
        for (int r = 0; r < kRunBatch; ++r)
            v[r] = get(i0 + r < b1 ? i0 + r : b1 - 1);
#pragma unroll
        for (int r = 0; r < kRunBatch; ++r) {
            if (i0 + r < b1) {
                put(i0 + r, run);
                run += v[r];
            }
        }
    }
    const uint32_t all = part[cur][nthr - 1];
    __syncthreads();
    return all;
}

// Exclusive prefix sum of one value per thread over the workgroup (wave
// shuffles, then the wave totals through LDS); `red` is LDS room for the wave
// totals (kMaxThreads / 64 words).  Returns the prefix; `total` gets the sum.
__device__ __forceinline__ uint32_t block_scan_excl(uint32_t v, uint32_t *red, uint32_t &total)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        const uint32_t y = __shfl_up(x, off, kWave);
        if (lane >= off)
            x += y;
    }
    if (lane == kWave - 1)
        red[wave] = x;
    __syncthreads();
    if (wave == 0) {
        uint32_t t = lane < nw ? red[lane] : 0u;
#pragma unroll
        for (int off = 1; off < kWave; off <<= 1) {
            const uint32_t y = __shfl_up(t, off, kWave);
            if (lane >= off)
                t += y;
        }
        if (lane < nw)
            red[lane] = t;
    }
    __syncthreads();
    const uint32_t before = wave ? red[wave - 1] : 0u;
    total = red[nw - 1];
    __syncthreads();
    return before + x - v;
}

// Scan pass (one workgroup of 1024 threads) over the events per bucket:
// bucket j holds slots [bucket_start[j], bucket_start[j+1]), its scatter
// cursor starts at bucket_start[j], and its records are cut into chunks of at
// most `chunk`, numbered from chunk_start[j] (chunk count in
// chunk_start[nbuckets]).
__device__ __forceinline__ void part_scan(const uint32_t *totals, uint32_t *bucket_start,
                                          uint32_t *chunk_start, uint32_t *cursor, int nbuckets,
                                          uint32_t chunk)
{
    if (nbuckets <= (int)blockDim.x) {
        // one bucket per thread: both prefix sums from one read of the totals
        __shared__ uint32_t red[16];
        const int j = threadIdx.x;
        const uint32_t t = j < nbuckets ? __hip_atomic_load(&totals[j], __ATOMIC_RELAXED,
                                                            __HIP_MEMORY_SCOPE_AGENT)
                                        : 0u;
        uint32_t all_t, all_c;
        const uint32_t bs = block_scan_excl(t, red, all_t);
        const uint32_t cs = block_scan_excl((t + chunk - 1) / chunk, red, all_c);
        if (j < nbuckets) {
            bucket_start[j] = bs;
            cursor[j] = bs;
            chunk_start[j] = cs;
        }
        if (j == 0) {
            bucket_start[nbuckets] = all_t;
            chunk_start[nbuckets] = all_c;
        }
        return;
    }
    const uint32_t total = block_exclusive_scan(
        nbuckets, [&](int64_t j) { return totals[j]; },
        [&](int64_t j, uint32_t v) {
            bucket_start[j] = v;
            cursor[j] = v;
        });
    if (threadIdx.x == 0)
        bucket_start[nbuckets] = total;
    __syncthreads();
    const uint32_t chunks = block_exclusive_scan(
        nbuckets,
        [&](int64_t j) {
            const uint32_t r = bucket_start[j + 1] - bucket_start[j];
            return (r + chunk - 1) / chunk;
        },
        [&](int64_t j, uint32_t v) { chunk_start[j] = v; });
    if (threadIdx.x == 0)
        chunk_start[nbuckets] = chunks;
}


// Scatter of the events [begin, end) of range `col`: the range reserves its
// slots in every bucket with one atomic add on the bucket's cursor (ranges
// thus take their places in a bucket in any order), then each event, in bucket
// order, gets its bin's offset in the bucket (and its weight).  With few
// buckets, sub-tiles of scatter_tile(W) events are first sorted by bucket in LDS
// (a counting sort), so the writes to each bucket leave as contiguous runs.
template <typename T, bool W>
__device__ __forceinline__ void part_scatter(const int32_t *__restrict__ gbins, const T *__restrict__ w,
                                             int64_t begin, int64_t end, const uint32_t *table,
                                             uint32_t *cursor, int G, int col, int nbuckets,
                                             int bshift, uint16_t *__restrict__ rec_off,
                                             double *__restrict__ rec_w, char *smem)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    uint32_t *cur = reinterpret_cast<uint32_t *>(smem);
    for (int j = tid; j < nbuckets; j += nthr) {
        const uint32_t c = table[(int64_t)j * G + col];
        cur[j] = c ? __hip_atomic_fetch_add(&cursor[j], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0u;
    }
    __syncthreads();
    const uint32_t mask = (1u << bshift) - 1u;
    if (nbuckets > kScatterStagedBuckets || nthr != kMaxThreads) {
        for (int64_t i = begin + tid; i < end; i += nthr) {
            const uint32_t g = (uint32_t)gbins[i];
            const uint32_t slot = __hip_atomic_fetch_add(&cur[g >> bshift], 1u, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_WORKGROUP);
            rec_off[slot] = (uint16_t)(g & mask);
            if (W)
                rec_w[slot] = (double)__builtin_nontemporal_load(w + i);
        }
        return;
    }
    uint32_t *hist = cur + nbuckets;
    uint32_t *off = hist + nbuckets;
    uint32_t *red = off + nbuckets;             // 16 words
    uint32_t *sg = red + 16;                    // staged bins
    constexpr int kTile = scatter_tile(W);
    double *sw = reinterpret_cast<double *>(smem + ((3 * nbuckets * 4 + 64 + kTile * 4 + 7) & ~7));
    constexpr int K = kTile / kMaxThreads;      // events per thread and sub-tile (nthr = 1024)
    for (int64_t t0 = begin; t0 < end; t0 += kTile) {
        const int cnt = (int)(end - t0 < kTile ? end - t0 : kTile);
        for (int j = tid; j < nbuckets; j += nthr)
            hist[j] = 0u;
        uint32_t g[K], rank[K];
        double wv[K];
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int e = tid + k * nthr;
            if (e < cnt) {
                g[k] = (uint32_t)__builtin_nontemporal_load(gbins + t0 + e);
                if (W)
                    wv[k] = (double)__builtin_nontemporal_load(w + t0 + e);
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k)
            if (tid + k * nthr < cnt)
                rank[k] = __hip_atomic_fetch_add(&hist[g[k] >> bshift], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP);
        __syncthreads();
        // bucket offsets inside the sub-tile: each thread scans two buckets
        {
            const int j0 = 2 * tid;
            const uint32_t h0 = j0 < nbuckets ? hist[j0] : 0u;
            const uint32_t h1 = j0 + 1 < nbuckets ? hist[j0 + 1] : 0u;
            uint32_t total;
            const uint32_t p = block_scan_excl(h0 + h1, red, total);
            if (j0 < nbuckets)
                off[j0] = p;
            if (j0 + 1 < nbuckets)
                off[j0 + 1] = p + h0;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < K; ++k) {
            if (tid + k * nthr < cnt) {
                const uint32_t pos = off[g[k] >> bshift] + rank[k];
                sg[pos] = g[k];
                if (W)
                    sw[pos] = wv[k];
            }
        }
        __syncthreads();
        // consecutive staged events of a bucket go to consecutive slots
        for (int e = tid; e < cnt; e += nthr) {
            const uint32_t gg = sg[e];
            const uint32_t b = gg >> bshift;
            const uint32_t slot = cur[b] + (uint32_t)e - off[b];
            rec_off[slot] = (uint16_t)(gg & mask);
            if (W)
                rec_w[slot] = sw[e];
        }
        __syncthreads();
        for (int j = tid; j < nbuckets; j += nthr)
            cur[j] += hist[j];
        __syncthreads();
    }
}

// Accumulate pass for chunk t of a histogram (chunks numbered by part_scan;
// workgroups with t past the last chunk return).  The chunk's records are
// added in LDS over its bucket's bins [g0, g0 + len); a bucket of one chunk is
// owned by this workgroup alone and is updated with plain loads and stores,
// otherwise its chunks merge with coalesced atomics.
template <bool W>
__device__ __forceinline__ void part_accum_chunk(uint32_t t, const uint32_t *bucket_start,
                                                 const uint32_t *chunk_start, int nbuckets,
                                                 int bshift, int64_t T,
                                                 const uint16_t *__restrict__ rec_off,
                                                 const double *__restrict__ rec_w, uint64_t *cnt,
                                                 double *sumw, double *sumw2, char *smem,
                                                 uint32_t chunk)
{
    if (t >= chunk_start[nbuckets])
        return;
    // bucket of chunk t: the last j with chunk_start[j] <= t (empty buckets
    // have no chunks and are skipped by the search)
    int lo = 0, hi = nbuckets - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_start[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    const int j = lo;
    const uint32_t c = t - chunk_start[j];
    const bool shared = chunk_start[j + 1] - chunk_start[j] > 1;
    const uint32_t b0 = bucket_start[j], b1 = bucket_start[j + 1];
    const uint32_t r0 = b0 + c * chunk;
    const uint32_t r1 = r0 + chunk < b1 ? r0 + chunk : b1;
    const int64_t g0 = (int64_t)j << bshift;
    const int64_t bw = (int64_t)1 << bshift;
    const int len = (int)((T - g0) < bw ? (T - g0) : bw);

    const int tid = threadIdx.x, nthr = blockDim.x;
    uint32_t *c32 = reinterpret_cast<uint32_t *>(smem);
    double *s64 = reinterpret_cast<double *>(smem);
    const int words = W ? len * 4 : len;
    for (int i = tid; i < words; i += nthr)
        c32[i] = 0u;
    __syncthreads();
    // records four at a time (8-byte loads of offsets) from the first
    // 4-aligned record; the unaligned head and the tail one at a time
    const uint32_t r0a = (r0 + 3u) & ~3u;
    const uint32_t a0 = r0a < r1 ? r0a : r1;
    const uint32_t a1 = a0 + ((r1 - a0) & ~3u);
    auto add = [&](uint32_t r, uint32_t l) {
        if (W) {
            const double wv = rec_w[r];
            lds_add_f64(&s64[l], wv);
            lds_add_f64(&s64[len + l], wv * wv);
        } else {
            lds_add_u32(&c32[l], 1u);
        }
    };
    for (uint32_t r = r0 + tid; r < a0; r += nthr)
        add(r, rec_off[r]);
    for (uint32_t r = a0 + 4u * tid; r < a1; r += 4u * nthr) {
        const uint2 q = *reinterpret_cast<const uint2 *>(rec_off + r);
        add(r, q.x & 0xFFFFu);
        add(r + 1, q.x >> 16);
        add(r + 2, q.y & 0xFFFFu);
        add(r + 3, q.y >> 16);
    }
    for (uint32_t r = a1 + tid; r < r1; r += nthr)
        add(r, rec_off[r]);
    __syncthreads();
    for (int l = tid; l < len; l += nthr) {
        if (W) {
            const double s = s64[l], s2 = s64[len + l];
            if (s != 0.0 || s2 != 0.0) {
                if (shared) {
                    gl_add_f64(&sumw[g0 + l], s);
                    gl_add_f64(&sumw2[g0 + l], s2);
                } else {
                    sumw[g0 + l] += s;
                    sumw2[g0 + l] += s2;
                }
            }
        } else if (c32[l]) {
            if (shared)
                gl_add_u64(&cnt[g0 + l], c32[l]);
            else
                cnt[g0 + l] += c32[l];
        }
    }
}

}  // namespace hg
