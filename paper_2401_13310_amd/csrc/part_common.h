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
template <typename Get, typename Put>
__device__ __forceinline__ uint32_t block_exclusive_scan(int64_t total, Get &&get, Put &&put)
{
    __shared__ uint32_t part[2][1024];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int64_t per = (total + nthr - 1) / nthr;
    const int64_t b0 = (int64_t)tid * per < total ? (int64_t)tid * per : total;
    const int64_t b1 = b0 + per < total ? b0 + per : total;
    uint32_t s = 0;
    for (int64_t i = b0; i < b1; ++i)
        s += get(i);
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
    for (int64_t i = b0; i < b1; ++i) {
        const uint32_t v = get(i);
        put(i, run);
        run += v;
    }
    const uint32_t all = part[cur][nthr - 1];
    __syncthreads();
    return all;
}

// Scan pass (one workgroup of 1024 threads).  The bucket-major count table
// table[j*G + c] becomes the first slot of range c in bucket j; bucket j holds
// slots [bucket_start[j], bucket_start[j+1]); and bucket j's records are
// cut into chunks of at most kPartChunk, numbered from chunk_start[j] (chunk
// count in chunk_start[nbuckets]).
__device__ __forceinline__ void part_scan(uint32_t *table, uint32_t *bucket_start,
                                          uint32_t *chunk_start, int nbuckets, int G)
{
    const uint32_t total = block_exclusive_scan(
        (int64_t)nbuckets * G, [&](int64_t i) { return table[i]; },
        [&](int64_t i, uint32_t v) {
            table[i] = v;
            if (i % G == 0)
                bucket_start[i / G] = v;
        });
    if (threadIdx.x == 0)
        bucket_start[nbuckets] = total;
    __syncthreads();
    const uint32_t chunks = block_exclusive_scan(
        nbuckets,
        [&](int64_t j) {
            const uint32_t r = bucket_start[j + 1] - bucket_start[j];
            return (r + kPartChunk - 1) / kPartChunk;
        },
        [&](int64_t j, uint32_t v) { chunk_start[j] = v; });
    if (threadIdx.x == 0)
        chunk_start[nbuckets] = chunks;
}

// Scatter of the events [begin, end) of range `col`: each event, in bucket
// order, gets its bin's offset in the bucket (and its weight).  `cur` is LDS
// room for nbuckets cursors.
template <typename T, bool W>
__device__ __forceinline__ void part_scatter(const int32_t *__restrict__ gbins, const T *__restrict__ w,
                                             int64_t begin, int64_t end, const uint32_t *table,
                                             int G, int col, int nbuckets, int bshift,
                                             uint16_t *__restrict__ rec_off,
                                             double *__restrict__ rec_w, uint32_t *cur)
{
    const int tid = threadIdx.x, nthr = blockDim.x;
    for (int j = tid; j < nbuckets; j += nthr)
        cur[j] = table[(int64_t)j * G + col];
    __syncthreads();
    const uint32_t mask = (1u << bshift) - 1u;
    for (int64_t i = begin + tid; i < end; i += nthr) {
        const uint32_t g = (uint32_t)gbins[i];
        const uint32_t slot =
            __hip_atomic_fetch_add(&cur[g >> bshift], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        rec_off[slot] = (uint16_t)(g & mask);
        if (W)
            rec_w[slot] = (double)__builtin_nontemporal_load(w + i);
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
                                                 double *sumw, double *sumw2, char *smem)
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
    const uint32_t r0 = b0 + c * kPartChunk;
    const uint32_t r1 = r0 + kPartChunk < b1 ? r0 + kPartChunk : b1;
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
    for (uint32_t r = r0 + tid; r < r1; r += nthr) {
        const uint32_t l = rec_off[r];
        if (W) {
            const double wv = rec_w[r];
            lds_add_f64(&s64[l], wv);
            lds_add_f64(&s64[len + l], wv * wv);
        } else {
            lds_add_u32(&c32[l], 1u);
        }
    }
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
