// part_common.h -- workgroup-level pieces of the partitioned strategy (see
// partition.hip), shared by single fills and batches.
//
// A histogram of T bins is cut into buckets of 2^bshift consecutive global
// bins.  G workgroups (or tiles) each own a contiguous range of events; the
// count pass leaves, in a bucket-major table, how many events of each range
// fall in each bucket.
#pragma once

#include "device_common.h"

namespace hg {

// Exclusive prefix sum of a bucket-major count table table[j*G + c] (one
// workgroup of 1024 threads): afterwards table[j*G + c] is the first slot of
// range c in bucket j, and bucket j holds slots [bucket_start[j],
// bucket_start[j+1]).  Each thread sums a contiguous run of entries; the run
// sums are scanned in LDS (Hillis-Steele), then each thread rewrites its run.
__device__ __forceinline__ void part_scan(uint32_t *table, uint32_t *bucket_start, int nbuckets,
                                          int G)
{
    __shared__ uint32_t part[2][1024];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int64_t total = (int64_t)nbuckets * G;
    const int64_t per = (total + nthr - 1) / nthr;
    const int64_t b0 = (int64_t)tid * per < total ? (int64_t)tid * per : total;
    const int64_t b1 = b0 + per < total ? b0 + per : total;
    uint32_t s = 0;
    for (int64_t i = b0; i < b1; ++i)
        s += table[i];
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
        const uint32_t v = table[i];
        table[i] = run;
        if (i % G == 0)
            bucket_start[i / G] = run;
        run += v;
    }
    if (tid == nthr - 1)
        bucket_start[nbuckets] = part[cur][tid];
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

// Accumulation of one bucket (bins [g0, g0 + len), records [r0, r1)) in LDS,
// then added to the histogram.  The calling workgroup alone owns these bins
// during the launch, so the histogram is updated with plain loads and stores.
template <bool W>
__device__ __forceinline__ void part_accum(const uint16_t *__restrict__ rec_off,
                                           const double *__restrict__ rec_w, uint32_t r0,
                                           uint32_t r1, int64_t g0, int len, uint64_t *cnt,
                                           double *sumw, double *sumw2, char *smem)
{
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
                sumw[g0 + l] += s;
                sumw2[g0 + l] += s2;
            }
        } else if (c32[l]) {
            cnt[g0 + l] += c32[l];
        }
    }
}

}  // namespace hg
