// partition.hip -- the partitioned strategy for histograms far larger than LDS.
//
// When the bins cannot be privatized per workgroup (a million bins, a few
// events per bin), the two-stage fill of arXiv:2401.13310 Sec. 3.2 (per-block
// shared-memory copies merged into the global histogram) would merge more bins
// than it accumulates, and global atomics are bound by the L2 atomic rate, not
// by HBM.  A fill of m events is done in four passes instead, with no atomics
// on the histogram at all:
//   1. count:   the global bin of every event (Sec. 3.1, step 1) into a
//               scratch array, the statistics, and per-workgroup counts of the
//               events in each bucket (2^bshift consecutive global bins) --
//               the fill kernel in its ACC_PCOUNT mode (fill.hip);
//   2. scan:    exclusive prefix sum over the bucket-major count table, which
//               gives every workgroup its slots in every bucket;
//   3. scatter: each workgroup writes its events to its slots as 16-bit
//               in-bucket offsets (and weights);
//   4. accumulate: one workgroup per chunk of at most kPartChunk records of
//               a bucket adds them in LDS; a bucket of one chunk is owned by
//               its workgroup and written with plain stores, the chunks of a
//               larger bucket merge with coalesced atomics.
// Passes 1 and 3 give each workgroup the same contiguous range of events.
#include "kernels.h"
#include "part_common.h"

namespace hg {

__global__ void __launch_bounds__(1024) part_scan_kernel(PartArgs P)
{
    part_scan(P.totals, P.bucket_start, P.chunk_start, P.cursor, P.nbuckets, kPartChunk);
}

// Unit weights: 64 VGPRs, so two workgroups share a CU and one's barriers
// overlap the other's loads and stores.
template <typename T, bool W>
__global__ void __launch_bounds__(kMaxThreads, W ? 4 : 8) part_scatter_kernel(const FillArgs A, PartArgs P)
{
    extern __shared__ __align__(16) char smem[];
    // the scan has read the bucket totals: clear them for the next count pass
    // (so no separate clearing launch precedes it)
    if (blockIdx.x == 0)
        for (int j = threadIdx.x; j < P.nbuckets; j += blockDim.x)
            P.totals[j] = 0u;
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    part_scatter<T, W>(A.gbins, static_cast<const T *>(A.w), start, end, P.table, P.cursor,
                       gridDim.x, blockIdx.x, P.nbuckets, P.bshift, P.rec_off, P.rec_w, smem);
}

template <bool W>
__global__ void __launch_bounds__(1024) part_accum_kernel(const FillArgs A, PartArgs P)
{
    extern __shared__ __align__(16) char smem[];
    part_accum_chunk<W>(blockIdx.x, P.bucket_start, P.chunk_start, P.nbuckets, P.bshift, P.T,
                        P.rec_off, P.rec_w, A.cnt, A.sumw, A.sumw2, smem, kPartChunk);
}

// ------------------------------------------------------------------ launchers

hipError_t launch_part_scan(const PartArgs &p, hipStream_t s)
{
    hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, s, p);
    return hipGetLastError();
}

__global__ void zero_u32_grid_kernel(uint32_t *p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

hipError_t launch_zero_u32(uint32_t *p, int64_t n, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    int blocks = (int)((n + 255) / 256);
    if (blocks > 1024)
        blocks = 1024;
    hipLaunchKernelGGL(zero_u32_grid_kernel, dim3(blocks), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

template <typename T, bool W>
static hipError_t launch_ps(int threads, int blocks, size_t lds, const FillArgs &a, const PartArgs &p,
                            hipStream_t s)
{
    auto k = part_scatter_kernel<T, W>;
    allow_big_lds_ptr(reinterpret_cast<const void *>(k));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a, p);
    return hipGetLastError();
}

hipError_t launch_part_scatter(bool f32, bool weighted, int threads, int blocks, size_t lds,
                               const FillArgs &a, const PartArgs &p, hipStream_t s)
{
    if (!weighted)
        return launch_ps<double, false>(threads, blocks, lds, a, p, s);
    if (f32)
        return launch_ps<float, true>(threads, blocks, lds, a, p, s);
    return launch_ps<double, true>(threads, blocks, lds, a, p, s);
}

hipError_t launch_part_accum(bool weighted, int threads, int blocks, size_t lds,
                             const FillArgs &a, const PartArgs &p, hipStream_t s)
{
    if (weighted) {
        auto k = part_accum_kernel<true>;
        allow_big_lds_ptr(reinterpret_cast<const void *>(k));
        hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a, p);
    } else {
        auto k = part_accum_kernel<false>;
        allow_big_lds_ptr(reinterpret_cast<const void *>(k));
        hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a, p);
    }
    return hipGetLastError();
}

}  // namespace hg
