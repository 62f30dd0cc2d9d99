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
//               events in each bucket (2^bshift consecutive global bins);
//   2. scan:    exclusive prefix sum over the bucket-major count table, which
//               gives every workgroup its slots in every bucket;
//   3. scatter: each workgroup writes its events to its slots as 16-bit
//               in-bucket offsets (and weights);
//   4. accumulate: one workgroup per bucket adds the bucket's events in LDS
//               and adds its bins to the histogram; it alone owns them.
// Passes 1 and 3 give each workgroup the same contiguous range of events.
#include "kernels.h"
#include "part_common.h"

namespace hg {

template <int D, typename T, bool W>
__global__ void __launch_bounds__(kMaxThreads) part_count_kernel(const FillArgs A, PartArgs P)
{
    extern __shared__ __align__(16) char smem[];
    constexpr int NS = NStats<D>::v;
    const int tid = threadIdx.x, nthr = blockDim.x;
    uint32_t *cnt = reinterpret_cast<uint32_t *>(smem + P.lds_buckets);
    for (int i = tid; i < P.nbuckets; i += nthr)
        cnt[i] = 0u;
    stage_models<D>(A.ax, smem);
    __syncthreads();
    double st[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        st[k] = 0.0;
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    for (int64_t i = start + tid; i < end; i += nthr) {
        double x[D];
        int32_t g = 0;
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            x[a] = (double)__builtin_nontemporal_load(static_cast<const T *>(A.coords[a]) + i);
            const int32_t b = axis_bin(x[a], A.ax[a], smem);
            inside = inside && (uint32_t)(b - 1) < (uint32_t)A.ax[a].nbins;
            g += (a == 0) ? b : b * A.ax[a].stride;
        }
        A.gbins[i] = g;
        if (inside)
            stats_add<D>(st, x, W ? (double)static_cast<const T *>(A.w)[i] : 1.0);
        lds_add_u32(&cnt[(uint32_t)g >> P.bshift], 1u);
    }
    __syncthreads();
    for (int j = tid; j < P.nbuckets; j += nthr)
        P.table[(int64_t)j * gridDim.x + blockIdx.x] = cnt[j];
    reduce_stats<NS>(st, reinterpret_cast<double *>(smem), A.stats);
}

__global__ void __launch_bounds__(1024) part_scan_kernel(PartArgs P, int G)
{
    part_scan(P.table, P.bucket_start, P.chunk_start, P.nbuckets, G);
}

template <typename T, bool W>
__global__ void __launch_bounds__(kMaxThreads) part_scatter_kernel(const FillArgs A, PartArgs P)
{
    extern __shared__ __align__(16) char smem[];
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    part_scatter<T, W>(A.gbins, static_cast<const T *>(A.w), start, end, P.table, gridDim.x,
                       blockIdx.x, P.nbuckets, P.bshift, P.rec_off, P.rec_w,
                       reinterpret_cast<uint32_t *>(smem + P.lds_buckets));
}

template <bool W>
__global__ void __launch_bounds__(1024) part_accum_kernel(const FillArgs A, PartArgs P)
{
    extern __shared__ __align__(16) char smem[];
    part_accum_chunk<W>(blockIdx.x, P.bucket_start, P.chunk_start, P.nbuckets, P.bshift, P.T,
                        P.rec_off, P.rec_w, A.cnt, A.sumw, A.sumw2, smem);
}

// ------------------------------------------------------------------ launchers

template <int D, typename T, bool W>
static hipError_t launch_pc(int threads, int blocks, size_t lds, const FillArgs &a, const PartArgs &p,
                            hipStream_t s)
{
    auto k = part_count_kernel<D, T, W>;
    allow_big_lds_ptr(reinterpret_cast<const void *>(k));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a, p);
    return hipGetLastError();
}

hipError_t launch_part_count(int dims, bool f32, bool weighted, int threads, int blocks, size_t lds,
                             const FillArgs &a, const PartArgs &p, hipStream_t s)
{
    switch ((dims * 2 + (f32 ? 1 : 0)) * 2 + (weighted ? 1 : 0)) {
    case 4: return launch_pc<1, double, false>(threads, blocks, lds, a, p, s);
    case 5: return launch_pc<1, double, true>(threads, blocks, lds, a, p, s);
    case 6: return launch_pc<1, float, false>(threads, blocks, lds, a, p, s);
    case 7: return launch_pc<1, float, true>(threads, blocks, lds, a, p, s);
    case 8: return launch_pc<2, double, false>(threads, blocks, lds, a, p, s);
    case 9: return launch_pc<2, double, true>(threads, blocks, lds, a, p, s);
    case 10: return launch_pc<2, float, false>(threads, blocks, lds, a, p, s);
    case 11: return launch_pc<2, float, true>(threads, blocks, lds, a, p, s);
    case 12: return launch_pc<3, double, false>(threads, blocks, lds, a, p, s);
    case 13: return launch_pc<3, double, true>(threads, blocks, lds, a, p, s);
    case 14: return launch_pc<3, float, false>(threads, blocks, lds, a, p, s);
    case 15: return launch_pc<3, float, true>(threads, blocks, lds, a, p, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_part_scan(const PartArgs &p, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL(part_scan_kernel, dim3(1), dim3(1024), 0, s, p, blocks);
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
