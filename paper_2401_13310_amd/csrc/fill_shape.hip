// fill_shape.hip -- launch-shape variants of the one-axis binary64 fill.
//
// The paper's tuning study (arXiv:2401.13310 Sec. 4.3) finds that the number
// of elements each work-item reduces, and whether the statistics reductions
// are fused into one kernel or run one kernel per statistic, change the fill
// time markedly.  These variants let the autotuner and the benchmark ask the
// same questions on gfx950:
//   - the fill body with 1, 2, 4 or 8 events per thread and loop iteration
//     (the single-histogram kernel otherwise uses one count per variant);
//   - the fill without its statistics (ST = false), followed by one reduction
//     kernel per statistic that re-reads the columns (the paper's CUDA
//     layout, one transform-reduce per statistic), each with EPT events per
//     thread and iteration.
// Variants exist for one binary64 axis with unit weights (fixed-width,
// learned, or edges staged in LDS) and for fixed-width weighted fills.
#include "fill_body.h"

namespace hg {

template <int ACC, bool W, int U, int KS, bool ST>
__global__ void __launch_bounds__(kMaxThreads) fill_shape_kernel(const FillArgs A)
{
    extern __shared__ __align__(16) char smem[];
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    fill_range<1, double, ACC, W, U, KS, ST>(A, smem, start, end, blockIdx.x, gridDim.x);
}

// One statistic of a one-axis fill (K: 0 sum w, 1 sum w^2, 2 sum w x,
// 3 sum (w x) x) over the events in range, reduced per workgroup and added
// with one binary64 atomic.  Grid-stride, EPT events per thread per step.
template <int K, bool W, int EPT>
__global__ void __launch_bounds__(256) stat_kernel(const FillArgs A)
{
#pragma clang fp contract(off)
    __shared__ double red[256 / kWave];
    const double *x = static_cast<const double *>(A.coords[0]);
    const double *w = static_cast<const double *>(A.w);
    const double lo = A.ax[0].xmin, hi = A.ax[0].xmax;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * EPT;
    double acc = 0.0;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * EPT; base < A.n; base += stride) {
#pragma unroll
        for (int j = 0; j < EPT; ++j) {
            const int64_t i = base + (int64_t)j * blockDim.x + threadIdx.x;
            if (i < A.n) {
                const double xi = x[i];
                const double wi = W ? w[i] : 1.0;
                const bool in = !(xi < lo) && xi < hi;
                double t;
                if (K == 0)
                    t = wi;
                else if (K == 1)
                    t = wi * wi;
                else if (K == 2)
                    t = wi * xi;
                else
                    t = (wi * xi) * xi;
                acc += in ? t : 0.0;
            }
        }
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        acc += __shfl_xor(acc, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0)
        red[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k)
            s += red[k];
        if (s != 0.0)
            gl_add_f64(&A.stats[K], s);
    }
}

template <typename Kern>
static hipError_t launch_big(Kern k, int threads, int blocks, size_t lds, const FillArgs &a,
                             hipStream_t s)
{
    allow_big_lds_ptr(reinterpret_cast<const void *>(k));
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

template <int ACC, bool W, int KS, bool ST>
static hipError_t launch_u(int unroll, int threads, int blocks, size_t lds, const FillArgs &a,
                           hipStream_t s)
{
    switch (unroll) {
    case 1: return launch_big(fill_shape_kernel<ACC, W, 1, KS, ST>, threads, blocks, lds, a, s);
    case 2: return launch_big(fill_shape_kernel<ACC, W, 2, KS, ST>, threads, blocks, lds, a, s);
    case 4: return launch_big(fill_shape_kernel<ACC, W, 4, KS, ST>, threads, blocks, lds, a, s);
    case 8: return launch_big(fill_shape_kernel<ACC, W, 8, KS, ST>, threads, blocks, lds, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int ACC, bool W, int KS>
static hipError_t launch_st(int unroll, bool fused, int threads, int blocks, size_t lds,
                            const FillArgs &a, hipStream_t s)
{
    return fused ? launch_u<ACC, W, KS, true>(unroll, threads, blocks, lds, a, s)
                 : launch_u<ACC, W, KS, false>(unroll, threads, blocks, lds, a, s);
}

bool fill_shape_supported(int dims, bool f32, int acc, bool weighted, int ks, int unroll)
{
    if (dims != 1 || f32 || (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8))
        return false;
    if (weighted)
        return acc == ACC_F64 && ks == KS_UNIFORM;
    return (acc == ACC_U32 && (ks == KS_UNIFORM || ks == KS_STAGED)) ||
           (acc == ACC_U16 && ks == KS_LEARNED1);
}

hipError_t launch_fill_shape(int acc, bool weighted, int ks, int unroll, bool fused_stats,
                             int threads, int blocks, size_t lds, const FillArgs &a, hipStream_t s)
{
    if (weighted)
        return launch_st<ACC_F64, true, KS_UNIFORM>(unroll, fused_stats, threads, blocks, lds, a, s);
    if (acc == ACC_U16)
        return launch_st<ACC_U16, false, KS_LEARNED1>(unroll, fused_stats, threads, blocks, lds, a, s);
    if (ks == KS_STAGED)
        return launch_st<ACC_U32, false, KS_STAGED>(unroll, fused_stats, threads, blocks, lds, a, s);
    return launch_st<ACC_U32, false, KS_UNIFORM>(unroll, fused_stats, threads, blocks, lds, a, s);
}

template <bool W, int EPT>
static hipError_t launch_stats_ept(int blocks, const FillArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL((stat_kernel<0, W, EPT>), dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL((stat_kernel<1, W, EPT>), dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL((stat_kernel<2, W, EPT>), dim3(blocks), dim3(256), 0, s, a);
    hipLaunchKernelGGL((stat_kernel<3, W, EPT>), dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_stats_separate(bool weighted, int ept, int num_cu, const FillArgs &a, hipStream_t s)
{
    const int64_t per_block = 256LL * ept;
    int64_t blocks = (a.n + per_block - 1) / per_block;
    if (blocks > (int64_t)num_cu * 8)
        blocks = (int64_t)num_cu * 8;
    if (blocks < 1)
        blocks = 1;
    const int b = (int)blocks;
    switch (ept * 2 + (weighted ? 1 : 0)) {
    case 2: return launch_stats_ept<false, 1>(b, a, s);
    case 3: return launch_stats_ept<true, 1>(b, a, s);
    case 8: return launch_stats_ept<false, 4>(b, a, s);
    case 9: return launch_stats_ept<true, 4>(b, a, s);
    case 32: return launch_stats_ept<false, 16>(b, a, s);
    case 33: return launch_stats_ept<true, 16>(b, a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace hg
