// device_common.h -- device helpers shared by the fill and batch kernels:
// LDS and global atomics, the compensated-sum error term, and the statistics
// sums of arXiv:2401.13310 Sec. 3.2 with their workgroup reduction.
#pragma once

#include "hist_internal.h"

namespace hg {

template <int D>
struct NStats {
    static constexpr int v = 2 + 2 * D + D * (D - 1) / 2;
};

__device__ __forceinline__ void lds_add_u32(uint32_t *p, uint32_t v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add_f64(double *p, double v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void gl_add_u64(uint64_t *p, uint64_t v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gl_add_f64(double *p, double v)
{
    unsafeAtomicAdd(p, v);
}

// Exact rounding error of fl(a + b) (Knuth's TwoSum).  The sum is formed here,
// with contraction off, so it is the same rounded value the LDS atomic stored
// (a product feeding b must not be fused into it).
__device__ __forceinline__ float two_sum_err(float a, float b)
{
#pragma clang fp contract(off)
    float s = a + b;
    float bp = s - a;
    float ap = s - bp;
    return (a - ap) + (b - bp);
}

// Compensated FP32 addition of v (plus an exact extra error term) into a
// (sum, compensation) pair kept as one 64-bit LDS word, sum in the low half:
// sum' = fl(sum + v), comp' = fl(comp + (err(sum + v) + extra)), with the
// TwoSum error err.  `old` is the pair as last read; a compare-and-swap makes
// the pair update atomic and is retried with the word it found when another
// lane changed the pair first.
__device__ __forceinline__ void lds_add_compensated(uint64_t *p, uint64_t old, float v, float extra)
{
#pragma clang fp contract(off)
    for (;;) {
        const float s = __uint_as_float((uint32_t)old);
        const float c = __uint_as_float((uint32_t)(old >> 32));
        const float ns = s + v;
        const float nc = c + (two_sum_err(s, v) + extra);
        const uint64_t nw = (uint64_t)__float_as_uint(ns) | ((uint64_t)__float_as_uint(nc) << 32);
        uint64_t expected = old;
        if (__hip_atomic_compare_exchange_strong(p, &expected, nw, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_WORKGROUP))
            return;
        old = expected;
    }
}

// Per-event statistics terms, rounded in the order w, w*w, w*x, (w*x)*x,
// (w*x_c)*x_a -- the same products the reference definition forms.
template <int D>
__device__ __forceinline__ void stats_add(double (&st)[NStats<D>::v], const double (&x)[D],
                                          double w)
{
#pragma clang fp contract(off)
    st[0] += w;
    st[1] += w * w;
    int k = 2;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        const double wx = w * x[a];
        st[k++] += wx;
        st[k++] += wx * x[a];
#pragma unroll
        for (int c = 0; c < a; ++c)
            st[k++] += (w * x[c]) * x[a];
    }
}

// The same terms for unit weights, except w and w*w (the caller counts the
// events): w*x = x and (w*x)*x = x*x exactly.
template <int D>
__device__ __forceinline__ void stats_add_unit(double (&st)[NStats<D>::v], const double (&x)[D])
{
#pragma clang fp contract(off)
    int k = 2;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        st[k++] += x[a];
        st[k++] += x[a] * x[a];
#pragma unroll
        for (int c = 0; c < a; ++c)
            st[k++] += x[c] * x[a];
    }
}

// Block reduction of the statistics partials, then one binary64 atomic per
// statistic per workgroup (sums accumulate across fills).
template <int NS>
__device__ __forceinline__ void reduce_stats(double (&st)[NS], double *red, double *out)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        double v = st[k];
#pragma unroll
        for (int off = kWave / 2; off > 0; off >>= 1)
            v += __shfl_xor(v, off, kWave);
        st[k] = v;
    }
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NS; ++k)
            red[wave * NS + k] = st[k];
    }
    __syncthreads();
    if (threadIdx.x < NS) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w)
            s += red[w * NS + threadIdx.x];
        if (s != 0.0)
            gl_add_f64(&out[threadIdx.x], s);
    }
}


// Statistics terms for a runtime number of axes (batched kernels).
__device__ __forceinline__ void stats_add_rt(double (&st)[kMaxStats], const double (&x)[kMaxDims],
                                             double w, int dims)
{
#pragma clang fp contract(off)
    st[0] += w;
    st[1] += w * w;
    int k = 2;
    for (int a = 0; a < dims; ++a) {
        const double wx = w * x[a];
        st[k] += wx;
        st[k + 1] += wx * x[a];
        k += 2;
        for (int c = 0; c < a; ++c) {
            st[k] += (w * x[c]) * x[a];
            ++k;
        }
    }
}

}  // namespace hg
