// fill.hip -- histogram fill kernels for gfx950 (MI355X).
//
// One pass over a bulk of events does the three Fill steps of arXiv:2401.13310
// Sec. 3.1 together: find the bin on every axis, add the weight (and its
// square) to that bin, and add the event's terms to the statistics sums of
// Sec. 3.2.  Like the paper's two-stage kernel (Sec. 3.2), each workgroup
// first accumulates into a private copy of (a window of) the histogram in LDS
// and merges it into the global histogram at the end; the statistics are
// reduced in the same pass instead of by separate reduction kernels.
//
// gfx950 specifics that shape the code:
//   - 160 KB of LDS per workgroup: one workgroup per CU can privatize 80K
//     16-bit counters, 40K 32-bit counters or 10K binary64 (sum, sum2) pairs;
//   - scattered global atomics are two orders of magnitude slower than LDS
//     atomics, so they are only a fallback for bins outside the LDS window,
//     and large windows merge through a staging buffer and a reduction kernel
//     instead of coalesced atomics;
//   - small histograms keep up to 64 interleaved copies so the 64 lanes of a
//     wave that hit the same bin update different LDS words (no serialized
//     same-address atomics).
#include "fill_body.h"

#include <mutex>
#include <unordered_set>

namespace hg {

template <int D, typename T, int ACC, bool W, int U, int KS>
__global__ void __launch_bounds__(kMaxThreads) fill_kernel(const FillArgs A)
{
    extern __shared__ __align__(16) char smem[];
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    fill_range<D, T, ACC, W, U, KS>(A, smem, start, end, blockIdx.x, gridDim.x);
}

// The same body at two workgroups per CU (the partition count pass of
// fixed-width axes).
template <int D, typename T, int ACC, bool W, int U, int KS>
__global__ void __launch_bounds__(kMaxThreads, kCountWavesPerSimd) fill_kernel_x2(const FillArgs A)
{
    extern __shared__ __align__(16) char smem[];
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    fill_range<D, T, ACC, W, U, KS>(A, smem, start, end, blockIdx.x, gridDim.x);
}

// Sums the staging slots (32-bit counters or binary64 sums) of `nblocks` fill
// workgroups into the histogram.  blockIdx.y selects a group of slots; groups
// add with coalesced atomics.
template <int ACC>
__global__ void __launch_bounds__(256) stage_reduce_kernel(const FillArgs A, int nblocks,
                                                           int per_group)
{
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int b0 = blockIdx.y * per_group;
    const int b1 = b0 + per_group < nblocks ? b0 + per_group : nblocks;
    const int W = A.win_len;
    if (ACC == ACC_U32) {
        if (u >= W)
            return;
        const uint32_t *st = static_cast<const uint32_t *>(A.stage);
        uint64_t s = 0;
#pragma unroll 8
        for (int b = b0; b < b1; ++b)
            s += st[(int64_t)b * A.stage_stride + u];
        if (s)
            gl_add_u64(&A.cnt[A.win_lo + u], s);
    } else {
        if (u >= W)
            return;
        const double *st = static_cast<const double *>(A.stage);
        double s = 0.0, s2 = 0.0;
#pragma unroll 8
        for (int b = b0; b < b1; ++b) {
            s += st[(int64_t)b * 2 * A.stage_stride + u];
            s2 += st[(int64_t)b * 2 * A.stage_stride + A.stage_stride + u];
        }
        if (s != 0.0 || s2 != 0.0) {
            gl_add_f64(&A.sumw[A.win_lo + u], s);
            gl_add_f64(&A.sumw2[A.win_lo + u], s2);
        }
    }
}

// The 8-bit slots of the 16-bit windows: one workgroup per 64 consecutive
// words (256 bins), its 256 threads 16 quads of words x 16 groups of slots,
// 16-byte loads (slot strides are whole 128-byte lines), every thread
// summing up to 16 slots.  Eight slots at a time are summed as 16-bit halves
// (even and odd bytes apart, at most 8 x 255 each), then widened.  The partial
// sums of each bin meet in LDS; one thread per bin adds the total.
__global__ void __launch_bounds__(256) stage_reduce_u8_kernel(const FillArgs A, int nblocks)
{
    __shared__ uint32_t part[16][256];
    const int q = threadIdx.x & 15;   // quad of words in the tile
    const int g = threadIdx.x >> 4;   // group of slots: g, g + 16, ...
    const int swords = (A.win_len + 3) >> 2;
    const int64_t w0 = (int64_t)blockIdx.x * 64 + 4 * q;
    uint32_t sum[16];
#pragma unroll
    for (int k = 0; k < 16; ++k)
        sum[k] = 0u;
    if (w0 < swords) {
        const uint32_t *st = static_cast<const uint32_t *>(A.stage) + w0;
        // eight slots at a time, all loads issued before any is used (slots
        // past the last read the last one, and count 0)
        for (int b0 = g; b0 < nblocks; b0 += 8 * 16) {
            uint4 v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const int b = b0 + 16 * k < nblocks ? b0 + 16 * k : nblocks - 1;
                v[k] = *reinterpret_cast<const uint4 *>(st + (int64_t)b * A.stage_stride);
            }
            uint32_t ev[4] = {0u, 0u, 0u, 0u}, od[4] = {0u, 0u, 0u, 0u};
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const uint32_t m = b0 + 16 * k < nblocks ? 0x00FF00FFu : 0u;
                const uint32_t u[4] = {v[k].x, v[k].y, v[k].z, v[k].w};
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    ev[e] += u[e] & m;
                    od[e] += (u[e] >> 8) & m;
                }
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                sum[4 * e + 0] += ev[e] & 0xFFFFu;
                sum[4 * e + 1] += od[e] & 0xFFFFu;
                sum[4 * e + 2] += ev[e] >> 16;
                sum[4 * e + 3] += od[e] >> 16;
            }
        }
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
        part[g][16 * q + k] = sum[k];
    __syncthreads();
    const int l = blockIdx.x * 256 + threadIdx.x;   // bin in the window
    uint64_t t = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        t += part[i][threadIdx.x];
    if (l < A.win_len && t)
        gl_add_u64(&A.cnt[A.win_lo + l], t);
}

// Find bin only: the global bin of every event (grid-stride).
template <int D, typename T>
__global__ void __launch_bounds__(kMaxThreads) findbin_kernel(const FillArgs A, int32_t *out)
{
    extern __shared__ __align__(16) char smem[];
    stage_axes<D>(A.ax, smem);
    __syncthreads();
    const int64_t stride = (int64_t)blockDim.x * gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride) {
        int32_t g = 0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            const double x = (double)static_cast<const T *>(A.coords[a])[i];
            const int32_t b = axis_bin(x, A.ax[a], smem);
            g += (a == 0) ? b : b * A.ax[a].stride;
        }
        out[i] = g;
    }
}

// Tiled strategy, pass 1: global bin of every event into A.gbins, with the
// statistics reduced in the same pass.
template <int D, typename T, bool W>
__global__ void __launch_bounds__(kMaxThreads) tiled_bins_kernel(const FillArgs A)
{
    extern __shared__ __align__(16) char smem[];
    constexpr int NS = NStats<D>::v;
    if (blockIdx.x == 0 && threadIdx.x == 0 && A.entries)
        gl_add_u64(A.entries, (uint64_t)A.n);
    stage_axes<D>(A.ax, smem);
    __syncthreads();
    double st[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        st[k] = 0.0;
    const int64_t stride = (int64_t)blockDim.x * gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A.n; i += stride) {
        double x[D];
        int32_t g = 0;
        bool inside = true;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            x[a] = (double)static_cast<const T *>(A.coords[a])[i];
            const int32_t b = axis_bin(x[a], A.ax[a], smem);
            inside = inside && (uint32_t)(b - 1) < (uint32_t)A.ax[a].nbins;
            g += (a == 0) ? b : b * A.ax[a].stride;
        }
        A.gbins[i] = g;
        if (inside)
            stats_add<D>(st, x, W ? (double)static_cast<const T *>(A.w)[i] : 1.0);
    }
    __syncthreads();
    reduce_stats<NS>(st, reinterpret_cast<double *>(smem), A.stats);
}

// Tiled strategy, pass 2: block (x, y) accumulates the events of chunk x whose
// bin falls in tile y (bins [y*tile_len, (y+1)*tile_len)) in LDS, then merges.
template <int ACC, typename T, bool W>
__global__ void __launch_bounds__(kMaxThreads) tile_kernel(const TileArgs A)
{
    extern __shared__ __align__(16) char smem[];
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int32_t t0 = blockIdx.y * A.tile_len;
    const int32_t tlen = (A.T - t0) < A.tile_len ? (A.T - t0) : A.tile_len;
    uint32_t *win = reinterpret_cast<uint32_t *>(smem + A.lds_win);
    const int words = window_words(ACC, tlen, A.copies);
    for (int i = tid; i < words; i += nthr)
        win[i] = 0u;
    __syncthreads();
    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    const int cp = (ACC == ACC_U16) ? 0 : tid % A.copies;
    int it = 0;
    constexpr int U = kTileUnroll;
    for (int64_t base = start; base < end; base += (int64_t)nthr * U) {
        int32_t gv[U];
        T wv[U];
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const int64_t i = base + (int64_t)j * nthr + tid;
            const bool ok = i < end;
            gv[j] = ok ? A.gbins[i] : -1;
            if (W)
                wv[j] = ok ? static_cast<const T *>(A.w)[i] : T(0);
        }
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const uint32_t l = (uint32_t)(gv[j] - t0);
            if (gv[j] >= 0 && l < (uint32_t)tlen) {
                if (ACC == ACC_U32) {
                    lds_add_u32(&win[l * A.copies + cp], 1u);
                } else if (ACC == ACC_U16) {
                    lds_add_u32(&win[l >> 1], 1u << ((l & 1u) << 4));
                } else {
                    const double w = (double)wv[j];
                    double *s = reinterpret_cast<double *>(win);
                    const uint32_t idx = l * A.copies + cp;
                    lds_add_f64(&s[idx], w);
                    lds_add_f64(&s[(uint32_t)tlen * A.copies + idx], w * w);
                }
            }
        }
        if (ACC == ACC_U16 && ++it == A.epoch_iters) {
            it = 0;
            __syncthreads();
            drain_u16(win, words, t0, A.cnt);
            __syncthreads();
        }
    }
    __syncthreads();
    if (ACC == ACC_U32) {
        for (int l = tid; l < tlen; l += nthr) {
            uint32_t c = 0;
            for (int r = 0; r < A.copies; ++r)
                c += win[l * A.copies + r];
            if (c)
                gl_add_u64(&A.cnt[t0 + l], c);
        }
    } else if (ACC == ACC_U16) {
        for (int i = tid; i < words; i += nthr) {
            const uint32_t v = win[i];
            const int64_t g0 = (int64_t)t0 + 2 * (int64_t)i;
            if (v & 0xFFFFu)
                gl_add_u64(&A.cnt[g0], v & 0xFFFFu);
            if (v >> 16)
                gl_add_u64(&A.cnt[g0 + 1], v >> 16);
        }
    } else {
        const double *d = reinterpret_cast<const double *>(win);
        const int n1 = tlen * A.copies;
        for (int l = tid; l < tlen; l += nthr) {
            double s = 0.0, s2 = 0.0;
            for (int r = 0; r < A.copies; ++r) {
                s += d[l * A.copies + r];
                s2 += d[n1 + l * A.copies + r];
            }
            if (s != 0.0 || s2 != 0.0) {
                gl_add_f64(&A.sumw[t0 + l], s);
                gl_add_f64(&A.sumw2[t0 + l], s2);
            }
        }
    }
}

__global__ void zero_u64_kernel(uint64_t *p, int64_t n)
{
    const int64_t stride = (int64_t)blockDim.x * gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0ull;
}
__global__ void zero_f64_kernel(double *p, int64_t n)
{
    const int64_t stride = (int64_t)blockDim.x * gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = 0.0;
}
__global__ void add_u64_to_f64_kernel(double *dst, const uint64_t *src, int64_t n)
{
    const int64_t stride = (int64_t)blockDim.x * gridDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] += (double)src[i];
}

// ------------------------------------------------------------------ launchers

// Lets a kernel take the whole 160 KB of gfx950 LDS (once per kernel).
template <typename K>
static void allow_big_lds(K kernel)
{
    static std::mutex mu;
    static std::unordered_set<const void *> done;
    const void *key = reinterpret_cast<const void *>(kernel);
    std::lock_guard<std::mutex> lock(mu);
    if (done.insert(key).second)
        (void)hipFuncSetAttribute(key, hipFuncAttributeMaxDynamicSharedMemorySize, 163840);
}

void allow_big_lds_ptr(const void *kernel) { allow_big_lds(kernel); }

template <int D, typename T, int ACC, bool W, int KS>
static hipError_t launch_fill_t(int threads, int blocks, size_t lds, const FillArgs &a,
                                hipStream_t s)
{
    constexpr int U = fill_unroll(D, sizeof(T) == 4, W, ACC, KS);
    if constexpr (ACC == ACC_PCOUNT && KS == KS_UNIFORM) {
        auto k = fill_kernel_x2<D, T, ACC, W, U, KS>;
        allow_big_lds(k);
        hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a);
    } else {
        auto k = fill_kernel<D, T, ACC, W, U, KS>;
        allow_big_lds(k);
        hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a);
    }
    return hipGetLastError();
}

template <int D, typename T, int KS>
static hipError_t launch_fill_k(int acc, bool weighted, int threads, int blocks, size_t lds,
                                const FillArgs &a, hipStream_t s)
{
    if (acc == ACC_PCOUNT)
        return weighted ? launch_fill_t<D, T, ACC_PCOUNT, true, KS>(threads, blocks, lds, a, s)
                        : launch_fill_t<D, T, ACC_PCOUNT, false, KS>(threads, blocks, lds, a, s);
    if (!weighted) {
        if (acc == ACC_U32)
            return launch_fill_t<D, T, ACC_U32, false, KS>(threads, blocks, lds, a, s);
        if (acc == ACC_U16)
            return launch_fill_t<D, T, ACC_U16, false, KS>(threads, blocks, lds, a, s);
        return hipErrorInvalidValue;
    }
    if (acc == ACC_F64)
        return launch_fill_t<D, T, ACC_F64, true, KS>(threads, blocks, lds, a, s);
    if constexpr (sizeof(T) == 4) {
        if (acc == ACC_F32C)
            return launch_fill_t<D, T, ACC_F32C, true, KS>(threads, blocks, lds, a, s);
    }
    return hipErrorInvalidValue;
}

template <int D, typename T>
static hipError_t launch_fill_d(int acc, bool weighted, int ks, int threads, int blocks,
                                size_t lds, const FillArgs &a, hipStream_t s)
{
    if (ks == KS_UNIFORM)
        return launch_fill_k<D, T, KS_UNIFORM>(acc, weighted, threads, blocks, lds, a, s);
    if (ks == KS_STAGED)
        return launch_fill_k<D, T, KS_STAGED>(acc, weighted, threads, blocks, lds, a, s);
    if constexpr (D == 1) {
        if (ks == KS_LEARNED1)
            return launch_fill_k<D, T, KS_LEARNED1>(acc, weighted, threads, blocks, lds, a, s);
        return launch_fill_k<D, T, KS_BSEARCH1>(acc, weighted, threads, blocks, lds, a, s);
    } else {
        return launch_fill_k<D, T, KS_MIXED>(acc, weighted, threads, blocks, lds, a, s);
    }
}


hipError_t launch_fill(int dims, bool f32, int acc, bool weighted, int threads, int blocks,
                       size_t lds, const FillArgs &a, hipStream_t s)
{
    const int ks = kind_set(dims, a.ax);
    switch (dims * 2 + (f32 ? 1 : 0)) {
    case 2: return launch_fill_d<1, double>(acc, weighted, ks, threads, blocks, lds, a, s);
    case 3: return launch_fill_d<1, float>(acc, weighted, ks, threads, blocks, lds, a, s);
    case 4: return launch_fill_d<2, double>(acc, weighted, ks, threads, blocks, lds, a, s);
    case 5: return launch_fill_d<2, float>(acc, weighted, ks, threads, blocks, lds, a, s);
    case 6: return launch_fill_d<3, double>(acc, weighted, ks, threads, blocks, lds, a, s);
    case 7: return launch_fill_d<3, float>(acc, weighted, ks, threads, blocks, lds, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_stage_reduce(int acc, int blocks_used, const FillArgs &a, hipStream_t s)
{
    if (acc == ACC_U16) {
        const int swords = (a.win_len + 3) / 4;
        hipLaunchKernelGGL(stage_reduce_u8_kernel, dim3((swords + 63) / 64), dim3(256), 0, s, a, blocks_used);
        return hipGetLastError();
    }
    const int units = a.win_len;
    const int per_group = 32;
    const int groups = (blocks_used + per_group - 1) / per_group;
    dim3 grid((units + 255) / 256, groups);
    switch (acc) {
    case ACC_U32: hipLaunchKernelGGL(stage_reduce_kernel<ACC_U32>, grid, dim3(256), 0, s, a, blocks_used, per_group); break;
    default: hipLaunchKernelGGL(stage_reduce_kernel<ACC_F64>, grid, dim3(256), 0, s, a, blocks_used, per_group); break;
    }
    return hipGetLastError();
}

template <int D, typename T>
static hipError_t launch_findbin_t(int threads, int blocks, size_t lds, const FillArgs &a,
                                   int32_t *out, hipStream_t s)
{
    auto k = findbin_kernel<D, T>;
    allow_big_lds(k);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a, out);
    return hipGetLastError();
}

hipError_t launch_findbin(int dims, bool f32, int threads, int blocks, size_t lds,
                          const FillArgs &a, int32_t *out, hipStream_t s)
{
    switch (dims * 2 + (f32 ? 1 : 0)) {
    case 2: return launch_findbin_t<1, double>(threads, blocks, lds, a, out, s);
    case 3: return launch_findbin_t<1, float>(threads, blocks, lds, a, out, s);
    case 4: return launch_findbin_t<2, double>(threads, blocks, lds, a, out, s);
    case 5: return launch_findbin_t<2, float>(threads, blocks, lds, a, out, s);
    case 6: return launch_findbin_t<3, double>(threads, blocks, lds, a, out, s);
    case 7: return launch_findbin_t<3, float>(threads, blocks, lds, a, out, s);
    default: return hipErrorInvalidValue;
    }
}

template <int D, typename T, bool W>
static hipError_t launch_tb_t(int threads, int blocks, size_t lds, const FillArgs &a, hipStream_t s)
{
    auto k = tiled_bins_kernel<D, T, W>;
    allow_big_lds(k);
    hipLaunchKernelGGL(k, dim3(blocks), dim3(threads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_tiled_bins(int dims, bool f32, bool weighted, int threads, int blocks,
                             size_t lds, const FillArgs &a, hipStream_t s)
{
    const int key = (dims * 2 + (f32 ? 1 : 0)) * 2 + (weighted ? 1 : 0);
    switch (key) {
    case 4: return launch_tb_t<1, double, false>(threads, blocks, lds, a, s);
    case 5: return launch_tb_t<1, double, true>(threads, blocks, lds, a, s);
    case 6: return launch_tb_t<1, float, false>(threads, blocks, lds, a, s);
    case 7: return launch_tb_t<1, float, true>(threads, blocks, lds, a, s);
    case 8: return launch_tb_t<2, double, false>(threads, blocks, lds, a, s);
    case 9: return launch_tb_t<2, double, true>(threads, blocks, lds, a, s);
    case 10: return launch_tb_t<2, float, false>(threads, blocks, lds, a, s);
    case 11: return launch_tb_t<2, float, true>(threads, blocks, lds, a, s);
    case 12: return launch_tb_t<3, double, false>(threads, blocks, lds, a, s);
    case 13: return launch_tb_t<3, double, true>(threads, blocks, lds, a, s);
    case 14: return launch_tb_t<3, float, false>(threads, blocks, lds, a, s);
    case 15: return launch_tb_t<3, float, true>(threads, blocks, lds, a, s);
    default: return hipErrorInvalidValue;
    }
}

template <int ACC, typename T, bool W>
static hipError_t launch_tile_t(int threads, int bx, int tiles, size_t lds, const TileArgs &t,
                                hipStream_t s)
{
    auto k = tile_kernel<ACC, T, W>;
    allow_big_lds(k);
    hipLaunchKernelGGL(k, dim3(bx, tiles), dim3(threads), lds, s, t);
    return hipGetLastError();
}

hipError_t launch_tile(int acc, bool f32, int threads, int blocks_x, int tiles, size_t lds,
                       const TileArgs &t, hipStream_t s)
{
    if (acc == ACC_U32)
        return launch_tile_t<ACC_U32, double, false>(threads, blocks_x, tiles, lds, t, s);
    if (acc == ACC_U16)
        return launch_tile_t<ACC_U16, double, false>(threads, blocks_x, tiles, lds, t, s);
    if (f32)
        return launch_tile_t<ACC_F64, float, true>(threads, blocks_x, tiles, lds, t, s);
    return launch_tile_t<ACC_F64, double, true>(threads, blocks_x, tiles, lds, t, s);
}

static int grid_for(int64_t n)
{
    int64_t b = (n + 255) / 256;
    return (int)(b < 4096 ? (b < 1 ? 1 : b) : 4096);
}

hipError_t launch_zero_u64(uint64_t *p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_u64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_zero_f64(double *p, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(zero_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}
hipError_t launch_add_u64_to_f64(double *dst, const uint64_t *src, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(add_u64_to_f64_kernel, dim3(grid_for(n)), dim3(256), 0, s, dst, src, n);
    return hipGetLastError();
}

}  // namespace hg
