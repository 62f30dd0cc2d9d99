// probe.hip -- measurement probes for the roofline of the fill kernels: the
// read bandwidth a plain streaming kernel reaches from HBM, and the rates of
// the atomics the fill's accumulation stage is made of (LDS atomics into
// workgroup-private sub-histograms and device-scope atomics in L2, the two
// stages of the paper's fill kernel, arXiv:2401.13310 Sec. 3.2).  Timed with
// HIP events on the caller's stream.
#include "../../include/hist.h"
#include "device_common.h"
#include "kernels.h"
#include "plan.h"

namespace hg {

using u32x4 = uint32_t __attribute__((ext_vector_type(4)));

// Streaming read of `n16` 16-byte words, 4 per thread per step, non-temporal;
// a per-block checksum keeps the loads live.
__global__ void __launch_bounds__(1024) read_probe_kernel(const u32x4 *__restrict__ p, int64_t n16,
                                                          uint32_t *sink)
{
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x * 4; base < n16; base += stride) {
        u32x4 v[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int64_t i = base + (int64_t)j * blockDim.x + threadIdx.x;
            v[j] = i < n16 ? __builtin_nontemporal_load(p + i) : u32x4{0u, 0u, 0u, 0u};
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            acc ^= v[j].x ^ v[j].y ^ v[j].z ^ v[j].w;
    }
    if (acc == 0x9E3779B9u)   // practically never; keeps the reads
        sink[blockIdx.x] = acc;
}

// Integer hash of (lane, step): a spread of LDS or L2 addresses.
__device__ __forceinline__ uint32_t mix(uint32_t x)
{
    x ^= x >> 16;
    x *= 0x7feb352dU;
    x ^= x >> 15;
    x *= 0x846ca68bU;
    x ^= x >> 16;
    return x;
}

// LDS atomic adds to hashed addresses of a `words`-word region (power of two):
// KIND 0 u32, 1 binary64.
template <int KIND>
__global__ void __launch_bounds__(1024) lds_atomic_probe_kernel(int steps, int words, uint32_t *sink)
{
    extern __shared__ __align__(16) char smem[];
    uint32_t *u = reinterpret_cast<uint32_t *>(smem);
    double *d = reinterpret_cast<double *>(smem);
    const int n = KIND == 0 ? words : words / 2;
    for (int i = threadIdx.x; i < words; i += blockDim.x)
        u[i] = 0u;
    __syncthreads();
    const uint32_t seed = mix(blockIdx.x * 1024u + threadIdx.x);
    for (int s = 0; s < steps; ++s) {
        const uint32_t a = mix(seed + (uint32_t)s) & (uint32_t)(n - 1);
        if (KIND == 0)
            lds_add_u32(&u[a], 1u);
        else
            lds_add_f64(&d[a], 1.0);
    }
    __syncthreads();
    if (threadIdx.x == 0 && u[0] == 0xFFFFFFFFu)
        sink[blockIdx.x] = u[0];
}

// Device-scope atomic adds (no return) to hashed addresses of an `n`-element
// array (power of two): KIND 0 u64, 1 binary64.
template <int KIND>
__global__ void __launch_bounds__(256) global_atomic_probe_kernel(void *arr, int64_t n, int steps)
{
    const uint32_t seed = mix(blockIdx.x * 256u + threadIdx.x);
    for (int s = 0; s < steps; ++s) {
        const int64_t a = (int64_t)(mix(seed ^ (uint32_t)(s * 0x9E3779B9u)) & (uint32_t)(n - 1));
        if (KIND == 0)
            gl_add_u64(static_cast<uint64_t *>(arr) + a, 1ull);
        else
            gl_add_f64(static_cast<double *>(arr) + a, 1.0);
    }
}

}  // namespace hg

using namespace hg;

static hist_status probe_fail(const char *what)
{
    const hipError_t e = hipGetLastError();
    return set_error(HIST_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

extern "C" hist_status hist_probe(int kind, const void *buf, int64_t bytes, int reps, void *stream,
                                  double *rate, double *ms_out)
{
    if (!rate || reps < 1)
        return set_error(HIST_EINVAL, "hist_probe: need rate and reps >= 1");
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0, ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ncu = prop.multiProcessorCount;
    uint32_t *sink = nullptr;
    if (hipMalloc(&sink, sizeof(uint32_t) * 65536) != hipSuccess)
        return probe_fail("hist_probe: sink");
    hipEvent_t e0, e1;
    (void)hipEventCreate(&e0);
    (void)hipEventCreate(&e1);
    hist_status st = HIST_OK;
    double work = 0.0;   // bytes or atomic operations of one repetition
    auto launch = [&]() -> bool {
        switch (kind) {
        case HIST_PROBE_READ: {
            const int64_t n16 = bytes / 16;
            hipLaunchKernelGGL(read_probe_kernel, dim3(ncu * 4), dim3(1024), 0, s,
                               static_cast<const u32x4 *>(buf), n16, sink);
            work = (double)n16 * 16.0;
            break;
        }
        case HIST_PROBE_LDS_U32:
        case HIST_PROBE_LDS_F64: {
            const int steps = 4096, words = 16384;   // a 64 KB region
            allow_big_lds_ptr(reinterpret_cast<const void *>(lds_atomic_probe_kernel<0>));
            allow_big_lds_ptr(reinterpret_cast<const void *>(lds_atomic_probe_kernel<1>));
            if (kind == HIST_PROBE_LDS_U32)
                hipLaunchKernelGGL(lds_atomic_probe_kernel<0>, dim3(ncu), dim3(1024), words * 4, s, steps,
                                   words, sink);
            else
                hipLaunchKernelGGL(lds_atomic_probe_kernel<1>, dim3(ncu), dim3(1024), words * 4, s, steps,
                                   words, sink);
            work = (double)ncu * 1024.0 * steps;
            break;
        }
        case HIST_PROBE_GLOBAL_U64:
        case HIST_PROBE_GLOBAL_F64: {
            int64_t n = 1;   // largest power of two of 8-byte elements within `bytes`
            while ((n << 1) * 8 <= bytes)
                n <<= 1;
            const int steps = 64;
            if (kind == HIST_PROBE_GLOBAL_U64)
                hipLaunchKernelGGL(global_atomic_probe_kernel<0>, dim3(ncu * 8), dim3(256), 0, s,
                                   const_cast<void *>(buf), n, steps);
            else
                hipLaunchKernelGGL(global_atomic_probe_kernel<1>, dim3(ncu * 8), dim3(256), 0, s,
                                   const_cast<void *>(buf), n, steps);
            work = (double)ncu * 8.0 * 256.0 * steps;
            break;
        }
        default:
            return false;
        }
        return hipGetLastError() == hipSuccess;
    };
    if ((kind == HIST_PROBE_READ || kind == HIST_PROBE_GLOBAL_U64 || kind == HIST_PROBE_GLOBAL_F64) &&
        (!buf || bytes < 4096)) {
        st = set_error(HIST_EINVAL, "hist_probe: this probe needs a device buffer of >= 4096 bytes");
    } else if (!launch()) {   // warm-up
        st = kind < HIST_PROBE_READ || kind > HIST_PROBE_GLOBAL_F64
                 ? set_error(HIST_EINVAL, "hist_probe: unknown kind %d", kind)
                 : probe_fail("hist_probe: launch");
    } else {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r)
            (void)launch();
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) {
            st = probe_fail("hist_probe: synchronize");
        } else {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            const double per = ms / reps;
            *rate = work / (per * 1e-3);
            if (ms_out)
                *ms_out = per;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipFree(sink);
    return st;
}
