// learned.hip -- training of the learned find-bin index of a variable axis.
//
// The binary search of arXiv:2401.13310 Sec. 3.1 / 3.2 costs about log2(nbins)
// dependent loads per coordinate.  The learned index replaces most of them by
// arithmetic: an order-preserving feature of x is cut into `nseg` equal
// segments; each segment fits the bin position as a quadratic of the
// segment-local feature z on training pairs made from the edge array by the
// find-bin rule (edge e_i lies at the start of bin i+1; the midpoint of bin
// i+1 lies half a bin further), and stores error bounds measured at every
// edge the segment can see.  The segment map and z are monotone in x, the
// stored quadratic is checked to be monotone over the z range of those edges,
// and the FP32 Horner rounding is bounded by gamma = 4u (1 + |b||z| + |c|z^2),
// so for any x in the segment the bin lies in
//   [ai + ceil(y(z)), ai + floor(y(z) + w)]
// with the lower-bound offset folded into the intercept and w rounded up.  The
// search that follows is exact; when that interval has one element no edge is
// read at all.
#include "kernels.h"

namespace hg {

__global__ void seg_of_edges_kernel(const AxisDev ax, int32_t *seg)
{
    const int32_t ne = ax.nbins + 1;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += blockDim.x * gridDim.x)
    {
        int32_t sg;
        float z;
        seg_and_z(ax.edges[i], ax, sg, z);
        seg[i] = sg;
    }
}

// first index i in [0, n) with seg[i] >= s (seg is non-decreasing)
__device__ int32_t first_at_least(const int32_t *seg, int32_t n, int32_t s)
{
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo) / 2;
        if (seg[mid] < s)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

template <int NV>
__device__ void block_sum(double (&v)[NV], double *red)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double x = v[k];
        for (int off = kWave / 2; off > 0; off >>= 1)
            x += __shfl_xor(x, off, kWave);
        v[k] = x;
    }
    __syncthreads();
    if (lane == 0)
        for (int k = 0; k < NV; ++k)
            red[wave * NV + k] = v[k];
    __syncthreads();
    for (int k = 0; k < NV; ++k) {
        double s = 0.0;
        for (int w = 0; w < nw; ++w)
            s += red[w * NV + k];
        v[k] = s;
    }
    __syncthreads();
}

__device__ void block_minmax(double &mn, double &mx, double &gm, double *red)
{
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    for (int off = kWave / 2; off > 0; off >>= 1) {
        mn = fmin(mn, __shfl_xor(mn, off, kWave));
        mx = fmax(mx, __shfl_xor(mx, off, kWave));
        gm = fmax(gm, __shfl_xor(gm, off, kWave));
    }
    __syncthreads();
    if (lane == 0) {
        red[wave * 3 + 0] = mn;
        red[wave * 3 + 1] = mx;
        red[wave * 3 + 2] = gm;
    }
    __syncthreads();
    for (int w = 0; w < nw; ++w) {
        mn = fmin(mn, red[w * 3 + 0]);
        mx = fmax(mx, red[w * 3 + 1]);
        gm = fmax(gm, red[w * 3 + 2]);
    }
    __syncthreads();
}

// z of x relative to segment s: for x in segment s exactly the value inference
// computes, and a monotone extension of it for the neighbouring edges.
__device__ __forceinline__ float z_in_seg(double x, const AxisDev &ax, int32_t s)
{
    if (ax.feature == FEAT_KEY) {
        const int64_t d = (int64_t)key_feature(x, ax) - ((int64_t)s << ax.kshift);
        return (float)d * ax.zscale;
    }
    const double t = (x - ax.x0) * ax.fscale;
    return (float)(t - (double)s);
}

// One workgroup per segment.  diag[2*s] = candidate-interval width, diag[2*s+1]
// = number of edges inside the segment.
__global__ void __launch_bounds__(256) fit_segments_kernel(const AxisDev ax, const int32_t *seg,
                                                           ModelSeg *model, double *diag)
{
    __shared__ double red[4 * 9];
    const int32_t s = blockIdx.x;
    const int32_t n = ax.nbins;
    const double *e = ax.edges;
    const int32_t lo_s = first_at_least(seg, n + 1, s);
    const int32_t hi_s = first_at_least(seg, n + 1, s + 1);
    const int32_t j0 = lo_s > 0 ? lo_s - 1 : 0;
    const int32_t j1 = hi_s < n ? hi_s : n;   // inclusive
    const double ymid = 0.5 * ((double)j0 + (double)j1) + 1.0;

    // least-squares sums over edges (target i+1) and midpoints (target i+1.5)
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // S0..S4, T0..T2, unused
    for (int32_t i = j0 + (int32_t)threadIdx.x; i <= j1; i += blockDim.x) {
        for (int h = 0; h < 2; ++h) {
            if (h == 1 && i == j1)
                break;
            const double x = h == 0 ? e[i] : 0.5 * e[i] + 0.5 * e[i + 1];
            const double y = (double)i + (h == 0 ? 1.0 : 1.5) - ymid;
            const double z = (double)z_in_seg(x, ax, s);
            const double z2 = z * z;
            v[0] += 1.0;
            v[1] += z;
            v[2] += z2;
            v[3] += z2 * z;
            v[4] += z2 * z2;
            v[5] += y;
            v[6] += z * y;
            v[7] += z2 * y;
        }
    }
    block_sum<9>(v, red);

    // solve the 3x3 normal equations (thread-uniform arithmetic)
    double a = 0.0, b = 0.0, c = 0.0;
    {
        double M[3][4] = {{v[0], v[1], v[2], v[5]}, {v[1], v[2], v[3], v[6]}, {v[2], v[3], v[4], v[7]}};
        bool ok = true;
        for (int col = 0; col < 3 && ok; ++col) {
            int piv = col;
            for (int r = col + 1; r < 3; ++r)
                if (fabs(M[r][col]) > fabs(M[piv][col]))
                    piv = r;
            if (!(fabs(M[piv][col]) > 1e-12 * (fabs(M[0][0]) + 1.0))) {
                ok = false;
                break;
            }
            if (piv != col)
                for (int k = 0; k < 4; ++k) {
                    double t = M[col][k];
                    M[col][k] = M[piv][k];
                    M[piv][k] = t;
                }
            for (int r = 0; r < 3; ++r) {
                if (r == col)
                    continue;
                const double f = M[r][col] / M[col][col];
                for (int k = col; k < 4; ++k)
                    M[r][k] -= f * M[col][k];
            }
        }
        if (ok) {
            a = M[0][3] / M[0][0];
            b = M[1][3] / M[1][1];
            c = M[2][3] / M[2][2];
        }
        if (!ok || !isfinite(a) || !isfinite(b) || !isfinite(c)) {
            // linear fit, then constant
            const double den = v[0] * v[2] - v[1] * v[1];
            c = 0.0;
            if (den > 1e-300 && v[0] >= 2.0) {
                b = (v[0] * v[6] - v[1] * v[5]) / den;
                a = (v[5] - b * v[1]) / v[0];
            } else {
                b = 0.0;
                a = v[0] > 0 ? v[5] / v[0] : 0.0;
            }
        }
    }
    // Stored coefficients: b in FP32, c in half.  The exact polynomial must be
    // monotone over the z range of the evaluated edges, else fall back to a
    // linear (then constant) model.
    const double zmin = (double)z_in_seg(e[j0], ax, s);
    const double zmax = (double)z_in_seg(e[j1], ax, s);
    float bq = (float)b;
    float cq = (float)(_Float16)c;
    if (!((double)bq + 2.0 * (double)cq * zmin >= 0.0) || !((double)bq + 2.0 * (double)cq * zmax >= 0.0) ||
        !isfinite(a) || !isfinite(bq) || !isfinite(cq)) {
        const double den = v[0] * v[2] - v[1] * v[1];
        cq = 0.0f;
        if (den > 1e-300 && v[0] >= 2.0) {
            b = (v[0] * v[6] - v[1] * v[5]) / den;
            a = (v[5] - b * v[1]) / v[0];
        } else {
            b = 0.0;
            a = v[0] > 0 ? v[5] / v[0] : 0.0;
        }
        bq = (float)b;
        if (!(bq >= 0.0f) || !isfinite(bq)) {
            bq = 0.0f;
            a = v[0] > 0 ? v[5] / v[0] : 0.0;
        }
    }
    a += ymid;
    const double ai0 = floor(a);
    ModelSeg m;
    m.af = (float)(a - ai0);
    m.b = bq;
    m.ai = 0;
    m.cw = (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)cq);

    // residuals of ai0 + y(z) at every evaluated edge (the FP32 evaluation
    // inference performs), and the FP32 Horner error bound gamma
    double dlo = 1e300, dhi = -1e300, gmax = 0.0;
    for (int32_t i = j0 + (int32_t)threadIdx.x; i <= j1; i += blockDim.x) {
        const float z = z_in_seg(e[i], ax, s);
        const double p = ai0 + (double)model_eval(m, z);
        const double r = p - (double)(i + 1);
        dlo = fmin(dlo, r);
        dhi = fmax(dhi, r);
        // |af| <= 1 both before and after the lower bound is folded into it
        gmax = fmax(gmax, 1.0 + fabs((double)bq) * fabs((double)z) +
                              fabs((double)cq) * (double)z * (double)z);
    }
    block_minmax(dlo, dhi, gmax, red);
    if (threadIdx.x == 0) {
        const double u = 0x1p-24;
        const double gamma = 4.0 * u * gmax;               // |fl(y) - y| on the segment
        const double eta = 8.0 * u * (gmax + 2.0) + 1e-9;  // roundings of y+w, residuals
        // lower bound: bin >= ai0 + y - 1 - dhi - 2 gamma; fold it into af with
        // room for the rounding of the folded evaluation
        const double clo = -1.0 - dhi - 4.0 * gamma - eta;
        const double tot = (double)m.af + clo;
        const double fl = floor(tot);
        m.ai = (int32_t)fmax(-2147483647.0, fmin(2147483647.0, ai0 + fl));
        m.af = __double2float_rd(tot - fl);
        // width: bin <= ai0 + y - dlo + 2 gamma
        const double wdt = (-dlo + 2.0 * gamma) - clo + 4.0 * gamma + eta;
        _Float16 wh = (_Float16)wdt;
        if ((double)(float)wh < wdt) {
            uint16_t bits = __builtin_bit_cast(uint16_t, wh);
            wh = __builtin_bit_cast(_Float16, (uint16_t)(bits + 1));   // next half up (to +inf past max)
        }
        if (!(wdt < 65504.0))
            wh = __builtin_bit_cast(_Float16, (uint16_t)0x7C00);        // +inf: search the whole axis
        m.cw = (m.cw & 0xFFFFu) | ((uint32_t)__builtin_bit_cast(uint16_t, wh) << 16);
        model[s] = m;
        diag[2 * s] = (double)(float)wh;
        diag[2 * s + 1] = (double)(hi_s - lo_s);
    }
}

hipError_t launch_seg_of_edges(const AxisDev &ax, int32_t *seg, hipStream_t s)
{
    const int ne = ax.nbins + 1;
    int blocks = (ne + 255) / 256;
    if (blocks > 4096)
        blocks = 4096;
    hipLaunchKernelGGL(seg_of_edges_kernel, dim3(blocks), dim3(256), 0, s, ax, seg);
    return hipGetLastError();
}

hipError_t launch_fit_segments(const AxisDev &ax, const int32_t *seg, ModelSeg *model,
                               double *diag, hipStream_t s)
{
    hipLaunchKernelGGL(fit_segments_kernel, dim3(ax.nseg), dim3(256), 0, s, ax, seg, model, diag);
    return hipGetLastError();
}

}  // namespace hg
