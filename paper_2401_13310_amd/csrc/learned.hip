// learned.hip -- training of the learned find-bin index of a variable axis.
//
// The binary search of arXiv:2401.13310 Sec. 3.1 / 3.2 costs about log2(nbins)
// dependent loads per coordinate.  The learned index replaces most of them by
// arithmetic: an order-preserving feature of x is cut into `nseg` equal
// segments; each segment fits the bin position as a quadratic of the
// segment-local feature z on training pairs made from the edge array by the
// find-bin rule (edge e_i lies at the start of bin i+1; the midpoint of bin
// i+1 lies half a bin further), and stores error bounds measured at every
// edge the segment can see.  Because the feature, the segment map and the
// model are all monotone non-decreasing and the Horner rounding error is
// bounded, the bin of any x in the segment lies in
//   [ceil(p(z) + clo), floor(p(z) + chi)]
// so the search that follows is exact; when that interval has one element no
// edge is read at all.
#include "kernels.h"

namespace hg {

__global__ void seg_of_edges_kernel(const AxisDev ax, int32_t *seg)
{
    const int32_t ne = ax.nbins + 1;
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += blockDim.x * gridDim.x)
        seg[i] = seg_of(feature_t(ax.edges[i], ax), ax.nseg);
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

// z of x relative to segment s, exactly as inference computes it.
__device__ __forceinline__ double z_in_seg(double x, const AxisDev &ax, int32_t s)
{
    return feature_t(x, ax) - (double)s;
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
            const double z = z_in_seg(x, ax, s);
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
    // z range of the evaluated edges: monotone model there, else linear
    double zmin = z_in_seg(e[j0], ax, s);
    double zmax = z_in_seg(e[j1], ax, s);
    if (!(b + 2.0 * c * zmin >= 0.0) || !(b + 2.0 * c * zmax >= 0.0) || !isfinite(a)) {
        const double den = v[0] * v[2] - v[1] * v[1];
        c = 0.0;
        if (den > 1e-300 && v[0] >= 2.0) {
            b = (v[0] * v[6] - v[1] * v[5]) / den;
            a = (v[5] - b * v[1]) / v[0];
        } else {
            b = 0.0;
            a = v[0] > 0 ? v[5] / v[0] : 0.0;
        }
        if (!(b >= 0.0) || !isfinite(b)) {
            b = 0.0;
            a = v[0] > 0 ? v[5] / v[0] : 0.0;
        }
    }
    a += ymid;
    ModelSeg m;
    m.a = a;
    m.b = b;
    m.c = c;
    m.clo = 0.0;
    m.chi = 0.0;

    // residuals at every evaluated edge, and the Horner error bound
    double dlo = 1e300, dhi = -1e300, gmax = 0.0;
    for (int32_t i = j0 + (int32_t)threadIdx.x; i <= j1; i += blockDim.x) {
        const double z = z_in_seg(e[i], ax, s);
        const double p = model_eval(m, z);
        const double r = p - (double)(i + 1);
        dlo = fmin(dlo, r);
        dhi = fmax(dhi, r);
        gmax = fmax(gmax, fabs(a) + fabs(b) * fabs(z) + fabs(c) * z * z);
    }
    block_minmax(dlo, dhi, gmax, red);
    if (threadIdx.x == 0) {
        const double gamma = 4.0 * 0x1p-53 * gmax;   // |fl(p) - p| <= gamma on the segment
        const double eta = 4e-6;                     // rounding of p + clo, p + chi, residuals
        m.clo = -1.0 - dhi - 2.0 * gamma - eta;
        m.chi = -dlo + 2.0 * gamma + eta;
        model[s] = m;
        diag[2 * s] = m.chi - m.clo;
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
