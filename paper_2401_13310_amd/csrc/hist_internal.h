// hist_internal.h -- device-side data layout and find-bin routines shared by
// the kernels of the histogram library (gfx950).
//
// Find bin follows arXiv:2401.13310 Sec. 3.1: fixed-width axes use
// 1 + floor(nbins (x - min) / (max - min)); variable axes search the edge
// array; values outside the range go to the underflow (0) or overflow
// (nbins+1) bin.  Bins include their lower edge (upper_bound on edges) and NaN
// goes to overflow.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hg {

constexpr int kMaxDims = 3;
constexpr int kMaxStats = 11;
constexpr int kWave = 64;

enum AxisKind : int32_t { AX_UNIFORM = 0, AX_BSEARCH = 1, AX_LEARNED = 2 };
enum Feature : int32_t { FEAT_KEY = 0, FEAT_LINEAR = 1 };

// One segment of the learned index: bin position p = a + z (b + c z) over the
// segment-local feature z, and the offsets that turn p into the candidate
// interval [ceil(p + clo), floor(p + chi)] that provably holds the bin.
struct ModelSeg {
    double a, b, c, clo, chi;
};
static_assert(sizeof(ModelSeg) == 40, "ModelSeg layout");

struct AxisDev {
    int32_t nbins;
    int32_t kind;           // AxisKind
    double xmin, xmax;      // range; variable axes: e[0] and e[nbins]
    double nbins_d;         // (double)nbins
    double width;           // xmax - xmin, rounded once (the formula's denominator)
    double inv_width;       // 1 / width rounded: only for the guess of the fast path
    const double *edges;    // device, nbins+1 values (variable axes)
    const ModelSeg *model;  // device, nseg segments (learned)
    int32_t nseg;
    int32_t feature;        // Feature
    double fscale;          // segment coordinate t = feature(x) * fscale
    uint64_t key0;          // feature origin for FEAT_KEY
    double x0;              // feature origin for FEAT_LINEAR
    int32_t lds_model;      // byte offset of the model staged in LDS, -1 if none
    int32_t stride;         // product of (nbins+2) of the lower axes
};

// --------------------------------------------------------------------------
// Fixed-width axis.  The result is defined by the binary64 evaluation
// t = x - xmin, u = nbins * t, v = u / width (each rounded to nearest, no
// fused multiply-add), bin = 1 + trunc(v) clamped to nbins.  The kernel first
// guesses v with a multiply by the rounded reciprocal; that guess differs from
// the correctly rounded quotient by under 3 ulp, so when it lies more than
// 1e-15 * v (about 9 ulp) away from every integer its floor equals floor(v)
// and the division is skipped.  Otherwise the exact division decides.
// --------------------------------------------------------------------------
__device__ __forceinline__ int32_t bin_uniform(double x, const AxisDev &ax)
{
#pragma clang fp contract(off)
    if (x < ax.xmin)
        return 0;
    if (!(x < ax.xmax))
        return ax.nbins + 1;
    double t = x - ax.xmin;
    double u = ax.nbins_d * t;
    double q = u * ax.inv_width;
    double k = __builtin_floor(q);
    double m = q * 1e-15 + 1e-300;
    int32_t b;
    if ((q - k) > m && ((k + 1.0) - q) > m)
        b = (int32_t)k + 1;
    else
        b = (int32_t)(u / ax.width) + 1;
    return b < ax.nbins ? b : ax.nbins;
}

// --------------------------------------------------------------------------
// Variable axis, binary search.  For e[0] <= x < e[nbins], the bin is one
// more than the largest index i with e[i] <= x.  The loop runs
// ceil(log2 nbins) steps for every lane, so a wave never diverges.
// --------------------------------------------------------------------------
__device__ __forceinline__ int32_t search_edges(double x, const double *__restrict__ e,
                                                int32_t base, int32_t len)
{
    // largest i in [base, base+len) with e[i] <= x, given e[base] <= x
    while (len > 1) {
        int32_t half = len >> 1;
        if (!(x < e[base + half]))
            base += half;
        len -= half;
    }
    return base;
}

__device__ __forceinline__ int32_t bin_bsearch(double x, const AxisDev &ax)
{
    if (x < ax.xmin)
        return 0;
    if (!(x < ax.xmax))
        return ax.nbins + 1;
    return search_edges(x, ax.edges, 0, ax.nbins) + 1;
}

// --------------------------------------------------------------------------
// Learned index.  Order-preserving feature of x, monotone non-decreasing in x:
//   FEAT_KEY:    (orderkey(x + 0.0) - key0) >> 11, exact as a double (< 2^53)
//   FEAT_LINEAR: x - x0, rounded
// t = feature * fscale (monotone), segment s = min(trunc(t), nseg - 1),
// z = t - s (monotone within a segment).  The same functions run in the
// training kernels, so training sees exactly the values inference computes.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint64_t order_key(double x)
{
    uint64_t k = (uint64_t)__double_as_longlong(x + 0.0);   // -0.0 -> +0.0
    return (k >> 63) ? ~k : (k | 0x8000000000000000ull);
}

__device__ __forceinline__ double feature_t(double x, const AxisDev &ax)
{
    double f;
    if (ax.feature == FEAT_KEY)
        f = (double)(int64_t)((order_key(x) - ax.key0) >> 11);
    else
        f = x - ax.x0;
    return f * ax.fscale;
}

__device__ __forceinline__ int32_t seg_of(double t, int32_t nseg)
{
    int32_t s = (int32_t)t;   // t >= 0 for x >= e[0]
    return s < nseg - 1 ? s : nseg - 1;
}

__device__ __forceinline__ double model_eval(const ModelSeg &m, double z)
{
    return __builtin_fma(__builtin_fma(m.c, z, m.b), z, m.a);
}

// Bin on a variable axis from the learned model `m` (already loaded, from LDS
// or global memory).  The candidate interval from the segment's bounds always
// holds the bin; when it has one element no edge is read, otherwise a binary
// search over that interval reads the edges.  An empty interval cannot occur
// for a correctly trained model; binary search over all edges answers then.
__device__ __forceinline__ int32_t bin_learned_with(double x, const AxisDev &ax,
                                                    const ModelSeg *__restrict__ model)
{
    if (x < ax.xmin)
        return 0;
    if (!(x < ax.xmax))
        return ax.nbins + 1;
    double t = feature_t(x, ax);
    int32_t s = seg_of(t, ax.nseg);
    double z = t - (double)s;
    ModelSeg m = model[s];
    double p = model_eval(m, z);
    double flo = __builtin_ceil(p + m.clo);
    double fhi = __builtin_floor(p + m.chi);
    int32_t lo = flo < 1.0 ? 1 : (flo > ax.nbins_d ? ax.nbins : (int32_t)flo);
    int32_t hi = fhi > ax.nbins_d ? ax.nbins : (fhi < 1.0 ? 1 : (int32_t)fhi);
    if (lo == hi)
        return lo;
    if (lo > hi)
        return search_edges(x, ax.edges, 0, ax.nbins) + 1;
    // bin in [lo, hi]: e[lo-1] <= x < e[hi]; count edges e[lo..hi-1] <= x
    return search_edges(x, ax.edges, lo - 1, hi - lo + 1) + 1;
}

// Dispatch on the axis kind (uniform across a wave: no divergence).
__device__ __forceinline__ int32_t axis_bin(double x, const AxisDev &ax, const char *smem)
{
    if (ax.kind == AX_UNIFORM)
        return bin_uniform(x, ax);
    if (ax.kind == AX_LEARNED) {
        const ModelSeg *m = ax.lds_model >= 0
                                ? reinterpret_cast<const ModelSeg *>(smem + ax.lds_model)
                                : ax.model;
        return bin_learned_with(x, ax, m);
    }
    return bin_bsearch(x, ax);
}

}  // namespace hg
