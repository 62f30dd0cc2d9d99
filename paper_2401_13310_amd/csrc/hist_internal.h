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

// One segment of the learned index, 16 bytes (one LDS read): over the
// segment-local feature z, y = af + z (b + c z) is evaluated in FP32 and the
// bin provably lies in [ai + ceil(y), ai + floor(y + w)].  c and w are stored
// as IEEE half in cw (c low, w high); the lower-bound offset is folded into af.
struct alignas(16) ModelSeg {
    float af, b;
    int32_t ai;
    uint32_t cw;
};
static_assert(sizeof(ModelSeg) == 16, "ModelSeg layout");

struct AxisDev {
    int32_t nbins;
    int32_t kind;           // AxisKind
    double xmin, xmax;      // range; variable axes: e[0] and e[nbins]
    double nbins_d;         // (double)nbins
    double width;           // xmax - xmin, rounded once (the formula's denominator)
    double guess;           // nbins / width rounded: only for the guess of the fast path
    const double *edges;    // device, nbins+1 values (variable axes)
    const ModelSeg *model;  // device, nseg segments (learned)
    int32_t nseg;
    int32_t feature;        // Feature
    double fscale;          // FEAT_LINEAR: segment coordinate t = (x - x0) * fscale
    double x0;              // FEAT_LINEAR: feature origin
    double margin;          // fixed-width axes: fast-path margin, > 4 ulp of nbins
    uint32_t key0;          // FEAT_KEY: feature origin (a segment boundary)
    uint32_t kmask;         // FEAT_KEY: 2^kshift - 1
    int32_t kshift;         // FEAT_KEY: log2 of the segment width in key units
    float zscale;           // FEAT_KEY: 2^-kshift
    int32_t keypos;         // FEAT_KEY: e[0] > 0, so every in-range x is positive
    int32_t lds_model;      // byte offset of the model staged in LDS, -1 if none
    int32_t stride;         // product of (nbins+2) of the lower axes
    int32_t lds_edges;      // byte offset of the edges staged in LDS, -1 if read from HBM
};

// Variable axes with few edges keep a copy of them in LDS, so the search steps
// read LDS instead of waiting on L2.
constexpr int kStageEdgesMax = 4096;       // edges of one axis
constexpr int kStageEdgesBytes = 32768;    // all staged edges of a histogram

// Which of the first dims axes get their edges staged in LDS: variable axes
// of at most kStageEdgesMax edges, in axis order while the total stays within
// kStageEdgesBytes.  Bit a of the result is axis a.
__host__ __device__ inline uint32_t staged_edges_mask(int dims, const AxisDev *ax)
{
    uint32_t mask = 0;
    int bytes = 0;
    for (int d = 0; d < dims; ++d) {
        const int eb = (ax[d].nbins + 1) * (int)sizeof(double);
        if (ax[d].kind != AX_UNIFORM && ax[d].nbins + 1 <= kStageEdgesMax && bytes + eb <= kStageEdgesBytes) {
            mask |= 1u << d;
            bytes += eb;
        }
    }
    return mask;
}

// Edges as an LDS pointer: a distinct address space, so a staged search can
// never be merged with the HBM one into flat loads.
using lds_f64 = __attribute__((address_space(3))) const double;

__device__ __forceinline__ lds_f64 *lds_edge_ptr(const char *smem, const AxisDev &ax)
{
    return (lds_f64 *)(smem + ax.lds_edges);
}

// --------------------------------------------------------------------------
// Fixed-width axis.  The result is defined by the binary64 evaluation
// t = x - xmin, u = nbins * t, v = u / width (each rounded to nearest, no
// fused multiply-add), bin = 1 + trunc(v) clamped to nbins.  The kernels first
// guess v as q = t * guess with guess = nbins / width rounded: q and v each
// lie within two roundings (relative 2u, u = 2^-53) of the exact nbins t /
// width, so |q - v| < 4.0001 u nbins, below `margin` = 1e-15 (nbins + 1).
// When the fractional part of q is farther than margin from 0 and from 1,
// floor(q) = floor(v) and the division is skipped; otherwise (in practice
// never, for random data) the exact division decides.  The guess is formed
// for every coordinate (clamped to stay finite for out-of-range x) without
// branches, and the division runs only when some lane of the wave needs it.
// --------------------------------------------------------------------------
template <int U>
__device__ __forceinline__ void bins_uniform(const double (&x)[U], const AxisDev &ax,
                                             int32_t (&b)[U], bool (&inr)[U])
{
#pragma clang fp contract(off)
    double t[U];
    bool slow[U];
    bool any_slow = false;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const bool in = !(x[j] < ax.xmin) && x[j] < ax.xmax;
        inr[j] = in;
        t[j] = x[j] - ax.xmin;
        const double q = t[j] * ax.guess;
        const double k = __builtin_floor(q);
        slow[j] = in && !(__builtin_fabs((q - k) - 0.5) < 0.5 - ax.margin);
        any_slow = any_slow || slow[j];
        b[j] = (int32_t)__builtin_fmin(__builtin_fmax(k, 0.0), ax.nbins_d) + 1;
    }
    if (__builtin_amdgcn_ballot_w64(any_slow)) {
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (slow[j])
                b[j] = (int32_t)((ax.nbins_d * t[j]) / ax.width) + 1;
    }
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const int32_t v = b[j] < ax.nbins ? b[j] : ax.nbins;
        b[j] = x[j] < ax.xmin ? 0 : (x[j] < ax.xmax ? v : ax.nbins + 1);
    }
}

// --------------------------------------------------------------------------
// Variable axis, binary search (search_lockstep below with the interval
// [1, nbins]): for e[0] <= x < e[nbins] the bin is one more than the largest
// index i with e[i] <= x, found in ceil(log2 nbins) halving steps.
// --------------------------------------------------------------------------

// --------------------------------------------------------------------------
// Learned index.  Segment s and segment-local coordinate z of x, both
// monotone non-decreasing in x (z within a segment):
//   FEAT_KEY:    f = top 32 bits of the order-preserving integer key of x
//                (sign, exponent, 20 mantissa bits -- close to log2|x|) minus
//                key0; s = f >> kshift, z = (f & kmask) * 2^-kshift.  Segment
//                boundaries are binade boundaries or finer, where the key is
//                linear in x.
//   FEAT_LINEAR: t = (x - x0) * fscale, s = min(trunc(t), nseg - 1),
//                z = t - s.
// The training kernels use the same functions, so they see exactly the
// values inference computes.
// --------------------------------------------------------------------------
__device__ __forceinline__ uint32_t order_key32(double x)
{
    const uint32_t hi = (uint32_t)((uint64_t)__double_as_longlong(x + 0.0) >> 32);   // -0 -> +0
    return (hi >> 31) ? ~hi : (hi | 0x80000000u);
}

// f of the key feature; x must be in [e[0], e[nbins]).
__device__ __forceinline__ uint32_t key_feature(double x, const AxisDev &ax)
{
    uint32_t k;
    if (ax.keypos)
        k = (uint32_t)((uint64_t)__double_as_longlong(x) >> 32) | 0x80000000u;
    else
        k = order_key32(x);
    return k - ax.key0;
}

// The segments cover the keys of [e[0], e[nbins]], so for in-range x the
// clamp of s never acts and z is the key's offset in its segment; the clamp
// keeps the model read in bounds for any other x (whose result is discarded).
__device__ __forceinline__ void key_seg(uint32_t f, const AxisDev &ax, int32_t &s, float &z)
{
#pragma clang fp contract(off)
    const uint32_t sf = f >> ax.kshift;
    s = (int32_t)(sf < (uint32_t)(ax.nseg - 1) ? sf : (uint32_t)(ax.nseg - 1));
    z = (float)(f & ax.kmask) * ax.zscale;
}

__device__ __forceinline__ void linear_seg(double x, const AxisDev &ax, int32_t &s, float &z)
{
#pragma clang fp contract(off)   // t and z rounded exactly as in training
    const double t = (x - ax.x0) * ax.fscale;
    // the clamp only matters outside [e[0], e[nbins]) (and for NaN): it keeps
    // the segment index in [0, nseg) for any x
    const double tc = __builtin_fmin(__builtin_fmax(t, 0.0), (double)(ax.nseg - 1));
    s = (int32_t)tc;
    z = (float)(t - (double)s);
}

__device__ __forceinline__ void seg_and_z(double x, const AxisDev &ax, int32_t &s, float &z)
{
    if (ax.feature == FEAT_KEY)
        key_seg(key_feature(x, ax), ax, s, z);
    else
        linear_seg(x, ax, s, z);
}

// seg_and_z of U coordinates, with the (wave-uniform) choice of feature taken
// once for the batch.
template <int U>
__device__ __forceinline__ void seg_and_z_batch(const double (&x)[U], const AxisDev &ax,
                                                int32_t (&s)[U], float (&z)[U])
{
    if (ax.feature == FEAT_KEY) {
        if (ax.keypos) {
            // in-range x is positive, so setting the sign bit of its high
            // word is adding 2^31 (other x get a discarded result)
            const uint32_t kadd = 0x80000000u - ax.key0;
#pragma unroll
            for (int j = 0; j < U; ++j)
                key_seg((uint32_t)((uint64_t)__double_as_longlong(x[j]) >> 32) + kadd, ax, s[j], z[j]);
        } else {
#pragma unroll
            for (int j = 0; j < U; ++j)
                key_seg(order_key32(x[j]) - ax.key0, ax, s[j], z[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j < U; ++j)
            linear_seg(x[j], ax, s[j], z[j]);
    }
}

__device__ __forceinline__ float half_lo(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v & 0xFFFFu));
}
__device__ __forceinline__ float half_hi(uint32_t v)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(v >> 16));
}

// y = af + z (b + c z), two FP32 fused multiply-adds (the same code in
// training and inference).
__device__ __forceinline__ float model_eval(const ModelSeg &m, float z)
{
    return __builtin_fmaf(__builtin_fmaf(half_lo(m.cw), z, m.b), z, m.af);
}

// Candidate intervals [lo, hi] of the bins of U coordinates on a variable
// axis from the learned model (in LDS).  Underflow and overflow give lo = hi =
// 0 or nbins+1.  The interval always holds the bin (see learned.hip); an empty
// interval cannot occur for a correctly trained model, and the full range
// [1, nbins] is searched then.  Branch-free: the segment of every coordinate
// (clamped into the model for out-of-range x) is read before any is used, so
// the U LDS reads overlap.
template <int U>
__device__ __forceinline__ void learned_intervals(const double (&x)[U], const AxisDev &ax,
                                                  const ModelSeg *__restrict__ model,
                                                  int32_t (&lo)[U], int32_t (&hi)[U],
                                                  bool (&inr)[U])
{
    int32_t s[U];
    float z[U];
    seg_and_z_batch<U>(x, ax, s, z);
    bool bad = false;
    ModelSeg m[U];
#pragma unroll
    for (int j = 0; j < U; ++j)
        m[j] = model[s[j]];
    // all U reads in flight before the first is used
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const float y = model_eval(m[j], z[j]);
        // clamp before converting so ai + offset stays in int32 (an infinite
        // width becomes the whole axis)
        const float ylo = __builtin_fminf(__builtin_fmaxf(__builtin_ceilf(y), -0x1p30f), 0x1p30f);
        const float yhi =
            __builtin_fminf(__builtin_fmaxf(__builtin_floorf(y + half_hi(m[j].cw)), -0x1p30f), 0x1p30f);
        // the interval may reach past [1, nbins] near the ends of the axis;
        // the searches read the edges clamped to e[0] .. e[nbins], which for
        // an in-range x decides like edges at -inf and +inf beyond them
        const int32_t a = (int32_t)((uint32_t)m[j].ai + (uint32_t)(int32_t)ylo);
        const int32_t b = (int32_t)((uint32_t)m[j].ai + (uint32_t)(int32_t)yhi);
        const bool under = x[j] < ax.xmin;
        const bool in = !under && x[j] < ax.xmax;   // false for NaN
        const int32_t flow = under ? 0 : ax.nbins + 1;
        inr[j] = in;
        lo[j] = in ? a : flow;
        hi[j] = in ? b : flow;
        bad = bad || lo[j] > hi[j];
    }
    if (__builtin_amdgcn_ballot_w64(bad)) {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (lo[j] > hi[j]) {
                lo[j] = 1;
                hi[j] = ax.nbins;
            }
        }
    }
}

// Edge index clamped to the array: for an in-range x, e[0] <= x < e[nbins],
// so a clamped read decides exactly like the virtual edges -inf below 0 and
// +inf above nbins.
__device__ __forceinline__ int32_t edge_index(int32_t k, int32_t nbins)
{
    return __builtin_elementwise_min(__builtin_elementwise_max(k, 0), nbins);
}

// Resolves U searches at once: each bin is known to lie in [lo, hi] with
// e[lo-1] <= x < e[hi].  Intervals of two candidates (the common case after
// the learned index) take one compare with e[lo]; wider ones halve per step.
// The edge loads of all U events of a step are issued together so their
// latencies overlap; in the halving loop unconditionally (a finished search
// reads a valid clamped edge and ignores it: in a plain binary search nearly
// every search takes the same number of steps, and predicated loads would be
// waited for one by one).  Edge indices are clamped to [0, nbins].
template <int U, typename EP>
__device__ __forceinline__ void search_lockstep(const double (&x)[U], EP e, int32_t nbins,
                                                int32_t (&lo)[U], int32_t (&hi)[U])
{
    bool wide = false;
#pragma unroll
    for (int j = 0; j < U; ++j)
        wide = wide || hi[j] - lo[j] > 1;
    if (!wide) {
        double ev[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (hi[j] > lo[j])
                ev[j] = e[edge_index(lo[j], nbins)];
#pragma unroll
        for (int j = 0; j < U; ++j)
            if (hi[j] > lo[j])
                lo[j] += (x[j] < ev[j]) ? 0 : 1;
        return;
    }
    bool open = false;
#pragma unroll
    for (int j = 0; j < U; ++j)
        open = open || lo[j] < hi[j];
    while (open) {
        double ev[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            ev[j] = e[edge_index(((lo[j] + hi[j] + 1) >> 1) - 1, nbins)];
        open = false;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            if (lo[j] < hi[j]) {
                const int32_t m = (lo[j] + hi[j] + 1) >> 1;
                if (!(x[j] < ev[j]))
                    lo[j] = m;
                else
                    hi[j] = m - 1;
                open = open || lo[j] < hi[j];
            }
        }
    }
}

// The halving search of one coordinate (same steps as search_lockstep).
template <typename EP>
__device__ __forceinline__ void search_one(double x, EP e, int32_t nbins, int32_t &lo, int32_t &hi)
{
    while (lo < hi) {
        const int32_t m = (lo + hi + 1) >> 1;
        if (!(x < e[edge_index(m - 1, nbins)]))
            lo = m;
        else
            hi = m - 1;
    }
}

// Bins of U coordinates on one axis, in two halves so that a caller can issue
// other memory loads in between: axis_bins_begin bounds every bin to [lo, hi]
// (a single value for fixed-width axes and under/overflow) and issues the edge
// loads of the first halving step; axis_bins_finish completes the searches.
// Global loads complete in issue order, so loads issued between the two halves
// (the next batch of events) are not waited for by the first step.  KIND is
// the axis kind when known at compile time, or -1 to dispatch on ax.kind
// (uniform across a wave).  `smem` is the kernel's dynamic LDS array, holding
// the staged learned models.
// The edge loads of the first halving step of U searches, only for the
// coordinates whose bin is not known yet (after the learned index, most):
// random gathers cost cache bandwidth even when they hit.
template <int U, typename EP>
__device__ __forceinline__ void first_step_loads(EP e, int32_t nbins, const int32_t (&lo)[U],
                                                 const int32_t (&hi)[U], double (&ev)[U])
{
#pragma unroll
    for (int j = 0; j < U; ++j) {
        ev[j] = 0.0;
        if (lo[j] < hi[j])
            ev[j] = e[edge_index(((lo[j] + hi[j] + 1) >> 1) - 1, nbins)];
    }
}

// The searches after the first step.  After the learned index one step usually
// decides every bin: the rest is searched one coordinate at a time, which keeps
// this rare path from holding registers for all U searches at once.
template <int U, typename EP>
__device__ __forceinline__ void finish_searches(const double (&x)[U], EP e, int32_t nbins,
                                                bool learned, int32_t (&lo)[U], int32_t (&hi)[U])
{
    if (learned) {
#pragma unroll
        for (int j = 0; j < U; ++j)
            search_one(x[j], e, nbins, lo[j], hi[j]);
    } else {
        search_lockstep<U>(x, e, nbins, lo, hi);
    }
}

// Where a variable axis's edges are read from: HBM only (kernels whose kind
// set excludes staged edges), or LDS whenever ax.lds_edges >= 0.
enum EdgeSource : int32_t { EDGES_HBM = 0, EDGES_ANY = 1 };

template <int U, int KIND = -1, int ES = EDGES_ANY>
__device__ __forceinline__ void axis_bins_begin(const double (&x)[U], const AxisDev &ax,
                                                const char *smem, int32_t (&lo)[U],
                                                int32_t (&hi)[U], double (&ev)[U], bool (&inr)[U])
{
    const int kind = KIND >= 0 ? KIND : ax.kind;
    if (kind == AX_UNIFORM) {
        bins_uniform<U>(x, ax, lo, inr);
#pragma unroll
        for (int j = 0; j < U; ++j)
            hi[j] = lo[j];
        return;
    }
    if (kind == AX_LEARNED) {
        // kernels always stage the model in LDS; deriving the pointer from the
        // LDS array keeps these reads ds_read instructions (not flat loads)
        learned_intervals<U>(x, ax, reinterpret_cast<const ModelSeg *>(smem + ax.lds_model), lo, hi,
                             inr);
    } else {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool under = x[j] < ax.xmin;
            inr[j] = !under && x[j] < ax.xmax;
            const int32_t flow = under ? 0 : ax.nbins + 1;
            lo[j] = inr[j] ? 1 : flow;
            hi[j] = inr[j] ? ax.nbins : flow;
        }
    }
    if (ES == EDGES_ANY && ax.lds_edges >= 0)
        first_step_loads<U>(lds_edge_ptr(smem, ax), ax.nbins, lo, hi, ev);
    else
        first_step_loads<U>(ax.edges, ax.nbins, lo, hi, ev);
}

template <int U, int KIND = -1, int ES = EDGES_ANY>
__device__ __forceinline__ void axis_bins_finish(const double (&x)[U], const AxisDev &ax,
                                                 const char *smem, int32_t (&lo)[U], int32_t (&hi)[U],
                                                 const double (&ev)[U], int32_t (&b)[U])
{
    const int kind = KIND >= 0 ? KIND : ax.kind;
    if (kind != AX_UNIFORM) {
        bool open = false;
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool step = lo[j] < hi[j];
            const int32_t m = (lo[j] + hi[j] + 1) >> 1;
            const bool ge = !(x[j] < ev[j]);
            lo[j] = (step && ge) ? m : lo[j];
            hi[j] = (step && !ge) ? m - 1 : hi[j];
            open = open || lo[j] < hi[j];
        }
        if (__builtin_amdgcn_ballot_w64(open)) {
            if (ES == EDGES_ANY && ax.lds_edges >= 0)
                finish_searches<U>(x, lds_edge_ptr(smem, ax), ax.nbins, kind == AX_LEARNED, lo, hi);
            else
                finish_searches<U>(x, ax.edges, ax.nbins, kind == AX_LEARNED, lo, hi);
        }
    }
#pragma unroll
    for (int j = 0; j < U; ++j)
        b[j] = lo[j];
}

template <int U, int KIND = -1>
__device__ __forceinline__ void axis_bins(const double (&x)[U], const AxisDev &ax,
                                          const char *smem, int32_t (&b)[U])
{
    int32_t lo[U], hi[U];
    double ev[U];
    bool inr[U];
    axis_bins_begin<U, KIND>(x, ax, smem, lo, hi, ev, inr);
    axis_bins_finish<U, KIND>(x, ax, smem, lo, hi, ev, b);
}

// Bins of U coordinates on an axis of any kind whose edges (if any) are staged
// in LDS: every step reads LDS, so nothing here waits on the event loads in
// flight, and one axis is finished before the next is begun (only one axis's
// search state is live at a time).  MAY_UNIFORM false: the axis is known to be
// variable.
template <int U, bool MAY_UNIFORM>
__device__ __forceinline__ void axis_bins_staged(const double (&x)[U], const AxisDev &ax,
                                                 const char *smem, int32_t (&b)[U], bool (&inr)[U])
{
    if (MAY_UNIFORM && ax.kind == AX_UNIFORM) {
        bins_uniform<U>(x, ax, b, inr);
        return;
    }
    int32_t lo[U], hi[U];
    if (ax.kind == AX_LEARNED) {
        learned_intervals<U>(x, ax, reinterpret_cast<const ModelSeg *>(smem + ax.lds_model), lo, hi,
                             inr);
    } else {
#pragma unroll
        for (int j = 0; j < U; ++j) {
            const bool under = x[j] < ax.xmin;
            inr[j] = !under && x[j] < ax.xmax;
            const int32_t flow = under ? 0 : ax.nbins + 1;
            lo[j] = inr[j] ? 1 : flow;
            hi[j] = inr[j] ? ax.nbins : flow;
        }
    }
    search_lockstep<U>(x, lds_edge_ptr(smem, ax), ax.nbins, lo, hi);
#pragma unroll
    for (int j = 0; j < U; ++j)
        b[j] = lo[j];
}

// Copies the learned models and the staged edges of the first D axes to
// their LDS offsets.
template <int D>
__device__ __forceinline__ void stage_axes(const AxisDev (&ax)[kMaxDims], char *smem)
{
#pragma unroll
    for (int a = 0; a < D; ++a) {
        if (ax[a].kind == AX_LEARNED && ax[a].lds_model >= 0) {
            const double *src = reinterpret_cast<const double *>(ax[a].model);
            double *dst = reinterpret_cast<double *>(smem + ax[a].lds_model);
            const int nd = ax[a].nseg * (int)(sizeof(ModelSeg) / sizeof(double));
            for (int i = threadIdx.x; i < nd; i += blockDim.x)
                dst[i] = src[i];
        }
        if (ax[a].kind != AX_UNIFORM && ax[a].lds_edges >= 0) {
            double *dst = reinterpret_cast<double *>(smem + ax[a].lds_edges);
            for (int i = threadIdx.x; i <= ax[a].nbins; i += blockDim.x)
                dst[i] = ax[a].edges[i];
        }
    }
}

// Kernel specializations by the kinds of the axes.
// KS_STAGED: some axis is variable and every variable axis has its edges in
// LDS (any dims, kinds dispatched at run time).
enum KindSet : int32_t { KS_UNIFORM = 0, KS_LEARNED1 = 1, KS_BSEARCH1 = 2, KS_MIXED = 3, KS_STAGED = 4 };
constexpr int kKindSets = 5;

template <int KS>
__host__ __device__ constexpr int kind_of_set()
{
    return KS == KS_UNIFORM ? AX_UNIFORM
                            : (KS == KS_LEARNED1 ? AX_LEARNED : (KS == KS_BSEARCH1 ? AX_BSEARCH : -1));
}

// Single coordinate.
__device__ __forceinline__ int32_t axis_bin(double x, const AxisDev &ax, const char *smem)
{
    double xs[1] = {x};
    int32_t b[1];
    axis_bins<1>(xs, ax, smem, b);
    return b[0];
}

}  // namespace hg
