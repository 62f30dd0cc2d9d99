// multi.hip -- one pass over shared event columns that fills several
// histograms, each behind its own event filter and computed columns.
//
// The paper fills one histogram per pass and names several histograms per
// event loop as future work (arXiv:2401.13310 Sec. 6).  Its RDataFrame usage
// (Sec. 3, Listing 1) puts a Filter and a Define in front of the histogram
// fill, and its CUDA kernel skips events whose bin was marked invalid
// (Sec. 3.2).  Here the columns of a batch of events are read from HBM once;
// for every member histogram the kernel then evaluates the member's filter,
// coordinate and weight programs on those values, finds the bins (Sec. 3.1)
// and accumulates into the member's private LDS copy (Sec. 3.2 two-stage
// fill) or, for a member too large for the LDS left, with global atomics.
// Statistics sums and entry counts are kept per member; filtered-out events
// count nowhere.
//
// Programs are postfix expressions over binary64 values (hist.h lists the
// operations).  The stack depth before every operation is fixed by the
// program, so the host stores it with the operation and the kernel dispatches
// on (depth, operation): every stack slot is then a register named at compile
// time.  Programs and depths are the same for every lane, so the dispatch is
// scalar branching, paid once per wave and event slot.
#include "../../include/hist.h"
#include "device_common.h"
#include "kernels.h"
#include "plan.h"

#include <algorithm>
#include <cstring>
#include <vector>

namespace hg {

constexpr int kMultiMembers = 16;
constexpr int kMultiCols = 8;
constexpr int kExprStack = 6;       // at most 8 (one vector of registers)
constexpr int kExprMaxOps = 32;
constexpr int kMultiU = 1;           // events per thread per batch
constexpr int kMultiStatsBytes = 96; // per member: kMaxStats doubles, kept and in-range counts

struct ExprOp {
    int32_t code;    // hist_opcode
    int32_t sp;      // stack depth before the operation
    int32_t col;     // HIST_OP_COL: column index
    int32_t pad;
    double value;    // HIST_OP_CONST
};

struct ExprRef {
    int32_t first;   // index of the first operation
    int32_t nops;    // 0: absent
};

struct MultiMember {
    AxisDev ax[kMaxDims];
    int32_t dims;
    int32_t nstats;
    int32_t lds_win;      // byte offset of the LDS copy of the histogram, -1: global atomics
    int32_t copies;       // interleaved copies in that LDS region
    int32_t lds_stats;    // byte offset of the statistics partials, kept and in-range counts
    int32_t lds_tstats;   // byte offset of per-thread sums [nsums][threads], -1: per-wave reduction
    int32_t nsums;        // sums per event: all statistics (weighted) or all but the counts
    int32_t total_bins;
    ExprRef filter, coord[kMaxDims], weight;
    int32_t coord_col[kMaxDims];   // coordinate read straight from this column, -1: program
    int32_t weight_col;            // weight column, -1: program or unit weights
    int32_t weighted;              // a weight program or column
    int32_t lean;                  // one fixed-width axis read from a column, unit weights, no
                                   // filter, LDS copy and per-thread sums: the short path
    uint64_t *cnt;
    double *sumw, *sumw2, *stats;
    uint64_t *entries;
};

// Members and operations are read through the constant address space: every
// field is then a scalar load (the values are the same for every lane).
using ConstMultiMember = __attribute__((address_space(4))) const MultiMember;
using ConstExprOp = __attribute__((address_space(4))) const ExprOp;

struct MultiArgs {
    const MultiMember *members;
    const ExprOp *ops;
    const void *cols[kMultiCols];
    int32_t k;
    int32_t ncols;
    int64_t n;
    int64_t per_block;
};

// ---------------------------------------------------------------- programs --

__device__ __forceinline__ double truth(bool b) { return b ? 1.0 : 0.0; }

// Programs run on one event per lane with the stack held in registers as one
// vector: every operation reads its operands and writes its result at the
// (uniform) stack depth the host recorded, i.e. an indexed register move
// each, so the operation's own code is the only thing the dispatch selects.
using dvec8 = double __attribute__((ext_vector_type(8)));

template <int NC>
__device__ __forceinline__ double run_expr(ConstExprOp *ops, ExprRef e, dvec8 &stk, const dvec8 &cv)
{
#pragma clang fp contract(off)
    for (int pc = 0; pc < e.nops; ++pc) {
        const ExprOp op = *(const ExprOp *)&ops[e.first + pc];
        const int sp = op.sp;
        const int code = op.code;
        if (code == HIST_OP_CONST) {
            stk[sp] = op.value;
        } else if (code == HIST_OP_COL) {
            stk[sp] = cv[op.col];
        } else if (code == HIST_OP_NEG || code == HIST_OP_ABS || code == HIST_OP_SQRT ||
                   code == HIST_OP_NOT) {
            const double a = stk[sp - 1];
            stk[sp - 1] = code == HIST_OP_NEG   ? -a
                          : code == HIST_OP_ABS ? __builtin_fabs(a)
                          : code == HIST_OP_NOT ? truth(a == 0.0)
                                                : __builtin_sqrt(a);
        } else if (code == HIST_OP_SELECT) {
            const double c = stk[sp - 3], a = stk[sp - 2], b = stk[sp - 1];
            stk[sp - 3] = c != 0.0 ? a : b;
        } else {
            const double a = stk[sp - 2], b = stk[sp - 1];
            double v;
            switch (code) {
            case HIST_OP_ADD: v = a + b; break;
            case HIST_OP_SUB: v = a - b; break;
            case HIST_OP_MUL: v = a * b; break;
            case HIST_OP_DIV: v = a / b; break;
            case HIST_OP_MIN: v = b < a ? b : a; break;
            case HIST_OP_MAX: v = a < b ? b : a; break;
            case HIST_OP_LT: v = truth(a < b); break;
            case HIST_OP_LE: v = truth(a <= b); break;
            case HIST_OP_GT: v = truth(a > b); break;
            case HIST_OP_GE: v = truth(a >= b); break;
            case HIST_OP_EQ: v = truth(a == b); break;
            case HIST_OP_NE: v = truth(a != b); break;
            case HIST_OP_AND: v = truth(a != 0.0 && b != 0.0); break;
            default: v = truth(a != 0.0 || b != 0.0); break;   // HIST_OP_OR
            }
            stk[sp - 2] = v;
        }
    }
    return stk[0];
}

// ------------------------------------------------------------------ kernel --

// Statistics terms of one event of a member with `dims` axes, in the order of
// the statistics array (every index fixed at compile time).
__device__ __forceinline__ void member_stats_add(double (&st)[kMaxStats], const double (&x)[kMaxDims],
                                                 double w, int dims)
{
#pragma clang fp contract(off)
    st[0] += w;
    st[1] += w * w;
    const double w0 = w * x[0];
    st[2] += w0;
    st[3] += w0 * x[0];
    if (dims > 1) {
        const double w1 = w * x[1];
        st[4] += w1;
        st[5] += w1 * x[1];
        st[6] += w0 * x[1];
        if (dims > 2) {
            const double w2 = w * x[2];
            st[7] += w2;
            st[8] += w2 * x[2];
            st[9] += w0 * x[2];
            st[10] += w1 * x[2];
        }
    }
}

// Bins of U coordinates on one axis of a member: the fixed-width formula, or
// a binary search over the edges (staged in LDS when the plan put them
// there).  Learned indexes are not used in these passes: the plan turns such
// axes into binary-search axes, which keeps the per-member code small.
template <int U>
__device__ __forceinline__ void member_axis_bins(const double (&x)[U], const AxisDev &ax,
                                                 const char *smem, int32_t (&b)[U], bool (&inr)[U])
{
    if (ax.kind == AX_UNIFORM) {
        bins_uniform<U>(x, ax, b, inr);
        return;
    }
    int32_t lo[U], hi[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        const bool under = x[j] < ax.xmin;
        inr[j] = !under && x[j] < ax.xmax;
        const int32_t flow = under ? 0 : ax.nbins + 1;
        lo[j] = inr[j] ? 1 : flow;
        hi[j] = inr[j] ? ax.nbins : flow;
    }
    if (ax.lds_edges >= 0)
        search_lockstep<U>(x, lds_edge_ptr(smem, ax), ax.nbins, lo, hi);
    else
        search_lockstep<U>(x, ax.edges, ax.nbins, lo, hi);
#pragma unroll
    for (int j = 0; j < U; ++j)
        b[j] = lo[j];
}

template <typename T>
__device__ __forceinline__ T load_col(const void *p, int64_t i)
{
    return __builtin_nontemporal_load(static_cast<const T *>(p) + i);
}

// Wave sum of a double, then one LDS atomic by the wave's first lane.
__device__ __forceinline__ void wave_add_lds(double v, double *dst)
{
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1)
        v += __shfl_xor(v, off, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0 && v != 0.0)
        lds_add_f64(dst, v);
}

// NC: columns held in registers (at least the plan's ncols).
template <typename T, int NC>
__global__ void __launch_bounds__(kMaxThreads) multi_fill_kernel(const MultiArgs A)
{
    constexpr int U = kMultiU;
    extern __shared__ __align__(16) char smem[];
    ConstMultiMember *mem = (ConstMultiMember *)A.members;
    ConstExprOp *ops = (ConstExprOp *)A.ops;
    const int tid = threadIdx.x, nthr = blockDim.x;

    // stage small edge arrays, zero the statistics and windows
    for (int m = 0; m < A.k; ++m) {
        const MultiMember &M = *(const MultiMember *)&mem[m];
        for (int a = 0; a < M.dims; ++a) {
            const AxisDev &ax = M.ax[a];
            if (ax.kind != AX_UNIFORM && ax.lds_edges >= 0) {
                double *dst = reinterpret_cast<double *>(smem + ax.lds_edges);
                for (int i = tid; i <= ax.nbins; i += nthr)
                    dst[i] = ax.edges[i];
            }
        }
        uint32_t *st = reinterpret_cast<uint32_t *>(smem + M.lds_stats);
        for (int i = tid; i < kMultiStatsBytes / 4; i += nthr)
            st[i] = 0u;
        if (M.lds_tstats >= 0) {
            double *ts = reinterpret_cast<double *>(smem + M.lds_tstats);
            for (int i = tid; i < M.nsums * nthr; i += nthr)
                ts[i] = 0.0;
        }
        if (M.lds_win >= 0) {
            uint32_t *win = reinterpret_cast<uint32_t *>(smem + M.lds_win);
            const int words = M.total_bins * M.copies * (M.weighted ? 4 : 1);
            for (int i = tid; i < words; i += nthr)
                win[i] = 0u;
        }
    }
    __syncthreads();

    const int64_t start = (int64_t)blockIdx.x * A.per_block;
    const int64_t end = start + A.per_block < A.n ? start + A.per_block : A.n;
    static_assert(U == 1, "programs run on one event per lane");
    static_assert(kExprStack <= 8 && NC <= 8, "stack and columns fit one 8-wide vector");
    dvec8 stk = 0.0;

    // every column of a batch is read once, for all members; the next batch
    // is requested before the current one is processed
    T nv[NC][U];
    auto load_batch = [&](int64_t b) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int64_t i = b + (int64_t)j * nthr + tid;
                nv[c][j] = (c < A.ncols && i < end) ? load_col<T>(A.cols[c], i) : T(0);
            }
        }
    };
    if (start < end)
        load_batch(start);
    for (int64_t base = start; base < end; base += (int64_t)nthr * U) {
        dvec8 cv = 0.0;
        bool ok[U];
#pragma unroll
        for (int j = 0; j < U; ++j)
            ok[j] = base + (int64_t)j * nthr + tid < end;
#pragma unroll
        for (int c = 0; c < NC; ++c)
            cv[c] = (double)nv[c][0];
        if (base + (int64_t)nthr * U < end)
            load_batch(base + (int64_t)nthr * U);
        for (int m = 0; m < A.k; ++m) {
            const MultiMember &M = *(const MultiMember *)&mem[m];
            if (M.lean) {
                // a plain projection: bin, count in LDS, sums of x and x^2
                const double xs[1] = {cv[M.coord_col[0]]};
                int32_t b[1];
                bool inr[1];
                bins_uniform<1>(xs, M.ax[0], b, inr);
                if (ok[0])
                    lds_add_u32(reinterpret_cast<uint32_t *>(smem + M.lds_win) +
                                    ((uint32_t)b[0] * (uint32_t)M.copies + (uint32_t)(tid % M.copies)), 1u);
                const bool take = ok[0] && inr[0];
                const uint32_t nk = (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(ok[0]));
                const uint32_t ni = (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(take));
                if ((tid & (kWave - 1)) == 0) {
                    uint32_t *lcnt = reinterpret_cast<uint32_t *>(
                        reinterpret_cast<double *>(smem + M.lds_stats) + kMaxStats);
                    if (nk)
                        lds_add_u32(&lcnt[0], nk);
                    if (ni)
                        lds_add_u32(&lcnt[1], ni);
                }
                const double xm = take ? xs[0] : 0.0;
                double *ts = reinterpret_cast<double *>(smem + M.lds_tstats) + tid;
                ts[0] += xm;
                ts[nthr] += xm * xm;
                continue;
            }
            bool keep[U];
            {
                double f[U];
                if (M.filter.nops > 0) {
                    f[0] = run_expr<NC>(ops, M.filter, stk, cv);
#pragma unroll
                    for (int j = 0; j < U; ++j)
                        keep[j] = ok[j] && f[j] != 0.0;
                } else {
#pragma unroll
                    for (int j = 0; j < U; ++j)
                        keep[j] = ok[j];
                }
            }
            double x[kMaxDims][U];
#pragma unroll
            for (int a = 0; a < kMaxDims; ++a) {
                if (a < M.dims && M.coord[a].nops > 0)
                    x[a][0] = run_expr<NC>(ops, M.coord[a], stk, cv);
                else
                    x[a][0] = a < M.dims ? cv[M.coord_col[a]] : 0.0;
            }
            const bool weighted = M.weighted != 0;
            double w[U];
            if (M.weight.nops > 0) {
                w[0] = run_expr<NC>(ops, M.weight, stk, cv);
            } else if (weighted) {
                w[0] = cv[M.weight_col];
            } else {
#pragma unroll
                for (int j = 0; j < U; ++j)
                    w[j] = 1.0;
            }
            // bins on every axis of the member (kinds are uniform)
            int32_t g[U];
            bool inside[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                g[j] = 0;
                inside[j] = true;
            }
#pragma unroll
            for (int a = 0; a < kMaxDims; ++a) {
                if (a < M.dims) {
                    int32_t b[U];
                    bool inr[U];
                    member_axis_bins<U>(x[a], M.ax[a], smem, b, inr);
#pragma unroll
                    for (int j = 0; j < U; ++j) {
                        g[j] += a == 0 ? b[j] : b[j] * M.ax[a].stride;
                        inside[j] = inside[j] && inr[j];
                    }
                }
            }
            // accumulate
#pragma unroll
            for (int j = 0; j < U; ++j) {
                if (!keep[j])
                    continue;
                if (M.lds_win >= 0) {
                    const uint32_t idx = (uint32_t)g[j] * (uint32_t)M.copies + (uint32_t)(tid % M.copies);
                    if (weighted) {
                        double *s = reinterpret_cast<double *>(smem + M.lds_win);
                        lds_add_f64(&s[idx], w[j]);
                        lds_add_f64(&s[(uint32_t)M.total_bins * M.copies + idx], w[j] * w[j]);
                    } else {
                        lds_add_u32(reinterpret_cast<uint32_t *>(smem + M.lds_win) + idx, 1u);
                    }
                } else if (weighted) {
                    gl_add_f64(&M.sumw[g[j]], w[j]);
                    gl_add_f64(&M.sumw2[g[j]], w[j] * w[j]);
                } else {
                    gl_add_u64(&M.cnt[g[j]], 1ull);
                }
            }
            // statistics of the kept in-range events: counts by wave votes,
            // sums into per-thread LDS partials (or a wave reduction when the
            // plan had no room for them)
            double st[kMaxStats];
#pragma unroll
            for (int s = 0; s < kMaxStats; ++s)
                st[s] = 0.0;
            uint32_t nkept = 0, nin = 0;
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const bool take = keep[j] && inside[j];
                nkept += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(keep[j]));
                nin += (uint32_t)__builtin_popcountll(__builtin_amdgcn_ballot_w64(take));
                double xm[kMaxDims];
#pragma unroll
                for (int a = 0; a < kMaxDims; ++a)
                    xm[a] = take ? x[a][j] : 0.0;
                member_stats_add(st, xm, take ? w[j] : 0.0, M.dims);
            }
            double *lst = reinterpret_cast<double *>(smem + M.lds_stats);
            uint32_t *lcnt = reinterpret_cast<uint32_t *>(lst + kMaxStats);
            if ((tid & (kWave - 1)) == 0) {
                if (nkept)
                    lds_add_u32(&lcnt[0], nkept);
                if (nin)
                    lds_add_u32(&lcnt[1], nin);
            }
            const int s0 = weighted ? 0 : 2;   // unit weights: w and w^2 are the count
            if (M.lds_tstats >= 0) {
                double *ts = reinterpret_cast<double *>(smem + M.lds_tstats) + tid;
#pragma unroll
                for (int s = 0; s < kMaxStats; ++s)
                    if (s >= s0 && s < M.nstats)
                        ts[(s - s0) * nthr] += st[s];
            } else {
#pragma unroll
                for (int s = 0; s < kMaxStats; ++s)
                    if (s >= s0 && s < M.nstats)
                        wave_add_lds(st[s], &lst[s]);
            }
        }
    }
    __syncthreads();
    // per-thread sums -> the member's statistics partials (once per block)
    for (int m = 0; m < A.k; ++m) {
        const MultiMember &M = *(const MultiMember *)&mem[m];
        if (M.lds_tstats < 0)
            continue;
        const double *ts = reinterpret_cast<const double *>(smem + M.lds_tstats);
        double *lst = reinterpret_cast<double *>(smem + M.lds_stats);
        const int s0 = M.weighted ? 0 : 2;
        for (int s = s0; s < M.nstats; ++s)
            wave_add_lds(ts[(s - s0) * nthr + tid], &lst[s]);
    }
    __syncthreads();

    // merge: LDS copies into the member histograms, statistics, kept counts
    for (int m = 0; m < A.k; ++m) {
        const MultiMember &M = *(const MultiMember *)&mem[m];
        const bool weighted = M.weighted != 0;
        if (M.lds_win >= 0) {
            const int C = M.copies;
            if (weighted) {
                const double *s = reinterpret_cast<const double *>(smem + M.lds_win);
                const int n1 = M.total_bins * C;
                for (int l = tid; l < M.total_bins; l += nthr) {
                    double a = 0.0, b = 0.0;
                    for (int c = 0; c < C; ++c) {
                        a += s[l * C + c];
                        b += s[n1 + l * C + c];
                    }
                    if (a != 0.0 || b != 0.0) {
                        gl_add_f64(&M.sumw[l], a);
                        gl_add_f64(&M.sumw2[l], b);
                    }
                }
            } else {
                const uint32_t *s = reinterpret_cast<const uint32_t *>(smem + M.lds_win);
                for (int l = tid; l < M.total_bins; l += nthr) {
                    uint32_t a = 0;
                    for (int c = 0; c < C; ++c)
                        a += s[l * C + c];
                    if (a)
                        gl_add_u64(&M.cnt[l], a);
                }
            }
        }
        const double *lst = reinterpret_cast<const double *>(smem + M.lds_stats);
        const uint32_t *lcnt = reinterpret_cast<const uint32_t *>(lst + kMaxStats);
        const int s0 = weighted ? 0 : 2;
        if (tid >= s0 && tid < M.nstats && lst[tid] != 0.0)
            gl_add_f64(&M.stats[tid], lst[tid]);
        if (!weighted && tid < 2 && lcnt[1])
            gl_add_f64(&M.stats[tid], (double)lcnt[1]);
        if (tid == nthr - 1 && lcnt[0])
            gl_add_u64(M.entries, lcnt[0]);
    }
}

}  // namespace hg

// -------------------------------------------------------------------- host --

using namespace hg;

struct hist_multi_s {
    int k = 0;
    int ncols = 0;
    hist_dtype dtype = HIST_F64;
    int device = 0;
    int num_cu = 256;
    int lds = 0;
    MultiMember *d_members = nullptr;
    ExprOp *d_ops = nullptr;
    std::vector<MultiMember> members;
    std::vector<int> window_members;   // indices of members accumulated in LDS
    std::vector<hist_t *> hs;          // the member handles (held: see hist_destroy)
};

// Checks a postfix program and records the stack depth before each operation.
static hist_status compile_expr(const hist_expr &e, int ncols, const char *what, int m,
                                std::vector<ExprOp> &out, ExprRef &ref)
{
    ref.first = (int32_t)out.size();
    ref.nops = 0;
    if (e.nops == 0)
        return HIST_OK;
    if (e.nops < 0 || e.nops > kExprMaxOps || !e.ops)
        return set_error(HIST_EINVAL, "hist_multi_create: member %d %s: need 1..%d operations", m, what,
                         kExprMaxOps);
    int sp = 0;
    for (int i = 0; i < e.nops; ++i) {
        const hist_op &o = e.ops[i];
        int pop, push = 1;
        switch (o.op) {
        case HIST_OP_COL:
            if (o.col < 0 || o.col >= ncols)
                return set_error(HIST_EINVAL, "hist_multi_create: member %d %s: column %d of %d", m,
                                 what, o.col, ncols);
            pop = 0;
            break;
        case HIST_OP_CONST: pop = 0; break;
        case HIST_OP_NEG: case HIST_OP_ABS: case HIST_OP_SQRT: case HIST_OP_NOT: pop = 1; break;
        case HIST_OP_SELECT: pop = 3; break;
        case HIST_OP_ADD: case HIST_OP_SUB: case HIST_OP_MUL: case HIST_OP_DIV: case HIST_OP_MIN:
        case HIST_OP_MAX: case HIST_OP_LT: case HIST_OP_LE: case HIST_OP_GT: case HIST_OP_GE:
        case HIST_OP_EQ: case HIST_OP_NE: case HIST_OP_AND: case HIST_OP_OR: pop = 2; break;
        default:
            return set_error(HIST_EINVAL, "hist_multi_create: member %d %s: unknown operation %d", m,
                             what, o.op);
        }
        if (sp < pop)
            return set_error(HIST_EINVAL, "hist_multi_create: member %d %s: operation %d needs %d "
                                          "operands, stack holds %d", m, what, i, pop, sp);
        if (sp - pop + push > kExprStack)
            return set_error(HIST_EINVAL, "hist_multi_create: member %d %s: stack deeper than %d", m,
                             what, kExprStack);
        ExprOp d;
        d.code = o.op;
        d.sp = sp;
        d.col = o.op == HIST_OP_COL ? o.col : 0;
        d.pad = 0;
        d.value = o.op == HIST_OP_CONST ? o.value : 0.0;
        out.push_back(d);
        sp = sp - pop + push;
    }
    if (sp != 1)
        return set_error(HIST_EINVAL, "hist_multi_create: member %d %s: program leaves %d values, "
                                      "needs exactly 1", m, what, sp);
    ref.nops = e.nops;
    return HIST_OK;
}

static void free_multi(hist_multi_s *m)
{
    if (!m)
        return;
    if (m->d_members)
        (void)hipFree(m->d_members);
    if (m->d_ops)
        (void)hipFree(m->d_ops);
    (void)hipGetLastError();
    delete m;
}

extern "C" hist_status hist_multi_create(int k, hist_t *const *hs, const hist_define *defs,
                                         int ncols, hist_dtype dtype, hist_multi_t **out)
{
    if (!out)
        return set_error(HIST_EINVAL, "hist_multi_create: out is NULL");
    *out = nullptr;
    if (k < 1 || k > kMultiMembers || !hs)
        return set_error(HIST_EINVAL, "hist_multi_create: need 1..%d handles", kMultiMembers);
    if (ncols < 1 || ncols > kMultiCols)
        return set_error(HIST_EINVAL, "hist_multi_create: ncols must be 1..%d", kMultiCols);
    if (dtype != HIST_F64 && dtype != HIST_F32)
        return set_error(HIST_EINVAL, "hist_multi_create: unknown dtype %d", (int)dtype);
    for (int i = 0; i < k; ++i) {
        if (!hs[i])
            return set_error(HIST_EINVAL, "hist_multi_create: handle %d is NULL", i);
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i])
                return set_error(HIST_EINVAL, "hist_multi_create: handle %d repeats handle %d", i, j);
        if (hs[i]->device != hs[0]->device)
            return set_error(HIST_EINVAL, "hist_multi_create: handles on different devices");
    }
    hist_multi_s *M = new (std::nothrow) hist_multi_s();
    if (!M)
        return set_error(HIST_ENOMEM, "hist_multi_create: host allocation");
    M->k = k;
    M->ncols = ncols;
    M->dtype = dtype;
    M->device = hs[0]->device;
    M->num_cu = hs[0]->num_cu;
    const int lds_max = hs[0]->lds_max;

    std::vector<ExprOp> ops;
    M->members.resize(k);
    for (int i = 0; i < k; ++i) {
        const hist_s *h = hs[i];
        MultiMember &d = M->members[i];
        std::memset(&d, 0, sizeof(d));
        hist_define def;
        std::memset(&def, 0, sizeof(def));
        if (defs)
            def = defs[i];
        hist_status st = compile_expr(def.filter, ncols, "filter", i, ops, d.filter);
        for (int a = 0; a < kMaxDims && st == HIST_OK; ++a) {
            if (a < h->dims)
                st = compile_expr(def.coord[a], ncols, "coordinate", i, ops, d.coord[a]);
            else
                d.coord[a] = ExprRef{(int32_t)ops.size(), 0};
        }
        if (st == HIST_OK)
            st = compile_expr(def.weight, ncols, "weight", i, ops, d.weight);
        if (st != HIST_OK) {
            free_multi(M);
            return st;
        }
        // a program that only reads a column is read directly
        for (int a = 0; a < kMaxDims; ++a) {
            d.coord_col[a] = a < h->dims && a < ncols ? a : 0;
            if (d.coord[a].nops == 1 && def.coord[a].ops[0].op == HIST_OP_COL) {
                d.coord_col[a] = def.coord[a].ops[0].col;
                d.coord[a].nops = 0;
            }
        }
        d.weighted = d.weight.nops > 0 ? 1 : 0;
        d.weight_col = -1;
        if (d.weight.nops == 1 && def.weight.ops[0].op == HIST_OP_COL) {
            d.weight_col = def.weight.ops[0].col;
            d.weight.nops = 0;
        }
        for (int a = 0; a < h->dims; ++a) {
            if (def.coord[a].nops == 0 && a >= ncols) {
                free_multi(M);
                return set_error(HIST_EINVAL, "hist_multi_create: member %d axis %d reads column %d "
                                              "of %d", i, a, a, ncols);
            }
        }
        for (int a = 0; a < kMaxDims; ++a) {
            d.ax[a] = h->ax[a];
            d.ax[a].lds_model = -1;
            d.ax[a].lds_edges = -1;
        }
        d.dims = h->dims;
        d.nstats = h->S;
        d.total_bins = (int32_t)h->T;
        d.cnt = h->d_cnt;
        d.sumw = h->d_sumw;
        d.sumw2 = h->d_sumw2;
        d.stats = h->d_stats;
        d.entries = h->d_entries;
        d.lds_win = -1;
        d.copies = 1;
        d.lds_tstats = -1;
        d.nsums = d.weighted ? h->S : h->S - 2;
    }

    // LDS: statistics of every member, then learned models (a learned axis
    // whose model does not fit falls back to binary search), edge arrays of at
    // most kStageEdgesMax edges, then whole-histogram copies, smallest
    // histograms first; members left over use global atomics.
    int off = 0;
    for (int i = 0; i < k; ++i) {
        M->members[i].lds_stats = off;
        off += kMultiStatsBytes;
    }
    for (int i = 0; i < k; ++i) {
        MultiMember &d = M->members[i];
        for (int a = 0; a < d.dims; ++a) {
            AxisDev &ax = d.ax[a];
            if (ax.kind == AX_LEARNED)
                ax.kind = AX_BSEARCH;
            if (ax.kind != AX_UNIFORM && ax.nbins + 1 <= kStageEdgesMax) {
                const int eb = (ax.nbins + 1) * (int)sizeof(double);
                if (off + eb <= lds_max / 2) {
                    ax.lds_edges = off;
                    off = (off + eb + 15) & ~15;
                }
            }
        }
    }
    std::vector<int> order(k);
    for (int i = 0; i < k; ++i)
        order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return M->members[a].total_bins < M->members[b].total_bins; });
    auto bin_bytes = [&](const MultiMember &d) { return d.weighted ? 16 : 4; };
    auto up16 = [](int64_t x) { return (x + 15) & ~(int64_t)15; };
    // 1. whole-histogram windows (one copy), smallest histograms first
    int64_t win_total = 0;
    for (int i : order) {
        const MultiMember &d = M->members[i];
        const int64_t need = up16((int64_t)d.total_bins * bin_bytes(d));
        if (off + win_total + need <= lds_max) {
            win_total += need;
            M->window_members.push_back(i);
        }
    }
    // 2. per-thread statistics sums, in member order, with the LDS left; the
    //    others reduce per wave and event slot (far slower)
    int64_t ts_total = 0;
    std::vector<int> ts_members;
    for (int i = 0; i < k; ++i) {
        const MultiMember &d = M->members[i];
        const int64_t need = up16((int64_t)d.nsums * kMaxThreads * 8);
        if (d.nsums > 0 && off + win_total + ts_total + need <= lds_max) {
            ts_total += need;
            ts_members.push_back(i);
        }
    }
    // 3. interleaved copies of the windows with what is left (up to 16), so
    //    lanes of a wave that hit one bin of a small histogram update
    //    different words
    int copies = 1;
    while (copies < 16 && !M->window_members.empty()) {
        int64_t w2 = 0;
        for (int i : M->window_members)
            w2 += up16((int64_t)M->members[i].total_bins * bin_bytes(M->members[i]) * copies * 2);
        if (off + w2 + ts_total > lds_max)
            break;
        copies *= 2;
    }
    for (int i : M->window_members) {
        MultiMember &d = M->members[i];
        d.copies = copies;
        d.lds_win = off;
        off = (int)(off + up16((int64_t)d.total_bins * bin_bytes(d) * copies));
    }
    for (int i : ts_members) {
        MultiMember &d = M->members[i];
        d.lds_tstats = off;
        off = (int)(off + up16((int64_t)d.nsums * kMaxThreads * 8));
    }
    for (int i = 0; i < k; ++i) {
        MultiMember &d = M->members[i];
        d.lean = d.dims == 1 && d.ax[0].kind == AX_UNIFORM && d.filter.nops == 0 &&
                 d.coord[0].nops == 0 && !d.weighted && d.lds_win >= 0 && d.lds_tstats >= 0;
    }
    M->lds = std::max(off, 16);

    hipError_t e = hipMalloc(&M->d_members, sizeof(MultiMember) * k);
    if (e == hipSuccess)
        e = hipMalloc(&M->d_ops, sizeof(ExprOp) * std::max<size_t>(ops.size(), 1));
    if (e == hipSuccess)
        e = hipMemcpy(M->d_members, M->members.data(), sizeof(MultiMember) * k, hipMemcpyHostToDevice);
    if (e == hipSuccess && !ops.empty())
        e = hipMemcpy(M->d_ops, ops.data(), sizeof(ExprOp) * ops.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        free_multi(M);
        return set_error(e == hipErrorOutOfMemory ? HIST_ENOMEM : HIST_EDEVICE,
                         "hist_multi_create: %s", hipGetErrorString(e));
    }
    M->hs.assign(hs, hs + k);
    for (hist_t *h : M->hs)
        ++h->users;
    *out = M;
    return HIST_OK;
}

extern "C" hist_status hist_multi_fill(hist_multi_t *M, const void *const *columns, int64_t n,
                                       void *stream)
{
    if (!M)
        return set_error(HIST_EINVAL, "hist_multi_fill: NULL plan");
    if (n < 0)
        return set_error(HIST_EINVAL, "hist_multi_fill: n < 0");
    if (n == 0)
        return HIST_OK;
    if (!columns)
        return set_error(HIST_EINVAL, "hist_multi_fill: columns is NULL");
    MultiArgs a;
    std::memset(&a, 0, sizeof(a));
    for (int c = 0; c < M->ncols; ++c) {
        if (!columns[c])
            return set_error(HIST_EINVAL, "hist_multi_fill: column %d is NULL", c);
        a.cols[c] = columns[c];
    }
    a.members = M->d_members;
    a.ops = M->d_ops;
    a.k = M->k;
    a.ncols = M->ncols;
    a.n = n;
    const int threads = kMaxThreads;
    const int64_t step = (int64_t)threads * kMultiU;
    int64_t G = M->num_cu;
    const int64_t need = (n + step - 1) / step;
    if (G > need)
        G = need;
    int64_t per = (n + G - 1) / G;
    per = (per + step - 1) / step * step;
    G = (n + per - 1) / per;
    a.per_block = per;
    (void)hipGetLastError();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const dim3 grid((unsigned)G), block(threads);
    const size_t lds = (size_t)M->lds;
    const bool f32 = M->dtype == HIST_F32;
    if (M->ncols <= 2) {
        if (f32)
            hipLaunchKernelGGL((multi_fill_kernel<float, 2>), grid, block, lds, s, a);
        else
            hipLaunchKernelGGL((multi_fill_kernel<double, 2>), grid, block, lds, s, a);
    } else if (M->ncols <= 4) {
        if (f32)
            hipLaunchKernelGGL((multi_fill_kernel<float, 4>), grid, block, lds, s, a);
        else
            hipLaunchKernelGGL((multi_fill_kernel<double, 4>), grid, block, lds, s, a);
    } else {
        if (f32)
            hipLaunchKernelGGL((multi_fill_kernel<float, kMultiCols>), grid, block, lds, s, a);
        else
            hipLaunchKernelGGL((multi_fill_kernel<double, kMultiCols>), grid, block, lds, s, a);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
        return set_error(HIST_EDEVICE, "hist_multi_fill: launch: %s", hipGetErrorString(e));
    return HIST_OK;
}

extern "C" hist_status hist_multi_info(const hist_multi_t *M, int member, int *in_lds, int *copies,
                                       int *lds_bytes)
{
    if (!M || member < 0 || member >= M->k)
        return set_error(HIST_EINVAL, "hist_multi_info: bad plan or member");
    if (in_lds)
        *in_lds = M->members[member].lds_win >= 0 ? 1 : 0;
    if (copies)
        *copies = M->members[member].copies;
    if (lds_bytes)
        *lds_bytes = M->lds;
    return HIST_OK;
}

extern "C" hist_status hist_multi_destroy(hist_multi_t *M)
{
    if (!M)
        return HIST_OK;
    (void)hipDeviceSynchronize();
    for (hist_t *h : M->hs)
        --h->users;
    free_multi(M);
    return HIST_OK;
}
