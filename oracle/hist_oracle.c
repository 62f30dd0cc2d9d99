/*
 * hist_oracle.c -- plain, slow, sequential CPU oracle for histogram filling.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * shares no code, header, table or helper with it.
 *
 * What it computes (Chen, Dessole, Varbanescu, "Lessons Learned Migrating
 * CUDA to SYCL: A HEP Case Study with ROOT RDataFrame", arXiv:2401.13310):
 *
 *   Sec. 3.1 (Histogramming Action), the three steps of Fill for a bulk:
 *     (1) find the bin of each coordinate -- fixed-width axes by the closed
 *         formula 1 + floor(nbins * (x - min) / (max - min)), variable axes by
 *         a binary search over the edge array, and coordinates outside the
 *         range go to a dedicated underflow / overflow bin;
 *         higher dimensions repeat the find-bin step per axis;
 *     (2) increment that bin by the event weight (1 when unweighted);
 *     (3) update the running sums from which the statistics (mean, standard
 *         deviation) are derived.
 *   Sec. 3.2: the statistics are transform-reduce operations; for 1D they are
 *         the sum of weights, of squared weights, of weight*x and of
 *         weight*x^2.
 *   Sec. 3.3: the sums of each bulk are added to those of earlier bulks, never
 *         overwritten.
 *
 * Readings where the paper is silent or ambiguous (all are also listed in the
 * design notes of the repository):
 *   - variable axes use upper_bound: bins include their lower edge, so an
 *     exact hit on edge e_i lands in bin i+1 (the paper names lower_bound; the
 *     uniform formula and ROOT's convention are lower-edge inclusive);
 *   - NaN goes to the overflow bin on every axis kind (!(x < max) is true);
 *   - the uniform formula is evaluated left to right in IEEE binary64 with
 *     round-to-nearest and no fused multiply-add: t = x - min,
 *     u = nbins * t, v = u / (max - min), bin = 1 + trunc(v), clamped to
 *     nbins (v >= 0 there, so trunc == floor);
 *   - the per-bin sum of squared weights (ROOT's Sumw2) is kept next to the
 *     sum of weights; each event adds w and w*w;
 *   - statistics take only events that are inside the range on every axis
 *     (ROOT's default), and for d > 1 follow ROOT's moment set:
 *       d=1: [Sw, Sw2, Swx, Swx2]
 *       d=2: + [Swy, Swy2, Swxy]
 *       d=3: + [Swz, Swz2, Swxz, Swyz]
 *     with per-event terms w, w*w, w*x, (w*x)*x, (w*x)*y, ...;
 *   - entries counts every event, including flow and NaN.
 *
 * Summation.  The mathematical result is the exact sum of the per-event terms;
 * the paper fixes no summation order.  The oracle accumulates every sum with
 * Neumaier's compensated summation (Neumaier 1974), so its own error is about
 * one rounding of the result plus n*u^2*sum|t|, far below the 1e-12 relative
 * tolerance the GPU path is held to.  Per-event terms are rounded products in
 * the order written above; the file is compiled with -ffp-contract=off so no
 * product is fused into an add.
 *
 * Global bin number: g = b0 + (n0+2) * (b1 + (n1+2) * b2), x fastest (ROOT).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_MAX_DIMS 3

typedef struct {
    int32_t nbins;
    double xmin, xmax;     /* fixed-width axis when edges == NULL */
    const double *edges;   /* else nbins+1 strictly increasing values */
} oracle_axis;

/* ---- step (1): find bin, Sec. 3.1 ------------------------------------- */

/* Fixed-width axis: the closed formula of Sec. 3.1 with flow checks. */
int32_t oracle_bin_uniform(double x, int32_t nbins, double xmin, double xmax)
{
    if (x < xmin)
        return 0;                       /* underflow, also -inf */
    if (!(x < xmax))
        return nbins + 1;               /* overflow, also +inf and NaN */
    double t = x - xmin;
    double u = (double)nbins * t;
    double v = u / (xmax - xmin);
    int32_t b = 1 + (int32_t)v;
    if (b > nbins)
        b = nbins;                      /* rounding can reach nbins+1 just below max */
    return b;
}

/* Variable axis by definition: the number of edges e_i with !(x < e_i).
 * O(nbins); used to pin the binary search on small inputs. */
int32_t oracle_bin_variable_count(double x, int32_t nbins, const double *e)
{
    int32_t c = 0;
    for (int32_t i = 0; i <= nbins; ++i)
        if (!(x < e[i]))
            ++c;
    return c;
}

/* Variable axis by binary search (Sec. 3.1): the first index i in
 * [0, nbins+1) with x < e_i, i.e. upper_bound; nbins+1 when there is none. */
int32_t oracle_bin_variable(double x, int32_t nbins, const double *e)
{
    int32_t lo = 0, hi = nbins + 1;
    while (lo < hi) {
        int32_t mid = lo + (hi - lo) / 2;
        if (x < e[mid])
            hi = mid;
        else
            lo = mid + 1;
    }
    return lo;
}

static int32_t axis_bin(const oracle_axis *a, double x)
{
    if (a->edges)
        return oracle_bin_variable(x, a->nbins, a->edges);
    return oracle_bin_uniform(x, a->nbins, a->xmin, a->xmax);
}

/* Global bin number from per-axis bins, x fastest. */
int64_t oracle_global_bin(int dims, const oracle_axis *axes, const int32_t *b)
{
    int64_t g = b[dims - 1];
    for (int a = dims - 2; a >= 0; --a)
        g = g * (int64_t)(axes[a].nbins + 2) + b[a];
    return g;
}

/* Global bins of n events; coords[a][i] is coordinate a of event i. */
void oracle_findbin(int dims, const oracle_axis *axes, const double *const *coords,
                    int64_t n, int32_t *out)
{
    int32_t b[ORACLE_MAX_DIMS];
    for (int64_t i = 0; i < n; ++i) {
        for (int a = 0; a < dims; ++a)
            b[a] = axis_bin(&axes[a], coords[a][i]);
        out[i] = (int32_t)oracle_global_bin(dims, axes, b);
    }
}

/* ---- histogram state, steps (2) and (3) -------------------------------- */

typedef struct {
    int dims;
    oracle_axis axes[ORACLE_MAX_DIMS];
    double *edge_store[ORACLE_MAX_DIMS];
    int64_t nbins_total;
    int nstats;
    double *sumw, *sumw_c;     /* value and Neumaier compensation */
    double *sumw2, *sumw2_c;
    double stats[11], stats_c[11];
    int64_t entries;
} oracle_hist;

static void nadd(double *s, double *c, double t)
{
    double a = *s + t;
    if (fabs(*s) >= fabs(t))
        *c += (*s - a) + t;
    else
        *c += (t - a) + *s;
    *s = a;
}

int oracle_nstats(int dims)
{
    return 2 + 2 * dims + dims * (dims - 1) / 2;
}

/* Returns NULL on invalid arguments or allocation failure.  Edge arrays are
 * copied. */
oracle_hist *oracle_hist_create(int dims, const oracle_axis *axes)
{
    if (dims < 1 || dims > ORACLE_MAX_DIMS)
        return NULL;
    oracle_hist *h = calloc(1, sizeof(*h));
    if (!h)
        return NULL;
    h->dims = dims;
    h->nbins_total = 1;
    for (int a = 0; a < dims; ++a) {
        h->axes[a] = axes[a];
        if (axes[a].nbins < 1)
            goto fail;
        if (axes[a].edges) {
            size_t ne = (size_t)axes[a].nbins + 1;
            h->edge_store[a] = malloc(ne * sizeof(double));
            if (!h->edge_store[a])
                goto fail;
            memcpy(h->edge_store[a], axes[a].edges, ne * sizeof(double));
            h->axes[a].edges = h->edge_store[a];
        }
        h->nbins_total *= (int64_t)axes[a].nbins + 2;
    }
    h->nstats = oracle_nstats(dims);
    size_t T = (size_t)h->nbins_total;
    h->sumw = calloc(T, sizeof(double));
    h->sumw_c = calloc(T, sizeof(double));
    h->sumw2 = calloc(T, sizeof(double));
    h->sumw2_c = calloc(T, sizeof(double));
    if (!h->sumw || !h->sumw_c || !h->sumw2 || !h->sumw2_c)
        goto fail;
    return h;
fail:
    for (int a = 0; a < ORACLE_MAX_DIMS; ++a)
        free(h->edge_store[a]);
    free(h->sumw); free(h->sumw_c); free(h->sumw2); free(h->sumw2_c);
    free(h);
    return NULL;
}

void oracle_hist_destroy(oracle_hist *h)
{
    if (!h)
        return;
    for (int a = 0; a < ORACLE_MAX_DIMS; ++a)
        free(h->edge_store[a]);
    free(h->sumw); free(h->sumw_c); free(h->sumw2); free(h->sumw2_c);
    free(h);
}

int64_t oracle_hist_nbins_total(const oracle_hist *h) { return h->nbins_total; }

/* Fill n events, adding to what earlier fills left (Sec. 3.3).  weights may
 * be NULL for unit weights. */
void oracle_hist_fill(oracle_hist *h, const double *const *coords, const double *weights,
                      int64_t n)
{
    const int d = h->dims;
    int32_t b[ORACLE_MAX_DIMS];
    double x[ORACLE_MAX_DIMS];
    for (int64_t i = 0; i < n; ++i) {
        double w = weights ? weights[i] : 1.0;
        int inside = 1;
        for (int a = 0; a < d; ++a) {
            x[a] = coords[a][i];
            b[a] = axis_bin(&h->axes[a], x[a]);
            if (b[a] < 1 || b[a] > h->axes[a].nbins)
                inside = 0;
        }
        int64_t g = oracle_global_bin(d, h->axes, b);
        double ww = w * w;
        nadd(&h->sumw[g], &h->sumw_c[g], w);
        nadd(&h->sumw2[g], &h->sumw2_c[g], ww);
        h->entries += 1;
        if (!inside)
            continue;
        int k = 0;
        nadd(&h->stats[k], &h->stats_c[k], w);  ++k;
        nadd(&h->stats[k], &h->stats_c[k], ww); ++k;
        for (int a = 0; a < d; ++a) {
            double wx = w * x[a];
            nadd(&h->stats[k], &h->stats_c[k], wx);        ++k;
            nadd(&h->stats[k], &h->stats_c[k], wx * x[a]); ++k;
            for (int c = 0; c < a; ++c) {   /* cross terms w*x_c*x_a, c < a */
                nadd(&h->stats[k], &h->stats_c[k], (w * x[c]) * x[a]);
                ++k;
            }
        }
    }
}

/* Copy out the accumulated sums (value + compensation).  Any output pointer
 * may be NULL. */
void oracle_hist_read(const oracle_hist *h, double *sumw, double *sumw2, double *stats,
                      int64_t *entries)
{
    size_t T = (size_t)h->nbins_total;
    if (sumw)
        for (size_t g = 0; g < T; ++g)
            sumw[g] = h->sumw[g] + h->sumw_c[g];
    if (sumw2)
        for (size_t g = 0; g < T; ++g)
            sumw2[g] = h->sumw2[g] + h->sumw2_c[g];
    if (stats)
        for (int k = 0; k < h->nstats; ++k)
            stats[k] = h->stats[k] + h->stats_c[k];
    if (entries)
        *entries = h->entries;
}

/* Sum of |term| for every statistic over n events, used to scale the
 * tolerance of statistics that can cancel. */
void oracle_stats_abs(int dims, const oracle_axis *axes, const double *const *coords,
                      const double *weights, int64_t n, double *out)
{
    int ns = oracle_nstats(dims);
    double c[11];
    for (int k = 0; k < ns; ++k)
        out[k] = c[k] = 0.0;
    double x[ORACLE_MAX_DIMS];
    for (int64_t i = 0; i < n; ++i) {
        double w = weights ? weights[i] : 1.0;
        int inside = 1;
        for (int a = 0; a < dims; ++a) {
            x[a] = coords[a][i];
            int32_t bb = axis_bin(&axes[a], x[a]);
            if (bb < 1 || bb > axes[a].nbins)
                inside = 0;
        }
        if (!inside)
            continue;
        int k = 0;
        nadd(&out[k], &c[k], fabs(w));     ++k;
        nadd(&out[k], &c[k], fabs(w * w)); ++k;
        for (int a = 0; a < dims; ++a) {
            double wx = w * x[a];
            nadd(&out[k], &c[k], fabs(wx));        ++k;
            nadd(&out[k], &c[k], fabs(wx * x[a])); ++k;
            for (int cc = 0; cc < a; ++cc) {
                nadd(&out[k], &c[k], fabs((w * x[cc]) * x[a]));
                ++k;
            }
        }
    }
    for (int k = 0; k < ns; ++k)
        out[k] += c[k];
}
