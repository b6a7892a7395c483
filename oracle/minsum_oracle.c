/*
 * Oracle: plain FP64 min-sum LDPC decoders (flooding and layered schedules).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may.  It shares no code with the GPU decoder.
 *
 * What it computes (arxiv 1812.06545, Section II): Algorithm 1 is named the
 * min-sum algorithm, the variant of message passing the paper says designers
 * prefer.  Its check-to-variable message keeps the sign rule of the tanh
 * product and replaces the magnitude by the smallest magnitude among the
 * other incoming messages:
 *     r_mn = prod_{n' != n} sgn(q_mn') * min_{n' != n} |q_mn'|.
 * The common corrections are applied to the magnitude (a reading: the paper
 * names only the plain rule): |r| = max(scale * min - offset, 0), with
 * scale = 1, offset = 0 for plain min-sum; then the clamp to [-r_max, r_max]
 * of the sum-product decoders.  sgn(0) = +1; an edge with no other edges
 * (degree-1 check) has min = +infinity and sends +r_max.
 *
 * The schedules are those of spa_oracle.c (flooding) and layered_oracle.c
 * (rows one at a time in ascending order), with the same initialisation,
 * hard decision, early stop and iteration count.  Every step is written out
 * plainly; the exclusive minimum scans every other edge of the row.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

static int ms_syndrome_is_zero(int m, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *x)
{
    for (int i = 0; i < m; ++i) {
        int parity = 0;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
            parity ^= x[col_idx[e]];
        if (parity)
            return 0;
    }
    return 1;
}

static double ms_min_abs(int n, const double *L)
{
    double v = INFINITY;
    for (int j = 0; j < n; ++j)
        if (fabs(L[j]) < v)
            v = fabs(L[j]);
    return v;
}

/* Min-sum message of edge e of row [e0, e1) from the incoming messages q. */
static double ms_message(const double *q, int32_t e0, int32_t e1, int32_t e, double scale, double offset,
                         double r_max)
{
    double mn = INFINITY;
    int negative = 0;
    for (int32_t o = e0; o < e1; ++o) {
        if (o == e)
            continue;
        if (fabs(q[o]) < mn)
            mn = fabs(q[o]);
        if (q[o] < 0.0)
            negative ^= 1;
    }
    double mag = scale * mn - offset;
    if (mag < 0.0)
        mag = 0.0;
    if (mag > r_max)
        mag = r_max;
    return negative ? -mag : mag;
}

struct ms_graph {
    int m, n;
    const int32_t *row_ptr, *col_idx;
    int32_t *col_ptr, *col_edge;
};

static void ms_frame(const struct ms_graph *g, int layered, const double *llr, int max_iter, int early_stop,
                     double scale, double offset, double r_max, uint8_t *bits, int32_t *iters, double *posterior,
                     double *cond, double *min_abs, double *q, double *r, double *L, uint8_t *x)
{
    const int m = g->m, n = g->n;
    const int32_t E = g->row_ptr[m];
    int t_done = max_iter;
    for (int t = 0; t <= max_iter && min_abs; ++t)
        min_abs[t] = NAN;
    for (int j = 0; j < n; ++j) {
        L[j] = llr[j];
        x[j] = (uint8_t)(L[j] < 0.0);
    }
    for (int32_t e = 0; e < E; ++e) {
        q[e] = llr[g->col_idx[e]];
        r[e] = 0.0;
    }
    if (min_abs)
        min_abs[0] = ms_min_abs(n, L);
    if (early_stop && ms_syndrome_is_zero(m, g->row_ptr, g->col_idx, x)) {
        t_done = 0;
    } else {
        for (int t = 1; t <= max_iter; ++t) {
            if (!layered) {
                /* Loop 2 for every row from the previous q, then Loop 3. */
                for (int i = 0; i < m; ++i)
                    for (int32_t e = g->row_ptr[i]; e < g->row_ptr[i + 1]; ++e)
                        r[e] = ms_message(q, g->row_ptr[i], g->row_ptr[i + 1], e, scale, offset, r_max);
                for (int j = 0; j < n; ++j) {
                    double s = llr[j];
                    for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)
                        s += r[g->col_edge[k]];
                    L[j] = s;
                    for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)
                        q[g->col_edge[k]] = s - r[g->col_edge[k]];
                }
            } else {
                /* Rows one at a time: q from the current posteriors, new
                 * messages, posteriors updated at once. */
                for (int i = 0; i < m; ++i) {
                    const int32_t e0 = g->row_ptr[i], e1 = g->row_ptr[i + 1];
                    for (int32_t e = e0; e < e1; ++e)
                        q[e] = L[g->col_idx[e]] - r[e];
                    for (int32_t e = e0; e < e1; ++e)
                        r[e] = ms_message(q, e0, e1, e, scale, offset, r_max);
                    for (int32_t e = e0; e < e1; ++e)
                        L[g->col_idx[e]] = q[e] + r[e];
                }
            }
            for (int j = 0; j < n; ++j)
                x[j] = (uint8_t)(L[j] < 0.0);
            if (min_abs)
                min_abs[t] = ms_min_abs(n, L);
            if (early_stop && ms_syndrome_is_zero(m, g->row_ptr, g->col_idx, x)) {
                t_done = t;
                break;
            }
        }
    }
    *iters = t_done;
    for (int j = 0; j < n; ++j) {
        bits[j] = x[j];
        if (posterior)
            posterior[j] = L[j];
        if (cond) {
            double a = fabs(llr[j]);
            for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)
                a += fabs(r[g->col_edge[k]]);
            cond[j] = a;
        }
    }
}

/*
 * Same arguments and outputs as oracle_spa_decode, plus: layered (0 =
 * flooding, 1 = layered schedule), scale and offset of the min-sum
 * magnitude.  Returns 0, or a negative value for invalid arguments or
 * allocation failure.
 */
int oracle_minsum_decode(int m, int n, const int32_t *row_ptr, const int32_t *col_idx, int frames, const double *llr,
                         int max_iter, int early_stop, int layered, double scale, double offset, double r_max,
                         uint8_t *bits, int32_t *iters, double *posterior, double *cond, double *min_abs,
                         int nthreads)
{
    if (m < 0 || n < 1 || frames < 0 || max_iter < 0 || !row_ptr || !llr || !bits || !iters || !(scale > 0.0) ||
        !(offset >= 0.0))
        return ORACLE_EINVAL;
    if (row_ptr[0] != 0)
        return ORACLE_EINVAL;
    for (int i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i])
            return ORACLE_EINVAL;
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= n)
                return ORACLE_EINVAL;
            for (int32_t o = row_ptr[i]; o < e; ++o)
                if (col_idx[o] == col_idx[e])
                    return ORACLE_EINVAL;
        }
    }
    const int32_t E = row_ptr[m];
    struct ms_graph g = {m, n, row_ptr, col_idx, NULL, NULL};
    g.col_ptr = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    g.col_edge = (int32_t *)malloc(((size_t)E + 1) * sizeof(int32_t));
    int32_t *fill = (int32_t *)calloc((size_t)n + 1, sizeof(int32_t));
    if (!g.col_ptr || !g.col_edge || !fill) {
        free(g.col_ptr);
        free(g.col_edge);
        free(fill);
        return ORACLE_ENOMEM;
    }
    for (int32_t e = 0; e < E; ++e)
        g.col_ptr[col_idx[e] + 1]++;
    for (int j = 0; j < n; ++j)
        g.col_ptr[j + 1] += g.col_ptr[j];
    for (int i = 0; i < m; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            const int32_t j = col_idx[e];
            g.col_edge[g.col_ptr[j] + fill[j]++] = e;
        }
    free(fill);

    int status = 0;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        double *q = (double *)malloc(((size_t)E + 1) * sizeof(double));
        double *r = (double *)malloc(((size_t)E + 1) * sizeof(double));
        double *L = (double *)malloc((size_t)n * sizeof(double));
        uint8_t *x = (uint8_t *)malloc((size_t)n);
        int ok = q && r && L && x;
        if (!ok) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        }
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f < frames; ++f) {
            if (!ok)
                continue;
            const size_t off = (size_t)f * (size_t)n;
            ms_frame(&g, layered, llr + off, max_iter, early_stop, scale, offset, r_max, bits + off, iters + f,
                     posterior ? posterior + off : NULL, cond ? cond + off : NULL,
                     min_abs ? min_abs + (size_t)f * (size_t)(max_iter + 1) : NULL, q, r, L, x);
        }
        free(q);
        free(r);
        free(L);
        free(x);
    }
    free(g.col_ptr);
    free(g.col_edge);
    return status;
}
