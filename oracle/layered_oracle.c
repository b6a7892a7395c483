/*
 * Oracle: plain FP64 layered (serial check-node schedule) sum-product decoder.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may.  It shares no code with the GPU decoder.
 *
 * What it computes (arxiv 1812.06545, Section II, the layered algorithm the
 * paper names Algorithm 2 and describes in three steps):
 *   - A check node's messages are computed from the variable-node messages
 *     linked to it; right after that check node, the variable nodes it touches
 *     are updated with the new messages; this repeats up to the maximum
 *     iteration count.  One iteration is one pass over all check nodes.
 *   - Check nodes are visited one at a time in ascending row index (a
 *     reading: the paper gives no order; a caller wanting another order
 *     permutes the rows of H).  Rows that share no variable node can be
 *     visited in any order without changing the result.
 *   - State: the posterior L_n (initialised to the channel LLR) and one
 *     check-to-variable message r_mn per edge (initialised to 0).  Visiting
 *     row m:  q_mn = L_n - r_mn (the variable-to-check message, extrinsic to
 *     row m);  r_mn = 2 atanh( prod_{n' in N(m), n' != n} tanh(q_mn' / 2) ),
 *     clamped to [-r_max, r_max];  L_n = q_mn + r_mn.  So L_n always equals
 *     Lch_n + sum_m r_mn over the current messages.
 *   - Hard decision x_n = 1 iff L_n < 0 after every pass; with early stop the
 *     syndrome H x (mod 2) is tested before the first pass and after every
 *     pass, and decoding stops at the first all-zero syndrome.  iters = number
 *     of passes run (0 if the channel decision is already a codeword).
 *
 * Every formula is the textbook definition, evaluated in double precision in
 * the order written; the exclusive product multiplies every other edge of the
 * row directly (no division).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

static int layered_syndrome_is_zero(int m, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *x)
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

static double layered_min_abs(int n, const double *L)
{
    double v = INFINITY;
    for (int j = 0; j < n; ++j)
        if (fabs(L[j]) < v)
            v = fabs(L[j]);
    return v;
}

/* Visit check row i: new messages from the current posteriors, then the
 * posteriors of the row's variables take the new messages at once. */
static void visit_row(const int32_t *row_ptr, const int32_t *col_idx, int i, double r_max, double *L, double *r,
                      double *q, double *th)
{
    const int32_t e0 = row_ptr[i], e1 = row_ptr[i + 1];
    for (int32_t e = e0; e < e1; ++e) {
        q[e - e0] = L[col_idx[e]] - r[e];
        th[e - e0] = tanh(q[e - e0] / 2.0);
    }
    for (int32_t e = e0; e < e1; ++e) {
        double p = 1.0;
        for (int32_t o = e0; o < e1; ++o)
            if (o != e)
                p *= th[o - e0];
        double v = 2.0 * atanh(p);
        if (v > r_max)
            v = r_max;
        if (v < -r_max)
            v = -r_max;
        r[e] = v;
    }
    for (int32_t e = e0; e < e1; ++e)
        L[col_idx[e]] = q[e - e0] + r[e];
}

static void layered_one_frame(int m, int n, const int32_t *row_ptr, const int32_t *col_idx, const double *llr,
                              int max_iter, int early_stop, double r_max, uint8_t *bits, int32_t *iters,
                              double *posterior, double *cond, double *min_abs, double *r, double *q, double *th,
                              double *L, uint8_t *x)
{
    const int32_t E = row_ptr[m];
    int t_done = max_iter;
    for (int t = 0; t <= max_iter && min_abs; ++t)
        min_abs[t] = NAN;

    for (int j = 0; j < n; ++j) {
        L[j] = llr[j];
        x[j] = (uint8_t)(L[j] < 0.0);
    }
    for (int32_t e = 0; e < E; ++e)
        r[e] = 0.0;
    if (min_abs)
        min_abs[0] = layered_min_abs(n, L);

    if (early_stop && layered_syndrome_is_zero(m, row_ptr, col_idx, x)) {
        t_done = 0;
    } else {
        for (int t = 1; t <= max_iter; ++t) {
            for (int i = 0; i < m; ++i)
                visit_row(row_ptr, col_idx, i, r_max, L, r, q, th);
            for (int j = 0; j < n; ++j)
                x[j] = (uint8_t)(L[j] < 0.0);
            if (min_abs)
                min_abs[t] = layered_min_abs(n, L);
            if (early_stop && layered_syndrome_is_zero(m, row_ptr, col_idx, x)) {
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
        if (cond)
            cond[j] = fabs(llr[j]);
    }
    if (cond)
        for (int32_t e = 0; e < E; ++e)
            cond[col_idx[e]] += fabs(r[e]);
}

/*
 * Same arguments and outputs as oracle_spa_decode (flooding), for the layered
 * schedule: cond is |Lch_n| + sum_m |r_mn| over the final messages, min_abs
 * the minimum |L_n| after each pass.
 */
int oracle_spa_layered_decode(int m, int n, const int32_t *row_ptr, const int32_t *col_idx, int frames,
                              const double *llr, int max_iter, int early_stop, double r_max, uint8_t *bits,
                              int32_t *iters, double *posterior, double *cond, double *min_abs, int nthreads)
{
    if (m < 0 || n < 1 || frames < 0 || max_iter < 0 || !row_ptr || !llr || !bits || !iters)
        return ORACLE_EINVAL;
    if (row_ptr[0] != 0)
        return ORACLE_EINVAL;
    int32_t dmax = 0;
    for (int i = 0; i < m; ++i) {
        if (row_ptr[i + 1] < row_ptr[i])
            return ORACLE_EINVAL;
        if (row_ptr[i + 1] - row_ptr[i] > dmax)
            dmax = row_ptr[i + 1] - row_ptr[i];
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= n)
                return ORACLE_EINVAL;
            for (int32_t o = row_ptr[i]; o < e; ++o)
                if (col_idx[o] == col_idx[e])
                    return ORACLE_EINVAL; /* duplicate edge */
        }
    }
    const int32_t E = row_ptr[m];
    int status = 0;
    if (nthreads < 1)
        nthreads = 1;
#pragma omp parallel num_threads(nthreads)
    {
        double *r = (double *)malloc(((size_t)E + 1) * sizeof(double));
        double *q = (double *)malloc(((size_t)dmax + 1) * sizeof(double));
        double *th = (double *)malloc(((size_t)dmax + 1) * sizeof(double));
        double *L = (double *)malloc((size_t)n * sizeof(double));
        uint8_t *x = (uint8_t *)malloc((size_t)n);
        int ok = r && q && th && L && x;
        if (!ok) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        }
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f < frames; ++f) {
            if (!ok)
                continue;
            const size_t off = (size_t)f * (size_t)n;
            layered_one_frame(m, n, row_ptr, col_idx, llr + off, max_iter, early_stop, r_max, bits + off,
                              iters + f, posterior ? posterior + off : NULL, cond ? cond + off : NULL,
                              min_abs ? min_abs + (size_t)f * (size_t)(max_iter + 1) : NULL, r, q, th, L, x);
        }
        free(r);
        free(q);
        free(th);
        free(L);
        free(x);
    }
    return status;
}
