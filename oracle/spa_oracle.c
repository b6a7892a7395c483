/*
 * Oracle: plain FP64 flooding sum-product (belief-propagation) LDPC decoder.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * loads this file; only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may.  It shares no code with the GPU decoder.
 *
 * What it computes (arxiv 1812.06545, Section II):
 *   - H is the sparse m x n parity-check matrix; H[i][j] = 1 joins check node
 *     i to variable node j of the Tanner graph (text around eq. (1)).
 *   - Decoding is two-phase message passing on a flooding schedule: all
 *     check-to-variable messages of an iteration are formed from the previous
 *     variable-to-check messages, then all variable nodes update (Section II,
 *     two-phase message passing; Algorithm 1: Loop 1 initialisation, then per
 *     iteration Loop 2 check->variable, Loop 3 variable->check, Loop 4 hard
 *     decision).
 *   - The check rule is the sum-product (tanh) rule named in Section I:
 *     r_mn = 2 atanh( prod_{n' in N(m), n' != n} tanh(q_mn' / 2) ),
 *     clamped to [-r_max, r_max].  The exclusive product is formed directly,
 *     by multiplying every other edge of the row (no division).
 *   - Variable rule: L_n = Lch_n + sum_{m in M(n)} r_mn ; q_mn = L_n - r_mn.
 *   - Hard decision x_n = 1 iff L_n < 0 (LLR = ln P(0)/P(1)).
 *   - The paper states no stopping rule; with early stop the syndrome H x
 *     (mod 2) is tested before iteration 1 and after every hard decision, and
 *     decoding stops at the first all-zero syndrome.  iters = number of
 *     iterations run (0 if the channel decision is already a codeword).
 *
 * Every formula above is the textbook definition, evaluated in double
 * precision in the order written.  Summation order: CSR order for rows,
 * ascending row order for columns.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Precision of the check-node evaluation (the tanh terms, their product and
 * 2 atanh).  Double by default.  The build also compiles a copy with
 * ORACLE_CHECK_LD defined, which evaluates the same expressions in x87 80-bit
 * long double and rounds each message to double: the same definition at
 * higher precision, used to measure the rounding of the double version (near
 * the clamp 2 atanh(p) with p close to 1 loses digits) and to hold FP64 GPU
 * results to a tighter bound than that rounding allows. */
#ifdef ORACLE_CHECK_LD
typedef long double chk_real;
#define CHK_TANH tanhl
#define CHK_ATANH atanhl
#else
typedef double chk_real;
#define CHK_TANH tanh
#define CHK_ATANH atanh
#endif

#define ORACLE_EINVAL (-1)
#define ORACLE_ENOMEM (-2)

/* 1 if every row of H has even parity over x, else 0. */
static int syndrome_is_zero(int m, const int32_t *row_ptr, const int32_t *col_idx, const uint8_t *x)
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

static double min_abs_of(int n, const double *L)
{
    double v = INFINITY;
    for (int j = 0; j < n; ++j)
        if (fabs(L[j]) < v)
            v = fabs(L[j]);
    return v;
}

struct graph {
    int m, n;
    const int32_t *row_ptr, *col_idx;
    int32_t *col_ptr;   /* n + 1 */
    int32_t *col_edge;  /* E: edges of column j in ascending row order */
};

static void decode_one_frame(const struct graph *g, const double *llr, int max_iter, int early_stop,
                             double r_max, uint8_t *bits, int32_t *iters, double *posterior,
                             double *cond, double *min_abs, double *q, double *r, chk_real *th,
                             double *L, uint8_t *x)
{
    const int m = g->m, n = g->n;
    const int32_t E = g->row_ptr[m];
    int t_done = max_iter;

    for (int t = 0; t <= max_iter && min_abs; ++t)
        min_abs[t] = NAN;

    /* Loop 1: initialisation.  L = Lch, q_mn = Lch_n, r = 0. */
    for (int j = 0; j < n; ++j) {
        L[j] = llr[j];
        x[j] = (uint8_t)(L[j] < 0.0);
    }
    for (int32_t e = 0; e < E; ++e) {
        q[e] = llr[g->col_idx[e]];
        r[e] = 0.0;
    }
    if (min_abs)
        min_abs[0] = min_abs_of(n, L);

    if (early_stop && syndrome_is_zero(m, g->row_ptr, g->col_idx, x)) {
        t_done = 0;
    } else {
        for (int t = 1; t <= max_iter; ++t) {
            /* Loop 2: check node -> variable node messages. */
            for (int i = 0; i < m; ++i) {
                const int32_t e0 = g->row_ptr[i], e1 = g->row_ptr[i + 1];
                for (int32_t e = e0; e < e1; ++e)
                    th[e] = CHK_TANH((chk_real)q[e] / 2);
                for (int32_t e = e0; e < e1; ++e) {
                    chk_real p = 1;
                    for (int32_t o = e0; o < e1; ++o)
                        if (o != e)
                            p *= th[o];
                    double v = (double)(2 * CHK_ATANH(p));
                    if (v > r_max)
                        v = r_max;
                    if (v < -r_max)
                        v = -r_max;
                    r[e] = v;
                }
            }
            /* Loop 3: variable node -> check node messages (and posterior). */
            for (int j = 0; j < n; ++j) {
                double s = llr[j];
                for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)
                    s += r[g->col_edge[k]];
                L[j] = s;
                for (int32_t k = g->col_ptr[j]; k < g->col_ptr[j + 1]; ++k)
                    q[g->col_edge[k]] = s - r[g->col_edge[k]];
            }
            /* Loop 4: hard decision from the posterior. */
            for (int j = 0; j < n; ++j)
                x[j] = (uint8_t)(L[j] < 0.0);
            if (min_abs)
                min_abs[t] = min_abs_of(n, L);
            if (early_stop && syndrome_is_zero(m, g->row_ptr, g->col_idx, x)) {
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
 * Decode `frames` frames of n channel LLRs each (row-major, frame f at
 * llr[f*n]).  Outputs: bits (frames*n, 0/1), iters (frames), posterior
 * (frames*n or NULL), cond (frames*n conditioning scale |Lch_n| + sum |r_mn|
 * of the final messages, or NULL), min_abs (frames*(max_iter+1): min_n |L_n|
 * at decision points 0..iters, NaN afterwards; or NULL).
 * Returns 0, or a negative value for invalid arguments (duplicate edges,
 * columns out of range, negative sizes) or allocation failure.
 */
int oracle_spa_decode(int m, int n, const int32_t *row_ptr, const int32_t *col_idx, int frames,
                      const double *llr, int max_iter, int early_stop, double r_max, uint8_t *bits,
                      int32_t *iters, double *posterior, double *cond, double *min_abs, int nthreads)
{
    if (m < 0 || n < 1 || frames < 0 || max_iter < 0 || !row_ptr || !llr || !bits || !iters)
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
                    return ORACLE_EINVAL; /* duplicate edge */
        }
    }
    const int32_t E = row_ptr[m];

    struct graph g = {m, n, row_ptr, col_idx, NULL, NULL};
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
    /* rows are visited in ascending order, so each column's list is row-sorted */
    for (int i = 0; i < m; ++i)
        for (int32_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int32_t j = col_idx[e];
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
        chk_real *th = (chk_real *)malloc(((size_t)E + 1) * sizeof(chk_real));
        double *L = (double *)malloc((size_t)n * sizeof(double));
        uint8_t *x = (uint8_t *)malloc((size_t)n);
        int ok = q && r && th && L && x;
        if (!ok) {
#pragma omp atomic write
            status = ORACLE_ENOMEM;
        }
#pragma omp for schedule(dynamic, 1)
        for (int f = 0; f < frames; ++f) {
            if (!ok)
                continue;
            const size_t off = (size_t)f * (size_t)n;
            decode_one_frame(&g, llr + off, max_iter, early_stop, r_max, bits + off, iters + f,
                             posterior ? posterior + off : NULL, cond ? cond + off : NULL,
                             min_abs ? min_abs + (size_t)f * (size_t)(max_iter + 1) : NULL, q, r, th, L,
                             x);
        }
        free(q);
        free(r);
        free(th);
        free(L);
        free(x);
    }
    free(g.col_ptr);
    free(g.col_edge);
    return status;
}
