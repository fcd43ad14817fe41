/*
 * Plain, slow, sequential CPU oracle for the BOBA hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * shares no code, header or table with this file.
 *
 * Paper: "BOBA: A Parallel Lightweight Graph Reordering Algorithm with Heavyweight
 * Implications" (Batched Order By Attachment), arXiv 2306.10410.
 *
 * Every function is the plain definition of what the method computes, written
 * out in the paper's order and notation (0-based indices throughout):
 *
 *   oracle_boba      Sec. 4.3, Algorithm 1 (Sequential BOBA): scan I, then J,
 *                    handing the next new ID to every vertex on first sight.
 *                    Extended with the isolated-vertex tail (vertices that
 *                    never occur follow in increasing old ID), which equals a
 *                    stable ParMapKeys over p = (0..n-1) in Algorithm 2.
 *                    `interleaved` = 1 scans I(0) J(0) I(1) J(1) ... instead,
 *                    the flattening drawn in Fig. 1.
 *   oracle_relabel   applying the permutation to both endpoint arrays.
 *   oracle_coo_to_csr  stable counting sort of the edges by row (Sec. 1.1 and
 *                    Sec. 5.3: COO -> CSR conversion); duplicates kept.
 *   oracle_spmv64    Algorithm 3 (SpMV) over CSR rows, accumulated in FP64 in
 *                    index order.
 *   oracle_mlp_*     the 16-64-64-1 ReLU regressor used by the reorder
 *                    selector (not in the paper), FP64 forward, analytic
 *                    backward of the mean squared error, and one Adam step.
 *   oracle_nbr       the NBR spatial-locality metric of Sec. 5.2.
 *   oracle_bin_by_dst  binning of the edge list by destination before BOBA,
 *                    the remedy Sec. 5.6 suggests for edges in random order:
 *                    a stable counting sort by dst >> shift.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG 1
#define ORACLE_ERR_RANGE 2

/* Algorithm 1 + isolated-vertex tail.  perm[v] = new ID of old vertex v;
 * order[k] = old vertex placed k-th (the paper's p).  Either may be NULL. */
int oracle_boba(const int32_t *I, const int32_t *J, int64_t m, int64_t n,
                int interleaved, int32_t *perm, int32_t *order)
{
    if (m < 0 || n < 0) return ORACLE_ERR_ARG;
    if (m > 0 && (!I || !J)) return ORACLE_ERR_ARG;
    int32_t *seen = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!seen) return ORACLE_ERR_ARG;
    for (int64_t v = 0; v < n; ++v) seen[v] = -1;      /* S <- empty set */
    int64_t next = 0;                                    /* i <- 0 */

    /* visit one occurrence: if v is not in S, p_i <- v, i <- i+1, S <- S u {v} */
#define VISIT(vv)                                                   \
    do {                                                            \
        int64_t v_ = (vv);                                          \
        if (v_ < 0 || v_ >= n) { free(seen); return ORACLE_ERR_RANGE; } \
        if (seen[v_] < 0) seen[v_] = (int32_t)next++;               \
    } while (0)

    if (!interleaved) {
        for (int64_t j = 0; j < m; ++j) VISIT(I[j]);     /* first loop: sources */
        for (int64_t j = 0; j < m; ++j) VISIT(J[j]);     /* second loop: destinations */
    } else {
        for (int64_t j = 0; j < m; ++j) { VISIT(I[j]); VISIT(J[j]); }
    }
    /* vertices that never occur: appended in increasing old ID */
    for (int64_t v = 0; v < n; ++v) VISIT(v);
#undef VISIT

    for (int64_t v = 0; v < n; ++v) {
        if (perm) perm[v] = seen[v];
        if (order) order[seen[v]] = (int32_t)v;
    }
    free(seen);
    return ORACLE_OK;
}

/* I'(k) = perm(I(k)), J'(k) = perm(J(k)); edge order untouched. */
int oracle_relabel(const int32_t *I, const int32_t *J, int64_t m,
                   const int32_t *perm, int64_t n, int32_t *I2, int32_t *J2)
{
    if (m < 0 || n < 0) return ORACLE_ERR_ARG;
    for (int64_t k = 0; k < m; ++k) {
        if (I[k] < 0 || I[k] >= n || J[k] < 0 || J[k] >= n) return ORACLE_ERR_RANGE;
        I2[k] = perm[I[k]];
        J2[k] = perm[J[k]];
    }
    return ORACLE_OK;
}

/* Stable counting sort by row.  rowptr[r+1]-rowptr[r] = #edges with row r;
 * within a row, edges keep their input order.  val / val_out may be NULL. */
int oracle_coo_to_csr(const int32_t *row, const int32_t *col, const float *val,
                      int64_t m, int64_t n_rows, int32_t *rowptr,
                      int32_t *col_out, float *val_out)
{
    if (m < 0 || n_rows < 0) return ORACLE_ERR_ARG;
    for (int64_t r = 0; r <= n_rows; ++r) rowptr[r] = 0;
    for (int64_t k = 0; k < m; ++k) {
        if (row[k] < 0 || row[k] >= n_rows) return ORACLE_ERR_RANGE;
        rowptr[row[k] + 1] += 1;                         /* degree count */
    }
    for (int64_t r = 0; r < n_rows; ++r) rowptr[r + 1] += rowptr[r];  /* prefix sum */
    int32_t *cursor = (int32_t *)malloc((size_t)(n_rows > 0 ? n_rows : 1) * sizeof(int32_t));
    if (!cursor) return ORACLE_ERR_ARG;
    for (int64_t r = 0; r < n_rows; ++r) cursor[r] = rowptr[r];
    for (int64_t k = 0; k < m; ++k) {                    /* in input order: stable */
        int32_t dst = cursor[row[k]]++;
        col_out[dst] = col[k];
        if (val && val_out) val_out[dst] = val[k];
    }
    free(cursor);
    return ORACLE_OK;
}

/* y(v) = sum over the entries e of row v of val(e) * x(col(e)), in FP64,
 * summed in increasing e (Algorithm 3 over CSR rows).  val NULL means 1. */
int oracle_spmv64(const int32_t *rowptr, const int32_t *col, const float *val,
                  int64_t n_rows, int64_t n_cols, const float *x, double *y)
{
    if (n_rows < 0 || n_cols < 0) return ORACLE_ERR_ARG;
    for (int64_t r = 0; r < n_rows; ++r) {
        double acc = 0.0;
        for (int64_t e = rowptr[r]; e < rowptr[r + 1]; ++e) {
            if (col[e] < 0 || col[e] >= n_cols) return ORACLE_ERR_RANGE;
            double a = val ? (double)val[e] : 1.0;
            acc += a * (double)x[col[e]];
        }
        y[r] = acc;
    }
    return ORACLE_OK;
}

/* ---- selector MLP: 16 -> 64 -> 64 -> 1, ReLU, parameters row-major:
 *      W1[64][16] b1[64] W2[64][64] b2[64] W3[1][64] b3[1]  (5313 values) */
#define MLP_IN 16
#define MLP_H 64
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + MLP_H * MLP_IN)
#define OFF_W2 (OFF_B1 + MLP_H)
#define OFF_B2 (OFF_W2 + MLP_H * MLP_H)
#define OFF_W3 (OFF_B2 + MLP_H)
#define OFF_B3 (OFF_W3 + MLP_H)
#define MLP_NPARAM (OFF_B3 + 1)

int64_t oracle_mlp_nparam(void) { return MLP_NPARAM; }

static void mlp_row(const double *P, const double *x, double *z1, double *h1,
                    double *z2, double *h2, double *out)
{
    for (int o = 0; o < MLP_H; ++o) {
        double s = P[OFF_B1 + o];
        for (int i = 0; i < MLP_IN; ++i) s += P[OFF_W1 + o * MLP_IN + i] * x[i];
        z1[o] = s;
        h1[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < MLP_H; ++o) {
        double s = P[OFF_B2 + o];
        for (int i = 0; i < MLP_H; ++i) s += P[OFF_W2 + o * MLP_H + i] * h1[i];
        z2[o] = s;
        h2[o] = s > 0.0 ? s : 0.0;
    }
    double s = P[OFF_B3];
    for (int i = 0; i < MLP_H; ++i) s += P[OFF_W3 + i] * h2[i];
    *out = s;
}

int oracle_mlp_forward(const double *params, const double *X, int64_t B, double *yhat)
{
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H];
    for (int64_t b = 0; b < B; ++b)
        mlp_row(params, X + b * MLP_IN, z1, h1, z2, h2, &yhat[b]);
    return ORACLE_OK;
}

/* loss = (1/B) sum_b (yhat_b - y_b)^2 ; grad = d loss / d params. */
int oracle_mlp_backward(const double *params, const double *X, const double *y,
                        int64_t B, double *grad, double *loss)
{
    double z1[MLP_H], h1[MLP_H], z2[MLP_H], h2[MLP_H], g1[MLP_H], g2[MLP_H];
    for (int k = 0; k < MLP_NPARAM; ++k) grad[k] = 0.0;
    double L = 0.0;
    for (int64_t b = 0; b < B; ++b) {
        const double *x = X + b * MLP_IN;
        double out;
        mlp_row(params, x, z1, h1, z2, h2, &out);
        double d = out - y[b];
        L += d * d;
        double go = 2.0 * d / (double)B;                 /* d loss / d out */
        grad[OFF_B3] += go;
        for (int i = 0; i < MLP_H; ++i) {
            grad[OFF_W3 + i] += go * h2[i];
            g2[i] = z2[i] > 0.0 ? go * params[OFF_W3 + i] : 0.0;   /* d / d z2 */
        }
        for (int i = 0; i < MLP_H; ++i) g1[i] = 0.0;
        for (int o = 0; o < MLP_H; ++o) {
            grad[OFF_B2 + o] += g2[o];
            for (int i = 0; i < MLP_H; ++i) {
                grad[OFF_W2 + o * MLP_H + i] += g2[o] * h1[i];
                g1[i] += g2[o] * params[OFF_W2 + o * MLP_H + i];
            }
        }
        for (int o = 0; o < MLP_H; ++o) {
            double gz = z1[o] > 0.0 ? g1[o] : 0.0;       /* d / d z1 */
            grad[OFF_B1 + o] += gz;
            for (int i = 0; i < MLP_IN; ++i) grad[OFF_W1 + o * MLP_IN + i] += gz * x[i];
        }
    }
    if (loss) *loss = B > 0 ? L / (double)B : 0.0;
    return ORACLE_OK;
}

/* One Adam step (Kingma & Ba, 2015) with bias correction; t is 1-based. */
int oracle_adam(double *params, double *m1, double *m2, const double *grad, int64_t count,
                int64_t t, double lr, double b1, double b2, double eps)
{
    if (t < 1) return ORACLE_ERR_ARG;
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < count; ++k) {
        m1[k] = b1 * m1[k] + (1.0 - b1) * grad[k];
        m2[k] = b2 * m2[k] + (1.0 - b2) * grad[k] * grad[k];
        double mh = m1[k] / c1, vh = m2[k] / c2;
        params[k] -= lr * mh / (sqrt(vh) + eps);
    }
    return ORACLE_OK;
}

/* NBR (Sec. 5.2): (1/n) sum over vertices with a non-empty neighbourhood of
 * (#distinct cache lines spanned by N(v)) / |N(v)|, a line holding `line_ids`
 * consecutive IDs.  Neighbourhoods are CSR rows; duplicates count in |N(v)|
 * as they occur.  Returns the sum and the number of vertices counted, and
 * when `distinct` is not NULL the distinct lines of every row (0 if empty). */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int oracle_nbr(const int32_t *rowptr, const int32_t *col, int64_t n, int64_t line_ids,
               double *sum_ratio, int64_t *counted, int32_t *distinct)
{
    if (line_ids <= 0) return ORACLE_ERR_ARG;
    double s = 0.0;
    int64_t c = 0;
    int64_t cap = 0;
    int64_t *lines = NULL;
    for (int64_t v = 0; v < n; ++v) {
        int64_t deg = rowptr[v + 1] - rowptr[v];
        if (distinct) distinct[v] = 0;
        if (deg == 0) continue;
        if (deg > cap) {
            free(lines);
            cap = deg;
            lines = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
            if (!lines) return ORACLE_ERR_ARG;
        }
        for (int64_t e = 0; e < deg; ++e) lines[e] = col[rowptr[v] + e] / line_ids;
        qsort(lines, (size_t)deg, sizeof(int64_t), cmp_i64);
        int64_t nd = 1;
        for (int64_t e = 1; e < deg; ++e) nd += lines[e] != lines[e - 1];
        if (distinct) distinct[v] = (int32_t)nd;
        s += (double)nd / (double)deg;
        c += 1;
    }
    free(lines);
    *sum_ratio = s;
    *counted = c;
    return ORACLE_OK;
}

/* Stable counting sort of the edges by bin = dst >> shift; the bins are the
 * 2^bin_bits leading values of the bits(n - 1)-bit vertex IDs (shift =
 * max(0, bits - bin_bits)).  Inside a bin the input order is kept. */
int oracle_bin_by_dst(const int32_t *src, const int32_t *dst, int64_t m, int64_t n, int bin_bits,
                      int32_t *src_out, int32_t *dst_out)
{
    if (m < 0 || n < 0 || bin_bits < 1) return ORACLE_ERR_ARG;
    int bits = 0;
    while (bits < 31 && ((int64_t)1 << bits) < n) ++bits;
    const int key_bits = bin_bits < bits ? bin_bits : bits;
    const int shift = bits - key_bits;
    const int64_t nbins = (int64_t)1 << key_bits;
    int64_t *start = (int64_t *)calloc((size_t)nbins + 1, sizeof(int64_t));
    if (!start) return ORACLE_ERR_ARG;
    for (int64_t k = 0; k < m; ++k) {
        if (dst[k] < 0 || dst[k] >= n) { free(start); return ORACLE_ERR_RANGE; }
        start[(dst[k] >> shift) + 1] += 1;                 /* bin sizes */
    }
    for (int64_t b = 0; b < nbins; ++b) start[b + 1] += start[b];   /* bin starts */
    for (int64_t k = 0; k < m; ++k) {                      /* in input order: stable */
        const int64_t at = start[dst[k] >> shift]++;
        src_out[at] = src[k];
        dst_out[at] = dst[k];
    }
    free(start);
    return ORACLE_OK;
}
