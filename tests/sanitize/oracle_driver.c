/*
 * Drives every function of the CPU oracle (oracle/boba_oracle.c, included
 * below) over small seeded inputs and edge cases, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: any out-of-bounds access,
 * leak or undefined operation aborts with a report.  Also checks the results'
 * basic invariants so that every branch does real work.  Exit status 0: clean.
 */
#include "oracle/boba_oracle.c" /* compiled with -I <repository root> */

#include <stdio.h>

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void)
{
    /* xorshift64*, enough for test inputs */
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 32);
}

#define CHECK(c)                                                              \
    do {                                                                      \
        if (!(c)) {                                                           \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);   \
            return 1;                                                         \
        }                                                                     \
    } while (0)

static int graph_case(int64_t n, int64_t m)
{
    int32_t *I = malloc((size_t)(m > 0 ? m : 1) * 4), *J = malloc((size_t)(m > 0 ? m : 1) * 4);
    int32_t *perm = malloc((size_t)(n > 0 ? n : 1) * 4), *order = malloc((size_t)(n > 0 ? n : 1) * 4);
    int32_t *I2 = malloc((size_t)(m > 0 ? m : 1) * 4), *J2 = malloc((size_t)(m > 0 ? m : 1) * 4);
    int32_t *rowptr = malloc((size_t)(n + 1) * 4), *col = malloc((size_t)(m > 0 ? m : 1) * 4);
    int32_t *distinct = malloc((size_t)(n > 0 ? n : 1) * 4);
    float *val = malloc((size_t)(m > 0 ? m : 1) * 4), *val2 = malloc((size_t)(m > 0 ? m : 1) * 4);
    float *x = malloc((size_t)(n > 0 ? n : 1) * 4);
    double *y = malloc((size_t)(n > 0 ? n : 1) * 8);
    char *hit = calloc((size_t)(n > 0 ? n : 1), 1);
    for (int64_t k = 0; k < m; ++k) {
        I[k] = (int32_t)(rnd() % (uint32_t)n);
        J[k] = (int32_t)(rnd() % (uint32_t)n);
        val[k] = (float)(rnd() % 2001) / 1000.0f - 1.0f;
    }
    for (int64_t v = 0; v < n; ++v) x[v] = (float)(rnd() % 2001) / 1000.0f - 1.0f;
    for (int inter = 0; inter < 2; ++inter) {
        CHECK(oracle_boba(I, J, m, n, inter, perm, order) == ORACLE_OK);
        memset(hit, 0, (size_t)(n > 0 ? n : 1));
        for (int64_t v = 0; v < n; ++v) {
            CHECK(perm[v] >= 0 && perm[v] < n && !hit[perm[v]]);
            hit[perm[v]] = 1;
            CHECK(order[perm[v]] == v);
        }
    }
    CHECK(oracle_relabel(I, J, m, perm, n, I2, J2) == ORACLE_OK);
    CHECK(oracle_coo_to_csr(I2, J2, val, m, n, rowptr, col, val2) == ORACLE_OK);
    CHECK(rowptr[0] == 0 && rowptr[n] == m);
    CHECK(oracle_coo_to_csr(I2, J2, NULL, m, n, rowptr, col, NULL) == ORACLE_OK);
    CHECK(oracle_spmv64(rowptr, col, val2, n, n, x, y) == ORACLE_OK);
    CHECK(oracle_spmv64(rowptr, col, NULL, n, n, x, y) == ORACLE_OK);
    double s = 0.0;
    int64_t counted = 0;
    CHECK(oracle_nbr(rowptr, col, n, 32, &s, &counted, distinct) == ORACLE_OK);
    CHECK(oracle_nbr(rowptr, col, n, 1, &s, &counted, NULL) == ORACLE_OK);
    CHECK(counted <= n && s <= (double)counted + 1e-9);
    for (int bb = 1; bb <= 12; bb += 5) CHECK(oracle_bin_by_dst(I, J, m, n, bb, I2, J2) == ORACLE_OK);
    if (m > 0) {  /* an out-of-range ID is an error, never an access past the arrays */
        int32_t keep = J[m - 1];
        J[m - 1] = (int32_t)n;
        CHECK(oracle_boba(I, J, m, n, 0, perm, order) == ORACLE_ERR_RANGE);
        CHECK(oracle_relabel(I, J, m, perm, n, I2, J2) == ORACLE_ERR_RANGE);
        CHECK(oracle_bin_by_dst(I, J, m, n, 3, I2, J2) == ORACLE_ERR_RANGE);
        J[m - 1] = -1;
        CHECK(oracle_boba(I, J, m, n, 1, perm, order) == ORACLE_ERR_RANGE);
        CHECK(oracle_coo_to_csr(J, I, val, m, n, rowptr, col, val2) == ORACLE_ERR_RANGE);
        J[m - 1] = keep;
    }
    free(I); free(J); free(perm); free(order); free(I2); free(J2); free(rowptr); free(col);
    free(distinct); free(val); free(val2); free(x); free(y); free(hit);
    return 0;
}

static int mlp_case(int64_t B)
{
    const int64_t np = oracle_mlp_nparam();
    double *P = malloc((size_t)np * 8), *G = malloc((size_t)np * 8), *m1 = calloc((size_t)np, 8),
           *m2 = calloc((size_t)np, 8);
    double *X = malloc((size_t)(B > 0 ? B : 1) * MLP_IN * 8), *Y = malloc((size_t)(B > 0 ? B : 1) * 8),
           *Yh = malloc((size_t)(B > 0 ? B : 1) * 8);
    for (int64_t k = 0; k < np; ++k) P[k] = (double)(rnd() % 2001) / 10000.0 - 0.1;
    for (int64_t k = 0; k < B * MLP_IN; ++k) X[k] = (double)(rnd() % 2001) / 1000.0 - 1.0;
    for (int64_t b = 0; b < B; ++b) Y[b] = (double)(rnd() % 2001) / 1000.0 - 1.0;
    double loss = 0.0;
    CHECK(oracle_mlp_forward(P, X, B, Yh) == ORACLE_OK);
    for (int t = 1; t <= 3; ++t) {
        CHECK(oracle_mlp_backward(P, X, Y, B, G, &loss) == ORACLE_OK);
        CHECK(oracle_adam(P, m1, m2, G, np, t, 1e-3, 0.9, 0.999, 1e-8) == ORACLE_OK);
    }
    CHECK(oracle_adam(P, m1, m2, G, np, 0, 1e-3, 0.9, 0.999, 1e-8) == ORACLE_ERR_ARG);
    free(P); free(G); free(m1); free(m2); free(X); free(Y); free(Yh);
    return 0;
}

int main(void)
{
    static const int64_t sizes[][2] = {{0, 0}, {1, 0}, {1, 9}, {5, 4}, {100, 7}, {1000, 1000}, {777, 5000},
                                       {4096, 40001}};
    for (size_t c = 0; c < sizeof(sizes) / sizeof(sizes[0]); ++c)
        if (graph_case(sizes[c][0], sizes[c][1])) return 1;
    CHECK(oracle_boba(NULL, NULL, -1, 3, 0, NULL, NULL) == ORACLE_ERR_ARG);
    CHECK(oracle_boba(NULL, NULL, 2, 3, 0, NULL, NULL) == ORACLE_ERR_ARG);
    CHECK(oracle_bin_by_dst(NULL, NULL, 0, 3, 0, NULL, NULL) == ORACLE_ERR_ARG);
    if (mlp_case(1) || mlp_case(7) || mlp_case(256)) return 1;
    puts("oracle driver ok");
    return 0;
}
