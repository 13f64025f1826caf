/*
 * Runs the FP64 oracle on small point sets of every kind, randomisation and
 * map under AddressSanitizer and UndefinedBehaviorSanitizer (built by
 * tests/test_sanitizers.py).  The oracle's values are checked elsewhere; here
 * every call must succeed, return finite numbers and touch no memory it does
 * not own.  Exit status 0 on success.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/qmc_oracle.c"

static uint64_t rng_state = 88172645463325252ull;
static uint64_t next_u64(void) {  /* xorshift64: test inputs only */
    rng_state ^= rng_state << 13;
    rng_state ^= rng_state >> 7;
    rng_state ^= rng_state << 17;
    return rng_state;
}

static int check_finite(const double *v, int64_t n, const char *what) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(v[i])) {
            fprintf(stderr, "%s: non-finite value at %lld\n", what, (long long)i);
            return 1;
        }
    return 0;
}

static int run_case(int b, int kind, int rand, int map, int m, int s, int t, int R, int upper) {
    int32_t *w = malloc(sizeof(int32_t) * s);
    int e_max = 0;
    for (int j = 0; j < s; ++j) {
        int q = 0;
        while (q < m + 1) {  /* w_j = floor(log_b(j+1)), capped at m + 1 */
            uint64_t p = 1;
            for (int i = 0; i <= q; ++i) p *= (uint64_t)b;
            if (p > (uint64_t)(j + 1)) break;
            ++q;
        }
        w[j] = q;
        (void)e_max;
    }
    uint64_t nb_total = 1;
    for (int i = 0; i < m; ++i) nb_total *= (uint64_t)b;
    int ngen = kind == QO_DIGITAL_NET ? s * m : s;
    uint64_t *gen = malloc(sizeof(uint64_t) * ngen);
    for (int j = 0; j < s; ++j) {
        int e = m - (w[j] < m ? w[j] : m);
        uint64_t ne = 1;
        for (int i = 0; i < e; ++i) ne *= (uint64_t)b;
        if (kind == QO_DIGITAL_NET) {
            for (int q = 0; q < m; ++q) {  /* triangular with a unit diagonal, digits below b */
                uint64_t word = 0, pw = 1;
                for (int p = 0; p < m; ++p) {
                    uint64_t d = p == q ? 1 : ((upper ? p < q : p > q) ? next_u64() % (uint64_t)b : 0);
                    word += d * pw;
                    pw *= (uint64_t)b;
                }
                gen[j * m + q] = word;
            }
        } else if (e == 0) {
            gen[j] = 1;
        } else {  /* a unit below b^e: the constant digit nonzero */
            uint64_t g = next_u64() % ne;
            g -= g % (uint64_t)b;
            gen[j] = g + 1 + next_u64() % (uint64_t)(b - 1);
            if (gen[j] >= ne) gen[j] = 1;
        }
    }
    double *shift = malloc(sizeof(double) * R * s);
    uint64_t *dshift = malloc(sizeof(uint64_t) * R * s);
    for (int i = 0; i < R * s; ++i) {
        shift[i] = (double)(next_u64() >> 11) * 0x1p-53;
        dshift[i] = b == 2 ? next_u64() >> 12 : (next_u64() >> 12) % 1000000007ull;
    }
    int64_t sample_total = 0;
    for (int j = 0; j < s; ++j) {
        int e = m - (w[j] < m ? w[j] : m);
        int64_t ne = 1;
        for (int i = 0; i < e; ++i) ne *= b;
        sample_total += ne;
    }
    double *samples = malloc(sizeof(double) * R * sample_total);
    for (int64_t i = 0; i < R * sample_total; ++i) samples[i] = ((double)(next_u64() >> 11) + 0.5) * 0x1p-53;
    qo_spec sp = {b, kind, m, s, w, gen, rand, R, shift, dshift, map, samples};
    int64_t N = (int64_t)nb_total;
    double *A = malloc(sizeof(double) * s * t);
    for (int i = 0; i < s * t; ++i) A[i] = ((double)(next_u64() >> 11) * 0x1p-53 - 0.5) * 0.3;
    double *X = malloc(sizeof(double) * N * s);
    double *Y = malloc(sizeof(double) * N * t);
    double *Q = malloc(sizeof(double) * R);
    double *dA = malloc(sizeof(double) * R * s * t);
    int bad = 0;
    int64_t cnt = 0;
    if (qo_point_matrix_unreduced(&sp, 0, X)) bad |= 1;
    bad |= check_finite(X, N * s, "point matrix");
    if (qo_reduced_matvec(&sp, 0, A, t, Y, &cnt)) bad |= 2;
    bad |= check_finite(Y, N * t, "reduced matvec");
    qo_integrand f = {QO_G_COS, 1.0, QO_H_ID, 0.0};
    if (qo_estimate(&sp, A, t, &f, Q, &cnt)) bad |= 4;
    bad |= check_finite(Q, R, "estimate");
    qo_integrand fc = {QO_G_EXP, 0.2, QO_H_CALL, 1.0};
    if (qo_estimate_grad(&sp, A, t, &fc, Q, dA)) bad |= 8;
    bad |= check_finite(dA, R * s * t, "gradient");
    for (int j = 0; j < s; ++j) {
        int e = m - (w[j] < m ? w[j] : m);
        int64_t ne = 1;
        for (int i = 0; i < e; ++i) ne *= b;
        double *v = malloc(sizeof(double) * ne);
        if (qo_point_values(&sp, R - 1, j, v)) bad |= 16;
        bad |= check_finite(v, ne, "point values");
        free(v);
    }
    if (bad) fprintf(stderr, "case b=%d kind=%d rand=%d map=%d: failure mask %d\n", b, kind, rand, map, bad);
    free(w); free(gen); free(shift); free(dshift); free(samples); free(A); free(X); free(Y); free(Q); free(dA);
    return bad;
}

int main(void) {
    int bad = 0;
    for (int kind = 0; kind < 4; ++kind)
        for (int rand = 0; rand < 3; ++rand)
            for (int map = 0; map < 4; ++map) {
                if (kind == QO_IID && rand != QO_NO_SHIFT) continue;
                if (map == QO_MAP_INVNORM && rand == QO_NO_SHIFT && kind != QO_IID) continue;
                int R = rand == QO_NO_SHIFT && kind != QO_IID ? 1 : 2;
                bad |= run_case(2, kind, rand, map, 7, 20, 9, R, 0);
                if (kind == QO_DIGITAL_NET) bad |= run_case(2, kind, rand, map, 6, 12, 5, R, 1);
                bad |= run_case(3, kind, rand, map, 4, 15, 7, R, 0);
            }
    printf(bad ? "oracle driver: FAILED\n" : "oracle driver: ok\n");
    return bad ? 1 : 0;
}
