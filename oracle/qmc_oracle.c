/*
 * FP64 CPU oracle for the reduced QMC matrix-vector product.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  The product path
 * (the HIP library) shares no code, header, table or helper with it.
 *
 * Everything here is plain, slow and written to be checked by eye against the
 * paper (Dick, Ebert, Herrmann, Kritzer, Longo, "The fast reduced QMC
 * matrix-vector product"):
 *
 *   point sets   Sec. 1.1 (rank-1 lattice, polynomial lattice and the map nu),
 *                Sec. 1.3 (reduced lattices: z = (b^{w_j} z_j), values
 *                (k z_j mod b^{m-w_j}) / b^{m-w_j}), Sec. 3 (digital nets,
 *                eq. def:digital; reduced generating matrices,
 *                eq. reduced_genmat_net2; Algorithm 3),
 *   shift / maps Sec. 1.2 (random shift {x + Delta}; tent map), Sec. 2.3
 *                (maps applied component-wise to the repeated values),
 *   product      Algorithm 1 (fast reduced matrix product), the dense product
 *                X A of eq. QMC_matrix,
 *   estimate     eq. QMC-rule, Q_N(f) = N^{-1} sum_k f(x_k^T A),
 *   reduced MC   Sec. 4, eq. randpts: coordinate j draws N_j i.i.d. samples
 *                and point n uses the one selected by the mixed-radix digits
 *                of n (the samples are inputs, drawn by the caller).
 *
 * Readings where the paper is silent (all listed in the design notes):
 *   - the digital shift XORs the first 52 base-2 digits with a 52-bit integer
 *     delta and takes the midpoint of the remaining digits:
 *     x = (2U + 1) 2^-53,  U = (c << (52 - n)) ^ delta;
 *   - the random shift is one IEEE FP64 addition followed by "subtract 1 if the
 *     sum is >= 1";
 *   - in a prime base b > 2 a value c / b^e is one correctly rounded FP64
 *     division; polynomials and generating-matrix columns are the base-b
 *     digits of the integers given (b = 2: the bit masks); the digital shift
 *     adds the K base-b digits of an integer delta < b^K (b^K <= 2^52, most
 *     significant first) digit by digit mod b and takes the midpoint of the
 *     rest: x = (U + 1/2) / b^K (for b = 2, K = 52 and x = (2U + 1) 2^-53);
 *     a net that is not periodic after reduction takes Algorithm 4 in any
 *     prime base, its values indexed by the integer of the output digits;
 *   - the inverse normal map is Wichura's algorithm AS241 (PPND16);
 *   - the integrand is f(y) = h(t^-1 sum_i g(y_i)) with g in {y, cos y,
 *     exp(c y)} and h in {u, max(0, u - K)}; h'(K) is taken as 0;
 *   - the gradient dQ/dA is the plain chain rule; its reduced form (fold of
 *     the point-wise sensitivities over residue classes, then the distinct
 *     values) is the transpose of Algorithm 1, or of Algorithm 4 for a net
 *     that is not periodic (sums over the points sharing a value).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no FMA contraction,
 * so every table value is one IEEE operation sequence).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

enum { QO_LATTICE = 0, QO_POLY_LATTICE = 1, QO_DIGITAL_NET = 2, QO_IID = 3 };
enum { QO_NO_SHIFT = 0, QO_RANDOM_SHIFT = 1, QO_DIGITAL_SHIFT = 2 };
enum { QO_MAP_ID = 0, QO_MAP_CENTER = 1, QO_MAP_INVNORM = 2, QO_MAP_TENT = 3 };
enum { QO_G_ID = 0, QO_G_COS = 1, QO_G_EXP = 2 };
enum { QO_H_ID = 0, QO_H_CALL = 1 };

/* A point set: prime base b, N = b^m points in s dimensions (digital nets and
 * polynomial lattices: b = 2). */
typedef struct {
    int32_t b, kind, m, s;
    const int32_t *w;         /* [s] reduction indices, w[0] = 0, non-decreasing */
    const uint64_t *gen;      /* lattice z'_j [s]; poly g'_j bits [s]; net column words [s*m] */
    int32_t rand, R;
    const double *shift;      /* [R*s] random shifts in [0,1) */
    const uint64_t *dshift;   /* [R*s] digital shifts, 52-bit integers */
    int32_t map;
    const double *samples;    /* QO_IID: [R][sum_j n_j] uniforms, coordinate blocks contiguous */
} qo_spec;

typedef struct {
    int32_t g;   /* QO_G_* */
    double c;    /* g = exp(c y) */
    int32_t h;   /* QO_H_* */
    double K;    /* h = max(0, u - K) */
} qo_integrand;

/* ------------------------------------------------------------ small helpers */

/* e_j = m - min(w_j, m): coordinate j has n_j = b^{e_j} distinct values */
static int nbits_of(const qo_spec *sp, int j) {
    int w = sp->w[j];
    return sp->m - (w < sp->m ? w : sp->m);
}

static uint64_t ipow(uint64_t b, int e) {
    uint64_t r = 1;
    for (int i = 0; i < e; ++i) r *= b;
    return r;
}

static uint64_t n_of(const qo_spec *sp, int j) { return ipow((uint64_t)sp->b, nbits_of(sp, j)); }
static int64_t N_of(const qo_spec *sp) { return (int64_t)ipow((uint64_t)sp->b, sp->m); }

/* base-b digits of v, least significant first: d[i] = floor(v / b^i) mod b, i < n */
static void digits_b(uint64_t v, uint64_t b, int n, int *d) {
    for (int i = 0; i < n; ++i) { d[i] = (int)(v % b); v /= b; }
}

/* the integer sum_{i<n} d[i] b^i */
static uint64_t undigits_b(const int *d, uint64_t b, int n) {
    uint64_t v = 0;
    for (int i = n - 1; i >= 0; --i) v = v * b + (uint64_t)d[i];
    return v;
}

/* K: the number of base-b digits of the digital shift, the largest with b^K <= 2^52 */
static int shift_digits(uint64_t b) {
    int K = 0;
    uint64_t v = 1;
    while (v <= (UINT64_C(1) << 52) / b) { v *= b; ++K; }
    return K;
}

/* F_b[x]: coefficients of a(x) g(x) mod x^e, a and g given by their base-b
 * digits (coefficient i = digit i), returned as the integer with those digits */
static uint64_t polymul_mod_b(uint64_t a, uint64_t g, int e, uint64_t b) {
    int da[64], dg[64], dr[64];
    digits_b(a, b, e, da);
    digits_b(g, b, e, dg);
    for (int i = 0; i < e; ++i) {
        int acc = 0;
        for (int k = 0; k <= i; ++k) acc = (acc + da[k] * dg[i - k]) % (int)b;
        dr[i] = acc;
    }
    return undigits_b(dr, b, e);
}

/* Net over F_b: output digits y_p = sum_q C_{p,q} a_q mod b for p <= e (rows
 * past e of the reduced matrix are zero), a_q the digits of a (q <= m); the
 * column words hold C_{p,q} as base-b digit p-1.  Returns c = sum_{p<=e}
 * y_p b^{e-p} (y_1 most significant). */
static uint64_t netmul_b(const qo_spec *sp, int j, uint64_t a, int e) {
    uint64_t b = (uint64_t)sp->b;
    int m = sp->m, da[64], y[64] = {0}, col[64];
    digits_b(a, b, m, da);
    for (int q = 0; q < m; ++q) {
        if (!da[q]) continue;
        digits_b(sp->gen[(size_t)j * m + q], b, e, col);
        for (int p = 0; p < e; ++p) y[p] = (y[p] + col[p] * da[q]) % (int)b;
    }
    uint64_t c = 0;
    for (int p = 0; p < e; ++p) c = c * b + (uint64_t)y[p];
    return c;
}

/* carry-less product of two F_2[x] polynomials given as bit masks, mod x^nb */
static uint64_t clmul_mod(uint64_t a, uint64_t b, int nb) {
    uint64_t r = 0;
    for (int i = 0; i < nb && i < 64; ++i)
        if ((a >> i) & 1u) r ^= b << i;   /* terms of degree >= 64 are >= nb: dropped */
    return nb >= 64 ? r : (r & ((UINT64_C(1) << nb) - 1));
}

/* reverse the low nb bits of v */
static uint64_t bitrev(uint64_t v, int nb) {
    uint64_t r = 0;
    for (int i = 0; i < nb; ++i)
        if ((v >> i) & 1u) r |= UINT64_C(1) << (nb - 1 - i);
    return r;
}

/* Wichura (1988), Algorithm AS241 PPND16: the normal quantile, FP64. */
double qo_invnorm(double p) {
    static const double a[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2,
        1.9715909503065514427e+3, 1.3731693765509461125e+4, 4.5921953931549871457e+4,
        6.7265770927008700853e+4, 3.3430575583588128105e+4, 2.5090809287301226727e+3};
    static const double b[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
        5.3941960214247511077e+3, 2.1213794301586595867e+4, 3.9307895800092710610e+4,
        2.8729085735721942674e+4, 5.2264952788528545610e+3};
    static const double c[8] = {1.42343711074968357734e0, 4.63033784615654529590e0,
        5.76949722146069140550e0, 3.64784832476320460504e0, 1.27045825245236838258e0,
        2.41780725177450611770e-1, 2.27238449892691845833e-2, 7.74545014278341407640e-4};
    static const double d[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
        6.89767334985100004550e-1, 1.48103976427480074590e-1, 1.51986665636164571966e-2,
        5.47593808499534494600e-4, 1.05075007164441684324e-9};
    static const double e[8] = {6.65790464350110377720e0, 5.46378491116411436990e0,
        1.78482653991729133580e0, 2.96560571828504891230e-1, 2.65321895265761230930e-2,
        1.24266094738807843860e-3, 2.71155556874348757815e-5, 2.01033439929228813265e-7};
    static const double f[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
        1.48753612908506148525e-2, 7.86869131145613259100e-4, 1.84631831751005468180e-5,
        1.42151175831644588870e-7, 2.04426310338993978564e-15};
    double q = p - 0.5;
    if (fabs(q) <= 0.425) {
        double r = 0.180625 - q * q, num = a[7], den = b[7];
        for (int i = 6; i >= 0; --i) { num = num * r + a[i]; den = den * r + b[i]; }
        return q * num / den;
    }
    double r = q < 0 ? p : 1.0 - p;
    if (r <= 0) return q < 0 ? -HUGE_VAL : HUGE_VAL;
    r = sqrt(-log(r));
    double num, den;
    if (r <= 5.0) {
        r -= 1.6; num = c[7]; den = d[7];
        for (int i = 6; i >= 0; --i) { num = num * r + c[i]; den = den * r + d[i]; }
    } else {
        r -= 5.0; num = e[7]; den = f[7];
        for (int i = 6; i >= 0; --i) { num = num * r + e[i]; den = den * r + f[i]; }
    }
    double v = num / den;
    return q < 0 ? -v : v;
}

/* The component map (Sec. 2.3; tent map of Sec. 1.2). */
static double apply_map(const qo_spec *sp, double x) {
    switch (sp->map) {
        case QO_MAP_CENTER: return x - 0.5;
        case QO_MAP_INVNORM: return qo_invnorm(x);
        case QO_MAP_TENT: return 1.0 - fabs(1.0 - 2.0 * x);
        default: return x;
    }
}

/* Shift then map one coordinate value given as the integer c of c / b^nb. */
static double shift_and_map(const qo_spec *sp, int r, int j, uint64_t c, int nb) {
    double x;
    if (sp->rand == QO_DIGITAL_SHIFT && sp->b == 2) {
        uint64_t U = (c << (52 - nb)) ^ sp->dshift[(size_t)r * sp->s + j];
        x = (double)(2 * U + 1) * 0x1p-53;                  /* exact */
    } else if (sp->rand == QO_DIGITAL_SHIFT) {
        /* digits p = 1..K of x: those of c (p <= nb) plus those of delta, mod b */
        uint64_t b = (uint64_t)sp->b;
        int K = shift_digits(b), dc[64], dd[64], du[64];
        digits_b(c, b, nb, dc);                               /* dc[nb - p] = digit p */
        digits_b(sp->dshift[(size_t)r * sp->s + j], b, K, dd);  /* dd[K - p] = digit p */
        for (int p = 1; p <= K; ++p) {
            int yp = p <= nb ? dc[nb - p] : 0;
            du[K - p] = (yp + dd[K - p]) % (int)b;
        }
        double U = (double)undigits_b(du, b, K);               /* exact, < 2^52 */
        x = (U + 0.5) / (double)ipow(b, K);                    /* one rounding */
    } else {
        /* one correctly rounded division (exact for b = 2) */
        x = (double)c / (double)ipow((uint64_t)sp->b, nb);
        if (sp->rand == QO_RANDOM_SHIFT) {
            x = x + sp->shift[(size_t)r * sp->s + j];        /* one rounding */
            if (x >= 1.0) x = x - 1.0;                       /* exact */
        }
    }
    return apply_map(sp, x);
}

/* ------------------------------------------------------------ reduced Monte Carlo
 *
 * Sec. 4: with N_j = b^{m - w_j} (capped at m), N_{s+1} = 1 and
 * M_j = N_j / N_{j+1}, every n < N is n = sum_i m_i N_{i+1} with 0 <= m_i < M_i,
 * and eq. randpts gives coordinate j of point n the sample with index
 * sum_{i >= j} m_i N_{i+1} among the N_j i.i.d. samples of that coordinate.
 * Indices below are 0-based (the paper's j is j + 1 here).
 */
static int64_t iid_offset(const qo_spec *sp, int j) {   /* start of coordinate j's samples */
    int64_t off = 0;
    for (int i = 0; i < j; ++i) off += (int64_t)n_of(sp, i);
    return off;
}

static uint64_t iid_N(const qo_spec *sp, int i) {       /* N_i, and N_s = 1 past the last */
    return i >= sp->s ? 1 : n_of(sp, i);
}

static uint64_t iid_index(const qo_spec *sp, int j, uint64_t n) {
    uint64_t idx = 0;
    for (int i = sp->s - 1; i >= j; --i) {
        uint64_t weight = iid_N(sp, i + 1);               /* N_{i+1} */
        uint64_t M = iid_N(sp, i) / weight;                /* M_i */
        uint64_t digit = (n / weight) % M;                 /* m_i */
        idx += digit * weight;
    }
    return idx;
}

static double iid_value(const qo_spec *sp, int r, int j, uint64_t index) {
    const double *y = sp->samples + (size_t)r * iid_offset(sp, sp->s) + iid_offset(sp, j);
    return apply_map(sp, y[index]);
}

/* ------------------------------------------------------------ point sets */

/*
 * Integer c_j(rho) of the distinct value c / n_j of coordinate j at residue
 * rho < n_j, from the reduced definitions.
 *   lattice (Sec. 1.3):   c = rho * z'_j mod n_j, n_j = b^nb
 *   polynomial (Sec. 1.1 with g_j = x^{w_j} g'_j): nu(k g_j / x^m) reduces to
 *                         int(k g'_j mod x^nb) / 2^nb, no digit reversal
 *   net (eq. def:digital with reduced_genmat_net2): digits y_p = sum_q
 *                         C_{p,q} rho_q for p <= nb, x = sum_p y_p 2^-p
 */
static uint64_t reduced_int(const qo_spec *sp, int j, uint64_t rho) {
    int nb = nbits_of(sp, j);
    uint64_t mask = nb >= 64 ? ~UINT64_C(0) : ((UINT64_C(1) << nb) - 1);
    if (sp->kind == QO_LATTICE) return (uint64_t)(((unsigned __int128)rho * sp->gen[j]) % n_of(sp, j));
    if (sp->b != 2 && sp->kind == QO_POLY_LATTICE) return polymul_mod_b(rho, sp->gen[j], nb, (uint64_t)sp->b);
    if (sp->b != 2) return netmul_b(sp, j, rho, nb);
    if (sp->kind == QO_POLY_LATTICE) return clmul_mod(rho, sp->gen[j], nb);
    uint64_t y = 0;   /* digital net: XOR of the columns selected by the digits of rho */
    for (int q = 0; q < sp->m; ++q)
        if ((rho >> q) & 1u) y ^= sp->gen[(size_t)j * sp->m + q];
    y &= mask;        /* rows p > nb of the reduced matrix are zero */
    return bitrev(y, nb);
}

static int net_is_periodic(const qo_spec *sp);

/* The bases taken here: every prime b, for every kind (reduced Monte Carlo
 * takes no shift in any base). */
static int base_supported(const qo_spec *sp) {
    if (sp->b == 2) return 1;
    if (sp->b < 2) return 0;
    for (int d = 2; d * d <= sp->b; ++d)
        if (sp->b % d == 0) return 0;
    return 1;
}

/* Distinct values X_j[rho], rho < n_j, of coordinate j for shift r (FP64). */
int qo_point_values(const qo_spec *sp, int r, int j, double *out) {
    if (!base_supported(sp)) return 3;
    int nb = nbits_of(sp, j);
    uint64_t n = n_of(sp, j);
    for (uint64_t rho = 0; rho < n; ++rho)
        out[rho] = sp->kind == QO_IID ? iid_value(sp, r, j, rho)
                                      : shift_and_map(sp, r, j, reduced_int(sp, j, rho), nb);
    return 0;
}

/*
 * Point k, coordinate j, from the UNREDUCED definitions (used only by the
 * dense check): lattice {k b^{w_j} z'_j / b^m}; polynomial nu(k(x) x^{w_j}
 * g'_j(x) / x^m); net with the full m x m reduced matrix applied to all m
 * digits of k.  Expressed as an integer over N = b^m.
 */
static uint64_t unreduced_int_over_N(const qo_spec *sp, int j, uint64_t k) {
    int m = sp->m, w = sp->w[j];
    if (sp->kind == QO_LATTICE) {
        /* z_j = b^{w_j} z'_j; when w_j >= m the component is a multiple of N */
        if (w >= m) return 0;
        uint64_t N = (uint64_t)N_of(sp);
        uint64_t z = (uint64_t)(((unsigned __int128)ipow((uint64_t)sp->b, w) * sp->gen[j]) % N);
        return (uint64_t)(((unsigned __int128)k * z) % N);
    }
    if (sp->kind == QO_POLY_LATTICE) {
        if (w >= m) return 0;
        if (sp->b != 2) {                      /* x^{w_j} g'_j: the digits shifted up by w */
            uint64_t g = (uint64_t)(((unsigned __int128)sp->gen[j] * ipow((uint64_t)sp->b, w)) % (uint64_t)N_of(sp));
            return polymul_mod_b(k, g, m, (uint64_t)sp->b);
        }
        uint64_t g = sp->gen[j] << w;          /* x^{w_j} g'_j */
        return clmul_mod(k, g, m);
    }
    int nb = nbits_of(sp, j);
    if (sp->b != 2) {
        /* the reduced matrix (rows past nb zero) on all m digits of k, read as
         * an integer over b^m: the nb leading digits, then m - nb zeros */
        return netmul_b(sp, j, k, nb) * ipow((uint64_t)sp->b, m - nb);
    }
    uint64_t y = 0;
    for (int q = 0; q < m; ++q) {
        uint64_t col = sp->gen[(size_t)j * m + q];
        /* Chat: zero rows p in {m - min(w,m) + 1, ..., m} */
        col &= nb >= 64 ? ~UINT64_C(0) : ((UINT64_C(1) << nb) - 1);
        if ((k >> q) & 1u) y ^= col;
    }
    return bitrev(y, m);
}

/* Full N x s point matrix (row k = point x_k) from the unreduced definitions. */
int qo_point_matrix_unreduced(const qo_spec *sp, int r, double *X) {
    if (!base_supported(sp)) return 3;
    int64_t N = N_of(sp);
    int s = sp->s;
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k) {
        for (int j = 0; j < s; ++j) {
            if (sp->kind == QO_IID) {   /* eq. randpts, digit by digit */
                X[k * s + j] = iid_value(sp, r, j, iid_index(sp, j, (uint64_t)k));
                continue;
            }
            uint64_t cN = unreduced_int_over_N(sp, j, (uint64_t)k);
            /* value cN / b^m; shift_and_map takes c / b^nb, so pass nb = m */
            X[k * s + j] = shift_and_map(sp, r, j, cN, sp->m);
        }
    }
    return 0;
}

/* Plain dense product Y = X A (N x s times s x t), FP64, natural order. */
int qo_dense_matvec(const double *X, int64_t N, int s, const double *A, int t, double *Y) {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < N; ++k)
        for (int i = 0; i < t; ++i) {
            double acc = 0.0;
            for (int j = 0; j < s; ++j) acc = acc + X[k * s + j] * A[(size_t)j * t + i];
            Y[k * t + i] = acc;
        }
    return 0;
}

/* ------------------------------------------------------------ Algorithm 1 */

/* a coordinate whose every value is exactly zero contributes nothing (j > s*) */
static int column_is_zero(const qo_spec *sp, int j) {
    return sp->kind != QO_IID && sp->w[j] >= sp->m && sp->rand == QO_NO_SHIFT && sp->map == QO_MAP_ID;
}

/* randomisations (shifts) or, for reduced Monte Carlo, independent replicates */
static int replicates(const qo_spec *sp) {
    return sp->kind == QO_IID || sp->rand != QO_NO_SHIFT ? sp->R : 1;
}

/*
 * Algorithm 1 for the column block [i0, i1) of A (t columns, row-major) and
 * shift r.  P must hold N x (i1 - i0) doubles; on return P = (X A)[:, i0:i1].
 * Steps j = s-1 .. 0 (0-based): P <- tile(P) to n_j rows, then P += X_j a_j.
 * The multiply-add count of the reduced columns (w_j < m) is added to *nmadd.
 */
int qo_alg1(const qo_spec *sp, int r, const double *A, int t, int i0, int i1,
            double *P, int64_t *nmadd) {
    if (!base_supported(sp)) return 3;
    int tb = i1 - i0;
    int64_t rows = 1;                 /* P_{s*+1} = 0 (1 x tb), w_{s+1} := m */
    for (int i = 0; i < tb; ++i) P[i] = 0.0;
    double *v = (double *)malloc(sizeof(double) * (size_t)N_of(sp));
    if (!v) return 1;
    int64_t count = 0;
    for (int j = sp->s - 1; j >= 0; --j) {
        if (column_is_zero(sp, j)) continue;
        int64_t nj = (int64_t)n_of(sp, j);
        /* tile: rows [rows, nj) repeat rows [0, rows) */
#pragma omp parallel for schedule(static)
        for (int64_t rho = rows; rho < nj; ++rho)
            memcpy(P + rho * tb, P + (rho % rows) * tb, sizeof(double) * tb);
        rows = nj;
        qo_point_values(sp, r, j, v);
        const double *aj = A + (size_t)j * t + i0;
#pragma omp parallel for schedule(static)
        for (int64_t rho = 0; rho < nj; ++rho)
            for (int i = 0; i < tb; ++i) P[rho * tb + i] = P[rho * tb + i] + v[rho] * aj[i];
        if (sp->w[j] < sp->m) count += nj * tb;
    }
    /* if every column was zero, P is still one row: tile to N rows */
    int64_t N = N_of(sp);
    for (int64_t rho = rows; rho < N; ++rho) memcpy(P + rho * tb, P + (rho % rows) * tb, sizeof(double) * tb);
    free(v);
    if (nmadd) *nmadd += count;
    return 0;
}

/* ------------------------------------------------------------ Algorithm 4 */

/*
 * A reduced net is periodic in k with period n_j (and Algorithm 1 applies)
 * when its reduced matrix has zero columns q > n_j; otherwise coordinate j
 * depends on every digit of k and the product needs Algorithm 4.
 */
static int net_is_periodic(const qo_spec *sp) {
    if (sp->kind != QO_DIGITAL_NET) return 1;
    for (int j = 0; j < sp->s; ++j) {
        int nb = nbits_of(sp, j);
        for (int q = nb; q < sp->m; ++q) {
            uint64_t wd = sp->gen[(size_t)j * sp->m + q];
            /* a column past nb with a nonzero digit in the first nb rows */
            if (sp->b == 2 ? (nb >= 64 ? wd : wd & ((UINT64_C(1) << nb) - 1)) != 0
                           : wd % ipow((uint64_t)sp->b, nb) != 0)
                return 0;
        }
    }
    return 1;
}

int qo_net_is_periodic(const qo_spec *sp) { return net_is_periodic(sp); }

/* Values X_j[c] of coordinate j indexed by the integer c of the reduced output
 * digits (x = c / b^nb before shift and map), c < n_j: the n_j possible values
 * of Section 3 (after eq. reduced_genmat_net2). */
int qo_output_values(const qo_spec *sp, int r, int j, double *out) {
    int nb = nbits_of(sp, j);
    uint64_t n = n_of(sp, j);
    for (uint64_t c = 0; c < n; ++c) out[c] = shift_and_map(sp, r, j, c, nb);
    return 0;
}

/* The integer of the reduced output digits of point n in coordinate j: the
 * nb leading base-b digits of the unreduced value times b^m. */
static uint64_t output_int(const qo_spec *sp, int j, uint64_t n) {
    int nb = nbits_of(sp, j);
    return unreduced_int_over_N(sp, j, n) / ipow((uint64_t)sp->b, sp->m - nb);
}

/*
 * Algorithm 4 (fast reduced matrix product for digital nets) on the column
 * block [i0, i1) for shift r: for j = s*..1, the row vectors
 * c_k = X_j[k] a_j (k < n_j) are formed and P_j = P_{j+1} + (c_{k_j(n)})_n,
 * k_j(n) = floor(y_{n,j} n_j) = the integer of the reduced output digits of n.
 * The multiplication count (n_j per column) is added to *nmadd.
 */
int qo_alg4(const qo_spec *sp, int r, const double *A, int t, int i0, int i1,
            double *P, int64_t *nmadd) {
    if (!base_supported(sp)) return 3;
    int tb = i1 - i0;
    int64_t N = N_of(sp);
    for (int64_t e = 0; e < N * tb; ++e) P[e] = 0.0;
    double *v = (double *)malloc(sizeof(double) * (size_t)N);
    double *c = (double *)malloc(sizeof(double) * (size_t)N * tb);
    if (!v || !c) { free(v); free(c); return 1; }
    int64_t count = 0;
    for (int j = sp->s - 1; j >= 0; --j) {
        if (column_is_zero(sp, j)) continue;
        int64_t nj = (int64_t)n_of(sp, j);
        qo_output_values(sp, r, j, v);
        const double *aj = A + (size_t)j * t + i0;
        for (int64_t k = 0; k < nj; ++k)
            for (int i = 0; i < tb; ++i) c[k * tb + i] = v[k] * aj[i];
        if (sp->w[j] < sp->m) count += nj * tb;
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < N; ++n) {
            uint64_t k = output_int(sp, j, (uint64_t)n);
            for (int i = 0; i < tb; ++i) P[n * tb + i] = P[n * tb + i] + c[k * tb + i];
        }
    }
    free(v); free(c);
    if (nmadd) *nmadd += count;
    return 0;
}

/* The reduced product of one column block: Algorithm 1 when the point set is
 * periodic after reduction, Algorithm 4 otherwise. */
static int reduced_product(const qo_spec *sp, int r, const double *A, int t, int i0, int i1,
                           double *P, int64_t *nmadd) {
    return net_is_periodic(sp) ? qo_alg1(sp, r, A, t, i0, i1, P, nmadd)
                               : qo_alg4(sp, r, A, t, i0, i1, P, nmadd);
}

/* ------------------------------------------------------------ integrand */

static double g_val(const qo_integrand *f, double y) {
    switch (f->g) {
        case QO_G_COS: return cos(y);
        case QO_G_EXP: return exp(f->c * y);
        default: return y;
    }
}
static double g_der(const qo_integrand *f, double y) {
    switch (f->g) {
        case QO_G_COS: return -sin(y);
        case QO_G_EXP: return f->c * exp(f->c * y);
        default: return 1.0;
    }
}
static double h_val(const qo_integrand *f, double u) {
    if (f->h == QO_H_CALL) return u > f->K ? u - f->K : 0.0;
    return u;
}
static double h_der(const qo_integrand *f, double u) {
    if (f->h == QO_H_CALL) return u > f->K ? 1.0 : 0.0;
    return 1.0;
}

/* Neumaier's compensated sum of x[0..n) in natural order. */
double qo_neumaier(const double *x, int64_t n) {
    double s = 0.0, comp = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double v = x[i], u = s + v;
        if (fabs(s) >= fabs(v)) comp += (s - u) + v; else comp += (v - u) + s;
        s = u;
    }
    return s + comp;
}

/* Column-block width used by the estimate and gradient drivers. */
static int block_width(int t) { return t < 64 ? t : 64; }

/*
 * u_k = t^-1 sum_i g(y_ki) for all points of shift r, with Y = X A built by
 * Algorithm 1 one column block at a time (columns in natural order).
 */
static int point_means(const qo_spec *sp, int r, const double *A, int t,
                       const qo_integrand *f, double *u, double *P, int64_t *nmadd) {
    int64_t N = N_of(sp);
    for (int64_t k = 0; k < N; ++k) u[k] = 0.0;
    int tb = block_width(t);
    for (int i0 = 0; i0 < t; i0 += tb) {
        int i1 = i0 + tb < t ? i0 + tb : t, w = i1 - i0;
        if (reduced_product(sp, r, A, t, i0, i1, P, nmadd)) return 1;
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < N; ++k)
            for (int i = 0; i < w; ++i) u[k] = u[k] + g_val(f, P[k * w + i]);
    }
    for (int64_t k = 0; k < N; ++k) u[k] = u[k] / (double)t;
    return 0;
}

/* Q[r] = N^-1 sum_k h(u_k) for every shift r (eq. QMC-rule). */
int qo_estimate(const qo_spec *sp, const double *A, int t, const qo_integrand *f,
                double *Q, int64_t *nmadd) {
    int64_t N = N_of(sp);
    int tb = block_width(t);
    double *P = (double *)malloc(sizeof(double) * (size_t)N * tb);
    double *u = (double *)malloc(sizeof(double) * (size_t)N);
    if (!P || !u) { free(P); free(u); return 1; }
    int R = replicates(sp);
    for (int r = 0; r < R; ++r) {
        if (point_means(sp, r, A, t, f, u, P, nmadd)) { free(P); free(u); return 1; }
        for (int64_t k = 0; k < N; ++k) u[k] = h_val(f, u[k]);
        Q[r] = qo_neumaier(u, N) / (double)N;
    }
    free(P); free(u);
    return 0;
}

/*
 * Gradient of Q_r with respect to A: dA[r][j][i] = sum_k x_kj G_ki with
 * G_ki = N^-1 h'(u_k) t^-1 g'(y_ki).  Because x_kj = X_j[k mod n_j], the sum
 * over k folds into residue classes: S_j[rho] = sum_{k = rho mod n_j} G_k,
 * dA_j = sum_rho X_j[rho] S_j[rho].  The fold is done j = 0 .. s-1, each
 * step summing the classes of the previous (finer) one: the transpose of the
 * tiling in Algorithm 1.  A net that is not periodic after reduction takes
 * the transpose of Algorithm 4 instead (see there).  Also returns Q.
 */
int qo_estimate_grad(const qo_spec *sp, const double *A, int t, const qo_integrand *f,
                     double *Q, double *dA) {
    int64_t N = N_of(sp);
    int s = sp->s, tb = block_width(t);
    const int periodic = net_is_periodic(sp);
    double *P = (double *)malloc(sizeof(double) * (size_t)N * tb);
    double *u = (double *)malloc(sizeof(double) * (size_t)N);
    double *hv = (double *)malloc(sizeof(double) * (size_t)N);
    double *v = (double *)malloc(sizeof(double) * (size_t)N);
    double *S = periodic ? NULL : (double *)malloc(sizeof(double) * (size_t)N * tb);
    if (!P || !u || !hv || !v || (!periodic && !S)) {
        free(P); free(u); free(hv); free(v); free(S); return 1;
    }
    int R = replicates(sp);
    for (int r = 0; r < R; ++r) {
        if (point_means(sp, r, A, t, f, u, P, NULL)) { free(P); free(u); free(hv); free(v); free(S); return 1; }
        for (int64_t k = 0; k < N; ++k) hv[k] = h_val(f, u[k]);
        Q[r] = qo_neumaier(hv, N) / (double)N;
        double *dAr = dA + (size_t)r * s * t;
        for (int i0 = 0; i0 < t; i0 += tb) {
            int i1 = i0 + tb < t ? i0 + tb : t, w = i1 - i0;
            if (reduced_product(sp, r, A, t, i0, i1, P, NULL)) {
                free(P); free(u); free(hv); free(v); free(S); return 1;
            }
            /* G in place of Y */
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < N; ++k) {
                double hk = h_der(f, u[k]) / ((double)N * (double)t);
                for (int i = 0; i < w; ++i) P[k * w + i] = hk * g_der(f, P[k * w + i]);
            }
            if (!periodic) {
                /* Algorithm 4 transposed (a net that is not periodic):
                 * point n contributes to the value X_j[c] with c = floor(y_{n,j} n_j),
                 * the integer of its reduced output digits, so
                 * dA_j = sum_c X_j[c] S_j[c],  S_j[c] = sum of G_n over those n */
                for (int j = 0; j < s; ++j) {
                    int64_t nj = (int64_t)n_of(sp, j);
                    for (int64_t e = 0; e < nj * w; ++e) S[e] = 0.0;
                    for (int64_t n = 0; n < N; ++n) {
                        uint64_t c = output_int(sp, j, (uint64_t)n);
                        for (int i = 0; i < w; ++i) S[c * w + i] = S[c * w + i] + P[n * w + i];
                    }
                    qo_output_values(sp, r, j, v);
                    for (int i = 0; i < w; ++i) {
                        double acc = 0.0;
                        for (int64_t c = 0; c < nj; ++c) acc = acc + v[c] * S[c * w + i];
                        dAr[(size_t)j * t + i0 + i] = acc;
                    }
                }
                continue;
            }
            int64_t rows = N;
            for (int j = 0; j < s; ++j) {
                int64_t nj = (int64_t)n_of(sp, j);
                /* fold: S[rho] = sum_c S[rho + c nj], rho < nj */
                if (nj < rows) {
                    int64_t reps = rows / nj;
#pragma omp parallel for schedule(static)
                    for (int64_t rho = 0; rho < nj; ++rho)
                        for (int64_t c = 1; c < reps; ++c)
                            for (int i = 0; i < w; ++i)
                                P[rho * w + i] = P[rho * w + i] + P[(rho + c * nj) * w + i];
                    rows = nj;
                }
                qo_point_values(sp, r, j, v);
#pragma omp parallel for schedule(static)
                for (int i = 0; i < w; ++i) {
                    double acc = 0.0;
                    for (int64_t rho = 0; rho < nj; ++rho) acc = acc + v[rho] * P[rho * w + i];
                    dAr[(size_t)j * t + i0 + i] = acc;
                }
            }
        }
    }
    free(P); free(u); free(hv); free(v); free(S);
    return 0;
}

/* Y = X A for one shift by Algorithm 1 over all columns (column blocks of 64). */
int qo_reduced_matvec(const qo_spec *sp, int r, const double *A, int t, double *Y, int64_t *nmadd) {
    int64_t N = N_of(sp);
    int tb = block_width(t);
    double *P = (double *)malloc(sizeof(double) * (size_t)N * tb);
    if (!P) return 1;
    for (int i0 = 0; i0 < t; i0 += tb) {
        int i1 = i0 + tb < t ? i0 + tb : t, w = i1 - i0;
        if (reduced_product(sp, r, A, t, i0, i1, P, nmadd)) { free(P); return 1; }
        for (int64_t k = 0; k < N; ++k) memcpy(Y + k * t + i0, P + k * w, sizeof(double) * w);
    }
    free(P);
    return 0;
}

int qo_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
