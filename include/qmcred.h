/*
 * qmcred.h -- reduced QMC matrix-vector products on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for the N = b^m points x_0..x_{N-1} of a reduced
 * rank-1 lattice, reduced polynomial lattice or reduced digital net (Dick,
 * Ebert, Herrmann, Kritzer, Longo, "The fast reduced QMC matrix-vector
 * product"), the products x_k^T A (eq. QMC_matrix: the N x t matrix X A) and
 * the QMC rule of eq. QMC-rule,
 *
 *     Q_N(f) = N^-1 sum_k f(x_k^T A),   f(y) = h( t^-1 sum_i g(y_i) ),
 *
 * together with its gradient dQ/dA.  Coordinate j of a reduced point set has
 * reduction index w_j (non-decreasing, w_0 = 0) and takes only
 * n_j = b^{m - min(w_j, m)} distinct values, repeated periodically in k
 * (Section 2.1, the repetition xi_j = (X_j, ..., X_j)); the library builds the
 * product from those distinct values (the grouped form of Algorithm 2) and
 * never materialises the N x t product unless asked to.
 *
 * Conventions for every call:
 *   - Indices are 0-based: coordinate j = 0..s-1 is the paper's j+1.
 *   - b is a prime, 1 <= m <= 24 and N = b^m <= 2^24 (QMC_EUNSUPPORTED
 *     otherwise).  Every kind is supported in every prime base; a net over
 *     F_b, b > 2, that is not periodic after reduction needs N s <= 2^29.
 *   - Matrices are row-major FP32 with an explicit leading dimension.
 *   - "device" pointers are HIP device memory on the device that was current
 *     when the point set was created; "host" pointers are ordinary memory.
 *   - stream is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Every compute call is asynchronous on that stream; results
 *     are valid once the stream has reached that point.
 *   - Every call returns a qmc_status.  Arguments are validated on the host
 *     before anything is launched: on an error status nothing is written and
 *     the point set is unchanged.  qmc_last_error() then returns a
 *     thread-local message with the detail.
 *   - A point set is immutable after qmc_points_init, so calls on different
 *     streams may use it concurrently as long as each has its own workspace.
 */
#ifndef QMCRED_H
#define QMCRED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    QMC_OK = 0,
    QMC_EINVAL = 1,        /* an argument violates a requirement stated below        */
    QMC_EUNSUPPORTED = 2,  /* valid in the paper, not handled by this library         */
    QMC_ENOMEM = 3,        /* device or host allocation failed, or workspace too small */
    QMC_EDEVICE = 4        /* a HIP runtime call or kernel launch failed               */
} qmc_status;

/* Point-set families (Section 1.1, Section 3, Section 4). */
typedef enum {
    QMC_LATTICE = 0,       /* reduced rank-1 lattice, Section 1.3                     */
    QMC_POLY_LATTICE = 1,  /* reduced polynomial lattice, g_j = x^{w_j} g'_j          */
    QMC_DIGITAL_NET = 2,   /* reduced digital net, eq. reduced_genmat_net2           */
    QMC_IID = 3            /* reduced Monte Carlo, Section 4 eq. randpts: coordinate j
                              has n_j i.i.d. samples (caller-drawn), point k uses
                              sample k mod n_j                                      */
} qmc_kind;

/* Randomisation (Section 1.2 random shift; base-2 digital shift). */
typedef enum {
    QMC_NO_SHIFT = 0,
    QMC_RANDOM_SHIFT = 1,  /* x <- {x + Delta_j}: one FP64 add, then minus 1 if >= 1  */
    QMC_DIGITAL_SHIFT = 2  /* first 52 digits XOR delta_j, tail set to its midpoint:
                              x = (2U + 1) 2^-53, U = (c << (52 - n)) ^ delta_j       */
} qmc_rand;

/* Component maps applied to the distinct values (Section 2.3; tent map of Section 1.2). */
typedef enum {
    QMC_MAP_ID = 0,
    QMC_MAP_CENTER = 1,    /* x - 1/2                                                 */
    QMC_MAP_INVNORM = 2,   /* Phi^-1(x), inverse standard normal CDF (needs a shift)  */
    QMC_MAP_TENT = 3       /* 1 - |1 - 2x|                                            */
} qmc_map;

/* Arithmetic of the grouped products on the matrix cores. */
typedef enum {
    QMC_FP32 = 0,          /* FP32 MFMA, FP32 accumulation                            */
    QMC_SPLIT_BF16X3 = 1   /* x = x_hi + x_lo in bf16; hi*hi + hi*lo + lo*hi on BF16
                              MFMA, FP32 accumulation (upper levels only)             */
} qmc_prec;

typedef enum { QMC_G_ID = 0, QMC_G_COS = 1, QMC_G_EXP = 2 /* exp(c*y) */ } qmc_g;
typedef enum { QMC_H_ID = 0, QMC_H_CALL = 1 /* max(0, u - K) */ } qmc_h;

/*
 * A reduced point set with N = b^m points in s dimensions.  All arrays are
 * host memory and are copied by qmc_points_init.
 *   w      [s]    reduction indices, w[0] = 0, non-decreasing, w[j] >= 0
 *                 (Section 1.3).  Coordinates with w[j] >= m take one value.
 *   gen    lattice: [s] z'_j below b^{m-w_j} and not divisible by b (odd for
 *                 b = 2), or z'_j = 1 when w_j >= m (the set U_{b^{m-w}} of
 *                 Section 1.3); the generating vector is z_j = b^{w_j} z'_j.
 *          In a base b > 2, polynomials and matrix columns below are given by
 *          their base-b digits instead of bits: g'_j as the integer g'_j(b)
 *          (digit i = coefficient of x^i, nonzero constant term, degree
 *          < m - w_j), and column word [j*m + q-1] = sum_p C_{p,q} b^{p-1}.
 *          poly lattice: [s] bit masks of g'_j in F_2[x] (bit i = coefficient
 *                 of x^i), g'_j(0) = 1, deg g'_j < m - w_j (g'_j = 1 when
 *                 w_j >= m); the generating polynomial is x^{w_j} g'_j.
 *          digital net: [s*m] column words of the m x m generating matrices
 *                 C^{(j)} of eq. def:digital: word [j*m + q-1] has bit p-1 set
 *                 iff C^{(j)}_{p,q} = 1 (row p = output digit with weight 2^-p,
 *                 column q = input digit of weight 2^{q-1}).  The library
 *                 applies the reduction of eq. reduced_genmat_net2 itself.
 *                 When the reduced matrix has zero columns q > m - min(w_j,m)
 *                 (true for lower-triangular C^{(j)}) the points repeat with
 *                 period n_j and the cascade of Algorithm 2 applies;
 *                 otherwise (Sobol'-type, upper-triangular C^{(j)}) every
 *                 product uses Algorithm 4 (Section 3).
 *          reduced Monte Carlo (QMC_IID): ignored (may be NULL).
 *   rand, R, shift [R*s] in [0,1) (QMC_RANDOM_SHIFT) or dshift [R*s] < b^K
 *                 (QMC_DIGITAL_SHIFT; K the largest with b^K <= 2^52, so 2^52
 *                 for b = 2): the K base-b digits of dshift (most significant
 *                 first) are added digit by digit mod b (XOR for b = 2) to
 *                 the point's first K digits and the rest is replaced by its
 *                 midpoint, x = (U + 1/2) / b^K.  R independent randomisations, all
 *                 evaluated by one call.  With QMC_NO_SHIFT, R must be 1,
 *                 except for QMC_IID, where rand must be QMC_NO_SHIFT and R
 *                 counts independent replicates.
 *   map           component map; QMC_MAP_INVNORM requires a shift because the
 *                 unshifted point x_0 = 0 (Section 2.3), or QMC_IID samples.
 *   samples       QMC_IID only: [R][sum_j n_j] uniforms in [0,1) (in (0,1)
 *                 with QMC_MAP_INVNORM), n_j = b^{m - min(w_j, m)}; replicate
 *                 r holds coordinate 0's n_0 samples, then coordinate 1's, ...
 *                 Copied to the device by qmc_points_init.
 */
typedef struct {
    int32_t b, m, s;
    int32_t kind;             /* qmc_kind */
    const int32_t *w;
    const uint64_t *gen;
    int32_t rand;             /* qmc_rand */
    int32_t R;
    const double *shift;
    const uint64_t *dshift;
    int32_t map;              /* qmc_map */
    const double *samples;    /* QMC_IID: i.i.d. uniforms, see above */
} qmc_point_spec;

/* f(y) = h(t^-1 sum_i g(y_i)), y = x^T A in R^t.  h is applied per point. */
typedef struct {
    int32_t g;                /* qmc_g; QMC_G_EXP is exp(c * y) */
    double c;
    int32_t h;                /* qmc_h; QMC_H_CALL is max(0, u - K), h'(K) := 0 */
    double K;
} qmc_integrand;

typedef struct qmc_points_s *qmc_points;

/*
 * Create a point set on the current HIP device (Section 1.3, Section 3,
 * Algorithm 3, Section 4).  Validates spec (EINVAL: b not prime, w[0] != 0, w
 * decreasing, a generator outside its allowed set, shift outside [0,1) or
 * >= 2^52, R < 1, INVNORM without a shift, QMC_IID with a shift, without
 * samples or with a sample outside [0,1) ((0,1) under INVNORM);
 * EUNSUPPORTED: m outside [1, 24], b^m > 2^24, a net over F_b, b > 2, that is
 * not periodic after reduction with N s > 2^29), plans the levels and uploads
 * generators, shifts and samples.  A net that is not periodic after
 * reduction (any prime b) takes Algorithm 4: its values are tabulated by the
 * integer of their reduced output digits; over F_b, b > 2, the index of every
 * point and coordinate is tabulated once here (N s words).  A base b > 2 is evaluated like Algorithm 4: the n_j
 * values of every coordinate (c / b^e, one correctly rounded FP64 division
 * before shift and map; Section 4 for samples) are tabulated, and point k
 * reads value k mod n_j.
 * Synchronous.  *out owns device memory; release with qmc_points_free.
 */
qmc_status qmc_points_init(qmc_points *out, const qmc_point_spec *spec);

/* Release a point set.  NULL is accepted.  The caller ensures no call is in flight. */
qmc_status qmc_points_free(qmc_points p);

/* Host-side facts about a point set: N = b^m, s, R, the split level used by
 * the fused kernels (-1 for a net that is not periodic after reduction, whose
 * products use Algorithm 4, and for a base b > 2) and the number of distinct
 * values sum_j n_j per shift. */
qmc_status qmc_points_info(qmc_points p, int64_t *N, int32_t *s, int32_t *R, int32_t *split_level,
                           int64_t *distinct_values);

/* The split level L' of the gradient (qmc_estimate_grad; Section 3's
 * transposed cascade): the estimate's, capped at 5.  Levels at and above it
 * go to the matrix-core products, the lower ones to the fused leaf pass, whose
 * gradient form holds a subtree's leaves and one accumulator per lower
 * coordinate in registers: with 32 leaves per subtree it keeps four waves per
 * SIMD.  -1 as for qmc_points_info.  EINVAL: p or split_level null. */
qmc_status qmc_points_grad_split(qmc_points p, int32_t *split_level);

/*
 * Distinct values X_j[rho], rho < n_j, of coordinate j for randomisation r, in
 * FP64 after shift and map (Section 2.1 X_j; Section 2.3 maps).  out: device,
 * n_j doubles.  Integer-exact up to the shift and map; the same FP64
 * operation sequence as the documented randomisations.  For a net that is not
 * periodic after reduction, rho is the integer of the reduced output digits
 * (the value is rho / n_j before shift and map; Algorithm 4's index).
 */
qmc_status qmc_point_values(qmc_points p, int32_t r, int32_t j, double *out, void *stream);

/*
 * The full N x s point matrix X of eq. QMC_matrix for randomisation r, FP32,
 * row-major with leading dimension ldx >= s (device).  For the dense baseline
 * and for tests; the reduced calls below never build it.
 */
qmc_status qmc_point_matrix(qmc_points p, int32_t r, float *X, int64_t ldx, void *stream);

/*
 * Workspace bytes needed by the call `op` (0 = qmc_reduced_matvec,
 * 1 = qmc_estimate, 2 = qmc_estimate_grad) for t columns and this integrand
 * (f may be NULL for op 0).  A caller that passes its own workspace must pass
 * at least this many bytes, 256-byte aligned.
 */
qmc_status qmc_workspace_size(qmc_points p, int32_t op, int32_t t, const qmc_integrand *f,
                              int32_t prec, size_t *bytes);

/*
 * Y = X A for randomisation r (Algorithm 1 / Algorithm 2 result), written to
 * Y (device, N x t FP32, leading dimension ldy >= t).  A: device, s x t FP32,
 * lda >= t.  workspace: device memory of qmc_workspace_size(op=0) bytes, or
 * NULL to let the library allocate it stream-ordered for this call.
 */
qmc_status qmc_reduced_matvec(qmc_points p, int32_t r, const float *A, int32_t t, int64_t lda,
                              int32_t prec, float *Y, int64_t ldy, void *workspace,
                              size_t workspace_bytes, void *stream);

/*
 * Q[r] = N^-1 sum_k f(x_k^T A) for every randomisation r < R (eq. QMC-rule),
 * with the product built from the distinct values and fused with f and the
 * mean: Y is never written to memory.  The mean is accumulated in FP64 in a
 * fixed order (bitwise reproducible).  A: device s x t FP32, lda >= t.
 * Q: device, R doubles.  workspace as above (op = 1).
 */
qmc_status qmc_estimate(qmc_points p, const float *A, int32_t t, int64_t lda, const qmc_integrand *f,
                        int32_t prec, double *Q, void *workspace, size_t workspace_bytes, void *stream);

/*
 * qmc_estimate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same computation and the same kernels, with the workspace taken from a
 * static device array of 64 MiB that the library holds on every device it
 * runs on until the process ends.  Makes no allocation of any kind.
 * Returns QMC_ENOMEM, before anything is launched, when the call needs more
 * than 64 MiB of workspace (qmc_workspace_size with op = 1 tells).  Every call
 * on one device shares that device's array: calls that overlap in time on one
 * device (other streams, other threads) race and must be serialised by the
 * caller.  The results equal those of qmc_estimate bit for bit.
 */
qmc_status qmc_estimate_static(qmc_points p, const float *A, int32_t t, int64_t lda,
                               const qmc_integrand *f, int32_t prec, double *Q, void *stream);

/*
 * Q as qmc_estimate, and dA[r] = dQ_r/dA = N^-1 sum_k x_k (x) grad f(x_k^T A)
 * for every r: the transpose of the reduced product (sums of the point-wise
 * sensitivities over the residue classes k mod n_j, then the distinct values),
 * with Y recomputed rather than stored.  dA: device, R x s x t FP32, rows of
 * length t (leading dimension t).  workspace as above (op = 2).
 * A net that is not periodic after reduction (Algorithm 4) and every base
 * b > 2 take the transpose of the gathered products instead: the point-wise
 * sensitivities G (R x N x t FP32, part of the workspace) are formed, then
 * dA = X^T G on the matrix cores (in base b > 2 the coordinates with
 * n_j <= b^{m-L'} contract over G summed into the b^{m-L'} residues), the
 * chunk partials added in FP64 in fixed order.
 */
qmc_status qmc_estimate_grad(qmc_points p, const float *A, int32_t t, int64_t lda,
                             const qmc_integrand *f, int32_t prec, double *Q, float *dA,
                             void *workspace, size_t workspace_bytes, void *stream);

/* Static text for a status code. */
const char *qmc_status_string(qmc_status s);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *qmc_last_error(void);

/*
 * Per-kernel timing for measurement tools.  When enabled, every kernel launch
 * of this library is bracketed by HIP events on its stream; qmc_timing_read
 * returns, for the kernel family `name` ("tables", "levels", "leaf", "reduce",
 * "fold", "levels_adj", "combine", "points"), the summed event time in
 * milliseconds and the number of launches since the last reset.  Reading
 * synchronises the recorded events.  Not for production use: it adds event
 * records to the stream.
 */
qmc_status qmc_timing_enable(int32_t on);
/*
 * Measured issue rates of the vector ALU on the current device, for the
 * roofline of the ALU-bound kernels: lane operations per second of FP32
 * v_fma_f32 (the unpacked form, the only FP32 form this library emits), of
 * v_exp_f32 (each followed by one v_mul_f32) and of v_sin_f32.  Runs short
 * timed kernels on `stream` (allocates and frees a small buffer; synchronous).
 * Not for production use.
 */
qmc_status qmc_probe_valu(double *fma_per_s, double *exp_per_s, double *sin_per_s, void *stream);
/*
 * Measured matrix-core rates of the current device in flop/s, for the roofline
 * of the grouped products: v_mfma_f32_32x32x2_f32 and v_mfma_f32_16x16x4_f32
 * (FP32) and v_mfma_f32_32x32x16_bf16, four independent accumulators per wave.
 * Same conditions as qmc_probe_valu.
 */
qmc_status qmc_probe_mfma(double *f32_32x32x2, double *f32_16x16x4, double *bf16_32x32x16, void *stream);
qmc_status qmc_timing_reset(void);
qmc_status qmc_timing_read(const char *name, double *ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* QMCRED_H */
