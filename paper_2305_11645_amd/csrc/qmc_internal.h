// Internal definitions shared by the HIP sources of libqmcred (not installed).
//
// Level structure.  With w non-decreasing, the coordinates with
// min(w_j, m) = I form one contiguous block G_I = [j0, j0 + tau) of rows of A
// (the groups of Algorithm 2).  Level I has n_I = 2^{m-I} distinct values per
// coordinate.  The planner picks a split level L' (at most 6):
//   * upper levels I >= L' are evaluated as small dense products
//     U_I = X~_I A_I (n_I x t) on the matrix cores, one grouped launch;
//   * lower levels I < L' are evaluated inside the fused leaf kernel: a point
//     k = rho + c n_{L'} (rho < n_{L'}, c < 2^{L'}) is a leaf of the subtree
//     rooted at residue rho, and the partial sums of the cascade
//     P_I = tile(P_{I+1}) + X~_I A_I (Algorithm 2) are formed node by node.
//
// Point tables per randomisation r (FP32, sum_j n_j values in total):
//   lower part  one record of S_rec floats per subtree root rho < n_{L'}:
//               for I = L'-1 down to 0, for j in G_I, for c < 2^{L'-I}:
//               value_j(rho + c n_{L'}).  A wave reads a record with scalar
//               loads: every lane (column) needs the same values.
//   upper part  for I >= L': X~_I row-major n_I x tau_I (K-contiguous).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "qmcred.h"

namespace qmc {

constexpr int kMaxM = 24;
constexpr int64_t kMaxPoints = int64_t(1) << 24;  // N = b^m
constexpr int kMaxLevels = kMaxM + 1;
constexpr int kMaxSplit = 6;       // at most 64 leaves per subtree
// The gradient's split level is at most 5: its fused leaf pass keeps one
// accumulator per lower coordinate and the subtree's leaves in registers, and
// a 64-leaf subtree needs more than a quarter of a SIMD's registers (three
// waves per SIMD instead of four; measured slower than moving level 5 onto
// the matrix cores).
constexpr int kMaxSplitGrad = 5;
constexpr int kTileT = 64;         // columns per wave in the leaf kernels
constexpr int kMaxLowRows = 64;    // rows of A kept in LDS by the leaf kernels
constexpr int kLdsPadRows = 8;   // zero rows after the leaf kernel's rows of A in LDS
constexpr int kTablePad = 64;    // floats after the point tables (the leaf's batched loads over-read)

struct Level {
  int32_t tau;     // coordinates in the level
  int32_t j0;      // first coordinate
  int32_t nb;      // n_I = 1 << nb
  int32_t pad;
  int64_t off;     // lower level: offset inside a subtree record; upper: offset in the table
  int64_t uoff;    // upper level: first row of U_I inside the per-shift U buffer
};

// Everything a kernel needs to know about the point set (passed by value).
struct Geometry {
  int32_t m, s, kind, rand, map, R;
  int32_t b;             // prime base: N = b^m, n_j = b^{m - min(w_j, m)}
  int32_t nonperiodic;   // a reduced net that is not periodic: products by Algorithm 4 (any prime b)
  int32_t gather;        // products by gathered value tiles on the matrix cores: nets that
                         // are not periodic (index by XOR) and every base b > 2 (index by add)
  int64_t gather_total;  // floats per randomisation in the value tables of the gather path
  int32_t split;         // L'
  int32_t jlow;          // rows 0..jlow-1 of A belong to the lower levels
  int32_t nup;           // number of upper levels with tau > 0
  int32_t up[kMaxLevels];  // their indices I, increasing
  int64_t N;
  int64_t rec;           // floats per subtree record
  int64_t nsub;          // n_{L'}: subtree roots
  int64_t lower_total;   // nsub * rec
  int64_t table_total;   // floats per shift = sum_j n_j
  int64_t urows;         // rows of the U buffer per shift = sum over upper levels of n_I
  Level lev[kMaxLevels];
};

// Device-side copy of the generators and shifts.
struct DevSpec {
  const uint32_t *gen;     // lattice/poly: [s]; net: [s*m] column words
  const int32_t *nbj;      // [s] m - min(w_j, m)
  const double *shift;     // [R*s]
  const uint64_t *dshift;  // [R*s]
  const double *samples;   // reduced Monte Carlo: [R][sample_total]
  const int64_t *soff;     // [s] start of coordinate j's samples in a replicate
  int64_t sample_total;    // sum_j n_j
  // Gather path: aoff[j] = start of coordinate j's value table; point n0 + r of
  // tile h (n0 = 64 h, r < 64) reads the value at ytile[h * s + j] op
  // ylo[j * 64 + r].
  //   nets that are not periodic (op XOR): the words are the digit words y_j
  //   restricted to the first n_j digits, ylo = y_j(r), ytile = aoff[j] XOR
  //   y_j(64 h), and aoff[j] is a multiple of n_j;
  //   base b > 2 (op +): the table holds the n_j values twice (2 n_j floats),
  //   ylo = r mod n_j, ytile = aoff[j] + (64 h mod n_j).
  const uint32_t *aoff;
  const uint32_t *ylo;
  const uint32_t *ytile;
};

// The integrand's g on the scaled argument y' = sigma y (sigma folded into the
// staged rows of A).  // cos and sin take the angle in revolutions on v_cos / v_sin; v_fract reduces
// it exactly.  exp(c y) = 2^(y'), y' = c log2(e) y, on v_exp.
template <int GF>
__device__ __forceinline__ float g_val(float ys) {
  if (GF == QMC_G_COS) return __builtin_amdgcn_cosf(__builtin_amdgcn_fractf(ys));
  if (GF == QMC_G_EXP) return __builtin_amdgcn_exp2f(ys);
  return ys;
}

// Same, for an argument known to lie inside v_cos's input domain (+-256 revolutions).
template <int GF>
__device__ __forceinline__ float g_val_near(float ys) {
  if (GF == QMC_G_COS) return __builtin_amdgcn_cosf(ys);
  return g_val<GF>(ys);
}

// g'(y) from the scaled argument y'; c is the parameter of exp(c y)
template <int GF>
__device__ __forceinline__ float g_der(float ys, float c) {
  if (GF == QMC_G_COS) return -__builtin_amdgcn_sinf(__builtin_amdgcn_fractf(ys));
  if (GF == QMC_G_EXP) return c * __builtin_amdgcn_exp2f(ys);
  return 1.0f;
}

// The per-point part of g'(y) from the scaled argument y': sin (cos: g' is
// -sin), 2^{y'} (exp(c y): g' is c exp(c y)) or 1; the constant factor
// g_der_factor (-1, c or 1) multiplies the summed adjoint instead.  NEAR: the
// argument is known to lie inside v_sin's input domain (+-256 revolutions).
template <int GF, bool NEAR>
__device__ __forceinline__ float g_der_unit(float ys) {
  if (GF == QMC_G_COS) return __builtin_amdgcn_sinf(NEAR ? ys : __builtin_amdgcn_fractf(ys));
  if (GF == QMC_G_EXP) return __builtin_amdgcn_exp2f(ys);
  return 1.0f;
}
inline double g_der_factor(const qmc_integrand &f) {
  return f.g == QMC_G_COS ? -1.0 : f.g == QMC_G_EXP ? f.c : 1.0;
}

// Per-call timing hook (no-op unless enabled).
struct LaunchTimer {
  const char *name;
  hipStream_t st;
  void *ev0 = nullptr;
  LaunchTimer(const char *n, hipStream_t s);
  ~LaunchTimer();
};

// Records the detail returned by qmc_last_error() and passes the status through.
qmc_status record_error(qmc_status s, const char *fmt, ...);

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.

// Point tables (FP32) for shifts [r0, r0 + nr): out[(r - r0) * table_total + e].
// Also zeroes counters[0..ncounters) (may be null) for the kernels that follow.
hipError_t launch_tables(const Geometry &G, const DevSpec &D, int r0, int nr, float *out,
                         uint32_t *counters, int ncounters, hipStream_t st);
// Distinct FP64 values of coordinate j for shift r.
hipError_t launch_point_values(const Geometry &G, const DevSpec &D, int r, int j, double *out,
                               hipStream_t st);
// Dense FP32 point matrix for shift r.
// Value tables of the gather path, coordinate j's block at DevSpec::aoff[j],
// Geometry::gather_total floats per randomisation.  Nets that are not periodic
// (Algorithm 4): digit order, T_j[y] = X_j[c] for y < n_j, c the integer of the
// reduced output digits and y its n_j-digit bit reversal (the digits as the
// generating matrix produces them).  Base b > 2: T_j[i] = X_j[i mod n_j] for
// i < 2 n_j, X_j[rho] the value at residue rho.
hipError_t launch_output_tables(const Geometry &G, const DevSpec &D, int r0, int nr, float *out,
                                hipStream_t st);
hipError_t launch_point_matrix(const Geometry &G, const DevSpec &D, int r, float *X, int64_t ldx,
                               hipStream_t st);

// Grouped upper-level products U_I = oscale X~_I A_I for shifts [0, nr) of the table buffer.
// pack (levels_pack_bytes(G, nr, t) bytes, 16-byte aligned) receives the
// operands packed into K-step slabs (split BF16: split into hi and lo) once,
// then multiplied; ldu is a multiple of 4.
hipError_t launch_levels(const Geometry &G, int prec, const float *tables, int nr, const float *A,
                         int t, int64_t lda, float *U, int64_t ldu, float oscale, void *pack, hipStream_t st);
int64_t levels_pack_bytes(const Geometry &G, int nr, int t);

// Adjoint of the upper levels: dA_I = X~_I^T S_I; S pyramid rows as in fold.
hipError_t launch_levels_adj(const Geometry &G, int prec, const float *tables, int nr,
                             const float *S, int t, int64_t ldu, float *part, hipStream_t st);
int64_t levels_adj_part_floats(const Geometry &G, int t, int64_t ldu);
// K-chunk (rows of S per partial) of the adjoint level products
int64_t levels_adj_kchunk(int64_t K);

// Fold of the subtree-root sums over the upper levels (S_{I+1} from S_I).
hipError_t launch_fold(const Geometry &G, int nr, float *S, int t, int64_t ldu, hipStream_t st);

enum LeafMode { kModeSum = 0, kModePoint = 1, kModeStoreY = 2, kModeGrad = 3 };

// Compact per-launch description of the lower levels for the leaf kernel.
struct LeafLevel {
  int32_t tau, off, j0, pad;   // coordinates, record offset (floats), first coordinate
};

constexpr int kMaxUpPadded = (kMaxLevels + 7) / 8 * 8;

struct LeafArgs {
  int32_t t, tct, nsub, rec, gx, gy, nw, jlow, r0, nup, nparts;
  int32_t sub_per, sub_rem;     // subtrees per workgroup: nsub = sub_per gx + sub_rem
  float xmax;                   // bound on |x| of every point value
  // offset (floats) of the first U row and n_I - 1 of each upper level (per
  // shift); the entries past nup are zero, and the arrays are padded to whole
  // batches of the root loads
  int64_t up_off[kMaxUpPadded];
  int32_t up_mask[kMaxUpPadded];
  LeafLevel lv[kMaxSplit];
  uint64_t taus;                // tau_I of the lower levels, one byte per level (level I at bit 8 I)
  int64_t tstride, ustride, lda, ldu, ldy;
  uint32_t ldu32;               // ldu (< 2^32)
  float sigma;                  // y' = sigma y: 1/(2 pi) for cos, c log2(e) for exp
};

// sigma for an integrand and leaf mode
float g_scale(const qmc_integrand &f, int mode);

struct LeafOut {
  double *partial;     // kModeSum / kModeGrad: [nr][gx][gy] FP64 sums of g, one per workgroup
  float *ppart;        // kModePoint: [nr][tct][N] per-point sums over a column tile
  float *Y;            // kModeStoreY
  int64_t ldy;
  // kModeGrad works with the unscaled sensitivities G'_ki = h'(u_k) g'_unit(y_ki)
  // (g_der_unit); the factor g_der_factor / (N t) is applied by launch_combine.
  float *dApart;       // kModeGrad: [nr][gx][tct][jlow][64] lower-level dA partials
  float *Sroot;        // kModeGrad: [nr][2 nsub][ldu] subtree-root sums of G' (pyramid base)
  const float *hd;     // kModeGrad, non-separable h: [nr][N] per-point factor h'(u)
};

struct LeafPlan {
  int gx;              // workgroups along the subtree axis
  int gy;              // workgroups along the column axis (64 cpl columns each)
  int spw;             // subtrees per wave (before the one-round choice)
  int nw;              // waves per workgroup
  int cpl;             // columns of A per lane (the workgroup's tile is 64 cpl columns)
};
LeafPlan leaf_plan(const Geometry &G, int t, int nr, int mode, int gf);
// Workgroups of kernel fn that fit on the current device at once (occupancy x
// compute units), cached; 0 when the query fails.
int64_t resident_workgroups(const void *fn, int threads, size_t lds);

// The register form of the gradient mode (adjoint.hip): whether it applies
// (every lower level I holds at most 2^I coordinates) and its kernel for an
// integrand g and a per-point factor h' (hd).  It takes the LeafArgs of
// launch_leaf and (tables, U, A, partial, dApart, Sroot, hd).
bool grad_reg_ok(const Geometry &G);
const void *grad_fn(const Geometry &G, int gf, bool hd);

hipError_t launch_leaf(const Geometry &G, int mode, const qmc_integrand &f, const float *tables,
                       const float *U, int nr, int r0, const float *A, int t, int64_t lda,
                       int64_t ldu, const LeafPlan &lp, const LeafOut &o, hipStream_t st);

// Gather path (Algorithm 4 nets, base b > 2): one 64-point x 256-column tile per
// workgroup (alg4_col_tiles(t) column tiles); modes kModeStoreY, kModeSum
// (partial[r][point tile][column tile]) and kModePoint (ppart[r][column tile][N]).
// tab: the digit-order value tables of launch_output_tables for the nr
// randomisations.
struct Alg4Out {
  float *Y;         // StoreY: Y; Grad: the sensitivities G (same layout)
  int64_t ldy;
  int64_t ystride;  // StoreY, Grad: floats between the randomisations' outputs
  double *partial;
  float *ppart;
  const float *hd;  // Grad: per-point factor h'(u) ([randomisation][N]) or null
  double gscale;    // Grad: factor of g' (1/(N t))
};
// One pass of the gather path: coordinates [j0, j0 + sc) over points n < npts,
// optionally adding root[r][n mod nsplit][col] (leading dimension ldp, stride
// root_stride per randomisation, nsplit >= 64) to every y before the epilogue.
// Base b > 2 splits the product in two passes (the grouped cascade of
// Algorithm 2 at one level): the upper coordinates (n_j <= nsplit) over the
// nsplit residues into the root table, then the lower ones over all N points.
struct Alg4Pass {
  int32_t j0, sc;
  int64_t npts;
  const float *root;
  int64_t ldp, root_stride, nsplit;
  const char *timer;  // launch-timer name
};
Alg4Pass alg4_whole(const Geometry &G);  // one pass over every coordinate and point
int64_t alg4_point_tiles(const Geometry &G);
int64_t alg4_index_words(const Geometry &G);  // (64 + tiles) * s
int alg4_col_tiles(int t);
constexpr int64_t kAlg4MaxLda = int64_t(1) << 24;     // leading dimension of A
constexpr int64_t kAlg4MaxValues = int64_t(1) << 30;  // value-table floats: below 2^30 (4-byte offsets < 2^32)
constexpr int64_t kMaxIndexWords = int64_t(1) << 29;  // per-point index words (nets over F_b not periodic): 2 GiB
// Adjoint of the gather path, dA = X^T G (Algorithm 4 transposed).
// alg4_adj_chunks: point chunks of a pass over sc coordinates and npts points
// (its partials hold nr x chunks x sc x t FP64 values).  launch_alg4_adj:
// coordinates [j0, j0 + sc) over the first npts rows of G ([randomisation][npts
// rows of t], gstride floats apart) into part[r][chunk][j - j0][i].
// launch_alg4_fold: S[r][rho] = sum of G[r][n] over n = rho mod nsplit
// (Geometry::nsub).  launch_alg4_adj_combine: dA[r][j][i] = FP64 sum of the
// chunks' partials, rows j < jlow from the lower pass's, the others from the
// upper pass's.
// The partials are FP64: within a chunk the matrix cores sum in FP32 over at
// most kAdjFlushPoints points at a time, then add into the chunk's partial.
constexpr int kAdjFlushPoints = 4096;
int alg4_adj_chunks(int sc, int64_t npts, int t, int nr);
hipError_t launch_alg4_adj(const Geometry &G, const DevSpec &D, int prec, const float *tab, int nr,
                           const float *Gm, int64_t gstride, int j0, int sc, int64_t npts, int nchunk, int t,
                           double *part, hipStream_t st);
hipError_t launch_alg4_fold(const Geometry &G, const float *Gm, int nr, int t, float *S, hipStream_t st);
hipError_t launch_alg4_adj_combine(const Geometry &G, const double *plo, int nlo, const double *pup, int nup, int nr,
                                   int t, float *dA, hipStream_t st);
hipError_t launch_alg4_index(const Geometry &G, const uint32_t *gen, const int32_t *nbj, const uint32_t *aoff,
                             uint32_t *ylo, uint32_t *ytile, hipStream_t st);
hipError_t launch_alg4(const Geometry &G, const DevSpec &D, int mode, const qmc_integrand &f,
                       int prec, const float *tab, int nr, const float *A, int t, int64_t lda,
                       const Alg4Pass &ps, const Alg4Out &o, hipStream_t st);

// Q[r] = scale * sum of partial[r][*] (fixed order, compensated).
hipError_t launch_reduce(const double *partial, int nr, int64_t per, double scale, double *Q,
                         hipStream_t st);
// Per-point h: partial[r][blk] = sum over points of h(t^-1 sum_ct ppart), and
// optionally hd[r][k] = h'(u_k) * hscale.
hipError_t launch_point_h(const Geometry &G, const qmc_integrand &f, const float *ppart, int nr,
                          int tct, int t, double *partial, int64_t blocks, float *hd,
                          double hscale, hipStream_t st);
int64_t point_h_blocks(const Geometry &G);

// dA[r][j][i] = scale x (sum of the lower partials (rows j < jlow) or of the
// upper partials (rows of the upper levels)), FP64 accumulation, FP32 result.
hipError_t launch_combine(const Geometry &G, const float *dApart_low, int gx, int tct,
                          const float *dApart_up, int nr, int t, int64_t ldu, double scale, float *dA,
                          hipStream_t st);

}  // namespace qmc
