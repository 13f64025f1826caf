// Fused leaf pass: the lower levels of the cascade, the integrand and the sum.
//
// Point k = rho + c n_{L'} (rho < n_{L'} subtree root, c < 2^{L'} leaf) has
//     y_k = P_{L'}[rho] + sum_{I < L'} U_I[k mod n_I],
// where P_{L'}[rho] = sum_{I >= L'} U_I[rho mod n_I] comes from the grouped
// upper-level products, and the lower levels follow the recursion of
// Algorithm 2 inside the subtree: the node c (< 2^{L'-I}) of level I is the
// residue rho + c n_{L'} mod n_I, and its value is the value of its parent
// c mod 2^{L'-I-1} plus X~_I[node] A_I.  Each level's distinct values are thus
// combined once per node, not once per point.
//
// Work layout: a wave owns 64 consecutive columns of A (one per lane) and one
// subtree at a time.  The point values of a subtree are the same for all lanes
// and are read with scalar loads from the subtree's record; the rows of A of
// the lower levels sit in LDS, pre-multiplied by the scale sigma of g (so the
// kernel forms y' = sigma y directly: 1/(2 pi) for cos, c log2 e for exp).
// The 2^{L'-I} partial sums of a level live in registers; when level 0 holds a
// single coordinate its leaves are consumed as they are formed, so only the
// level-1 values stay live.  Y is never written (except in the matvec mode).
//
// Modes:
//   Sum    sum_k sum_i g(y_ki): FP32 inside a subtree, FP64 across subtrees;
//          one FP64 partial per workgroup (reduced in a fixed order afterwards)
//   Point  per-point sums over the wave's 64 columns (for non-separable h)
//   StoreY write y_ki (the matrix-vector product)
//   Grad   G_ki = s_k g'(y_ki); sums of G up the subtree give S_I for the
//          lower levels (the transpose of the recursion), dA_I += X~_I^T S_I
//          per wave in LDS, the subtree-root sums S_{L'} go to memory.
#include <algorithm>
#include <cstdlib>

#include "qmc_internal.h"

namespace qmc {

constexpr int kRootBatch = 8;  // upper-level rows of a subtree root loaded together (summing mode)
static_assert(kMaxUpPadded % kRootBatch == 0, "root batches must tile the padded level arrays");

// cos and sin take the angle in revolutions on v_cos / v_sin; v_fract reduces
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

// Summing mode, lean form.  Only the per-level counts tau_I travel with the
// kernel (one byte per level); the record offset and the first row of A of a
// level follow from the counts while descending, so few scalar registers stay
// live.  The point values of up to kBatchFloats nodes x coordinates and their
// rows of A are requested together, then consumed: one memory round trip per
// batch instead of one per coordinate.  The scalar loads may read up to 31
// floats past a level's block (the point tables carry padding at their end);
// the LDS reads of A up to 7 rows past a level's rows (kLdsPadRows zero rows
// follow the staged rows).
constexpr int kBatchFloats = 32;

template <int NC>
constexpr int batch_coords() {
  return NC >= kBatchFloats ? 1 : (kBatchFloats / NC < 8 ? kBatchFloats / NC : 8);
}

// y[c] += x[c] a for c < NC, reading x in chunks of at most kBatchFloats.
template <int NC>
__device__ __forceinline__ void axpy_chunks(float *y, const float *__restrict__ x, float a) {
  constexpr int CH = NC < kBatchFloats ? NC : kBatchFloats;
#pragma unroll
  for (int h = 0; h < NC / CH; ++h) {
    float xs[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) xs[i] = x[h * CH + i];
#pragma unroll
    for (int i = 0; i < CH; ++i) asm volatile("" ::"s"(xs[i]));
#pragma unroll
    for (int i = 0; i < CH; ++i) y[h * CH + i] = fmaf(xs[i], a, y[h * CH + i]);
  }
}

template <int LP, int L, int LAST>
__device__ __forceinline__ void descend_lean(float (&y)[1 << LP], const float *__restrict__ rec,
                                             int &xo, int &j0, uint64_t taus, const float *Al) {
  if constexpr (L >= LAST) {
    constexpr int NC = 1 << (LP - L);
    constexpr int H = NC / 2;
    constexpr int B = batch_coords<NC>();
    const int tau = (int)((taus >> (8 * L)) & 0xff);
    j0 -= tau;
    if (tau == 0) {
#pragma unroll
      for (int c = 0; c < H; ++c) y[c + H] = y[c];
    } else {
      const float *x = rec + xo;
      const float *Aj = Al + j0 * kTileT;  // row stride kTileT; kLdsPadRows zero rows follow
      if constexpr (B * NC <= kBatchFloats) {
        // first batch: coordinate 0 forms the children (the tile step)
        float xs[B * NC], av[B];
#pragma unroll
        for (int i = 0; i < B * NC; ++i) xs[i] = x[i];
#pragma unroll
        for (int i = 0; i < B; ++i) av[i] = Aj[i * kTileT];
        // consume every value here, so no load sinks into the guarded uses
#pragma unroll
        for (int i = 0; i < B * NC; ++i) asm volatile("" ::"s"(xs[i]));
#pragma unroll
        for (int i = 0; i < B; ++i) asm volatile("" ::"v"(av[i]));
#pragma unroll
        for (int c = 0; c < H; ++c) y[c + H] = fmaf(xs[c + H], av[0], y[c]);
#pragma unroll
        for (int c = 0; c < H; ++c) y[c] = fmaf(xs[c], av[0], y[c]);
#pragma unroll
        for (int i = 1; i < B; ++i) {
          if (i >= tau) break;
#pragma unroll
          for (int c = 0; c < NC; ++c) y[c] = fmaf(xs[i * NC + c], av[i], y[c]);
        }
#pragma unroll 1
        for (int jb = B; jb < tau; jb += B) {
#pragma unroll
          for (int i = 0; i < B * NC; ++i) xs[i] = x[jb * NC + i];
#pragma unroll
          for (int i = 0; i < B; ++i) av[i] = Aj[(jb + i) * kTileT];
#pragma unroll
          for (int i = 0; i < B * NC; ++i) asm volatile("" ::"s"(xs[i]));
#pragma unroll
          for (int i = 0; i < B; ++i) asm volatile("" ::"v"(av[i]));
#pragma unroll
          for (int i = 0; i < B; ++i) {
            if (jb + i >= tau) break;
#pragma unroll
            for (int c = 0; c < NC; ++c) y[c] = fmaf(xs[i * NC + c], av[i], y[c]);
          }
        }
      } else {  // NC = 64 (level 0 with more than one coordinate): one at a time, in chunks
        const float a0 = Aj[0];
        float z[H];
#pragma unroll
        for (int c = 0; c < H; ++c) z[c] = y[c];
        axpy_chunks<H>(y, x, a0);
        axpy_chunks<H>(z, x + H, a0);
#pragma unroll
        for (int c = 0; c < H; ++c) y[c + H] = z[c];
#pragma unroll 1
        for (int jj = 1; jj < tau; ++jj) axpy_chunks<NC>(y, x + jj * NC, Aj[jj * kTileT]);
      }
      xo += tau * NC;
    }
    descend_lean<LP, L - 1, LAST>(y, rec, xo, j0, taus, Al);
  }
}

// Level 0 with a single coordinate, fused with g: leaf c and c + H0 come from
// the level-1 node c.  The 2 H0 point values are read in halves of at most
// kBatchFloats.  Returns the FP32 sum of g over the subtree's leaves.
template <int LP, int GF, bool NEAR>
__device__ __forceinline__ float leaf_block(const float (&y)[1 << LP], const float *__restrict__ x0,
                                            float a0) {
  constexpr int H0 = (1 << LP) / 2;
  constexpr int HB = H0 < kBatchFloats / 2 ? H0 : kBatchFloats / 2;
  float s = 0.f;
#pragma unroll
  for (int h = 0; h < H0 / HB; ++h) {
    float xa[HB], xb[HB];
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      xa[i] = x0[h * HB + i];
      xb[i] = x0[H0 + h * HB + i];
    }
#pragma unroll
    for (int i = 0; i < HB; ++i) asm volatile("" ::"s"(xa[i]), "s"(xb[i]));
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int c = h * HB + i;
      if (NEAR) {
        s += g_val_near<GF>(fmaf(xa[i], a0, y[c]));
        s += g_val_near<GF>(fmaf(xb[i], a0, y[c]));
      } else {
        s += g_val<GF>(fmaf(xa[i], a0, y[c]));
        s += g_val<GF>(fmaf(xb[i], a0, y[c]));
      }
    }
  }
  return s;
}

// One level of the descent, one coordinate at a time (the modes that keep
// per-point state): y[0 .. 2^{LP-L}) becomes the level-L node values.
template <int LP, int L>
__device__ __forceinline__ void descend(float (&y)[1 << LP], const float *__restrict__ rec,
                                        const LeafLevel &lv, const float *Alds, int lda_s, int lane) {
  constexpr int NC = 1 << (LP - L);
  constexpr int H = NC / 2;
  const int tau = lv.tau;
  if (tau == 0) {
#pragma unroll
    for (int c = 0; c < H; ++c) y[c + H] = y[c];
    return;
  }
  const float *x = rec + lv.off;
  float a = Alds[lv.j0 * lda_s + lane];
#pragma unroll
  for (int c = 0; c < H; ++c) y[c + H] = fmaf(x[c + H], a, y[c]);
#pragma unroll
  for (int c = 0; c < H; ++c) y[c] = fmaf(x[c], a, y[c]);
#pragma unroll 1
  for (int jj = 1; jj < tau; ++jj) {
    x += NC;
    a = Alds[(lv.j0 + jj) * lda_s + lane];
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c] = fmaf(x[c], a, y[c]);
  }
}

template <int LP, int L, int LAST>
__device__ __forceinline__ void descend_to(float (&y)[1 << LP], const float *__restrict__ rec,
                                           const LeafLevel *lv, const float *Alds, int lda_s,
                                           int lane) {
  if constexpr (L >= LAST) {
    descend<LP, L>(y, rec, lv[L], Alds, lda_s, lane);
    descend_to<LP, L - 1, LAST>(y, rec, lv, Alds, lda_s, lane);
  }
}

// Adjoint of one level: dA_j += sum_c X~_L[c][j] S[c] for j in G_L, then fold
// the level-L node sums into their parents.
template <int LP, int L>
__device__ __forceinline__ void ascend(float (&S)[1 << LP], const float *__restrict__ rec,
                                       const LeafLevel &lv, float *dAl, int lane) {
  constexpr int NC = 1 << (LP - L);
  constexpr int H = NC / 2;
  const float *x = rec + lv.off;
#pragma unroll 1
  for (int jj = 0; jj < lv.tau; ++jj) {
    float d = 0.f;
#pragma unroll
    for (int c = 0; c < NC; ++c) d = fmaf(x[c], S[c], d);
    dAl[(lv.j0 + jj) * kTileT + lane] += d;
    x += NC;
  }
#pragma unroll
  for (int c = 0; c < H; ++c) S[c] = S[c] + S[c + H];
}

template <int LP, int L>
__device__ __forceinline__ void ascend_all(float (&S)[1 << LP], const float *__restrict__ rec,
                                           const LeafLevel *lv, float *dAl, int lane) {
  if constexpr (L < LP) {
    ascend<LP, L>(S, rec, lv[L], dAl, lane);
    ascend_all<LP, L + 1>(S, rec, lv, dAl, lane);
  }
}

// Sum over the 64 lanes of each of 64 per-lane values: afterwards v[0] of
// lane l holds sum over lanes of v[l] (butterfly transpose-reduction: at
// distance D a lane keeps the half of its slots selected by bit D of its
// lane id and adds the partner's copy of those slots).
template <int D>
__device__ __forceinline__ void transpose_step(float (&v)[64], int lane) {
  if constexpr (D >= 1) {
    const bool hi = (lane & D) != 0;
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const float send = hi ? v[c] : v[c + D];
      const float keep = hi ? v[c + D] : v[c];
      v[c] = keep + __shfl_xor(send, D, 64);
    }
    transpose_step<D / 2>(v, lane);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <int LP, int MODE, int GF, bool FUSE0>
__global__ __launch_bounds__(256) void leaf_kernel(LeafArgs a, const float *__restrict__ tables,
                                                   const float *__restrict__ U,
                                                   const float *__restrict__ A,
                                                   double *__restrict__ partial,
                                                   float *__restrict__ ppart, float *__restrict__ Y,
                                                   float *__restrict__ dApart,
                                                   float *__restrict__ Sroot,
                                                   const float *__restrict__ hd) {
  constexpr int NL = 1 << LP;
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // every wave of the workgroup works on column tile by, on its own subtrees
  const int bx = blockIdx.x, ct = blockIdx.y, rl = blockIdx.z;
  const int col = ct * kTileT + lane;
  const bool live = col < a.t;
  const int jlow = a.jlow;

  // rows 0 .. jlow-1 of sigma A for the tile, then kLdsPadRows zero rows
  float *Alds = smem;
  for (int e = tid; e < (jlow + kLdsPadRows) * kTileT; e += blockDim.x) {
    const int jr = e / kTileT, cl = ct * kTileT + (e % kTileT);
    Alds[e] = jr < jlow && cl < a.t ? a.sigma * A[(int64_t)jr * a.lda + cl] : 0.f;
  }
  float *dAl = smem + (jlow + kLdsPadRows) * kTileT + w * jlow * kTileT;
  if (MODE == kModeGrad)
    for (int e = lane; e < jlow * kTileT; e += 64) dAl[e] = 0.f;
  __syncthreads();
  const float *Al = Alds + lane;  // this lane's column; row stride kTileT

  // For cos: the subtree root is reduced to [0, 1) revolutions once; if the
  // lower levels add at most 250 revolutions in magnitude on every lane, the
  // leaves stay inside v_cos's domain and need no further reduction.
  bool near = false;
  if (GF == QMC_G_COS) {
    float bound = 0.f;
    for (int j = 0; j < jlow; ++j) bound += fabsf(Al[j * kTileT]);
    near = __all(bound * a.xmax < 250.0f);
  }

  const float *tab = tables + (int64_t)rl * a.tstride;
  const float *Ub = U + (int64_t)rl * a.ustride;
  double acc = 0.0;

  const int first = (bx * a.nw + w) * a.spw;
  const int last = min(first + a.spw, a.nsub);
  for (int rho = first; rho < last; ++rho) {
    const float *rec = tab + (int64_t)rho * a.rec;

    // subtree root: the upper levels' rows, requested RB at a time
    constexpr int RB = MODE == kModeSum ? kRootBatch : 1;
    float root = 0.f;
#pragma unroll 1
    for (int u0 = 0; u0 < a.nup; u0 += RB) {
      float rv[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i)  // entries past nup are zero: they read row 0
        rv[i] = Ub[(int64_t)(a.up_row0[u0 + i] + (rho & a.up_mask[u0 + i])) * a.ldu + col];
#pragma unroll
      for (int i = 0; i < RB; ++i) asm volatile("" ::"v"(rv[i]));
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if (u0 + i < a.nup) root += rv[i];
    }
    if (GF == QMC_G_COS) root = __builtin_amdgcn_fractf(root);

    float y[NL];
    y[0] = root;
    if (MODE == kModeSum) {
      // the level counts are re-read per subtree (opaque to the compiler), so
      // the per-level offsets are not hoisted into registers held for the
      // whole loop
      uint64_t taus = a.taus;
      asm volatile("" : "+s"(taus));
      int xo = 0, j0 = jlow;
      float s = 0.f;
      if constexpr (FUSE0) {
        descend_lean<LP, LP - 1, 1>(y, rec, xo, j0, taus, Al);
        const float a0 = Al[0];  // level 0 is row 0
        s = near ? leaf_block<LP, GF, true>(y, rec + xo, a0) : leaf_block<LP, GF, false>(y, rec + xo, a0);
      } else {
        descend_lean<LP, LP - 1, 0>(y, rec, xo, j0, taus, Al);
#pragma unroll
        for (int c = 0; c < NL; ++c) s += g_val<GF>(y[c]);
      }
      if (live) acc += (double)s;
    } else {
      descend_to<LP, LP - 1, 0>(y, rec, a.lv, Alds, kTileT, lane);
      if (MODE == kModePoint) {
        float v[64];
#pragma unroll
        for (int c = 0; c < 64; ++c) v[c] = (c < NL && live) ? g_val<GF>(y[c < NL ? c : 0]) : 0.f;
        transpose_step<32>(v, lane);
        if (lane < NL) ppart[(((int64_t)rl * a.tct + ct) * a.nsub + rho) * NL + lane] = v[0];
      } else if (MODE == kModeStoreY) {
        if (live) {
#pragma unroll
          for (int c = 0; c < NL; ++c) Y[((int64_t)rho + (int64_t)c * a.nsub) * a.ldy + col] = y[c];
        }
      } else {  // kModeGrad
        float S[NL];
        float s = 0.f;
        const float *hk = hd ? hd + ((int64_t)rl * a.nsub + rho) * NL : nullptr;
#pragma unroll
        for (int c = 0; c < NL; ++c) {
          if (hd == nullptr) s += g_val<GF>(y[c]);
          const float fac = hk ? hk[c] : 1.0f;
          S[c] = live ? (float)(a.gscale * (double)(fac * g_der<GF>(y[c], a.gc))) : 0.f;
        }
        if (live && hd == nullptr) acc += (double)s;
        ascend_all<LP, 0>(S, rec, a.lv, dAl, lane);
        if (live) Sroot[((int64_t)rl * 2 * a.nsub + rho) * a.ldu + col] = S[0];
      }
    }
  }

  if (MODE == kModeSum || MODE == kModeGrad) {
    __shared__ double red[4];
    const double wsum = wave_sum(acc);
    if (lane == 0) red[w] = wsum;
    __syncthreads();
    if (tid == 0) {
      double tot = red[0];
      for (int q = 1; q < a.nw; ++q) tot += red[q];
      partial[(int64_t)rl * a.nparts + bx * a.gy + ct] = tot;
    }
  }
  if (MODE == kModeGrad) {
    __syncthreads();
    // sum the per-wave dA accumulators of the workgroup
    const float *base = smem + (jlow + kLdsPadRows) * kTileT;
    const int64_t st = (int64_t)jlow * kTileT;
    for (int e = tid; e < st; e += blockDim.x) {
      float v = 0.f;
      for (int g = 0; g < a.nw; ++g) v += base[g * st + e];
      dApart[(((int64_t)rl * a.gx + bx) * a.tct + ct) * st + e] = v;
    }
  }
}

LeafPlan leaf_plan(const Geometry &G, int t, int nr, int mode) {
  const int64_t tct = ceil_div(t, kTileT);
  const int64_t units = G.nsub * tct * nr;  // subtree x column-tile pieces
  int spw = 1;
  while (spw < 32 && units / (spw * 2) >= 16384) spw *= 2;
  if (const char *env = getenv("QMC_LEAF_SPW")) {
    const int v = atoi(env);
    if (v >= 1 && v <= 1024) spw = v;
  }
  LeafPlan p;
  p.spw = spw;
  p.nw = mode == kModeGrad ? 2 : 4;  // waves per workgroup, each on its own subtrees
  p.gy = (int)tct;
  p.gx = (int)ceil_div(G.nsub, (int64_t)p.nw * spw);
  return p;
}

template <int LP, int MODE, bool F0>
static void leaf_launch_g(int gf, dim3 grid, size_t lds, hipStream_t st, const LeafArgs &a,
                          const float *tables, const float *U, const float *A, const LeafOut &o) {
#define QMC_LEAF_LAUNCH(GF)                                                                       \
  hipLaunchKernelGGL((leaf_kernel<LP, MODE, GF, F0>), grid, dim3(64 * a.nw), lds, st, a, tables, \
                     U, A, o.partial, o.ppart, o.Y, o.dApart, o.Sroot, o.hd)
  if (gf == QMC_G_COS) QMC_LEAF_LAUNCH(QMC_G_COS);
  else if (gf == QMC_G_EXP) QMC_LEAF_LAUNCH(QMC_G_EXP);
  else QMC_LEAF_LAUNCH(QMC_G_ID);
#undef QMC_LEAF_LAUNCH
}

template <int LP, int MODE>
static void leaf_launch_f(bool fuse0, int gf, dim3 grid, size_t lds, hipStream_t st,
                          const LeafArgs &a, const float *tables, const float *U, const float *A,
                          const LeafOut &o) {
  if constexpr (LP >= 1) {
    if (fuse0) return leaf_launch_g<LP, MODE, true>(gf, grid, lds, st, a, tables, U, A, o);
  }
  leaf_launch_g<LP, MODE, false>(gf, grid, lds, st, a, tables, U, A, o);
}

template <int LP>
static void leaf_launch_m(int mode, bool fuse0, int gf, dim3 grid, size_t lds, hipStream_t st,
                          const LeafArgs &a, const float *tables, const float *U, const float *A,
                          const LeafOut &o) {
  switch (mode) {
    case kModeSum: return leaf_launch_f<LP, kModeSum>(fuse0, gf, grid, lds, st, a, tables, U, A, o);
    case kModePoint: return leaf_launch_f<LP, kModePoint>(fuse0, gf, grid, lds, st, a, tables, U, A, o);
    case kModeStoreY: return leaf_launch_f<LP, kModeStoreY>(fuse0, gf, grid, lds, st, a, tables, U, A, o);
    default: return leaf_launch_f<LP, kModeGrad>(false, gf, grid, lds, st, a, tables, U, A, o);
  }
}

float g_scale(const qmc_integrand &f, int mode) {
  if (mode == kModeStoreY) return 1.0f;
  if (f.g == QMC_G_COS) return (float)(1.0 / (2.0 * 3.14159265358979323846));
  if (f.g == QMC_G_EXP) return (float)(f.c * 1.4426950408889634074);
  return 1.0f;
}

hipError_t launch_leaf(const Geometry &G, int mode, const qmc_integrand &f, const float *tables,
                       const float *U, int nr, int r0, const float *A, int t, int64_t lda,
                       int64_t ldu, const LeafPlan &lp, const LeafOut &o, hipStream_t st) {
  LaunchTimer tm("leaf", st);
  LeafArgs a{};
  a.t = t;
  a.tct = (int)ceil_div(t, kTileT);
  a.nsub = (int)G.nsub;
  a.rec = (int)G.rec;
  a.spw = lp.spw;
  a.gx = lp.gx;
  a.nw = lp.nw;
  a.jlow = G.jlow;
  a.r0 = r0;
  a.nup = G.nup;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    a.up_row0[u] = (int)L.uoff;
    a.up_mask[u] = (1 << L.nb) - 1;
  }
  a.taus = 0;
  for (int I = 0; I < G.split; ++I) {
    a.taus |= (uint64_t)G.lev[I].tau << (8 * I);
    a.lv[I].tau = G.lev[I].tau;
    a.lv[I].off = (int)G.lev[I].off;
    a.lv[I].j0 = G.lev[I].j0;
  }
  a.tstride = G.table_total;
  a.ustride = G.urows * ldu;
  a.lda = lda;
  a.ldu = ldu;
  a.ldy = o.ldy;
  a.sigma = g_scale(f, mode);
  a.gc = (float)f.c;
  a.gscale = o.gscale;
  a.gy = lp.gy;
  a.nparts = lp.gx * lp.gy;
  // largest |x| of a point value after the map (bounds the cos argument)
  a.xmax = G.map == QMC_MAP_INVNORM ? 8.5f : 1.0f;
  dim3 grid(lp.gx, lp.gy, nr);
  const size_t lds =
      sizeof(float) * kTileT * ((size_t)G.jlow + kLdsPadRows + (mode == kModeGrad ? (size_t)lp.nw * G.jlow : 0));
  // the matvec mode does not evaluate g
  const int gf = mode == kModeStoreY ? QMC_G_ID : f.g;
  const bool fuse0 = G.split >= 1 && G.lev[0].tau == 1;
  switch (G.split) {
    case 0: leaf_launch_m<0>(mode, false, gf, grid, lds, st, a, tables, U, A, o); break;
    case 1: leaf_launch_m<1>(mode, fuse0, gf, grid, lds, st, a, tables, U, A, o); break;
    case 2: leaf_launch_m<2>(mode, fuse0, gf, grid, lds, st, a, tables, U, A, o); break;
    case 3: leaf_launch_m<3>(mode, fuse0, gf, grid, lds, st, a, tables, U, A, o); break;
    case 4: leaf_launch_m<4>(mode, fuse0, gf, grid, lds, st, a, tables, U, A, o); break;
    case 5: leaf_launch_m<5>(mode, fuse0, gf, grid, lds, st, a, tables, U, A, o); break;
    default: leaf_launch_m<6>(mode, fuse0, gf, grid, lds, st, a, tables, U, A, o); break;
  }
  return hipGetLastError();
}

}  // namespace qmc
