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
// the lower levels sit in LDS.  All 2^{L'} partial sums of a level live in
// registers, so Y is never written (except in the matvec mode).
//
// Modes:
//   Sum    sum_k sum_i g(y_ki) per workgroup, FP32 inside a subtree, FP64 across
//   Point  per-point sums over the wave's 64 columns (for non-separable h)
//   StoreY write y_ki (the matrix-vector product)
//   Grad   G_ki = s_k g'(y_ki); sums of G up the subtree give S_I for the
//          lower levels (the transpose of the recursion), dA_I += X~_I^T S_I
//          per wave in LDS, the subtree-root sums S_{L'} go to memory.
#include "qmc_internal.h"

namespace qmc {

struct LeafArgs {
  Geometry G;
  int32_t t, r0, spw, tct, nr;
  int32_t gx, nw;
  int64_t lda, ldu, ldy;
  float gc;        // parameter c of g = exp(c y)
  float gcl2;      // c log2(e)
  double gscale;   // factor of g' in the adjoint
};

// g and g' on the transcendental unit.  cos and sin: v_cos/v_sin take the
// angle in revolutions; the argument y / (2 pi) is rounded once and reduced
// exactly with v_fract, so the only error beyond the FP32 rounding already
// present in y is that of the hardware approximation.  exp(c y) is
// 2^(y c log2 e) on v_exp, with c log2 e precomputed.
constexpr float kInv2Pi = 0.15915494309189533577f;

__device__ __forceinline__ float rev(float y) { return __builtin_amdgcn_fractf(y * kInv2Pi); }

template <int GF>
__device__ __forceinline__ float g_val(float y, float cl2) {
  if (GF == QMC_G_COS) return __builtin_amdgcn_cosf(rev(y));
  if (GF == QMC_G_EXP) return __builtin_amdgcn_exp2f(y * cl2);
  return y;
}

// derivative g'(y); c is the parameter of exp(c y)
template <int GF>
__device__ __forceinline__ float g_der(float y, float cl2, float c) {
  if (GF == QMC_G_COS) return -__builtin_amdgcn_sinf(rev(y));
  if (GF == QMC_G_EXP) return c * __builtin_amdgcn_exp2f(y * cl2);
  return 1.0f;
}

// One level of the descent: y[0 .. 2^{LP-L}) becomes the level-L node values.
template <int LP, int L>
__device__ __forceinline__ void descend(float (&y)[1 << LP], const float *__restrict__ rec,
                                        const Level &lv, const float *Alds, int lane) {
  constexpr int NC = 1 << (LP - L);
  constexpr int H = NC / 2;
  const int tau = lv.tau;
  if (tau == 0) {
#pragma unroll
    for (int c = 0; c < H; ++c) y[c + H] = y[c];
    return;
  }
  const float *x = rec + lv.off;
  float a = Alds[lv.j0 * kTileT + lane];
#pragma unroll
  for (int c = 0; c < H; ++c) y[c + H] = fmaf(x[c + H], a, y[c]);
#pragma unroll
  for (int c = 0; c < H; ++c) y[c] = fmaf(x[c], a, y[c]);
  for (int jj = 1; jj < tau; ++jj) {
    x += NC;
    a = Alds[(lv.j0 + jj) * kTileT + lane];
#pragma unroll
    for (int c = 0; c < NC; ++c) y[c] = fmaf(x[c], a, y[c]);
  }
}

template <int LP, int L>
__device__ __forceinline__ void descend_all(float (&y)[1 << LP], const float *__restrict__ rec,
                                            const Geometry &G, const float *Alds, int lane) {
  if constexpr (L >= 0) {
    descend<LP, L>(y, rec, G.lev[L], Alds, lane);
    descend_all<LP, L - 1>(y, rec, G, Alds, lane);
  }
}

// Adjoint of one level: dA_j += sum_c X~_L[c][j] S[c] for j in G_L, then fold
// the level-L node sums into their parents.
template <int LP, int L>
__device__ __forceinline__ void ascend(float (&S)[1 << LP], const float *__restrict__ rec,
                                       const Level &lv, float *dAl, int lane) {
  constexpr int NC = 1 << (LP - L);
  constexpr int H = NC / 2;
  const float *x = rec + lv.off;
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
                                           const Geometry &G, float *dAl, int lane) {
  if constexpr (L < LP) {
    ascend<LP, L>(S, rec, G.lev[L], dAl, lane);
    ascend_all<LP, L + 1>(S, rec, G, dAl, lane);
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

__device__ __forceinline__ float transpose_reduce64(float (&v)[64], int lane) {
  transpose_step<32>(v, lane);
  return v[0];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

template <int LP, int MODE, int GF>
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
  const Geometry &G = a.G;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nw = blockDim.x >> 6;  // waves per workgroup (4, or 2 for the adjoint)
  const int bx = blockIdx.x, ct = blockIdx.y, rl = blockIdx.z;
  const int r = a.r0 + rl;
  const int col = ct * kTileT + lane;
  const bool live = col < a.t;
  const int jlow = G.jlow;

  float *Alds = smem;
  for (int e = tid; e < jlow * kTileT; e += blockDim.x) {
    const int jr = e / kTileT, cl = ct * kTileT + (e % kTileT);
    Alds[e] = cl < a.t ? A[(int64_t)jr * a.lda + cl] : 0.f;
  }
  float *dAl = smem + jlow * kTileT + w * jlow * kTileT;
  if (MODE == kModeGrad)
    for (int e = lane; e < jlow * kTileT; e += 64) dAl[e] = 0.f;
  __syncthreads();

  const float *tab = tables + (int64_t)rl * G.table_total;
  const float *Ur = U + (int64_t)rl * G.urows * a.ldu;
  double acc = 0.0;

  const int64_t first = ((int64_t)bx * nw + w) * a.spw;
  for (int q = 0; q < a.spw; ++q) {
    const int64_t rho = first + q;
    if (rho >= G.nsub) break;
    const float *rec = tab + rho * G.rec;

    float root = 0.f;
    for (int u = 0; u < G.nup; ++u) {
      const Level &L = G.lev[G.up[u]];
      const int64_t row = L.uoff + (rho & ((int64_t(1) << L.nb) - 1));
      root += Ur[row * a.ldu + col];
    }

    float y[NL];
    y[0] = root;
    descend_all<LP, LP - 1>(y, rec, G, Alds, lane);

    if (MODE == kModeSum) {
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < NL; ++c) s += g_val<GF>(y[c], a.gcl2);
      if (live) acc += (double)s;
    } else if (MODE == kModePoint) {
      float v[64];
#pragma unroll
      for (int c = 0; c < 64; ++c) v[c] = (c < NL && live) ? g_val<GF>(y[c < NL ? c : 0], a.gcl2) : 0.f;
      const float tot = transpose_reduce64(v, lane);
      if (lane < NL) ppart[(((int64_t)rl * a.tct + ct) * G.nsub + rho) * NL + lane] = tot;
    } else if (MODE == kModeStoreY) {
      if (live) {
#pragma unroll
        for (int c = 0; c < NL; ++c) Y[(rho + (int64_t)c * G.nsub) * a.ldy + col] = y[c];
      }
    } else {  // kModeGrad
      float S[NL];
      float s = 0.f;
      const float *hk = hd ? hd + ((int64_t)rl * G.nsub + rho) * NL : nullptr;
#pragma unroll
      for (int c = 0; c < NL; ++c) {
        if (hd == nullptr) s += g_val<GF>(y[c], a.gcl2);
        const float fac = hk ? hk[c] : 1.0f;
        S[c] = live ? (float)(a.gscale * (double)(fac * g_der<GF>(y[c], a.gcl2, a.gc))) : 0.f;
      }
      if (live && hd == nullptr) acc += (double)s;
      ascend_all<LP, 0>(S, rec, G, dAl, lane);
      if (live) Sroot[((int64_t)rl * 2 * G.nsub + rho) * a.ldu + col] = S[0];
    }
  }

  if (MODE == kModeSum || MODE == kModeGrad) {
    __shared__ double red[4];
    const double ws = wave_sum(acc);
    if (lane == 0) red[w] = ws;
    __syncthreads();
    if (tid == 0) {
      double tot = red[0];
      for (int q = 1; q < nw; ++q) tot += red[q];
      partial[((int64_t)rl * a.gx + bx) * a.tct + ct] = tot;
    }
  }
  if (MODE == kModeGrad) {
    __syncthreads();
    float *out = dApart + (((int64_t)rl * a.gx + bx) * a.tct + ct) * (int64_t)jlow * kTileT;
    const float *base = smem + jlow * kTileT;
    const int64_t st = (int64_t)jlow * kTileT;
    for (int e = tid; e < jlow * kTileT; e += blockDim.x) {
      float v = base[e];
      for (int q = 1; q < nw; ++q) v += base[e + q * st];
      out[e] = v;
    }
  }
}

LeafPlan leaf_plan(const Geometry &G, int t, int nr, int mode) {
  const int64_t tct = ceil_div(t, kTileT);
  const int64_t units = G.nsub * tct * nr;  // subtree x column-tile pieces
  int spw = 1;
  while (spw < 32 && units / (spw * 2) >= 16384) spw *= 2;
  LeafPlan p;
  p.spw = spw;
  p.nw = mode == kModeGrad ? 2 : 4;
  p.gx = (int)ceil_div(G.nsub, p.nw * spw);
  return p;
}

template <int LP, int MODE>
static hipError_t leaf_dispatch_g(int gf, dim3 grid, size_t lds, hipStream_t st, const LeafArgs &a,
                                  const float *tables, const float *U, const float *A,
                                  const LeafOut &o) {
#define QMC_LEAF_LAUNCH(GF)                                                                       \
  hipLaunchKernelGGL((leaf_kernel<LP, MODE, GF>), grid, dim3(64 * a.nw), lds, st, a, tables, U, A, \
                     o.partial, o.ppart, o.Y, o.dApart, o.Sroot, o.hd)
  if (gf == QMC_G_COS) QMC_LEAF_LAUNCH(QMC_G_COS);
  else if (gf == QMC_G_EXP) QMC_LEAF_LAUNCH(QMC_G_EXP);
  else QMC_LEAF_LAUNCH(QMC_G_ID);
#undef QMC_LEAF_LAUNCH
  return hipGetLastError();
}

template <int LP>
static hipError_t leaf_dispatch_mode(int mode, int gf, dim3 grid, size_t lds, hipStream_t st,
                                     const LeafArgs &a, const float *tables, const float *U,
                                     const float *A, const LeafOut &o) {
  switch (mode) {
    case kModeSum: return leaf_dispatch_g<LP, kModeSum>(gf, grid, lds, st, a, tables, U, A, o);
    case kModePoint: return leaf_dispatch_g<LP, kModePoint>(gf, grid, lds, st, a, tables, U, A, o);
    case kModeStoreY: return leaf_dispatch_g<LP, kModeStoreY>(gf, grid, lds, st, a, tables, U, A, o);
    default: return leaf_dispatch_g<LP, kModeGrad>(gf, grid, lds, st, a, tables, U, A, o);
  }
}

hipError_t launch_leaf(const Geometry &G, int mode, const qmc_integrand &f, const float *tables,
                       const float *U, int nr, int r0, const float *A, int t, int64_t lda,
                       int64_t ldu, const LeafPlan &lp, const LeafOut &o, hipStream_t st) {
  LaunchTimer tm("leaf", st);
  LeafArgs a;
  a.G = G;
  a.t = t;
  a.r0 = r0;
  a.spw = lp.spw;
  a.tct = (int)ceil_div(t, kTileT);
  a.nr = nr;
  a.gx = lp.gx;
  a.nw = lp.nw;
  a.lda = lda;
  a.ldu = ldu;
  a.ldy = o.ldy;
  a.gc = (float)f.c;
  a.gcl2 = (float)(f.c * 1.4426950408889634074);
  a.gscale = o.gscale;
  dim3 grid(lp.gx, a.tct, nr);
  const size_t lds = sizeof(float) * (size_t)G.jlow * kTileT * (mode == kModeGrad ? 1 + lp.nw : 1);
  // the matvec mode does not evaluate g
  const int gf = mode == kModeStoreY ? QMC_G_ID : f.g;
  switch (G.split) {
    case 0: return leaf_dispatch_mode<0>(mode, gf, grid, lds, st, a, tables, U, A, o);
    case 1: return leaf_dispatch_mode<1>(mode, gf, grid, lds, st, a, tables, U, A, o);
    case 2: return leaf_dispatch_mode<2>(mode, gf, grid, lds, st, a, tables, U, A, o);
    case 3: return leaf_dispatch_mode<3>(mode, gf, grid, lds, st, a, tables, U, A, o);
    case 4: return leaf_dispatch_mode<4>(mode, gf, grid, lds, st, a, tables, U, A, o);
    case 5: return leaf_dispatch_mode<5>(mode, gf, grid, lds, st, a, tables, U, A, o);
    default: return leaf_dispatch_mode<6>(mode, gf, grid, lds, st, a, tables, U, A, o);
  }
}

}  // namespace qmc
