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

// One level of the descent: y[0 .. 2^{LP-L}) becomes the level-L node values.
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
  constexpr int H0 = NL / 2;
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // wave layout: cw column tiles x sw subtree groups per workgroup
  const int wc = w % a.cw, ws = w / a.cw;
  const int bx = blockIdx.x, by = blockIdx.y, rl = blockIdx.z;
  const int ct = by * a.cw + wc;
  const int col = ct * kTileT + lane;
  const bool live = col < a.t;
  const int jlow = a.jlow;
  const int wcols = a.cw * kTileT;  // columns of A staged by this workgroup

  float *Alds = smem;
  for (int e = tid; e < jlow * wcols; e += blockDim.x) {
    const int jr = e / wcols, cl = by * wcols + (e % wcols);
    Alds[e] = cl < a.t ? a.sigma * A[(int64_t)jr * a.lda + cl] : 0.f;
  }
  float *dAl = smem + jlow * wcols + w * jlow * kTileT;
  if (MODE == kModeGrad)
    for (int e = lane; e < jlow * kTileT; e += 64) dAl[e] = 0.f;
  __syncthreads();
  const float *Aw = Alds + wc * kTileT;  // this wave's columns; row stride wcols

  // For cos: the subtree root is reduced to [0, 1) revolutions once; if the
  // lower levels add at most 250 revolutions in magnitude on every lane, the
  // leaves stay inside v_cos's domain and need no further reduction.
  bool near = false;
  if (GF == QMC_G_COS) {
    float bound = 0.f;
    for (int j = 0; j < jlow; ++j) bound += fabsf(Aw[j * wcols + lane]);
    near = __all(bound * a.xmax < 250.0f);
  }

  const float *tab = tables + (int64_t)rl * a.tstride;
  const float *Ub = U + (int64_t)rl * a.ustride;
  double acc = 0.0;

  const int first = (bx * a.sw + ws) * a.spw;
  const int last = min(first + a.spw, a.nsub);
  for (int rho = first; rho < last; ++rho) {
    const float *rec = tab + (int64_t)rho * a.rec;

    float root = 0.f;
#pragma unroll 1
    for (int u = 0; u < a.nup; ++u) {
      const float *row = Ub + (int64_t)(a.up_row0[u] + (rho & a.up_mask[u])) * a.ldu;
      root += row[col];
    }
    if (GF == QMC_G_COS) root = __builtin_amdgcn_fractf(root);

    float y[NL];
    y[0] = root;
    if (FUSE0) {
      descend_to<LP, LP - 1, 1>(y, rec, a.lv, Aw, wcols, lane);
    } else {
      descend_to<LP, LP - 1, 0>(y, rec, a.lv, Aw, wcols, lane);
    }

    if (MODE == kModeSum) {
      float s = 0.f;
      if (FUSE0) {
        const float *x0 = rec + a.lv[0].off;
        const float a0 = Aw[a.lv[0].j0 * wcols + lane];
        if (near) {
#pragma unroll
          for (int c = 0; c < H0; ++c) {
            s += g_val_near<GF>(fmaf(x0[c], a0, y[c]));
            s += g_val_near<GF>(fmaf(x0[c + H0], a0, y[c]));
          }
        } else {
#pragma unroll
          for (int c = 0; c < H0; ++c) {
            s += g_val<GF>(fmaf(x0[c], a0, y[c]));
            s += g_val<GF>(fmaf(x0[c + H0], a0, y[c]));
          }
        }
      } else {
#pragma unroll
        for (int c = 0; c < NL; ++c) s += g_val<GF>(y[c]);
      }
      if (live) acc += (double)s;
    } else {
      if (FUSE0) descend<LP, 0>(y, rec, a.lv[0], Aw, wcols, lane);
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
      partial[(int64_t)rl * a.nparts + bx * a.gy + by] = tot;
    }
  }
  if (MODE == kModeGrad) {
    __syncthreads();
    // per column tile of the workgroup: sum the waves of all subtree groups
    const float *base = smem + jlow * wcols;
    const int64_t st = (int64_t)jlow * kTileT;
    for (int e = tid; e < a.cw * jlow * kTileT; e += blockDim.x) {
      const int q = e / (jlow * kTileT), o = e % (jlow * kTileT);
      const int ctq = by * a.cw + q;
      if (ctq >= a.tct) continue;
      float v = 0.f;
      for (int g = 0; g < a.sw; ++g) v += base[(g * a.cw + q) * st + o];
      dApart[(((int64_t)rl * a.gx + bx) * a.tct + ctq) * st + o] = v;
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
  p.nw = mode == kModeGrad ? 2 : 4;
  p.cw = 1;  // waves side by side over column tiles (1: each wave its own subtrees)
  if (const char *env = getenv("QMC_LEAF_CW")) {
    const int v = atoi(env);
    if (v >= 1 && v <= p.nw) p.cw = v;
  }
  p.cw = (int)std::min<int64_t>(p.cw, tct);
  while (p.nw % p.cw) --p.cw;
  p.sw = p.nw / p.cw;                         // and over subtree groups
  p.gy = (int)ceil_div(tct, p.cw);
  p.gx = (int)ceil_div(G.nsub, p.sw * spw);
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
  for (int I = 0; I < G.split; ++I) {
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
  a.cw = lp.cw;
  a.sw = lp.sw;
  a.gy = lp.gy;
  a.nparts = lp.gx * lp.gy;
  // largest |x| of a point value after the map (bounds the cos argument)
  a.xmax = G.map == QMC_MAP_INVNORM ? 8.5f : 1.0f;
  dim3 grid(lp.gx, lp.gy, nr);
  const size_t lds =
      sizeof(float) * (size_t)G.jlow * kTileT * (lp.cw + (mode == kModeGrad ? lp.nw : 0));
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
