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
//   StoreY write y_ki (the matrix-vector product): the subtree's record is
//          first copied to a per-wave LDS slot (one round of vector loads)
//          when it has at most kRecLds floats, the workgroups are taken
//          column tile first, and Y is written with non-temporal stores
//   Grad   G'_ki = h'(u_k) g'_unit(y_ki); sums of G' up the subtree give S_I
//          for the lower levels (the transpose of the recursion), dA_I +=
//          X~_I^T S_I, the subtree-root sums S_{L'} go to memory.  This file
//          holds the form that accumulates dA per wave in LDS (any level
//          shape); adjoint.hip the register form used when every lower level
//          I holds at most 2^I coordinates.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "leaf_common.h"

namespace qmc {

// Level 0 with a single coordinate, fused with g: leaf c and c + H0 come from
// the level-1 node c.  The 2 H0 point values are read in halves of at most
// kBatchFloats (a quarter for cos).  s[q] receives the FP32 sum of g over the subtree's leaves in
// column q of the lane.
template <int LP, int GF, bool NEAR, int CPL>
__device__ __forceinline__ void leaf_block(const float (&y)[CPL][1 << LP],
                                           const float *__restrict__ x0, const float (&a0)[CPL],
                                           float (&s)[CPL]) {
  constexpr int H0 = (1 << LP) / 2;
  // cos needs more scalar registers than the other integrands: half batches
  // let it fit eight waves per SIMD
  constexpr int HBF = GF == QMC_G_COS ? kBatchFloats / 4 : kBatchFloats / 2;
  constexpr int HB = H0 < HBF ? H0 : HBF;
  constexpr int NA = 4;  // independent partial sums per column (breaks the add chain)
  float sp[CPL][NA];
#pragma unroll
  for (int q = 0; q < CPL; ++q)
#pragma unroll
    for (int k = 0; k < NA; ++k) sp[q][k] = 0.f;
#pragma unroll
  for (int h = 0; h < H0 / HB; ++h) {
    float xa[HB], xb[HB];
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      xa[i] = x0[h * HB + i];
      xb[i] = x0[H0 + h * HB + i];
    }
    keep_scalar(xa);
    keep_scalar(xb);
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int c = h * HB + i;
#pragma unroll
      for (int q = 0; q < CPL; ++q) {
        float ga, gb;
        if (NEAR) {
          ga = g_val_near<GF>(fmaf(xa[i], a0[q], y[q][c]));
          gb = g_val_near<GF>(fmaf(xb[i], a0[q], y[q][c]));
        } else {
          ga = g_val<GF>(fmaf(xa[i], a0[q], y[q][c]));
          gb = g_val<GF>(fmaf(xb[i], a0[q], y[q][c]));
        }
        sp[q][(2 * c) % NA] += ga;
        sp[q][(2 * c + 1) % NA] += gb;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < CPL; ++q) s[q] = (sp[q][0] + sp[q][1]) + (sp[q][2] + sp[q][3]);
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
  // the first coordinate forms the new nodes from their parents, 2 x CH point
  // values at a time (a whole level-0 block would hold 64 scalar registers)
  constexpr int CH = H < 16 ? H : 16;
#pragma unroll
  for (int h0 = 0; h0 < H; h0 += CH) {
    float xa[CH], xb[CH];
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      xa[i] = x[h0 + i];
      xb[i] = x[H + h0 + i];
    }
    keep_scalar(xa);
    keep_scalar(xb);
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      y[h0 + i + H] = fmaf(xb[i], a, y[h0 + i]);
      y[h0 + i] = fmaf(xa[i], a, y[h0 + i]);
    }
  }
#pragma unroll 1
  for (int jj = 1; jj < tau; ++jj) {
    x += NC;
    a = Alds[(lv.j0 + jj) * lda_s + lane];
    constexpr int CB = NC < 32 ? NC : 32;
#pragma unroll
    for (int c0 = 0; c0 < NC; c0 += CB) {
      float xs[CB];
#pragma unroll
      for (int i = 0; i < CB; ++i) xs[i] = x[c0 + i];
      keep_scalar(xs);
#pragma unroll
      for (int i = 0; i < CB; ++i) y[c0 + i] = fmaf(xs[i], a, y[c0 + i]);
    }
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
// At distances 32 and 16 one lane-swap instruction does the exchange:
// v_permlane32_swap(X, Y) returns (X of lanes 0-31, Y of lanes 0-31) and
// (X of lanes 32-63, Y of lanes 32-63) as the lower and upper halves of its
// two results (v_permlane16_swap the same for 16-lane rows), so each lane's
// kept slot and its partner's copy are the two results, and one add finishes
// the pair (the same sums as the selected exchange below, bit for bit).
template <int D>
__device__ __forceinline__ void transpose_step(float (&v)[64], int lane) {
  if constexpr (D == 32 || D == 16) {
#pragma unroll
    for (int c = 0; c < D; ++c) {
      const auto r = D == 32
                         ? __builtin_amdgcn_permlane32_swap(__float_as_uint(v[c]), __float_as_uint(v[c + D]), false, false)
                         : __builtin_amdgcn_permlane16_swap(__float_as_uint(v[c]), __float_as_uint(v[c + D]), false, false);
      v[c] = __uint_as_float(r[0]) + __uint_as_float(r[1]);
    }
    transpose_step<D / 2>(v, lane);
  } else if constexpr (D >= 1) {
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


// The summing mode with one column per lane fits eight waves per SIMD in its
// scalar registers (cos with its leaf values read 2 x 8 at a time), so it asks
// for eight: C2 and C4 then run their 16 waves per SIMD in two full rounds.
template <int LP, int MODE, int GF, bool FUSE0, int CPL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(
    MODE == kModeSum && CPL == 1 ? 8 : 1))) void leaf_kernel(LeafArgs a, const float *__restrict__ tables,
                                                   const float *__restrict__ U,
                                                   const float *__restrict__ A,
                                                   double *__restrict__ partial,
                                                   float *__restrict__ ppart, float *__restrict__ Y,
                                                   float *__restrict__ dApart,
                                                   float *__restrict__ Sroot,
                                                   const float *__restrict__ hd) {
  constexpr int NL = 1 << LP;
  constexpr int CW = CPL * kTileT;  // columns of A per workgroup (CPL per lane)
  static_assert(CPL == 1 || MODE == kModeSum, "several columns per lane: summing mode only");
  extern __shared__ float smem[];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  // every wave of the workgroup works on column tile ct (CW columns), on its
  // own subtrees; lane column q is ct CW + q 64 + lane
  // Storing mode: workgroups are taken column tile first, so the tiles of one
  // subtree group run together and their stores fill whole rows of Y at once.
  const int lin = (int)(blockIdx.x + blockIdx.y * gridDim.x);
  const int bx = MODE == kModeStoreY ? lin / (int)gridDim.y : (int)blockIdx.x;
  const int ct = MODE == kModeStoreY ? lin % (int)gridDim.y : (int)blockIdx.y;
  const int rl = blockIdx.z;
  const int col = ct * CW + lane;
  // Storing mode: a lane past column t does the last column's work and stores
  // the same values to the same addresses, so the stores need no branch (a
  // branch around them would keep the prefetch below from overlapping them).
  const int lcol = MODE == kModeStoreY && col >= a.t ? a.t - 1 - ct * CW : lane;
  bool live[CPL];
#pragma unroll
  for (int q = 0; q < CPL; ++q) live[q] = col + q * kTileT < a.t;
  const int jlow = a.jlow;

  // rows 0 .. jlow-1 of sigma A for the tile, then kLdsPadRows zero rows
  // Every load of a pass is issued before the first is used (addresses are
  // clamped into A, out-of-range elements are then replaced by 0), so a pass
  // costs one memory round trip.
  __shared__ double red[4];  // per-wave sums
  __shared__ int arrived;     // waves done (counted in LDS)
  if (tid == 0) arrived = 0;  // visible to all after the barrier below
  float *Alds = smem;
  const int stage_total = (jlow + kLdsPadRows) * CW;
  for (int e0 = 0; e0 < stage_total; e0 += kStagePerThread * (int)blockDim.x) {
    float v[kStagePerThread];
#pragma unroll
    for (int k = 0; k < kStagePerThread; ++k) {
      const int e = e0 + k * (int)blockDim.x + tid;
      const int jr = e / CW, cl = ct * CW + (e % CW);
      const int jrc = min(jr, max(jlow - 1, 0)), clc = min(cl, a.t - 1);
      const float x = A[(int64_t)jrc * a.lda + clc];
      v[k] = e < stage_total && jr < jlow && cl < a.t ? a.sigma * x : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kStagePerThread; ++k) {
      const int e = e0 + k * (int)blockDim.x + tid;
      if (e < stage_total) Alds[e] = v[k];
    }
  }
  float *dAl = smem + (jlow + kLdsPadRows) * CW + w * jlow * kTileT;
  // Storing mode: a record of at most kRecLds floats is copied to the wave's
  // own LDS slot with one round of vector loads, and the descent reads its
  // point values there instead of in one scalar round trip per batch.
  float *recl = smem + (jlow + kLdsPadRows) * CW + w * kRecSlot;
  const bool rec_lds = MODE == kModeStoreY && a.rec >= 1 && a.rec <= kRecLds;  // split 0: no record
  if (MODE == kModeGrad)
    for (int e = lane; e < jlow * kTileT; e += 64) dAl[e] = 0.f;
  __syncthreads();
  const float *Al = Alds + lane;  // this lane's first column; row stride CW

  // For cos: the subtree root is reduced to [0, 1) revolutions once; if the
  // lower levels add at most 250 revolutions in magnitude on every lane, the
  // leaves stay inside v_cos's domain and need no further reduction.
  bool near = false;
  if (GF == QMC_G_COS) {
    float bound = 0.f, bq[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) bq[q] = 0.f;
    for (int j = 0; j < jlow; ++j)
#pragma unroll
      for (int q = 0; q < CPL; ++q) bq[q] += fabsf(Al[j * CW + q * kTileT]);
#pragma unroll
    for (int q = 0; q < CPL; ++q) bound = fmaxf(bound, bq[q]);
    near = __all(bound * a.xmax < 250.0f);
  }

  const float *tab = tables + (int64_t)rl * a.tstride;
  const float *Ub = U + (int64_t)rl * a.ustride;
  double acc = 0.0;

  // the workgroup's share of the subtrees, dealt to its waves in turn
  // (balanced: the first sub_rem workgroups take sub_per + 1 subtrees)
  const int first = bx * a.sub_per + min(bx, a.sub_rem);
  const int last = first + a.sub_per + (bx < a.sub_rem ? 1 : 0);
  // subtree root: the upper levels' rows, requested RB at a time
  constexpr int RB = MODE == kModeGrad ? 1 : kRootBatch;
  auto root_batch = [&](int rho, int u0, float (&rv)[RB][CPL]) {
#pragma unroll
    for (int i = 0; i < RB; ++i) {  // entries past nup are zero: they read row 0
      // uniform row address (scalar unit), then this lane's column
      const float *row = Ub + a.up_off[u0 + i] + (uint64_t)(uint32_t)(rho & a.up_mask[u0 + i]) * a.ldu32;
#pragma unroll
      for (int q = 0; q < CPL; ++q) rv[i][q] = row[ct * CW + lcol + q * kTileT];
    }
  };
  // Storing mode: the first root batch of the wave's next subtree is requested
  // before this subtree's rows of Y are stored, so waiting for it does not
  // wait for those stores too (one vector memory counter covers both).  The
  // wave's first subtree loads its own.
  float rvn[RB][CPL];
  for (int rho = first + w; rho < last; rho += a.nw) {
    const float *rec = tab + (int64_t)rho * a.rec;

    float root[CPL];
#pragma unroll
    for (int q = 0; q < CPL; ++q) root[q] = 0.f;
    int ubeg = 0;
    if (MODE == kModeStoreY && rho != first + w) {
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          asm volatile("" ::"v"(rvn[i][q]));
          if (i < a.nup) root[q] += rvn[i][q];
        }
      ubeg = RB;
    }
#pragma unroll 1
    for (int u0 = ubeg; u0 < a.nup; u0 += RB) {
      float rv[RB][CPL];
      root_batch(rho, u0, rv);
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int q = 0; q < CPL; ++q) asm volatile("" ::"v"(rv[i][q]));
#pragma unroll
      for (int i = 0; i < RB; ++i)
        if (u0 + i < a.nup)
#pragma unroll
          for (int q = 0; q < CPL; ++q) root[q] += rv[i][q];
    }
    if (GF == QMC_G_COS)
#pragma unroll
      for (int q = 0; q < CPL; ++q) root[q] = __builtin_amdgcn_fractf(root[q]);

    if constexpr (MODE == kModeSum) {
      // the level counts are re-read per subtree (opaque to the compiler), so
      // the per-level offsets are not hoisted into registers held for the
      // whole loop
      uint64_t taus = a.taus;
      asm volatile("" : "+s"(taus));
      int xo = 0, j0 = jlow;
      float y[CPL][NL], s[CPL];
#pragma unroll
      for (int q = 0; q < CPL; ++q) y[q][0] = root[q];
      if constexpr (FUSE0) {
        descend_lean<LP, LP - 1, 1, CPL>(y, rec, xo, j0, taus, Al);
        float a0[CPL];  // level 0 is row 0
#pragma unroll
        for (int q = 0; q < CPL; ++q) a0[q] = Al[q * kTileT];
        if (near) leaf_block<LP, GF, true, CPL>(y, rec + xo, a0, s);
        else leaf_block<LP, GF, false, CPL>(y, rec + xo, a0, s);
      } else {
        descend_lean<LP, LP - 1, 0, CPL>(y, rec, xo, j0, taus, Al);
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
          s[q] = 0.f;
#pragma unroll
          for (int c = 0; c < NL; ++c) s[q] += g_val<GF>(y[q][c]);
        }
      }
#pragma unroll
      for (int q = 0; q < CPL; ++q)
        if (live[q]) acc += (double)s[q];
    } else if constexpr (MODE == kModeStoreY || MODE == kModePoint) {
      // the lean descent of the summing mode, then the 64 rows of Y, or the
      // leaves' g summed over the wave's columns (one sum per point)
      uint64_t taus = a.taus;
      asm volatile("" : "+s"(taus));
      int xo = 0, j0 = jlow;
      float y[1][NL];
      y[0][0] = root[0];
      if (MODE == kModeStoreY && rec_lds) {
        // every load is issued before the first store; addresses past the
        // record are clamped to its last float
        float v[kRecLds / 64];
#pragma unroll
        for (int i = 0; i < kRecLds / 64; ++i) v[i] = rec[min(lane + 64 * i, (int)a.rec - 1)];
#pragma unroll
        for (int i = 0; i < kRecLds / 64; ++i) recl[lane + 64 * i] = v[i];
        descend_lean<LP, LP - 1, 0, 1, true>(y, recl, xo, j0, taus, Alds + lcol);
      } else {
        descend_lean<LP, LP - 1, 0, 1>(y, rec, xo, j0, taus, Alds + lcol);
      }
      if constexpr (MODE == kModeStoreY) {
        if (a.nup > 0 && rho + a.nw < last) root_batch(rho + a.nw, 0, rvn);
        // Y is streamed past the caches (it is not read back here, and a large
        // one would only evict the records and root rows)
#pragma unroll
        for (int c = 0; c < NL; ++c)
          __builtin_nontemporal_store(y[0][c], &Y[((int64_t)rho + (int64_t)c * a.nsub) * a.ldy + ct * CW + lcol]);
      } else {
        float v[64];
#pragma unroll
        for (int c = 0; c < 64; ++c) v[c] = (c < NL && live[0]) ? g_val<GF>(y[0][c < NL ? c : 0]) : 0.f;
        transpose_step<32>(v, lane);
        if (lane < NL) ppart[(((int64_t)rl * a.tct + ct) * a.nsub + rho) * NL + lane] = v[0];
      }
    } else {
      float y[NL];
      y[0] = root[0];
      const bool live0 = live[0];
      descend_to<LP, LP - 1, 0>(y, rec, a.lv, Alds, kTileT, lane);
      {  // kModeGrad
        float S[NL];
        float s = 0.f;
        const float *hk = hd ? hd + ((int64_t)rl * a.nsub + rho) * NL : nullptr;
#pragma unroll
        for (int c = 0; c < NL; ++c) {
          if (hd == nullptr) s += g_val<GF>(y[c]);
          const float fac = hk ? hk[c] : 1.0f;
          S[c] = live0 ? fac * g_der_unit<GF, false>(y[c]) : 0.f;
        }
        if (live0 && hd == nullptr) acc += (double)s;
        ascend_all<LP, 0>(S, rec, a.lv, dAl, lane);
        if (live0) Sroot[((int64_t)rl * 2 * a.nsub + rho) * a.ldu + col] = S[0];
      }
    }
  }

  if (MODE == kModeSum || MODE == kModeGrad) {
    // One FP64 partial per workgroup without a barrier: each wave leaves its
    // sum in LDS and counts itself in; the last to arrive adds the sums in
    // wave order (deterministic) and writes the partial.
    const double wsum = wave_sum(acc);
    if (lane == 0) {
      red[w] = wsum;
      __threadfence_block();
      if (atomicAdd(&arrived, 1) == a.nw - 1) {
        __threadfence_block();
        double tot = red[0];
        for (int q = 1; q < a.nw; ++q) tot += red[q];
        partial[(int64_t)rl * a.nparts + bx * a.gy + ct] = tot;
      }
    }
  }
  if (MODE == kModeGrad) {
    __syncthreads();
    // sum the per-wave dA accumulators of the workgroup
    const float *base = smem + (jlow + kLdsPadRows) * CW;
    const int64_t st = (int64_t)jlow * kTileT;
    for (int e = tid; e < st; e += blockDim.x) {
      float v = 0.f;
      for (int g = 0; g < a.nw; ++g) v += base[g * st + e];
      dApart[(((int64_t)rl * a.gx + bx) * a.tct + ct) * st + e] = v;
    }
  }
}

static size_t leaf_lds_bytes(const Geometry &G, int mode, int cpl, int nw);
static const void *leaf_fn(const Geometry &G, int mode, int gf, int cpl);

LeafPlan leaf_plan(const Geometry &G, int t, int nr, int mode, int gf) {
  const int64_t tct = ceil_div(t, kTileT);
  LeafPlan p;
  // the summing mode can give each lane two columns (QMC_LEAF_CPL=2), unless
  // the lane would then hold two full 64-leaf arrays (level 0 not fused)
  const bool fuse0 = G.split >= 1 && G.lev[0].tau == 1;
  const bool two_ok = mode == kModeSum && (fuse0 || G.split < kMaxSplit);
  p.cpl = 1;  // two columns per lane measured slower (lower occupancy); kept selectable
  if (const char *env = getenv("QMC_LEAF_CPL")) {
    const int v = atoi(env);
    if (two_ok && (v == 1 || v == 2)) p.cpl = v;
  }
  if (p.cpl == 2 && tct < 2) p.cpl = 1;
  p.gy = (int)ceil_div(tct, p.cpl);
  // waves per workgroup, each on its own subtrees (the LDS form of the adjoint
  // keeps one accumulator block per wave in LDS: two waves)
  p.nw = mode == kModeGrad && !grad_reg_ok(G) ? 2 : 4;
  const int64_t pairs = (int64_t)p.gy * nr;  // (shift, column tile) pairs
  const int64_t units = G.nsub * pairs;      // subtree x column-tile pieces
  // more subtrees per wave amortise the staging of A and the final reduction,
  // as long as more than 8192 waves (eight per SIMD) remain to hide latency
  int spw = 1;
  while (spw < 32 && units / (spw * 2) > 8192) spw *= 2;
  if (const char *env = getenv("QMC_LEAF_SPW")) {
    const int v = atoi(env);
    if (v >= 1 && v <= 1024) spw = v;
  }
  p.spw = spw;
  p.gx = (int)ceil_div(G.nsub, (int64_t)p.nw * spw);
  // A grid that needs only a few rounds of resident workgroups loses much of
  // its time to the staging at the start of each round and to the last,
  // partly filled round.  Then launch exactly one round instead: every
  // resident workgroup takes an equal share of its pair's subtrees.
  // (measured: a gain for the per-point mode, a loss for the summing mode,
  // whose short waves overlap their start-up latency better)
  bool one_round = mode == kModePoint;
  if (const char *env = getenv("QMC_LEAF_ONE_ROUND")) one_round = atoi(env) != 0;
  if (one_round) {
    const void *fn = leaf_fn(G, mode, gf, p.cpl);
    const int64_t cap = resident_workgroups(fn, 64 * p.nw, leaf_lds_bytes(G, mode, p.cpl, p.nw));
    const int64_t wgs = pairs * p.gx;
    if (cap > 0 && wgs > cap && wgs <= 4 * cap && pairs <= cap) {
      const int64_t gx = std::min<int64_t>(cap / pairs, ceil_div(G.nsub, (int64_t)p.nw));
      p.gx = (int)std::max<int64_t>(gx, 1);
    }
  }
  return p;
}

// The kernel instance for a geometry, mode, g and columns per lane.
template <int LP, int MODE, bool F0>
static const void *leaf_fn_g(int gf, int cpl) {
#define QMC_LEAF_FN(GF, CPL) reinterpret_cast<const void *>(&leaf_kernel<LP, MODE, GF, F0, CPL>)
  if constexpr (MODE == kModeSum && (F0 || LP < kMaxSplit)) {
    if (cpl == 2) {
      if (gf == QMC_G_COS) return QMC_LEAF_FN(QMC_G_COS, 2);
      if (gf == QMC_G_EXP) return QMC_LEAF_FN(QMC_G_EXP, 2);
      return QMC_LEAF_FN(QMC_G_ID, 2);
    }
  }
  if (gf == QMC_G_COS) return QMC_LEAF_FN(QMC_G_COS, 1);
  if (gf == QMC_G_EXP) return QMC_LEAF_FN(QMC_G_EXP, 1);
  return QMC_LEAF_FN(QMC_G_ID, 1);
#undef QMC_LEAF_FN
}

template <int LP, int MODE>
static const void *leaf_fn_f(bool fuse0, int gf, int cpl) {
  if constexpr (LP >= 1 && MODE != kModeGrad) {
    if (fuse0) return leaf_fn_g<LP, MODE, true>(gf, cpl);
  }
  return leaf_fn_g<LP, MODE, false>(gf, cpl);
}

template <int LP>
static const void *leaf_fn_m(int mode, bool fuse0, int gf, int cpl) {
  switch (mode) {
    case kModeSum: return leaf_fn_f<LP, kModeSum>(fuse0, gf, cpl);
    case kModePoint: return leaf_fn_f<LP, kModePoint>(fuse0, gf, cpl);
    case kModeStoreY: return leaf_fn_f<LP, kModeStoreY>(fuse0, gf, cpl);
    default:  // the gradient's split level is at most kMaxSplitGrad
      if constexpr (LP <= kMaxSplitGrad) return leaf_fn_f<LP, kModeGrad>(fuse0, gf, cpl);
      else return nullptr;
  }
}

static const void *leaf_fn(const Geometry &G, int mode, int gf, int cpl) {
  if (mode == kModeStoreY) gf = QMC_G_ID;  // the matvec mode does not evaluate g
  if (mode != kModeSum) cpl = 1;
  const bool fuse0 = G.split >= 1 && G.lev[0].tau == 1;
  switch (G.split) {
    case 0: return leaf_fn_m<0>(mode, false, gf, cpl);
    case 1: return leaf_fn_m<1>(mode, fuse0, gf, cpl);
    case 2: return leaf_fn_m<2>(mode, fuse0, gf, cpl);
    case 3: return leaf_fn_m<3>(mode, fuse0, gf, cpl);
    case 4: return leaf_fn_m<4>(mode, fuse0, gf, cpl);
    case 5: return leaf_fn_m<5>(mode, fuse0, gf, cpl);
    default: return leaf_fn_m<6>(mode, fuse0, gf, cpl);
  }
}

static size_t leaf_lds_bytes(const Geometry &G, int mode, int cpl, int nw) {
  size_t floats = (size_t)kTileT *
                  ((size_t)cpl * (G.jlow + kLdsPadRows) + (mode == kModeGrad ? (size_t)nw * G.jlow : 0));
  if (mode == kModeStoreY && G.rec >= 1 && G.rec <= kRecLds) floats += (size_t)nw * kRecSlot;
  return sizeof(float) * floats;
}

// Workgroups of a kernel instance that fit on the current device at once.
int64_t resident_workgroups(const void *fn, int threads, size_t lds) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void *, int, size_t>, int64_t> cache;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  const auto key = std::make_tuple(dev, fn, threads, lds);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  int64_t cap = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds) == hipSuccess &&
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
    cap = (int64_t)per_cu * cus;
  (void)hipGetLastError();  // a failed query only disables the resident-grid choice
  cache[key] = cap;
  return cap;
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
  LaunchTimer tm(mode == kModeGrad ? "leaf_grad" : "leaf", st);
  // several columns per lane exist in the summing mode only; a plan made for
  // another mode would leave column tiles out
  if (lp.cpl != 1 && mode != kModeSum) return hipErrorInvalidValue;
  LeafArgs a{};
  a.t = t;
  a.tct = (int)ceil_div(t, kTileT);
  a.nsub = (int)G.nsub;
  a.rec = (int)G.rec;
  a.gx = lp.gx;
  a.sub_per = (int)(G.nsub / lp.gx);
  a.sub_rem = (int)(G.nsub % lp.gx);
  a.nw = lp.nw;
  a.jlow = G.jlow;
  a.r0 = r0;
  a.nup = G.nup;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    a.up_off[u] = L.uoff * ldu;
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
  a.ldu32 = (uint32_t)ldu;
  a.ldy = o.ldy;
  a.sigma = g_scale(f, mode);
  a.gy = lp.gy;
  a.nparts = lp.gx * lp.gy;
  // largest |x| of a point value after the map (bounds the cos argument)
  // (Phi^-1 of any positive double is below 38.5 in magnitude)
  a.xmax = G.map == QMC_MAP_INVNORM ? 40.0f : 1.0f;
  const dim3 grid(lp.gx, lp.gy, nr), block(64 * lp.nw);
  if (mode == kModeGrad && grad_reg_ok(G)) {
    if (lp.nw > 8) return hipErrorInvalidValue;  // the kernel keeps one sum per wave
    const size_t lds = sizeof(float) * kTileT * (size_t)(G.jlow + kLdsPadRows);
    void *args[] = {&a, (void *)&tables, (void *)&U, (void *)&A, (void *)&o.partial, (void *)&o.dApart,
                    (void *)&o.Sroot, (void *)&o.hd};
    const hipError_t e = hipLaunchKernel(grad_fn(G, f.g, o.hd != nullptr), grid, block, args, lds, st);
    if (e != hipSuccess) return e;
    return hipGetLastError();
  }
  const size_t lds = leaf_lds_bytes(G, mode, lp.cpl, lp.nw);
  const void *fn = leaf_fn(G, mode, f.g, lp.cpl);
  if (!fn) return hipErrorInvalidDeviceFunction;
  void *args[] = {&a, (void *)&tables, (void *)&U, (void *)&A, (void *)&o.partial, (void *)&o.ppart,
                  (void *)&o.Y, (void *)&o.dApart, (void *)&o.Sroot, (void *)&o.hd};
  const hipError_t e = hipLaunchKernel(fn, grid, block, args, lds, st);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace qmc
