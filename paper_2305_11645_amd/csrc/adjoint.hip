// Gradient mode of the fused leaf pass, register form: the transposed
// recursion of the lower levels with one accumulator per lower coordinate and
// column in registers.
#include <cstdlib>

#include "leaf_common.h"

namespace qmc {

// The gradient mode for lower levels with tau_I <= 2^I coordinates (I < L'),
// which is every w with at most 2^I coordinates of reduction index I (w_j =
// floor(c log2(j+1)) with c >= 1 among them).  Each lane keeps one FP32
// accumulator per lower coordinate and its column in registers (2^{L'} - 1
// of them, indexed at compile time by level and position in the level), so
// the transposed recursion needs no LDS traffic per subtree, and a workgroup
// only stages its rows of A: four waves per workgroup and, with L' <= 5 (at
// most 31 accumulators and 32 leaves per lane), six waves per SIMD for cos and
// y (80 registers, 12 bytes spilled for cos: measured faster than five) and
// five for exp, whose leaf block holds more values (six would spill 36 bytes).
// Per subtree: the forward descent of the summing mode to the level-1 nodes,
// then level 0 fused with the integrand (leaves c and c + 2^{L'-1} of node c:
// their sensitivities G'_k, the level-0 product, and their sum as the node's
// S_1), then each level L = 1 .. L'-1 in turn: d_j += sum_c X~_L[c][j] S_L[c]
// for j in G_L, and S_{L+1}[c] = S_L[c] + S_L[c + half] (the transpose of the
// tiling step).  S_{L'} (the subtree's total) goes to the subtree-root array.
// At the end the workgroup's waves add their accumulators in wave order in
// LDS (deterministic) and write one partial per workgroup.

// Adjoint of level L: d[jj] += sum_c x[jj NC + c] S[c] for jj < tau (at most
// 2^L), then the fold of the NC node sums into their NC / 2 parents.  The point
// values of up to kBatchFloats nodes x coordinates are read together (the last
// batch may read up to 31 floats past the level's block: the tables are padded).
template <int LP, int L>
__device__ __forceinline__ void ascend_reg(float (&S)[1 << LP], const float *__restrict__ x, int tau,
                                           float (&d)[1 << L]) {
  constexpr int NC = 1 << (LP - L);
  constexpr int TM = 1 << L;
  constexpr int BF = kBatchFloats / 2;  // fewer scalars in flight than the descent (16)
  constexpr int B0 = BF / NC > 0 ? BF / NC : 1;
  constexpr int B = B0 < TM ? B0 : TM;
  // independent partial sums per coordinate: the level with the most nodes has
  // at most two coordinates, so it splits its chain in two; elsewhere the
  // coordinates' chains are independent of one another
  constexpr int NP = NC >= 32 ? 2 : 1;
#pragma unroll
  for (int jb = 0; jb < TM; jb += B) {
    if (jb >= tau) break;
    float xs[B * NC];
#pragma unroll
    for (int i = 0; i < B * NC; ++i) xs[i] = x[jb * NC + i];
    keep_scalar(xs);
#pragma unroll
    for (int i = 0; i < B; ++i) {
      if (jb + i < tau) {
        if constexpr (NP == 1) {
#pragma unroll
          for (int c = 0; c < NC; ++c) d[jb + i] = fmaf(xs[i * NC + c], S[c], d[jb + i]);
        } else {
          float e[NP];
#pragma unroll
          for (int p = 0; p < NP; ++p) e[p] = xs[i * NC + p] * S[p];
#pragma unroll
          for (int c = NP; c < NC; ++c) e[c % NP] = fmaf(xs[i * NC + c], S[c], e[c % NP]);
          float t = e[0];
#pragma unroll
          for (int p = 1; p < NP; ++p) t += e[p];
          d[jb + i] += t;
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC / 2; ++c) S[c] += S[c + NC / 2];
}

// Level 0 (one coordinate, row 0 of A) fused with the integrand.  y[c] holds
// the level-1 node c; leaves c and c + H0 read their level-0 values from x0.
// Afterwards y[c] holds S_1[c], d0 has the level-0 product added, and s the
// FP32 sum of g over the leaves (separable h only).
template <int LP, int GF, bool NEAR, bool HD>
__device__ __forceinline__ void leaf_grad_block(float (&y)[1 << LP], const float *__restrict__ x0,
                                                const float *__restrict__ hk, float a0, float &d0, float &s) {
  constexpr int H0 = 1 << (LP - 1);
  constexpr int HB = H0 < 8 ? H0 : 8;  // 2 HB point values (and 2 HB factors h') per batch
  float da = 0.f, db = 0.f, sa = 0.f, sb = 0.f;
#pragma unroll
  for (int h = 0; h < H0 / HB; ++h) {
    float xa[HB], xb[HB], fa[HB], fb[HB];
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      xa[i] = x0[h * HB + i];
      xb[i] = x0[H0 + h * HB + i];
    }
    keep_scalar(xa);
    keep_scalar(xb);
    if (HD) {
#pragma unroll
      for (int i = 0; i < HB; ++i) {
        fa[i] = hk[h * HB + i];
        fb[i] = hk[H0 + h * HB + i];
      }
      keep_scalar(fa);
      keep_scalar(fb);
    }
#pragma unroll
    for (int i = 0; i < HB; ++i) {
      const int c = h * HB + i;
      const float ya = fmaf(xa[i], a0, y[c]);
      const float yb = fmaf(xb[i], a0, y[c]);
      if (!HD) {
        sa += NEAR ? g_val_near<GF>(ya) : g_val<GF>(ya);
        sb += NEAR ? g_val_near<GF>(yb) : g_val<GF>(yb);
      }
      float Sa = g_der_unit<GF, NEAR>(ya), Sb = g_der_unit<GF, NEAR>(yb);
      if (HD) {
        Sa *= fa[i];
        Sb *= fb[i];
      }
      da = fmaf(xa[i], Sa, da);
      db = fmaf(xb[i], Sb, db);
      y[c] = Sa + Sb;
    }
  }
  d0 += da + db;
  s += sa + sb;
}

template <int LP, int GF, bool HD>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(GF == QMC_G_EXP ? 5 : 6))) void grad_kernel(
    LeafArgs a, const float *__restrict__ tables, const float *__restrict__ U, const float *__restrict__ A,
    double *__restrict__ partial, float *__restrict__ dApart, float *__restrict__ Sroot,
    const float *__restrict__ hd) {
  static_assert(LP >= 1 && LP <= kMaxSplitGrad, "register adjoint needs 1 <= L' <= kMaxSplitGrad");
  constexpr int NL = 1 << LP;
  extern __shared__ float smem[];
  __shared__ double red[8];
  __shared__ int arrived;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int bx = blockIdx.x, ct = blockIdx.y, rl = blockIdx.z;
  const int col = ct * kTileT + lane;
  const bool live = col < a.t;
  const int jlow = a.jlow;
  if (tid == 0) arrived = 0;

  // rows 0 .. jlow-1 of sigma A for the column tile, then kLdsPadRows zero rows
  float *Alds = smem;
  const int stage_total = (jlow + kLdsPadRows) * kTileT;
  for (int e0 = 0; e0 < stage_total; e0 += kStagePerThread * (int)blockDim.x) {
    float v[kStagePerThread];
#pragma unroll
    for (int k = 0; k < kStagePerThread; ++k) {
      const int e = e0 + k * (int)blockDim.x + tid;
      const int jr = e / kTileT, cl = ct * kTileT + (e % kTileT);
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
  __syncthreads();
  const float *Al = Alds + lane;

  bool near = false;
  if (GF == QMC_G_COS) {
    float bound = 0.f;
    for (int j = 0; j < jlow; ++j) bound += fabsf(Al[j * kTileT]);
    near = __all(bound * a.xmax < 250.0f);
  }

  const float *tab = tables + (int64_t)rl * a.tstride;
  const float *Ub = U + (int64_t)rl * a.ustride;
  float d0 = 0.f, d1[2], d2[4], d3[8], d4[16];
#pragma unroll
  for (int i = 0; i < 2; ++i) d1[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 4; ++i) d2[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 8; ++i) d3[i] = 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) d4[i] = 0.f;
  double acc = 0.0;

  const int first = bx * a.sub_per + min(bx, a.sub_rem);
  const int last = first + a.sub_per + (bx < a.sub_rem ? 1 : 0);
  for (int rho = first + w; rho < last; rho += a.nw) {
    const float *rec = tab + (int64_t)rho * a.rec;
    // subtree root: the upper levels' rows, kRootBatch at a time
    float root = 0.f;
#pragma unroll 1
    for (int u0 = 0; u0 < a.nup; u0 += kRootBatch) {
      float rv[kRootBatch];
#pragma unroll
      for (int i = 0; i < kRootBatch; ++i) {
        const float *row = Ub + a.up_off[u0 + i] + (uint64_t)(uint32_t)(rho & a.up_mask[u0 + i]) * a.ldu32;
        rv[i] = row[col];
      }
#pragma unroll
      for (int i = 0; i < kRootBatch; ++i) asm volatile("" ::"v"(rv[i]));
#pragma unroll
      for (int i = 0; i < kRootBatch; ++i)
        if (u0 + i < a.nup) root += rv[i];
    }
    if (GF == QMC_G_COS) root = __builtin_amdgcn_fractf(root);

    uint64_t taus = a.taus;
    asm volatile("" : "+s"(taus));
    int xo = 0, j0 = jlow;
    float y[1][NL];
    y[0][0] = root;
    descend_lean<LP, LP - 1, 1, 1>(y, rec, xo, j0, taus, Al);
    const float a0 = Al[0];  // level 0 is row 0
    float s = 0.f;
    const float *hk = HD ? hd + ((int64_t)rl * a.nsub + rho) * NL : nullptr;
    if (near) leaf_grad_block<LP, GF, true, HD>(y[0], rec + xo, hk, a0, d0, s);
    else leaf_grad_block<LP, GF, false, HD>(y[0], rec + xo, hk, a0, d0, s);
    // levels 1 .. L'-1: level L's block precedes level L-1's in the record
    int xl = xo;
    if constexpr (LP > 1) {
      const int tau = (int)((taus >> 8) & 0xff);
      xl -= tau * (NL >> 1);
      ascend_reg<LP, 1>(y[0], rec + xl, tau, d1);
    }
    if constexpr (LP > 2) {
      const int tau = (int)((taus >> 16) & 0xff);
      xl -= tau * (NL >> 2);
      ascend_reg<LP, 2>(y[0], rec + xl, tau, d2);
    }
    if constexpr (LP > 3) {
      const int tau = (int)((taus >> 24) & 0xff);
      xl -= tau * (NL >> 3);
      ascend_reg<LP, 3>(y[0], rec + xl, tau, d3);
    }
    if constexpr (LP > 4) {
      const int tau = (int)((taus >> 32) & 0xff);
      xl -= tau * (NL >> 4);
      ascend_reg<LP, 4>(y[0], rec + xl, tau, d4);
    }
    if (live) {
      Sroot[((int64_t)rl * 2 * a.nsub + rho) * a.ldu + col] = y[0][0];
      if (!HD) acc += (double)s;
    }
  }

  if (!HD) {  // one FP64 partial of sum g per workgroup (waves added in wave order)
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

  // the waves' accumulators, added in wave order in LDS (the rows of A are no
  // longer needed), then one partial per workgroup
  __syncthreads();
  float *buf = smem;
  for (int e = tid; e < jlow * kTileT; e += blockDim.x) buf[e] = 0.f;
  const uint64_t taus = a.taus;
  for (int q = 0; q < a.nw; ++q) {
    __syncthreads();
    if (w == q) {
      buf[lane] += d0;
      int jj0 = (int)(taus & 0xff);
      auto put = [&](auto &d, int L) {
        const int tau = (int)((taus >> (8 * L)) & 0xff);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(d) / sizeof(float)); ++i)
          if (i < tau) buf[(jj0 + i) * kTileT + lane] += d[i];
        jj0 += tau;
      };
      if constexpr (LP > 1) put(d1, 1);
      if constexpr (LP > 2) put(d2, 2);
      if constexpr (LP > 3) put(d3, 3);
      if constexpr (LP > 4) put(d4, 4);
    }
  }
  __syncthreads();
  const int64_t blk = (int64_t)jlow * kTileT;
  for (int e = tid; e < blk; e += blockDim.x)
    dApart[(((int64_t)rl * a.gx + bx) * a.tct + ct) * blk + e] = buf[e];
}

// Whether the register form of the adjoint applies: 1 <= L' and tau_I <= 2^I
// for every lower level.
bool grad_reg_ok(const Geometry &G) {
  if (G.split < 1 || G.split > kMaxSplitGrad) return false;
  for (int I = 0; I < G.split; ++I)
    if (G.lev[I].tau > (1 << I)) return false;
  if (getenv("QMC_GRAD_GENERIC")) return false;  // measurement switch: the LDS form
  return true;
}

template <int LP>
static const void *grad_fn_lp(int gf, bool hd) {
#define QMC_GRAD_FN(GF) \
  (hd ? reinterpret_cast<const void *>(&grad_kernel<LP, GF, true>) : reinterpret_cast<const void *>(&grad_kernel<LP, GF, false>))
  if (gf == QMC_G_COS) return QMC_GRAD_FN(QMC_G_COS);
  if (gf == QMC_G_EXP) return QMC_GRAD_FN(QMC_G_EXP);
  return QMC_GRAD_FN(QMC_G_ID);
#undef QMC_GRAD_FN
}

const void *grad_fn(const Geometry &G, int gf, bool hd) {
  switch (G.split) {
    case 1: return grad_fn_lp<1>(gf, hd);
    case 2: return grad_fn_lp<2>(gf, hd);
    case 3: return grad_fn_lp<3>(gf, hd);
    case 4: return grad_fn_lp<4>(gf, hd);
    default: return grad_fn_lp<5>(gf, hd);  // the gradient's split level is at most kMaxSplitGrad
  }
}


}  // namespace qmc
