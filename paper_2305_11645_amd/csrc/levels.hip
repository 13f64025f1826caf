// Grouped products of the upper levels on the matrix cores.
//
// Forward (Algorithm 2, the product X~_I A~_I of one level):
//     U_I = X~_I A_I,      X~_I: n_I x tau_I point table, A_I: rows G_I of A.
// Adjoint (transpose of the same step):
//     dA_I = X~_I^T S_I,   S_I: n_I x t sums of dQ/dy over the residue classes.
// All levels and all randomisations go in one launch; every workgroup owns
// one 64 x 64 output tile of one (level, shift, K-chunk).  The adjoint
// contracts over n_I rows, so it is split into K-chunks of at most 1024 whose
// FP32 partials are combined later in FP64.
//
// Precision:
//   FP32        v_mfma_f32_32x32x2_f32, FP32 accumulation.
//   SPLIT_BF16  each FP32 operand x = hi + lo with hi = bf16(x),
//               lo = bf16(x - hi); hi*hi on one accumulator, hi*lo + lo*hi on
//               a second, v_mfma_f32_32x32x16_bf16, summed at the end.
//
// MFMA operand layouts (wave64, one 32 x 32 block):
//   32x32x2 f32:  A: lane l holds A[l%32][l/32]; B: B[l/32][l%32];
//                 D: acc[v] = D[8(v/4) + 4(l/32) + v%4][l%32].
//   32x32x16 bf16: A: lane l holds A[l%32][8(l/32) + 0..7]; B: B[8(l/32)+0..7][l%32];
//                 D as above.
#include "qmc_internal.h"

namespace qmc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 16;
constexpr int APAD = BK + 1;   // As row stride (odd: conflict-free column reads)
constexpr int BPAD = BN + 4;

struct GemmProb {
  int32_t M, N, K;
  int32_t tiles_m, tiles_n, kchunks, kchunk;
  int32_t tile0;          // first flat tile of this problem
  int64_t a_off, a_si, a_sk;  // A(i,k) = Abase[a_off + i*a_si + k*a_sk]
  int64_t b_off;              // B(k,j) = Bbase[b_off + k*ldb + j]
  int64_t c_off, c_chunk;     // C(i,j) = Cbase[c_off + chunk*c_chunk + i*ldc + j]
};

struct GemmArgs {
  int32_t nprob, total_tiles;
  float oscale;               // C = oscale * A B
  int64_t a_rs, b_rs, c_rs;   // per-shift strides of the three bases
  int64_t ldb, ldc;
  GemmProb p[kMaxLevels];
};

template <bool TA, int PREC>
__global__ __launch_bounds__(256) void levels_gemm(GemmArgs g, const float *__restrict__ Abase,
                                                   const float *__restrict__ Bbase,
                                                   float *__restrict__ Cbase) {
  __shared__ float As[BM * APAD];
  __shared__ float Bs[BK * BPAD];
  const int r = blockIdx.y;
  int tile = blockIdx.x;
  int pi = 0;
  for (int q = 1; q < g.nprob; ++q)
    if (tile >= g.p[q].tile0) pi = q;
  const GemmProb &P = g.p[pi];
  tile -= P.tile0;
  const int chunk = tile % P.kchunks;
  tile /= P.kchunks;
  const int tn = tile % P.tiles_n;
  const int tm = tile / P.tiles_n;
  const int i0 = tm * BM, j0 = tn * BN;
  const int kbeg = chunk * P.kchunk;
  const int kend = min(P.K, kbeg + P.kchunk);

  const float *Ab = Abase + r * g.a_rs + P.a_off;
  const float *Bb = Bbase + r * g.b_rs + P.b_off;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 32, wc = (w & 1) * 32;

  f32x16 acc = {0};
  f32x16 acc2 = {0};

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    // stage A (BM x BK) and B (BK x BN), zero outside the problem
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      int i, k;
      if (TA) { k = e / BM; i = e % BM; } else { i = e / BK; k = e % BK; }
      const int gi = i0 + i, gk = k0 + k;
      float v = 0.f;
      if (gi < P.M && gk < kend) v = Ab[gi * P.a_si + gk * P.a_sk];
      As[i * APAD + k] = v;
      const int kb = e / BN, jb = e % BN;
      const int gkb = k0 + kb, gj = j0 + jb;
      float u = 0.f;
      if (gkb < kend && gj < P.N) u = Bb[(int64_t)gkb * g.ldb + gj];
      Bs[kb * BPAD + jb] = u;
    }
    __syncthreads();
    if (PREC == QMC_FP32) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        const float a = As[(wr + (lane & 31)) * APAD + kk + (lane >> 5)];
        const float b = Bs[(kk + (lane >> 5)) * BPAD + wc + (lane & 31)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
    } else {
      bf16x8 ah, al, bh, bl;
      const int kq = 8 * (lane >> 5);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const float a = As[(wr + (lane & 31)) * APAD + kq + q];
        const __bf16 a_hi = (__bf16)a;
        ah[q] = a_hi;
        al[q] = (__bf16)(a - (float)a_hi);
        const float b = Bs[(kq + q) * BPAD + wc + (lane & 31)];
        const __bf16 b_hi = (__bf16)b;
        bh[q] = b_hi;
        bl[q] = (__bf16)(b - (float)b_hi);
      }
      acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc2, 0, 0, 0);
      acc2 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc2, 0, 0, 0);
    }
    __syncthreads();
  }

  float *Cb = Cbase + r * g.c_rs + P.c_off + (int64_t)chunk * P.c_chunk;
  const int col = j0 + wc + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = i0 + wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (row < P.M && col < P.N) {
      float out = acc[v];
      if (PREC != QMC_FP32) out += acc2[v];
      Cb[(int64_t)row * g.ldc + col] = g.oscale * out;
    }
  }
}

template <bool TA>
static hipError_t run_gemm(const GemmArgs &a, int prec, int nr, const float *A, const float *B,
                           float *C, hipStream_t st) {
  if (a.total_tiles == 0 || nr == 0) return hipSuccess;
  dim3 grid(a.total_tiles, nr);
  if (prec == QMC_FP32)
    hipLaunchKernelGGL((levels_gemm<TA, QMC_FP32>), grid, dim3(256), 0, st, a, A, B, C);
  else
    hipLaunchKernelGGL((levels_gemm<TA, QMC_SPLIT_BF16X3>), grid, dim3(256), 0, st, a, A, B, C);
  return hipGetLastError();
}

hipError_t launch_levels(const Geometry &G, int prec, const float *tables, int nr, const float *A,
                         int t, int64_t lda, float *U, int64_t ldu, float oscale, hipStream_t st) {
  LaunchTimer tm("levels", st);
  GemmArgs a = {};
  a.oscale = oscale;
  a.a_rs = G.table_total;
  a.b_rs = 0;
  a.c_rs = G.urows * ldu;
  a.ldb = lda;
  a.ldc = ldu;
  int tiles = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    GemmProb &P = a.p[a.nprob++];
    P.M = 1 << L.nb;
    P.N = t;
    P.K = L.tau;
    P.tiles_m = (int)ceil_div(P.M, BM);
    P.tiles_n = (int)ceil_div(t, BN);
    P.kchunk = (int)round_up(P.K, BK);
    P.kchunks = 1;
    P.tile0 = tiles;
    P.a_off = G.lower_total + L.off;
    P.a_si = L.tau;
    P.a_sk = 1;
    P.b_off = (int64_t)L.j0 * lda;
    P.c_off = L.uoff * ldu;
    P.c_chunk = 0;
    tiles += P.tiles_m * P.tiles_n;
  }
  a.total_tiles = tiles;
  return run_gemm<false>(a, prec, nr, tables, A, U, st);
}

// Adjoint partial layout: for each upper level (in order) kchunks blocks of
// tau_I x ldu floats, per shift.
static int adj_chunk(int64_t K) { return (int)(K < 1024 ? round_up(K, BK) : 1024); }

int64_t levels_adj_part_floats(const Geometry &G, int t, int64_t ldu) {
  (void)t;
  int64_t n = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    const int64_t K = int64_t(1) << L.nb;
    n += ceil_div(K, adj_chunk(K)) * L.tau * ldu;
  }
  return n;
}

hipError_t launch_levels_adj(const Geometry &G, int prec, const float *tables, int nr,
                             const float *S, int t, int64_t ldu, float *part, hipStream_t st) {
  LaunchTimer tm("levels_adj", st);
  GemmArgs a = {};
  a.oscale = 1.0f;
  a.a_rs = G.table_total;
  a.b_rs = (2 * G.nsub) * ldu;  // S pyramid rows per shift
  a.c_rs = levels_adj_part_floats(G, t, ldu);
  a.ldb = ldu;
  a.ldc = ldu;
  int tiles = 0;
  int64_t poff = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    GemmProb &P = a.p[a.nprob++];
    P.M = L.tau;
    P.N = t;
    P.K = 1 << L.nb;
    P.kchunk = adj_chunk(P.K);
    P.kchunks = (int)ceil_div(P.K, P.kchunk);
    P.tiles_m = (int)ceil_div(P.M, BM);
    P.tiles_n = (int)ceil_div(t, BN);
    P.tile0 = tiles;
    P.a_off = G.lower_total + L.off;
    P.a_si = 1;
    P.a_sk = L.tau;
    // S_I rows start after the levels split .. I-1 of the pyramid
    int64_t soff = 0;
    for (int I = G.split; I < G.up[u]; ++I) soff += int64_t(1) << (G.m - I);
    P.b_off = soff * ldu;
    P.c_off = poff;
    P.c_chunk = (int64_t)L.tau * ldu;
    poff += (int64_t)P.kchunks * L.tau * ldu;
    tiles += P.tiles_m * P.tiles_n * P.kchunks;
  }
  a.total_tiles = tiles;
  return run_gemm<true>(a, prec, nr, tables, S, part, st);
}

}  // namespace qmc
