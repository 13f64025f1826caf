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
#include <algorithm>

#include "qmc_internal.h"

namespace qmc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int BM = 64, BN = 64, BK = 32;
constexpr int APAD = BK + 1;   // As row stride (odd: conflict-free column reads)
constexpr int BPAD = BN + 4;
constexpr int PER_T = BM * BK / 256;  // elements of each operand tile per thread (8)

struct GemmProb {
  int32_t M, N, K;
  int32_t tiles_m, tiles_n, kchunks, kchunk;
  int32_t tile0;          // first flat tile of this problem
  int64_t a_off, a_si, a_sk;  // A(i,k) = Abase[a_off + i*a_si + k*a_sk]
  int64_t b_off;              // B(k,j) = Bbase[b_off + k*ldb + j]
  int64_t c_off, c_chunk;     // C(i,j) = Cbase[c_off + chunk*c_chunk + i*ldc + j]
};

constexpr int kMaxGemmProbs = 32;  // >= kMaxLevels: the tile table is read in whole batches

struct GemmArgs {
  int32_t tile0[kMaxGemmProbs];  // first flat tile of each problem (unused entries: INT_MAX)
  int32_t nprob, total_tiles;
  float oscale;               // C = oscale * A B
  int64_t a_rs, b_rs, c_rs;   // per-shift strides of the three bases
  int64_t ldb, ldc;
  GemmProb p[kMaxLevels];
};
static_assert(kMaxGemmProbs >= kMaxLevels, "tile table too short");

static void finish_tile_table(GemmArgs &a) {
  for (int q = 0; q < kMaxGemmProbs; ++q) a.tile0[q] = q < a.nprob ? a.p[q].tile0 : 0x7fffffff;
}

// Operand tile coordinates of element q of this thread: A as (i, k), B as (k, j).
template <bool TA>
__device__ __forceinline__ void a_coord(int e, int &i, int &k) {
  if (TA) { k = e / BM; i = e % BM; } else { i = e / BK; k = e % BK; }
}

// Loads the A and B tiles at K offset k0.  Ab and Bb already point at this
// thread's first element (row i0 + i, column k of A; row k, column j0 + j of B);
// element q of the thread lies q * (256 / BK) rows further for A (BK/256 * q for
// TA) and q * (256 / BN) rows further for B.
template <bool TA>
__device__ __forceinline__ void load_tile(const float *__restrict__ Ab, const float *__restrict__ Bb,
                                          int64_t a_step, int64_t b_step, int a_rows_left,
                                          int b_k0, int k0, int kend, bool a_col_ok, bool b_col_ok,
                                          int a_k, float (&ra)[PER_T], float (&rb)[PER_T]) {
#pragma unroll
  for (int q = 0; q < PER_T; ++q) {
    // A element q: TA: k advances by 256/BM per q; else the row advances by 256/BK
    bool aok;
    if (TA) aok = a_col_ok && (k0 + a_k + q * (256 / BM)) < kend;
    else aok = (q * (256 / BK)) < a_rows_left && (k0 + a_k) < kend;
    ra[q] = aok ? Ab[q * a_step] : 0.f;
    const bool bok = b_col_ok && (k0 + b_k0 + q * (256 / BN)) < kend;
    rb[q] = bok ? Bb[q * b_step] : 0.f;
  }
}

template <bool TA, int PREC>
__global__ __launch_bounds__(256) void levels_gemm(GemmArgs g, const float *__restrict__ Abase,
                                                   const float *__restrict__ Bbase,
                                                   float *__restrict__ Cbase) {
  __shared__ float As[BM * APAD];
  __shared__ float Bs[BK * BPAD];
  const int r = blockIdx.y;
  int tile = blockIdx.x;
  // problem of this tile: the tile table is contiguous, so its scalar loads
  // are issued together (one round trip) and scanned in registers
  int pi = 0;
#pragma unroll
  for (int q = 1; q < kMaxGemmProbs; ++q)
    if (tile >= g.tile0[q]) pi = q;
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
  // this thread's element 0 of each operand tile
  int ai, ak;
  a_coord<TA>(tid, ai, ak);
  const int bk = tid / BN, bj = tid % BN;
  const bool a_col_ok = TA ? (i0 + ai) < P.M : true;
  const int a_rows_left = TA ? 0 : P.M - (i0 + ai);
  const bool b_col_ok = (j0 + bj) < P.N;
  // per-q steps: A rows (or k) and B rows advance with q
  const int64_t a_step = TA ? (int64_t)(256 / BM) * P.a_sk : (int64_t)(256 / BK) * P.a_si;
  const int64_t b_step = (int64_t)(256 / BN) * g.ldb;
  const float *Ap = Ab + (int64_t)(i0 + ai) * P.a_si + (int64_t)(kbeg + ak) * P.a_sk;
  const float *Bp = Bb + (int64_t)(kbeg + bk) * g.ldb + (j0 + bj);
  const int64_t a_kstep = (int64_t)BK * P.a_sk, b_kstep = (int64_t)BK * g.ldb;
  float ra[PER_T], rb[PER_T];
  load_tile<TA>(Ap, Bp, a_step, b_step, a_rows_left, bk, kbeg, kend, a_col_ok, b_col_ok, ak, ra, rb);

  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();  // the previous tile has been consumed
#pragma unroll
    for (int q = 0; q < PER_T; ++q) {
      const int e = tid + 256 * q;
      int i, k;
      a_coord<TA>(e, i, k);
      As[i * APAD + k] = ra[q];
      Bs[(e / BN) * BPAD + (e % BN)] = rb[q];
    }
    __syncthreads();
    // the next tile's loads are in flight while this one is multiplied
    if (k0 + BK < kend) {
      Ap += a_kstep;
      Bp += b_kstep;
      load_tile<TA>(Ap, Bp, a_step, b_step, a_rows_left, bk, k0 + BK, kend, a_col_ok, b_col_ok, ak,
                    ra, rb);
    }
    if (PREC == QMC_FP32) {
#pragma unroll
      for (int kk = 0; kk < BK; kk += 2) {
        const float a = As[(wr + (lane & 31)) * APAD + kk + (lane >> 5)];
        const float b = Bs[(kk + (lane >> 5)) * BPAD + wc + (lane & 31)];
        acc = __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, acc, 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kc = 0; kc < BK; kc += 16) {
        bf16x8 ah, al, bh, bl;
        const int kq = kc + 8 * (lane >> 5);
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
    }
  }

  float *Cb = Cbase + r * g.c_rs + P.c_off + (int64_t)chunk * P.c_chunk;
  const int col = j0 + wc + (lane & 31);
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int row = i0 + wr + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
    if (row < P.M && col < P.N) {
      float out = acc[v];
      if (PREC != QMC_FP32) out += acc2[v];
      // streamed past the L2 (read next by another kernel, on other XCDs)
      __builtin_nontemporal_store(g.oscale * out, &Cb[(int64_t)row * g.ldc + col]);
    }
  }
}

// ------------------------------------------------------------------ split BF16, operands split once
// The forward level products in split BF16 with both operands split into
// (hi, lo) once per call instead of inside the product loop:
//   split_kernel   the upper-level tables X~_I (per randomisation, rows padded
//                  to a multiple of 8 values) and the rows of A of the upper
//                  levels, transposed so that K is contiguous for both operands
//                  (A^T[col][koff_I + k], koff_I a multiple of 8);
//   gemm_bf16x3    128 x 128 output tiles, four waves of 64 x 64 (four 32 x 32
//                  MFMA blocks each), K-steps of 16 loaded as 16-byte chunks,
//                  two LDS buffers; per block and step lo*hi, hi*lo, hi*hi on
//                  v_mfma_f32_32x32x16_bf16 into one FP32 accumulator.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));

constexpr int SBM = 128, SBN = 128, SBK = 16;
constexpr int SRS = SBK + 8;  // LDS row stride in bf16: 48 bytes, so eight lanes' 16-byte reads hit distinct banks

struct SplitLayout {
  int64_t up_pad;                  // bf16 of one randomisation's split upper tables (hi or lo)
  int64_t kpad;                    // padded upper coordinates: row stride of the split A^T
  int64_t tab_off[kMaxLevels];     // per upper level u: offset of its split table (bf16)
  int32_t koff[kMaxLevels];        // per upper level u: first K index in the split A^T
  int32_t taup[kMaxLevels];        // per upper level u: tau_I rounded up to 8
};

static SplitLayout split_layout(const Geometry &G) {
  SplitLayout L{};
  int64_t off = 0;
  int32_t k = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &lv = G.lev[G.up[u]];
    L.taup[u] = (int32_t)round_up(lv.tau, 8);
    L.tab_off[u] = off;
    L.koff[u] = k;
    off += (int64_t(1) << lv.nb) * L.taup[u];
    k += L.taup[u];
  }
  L.up_pad = off;
  L.kpad = k;
  return L;
}

int64_t levels_split_bytes(const Geometry &G, int nr, int t) {
  const SplitLayout L = split_layout(G);
  return 2 * 2 * ((int64_t)nr * L.up_pad + L.kpad * (int64_t)t);  // hi and lo, 2 bytes each
}

struct SplitArgs {
  Geometry G;
  SplitLayout L;
  int32_t nr, t;
  int64_t lda;
};

// Elements: [nr][up_pad] table values, then [t][kpad] of A^T.  Padding reads 0.
__global__ __launch_bounds__(256) void split_kernel(SplitArgs a, const float *__restrict__ tables,
                                                    const float *__restrict__ A, __bf16 *__restrict__ hi,
                                                    __bf16 *__restrict__ lo) {
  const Geometry &G = a.G;
  const int64_t ntab = (int64_t)a.nr * a.L.up_pad, total = ntab + (int64_t)a.t * a.L.kpad;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    float x = 0.f;
    if (e < ntab) {
      const int64_t r = e / a.L.up_pad, o = e - r * a.L.up_pad;
      int u = 0;
      while (u + 1 < G.nup && a.L.tab_off[u + 1] <= o) ++u;
      const Level &lv = G.lev[G.up[u]];
      const int64_t q = o - a.L.tab_off[u], row = q / a.L.taup[u], k = q - row * a.L.taup[u];
      if (k < lv.tau) x = tables[r * G.table_total + G.lower_total + lv.off + row * lv.tau + k];
    } else {
      const int64_t q = e - ntab, col = q / a.L.kpad, kk = q - col * a.L.kpad;
      int u = 0;
      while (u + 1 < G.nup && a.L.koff[u + 1] <= kk) ++u;
      const Level &lv = G.lev[G.up[u]];
      const int64_t k = kk - a.L.koff[u];
      if (k < lv.tau) x = A[(int64_t)(lv.j0 + k) * a.lda + col];
    }
    const __bf16 h = (__bf16)x;
    hi[e] = h;
    lo[e] = (__bf16)(x - (float)h);
  }
}

struct SplitGemmArgs {
  int32_t tile0[kMaxGemmProbs];
  int32_t nprob;
  float oscale;
  int64_t a_rs, c_rs, ldc, kpad;
  struct {
    int32_t M, K, tiles_n;
    int64_t a_off, b_off, c_off;
  } p[kMaxLevels];
};

__global__ __launch_bounds__(256) void gemm_bf16x3(SplitGemmArgs g, int N, const __bf16 *__restrict__ Ahi,
                                                   const __bf16 *__restrict__ Alo,
                                                   const __bf16 *__restrict__ Bhi,
                                                   const __bf16 *__restrict__ Blo, float *__restrict__ Cbase) {
  __shared__ __attribute__((aligned(16))) __bf16 As[2][2][SBM * SRS];  // [buffer][hi, lo][row][k]
  __shared__ __attribute__((aligned(16))) __bf16 Bs[2][2][SBN * SRS];  // [buffer][hi, lo][col][k]
  const int r = blockIdx.y;
  int tile = blockIdx.x;
  int pi = 0;
#pragma unroll
  for (int q = 1; q < kMaxGemmProbs; ++q)
    if (tile >= g.tile0[q]) pi = q;
  const auto &P = g.p[pi];
  tile -= g.tile0[pi];
  const int tn = tile % P.tiles_n, tm = tile / P.tiles_n;
  const int i0 = tm * SBM, j0 = tn * SBN;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 64;
  // loader: row (A) or column (B) ld = tid / 2, 8 K-values at kh = 8 (tid % 2)
  const int ld = tid >> 1, kh = 8 * (tid & 1);
  const int64_t aoff = r * g.a_rs + P.a_off;
  const bool arow_ok = i0 + ld < P.M, bcol_ok = j0 + ld < N;
  const __bf16 *ah_p = Ahi + aoff + (int64_t)(arow_ok ? i0 + ld : 0) * P.K + kh;
  const __bf16 *al_p = Alo + aoff + (int64_t)(arow_ok ? i0 + ld : 0) * P.K + kh;
  const __bf16 *bh_p = Bhi + P.b_off + (int64_t)(bcol_ok ? j0 + ld : 0) * g.kpad + kh;
  const __bf16 *bl_p = Blo + P.b_off + (int64_t)(bcol_ok ? j0 + ld : 0) * g.kpad + kh;
  bf16x8v ra[2], rb[2];
  const bf16x8v zero = {};
  auto load = [&](int k0) {
    const bool kok = k0 + kh < P.K;  // K is a multiple of 8: a chunk is whole or absent
    ra[0] = arow_ok && kok ? *reinterpret_cast<const bf16x8v *>(ah_p + k0) : zero;
    ra[1] = arow_ok && kok ? *reinterpret_cast<const bf16x8v *>(al_p + k0) : zero;
    rb[0] = bcol_ok && kok ? *reinterpret_cast<const bf16x8v *>(bh_p + k0) : zero;
    rb[1] = bcol_ok && kok ? *reinterpret_cast<const bf16x8v *>(bl_p + k0) : zero;
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<bf16x8v *>(&As[buf][h][ld * SRS + kh]) = ra[h];
      *reinterpret_cast<bf16x8v *>(&Bs[buf][h][ld * SRS + kh]) = rb[h];
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x16{0};
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  const int ko = 8 * (lane >> 5);  // this lane's K-values of a step: ko .. ko + 7
  for (int k0 = 0; k0 < P.K; k0 += SBK) {
    const bool more = k0 + SBK < P.K;
    if (more) load(k0 + SBK);
    bf16x8v xa[2][2], xb[2][2];  // [block][hi, lo]
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        xa[i][h] = *reinterpret_cast<const bf16x8v *>(&As[cur][h][(wr + 32 * i + (lane & 31)) * SRS + ko]);
        xb[i][h] = *reinterpret_cast<const bf16x8v *>(&Bs[cur][h][(wc + 32 * i + (lane & 31)) * SRS + ko]);
      }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][1], xb[j][0], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[j][1], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[j][0], acc[i][j], 0, 0, 0);
      }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  float *Cb = Cbase + r * g.c_rs + P.c_off;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = j0 + wc + 32 * j + (lane & 31);
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = i0 + wr + 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3);
        if (row < P.M && col < N)
          __builtin_nontemporal_store(g.oscale * acc[i][j][v], &Cb[(int64_t)row * g.ldc + col]);
      }
    }
}

static hipError_t launch_levels_split(const Geometry &G, const float *tables, int nr, const float *A, int t,
                                      int64_t lda, float *U, int64_t ldu, float oscale, void *bsplit,
                                      hipStream_t st) {
  const SplitLayout L = split_layout(G);
  __bf16 *hi = static_cast<__bf16 *>(bsplit);
  const int64_t half = (int64_t)nr * L.up_pad + L.kpad * (int64_t)t;  // elements per hi / lo array
  __bf16 *lo = hi + half;
  SplitArgs sa;
  sa.G = G;
  sa.L = L;
  sa.nr = nr;
  sa.t = t;
  sa.lda = lda;
  const int64_t blocks = std::min<int64_t>(ceil_div(half, 256), 16384);
  hipLaunchKernelGGL(split_kernel, dim3((unsigned)blocks), dim3(256), 0, st, sa, tables, A, hi, lo);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  SplitGemmArgs g{};
  g.nprob = G.nup;
  g.oscale = oscale;
  g.a_rs = L.up_pad;
  g.c_rs = G.urows * ldu;
  g.ldc = ldu;
  g.kpad = L.kpad;
  int tiles = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &lv = G.lev[G.up[u]];
    auto &P = g.p[u];
    P.M = 1 << lv.nb;
    P.K = L.taup[u];
    P.tiles_n = (int)ceil_div(t, SBN);
    P.a_off = L.tab_off[u];
    P.b_off = (int64_t)nr * L.up_pad + L.koff[u];
    P.c_off = lv.uoff * ldu;
    g.tile0[u] = tiles;
    tiles += (int)ceil_div(P.M, SBM) * P.tiles_n;
  }
  for (int q = G.nup; q < kMaxGemmProbs; ++q) g.tile0[q] = 0x7fffffff;
  if (tiles == 0 || nr == 0) return hipSuccess;
  // B (the split A^T) lives after the tables in both arrays: its offset is in b_off
  hipLaunchKernelGGL(gemm_bf16x3, dim3(tiles, nr), dim3(256), 0, st, g, t, hi, lo, hi, lo, U);
  return hipGetLastError();
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
                         int t, int64_t lda, float *U, int64_t ldu, float oscale, void *bsplit, hipStream_t st) {
  LaunchTimer tm("levels", st);
  if (prec == QMC_SPLIT_BF16X3 && bsplit && G.nup > 0)
    return launch_levels_split(G, tables, nr, A, t, lda, U, ldu, oscale, bsplit, st);
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
  finish_tile_table(a);
  return run_gemm<false>(a, prec, nr, tables, A, U, st);
}

// Adjoint partial layout: for each upper level (in order) kchunks blocks of
// tau_I x ldu floats, per shift.
int64_t levels_adj_kchunk(int64_t K) { return K < 1024 ? round_up(K, BK) : 1024; }
static int adj_chunk(int64_t K) { return (int)levels_adj_kchunk(K); }

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
  finish_tile_table(a);
  return run_gemm<true>(a, prec, nr, tables, S, part, st);
}

}  // namespace qmc
