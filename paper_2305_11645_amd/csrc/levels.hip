// Grouped products of the upper levels on the matrix cores.
//
// Forward (Algorithm 2, the product X~_I A~_I of one level):
//     U_I = X~_I A_I,      X~_I: n_I x tau_I point table, A_I: rows G_I of A.
// Adjoint (transpose of the same step):
//     dA_I = X~_I^T S_I,   S_I: n_I x t sums of dQ/dy over the residue classes.
// All levels and all randomisations go in one launch.  The forward operands
// are packed once per call into K-step slabs (the section "forward, packed
// operands" below), and each workgroup owns a 128 x 256 output tile.  In the
// adjoint every workgroup owns one 64 x 64 output tile of one (level, shift,
// K-chunk); it contracts over n_I rows, so it is split into K-chunks of at
// most 1024 whose FP32 partials are combined later in FP64.
//
// Precision:
//   FP32        forward v_mfma_f32_16x16x4_f32, adjoint v_mfma_f32_32x32x2_f32,
//               FP32 accumulation.
//   SPLIT_BF16  each FP32 operand x = hi + lo with hi = bf16(x),
//               lo = bf16(x - hi); lo*hi + hi*lo + hi*hi (forward, one
//               accumulator) or hi*hi on one and hi*lo + lo*hi on a second
//               (adjoint), v_mfma_f32_32x32x16_bf16.
//
// MFMA operand layouts (wave64):
//   32x32x2 f32:  A: lane l holds A[l%32][l/32]; B: B[l/32][l%32];
//                 D: acc[v] = D[8(v/4) + 4(l/32) + v%4][l%32].
//   16x16x4 f32:  A: lane l holds A[l%16][l/16]; B: B[l/16][l%16];
//                 D: acc[v] = D[4(l/16) + v][l%16].
//   32x32x16 bf16: A: lane l holds A[l%32][8(l/32) + 0..7]; B: B[8(l/32)+0..7][l%32];
//                 D as for 32x32x2.
#include <algorithm>
#include <cstdlib>
#include <cstring>

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

// ------------------------------------------------------------------ forward, packed operands
// The forward level products with both operands packed once per call into
// K-step slabs (FP32), or split into (hi, lo) and packed (split BF16):
//   pack_tables_kernel, pack_a_kernel
//                  the upper-level tables X~_I (per randomisation) and the rows
//                  of A of the upper levels, zero-padded to whole tiles and
//                  K-steps of 16;
//   gemm_f32p      FP32: v_mfma_f32_16x16x4_f32;
//   gemm_bf16x3    split BF16: per block pair and K-step lo*hi, hi*lo, hi*hi on
//                  v_mfma_f32_32x32x16_bf16 into one FP32 accumulator.
// Both: 128 x 256 output tiles, four waves of 64 x 128, two LDS buffers, and
// an epilogue that stages each wave's rows through LDS so that every store is
// a 512-byte run of one output row.
// Slab layout: the operand rows of one tile (128 table rows, or 256 columns of
// A) for one K-step of 16 are one contiguous slab [k / RUN][row][k % RUN], RUN
// = 4 values (FP32) or 8 (BF16) = 16 bytes.  A slab is copied to LDS unchanged
// with 16-byte loads and stores in lane order, and a wave's fragment reads
// (lane groups on consecutive rows at one k / RUN) are contiguous runs: no bank
// conflicts and no predicates in the product loop.  In FP32 lane group g of a
// 16 x 16 x 4 block holds k = 4 g .. 4 g + 3 in one 16-byte read, and the
// block's four MFMAs of a K-step contract k = c, 4 + c, 8 + c, 12 + c (c =
// 0..3): every k once, in another order.
typedef __bf16 bf16x8v __attribute__((ext_vector_type(8)));
typedef float f32x4v __attribute__((ext_vector_type(4)));

constexpr int SBM = 128, SBN = 256, SBK = 16;
constexpr int SLAB_A = SBM * SBK, SLAB_B = SBN * SBK;  // values per slab

struct PackLayout {
  int64_t up_pad;                  // values of one randomisation's packed upper tables
  int64_t kpad;                    // padded upper coordinates (K-steps of 16) of the packed A
  int32_t ntn;                     // column tiles of 256
  int64_t tab_off[kMaxLevels];     // per upper level u: offset of its packed table
  int32_t koff[kMaxLevels];        // per upper level u: first K index in the packed A
  int32_t taup[kMaxLevels];        // per upper level u: tau_I rounded up to 16
  int32_t tiles_m[kMaxLevels];     // per upper level u: row tiles of 128
};

static PackLayout pack_layout(const Geometry &G, int t) {
  PackLayout L{};
  int64_t off = 0;
  int32_t k = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &lv = G.lev[G.up[u]];
    L.taup[u] = (int32_t)round_up(lv.tau, SBK);
    L.tiles_m[u] = (int32_t)ceil_div(int64_t(1) << lv.nb, SBM);
    L.tab_off[u] = off;
    L.koff[u] = k;
    off += (int64_t)L.tiles_m[u] * SBM * L.taup[u];
    k += L.taup[u];
  }
  L.up_pad = off;
  L.kpad = k;
  L.ntn = (int32_t)ceil_div(t, SBN);
  return L;
}

// values of the packed tables of nr randomisations plus the packed A
static int64_t packed_values(const PackLayout &L, int nr) {
  return (int64_t)nr * L.up_pad + (int64_t)L.ntn * SBN * L.kpad;
}

int64_t levels_pack_bytes(const Geometry &G, int nr, int t) {
  return 4 * packed_values(pack_layout(G, t), nr);  // FP32, or bf16 hi and lo
}

struct PackArgs {
  Geometry G;
  PackLayout L;
  int32_t nr, t;
  int64_t lda;
  int64_t half;  // split BF16: values per hi / lo array
};

// Arrays: [nr][up_pad] of the tables, then [ntn * 256 * kpad] of A, both in
// slab order; padding (rows past n_I, columns past t, k past tau_I) is 0.  In
// split BF16 the hi array is followed (a.half values later) by the lo array.

// The tables: one workgroup per slab (128 rows x 16 k of one level, one
// randomisation), read in runs of 16 k per row (a wave reads four 64-byte
// row pieces per load), turned in LDS and written as one contiguous slab.
template <bool F32>
__global__ __launch_bounds__(256) void pack_tables_kernel(PackArgs a, const float *__restrict__ tables,
                                                          void *__restrict__ out) {
  constexpr int RUN = F32 ? 4 : 8;
  __shared__ __attribute__((aligned(16))) float lds[SLAB_A];
  const Geometry &G = a.G;
  const int r = blockIdx.y, tid = threadIdx.x;
  const int64_t q = (int64_t)blockIdx.x * SLAB_A;  // this slab's offset in the randomisation's tables
  int u = 0;
  while (u + 1 < G.nup && a.L.tab_off[u + 1] <= q) ++u;
  const Level &lv = G.lev[G.up[u]];
  const int ksteps = a.L.taup[u] / SBK;
  const int64_t sl = (q - a.L.tab_off[u]) / SLAB_A;
  const int64_t row0 = (sl / ksteps) * SBM;
  const int k0 = (int)(sl % ksteps) * SBK;
  const int64_t M = int64_t(1) << lv.nb;
  const float *src = tables + r * G.table_total + G.lower_total + lv.off;
#pragma unroll
  for (int it = 0; it < SLAB_A / 256; ++it) {
    const int e = it * 256 + tid, ri = e / SBK, k = e % SBK;
    const int64_t row = row0 + ri;
    const float x = row < M && k0 + k < lv.tau ? src[row * lv.tau + k0 + k] : 0.f;
    lds[(k / RUN) * (SBM * RUN) + ri * RUN + k % RUN] = x;
  }
  __syncthreads();
  const int64_t base = (int64_t)r * a.L.up_pad + q;
  if constexpr (F32) {
#pragma unroll
    for (int it = 0; it < SLAB_A / 1024; ++it) {
      const int o = (it * 256 + tid) * 4;
      *reinterpret_cast<f32x4v *>(static_cast<float *>(out) + base + o) = *reinterpret_cast<const f32x4v *>(&lds[o]);
    }
  } else {
    static_assert(SLAB_A == 256 * 8, "one run of 8 per thread");
    const int o = tid * 8;
    bf16x8v h, l;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const float x = lds[o + i];
      h[i] = (__bf16)x;
      l[i] = (__bf16)(x - (float)h[i]);
    }
    __bf16 *hi = static_cast<__bf16 *>(out);
    *reinterpret_cast<bf16x8v *>(hi + base + o) = h;
    *reinterpret_cast<bf16x8v *>(hi + a.half + base + o) = l;
  }
}

// The rows of A: one thread writes one run of RUN k-values of one column
// (16 bytes; split BF16: 16 bytes of hi and of lo); consecutive threads take
// consecutive columns, so each row of A is read in whole wave-wide runs.
template <bool F32>
__global__ __launch_bounds__(256) void pack_a_kernel(PackArgs a, const float *__restrict__ A,
                                                     void *__restrict__ out) {
  constexpr int RUN = F32 ? 4 : 8;
  const Geometry &G = a.G;
  const int64_t runs = (int64_t)a.L.ntn * SBN * a.L.kpad / RUN;
  const int64_t base = (int64_t)a.nr * a.L.up_pad;  // the A follows the tables
  const uint32_t ksteps = (uint32_t)(a.L.kpad / SBK);
  for (int64_t c = (int64_t)blockIdx.x * 256 + threadIdx.x; c < runs; c += (int64_t)gridDim.x * 256) {
    const int64_t q0 = c * RUN;
    const uint32_t slab = (uint32_t)(q0 / SLAB_B), in = (uint32_t)(q0 % SLAB_B);
    const int64_t col = (int64_t)(slab / ksteps) * SBN + (in % (SBN * RUN)) / RUN;
    const int kk0 = (int)(slab % ksteps) * SBK + (int)(in / (SBN * RUN)) * RUN;
    int u = 0;
    while (u + 1 < G.nup && a.L.koff[u + 1] <= kk0) ++u;  // a run lies in one level
    const Level &lv = G.lev[G.up[u]];
    const int k0 = kk0 - a.L.koff[u];
    const bool cok = col < a.t;
    const float *src = A + (int64_t)(lv.j0 + k0) * a.lda + (cok ? col : 0);
    float x[RUN];
#pragma unroll
    for (int i = 0; i < RUN; ++i) x[i] = cok && k0 + i < lv.tau ? src[(int64_t)i * a.lda] : 0.f;
    if constexpr (F32) {
      f32x4v v;
#pragma unroll
      for (int i = 0; i < 4; ++i) v[i] = x[i];
      *reinterpret_cast<f32x4v *>(static_cast<float *>(out) + base + q0) = v;
    } else {
      bf16x8v h, l;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        h[i] = (__bf16)x[i];
        l[i] = (__bf16)(x[i] - (float)h[i]);
      }
      __bf16 *hi = static_cast<__bf16 *>(out);
      *reinterpret_cast<bf16x8v *>(hi + base + q0) = h;
      *reinterpret_cast<bf16x8v *>(hi + a.half + base + q0) = l;
    }
  }
}

struct PackGemmArgs {
  int32_t tile0[kMaxGemmProbs];
  int32_t nprob;
  float oscale;
  int64_t a_rs, c_rs, ldc, b_tile;  // b_tile: values of one column tile of the packed A (256 kpad)
  struct {
    int32_t M, ksteps, tiles_n;
    int64_t a_off, b_off, c_off;
  } p[kMaxLevels];
};

// Problem, row tile and column tile of this workgroup.
struct TileRef {
  int pi, tm, tn;
};
__device__ __forceinline__ TileRef tile_of(const PackGemmArgs &g) {
  int tile = blockIdx.x, pi = 0;
#pragma unroll
  for (int q = 1; q < kMaxGemmProbs; ++q)
    if (tile >= g.tile0[q]) pi = q;
  tile -= g.tile0[pi];
  return TileRef{pi, tile / g.p[pi].tiles_n, tile % g.p[pi].tiles_n};
}

// Epilogue: a wave's 16 x 128 block of output rows row0.. and columns col0..,
// already in its LDS region E (row stride ES floats), stored as 512-byte row runs.
// Columns up to ldc are written (past t the packed A is 0, so are they).
template <int ES>
__device__ __forceinline__ void store_rows(const float *E, float *C, int64_t ldc, int M, int row0, int col0,
                                           float oscale, int lane) {
#pragma unroll
  for (int p = 0; p < 8; ++p) {
    const int rr = 2 * p + (lane >> 5), cc = 4 * (lane & 31);
    f32x4v v = *reinterpret_cast<const f32x4v *>(&E[rr * ES + cc]);
    if (row0 + rr < M && col0 + cc < ldc)
      __builtin_nontemporal_store(oscale * v, reinterpret_cast<f32x4v *>(&C[(int64_t)(row0 + rr) * ldc + col0 + cc]));
  }
}

constexpr int ES32 = 132, ES16 = 136;  // epilogue row strides: the 16-row groups' writes on distinct banks

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_f32p(
    PackGemmArgs g, const float *__restrict__ Ap, const float *__restrict__ Bp, float *__restrict__ Cbase) {
  __shared__ __attribute__((aligned(16))) float Ls[2 * (SLAB_A + SLAB_B)];  // [buffer][A slab, B slab]
  static_assert(4 * 16 * ES32 <= 2 * (SLAB_A + SLAB_B), "epilogue does not fit");
  const int r = blockIdx.y;
  const TileRef T = tile_of(g);
  const auto &P = g.p[T.pi];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 128;
  const float *ap = Ap + r * g.a_rs + P.a_off + (int64_t)T.tm * P.ksteps * SLAB_A + tid * 4;
  const float *bp = Bp + P.b_off + T.tn * g.b_tile + tid * 4;
  f32x4v ra[2], rb[4];
  auto load = [&](int ks) {
    const int64_t ao = (int64_t)ks * SLAB_A, bo = (int64_t)ks * SLAB_B;
#pragma unroll
    for (int q = 0; q < 2; ++q) ra[q] = *reinterpret_cast<const f32x4v *>(ap + ao + 1024 * q);
#pragma unroll
    for (int q = 0; q < 4; ++q) rb[q] = *reinterpret_cast<const f32x4v *>(bp + bo + 1024 * q);
  };
  auto store = [&](int buf) {
    float *As = Ls + buf * (SLAB_A + SLAB_B), *Bs = As + SLAB_A;
#pragma unroll
    for (int q = 0; q < 2; ++q) *reinterpret_cast<f32x4v *>(&As[1024 * q + tid * 4]) = ra[q];
#pragma unroll
    for (int q = 0; q < 4; ++q) *reinterpret_cast<f32x4v *>(&Bs[1024 * q + tid * 4]) = rb[q];
  };
  f32x4v acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = f32x4v{0.f, 0.f, 0.f, 0.f};
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  // fragment offsets: row (column) wr + 16 i + lane % 16, k = 4 (lane / 16) .. + 3
  const int fa = (lane >> 4) * (SBM * 4) + (wr + (lane & 15)) * 4;
  const int fb = (lane >> 4) * (SBN * 4) + (wc + (lane & 15)) * 4;
  for (int ks = 0; ks < P.ksteps; ++ks) {
    const bool more = ks + 1 < P.ksteps;
    if (more) load(ks + 1);
    const float *As = Ls + cur * (SLAB_A + SLAB_B), *Bs = As + SLAB_A;
    f32x4v xa[4], xb[8];
#pragma unroll
    for (int i = 0; i < 4; ++i) xa[i] = *reinterpret_cast<const f32x4v *>(&As[fa + 64 * i]);
#pragma unroll
    for (int j = 0; j < 8; ++j) xb[j] = *reinterpret_cast<const f32x4v *>(&Bs[fb + 64 * j]);
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[i][c], xb[j][c], acc[i][j], 0, 0, 0);
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // D of a 16 x 16 block: acc[v] at row 4 (lane / 16) + v, column lane % 16
  float *E = Ls + w * 16 * ES32;
  float *Cb = Cbase + r * g.c_rs + P.c_off;
  const int i0 = T.tm * SBM + wr, j0 = T.tn * SBN + wc;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) E[(4 * (lane >> 4) + v) * ES32 + 16 * j + (lane & 15)] = acc[i][j][v];
    __syncthreads();
    store_rows<ES32>(E, Cb, g.ldc, P.M, i0 + 16 * i, j0, g.oscale, lane);
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16x3(
    PackGemmArgs g, const __bf16 *__restrict__ Ahi, const __bf16 *__restrict__ Alo,
    const __bf16 *__restrict__ Bhi, const __bf16 *__restrict__ Blo, float *__restrict__ Cbase) {
  __shared__ __attribute__((aligned(16))) __bf16 Ls[2 * 2 * (SLAB_A + SLAB_B)];  // [buffer][hi, lo][A, B slab]
  static_assert(4 * 16 * ES16 * 4 <= 2 * 2 * (SLAB_A + SLAB_B) * 2, "epilogue does not fit");
  const int r = blockIdx.y;
  const TileRef T = tile_of(g);
  const auto &P = g.p[T.pi];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wr = (w >> 1) * 64, wc = (w & 1) * 128;
  // this thread's 16-byte chunks of each slab: A chunk tid, B chunks tid and tid + 256
  const int64_t aoff = r * g.a_rs + P.a_off + (int64_t)T.tm * P.ksteps * SLAB_A + tid * 8;
  const int64_t boff = P.b_off + T.tn * g.b_tile + tid * 8;
  const __bf16 *ah_p = Ahi + aoff, *al_p = Alo + aoff, *bh_p = Bhi + boff, *bl_p = Blo + boff;
  bf16x8v ra[2], rb[2][2];
  auto load = [&](int ks) {
    const int64_t ao = (int64_t)ks * SLAB_A, bo = (int64_t)ks * SLAB_B;
    ra[0] = *reinterpret_cast<const bf16x8v *>(ah_p + ao);
    ra[1] = *reinterpret_cast<const bf16x8v *>(al_p + ao);
    rb[0][0] = *reinterpret_cast<const bf16x8v *>(bh_p + bo);
    rb[0][1] = *reinterpret_cast<const bf16x8v *>(bh_p + bo + SLAB_B / 2);
    rb[1][0] = *reinterpret_cast<const bf16x8v *>(bl_p + bo);
    rb[1][1] = *reinterpret_cast<const bf16x8v *>(bl_p + bo + SLAB_B / 2);
  };
  // buffer b, h = hi / lo: A slab at (2 b + h) (SLAB_A + SLAB_B), its B slab SLAB_A further
  auto slab = [&](int buf, int h) { return Ls + (2 * buf + h) * (SLAB_A + SLAB_B); };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      __bf16 *As = slab(buf, h), *Bs = As + SLAB_A;
      *reinterpret_cast<bf16x8v *>(&As[tid * 8]) = ra[h];
      *reinterpret_cast<bf16x8v *>(&Bs[tid * 8]) = rb[h][0];
      *reinterpret_cast<bf16x8v *>(&Bs[SLAB_B / 2 + tid * 8]) = rb[h][1];
    }
  };
  f32x16 acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x16{0};
  load(0);
  store(0);
  __syncthreads();
  int cur = 0;
  // fragment offsets inside a slab: row (or column) wr + 32 i + lane % 32 at k-half lane / 32
  const int fa = (lane >> 5) * (SBM * 8) + (wr + (lane & 31)) * 8;
  const int fb = (lane >> 5) * (SBN * 8) + (wc + (lane & 31)) * 8;
  for (int ks = 0; ks < P.ksteps; ++ks) {
    const bool more = ks + 1 < P.ksteps;
    if (more) load(ks + 1);
    bf16x8v xa[2][2], xb[4][2];  // [block][hi, lo]
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const __bf16 *As = slab(cur, h), *Bs = As + SLAB_A;
#pragma unroll
      for (int i = 0; i < 2; ++i) xa[i][h] = *reinterpret_cast<const bf16x8v *>(&As[fa + 256 * i]);
#pragma unroll
      for (int j = 0; j < 4; ++j) xb[j][h] = *reinterpret_cast<const bf16x8v *>(&Bs[fb + 256 * j]);
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][1], xb[j][0], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[j][1], acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xa[i][0], xb[j][0], acc[i][j], 0, 0, 0);
      }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // D of a 32 x 32 block: acc[v] at row 8 (v / 4) + 4 (lane / 32) + v % 4, column lane % 32;
  // v < 8 are its rows 0..15, v >= 8 its rows 16..31
  float *E = reinterpret_cast<float *>(Ls) + w * 16 * ES16;
  float *Cb = Cbase + r * g.c_rs + P.c_off;
  const int i0 = T.tm * SBM + wr, j0 = T.tn * SBN + wc;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int hf = 0; hf < 2; ++hf) {
#pragma unroll
      for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int v = 0; v < 8; ++v)
          E[(8 * (v >> 2) + 4 * (lane >> 5) + (v & 3)) * ES16 + 32 * j + (lane & 31)] = acc[i][j][8 * hf + v];
      __syncthreads();
      store_rows<ES16>(E, Cb, g.ldc, P.M, i0 + 32 * i + 16 * hf, j0, g.oscale, lane);
      __syncthreads();
    }
}

static hipError_t launch_levels_packed(const Geometry &G, int prec, const float *tables, int nr, const float *A,
                                       int t, int64_t lda, float *U, int64_t ldu, float oscale, void *buf,
                                       hipStream_t st) {
  const PackLayout L = pack_layout(G, t);
  const int64_t ntab = (int64_t)nr * L.up_pad;
  PackArgs sa;
  sa.G = G;
  sa.L = L;
  sa.nr = nr;
  sa.t = t;
  sa.lda = lda;
  sa.half = packed_values(L, nr);
  const bool f32 = prec == QMC_FP32;
  const int64_t slabs = L.up_pad / SLAB_A, aruns = (int64_t)L.ntn * SBN * L.kpad / (f32 ? 4 : 8);
  if (nr > 0 && slabs > 0)
    hipLaunchKernelGGL(f32 ? pack_tables_kernel<true> : pack_tables_kernel<false>, dim3((unsigned)slabs, nr),
                       dim3(256), 0, st, sa, tables, buf);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(f32 ? pack_a_kernel<true> : pack_a_kernel<false>,
                     dim3((unsigned)std::min<int64_t>(ceil_div(aruns, 256), 4096)), dim3(256), 0, st, sa, A, buf);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  PackGemmArgs g{};
  g.nprob = G.nup;
  g.oscale = oscale;
  g.a_rs = L.up_pad;
  g.c_rs = G.urows * ldu;
  g.ldc = ldu;
  g.b_tile = (int64_t)SBN * L.kpad;
  // problems in decreasing K: the longest tiles are dispatched first and the
  // short ones fill the tail
  int order[kMaxLevels];
  for (int u = 0; u < G.nup; ++u) order[u] = u;
  std::stable_sort(order, order + G.nup, [&](int x, int y) { return L.taup[x] > L.taup[y]; });
  int tiles = 0;
  for (int q = 0; q < G.nup; ++q) {
    const int u = order[q];
    const Level &lv = G.lev[G.up[u]];
    auto &P = g.p[q];
    P.M = 1 << lv.nb;
    P.ksteps = L.taup[u] / SBK;
    P.tiles_n = L.ntn;
    P.a_off = L.tab_off[u];
    P.b_off = ntab + (int64_t)(L.koff[u] / SBK) * SLAB_B;
    P.c_off = lv.uoff * ldu;
    g.tile0[q] = tiles;
    tiles += L.tiles_m[u] * P.tiles_n;
  }
  for (int q = G.nup; q < kMaxGemmProbs; ++q) g.tile0[q] = 0x7fffffff;
  if (tiles == 0 || nr == 0) return hipSuccess;
  // the packed A follows the tables: its offset is in b_off
  if (f32) {
    const float *p = static_cast<const float *>(buf);
    hipLaunchKernelGGL(gemm_f32p, dim3(tiles, nr), dim3(256), 0, st, g, p, p, U);
  } else {
    const __bf16 *hi = static_cast<const __bf16 *>(buf), *lo = hi + sa.half;
    hipLaunchKernelGGL(gemm_bf16x3, dim3(tiles, nr), dim3(256), 0, st, g, hi, lo, hi, lo, U);
  }
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

// The forward products straight from the tables and A on 64 x 64 tiles (no
// packing pass): for grids too small to fill the chip with 128 x 256 tiles.
static hipError_t launch_levels_direct(const Geometry &G, int prec, const float *tables, int nr, const float *A,
                                       int t, int64_t lda, float *U, int64_t ldu, float oscale, hipStream_t st) {
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

// Packed 128 x 256 tiles are taken when there are enough of them to fill the
// chip (all randomisations), or half as many when no level has more than 512
// coordinates (the longest tiles, dispatched first, then end in time);
// otherwise the 64 x 64 direct form, with eight times as many tiles and no
// packing pass (measured: C2, C4's stored-Y product, C5).
constexpr int64_t kMinPackedTiles = 1536;

hipError_t launch_levels(const Geometry &G, int prec, const float *tables, int nr, const float *A,
                         int t, int64_t lda, float *U, int64_t ldu, float oscale, void *pack, hipStream_t st) {
  LaunchTimer tm("levels", st);
  if (G.nup == 0 || nr == 0) return hipSuccess;
  const PackLayout L = pack_layout(G, t);
  int64_t tiles = 0;
  int kmax = 0;
  for (int u = 0; u < G.nup; ++u) {
    tiles += (int64_t)L.tiles_m[u] * L.ntn;
    kmax = std::max(kmax, L.taup[u]);
  }
  bool direct = tiles * nr < (kmax <= 512 ? kMinPackedTiles / 2 : kMinPackedTiles);
  if (const char *env = getenv("QMC_LEVELS_FORM")) {  // test and measurement switch: "direct" or "packed"
    if (!strcmp(env, "direct")) direct = true;
    if (!strcmp(env, "packed")) direct = false;
  }
  if (direct) return launch_levels_direct(G, prec, tables, nr, A, t, lda, U, ldu, oscale, st);
  if (!pack || ldu % 4 != 0) return hipErrorInvalidValue;
  return launch_levels_packed(G, prec, tables, nr, A, t, lda, U, ldu, oscale, pack, st);
}

// Adjoint partial layout: for each upper level (in order) kchunks blocks of
// tau_I x ldu floats, per shift.
int64_t levels_adj_kchunk(int64_t K) { return K < 256 ? round_up(K, BK) : 256; }
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

// ------------------------------------------------------------------ adjoint, FP32
// dA_I = X~_I^T S_I on v_mfma_f32_16x16x4_f32: workgroup tiles of TI
// coordinates x TJ columns over one K-chunk of rows, four waves in a WI x
// (4 / WI) grid, K-steps of 16 rows staged in LDS with padded row strides (the
// four rows a wave reads at once fall on distinct banks).  Both operands are
// row-major in K: X~_I[k][i] (the table) and S_I[k][j].  Levels with at most
// 32 coordinates take 32 x 256 tiles, at most 64 take 64 x 256, the others
// 128 x 128, so that a row of S is re-read by few workgroups.
constexpr int ABK = 16;

struct AdjArgs {
  int32_t tile0[kMaxGemmProbs];
  int32_t nprob;
  int64_t a_rs, b_rs, c_rs, ldb, ldc;
  struct {
    int32_t tau, K, kchunk, kchunks, tiles_i, tiles_j;
    int64_t a_off, b_off, c_off, c_chunk;
  } p[kMaxLevels];
};

template <int TI, int TJ, int WI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_adj_f32(
    AdjArgs g, int t, const float *__restrict__ tables, const float *__restrict__ S, float *__restrict__ part) {
  constexpr int WJ = 4 / WI, BI = TI / (16 * WI), BJ = TJ / (16 * WJ);
  constexpr int AS = TI + 16, BS = TJ + 16;  // row strides of 16 or 48 (mod 64) floats
  static_assert(AS % 64 == 16 || AS % 64 == 48, "A rows must fall on distinct banks");
  static_assert(BS % 64 == 16 || BS % 64 == 48, "B rows must fall on distinct banks");
  constexpr int NA = ABK * TI / 256, NB4 = ABK * TJ / 1024;  // per thread: X floats, S float4s
  static_assert(NA >= 1 && NB4 >= 1, "tile too small for the loaders");
  __shared__ __attribute__((aligned(16))) float As[2][ABK * AS];
  __shared__ __attribute__((aligned(16))) float Bs[2][ABK * BS];
  const int r = blockIdx.y;
  int tile = blockIdx.x, pi = 0;
#pragma unroll
  for (int q = 1; q < kMaxGemmProbs; ++q)
    if (tile >= g.tile0[q]) pi = q;
  const auto &P = g.p[pi];
  tile -= g.tile0[pi];
  // coordinate tiles fastest: neighbouring workgroups share their rows of S
  const int ti = tile % P.tiles_i;
  tile /= P.tiles_i;
  const int tj = tile % P.tiles_j, chunk = tile / P.tiles_j;
  const int i0 = ti * TI, j0 = tj * TJ;
  const int kbeg = chunk * P.kchunk, kend = min(P.K, kbeg + P.kchunk);
  const float *X = tables + r * g.a_rs + P.a_off;
  const float *Sb = S + r * g.b_rs + P.b_off;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // loaders: X element tid + 256 q is (row e / TI, coordinate i0 + e % TI);
  // S float4 tid + 256 q is (row e / (TJ / 4), columns j0 + 4 (e % (TJ / 4)) + 0..3)
  float ra[NA];
  f32x4v rb[NB4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q, k = k0 + e / TI, i = i0 + e % TI;
      ra[q] = k < kend && i < P.tau ? X[(int64_t)k * P.tau + i] : 0.f;
    }
#pragma unroll
    for (int q = 0; q < NB4; ++q) {
      const int e = tid + 256 * q, k = k0 + e / (TJ / 4), j = j0 + 4 * (e % (TJ / 4));
      // columns past t (up to ldb) only reach outputs that are not stored
      rb[q] = k < kend && j < g.ldb ? *reinterpret_cast<const f32x4v *>(&Sb[(int64_t)k * g.ldb + j])
                                    : f32x4v{0.f, 0.f, 0.f, 0.f};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + 256 * q;
      As[buf][(e / TI) * AS + e % TI] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB4; ++q) {
      const int e = tid + 256 * q;
      *reinterpret_cast<f32x4v *>(&Bs[buf][(e / (TJ / 4)) * BS + 4 * (e % (TJ / 4))]) = rb[q];
    }
  };
  f32x4v acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = f32x4v{0.f, 0.f, 0.f, 0.f};
  load(kbeg);
  store(0);
  __syncthreads();
  int cur = 0;
  const int wi = (w / WJ) * (16 * BI), wj = (w % WJ) * (16 * BJ), kl = lane >> 4, cl = lane & 15;
  for (int k0 = kbeg; k0 < kend; k0 += ABK) {
    const bool more = k0 + ABK < kend;
    if (more) load(k0 + ABK);
#pragma unroll
    for (int c = 0; c < ABK / 4; ++c) {
      const int kr = 4 * c + kl;  // this lane's row of the 4-row step
      float xa[BI], xb[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) xa[i] = As[cur][kr * AS + wi + 16 * i + cl];
#pragma unroll
      for (int j = 0; j < BJ; ++j) xb[j] = Bs[cur][kr * BS + wj + 16 * j + cl];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xa[i], xb[j], acc[i][j], 0, 0, 0);
    }
    if (more) store(cur ^ 1);
    __syncthreads();
    cur ^= 1;
  }
  // D of a 16 x 16 block: acc[v] at row 4 (lane / 16) + v, column lane % 16
  float *C = part + r * g.c_rs + P.c_off + (int64_t)chunk * P.c_chunk;
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      const int col = j0 + wj + 16 * j + cl;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = i0 + wi + 16 * i + 4 * kl + v;
        if (row < P.tau && col < t) C[(int64_t)row * g.ldc + col] = acc[i][j][v];
      }
    }
}

hipError_t launch_levels_adj(const Geometry &G, int prec, const float *tables, int nr,
                             const float *S, int t, int64_t ldu, float *part, hipStream_t st) {
  LaunchTimer tm("levels_adj", st);
  // below about 2 GFLOP the three launches of the tiled form cost more than
  // the products; the one-launch 64 x 64 form then takes them (C2's gradient)
  double flops = 0.0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    flops += 2.0 * L.tau * (double)(int64_t(1) << L.nb) * t * nr;
  }
  bool tiled = flops >= 2e9;
  if (const char *env = getenv("QMC_LEVELS_FORM")) {  // test and measurement switch, as for the forward form
    if (!strcmp(env, "direct")) tiled = false;
    if (!strcmp(env, "packed")) tiled = true;
  }
  if (prec == QMC_FP32 && tiled) {
    if (G.nup == 0 || nr == 0) return hipSuccess;
    if (ldu % 4 != 0) return hipErrorInvalidValue;
    // three launches: levels with tau <= 32 on 32 x 256 tiles, tau <= 64 on
    // 64 x 256, the others on 128 x 128
    for (int shape = 0; shape < 3; ++shape) {
      const int TI = shape == 0 ? 32 : shape == 1 ? 64 : 128, TJ = shape == 2 ? 128 : 256;
      AdjArgs a{};
      a.a_rs = G.table_total;
      a.b_rs = (2 * G.nsub) * ldu;  // S pyramid rows per shift
      a.c_rs = levels_adj_part_floats(G, t, ldu);
      a.ldb = ldu;
      a.ldc = ldu;
      int tiles = 0;
      int64_t poff = 0, soff = 0;
      int Iprev = G.split;
      for (int u = 0; u < G.nup; ++u) {
        const Level &L = G.lev[G.up[u]];
        for (int I = Iprev; I < G.up[u]; ++I) soff += int64_t(1) << (G.m - I);  // S_I follows levels split .. I-1
        Iprev = G.up[u];
        const int K = 1 << L.nb, kchunk = adj_chunk(K), kchunks = (int)ceil_div(K, kchunk);
        const int64_t c_off = poff;
        poff += (int64_t)kchunks * L.tau * ldu;
        if ((L.tau <= 32 ? 0 : L.tau <= 64 ? 1 : 2) != shape) continue;
        auto &P = a.p[a.nprob];
        P.tau = L.tau;
        P.K = K;
        P.kchunk = kchunk;
        P.kchunks = kchunks;
        P.tiles_i = (int)ceil_div(P.tau, TI);
        P.tiles_j = (int)ceil_div(t, TJ);
        P.a_off = G.lower_total + L.off;
        P.b_off = soff * ldu;
        P.c_off = c_off;
        P.c_chunk = (int64_t)L.tau * ldu;
        a.tile0[a.nprob++] = tiles;
        tiles += P.tiles_i * P.tiles_j * P.kchunks;
      }
      if (tiles == 0) continue;
      for (int q = a.nprob; q < kMaxGemmProbs; ++q) a.tile0[q] = 0x7fffffff;
      if (shape == 2)
        hipLaunchKernelGGL((gemm_adj_f32<128, 128, 2>), dim3(tiles, nr), dim3(256), 0, st, a, t, tables, S, part);
      else if (shape == 1)
        hipLaunchKernelGGL((gemm_adj_f32<64, 256, 1>), dim3(tiles, nr), dim3(256), 0, st, a, t, tables, S, part);
      else
        hipLaunchKernelGGL((gemm_adj_f32<32, 256, 1>), dim3(tiles, nr), dim3(256), 0, st, a, t, tables, S, part);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
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
