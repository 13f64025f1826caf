// Products by gathered value tiles on the matrix cores: reduced digital nets
// that are not periodic (Section 3, Algorithm 4), and reduced point sets in a
// prime base b > 2 (Section 1.3, Section 4), whose index is n mod n_j.
//
// After the row reduction of eq. reduced_genmat_net2, coordinate j of such a
// net still depends on every digit of the point index n, but takes only the
// n_j values X_j[c], c < n_j (c = floor(y_{n,j} n_j), the integer of its
// reduced output digits).  Algorithm 4 forms c_k = X_j[k] a_j once per value
// and adds the selected rows for every point: multiplications drop to
// t sum_j n_j, additions stay s N t.  On MI355X a multiply-add costs what an
// add costs, and the table of all c_k would hold sum_j n_j x t floats, so the
// same sum is evaluated as products on the matrix cores: the point-value tile
// of 64 points x 32 coordinates is gathered from the n_j-value tables and
// multiplied by the rows of A, the n_j values (shift and map included) being
// computed once per coordinate and randomisation.
//
// The value index of a point is F_2-linear in its digits: with
// y_j(n) = XOR of the generating-matrix columns selected by the digits of n,
// restricted to the first n_j rows, c = bitreverse(y_j(n)).  The value tables
// are therefore stored in digit order, T_j[y] = X_j[bitreverse(y)], so that a
// point reads T_j[y_j(n)].  For the 64 points n0 + r of a tile (n0 a multiple
// of 64), y_j(n0 + r) = y_j(n0) XOR y_j(r); both words depend only on the
// generating matrices, and qmc_points_init tabulates y_j(n0) for every tile and
// y_j(r) for r < 64 once (DevSpec::ytile, DevSpec::ylo).  For a Sobol'-type net
// (upper triangular matrices) y_j(r), r < 64, lives in the low 6 digits, so the
// 64 points of a tile read one aligned block of 64 values per coordinate.
//
// Modes (one 64-point x 256-column tile per workgroup, Y never stored except
// in the matvec mode):
//   StoreY  Y = X A
//   Sum     per-workgroup FP64 sum of g(y) over the tile (separable f)
//   Point   per point, the sum of g(y) over the tile's 256 columns (non-separable h)
#include <algorithm>

#include "qmc_internal.h"

namespace qmc {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 256, TK = 32;  // points x columns x coordinates per step
constexpr int NWAVE = 4;                   // wave w owns columns [64 w, 64 w + 64) of the tile
constexpr int KPW = TK / NWAVE;            // coordinates gathered by each wave per step
constexpr int XPAD = TK + 1;               // X tile row stride (odd: conflict-free)

struct Alg4Args {
  int32_t m, s, t, tct;
  int32_t j0, sc;        // the pass sums coordinates [j0, j0 + sc)
  int64_t N, lda, ldy, tab_stride;  // N: points of the pass
  int64_t ntiles;        // ceil(N / 64)
  int64_t ystride;       // StoreY: floats between the randomisations' outputs
  const float *root;     // optional root table added to y: row n mod nsplit
  int64_t ldp, root_stride, nsplit;
  float sigma;           // y' = sigma y (scale of g)
};

// Buffer resource of `bytes` bytes at `base` (raw, stride 0): loads at byte
// offsets at or past `bytes` return zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t raw_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}

__device__ __forceinline__ float load_f32(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}

// IDX: how a point's value index combines the tile word and the lane word
// (0: XOR, nets that are not periodic; 1: add, base b > 2).
// (FP32 nets run at three waves per SIMD; the root-table epilogue of the add
// index needs the registers of two.)
template <int PREC, int MODE, int GF, int IDX>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == QMC_FP32 && !IDX ? 3 : 2))) void alg4_kernel(Alg4Args a, DevSpec D, const float *__restrict__ tab,
                                                   const float *__restrict__ A, float *__restrict__ Y,
                                                   double *__restrict__ partial,
                                                   float *__restrict__ ppart) {
  __shared__ float Xs[2][TM * XPAD];  // point values, two steps: [point][coordinate]
  __shared__ double red[NWAVE];
  __shared__ float rsum[NWAVE][TM];

  const int tn = blockIdx.x, ct = blockIdx.y, rl = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wc = w * 64;
  const int64_t n0 = (int64_t)tn * TM;
  const __amdgpu_buffer_rsrc_t trs = raw_rsrc(tab + (int64_t)rl * a.tab_stride, (uint32_t)(a.tab_stride * 4));
  const uint32_t *ytile = D.ytile + (int64_t)tn * a.s;  // the tile words of every coordinate

  // Only wave w reads columns [wc, wc + 64) of the tile, so its B operands come
  // straight from A into registers, one step ahead.  Element e < TK of a lane:
  // row k0 + brow(e) + bh, column colc[bblk(e)] (FP32 32x32x2: e = kk + c,
  // bh = lane / 32; BF16 32x32x16: e = kc + 8 c + q, bh = 8 (lane / 32)).
  // Columns past t read column t - 1 (their outputs are dropped); rows past s
  // read zero (the step's buffer ends at row s).
  auto brow = [&](int e) { return PREC == QMC_FP32 ? (e & ~1) : (e & ~15) + (e & 7); };
  auto bblk = [&](int e) { return PREC == QMC_FP32 ? (e & 1) : ((e >> 3) & 1); };
  const int bh = PREC == QMC_FP32 ? (lane >> 5) : 8 * (lane >> 5);
  uint32_t boff[2];  // byte offset of this lane's element in row k0 of the step
#pragma unroll
  for (int c = 0; c < 2; ++c)
    boff[c] = (uint32_t)(((int64_t)bh * a.lda + min(ct * TN + wc + 32 * c + (lane & 31), a.t - 1)) * 4);

  // Step k0: wave w gathers coordinates j0 + k0 + KPW w + q (q < KPW) of the 64
  // points (lane = point); a value's byte offset is 4 (ytile_j op ylo_j(lane)).
  // Coordinates past the pass's last gather that one (its rows of A read zero),
  // points past N gather valid values (their outputs are dropped).
  uint32_t yl[KPW], yt[KPW];  // index words of the next coordinates to gather
  float xv[KPW];
  auto load_index = [&](int k0) {
#pragma unroll
    for (int q = 0; q < KPW; ++q) {
      const int j = a.j0 + min(k0 + KPW * w + q, a.sc - 1);
      yl[q] = D.ylo[(int64_t)j * 64 + lane];
      yt[q] = ytile[j];
    }
  };
  auto load_values = [&](int k0, float (&b)[TK]) {
#pragma unroll
    for (int q = 0; q < KPW; ++q) xv[q] = load_f32(trs, (IDX ? yt[q] + yl[q] : yt[q] ^ yl[q]) << 2);
    const int64_t left = (int64_t)a.sc - k0;  // rows of A from row k0 on
    const int64_t want = ((left - 1) * a.lda + a.t) * 4;
    const uint32_t bytes = left <= 0 ? 0u : want > 0xffffffffll ? 0xffffffffu : (uint32_t)want;
    const __amdgpu_buffer_rsrc_t ars = raw_rsrc(left <= 0 ? A : A + (int64_t)k0 * a.lda, bytes);
#pragma unroll
    for (int e = 0; e < TK; ++e) b[e] = load_f32(ars, (uint32_t)(brow(e) * a.lda * 4) + boff[bblk(e)]);
  };
  auto store_x = [&](float *xs) {
#pragma unroll
    for (int q = 0; q < KPW; ++q) xs[lane * XPAD + KPW * w + q] = xv[q];
  };

  f32x16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[i][c] = f32x16{0};

  auto products = [&](const float *xs, const float (&b)[TK]) {
    if (PREC == QMC_FP32) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 2) {
        float x[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) x[i] = xs[(32 * i + (lane & 31)) * XPAD + kk + (lane >> 5)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[i], b[kk + c], acc[i][c], 0, 0, 0);
      }
    } else {
      // split BF16: x b ~ xh bh + xh bl + xl bh, the small terms first
#pragma unroll
      for (int kc = 0; kc < TK; kc += 16) {
        const int kq = kc + 8 * (lane >> 5);
        bf16x8 xh[2], xl[2], bh8[2], bl8[2];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int i = 0; i < 2; ++i) {
            const float x = xs[(32 * i + (lane & 31)) * XPAD + kq + q];
            const __bf16 hi = (__bf16)x;
            xh[i][q] = hi;
            xl[i][q] = (__bf16)(x - (float)hi);
          }
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const float v = b[kc + 8 * c + q];
            const __bf16 hi = (__bf16)v;
            bh8[c][q] = hi;
            bl8[c][q] = (__bf16)(v - (float)hi);
          }
        }
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[i], bh8[c], acc[i][c], 0, 0, 0);
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], bl8[c], acc[i][c], 0, 0, 0);
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], bh8[c], acc[i][c], 0, 0, 0);
          }
      }
    }
  };
  // one step, without branches: the next step's gathers and rows of A and the
  // index words of the step after are issued before this step's products; one
  // barrier per step (the X tile is double-buffered)
  auto step = [&](int k0, const float (&bcur)[TK], float (&bnext)[TK], const float *xcur, float *xnext) {
    load_values(k0 + TK, bnext);
    load_index(k0 + 2 * TK);
    products(xcur, bcur);
    store_x(xnext);
    __syncthreads();
  };

  float b0[TK], b1[TK];
  load_index(0);
  load_values(0, b0);
  load_index(TK);
  store_x(Xs[0]);
  __syncthreads();
  // steps past the pass's coordinates multiply zero rows of A
  for (int k0 = 0; k0 < a.sc; k0 += 2 * TK) {
    step(k0, b0, b1, Xs[0], Xs[1]);
    step(k0 + TK, b1, b0, Xs[1], Xs[0]);
  }

  // epilogue: acc[i][c][v] is element (32 i + 8 (v / 4) + 4 (lane / 32) + v % 4,
  // wc + 32 c + lane % 32) of the tile
  auto row_of = [&](int i, int v) { return 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); };
  const int colw = ct * TN + wc + (lane & 31);
  if (IDX && a.root) {  // the upper levels' sum, P[n mod nsplit] (nsplit >= 64; base b > 2 only)
    const float *rt = a.root + (int64_t)rl * a.root_stride;
    const int64_t base = n0 % a.nsplit;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        int64_t p = base + row_of(i, v);
        if (p >= a.nsplit) p -= a.nsplit;
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[i][c][v] += rt[p * a.ldp + min(colw + 32 * c, a.t - 1)];
      }
  }
  if (MODE == kModeStoreY) {
    Y += (int64_t)rl * a.ystride;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = n0 + row_of(i, v);
          const int col = colw + 32 * c;
          if (row < a.N && col < a.t) Y[row * a.ldy + col] = a.sigma * acc[i][c][v];
        }
    return;
  }
  float gv[2][2][16];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const bool ok = n0 + row_of(i, v) < a.N && colw + 32 * c < a.t;
        gv[i][c][v] = ok ? g_val<GF>(a.sigma * acc[i][c][v]) : 0.f;
      }
  if (MODE == kModeSum) {
    float sl = 0.f;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int v = 0; v < 16; ++v) sl += gv[i][c][v];
    double d = (double)sl;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
    if (lane == 0) red[w] = d;
    __syncthreads();
    if (tid == 0)
      partial[((int64_t)rl * a.ntiles + tn) * a.tct + ct] = ((red[0] + red[1]) + red[2]) + red[3];
    return;
  }
  // kModePoint: per row, the sum over this wave's 64 columns (both column
  // blocks, then the 32 lanes with equal lane / 32), then over the 4 waves
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      float r = gv[i][0][v] + gv[i][1][v];
#pragma unroll
      for (int o = 16; o >= 1; o >>= 1) r += __shfl_xor(r, o, 64);
      if ((lane & 31) == 0) rsum[w][row_of(i, v)] = r;
    }
  __syncthreads();
  if (tid < TM && n0 + tid < a.N)
    ppart[((int64_t)rl * a.tct + ct) * a.N + n0 + tid] =
        ((rsum[0][tid] + rsum[1][tid]) + rsum[2][tid]) + rsum[3][tid];
}

template <int PREC, int MODE, int IDX>
static void launch_g(int gf, dim3 grid, hipStream_t st, const Alg4Args &a, const DevSpec &D,
                     const float *tab, const float *A, const Alg4Out &o) {
#define QMC_ALG4(GF)                                                                                    \
  hipLaunchKernelGGL((alg4_kernel<PREC, MODE, GF, IDX>), grid, dim3(256), 0, st, a, D, tab, A, o.Y, \
                     o.partial, o.ppart)
  if (gf == QMC_G_COS) QMC_ALG4(QMC_G_COS);
  else if (gf == QMC_G_EXP) QMC_ALG4(QMC_G_EXP);
  else QMC_ALG4(QMC_G_ID);
#undef QMC_ALG4
}

template <int PREC, int IDX>
static void launch_m(int mode, int gf, dim3 grid, hipStream_t st, const Alg4Args &a,
                     const DevSpec &D, const float *tab, const float *A, const Alg4Out &o) {
  if (mode == kModeStoreY) launch_g<PREC, kModeStoreY, IDX>(QMC_G_ID, grid, st, a, D, tab, A, o);
  else if (mode == kModeSum) launch_g<PREC, kModeSum, IDX>(gf, grid, st, a, D, tab, A, o);
  else launch_g<PREC, kModePoint, IDX>(gf, grid, st, a, D, tab, A, o);
}

}  // namespace

// Index words of the gather path (layout at DevSpec::aoff).  Nets (add = 0):
// ylo[j][r] = y_j(r) for r < 64 (rows past N: digits that do not exist are
// dropped) and ytile[h][j] = aoff_j XOR y_j(64 h), each word restricted to its
// first n_j digits; aoff_j is a multiple of n_j, so aoff_j XOR y = aoff_j + y
// for y < n_j.  Base b > 2 (add = 1): ylo[j][r] = r mod n_j and ytile[h][j] =
// aoff_j + (64 h mod n_j), whose sum stays below aoff_j + 2 n_j.
__global__ __launch_bounds__(256) void alg4_index_kernel(int32_t m, int32_t s, int32_t b, int64_t ntiles,
                                                         const uint32_t *__restrict__ gen,
                                                         const int32_t *__restrict__ nbj,
                                                         const uint32_t *__restrict__ aoff,
                                                         uint32_t *__restrict__ ylo,
                                                         uint32_t *__restrict__ ytile) {
  const int64_t nlo = (int64_t)64 * s, total = nlo + ntiles * s;
  const uint32_t lowmask = m >= 6 ? 63u : ((1u << m) - 1u);
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const bool lo = e < nlo;
    const int64_t h = lo ? 0 : (e - nlo) / s;
    const int64_t j = lo ? e >> 6 : (e - nlo) - h * s;
    const int nb = nbj[j];
    if (b != 2) {
      uint64_t n = 1;
      for (int i = 0; i < nb; ++i) n *= (uint32_t)b;
      if (lo) ylo[e] = (uint32_t)((uint64_t)(e & 63) % n);
      else ytile[e - nlo] = aoff[j] + (uint32_t)((uint64_t)(64 * h) % n);
      continue;
    }
    const uint32_t *col = gen + j * m;
    const uint32_t msk = nb >= 32 ? 0xffffffffu : (1u << nb) - 1u;
    uint32_t y = 0;
    if (lo) {
      for (uint32_t bits = (uint32_t)(e & 63) & lowmask; bits; bits &= bits - 1u) y ^= col[__builtin_ctz(bits)];
      ylo[e] = y & msk;
    } else {
      for (uint32_t bits = (uint32_t)h; bits; bits &= bits - 1u) y ^= col[6 + __builtin_ctz(bits)];
      ytile[e - nlo] = aoff[j] ^ (y & msk);
    }
  }
}

int64_t alg4_point_tiles(const Geometry &G) { return ceil_div(G.N, TM); }

int64_t alg4_index_words(const Geometry &G) { return (64 + alg4_point_tiles(G)) * G.s; }

int alg4_col_tiles(int t) { return (int)ceil_div(t, TN); }

hipError_t launch_alg4_index(const Geometry &G, const uint32_t *gen, const int32_t *nbj, const uint32_t *aoff,
                             uint32_t *ylo, uint32_t *ytile, hipStream_t st) {
  const int64_t total = alg4_index_words(G);
  const int64_t blocks = std::min<int64_t>(ceil_div(total, 256), 65535);
  hipLaunchKernelGGL(alg4_index_kernel, dim3((unsigned)blocks), dim3(256), 0, st, G.m, G.s, G.b,
                     alg4_point_tiles(G), gen, nbj, aoff, ylo, ytile);
  return hipGetLastError();
}

Alg4Pass alg4_whole(const Geometry &G) {
  Alg4Pass ps{};
  ps.j0 = 0;
  ps.sc = G.s;
  ps.npts = G.N;
  ps.timer = "leaf";
  return ps;
}

hipError_t launch_alg4(const Geometry &G, const DevSpec &D, int mode, const qmc_integrand &f,
                       int prec, const float *tab, int nr, const float *A, int t, int64_t lda,
                       const Alg4Pass &ps, const Alg4Out &o, hipStream_t st) {
  LaunchTimer tm(ps.timer, st);
  if (mode != kModeStoreY && mode != kModeSum && mode != kModePoint) return hipErrorInvalidValue;
  // byte offsets of a step's rows of A and of the value tables are 32-bit
  if (lda > kAlg4MaxLda || G.gather_total * 4 > 0xffffffffll) return hipErrorInvalidValue;
  if (ps.sc < 1 || ps.j0 < 0 || ps.j0 + ps.sc > G.s || ps.npts < 1 || ps.npts > G.N ||
      (ps.root && ps.nsplit < TM))
    return hipErrorInvalidValue;
  Alg4Args a{};
  a.m = G.m;
  a.s = G.s;
  a.t = t;
  a.tct = alg4_col_tiles(t);
  a.j0 = ps.j0;
  a.sc = ps.sc;
  a.N = ps.npts;
  a.lda = lda;
  a.ldy = o.ldy;
  a.ystride = o.ystride;
  a.tab_stride = G.gather_total;
  a.ntiles = ceil_div(ps.npts, TM);
  a.root = ps.root;
  a.ldp = ps.ldp;
  a.root_stride = ps.root_stride;
  a.nsplit = ps.nsplit;
  a.sigma = g_scale(f, mode);
  A += (int64_t)ps.j0 * lda;
  const dim3 grid((unsigned)a.ntiles, a.tct, nr);
  const bool add = G.b != 2;
  if (prec == QMC_FP32) {
    if (add) launch_m<QMC_FP32, 1>(mode, f.g, grid, st, a, D, tab, A, o);
    else launch_m<QMC_FP32, 0>(mode, f.g, grid, st, a, D, tab, A, o);
  } else {
    if (add) launch_m<QMC_SPLIT_BF16X3, 1>(mode, f.g, grid, st, a, D, tab, A, o);
    else launch_m<QMC_SPLIT_BF16X3, 0>(mode, f.g, grid, st, a, D, tab, A, o);
  }
  return hipGetLastError();
}

}  // namespace qmc
