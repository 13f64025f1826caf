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
//   Grad    the sensitivities G = gscale h'(u_n) g'(y) stored like Y (h' read per
//           point, or 1 for a separable f, which also writes the Sum partials)
//
// The adjoint dA = X^T G (Algorithm 4 transposed) runs on the same tiles with
// the roles of points and coordinates swapped (alg4_adj_kernel below).
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
  int32_t nitems;        // ntiles x tct x randomisations
  int32_t nsteps;        // 32-coordinate steps per item
  int64_t ystride;       // StoreY: floats between the randomisations' outputs
  const float *root;     // optional root table added to y: row n mod nsplit
  int64_t ldp, root_stride, nsplit;
  float sigma;           // y' = sigma y (scale of g)
  float gc;              // Grad: parameter c of exp(c y)
  double gscale;         // Grad: factor of the sensitivities
  const float *hd;       // Grad: per-point factor h'(u_n) ([randomisation][N]) or null
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
// (0: XOR, nets that are not periodic over F_2; 1: add, base b > 2; 2: one
// word per point and coordinate, nets over F_b, b > 2, that are not periodic).
//
// Work items are (64-point tile tn, 256-column tile ct, randomisation rl),
// item = tn + ntiles (ct + tct rl).  A workgroup takes a contiguous range of
// items, the ranges of the workgroups on one XCD adjacent (workgroup b runs on
// XCD b mod 8), so each XCD's L2 holds the tables, rows of A and root rows of
// its own part.  The steps of all its items form one stream: the loads of the
// next step, which may belong to the next item, are in flight during this
// step's products and the finished item's epilogue.
// (FP32 nets run at three waves per SIMD; the other variants need the
// registers of two.)
// STREAM: a workgroup streams a range of short items (see above); otherwise it
// takes the one item blockIdx.x and runs its steps two per loop iteration.
template <int PREC, int MODE, int GF, int IDX, bool STREAM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PREC == QMC_FP32 && !IDX ? 3 : 2))) void alg4_kernel(
    Alg4Args a, DevSpec D, const float *__restrict__ tab, const float *__restrict__ A, float *__restrict__ Y,
    double *__restrict__ partial, float *__restrict__ ppart) {
  __shared__ float Xs[2][TM * XPAD];  // point values, two steps: [point][coordinate]
  __shared__ double red[NWAVE];
  __shared__ float rsum[NWAVE][TM];

  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wc = w * 64;
  int i0, i1;
  if constexpr (STREAM) {
    const int nwg = gridDim.x;  // a multiple of 8
    const int rank = (blockIdx.x & 7) * (nwg >> 3) + (blockIdx.x >> 3);
    i0 = (int)((int64_t)rank * a.nitems / nwg);
    i1 = (int)((int64_t)(rank + 1) * a.nitems / nwg);
  } else {
    i0 = blockIdx.x;
    i1 = min(i0 + 1, a.nitems);
  }
  if (i0 >= i1) return;
  const int nst = a.nsteps;          // steps per item
  const int total = (i1 - i0) * nst;  // steps of this workgroup
  // A position in the stream: step p, coordinate offset k0 inside item
  // (tn, ct, rl).  Cursors advance one step at a time and stop at the last.
  struct Cursor {
    int p, k0, tn, ct, rl;
  };
  Cursor cur;
  {
    const int rest = i0 / (int)a.ntiles;
    cur = Cursor{0, 0, i0 - rest * (int)a.ntiles, rest % a.tct, rest / a.tct};
  }
  auto advance = [&](Cursor c) {
    if (c.p + 1 >= total) return c;
    ++c.p;
    c.k0 += TK;
    if (c.k0 == nst * TK) {
      c.k0 = 0;
      if (++c.tn == (int)a.ntiles) {
        c.tn = 0;
        if (++c.ct == a.tct) {
          c.ct = 0;
          ++c.rl;
        }
      }
    }
    return c;
  };

  // Only wave w reads columns [wc, wc + 64) of the tile, so its B operands come
  // straight from A into registers, one step ahead.  Element e < TK of a lane:
  // row k0 + brow(e) + bh, column bblk(e) (FP32 32x32x2: e = kk + c,
  // bh = lane / 32; BF16 32x32x16: e = kc + 8 c + q, bh = 8 (lane / 32)).
  // Columns past t read column t - 1 (their outputs are dropped); rows past the
  // pass's coordinates read zero (the step's buffer ends there).
  auto brow = [&](int e) { return PREC == QMC_FP32 ? (e & ~1) : (e & ~15) + (e & 7); };
  auto bblk = [&](int e) { return PREC == QMC_FP32 ? (e & 1) : ((e >> 3) & 1); };
  const int bh = PREC == QMC_FP32 ? (lane >> 5) : 8 * (lane >> 5);

  // Step p: wave w gathers coordinates j0 + k0 + KPW w + q (q < KPW) of the 64
  // points of its item (lane = point); a value's byte offset is
  // 4 (ytile_j op ylo_j(lane)).  Coordinates past the pass's last gather that
  // one (its rows of A read zero), points past N gather valid values (their
  // outputs are dropped).
  uint32_t yl[KPW], yt[KPW];  // index words of the next coordinates to gather
  float xv[KPW];
  auto load_index = [&](const Cursor &c) {
    const uint32_t *ytile = D.ytile + (int64_t)c.tn * a.s;
#pragma unroll
    for (int q = 0; q < KPW; ++q) {
      const int j = a.j0 + min(c.k0 + KPW * w + q, a.sc - 1);
      if (IDX == 2) {  // a word per point and coordinate
        yl[q] = D.ylo[((int64_t)c.tn * a.s + j) * 64 + lane];
        yt[q] = 0u;
      } else {
        yl[q] = D.ylo[(int64_t)j * 64 + lane];
        yt[q] = ytile[j];
      }
    }
  };
  // pad: a step past the stream (its rows of A read zero)
  auto load_values = [&](const Cursor &c, bool pad, float (&b)[TK]) {
    const int k0 = c.k0, ct = c.ct;
    const __amdgpu_buffer_rsrc_t trs = raw_rsrc(tab + (int64_t)c.rl * a.tab_stride, (uint32_t)(a.tab_stride * 4));
#pragma unroll
    for (int q = 0; q < KPW; ++q) xv[q] = load_f32(trs, (IDX ? yt[q] + yl[q] : yt[q] ^ yl[q]) << 2);
    // rows of A from row k0 on
    const int64_t left = pad ? 0 : (int64_t)a.sc - k0;
    const int64_t want = ((left - 1) * a.lda + a.t) * 4;
    const uint32_t bytes = left <= 0 ? 0u : want > 0xffffffffll ? 0xffffffffu : (uint32_t)want;
    const __amdgpu_buffer_rsrc_t ars = raw_rsrc(left <= 0 ? A : A + (int64_t)k0 * a.lda, bytes);
    uint32_t boff[2];  // byte offset of this lane's element in row k0 of the step
#pragma unroll
    for (int c = 0; c < 2; ++c)
      boff[c] = (uint32_t)(((int64_t)bh * a.lda + min(ct * TN + wc + 32 * c + (lane & 31), a.t - 1)) * 4);
#pragma unroll
    for (int e = 0; e < TK; ++e) b[e] = load_f32(ars, (uint32_t)(brow(e) * a.lda * 4) + boff[bblk(e)]);
  };
  auto store_x = [&](float *xs) {
#pragma unroll
    for (int q = 0; q < KPW; ++q) xs[lane * XPAD + KPW * w + q] = xv[q];
  };

  // The accumulators start an item at zero, or (base b > 2 with a root table)
  // at the upper levels' sum P[n mod nsplit] of its points (nsplit >= 64), read
  // straight into them.
  auto row_of = [&](int i, int v) { return 32 * i + 8 * (v >> 2) + 4 * (lane >> 5) + (v & 3); };
  f32x16 acc[2][2];
  auto init_acc = [&](const Cursor &c) {
    if (IDX == 1 && a.root) {
      const __amdgpu_buffer_rsrc_t rrs =
          raw_rsrc(a.root + (int64_t)c.rl * a.root_stride, (uint32_t)(a.nsplit * a.ldp * 4));
      const int base = (int)(((int64_t)c.tn * TM) % a.nsplit);
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) {
        const uint32_t col = (uint32_t)min(c.ct * TN + wc + 32 * cc + (lane & 31), a.t - 1);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            int p = base + row_of(i, v);
            if (p >= a.nsplit) p -= (int)a.nsplit;
            acc[i][cc][v] = load_f32(rrs, ((uint32_t)p * (uint32_t)a.ldp + col) * 4u);
          }
      }
    } else {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc) acc[i][cc] = f32x16{0};
    }
  };
  init_acc(cur);

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

  // The finished item's outputs; acc[i][c][v] is element (32 i + 8 (v / 4) +
  // 4 (lane / 32) + v % 4, wc + 32 c + lane % 32) of its tile.
  auto epilogue = [&](const Cursor &c) {
    const int tn = c.tn, ct = c.ct, rl = c.rl;
    const int64_t n0 = (int64_t)tn * TM;
    const int colw = ct * TN + wc + (lane & 31);
    if (MODE == kModeStoreY) {
      float *Yr = Y + (int64_t)rl * a.ystride;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int64_t row = n0 + row_of(i, v);
            const int col = colw + 32 * c;
            if (row < a.N && col < a.t) Yr[row * a.ldy + col] = a.sigma * acc[i][c][v];
          }
    } else if (MODE == kModeGrad) {
      // G = gscale h'(u_n) g'(y), stored like Y; without a per-point factor
      // (separable f) also the tile's sum of g, as in the summing mode
      float *Gr = Y + (int64_t)rl * a.ystride;
      const float *hk = a.hd ? a.hd + (int64_t)rl * a.N : nullptr;
      const float gs = (float)a.gscale;
      float sl = 0.f;
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int64_t row = n0 + row_of(i, v);
          const float fac = (hk && row < a.N) ? hk[row] : 1.0f;
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            const int col = colw + 32 * c;
            const float ys = a.sigma * acc[i][c][v];
            if (row < a.N && col < a.t) {
              Gr[row * a.ldy + col] = gs * (fac * g_der<GF>(ys, a.gc));
              sl += g_val<GF>(ys);
            }
          }
        }
      if (a.hd == nullptr) {
        double d = (double)sl;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) d += __shfl_xor(d, o, 64);
        if (lane == 0) red[w] = d;
        __syncthreads();
        if (tid == 0)
          partial[((int64_t)rl * a.ntiles + tn) * a.tct + ct] = ((red[0] + red[1]) + red[2]) + red[3];
      }
    } else {
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
      } else {
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
    }
  };

  // one step: the next step's gathers and rows of A and the index words of the
  // step after are issued first; then this step's products, the epilogue when
  // it ends an item, the next step's point values into the other X buffer and
  // one barrier (the X tile is double-buffered)
  // cur: this step; nv: the next (its values and rows of A); ni: the one after
  // (its index words).  Each step issues nv's and ni's loads, runs cur's
  // products, the epilogue when cur ends an item, stores nv's point values into
  // the other X buffer (one barrier per step: the X tile is double-buffered)
  // and moves nv's rows of A, which have arrived by then, into the current set.
  float bc[TK], bn[TK];
  if constexpr (STREAM) {
    Cursor nv = advance(cur), ni = advance(nv);
    load_index(cur);
    load_values(cur, false, bc);
    load_index(nv);
    store_x(Xs[0]);
    __syncthreads();
    int xb = 0;
    for (int p = 0; p < total; ++p) {
      load_values(nv, p + 1 >= total, bn);
      load_index(ni);
      products(Xs[xb], bc);
      if (cur.k0 == (nst - 1) * TK) {
        epilogue(cur);
        init_acc(nv);  // the next item's start (its root rows travel over the barrier)
      }
      store_x(Xs[xb ^ 1]);
      __syncthreads();
#pragma unroll
      for (int e = 0; e < TK; ++e) bc[e] = bn[e];  // nv's rows of A have arrived
      xb ^= 1;
      cur = nv;
      nv = ni;
      ni = advance(ni);
    }
  } else {
    // one item: steps k0 = 0, 32, ... two per iteration, the operand buffers
    // swapped by name; steps past the pass's coordinates multiply zero rows
    auto at = [&](int k0) { return Cursor{0, k0, cur.tn, cur.ct, cur.rl}; };
    load_index(at(0));
    load_values(at(0), false, bc);
    load_index(at(TK));
    store_x(Xs[0]);
    __syncthreads();
    auto step = [&](int k0, const float (&bcur)[TK], float (&bnext)[TK], const float *xcur, float *xnext) {
      load_values(at(k0 + TK), false, bnext);
      load_index(at(k0 + 2 * TK));
      products(xcur, bcur);
      store_x(xnext);
      __syncthreads();
    };
    for (int k0 = 0; k0 < a.sc; k0 += 2 * TK) {
      step(k0, bc, bn, Xs[0], Xs[1]);
      step(k0 + TK, bn, bc, Xs[1], Xs[0]);
    }
    epilogue(cur);
  }
}

// ------------------------------------------------------------------ adjoint
// dA = X^T G over the points of a pass.  Read as Algorithm 4 transposed, every
// point adds its sensitivities G_n to the value it selects in each coordinate,
// and dA_j is the sum over values of X_j[c] times that sum: X^T G with the
// gathered point matrix, which is what the matrix cores evaluate.  The tiles of
// the forward pass with the roles of points and coordinates swapped: a
// workgroup owns 32 MI coordinates x 256 columns of dA (MI = 1 for a pass of
// at most 32 coordinates, else 2) and contracts over one chunk of points, 32
// per step.  The X^T tile (coordinate-major, gathered as in
// the forward pass, lane = point) is double-buffered in LDS; the rows of G come
// straight from HBM into the B operand, one step ahead.  The matrix cores
// accumulate in FP32 over at most kAdjFlushPoints points; then the
// accumulators are added into the chunk's FP64 partial of the pass's sc rows
// (owned by this workgroup alone) and restart from zero, so no FP32 sum runs
// over more than kAdjFlushPoints terms whatever the chunk size.
// alg4_adj_combine adds the chunks in FP64, in chunk order.
struct AdjArgs {
  int32_t s, t, tct;
  int32_t j0, sc, jtiles;          // coordinates [j0, j0 + sc) in tiles of 64
  int32_t nchunk, ngroups;         // ngroups = column tiles x chunks x randomisations
  int64_t npts, chunk;             // points of the pass; points per chunk (a multiple of 64)
  int64_t ldg, gstride;            // G: row stride, floats per randomisation
  int64_t tab_stride, ntiles_tab;  // value tables per randomisation; point tiles of the index words
};

constexpr int kAdjFlushSteps = kAdjFlushPoints / TK;
static_assert(kAdjFlushSteps % 2 == 0, "the step loop advances two steps at a time");

template <int PREC, int IDX, int MI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void alg4_adj_kernel(
    AdjArgs a, DevSpec D, const float *__restrict__ tab, const float *__restrict__ Gm,
    double *__restrict__ part) {
  constexpr int TMA = 32 * MI, KPL = 4 * MI;  // coordinates per tile, gathers per lane and step
  __shared__ float Xs[2][TMA * XPAD];  // two steps of X^T: [coordinate][point]
  const int tid = threadIdx.x, lane = tid & 63, pl = lane & 31, hh = lane >> 5;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int wc = w * 64;
  // The jtiles workgroups of one (column tile, chunk, randomisation) group read
  // the same rows of G: they run on one XCD (workgroup b runs on XCD b mod 8),
  // so its L2 fetches those rows once.  Groups past the last are padding.
  const int xcd = blockIdx.x & 7, k8 = blockIdx.x >> 3;
  int it = (k8 / a.jtiles) * 8 + xcd;
  const int jt = k8 % a.jtiles;
  if (it >= a.ngroups) return;
  const int ct = it % a.tct;
  it /= a.tct;
  const int ch = it % a.nchunk;
  const int rl = it / a.nchunk;
  const int64_t p0 = (int64_t)ch * a.chunk;
  const int64_t p1 = min(p0 + a.chunk, a.npts);
  const int64_t nst = p1 > p0 ? (p1 - p0 + TK - 1) / TK : 0;
  const float *tabr = tab + (int64_t)rl * a.tab_stride;
  const float *Gr = Gm + (int64_t)rl * a.gstride;

  // this lane's gathers: coordinates 16 MI hh + 4 MI w + q (q < KPL) of the
  // tile, at point pl of the step (past the pass's coordinates: the last one,
  // dropped)
  auto crow = [&](int q) { return 16 * MI * hh + 4 * MI * w + q; };
  int jq[KPL];
#pragma unroll
  for (int q = 0; q < KPL; ++q) jq[q] = a.j0 + min(TMA * jt + crow(q), a.sc - 1);
  // B element e (as in the forward pass): row (point) kp + brow(e) + bh of G
  auto brow = [&](int e) { return PREC == QMC_FP32 ? (e & ~1) : (e & ~15) + (e & 7); };
  auto bblk = [&](int e) { return PREC == QMC_FP32 ? (e & 1) : ((e >> 3) & 1); };
  const int bh = PREC == QMC_FP32 ? hh : 8 * hh;

  // index words of the step at point kp (a multiple of 32): tile kp / 64, in
  // which the lane's point is 32 (kp / 32 mod 2) + pl; steps past the chunk
  // gather valid values (their rows of G read zero)
  uint32_t yl[KPL], yt[KPL];
  float xv[KPL];
  auto load_index = [&](int64_t kp) {
    const int64_t tn = min(kp >> 6, a.ntiles_tab - 1);
    const int r = 32 * (int)((kp >> 5) & 1) + pl;
#pragma unroll
    for (int q = 0; q < KPL; ++q) {
      if (IDX == 2) {
        yl[q] = D.ylo[((int64_t)tn * a.s + jq[q]) * 64 + r];
        yt[q] = 0u;
      } else {
        yl[q] = D.ylo[(int64_t)jq[q] * 64 + r];
        yt[q] = D.ytile[tn * a.s + jq[q]];
      }
    }
  };
  auto load_values = [&](int64_t kp, float (&b)[TK]) {
    const __amdgpu_buffer_rsrc_t trs = raw_rsrc(tabr, (uint32_t)(a.tab_stride * 4));
#pragma unroll
    for (int q = 0; q < KPL; ++q) xv[q] = load_f32(trs, (IDX ? yt[q] + yl[q] : yt[q] ^ yl[q]) << 2);
    const int64_t left = p1 - kp;  // rows of G of this chunk from row kp on
    const int64_t want = ((left - 1) * a.ldg + a.t) * 4;
    const uint32_t bytes = left <= 0 ? 0u : want > 0xffffffffll ? 0xffffffffu : (uint32_t)want;
    const __amdgpu_buffer_rsrc_t grs = raw_rsrc(left <= 0 ? Gr : Gr + kp * a.ldg, bytes);
    uint32_t boff[2];
#pragma unroll
    for (int c = 0; c < 2; ++c)
      boff[c] = (uint32_t)(((int64_t)bh * a.ldg + min(ct * TN + wc + 32 * c + pl, a.t - 1)) * 4);
#pragma unroll
    for (int e = 0; e < TK; ++e) b[e] = load_f32(grs, (uint32_t)(brow(e) * a.ldg * 4) + boff[bblk(e)]);
  };
  auto store_x = [&](float *xs) {
#pragma unroll
    for (int q = 0; q < KPL; ++q) xs[crow(q) * XPAD + pl] = xv[q];
  };

  f32x16 acc[MI][2];
#pragma unroll
  for (int i = 0; i < MI; ++i)
#pragma unroll
    for (int c = 0; c < 2; ++c) acc[i][c] = f32x16{0};

  // the forward pass's product step: acc[i][c] += (rows 32 i.. of the tile) x
  // (this wave's columns 32 c..), here rows = coordinates and k = points
  auto products = [&](const float *xs, const float (&b)[TK]) {
    if (PREC == QMC_FP32) {
#pragma unroll
      for (int kk = 0; kk < TK; kk += 2) {
        float x[MI];
#pragma unroll
        for (int i = 0; i < MI; ++i) x[i] = xs[(32 * i + pl) * XPAD + kk + hh];
#pragma unroll
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int c = 0; c < 2; ++c)
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x2f32(x[i], b[kk + c], acc[i][c], 0, 0, 0);
      }
    } else {
#pragma unroll
      for (int kc = 0; kc < TK; kc += 16) {
        const int kq = kc + 8 * hh;
        bf16x8 xh[MI], xl[MI], bh8[2], bl8[2];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
#pragma unroll
          for (int i = 0; i < MI; ++i) {
            const float x = xs[(32 * i + pl) * XPAD + kq + q];
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
        for (int i = 0; i < MI; ++i)
#pragma unroll
          for (int c = 0; c < 2; ++c) {
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xl[i], bh8[c], acc[i][c], 0, 0, 0);
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], bl8[c], acc[i][c], 0, 0, 0);
            acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[i], bh8[c], acc[i][c], 0, 0, 0);
          }
      }
    }
  };

  // steps kp = p0, p0 + 32, ... two per iteration, the operand buffers swapped
  // by name; a step past the chunk multiplies zero rows of G
  float bc[TK], bn[TK];
  load_index(p0);
  load_values(p0, bc);
  load_index(p0 + TK);
  store_x(Xs[0]);
  __syncthreads();
  auto step = [&](int64_t kp, const float (&bcur)[TK], float (&bnext)[TK], const float *xcur, float *xnext) {
    load_values(kp + TK, bnext);
    load_index(kp + 2 * TK);
    products(xcur, bcur);
    store_x(xnext);
    __syncthreads();
  };
  // acc[i][c][v] is element (32 i + 8 (v / 4) + 4 hh + v % 4, wc + 32 c + pl)
  // of the 32 MI x 256 tile; the partial holds the pass's rows j0 .. j0 + sc - 1
  double *Pr = part + ((int64_t)rl * a.nchunk + ch) * a.sc * (int64_t)a.t;
  auto flush = [&](bool first) {
#pragma unroll
    for (int i = 0; i < MI; ++i)
#pragma unroll
      for (int c = 0; c < 2; ++c) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          const int jj = TMA * jt + 32 * i + 8 * (v >> 2) + 4 * hh + (v & 3);
          const int col = ct * TN + wc + 32 * c + pl;
          if (jj < a.sc && col < a.t) {
            double *d = Pr + (int64_t)jj * a.t + col;
            *d = (first ? 0.0 : *d) + (double)acc[i][c][v];
          }
        }
        acc[i][c] = f32x16{0};
      }
  };
  // sub-chunks of kAdjFlushSteps steps (an even count, so only the last
  // sub-chunk can run one step past the chunk: that step reads zero rows of G)
  for (int64_t k0 = 0; k0 < nst || k0 == 0; k0 += kAdjFlushSteps) {
    const int64_t k1 = min(k0 + (int64_t)kAdjFlushSteps, nst);
    for (int64_t k = k0; k < k1; k += 2) {
      step(p0 + k * TK, bc, bn, Xs[0], Xs[1]);
      step(p0 + (k + 1) * TK, bn, bc, Xs[1], Xs[0]);
    }
    flush(k0 == 0);
  }
}

// dA[r][j][i] = sum over chunks of the partials, FP64, chunk order: rows
// j < jlow from the lower pass (plo[r][chunk][j][i], nlo chunks), the others
// from the upper pass (pup[r][chunk][j - jlow][i], nup chunks).
__global__ __launch_bounds__(256) void alg4_adj_combine(const double *__restrict__ plo, int nlo,
                                                        const double *__restrict__ pup, int nup, int s, int jlow,
                                                        int t, int64_t total, float *__restrict__ dA) {
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t per = (int64_t)s * t;
    const int64_t rl = e / per, o = e - rl * per;
    const int64_t j = o / t;
    const bool lo = j < jlow;
    const int n = lo ? nlo : nup;
    const int64_t pper = (int64_t)(lo ? jlow : s - jlow) * t;
    const double *p = (lo ? plo : pup) + rl * n * pper + (lo ? o : o - (int64_t)jlow * t);
    double acc = 0.0;
#pragma unroll 8
    for (int c = 0; c < n; ++c) acc += p[c * pper];  // eight loads in flight, order kept
    dA[e] = (float)acc;
  }
}

// S[r][rho][i] = sum of G[r][n][i] over n = rho mod nsplit (FP64, increasing n):
// the sensitivities of the residues of the upper coordinates (n_j | nsplit).
// V consecutive columns per thread (V = 4 when t is a multiple of 4).
template <int V>
__global__ __launch_bounds__(256) void alg4_fold_kernel(const float *__restrict__ Gm, int64_t N, int64_t nsplit,
                                                        int t, int64_t total, float *__restrict__ S) {
  typedef float fv __attribute__((ext_vector_type(V)));
  const int tv = t / V;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t per = nsplit * tv;
    const int64_t rl = e / per, o = e - rl * per;
    const int64_t rho = o / tv, cv = o - rho * tv;
    const fv *g = reinterpret_cast<const fv *>(Gm + rl * N * t) + cv;
    double acc[V];
#pragma unroll
    for (int k = 0; k < V; ++k) acc[k] = 0.0;
#pragma unroll 4
    for (int64_t n = rho; n < N; n += nsplit) {
      const fv x = g[n * tv];
#pragma unroll
      for (int k = 0; k < V; ++k) acc[k] += (double)x[k];
    }
    fv out;
#pragma unroll
    for (int k = 0; k < V; ++k) out[k] = (float)acc[k];
    reinterpret_cast<fv *>(S + (rl * nsplit + rho) * t)[cv] = out;
  }
}

template <int PREC>
static const void *adj_fn(int idx, int mi) {
  if (idx == 2) return mi == 1 ? reinterpret_cast<const void *>(&alg4_adj_kernel<PREC, 2, 1>)
                               : reinterpret_cast<const void *>(&alg4_adj_kernel<PREC, 2, 2>);
  if (idx == 1) return mi == 1 ? reinterpret_cast<const void *>(&alg4_adj_kernel<PREC, 1, 1>)
                               : reinterpret_cast<const void *>(&alg4_adj_kernel<PREC, 1, 2>);
  return mi == 1 ? reinterpret_cast<const void *>(&alg4_adj_kernel<PREC, 0, 1>)
                 : reinterpret_cast<const void *>(&alg4_adj_kernel<PREC, 0, 2>);
}

// The index mode of a point set (see IDX at alg4_kernel).
static int index_mode(const Geometry &G) { return G.b == 2 ? 0 : G.nonperiodic ? 2 : 1; }

template <int PREC, int MODE, int IDX, bool STREAM>
static const void *fn_g(int gf) {
  if (gf == QMC_G_COS) return reinterpret_cast<const void *>(&alg4_kernel<PREC, MODE, QMC_G_COS, IDX, STREAM>);
  if (gf == QMC_G_EXP) return reinterpret_cast<const void *>(&alg4_kernel<PREC, MODE, QMC_G_EXP, IDX, STREAM>);
  return reinterpret_cast<const void *>(&alg4_kernel<PREC, MODE, QMC_G_ID, IDX, STREAM>);
}

template <int PREC, int IDX, bool STREAM>
static const void *fn_m(int mode, int gf) {
  if (mode == kModeStoreY) return fn_g<PREC, kModeStoreY, IDX, STREAM>(QMC_G_ID);
  if (mode == kModeSum) return fn_g<PREC, kModeSum, IDX, STREAM>(gf);
  if (mode == kModeGrad) return fn_g<PREC, kModeGrad, IDX, STREAM>(gf);
  return fn_g<PREC, kModePoint, IDX, STREAM>(gf);
}

template <int PREC>
static const void *fn_p(int idx, bool stream, int mode, int gf) {
  if (idx == 2) return stream ? fn_m<PREC, 2, true>(mode, gf) : fn_m<PREC, 2, false>(mode, gf);
  if (idx == 1) return stream ? fn_m<PREC, 1, true>(mode, gf) : fn_m<PREC, 1, false>(mode, gf);
  return stream ? fn_m<PREC, 0, true>(mode, gf) : fn_m<PREC, 0, false>(mode, gf);
}

}  // namespace

// Index words of the gather path (layout at DevSpec::aoff).  Nets (add = 0):
// ylo[j][r] = y_j(r) for r < 64 (rows past N: digits that do not exist are
// dropped) and ytile[h][j] = aoff_j XOR y_j(64 h), each word restricted to its
// first n_j digits; aoff_j is a multiple of n_j, so aoff_j XOR y = aoff_j + y
// for y < n_j.  Base b > 2 (add = 1): ylo[j][r] = r mod n_j and ytile[h][j] =
// aoff_j + (64 h mod n_j), whose sum stays below aoff_j + 2 n_j.  A net over
// F_b, b > 2, that is not periodic (full): its output digits have no such
// split (digit-wise sums mod b carry no structure an integer add or XOR
// reproduces), so ylo holds one word aoff_j + c per point and coordinate,
// [tile][j][r], and ytile is unused.
// Net over F_b (column words hold C_{p,q} as base-b digit p-1): the integer
// c = sum_{p <= nb} y_p b^{nb-p} of the output digits y_p = sum_q C_{p,q} n_q
// mod b of point n (all m digits of n; rows past nb of the reduced matrix are
// zero).
__device__ uint32_t net_output_int_b(const uint32_t *__restrict__ col, int m, int b, int nb, uint64_t n) {
  uint32_t y[32];
  for (int p = 0; p < nb; ++p) y[p] = 0u;
  for (int q = 0; q < m; ++q) {
    const uint32_t d = (uint32_t)(n % (uint32_t)b);
    n /= (uint32_t)b;
    if (!d) continue;
    uint32_t wd = col[q];
    for (int p = 0; p < nb; ++p) {
      y[p] = (uint32_t)((y[p] + (uint64_t)(wd % (uint32_t)b) * d) % (uint32_t)b);
      wd /= (uint32_t)b;
    }
  }
  uint32_t c = 0;
  for (int p = 0; p < nb; ++p) c = c * (uint32_t)b + y[p];
  return c;
}

__global__ __launch_bounds__(256) void alg4_index_kernel(int32_t m, int32_t s, int32_t b, int64_t ntiles,
                                                         int64_t N, bool full,
                                                         const uint32_t *__restrict__ gen,
                                                         const int32_t *__restrict__ nbj,
                                                         const uint32_t *__restrict__ aoff,
                                                         uint32_t *__restrict__ ylo,
                                                         uint32_t *__restrict__ ytile) {
  if (full) {
    // word [h][j][r]: aoff_j + the output integer of point min(64 h + r, N - 1)
    const int64_t total = ntiles * s * 64;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
      const int64_t h = e / ((int64_t)s * 64);
      const int j = (int)((e / 64) % s);
      const int64_t n = min((int64_t)64 * h + (e & 63), N - 1);
      ylo[e] = aoff[j] + net_output_int_b(gen + (int64_t)j * m, m, b, nbj[j], (uint64_t)n);
    }
    return;
  }
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

int64_t alg4_index_words(const Geometry &G) {
  if (G.b != 2 && G.nonperiodic) return alg4_point_tiles(G) * 64 * G.s;  // one word per point and coordinate
  return (64 + alg4_point_tiles(G)) * G.s;
}

int alg4_col_tiles(int t) { return (int)ceil_div(t, TN); }

hipError_t launch_alg4_index(const Geometry &G, const uint32_t *gen, const int32_t *nbj, const uint32_t *aoff,
                             uint32_t *ylo, uint32_t *ytile, hipStream_t st) {
  const int64_t total = alg4_index_words(G);
  const int64_t blocks = std::min<int64_t>(ceil_div(total, 256), 65535);
  hipLaunchKernelGGL(alg4_index_kernel, dim3((unsigned)blocks), dim3(256), 0, st, G.m, G.s, G.b,
                     alg4_point_tiles(G), G.N, G.b != 2 && G.nonperiodic != 0, gen, nbj, aoff, ylo, ytile);
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
  if (mode != kModeStoreY && mode != kModeSum && mode != kModePoint && mode != kModeGrad)
    return hipErrorInvalidValue;
  // byte offsets of a step's rows of A and of the value tables are 32-bit
  if (lda > kAlg4MaxLda || G.gather_total * 4 > 0xffffffffll) return hipErrorInvalidValue;
  if (ps.sc < 1 || ps.j0 < 0 || ps.j0 + ps.sc > G.s || ps.npts < 1 || ps.npts > G.N ||
      (ps.root && (ps.nsplit < TM || ps.ldp < t || ps.nsplit * ps.ldp * 4 > 0xffffffffll)))
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
  a.gc = (float)f.c;
  a.gscale = o.gscale;
  a.hd = o.hd;
  const int64_t nitems = a.ntiles * a.tct * nr;
  if (nitems > 0x7fffffffll) return hipErrorInvalidValue;
  a.nitems = (int32_t)nitems;
  a.nsteps = (int32_t)ceil_div(ps.sc, TK);
  const int idx = index_mode(G);
  const int gf = mode == kModeStoreY ? QMC_G_ID : f.g;
  // Items of four or more steps hide their own start and end: one item per
  // workgroup, scheduled by the hardware.  Shorter items (the lower pass of a
  // base b > 2): one resident wave of workgroups (a multiple of 8, one share
  // per XCD), each streaming a contiguous range of items.
  const bool stream = a.nsteps < 4;
  const void *fn = prec == QMC_FP32 ? fn_p<QMC_FP32>(idx, stream, mode, gf) : fn_p<QMC_SPLIT_BF16X3>(idx, stream, mode, gf);
  int64_t wgs = nitems;
  if (stream) wgs = round_up(std::min<int64_t>(nitems, std::max<int64_t>(resident_workgroups(fn, 256, 0), 8)), 8);
  const float *Ap = A + (int64_t)ps.j0 * lda;
  float *Y = o.Y;
  double *partial = o.partial;
  float *ppart = o.ppart;
  DevSpec Dv = D;
  void *args[] = {&a, &Dv, &tab, &Ap, &Y, &partial, &ppart};
  const hipError_t e = hipLaunchKernel(fn, dim3((unsigned)wgs), dim3(256), args, 0, st);
  return e != hipSuccess ? e : hipGetLastError();
}

int alg4_adj_chunks(int sc, int64_t npts, int t, int nr) {
  // about 1024 workgroups over the pass's tiles, chunks of at least 256 points
  // (8 steps), and at most 2^26 FP64 partials
  if (sc < 1) return 0;
  const int64_t items = ceil_div(sc, sc <= 32 ? 32 : TM) * alg4_col_tiles(t) * (int64_t)nr;
  int64_t nch = ceil_div(1024, items);
  nch = std::min<int64_t>(nch, ceil_div(npts, 256));
  nch = std::min<int64_t>(nch, (int64_t(1) << 26) / std::max<int64_t>((int64_t)nr * sc * t, 1));
  return (int)std::max<int64_t>(nch, 1);
}

hipError_t launch_alg4_adj(const Geometry &G, const DevSpec &D, int prec, const float *tab, int nr,
                           const float *Gm, int64_t gstride, int j0, int sc, int64_t npts, int nchunk, int t,
                           double *part, hipStream_t st) {
  LaunchTimer tm("adjoint", st);
  if (nr == 0) return hipSuccess;
  if (sc < 1 || j0 < 0 || j0 + sc > G.s || npts < 1 || npts > G.N || nchunk < 1 || t > kAlg4MaxLda ||
      G.gather_total * 4 > 0xffffffffll)
    return hipErrorInvalidValue;
  AdjArgs a{};
  a.s = G.s;
  a.t = t;
  a.tct = alg4_col_tiles(t);
  a.j0 = j0;
  a.sc = sc;
  const int mi = sc <= 32 ? 1 : 2;
  a.jtiles = (int)ceil_div(sc, 32 * mi);
  a.nchunk = nchunk;
  a.npts = npts;
  a.chunk = round_up(ceil_div(npts, nchunk), TM);
  a.ldg = t;
  a.gstride = gstride;
  a.tab_stride = G.gather_total;
  a.ntiles_tab = alg4_point_tiles(G);
  const int64_t groups = (int64_t)a.tct * nchunk * nr;
  const int64_t items = round_up(groups, 8) * a.jtiles;  // whole groups of 8 (one per XCD)
  if (items > 0x7fffffffll) return hipErrorInvalidValue;
  a.ngroups = (int32_t)groups;
  const int idx = index_mode(G);
  const void *fn = prec == QMC_FP32 ? adj_fn<QMC_FP32>(idx, mi) : adj_fn<QMC_SPLIT_BF16X3>(idx, mi);
  void *args[] = {&a, const_cast<DevSpec *>(&D), &tab, &Gm, &part};
  const hipError_t e = hipLaunchKernel(fn, dim3((unsigned)items), dim3(256), args, 0, st);
  return e != hipSuccess ? e : hipGetLastError();
}

hipError_t launch_alg4_fold(const Geometry &G, const float *Gm, int nr, int t, float *S, hipStream_t st) {
  LaunchTimer tm("fold", st);
  const int V = t % 4 == 0 ? 4 : 1;
  const int64_t total = (int64_t)nr * G.nsub * (t / V);
  if (total == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(ceil_div(total, 256), 16384);
  if (V == 4)
    hipLaunchKernelGGL(alg4_fold_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, Gm, G.N, G.nsub, t, total, S);
  else
    hipLaunchKernelGGL(alg4_fold_kernel<1>, dim3((unsigned)blocks), dim3(256), 0, st, Gm, G.N, G.nsub, t, total, S);
  return hipGetLastError();
}

hipError_t launch_alg4_adj_combine(const Geometry &G, const double *plo, int nlo, const double *pup, int nup, int nr,
                                   int t, float *dA, hipStream_t st) {
  LaunchTimer tm("combine", st);
  const int64_t total = (int64_t)G.s * t * nr;
  if (total == 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(ceil_div(total, 256), 8192);
  hipLaunchKernelGGL(alg4_adj_combine, dim3((unsigned)blocks), dim3(256), 0, st, plo, nlo, pup, nup, G.s, G.jlow, t,
                     total, dA);
  return hipGetLastError();
}

}  // namespace qmc
