// Device helpers shared by the fused leaf kernels (leaf.hip: the summing,
// per-point, matrix-vector and LDS-accumulating gradient modes; adjoint.hip:
// the register form of the gradient mode).  See leaf.hip for the layout of a
// subtree record and the meaning of the descent.
#pragma once

#include <type_traits>

#include "qmc_internal.h"

namespace qmc {

constexpr int kRootBatch = 8;  // upper-level rows of a subtree root loaded together (summing mode)
constexpr int kStagePerThread = 8;  // elements of A per thread and staging pass
static_assert(kMaxUpPadded % kRootBatch == 0, "root batches must tile the padded level arrays");

// Summing mode, lean form.  A lane carries CPL columns of A (the wave 64 CPL
// columns), so every point value loaded into a scalar register feeds CPL
// multiply-adds.  Only the per-level counts tau_I travel with the kernel (one
// byte per level); the record offset and the first row of A of a level follow
// from the counts while descending, so few scalar registers stay live.  The
// point values of up to kBatchFloats nodes x coordinates and their rows of A
// are requested together, then consumed: one memory round trip per batch
// instead of one per coordinate.  The scalar loads may read up to 31 floats
// past a level's block (the point tables carry padding at their end); the LDS
// reads of A up to 7 rows past a level's rows (kLdsPadRows zero rows follow
// the staged rows).
constexpr int kBatchFloats = 32;

template <int NC, int CPL>
constexpr int batch_coords() {
  constexpr int cap = 8 / CPL;  // rows of A per batch (B x CPL registers)
  return NC >= kBatchFloats ? 1 : (kBatchFloats / NC < cap ? kBatchFloats / NC : cap);
}

template <int N>
__device__ __forceinline__ void keep_scalar(const float (&v)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) asm volatile("" ::"s"(v[i]));
}

// A point value of the record: from global memory through the scalar cache,
// or (VX) from the wave's LDS copy, moved to a scalar register, so that a
// batch occupies scalar registers only in either case.
template <bool VX>
__device__ __forceinline__ float ldx(const float *__restrict__ x, int i) {
  if constexpr (VX) return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(x[i])));
  else return x[i];
}

// Records of at most kRecLds floats can be copied to a per-wave LDS slot
// (storing and per-point modes); the slot has room for the descent's reads
// past a level's block.
constexpr int kRecLds = 512;
constexpr int kRecSlot = kRecLds + kBatchFloats;

// VX: the record is in LDS (see ldx).
template <int LP, int L, int LAST, int CPL, bool VX = false>
__device__ __forceinline__ void descend_lean(float (&y)[CPL][1 << LP], const float *__restrict__ rec,
                                             int &xo, int &j0, uint64_t taus, const float *Al) {
  if constexpr (L >= LAST) {
    constexpr int NC = 1 << (LP - L);
    constexpr int H = NC / 2;
    constexpr int B = batch_coords<NC, CPL>();
    constexpr int RS = CPL * kTileT;  // LDS row stride; column q of the lane at q kTileT
    const int tau = (int)((taus >> (8 * L)) & 0xff);
    j0 -= tau;
    if (tau == 0) {
#pragma unroll
      for (int q = 0; q < CPL; ++q)
#pragma unroll
        for (int c = 0; c < H; ++c) y[q][c + H] = y[q][c];
    } else {
      const float *x = rec + xo;
      const float *Aj = Al + j0 * RS;
      if constexpr (B * NC <= kBatchFloats) {
        // first batch: coordinate 0 forms the children (the tile step)
        float xs[B * NC], av[B][CPL];
#pragma unroll
        for (int i = 0; i < B * NC; ++i) xs[i] = ldx<VX>(x, i);
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
          for (int q = 0; q < CPL; ++q) av[i][q] = Aj[i * RS + q * kTileT];
        // consume every value here, so no load sinks into the guarded uses
        keep_scalar(xs);
#pragma unroll
        for (int i = 0; i < B; ++i)
#pragma unroll
          for (int q = 0; q < CPL; ++q) asm volatile("" ::"v"(av[i][q]));
#pragma unroll
        for (int q = 0; q < CPL; ++q) {
#pragma unroll
          for (int c = 0; c < H; ++c) y[q][c + H] = fmaf(xs[c + H], av[0][q], y[q][c]);
#pragma unroll
          for (int c = 0; c < H; ++c) y[q][c] = fmaf(xs[c], av[0][q], y[q][c]);
        }
        // batches that hold B coordinates need no per-coordinate check; only
        // a last, partial one does
        auto madd = [&](int jb, int i0, auto checked) {
#pragma unroll
          for (int i = i0; i < B; ++i) {
            if (decltype(checked)::value && jb + i >= tau) break;
#pragma unroll
            for (int q = 0; q < CPL; ++q)
#pragma unroll
              for (int c = 0; c < NC; ++c) y[q][c] = fmaf(xs[i * NC + c], av[i][q], y[q][c]);
          }
        };
        auto fetch = [&](int jb) {
#pragma unroll
          for (int i = 0; i < B * NC; ++i) xs[i] = ldx<VX>(x, jb * NC + i);
#pragma unroll
          for (int i = 0; i < B; ++i)
#pragma unroll
            for (int q = 0; q < CPL; ++q) av[i][q] = Aj[(jb + i) * RS + q * kTileT];
          keep_scalar(xs);
#pragma unroll
          for (int i = 0; i < B; ++i)
#pragma unroll
            for (int q = 0; q < CPL; ++q) asm volatile("" ::"v"(av[i][q]));
        };
        if (tau >= B) madd(0, 1, std::false_type{});
        else madd(0, 1, std::true_type{});
        int jb = B;
#pragma unroll 1
        for (; jb + B <= tau; jb += B) {
          fetch(jb);
          madd(jb, 0, std::false_type{});
        }
        if (jb < tau) {
          fetch(jb);
          madd(jb, 0, std::true_type{});
        }
      } else {
        // NC = 64 (level 0 with more than one coordinate): one coordinate at a
        // time, its 64 point values in two chunks of 32.  The tile step forms
        // the upper half first, while the lower half still holds the parents.
        static_assert(NC == 2 * kBatchFloats, "chunking assumes 64 nodes");
        float a[CPL], xs[kBatchFloats];
#pragma unroll
        for (int q = 0; q < CPL; ++q) a[q] = Aj[q * kTileT];
#pragma unroll
        for (int i = 0; i < H; ++i) xs[i] = ldx<VX>(x, H + i);
        keep_scalar(xs);
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
          for (int c = 0; c < H; ++c) y[q][c + H] = fmaf(xs[c], a[q], y[q][c]);
#pragma unroll
        for (int i = 0; i < H; ++i) xs[i] = ldx<VX>(x, i);
        keep_scalar(xs);
#pragma unroll
        for (int q = 0; q < CPL; ++q)
#pragma unroll
          for (int c = 0; c < H; ++c) y[q][c] = fmaf(xs[c], a[q], y[q][c]);
#pragma unroll 1
        for (int jj = 1; jj < tau; ++jj) {
#pragma unroll
          for (int q = 0; q < CPL; ++q) a[q] = Aj[jj * RS + q * kTileT];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int i = 0; i < H; ++i) xs[i] = ldx<VX>(x, jj * NC + h * H + i);
            keep_scalar(xs);
#pragma unroll
            for (int q = 0; q < CPL; ++q)
#pragma unroll
              for (int c = 0; c < H; ++c) y[q][h * H + c] = fmaf(xs[c], a[q], y[q][h * H + c]);
          }
        }
      }
      xo += tau * NC;
    }
    descend_lean<LP, L - 1, LAST, CPL, VX>(y, rec, xo, j0, taus, Al);
  }
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

}  // namespace qmc
