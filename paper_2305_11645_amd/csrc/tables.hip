// Point-table generation (the distinct values of every coordinate).
//
// For coordinate j with n_j = 2^nb distinct values the integer c of the value
// c / 2^nb at residue rho < n_j is
//   lattice       c = rho * z'_j mod 2^nb                      (Section 1.3)
//   poly lattice  c = int(rho(x) g'_j(x) mod x^nb)             (Section 1.1, nu)
//   digital net   digits y_p = sum_q C_{p,q} rho_q (p <= nb)   (eq. def:digital,
//                 c = sum_p y_p 2^{nb-p}                        reduced_genmat_net2)
// then the randomisation and the map are applied in FP64 (Section 1.2,
// Section 2.3) and the result is rounded once to FP32.  All integer work is
// exact; the FP64 sequence is fixed (no contraction) so tables are
// reproducible bit for bit.
#include <algorithm>

#include "qmc_internal.h"

#pragma clang fp contract(off)

namespace qmc {

__device__ __forceinline__ uint32_t value_int(const Geometry &G, const uint32_t *__restrict__ gen,
                                              int j, uint32_t rho, int nb) {
  if (nb == 0) return 0u;
  const uint32_t mask = (nb >= 32) ? 0xffffffffu : ((1u << nb) - 1u);
  if (G.kind == QMC_LATTICE) return (rho * gen[j]) & mask;
  if (G.kind == QMC_POLY_LATTICE) {
    const uint32_t g = gen[j];
    uint32_t acc = 0;
    for (int i = 0; i < nb; ++i)
      if ((rho >> i) & 1u) acc ^= g << i;
    return acc & mask;
  }
  const uint32_t *col = gen + (size_t)j * G.m;
  uint32_t y = 0;
  for (int q = 0; q < nb; ++q)
    if ((rho >> q) & 1u) y ^= col[q];
  y &= mask;  // rows p > nb of the reduced matrix are zero
  return __builtin_bitreverse32(y) >> (32 - nb);
}

template <bool INVNORM>
__device__ __forceinline__ double value_f64(const Geometry &G, const DevSpec &D, int r, int j,
                                            uint32_t rho, int nb) {
  const uint32_t c = value_int(G, D.gen, j, rho, nb);
  double x;
  if (G.rand == QMC_DIGITAL_SHIFT) {
    const uint64_t U = ((uint64_t)c << (52 - nb)) ^ D.dshift[(size_t)r * G.s + j];
    x = (double)(2 * U + 1) * 0x1p-53;  // exact
  } else {
    x = (double)c * __builtin_ldexp(1.0, -nb);  // exact
    if (G.rand == QMC_RANDOM_SHIFT) {
      x = __dadd_rn(x, D.shift[(size_t)r * G.s + j]);
      if (x >= 1.0) x = __dsub_rn(x, 1.0);
    }
  }
  if (INVNORM) return normcdfinv(x);
  switch (G.map) {
    case QMC_MAP_CENTER: return __dsub_rn(x, 0.5);
    case QMC_MAP_TENT: return __dsub_rn(1.0, fabs(__dsub_rn(1.0, __dmul_rn(2.0, x))));
    default: return x;
  }
}

// One launch covers every level ("segment") and every shift: blockIdx.y is
// the segment (lower levels L'-1..0, then the upper levels), blockIdx.z the
// shift.  A segment holds tau_I * n_I values.
//   lower level I: o -> (c = o mod 2^{L'-I}, jj, subtree root sub); the value
//                  of coordinate j0 + jj at residue sub + c n_{L'} goes to
//                  record sub, offset off_I + jj 2^{L'-I} + c
//   upper level I: o -> (row = o / tau_I, jj = o mod tau_I), stored row-major
// Flattened grid: block b belongs to (shift, segment) through the prefix sums
// of per-segment block counts.
struct TableGrid {
  int32_t nseg;
  int32_t blk0[kMaxLevels + 1];  // first block of each segment (per shift); blk0[nseg] = total
};

template <bool INVNORM>
__global__ __launch_bounds__(256) void tables_kernel(Geometry G, DevSpec D, TableGrid tg, int r0,
                                                     float *__restrict__ out,
                                                     uint32_t *__restrict__ counters, int ncounters) {
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < ncounters; i += blockDim.x) counters[i] = 0u;
  const int rl = blockIdx.y;
  int seg = 0;
  for (int q = 1; q < tg.nseg; ++q)
    if ((int)blockIdx.x >= tg.blk0[q]) seg = q;
  const uint32_t b0 = blockIdx.x - tg.blk0[seg];
  const uint32_t nb_seg = tg.blk0[seg + 1] - tg.blk0[seg];
  const bool lower = seg < G.split;
  const int I = lower ? G.split - 1 - seg : G.up[seg - G.split];
  const Level &L = G.lev[I];
  const uint32_t tau = (uint32_t)L.tau;
  const uint32_t count = tau << L.nb;
  float *o_r = out + (int64_t)rl * G.table_total;
  const int shiftc = G.split - I;  // log2 of the nodes per subtree at a lower level
  for (uint32_t o = b0 * 256 + threadIdx.x; o < count; o += nb_seg * 256) {
    uint32_t rho, jj;
    int64_t dst;
    if (lower) {
      const uint32_t c = o & ((1u << shiftc) - 1u);
      const uint32_t qq = o >> shiftc;
      jj = qq % tau;
      const uint32_t sub = qq / tau;
      rho = sub + (c << (G.m - G.split));
      dst = (int64_t)sub * G.rec + L.off + ((int64_t)jj << shiftc) + c;
    } else {
      rho = o / tau;
      jj = o - rho * tau;
      dst = G.lower_total + L.off + o;
    }
    o_r[dst] = (float)value_f64<INVNORM>(G, D, r0 + rl, L.j0 + (int)jj, rho, L.nb);
  }
}

template <bool INVNORM>
__global__ void values_kernel(Geometry G, DevSpec D, int r, int j, int nb, double *__restrict__ out) {
  const uint32_t n = 1u << nb;
  for (uint32_t rho = blockIdx.x * blockDim.x + threadIdx.x; rho < n; rho += gridDim.x * blockDim.x)
    out[rho] = value_f64<INVNORM>(G, D, r, j, rho, nb);
}

template <bool INVNORM>
__global__ void point_matrix_kernel(Geometry G, DevSpec D, int r, float *__restrict__ X, int64_t ldx) {
  const int64_t total = G.N * G.s;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx / G.s;
    const int j = (int)(idx - k * G.s);
    const int nb = D.nbj[j];
    const uint32_t rho = (uint32_t)(k & ((int64_t(1) << nb) - 1));
    X[k * ldx + j] = (float)value_f64<INVNORM>(G, D, r, j, rho, nb);
  }
}

static int grid_for(int64_t work, int threads) {
  int64_t g = ceil_div(work, threads);
  if (g > 65535) g = 65535;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_tables(const Geometry &G, const DevSpec &D, int r0, int nr, float *out,
                         uint32_t *counters, int ncounters, hipStream_t st) {
  LaunchTimer tm("tables", st);
  TableGrid tg{};
  tg.nseg = G.split + G.nup;
  int total = 0;
  for (int q = 0; q < tg.nseg; ++q) {
    const int I = q < G.split ? G.split - 1 - q : G.up[q - G.split];
    const int64_t count = (int64_t)G.lev[I].tau << G.lev[I].nb;
    tg.blk0[q] = total;
    total += (int)std::min<int64_t>(ceil_div(count, 256), 512);
  }
  tg.blk0[tg.nseg] = total;
  if (total == 0) total = 1;  // still zero the counters
  dim3 grid(total, nr);
  if (G.map == QMC_MAP_INVNORM)
    hipLaunchKernelGGL(tables_kernel<true>, grid, dim3(256), 0, st, G, D, tg, r0, out, counters, ncounters);
  else
    hipLaunchKernelGGL(tables_kernel<false>, grid, dim3(256), 0, st, G, D, tg, r0, out, counters, ncounters);
  return hipGetLastError();
}

hipError_t launch_point_values(const Geometry &G, const DevSpec &D, int r, int j, double *out,
                               hipStream_t st) {
  LaunchTimer tm("points", st);
  // nb of coordinate j from the level table
  int nb = 0;
  for (int I = 0; I <= G.m; ++I)
    if (j >= G.lev[I].j0 && j < G.lev[I].j0 + G.lev[I].tau) nb = G.lev[I].nb;
  const dim3 grid(grid_for(int64_t(1) << nb, 256));
  if (G.map == QMC_MAP_INVNORM)
    hipLaunchKernelGGL(values_kernel<true>, grid, dim3(256), 0, st, G, D, r, j, nb, out);
  else
    hipLaunchKernelGGL(values_kernel<false>, grid, dim3(256), 0, st, G, D, r, j, nb, out);
  return hipGetLastError();
}

hipError_t launch_point_matrix(const Geometry &G, const DevSpec &D, int r, float *X, int64_t ldx,
                               hipStream_t st) {
  LaunchTimer tm("points", st);
  const dim3 grid(grid_for(G.N * G.s, 256));
  if (G.map == QMC_MAP_INVNORM)
    hipLaunchKernelGGL(point_matrix_kernel<true>, grid, dim3(256), 0, st, G, D, r, X, ldx);
  else
    hipLaunchKernelGGL(point_matrix_kernel<false>, grid, dim3(256), 0, st, G, D, r, X, ldx);
  return hipGetLastError();
}

}  // namespace qmc
