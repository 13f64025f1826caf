// Point-table generation (the distinct values of every coordinate).
//
// For coordinate j with n_j = b^nb distinct values the integer c of the value
// c / n_j at residue rho < n_j is
//   lattice       c = rho * z'_j mod n_j                       (Section 1.3)
//   poly lattice  c = int(rho(x) g'_j(x) mod x^nb)             (Section 1.1, nu)
//   digital net   digits y_p = sum_q C_{p,q} rho_q (p <= nb)   (eq. def:digital,
//                 c = sum_p y_p 2^{nb-p}                        reduced_genmat_net2)
// (polynomial lattices and nets in base 2), then the randomisation and the map
// are applied in FP64 (Section 1.2, Section 2.3) and the result is rounded
// once to FP32.  All integer work is exact; c / n_j is exact for b = 2 and one
// correctly rounded division otherwise; the FP64 sequence is fixed (no
// contraction) so tables are reproducible bit for bit.
#include <algorithm>

#include "qmc_internal.h"

#pragma clang fp contract(off)

namespace qmc {

// The point-set constants the value computation needs.
struct PointConsts {
  int32_t m, s, kind, rand, map, b;
  int32_t kdig;         // base b > 2, digital shift: K digits, b^K <= 2^52
  double bK;            // b^K (exact)
  int32_t by_output;    // rho is already the integer c of the value c / 2^nb (value tables of nets)
  int32_t nonperiodic;  // a reduced net that depends on every input digit
};

static PointConsts consts_of(const Geometry &G) {
  PointConsts pc{G.m, G.s, G.kind, G.rand, G.map, G.b, 0, 1.0, 0, G.nonperiodic};
  if (G.b != 2) {
    uint64_t v = 1;
    while (v <= (uint64_t(1) << 52) / (uint64_t)G.b) {
      v *= (uint64_t)G.b;
      ++pc.kdig;
    }
    pc.bK = (double)v;
  }
  return pc;
}

__host__ __device__ __forceinline__ uint64_t ipow_u64(uint32_t b, int e) {
  uint64_t r = 1;
  for (int i = 0; i < e; ++i) r *= b;
  return r;
}

// Base b > 2 (every point set periodic in k mod n_j, n_j = b^nb): the integer
// c of c / n_j at residue rho.  Lattice rho z' mod n_j; polynomial lattice
// the digits of rho(x) g'_j(x) mod (b, x^nb) (coefficient i = digit i);
// net the output digits y_p = sum_q C_{p,q} rho_q mod b (p <= nb, column word
// q holds C_{p,q} as digit p-1), read most significant first.
// (out of line: the digit arrays live in scratch; lattices take the inline
// path in value_int)
__device__ __noinline__ uint32_t value_int_b(const PointConsts &G, const uint32_t *__restrict__ gen, int j,
                                             uint32_t rho, int nb) {
  if (G.by_output) return rho;  // already the integer of the output digits
  const uint32_t b = (uint32_t)G.b;
  // a net that is not periodic reads every digit of the point index (m <= 24)
  const int nd = G.nonperiodic && G.kind == QMC_DIGITAL_NET ? G.m : nb;
  uint32_t rd[32];
  uint64_t y[32];  // sums of up to m products below b^2
  for (int i = 0; i < nd; ++i) {
    rd[i] = rho % b;
    rho /= b;
    y[i] = 0;
  }
  if (G.kind == QMC_POLY_LATTICE) {
    uint32_t g = gen[j], gd[32];
    for (int i = 0; i < nb; ++i) {
      gd[i] = g % b;
      g /= b;
    }
    uint32_t c = 0;
    for (int i = nb - 1; i >= 0; --i) {  // coefficient i of the product is digit i
      uint64_t acc = 0;
      for (int k = 0; k <= i; ++k) acc += (uint64_t)rd[k] * gd[i - k];
      c = c * b + (uint32_t)(acc % b);
    }
    return c;
  }
  const uint32_t *col = gen + (size_t)j * G.m;
  for (int q = 0; q < nd; ++q) {  // periodic: digits of rho past nb are zero
    if (!rd[q]) continue;
    uint32_t wd = col[q];
    for (int p = 0; p < nb; ++p) {
      y[p] += (uint64_t)(wd % b) * rd[q];
      wd /= b;
    }
  }
  uint32_t c = 0;
  for (int p = 0; p < nb; ++p) c = c * b + (uint32_t)(y[p] % b);
  return c;
}

// The integer c of the value c / 2^nb of coordinate j at input index rho:
// lattice rho z' mod 2^nb; polynomial lattice the carry-less product; net the
// XOR of the generating-matrix columns selected by the digits of rho (all of
// them: for a net that repeats with period n_j the columns past nb carry no
// bits in the first nb rows), truncated to nb rows and read most significant
// digit first.
// VB: the class of point sets a kernel serves, so that each kernel holds only
// its own code (the digit arithmetic of value_int_b needs scratch memory, which
// costs every launch of a kernel that contains it):
//   0  base 2;  1  base b > 2, lattices (and reduced Monte Carlo);
//   2  base b > 2, polynomial lattices and nets.
template <int VB>
__device__ __forceinline__ uint32_t value_int(const PointConsts &G, const uint32_t *__restrict__ gen,
                                              int j, uint32_t rho, int nb) {
  if (nb == 0) return 0u;
  if constexpr (VB == 1) return (uint32_t)(((uint64_t)rho * gen[j]) % ipow_u64(G.b, nb));
  if constexpr (VB == 2) return value_int_b(G, gen, j, rho, nb);
  const uint32_t mask = (nb >= 32) ? 0xffffffffu : ((1u << nb) - 1u);
  if (G.by_output) return rho & mask;
  if (G.kind == QMC_LATTICE) return (rho * gen[j]) & mask;
  if (G.kind == QMC_POLY_LATTICE) {
    const uint32_t g = gen[j];
    uint32_t acc = 0;
    for (int i = 0; i < nb; ++i)
      if ((rho >> i) & 1u) acc ^= g << i;
    return acc & mask;
  }
  // digit q of rho selects column q (rho < 2^m: the residue, or the whole
  // point index of a net that is not periodic).  Every column up to the
  // highest digit is loaded and masked by its digit, so the loads do not wait
  // on one another
  const uint32_t *col = gen + (size_t)j * G.m;
  const int nq = rho ? 32 - __builtin_clz(rho) : 0;
  uint32_t y = 0;
#pragma unroll 4
  for (int q = 0; q < nq; ++q) y ^= col[q] & (0u - ((rho >> q) & 1u));
  y &= mask;  // rows p > nb of the reduced matrix are zero
  return __builtin_bitreverse32(y) >> (32 - nb);
}

// Inverse standard normal CDF in FP64: Wichura, "Algorithm AS 241: The
// percentage points of the normal distribution", Applied Statistics 37
// (1988), PPND16 -- rational approximations of degree 7 in three regions,
// relative accuracy about 1e-16.  Evaluated with Horner's rule.
__device__ __forceinline__ double ppnd16(double p) {
  const double q = p - 0.5;
  if (fabs(q) <= 0.425) {
    const double r = 0.180625 - q * q;
    const double num =
        ((((((2.5090809287301226727e+3 * r + 3.3430575583588128105e+4) * r + 6.7265770927008700853e+4) * r +
            4.5921953931549871457e+4) * r + 1.3731693765509461125e+4) * r + 1.9715909503065514427e+3) * r +
         1.3314166789178437745e+2) * r + 3.3871328727963666080e0;
    const double den =
        ((((((5.2264952788528545610e+3 * r + 2.8729085735721942674e+4) * r + 3.9307895800092710610e+4) * r +
            2.1213794301586595867e+4) * r + 5.3941960214247511077e+3) * r + 6.8718700749205790830e+2) * r +
         4.2313330701600911252e+1) * r + 1.0;
    return q * num / den;
  }
  double r = q < 0.0 ? p : 1.0 - p;
  if (r <= 0.0) return q < 0.0 ? -HUGE_VAL : HUGE_VAL;
  r = sqrt(-log(r));
  double v;
  if (r <= 5.0) {
    r -= 1.6;
    const double num =
        ((((((7.74545014278341407640e-4 * r + 2.27238449892691845833e-2) * r + 2.41780725177450611770e-1) * r +
            1.27045825245236838258e0) * r + 3.64784832476320460504e0) * r + 5.76949722146069140550e0) * r +
         4.63033784615654529590e0) * r + 1.42343711074968357734e0;
    const double den =
        ((((((1.05075007164441684324e-9 * r + 5.47593808499534494600e-4) * r + 1.51986665636164571966e-2) * r +
            1.48103976427480074590e-1) * r + 6.89767334985100004550e-1) * r + 1.67638483018380384940e0) * r +
         2.05319162663775882187e0) * r + 1.0;
    v = num / den;
  } else {
    r -= 5.0;
    const double num =
        ((((((2.01033439929228813265e-7 * r + 2.71155556874348757815e-5) * r + 1.24266094738807843860e-3) * r +
            2.65321895265761230930e-2) * r + 2.96560571828504891230e-1) * r + 1.78482653991729133580e0) * r +
         5.46378491116411436990e0) * r + 6.65790464350110377720e0;
    const double den =
        ((((((2.04426310338993978564e-15 * r + 1.42151175831644588870e-7) * r + 1.84631831751005468180e-5) * r +
            7.86869131145613259100e-4) * r + 1.48753612908506148525e-2) * r + 1.36929880922735805310e-1) * r +
         5.99832206555887937690e-1) * r + 1.0;
    v = num / den;
  }
  return q < 0.0 ? -v : v;
}

// IIDK: the point set is known to be reduced Monte Carlo, so the other kinds'
// code (and registers) is left out.
template <bool INVNORM, int VB = 0, bool IIDK = false>
__device__ __forceinline__ double value_f64(const PointConsts &G, const DevSpec &D, int r, int j,
                                            uint32_t rho, int nb) {
  double x;
  if (IIDK || G.kind == QMC_IID) {
    // reduced Monte Carlo (Section 4, eq. randpts): the distinct values of
    // coordinate j are its own i.i.d. samples, point k taking sample k mod n_j
    x = D.samples[(size_t)r * D.sample_total + D.soff[j] + rho];
  } else if constexpr (IIDK) {
    x = 0.0;  // not reached
  } else if (VB == 0 && G.rand == QMC_DIGITAL_SHIFT) {
    const uint32_t c = value_int<0>(G, D.gen, j, rho, nb);
    const uint64_t U = ((uint64_t)c << (52 - nb)) ^ D.dshift[(size_t)r * G.s + j];
    x = (double)(2 * U + 1) * 0x1p-53;  // exact
  } else if (G.rand == QMC_DIGITAL_SHIFT) {
    // base b: digits p = 1..K of x are those of c (p <= nb) plus those of
    // delta (most significant first), mod b; then the midpoint of the rest
    const uint64_t b = (uint64_t)G.b;
    const uint32_t c = value_int<VB>(G, D.gen, j, rho, nb);
    uint64_t dl = D.dshift[(size_t)r * G.s + j], cc = c, U = 0, pw = 1;
    for (int i = 0; i < G.kdig; ++i) {  // digit p = K - i
      const int p = G.kdig - i;
      uint64_t yp = 0;
      if (p <= nb) {  // digit p of c / b^nb is digit nb - p of c
        uint64_t t = cc;
        for (int k = 0; k < nb - p; ++k) t /= b;
        yp = t % b;
      }
      U += ((yp + dl % b) % b) * pw;
      dl /= b;
      pw *= b;
    }
    x = __ddiv_rn((double)U + 0.5, G.bK);  // U + 1/2 exact (U < 2^52); one rounding
  } else {
    const uint32_t c = value_int<VB>(G, D.gen, j, rho, nb);
    if constexpr (VB != 0) x = __ddiv_rn((double)c, (double)ipow_u64(G.b, nb));
    else x = (double)c * __builtin_ldexp(1.0, -nb);  // exact
    if (G.rand == QMC_RANDOM_SHIFT) {
      x = __dadd_rn(x, D.shift[(size_t)r * G.s + j]);
      if (x >= 1.0) x = __dsub_rn(x, 1.0);
    }
  }
  if (INVNORM) return ppnd16(x);
  switch (G.map) {
    case QMC_MAP_CENTER: return __dsub_rn(x, 0.5);
    case QMC_MAP_TENT: return __dsub_rn(1.0, fabs(__dsub_rn(1.0, __dmul_rn(2.0, x))));
    default: return x;
  }
}

// One launch covers every level ("segment") and every shift: blockIdx.x runs
// over the blocks of all segments (lower levels L'-1..0, then the upper
// levels), blockIdx.y is the shift.  A segment holds tau_I * n_I values.
//   lower level I: o -> (c = o mod 2^{L'-I}, jj, subtree root sub); the value
//                  of coordinate j0 + jj at residue sub + c n_{L'} goes to
//                  record sub, offset off_I + jj 2^{L'-I} + c
//   upper level I: o -> (row = o / tau_I, jj = o mod tau_I), stored row-major
struct TabSeg {
  int32_t blk0, nblk;   // blocks of this segment
  int32_t lower, sh;    // lower level?  log2 of its nodes per subtree
  uint32_t tau, count;  // coordinates, values
  int32_t j0, nb;       // first coordinate, n_I = 2^nb
  int64_t dst;          // first table entry of the segment
};

constexpr int kTabSegPad = 32;  // >= kMaxLevels: the segment starts are scanned in whole batches
static_assert(kTabSegPad >= kMaxLevels, "segment start table too short");

struct TabArgs {
  // first block of each segment, contiguous and padded with INT_MAX, so that a
  // block finds its segment from one batch of scalar loads (a scan through
  // seg[] would chain one dependent load per segment)
  int32_t blk0[kTabSegPad];
  int32_t nseg, nblk;
  int32_t rec;          // floats per subtree record
  int32_t sub_sh;       // log2 n_{L'}
  int64_t table_total;
  PointConsts G;
  TabSeg seg[kMaxLevels];
};

// Values per thread: the index math and gathers of all of them are issued
// before their arithmetic.  Two with the inverse normal map, whose FP64
// evaluation holds many registers per value in flight.
template <bool INVNORM>
constexpr int vals_per_thread() { return INVNORM ? 2 : 8; }

// The inverse normal map asks for eight waves per SIMD: left free, the compiler
// interleaves the FP64 evaluations of a thread's values into about 126
// registers (four waves); at 64 nothing spills.
template <bool INVNORM, bool IIDK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(INVNORM ? 8 : 1))) void tables_kernel(
    TabArgs ta, DevSpec D, int r0,
                                                     float *__restrict__ out,
                                                     uint32_t *__restrict__ counters, int ncounters) {
  constexpr int VPT = vals_per_thread<INVNORM>();
  if (blockIdx.x == 0 && blockIdx.y == 0)
    for (int i = threadIdx.x; i < ncounters; i += blockDim.x) counters[i] = 0u;
  const int rl = blockIdx.y;
  int q = 0;
#pragma unroll
  for (int i = 1; i < kTabSegPad; ++i)
    if ((int)blockIdx.x >= ta.blk0[i]) q = i;
  const TabSeg sg = ta.seg[q];
  const uint32_t b0 = blockIdx.x - sg.blk0;
  float *o_r = out + (int64_t)rl * ta.table_total + sg.dst;
  const uint32_t step = sg.nblk * 256u * VPT;
  for (uint32_t base = b0 * 256u * VPT + threadIdx.x; base < sg.count; base += step) {
    // all index math and gathers first, then the arithmetic: the loads overlap
    uint32_t rho[VPT], jv[VPT], dst[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
      const uint32_t o = min(base + 256u * v, sg.count - 1);
      uint32_t jj;
      if (sg.lower) {
        const uint32_t c = o & ((1u << sg.sh) - 1u);
        const uint32_t qq = o >> sg.sh;
        jj = qq % sg.tau;
        const uint32_t sub = qq / sg.tau;
        rho[v] = sub + (c << ta.sub_sh);
        dst[v] = sub * (uint32_t)ta.rec + (jj << sg.sh) + c;
      } else {
        rho[v] = o / sg.tau;
        jj = o - rho[v] * sg.tau;
        dst[v] = o;
      }
      jv[v] = sg.j0 + jj;
    }
    float val[VPT];
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      val[v] = (float)value_f64<INVNORM, 0, IIDK>(ta.G, D, r0 + rl, (int)jv[v], rho[v], sg.nb);
#pragma unroll
    for (int v = 0; v < VPT; ++v)
      if (base + 256u * v < sg.count) o_r[dst[v]] = val[v];
  }
}

template <bool INVNORM, int VB>
__global__ void values_kernel(PointConsts G, DevSpec D, int r, int j, int nb, double *__restrict__ out) {
  const uint32_t n = (uint32_t)ipow_u64(G.b, nb);
  for (uint32_t rho = blockIdx.x * blockDim.x + threadIdx.x; rho < n; rho += gridDim.x * blockDim.x)
    out[rho] = value_f64<INVNORM, VB>(G, D, r, j, rho, nb);
}

template <bool INVNORM, int VB>
__global__ void point_matrix_kernel(PointConsts G, DevSpec D, int r, float *__restrict__ X, int64_t ldx) {
  const int64_t total = (int64_t)ipow_u64(G.b, G.m) * G.s;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = idx / G.s;
    const int j = (int)(idx - k * G.s);
    const int nb = D.nbj[j];
    // a net that is not periodic needs every digit of k
    const uint32_t rho = G.nonperiodic ? (uint32_t)k
                         : G.b == 2    ? (uint32_t)(k & ((int64_t(1) << nb) - 1))
                                       : (uint32_t)(k % (int64_t)ipow_u64(G.b, nb));
    X[k * ldx + j] = (float)value_f64<INVNORM, VB>(G, D, r, j, rho, nb);
  }
}

// The kernel instance for a point set: inverse-normal map or not, and its
// value class VB (see value_int).
static int value_class(const Geometry &G) {
  if (G.b == 2) return 0;
  return G.kind == QMC_POLY_LATTICE || G.kind == QMC_DIGITAL_NET ? 2 : 1;
}
#define QMC_DISPATCH_VB(G, LAUNCH)                         \
  do {                                                     \
    const bool inv_ = (G).map == QMC_MAP_INVNORM;          \
    switch (value_class(G)) {                              \
      case 0: if (inv_) LAUNCH(true, 0); else LAUNCH(false, 0); break; \
      case 1: if (inv_) LAUNCH(true, 1); else LAUNCH(false, 1); break; \
      default: if (inv_) LAUNCH(true, 2); else LAUNCH(false, 2); break; \
    }                                                      \
  } while (0)

static int grid_for(int64_t work, int threads) {
  int64_t g = ceil_div(work, threads);
  if (g > 65535) g = 65535;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_tables(const Geometry &G, const DevSpec &D, int r0, int nr, float *out,
                         uint32_t *counters, int ncounters, hipStream_t st) {
  LaunchTimer tm("tables", st);
  TabArgs ta{};
  ta.G = consts_of(G);
  ta.nseg = G.split + G.nup;
  ta.rec = (int)G.rec;
  ta.sub_sh = G.m - G.split;
  ta.table_total = G.table_total;
  const int vpt = G.map == QMC_MAP_INVNORM ? vals_per_thread<true>() : vals_per_thread<false>();
  int total = 0;
  for (int q = 0; q < ta.nseg; ++q) {
    const bool lower = q < G.split;
    const int I = lower ? G.split - 1 - q : G.up[q - G.split];
    const Level &L = G.lev[I];
    TabSeg &sg = ta.seg[q];
    sg.lower = lower;
    sg.sh = lower ? G.split - I : 0;
    sg.tau = (uint32_t)L.tau;
    sg.count = (uint32_t)L.tau << L.nb;
    sg.j0 = L.j0;
    sg.nb = L.nb;
    sg.dst = lower ? L.off : G.lower_total + L.off;
    sg.blk0 = total;
    sg.nblk = (int)std::min<int64_t>(ceil_div(sg.count, 256 * vpt), 512);
    total += sg.nblk;
  }
  for (int q = 0; q < kTabSegPad; ++q) ta.blk0[q] = q < ta.nseg ? ta.seg[q].blk0 : 0x7fffffff;
  ta.nblk = total;
  if (total == 0) total = 1;  // still zero the counters
  dim3 grid(total, nr);
  const bool iid = G.kind == QMC_IID;
  if (G.map == QMC_MAP_INVNORM && iid)
    hipLaunchKernelGGL((tables_kernel<true, true>), grid, dim3(256), 0, st, ta, D, r0, out, counters, ncounters);
  else if (G.map == QMC_MAP_INVNORM)
    hipLaunchKernelGGL((tables_kernel<true, false>), grid, dim3(256), 0, st, ta, D, r0, out, counters, ncounters);
  else if (iid)
    hipLaunchKernelGGL((tables_kernel<false, true>), grid, dim3(256), 0, st, ta, D, r0, out, counters, ncounters);
  else
    hipLaunchKernelGGL((tables_kernel<false, false>), grid, dim3(256), 0, st, ta, D, r0, out, counters, ncounters);
  return hipGetLastError();
}

hipError_t launch_point_values(const Geometry &G, const DevSpec &D, int r, int j, double *out,
                               hipStream_t st) {
  LaunchTimer tm("points", st);
  // nb of coordinate j from the level table
  int nb = 0;
  for (int I = 0; I <= G.m; ++I)
    if (j >= G.lev[I].j0 && j < G.lev[I].j0 + G.lev[I].tau) nb = G.lev[I].nb;
  const dim3 grid(grid_for((int64_t)ipow_u64(G.b, nb), 256));
  PointConsts pc = consts_of(G);
  pc.by_output = G.nonperiodic;  // such a net's values are listed by their output digits
#define QMC_VALUES(I, V) hipLaunchKernelGGL((values_kernel<I, V>), grid, dim3(256), 0, st, pc, D, r, j, nb, out)
  QMC_DISPATCH_VB(G, QMC_VALUES);
#undef QMC_VALUES
  return hipGetLastError();
}

hipError_t launch_point_matrix(const Geometry &G, const DevSpec &D, int r, float *X, int64_t ldx,
                               hipStream_t st) {
  LaunchTimer tm("points", st);
  const dim3 grid(grid_for(G.N * G.s, 256));
  const PointConsts pc = consts_of(G);
#define QMC_PMAT(I, V) hipLaunchKernelGGL((point_matrix_kernel<I, V>), grid, dim3(256), 0, st, pc, D, r, X, ldx)
  QMC_DISPATCH_VB(G, QMC_PMAT);
#undef QMC_PMAT
  return hipGetLastError();
}

// Value tables of the gather path (layout at launch_output_tables' declaration):
// every value X_j(rho), rho < n_j, of every coordinate is computed once; the
// flat index e over sum_j n_j is mapped to (j, rho) by a binary search over
// soff.  Nets (digit order): rho is the digit word y, stored at aoff_j + y,
// the value that of the output integer bitreverse(y).  Base b > 2: rho is the
// residue, stored at aoff_j + rho and aoff_j + rho + n_j; for a net over F_b
// that is not periodic rho is the output integer c, stored once at aoff_j + c.
template <bool INVNORM, int VB>
__global__ __launch_bounds__(256) void outvals_kernel(PointConsts G, DevSpec D, int r0, int64_t stride,
                                                      float *__restrict__ out) {
  const int rl = blockIdx.y;
  const int64_t total = D.sample_total;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    int lo = 0, hi = G.s - 1;  // last j with soff[j] <= e
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (D.soff[mid] <= e) lo = mid; else hi = mid - 1;
    }
    const int nb = D.nbj[lo];
    const uint32_t y = (uint32_t)(e - D.soff[lo]);
    float *o = out + (int64_t)rl * stride + D.aoff[lo];
    if constexpr (VB == 0) {
      const uint32_t c = nb == 0 ? 0u : __builtin_bitreverse32(y) >> (32 - nb);
      o[y] = (float)value_f64<INVNORM, 0>(G, D, r0 + rl, lo, c, nb);
    } else if (G.nonperiodic) {
      // a net over F_b that is not periodic: y is the output integer c itself
      o[y] = (float)value_f64<INVNORM, VB>(G, D, r0 + rl, lo, y, nb);
    } else {
      const int64_t n = (lo + 1 < G.s ? D.soff[lo + 1] : total) - D.soff[lo];
      const float v = (float)value_f64<INVNORM, VB>(G, D, r0 + rl, lo, y, nb);
      o[y] = v;
      o[y + n] = v;
    }
  }
}

hipError_t launch_output_tables(const Geometry &G, const DevSpec &D, int r0, int nr, float *out,
                                hipStream_t st) {
  LaunchTimer tm("tables", st);
  PointConsts pc = consts_of(G);
  pc.by_output = G.nonperiodic;  // nets: the value of an output integer
  const dim3 grid(grid_for(D.sample_total, 256), nr);
#define QMC_OUTVALS(I, V) \
  hipLaunchKernelGGL((outvals_kernel<I, V>), grid, dim3(256), 0, st, pc, D, r0, G.gather_total, out)
  QMC_DISPATCH_VB(G, QMC_OUTVALS);
#undef QMC_OUTVALS
  return hipGetLastError();
}

}  // namespace qmc
