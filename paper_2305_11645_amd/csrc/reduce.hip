// Reductions: the N^-1 mean of eq. QMC-rule in FP64, the per-point outer
// function h, the fold of subtree-root sums over the upper levels, and the
// final assembly of dA.  Every reduction runs in a fixed order, so results
// are bitwise reproducible.
#include "qmc_internal.h"

namespace qmc {

// Neumaier two-sum accumulator.
struct Comp {
  double s = 0.0, c = 0.0;
  __device__ __forceinline__ void add(double v) {
    const double u = s + v;
    if (fabs(s) >= fabs(v)) c += (s - u) + v; else c += (v - u) + s;
    s = u;
  }
};

__global__ __launch_bounds__(256) void reduce_kernel(const double *__restrict__ partial, int64_t per,
                                                     double scale, double *__restrict__ Q) {
  __shared__ double ss[256], sc[256];
  const int r = blockIdx.x, tid = threadIdx.x;
  const double *p = partial + (int64_t)r * per;
  Comp acc;
  for (int64_t i = tid; i < per; i += 256) acc.add(p[i]);
  ss[tid] = acc.s;
  sc[tid] = acc.c;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if (tid < d) {
      Comp m;
      m.s = ss[tid];
      m.c = sc[tid] + sc[tid + d];
      m.add(ss[tid + d]);
      ss[tid] = m.s;
      sc[tid] = m.c;
    }
    __syncthreads();
  }
  if (tid == 0) Q[r] = (ss[0] + sc[0]) * scale;
}

hipError_t launch_reduce(const double *partial, int nr, int64_t per, double scale, double *Q,
                         hipStream_t st) {
  LaunchTimer tm("reduce", st);
  hipLaunchKernelGGL(reduce_kernel, dim3(nr), dim3(256), 0, st, partial, per, scale, Q);
  return hipGetLastError();
}

constexpr int kPointsPerBlock = 1024;

int64_t point_h_blocks(const Geometry &G) { return ceil_div(G.N, kPointsPerBlock); }

// u_k = t^-1 sum over column tiles of the per-tile sums; f_k = h(u_k);
// partial[r][blk] = sum of f_k over the block's points; hd[r][k] = h'(u_k) hscale.
__global__ __launch_bounds__(256) void point_h_kernel(int64_t N, int tct, double inv_t, int h,
                                                      double K, const float *__restrict__ ppart,
                                                      double *__restrict__ partial, int64_t blocks,
                                                      float *__restrict__ hd, double hscale) {
  __shared__ double ss[256];
  const int r = blockIdx.y, tid = threadIdx.x;
  const int64_t k0 = (int64_t)blockIdx.x * kPointsPerBlock;
  const float *pp = ppart + (int64_t)r * tct * N;
  double acc = 0.0;
  for (int64_t k = k0 + tid; k < min(N, k0 + kPointsPerBlock); k += 256) {
    double u = 0.0;
    for (int c = 0; c < tct; ++c) u += (double)pp[(int64_t)c * N + k];
    u *= inv_t;
    double fk, dk;
    if (h == QMC_H_CALL) { fk = u > K ? u - K : 0.0; dk = u > K ? 1.0 : 0.0; }
    else { fk = u; dk = 1.0; }
    acc += fk;
    if (hd) hd[(int64_t)r * N + k] = (float)(dk * hscale);
  }
  ss[tid] = acc;
  __syncthreads();
  for (int d = 128; d >= 1; d >>= 1) {
    if (tid < d) ss[tid] += ss[tid + d];
    __syncthreads();
  }
  if (tid == 0) partial[(int64_t)r * blocks + blockIdx.x] = ss[0];
}

hipError_t launch_point_h(const Geometry &G, const qmc_integrand &f, const float *ppart, int nr,
                          int tct, int t, double *partial, int64_t blocks, float *hd,
                          double hscale, hipStream_t st) {
  LaunchTimer tm("reduce", st);
  hipLaunchKernelGGL(point_h_kernel, dim3((unsigned)blocks, nr), dim3(256), 0, st, G.N, tct,
                     1.0 / (double)t, f.h, f.K, ppart, partial, blocks, hd, hscale);
  return hipGetLastError();
}

// S_{I+1}[rho] = S_I[rho] + S_I[rho + n_{I+1}], rho < n_{I+1}: the adjoint of
// the tiling step of Algorithm 2.  S holds the pyramid of all levels >= L'.
__global__ __launch_bounds__(256) void fold_kernel(float *__restrict__ S, int64_t src_off,
                                                   int64_t dst_off, int64_t nrows, int t,
                                                   int64_t ldu, int64_t rstride) {
  const int r = blockIdx.y;
  float *Sr = S + r * rstride;
  const int64_t total = nrows * t;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t row = e / t, col = e - (e / t) * t;
    Sr[(dst_off + row) * ldu + col] =
        Sr[(src_off + row) * ldu + col] + Sr[(src_off + row + nrows) * ldu + col];
  }
}

hipError_t launch_fold(const Geometry &G, int nr, float *S, int t, int64_t ldu, hipStream_t st) {
  LaunchTimer tm("fold", st);
  if (G.nup == 0) return hipSuccess;
  const int top = G.up[G.nup - 1];
  int64_t off = 0;
  for (int I = G.split; I < top; ++I) {
    const int64_t n = int64_t(1) << (G.m - I);
    const int64_t half = n / 2;
    int64_t blocks = ceil_div(half * t, 256);
    if (blocks > 16384) blocks = 16384;
    hipLaunchKernelGGL(fold_kernel, dim3((unsigned)blocks, nr), dim3(256), 0, st, S, off, off + n,
                       half, t, ldu, 2 * G.nsub * ldu);
    off += n;
  }
  return hipGetLastError();
}

struct CombineArgs {
  Geometry G;
  double scale;
  int32_t gx, tct, t, nr;
  int64_t ldu, up_rs;
  int64_t poff[kMaxLevels];    // per upper level u: offset of its partial blocks
  int32_t kchunks[kMaxLevels];
};

__global__ __launch_bounds__(256) void combine_kernel(CombineArgs a, const float *__restrict__ low,
                                                      const float *__restrict__ up,
                                                      float *__restrict__ dA) {
  const Geometry &G = a.G;
  const int r = blockIdx.y;
  const int64_t total = (int64_t)G.s * a.t;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int j = (int)(e / a.t), col = (int)(e - (e / a.t) * a.t);
    double acc = 0.0;
    if (j < G.jlow) {
      const int ct = col / kTileT, lane = col % kTileT;
      const int64_t blk = (int64_t)G.jlow * kTileT;
      // unrolled so that eight loads are in flight (the sum keeps its order)
#pragma unroll 8
      for (int bx = 0; bx < a.gx; ++bx)
        acc += (double)low[(((int64_t)r * a.gx + bx) * a.tct + ct) * blk + (int64_t)j * kTileT + lane];
    } else {
      for (int u = 0; u < G.nup; ++u) {
        const Level &L = G.lev[G.up[u]];
        if (j < L.j0 || j >= L.j0 + L.tau) continue;
        const float *p = up + r * a.up_rs + a.poff[u] + (int64_t)(j - L.j0) * a.ldu + col;
#pragma unroll 8
        for (int c = 0; c < a.kchunks[u]; ++c) acc += (double)p[(int64_t)c * L.tau * a.ldu];
      }
    }
    dA[((int64_t)r * G.s + j) * a.t + col] = (float)(a.scale * acc);
  }
}

hipError_t launch_combine(const Geometry &G, const float *dApart_low, int gx, int tct,
                          const float *dApart_up, int nr, int t, int64_t ldu, double scale, float *dA,
                          hipStream_t st) {
  LaunchTimer tm("combine", st);
  CombineArgs a;
  a.G = G;
  a.scale = scale;
  a.gx = gx;
  a.tct = tct;
  a.t = t;
  a.nr = nr;
  a.ldu = ldu;
  a.up_rs = levels_adj_part_floats(G, t, ldu);
  int64_t poff = 0;
  for (int u = 0; u < G.nup; ++u) {
    const Level &L = G.lev[G.up[u]];
    const int64_t K = int64_t(1) << L.nb;
    const int64_t kc = levels_adj_kchunk(K);
    a.kchunks[u] = (int)ceil_div(K, kc);
    a.poff[u] = poff;
    poff += (int64_t)a.kchunks[u] * L.tau * ldu;
  }
  int64_t blocks = ceil_div((int64_t)G.s * t, 256);
  if (blocks > 16384) blocks = 16384;
  hipLaunchKernelGGL(combine_kernel, dim3((unsigned)blocks, nr), dim3(256), 0, st, a, dApart_low,
                     dApart_up, dA);
  return hipGetLastError();
}

}  // namespace qmc
