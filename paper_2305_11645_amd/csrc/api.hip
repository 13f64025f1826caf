// C ABI of libqmcred: validation, level planning, workspace and launch order.
#include <algorithm>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "qmc_internal.h"

struct qmc_points_s {
  int device = 0;
  qmc::Geometry G{};   // the estimate's and the matrix-vector product's
  qmc::Geometry Gg{};  // the gradient's: the split level capped at kMaxSplitGrad
  qmc::DevSpec D{};
  void *d_gen = nullptr, *d_nb = nullptr, *d_shift = nullptr, *d_dshift = nullptr;
  void *d_samples = nullptr, *d_soff = nullptr;
  void *d_yidx = nullptr;  // Algorithm 4 index words
};

namespace {

thread_local std::string g_last_error;

qmc_status fail(qmc_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

qmc_status hip_fail(hipError_t e, const char *what) {
  return fail(QMC_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define QMC_HIP(call, what)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hip_fail(e_, what);         \
  } while (0)

// ------------------------------------------------------------ timing registry
std::mutex g_tm_mu;
bool g_tm_on = false;
std::unordered_map<std::string, std::vector<std::pair<hipEvent_t, hipEvent_t>>> g_tm;

// Restores the caller's device on scope exit.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
    else prev = -1;
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

bool is_prime(int b) {
  if (b < 2) return false;
  for (int d = 2; d * d <= b; ++d)
    if (b % d == 0) return false;
  return true;
}

// Split level L' (at most max_split) and record/table layout (see qmc_internal.h).
void plan_geometry(qmc::Geometry &G, const int32_t *w, int max_split) {
  using namespace qmc;
  const int m = G.m;
  for (int I = 0; I <= m; ++I) {
    G.lev[I] = Level{};
    G.lev[I].nb = m - I;
    G.lev[I].j0 = -1;
  }
  for (int j = 0; j < G.s; ++j) {
    const int I = w[j] < m ? w[j] : m;
    if (G.lev[I].j0 < 0) G.lev[I].j0 = j;
    G.lev[I].tau++;
  }
  int jcur = 0;
  for (int I = 0; I <= m; ++I) {  // empty levels get the j0 of the next block
    if (G.lev[I].j0 < 0) G.lev[I].j0 = jcur;
    jcur = G.lev[I].j0 + G.lev[I].tau;
  }
  int split = m < max_split ? m : max_split;
  if (const char *env = getenv("QMC_SPLIT_LEVEL")) {
    const int v = atoi(env);
    if (v >= 0 && v <= split) split = v;
  }
  while (split > 0) {
    int jl = 0;
    for (int I = 0; I < split; ++I) jl += G.lev[I].tau;
    if (jl <= kMaxLowRows) break;
    --split;
  }
  G.split = split;
  G.jlow = 0;
  for (int I = 0; I < split; ++I) G.jlow += G.lev[I].tau;
  G.N = int64_t(1) << m;
  G.nsub = int64_t(1) << (m - split);
  int64_t off = 0;
  for (int I = split - 1; I >= 0; --I) {
    G.lev[I].off = off;
    off += (int64_t)G.lev[I].tau << (split - I);
  }
  G.rec = off;
  G.lower_total = G.nsub * G.rec;
  G.nup = 0;
  int64_t toff = 0, uoff = 0;
  for (int I = split; I <= m; ++I) {
    if (G.lev[I].tau == 0) continue;
    G.up[G.nup++] = I;
    G.lev[I].off = toff;
    G.lev[I].uoff = uoff;
    toff += (int64_t(1) << G.lev[I].nb) * G.lev[I].tau;
    uoff += int64_t(1) << G.lev[I].nb;
  }
  G.table_total = G.lower_total + toff;
  G.urows = uoff;
}

// Base b > 2: the gather path in two passes.  With n_split = b^{m - L'}, the
// coordinates with min(w_j, m) >= L' (n_j <= n_split) are summed over the
// n_split residues into a root table (the upper levels of Algorithm 2's
// cascade), the jlow lower ones over all N points, which add the root row
// n mod n_split.  L' (with n_split >= 64) minimises the matrix-core work in
// whole 32-coordinate steps, N ceil32(jlow) + n_split ceil32(s - jlow), plus
// the root rows read by every point, priced as 16 multiply-adds per column;
// one pass (jlow = s) when that is cheaper.
void plan_gather_split(qmc::Geometry &G, const int32_t *w, int64_t Nb) {
  G.N = Nb;
  G.split = -1;
  G.jlow = G.s;
  G.nsub = 0;
  auto steps = [](int64_t k) { return (k + 31) / 32 * 32; };
  int64_t best = Nb * steps(G.s);
  int64_t nsplit = Nb;
  int force = -2;  // QMC_SPLIT_LEVEL: a level to take instead of the cheapest (-1: one pass)
  if (const char *env = getenv("QMC_SPLIT_LEVEL")) force = atoi(env);
  for (int L = 1; L <= G.m; ++L) {
    nsplit /= G.b;
    if (nsplit < 64) break;
    int jl = 0;
    while (jl < G.s && (w[jl] < G.m ? w[jl] : G.m) < L) ++jl;
    const int64_t cost = force == L ? 0 : force >= -1 ? best
                                                      : Nb * steps(jl) + nsplit * steps(G.s - jl) + 16 * Nb;
    if (cost < best) {
      best = cost;
      G.split = L;
      G.jlow = jl;
      G.nsub = nsplit;
    }
  }
}

// ------------------------------------------------------------ workspace
struct Carve {
  char *base;
  size_t used = 0;
  template <class T>
  T *take(size_t count) {
    T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
    used += qmc::round_up((int64_t)(count * sizeof(T)), 256);
    return p;
  }
};

enum Op { kOpMatvec = 0, kOpEstimate = 1, kOpGrad = 2 };

struct Work {
  float *tables, *U, *ppart, *S, *dlow, *dup, *hd, *root;
  void *pack;  // the packed operands of the upper-level products
  float *Gm;  // gather path, gradient: the sensitivities G, [nr][N][t]
  double *partial, *ppartial;
  double *glow, *gup;  // gather path, gradient: FP64 chunk partials of dA
};

size_t carve(const qmc::Geometry &G, int op, int t, const qmc_integrand *f, int nr, int prec, char *base,
             Work &wk) {
  using namespace qmc;
  Carve c{base};
  const int64_t ldu = round_up(t, kTileT);
  const int64_t tct = ceil_div(t, kTileT);
  const LeafPlan lp = leaf_plan(G, t, nr, kModeSum, f->g);
  const LeafPlan lg = leaf_plan(G, t, nr, kModeGrad, f->g);
  wk = Work{};
  if (G.gather) {  // value tables, root table, partials of the 64-point x 256-column tiles
    wk.tables = c.take<float>((size_t)nr * G.gather_total);
    if (G.jlow < G.s) wk.root = c.take<float>((size_t)nr * G.nsub * t);
    if (op == kOpMatvec) return c.used;
    const int64_t atct = alg4_col_tiles(t);
    wk.partial = c.take<double>((size_t)nr * alg4_point_tiles(G) * atct);
    if (f->h != QMC_H_ID) {
      wk.ppart = c.take<float>((size_t)nr * atct * G.N);
      wk.ppartial = c.take<double>((size_t)nr * point_h_blocks(G));
    }
    if (op == kOpGrad) {  // G, the folded G of the upper coordinates, h', the chunk partials
      wk.Gm = c.take<float>((size_t)nr * G.N * t);
      if (G.jlow < G.s) wk.S = c.take<float>((size_t)nr * G.nsub * t);
      if (f->h != QMC_H_ID) wk.hd = c.take<float>((size_t)nr * G.N);
      const int nlo = alg4_adj_chunks(G.jlow, G.N, t, nr), nup = alg4_adj_chunks(G.s - G.jlow, G.nsub, t, nr);
      wk.glow = c.take<double>((size_t)nr * nlo * G.jlow * t);
      if (nup > 0) wk.gup = c.take<double>((size_t)nr * nup * (G.s - G.jlow) * t);
    }
    return c.used;
  }
  wk.tables = c.take<float>((size_t)nr * G.table_total + kTablePad);
  wk.U = c.take<float>((size_t)nr * G.urows * ldu);
  if (G.nup > 0) wk.pack = c.take<char>((size_t)levels_pack_bytes(G, nr, t));
  if (op == kOpMatvec) return c.used;
  const bool sep = f->h == QMC_H_ID;
  wk.partial = c.take<double>((size_t)nr * std::max(lp.gx * lp.gy, lg.gx * lg.gy));
  if (!sep) {
    wk.ppart = c.take<float>((size_t)nr * tct * G.N);
    wk.ppartial = c.take<double>((size_t)nr * point_h_blocks(G));
  }
  if (op == kOpGrad) {
    wk.S = c.take<float>((size_t)nr * 2 * G.nsub * ldu);
    wk.dlow = c.take<float>((size_t)nr * lg.gx * tct * (G.jlow > 0 ? G.jlow : 1) * kTileT);
    wk.dup = c.take<float>((size_t)nr * (levels_adj_part_floats(G, t, ldu) + 1));
    if (!sep) wk.hd = c.take<float>((size_t)nr * G.N);
  }
  return c.used;
}

// Stream-ordered workspace owned by one call when the caller passes none.
struct CallWorkspace {
  void *ptr = nullptr;
  hipStream_t st = nullptr;
  ~CallWorkspace() {
    if (ptr) (void)hipFreeAsync(ptr, st);
  }
};

// Workspace of qmc_estimate_static: one array per device for the life of the
// process.  Host code never uses the array's name as an address (on the host
// it is only a stand-in for the symbol): static_scratch() looks up its device
// address once per device, with that device current, and every use goes
// through the address found.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
std::unordered_map<int, void *> g_scratch_ptr;  // device -> device address of scratch

// The device address of `scratch` on `device` (which the caller has made current).
qmc_status static_scratch(int device, void **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch_ptr.find(device);
  if (it == g_scratch_ptr.end()) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr) {
      return fail(QMC_EDEVICE, "static scratch address on device %d: %s", device,
                  e != hipSuccess ? hipGetErrorString(e) : "null address");
    }
    it = g_scratch_ptr.emplace(device, ptr).first;
  }
  *out = it->second;
  return QMC_OK;
}

qmc_status check_points(qmc_points p) {
  if (!p) return fail(QMC_EINVAL, "null point set");
  return QMC_OK;
}

qmc_status check_matrix(const float *A, int32_t t, int64_t lda, int32_t prec) {
  if (!A) return fail(QMC_EINVAL, "A is null");
  if (t < 1) return fail(QMC_EINVAL, "t = %d must be >= 1", t);
  if (t > (1 << 24)) return fail(QMC_EUNSUPPORTED, "t = %d exceeds 2^24", t);
  if (lda < t) return fail(QMC_EINVAL, "lda = %lld < t = %d", (long long)lda, t);
  if (prec != QMC_FP32 && prec != QMC_SPLIT_BF16X3)
    return fail(QMC_EINVAL, "unknown precision %d", prec);
  return QMC_OK;
}

qmc_status check_integrand(const qmc_integrand *f) {
  if (!f) return fail(QMC_EINVAL, "integrand is null");
  if (f->g < QMC_G_ID || f->g > QMC_G_EXP) return fail(QMC_EINVAL, "unknown g %d", f->g);
  if (f->h < QMC_H_ID || f->h > QMC_H_CALL) return fail(QMC_EINVAL, "unknown h %d", f->h);
  return QMC_OK;
}

qmc_status get_workspace(qmc_points p, size_t need, void *ws, size_t ws_bytes, hipStream_t st,
                         CallWorkspace &own, char *&base) {
  (void)p;
  if (ws) {
    if (ws_bytes < need)
      return fail(QMC_ENOMEM, "workspace of %zu bytes is smaller than the %zu required", ws_bytes, need);
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(QMC_EINVAL, "workspace not 256-byte aligned");
    base = static_cast<char *>(ws);
    return QMC_OK;
  }
  if (getenv("QMC_FAULT_INJECT") && strcmp(getenv("QMC_FAULT_INJECT"), "alloc") == 0)
    return fail(QMC_ENOMEM, "workspace allocation failed (fault injection)");
  hipError_t e = hipMallocAsync(&own.ptr, need > 0 ? need : 256, st);
  if (e != hipSuccess) {
    own.ptr = nullptr;
    return fail(QMC_ENOMEM, "workspace allocation of %zu bytes failed: %s", need, hipGetErrorString(e));
  }
  own.st = st;
  base = static_cast<char *>(own.ptr);
  return QMC_OK;
}

}  // namespace

// ------------------------------------------------------------ timing hook
namespace qmc {
qmc_status record_error(qmc_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

LaunchTimer::LaunchTimer(const char *n, hipStream_t s) : name(n), st(s) {
  if (!g_tm_on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) == hipSuccess && hipEventRecord(e, st) == hipSuccess) ev0 = e;
}
LaunchTimer::~LaunchTimer() {
  if (!ev0) return;
  hipEvent_t e1;
  if (hipEventCreate(&e1) != hipSuccess) return;
  if (hipEventRecord(e1, st) != hipSuccess) return;
  std::lock_guard<std::mutex> lk(g_tm_mu);
  g_tm[name].emplace_back((hipEvent_t)ev0, e1);
}
}  // namespace qmc

extern "C" {

const char *qmc_status_string(qmc_status s) {
  switch (s) {
    case QMC_OK: return "success";
    case QMC_EINVAL: return "invalid argument";
    case QMC_EUNSUPPORTED: return "unsupported";
    case QMC_ENOMEM: return "out of memory";
    case QMC_EDEVICE: return "device error";
  }
  return "unknown status";
}

const char *qmc_last_error(void) { return g_last_error.c_str(); }

qmc_status qmc_timing_enable(int32_t on) {
  g_tm_on = on != 0;
  return QMC_OK;
}

qmc_status qmc_timing_reset(void) {
  std::lock_guard<std::mutex> lk(g_tm_mu);
  for (auto &kv : g_tm)
    for (auto &pr : kv.second) {
      (void)hipEventSynchronize(pr.second);
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  g_tm.clear();
  return QMC_OK;
}

qmc_status qmc_timing_read(const char *name, double *ms, int64_t *launches) {
  if (!name || !ms || !launches) return fail(QMC_EINVAL, "null argument");
  std::lock_guard<std::mutex> lk(g_tm_mu);
  *ms = 0.0;
  *launches = 0;
  auto it = g_tm.find(name);
  if (it == g_tm.end()) return QMC_OK;
  for (auto &pr : it->second) {
    QMC_HIP(hipEventSynchronize(pr.second), "hipEventSynchronize");
    float x = 0.f;
    QMC_HIP(hipEventElapsedTime(&x, pr.first, pr.second), "hipEventElapsedTime");
    *ms += x;
    ++*launches;
  }
  return QMC_OK;
}

qmc_status qmc_points_init(qmc_points *out, const qmc_point_spec *sp) {
  using namespace qmc;
  if (!out) return fail(QMC_EINVAL, "out is null");
  *out = nullptr;
  if (!sp) return fail(QMC_EINVAL, "spec is null");
  if (!is_prime(sp->b)) return fail(QMC_EINVAL, "b = %d is not prime", sp->b);
  const int b = sp->b;
  if (sp->m < 1 || sp->m > kMaxM) return fail(QMC_EUNSUPPORTED, "m = %d outside [1, %d]", sp->m, kMaxM);
  int64_t Nb = 1;  // N = b^m
  for (int i = 0; i < sp->m && Nb <= kMaxPoints; ++i) Nb *= b;
  if (Nb > kMaxPoints) return fail(QMC_EUNSUPPORTED, "N = %d^%d exceeds %lld points", b, sp->m, (long long)kMaxPoints);
  if (sp->s < 1) return fail(QMC_EINVAL, "s = %d must be >= 1", sp->s);
  if (sp->kind < QMC_LATTICE || sp->kind > QMC_IID) return fail(QMC_EINVAL, "unknown kind %d", sp->kind);
  const bool iid = sp->kind == QMC_IID;
  if (!sp->w || (!sp->gen && !iid)) return fail(QMC_EINVAL, "w or gen is null");
  const int m = sp->m, s = sp->s;
  if (sp->w[0] != 0) return fail(QMC_EINVAL, "w[0] = %d must be 0", sp->w[0]);
  for (int j = 1; j < s; ++j) {
    if (sp->w[j] < sp->w[j - 1]) return fail(QMC_EINVAL, "w decreases at j = %d", j);
  }
  std::vector<uint32_t> gen;
  std::vector<int32_t> nbv(s);
  for (int j = 0; j < s; ++j) nbv[j] = m - (sp->w[j] < m ? sp->w[j] : m);
  bool nonperiodic = false;
  if (sp->kind == QMC_DIGITAL_NET) {
    gen.resize((size_t)s * m);
    for (int j = 0; j < s; ++j) {
      uint64_t ne = 1;  // b^{e_j}
      for (int i = 0; i < nbv[j]; ++i) ne *= (uint64_t)b;
      for (int q = 0; q < m; ++q) {
        const uint64_t wd = sp->gen[(size_t)j * m + q];
        // base-b digit p-1 of the word is C_{p,q}: the word is below b^m
        if (wd >= (uint64_t)Nb) return fail(QMC_EINVAL, "net column word (j=%d, q=%d) has digits beyond row m", j, q + 1);
        // a column past n_j with nonzero digits in the first n_j rows: the
        // reduced net depends on every digit of k and its products use
        // Algorithm 4 (base 2)
        if (q >= nbv[j] && (b == 2 ? (wd & (ne - 1)) : wd % ne) != 0) nonperiodic = true;
        gen[(size_t)j * m + q] = (uint32_t)wd;
      }
    }
  } else if (sp->kind == QMC_POLY_LATTICE && b != 2) {
    gen.resize(s);
    for (int j = 0; j < s; ++j) {
      const uint64_t g = sp->gen[j];
      uint64_t ne = 1;
      for (int i = 0; i < nbv[j]; ++i) ne *= (uint64_t)b;
      // g'_j(b): digits are the coefficients, degree < e_j, nonzero constant term
      if (nbv[j] == 0 ? g != 1 : (g >= ne || g % (uint64_t)b == 0))
        return fail(QMC_EINVAL, "polynomial %llu of coordinate %d is not a unit of degree < %d over F_%d",
                    (unsigned long long)g, j, nbv[j], b);
      gen[j] = (uint32_t)g;
    }
  } else if (iid) {
    gen.assign(s, 0u);  // reduced Monte Carlo draws no generators
  } else {
    gen.resize(s);
    for (int j = 0; j < s; ++j) {
      const uint64_t z = sp->gen[j];
      uint64_t nj = 1;
      for (int i = 0; i < nbv[j]; ++i) nj *= (uint64_t)b;
      if (nbv[j] == 0) {
        if (z != 1) return fail(QMC_EINVAL, "generator of coordinate %d must be 1 (w_j >= m)", j);
      } else if (z % (uint64_t)b == 0 || z >= nj) {
        // a unit modulo b^e: below b^e and not divisible by the prime b
        return fail(QMC_EINVAL, "generator %llu of coordinate %d is not a unit below %d^%d",
                    (unsigned long long)z, j, b, nbv[j]);
      }
      gen[j] = (uint32_t)z;
    }
  }
  if (sp->rand < QMC_NO_SHIFT || sp->rand > QMC_DIGITAL_SHIFT) return fail(QMC_EINVAL, "unknown randomisation %d", sp->rand);
  if (sp->R < 1) return fail(QMC_EINVAL, "R = %d must be >= 1", sp->R);
  if (iid && sp->rand != QMC_NO_SHIFT)
    return fail(QMC_EINVAL, "reduced Monte Carlo takes no shift (R counts independent replicates)");
  if (!iid && sp->rand == QMC_NO_SHIFT && sp->R != 1) return fail(QMC_EINVAL, "R must be 1 without a shift");
  if (sp->R > 65535) return fail(QMC_EUNSUPPORTED, "R = %d exceeds 65535", sp->R);
  if (sp->rand == QMC_RANDOM_SHIFT) {
    if (!sp->shift) return fail(QMC_EINVAL, "shift is null");
    for (int64_t i = 0; i < (int64_t)sp->R * s; ++i)
      if (!(sp->shift[i] >= 0.0 && sp->shift[i] < 1.0)) return fail(QMC_EINVAL, "shift[%lld] outside [0,1)", (long long)i);
  }
  if (sp->rand == QMC_DIGITAL_SHIFT) {
    if (!sp->dshift) return fail(QMC_EINVAL, "dshift is null");
    uint64_t bK = 1;  // b^K, K digits of the shift: the largest with b^K <= 2^52
    while (bK <= (uint64_t(1) << 52) / (uint64_t)b) bK *= (uint64_t)b;
    for (int64_t i = 0; i < (int64_t)sp->R * s; ++i)
      if (sp->dshift[i] >= bK) return fail(QMC_EINVAL, "dshift[%lld] >= %llu (b^K)", (long long)i, (unsigned long long)bK);
  }
  if (sp->map < QMC_MAP_ID || sp->map > QMC_MAP_TENT) return fail(QMC_EINVAL, "unknown map %d", sp->map);
  if (sp->map == QMC_MAP_INVNORM && sp->rand == QMC_NO_SHIFT && !iid)
    return fail(QMC_EINVAL, "the inverse-normal map needs a shift (x_0 = 0)");
  std::vector<int64_t> soff(s);
  int64_t sample_total = 0;
  for (int j = 0; j < s; ++j) {
    soff[j] = sample_total;
    int64_t nj = 1;
    for (int i = 0; i < nbv[j]; ++i) nj *= b;
    sample_total += nj;
  }
  if (iid) {
    if (!sp->samples) return fail(QMC_EINVAL, "samples is null");
    const bool open = sp->map == QMC_MAP_INVNORM;
    for (int64_t i = 0; i < (int64_t)sp->R * sample_total; ++i) {
      const double u = sp->samples[i];
      if (!(u >= 0.0 && u < 1.0) || (open && u == 0.0))
        return fail(QMC_EINVAL, "samples[%lld] = %g outside %s", (long long)i, u, open ? "(0,1)" : "[0,1)");
    }
  }

  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return fail(QMC_EDEVICE, "no HIP device");

  int device = 0;
  QMC_HIP(hipGetDevice(&device), "hipGetDevice");
  // value tables of the gather path: their byte offsets are 32-bit in the kernels
  const int64_t gather_total = nonperiodic ? sample_total : b != 2 ? 2 * sample_total : 0;
  if (gather_total >= kAlg4MaxValues)
    return fail(QMC_EUNSUPPORTED, "value tables of %lld floats reach %lld", (long long)gather_total,
                (long long)kAlg4MaxValues);
  // a net over F_b, b > 2, that is not periodic keeps one index word per point
  // and coordinate
  if (nonperiodic && b != 2 && ceil_div(Nb, 64) * 64 * s > kMaxIndexWords)
    return fail(QMC_EUNSUPPORTED, "a net over F_%d that is not periodic needs N s = %lld index words (at most %lld)",
                b, (long long)(Nb * s), (long long)kMaxIndexWords);

  qmc_points p = new qmc_points_s();
  p->device = device;
  qmc::Geometry &G = p->G;
  G.m = m;
  G.s = s;
  G.kind = sp->kind;
  G.rand = sp->rand;
  G.map = sp->map;
  G.R = sp->R;
  G.b = b;
  G.nonperiodic = nonperiodic ? 1 : 0;
  p->Gg = G;
  plan_geometry(G, sp->w, kMaxSplit);
  plan_geometry(p->Gg, sp->w, kMaxSplitGrad);
  // the cascade below is planned in base 2; a base b > 2 takes the gather path
  G.gather = nonperiodic || b != 2 ? 1 : 0;
  if (nonperiodic) {  // one pass over every coordinate and point
    G.N = Nb;
    G.jlow = s;
    G.split = -1;
    G.nsub = 0;
  } else if (b != 2) {
    plan_gather_split(G, sp->w, Nb);
  }
  G.gather_total = gather_total;
  if (G.gather) p->Gg = G;  // the gathered path plans one layout for every operation

  auto cleanup = [&](qmc_status st) {
    qmc_points_free(p);
    return st;
  };
  hipError_t e;
  if ((e = hipMalloc(&p->d_gen, gen.size() * 4)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipMemcpy(p->d_gen, gen.data(), gen.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy"));
  if ((e = hipMalloc(&p->d_nb, (size_t)s * 4)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipMemcpy(p->d_nb, nbv.data(), (size_t)s * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy"));
  const size_t nshift = (size_t)sp->R * s;
  if (sp->rand == QMC_RANDOM_SHIFT) {
    if ((e = hipMalloc(&p->d_shift, nshift * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(p->d_shift, sp->shift, nshift * 8, hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemcpy"));
  }
  if (sp->rand == QMC_DIGITAL_SHIFT) {
    if ((e = hipMalloc(&p->d_dshift, nshift * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(p->d_dshift, sp->dshift, nshift * 8, hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemcpy"));
  }
  if (iid) {
    const size_t nsamp = (size_t)sp->R * sample_total;
    if ((e = hipMalloc(&p->d_samples, nsamp * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
    if ((e = hipMemcpy(p->d_samples, sp->samples, nsamp * 8, hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemcpy"));
  }
  // start of each coordinate's n_j values (samples of reduced Monte Carlo,
  // value tables of Algorithm 4)
  if ((e = hipMalloc(&p->d_soff, (size_t)s * 8)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
  if ((e = hipMemcpy(p->d_soff, soff.data(), (size_t)s * 8, hipMemcpyHostToDevice)) != hipSuccess)
    return cleanup(hip_fail(e, "hipMemcpy"));
  if (G.gather) {  // gather path: table starts and index words, once
    std::vector<uint32_t> aoff(s);
    if (nonperiodic && b != 2) {
      // one table of n_j values per coordinate, read by their output integer
      for (int j = 0; j < s; ++j) aoff[j] = (uint32_t)soff[j];
    } else if (nonperiodic) {
      // tables in order of decreasing n_j: every start is a multiple of its n_j
      std::vector<int> ord(s);
      for (int j = 0; j < s; ++j) ord[j] = j;
      std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return nbv[x] > nbv[y]; });
      int64_t pos = 0;
      for (int j : ord) {
        aoff[j] = (uint32_t)pos;
        pos += int64_t(1) << nbv[j];
      }
    } else {
      // base b > 2: each table holds its n_j values twice
      for (int j = 0; j < s; ++j) aoff[j] = (uint32_t)(2 * soff[j]);
    }
    const size_t words = (size_t)alg4_index_words(G);
    if ((e = hipMalloc(&p->d_yidx, (words + s) * 4)) != hipSuccess) return cleanup(hip_fail(e, "hipMalloc"));
    uint32_t *ylo = static_cast<uint32_t *>(p->d_yidx), *ytile = ylo + (size_t)64 * s, *daoff = ylo + words;
    if ((e = hipMemcpy(daoff, aoff.data(), (size_t)s * 4, hipMemcpyHostToDevice)) != hipSuccess)
      return cleanup(hip_fail(e, "hipMemcpy"));
    if ((e = launch_alg4_index(G, static_cast<const uint32_t *>(p->d_gen), static_cast<const int32_t *>(p->d_nb),
                               daoff, ylo, ytile, nullptr)) != hipSuccess ||
        (e = hipDeviceSynchronize()) != hipSuccess)
      return cleanup(hip_fail(e, "Algorithm 4 index tables"));
    p->D.aoff = daoff;
    p->D.ylo = ylo;
    p->D.ytile = ytile;
  }
  p->D.samples = static_cast<const double *>(p->d_samples);
  p->D.soff = static_cast<const int64_t *>(p->d_soff);
  p->D.sample_total = sample_total;
  p->D.gen = static_cast<const uint32_t *>(p->d_gen);
  p->D.nbj = static_cast<const int32_t *>(p->d_nb);
  p->D.shift = static_cast<const double *>(p->d_shift);
  p->D.dshift = static_cast<const uint64_t *>(p->d_dshift);
  *out = p;
  return QMC_OK;
}

qmc_status qmc_points_free(qmc_points p) {
  if (!p) return QMC_OK;
  DeviceGuard dg(p->device);
  if (p->d_gen) (void)hipFree(p->d_gen);
  if (p->d_nb) (void)hipFree(p->d_nb);
  if (p->d_shift) (void)hipFree(p->d_shift);
  if (p->d_dshift) (void)hipFree(p->d_dshift);
  if (p->d_samples) (void)hipFree(p->d_samples);
  if (p->d_soff) (void)hipFree(p->d_soff);
  if (p->d_yidx) (void)hipFree(p->d_yidx);
  delete p;
  return QMC_OK;
}

qmc_status qmc_points_info(qmc_points p, int64_t *N, int32_t *s, int32_t *R, int32_t *split_level,
                           int64_t *distinct_values) {
  if (qmc_status st = check_points(p)) return st;
  if (N) *N = p->G.N;
  if (s) *s = p->G.s;
  if (R) *R = p->G.R;
  // -1: gathered tiles in one pass; base b > 2 with a root table reports its level
  if (split_level) *split_level = p->G.gather && p->G.jlow == p->G.s ? -1 : p->G.split;
  if (distinct_values) *distinct_values = p->G.gather ? p->D.sample_total : p->G.table_total;
  return QMC_OK;
}

qmc_status qmc_points_grad_split(qmc_points p, int32_t *split_level) {
  if (qmc_status st = check_points(p)) return st;
  if (!split_level) return fail(QMC_EINVAL, "split_level is null");
  *split_level = p->Gg.gather && p->Gg.jlow == p->Gg.s ? -1 : p->Gg.split;
  return QMC_OK;
}

qmc_status qmc_point_values(qmc_points p, int32_t r, int32_t j, double *out, void *stream) {
  if (qmc_status st = check_points(p)) return st;
  if (r < 0 || r >= p->G.R) return fail(QMC_EINVAL, "r = %d outside [0, %d)", r, p->G.R);
  if (j < 0 || j >= p->G.s) return fail(QMC_EINVAL, "j = %d outside [0, %d)", j, p->G.s);
  if (!out) return fail(QMC_EINVAL, "out is null");
  DeviceGuard dg(p->device);
  QMC_HIP(qmc::launch_point_values(p->G, p->D, r, j, out, (hipStream_t)stream), "point values launch");
  return QMC_OK;
}

qmc_status qmc_point_matrix(qmc_points p, int32_t r, float *X, int64_t ldx, void *stream) {
  if (qmc_status st = check_points(p)) return st;
  if (r < 0 || r >= p->G.R) return fail(QMC_EINVAL, "r = %d outside [0, %d)", r, p->G.R);
  if (!X) return fail(QMC_EINVAL, "X is null");
  if (ldx < p->G.s) return fail(QMC_EINVAL, "ldx = %lld < s = %d", (long long)ldx, p->G.s);
  DeviceGuard dg(p->device);
  QMC_HIP(qmc::launch_point_matrix(p->G, p->D, r, X, ldx, (hipStream_t)stream), "point matrix launch");
  return QMC_OK;
}

qmc_status qmc_workspace_size(qmc_points p, int32_t op, int32_t t, const qmc_integrand *f,
                              int32_t prec, size_t *bytes) {
  if (qmc_status st = check_points(p)) return st;
  if (!bytes) return fail(QMC_EINVAL, "bytes is null");
  if (op < kOpMatvec || op > kOpGrad) return fail(QMC_EINVAL, "unknown op %d", op);
  if (t < 1) return fail(QMC_EINVAL, "t = %d must be >= 1", t);
  if (prec != QMC_FP32 && prec != QMC_SPLIT_BF16X3) return fail(QMC_EINVAL, "unknown precision %d", prec);
  qmc_integrand dflt{QMC_G_ID, 0.0, QMC_H_ID, 0.0};
  if (op != kOpMatvec) {
    if (qmc_status st = check_integrand(f)) return st;
  } else {
    f = &dflt;
  }
  DeviceGuard dg(p->device);  // the leaf plan queries the device's occupancy
  Work wk;
  *bytes = carve(op == kOpGrad ? p->Gg : p->G, op, t, f, op == kOpMatvec ? 1 : p->G.R, prec, nullptr, wk);
  return QMC_OK;
}

// Gather path: for a base b > 2 with a split, the upper coordinates over the
// n_split residues into the root table (timed as "levels"); `lower` becomes
// the pass of the lower coordinates over all N points adding the root rows
// (otherwise the one pass over everything).
static hipError_t gather_root(const qmc::Geometry &G, const qmc::DevSpec &D, int prec, const float *tables,
                              int nr, const float *A, int t, int64_t lda, float *root, qmc::Alg4Pass &lower,
                              hipStream_t st) {
  using namespace qmc;
  lower = alg4_whole(G);
  if (G.jlow < G.s) {
    Alg4Pass up{};
    up.j0 = G.jlow;
    up.sc = G.s - G.jlow;
    up.npts = G.nsub;
    up.timer = "levels";
    Alg4Out ro{};
    ro.Y = root;
    ro.ldy = t;
    ro.ystride = G.nsub * t;
    const qmc_integrand fid{QMC_G_ID, 0.0, QMC_H_ID, 0.0};
    const hipError_t e = launch_alg4(G, D, kModeStoreY, fid, prec, tables, nr, A, t, lda, up, ro, st);
    if (e != hipSuccess) return e;
    lower.sc = G.jlow;
    lower.root = root;
    lower.ldp = t;
    lower.root_stride = G.nsub * t;
    lower.nsplit = G.nsub;
  }
  return hipSuccess;
}

static hipError_t gather_passes(const qmc::Geometry &G, const qmc::DevSpec &D, int mode,
                                const qmc_integrand &f, int prec, const float *tables, int nr,
                                const float *A, int t, int64_t lda, float *root, const qmc::Alg4Out &o,
                                hipStream_t st) {
  using namespace qmc;
  Alg4Pass lower;
  const hipError_t e = gather_root(G, D, prec, tables, nr, A, t, lda, root, lower, st);
  if (e != hipSuccess) return e;
  return launch_alg4(G, D, mode, f, prec, tables, nr, A, t, lda, lower, o, st);
}

// Gradient on the gather path: the sensitivities G_n = h'(u_n) g'(y_n) / (N t)
// of every point (a pass over the points in the gradient mode, after the point
// means when h is not the identity), then dA = X^T G: the lower coordinates
// over all N points, the upper ones (base b > 2 with a split) over the fold of
// G into the n_split residues, and the chunk partials added in FP64.
static hipError_t gather_grad(const qmc::Geometry &G, const qmc::DevSpec &D, const qmc_integrand &f, int prec,
                              const Work &wk, int nr, const float *A, int t, int64_t lda, double *Q, float *dA,
                              hipStream_t st) {
  using namespace qmc;
  const bool sep = f.h == QMC_H_ID;
  const double inv_nt = 1.0 / ((double)G.N * (double)t);
  Alg4Pass lower;
  hipError_t e = gather_root(G, D, prec, wk.tables, nr, A, t, lda, wk.root, lower, st);
  if (e != hipSuccess) return e;
  Alg4Out o{};
  o.Y = wk.Gm;
  o.ldy = t;
  o.ystride = G.N * t;
  o.gscale = inv_nt;
  if (sep) {
    o.partial = wk.partial;
    if ((e = launch_alg4(G, D, kModeGrad, f, prec, wk.tables, nr, A, t, lda, lower, o, st)) != hipSuccess) return e;
    if ((e = launch_reduce(wk.partial, nr, alg4_point_tiles(G) * alg4_col_tiles(t), inv_nt, Q, st)) != hipSuccess)
      return e;
  } else {
    Alg4Out op{};
    op.ppart = wk.ppart;
    if ((e = launch_alg4(G, D, kModePoint, f, prec, wk.tables, nr, A, t, lda, lower, op, st)) != hipSuccess) return e;
    const int64_t blocks = point_h_blocks(G);
    if ((e = launch_point_h(G, f, wk.ppart, nr, alg4_col_tiles(t), t, wk.ppartial, blocks, wk.hd, 1.0, st)) !=
        hipSuccess)
      return e;
    if ((e = launch_reduce(wk.ppartial, nr, blocks, 1.0 / (double)G.N, Q, st)) != hipSuccess) return e;
    o.hd = wk.hd;
    if ((e = launch_alg4(G, D, kModeGrad, f, prec, wk.tables, nr, A, t, lda, lower, o, st)) != hipSuccess) return e;
  }
  const int nlo = alg4_adj_chunks(G.jlow, G.N, t, nr), nup = alg4_adj_chunks(G.s - G.jlow, G.nsub, t, nr);
  if ((e = launch_alg4_adj(G, D, prec, wk.tables, nr, wk.Gm, G.N * t, 0, G.jlow, G.N, nlo, t, wk.glow, st)) !=
      hipSuccess)
    return e;
  if (nup > 0) {
    if ((e = launch_alg4_fold(G, wk.Gm, nr, t, wk.S, st)) != hipSuccess) return e;
    if ((e = launch_alg4_adj(G, D, prec, wk.tables, nr, wk.S, G.nsub * t, G.jlow, G.s - G.jlow, G.nsub, nup, t,
                             wk.gup, st)) != hipSuccess)
      return e;
  }
  return launch_alg4_adj_combine(G, wk.glow, nlo, wk.gup, nup, nr, t, dA, st);
}

qmc_status qmc_reduced_matvec(qmc_points p, int32_t r, const float *A, int32_t t, int64_t lda,
                              int32_t prec, float *Y, int64_t ldy, void *workspace,
                              size_t workspace_bytes, void *stream) {
  using namespace qmc;
  if (qmc_status st = check_points(p)) return st;
  if (qmc_status st = check_matrix(A, t, lda, prec)) return st;
  if (r < 0 || r >= p->G.R) return fail(QMC_EINVAL, "r = %d outside [0, %d)", r, p->G.R);
  if (!Y) return fail(QMC_EINVAL, "Y is null");
  if (ldy < t) return fail(QMC_EINVAL, "ldy = %lld < t = %d", (long long)ldy, t);
  DeviceGuard dg(p->device);
  hipStream_t st = (hipStream_t)stream;
  const qmc_integrand fid{QMC_G_ID, 0.0, QMC_H_ID, 0.0};
  Work wk;
  const size_t need = carve(p->G, kOpMatvec, t, &fid, 1, prec, nullptr, wk);
  CallWorkspace own;
  char *base = nullptr;
  if (qmc_status s2 = get_workspace(p, need, workspace, workspace_bytes, st, own, base)) return s2;
  carve(p->G, kOpMatvec, t, &fid, 1, prec, base, wk);
  const int64_t ldu = round_up(t, kTileT);
  const Geometry &G = p->G;
  if (G.gather) {  // gathered value tiles
    QMC_HIP(launch_output_tables(G, p->D, r, 1, wk.tables, st), "tables launch");
    Alg4Out o{};
    o.Y = Y;
    o.ldy = ldy;
    QMC_HIP(gather_passes(G, p->D, kModeStoreY, fid, prec, wk.tables, 1, A, t, lda, wk.root, o, st),
            "gathered tiles launch");
    return QMC_OK;
  }
  QMC_HIP(launch_tables(G, p->D, r, 1, wk.tables, nullptr, 0, st), "tables launch");
  QMC_HIP(launch_levels(G, prec, wk.tables, 1, A, t, lda, wk.U, ldu, 1.0f, wk.pack, st), "levels launch");
  LeafOut o{};
  o.Y = Y;
  o.ldy = ldy;
  QMC_HIP(launch_leaf(G, kModeStoreY, fid, wk.tables, wk.U, 1, r, A, t, lda, ldu, leaf_plan(G, t, 1, kModeStoreY, QMC_G_ID), o, st),
          "leaf launch");
  return QMC_OK;
}

static qmc_status estimate_impl(qmc_points p, const float *A, int32_t t, int64_t lda,
                                const qmc_integrand *f, int32_t prec, double *Q, float *dA,
                                void *workspace, size_t workspace_bytes, void *stream) {
  using namespace qmc;
  if (qmc_status st = check_points(p)) return st;
  if (qmc_status st = check_matrix(A, t, lda, prec)) return st;
  if (qmc_status st = check_integrand(f)) return st;
  if (!Q) return fail(QMC_EINVAL, "Q is null");
  const bool grad = dA != nullptr;
  DeviceGuard dg(p->device);
  hipStream_t st = (hipStream_t)stream;
  const Geometry &G = grad ? p->Gg : p->G;
  const int nr = G.R;
  const int op = grad ? kOpGrad : kOpEstimate;
  Work wk;
  const size_t need = carve(G, op, t, f, nr, prec, nullptr, wk);
  CallWorkspace own;
  char *base = nullptr;
  if (qmc_status s2 = get_workspace(p, need, workspace, workspace_bytes, st, own, base)) return s2;
  carve(G, op, t, f, nr, prec, base, wk);
  const int64_t ldu = round_up(t, kTileT);
  const int tct = (int)ceil_div(t, kTileT);
  const LeafPlan lp = leaf_plan(G, t, nr, kModeSum, f->g);
  const LeafPlan lg = leaf_plan(G, t, nr, kModeGrad, f->g);
  const bool sep = f->h == QMC_H_ID;
  const double inv_nt = 1.0 / ((double)G.N * (double)t);

  if (G.gather) {  // value tables, then the fused tile products
    QMC_HIP(launch_output_tables(G, p->D, 0, nr, wk.tables, st), "tables launch");
    if (grad) {
      QMC_HIP(gather_grad(G, p->D, *f, prec, wk, nr, A, t, lda, Q, dA, st), "gradient launch");
      return QMC_OK;
    }
    Alg4Out o{};
    if (sep) {
      o.partial = wk.partial;
      QMC_HIP(gather_passes(G, p->D, kModeSum, *f, prec, wk.tables, nr, A, t, lda, wk.root, o, st),
              "gathered tiles launch");
      QMC_HIP(launch_reduce(wk.partial, nr, alg4_point_tiles(G) * alg4_col_tiles(t), inv_nt, Q, st),
              "reduce launch");
    } else {
      o.ppart = wk.ppart;
      QMC_HIP(gather_passes(G, p->D, kModePoint, *f, prec, wk.tables, nr, A, t, lda, wk.root, o, st),
              "gathered tiles launch");
      const int64_t blocks = point_h_blocks(G);
      QMC_HIP(launch_point_h(G, *f, wk.ppart, nr, alg4_col_tiles(t), t, wk.ppartial, blocks, nullptr, 1.0, st),
              "point h launch");
      QMC_HIP(launch_reduce(wk.ppartial, nr, blocks, 1.0 / (double)G.N, Q, st), "reduce launch");
    }
    return QMC_OK;
  }

  QMC_HIP(launch_tables(G, p->D, 0, nr, wk.tables, nullptr, 0, st), "tables launch");
  const int leaf_mode = !sep ? kModePoint : (grad ? kModeGrad : kModeSum);
  QMC_HIP(launch_levels(G, prec, wk.tables, nr, A, t, lda, wk.U, ldu, g_scale(*f, leaf_mode), wk.pack, st),
          "levels launch");
  LeafOut o{};
  if (sep) {
    if (!grad) {
      o.partial = wk.partial;
      QMC_HIP(launch_leaf(G, kModeSum, *f, wk.tables, wk.U, nr, 0, A, t, lda, ldu, lp, o, st), "leaf launch");
      QMC_HIP(launch_reduce(wk.partial, nr, (int64_t)lp.gx * lp.gy, inv_nt, Q, st), "reduce launch");
      return QMC_OK;
    }
  } else {
    // per-point sums over all columns, then h and the mean
    o.ppart = wk.ppart;
    const LeafPlan lpp = leaf_plan(G, t, nr, kModePoint, f->g);
    QMC_HIP(launch_leaf(G, kModePoint, *f, wk.tables, wk.U, nr, 0, A, t, lda, ldu, lpp, o, st), "leaf launch");
    const int64_t blocks = point_h_blocks(G);
    QMC_HIP(launch_point_h(G, *f, wk.ppart, nr, tct, t, wk.ppartial, blocks, grad ? wk.hd : nullptr,
                           1.0, st),
            "point h launch");
    QMC_HIP(launch_reduce(wk.ppartial, nr, blocks, 1.0 / (double)G.N, Q, st), "reduce launch");
    if (!grad) return QMC_OK;
  }
  // adjoint: G_ki = h'(u_k) g'(y_ki) / (N t); the kernels work with
  // G'_ki = h'(u_k) g'_unit(y_ki) and the combination applies the factor
  LeafOut g{};
  g.partial = wk.partial;
  g.dApart = wk.dlow;
  g.Sroot = wk.S;
  g.hd = sep ? nullptr : wk.hd;
  QMC_HIP(launch_leaf(G, kModeGrad, *f, wk.tables, wk.U, nr, 0, A, t, lda, ldu, lg, g, st), "adjoint leaf launch");
  if (sep) QMC_HIP(launch_reduce(wk.partial, nr, (int64_t)lg.gx * lg.gy, inv_nt, Q, st), "reduce launch");
  QMC_HIP(launch_fold(G, nr, wk.S, t, ldu, st), "fold launch");
  QMC_HIP(launch_levels_adj(G, prec, wk.tables, nr, wk.S, t, ldu, wk.dup, st), "adjoint levels launch");
  QMC_HIP(launch_combine(G, wk.dlow, lg.gx, tct, wk.dup, nr, t, ldu, inv_nt * g_der_factor(*f), dA, st),
          "combine launch");
  return QMC_OK;
}

qmc_status qmc_estimate(qmc_points p, const float *A, int32_t t, int64_t lda, const qmc_integrand *f,
                        int32_t prec, double *Q, void *workspace, size_t workspace_bytes, void *stream) {
  return estimate_impl(p, A, t, lda, f, prec, Q, nullptr, workspace, workspace_bytes, stream);
}

qmc_status qmc_estimate_static(qmc_points p, const float *A, int32_t t, int64_t lda,
                               const qmc_integrand *f, int32_t prec, double *Q, void *stream) {
  using namespace qmc;
  if (qmc_status st = check_points(p)) return st;
  if (qmc_status st = check_matrix(A, t, lda, prec)) return st;
  if (qmc_status st = check_integrand(f)) return st;
  if (!Q) return fail(QMC_EINVAL, "Q is null");
  DeviceGuard dg(p->device);
  Work wk;
  const size_t need = carve(p->G, kOpEstimate, t, f, p->G.R, prec, nullptr, wk);
  if (need > kStaticScratchBytes)
    return fail(QMC_ENOMEM, "the estimate needs %zu bytes of workspace; the static scratch holds %zu",
                need, (size_t)kStaticScratchBytes);
  void *ws = nullptr;
  if (qmc_status st = static_scratch(p->device, &ws)) return st;
  return estimate_impl(p, A, t, lda, f, prec, Q, nullptr, ws, kStaticScratchBytes, stream);
}

qmc_status qmc_estimate_grad(qmc_points p, const float *A, int32_t t, int64_t lda,
                             const qmc_integrand *f, int32_t prec, double *Q, float *dA,
                             void *workspace, size_t workspace_bytes, void *stream) {
  if (!dA) return fail(QMC_EINVAL, "dA is null");
  return estimate_impl(p, A, t, lda, f, prec, Q, dA, workspace, workspace_bytes, stream);
}

}  // extern "C"
