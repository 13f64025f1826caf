// Drives the host-side validation of libqmcred's C ABI under AddressSanitizer
// and UndefinedBehaviorSanitizer (the library's host code built with
// -Xarch_host sanitizers by tests/test_sanitizers.py).  Every call here is
// refused on the host before any device call, so no GPU is needed.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "qmcred.h"

static int expect(qmc_status got, qmc_status want, const char *what) {
  if (got != want) {
    std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, qmc_last_error());
    return 1;
  }
  if (got != QMC_OK && std::strlen(qmc_last_error()) == 0) {
    std::fprintf(stderr, "%s: no error detail\n", what);
    return 1;
  }
  return 0;
}

int main() {
  int bad = 0;
  const int s = 8, m = 6;
  std::vector<int32_t> w = {0, 1, 1, 2, 2, 2, 2, 3};
  std::vector<uint64_t> gen = {1, 3, 5, 7, 9, 11, 13, 3};
  std::vector<double> shift(2 * s, 0.25);
  std::vector<uint64_t> dshift(2 * s, 12345);
  qmc_point_spec sp{};
  auto reset = [&]() {
    sp = qmc_point_spec{};
    sp.b = 2; sp.m = m; sp.s = s; sp.kind = QMC_LATTICE; sp.w = w.data(); sp.gen = gen.data();
    sp.rand = QMC_RANDOM_SHIFT; sp.R = 2; sp.shift = shift.data(); sp.dshift = dshift.data(); sp.map = QMC_MAP_ID;
  };
  qmc_points p = nullptr;
  reset(); sp.b = 4;  bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "b not prime");
  reset(); sp.m = 0;  bad |= expect(qmc_points_init(&p, &sp), QMC_EUNSUPPORTED, "m = 0");
  reset(); sp.m = 25; bad |= expect(qmc_points_init(&p, &sp), QMC_EUNSUPPORTED, "m = 25");
  reset(); sp.b = 3; sp.m = 16; bad |= expect(qmc_points_init(&p, &sp), QMC_EUNSUPPORTED, "3^16 points");
  reset(); sp.s = 0;  bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "s = 0");
  reset(); sp.kind = 9; bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "unknown kind");
  reset(); sp.w = nullptr; bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "w null");
  {
    std::vector<int32_t> w2 = w; w2[0] = 1;
    reset(); sp.w = w2.data(); bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "w[0] != 0");
    w2 = w; w2[5] = 1;
    reset(); sp.w = w2.data(); bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "w decreasing");
  }
  {
    std::vector<uint64_t> g2 = gen; g2[3] = 4;  // even: not a unit modulo 2^e
    reset(); sp.gen = g2.data(); bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "even generator");
    g2 = gen; g2[1] = 1u << 20;
    reset(); sp.gen = g2.data(); bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "generator too large");
  }
  {
    std::vector<uint64_t> net((size_t)s * m, 1);
    net[3] = uint64_t(1) << 40;  // digits beyond row m
    reset(); sp.kind = QMC_DIGITAL_NET; sp.gen = net.data(); sp.rand = QMC_DIGITAL_SHIFT;
    bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "net word beyond row m");
  }
  reset(); sp.rand = 7; bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "unknown randomisation");
  reset(); sp.R = 0; bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "R = 0");
  reset(); sp.rand = QMC_NO_SHIFT; bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "R > 1 without shift");
  {
    std::vector<double> sh = shift; sh[5] = 1.0;
    reset(); sp.shift = sh.data(); bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "shift = 1");
    sh[5] = std::nan("");
    reset(); sp.shift = sh.data(); bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "shift NaN");
  }
  {
    std::vector<uint64_t> ds = dshift; ds[2] = uint64_t(1) << 52;
    reset(); sp.rand = QMC_DIGITAL_SHIFT; sp.dshift = ds.data();
    bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "digital shift 2^52");
  }
  reset(); sp.map = QMC_MAP_INVNORM; sp.rand = QMC_NO_SHIFT; sp.R = 1;
  bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "inverse normal without shift");
  reset(); sp.kind = QMC_IID; sp.rand = QMC_NO_SHIFT; sp.samples = nullptr;
  bad |= expect(qmc_points_init(&p, &sp), QMC_EINVAL, "reduced Monte Carlo without samples");
  bad |= expect(qmc_points_init(nullptr, &sp), QMC_EINVAL, "out null");
  bad |= expect(qmc_points_init(&p, nullptr), QMC_EINVAL, "spec null");
  // calls on a null point set are refused before anything else
  float dummy = 0.f;
  double q = 0.0;
  qmc_integrand f{QMC_G_COS, 1.0, QMC_H_ID, 0.0};
  bad |= expect(qmc_estimate(nullptr, &dummy, 4, 4, &f, 0, &q, nullptr, 0, nullptr), QMC_EINVAL, "estimate null points");
  bad |= expect(qmc_estimate_static(nullptr, &dummy, 4, 4, &f, 0, &q, nullptr), QMC_EINVAL, "static null points");
  bad |= expect(qmc_estimate_grad(nullptr, &dummy, 4, 4, &f, 0, &q, &dummy, nullptr, 0, nullptr), QMC_EINVAL,
                "grad null points");
  bad |= expect(qmc_reduced_matvec(nullptr, 0, &dummy, 4, 4, 0, &dummy, 4, nullptr, 0, nullptr), QMC_EINVAL,
                "matvec null points");
  bad |= expect(qmc_points_free(nullptr), QMC_OK, "free null");
  for (int c = 0; c <= 5; ++c)
    if (!qmc_status_string((qmc_status)c) || !*qmc_status_string((qmc_status)c)) bad = 1;
  std::printf(bad ? "host driver: FAILED\n" : "host driver: ok\n");
  return bad;
}
