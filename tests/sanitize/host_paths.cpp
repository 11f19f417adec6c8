// Host paths of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer:
// the coefficient solves, configuration planning and validation, and the
// error and cleanup paths of creation, which run before (or without) any
// device work.  Built and run by tests/test_host_sanitizers.py; exits 0 when
// every check holds (a sanitizer report aborts with a nonzero status).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "nflbm.h"

static int failures = 0;
#define CHECK(cond)                                              \
  do {                                                           \
    if (!(cond)) {                                               \
      std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                \
    }                                                            \
  } while (0)

// deterministic tensions in [0.003, 0.009]
static std::vector<double> tensions(int N, unsigned seed) {
  std::vector<double> s(size_t(N) * N, 0.0);
  unsigned x = seed * 2654435761u + 12345u;
  for (int i = 0; i < N; ++i)
    for (int j = i + 1; j < N; ++j) {
      x = x * 1664525u + 1013904223u;
      const double v = 0.003 + 0.006 * double(x >> 8) / double(1u << 24);
      s[size_t(i) * N + j] = s[size_t(j) * N + i] = v;
    }
  return s;
}

static nflbm_config config(int lattice, int nx, int ny, int nz, int N, const double* sigma, const double* tau) {
  nflbm_config c;
  std::memset(&c, 0, sizeof(c));
  c.lattice = lattice;
  c.nx = nx;
  c.ny = ny;
  c.nz = nz;
  c.ncomp = N;
  c.implicit_comp = -1;
  c.sigma = sigma;
  c.tau = tau;
  c.width_D = 4.0;
  c.m = 0.05;
  c.precision = NFLBM_FP32;
  return c;
}

int main() {
  CHECK(nflbm_abi_version() == NFLBM_ABI_VERSION);

  // coefficient tables for every N: alpha symmetric with zero row sums
  for (int N = 2; N <= NFLBM_MAX_COMP; ++N) {
    const std::vector<double> s = tensions(N, unsigned(N));
    std::vector<double> a(size_t(N) * N), g(N), psi(size_t(N) * N * N), x(psi.size()), z(psi.size());
    CHECK(nflbm_coefficients(N, s.data(), 4.0, a.data(), g.data(), psi.data(), x.data(), z.data()) == NFLBM_OK);
    for (int i = 0; i < N; ++i) {
      double row = 0.0;
      for (int j = 0; j < N; ++j) {
        row += a[size_t(i) * N + j];
        CHECK(std::fabs(a[size_t(i) * N + j] - a[size_t(j) * N + i]) <= 1e-9 * std::fabs(a[size_t(i) * N + i]));
      }
      CHECK(std::fabs(row) <= 1e-9 * std::fabs(a[size_t(i) * N + i]));
    }
    CHECK(nflbm_coefficients(N, s.data(), 4.0, nullptr, nullptr, nullptr, nullptr, nullptr) == NFLBM_OK);
  }
  {
    const double bad[4] = {0.0, -1.0, -1.0, 0.0};
    CHECK(nflbm_coefficients(2, bad, 4.0, nullptr, nullptr, nullptr, nullptr, nullptr) == NFLBM_EINVAL);
    CHECK(nflbm_coefficients(1, bad, 4.0, nullptr, nullptr, nullptr, nullptr, nullptr) == NFLBM_EINVAL);
    CHECK(nflbm_coefficients(9, bad, 4.0, nullptr, nullptr, nullptr, nullptr, nullptr) == NFLBM_EINVAL);
    CHECK(nflbm_coefficients(3, nullptr, 4.0, nullptr, nullptr, nullptr, nullptr, nullptr) == NFLBM_EINVAL);
    CHECK(std::strlen(nflbm_last_error(nullptr)) > 0);
  }

  // planning: every lattice, precision and storage form; invalid inputs
  const std::vector<double> s5 = tensions(5, 5u);
  const double tau5[5] = {1.0, 1.0, 1.0, 1.0, 1.0};
  const double taug[5] = {1.0, 0.8, 1.0, 1.0, 1.0};
  for (int lat = 0; lat < 2; ++lat)
    for (int prec = 0; prec < 3; ++prec)
      for (int flags : {0, int(NFLBM_FLAG_G_POPULATIONS), int(NFLBM_FLAG_C2C2_MOBILITY), int(NFLBM_FLAG_NO_HYDRO)}) {
        nflbm_config c = config(lat, 20, 16, lat ? 12 : 1, 5, s5.data(), tau5);
        c.precision = prec;
        c.flags = flags;
        if (flags == NFLBM_FLAG_C2C2_MOBILITY) c.m = 10.0;
        size_t bytes = 0;
        CHECK(nflbm_device_bytes(&c, &bytes) == NFLBM_OK);
        CHECK(bytes > 0);
        c.tau_g = taug;
        if (flags != NFLBM_FLAG_C2C2_MOBILITY) CHECK(nflbm_device_bytes(&c, &bytes) == NFLBM_OK);
      }
  {
    size_t bytes = 0;
    nflbm_config c = config(NFLBM_D3Q19, 646, 646, 646, 4, s5.data(), tau5);
    std::vector<double> s4 = tensions(4, 4u);
    c.sigma = s4.data();
    c.m = 0.1;
    CHECK(nflbm_device_bytes(&c, &bytes) == NFLBM_ENOTSUP);      // 32-bit per-node offsets
    nflbm_config bad = config(NFLBM_D2Q9, 8, 8, 2, 5, s5.data(), tau5);
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EINVAL);     // D2Q9 needs nz = 1
    bad = config(NFLBM_D2Q9, 0, 8, 1, 5, s5.data(), tau5);
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EINVAL);
    bad = config(7, 8, 8, 1, 5, s5.data(), tau5);
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EINVAL);
    bad = config(NFLBM_D2Q9, 8, 8, 1, 5, nullptr, tau5);
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EINVAL);
    bad = config(NFLBM_D2Q9, 8, 8, 1, 5, s5.data(), tau5);
    bad.m = 0.3;
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EUNSTABLE);
    bad.flags = NFLBM_FLAG_ALLOW_UNSTABLE;
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_OK);
    const double tbad[5] = {1.0, 0.5, 1.0, 1.0, 1.0};
    bad = config(NFLBM_D2Q9, 8, 8, 1, 5, s5.data(), tbad);
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EINVAL);
    bad = config(NFLBM_D2Q9, 8, 8, 1, 5, s5.data(), tau5);
    bad.implicit_comp = 5;
    CHECK(nflbm_device_bytes(&bad, &bytes) == NFLBM_EINVAL);
    CHECK(nflbm_device_bytes(nullptr, &bytes) == NFLBM_EINVAL);
  }

  // creation: invalid configurations fail before the device; a valid one
  // either runs (a GPU is present) or fails cleanly without one
  {
    nflbm_sim* sim = nullptr;
    nflbm_config bad = config(NFLBM_D2Q9, 8, 8, 1, 9, s5.data(), tau5);
    CHECK(nflbm_create(&bad, &sim) == NFLBM_EINVAL && sim == nullptr);
    nflbm_config c = config(NFLBM_D2Q9, 24, 20, 1, 5, s5.data(), tau5);
    const int rc = nflbm_create(&c, &sim);
    if (rc == NFLBM_OK) {
      CHECK(nflbm_step(sim, 4) == NFLBM_OK);
      CHECK(nflbm_synchronize(sim) == NFLBM_OK);
      nflbm_diag d;
      CHECK(nflbm_diagnostics(sim, 0, &d) == NFLBM_OK);
      CHECK(nflbm_set_nan_check(sim, -1) == NFLBM_EINVAL);
      nflbm_destroy(sim);
    } else {
      CHECK(sim == nullptr);
      CHECK(std::strlen(nflbm_last_error(nullptr)) > 0);
    }
  }

  // batches: members must agree; the check runs before any member exists
  {
    const std::vector<double> s3 = tensions(3, 3u);
    const double tau3[3] = {1.0, 1.0, 1.0};
    nflbm_config cs[2] = {config(NFLBM_D2Q9, 16, 16, 1, 3, s3.data(), tau3),
                          config(NFLBM_D2Q9, 16, 16, 1, 5, s5.data(), tau5)};
    nflbm_batch* b = nullptr;
    CHECK(nflbm_batch_create(cs, 2, &b) == NFLBM_EINVAL && b == nullptr);
    CHECK(nflbm_batch_create(cs, 0, &b) == NFLBM_EINVAL);
    CHECK(nflbm_batch_count(nullptr) == 0);
    CHECK(nflbm_batch_member(nullptr, 0) == nullptr);
    CHECK(std::strlen(nflbm_batch_last_error(nullptr)) > 0);
    nflbm_batch_destroy(nullptr);
  }

  // NULL handles are rejected, never dereferenced
  nflbm_destroy(nullptr);
  CHECK(nflbm_step(nullptr, 1) == NFLBM_EINVAL);
  CHECK(nflbm_synchronize(nullptr) == NFLBM_EINVAL);
  CHECK(nflbm_set_nan_check(nullptr, 4) == NFLBM_EINVAL);
  CHECK(nflbm_set_fields(nullptr, nullptr, nullptr, nullptr) == NFLBM_EINVAL);
  CHECK(nflbm_get_field(nullptr, 0, nullptr) == NFLBM_EINVAL);
  CHECK(nflbm_diagnostics(nullptr, 0, nullptr) == NFLBM_EINVAL);
  CHECK(nflbm_set_stream(nullptr, nullptr) == NFLBM_EINVAL);
  CHECK(nflbm_batch_step(nullptr, 1, 0) == NFLBM_EINVAL);
  CHECK(nflbm_storage_form(nullptr) == NFLBM_EINVAL);

  if (failures) std::fprintf(stderr, "%d checks failed\n", failures);
  else std::printf("host paths: all checks passed\n");
  return failures ? 1 : 0;
}
