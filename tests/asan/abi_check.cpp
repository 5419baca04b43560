// Host memory-safety check of the library's host-only code (test infrastructure): the
// native scheduler's decision functions (Eq. blockcondition, Algorithm 1, Algorithm 3)
// on random and extreme inputs, and the argument checks of the C entry points that
// return before any device work (null context, invalid sizes and arguments).  Built with
// AddressSanitizer and UBSan on the host side; the exit status is 0 when every result
// has the properties stated by include/tsbts.h.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <limits>
#include <vector>

#include "../../include/tsbts.h"

namespace {

uint64_t rng_state = 0x2545F4914F6CDD1Dull;
double uniform() {  // xorshift64*, in [0, 1)
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return static_cast<double>((rng_state * 2685821657736338717ull) >> 11) *
         (1.0 / 9007199254740992.0);
}
bool pow2(int64_t x) { return x > 0 && (x & (x - 1)) == 0; }

int failures = 0;
void expect(bool ok, const char *what) {
  if (!ok) {
    std::printf("failed: %s\n", what);
    ++failures;
  }
}

}  // namespace

int main() {
  const double inf = std::numeric_limits<double>::infinity();
  const double nan = std::numeric_limits<double>::quiet_NaN();
  const int64_t DMIN = 1, DMAX = int64_t(1) << 14;
  // Eq. blockcondition: a power of two within the bounds, for any criterion values
  const double extremes[] = {0.0, -1.0, 1e-300, 1e300, inf, nan, 2.0 - 1e-16, 1.0};
  for (double b : extremes)
    for (double e : extremes) {
      int64_t out = -1;
      expect(tsbts_sched_admissible(b, e, DMIN, DMAX, &out) == TSBTS_OK, "admissible status");
      expect(pow2(out) && out >= DMIN && out <= DMAX, "admissible range");
    }
  expect(tsbts_sched_admissible(1.0, 1.0, 0, DMAX, nullptr) == TSBTS_EINVAL, "null out");
  expect(tsbts_sched_admissible(1.0, 1.0, 4, 2, nullptr) == TSBTS_EINVAL, "bounds");
  // step rules: the new step is dt/2, dt or 2 dt within the bounds
  for (int trial = 0; trial < 20000; ++trial) {
    const int64_t dt = DMAX >> static_cast<int>(uniform() * 15);
    const int64_t tb = dt * static_cast<int64_t>(1 + uniform() * 64);
    const double scale = static_cast<double>(dt) * std::ldexp(1.0, -20);
    const double b = scale * std::ldexp(1.0, static_cast<int>(uniform() * 8) - 4);
    const double e1 = trial % 7 == 0 ? nan : scale * std::ldexp(1.0, static_cast<int>(uniform() * 8) - 4);
    const double e2 = trial % 11 == 0 ? inf : scale * std::ldexp(1.0, static_cast<int>(uniform() * 8) - 4);
    int64_t out = -1;
    const int first = trial % 3 == 0;
    expect(tsbts_sched_rule(first, dt, tb, b, e1, e2, DMIN, DMAX, &out) == TSBTS_OK, "rule status");
    const bool step_ok = first ? (pow2(out) && out <= 2 * dt && out >= DMIN && out <= DMAX)
                               : (out == dt / 2 || out == dt || out == 2 * dt || out == DMIN);
    expect(step_ok && out <= DMAX && out >= DMIN, "rule result");
  }
  int64_t dummy = 0;
  expect(tsbts_sched_rule(0, 3 * 64, 64, 1, 1, 1, DMIN, DMAX, &dummy) == TSBTS_EINVAL,
         "rule: time not a multiple of the step");
  // Algorithm 3 on random era-start tables: the era ends after t0, at a multiple of a
  // power of two between dt_max/8 and dt_max
  for (int trial = 0; trial < 2000; ++trial) {
    const int64_t n = 1 + static_cast<int64_t>(uniform() * 50);
    const int64_t t0 = (DMAX >> 5) * static_cast<int64_t>(uniform() * 128);
    std::vector<int64_t> t(n), dt(n);
    for (int64_t i = 0; i < n; ++i) {
      dt[i] = DMAX >> static_cast<int>(uniform() * 12);
      t[i] = t0 / dt[i] * dt[i];
    }
    int64_t end = -1;
    expect(tsbts_sched_era_end(t0, t.data(), dt.data(), n, DMAX, 0, &end) == TSBTS_OK,
           "era end status");
    const int64_t size = end - t0;
    expect(end > t0 && size <= DMAX, "era end after t0, at most dt_max later");
    int64_t p = DMAX / 8;
    bool aligned = false;
    for (; p <= DMAX; p *= 2) aligned |= (end % p == 0 && end - p < t0 + p);
    expect(aligned, "era end on a multiple of its size");
    expect(tsbts_sched_era_end(t0, t.data(), dt.data(), n, DMAX, 2 * DMAX, &end) == TSBTS_OK &&
               end == t0 + 2 * DMAX, "fixed era");
    dt[0] = 3;  // not a power of two
    expect(tsbts_sched_era_end(t0, t.data(), dt.data(), n, DMAX, 0, &end) == TSBTS_EINVAL,
           "era end refuses a bad table");
  }
  expect(tsbts_sched_era_end(0, nullptr, nullptr, 1, DMAX, 0, &dummy) == TSBTS_EINVAL,
         "era end null tables");
  // argument checks that return before any device work
  tsbts_ctx *ctx = nullptr;
  expect(tsbts_create(nullptr, 10, 0.1, TSBTS_MIXED, 0) == TSBTS_EINVAL, "create null out");
  expect(tsbts_create(&ctx, 0, 0.1, TSBTS_MIXED, 0) == TSBTS_EINVAL && !ctx, "create n = 0");
  expect(tsbts_create(&ctx, 10, -1.0, TSBTS_MIXED, 0) == TSBTS_EINVAL && !ctx, "create eps < 0");
  expect(tsbts_create(&ctx, 10, nan, TSBTS_MIXED, 0) == TSBTS_EINVAL && !ctx, "create eps nan");
  expect(tsbts_create(&ctx, 10, 0.1, 7, 0) == TSBTS_EINVAL && !ctx, "create precision");
  expect(tsbts_create(&ctx, 10, 0.1, TSBTS_MIXED, 64) == TSBTS_EINVAL && !ctx, "create flags");
  expect(tsbts_predict(nullptr, 0.0, 0, nullptr) == TSBTS_EINVAL, "predict null ctx");
  expect(tsbts_force(nullptr, nullptr, 1, 0.0, nullptr, nullptr, nullptr) == TSBTS_EINVAL,
         "force null ctx");
  expect(tsbts_force_noalloc(nullptr, nullptr, 1, 0.0, nullptr, nullptr, nullptr) ==
             TSBTS_EINVAL, "noalloc null ctx");
  expect(tsbts_force_backward(nullptr, nullptr, 1, 0.0, nullptr, nullptr, nullptr, nullptr,
                              nullptr) == TSBTS_EINVAL, "backward null ctx");
  expect(tsbts_timestep(nullptr, nullptr, 1, 0.1, nullptr, nullptr) == TSBTS_EINVAL,
         "timestep null ctx");
  expect(tsbts_correct(nullptr, nullptr, 1, 0.0, nullptr, nullptr) == TSBTS_EINVAL,
         "correct null ctx");
  expect(tsbts_energy(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == TSBTS_EINVAL,
         "energy null ctx");
  expect(tsbts_sched_era(nullptr, nullptr, nullptr) == TSBTS_EINVAL, "era null ctx");
  expect(tsbts_sched_state(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
             TSBTS_EINVAL, "state null ctx");
  expect(tsbts_destroy(nullptr) == TSBTS_OK, "destroy null");
  for (int st = -6; st <= 1; ++st) expect(tsbts_strerror(st) != nullptr, "strerror");
  expect(tsbts_last_error(nullptr) != nullptr, "last_error null");
  if (failures) return 1;
  std::printf("host rule and argument check ok\n");
  return 0;
}
