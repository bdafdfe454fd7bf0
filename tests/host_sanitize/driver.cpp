// Host-side checks of the library under AddressSanitizer and
// UndefinedBehaviorSanitizer (built host-only; no GPU is touched): the
// observation layout builder and its invariant checker on many shapes, the
// rejection of invalid inputs and options, the footprint bound, and the
// seeded initial cameras.  Exit status 0 when every check holds.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "povar.h"
#include "povar_host.h"

static int failures = 0;
#define CHECK(cond, ...)                                  \
  do {                                                    \
    if (!(cond)) {                                        \
      std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
      std::fprintf(stderr, __VA_ARGS__);                  \
      std::fprintf(stderr, "\n");                         \
      ++failures;                                         \
    }                                                     \
  } while (0)

struct Obs {
  int32_t n_cams, n_pts;
  std::vector<int32_t> cam, pt;
  std::vector<double> meas;
};

// n_pts landmarks, each seen by `lo`..`hi` distinct cameras; zipf: camera
// choice weighted rank^-0.8; every camera gets at least one observation.
static Obs make_obs(int32_t n_cams, int32_t n_pts, int lo, int hi, bool zipf, unsigned seed) {
  std::mt19937_64 rng(seed);
  Obs o{n_cams, n_pts, {}, {}, {}};
  std::vector<double> w(n_cams);
  for (int32_t c = 0; c < n_cams; ++c) w[c] = zipf ? std::pow(c + 1.0, -0.8) : 1.0;
  std::discrete_distribution<int32_t> pick(w.begin(), w.end());
  std::uniform_int_distribution<int> len(lo, hi);
  std::uniform_real_distribution<double> u(-0.5, 0.5);
  for (int32_t j = 0; j < n_pts; ++j) {
    const int L = std::min<int>(len(rng), n_cams);
    std::vector<int32_t> seen;
    while ((int)seen.size() < L) {
      const int32_t c = pick(rng);
      bool dup = false;
      for (int32_t s : seen) dup = dup || s == c;
      if (!dup) seen.push_back(c);
    }
    for (int32_t c : seen) {
      o.cam.push_back(c);
      o.pt.push_back(j);
      o.meas.push_back(u(rng));
      o.meas.push_back(u(rng));
    }
  }
  for (int32_t c = 0; c < n_cams; ++c) {   // cameras nobody picked see landmark 0
    bool any = false;
    for (int32_t x : o.cam) any = any || x == c;
    if (!any) {
      o.cam.push_back(c);
      o.pt.push_back(0);
      o.meas.push_back(0.1);
      o.meas.push_back(-0.1);
    }
  }
  return o;
}

static void check_layouts() {
  struct Shape {
    int32_t n_cams, n_pts;
    int lo, hi;
    bool zipf;
  };
  const Shape shapes[] = {
      {1, 1, 1, 1, false},        {5, 64, 2, 5, false},        {30, 129, 1, 8, false},
      {100, 50, 60, 90, false},   {2, 20000, 2, 2, false},     {300, 140000, 2, 3, true},
      {40, 70000, 2, 4, false},   {1200, 40000, 2, 4, true},   {7, 3, 7, 7, false},
  };
  unsigned seed = 1;
  for (const Shape& sh : shapes)
    for (int32_t prec : {POVAR_PREC_FP64, POVAR_PREC_FP32_BULK}) {
      const Obs o = make_obs(sh.n_cams, sh.n_pts, sh.lo, sh.hi, sh.zipf, seed++);
      int64_t out[8] = {0};
      const povar_status st = povar_debug_layout_check(o.n_cams, o.n_pts, (int64_t)o.cam.size(), o.cam.data(),
                                                       o.pt.data(), o.meas.data(), prec, out);
      CHECK(st == POVAR_OK, "layout %d cams %d pts: %s", sh.n_cams, sh.n_pts, povar_last_error(nullptr));
      uint64_t fp = 0;
      CHECK(povar_problem_footprint(o.n_cams, o.n_pts, (int64_t)o.cam.size(), prec, &fp) == POVAR_OK, "footprint");
      CHECK((int64_t)fp >= out[6], "footprint %llu below the built layout's %lld bytes", (unsigned long long)fp,
            (long long)out[6]);
    }
}

static void check_invalid_inputs() {
  Obs o = make_obs(6, 100, 3, 5, false, 99);
  const int64_t n = (int64_t)o.cam.size();
  int64_t out[8];
  auto layout = [&](const Obs& x, int32_t prec = POVAR_PREC_FP64) {
    return povar_debug_layout_check(x.n_cams, x.n_pts, (int64_t)x.cam.size(), x.cam.data(), x.pt.data(),
                                    x.meas.data(), prec, out);
  };
  Obs bad = o;
  bad.cam[3] = o.n_cams;
  CHECK(layout(bad) == POVAR_EINVAL, "camera index out of range accepted");
  bad = o;
  bad.pt[5] = -1;
  CHECK(layout(bad) == POVAR_EINVAL, "negative point index accepted");
  bad = o;
  bad.meas[7] = std::nan("");
  CHECK(layout(bad) == POVAR_EINVAL, "NaN measurement accepted");
  bad = o;
  bad.meas[2] = INFINITY;
  CHECK(layout(bad) == POVAR_EINVAL, "infinite measurement accepted");
  bad = o;
  bad.n_cams += 1;   // a camera without observations
  CHECK(layout(bad) == POVAR_EINVAL, "camera without observations accepted");
  bad = o;
  bad.n_pts += 1;    // a point without observations
  CHECK(layout(bad) == POVAR_EINVAL, "point without observations accepted");
  CHECK(povar_debug_layout_check(0, 10, n, o.cam.data(), o.pt.data(), o.meas.data(), 0, out) == POVAR_EINVAL,
        "zero cameras accepted");
  CHECK(povar_debug_layout_check(o.n_cams, o.n_pts, n, nullptr, o.pt.data(), o.meas.data(), 0, out) ==
            POVAR_EINVAL, "NULL camera indices accepted");
  CHECK(layout(o, 7) == POVAR_EINVAL, "unknown precision accepted");
  uint64_t fp;
  CHECK(povar_problem_footprint(-1, 5, 10, 0, &fp) == POVAR_EINVAL, "negative size accepted");
}

static void check_options() {
  povar_options o;
  CHECK(povar_options_default(&o) == POVAR_OK, "defaults");
  CHECK(povar::check_options(nullptr, &o) == POVAR_OK, "defaults rejected: %s", povar_last_error(nullptr));
  auto reject = [&](void (*edit)(povar_options&), const char* what) {
    povar_options x;
    povar_options_default(&x);
    edit(x);
    CHECK(povar::check_options(nullptr, &x) == POVAR_EINVAL, "accepted: %s", what);
  };
  reject([](povar_options& x) { x.struct_size = 8; }, "struct_size");
  reject([](povar_options& x) { x.eta = 1.5; }, "eta 1.5");
  reject([](povar_options& x) { x.eta = std::nan(""); }, "eta NaN");
  reject([](povar_options& x) { x.series_order = -1; }, "order -1");
  reject([](povar_options& x) { x.lambda0 = 0.0; }, "lambda0 0");
  reject([](povar_options& x) { x.lambda_max = INFINITY; }, "lambda_max inf");
  reject([](povar_options& x) { x.precision = 9; }, "precision 9");
  reject([](povar_options& x) { x.manifold = -1; }, "manifold -1");
  reject([](povar_options& x) { x.series_rtol = 1.0; }, "series_rtol 1");
  CHECK(povar::check_options(nullptr, nullptr) == POVAR_EINVAL, "NULL options accepted");
}

static void check_seeded_cameras() {
  for (uint64_t seed : {0ull, 1ull, 12345ull, ~0ull}) {
    std::vector<double> c(37 * 12);
    povar::seeded_cameras(seed, 37, c.data());
    for (int i = 0; i < 37; ++i) {
      double n2 = 0.0;
      for (int k = 0; k < 12; ++k) n2 += c[i * 12 + k] * c[i * 12 + k];
      CHECK(std::fabs(n2 - 1.0) < 1e-14, "seeded camera %d of seed %llu not unit norm", i,
            (unsigned long long)seed);
    }
  }
}

int main() {
  check_layouts();
  check_invalid_inputs();
  check_options();
  check_seeded_cameras();
  std::printf("host checks: %d failure(s)\n", failures);
  return failures == 0 ? 0 : 1;
}
