// Host-side exercise of the C ABI for the address and undefined-behaviour sanitizer
// build (tests/test_host_sanitizers.py): argument checks of every entry point, and plan
// construction (tau-weight tables, FFT plans, filter responses, work lists, search size
// classes) for 2D Haar, general-wavelet and volume plans over many shapes and flags.
// Without a GPU every valid plan stops at its first device upload (VDAMP_ERR_HIP) after
// all of its host work; with one it completes and is described and destroyed.
// Usage: host_checks <filters.txt>, one orthonormal lowpass filter per line.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "vdamp.h"

static int g_fail = 0, g_checks = 0, g_planned = 0;

#define EXPECT(cond)                                                                  \
  do {                                                                                \
    ++g_checks;                                                                       \
    if (!(cond)) {                                                                    \
      std::fprintf(stderr, "FAIL line %d: %s [%s]\n", __LINE__, #cond, vdamp_last_error()); \
      ++g_fail;                                                                       \
    }                                                                                 \
  } while (0)

// A valid configuration: planned on a GPU, or stopped by the runtime without one.
static void finish(vdamp_status st, vdamp_plan_h h, const char* what) {
  if (st == VDAMP_OK) {
    size_t need = 0;
    EXPECT(vdamp_plan_describe(h, nullptr, 0, &need) == VDAMP_OK && need > 1);
    std::vector<char> buf(need);
    EXPECT(vdamp_plan_describe(h, buf.data(), buf.size(), nullptr) == VDAMP_OK);
    EXPECT(buf[need - 1] == '\0');
    char small[8];
    EXPECT(vdamp_plan_describe(h, small, sizeof small, nullptr) == VDAMP_OK && small[7] == '\0');
    EXPECT(vdamp_plan_destroy(h) == VDAMP_OK);
    ++g_planned;
  } else if (st != VDAMP_ERR_HIP || !std::strstr(vdamp_last_error(), "upload")) {
    // without a device the plan must have done all of its host work first
    std::fprintf(stderr, "FAIL %s: status %d [%s]\n", what, (int)st, vdamp_last_error());
    ++g_fail;
  }
  ++g_checks;
}

static vdamp_status plan2d(const std::vector<int32_t>& ny, const std::vector<int32_t>& nx, int levels,
                           uint32_t flags, vdamp_plan_h* h) {
  size_t ws = 0;
  *h = nullptr;
  return vdamp_plan(h, (int32_t)ny.size(), ny.data(), nx.data(), levels, VDAMP_WAVELET_HAAR, flags, &ws);
}

static void valid2d(const std::vector<int32_t>& ny, const std::vector<int32_t>& nx, int levels, uint32_t flags) {
  vdamp_plan_h h;
  finish(plan2d(ny, nx, levels, flags, &h), h, "2D plan");
}

static std::vector<std::vector<double>> read_filters(const char* path) {
  std::vector<std::vector<double>> out;
  std::ifstream f(path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream is(line);
    std::vector<double> h;
    double v;
    while (is >> v) h.push_back(v);
    if (!h.empty()) out.push_back(h);
  }
  return out;
}

int main(int argc, char** argv) {
  if (argc < 2) {
    std::fprintf(stderr, "usage: host_checks <filters.txt>\n");
    return 2;
  }
  // status strings
  for (int s = 0; s < 8; ++s) EXPECT(vdamp_status_string((vdamp_status)s)[0] != '\0');
  EXPECT(std::string(vdamp_status_string((vdamp_status)99)) == "unknown status");

  // null handles and pointers: every entry point returns VDAMP_ERR_ARG before any launch
  EXPECT(vdamp_plan_destroy(nullptr) == VDAMP_ERR_ARG);
  EXPECT(vdamp_plan_describe(nullptr, nullptr, 0, nullptr) == VDAMP_ERR_ARG);
  EXPECT(vdamp_solve(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, 1, nullptr, nullptr) ==
         VDAMP_ERR_ARG);
  EXPECT(vdamp_solve_resume(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                            nullptr, nullptr, 1, nullptr, nullptr, nullptr) == VDAMP_ERR_ARG);
  EXPECT(fista_solve(nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr, 1, nullptr, nullptr) == VDAMP_ERR_ARG);
  EXPECT(vdamp_state_export(nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
         VDAMP_ERR_ARG);
  EXPECT(vdamp_pass_times(nullptr, nullptr, nullptr, 0) == VDAMP_ERR_ARG);
  EXPECT(vdamp_cnn_destroy(nullptr) == VDAMP_ERR_ARG);
  EXPECT(vdamp_cnn_create(nullptr, 13) == VDAMP_ERR_ARG);
  int64_t cnt = 0;
  EXPECT(vdamp_cnn_param_count(nullptr, &cnt) == VDAMP_ERR_ARG);
  size_t wsb = 0;
  EXPECT(vdamp_cnn_workspace(nullptr, nullptr, 0, &wsb) == VDAMP_ERR_ARG);

  // plan argument errors (checked on the host before anything is allocated)
  {
    vdamp_plan_h h;
    size_t ws;
    const int32_t n64[2] = {64, 64}, n60[1] = {60}, n1024[1] = {1024}, n56[1] = {56}, n4[2] = {64, 4}, n48[1] = {48};
    EXPECT(vdamp_plan(&h, 0, n64, n64, 3, 0, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan(&h, 1, n64, n64, 0, 0, 0, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan(&h, 1, n64, n64, 5, 0, 0, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan(&h, 1, n60, n64, 3, 0, 0, &ws) == VDAMP_ERR_SHAPE);
    EXPECT(vdamp_plan(&h, 1, n64, n1024, 3, 0, 0, &ws) == VDAMP_ERR_SHAPE);
    EXPECT(vdamp_plan(&h, 1, n64, n56, 3, 0, 0, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan(&h, 2, n64, n4, 3, 0, 0, &ws) == VDAMP_ERR_SHAPE);
    EXPECT(vdamp_plan(&h, 1, n64, n64, 3, 1, 0, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan(&h, 1, n64, n64, 3, 0, 1u << 30, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan(&h, 1, n64, n48, 4, 0, 0, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan(nullptr, 1, n64, n64, 3, 0, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan(&h, 1, n64, n64, 3, 0, 0, nullptr) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan(&h, 1, nullptr, n64, 3, 0, 0, &ws) == VDAMP_ERR_ARG);
  }

  // 2D Haar plans: square, non-square and mixed batches, every level count, every flag
  const uint32_t all = VDAMP_FLAG_DETERMINISTIC | VDAMP_FLAG_USE_GRAPH | VDAMP_FLAG_CHECK_FINITE |
                       VDAMP_FLAG_TIMING | VDAMP_FLAG_SURE_CONTINUOUS;
  const int32_t sizes[] = {16, 32, 48, 64, 80, 96, 128, 160, 192, 240, 256, 320, 384, 480, 512};
  for (int32_t n : sizes)
    for (int s = 1; s <= 4; ++s)
      if (n % (1 << s) == 0 && (n >> s) % 2 == 0) {
        valid2d({n}, {n}, s, 0);
        valid2d({n, n}, {n, n}, s, all);
        valid2d({n}, {n}, s, VDAMP_FLAG_GROUP_PAIRS | VDAMP_FLAG_SURE_CONTINUOUS);
      }
  valid2d({96}, {320}, 4, 0);
  valid2d({320}, {96}, 4, VDAMP_FLAG_GROUP_PAIRS);
  valid2d({128}, {256}, 4, 0);
  valid2d({128, 192, 256, 320, 128, 192, 256, 320}, {128, 192, 256, 320, 320, 256, 192, 128}, 4, all);
  valid2d({512, 256, 64}, {512, 256, 64}, 4, VDAMP_FLAG_GROUP_PAIRS);
  {
    std::vector<int32_t> big(300, 256);
    valid2d(big, big, 4, 0);
  }

  // general orthonormal wavelets: every filter of the file at several shapes, then the
  // filter checks
  const auto filters = read_filters(argv[1]);
  EXPECT(filters.size() >= 2);
  for (const auto& hf : filters)
    for (int32_t n : {32, 64, 128, 192, 256})
      for (int s = 1; s <= 4; ++s) {
        if (n % (1 << s) || (n >> s) % 2) continue;
        vdamp_plan_h h = nullptr;
        size_t ws = 0;
        const int32_t nn[2] = {n, n};
        finish(vdamp_plan_ortho(&h, 2, nn, nn, s, hf.data(), (int32_t)hf.size(), VDAMP_FLAG_SURE_CONTINUOUS, &ws),
               h, "ortho plan");
      }
  {
    vdamp_plan_h h;
    size_t ws;
    const int32_t n64[1] = {64};
    const double r2 = 1.0 / std::sqrt(2.0);
    const double haar[2] = {r2, r2}, notsum[2] = {1.0, 1.0}, notorth[4] = {0.5, 0.5, 0.5, 0.5};
    const double nanf[2] = {NAN, 1.0};
    std::vector<double> longf(66, 0.0);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, nullptr, 2, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, haar, 1, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, haar, 0, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, longf.data(), 66, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, notsum, 2, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, notorth, 4, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, nanf, 2, 0, &ws) == VDAMP_ERR_ARG);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, haar, 2, VDAMP_FLAG_AUTOTUNE, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan_ortho(&h, 1, n64, n64, 3, haar, 2, VDAMP_FLAG_GROUP_PAIRS, &ws) == VDAMP_ERR_UNSUPPORTED);
  }

  // volumes
  {
    struct V3 { int32_t nz, ny, nx; int s; };
    const V3 vols[] = {{16, 16, 16, 1}, {16, 32, 48, 2}, {32, 32, 32, 2}, {48, 48, 48, 3},
                       {64, 64, 64, 3}, {32, 64, 128, 3}, {64, 32, 16, 4}, {80, 80, 80, 4}};
    for (const V3& v : vols) {
      vdamp_plan_h h = nullptr;
      size_t ws = 0;
      const int32_t z[2] = {v.nz, v.nz}, y[2] = {v.ny, v.ny}, x[2] = {v.nx, v.nx};
      finish(vdamp_plan_3d(&h, 2, z, y, x, v.s, VDAMP_FLAG_SURE_CONTINUOUS, &ws), h, "3D plan");
    }
    vdamp_plan_h h;
    size_t ws;
    const int32_t a32[1] = {32}, a24[1] = {24}, a128[1] = {128};
    EXPECT(vdamp_plan_3d(&h, 1, a32, a32, a24, 2, 0, &ws) != VDAMP_OK);          // nx not a multiple of 16
    EXPECT(vdamp_plan_3d(&h, 1, a128, a128, a128, 3, 0, &ws) != VDAMP_OK);       // finest band > 65536
    EXPECT(vdamp_plan_3d(&h, 1, a32, a32, a32, 2, VDAMP_FLAG_AUTOTUNE, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan_3d(&h, 1, a32, a32, a32, 2, VDAMP_FLAG_GROUP_PAIRS, &ws) == VDAMP_ERR_UNSUPPORTED);
    EXPECT(vdamp_plan_3d(&h, 0, a32, a32, a32, 2, 0, &ws) == VDAMP_ERR_ARG);
  }

  std::printf("host checks: %d checks, %d failures, %d plans completed on a device\n", g_checks, g_fail,
              g_planned);
  return g_fail ? 1 : 0;
}
