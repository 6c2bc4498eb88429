// Host-only checks of libfftpl's C-ABI host code under AddressSanitizer and
// UndefinedBehaviorSanitizer (the host part of the library is built with
// them; no device work is enqueued): the dark-node decomposition of
// irregular regions on random and malformed rectangles, the argument checks
// that return before any launch, the problem path decision, and the net
// block packing of the exchange index build.  Prints "OK" and exits 0 when
// every check holds; the sanitizers abort on the first memory or UB error.
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <random>
#include <vector>

#include "../../include/fftpl.h"

namespace fftpl {
int pack_net_blocks(const int32_t* ptr, int E, int P, int max_degree, int cap, int nnb,
                    int32_t* first);
}

static int failures = 0;
#define CHECK(c)                                                      \
  do {                                                                \
    if (!(c)) {                                                       \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

// Area of the union of axis-aligned boxes by a fine grid count (brute force).
static double union_area_grid(const std::vector<double>& r, int k, double xl, double yl,
                              double xh, double yh, int res) {
  double a = 0.0;
  const double dx = (xh - xl) / res, dy = (yh - yl) / res;
  for (int i = 0; i < res; ++i)
    for (int j = 0; j < res; ++j) {
      const double x = xl + (i + 0.5) * dx, y = yl + (j + 0.5) * dy;
      for (int q = 0; q < k; ++q)
        if (x >= r[4 * q] && x < r[4 * q + 2] && y >= r[4 * q + 1] && y < r[4 * q + 3]) {
          a += dx * dy;
          break;
        }
    }
  return a;
}

static void dark_nodes_checks() {
  std::mt19937 rng(7);
  std::uniform_real_distribution<double> u(0.0, 100.0);
  for (int trial = 0; trial < 300; ++trial) {
    const int k = trial % 9;
    std::vector<double> rects(4 * (size_t)k + 4);
    for (int q = 0; q < k; ++q) {
      double a = u(rng), b = u(rng), c = u(rng), d = u(rng);
      if (trial % 5 == 0) {   // rectangles reaching outside R, on its edges
        a -= 30.0;
        d += 30.0;
      }
      rects[4 * q] = fmin(a, b);
      rects[4 * q + 2] = fmax(a, b);
      rects[4 * q + 1] = fmin(c, d);
      rects[4 * q + 3] = fmax(c, d);
    }
    int32_t need = -1;
    // too small an output: the count needed comes back, nothing past max_out
    // is written (the sanitizer checks the bound of the one-element buffer)
    double one[4];
    const int st0 = fftpl_dark_nodes(0.0, 0.0, 100.0, 100.0, k, k ? rects.data() : nullptr, 1,
                                     one, &need);
    CHECK(need >= 0);
    CHECK(st0 == (need > 1 ? FFTPL_E_INVAL : FFTPL_OK));
    std::vector<double> out(4 * (size_t)(need > 0 ? need : 1));
    int32_t got = -1;
    CHECK(fftpl_dark_nodes(0.0, 0.0, 100.0, 100.0, k, k ? rects.data() : nullptr, need,
                           out.data(), &got) == FFTPL_OK);
    CHECK(got == need);
    // the pieces are disjoint, inside R, and cover R minus the placeable union
    double dark = 0.0;
    for (int i = 0; i < got; ++i) {
      const double* o = &out[4 * (size_t)i];
      CHECK(o[0] >= 0.0 && o[2] <= 100.0 && o[1] >= 0.0 && o[3] <= 100.0);
      CHECK(o[2] > o[0] && o[3] > o[1]);
      dark += (o[2] - o[0]) * (o[3] - o[1]);
      for (int j = 0; j < i; ++j) {
        const double* p = &out[4 * (size_t)j];
        const double ox = fmin(o[2], p[2]) - fmax(o[0], p[0]);
        const double oy = fmin(o[3], p[3]) - fmax(o[1], p[1]);
        CHECK(!(ox > 1e-12 && oy > 1e-12));
      }
    }
    std::vector<double> clip(rects.begin(), rects.end());
    const double place = union_area_grid(clip, k, 0.0, 0.0, 100.0, 100.0, 400);
    CHECK(fabs(dark + place - 10000.0) < 0.02 * 10000.0);
  }
  // malformed input: refused on the host
  int32_t n = 0;
  double bad[4] = {5.0, 5.0, 1.0, 9.0};   // x1 < x0
  double buf[16];
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, 1, bad, 4, buf, &n) == FFTPL_E_INVAL);
  double nanr[4] = {NAN, 0.0, 1.0, 1.0};
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, 1, nanr, 4, buf, &n) == FFTPL_E_INVAL);
  CHECK(fftpl_dark_nodes(0, 0, 0, 10, 0, nullptr, 4, buf, &n) == FFTPL_E_INVAL);
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, -1, nullptr, 4, buf, &n) == FFTPL_E_INVAL);
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, 2, nullptr, 4, buf, &n) == FFTPL_E_INVAL);
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, 0, nullptr, 4, nullptr, &n) == FFTPL_E_INVAL);
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, 0, nullptr, 0, nullptr, nullptr) == FFTPL_E_INVAL);
  CHECK(fftpl_dark_nodes(0, 0, 10, 10, 0, nullptr, 1, buf, &n) == FFTPL_OK && n == 1);
}

static void argument_checks() {
  fftpl_grid g = {64, 0, 0.0, 0.0, 1.0, 1.0, 1.0};
  void* p = reinterpret_cast<void*>(uintptr_t(1) << 20);
  const float* fp = static_cast<const float*>(p);
  const int32_t* ip = static_cast<const int32_t*>(p);
  fftpl_plan* plan = nullptr;
  CHECK(fftpl_plan_create(nullptr, 64, 0, 1, nullptr) == FFTPL_E_INVAL);
  CHECK(fftpl_plan_create(&plan, 64, 0, 0, nullptr) == FFTPL_E_INVAL);
  CHECK(fftpl_plan_create(&plan, 100, 0, 1, nullptr) == FFTPL_E_UNSUPPORTED);
  CHECK(plan == nullptr);
  CHECK(fftpl_density_map(&g, -1, fp, fp, fp, fp, nullptr, (float*)p, nullptr) ==
        FFTPL_E_INVAL);
  CHECK(fftpl_wa_grad(3, ip, 6, ip, fp, fp, 4, fp, fp, -1.0f, 0, (float*)p, (float*)p,
                      nullptr, nullptr, nullptr) == FFTPL_E_INVAL);
  CHECK(fftpl_eval(nullptr, nullptr, fp, fp, 1.0f, 1.0f, 0, nullptr, nullptr, nullptr,
                   nullptr) == FFTPL_E_INVAL);
  uint64_t ib = 0, wb = 0, work = 0;
  CHECK(fftpl_xindex_bytes(1000, 1100, 3300, 8, &ib, &wb) == FFTPL_OK && ib > 0 && wb > 0);
  CHECK(fftpl_xindex_bytes(1000, 1100, 3300, 9000, &ib, &wb) == FFTPL_E_UNSUPPORTED);
  CHECK(fftpl_problem_work_bytes(64, 1000, 1100, 3300, &work) == FFTPL_OK && work > 0);
  // the path decision, over fake addresses that are never dereferenced
  fftpl_problem pr;
  memset(&pr, 0, sizeof(pr));
  pr.grid = g;
  pr.num_cells = 1000;
  pr.num_nets = 1100;
  pr.num_pins = 3300;
  pr.w = pr.h = fp;
  pr.net_ptr = pr.pin_cell = ip;
  pr.pin_dx = pr.pin_dy = fp;
  pr.max_degree = 8;
  int32_t path = -1;
  CHECK(fftpl_problem_path(&pr, &path) == FFTPL_OK && path == FFTPL_PATH_ATOMIC);
  pr.work = reinterpret_cast<void*>(uintptr_t(1) << 30);
  pr.work_bytes = work;
  CHECK(fftpl_problem_path(&pr, &path) == FFTPL_E_INVAL);   // no index
  pr.xindex = reinterpret_cast<void*>(uintptr_t(1) << 31);
  pr.xindex_bytes = ib;
  pr.xindex_key = 99;
  CHECK(fftpl_problem_path(&pr, &path) == FFTPL_E_STATE);   // another netlist's index
  pr.grid.n = 2048;
  CHECK(fftpl_problem_path(&pr, &path) == FFTPL_E_UNSUPPORTED);
}

static void packing_checks() {
  std::mt19937 rng(11);
  for (int trial = 0; trial < 200; ++trial) {
    const int E = (int)(rng() % 400);
    const int maxd = 1 + (int)(rng() % 60);
    std::vector<int32_t> ptr((size_t)E + 1, 0);
    for (int e = 0; e < E; ++e) ptr[(size_t)e + 1] = ptr[e] + (int32_t)(rng() % (maxd + 1));
    const int P = ptr[E];
    const int cap = maxd + (int)(rng() % 200);
    const int nnb = P / (cap - maxd + 1) + 2;
    std::vector<int32_t> first((size_t)nnb + 1, -7);
    CHECK(fftpl::pack_net_blocks(ptr.data(), E, P, maxd, cap, nnb, first.data()) ==
          FFTPL_OK);
    // every block holds whole nets in order, at most cap pins, and is closed
    // only when the next net would not fit
    CHECK(first[0] == 0);
    for (int k = 0; k < nnb; ++k) {
      CHECK(first[k] <= first[(size_t)k + 1]);
      const int a = first[k], b = first[(size_t)k + 1];
      CHECK(ptr[b] - ptr[a] <= cap);
      if (b < E && a < b) CHECK(ptr[(size_t)b + 1] - ptr[a] > cap);
    }
    CHECK(first[nnb] == E);
  }
  // malformed CSRs: refused, nothing written past the output
  std::vector<int32_t> bad = {0, 3, 2, 5};   // decreasing
  std::vector<int32_t> out(3);
  CHECK(fftpl::pack_net_blocks(bad.data(), 3, 5, 8, 16, 2, out.data()) == FFTPL_E_INVAL);
  std::vector<int32_t> big = {0, 2, 40};     // a net above max_degree
  CHECK(fftpl::pack_net_blocks(big.data(), 2, 40, 8, 16, 2, out.data()) == FFTPL_E_INVAL);
  std::vector<int32_t> off = {1, 2, 3};      // does not start at 0
  CHECK(fftpl::pack_net_blocks(off.data(), 2, 3, 8, 16, 2, out.data()) == FFTPL_E_INVAL);
  std::vector<int32_t> many = {0, 8, 16, 24};  // needs three blocks of 8, two allowed
  CHECK(fftpl::pack_net_blocks(many.data(), 3, 24, 8, 8, 2, out.data()) == FFTPL_E_INVAL);
}

int main() {
  dark_nodes_checks();
  argument_checks();
  packing_checks();
  if (failures) {
    fprintf(stderr, "%d checks failed\n", failures);
    return 1;
  }
  printf("OK\n");
  return 0;
}
