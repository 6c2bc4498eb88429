// extern "C" entry points of libfftpl: host-side argument validation, plan
// lifecycle and the launch sequences of the hot path.  Argument meaning,
// layout, ownership and error behaviour are specified in include/fftpl.h.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <vector>

#include "fftpl_internal.hpp"

using namespace fftpl;

struct fftpl_plan {
  Plan p;
};


// A profiler range around each entry point that enqueues device work: built
// with FFTPL_ROCTX (and linked against the roctx library) every call appears
// by name in a rocprofv3 --marker-trace; otherwise this compiles to nothing.
#ifdef FFTPL_ROCTX
#include <rocprofiler-sdk-roctx/roctx.h>
namespace {
struct RoctxRange {
  explicit RoctxRange(const char* name) { roctxRangePush(name); }
  ~RoctxRange() { roctxRangePop(); }
};
}  // namespace
#define FFTPL_RANGE() RoctxRange fftpl_roctx_range_(__func__)
#else
#define FFTPL_RANGE() ((void)0)
#endif

namespace {

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int dev_status(hipError_t e) { return e == hipSuccess ? FFTPL_OK : FFTPL_E_DEVICE; }

bool validate_env() {
  const char* v = getenv("FFTPL_VALIDATE");
  return v && v[0] == '1';
}

bool grid_ok(const fftpl_grid* g) {
  return g && g->n >= 1 && g->n <= 65536 && g->reserved == 0 && isfinite(g->xl) &&
         isfinite(g->yl) && isfinite(g->bin_w) && isfinite(g->bin_h) && g->bin_w > 0 &&
         g->bin_h > 0 && isfinite(g->target_density) && g->target_density >= 0;
}

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

template <typename T>
std::vector<T> to_host(const T* d, size_t count) {
  std::vector<T> h(count);
  if (count) hipMemcpy(h.data(), d, count * sizeof(T), hipMemcpyDeviceToHost);
  return h;
}

// O(pins) content checks, only under FFTPL_VALIDATE=1 (synchronous).
int validate_netlist(int num_nets, const int32_t* net_ptr, int num_pins,
                     const int32_t* pin_cell, int num_cells) {
  if (hipDeviceSynchronize() != hipSuccess) return FFTPL_E_DEVICE;
  auto ptr = to_host(net_ptr, (size_t)num_nets + 1);
  if (ptr[0] != 0 || ptr[num_nets] != num_pins) return FFTPL_E_INVAL;
  for (int e = 0; e < num_nets; ++e)
    if (ptr[e + 1] < ptr[e]) return FFTPL_E_INVAL;
  auto pc = to_host(pin_cell, (size_t)num_pins);
  for (int p = 0; p < num_pins; ++p)
    if (pc[p] < 0 || pc[p] >= num_cells) return FFTPL_E_INVAL;
  return FFTPL_OK;
}

int validate_cells(int m, const float* x, const float* y, const float* w, const float* h) {
  if (hipDeviceSynchronize() != hipSuccess) return FFTPL_E_DEVICE;
  auto hx = to_host(x, m), hy = to_host(y, m), hw = to_host(w, m), hh = to_host(h, m);
  for (int i = 0; i < m; ++i)
    if (!isfinite(hx[i]) || !isfinite(hy[i]) || !(hw[i] > 0) || !(hh[i] > 0) ||
        !isfinite(hw[i]) || !isfinite(hh[i]))
      return FFTPL_E_INVAL;
  return FFTPL_OK;
}

// Sizes the per-block partial sums of the solve (see Plan::partials) and
// returns the number of doubles to allocate for one batch slot.
size_t plan_partials(Plan& p, int n, int mode) {
  if (mode == FFTPL_DCT_FFT) {
    p.n_en = n / 2;
    p.n_tau = n / 2;
  } else {
    p.n_en = 2 * (n / 64) * (n / 64);
    p.n_tau = n;
  }
  p.en_max = p.n_en;
  return (size_t)p.en_max + 2 * (size_t)p.n_tau + 2;
}

// Host-side fingerprint of an exchange index: the sizes and arrays it was
// built from and the buffer it lives in (FNV-1a over their bytes; never 0).
uint64_t xindex_fingerprint(int m, int E, int P, int max_degree, const void* net_ptr,
                            const void* pin_cell, const void* index) {
  uint64_t h = 1469598103934665603ull;
  auto mix = [&h](uint64_t v) {
    for (int i = 0; i < 8; ++i) {
      h ^= (v >> (8 * i)) & 0xffu;
      h *= 1099511628211ull;
    }
  };
  mix((uint64_t)(uint32_t)m);
  mix((uint64_t)(uint32_t)E);
  mix((uint64_t)(uint32_t)P);
  mix((uint64_t)(uint32_t)max_degree);
  mix((uint64_t)(uintptr_t)net_ptr);
  mix((uint64_t)(uintptr_t)pin_cell);
  mix((uint64_t)(uintptr_t)index);
  return h ? h : 1;
}

void free_plan(Plan& p) {
  hipFree(p.fft_tw);
  hipFree(p.dct_cs);
  hipFree(p.wfreq);
  hipFree(p.rho);
  hipFree(p.tmp0);
  hipFree(p.tmp1);
  hipFree(p.tmp2);
  hipFree(p.psi);
  hipFree(p.exy);
  hipFree(p.rowsum);
  hipFree(p.partials);
  for (int i = 0; i < Plan::kMaxEvents; ++i)
    if (p.ev[i]) hipEventDestroy(p.ev[i]);
  if (p.fork) hipEventDestroy(p.fork);
  if (p.join) hipEventDestroy(p.join);
  if (p.side) hipStreamDestroy(p.side);
  gemm_plan_free(p);
}

}  // namespace

extern "C" {

int fftpl_version(void) { return FFTPL_VERSION; }

const char* fftpl_status_string(int status) {
  switch (status) {
    case FFTPL_OK: return "FFTPL_OK: success";
    case FFTPL_E_INVAL: return "FFTPL_E_INVAL: invalid argument";
    case FFTPL_E_NOMEM: return "FFTPL_E_NOMEM: device allocation failed";
    case FFTPL_E_DEVICE: return "FFTPL_E_DEVICE: HIP runtime or kernel launch error";
    case FFTPL_E_UNSUPPORTED: return "FFTPL_E_UNSUPPORTED: unsupported size or mode";
    case FFTPL_E_STATE: return "FFTPL_E_STATE: plan does not match the grid";
    default: return "unknown fftpl status";
  }
}

int fftpl_plan_create(fftpl_plan** out, int32_t n, int32_t dct_mode, int32_t max_batch,
                      void* stream) {
  if (!out) return FFTPL_E_INVAL;
  *out = nullptr;
  if (dct_mode < FFTPL_DCT_FFT || dct_mode > FFTPL_DCT_GEMM_BF16X3) return FFTPL_E_INVAL;
  if (max_batch < 1 || max_batch > FFTPL_MAX_BATCH) return FFTPL_E_INVAL;
  if (dct_mode == FFTPL_DCT_FFT) {
    if (!is_pow2(n) || n < 8 || n > 1024) return FFTPL_E_UNSUPPORTED;
  } else {
    if (n < 64 || n > 4096 || n % 64) return FFTPL_E_UNSUPPORTED;
  }
  fftpl_plan* pl = new (std::nothrow) fftpl_plan();
  if (!pl) return FFTPL_E_NOMEM;
  Plan& p = pl->p;
  p.n = n;
  p.mode = dct_mode;
  p.max_batch = max_batch;
  hipGetDevice(&p.device);
  const size_t nn = (size_t)n * n, B = (size_t)max_batch;
  p.part_stride = plan_partials(p, n, dct_mode);
  bool ok = hipMalloc(&p.fft_tw, sizeof(float2) * n) == hipSuccess &&
            hipMalloc(&p.dct_cs, sizeof(float2) * (n / 2 + 1)) == hipSuccess &&
            hipMalloc(&p.wfreq, sizeof(float) * n) == hipSuccess &&
            hipMalloc(&p.rho, sizeof(float) * nn * B) == hipSuccess &&
            hipMalloc(&p.tmp0, sizeof(float) * nn * B) == hipSuccess &&
            hipMalloc(&p.tmp1, sizeof(float) * nn * B) == hipSuccess &&
            hipMalloc(&p.tmp2, sizeof(float) * nn * B) == hipSuccess &&
            hipMalloc(&p.psi, sizeof(float) * nn * B) == hipSuccess &&
            hipMalloc(&p.exy, sizeof(float) * 2 * nn * B) == hipSuccess &&
            hipMalloc(&p.rowsum, sizeof(double) * n * B) == hipSuccess &&
            hipMalloc(&p.partials, sizeof(double) * p.part_stride * B) == hipSuccess;
  ok = ok && hipStreamCreateWithFlags(&p.side, hipStreamNonBlocking) == hipSuccess &&
       hipEventCreateWithFlags(&p.fork, hipEventDisableTiming) == hipSuccess &&
       hipEventCreateWithFlags(&p.join, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    hipGetLastError();
    free_plan(p);
    delete pl;
    return FFTPL_E_NOMEM;
  }
  std::vector<float2> tw(n), cs(n / 2 + 1);
  std::vector<float> wf(n);
  const double pi = 3.14159265358979323846;
  for (int t = 0; t < n; ++t) {
    tw[t] = make_float2((float)cos(2.0 * pi * t / n), (float)(-sin(2.0 * pi * t / n)));
    wf[t] = (float)(pi * t / n);
  }
  for (int k = 0; k <= n / 2; ++k)
    cs[k] = make_float2((float)cos(pi * k / (2.0 * n)), (float)sin(pi * k / (2.0 * n)));
  hipStream_t s = as_stream(stream);
  hipError_t e = hipMemcpyAsync(p.fft_tw, tw.data(), sizeof(float2) * n,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p.dct_cs, cs.data(), sizeof(float2) * (n / 2 + 1),
                       hipMemcpyHostToDevice, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(p.wfreq, wf.data(), sizeof(float) * n, hipMemcpyHostToDevice, s);
  int st = FFTPL_OK;
  if (e == hipSuccess && dct_mode != FFTPL_DCT_FFT) st = gemm_plan_init(p, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess || st != FFTPL_OK) {
    free_plan(p);
    delete pl;
    return st != FFTPL_OK ? st : FFTPL_E_DEVICE;
  }
  *out = pl;
  return FFTPL_OK;
}

int fftpl_plan_destroy(fftpl_plan* plan) {
  if (!plan) return FFTPL_OK;
  hipError_t e = hipDeviceSynchronize();
  free_plan(plan->p);
  delete plan;
  return dev_status(e);
}

int fftpl_plan_info(const fftpl_plan* plan, int32_t* n, int32_t* dct_mode,
                    int32_t* max_batch) {
  if (!plan) return FFTPL_E_INVAL;
  if (n) *n = plan->p.n;
  if (dct_mode) *dct_mode = plan->p.mode;
  if (max_batch) *max_batch = plan->p.max_batch;
  return FFTPL_OK;
}

int fftpl_plan_maps(const fftpl_plan* plan, const float** rho, const float** psi,
                    const float** exy) {
  if (!plan) return FFTPL_E_INVAL;
  if (rho) *rho = plan->p.rho;
  if (psi) *psi = plan->p.psi;
  if (exy) *exy = plan->p.exy;
  return FFTPL_OK;
}

int fftpl_fixed_map(const fftpl_grid* grid, int32_t num_fixed, const float* fx,
                    const float* fy, const float* fw, const float* fh, float* base,
                    float* cap, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(grid) || num_fixed < 0 || !base) return FFTPL_E_INVAL;
  if (num_fixed > 0 && (!fx || !fy || !fw || !fh)) return FFTPL_E_INVAL;
  return dev_status(launch_fixed_map(make_gridf(*grid), num_fixed, fx, fy, fw, fh, base,
                                     cap, as_stream(stream)));
}

int fftpl_dark_nodes(double xl, double yl, double xh, double yh, int32_t num_rects,
                     const double* rects, int32_t max_out, double* out, int32_t* num_out) {
  if (!num_out || num_rects < 0 || max_out < 0) return FFTPL_E_INVAL;
  if ((num_rects > 0 && !rects) || (max_out > 0 && !out)) return FFTPL_E_INVAL;
  if (!isfinite(xl) || !isfinite(yl) || !isfinite(xh) || !isfinite(yh) || !(xh > xl) ||
      !(yh > yl))
    return FFTPL_E_INVAL;
  struct Box {
    double x0, y0, x1, y1;
  };
  std::vector<Box> place;
  std::vector<double> ys = {yl, yh};
  for (int32_t i = 0; i < num_rects; ++i) {
    const double* r = rects + 4 * (size_t)i;
    for (int k = 0; k < 4; ++k)
      if (!isfinite(r[k])) return FFTPL_E_INVAL;
    if (r[2] < r[0] || r[3] < r[1]) return FFTPL_E_INVAL;
    const Box b{fmax(r[0], xl), fmax(r[1], yl), fmin(r[2], xh), fmin(r[3], yh)};
    if (b.x1 <= b.x0 || b.y1 <= b.y0) continue;   // empty inside R
    place.push_back(b);
    ys.push_back(b.y0);
    ys.push_back(b.y1);
  }
  std::sort(ys.begin(), ys.end());
  ys.erase(std::unique(ys.begin(), ys.end()), ys.end());
  // Horizontal slabs between consecutive y edges: in each, the placeable x
  // intervals are those of the rectangles spanning the whole slab; their
  // complement in [xl, xh] is dark.  A slab whose dark intervals equal the
  // previous slab's extends those rectangles upwards.
  std::vector<std::pair<double, double>> open, cur, iv;
  double open_y = yl;
  int64_t count = 0;
  auto emit = [&](double y1) {
    for (const auto& d : open) {
      if (count < max_out) {
        double* o = out + 4 * (size_t)count;
        o[0] = d.first;
        o[1] = open_y;
        o[2] = d.second;
        o[3] = y1;
      }
      ++count;
    }
  };
  for (size_t k = 0; k + 1 < ys.size(); ++k) {
    const double a = ys[k], b = ys[k + 1];
    iv.clear();
    for (const Box& r : place)
      if (r.y0 <= a && r.y1 >= b) iv.emplace_back(r.x0, r.x1);
    std::sort(iv.begin(), iv.end());
    cur.clear();
    double x = xl;   // left end of the part not yet known to be placeable
    for (const auto& q : iv) {
      if (q.first > x) cur.emplace_back(x, q.first);
      x = fmax(x, q.second);
    }
    if (x < xh) cur.emplace_back(x, xh);
    if (k > 0 && cur == open) continue;
    emit(a);
    open = cur;
    open_y = a;
  }
  emit(yh);
  if (count > INT32_MAX) return FFTPL_E_INVAL;
  *num_out = (int32_t)count;
  return count > max_out ? FFTPL_E_INVAL : FFTPL_OK;
}

int fftpl_density_map(const fftpl_grid* grid, int32_t num_cells, const float* x,
                      const float* y, const float* w, const float* h,
                      const float* base, float* rho, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(grid) || num_cells < 0 || !rho) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!x || !y || !w || !h)) return FFTPL_E_INVAL;
  if (validate_env() && num_cells > 0) {
    int v = validate_cells(num_cells, x, y, w, h);
    if (v != FFTPL_OK) return v;
  }
  const GridF g = make_gridf(*grid);
  hipStream_t s = as_stream(stream);
  if (grid->n <= kBandMaxN) {
    // the banded scatter of the evaluation, its band lists in a temporary
    // stream-ordered allocation released on the stream after the scatter
    size_t need = 0;
    band_layout_density(grid->n, num_cells, nullptr, &need);
    void* work = nullptr;
    if (hipMallocAsync(&work, need, s) != hipSuccess || !work) {
      (void)hipGetLastError();
      return FFTPL_E_NOMEM;
    }
    const BandLayout L = band_layout_density(grid->n, num_cells, work, nullptr);
    hipError_t e = launch_band_scatter(g, L, x, y, w, h, base, rho, s);
    const hipError_t f = hipFreeAsync(work, s);
    if (e == hipSuccess) e = f;
    return dev_status(e);
  }
  // grids past the band kernels' LDS rows: float atomics
  hipError_t e = launch_fill(rho, base, 0.0f, (int64_t)grid->n * grid->n, s);
  if (e == hipSuccess) e = launch_scatter(g, num_cells, x, y, w, h, rho, s);
  return dev_status(e);
}

int fftpl_density_map_noalloc(const fftpl_grid* grid, int32_t num_cells, const float* x,
                              const float* y, const float* w, const float* h,
                              const float* base, float* rho, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(grid) || num_cells < 0 || !rho) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!x || !y || !w || !h)) return FFTPL_E_INVAL;
  if (grid->n > kBandMaxN || num_cells > FFTPL_NOALLOC_MAX_CELLS) return FFTPL_E_UNSUPPORTED;
  size_t need = 0;
  band_layout_density(grid->n, num_cells, nullptr, &need);
  if (need > kNoallocScratchBytes) return FFTPL_E_UNSUPPORTED;
  if (validate_env() && num_cells > 0) {
    const int v = validate_cells(num_cells, x, y, w, h);
    if (v != FFTPL_OK) return v;
  }
  void* scr = nullptr;
  hipError_t e = noalloc_scratch(&scr);
  if (e != hipSuccess) return FFTPL_E_DEVICE;
  const BandLayout L = band_layout_density(grid->n, num_cells, scr, nullptr);
  return dev_status(launch_band_scatter(make_gridf(*grid), L, x, y, w, h, base, rho,
                                        as_stream(stream)));
}

int fftpl_helmholtz_solve(fftpl_plan* plan, const fftpl_grid* grid, float eps,
                          const float* rho, float* psi, float* ex, float* ey,
                          double* energy, void* stream) {
  FFTPL_RANGE();
  if (!plan || !grid_ok(grid) || !rho || !psi) return FFTPL_E_INVAL;
  if (!(eps >= 0.0f) || !isfinite(eps)) return FFTPL_E_INVAL;
  if ((ex == nullptr) != (ey == nullptr)) return FFTPL_E_INVAL;
  if (grid->n != plan->p.n) return FFTPL_E_STATE;
  hipStream_t s = as_stream(stream);
  SpectralArgs a;
  a.rho = rho;
  a.psi = psi;
  a.ex = ex;
  a.ey = ey;
  a.eps = eps;
  a.en_part = energy ? plan->p.partials : nullptr;
  hipError_t e = hipSuccess;
  plan->p.nev = 0;
  plan_mark(plan->p, "start", s);
  e = plan->p.mode == FFTPL_DCT_FFT ? spectral_fft(plan->p, a, s)
                                    : spectral_gemm(plan->p, a, s);
  if (e == hipSuccess && energy) {
    e = launch_eval_finalize(plan->p.partials, plan->p.n_en, nullptr, 0, nullptr, 0, 0, energy,
                             nullptr, nullptr, nullptr, s);
    plan_mark(plan->p, "k_eval_finalize", s);
  }
  return dev_status(e);
}

int fftpl_poisson_solve(fftpl_plan* plan, const fftpl_grid* grid, const float* rho,
                        float* psi, float* ex, float* ey, double* energy,
                        void* stream) {
  FFTPL_RANGE();
  return fftpl_helmholtz_solve(plan, grid, 0.0f, rho, psi, ex, ey, energy, stream);
}

int fftpl_field_gather(const fftpl_grid* grid, int32_t num_cells, const float* x,
                       const float* y, const float* w, const float* h,
                       const float* ex, const float* ey, const float* psi,
                       int32_t grad_mode, float scale, int32_t accumulate,
                       float* gx, float* gy, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(grid) || num_cells < 0 || !isfinite(scale)) return FFTPL_E_INVAL;
  if (grad_mode != FFTPL_GRAD_FIELD && grad_mode != FFTPL_GRAD_EXACT) return FFTPL_E_INVAL;
  if (accumulate != 0 && accumulate != 1) return FFTPL_E_INVAL;
  if (num_cells == 0) return FFTPL_OK;
  if (!x || !y || !w || !h || !gx || !gy) return FFTPL_E_INVAL;
  if (grad_mode == FFTPL_GRAD_FIELD && (!ex || !ey)) return FFTPL_E_INVAL;
  if (grad_mode == FFTPL_GRAD_EXACT && !psi) return FFTPL_E_INVAL;
  return dev_status(launch_gather(make_gridf(*grid), num_cells, x, y, w, h, ex, ey,
                                  nullptr, psi, grad_mode, scale, accumulate, gx, gy,
                                  as_stream(stream)));
}

static int wl_grad(int wl_model, int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                   const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                   int32_t num_cells, const float* x, const float* y, float gamma,
                   int32_t accumulate, float* gx, float* gy, double* wa, double* hpwl,
                   void* stream) {
  if (num_nets < 0 || num_pins < 0 || num_cells < 0) return FFTPL_E_INVAL;
  if (!(gamma > 0) || !isfinite(gamma)) return FFTPL_E_INVAL;
  if (accumulate != 0 && accumulate != 1) return FFTPL_E_INVAL;
  if (!net_ptr || (num_pins > 0 && (!pin_cell || !pin_dx || !pin_dy))) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!x || !y || !gx || !gy)) return FFTPL_E_INVAL;
  if (num_pins > 0 && num_cells == 0) return FFTPL_E_INVAL;
  if (validate_env()) {
    int v = validate_netlist(num_nets, net_ptr, num_pins, pin_cell, num_cells);
    if (v != FFTPL_OK) return v;
  }
  hipStream_t s = as_stream(stream);
  hipError_t e = hipSuccess;
  if (num_nets > 0 && num_pins > 0) {
    // fixed-point per-cell sums in a temporary stream-ordered workspace:
    // the same bits on every run
    void* work = nullptr;
    if (hipMallocAsync(&work, wa_fixed_work_bytes(num_cells, num_nets), s) != hipSuccess ||
        !work) {
      (void)hipGetLastError();
      return FFTPL_E_NOMEM;
    }
    e = launch_wa_fixed(num_nets, net_ptr, pin_cell, pin_dx, pin_dy, num_cells, x, y, gamma,
                        wl_model, accumulate, gx, gy, wa, hpwl, work, s);
    const hipError_t f = hipFreeAsync(work, s);
    if (e == hipSuccess) e = f;
    return dev_status(e);
  }
  // no pins: zero gradients (unless accumulating) and zero totals
  if (!accumulate && num_cells > 0) {
    e = launch_fill(gx, nullptr, 0.0f, num_cells, s);
    if (e == hipSuccess) e = launch_fill(gy, nullptr, 0.0f, num_cells, s);
  }
  if (e == hipSuccess && wa) e = launch_fill_f64(wa, 0.0, 1, s);
  if (e == hipSuccess && hpwl) e = launch_fill_f64(hpwl, 0.0, 1, s);
  return dev_status(e);
}

int fftpl_wa_grad(int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                  const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                  int32_t num_cells, const float* x, const float* y, float gamma,
                  int32_t accumulate, float* gx, float* gy, double* wa, double* hpwl,
                  void* stream) {
  FFTPL_RANGE();
  return wl_grad(FFTPL_WL_WA, num_nets, net_ptr, num_pins, pin_cell, pin_dx, pin_dy, num_cells,
                 x, y, gamma, accumulate, gx, gy, wa, hpwl, stream);
}

int fftpl_lse_grad(int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                   const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                   int32_t num_cells, const float* x, const float* y, float gamma,
                   int32_t accumulate, float* gx, float* gy, double* wa, double* hpwl,
                   void* stream) {
  FFTPL_RANGE();
  return wl_grad(FFTPL_WL_LSE, num_nets, net_ptr, num_pins, pin_cell, pin_dx, pin_dy,
                 num_cells, x, y, gamma, accumulate, gx, gy, wa, hpwl, stream);
}

}  // extern "C"

namespace {

// The path an evaluation of prob takes, after the host checks of its
// workspace and index fields (enum fftpl_path in *path), or their status.
int problem_path(const fftpl_problem* prob, int* path, XchDims* xd, size_t* need_out) {
  if (!prob || !grid_ok(&prob->grid)) return FFTPL_E_INVAL;
  const int m = prob->num_cells;
  if (m < 0 || prob->num_nets < 0 || prob->num_pins < 0) return FFTPL_E_INVAL;
  // the workspace and the index are read in 16-byte vectors: device
  // allocations are 256-byte aligned, and so must these be
  if ((reinterpret_cast<uintptr_t>(prob->work) & 255) != 0 ||
      (reinterpret_cast<uintptr_t>(prob->xindex) & 255) != 0)
    return FFTPL_E_INVAL;
  const bool any = prob->work || prob->xindex || prob->cell_ptr || prob->pin_slot;
  if (!any) {
    *path = FFTPL_PATH_ATOMIC;
    return FFTPL_OK;
  }
  // a workspace or an index was given: it is used, or the call fails
  if (prob->grid.n > kBandMaxN) return FFTPL_E_UNSUPPORTED;
  size_t need = 0;
  band_layout(prob->grid.n, m, prob->num_nets, prob->num_pins, nullptr, &need);
  if (need_out) *need_out = need;
  if (!prob->work || prob->work_bytes < need) return FFTPL_E_INVAL;
  if (prob->xindex) {
    XchDims d;
    const int st = xch_dims(m, prob->num_nets, prob->num_pins, prob->max_degree, &d);
    if (st != FFTPL_OK) return st;
    if (prob->xindex_bytes < d.index_bytes) return FFTPL_E_INVAL;
    if (prob->xindex_key != xindex_fingerprint(m, prob->num_nets, prob->num_pins,
                                               prob->max_degree, prob->net_ptr,
                                               prob->pin_cell, prob->xindex))
      return FFTPL_E_STATE;
    if (xd) *xd = d;
    *path = FFTPL_PATH_EXCHANGE;
    return FFTPL_OK;
  }
  if (prob->cell_ptr && prob->pin_slot) {
    *path = FFTPL_PATH_SLOTS;
    return FFTPL_OK;
  }
  return FFTPL_E_INVAL;   // a workspace without a pin index, or half an index
}

// Under FFTPL_VALIDATE=1: the index header read back against the problem.
int validate_index(const fftpl_problem* prob, const XchDims& xd) {
  int32_t hdr[9];
  if (hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(hdr, prob->xindex, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess)
    return FFTPL_E_DEVICE;
  if (hdr[1] != prob->num_cells || hdr[2] != prob->num_nets || hdr[3] != prob->num_pins ||
      hdr[4] != prob->max_degree || hdr[5] != xd.npt || hdr[8] != xd.cpb)
    return FFTPL_E_STATE;
  return FFTPL_OK;
}

// One checked evaluation request.
struct EvalReq {
  const fftpl_problem* prob = nullptr;
  const float *x = nullptr, *y = nullptr;
  float lambda = 0.0f, gamma = 1.0f;
  // if set, lambda and gamma are read on the device from params[0], params[1]
  const float* params = nullptr;
  float *gx = nullptr, *gy = nullptr;
  double* out4 = nullptr;
  int path = FFTPL_PATH_ATOMIC;
  GridF g;
  BandLayout L;
  XchDims xd;
  XchIndex X;
};

// Host-side checks of one evaluation (nothing is enqueued); fills r.
int check_eval(const Plan& p, const fftpl_problem* prob, const float* x, const float* y,
               float lambda, float gamma, int32_t grad_mode, float* gx, float* gy,
               double* out4, EvalReq* r) {
  if (!prob || !out4 || !grid_ok(&prob->grid)) return FFTPL_E_INVAL;
  if (prob->wl_model != FFTPL_WL_WA && prob->wl_model != FFTPL_WL_LSE) return FFTPL_E_INVAL;
  if (!(prob->screening >= 0.0f) || !isfinite(prob->screening)) return FFTPL_E_INVAL;
  if (prob->grid.n != p.n) return FFTPL_E_STATE;
  const int m = prob->num_cells;
  if (m < 0 || prob->num_nets < 0 || prob->num_pins < 0) return FFTPL_E_INVAL;
  if (grad_mode != FFTPL_GRAD_FIELD && grad_mode != FFTPL_GRAD_EXACT) return FFTPL_E_INVAL;
  if (!isfinite(lambda) || !(gamma > 0) || !isfinite(gamma)) return FFTPL_E_INVAL;
  // gx, gy both NULL: the scalars only (needs an atomic-free path, below)
  const bool grads = gx || gy;
  if (grads && (!gx || !gy)) return FFTPL_E_INVAL;
  if (m > 0 && (!x || !y || !prob->w || !prob->h)) return FFTPL_E_INVAL;
  if (!prob->net_ptr) return FFTPL_E_INVAL;
  if (prob->num_pins > 0 && (!prob->pin_cell || !prob->pin_dx || !prob->pin_dy || m == 0))
    return FFTPL_E_INVAL;
  int path = FFTPL_PATH_ATOMIC;
  XchDims xd;
  const int st = problem_path(prob, &path, &xd, nullptr);
  if (st != FFTPL_OK) return st;
  if (!grads && path == FFTPL_PATH_ATOMIC && m > 0) return FFTPL_E_INVAL;
  if (validate_env()) {
    int v = validate_netlist(prob->num_nets, prob->net_ptr, prob->num_pins, prob->pin_cell, m);
    if (v == FFTPL_OK && m > 0) v = validate_cells(m, x, y, prob->w, prob->h);
    if (v == FFTPL_OK && path == FFTPL_PATH_EXCHANGE) v = validate_index(prob, xd);
    if (v != FFTPL_OK) return v;
  }
  r->prob = prob;
  r->x = x;
  r->y = y;
  r->lambda = lambda;
  r->gamma = gamma;
  r->gx = gx;
  r->gy = gy;
  r->out4 = out4;
  r->path = path;
  r->g = make_gridf(prob->grid);
  r->L = band_layout(p.n, m, prob->num_nets, prob->num_pins,
                     path == FFTPL_PATH_ATOMIC ? nullptr : prob->work, nullptr);
  if (path == FFTPL_PATH_EXCHANGE) {
    r->xd = xd;
    r->X = xch_index(xd, prob->xindex);
  }
  return FFTPL_OK;
}

// The solve's arguments for a request in batch slot `slot` of the plan.
SpectralArgs spectral_args(Plan& p, const EvalReq& r, int slot, int grad_mode, bool grads) {
  const size_t nn = (size_t)p.n * p.n;
  SpectralArgs a;
  a.rho = p.rho + slot * nn;
  // FIELD: (Ex, Ey); EXACT: psi and the difference maps (Dx, Dy) the exact
  // gradient is summed from; scalars only: neither map
  a.psi = grads && grad_mode == FFTPL_GRAD_EXACT ? p.psi + slot * nn : nullptr;
  a.exy = grads ? p.exy + 2 * slot * nn : nullptr;
  a.diff = grad_mode == FFTPL_GRAD_EXACT;
  a.en_part = p.partials + slot * p.part_stride;
  a.base = r.prob->base;
  a.cap = r.prob->cap;
  a.rho_t = r.g.rho_t;
  a.tau_part = a.en_part + p.en_max;
  a.eps = r.prob->screening;
  return a;
}

// The exchange path for count requests (count <= the plan's max_batch, one
// wirelength model, workspaces that do not overlap): every stage is one
// launch over all of them, request i in batch slot i of the plan.  The
// wirelength branch (spread, net blocks) runs on the plan's side stream
// while the density branch (banded scatter, solve, band gather), the longer
// of the two when they share the chip, stays on `s`: the hand-over between
// streams costs several microseconds each way, and this way the fork delays
// only the shorter branch and the join is usually complete by the time the
// density branch reaches it.  With per-kernel timing on, everything runs on
// `s` so that consecutive events bracket single kernels.
int run_exchange_group(Plan& p, EvalReq* rs, int count, int grad_mode, hipStream_t s) {
  const bool grads = rs[0].gx != nullptr;
  const size_t nn = (size_t)p.n * p.n;
  const bool overlap = !p.timing;
  hipStream_t ds = s, ws = overlap ? p.side : s;
  hipError_t e = hipSuccess;
  p.nev = 0;
  plan_mark(p, "start", s);
  if (overlap) {
    e = hipEventRecord(p.fork, s);
    if (e == hipSuccess) e = hipStreamWaitEvent(ws, p.fork, 0);
  }
  BandReq br[kMaxBatch];
  XchReq xr[kMaxBatch];
  SpectralArgs sa[kMaxBatch];
  for (int i = 0; i < count; ++i) {
    const EvalReq& r = rs[i];
    br[i].g = r.g;
    br[i].L = r.L;
    br[i].x = r.x;
    br[i].y = r.y;
    br[i].w = r.prob->w;
    br[i].h = r.prob->h;
    br[i].base = r.prob->base;
    br[i].rho = p.rho + i * nn;
    br[i].exy = reinterpret_cast<const float2*>(p.exy + 2 * i * nn);
    br[i].psi = p.psi + i * nn;
    xr[i] = xch_req(r.xd, r.X, r.x, r.y, r.L.pin_grad, r.prob->net_ptr, r.prob->pin_dx,
                    r.prob->pin_dy, r.gamma, r.L.wa_part);
    if (r.params) xr[i].dgamma = r.params + 1;
    sa[i] = spectral_args(p, r, i, grad_mode, grads);
  }
  // density branch: banded scatter (its counters and the scalars are all
  // written, not accumulated, so nothing needs zeroing first)
  if (e == hipSuccess) e = launch_band_scatter_batch(br, count, ds, &p);
  // wirelength branch: pin positions into the exchange buffer, then every
  // net block (the per-cell sums follow the join)
  if (e == hipSuccess) e = launch_xch_spread_batch(xr, count, ws);
  plan_mark(p, "k_xch_spread", ws);
  if (e == hipSuccess) e = launch_xch_wa_batch(xr, count, rs[0].prob->wl_model, ws);
  plan_mark(p, "k_xch_wa", ws);
  // spectral solve (density branch); overflow sums in the first pass, energy
  // in the last
  if (e == hipSuccess) {
    if (p.mode == FFTPL_DCT_FFT) {
      e = spectral_fft_batch(p, sa, count, ds);
    } else {
      for (int i = 0; i < count && e == hipSuccess; ++i) e = spectral_gemm(p, sa[i], ds);
    }
  }
  // each cell's density gradient, computed band by band from the band
  // entries (L2-local reads of the field), still on the density branch
  if (grads) {
    if (e == hipSuccess) e = launch_band_gather_batch(br, count, grad_mode, ds);
    plan_mark(p, "k_band_gather", ds);
  }
  if (e == hipSuccess && overlap) {
    e = hipEventRecord(p.join, ws);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p.join, 0);
  }
  // per cell: lambda times the density gradient plus the sum of its pins'
  // gradients; the last cell block of each design also reduces its scalars
  // (N, W~, HPWL, tau from the per-block partials, complete by then)
  SumReq sr[kMaxBatch];
  bool fin_separate[kMaxBatch];
  for (int i = 0; i < count; ++i) {
    const EvalReq& r = rs[i];
    FinalArgs fin;
    fin.en = sa[i].en_part;
    fin.n_en = p.n_en;
    fin.tau = sa[i].tau_part;
    fin.n_tau = p.n_tau;
    fin.wa = r.L.wa_part;
    fin.n_s = r.xd.nnb;
    fin.n_b = 0;
    fin.o_en = &r.out4[0];
    fin.o_wa = &r.out4[1];
    fin.o_hp = &r.out4[2];
    fin.o_tau = &r.out4[3];
    CellGradArgs ca;
    ca.g = r.g;
    ca.x = r.x;
    ca.y = r.y;
    ca.w = r.prob->w;
    ca.h = r.prob->h;
    ca.exy = reinterpret_cast<const float2*>(p.exy + 2 * i * nn);
    ca.psi = p.psi + i * nn;
    ca.epos = r.L.epos;
    ca.egrad = r.L.egrad;
    ca.scale = r.lambda;
    if (r.params) ca.dscale = r.params;
    ca.gx = r.gx;
    ca.gy = r.gy;
    ca.fin = fin;
    ca.fin_block = r.xd.ncb - 1;
    sr[i] = sum_req(r.xd, r.X, r.L.pin_grad, ca);
    // designs without cells (or the scalars alone) reduce in a separate launch
    fin_separate[i] = !grads || r.xd.ncb <= 0 || r.xd.m <= 0;
  }
  if (grads) {
    if (e == hipSuccess) e = launch_xch_cellsum_batch(sr, count, grad_mode, true, s);
    plan_mark(p, "k_xch_cellsum", s);
  }
  for (int i = 0; i < count; ++i) {
    if (!fin_separate[i]) continue;
    const FinalArgs& f = sr[i].a.fin;
    if (e == hipSuccess)
      e = launch_eval_finalize(f.en, f.n_en, f.tau, f.n_tau, f.wa, f.n_s, f.n_b, f.o_en,
                               f.o_wa, f.o_hp, f.o_tau, s);
    plan_mark(p, "k_eval_finalize", s);
  }
  return dev_status(e);
}

// One evaluation on the cell-major slot path or the float-atomic path.
int run_other(Plan& p, const EvalReq& r, int grad_mode, hipStream_t s) {
  const fftpl_problem* prob = r.prob;
  const bool grads = r.gx != nullptr;
  const bool slots = r.path == FFTPL_PATH_SLOTS;
  const int m = prob->num_cells;
  const BandLayout& L = r.L;
  const int64_t nn = (int64_t)p.n * p.n;
  hipError_t e = hipSuccess;
  p.nev = 0;
  plan_mark(p, "start", s);
  const bool overlap = slots && !p.timing;
  hipStream_t ws = overlap ? p.side : s;
  if (slots) {
    if (overlap) {
      e = hipEventRecord(p.fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(ws, p.fork, 0);
    }
    if (e == hipSuccess)
      e = launch_band_scatter(r.g, L, r.x, r.y, prob->w, prob->h, prob->base, p.rho, s, &p);
    // interleave positions, per-pin gradients into cell-major slots
    if (e == hipSuccess) e = launch_interleave(m, r.x, r.y, L.xy, ws);
    plan_mark(p, "k_interleave", ws);
    if (e == hipSuccess)
      e = launch_wa_pins(prob->num_nets, prob->net_ptr, prob->pin_cell, prob->pin_dx,
                         prob->pin_dy, L.xy, prob->pin_slot, r.gamma, prob->wl_model,
                         L.pin_grad, L.wa_part, ws, &p);
  } else {
    // 1. reset: rho = base, scalar accumulators = 0; 2. atomic scatter
    e = launch_fill(p.rho, prob->base, 0.0f, nn, s);
    plan_mark(p, "k_fill", s);
    if (e == hipSuccess) e = launch_init_eval(r.out4, nullptr, 0, s);
    plan_mark(p, "k_init_eval", s);
    if (e == hipSuccess) e = launch_scatter(r.g, m, r.x, r.y, prob->w, prob->h, p.rho, s);
    plan_mark(p, "k_scatter", s);
  }
  SpectralArgs a = spectral_args(p, r, 0, grad_mode, grads);
  if (e == hipSuccess) e = p.mode == FFTPL_DCT_FFT ? spectral_fft(p, a, s) : spectral_gemm(p, a, s);
  if (e == hipSuccess && overlap) {
    e = hipEventRecord(p.join, ws);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p.join, 0);
  }
  if (slots) {
    if (grads) {
      if (e == hipSuccess)
        e = launch_gather_pins(r.g, m, r.x, r.y, prob->w, prob->h, p.exy, p.psi, grad_mode,
                               r.lambda, prob->cell_ptr, L.pin_grad, r.gx, r.gy, s);
      plan_mark(p, "k_gather_pins", s);
    }
  } else {
    // 4. density gradient (overwrites g), 5. wirelength gradient (float atomics)
    if (e == hipSuccess && m > 0)
      e = launch_gather(r.g, m, r.x, r.y, prob->w, prob->h, nullptr, nullptr, p.exy, p.psi,
                        grad_mode, r.lambda, 0, r.gx, r.gy, s);
    plan_mark(p, "k_gather", s);
    if (e == hipSuccess)
      e = launch_wa(prob->num_nets, prob->net_ptr, prob->pin_cell, prob->pin_dx, prob->pin_dy,
                    r.x, r.y, r.gamma, prob->wl_model, r.gx, r.gy, &r.out4[1], &r.out4[2], s);
    plan_mark(p, "k_wa_atomic", s);
  }
  // 6. N, W~, HPWL, tau from the per-block partials (the atomic path added
  // W~ and HPWL into out4 directly)
  if (e == hipSuccess)
    e = launch_eval_finalize(a.en_part, p.n_en, a.tau_part, p.n_tau, slots ? L.wa_part : nullptr,
                             slots ? (prob->num_nets + 255) / 256 : 0,
                             slots ? wa_big_grid(prob->num_nets) : 0, &r.out4[0], &r.out4[1],
                             &r.out4[2], &r.out4[3], s);
  plan_mark(p, "k_eval_finalize", s);
  return dev_status(e);
}

bool ranges_overlap(const void* a, uint64_t na, const void* b, uint64_t nb) {
  const uintptr_t a0 = reinterpret_cast<uintptr_t>(a), b0 = reinterpret_cast<uintptr_t>(b);
  return a0 < b0 + nb && b0 < a0 + na;
}

// Whether request r can join a group of exchange-path requests.
bool joins_group(const EvalReq* g, int count, const EvalReq& r, int max_batch) {
  if (count >= max_batch || r.path != FFTPL_PATH_EXCHANGE) return false;
  if (count == 0) return true;
  const bool big = g[0].xd.cap > kXchPinLds2;
  if (r.prob->wl_model != g[0].prob->wl_model || (r.xd.cap > kXchPinLds2) != big) return false;
  for (int i = 0; i < count; ++i)
    if (ranges_overlap(g[i].prob->work, g[i].prob->work_bytes, r.prob->work,
                       r.prob->work_bytes))
      return false;
  return true;
}

}  // namespace

extern "C" {

int fftpl_eval(fftpl_plan* plan, const fftpl_problem* prob, const float* x,
               const float* y, float lambda, float gamma, int32_t grad_mode, float* gx,
               float* gy, double* out4, void* stream) {
  FFTPL_RANGE();
  if (!plan) return FFTPL_E_INVAL;
  EvalReq r;
  const int st = check_eval(plan->p, prob, x, y, lambda, gamma, grad_mode, gx, gy, out4, &r);
  if (st != FFTPL_OK) return st;
  hipStream_t s = as_stream(stream);
  if (r.path == FFTPL_PATH_EXCHANGE) return run_exchange_group(plan->p, &r, 1, grad_mode, s);
  return run_other(plan->p, r, grad_mode, s);
}

int fftpl_eval_params(fftpl_plan* plan, const fftpl_problem* prob, const float* x,
                      const float* y, const float* params, int32_t grad_mode, float* gx,
                      float* gy, double* out4, void* stream) {
  FFTPL_RANGE();
  if (!plan || !params || !gx || !gy) return FFTPL_E_INVAL;
  EvalReq r;
  // lambda and gamma are not known on the host: the checks take placeholders
  const int st = check_eval(plan->p, prob, x, y, 0.0f, 1.0f, grad_mode, gx, gy, out4, &r);
  if (st != FFTPL_OK) return st;
  if (r.path != FFTPL_PATH_EXCHANGE) return FFTPL_E_UNSUPPORTED;
  r.params = params;
  return run_exchange_group(plan->p, &r, 1, grad_mode, as_stream(stream));
}

int fftpl_eval_batch(fftpl_plan* plan, int32_t count, const fftpl_problem* const* probs,
                     const float* const* xs, const float* const* ys, const float* lambdas,
                     const float* gammas, int32_t grad_mode, float* const* gxs,
                     float* const* gys, double* out4s, void* stream) {
  FFTPL_RANGE();
  if (count < 0) return FFTPL_E_INVAL;
  if (count == 0) return FFTPL_OK;
  if (!plan || !probs || !xs || !ys || !lambdas || !gammas || !out4s) return FFTPL_E_INVAL;
  if ((gxs == nullptr) != (gys == nullptr)) return FFTPL_E_INVAL;
  // every request is checked before any is enqueued
  std::vector<EvalReq> rs((size_t)count);
  for (int32_t i = 0; i < count; ++i) {
    const int st = check_eval(plan->p, probs[i], xs[i], ys[i], lambdas[i], gammas[i],
                              grad_mode, gxs ? gxs[i] : nullptr, gys ? gys[i] : nullptr,
                              out4s + 4 * (size_t)i, &rs[(size_t)i]);
    if (st != FFTPL_OK) return st;
  }
  hipStream_t s = as_stream(stream);
  EvalReq group[kMaxBatch];
  int ng = 0;
  for (int32_t i = 0; i < count; ++i) {
    const EvalReq& r = rs[(size_t)i];
    if (!joins_group(group, ng, r, plan->p.max_batch) && ng > 0) {
      const int st = run_exchange_group(plan->p, group, ng, grad_mode, s);
      if (st != FFTPL_OK) return st;
      ng = 0;
    }
    if (joins_group(group, ng, r, plan->p.max_batch)) {
      group[ng++] = r;
    } else {
      const int st = run_other(plan->p, r, grad_mode, s);
      if (st != FFTPL_OK) return st;
    }
  }
  if (ng > 0) return run_exchange_group(plan->p, group, ng, grad_mode, s);
  return FFTPL_OK;
}

int fftpl_problem_path(const fftpl_problem* prob, int32_t* path) {
  if (!path) return FFTPL_E_INVAL;
  int pth = FFTPL_PATH_ATOMIC;
  const int st = problem_path(prob, &pth, nullptr, nullptr);
  if (st == FFTPL_OK) *path = pth;
  return st;
}

int fftpl_problem_density(const fftpl_problem* prob, const float* x, const float* y,
                          float* rho, void* stream) {
  FFTPL_RANGE();
  if (!prob || !rho || !grid_ok(&prob->grid)) return FFTPL_E_INVAL;
  const int m = prob->num_cells;
  if (m < 0) return FFTPL_E_INVAL;
  if (m > 0 && (!x || !y || !prob->w || !prob->h)) return FFTPL_E_INVAL;
  if (prob->grid.n > kBandMaxN) return FFTPL_E_UNSUPPORTED;
  if ((reinterpret_cast<uintptr_t>(prob->work) & 255) != 0) return FFTPL_E_INVAL;
  size_t need = 0;
  band_layout(prob->grid.n, m, prob->num_nets, prob->num_pins, nullptr, &need);
  if (!prob->work || prob->work_bytes < need) return FFTPL_E_INVAL;
  if (validate_env() && m > 0) {
    const int v = validate_cells(m, x, y, prob->w, prob->h);
    if (v != FFTPL_OK) return v;
  }
  const BandLayout L =
      band_layout(prob->grid.n, m, prob->num_nets, prob->num_pins, prob->work, nullptr);
  return dev_status(launch_band_scatter(make_gridf(prob->grid), L, x, y, prob->w, prob->h,
                                        prob->base, rho, as_stream(stream)));
}

// The wirelength through the exchange path alone (wl_grad), or its per-net
// values (net_wl, net_hp: the test export).
static int problem_wl(const fftpl_problem* prob, const float* x, const float* y, float gamma,
                      int32_t accumulate, float* gx, float* gy, double* wl, double* hpwl,
                      double* net_wl, double* net_hp, void* stream) {
  if (!prob || !grid_ok(&prob->grid)) return FFTPL_E_INVAL;
  if (!(gamma > 0) || !isfinite(gamma)) return FFTPL_E_INVAL;
  if (accumulate != 0 && accumulate != 1) return FFTPL_E_INVAL;
  if (prob->wl_model != FFTPL_WL_WA && prob->wl_model != FFTPL_WL_LSE) return FFTPL_E_INVAL;
  const int m = prob->num_cells;
  if (m < 0 || prob->num_nets < 0 || prob->num_pins < 0) return FFTPL_E_INVAL;
  if (m > 0 && (!x || !y)) return FFTPL_E_INVAL;
  if (!net_wl && m > 0 && (!gx || !gy)) return FFTPL_E_INVAL;
  if (!prob->net_ptr) return FFTPL_E_INVAL;
  if (prob->num_pins > 0 && (!prob->pin_cell || !prob->pin_dx || !prob->pin_dy || m == 0))
    return FFTPL_E_INVAL;
  int path = FFTPL_PATH_ATOMIC;
  XchDims xd;
  const int st = problem_path(prob, &path, &xd, nullptr);
  if (st != FFTPL_OK) return st;
  if (path != FFTPL_PATH_EXCHANGE) return FFTPL_E_INVAL;
  if (validate_env()) {
    int v = validate_netlist(prob->num_nets, prob->net_ptr, prob->num_pins, prob->pin_cell, m);
    if (v == FFTPL_OK) v = validate_index(prob, xd);
    if (v != FFTPL_OK) return v;
  }
  hipStream_t s = as_stream(stream);
  const BandLayout L =
      band_layout(prob->grid.n, m, prob->num_nets, prob->num_pins, prob->work, nullptr);
  const XchIndex X = xch_index(xd, prob->xindex);
  XchReq xr = xch_req(xd, X, x, y, L.pin_grad, prob->net_ptr, prob->pin_dx, prob->pin_dy,
                      gamma, L.wa_part);
  xr.net_wl = net_wl;
  xr.net_hp = net_hp;
  hipError_t e = launch_xch_spread_batch(&xr, 1, s);
  if (e == hipSuccess) e = launch_xch_wa_batch(&xr, 1, prob->wl_model, s);
  if (net_wl) return dev_status(e);
  FinalArgs fin;
  fin.wa = L.wa_part;
  fin.n_s = xd.nnb;
  fin.o_wa = wl;
  fin.o_hp = hpwl;
  const bool want = wl || hpwl;
  if (m > 0 && xd.ncb > 0) {
    CellGradArgs ca;
    ca.g = make_gridf(prob->grid);
    ca.gx = gx;
    ca.gy = gy;
    ca.accumulate = accumulate;
    ca.fin = fin;
    ca.fin_block = want ? xd.ncb - 1 : -1;
    const SumReq sr = sum_req(xd, X, L.pin_grad, ca);
    if (e == hipSuccess) e = launch_xch_cellsum_batch(&sr, 1, FFTPL_GRAD_FIELD, false, s);
  } else if (want && e == hipSuccess) {
    e = launch_eval_finalize(nullptr, 0, nullptr, 0, fin.wa, fin.n_s, 0, nullptr, wl, hpwl,
                             nullptr, s);
  }
  return dev_status(e);
}

int fftpl_problem_wl_grad(const fftpl_problem* prob, const float* x, const float* y,
                          float gamma, int32_t accumulate, float* gx, float* gy, double* wl,
                          double* hpwl, void* stream) {
  FFTPL_RANGE();
  return problem_wl(prob, x, y, gamma, accumulate, gx, gy, wl, hpwl, nullptr, nullptr, stream);
}

int fftpl_debug_net_values(const fftpl_problem* prob, const float* x, const float* y,
                           float gamma, double* wl_first, double* hpwl_first, void* stream) {
  FFTPL_RANGE();
  if (!wl_first || !hpwl_first) return FFTPL_E_INVAL;
  return problem_wl(prob, x, y, gamma, 0, nullptr, nullptr, nullptr, nullptr, wl_first,
                    hpwl_first, stream);
}

int fftpl_plan_timing(fftpl_plan* plan, int32_t enable) {
  if (!plan || (enable != 0 && enable != 1)) return FFTPL_E_INVAL;
  Plan& p = plan->p;
  if (enable && !p.ev[0]) {
    for (int i = 0; i < Plan::kMaxEvents; ++i)
      if (hipEventCreate(&p.ev[i]) != hipSuccess) return FFTPL_E_DEVICE;
  }
  p.timing = enable != 0;
  p.nev = 0;
  return FFTPL_OK;
}

int fftpl_plan_kernel_times(fftpl_plan* plan, int32_t max, float* ms, const char** names,
                            int32_t* count) {
  if (!plan || !count || max < 0 || (max > 0 && (!ms || !names))) return FFTPL_E_INVAL;
  Plan& p = plan->p;
  *count = 0;
  if (!p.timing || p.nev < 2) return FFTPL_OK;
  if (hipEventSynchronize(p.ev[p.nev - 1]) != hipSuccess) return FFTPL_E_DEVICE;
  const int k = p.nev - 1 < max ? p.nev - 1 : max;
  for (int i = 0; i < k; ++i) {
    float t = 0.0f;
    if (hipEventElapsedTime(&t, p.ev[i], p.ev[i + 1]) != hipSuccess) return FFTPL_E_DEVICE;
    ms[i] = t;
    names[i] = p.ev_name[i + 1];
  }
  *count = k;
  return FFTPL_OK;
}

int fftpl_problem_work_bytes(int32_t n, int32_t num_cells, int32_t num_nets,
                             int32_t num_pins, uint64_t* bytes) {
  if (!bytes || n < 1 || num_cells < 0 || num_nets < 0 || num_pins < 0)
    return FFTPL_E_INVAL;
  size_t need = 0;
  band_layout(n, num_cells, num_nets, num_pins, nullptr, &need);
  *bytes = need;
  return FFTPL_OK;
}

int fftpl_netlist_index(int32_t num_cells, int32_t num_pins, const int32_t* pin_cell,
                        int32_t* cell_ptr, int32_t* pin_slot, int32_t* work, void* stream) {
  FFTPL_RANGE();
  if (num_cells < 0 || num_pins < 0 || !cell_ptr || !work) return FFTPL_E_INVAL;
  if (num_pins > 0 && (!pin_cell || !pin_slot || num_cells == 0)) return FFTPL_E_INVAL;
  if (validate_env() && num_pins > 0) {
    if (hipDeviceSynchronize() != hipSuccess) return FFTPL_E_DEVICE;
    auto pc = to_host(pin_cell, (size_t)num_pins);
    for (int q = 0; q < num_pins; ++q)
      if (pc[q] < 0 || pc[q] >= num_cells) return FFTPL_E_INVAL;
  }
  return dev_status(launch_netlist_index(num_cells, num_pins, pin_cell, cell_ptr, pin_slot,
                                         work, as_stream(stream)));
}

int fftpl_xindex_bytes(int32_t num_cells, int32_t num_nets, int32_t num_pins,
                       int32_t max_degree, uint64_t* index_bytes, uint64_t* work_bytes) {
  if (!index_bytes || !work_bytes) return FFTPL_E_INVAL;
  XchDims d;
  const int st = xch_dims(num_cells, num_nets, num_pins, max_degree, &d);
  if (st != FFTPL_OK) return st;
  *index_bytes = d.index_bytes;
  *work_bytes = d.work_bytes;
  return FFTPL_OK;
}

int fftpl_xindex_build(int32_t num_cells, int32_t num_nets, int32_t num_pins,
                       const int32_t* net_ptr, const int32_t* pin_cell, int32_t max_degree,
                       void* index, uint64_t index_bytes, void* work, uint64_t work_bytes,
                       uint64_t* key, void* stream) {
  FFTPL_RANGE();
  XchDims d;
  const int st = xch_dims(num_cells, num_nets, num_pins, max_degree, &d);
  if (st != FFTPL_OK) return st;
  if (!net_ptr || !index || !work || (num_pins > 0 && !pin_cell)) return FFTPL_E_INVAL;
  if (num_pins > 0 && num_cells == 0) return FFTPL_E_INVAL;
  if (index_bytes < d.index_bytes || work_bytes < d.work_bytes) return FFTPL_E_INVAL;
  if ((reinterpret_cast<uintptr_t>(index) & 255) != 0 ||
      (reinterpret_cast<uintptr_t>(work) & 255) != 0)
    return FFTPL_E_INVAL;
  const int st2 = xch_build(d, net_ptr, pin_cell, index, work, as_stream(stream));
  if (st2 == FFTPL_OK && key)
    *key = xindex_fingerprint(num_cells, num_nets, num_pins, max_degree, net_ptr, pin_cell,
                              index);
  return st2;
}

int fftpl_step_stats(int32_t num_cells, const float* ux, const float* uy, const float* upx,
                     const float* upy, const float* gx, const float* gy, const float* gpx,
                     const float* gpy, double* out4, double* work, uint64_t work_doubles,
                     void* stream) {
  FFTPL_RANGE();
  if (num_cells < 0 || !out4 || !work || work_doubles < step_stats_work_doubles())
    return FFTPL_E_INVAL;
  if (num_cells > 0 && (!ux || !uy || !gx || !gy)) return FFTPL_E_INVAL;
  const bool prev = upx || upy || gpx || gpy;
  if (prev && (!upx || !upy || !gpx || !gpy)) return FFTPL_E_INVAL;
  return dev_status(launch_step_stats(num_cells, ux, uy, upx, upy, gx, gy, gpx, gpy, out4, work,
                                      as_stream(stream)));
}

int fftpl_nesterov_update(const fftpl_grid* region, int32_t num_cells, const float* w,
                          const float* h, float* x, float* y, float* ux, float* uy, float* upx,
                          float* upy, float* gpx, float* gpy, const float* gx, const float* gy,
                          float step, float beta, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(region) || num_cells < 0) return FFTPL_E_INVAL;
  if (!isfinite(step) || step < 0.0f || !isfinite(beta) || beta < 0.0f || beta >= 1.0f)
    return FFTPL_E_INVAL;
  if (num_cells > 0 &&
      (!w || !h || !x || !y || !ux || !uy || !upx || !upy || !gpx || !gpy || !gx || !gy))
    return FFTPL_E_INVAL;
  const float xl = (float)region->xl, yl = (float)region->yl;
  const float xh = (float)(region->xl + region->n * region->bin_w);
  const float yh = (float)(region->yl + region->n * region->bin_h);
  return dev_status(launch_nesterov_update(num_cells, x, y, ux, uy, upx, upy, gpx, gpy, gx, gy,
                                           w, h, step, beta, nullptr, xl, yl, xh, yh,
                                           as_stream(stream)));
}

int fftpl_nesterov_update_dev(const fftpl_grid* region, int32_t num_cells, const float* w,
                              const float* h, float* x, float* y, float* ux, float* uy,
                              float* upx, float* upy, float* gpx, float* gpy, const float* gx,
                              const float* gy, const double* step_beta, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(region) || num_cells < 0 || !step_beta) return FFTPL_E_INVAL;
  if (num_cells > 0 &&
      (!w || !h || !x || !y || !ux || !uy || !upx || !upy || !gpx || !gpy || !gx || !gy))
    return FFTPL_E_INVAL;
  const float xl = (float)region->xl, yl = (float)region->yl;
  const float xh = (float)(region->xl + region->n * region->bin_w);
  const float yh = (float)(region->yl + region->n * region->bin_h);
  return dev_status(launch_nesterov_update(num_cells, x, y, ux, uy, upx, upy, gpx, gpy, gx, gy,
                                           w, h, 0.0f, 0.0f, step_beta, xl, yl, xh, yh,
                                           as_stream(stream)));
}

int fftpl_nesterov_schedule(const double* stats, const double* out4, double* state,
                            float* params, double* log, int32_t log_cap, void* stream) {
  FFTPL_RANGE();
  if (!stats || !out4 || !state || !params || log_cap < 0 || (log_cap > 0 && !log))
    return FFTPL_E_INVAL;
  return dev_status(launch_nesterov_schedule(stats, out4, state, params, log, log_cap,
                                             as_stream(stream)));
}

int fftpl_cg_dots(int32_t num_cells, const float* gx, const float* gy, const float* gpx,
                  const float* gpy, const float* dx, const float* dy, double* out4,
                  double* work, uint64_t work_doubles, void* stream) {
  FFTPL_RANGE();
  if (num_cells < 0 || !out4 || !work || work_doubles < step_stats_work_doubles())
    return FFTPL_E_INVAL;
  if (num_cells > 0 && (!gx || !gy)) return FFTPL_E_INVAL;
  if ((gpx == nullptr) != (gpy == nullptr) || (dx == nullptr) != (dy == nullptr))
    return FFTPL_E_INVAL;
  return dev_status(
      launch_cg_dots(num_cells, gx, gy, gpx, gpy, dx, dy, out4, work, as_stream(stream)));
}

int fftpl_cg_direction(int32_t num_cells, const float* gx, const float* gy, float beta,
                       float* dx, float* dy, double* dmax, double* work, uint64_t work_doubles,
                       void* stream) {
  FFTPL_RANGE();
  if (num_cells < 0 || !dmax || !work || work_doubles < step_stats_work_doubles())
    return FFTPL_E_INVAL;
  if (!isfinite(beta) || beta < 0.0f) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!gx || !gy || !dx || !dy)) return FFTPL_E_INVAL;
  return dev_status(
      launch_cg_direction(num_cells, gx, gy, beta, dx, dy, dmax, work, as_stream(stream)));
}

int fftpl_cg_move(const fftpl_grid* region, int32_t num_cells, const float* w, const float* h,
                  const float* x, const float* y, const float* dx, const float* dy, float t,
                  float* xo, float* yo, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(region) || num_cells < 0 || !isfinite(t)) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!w || !h || !x || !y || !dx || !dy || !xo || !yo))
    return FFTPL_E_INVAL;
  const float xl = (float)region->xl, yl = (float)region->yl;
  const float xh = (float)(region->xl + region->n * region->bin_w);
  const float yh = (float)(region->yl + region->n * region->bin_h);
  return dev_status(launch_cg_move(num_cells, x, y, dx, dy, t, w, h, xl, yl, xh, yh, xo, yo,
                                   as_stream(stream)));
}

int fftpl_debug_cell_bins(const fftpl_grid* grid, int32_t num_cells, const float* x,
                          const float* y, const float* w, const float* h,
                          int32_t* ranges, void* stream) {
  FFTPL_RANGE();
  if (!grid_ok(grid) || num_cells < 0) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!x || !y || !w || !h || !ranges)) return FFTPL_E_INVAL;
  return dev_status(
      launch_cell_bins(make_gridf(*grid), num_cells, x, y, w, h, ranges, as_stream(stream)));
}

}  // extern "C"
