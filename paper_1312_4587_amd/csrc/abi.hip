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
// returns the number of doubles to allocate.
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

int fftpl_plan_create(fftpl_plan** out, int32_t n, int32_t dct_mode, void* stream) {
  if (!out) return FFTPL_E_INVAL;
  *out = nullptr;
  if (dct_mode < FFTPL_DCT_FFT || dct_mode > FFTPL_DCT_GEMM_BF16X3) return FFTPL_E_INVAL;
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
  hipGetDevice(&p.device);
  const size_t nn = (size_t)n * n;
  bool ok = hipMalloc(&p.fft_tw, sizeof(float2) * n) == hipSuccess &&
            hipMalloc(&p.dct_cs, sizeof(float2) * (n / 2 + 1)) == hipSuccess &&
            hipMalloc(&p.wfreq, sizeof(float) * n) == hipSuccess &&
            hipMalloc(&p.rho, sizeof(float) * nn) == hipSuccess &&
            hipMalloc(&p.tmp0, sizeof(float) * nn) == hipSuccess &&
            hipMalloc(&p.tmp1, sizeof(float) * nn) == hipSuccess &&
            hipMalloc(&p.tmp2, sizeof(float) * nn) == hipSuccess &&
            hipMalloc(&p.psi, sizeof(float) * nn) == hipSuccess &&
            hipMalloc(&p.exy, sizeof(float) * 2 * nn) == hipSuccess &&
            hipMalloc(&p.rowsum, sizeof(double) * n) == hipSuccess &&
            hipMalloc(&p.partials, sizeof(double) * plan_partials(p, n, dct_mode)) == hipSuccess;
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

int fftpl_plan_info(const fftpl_plan* plan, int32_t* n, int32_t* dct_mode) {
  if (!plan) return FFTPL_E_INVAL;
  if (n) *n = plan->p.n;
  if (dct_mode) *dct_mode = plan->p.mode;
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
  if (!grid_ok(grid) || num_cells < 0 || !rho) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!x || !y || !w || !h)) return FFTPL_E_INVAL;
  if (validate_env() && num_cells > 0) {
    int v = validate_cells(num_cells, x, y, w, h);
    if (v != FFTPL_OK) return v;
  }
  const GridF g = make_gridf(*grid);
  hipStream_t s = as_stream(stream);
  hipError_t e = launch_fill(rho, base, 0.0f, (int64_t)grid->n * grid->n, s);
  if (e == hipSuccess) e = launch_scatter(g, num_cells, x, y, w, h, rho, s);
  return dev_status(e);
}

int fftpl_helmholtz_solve(fftpl_plan* plan, const fftpl_grid* grid, float eps,
                          const float* rho, float* psi, float* ex, float* ey,
                          double* energy, void* stream) {
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
  return fftpl_helmholtz_solve(plan, grid, 0.0f, rho, psi, ex, ey, energy, stream);
}

int fftpl_field_gather(const fftpl_grid* grid, int32_t num_cells, const float* x,
                       const float* y, const float* w, const float* h,
                       const float* ex, const float* ey, const float* psi,
                       int32_t grad_mode, float scale, int32_t accumulate,
                       float* gx, float* gy, void* stream) {
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
  if (!accumulate && num_cells > 0) {
    e = launch_fill(gx, nullptr, 0.0f, num_cells, s);
    if (e == hipSuccess) e = launch_fill(gy, nullptr, 0.0f, num_cells, s);
  }
  if (e == hipSuccess && wa) e = launch_fill_f64(wa, 0.0, 1, s);
  if (e == hipSuccess && hpwl) e = launch_fill_f64(hpwl, 0.0, 1, s);
  if (e == hipSuccess)
    e = launch_wa(num_nets, net_ptr, pin_cell, pin_dx, pin_dy, x, y, gamma, wl_model, gx, gy,
                  wa, hpwl, s);
  return dev_status(e);
}

int fftpl_wa_grad(int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                  const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                  int32_t num_cells, const float* x, const float* y, float gamma,
                  int32_t accumulate, float* gx, float* gy, double* wa, double* hpwl,
                  void* stream) {
  return wl_grad(FFTPL_WL_WA, num_nets, net_ptr, num_pins, pin_cell, pin_dx, pin_dy, num_cells,
                 x, y, gamma, accumulate, gx, gy, wa, hpwl, stream);
}

int fftpl_lse_grad(int32_t num_nets, const int32_t* net_ptr, int32_t num_pins,
                   const int32_t* pin_cell, const float* pin_dx, const float* pin_dy,
                   int32_t num_cells, const float* x, const float* y, float gamma,
                   int32_t accumulate, float* gx, float* gy, double* wa, double* hpwl,
                   void* stream) {
  return wl_grad(FFTPL_WL_LSE, num_nets, net_ptr, num_pins, pin_cell, pin_dx, pin_dy,
                 num_cells, x, y, gamma, accumulate, gx, gy, wa, hpwl, stream);
}

// One evaluation; with check_only, the host-side checks alone (nothing is
// enqueued).
static int eval_impl(fftpl_plan* plan, const fftpl_problem* prob, const float* x,
                     const float* y, float lambda, float gamma, int32_t grad_mode, float* gx,
                     float* gy, double* out4, void* stream, bool check_only) {
  if (!plan || !prob || !out4 || !grid_ok(&prob->grid)) return FFTPL_E_INVAL;
  if (prob->wl_model != FFTPL_WL_WA && prob->wl_model != FFTPL_WL_LSE) return FFTPL_E_INVAL;
  if (!(prob->screening >= 0.0f) || !isfinite(prob->screening)) return FFTPL_E_INVAL;
  if (prob->grid.n != plan->p.n) return FFTPL_E_STATE;
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
  if (validate_env()) {
    int v = validate_netlist(prob->num_nets, prob->net_ptr, prob->num_pins, prob->pin_cell, m);
    if (v == FFTPL_OK && m > 0) v = validate_cells(m, x, y, prob->w, prob->h);
    if (v != FFTPL_OK) return v;
  }
  Plan& p = plan->p;
  const GridF g = make_gridf(prob->grid);
  hipStream_t s = as_stream(stream);
  const int64_t nn = (int64_t)p.n * p.n;
  // Atomic-free paths when the caller supplied a workspace and a pin index:
  // the exchange index (xch) or the cell-major slots (slots).
  size_t need = 0;
  BandLayout L = band_layout(p.n, m, prob->num_nets, prob->num_pins, nullptr, &need);
  // the workspace and the index are read in 16-byte vectors: device
  // allocations are 256-byte aligned, and so must these be
  if ((reinterpret_cast<uintptr_t>(prob->work) & 255) != 0 ||
      (reinterpret_cast<uintptr_t>(prob->xindex) & 255) != 0)
    return FFTPL_E_INVAL;
  const bool ws_ok = prob->work && prob->work_bytes >= need && p.n <= kBandMaxN;
  XchDims xd;
  const bool xch = ws_ok && prob->xindex &&
                   xch_dims(m, prob->num_nets, prob->num_pins, prob->max_degree, &xd) ==
                       FFTPL_OK &&
                   prob->xindex_bytes >= xd.index_bytes;
  const bool slots = !xch && ws_ok && prob->cell_ptr && prob->pin_slot;
  const bool fast = xch || slots;
  if (!grads && !fast && m > 0) return FFTPL_E_INVAL;
  if (fast) L = band_layout(p.n, m, prob->num_nets, prob->num_pins, prob->work, nullptr);
  XchIndex X;
  if (xch) {
    X = xch_index(xd, prob->xindex);
    if (validate_env()) {
      int32_t hdr[9];
      if (hipDeviceSynchronize() != hipSuccess ||
          hipMemcpy(hdr, prob->xindex, sizeof(hdr), hipMemcpyDeviceToHost) != hipSuccess)
        return FFTPL_E_DEVICE;
      if (hdr[1] != m || hdr[2] != prob->num_nets || hdr[3] != prob->num_pins ||
          hdr[4] != prob->max_degree || hdr[5] != xd.npt || hdr[8] != xd.cpb)
        return FFTPL_E_STATE;
    }
  }
  if (check_only) return FFTPL_OK;
  hipError_t e = hipSuccess;
  p.nev = 0;
  plan_mark(p, "start", s);
  // With per-kernel timing on, everything runs on `s` so that consecutive
  // events bracket single kernels.  Otherwise the wirelength branch (spread,
  // net blocks) runs on the plan's side stream `ws` while the density branch
  // (banded scatter, solve, band gather), the longer of the two when they
  // share the chip, stays on `s`: the hand-over between streams costs
  // several microseconds each way, and this way the fork delays only the
  // shorter branch and the join is usually complete by the time the density
  // branch reaches it.
  const bool overlap = fast && !p.timing;
  hipStream_t ds = s;
  hipStream_t ws = overlap ? p.side : s;
  if (fast) {
    if (overlap) {
      e = hipEventRecord(p.fork, s);
      if (e == hipSuccess) e = hipStreamWaitEvent(ws, p.fork, 0);
    }
    // density branch: banded scatter (its counters and the scalars are all
    // written, not accumulated, so nothing needs zeroing first)
    if (e == hipSuccess)
      e = launch_band_scatter(g, L, x, y, prob->w, prob->h, prob->base, p.rho, ds, &p);
    // wirelength branch
    if (xch) {
      // pin positions into the exchange buffer, then every net block (the
      // per-cell sums follow the join)
      if (e == hipSuccess) e = launch_xch_spread(xd, X, x, y, L.pin_grad, ws);
      plan_mark(p, "k_xch_spread", ws);
      if (e == hipSuccess)
        e = launch_xch_wa(xd, X, prob->net_ptr, prob->pin_dx, prob->pin_dy, gamma,
                          prob->wl_model, L.pin_grad, L.wa_part, ws);
      plan_mark(p, "k_xch_wa", ws);
    } else {
      // interleave positions, per-pin WA gradients into cell-major slots
      if (e == hipSuccess) e = launch_interleave(m, x, y, L.xy, ws);
      plan_mark(p, "k_interleave", ws);
      if (e == hipSuccess)
        e = launch_wa_pins(prob->num_nets, prob->net_ptr, prob->pin_cell, prob->pin_dx,
                           prob->pin_dy, L.xy, prob->pin_slot, gamma, prob->wl_model,
                           L.pin_grad, L.wa_part, ws, &p);
    }
  } else {
    // 1. reset: rho = base, scalar accumulators = 0; 2. atomic scatter
    e = launch_fill(p.rho, prob->base, 0.0f, nn, s);
    plan_mark(p, "k_fill", s);
    if (e == hipSuccess) e = launch_init_eval(out4, nullptr, 0, s);
    plan_mark(p, "k_init_eval", s);
    if (e == hipSuccess) e = launch_scatter(g, m, x, y, prob->w, prob->h, p.rho, s);
    plan_mark(p, "k_scatter", s);
  }
  // 3. spectral solve (density branch); overflow sums in the first pass,
  // energy in the last
  if (e == hipSuccess) {
    SpectralArgs a;
    a.rho = p.rho;
    // FIELD: (Ex, Ey); EXACT: psi and the difference maps (Dx, Dy) the exact
    // gradient is summed from; scalars only: neither map
    a.psi = grads && grad_mode == FFTPL_GRAD_EXACT ? p.psi : nullptr;
    a.exy = grads ? p.exy : nullptr;
    a.diff = grad_mode == FFTPL_GRAD_EXACT;
    a.en_part = p.partials;
    a.base = prob->base;
    a.cap = prob->cap;
    a.rho_t = g.rho_t;
    a.tau_part = p.partials + p.en_max;
    a.eps = prob->screening;
    e = p.mode == FFTPL_DCT_FFT ? spectral_fft(p, a, ds) : spectral_gemm(p, a, ds);
  }
  // exchange path: each cell's density gradient, computed band by band from
  // the band entries (L2-local reads of the field), still on the density
  // branch
  if (fast && xch && grads) {
    if (e == hipSuccess) e = launch_band_gather(g, L, p.exy, p.psi, grad_mode, ds);
    plan_mark(p, "k_band_gather", ds);
  }
  // join the wirelength branch
  if (e == hipSuccess && overlap) {
    e = hipEventRecord(p.join, ws);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p.join, 0);
  }
  bool fin_in_cellsum = false;
  FinalArgs fin;
  fin.en = p.partials;
  fin.n_en = p.n_en;
  fin.tau = p.partials + p.en_max;
  fin.n_tau = p.n_tau;
  fin.wa = fast ? L.wa_part : nullptr;
  fin.n_s = fast ? (xch ? xd.nnb : (prob->num_nets + 255) / 256) : 0;
  fin.n_b = fast ? (xch ? 0 : wa_big_grid(prob->num_nets)) : 0;
  fin.o_en = &out4[0];
  fin.o_wa = &out4[1];
  fin.o_hp = &out4[2];
  fin.o_tau = &out4[3];
  if (fast) {
    // 5. per cell: density gradient plus the sum of its pins' gradients
    if (!grads) {
      // scalars only
    } else if (xch) {
      // g = lambda * density gradient + each cell's sum of pin gradients
      CellGradArgs ca;
      ca.g = g;
      ca.x = x;
      ca.y = y;
      ca.w = prob->w;
      ca.h = prob->h;
      ca.exy = reinterpret_cast<const float2*>(p.exy);
      ca.psi = p.psi;
      ca.epos = L.epos;
      ca.egrad = L.egrad;
      ca.scale = lambda;
      ca.gx = gx;
      ca.gy = gy;
      // the last cell block (the last one dispatched, and at most as large as
      // the others) reduces the scalars too
      ca.fin = fin;
      ca.fin_block = xd.ncb - 1;
      fin_in_cellsum = xd.ncb > 0;
      if (e == hipSuccess) e = launch_xch_cellsum(xd, X, L.pin_grad, ca, grad_mode, s);
      plan_mark(p, "k_xch_cellsum", s);
    } else {
      if (e == hipSuccess)
        e = launch_gather_pins(g, m, x, y, prob->w, prob->h, p.exy, p.psi, grad_mode, lambda,
                               prob->cell_ptr, L.pin_grad, gx, gy, s);
      plan_mark(p, "k_gather_pins", s);
    }
  } else {
    // 4. density gradient (overwrites g), 5. WA gradient (float atomics)
    if (e == hipSuccess && m > 0)
      e = launch_gather(g, m, x, y, prob->w, prob->h, nullptr, nullptr, p.exy, p.psi,
                        grad_mode, lambda, 0, gx, gy, s);
    plan_mark(p, "k_gather", s);
    if (e == hipSuccess)
      e = launch_wa(prob->num_nets, prob->net_ptr, prob->pin_cell, prob->pin_dx,
                    prob->pin_dy, x, y, gamma, prob->wl_model, gx, gy, &out4[1], &out4[2],
                    s);
    plan_mark(p, "k_wa_atomic", s);
  }
  // 6. N, W~, HPWL, tau from the per-block partials (the atomic path added
  // W~ and HPWL into out4 directly): by the exchange path's cell sums, or a
  // separate one-block launch (a last-block-done count in the gather would
  // put every gather block's atomic on one address, which costs far more
  // than the launch).
  if (!fin_in_cellsum) {
    if (e == hipSuccess)
      e = launch_eval_finalize(fin.en, fin.n_en, fin.tau, fin.n_tau, fin.wa, fin.n_s, fin.n_b,
                               fin.o_en, fin.o_wa, fin.o_hp, fin.o_tau, s);
    plan_mark(p, "k_eval_finalize", s);
  }
  return dev_status(e);
}

int fftpl_eval(fftpl_plan* plan, const fftpl_problem* prob, const float* x,
               const float* y, float lambda, float gamma, int32_t grad_mode, float* gx,
               float* gy, double* out4, void* stream) {
  return eval_impl(plan, prob, x, y, lambda, gamma, grad_mode, gx, gy, out4, stream, false);
}

int fftpl_eval_batch(fftpl_plan* plan, int32_t count, const fftpl_problem* const* probs,
                     const float* const* xs, const float* const* ys, const float* lambdas,
                     const float* gammas, int32_t grad_mode, float* const* gxs,
                     float* const* gys, double* out4s, void* stream) {
  if (count < 0) return FFTPL_E_INVAL;
  if (count == 0) return FFTPL_OK;
  if (!plan || !probs || !xs || !ys || !lambdas || !gammas || !out4s) return FFTPL_E_INVAL;
  if ((gxs == nullptr) != (gys == nullptr)) return FFTPL_E_INVAL;
  // every request is checked before any is enqueued
  for (int32_t i = 0; i < count; ++i) {
    const int st = eval_impl(plan, probs[i], xs[i], ys[i], lambdas[i], gammas[i], grad_mode,
                             gxs ? gxs[i] : nullptr, gys ? gys[i] : nullptr,
                             out4s + 4 * (size_t)i, stream, true);
    if (st != FFTPL_OK) return st;
  }
  for (int32_t i = 0; i < count; ++i) {
    const int st = eval_impl(plan, probs[i], xs[i], ys[i], lambdas[i], gammas[i], grad_mode,
                             gxs ? gxs[i] : nullptr, gys ? gys[i] : nullptr,
                             out4s + 4 * (size_t)i, stream, false);
    if (st != FFTPL_OK) return st;
  }
  return FFTPL_OK;
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
                       void* stream) {
  XchDims d;
  const int st = xch_dims(num_cells, num_nets, num_pins, max_degree, &d);
  if (st != FFTPL_OK) return st;
  if (!net_ptr || !index || !work || (num_pins > 0 && !pin_cell)) return FFTPL_E_INVAL;
  if (num_pins > 0 && num_cells == 0) return FFTPL_E_INVAL;
  if (index_bytes < d.index_bytes || work_bytes < d.work_bytes) return FFTPL_E_INVAL;
  if ((reinterpret_cast<uintptr_t>(index) & 255) != 0 ||
      (reinterpret_cast<uintptr_t>(work) & 255) != 0)
    return FFTPL_E_INVAL;
  return xch_build(d, net_ptr, pin_cell, index, work, as_stream(stream));
}

int fftpl_step_stats(int32_t num_cells, const float* ux, const float* uy, const float* upx,
                     const float* upy, const float* gx, const float* gy, const float* gpx,
                     const float* gpy, double* out4, double* work, uint64_t work_doubles,
                     void* stream) {
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
                                           w, h, step, beta, xl, yl, xh, yh,
                                           as_stream(stream)));
}

int fftpl_debug_cell_bins(const fftpl_grid* grid, int32_t num_cells, const float* x,
                          const float* y, const float* w, const float* h,
                          int32_t* ranges, void* stream) {
  if (!grid_ok(grid) || num_cells < 0) return FFTPL_E_INVAL;
  if (num_cells > 0 && (!x || !y || !w || !h || !ranges)) return FFTPL_E_INVAL;
  return dev_status(
      launch_cell_bins(make_gridf(*grid), num_cells, x, y, w, h, ranges, as_stream(stream)));
}

}  // extern "C"
