// Device side of the global placement iteration (Algorithm 1, the update of
// the positions after each gradient evaluation): the reductions that pick the
// step length, the Nesterov update of the cell centres, and the vector steps
// of nonlinear conjugate gradients (dots, direction, move along it).
//
// Step statistics, in double, from per-block partials summed in a fixed order:
//   out[0] = sum |u - u_prev|^2    (both axes)
//   out[1] = sum |g - g_prev|^2
//   out[2] = max |g|               (largest gradient component)
//   out[3] = sum |g|_1
// Update, per cell and axis, with the look-ahead point u at which g was taken:
//   x_new = clamp(u - step * g),  u_new = clamp(x_new + beta (x_new - x)),
//   u_prev = u, g_prev = g, x = x_new, u = u_new,
// where clamp keeps the cell inside the placement region.
#include <math.h>

#include "fftpl_internal.hpp"

namespace fftpl {

namespace {

constexpr int kStatBlocks = 256;
constexpr int kStatThreads = 256;

__global__ void __launch_bounds__(kStatThreads)
    k_step_stats(int m, const float* __restrict__ ux, const float* __restrict__ uy,
                 const float* __restrict__ upx, const float* __restrict__ upy,
                 const float* __restrict__ gx, const float* __restrict__ gy,
                 const float* __restrict__ gpx, const float* __restrict__ gpy,
                 double* __restrict__ part) {
  double du = 0.0, dg = 0.0, gs = 0.0;
  float gm = 0.0f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const float a = gx[i], b = gy[i];
    if (upx) {
      const double ex = (double)ux[i] - upx[i], ey = (double)uy[i] - upy[i];
      const double fx = (double)a - gpx[i], fy = (double)b - gpy[i];
      du += ex * ex + ey * ey;
      dg += fx * fx + fy * fy;
    }
    gm = fmaxf(gm, fmaxf(fabsf(a), fabsf(b)));
    gs += (double)fabsf(a) + fabsf(b);
  }
  block_sum_to<false>(du, &part[blockIdx.x]);
  block_sum_to<false>(dg, &part[gridDim.x + blockIdx.x]);
  block_sum_to<false>(gs, &part[3 * gridDim.x + blockIdx.x]);
  // max of non-negative floats: exact in any order
  __shared__ float wm[kStatThreads / kWave];
  gm = wave_max(gm);
  if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = gm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float v = 0.0f;
    for (int k = 0; k < kStatThreads / kWave; ++k) v = fmaxf(v, wm[k]);
    part[2 * gridDim.x + blockIdx.x] = v;
  }
}

__global__ void __launch_bounds__(64)
    k_step_stats_final(const double* __restrict__ part, int nblk, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j < 4) {
    double v = 0.0;
    for (int b = 0; b < nblk; ++b) {
      const double p = part[j * nblk + b];
      v = j == 2 ? fmax(v, p) : v + p;
    }
    out[j] = v;
  }
}

__device__ __forceinline__ float clampc(float v, float lo, float hi) {
  return lo <= hi ? fminf(fmaxf(v, lo), hi) : 0.5f * (lo + hi);
}

__global__ void __launch_bounds__(256)
    k_nesterov_update(int m, float* __restrict__ x, float* __restrict__ y,
                      float* __restrict__ ux, float* __restrict__ uy,
                      float* __restrict__ upx, float* __restrict__ upy,
                      float* __restrict__ gpx, float* __restrict__ gpy,
                      const float* __restrict__ gx, const float* __restrict__ gy,
                      const float* __restrict__ w, const float* __restrict__ h, float step,
                      float beta, const double* __restrict__ step_beta, float xl, float yl,
                      float xh, float yh) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (step_beta) {   // set on the device by the schedule
    step = (float)step_beta[0];
    beta = (float)step_beta[1];
  }
  const float hw = 0.5f * w[i], hh = 0.5f * h[i];
  const float ax = ux[i], ay = uy[i], bx = gx[i], by = gy[i];
  const float nx = clampc(ax - step * bx, xl + hw, xh - hw);
  const float ny = clampc(ay - step * by, yl + hh, yh - hh);
  const float vx = clampc(nx + beta * (nx - x[i]), xl + hw, xh - hw);
  const float vy = clampc(ny + beta * (ny - y[i]), yl + hh, yh - hh);
  upx[i] = ax;
  upy[i] = ay;
  gpx[i] = bx;
  gpy[i] = by;
  x[i] = nx;
  y[i] = ny;
  ux[i] = vx;
  uy[i] = vy;
}

// The host schedule of one Nesterov iteration, on the device (Section IV-A),
// in double with the host's operation order (no contraction), so that a loop
// of evaluations can run without a host read per iteration.  State layout:
// see fftpl_nesterov_schedule.
__global__ void __launch_bounds__(64)
    k_nesterov_schedule(const double* __restrict__ stats, const double* __restrict__ out4,
                        double* __restrict__ st, float* __restrict__ params,
                        double* __restrict__ log, int log_cap) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  const double du2 = stats[0], dg2 = stats[1], gmax = stats[2];
  const double N = out4[0], W = out4[1], H = out4[2], tau = out4[3];
  const double a = st[0], amax = st[1], amin = st[2], lam = st[3], gamma = st[4];
  const double k = st[5], last_h = st[6], amax0 = st[7], bw = st[8];
  // step length: the Barzilai-Borwein estimate as the largest displacement
  double alpha = amax;
  if (!(k == 0.0 || dg2 <= 0.0 || du2 <= 0.0)) alpha = fmin(amax, fmax(amin, sqrt(du2 / dg2) * gmax));
  const double a1 = 0.5 * (1.0 + sqrt(4.0 * a * a + 1.0));
  st[12] = gmax > 0.0 ? alpha / gmax : 0.0;
  st[13] = (a - 1.0) / a1;
  const double rel = k - st[14];
  if (log && rel >= 0.0 && rel < (double)log_cap) {
    double* r = log + 8 * (long long)rel;
    r[0] = k;
    r[1] = N;
    r[2] = W;
    r[3] = H;
    r[4] = tau;
    r[5] = lam;
    r[6] = gamma;
    r[7] = alpha;
  }
  // the next iteration's parameters
  double na = a1, nlam = lam;
  const double namax = fmax(amax0, 2.0 * alpha);
  const double ngamma = 8.0 * bw * pow(10.0, 20.0 / 9.0 * (tau - 0.1) - 1.0);
  if (st[9] == 0.0) {
    const double every = st[10];
    if (every >= 1.0 && fmod(k + 1.0, every) == 0.0) {
      nlam = lam * 2.0;
      if (st[11] != 0.0) na = 1.0;
    }
  } else if (last_h == last_h) {   // not NaN: a previous HPWL exists
    const double mu = pow(1.1, 1.0 - (H - last_h) / 3.5e5);
    nlam = lam * fmin(1.1, fmax(0.75, mu));
  }
  st[0] = na;
  st[1] = namax;
  st[2] = 0.01 * namax;
  st[3] = nlam;
  st[4] = ngamma;
  st[5] = k + 1.0;
  st[6] = H;
  params[0] = (float)nlam;
  params[1] = (float)ngamma;
}

// Nonlinear conjugate gradients (the inner solver of Algorithm 1).
// Dots over both axes, per-block partials: [g.g, g.gp, gp.gp, g.d] (the
// previous gradient gp and the previous direction d may be null: zeros).
__global__ void __launch_bounds__(kStatThreads)
    k_cg_dots(int m, const float* __restrict__ gx, const float* __restrict__ gy,
              const float* __restrict__ gpx, const float* __restrict__ gpy,
              const float* __restrict__ dx, const float* __restrict__ dy,
              double* __restrict__ part) {
  double gg = 0.0, gq = 0.0, qq = 0.0, gd = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const double a = gx[i], b = gy[i];
    gg += a * a + b * b;
    if (gpx) {
      const double p = gpx[i], q = gpy[i];
      gq += a * p + b * q;
      qq += p * p + q * q;
    }
    if (dx) gd += a * (double)dx[i] + b * (double)dy[i];
  }
  block_sum_to<false>(gg, &part[blockIdx.x]);
  block_sum_to<false>(gq, &part[gridDim.x + blockIdx.x]);
  block_sum_to<false>(qq, &part[2 * gridDim.x + blockIdx.x]);
  block_sum_to<false>(gd, &part[3 * gridDim.x + blockIdx.x]);
}

// d = -g + beta d (beta = 0: d = -g, d read only otherwise); per-block max |d|.
__global__ void __launch_bounds__(kStatThreads)
    k_cg_direction(int m, const float* __restrict__ gx, const float* __restrict__ gy,
                   float beta, float* __restrict__ dx, float* __restrict__ dy,
                   double* __restrict__ part) {
  float dm = 0.0f;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const float a = beta != 0.0f ? beta * dx[i] - gx[i] : -gx[i];
    const float b = beta != 0.0f ? beta * dy[i] - gy[i] : -gy[i];
    dx[i] = a;
    dy[i] = b;
    dm = fmaxf(dm, fmaxf(fabsf(a), fabsf(b)));
  }
  __shared__ float wm[kStatThreads / kWave];
  dm = wave_max(dm);
  if ((threadIdx.x & (kWave - 1)) == 0) wm[threadIdx.x / kWave] = dm;
  __syncthreads();
  if (threadIdx.x == 0) {
    float v = 0.0f;
    for (int k = 0; k < kStatThreads / kWave; ++k) v = fmaxf(v, wm[k]);
    part[blockIdx.x] = v;
  }
}

// Fixed-order totals of `count` partial rows of nblk entries each; rows in
// max_mask take the maximum instead of the sum.
__global__ void __launch_bounds__(64)
    k_rows_final(const double* __restrict__ part, int nblk, int count, int max_mask,
                 double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j < count) {
    const bool mx = (max_mask >> j) & 1;
    double v = 0.0;
    for (int b = 0; b < nblk; ++b) {
      const double p = part[j * nblk + b];
      v = mx ? fmax(v, p) : v + p;
    }
    out[j] = v;
  }
}

// xo = clamp(x + t d), per cell and axis (xo may alias x).
__global__ void __launch_bounds__(256)
    k_cg_move(int m, const float* x, const float* y, const float* __restrict__ dx,
              const float* __restrict__ dy, float t,
              const float* __restrict__ w, const float* __restrict__ h, float xl, float yl,
              float xh, float yh, float* xo, float* yo) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const float hw = 0.5f * w[i], hh = 0.5f * h[i];
  const float nx = clampc(x[i] + t * dx[i], xl + hw, xh - hw);
  const float ny = clampc(y[i] + t * dy[i], yl + hh, yh - hh);
  xo[i] = nx;
  yo[i] = ny;
}

}  // namespace

size_t step_stats_work_doubles() { return 4 * (size_t)kStatBlocks; }

hipError_t launch_cg_dots(int m, const float* gx, const float* gy, const float* gpx,
                          const float* gpy, const float* dx, const float* dy, double* out,
                          double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dots, dim3(kStatBlocks), dim3(kStatThreads), 0, s, m, gx, gy, gpx,
                     gpy, dx, dy, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_final, dim3(1), dim3(64), 0, s, work, kStatBlocks, 4, 0, out);
  return hipGetLastError();
}

hipError_t launch_cg_direction(int m, const float* gx, const float* gy, float beta, float* dx,
                               float* dy, double* dmax, double* work, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_direction, dim3(kStatBlocks), dim3(kStatThreads), 0, s, m, gx, gy,
                     beta, dx, dy, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_rows_final, dim3(1), dim3(64), 0, s, work, kStatBlocks, 1, 1, dmax);
  return hipGetLastError();
}

hipError_t launch_cg_move(int m, const float* x, const float* y, const float* dx,
                          const float* dy, float t, const float* w, const float* h, float xl,
                          float yl, float xh, float yh, float* xo, float* yo, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cg_move, dim3((m + 255) / 256), dim3(256), 0, s, m, x, y, dx, dy, t, w,
                     h, xl, yl, xh, yh, xo, yo);
  return hipGetLastError();
}

hipError_t launch_step_stats(int m, const float* ux, const float* uy, const float* upx,
                             const float* upy, const float* gx, const float* gy,
                             const float* gpx, const float* gpy, double* out, double* work,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_step_stats, dim3(kStatBlocks), dim3(kStatThreads), 0, s, m, ux, uy,
                     upx, upy, gx, gy, gpx, gpy, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_step_stats_final, dim3(1), dim3(64), 0, s, work, kStatBlocks, out);
  return hipGetLastError();
}

hipError_t launch_nesterov_update(int m, float* x, float* y, float* ux, float* uy, float* upx,
                                  float* upy, float* gpx, float* gpy, const float* gx,
                                  const float* gy, const float* w, const float* h, float step,
                                  float beta, const double* step_beta, float xl, float yl,
                                  float xh, float yh, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nesterov_update, dim3((m + 255) / 256), dim3(256), 0, s, m, x, y, ux,
                     uy, upx, upy, gpx, gpy, gx, gy, w, h, step, beta, step_beta, xl, yl, xh,
                     yh);
  return hipGetLastError();
}

hipError_t launch_nesterov_schedule(const double* stats, const double* out4, double* state,
                                    float* params, double* log, int log_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_nesterov_schedule, dim3(1), dim3(64), 0, s, stats, out4, state, params,
                     log, log_cap);
  return hipGetLastError();
}

}  // namespace fftpl
