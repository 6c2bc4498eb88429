// Weighted-average wirelength (Eq. (3)) gradient and HPWL (Eq. (1)) over the
// pin-net CSR.
//
// For each net and axis with pin coordinates X_p = x[cell_p] + dx_p, M = max,
// L = min, e+_p = exp((X_p - M)/gamma), e-_p = exp((L - X_p)/gamma):
//   W+ = M + sum (X-M) e+ / sum e+,   W- = L + sum (X-L) e- / sum e-,
//   W~ = W+ - W-,
//   dW~/dX_p = e+_p/S+ (1 + (X_p - W+)/gamma) - e-_p/S- (1 - (X_p - W-)/gamma).
// Coordinates are taken relative to the first pin's cell centre, so float32
// keeps the small differences exact where the absolute positions (thousands
// of sites) would not.
//
// One thread per net for degree <= kSmallDeg (the bulk of every netlist);
// larger nets found in a wavefront are processed by the whole wavefront
// cooperatively, one after another.  Gradients go to the cells with float
// atomics; the W~ and HPWL totals are reduced in double.
#include <math.h>

#include "fftpl_internal.hpp"

namespace fftpl {

constexpr int kSmallDeg = 8;

__global__ void __launch_bounds__(256)
    k_wa(int num_nets, const int32_t* __restrict__ net_ptr,
         const int32_t* __restrict__ pin_cell, const float* __restrict__ pin_dx,
         const float* __restrict__ pin_dy, const float* __restrict__ x,
         const float* __restrict__ y, float inv_gamma, float* __restrict__ gx,
         float* __restrict__ gy, double* __restrict__ wa_out, double* __restrict__ hp_out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int p0 = 0, p1 = 0;
  if (e < num_nets) {
    p0 = net_ptr[e];
    p1 = net_ptr[e + 1];
  }
  const int deg = p1 - p0;
  double acc_wa = 0.0, acc_hp = 0.0;

  if (deg >= 2 && deg <= kSmallDeg) {
    int cell[kSmallDeg];
    float px[kSmallDeg], py[kSmallDeg];
    const int c0 = pin_cell[p0];
    const float x0 = x[c0], y0 = y[c0];
    float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k) {
      if (k < deg) {
        const int c = pin_cell[p0 + k];
        cell[k] = c;
        px[k] = (x[c] - x0) + pin_dx[p0 + k];
        py[k] = (y[c] - y0) + pin_dy[p0 + k];
        mx = fmaxf(mx, px[k]);
        lx = fminf(lx, px[k]);
        my = fmaxf(my, py[k]);
        ly = fminf(ly, py[k]);
      }
    }
    float spx = 0.f, tpx = 0.f, smx = 0.f, tmx = 0.f;
    float spy = 0.f, tpy = 0.f, smy = 0.f, tmy = 0.f;
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k) {
      if (k < deg) {
        float d = px[k] - mx, ee = expf(d * inv_gamma);
        spx += ee;
        tpx += d * ee;
        d = px[k] - lx;
        ee = expf(-d * inv_gamma);
        smx += ee;
        tmx += d * ee;
        d = py[k] - my;
        ee = expf(d * inv_gamma);
        spy += ee;
        tpy += d * ee;
        d = py[k] - ly;
        ee = expf(-d * inv_gamma);
        smy += ee;
        tmy += d * ee;
      }
    }
    // W+ - M and W- - L per axis
    const float wpx = tpx / spx, wmx = tmx / smx, wpy = tpy / spy, wmy = tmy / smy;
    const float rspx = 1.0f / spx, rsmx = 1.0f / smx, rspy = 1.0f / spy, rsmy = 1.0f / smy;
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k) {
      if (k < deg) {
        float dp = px[k] - mx, dm = px[k] - lx;
        float g = expf(dp * inv_gamma) * rspx * (1.0f + (dp - wpx) * inv_gamma) -
                  expf(-dm * inv_gamma) * rsmx * (1.0f - (dm - wmx) * inv_gamma);
        unsafeAtomicAdd(&gx[cell[k]], g);
        dp = py[k] - my;
        dm = py[k] - ly;
        g = expf(dp * inv_gamma) * rspy * (1.0f + (dp - wpy) * inv_gamma) -
            expf(-dm * inv_gamma) * rsmy * (1.0f - (dm - wmy) * inv_gamma);
        unsafeAtomicAdd(&gy[cell[k]], g);
      }
    }
    acc_wa = (double)((mx - lx) + wpx - wmx) + (double)((my - ly) + wpy - wmy);
    acc_hp = (double)(mx - lx) + (double)(my - ly);
  }

  // Larger nets: the whole wavefront cooperates on each in turn.
  unsigned long long big = __ballot(deg > kSmallDeg);
  while (big) {
    const int src = __ffsll((long long)big) - 1;
    big &= big - 1;
    const int b0 = __shfl(p0, src, kWave), b1 = __shfl(p1, src, kWave);
    const int c0 = pin_cell[b0];
    const float x0 = x[c0], y0 = y[c0];
    float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
    for (int p = b0 + lane; p < b1; p += kWave) {
      const int c = pin_cell[p];
      const float X = (x[c] - x0) + pin_dx[p], Y = (y[c] - y0) + pin_dy[p];
      mx = fmaxf(mx, X);
      lx = fminf(lx, X);
      my = fmaxf(my, Y);
      ly = fminf(ly, Y);
    }
    mx = wave_max(mx);
    lx = wave_min(lx);
    my = wave_max(my);
    ly = wave_min(ly);
    float spx = 0.f, tpx = 0.f, smx = 0.f, tmx = 0.f;
    float spy = 0.f, tpy = 0.f, smy = 0.f, tmy = 0.f;
    for (int p = b0 + lane; p < b1; p += kWave) {
      const int c = pin_cell[p];
      const float X = (x[c] - x0) + pin_dx[p], Y = (y[c] - y0) + pin_dy[p];
      float d = X - mx, ee = expf(d * inv_gamma);
      spx += ee;
      tpx += d * ee;
      d = X - lx;
      ee = expf(-d * inv_gamma);
      smx += ee;
      tmx += d * ee;
      d = Y - my;
      ee = expf(d * inv_gamma);
      spy += ee;
      tpy += d * ee;
      d = Y - ly;
      ee = expf(-d * inv_gamma);
      smy += ee;
      tmy += d * ee;
    }
    spx = wave_sum(spx);
    tpx = wave_sum(tpx);
    smx = wave_sum(smx);
    tmx = wave_sum(tmx);
    spy = wave_sum(spy);
    tpy = wave_sum(tpy);
    smy = wave_sum(smy);
    tmy = wave_sum(tmy);
    const float wpx = tpx / spx, wmx = tmx / smx, wpy = tpy / spy, wmy = tmy / smy;
    const float rspx = 1.0f / spx, rsmx = 1.0f / smx, rspy = 1.0f / spy, rsmy = 1.0f / smy;
    for (int p = b0 + lane; p < b1; p += kWave) {
      const int c = pin_cell[p];
      const float X = (x[c] - x0) + pin_dx[p], Y = (y[c] - y0) + pin_dy[p];
      float dp = X - mx, dm = X - lx;
      float g = expf(dp * inv_gamma) * rspx * (1.0f + (dp - wpx) * inv_gamma) -
                expf(-dm * inv_gamma) * rsmx * (1.0f - (dm - wmx) * inv_gamma);
      unsafeAtomicAdd(&gx[c], g);
      dp = Y - my;
      dm = Y - ly;
      g = expf(dp * inv_gamma) * rspy * (1.0f + (dp - wpy) * inv_gamma) -
          expf(-dm * inv_gamma) * rsmy * (1.0f - (dm - wmy) * inv_gamma);
      unsafeAtomicAdd(&gy[c], g);
    }
    if (lane == src) {
      acc_wa += (double)((mx - lx) + wpx - wmx) + (double)((my - ly) + wpy - wmy);
      acc_hp += (double)(mx - lx) + (double)(my - ly);
    }
  }
  if (wa_out) block_atomic_add(acc_wa, wa_out);
  if (hp_out) block_atomic_add(acc_hp, hp_out);
}

hipError_t launch_wa(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                     const float* pin_dx, const float* pin_dy, const float* x,
                     const float* y, float gamma, float* gx, float* gy,
                     double* wa_out, double* hp_out, hipStream_t s) {
  if (num_nets <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_wa, dim3((num_nets + 255) / 256), dim3(256), 0, s, num_nets,
                     net_ptr, pin_cell, pin_dx, pin_dy, x, y, 1.0f / gamma, gx, gy,
                     wa_out, hp_out);
  return hipGetLastError();
}

// out4[3] = tau = scal[0] / scal[1] (0 when there is no movable area).
__global__ void k_overflow_finalize(double* __restrict__ out4, const double* __restrict__ scal) {
  if (threadIdx.x == 0 && blockIdx.x == 0) out4[3] = scal[1] > 0.0 ? scal[0] / scal[1] : 0.0;
}

hipError_t launch_overflow_finalize(double* out4, const double* scal, hipStream_t s) {
  hipLaunchKernelGGL(k_overflow_finalize, dim3(1), dim3(64), 0, s, out4, scal);
  return hipGetLastError();
}

}  // namespace fftpl
