// Bin-grid kernels: map fill, fixed-charge rasterisation, the movable-cell
// density scatter (Eq. (2), Section III-B) and the field gather that turns
// E or psi back into per-cell density gradients (Section III-C).
#include "fftpl_internal.hpp"

namespace fftpl {

GridF make_gridf(const fftpl_grid& g) {
  GridF f;
  f.n = g.n;
  f.xl = (float)g.xl;
  f.yl = (float)g.yl;
  f.inv_bw = (float)(1.0 / g.bin_w);
  f.inv_bh = (float)(1.0 / g.bin_h);
  f.bin_w = (float)g.bin_w;
  f.bin_h = (float)g.bin_h;
  f.rho_t = (float)g.target_density;
  return f;
}

// dst[i] = src ? src[i] : value
__global__ void k_fill(float* __restrict__ dst, const float* __restrict__ src,
                       float value, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < count; i += stride) dst[i] = src ? src[i] : value;
}

__global__ void k_fill_f64(double* __restrict__ dst, double value, int count) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) dst[i] = value;
}

hipError_t launch_fill(float* dst, const float* src, float value, int64_t count,
                       hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, s, dst, src, value,
                     count);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* dst, double value, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_f64, dim3((count + 63) / 64), dim3(64), 0, s, dst, value,
                     count);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fixed charge: one block per rectangle accumulates its overlap f_b, then a
// pointwise pass scales by rho_t and derives the movable capacity.
// ---------------------------------------------------------------------------
__global__ void k_fixed_cover(GridF g, const float* __restrict__ fx,
                              const float* __restrict__ fy, const float* __restrict__ fw,
                              const float* __restrict__ fh, float* __restrict__ cover) {
  const int i = blockIdx.x;
  const Span sx = cell_span(fx[i], fw[i], g.xl, g.inv_bw, g.n);
  const Span sy = cell_span(fy[i], fh[i], g.yl, g.inv_bh, g.n);
  if (sx.i0 > sx.i1 || sy.i0 > sy.i1) return;
  const int nx = sx.i1 - sx.i0 + 1;
  const int ny = sy.i1 - sy.i0 + 1;
  const int64_t total = (int64_t)nx * ny;
  for (int64_t t = threadIdx.x; t < total; t += blockDim.x) {
    const int ix = sx.i0 + (int)(t % nx);
    const int iy = sy.i0 + (int)(t / nx);
    const float ov = span_overlap(sx, ix) * span_overlap(sy, iy);
    atomicAdd(&cover[(int64_t)iy * g.n + ix], ov);
  }
}

__global__ void k_fixed_finalize(float* __restrict__ base, float* __restrict__ cap,
                                 float rho_t, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float f = base[i];
  base[i] = rho_t * f;
  if (cap) cap[i] = rho_t * fmaxf(0.0f, 1.0f - fminf(1.0f, f));
}

hipError_t launch_fixed_map(const GridF& g, int num_fixed, const float* fx,
                            const float* fy, const float* fw, const float* fh,
                            float* base, float* cap, hipStream_t s) {
  const int64_t nn = (int64_t)g.n * g.n;
  hipError_t e = launch_fill(base, nullptr, 0.0f, nn, s);
  if (e != hipSuccess) return e;
  if (num_fixed > 0) {
    hipLaunchKernelGGL(k_fixed_cover, dim3(num_fixed), dim3(256), 0, s, g, fx, fy, fw,
                       fh, base);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_fixed_finalize, dim3((unsigned)((nn + 255) / 256)), dim3(256), 0,
                     s, base, cap, g.rho_t, nn);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Movable-cell scatter: one thread per cell adds ox*oy into every bin of its
// span with float atomics on the n*n map (4 MB at n = 1024, cache resident).
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scatter(GridF g, int m, const float* __restrict__ x,
                                                 const float* __restrict__ y,
                                                 const float* __restrict__ w,
                                                 const float* __restrict__ h,
                                                 float* __restrict__ rho) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const Span sx = cell_span(x[i], w[i], g.xl, g.inv_bw, g.n);
  const Span sy = cell_span(y[i], h[i], g.yl, g.inv_bh, g.n);
  for (int iy = sy.i0; iy <= sy.i1; ++iy) {
    const float oy = span_overlap(sy, iy);
    float* row = rho + (int64_t)iy * g.n;
    for (int ix = sx.i0; ix <= sx.i1; ++ix) {
      unsafeAtomicAdd(&row[ix], span_overlap(sx, ix) * oy);
    }
  }
}

hipError_t launch_scatter(const GridF& g, int m, const float* x, const float* y,
                          const float* w, const float* h, float* rho, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scatter, dim3((m + 255) / 256), dim3(256), 0, s, g, m, x, y, w, h,
                     rho);
  return hipGetLastError();
}

// Zero the per-evaluation scalars and the band counters in one launch.
__global__ void k_init_eval(double* __restrict__ out4, int32_t* __restrict__ counters,
                            int ncount) {
  const int t = threadIdx.x;
  if (t < 4) out4[t] = 0.0;
  if (counters)
    for (int k = t; k < ncount; k += blockDim.x) counters[k] = 0;
}

hipError_t launch_init_eval(double* out4, int32_t* counters, int ncount, hipStream_t s) {
  hipLaunchKernelGGL(k_init_eval, dim3(1), dim3(256), 0, s, out4, counters, ncount);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Field gather.  FIELD: g = -scale/bin * sum ov * E (E separate or
// interleaved).  EXACT: g = 2*scale/bin * sum_other-axis ov *
// [psi at right edge - psi at left edge] for edges strictly inside (0, n).
// ---------------------------------------------------------------------------
// PINS: 0 density gradient only; 1 plus the sum of the cell's contiguous pin
// slots (cell_ptr, pin_grad).
constexpr int kGatherThreads = 256;

template <int MODE, bool INTERLEAVED, int PINS>
__global__ void __launch_bounds__(kGatherThreads)
    k_gather(GridF g, int m, const float* __restrict__ x, const float* __restrict__ y,
             const float* __restrict__ w, const float* __restrict__ h,
             const float* __restrict__ ex, const float* __restrict__ ey,
             const float2* __restrict__ exy, const float* __restrict__ psi, float scale,
             int accumulate, const int32_t* __restrict__ cell_ptr,
             const float2* __restrict__ pin_grad, float* __restrict__ gx,
             float* __restrict__ gy) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) {
    // the cell's own loads go out together, before the map reads that
    // depend on them
    const float xi = x[i], yi = y[i], wi = w[i], hi = h[i];
    const float2 d =
        cell_density_grad<MODE, INTERLEAVED>(g, xi, yi, wi, hi, ex, ey, exy, psi);
    float ax = scale * d.x, ay = scale * d.y;
    if (PINS == 1) {
      // the cell's wirelength gradient: its pins' slots are contiguous
      const int k1 = cell_ptr[i + 1];
      for (int k = cell_ptr[i]; k < k1; ++k) {
        const float2 q = pin_grad[k];
        ax += q.x;
        ay += q.y;
      }
    }
    if (accumulate) {
      gx[i] += ax;
      gy[i] += ay;
    } else {
      gx[i] = ax;
      gy[i] = ay;
    }
  }
}

hipError_t launch_gather(const GridF& g, int m, const float* x, const float* y,
                         const float* w, const float* h, const float* ex,
                         const float* ey, const float* exy, const float* psi,
                         int grad_mode, float scale, int accumulate, float* gx,
                         float* gy, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  dim3 grid((m + kGatherThreads - 1) / kGatherThreads), block(kGatherThreads);
  const float2* e2 = reinterpret_cast<const float2*>(exy);
  if (grad_mode == FFTPL_GRAD_EXACT && exy) {
    // difference maps (Dx, Dy) in exy, psi for cells at the border
    hipLaunchKernelGGL((k_gather<FFTPL_GRAD_EXACT, true, 0>), grid, block, 0, s, g, m, x, y,
                       w, h, ex, ey, e2, psi, scale, accumulate, nullptr, nullptr, gx, gy);
  } else if (grad_mode == FFTPL_GRAD_EXACT) {
    hipLaunchKernelGGL((k_gather<FFTPL_GRAD_EXACT, false, 0>), grid, block, 0, s, g, m, x, y,
                       w, h, ex, ey, e2, psi, scale, accumulate, nullptr, nullptr, gx, gy);
  } else if (exy) {
    hipLaunchKernelGGL((k_gather<FFTPL_GRAD_FIELD, true, 0>), grid, block, 0, s, g, m, x, y,
                       w, h, ex, ey, e2, psi, scale, accumulate, nullptr, nullptr, gx, gy);
  } else {
    hipLaunchKernelGGL((k_gather<FFTPL_GRAD_FIELD, false, 0>), grid, block, 0, s, g, m, x, y,
                       w, h, ex, ey, e2, psi, scale, accumulate, nullptr, nullptr, gx, gy);
  }
  return hipGetLastError();
}

hipError_t launch_gather_pins(const GridF& g, int m, const float* x, const float* y,
                              const float* w, const float* h, const float* exy,
                              const float* psi, int grad_mode, float scale,
                              const int32_t* cell_ptr, const float2* pin_grad, float* gx,
                              float* gy, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  dim3 grid((m + kGatherThreads - 1) / kGatherThreads), block(kGatherThreads);
  const float2* e2 = reinterpret_cast<const float2*>(exy);
  if (grad_mode == FFTPL_GRAD_EXACT) {
    hipLaunchKernelGGL((k_gather<FFTPL_GRAD_EXACT, true, 1>), grid, block, 0, s, g, m, x,
                       y, w, h, nullptr, nullptr, e2, psi, scale, 0, cell_ptr, pin_grad, gx, gy);
  } else {
    hipLaunchKernelGGL((k_gather<FFTPL_GRAD_FIELD, true, 1>), grid, block, 0, s, g, m, x,
                       y, w, h, nullptr, nullptr, e2, psi, scale, 0, cell_ptr, pin_grad, gx, gy);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Test export: the integer span of every cell.
// ---------------------------------------------------------------------------
__global__ void k_cell_bins(GridF g, int m, const float* __restrict__ x,
                            const float* __restrict__ y, const float* __restrict__ w,
                            const float* __restrict__ h, int32_t* __restrict__ ranges) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const Span sx = cell_span(x[i], w[i], g.xl, g.inv_bw, g.n);
  const Span sy = cell_span(y[i], h[i], g.yl, g.inv_bh, g.n);
  int32_t* r = ranges + 4 * (int64_t)i;
  r[0] = sx.i0;
  r[1] = sx.i1;
  r[2] = sy.i0;
  r[3] = sy.i1;
}

hipError_t launch_cell_bins(const GridF& g, int m, const float* x, const float* y,
                            const float* w, const float* h, int32_t* ranges,
                            hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cell_bins, dim3((m + 255) / 256), dim3(256), 0, s, g, m, x, y, w, h,
                     ranges);
  return hipGetLastError();
}

}  // namespace fftpl
