// Weighted-average wirelength (Eq. (3)) gradient and HPWL (Eq. (1)) over the
// pin-net CSR (or, on request, the log-sum-exp model named in Section II).
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
// cooperatively, one after another.  The W~ and HPWL totals are reduced in
// double.  Three ways to hand the per-pin gradients to the cells:
//   ATOMIC: float atomics into gx, gy (the float-atomic evaluation path; each
//           atomic costs about as much as a random cache-line transfer, two
//           per pin);
//   FIXED:  64-bit integer atomics of the gradients in fixed point (units of
//           2^-32, exact for every component of magnitude >= 2^-9) into
//           per-cell accumulators, converted once per cell: the sums do not
//           depend on the order of the adds (the stateless calls);
//   SLOTS:  each pin's (gx, gy) is stored at its slot in a cell-major copy of
//           the pins (one random 8-byte write per pin); the cell pass then sums
//           contiguous slots.  Positions come interleaved as float2 so the
//           gather is one random read per pin.
#include <math.h>

#include "fftpl_internal.hpp"

namespace fftpl {

constexpr int kSmallDeg = 8;
constexpr int kBigRegs = 16;   // pins per lane kept in registers for one wave's net

constexpr int kIoAtomic = 0, kIoSlots = 1, kIoFixed = 2;
constexpr float kFixScale = 4294967296.0f;   // 2^32
constexpr float kFixLimit = 1073741824.0f;   // 2^30: far above any pin gradient

template <int IO>
struct PinIO {
  const float* x;
  const float* y;
  const float2* xy;
  const int32_t* slot;
  float* gx;
  float* gy;
  float2* pin_grad;
  unsigned long long* fx = nullptr;   // FIXED: per-cell sums (2^-32 units)
  unsigned long long* fy = nullptr;
  unsigned int* bad = nullptr;        // FIXED: a non-finite (or absurd) pin gradient
  __device__ __forceinline__ float2 pos(int c) const {
    if (IO == kIoSlots) return xy[c];
    return make_float2(x[c], y[c]);
  }
  __device__ __forceinline__ void put(int p, int c, float vx, float vy) const {
    if (IO == kIoSlots) {
      pin_grad[slot[p]] = make_float2(vx, vy);
    } else if (IO == kIoFixed) {
      if (fabsf(vx) <= kFixLimit && fabsf(vy) <= kFixLimit) {
        atomicAdd(&fx[c], (unsigned long long)__float2ll_rn(vx * kFixScale));
        atomicAdd(&fy[c], (unsigned long long)__float2ll_rn(vy * kFixScale));
      } else {
        atomicOr(&bad[c], 1u);
      }
    } else {
      unsafeAtomicAdd(&gx[c], vx);
      unsafeAtomicAdd(&gy[c], vy);
    }
  }
};

// PART 0: nets of degree <= kSmallDeg; 1: larger nets.  LSE: the log-sum-exp
// model instead of the weighted average (same sums, pin_wl_grad / net_wl_value).
template <int IO, int PART, bool LSE>
__global__ void __launch_bounds__(256)
    k_wa(int num_nets, const int32_t* __restrict__ net_ptr,
         const int32_t* __restrict__ pin_cell, const float* __restrict__ pin_dx,
         const float* __restrict__ pin_dy, PinIO<IO> io, float gamma, float inv_gamma,
         double* __restrict__ wa_out, double* __restrict__ hp_out,
         double* __restrict__ part) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int lane = threadIdx.x & (kWave - 1);
  int p0 = 0, p1 = 0;
  if (PART == 0 && e < num_nets) {
    p0 = net_ptr[e];
    p1 = net_ptr[e + 1];
  }
  const int deg = p1 - p0;
  double acc_wa = 0.0, acc_hp = 0.0;

  if (PART == 0 && deg >= 2 && deg <= kSmallDeg) {
    int cell[kSmallDeg];
    float px[kSmallDeg], py[kSmallDeg];
    // all loads first (independent), positions relative to the first pin's cell
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k)
      if (k < deg) cell[k] = pin_cell[p0 + k];
    float2 q[kSmallDeg];
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k)
      if (k < deg) q[k] = io.pos(cell[k]);
    float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k) {
      if (k < deg) {
        px[k] = (q[k].x - q[0].x) + pin_dx[p0 + k];
        py[k] = (q[k].y - q[0].y) + pin_dy[p0 + k];
        mx = fmaxf(mx, px[k]);
        lx = fminf(lx, px[k]);
        my = fmaxf(my, py[k]);
        ly = fminf(ly, py[k]);
      }
    }
    AxisSums sx = {0.f, 0.f, 0.f, 0.f}, sy = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k) {
      if (k < deg) {
        axis_accum(sx, px[k], mx, lx, inv_gamma);
        axis_accum(sy, py[k], my, ly, inv_gamma);
      }
    }
    const float wpx = sx.tp / sx.sp, wmx = sx.tm / sx.sm;
    const float wpy = sy.tp / sy.sp, wmy = sy.tm / sy.sm;
    const float rspx = 1.0f / sx.sp, rsmx = 1.0f / sx.sm;
    const float rspy = 1.0f / sy.sp, rsmy = 1.0f / sy.sm;
#pragma unroll
    for (int k = 0; k < kSmallDeg; ++k) {
      if (k < deg) {
        io.put(p0 + k, cell[k], pin_wl_grad<LSE>(px[k], mx, lx, wpx, wmx, rspx, rsmx, inv_gamma),
               pin_wl_grad<LSE>(py[k], my, ly, wpy, wmy, rspy, rsmy, inv_gamma));
      }
    }
    acc_wa = net_wl_value<LSE>(mx, lx, wpx, wmx, sx.sp, sx.sm, gamma) +
             net_wl_value<LSE>(my, ly, wpy, wmy, sy.sp, sy.sm, gamma);
    acc_hp = (double)(mx - lx) + (double)(my - ly);
  } else if (IO == kIoSlots && PART == 0 && deg == 1) {
    io.put(p0, 0, 0.0f, 0.0f);   // a one-pin net has no wirelength: its slot holds zero
  }

  // Larger nets: the whole wavefront cooperates on each in turn.  This part
  // runs on a persistent grid (every wavefront walks chunks of kWave nets), so
  // a few slow nets do not hold back the dispatch of thousands of blocks.
  const int wid = (blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int nwaves = gridDim.x * blockDim.x / kWave;
  const int nchunks = PART == 1 ? (num_nets + kWave - 1) / kWave : 0;
  for (int ch = wid; ch < nchunks; ch += nwaves) {
  const int ec = ch * kWave + lane;
  int c0 = 0, c1 = 0;
  if (ec < num_nets) {
    c0 = net_ptr[ec];
    c1 = net_ptr[ec + 1];
  }
  unsigned long long big = __ballot(c1 - c0 > kSmallDeg);
  while (big) {
    const int src = __ffsll((long long)big) - 1;
    big &= big - 1;
    const int b0 = __shfl(c0, src, kWave), b1 = __shfl(c1, src, kWave);
    if (b1 - b0 <= kWave * kBigRegs) {
      // up to kBigRegs pins per lane held in registers: one pass over memory
      int cj[kBigRegs];
      float2 q[kBigRegs];
#pragma unroll
      for (int j = 0; j < kBigRegs; ++j) {
        const int p = b0 + lane + kWave * j;
        if (p < b1) cj[j] = pin_cell[p];
      }
#pragma unroll
      for (int j = 0; j < kBigRegs; ++j) {
        const int p = b0 + lane + kWave * j;
        if (p < b1) q[j] = io.pos(cj[j]);
      }
      const float rx = __shfl(q[0].x, 0, kWave), ry = __shfl(q[0].y, 0, kWave);
      float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
#pragma unroll
      for (int j = 0; j < kBigRegs; ++j) {
        const int p = b0 + lane + kWave * j;
        if (p < b1) {
          q[j].x = (q[j].x - rx) + pin_dx[p];
          q[j].y = (q[j].y - ry) + pin_dy[p];
          mx = fmaxf(mx, q[j].x);
          lx = fminf(lx, q[j].x);
          my = fmaxf(my, q[j].y);
          ly = fminf(ly, q[j].y);
        }
      }
      mx = wave_max(mx);
      lx = wave_min(lx);
      my = wave_max(my);
      ly = wave_min(ly);
      AxisSums sx = {0.f, 0.f, 0.f, 0.f}, sy = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int j = 0; j < kBigRegs; ++j) {
        if (b0 + lane + kWave * j < b1) {
          axis_accum(sx, q[j].x, mx, lx, inv_gamma);
          axis_accum(sy, q[j].y, my, ly, inv_gamma);
        }
      }
      sx.sp = wave_sum(sx.sp);
      sx.tp = wave_sum(sx.tp);
      sx.sm = wave_sum(sx.sm);
      sx.tm = wave_sum(sx.tm);
      sy.sp = wave_sum(sy.sp);
      sy.tp = wave_sum(sy.tp);
      sy.sm = wave_sum(sy.sm);
      sy.tm = wave_sum(sy.tm);
      const float wpx = sx.tp / sx.sp, wmx = sx.tm / sx.sm;
      const float wpy = sy.tp / sy.sp, wmy = sy.tm / sy.sm;
      const float rspx = 1.0f / sx.sp, rsmx = 1.0f / sx.sm;
      const float rspy = 1.0f / sy.sp, rsmy = 1.0f / sy.sm;
#pragma unroll
      for (int j = 0; j < kBigRegs; ++j) {
        const int p = b0 + lane + kWave * j;
        if (p < b1)
          io.put(p, cj[j], pin_wl_grad<LSE>(q[j].x, mx, lx, wpx, wmx, rspx, rsmx, inv_gamma),
                 pin_wl_grad<LSE>(q[j].y, my, ly, wpy, wmy, rspy, rsmy, inv_gamma));
      }
      if (lane == src) {
        acc_wa += net_wl_value<LSE>(mx, lx, wpx, wmx, sx.sp, sx.sm, gamma) +
                  net_wl_value<LSE>(my, ly, wpy, wmy, sy.sp, sy.sm, gamma);
        acc_hp += (double)(mx - lx) + (double)(my - ly);
      }
      continue;
    }
    // nets beyond the register capacity: three passes over the pins
    const float2 r = io.pos(pin_cell[b0]);
    float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
    for (int p = b0 + lane; p < b1; p += kWave) {
      const float2 q = io.pos(pin_cell[p]);
      const float X = (q.x - r.x) + pin_dx[p], Y = (q.y - r.y) + pin_dy[p];
      mx = fmaxf(mx, X);
      lx = fminf(lx, X);
      my = fmaxf(my, Y);
      ly = fminf(ly, Y);
    }
    mx = wave_max(mx);
    lx = wave_min(lx);
    my = wave_max(my);
    ly = wave_min(ly);
    AxisSums sx = {0.f, 0.f, 0.f, 0.f}, sy = {0.f, 0.f, 0.f, 0.f};
    for (int p = b0 + lane; p < b1; p += kWave) {
      const float2 q = io.pos(pin_cell[p]);
      axis_accum(sx, (q.x - r.x) + pin_dx[p], mx, lx, inv_gamma);
      axis_accum(sy, (q.y - r.y) + pin_dy[p], my, ly, inv_gamma);
    }
    sx.sp = wave_sum(sx.sp);
    sx.tp = wave_sum(sx.tp);
    sx.sm = wave_sum(sx.sm);
    sx.tm = wave_sum(sx.tm);
    sy.sp = wave_sum(sy.sp);
    sy.tp = wave_sum(sy.tp);
    sy.sm = wave_sum(sy.sm);
    sy.tm = wave_sum(sy.tm);
    const float wpx = sx.tp / sx.sp, wmx = sx.tm / sx.sm;
    const float wpy = sy.tp / sy.sp, wmy = sy.tm / sy.sm;
    const float rspx = 1.0f / sx.sp, rsmx = 1.0f / sx.sm;
    const float rspy = 1.0f / sy.sp, rsmy = 1.0f / sy.sm;
    for (int p = b0 + lane; p < b1; p += kWave) {
      const int c = pin_cell[p];
      const float2 q = io.pos(c);
      const float X = (q.x - r.x) + pin_dx[p], Y = (q.y - r.y) + pin_dy[p];
      io.put(p, c, pin_wl_grad<LSE>(X, mx, lx, wpx, wmx, rspx, rsmx, inv_gamma),
             pin_wl_grad<LSE>(Y, my, ly, wpy, wmy, rspy, rsmy, inv_gamma));
    }
    if (lane == src) {
      acc_wa += net_wl_value<LSE>(mx, lx, wpx, wmx, sx.sp, sx.sm, gamma) +
                net_wl_value<LSE>(my, ly, wpy, wmy, sy.sp, sy.sm, gamma);
      acc_hp += (double)(mx - lx) + (double)(my - ly);
    }
  }
  }
  if (part) {
    // per-block partials: part[b] = W~, part[gridDim.x + b] = HPWL
    block_sum_to<false>(acc_wa, &part[blockIdx.x]);
    block_sum_to<false>(acc_hp, &part[gridDim.x + blockIdx.x]);
  } else {
    if (wa_out) block_atomic_add(acc_wa, wa_out);
    if (hp_out) block_atomic_add(acc_hp, hp_out);
  }
}

template <int IO, bool LSE>
hipError_t launch_wa_parts(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                           const float* pin_dx, const float* pin_dy, PinIO<IO> io,
                           float gamma, double* wa_out, double* hp_out, double* part,
                           hipStream_t s, Plan* tp) {
  const int nblk = (num_nets + 255) / 256;
  hipLaunchKernelGGL((k_wa<IO, 0, LSE>), dim3(nblk), dim3(256), 0, s, num_nets, net_ptr,
                     pin_cell, pin_dx, pin_dy, io, gamma, 1.0f / gamma, wa_out, hp_out, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (tp) plan_mark(*tp, "k_wa_slots_small", s);
  hipLaunchKernelGGL((k_wa<IO, 1, LSE>), dim3(wa_big_grid(num_nets)), dim3(256), 0, s,
                     num_nets, net_ptr, pin_cell, pin_dx, pin_dy, io, gamma, 1.0f / gamma,
                     wa_out, hp_out, part ? part + 2 * (size_t)nblk : nullptr);
  e = hipGetLastError();
  if (tp) plan_mark(*tp, "k_wa_slots_big", s);
  return e;
}

hipError_t launch_wa(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                     const float* pin_dx, const float* pin_dy, const float* x,
                     const float* y, float gamma, int wl_model, float* gx, float* gy,
                     double* wa_out, double* hp_out, hipStream_t s) {
  if (num_nets <= 0) return hipSuccess;
  PinIO<kIoAtomic> io{x, y, nullptr, nullptr, gx, gy, nullptr};
  return wl_model == FFTPL_WL_LSE
             ? launch_wa_parts<kIoAtomic, true>(num_nets, net_ptr, pin_cell, pin_dx, pin_dy,
                                                io, gamma, wa_out, hp_out, nullptr, s, nullptr)
             : launch_wa_parts<kIoAtomic, false>(num_nets, net_ptr, pin_cell, pin_dx, pin_dy,
                                                 io, gamma, wa_out, hp_out, nullptr, s, nullptr);
}

// Per cell: the fixed-point sums back to float (NaN for a cell that had a
// non-finite pin gradient), written or added to gx, gy.
__global__ void __launch_bounds__(256)
    k_fix_cells(int m, const unsigned long long* __restrict__ fx,
                const unsigned long long* __restrict__ fy, const unsigned int* __restrict__ bad,
                int accumulate, float* __restrict__ gx, float* __restrict__ gy) {
  constexpr double unit = 1.0 / 4294967296.0;
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < m; c += gridDim.x * blockDim.x) {
    const bool b = bad[c] != 0u;
    const float vx = b ? __builtin_nanf("") : (float)((double)(long long)fx[c] * unit);
    const float vy = b ? __builtin_nanf("") : (float)((double)(long long)fy[c] * unit);
    gx[c] = accumulate ? gx[c] + vx : vx;
    gy[c] = accumulate ? gy[c] + vy : vy;
  }
}

size_t wa_fixed_work_bytes(int num_cells, int num_nets) {
  const size_t parts = 2 * ((size_t)(num_nets + 255) / 256 + (size_t)wa_big_grid(num_nets));
  return 16 * (size_t)num_cells + 4 * (size_t)num_cells + 8 * parts + 256;
}

hipError_t launch_wa_fixed(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                           const float* pin_dx, const float* pin_dy, int num_cells,
                           const float* x, const float* y, float gamma, int wl_model,
                           int accumulate, float* gx, float* gy, double* wa_out,
                           double* hp_out, void* work, hipStream_t s) {
  // work: fx, fy [m] (u64), W~/HPWL partials, bad [m] (u32), cleared first
  char* w = static_cast<char*>(work);
  unsigned long long* fx = reinterpret_cast<unsigned long long*>(w);
  unsigned long long* fy = fx + num_cells;
  double* part = reinterpret_cast<double*>(fy + num_cells);
  const int nblk = (num_nets + 255) / 256, nbig = wa_big_grid(num_nets);
  unsigned int* bad = reinterpret_cast<unsigned int*>(part + 2 * ((size_t)nblk + nbig));
  const int64_t words = (16 * (int64_t)num_cells + 4 * (int64_t)num_cells) / 4 +
                        4 * ((int64_t)nblk + nbig);
  hipError_t e = launch_zero_i32(reinterpret_cast<int32_t*>(work), words, s);
  if (e != hipSuccess) return e;
  PinIO<kIoFixed> io{x, y, nullptr, nullptr, nullptr, nullptr, nullptr, fx, fy, bad};
  e = wl_model == FFTPL_WL_LSE
          ? launch_wa_parts<kIoFixed, true>(num_nets, net_ptr, pin_cell, pin_dx, pin_dy, io,
                                            gamma, nullptr, nullptr, part, s, nullptr)
          : launch_wa_parts<kIoFixed, false>(num_nets, net_ptr, pin_cell, pin_dx, pin_dy, io,
                                             gamma, nullptr, nullptr, part, s, nullptr);
  if (e != hipSuccess) return e;
  if (num_cells > 0) {
    int blocks = (num_cells + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fix_cells, dim3(blocks), dim3(256), 0, s, num_cells, fx, fy, bad,
                       accumulate, gx, gy);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  // the totals from the per-block partials in a fixed order
  if (wa_out || hp_out)
    e = launch_eval_finalize(nullptr, 0, nullptr, 0, part, nblk, nbig, nullptr, wa_out, hp_out,
                             nullptr, s);
  return e;
}

hipError_t launch_wa_pins(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                          const float* pin_dx, const float* pin_dy, const float2* xy,
                          const int32_t* pin_slot, float gamma, int wl_model,
                          float2* pin_grad, double* wa_part, hipStream_t s, Plan* tp) {
  if (num_nets <= 0) return hipSuccess;
  PinIO<kIoSlots> io{nullptr, nullptr, xy, pin_slot, nullptr, nullptr, pin_grad};
  return wl_model == FFTPL_WL_LSE
             ? launch_wa_parts<kIoSlots, true>(num_nets, net_ptr, pin_cell, pin_dx, pin_dy, io,
                                               gamma, nullptr, nullptr, wa_part, s, tp)
             : launch_wa_parts<kIoSlots, false>(num_nets, net_ptr, pin_cell, pin_dx, pin_dy,
                                                io, gamma, nullptr, nullptr, wa_part, s, tp);
}

// The evaluation's scalars (FinalArgs) by one block, when no gather runs.
constexpr int kFinalThreads = 1024;

__global__ void __launch_bounds__(kFinalThreads) k_eval_finalize(FinalArgs f) {
  eval_scalars<kFinalThreads>(f);
}

hipError_t launch_eval_finalize(const double* en, int n_en, const double* tau, int n_tau,
                                const double* wa, int n_s, int n_b, double* o_en, double* o_wa,
                                double* o_hp, double* o_tau, hipStream_t s) {
  FinalArgs f;
  f.en = en;
  f.n_en = n_en;
  f.tau = tau;
  f.n_tau = n_tau;
  f.wa = wa;
  f.n_s = wa ? n_s : 0;
  f.n_b = wa ? n_b : 0;
  f.o_en = o_en;
  f.o_wa = o_wa;
  f.o_hp = o_hp;
  f.o_tau = o_tau;
  hipLaunchKernelGGL(k_eval_finalize, dim3(1), dim3(kFinalThreads), 0, s, f);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cell-major pin index (built once per netlist): cell_ptr = exclusive prefix
// sum of the pin count of every cell, pin_slot[p] = position of pin p among
// the slots of its cell.  Ranks inside a cell come from integer atomics, so
// the order of a cell's slots is arbitrary but fixed once built.
// ---------------------------------------------------------------------------
__global__ void k_zero_i32(int32_t* __restrict__ a, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x)
    a[i] = 0;
}

__global__ void k_count_pins(int num_pins, const int32_t* __restrict__ pin_cell,
                             int32_t* __restrict__ cnt) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < num_pins) atomicAdd(&cnt[pin_cell[p]], 1);
}

// Block-local exclusive scan of 1024 items (4 per thread); block totals out.
__global__ void __launch_bounds__(256)
    k_scan_blocks(const int32_t* __restrict__ in, int count, int32_t* __restrict__ out,
                  int32_t* __restrict__ sums) {
  const int base = blockIdx.x * 1024 + threadIdx.x * 4;
  int v[4], s = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = base + k < count ? in[base + k] : 0;
    s += v[k];
  }
  int total;
  int run = block_exclusive_scan256(s, &total);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (base + k < count) out[base + k] = run;
    run += v[k];
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of the block sums in place (one block, chunks of 256 with a
// running carry); the grand total goes to *total_out.
__global__ void __launch_bounds__(256)
    k_scan_sums(int32_t* __restrict__ sums, int nsums, int32_t* __restrict__ total_out) {
  int carry = 0;
  for (int c0 = 0; c0 < nsums; c0 += 256) {
    const int i = c0 + threadIdx.x;
    const int v = i < nsums ? sums[i] : 0;
    int tot;
    const int ex = block_exclusive_scan256(v, &tot);
    if (i < nsums) sums[i] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) *total_out = carry;
}

__global__ void k_scan_add(int32_t* __restrict__ out, int count, const int32_t* __restrict__ sums) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] += sums[i / 1024];
}

__global__ void k_pin_slots(int num_pins, const int32_t* __restrict__ pin_cell,
                            const int32_t* __restrict__ cell_ptr, int32_t* __restrict__ cursor,
                            int32_t* __restrict__ slot) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < num_pins) {
    const int c = pin_cell[p];
    slot[p] = cell_ptr[c] + atomicAdd(&cursor[c], 1);
  }
}

hipError_t launch_zero_i32(int32_t* a, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, a, (int)count);
  return hipGetLastError();
}

// out[i] = sum in[0..i) for i < count, *total = sum in[0..count); sums needs
// ceil(count/1024) ints.  in and out may be the same array.
hipError_t launch_exclusive_scan(const int32_t* in, int count, int32_t* out, int32_t* sums,
                                 int32_t* total, hipStream_t s) {
  const int nsb = (count + 1023) / 1024;
  hipError_t e = hipSuccess;
  if (count > 0) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(nsb), dim3(256), 0, s, in, count, out, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, nsb, total);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (count > 0) {
    hipLaunchKernelGGL(k_scan_add, dim3((count + 255) / 256), dim3(256), 0, s, out, count, sums);
    e = hipGetLastError();
  }
  return e;
}

hipError_t launch_netlist_index(int m, int num_pins, const int32_t* pin_cell,
                                int32_t* cell_ptr, int32_t* pin_slot, int32_t* work,
                                hipStream_t s) {
  // work: m counters followed by ceil(m/1024) block sums
  const int nsb = (m + 1023) / 1024;
  int32_t* sums = work + m;
  hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, work, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (num_pins > 0) {
    hipLaunchKernelGGL(k_count_pins, dim3((num_pins + 255) / 256), dim3(256), 0, s,
                       num_pins, pin_cell, work);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  if (m > 0) {
    hipLaunchKernelGGL(k_scan_blocks, dim3(nsb), dim3(256), 0, s, work, m, cell_ptr, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_scan_sums, dim3(1), dim3(256), 0, s, sums, nsb, cell_ptr + m);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (m > 0) {
    hipLaunchKernelGGL(k_scan_add, dim3((m + 255) / 256), dim3(256), 0, s, cell_ptr, m, sums);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_zero_i32, dim3(256), dim3(256), 0, s, work, m);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if (num_pins > 0) {
    hipLaunchKernelGGL(k_pin_slots, dim3((num_pins + 255) / 256), dim3(256), 0, s,
                       num_pins, pin_cell, cell_ptr, work, pin_slot);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace fftpl
