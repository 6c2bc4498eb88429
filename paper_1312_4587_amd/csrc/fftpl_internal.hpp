// Internal declarations shared by the HIP translation units of libfftpl.
// Device helpers: the float32 cell-rectangle rule, wave reductions and the
// XCD-aware block remap.  Host side: the plan layout and the launchers each
// translation unit exports to the C ABI layer.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/fftpl.h"

namespace fftpl {

constexpr int kWave = 64;
constexpr int kNumXcd = 8;   // MI355X: 256 CUs in 8 XCDs, blocks dealt round-robin

// ---------------------------------------------------------------------------
// Device helpers
// ---------------------------------------------------------------------------

// Float32 grid parameters as the kernels use them (origin, 1/bin size).
struct GridF {
  int n;
  float xl, yl;
  float inv_bw, inv_bh;   // fl32(1 / bin size), computed in double on the host
  float bin_w, bin_h;
  float rho_t;
};

// One axis of the cell-rectangle rule: edges in bin units (rounded once per
// operation, no contraction), the clipped edges, and the first/last bin.
struct Span {
  float lo, hi;     // unclipped edges in bin units
  float clo, chi;   // edges clipped to [0, n]
  int i0, i1;       // bins touched, empty when i0 > i1
};

// Clipped edges and bin range of the edges [lo, hi) in bin units.
__device__ __forceinline__ Span span_from_edges(float lo, float hi, int n) {
  Span s;
  s.lo = lo;
  s.hi = hi;
  const float fn = (float)n;
  s.clo = fminf(fmaxf(lo, 0.0f), fn);
  s.chi = fminf(fmaxf(hi, 0.0f), fn);
  s.i0 = (int)floorf(s.clo);
  s.i1 = (int)ceilf(fminf(fmaxf(hi, -1.0f), fn)) - 1;
  return s;
}

__device__ __forceinline__ Span cell_span(float centre, float size, float origin,
                                          float inv, int n) {
#pragma clang fp contract(off)
  const float c = (centre - origin) * inv;
  const float half = 0.5f * (size * inv);
  return span_from_edges(c - half, c + half, n);
}

// Overlap of the clipped edges [clo, chi) with bin j.
__device__ __forceinline__ float span_overlap(const Span& s, int j) {
  return fminf(s.chi, (float)(j + 1)) - fmaxf(s.clo, (float)j);
}

// Density gradient of one cell (Section III-C), before the factor lambda.
// FIELD: -1/bin * sum_b ov(i, b) E_b (E interleaved as (Ex, Ey) per bin, or
// two maps).  EXACT: dN/dx = 2/bin * sum over the other axis' overlaps of
// [psi at the right edge's bin - psi at the left edge's bin], for edges
// strictly inside (0, n) (an edge moving inside a bin moves area from the
// bin it leaves to the bin it enters); with INTERLEAVED and exy set, exy holds
// the difference maps (Dx, Dy) of the solve's difference mode and psi is read
// only for cells with one edge outside the region.
// density_grad_spans takes the cell's spans (from its geometry, or from the
// edges a band entry stores: the same Span either way).
template <int MODE, bool INTERLEAVED>
__device__ __forceinline__ float2 density_grad_spans(const GridF& g, const Span& sx,
                                                     const Span& sy,
                                                     const float* __restrict__ ex,
                                                     const float* __restrict__ ey,
                                                     const float2* __restrict__ exy,
                                                     const float* __restrict__ psi) {
  const int n = g.n;
  float ax = 0.0f, ay = 0.0f;
  if (MODE == FFTPL_GRAD_FIELD) {
    for (int iy = sy.i0; iy <= sy.i1; ++iy) {
      const float oy = span_overlap(sy, iy);
      for (int ix = sx.i0; ix <= sx.i1; ++ix) {
        const float ov = span_overlap(sx, ix) * oy;
        const int64_t b = (int64_t)iy * n + ix;
        if (INTERLEAVED) {
          const float2 e = exy[b];
          ax += ov * e.x;
          ay += ov * e.y;
        } else {
          ax += ov * ex[b];
          ay += ov * ey[b];
        }
      }
    }
    ax *= -g.inv_bw;
    ay *= -g.inv_bh;
  } else if (INTERLEAVED && exy) {
    // from the difference maps (Dx, Dy): with both edges inside, psi(right
    // edge's bin) - psi(left edge's bin) is the sum of Dx over the bins
    // between; with one edge inside, the single psi term
    const float fn = (float)n;
    const bool xr = sx.hi > 0.0f && sx.hi < fn, xl = sx.lo > 0.0f && sx.lo < fn;
    const bool yr = sy.hi > 0.0f && sy.hi < fn, yl = sy.lo > 0.0f && sy.lo < fn;
    const int cxr = xr ? (int)floorf(sx.hi) : 0, cxl = xl ? (int)floorf(sx.lo) : 0;
    const int cyr = yr ? (int)floorf(sy.hi) : 0, cyl = yl ? (int)floorf(sy.lo) : 0;
    for (int iy = sy.i0; iy <= sy.i1; ++iy) {
      const float oy = span_overlap(sy, iy);
      const int64_t row = (int64_t)iy * n;
      float d = 0.0f;
      if (xr && xl) {
        for (int c = cxl; c < cxr; ++c) d += exy[row + c].x;
      } else if (xr) {
        d = psi[row + cxr];
      } else if (xl) {
        d = -psi[row + cxl];
      }
      ax += oy * d;
    }
    for (int ix = sx.i0; ix <= sx.i1; ++ix) {
      const float ox = span_overlap(sx, ix);
      float d = 0.0f;
      if (yr && yl) {
        for (int r = cyl; r < cyr; ++r) d += exy[(int64_t)r * n + ix].y;
      } else if (yr) {
        d = psi[(int64_t)cyr * n + ix];
      } else if (yl) {
        d = -psi[(int64_t)cyl * n + ix];
      }
      ay += ox * d;
    }
    ax *= 2.0f * g.inv_bw;
    ay *= 2.0f * g.inv_bh;
  } else {
    // from psi alone (differences of psi values)
    const float fn = (float)n;
    const bool xr = sx.hi > 0.0f && sx.hi < fn, xl = sx.lo > 0.0f && sx.lo < fn;
    const bool yr = sy.hi > 0.0f && sy.hi < fn, yl = sy.lo > 0.0f && sy.lo < fn;
    const int cxr = xr ? (int)floorf(sx.hi) : 0, cxl = xl ? (int)floorf(sx.lo) : 0;
    const int cyr = yr ? (int)floorf(sy.hi) : 0, cyl = yl ? (int)floorf(sy.lo) : 0;
    for (int iy = sy.i0; iy <= sy.i1; ++iy) {
      const float oy = span_overlap(sy, iy);
      const float* row = psi + (int64_t)iy * n;
      float d = 0.0f;
      if (xr) d += row[cxr];
      if (xl) d -= row[cxl];
      ax += oy * d;
    }
    for (int ix = sx.i0; ix <= sx.i1; ++ix) {
      const float ox = span_overlap(sx, ix);
      float d = 0.0f;
      if (yr) d += psi[(int64_t)cyr * n + ix];
      if (yl) d -= psi[(int64_t)cyl * n + ix];
      ay += ox * d;
    }
    ax *= 2.0f * g.inv_bw;
    ay *= 2.0f * g.inv_bh;
  }
  return make_float2(ax, ay);
}

template <int MODE, bool INTERLEAVED>
__device__ __forceinline__ float2 cell_density_grad(const GridF& g, float x, float y, float w,
                                                    float h, const float* __restrict__ ex,
                                                    const float* __restrict__ ey,
                                                    const float2* __restrict__ exy,
                                                    const float* __restrict__ psi) {
  const Span sx = cell_span(x, w, g.xl, g.inv_bw, g.n);
  const Span sy = cell_span(y, h, g.yl, g.inv_bh, g.n);
  return density_grad_spans<MODE, INTERLEAVED>(g, sx, sy, ex, ey, exy, psi);
}

// ---- weighted-average wirelength, Eq. (3), per net and axis ----
// Per-axis sums of one net: S+ = sum e+, T+ = sum (X-M) e+, S-, T- likewise.
struct AxisSums {
  float sp, tp, sm, tm;
};

__device__ __forceinline__ void axis_accum(AxisSums& a, float X, float M, float L,
                                           float inv_gamma) {
  float d = X - M, ee = expf(d * inv_gamma);
  a.sp += ee;
  a.tp += d * ee;
  d = X - L;
  ee = expf(-d * inv_gamma);
  a.sm += ee;
  a.tm += d * ee;
}

// dW~/dX for one pin, given M, L and W+ - M = wp, W- - L = wm, 1/S+, 1/S-.
__device__ __forceinline__ float axis_grad(float X, float M, float L, float wp, float wm,
                                           float rsp, float rsm, float inv_gamma) {
  const float dp = X - M, dm = X - L;
  return expf(dp * inv_gamma) * rsp * (1.0f + (dp - wp) * inv_gamma) -
         expf(-dm * inv_gamma) * rsm * (1.0f - (dm - wm) * inv_gamma);
}

// The log-sum-exp model (Section II, the usual alternative to Eq. (3)) from
// the same shifted sums: per net and axis LSE = (M - L) + gamma (ln S+ +
// ln S-) and dLSE/dX = e+/S+ - e-/S-.  pin_wl_grad / net_wl_value pick the
// model: LSE = false is the weighted average of Eq. (3).
template <bool LSE>
__device__ __forceinline__ float pin_wl_grad(float X, float M, float L, float wp, float wm,
                                             float rsp, float rsm, float inv_gamma) {
  if (LSE) return expf((X - M) * inv_gamma) * rsp - expf((L - X) * inv_gamma) * rsm;
  return axis_grad(X, M, L, wp, wm, rsp, rsm, inv_gamma);
}

template <bool LSE>
__device__ __forceinline__ double net_wl_value(float M, float L, float wp, float wm, float sp,
                                               float sm, float gamma) {
  if (LSE) return (double)(M - L) + (double)gamma * (log((double)sp) + log((double)sm));
  return (double)((M - L) + wp - wm);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, kWave));
  return v;
}

__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fminf(v, __shfl_xor(v, off, kWave));
  return v;
}

// Wave-wide reductions on the DPP path (no LDS round trips): a butterfly
// inside each row of 16 lanes (row rotations by 8 and 4, then two quad
// permutations) leaves every lane holding its row's result; the four row
// results are combined in a fixed order from lanes 0, 16, 32 and 48.  The
// result is wave-uniform.  Every lane of the wave must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __builtin_bit_cast(
      float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
constexpr int kDppRowRor8 = 0x128, kDppRowRor4 = 0x124, kDppQuad2301 = 0x4e,
              kDppQuad1032 = 0xb1;

__device__ __forceinline__ float rows4_f(float v, int op) {
  const float a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 0));
  const float b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 16));
  const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 32));
  const float d = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 48));
  if (op == 0) return (a + b) + (c + d);
  if (op == 1) return fmaxf(fmaxf(a, b), fmaxf(c, d));
  return fminf(fminf(a, b), fminf(c, d));
}

__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_f<kDppRowRor8>(v);
  v += dpp_f<kDppRowRor4>(v);
  v += dpp_f<kDppQuad2301>(v);
  v += dpp_f<kDppQuad1032>(v);
  return rows4_f(v, 0);
}
__device__ __forceinline__ float wave_max_dpp(float v) {
  v = fmaxf(v, dpp_f<kDppRowRor8>(v));
  v = fmaxf(v, dpp_f<kDppRowRor4>(v));
  v = fmaxf(v, dpp_f<kDppQuad2301>(v));
  v = fmaxf(v, dpp_f<kDppQuad1032>(v));
  return rows4_f(v, 1);
}
__device__ __forceinline__ float wave_min_dpp(float v) {
  v = fminf(v, dpp_f<kDppRowRor8>(v));
  v = fminf(v, dpp_f<kDppRowRor4>(v));
  v = fminf(v, dpp_f<kDppQuad2301>(v));
  v = fminf(v, dpp_f<kDppQuad1032>(v));
  return rows4_f(v, 2);
}
__device__ __forceinline__ int wave_max_dpp_i(int v) {
  v = max(v, dpp_i<kDppRowRor8>(v));
  v = max(v, dpp_i<kDppRowRor4>(v));
  v = max(v, dpp_i<kDppQuad2301>(v));
  v = max(v, dpp_i<kDppQuad1032>(v));
  const int a = __builtin_amdgcn_readlane(v, 0), b = __builtin_amdgcn_readlane(v, 16);
  const int c = __builtin_amdgcn_readlane(v, 32), d = __builtin_amdgcn_readlane(v, 48);
  return max(max(a, b), max(c, d));
}

// Order LDS accesses of one wavefront (all lanes) without a block barrier.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Blocks are dealt to the 8 XCDs round-robin.  Remap so that XCD k runs a
// contiguous range of logical blocks (its writes then fill whole cache lines
// in its own L2).  Identity when the grid is not a multiple of 8.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  if (nb % kNumXcd) return b;
  return (b % kNumXcd) * (nb / kNumXcd) + b / kNumXcd;
}

// Exclusive prefix sum over a block of NT threads; *total gets the block sum.
template <int NT>
__device__ __forceinline__ int block_exclusive_scan(int v, int* total) {
  constexpr int NW = NT / kWave;
  __shared__ int wsum[NW];
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  int inc = v;
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const int u = __shfl_up(inc, off, kWave);
    if (lane >= off) inc += u;
  }
  if (lane == kWave - 1) wsum[w] = inc;
  __syncthreads();
  int woff = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NW; ++k) {
    if (k < w) woff += wsum[k];
    tot += wsum[k];
  }
  __syncthreads();
  *total = tot;
  return woff + inc - v;
}

__device__ __forceinline__ int block_exclusive_scan256(int v, int* total) {
  return block_exclusive_scan<256>(v, total);
}

// Block-wide double sum (blockDim a multiple of 64, <= 1024), either added to
// *dst with one atomic or stored to *dst.  Many blocks adding to one address
// serialise on it, so the hot paths store per-block partials instead and
// reduce them in a final kernel.
template <bool ATOMIC>
__device__ __forceinline__ void block_sum_to(double v, double* dst) {
  __shared__ double red[16];
  v = wave_sum(v);
  const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) red[w] = v;
  __syncthreads();
  if (w == 0) {
    const int nw = blockDim.x / kWave;
    double t = lane < nw ? red[lane] : 0.0;
    t = wave_sum(t);
    if (lane == 0) {
      if (ATOMIC)
        atomicAdd(dst, t);
      else
        *dst = t;
    }
  }
  __syncthreads();
}

__device__ __forceinline__ void block_atomic_add(double v, double* dst) {
  block_sum_to<true>(v, dst);
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

GridF make_gridf(const fftpl_grid& g);

struct Plan {
  int n = 0;
  int mode = 0;
  int device = 0;
  // batch slots: every map below (and rowsum, partials) holds max_batch
  // consecutive copies, one per design of a batched evaluation
  int max_batch = 1;
  size_t part_stride = 0;   // doubles of partials per slot
  // FFT-mode tables (float2): fft twiddles exp(-2 pi i t / n), t < n, and
  // (cos, sin)(pi k / (2n)), k <= n/2; frequency table w_u = pi u / n.
  float2* fft_tw = nullptr;
  float2* dct_cs = nullptr;
  float* wfreq = nullptr;
  // GEMM-mode tables: cosine and frequency-weighted sine matrices.
  void* gemm_tables = nullptr;
  size_t gemm_tables_bytes = 0;
  // Workspace maps.
  float* rho = nullptr;     // n*n
  float* tmp0 = nullptr;    // n*n  (bT / GEMM intermediate)
  float* tmp1 = nullptr;    // n*n  (P)
  float* tmp2 = nullptr;    // n*n  (Q)
  float* psi = nullptr;     // n*n
  float* exy = nullptr;     // 2*n*n interleaved (Ex, Ey)
  void* gemm_ws = nullptr;  // extra GEMM-mode workspace
  size_t gemm_ws_bytes = 0;
  double* rowsum = nullptr; // n doubles
  // Per-block partial sums of the solve: en_max energy slots, then overflow
  // pairs.  FFT: n/2 energy partials and n/2 pairs (one per row pair);
  // GEMM: 2 (n/64)^2 energy partials (one per output tile) and n pairs.
  double* partials = nullptr;
  int en_max = 0;
  int n_en = 0, n_tau = 0;
  // Optional per-kernel timing: an event is recorded on the launch stream
  // after every kernel of an evaluation (the first one before it).
  static constexpr int kMaxEvents = 24;
  // The wirelength kernels do not depend on the density or the solve: they
  // run on a second stream forked from and joined back into the caller's
  // stream with events (default priority; created with the plan).
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  bool timing = false;
  int nev = 0;
  hipEvent_t ev[kMaxEvents] = {};
  const char* ev_name[kMaxEvents] = {};
};

// Record a timing event named for the kernel that just finished (no-op
// unless timing is enabled on the plan).
inline void plan_mark(Plan& p, const char* name, hipStream_t s) {
  if (!p.timing || p.nev >= Plan::kMaxEvents) return;
  hipEventRecord(p.ev[p.nev], s);
  p.ev_name[p.nev] = name;
  ++p.nev;
}

// Launchers (return a hipError_t of the launch).
hipError_t launch_fill(float* dst, const float* src, float value, int64_t count,
                       hipStream_t s);
hipError_t launch_fill_f64(double* dst, double value, int count, hipStream_t s);
hipError_t launch_fixed_map(const GridF& g, int num_fixed, const float* fx,
                            const float* fy, const float* fw, const float* fh,
                            float* base, float* cap, hipStream_t s);
hipError_t launch_scatter(const GridF& g, int m, const float* x, const float* y,
                          const float* w, const float* h, float* rho, hipStream_t s);
hipError_t launch_gather(const GridF& g, int m, const float* x, const float* y,
                         const float* w, const float* h, const float* ex,
                         const float* ey, const float* exy, const float* psi,
                         int grad_mode, float scale, int accumulate, float* gx,
                         float* gy, hipStream_t s);
hipError_t launch_cell_bins(const GridF& g, int m, const float* x, const float* y,
                            const float* w, const float* h, int32_t* ranges,
                            hipStream_t s);
// wl_model: FFTPL_WL_WA (Eq. (3)) or FFTPL_WL_LSE (log-sum-exp)
hipError_t launch_wa(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                     const float* pin_dx, const float* pin_dy, const float* x,
                     const float* y, float gamma, int wl_model, float* gx, float* gy,
                     double* wa_out, double* hp_out, hipStream_t s);
// The stateless wirelength gradient with order-independent sums: per-pin
// gradients added to per-cell 64-bit fixed-point accumulators, then written
// (accumulate = 0) or added to gx, gy; wa_out / hp_out (if set) get the
// totals from per-block partials summed in a fixed order.  work: at least
// wa_fixed_work_bytes(num_cells, num_nets) bytes, 8-byte aligned.
size_t wa_fixed_work_bytes(int num_cells, int num_nets);
hipError_t launch_wa_fixed(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                           const float* pin_dx, const float* pin_dy, int num_cells,
                           const float* x, const float* y, float gamma, int wl_model,
                           int accumulate, float* gx, float* gy, double* wa_out,
                           double* hp_out, void* work, hipStream_t s);
// wa: per-block wirelength partials laid out [W~ (n_s), HPWL (n_s), W~ (n_b),
// HPWL (n_b)] (or null: W~ and HPWL are left as they are).
// The evaluation's scalars from per-block partials, summed in double in a
// fixed order (so repeated evaluations give identical scalars):
//   energy N   = sum en[0..n_en)
//   tau        = sum tau[2i] / sum tau[2i+1]   (overflow / movable area)
//   W~, HPWL   = sums of the wirelength kernels' per-block partials,
//                wa = [W_small(n_s), H_small(n_s), W_big(n_b), H_big(n_b)].
// Outputs may be null; W~ and HPWL are written only with wa.
struct FinalArgs {
  const double* en = nullptr;
  int n_en = 0;
  const double* tau = nullptr;
  int n_tau = 0;
  const double* wa = nullptr;
  int n_s = 0, n_b = 0;
  double *o_en = nullptr, *o_wa = nullptr, *o_hp = nullptr, *o_tau = nullptr;
};

// The sums of FinalArgs by one whole block of NT threads.
template <int NT>
__device__ __forceinline__ void eval_scalars(const FinalArgs& f) {
  const int t = threadIdx.x;
  // v = (energy, overflow, movable, W~, HPWL) partial sums; each batch's loads
  // (at clamped indices, the pointer tests uniform) are issued before any use
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  constexpr int U = 4;
  const int n_w = f.wa ? f.n_s + f.n_b : 0;
  const int most = max(max(f.n_en, f.n_tau), n_w);
  for (int i0 = t; i0 < most; i0 += U * NT) {
    double a[U], o[U], mv[U], sw[U], sh[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      a[u] = f.en && f.n_en > 0 ? f.en[min(i, f.n_en - 1)] : 0.0;
      o[u] = f.tau && f.n_tau > 0 ? f.tau[2 * min(i, f.n_tau - 1)] : 0.0;
      mv[u] = f.tau && f.n_tau > 0 ? f.tau[2 * min(i, f.n_tau - 1) + 1] : 0.0;
      const int j = min(i, n_w - 1);
      const int ws = j < f.n_s ? j : 2 * f.n_s + (j - f.n_s);
      const int hs = j < f.n_s ? f.n_s + j : 2 * f.n_s + f.n_b + (j - f.n_s);
      sw[u] = n_w > 0 ? f.wa[ws] : 0.0;
      sh[u] = n_w > 0 ? f.wa[hs] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + u * NT;
      v[0] += i < f.n_en ? a[u] : 0.0;
      v[1] += i < f.n_tau ? o[u] : 0.0;
      v[2] += i < f.n_tau ? mv[u] : 0.0;
      v[3] += i < n_w ? sw[u] : 0.0;
      v[4] += i < n_w ? sh[u] : 0.0;
    }
  }
  __shared__ double red[5][NT / kWave];
  const int lane = t & (kWave - 1), w = t / kWave;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    v[k] = wave_sum(v[k]);
    if (lane == 0) red[k][w] = v[k];
  }
  __syncthreads();
  if (t == 0) {
    double r[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      r[k] = 0.0;
      for (int j = 0; j < NT / kWave; ++j) r[k] += red[k][j];
    }
    if (f.o_en) *f.o_en = r[0];
    if (f.o_tau) *f.o_tau = r[2] > 0.0 ? r[1] / r[2] : 0.0;
    if (f.wa && f.o_wa) *f.o_wa = r[3];
    if (f.wa && f.o_hp) *f.o_hp = r[4];
  }
}

hipError_t launch_eval_finalize(const double* en, int n_en, const double* tau, int n_tau,
                                const double* wa, int n_s, int n_b, double* o_en, double* o_wa,
                                double* o_hp, double* o_tau, hipStream_t s);

// Blocks of the persistent big-net wirelength kernel (4 waves each; 512
// blocks keep every SIMD busy at its 2-wave occupancy).
inline int wa_big_grid(int num_nets) {
  const int nb = (num_nets + 255) / 256;
  return nb < 512 ? (nb > 0 ? nb : 1) : 512;
}

// ---- banded density scatter (atomic-free in global memory) ----------------
// Cells are counting-sorted into bands of `rows` bin rows (a cell is listed in
// every band its span touches, at most kMaxBands; taller cells go to a short
// list every band block walks), then one block per band accumulates its rows
// in LDS and writes them out.  Needs n <= kBandMaxN.
constexpr int kMaxBands = 4;
constexpr int kBandMaxN = 1024;
constexpr int kBandThreads = 512;      // threads of a counting / placing block
constexpr int kCellBatch = 8;          // cells whose loads a thread issues together
constexpr int kCellsPerBlock = kBandThreads * kCellBatch;   // 4096
constexpr int kBandRegion = kMaxBands * kCellsPerBlock;      // entries per block
constexpr int kAccThreads = 1024;      // threads of a band accumulation block

struct BandLayout {
  int n = 0, rows = 0, nb = 0;   // band height in rows, number of bands
  int m = 0, nblk = 0;           // cells, counting blocks
  // regions of the problem workspace
  float2* xy = nullptr;          // [m] interleaved positions
  float2* pin_grad = nullptr;    // [P] per-pin WA gradients, cell-major slots
  float4* entries = nullptr;     // [nblk*kBandRegion] band entries (cell edges in bins),
                                 // one region per counting block, sliced by band
  int32_t* epos = nullptr;       // [m] each cell's entry in its first band, -1 if none
  float2* egrad = nullptr;       // [nblk*kBandRegion] density gradient of the cell whose
                                 // first-band entry this is (band gather)
  int32_t* big = nullptr;        // [nblk*kCellsPerBlock] per block, its cells spanning
                                 // more than kMaxBands bands
  int32_t* blk_off = nullptr;    // [nb + 1][nblk] per band: each block's slice offset
  int32_t* blk_cnt = nullptr;    // [nb + 1][nblk] per band: each block's slice size
  double* wa_part = nullptr;     // per-block W~ / HPWL partials (slot or exchange path)
  int nwa = 0;                   // blocks of each wirelength kernel
};
BandLayout band_layout(int n, int m, int num_nets, int num_pins, void* work,
                       size_t* bytes_out);

// ---- batches: several designs of one grid side in one launch per stage ----
// Kernels take a batch of per-design descriptors by value (the kernel
// argument block, so nothing is staged through memory) and run design
// blockIdx.y; a design with fewer blocks than the launch's x extent leaves
// the rest idle.  NB = 1 for single designs keeps their argument blocks small.
constexpr int kMaxBatch = FFTPL_MAX_BATCH;

// One design's banded scatter and band gather.
struct BandReq {
  GridF g;
  BandLayout L;
  const float *x = nullptr, *y = nullptr, *w = nullptr, *h = nullptr;
  const float* base = nullptr;   // scatter: fixed charge (or null)
  float* rho = nullptr;          // scatter: the density map written
  const float2* exy = nullptr;   // gather: (Ex, Ey), or (Dx, Dy) in exact mode
  const float* psi = nullptr;    // gather: exact mode
};
template <int NB>
struct BandBatch {
  int count = 0;
  BandReq r[NB];
};
hipError_t launch_band_scatter_batch(const BandReq* reqs, int count, hipStream_t s,
                                     Plan* tp = nullptr);
// The density scatter's band lists alone (for the allocation-free density
// map), and the device address of the library's static scratch array on the
// current device (looked up once per device).
constexpr size_t kNoallocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevicesNoalloc = 64;
BandLayout band_layout_density(int n, int m, void* work, size_t* bytes_out);
hipError_t noalloc_scratch(void** ptr);
hipError_t launch_band_gather_batch(const BandReq* reqs, int count, int grad_mode,
                                    hipStream_t s);

// egrad[entry] = density gradient (before lambda) of each cell at its
// first-band entry (after launch_band_scatter and the solve).
hipError_t launch_band_gather(const GridF& g, const BandLayout& L, const float* exy,
                              const float* psi, int grad_mode, hipStream_t s);
hipError_t launch_band_scatter(const GridF& g, const BandLayout& L, const float* x,
                               const float* y, const float* w, const float* h,
                               const float* base, float* rho, hipStream_t s,
                               Plan* tp = nullptr);
hipError_t launch_init_eval(double* out4, int32_t* counters, int ncount, hipStream_t s);
hipError_t launch_interleave(int m, const float* x, const float* y, float2* xy,
                             hipStream_t s);
hipError_t launch_wa_pins(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                          const float* pin_dx, const float* pin_dy, const float2* xy,
                          const int32_t* pin_slot, float gamma, int wl_model,
                          float2* pin_grad, double* wa_part, hipStream_t s,
                          Plan* tp = nullptr);
hipError_t launch_gather_pins(const GridF& g, int m, const float* x, const float* y,
                              const float* w, const float* h, const float* exy,
                              const float* psi, int grad_mode, float scale,
                              const int32_t* cell_ptr, const float2* pin_grad, float* gx,
                              float* gy, hipStream_t s);
hipError_t launch_netlist_index(int m, int num_pins, const int32_t* pin_cell,
                                int32_t* cell_ptr, int32_t* pin_slot, int32_t* work,
                                hipStream_t s);
hipError_t launch_zero_i32(int32_t* a, int64_t count, hipStream_t s);
hipError_t launch_exclusive_scan(const int32_t* in, int count, int32_t* out, int32_t* sums,
                                 int32_t* total, hipStream_t s);

// ---- bucketed pin exchange for the wirelength gradient ---------------------
// Cells are cut into blocks of kXchCells consecutive cells, nets into blocks
// of whole nets holding at most kXchPinCap pins.  A pin's data moves between
// the cell side and the net side through a buffer T[num_pins] in "A order"
// (pins grouped by cell block, then by net block); a net block reads its pins
// in "B order" (grouped by cell block), so both sides move runs of pins
// instead of single random words, and every random access happens in LDS.
// Most cells of a cell block, 9 x 1024: the cell-sum accumulators (17 bytes
// per cell) then fill 153 KiB of LDS.  A design's cell blocks hold
// XchDims::cpb cells, a multiple of kXchCellStep chosen so that there are
// about as many blocks as CUs (kNumCus): the cell sums, one block per CU,
// then run in a single round at any size up to 2.36M cells, and small designs
// still spread over the chip.
constexpr int kXchCells = 9216;
constexpr int kXchCellStep = 256;
constexpr int kNumCus = 256;           // compute units of an MI355X (gfx950)
constexpr int kXchSpreadSplit = 2;     // spread blocks per cell block
constexpr int kXchThreads = 512;       // threads of the cell-block kernels
constexpr int kXchWaThreads = 512;     // threads of the net-block kernel
constexpr int kXchPinCap = 9728;       // most pins of a net block (2 x 76 KiB of float2 in LDS)
constexpr int kXchPinLds2 = 4864;      // pins of a net block that leave room for 2 blocks per CU
constexpr int kXchPinTarget = 4096;    // most of npt, the least pins of a full net block
constexpr int kXchMinTarget = 1024;
constexpr int kXchBuckets = 20;        // degree classes of the net order: 0..8, then
                                       // 9-16, 17-32, ..., > 8192

struct XchDims {
  int m = 0, num_nets = 0, num_pins = 0, max_degree = 0;
  int npt = 0;         // every net block but the last holds at least npt pins
  int cap = 0;         // bound on the pins of one net block: npt - 1 + max_degree
  int cpb = kXchCells;     // cells per cell block
  int ncb = 0, nnb = 0;   // cell blocks, net blocks
  size_t index_bytes = 0, work_bytes = 0;
  // offsets inside the index buffer
  size_t o_hdr = 0, o_cb = 0, o_nb = 0, o_ab = 0, o_lcsr = 0, o_lc = 0,
         o_ns = 0;
};
// Returns FFTPL_OK, or FFTPL_E_UNSUPPORTED when max_degree is too large for
// a net block, or FFTPL_E_INVAL for negative sizes.
int xch_dims(int m, int num_nets, int num_pins, int max_degree, XchDims* d);

struct XchIndex {
  const int32_t* cb_a_ptr = nullptr;    // [ncb+1] A range of each cell block
  const int32_t* nb_net_ptr = nullptr;  // [nnb+1] first net of each net block
  const int32_t* a_of_b = nullptr;      // [P] A position of each B-order pin
  const uint16_t* lcsr = nullptr;       // [P] pin offset inside its net block (B order)
  const uint16_t* lc = nullptr;         // [P] cell offset inside its cell block (A order)
  const uint32_t* nmeta = nullptr;      // [E] per net block, its nets by degree class:
                                       // (first pin - block's first pin) << 16 | degree
};
XchIndex xch_index(const XchDims& d, const void* index);

int xch_build(const XchDims& d, const int32_t* net_ptr, const int32_t* pin_cell, void* index,
              void* work, hipStream_t s);   // returns fftpl_status; synchronises s
// Host side of the build: net blocks packed greedily from a host copy of the
// CSR (whole nets in order, a block closed when the next net does not fit in
// cap pins): first[k] = first net of block k, first[k] = E past the last
// block, k <= nnb.  FFTPL_E_INVAL for a CSR that is not one over P pins,
// a net above max_degree, or more than nnb blocks.
int pack_net_blocks(const int32_t* ptr, int E, int P, int max_degree, int cap, int nnb,
                    int32_t* first);
hipError_t launch_xch_spread(const XchDims& d, const XchIndex& X, const float* x,
                             const float* y, float2* T, hipStream_t s);
hipError_t launch_xch_wa(const XchDims& d, const XchIndex& X, const int32_t* net_ptr,
                         const float* pin_dx, const float* pin_dy, float gamma, int wl_model,
                         float2* T, double* wa_part, hipStream_t s);
// gwa[c] = sum over cell c's pins of T[qa[j]] (after launch_xch_wa).
// The per-cell part of the gradient after the wirelength: g = scale * the
// density gradient (egrad at the cell's first-band entry, or computed from the
// maps for a cell without one) + the cell's wirelength sum.
struct CellGradArgs {
  GridF g;
  const float *x = nullptr, *y = nullptr, *w = nullptr, *h = nullptr;
  const float2* exy = nullptr;
  const float* psi = nullptr;
  const int32_t* epos = nullptr;
  const float2* egrad = nullptr;
  float scale = 0.0f;
  // if set, the scale is read on the device from dscale[0] when the kernel runs
  const float* dscale = nullptr;
  float *gx = nullptr, *gy = nullptr;
  // block fin_block (if >= 0) also reduces the evaluation's scalars (every
  // partial they need is complete before the cell sums start), in place of a
  // separate finalize launch
  FinalArgs fin;
  int fin_block = -1;
  // without a density part (the wirelength alone): add to gx, gy instead of
  // overwriting them
  int accumulate = 0;
};
// g (CellGradArgs) for every cell, the wirelength part being the sum over
// the cell's pins of their gradients in T (after launch_xch_wa).
hipError_t launch_xch_cellsum(const XchDims& d, const XchIndex& X, const float2* T,
                              const CellGradArgs& a, int grad_mode, hipStream_t s);

// One design's pin exchange: the spread (cells -> pins) and the net blocks.
struct XchReq {
  int m = 0, cpb = 0, ncb = 0;
  const int32_t* cb_a_ptr = nullptr;
  const uint16_t* lc = nullptr;
  const float *x = nullptr, *y = nullptr;
  float2* T = nullptr;
  int num_pins = 0, cap = 1, nnb = 0;
  const int32_t* net_ptr = nullptr;
  const int32_t* nb_net_ptr = nullptr;
  const uint32_t* nmeta = nullptr;
  const int32_t* a_of_b = nullptr;
  const uint16_t* lcsr = nullptr;
  const float *pin_dx = nullptr, *pin_dy = nullptr;
  float gamma = 1.0f, inv_gamma = 1.0f;
  // if set, gamma is read on the device from dgamma[0] when the kernel runs
  // (and 1/gamma formed there in float, as on the host)
  const float* dgamma = nullptr;
  double* part = nullptr;
  // per-net values at each net's first pin (a test export), or null
  double *net_wl = nullptr, *net_hp = nullptr;
};
template <int NB>
struct XchBatch {
  int count = 0;
  XchReq r[NB];
};
// One design's per-cell sums (and density part).
struct SumReq {
  int m = 0, cpb = 0, ncb = 0;
  const int32_t* cb_a_ptr = nullptr;
  const uint16_t* lc = nullptr;
  const float2* T = nullptr;
  float fx_scale = 1.0f;   // fixed-point scale of the pin gradients
  double inv_scale = 1.0;
  CellGradArgs a;
};
template <int NB>
struct SumBatch {
  int count = 0;
  SumReq r[NB];
};
XchReq xch_req(const XchDims& d, const XchIndex& X, const float* x, const float* y, float2* T,
               const int32_t* net_ptr, const float* pin_dx, const float* pin_dy, float gamma,
               double* part);
SumReq sum_req(const XchDims& d, const XchIndex& X, const float2* T, const CellGradArgs& a);
// count <= kMaxBatch designs per launch; the net blocks of one launch share
// the wirelength model.  dens = false: the cell sums without density part.
hipError_t launch_xch_spread_batch(const XchReq* reqs, int count, hipStream_t s);
hipError_t launch_xch_wa_batch(const XchReq* reqs, int count, int wl_model, hipStream_t s);
hipError_t launch_xch_cellsum_batch(const SumReq* reqs, int count, int grad_mode, bool dens,
                                    hipStream_t s);
// ---- placement iteration (driver.hip) --------------------------------------
size_t step_stats_work_doubles();
hipError_t launch_step_stats(int m, const float* ux, const float* uy, const float* upx,
                             const float* upy, const float* gx, const float* gy,
                             const float* gpx, const float* gpy, double* out, double* work,
                             hipStream_t s);
hipError_t launch_cg_dots(int m, const float* gx, const float* gy, const float* gpx,
                          const float* gpy, const float* dx, const float* dy, double* out,
                          double* work, hipStream_t s);
hipError_t launch_cg_direction(int m, const float* gx, const float* gy, float beta, float* dx,
                               float* dy, double* dmax, double* work, hipStream_t s);
hipError_t launch_cg_move(int m, const float* x, const float* y, const float* dx,
                          const float* dy, float t, const float* w, const float* h, float xl,
                          float yl, float xh, float yh, float* xo, float* yo, hipStream_t s);
// step_beta (if not null): step and beta read on the device instead
hipError_t launch_nesterov_update(int m, float* x, float* y, float* ux, float* uy, float* upx,
                                  float* upy, float* gpx, float* gpy, const float* gx,
                                  const float* gy, const float* w, const float* h, float step,
                                  float beta, const double* step_beta, float xl, float yl,
                                  float xh, float yh, hipStream_t s);
hipError_t launch_nesterov_schedule(const double* stats, const double* out4, double* state,
                                    float* params, double* log, int log_cap, hipStream_t s);

// Spectral solve.  psi/ex/ey/exy may be null individually.  en_part, if set,
// receives n/2 per-block partials of the energy sum rho*psi; tau_part, if
// set, n values: per-block pairs (overflow, movable area) of the first pass,
// read against base (or 0) and cap (or rho_t - min(rho_t, base)).
struct SpectralArgs {
  const float* rho = nullptr;
  float* psi = nullptr;
  float* ex = nullptr;
  float* ey = nullptr;
  float* exy = nullptr;
  double* en_part = nullptr;
  const float* base = nullptr;
  const float* cap = nullptr;
  float rho_t = 1.0f;
  double* tau_part = nullptr;
  // screening eps >= 0 (bin^-2): every mode divides by w_u^2 + w_v^2 + eps
  float eps = 0.0f;
  // difference mode: exy receives (Dx, Dy) = (psi(ix+1) - psi(ix), psi(iy+1) - psi(iy))
  // at every bin instead of (Ex, Ey); ex and ey must be null
  bool diff = false;
};
hipError_t spectral_fft(Plan& p, const SpectralArgs& a, hipStream_t s);
// count designs (count <= the plan's max_batch, one difference mode): design
// i uses batch slot i of the plan's intermediate maps; one launch per pass.
hipError_t spectral_fft_batch(Plan& p, const SpectralArgs* a, int count, hipStream_t s);

// One design of a batched FFT solve: its maps and the plan slot it uses.
struct SpecReq {
  const float* rho = nullptr;
  float *psi = nullptr, *ex = nullptr, *ey = nullptr;
  float2* exy = nullptr;
  float* bT = nullptr;        // plan slot: transposed row transforms
  double* rowsum = nullptr;   // plan slot: double row sums
  float *P = nullptr, *Q = nullptr;   // plan slot: column pass outputs
  const float *base = nullptr, *cap = nullptr;
  float rho_t = 1.0f, eps = 0.0f;
  double *en_part = nullptr, *tau_part = nullptr;
};
template <int NB>
struct SpecBatch {
  int count = 0;
  SpecReq r[NB];
};
hipError_t spectral_gemm(Plan& p, const SpectralArgs& a, hipStream_t s);
int gemm_plan_init(Plan& p, hipStream_t s);   // returns fftpl_status
void gemm_plan_free(Plan& p);

}  // namespace fftpl
