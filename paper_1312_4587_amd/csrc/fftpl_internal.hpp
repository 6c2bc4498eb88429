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
hipError_t launch_wa(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                     const float* pin_dx, const float* pin_dy, const float* x,
                     const float* y, float gamma, float* gx, float* gy,
                     double* wa_out, double* hp_out, hipStream_t s);
// wa: the wirelength partials of fftpl_eval's atomic-free path for num_nets
// nets (or null: W~ and HPWL are left as they are).
hipError_t launch_eval_finalize(const double* en, int n_en, const double* tau, int n_tau,
                                const double* wa, int num_nets, double* o_en, double* o_wa,
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
constexpr int kBandThreads = 1024;     // threads of every band-sort block
constexpr int kCellBatch = 8;          // cells whose loads a thread issues together
constexpr int kCellsPerBlock = kBandThreads * 2 * kCellBatch;   // 16384

struct BandLayout {
  int n = 0, rows = 0, nb = 0;   // band height in rows, number of bands
  int m = 0, nblk = 0;           // cells, counting blocks
  // regions of the problem workspace
  float2* xy = nullptr;          // [m] interleaved positions
  float2* pin_grad = nullptr;    // [P] per-pin WA gradients, cell-major slots
  float4* entries = nullptr;     // [kMaxBands*m] band entries: cell edges in bins
  int32_t* big = nullptr;        // [m] cells spanning more than kMaxBands bands
  int32_t* blk_base = nullptr;   // [nblk*nb] block offsets inside each band
  int32_t* counters = nullptr;   // [nb + 1] band counts, then the big-cell count
  double* wa_part = nullptr;     // [4*nwa] per-block W~ / HPWL partials
  int nwa = 0;                   // blocks of each wirelength kernel
};
BandLayout band_layout(int n, int m, int num_nets, int num_pins, void* work,
                       size_t* bytes_out);

hipError_t launch_band_scatter(const GridF& g, const BandLayout& L, const float* x,
                               const float* y, const float* w, const float* h,
                               const float* base, float* rho, hipStream_t s,
                               Plan* tp = nullptr);
hipError_t launch_init_eval(double* out4, int32_t* counters, int ncount, hipStream_t s);
hipError_t launch_interleave(int m, const float* x, const float* y, float2* xy,
                             hipStream_t s);
hipError_t launch_wa_pins(int num_nets, const int32_t* net_ptr, const int32_t* pin_cell,
                          const float* pin_dx, const float* pin_dy, const float2* xy,
                          const int32_t* pin_slot, float gamma, float2* pin_grad,
                          double* wa_part, hipStream_t s, Plan* tp = nullptr);
hipError_t launch_gather_pins(const GridF& g, int m, const float* x, const float* y,
                              const float* w, const float* h, const float* exy,
                              const float* psi, int grad_mode, float scale,
                              const int32_t* cell_ptr, const float2* pin_grad, float* gx,
                              float* gy, hipStream_t s);
hipError_t launch_netlist_index(int m, int num_pins, const int32_t* pin_cell,
                                int32_t* cell_ptr, int32_t* pin_slot, int32_t* work,
                                hipStream_t s);

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
};
hipError_t spectral_fft(Plan& p, const SpectralArgs& a, hipStream_t s);
hipError_t spectral_gemm(Plan& p, const SpectralArgs& a, hipStream_t s);
int gemm_plan_init(Plan& p, hipStream_t s);   // returns fftpl_status
void gemm_plan_free(Plan& p);

}  // namespace fftpl
