// Bucketed pin exchange for the weighted-average wirelength gradient
// (Eq. (3)) and HPWL (Eq. (1)).
//
// Nets pick their cells anywhere in the design, so handing cell positions to
// pins and pin gradients back to cells is a permutation of the pins.  Done
// directly, every pin costs one random 8-byte read and one random 8-byte
// write, each of which moves a whole cache line.  Here the permutation is
// split in two halves that both run through LDS:
//
//   cell blocks: cpb consecutive cells (a multiple of 256, at most kXchCells,
//                about one block per CU);
//   net blocks:  whole nets packed in CSR order, as many as fit in cap =
//                npt - 1 + max_degree <= kXchPinCap pins, so every block but
//                the last holds at least npt pins and there are at most
//                ceil(P / npt) blocks (the trailing ones may be empty);
//   A order:     pins sorted by (cell block, net block);
//   B order:     inside each net block's CSR range, pins sorted by cell block,
//                in the same order as A within each (cell block, net block)
//                segment.
//
//   spread  (one block per cell block): positions of the block's cells into
//           LDS, then T[a] = position of pin a's cell for its A range
//           (coalesced writes, random reads in LDS);
//   wa      (one block per net block): reads T in B order, i.e. runs of the
//           consecutive A positions of each segment, into LDS in CSR order;
//           evaluates every net from LDS (one thread per net of degree <= 8,
//           one wavefront per larger net); writes each pin's gradient back to
//           its own A position of T, again in runs;
//   cellsum (one block per cell block): streams the cell block's A
//           range of T and adds every pin's gradient into its cell's
//           accumulator in LDS (integer fixed point: order-independent),
//           then writes each cell's gradient: lambda times its density
//           gradient (computed per band entry on the density branch) plus
//           that sum.
//
// The index (A/B layout) is built once per netlist by xch_build.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <vector>

#include "fftpl_internal.hpp"

namespace fftpl {

namespace {

constexpr int NT = kXchThreads;
constexpr int kHdrInts = 16;
constexpr int32_t kXchMagic = 0x46584348;   // "FXCH"
constexpr int kSmall = 8;                   // degree handled by one thread
constexpr int NW = kXchWaThreads;
// B positions per thread of the net-block kernel: for blocks of up to
// kXchPinLds2 pins, or up to kXchPinCap
constexpr int kStageS = (kXchPinLds2 + NW - 1) / NW;
constexpr int kStageL = (kXchPinCap + NW - 1) / NW;
constexpr int kMaxDevices = 64;     // device ordinals with a per-device flag
constexpr int kSumThreads = 1024;   // cell sums: one block per cell block

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

int xch_dims(int m, int num_nets, int num_pins, int max_degree, XchDims* d) {
  if (m < 0 || num_nets < 0 || num_pins < 0 || max_degree < 0) return FFTPL_E_INVAL;
  // the largest block that still fits twice in one CU's LDS; failing that
  // (very large nets) one block per CU
  int npt = kXchPinTarget;
  if (npt > kXchPinLds2 + 1 - max_degree) npt = kXchPinLds2 + 1 - max_degree;
  if (npt < kXchMinTarget) {
    npt = kXchPinTarget;
    if (npt > kXchPinCap + 1 - max_degree) npt = kXchPinCap + 1 - max_degree;
  }
  if (npt < kXchMinTarget) return FFTPL_E_UNSUPPORTED;
  XchDims r;
  r.m = m;
  r.num_nets = num_nets;
  r.num_pins = num_pins;
  r.max_degree = max_degree;
  r.npt = npt;
  r.cap = max_degree > 0 ? npt - 1 + max_degree : 1;
  {
    const int64_t per_cu = ((int64_t)m + kNumCus - 1) / kNumCus;
    const int64_t step = (per_cu + kXchCellStep - 1) / kXchCellStep * kXchCellStep;
    r.cpb = (int)std::min<int64_t>(kXchCells, std::max<int64_t>(kXchCellStep, step));
  }
  r.ncb = (m + r.cpb - 1) / r.cpb;
  r.nnb = num_pins > 0 ? (num_pins + npt - 1) / npt : 1;
  size_t off = 0;
  r.o_hdr = off;
  off = align256(off + sizeof(int32_t) * kHdrInts);
  r.o_cb = off;
  off = align256(off + sizeof(int32_t) * ((size_t)r.ncb + 1));
  r.o_nb = off;
  off = align256(off + sizeof(int32_t) * ((size_t)r.nnb + 1));
  r.o_ab = off;
  off = align256(off + sizeof(int32_t) * (size_t)num_pins);
  r.o_lcsr = off;
  off = align256(off + sizeof(uint16_t) * (size_t)num_pins);
  r.o_lc = off;
  off = align256(off + sizeof(uint16_t) * (size_t)num_pins);
  r.o_ns = off;
  off = align256(off + sizeof(uint32_t) * (size_t)num_nets);
  r.index_bytes = off;
  // build workspace: counts / cursors, A starts, transposed counts, B starts,
  // scan block sums, flag and scan totals
  const size_t seg = (size_t)r.ncb * r.nnb;
  r.work_bytes = align256(sizeof(int32_t) * seg) * 4 +
                 align256(sizeof(int32_t) * ((seg + 1023) / 1024 + 1)) +
                 align256(sizeof(int32_t) * 4);
  *d = r;
  return FFTPL_OK;
}

XchIndex xch_index(const XchDims& d, const void* index) {
  XchIndex X;
  const char* b = static_cast<const char*>(index);
  X.cb_a_ptr = reinterpret_cast<const int32_t*>(b + d.o_cb);
  X.nb_net_ptr = reinterpret_cast<const int32_t*>(b + d.o_nb);
  X.a_of_b = reinterpret_cast<const int32_t*>(b + d.o_ab);
  X.lcsr = reinterpret_cast<const uint16_t*>(b + d.o_lcsr);
  X.lc = reinterpret_cast<const uint16_t*>(b + d.o_lc);
  X.nmeta = reinterpret_cast<const uint32_t*>(b + d.o_ns);
  return X;
}

// ---------------------------------------------------------------------------
// Index build
// ---------------------------------------------------------------------------
namespace {

// Checks the CSR (net_ptr[0] = 0, net_ptr[E] = P, monotone, degrees <=
// max_degree, pin cells in range) and, with PLACE = false, counts the pins of
// every (cell block, net block) segment; with PLACE = true, hands each pin its
// A and B positions (the same rank inside the segment on both sides).
template <bool PLACE>
__global__ void __launch_bounds__(256)
    k_xi_pins(int num_nets, const int32_t* __restrict__ net_ptr, int num_pins,
              const int32_t* __restrict__ pin_cell, int m, int cpb, int max_degree, int ncb,
              int nnb, int32_t* __restrict__ cnt, const int32_t* __restrict__ seg_a,
              const int32_t* __restrict__ seg_bt, const int32_t* __restrict__ nb_net_ptr,
              int32_t* __restrict__ a_of_b, uint16_t* __restrict__ lcsr,
              uint16_t* __restrict__ lc, int32_t* __restrict__ flag) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (!PLACE && e == 0 && (net_ptr[0] != 0 || net_ptr[num_nets] != num_pins))
    atomicOr(flag, 1);
  // placing is only safe when the count saw a valid CSR covering every pin
  // once: then every A and B position stays below num_pins
  if (PLACE && (flag[0] != 0 || flag[1] != num_pins)) return;
  if (e >= num_nets) return;
  const int p0 = net_ptr[e], p1 = net_ptr[e + 1];
  if (p0 < 0 || p1 < p0 || p1 > num_pins || p1 - p0 > max_degree) {
    if (!PLACE) atomicOr(flag, 2);
    return;
  }
  if (p1 == p0) return;
  // the net block holding net e: the last k with nb_net_ptr[k] <= e
  int lo = 0, hi = nnb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nb_net_ptr[mid] <= e)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int k = lo;
  if (e >= nb_net_ptr[k + 1]) {
    if (!PLACE) atomicOr(flag, 4);
    return;
  }
  const int base = PLACE ? net_ptr[nb_net_ptr[k]] : 0;
  for (int p = p0; p < p1; ++p) {
    const int c = pin_cell[p];
    if (c < 0 || c >= m) {
      if (!PLACE) atomicOr(flag, 8);
      continue;
    }
    const int cb = c / cpb;
    const size_t idx = (size_t)cb * nnb + k;
    if (!PLACE) {
      atomicAdd(&cnt[idx], 1);
    } else {
      const int r = atomicAdd(&cnt[idx], 1);
      const int a = seg_a[idx] + r;
      const int b = seg_bt[(size_t)k * ncb + cb] + r;
      a_of_b[b] = a;
      lcsr[b] = (uint16_t)(p - base);
      lc[a] = (uint16_t)(c - cb * cpb);
    }
  }
}

// Degree class of the net order: the degree itself up to kSmall, then one
// class per power of two (9-16, 17-32, ..., the last one open-ended).
__device__ __forceinline__ int degree_class(int deg) {
  if (deg <= kSmall) return deg;
  const int c = kSmall + 1 + (31 - __clz(deg - 1)) - 3;
  return c < kXchBuckets - 1 ? c : kXchBuckets - 1;
}

// Per net block, its nets in increasing degree class, each as (first pin -
// the block's first pin) << 16 | degree; the order inside a class is
// arbitrary.  A wavefront walking this order from the front sees small nets
// of equal degree together (its loops over pins run the length of the
// degree); walking it from the back it meets the largest nets first.  The
// kernel reads each net's extent from here with one coalesced load.
__global__ void __launch_bounds__(256)
    k_xi_netsort(const int32_t* __restrict__ net_ptr, const int32_t* __restrict__ nb_net_ptr,
                 uint32_t* __restrict__ nmeta) {
  __shared__ int cnt[kXchBuckets], cur[kXchBuckets];
  const int k = blockIdx.x, t = threadIdx.x;
  const int e0 = nb_net_ptr[k], e1 = nb_net_ptr[k + 1];
  const int p0 = net_ptr[e0];
  if (t < kXchBuckets) cnt[t] = 0;
  __syncthreads();
  for (int e = e0 + t; e < e1; e += blockDim.x)
    atomicAdd(&cnt[degree_class(net_ptr[e + 1] - net_ptr[e])], 1);
  __syncthreads();
  if (t == 0) {
    int run = 0;
    for (int b = 0; b < kXchBuckets; ++b) {
      cur[b] = run;
      run += cnt[b];
    }
  }
  __syncthreads();
  for (int e = e0 + t; e < e1; e += blockDim.x) {
    const int q0 = net_ptr[e], deg = net_ptr[e + 1] - q0;
    nmeta[e0 + atomicAdd(&cur[degree_class(deg)], 1)] =
        ((uint32_t)(q0 - p0) << 16) | (uint32_t)deg;
  }
}

__global__ void k_xi_transpose(int ncb, int nnb, const int32_t* __restrict__ cnt,
                               int32_t* __restrict__ cnt_t) {
  const size_t total = (size_t)ncb * nnb;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const size_t cb = i / nnb, k = i % nnb;
    cnt_t[k * ncb + cb] = cnt[i];
  }
}

__global__ void k_xi_finish(int ncb, int nnb, int num_pins, const int32_t* __restrict__ seg_a,
                            int32_t* __restrict__ cb_a_ptr, int32_t* __restrict__ hdr,
                            int m, int num_nets, int max_degree, int npt, int cpb) {
  const int cb = blockIdx.x * blockDim.x + threadIdx.x;
  if (cb < ncb) cb_a_ptr[cb] = seg_a[(size_t)cb * nnb];
  if (cb == ncb) cb_a_ptr[cb] = num_pins;
  if (cb == 0) {
    hdr[0] = kXchMagic;
    hdr[1] = m;
    hdr[2] = num_nets;
    hdr[3] = num_pins;
    hdr[4] = max_degree;
    hdr[5] = npt;
    hdr[6] = ncb;
    hdr[7] = nnb;
    hdr[8] = cpb;
  }
}

}  // namespace

int pack_net_blocks(const int32_t* ptr, int E, int P, int max_degree, int cap, int nnb,
                    int32_t* first) {
  if (E < 0 || nnb < 1 || cap < 1) return FFTPL_E_INVAL;
  if (ptr[0] != 0 || ptr[E] != P) return FFTPL_E_INVAL;
  for (int k = 0; k <= nnb; ++k) first[k] = E;
  int k = 0;
  int64_t cur = 0;
  first[0] = 0;
  for (int en = 0; en < E; ++en) {
    const int64_t deg = (int64_t)ptr[(size_t)en + 1] - ptr[en];
    if (deg < 0 || deg > max_degree) return FFTPL_E_INVAL;
    if (cur + deg > cap) {
      if (++k >= nnb) return FFTPL_E_INVAL;   // cannot happen for a valid CSR
      first[k] = en;
      cur = 0;
    }
    cur += deg;
  }
  return FFTPL_OK;
}

int xch_build(const XchDims& d, const int32_t* net_ptr, const int32_t* pin_cell, void* index,
              void* work, hipStream_t s) {
  const size_t seg = (size_t)d.ncb * d.nnb;
  if (seg > (size_t)INT32_MAX) return FFTPL_E_UNSUPPORTED;
  char* w = static_cast<char*>(work);
  int32_t* cnt = reinterpret_cast<int32_t*>(w);
  w += align256(sizeof(int32_t) * seg);
  int32_t* seg_a = reinterpret_cast<int32_t*>(w);
  w += align256(sizeof(int32_t) * seg);
  int32_t* cnt_t = reinterpret_cast<int32_t*>(w);
  w += align256(sizeof(int32_t) * seg);
  int32_t* seg_bt = reinterpret_cast<int32_t*>(w);
  w += align256(sizeof(int32_t) * seg);
  int32_t* sums = reinterpret_cast<int32_t*>(w);
  w += align256(sizeof(int32_t) * ((seg + 1023) / 1024 + 1));
  int32_t* flag = reinterpret_cast<int32_t*>(w);   // [0] error bits, [1] [2] scan totals

  char* ib = static_cast<char*>(index);
  int32_t* hdr = reinterpret_cast<int32_t*>(ib + d.o_hdr);
  int32_t* cb_a_ptr = reinterpret_cast<int32_t*>(ib + d.o_cb);
  int32_t* nb_net_ptr = reinterpret_cast<int32_t*>(ib + d.o_nb);
  int32_t* a_of_b = reinterpret_cast<int32_t*>(ib + d.o_ab);
  uint16_t* lcsr = reinterpret_cast<uint16_t*>(ib + d.o_lcsr);
  uint16_t* lc = reinterpret_cast<uint16_t*>(ib + d.o_lc);

  const int E = d.num_nets, P = d.num_pins;
  const dim3 net_grid((E + 255) / 256 > 0 ? (E + 255) / 256 : 1);
  // Net blocks, packed greedily on the host from the CSR (a sequential scan
  // of the net sizes, once per netlist): a block is closed when the next net
  // does not fit in cap pins.  Packing instead of cutting at fixed pin counts
  // fills the blocks (the LDS is sized for cap) rather than reserving room
  // for a largest net at every block end.
  {
    std::vector<int32_t> hptr((size_t)E + 1), hnb((size_t)d.nnb + 1, E);
    if (hipMemcpyAsync(hptr.data(), net_ptr, sizeof(int32_t) * ((size_t)E + 1),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FFTPL_E_DEVICE;
    const int st = pack_net_blocks(hptr.data(), E, P, d.max_degree, d.cap, d.nnb, hnb.data());
    if (st != FFTPL_OK) return st;
    if (hipMemcpyAsync(nb_net_ptr, hnb.data(), sizeof(int32_t) * hnb.size(),
                       hipMemcpyHostToDevice, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return FFTPL_E_DEVICE;
  }
  hipError_t e = launch_zero_i32(cnt, (int64_t)seg, s);
  if (e == hipSuccess) e = launch_zero_i32(flag, 4, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_xi_pins<false>), net_grid, dim3(256), 0, s, E, net_ptr, P, pin_cell,
                       d.m, d.cpb, d.max_degree, d.ncb, d.nnb, cnt, nullptr, nullptr, nb_net_ptr,
                       nullptr, nullptr, nullptr, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_exclusive_scan(cnt, (int)seg, seg_a, sums, flag + 1, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_xi_transpose, dim3(1024), dim3(256), 0, s, d.ncb, d.nnb, cnt, cnt_t);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = launch_exclusive_scan(cnt_t, (int)seg, seg_bt, sums, flag + 2, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_xi_finish, dim3((d.ncb + 256) / 256), dim3(256), 0, s, d.ncb, d.nnb,
                       P, seg_a, cb_a_ptr, hdr, d.m, E, d.max_degree, d.npt, d.cpb);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return FFTPL_E_DEVICE;
  // the netlist is valid (every pin counted once, cells in range) before
  // anything indexes by it
  int32_t hflag[3] = {0, 0, 0};
  if (hipMemcpyAsync(hflag, flag, sizeof(hflag), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FFTPL_E_DEVICE;
  if (hflag[0] != 0 || hflag[1] != P || hflag[2] != P) return FFTPL_E_INVAL;
  e = launch_zero_i32(cnt, (int64_t)seg, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_xi_pins<true>), net_grid, dim3(256), 0, s, E, net_ptr, P, pin_cell,
                       d.m, d.cpb, d.max_degree, d.ncb, d.nnb, cnt, seg_a, seg_bt, nb_net_ptr,
                       a_of_b, lcsr, lc, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    uint32_t* nmeta = reinterpret_cast<uint32_t*>(ib + d.o_ns);
    hipLaunchKernelGGL(k_xi_netsort, dim3(d.nnb), dim3(256), 0, s, net_ptr, nb_net_ptr, nmeta);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? FFTPL_OK : FFTPL_E_DEVICE;
}

// ---------------------------------------------------------------------------
// Evaluation kernels
// ---------------------------------------------------------------------------
namespace {

// T[a] = (x, y) of pin a's cell, over part blockIdx.x % kXchSpreadSplit of
// the A range of cell block blockIdx.x / kXchSpreadSplit.
template <int NB>
__global__ void __launch_bounds__(NT) k_xch_spread(XchBatch<NB> xb) {
  // design blockIdx.y of the batch; blocks past its cell blocks idle
  const XchReq& rq = xb.r[blockIdx.y];
  const int m = rq.m, cpb = rq.cpb;
  if ((int)blockIdx.x >= rq.ncb * kXchSpreadSplit) return;
  const int32_t* __restrict__ cb_a_ptr = rq.cb_a_ptr;
  const uint16_t* __restrict__ lc = rq.lc;
  const float* __restrict__ x = rq.x;
  const float* __restrict__ y = rq.y;
  float2* __restrict__ T = rq.T;
  __shared__ float2 win[kXchCells];
  const int cb = blockIdx.x / kXchSpreadSplit, part = blockIdx.x % kXchSpreadSplit;
  const int t = threadIdx.x;
  const int c0 = cb * cpb;
  const int nc = min(cpb, m - c0);
  {
    constexpr int W = kXchCells / NT;
    float xv[W], yv[W];
#pragma unroll
    for (int k = 0; k < W; ++k) {
      const int i = c0 + min(t + k * NT, nc - 1);
      xv[k] = x[i];
      yv[k] = y[i];
    }
#pragma unroll
    for (int k = 0; k < W; ++k)
      if (t + k * NT < nc) win[t + k * NT] = make_float2(xv[k], yv[k]);
  }
  __syncthreads();
  const int b0 = cb_a_ptr[cb], b1 = cb_a_ptr[cb + 1];
  const int len = (b1 - b0 + kXchSpreadSplit - 1) / kXchSpreadSplit;
  const int a0 = b0 + part * len, a1 = min(b1, a0 + len);
  if (a0 >= a1) return;
  // pairs of consecutive A positions aligned to 2, consecutive pairs on
  // consecutive lanes: one 4-byte load of their cell indices and one 16-byte
  // store of their positions per pair, both coalesced across the wavefront;
  // a pair straddling either end of the range is stored only inside it (its
  // index load stays inside the index allocation)
  const int g0 = a0 >> 1, g1 = (a1 + 1) >> 1;
  const uint32_t* lc2 = reinterpret_cast<const uint32_t*>(lc);
  float4* T2 = reinterpret_cast<float4*>(T);
  constexpr int U = 8;
  for (int g = g0 + t; g < g1; g += U * NT) {
    uint32_t q[U];
#pragma unroll
    for (int k = 0; k < U; ++k) q[k] = lc2[min(g + k * NT, g1 - 1)];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int gg = g + k * NT;
      if (gg >= g1) continue;
      const float2 v0 = win[min((int)(q[k] & 0xffffu), kXchCells - 1)];
      const float2 v1 = win[min((int)(q[k] >> 16), kXchCells - 1)];
      const int a = gg * 2;
      if (a >= a0 && a + 2 <= a1) {
        T2[gg] = make_float4(v0.x, v0.y, v1.x, v1.y);
      } else {
        if (a >= a0) T[a] = v0;
        if (a + 1 < a1) T[a + 1] = v1;
      }
    }
  }
}

// Weighted-average terms of one axis with the exponentials computed once:
// e+ = exp((X - M)/gamma), e- = exp((L - X)/gamma) (fast exp2-based exp: the
// arguments are <= 0 and the terms that matter are near 0).
__device__ __forceinline__ float fexp(float v) { return __expf(v); }

// One net block: cell positions and pin offsets staged in LDS in CSR order,
// nets evaluated from LDS, gradients written back over the pins' positions in
// T.  LDS: pos[cap], off[cap] (dynamic, 16 bytes per pin of the block).
// LSE: the log-sum-exp model in place of the weighted average (same sums;
// the gradient is e+/S+ - e-/S-, the value (M - L) + gamma (ln S+ + ln S-)).
template <int STAGE, bool LSE, int NB>
__global__ void __launch_bounds__(NW) k_xch_wa(XchBatch<NB> xb) {
  const XchReq& rq = xb.r[blockIdx.y];
  const int k = blockIdx.x, t = threadIdx.x, nblk = rq.nnb;
  if (k >= nblk) return;
  const int num_pins = rq.num_pins, cap = rq.cap;
  const int32_t* __restrict__ net_ptr = rq.net_ptr;
  const int32_t* __restrict__ nb_net_ptr = rq.nb_net_ptr;
  const uint32_t* __restrict__ nmeta = rq.nmeta;
  const int32_t* __restrict__ a_of_b = rq.a_of_b;
  const uint16_t* __restrict__ lcsr = rq.lcsr;
  const float* __restrict__ pin_dx = rq.pin_dx;
  const float* __restrict__ pin_dy = rq.pin_dy;
  const float gamma = rq.dgamma ? rq.dgamma[0] : rq.gamma;
  const float inv_gamma = rq.dgamma ? 1.0f / gamma : rq.inv_gamma;
  float2* __restrict__ T = rq.T;
  double* __restrict__ part = rq.part;
  double* __restrict__ net_wl = rq.net_wl;
  double* __restrict__ net_hp = rq.net_hp;
  extern __shared__ float2 smem[];
  float2* pos = smem;
  float2* off = smem + cap;
  __shared__ uint32_t bigmeta[NW];   // extents of the last NW nets of the order
  __shared__ int q_big, q_small;     // work counters
  const int lane = t & (kWave - 1), wv = t / kWave;
  const int e0 = nb_net_ptr[k], e1 = nb_net_ptr[k + 1];
  const int p0 = net_ptr[e0], p1 = net_ptr[e1];
  const int np = p1 - p0;
  double acc_wa = 0.0, acc_hp = 0.0;
  if (np > 0 && np <= cap && np <= STAGE * NW) {
    // 0. net extents, read before the staging loads so that the latency of
    // both overlaps: the last NW entries of the order (the large nets, largest
    // first) for LDS, and this wavefront's first chunk of small nets.
    const int nn = e1 - e0;
    constexpr int NWV = NW / kWave;
    const uint32_t* meta = nmeta + e0;
    const uint32_t mbig = meta[max(nn - 1 - t, 0)];
    const uint32_t msm0 = meta[min(wv * kWave + lane, nn - 1)];
    // 1. stage: off[csr offset] = pin offset (coalesced), pos[csr offset] =
    // cell position read from T in B order (runs of consecutive A positions).
    // Loads are unconditional (index clamped into the block) so that each
    // batch is in flight at once; only the LDS stores are masked.
    int av[STAGE], lv[STAGE];
    {
      float dx[STAGE], dy[STAGE];
      const int blast = p1 - 1;
#pragma unroll
      for (int j = 0; j < STAGE; ++j) {
        const int b = min(p0 + t + j * NW, blast);
        av[j] = a_of_b[b];
        lv[j] = lcsr[b];
        dx[j] = pin_dx[b];
        dy[j] = pin_dy[b];
      }
#pragma unroll
      for (int j = 0; j < STAGE; ++j) {
        av[j] = min((unsigned)av[j], (unsigned)(num_pins - 1));
        lv[j] = min(lv[j], cap - 1);
      }
      float2 q[STAGE];
#pragma unroll
      for (int j = 0; j < STAGE; ++j) q[j] = T[av[j]];
#pragma unroll
      for (int j = 0; j < STAGE; ++j) {
        if (p0 + t + j * NW < p1) {
          off[t + j * NW] = make_float2(dx[j], dy[j]);
          pos[lv[j]] = q[j];
        }
      }
    }
    bigmeta[t] = mbig;
    if (t == 0) {
      q_big = 0;
      q_small = NWV;   // chunks 0..NWV-1 are the wavefronts' first ones
    }
    __syncthreads();

    // 2. nets in degree order, work handed out by block-wide counters so
    // that every wavefront stays busy until the block's nets run out.  Nets
    // above kSmall sit at the back of the order, largest class last: each is
    // taken by one wavefront, largest first (three passes over its pins in
    // LDS: pass 1 turns positions into pin coordinates relative to the first
    // pin's cell, pass 3 overwrites them with the gradient).  Then the
    // others: one lane per net, a wavefront per chunk of kWave nets of
    // (nearly) equal degree, loops as long as the chunk's largest degree.
    for (;;) {
      int j = 0;
      if (lane == 0) j = atomicAdd(&q_big, 1);
      j = __builtin_amdgcn_readfirstlane(j);
      if (j >= nn) break;
      // beyond the NW staged extents (more than NW large nets): from memory
      const uint32_t mj = j < NW ? bigmeta[j] : meta[nn - 1 - j];
      const int deg = (int)(mj & 0xffffu);
      if (deg <= kSmall) break;   // every net left is small
      // extents come from the index; kept inside the staged pins whatever it
      // holds, so a block never leaves its LDS
      const int b0 = min((int)(mj >> 16), np - 1), b1 = min(b0 + deg, np);
      const float2 r = pos[b0];
      wave_lds_sync();
      constexpr int H = 4;   // pins per lane whose LDS loads are issued together
      float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
      for (int l = b0 + lane; l < b1; l += H * kWave) {
        float2 c[H], d[H];
#pragma unroll
        for (int u = 0; u < H; ++u) {
          const int li = min(l + u * kWave, b1 - 1);
          c[u] = pos[li];
          d[u] = off[li];
        }
#pragma unroll
        for (int u = 0; u < H; ++u) {
          if (l + u * kWave < b1) {
            const float X = (c[u].x - r.x) + d[u].x, Y = (c[u].y - r.y) + d[u].y;
            pos[l + u * kWave] = make_float2(X, Y);
            mx = fmaxf(mx, X);
            lx = fminf(lx, X);
            my = fmaxf(my, Y);
            ly = fminf(ly, Y);
          }
        }
      }
      mx = wave_max_dpp(mx);
      lx = wave_min_dpp(lx);
      my = wave_max_dpp(my);
      ly = wave_min_dpp(ly);
      wave_lds_sync();
      float spx = 0.f, tpx = 0.f, smx = 0.f, tmx = 0.f;
      float spy = 0.f, tpy = 0.f, smy = 0.f, tmy = 0.f;
      for (int l = b0 + lane; l < b1; l += H * kWave) {
        float2 c[H];
#pragma unroll
        for (int u = 0; u < H; ++u) c[u] = pos[min(l + u * kWave, b1 - 1)];
#pragma unroll
        for (int u = 0; u < H; ++u) {
          if (l + u * kWave < b1) {
            float dd = c[u].x - mx, ee = fexp(dd * inv_gamma);
            spx += ee;
            tpx += dd * ee;
            dd = c[u].x - lx;
            ee = fexp(-dd * inv_gamma);
            smx += ee;
            tmx += dd * ee;
            dd = c[u].y - my;
            ee = fexp(dd * inv_gamma);
            spy += ee;
            tpy += dd * ee;
            dd = c[u].y - ly;
            ee = fexp(-dd * inv_gamma);
            smy += ee;
            tmy += dd * ee;
          }
        }
      }
      spx = wave_sum_dpp(spx);
      tpx = wave_sum_dpp(tpx);
      smx = wave_sum_dpp(smx);
      tmx = wave_sum_dpp(tmx);
      spy = wave_sum_dpp(spy);
      tpy = wave_sum_dpp(tpy);
      smy = wave_sum_dpp(smy);
      tmy = wave_sum_dpp(tmy);
      const float rspx = 1.0f / spx, rsmx = 1.0f / smx;
      const float rspy = 1.0f / spy, rsmy = 1.0f / smy;
      const float wpx = tpx * rspx, wmx = tmx * rsmx;
      const float wpy = tpy * rspy, wmy = tmy * rsmy;
      for (int l = b0 + lane; l < b1; l += H * kWave) {
        float2 c[H];
#pragma unroll
        for (int u = 0; u < H; ++u) c[u] = pos[min(l + u * kWave, b1 - 1)];
#pragma unroll
        for (int u = 0; u < H; ++u) {
          if (l + u * kWave < b1) {
            const float dpx = c[u].x - mx, dmx = c[u].x - lx;
            const float dpy = c[u].y - my, dmy = c[u].y - ly;
            if (LSE)
              pos[l + u * kWave] = make_float2(
                  fexp(dpx * inv_gamma) * rspx - fexp(-dmx * inv_gamma) * rsmx,
                  fexp(dpy * inv_gamma) * rspy - fexp(-dmy * inv_gamma) * rsmy);
            else
              pos[l + u * kWave] = make_float2(
                  fexp(dpx * inv_gamma) * rspx * (1.0f + (dpx - wpx) * inv_gamma) -
                      fexp(-dmx * inv_gamma) * rsmx * (1.0f - (dmx - wmx) * inv_gamma),
                  fexp(dpy * inv_gamma) * rspy * (1.0f + (dpy - wpy) * inv_gamma) -
                      fexp(-dmy * inv_gamma) * rsmy * (1.0f - (dmy - wmy) * inv_gamma));
          }
        }
      }
      if (lane == 0) {
        const double vw = net_wl_value<LSE>(mx, lx, wpx, wmx, spx, smx, gamma) +
                          net_wl_value<LSE>(my, ly, wpy, wmy, spy, smy, gamma);
        const double vh = (double)(mx - lx) + (double)(my - ly);
        acc_wa += vw;
        acc_hp += vh;
        if (net_wl) {
          net_wl[p0 + b0] = vw;
          net_hp[p0 + b0] = vh;
        }
      }
    }

    // small nets: chunk c holds order entries c * kWave + lane; a
    // wavefront's first chunk is its own (extents read before staging), the
    // rest come from the counter, each one's extents read while the previous
    // chunk is evaluated
    int cc = wv;
    uint32_t mcur = msm0;
    for (;;) {
      if (cc * kWave >= nn) break;
      int cn = 0;
      if (lane == 0) cn = atomicAdd(&q_small, 1);
      cn = __builtin_amdgcn_readfirstlane(cn);
      uint32_t mnext = 0u;
      if (cn * kWave < nn) mnext = meta[min(cn * kWave + lane, nn - 1)];
      const int li = cc * kWave + lane;
      int deg = li < nn ? (int)(mcur & 0xffffu) : 0;
      if (deg > kSmall) deg = 0;   // done above
      // kept inside the staged pins whatever the index holds
      const int l0 = min((int)(mcur >> 16), np - 1);
      deg = min(deg, np - l0);
      // the chunk's largest small degree, uniform across the wavefront
      const int wdeg = wave_max_dpp_i(deg);
      if (deg == 1) {
        // a one-pin net: no gradient, zero wirelength and half-perimeter
        pos[l0] = make_float2(0.0f, 0.0f);
        if (net_wl) {
          net_wl[p0 + l0] = 0.0;
          net_hp[p0 + l0] = 0.0;
        }
      }
      if (wdeg >= 2) {
        float px[kSmall], py[kSmall];
        const float2 r = pos[deg >= 1 ? l0 : 0];
        float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
#pragma unroll
        for (int j = 0; j < kSmall; ++j) {
          if (j < wdeg) {
            px[j] = 0.0f;
            py[j] = 0.0f;
            if (j < deg) {
              const float2 c = pos[l0 + j], d = off[l0 + j];
              px[j] = (c.x - r.x) + d.x;
              py[j] = (c.y - r.y) + d.y;
              mx = fmaxf(mx, px[j]);
              lx = fminf(lx, px[j]);
              my = fmaxf(my, py[j]);
              ly = fminf(ly, py[j]);
            }
          }
        }
        float epx[kSmall], emx[kSmall], epy[kSmall], emy[kSmall];
        float spx = 0.f, tpx = 0.f, smx = 0.f, tmx = 0.f;
        float spy = 0.f, tpy = 0.f, smy = 0.f, tmy = 0.f;
#pragma unroll
        for (int j = 0; j < kSmall; ++j) {
          if (j < wdeg) {
            const bool in = j < deg;
            const float dpx = px[j] - mx, dmx = px[j] - lx;
            const float dpy = py[j] - my, dmy = py[j] - ly;
            epx[j] = in ? fexp(dpx * inv_gamma) : 0.0f;
            emx[j] = in ? fexp(-dmx * inv_gamma) : 0.0f;
            epy[j] = in ? fexp(dpy * inv_gamma) : 0.0f;
            emy[j] = in ? fexp(-dmy * inv_gamma) : 0.0f;
            spx += epx[j];
            tpx += dpx * epx[j];
            smx += emx[j];
            tmx += dmx * emx[j];
            spy += epy[j];
            tpy += dpy * epy[j];
            smy += emy[j];
            tmy += dmy * emy[j];
          }
        }
        if (deg >= 2) {
          const float rspx = 1.0f / spx, rsmx = 1.0f / smx;
          const float rspy = 1.0f / spy, rsmy = 1.0f / smy;
          const float wpx = tpx * rspx, wmx = tmx * rsmx;
          const float wpy = tpy * rspy, wmy = tmy * rsmy;
#pragma unroll
          for (int j = 0; j < kSmall; ++j) {
            if (j < wdeg && j < deg) {
              const float dpx = px[j] - mx, dmx = px[j] - lx;
              const float dpy = py[j] - my, dmy = py[j] - ly;
              if (LSE)
                pos[l0 + j] = make_float2(epx[j] * rspx - emx[j] * rsmx,
                                          epy[j] * rspy - emy[j] * rsmy);
              else
                pos[l0 + j] = make_float2(
                    epx[j] * rspx * (1.0f + (dpx - wpx) * inv_gamma) -
                        emx[j] * rsmx * (1.0f - (dmx - wmx) * inv_gamma),
                    epy[j] * rspy * (1.0f + (dpy - wpy) * inv_gamma) -
                        emy[j] * rsmy * (1.0f - (dmy - wmy) * inv_gamma));
            }
          }
          const double vw = net_wl_value<LSE>(mx, lx, wpx, wmx, spx, smx, gamma) +
                            net_wl_value<LSE>(my, ly, wpy, wmy, spy, smy, gamma);
          const double vh = (double)(mx - lx) + (double)(my - ly);
          acc_wa += vw;
          acc_hp += vh;
          if (net_wl) {
            net_wl[p0 + l0] = vw;
            net_hp[p0 + l0] = vh;
          }
        }
      }
      cc = cn;
      mcur = mnext;
    }
    __syncthreads();

    // 3. gradients back to the pins' A positions
#pragma unroll
    for (int j = 0; j < STAGE; ++j)
      if (p0 + t + j * NW < p1) T[av[j]] = pos[lv[j]];
  }
  block_sum_to<false>(acc_wa, &part[k]);
  block_sum_to<false>(acc_hp, &part[nblk + k]);
}

// The gradient of every cell (CellGradArgs): its density part plus the sum
// of the gradients in T of its pins.  One block per cell
// block: the block streams the cell block's A range of T together with the
// cell-local index lc (both coalesced) and adds each pin into per-cell
// accumulators in LDS.  The adds are 64-bit integer adds of the gradients in
// fixed point (units of 2^-S), so the sums come out the same whatever order
// the atomics land in (LDS float atomics would not, and run several times
// slower).  One pin's gradient component is bounded by 1.15 + ln(largest
// degree) (its softmax weight times one plus its distance to the weighted
// mean, and that distance is at most ln(degree) in units of gamma), so S is
// the largest scale that keeps every pin within a 32-bit conversion; the
// 64-bit sums then hold any number of pins.  A non-finite pin gradient makes
// its cell's sum NaN.
template <int MODE, bool DENS, int NB>
__global__ void __launch_bounds__(kSumThreads) k_xch_cellsum(SumBatch<NB> sb) {
  const SumReq& rq = sb.r[blockIdx.y];
  const int cb = blockIdx.x, t = threadIdx.x;
  if (cb >= rq.ncb) return;
  const int m = rq.m, cpb = rq.cpb;
  const int32_t* __restrict__ cb_a_ptr = rq.cb_a_ptr;
  const uint16_t* __restrict__ lc = rq.lc;
  const float2* __restrict__ T = rq.T;
  const float scale = rq.fx_scale;
  const double inv_scale = rq.inv_scale;
  const CellGradArgs& a = rq.a;
  __shared__ unsigned long long ax[kXchCells], ay[kXchCells];
  __shared__ unsigned char bad[kXchCells];
  // the block's A range, then the first-band entry of each of the thread's
  // cells and its first group of pins: all in flight while LDS is cleared
  const int a0 = cb_a_ptr[cb], a1 = cb_a_ptr[cb + 1];
  constexpr int PC = kXchCells / kSumThreads;
  const int c0 = cb * cpb;
  int ep[PC];
  if (DENS) {
#pragma unroll
    for (int k = 0; k < PC; ++k) ep[k] = a.epos[min(c0 + t + k * kSumThreads, m - 1)];
  }
  // pairs of consecutive A positions aligned to 2, consecutive pairs on
  // consecutive lanes (one 4-byte load of their cell indices and one 16-byte
  // load of their gradients, coalesced); positions outside the range are
  // skipped (the loads of a straddling pair stay inside the allocations)
  const int g0 = a0 >> 1, g1 = (a1 + 1) >> 1;
  const uint32_t* lc2 = reinterpret_cast<const uint32_t*>(lc);
  const float4* T2 = reinterpret_cast<const float4*>(T);
  constexpr int U = 4, STEP = U * kSumThreads;
  // two groups of U pairs per thread in flight: the next group's loads are
  // issued before the current group's adds
  uint32_t q[U], qn[U];
  float4 v[U], vn[U];
  auto fetch = [&](uint32_t (&qq)[U], float4 (&vv)[U], int g) {
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int gg = min(g + k * kSumThreads, g1 - 1);
      qq[k] = lc2[gg];
      vv[k] = T2[gg];
    }
  };
  int g = g0 + t;
  if (g < g1) fetch(q, v, g);
  for (int c = t; c < kXchCells; c += kSumThreads) {
    ax[c] = 0ull;
    ay[c] = 0ull;
    bad[c] = 0;
  }
  __syncthreads();
  for (; g < g1; g += STEP) {
    if (g + STEP < g1) fetch(qn, vn, g + STEP);
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const int gg = g + k * kSumThreads;
      if (gg >= g1) continue;
      const int a = gg * 2;
#pragma unroll
      for (int e = 0; e < 2; ++e) {
        if (a + e < a0 || a + e >= a1) continue;
        const int l = min((int)(e ? q[k] >> 16 : q[k] & 0xffffu), kXchCells - 1);
        const float gxv = e ? v[k].z : v[k].x, gyv = e ? v[k].w : v[k].y;
        if (fabsf(gxv) <= 3.0e38f && fabsf(gyv) <= 3.0e38f) {
          atomicAdd(&ax[l], (unsigned long long)(long long)__float2int_rn(gxv * scale));
          atomicAdd(&ay[l], (unsigned long long)(long long)__float2int_rn(gyv * scale));
        } else {
          bad[l] = 1;
        }
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      q[k] = qn[k];
      v[k] = vn[k];
    }
  }
  __syncthreads();
  // each cell's gradient: its density part from its first-band entry (one
  // 8-byte read; all of a thread's reads issued together) or, for a cell
  // without one, from the maps; plus its wirelength sum (DENS = false: the
  // wirelength sum alone, written or added to the gradient)
  float2 d[PC];
  const float lam = DENS && a.dscale ? a.dscale[0] : a.scale;
  if (DENS) {
#pragma unroll
    for (int k = 0; k < PC; ++k) d[k] = a.egrad[max(ep[k], 0)];
  } else if (a.accumulate) {
#pragma unroll
    for (int k = 0; k < PC; ++k) {
      const int ci = min(c0 + t + k * kSumThreads, m - 1);
      d[k] = make_float2(a.gx[ci], a.gy[ci]);
    }
  }
#pragma unroll
  for (int k = 0; k < PC; ++k) {
    const int c = t + k * kSumThreads, ci = c0 + c;
    if (c >= cpb || ci >= m) break;
    if (DENS && ep[k] < 0)
      d[k] = cell_density_grad<MODE, true>(a.g, a.x[ci], a.y[ci], a.w[ci], a.h[ci], nullptr,
                                           nullptr, a.exy, a.psi);
    const float sx = bad[c] ? __builtin_nanf("") : (float)((double)(long long)ax[c] * inv_scale);
    const float sy = bad[c] ? __builtin_nanf("") : (float)((double)(long long)ay[c] * inv_scale);
    if (DENS) {
      a.gx[ci] = lam * d[k].x + sx;
      a.gy[ci] = lam * d[k].y + sy;
    } else if (a.accumulate) {
      a.gx[ci] = d[k].x + sx;
      a.gy[ci] = d[k].y + sy;
    } else {
      a.gx[ci] = sx;
      a.gy[ci] = sy;
    }
  }
  if (cb == a.fin_block) {
    __syncthreads();
    eval_scalars<kSumThreads>(a.fin);
  }
}

}  // namespace

// Fixed-point scale 2^S of the cell sums: the largest S <= 26 with
// bound * 2^S <= 2^30 for the largest pin gradient component bound.
static int cellsum_shift(int max_degree) {
  const double bound = 1.15 + log((double)(max_degree > 2 ? max_degree : 2));
  int S = 26;
  while (S > 0 && bound * ldexp(1.0, S) > ldexp(1.0, 30)) --S;
  return S;
}

SumReq sum_req(const XchDims& d, const XchIndex& X, const float2* T, const CellGradArgs& a) {
  SumReq q;
  q.m = d.m;
  q.cpb = d.cpb;
  q.ncb = d.ncb;
  q.cb_a_ptr = X.cb_a_ptr;
  q.lc = X.lc;
  q.T = T;
  const int S = cellsum_shift(d.max_degree);
  q.fx_scale = (float)ldexp(1.0, S);
  q.inv_scale = ldexp(1.0, -S);
  q.a = a;
  return q;
}

template <int NB>
static hipError_t cellsum_nb(const SumBatch<NB>& sb, int max_ncb, int grad_mode, bool dens,
                             hipStream_t s) {
  const dim3 grid(max_ncb, sb.count), block(kSumThreads);
  if (!dens)
    hipLaunchKernelGGL((k_xch_cellsum<FFTPL_GRAD_FIELD, false, NB>), grid, block, 0, s, sb);
  else if (grad_mode == FFTPL_GRAD_EXACT)
    hipLaunchKernelGGL((k_xch_cellsum<FFTPL_GRAD_EXACT, true, NB>), grid, block, 0, s, sb);
  else
    hipLaunchKernelGGL((k_xch_cellsum<FFTPL_GRAD_FIELD, true, NB>), grid, block, 0, s, sb);
  return hipGetLastError();
}

hipError_t launch_xch_cellsum_batch(const SumReq* reqs, int count, int grad_mode, bool dens,
                                    hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxBatch) return hipErrorInvalidValue;
  int max_ncb = 0;
  for (int i = 0; i < count; ++i)
    if (reqs[i].m > 0) max_ncb = std::max(max_ncb, reqs[i].ncb);
  if (max_ncb == 0) return hipSuccess;
  if (count == 1) {
    SumBatch<1> sb;
    sb.count = 1;
    sb.r[0] = reqs[0];
    return cellsum_nb(sb, max_ncb, grad_mode, dens, s);
  }
  SumBatch<kMaxBatch> sb;
  sb.count = count;
  for (int i = 0; i < count; ++i) sb.r[i] = reqs[i];
  return cellsum_nb(sb, max_ncb, grad_mode, dens, s);
}

hipError_t launch_xch_cellsum(const XchDims& d, const XchIndex& X, const float2* T,
                              const CellGradArgs& a, int grad_mode, hipStream_t s) {
  if (d.m <= 0) return hipSuccess;
  const SumReq q = sum_req(d, X, T, a);
  return launch_xch_cellsum_batch(&q, 1, grad_mode, true, s);
}

XchReq xch_req(const XchDims& d, const XchIndex& X, const float* x, const float* y, float2* T,
               const int32_t* net_ptr, const float* pin_dx, const float* pin_dy, float gamma,
               double* part) {
  XchReq q;
  q.m = d.m;
  q.cpb = d.cpb;
  q.ncb = d.ncb;
  q.cb_a_ptr = X.cb_a_ptr;
  q.lc = X.lc;
  q.x = x;
  q.y = y;
  q.T = T;
  q.num_pins = d.num_pins;
  q.cap = d.cap;
  q.nnb = d.nnb;
  q.net_ptr = net_ptr;
  q.nb_net_ptr = X.nb_net_ptr;
  q.nmeta = X.nmeta;
  q.a_of_b = X.a_of_b;
  q.lcsr = X.lcsr;
  q.pin_dx = pin_dx;
  q.pin_dy = pin_dy;
  q.gamma = gamma;
  q.inv_gamma = 1.0f / gamma;
  q.part = part;
  return q;
}

template <int NB>
static hipError_t spread_nb(const XchBatch<NB>& xb, int max_ncb, hipStream_t s) {
  hipLaunchKernelGGL((k_xch_spread<NB>), dim3(max_ncb * kXchSpreadSplit, xb.count), dim3(NT),
                     0, s, xb);
  return hipGetLastError();
}

hipError_t launch_xch_spread_batch(const XchReq* reqs, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxBatch) return hipErrorInvalidValue;
  int max_ncb = 0;
  for (int i = 0; i < count; ++i) max_ncb = std::max(max_ncb, reqs[i].ncb);
  if (max_ncb == 0) return hipSuccess;
  if (count == 1) {
    XchBatch<1> xb;
    xb.count = 1;
    xb.r[0] = reqs[0];
    return spread_nb(xb, max_ncb, s);
  }
  XchBatch<kMaxBatch> xb;
  xb.count = count;
  for (int i = 0; i < count; ++i) xb.r[i] = reqs[i];
  return spread_nb(xb, max_ncb, s);
}

hipError_t launch_xch_spread(const XchDims& d, const XchIndex& X, const float* x,
                             const float* y, float2* T, hipStream_t s) {
  if (d.ncb <= 0) return hipSuccess;
  const XchReq q = xch_req(d, X, x, y, T, nullptr, nullptr, nullptr, 1.0f, nullptr);
  return launch_xch_spread_batch(&q, 1, s);
}

// more than 64 KiB of dynamic LDS has to be allowed explicitly, once per
// device and kernel instantiation (setting it twice from racing threads is
// harmless)
template <typename K>
static hipError_t allow_big_lds(K* kernel, std::atomic<bool>* flags) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  if (!flags[dev].load(std::memory_order_acquire)) {
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                            hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)(sizeof(float2) * 2 * kXchPinCap));
    if (e != hipSuccess) return e;
    flags[dev].store(true, std::memory_order_release);
  }
  return hipSuccess;
}

template <bool LSE, int NB>
static hipError_t wa_nb(const XchBatch<NB>& xb, int max_nnb, int max_cap, hipStream_t s) {
  const size_t lds = sizeof(float2) * 2 * (size_t)max_cap;
  const dim3 grid(max_nnb, xb.count);
  if (max_cap <= kXchPinLds2) {
    hipLaunchKernelGGL((k_xch_wa<kStageS, LSE, NB>), grid, dim3(NW), lds, s, xb);
  } else {
    static std::atomic<bool> attr[kMaxDevices];
    const hipError_t e = allow_big_lds(&k_xch_wa<kStageL, LSE, NB>, attr);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_xch_wa<kStageL, LSE, NB>), grid, dim3(NW), lds, s, xb);
  }
  return hipGetLastError();
}

template <bool LSE>
static hipError_t wa_model(const XchReq* reqs, int count, hipStream_t s) {
  int max_nnb = 0, max_cap = 1;
  for (int i = 0; i < count; ++i) {
    max_nnb = std::max(max_nnb, reqs[i].nnb);
    max_cap = std::max(max_cap, reqs[i].cap);
  }
  if (max_nnb == 0) return hipSuccess;
  if (count == 1) {
    XchBatch<1> xb;
    xb.count = 1;
    xb.r[0] = reqs[0];
    return wa_nb<LSE, 1>(xb, max_nnb, max_cap, s);
  }
  XchBatch<kMaxBatch> xb;
  xb.count = count;
  for (int i = 0; i < count; ++i) xb.r[i] = reqs[i];
  return wa_nb<LSE, kMaxBatch>(xb, max_nnb, max_cap, s);
}

hipError_t launch_xch_wa_batch(const XchReq* reqs, int count, int wl_model, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxBatch) return hipErrorInvalidValue;
  return wl_model == FFTPL_WL_LSE ? wa_model<true>(reqs, count, s)
                                  : wa_model<false>(reqs, count, s);
}

hipError_t launch_xch_wa(const XchDims& d, const XchIndex& X, const int32_t* net_ptr,
                         const float* pin_dx, const float* pin_dy, float gamma, int wl_model,
                         float2* T, double* wa_part, hipStream_t s) {
  const XchReq q = xch_req(d, X, nullptr, nullptr, T, net_ptr, pin_dx, pin_dy, gamma, wa_part);
  return launch_xch_wa_batch(&q, 1, wl_model, s);
}

}  // namespace fftpl
