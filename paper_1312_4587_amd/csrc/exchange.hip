// Bucketed pin exchange for the weighted-average wirelength gradient
// (Eq. (3)) and HPWL (Eq. (1)).
//
// Nets pick their cells anywhere in the design, so handing cell positions to
// pins and pin gradients back to cells is a permutation of the pins.  Done
// directly, every pin costs one random 8-byte read and one random 8-byte
// write, each of which moves a whole cache line.  Here the permutation is
// split in two halves that both run through LDS:
//
//   cell blocks: kXchCells consecutive cells;
//   net blocks:  the nets whose first pin lies in [k*npt, (k+1)*npt), so a
//                block holds at most npt - 1 + max_degree <= kXchPinCap pins;
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
//   gather  (one thread per cell): the density gradient plus the sum of the
//           cell's pin gradients, read from T at the A positions the index
//           lists per cell (cell-major); the blocks of one cell block run on
//           one XCD, so its window of T is read from HBM once.
//
// The index (A/B layout) is built once per netlist by xch_build.
#include <math.h>

#include "fftpl_internal.hpp"

namespace fftpl {

namespace {

constexpr int NT = kXchThreads;
constexpr int kHdrInts = 16;
constexpr int32_t kXchMagic = 0x46584348;   // "FXCH"
constexpr int kSmall = 8;                   // degree handled by one thread
constexpr int NW = kXchWaThreads;
constexpr int kStage = (kXchPinCap + NW - 1) / NW;   // B positions per thread in wa

inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

int xch_dims(int m, int num_nets, int num_pins, int max_degree, XchDims* d) {
  if (m < 0 || num_nets < 0 || num_pins < 0 || max_degree < 0) return FFTPL_E_INVAL;
  int npt = kXchPinTarget;
  if (npt > kXchPinCap + 1 - max_degree) npt = kXchPinCap + 1 - max_degree;
  if (npt < kXchMinTarget) return FFTPL_E_UNSUPPORTED;
  XchDims r;
  r.m = m;
  r.num_nets = num_nets;
  r.num_pins = num_pins;
  r.max_degree = max_degree;
  r.npt = npt;
  r.ncb = (m + kXchCells - 1) / kXchCells;
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
  r.o_cp = off;
  off = align256(off + sizeof(int32_t) * ((size_t)m + 1));
  r.o_qa = off;
  off = align256(off + sizeof(int32_t) * (size_t)num_pins);
  r.index_bytes = off;
  // build workspace: counts / cursors, A starts, transposed counts, B starts,
  // scan block sums, flag and scan totals
  const size_t seg = (size_t)r.ncb * r.nnb;
  // ... then the cell-major index's counters and block sums, and each pin's
  // cell-major slot
  r.work_bytes = align256(sizeof(int32_t) * seg) * 4 +
                 align256(sizeof(int32_t) * ((seg + 1023) / 1024 + 1)) +
                 align256(sizeof(int32_t) * 4) +
                 align256(sizeof(int32_t) * ((size_t)m + (m + 1023) / 1024 + 1)) +
                 align256(sizeof(int32_t) * (size_t)num_pins);
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
  X.cell_ptr = reinterpret_cast<const int32_t*>(b + d.o_cp);
  X.qa = reinterpret_cast<const int32_t*>(b + d.o_qa);
  return X;
}

// ---------------------------------------------------------------------------
// Index build
// ---------------------------------------------------------------------------
namespace {

// nb_net_ptr[k] = first net whose first pin is >= k*npt (k < nnb); [nnb] = E.
__global__ void k_xi_netblocks(int num_nets, const int32_t* __restrict__ net_ptr, int npt,
                               int nnb, int32_t* __restrict__ nb_net_ptr) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k > nnb) return;
  if (k == nnb) {
    nb_net_ptr[k] = num_nets;
    return;
  }
  const int64_t target = (int64_t)k * npt;
  int lo = 0, hi = num_nets + 1;   // lower bound over net_ptr[0..E]
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if ((int64_t)net_ptr[mid] < target)
      lo = mid + 1;
    else
      hi = mid;
  }
  nb_net_ptr[k] = lo < num_nets ? lo : num_nets;
}

// Checks the CSR (net_ptr[0] = 0, net_ptr[E] = P, monotone, degrees <=
// max_degree, pin cells in range) and, with PLACE = false, counts the pins of
// every (cell block, net block) segment; with PLACE = true, hands each pin its
// A and B positions (the same rank inside the segment on both sides).
template <bool PLACE>
__global__ void __launch_bounds__(256)
    k_xi_pins(int num_nets, const int32_t* __restrict__ net_ptr, int num_pins,
              const int32_t* __restrict__ pin_cell, int m, int max_degree, int npt, int ncb,
              int nnb, int32_t* __restrict__ cnt, const int32_t* __restrict__ seg_a,
              const int32_t* __restrict__ seg_bt, const int32_t* __restrict__ nb_net_ptr,
              int32_t* __restrict__ a_of_b, uint16_t* __restrict__ lcsr,
              uint16_t* __restrict__ lc, const int32_t* __restrict__ pin_slot,
              int32_t* __restrict__ qa, int32_t* __restrict__ flag) {
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
  const int k = p0 / npt;
  if (k >= nnb) {
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
    const int cb = c / kXchCells;
    const size_t idx = (size_t)cb * nnb + k;
    if (!PLACE) {
      atomicAdd(&cnt[idx], 1);
    } else {
      const int r = atomicAdd(&cnt[idx], 1);
      const int a = seg_a[idx] + r;
      const int b = seg_bt[(size_t)k * ncb + cb] + r;
      a_of_b[b] = a;
      lcsr[b] = (uint16_t)(p - base);
      lc[a] = (uint16_t)(c - cb * kXchCells);
      qa[pin_slot[p]] = a;
    }
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
                            int m, int num_nets, int max_degree, int npt) {
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
  }
}

}  // namespace

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
  w += align256(sizeof(int32_t) * 4);
  int32_t* nl_work = reinterpret_cast<int32_t*>(w);
  w += align256(sizeof(int32_t) * ((size_t)d.m + (d.m + 1023) / 1024 + 1));
  int32_t* pin_slot = reinterpret_cast<int32_t*>(w);

  char* ib = static_cast<char*>(index);
  int32_t* hdr = reinterpret_cast<int32_t*>(ib + d.o_hdr);
  int32_t* cb_a_ptr = reinterpret_cast<int32_t*>(ib + d.o_cb);
  int32_t* nb_net_ptr = reinterpret_cast<int32_t*>(ib + d.o_nb);
  int32_t* a_of_b = reinterpret_cast<int32_t*>(ib + d.o_ab);
  uint16_t* lcsr = reinterpret_cast<uint16_t*>(ib + d.o_lcsr);
  uint16_t* lc = reinterpret_cast<uint16_t*>(ib + d.o_lc);
  int32_t* cell_ptr = reinterpret_cast<int32_t*>(ib + d.o_cp);
  int32_t* qa = reinterpret_cast<int32_t*>(ib + d.o_qa);

  const int E = d.num_nets, P = d.num_pins;
  const dim3 net_grid((E + 255) / 256 > 0 ? (E + 255) / 256 : 1);
  hipError_t e = launch_zero_i32(cnt, (int64_t)seg, s);
  if (e == hipSuccess) e = launch_zero_i32(flag, 4, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_xi_netblocks, dim3((d.nnb + 256) / 256), dim3(256), 0, s, E, net_ptr,
                       d.npt, d.nnb, nb_net_ptr);
    e = hipGetLastError();
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_xi_pins<false>), net_grid, dim3(256), 0, s, E, net_ptr, P, pin_cell,
                       d.m, d.max_degree, d.npt, d.ncb, d.nnb, cnt, nullptr, nullptr, nullptr,
                       nullptr, nullptr, nullptr, nullptr, nullptr, flag);
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
                       P, seg_a, cb_a_ptr, hdr, d.m, E, d.max_degree, d.npt);
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
  e = launch_netlist_index(d.m, P, pin_cell, cell_ptr, pin_slot, nl_work, s);
  if (e == hipSuccess) e = launch_zero_i32(cnt, (int64_t)seg, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL((k_xi_pins<true>), net_grid, dim3(256), 0, s, E, net_ptr, P, pin_cell,
                       d.m, d.max_degree, d.npt, d.ncb, d.nnb, cnt, seg_a, seg_bt, nb_net_ptr,
                       a_of_b, lcsr, lc, pin_slot, qa, flag);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? FFTPL_OK : FFTPL_E_DEVICE;
}

// ---------------------------------------------------------------------------
// Evaluation kernels
// ---------------------------------------------------------------------------
namespace {

// T[a] = (x, y) of pin a's cell, over the block's A range.
__global__ void __launch_bounds__(NT)
    k_xch_spread(int m, const int32_t* __restrict__ cb_a_ptr, const uint16_t* __restrict__ lc,
                 const float* __restrict__ x, const float* __restrict__ y,
                 float2* __restrict__ T) {
  __shared__ float2 win[kXchCells];
  const int cb = blockIdx.x, t = threadIdx.x;
  const int c0 = cb * kXchCells;
  const int nc = min(kXchCells, m - c0);
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
  const int a0 = cb_a_ptr[cb], a1 = cb_a_ptr[cb + 1];
  // loads of one batch are unconditional (clamped index) so they are all in
  // flight together; only the stores are masked
  constexpr int U = 8;
  for (int a = a0 + t; a < a1; a += U * NT) {
    int l[U];
#pragma unroll
    for (int k = 0; k < U; ++k) l[k] = lc[min(a + k * NT, a1 - 1)];
#pragma unroll
    for (int k = 0; k < U; ++k)
      if (a + k * NT < a1) T[a + k * NT] = win[min(l[k], kXchCells - 1)];
  }
}

// One net block: cell positions and pin offsets staged in LDS in CSR order,
// nets evaluated from LDS, gradients written back over the pins' positions in
// T.
__global__ void __launch_bounds__(NW)
    k_xch_wa(int num_pins, const int32_t* __restrict__ net_ptr,
             const int32_t* __restrict__ nb_net_ptr, const int32_t* __restrict__ a_of_b,
             const uint16_t* __restrict__ lcsr, const float* __restrict__ pin_dx,
             const float* __restrict__ pin_dy, float inv_gamma, float2* __restrict__ T,
             double* __restrict__ part) {
  __shared__ float2 pos[kXchPinCap];
  __shared__ float2 off[kXchPinCap];
  const int k = blockIdx.x, t = threadIdx.x, nblk = gridDim.x;
  const int lane = t & (kWave - 1), wv = t / kWave;
  const int e0 = nb_net_ptr[k], e1 = nb_net_ptr[k + 1];
  const int p0 = net_ptr[e0], p1 = net_ptr[e1];
  const int np = p1 - p0;
  double acc_wa = 0.0, acc_hp = 0.0;
  if (np > 0 && np <= kXchPinCap) {
    // 1. stage: off[csr offset] = pin offset (coalesced), pos[csr offset] =
    // cell position read from T in B order (runs of consecutive A positions)
    // loads unconditional (index clamped into the block) so that each batch
    // is in flight at once; only the LDS stores are masked
    int av[kStage], lv[kStage];
    float dx[kStage], dy[kStage];
    const int blast = p1 - 1;
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      const int b = max(min(p0 + t + j * NW, blast), 0);
      av[j] = a_of_b[b];
      lv[j] = lcsr[b];
      dx[j] = pin_dx[b];
      dy[j] = pin_dy[b];
    }
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      av[j] = min((unsigned)av[j], (unsigned)(num_pins - 1));
      lv[j] = min(lv[j], kXchPinCap - 1);
    }
    float2 q[kStage];
#pragma unroll
    for (int j = 0; j < kStage; ++j) q[j] = T[av[j]];
#pragma unroll
    for (int j = 0; j < kStage; ++j) {
      if (p0 + t + j * NW < p1) {
        off[t + j * NW] = make_float2(dx[j], dy[j]);
        pos[lv[j]] = q[j];
      }
    }
    __syncthreads();

    // 2. nets, walked in chunks of kWave consecutive nets per wavefront (the
    // next chunk's pointers are loaded before the current chunk is done):
    // larger nets by the whole wavefront, three passes over the pins in LDS
    // (pass 1 turns positions into pin coordinates relative to the first
    // pin's cell, pass 3 overwrites them with the gradient); nets of degree
    // <= kSmall by one lane each.
    int e = e0 + wv * kWave + lane;
    int c0 = 0, c1 = 0;
    if (e < e1) {
      c0 = net_ptr[e];
      c1 = net_ptr[e + 1];
    }
    for (int base = e0 + wv * kWave; base < e1; base += NW, e += NW) {
      int n0 = 0, n1 = 0;
      if (e + NW < e1) {
        n0 = net_ptr[e + NW];
        n1 = net_ptr[e + NW + 1];
      }
      unsigned long long big = __ballot(c1 - c0 > kSmall);
      while (big) {
        const int src = __ffsll((long long)big) - 1;
        big &= big - 1;
        const int b0 = __shfl(c0, src, kWave) - p0, b1 = __shfl(c1, src, kWave) - p0;
        const float2 r = pos[b0];
        wave_lds_sync();
        float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
        for (int l = b0 + lane; l < b1; l += kWave) {
          const float2 c = pos[l], d = off[l];
          const float X = (c.x - r.x) + d.x, Y = (c.y - r.y) + d.y;
          pos[l] = make_float2(X, Y);
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
        for (int l = b0 + lane; l < b1; l += kWave) {
          const float2 c = pos[l];
          axis_accum(sx, c.x, mx, lx, inv_gamma);
          axis_accum(sy, c.y, my, ly, inv_gamma);
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
        for (int l = b0 + lane; l < b1; l += kWave) {
          const float2 c = pos[l];
          pos[l] = make_float2(axis_grad(c.x, mx, lx, wpx, wmx, rspx, rsmx, inv_gamma),
                               axis_grad(c.y, my, ly, wpy, wmy, rspy, rsmy, inv_gamma));
        }
        if (lane == src) {
          acc_wa += (double)((mx - lx) + wpx - wmx) + (double)((my - ly) + wpy - wmy);
          acc_hp += (double)(mx - lx) + (double)(my - ly);
        }
      }
      const int deg = c1 - c0, l0 = c0 - p0;
      if (deg == 1) {
        pos[l0] = make_float2(0.0f, 0.0f);
      } else if (deg >= 2 && deg <= kSmall) {
        float px[kSmall], py[kSmall];
        const float2 r = pos[l0];
        float mx = -INFINITY, lx = INFINITY, my = -INFINITY, ly = INFINITY;
#pragma unroll
        for (int j = 0; j < kSmall; ++j) {
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
        AxisSums sx = {0.f, 0.f, 0.f, 0.f}, sy = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int j = 0; j < kSmall; ++j) {
          if (j < deg) {
            axis_accum(sx, px[j], mx, lx, inv_gamma);
            axis_accum(sy, py[j], my, ly, inv_gamma);
          }
        }
        const float wpx = sx.tp / sx.sp, wmx = sx.tm / sx.sm;
        const float wpy = sy.tp / sy.sp, wmy = sy.tm / sy.sm;
        const float rspx = 1.0f / sx.sp, rsmx = 1.0f / sx.sm;
        const float rspy = 1.0f / sy.sp, rsmy = 1.0f / sy.sm;
#pragma unroll
        for (int j = 0; j < kSmall; ++j)
          if (j < deg)
            pos[l0 + j] = make_float2(axis_grad(px[j], mx, lx, wpx, wmx, rspx, rsmx, inv_gamma),
                                      axis_grad(py[j], my, ly, wpy, wmy, rspy, rsmy, inv_gamma));
        acc_wa += (double)((mx - lx) + wpx - wmx) + (double)((my - ly) + wpy - wmy);
        acc_hp += (double)(mx - lx) + (double)(my - ly);
      }
      c0 = n0;
      c1 = n1;
    }
    __syncthreads();

    // 3. gradients back to the pins' A positions
#pragma unroll
    for (int j = 0; j < kStage; ++j)
      if (p0 + t + j * NW < p1) T[av[j]] = pos[lv[j]];
  }
  block_sum_to<false>(acc_wa, &part[k]);
  block_sum_to<false>(acc_hp, &part[nblk + k]);
}

}  // namespace

hipError_t launch_xch_spread(const XchDims& d, const XchIndex& X, const float* x,
                             const float* y, float2* T, hipStream_t s) {
  if (d.ncb <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_xch_spread, dim3(d.ncb), dim3(NT), 0, s, d.m, X.cb_a_ptr, X.lc, x, y,
                     T);
  return hipGetLastError();
}

hipError_t launch_xch_wa(const XchDims& d, const XchIndex& X, const int32_t* net_ptr,
                         const float* pin_dx, const float* pin_dy, float gamma, float2* T,
                         double* wa_part, hipStream_t s) {
  hipLaunchKernelGGL(k_xch_wa, dim3(d.nnb), dim3(NW), 0, s, d.num_pins, net_ptr, X.nb_net_ptr,
                     X.a_of_b, X.lcsr, pin_dx, pin_dy, 1.0f / gamma, T, wa_part);
  return hipGetLastError();
}

}  // namespace fftpl
