// Banded density scatter (Eq. (2), Section III-B) without float atomics in
// global memory, which retire at roughly 20 G/s on the whole chip whatever
// their scope:
//   count: each block of kCellsPerBlock cells histograms the bands its
//          cells touch in LDS (plus one slot for cells too tall to list
//          per band) and stores the histogram (band-major);
//   scan:  one block per band turns its row of block counts into each
//          block's offset inside the band and the band's total (no global
//          atomics, whose contention on 256 counters would serialise);
//   place: the counting blocks write each cell's edges (bin units) into
//          every band it touches, at LDS-atomic ranks inside their slice;
//   accum: one block per band adds its entries into an LDS copy of its rows
//          and writes rho = base + rows once.  The LDS adds are 64-bit
//          integer adds of the overlaps in fixed point (every overlap lies in
//          [0, 1], units of 2^-31): they retire many times faster than LDS
//          float atomics, and the sums do not depend on the order of the
//          entries, so rho is the same on every run.
// Every thread issues the loads of kCellBatch cells (or entries) before it
// uses any of them, so each block keeps many misses in flight.
#include "fftpl_internal.hpp"

namespace fftpl {

static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

BandLayout band_layout(int n, int m, int num_nets, int num_pins, void* work,
                       size_t* bytes_out) {
  BandLayout L;
  L.n = n;
  L.rows = (n + 255) / 256;              // <= 4 rows for n <= 1024: rows*n <= 4096
  L.nb = (n + L.rows - 1) / L.rows;      // <= 256 bands; the last may be short
  L.m = m;
  L.nblk = m > 0 ? (m + kCellsPerBlock - 1) / kCellsPerBlock : 1;
  L.nwa = (num_nets + 255) / 256;
  // wirelength partials: 4 per 256 nets (slot path) or 2 per net block of at
  // least kXchMinTarget pins (exchange path)
  size_t nwp = 4 * (size_t)L.nwa;
  const size_t nxp = 2 * ((size_t)(num_pins + kXchMinTarget - 1) / kXchMinTarget + 1);
  if (nwp < nxp) nwp = nxp;
  size_t off = 0;
  const size_t o_wp = off;
  off = align256(off + sizeof(double) * nwp);
  const size_t o_xy = off;
  off = align256(off + sizeof(float2) * (size_t)m);
  const size_t o_pg = off;
  off = align256(off + sizeof(float2) * (size_t)num_pins);
  const size_t o_en = off;
  off = align256(off + sizeof(float4) * (size_t)kMaxBands * m);
  const size_t o_big = off;
  off = align256(off + sizeof(int32_t) * (size_t)m);
  const size_t o_ep = off;
  off = align256(off + sizeof(int32_t) * (size_t)m);
  const size_t o_eg = off;
  off = align256(off + sizeof(float2) * (size_t)kMaxBands * m);
  const size_t o_bb = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * (L.nb + 1));
  const size_t o_ct = off;
  off = align256(off + sizeof(int32_t) * (size_t)(L.nb + 1));
  if (bytes_out) *bytes_out = off;
  if (work) {
    char* b = static_cast<char*>(work);
    L.wa_part = reinterpret_cast<double*>(b + o_wp);
    L.xy = reinterpret_cast<float2*>(b + o_xy);
    L.pin_grad = reinterpret_cast<float2*>(b + o_pg);
    L.entries = reinterpret_cast<float4*>(b + o_en);
    L.big = reinterpret_cast<int32_t*>(b + o_big);
    L.epos = reinterpret_cast<int32_t*>(b + o_ep);
    L.egrad = reinterpret_cast<float2*>(b + o_eg);
    L.blk_base = reinterpret_cast<int32_t*>(b + o_bb);
    L.counters = reinterpret_cast<int32_t*>(b + o_ct);
  }
  return L;
}

namespace {

constexpr int NT = kBandThreads;
constexpr int NTA = kAccThreads;
constexpr int B = kCellBatch;

struct CellBatch {
  float x[B], y[B], w[B], h[B];
};

__device__ __forceinline__ void load_batch(CellBatch& c, int base, int m,
                                           const float* __restrict__ x,
                                           const float* __restrict__ y,
                                           const float* __restrict__ w,
                                           const float* __restrict__ h) {
  // unconditional (index clamped, m >= 1) so the whole batch is in flight
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int i = min(base + j * NT + (int)threadIdx.x, m - 1);
    c.x[j] = x[i];
    c.y[j] = y[i];
    c.w[j] = w[i];
    c.h[j] = h[i];
  }
}

}  // namespace

__global__ void __launch_bounds__(kBandThreads)
    k_band_count(GridF g, BandLayout L, const float* __restrict__ x,
                 const float* __restrict__ y, const float* __restrict__ w,
                 const float* __restrict__ h) {
  __shared__ int hist[257];   // the bands, then the cells too tall to list per band
  const int t = threadIdx.x;
  for (int b = t; b <= L.nb; b += NT) hist[b] = 0;
  __syncthreads();
  const int c0 = blockIdx.x * kCellsPerBlock;
  for (int base = c0; base < c0 + kCellsPerBlock && base < L.m; base += NT * B) {
    CellBatch c;
    load_batch(c, base, L.m, x, y, w, h);
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int i = base + j * NT + t;
      if (i >= L.m) continue;
      const Span sx = cell_span(c.x[j], c.w[j], g.xl, g.inv_bw, g.n);
      const Span sy = cell_span(c.y[j], c.h[j], g.yl, g.inv_bh, g.n);
      if (sx.i0 > sx.i1 || sy.i0 > sy.i1) continue;
      const int b0 = sy.i0 / L.rows, b1 = sy.i1 / L.rows;
      if (b1 - b0 >= kMaxBands) {
        atomicAdd(&hist[L.nb], 1);
        continue;
      }
      for (int b = b0; b <= b1; ++b) atomicAdd(&hist[b], 1);
    }
  }
  __syncthreads();
  for (int b = t; b <= L.nb; b += NT) L.blk_base[(size_t)b * L.nblk + blockIdx.x] = hist[b];
}

// Band b (b = nb: the tall cells' list): blk_base[b][k] = sum of the counts
// of blocks < k, counters[b] = the band's total.
constexpr int kScanThreads = 256;
__global__ void __launch_bounds__(kScanThreads) k_band_scan(BandLayout L) {
  int32_t* row = L.blk_base + (size_t)blockIdx.x * L.nblk;
  int carry = 0;
  for (int k0 = 0; k0 < L.nblk; k0 += 4 * kScanThreads) {
    int v[4], s = 0;
    const int base = k0 + 4 * (int)threadIdx.x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      v[j] = base + j < L.nblk ? row[base + j] : 0;
      s += v[j];
    }
    int total;
    int run = carry + block_exclusive_scan<kScanThreads>(s, &total);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (base + j < L.nblk) row[base + j] = run;
      run += v[j];
    }
    carry += total;
  }
  if (threadIdx.x == 0) L.counters[blockIdx.x] = carry;
}

__global__ void __launch_bounds__(kBandThreads)
    k_band_place(GridF g, BandLayout L, const float* __restrict__ x,
                 const float* __restrict__ y, const float* __restrict__ w,
                 const float* __restrict__ h) {
  __shared__ int cursor[257];
  const int t = threadIdx.x;
  int total;
  const int ex = block_exclusive_scan<NT>(t < L.nb ? L.counters[t] : 0, &total);
  if (t < L.nb) cursor[t] = ex + L.blk_base[(size_t)t * L.nblk + blockIdx.x];
  // the tall cells' list has its own offsets, from 0
  if (t == L.nb) cursor[t] = L.blk_base[(size_t)t * L.nblk + blockIdx.x];
  __syncthreads();
  const int c0 = blockIdx.x * kCellsPerBlock;
  for (int base = c0; base < c0 + kCellsPerBlock && base < L.m; base += NT * B) {
    CellBatch c;
    load_batch(c, base, L.m, x, y, w, h);
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int i = base + j * NT + t;
      if (i >= L.m) continue;
      const Span sx = cell_span(c.x[j], c.w[j], g.xl, g.inv_bw, g.n);
      const Span sy = cell_span(c.y[j], c.h[j], g.yl, g.inv_bh, g.n);
      int first = -1;   // the cell's entry in its first band, if listed
      if (sx.i0 <= sx.i1 && sy.i0 <= sy.i1) {
        const int b0 = sy.i0 / L.rows, b1 = sy.i1 / L.rows;
        if (b1 - b0 < kMaxBands) {
          const float4 e = make_float4(sx.lo, sx.hi, sy.lo, sy.hi);
          for (int b = b0; b <= b1; ++b) {
            const int q = atomicAdd(&cursor[b], 1);
            L.entries[q] = e;
            if (b == b0) first = q;
          }
        } else {
          L.big[atomicAdd(&cursor[L.nb], 1)] = i;
        }
      }
      L.epos[i] = first;
    }
  }
}

// Fixed-point LDS add of an overlap v in [0, 1] (units of 2^-31; a sum of
// up to 2^32 entries stays inside 64 bits).
constexpr double kAccUnit = 1.0 / 2147483648.0;
__device__ __forceinline__ void add_fixed(unsigned long long* a, float v) {
  atomicAdd(a, (unsigned long long)__float2uint_rn(v * 2147483648.0f));
}

__global__ void __launch_bounds__(kAccThreads)
    k_band_accum(GridF g, BandLayout L, const float* __restrict__ x,
                 const float* __restrict__ y, const float* __restrict__ w,
                 const float* __restrict__ h, const float* __restrict__ base,
                 float* __restrict__ rho) {
  __shared__ unsigned long long acc[kBandMaxN * 4];   // rows * n <= 4096 bins
  const int t = threadIdx.x;
  const int n = g.n, R = L.rows, band = blockIdx.x, r0 = band * R;
  const int cells = min(R, n - r0) * n;
  for (int k = t; k < cells; k += NTA) acc[k] = 0ull;
  int start;
  block_exclusive_scan<NTA>(t < band ? L.counters[t] : 0, &start);   // earlier bands
  const int end = start + L.counters[band];
  __syncthreads();
  for (int e0 = start; e0 < end; e0 += NTA * B) {
    float4 q[B];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int e = e0 + j * NTA + t;
      q[j] = L.entries[min(e, end - 1)];   // unconditional: the batch is in flight at once
    }
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if (e0 + j * NTA + t >= end) continue;
      const Span sx = span_from_edges(q[j].x, q[j].y, n);
      const Span sy = span_from_edges(q[j].z, q[j].w, n);
      const int ya = max(sy.i0, r0), yb = min(sy.i1, r0 + R - 1);
      for (int iy = ya; iy <= yb; ++iy) {
        const float oy = span_overlap(sy, iy);
        unsigned long long* row = acc + (iy - r0) * n;
        for (int ix = sx.i0; ix <= sx.i1; ++ix) add_fixed(&row[ix], span_overlap(sx, ix) * oy);
      }
    }
  }
  // cells too tall to be listed per band: every band block adds its rows of them
  const int nbig = L.counters[L.nb];
  for (int j = 0; j < nbig; ++j) {
    const int i = L.big[j];
    const Span sx = cell_span(x[i], w[i], g.xl, g.inv_bw, n);
    const Span sy = cell_span(y[i], h[i], g.yl, g.inv_bh, n);
    const int ya = max(sy.i0, r0), yb = min(sy.i1, r0 + R - 1);
    if (ya > yb) continue;
    const int nx = sx.i1 - sx.i0 + 1;
    const int tot = nx * (yb - ya + 1);
    for (int k = t; k < tot; k += NTA) {
      const int ix = sx.i0 + k % nx, iy = ya + k / nx;
      add_fixed(&acc[(iy - r0) * n + ix], span_overlap(sx, ix) * span_overlap(sy, iy));
    }
  }
  __syncthreads();
  const size_t o = (size_t)r0 * n;
  for (int k = t; k < cells; k += NTA)
    rho[o + k] = (base ? base[o + k] : 0.0f) + (float)((double)acc[k] * kAccUnit);
}

// Density gradient of every cell listed in band b with b its first band,
// from the cell's entry (its edges), into egrad at the entry's position.  A
// band's cells read the field rows of that band and the next, so the map
// reads of one block stay within a few tens of KiB (L2-resident), where a
// per-cell gather in cell order reads the whole map at random.
constexpr int kGatherSplit = 1;   // blocks per band
constexpr int NTG = 1024;         // threads of a band-gather block
template <int MODE>
__global__ void __launch_bounds__(NTG)
    k_band_gather(GridF g, BandLayout L, const float2* __restrict__ exy,
                  const float* __restrict__ psi) {
  // the band's field rows and the next one (cells of up to two rows whose
  // first row is in the band read only these) staged in LDS
  __shared__ float2 rows[5 * kBandMaxN];
  const int t = threadIdx.x;
  const int n = g.n, R = L.rows;
  // XCD k runs a contiguous range of bands, all pieces of a band on one XCD
  const int r = kGatherSplit > 1 ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
  const int band = r / kGatherSplit, part = r % kGatherSplit;
  const int r0 = band * R, nr = min(R + 1, n - r0);
  if (MODE == FFTPL_GRAD_FIELD) {
    for (int k = t; k < nr * n; k += NTG) rows[k] = exy[(int64_t)r0 * n + k];
  }
  // start of the band: the counts of the earlier bands
  int start;
  block_exclusive_scan<NTG>(t < band ? L.counters[t] : 0, &start);   // (synchronises)
  const int len = L.counters[band], piece = (len + kGatherSplit - 1) / kGatherSplit;
  const int lo = start + part * piece, end = min(start + len, lo + piece);
  for (int e0 = lo; e0 < end; e0 += NTG * B) {
    float4 q[B];
#pragma unroll
    for (int j = 0; j < B; ++j) q[j] = L.entries[min(e0 + j * NTG + t, end - 1)];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      const int e = e0 + j * NTG + t;
      if (e >= end) continue;
      const Span sx = span_from_edges(q[j].x, q[j].y, n);
      const Span sy = span_from_edges(q[j].z, q[j].w, n);
      if (sy.i0 / R != band) continue;   // listed again below its first band
      if (MODE == FFTPL_GRAD_FIELD && sy.i1 < r0 + nr) {
        // the same sum as the per-cell gather, from the staged rows
        float ax = 0.0f, ay = 0.0f;
        for (int iy = sy.i0; iy <= sy.i1; ++iy) {
          const float oy = span_overlap(sy, iy);
          const float2* row = rows + (iy - r0) * n;
          for (int ix = sx.i0; ix <= sx.i1; ++ix) {
            const float ov = span_overlap(sx, ix) * oy;
            const float2 f = row[ix];
            ax += ov * f.x;
            ay += ov * f.y;
          }
        }
        L.egrad[e] = make_float2(ax * -g.inv_bw, ay * -g.inv_bh);
      } else {
        L.egrad[e] = density_grad_spans<MODE, true>(g, sx, sy, nullptr, nullptr, exy, psi);
      }
    }
  }
}

hipError_t launch_band_gather(const GridF& g, const BandLayout& L, const float* exy,
                              const float* psi, int grad_mode, hipStream_t s) {
  const float2* e2 = reinterpret_cast<const float2*>(exy);
  if (grad_mode == FFTPL_GRAD_EXACT)
    hipLaunchKernelGGL(k_band_gather<FFTPL_GRAD_EXACT>, dim3(L.nb * kGatherSplit), dim3(NTG),
                       0, s, g, L, e2, psi);
  else
    hipLaunchKernelGGL(k_band_gather<FFTPL_GRAD_FIELD>, dim3(L.nb * kGatherSplit), dim3(NTG),
                       0, s, g, L, e2, psi);
  return hipGetLastError();
}

// xy[i] = (x[i], y[i]): the wirelength pass then gathers one float2 per pin.
__global__ void __launch_bounds__(256)
    k_interleave(int m, const float* __restrict__ x, const float* __restrict__ y,
                 float2* __restrict__ xy) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    xy[i] = make_float2(x[i], y[i]);
}

hipError_t launch_interleave(int m, const float* x, const float* y, float2* xy,
                             hipStream_t s) {
  if (m <= 0) return hipSuccess;
  int blocks = (m + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_interleave, dim3(blocks), dim3(256), 0, s, m, x, y, xy);
  return hipGetLastError();
}

hipError_t launch_band_scatter(const GridF& g, const BandLayout& L, const float* x,
                               const float* y, const float* w, const float* h,
                               const float* base, float* rho, hipStream_t s, Plan* tp) {
  if (L.m > 0) {
    hipLaunchKernelGGL(k_band_count, dim3(L.nblk), dim3(NT), 0, s, g, L, x, y, w, h);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (tp) plan_mark(*tp, "k_band_count", s);
    hipLaunchKernelGGL(k_band_scan, dim3(L.nb + 1), dim3(kScanThreads), 0, s, L);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (tp) plan_mark(*tp, "k_band_scan", s);
    hipLaunchKernelGGL(k_band_place, dim3(L.nblk), dim3(NT), 0, s, g, L, x, y, w, h);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (tp) plan_mark(*tp, "k_band_place", s);
  } else {
    // no cells: empty bands and no tall cells
    hipError_t e = launch_zero_i32(L.counters, L.nb + 1, s);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_band_accum, dim3(L.nb), dim3(NTA), 0, s, g, L, x, y, w, h, base, rho);
  hipError_t e = hipGetLastError();
  if (tp) plan_mark(*tp, "k_band_accum", s);
  return e;
}

}  // namespace fftpl
