// Banded density scatter (Eq. (2), Section III-B) without float atomics in
// global memory, which retire at roughly 20 G/s on the whole chip whatever
// their scope:
//   place: each block of kCellsPerBlock cells histograms the bands its cells
//          touch in LDS (plus one slot for cells too tall to list per band),
//          scans the histogram, and writes each cell's edges (bin units)
//          into every band it touches, in a region of its own sliced by band
//          (LDS-atomic ranks inside each slice); per band, each block's slice
//          offset and count go out band-major;
//   accum: one block per band walks the band's slices of every region and
//          adds its entries into an LDS copy of its rows, then writes
//          rho = base + rows once.  The LDS adds are 64-bit integer adds of
//          the overlaps in fixed point (every overlap lies in [0, 1], units
//          of 2^-31): they retire many times faster than LDS float atomics,
//          and the sums do not depend on the order of the entries, so rho is
//          the same on every run;
//   gather (after the solve): one block per band walks the same slices and
//          computes the density gradient of every cell whose first band it
//          is, from the band's field rows staged in LDS.
// Every thread issues the loads of its cells (or entries) before it uses any
// of them, so each block keeps many misses in flight.
#include <algorithm>
#include <mutex>

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
  const size_t nreg = (size_t)L.nblk * kBandRegion;   // entries of all regions
  const size_t o_en = off;
  off = align256(off + sizeof(float4) * nreg);
  const size_t o_big = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * kCellsPerBlock);
  const size_t o_ep = off;
  off = align256(off + sizeof(int32_t) * (size_t)m);
  const size_t o_eg = off;
  off = align256(off + sizeof(float2) * nreg);
  const size_t o_bo = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * (L.nb + 1));
  const size_t o_bc = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * (L.nb + 1));
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
    L.blk_off = reinterpret_cast<int32_t*>(b + o_bo);
    L.blk_cnt = reinterpret_cast<int32_t*>(b + o_bc);
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

// The entries of band `band` (band = nb: the tall cells) lie in one slice per
// region: slice k holds blk_cnt[band][k] entries from index
// k * stride + blk_off[band][k].  A block of NTB threads walks them in chunks
// of NTB slices: the chunk's counts are scanned, and the chunk's entries are
// taken in windows of NTB * KB.  For each window every slice writes its own
// number into an LDS owner map at the window positions it covers (slices
// longer than a wavefront are written by the whole wavefront), so a
// thread finds the slice of its entry with one LDS read (a binary search over
// the scan, ten dependent LDS reads per entry, cost the walk more than its
// loads).  Thread t takes window entries t, t + NTB, ...: KB of them, whose
// indices are all known before f(index) uses any, so the caller can issue
// their loads together.  Every thread of the block must call it; `owner`
// holds NTB * KB entries.
template <int NTB, int KB, typename F>
__device__ __forceinline__ void walk_band(const BandLayout& L, int band, int64_t stride,
                                          int* pre, int64_t* start, unsigned short* owner,
                                          F f) {
  static_assert(NTB <= 65536, "slice numbers are u16");
  constexpr int W = NTB * KB;
  const int t = threadIdx.x;
  for (int k0 = 0; k0 < L.nblk; k0 += NTB) {
    const int k = k0 + t;
    const int c = k < L.nblk ? L.blk_cnt[(size_t)band * L.nblk + k] : 0;
    const int o = k < L.nblk ? L.blk_off[(size_t)band * L.nblk + k] : 0;
    int tot;
    const int ex = block_exclusive_scan<NTB>(c, &tot);
    pre[t] = ex;
    start[t] = (int64_t)k * stride + o;
    for (int w0 = 0; w0 < tot; w0 += W) {
      // a slice of up to 64 window entries is written by its own thread,
      // a longer one by its whole wavefront
      const int a = max(ex, w0), e = min(ex + c, w0 + W);
      const bool big = e - a > kWave;
      if (!big)
        for (int v = a; v < e; ++v) owner[v - w0] = (unsigned short)t;
      unsigned long long bm = __ballot(big);
      while (bm) {
        const int l = __ffsll((long long)bm) - 1;
        bm &= bm - 1;
        const int ba = __shfl(a, l), be = __shfl(e, l), bt = __shfl(t, l);
        for (int v = ba + (t & (kWave - 1)); v < be; v += kWave) owner[v - w0] = (unsigned short)bt;
      }
      __syncthreads();
      int64_t idx[KB];
#pragma unroll
      for (int j = 0; j < KB; ++j) {
        const int v = w0 + j * NTB + t;
        idx[j] = -1;
        if (v < tot) {
          const int sl = owner[v - w0];
          idx[j] = start[sl] + (v - pre[sl]);
        }
      }
      f(idx);
      __syncthreads();   // owner, pre and start are rewritten next
    }
  }
}

template <int NB>
__global__ void __launch_bounds__(kBandThreads) k_band_place(BandBatch<NB> bb) {
  // design blockIdx.y of the batch; blocks past its count of cell blocks idle
  const BandReq& q = bb.r[blockIdx.y];
  const GridF g = q.g;
  const BandLayout L = q.L;
  const int t = threadIdx.x, k = blockIdx.x;
  if (L.m <= 0 || k >= L.nblk) return;
  const float* __restrict__ x = q.x;
  const float* __restrict__ y = q.y;
  const float* __restrict__ w = q.w;
  const float* __restrict__ h = q.h;
  __shared__ int hist[257], cur[257];   // the bands, then the tall cells
  for (int b = t; b <= L.nb; b += NT) hist[b] = 0;
  __syncthreads();
  const int c0 = k * kCellsPerBlock;   // one batch of B cells per thread
  CellBatch c;
  load_batch(c, c0, L.m, x, y, w, h);
  float4 e[B];
  int b0[B], nbd[B];   // first band, bands listed (0: none, -1: tall)
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int i = c0 + j * NT + t;
    nbd[j] = 0;
    b0[j] = 0;
    if (i >= L.m) continue;
    const Span sx = cell_span(c.x[j], c.w[j], g.xl, g.inv_bw, g.n);
    const Span sy = cell_span(c.y[j], c.h[j], g.yl, g.inv_bh, g.n);
    if (sx.i0 > sx.i1 || sy.i0 > sy.i1) continue;
    b0[j] = sy.i0 / L.rows;
    const int b1 = sy.i1 / L.rows;
    e[j] = make_float4(sx.lo, sx.hi, sy.lo, sy.hi);
    if (b1 - b0[j] >= kMaxBands) {
      nbd[j] = -1;
      atomicAdd(&hist[L.nb], 1);
    } else {
      nbd[j] = b1 - b0[j] + 1;
      for (int b = b0[j]; b <= b1; ++b) atomicAdd(&hist[b], 1);
    }
  }
  __syncthreads();
  int tot;
  const int ex = block_exclusive_scan<NT>(t < L.nb ? hist[t] : 0, &tot);
  if (t <= L.nb) {
    const int off = t < L.nb ? ex : 0;   // the tall cells have a list of their own
    L.blk_off[(size_t)t * L.nblk + k] = off;
    L.blk_cnt[(size_t)t * L.nblk + k] = hist[t];
    cur[t] = off;
  }
  __syncthreads();
  const int64_t rbase = (int64_t)k * kBandRegion;
#pragma unroll
  for (int j = 0; j < B; ++j) {
    const int i = c0 + j * NT + t;
    if (i >= L.m) continue;
    int first = -1;   // the cell's entry in its first band, if listed
    if (nbd[j] > 0) {
      for (int b = b0[j]; b < b0[j] + nbd[j]; ++b) {
        const int q = atomicAdd(&cur[b], 1);
        L.entries[rbase + q] = e[j];
        if (b == b0[j]) first = (int)(rbase + q);
      }
    } else if (nbd[j] < 0) {
      L.big[(int64_t)k * kCellsPerBlock + atomicAdd(&cur[L.nb], 1)] = i;
    }
    L.epos[i] = first;
  }
}

// Fixed-point LDS add of an overlap v in [0, 1] (units of 2^-31; a sum of
// up to 2^32 entries stays inside 64 bits).
constexpr double kAccUnit = 1.0 / 2147483648.0;
__device__ __forceinline__ void add_fixed(unsigned long long* a, float v) {
  atomicAdd(a, (unsigned long long)__float2uint_rn(v * 2147483648.0f));
}

template <int NB>
__global__ void __launch_bounds__(kAccThreads) k_band_accum(BandBatch<NB> bb) {
  const BandReq& q = bb.r[blockIdx.y];
  const GridF g = q.g;
  const BandLayout L = q.L;
  const float* __restrict__ x = q.x;
  const float* __restrict__ y = q.y;
  const float* __restrict__ w = q.w;
  const float* __restrict__ h = q.h;
  const float* __restrict__ base = q.base;
  float* __restrict__ rho = q.rho;
  __shared__ unsigned long long acc[kBandMaxN * 4];   // rows * n <= 4096 bins
  __shared__ int pre[NTA];
  __shared__ int64_t start[NTA];
  __shared__ unsigned short owner[NTA * B];
  const int t = threadIdx.x;
  const int n = g.n, R = L.rows, band = blockIdx.x, r0 = band * R;
  const int cells = min(R, n - r0) * n;
  for (int k = t; k < cells; k += NTA) acc[k] = 0ull;
  __syncthreads();
  walk_band<NTA, B>(L, band, kBandRegion, pre, start, owner, [&](const int64_t (&idx)[B]) {
    float4 q[B];
#pragma unroll
    for (int j = 0; j < B; ++j) q[j] = L.entries[idx[j] >= 0 ? idx[j] : 0];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if (idx[j] < 0) continue;
      const Span sx = span_from_edges(q[j].x, q[j].y, n);
      const Span sy = span_from_edges(q[j].z, q[j].w, n);
      const int ya = max(sy.i0, r0), yb = min(sy.i1, r0 + R - 1);
      for (int iy = ya; iy <= yb; ++iy) {
        const float oy = span_overlap(sy, iy);
        unsigned long long* row = acc + (iy - r0) * n;
        for (int ix = sx.i0; ix <= sx.i1; ++ix) add_fixed(&row[ix], span_overlap(sx, ix) * oy);
      }
    }
  });
  // cells too tall to be listed per band: every band block adds its rows of
  // them, one thread per cell
  walk_band<NTA, 1>(L, L.nb, kCellsPerBlock, pre, start, owner, [&](const int64_t (&idx)[1]) {
    if (idx[0] < 0) return;
    const int i = L.big[idx[0]];
    const Span sx = cell_span(x[i], w[i], g.xl, g.inv_bw, n);
    const Span sy = cell_span(y[i], h[i], g.yl, g.inv_bh, n);
    const int ya = max(sy.i0, r0), yb = min(sy.i1, r0 + R - 1);
    for (int iy = ya; iy <= yb; ++iy) {
      const float oy = span_overlap(sy, iy);
      for (int ix = sx.i0; ix <= sx.i1; ++ix)
        add_fixed(&acc[(iy - r0) * n + ix], span_overlap(sx, ix) * oy);
    }
  });
  __syncthreads();
  // rho = base + rows: all of a thread's base loads issued before any store
  constexpr int PA = kBandMaxN * 4 / NTA;
  const size_t o = (size_t)r0 * n;
  float bv[PA];
#pragma unroll
  for (int j = 0; j < PA; ++j) bv[j] = base ? base[o + min(t + j * NTA, cells - 1)] : 0.0f;
#pragma unroll
  for (int j = 0; j < PA; ++j) {
    const int k = t + j * NTA;
    if (k < cells) rho[o + k] = bv[j] + (float)((double)acc[k] * kAccUnit);
  }
}

// Density gradient of every cell listed in band b with b its first band,
// from the cell's entry (its edges), into egrad at the entry's position.  A
// band's cells read the field rows of that band and the next, so the map
// reads of one block stay within a few tens of KiB (staged in LDS), where a
// per-cell gather in cell order reads the whole map at random.
constexpr int NTG = 1024;   // threads of a band-gather block
template <int MODE, int NB>
__global__ void __launch_bounds__(NTG) k_band_gather(BandBatch<NB> bb) {
  const BandReq& q = bb.r[blockIdx.y];
  const GridF g = q.g;
  const BandLayout L = q.L;
  const float2* __restrict__ exy = q.exy;
  const float* __restrict__ psi = q.psi;
  // the band's field rows and the next one (cells of up to two rows whose
  // first row is in the band read only these) staged in LDS
  __shared__ float2 rows[5 * kBandMaxN];
  __shared__ int pre[NTG];
  __shared__ int64_t start[NTG];
  __shared__ unsigned short owner[NTG * B];
  const int t = threadIdx.x;
  const int n = g.n, R = L.rows, band = blockIdx.x;
  const int r0 = band * R, nr = min(R + 1, n - r0);
  if (MODE == FFTPL_GRAD_FIELD) {
    // all of a thread's loads issued before its LDS stores
    constexpr int PS = (5 * kBandMaxN + NTG - 1) / NTG;
    const int cnt = nr * n;
    float2 v[PS];
#pragma unroll
    for (int j = 0; j < PS; ++j) v[j] = exy[(int64_t)r0 * n + min(t + j * NTG, cnt - 1)];
#pragma unroll
    for (int j = 0; j < PS; ++j)
      if (t + j * NTG < cnt) rows[t + j * NTG] = v[j];
  }
  // (the walk's first scan synchronises the block after the staging)
  walk_band<NTG, B>(L, band, kBandRegion, pre, start, owner, [&](const int64_t (&idx)[B]) {
    float4 q[B];
#pragma unroll
    for (int j = 0; j < B; ++j) q[j] = L.entries[idx[j] >= 0 ? idx[j] : 0];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      if (idx[j] < 0) continue;
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
        L.egrad[idx[j]] = make_float2(ax * -g.inv_bw, ay * -g.inv_bh);
      } else {
        L.egrad[idx[j]] = density_grad_spans<MODE, true>(g, sx, sy, nullptr, nullptr, exy, psi);
      }
    }
  });
}

template <int NB>
static hipError_t band_gather_nb(const BandBatch<NB>& bb, int nb, int grad_mode,
                                 hipStream_t s) {
  const dim3 grid(nb, bb.count);
  if (grad_mode == FFTPL_GRAD_EXACT)
    hipLaunchKernelGGL((k_band_gather<FFTPL_GRAD_EXACT, NB>), grid, dim3(NTG), 0, s, bb);
  else
    hipLaunchKernelGGL((k_band_gather<FFTPL_GRAD_FIELD, NB>), grid, dim3(NTG), 0, s, bb);
  return hipGetLastError();
}

hipError_t launch_band_gather_batch(const BandReq* reqs, int count, int grad_mode,
                                    hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxBatch) return hipErrorInvalidValue;
  const int nb = reqs[0].L.nb;
  if (count == 1) {
    BandBatch<1> bb;
    bb.count = 1;
    bb.r[0] = reqs[0];
    return band_gather_nb(bb, nb, grad_mode, s);
  }
  BandBatch<kMaxBatch> bb;
  bb.count = count;
  for (int i = 0; i < count; ++i) bb.r[i] = reqs[i];
  return band_gather_nb(bb, nb, grad_mode, s);
}

hipError_t launch_band_gather(const GridF& g, const BandLayout& L, const float* exy,
                              const float* psi, int grad_mode, hipStream_t s) {
  BandReq q;
  q.g = g;
  q.L = L;
  q.exy = reinterpret_cast<const float2*>(exy);
  q.psi = psi;
  return launch_band_gather_batch(&q, 1, grad_mode, s);
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

template <int NB>
static hipError_t band_scatter_nb(const BandBatch<NB>& bb, int max_nblk, int nb,
                                  bool any_cells, hipStream_t s, Plan* tp) {
  hipError_t e = hipSuccess;
  if (any_cells) {
    hipLaunchKernelGGL((k_band_place<NB>), dim3(max_nblk, bb.count), dim3(NT), 0, s, bb);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (tp) plan_mark(*tp, "k_band_place", s);
  }
  hipLaunchKernelGGL((k_band_accum<NB>), dim3(nb, bb.count), dim3(NTA), 0, s, bb);
  e = hipGetLastError();
  if (tp) plan_mark(*tp, "k_band_accum", s);
  return e;
}

hipError_t launch_band_scatter_batch(const BandReq* reqs, int count, hipStream_t s,
                                     Plan* tp) {
  if (count <= 0) return hipSuccess;
  if (count > kMaxBatch) return hipErrorInvalidValue;
  int max_nblk = 1;
  bool any = false;
  for (int i = 0; i < count; ++i) {
    if (reqs[i].L.m > 0) {
      any = true;
      max_nblk = std::max(max_nblk, reqs[i].L.nblk);
    } else {
      // no cells: one empty region
      hipError_t e = launch_zero_i32(reqs[i].L.blk_cnt,
                                     (int64_t)reqs[i].L.nblk * (reqs[i].L.nb + 1), s);
      if (e != hipSuccess) return e;
    }
  }
  const int nb = reqs[0].L.nb;
  if (count == 1) {
    BandBatch<1> bb;
    bb.count = 1;
    bb.r[0] = reqs[0];
    return band_scatter_nb(bb, max_nblk, nb, any, s, tp);
  }
  BandBatch<kMaxBatch> bb;
  bb.count = count;
  for (int i = 0; i < count; ++i) bb.r[i] = reqs[i];
  return band_scatter_nb(bb, max_nblk, nb, any, s, tp);
}

// ---- the density map without allocation -----------------------------------
// A file-scope device array holds the band lists for callers that cannot
// allocate (see fftpl_density_map_noalloc).  Host code never passes the
// array's name to a kernel: its device address, looked up once per device,
// is what the launches get.
static __device__ __align__(256) unsigned char scratch[kNoallocScratchBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevicesNoalloc] = {};
}  // namespace

// Band lists of the density scatter alone (no wirelength or gather arrays).
BandLayout band_layout_density(int n, int m, void* work, size_t* bytes_out) {
  BandLayout L;
  L.n = n;
  L.rows = (n + 255) / 256;
  L.nb = (n + L.rows - 1) / L.rows;
  L.m = m;
  L.nblk = m > 0 ? (m + kCellsPerBlock - 1) / kCellsPerBlock : 1;
  size_t off = 0;
  const size_t o_en = off;
  off = align256(off + sizeof(float4) * (size_t)L.nblk * kBandRegion);
  const size_t o_big = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * kCellsPerBlock);
  const size_t o_ep = off;
  off = align256(off + sizeof(int32_t) * (size_t)m);
  const size_t o_bo = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * (L.nb + 1));
  const size_t o_bc = off;
  off = align256(off + sizeof(int32_t) * (size_t)L.nblk * (L.nb + 1));
  if (bytes_out) *bytes_out = off;
  if (work) {
    char* b = static_cast<char*>(work);
    L.entries = reinterpret_cast<float4*>(b + o_en);
    L.big = reinterpret_cast<int32_t*>(b + o_big);
    L.epos = reinterpret_cast<int32_t*>(b + o_ep);
    L.blk_off = reinterpret_cast<int32_t*>(b + o_bo);
    L.blk_cnt = reinterpret_cast<int32_t*>(b + o_bc);
  }
  return L;
}

hipError_t noalloc_scratch(void** ptr) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevicesNoalloc) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_band_scatter(const GridF& g, const BandLayout& L, const float* x,
                               const float* y, const float* w, const float* h,
                               const float* base, float* rho, hipStream_t s, Plan* tp) {
  BandReq q;
  q.g = g;
  q.L = L;
  q.x = x;
  q.y = y;
  q.w = w;
  q.h = h;
  q.base = base;
  q.rho = rho;
  return launch_band_scatter_batch(&q, 1, s, tp);
}

}  // namespace fftpl
