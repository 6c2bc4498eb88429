// Spectral Neumann Poisson solve (Eqs. (8)-(12)) with hand-written FFTs.
//
// The 2-D transforms are separable; the solve is three passes over the map,
// each one block per pair of rows (or columns), the 1-D transforms done in
// LDS by the whole block:
//   A  rows:    DCT-II along x of rho           -> bT[u][iy] (written transposed)
//   B  columns: DCT-II along y, scale by c_u c_v / n^2 / (w_u^2 + w_v^2 + eps)
//               (zero at (0,0): the DC is removed), then DCT-III along y
//               (-> P) and the sine transform along y weighted by w_v (-> Q)
//                                               -> P[iy][u], Q[iy][u]
//   C  rows:    DCT-III along x of P (-> psi) and of Q (-> Ey), sine
//               transform along x of w_u P (-> Ex); energy sum rho*psi.
// Difference mode (for the exact density gradient) replaces the fields by
// the differences of psi between neighbouring bin centres,
//   Dx(iy, ix) = psi(iy, ix+1) - psi(iy, ix),  Dy(iy, ix) = psi(iy+1, ix) - psi(iy, ix),
// taken in the spectral domain: cos(w (i + 3/2)) - cos(w (i + 1/2)) =
// (cos w - 1) cos(w (i + 1/2)) - sin w sin(w (i + 1/2)), so each difference is
// a DCT-III with weights cos w - 1 minus a sine transform with weights sin w.
// Both weights vanish at low frequency, so the small differences come out
// with float32 accuracy relative to themselves instead of to psi.  Pass B
// then outputs R = DCT-III((cos w_v - 1) G) - sine(sin w_v G) in place of Q,
// and pass C gives Dy = DCT-III(R) and Dx from P the same way along x.
// A length-n DCT-II is an n-point complex FFT of the even/odd reordered
// sequence followed by a quarter-sample twiddle (Makhoul's algorithm); two
// real sequences share one complex FFT as its real and imaginary parts.  A
// DCT-III runs the same steps backwards.  The sine transform is a DCT-III of
// the reversed coefficients with alternating output signs:
//   sum_{k>=1} b_k sin(pi k (2i+1)/2n) = (-1)^i sum_{k>=1} b_{n-k} cos(pi k (2i+1)/2n).
// The 1-D FFT is a Stockham autosort radix-4 (one radix-2 stage first when
// log2 n is odd), in place in LDS, every stage reading all its inputs into
// registers before a barrier and writing after it.  The independent
// transforms of a pass share the stages.  Each pass issues all its global
// loads (rows and tables) before touching LDS, so a block waits on memory
// once rather than once per loop trip.
#include "fftpl_internal.hpp"

namespace fftpl {

namespace {

constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v / 2); }

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}

// Position of sample i in the even/odd reordered sequence.
template <int N>
__device__ __forceinline__ int mk_pos(int i) {
  return (i & 1) ? N - ((i + 1) >> 1) : (i >> 1);
}

// Threads per block for a length-N transform: one radix-4 butterfly per
// thread and stage at N = 1024 (four wavefronts), never less than one
// wavefront.
template <int N>
struct FftShape {
  static constexpr int NT = N / 4 >= 256 ? 256 : (N / 4 >= kWave ? N / 4 : kWave);
};

template <int NT>
__device__ __forceinline__ void block_lds_sync() {
  if constexpr (NT > kWave)
    __syncthreads();
  else
    wave_lds_sync();
}

// Unnormalised in-place DFTs of NB buffers of length N (b0..b{NB-1}) by a
// block of NT threads.  The buffers go through the stages together, so one
// barrier per stage serves all of them and each twiddle is read once for all.
// INV selects exp(+).  tw[t] = exp(-2 pi i t / N).
template <int N, int NT, bool INV, int NB>
__device__ __forceinline__ void block_fft(float2* b0, float2* b1, float2* b2, float2* b3,
                                          const float2* __restrict__ tw, int tid) {
  float2* const bufs[4] = {b0, b1, b2, b3};
  constexpr int LOG = ilog2c(N);
  int ns = 1;
  if constexpr (LOG & 1) {
    constexpr int B = N / 2;
    constexpr int PER = (B + NT - 1) / NT;
    float2 v0[NB][PER], v1[NB][PER];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const int j = tid + NT * t;
        if (B % NT == 0 || j < B) {
          v0[q][t] = bufs[q][j];
          v1[q][t] = bufs[q][j + B];
        }
      }
    block_lds_sync<NT>();
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const int j = tid + NT * t;
        if (B % NT == 0 || j < B) {
          bufs[q][2 * j] = make_float2(v0[q][t].x + v1[q][t].x, v0[q][t].y + v1[q][t].y);
          bufs[q][2 * j + 1] = make_float2(v0[q][t].x - v1[q][t].x, v0[q][t].y - v1[q][t].y);
        }
      }
    block_lds_sync<NT>();
    ns = 2;
  }
  constexpr int B = N / 4;
  constexpr int PER = (B + NT - 1) / NT;
#pragma unroll
  for (int st = 0; st < LOG / 2; ++st) {
    float2 v[NB][PER][4];
#pragma unroll
    for (int q = 0; q < NB; ++q)
#pragma unroll
      for (int t = 0; t < PER; ++t) {
        const int j = tid + NT * t;
        if (B % NT == 0 || j < B) {
#pragma unroll
          for (int r = 0; r < 4; ++r) v[q][t][r] = bufs[q][j + r * B];
        }
      }
    block_lds_sync<NT>();
    const int stride = N / (4 * ns);
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int j = tid + NT * t;
      if (B % NT == 0 || j < B) {
        const int k = j & (ns - 1);
        float2 w[4];
        if (ns > 1) {
#pragma unroll
          for (int r = 1; r < 4; ++r) {
            w[r] = tw[k * r * stride];
            if (INV) w[r].y = -w[r].y;
          }
        }
        const int o = (j - k) * 4 + k;
#pragma unroll
        for (int q = 0; q < NB; ++q) {
          float2* u = v[q][t];
          if (ns > 1) {
#pragma unroll
            for (int r = 1; r < 4; ++r) u[r] = cmul(u[r], w[r]);
          }
          const float2 t0 = make_float2(u[0].x + u[2].x, u[0].y + u[2].y);
          const float2 t1 = make_float2(u[0].x - u[2].x, u[0].y - u[2].y);
          const float2 t2 = make_float2(u[1].x + u[3].x, u[1].y + u[3].y);
          const float2 d = make_float2(u[1].x - u[3].x, u[1].y - u[3].y);
          // forward: t3 = -i * d ; inverse: t3 = +i * d
          const float2 t3 = INV ? make_float2(-d.y, d.x) : make_float2(d.y, -d.x);
          float2* b = bufs[q];
          b[o] = make_float2(t0.x + t2.x, t0.y + t2.y);
          b[o + ns] = make_float2(t1.x + t3.x, t1.y + t3.y);
          b[o + 2 * ns] = make_float2(t0.x - t2.x, t0.y - t2.y);
          b[o + 3 * ns] = make_float2(t1.x - t3.x, t1.y - t3.y);
        }
      }
    }
    block_lds_sync<NT>();
    ns *= 4;
  }
}

// Copy the twiddle table, the quarter-sample table cs and (WF) the frequency
// table wf into LDS.  All global loads are issued before the first LDS write,
// so the block waits on memory once; the caller synchronises.
template <int N, int NT, bool WF>
__device__ __forceinline__ void stage_tables(float2* tw, const float2* __restrict__ tw_g,
                                             float2* cs, const float2* __restrict__ cs_g,
                                             float* wf, const float* __restrict__ wf_g,
                                             int tid) {
  constexpr int PT = (N + NT - 1) / NT, PC = (N / 2 + NT) / NT;
  float2 a[PT], c[PC];
  float f[PT];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int i = min(tid + NT * t, N - 1);
    a[t] = tw_g[i];
    if (WF) f[t] = wf_g[i];
  }
#pragma unroll
  for (int t = 0; t < PC; ++t) c[t] = cs_g[min(tid + NT * t, N / 2)];
#pragma unroll
  for (int t = 0; t < PT; ++t) {
    const int i = tid + NT * t;
    if (N % NT == 0 || i < N) {
      tw[i] = a[t];
      if (WF) wf[i] = f[t];
    }
  }
#pragma unroll
  for (int t = 0; t < PC; ++t) {
    const int i = tid + NT * t;
    if (i <= N / 2) cs[i] = c[t];
  }
}

// Sums over the block of K per-thread doubles, added in a fixed order, so
// every thread gets the same bits.  red holds K * NT / 64 doubles of LDS.
template <int NT, int K>
__device__ __forceinline__ void block_sums(double (&v)[K], double* red, int tid) {
  constexpr int NW = NT / kWave;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if constexpr (NW > 1) {
    if ((tid & (kWave - 1)) == 0) {
#pragma unroll
      for (int k = 0; k < K; ++k) red[k * NW + tid / kWave] = v[k];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < NW; ++w) s += red[k * NW + w];
      v[k] = s;
    }
  }
}

// Forward post-processing for the pair (k, n-k) of a two-real-sequence FFT
// V = FFT(v1 + i v2): returns the DCT-II outputs X1, X2 at k and n-k.
// cs = (cos, sin)(pi k / 2n).
__device__ __forceinline__ void dct2_pair(float2 A, float2 B, float2 cs, float& x1k,
                                          float& x2k, float& x1kp, float& x2kp) {
  const float v1x = 0.5f * (A.x + B.x), v1y = 0.5f * (A.y - B.y);
  const float v2x = 0.5f * (A.y + B.y), v2y = -0.5f * (A.x - B.x);
  x1k = cs.x * v1x + cs.y * v1y;
  x2k = cs.x * v2x + cs.y * v2y;
  x1kp = cs.y * v1x - cs.x * v1y;
  x2kp = cs.y * v2x - cs.x * v2y;
}

// Hermitian input of a DCT-III of real coefficients Y at the pair (k, n-k):
// H_k = exp(i pi k / 2n) (Y_k - i Y_{n-k}) / 2, H_{n-k} = conj(H_k), H_0 = Y_0.
__device__ __forceinline__ void dct3_herm(float yk, float ykp, float2 cs, bool k0,
                                          float2& hk, float2& hkp) {
  if (k0) {
    hk = make_float2(yk, 0.0f);
    hkp = hk;
    return;
  }
  hk = make_float2(0.5f * (cs.x * yk + cs.y * ykp), 0.5f * (cs.y * yk - cs.x * ykp));
  hkp = make_float2(hk.x, -hk.y);
}

// z = ha + i hb
__device__ __forceinline__ float2 pack2(float2 ha, float2 hb) {
  return make_float2(ha.x - hb.y, ha.y + hb.x);
}

// Difference-mode weights at the pair (k, n-k) from cs = (cos, sin)(pi k / 2n):
// cos w_k - 1 = -2 sin^2(w_k / 2), cos w_{n-k} - 1 = -2 cos^2(w_k / 2),
// sin w_k = sin w_{n-k} = 2 sin(w_k / 2) cos(w_k / 2).
__device__ __forceinline__ void diff_weights(float2 cs, float& dm_k, float& dm_kp, float& sw) {
  dm_k = -2.0f * cs.y * cs.y;
  dm_kp = -2.0f * cs.x * cs.x;
  sw = 2.0f * cs.y * cs.x;
}

// ---------------------------------------------------------------------------
// Pass A: rows -> bT (transposed), row sums in double; optional overflow sums.
// ---------------------------------------------------------------------------
template <int N, int NB>
__global__ void __launch_bounds__(FftShape<N>::NT)
    k_rows_dct2(SpecBatch<NB> sb, const float2* __restrict__ tw_g,
                const float2* __restrict__ cs_g) {
  // design blockIdx.y of the batch
  const SpecReq& rq = sb.r[blockIdx.y];
  const float* __restrict__ rho = rq.rho;
  float* __restrict__ bT = rq.bT;
  double* __restrict__ rowsum = rq.rowsum;
  const float* __restrict__ base = rq.base;
  const float* __restrict__ cap = rq.cap;
  const float rho_t = rq.rho_t;
  double* __restrict__ tau_part = rq.tau_part;
  constexpr int NT = FftShape<N>::NT;
  constexpr int PER = (N + NT - 1) / NT, PK = (N / 2 + NT) / NT;
  __shared__ float2 buf[N];
  __shared__ float2 tw[N];
  __shared__ float2 cs[N / 2 + 1];
  __shared__ double red[4 * (NT / kWave)];
  const int tid = threadIdx.x;
  const int pair = xcd_block(blockIdx.x, gridDim.x);
  const int r1 = 2 * pair, r2 = r1 + 1;
  float a1[PER], a2[PER], b1[PER], b2[PER], c1[PER], c2[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int i = min(tid + NT * t, N - 1);
    a1[t] = rho[(int64_t)r1 * N + i];
    a2[t] = rho[(int64_t)r2 * N + i];
  }
  // (pointer tests hoisted out of the loops so that the loads issue together)
  if (tau_part && base) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int i = min(tid + NT * t, N - 1);
      b1[t] = base[(int64_t)r1 * N + i];
      b2[t] = base[(int64_t)r2 * N + i];
    }
  } else {
#pragma unroll
    for (int t = 0; t < PER; ++t) b1[t] = b2[t] = 0.0f;
  }
  if (tau_part && cap) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int i = min(tid + NT * t, N - 1);
      c1[t] = cap[(int64_t)r1 * N + i];
      c2[t] = cap[(int64_t)r2 * N + i];
    }
  } else {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      c1[t] = fmaxf(0.0f, rho_t - fminf(rho_t, b1[t]));
      c2[t] = fmaxf(0.0f, rho_t - fminf(rho_t, b2[t]));
    }
  }
  stage_tables<N, NT, false>(tw, tw_g, cs, cs_g, nullptr, nullptr, tid);
  double s[4] = {0.0, 0.0, 0.0, 0.0};   // row sums r1, r2; overflow; movable
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    if (N % NT == 0 || tid + NT * t < N) {
      s[0] += a1[t];
      s[1] += a2[t];
      if (tau_part) {
        const float m1 = a1[t] - b1[t], m2 = a2[t] - b2[t];
        s[2] += fmaxf(0.0f, m1 - c1[t]);
        s[2] += fmaxf(0.0f, m2 - c2[t]);
        s[3] += m1;
        s[3] += m2;
      }
    }
  }
  block_sums<NT, 4>(s, red, tid);
  if (tid == 0) {
    rowsum[r1] = s[0];
    rowsum[r2] = s[1];
    if (tau_part) {
      tau_part[2 * pair] = s[2];
      tau_part[2 * pair + 1] = s[3];
    }
  }
  const float m1 = (float)(s[0] / N), m2 = (float)(s[1] / N);
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int i = tid + NT * t;
    if (N % NT == 0 || i < N) buf[mk_pos<N>(i)] = make_float2(a1[t] - m1, a2[t] - m2);
  }
  block_lds_sync<NT>();
  block_fft<N, NT, false, 1>(buf, nullptr, nullptr, nullptr, tw, tid);
#pragma unroll
  for (int t = 0; t < PK; ++t) {
    const int k = tid + NT * t;
    if (k > N / 2) continue;
    const int kp = (N - k) & (N - 1);
    float x1k, x2k, x1kp, x2kp;
    dct2_pair(buf[k], buf[kp], cs[k], x1k, x2k, x1kp, x2kp);
    if (k == 0) {
      x1k = (float)s[0];
      x2k = (float)s[1];
    }
    *reinterpret_cast<float2*>(&bT[(int64_t)k * N + r1]) = make_float2(x1k, x2k);
    if (k != 0 && k != N / 2)
      *reinterpret_cast<float2*>(&bT[(int64_t)kp * N + r1]) = make_float2(x1kp, x2kp);
  }
}

// ---------------------------------------------------------------------------
// Pass B: columns u1 = 2q, u2 = 2q+1 (rows of bT).  Column 0 is rebuilt from
// the double row sums minus their mean so that the DC never enters float32.
// ---------------------------------------------------------------------------
template <int N, bool DIFF, int NB>
__global__ void __launch_bounds__(FftShape<N>::NT)
    k_cols_solve(SpecBatch<NB> sb, const float2* __restrict__ tw_g,
                 const float2* __restrict__ cs_g, const float* __restrict__ wf_g) {
  const SpecReq& rq = sb.r[blockIdx.y];
  const float* __restrict__ bT = rq.bT;
  const double* __restrict__ rowsum = rq.rowsum;
  float* __restrict__ P = rq.P;
  float* __restrict__ Q = rq.Q;
  const float eps = rq.eps;
  constexpr int NT = FftShape<N>::NT;
  constexpr int PER = (N + NT - 1) / NT, PK = (N / 2 + NT) / NT;
  __shared__ float2 buf0[N];
  __shared__ float2 buf1[N];
  __shared__ float2 buf2[DIFF ? N : 1];
  __shared__ float2 tw[N];
  __shared__ float2 cs[N / 2 + 1];
  __shared__ float wf[N];
  __shared__ double red[NT / kWave];
  const int tid = threadIdx.x;
  const int q = xcd_block(blockIdx.x, gridDim.x);
  const int u1 = 2 * q, u2 = u1 + 1;
  float c1[PER], c2[PER];
  if (u1 == 0) {
    double rs[PER];
    double s[1] = {0.0};
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      rs[t] = rowsum[min(tid + NT * t, N - 1)];
      if (N % NT == 0 || tid + NT * t < N) s[0] += rs[t];
    }
    block_sums<NT, 1>(s, red, tid);
    const double mean0 = s[0] / N;
#pragma unroll
    for (int t = 0; t < PER; ++t) c1[t] = (float)(rs[t] - mean0);
  } else {
#pragma unroll
    for (int t = 0; t < PER; ++t) c1[t] = bT[(int64_t)u1 * N + min(tid + NT * t, N - 1)];
  }
#pragma unroll
  for (int t = 0; t < PER; ++t) c2[t] = bT[(int64_t)u2 * N + min(tid + NT * t, N - 1)];
  stage_tables<N, NT, true>(tw, tw_g, cs, cs_g, wf, wf_g, tid);
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int i = tid + NT * t;
    if (N % NT == 0 || i < N) buf0[mk_pos<N>(i)] = make_float2(c1[t], c2[t]);
  }
  block_lds_sync<NT>();
  block_fft<N, NT, false, 1>(buf0, nullptr, nullptr, nullptr, tw, tid);
  const float inv_n2 = 1.0f / ((float)N * (float)N);
  const float wu1 = wf[u1], wu2 = wf[u2];
  const float f1 = (u1 == 0 ? 1.0f : 2.0f) * inv_n2, f2 = 2.0f * inv_n2;
#pragma unroll
  for (int t = 0; t < PK; ++t) {
    const int k = tid + NT * t;
    if (k > N / 2) continue;
    const int kp = (N - k) & (N - 1);
    const float2 c = cs[k];
    float x1k, x2k, x1kp, x2kp;
    dct2_pair(buf0[k], buf0[kp], c, x1k, x2k, x1kp, x2kp);
    const float wk = wf[k], wkp = wf[kp];
    const float ck = (k == 0 ? 1.0f : 2.0f), ckp = (kp == 0 ? 1.0f : 2.0f);
    float g1k = x1k * (f1 * ck) / (wu1 * wu1 + wk * wk + eps);
    float g1kp = x1kp * (f1 * ckp) / (wu1 * wu1 + wkp * wkp + eps);
    const float g2k = x2k * (f2 * ck) / (wu2 * wu2 + wk * wk + eps);
    const float g2kp = x2kp * (f2 * ckp) / (wu2 * wu2 + wkp * wkp + eps);
    if (u1 == 0 && k == 0) g1k = 0.0f;   // a_00 := 0
    // P: DCT-III of G.  Q: DCT-III of Yb with Yb_k = w_{n-k} G_{n-k} (k >= 1),
    // Yb_0 = 0.  The two columns' P share one complex FFT and their Q another:
    // sequences packed together must have similar magnitudes (P ~ 1/w^2 is far
    // larger than Q ~ 1/w), or the rounding of one swamps the other.
    const bool k0 = (k == 0);
    float2 h1, h1p, h2, h2p;
    dct3_herm(g1k, g1kp, c, k0, h1, h1p);
    dct3_herm(g2k, g2kp, c, k0, h2, h2p);
    buf0[k] = pack2(h1, h2);
    if (!k0 && k != N / 2) buf0[kp] = pack2(h1p, h2p);
    if (!DIFF) {
      dct3_herm(k0 ? 0.0f : wkp * g1kp, k0 ? 0.0f : wk * g1k, c, k0, h1, h1p);
      dct3_herm(k0 ? 0.0f : wkp * g2kp, k0 ? 0.0f : wk * g2k, c, k0, h2, h2p);
      buf1[k] = pack2(h1, h2);
      if (!k0 && k != N / 2) buf1[kp] = pack2(h1p, h2p);
    } else {
      // R = DCT-III((cos w - 1) G) (buf1) - sine transform of sin(w) G (buf2)
      float dmk, dmkp, sw;
      diff_weights(c, dmk, dmkp, sw);
      dct3_herm(dmk * g1k, dmkp * g1kp, c, k0, h1, h1p);
      dct3_herm(dmk * g2k, dmkp * g2kp, c, k0, h2, h2p);
      buf1[k] = pack2(h1, h2);
      if (!k0 && k != N / 2) buf1[kp] = pack2(h1p, h2p);
      dct3_herm(k0 ? 0.0f : sw * g1kp, k0 ? 0.0f : sw * g1k, c, k0, h1, h1p);
      dct3_herm(k0 ? 0.0f : sw * g2kp, k0 ? 0.0f : sw * g2k, c, k0, h2, h2p);
      buf2[k] = pack2(h1, h2);
      if (!k0 && k != N / 2) buf2[kp] = pack2(h1p, h2p);
    }
  }
  block_lds_sync<NT>();
  block_fft<N, NT, true, DIFF ? 3 : 2>(buf0, buf1, buf2, nullptr, tw, tid);
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int iy = tid + NT * t;
    if (N % NT != 0 && iy >= N) continue;
    const int mpos = mk_pos<N>(iy);
    const float2 zp = buf0[mpos], zq = buf1[mpos];
    const float sg = (iy & 1) ? -1.0f : 1.0f;
    *reinterpret_cast<float2*>(&P[(int64_t)iy * N + u1]) = zp;
    if (!DIFF) {
      *reinterpret_cast<float2*>(&Q[(int64_t)iy * N + u1]) = make_float2(sg * zq.x, sg * zq.y);
    } else {
      const float2 zs = buf2[mpos];
      *reinterpret_cast<float2*>(&Q[(int64_t)iy * N + u1]) =
          make_float2(zq.x - sg * zs.x, zq.y - sg * zs.y);
    }
  }
}

// ---------------------------------------------------------------------------
// Pass C: rows r1 = 2p, r2 = 2p+1 of P and Q -> psi, Ex, Ey; energy.
// ---------------------------------------------------------------------------
template <int N, bool DIFF, int NB>
__global__ void __launch_bounds__(FftShape<N>::NT)
    k_rows_inverse(SpecBatch<NB> sb, const float2* __restrict__ tw_g,
                   const float2* __restrict__ cs_g, const float* __restrict__ wf_g) {
  const SpecReq& rq = sb.r[blockIdx.y];
  const float* __restrict__ P = rq.P;
  const float* __restrict__ Q = rq.Q;
  const float* __restrict__ rho = rq.rho;
  float* __restrict__ psi = rq.psi;
  float* __restrict__ ex = rq.ex;
  float* __restrict__ ey = rq.ey;
  float2* __restrict__ exy = rq.exy;
  double* __restrict__ energy = rq.en_part;
  constexpr int NT = FftShape<N>::NT;
  constexpr int PER = (N + NT - 1) / NT, PK = (N / 2 + NT) / NT;
  __shared__ float2 bufa[N];
  __shared__ float2 bufb[N];
  __shared__ float2 bufc[N];
  __shared__ float2 bufd[DIFF ? N : 1];
  __shared__ float2 tw[N];
  __shared__ float2 cs[N / 2 + 1];
  __shared__ float wf[N];
  __shared__ float rows[4 * N];
  __shared__ double red[NT / kWave];
  const int tid = threadIdx.x;
  const int pr = xcd_block(blockIdx.x, gridDim.x);
  const int r1 = 2 * pr, r2 = r1 + 1;
  // rows P[r1], P[r2], Q[r1], Q[r2] (and rho for the energy): all loads first
  float v[4][PER], e1[PER], e2[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int i = min(tid + NT * t, N - 1);
    v[0][t] = P[(int64_t)r1 * N + i];
    v[1][t] = P[(int64_t)r2 * N + i];
    v[2][t] = Q[(int64_t)r1 * N + i];
    v[3][t] = Q[(int64_t)r2 * N + i];
  }
  if (energy) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int i = min(tid + NT * t, N - 1);
      e1[t] = rho[(int64_t)r1 * N + i];
      e2[t] = rho[(int64_t)r2 * N + i];
    }
  }
  stage_tables<N, NT, true>(tw, tw_g, cs, cs_g, wf, wf_g, tid);
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int i = tid + NT * t;
    if (N % NT == 0 || i < N) {
#pragma unroll
      for (int r = 0; r < 4; ++r) rows[r * N + i] = v[r][t];
    }
  }
  block_lds_sync<NT>();
  const float* P1 = rows;
  const float* P2 = rows + N;
  const float* Q1 = rows + 2 * N;
  const float* Q2 = rows + 3 * N;
#pragma unroll
  for (int t = 0; t < PK; ++t) {
    const int k = tid + NT * t;
    if (k > N / 2) continue;
    const int kp = (N - k) & (N - 1);
    const bool k0 = (k == 0), self = k0 || k == N / 2;
    const float2 c = cs[k];
    const float wk = wf[k], wkp = wf[kp];
    const float p1k = P1[k], p1kp = P1[kp], p2k = P2[k], p2kp = P2[kp];
    // like-magnitude pairs share a complex FFT: (psi r1, psi r2), (Ey r1, Ey r2),
    // (Ex r1, Ex r2)
    float2 ha, hap, hb, hbp;
    dct3_herm(p1k, p1kp, c, k0, ha, hap);
    dct3_herm(p2k, p2kp, c, k0, hb, hbp);
    bufa[k] = pack2(ha, hb);
    if (!self) bufa[kp] = pack2(hap, hbp);
    dct3_herm(Q1[k], Q1[kp], c, k0, ha, hap);
    dct3_herm(Q2[k], Q2[kp], c, k0, hb, hbp);
    bufb[k] = pack2(ha, hb);
    if (!self) bufb[kp] = pack2(hap, hbp);
    if (!DIFF) {
      dct3_herm(k0 ? 0.0f : wkp * p1kp, k0 ? 0.0f : wk * p1k, c, k0, ha, hap);
      dct3_herm(k0 ? 0.0f : wkp * p2kp, k0 ? 0.0f : wk * p2k, c, k0, hb, hbp);
      bufc[k] = pack2(ha, hb);
      if (!self) bufc[kp] = pack2(hap, hbp);
    } else {
      // Dx = DCT-III((cos w - 1) P) (bufc) - sine transform of sin(w) P (bufd)
      float dmk, dmkp, sw;
      diff_weights(c, dmk, dmkp, sw);
      dct3_herm(dmk * p1k, dmkp * p1kp, c, k0, ha, hap);
      dct3_herm(dmk * p2k, dmkp * p2kp, c, k0, hb, hbp);
      bufc[k] = pack2(ha, hb);
      if (!self) bufc[kp] = pack2(hap, hbp);
      dct3_herm(k0 ? 0.0f : sw * p1kp, k0 ? 0.0f : sw * p1k, c, k0, ha, hap);
      dct3_herm(k0 ? 0.0f : sw * p2kp, k0 ? 0.0f : sw * p2k, c, k0, hb, hbp);
      bufd[k] = pack2(ha, hb);
      if (!self) bufd[kp] = pack2(hap, hbp);
    }
  }
  block_lds_sync<NT>();
  block_fft<N, NT, true, DIFF ? 4 : 3>(bufa, bufb, bufc, bufd, tw, tid);
  double en[1] = {0.0};
#pragma unroll
  for (int t = 0; t < PER; ++t) {
    const int ix = tid + NT * t;
    if (N % NT != 0 && ix >= N) continue;
    const int mpos = mk_pos<N>(ix);
    const float2 za = bufa[mpos], zb = bufb[mpos];
    const float sg = (ix & 1) ? -1.0f : 1.0f;
    float2 zc = bufc[mpos];
    if (DIFF) {
      // (Dx, Dy) instead of (Ex, Ey): zc holds Dx after the sign below
      const float2 zd = bufd[mpos];
      zc = make_float2(sg * (zc.x - sg * zd.x), sg * (zc.y - sg * zd.y));
    }
    const int64_t o1 = (int64_t)r1 * N + ix, o2 = (int64_t)r2 * N + ix;
    if (psi) {
      psi[o1] = za.x;
      psi[o2] = za.y;
    }
    if (ex) {
      ex[o1] = sg * zc.x;
      ex[o2] = sg * zc.y;
    }
    if (ey) {
      ey[o1] = zb.x;
      ey[o2] = zb.y;
    }
    if (exy) {
      exy[o1] = make_float2(sg * zc.x, zb.x);
      exy[o2] = make_float2(sg * zc.y, zb.y);
    }
    if (energy) en[0] += (double)e1[t] * za.x + (double)e2[t] * za.y;
  }
  if (energy) {
    block_sums<NT, 1>(en, red, tid);
    if (tid == 0) energy[pr] = en[0];   // per-block partial
  }
}

template <int N, int NB>
hipError_t run_fft_nb(Plan& p, const SpecBatch<NB>& sb, bool diff, hipStream_t s) {
  const dim3 grid(N / 2, sb.count), block(FftShape<N>::NT);
  hipLaunchKernelGGL((k_rows_dct2<N, NB>), grid, block, 0, s, sb, p.fft_tw, p.dct_cs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  plan_mark(p, "k_rows_dct2", s);
  if (diff)
    hipLaunchKernelGGL((k_cols_solve<N, true, NB>), grid, block, 0, s, sb, p.fft_tw, p.dct_cs,
                       p.wfreq);
  else
    hipLaunchKernelGGL((k_cols_solve<N, false, NB>), grid, block, 0, s, sb, p.fft_tw,
                       p.dct_cs, p.wfreq);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  plan_mark(p, "k_cols_solve", s);
  if (diff)
    hipLaunchKernelGGL((k_rows_inverse<N, true, NB>), grid, block, 0, s, sb, p.fft_tw,
                       p.dct_cs, p.wfreq);
  else
    hipLaunchKernelGGL((k_rows_inverse<N, false, NB>), grid, block, 0, s, sb, p.fft_tw,
                       p.dct_cs, p.wfreq);
  e = hipGetLastError();
  plan_mark(p, "k_rows_inverse", s);
  return e;
}

// The descriptor of request a for the plan's batch slot `slot`.
SpecReq spec_req(Plan& p, const SpectralArgs& a, int slot) {
  const size_t nn = (size_t)p.n * p.n;
  SpecReq q;
  q.rho = a.rho;
  q.psi = a.psi;
  q.ex = a.ex;
  q.ey = a.ey;
  q.exy = reinterpret_cast<float2*>(a.exy);
  q.bT = p.tmp0 + slot * nn;
  q.rowsum = p.rowsum + (size_t)slot * p.n;
  q.P = p.tmp1 + slot * nn;
  q.Q = p.tmp2 + slot * nn;
  q.base = a.base;
  q.cap = a.cap;
  q.rho_t = a.rho_t;
  q.eps = a.eps;
  q.en_part = a.en_part;
  q.tau_part = a.tau_part;
  return q;
}

template <int N>
hipError_t run_fft(Plan& p, const SpectralArgs* a, int count, hipStream_t s) {
  if (count == 1) {
    SpecBatch<1> sb;
    sb.count = 1;
    sb.r[0] = spec_req(p, a[0], 0);
    return run_fft_nb<N, 1>(p, sb, a[0].diff, s);
  }
  SpecBatch<kMaxBatch> sb;
  sb.count = count;
  for (int i = 0; i < count; ++i) sb.r[i] = spec_req(p, a[i], i);
  return run_fft_nb<N, kMaxBatch>(p, sb, a[0].diff, s);
}

}  // namespace

hipError_t spectral_fft_batch(Plan& p, const SpectralArgs* a, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  if (count > p.max_batch) return hipErrorInvalidValue;
  for (int i = 1; i < count; ++i)
    if (a[i].diff != a[0].diff) return hipErrorInvalidValue;
  switch (p.n) {
    case 8: return run_fft<8>(p, a, count, s);
    case 16: return run_fft<16>(p, a, count, s);
    case 32: return run_fft<32>(p, a, count, s);
    case 64: return run_fft<64>(p, a, count, s);
    case 128: return run_fft<128>(p, a, count, s);
    case 256: return run_fft<256>(p, a, count, s);
    case 512: return run_fft<512>(p, a, count, s);
    case 1024: return run_fft<1024>(p, a, count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t spectral_fft(Plan& p, const SpectralArgs& a, hipStream_t s) {
  return spectral_fft_batch(p, &a, 1, s);
}

}  // namespace fftpl
