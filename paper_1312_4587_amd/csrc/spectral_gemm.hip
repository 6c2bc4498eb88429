// Spectral solve (Eqs. (9)-(12)) as dense cosine/sine-matrix products on the
// matrix cores: the same transforms as the FFT path, written as five GEMMs.
// With K[u][i] = cos(w_u (i+1/2)), S[u][i] = sin(w_u (i+1/2)), w_u = pi u / n,
// Sw = diag(w) S and R = rho - mean(rho) (mean in double, so the large DC
// never enters the float32 sums):
//   W  = R K^T                         (along x)
//   G  = scale(K W)                    (along y; c_u c_v / n^2 / (w_u^2+w_v^2+eps),
//                                       zero at (0,0): the DC is removed)
//   [U | V]     = G [K | Sw]           (inverse along x: cos for psi and Ey,
//                                       frequency-weighted sine for Ex)
//   [psi ; Ey]  = [K^T ; Sw^T] U       (inverse along y)
//   Ex          = K^T V
// 7 n^3 multiply-adds in all as written; with n a multiple of 128 and the
// fields (not the differences) wanted, the even/odd symmetry of K and Sw
// halves that (the split products, below run_gemm_split).  Two precisions:
//   FP32:   v_mfma_f32_16x16x4_f32 on float32 operands;
//   BF16X3: every float32 operand X is split into bf16 hi = bf16(X) and
//           lo = bf16(X - hi); each product is Ah Bh + Ah Bl + Al Bh on
//           v_mfma_f32_16x16x32_bf16 with float32 accumulation.
// Block tile 64 x 64, eight waves: four quarters of 32 x 32 (2 x 2 MFMA
// tiles of 16 x 16) times two halves of every K step of 64, staged in LDS,
// double-buffered.  The constant matrices are built once per plan in
// double and rounded (and split) once.
#include <math.h>
#include <string.h>

#include <type_traits>
#include <vector>

#include "fftpl_internal.hpp"

namespace fftpl {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int TM = 64, TN = 64, TK = 32;

// EPI_F32_T: float32 stored transposed.  EPI_DUAL_X / EPI_DUAL_Y (dual
// products, see GemmArgs): P1 + P2 at (row, col) and dsign (P1 - P2) at the
// mirrored column n - 1 - col (X) or row n - 1 - row (Y).
enum EpiMode {
  EPI_F32 = 0, EPI_SPLIT = 1, EPI_SPLIT_T = 2, EPI_PSI_EY = 3, EPI_EX = 4, EPI_F32_T = 5,
  EPI_DUAL_X = 6, EPI_DUAL_Y = 7
};

struct GemmArgs {
  const void* a_hi = nullptr;   // A [M][K] row-major (float32, or bf16 hi)
  const void* a_lo = nullptr;   // bf16 lo of A
  int lda = 0;
  const void* b_hi = nullptr;   // float32: B [K][N] row-major; bf16: B^T [N][K] row-major
  const void* b_lo = nullptr;
  int ldb = 0;
  int M = 0, N = 0, K = 0;
  // dual: a second product P2 = A2 B2 of the same shape (same leading
  // dimensions) beside P1 = A B; the block's two K halves run one each and
  // the epilogue receives P1 + P2 and P1 - P2 (the even/odd butterfly)
  int dual = 0;
  const void* a2_hi = nullptr;
  const void* a2_lo = nullptr;
  const void* b2_hi = nullptr;
  const void* b2_lo = nullptr;
};

struct Epi {
  int mode = EPI_F32;
  // 1: scale element (row v, col u) by c_u c_v / (n^2 (w_u^2 + w_v^2 + eps));
  // 2: the same for an even/odd split product, row b being v = 2 b + vpar
  // and column u' being u = 2 u' (u' < n/2) or 2 (u' - n/2) + 1
  int spectral = 0;
  int vpar = 0;
  float eps = 0.0f;
  int n = 0;
  const float* wf = nullptr;
  float* out = nullptr;
  int ldo = 0;
  __bf16* hi = nullptr;
  __bf16* lo = nullptr;
  float* psi = nullptr;
  float* ex = nullptr;
  float* ey = nullptr;
  float* exy = nullptr;
  const float* rho = nullptr;
  double* en_part = nullptr;
  int en_slots = 1;       // energy partials per block: the sum, then zeros
  float dsign = 1.0f;     // dual: the mirrored output is dsign (P1 - P2)
  float* f = nullptr;     // EPI_DUAL_Y: the map written (psi, Ex or Ey)
  int exy_off = -1;       // EPI_DUAL_Y: also exy[2 o + exy_off] (0: Ex, 1: Ey)
};

constexpr int kGemmMaxProb = 3;
// Up to kGemmMaxProb products of one shape in one launch (blockIdx.y).
struct GemmBatch {
  int count = 1;
  GemmArgs g[kGemmMaxProb];
  Epi ep[kGemmMaxProb];
};

__device__ __forceinline__ void split_bf16(float v, __bf16& hi, __bf16& lo) {
  hi = (__bf16)v;
  lo = (__bf16)(v - (float)hi);
}

// One element of a product's result: optional spectral scaling, then the
// store the step needs (see EpiMode); en gathers rho * psi for the energy.
__device__ __forceinline__ float spectral_scale(const Epi& ep, int row, int col, float v) {
  const int n = ep.n;
  const float inv_n2 = 1.0f / ((float)n * (float)n);
  int u = col, w = row;
  if (ep.spectral == 2) {
    const int h = n / 2;
    w = 2 * row + ep.vpar;
    u = col < h ? 2 * col : 2 * (col - h) + 1;
  }
  const float wu = ep.wf[u], wv = ep.wf[w];
  const float cu = u ? 2.0f : 1.0f, cv = w ? 2.0f : 1.0f;
  return (w == 0 && u == 0) ? 0.0f : v * (cu * cv * inv_n2) / (wu * wu + wv * wv + ep.eps);
}

__device__ __forceinline__ void epi_store(const Epi& ep, int row, int col, float v, double& en) {
  const int n = ep.n;
  if (ep.spectral) v = spectral_scale(ep, row, col, v);
  if (ep.mode == EPI_F32) {
    ep.out[(size_t)row * ep.ldo + col] = v;
  } else if (ep.mode == EPI_F32_T) {
    ep.out[(size_t)col * ep.ldo + row] = v;
  } else if (ep.mode == EPI_SPLIT || ep.mode == EPI_SPLIT_T) {
    __bf16 h, l;
    split_bf16(v, h, l);
    const size_t o =
        ep.mode == EPI_SPLIT ? (size_t)row * ep.ldo + col : (size_t)col * ep.ldo + row;
    ep.hi[o] = h;
    ep.lo[o] = l;
  } else if (ep.mode == EPI_PSI_EY) {
    if (row < n) {
      const size_t o = (size_t)row * n + col;
      if (ep.psi) ep.psi[o] = v;
      if (ep.rho) en += (double)ep.rho[o] * v;
    } else {
      const size_t o = (size_t)(row - n) * n + col;
      if (ep.ey) ep.ey[o] = v;
      if (ep.exy) ep.exy[2 * o + 1] = v;
    }
  } else {   // EPI_EX
    const size_t o = (size_t)row * n + col;
    if (ep.ex) ep.ex[o] = v;
    if (ep.exy) ep.exy[2 * o] = v;
  }
}

// The two outputs of a dual product's element (row, col): vs = P1 + P2 there,
// dsign vd = dsign (P1 - P2) at the mirrored column (EPI_DUAL_X: bf16 hi/lo
// stored transposed, or float32 row-major) or row (EPI_DUAL_Y: n x n maps).
__device__ __forceinline__ void epi_store_dual(const Epi& ep, int row, int col, float vs,
                                               float vd, double& en) {
  const int n = ep.n;
  const float v2 = ep.dsign * vd;
  if (ep.mode == EPI_DUAL_X) {
    const int c2 = n - 1 - col;
    if (ep.hi) {
      __bf16 h, l;
      split_bf16(vs, h, l);
      ep.hi[(size_t)col * ep.ldo + row] = h;
      ep.lo[(size_t)col * ep.ldo + row] = l;
      split_bf16(v2, h, l);
      ep.hi[(size_t)c2 * ep.ldo + row] = h;
      ep.lo[(size_t)c2 * ep.ldo + row] = l;
    } else {
      ep.out[(size_t)row * ep.ldo + col] = vs;
      ep.out[(size_t)row * ep.ldo + c2] = v2;
    }
  } else {   // EPI_DUAL_Y
    const size_t o1 = (size_t)row * n + col, o2 = (size_t)(n - 1 - row) * n + col;
    if (ep.f) {
      ep.f[o1] = vs;
      ep.f[o2] = v2;
    }
    if (ep.exy) {
      ep.exy[2 * o1 + ep.exy_off] = vs;
      ep.exy[2 * o2 + ep.exy_off] = v2;
    }
    if (ep.rho) en += (double)ep.rho[o1] * vs + (double)ep.rho[o2] * v2;
  }
}

// KS x 4 waves: wave w works on the 32 x 32 quarter (w & 3) of the tile over
// the K part (w >> 2) of every K step of TKB = KS * 32; with KS = 2 the two
// parts' partial tiles are added through LDS before the epilogue (in a fixed
// order).  KS = 2 doubles the waves per CU for grids of one block per CU.
template <bool BF16, int KS>
__global__ void __launch_bounds__(256 * KS) k_gemm(GemmBatch gb) {
  const GemmArgs& g = gb.g[blockIdx.y];
  const Epi& ep = gb.ep[blockIdx.y];
  constexpr int TKB = KS * TK;
  // dual (KS = 2 only): each K step holds TK of the first product, then TK of
  // the second, so the wavefronts of K half 0 run P1 and those of half 1 P2
  const bool dual = KS == 2 && g.dual;
  const int kstep = dual ? TK : TKB;   // K of each product per step
  const int steps = g.K / kstep;
  // Each XCD runs a contiguous range of logical tiles (xcd_block); inside
  // it the tiles go down gsz rows of tiles before moving one column right, so
  // the range covers a compact patch whose A row panels and B column panels
  // share the XCD's L2.
  const int tiles_n = g.N / TN, tiles_m = g.M / TM;
  const int lt = xcd_block(blockIdx.x, gridDim.x);
  const int per_xcd = gridDim.x % kNumXcd ? (int)gridDim.x : (int)gridDim.x / kNumXcd;
  const int gsz = per_xcd >= 64 ? 8 : per_xcd >= 16 ? 4 : per_xcd >= 4 ? 2 : 1;
  const int group = lt / (gsz * tiles_n), first = group * gsz;
  const int gm = min(tiles_m - first, gsz);
  const int m0 = (first + (lt % (gsz * tiles_n)) % gm) * TM;
  const int n0 = ((lt % (gsz * tiles_n)) / gm) * TN;
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  const int wq = w & 3, wk = w >> 2;
  const int wm = (wq >> 1) * 32, wn = (wq & 1) * 32;
  const int l16 = lane & 15, lg = lane >> 4;
  f4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  // Double-buffered K loop: the next K step's operands are loaded from
  // global memory into registers while the MFMAs run on the current LDS
  // tile, then stored to the other LDS buffer; one barrier per step.
  // bf16: [hi, lo] x [A, B] x 2 buffers of TM rows of TKB / 8 + 1 chunks of
  // 16 bytes (one chunk of padding per row, see below)
  constexpr int kFloatsF32 = 2 * 2 * 2 * TK * (TM + 4);
  constexpr int kFloatsBf16 = 2 * 2 * 2 * TM * (TKB / 8 + 1) * 4;
  constexpr int kFloats = BF16 ? kFloatsBf16 : kFloatsF32;
  __shared__ __attribute__((aligned(16))) float smem[kFloats];
  if constexpr (!BF16) {
    float(*As)[TKB][TM + 4] = reinterpret_cast<float(*)[TKB][TM + 4]>(smem);   // [buf][k][m]
    float(*Bs)[TKB][TN + 4] =
        reinterpret_cast<float(*)[TKB][TN + 4]>(smem + 2 * TKB * (TM + 4));   // [buf][k][n]
    const int ar = t / (TKB / 8), ak = (t % (TKB / 8)) * 8;   // A: row, first k of 8
    const int bk = t >> 3, bn = (t & 7) * 8;     // B: k, first n of 8
    const bool a2 = dual && ak >= TK, b2 = dual && bk >= TK;
    const float* A = static_cast<const float*>(a2 ? g.a2_hi : g.a_hi);
    const float* B = static_cast<const float*>(b2 ? g.b2_hi : g.b_hi);
    const int akc = a2 ? ak - TK : ak, bkr = b2 ? bk - TK : bk;
    float4 a0, a1, b0, b1;
    auto fetch = [&](int s) {
      const int k0 = s * kstep;
      const float4* sa = reinterpret_cast<const float4*>(A + (size_t)(m0 + ar) * g.lda + k0 + akc);
      const float4* sb = reinterpret_cast<const float4*>(B + (size_t)(k0 + bkr) * g.ldb + n0 + bn);
      a0 = sa[0];
      a1 = sa[1];
      b0 = sb[0];
      b1 = sb[1];
    };
    auto stash = [&](int buf) {
      As[buf][ak + 0][ar] = a0.x;
      As[buf][ak + 1][ar] = a0.y;
      As[buf][ak + 2][ar] = a0.z;
      As[buf][ak + 3][ar] = a0.w;
      As[buf][ak + 4][ar] = a1.x;
      As[buf][ak + 5][ar] = a1.y;
      As[buf][ak + 6][ar] = a1.z;
      As[buf][ak + 7][ar] = a1.w;
      *reinterpret_cast<float4*>(&Bs[buf][bk][bn]) = b0;
      *reinterpret_cast<float4*>(&Bs[buf][bk][bn + 4]) = b1;
    };
    fetch(0);
    stash(0);
    __syncthreads();
    int cur = 0;
    for (int s = 0; s < steps; ++s) {
      const bool more = s + 1 < steps;
      if (more) fetch(s + 1);
#pragma unroll
      for (int kk = 0; kk < TK; kk += 4) {
        const int kq = wk * TK + kk + lg;
        const float x0 = As[cur][kq][wm + l16], x1 = As[cur][kq][wm + 16 + l16];
        const float y0 = Bs[cur][kq][wn + l16], y1 = Bs[cur][kq][wn + 16 + l16];
        acc[0][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, y0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x0, y1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, y0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_16x16x4f32(x1, y1, acc[1][1], 0, 0, 0);
      }
      if (more) stash(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  } else {
    // tiles keep 8 consecutive k of one row (A) or one column (B^T) together,
    // which is what one lane feeds to the 16x16x32 bf16 MFMA
    // Rows are KC + 1 chunks long: the eight lanes one LDS cycle serves read
    // the same chunk of eight consecutive rows, which with unpadded rows of
    // 128 (or 64) bytes would all fall on the same banks.
    constexpr int KC = TKB / 8;   // bf8 chunks per row and K step
    constexpr int KCP = KC + 1;
    static_assert(TM == TN, "A and B tiles share the padded row layout");
    bf8(*Ah)[TM][KCP] = reinterpret_cast<bf8(*)[TM][KCP]>(smem);
    bf8(*Al)[TM][KCP] = Ah + 2;
    bf8(*Bh)[TN][KCP] = reinterpret_cast<bf8(*)[TN][KCP]>(Ah + 4);
    bf8(*Bl)[TN][KCP] = Bh + 2;
    const int r = t / KC, kc = t % KC;
    const bool two = dual && kc >= KC / 2;   // this thread loads the second product
    const __bf16* gah = static_cast<const __bf16*>(two ? g.a2_hi : g.a_hi);
    const __bf16* gal = static_cast<const __bf16*>(two ? g.a2_lo : g.a_lo);
    const __bf16* gbh = static_cast<const __bf16*>(two ? g.b2_hi : g.b_hi);
    const __bf16* gbl = static_cast<const __bf16*>(two ? g.b2_lo : g.b_lo);
    const int kcol = (two ? kc - KC / 2 : kc) * 8;
    // Operands of the next PRE K steps are in flight in registers while the
    // MFMAs of the current step run from LDS.  Register set j holds step
    // s0 + j and is refilled right after being stored to LDS.  The body has
    // no data-dependent branches (loads past the last step re-read the last
    // step, the store after the last step fills the idle buffer) so that
    // every wait is for the oldest loads only.
    const int kq = wk * (TK / 8) + lg;
    auto run = [&](auto pre) {
      constexpr int PRE = decltype(pre)::value;
      bf8 rah[PRE], ral[PRE], rbh[PRE], rbl[PRE];
      auto fetch = [&](int q, int step) {
        const int k0 = min(step, steps - 1) * kstep + kcol;
        const size_t oa = (size_t)(m0 + r) * g.lda + k0;
        const size_t ob = (size_t)(n0 + r) * g.ldb + k0;
        rah[q] = *reinterpret_cast<const bf8*>(gah + oa);
        ral[q] = *reinterpret_cast<const bf8*>(gal + oa);
        rbh[q] = *reinterpret_cast<const bf8*>(gbh + ob);
        rbl[q] = *reinterpret_cast<const bf8*>(gbl + ob);
      };
      auto stash = [&](int q, int buf) {
        Ah[buf][r][kc] = rah[q];
        Al[buf][r][kc] = ral[q];
        Bh[buf][r][kc] = rbh[q];
        Bl[buf][r][kc] = rbl[q];
      };
#pragma unroll
      for (int q = 0; q < PRE; ++q) fetch(q, q);
      stash(0, 0);
      __syncthreads();
      for (int s0 = 0; s0 < steps; s0 += PRE) {
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
          const int cur = (s0 + j) & 1;
          fetch(j, s0 + j + PRE);
          const bf8 xh0 = Ah[cur][wm + l16][kq], xl0 = Al[cur][wm + l16][kq];
          const bf8 xh1 = Ah[cur][wm + 16 + l16][kq], xl1 = Al[cur][wm + 16 + l16][kq];
          const bf8 yh0 = Bh[cur][wn + l16][kq], yl0 = Bl[cur][wn + l16][kq];
          const bf8 yh1 = Bh[cur][wn + 16 + l16][kq], yl1 = Bl[cur][wn + 16 + l16][kq];
#define FFTPL_MFMA3(ACC, XH, XL, YH, YL)                                      \
  ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(XH, YH, ACC, 0, 0, 0);        \
  ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(XH, YL, ACC, 0, 0, 0);        \
  ACC = __builtin_amdgcn_mfma_f32_16x16x32_bf16(XL, YH, ACC, 0, 0, 0);
          FFTPL_MFMA3(acc[0][0], xh0, xl0, yh0, yl0)
          FFTPL_MFMA3(acc[0][1], xh0, xl0, yh1, yl1)
          FFTPL_MFMA3(acc[1][0], xh1, xl1, yh0, yl0)
          FFTPL_MFMA3(acc[1][1], xh1, xl1, yh1, yl1)
#undef FFTPL_MFMA3
          stash((j + 1) % PRE, cur ^ 1);
          __syncthreads();
        }
      }
    };
    if (steps % 4 == 0)
      run(std::integral_constant<int, 4>{});
    else
      run(std::integral_constant<int, 1>{});
  }

  // the second K half's partial tile joins the first one's (waves 0-3 keep
  // going to the epilogue; the loop's last barrier has freed the buffers);
  // dual: acc = P1 + P2 and dif = P1 - P2
  f4 dif[2][2];
  if (KS == 2) {
    f4* red = reinterpret_cast<f4*>(smem);   // [quarter][i][j][lane]
    if (wk == 1) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) red[((wq * 2 + i) * 2 + j) * kWave + lane] = acc[i][j];
    }
    __syncthreads();
    if (wk == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const f4 o = red[((wq * 2 + i) * 2 + j) * kWave + lane];
          dif[i][j] = acc[i][j] - o;
          acc[i][j] += o;
        }
    }
  }

  // Single-map outputs (EPI_F32, EPI_SPLIT, their transposed forms and
  // EPI_DUAL_X): the tile goes through LDS so that each thread writes a
  // contiguous run of one output row (for the transposed forms, instead of
  // single elements one row apart; for the mirrored half of a float32
  // EPI_DUAL_X, a run in reverse order).
  const bool trans = ep.mode == EPI_F32_T || ep.mode == EPI_SPLIT_T ||
                     (ep.mode == EPI_DUAL_X && ep.hi);
  if (trans || ep.mode == EPI_F32 || ep.mode == EPI_SPLIT || ep.mode == EPI_DUAL_X) {
    constexpr int TP = TM + 1;                       // padded row of a transposed tile
    constexpr int SEG = TM * TN / (256 * KS);        // elements per thread: 16 or 8
    static_assert(2 * TN * TP <= kFloats, "two transposed tiles fit the LDS buffers");
    float* T1 = smem;             // [col][row] (transposed) or [row][col]
    float* T2 = smem + TN * TP;   // dual: the mirrored output
    __syncthreads();              // every read of the K-half reduction is done
    if (wk == 0) {
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int c = wn + 16 * j + l16, rr = wm + 16 * i + 4 * lg + r;
            const int x = trans ? c * TP + rr : rr * TP + c;
            T1[x] = acc[i][j][r];
            if (dual) T2[x] = ep.dsign * dif[i][j][r];
          }
    }
    __syncthreads();
    // thread t: line c of the staged tile (an output row), elements r0..
    const int c = t / (TM / SEG), r0 = (t % (TM / SEG)) * SEG;
    auto put = [&](const float* T, int oline) {
      float v[SEG];
#pragma unroll
      for (int q = 0; q < SEG; ++q) v[q] = T[c * TP + r0 + q];
      if (!trans && ep.spectral) {
#pragma unroll
        for (int q = 0; q < SEG; ++q) v[q] = spectral_scale(ep, m0 + c, n0 + r0 + q, v[q]);
      }
      const size_t o = trans ? (size_t)oline * ep.ldo + m0 + r0
                             : (size_t)(m0 + c) * ep.ldo + n0 + r0;
      if (!trans && ep.mode == EPI_DUAL_X) {
        // float32 row-major: the first output at (row, n0 + r0 ..), the
        // mirrored one at (row, n - 1 - (n0 + r0 + SEG - 1) ..) reversed
        if (T == T1) {
#pragma unroll
          for (int q = 0; q < SEG; q += 4)
            *reinterpret_cast<float4*>(ep.out + o + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
        } else {
          const size_t o2 = (size_t)(m0 + c) * ep.ldo + (ep.n - n0 - r0 - SEG);
#pragma unroll
          for (int q = 0; q < SEG; q += 4)
            *reinterpret_cast<float4*>(ep.out + o2 + q) =
                make_float4(v[SEG - 1 - q], v[SEG - 2 - q], v[SEG - 3 - q], v[SEG - 4 - q]);
        }
      } else if (ep.mode == EPI_F32_T || ep.mode == EPI_F32) {
#pragma unroll
        for (int q = 0; q < SEG; q += 4)
          *reinterpret_cast<float4*>(ep.out + o + q) = make_float4(v[q], v[q + 1], v[q + 2], v[q + 3]);
      } else {
#pragma unroll
        for (int q = 0; q < SEG; q += 8) {
          bf8 h, l;
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            __bf16 a, b;
            split_bf16(v[q + e], a, b);
            h[e] = a;
            l[e] = b;
          }
          *reinterpret_cast<bf8*>(ep.hi + o + q) = h;
          *reinterpret_cast<bf8*>(ep.lo + o + q) = l;
        }
      }
    };
    put(T1, n0 + c);
    if (dual) put(T2, ep.n - 1 - (n0 + c));
    return;
  }

  // Epilogue (waves 0-3).  Lane l of a 16x16 tile holds column l%16, rows
  // 4*(l/16)+r.
  double en = 0.0;
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    if (wk != 0) break;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 16 * j + l16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = m0 + wm + 16 * i + 4 * lg + r;
        if (dual)
          epi_store_dual(ep, row, col, acc[i][j][r], dif[i][j][r], en);
        else
          epi_store(ep, row, col, acc[i][j][r], en);
      }
    }
  }
  if ((ep.mode == EPI_PSI_EY || ep.mode == EPI_DUAL_Y) && ep.en_part) {
    double* slot = ep.en_part + (size_t)lt * ep.en_slots;
    block_sum_to<false>(en, slot);
    if (t > 0 && t < ep.en_slots) slot[t] = 0.0;
  }
}

// Row sums of rho in double, and the per-row overflow pairs (overflow,
// movable area) against base and cap (cap or rho_t - min(rho_t, base)).
__global__ void __launch_bounds__(256)
    k_gemm_rowsum(const float* __restrict__ rho, int n, double* __restrict__ rowsum,
                  const float* __restrict__ base, const float* __restrict__ cap, float rho_t,
                  double* __restrict__ tau_part) {
  const int row = blockIdx.x;
  double s = 0.0, ovf = 0.0, mov = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const size_t o = (size_t)row * n + i;
    const float v = rho[o];
    s += v;
    if (tau_part) {
      const float bb = base ? base[o] : 0.0f;
      const float cc = cap ? cap[o] : fmaxf(0.0f, rho_t - fminf(rho_t, bb));
      const float mv = v - bb;
      ovf += fmaxf(0.0f, mv - cc);
      mov += mv;
    }
  }
  block_sum_to<false>(s, &rowsum[row]);
  if (tau_part) {
    block_sum_to<false>(ovf, &tau_part[2 * row]);
    block_sum_to<false>(mov, &tau_part[2 * row + 1]);
  }
}

// R = rho - mean(rho), mean from the double row sums; float32 or bf16 hi/lo.
template <bool BF16>
__global__ void __launch_bounds__(256)
    k_gemm_prep(const float* __restrict__ rho, int n, const double* __restrict__ rowsum,
                float* __restrict__ out, __bf16* __restrict__ hi, __bf16* __restrict__ lo) {
  __shared__ double red[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += rowsum[i];
  s = wave_sum(s);
  if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
  __syncthreads();
  const float mean = (float)((red[0] + red[1] + red[2] + red[3]) / ((double)n * n));
  const size_t total = (size_t)n * n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (size_t)gridDim.x * blockDim.x) {
    const float v = rho[i] - mean;
    if (BF16) {
      __bf16 h, l;
      split_bf16(v, h, l);
      hi[i] = h;
      lo[i] = l;
    } else {
      out[i] = v;
    }
  }
}

// Even/odd butterfly for the split products.  Columns (ROWS = false): for
// every row r and i < n/2, S[r][i] = v(r, i) + v(r, n-1-i) and D[r][i] =
// v(r, i) - v(r, n-1-i), [n][n/2]; rows (ROWS = true): S[r][c] = v(r, c) +
// v(n-1-r, c), D likewise, r < n/2, [n/2][n].  v = in - mean, the mean taken
// from the double row sums when rowsum is given (else 0).  float32 (s32,
// d32) or bf16 hi/lo (sh, sl, dh, dl).
template <bool BF16, bool ROWS>
__global__ void __launch_bounds__(256)
    k_gemm_bfly(const float* __restrict__ in, int n, const double* __restrict__ rowsum,
                float* __restrict__ s32, float* __restrict__ d32, __bf16* __restrict__ sh,
                __bf16* __restrict__ sl, __bf16* __restrict__ dh, __bf16* __restrict__ dl) {
  float mean = 0.0f;
  if (rowsum) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += rowsum[i];
    s = wave_sum(s);
    if ((threadIdx.x & (kWave - 1)) == 0) red[threadIdx.x / kWave] = s;
    __syncthreads();
    mean = (float)((red[0] + red[1] + red[2] + red[3]) / ((double)n * n));
  }
  const int h = n / 2;
  const size_t total = (size_t)n * h;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    float v1, v2;
    if (ROWS) {
      const size_t r = e / n, c = e % n;
      v1 = in[r * n + c];
      v2 = in[(n - 1 - r) * n + c];
    } else {
      const size_t r = e / h, i = e % h;
      v1 = in[r * n + i];
      v2 = in[r * n + (n - 1 - i)];
    }
    v1 -= mean;
    v2 -= mean;
    const float sv = v1 + v2, dv = v1 - v2;
    if (BF16) {
      __bf16 a, b;
      split_bf16(sv, a, b);
      sh[e] = a;
      sl[e] = b;
      split_bf16(dv, a, b);
      dh[e] = a;
      dl[e] = b;
    } else {
      s32[e] = sv;
      d32[e] = dv;
    }
  }
}

// ---- host-side tables ------------------------------------------------------

uint16_t f32_to_bf16_rne(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float bf16_to_f32(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  memcpy(&f, &u, 4);
  return f;
}

// Region offsets (in bytes) inside the plan's table and workspace blocks.
struct GemmLayout {
  size_t nn;
  // float32 tables: K [n][n], KSw [n][2n], KTSwT [2n][n], and the same two
  // with the difference matrix Kd in place of Sw
  size_t t_k, t_ksw, t_ktswt, t_kkd, t_ktkdt;
  // bf16 tables (hi, lo): K [n][n], KSwT [2n][n], KTSwT [2n][n], KKdT, KTKdT
  size_t b_kh, b_kl, b_kswth, b_kswtl, b_ktswth, b_ktswtl, b_kkdth, b_kkdtl, b_ktkdth,
      b_ktkdtl;
  size_t tables_bytes;
  // workspace float32: R [n][n], W [n][n], G [n][n], UV [n][2n]
  size_t w_r, w_w, w_g, w_uv;
  // workspace bf16 (hi, lo): R, W^T, G [n][n], UV^T [2n][n]
  size_t v_rh, v_rl, v_wth, v_wtl, v_gh, v_gl, v_uvth, v_uvtl;
  size_t ws_bytes;
};

GemmLayout gemm_layout(int n) {
  GemmLayout L;
  const size_t nn = (size_t)n * n;
  L.nn = nn;
  L.t_k = 0;
  L.t_ksw = L.t_k + 4 * nn;
  L.t_ktswt = L.t_ksw + 8 * nn;
  L.t_kkd = L.t_ktswt + 8 * nn;
  L.t_ktkdt = L.t_kkd + 8 * nn;
  const size_t f32_end = L.t_ktkdt + 8 * nn;
  L.b_kh = 0;
  L.b_kl = L.b_kh + 2 * nn;
  L.b_kswth = L.b_kl + 2 * nn;
  L.b_kswtl = L.b_kswth + 4 * nn;
  L.b_ktswth = L.b_kswtl + 4 * nn;
  L.b_ktswtl = L.b_ktswth + 4 * nn;
  L.b_kkdth = L.b_ktswtl + 4 * nn;
  L.b_kkdtl = L.b_kkdth + 4 * nn;
  L.b_ktkdth = L.b_kkdtl + 4 * nn;
  L.b_ktkdtl = L.b_ktkdth + 4 * nn;
  const size_t bf_end = L.b_ktkdtl + 4 * nn;
  L.tables_bytes = f32_end > bf_end ? f32_end : bf_end;
  L.w_r = 0;
  L.w_w = 4 * nn;
  L.w_g = 8 * nn;
  L.w_uv = 12 * nn;
  const size_t wf_end = 20 * nn;
  L.v_rh = 0;
  L.v_rl = 2 * nn;
  L.v_wth = 4 * nn;
  L.v_wtl = 6 * nn;
  L.v_gh = 8 * nn;
  L.v_gl = 10 * nn;
  L.v_uvth = 12 * nn;
  L.v_uvtl = 16 * nn;
  const size_t wb_end = 20 * nn;
  L.ws_bytes = wf_end > wb_end ? wf_end : wb_end;
  return L;
}

// The even/odd split of the products (n a multiple of 128, fields rather
// than differences).  With h = n/2, the cosine rows of even and odd
// frequency restricted to the first h samples, Ke[a][i] = K[2a][i] and
// Ko[a][i] = K[2a+1][i] (K[u][n-1-i] = (-1)^u K[u][i]), and the same for Sw
// (Sw[u][n-1-i] = (-1)^(u+1) Sw[u][i]), turn every n-point transform into two
// h-point products and a butterfly: half the multiply-adds and operand bytes.
// Frequencies are kept in the order (even | odd) between the steps.
//   W'  = [Sx Ke^T | Dx Ko^T]       Sx, Dx = R left half +/- mirrored right half
//   G'  = scale([Ke Sy ; Ko Dy])    Sy, Dy = W' top half +/- mirrored bottom half
//   U'  = G'_e Ke + G'_o Ko | mirror(G'_e Ke - G'_o Ko)      (columns)
//   V'  = G'_e Swe + G'_o Swo | mirror(G'_o Swo - G'_e Swe)
//   psi = Ke^T U'_e + Ko^T U'_o ; mirror(Ke^T U'_e - Ko^T U'_o)   (rows)
//   Ey  = Swe^T U'_e + Swo^T U'_o ; mirror(Swo^T U'_o - Swe^T U'_e)
//   Ex  = Ke^T V'_e + Ko^T V'_o ; mirror(Ke^T V'_e - Ko^T V'_o)
// (_e, _o: the first and second h frequency rows or columns).  Each pair of
// half products sharing an output runs as one dual product (GemmArgs).
bool gemm_split(int n) { return n % 128 == 0; }

struct SplitLayout {
  size_t hh, nh;
  // tables after the dense ones, h x h each; float32: Ke, Ko, Swe, Swo and
  // their transposes; bf16 (hi, then lo at + 2 hh bytes): Ke, Ko, KeT, KoT,
  // SweT, SwoT
  size_t t_ke, t_ko, t_ket, t_kot, t_swe, t_swo, t_swet, t_swot;
  size_t b_ke, b_ko, b_ket, b_kot, b_swet, b_swot;
  size_t tables_bytes;
  // workspace; float32: Sx, Dx [n][h], W' [n][n], Sy, Dy [h][n], G', U', V'
  // [n][n]; bf16 (hi, then lo at + half the region): Sx, Dx [n][h], W'^T
  // float32 [n][n], Sy^T, Dy^T [n][h], G' [n][n], [U' | V']^T [2n][n]
  size_t w_sx, w_dx, w_w, w_sy, w_dy, w_g, w_u, w_v;
  size_t v_sx, v_dx, v_wt, v_syt, v_dyt, v_g, v_uvt;
  size_t ws_bytes;
};

SplitLayout split_layout(int n) {
  SplitLayout S;
  const size_t h = (size_t)n / 2, nn = (size_t)n * n;
  S.hh = h * h;
  S.nh = (size_t)n * h;
  const size_t t4 = 4 * S.hh;   // one float32 table, or one bf16 hi/lo pair
  S.t_ke = 0;
  S.t_ko = t4;
  S.t_ket = 2 * t4;
  S.t_kot = 3 * t4;
  S.t_swe = 4 * t4;
  S.t_swo = 5 * t4;
  S.t_swet = 6 * t4;
  S.t_swot = 7 * t4;
  S.b_ke = 0;
  S.b_ko = t4;
  S.b_ket = 2 * t4;
  S.b_kot = 3 * t4;
  S.b_swet = 4 * t4;
  S.b_swot = 5 * t4;
  S.tables_bytes = 8 * t4;
  S.w_sx = 0;
  S.w_dx = 2 * nn;
  S.w_w = 4 * nn;
  S.w_sy = 8 * nn;
  S.w_dy = 10 * nn;
  S.w_g = 12 * nn;
  S.w_u = 16 * nn;
  S.w_v = 20 * nn;
  S.v_sx = 0;
  S.v_dx = 2 * nn;
  S.v_wt = 4 * nn;
  S.v_syt = 8 * nn;
  S.v_dyt = 10 * nn;
  S.v_g = 12 * nn;
  S.v_uvt = 16 * nn;
  S.ws_bytes = 24 * nn;
  return S;
}

// One launch over gb.count products of one shape (grid.y = product).  Dual
// products take the 512-thread form (two K halves); otherwise it is used
// when the launch has one block per CU or fewer, so that each CU runs twice
// the waves.
template <bool BF16>
hipError_t launch_gemm(const GemmBatch& gb, hipStream_t s) {
  const GemmArgs& g = gb.g[0];
  const int tiles = (g.M / TM) * (g.N / TN);
  const dim3 grid(tiles, gb.count);
  if (g.dual || tiles * gb.count <= 256)
    hipLaunchKernelGGL((k_gemm<BF16, 2>), grid, dim3(512), 0, s, gb);
  else
    hipLaunchKernelGGL((k_gemm<BF16, 1>), grid, dim3(256), 0, s, gb);
  return hipGetLastError();
}

template <bool BF16>
hipError_t launch_gemm(const GemmArgs& g, const Epi& ep, hipStream_t s) {
  GemmBatch gb;
  gb.count = 1;
  gb.g[0] = g;
  gb.ep[0] = ep;
  return launch_gemm<BF16>(gb, s);
}

// The solve through the split products (after k_gemm_rowsum).
template <bool BF16>
hipError_t run_gemm_split(Plan& p, const SpectralArgs& a, hipStream_t s) {
  const int n = p.n, h = n / 2;
  const GemmLayout L = gemm_layout(n);
  const SplitLayout S = split_layout(n);
  const size_t nn = (size_t)n * n, nh = S.nh;
  char* tb = static_cast<char*>(p.gemm_tables) + L.tables_bytes;
  char* wb = static_cast<char*>(p.gemm_ws);
  auto f32 = [&](size_t off) { return reinterpret_cast<float*>(wb + off); };
  auto bfw = [&](size_t off) { return reinterpret_cast<__bf16*>(wb + off); };
  auto bft = [&](size_t off) { return reinterpret_cast<const __bf16*>(tb + off); };
  auto ft = [&](size_t off) { return reinterpret_cast<const float*>(tb + off); };
  int pblocks = (int)((nh + 1023) / 1024);
  if (pblocks > 4096) pblocks = 4096;
  // Sx, Dx from R = rho - mean
  if (BF16)
    hipLaunchKernelGGL((k_gemm_bfly<true, false>), dim3(pblocks), dim3(256), 0, s, a.rho, n,
                       p.rowsum, nullptr, nullptr, bfw(S.v_sx), bfw(S.v_sx) + nh, bfw(S.v_dx),
                       bfw(S.v_dx) + nh);
  else
    hipLaunchKernelGGL((k_gemm_bfly<false, false>), dim3(pblocks), dim3(256), 0, s, a.rho, n,
                       p.rowsum, f32(S.w_sx), f32(S.w_dx), nullptr, nullptr, nullptr, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  plan_mark(p, "k_gemm_prep", s);

  // 1. W' = [Sx Ke^T | Dx Ko^T]   (bf16: stored transposed in float32)
  GemmBatch gb;
  gb.count = 2;
  for (int q = 0; q < 2; ++q) {
    GemmArgs& g = gb.g[q];
    Epi& ep = gb.ep[q];
    ep.n = n;
    g.M = n; g.N = h; g.K = h;
    g.lda = h;
    g.ldb = h;
    if (BF16) {
      const size_t ax = q ? S.v_dx : S.v_sx, bx = q ? S.b_ko : S.b_ke;
      g.a_hi = bfw(ax); g.a_lo = bfw(ax) + nh;
      g.b_hi = bft(bx); g.b_lo = bft(bx) + S.hh;
      ep.mode = EPI_F32_T;
      ep.out = f32(S.v_wt) + (size_t)q * h * n;
    } else {
      g.a_hi = f32(q ? S.w_dx : S.w_sx);
      g.b_hi = ft(q ? S.t_kot : S.t_ket);
      ep.mode = EPI_F32;
      ep.out = f32(S.w_w) + (size_t)q * h;
    }
    ep.ldo = n;
  }
  if ((e = launch_gemm<BF16>(gb, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_w", s);
  // Sy, Dy: the butterfly along y of W'
  if (BF16)
    hipLaunchKernelGGL((k_gemm_bfly<true, false>), dim3(pblocks), dim3(256), 0, s,
                       f32(S.v_wt), n, nullptr, nullptr, nullptr, bfw(S.v_syt),
                       bfw(S.v_syt) + nh, bfw(S.v_dyt), bfw(S.v_dyt) + nh);
  else
    hipLaunchKernelGGL((k_gemm_bfly<false, true>), dim3(pblocks), dim3(256), 0, s,
                       f32(S.w_w), n, nullptr, f32(S.w_sy), f32(S.w_dy), nullptr, nullptr,
                       nullptr, nullptr);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  plan_mark(p, "k_gemm_bfly", s);
  // 2. G' = scale([Ke Sy ; Ko Dy])
  gb = GemmBatch();
  gb.count = 2;
  for (int q = 0; q < 2; ++q) {
    GemmArgs& g = gb.g[q];
    Epi& ep = gb.ep[q];
    ep.n = n;
    ep.wf = p.wfreq;
    ep.spectral = 2;
    ep.vpar = q;
    ep.eps = a.eps;
    g.M = h; g.N = n; g.K = h;
    g.lda = h;
    if (BF16) {
      const size_t ax = q ? S.b_ko : S.b_ke, bx = q ? S.v_dyt : S.v_syt;
      g.a_hi = bft(ax); g.a_lo = bft(ax) + S.hh;
      g.b_hi = bfw(bx); g.b_lo = bfw(bx) + nh; g.ldb = h;
      ep.mode = EPI_SPLIT;
      ep.hi = bfw(S.v_g) + (size_t)q * h * n;
      ep.lo = bfw(S.v_g) + nn + (size_t)q * h * n;
    } else {
      g.a_hi = ft(q ? S.t_ko : S.t_ke);
      g.b_hi = f32(q ? S.w_dy : S.w_sy); g.ldb = n;
      ep.mode = EPI_F32;
      ep.out = f32(S.w_g) + (size_t)q * h * n;
    }
    ep.ldo = n;
  }
  if ((e = launch_gemm<BF16>(gb, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_g", s);
  // 3. U' (q = 0) and V' (q = 1) along x, dual: even frequencies times the
  // even rows of the table, odd times odd
  gb = GemmBatch();
  gb.count = 2;
  for (int q = 0; q < 2; ++q) {
    GemmArgs& g = gb.g[q];
    Epi& ep = gb.ep[q];
    ep.n = n;
    ep.mode = EPI_DUAL_X;
    ep.dsign = q ? -1.0f : 1.0f;
    g.M = n; g.N = h; g.K = h;
    g.dual = 1;
    g.lda = n;
    g.ldb = h;
    if (BF16) {
      const size_t b1 = q ? S.b_swet : S.b_ket, b2 = q ? S.b_swot : S.b_kot;
      g.a_hi = bfw(S.v_g); g.a_lo = bfw(S.v_g) + nn;
      g.a2_hi = bfw(S.v_g) + h; g.a2_lo = bfw(S.v_g) + nn + h;
      g.b_hi = bft(b1); g.b_lo = bft(b1) + S.hh;
      g.b2_hi = bft(b2); g.b2_lo = bft(b2) + S.hh;
      ep.hi = bfw(S.v_uvt) + (size_t)q * nn;
      ep.lo = bfw(S.v_uvt) + 2 * nn + (size_t)q * nn;
    } else {
      g.a_hi = f32(S.w_g);
      g.a2_hi = f32(S.w_g) + h;
      g.b_hi = ft(q ? S.t_swe : S.t_ke);
      g.b2_hi = ft(q ? S.t_swo : S.t_ko);
      ep.out = f32(q ? S.w_v : S.w_u);
    }
    ep.ldo = n;
  }
  if ((e = launch_gemm<BF16>(gb, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_uv", s);
  // 4. psi (q = 0), Ey (q = 1), Ex (q = 2) along y, dual; energy partials
  // from the psi blocks
  gb = GemmBatch();
  gb.count = 3;
  for (int q = 0; q < 3; ++q) {
    GemmArgs& g = gb.g[q];
    Epi& ep = gb.ep[q];
    ep.n = n;
    ep.mode = EPI_DUAL_Y;
    ep.dsign = q == 1 ? -1.0f : 1.0f;
    ep.f = q == 0 ? a.psi : q == 1 ? a.ey : a.ex;
    ep.exy = q ? a.exy : nullptr;
    ep.exy_off = q == 1 ? 1 : 0;
    if (q == 0) {
      ep.rho = a.en_part ? a.rho : nullptr;
      ep.en_part = a.en_part;
      ep.en_slots = 4;   // (h/64)(n/64) blocks fill the 2 (n/64)^2 partials
    }
    g.M = h; g.N = n; g.K = h;
    g.dual = 1;
    g.lda = h;
    g.ldb = n;
    if (BF16) {
      const size_t a1 = q == 1 ? S.b_swet : S.b_ket, a2 = q == 1 ? S.b_swot : S.b_kot;
      const __bf16* bh = bfw(S.v_uvt) + (q == 2 ? nn : 0);
      const __bf16* bl = bfw(S.v_uvt) + 2 * nn + (q == 2 ? nn : 0);
      g.a_hi = bft(a1); g.a_lo = bft(a1) + S.hh;
      g.a2_hi = bft(a2); g.a2_lo = bft(a2) + S.hh;
      g.b_hi = bh; g.b_lo = bl;
      g.b2_hi = bh + h; g.b2_lo = bl + h;
    } else {
      const float* b = f32(q == 2 ? S.w_v : S.w_u);
      g.a_hi = ft(q == 1 ? S.t_swet : S.t_ket);
      g.a2_hi = ft(q == 1 ? S.t_swot : S.t_kot);
      g.b_hi = b;
      g.b2_hi = b + (size_t)h * n;
    }
  }
  if ((e = launch_gemm<BF16>(gb, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_psi_ey", s);
  return hipSuccess;
}

template <bool BF16>
hipError_t run_gemm_path(Plan& p, const SpectralArgs& a, hipStream_t s) {
  const int n = p.n;
  const GemmLayout L = gemm_layout(n);
  char* tb = static_cast<char*>(p.gemm_tables);
  char* wb = static_cast<char*>(p.gemm_ws);
  double* tau_part = a.tau_part;
  hipLaunchKernelGGL(k_gemm_rowsum, dim3(n), dim3(256), 0, s, a.rho, n, p.rowsum, a.base,
                     a.cap, a.rho_t, tau_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  plan_mark(p, "k_gemm_rowsum", s);
  if (gemm_split(n) && !a.diff) return run_gemm_split<BF16>(p, a, s);
  int pblocks = (int)((L.nn + 1023) / 1024);
  if (pblocks > 4096) pblocks = 4096;
  if (BF16) {
    hipLaunchKernelGGL(k_gemm_prep<true>, dim3(pblocks), dim3(256), 0, s, a.rho, n, p.rowsum,
                       nullptr, reinterpret_cast<__bf16*>(wb + L.v_rh),
                       reinterpret_cast<__bf16*>(wb + L.v_rl));
  } else {
    hipLaunchKernelGGL(k_gemm_prep<false>, dim3(pblocks), dim3(256), 0, s, a.rho, n,
                       p.rowsum, reinterpret_cast<float*>(wb + L.w_r), nullptr, nullptr);
  }
  if ((e = hipGetLastError()) != hipSuccess) return e;
  plan_mark(p, "k_gemm_prep", s);

  GemmArgs g;
  Epi ep;
  ep.n = n;
  ep.wf = p.wfreq;
  // 1. W = R K^T            (fp32: B = K^T [ix][u];   bf16: B^T = K [u][ix])
  g.M = n; g.N = n; g.K = n;
  if (BF16) {
    g.a_hi = wb + L.v_rh; g.a_lo = wb + L.v_rl; g.lda = n;
    g.b_hi = tb + L.b_kh; g.b_lo = tb + L.b_kl; g.ldb = n;
    ep.mode = EPI_SPLIT_T;   // stored as W^T [u][iy]: the B^T of the next product
    ep.hi = reinterpret_cast<__bf16*>(wb + L.v_wth);
    ep.lo = reinterpret_cast<__bf16*>(wb + L.v_wtl);
    ep.ldo = n;
  } else {
    g.a_hi = wb + L.w_r; g.lda = n;
    g.b_hi = tb + L.t_ktswt; g.ldb = n;   // K^T = first n rows of [K^T ; Sw^T]
    ep.mode = EPI_F32;
    ep.out = reinterpret_cast<float*>(wb + L.w_w);
    ep.ldo = n;
  }
  if ((e = launch_gemm<BF16>(g, ep, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_w", s);
  // 2. G = scale(K W)
  ep = Epi();
  ep.n = n;
  ep.wf = p.wfreq;
  ep.spectral = 1;
  ep.eps = a.eps;
  if (BF16) {
    g.a_hi = tb + L.b_kh; g.a_lo = tb + L.b_kl; g.lda = n;
    g.b_hi = wb + L.v_wth; g.b_lo = wb + L.v_wtl; g.ldb = n;
    ep.mode = EPI_SPLIT;
    ep.hi = reinterpret_cast<__bf16*>(wb + L.v_gh);
    ep.lo = reinterpret_cast<__bf16*>(wb + L.v_gl);
    ep.ldo = n;
  } else {
    g.a_hi = tb + L.t_k; g.lda = n;
    g.b_hi = wb + L.w_w; g.ldb = n;
    ep.mode = EPI_F32;
    ep.out = reinterpret_cast<float*>(wb + L.w_g);
    ep.ldo = n;
  }
  if ((e = launch_gemm<BF16>(g, ep, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_g", s);
  // 3. [U | V] = G [K | Sw]   (bf16: stored transposed, [2n][n])
  ep = Epi();
  ep.n = n;
  g.M = n; g.N = 2 * n; g.K = n;
  if (BF16) {
    g.a_hi = wb + L.v_gh; g.a_lo = wb + L.v_gl; g.lda = n;
    g.b_hi = tb + (a.diff ? L.b_kkdth : L.b_kswth);
    g.b_lo = tb + (a.diff ? L.b_kkdtl : L.b_kswtl);
    g.ldb = n;
    ep.mode = EPI_SPLIT_T;
    ep.hi = reinterpret_cast<__bf16*>(wb + L.v_uvth);
    ep.lo = reinterpret_cast<__bf16*>(wb + L.v_uvtl);
    ep.ldo = n;
  } else {
    g.a_hi = wb + L.w_g; g.lda = n;
    g.b_hi = tb + (a.diff ? L.t_kkd : L.t_ksw); g.ldb = 2 * n;
    ep.mode = EPI_F32;
    ep.out = reinterpret_cast<float*>(wb + L.w_uv);
    ep.ldo = 2 * n;
  }
  if ((e = launch_gemm<BF16>(g, ep, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_uv", s);
  // 4. [psi ; Ey] = [K^T ; Sw^T] U   (+ energy partials)
  ep = Epi();
  ep.n = n;
  ep.mode = EPI_PSI_EY;
  ep.psi = a.psi;
  ep.ey = a.ey;
  ep.exy = a.exy;
  ep.rho = a.en_part ? a.rho : nullptr;
  ep.en_part = a.en_part;
  g.M = 2 * n; g.N = n; g.K = n;
  if (BF16) {
    g.a_hi = tb + (a.diff ? L.b_ktkdth : L.b_ktswth);
    g.a_lo = tb + (a.diff ? L.b_ktkdtl : L.b_ktswtl);
    g.lda = n;
    g.b_hi = wb + L.v_uvth; g.b_lo = wb + L.v_uvtl; g.ldb = n;
  } else {
    g.a_hi = tb + (a.diff ? L.t_ktkdt : L.t_ktswt); g.lda = n;
    g.b_hi = wb + L.w_uv; g.ldb = 2 * n;
  }
  if ((e = launch_gemm<BF16>(g, ep, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_psi_ey", s);
  // 5. Ex = K^T V
  ep = Epi();
  ep.n = n;
  ep.mode = EPI_EX;
  ep.ex = a.ex;
  ep.exy = a.exy;
  g.M = n; g.N = n; g.K = n;
  if (BF16) {
    g.a_hi = tb + L.b_ktswth; g.a_lo = tb + L.b_ktswtl; g.lda = n;
    g.b_hi = wb + L.v_uvth + 2 * L.nn; g.b_lo = wb + L.v_uvtl + 2 * L.nn; g.ldb = n;
  } else {
    g.a_hi = tb + L.t_ktswt; g.lda = n;
    g.b_hi = wb + L.w_uv + 4 * (size_t)n; g.ldb = 2 * n;
  }
  if ((e = launch_gemm<BF16>(g, ep, s)) != hipSuccess) return e;
  plan_mark(p, "k_gemm_ex", s);
  return hipSuccess;
}

}  // namespace

int gemm_plan_init(Plan& p, hipStream_t s) {
  const int n = p.n;
  const GemmLayout L = gemm_layout(n);
  const bool split = gemm_split(n);
  const SplitLayout S = split_layout(n);
  const size_t tables_bytes = L.tables_bytes + (split ? S.tables_bytes : 0);
  const size_t ws_bytes = split && S.ws_bytes > L.ws_bytes ? S.ws_bytes : L.ws_bytes;
  if (hipMalloc(&p.gemm_tables, tables_bytes) != hipSuccess ||
      hipMalloc(&p.gemm_ws, ws_bytes) != hipSuccess) {
    hipGetLastError();
    return FFTPL_E_NOMEM;
  }
  p.gemm_tables_bytes = tables_bytes;
  p.gemm_ws_bytes = ws_bytes;
  const double pi = 3.14159265358979323846;
  const size_t nn = L.nn;
  // K[u][i] and Sw[u][i] = w_u S[u][i], argument reduced as pi*((u(2i+1)) mod 4n)/(2n)
  // Kd[u][i] = cos(w_u (i + 3/2)) - cos(w_u (i + 1/2)) = -2 sin(w_u / 2) sin(w_u (i + 1)):
  // psi at the next bin centre minus psi at this one (the difference mode)
  std::vector<double> K(nn), Sw(nn), Kd(nn);
  for (int u = 0; u < n; ++u) {
    const double wu = pi * u / n;
    const double sh = sin(pi * u / (2.0 * n));
    for (int i = 0; i < n; ++i) {
      const long long r = ((long long)u * (2 * i + 1)) % (4LL * n);
      const double ang = pi * (double)r / (2.0 * n);
      K[(size_t)u * n + i] = cos(ang);
      Sw[(size_t)u * n + i] = wu * sin(ang);
      const long long r2 = ((long long)u * (i + 1)) % (2LL * n);
      Kd[(size_t)u * n + i] = -2.0 * sh * sin(pi * (double)r2 / n);
    }
  }
  std::vector<char> host(tables_bytes);
  if (p.mode == FFTPL_DCT_GEMM_F32) {
    float* tk = reinterpret_cast<float*>(host.data() + L.t_k);
    float* tksw = reinterpret_cast<float*>(host.data() + L.t_ksw);
    float* tkt = reinterpret_cast<float*>(host.data() + L.t_ktswt);
    float* tkkd = reinterpret_cast<float*>(host.data() + L.t_kkd);
    float* tktkd = reinterpret_cast<float*>(host.data() + L.t_ktkdt);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        tk[(size_t)a * n + b] = (float)K[(size_t)a * n + b];
        tksw[(size_t)a * 2 * n + b] = (float)K[(size_t)a * n + b];          // [u][ix]
        tksw[(size_t)a * 2 * n + n + b] = (float)Sw[(size_t)a * n + b];
        tkt[(size_t)a * n + b] = (float)K[(size_t)b * n + a];               // [iy][v]
        tkt[(size_t)(n + a) * n + b] = (float)Sw[(size_t)b * n + a];
        tkkd[(size_t)a * 2 * n + b] = (float)K[(size_t)a * n + b];
        tkkd[(size_t)a * 2 * n + n + b] = (float)Kd[(size_t)a * n + b];
        tktkd[(size_t)a * n + b] = (float)K[(size_t)b * n + a];
        tktkd[(size_t)(n + a) * n + b] = (float)Kd[(size_t)b * n + a];
      }
  } else {
    uint16_t* kh = reinterpret_cast<uint16_t*>(host.data() + L.b_kh);
    uint16_t* kl = reinterpret_cast<uint16_t*>(host.data() + L.b_kl);
    uint16_t* sh = reinterpret_cast<uint16_t*>(host.data() + L.b_kswth);
    uint16_t* sl = reinterpret_cast<uint16_t*>(host.data() + L.b_kswtl);
    uint16_t* th = reinterpret_cast<uint16_t*>(host.data() + L.b_ktswth);
    uint16_t* tl = reinterpret_cast<uint16_t*>(host.data() + L.b_ktswtl);
    uint16_t* dh = reinterpret_cast<uint16_t*>(host.data() + L.b_kkdth);
    uint16_t* dl = reinterpret_cast<uint16_t*>(host.data() + L.b_kkdtl);
    uint16_t* eh = reinterpret_cast<uint16_t*>(host.data() + L.b_ktkdth);
    uint16_t* el = reinterpret_cast<uint16_t*>(host.data() + L.b_ktkdtl);
    auto split = [](double v, uint16_t& h, uint16_t& l) {
      const float f = (float)v;
      h = f32_to_bf16_rne(f);
      l = f32_to_bf16_rne(f - bf16_to_f32(h));
    };
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        split(K[(size_t)a * n + b], kh[(size_t)a * n + b], kl[(size_t)a * n + b]);
        // [K | Sw]^T: row ix' (n + ix for the sine half), column u
        split(K[(size_t)b * n + a], sh[(size_t)a * n + b], sl[(size_t)a * n + b]);
        split(Sw[(size_t)b * n + a], sh[(size_t)(n + a) * n + b], sl[(size_t)(n + a) * n + b]);
        // [K^T ; Sw^T]: row iy (n + iy), column v
        split(K[(size_t)b * n + a], th[(size_t)a * n + b], tl[(size_t)a * n + b]);
        split(Sw[(size_t)b * n + a], th[(size_t)(n + a) * n + b], tl[(size_t)(n + a) * n + b]);
        // the same two with Kd in place of Sw
        dh[(size_t)a * n + b] = sh[(size_t)a * n + b];
        dl[(size_t)a * n + b] = sl[(size_t)a * n + b];
        split(Kd[(size_t)b * n + a], dh[(size_t)(n + a) * n + b], dl[(size_t)(n + a) * n + b]);
        eh[(size_t)a * n + b] = th[(size_t)a * n + b];
        el[(size_t)a * n + b] = tl[(size_t)a * n + b];
        split(Kd[(size_t)b * n + a], eh[(size_t)(n + a) * n + b], el[(size_t)(n + a) * n + b]);
      }
  }
  if (split) {
    // the split tables: rows 2a (even) and 2a + 1 (odd) of K and Sw over the
    // first h samples, and their transposes
    const int h = n / 2;
    char* st = host.data() + L.tables_bytes;
    auto kv = [&](int u, int i) { return K[(size_t)u * n + i]; };
    auto sv = [&](int u, int i) { return Sw[(size_t)u * n + i]; };
    for (int a = 0; a < h; ++a)
      for (int i = 0; i < h; ++i) {
        const size_t ai = (size_t)a * h + i, ia = (size_t)i * h + a;
        const double ke = kv(2 * a, i), ko = kv(2 * a + 1, i);
        const double se = sv(2 * a, i), so = sv(2 * a + 1, i);
        if (p.mode == FFTPL_DCT_GEMM_F32) {
          float* t = reinterpret_cast<float*>(st);
          t[S.t_ke / 4 + ai] = (float)ke;
          t[S.t_ko / 4 + ai] = (float)ko;
          t[S.t_ket / 4 + ia] = (float)ke;
          t[S.t_kot / 4 + ia] = (float)ko;
          t[S.t_swe / 4 + ai] = (float)se;
          t[S.t_swo / 4 + ai] = (float)so;
          t[S.t_swet / 4 + ia] = (float)se;
          t[S.t_swot / 4 + ia] = (float)so;
        } else {
          uint16_t* t = reinterpret_cast<uint16_t*>(st);
          auto put = [&](size_t off, size_t idx, double v) {
            const float f = (float)v;
            const uint16_t hv = f32_to_bf16_rne(f);
            t[off / 2 + idx] = hv;
            t[off / 2 + S.hh + idx] = f32_to_bf16_rne(f - bf16_to_f32(hv));
          };
          put(S.b_ke, ai, ke);
          put(S.b_ko, ai, ko);
          put(S.b_ket, ia, ke);
          put(S.b_kot, ia, ko);
          put(S.b_swet, ia, se);
          put(S.b_swot, ia, so);
        }
      }
  }
  if (hipMemcpyAsync(p.gemm_tables, host.data(), tables_bytes, hipMemcpyHostToDevice, s) !=
          hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return FFTPL_E_DEVICE;
  return FFTPL_OK;
}

void gemm_plan_free(Plan& p) {
  hipFree(p.gemm_tables);
  hipFree(p.gemm_ws);
  p.gemm_tables = nullptr;
  p.gemm_ws = nullptr;
}

hipError_t spectral_gemm(Plan& p, const SpectralArgs& a, hipStream_t s) {
  return p.mode == FFTPL_DCT_GEMM_BF16X3 ? run_gemm_path<true>(p, a, s)
                                         : run_gemm_path<false>(p, a, s);
}

}  // namespace fftpl
