// ms_gemm.hip -- bfloat16 GEMM on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// A workgroup of 4 wavefronts computes a 128 x 128 tile of C; each
// wavefront owns a 64 x 64 quadrant as a 4 x 4 grid of 16 x 16 MFMA tiles
// with float32 accumulators. Operand tiles of 32 along K are staged through
// LDS as [row][k] (k contiguous, rows padded to 40 elements), so every lane
// reads its 8 consecutive k values of a row with one 128-bit LDS load;
// operands stored K-major in memory are transposed while being staged. The
// next K tile is fetched into registers while the current one is multiplied.
#include "ms_gemm.h"

#include <type_traits>

// tile configurations of the forward-shape kernel: BM, BN, wavefronts along
// M and N, register prefetch depth (large, medium and small tiles)
#ifndef MS_NT0
#define MS_NT0 128, 128, 4, 4, 1
#define MS_NT1 64, 128, 2, 4, 1
#define MS_NT2 64, 64, 2, 4, 1
#endif

namespace ms {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr int BM = 128, BN = 128, BK = 32, LK = BK + 8;

// A 128 (rows) x 32 (k) tile of a matrix whose element (o, k) lives at
// G[o * ld + k] (row-major, KMAJOR = false) or G[k * ld + o] (KMAJOR = true),
// in two steps so the next tile's global loads can be in flight while the
// current one is multiplied: fetch (two 128-bit global loads per thread
// into registers; out-of-range elements are zero), then store into
// S[o * LK + k] (K-major tiles transposed on the way).
template <bool KMAJOR>
__device__ __forceinline__ void fetch(uint4 v[2], const bf16 *G, int ld, int o0, int O, int k0, int K,
                                      int tid) {
  const unsigned short *g = reinterpret_cast<const unsigned short *>(G);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int c = tid + 256 * it;
    v[it] = make_uint4(0, 0, 0, 0);
    if (!KMAJOR) {
      const int o = c >> 2, kc = (c & 3) * 8;
      const int go = o0 + o, gk = k0 + kc;
      if (go < O && gk < K) v[it] = *reinterpret_cast<const uint4 *>(g + (size_t)go * ld + gk);
    } else {
      const int kk = c >> 4, oc = (c & 15) * 8;
      const int go = o0 + oc, gk = k0 + kk;
      if (go < O && gk < K) v[it] = *reinterpret_cast<const uint4 *>(g + (size_t)gk * ld + go);
    }
  }
}

template <bool KMAJOR>
__device__ __forceinline__ void store(unsigned short *S, const uint4 v[2], int tid) {
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const int c = tid + 256 * it;
    if (!KMAJOR) {
      const int o = c >> 2, kc = (c & 3) * 8;
      *reinterpret_cast<uint4 *>(S + o * LK + kc) = v[it];
    } else {
      const int kk = c >> 4, oc = (c & 15) * 8;
      const uint4 w = v[it];
      const unsigned short e[8] = {(unsigned short)(w.x & 0xFFFF), (unsigned short)(w.x >> 16),
                                   (unsigned short)(w.y & 0xFFFF), (unsigned short)(w.y >> 16),
                                   (unsigned short)(w.z & 0xFFFF), (unsigned short)(w.z >> 16),
                                   (unsigned short)(w.w & 0xFFFF), (unsigned short)(w.w >> 16)};
#pragma unroll
      for (int j = 0; j < 8; ++j) S[(oc + j) * LK + kk] = e[j];
    }
  }
}

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_slope(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
}

// K slice z = blockIdx.z covers [z k_slice, min(K, (z + 1) k_slice)) and
// writes its partial product at an offset of z z_stride floats
template <bool TA, bool TB>
__global__ __launch_bounds__(256) void k_gemm(int M, int N, int K, const bf16 *A, int lda,
                                              const bf16 *B, int ldb, GemmEpi epi, int k_slice,
                                              size_t z_stride) {
  __shared__ __align__(16) unsigned short As[BM * LK];
  __shared__ __align__(16) unsigned short Bs[BN * LK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w >> 1, wn = w & 1;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  f32x4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

  const int kb = blockIdx.z * k_slice, ke = min(K, kb + k_slice);
  uint4 ra[2], rb[2];
  if (kb < ke) {
    fetch<TA>(ra, A, lda, m0, M, kb, ke, tid);
    fetch<!TB>(rb, B, ldb, n0, N, kb, ke, tid);
  }
  for (int k0 = kb; k0 < ke; k0 += BK) {
    store<TA>(As, ra, tid);
    store<!TB>(Bs, rb, tid);
    __syncthreads();
    // the next tile's loads travel while this one is multiplied
    if (k0 + BK < ke) {
      fetch<TA>(ra, A, lda, m0, M, k0 + BK, ke, tid);
      fetch<!TB>(rb, B, ldb, n0, N, k0 + BK, ke, tid);
    }
    bf16x8 a[4], b[4];
    const int kq = (lane >> 4) * 8, r = lane & 15;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *reinterpret_cast<const bf16x8 *>(As + (wm * 64 + i * 16 + r) * LK + kq);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const bf16x8 *>(Bs + (wn * 64 + j * 16 + r) * LK + kq);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    __syncthreads();
  }

  // accumulator element e of tile (i, j): row 4*(lane/16) + e, column lane%16
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * 64 + i * 16 + (lane >> 4) * 4 + e;
        const int n = n0 + wn * 64 + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        const size_t o = (size_t)blockIdx.z * z_stride + (size_t)m * epi.ldc + n;
        float v = acc[i][j][e] * epi.alpha;
        if (epi.bias) v += epi.bias[n];
        if (epi.addc) v += epi.addc[o];
        if (epi.dact) v *= silu_slope(epi.dact[o]);
        if (epi.z_out) epi.z_out[o] = v;
        if (epi.act == 1) v = silu(v);
        if (epi.act == 2) v = 1.0f / (1.0f + expf(-v));
        if (epi.scale) v = v * epi.scale[n] + epi.shift[n];
        if (epi.c2 && n >= epi.split)
          epi.c2[(size_t)m * epi.ldc2 + (n - epi.split)] = v;
        else if (epi.c_f32)
          epi.c_f32[o] = v;
        if (epi.c_bf16) epi.c_bf16[o] = __float2bfloat16(v);
      }
}

// The forward shape, C = A B^T with A [M][K] and B [N][K] both row-major
// (activations times a weight matrix stored [out][in]): a BM x BN tile per
// workgroup of WM x WN wavefronts (each BM/WM x BN/WN as 16 x 16 MFMA tiles),
// K in steps of 64 through two LDS buffers, one barrier per step. Global
// loads run DEPTH steps ahead in registers (register sets alternate with the
// step's parity; the K loop is unrolled by two so every set index is a
// compile-time constant).
constexpr int NK = 64, NLK = NK + 8;

template <int BMt, int BNt, int WM, int WN, int DEPTH>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt(int M, int N, int K, const bf16 *A,
                                                         int lda, const bf16 *B, int ldb,
                                                         GemmEpi epi) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BMt / WM / 16, TN = BNt / WN / 16;   // MFMA tiles per wavefront
  constexpr int CA = BMt * 8 / NT, CB = BNt * 8 / NT;     // 16-byte chunks per thread and step
  static_assert(CA >= 1 && CB >= 1 && TM >= 1 && TN >= 1, "tile too small for the workgroup");
  __shared__ __align__(16) unsigned short As[2][BMt * NLK];
  __shared__ __align__(16) unsigned short Bs[2][BNt * NLK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;
  const int m0 = blockIdx.y * BMt, n0 = blockIdx.x * BNt;
  const unsigned short *ga = reinterpret_cast<const unsigned short *>(A);
  const unsigned short *gb = reinterpret_cast<const unsigned short *>(B);
  uint4 ra[DEPTH][CA], rb[DEPTH][CB];
  auto fetch = [&](uint4 (&xa)[CA], uint4 (&xb)[CB], int k0) {
#pragma unroll
    for (int it = 0; it < CA; ++it) {
      const int c = tid + NT * it, row = c >> 3, kc = (c & 7) * 8;
      const int gm = m0 + row, gk = k0 + kc;
      xa[it] = make_uint4(0, 0, 0, 0);
      if (gm < M && gk < K) xa[it] = *reinterpret_cast<const uint4 *>(ga + (size_t)gm * lda + gk);
    }
#pragma unroll
    for (int it = 0; it < CB; ++it) {
      const int c = tid + NT * it, row = c >> 3, kc = (c & 7) * 8;
      const int gn = n0 + row, gk = k0 + kc;
      xb[it] = make_uint4(0, 0, 0, 0);
      if (gn < N && gk < K) xb[it] = *reinterpret_cast<const uint4 *>(gb + (size_t)gn * ldb + gk);
    }
  };
  auto stash = [&](const uint4 (&xa)[CA], const uint4 (&xb)[CB], int buf) {
#pragma unroll
    for (int it = 0; it < CA; ++it) {
      const int c = tid + NT * it, row = c >> 3, kc = (c & 7) * 8;
      *reinterpret_cast<uint4 *>(&As[buf][row * NLK + kc]) = xa[it];
    }
#pragma unroll
    for (int it = 0; it < CB; ++it) {
      const int c = tid + NT * it, row = c >> 3, kc = (c & 7) * 8;
      *reinterpret_cast<uint4 *>(&Bs[buf][row * NLK + kc]) = xb[it];
    }
  };
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int kq = (lane >> 4) * 8, r = lane & 15;
  auto compute = [&](int buf) {
#pragma unroll
    for (int s = 0; s < NK / 32; ++s) {
      bf16x8 a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        a[i] = *reinterpret_cast<const bf16x8 *>(
            &As[buf][(wm * (BMt / WM) + i * 16 + r) * NLK + s * 32 + kq]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        b[j] = *reinterpret_cast<const bf16x8 *>(
            &Bs[buf][(wn * (BNt / WN) + j * 16 + r) * NLK + s * 32 + kq]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  };
  const int nk = (K + NK - 1) / NK;
  // step j's tile waits in register set j % DEPTH, then in LDS buffer j % 2
  fetch(ra[0], rb[0], 0);
  stash(ra[0], rb[0], 0);
  if (DEPTH == 2 && nk > 1) fetch(ra[DEPTH - 1], rb[DEPTH - 1], NK);
  __syncthreads();
  // one step kt of parity P: the load of step kt + DEPTH into set
  // (kt + DEPTH) % DEPTH, the MFMAs on buffer P, then step kt + 1's tile from
  // its register set into buffer 1 - P
  auto step = [&](int kt, auto parity) {
    constexpr int P = decltype(parity)::value;
    constexpr int SL = (P + DEPTH) % DEPTH;        // set receiving step kt + DEPTH
    constexpr int SN = (P + 1) % DEPTH;            // set holding step kt + 1
    if (kt + DEPTH < nk) fetch(ra[SL], rb[SL], (kt + DEPTH) * NK);
    compute(P);
    if (kt + 1 < nk) stash(ra[SN], rb[SN], 1 - P);
    __syncthreads();
  };
  using P0 = std::integral_constant<int, 0>;
  using P1 = std::integral_constant<int, 1>;
  if (DEPTH == 1) {
    // one register set: a plain loop over the steps
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      if (kt + 1 < nk) fetch(ra[0], rb[0], (kt + 1) * NK);
      compute(cur);
      if (kt + 1 < nk) stash(ra[0], rb[0], cur ^ 1);
      __syncthreads();
    }
  } else {
    for (int kt = 0; kt < nk; kt += 2) {
      step(kt, P0{});
      if (kt + 1 < nk) step(kt + 1, P1{});
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = m0 + wm * (BMt / WM) + i * 16 + (lane >> 4) * 4 + e;
        const int n = n0 + wn * (BNt / WN) + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        const size_t o = (size_t)m * epi.ldc + n;
        float v = acc[i][j][e] * epi.alpha;
        if (epi.bias) v += epi.bias[n];
        if (epi.addc) v += epi.addc[o];
        if (epi.dact) v *= silu_slope(epi.dact[o]);
        if (epi.z_out) epi.z_out[o] = v;
        if (epi.act == 1) v = silu(v);
        if (epi.act == 2) v = 1.0f / (1.0f + expf(-v));
        if (epi.scale) v = v * epi.scale[n] + epi.shift[n];
        if (epi.c2 && n >= epi.split)
          epi.c2[(size_t)m * epi.ldc2 + (n - epi.split)] = v;
        else if (epi.c_f32)
          epi.c_f32[o] = v;
        if (epi.c_bf16) epi.c_bf16[o] = __float2bfloat16(v);
      }
}

// C[m][n] = sum over z of work[z][m][n], slice order
__global__ void k_splitk_sum(const float *work, int S, size_t stride, int M, int N, int ldc,
                             float *C) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)M * N) return;
  const int m = (int)(t / N), n = (int)(t % N);
  const size_t o = (size_t)m * ldc + n;
  float s = 0.0f;
  for (int z = 0; z < S; ++z) s += work[z * stride + o];
  C[o] = s;
}

}  // namespace

static hipError_t gemm_launch(bool ta, bool tb, int M, int N, int K, const bf16 *A, int lda,
                              const bf16 *B, int ldb, const GemmEpi &epi, int S, int ks,
                              size_t stride, hipStream_t st) {
  dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, S), block(256);
  if (!ta && !tb)
    hipLaunchKernelGGL((k_gemm<false, false>), grid, block, 0, st, M, N, K, A, lda, B, ldb, epi, ks, stride);
  if (!ta && tb)
    hipLaunchKernelGGL((k_gemm<false, true>), grid, block, 0, st, M, N, K, A, lda, B, ldb, epi, ks, stride);
  if (ta && !tb)
    hipLaunchKernelGGL((k_gemm<true, false>), grid, block, 0, st, M, N, K, A, lda, B, ldb, epi, ks, stride);
  if (ta && tb)
    hipLaunchKernelGGL((k_gemm<true, true>), grid, block, 0, st, M, N, K, A, lda, B, ldb, epi, ks, stride);
  return hipGetLastError();
}

namespace {
int cu_count() {
  static int n = 0;
  if (!n) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n = v;
    else
      n = 256;
  }
  return n;
}
}  // namespace

int gemm_nt_tile(int M, int N) {
  const int cus = cu_count();
  auto tiles = [&](int bm, int bn) { return (long long)((M + bm - 1) / bm) * ((N + bn - 1) / bn); };
  // the largest tile that still gives every CU two workgroups
  if (tiles(128, 128) >= 2 * cus) return 0;
  if (tiles(64, 128) >= 2 * cus) return 1;
  return 2;
}

template <int BM, int BN, int WM, int WN, int D>
void launch_nt(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
               const GemmEpi &epi, hipStream_t st) {
  hipLaunchKernelGGL((k_gemm_nt<BM, BN, WM, WN, D>), dim3((N + BN - 1) / BN, (M + BM - 1) / BM),
                     dim3(64 * WM * WN), 0, st, M, N, K, A, lda, B, ldb, epi);
}

hipError_t gemm_bf16(bool ta, bool tb, int M, int N, int K, const bf16 *A, int lda, const bf16 *B,
                     int ldb, const GemmEpi &epi, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K % 8 || lda % 8 || ldb % 8 || (ta && M % 8) || (!tb && N % 8)) return hipErrorInvalidValue;
  if (!ta && tb) {
    const int t = gemm_nt_tile(M, N);
    if (t == 0)
      launch_nt<MS_NT0>(M, N, K, A, lda, B, ldb, epi, st);
    else if (t == 1)
      launch_nt<MS_NT1>(M, N, K, A, lda, B, ldb, epi, st);
    else
      launch_nt<MS_NT2>(M, N, K, A, lda, B, ldb, epi, st);
    return hipGetLastError();
  }
  return gemm_launch(ta, tb, M, N, K, A, lda, B, ldb, epi, 1, K, 0, st);
}

int splitk_slices(int M, int N, int K) {
  const int tiles = ((M + BM - 1) / BM) * ((N + BN - 1) / BN);
  int S = 1;
  // at least ~1024 workgroups, slices of at least 256 along K
  while (S < 64 && tiles * S < 1024 && K / (2 * S) >= 256) S *= 2;
  return S;
}

hipError_t gemm_bf16_splitk(bool ta, bool tb, int M, int N, int K, const bf16 *A, int lda,
                            const bf16 *B, int ldb, float *C, int ldc, float *work, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K % 8 || lda % 8 || ldb % 8 || (ta && M % 8) || (!tb && N % 8)) return hipErrorInvalidValue;
  const int S = splitk_slices(M, N, K);
  int ks = (K + S - 1) / S;
  ks = (ks + BK - 1) / BK * BK;
  GemmEpi epi;
  epi.c_f32 = work;
  epi.ldc = ldc;
  const size_t stride = (size_t)M * ldc;
  hipError_t e = gemm_launch(ta, tb, M, N, K, A, lda, B, ldb, epi, S, ks, stride, st);
  if (e != hipSuccess) return e;
  const size_t n = (size_t)M * N;
  hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, work, S,
                     stride, M, N, ldc, C);
  return hipGetLastError();
}

}  // namespace ms
