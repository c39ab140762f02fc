// ms_gemm.hip -- bfloat16 GEMM on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// Two kernels. k_gemm_nt serves the network forward shape (activations
// times weights stored [out][in]): operand tiles go from memory straight
// into LDS, double-buffered, in XOR-swizzled unpadded rows, 16 x 16 MFMA
// tiles per wavefront, a tile size picked per shape. k_gemm serves every
// layout (the backward products): a workgroup of 4 wavefronts computes a
// 128 x 128 tile, each wavefront a 64 x 64 quadrant; operand tiles of 32
// along K are staged through registers into LDS as [row][k] (rows padded to
// 40 elements; K-major operands transposed on the way), the next K tile
// fetched while the current one is multiplied. Both fuse the epilogue
// (GemmEpi); float32 outputs of the forward kernel are stored
// non-temporally.
#include "ms_gemm.h"

#include <type_traits>

// tile configurations of the forward-shape kernel: BM, BN, wavefronts along
// M and N (large and small tiles)
#ifndef MS_NT0
#define MS_NT0 128, 128, 4, 4
#define MS_NT1 64, 64, 2, 4
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

constexpr int NK = 64;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
// buffer resource word 3 for raw (untyped) loads on gfx9-family chips, and
// an offset beyond any range (the load then returns zeros)
constexpr int kBufWord3 = 0x00020000;
constexpr int kBufPastEnd = 0x7FFFFFF0;
// s_waitcnt immediate: vector memory count 0, the other counters unconstrained
constexpr int kWaitVm0 = (7 << 4) | (15 << 8);

// buffer resource over `bytes` bytes from p (the same in every lane: made
// from scalar copies, so the loads take it from scalar registers)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_rsrc(const bf16 *p, int bytes) {
  const unsigned long long a = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
  void *u = reinterpret_cast<void *>(((unsigned long long)hi << 32) | lo);
  return __builtin_amdgcn_make_buffer_rsrc(u, 0, __builtin_amdgcn_readfirstlane(bytes), kBufWord3);
}

// Epilogue of a wavefront's TM x TN grid of 16 x 16 MFMA tiles whose first
// row and column are mw, nw (see GemmEpi). float32 outputs are stored
// non-temporally when NTS: they stream past the L2, which keeps the operand
// tiles the workgroups still read.
template <int TM, int TN, bool NTS = true>
__device__ __forceinline__ void store_tile(const f32x4 (&acc)[TM][TN], int mw, int nw, int lane,
                                           int M, int N, const GemmEpi &epi) {
  auto put = [](float *p, float v) {
    if (NTS)
      __builtin_nontemporal_store(v, p);
    else
      *p = v;
  };
  // the per-column vectors are loaded before the first store: the outputs
  // may alias them as far as the compiler knows, so a load placed after a
  // store would wait a full memory latency per element
  float bias[TN], scl[TN], sft[TN];
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = min(nw + j * 16 + (lane & 15), N - 1);
    bias[j] = epi.bias ? epi.bias[n] : 0.f;
    scl[j] = epi.scale ? epi.scale[n] : 1.f;
    sft[j] = epi.scale ? epi.shift[n] : 0.f;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int m = mw + i * 16 + (lane >> 4) * 4 + e;
        const int n = nw + j * 16 + (lane & 15);
        if (m >= M || n >= N) continue;
        const size_t o = (size_t)m * epi.ldc + n;
        float v = acc[i][j][e] * epi.alpha;
        if (epi.bias) v += bias[j];
        if (epi.addc) v += epi.addc[o];
        if (epi.dact) v *= silu_slope(epi.dact[o]);
        if (epi.z_out) put(&epi.z_out[o], v);
        if (epi.act == 1) v = silu(v);
        if (epi.act == 2) v = 1.0f / (1.0f + expf(-v));
        if (epi.scale) v = v * scl[j] + sft[j];
        if (epi.c2 && n >= epi.split)
          put(&epi.c2[(size_t)m * epi.ldc2 + (n - epi.split)], v);
        else if (epi.c_f32)
          put(&epi.c_f32[o], v);
        if (epi.c_bf16) epi.c_bf16[o] = __float2bfloat16(v);
      }
}

// The forward shape, C = A B^T with A [M][K] and B [N][K] both row-major
// (activations times a weight matrix stored [out][in]): a BM x BN tile per
// workgroup of WM x WN wavefronts (each BM/WM x BN/WN as 16 x 16 MFMA tiles),
// K in steps of 64. The operand tiles are copied from memory straight into
// LDS (buffer loads with the LDS bit, no staging registers), double-buffered,
// one barrier per step. Tiles are unpadded 128-byte
// rows; chunk q (8 k values) of row r sits in slot q ^ g(r),
// g(r) = (r & 7) ^ ((r >> 3) & 1), so the 16 rows an MFMA operand read
// touches fall in distinct bank groups. Out-of-range rows and K chunks read
// as zeros.
template <int BMt, int BNt, int WM, int WN>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt(int M, int N, int K, const bf16 *A,
                                                             int lda, const bf16 *B, int ldb,
                                                             GemmEpi epi) {
  constexpr int NT = 64 * WM * WN;
  constexpr int TM = BMt / WM / 16, TN = BNt / WN / 16;
  constexpr int CA = BMt * 8 / NT, CB = BNt * 8 / NT;     // chunks per thread and step
  static_assert(CA >= 1 && CB >= 1 && TM >= 1 && TN >= 1, "bad configuration");
  __shared__ __align__(16) unsigned short As[2][BMt * NK];
  __shared__ __align__(16) unsigned short Bs[2][BNt * NK];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int wm = w / WN, wn = w % WN;
  // workgroups are handed to the 8 XCDs round-robin by linear id; renumber
  // them so that each XCD takes one contiguous run of tiles, row-major over
  // N (consecutive tiles share their A rows, and B stays in that XCD's L2)
  int m0, n0;
  {
    const int nt = gridDim.x * gridDim.y, id = blockIdx.y * gridDim.x + blockIdx.x;
    const int q = nt / 8, rm = nt % 8, x = id % 8, slot = id / 8;
    const int t = (x < rm ? x * (q + 1) : rm * (q + 1) + (x - rm) * q) + slot;
    m0 = (t / gridDim.x) * BMt;
    n0 = (t % gridDim.x) * BNt;
  }
  const __amdgpu_buffer_rsrc_t rsa =
      tile_rsrc(A + (size_t)m0 * lda, 2 * lda * max(0, min(BMt, M - m0)));
  const __amdgpu_buffer_rsrc_t rsb =
      tile_rsrc(B + (size_t)n0 * ldb, 2 * ldb * max(0, min(BNt, N - n0)));
  auto swz = [](int r) { return (r & 7) ^ ((r >> 3) & 1); };
  // step kt's tiles into stage buffer st: chunk c = tid + NT it is row
  // c >> 3, slot c & 7 (the wavefront's 64 chunks are 1 KB of LDS)
  auto copy = [&](int st, int kt) {
    const int k0 = kt * NK;
#pragma unroll
    for (int it = 0; it < CA; ++it) {
      const int c = tid + NT * it, row = c >> 3, gk = k0 + (((c & 7) ^ swz(row)) * 8);
      const int off = gk < K ? 2 * (row * lda + gk) : kBufPastEnd;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsa, (__attribute__((address_space(3))) void *)&As[st][(c - lane) * 8], 16, off, 0, 0, 0);
    }
#pragma unroll
    for (int it = 0; it < CB; ++it) {
      const int c = tid + NT * it, row = c >> 3, gk = k0 + (((c & 7) ^ swz(row)) * 8);
      const int off = gk < K ? 2 * (row * ldb + gk) : kBufPastEnd;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rsb, (__attribute__((address_space(3))) void *)&Bs[st][(c - lane) * 8], 16, off, 0, 0, 0);
    }
  };
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int r16 = lane & 15, kq = lane >> 4;
  // a step's operands, both 32-wide K halves, read from LDS at once
  bf16x8 a[NK / 32][TM], b[NK / 32][TN];
  auto read = [&](int st) {
#pragma unroll
    for (int s = 0; s < NK / 32; ++s) {
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int row = wm * (BMt / WM) + i * 16 + r16;
        a[s][i] = *reinterpret_cast<const bf16x8 *>(&As[st][row * NK + (((s * 4 + kq) ^ swz(row)) * 8)]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int row = wn * (BNt / WN) + j * 16 + r16;
        b[s][j] = *reinterpret_cast<const bf16x8 *>(&Bs[st][row * NK + (((s * 4 + kq) ^ swz(row)) * 8)]);
      }
    }
  };
  auto mfma = [&] {
#pragma unroll
    for (int s = 0; s < NK / 32; ++s)
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[s][i], b[s][j], acc[i][j], 0, 0, 0);
  };
  const int nk = (K + NK - 1) / NK;
  // Two stage buffers: step kt's operands are read into registers, then the
  // copy of step kt + 1 into the other buffer is issued, then the MFMAs run
  // while it travels. (An LDS read waits for every copy still in flight, so
  // deeper pipelines would gain nothing.)
  copy(0, 0);
  int st = 0;
  for (int kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(kWaitVm0);
    __syncthreads();   // step kt is in LDS for every wavefront, and every
                       // wavefront has read step kt - 1's buffer
    read(st);
    __builtin_amdgcn_sched_barrier(0);
    copy(st ^ 1, kt + 1);
    __builtin_amdgcn_sched_barrier(0);
    mfma();
    st ^= 1;
  }
  __builtin_amdgcn_s_waitcnt(0);     // no copy may land after the workgroup ends
  store_tile<TM, TN, true>(acc, m0 + wm * (BMt / WM), n0 + wn * (BNt / WN), lane, M, N, epi);
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

// Tile of the forward-shape kernel (measured on MI355X): 128 x 128 with 16
// wavefronts when it still gives every CU two workgroups and the epilogue
// is plain (bias, activation, one output); otherwise 64 x 64 with 8
// wavefronts, which is faster for narrow outputs and also for the
// de-standardising, column-split epilogue (the larger tile's 16-wavefront
// epilogue then doubles its time).
int gemm_nt_tile(int M, int N, const GemmEpi &epi) {
  const int cus = cu_count();
  const long long big = (long long)((M + 127) / 128) * ((N + 127) / 128);
  if (big >= 2 * cus && !epi.scale && !epi.c2) return 0;
  return 1;
}

template <int BM, int BN, int WM, int WN>
void launch_nt(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
               const GemmEpi &epi, hipStream_t st) {
  hipLaunchKernelGGL((k_gemm_nt<BM, BN, WM, WN>), dim3((N + BN - 1) / BN, (M + BM - 1) / BM),
                     dim3(64 * WM * WN), 0, st, M, N, K, A, lda, B, ldb, epi);
}

hipError_t gemm_bf16(bool ta, bool tb, int M, int N, int K, const bf16 *A, int lda, const bf16 *B,
                     int ldb, const GemmEpi &epi, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K % 8 || lda % 8 || ldb % 8 || (ta && M % 8) || (!tb && N % 8)) return hipErrorInvalidValue;
  if (!ta && tb) {
    // byte offsets within a tile's rows are 32-bit
    if (lda > (1 << 20) || ldb > (1 << 20)) return hipErrorInvalidValue;
    if (gemm_nt_tile(M, N, epi) == 0)
      launch_nt<MS_NT0>(M, N, K, A, lda, B, ldb, epi, st);
    else
      launch_nt<MS_NT1>(M, N, K, A, lda, B, ldb, epi, st);
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
