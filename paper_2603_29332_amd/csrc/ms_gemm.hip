// ms_gemm.hip -- bfloat16 GEMM on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16).
//
// One kernel, k_gemm_nt, for C = A B^T with both operands row-major along K
// (activations times weights stored [out][in]; the backward products use
// transposed weight copies and the weight gradients transposed activations,
// so every product of the networks has this shape). Operand tiles go from
// memory straight into LDS, double-buffered, in XOR-swizzled unpadded rows,
// 16 x 16 MFMA tiles per wavefront, a tile size picked per shape, the
// epilogue fused (GemmEpi), float32 outputs stored non-temporally. Long K
// with few output tiles is split into slices summed afterwards in a fixed
// order.
#include "ms_gemm.h"


// tile configurations of the kernel: BM, BN, wavefronts along M and N
#ifndef MS_NT0
#define MS_NT0 128, 128, 4, 4
#define MS_NT1 64, 64, 2, 4
#define MS_NT2 128, 64, 4, 2
#define MS_NT3 32, 64, 1, 4
#endif

namespace ms {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float silu(float z) { return z / (1.0f + expf(-z)); }
__device__ __forceinline__ float silu_slope(float z) {
  const float s = 1.0f / (1.0f + expf(-z));
  return s * (1.0f + z * (1.0f - s));
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
// as zeros. SPLIT: K is split into slices of ks; slice z = blockIdx.z takes
// columns [z ks, min(K, (z + 1) ks)) and writes its partial product to
// epi.c_f32 + z cstride (plain float32 output, summed afterwards). The
// split is a template choice so that the other instantiations keep their
// register count.
template <int BMt, int BNt, int WM, int WN, bool SPLIT = false>
__global__ __launch_bounds__(64 * WM * WN) void k_gemm_nt(int M, int N, int K, const bf16 *A,
                                                             int lda, const bf16 *B, int ldb,
                                                             GemmEpi epi, int ks, size_t cstride) {
  constexpr int NT = 64 * WM * WN;
  if (SPLIT) {
    const int kb = blockIdx.z * ks;
    A += kb;
    B += kb;
    K = max(0, min(K - kb, ks));
    epi.c_f32 += blockIdx.z * cstride;
  }
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

// XT[c][r] = X[r][c] for 16-bit X[rows][cols] (rows, cols multiples of 4):
// 64 x 64 tiles through LDS, 8-byte loads along X's rows and 8-byte stores
// along XT's rows; 256 threads.
__global__ void k_transpose16(const unsigned short *X, int rows, int cols, unsigned short *XT) {
  __shared__ unsigned short t[64][68];
  const int c0 = blockIdx.x * 64, r0 = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int r = ty + 16 * i, c = c0 + 4 * tx;
    ushort4 v = make_ushort4(0, 0, 0, 0);
    if (r0 + r < rows && c < cols) v = *reinterpret_cast<const ushort4 *>(&X[(size_t)(r0 + r) * cols + c]);
    *reinterpret_cast<ushort4 *>(&t[r][4 * tx]) = v;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = ty + 16 * i, r = 4 * tx;
    if (c0 + c < cols && r0 + r < rows)
      *reinterpret_cast<ushort4 *>(&XT[(size_t)(c0 + c) * rows + r0 + r]) =
          make_ushort4(t[r][c], t[r + 1][c], t[r + 2][c], t[r + 3][c]);
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

// Tile of a product (measured on MI355X):
// - 128 x 128 with 16 wavefronts when that gives every CU two workgroups
//   and the epilogue is plain (bias, activation, one output);
// - 128 x 64 with 8 wavefronts for long K (at least 2048) when that still
//   gives every CU two workgroups;
// - 32 x 64 with 4 wavefronts when 64 x 64 tiles would not give every CU
//   two workgroups (small batches, narrow outputs);
// - otherwise 64 x 64 with 8 wavefronts, which is also faster for the
//   de-standardising, column-split epilogue (the 16-wavefront epilogue then
//   doubles its time).
int gemm_nt_tile(int M, int N, int K, const GemmEpi &epi) {
  const int cus = cu_count();
  const long long big = (long long)((M + 127) / 128) * ((N + 127) / 128);
  const long long tall = (long long)((M + 127) / 128) * ((N + 63) / 64);
  const long long mid = (long long)((M + 63) / 64) * ((N + 63) / 64);
  if (big >= 2 * cus && !epi.scale && !epi.c2) return 0;
  if (K >= 2048 && tall >= 2 * cus) return 2;
  if (mid < 2 * cus) return 3;
  return 1;
}

template <int BM, int BN, int WM, int WN>
void launch_nt(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
               const GemmEpi &epi, hipStream_t st, int S = 1, int ks = 0, size_t cstride = 0) {
  const dim3 grid((N + BN - 1) / BN, (M + BM - 1) / BM, S), block(64 * WM * WN);
  if (S > 1)
    hipLaunchKernelGGL((k_gemm_nt<BM, BN, WM, WN, true>), grid, block, 0, st, M, N, K, A, lda, B,
                       ldb, epi, ks, cstride);
  else
    hipLaunchKernelGGL((k_gemm_nt<BM, BN, WM, WN, false>), grid, block, 0, st, M, N, K, A, lda, B,
                       ldb, epi, K, (size_t)0);
}

hipError_t transpose_bf16(const bf16 *X, int rows, int cols, bf16 *XT, hipStream_t st) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  if (rows % 4 || cols % 4 || rows / 64 >= 65536) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_transpose16, dim3((cols + 63) / 64, (rows + 63) / 64), dim3(256), 0, st,
                     reinterpret_cast<const unsigned short *>(X), rows, cols,
                     reinterpret_cast<unsigned short *>(XT));
  return hipGetLastError();
}

hipError_t gemm_bf16(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
                     const GemmEpi &epi, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K % 8 || lda % 8 || ldb % 8) return hipErrorInvalidValue;
  // byte offsets within a tile's rows are 32-bit
  if (lda > (1 << 20) || ldb > (1 << 20)) return hipErrorInvalidValue;
  switch (gemm_nt_tile(M, N, K, epi)) {
    case 0: launch_nt<MS_NT0>(M, N, K, A, lda, B, ldb, epi, st); break;
    case 2: launch_nt<MS_NT2>(M, N, K, A, lda, B, ldb, epi, st); break;
    case 3: launch_nt<MS_NT3>(M, N, K, A, lda, B, ldb, epi, st); break;
    default: launch_nt<MS_NT1>(M, N, K, A, lda, B, ldb, epi, st);
  }
  return hipGetLastError();
}

// Split-K tile: 128 x 64 with 8 wavefronts when the output has at least 128
// of them, else 64 x 64.
static bool splitk_tall(int M, int N) {
  return (long long)((M + 127) / 128) * ((N + 63) / 64) >= 128;
}

int splitk_slices(int M, int N, int K) {
  // about two workgroups per CU, slices of at least 512 along K (8 of the
  // kernel's K steps)
  const long long tiles = splitk_tall(M, N) ? (long long)((M + 127) / 128) * ((N + 63) / 64)
                                            : (long long)((M + 63) / 64) * ((N + 63) / 64);
  int S = 1;
  while (S < 32 && tiles * S < 2 * cu_count() && K / (2 * S) >= 512) S *= 2;
  return S;
}

hipError_t gemm_bf16_splitk(int M, int N, int K, const bf16 *A, int lda, const bf16 *B, int ldb,
                            float *C, int ldc, float *work, hipStream_t st) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K % 8 || lda % 8 || ldb % 8) return hipErrorInvalidValue;
  if (lda > (1 << 20) || ldb > (1 << 20)) return hipErrorInvalidValue;
  const int S = splitk_slices(M, N, K);
  const int ks = ((K + S - 1) / S + NK - 1) / NK * NK;
  GemmEpi epi;
  epi.c_f32 = S > 1 ? work : C;
  epi.ldc = ldc;
  const size_t stride = (size_t)M * ldc;
  if (splitk_tall(M, N))
    launch_nt<MS_NT2>(M, N, K, A, lda, B, ldb, epi, st, S, ks, stride);
  else
    launch_nt<MS_NT1>(M, N, K, A, lda, B, ldb, epi, st, S, ks, stride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || S == 1) return e;
  const size_t n = (size_t)M * N;
  hipLaunchKernelGGL(k_splitk_sum, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, work, S,
                     stride, M, N, ldc, C);
  return hipGetLastError();
}

}  // namespace ms
