// ms_mlp.hip -- the learned muscle-geometry surrogate: a pose -> (muscle
// lengths, moment arms) multilayer perceptron trained and evaluated with the
// library's own bfloat16 matrix-core kernels (ms_gemm.hip).
//
// Network: x (hinge angles mapped from their pose box onto [-1, 1], padded
// to a multiple of 16) -> SiLU(W1 x + b1)
// -> SiLU(W2 h1 + b2) -> W3 h2 + b3, standardised outputs. Output layout per
// pose: [L (n_mus) | r (n_mus x 3, the model's span slots)], caller's
// muscle order. Weights live as float32 masters ([out][in]) with bfloat16
// copies for the GEMMs ([out][in] for the forward, [in][out] for the input
// gradients of the backward pass); Adam (Kingma & Ba 2015) updates the
// masters and refreshes both copies.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ms.h"
#include "ms_gemm.h"
#include "ms_model.h"
#include "ms_step_types.h"

// Tables of the model this surrogate serves (filled from the model).
struct ms_surrogate {
  int n_in = 0, h1 = 0, h2 = 0, n_out = 0, n_mus = 0, nq = 0, free_root = 0;
  // device buffers
  float *W[3] = {}, *b[3] = {}, *gW[3] = {}, *gb[3] = {};
  float *mW[3] = {}, *vW[3] = {}, *mb[3] = {}, *vb[3] = {};
  ms::bf16 *Wb[3] = {};
  // WbT[l][j][o] = Wb[l][o][j] for the two layers whose input gradient the
  // backward pass needs, so dZ = dY W is a product with B stored [N][K]
  ms::bf16 *WbT[3] = {};
  float *mean = nullptr, *stdv = nullptr, *istd = nullptr, *mask = nullptr;
  float *lo = nullptr, *hi = nullptr;
  int *hinge_q = nullptr;  // q index of each input (-1 = padding)
  int *q_input = nullptr;  // input driving each q index (-1: none)
  // workspace for up to cap poses
  int cap = 0;
  ms::bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *dYb = nullptr, *dZ2b = nullptr,
           *dZ1b = nullptr;
  float *Z1 = nullptr, *Z2 = nullptr, *Y = nullptr, *dZ2 = nullptr,
        *dZ1 = nullptr, *part = nullptr, *cpart = nullptr, *kwork = nullptr;
  // transposed copies [features][batch] of a layer's output gradient (tA)
  // and input (tB), the operands of its weight gradient
  ms::bf16 *tA = nullptr, *tB = nullptr;
  // training batches: poses, exact labels, output statistics
  float *Qb = nullptr, *Lb = nullptr, *Rb = nullptr, *acc = nullptr, *acc2 = nullptr;
  std::vector<void *> owned;
};

namespace ms {
namespace {

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ float unit24(unsigned long long z) {
  return (float)((unsigned)(z >> 40)) * 5.9604644775390625e-8f;
}

// LeCun-uniform weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) from a counter
// hash; biases zero.
__global__ void k_init(float *W, int n, int fan_in, unsigned long long seed) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float a = 1.0f / sqrtf((float)fan_in);
  W[i] = (2.0f * unit24(splitmix64(seed ^ (unsigned long long)i)) - 1.0f) * a;
}

__global__ void k_to_bf16(const float *x, bf16 *y, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = __float2bfloat16(x[i]);
}

// x[p][i] = bf16(q[p][hinge_q[i]]) (0 for padding inputs)
// x[p][i] = bf16((q[p][hinge_q[i]] - c_i) * 2 / (hi_i - lo_i)) with
// c_i = (lo_i + hi_i) / 2: each input's pose box mapped onto [-1, 1]
__global__ void k_pack(const float *q, int nq, const int *hq, const float *lo, const float *hi,
                       int n_in, int n, bf16 *X) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n_in) return;
  const int p = t / n_in, i = t % n_in;
  const int j = hq[i];
  float x = 0.0f;
  if (j >= 0) {
    const float c = 0.5f * (lo[i] + hi[i]), is = 2.0f / (hi[i] - lo[i]);
    x = (q[(size_t)p * nq + j] - c) * is;
  }
  X[t] = __float2bfloat16(x);
}

// poses uniform in the surrogate's box: hinge i of pose p from
// SplitMix64(SplitMix64(seed ^ (offset + p)) ^ i); the root at the origin.
// One thread per pose coordinate j; qi[j] is the input that drives it.
__global__ void k_sample(int n, int nq, int free_root, const int *qi, const float *lo,
                         const float *hi, unsigned long long seed, long long offset, float *q) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * nq) return;
  const int p = (int)(t / nq), j = (int)(t % nq), i = qi[j];
  float v = free_root && j == 3 ? 1.0f : 0.0f;
  if (i >= 0) {
    const unsigned long long key = splitmix64(seed ^ (unsigned long long)(offset + p));
    v = lo[i] + (hi[i] - lo[i]) * unit24(splitmix64(key ^ (unsigned long long)i));
  }
  q[t] = v;
}

// Rows per chunk of the column sums and of the loss kernel.
constexpr int kCS = 64;

// Loss and output gradient of one training batch, the standardised target
// computed in place from the labels: T[p][o] = mask[o] (y - mean[o]) istd[o]
// with y = L[p][o] for o < n_mus, else r[p][(o - n_mus)]; d = mask (Y - T),
// dYb = bf16(2 d / (n n_out)). Block (x, y) takes 256 consecutive outputs o
// over rows [kCS y, kCS (y + 1)) and writes cpart[y][o] = sum over those
// rows of 2 d / (n n_out) (float32, row order) and part[block] = sum of d^2
// over its outputs and rows (fixed-order tree).
__global__ __launch_bounds__(256) void k_loss(const float *Y, const float *L, const float *r,
                                              int n_mus, int n, const float *mean,
                                              const float *istd, const float *mask, bf16 *dYb,
                                              float *cpart, float *part) {
  __shared__ float red[256];
  const int n_out = 4 * n_mus;
  const int o = blockIdx.x * 256 + threadIdx.x, p0 = blockIdx.y * kCS, p1 = min(n, p0 + kCS);
  float l = 0.0f;
  if (o < n_out) {
    const float mk = mask[o], mu = mean[o], is = istd[o], sc = 2.0f / ((float)n * (float)n_out);
    const float *lab = o < n_mus ? L + o : r + (o - n_mus);
    const size_t lp = o < n_mus ? (size_t)n_mus : (size_t)3 * n_mus;
    float gs = 0.0f;
    for (int p = p0; p < p1; p += 8) {
      float y[8], t[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        y[u] = p + u < p1 ? Y[(size_t)(p + u) * n_out + o] : 0.0f;
        t[u] = p + u < p1 ? lab[(size_t)(p + u) * lp] : 0.0f;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        if (p + u >= p1) break;
        const float tt = mk != 0.0f ? (t[u] - mu) * is : 0.0f;
        const float d = mk * (y[u] - tt), g = sc * d;
        l += d * d;
        gs += g;
        dYb[(size_t)(p + u) * n_out + o] = __float2bfloat16(g);
      }
    }
    cpart[(size_t)blockIdx.y * n_out + o] = gs;
  }
  red[threadIdx.x] = l;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.y * gridDim.x + blockIdx.x] = red[0];
}

// loss = sum(part) / (n n_out): 256 threads sum strided slices (loads eight
// at a time), then a fixed-order tree (deterministic)
__global__ __launch_bounds__(256) void k_loss_final(const float *part, int nb, int n, int n_out,
                                                    float *loss) {
  __shared__ double red[256];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 8 * 256) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = i + u * 256 < nb ? part[i + u * 256] : 0.0f;
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) *loss = (float)(red[0] / ((double)n * (double)n_out));
}

// Column sums, fixed order: block (x, y) takes 64 columns over rows
// [chunk y, chunk (y + 1)); wavefront g of 4 sums rows g, g + 4, ... of
// that range (loads eight at a time), and the four partial sums are added
// in order into out[y][c].
__global__ __launch_bounds__(256) void k_colsum(const float *X, int rows, int cols, int chunk,
                                                float *out) {
  __shared__ float red[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63), g = threadIdx.x >> 6;
  const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
  float s = 0.0f;
  if (c < cols) {
    for (int r = r0 + g; r < r1; r += 32) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = r + 4 * u < r1 ? X[(size_t)(r + 4 * u) * cols + c] : 0.0f;
#pragma unroll
      for (int u = 0; u < 8; ++u) s += v[u];
    }
  }
  red[g][threadIdx.x & 63] = s;
  __syncthreads();
  if (g == 0 && c < cols) {
    const int t = threadIdx.x;
    out[(size_t)blockIdx.y * cols + c] = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
  }
}

// acc[o] (+)= sum over the rows of Y[n][n_out] of y (pass 1) or of
// (y - mean[o])^2 (pass 2, mean given), in row order
__global__ void k_stat_rows(const float *Y, int n, int n_out, const float *mean, int init,
                            float *acc) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  float s = init ? 0.0f : acc[o];
  for (int p = 0; p < n; ++p) {
    const float y = Y[(size_t)p * n_out + o];
    if (mean) {
      const float d = y - mean[o];
      s += d * d;
    } else {
      s += y;
    }
  }
  acc[o] = s;
}

// labels [L | r] of one batch of poses into Y[n][n_out]
__global__ void k_pack_labels(const float *L, const float *r, int n_mus, int n, float *Y) {
  const int n_out = 4 * n_mus;
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * n_out) return;
  const int p = t / n_out, o = t % n_out;
  Y[t] = o < n_mus ? L[(size_t)p * n_mus + o] : r[(size_t)p * 3 * n_mus + (o - n_mus)];
}

// mean = acc / n; empty moment-arm slots (mask 0) get mean 0
__global__ void k_stat_mean(const float *acc, const float *mask, int n, int n_out, float *mean) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  mean[o] = mask[o] != 0.0f ? acc[o] / (float)n : 0.0f;
}

// std = max(sqrt(acc2 / n), 1e-6) (1 for empty slots), and its reciprocal
__global__ void k_stat_std(const float *acc2, const float *mask, int n, int n_out, float *stdv,
                           float *istd) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= n_out) return;
  const float v = mask[o] != 0.0f ? fmaxf(sqrtf(acc2[o] / (float)n), 1e-6f) : 1.0f;
  stdv[o] = v;
  istd[o] = 1.0f / v;
}

__global__ void k_adam(float *w, float *m, float *v, const float *g, int n, float lr, float b1,
                       float b2, float eps, float c1, float c2, bf16 *wb) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  w[i] = wi;
  if (wb) wb[i] = __float2bfloat16(wi);
}

inline int blocks(long long n, int b = 256) { return (int)((n + b - 1) / b); }

// WT[c][r] = bf16(W[r][c]) for W[rows][cols], through 32 x 32 LDS tiles so
// both the reads and the writes are row-contiguous; 256 threads per tile.
__global__ void k_transpose_bf16(const float *W, bf16 *WT, int rows, int cols) {
  __shared__ float t[32][33];
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int r = r0 + k, c = c0 + tx;
    t[k][tx] = (r < rows && c < cols) ? W[(size_t)r * cols + c] : 0.0f;
  }
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int c = c0 + k, r = r0 + tx;
    if (r < rows && c < cols) WT[(size_t)c * rows + r] = __float2bfloat16(t[tx][k]);
  }
}

void transpose_w(const float *W, bf16 *WT, int rows, int cols, hipStream_t st) {
  hipLaunchKernelGGL(k_transpose_bf16, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(256), 0, st,
                     W, WT, rows, cols);
}

// out[c] = column sums of X[rows][cols], deterministic order
void colsum(ms_surrogate *s, const float *X, int rows, int cols, float *out, hipStream_t st) {
  const int nk = (rows + kCS - 1) / kCS;
  hipLaunchKernelGGL(k_colsum, dim3((cols + 63) / 64, nk), dim3(256), 0, st, X, rows, cols, kCS,
                     s->cpart);
  hipLaunchKernelGGL(k_colsum, dim3((cols + 63) / 64, 1), dim3(256), 0, st, s->cpart, nk, cols, nk,
                     out);
}

thread_local std::string s_err;
ms_status sfail(ms_status s, const std::string &m) {
  s_err = m;
  return s;
}

template <class T>
T *dalloc(ms_surrogate *s, size_t n) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
  (void)hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T));
  s->owned.push_back(p);
  return (T *)p;
}

// Allocate every buffer of a request or none: on a failure the buffers
// already taken are freed and the caller's fields stay as they were.
struct AllocSet {
  std::vector<std::pair<void **, size_t>> want;
  template <class T>
  void add(T **field, size_t n) {
    want.push_back({(void **)field, std::max<size_t>(n, 1) * sizeof(T)});
  }
  bool commit(std::vector<void *> &owned) {
    std::vector<void *> got(want.size(), nullptr);
    for (size_t i = 0; i < want.size(); ++i) {
      if (hipMalloc(&got[i], want[i].second) != hipSuccess) {
        for (size_t j = 0; j < i; ++j) (void)hipFree(got[j]);
        return false;
      }
    }
    for (size_t i = 0; i < want.size(); ++i) {
      *want[i].first = got[i];
      owned.push_back(got[i]);
    }
    return true;
  }
};

// Workspace for n poses. The kernels write every workspace element before
// reading it, so nothing is cleared. A larger workspace replaces the old
// one, which stays allocated until destroy: launches still queued may use it.
ms_status ensure_cap(ms_surrogate *s, int n) {
  if (n <= s->cap) return MS_OK;
  const size_t B = (size_t)n;
  AllocSet a;
  a.add(&s->X, B * s->n_in);
  a.add(&s->Z1, B * s->h1);
  a.add(&s->H1, B * s->h1);
  a.add(&s->Z2, B * s->h2);
  a.add(&s->H2, B * s->h2);
  a.add(&s->Y, B * s->n_out);
  a.add(&s->dYb, B * s->n_out);
  a.add(&s->dZ2, B * s->h2);
  a.add(&s->dZ2b, B * s->h2);
  a.add(&s->dZ1, B * s->h1);
  a.add(&s->dZ1b, B * s->h1);
  a.add(&s->part, (size_t)blocks(s->n_out) * ((B + kCS - 1) / kCS));
  a.add(&s->cpart, (size_t)((B + kCS - 1) / kCS) * std::max(s->n_out, std::max(s->h1, s->h2)));
  {
    // split-K partials of the weight gradients (K = batch)
    const int M[3] = {s->n_out, s->h2, s->h1}, N[3] = {s->h2, s->h1, s->n_in};
    size_t w = 0;
    for (int l = 0; l < 3; ++l)
      w = std::max(w, (size_t)splitk_slices(M[l], N[l], n) * M[l] * N[l]);
    a.add(&s->kwork, w);
    a.add(&s->tA, B * std::max(s->n_out, std::max(s->h1, s->h2)));
    a.add(&s->tB, B * std::max(s->n_in, std::max(s->h1, s->h2)));
  }
  a.add(&s->Qb, B * s->nq);
  a.add(&s->Lb, B * s->n_mus);
  a.add(&s->Rb, B * 3 * s->n_mus);
  a.add(&s->acc, (size_t)s->n_out);
  a.add(&s->acc2, (size_t)s->n_out);
  if (!a.commit(s->owned)) return sfail(MS_E_ALLOC, "surrogate workspace allocation failed");
  s->cap = n;
  return MS_OK;
}

ms_status hipst(hipError_t e, const char *what) {
  if (e != hipSuccess) return sfail(MS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MS_OK;
}

// Buffers of one forward pass: packed inputs, hidden activations (with
// the pre-activations when training needs them) and the outputs.
struct FwdWork {
  bf16 *X, *H1, *H2;
  float *Z1, *Z2, *Y;
  float *L = nullptr, *R = nullptr;  // when set: lengths and moment arms instead of Y
};
FwdWork own_work(ms_surrogate *s, bool keep) {
  return FwdWork{s->X, s->H1, s->H2, keep ? s->Z1 : nullptr, keep ? s->Z2 : nullptr, s->Y};
}

// forward through the three layers into w.Y (standardised, or
// de-standardised when destd), keeping Z1/Z2 when w holds them (training)
ms_status forward(ms_surrogate *s, int n, const float *q, bool destd, const FwdWork &w,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_pack, dim3(blocks((long long)n * s->n_in)), dim3(256), 0, st, q, s->nq,
                     s->hinge_q, s->lo, s->hi, s->n_in, n, w.X);
  GemmEpi e1;
  e1.bias = s->b[0];
  e1.z_out = w.Z1;
  e1.act = 1;
  e1.c_bf16 = w.H1;
  e1.ldc = s->h1;
  hipError_t e = gemm_bf16(n, s->h1, s->n_in, w.X, s->n_in, s->Wb[0], s->n_in, e1, st);
  if (e != hipSuccess) return hipst(e, "gemm 1");
  GemmEpi e2;
  e2.bias = s->b[1];
  e2.z_out = w.Z2;
  e2.act = 1;
  e2.c_bf16 = w.H2;
  e2.ldc = s->h2;
  e = gemm_bf16(n, s->h2, s->h1, w.H1, s->h1, s->Wb[1], s->h1, e2, st);
  if (e != hipSuccess) return hipst(e, "gemm 2");
  GemmEpi e3;
  e3.bias = s->b[2];
  e3.c_f32 = w.L ? w.L : w.Y;
  e3.ldc = w.L ? s->n_mus : s->n_out;
  if (w.L) {
    e3.c2 = w.R;
    e3.split = s->n_mus;
    e3.ldc2 = 3 * s->n_mus;
  }
  if (destd) {
    e3.scale = s->stdv;
    e3.shift = s->mean;
  }
  e = gemm_bf16(n, s->n_out, s->h2, w.H2, s->h2, s->Wb[2], s->h2, e3, st);
  return hipst(e, "gemm 3");
}

// ---------------------------------------------- allocation-free forward
// Device memory of ms_surrogate_forward_noalloc: one static array per GPU
// (each device holds its own copy until the process ends). Host code never
// uses the array's name as an address: its device address is taken once
// per device with hipGetSymbolAddress, with that device current, and kept
// in scratch_dev[device].
constexpr size_t kScratchBytes = (size_t)16 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kScratchBytes];
void *scratch_dev[kMaxDevices] = {};
std::mutex scratch_mu;

// Address of the current device's scratch array (looked up on first use).
ms_status scratch_address(void **out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hipst(e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return sfail(MS_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hipst(e, "hipGetSymbolAddress(scratch)");
    scratch_dev[dev] = p;
  }
  *out = scratch_dev[dev];
  return MS_OK;
}

inline size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// Bytes of scratch a forward of n poses takes: X, H1, H2 (bfloat16); the
// output layer writes the caller's L and r directly.
size_t noalloc_bytes(const ms_surrogate *s, long long n) {
  return align256((size_t)n * s->n_in * 2) + align256((size_t)n * s->h1 * 2) +
         align256((size_t)n * s->h2 * 2);
}

}  // namespace
}  // namespace ms

using namespace ms;

ms_status ms_surrogate_predict(ms_surrogate *s, int n, const float *q, const float **Y,
                               hipStream_t st) {
  ms_status r = ensure_cap(s, n);
  if (r != MS_OK) return r;
  r = forward(s, n, q, true, own_work(s, false), st);
  *Y = s->Y;
  return r;
}

extern "C" {

const char *ms_surrogate_last_error(void) { return s_err.c_str(); }

ms_status ms_surrogate_create(const ms_model *m, int32_t hidden, uint64_t seed, ms_surrogate **out) {
  s_err.clear();
  if (!m || !out || hidden <= 0 || hidden % 8) return sfail(MS_E_ARG, "bad arguments (hidden must be a positive multiple of 8)");
  ms_model_info info;
  if (ms_model_info_get(m, &info) != MS_OK) return sfail(MS_E_ARG, "model info failed");
  std::vector<int> hq;
  std::vector<float> lo, hi;
  ms_surrogate_tables(m, &hq, &lo, &hi);
  ms_surrogate *s = new ms_surrogate();
  s->n_mus = info.n_mus;
  s->nq = info.nq;
  s->free_root = info.nq != info.nv;
  s->n_in = ((int)hq.size() + 15) / 16 * 16;
  s->h1 = s->h2 = hidden;
  s->n_out = 4 * info.n_mus;
  hq.resize(s->n_in, -1);
  lo.resize(s->n_in, 0.0f);
  hi.resize(s->n_in, 0.0f);
  const int in[3] = {s->n_in, s->h1, s->h2}, outd[3] = {s->h1, s->h2, s->n_out};
  for (int l = 0; l < 3; ++l) {
    const size_t nw = (size_t)in[l] * outd[l];
    s->W[l] = dalloc<float>(s, nw);
    s->gW[l] = dalloc<float>(s, nw);
    s->mW[l] = dalloc<float>(s, nw);
    s->vW[l] = dalloc<float>(s, nw);
    s->Wb[l] = dalloc<bf16>(s, nw);
    if (l > 0) s->WbT[l] = dalloc<bf16>(s, nw);
    s->b[l] = dalloc<float>(s, outd[l]);
    s->gb[l] = dalloc<float>(s, outd[l]);
    s->mb[l] = dalloc<float>(s, outd[l]);
    s->vb[l] = dalloc<float>(s, outd[l]);
    if (!s->W[l] || !s->gW[l] || !s->mW[l] || !s->vW[l] || !s->Wb[l] || (l > 0 && !s->WbT[l]) ||
        !s->b[l] || !s->gb[l] || !s->mb[l] || !s->vb[l]) {
      ms_surrogate_destroy(s);
      return sfail(MS_E_ALLOC, "surrogate allocation failed");
    }
    hipLaunchKernelGGL(k_init, dim3(blocks((long long)nw)), dim3(256), 0, 0, s->W[l], (int)nw, in[l],
                       (unsigned long long)seed * 3ull + (unsigned long long)l);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long long)nw)), dim3(256), 0, 0, s->W[l], s->Wb[l], (int)nw);
    if (s->WbT[l]) transpose_w(s->W[l], s->WbT[l], outd[l], in[l], 0);
  }
  s->mean = dalloc<float>(s, s->n_out);
  s->stdv = dalloc<float>(s, s->n_out);
  s->istd = dalloc<float>(s, s->n_out);
  s->mask = dalloc<float>(s, s->n_out);
  s->lo = dalloc<float>(s, s->n_in);
  s->hi = dalloc<float>(s, s->n_in);
  s->hinge_q = dalloc<int>(s, s->n_in);
  s->q_input = dalloc<int>(s, s->nq);
  if (!s->mean || !s->stdv || !s->istd || !s->mask || !s->lo || !s->hi || !s->hinge_q ||
      !s->q_input) {
    ms_surrogate_destroy(s);
    return sfail(MS_E_ALLOC, "surrogate allocation failed");
  }
  // identity standardisation until set; mask from the span table
  std::vector<int32_t> spans((size_t)3 * s->n_mus);
  if (s->n_mus > 0) ms_model_spans(m, spans.data());
  std::vector<float> ones(s->n_out, 1.0f), zeros(s->n_out, 0.0f), msk(s->n_out, 1.0f);
  for (int i = 0; i < 3 * s->n_mus; ++i) msk[s->n_mus + i] = spans[i] >= 0 ? 1.0f : 0.0f;
  hipError_t e = hipMemcpy(s->mean, zeros.data(), 4 * s->n_out, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->stdv, ones.data(), 4 * s->n_out, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->istd, ones.data(), 4 * s->n_out, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->mask, msk.data(), 4 * s->n_out, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->lo, lo.data(), 4 * s->n_in, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->hi, hi.data(), 4 * s->n_in, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->hinge_q, hq.data(), 4 * s->n_in, hipMemcpyHostToDevice);
  std::vector<int> qi(s->nq, -1);
  for (int i = 0; i < s->n_in; ++i)
    if (hq[i] >= 0) qi[hq[i]] = i;
  if (e == hipSuccess) e = hipMemcpy(s->q_input, qi.data(), 4 * s->nq, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    ms_surrogate_destroy(s);
    return hipst(e, "surrogate setup");
  }
  // the allocation-free forward's scratch address on this device
  void *scr = nullptr;
  const ms_status ss = scratch_address(&scr);
  if (ss != MS_OK) {
    ms_surrogate_destroy(s);
    return ss;
  }
  *out = s;
  return MS_OK;
}

void ms_surrogate_destroy(ms_surrogate *s) {
  if (!s) return;
  for (void *p : s->owned) (void)hipFree(p);
  delete s;
}

ms_status ms_surrogate_dims(const ms_surrogate *s, int32_t *dims) {
  if (!s || !dims) return sfail(MS_E_ARG, "NULL argument");
  dims[0] = s->n_in;
  dims[1] = s->h1;
  dims[2] = s->h2;
  dims[3] = s->n_out;
  return MS_OK;
}

ms_status ms_surrogate_params(ms_surrogate *s, int32_t set, float *W1, float *b1, float *W2, float *b2,
                              float *W3, float *b3) {
  if (!s || !W1 || !b1 || !W2 || !b2 || !W3 || !b3) return sfail(MS_E_ARG, "NULL argument");
  float *hw[3] = {W1, W2, W3}, *hb[3] = {b1, b2, b3};
  const int in[3] = {s->n_in, s->h1, s->h2}, outd[3] = {s->h1, s->h2, s->n_out};
  hipError_t e = hipDeviceSynchronize();
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    const size_t nw = (size_t)in[l] * outd[l];
    if (set) {
      e = hipMemcpy(s->W[l], hw[l], 4 * nw, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(s->b[l], hb[l], 4 * outd[l], hipMemcpyHostToDevice);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long long)nw)), dim3(256), 0, 0, s->W[l], s->Wb[l], (int)nw);
        if (s->WbT[l]) transpose_w(s->W[l], s->WbT[l], outd[l], in[l], 0);
        e = hipGetLastError();
      }
    } else {
      e = hipMemcpy(hw[l], s->W[l], 4 * nw, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(hb[l], s->b[l], 4 * outd[l], hipMemcpyDeviceToHost);
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return hipst(e, "params copy");
}

ms_status ms_surrogate_grads(ms_surrogate *s, float *W1, float *b1, float *W2, float *b2, float *W3,
                             float *b3) {
  if (!s || !W1 || !b1 || !W2 || !b2 || !W3 || !b3) return sfail(MS_E_ARG, "NULL argument");
  float *hw[3] = {W1, W2, W3}, *hb[3] = {b1, b2, b3};
  const int in[3] = {s->n_in, s->h1, s->h2}, outd[3] = {s->h1, s->h2, s->n_out};
  hipError_t e = hipDeviceSynchronize();
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    e = hipMemcpy(hw[l], s->gW[l], 4 * (size_t)in[l] * outd[l], hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(hb[l], s->gb[l], 4 * outd[l], hipMemcpyDeviceToHost);
  }
  return hipst(e, "grads copy");
}

ms_status ms_surrogate_set_norm(ms_surrogate *s, const float *mean, const float *stdv) {
  if (!s || !mean || !stdv) return sfail(MS_E_ARG, "NULL argument");
  std::vector<float> is(s->n_out);
  for (int i = 0; i < s->n_out; ++i) {
    if (!(stdv[i] > 0.0f) || !std::isfinite(mean[i])) return sfail(MS_E_ARG, "std must be > 0");
    is[i] = 1.0f / stdv[i];
  }
  hipError_t e = hipMemcpy(s->mean, mean, 4 * s->n_out, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->stdv, stdv, 4 * s->n_out, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->istd, is.data(), 4 * s->n_out, hipMemcpyHostToDevice);
  return hipst(e, "set norm");
}

ms_status ms_surrogate_sample(ms_surrogate *s, int32_t n, uint64_t seed, int64_t offset, float *q,
                              void *stream) {
  if (!s || n <= 0 || !q) return sfail(MS_E_ARG, "bad arguments");
  hipLaunchKernelGGL(k_sample, dim3(blocks((long long)n * s->nq)), dim3(256), 0, (hipStream_t)stream, n, s->nq,
                     s->free_root, s->q_input, s->lo, s->hi, (unsigned long long)seed,
                     (long long)offset, q);
  return hipst(hipGetLastError(), "sample");
}

ms_status ms_surrogate_forward(ms_surrogate *s, int32_t n, const float *q, float *L, float *r,
                               void *stream) {
  s_err.clear();
  if (!s || n <= 0 || !q || !L || !r) return sfail(MS_E_ARG, "bad arguments");
  ms_status st = ensure_cap(s, n);
  if (st != MS_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  FwdWork w = own_work(s, false);
  w.L = L;
  w.R = r;
  return forward(s, n, q, true, w, hs);
}

ms_status ms_surrogate_reserve(ms_surrogate *s, int32_t n) {
  s_err.clear();
  if (!s || n <= 0) return sfail(MS_E_ARG, "bad arguments");
  return ensure_cap(s, n);
}

ms_status ms_surrogate_forward_noalloc(ms_surrogate *s, int32_t n, const float *q, float *L,
                                       float *r, void *stream) {
  s_err.clear();
  if (!s || n <= 0 || !q || !L || !r) return sfail(MS_E_ARG, "bad arguments");
  const size_t need = noalloc_bytes(s, n);
  if (need > kScratchBytes)
    return sfail(MS_E_UNSUPPORTED, "ms_surrogate_forward_noalloc: " + std::to_string(n) +
                                       " poses need " + std::to_string(need) +
                                       " bytes of scratch, beyond its " +
                                       std::to_string(kScratchBytes) + " (at most " +
                                       std::to_string(ms_surrogate_noalloc_max(s)) + " poses)");
  void *base = nullptr;
  ms_status st = scratch_address(&base);
  if (st != MS_OK) return st;
  unsigned char *p = (unsigned char *)base;
  FwdWork w;
  w.X = (bf16 *)p;
  p += align256((size_t)n * s->n_in * 2);
  w.H1 = (bf16 *)p;
  p += align256((size_t)n * s->h1 * 2);
  w.H2 = (bf16 *)p;
  w.Y = nullptr;
  w.Z1 = w.Z2 = nullptr;
  w.L = L;
  w.R = r;
  return forward(s, n, q, true, w, (hipStream_t)stream);
}

int32_t ms_surrogate_noalloc_max(const ms_surrogate *s) {
  if (!s) return 0;
  long long lo = 0, hi = 1;
  while (noalloc_bytes(s, hi) <= kScratchBytes) hi *= 2;
  while (hi - lo > 1) {
    const long long mid = (lo + hi) / 2;
    (noalloc_bytes(s, mid) <= kScratchBytes ? lo : hi) = mid;
  }
  return (int32_t)lo;
}

ms_status ms_surrogate_train(ms_model *m, ms_surrogate *s, const ms_train_cfg *c, void *stream) {
  s_err.clear();
  if (!m || !s || !c) return sfail(MS_E_ARG, "NULL argument");
  if (c->batch <= 0 || c->batch % 8 || c->batch > (1 << 20) || c->iters < 0 ||
      c->n_samples <= 0 || c->step0 < 0 || c->norm_samples < 0 || !(c->lr0 >= 0.0f) ||
      !(c->lr1 >= 0.0f))
    return sfail(MS_E_ARG, "bad training configuration (batch a positive multiple of 8 up to "
                           "2^20, iters, n_samples > 0, step0 >= 0, norm_samples >= 0, lr >= 0)");
  ms_model_info info;
  if (ms_model_info_get(m, &info) != MS_OK || info.n_mus != s->n_mus || info.nq != s->nq)
    return sfail(MS_E_ARG, "surrogate does not belong to this model");
  ms_status st = ensure_cap(s, c->batch);
  if (st != MS_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  const int B = c->batch, no = s->n_out;
  auto labels = [&](int n, unsigned long long seed, long long offset) -> ms_status {
    hipLaunchKernelGGL(k_sample, dim3(blocks((long long)n * s->nq)), dim3(256), 0, hs, n, s->nq, s->free_root,
                       s->q_input, s->lo, s->hi, seed, offset, s->Qb);
    if (ms_geometry(m, n, s->Qb, s->Lb, s->Rb, hs) != MS_OK)
      return sfail(MS_E_HIP, std::string("labels: ") + ms_last_error());
    return MS_OK;
  };
  // output standardisation: mean, then std about it, over norm_samples poses
  // sampled with norm_seed, in batches of B (fixed order)
  if (c->norm_samples > 0) {
    for (int pass = 0; pass < 2; ++pass) {
      for (long long o = 0; o < c->norm_samples; o += B) {
        const int n = (int)std::min<long long>(B, c->norm_samples - o);
        st = labels(n, c->norm_seed, o);
        if (st != MS_OK) return st;
        hipLaunchKernelGGL(k_pack_labels, dim3(blocks((long long)n * no)), dim3(256), 0, hs, s->Lb,
                           s->Rb, s->n_mus, n, s->Y);
        hipLaunchKernelGGL(k_stat_rows, dim3(blocks(no)), dim3(256), 0, hs, s->Y, n, no,
                           pass ? s->mean : (const float *)nullptr, o == 0 ? 1 : 0,
                           pass ? s->acc2 : s->acc);
      }
      if (pass == 0)
        hipLaunchKernelGGL(k_stat_mean, dim3(blocks(no)), dim3(256), 0, hs, s->acc, s->mask,
                           (int)c->norm_samples, no, s->mean);
      else
        hipLaunchKernelGGL(k_stat_std, dim3(blocks(no)), dim3(256), 0, hs, s->acc2, s->mask,
                           (int)c->norm_samples, no, s->stdv, s->istd);
    }
    st = hipst(hipGetLastError(), "output statistics");
    if (st != MS_OK) return st;
  }
  // Adam with the learning rate decayed from lr0 to lr1 along a half cosine
  for (int it = 0; it < c->iters; ++it) {
    const long long offset = ((long long)it * B) % c->n_samples;
    st = labels(B, c->seed, offset);
    if (st != MS_OK) return st;
    const double ph = 3.14159265358979323846 * (double)it / (double)c->iters;
    const float lr = (float)(c->lr1 + 0.5 * ((double)c->lr0 - c->lr1) * (1.0 + std::cos(ph)));
    st = ms_surrogate_train_step(s, B, s->Qb, s->Lb, s->Rb, lr, c->step0 + it + 1,
                                 c->loss ? c->loss + it : nullptr, stream);
    if (st != MS_OK) return st;
  }
  return MS_OK;
}

namespace {
constexpr uint32_t kBlobMagic = 0x4D534731u;  // "MSG1"
}

ms_status ms_surrogate_save(ms_surrogate *s, void *blob, size_t cap, size_t *size) {
  s_err.clear();
  if (!s || !size) return sfail(MS_E_ARG, "NULL argument");
  const int in[3] = {s->n_in, s->h1, s->h2}, outd[3] = {s->h1, s->h2, s->n_out};
  size_t n = 8 * 4;
  for (int l = 0; l < 3; ++l) n += 4 * ((size_t)in[l] * outd[l] + outd[l]);
  n += 8 * (size_t)s->n_out;
  *size = n;
  if (!blob) return MS_OK;  // size query
  if (cap < n) return sfail(MS_E_ARG, "blob too small (" + std::to_string(n) + " bytes needed)");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hipst(e, "synchronise");
  unsigned char *p = (unsigned char *)blob;
  const uint32_t head[8] = {kBlobMagic, 1u, (uint32_t)s->n_in, (uint32_t)s->h1, (uint32_t)s->h2,
                            (uint32_t)s->n_out, 0u, 0u};
  std::memcpy(p, head, sizeof head);
  p += sizeof head;
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    const size_t nw = (size_t)in[l] * outd[l];
    e = hipMemcpy(p, s->W[l], 4 * nw, hipMemcpyDeviceToHost);
    p += 4 * nw;
    if (e == hipSuccess) e = hipMemcpy(p, s->b[l], 4 * (size_t)outd[l], hipMemcpyDeviceToHost);
    p += 4 * (size_t)outd[l];
  }
  if (e == hipSuccess) e = hipMemcpy(p, s->mean, 4 * (size_t)s->n_out, hipMemcpyDeviceToHost);
  p += 4 * (size_t)s->n_out;
  if (e == hipSuccess) e = hipMemcpy(p, s->stdv, 4 * (size_t)s->n_out, hipMemcpyDeviceToHost);
  return hipst(e, "save");
}

ms_status ms_surrogate_load(ms_surrogate *s, const void *blob, size_t size) {
  s_err.clear();
  if (!s || !blob) return sfail(MS_E_ARG, "NULL argument");
  size_t need = 0;
  ms_status st = ms_surrogate_save(s, nullptr, 0, &need);
  if (st != MS_OK) return st;
  uint32_t head[8];
  if (size < sizeof head) return sfail(MS_E_ARG, "blob too small");
  std::memcpy(head, blob, sizeof head);
  if (head[0] != kBlobMagic || head[1] != 1u) return sfail(MS_E_ARG, "not a surrogate blob");
  if ((int)head[2] != s->n_in || (int)head[3] != s->h1 || (int)head[4] != s->h2 ||
      (int)head[5] != s->n_out)
    return sfail(MS_E_ARG, "blob layer sizes differ from this network's");
  if (size != need) return sfail(MS_E_ARG, "blob size does not match its layer sizes");
  const unsigned char *p = (const unsigned char *)blob + sizeof head;
  const int in[3] = {s->n_in, s->h1, s->h2}, outd[3] = {s->h1, s->h2, s->n_out};
  std::vector<float> w[3], b[3];
  for (int l = 0; l < 3; ++l) {
    w[l].resize((size_t)in[l] * outd[l]);
    std::memcpy(w[l].data(), p, 4 * w[l].size());
    p += 4 * w[l].size();
    b[l].resize(outd[l]);
    std::memcpy(b[l].data(), p, 4 * b[l].size());
    p += 4 * b[l].size();
  }
  std::vector<float> mean(s->n_out), stdv(s->n_out);
  std::memcpy(mean.data(), p, 4 * mean.size());
  p += 4 * mean.size();
  std::memcpy(stdv.data(), p, 4 * stdv.size());
  st = ms_surrogate_set_norm(s, mean.data(), stdv.data());
  if (st != MS_OK) return st;
  return ms_surrogate_params(s, 1, w[0].data(), b[0].data(), w[1].data(), b[1].data(),
                             w[2].data(), b[2].data());
}

ms_status ms_surrogate_train_step(ms_surrogate *s, int32_t n, const float *q, const float *L,
                                  const float *r, float lr, int32_t step, float *loss,
                                  void *stream) {
  s_err.clear();
  if (!s || n <= 0 || n % 8 || n > (1 << 20) || !q || !L || !r || step < 1)
    return sfail(MS_E_ARG,
                 "bad arguments (batch must be a positive multiple of 8, at most 2^20; step >= 1)");
  ms_status st = ensure_cap(s, n);
  if (st != MS_OK) return st;
  hipStream_t hs = (hipStream_t)stream;
  st = forward(s, n, q, false, own_work(s, true), hs);
  if (st != MS_OK) return st;
  // loss, dY (bfloat16) and gb3 = colsum dY (the loss kernel's per-chunk
  // column sums, then their sum)
  const int nk = (n + kCS - 1) / kCS, nb = blocks(s->n_out) * nk;
  hipLaunchKernelGGL(k_loss, dim3(blocks(s->n_out), nk), dim3(256), 0, hs, s->Y, L, r, s->n_mus, n,
                     s->mean, s->istd, s->mask, s->dYb, s->cpart, s->part);
  if (loss) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(256), 0, hs, s->part, nb, n, s->n_out, loss);
  hipLaunchKernelGGL(k_colsum, dim3((s->n_out + 63) / 64, 1), dim3(256), 0, hs, s->cpart, nk,
                     s->n_out, nk, s->gb[2]);
  // layer 3: gW3[o][j] = sum_p dY[p][o] H2[p][j], dH2 -> dZ2. Each weight
  // gradient is the forward-shape product of the transposed output gradient
  // [out][batch] and the transposed layer input [in][batch].
  hipError_t e = transpose_bf16(s->dYb, n, s->n_out, s->tA, hs);
  if (e == hipSuccess) e = transpose_bf16(s->H2, n, s->h2, s->tB, hs);
  if (e == hipSuccess)
    e = gemm_bf16_splitk(s->n_out, s->h2, n, s->tA, n, s->tB, n, s->gW[2], s->h2,
                         s->kwork, hs);
  if (e != hipSuccess) return hipst(e, "gemm dW3");
  GemmEpi d2;
  d2.dact = s->Z2;
  d2.c_f32 = s->dZ2;
  d2.c_bf16 = s->dZ2b;
  d2.ldc = s->h2;
  e = gemm_bf16(n, s->h2, s->n_out, s->dYb, s->n_out, s->WbT[2], s->n_out, d2, hs);
  if (e != hipSuccess) return hipst(e, "gemm dZ2");
  // layer 2
  colsum(s, s->dZ2, n, s->h2, s->gb[1], hs);
  e = transpose_bf16(s->dZ2b, n, s->h2, s->tA, hs);
  if (e == hipSuccess) e = transpose_bf16(s->H1, n, s->h1, s->tB, hs);
  if (e == hipSuccess)
    e = gemm_bf16_splitk(s->h2, s->h1, n, s->tA, n, s->tB, n, s->gW[1], s->h1,
                         s->kwork, hs);
  if (e != hipSuccess) return hipst(e, "gemm dW2");
  GemmEpi d1;
  d1.dact = s->Z1;
  d1.c_f32 = s->dZ1;
  d1.c_bf16 = s->dZ1b;
  d1.ldc = s->h1;
  e = gemm_bf16(n, s->h1, s->h2, s->dZ2b, s->h2, s->WbT[1], s->h2, d1, hs);
  if (e != hipSuccess) return hipst(e, "gemm dZ1");
  // layer 1
  colsum(s, s->dZ1, n, s->h1, s->gb[0], hs);
  e = transpose_bf16(s->dZ1b, n, s->h1, s->tA, hs);
  if (e == hipSuccess) e = transpose_bf16(s->X, n, s->n_in, s->tB, hs);
  if (e == hipSuccess)
    e = gemm_bf16_splitk(s->h1, s->n_in, n, s->tA, n, s->tB, n, s->gW[0], s->n_in,
                         s->kwork, hs);
  if (e != hipSuccess) return hipst(e, "gemm dW1");
  // Adam
  if (lr > 0.0f) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    const int in[3] = {s->n_in, s->h1, s->h2}, outd[3] = {s->h1, s->h2, s->n_out};
    for (int l = 0; l < 3; ++l) {
      const int nw = in[l] * outd[l];
      hipLaunchKernelGGL(k_adam, dim3(blocks(nw)), dim3(256), 0, hs, s->W[l], s->mW[l], s->vW[l],
                         s->gW[l], nw, lr, b1, b2, eps, c1, c2, s->Wb[l]);
      if (s->WbT[l]) transpose_w(s->W[l], s->WbT[l], outd[l], in[l], hs);
      hipLaunchKernelGGL(k_adam, dim3(blocks(outd[l])), dim3(256), 0, hs, s->b[l], s->mb[l], s->vb[l],
                         s->gb[l], outd[l], lr, b1, b2, eps, c1, c2, (bf16 *)nullptr);
    }
  }
  return hipst(hipGetLastError(), "train step");
}

}  // extern "C"

// =============================================================== policy
// A policy network mapping each env's observation to excitations: obs ->
// SiLU(W1 obs + b1) -> SiLU(W2 h1 + b2) -> sigmoid(W3 h2 + b3) in [0, 1]^n_mus,
// bfloat16 matrix-core GEMMs with float32 accumulation, LeCun-uniform
// weights from a seed (random initialisation; no training here).
//
// Observation of env e at time t (n_obs = 2 nv + n_ref, zero-padded to a
// multiple of 16): the generalised position with a free root's quaternion
// folded into a rotation vector (nv values), the generalised velocity (nv),
// and n_ref reference targets, each a sum of three sinusoids
// A sin(2 pi f t + phi) with A = 0.3 u, f = 0.5 + 1.5 u, phi = 2 pi u drawn
// from SplitMix64 on (ref_seed, env, 3 k + j), a synthetic stand-in for the
// retargeted reference motion the policy tracks.
struct ms_policy {
  int nq = 0, nv = 0, n_mus = 0, free_root = 0, n_ref = 0, n_obs = 0, n_in = 0, h = 0;
  unsigned long long ref_seed = 0;
  float *W[3] = {}, *b[3] = {};
  ms::bf16 *Wb[3] = {};
  int cap = 0;
  ms::bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr;
  float *U = nullptr;  // held excitations of the last decision [cap][n_mus]
  std::vector<void *> owned;
};

namespace ms {
namespace {

template <class T>
T *palloc(ms_policy *p, size_t n) {
  void *q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
  (void)hipMemset(q, 0, std::max<size_t>(n, 1) * sizeof(T));
  p->owned.push_back(q);
  return (T *)q;
}

__device__ __forceinline__ float ref_target(unsigned long long seed, long long env, int k, float t) {
  const unsigned long long ke = splitmix64(seed ^ (unsigned long long)env);
  float s = 0.0f;
  for (int j = 0; j < 3; ++j) {
    const unsigned long long key = splitmix64(ke ^ (unsigned long long)(3 * k + j));
    const float A = 0.3f * unit24(splitmix64(key ^ 0ull));
    const float f = 0.5f + 1.5f * unit24(splitmix64(key ^ 1ull));
    const float ph = 6.28318530717958647692f * unit24(splitmix64(key ^ 2ull));
    s += A * sinf(6.28318530717958647692f * f * t + ph);
  }
  return s;
}

// one thread per (env, input); obs_out (optional) gets the unpadded float32
// observation
__global__ void k_obs(int n, int nq, int nv, int free_root, int n_obs, int n_in,
                      const float *q, const float *qd, float t, unsigned long long seed,
                      long long env0, bf16 *X, float *obs_out) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long long)n * n_in) return;
  const int p = (int)(tid / n_in), i = (int)(tid % n_in);
  const float *qp = q + (size_t)p * nq;
  float v = 0.0f;
  if (i < nv) {
    if (!free_root) {
      v = qp[i];
    } else if (i < 3) {
      v = qp[i];
    } else if (i < 6) {
      // rotation vector of the unit quaternion (w, x, y, z), w >= 0 branch
      float w = qp[3], x = qp[4], y = qp[5], z = qp[6];
      if (w < 0.0f) { w = -w; x = -x; y = -y; z = -z; }
      const float sn = sqrtf(x * x + y * y + z * z);
      const float sc = sn > 1e-12f ? 2.0f * atan2f(sn, w) / sn : 2.0f;
      v = (i == 3 ? x : i == 4 ? y : z) * sc;
    } else {
      v = qp[i + 1];
    }
  } else if (i < 2 * nv) {
    v = qd[(size_t)p * nv + (i - nv)];
  } else if (i < n_obs) {
    v = ref_target(seed, env0 + p, i - 2 * nv, t);
  }
  X[tid] = __float2bfloat16(v);
  if (obs_out && i < n_obs) obs_out[(size_t)p * n_obs + i] = v;
}

ms_status policy_cap(ms_policy *p, int n) {
  if (n <= p->cap) return MS_OK;
  AllocSet a;
  a.add(&p->X, (size_t)n * p->n_in);
  a.add(&p->H1, (size_t)n * p->h);
  a.add(&p->H2, (size_t)n * p->h);
  a.add(&p->U, (size_t)n * p->n_mus);
  if (!a.commit(p->owned)) return sfail(MS_E_ALLOC, "policy workspace allocation failed");
  p->cap = n;
  return MS_OK;
}

ms_status policy_forward(ms_policy *p, int n, const float *q, const float *qd, double t, long long env0,
                         float *u, float *obs_out, hipStream_t st) {
  ms_status r = policy_cap(p, n);
  if (r != MS_OK) return r;
  hipLaunchKernelGGL(k_obs, dim3(blocks((long long)n * p->n_in)), dim3(256), 0, st, n, p->nq, p->nv,
                     p->free_root, p->n_obs, p->n_in, q, qd, (float)t, p->ref_seed,
                     (long long)env0, p->X, obs_out);
  GemmEpi e1;
  e1.bias = p->b[0];
  e1.act = 1;
  e1.c_bf16 = p->H1;
  e1.ldc = p->h;
  hipError_t e = gemm_bf16(n, p->h, p->n_in, p->X, p->n_in, p->Wb[0], p->n_in, e1, st);
  if (e != hipSuccess) return hipst(e, "policy gemm 1");
  GemmEpi e2;
  e2.bias = p->b[1];
  e2.act = 1;
  e2.c_bf16 = p->H2;
  e2.ldc = p->h;
  e = gemm_bf16(n, p->h, p->h, p->H1, p->h, p->Wb[1], p->h, e2, st);
  if (e != hipSuccess) return hipst(e, "policy gemm 2");
  GemmEpi e3;
  e3.bias = p->b[2];
  e3.act = 2;
  e3.c_f32 = u;
  e3.ldc = p->n_mus;
  e = gemm_bf16(n, p->n_mus, p->h, p->H2, p->h, p->Wb[2], p->h, e3, st);
  return hipst(e, "policy gemm 3");
}

}  // namespace
}  // namespace ms

extern "C" {

ms_status ms_policy_reserve(ms_policy *p, int32_t n) {
  s_err.clear();
  if (!p || n <= 0) return sfail(MS_E_ARG, "bad arguments");
  return policy_cap(p, n);
}

ms_status ms_policy_create(const ms_model *m, int32_t hidden, int32_t n_ref, uint64_t ref_seed,
                           uint64_t seed, ms_policy **out) {
  s_err.clear();
  if (!m || !out || hidden <= 0 || hidden % 8 || n_ref < 0)
    return sfail(MS_E_ARG, "bad arguments (hidden must be a positive multiple of 8)");
  ms_model_info info;
  if (ms_model_info_get(m, &info) != MS_OK) return sfail(MS_E_ARG, "model info failed");
  ms_policy *p = new ms_policy();
  p->nq = info.nq;
  p->nv = info.nv;
  p->n_mus = info.n_mus;
  p->free_root = info.nq != info.nv;
  p->n_ref = n_ref;
  p->n_obs = 2 * info.nv + n_ref;
  p->n_in = (p->n_obs + 15) / 16 * 16;
  p->h = hidden;
  p->ref_seed = ref_seed;
  const int in[3] = {p->n_in, p->h, p->h}, outd[3] = {p->h, p->h, p->n_mus};
  for (int l = 0; l < 3; ++l) {
    const size_t nw = (size_t)in[l] * outd[l];
    p->W[l] = palloc<float>(p, nw);
    p->Wb[l] = palloc<bf16>(p, nw);
    p->b[l] = palloc<float>(p, outd[l]);
    if (!p->W[l] || !p->Wb[l] || !p->b[l]) {
      ms_policy_destroy(p);
      return sfail(MS_E_ALLOC, "policy allocation failed");
    }
    hipLaunchKernelGGL(k_init, dim3(blocks((long long)nw)), dim3(256), 0, 0, p->W[l], (int)nw,
                       l == 0 ? p->n_obs : in[l], (unsigned long long)seed * 3ull + (unsigned long long)l);
    hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long long)nw)), dim3(256), 0, 0, p->W[l], p->Wb[l], (int)nw);
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    ms_policy_destroy(p);
    return hipst(e, "policy init");
  }
  *out = p;
  return MS_OK;
}

void ms_policy_destroy(ms_policy *p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  for (void *q : p->owned) (void)hipFree(q);
  delete p;
}

ms_status ms_policy_dims(const ms_policy *p, int32_t *dims) {
  if (!p || !dims) return sfail(MS_E_ARG, "NULL argument");
  dims[0] = p->n_obs;
  dims[1] = p->n_in;
  dims[2] = p->h;
  dims[3] = p->n_mus;
  return MS_OK;
}

ms_status ms_policy_params(ms_policy *p, int32_t set, float *W1, float *b1, float *W2, float *b2,
                           float *W3, float *b3) {
  if (!p || !W1 || !b1 || !W2 || !b2 || !W3 || !b3) return sfail(MS_E_ARG, "NULL argument");
  float *hw[3] = {W1, W2, W3}, *hb[3] = {b1, b2, b3};
  const int in[3] = {p->n_in, p->h, p->h}, outd[3] = {p->h, p->h, p->n_mus};
  hipError_t e = hipDeviceSynchronize();
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    const size_t nw = (size_t)in[l] * outd[l];
    if (set) {
      e = hipMemcpy(p->W[l], hw[l], 4 * nw, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(p->b[l], hb[l], 4 * outd[l], hipMemcpyHostToDevice);
      if (e == hipSuccess) {
        hipLaunchKernelGGL(k_to_bf16, dim3(blocks((long long)nw)), dim3(256), 0, 0, p->W[l], p->Wb[l], (int)nw);
        e = hipGetLastError();
      }
    } else {
      e = hipMemcpy(hw[l], p->W[l], 4 * nw, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(hb[l], p->b[l], 4 * outd[l], hipMemcpyDeviceToHost);
    }
  }
  if (e == hipSuccess) e = hipDeviceSynchronize();
  return hipst(e, "policy params copy");
}

ms_status ms_policy_act(ms_policy *p, int32_t n, const float *q, const float *qd, double t,
                        int64_t env0, float *u, float *obs_out, void *stream) {
  s_err.clear();
  if (!p || n <= 0 || !q || !qd || !u) return sfail(MS_E_ARG, "bad arguments");
  return policy_forward(p, n, q, qd, t, env0, u, obs_out, (hipStream_t)stream);
}

ms_status ms_policy_rollout(ms_model *m, ms_policy *p, ms_surrogate *sg, int32_t n_env, float *q,
                            float *qd, float *act, uint32_t *status, int32_t n_steps, int32_t decim,
                            double t0, const ms_step_opts *opts, float tol, uint32_t *fb_count,
                            float *u_record, void *stream) {
  s_err.clear();
  if (!m || !p || n_env <= 0 || !q || !qd || !act || !opts || n_steps < 0 || decim <= 0)
    return sfail(MS_E_ARG, "bad arguments");
  ms_model_info info;
  if (ms_model_info_get(m, &info) != MS_OK || info.n_mus != p->n_mus || info.nv != p->nv)
    return sfail(MS_E_ARG, "policy does not belong to this model");
  hipStream_t st = (hipStream_t)stream;
  ms_status r = policy_cap(p, n_env);
  if (r != MS_OK) return r;
  for (int t = 0; t < n_steps; t += decim) {
    const int k = std::min(decim, n_steps - t);
    r = policy_forward(p, n_env, q, qd, t0 + (double)t * opts->dt, 0, p->U, nullptr, st);
    if (r != MS_OK) return r;
    if (u_record) {
      hipError_t e = hipMemcpyAsync(u_record + (size_t)(t / decim) * n_env * p->n_mus, p->U,
                                    (size_t)n_env * p->n_mus * 4, hipMemcpyDeviceToDevice, st);
      if (e != hipSuccess) return hipst(e, "u record");
    }
    for (int j = 0; j < (sg ? k : 1); ++j) {
      ms::KRun rr{};
      rr.q = q; rr.qd = qd; rr.act = act; rr.status = status; rr.n_env = n_env;
      rr.dt = opts->dt; rr.contact = opts->contact;
      rr.u = p->U; rr.u_hold = 1; rr.exc = MS_EXC_ARRAY;
      int steps = k;
      if (sg) {
        const float *Y = nullptr;
        r = ms_surrogate_predict(sg, n_env, q, &Y, st);
        if (r != MS_OK) return r;
        rr.geomY = Y; rr.fb_tol = tol; rr.fb_count = fb_count;
        rr.step0 = t + j;
        steps = 1;
      }
      r = run_steps(m, rr, n_env, steps, st);
      if (r != MS_OK) return sfail(r, std::string("policy rollout step: ") + ms_last_error());
    }
  }
  return MS_OK;
}

}  // extern "C"
