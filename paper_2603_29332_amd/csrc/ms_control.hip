// ms_control.hip -- the control step around the physics: observation,
// policy sampling (Gaussian initial sampler refined by a flow velocity
// field), n_sub physics substeps with the excitations held, and the
// discriminator's imitation reward (Methods: "Observation space", "Action
// space", "Unified imitation environment", "Reinforcement learning with
// flow-based exploration", "Simulation parameters" for the substeps).
//
// Every network is a three-layer perceptron (SiLU hidden layers) on the
// library's bfloat16 matrix-core GEMMs with float32 accumulation, weights
// LeCun-uniform from a seed (random initialisation; training is outside the
// step). The flow network's first layer is split into an observation block,
// multiplied once per control step, and an (action, time) block multiplied
// at each of the flow steps; the sum is the same product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/ms.h"
#include "ms_gemm.h"
#include "ms_step_kernel.h"

namespace {

struct Net {
  int in = 0, h = 0, out = 0;
  float *W[3] = {}, *b[3] = {};
  ms::bf16 *Wb[3] = {};
};

inline int pad16(int x) { return (x + 15) / 16 * 16; }
inline int blocks(long long n, int b = 256) { return (int)((n + b - 1) / b); }

}  // namespace

struct ms_controller {
  ms_model *m = nullptr;
  int nq = 0, nv = 0, n_mus = 0, free_root = 0, n_h = 0, n_key = 0;
  int n_obs = 0, n_in = 0, n_at = 0, n_din = 0, hidden = 0, n_sub = 0, flow_steps = 0;
  float flow_dt = 0.0f;
  unsigned long long ref_seed = 0, noise_seed = 0;
  int *key_node = nullptr;  // device [n_key]
  int *q_hinge = nullptr;   // device [nq]: hinge index of each coordinate (-1: root)
  int *hinge_q = nullptr;   // device [n_h]: coordinate of each hinge
  float *f0 = nullptr;      // device [n_mus], caller's order
  float *log_std = nullptr; // device [n_mus]
  Net pi, flow, disc;
  ms::bf16 *Wat = nullptr;  // flow layer 1, (action, time) block [hidden][n_at]
  // per control step: the time column's contribution to flow layer 1 at
  // each flow step ([flow_steps][hidden]) and the output bias times the
  // flow step size ([n_mus])
  float *TB = nullptr, *HB3 = nullptr;
  // workspace for up to cap envs
  int cap = 0;
  ms::bf16 *X = nullptr, *H1 = nullptr, *H2 = nullptr, *XA = nullptr, *XD = nullptr;
  // A: the flow's state [cap][n_at] (rows padded like XA, whose bfloat16
  // copy the flow's output layer writes beside it)
  float *P = nullptr, *A = nullptr, *PSI = nullptr, *U = nullptr, *Z = nullptr, *qref = nullptr;
  float *kpos = nullptr, *krot = nullptr, *rpos = nullptr, *rrot = nullptr;
  std::vector<void *> owned;
};

namespace ms {
namespace {

thread_local std::string c_err;
ms_status cfail(ms_status s, const std::string &m) {
  c_err = m;
  return s;
}
ms_status chip(hipError_t e, const char *what) {
  if (e != hipSuccess) return cfail(MS_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
  return MS_OK;
}

__device__ __forceinline__ float unit24c(unsigned long long z) {
  return (float)((unsigned)(z >> 40)) * 5.9604644775390625e-8f;
}

// LeCun-uniform weights U(-1/sqrt(fan_in), 1/sqrt(fan_in)) of an [out][in]
// matrix whose columns >= used are zero (padding inputs)
__global__ void k_init_w(float *W, bf16 *Wb, int out, int in, int used, int fan_in,
                         unsigned long long seed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)out * in) return;
  const int c = (int)(i % in);
  float w = 0.0f;
  if (c < used)
    w = (2.0f * unit24c(splitmix64(seed ^ (unsigned long long)i)) - 1.0f) / sqrtf((float)fan_in);
  W[i] = w;
  Wb[i] = __float2bfloat16(w);
}

__global__ void k_fill(float *x, int n, float v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}

// reference target of hinge h of env e at time t: a sum of three sinusoids
// A sin(2 pi f t + phi), A = 0.3 a, f = 0.5 + 1.5 b Hz, phi = 2 pi c, with
// a, b, c the top 24 bits x 2^-24 of SplitMix64(K ^ 0), (K ^ 1), (K ^ 2),
// K = SplitMix64(SplitMix64(seed ^ e) ^ (3 h + j))
__device__ float ref_hinge(unsigned long long seed, long long env, int h, float t) {
  const unsigned long long ke = splitmix64(seed ^ (unsigned long long)env);
  float s = 0.0f;
  for (int j = 0; j < 3; ++j) {
    const unsigned long long key = splitmix64(ke ^ (unsigned long long)(3 * h + j));
    const float A = 0.3f * unit24c(splitmix64(key ^ 0ull));
    const float f = 0.5f + 1.5f * unit24c(splitmix64(key ^ 1ull));
    const float ph = 6.28318530717958647692f * unit24c(splitmix64(key ^ 2ull));
    s += A * sinf(6.28318530717958647692f * f * t + ph);
  }
  return s;
}

// reference pose: the env's own root, hinges at their reference targets
__global__ void k_ref_pose(int n, int nq, const float *q, const int *q_hinge,
                           unsigned long long seed, long long env0, float t, float *qref) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * nq) return;
  const int p = (int)(i / nq), j = (int)(i % nq);
  const int h = q_hinge[j];
  qref[i] = h < 0 ? q[i] : ref_hinge(seed, env0 + p, h, t);
}

// World position and orientation of the key nodes of two sets of n poses
// (the state and its reference pose), one wavefront per pose, forward
// kinematics of the step: workgroup b < n takes pose b of set a, the others
// pose b - n of set b.
__global__ __launch_bounds__(64) void k_key_frames(KModel M, int n, const int *keys, int n_key,
                                                   const float *qa, float *xpos_a, float *xrot_a,
                                                   const float *qb, float *xpos_b, float *xrot_b) {
  extern __shared__ __align__(16) unsigned char lds_k[];
  const bool second = (int)blockIdx.x >= n;
  const int p = second ? blockIdx.x - n : blockIdx.x, lane = threadIdx.x;
  if (p >= n) return;
  const float *qs = second ? qb : qa;
  float *xpos = second ? xpos_b : xpos_a, *xrot = second ? xrot_b : xrot_a;
  const int nq = M.nq, nv = M.nv, nn = M.n_node;
  float *Rl = (float *)lds_k;
  float *Sl = Rl + 12 * nn;
  float *Vl = Sl + 6 * nv;
  float *Al = Vl + 6 * nn;
  float *q = Al + 6 * nn;
  float *qd = q + nq;
  for (int i = lane; i < nq; i += 64) q[i] = qs[(size_t)p * nq + i];
  for (int i = lane; i < nv; i += 64) qd[i] = 0.0f;
  wave_sync();
  const V3 O = M.free_root ? v3(q[0], q[1], q[2]) : v3(0.f, 0.f, 0.f);
  stage_fk(M, lane, M.lt + M.lt_tlev, M.lt + M.lt_tnode, q, qd, Rl, Sl, Vl, Al, O,
           v3(M.gx, M.gy, M.gz));
  for (int k = lane; k < n_key; k += 64) {
    const float *F = Rl + 12 * keys[k];
    for (int e = 0; e < 9; ++e) xrot[((size_t)p * n_key + k) * 9 + e] = F[e];
    xpos[((size_t)p * n_key + k) * 3 + 0] = F[9] + O.x;
    xpos[((size_t)p * n_key + k) * 3 + 1] = F[10] + O.y;
    xpos[((size_t)p * n_key + k) * 3 + 2] = F[11] + O.z;
  }
}

// Observation of env p (n_obs values, zero-padded to n_in): q with a free
// root's unit quaternion as its rotation vector (nv), q' (nv), key-node
// positions (3 n_key) and orientations as the first two columns of R
// (6 n_key), muscle activations, forces / F0, normalised fibre lengths and
// velocities of the last substep (4 n_mus), the hinges' reference targets
// (n_h), the reference pose's key-node positions and orientations.
__global__ void k_ctl_obs(int n, int nq, int nv, int free_root, int n_mus, int n_key, int n_h,
                          int n_obs, int n_in, const float *q, const float *qd, const float *kpos,
                          const float *krot, const float *ms, const float *f0, const float *qref,
                          const int *hinge_q, const float *rpos, const float *rrot, bf16 *X,
                          float *obs_out) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= (long long)n * n_in) return;
  const int p = (int)(tid / n_in);
  int i = (int)(tid % n_in);
  const int col = i;
  float v = 0.0f;
  const float *qp = q + (size_t)p * nq;
  const size_t mb = (size_t)n * n_mus;
  if (i < nv) {
    if (!free_root || i < 3) {
      v = qp[i];
    } else if (i < 6) {
      float w = qp[3], x = qp[4], y = qp[5], z = qp[6];
      if (w < 0.0f) { w = -w; x = -x; y = -y; z = -z; }
      const float sn = sqrtf(x * x + y * y + z * z);
      const float sc = sn > 1e-12f ? 2.0f * atan2f(sn, w) / sn : 2.0f;
      v = (i == 3 ? x : i == 4 ? y : z) * sc;
    } else {
      v = qp[i + 1];
    }
  } else if ((i -= nv) < nv) {
    v = qd[(size_t)p * nv + i];
  } else if ((i -= nv) < 3 * n_key) {
    v = kpos[(size_t)p * 3 * n_key + i];
  } else if ((i -= 3 * n_key) < 6 * n_key) {
    const int k = i / 6, c = i % 6;
    v = krot[((size_t)p * n_key + k) * 9 + 3 * (c % 3) + c / 3];
  } else if ((i -= 6 * n_key) < 4 * n_mus) {
    const int blk = i / n_mus, mx = i % n_mus;
    v = ms[blk * mb + (size_t)p * n_mus + mx];
    if (blk == 1) v /= f0[mx];
  } else if ((i -= 4 * n_mus) < n_h) {
    v = qref[(size_t)p * nq + hinge_q[i]];
  } else if ((i -= n_h) < 3 * n_key) {
    v = rpos[(size_t)p * 3 * n_key + i];
  } else if ((i -= 3 * n_key) < 6 * n_key) {
    const int k = i / 6, c = i % 6;
    v = rrot[((size_t)p * n_key + k) * 9 + 3 * (c % 3) + c / 3];
  }
  X[tid] = __float2bfloat16(v);
  if (obs_out && col < n_obs) obs_out[(size_t)p * n_obs + col] = v;
}

// a0 = mu + exp(log_std) xi, xi a standard normal by the Box-Muller
// transform of two 24-bit uniforms u1 = (i1 + 1/2) 2^-24, u2 = (i2 + 1/2)
// 2^-24 from z = SplitMix64(K ^ m), i1 = z >> 40, i2 = (z >> 16) & 0xFFFFFF,
// K = SplitMix64(SplitMix64(seed ^ env) ^ step): xi = sqrt(-2 ln u1) cos(2 pi u2);
// a has row stride lda
__global__ void k_gauss(int n, int n_mus, const float *mu, const float *log_std,
                        unsigned long long seed, long long env0, long long step, float *a, int lda) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n_mus) return;
  const int p = (int)(i / n_mus), mx = (int)(i % n_mus);
  const unsigned long long K =
      splitmix64(splitmix64(seed ^ (unsigned long long)(env0 + p)) ^ (unsigned long long)step);
  const unsigned long long z = splitmix64(K ^ (unsigned long long)mx);
  const float u1 = ((float)(unsigned)(z >> 40) + 0.5f) * 5.9604644775390625e-8f;
  const float u2 = ((float)(unsigned)((z >> 16) & 0xFFFFFFull) + 0.5f) * 5.9604644775390625e-8f;
  const float xi = sqrtf(-2.0f * logf(u1)) * cosf(6.28318530717958647692f * u2);
  a[(size_t)p * lda + mx] = mu[i] + expf(log_std[mx]) * xi;
}

// The flow network's (action, time) input block XA = [a, 0, 0 ...] (n_at):
// the time column stays zero, its contribution enters flow layer 1 as a
// per-step bias (k_flow_bias)
__global__ void k_pack_at(int n, int n_mus, int n_at, const float *a, bf16 *XA) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n_at) return;
  const int c = (int)(i % n_at);
  XA[i] = __float2bfloat16(c < n_mus ? a[i] : 0.0f);
}

// TB[k][j] = bf16(t_k) Wat[j][n_mus], t_k = k h: the time column of flow
// layer 1 at flow step k (the product the matrix core would form from the
// bfloat16 time input); HB3[c] = h b3[c], so that the output layer's
// epilogue h acc + h b3 + a is one explicit Euler step a + h psi
__global__ void k_flow_bias(int flow_steps, int hidden, int n_mus, int n_at, float h,
                            const bf16 *Wat, const float *b3, float *TB, float *HB3) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < flow_steps * hidden) {
    const int k = i / hidden, j = i % hidden;
    const float tk = __bfloat162float(__float2bfloat16((float)k * h));
    TB[i] = tk * __bfloat162float(Wat[(size_t)j * n_at + n_mus]);
  }
  if (i < n_mus) HB3[i] = h * b3[i];
}

// u = clamp(a, 0, 1) (a with row stride lda, u contiguous)
__global__ void k_clamp01(int n, int n_mus, int lda, const float *a, float *u, float *u_out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n_mus) return;
  const int p = (int)(i / n_mus), c = (int)(i % n_mus);
  const float v = fminf(fmaxf(a[(size_t)p * lda + c], 0.0f), 1.0f);
  u[i] = v;
  if (u_out) u_out[i] = v;
}

// tracking error [q_h - q_ref_h (n_h), key positions - reference key
// positions (3 n_key), 0 ...] (n_din)
__global__ void k_delta(int n, int nq, int n_h, int n_key, int n_din, const float *q,
                        const float *qref, const int *hinge_q, const float *kpos,
                        const float *rpos, bf16 *XD, float *delta_out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)n * n_din) return;
  const int p = (int)(i / n_din), c = (int)(i % n_din);
  float v = 0.0f;
  if (c < n_h) {
    const int j = hinge_q[c];
    v = q[(size_t)p * nq + j] - qref[(size_t)p * nq + j];
  } else if (c < n_h + 3 * n_key) {
    const size_t o = (size_t)p * 3 * n_key + (c - n_h);
    v = kpos[o] - rpos[o];
  }
  XD[i] = __float2bfloat16(v);
  if (delta_out && c < n_h + 3 * n_key) delta_out[(size_t)p * (n_h + 3 * n_key) + c] = v;
}

// r = -log(1 - sigmoid(z)) = softplus(z), computed stably
__global__ void k_reward(int n, const float *z, float *r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float x = z[i];
  r[i] = fmaxf(x, 0.0f) + log1pf(expf(-fabsf(x)));
}

template <class T>
T *calloc_dev(ms_controller *c, size_t n) {
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) return nullptr;
  if (hipMemset(p, 0, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    (void)hipFree(p);
    return nullptr;
  }
  c->owned.push_back(p);
  return (T *)p;
}

// weights of one network: in (padded) -> h -> h -> out; `used` inputs
bool make_net(ms_controller *c, Net &net, int in, int used, int h, int out,
              unsigned long long seed) {
  net.in = in;
  net.h = h;
  net.out = out;
  const int ins[3] = {in, h, h}, outs[3] = {h, h, out}, fan[3] = {used, h, h};
  for (int l = 0; l < 3; ++l) {
    const size_t nw = (size_t)ins[l] * outs[l];
    net.W[l] = calloc_dev<float>(c, nw);
    net.Wb[l] = calloc_dev<bf16>(c, nw);
    net.b[l] = calloc_dev<float>(c, outs[l]);
    if (!net.W[l] || !net.Wb[l] || !net.b[l]) return false;
    hipLaunchKernelGGL(k_init_w, dim3(blocks((long long)nw)), dim3(256), 0, 0, net.W[l], net.Wb[l],
                       outs[l], ins[l], l == 0 ? used : ins[l], fan[l],
                       seed * 3ull + (unsigned long long)l);
  }
  return true;
}

// hidden layers of a network on X (rows n, K = net.in) into H2
hipError_t hidden_layers(const ms_controller *c, const Net &net, int n, const bf16 *X,
                         hipStream_t st) {
  GemmEpi e1;
  e1.bias = net.b[0];
  e1.act = 1;
  e1.c_bf16 = c->H1;
  e1.ldc = net.h;
  hipError_t e = gemm_bf16(n, net.h, net.in, X, net.in, net.Wb[0], net.in, e1, st);
  if (e != hipSuccess) return e;
  GemmEpi e2;
  e2.bias = net.b[1];
  e2.act = 1;
  e2.c_bf16 = c->H2;
  e2.ldc = net.h;
  return gemm_bf16(n, net.h, net.h, c->H1, net.h, net.Wb[1], net.h, e2, st);
}

// output layer (linear) of a network from H2 into out[n][net.out]
hipError_t output_layer(const ms_controller *c, const Net &net, int n, float *out,
                        hipStream_t st) {
  GemmEpi e3;
  e3.bias = net.b[2];
  e3.c_f32 = out;
  e3.ldc = net.out;
  return gemm_bf16(n, net.out, net.h, c->H2, net.h, net.Wb[2], net.h, e3, st);
}

ms_status ctl_cap(ms_controller *c, int n) {
  if (n <= c->cap) return MS_OK;
  const size_t B = (size_t)n;
  std::vector<std::pair<void **, size_t>> want = {
      {(void **)&c->X, B * c->n_in * 2},      {(void **)&c->H1, B * c->hidden * 2},
      {(void **)&c->H2, B * c->hidden * 2},   {(void **)&c->XA, B * c->n_at * 2},
      {(void **)&c->XD, B * c->n_din * 2},    {(void **)&c->P, B * c->hidden * 4},
      {(void **)&c->A, B * c->n_at * 4},      {(void **)&c->PSI, B * c->n_mus * 4},
      {(void **)&c->U, B * c->n_mus * 4},     {(void **)&c->Z, B * 4},
      {(void **)&c->qref, B * c->nq * 4},     {(void **)&c->kpos, B * c->n_key * 12},
      {(void **)&c->krot, B * c->n_key * 36}, {(void **)&c->rpos, B * c->n_key * 12},
      {(void **)&c->rrot, B * c->n_key * 36}};
  std::vector<void *> got(want.size(), nullptr);
  for (size_t i = 0; i < want.size(); ++i) {
    if (hipMalloc(&got[i], std::max<size_t>(want[i].second, 4)) != hipSuccess) {
      for (size_t j = 0; j < i; ++j) (void)hipFree(got[j]);
      return cfail(MS_E_ALLOC, "controller workspace allocation failed");
    }
  }
  for (size_t i = 0; i < want.size(); ++i) {
    *want[i].first = got[i];
    c->owned.push_back(got[i]);
  }
  c->cap = n;
  return MS_OK;
}

// key frames of the state q (into kpos, krot) and of the reference pose
// qref (into rpos, rrot), one launch
hipError_t key_frames(const ms_controller *c, int n, const float *q, hipStream_t st) {
  const KModel &M = c->m->k;
  const size_t lds = 4 * (size_t)(12 * M.n_node + 6 * M.nv + 12 * M.n_node + M.nq + M.nv);
  hipLaunchKernelGGL(k_key_frames, dim3(2 * n), dim3(64), lds, st, M, n, c->key_node, c->n_key, q,
                     c->kpos, c->krot, (const float *)c->qref, c->rpos, c->rrot);
  return hipGetLastError();
}

}  // namespace
}  // namespace ms

using namespace ms;

extern "C" {

const char *ms_controller_last_error(void) { return c_err.c_str(); }

ms_status ms_controller_create(ms_model *m, const ms_controller_desc *d, ms_controller **out) {
  c_err.clear();
  if (!m || !d || !out) return cfail(MS_E_ARG, "NULL argument");
  *out = nullptr;
  if (d->hidden <= 0 || d->hidden % 8 || d->n_sub < 1 || d->flow_steps < 0 ||
      !(d->flow_dt >= 0.0f) || !(d->sigma0 > 0.0f) || d->n_key < 0 || d->n_key > 64 ||
      (d->n_key > 0 && !d->key_nodes))
    return cfail(MS_E_ARG, "bad controller description");
  const Tables &t = m->t;
  for (int k = 0; k < d->n_key; ++k)
    if (d->key_nodes[k] < 0 || d->key_nodes[k] >= t.n_node)
      return cfail(MS_E_ARG, "key node out of range");
  ms_controller *c = new ms_controller();
  c->m = m;
  c->nq = t.nq;
  c->nv = t.nv;
  c->n_mus = t.n_mus;
  c->free_root = t.free_root;
  c->n_key = d->n_key;
  c->hidden = d->hidden;
  c->n_sub = d->n_sub;
  c->flow_steps = d->flow_steps;
  c->flow_dt = d->flow_dt;
  c->ref_seed = d->ref_seed;
  c->noise_seed = d->noise_seed;
  std::vector<int> q_hinge(t.nq, -1), hinge_q;
  for (int i = 0; i < t.n_node; ++i)
    if (t.jtype[i] != 2) {
      q_hinge[t.qadr[i]] = (int)hinge_q.size();
      hinge_q.push_back(t.qadr[i]);
    }
  c->n_h = (int)hinge_q.size();
  c->n_obs = 2 * t.nv + 9 * c->n_key + 4 * t.n_mus + c->n_h + 9 * c->n_key;
  c->n_in = pad16(c->n_obs);
  c->n_at = pad16(t.n_mus + 1);
  c->n_din = pad16(c->n_h + 3 * c->n_key);
  std::vector<float> f0(t.n_mus);
  for (int mx = 0; mx < t.n_mus; ++mx) f0[mx] = t.mus_f0[t.mus_int[mx]];
  c->key_node = calloc_dev<int>(c, c->n_key);
  c->q_hinge = calloc_dev<int>(c, t.nq);
  c->hinge_q = calloc_dev<int>(c, c->n_h);
  c->f0 = calloc_dev<float>(c, t.n_mus);
  c->log_std = calloc_dev<float>(c, t.n_mus);
  bool ok = c->key_node && c->q_hinge && c->hinge_q && c->f0 && c->log_std;
  ok = ok && make_net(c, c->pi, c->n_in, c->n_obs, c->hidden, t.n_mus, d->pi_seed);
  // the flow network: input [observation (n_in) | action, time (n_at)];
  // its first layer is kept as the two column blocks
  ok = ok && make_net(c, c->flow, c->n_in, c->n_obs, c->hidden, t.n_mus, d->flow_seed);
  ok = ok && make_net(c, c->disc, c->n_din, c->n_h + 3 * c->n_key, c->hidden, 1, d->disc_seed);
  c->TB = ok ? calloc_dev<float>(c, (size_t)std::max(c->flow_steps, 1) * c->hidden) : nullptr;
  c->HB3 = ok ? calloc_dev<float>(c, (size_t)t.n_mus) : nullptr;
  ok = ok && c->TB && c->HB3;
  float *wat = ok ? calloc_dev<float>(c, (size_t)c->hidden * c->n_at) : nullptr;
  c->Wat = ok ? calloc_dev<bf16>(c, (size_t)c->hidden * c->n_at) : nullptr;
  hipError_t e = hipSuccess;
  if (ok && wat && c->Wat) {
    // fan-in of the whole first layer: observation and (action, time) inputs
    const int fan = c->n_obs + t.n_mus + 1;
    hipLaunchKernelGGL(k_init_w, dim3(blocks((long long)c->hidden * c->n_at)), dim3(256), 0, 0, wat,
                       c->Wat, c->hidden, c->n_at, t.n_mus + 1, fan,
                       d->flow_seed * 3ull + 7ull);
    hipLaunchKernelGGL(k_init_w, dim3(blocks((long long)c->hidden * c->n_in)), dim3(256), 0, 0,
                       c->flow.W[0], c->flow.Wb[0], c->hidden, c->n_in, c->n_obs, fan,
                       d->flow_seed * 3ull);
    hipLaunchKernelGGL(k_fill, dim3(blocks(t.n_mus)), dim3(256), 0, 0, c->log_std, t.n_mus,
                       std::log(d->sigma0));
    e = hipMemcpy(c->key_node, d->key_nodes, 4 * (size_t)c->n_key, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->q_hinge, q_hinge.data(), 4 * (size_t)t.nq, hipMemcpyHostToDevice);
    if (e == hipSuccess)
      e = hipMemcpy(c->hinge_q, hinge_q.data(), 4 * (size_t)c->n_h, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(c->f0, f0.data(), 4 * (size_t)t.n_mus, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipDeviceSynchronize();
  } else {
    ok = false;
  }
  if (!ok || e != hipSuccess) {
    ms_controller_destroy(c);
    return ok ? chip(e, "controller setup") : cfail(MS_E_ALLOC, "controller allocation failed");
  }
  *out = c;
  return MS_OK;
}

void ms_controller_destroy(ms_controller *c) {
  if (!c) return;
  for (void *p : c->owned) (void)hipFree(p);
  delete c;
}

ms_status ms_controller_dims(const ms_controller *c, int32_t *dims) {
  if (!c || !dims) return cfail(MS_E_ARG, "NULL argument");
  dims[0] = c->n_obs;
  dims[1] = c->n_in;
  dims[2] = c->n_at;
  dims[3] = c->n_din;
  dims[4] = c->hidden;
  dims[5] = c->n_h;
  return MS_OK;
}

ms_status ms_controller_params(ms_controller *c, int32_t which, int32_t set, float **W, float **b,
                               float *w_at, float *log_std) {
  c_err.clear();
  if (!c || which < 0 || which > 2 || !W || !b) return cfail(MS_E_ARG, "bad arguments");
  Net &net = which == 0 ? c->pi : which == 1 ? c->flow : c->disc;
  const int ins[3] = {net.in, net.h, net.h}, outs[3] = {net.h, net.h, net.out};
  hipError_t e = hipDeviceSynchronize();
  for (int l = 0; l < 3 && e == hipSuccess; ++l) {
    const size_t nw = (size_t)ins[l] * outs[l];
    if (!W[l] || !b[l]) return cfail(MS_E_ARG, "NULL parameter buffer");
    if (set) {
      e = hipMemcpy(net.W[l], W[l], 4 * nw, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = hipMemcpy(net.b[l], b[l], 4 * (size_t)outs[l], hipMemcpyHostToDevice);
    } else {
      e = hipMemcpy(W[l], net.W[l], 4 * nw, hipMemcpyDeviceToHost);
      if (e == hipSuccess) e = hipMemcpy(b[l], net.b[l], 4 * (size_t)outs[l], hipMemcpyDeviceToHost);
    }
  }
  if (e != hipSuccess) return chip(e, "controller params");
  if (set) {
    // bfloat16 copies of the set weights
    for (int l = 0; l < 3; ++l) {
      const size_t nw = (size_t)ins[l] * outs[l];
      std::vector<bf16> hb(nw);
      for (size_t i = 0; i < nw; ++i) hb[i] = __float2bfloat16(W[l][i]);
      e = hipMemcpy(net.Wb[l], hb.data(), 2 * nw, hipMemcpyHostToDevice);
      if (e != hipSuccess) return chip(e, "controller params");
    }
  }
  if (which == 1 && w_at) {
    const size_t nw = (size_t)c->hidden * c->n_at;
    if (set) {
      std::vector<bf16> hb(nw);
      for (size_t i = 0; i < nw; ++i) hb[i] = __float2bfloat16(w_at[i]);
      e = hipMemcpy(c->Wat, hb.data(), 2 * nw, hipMemcpyHostToDevice);
    } else {
      std::vector<bf16> hb(nw);
      e = hipMemcpy(hb.data(), c->Wat, 2 * nw, hipMemcpyDeviceToHost);
      for (size_t i = 0; i < nw; ++i) w_at[i] = __bfloat162float(hb[i]);
    }
    if (e != hipSuccess) return chip(e, "controller params");
  }
  if (which == 0 && log_std) {
    e = set ? hipMemcpy(c->log_std, log_std, 4 * (size_t)c->n_mus, hipMemcpyHostToDevice)
            : hipMemcpy(log_std, c->log_std, 4 * (size_t)c->n_mus, hipMemcpyDeviceToHost);
    if (e != hipSuccess) return chip(e, "controller params");
  }
  return MS_OK;
}

ms_status ms_controller_reserve(ms_controller *c, int32_t n_env) {
  c_err.clear();
  if (!c || n_env <= 0) return cfail(MS_E_ARG, "bad arguments");
  ms_status s = ctl_cap(c, n_env);
  if (s != MS_OK) return s;
  if (ms_model_reserve(c->m, n_env) != MS_OK)
    return cfail(MS_E_ALLOC, std::string("model workspace: ") + ms_last_error());
  return MS_OK;
}

ms_status ms_controller_step(ms_controller *c, int32_t n_env, float *q, float *qd, float *act,
                             uint32_t *status, float *mstate, int64_t ctl_step, double t,
                             const ms_step_opts *opts, const float *u_in, float *reward,
                             const ms_ctl_out *out, void *stream) {
  c_err.clear();
  if (!c || n_env <= 0 || !q || !qd || !act || !mstate || !opts || !reward)
    return cfail(MS_E_ARG, "NULL argument or n_env <= 0");
  if (!(opts->dt > 0.0f) || !std::isfinite(opts->dt)) return cfail(MS_E_ARG, "dt must be positive");
  hipStream_t st = (hipStream_t)stream;
  ms_status s = ctl_cap(c, n_env);
  if (s != MS_OK) return s;
  const int n = n_env, nm = c->n_mus;
  const long long nmu = (long long)n * nm;
  float *o_obs = out ? out->obs : nullptr;
  // 1. observation at time t
  hipLaunchKernelGGL(k_ref_pose, dim3(blocks((long long)n * c->nq)), dim3(256), 0, st, n, c->nq, q,
                     c->q_hinge, c->ref_seed, 0ll, (float)t, c->qref);
  hipError_t e = key_frames(c, n, q, st);
  if (e != hipSuccess) return chip(e, "key frames");
  hipLaunchKernelGGL(k_ctl_obs, dim3(blocks((long long)n * c->n_in)), dim3(256), 0, st, n, c->nq,
                     c->nv, c->free_root, nm, c->n_key, c->n_h, c->n_obs, c->n_in, q, qd, c->kpos,
                     c->krot, mstate, c->f0, c->qref, c->hinge_q, c->rpos, c->rrot, c->X, o_obs);
  // 2. excitations: Gaussian initial sample refined along the flow, or given
  const float *u = u_in;
  if (!u_in) {
    e = hidden_layers(c, c->pi, n, c->X, st);
    if (e == hipSuccess) e = output_layer(c, c->pi, n, c->PSI, st);  // mean, in PSI
    if (e != hipSuccess) return chip(e, "initial sampler");
    hipLaunchKernelGGL(k_gauss, dim3(blocks(nmu)), dim3(256), 0, st, n, nm, c->PSI, c->log_std,
                       c->noise_seed, 0ll, (long long)ctl_step, c->A, c->n_at);
    if (out && out->a0)
      (void)hipMemcpy2DAsync(out->a0, 4 * (size_t)nm, c->A, 4 * (size_t)c->n_at, 4 * (size_t)nm,
                             n, hipMemcpyDeviceToDevice, st);
    // observation block of the flow's first layer, once: P = W1_s s + b1
    GemmEpi ep;
    ep.bias = c->flow.b[0];
    ep.c_f32 = c->P;
    ep.ldc = c->hidden;
    e = gemm_bf16(n, c->hidden, c->n_in, c->X, c->n_in, c->flow.Wb[0], c->n_in, ep, st);
    if (e != hipSuccess) return chip(e, "flow layer 1");
    if (c->flow_steps > 0) {
      const int nb = std::max(c->flow_steps * c->hidden, nm);
      hipLaunchKernelGGL(k_flow_bias, dim3(blocks(nb)), dim3(256), 0, st, c->flow_steps, c->hidden,
                         nm, c->n_at, c->flow_dt, c->Wat, c->flow.b[2], c->TB, c->HB3);
      hipLaunchKernelGGL(k_pack_at, dim3(blocks((long long)n * c->n_at)), dim3(256), 0, st, n, nm,
                         c->n_at, c->A, c->XA);
    }
    for (int k = 0; k < c->flow_steps; ++k) {
      // psi(a, t_k, s) through the flow network; its output layer's
      // epilogue takes the Euler step a += h psi in place and writes the
      // next step's bfloat16 input beside it
      GemmEpi e1;
      e1.addc = c->P;
      e1.bias = c->TB + (size_t)k * c->hidden;
      e1.act = 1;
      e1.c_bf16 = c->H1;
      e1.ldc = c->hidden;
      e = gemm_bf16(n, c->hidden, c->n_at, c->XA, c->n_at, c->Wat, c->n_at, e1, st);
      GemmEpi e2;
      e2.bias = c->flow.b[1];
      e2.act = 1;
      e2.c_bf16 = c->H2;
      e2.ldc = c->hidden;
      if (e == hipSuccess)
        e = gemm_bf16(n, c->hidden, c->hidden, c->H1, c->hidden, c->flow.Wb[1],
                      c->hidden, e2, st);
      GemmEpi e3;
      e3.alpha = c->flow_dt;
      e3.bias = c->HB3;
      e3.addc = c->A;
      e3.c_f32 = c->A;
      e3.c_bf16 = c->XA;
      e3.ldc = c->n_at;
      if (e == hipSuccess)
        e = gemm_bf16(n, nm, c->hidden, c->H2, c->hidden, c->flow.Wb[2], c->hidden, e3, st);
      if (e != hipSuccess) return chip(e, "flow step");
    }
    hipLaunchKernelGGL(k_clamp01, dim3(blocks(nmu)), dim3(256), 0, st, n, nm, c->n_at, c->A, c->U,
                       out ? out->u : nullptr);
    u = c->U;
  }
  e = hipGetLastError();
  if (e != hipSuccess) return chip(e, "policy kernels");
  // 3. n_sub substeps with the excitations held; the last one records the
  // muscle state the next observation reads
  KRun r{};
  r.q = q; r.qd = qd; r.act = act; r.status = status; r.n_env = n;
  r.dt = opts->dt; r.contact = opts->contact;
  r.u = u; r.u_hold = 1; r.exc = MS_EXC_ARRAY;
  r.n_applied = out ? out->n_applied : nullptr;
  if (c->n_sub > 1) {
    s = run_steps(c->m, r, n, c->n_sub - 1, st);
    if (s != MS_OK) return cfail(s, std::string("substeps: ") + ms_last_error());
  }
  r.rec_every = 1;
  r.r_act = mstate;
  r.r_F = mstate + nmu;
  r.r_lm = mstate + 2 * nmu;
  r.r_vm = mstate + 3 * nmu;
  s = run_steps(c->m, r, n, 1, st);
  if (s != MS_OK) return cfail(s, std::string("substeps: ") + ms_last_error());
  // 4. reward on the tracking error at the end of the control step
  const float t1 = (float)(t + (double)c->n_sub * opts->dt);
  hipLaunchKernelGGL(k_ref_pose, dim3(blocks((long long)n * c->nq)), dim3(256), 0, st, n, c->nq, q,
                     c->q_hinge, c->ref_seed, 0ll, t1, c->qref);
  e = key_frames(c, n, q, st);
  if (e != hipSuccess) return chip(e, "key frames");
  hipLaunchKernelGGL(k_delta, dim3(blocks((long long)n * c->n_din)), dim3(256), 0, st, n, c->nq,
                     c->n_h, c->n_key, c->n_din, q, c->qref, c->hinge_q, c->kpos, c->rpos, c->XD,
                     out ? out->delta : nullptr);
  e = hidden_layers(c, c->disc, n, c->XD, st);
  if (e == hipSuccess) e = output_layer(c, c->disc, n, c->Z, st);
  if (e != hipSuccess) return chip(e, "discriminator");
  hipLaunchKernelGGL(k_reward, dim3(blocks(n)), dim3(256), 0, st, n, c->Z, reward);
  return chip(hipGetLastError(), "reward");
}

}  // extern "C"
