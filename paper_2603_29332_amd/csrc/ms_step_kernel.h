// ms_step_kernel.h -- the batched musculoskeletal forward-dynamics step on gfx950.
//
// The step's stages as device functions, composed two ways:
//  - the fused step (k_step): one wavefront (64 lanes) advances one
//    environment through whole rollouts with its kinematic tree (node
//    frames, motion subspaces, spatial velocities and accelerations),
//    contact state and tree-sparse FP64 mass matrix in LDS;
//  - the split step: per physics step a kinematics/dynamics kernel (one
//    wavefront per env), a muscle kernel (one 256-thread workgroup per env)
//    and a factorisation kernel (one wavefront per env), exchanging per-env
//    intermediates through a device workspace; each kernel's smaller LDS
//    block keeps more envs resident per CU. Both compositions perform the
//    same operations in the same order, so their results are identical.
// Muscle work is spread over a team's threads (thread t owns muscles t,
// t + n, ...), tree work over nodes/DoFs, and the LTDL factorisation over
// the entries of each height level.
//
// All spatial quantities are expressed in world axes about a reference point
// O that is the root origin of a floating model (the world origin for a
// fixed base), so subtree sums (composite inertias, net forces) are plain
// sums. FP32 throughout except the mass matrix assembly, its factorisation
// and the solve, which run in FP64.
#pragma once
#include <hip/hip_runtime.h>

#include <cmath>

#include "ms_step_types.h"

namespace ms {

// ------------------------------------------------------------ small maths
struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(float s, V3 a) { return v3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// y = R x, R row-major 3x3
__device__ __forceinline__ V3 mulR(const float *R, V3 x) {
  return v3(R[0] * x.x + R[1] * x.y + R[2] * x.z, R[3] * x.x + R[4] * x.y + R[5] * x.z,
            R[6] * x.x + R[7] * x.y + R[8] * x.z);
}
__device__ __forceinline__ V3 ld3(const float *p) { return v3(p[0], p[1], p[2]); }
__device__ __forceinline__ void st3(float *p, V3 a) {
  p[0] = a.x;
  p[1] = a.y;
  p[2] = a.z;
}

// Apply node frame F (12 floats, 16-byte aligned: R row-major, then P) to
// a local point: three 128-bit LDS reads.
__device__ __forceinline__ V3 frame_apply(const float *F, V3 x) {
  const float4 a = *(const float4 *)F, b = *(const float4 *)(F + 4), c = *(const float4 *)(F + 8);
  return v3(a.x * x.x + a.y * x.y + a.z * x.z + c.y, a.w * x.x + b.x * x.y + b.y * x.z + c.z,
            b.z * x.x + b.w * x.y + c.x * x.z + c.w);
}

// SplitMix64 output function (Steele, Lea & Flood 2014).
__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ float u24(unsigned long long z, int shift) {
  return (float)((unsigned)((z >> shift) & 0xFFFFFFull)) * 5.9604644775390625e-8f;
}

// One step of the smooth-noise excitation for muscle mi: four 24-bit
// uniforms from two SplitMix64 draws, their sum standardised
// (Irwin-Hall(4): mean 2, variance 1/3), x <- rho x + s xi,
// u = clamp(mean + x, 0, 1). Each operation is rounded to float32 in this
// order: no contraction into fused multiply-adds.
struct AR1 {
  float u, x;
};
__device__ __forceinline__ AR1 ar1_step(unsigned long long key, int mi, float x, float rho, float s,
                                        float mean) {
#pragma clang fp contract(off)
  const unsigned long long z1 = splitmix64(key ^ (2ull * (unsigned long long)mi));
  const unsigned long long z2 = splitmix64(key ^ (2ull * (unsigned long long)mi + 1ull));
  const float t = ((u24(z1, 40) + u24(z1, 16)) + u24(z2, 40)) + u24(z2, 16);
  const float xi = (t - 2.0f) * 1.7320508075688772f;
  const float a = rho * x;
  const float b = s * xi;
  const float xn = a + b;
  return AR1{fminf(fmaxf(mean + xn, 0.0f), 1.0f), xn};
}

// Hill curves: Gaussian active force-length, exponential passive
// force-length with a linear tail past 1.6, hyperbolic force-velocity.
// The curves use the hardware exponential (a few ulp), far inside the
// step's error bound.
__device__ __forceinline__ float hill_fl(float lm) {
  float d = lm - 1.0f;
  return __expf(-d * d * (1.0f / 0.45f));
}
__device__ __forceinline__ float hill_fp(float lm) {
  const float e4m1 = 53.598150033144236f;  // e^4 - 1
  if (lm <= 1.0f) return 0.0f;
  if (lm <= 1.6f) return (__expf((4.0f / 0.6f) * (lm - 1.0f)) - 1.0f) * (1.0f / e4m1);
  return 1.0f + 6.7910995f * (lm - 1.6f);  // slope (4/0.6) e^4/(e^4-1)
}
__device__ __forceinline__ float hill_fv(float vm) {
  if (vm <= -1.0f) return 0.0f;
  if (vm <= 0.0f) return (1.0f + vm) / (1.0f - 4.0f * vm);
  return 1.0f + 0.4f * vm / (vm + 0.08f);
}
__device__ __forceinline__ float hill_fv_slope(float vm) {
  if (vm <= -1.0f) return 0.0f;
  if (vm <= 0.0f) {
    float a = 1.0f - 4.0f * vm;
    return 5.0f / (a * a);
  }
  float b = vm + 0.08f;
  return 0.032f / (b * b);
}
// Slopes of f_l and f_p.
__device__ __forceinline__ float hill_fl_slope(float lm) {
  return -2.0f * (lm - 1.0f) * (1.0f / 0.45f) * hill_fl(lm);
}
__device__ __forceinline__ float hill_fp_slope(float lm) {
  const float e4m1 = 53.598150033144236f;  // e^4 - 1
  if (lm <= 1.0f) return 0.0f;
  if (lm <= 1.6f) return (4.0f / 0.6f) * __expf((4.0f / 0.6f) * (lm - 1.0f)) * (1.0f / e4m1);
  return 6.7910995f;
}
// The normalised fibre velocity v with A f_v(v) + beta v = R (A >= 0,
// beta > 0): the left-hand side rises from -beta at v = -1 to A at v = 0,
// so R picks the branch; on each hyperbola branch the balance is a
// quadratic in v, solved in the form that does not cancel near its small
// root.
__device__ __forceinline__ float hill_fv_root(float A, float R, float beta) {
  if (R <= -beta) return R / beta;  // f_v = 0 below v = -1
  if (R <= A) {
    // concentric: 4 beta v^2 - (A + beta + 4 R) v + (R - A) = 0, v in [-1, 0]
    const float b = A + beta + 4.0f * R;
    return 2.0f * (R - A) / (b + sqrtf(b * b + 16.0f * beta * (A - R)));
  }
  // eccentric: beta v^2 + (1.4 A + 0.08 beta - R) v - 0.08 (R - A) = 0, v > 0
  const float b = 1.4f * A + 0.08f * beta - R;
  return 0.16f * (R - A) / (b + sqrtf(b * b + 0.32f * beta * (R - A)));
}

// Value of v held by lane `src` (uniform), for every lane.
__device__ __forceinline__ double lane_bcast(double v, int src) {
  const unsigned long long b = __double_as_longlong(v);
  const unsigned lo = __builtin_amdgcn_readlane((unsigned)b, src);
  const unsigned hi = __builtin_amdgcn_readlane((unsigned)(b >> 32), src);
  return __longlong_as_double(((unsigned long long)hi << 32) | lo);
}

// Sum over the 64 lanes of a wavefront (butterfly exchange); every lane
// receives the total.
// Barrier and LDS ordering among the lanes of one wavefront (an env never
// waits for other wavefronts of its workgroup).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// log2 of the lanes per item when n items share a wavefront (n >= 1):
// the largest power of two P with n P <= 64
__device__ __forceinline__ int group_log2(int n) {
  int l = 0;
  while (l < 6 && (n << (l + 1)) <= 64) ++l;
  return l;
}

// A double moved across lanes by a DPP control (rows of 16 lanes; lanes with
// no source, or in rows outside ROWS, read 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Inclusive prefix sums within aligned groups of 2^lp lanes, in a fixed
// order (shift-and-add within rows of 16, then the row totals carried by
// row broadcasts); the group's total ends in its last lane.
__device__ __forceinline__ double group_sum_last(double v, int lp, int lane) {
  const int p = lane & ((1 << lp) - 1);
  double t;
  if (lp >= 1) { t = dpp_d<0x111, 0xF>(v); if (p >= 1) v += t; }   // row_shr:1
  if (lp >= 2) { t = dpp_d<0x112, 0xF>(v); if (p >= 2) v += t; }   // row_shr:2
  if (lp >= 3) { t = dpp_d<0x114, 0xF>(v); if (p >= 4) v += t; }   // row_shr:4
  if (lp >= 4) { t = dpp_d<0x118, 0xF>(v); if (p >= 8) v += t; }   // row_shr:8
  if (lp >= 5) { t = dpp_d<0x142, 0xA>(v); if (p >= 16) v += t; }  // row_bcast:15
  if (lp >= 6) { t = dpp_d<0x143, 0xC>(v); if (p >= 32) v += t; }  // row_bcast:31
  return v;
}

// Exact via-point geometry of muscle slot m: path length L, moment arms
// r[3] = -dL/dq of its span DoFs and Ldot. Path w_0..w_{P-1}; with unit
// segment vectors e_k, dL/dq_j = sum_k g_k . (a_j x (w_k - o_j)) over the
// via-points moved by hinge j (g_k = e_{k-1} - e_k), a_j . sum_k g_k for a
// slide. Pg bounds the via-point loops uniformly across the wavefront.
template <int NVIA>
__device__ __forceinline__ float muscle_geometry(const KModel &M, int m, int Pg, const float *Rl,
                                                 const float *Pl, const float *Sl, const float *qd,
                                                 V3 O, float r3[3], float &Ld) {
  const int nm = M.n_mus;
  const int P = M.mus_nvia[m];
  V3 w[NVIA], gk[NVIA];
#pragma unroll
  for (int k = 0; k < NVIA; ++k) {
    w[k] = v3(0.f, 0.f, 0.f);
    if (k < Pg && k < P) {
      const int b = M.via_node[(size_t)k * nm + m];
      V3 x = v3(M.via_pos[((size_t)k * 3 + 0) * nm + m], M.via_pos[((size_t)k * 3 + 1) * nm + m],
                M.via_pos[((size_t)k * 3 + 2) * nm + m]);
      w[k] = b >= 0 ? frame_apply(Rl + 12 * b, x) : x - O;
    }
  }
  float L = 0.f;
  V3 eprev = v3(0.f, 0.f, 0.f);
#pragma unroll
  for (int k = 0; k < NVIA; ++k) {
    gk[k] = v3(0.f, 0.f, 0.f);
    if (k < Pg) {
      if (k + 1 < P) {
        // segment length and unit vector from one hardware reciprocal
        // square root (about 1 ulp)
        V3 d = w[k + 1] - w[k];
        const float dd = dot(d, d), rl = __builtin_amdgcn_rsqf(dd);
        L += dd * rl;
        V3 e = rl * d;
        gk[k] = eprev - e;
        eprev = e;
      } else if (k + 1 == P) {
        gk[k] = eprev;
      }
    }
  }
  const unsigned mask = M.mus_mask[m];
  Ld = 0.f;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    r3[s] = 0.f;
    const int rec = M.mus_srec[s * nm + m];
    if (rec >= 0) {
      const int j = rec & 0xFF;
      const unsigned mk = (mask >> (8 * s)) & 0xFFu;
      const float *S = Sl + 6 * j;
      float dl;
      if ((rec >> 8) & 1) {
        V3 o = ld3(Pl + 12 * (rec >> 16));
        V3 acc = v3(0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < NVIA; ++k)
          if ((mk >> k) & 1u) acc = acc + cross(w[k] - o, gk[k]);
        dl = dot(ld3(S), acc);
      } else {
        V3 acc = v3(0.f, 0.f, 0.f);
#pragma unroll
        for (int k = 0; k < NVIA; ++k)
          if ((mk >> k) & 1u) acc = acc + gk[k];
        dl = dot(ld3(S + 3), acc);
      }
      r3[s] = -dl;
      Ld += dl * qd[j];
    }
  }
  return L;
}

// ------------------------------------------------------------ work teams
// The threads that share one env's work: a wavefront (the fused step, the
// kinematics/dynamics and the factorisation kernels) or a 256-thread
// workgroup (the muscle kernel). t is the thread's index in the team.
struct WaveTeam {
  int t;
  static constexpr int n = 64;
  __device__ __forceinline__ void sync() const { wave_sync(); }
  __device__ __forceinline__ bool any(bool v) const { return __any(v); }
};
struct BlockTeam {
  int t;
  static constexpr int n = 256;
  __device__ __forceinline__ void sync() const { __syncthreads(); }
  __device__ __forceinline__ bool any(bool v) const { return __syncthreads_or(v ? 1 : 0) != 0; }
};

// ------------------------------------------------------------ stages
// Forward kinematics, motion subspaces, spatial velocities V and bias
// accelerations A of every node. O = root origin (floating) or world origin
// (fixed base).
__device__ __forceinline__ void stage_fk(const KModel &M, int lane, const int *tlev, const int *tnode,
                                         const float *q, const float *qd, float *Rl, float *Sl,
                                         float *Vl, float *Al, V3 O, V3 g) {
  const int nn = M.n_node;
  // (1) every node's joint transform in parallel: rotation jrot Rot(axis, q)
  // and offset parked in the node's frame slot, the axis jrot*axis in its A
  // slot; the floating root is finished here
  for (int i = lane; i < nn; i += 64) {
    const int jt = M.jtype[i];
    float *F = Rl + 12 * i;
    const int da = M.dadr[i];
    if (jt == 2) {
      const float *x = q + M.qadr[i] + 3;
      float nrm = sqrtf(x[0] * x[0] + x[1] * x[1] + x[2] * x[2] + x[3] * x[3]);
      float w = x[0] / nrm, a = x[1] / nrm, b = x[2] / nrm, c = x[3] / nrm;
      float *R = F;
      R[0] = 1 - 2 * (b * b + c * c); R[1] = 2 * (a * b - w * c); R[2] = 2 * (a * c + w * b);
      R[3] = 2 * (a * b + w * c); R[4] = 1 - 2 * (a * a + c * c); R[5] = 2 * (b * c - w * a);
      R[6] = 2 * (a * c - w * b); R[7] = 2 * (b * c + w * a); R[8] = 1 - 2 * (a * a + b * b);
      st3(F + 9, v3(0.f, 0.f, 0.f));
      for (int kk = 0; kk < 3; ++kk) {
        float *S = Sl + 6 * (da + kk);
        S[0] = S[1] = S[2] = 0.f;
        S[3] = kk == 0; S[4] = kk == 1; S[5] = kk == 2;
        float *S2 = Sl + 6 * (da + 3 + kk);
        S2[0] = R[kk]; S2[1] = R[3 + kk]; S2[2] = R[6 + kk];
        S2[3] = S2[4] = S2[5] = 0.f;
      }
      V3 v = ld3(qd + da);
      V3 ww = mulR(R, ld3(qd + da + 3));
      float *V = Vl + 6 * i, *A = Al + 6 * i;
      st3(V, ww);
      st3(V + 3, v);
      st3(A, v3(0.f, 0.f, 0.f));
      st3(A + 3, cross(v, ww) - g);
      continue;
    }
    const float *E = M.jrot + 9 * i;
    const V3 ax = ld3(M.axis + 3 * i);
    const float qi = q[M.qadr[i]];
    const V3 al = mulR(E, ax);
    V3 t = ld3(M.jpos + 3 * i);
    if (jt == 0) {
      float sn, cs;
      sincosf(qi, &sn, &cs);
      const float vc = 1.0f - cs;
      const float Q[9] = {cs + ax.x * ax.x * vc, ax.x * ax.y * vc - ax.z * sn, ax.x * ax.z * vc + ax.y * sn,
                          ax.y * ax.x * vc + ax.z * sn, cs + ax.y * ax.y * vc, ax.y * ax.z * vc - ax.x * sn,
                          ax.z * ax.x * vc - ax.y * sn, ax.z * ax.y * vc + ax.x * sn, cs + ax.z * ax.z * vc};
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          F[3 * r + c] = E[3 * r] * Q[c] + E[3 * r + 1] * Q[3 + c] + E[3 * r + 2] * Q[6 + c];
    } else {
      for (int e = 0; e < 9; ++e) F[e] = E[e];
      t = t + qi * al;
    }
    st3(F + 9, t);
    st3(Al + 6 * i, al);
  }
  wave_sync();
  // (2) compose down the tree level by level, reading only LDS:
  // R = R_p Lr, P = P_p + R_p t, axis = R_p al, S, V = V_p + S qd,
  // A = A_p + V_p x (S qd)
  for (int l = 0; l < M.n_level; ++l) {
    const int b0 = tlev[l], b1 = tlev[l + 1];
    for (int k = b0 + lane; k < b1; k += 64) {
      const int info = tnode[k], i = info >> 18;
      const int jt = info & 3;
      if (jt == 2) continue;
      const int p = (info >> 2 & 0xFF) - 1, da = info >> 10 & 0xFF;
      float *F = Rl + 12 * i;
      // frames are 16-byte aligned 12-float records, V and A 8-byte aligned
      // 6-float records: vector LDS accesses
      const float4 f0 = ((const float4 *)F)[0], f1 = ((const float4 *)F)[1],
                   f2 = ((const float4 *)F)[2];
      const float Lr[9] = {f0.x, f0.y, f0.z, f0.w, f1.x, f1.y, f1.z, f1.w, f2.x};
      const V3 t = v3(f2.y, f2.z, f2.w);
      const float2 a0 = ((const float2 *)(Al + 6 * i))[0], a1 = ((const float2 *)(Al + 6 * i))[1];
      const V3 al = v3(a0.x, a0.y, a1.x);
      float Rp[9];
      V3 Pp, wp, vp, ap, lp;
      if (p >= 0) {
        const float4 *P4 = (const float4 *)(Rl + 12 * p);
        const float4 r0 = P4[0], r1 = P4[1], r2 = P4[2];
        Rp[0] = r0.x; Rp[1] = r0.y; Rp[2] = r0.z; Rp[3] = r0.w; Rp[4] = r1.x; Rp[5] = r1.y;
        Rp[6] = r1.z; Rp[7] = r1.w; Rp[8] = r2.x;
        Pp = v3(r2.y, r2.z, r2.w);
        const float2 *V2 = (const float2 *)(Vl + 6 * p), *A2 = (const float2 *)(Al + 6 * p);
        const float2 v0 = V2[0], v1 = V2[1], v2 = V2[2], b0 = A2[0], b1 = A2[1], b2 = A2[2];
        wp = v3(v0.x, v0.y, v1.x); vp = v3(v1.y, v2.x, v2.y);
        ap = v3(b0.x, b0.y, b1.x); lp = v3(b1.y, b2.x, b2.y);
      } else {
        for (int e = 0; e < 9; ++e) Rp[e] = (e % 4 == 0) ? 1.f : 0.f;
        Pp = v3(0.f, 0.f, 0.f) - O;
        wp = vp = ap = v3(0.f, 0.f, 0.f);
        lp = v3(0.f, 0.f, 0.f) - g;
      }
      float Rn9[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
          Rn9[3 * r + c] = Rp[3 * r] * Lr[c] + Rp[3 * r + 1] * Lr[3 + c] + Rp[3 * r + 2] * Lr[6 + c];
      const V3 Pi = Pp + mulR(Rp, t);
      const V3 ah = mulR(Rp, al);
      ((float4 *)F)[0] = make_float4(Rn9[0], Rn9[1], Rn9[2], Rn9[3]);
      ((float4 *)F)[1] = make_float4(Rn9[4], Rn9[5], Rn9[6], Rn9[7]);
      ((float4 *)F)[2] = make_float4(Rn9[8], Pi.x, Pi.y, Pi.z);
      V3 sw, sv;
      if (jt == 0) {
        sw = ah;
        sv = cross(Pi, ah);
      } else {
        sw = v3(0.f, 0.f, 0.f);
        sv = ah;
      }
      float *S = Sl + 6 * da;
      st3(S, sw);
      st3(S + 3, sv);
      const float qdi = qd[da];
      const V3 xw = qdi * sw, xv = qdi * sv;  // S qd
      const V3 vw = wp + xw, vv = vp + xv;
      const V3 aw = ap + cross(wp, xw), av = lp + cross(wp, xv) + cross(vp, xw);
      float2 *V2 = (float2 *)(Vl + 6 * i), *A2 = (float2 *)(Al + 6 * i);
      V2[0] = make_float2(vw.x, vw.y); V2[1] = make_float2(vw.z, vv.x); V2[2] = make_float2(vv.y, vv.z);
      A2[0] = make_float2(aw.x, aw.y); A2[1] = make_float2(aw.z, av.x); A2[2] = make_float2(av.y, av.z);
    }
    wave_sync();
  }
}

// Penalty contact of every sphere: a record per sphere of 16 floats
// (active, contact point, wrench about O, force, friction and damping slopes).
__device__ __forceinline__ void stage_contacts(const KModel &M, int lane, const float *Rl,
                                               const float *Vl, float *Cl, V3 O, float dt,
                                               int contact) {
  for (int c = lane; c < M.n_con; c += 64) {
    float *C = Cl + 16 * c;
    const int b = M.con_node[c];
    V3 w = frame_apply(Rl + 12 * b, ld3(M.con_pos + 3 * c));
    const float rho = M.con_radius[c];
    const float pen = rho - (w.z + O.z);
    for (int e = 0; e < 16; ++e) C[e] = 0.f;
    if (contact && pen > 0.f) {
      V3 cp = w - v3(0.f, 0.f, rho);
      V3 vel = ld3(Vl + 6 * b + 3) + cross(ld3(Vl + 6 * b), cp);
      // spring taken linearly implicitly over the step: damping c + dt k
      const float ceff = M.cc + dt * M.kc;
      float fn = fmaxf(0.f, M.kc * pen - ceff * vel.z);
      float s2 = vel.x * vel.x + vel.y * vel.y + M.vs * M.vs;
      float s = sqrtf(s2);
      V3 f = v3(-M.mu * fn * vel.x / s, -M.mu * fn * vel.y / s, fn);
      C[0] = 1.f;
      st3(C + 1, cp);
      st3(C + 4, cross(cp, f));
      st3(C + 7, f);
      if (fn > 0.f) {
        float gg = M.mu * fn / s;
        C[10] = gg * (1.f - vel.x * vel.x / s2);
        C[11] = -gg * vel.x * vel.y / s2;
        C[12] = gg * (1.f - vel.y * vel.y / s2);
        C[13] = ceff;
      }
    }
  }
}

// Recursive Newton-Euler bias forces with the contact wrenches injected on
// the backward sum: rhs[j] = -(C - tau_ext)_j - b_j qd_j (o_bias, when
// given, receives C - tau_ext).
__device__ __forceinline__ void stage_rnea(const KModel &M, int lane, const float *Rl, const float *Pl,
                                           const float *Vl, const float *Al, float *Fl,
                                           const float *Cl, const float *Sl, const float *qd,
                                           const int *sbs, const unsigned char *sbl, const int *scs,
                                           const unsigned char *scl, double *rhs, float *o_bias) {
  const int nn = M.n_node, nv = M.nv;
  for (int b = lane; b < M.n_body; b += 64) {
    const int i = M.body_node[b];
    const float *R = Rl + 12 * i;
    const float m = M.body_mass[b];
    V3 c = mulR(R, ld3(M.body_com + 3 * b)) + ld3(Pl + 12 * i);
    V3 h = m * c;
    const float I0 = M.body_inertia[3 * b], I1 = M.body_inertia[3 * b + 1], I2 = M.body_inertia[3 * b + 2];
    // I_O = R diag(I) R^T + m (|c|^2 1 - c c^T)
    float Io[9];
    const float cc = dot(c, c);
    const float cv[3] = {c.x, c.y, c.z};
    for (int r = 0; r < 3; ++r)
      for (int s = 0; s < 3; ++s)
        Io[3 * r + s] = R[3 * r] * I0 * R[3 * s] + R[3 * r + 1] * I1 * R[3 * s + 1] +
                        R[3 * r + 2] * I2 * R[3 * s + 2] + m * ((r == s ? cc : 0.f) - cv[r] * cv[s]);
    V3 w = ld3(Vl + 6 * i), v = ld3(Vl + 6 * i + 3);
    V3 aw = ld3(Al + 6 * i), al = ld3(Al + 6 * i + 3);
    // I (w; v) = (I_O w + h x v; m v - h x w)
    V3 Iaw = mulR(Io, aw) + cross(h, al), Ial = m * al - cross(h, aw);
    V3 Ivw = mulR(Io, w) + cross(h, v), Ivl = m * v - cross(h, w);
    // f = I a + v x* (I v), (w, v) x* (n, f) = (w x n + v x f, w x f)
    V3 fw = Iaw + cross(w, Ivw) + cross(v, Ivl);
    V3 fl = Ial + cross(w, Ivl);
    st3(Fl + 6 * b, fw);
    st3(Fl + 6 * b + 3, fl);
  }
  wave_sync();
  float *Fn = Fl + 6 * M.n_body;
  for (int t = lane; t < 6 * nn; t += 64) {
    const int n = t / 6, k = t % 6;
    float s = 0.f;
    for (int e = sbs[n]; e < sbs[n + 1]; ++e) s += Fl[6 * sbl[e] + k];
    for (int e = scs[n]; e < scs[n + 1]; ++e) s -= Cl[16 * scl[e] + 4 + k];
    Fn[t] = s;
  }
  wave_sync();
  for (int j = lane; j < nv; j += 64) {
    const float *S = Sl + 6 * j;
    const float *F = Fn + 6 * M.dof_node[j];
    float cb = S[0] * F[0] + S[1] * F[1] + S[2] * F[2] + S[3] * F[3] + S[4] * F[4] + S[5] * F[5];
    if (o_bias) o_bias[j] = cb;
    rhs[j] = (double)(-cb - M.damping[j] * qd[j]);
  }
  wave_sync();
}

// Composite-rigid-body mass matrix in FP64 with the contacts' implicit
// damping, H[e] = S_i^T F_j for the stored entries e = (j, i) (H may be in
// LDS or device memory). dmp receives this lane's joint damping (DoFs lane,
// lane + 64), loaded early so that no entry waits on global memory.
__device__ __forceinline__ void stage_crba(const KModel &M, int lane, const int *LT, const float *Rl,
                                           const float *Pl, const float *Sl, const float *Cl,
                                           unsigned char *scr, float dt, double *H, float dmp[2]) {
  const int nv = M.nv;
  const int *sbs = LT + M.lt_subb_start, *scs = LT + M.lt_subc_start;
  const unsigned char *sbl = (const unsigned char *)(LT + M.lt_subb);
  const unsigned char *scl = (const unsigned char *)(LT + M.lt_subc);
  const unsigned char *cin = (const unsigned char *)(LT + M.lt_cinode);
  const unsigned char *dci = (const unsigned char *)(LT + M.lt_dofci);
  double *BI = (double *)scr;           // [n_body][10]: m, h, I_O (xx xy xz yy yz zz)
  double *CI = BI + 10 * M.n_body;      // [n_ci][10], one per distinct subtree body set
  double *FJ = CI + 10 * M.n_ci;        // [nv][6]
#pragma unroll
  for (int t = 0; t < 2; ++t) dmp[t] = lane + 64 * t < nv ? M.damping[lane + 64 * t] : 0.f;
  for (int b = lane; b < M.n_body; b += 64) {
    const int i = M.body_node[b];
    const float *R = Rl + 12 * i;
    const double m = M.body_mass[b];
    V3 cf = mulR(R, ld3(M.body_com + 3 * b)) + ld3(Pl + 12 * i);
    const double c[3] = {cf.x, cf.y, cf.z};
    const double In[3] = {M.body_inertia[3 * b], M.body_inertia[3 * b + 1], M.body_inertia[3 * b + 2]};
    double *o = BI + 10 * b;
    o[0] = m;
    o[1] = m * c[0]; o[2] = m * c[1]; o[3] = m * c[2];
    const double cc = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const int rr[6] = {0, 0, 0, 1, 1, 2}, ss[6] = {0, 1, 2, 1, 2, 2};
    for (int e = 0; e < 6; ++e) {
      int r = rr[e], s = ss[e];
      double v = (double)R[3 * r] * In[0] * R[3 * s] + (double)R[3 * r + 1] * In[1] * R[3 * s + 1] +
                 (double)R[3 * r + 2] * In[2] * R[3 * s + 2];
      o[4 + e] = v + m * ((r == s ? cc : 0.0) - c[r] * c[s]);
    }
  }
  wave_sync();
  for (int t = lane; t < 10 * M.n_ci; t += 64) {
    const int n = cin[t / 10], k = t % 10;
    double s = 0.0;
    for (int e = sbs[n]; e < sbs[n + 1]; ++e) s += BI[10 * sbl[e] + k];
    CI[t] = s;
  }
  wave_sync();
  for (int j = lane; j < nv; j += 64) {
    const int n = M.dof_node[j];
    const double *I = CI + 10 * dci[j];
    const float *Sf = Sl + 6 * j;
    const double w[3] = {Sf[0], Sf[1], Sf[2]}, v[3] = {Sf[3], Sf[4], Sf[5]};
    const double m = I[0], h[3] = {I[1], I[2], I[3]};
    const double Io[9] = {I[4], I[5], I[6], I[5], I[7], I[8], I[6], I[8], I[9]};
    double f[6];
    // (I_O w + h x v ; m v - h x w)
    f[0] = Io[0] * w[0] + Io[1] * w[1] + Io[2] * w[2] + (h[1] * v[2] - h[2] * v[1]);
    f[1] = Io[3] * w[0] + Io[4] * w[1] + Io[5] * w[2] + (h[2] * v[0] - h[0] * v[2]);
    f[2] = Io[6] * w[0] + Io[7] * w[1] + Io[8] * w[2] + (h[0] * v[1] - h[1] * v[0]);
    f[3] = m * v[0] - (h[1] * w[2] - h[2] * w[1]);
    f[4] = m * v[1] - (h[2] * w[0] - h[0] * w[2]);
    f[5] = m * v[2] - (h[0] * w[1] - h[1] * w[0]);
    // implicit contact damping: dt * Phi^T D Phi S for contacts below
    for (int e = scs[n]; e < scs[n + 1]; ++e) {
      const float *C = Cl + 16 * scl[e];
      if (C[0] == 0.f) continue;
      const double cp[3] = {C[1], C[2], C[3]};
      // point velocity of the contact for unit qd_j: v + w x cp
      const double J[3] = {v[0] + w[1] * cp[2] - w[2] * cp[1], v[1] + w[2] * cp[0] - w[0] * cp[2],
                           v[2] + w[0] * cp[1] - w[1] * cp[0]};
      const double u0 = (double)C[10] * J[0] + (double)C[11] * J[1];
      const double u1 = (double)C[11] * J[0] + (double)C[12] * J[1];
      const double u2 = (double)C[13] * J[2];
      const double dd = dt;
      f[0] += dd * (cp[1] * u2 - cp[2] * u1);
      f[1] += dd * (cp[2] * u0 - cp[0] * u2);
      f[2] += dd * (cp[0] * u1 - cp[1] * u0);
      f[3] += dd * u0;
      f[4] += dd * u1;
      f[5] += dd * u2;
    }
    for (int k = 0; k < 6; ++k) FJ[6 * j + k] = f[k];
  }
  wave_sync();
  const unsigned char *rowb = (const unsigned char *)(LT + M.lt_nnzrow);
  const unsigned char *pathb = (const unsigned char *)(LT + M.lt_path);
  for (int e = lane; e < M.nnz; e += 64) {
    const int j = rowb[e], i = pathb[e];
    const float *Sf = Sl + 6 * i;
    const double *f = FJ + 6 * j;
    double h = (double)Sf[0] * f[0] + (double)Sf[1] * f[1] + (double)Sf[2] * f[2] +
               (double)Sf[3] * f[3] + (double)Sf[4] * f[4] + (double)Sf[5] * f[5];
    H[e] = h;
  }
  wave_sync();
}

// H_jj += dt b_j on the diagonals (the last entry of row j), with this
// lane's damping values from stage_crba.
__device__ __forceinline__ void add_joint_damping(const KModel &M, int lane, const int *LT, double *H,
                                                  float dt, const float dmp[2]) {
  const int *rs = LT + M.lt_rs;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int j = lane + 64 * t;
    if (j < M.nv) H[rs[j + 1] - 1] += (double)dt * dmp[t];
  }
  wave_sync();
}

// Anatomical joint coupling as penalty equality constraints: with
// d_eff = d + dt k, rhs -= J^T (k phi(q) + d_eff J q') and H += dt d_eff
// J^T J (the spring linearly implicit, as the contact spring is).
// phi_c and (J q')_c in FP64 by lane c; the per-constraint force goes
// through scr (n_eq doubles), then each coupled DoF and each J^T J entry
// is one lane's (no two lanes write the same element).
__device__ __forceinline__ void add_coupling(const KModel &M, int lane, const float *q,
                                             const float *qd, double *H, double *rhs, double *scr,
                                             float dt) {
  if (!M.n_eq) return;
  const double deff = (double)M.eq_d + (double)dt * (double)M.eq_k;
  if (lane < M.n_eq) {
    double ph = -(double)M.eq_off[lane], jv = 0.0;
    for (int t = M.eq_start[lane]; t < M.eq_start[lane + 1]; ++t) {
      const double c = (double)M.eq_coef[t];
      ph += c * (double)q[M.eq_qi[t]];
      jv += c * (double)qd[M.eq_dof[t]];
    }
    scr[lane] = (double)M.eq_k * ph + deff * jv;
  }
  wave_sync();
  for (int x = lane; x < M.n_eqd; x += 64) {
    double f = 0.0;
    for (int t = M.eqd_start[x]; t < M.eqd_start[x + 1]; ++t)
      f += (double)M.eqd_coef[t] * scr[M.eqd_c[t]];
    rhs[M.eqd_dof[x]] -= f;
  }
  for (int e = lane; e < M.n_eqh; e += 64) H[M.eqh_h[e]] += (double)dt * deff * (double)M.eqh_w[e];
  wave_sync();
}

// Observables of a recorded step: the muscle slices of env `env` in record
// t / rec_every (all NULL when step t is not recorded), and the key nodes'
// world positions and orientations.
__device__ __forceinline__ RecOut rec_slices(const KModel &M, const KRun &Rn, int env, int step) {
  RecOut o{nullptr, nullptr, nullptr, nullptr, nullptr};
  if (Rn.rec_every <= 0 || step % Rn.rec_every) return o;
  const size_t b = ((size_t)(step / Rn.rec_every) * Rn.n_env + env) * M.n_mus;
  o.act = Rn.r_act ? Rn.r_act + b : nullptr;
  o.F = Rn.r_F ? Rn.r_F + b : nullptr;
  o.lm = Rn.r_lm ? Rn.r_lm + b : nullptr;
  o.vm = Rn.r_vm ? Rn.r_vm + b : nullptr;
  o.pw = Rn.r_pow ? Rn.r_pow + b : nullptr;
  return o;
}

__device__ __forceinline__ void record_keys(const KModel &M, const KRun &Rn, int lane, int env,
                                            int step, const float *Rl, V3 O) {
  if (Rn.rec_every <= 0 || step % Rn.rec_every) return;
  const size_t b = ((size_t)(step / Rn.rec_every) * Rn.n_env + env) * M.n_key;
  for (int k = lane; k < M.n_key; k += 64) {
    const float *F = Rl + 12 * M.key_node[k];
    if (Rn.r_xmat)
      for (int e = 0; e < 9; ++e) Rn.r_xmat[(b + k) * 9 + e] = F[e];
    if (Rn.r_xpos) {
      Rn.r_xpos[(b + k) * 3 + 0] = F[9] + O.x;
      Rn.r_xpos[(b + k) * 3 + 1] = F[10] + O.y;
      Rn.r_xpos[(b + k) * 3 + 2] = F[11] + O.z;
    }
  }
}

// Excitations u of this thread's muscles (internal slots t + n k) for
// absolute step `step`, advancing the smooth-noise state xar; returns true
// when one of this thread's activations is not finite.
template <int MPT, class Team>
__device__ __forceinline__ bool excite(const KModel &M, const KRun &Rn, const Team &T, int env,
                                       int step, const float act[MPT], float xar[MPT], float u[MPT]) {
  const int nm = M.n_mus;
  bool bad = false;
  unsigned long long key = 0;
  if (Rn.exc != EXC_ARRAY)
    key = splitmix64(splitmix64(Rn.seed ^ (unsigned long long)env) ^ (unsigned long long)(Rn.step0 + step));
#pragma unroll
  for (int k = 0; k < MPT; ++k) {
    const int mi = T.t + T.n * k;
    u[k] = 0.0f;
    if (mi < nm) {
      const int mx = M.mus_ext[mi];
      bad |= !isfinite(act[k]);
      if (Rn.exc == EXC_ARRAY) {
        u[k] = Rn.u ? Rn.u[((size_t)(Rn.u_hold ? 0 : step) * Rn.n_env + env) * nm + mx] : 0.0f;
      } else if (Rn.exc == EXC_IID) {
        u[k] = u24(splitmix64(key ^ (unsigned long long)mx), 40);
      } else {
        const AR1 r = ar1_step(key, mx, xar[k], Rn.rho, Rn.s, Rn.mean);
        u[k] = r.u;
        xar[k] = r.x;
      }
    }
  }
  return bad;
}

// Activation dynamics act' = clamp(act + dt (u - act) / tau(u, act), 0, 1).
template <int MPT, class Team>
__device__ __forceinline__ void activate(const KModel &M, const KRun &Rn, const Team &T, int env,
                                         float dt, const float u[MPT], const float act[MPT],
                                         float act1[MPT], bool stages) {
  const int nm = M.n_mus;
#pragma unroll
  for (int k = 0; k < MPT; ++k) {
    const int mi = T.t + T.n * k;
    act1[k] = 0.0f;
    if (mi < nm) {
      float uc = fminf(fmaxf(u[k], 0.0f), 1.0f);
      float a = act[k];
      float tau = uc > a ? M.mus_tact[mi] * (0.5f + 1.5f * a) : M.mus_tdeact[mi] / (0.5f + 1.5f * a);
      act1[k] = fminf(fmaxf(a + dt * (uc - a) / tau, 0.0f), 1.0f);
      if (stages && Rn.o_act) Rn.o_act[(size_t)env * nm + M.mus_ext[mi]] = act1[k];
    }
  }
}

// Muscle geometry (exact, or the surrogate's predictions with the per-env
// fallback check), Hill force, J_m^T F and the muscles' implicit damping.
// Outputs either accumulate into the fused step's LDS right-hand side and
// mass matrix (rhs, H) or go to the split step's device workspace
// (tau_out[nv], dsum_out[n_dent]). Returns false for the geometry-only
// variant, which stops after the geometry.
//
// TEN: compliant tendons. With the fibre length l_f (Rn.lm) the tendon
// (strain e = (L - l_f - l_s) / l_s, force F0 e / eps0 above slack, slope k)
// and the fibre (F0 [a f_l f_v(v) + f_p + beta v], slope b at the velocity v
// that balances the tendon) act in series: the force F_t + c (Ldot' - v) of
// the new lengthening rate Ldot', c = k dt / (1 + k dt / b), enters as the
// explicit force F_t + c (Ldot - v) and the implicit slope c. The moment
// arms, the path length and the activation go to Rn.fib for the fibre
// update after the solve.
template <int MPT, int NVIA, bool SURR, bool GEOM, bool TEN = false, class Team>
__device__ __forceinline__ void stage_muscles(const KModel &M, const KRun &Rn, const Team &T, int env,
                                              int step, const float *Rl, const float *Pl,
                                              const float *Sl, const float *q, const float *qd,
                                              V3 O, const float act1[MPT], unsigned char *scr,
                                              float dt, bool stages, double *rhs, double *H,
                                              float *tau_out, double *dsum_out, unsigned &status,
                                              const RecOut &ro) {
  const int nm = M.n_mus, nn = M.n_node, nv = M.nv;
  float *mr = (float *)scr;          // [n_mus][3]
  float *mF = mr + 3 * nm;           // [n_mus]
  float *mc = mF + nm;               // [n_mus]
  // surrogate geometry (when predictions are given): an env falls back to
  // the exact geometry when a hinge leaves the training box or when the
  // prediction misses the exact length or one of the moment arms of one of
  // 32 sentinel muscles, rotated each step, by more than the tolerance. The
  // decision is uniform over the env's team.
  bool exact = true;
  if (SURR) {
    const float *Y = Rn.geomY + (size_t)env * 4 * nm;
    bool out = false;
    for (int i = T.t; i < nn; i += T.n) {
      if (M.jtype[i] == 2) continue;
      const int j = M.dadr[i];
      const float qi = q[M.qadr[i]];
      out |= !(qi >= M.qlo[j] && qi <= M.qhi[j]);
    }
    bool miss = false;
    const int ns = nm < 32 ? nm : 32;
    if (T.t < ns) {
      const int mx = (int)((32ll * (Rn.step0 + step) + T.t) % nm);
      const int m = M.mus_int[mx];
      float r3[3], Ld;
      const float L = muscle_geometry<NVIA>(M, m, NVIA, Rl, Pl, Sl, qd, O, r3, Ld);
      miss = !(fabsf(Y[mx] - L) <= Rn.fb_tol);
#pragma unroll
      for (int sl = 0; sl < 3; ++sl)
        if (M.mus_span[sl * nm + m] >= 0) miss |= !(fabsf(Y[nm + 3 * mx + sl] - r3[sl]) <= Rn.fb_tol);
    }
    const bool o1 = T.any(out);
    const bool o2 = T.any(miss);
    exact = o1 || o2;
    if (exact) {
      status |= MS_ST_FALLBACK;
      if (Rn.fb_count && T.t == 0) Rn.fb_count[env] += 1u;
    } else {
      // the predictions are read in the caller's muscle order (contiguous)
      // and placed at each muscle's internal slot
      for (int x = T.t; x < nm; x += T.n) mF[M.mus_int[x]] = Y[x];
      for (int i = T.t; i < 3 * nm; i += T.n) {
        const int x = i / 3, sl = i - 3 * x, m = M.mus_int[x];
        mr[3 * m + sl] = M.mus_span[sl * nm + m] >= 0 ? Y[nm + i] : 0.f;
      }
      T.sync();
      for (int m = T.t; m < nm; m += T.n) {
        float Ld = 0.f;
#pragma unroll
        for (int sl = 0; sl < 3; ++sl) {
          const int j = M.mus_span[sl * nm + m];
          if (j >= 0) Ld -= mr[3 * m + sl] * qd[j];
        }
        mc[m] = Ld;
      }
    }
  }
  // exact geometry: one muscle per thread and iteration (L, Ldot parked in
  // mF, mc); a wavefront's 64 muscles share one via-point bound
#pragma unroll 1
  for (int m = T.t; exact && m < nm; m += T.n) {
    float r3[3], Ld;
    const float L = muscle_geometry<NVIA>(M, m, M.grp_nvia[m >> 6], Rl, Pl, Sl, qd, O, r3, Ld);
    if (!GEOM) {   // the geometry-only layout has no muscle scratch
      mr[3 * m] = r3[0];
      mr[3 * m + 1] = r3[1];
      mr[3 * m + 2] = r3[2];
      mF[m] = L;
      mc[m] = Ld;
    }
    if (stages) {
      const size_t o = (size_t)env * nm + M.mus_ext[m];
      Rn.o_L[o] = L;
      if (Rn.o_Ldot) Rn.o_Ldot[o] = Ld;
      Rn.o_r[3 * o] = r3[0];
      Rn.o_r[3 * o + 1] = r3[1];
      Rn.o_r[3 * o + 2] = r3[2];
    }
  }
  if (GEOM) return;
  // Hill force and its velocity slope (the same thread re-reads its muscles)
#pragma unroll
  for (int k = 0; k < MPT; ++k) {
    const int m = T.t + T.n * k;
    if (m >= nm) continue;
    const float L = mF[m], Ld = mc[m];
    const float f0 = M.mus_f0[m];
    float F, cdamp, lm, vm;
    if constexpr (TEN) {
      const float ls = M.mus_lslack[m];
      const float lf = Rn.lm[(size_t)env * nm + M.mus_ext[m]];
      const float strain = (L - lf - ls) / ls;
      const float ft = strain > 0.0f ? strain * Rn.ten_ieps : 0.0f;
      const float kdt = strain > 0.0f ? f0 * Rn.ten_ieps / ls * dt : 0.0f;
      lm = lf * M.mus_ilopt[m];
      const float A = act1[k] * hill_fl(lm);
      vm = hill_fv_root(A, ft - hill_fp(lm), Rn.ten_beta);
      const float b = f0 * (A * hill_fv_slope(vm) + Rn.ten_beta) * M.mus_ivl[m];
      const float c = kdt / (1.0f + kdt / b);
      const float v = vm / M.mus_ivl[m];
      F = f0 * ft + c * (Ld - v);
      cdamp = c;
      float *fb = Rn.fib + (size_t)env * Rn.fib_stride;
      fb[m] = mr[3 * m];
      fb[nm + m] = mr[3 * m + 1];
      fb[2 * nm + m] = mr[3 * m + 2];
      fb[3 * nm + m] = L;
      fb[4 * nm + m] = act1[k];
    } else {
      lm = (L - M.mus_lslack[m]) * M.mus_ilopt[m];
      vm = Ld * M.mus_ivl[m];
      const float fl = hill_fl(lm), fv = hill_fv(vm), fp = hill_fp(lm);
      F = f0 * (act1[k] * fl * fv + fp);
      cdamp = f0 * act1[k] * fl * hill_fv_slope(vm) * M.mus_ivl[m];
    }
    mF[m] = F;
    mc[m] = cdamp;
    if (stages) Rn.o_F[(size_t)env * nm + M.mus_ext[m]] = F;
    if (ro.act || ro.F || ro.lm || ro.vm || ro.pw) {
      // observables: the activation driving the force, the force, fibre
      // length and velocity (normalised) and the power |F Ldot| (W)
      const int mx = M.mus_ext[m];
      if (ro.act) ro.act[mx] = act1[k];
      if (ro.F) ro.F[mx] = F;
      if (ro.lm) ro.lm[mx] = lm;
      if (ro.vm) ro.vm[mx] = vm;
      if (ro.pw) ro.pw[mx] = fabsf(F * Ld);
    }
  }
  T.sync();
  for (int x = T.t; x < nv; x += T.n) {
    const int j = M.proj_dof[x];
    float tau = 0.f;
#pragma unroll 8
    for (int e = M.proj_start[x]; e < M.proj_start[x + 1]; ++e) {
      const int it = M.proj_item[e];
      tau += mr[it] * mF[it / 3];
    }
    if (stages) Rn.o_tau[(size_t)env * nv + j] = tau;
    if (tau_out)
      tau_out[j] = tau;
    else
      rhs[j] += (double)tau;
  }
  for (int e = T.t; e < M.n_dent; e += T.n) {
    double s = 0.0;
#pragma unroll 8
    for (int k = M.dent_start[e]; k < M.dent_start[e + 1]; ++k) {
      const int it = M.dent_item[k];
      const int m = it >> 4, a = (it >> 2) & 3, b = it & 3;
      s += (double)mc[m] * (double)mr[3 * m + a] * (double)mr[3 * m + b];
    }
    if (dsum_out)
      dsum_out[e] = s;
    else
      H[M.dent_h[e]] += (double)dt * s;
  }
  T.sync();
}

// LTDL factorisation of H (FP64, in LDS) with the L^T solve riding along,
// then the L solve; the solution is left in xs. rhs may be xs itself (row
// k's right-hand side is read only when row k is finished, before anything
// writes xs[k]). Returns true (the same in every lane) when a pivot is not
// positive.
//
// H = L^T D L with Featherstone's branch-induced sparsity, as gathers:
// finished row k holds H_kj - sum over the descendants i of k of
// H_ik H_ij / d_i (j = k or an ancestor of k), and reads only finished
// rows of lower height. The right-hand side rides along as one more
// column: y_k = rhs_k - sum_i (H_ik / d_i) y_i is the solve of L^T y =
// rhs. Rows of equal height are independent, so a height level is one
// pass over its entries; when a level has few entries, P lanes split each
// entry's sum (fixed-order prefix sums). All tables come from the
// workgroup's LDS copy.
__device__ __forceinline__ bool stage_solve(const KModel &M, int lane, const int *LT, double *H,
                                            const double *rhs, double *xs, double *invd) {
  const int nv = M.nv;
  bool nonspd = false;
  const int *Lrs = LT + M.lt_rs, *Ldesc = LT + M.lt_desc, *Ldr = LT + M.lt_drange;
  // leaves: y = rhs, pivots as assembled
  bool fbad = false;
  for (int j = lane; j < nv; j += 64) xs[j] = rhs[j];
  for (int e = LT[M.lt_hlev_start] + lane; e < LT[M.lt_hlev_start + 1]; e += 64) {
    const int w = LT[M.lt_hdof + e];
    const int k = w & 0xFF;
    const double d = H[Lrs[k] + (w >> 8)];
    fbad |= !(d > 0.0);
    invd[k] = 1.0 / d;
  }
  nonspd = __any(fbad);
  wave_sync();
  // one entry of a row at height >= 1: finished value (and its pivot when
  // it is the diagonal) from the descendants' finished rows
  auto entry = [&](int w, int p, int P, double &sum, int &e, int &k, int &ck, int &cj) {
    k = w & 0xFF;
    ck = (w >> 8) & 0xFF;
    cj = w >> 16;
    const bool rcol = cj == 255;
    e = Lrs[k] + (rcol ? 0 : cj);
    const int dr = Ldr[k], t1 = dr >> 16;
    sum = 0.0;
#pragma unroll 4
    for (int t = (dr & 0xFFFF) + p; t < t1; t += P) {
      const int di = Ldesc[t];
      const int ri = di & 0xFFFF, i = di >> 16;
      const double hij = rcol ? xs[i] : H[ri + cj];
      sum += H[ri + ck] * hij * invd[i];
    }
  };
  auto finish = [&](double sum, int e, int k, int ck, int cj, bool &badf) {
    if (cj == 255) {
      xs[k] = rhs[k] - sum;
    } else {
      const double v = H[e] - sum;
      H[e] = v;
      if (cj == ck) {
        badf |= !(v > 0.0);
        invd[k] = 1.0 / v;
      }
    }
  };
  for (int h = 1; h < M.n_hgat && !nonspd; ++h) {
    const int s0 = LT[M.lt_hent_start + h], ne = LT[M.lt_hent_start + h + 1] - s0;
    const int lp = group_log2(ne), P = 1 << lp;
    fbad = false;
    if (lp == 0) {
      // more entries than lanes: two independent entries per lane in flight
      for (int base = 0; base < ne; base += 128) {
        const int ga = base + lane, gb = base + 64 + lane;
        double sa = 0.0, sb = 0.0;
        int ea = 0, ka = 0, cka = 0, cja = 0, eb = 0, kb = 0, ckb = 0, cjb = 0;
        if (ga < ne) entry(LT[M.lt_hent + s0 + ga], 0, 1, sa, ea, ka, cka, cja);
        if (gb < ne) entry(LT[M.lt_hent + s0 + gb], 0, 1, sb, eb, kb, ckb, cjb);
        if (ga < ne) finish(sa, ea, ka, cka, cja, fbad);
        if (gb < ne) finish(sb, eb, kb, ckb, cjb, fbad);
      }
    } else {
      const int g = lane >> lp, p = lane & (P - 1);
      double sum = 0.0;
      int e = 0, k = 0, ck = 0, cj = 0;
      if (g < ne) entry(LT[M.lt_hent + s0 + g], p, P, sum, e, k, ck, cj);
      sum = group_sum_last(sum, lp, lane);
      if (g < ne && p == P - 1) finish(sum, e, k, ck, cj, fbad);
    }
    nonspd = __any(fbad);
    wave_sync();
  }
  // The trunk (single-row levels at the top, ancestor counts 0 .. n_trunk-1):
  // its rows were gathered over their non-trunk descendants only, which
  // leaves the block that remains once every other row is eliminated.
  // Eliminating its rows bottom-up, row k (final once the rows below it
  // are eliminated) updates every entry (a, b) of the rows above it, b = a
  // or an ancestor of a, and their right-hand sides:
  // H_ab -= H_ka H_kb / d_k, y_a -= H_ka y_k / d_k. One level per row, one
  // FMA per entry, no two lanes writing the same entry.
  if (M.n_trunk && !nonspd) {
    const int *trow = LT + M.lt_trow, *tpair = LT + M.lt_tpair;
    const int nt = M.n_trunk, npair = (nt - 1) * (nt + 2) / 2;
    // this lane's first three entries stay in registers; all of a level's
    // loads are issued before its stores
    int tw[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) tw[u] = lane + 64 * u < npair ? tpair[lane + 64 * u] : -1;
    int wk = trow[nt - 1];
    for (int dk = nt - 1; dk >= 0; --dk) {
      const int k = wk & 0xFF, rk = wk >> 8;
      const double d = H[rk + dk], xk = xs[k];
      double hka[3], hkb[3], hab[3];
      bool on[3], rhsc[3];
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        const int w = tw[u], da = (w >> 16) & 0x7F, db = (w >> 23) & 0x7F;
        on[u] = w >= 0 && da < dk;
        rhsc[u] = (w >> 30) & 1;
        hka[u] = hkb[u] = hab[u] = 0.0;
        if (on[u]) {
          hka[u] = H[rk + da];
          if (!rhsc[u]) hkb[u] = H[rk + db];
          hab[u] = rhsc[u] ? xs[w & 0xFFFF] : H[w & 0xFFFF];
        }
      }
      if (dk > 0) wk = trow[dk - 1];
      if (!(d > 0.0)) {  // the same value in every lane
        nonspd = true;
        break;
      }
      const double id = 1.0 / d, yk = xk * id;
      if (lane == 0) invd[k] = id;
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        if (!on[u]) continue;
        const int e = tw[u] & 0xFFFF;
        if (rhsc[u]) xs[e] = hab[u] - hka[u] * yk;
        else H[e] = hab[u] - hka[u] * hkb[u] * id;
      }
      // entries beyond the first 192 (trunks longer than 18 rows)
      const int na = dk * (dk + 3) / 2;
      for (int t = lane + 192; t < na; t += 64) {
        const int w = tpair[t], e = w & 0xFFFF, da = (w >> 16) & 0x7F;
        const double h1 = H[rk + da];
        if (w >> 30) {
          xs[e] -= h1 * yk;
        } else {
          const int db = (w >> 23) & 0x7F;
          H[e] -= h1 * H[rk + db] * id;
        }
      }
      wave_sync();
    }
  }
  if (!nonspd) {
    // L x = z with z = y / d, root first: x_k = z_k - (1/d_k) sum over the
    // ancestors a of k of H_ka x_a. Each lane keeps its rows' sums in
    // registers; at depth l the rows of that depth are final, and every
    // deeper row adds the term of its (single) depth-l ancestor, which is
    // entry l of its root-first row.
    const unsigned char *path8 = (const unsigned char *)(LT + M.lt_path);
    double z[2], id[2], acc[2] = {0.0, 0.0};
    int rk[2], dk[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int j = lane + 64 * t;
      dk[t] = -1;
      rk[t] = 0;
      id[t] = z[t] = 0.0;
      if (j < nv) {
        rk[t] = Lrs[j];
        dk[t] = Lrs[j + 1] - rk[t] - 1;
        id[t] = invd[j];
        z[t] = xs[j] * id[t];
      }
    }
    for (int l = 0;; ++l) {
      double h[2];
      int c[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        h[t] = 0.0;
        c[t] = 0;
        if (dk[t] > l) {
          h[t] = H[rk[t] + l];
          c[t] = path8[rk[t] + l];
        }
        if (dk[t] == l) xs[lane + 64 * t] = z[t] - acc[t] * id[t];
      }
      wave_sync();
      if (l + 1 >= M.n_dlev) break;
#pragma unroll
      for (int t = 0; t < 2; ++t)
        if (dk[t] > l) acc[t] += h[t] * xs[c[t]];
    }
  }
  return nonspd;
}

// Semi-implicit Euler update in LDS: qd += dt qdd (qdd = xs), then q += dt
// qd (root orientation by the quaternion exponential of the body angular
// velocity). Nothing changes and false is returned (the same in every
// lane) when a new velocity is not finite or act_bad is set.
__device__ __forceinline__ bool stage_integrate(const KModel &M, int lane, float *q, float *qd,
                                                const double *xs, float dt, bool act_bad) {
  const int nv = M.nv, nn = M.n_node;
  // new velocities and hinge/slide positions in registers, checked first
  float qdn[2], qn[2];
  bool badn = act_bad;
  for (int t = 0; t < 2; ++t) {
    const int j = lane + 64 * t;
    qdn[t] = 0.f;
    qn[t] = 0.f;
    if (j < nv) {
      qdn[t] = qd[j] + dt * (float)xs[j];
      badn |= !isfinite(qdn[t]);
    }
  }
  badn = __any(badn);
  if (badn) return false;
  wave_sync();
  for (int t = 0; t < 2; ++t) {
    const int j = lane + 64 * t;
    if (j < nv) qd[j] = qdn[t];
  }
  wave_sync();
  // positions: each node's q from its own DoFs
  for (int i = lane; i < nn; i += 64) {
    const int a = M.qadr[i], d = M.dadr[i];
    if (M.jtype[i] != 2) {
      qn[0] = q[a] + dt * qd[d];
      q[a] = qn[0];
      continue;
    }
    for (int k = 0; k < 3; ++k) q[a + k] = q[a + k] + dt * qd[d + k];
    float th[3] = {qd[d + 3] * dt, qd[d + 4] * dt, qd[d + 5] * dt};
    float ang = sqrtf(th[0] * th[0] + th[1] * th[1] + th[2] * th[2]);
    float dq[4];
    if (ang < 1e-8f) {
      dq[0] = 1.f; dq[1] = 0.5f * th[0]; dq[2] = 0.5f * th[1]; dq[3] = 0.5f * th[2];
    } else {
      float sn, cs;
      sincosf(0.5f * ang, &sn, &cs);
      float sc = sn / ang;
      dq[0] = cs; dq[1] = sc * th[0]; dq[2] = sc * th[1]; dq[3] = sc * th[2];
    }
    float *x = q + a + 3;
    float o0 = x[0] * dq[0] - x[1] * dq[1] - x[2] * dq[2] - x[3] * dq[3];
    float o1 = x[0] * dq[1] + x[1] * dq[0] + x[2] * dq[3] - x[3] * dq[2];
    float o2 = x[0] * dq[2] - x[1] * dq[3] + x[2] * dq[0] + x[3] * dq[1];
    float o3 = x[0] * dq[3] + x[1] * dq[2] - x[2] * dq[1] + x[3] * dq[0];
    float nrm = sqrtf(o0 * o0 + o1 * o1 + o2 * o2 + o3 * o3);
    x[0] = o0 / nrm; x[1] = o1 / nrm; x[2] = o2 / nrm; x[3] = o3 / nrm;
  }
  wave_sync();
  return true;
}

// ------------------------------------------------------- the fused step
// One wavefront steps one env n_steps times with every intermediate in LDS
// and registers. SURR: muscle geometry from the surrogate's predictions with
// the per-env fallback check; GEOM: exact geometry only (stage outputs).
template <int MPL, int NVIA, bool SURR, bool GEOM, bool COUPLE = false>
__device__ __forceinline__ void step_body(const KModel &M, const KRun &Rn, int n_steps) {
  // a workgroup holds blockDim.x / 64 envs, one per wavefront, each with its
  // own LDS block; envs never synchronise with each other
  // LDS: the factorisation's gather tables (shared by the workgroup's envs,
  // staged once per launch), then one block per env.
  extern __shared__ __align__(16) unsigned char lds_all[];
  const int wave = threadIdx.x >> 6;
  const int env = blockIdx.x * (blockDim.x >> 6) + wave;
  const int lane = threadIdx.x & 63;
  const WaveTeam T{lane};
  int *LT = (int *)lds_all;
  // every variant reads the tree schedule from this table
  for (int i = threadIdx.x; i < M.lt_words; i += blockDim.x) LT[i] = M.lt[i];
  __syncthreads();  // the only workgroup-wide barrier: every wavefront reaches it
  if (env >= Rn.n_env) return;
  unsigned char *lds = lds_all + (size_t)M.lt_words * 4 + (size_t)wave * M.lds_env;
  const int nq = M.nq, nv = M.nv, nm = M.n_mus;
  float *__restrict__ q = (float *)(lds + M.off_q);
  float *__restrict__ qd = (float *)(lds + M.off_qd);
  // node frames: 12 floats per node, 16-byte aligned: R (row-major) then P
  float *Rl = (float *)(lds + M.off_R);
  float *Pl = Rl + 9;
  float *__restrict__ Sl = (float *)(lds + M.off_S);
  float *Vl = (float *)(lds + M.off_V);
  float *Al = (float *)(lds + M.off_A);
  float *Fl = (float *)(lds + M.off_F);  // f_b[n_body][6] then F_n[n_node][6]
  float *__restrict__ Cl = (float *)(lds + M.off_con);
  double *__restrict__ rhs = (double *)(lds + M.off_rhs);
  double *__restrict__ xs = (double *)(lds + M.off_x);
  double *__restrict__ H = (double *)(lds + M.off_H);
  unsigned char *scr = lds + M.off_scr;
  // tree schedule and subtree lists from the workgroup's table
  const int *tlev = LT + M.lt_tlev, *tnode = LT + M.lt_tnode;
  const int *sbs = LT + M.lt_subb_start, *scs = LT + M.lt_subc_start;
  const unsigned char *sbl = (const unsigned char *)(LT + M.lt_subb);
  const unsigned char *scl = (const unsigned char *)(LT + M.lt_subc);
  const float dt = Rn.dt;
  const bool stages = Rn.stages != 0;

  for (int i = lane; i < nq; i += 64) q[i] = Rn.q[(size_t)env * nq + i];
  for (int i = lane; i < nv; i += 64) qd[i] = Rn.qd ? Rn.qd[(size_t)env * nv + i] : 0.0f;
  float act[MPL], xar[MPL];
#pragma unroll
  for (int t = 0; t < MPL; ++t) {
    int mi = lane + 64 * t;
    const int mx = mi < nm ? M.mus_ext[mi] : 0;
    act[t] = (mi < nm && Rn.act) ? Rn.act[(size_t)env * nm + mx] : 0.0f;
    xar[t] = 0.0f;
    if (Rn.exc == EXC_AR1 && mi < nm) xar[t] = Rn.xar[(size_t)env * nm + mx];
  }
  unsigned status = Rn.status ? Rn.status[env] : 0u;
  unsigned applied = 0;
  wave_sync();

  for (int step = 0; step < n_steps; ++step) {
    // ---------------------------------------------- excitation and state check
    float u[MPL];
    bool bad = false;
    for (int i = lane; i < nq; i += 64) bad |= !isfinite(q[i]);
    for (int i = lane; i < nv; i += 64) bad |= !isfinite(qd[i]);
    bad |= excite<MPL>(M, Rn, T, env, step, act, xar, u);
    if (__any(bad)) {
      status |= MS_ST_NONFINITE;
      continue;  // the state stays as it is
    }
    float act1[MPL];
    activate<MPL>(M, Rn, T, env, dt, u, act, act1, stages);
    const V3 O = M.free_root ? v3(q[0], q[1], q[2]) : v3(0.f, 0.f, 0.f);
    const V3 g = v3(M.gx, M.gy, M.gz);
    stage_fk(M, lane, tlev, tnode, q, qd, Rl, Sl, Vl, Al, O, g);
    record_keys(M, Rn, lane, env, step, Rl, O);
    if (!GEOM) {
      stage_contacts(M, lane, Rl, Vl, Cl, O, dt, Rn.contact);
      stage_rnea(M, lane, Rl, Pl, Vl, Al, Fl, Cl, Sl, qd, sbs, sbl, scs, scl, rhs,
                 stages ? Rn.o_bias + (size_t)env * nv : nullptr);
      float dmp[2];
      stage_crba(M, lane, LT, Rl, Pl, Sl, Cl, scr, dt, H, dmp);
      add_joint_damping(M, lane, LT, H, dt, dmp);
    }
    stage_muscles<MPL, NVIA, SURR, GEOM>(M, Rn, T, env, step, Rl, Pl, Sl, q, qd, O, act1, scr, dt,
                                         stages, rhs, H, nullptr, nullptr, status,
                                         rec_slices(M, Rn, env, step));
    if (GEOM) return;
    // a separate instantiation: the uncoupled kernel sits at the register
    // limit, and the coupling's code costs it 13 % when compiled in
    if (COUPLE) add_coupling(M, lane, q, qd, H, rhs, (double *)scr, dt);
    if (stages) {
      for (int e = lane; e < M.nnz; e += 64) Rn.o_H[(size_t)env * M.nnz + e] = H[e];
    }
    const bool nonspd = stage_solve(M, lane, LT, H, rhs, xs, (double *)scr);
    if (stages) {
      for (int j = lane; j < nv; j += 64) Rn.o_qdd[(size_t)env * nv + j] = nonspd ? NAN : (float)xs[j];
      break;
    }
    if (nonspd) {
      status |= MS_ST_NONSPD;
      continue;
    }
    bool abad = false;
#pragma unroll
    for (int t = 0; t < MPL; ++t) abad |= !isfinite(act1[t]);
    if (!stage_integrate(M, lane, q, qd, xs, dt, abad)) {
      status |= MS_ST_NONFINITE;
      continue;
    }
#pragma unroll
    for (int t = 0; t < MPL; ++t) act[t] = act1[t];
    ++applied;
  }

  if (stages) return;
  for (int i = lane; i < nq; i += 64) Rn.q[(size_t)env * nq + i] = q[i];
  for (int i = lane; i < nv; i += 64) Rn.qd[(size_t)env * nv + i] = qd[i];
#pragma unroll
  for (int t = 0; t < MPL; ++t) {
    const int mi = lane + 64 * t;
    if (mi < nm) {
      const int mx = M.mus_ext[mi];
      Rn.act[(size_t)env * nm + mx] = act[t];
      if (Rn.exc == EXC_AR1) Rn.xar[(size_t)env * nm + mx] = xar[t];
    }
  }
  if (Rn.status && lane == 0) Rn.status[env] = status;
  if (Rn.n_applied && lane == 0) Rn.n_applied[env] += applied;
}

template <int MPL, int NVIA>
__global__ __launch_bounds__(256) void k_step(KModel M, KRun Rn, int n_steps) {
  step_body<MPL, NVIA, false, false>(M, Rn, n_steps);
}

// the exact step of a model with joint coupling
template <int MPL, int NVIA>
__global__ __launch_bounds__(256) void k_step_coupled(KModel M, KRun Rn, int n_steps) {
  step_body<MPL, NVIA, false, false, true>(M, Rn, n_steps);
}

template <int MPL, int NVIA>
__global__ __launch_bounds__(256) void k_step_surrogate(KModel M, KRun Rn, int n_steps) {
  step_body<MPL, NVIA, true, false>(M, Rn, n_steps);
}

// exact muscle geometry only (L, Ldot, r as stage outputs)
template <int MPL, int NVIA>
__global__ __launch_bounds__(256) void k_geometry(KModel M, KRun Rn, int n_steps) {
  step_body<MPL, NVIA, false, true>(M, Rn, n_steps);
}

// ------------------------------------------------------- the split step
// The muscle kernel of the split step (one env per 256-thread workgroup):
// excitation and activation, muscle geometry (or the surrogate with its
// fallback check), Hill force, J_m^T F and the muscles' implicit damping,
// from the node frames and motion subspaces the kinematics kernel left in
// the workspace. MPT = muscles per thread.
template <int MPT, int NVIA, bool SURR, bool TEN = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(7, 7))) void k_muscle(KModel M, KRun Rn, KSplit W, int step) {
  extern __shared__ __align__(16) unsigned char lds_m[];
  const int env = Rn.env_begin + blockIdx.x;
  if (env >= (Rn.env_end ? Rn.env_end : Rn.n_env)) return;  // uniform over the workgroup
  const BlockTeam T{(int)threadIdx.x};
  const int nq = M.nq, nv = M.nv, nm = M.n_mus, nn = M.n_node;
  float *Rl = (float *)(lds_m + W.m_R);
  float *Pl = Rl + 9;
  float *Sl = (float *)(lds_m + W.m_S);
  float *q = (float *)(lds_m + W.m_q);
  float *qd = (float *)(lds_m + W.m_qd);
  unsigned char *scr = lds_m + W.m_scr;
  const int fl = W.flag[env];
  float act[MPT], xar[MPT], u[MPT];
#pragma unroll
  for (int k = 0; k < MPT; ++k) {
    const int mi = T.t + 256 * k;
    const int mx = mi < nm ? M.mus_ext[mi] : 0;
    act[k] = mi < nm ? Rn.act[(size_t)env * nm + mx] : 0.0f;
    xar[k] = 0.0f;
    if (Rn.exc == EXC_AR1 && mi < nm) xar[k] = Rn.xar[(size_t)env * nm + mx];
  }
  bool abad = excite<MPT>(M, Rn, T, env, step, act, xar, u);
  if constexpr (TEN) {
    // the fibre lengths are state: a non-finite one stops the env like a
    // non-finite activation
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      const int mi = T.t + 256 * k;
      if (mi < nm) abad |= !isfinite(Rn.lm[(size_t)env * nm + M.mus_ext[mi]]);
    }
  }
  // the smooth-noise state advances whatever the env's state (as in the
  // fused step)
  if (Rn.exc == EXC_AR1) {
#pragma unroll
    for (int k = 0; k < MPT; ++k) {
      const int mi = T.t + 256 * k;
      if (mi < nm) Rn.xar[(size_t)env * nm + M.mus_ext[mi]] = xar[k];
    }
  }
  if (T.any(abad) || fl != 0) {
    if (T.t == 0) W.mflag[env] = 1;
    return;
  }
  for (int i = T.t; i < 12 * nn; i += 256) Rl[i] = W.frames[(size_t)env * W.fr_stride + i];
  for (int i = T.t; i < 6 * nv; i += 256) Sl[i] = W.S[(size_t)env * W.S_stride + i];
  for (int i = T.t; i < nq; i += 256) q[i] = Rn.q[(size_t)env * nq + i];
  for (int i = T.t; i < nv; i += 256) qd[i] = Rn.qd[(size_t)env * nv + i];
  float act1[MPT];
  activate<MPT>(M, Rn, T, env, Rn.dt, u, act, act1, false);
  __syncthreads();
  const V3 O = M.free_root ? v3(q[0], q[1], q[2]) : v3(0.f, 0.f, 0.f);
  unsigned status = 0;
  stage_muscles<MPT, NVIA, SURR, false, TEN>(M, Rn, T, env, step, Rl, Pl, Sl, q, qd, O, act1, scr, Rn.dt,
                                        false, nullptr, nullptr, W.tau + (size_t)env * W.tau_stride,
                                        W.dsum + (size_t)env * W.dsum_stride, status,
                                        rec_slices(M, Rn, env, step));
  bool bad1 = false;
#pragma unroll
  for (int k = 0; k < MPT; ++k) {
    const int mi = T.t + 256 * k;
    if (mi < nm) {
      W.actn[(size_t)env * W.act_stride + M.mus_ext[mi]] = act1[k];
      bad1 |= !isfinite(act1[k]);
    }
  }
  bad1 = T.any(bad1);
  if (T.t == 0) {
    W.mflag[env] = bad1 ? 2 : 0;
    if (status && Rn.status) Rn.status[env] |= status;
  }
}

// Launch the muscle kernel of the split step for step `step`.
template <int NVIA>
hipError_t launch_muscle(const KModel &k, const KRun &r, const KSplit &w, int mpt, int step,
                         hipStream_t st) {
  const bool surr = r.geomY != nullptr, ten = r.lm != nullptr;
  if (surr && ten) return hipErrorNotSupported;
  const dim3 grid((r.env_end ? r.env_end : r.n_env) - r.env_begin), block(256);
  const size_t lds = w.m_bytes;
#define MS_LAUNCH_M(P)                                                                         \
  do {                                                                                         \
    const void *fn = surr  ? (const void *)&k_muscle<P, NVIA, true>                            \
                     : ten ? (const void *)&k_muscle<P, NVIA, false, true>                     \
                           : (const void *)&k_muscle<P, NVIA, false>;                          \
    if (lds > 65536) {                                                                         \
      hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds); \
      if (e != hipSuccess) return e;                                                           \
    }                                                                                          \
    if (surr)                                                                                  \
      hipLaunchKernelGGL((k_muscle<P, NVIA, true>), grid, block, lds, st, k, r, w, step);     \
    else if (ten)                                                                              \
      hipLaunchKernelGGL((k_muscle<P, NVIA, false, true>), grid, block, lds, st, k, r, w, step); \
    else                                                                                       \
      hipLaunchKernelGGL((k_muscle<P, NVIA, false>), grid, block, lds, st, k, r, w, step);    \
  } while (0)
  if (mpt <= 1)
    MS_LAUNCH_M(1);
  else if (mpt <= 2)
    MS_LAUNCH_M(2);
  else if (mpt <= 3)
    MS_LAUNCH_M(3);
  else
    MS_LAUNCH_M(4);
#undef MS_LAUNCH_M
  return hipGetLastError();
}

// ------------------------------------------------------------ launchers
template <int MPL, int NVIA>
hipError_t launch_k(const Tables &t, const KModel &k, const KRun &r, int n_env, int n_steps,
                    hipStream_t st) {
  const bool geom = r.stages == 2, surr = r.geomY != nullptr;
  const bool coupled = k.n_eq > 0 && !geom;
  if (coupled && surr) return hipErrorNotSupported;  // the split schedule steps these
  int W = r.env_per_wg > 0 ? r.env_per_wg : default_env_per_wg(t);
  size_t lds = t.lt.size() * 4 + (size_t)W * t.lds_bytes;
  if (geom) {
    // geometry only: the compact per-env layout and the tree schedule's part
    // of the table, so several times more envs stay resident per CU
    KModel g = k;
    g.off_q = t.geo_q;
    g.off_qd = t.geo_qd;
    g.off_R = t.geo_R;
    g.off_P = t.geo_R + 36;
    g.off_S = t.geo_S;
    g.off_V = g.off_scr = t.geo_V;
    g.off_A = g.off_F = t.geo_V + 4 * 6 * k.n_node;
    g.off_con = g.off_rhs = g.off_x = g.off_H = g.off_flag = 0;   // not read
    g.lds_env = t.geo_bytes;
    g.lt_words = t.geo_lt_words;
    const void *fg = (const void *)&k_geometry<MPL, NVIA>;
    int best = 0;
    for (int w = 1; w <= 4; w *= 2) {
      const size_t l = (size_t)g.lt_words * 4 + (size_t)w * t.geo_bytes;
      if (l > 160 * 1024) break;
      if (l > 65536 && hipFuncSetAttribute(fg, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)l) != hipSuccess)
        break;
      int nb = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fg, 64 * w, l) != hipSuccess) break;
      if (nb * w >= best) {
        best = nb * w;
        W = w;
        lds = l;
      }
    }
    if (best == 0) return hipErrorInvalidConfiguration;
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(fg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((k_geometry<MPL, NVIA>), dim3((n_env + W - 1) / W), dim3(64 * W), lds, st,
                       g, r, n_steps);
    return hipGetLastError();
  }
  const void *fn = surr ? (const void *)&k_step_surrogate<MPL, NVIA>
                   : coupled ? (const void *)&k_step_coupled<MPL, NVIA>
                             : (const void *)&k_step<MPL, NVIA>;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const dim3 grid((n_env + W - 1) / W), block(64 * W);
  if (surr)
    hipLaunchKernelGGL((k_step_surrogate<MPL, NVIA>), grid, block, lds, st, k, r, n_steps);
  else if (coupled)
    hipLaunchKernelGGL((k_step_coupled<MPL, NVIA>), grid, block, lds, st, k, r, n_steps);
  else
    hipLaunchKernelGGL((k_step<MPL, NVIA>), grid, block, lds, st, k, r, n_steps);
  return hipGetLastError();
}

template <int NVIA>
hipError_t launch_nvia(const Tables &t, const KModel &k, const KRun &r, int n_env, int n_steps,
                       hipStream_t st) {
  const int mpl = t.mpl;
  if (mpl <= 1) return launch_k<1, NVIA>(t, k, r, n_env, n_steps, st);
  if (mpl <= 2) return launch_k<2, NVIA>(t, k, r, n_env, n_steps, st);
  if (mpl <= 4) return launch_k<4, NVIA>(t, k, r, n_env, n_steps, st);
  if (mpl <= 8) return launch_k<8, NVIA>(t, k, r, n_env, n_steps, st);
  if (mpl <= 12) return launch_k<12, NVIA>(t, k, r, n_env, n_steps, st);
  return launch_k<16, NVIA>(t, k, r, n_env, n_steps, st);
}

}  // namespace ms
