// ms_step_split.hip -- the kinematics/dynamics and factorisation kernels of
// the split step (the muscle kernel sits with the via-point instantiations).
//
// Per physics step, for every env:
//  1. k_front (one wavefront per env): state check, forward kinematics,
//     contacts, Newton-Euler bias (right-hand side), composite-rigid-body
//     mass matrix; leaves node frames, motion subspaces, H and rhs in the
//     workspace;
//  2. k_muscle (ms_step_kernel.h): excitation, activation, muscles;
//  3. k_back (one wavefront per env): H += dt (joint and muscle damping),
//     rhs += J_m^T F, LTDL factorisation and solves in FP64, semi-implicit
//     Euler, commit of the new state.
// Each kernel stages only its part of the model's LDS table, so its LDS
// block per env is about half the fused step's and more envs stay resident
// per CU.
#include "ms_step_kernel.h"

#include <algorithm>

namespace ms {

__global__ __launch_bounds__(1024) void k_front(KModel M, KRun Rn, KSplit W, int step) {
  extern __shared__ __align__(16) unsigned char lds_f[];
  const int wave = threadIdx.x >> 6;
  const int env = Rn.env_begin + blockIdx.x * (blockDim.x >> 6) + wave;
  const int lane = threadIdx.x & 63;
  int *LT = (int *)lds_f;  // words [0, lt_front_end) of the model's table
  for (int i = threadIdx.x; i < M.lt_front_end; i += blockDim.x) LT[i] = M.lt[i];
  __syncthreads();  // the only workgroup-wide barrier
  if (env >= (Rn.env_end ? Rn.env_end : Rn.n_env)) return;
  unsigned char *lds = lds_f + (size_t)M.lt_front_end * 4 + (size_t)wave * W.f_bytes;
  const int nq = M.nq, nv = M.nv, nn = M.n_node;
  // q and qd are read where they lie (the kernel does not change them),
  // which leaves LDS for one more env per CU
  const float *q = Rn.q + (size_t)env * nq;
  const float *qd = Rn.qd + (size_t)env * nv;
  float *Rl = (float *)(lds + W.f_R);
  float *Pl = Rl + 9;
  float *Sl = (float *)(lds + W.f_S);
  float *Cl = (float *)(lds + W.f_con);
  unsigned char *scr = lds + W.f_scr;
  float *Vl = (float *)scr;
  float *Al = Vl + 6 * nn;
  float *Fl = Al + 6 * nn;
  bool bad = false;
  for (int i = lane; i < nq; i += 64) bad |= !isfinite(q[i]);
  for (int i = lane; i < nv; i += 64) bad |= !isfinite(qd[i]);
  if (__any(bad)) {
    if (lane == 0) W.flag[env] = 1;
    return;
  }
  wave_sync();
  const int *tlev = LT + M.lt_tlev, *tnode = LT + M.lt_tnode;
  const int *sbs = LT + M.lt_subb_start, *scs = LT + M.lt_subc_start;
  const unsigned char *sbl = (const unsigned char *)(LT + M.lt_subb);
  const unsigned char *scl = (const unsigned char *)(LT + M.lt_subc);
  const V3 O = M.free_root ? v3(q[0], q[1], q[2]) : v3(0.f, 0.f, 0.f);
  const V3 g = v3(M.gx, M.gy, M.gz);
  stage_fk(M, lane, tlev, tnode, q, qd, Rl, Sl, Vl, Al, O, g);
  record_keys(M, Rn, lane, env, step, Rl, O);
  // node frames and motion subspaces for the muscle kernel
  float *gf = W.frames + (size_t)env * W.fr_stride;
  for (int i = lane; i < 3 * nn; i += 64) ((float4 *)gf)[i] = ((const float4 *)Rl)[i];
  float *gs = W.S + (size_t)env * W.S_stride;
  for (int i = lane; i < 3 * nv; i += 64) ((float2 *)gs)[i] = ((const float2 *)Sl)[i];
  stage_contacts(M, lane, Rl, Vl, Cl, O, Rn.dt, Rn.contact);
  stage_rnea(M, lane, Rl, Pl, Vl, Al, Fl, Cl, Sl, qd, sbs, sbl, scs, scl,
             W.rhs + (size_t)env * W.rhs_stride, nullptr);
  float dmp[2];
  stage_crba(M, lane, LT, Rl, Pl, Sl, Cl, scr, Rn.dt, W.H + (size_t)env * W.H_stride, dmp);
  if (lane == 0) W.flag[env] = 0;
}

__global__ __launch_bounds__(1024) void k_back(KModel M, KRun Rn, KSplit W, int step) {
  extern __shared__ __align__(16) unsigned char lds_b[];
  const int wave = threadIdx.x >> 6;
  const int env = Rn.env_begin + blockIdx.x * (blockDim.x >> 6) + wave;
  const int lane = threadIdx.x & 63;
  // words [lt_back_begin, lt_words) of the model's table, indexed with the
  // table's own offsets
  const int nw = M.lt_words - M.lt_back_begin;
  for (int i = threadIdx.x; i < nw; i += blockDim.x) ((int *)lds_b)[i] = M.lt[M.lt_back_begin + i];
  __syncthreads();  // the only workgroup-wide barrier
  if (env >= (Rn.env_end ? Rn.env_end : Rn.n_env)) return;
  const int *LT = (const int *)lds_b - M.lt_back_begin;
  unsigned char *lds = lds_b + (size_t)nw * 4 + (size_t)wave * W.b_bytes;
  const int nq = M.nq, nv = M.nv, nm = M.n_mus;
  const int fl = W.flag[env] | W.mflag[env];
  if (fl & 1) {
    if (lane == 0 && Rn.status) Rn.status[env] |= MS_ST_NONFINITE;
    return;
  }
  float *q = (float *)(lds + W.b_q);
  float *qd = (float *)(lds + W.b_qd);
  double *xs = (double *)(lds + W.b_x);   // the right-hand side, solved in place
  double *invd = (double *)(lds + W.b_invd);
  double *H = (double *)(lds + W.b_H);
  const float dt = Rn.dt;
  float dmp[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) dmp[t] = lane + 64 * t < nv ? M.damping[lane + 64 * t] : 0.f;
  for (int i = lane; i < nq; i += 64) q[i] = Rn.q[(size_t)env * nq + i];
  for (int i = lane; i < nv; i += 64) {
    qd[i] = Rn.qd[(size_t)env * nv + i];
    xs[i] = W.rhs[(size_t)env * W.rhs_stride + i] + (double)W.tau[(size_t)env * W.tau_stride + i];
  }
  const double *gH = W.H + (size_t)env * W.H_stride;
  for (int e = lane; e < M.nnz; e += 64) H[e] = gH[e];
  wave_sync();
  add_joint_damping(M, lane, LT, H, dt, dmp);
  const double *gd = W.dsum + (size_t)env * W.dsum_stride;
  for (int e = lane; e < M.n_dent; e += 64) H[M.dent_h[e]] += (double)dt * gd[e];
  wave_sync();
  add_coupling(M, lane, q, qd, H, xs, invd, dt);   // invd is free until the solve
  if (stage_solve(M, lane, LT, H, xs, xs, invd)) {
    if (lane == 0 && Rn.status) Rn.status[env] |= MS_ST_NONSPD;
    return;
  }
  if (!stage_integrate(M, lane, q, qd, xs, dt, (fl & 2) != 0)) {
    if (lane == 0 && Rn.status) Rn.status[env] |= MS_ST_NONFINITE;
    return;
  }
  for (int i = lane; i < nq; i += 64) Rn.q[(size_t)env * nq + i] = q[i];
  for (int i = lane; i < nv; i += 64) Rn.qd[(size_t)env * nv + i] = qd[i];
  const float *an = W.actn + (size_t)env * W.act_stride;
  for (int i = lane; i < nm; i += 64) Rn.act[(size_t)env * nm + i] = an[i];
  if (Rn.n_applied && lane == 0) Rn.n_applied[env] += 1u;
  if (Rn.lm && lane == 0) W.mflag[env] = 4;   // committed: k_fibre moves its fibres
}

// Compliant tendons, after k_back: one thread per env and muscle (internal
// slot m) of an env whose step k_back committed. The fibre takes a
// backward-Euler step: its new length l' = l + dt v_max l_opt v' balances
// fibre and tendon at the path length L + dt Ldot' (Ldot' = -r qd', moment
// arms of the step's start):
//   g(v') = a f_l(l') f_v(v') + f_p(l') + beta v' - f_t(L' - l') = 0.
// g rises strictly in v' (slope at least beta - 1.82 dt v_max > 0, checked
// by the entry point), below zero at v' = min(0, -(1.4 a + f_p(l)) / beta)
// - 1 and above it at max(0, f_t(L' - l) / beta) + 1. Newton's method from
// v' = 0, kept inside that shrinking bracket (a step that leaves it bisects
// instead), stops when a step moves the length by at most 2e-8 l (under
// half an ulp of l in float32) or v' by at most its own resolution. A
// length that is not finite is not written and flags the env (its skeleton
// state of this step stands).
__global__ __launch_bounds__(256) void k_fibre(KModel M, KRun Rn, KSplit W) {
  const int nm = M.n_mus;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int e0 = Rn.env_begin, e1 = Rn.env_end ? Rn.env_end : Rn.n_env;
  if (t >= (long long)(e1 - e0) * nm) return;
  const int env = e0 + (int)(t / nm), m = (int)(t % nm);
  if (W.mflag[env] != 4) return;
  const float dt = Rn.dt, beta = Rn.ten_beta, ieps = Rn.ten_ieps;
  const float *fb = Rn.fib + (size_t)env * Rn.fib_stride;
  const float *qd = Rn.qd + (size_t)env * M.nv;
  float ld = 0.0f;
#pragma unroll
  for (int sl = 0; sl < 3; ++sl) {
    const int j = M.mus_span[sl * nm + m];
    if (j >= 0) ld -= fb[sl * nm + m] * qd[j];
  }
  const float Ln = fb[3 * nm + m] + dt * ld, a = fb[4 * nm + m];
  float *lp = Rn.lm + (size_t)env * nm + M.mus_ext[m];
  const float l = *lp, ls = M.mus_lslack[m], ilo = M.mus_ilopt[m];
  const float dl = dt / M.mus_ivl[m], dx = dl * ilo;   // d l' / d v', d (l' / l_opt) / d v'
  float lo = fminf(0.0f, -(1.4f * a + hill_fp(l * ilo)) / beta) - 1.0f;
  float hi = fmaxf(0.0f, fmaxf(0.0f, (Ln - l - ls) / ls) * ieps / beta) + 1.0f;
  float v = 0.0f;
  for (int it = 0; it < 64; ++it) {
    const float ln = l + dl * v, x = ln * ilo, e = (Ln - ln - ls) / ls;
    const float fl = hill_fl(x), fv = hill_fv(v);
    const float g = a * fl * fv + hill_fp(x) + beta * v - fmaxf(0.0f, e) * ieps;
    if (g < 0.0f)
      lo = v;
    else
      hi = v;
    const float gp = a * (hill_fl_slope(x) * dx * fv + fl * hill_fv_slope(v)) +
                     hill_fp_slope(x) * dx + beta + (e > 0.0f ? ieps * dl / ls : 0.0f);
    float vn = v - g / gp;
    if (!(vn > lo && vn < hi)) vn = 0.5f * (lo + hi);
    const float dv = fabsf(vn - v);
    const bool done = dv * dl <= 2e-8f * l || dv <= 2.4e-7f * fabsf(v);
    v = vn;
    if (done) break;
  }
  const float l1 = l + dl * v;
  if (isfinite(l1))
    *lp = l1;
  else if (Rn.status)
    atomicOr(Rn.status + env, MS_ST_NONFINITE);
}

namespace {
size_t front_lds(const KModel &k, const KSplit &w, int W) {
  return (size_t)k.lt_front_end * 4 + (size_t)W * w.f_bytes;
}
size_t back_lds(const KModel &k, const KSplit &w, int W) {
  return (size_t)(k.lt_words - k.lt_back_begin) * 4 + (size_t)W * w.b_bytes;
}
hipError_t allow_lds(const void *fn, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}
// Envs per workgroup (1..16) for n_env envs on n_cu CUs. With W envs per
// workgroup and nb workgroups resident per CU, the busiest CU receives
// ceil(ceil(n_env / W) / n_cu) workgroups and runs them in rounds of nb; a
// latency-bound kernel takes about as long per round whatever the round
// holds, but a fuller round shares each CU among more envs. The cost is
// rounds x (envs resident in a round); ties go to the larger W (fewer copies
// of the shared table). When the launch is one of several concurrent parts
// (fill), the cost is minus the envs resident per CU instead: the parts'
// kernels share the CUs, so what counts is how many envs a CU's LDS holds
// (measured on the whole body, 2 x 2048 envs: 10 envs per workgroup
// 0.298 ms per step against 8 per workgroup 0.307).
int best_w(const void *fn, size_t (*lds_of)(const KModel &, const KSplit &, int), const KModel &k,
           const KSplit &w, int n_env, int n_cu, bool fill) {
  int best = 1;
  long long best_cost = -1;
  for (int W = 1; W <= 16; ++W) {
    const size_t lds = lds_of(k, w, W);
    if (lds > 160 * 1024) break;
    if (allow_lds(fn, lds) != hipSuccess) break;
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, 64 * W, lds) != hipSuccess) break;
    if (nb <= 0) continue;
    const long long wgs = (n_env + W - 1) / W, wgs_cu = (wgs + n_cu - 1) / n_cu;
    const long long rounds = (wgs_cu + nb - 1) / nb;
    const long long cost = fill ? -(long long)nb * W : rounds * std::min<long long>(nb, wgs_cu) * W;
    if (best_cost < 0 || cost <= best_cost) {
      best = W;
      best_cost = cost;
    }
  }
  return best;
}
}  // namespace

int device_cu_count() {
  int dev = 0, n_cu = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      n_cu = v;
  }
  return n_cu;
}

void split_env_per_wg(const KModel &k, const KSplit &w, int n_env, int parts, int *w_front,
                      int *w_back) {
  const int n_cu = device_cu_count();
  *w_front = best_w((const void *)&k_front, front_lds, k, w, n_env, n_cu, parts > 1);
  *w_back = best_w((const void *)&k_back, back_lds, k, w, n_env, n_cu, parts > 1);
}

hipError_t launch_fibre(const KModel &k, const KRun &r, const KSplit &w, hipStream_t st) {
  const long long n = (long long)((r.env_end ? r.env_end : r.n_env) - r.env_begin) * k.n_mus;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fibre, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, k, r, w);
  return hipGetLastError();
}

hipError_t launch_front(const KModel &k, const KRun &r, const KSplit &w, int W, int step,
                        hipStream_t st) {
  const size_t lds = front_lds(k, w, W);
  hipError_t e = allow_lds((const void *)&k_front, lds);
  if (e != hipSuccess) return e;
  const int n = (r.env_end ? r.env_end : r.n_env) - r.env_begin;
  hipLaunchKernelGGL(k_front, dim3((n + W - 1) / W), dim3(64 * W), lds, st, k, r, w, step);
  return hipGetLastError();
}

hipError_t launch_back(const KModel &k, const KRun &r, const KSplit &w, int W, int step,
                       hipStream_t st) {
  const size_t lds = back_lds(k, w, W);
  hipError_t e = allow_lds((const void *)&k_back, lds);
  if (e != hipSuccess) return e;
  const int n = (r.env_end ? r.env_end : r.n_env) - r.env_begin;
  hipLaunchKernelGGL(k_back, dim3((n + W - 1) / W), dim3(64 * W), lds, st, k, r, w, step);
  return hipGetLastError();
}

}  // namespace ms
