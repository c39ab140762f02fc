// ms_step_types.h -- parameters of the step kernel (internal): the model
// tables as device pointers and scalars, and one launch's run arguments.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/ms.h"
#include "ms_model.h"

#include <vector>

namespace ms {

// ----------------------------------------------------------------- params
struct KModel {
  int n_node, nq, nv, n_mus, n_con, n_body, nnz, n_level, free_root, n_dent;
  float kc, cc, mu, vs, gx, gy, gz;
  const int *parent, *jtype, *qadr, *dadr, *level_start, *level_nodes;
  const float *jpos, *jrot, *axis;
  const int *body_node;
  const float *body_mass, *body_com, *body_inertia;
  const int *subb_start, *subb, *subc_start, *subc;
  const int *con_node;
  const float *con_pos, *con_radius;
  const int *dof_node, *dof_kind;
  const float *damping;
  const float *mus_f0, *mus_ilopt, *mus_lslack, *mus_ivl, *mus_tact, *mus_tdeact;
  const int *mus_nvia, *via_node, *mus_ext, *mus_int, *grp_nvia;
  const float *qlo, *qhi;
  const float *via_pos;
  const int *mus_span, *mus_srec;
  const unsigned *mus_mask;
  const int *proj_dof, *proj_start, *proj_item;
  const int *dent_h, *dent_start, *dent_item;
  const int *row_start, *dof_depth, *path, *nnz_row;
  int n_hlev, n_dlev, n_hgat, n_trunk;
  const int *hlev_start, *hlev_dof;
  // the factorisation's gather tables (staged in LDS per workgroup)
  const int *lt;
  int lt_words, lt_hent_start, lt_hlev_start, lt_hent, lt_hdof, lt_desc, lt_drange,
      lt_rs, lt_trow, lt_tpair, lt_path, lt_tlev, lt_tnode, lt_subb_start, lt_subc_start, lt_subb,
      lt_subc, lt_nnzrow, lt_cinode, lt_dofci, lt_front_end, lt_back_begin;
  int n_ci;
  int off_flag, off_q, off_qd, off_R, off_P, off_S, off_con, off_rhs, off_x, off_H,
      off_scr, off_V, off_A, off_F;
  // joint coupling (penalty equality constraints)
  int n_eq, n_eqd, n_eqh;
  float eq_k, eq_d;
  const int *eq_start, *eq_qi, *eq_dof, *eqd_start, *eqd_dof, *eqd_c, *eqh_h;
  const float *eq_coef, *eq_off, *eqd_coef, *eqh_w;
  // key nodes whose frames the observables record
  const int *key_node;
  int n_key;
  int lds_env;  // bytes of one env's LDS block
};

struct KRun {
  float *q, *qd, *act;
  unsigned *status;
  const float *u;  // array excitations
  int n_env;
  float dt;
  int contact;
  unsigned long long seed;
  long long step0;
  float *xar;
  float rho, s, mean;
  int exc;     // EXC_ARRAY, EXC_IID or EXC_AR1
  // surrogate geometry: predictions [n_env][4 n_mus] (caller's muscle
  // order, L then r[3]), fallback tolerance (m), fallback counters
  const float *geomY;
  float fb_tol;
  unsigned *fb_count;
  int stages;  // 1: write stage outputs, do not advance the state;
               // 2: geometry only (L, Ldot, r), nothing else
  // stage outputs (ms_step_stages)
  float *o_act, *o_L, *o_Ldot, *o_F, *o_r, *o_tau, *o_bias, *o_qdd;
  double *o_H;
  int env_per_wg;  // envs (wavefronts) per workgroup, 1, 2 or 4 (0: the most resident envs)
  int u_hold;      // array excitations: the same u[n_env][n_mus] for every step
  // per-step observables of steps t % rec_every == 0 (0: none), record
  // t / rec_every: muscle arrays [n_rec][n_env][n_mus] (caller's order), key
  // node frames [n_rec][n_env][n_key][3 | 9]; applied-step counters
  int rec_every;
  float *r_act, *r_F, *r_lm, *r_vm, *r_pow, *r_xpos, *r_xmat;
  unsigned *n_applied;
  // the split step's kernels cover envs [env_begin, env_end) of the batch
  // (env_end 0: up to n_env); every array stays indexed by the env's place
  // in the whole batch
  int env_begin, env_end;
  // split step: keep every kernel on the launch stream (no half-batch on
  // the model's second stream); set for launches an ms_batch drives
  int one_stream;
  // compliant tendons (split step only; lm NULL: rigid tendons): fibre
  // lengths lm[n_env][n_mus] (m, caller's muscle order), 1 / eps0 and the
  // fibre damping beta. The muscle kernel leaves, per env and internal
  // muscle slot m, fib[env * fib_stride + k * n_mus + m] for k = 0..4: the
  // moment arms r[3] of the span slots, the path length L and the
  // activation act' of the step, read by the fibre update after the solve.
  float *lm, *fib;
  int fib_stride;
  float ten_ieps, ten_beta;
};

// This env's slices of the muscle observables of one recorded step (NULL:
// not recorded).
struct RecOut {
  float *act, *F, *lm, *vm, *pw;
};

enum { EXC_ARRAY = MS_EXC_ARRAY, EXC_IID = MS_EXC_IID, EXC_AR1 = MS_EXC_AR1 };

// The split step's per-env device workspace (arrays [n_env][stride],
// strides in elements) and its kernels' LDS layouts (byte offsets into one
// env's block). The kinematics/dynamics kernel writes frames, S, H and rhs
// and flag; the muscle kernel writes tau, dsum, actn and mflag; the
// factorisation kernel reads them all.
struct KSplit {
  float *frames, *S, *tau, *actn;
  double *H, *rhs, *dsum;
  int *flag, *mflag;
  int fr_stride, S_stride, H_stride, rhs_stride, tau_stride, dsum_stride, act_stride;
  int f_R, f_S, f_con, f_scr, f_bytes;
  int b_q, b_qd, b_x, b_invd, b_H, b_bytes;
  int m_R, m_S, m_q, m_qd, m_scr, m_bytes;
};

// Envs per workgroup that keep the most envs resident per CU (160 KiB of
// LDS; the workgroup's copy of the factorisation tables is shared by its
// envs); ties go to fewer envs per workgroup.
inline int default_env_per_wg(const Tables &t) {
  int best = 1, most = 0;
  for (int w = 1; w <= 4; w *= 2) {
    const size_t per_wg = t.lt.size() * 4 + (size_t)w * t.lds_bytes;
    if (per_wg > 160 * 1024) break;
    const int envs = w * (int)((160 * 1024) / per_wg);
    if (envs > most) {
      most = envs;
      best = w;
    }
  }
  return best;
}

// Launch k_step (or k_step_surrogate when r.geomY is set) for a model whose
// muscles have at most NVIA via-points; one instantiation per translation
// unit (ms_step_v2/4/6/8.hip).
template <int NVIA>
hipError_t launch_nvia(const Tables &t, const KModel &k, const KRun &r, int n_env, int n_steps,
                       hipStream_t st);
extern template hipError_t launch_nvia<2>(const Tables &, const KModel &, const KRun &, int, int, hipStream_t);
extern template hipError_t launch_nvia<4>(const Tables &, const KModel &, const KRun &, int, int, hipStream_t);
extern template hipError_t launch_nvia<6>(const Tables &, const KModel &, const KRun &, int, int, hipStream_t);
extern template hipError_t launch_nvia<8>(const Tables &, const KModel &, const KRun &, int, int, hipStream_t);

// The split step's muscle kernel for step `step` (mpt muscles per thread).
template <int NVIA>
hipError_t launch_muscle(const KModel &k, const KRun &r, const KSplit &w, int mpt, int step,
                         hipStream_t st);
extern template hipError_t launch_muscle<2>(const KModel &, const KRun &, const KSplit &, int, int, hipStream_t);
extern template hipError_t launch_muscle<4>(const KModel &, const KRun &, const KSplit &, int, int, hipStream_t);
extern template hipError_t launch_muscle<6>(const KModel &, const KRun &, const KSplit &, int, int, hipStream_t);
extern template hipError_t launch_muscle<8>(const KModel &, const KRun &, const KSplit &, int, int, hipStream_t);

// The split step's kinematics/dynamics and factorisation kernels for step
// `step`, w_front / w_back envs per workgroup (ms_step_split.hip).
hipError_t launch_front(const KModel &k, const KRun &r, const KSplit &w, int w_front, int step,
                        hipStream_t st);
hipError_t launch_back(const KModel &k, const KRun &r, const KSplit &w, int w_back, int step,
                       hipStream_t st);
// The compliant-tendon fibre update (k_fibre) after launch_back, for the
// envs [r.env_begin, r.env_end) whose step k_back committed.
hipError_t launch_fibre(const KModel &k, const KRun &r, const KSplit &w, hipStream_t st);
// Envs per workgroup of those two kernels for a launch over n_env envs, one
// of `parts` concurrent parts: alone, the fewest rounds of resident envs on
// the device's CUs (occupancy calculator over 1..16 envs per workgroup),
// then the fewest envs per CU giving that many rounds; beside other parts,
// the most envs resident per CU.
void split_env_per_wg(const KModel &k, const KSplit &w, int n_env, int parts, int *w_front,
                      int *w_back);
// CUs of the current device (256 if the query fails).
int device_cu_count();

}  // namespace ms

// The model object behind the C ABI's opaque handle.
struct ms_model {
  ms::Tables t;
  ms::KModel k;
  void *dbuf = nullptr;
  size_t dbytes = 0;
  int schedule = MS_SCHED_AUTO;  // as set by ms_model_set_schedule
  // the split step's workspace for up to ws_cap envs (replaced buffers stay
  // allocated until destroy: queued launches may still use them)
  ms::KSplit ks{};
  int ws_cap = 0;
  std::vector<void *> ws_owned;
  // compliant-tendon fibre scratch for up to fib_cap envs (5 n_mus floats
  // each; replaced buffers stay in ws_owned)
  float *fib = nullptr;
  int fib_cap = 0;
  // envs per workgroup of its kernels, chosen for w_n_env envs in w_parts concurrent parts
  int w_front = 0, w_back = 0, w_n_env = 0, w_parts = 0;
  // the split step's second stream and its fork/join events (two halves of
  // the batch stepped concurrently)
  // split step: the batch in this many parts, each on a stream of its own
  // (the caller's, then the model's); 0 automatic (ms_model_set_split_streams)
  int split_streams = 0;
  static constexpr int kMaxParts = 4;
  hipStream_t sx[kMaxParts - 1] = {};            // the model's streams
  hipEvent_t ev_fork = nullptr, ev_join[kMaxParts - 1] = {};
  void *key_buf = nullptr;  // device copy of the key nodes
  // per-kernel timing of the split schedule (ms_model_set_kernel_timing):
  // event pairs recorded around each kernel, (kernel, start, end)
  int timing = 0;  // time every timing-th step of each call (0: off)
  std::vector<hipEvent_t> ev_free;
  struct Timed {
    int kernel;
    hipEvent_t a, b;
  };
  std::vector<Timed> ev_pending;
};

// The schedule a model's steps run with (MS_SCHED_FUSED or MS_SCHED_SPLIT).
int effective_schedule(const ms_model *m);

// Grow the split step's workspace to n_env envs (allocates; refused inside
// a stream capture on st, where no allocation may happen).
ms_status reserve_split(ms_model *m, int n_env, hipStream_t st);

// Launch the step for n_env envs and n_steps steps on stream st: the fused
// kernel variant the run arguments select (exact, surrogate or geometry
// only), or, for a model on the split schedule, its three kernels per step
// (stage outputs and geometry-only runs always use the fused kernel).
// Returns hipErrorOutOfMemory when the split workspace cannot be grown
// (message in ms_last_error).
hipError_t launch(ms_model *m, const ms::KRun &r, int n_env, int n_steps, hipStream_t st);
// launch() behind the C ABI: grows the split workspace first, returns an
// ms_status with the message in ms_last_error.
ms_status run_steps(ms_model *m, const ms::KRun &r, int n_env, int n_steps, hipStream_t st);

// ms_rollout with a chosen number of envs per workgroup (1, 2 or 4; 0 picks
// the count that keeps the most envs resident per CU), with one_stream,
// every kernel of the split step on st, and with lm, compliant tendons
// (ms_rollout_tendon, whose checks the caller has made); errors as
// ms_rollout (message in ms_last_error).
ms_status rollout_impl(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                       uint32_t *status, const ms_excitation *exc, int32_t n_steps,
                       const ms_step_opts *opts, int env_per_wg, hipStream_t st,
                       const ms_record *rec = nullptr, bool one_stream = false,
                       float *lm = nullptr, const ms_tendon *ten = nullptr);
