// ms_step_types.h -- parameters of the step kernel (internal): the model
// tables as device pointers and scalars, and one launch's run arguments.
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/ms.h"
#include "ms_model.h"

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
      lt_subc, lt_nnzrow;
  int off_flag, off_q, off_qd, off_R, off_P, off_S, off_con, off_rhs, off_x, off_H,
      off_scr, off_V, off_A, off_F;
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
};

enum { EXC_ARRAY = MS_EXC_ARRAY, EXC_IID = MS_EXC_IID, EXC_AR1 = MS_EXC_AR1 };

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

}  // namespace ms

// The model object behind the C ABI's opaque handle.
struct ms_model {
  ms::Tables t;
  ms::KModel k;
  void *dbuf = nullptr;
  size_t dbytes = 0;
};

// Launch the step kernel variant the run arguments select (exact, surrogate
// or geometry only) for n_env envs and n_steps steps on stream st.
hipError_t launch(const ms_model *m, const ms::KRun &r, int n_env, int n_steps, hipStream_t st);

// ms_rollout with a chosen number of envs per workgroup (1, 2 or 4; 0 picks
// the count that keeps the most envs resident per CU); errors
// as ms_rollout (message in ms_last_error).
ms_status rollout_impl(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                       uint32_t *status, const ms_excitation *exc, int32_t n_steps,
                       const ms_step_opts *opts, int env_per_wg, hipStream_t st);
