/*
 * ms.h -- C ABI of the MI355X batched musculoskeletal forward-dynamics step.
 *
 * One step advances E independent environments of one muscle-driven
 * articulated body (Methods, "Whole-body musculoskeletal model"):
 *   1. activation dynamics act' = act + dt (u - act) / tau(u, act)
 *      (Eq. excitation-activation; u clamped to [0, 1]);
 *   2. via-point muscle-tendon length L, moment arms r = -dL/dq (the
 *      moment-arm matrix J_m of the equations of motion) and Ldot;
 *   3. Hill force F = F_max [act' f_l(l_m) f_v(v_m) + f_p(l_m)] (Eq. flv);
 *   4. projection tau_mus = J_m^T F;
 *   5. generalized mass matrix M(q) (composite-rigid-body algorithm);
 *   6. bias C(q, qd) (Coriolis, centrifugal, gravity; recursive
 *      Newton-Euler);
 *   7. penalty ground contact tau_ext from spheres on the body (spring
 *      k and damper c per sphere, the spring taken linearly implicitly:
 *      F_n = max(0, k d - (c + dt k) zdot), regularised Coulomb friction);
 *   8. a Cholesky-type (LTDL) solve in FP64 of
 *      (M + dt D) qdd = tau_mus + tau_ext - b qd - C, D being the velocity
 *      slope of the dissipative forces (joint damping, muscle
 *      force-velocity, contact damping and friction) taken implicitly;
 *   9. semi-implicit Euler: qd += dt qdd, q += dt qd (root orientation by
 *      the quaternion exponential of the body angular velocity).
 * M(q) q'' + C(q, q') = J_m^T F + tau_ext is the paper's equation of motion
 * (Methods, "Musculoskeletal dynamics").
 *
 * Conventions
 *  - All state buffers are DEVICE pointers owned by the caller, float32,
 *    environment-major (structure of arrays per field):
 *      q[n_env][nq], qd[n_env][nv], act[n_env][n_mus], status[n_env] (u32).
 *    A free root stores q = (px, py, pz, qw, qx, qy, qz, hinges...) and
 *    qd = (world linear velocity, body angular velocity, hinge rates...).
 *  - Every call is asynchronous on `stream` (a hipStream_t passed as void*;
 *    NULL = the default stream) and never synchronises implicitly, except
 *    where a call says it allocates: create calls, reservations, and the
 *    workspace growth of the surrogate and policy calls (avoided by
 *    reserving first).
 *  - Calls return an ms_status; nothing throws across the ABI. On error the
 *    message is available from ms_last_error() (thread-local).
 *  - Per-environment numerical failures are not return codes: they are
 *    OR-ed into status[env] (MS_ST_*) and that env's state is left
 *    unchanged for the step.
 *  - A model is not safe for concurrent calls from several host threads.
 */
#ifndef MS_H
#define MS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MS_OK = 0,
  MS_E_ARG = -1,         /* invalid argument (NULL, size, dt, ...) */
  MS_E_ALLOC = -2,       /* device or host allocation failed */
  MS_E_HIP = -3,         /* a HIP runtime call failed */
  MS_E_MODEL = -4,       /* the model description is invalid */
  MS_E_UNSUPPORTED = -5  /* valid but beyond this library's limits */
} ms_status;

/* Per-env status bits. */
#define MS_ST_NONFINITE 1u /* non-finite state or result; step not applied */
#define MS_ST_NONSPD 2u    /* LTDL pivot <= 0; step not applied */
#define MS_ST_FALLBACK 4u  /* surrogate geometry replaced by the exact one in
                              some step (informational; the step is applied) */

/* Model description (host memory; deep-copied by ms_model_create).
 * Kinematic tree of n_node nodes in topological order (parent < child).
 * Node i frame = parent frame * (jrot_i, jpos_i) * joint motion, where a
 * hinge rotates by q about axis_i, a slide translates by q along axis_i,
 * and a free joint (node 0 only, parent -1) places the node at
 * (q0,q1,q2) with orientation quaternion (q3..q6). Mass properties,
 * via-points and contact spheres are given in node frames. */
typedef struct {
  int32_t n_node;
  const int32_t *parent;     /* [n_node], -1 = world */
  const int32_t *jtype;      /* [n_node]: 0 hinge, 1 slide, 2 free */
  const float *jpos;         /* [n_node][3] joint origin in the parent frame */
  const float *jrot;         /* [n_node][9] joint orientation, row-major */
  const float *axis;         /* [n_node][3] unit hinge/slide axis */
  const float *mass;         /* [n_node] kg (0 = massless frame) */
  const float *com;          /* [n_node][3] centre of mass, node frame */
  const float *inertia;      /* [n_node][3] principal moments at the COM */
  const float *damping;      /* [nv] joint damping b (N m s / rad) */
  const float *qlo, *qhi;    /* [nv] pose-domain limits of hinge/slide DoFs
                                (sampling box of the geometry surrogate and its
                                domain check; no limit forces); may be NULL */
  int32_t n_mus;
  const float *f0;           /* [n_mus] maximum isometric force (N) */
  const float *l_opt;        /* [n_mus] optimal fibre length (m) */
  const float *l_slack;      /* [n_mus] tendon slack length (m) */
  const float *v_max;        /* [n_mus] max shortening speed (l_opt / s) */
  const float *tau_act;      /* [n_mus] activation time constant (s) */
  const float *tau_deact;    /* [n_mus] deactivation time constant (s) */
  const int32_t *via_start;  /* [n_mus+1] CSR into the via-point arrays */
  const int32_t *via_node;   /* [n_via] node of each via-point, -1 = world */
  const float *via_pos;      /* [n_via][3] via-point in its node frame */
  int32_t n_con;
  const int32_t *con_node;   /* [n_con] node carrying each contact sphere */
  const float *con_pos;      /* [n_con][3] sphere centre in the node frame */
  const float *con_radius;   /* [n_con] sphere radius (m) */
  float contact[4];          /* stiffness k, damping c, friction mu, v_s */
  float gravity[3];          /* m/s^2, ground is the plane z = 0 */
  /* Anatomical joint coupling (Methods, "GPU-accelerated simulation
   * framework": anatomical joint coupling such as the scapulohumeral rhythm)
   * as equality constraints phi_c(q) = sum over the terms t of constraint c
   * of eq_coef[t] q(eq_dof[t]) - eq_off[c] = 0, enforced by a penalty:
   * tau = -J^T (eq_k phi + (eq_d + dt eq_k) J q'), J[c][eq_dof[t]] = eq_coef[t],
   * with its velocity slope (eq_d + dt eq_k) J^T J taken implicitly into the
   * step's matrix (the spring linearly implicit, as the contact spring is).
   * Terms of constraint c are eq_start[c] .. eq_start[c+1]-1; eq_dof are
   * hinge/slide DoFs (not a free root's), and every two DoFs of one
   * constraint must lie on one root-to-leaf path (so the matrix keeps its
   * tree sparsity). n_eq = 0 (or a zero-initialised tail) means none.
   * Limits: n_eq <= 64, at most 8 terms per constraint. */
  int32_t n_eq;
  const int32_t *eq_start;   /* [n_eq + 1] */
  const int32_t *eq_dof;     /* [eq_start[n_eq]] */
  const float *eq_coef;      /* [eq_start[n_eq]] */
  const float *eq_off;       /* [n_eq] */
  float eq_k;                /* N m / rad (per unit of phi), >= 0 */
  float eq_d;                /* N m s / rad, >= 0 */
} ms_model_desc;

typedef struct ms_model ms_model;

typedef struct {
  int32_t nq, nv, n_node, n_mus, n_con, n_body;
  int32_t max_dof_depth;   /* longest root-to-leaf DoF chain */
  int32_t nnz_mass;        /* stored entries of the tree-sparse M */
  int32_t lds_bytes;       /* per-environment LDS footprint of the step */
  int32_t lds_shared_bytes; /* LDS table shared by a workgroup's envs: a
                               workgroup of W envs takes lds_shared_bytes +
                               W * lds_bytes (at most 160 KiB) */
} ms_model_info;

typedef struct {
  float dt;            /* step (s), > 0 and finite */
  int32_t contact;     /* 1 = ground contact on, 0 = off */
} ms_step_opts;

/* Excitation source for ms_rollout. */
typedef enum {
  MS_EXC_ARRAY = 0,  /* u[n_steps][n_env][n_mus] float32 in device memory */
  MS_EXC_IID = 1,    /* u = top 24 bits of SplitMix64(key ^ m) * 2^-24 */
  MS_EXC_AR1 = 2     /* smooth noise x <- rho x + s xi, u = clamp(mean + x) */
} ms_exc_kind;

typedef struct {
  int32_t kind;          /* ms_exc_kind */
  const float *u;        /* MS_EXC_ARRAY: device [n_steps][n_env][n_mus] */
  uint64_t seed;         /* generators: key = SplitMix64(SplitMix64(seed ^ env) ^ step) */
  int64_t step0;         /* absolute index of the rollout's first step */
  float *x;              /* MS_EXC_AR1: device noise state [n_env][n_mus] (in/out) */
  float rho, s, mean;    /* MS_EXC_AR1 constants (float32) */
} ms_excitation;

/* Validate a description, build the device tables (tree levels, muscle
 * spans and moment-arm reduction lists, the tree-sparse M pattern) and
 * upload them. Returns MS_E_MODEL on an invalid description and
 * MS_E_UNSUPPORTED beyond the limits (nodes <= 128, nv <= 128,
 * muscles <= 1024, 2..8 via-points, a muscle spans <= 3 DoFs, contacts <=
 * 64, tree depth <= 64). Synchronous. */
ms_status ms_model_create(const ms_model_desc *desc, ms_model **out);

/* Free the model and its device tables. NULL-safe. */
void ms_model_destroy(ms_model *m);

/* Step schedules (the same operations in the same order, so the same
 * results bit for bit; they differ in speed):
 *  MS_SCHED_FUSED: one kernel per rollout, one wavefront per env with the
 *    whole step's intermediates in LDS and the state on chip across steps;
 *  MS_SCHED_SPLIT: three kernels per physics step (kinematics and dynamics;
 *    muscles, one 256-thread workgroup per env; LTDL factorisation, solve
 *    and update), exchanging per-env intermediates (about 26 KB per env at
 *    80 DoF / 700 muscles) through a device workspace the model owns;
 *    smaller LDS blocks keep more envs resident per CU;
 *  MS_SCHED_AUTO (default): SPLIT for models whose fused step keeps at most
 *    four envs resident per CU (one wavefront per SIMD), else FUSED.
 * Stage outputs (ms_step_stages) and ms_geometry always use the fused
 * kernel. Set before use; MS_E_ARG for an unknown value. */
#define MS_SCHED_AUTO 0
#define MS_SCHED_FUSED 1
#define MS_SCHED_SPLIT 2
ms_status ms_model_set_schedule(ms_model *m, int32_t schedule);
/* Split schedule only: streams = P (1 to 4) steps the batch in P contiguous
 * parts concurrently, the first on the caller's stream and the others on
 * streams of the model's own (forked from and joined back to the caller's
 * with events, so stream order and graph capture hold); 0 (default) uses
 * two parts for batches of at least 4096 envs and one below (the part sizes:
 * ms_model_split_parts). Launches that an ms_batch drives use one stream.
 * Results do not depend on it. */
ms_status ms_model_set_split_streams(ms_model *m, int32_t streams);
/* The parts a step of n_env envs (not driven by an ms_batch, not under
 * capture) runs in with the current settings (one on the fused schedule): *n_parts (1 to 4)
 * and bounds[0 .. *n_parts] (bounds[h] .. bounds[h + 1] are part h's envs;
 * bounds holds at least 5 entries). Equal parts, except that with two parts
 * the first takes one full round of the kinematics kernel when that holds
 * more than half the batch. For callers that time or size per part. */
ms_status ms_model_split_parts(ms_model *m, int32_t n_env, int32_t *bounds, int32_t *n_parts);
/* The schedule the model's steps use now (MS_SCHED_FUSED or MS_SCHED_SPLIT). */
ms_status ms_model_get_schedule(const ms_model *m, int32_t *schedule);
/* Reserve the split schedule's workspace for up to n_env envs now
 * (synchronous allocation). A step or rollout on the split schedule with
 * more envs than reserved grows it first (allocating and synchronising);
 * inside a stream capture that growth is refused with MS_E_ARG, so reserve
 * before capturing. All buffers of a growth are taken or none (MS_E_ALLOC
 * keeps the previous workspace). */
ms_status ms_model_reserve(ms_model *m, int32_t n_env);
/* Per-kernel timing of the split schedule, for measurement: with every =
 * N > 0, every N-th step of each later split call (steps 0, N, 2N, ... of
 * the call; outside stream captures) records a pair of HIP events around
 * each of its three kernels on the launch stream (each pair costs a few
 * microseconds of gap between kernels, so sampling keeps the overhead
 * small); every = 0 turns it off (the default). ms_model_kernel_times waits
 * for the recorded events, writes the summed durations in milliseconds of
 * the kinematics/dynamics, muscle and factorisation kernels to ms3[0..2]
 * and the number of steps timed to *n_steps, and starts a new count. */
ms_status ms_model_set_kernel_timing(ms_model *m, int32_t every);
ms_status ms_model_kernel_times(ms_model *m, double *ms3, int64_t *n_steps);

ms_status ms_model_info_get(const ms_model *m, ms_model_info *out);

/* One step for n_env envs, in place on the caller's device state, reading
 * excitations u[n_env][n_mus] (device). env i uses row i of every array.
 * status may be NULL (failures then go unreported; the failed env's state
 * is still left unchanged for the step); an env whose status already has
 * bits set is stepped like any other. MS_E_ARG, before any launch and with
 * no state touched: NULL model, n_env <= 0, a NULL state pointer (act and u
 * may be NULL only for a model without muscles), NULL opts, dt not positive
 * and finite. */
ms_status ms_step_batch(ms_model *m, int32_t n_env, float *q, float *qd,
                        float *act, uint32_t *status, const float *u,
                        const ms_step_opts *opts, void *stream);

/* n_steps steps for n_env envs in one launch, the state kept on chip
 * between steps; excitations from exc. Bitwise equal to n_steps calls of
 * ms_step_batch with the same excitations. n_steps = 0 does nothing.
 * MS_E_ARG as for ms_step_batch, and for a NULL exc, n_steps < 0, an
 * unknown exc->kind, MS_EXC_ARRAY without exc->u or MS_EXC_AR1 without
 * exc->x. */
ms_status ms_rollout(ms_model *m, int32_t n_env, float *q, float *qd,
                     float *act, uint32_t *status, const ms_excitation *exc,
                     int32_t n_steps, const ms_step_opts *opts, void *stream);

/* Per-step observables of a rollout (Methods, "Observation space": muscle
 * activation, force, fibre length and velocity, and key-body positions and
 * orientations; the power term |F_m v_m| of the reward in "Analysis of
 * neuro-actuated musculoskeletal dynamics"), written structure-of-arrays
 * for the steps t = 0, every, 2 every, ... of the call (t counted from the
 * call's first step; n_rec = ceil(n_steps / every) records; record
 * t / every). Device buffers owned by the caller, each may be NULL:
 *   act[n_rec][n_env][n_mus]   activation act' driving step t's force
 *   force[n_rec][n_env][n_mus] F (N)
 *   lm, vm [n_rec][n_env][n_mus] fibre length / l_opt and lengthening
 *                              velocity / (v_max l_opt) (rigid tendon)
 *   power[n_rec][n_env][n_mus] |F Ldot| (W), Ldot the path lengthening
 *                              rate (the fibre's, under a rigid tendon)
 *   xpos[n_rec][n_env][n_key][3], xmat[n_rec][n_env][n_key][9] (row-major)
 *                              world frame of each key node (the model's
 *                              key nodes, ms_model_set_key_nodes) at the
 *                              step's start
 * in the caller's muscle order. A step an env does not take (a status bit
 * set at its start) leaves that env's entries unwritten.
 *   n_applied[n_env] (u32)     += the number of steps applied to each env
 *                              (state advanced), whatever `every` is. */
typedef struct {
  int32_t every;
  float *act, *force, *lm, *vm, *power;
  float *xpos, *xmat;
  uint32_t *n_applied;
} ms_record;

/* Key nodes whose frames ms_rollout_record writes (host nodes[n_key], node
 * indices, 0 <= n_key <= 64; 0 clears them). Synchronises the device. */
ms_status ms_model_set_key_nodes(ms_model *m, int32_t n_key, const int32_t *nodes);

/* ms_rollout that also writes the observables rec asks for (rec may be
 * NULL: ms_rollout). MS_E_ARG as for ms_rollout, and for rec->every < 1
 * with an observable requested, or key-node observables on a model without
 * key nodes. The state advances exactly as with ms_rollout. */
ms_status ms_rollout_record(ms_model *m, int32_t n_env, float *q, float *qd,
                            float *act, uint32_t *status, const ms_excitation *exc,
                            int32_t n_steps, const ms_step_opts *opts,
                            const ms_record *rec, void *stream);

/* Compliant tendons, a higher-fidelity variant of the Hill muscle-tendon
 * unit (Methods, "Whole-body musculoskeletal model": muscle-tendon units
 * driven by activation; the rigid tendon of ms_rollout is the paper's).
 * Each muscle carries a fibre length lm (m) as a state. The tendon is
 * linear above its slack length l_slack, with strain eps0 at F0, and
 * carries no force below it:
 *   F_t = F0 max(0, (L - lm - l_slack) / l_slack) / eps0.
 * The fibre (no pennation) obeys the damped balance
 *   F0 [act f_l(lm / l_opt) f_v(v) + f_p(lm / l_opt) + beta v]
 * with v its velocity in v_max l_opt. At the start of a step v balances the
 * fibre against the tendon (a closed-form root: the balance is strictly
 * increasing in v). The tendon (slope k) and the fibre (slope b) act in
 * series on the skeleton, as a force F_t + c (Ldot' - v) of the new
 * lengthening rate Ldot', with c = k dt / (1 + k dt / b). Its explicit part
 * goes into the right-hand side, c into the implicit muscle damping
 * J_m^T c J_m. After the solve each fibre takes a backward-Euler step: its
 * new length balances fibre and tendon at the path length L + dt Ldot',
 * Ldot' = -r qd' (moment arms of the step's start); on a linear element
 * this moves the fibre by dt (v + (c / b) (Ldot' - v)). */
typedef struct {
  float eps0; /* tendon strain at F0 (> 0; 0.033 is the usual value) */
  float beta; /* fibre damping in F0 per v_max l_opt (> 0; 0.1 is usual) */
} ms_tendon;

/* ms_rollout with compliant tendons. lm[n_env][n_mus] (device, float32,
 * caller's muscle order) holds the fibre lengths in metres and advances
 * with the state. An env that fails a step keeps its whole state, lm
 * included, as in ms_rollout; a fibre length that comes out of the fibre
 * update not finite (after the skeleton's step is committed) stays at its
 * old value and sets MS_ST_NONFINITE, which stops the env from the next
 * step on. Always on the split schedule, the batch in
 * stream parts as ms_rollout's. The first call with more envs than before
 * allocates a fibre scratch of 20 n_mus bytes per env, and synchronises;
 * inside a stream capture that growth is refused (MS_E_ARG), so a captured
 * rollout needs an eager call of at least as many envs before it.
 * rec (may be NULL) records observables as in ms_rollout_record, with the
 * compliant unit's meanings: force is the force of the step's right-hand
 * side F_t + c (Ldot - v), lm the fibre length / l_opt and vm the balancing
 * fibre velocity / (v_max l_opt) at the step's start, power |force Ldot|.
 * MS_E_ARG as for ms_rollout_record, and for ten or lm NULL, eps0 or beta not
 * positive and finite, a model with a muscle whose l_slack <= 0, or
 * beta <= 1.82 dt v_max for some muscle (the fibre balance then need not
 * rise strictly in the fibre velocity). */
ms_status ms_rollout_tendon(ms_model *m, int32_t n_env, float *q, float *qd,
                            float *act, float *lm, uint32_t *status,
                            const ms_excitation *exc, int32_t n_steps,
                            const ms_step_opts *opts, const ms_tendon *ten,
                            const ms_record *rec, void *stream);

/* Stage outputs of one step for n_env envs (device buffers, any may be
 * NULL): activation act'[E][n_mus], L, Ldot, F [E][n_mus], moment arms
 * r[E][n_mus][3] with their DoF indices from ms_model_spans, tau_mus[E][nv],
 * bias_minus_ext[E][nv] = C - tau_ext, qdd[E][nv], and the tree-sparse
 * (M + dt D) as mass[E][nnz] (float64) with its pattern from
 * ms_model_mass_pattern. The state is not advanced. */
typedef struct {
  float *act, *L, *Ldot, *F, *r, *tau_mus, *bias_minus_ext, *qdd;
  double *mass;
} ms_stage_out;
ms_status ms_step_stages(ms_model *m, int32_t n_env, const float *q,
                         const float *qd, const float *act, const float *u,
                         const ms_step_opts *opts, ms_stage_out *out,
                         void *stream);

/* Exact muscle geometry only, for n poses q[n][nq] (device): lengths
 * L[n][n_mus] and moment arms r[n][n_mus][3] in the DoF slots of
 * ms_model_spans (device outputs). Labels for the geometry surrogate. */
ms_status ms_geometry(ms_model *m, int32_t n, const float *q, float *L, float *r,
                      void *stream);

/* Host copies of the derived tables: spans[n_mus][3] DoF indices (-1 pad);
 * the sparse mass pattern rows[nnz], cols[nnz] (row >= col). */
ms_status ms_model_spans(const ms_model *m, int32_t *spans);
ms_status ms_model_mass_pattern(const ms_model *m, int32_t *rows,
                                int32_t *cols);

/* Last error message of this thread ("" if none). */
const char *ms_last_error(void);

/* ------------------------------------------------------------------------
 * Learned muscle-geometry surrogate (replaces the via-point geometry of
 * step 2 by a pose -> (L, moment arms) network; the paper names the
 * muscle-tendon path routing as the costly part of musculoskeletal
 * simulation). Multilayer perceptron x -> SiLU(W1 x + b1) ->
 * SiLU(W2 h1 + b2) -> W3 h2 + b3 with x the hinge/slide coordinates, each
 * mapped from its pose box [qlo, qhi] onto [-1, 1] (float32: (q - c) * is,
 * c = 0.5f (lo + hi), is = 2.0f / (hi - lo)), padded to a multiple of 16,
 * and n_out = 4 n_mus outputs per pose: lengths L[n_mus]
 * then moment arms r[n_mus][3] in the span slots of ms_model_spans (empty
 * slots masked), standardised by (mean, std). bfloat16 matrix-core GEMMs
 * with float32 accumulation; float32 master weights stored [out][in];
 * Adam (Kingma & Ba 2015; beta 0.9/0.999, eps 1e-8) with bias correction.
 * Weights start LeCun-uniform from `seed`, biases zero. */
typedef struct ms_surrogate ms_surrogate;
ms_status ms_surrogate_create(const ms_model *m, int32_t hidden, uint64_t seed,
                              ms_surrogate **out);
void ms_surrogate_destroy(ms_surrogate *s);
/* dims[4] = n_in, hidden, hidden, n_out */
ms_status ms_surrogate_dims(const ms_surrogate *s, int32_t *dims);
/* host copies of the float32 parameters (set = 0 reads, 1 writes);
 * W1[hidden][n_in], W2[hidden][hidden], W3[n_out][hidden] */
ms_status ms_surrogate_params(ms_surrogate *s, int32_t set, float *W1, float *b1,
                              float *W2, float *b2, float *W3, float *b3);
/* host copies of the gradients of the last training step */
ms_status ms_surrogate_grads(ms_surrogate *s, float *W1, float *b1, float *W2,
                             float *b2, float *W3, float *b3);
/* output standardisation (host [n_out]; std > 0) */
ms_status ms_surrogate_set_norm(ms_surrogate *s, const float *mean, const float *std);
/* n poses uniform in the model's pose-domain box (device q[n][nq]); pose p
 * uses SplitMix64(SplitMix64(seed ^ (offset + p)) ^ input index) */
ms_status ms_surrogate_sample(ms_surrogate *s, int32_t n, uint64_t seed, int64_t offset,
                              float *q, void *stream);
/* predictions for n poses q[n][nq] (device): L[n][n_mus], r[n][n_mus][3] */
ms_status ms_surrogate_forward(ms_surrogate *s, int32_t n, const float *q, float *L,
                               float *r, void *stream);
/* Reserve the surrogate's workspace for batches of up to n poses now
 * (synchronous device allocation), so that later forward, train-step and
 * surrogate-rollout calls of at most n poses/envs allocate nothing. Those
 * calls grow the workspace themselves when n exceeds it, and that growth
 * allocates and synchronises. All buffers of a growth are taken or none:
 * on MS_E_ALLOC the previous workspace stays in use. */
ms_status ms_surrogate_reserve(ms_surrogate *s, int32_t n);
/* ms_surrogate_forward for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): it calls no allocating routine and takes its intermediate
 * buffers (packed inputs and both hidden layers; the output layer writes L
 * and r) from a static device array of 16 MiB per GPU, held until the
 * process ends. The caller still passes inputs and outputs. n is limited to
 * what fits that array, ms_surrogate_noalloc_max(s) poses (7,598 for a
 * 74-input, 512-wide network); larger n returns MS_E_UNSUPPORTED with nothing
 * launched. Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (several streams or host threads) race and
 * must be serialised by the caller. Results equal ms_surrogate_forward's
 * bit for bit (the same kernels). */
ms_status ms_surrogate_forward_noalloc(ms_surrogate *s, int32_t n, const float *q,
                                       float *L, float *r, void *stream);
/* Largest n ms_surrogate_forward_noalloc accepts for this network. */
int32_t ms_surrogate_noalloc_max(const ms_surrogate *s);
/* one training step on n poses (n a multiple of 8, at most 2^20: the
 * weight gradients take the batch as a row length) with exact labels
 * L, r (device, as from ms_geometry): loss = mean over (pose, output) of
 * mask (y - t)^2 on standardised targets t, written to *loss (device) if
 * non-NULL; then an Adam step with learning rate lr at step count
 * `step` >= 1 (lr = 0: gradients only). */
ms_status ms_surrogate_train_step(ms_surrogate *s, int32_t n, const float *q,
                                  const float *L, const float *r, float lr,
                                  int32_t step, float *loss, void *stream);
/* Training on the GPU with exact labels (the geometry the network
 * replaces): every step samples `batch` poses uniformly in the pose box
 * (ids (step * batch + i) mod n_samples of `seed`, as ms_surrogate_sample),
 * labels them with ms_geometry and takes one Adam step (ms_surrogate_
 * train_step) with the learning rate lr1 + (lr0 - lr1)(1 + cos(pi it /
 * iters)) / 2 at step count step0 + it + 1. With norm_samples > 0 the
 * output standardisation is first set from that many poses of norm_seed:
 * mean, then the standard deviation about it (at least 1e-6), summed in a
 * fixed order; empty moment-arm slots get mean 0 and std 1. loss (device
 * [iters], may be NULL) receives each step's loss. Asynchronous on stream;
 * grows the workspace to `batch` first if needed (allocating and
 * synchronising; see ms_surrogate_reserve). */
typedef struct {
  int64_t n_samples;
  int32_t batch, iters, step0, norm_samples;
  float lr0, lr1;
  uint64_t seed, norm_seed;
  float *loss;
} ms_train_cfg;
ms_status ms_surrogate_train(ms_model *m, ms_surrogate *s, const ms_train_cfg *cfg,
                             void *stream);
/* The network as one plain little-endian binary blob: a header of eight
 * u32 (magic "MSG1" = 0x4D534731, version 1, n_in, hidden, hidden, n_out, 0,
 * 0), then float32 W1 [hidden][n_in], b1, W2, b2, W3 [n_out][hidden], b3,
 * the output mean and std. ms_surrogate_save writes it to blob (host, cap
 * bytes) and its size to *size; blob = NULL queries the size. Both
 * synchronise the device. ms_surrogate_load reads a blob of a network with
 * the same layer sizes (else MS_E_ARG). */
ms_status ms_surrogate_save(ms_surrogate *s, void *blob, size_t cap, size_t *size);
ms_status ms_surrogate_load(ms_surrogate *s, const void *blob, size_t size);
const char *ms_surrogate_last_error(void);

/* ------------------------------------------------------------------------
 * Policy-driven rollouts (the RL rollout shape of the paper's Methods:
 * Observation space, Action space, Simulation parameters for the control
 * rate). A policy network maps each env's observation to excitations:
 * obs -> SiLU(W1 obs + b1) -> SiLU(W2 h1 + b2) -> sigmoid(W3 h2 + b3), one
 * excitation in [0, 1] per muscle (caller's order), bfloat16 matrix-core
 * GEMMs with float32 accumulation, LeCun-uniform random weights from `seed`
 * (W stored [out][in]); it is not trained here (the paper's RL training is
 * out of scope).
 * Observation of env e at time t, n_obs = 2 nv + n_ref values: the
 * generalised position with a free root's unit quaternion (w >= 0 branch)
 * folded into its rotation vector (nv values), the generalised velocity (nv
 * values), and n_ref reference targets r_k(t) = sum_{j<3} A sin(2 pi f t +
 * phi) with A = 0.3 a, f = 0.5 + 1.5 b, phi = 2 pi c, where a, b, c are the
 * top 24 bits x 2^-24 of SplitMix64(K ^ 0), (K ^ 1), (K ^ 2) and K =
 * SplitMix64(SplitMix64(ref_seed ^ env) ^ (3 k + j)): a synthetic stand-in
 * for the retargeted reference motion. */
typedef struct ms_policy ms_policy;
ms_status ms_policy_create(const ms_model *m, int32_t hidden, int32_t n_ref,
                           uint64_t ref_seed, uint64_t seed, ms_policy **out);
void ms_policy_destroy(ms_policy *p);
/* Reserve the policy's workspace for up to n envs now (synchronous
 * allocation); ms_policy_act and ms_policy_rollout grow it themselves when
 * n exceeds it, allocating and synchronising, all buffers or none. */
ms_status ms_policy_reserve(ms_policy *p, int32_t n);
/* dims[4] = n_obs, n_in (n_obs padded to a multiple of 16), hidden, n_mus */
ms_status ms_policy_dims(const ms_policy *p, int32_t *dims);
/* host copies of the float32 parameters (set = 0 reads, 1 writes); W1 is
 * [hidden][n_in]; its columns beyond n_obs meet zero inputs */
ms_status ms_policy_params(ms_policy *p, int32_t set, float *W1, float *b1,
                           float *W2, float *b2, float *W3, float *b3);
/* u[n][n_mus] (device) for n envs with global indices env0.. at time t;
 * obs_out (device [n][n_obs], may be NULL) receives the observations. */
ms_status ms_policy_act(ms_policy *p, int32_t n, const float *q, const float *qd,
                        double t, int64_t env0, float *u, float *obs_out,
                        void *stream);
/* n_steps steps of n_env envs driven by the policy: every `decim` steps
 * (from step 0) the policy maps the current state at time t0 + step dt to
 * excitations, held for the next decim steps. Geometry: exact when s is
 * NULL, else the surrogate with per-env fallback exactly as in
 * ms_rollout_surrogate (tol, fallback_count, sentinel step = step index).
 * u_record (device, may be NULL) receives each decision's excitations,
 * [ceil(n_steps / decim)][n_env][n_mus]. */
ms_status ms_policy_rollout(ms_model *m, ms_policy *p, ms_surrogate *s,
                            int32_t n_env, float *q, float *qd, float *act,
                            uint32_t *status, int32_t n_steps, int32_t decim,
                            double t0, const ms_step_opts *opts, float tol,
                            uint32_t *fallback_count, float *u_record,
                            void *stream);

/* ------------------------------------------------------------------------
 * The control step around the physics (Methods: "Observation space",
 * "Action space", "Unified imitation environment", "Reinforcement learning
 * with flow-based exploration"; "Simulation parameters" for the substeps).
 * Per call and env, at time t (control step index ctl_step):
 *  1. observation s (n_obs values): q with a free root's unit quaternion as
 *     its rotation vector (nv), q' (nv), key-node world positions (3 n_key)
 *     and orientations as the first two columns of R, column by column
 *     (6 n_key), the muscle state of the previous call's last substep from
 *     mstate: activations, forces / F0, normalised fibre lengths and
 *     velocities (4 n_mus, caller's order), the hinges' reference targets
 *     (n_h, hinge coordinates in node order), and the key-node positions and
 *     orientations of the reference pose (the env's root, hinges at their
 *     targets; 9 n_key). Reference target of hinge h of env e at time t:
 *     sum over j < 3 of A sin(2 pi f t + phi), A = 0.3 a, f = 0.5 + 1.5 b Hz,
 *     phi = 2 pi c, a, b, c the top 24 bits x 2^-24 of SplitMix64(K ^ 0),
 *     (K ^ 1), (K ^ 2), K = SplitMix64(SplitMix64(ref_seed ^ e) ^ (3 h + j)):
 *     a synthetic stand-in for the retargeted reference motion;
 *  2. excitations (unless u_in is given): a0 = mu(s) + exp(log_std) xi from
 *     the initial sampler (mu its network's output, xi standard normal by the
 *     Box-Muller transform sqrt(-2 ln u1) cos(2 pi u2) of u1 = (i1 + 1/2)
 *     2^-24, u2 = (i2 + 1/2) 2^-24, i1 = z >> 40, i2 = (z >> 16) & 0xFFFFFF,
 *     z = SplitMix64(SplitMix64(SplitMix64(noise_seed ^ e) ^ ctl_step) ^ m)),
 *     refined by flow_steps explicit Euler steps of the flow velocity field
 *     a += flow_dt psi(t_k, s, a), t_k = k flow_dt (Eq. pi_ode), psi the flow
 *     network on [s, a, t_k] (padded to n_in + n_at), then u = clamp(a, 0, 1);
 *  3. n_sub physics substeps of dt with u held (status, n_applied as for
 *     ms_rollout); the last substep's muscle state goes to mstate;
 *  4. reward r = -log(1 - D(Delta)) = softplus(z) (Eq. tracking_r), z the
 *     discriminator network's output on the tracking error Delta = [hinge
 *     coordinates - their targets (n_h), key-node positions - the reference
 *     pose's (3 n_key)] at t + n_sub dt (padded to n_din).
 * Networks: three layers, SiLU hidden layers, linear outputs, bfloat16
 * matrix-core GEMMs with float32 accumulation, LeCun-uniform weights from
 * their seeds (the flow's first layer over all n_obs + n_mus + 1 inputs),
 * zero biases; log_std = log(sigma0). No training here. */
typedef struct ms_controller ms_controller;
typedef struct {
  int32_t hidden;          /* hidden width of every network (multiple of 8) */
  int32_t n_sub;           /* physics substeps per control step (>= 1) */
  int32_t flow_steps;      /* Euler steps of the flow (>= 0) */
  float flow_dt;           /* their step (>= 0) */
  float sigma0;            /* initial sampler's standard deviation (> 0) */
  int32_t n_key;           /* key nodes (<= 64) */
  const int32_t *key_nodes; /* host [n_key] */
  uint64_t ref_seed, noise_seed, pi_seed, flow_seed, disc_seed;
} ms_controller_desc;
/* Optional device outputs of a control step (each may be NULL): obs
 * [n_env][n_obs], a0 [n_env][n_mus] (initial sample), u [n_env][n_mus]
 * (excitations applied), delta [n_env][n_h + 3 n_key], n_applied [n_env]. */
typedef struct {
  float *obs, *a0, *u, *delta;
  uint32_t *n_applied;
} ms_ctl_out;
ms_status ms_controller_create(ms_model *m, const ms_controller_desc *d, ms_controller **out);
void ms_controller_destroy(ms_controller *c);
/* dims[6] = n_obs, n_in, n_at, n_din, hidden, n_h */
ms_status ms_controller_dims(const ms_controller *c, int32_t *dims);
/* host copies of a network's float32 parameters (which: 0 initial sampler,
 * 1 flow, 2 discriminator; set = 0 reads, 1 writes): W[l] [out][in], b[l];
 * the flow's W[0] is its observation block [hidden][n_in] and w_at (may be
 * NULL) its (action, time) block [hidden][n_at] (held in bfloat16); log_std
 * [n_mus] for which = 0 (may be NULL). */
ms_status ms_controller_params(ms_controller *c, int32_t which, int32_t set, float **W,
                               float **b, float *w_at, float *log_std);
/* Reserve the controller's and its model's workspaces for n_env envs. */
ms_status ms_controller_reserve(ms_controller *c, int32_t n_env);
/* One control step of n_env envs (state as ms_rollout; mstate device
 * [4][n_env][n_mus] in/out, zeros before the first step; reward device
 * [n_env]; u_in device [n_env][n_mus] or NULL). Asynchronous on stream;
 * grows the workspaces when n_env exceeds them (allocating). */
ms_status ms_controller_step(ms_controller *c, int32_t n_env, float *q, float *qd, float *act,
                             uint32_t *status, float *mstate, int64_t ctl_step, double t,
                             const ms_step_opts *opts, const float *u_in, float *reward,
                             const ms_ctl_out *out, void *stream);
const char *ms_controller_last_error(void);

/* ------------------------------------------------------------------------
 * Uneven batches: envs of several models (different sizes) stepped in one
 * call. Not a passage of the paper: the batched-rollout setting of its
 * Methods (many environments at once, Simulation throughput) with models of
 * different sizes in one batch.
 *
 * Each model's envs keep their own caller-owned state (layouts as for
 * ms_rollout) and excitation descriptor. One call steps every model's envs
 * n_steps times with each model's own step kernels, issued as the
 * batch's issue mode says: concurrently (each kernel on an internal stream
 * forked from `stream` and joined back; in the caller's model order or with
 * the model of most work first) or serially on `stream` (most work first).
 * Outside an active capture the launches are recorded once as a HIP graph
 * per argument set (state and excitation pointers and values, n_steps,
 * opts, configuration) and replayed. Inside a caller's stream capture the launches are simply issued.
 * Results are bitwise those of ms_rollout on each model alone, for any
 * configuration. A batch is not thread-safe; its models must not be used on
 * other streams during a call. */
typedef struct ms_batch ms_batch;
#define MS_ISSUE_CONCURRENT 0            /* forked streams, caller's order */
#define MS_ISSUE_CONCURRENT_MOST_WORK 1  /* forked streams, most work first */
#define MS_ISSUE_SERIAL 2                /* one after another on the stream */
typedef struct {
  float *q, *qd, *act; /* device, [n_env][nq], [n_env][nv], [n_env][n_mus] */
  uint32_t *status;    /* device [n_env], may be NULL */
} ms_batch_state;
/* models[n_models] stay owned by the caller and must outlive the batch. */
ms_status ms_batch_create(ms_model *const *models, const int32_t *n_env,
                          int32_t n_models, ms_batch **out);
void ms_batch_destroy(ms_batch *b);
/* states[n_models], exc[n_models] (host arrays of descriptors). */
ms_status ms_batch_rollout(ms_batch *b, const ms_batch_state *states,
                           const ms_excitation *exc, int32_t n_steps,
                           const ms_step_opts *opts, void *stream);
/* Autotuner: per model alone, probe rollouts of n_probe steps for 1, 2 and 4
 * envs per workgroup (each env is one wavefront with its own LDS block); then
 * (fastest of three probes each); then the whole batch in each of the
 * three issue modes, as graph replays (mean of three after a warm-up); a
 * concurrent mode is kept only if it beats serial issue by more than 2 %. Each workgroup steps its envs through a whole
 * rollout, so the best issue mode depends on the rollout length: probe with
 * the n_steps the batch will run. Probes run on scratch copies of the given states (left unchanged);
 * the fastest choices are kept in the batch. Synchronises `stream`. */
ms_status ms_batch_autotune(ms_batch *b, const ms_batch_state *states,
                            const ms_excitation *exc, int32_t n_probe,
                            const ms_step_opts *opts, void *stream);
/* Current configuration: env_per_wg[n_models], *issue_mode (MS_ISSUE_*). */
ms_status ms_batch_config(const ms_batch *b, int32_t *env_per_wg,
                          int32_t *issue_mode);
/* Set it by hand (env_per_wg in {1, 2, 4}, or 0 for the envs per workgroup
 * that keep the most envs resident per CU, the default of a new batch;
 * issue_mode an MS_ISSUE_* value,
 * else MS_E_ARG); MS_E_UNSUPPORTED if a workgroup's LDS would exceed
 * 160 KiB. */
ms_status ms_batch_set_config(ms_batch *b, const int32_t *env_per_wg,
                              int32_t issue_mode);
const char *ms_batch_last_error(void);

/* ms_rollout with the muscle geometry predicted by the surrogate: each step
 * runs the network on every env's pose, then the step, in which an env
 * falls back to the exact geometry (MS_ST_FALLBACK, fallback_count[env]++
 * when non-NULL) if a hinge/slide coordinate lies outside the pose-domain
 * box or if the predicted length or any predicted moment arm of any of 32
 * sentinel muscles (muscle (32 step + i) mod n_mus, i < 32, step =
 * exc->step0 + t) differs from the exact one by more than tol metres (the
 * paper gives no residual test; this one is the library's). tol < 0 always
 * falls back (exact
 * path); n_env must not exceed the surrogate workspace the device can hold. */
ms_status ms_rollout_surrogate(ms_model *m, ms_surrogate *s, int32_t n_env, float *q,
                               float *qd, float *act, uint32_t *status,
                               const ms_excitation *exc, int32_t n_steps,
                               const ms_step_opts *opts, float tol,
                               uint32_t *fallback_count, void *stream);

#ifdef __cplusplus
}
#endif
#endif
