/*
 * ora.h -- FP64 CPU oracle of the batched musculoskeletal forward-dynamics
 * step (TEST INFRASTRUCTURE: only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg use it; the product path never does).
 *
 * Plain, slow, obviously-correct definitions, in double precision, of what
 * one step computes (Methods, "Whole-body musculoskeletal model"):
 *   activation dynamics (Eq. excitation-activation), via-point muscle path
 *   length and moment arms (the moment-arm matrix J_m of the equations of
 *   motion), the Hill-type force (Eq. flv), the projection J_m^T F, the
 *   generalized mass matrix M(q) by its Jacobian-sum definition, the bias
 *   C(q, qd) (Coriolis, centrifugal, gravity) by textbook recursive
 *   Newton-Euler in body coordinates, penalty ground contact as tau_ext,
 *   joint damping, penalty joint coupling, a dense Cholesky solve of (M + dt D) qdd = rhs with the
 *   dissipative forces' velocity slope D taken implicitly, and a
 *   semi-implicit Euler update; and a compliant-tendon variant of the
 *   muscle (a fibre-length state, ora_step_tendon).
 *
 * Shares no code with the HIP library: own model struct, own parser of the
 * generator's arrays, own maths.
 */
#ifndef ORA_H
#define ORA_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ora_model ora_model;

/* Status bits (sticky, OR-ed per env). */
#define ORA_ST_NONFINITE 1u /* non-finite state: the step is not applied */
#define ORA_ST_NONSPD 2u    /* Cholesky pivot <= 0: the step is not applied */

/* Build a model from the generator's float32/int32 arrays (copied). */
ora_model *ora_model_create(int n_node, const int32_t *parent,
                            const int32_t *jtype, const float *jpos,
                            const float *jrot, const float *axis,
                            const float *mass, const float *com,
                            const float *inertia, const float *damping,
                            int n_mus, const float *f0, const float *l_opt,
                            const float *l_slack, const float *v_max,
                            const float *tau_act, const float *tau_deact,
                            const int32_t *via_start, const int32_t *via_node,
                            const float *via_pos, int n_con,
                            const int32_t *con_node, const float *con_pos,
                            const float *con_radius, const float *contact,
                            const float *gravity);
void ora_model_destroy(ora_model *m);

/* Anatomical joint coupling (Methods, "GPU-accelerated simulation
 * framework": joint coupling such as the scapulohumeral rhythm), as equality
 * constraints phi_c(q) = sum over the terms t of constraint c of
 * coef_t q_(dof_t) - off_c = 0 on hinge/slide DoFs, enforced by a penalty
 * spring k and damper d (copied into the model; n_eq = 0 removes them). */
void ora_model_set_coupling(ora_model *m, int n_eq, const int32_t *eq_start,
                            const int32_t *eq_dof, const float *eq_coef,
                            const float *eq_off, float k, float d);

/* The coupling's generalized force over a step dt, with the spring taken
 * linearly implicitly as the contact spring is (damping d + dt k):
 * tau_eq = -J^T (k phi(q) + (d + dt k) J qd), J the constraint Jacobian
 * (J[c][dof_t] = coef_t); added into tau[nv]. D (may be NULL) accumulates
 * its velocity slope -d(tau_eq)/d(qd) = (d + dt k) J^T J [nv][nv]. phi
 * (may be NULL) receives phi(q) [n_eq]. */
void ora_coupling(const ora_model *m, const double *q, const double *qd, double dt,
                  double *tau, double *D, double *phi);
int ora_nq(const ora_model *m);
int ora_nv(const ora_model *m);

/* Force-length, passive and force-velocity curves (normalized). */
double ora_fl(double lm);
double ora_fp(double lm);
double ora_fv(double vm);
double ora_fv_slope(double vm); /* d f_v / d v_m */

/* Forward kinematics: R[n_node][9] (row-major, world), p[n_node][3]. */
void ora_fk(const ora_model *m, const double *q, double *R, double *p);

/* Activation update for every muscle: act_out = act + dt (u-act)/tau,
 * clamped to [0,1]; u is first clamped to [0,1]. */
void ora_activation(const ora_model *m, double dt, const double *u,
                    const double *act, double *act_out);

/* Muscle path: L[n_mus], moment arms r[n_mus][nv] = -dL/dq, Ldot[n_mus]. */
void ora_geometry(const ora_model *m, const double *q, const double *qd,
                  double *L, double *r, double *Ldot);

/* Hill force from act, L, Ldot: F[n_mus]; lm, vm optional (may be NULL). */
void ora_hill(const ora_model *m, const double *act, const double *L,
              const double *Ldot, double *F, double *lm, double *vm);

/* M(q) [nv][nv] by the Jacobian-sum definition. */
void ora_mass_matrix(const ora_model *m, const double *q, double *M);

/* Inverse dynamics tau = M qdd + C(q,qd) (+ gravity if grav != 0) by
 * recursive Newton-Euler in body coordinates. */
void ora_rnea(const ora_model *m, const double *q, const double *qd,
              const double *qdd, int grav, double *tau);

/* Contact generalized force tau_ext[nv] over a step dt (the spring is taken
 * linearly implicitly: damping c_d + dt k); D (may be NULL) accumulates the
 * contact force's velocity slope -d(tau_ext)/d(qd) [nv][nv]; n_active (may
 * be NULL) counts penetrating spheres. */
void ora_contact(const ora_model *m, const double *q, const double *qd,
                 double dt, double *tau_ext, double *D, int *n_active);

/* Dense Cholesky solve M x = b (n x n). Returns 0, or -1 on a pivot <= 0. */
int ora_chol_solve(int n, const double *M, const double *b, double *x);

/* Kinetic + gravitational potential energy. */
double ora_energy(const ora_model *m, const double *q, const double *qd);

/* Per-stage outputs of one step (any pointer may be NULL). */
typedef struct {
  double *act;     /* [n_mus] updated activation */
  /* (tau_ext holds the contact force; the coupling's force is in tau_eq) */
  double *L, *Ldot, *F, *lm, *vm; /* [n_mus] */
  double *r;       /* [n_mus][nv] */
  double *tau_mus, *tau_ext, *tau_d, *C, *qdd; /* [nv] */
  double *tau_eq;  /* [nv] joint-coupling force (may be NULL) */
  double *M;       /* [nv][nv] mass matrix */
  double *D;       /* [nv][nv] velocity slope of the dissipative forces */
} ora_stage_out;

/* One step of one env, in place on (q, qd, act). Returns status bits. */
uint32_t ora_step(const ora_model *m, double dt, int contact_on,
                  double *q, double *qd, double *act, const double *u,
                  ora_stage_out *out);

/* Compliant tendon (a higher-fidelity muscle variant of the paper's Hill
 * actuator, Methods "Whole-body musculoskeletal model"): a fibre with the
 * damped force balance F0 [act f_l(l) f_v(v) + f_p(l) + beta v] in series
 * with a tendon that is linear above its slack length l_slack, F0 at strain
 * eps0, and slack below it. No pennation, as in the rigid model.
 *
 * ora_fv_root: the normalised fibre velocity v with
 * A f_v(v) + beta v = R (A = act f_l >= 0, beta > 0), by bisection on the
 * strictly increasing left-hand side. */
double ora_fv_root(double A, double R, double beta);

/* One step with a compliant tendon, in place on (q, qd, act, lm); lm[n_mus]
 * is the fibre length in metres. At the start of the step the fibre
 * velocity v balances the fibre against the tendon; the tendon (stiffness
 * k) and the fibre (velocity slope b) in series act on the skeleton as a
 * force F_t + c (Ldot' - v) linear in the new lengthening rate Ldot', with
 * c = k dt / (1 + k dt / b), taken implicitly like the rigid muscle's
 * damping. After the solve each fibre takes a backward-Euler step: its new
 * length balances fibre and tendon at the path length L + dt Ldot',
 * Ldot' = -r qd' (moment arms of the step's start); on a linear element
 * this is the fibre velocity v + c (Ldot' - v) / b. Stage outputs:
 * F is the force of the right-hand side, lm and vm the normalised fibre
 * length and velocity at the start. Returns status bits; on a failure
 * nothing is updated. */
uint32_t ora_step_tendon(const ora_model *m, double dt, int contact_on,
                         double *q, double *qd, double *act, double *lm,
                         const double *u, double eps0, double beta,
                         ora_stage_out *out);

/* ora_step with the muscle geometry given instead of computed: L_in[n_mus]
 * and moment arms r_in[n_mus][nv] (both NULL: ora_step). Ldot = -r qd. */
uint32_t ora_step_geo(const ora_model *m, double dt, int contact_on,
                      double *q, double *qd, double *act, const double *u,
                      const double *L_in, const double *r_in, ora_stage_out *out);

/* n_env envs for n_steps steps; u is float32 [n_steps][n_env][n_mus];
 * status[n_env] is OR-ed. Envs are split over n_threads threads. */
void ora_rollout(const ora_model *m, int n_env, int n_steps, double dt,
                 int contact_on, double *q, double *qd, double *act,
                 const float *u, uint32_t *status, int n_threads);

#ifdef __cplusplus
}
#endif
#endif
