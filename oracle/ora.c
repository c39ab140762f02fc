/*
 * ora.c -- FP64 CPU oracle (TEST INFRASTRUCTURE; see ora.h).
 *
 * Every function states the definition it writes out. Conventions:
 *  - z is up, gravity g from the model (default (0,0,-9.81)), ground z = 0.
 *  - Node i frame: R_i = R_parent * jrot_i * Rot(axis_i, q_i) for a hinge,
 *    origin p_i = p_parent + R_parent * jpos_i (a slide adds
 *    R_parent * jrot_i * axis_i * q_i); a free root has p = q[0:3] and R
 *    from the unit quaternion q[3:7] = (w, x, y, z).
 *  - Velocity coordinates: hinge/slide rates; a free root has the world
 *    linear velocity of its origin then its angular velocity in root-body
 *    axes.
 *  - Moment arm r_j = -dL/dq_j, so tau = sum_m r_m F_m (J_m^T F).
 */
#include "ora.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

struct ora_model {
  int n_node, nq, nv, n_mus, n_via, n_con;
  int *parent, *jtype, *qadr, *dadr;
  double *jpos, *jrot, *axis, *mass, *com, *inertia, *damping;
  double *f0, *l_opt, *l_slack, *v_max, *tau_act, *tau_deact;
  int *via_start, *via_node;
  double *via_pos;
  int *con_node;
  double *con_pos, *con_radius;
  double kc, cc, mu, vs, g[3];
  unsigned char *anc; /* anc[a*n+b] = 1 if node a is b or an ancestor of b */
  int n_eq, *eq_start, *eq_dof; /* joint coupling (ora_model_set_coupling) */
  double *eq_coef, *eq_off, eq_k, eq_d;
};

/* ---------------------------------------------------------------- helpers */
static double *dup_f(const float *x, int n) {
  double *y = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) y[i] = (double)x[i];
  return y;
}
static int *dup_i(const int32_t *x, int n) {
  int *y = (int *)malloc(sizeof(int) * (n > 0 ? n : 1));
  for (int i = 0; i < n; ++i) y[i] = (int)x[i];
  return y;
}
static void cross(const double *a, const double *b, double *c) {
  double t0 = a[1] * b[2] - a[2] * b[1];
  double t1 = a[2] * b[0] - a[0] * b[2];
  double t2 = a[0] * b[1] - a[1] * b[0];
  c[0] = t0; c[1] = t1; c[2] = t2;
}
static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
/* C = A B (3x3 row-major) */
static void mat_mul(const double *A, const double *B, double *C) {
  double T[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0;
      for (int k = 0; k < 3; ++k) s += A[3 * i + k] * B[3 * k + j];
      T[3 * i + j] = s;
    }
  memcpy(C, T, sizeof T);
}
/* y = A x */
static void mat_vec(const double *A, const double *x, double *y) {
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = A[3 * i] * x[0] + A[3 * i + 1] * x[1] + A[3 * i + 2] * x[2];
  y[0] = t[0]; y[1] = t[1]; y[2] = t[2];
}
/* y = A^T x */
static void mat_tvec(const double *A, const double *x, double *y) {
  double t[3];
  for (int i = 0; i < 3; ++i) t[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
  y[0] = t[0]; y[1] = t[1]; y[2] = t[2];
}
/* Rodrigues: rotation by angle th about unit axis a. */
static void axis_angle(const double *a, double th, double *R) {
  double c = cos(th), s = sin(th), v = 1.0 - c;
  double x = a[0], y = a[1], z = a[2];
  R[0] = c + x * x * v;     R[1] = x * y * v - z * s; R[2] = x * z * v + y * s;
  R[3] = y * x * v + z * s; R[4] = c + y * y * v;     R[5] = y * z * v - x * s;
  R[6] = z * x * v - y * s; R[7] = z * y * v + x * s; R[8] = c + z * z * v;
}
/* Rotation matrix of the quaternion (w,x,y,z) after normalisation. */
static void quat_to_mat(const double *qt, double *R) {
  double n = sqrt(qt[0] * qt[0] + qt[1] * qt[1] + qt[2] * qt[2] + qt[3] * qt[3]);
  double w = qt[0] / n, x = qt[1] / n, y = qt[2] / n, z = qt[3] / n;
  R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
  R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
  R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

/* ------------------------------------------------------------------ model */
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
                            const float *gravity) {
  ora_model *m = (ora_model *)calloc(1, sizeof(ora_model));
  int n = n_node;
  m->n_node = n;
  m->parent = dup_i(parent, n);
  m->jtype = dup_i(jtype, n);
  m->qadr = (int *)malloc(sizeof(int) * n);
  m->dadr = (int *)malloc(sizeof(int) * n);
  int nq = 0, nv = 0;
  for (int i = 0; i < n; ++i) {
    m->qadr[i] = nq;
    m->dadr[i] = nv;
    nq += (jtype[i] == 2) ? 7 : 1;
    nv += (jtype[i] == 2) ? 6 : 1;
  }
  m->nq = nq;
  m->nv = nv;
  m->jpos = dup_f(jpos, 3 * n);
  m->jrot = dup_f(jrot, 9 * n);
  m->axis = dup_f(axis, 3 * n);
  m->mass = dup_f(mass, n);
  m->com = dup_f(com, 3 * n);
  m->inertia = dup_f(inertia, 3 * n);
  m->damping = dup_f(damping, nv);
  m->n_mus = n_mus;
  m->f0 = dup_f(f0, n_mus);
  m->l_opt = dup_f(l_opt, n_mus);
  m->l_slack = dup_f(l_slack, n_mus);
  m->v_max = dup_f(v_max, n_mus);
  m->tau_act = dup_f(tau_act, n_mus);
  m->tau_deact = dup_f(tau_deact, n_mus);
  m->via_start = dup_i(via_start, n_mus + 1);
  m->n_via = via_start[n_mus];
  m->via_node = dup_i(via_node, m->n_via);
  m->via_pos = dup_f(via_pos, 3 * m->n_via);
  m->n_con = n_con;
  m->con_node = dup_i(con_node, n_con);
  m->con_pos = dup_f(con_pos, 3 * n_con);
  m->con_radius = dup_f(con_radius, n_con);
  m->kc = contact[0];
  m->cc = contact[1];
  m->mu = contact[2];
  m->vs = contact[3];
  for (int k = 0; k < 3; ++k) m->g[k] = gravity[k];
  m->anc = (unsigned char *)calloc((size_t)n * n, 1);
  for (int b = 0; b < n; ++b)
    for (int a = b; a >= 0; a = m->parent[a]) m->anc[a * n + b] = 1;
  return m;
}

void ora_model_destroy(ora_model *m) {
  if (!m) return;
  free(m->parent); free(m->jtype); free(m->qadr); free(m->dadr);
  free(m->jpos); free(m->jrot); free(m->axis); free(m->mass); free(m->com);
  free(m->inertia); free(m->damping); free(m->f0); free(m->l_opt);
  free(m->l_slack); free(m->v_max); free(m->tau_act); free(m->tau_deact);
  free(m->via_start); free(m->via_node); free(m->via_pos); free(m->con_node);
  free(m->con_pos); free(m->con_radius); free(m->anc);
  free(m->eq_start); free(m->eq_dof); free(m->eq_coef); free(m->eq_off); free(m);
}

void ora_model_set_coupling(ora_model *m, int n_eq, const int32_t *eq_start,
                            const int32_t *eq_dof, const float *eq_coef,
                            const float *eq_off, float k, float d) {
  free(m->eq_start); free(m->eq_dof); free(m->eq_coef); free(m->eq_off);
  m->eq_start = m->eq_dof = NULL;
  m->eq_coef = m->eq_off = NULL;
  m->n_eq = n_eq > 0 ? n_eq : 0;
  if (!m->n_eq) return;
  int nt = eq_start[n_eq];
  m->eq_start = dup_i(eq_start, n_eq + 1);
  m->eq_dof = dup_i(eq_dof, nt);
  m->eq_coef = dup_f(eq_coef, nt);
  m->eq_off = dup_f(eq_off, n_eq);
  m->eq_k = k;
  m->eq_d = d;
}

/* phi_c = sum_t coef_t q_(dof_t) - off_c; with d_eff = d + dt k,
 * tau -= J^T (k phi + d_eff J qd) and D += d_eff J^T J, written as the
 * plain sums over each constraint's terms. */
void ora_coupling(const ora_model *m, const double *q, const double *qd, double dt,
                  double *tau, double *D, double *phi) {
  const int nv = m->nv;
  const double deff = m->eq_d + dt * m->eq_k;
  for (int c = 0; c < m->n_eq; ++c) {
    double ph = -m->eq_off[c], jv = 0.0;
    for (int t = m->eq_start[c]; t < m->eq_start[c + 1]; ++t) {
      int j = m->eq_dof[t];
      int qi = j + (m->jtype[0] == 2 ? 1 : 0);  /* hinge/slide DoF -> its q */
      ph += m->eq_coef[t] * q[qi];
      jv += m->eq_coef[t] * qd[j];
    }
    if (phi) phi[c] = ph;
    double f = m->eq_k * ph + deff * jv;
    for (int t = m->eq_start[c]; t < m->eq_start[c + 1]; ++t) {
      tau[m->eq_dof[t]] -= m->eq_coef[t] * f;
      if (!D) continue;
      for (int u = m->eq_start[c]; u < m->eq_start[c + 1]; ++u)
        D[m->eq_dof[t] * nv + m->eq_dof[u]] += deff * m->eq_coef[t] * m->eq_coef[u];
    }
  }
}
int ora_nq(const ora_model *m) { return m->nq; }
int ora_nv(const ora_model *m) { return m->nv; }

/* ------------------------------------------------------- muscle curves
 * The paper names active force-length f_l, force-velocity f_v and passive
 * f_p curves (Eq. flv) without formulas; these are the closed forms used
 * on both sides (Thelen 2003 Gaussian f_l and exponential f_p with k_PE=4,
 * strain 0.6 and a linear tail past 1.6; a Hill hyperbola f_v with
 * concentric curvature 0.25 and an eccentric branch saturating at 1.4). */
double ora_fl(double lm) { return exp(-(lm - 1.0) * (lm - 1.0) / 0.45); }

double ora_fp(double lm) {
  const double e4 = exp(4.0);
  if (lm <= 1.0) return 0.0;
  if (lm <= 1.6) return (exp(4.0 * (lm - 1.0) / 0.6) - 1.0) / (e4 - 1.0);
  return 1.0 + (4.0 / 0.6) * e4 / (e4 - 1.0) * (lm - 1.6);
}

double ora_fv(double vm) {
  if (vm <= -1.0) return 0.0;
  if (vm <= 0.0) return (1.0 + vm) / (1.0 - vm / 0.25);
  return 1.0 + 0.4 * vm / (vm + 0.08);
}

/* Slope df_v/dv of the force-velocity curve above. */
double ora_fv_slope(double vm) {
  if (vm <= -1.0) return 0.0;
  if (vm <= 0.0) return 5.0 / ((1.0 - 4.0 * vm) * (1.0 - 4.0 * vm));
  return 0.032 / ((vm + 0.08) * (vm + 0.08));
}

/* The root v of A f_v(v) + beta v = R by bisection. A f_v lies in
 * [0, 1.4 A], so the left-hand side is below R at (R - 1.4 A)/beta - 1 and
 * above it at R/beta + 1; halving stops when the midpoint no longer splits
 * the bracket (full double precision). */
double ora_fv_root(double A, double R, double beta) {
  double lo = (R - 1.4 * A) / beta - 1.0, hi = R / beta + 1.0;
  for (int it = 0; it < 2000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (A * ora_fv(mid) + beta * mid - R < 0.0)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* --------------------------------------------------- forward kinematics */
void ora_fk(const ora_model *m, const double *q, double *R, double *p) {
  for (int i = 0; i < m->n_node; ++i) {
    int pa = m->parent[i];
    double Rp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, pp[3] = {0, 0, 0};
    if (pa >= 0) {
      memcpy(Rp, R + 9 * pa, sizeof Rp);
      memcpy(pp, p + 3 * pa, sizeof pp);
    }
    const double *qi = q + m->qadr[i];
    if (m->jtype[i] == 2) {
      p[3 * i] = qi[0]; p[3 * i + 1] = qi[1]; p[3 * i + 2] = qi[2];
      quat_to_mat(qi + 3, R + 9 * i);
      continue;
    }
    double Rj[9], t[3];
    mat_mul(Rp, m->jrot + 9 * i, Rj);
    mat_vec(Rp, m->jpos + 3 * i, t);
    for (int k = 0; k < 3; ++k) p[3 * i + k] = pp[k] + t[k];
    if (m->jtype[i] == 0) {
      double Rq[9];
      axis_angle(m->axis + 3 * i, qi[0], Rq);
      mat_mul(Rj, Rq, R + 9 * i);
    } else {
      double a[3];
      memcpy(R + 9 * i, Rj, sizeof Rj);
      mat_vec(Rj, m->axis + 3 * i, a);
      for (int k = 0; k < 3; ++k) p[3 * i + k] += a[k] * qi[0];
    }
  }
}

/* World position of a point with local coordinates x on node b (b = -1 is
 * the fixed world frame). */
static void world_point(const double *R, const double *p, int b,
                        const double *x, double *w) {
  if (b < 0) {
    w[0] = x[0]; w[1] = x[1]; w[2] = x[2];
    return;
  }
  mat_vec(R + 9 * b, x, w);
  for (int k = 0; k < 3; ++k) w[k] += p[3 * b + k];
}

/* Linear velocity Jacobian Jv[3][nv] (row-major) of world point w rigidly
 * attached to node b, and optionally the angular Jacobian Jw[3][nv]:
 * hinge j above b: column a_j x (w - o_j) (angular a_j);
 * slide j above b: column a_j; free root: e_k for the linear rates,
 * (R0 e_k) x (w - p0) for the body angular rates (angular R0 e_k). */
static void point_jacobian(const ora_model *m, const double *R,
                           const double *p, int b, const double *w, double *Jv,
                           double *Jw) {
  int nv = m->nv, n = m->n_node;
  memset(Jv, 0, sizeof(double) * 3 * nv);
  if (Jw) memset(Jw, 0, sizeof(double) * 3 * nv);
  if (b < 0) return;
  for (int j = 0; j < n; ++j) {
    if (!m->anc[j * n + b]) continue;
    int d = m->dadr[j];
    if (m->jtype[j] == 2) {
      for (int k = 0; k < 3; ++k) {
        Jv[k * nv + d + k] = 1.0;
        double e[3] = {R[9 * j + k], R[9 * j + 3 + k], R[9 * j + 6 + k]};
        double rel[3] = {w[0] - p[3 * j], w[1] - p[3 * j + 1], w[2] - p[3 * j + 2]};
        double c[3];
        cross(e, rel, c);
        for (int r = 0; r < 3; ++r) {
          Jv[r * nv + d + 3 + k] = c[r];
          if (Jw) Jw[r * nv + d + 3 + k] = e[r];
        }
      }
      continue;
    }
    double a[3];
    mat_vec(R + 9 * j, m->axis + 3 * j, a);
    if (m->jtype[j] == 0) {
      double rel[3] = {w[0] - p[3 * j], w[1] - p[3 * j + 1], w[2] - p[3 * j + 2]};
      double c[3];
      cross(a, rel, c);
      for (int r = 0; r < 3; ++r) {
        Jv[r * nv + d] = c[r];
        if (Jw) Jw[r * nv + d] = a[r];
      }
    } else {
      for (int r = 0; r < 3; ++r) Jv[r * nv + d] = a[r];
    }
  }
}

/* ------------------------------------------------ activation dynamics
 * Eq. excitation-activation: d act/dt = (u - act)/tau(u, act) with
 * tau = tau_act (0.5 + 1.5 act) when u > act, else
 * tau_deact / (0.5 + 1.5 act); one explicit Euler step, clamped to [0,1]. */
void ora_activation(const ora_model *m, double dt, const double *u,
                    const double *act, double *act_out) {
  for (int i = 0; i < m->n_mus; ++i) {
    double ui = fmin(fmax(u[i], 0.0), 1.0);
    double a = act[i];
    double tau = (ui > a) ? m->tau_act[i] * (0.5 + 1.5 * a)
                          : m->tau_deact[i] / (0.5 + 1.5 * a);
    double an = a + dt * (ui - a) / tau;
    act_out[i] = fmin(fmax(an, 0.0), 1.0);
  }
}

/* ---------------------------------------------------- muscle geometry
 * Path through via-points w_k: L = sum_k |w_{k+1} - w_k|; with unit
 * segment vectors e_k, dL/dq = sum_k e_k . (J(w_{k+1}) - J(w_k));
 * r = -dL/dq; Ldot = (dL/dq) . qd. */
void ora_geometry(const ora_model *m, const double *q, const double *qd,
                  double *L, double *r, double *Ldot) {
  int n = m->n_node, nv = m->nv;
  double *R = (double *)malloc(sizeof(double) * 9 * n);
  double *p = (double *)malloc(sizeof(double) * 3 * n);
  double *Ja = (double *)malloc(sizeof(double) * 3 * nv);
  double *Jb = (double *)malloc(sizeof(double) * 3 * nv);
  double *dL = (double *)malloc(sizeof(double) * nv);
  ora_fk(m, q, R, p);
  for (int mu = 0; mu < m->n_mus; ++mu) {
    int s = m->via_start[mu], e = m->via_start[mu + 1];
    double len = 0.0;
    memset(dL, 0, sizeof(double) * nv);
    for (int k = s; k + 1 < e; ++k) {
      double wa[3], wb[3], seg[3];
      world_point(R, p, m->via_node[k], m->via_pos + 3 * k, wa);
      world_point(R, p, m->via_node[k + 1], m->via_pos + 3 * (k + 1), wb);
      for (int c = 0; c < 3; ++c) seg[c] = wb[c] - wa[c];
      double l = sqrt(dot3(seg, seg));
      len += l;
      double ek[3] = {seg[0] / l, seg[1] / l, seg[2] / l};
      point_jacobian(m, R, p, m->via_node[k], wa, Ja, NULL);
      point_jacobian(m, R, p, m->via_node[k + 1], wb, Jb, NULL);
      for (int j = 0; j < nv; ++j)
        for (int c = 0; c < 3; ++c) dL[j] += ek[c] * (Jb[c * nv + j] - Ja[c * nv + j]);
    }
    if (L) L[mu] = len;
    double ld = 0.0;
    for (int j = 0; j < nv; ++j) {
      if (r) r[(size_t)mu * nv + j] = -dL[j];
      ld += dL[j] * qd[j];
    }
    if (Ldot) Ldot[mu] = ld;
  }
  free(R); free(p); free(Ja); free(Jb); free(dL);
}

/* ------------------------------------------------------- Hill force
 * Eq. flv: F = F_max [act f_l(l_m) f_v(v_m) + f_p(l_m)] with a rigid
 * tendon and no pennation: l_m = (L - l_slack)/l_opt and
 * v_m = Ldot / (v_max l_opt), v_max in optimal lengths per second. */
void ora_hill(const ora_model *m, const double *act, const double *L,
              const double *Ldot, double *F, double *lm_out, double *vm_out) {
  for (int i = 0; i < m->n_mus; ++i) {
    double lm = (L[i] - m->l_slack[i]) / m->l_opt[i];
    double vm = Ldot[i] / (m->v_max[i] * m->l_opt[i]);
    F[i] = m->f0[i] * (act[i] * ora_fl(lm) * ora_fv(vm) + ora_fp(lm));
    if (lm_out) lm_out[i] = lm;
    if (vm_out) vm_out[i] = vm;
  }
}

/* ---------------------------------------------------- mass matrix
 * M = sum_b m_b Jv_b^T Jv_b + Jw_b^T (R_b I_b R_b^T) Jw_b with Jv_b the
 * Jacobian of body b's centre of mass. */
void ora_mass_matrix(const ora_model *m, const double *q, double *M) {
  int n = m->n_node, nv = m->nv;
  double *R = (double *)malloc(sizeof(double) * 9 * n);
  double *p = (double *)malloc(sizeof(double) * 3 * n);
  double *Jv = (double *)malloc(sizeof(double) * 3 * nv);
  double *Jw = (double *)malloc(sizeof(double) * 3 * nv);
  ora_fk(m, q, R, p);
  memset(M, 0, sizeof(double) * nv * nv);
  for (int b = 0; b < n; ++b) {
    double mb = m->mass[b];
    if (mb == 0.0 && m->inertia[3 * b] == 0.0 && m->inertia[3 * b + 1] == 0.0 &&
        m->inertia[3 * b + 2] == 0.0)
      continue;
    double c[3];
    world_point(R, p, b, m->com + 3 * b, c);
    point_jacobian(m, R, p, b, c, Jv, Jw);
    /* world inertia Iw = R diag(I) R^T */
    double Iw[9];
    const double *Rb = R + 9 * b;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += Rb[3 * i + k] * m->inertia[3 * b + k] * Rb[3 * j + k];
        Iw[3 * i + j] = s;
      }
    for (int i = 0; i < nv; ++i)
      for (int j = 0; j < nv; ++j) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += mb * Jv[k * nv + i] * Jv[k * nv + j];
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) s += Jw[k * nv + i] * Iw[3 * k + l] * Jw[l * nv + j];
        M[i * nv + j] += s;
      }
  }
  free(R); free(p); free(Jv); free(Jw);
}

/* ------------------------------------------------ recursive Newton-Euler
 * Spatial vectors in node coordinates: motion (w; v), force (n; f).
 * Featherstone, Rigid Body Dynamics Algorithms (2008), ch. 5:
 *   v_i = X_i v_p + S_i qd_i,  a_i = X_i a_p + S_i qdd_i + v_i x S_i qd_i,
 *   f_i = I_i a_i + v_i x* I_i v_i,  tau_i = S_i^T f_i,  f_p += X_i^T f_i,
 * with the base accelerating at -g to account for gravity. */
static void crm(const double *v, const double *u, double *o) {
  /* motion cross product v x u */
  double a[3], b[3], c[3];
  cross(v, u, a);
  cross(v, u + 3, b);
  cross(v + 3, u, c);
  o[0] = a[0]; o[1] = a[1]; o[2] = a[2];
  o[3] = b[0] + c[0]; o[4] = b[1] + c[1]; o[5] = b[2] + c[2];
}
static void crf(const double *v, const double *f, double *o) {
  /* force cross product v x* f */
  double a[3], b[3], c[3];
  cross(v, f, a);
  cross(v + 3, f + 3, b);
  cross(v, f + 3, c);
  o[0] = a[0] + b[0]; o[1] = a[1] + b[1]; o[2] = a[2] + b[2];
  o[3] = c[0]; o[4] = c[1]; o[5] = c[2];
}
/* spatial inertia times motion: m, com c, rotational inertia Ic (3x3) */
static void inertia_mul(double mass, const double *c, const double *Ic,
                        const double *v, double *o) {
  /* linear momentum m (v + w x c); angular Ic w + m c x (v + w x c) */
  double wc[3], vv[3], t[3];
  cross(v, c, wc);
  for (int k = 0; k < 3; ++k) vv[k] = v[3 + k] + wc[k];
  mat_vec(Ic, v, t);
  double cv[3];
  cross(c, vv, cv);
  for (int k = 0; k < 3; ++k) {
    o[k] = t[k] + mass * cv[k];
    o[3 + k] = mass * vv[k];
  }
}

void ora_rnea(const ora_model *m, const double *q, const double *qd,
              const double *qdd, int grav, double *tau) {
  int n = m->n_node;
  double *R = (double *)malloc(sizeof(double) * 9 * n);
  double *p = (double *)malloc(sizeof(double) * 3 * n);
  double *v = (double *)malloc(sizeof(double) * 6 * n);
  double *a = (double *)malloc(sizeof(double) * 6 * n);
  double *f = (double *)malloc(sizeof(double) * 6 * n);
  ora_fk(m, q, R, p);
  double gvec[3] = {0, 0, 0};
  if (grav) { gvec[0] = m->g[0]; gvec[1] = m->g[1]; gvec[2] = m->g[2]; }
  for (int i = 0; i < n; ++i) {
    int pa = m->parent[i], d = m->dadr[i];
    double *vi = v + 6 * i, *ai = a + 6 * i;
    /* E = R_p^T R_i, r = R_p^T (p_i - p_p): node i in parent coordinates */
    double Rp[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, pp[3] = {0, 0, 0};
    double vp[6] = {0, 0, 0, 0, 0, 0};
    double ap[6] = {0, 0, 0, -gvec[0], -gvec[1], -gvec[2]};
    if (pa >= 0) {
      memcpy(Rp, R + 9 * pa, sizeof Rp);
      memcpy(pp, p + 3 * pa, sizeof pp);
      memcpy(vp, v + 6 * pa, sizeof vp);
      memcpy(ap, a + 6 * pa, sizeof ap);
    }
    double dpw[3] = {p[3 * i] - pp[0], p[3 * i + 1] - pp[1], p[3 * i + 2] - pp[2]};
    double rr[3], E[9];
    mat_tvec(Rp, dpw, rr);
    /* E = Rp^T Ri */
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        double s = 0;
        for (int k = 0; k < 3; ++k) s += Rp[3 * k + r] * R[9 * i + 3 * k + c];
        E[3 * r + c] = s;
      }
    /* X v: w_c = E^T w_p ; v_c = E^T (v_p + w_p x r) */
    double xv[6], xa[6], tmp[3];
    mat_tvec(E, vp, xv);
    cross(vp, rr, tmp);
    for (int k = 0; k < 3; ++k) tmp[k] += vp[3 + k];
    mat_tvec(E, tmp, xv + 3);
    mat_tvec(E, ap, xa);
    cross(ap, rr, tmp);
    for (int k = 0; k < 3; ++k) tmp[k] += ap[3 + k];
    mat_tvec(E, tmp, xa + 3);
    if (m->jtype[i] == 2) {
      /* root: body-coordinate velocity (w_b; R^T v_w); its derivative
       * adds (0; -w_b x R^T v_w) to R^T a_w */
      const double *Ri = R + 9 * i;
      double vb[3], ab[3];
      mat_tvec(Ri, qd + d, vb);
      mat_tvec(Ri, qdd + d, ab);
      double wxv[3];
      cross(qd + d + 3, vb, wxv);
      for (int k = 0; k < 3; ++k) {
        vi[k] = qd[d + 3 + k];
        vi[3 + k] = vb[k];
        ai[k] = xa[k] + qdd[d + 3 + k];
        ai[3 + k] = xa[3 + k] + ab[k] - wxv[k];
      }
      /* the world base is at rest: X v_base = 0 */
    } else {
      double S[6] = {0, 0, 0, 0, 0, 0};
      const double *ax = m->axis + 3 * i;
      if (m->jtype[i] == 0) { S[0] = ax[0]; S[1] = ax[1]; S[2] = ax[2]; }
      else { S[3] = ax[0]; S[4] = ax[1]; S[5] = ax[2]; }
      double sq[6], c6[6];
      for (int k = 0; k < 6; ++k) {
        sq[k] = S[k] * qd[d];
        vi[k] = xv[k] + sq[k];
      }
      crm(vi, sq, c6);
      for (int k = 0; k < 6; ++k) ai[k] = xa[k] + S[k] * qdd[d] + c6[k];
    }
    /* f = I a + v x* I v */
    double Ic[9] = {m->inertia[3 * i], 0, 0, 0, m->inertia[3 * i + 1], 0, 0, 0,
                    m->inertia[3 * i + 2]};
    double Ia[6], Iv[6], vxIv[6];
    inertia_mul(m->mass[i], m->com + 3 * i, Ic, ai, Ia);
    inertia_mul(m->mass[i], m->com + 3 * i, Ic, vi, Iv);
    crf(vi, Iv, vxIv);
    for (int k = 0; k < 6; ++k) f[6 * i + k] = Ia[k] + vxIv[k];
  }
  for (int i = n - 1; i >= 0; --i) {
    int pa = m->parent[i], d = m->dadr[i];
    double *fi = f + 6 * i;
    if (m->jtype[i] == 2) {
      double fw[3];
      mat_vec(R + 9 * i, fi + 3, fw);
      for (int k = 0; k < 3; ++k) {
        tau[d + k] = fw[k];
        tau[d + 3 + k] = fi[k];
      }
    } else {
      const double *ax = m->axis + 3 * i;
      tau[d] = (m->jtype[i] == 0) ? dot3(ax, fi) : dot3(ax, fi + 3);
    }
    if (pa >= 0) {
      /* X^T f: f_p = E f_c ; n_p = E n_c + r x (E f_c) */
      const double *Rp = R + 9 * pa;
      double dpw[3] = {p[3 * i] - p[3 * pa], p[3 * i + 1] - p[3 * pa + 1],
                       p[3 * i + 2] - p[3 * pa + 2]};
      double rr[3], E[9];
      mat_tvec(Rp, dpw, rr);
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
          double s = 0;
          for (int k = 0; k < 3; ++k) s += Rp[3 * k + r] * R[9 * i + 3 * k + c];
          E[3 * r + c] = s;
        }
      double Ef[3], En[3], rxf[3];
      mat_vec(E, fi + 3, Ef);
      mat_vec(E, fi, En);
      cross(rr, Ef, rxf);
      for (int k = 0; k < 3; ++k) {
        f[6 * pa + k] += En[k] + rxf[k];
        f[6 * pa + 3 + k] += Ef[k];
      }
    }
  }
  free(R); free(p); free(v); free(a); free(f);
}

/* ------------------------------------------------------ ground contact
 * Sphere (node b, centre x, radius rho) against the plane z = 0:
 * penetration d = rho - w_z of the centre w; the force acts at the lowest
 * point c = w - rho z. The penalty spring-damper is taken linearly
 * implicitly over the step (d at the end of the step ~ d - dt cdot_z), so
 * F_n = max(0, k d - (c_d + dt k) cdot_z); regularised Coulomb friction
 * F_t = -mu F_n v_t / s with s = sqrt(|v_t|^2 + v_s^2); tau_ext += J_c^T F.
 * If D is given, the velocity slope of the contact force is accumulated
 * into it: D += J_c^T diag(Dt, c_n) J_c with c_n = c_d + dt k while
 * F_n > 0 and Dt = mu F_n (I - v_t v_t^T / s^2) / s (the friction's own
 * Jacobian, dropping its dependence on F_n). */
void ora_contact(const ora_model *m, const double *q, const double *qd,
                 double dt, double *tau_ext, double *D, int *n_active) {
  int n = m->n_node, nv = m->nv, cnt = 0;
  memset(tau_ext, 0, sizeof(double) * nv);
  if (m->n_con == 0) {
    if (n_active) *n_active = 0;
    return;
  }
  double *R = (double *)malloc(sizeof(double) * 9 * n);
  double *p = (double *)malloc(sizeof(double) * 3 * n);
  double *Jv = (double *)malloc(sizeof(double) * 3 * nv);
  ora_fk(m, q, R, p);
  for (int c = 0; c < m->n_con; ++c) {
    double w[3];
    int b = m->con_node[c];
    world_point(R, p, b, m->con_pos + 3 * c, w);
    double rho = m->con_radius[c];
    double pen = rho - w[2];
    if (!(pen > 0.0)) continue;
    ++cnt;
    double cp[3] = {w[0], w[1], w[2] - rho};
    point_jacobian(m, R, p, b, cp, Jv, NULL);
    double cv[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
      for (int j = 0; j < nv; ++j) cv[r] += Jv[r * nv + j] * qd[j];
    double ceff = m->cc + dt * m->kc;
    double fn = fmax(0.0, m->kc * pen - ceff * cv[2]);
    double s = sqrt(cv[0] * cv[0] + cv[1] * cv[1] + m->vs * m->vs);
    double F[3] = {-m->mu * fn * cv[0] / s, -m->mu * fn * cv[1] / s, fn};
    for (int j = 0; j < nv; ++j)
      tau_ext[j] += Jv[j] * F[0] + Jv[nv + j] * F[1] + Jv[2 * nv + j] * F[2];
    if (D && fn > 0.0) {
      double Dc[9] = {0};
      double g = m->mu * fn / s;
      Dc[0] = g * (1.0 - cv[0] * cv[0] / (s * s));
      Dc[1] = Dc[3] = -g * cv[0] * cv[1] / (s * s);
      Dc[4] = g * (1.0 - cv[1] * cv[1] / (s * s));
      Dc[8] = ceff;
      for (int i = 0; i < nv; ++i)
        for (int j = 0; j < nv; ++j) {
          double t = 0;
          for (int a = 0; a < 3; ++a)
            for (int bb = 0; bb < 3; ++bb) t += Jv[a * nv + i] * Dc[3 * a + bb] * Jv[bb * nv + j];
          D[i * nv + j] += t;
        }
    }
  }
  if (n_active) *n_active = cnt;
  free(R); free(p); free(Jv);
}

/* ------------------------------------------------ dense Cholesky solve
 * M = L L^T (column by column), then L y = b, L^T x = y. */
int ora_chol_solve(int n, const double *M, const double *b, double *x) {
  double *L = (double *)calloc((size_t)n * n, sizeof(double));
  int ok = 0;
  for (int j = 0; j < n && ok == 0; ++j) {
    double s = M[j * n + j];
    for (int k = 0; k < j; ++k) s -= L[j * n + k] * L[j * n + k];
    if (!(s > 0.0)) { ok = -1; break; }
    double d = sqrt(s);
    L[j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = M[i * n + j];
      for (int k = 0; k < j; ++k) t -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = t / d;
    }
  }
  if (ok == 0) {
    for (int i = 0; i < n; ++i) {
      double t = b[i];
      for (int k = 0; k < i; ++k) t -= L[i * n + k] * x[k];
      x[i] = t / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
      double t = x[i];
      for (int k = i + 1; k < n; ++k) t -= L[k * n + i] * x[k];
      x[i] = t / L[i * n + i];
    }
  }
  free(L);
  return ok;
}

/* --------------------------------------------------------- energy */
double ora_energy(const ora_model *m, const double *q, const double *qd) {
  int n = m->n_node, nv = m->nv;
  double *M = (double *)malloc(sizeof(double) * nv * nv);
  double *R = (double *)malloc(sizeof(double) * 9 * n);
  double *p = (double *)malloc(sizeof(double) * 3 * n);
  ora_mass_matrix(m, q, M);
  ora_fk(m, q, R, p);
  double ke = 0.0, pe = 0.0;
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) ke += 0.5 * qd[i] * M[i * nv + j] * qd[j];
  for (int b = 0; b < n; ++b) {
    double c[3];
    world_point(R, p, b, m->com + 3 * b, c);
    pe -= m->mass[b] * dot3(m->g, c);
  }
  free(M); free(R); free(p);
  return ke + pe;
}

/* ------------------------------------------------------------ one step
 * Order: activation, geometry, Hill force, J_m^T F, M, C, contact,
 * damping, solve, then semi-implicit Euler (qd += dt qdd; q += dt qd;
 * root orientation xi <- normalise(xi * exp(w_b dt / 2))).
 * Dissipative forces are taken linearly-implicitly in velocity: the solve
 * is (M + dt D) qdd = tau_mus + tau_ext + tau_d - C with D the velocity
 * slope -d(tau)/d(qd) of joint damping (diag b), of the muscles'
 * force-velocity term (sum_m c_m r_m r_m^T, c_m = dF_m/dLdot =
 * F0 act f_l f_v'(v_m)/(v_max l_opt)) and of contact damping and friction.
 * Forces that depend on position stay explicit. */
static int all_finite(const double *x, int n) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(x[i])) return 0;
  return 1;
}

uint32_t ora_step(const ora_model *m, double dt, int contact_on, double *q,
                  double *qd, double *act, const double *u, ora_stage_out *out) {
  return ora_step_geo(m, dt, contact_on, q, qd, act, u, NULL, NULL, out);
}

/* Compliant-tendon muscles at the start of a step (see ora_step_tendon):
 * per muscle the force of the right-hand side F, its slope c in the new
 * lengthening rate and the balancing fibre velocity v (m/s). */
static void tendon_forces(const ora_model *m, const double *act1, const double *L,
                          const double *Ld, const double *lm, double dt, double eps0,
                          double beta, double *F, double *c, double *v, double *lm_out,
                          double *vm_out) {
  for (int i = 0; i < m->n_mus; ++i) {
    const double ls = m->l_slack[i], f0 = m->f0[i];
    const double strain = (L[i] - lm[i] - ls) / ls;           /* tendon strain */
    const double ft = strain > 0.0 ? strain / eps0 : 0.0;      /* F_t / F0 */
    const double k = strain > 0.0 ? f0 / (eps0 * ls) : 0.0;    /* dF_t / dl_t */
    const double l = lm[i] / m->l_opt[i];
    const double A = act1[i] * ora_fl(l);
    const double vn = ora_fv_root(A, ft - ora_fp(l), beta);   /* fibre balance */
    const double vs = m->v_max[i] * m->l_opt[i];               /* m/s per unit */
    const double b = f0 * (A * ora_fv_slope(vn) + beta) / vs;   /* dF_m / dv */
    const double cs = k * dt / (1.0 + k * dt / b);             /* series slope */
    v[i] = vn * vs;
    F[i] = f0 * ft + cs * (Ld[i] - v[i]);
    c[i] = cs;
    if (lm_out) lm_out[i] = l;
    if (vm_out) vm_out[i] = vn;
  }
}

/* Backward Euler on one fibre: the new length l' = l + dt v_max l_opt v'
 * balances fibre and tendon at the path length Ln,
 *   g(v') = act f_l(l'/l_opt) f_v(v') + f_p(l'/l_opt) + beta v'
 *           - max(0, (Ln - l' - l_slack) / l_slack) / eps0 = 0.
 * g rises strictly in v' when beta > 1.82 dt v_max (its slope is at least
 * beta - 1.4 max|f_l'| dt v_max, max|f_l'| < 1.3), so bisection finds the
 * one root: g <= 1.4 act + f_p(l / l_opt) + beta v' < 0 at
 * v' = min(0, -(1.4 act + f_p(l / l_opt)) / beta) - 1, and
 * g >= beta v' - f_t(Ln - l) > 0 at v' = max(0, f_t(Ln - l) / beta) + 1. */
static double fibre_update(const ora_model *m, int i, double act, double l, double Ln,
                           double dt, double eps0, double beta) {
  const double lo_m = m->l_opt[i], ls = m->l_slack[i];
  const double dl = dt * m->v_max[i] * lo_m;   /* metres per unit of v' */
  const double ft0 = fmax(0.0, (Ln - l - ls) / ls) / eps0;
  double lo = fmin(0.0, -(1.4 * act + ora_fp(l / lo_m)) / beta) - 1.0;
  double hi = fmax(0.0, ft0 / beta) + 1.0;
  for (int it = 0; it < 2000; ++it) {
    const double v = 0.5 * (lo + hi);
    if (v <= lo || v >= hi) break;
    const double ln = l + dl * v;
    const double g = act * ora_fl(ln / lo_m) * ora_fv(v) + ora_fp(ln / lo_m) + beta * v -
                     fmax(0.0, (Ln - ln - ls) / ls) / eps0;
    if (g < 0.0)
      lo = v;
    else
      hi = v;
  }
  return l + dl * 0.5 * (lo + hi);
}

static uint32_t step_core(const ora_model *m, double dt, int contact_on, double *q,
                          double *qd, double *act, const double *u, const double *L_in,
                          const double *r_in, double *lmf, double eps0, double beta,
                          ora_stage_out *out) {
  int nv = m->nv, nq = m->nq, nm = m->n_mus, n = m->n_node;
  if (!all_finite(q, nq) || !all_finite(qd, nv) || !all_finite(act, nm) ||
      (lmf && !all_finite(lmf, nm)))
    return ORA_ST_NONFINITE;
  double *cmu = (double *)malloc(sizeof(double) * nm);
  double *vf = (double *)malloc(sizeof(double) * nm);
  double *lmn = (double *)malloc(sizeof(double) * nm);
  double *act1 = (double *)malloc(sizeof(double) * nm);
  double *L = (double *)malloc(sizeof(double) * nm);
  double *Ld = (double *)malloc(sizeof(double) * nm);
  double *F = (double *)malloc(sizeof(double) * nm);
  double *r = (double *)malloc(sizeof(double) * (size_t)nm * nv);
  double *M = (double *)malloc(sizeof(double) * nv * nv);
  double *tm = (double *)calloc(nv, sizeof(double));
  double *te = (double *)calloc(nv, sizeof(double));
  double *td = (double *)malloc(sizeof(double) * nv);
  double *C = (double *)malloc(sizeof(double) * nv);
  double *rhs = (double *)malloc(sizeof(double) * nv);
  double *qdd = (double *)malloc(sizeof(double) * nv);
  double *zero = (double *)calloc(nv, sizeof(double));
  double *D = (double *)calloc((size_t)nv * nv, sizeof(double));
  double *qn = (double *)malloc(sizeof(double) * nq);
  double *qdn = (double *)malloc(sizeof(double) * nv);
  uint32_t st = 0;

  ora_activation(m, dt, u, act, act1);
  if (L_in) {
    /* given geometry; the lengthening rate follows from r = -dL/dq */
    memcpy(L, L_in, sizeof(double) * nm);
    memcpy(r, r_in, sizeof(double) * (size_t)nm * nv);
    for (int mu = 0; mu < nm; ++mu) {
      double s = 0.0;
      for (int j = 0; j < nv; ++j) s -= r[(size_t)mu * nv + j] * qd[j];
      Ld[mu] = s;
    }
  } else {
    ora_geometry(m, q, qd, L, r, Ld);
  }
  if (lmf) {
    tendon_forces(m, act1, L, Ld, lmf, dt, eps0, beta, F, cmu, vf, out ? out->lm : NULL,
                  out ? out->vm : NULL);
  } else {
    ora_hill(m, act1, L, Ld, F, out ? out->lm : NULL, out ? out->vm : NULL);
    for (int mu = 0; mu < nm; ++mu) {
      double lm = (L[mu] - m->l_slack[mu]) / m->l_opt[mu];
      double vm = Ld[mu] / (m->v_max[mu] * m->l_opt[mu]);
      cmu[mu] = m->f0[mu] * act1[mu] * ora_fl(lm) * ora_fv_slope(vm) /
                (m->v_max[mu] * m->l_opt[mu]);
    }
  }
  for (int mu = 0; mu < nm; ++mu)
    for (int j = 0; j < nv; ++j) tm[j] += r[(size_t)mu * nv + j] * F[mu];
  ora_mass_matrix(m, q, M);
  ora_rnea(m, q, qd, zero, 1, C);
  if (contact_on) ora_contact(m, q, qd, dt, te, D, NULL);
  double *teq = (double *)calloc(nv, sizeof(double));
  ora_coupling(m, q, qd, dt, teq, D, NULL);
  for (int j = 0; j < nv; ++j) {
    td[j] = -m->damping[j] * qd[j];
    rhs[j] = tm[j] + te[j] + td[j] + teq[j] - C[j];
    D[j * nv + j] += m->damping[j];
  }
  for (int mu = 0; mu < nm; ++mu) {
    const double cm = cmu[mu];
    const double *rm = r + (size_t)mu * nv;
    for (int i = 0; i < nv; ++i) {
      if (rm[i] == 0.0) continue;
      for (int j = 0; j < nv; ++j) D[i * nv + j] += cm * rm[i] * rm[j];
    }
  }
  double *Mt = (double *)malloc(sizeof(double) * nv * nv);
  for (int k = 0; k < nv * nv; ++k) Mt[k] = M[k] + dt * D[k];
  if (ora_chol_solve(nv, Mt, rhs, qdd) != 0) st |= ORA_ST_NONSPD;
  free(Mt);

  if (!st) {
    for (int j = 0; j < nv; ++j) qdn[j] = qd[j] + dt * qdd[j];
    for (int i = 0; i < n; ++i) {
      int a = m->qadr[i], d = m->dadr[i];
      if (m->jtype[i] != 2) {
        qn[a] = q[a] + dt * qdn[d];
        continue;
      }
      for (int k = 0; k < 3; ++k) qn[a + k] = q[a + k] + dt * qdn[d + k];
      double th[3] = {qdn[d + 3] * dt, qdn[d + 4] * dt, qdn[d + 5] * dt};
      double ang = sqrt(dot3(th, th));
      double dq[4];
      if (ang < 1e-8) {
        dq[0] = 1.0; dq[1] = 0.5 * th[0]; dq[2] = 0.5 * th[1]; dq[3] = 0.5 * th[2];
      } else {
        double s = sin(0.5 * ang) / ang;
        dq[0] = cos(0.5 * ang); dq[1] = s * th[0]; dq[2] = s * th[1]; dq[3] = s * th[2];
      }
      const double *x = q + a + 3;
      double o[4];
      o[0] = x[0] * dq[0] - x[1] * dq[1] - x[2] * dq[2] - x[3] * dq[3];
      o[1] = x[0] * dq[1] + x[1] * dq[0] + x[2] * dq[3] - x[3] * dq[2];
      o[2] = x[0] * dq[2] - x[1] * dq[3] + x[2] * dq[0] + x[3] * dq[1];
      o[3] = x[0] * dq[3] + x[1] * dq[2] - x[2] * dq[1] + x[3] * dq[0];
      double nrm = sqrt(o[0] * o[0] + o[1] * o[1] + o[2] * o[2] + o[3] * o[3]);
      for (int k = 0; k < 4; ++k) qn[a + 3 + k] = o[k] / nrm;
    }
    if (lmf) {
      /* the fibre takes a backward-Euler step against the path length at the
       * step's end (first order: L + dt Ldot', Ldot' = -r qd') */
      for (int mu = 0; mu < nm; ++mu) {
        double ldn = 0.0;
        for (int j = 0; j < nv; ++j) ldn -= r[(size_t)mu * nv + j] * qdn[j];
        lmn[mu] = fibre_update(m, mu, act1[mu], lmf[mu], L[mu] + dt * ldn, dt, eps0, beta);
      }
    }
    if (!all_finite(qn, nq) || !all_finite(qdn, nv) || !all_finite(act1, nm) ||
        (lmf && !all_finite(lmn, nm)))
      st |= ORA_ST_NONFINITE;
  }
  if (out) {
    if (out->act) memcpy(out->act, act1, sizeof(double) * nm);
    if (out->L) memcpy(out->L, L, sizeof(double) * nm);
    if (out->Ldot) memcpy(out->Ldot, Ld, sizeof(double) * nm);
    if (out->F) memcpy(out->F, F, sizeof(double) * nm);
    if (out->r) memcpy(out->r, r, sizeof(double) * (size_t)nm * nv);
    if (out->tau_mus) memcpy(out->tau_mus, tm, sizeof(double) * nv);
    if (out->tau_ext) memcpy(out->tau_ext, te, sizeof(double) * nv);
    if (out->tau_eq) memcpy(out->tau_eq, teq, sizeof(double) * nv);
    if (out->tau_d) memcpy(out->tau_d, td, sizeof(double) * nv);
    if (out->C) memcpy(out->C, C, sizeof(double) * nv);
    if (out->qdd) memcpy(out->qdd, qdd, sizeof(double) * nv);
    if (out->M) memcpy(out->M, M, sizeof(double) * nv * nv);
    if (out->D) memcpy(out->D, D, sizeof(double) * nv * nv);
  }
  if (!st) {
    memcpy(q, qn, sizeof(double) * nq);
    memcpy(qd, qdn, sizeof(double) * nv);
    memcpy(act, act1, sizeof(double) * nm);
    if (lmf) memcpy(lmf, lmn, sizeof(double) * nm);
  }
  free(cmu); free(vf); free(lmn);
  free(act1); free(L); free(Ld); free(F); free(r); free(M); free(tm); free(te);
  free(td); free(C); free(rhs); free(qdd); free(zero); free(qn); free(qdn);
  free(D); free(teq);
  return st;
}

uint32_t ora_step_geo(const ora_model *m, double dt, int contact_on, double *q,
                      double *qd, double *act, const double *u, const double *L_in,
                      const double *r_in, ora_stage_out *out) {
  return step_core(m, dt, contact_on, q, qd, act, u, L_in, r_in, NULL, 0.0, 0.0, out);
}

uint32_t ora_step_tendon(const ora_model *m, double dt, int contact_on, double *q,
                         double *qd, double *act, double *lm, const double *u, double eps0,
                         double beta, ora_stage_out *out) {
  return step_core(m, dt, contact_on, q, qd, act, u, NULL, NULL, lm, eps0, beta, out);
}

void ora_rollout(const ora_model *m, int n_env, int n_steps, double dt,
                 int contact_on, double *q, double *qd, double *act,
                 const float *u, uint32_t *status, int n_threads) {
  int nq = m->nq, nv = m->nv, nm = m->n_mus;
#ifdef _OPENMP
  if (n_threads < 1) n_threads = 1;
#pragma omp parallel num_threads(n_threads)
#endif
  {
    double *ue = (double *)malloc(sizeof(double) * nm);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
    for (int e = 0; e < n_env; ++e) {
      for (int t = 0; t < n_steps; ++t) {
        const float *ut = u + ((size_t)t * n_env + e) * nm;
        for (int i = 0; i < nm; ++i) ue[i] = (double)ut[i];
        status[e] |= ora_step(m, dt, contact_on, q + (size_t)e * nq,
                              qd + (size_t)e * nv, act + (size_t)e * nm, ue, NULL);
      }
    }
    free(ue);
  }
}
