// ms_step.hip -- host side of the step: the model object, the C ABI entry
// points and launch dispatch. The kernels are in ms_step_kernel.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ms.h"
#include "ms_model.h"
#include "ms_step_types.h"


// =============================================================== host / ABI
void ms_surrogate_tables(const ms_model *m, std::vector<int> *q_index, std::vector<float> *lo,
                         std::vector<float> *hi) {
  const ms::Tables &t = m->t;
  for (int i = 0; i < t.n_node; ++i) {
    if (t.jtype[i] == 2) continue;
    q_index->push_back(t.qadr[i]);
    lo->push_back(t.qlo[t.dadr[i]]);
    hi->push_back(t.qhi[t.dadr[i]]);
  }
}

namespace {
thread_local std::string g_err;

ms_status fail(ms_status s, const std::string &m) {
  g_err = m;
  return s;
}

struct Packer {
  std::vector<unsigned char> buf;
  template <class T>
  size_t add(const std::vector<T> &v) {
    size_t off = (buf.size() + 255) & ~size_t(255);
    buf.resize(off + std::max<size_t>(v.size() * sizeof(T), 4));
    if (!v.empty()) std::memcpy(buf.data() + off, v.data(), v.size() * sizeof(T));
    return off;
  }
};

ms_status check_opts(const ms_step_opts *o) {
  if (!o) return fail(MS_E_ARG, "opts is NULL");
  if (!(o->dt > 0.0f) || !std::isfinite(o->dt)) return fail(MS_E_ARG, "dt must be positive and finite");
  return MS_OK;
}
}  // namespace

// Launches of at least this many envs run in two concurrent parts when the
// model's split-stream setting is automatic.
constexpr int kTwoStreamEnvs = 4096;

int effective_schedule(const ms_model *m) {
  if (m->schedule != MS_SCHED_AUTO) return m->schedule;
  // split when the fused step keeps at most one wavefront per SIMD
  const int W = ms::default_env_per_wg(m->t);
  const size_t per_wg = m->t.lt.size() * 4 + (size_t)W * m->t.lds_bytes;
  const int resident = W * (int)((160 * 1024) / per_wg);
  return resident <= 4 ? MS_SCHED_SPLIT : MS_SCHED_FUSED;
}

// the model's extra streams and their fork/join events (made once, outside
// any capture)
hipError_t make_part_streams(ms_model *m) {
  if (m->sx[0]) return hipSuccess;
  hipError_t e = hipEventCreateWithFlags(&m->ev_fork, hipEventDisableTiming);
  for (int i = 0; i < ms_model::kMaxParts - 1 && e == hipSuccess; ++i) {
    e = hipStreamCreateWithFlags(&m->sx[i], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&m->ev_join[i], hipEventDisableTiming);
  }
  return e;
}

ms_status reserve_split(ms_model *m, int n_env, hipStream_t st) {
  if (n_env <= m->ws_cap) return MS_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(MS_E_ARG, "the split step's workspace holds " + std::to_string(m->ws_cap) +
                              " envs, fewer than " + std::to_string(n_env) +
                              ": call ms_model_reserve before capturing");
  const ms::SplitLayout &L = m->t.split;
  const size_t E = (size_t)n_env;
  const size_t sz[9] = {E * L.ws_frames, E * L.ws_S, E * L.ws_H, E * L.ws_rhs, E * L.ws_tau,
                        E * L.ws_dsum, E * L.ws_act, E * 4, E * 4};
  void *p[9] = {};
  for (int i = 0; i < 9; ++i) {
    if (hipMalloc(&p[i], std::max<size_t>(sz[i], 4)) != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipFree(p[j]);
      return fail(MS_E_ALLOC, "split step workspace allocation failed (" + std::to_string(n_env) +
                                  " envs)");
    }
  }
  for (int i = 0; i < 9; ++i) m->ws_owned.push_back(p[i]);
  ms::KSplit &w = m->ks;
  w.frames = (float *)p[0];
  w.S = (float *)p[1];
  w.H = (double *)p[2];
  w.rhs = (double *)p[3];
  w.tau = (float *)p[4];
  w.dsum = (double *)p[5];
  w.actn = (float *)p[6];
  w.flag = (int *)p[7];
  w.mflag = (int *)p[8];
  m->ws_cap = n_env;
  return MS_OK;
}

// The compliant-tendon fibre scratch (5 n_mus floats per env), grown like
// the split workspace.
ms_status reserve_fib(ms_model *m, int n_env, hipStream_t st) {
  if (n_env <= m->fib_cap) return MS_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(MS_E_ARG, "the fibre scratch holds " + std::to_string(m->fib_cap) +
                              " envs, fewer than " + std::to_string(n_env) +
                              ": run a tendon rollout of as many envs before capturing");
  void *p = nullptr;
  if (hipMalloc(&p, std::max<size_t>((size_t)n_env * 5 * m->t.n_mus * 4, 4)) != hipSuccess)
    return fail(MS_E_ALLOC, "fibre scratch allocation failed (" + std::to_string(n_env) + " envs)");
  m->ws_owned.push_back(p);
  m->fib = (float *)p;
  m->fib_cap = n_env;
  return MS_OK;
}

// Parts of a split-step launch over n_env envs when `parts` were asked for:
// sets the model's envs per workgroup for them and the env bounds
// (bounds[h] .. bounds[h + 1] for part h); returns the number of non-empty
// parts. Equal parts, except that with two parts the first takes exactly
// one full round of the kinematics kernel (a workgroup of w_front envs on
// every CU) when that holds more than half the batch (measured on the whole
// body at 4096 envs with 10 envs per workgroup: 2560 + 1536 envs 0.287 ms
// per step, 2048 + 2048 0.296; one env past the round costs a second round:
// 2688 + 1408 0.307).
int plan_parts(ms_model *m, int n_env, int parts, int *bounds) {
  parts = std::max(1, std::min(parts, std::min(n_env, (int)ms_model::kMaxParts)));
  const int per = (n_env + parts - 1) / parts;
  if (m->w_n_env != per || m->w_parts != parts) {
    ms::split_env_per_wg(m->k, m->ks, per, parts, &m->w_front, &m->w_back);
    m->w_n_env = per;
    m->w_parts = parts;
  }
  for (int h = 0; h <= parts; ++h) bounds[h] = std::min(n_env, h * per);
  if (parts == 2) {
    const int round = ms::device_cu_count() * m->w_front;
    if (round > per && round < n_env) bounds[1] = round;
  }
  while (parts > 1 && bounds[parts - 1] >= bounds[parts]) --parts;  // no empty part
  bounds[parts] = n_env;
  return parts;
}

hipError_t launch(ms_model *m, const ms::KRun &r, int n_env, int n_steps, hipStream_t st) {
  const int nvia = m->t.n_via_max;
  // a coupled model's surrogate step runs on the split schedule only
  const bool coupled_surr = m->t.n_eq > 0 && r.geomY;
  // compliant tendons run on the split schedule only
  if (r.stages || (effective_schedule(m) == MS_SCHED_FUSED && !coupled_surr && !r.lm)) {
    if (nvia <= 2) return ms::launch_nvia<2>(m->t, m->k, r, n_env, n_steps, st);
    if (nvia <= 4) return ms::launch_nvia<4>(m->t, m->k, r, n_env, n_steps, st);
    if (nvia <= 6) return ms::launch_nvia<6>(m->t, m->k, r, n_env, n_steps, st);
    return ms::launch_nvia<8>(m->t, m->k, r, n_env, n_steps, st);
  }
  if (reserve_split(m, n_env, st) != MS_OK) return hipErrorOutOfMemory;
  const ms::KSplit &w = m->ks;
  // the batch in parts on streams of their own (the caller's and the
  // model's), so that one part's kernels overlap the others'
  int parts = r.one_stream ? 1
              : m->split_streams > 0 ? m->split_streams
                                     : (n_env >= kTwoStreamEnvs ? 2 : 1);
  parts = std::max(1, std::min(parts, n_env));
  if (parts > 1 && !m->sx[0]) {
    // the streams are made outside a capture (ms_model_reserve makes them);
    // a capture that finds none steps the batch on one stream
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone)
      parts = 1;
    else if (hipError_t e = make_part_streams(m); e != hipSuccess)
      return e;
  }
  int bounds[ms_model::kMaxParts + 1];
  parts = plan_parts(m, n_env, parts, bounds);
  const int mpt = (m->t.n_mus + 255) / 256;
  bool timed = m->timing > 0;
  if (timed) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    timed = hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusNone;
  }
  // one kernel, bracketed by timing events when timing is on (the first
  // half's kernels on the caller's stream)
  int s = 0;
  auto timed_launch = [&](int kernel, bool on, auto &&fn) -> hipError_t {
    if (!on || !timed || s % m->timing) return fn();
    hipEvent_t ev[2];
    for (int i = 0; i < 2; ++i) {
      if (m->ev_free.empty()) {
        hipError_t e = hipEventCreate(&ev[i]);
        if (e != hipSuccess) return e;
      } else {
        ev[i] = m->ev_free.back();
        m->ev_free.pop_back();
      }
    }
    hipError_t e = hipEventRecord(ev[0], st);
    if (e == hipSuccess) e = fn();
    if (e == hipSuccess) e = hipEventRecord(ev[1], st);
    m->ev_pending.push_back({kernel, ev[0], ev[1]});
    return e;
  };
  constexpr int P = ms_model::kMaxParts;
  ms::KRun rh[P];
  hipStream_t sh[P] = {st};
  for (int h = 0; h < parts; ++h) {
    rh[h] = r;
    rh[h].env_begin = bounds[h];
    rh[h].env_end = bounds[h + 1];
    if (h) sh[h] = m->sx[h - 1];
  }
  if (parts > 1) {
    hipError_t e = hipEventRecord(m->ev_fork, st);
    for (int h = 1; h < parts && e == hipSuccess; ++h) e = hipStreamWaitEvent(sh[h], m->ev_fork, 0);
    if (e != hipSuccess) return e;
  }
  for (s = 0; s < n_steps; ++s) {
    hipError_t e = hipSuccess;
    for (int h = 0; h < parts && e == hipSuccess; ++h)
      e = timed_launch(0, h == 0, [&] { return ms::launch_front(m->k, rh[h], w, m->w_front, s, sh[h]); });
    for (int h = 0; h < parts && e == hipSuccess; ++h)
      e = timed_launch(1, h == 0, [&] {
        if (nvia <= 2) return ms::launch_muscle<2>(m->k, rh[h], w, mpt, s, sh[h]);
        if (nvia <= 4) return ms::launch_muscle<4>(m->k, rh[h], w, mpt, s, sh[h]);
        if (nvia <= 6) return ms::launch_muscle<6>(m->k, rh[h], w, mpt, s, sh[h]);
        return ms::launch_muscle<8>(m->k, rh[h], w, mpt, s, sh[h]);
      });
    for (int h = 0; h < parts && e == hipSuccess; ++h)
      e = timed_launch(2, h == 0, [&] { return ms::launch_back(m->k, rh[h], w, m->w_back, s, sh[h]); });
    for (int h = 0; h < parts && e == hipSuccess && r.lm; ++h)
      e = ms::launch_fibre(m->k, rh[h], w, sh[h]);
    if (e != hipSuccess) return e;
  }
  for (int h = 1; h < parts; ++h) {
    hipError_t e = hipEventRecord(m->ev_join[h - 1], sh[h]);
    if (e == hipSuccess) e = hipStreamWaitEvent(st, m->ev_join[h - 1], 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

ms_status run_steps(ms_model *m, const ms::KRun &r, int n_env, int n_steps, hipStream_t st) {
  if (!r.stages && (effective_schedule(m) == MS_SCHED_SPLIT || r.lm)) {
    const ms_status s = reserve_split(m, n_env, st);
    if (s != MS_OK) return s;
  }
  const hipError_t e = launch(m, r, n_env, n_steps, st);
  if (e != hipSuccess) return fail(MS_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return MS_OK;
}

extern "C" {

const char *ms_last_error(void) { return g_err.c_str(); }

ms_status ms_model_create(const ms_model_desc *desc, ms_model **out) {
  g_err.clear();
  if (!out) return fail(MS_E_ARG, "out is NULL");
  *out = nullptr;
  ms_model *m = new (std::nothrow) ms_model();
  if (!m) return fail(MS_E_ALLOC, "host allocation failed");
  std::string msg;
  ms_status s = ms::build_tables(desc, &m->t, &msg);
  if (s != MS_OK) {
    delete m;
    return fail(s, msg);
  }
  const ms::Tables &t = m->t;
  if (t.nv > 128) {
    delete m;
    return fail(MS_E_UNSUPPORTED, "more than 128 DoFs");
  }
  if (t.lt.size() * 4 + (size_t)t.lds_bytes > 160 * 1024) {
    delete m;
    return fail(MS_E_UNSUPPORTED,
                "model needs more than 160 KiB of LDS for a workgroup of one environment");
  }
  Packer p;
  size_t o_parent = p.add(t.parent), o_jtype = p.add(t.jtype), o_qadr = p.add(t.qadr),
         o_dadr = p.add(t.dadr), o_ls = p.add(t.level_start), o_ln = p.add(t.level_nodes),
         o_jpos = p.add(t.jpos), o_jrot = p.add(t.jrot), o_axis = p.add(t.axis),
         o_bnode = p.add(t.body_node), o_bmass = p.add(t.body_mass), o_bcom = p.add(t.body_com),
         o_bin = p.add(t.body_inertia), o_sbs = p.add(t.subb_start), o_sb = p.add(t.subb),
         o_scs = p.add(t.subc_start), o_sc = p.add(t.subc), o_cn = p.add(t.con_node),
         o_cp = p.add(t.con_pos), o_cr = p.add(t.con_radius), o_dn = p.add(t.dof_node),
         o_dk = p.add(t.dof_kind), o_damp = p.add(t.damping), o_f0 = p.add(t.mus_f0),
         o_il = p.add(t.mus_ilopt), o_ls2 = p.add(t.mus_lslack), o_ivl = p.add(t.mus_ivl),
         o_ta = p.add(t.mus_tact), o_td = p.add(t.mus_tdeact), o_nvia = p.add(t.mus_nvia),
         o_vn = p.add(t.via_node), o_vp = p.add(t.via_pos), o_span = p.add(t.mus_span), o_srec = p.add(t.mus_srec),
         o_mext = p.add(t.mus_ext), o_mint = p.add(t.mus_int), o_gnv = p.add(t.grp_nvia),
         o_qlo = p.add(t.qlo), o_qhi = p.add(t.qhi),
         o_mask = p.add(t.mus_mask), o_ps = p.add(t.proj_start), o_pd = p.add(t.proj_dof), o_pi = p.add(t.proj_item),
         o_dh = p.add(t.dent_h), o_ds = p.add(t.dent_start), o_di = p.add(t.dent_item),
         o_rs = p.add(t.row_start), o_dd = p.add(t.dof_depth), o_path = p.add(t.path),
         o_nr = p.add(t.nnz_row), o_hs = p.add(t.hlev_start),
         o_hd = p.add(t.hlev_dof),
         o_lt = p.add(t.lt),
         o_eqs = p.add(t.eq_start), o_eqq = p.add(t.eq_qi), o_eqdf = p.add(t.eq_dof),
         o_eqc = p.add(t.eq_coef), o_eqo = p.add(t.eq_off), o_eds = p.add(t.eqd_start),
         o_edd = p.add(t.eqd_dof), o_edc = p.add(t.eqd_c), o_edw = p.add(t.eqd_coef),
         o_ehh = p.add(t.eqh_h), o_ehw = p.add(t.eqh_w);
  m->dbytes = p.buf.size();
  hipError_t e = hipMalloc(&m->dbuf, m->dbytes);
  if (e != hipSuccess) {
    std::string es = hipGetErrorString(e);
    delete m;
    return fail(MS_E_ALLOC, "hipMalloc: " + es);
  }
  e = hipMemcpy(m->dbuf, p.buf.data(), m->dbytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    std::string es = hipGetErrorString(e);
    (void)hipFree(m->dbuf);
    delete m;
    return fail(MS_E_HIP, "hipMemcpy: " + es);
  }
  unsigned char *b = (unsigned char *)m->dbuf;
  ms::KModel &k = m->k;
  k.n_node = t.n_node; k.nq = t.nq; k.nv = t.nv; k.n_mus = t.n_mus; k.n_con = t.n_con;
  k.n_body = t.n_body; k.nnz = t.nnz; k.n_level = t.n_level; k.free_root = t.free_root;
  k.n_dent = t.n_dent;
  k.n_hlev = t.n_hlev; k.n_hgat = t.n_hgat; k.n_trunk = t.n_trunk;
  k.n_dlev = t.n_dlev;
  k.kc = t.kc; k.cc = t.cc; k.mu = t.mu; k.vs = t.vs; k.gx = t.g[0]; k.gy = t.g[1]; k.gz = t.g[2];
#define P_(field, off, T) k.field = (const T *)(b + off)
  P_(parent, o_parent, int); P_(jtype, o_jtype, int); P_(qadr, o_qadr, int); P_(dadr, o_dadr, int);
  P_(level_start, o_ls, int); P_(level_nodes, o_ln, int); P_(jpos, o_jpos, float);
  P_(jrot, o_jrot, float); P_(axis, o_axis, float); P_(body_node, o_bnode, int);
  P_(body_mass, o_bmass, float); P_(body_com, o_bcom, float); P_(body_inertia, o_bin, float);
  P_(subb_start, o_sbs, int); P_(subb, o_sb, int); P_(subc_start, o_scs, int); P_(subc, o_sc, int);
  P_(con_node, o_cn, int); P_(con_pos, o_cp, float); P_(con_radius, o_cr, float);
  P_(dof_node, o_dn, int); P_(dof_kind, o_dk, int); P_(damping, o_damp, float);
  P_(mus_f0, o_f0, float); P_(mus_ilopt, o_il, float); P_(mus_lslack, o_ls2, float);
  P_(mus_ivl, o_ivl, float); P_(mus_tact, o_ta, float); P_(mus_tdeact, o_td, float);
  P_(mus_nvia, o_nvia, int); P_(via_node, o_vn, int); P_(via_pos, o_vp, float);
  P_(mus_ext, o_mext, int); P_(mus_int, o_mint, int); P_(grp_nvia, o_gnv, int);
  P_(qlo, o_qlo, float); P_(qhi, o_qhi, float);
  P_(mus_span, o_span, int); P_(mus_srec, o_srec, int); P_(mus_mask, o_mask, unsigned); P_(proj_start, o_ps, int); P_(proj_dof, o_pd, int);
  P_(proj_item, o_pi, int); P_(dent_h, o_dh, int); P_(dent_start, o_ds, int);
  P_(dent_item, o_di, int); P_(row_start, o_rs, int); P_(dof_depth, o_dd, int);
  P_(path, o_path, int); P_(nnz_row, o_nr, int);
  P_(lt, o_lt, int);
  k.lt_words = (int)t.lt.size();
  k.lt_hent_start = t.lt_hent_start; k.lt_hlev_start = t.lt_hlev_start;
  k.lt_hent = t.lt_hent; k.lt_hdof = t.lt_hdof;
  k.lt_desc = t.lt_desc; k.lt_drange = t.lt_drange; k.lt_rs = t.lt_rs;
  k.lt_trow = t.lt_trow; k.lt_tpair = t.lt_tpair;
  k.lt_path = t.lt_path; k.lt_tlev = t.lt_tlev; k.lt_tnode = t.lt_tnode;
  k.lt_subb_start = t.lt_subb_start; k.lt_subc_start = t.lt_subc_start; k.lt_subb = t.lt_subb;
  k.lt_subc = t.lt_subc; k.lt_nnzrow = t.lt_nnzrow;
  k.lt_cinode = t.lt_cinode; k.lt_dofci = t.lt_dofci;
  k.lt_front_end = t.lt_front_end; k.lt_back_begin = t.lt_back_begin;
  k.n_ci = t.n_ci;
  P_(hlev_start, o_hs, int); P_(hlev_dof, o_hd, int);
  k.n_eq = t.n_eq; k.n_eqd = t.n_eqd; k.n_eqh = t.n_eqh; k.eq_k = t.eq_k; k.eq_d = t.eq_d;
  P_(eq_start, o_eqs, int); P_(eq_qi, o_eqq, int); P_(eq_dof, o_eqdf, int);
  P_(eq_coef, o_eqc, float); P_(eq_off, o_eqo, float); P_(eqd_start, o_eds, int);
  P_(eqd_dof, o_edd, int); P_(eqd_c, o_edc, int); P_(eqd_coef, o_edw, float);
  P_(eqh_h, o_ehh, int); P_(eqh_w, o_ehw, float);
#undef P_
  k.off_flag = t.off_flag; k.off_q = t.off_q; k.off_qd = t.off_qd; k.off_R = t.off_R;
  k.off_P = t.off_P; k.off_S = t.off_S; k.off_con = t.off_con; k.off_rhs = t.off_rhs;
  k.off_x = t.off_x; k.off_H = t.off_H; k.off_scr = t.off_scr; k.lds_env = t.lds_bytes; k.off_V = t.off_V;
  k.off_A = t.off_A; k.off_F = t.off_F;
  {
    const ms::SplitLayout &L = t.split;
    ms::KSplit &w = m->ks;
    w.fr_stride = (int)(L.ws_frames / 4);
    w.S_stride = (int)(L.ws_S / 4);
    w.H_stride = (int)(L.ws_H / 8);
    w.rhs_stride = (int)(L.ws_rhs / 8);
    w.tau_stride = (int)(L.ws_tau / 4);
    w.dsum_stride = (int)(L.ws_dsum / 8);
    w.act_stride = (int)(L.ws_act / 4);
    w.f_R = L.f_R; w.f_S = L.f_S; w.f_con = L.f_con;
    w.f_scr = L.f_scr; w.f_bytes = L.f_bytes;
    w.b_q = L.b_q; w.b_qd = L.b_qd; w.b_x = L.b_x; w.b_invd = L.b_invd;
    w.b_H = L.b_H; w.b_bytes = L.b_bytes;
    w.m_R = L.m_R; w.m_S = L.m_S; w.m_q = L.m_q; w.m_qd = L.m_qd; w.m_scr = L.m_scr;
    w.m_bytes = L.m_bytes;
  }
  *out = m;
  return MS_OK;
}

void ms_model_destroy(ms_model *m) {
  if (!m) return;
  if (m->dbuf) (void)hipFree(m->dbuf);
  for (void *p : m->ws_owned) (void)hipFree(p);
  for (const auto &p : m->ev_pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : m->ev_free) (void)hipEventDestroy(e);
  if (m->key_buf) (void)hipFree(m->key_buf);
  for (int i = 0; i < ms_model::kMaxParts - 1; ++i) {
    if (m->sx[i]) (void)hipStreamDestroy(m->sx[i]);
    if (m->ev_join[i]) (void)hipEventDestroy(m->ev_join[i]);
  }
  if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
  delete m;
}

ms_status ms_model_set_schedule(ms_model *m, int32_t schedule) {
  g_err.clear();
  if (!m) return fail(MS_E_ARG, "model is NULL");
  if (schedule != MS_SCHED_AUTO && schedule != MS_SCHED_FUSED && schedule != MS_SCHED_SPLIT)
    return fail(MS_E_ARG, "unknown schedule");
  m->schedule = schedule;
  return MS_OK;
}

ms_status ms_model_set_split_streams(ms_model *m, int32_t streams) {
  g_err.clear();
  if (!m || streams < 0 || streams > ms_model::kMaxParts)
    return fail(MS_E_ARG, "streams must be 0 (automatic) or 1 to 4");
  m->split_streams = streams;
  return MS_OK;
}

ms_status ms_model_split_parts(ms_model *m, int32_t n_env, int32_t *bounds, int32_t *n_parts) {
  g_err.clear();
  if (!m || !bounds || !n_parts || n_env <= 0) return fail(MS_E_ARG, "NULL argument or n_env <= 0");
  const int want = effective_schedule(m) != MS_SCHED_SPLIT ? 1
                   : m->split_streams > 0                   ? m->split_streams
                                                            : (n_env >= kTwoStreamEnvs ? 2 : 1);
  int b[ms_model::kMaxParts + 1];
  const int parts = plan_parts(m, n_env, want, b);
  for (int h = 0; h <= parts; ++h) bounds[h] = b[h];
  *n_parts = parts;
  return MS_OK;
}

ms_status ms_model_get_schedule(const ms_model *m, int32_t *schedule) {
  g_err.clear();
  if (!m || !schedule) return fail(MS_E_ARG, "NULL argument");
  *schedule = effective_schedule(m);
  return MS_OK;
}

ms_status ms_model_set_kernel_timing(ms_model *m, int32_t every) {
  g_err.clear();
  if (!m) return fail(MS_E_ARG, "model is NULL");
  if (every < 0) return fail(MS_E_ARG, "every must be >= 0");
  m->timing = every;
  return MS_OK;
}

ms_status ms_model_kernel_times(ms_model *m, double *ms3, int64_t *n_steps) {
  g_err.clear();
  if (!m || !ms3 || !n_steps) return fail(MS_E_ARG, "NULL argument");
  double sum[3] = {0.0, 0.0, 0.0};
  int64_t n[3] = {0, 0, 0};
  hipError_t e = hipSuccess;
  for (const auto &p : m->ev_pending) {
    if (e == hipSuccess) e = hipEventSynchronize(p.b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, p.a, p.b);
    if (e == hipSuccess) {
      sum[p.kernel] += t;
      n[p.kernel] += 1;
    }
    m->ev_free.push_back(p.a);
    m->ev_free.push_back(p.b);
  }
  m->ev_pending.clear();
  if (e != hipSuccess) return fail(MS_E_HIP, std::string("kernel timing: ") + hipGetErrorString(e));
  for (int k = 0; k < 3; ++k) ms3[k] = sum[k];
  *n_steps = n[2];
  return MS_OK;
}

ms_status ms_model_reserve(ms_model *m, int32_t n_env) {
  g_err.clear();
  if (!m || n_env <= 0) return fail(MS_E_ARG, "NULL model or n_env <= 0");
  if (m->split_streams != 1 && make_part_streams(m) != hipSuccess)
    return fail(MS_E_ALLOC, "could not create the split step's streams");
  return reserve_split(m, n_env, nullptr);
}

ms_status ms_model_info_get(const ms_model *m, ms_model_info *o) {
  if (!m || !o) return fail(MS_E_ARG, "NULL argument");
  o->nq = m->t.nq; o->nv = m->t.nv; o->n_node = m->t.n_node; o->n_mus = m->t.n_mus;
  o->n_con = m->t.n_con; o->n_body = m->t.n_body; o->max_dof_depth = m->t.max_depth;
  o->nnz_mass = m->t.nnz; o->lds_bytes = m->t.lds_bytes;
  o->lds_shared_bytes = (int32_t)(m->t.lt.size() * 4);
  return MS_OK;
}

ms_status ms_model_spans(const ms_model *m, int32_t *spans) {
  if (!m || !spans) return fail(MS_E_ARG, "NULL argument");
  const int nm = m->t.n_mus;
  for (int i = 0; i < nm; ++i)
    for (int s = 0; s < 3; ++s) spans[3 * m->t.mus_ext[i] + s] = m->t.mus_span[(size_t)s * nm + i];
  return MS_OK;
}

ms_status ms_model_mass_pattern(const ms_model *m, int32_t *rows, int32_t *cols) {
  if (!m || !rows || !cols) return fail(MS_E_ARG, "NULL argument");
  for (int e = 0; e < m->t.nnz; ++e) {
    rows[e] = m->t.nnz_row[e];
    cols[e] = m->t.path[e];
  }
  return MS_OK;
}

static ms_status common_checks(const ms_model *m, int32_t n_env, const void *q, const void *qd,
                               const void *act, const ms_step_opts *o) {
  if (!m) return fail(MS_E_ARG, "model is NULL");
  if (n_env <= 0) return fail(MS_E_ARG, "n_env must be > 0");
  if (!q || !qd || (!act && m->t.n_mus > 0)) return fail(MS_E_ARG, "a state pointer is NULL");
  return check_opts(o);
}

static ms_status hip_status(hipError_t e) {
  if (e != hipSuccess) return fail(MS_E_HIP, std::string("kernel launch: ") + hipGetErrorString(e));
  return MS_OK;
}

ms_status ms_step_batch(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                        uint32_t *status, const float *u, const ms_step_opts *opts, void *stream) {
  g_err.clear();
  ms_status s = common_checks(m, n_env, q, qd, act, opts);
  if (s != MS_OK) return s;
  if (!u && m->t.n_mus > 0) return fail(MS_E_ARG, "u is NULL");
  ms::KRun r{};
  r.q = q; r.qd = qd; r.act = act; r.status = status; r.u = u; r.n_env = n_env;
  r.dt = opts->dt; r.contact = opts->contact;
  r.exc = ms::EXC_ARRAY;
  return run_steps(m, r, n_env, 1, (hipStream_t)stream);
}

ms_status ms_rollout(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                     uint32_t *status, const ms_excitation *exc, int32_t n_steps,
                     const ms_step_opts *opts, void *stream) {
  return rollout_impl(m, n_env, q, qd, act, status, exc, n_steps, opts, 0, (hipStream_t)stream);
}

static ms_status check_rec(const ms_model *m, const ms_record *rec) {
  if (!rec) return MS_OK;
  const bool any_obs = rec->act || rec->force || rec->lm || rec->vm || rec->power || rec->xpos ||
                       rec->xmat;
  if (any_obs && rec->every < 1) return fail(MS_E_ARG, "rec->every must be >= 1");
  if ((rec->xpos || rec->xmat) && m && m->k.n_key == 0)
    return fail(MS_E_ARG, "key-node observables need ms_model_set_key_nodes first");
  return MS_OK;
}

ms_status ms_rollout_record(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                            uint32_t *status, const ms_excitation *exc, int32_t n_steps,
                            const ms_step_opts *opts, const ms_record *rec, void *stream) {
  g_err.clear();
  if (const ms_status c = check_rec(m, rec); c != MS_OK) return c;
  return rollout_impl(m, n_env, q, qd, act, status, exc, n_steps, opts, 0, (hipStream_t)stream,
                      rec);
}

ms_status ms_rollout_tendon(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                            float *lm, uint32_t *status, const ms_excitation *exc,
                            int32_t n_steps, const ms_step_opts *opts, const ms_tendon *ten,
                            const ms_record *rec, void *stream) {
  g_err.clear();
  if (const ms_status c = check_rec(m, rec); c != MS_OK) return c;
  if (!m) return fail(MS_E_ARG, "model is NULL");
  if (!ten || !lm) return fail(MS_E_ARG, "ten or lm is NULL");
  if (!(ten->eps0 > 0.0f) || !std::isfinite(ten->eps0) || !(ten->beta > 0.0f) ||
      !std::isfinite(ten->beta))
    return fail(MS_E_ARG, "ten->eps0 and ten->beta must be positive and finite");
  for (float ls : m->t.mus_lslack)
    if (!(ls > 0.0f)) return fail(MS_E_ARG, "compliant tendons need every l_slack > 0");
  // the fibre's backward-Euler balance rises strictly in its velocity when
  // beta exceeds 1.4 max|f_l'| dt v_max (max|f_l'| < 1.3)
  if (opts && opts->dt > 0.0f)
    for (int i = 0; i < m->t.n_mus; ++i) {
      const float vmax = m->t.mus_ilopt[i] / m->t.mus_ivl[i];   // optimal lengths per second
      if (!(ten->beta > 1.82f * opts->dt * vmax))
        return fail(MS_E_ARG, "compliant tendons need beta > 1.82 dt v_max for every muscle");
    }
  return rollout_impl(m, n_env, q, qd, act, status, exc, n_steps, opts, 0, (hipStream_t)stream,
                      rec, false, lm, ten);
}

ms_status ms_model_set_key_nodes(ms_model *m, int32_t n_key, const int32_t *nodes) {
  g_err.clear();
  if (!m || n_key < 0 || n_key > 64 || (n_key > 0 && !nodes))
    return fail(MS_E_ARG, "bad arguments (0 <= n_key <= 64)");
  for (int k = 0; k < n_key; ++k)
    if (nodes[k] < 0 || nodes[k] >= m->t.n_node) return fail(MS_E_ARG, "key node out of range");
  hipError_t e = hipDeviceSynchronize();  // queued steps may read the old table
  if (e != hipSuccess) return fail(MS_E_HIP, std::string("synchronise: ") + hipGetErrorString(e));
  if (m->key_buf) (void)hipFree(m->key_buf);
  m->key_buf = nullptr;
  m->k.key_node = nullptr;
  m->k.n_key = 0;
  if (n_key == 0) return MS_OK;
  e = hipMalloc(&m->key_buf, 4 * (size_t)n_key);
  if (e != hipSuccess) return fail(MS_E_ALLOC, "hipMalloc: key nodes");
  e = hipMemcpy(m->key_buf, nodes, 4 * (size_t)n_key, hipMemcpyHostToDevice);
  if (e != hipSuccess) return fail(MS_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  m->k.key_node = (const int *)m->key_buf;
  m->k.n_key = n_key;
  return MS_OK;
}

}  // extern "C"

ms_status rollout_impl(ms_model *m, int32_t n_env, float *q, float *qd, float *act,
                       uint32_t *status, const ms_excitation *exc, int32_t n_steps,
                       const ms_step_opts *opts, int env_per_wg, hipStream_t st,
                       const ms_record *rec, bool one_stream, float *lm,
                       const ms_tendon *ten) {
  g_err.clear();
  ms_status s = common_checks(m, n_env, q, qd, act, opts);
  if (s != MS_OK) return s;
  if (!exc) return fail(MS_E_ARG, "exc is NULL");
  if (n_steps < 0) return fail(MS_E_ARG, "n_steps must be >= 0");
  if (n_steps == 0) return MS_OK;
  ms::KRun r{};
  r.q = q; r.qd = qd; r.act = act; r.status = status; r.n_env = n_env;
  r.dt = opts->dt; r.contact = opts->contact;
  r.u = exc->u; r.seed = exc->seed; r.step0 = exc->step0; r.xar = exc->x;
  r.rho = exc->rho; r.s = exc->s; r.mean = exc->mean;
  r.env_per_wg = env_per_wg;
  r.one_stream = one_stream;
  switch (exc->kind) {
    case MS_EXC_ARRAY:
      if (!exc->u && m->t.n_mus > 0) return fail(MS_E_ARG, "exc->u is NULL");
      break;
    case MS_EXC_IID:
      break;
    case MS_EXC_AR1:
      if (!exc->x && m->t.n_mus > 0) return fail(MS_E_ARG, "exc->x is NULL");
      break;
    default:
      return fail(MS_E_ARG, "unknown excitation kind");
  }
  r.exc = exc->kind;
  if (rec) {
    r.rec_every = rec->every;
    r.r_act = rec->act; r.r_F = rec->force; r.r_lm = rec->lm; r.r_vm = rec->vm;
    r.r_pow = rec->power; r.r_xpos = rec->xpos; r.r_xmat = rec->xmat;
    r.n_applied = rec->n_applied;
  }
  if (lm) {
    const ms_status fs = reserve_fib(m, n_env, st);
    if (fs != MS_OK) return fs;
    r.lm = lm;
    r.fib = m->fib;
    r.fib_stride = 5 * m->t.n_mus;
    r.ten_ieps = 1.0f / ten->eps0;
    r.ten_beta = ten->beta;
  }
  return run_steps(m, r, n_env, n_steps, st);
}

extern "C" {

ms_status ms_rollout_surrogate(ms_model *m, ms_surrogate *sg, int32_t n_env, float *q, float *qd,
                               float *act, uint32_t *status, const ms_excitation *exc,
                               int32_t n_steps, const ms_step_opts *opts, float tol,
                               uint32_t *fallback_count, void *stream) {
  g_err.clear();
  ms_status s = common_checks(m, n_env, q, qd, act, opts);
  if (s != MS_OK) return s;
  if (!sg || !exc) return fail(MS_E_ARG, "surrogate or exc is NULL");
  if (n_steps < 0) return fail(MS_E_ARG, "n_steps must be >= 0");
  if (exc->kind == MS_EXC_ARRAY && !exc->u && m->t.n_mus > 0) return fail(MS_E_ARG, "exc->u is NULL");
  if (exc->kind == MS_EXC_AR1 && !exc->x && m->t.n_mus > 0) return fail(MS_E_ARG, "exc->x is NULL");
  if (exc->kind < 0 || exc->kind > 2) return fail(MS_E_ARG, "unknown excitation kind");
  hipStream_t st = (hipStream_t)stream;
  for (int t = 0; t < n_steps; ++t) {
    const float *Y = nullptr;
    s = ms_surrogate_predict(sg, n_env, q, &Y, st);
    if (s != MS_OK) return fail(s, std::string("surrogate: ") + ms_surrogate_last_error());
    ms::KRun r{};
    r.q = q; r.qd = qd; r.act = act; r.status = status; r.n_env = n_env;
    r.dt = opts->dt; r.contact = opts->contact;
    r.u = exc->u ? exc->u + (size_t)t * n_env * m->t.n_mus : nullptr;
    r.seed = exc->seed; r.step0 = exc->step0 + t; r.xar = exc->x;
    r.rho = exc->rho; r.s = exc->s; r.mean = exc->mean;
    r.exc = exc->kind;
    r.geomY = Y; r.fb_tol = tol; r.fb_count = fallback_count;
    s = run_steps(m, r, n_env, 1, st);
    if (s != MS_OK) return s;
  }
  return MS_OK;
}

ms_status ms_geometry(ms_model *m, int32_t n, const float *q, float *L, float *r, void *stream) {
  g_err.clear();
  if (!m || n <= 0 || !q || !L || !r) return fail(MS_E_ARG, "NULL argument or n <= 0");
  ms::KRun k{};
  k.q = const_cast<float *>(q); k.qd = nullptr; k.act = nullptr; k.n_env = n; k.dt = 1e-3f;
  k.o_L = L; k.o_r = r; k.o_Ldot = nullptr;
  k.exc = ms::EXC_ARRAY;
  k.stages = 2;
  return hip_status(launch(m, k, n, 1, (hipStream_t)stream));
}

ms_status ms_step_stages(ms_model *m, int32_t n_env, const float *q, const float *qd,
                         const float *act, const float *u, const ms_step_opts *opts,
                         ms_stage_out *out, void *stream) {
  g_err.clear();
  ms_status s = common_checks(m, n_env, q, qd, act, opts);
  if (s != MS_OK) return s;
  if (!out || !out->act || !out->L || !out->Ldot || !out->F || !out->r || !out->tau_mus ||
      !out->bias_minus_ext || !out->qdd || !out->mass)
    return fail(MS_E_ARG, "every stage output buffer is required");
  if (!u && m->t.n_mus > 0) return fail(MS_E_ARG, "u is NULL");
  ms::KRun r{};
  r.q = const_cast<float *>(q); r.qd = const_cast<float *>(qd); r.act = const_cast<float *>(act);
  r.status = nullptr; r.u = u; r.n_env = n_env; r.dt = opts->dt; r.contact = opts->contact;
  r.o_act = out->act; r.o_L = out->L; r.o_Ldot = out->Ldot; r.o_F = out->F; r.o_r = out->r;
  r.o_tau = out->tau_mus; r.o_bias = out->bias_minus_ext; r.o_qdd = out->qdd; r.o_H = out->mass;
  r.exc = ms::EXC_ARRAY;
  r.stages = 1;
  return hip_status(launch(m, r, n_env, 1, (hipStream_t)stream));
}

}  // extern "C"
