// ms_model.cpp -- validation of a model description and construction of the
// flat tables read by the step kernel. Pure host code.
#include "ms_model.h"

#include <algorithm>
#include <cmath>
#include <map>
#include <sstream>

namespace ms {
namespace {

template <class T>
void need(bool ok, T &&what, ms_status code, ms_status *st, std::string *msg) {
  if (!ok && *st == MS_OK) {
    *st = code;
    *msg = what;
  }
}

int align16(int x) { return (x + 15) & ~15; }

}  // namespace

ms_status build_tables(const ms_model_desc *d, Tables *t, std::string *msg) {
  ms_status st = MS_OK;
  if (!d) {
    *msg = "desc is NULL";
    return MS_E_ARG;
  }
  const int n = d->n_node;
  need(n >= 1, "n_node must be >= 1", MS_E_MODEL, &st, msg);
  need(n <= kMaxNode, "n_node exceeds 128", MS_E_UNSUPPORTED, &st, msg);
  need(d->parent && d->jtype && d->jpos && d->jrot && d->axis && d->mass &&
           d->com && d->inertia && d->damping,
       "a node array is NULL", MS_E_ARG, &st, msg);
  if (st != MS_OK) return st;

  t->n_node = n;
  t->parent.assign(d->parent, d->parent + n);
  t->jtype.assign(d->jtype, d->jtype + n);
  t->qadr.resize(n);
  t->dadr.resize(n);
  int nq = 0, nv = 0;
  for (int i = 0; i < n; ++i) {
    int p = d->parent[i], jt = d->jtype[i];
    need(p >= -1 && p < i, "parent must satisfy -1 <= parent[i] < i", MS_E_MODEL, &st, msg);
    need(jt >= 0 && jt <= 2, "jtype must be 0 (hinge), 1 (slide) or 2 (free)", MS_E_MODEL, &st, msg);
    need(jt != 2 || (i == 0 && p == -1), "a free joint is allowed only at node 0 with parent -1",
         MS_E_MODEL, &st, msg);
    if (jt != 2) {
      const float *a = d->axis + 3 * i;
      float na = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
      need(std::fabs(na - 1.0f) < 1e-3f, "hinge/slide axes must be unit vectors", MS_E_MODEL, &st, msg);
    }
    need(d->mass[i] >= 0 && d->inertia[3 * i] >= 0 && d->inertia[3 * i + 1] >= 0 &&
             d->inertia[3 * i + 2] >= 0,
         "mass and inertia must be non-negative", MS_E_MODEL, &st, msg);
    t->qadr[i] = nq;
    t->dadr[i] = nv;
    nq += jt == 2 ? 7 : 1;
    nv += jt == 2 ? 6 : 1;
  }
  if (st != MS_OK) return st;
  need(nv <= kMaxDof, "more than 128 DoFs", MS_E_UNSUPPORTED, &st, msg);
  t->nq = nq;
  t->nv = nv;
  t->free_root = d->jtype[0] == 2;
  t->jpos.assign(d->jpos, d->jpos + 3 * n);
  t->jrot.assign(d->jrot, d->jrot + 9 * n);
  t->axis.assign(d->axis, d->axis + 3 * n);
  t->damping.assign(d->damping, d->damping + nv);
  t->qlo.assign(nv, -3.14159265f);
  t->qhi.assign(nv, 3.14159265f);
  if (d->qlo && d->qhi)
    for (int j = 0; j < nv; ++j) {
      if (std::isfinite(d->qlo[j])) t->qlo[j] = d->qlo[j];
      if (std::isfinite(d->qhi[j])) t->qhi[j] = d->qhi[j];
      need(t->qlo[j] <= t->qhi[j], "qlo must not exceed qhi", MS_E_MODEL, &st, msg);
    }
  for (int j = 0; j < nv; ++j)
    need(std::isfinite(d->damping[j]) && d->damping[j] >= 0, "damping must be >= 0", MS_E_MODEL, &st, msg);

  // ancestor relation and node levels
  std::vector<std::vector<char>> anc(n, std::vector<char>(n, 0));
  std::vector<int> level(n, 0);
  for (int b = 0; b < n; ++b) {
    for (int a = b; a >= 0; a = d->parent[a]) anc[a][b] = 1;
    level[b] = d->parent[b] >= 0 ? level[d->parent[b]] + 1 : 0;
  }
  int nlev = 1 + *std::max_element(level.begin(), level.end());
  t->n_level = nlev;
  t->level_start.assign(nlev + 1, 0);
  for (int l = 0; l < nlev; ++l) {
    t->level_start[l] = (int)t->level_nodes.size();
    for (int i = 0; i < n; ++i)
      if (level[i] == l) t->level_nodes.push_back(i);
  }
  t->level_start[nlev] = (int)t->level_nodes.size();

  // bodies
  for (int i = 0; i < n; ++i) {
    if (d->mass[i] > 0 || d->inertia[3 * i] > 0 || d->inertia[3 * i + 1] > 0 ||
        d->inertia[3 * i + 2] > 0) {
      t->body_node.push_back(i);
      t->body_mass.push_back(d->mass[i]);
      for (int k = 0; k < 3; ++k) {
        t->body_com.push_back(d->com[3 * i + k]);
        t->body_inertia.push_back(d->inertia[3 * i + k]);
      }
    }
  }
  t->n_body = (int)t->body_node.size();

  // contacts
  t->n_con = d->n_con;
  need(d->n_con >= 0 && d->n_con <= kMaxCon, "n_con must be in [0, 64]", MS_E_UNSUPPORTED, &st, msg);
  if (d->n_con > 0)
    need(d->con_node && d->con_pos && d->con_radius, "a contact array is NULL", MS_E_ARG, &st, msg);
  if (st != MS_OK) return st;
  for (int c = 0; c < d->n_con; ++c) {
    need(d->con_node[c] >= 0 && d->con_node[c] < n, "con_node out of range", MS_E_MODEL, &st, msg);
    need(d->con_radius[c] >= 0, "contact radius must be >= 0", MS_E_MODEL, &st, msg);
    t->con_node.push_back(d->con_node[c]);
    for (int k = 0; k < 3; ++k) t->con_pos.push_back(d->con_pos[3 * c + k]);
    t->con_radius.push_back(d->con_radius[c]);
  }
  if (st != MS_OK) return st;
  t->kc = d->contact[0];
  t->cc = d->contact[1];
  t->mu = d->contact[2];
  t->vs = d->contact[3];
  need(t->kc >= 0 && t->cc >= 0 && t->mu >= 0 && (t->vs > 0 || d->n_con == 0),
       "contact constants must be >= 0 and v_s > 0", MS_E_MODEL, &st, msg);
  for (int k = 0; k < 3; ++k) t->g[k] = d->gravity[k];

  // subtree lists of bodies and contacts per node
  t->subb_start.assign(n + 1, 0);
  t->subc_start.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) {
    t->subb_start[i] = (int)t->subb.size();
    for (int b = 0; b < t->n_body; ++b)
      if (anc[i][t->body_node[b]]) t->subb.push_back(b);
    t->subc_start[i] = (int)t->subc.size();
    for (int c = 0; c < t->n_con; ++c)
      if (anc[i][t->con_node[c]]) t->subc.push_back(c);
  }
  t->subb_start[n] = (int)t->subb.size();
  t->subc_start[n] = (int)t->subc.size();
  // composite inertias: nodes whose subtrees hold the same bodies (a body's
  // node and the massless hinge nodes above it within one joint) share one
  // slot, represented by the first such node
  t->node_ci.assign(n, -1);
  for (int i = 0; i < n; ++i) {
    for (int c = 0; c < (int)t->ci_node.size() && t->node_ci[i] < 0; ++c) {
      const int r = t->ci_node[c];
      if (std::equal(t->subb.begin() + t->subb_start[i], t->subb.begin() + t->subb_start[i + 1],
                     t->subb.begin() + t->subb_start[r], t->subb.begin() + t->subb_start[r + 1]) &&
          t->subb_start[i + 1] - t->subb_start[i] == t->subb_start[r + 1] - t->subb_start[r])
        t->node_ci[i] = c;
    }
    if (t->node_ci[i] < 0) {
      t->node_ci[i] = (int)t->ci_node.size();
      t->ci_node.push_back(i);
    }
  }
  t->n_ci = (int)t->ci_node.size();

  // DoFs and the DoF tree (each DoF's parent is the previous DoF on the path)
  std::vector<int> dof_parent(nv, -1);
  t->dof_node.assign(nv, 0);
  t->dof_kind.assign(nv, 0);
  for (int i = 0; i < n; ++i) {
    int a = t->dadr[i];
    int pd = d->parent[i] >= 0 ? t->dadr[d->parent[i]] + (d->jtype[d->parent[i]] == 2 ? 5 : 0) : -1;
    if (d->jtype[i] == 2) {
      for (int k = 0; k < 6; ++k) {
        t->dof_node[a + k] = i;
        t->dof_kind[a + k] = k < 3 ? 2 : 3;
        dof_parent[a + k] = k == 0 ? pd : a + k - 1;
      }
    } else {
      t->dof_node[a] = i;
      t->dof_kind[a] = d->jtype[i];
      dof_parent[a] = pd;
    }
  }
  t->dof_depth.assign(nv, 0);
  t->row_start.assign(nv + 1, 0);
  std::vector<std::vector<int>> dpath(nv);
  for (int j = 0; j < nv; ++j) {
    if (dof_parent[j] >= 0) dpath[j] = dpath[dof_parent[j]];
    dpath[j].push_back(j);
    t->dof_depth[j] = (int)dpath[j].size();
    t->row_start[j] = (int)t->path.size();
    for (int x : dpath[j]) t->path.push_back(x);
  }
  t->row_start[nv] = (int)t->path.size();
  t->nnz = (int)t->path.size();
  t->nnz_row.resize(t->nnz);
  for (int j = 0; j < nv; ++j)
    for (int e = t->row_start[j]; e < t->row_start[j + 1]; ++e) t->nnz_row[e] = j;
  t->max_depth = *std::max_element(t->dof_depth.begin(), t->dof_depth.end());
  need(t->max_depth <= kMaxDepth, "DoF tree deeper than 64", MS_E_UNSUPPORTED, &st, msg);
  auto dof_anc = [&](int a, int b) {  // DoF a is b or an ancestor of b
    return t->dof_depth[a] <= t->dof_depth[b] && dpath[b][t->dof_depth[a] - 1] == a;
  };
  // level schedules: height (longest path to a leaf) and depth of each DoF
  std::vector<int> height(nv, 0);
  for (int j = nv - 1; j >= 0; --j)
    if (dof_parent[j] >= 0) height[dof_parent[j]] = std::max(height[dof_parent[j]], height[j] + 1);
  t->n_hlev = 1 + *std::max_element(height.begin(), height.end());
  t->n_dlev = t->max_depth;
  t->hlev_start.assign(t->n_hlev + 1, 0);
  for (int h = 0; h < t->n_hlev; ++h) {
    t->hlev_start[h] = (int)t->hlev_dof.size();
    for (int j = 0; j < nv; ++j)
      if (height[j] == h) t->hlev_dof.push_back(j);
  }
  t->hlev_start[t->n_hlev] = (int)t->hlev_dof.size();
  // the factorisation and the L^T solve as gathers over height levels, the
  // L solve by depth over root-first rows, the kinematics level by level: one
  // compact table (int32 words) that a workgroup stages in LDS once per launch
  // The trunk: the rows of the single-row height levels at the top (h >= 1),
  // a chain from a root down whose ancestor counts are 0, 1, ... Its block is
  // finished apart: one gather over the trunk rows' other descendants (all
  // of lower height, so finished before) gives the block left after
  // eliminating every non-trunk row, and the trunk rows are then eliminated
  // bottom-up by rank-1 updates of the rows above them.
  int h0 = t->n_hlev;
  while (h0 - 1 >= 1 && t->hlev_start[h0] - t->hlev_start[h0 - 1] == 1) --h0;
  t->n_trunk = t->n_hlev - h0;
  for (int h = h0; h < t->n_hlev; ++h)
    if (t->dof_depth[t->hlev_dof[t->hlev_start[h]]] - 1 != t->n_hlev - 1 - h) t->n_trunk = 0;
  if (t->n_trunk < 2) t->n_trunk = 0;
  if (!t->n_trunk) h0 = t->n_hlev;
  t->n_hgat = t->n_trunk ? h0 + 1 : t->n_hlev;
  std::vector<char> trunk(nv, 0);
  for (int h = h0; h < t->n_hlev; ++h) trunk[t->hlev_dof[t->hlev_start[h]]] = 1;
  // proper descendants of each DoF (of a trunk row: its non-trunk ones)
  std::vector<int32_t> desc_start(nv + 1, 0), desc;
  for (int k = 0; k < nv; ++k) {
    desc_start[k] = (int)desc.size();
    for (int i = 0; i < nv; ++i)
      if (i != k && dof_anc(k, i) && !(trunk[k] && trunk[i]))
        desc.push_back(t->row_start[i] | (i << 16));
  }
  desc_start[nv] = (int)desc.size();
  need(t->nnz < 65536 && (int)desc.size() < 65536, "mass matrix too large", MS_E_UNSUPPORTED, &st,
       msg);
  {
    std::vector<int32_t> &b = t->lt;
    auto section = [&](int *off, const std::vector<int32_t> &v) {
      *off = (int)b.size();
      b.insert(b.end(), v.begin(), v.end());
    };
    // gather levels: the height levels below the trunk, then one level with
    // every trunk row's entries
    std::vector<int32_t> hent, hent_start(t->n_hgat + 1, 0), hdof, drange(nv), rs(nv + 1);
    for (int h = 0; h < t->n_hlev; ++h) {
      if (h < t->n_hgat) hent_start[h] = (int)hent.size();
      for (int e = t->hlev_start[h]; e < t->hlev_start[h + 1]; ++e) {
        const int k = t->hlev_dof[e], ck = t->dof_depth[k] - 1;
        for (int x = 0; x <= ck; ++x) hent.push_back(k | (ck << 8) | (x << 16));
        hent.push_back(k | (ck << 8) | (255 << 16));  // the right-hand side column
        hdof.push_back(k | (ck << 8));
      }
    }
    hent_start[t->n_hgat] = (int)hent.size();
    // trunk rows by ancestor count (id | row start << 8) and the entries of
    // the rows above the lowest one, row by row, columns root first, then
    // the right-hand side: H index (rhs: row id) | row depth << 16 | column
    // depth << 23 | rhs << 30, so the pairs above trunk row d are a prefix
    std::vector<int32_t> trow(t->n_trunk), tpair;
    for (int dd = 0; dd < t->n_trunk; ++dd) {
      const int k = t->hlev_dof[t->hlev_start[t->n_hlev - 1 - dd]];
      trow[dd] = k | (t->row_start[k] << 8);
    }
    for (int da = 0; da + 1 < t->n_trunk; ++da) {
      const int a = trow[da] & 0xFF;
      for (int db = 0; db <= da; ++db) tpair.push_back((t->row_start[a] + db) | (da << 16) | (db << 23));
      tpair.push_back(a | (da << 16) | (1 << 30));
    }
    for (int k = 0; k < nv; ++k) drange[k] = desc_start[k] | (desc_start[k + 1] << 16);
    for (int k = 0; k <= nv; ++k) rs[k] = t->row_start[k];
    std::vector<int32_t> path8((t->nnz + 3) / 4, 0);
    for (int e = 0; e < t->nnz; ++e) path8[e / 4] |= (t->path[e] & 0xFF) << (8 * (e % 4));
    // tree schedule and subtree lists of the kinematics and dynamics
    // per node in level order: type | (parent + 1) << 2 | first DoF << 10 |
    // node << 18 (one table read per node and level)
    std::vector<int32_t> tnode(n);
    for (size_t k = 0; k < t->level_nodes.size(); ++k) {
      const int i = t->level_nodes[k];
      tnode[k] = t->jtype[i] | ((t->parent[i] + 1) << 2) | (t->dadr[i] << 10) | (i << 18);
    }
    auto bytes = [](const std::vector<int32_t> &v) {
      std::vector<int32_t> w((v.size() + 3) / 4, 0);
      for (size_t e = 0; e < v.size(); ++e) w[e / 4] |= (v[e] & 0xFF) << (8 * (e % 4));
      return w;
    };
    std::vector<int32_t> dof_ci(nv);
    for (int j = 0; j < nv; ++j) dof_ci[j] = t->node_ci[t->dof_node[j]];
    // sections in the order: kinematics and dynamics only, then the mass
    // pattern (path) and row starts both use, then the factorisation only;
    // so the kinematics/dynamics kernel stages words [0, lt_front_end) and
    // the factorisation kernel words [lt_back_begin, end), 16-byte aligned
    auto align4 = [&]() { b.resize((b.size() + 3) / 4 * 4, 0); };
    section(&t->lt_tlev, t->level_start);
    section(&t->lt_tnode, tnode);
    section(&t->lt_subb_start, t->subb_start);
    section(&t->lt_subc_start, t->subc_start);
    section(&t->lt_subb, bytes(t->subb));
    section(&t->lt_subc, bytes(t->subc));
    section(&t->lt_nnzrow, bytes(t->nnz_row));
    section(&t->lt_cinode, bytes(t->ci_node));
    section(&t->lt_dofci, bytes(dof_ci));
    align4();
    t->lt_back_begin = (int)b.size();
    section(&t->lt_path, path8);
    t->lt_front_end = (int)b.size();
    section(&t->lt_rs, rs);
    section(&t->lt_hent_start, hent_start);
    section(&t->lt_hlev_start, t->hlev_start);
    section(&t->lt_hent, hent);
    section(&t->lt_hdof, hdof);
    section(&t->lt_desc, desc);
    section(&t->lt_drange, drange);
    section(&t->lt_trow, trow);
    section(&t->lt_tpair, tpair);
    align4();
    t->lt_front_end = (t->lt_front_end + 3) / 4 * 4;
  }

  // muscles
  const int nm = d->n_mus;
  t->n_mus = nm;
  need(nm >= 0 && nm <= kMaxMus, "n_mus must be in [0, 1024]", MS_E_UNSUPPORTED, &st, msg);
  if (nm > 0)
    need(d->f0 && d->l_opt && d->l_slack && d->v_max && d->tau_act && d->tau_deact &&
             d->via_start && d->via_node && d->via_pos,
         "a muscle array is NULL", MS_E_ARG, &st, msg);
  if (st != MS_OK) return st;
  t->mpl = (nm + kWave - 1) / kWave;
  t->via_node.assign((size_t)kMaxVia * nm, -1);
  t->via_pos.assign((size_t)kMaxVia * 3 * nm, 0.0f);
  t->mus_span.assign((size_t)3 * nm, -1);
  t->mus_srec.assign((size_t)3 * nm, -1);
  t->mus_mask.assign(nm, 0u);
  t->mus_nvia.assign(nm, 0);
  std::vector<std::vector<int>> proj(nv);
  std::map<int, std::vector<int>> dent;  // H index -> items
  int via_max = 0;
  // internal muscle order: by via-point count (descending), so the 64
  // muscles a wavefront handles together mostly share their loop bounds
  t->mus_ext.resize(nm);
  for (int m = 0; m < nm; ++m) t->mus_ext[m] = m;
  std::stable_sort(t->mus_ext.begin(), t->mus_ext.end(), [&](int a, int b) {
    return d->via_start[a + 1] - d->via_start[a] > d->via_start[b + 1] - d->via_start[b];
  });
  t->mus_int.assign(nm, 0);
  for (int m = 0; m < nm; ++m) t->mus_int[t->mus_ext[m]] = m;
  for (int m = 0; m < nm; ++m) {
    const int ex = t->mus_ext[m];
    int s0 = d->via_start[ex], s1 = d->via_start[ex + 1], P = s1 - s0;
    need(s0 >= 0 && P >= 2, "each muscle needs >= 2 via-points", MS_E_MODEL, &st, msg);
    need(P <= kMaxVia, "more than 8 via-points in a muscle", MS_E_UNSUPPORTED, &st, msg);
    need(d->f0[ex] >= 0 && d->l_opt[ex] > 0 && d->v_max[ex] > 0 && d->tau_act[ex] > 0 &&
             d->tau_deact[ex] > 0 && std::isfinite(d->l_slack[ex]),
         "Hill parameters must be positive", MS_E_MODEL, &st, msg);
    if (st != MS_OK) return st;
    via_max = std::max(via_max, P);
    t->mus_f0.push_back(d->f0[ex]);
    t->mus_ilopt.push_back(1.0f / d->l_opt[ex]);
    t->mus_lslack.push_back(d->l_slack[ex]);
    t->mus_ivl.push_back(1.0f / (d->v_max[ex] * d->l_opt[ex]));
    t->mus_tact.push_back(d->tau_act[ex]);
    t->mus_tdeact.push_back(d->tau_deact[ex]);
    t->mus_nvia[m] = P;
    std::vector<int> nodes(P);
    for (int k = 0; k < P; ++k) {
      int b = d->via_node[s0 + k];
      need(b >= -1 && b < n, "via_node out of range", MS_E_MODEL, &st, msg);
      nodes[k] = b;
      t->via_node[(size_t)k * nm + m] = b;
      for (int c = 0; c < 3; ++c) t->via_pos[((size_t)k * 3 + c) * nm + m] = d->via_pos[3 * (s0 + k) + c];
    }
    if (st != MS_OK) return st;
    // DoF j changes the length iff it moves exactly one end of a segment
    std::vector<int> span;
    std::vector<uint32_t> masks;
    for (int j = 0; j < nv; ++j) {
      int nj = t->dof_node[j];
      uint32_t mk = 0;
      for (int k = 0; k < P; ++k)
        if (nodes[k] >= 0 && anc[nj][nodes[k]]) mk |= 1u << k;
      bool in = false;
      for (int k = 0; k + 1 < P; ++k)
        if (((mk >> k) & 1u) != ((mk >> (k + 1)) & 1u)) in = true;
      if (in) {
        span.push_back(j);
        masks.push_back(mk);
      }
    }
    if ((int)span.size() > 3) {
      std::ostringstream os;
      os << "muscle " << ex << " spans " << span.size() << " DoFs (at most 3 supported)";
      need(false, os.str(), MS_E_UNSUPPORTED, &st, msg);
      return st;
    }
    for (size_t a = 0; a < span.size(); ++a)
      for (size_t b = 0; b < span.size(); ++b)
        need(dof_anc(span[a], span[b]) || dof_anc(span[b], span[a]),
             "a muscle's DoFs must lie on one root-to-leaf chain", MS_E_UNSUPPORTED, &st, msg);
    if (st != MS_OK) return st;
    for (size_t s = 0; s < span.size(); ++s) {
      t->mus_span[s * nm + m] = span[s];
      t->mus_srec[s * nm + m] = span[s] | ((t->dof_kind[span[s]] == 0 ? 1 : 0) << 8) |
                                (t->dof_node[span[s]] << 16);
      t->mus_mask[m] |= masks[s] << (8 * s);
      proj[span[s]].push_back(m * 3 + (int)s);
    }
    for (size_t s = 0; s < span.size(); ++s)
      for (size_t u = 0; u <= s; ++u) {
        int js = span[s], ju = span[u];
        int row = t->dof_depth[js] >= t->dof_depth[ju] ? js : ju;
        int col = row == js ? ju : js;
        int h = t->row_start[row] + t->dof_depth[col] - 1;
        dent[h].push_back(m * 16 + (int)s * 4 + (int)u);
      }
  }
  t->n_via_max = via_max;
  t->grp_nvia.assign(t->mpl, 0);
  for (int m = 0; m < nm; ++m) t->grp_nvia[m / kWave] = std::max(t->grp_nvia[m / kWave], t->mus_nvia[m]);
  // DoFs with the most items first (a wavefront sums 64 DoFs at a time)
  t->proj_dof.resize(nv);
  for (int j = 0; j < nv; ++j) t->proj_dof[j] = j;
  std::stable_sort(t->proj_dof.begin(), t->proj_dof.end(),
                   [&](int a, int b) { return proj[a].size() > proj[b].size(); });
  t->proj_start.assign(nv + 1, 0);
  for (int x = 0; x < nv; ++x) {
    t->proj_start[x] = (int)t->proj_item.size();
    for (int it : proj[t->proj_dof[x]]) t->proj_item.push_back(it);
  }
  t->proj_start[nv] = (int)t->proj_item.size();
  // entries with the most items first: a wavefront sums 64 entries at a
  // time, each pass as long as its longest list
  std::vector<std::pair<int, std::vector<int>>> dlist(dent.begin(), dent.end());
  std::stable_sort(dlist.begin(), dlist.end(), [](const auto &x, const auto &y) {
    return x.second.size() > y.second.size();
  });
  for (auto &kv : dlist) {
    t->dent_h.push_back(kv.first);
    t->dent_start.push_back((int)t->dent_item.size());
    for (int x : kv.second) t->dent_item.push_back(x);
  }
  t->dent_start.push_back((int)t->dent_item.size());
  t->n_dent = (int)t->dent_h.size();
  // joint coupling (equality constraints by a penalty)
  if (d->n_eq > 0 && st == MS_OK) {
    const int ne = d->n_eq;
    need(ne <= kMaxEq, "n_eq exceeds 64", MS_E_UNSUPPORTED, &st, msg);
    need(ne <= nv - (t->free_root ? 6 : 0), "more constraints than hinge/slide DoFs", MS_E_MODEL,
         &st, msg);
    need(d->eq_start && d->eq_dof && d->eq_coef && d->eq_off, "coupling arrays are NULL",
         MS_E_MODEL, &st, msg);
    need(d->eq_k >= 0.f && d->eq_d >= 0.f && std::isfinite(d->eq_k) && std::isfinite(d->eq_d),
         "eq_k and eq_d must be finite and >= 0", MS_E_MODEL, &st, msg);
    if (st != MS_OK) return st;
    need(d->eq_start[0] == 0, "eq_start[0] must be 0", MS_E_MODEL, &st, msg);
    const int root_dofs = t->free_root ? 6 : 0;
    std::map<int, std::vector<std::pair<int, float>>> by_dof;  // DoF -> (constraint, coef)
    std::map<int, float> hw;                                     // entry -> weight
    for (int c = 0; c < ne && st == MS_OK; ++c) {
      const int a = d->eq_start[c], b = d->eq_start[c + 1];
      need(b > a && b - a <= kMaxEqTerms, "each constraint needs 1 to 8 terms", MS_E_MODEL, &st, msg);
      if (st != MS_OK) break;
      for (int x = a; x < b; ++x) {
        const int j = d->eq_dof[x];
        need(j >= root_dofs && j < nv, "eq_dof must be a hinge/slide DoF", MS_E_MODEL, &st, msg);
        need(std::isfinite(d->eq_coef[x]), "eq_coef must be finite", MS_E_MODEL, &st, msg);
        if (st != MS_OK) break;
        for (int y = a; y < x; ++y)
          need(d->eq_dof[y] != j, "a DoF appears twice in one constraint", MS_E_MODEL, &st, msg);
      }
      if (st != MS_OK) break;
      need(std::isfinite(d->eq_off[c]), "eq_off must be finite", MS_E_MODEL, &st, msg);
      for (int x = a; x < b && st == MS_OK; ++x) {
        const int jx = d->eq_dof[x];
        by_dof[jx].push_back({c, d->eq_coef[x]});
        for (int y = a; y <= x; ++y) {
          const int jy = d->eq_dof[y];
          need(dof_anc(jx, jy) || dof_anc(jy, jx),
               "the DoFs of one constraint must lie on one root-to-leaf path", MS_E_MODEL, &st,
               msg);
          if (st != MS_OK) break;
          const int row = t->dof_depth[jx] >= t->dof_depth[jy] ? jx : jy;
          const int col = row == jx ? jy : jx;
          hw[t->row_start[row] + t->dof_depth[col] - 1] += d->eq_coef[x] * d->eq_coef[y];
        }
      }
    }
    if (st != MS_OK) return st;
    t->n_eq = ne;
    t->eq_k = d->eq_k;
    t->eq_d = d->eq_d;
    t->eq_start.assign(d->eq_start, d->eq_start + ne + 1);
    for (int x = 0; x < d->eq_start[ne]; ++x) {
      const int j = d->eq_dof[x];
      t->eq_dof.push_back(j);
      t->eq_qi.push_back(t->qadr[t->dof_node[j]]);
      t->eq_coef.push_back(d->eq_coef[x]);
    }
    t->eq_off.assign(d->eq_off, d->eq_off + ne);
    t->eqd_start.push_back(0);
    for (auto &kv : by_dof) {
      t->eqd_dof.push_back(kv.first);
      for (auto &cc : kv.second) {
        t->eqd_c.push_back(cc.first);
        t->eqd_coef.push_back(cc.second);
      }
      t->eqd_start.push_back((int)t->eqd_c.size());
    }
    t->n_eqd = (int)t->eqd_dof.size();
    for (auto &kv : hw) {
      t->eqh_h.push_back(kv.first);
      t->eqh_w.push_back(kv.second);
    }
    t->n_eqh = (int)t->eqh_h.size();
  }
  if (t->free_root) {
    // a world-fixed via-point on a floating model would span the root
    for (int m = 0; m < nm; ++m)
      for (int k = 0; k < t->mus_nvia[m]; ++k)
        need(t->via_node[(size_t)k * nm + m] >= 0, "world via-points need a fixed base",
             MS_E_UNSUPPORTED, &st, msg);
  }
  if (st != MS_OK) return st;

  // LDS layout of one environment
  int off = 0;
  auto take = [&](int bytes) {
    int o = off;
    off = align16(off + bytes);
    return o;
  };
  t->off_flag = take(16);
  t->off_q = take(4 * nq);
  t->off_qd = take(4 * nv);
  t->off_R = take(4 * 12 * n);  // per node R (9) then P (3)
  t->off_P = t->off_R + 36;
  t->off_S = take(4 * 6 * nv);
  t->off_con = take(4 * 16 * std::max(t->n_con, 1));
  t->off_rhs = take(8 * nv);
  t->off_x = take(8 * nv);
  t->off_H = take(8 * t->nnz);
  const int u_rnea = 4 * 6 * (2 * n + t->n_body + n);          // V, A, f_b, F_n
  const int u_crba = 8 * 10 * (t->n_ci + t->n_body) + 8 * 6 * nv;  // bodies, composites, F_j
  const int u_mus = 4 * 5 * nm;                                // r[3], F, c per muscle
  int u = std::max(u_rnea, std::max(u_crba, u_mus));
  t->off_scr = take(u);
  t->off_V = t->off_scr;
  t->off_A = t->off_V + 4 * 6 * n;
  t->off_F = t->off_A + 4 * 6 * n;
  t->lds_bytes = off;

  // Geometry-only launches: no contacts, dynamics or mass matrix, so only
  // the state, the frames, the subspaces and the kinematics' V and A rows.
  off = 0;
  t->geo_q = take(4 * nq);
  t->geo_qd = take(4 * nv);
  t->geo_R = take(4 * 12 * n);
  t->geo_S = take(4 * 6 * nv);
  t->geo_V = take(4 * 6 * 2 * n);
  t->geo_bytes = off;
  t->geo_lt_words = std::min((int)t->lt.size(), (t->lt_subb_start + 3) / 4 * 4);

  // The split schedule's three kernels (one env per wavefront for the
  // kinematics/dynamics and the factorisation kernels, one env per
  // 256-thread workgroup for the muscle kernel), each with its own layout.
  SplitLayout &L = t->split;
  off = 0;
  L.f_R = take(4 * 12 * n);
  L.f_S = take(4 * 6 * nv);
  L.f_con = take(4 * 16 * std::max(t->n_con, 1));
  L.f_scr = take(std::max(u_rnea, u_crba));
  L.f_bytes = off;
  off = 0;
  L.b_q = take(4 * nq);
  L.b_qd = take(4 * nv);
  L.b_x = take(8 * nv);   // the right-hand side, solved in place
  L.b_invd = take(8 * nv);
  L.b_H = take(8 * t->nnz);
  L.b_bytes = off;
  off = 0;
  L.m_R = take(4 * 12 * n);
  L.m_S = take(4 * 6 * nv);
  L.m_q = take(4 * nq);
  L.m_qd = take(4 * nv);
  L.m_scr = take(std::max(u_mus, 4));
  L.m_bytes = off;
  // per-env workspace in device memory (bytes, 256-aligned arrays)
  auto wsz = [](size_t b) { return (b + 255) / 256 * 256; };
  L.ws_frames = 4 * 12 * n;
  L.ws_S = 4 * 6 * nv;
  L.ws_H = 8 * (size_t)t->nnz;
  L.ws_rhs = 8 * nv;
  L.ws_tau = 4 * nv;
  L.ws_dsum = 8 * std::max(t->n_dent, 1);
  L.ws_act = 4 * std::max(nm, 1);
  L.ws_env_bytes = wsz(L.ws_frames) + wsz(L.ws_S) + wsz(L.ws_H) + wsz(L.ws_rhs) +
                   wsz(L.ws_tau) + wsz(L.ws_dsum) + wsz(L.ws_act) + 2 * 4;
  return MS_OK;
}

}  // namespace ms
