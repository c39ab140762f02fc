// ms_model.h -- host-side compilation of a model description into the flat
// tables the step kernel reads (internal to libms).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include <hip/hip_runtime.h>

#include "../../include/ms.h"

namespace ms {

constexpr int kMaxNode = 128;
constexpr int kMaxDof = 128;
constexpr int kMaxMus = 1024;
constexpr int kMaxVia = 8;
constexpr int kMaxCon = 64;
constexpr int kMaxDepth = 64;
constexpr int kMaxEq = 64;       // joint-coupling constraints
constexpr int kMaxEqTerms = 8;   // terms per constraint
constexpr int kWave = 64;

// LDS layouts (byte offsets into one env's block) of the split schedule's
// kernels and the sizes of the per-env device workspace between them.
struct SplitLayout {
  // kinematics and dynamics kernel
  int f_R = 0, f_S = 0, f_con = 0, f_scr = 0, f_bytes = 0;
  // factorisation kernel
  int b_q = 0, b_qd = 0, b_x = 0, b_invd = 0, b_H = 0, b_bytes = 0;
  // muscle kernel
  int m_R = 0, m_S = 0, m_q = 0, m_qd = 0, m_scr = 0, m_bytes = 0;
  // per-env bytes of each workspace array: node frames, motion subspaces,
  // mass matrix (FP64), right-hand side (FP64), muscle torques, muscle
  // damping sums (FP64), new activations
  size_t ws_frames = 0, ws_S = 0, ws_H = 0, ws_rhs = 0, ws_tau = 0, ws_dsum = 0, ws_act = 0;
  size_t ws_env_bytes = 0;
};

// Offsets (in elements of the named type) of every table inside one device
// buffer; the kernel receives base pointer + this struct.
struct Tables {
  // sizes
  int n_node = 0, nq = 0, nv = 0, n_mus = 0, n_con = 0, n_body = 0;
  int nnz = 0, max_depth = 0, n_level = 0, free_root = 0, mpl = 0;
  int n_dent = 0, n_via_max = 0;
  float kc = 0, cc = 0, mu = 0, vs = 0, g[3] = {0, 0, 0};
  // per node
  std::vector<int32_t> parent, jtype, qadr, dadr, level_start, level_nodes;
  std::vector<float> jpos, jrot, axis;          // [n][3], [n][9], [n][3]
  // bodies (nodes with mass or inertia)
  std::vector<int32_t> body_node;
  std::vector<float> body_mass, body_com, body_inertia;  // [b], [b][3], [b][3]
  // per node: bodies and contacts in its subtree (CSR)
  std::vector<int32_t> subb_start, subb, subc_start, subc;
  // composite-inertia slots: node -> slot, slot -> its representative node
  std::vector<int32_t> node_ci, ci_node;
  int n_ci = 0;
  // contacts
  std::vector<int32_t> con_node;
  std::vector<float> con_pos, con_radius;
  // DoF
  std::vector<int32_t> dof_node, dof_kind;  // kind: 0 hinge, 1 slide, 2 root lin, 3 root ang
  std::vector<float> damping;
  std::vector<float> qlo, qhi;              // [nv] pose-domain limits (+-pi if absent)
  // muscles (SoA, internal order)
  std::vector<float> mus_f0, mus_ilopt, mus_lslack, mus_ivl, mus_tact, mus_tdeact;
  std::vector<int32_t> mus_ext;           // internal slot -> caller's muscle index
  std::vector<int32_t> mus_int;           // caller's muscle index -> internal slot
  std::vector<int32_t> grp_nvia;          // max via count of each 64-muscle group
  std::vector<int32_t> mus_nvia;          // via count
  std::vector<int32_t> via_node;          // [kMaxVia][n_mus] SoA, padded
  std::vector<float> via_pos;             // [kMaxVia][3][n_mus] SoA, padded
  std::vector<int32_t> mus_span;          // [3][n_mus], -1 pad
  std::vector<int32_t> mus_srec;          // [3][n_mus]: DoF | hinge << 8 | node << 16, -1 pad
  std::vector<uint32_t> mus_mask;         // [n_mus] 3 x 8-bit via masks
  // reductions over muscle products
  std::vector<int32_t> proj_dof;          // [nv] DoF order of the lists
  std::vector<int32_t> proj_start;        // [nv+1]
  std::vector<int32_t> proj_item;         // muscle*3 + slot
  std::vector<int32_t> dent_h, dent_start, dent_item;  // item: muscle*16 + s*4 + t
  // joint coupling: per constraint its terms (q index, DoF, coefficient) and
  // offset; per coupled DoF its terms (constraint, coefficient); the matrix
  // entries of J^T J (entry index, weight summed over constraints)
  int n_eq = 0, n_eqd = 0, n_eqh = 0;
  float eq_k = 0.f, eq_d = 0.f;
  std::vector<int32_t> eq_start, eq_qi, eq_dof, eqd_start, eqd_dof, eqd_c, eqh_h;
  std::vector<float> eq_coef, eq_off, eqd_coef, eqh_w;
  // tree-sparse mass matrix (row j holds its ancestors by depth, diag last)
  std::vector<int32_t> row_start, dof_depth, path;     // path[nnz] = DoF id
  std::vector<int32_t> nnz_row;                        // row of each entry
  // level schedule of the factorisation: DoFs grouped by height (leaves
  // first), of which the first n_hgat - 1 are gathered level by level and the
  // n_trunk single-row levels at the top form the trunk; the L solve runs
  // over the n_dlev depths (root first)
  int n_hlev = 0, n_dlev = 0, n_hgat = 0, n_trunk = 0;
  std::vector<int32_t> hlev_start, hlev_dof;
  // The factorisation and solves as gathers over tree levels, one int32
  // table (lt) staged in LDS per workgroup; lt_* are word offsets of its
  // sections: hent_start / hlev_start (level starts), hent
  // (per height level, its rows' entries: row | depth(row) << 8 |
  // depth(column) << 16, depth 255 standing for the right-hand side), hdof (per height level, its DoFs: id | depth << 8),
  // desc (per DoF its proper descendants: row start | id << 16), drange (per
  // DoF its desc range: begin | end << 16), rs (row starts), path (path[] as
  // bytes), trow and tpair (the trunk's rows and the entries its rank-1
  // updates touch).
  // The same table holds the tree schedule (tlev level starts, tnode per node
  // in level order: type | (parent + 1) << 2 | first DoF << 10 | node << 18)
  // and the subtree lists (subb_start/subc_start, subb/subc and nnzrow as
  // bytes).
  std::vector<int32_t> lt;
  int lt_hent_start = 0, lt_hlev_start = 0, lt_hent = 0, lt_hdof = 0,
      lt_desc = 0, lt_drange = 0, lt_rs = 0, lt_trow = 0, lt_tpair = 0, lt_path = 0, lt_tlev = 0, lt_tnode = 0,
      lt_subb_start = 0, lt_subc_start = 0, lt_subb = 0, lt_subc = 0, lt_nnzrow = 0,
      lt_cinode = 0, lt_dofci = 0, lt_front_end = 0, lt_back_begin = 0;
  // LDS layout (byte offsets into the per-env LDS block)
  int off_q = 0, off_qd = 0, off_R = 0, off_P = 0, off_S = 0, off_V = 0,
      off_A = 0, off_F = 0, off_con = 0, off_rhs = 0, off_H = 0, off_x = 0,
      off_scr = 0, off_flag = 0, lds_bytes = 0;
  SplitLayout split;
  // geometry-only launches (exact lengths and moment arms of given poses):
  // state, node frames, motion subspaces and the kinematics' velocity and
  // acceleration rows, per env; the tree schedule from the table's first
  // geo_lt_words words
  int geo_q = 0, geo_qd = 0, geo_R = 0, geo_S = 0, geo_V = 0, geo_bytes = 0, geo_lt_words = 0;
  int n_levels_dof = 0;
};

// Validate desc and build every table. Returns MS_OK or an error with msg.
ms_status build_tables(const ms_model_desc *d, Tables *t, std::string *msg);

}  // namespace ms

// q index and pose-domain limits of every hinge/slide coordinate of a model
// (the geometry surrogate's inputs), in node order.
void ms_surrogate_tables(const ms_model *m, std::vector<int> *q_index, std::vector<float> *lo,
                         std::vector<float> *hi);

// De-standardised predictions of the surrogate for n poses into its own
// workspace; *Y receives the device pointer ([n][4 n_mus]), valid until the
// next call on the surrogate.
ms_status ms_surrogate_predict(ms_surrogate *s, int n, const float *q, const float **Y,
                               hipStream_t st);
