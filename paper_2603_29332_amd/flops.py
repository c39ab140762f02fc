"""Algorithmic operation count of one exact step of one environment.

Counts the arithmetic the method needs per env-step for a given model, stage
by stage, with one flop per add, multiply, divide, square root or
transcendental and two per fused multiply-add. It counts the algorithm's
operations, not the instructions a particular kernel issues (no index
arithmetic, no loads, no predicated lanes). Used to place the measured step
against the ALU roofline.
"""
from __future__ import annotations

import numpy as np


def _subtree_sizes(parent, is_member):
    """For each node, how many members (bodies/contacts) lie in its subtree."""
    n = len(parent)
    cnt = np.zeros(n, int)
    for b in range(n):
        if not is_member[b]:
            continue
        a = b
        while a >= 0:
            cnt[a] += is_member[b]
            a = parent[a]
    return cnt


def step_flops(model: dict, spans: np.ndarray, nnz: int, contacts_active: float = None):
    """FP32 and FP64 flops of one env-step; returns (fp32, fp64, detail)."""
    m = model
    n, nv, nm = m["n_node"], m["nv"], m["n_mus"]
    parent = np.asarray(m["parent"])
    jt = np.asarray(m["jtype"])
    body = (np.asarray(m["mass"]) > 0) | (np.asarray(m["inertia"]).sum(1) > 0)
    nb = int(body.sum())
    ncon = m["n_con"]
    if contacts_active is None:
        contacts_active = ncon / 2.0
    nvia = np.diff(np.asarray(m["via_start"]))
    nspan = (spans >= 0).sum(1)
    d = {}
    d["activation"] = 9 * nm
    # FK, motion subspace, V and A per hinge/slide node
    nh = int((jt != 2).sum())
    d["kinematics"] = nh * (2 + 20 + 45 + 45 + 18 + 15 + 9 + 6 + 12 + 18) + 60
    d["contact"] = ncon * 25 + int(contacts_active) * 70
    subb = _subtree_sizes(parent, body.astype(int))
    cmem = np.zeros(n, int)
    for c in m["con_node"]:
        cmem[c] += 1
    subc = _subtree_sizes(parent, cmem)
    d["bias_rnea"] = nb * 150 + 6 * int(subb.sum() + subc.sum()) + nv * 13
    # muscles: via points, segments, moment arms, Hill
    nsv = sum(int(nspan[i]) * int(nvia[i]) for i in range(nm))
    d["geometry"] = int(nvia.sum()) * 18 + int((nvia - 1).sum()) * 17 + nsv * 15 + int(nspan.sum()) * 7
    d["hill"] = nm * 40
    d["projection"] = 2 * int(nspan.sum())
    dent_items = int(sum(k * (k + 1) // 2 for k in nspan))
    d["mass_fp64"] = nb * 60 + 10 * int(subb.sum()) + nv * 36 + 12 * nnz + 4 * dent_items \
        + int(contacts_active) * 25 * 10
    # LTDL: each eliminated DoF updates its (ancestor, ancestor) pairs;
    # DoF depth (ancestors + itself) from the node tree
    ddepth = {}
    dd = []
    for i in range(n):
        base = 0 if parent[i] < 0 else ddepth[parent[i]]
        cnt = 6 if jt[i] == 2 else 1
        for c in range(cnt):
            dd.append(base + c + 1)
        ddepth[i] = base + cnt
    dd = np.array(dd)
    pairs = int(((dd - 1) * dd // 2).sum())
    d["solve_fp64"] = 3 * pairs + nv + nnz + 4 * nnz + nv
    d["integrate"] = 6 * nv + 40
    fp64 = d["mass_fp64"] + d["solve_fp64"]
    fp32 = sum(v for kk, v in d.items() if kk not in ("mass_fp64", "solve_fp64"))
    return fp32, fp64, d


def split_kernel_flops(detail: dict, model: dict, spans: np.ndarray) -> dict:
    """The step's flops by kernel of the split schedule: kinematics/dynamics
    (forward kinematics, contacts, Newton-Euler bias, composite-rigid-body
    mass matrix), muscles (activation, geometry, Hill force, J_m^T F and the
    muscles' FP64 damping sums) and factorisation (LTDL factorisation and
    solves, semi-implicit Euler)."""
    nspan = (spans >= 0).sum(1)
    dent = 4 * int(sum(int(k) * (int(k) + 1) // 2 for k in nspan))
    return {
        "k_front": {"fp32": detail["kinematics"] + detail["contact"] + detail["bias_rnea"],
                    "fp64": detail["mass_fp64"] - dent},
        "k_muscle": {"fp32": detail["activation"] + detail["geometry"] + detail["hill"]
                     + detail["projection"], "fp64": dent},
        "k_back": {"fp32": detail["integrate"], "fp64": detail["solve_fp64"]},
    }
