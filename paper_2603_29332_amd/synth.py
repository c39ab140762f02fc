"""Seeded synthetic inputs: musculoskeletal models, initial states and excitations.

This module is shared by the HIP path's tests/bench and by the CPU oracle's
tests. It holds none of the stepping arithmetic (no kinematics at a general
pose, no dynamics, no muscle force law). It only *builds* inputs:

* model descriptions (kinematic tree of hinge/slide/free nodes, segment
  masses and inertias, via-point muscles with Hill parameters, contact
  spheres), laid out at the neutral pose where every node frame is aligned
  with the world frame, so a via-point's local position is its neutral world
  position minus its node's neutral origin;
* seeded initial states;
* excitation sequences u in [0, 1] (the paper's action, Methods
  "Musculoskeletal dynamics" / action definition) from a counter-based
  SplitMix64 hash (Steele, Lea & Flood 2014), either i.i.d. uniform per step
  or a first-order autoregressive smooth noise, computed in float32 with a
  fixed operation order so that an independent implementation of the same
  published definitions reproduces the bits.

Model array conventions (all float32 / int32, C-contiguous):

  parent[n]      parent node, -1 = world; parent < child
  jtype[n]       0 hinge, 1 slide, 2 free (root only)
  jpos[n,3]      joint-frame origin in the parent node frame
  jrot[n,9]      joint-frame orientation in the parent node frame (row-major)
  axis[n,3]      hinge/slide axis in the joint frame
  mass[n], com[n,3], inertia[n,3]   segment carried by the node (principal
                 moments about the COM, node axes); 0 for massless frames
  damping[nv], qlo[nv], qhi[nv]     per-DoF damping and pose-domain limits
  f0, l_opt, l_slack, v_max, tau_act, tau_deact  [n_mus]
  via_start[n_mus+1], via_node[n_via] (-1 = world), via_pos[n_via,3]
  con_node[n_con], con_pos[n_con,3], con_radius[n_con]
  contact[4] = (stiffness k, damping c, friction mu, slip velocity v_s)
  gravity[3]
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
MASK64 = (1 << 64) - 1

# ---------------------------------------------------------------------------
# counter-based uniforms (SplitMix64 finaliser, Steele, Lea & Flood 2014)
# ---------------------------------------------------------------------------
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """SplitMix64 output function applied to counter(s) x (uint64 array)."""
    with np.errstate(over="ignore"):
        z = np.asarray(x, dtype=np.uint64) + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def step_key(seed: int, env, step: int):
    """Per-(env, step) 64-bit key: SplitMix64(SplitMix64(seed ^ env) ^ step)."""
    env = np.asarray(env, dtype=np.uint64)
    return splitmix64(splitmix64(np.uint64(seed) ^ env) ^ np.uint64(step))


def _u24(z, shift: int):
    """24 bits of z starting at `shift`, scaled by 2^-24 (exact in float32)."""
    return (((z >> np.uint64(shift)) & np.uint64(0xFFFFFF)).astype(np.float64)
            * 2.0 ** -24).astype(F32)


def _envs(n_env, envs):
    return np.arange(n_env) if envs is None else np.asarray(envs)


def excitation_iid(seed: int, n_env: int, n_mus: int, step: int, envs=None):
    """u[e, m] = top 24 bits of SplitMix64(key(e, step) ^ m) * 2^-24."""
    key = step_key(seed, _envs(n_env, envs), step)[:, None]
    z = splitmix64(key ^ np.arange(n_mus, dtype=np.uint64)[None, :])
    return _u24(z, 40)


def reference_params(seed: int, n_env: int, n_ref: int, envs=None):
    """Parameters of the synthetic reference targets (stand-in for the
    retargeted reference motion a tracking policy observes): for env e,
    target k, sinusoid j, key K = SplitMix64(SplitMix64(seed ^ e) ^ (3k + j))
    and a, b, c = top 24 bits of SplitMix64(K ^ 0 / 1 / 2) * 2^-24; returns
    float32 amplitude 0.3 a, frequency 0.5 + 1.5 b (Hz) and phase 2 pi c,
    each [n_env][n_ref][3]."""
    e = _envs(n_env, envs).astype(np.uint64)
    ke = splitmix64(np.uint64(seed) ^ e)[:, None]
    idx = np.arange(3 * n_ref, dtype=np.uint64)[None, :]
    key = splitmix64(ke ^ idx)
    ua, ub, uc = (_u24(splitmix64(key ^ np.uint64(i)), 40) for i in range(3))
    shape = (len(e), n_ref, 3)
    amp = (F32(0.3) * ua).astype(F32).reshape(shape)
    freq = (F32(0.5) + F32(1.5) * ub).astype(F32).reshape(shape)
    phase = (F32(2.0 * math.pi) * uc).astype(F32).reshape(shape)
    return amp, freq, phase


def ar1_constants(dt: float, corr_time: float = 0.05, sigma: float = 0.25,
                  mean: float = 0.3):
    """float32 constants (rho, s, mean, sqrt3) of the smooth-noise process."""
    rho = math.exp(-dt / corr_time)
    s = sigma * math.sqrt(1.0 - rho * rho)
    return F32(rho), F32(s), F32(mean), F32(math.sqrt(3.0))


def excitation_ar1_step(seed: int, x, step: int, consts, envs=None):
    """One step of the smooth noise. x[e, m] (float32) is updated in place.

    Two SplitMix64 draws per (env, muscle) give four 24-bit uniforms; their
    sum (Irwin-Hall(4), mean 2, variance 1/3) is standardised to xi. Then
    x <- rho*x + s*xi and u = clamp(mean + x, 0, 1), every operation rounded
    to float32 in this order.
    """
    rho, s, mean, sqrt3 = consts
    n_env, n_mus = x.shape
    key = step_key(seed, _envs(n_env, envs), step)[:, None]
    m2 = 2 * np.arange(n_mus, dtype=np.uint64)[None, :]
    z1 = splitmix64(key ^ m2)
    z2 = splitmix64(key ^ (m2 + np.uint64(1)))
    u1, u2 = _u24(z1, 40), _u24(z1, 16)
    u3, u4 = _u24(z2, 40), _u24(z2, 16)
    t = ((u1 + u2) + u3) + u4
    xi = (t - F32(2.0)) * sqrt3
    x[...] = (rho * x) + (s * xi)
    u = np.minimum(np.maximum(mean + x, F32(0.0)), F32(1.0))
    return u.astype(F32)


def excitation_sequence(kind: str, seed: int, n_env: int, n_mus: int,
                        n_steps: int, dt: float, step0: int = 0, x0=None,
                        envs=None):
    """u[T, E, Mu] for steps step0 .. step0+T-1; returns (u, x_final).
    envs optionally names the env index of each row (default 0..E-1)."""
    if envs is not None:
        n_env = len(envs)
    out = np.empty((n_steps, n_env, n_mus), dtype=F32)
    x = np.zeros((n_env, n_mus), F32) if x0 is None else np.array(x0, F32)
    consts = ar1_constants(dt)
    for t in range(n_steps):
        if kind == "iid":
            out[t] = excitation_iid(seed, n_env, n_mus, step0 + t, envs)
        elif kind == "ar1":
            out[t] = excitation_ar1_step(seed, x, step0 + t, consts, envs)
        else:
            raise ValueError(kind)
    return out, x


# ---------------------------------------------------------------------------
# model assembly helpers
# ---------------------------------------------------------------------------
def _finish(model: dict) -> dict:
    """Cast arrays, derive nq/nv, validate topological order."""
    n = len(model["parent"])
    model["n_node"] = n
    for k in ("parent", "jtype", "via_start", "via_node", "con_node"):
        model[k] = np.ascontiguousarray(model[k], dtype=np.int32)
    for k in ("jpos", "jrot", "axis", "mass", "com", "inertia", "damping", "qlo",
              "qhi", "f0", "l_opt", "l_slack", "v_max", "tau_act", "tau_deact",
              "via_pos", "con_pos", "con_radius", "contact", "gravity"):
        model[k] = np.ascontiguousarray(model[k], dtype=F32)
    model["jpos"] = model["jpos"].reshape(n, 3)
    model["jrot"] = model["jrot"].reshape(n, 9)
    model["axis"] = model["axis"].reshape(n, 3)
    model["com"] = model["com"].reshape(n, 3)
    model["inertia"] = model["inertia"].reshape(n, 3)
    model["via_pos"] = model["via_pos"].reshape(-1, 3)
    model["con_pos"] = model["con_pos"].reshape(-1, 3)
    jt = model["jtype"]
    model["nq"] = int(sum(7 if t == 2 else 1 for t in jt))
    model["nv"] = int(sum(6 if t == 2 else 1 for t in jt))
    model["n_mus"] = int(len(model["f0"]))
    model["n_con"] = int(len(model["con_node"]))
    for i in range(n):
        assert model["parent"][i] < i
        if jt[i] == 2:
            assert i == 0 and model["parent"][i] == -1
    assert len(model["damping"]) == model["nv"]
    return model


def _hill_draw(rng):
    """F0 ~ U[200,1500] N, l_opt ~ U[0.05,0.15] m, l_s ~ U[0.1,0.3] m."""
    return (rng.uniform(200.0, 1500.0), rng.uniform(0.05, 0.15),
            rng.uniform(0.1, 0.3))


# ---------------------------------------------------------------------------
# tiny planar chain (8 hinges, 16 two-point muscles)
# ---------------------------------------------------------------------------
def chain_model(seed: int = 1, n_link: int = 8, n_mus: int = 16,
                link_len: float = 0.3, damping: float = 0.1) -> dict:
    """Fixed-base chain of hinges about y, hanging along -z at q = 0.

    Link i spans from joint i to joint i+1 (link_len along -z), COM at mid
    link, solid-cylinder inertia (radius 0.03 m). Each muscle crosses one or
    two adjacent joints with an origin on the proximal link (the ground for
    joint 0) and an insertion on the distal link, both offset laterally
    along link-local x by U[0.02, 0.05] m on one side; the insertion's axial
    place is solved so that the neutral path length is l_s + lambda0 * l_opt
    with lambda0 ~ U[0.9, 1.1].
    """
    rng = np.random.default_rng(seed)
    n = n_link
    parent = np.arange(-1, n - 1)
    jtype = np.zeros(n)
    jpos = np.zeros((n, 3))
    jpos[1:, 2] = -link_len
    jrot = np.tile(np.eye(3).ravel(), (n, 1))
    axis = np.tile([0.0, 1.0, 0.0], (n, 1))
    mass = rng.uniform(1.0, 5.0, n)
    com = np.tile([0.0, 0.0, -link_len / 2], (n, 1))
    r = 0.03
    inertia = np.stack([mass * (3 * r * r + link_len ** 2) / 12,
                        mass * (3 * r * r + link_len ** 2) / 12,
                        mass * r * r / 2], axis=1)
    f0, lo, ls, vn, vp = [], [], [], [], []
    for _ in range(n_mus):
        j = int(rng.integers(0, n))
        span = 1 if j == n - 1 else int(rng.integers(1, 3))
        sign = 1.0 if rng.uniform() < 0.5 else -1.0
        d_o, d_i = rng.uniform(0.02, 0.05, 2)
        x_o, x_i = sign * d_o, sign * d_i
        # world z ranges (q = 0) of origin link (j-1; ground above joint 0)
        # and insertion link (j+span-1)
        zo_rng = (-link_len * j, -link_len * (j - 1))
        zi_rng = (-link_len * (j + span), -link_len * (j + span - 1))
        for _attempt in range(200):
            F0, lopt, lsl = _hill_draw(rng)
            lam0 = rng.uniform(0.9, 1.1)
            L0 = lsl + lam0 * lopt
            z_o = rng.uniform(*zo_rng)
            dz2 = L0 * L0 - (x_o - x_i) ** 2
            if dz2 <= 0:
                continue
            z_i = z_o - math.sqrt(dz2)
            if zi_rng[0] <= z_i <= zi_rng[1]:
                break
        else:
            raise RuntimeError("chain muscle placement failed")
        on = j - 1
        ins = j + span - 1
        o_origin = 0.0 if on < 0 else -link_len * on
        vp.append([x_o, 0.0, z_o - o_origin] if on >= 0 else [x_o, 0.0, z_o])
        vp.append([x_i, 0.0, z_i + link_len * ins])
        vn += [on, ins]
        f0.append(F0)
        lo.append(lopt)
        ls.append(lsl)
    via_start = [0] + [2 * (k + 1) for k in range(n_mus)]
    model = dict(
        name=f"chain{n}_m{n_mus}_s{seed}", parent=parent, jtype=jtype, jpos=jpos,
        jrot=jrot, axis=axis, mass=mass, com=com, inertia=inertia,
        damping=np.full(n, damping), qlo=np.full(n, -math.pi),
        qhi=np.full(n, math.pi), f0=f0, l_opt=lo, l_slack=ls,
        v_max=np.full(n_mus, 10.0), tau_act=np.full(n_mus, 0.010),
        tau_deact=np.full(n_mus, 0.040), via_start=via_start,
        via_node=vn, via_pos=vp, con_node=np.zeros(0), con_pos=np.zeros((0, 3)),
        con_radius=np.zeros(0), contact=[1e5, 1e3, 1.0, 0.05],
        gravity=[0.0, 0.0, -9.81])
    return _finish(model)


def chain_initial_state(model: dict, n_env: int, seed: int = 7):
    """q ~ U[-0.1, 0.1] rad per hinge, qd = 0, act = 0."""
    rng = np.random.default_rng(seed)
    q = rng.uniform(-0.1, 0.1, (n_env, model["nq"])).astype(F32)
    qd = np.zeros((n_env, model["nv"]), F32)
    act = np.zeros((n_env, model["n_mus"]), F32)
    return q, qd, act


# ---------------------------------------------------------------------------
# synthetic whole-body human
# ---------------------------------------------------------------------------
X, Y, Z = (1.0, 0.0, 0.0), (0.0, 1.0, 0.0), (0.0, 0.0, 1.0)


def _seg(name, parent, center, hinges, mass, com, dims, scale=1.0, shape="cyl",
         limits=None):
    """Body spec: joint centre (world, neutral), hinges [(axis, anchor_off)],
    mass (unnormalised), COM (world), dims=(length, radius) for inertia."""
    return dict(name=name, parent=parent, center=np.array(center, float),
                hinges=hinges, mass=mass, com=np.array(com, float), dims=dims,
                scale=scale, shape=shape, limits=limits)


def _mirror(spec_fn, side):
    s = 1.0 if side == "L" else -1.0
    return spec_fn(s, side)


def _human_specs(full: bool):
    """Body table of the synthetic human (z up, facing +x, y to the left).

    full=True: 22 bodies, 74 hinges (+6 root) = 80 DoF. Three hinges at a
    joint form an intrinsic z-y'-x'' ball; hinges beyond three use axes
    offset from the joint centre (moving-axis knee, scapular complex).
    full=False: 13 bodies, 34 hinges (+6 root) = 40 DoF.
    """
    b = []
    ball = [(Z, (0, 0, 0)), (Y, (0, 0, 0)), (X, (0, 0, 0))]
    lim_ball = [(-0.8, 0.8), (-1.2, 1.2), (-1.0, 1.0)]
    pelvis_c = (0.0, 0.0, 1.00)
    b.append(_seg("pelvis", None, pelvis_c, [], 11.0, (0, 0, 1.00), (0.20, 0.14)))
    if full:
        b.append(_seg("lumbar", "pelvis", (0, 0, 1.10),
                      ball + [(Y, (0.06, 0, 0)), (X, (0, 0, 0.06)),
                              (Z, (0, 0.06, 0))], 10.0,
                      (0, 0, 1.19), (0.18, 0.13),
                      limits=lim_ball + [(-0.4, 0.4)] * 3))
        b.append(_seg("thorax", "lumbar", (0, 0, 1.28),
                      ball + [(Y, (0.06, 0, 0)), (X, (0, 0, 0.06))], 16.0,
                      (0, 0, 1.43), (0.30, 0.16),
                      limits=lim_ball + [(-0.4, 0.4)] * 2))
        b.append(_seg("head", "thorax", (0, 0, 1.56),
                      ball + [(Y, (0.05, 0, 0)), (X, (0, 0, 0.05))], 7.0,
                      (0.01, 0, 1.67), (0.20, 0.09),
                      limits=lim_ball + [(-0.4, 0.4)] * 2))
    else:
        b.append(_seg("thorax", "pelvis", (0, 0, 1.10),
                      ball + [(Y, (0.06, 0, 0)), (X, (0, 0, 0.06))], 26.0,
                      (0, 0, 1.33), (0.46, 0.15),
                      limits=lim_ball + [(-0.4, 0.4)] * 2))
        b.append(_seg("head", "thorax", (0, 0, 1.56),
                      [(Z, (0, 0, 0)), (Y, (0, 0, 0)), (X, (0, 0, 0))], 7.0,
                      (0.01, 0, 1.67), (0.20, 0.09), limits=lim_ball))
    for side in ("L", "R"):
        s = 1.0 if side == "L" else -1.0
        if full:
            b.append(_seg("clav" + side, "thorax", (0.03, 0.03 * s, 1.52),
                          [(Z, (0, 0, 0)), (X, (0, 0, 0))], 0.4,
                          (0.02, 0.09 * s, 1.53), (0.14, 0.02), scale=0.8,
                          limits=[(-0.4, 0.4)] * 2))
            b.append(_seg("scap" + side, "clav" + side, (0.0, 0.17 * s, 1.54),
                          ball, 0.8,
                          (-0.06, 0.14 * s, 1.46), (0.12, 0.05), scale=0.8,
                          limits=[(-0.4, 0.4)] * 3))
            hum_parent = "scap" + side
            hum_h = ball + [(Z, (0.05, 0, 0)), (Y, (0, 0, -0.05))]
        else:
            hum_parent = "thorax"
            hum_h = ball + [(Z, (0.05, 0, 0))]
        b.append(_seg("hum" + side, hum_parent, (0.0, 0.19 * s, 1.50), hum_h, 2.0,
                      (0, 0.19 * s, 1.35), (0.30, 0.045),
                      limits=lim_ball + [(-0.5, 0.5)] * (len(hum_h) - 3)))
        fa_h = [(Y, (0, 0, 0)), (Z, (0, 0, 0))] + ([(X, (0, 0, -0.05))] if full
                                                   else [])
        b.append(_seg("fore" + side, "hum" + side, (0.0, 0.19 * s, 1.20), fa_h,
                      1.25, (0, 0.19 * s, 1.08), (0.26, 0.035), scale=0.7,
                      limits=[(-2.2, 0.1), (-1.2, 1.2), (-0.4, 0.4)][:len(fa_h)]))
        if full:
            b.append(_seg("hand" + side, "fore" + side, (0.0, 0.19 * s, 0.94),
                          [(Y, (0, 0, 0)), (X, (0, 0, 0)), (Y, (0, 0, -0.04))],
                          0.5, (0, 0.19 * s, 0.87),
                          (0.03, 0.09, 0.18), scale=0.45, shape="box3",
                          limits=[(-1.0, 1.0)] * 3))
    for side in ("L", "R"):
        s = 1.0 if side == "L" else -1.0
        b.append(_seg("femur" + side, "pelvis", (0.0, 0.09 * s, 0.93),
                      ball + ([(Y, (0.05, 0, 0)), (X, (0, 0, -0.06))] if full
                              else []), 10.5,
                      (0, 0.09 * s, 0.75), (0.43, 0.06),
                      limits=lim_ball + [(-0.4, 0.4)] * (2 if full else 0)))
        kn = [(Y, (0, 0, 0))] + ([(Z, (0.05, 0, 0)), (X, (0, 0, -0.05)),
                                  (Y, (0, 0, -0.08))] if full
                                 else [(Z, (0.05, 0, 0))])
        b.append(_seg("tibia" + side, "femur" + side, (0.0, 0.09 * s, 0.50), kn,
                      3.3, (0, 0.09 * s, 0.32), (0.42, 0.045),
                      limits=[(-2.0, 0.1), (-0.3, 0.3), (-0.3, 0.3),
                              (-0.3, 0.3)][:len(kn)]))
        ft = [(Y, (0, 0, 0)), (X, (0.04, 0, -0.03)), (Z, (0.06, 0, 0))]
        if not full:
            ft = ft[:2]
        b.append(_seg("foot" + side, "tibia" + side, (0.0, 0.09 * s, 0.08), ft,
                      1.1, (0.05, 0.09 * s, 0.05), (0.22, 0.09, 0.06), scale=0.6,
                      shape="box3",
                      limits=[(-0.8, 0.6), (-0.4, 0.4), (-0.3, 0.3)][:len(ft)]))
        if full:
            b.append(_seg("toes" + side, "foot" + side, (0.15, 0.09 * s, 0.03),
                          [(Y, (0, 0, 0))], 0.35, (0.18, 0.09 * s, 0.025),
                          (0.06, 0.09, 0.03), scale=0.45, shape="box3",
                          limits=[(-0.5, 0.8)]))
    return b


def _inertia(mass, dims, shape, axis_long):
    """Principal moments (node axes) of a cylinder/box along axis_long, or
    of a box with world-axis extents dims when shape == "box3"."""
    if shape == "box3":
        lx, ly, lz = dims
        return mass / 12.0 * np.array([ly * ly + lz * lz, lx * lx + lz * lz,
                                       lx * lx + ly * ly])
    L, r = dims
    if shape == "cyl":
        Il = mass * r * r / 2.0
        It = mass * (3 * r * r + L * L) / 12.0
    else:
        Il = mass * (2 * r * r) / 12.0
        It = mass * (r * r + L * L) / 12.0
    I = np.full(3, It)
    I[axis_long] = Il
    return I


def human_model(seed: int = 2, full: bool = True, n_mus: int | None = None,
                total_mass: float = 75.0, damping: float = 0.1,
                contact=(1e5, 1e3, 1.0, 0.2), radius: float = 0.02) -> dict:
    """Synthetic whole-body model with a free root.

    full=True: 22 bodies, nv = 80 (6 root + 74 hinges), nq = 81, 24 contact
    spheres (8 per foot over heel/metatarsal/toe, 4 per hand), 700 muscles
    by default. full=False: 13 bodies, nv = 40, 16 foot spheres, 300
    muscles by default. Muscles cross a chain of 1-3
    consecutive hinge DoFs with 2-5 via-points; Hill parameters as in
    chain_model; insertion placed so the neutral path length is
    l_s + lambda0 * l_opt.
    """
    if n_mus is None:
        n_mus = 700 if full else 300
    rng = np.random.default_rng(seed)
    specs = _human_specs(full)
    for sp in specs:
        # each joint's hinges must span independent 6-D motions at neutral
        cols = [np.r_[ax, np.cross(np.array(off, float), ax)]
                for ax, off in sp["hinges"]]
        if cols:
            sv = np.linalg.svd(np.array(cols), compute_uv=False)
            assert sv.min() > 1e-3, (sp["name"], sv)
    msum = sum(sp["mass"] for sp in specs)
    mscale = total_mass / msum
    by_name = {sp["name"]: sp for sp in specs}
    # ---- nodes
    parent, jtype, jpos, axis, mass, com, inertia = [], [], [], [], [], [], []
    qlo, qhi, damp = [], [], []
    node_origin = []         # neutral world origin of each node
    node_body = []           # body spec index each node belongs to
    node_label = []          # "<body>:<hinge>" of each node ("<body>" for the root)
    body_last = {}           # body name -> node carrying its mass
    for bi, sp in enumerate(specs):
        if sp["parent"] is None:
            parent.append(-1)
            jtype.append(2)
            jpos.append([0, 0, 0])
            axis.append([0, 0, 0])
            node_origin.append(sp["center"].copy())
            node_body.append(bi)
            node_label.append(sp["name"])
            qlo += [-np.inf] * 6
            qhi += [np.inf] * 6
            damp += [0.0] * 6
        else:
            prev = body_last[sp["parent"]]
            for h, (ax, off) in enumerate(sp["hinges"]):
                origin = sp["center"] + np.array(off, float)
                parent.append(prev)
                jtype.append(0)
                jpos.append(origin - node_origin[prev])
                axis.append(ax)
                node_origin.append(origin)
                node_body.append(bi)
                node_label.append(f"{sp['name']}:{h}")
                lo, hi = sp["limits"][h]
                qlo.append(lo)
                qhi.append(hi)
                damp.append(damping)
                prev = len(parent) - 1
        last = len(parent) - 1
        body_last[sp["name"]] = last
        while len(mass) < len(parent):
            mass.append(0.0)
            com.append([0.0, 0.0, 0.0])
            inertia.append([0.0, 0.0, 0.0])
        m = sp["mass"] * mscale
        seg_dir = sp["com"] - sp["center"]
        axis_long = (int(np.argmax(np.abs(seg_dir)))
                     if np.linalg.norm(seg_dir) > 1e-9 else 2)
        mass[last] = m
        com[last] = list(sp["com"] - node_origin[last])
        inertia[last] = list(_inertia(m, sp["dims"], sp["shape"], axis_long))
    n = len(parent)
    # ---- per-node helpers for muscle placement
    dof_of_node = {}
    k = 0
    for i in range(n):
        dof_of_node[i] = k
        k += 6 if jtype[i] == 2 else 1
    body_mass_sub = {}
    for bi in reversed(range(len(specs))):
        sp = specs[bi]
        tot = sp["mass"] * mscale + sum(body_mass_sub[c["name"]] for c in specs
                                        if c["parent"] == sp["name"])
        body_mass_sub[sp["name"]] = tot
    hinge_nodes = [i for i in range(n) if jtype[i] == 0]
    w = np.array([body_mass_sub[specs[node_body[i]]["name"]] ** 0.5 *
                  specs[node_body[i]]["scale"] for i in hinge_nodes])
    w /= w.sum()

    def body_point(bi):
        """A point inside body bi (its COM at neutral)."""
        return specs[bi]["com"].copy()

    def seg_len(bi):
        sp = specs[bi]
        return max(float(np.linalg.norm(sp["com"] - sp["center"])) * 2.0, 0.05)

    f0, lo_, ls_, vn, vp, vstart = [], [], [], [], [], [0]
    for mi in range(n_mus):
        for _tries in range(400):
            end = hinge_nodes[int(rng.choice(len(hinge_nodes), p=w))]
            span = int(rng.choice([1, 2, 3], p=[0.35, 0.35, 0.30]))
            chain = [end]
            while len(chain) < span and jtype[parent[chain[0]]] == 0:
                chain.insert(0, parent[chain[0]])
            origin_node = parent[chain[0]]
            nodes_path = [origin_node] + chain
            P = int(rng.integers(2, 6))
            bo = node_body[origin_node]
            bd = node_body[end]
            J = node_origin[chain[0]]
            K = node_origin[end]
            up = body_point(bo) - J
            if bo == bd or np.linalg.norm(up) < 1e-3:
                up = -(body_point(bd) - K)
                if np.linalg.norm(up) < 1e-3:
                    up = np.array([0, 0, 1.0])
            up = up / np.linalg.norm(up)
            ud = body_point(bd) - K
            if np.linalg.norm(ud) < 1e-3:
                ud = -up
            ud = ud / np.linalg.norm(ud)
            scale = min(specs[bo]["scale"], specs[bd]["scale"])
            v = rng.normal(size=3)
            n_o = v - up * (v @ up)
            n_i = v - ud * (v @ ud)
            if np.linalg.norm(n_o) < 1e-6 or np.linalg.norm(n_i) < 1e-6:
                continue
            n_o /= np.linalg.norm(n_o)
            n_i /= np.linalg.norm(n_i)
            d_o, d_i = rng.uniform(0.02, 0.05, 2) * scale
            F0, lopt, lsl = _hill_draw(rng)
            lam0 = rng.uniform(0.9, 1.1)
            L0 = lsl + lam0 * lopt
            a = rng.uniform(0.1, 1.0) * seg_len(bo)
            O = J + a * up + d_o * n_o
            mid = 0.5 * (J + K) + 0.5 * (d_o + d_i) * (n_o + n_i) / max(
                np.linalg.norm(n_o + n_i), 1e-6)
            defl = rng.normal(size=(max(P - 2, 0), 3)) * 0.004 * scale

            def points(bb):
                I_ = K + bb * ud + d_i * n_i
                pts = [O]
                for kk in range(1, P - 1):
                    f = kk / (P - 1)
                    if f <= 0.5:
                        p = O + (mid - O) * (f / 0.5)
                    else:
                        p = mid + (I_ - mid) * ((f - 0.5) / 0.5)
                    pts.append(p + defl[kk - 1])
                pts.append(I_)
                return pts

            def length(pts):
                return sum(float(np.linalg.norm(pts[t + 1] - pts[t]))
                           for t in range(len(pts) - 1))

            bmax = max(seg_len(bd), 0.06) * 1.2
            if length(points(0.0)) > L0 or length(points(bmax)) < L0:
                continue
            lo_b, hi_b = 0.0, bmax
            for _ in range(60):
                mb = 0.5 * (lo_b + hi_b)
                if length(points(mb)) < L0:
                    lo_b = mb
                else:
                    hi_b = mb
            pts = points(0.5 * (lo_b + hi_b))
            break
        else:
            raise RuntimeError(f"muscle {mi} placement failed")
        for kk, p in enumerate(pts):
            if kk == 0:
                nd = origin_node
            elif kk == P - 1:
                nd = end
            else:
                nd = nodes_path[int(round(kk / (P - 1) * (len(nodes_path) - 1)))]
            vn.append(nd)
            vp.append(p - node_origin[nd])
        vstart.append(len(vn))
        f0.append(F0)
        lo_.append(lopt)
        ls_.append(lsl)
    # ---- contact spheres
    cn, cp = [], []

    def add_sphere(body, world):
        nd = body_last[body]
        cn.append(nd)
        cp.append(np.array(world, float) - node_origin[nd])

    for side in ("L", "R"):
        s = 1.0 if side == "L" else -1.0
        y0 = 0.09 * s
        foot = "foot" + side
        zc = 0.03 + radius - 0.03  # sphere centres at sole height
        if full:
            for dx, dy in ((-0.05, -0.025), (-0.05, 0.025), (0.02, -0.035),
                           (0.02, 0.035), (0.12, -0.04), (0.12, 0.04)):
                add_sphere(foot, (dx, y0 + dy, zc))
            for dy in (-0.03, 0.03):
                add_sphere("toes" + side, (0.19, y0 + dy, zc))
            hand = "hand" + side
            for dx, dz in ((0.02, 0.90), (-0.02, 0.90), (0.02, 0.82), (-0.02, 0.82)):
                add_sphere(hand, (dx, 0.19 * s, dz))
        else:
            for dx, dy in ((-0.05, -0.025), (-0.05, 0.025), (0.0, -0.035),
                           (0.0, 0.035), (0.06, -0.04), (0.06, 0.04),
                           (0.14, -0.03), (0.14, 0.03)):
                add_sphere(foot, (dx, y0 + dy, zc))
    con_world_z = min(node_origin[nd][2] + p[2] for nd, p in zip(cn, cp))
    root_z = node_origin[0][2] - (con_world_z - radius)
    model = dict(
        name=f"human{'80' if full else '40'}_m{n_mus}_s{seed}", parent=parent,
        jtype=jtype, jpos=jpos, jrot=np.tile(np.eye(3).ravel(), (n, 1)), axis=axis,
        mass=mass, com=com, inertia=inertia, damping=damp, qlo=qlo, qhi=qhi,
        f0=f0, l_opt=lo_, l_slack=ls_, v_max=np.full(n_mus, 10.0),
        tau_act=np.full(n_mus, 0.010), tau_deact=np.full(n_mus, 0.040),
        via_start=vstart, via_node=vn, via_pos=vp, con_node=cn, con_pos=cp,
        con_radius=np.full(len(cn), radius), contact=list(contact),
        gravity=[0.0, 0.0, -9.81])
    model = _finish(model)
    model["root_height"] = F32(root_z)
    model["n_body"] = int(sum(1 for m_ in model["mass"] if m_ > 0))
    model["node_label"] = node_label
    return model


def shoulder_coupling(model: dict, k: float = 5000.0, d: float = 50.0,
                      scap_ratio: float = 0.5, clav_ratio: float = 0.2) -> dict:
    """A copy of a whole-body model (full=True) with the scapulohumeral
    rhythm as joint-coupling equality constraints, per side: the scapula's
    third hinge follows scap_ratio times the humerus's third hinge (upward
    rotation with elevation, both about x), and the clavicle's second hinge
    (elevation, about x) clav_ratio times it; zero offsets (neutral pose
    consistent). Penalty stiffness k (N m / rad) and damping d (N m s / rad)."""
    lab = model["node_label"]
    dof, k_ = {}, 0
    for i, t in enumerate(model["jtype"]):
        dof[lab[i]] = k_
        k_ += 6 if t == 2 else 1
    start, dofs, coef = [0], [], []
    for side in ("L", "R"):
        hum = dof[f"hum{side}:2"]
        for part, ratio in ((f"scap{side}:2", scap_ratio), (f"clav{side}:1", clav_ratio)):
            dofs += [dof[part], hum]
            coef += [1.0, -ratio]
            start.append(len(dofs))
    out = dict(model)
    out["n_eq"] = len(start) - 1
    out["eq_start"] = np.asarray(start, np.int32)
    out["eq_dof"] = np.asarray(dofs, np.int32)
    out["eq_coef"] = np.asarray(coef, F32)
    out["eq_off"] = np.zeros(len(start) - 1, F32)
    out["eq_k"] = F32(k)
    out["eq_d"] = F32(d)
    out["name"] = model["name"] + "_coupled"
    return out


def human_initial_state(model: dict, n_env: int, seed: int = 8,
                        noise: float = 0.05):
    """Neutral standing pose, hinge noise U[-noise, noise], root at rest,
    root height such that the lowest sphere touches z = 0 at neutral."""
    rng = np.random.default_rng(seed)
    nq, nv = model["nq"], model["nv"]
    q = np.zeros((n_env, nq), F32)
    q[:, 2] = model["root_height"]
    q[:, 3] = 1.0
    q[:, 7:] = rng.uniform(-noise, noise, (n_env, nq - 7)).astype(F32)
    qd = np.zeros((n_env, nv), F32)
    act = np.zeros((n_env, model["n_mus"]), F32)
    return q, qd, act


def model_summary(model: dict) -> dict:
    """Sizes and tree depth (in DoFs) of a model."""
    n = model["n_node"]
    par = model["parent"]
    jt = model["jtype"]
    depth = np.zeros(n, int)
    for i in range(n):
        d = 6 if jt[i] == 2 else 1
        depth[i] = d + (depth[par[i]] if par[i] >= 0 else 0)
    return dict(name=model["name"], n_node=n, nq=model["nq"], nv=model["nv"],
                n_mus=model["n_mus"], n_con=model["n_con"],
                n_body=int((model["mass"] > 0).sum()),
                total_mass=float(model["mass"].sum()),
                max_dof_depth=int(depth.max()),
                n_via=int(model["via_start"][-1]))
