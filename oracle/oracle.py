"""ctypes binding of the FP64 C oracle (TEST INFRASTRUCTURE).

Builds ``liboracle.so`` from ``ora.c`` with gcc (plain -O2, no fast-math,
OpenMP over envs) and exposes each stage of the step as a numpy function.
Model arrays come from the seeded generator (float32/int32) and are promoted
to double inside the C code.

Pins (tests/test_oracle_pins.py, tests/test_oracle_mlp.py,
tests/test_oracle_tendon.py): every stage of the step, and the
compliant-tendon variant, against closed forms, finite differences,
invariants or a second route. The multi-step whole-body trajectory with contact as a whole has no
closed form and is pinned only through those parts: parity unpinned for the
composite.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "ora.c"), os.path.join(_HERE, "mlp.c")]
_LIB = os.path.join(_HERE, "liboracle.so")


def oracle_lib_path() -> str:
    return _LIB


def build_oracle(force: bool = True) -> str:
    """Compile the oracle (always when force=True)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-Wall", "-Wno-unused-function"] + _SRC + ["-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


_lib = None
_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_up = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


class _StageOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in
                ("act", "L", "Ldot", "F", "lm", "vm", "r", "tau_mus", "tau_ext",
                 "tau_d", "C", "qdd", "tau_eq", "M", "D")]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build_oracle(force=True)
    lib = C.CDLL(_LIB)
    lib.ora_model_create.restype = C.c_void_p
    lib.ora_model_create.argtypes = [
        C.c_int, _ip, _ip, _fp, _fp, _fp, _fp, _fp, _fp, _fp,
        C.c_int, _fp, _fp, _fp, _fp, _fp, _fp, _ip, _ip, _fp,
        C.c_int, _ip, _fp, _fp, _fp, _fp]
    lib.ora_model_destroy.argtypes = [C.c_void_p]
    lib.ora_model_set_coupling.argtypes = [C.c_void_p, C.c_int, _ip, _ip, _fp, _fp, C.c_float,
                                           C.c_float]
    lib.ora_coupling.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, C.c_void_p, C.c_void_p]
    for f in ("ora_fl", "ora_fp", "ora_fv", "ora_fv_slope"):
        getattr(lib, f).restype = C.c_double
        getattr(lib, f).argtypes = [C.c_double]
    lib.ora_fk.argtypes = [C.c_void_p, _dp, _dp, _dp]
    lib.ora_activation.argtypes = [C.c_void_p, C.c_double, _dp, _dp, _dp]
    lib.ora_geometry.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, _dp]
    lib.ora_hill.argtypes = [C.c_void_p, _dp, _dp, _dp, _dp, C.c_void_p, C.c_void_p]
    lib.ora_mass_matrix.argtypes = [C.c_void_p, _dp, _dp]
    lib.ora_rnea.argtypes = [C.c_void_p, _dp, _dp, _dp, C.c_int, _dp]
    lib.ora_contact.argtypes = [C.c_void_p, _dp, _dp, C.c_double, _dp, C.c_void_p,
                                C.POINTER(C.c_int)]
    lib.ora_chol_solve.restype = C.c_int
    lib.ora_chol_solve.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.ora_energy.restype = C.c_double
    lib.ora_energy.argtypes = [C.c_void_p, _dp, _dp]
    lib.ora_step.restype = C.c_uint32
    lib.ora_step.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp, _dp, _dp, _dp,
                             C.POINTER(_StageOut)]
    lib.ora_step_geo.restype = C.c_uint32
    lib.ora_step_geo.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp, _dp, _dp, _dp,
                                 C.c_void_p, C.c_void_p, C.POINTER(_StageOut)]
    lib.ora_fv_root.restype = C.c_double
    lib.ora_fv_root.argtypes = [C.c_double, C.c_double, C.c_double]
    lib.ora_step_tendon.restype = C.c_uint32
    lib.ora_step_tendon.argtypes = [C.c_void_p, C.c_double, C.c_int, _dp, _dp, _dp, _dp, _dp,
                                    C.c_double, C.c_double, C.POINTER(_StageOut)]
    lib.ora_rollout.argtypes = [C.c_void_p, C.c_int, C.c_int, C.c_double, C.c_int,
                                _dp, _dp, _dp, _fp, _up, C.c_int]
    lib.ora_bf16.restype = C.c_double
    lib.ora_bf16.argtypes = [C.c_double]
    lib.ora_mlp_forward.argtypes = [C.c_int] * 5 + [_fp] * 7 + [C.c_int, _dp] + [C.c_void_p] * 4
    lib.ora_mlp_grad.restype = C.c_double
    lib.ora_mlp_grad.argtypes = [C.c_int] * 5 + [_fp] * 7 + [_fp, C.c_void_p, C.c_int] + [_dp] * 6
    lib.ora_adam.argtypes = [C.c_int, _dp, _dp, _dp, _dp, C.c_double, C.c_double, C.c_double,
                             C.c_double, C.c_int]
    _lib = lib
    return lib


def _d(x):
    return np.ascontiguousarray(x, dtype=np.float64)


class Oracle:
    """FP64 oracle bound to one generated model."""

    def __init__(self, model: dict):
        self.lib = _load()
        m = model
        self.model = m
        self.nq, self.nv = m["nq"], m["nv"]
        self.n_mus, self.n_node = m["n_mus"], m["n_node"]
        c = np.ascontiguousarray
        self._keep = [c(m[k]) for k in (
            "parent", "jtype", "jpos", "jrot", "axis", "mass", "com", "inertia",
            "damping", "f0", "l_opt", "l_slack", "v_max", "tau_act", "tau_deact",
            "via_start", "via_node", "via_pos", "con_node", "con_pos",
            "con_radius", "contact", "gravity")]
        k = self._keep
        self.h = self.lib.ora_model_create(
            m["n_node"], k[0], k[1], k[2], k[3], k[4], k[5], k[6], k[7], k[8],
            m["n_mus"], k[9], k[10], k[11], k[12], k[13], k[14], k[15], k[16],
            k[17], m["n_con"], k[18], k[19], k[20], k[21], k[22])
        if m.get("n_eq", 0):
            self._keep_eq = [np.ascontiguousarray(m["eq_start"], np.int32),
                             np.ascontiguousarray(m["eq_dof"], np.int32),
                             np.ascontiguousarray(m["eq_coef"], np.float32),
                             np.ascontiguousarray(m["eq_off"], np.float32)]
            e = self._keep_eq
            self.lib.ora_model_set_coupling(self.h, int(m["n_eq"]), e[0], e[1], e[2], e[3],
                                            float(m["eq_k"]), float(m["eq_d"]))

    def __del__(self):
        try:
            self.lib.ora_model_destroy(self.h)
        except Exception:
            pass

    # ---- curves
    def fl(self, x):
        return self.lib.ora_fl(float(x))

    def fp(self, x):
        return self.lib.ora_fp(float(x))

    def fv(self, x):
        return self.lib.ora_fv(float(x))

    # ---- stages (single env, float64 arrays)
    def fk(self, q):
        R = np.zeros((self.n_node, 9))
        p = np.zeros((self.n_node, 3))
        self.lib.ora_fk(self.h, _d(q), R, p)
        return R.reshape(-1, 3, 3), p

    def activation(self, dt, u, act):
        out = np.zeros(self.n_mus)
        self.lib.ora_activation(self.h, dt, _d(u), _d(act), out)
        return out

    def geometry(self, q, qd):
        L = np.zeros(self.n_mus)
        r = np.zeros((self.n_mus, self.nv))
        Ld = np.zeros(self.n_mus)
        self.lib.ora_geometry(self.h, _d(q), _d(qd), L, r, Ld)
        return L, r, Ld

    def hill(self, act, L, Ldot):
        F = np.zeros(self.n_mus)
        self.lib.ora_hill(self.h, _d(act), _d(L), _d(Ldot), F, None, None)
        return F

    def mass_matrix(self, q):
        M = np.zeros((self.nv, self.nv))
        self.lib.ora_mass_matrix(self.h, _d(q), M)
        return M

    def rnea(self, q, qd, qdd, grav=True):
        tau = np.zeros(self.nv)
        self.lib.ora_rnea(self.h, _d(q), _d(qd), _d(qdd), int(grav), tau)
        return tau

    def bias(self, q, qd):
        return self.rnea(q, qd, np.zeros(self.nv), True)

    def fv_slope(self, x):
        return self.lib.ora_fv_slope(float(x))

    def fv_root(self, A, R, beta):
        """The fibre velocity v with A f_v(v) + beta v = R (bisection)."""
        return self.lib.ora_fv_root(float(A), float(R), float(beta))

    def step_tendon(self, dt, q, qd, act, lm, u, eps0, beta, contact=True, stages=False):
        """One step of one env with compliant tendons; lm[n_mus] is the
        fibre length in metres. Returns (q', qd', act', lm', status[,
        stages]); stages F is the force of the right-hand side, lm and vm
        the normalised fibre length and velocity at the start."""
        q, qd, act, lm = _d(q).copy(), _d(qd).copy(), _d(act).copy(), _d(lm).copy()
        out = None
        st_arrays = {}
        if stages:
            nm, nv = self.n_mus, self.nv
            shapes = dict(act=nm, L=nm, Ldot=nm, F=nm, lm=nm, vm=nm, r=(nm, nv),
                          tau_mus=nv, tau_ext=nv, tau_d=nv, C=nv, qdd=nv, tau_eq=nv,
                          M=(nv, nv), D=(nv, nv))
            st_arrays = {k: np.zeros(s) for k, s in shapes.items()}
            out = _StageOut(**{k: v.ctypes.data for k, v in st_arrays.items()})
        st = self.lib.ora_step_tendon(self.h, dt, int(contact), q, qd, act, lm, _d(u),
                                      float(eps0), float(beta),
                                      C.byref(out) if out is not None else None)
        if stages:
            return q, qd, act, lm, st, st_arrays
        return q, qd, act, lm, st

    def contact(self, q, qd, dt, with_slope=False):
        tau = np.zeros(self.nv)
        D = np.zeros((self.nv, self.nv))
        n = C.c_int(0)
        self.lib.ora_contact(self.h, _d(q), _d(qd), float(dt), tau,
                             D.ctypes.data if with_slope else None, C.byref(n))
        if with_slope:
            return tau, n.value, D
        return tau, n.value

    def chol_solve(self, M, b):
        x = np.zeros(len(b))
        rc = self.lib.ora_chol_solve(len(b), _d(M), _d(b), x)
        return x, rc

    def coupling(self, q, qd, dt):
        """(tau_eq[nv], D_eq[nv][nv], phi[n_eq]) of the joint coupling."""
        nv = self.nv
        tau = np.zeros(nv)
        D = np.zeros((nv, nv))
        phi = np.zeros(max(int(self.model.get("n_eq", 0)), 1))
        self.lib.ora_coupling(self.h, _d(q), _d(qd), float(dt), tau, D.ctypes.data,
                              phi.ctypes.data)
        return tau, D, phi[:int(self.model.get("n_eq", 0))]

    def energy(self, q, qd):
        return self.lib.ora_energy(self.h, _d(q), _d(qd))

    def step(self, dt, q, qd, act, u, contact=True, stages=False, geometry=None):
        """One step of one env; returns (q', qd', act', status[, stages]).
        geometry = (L[n_mus], r[n_mus][nv]) replaces the via-point geometry
        (the lengthening rate then follows as -r qd)."""
        q, qd, act = _d(q).copy(), _d(qd).copy(), _d(act).copy()
        gL = gr = None
        if geometry is not None:
            gL = _d(geometry[0]).copy()
            gr = _d(geometry[1]).reshape(self.n_mus, self.nv).copy()
        out = None
        st_arrays = {}
        if stages:
            nm, nv = self.n_mus, self.nv
            shapes = dict(act=nm, L=nm, Ldot=nm, F=nm, lm=nm, vm=nm, r=(nm, nv),
                          tau_mus=nv, tau_ext=nv, tau_d=nv, C=nv, qdd=nv, tau_eq=nv,
                          M=(nv, nv), D=(nv, nv))
            st_arrays = {k: np.zeros(s) for k, s in shapes.items()}
            out = _StageOut(**{k: v.ctypes.data for k, v in st_arrays.items()})
        st = self.lib.ora_step_geo(self.h, dt, int(contact), q, qd, act, _d(u),
                                   gL.ctypes.data if gL is not None else None,
                                   gr.ctypes.data if gr is not None else None,
                                   C.byref(out) if out is not None else None)
        if stages:
            return q, qd, act, st, st_arrays
        return q, qd, act, st

    def rollout(self, dt, q, qd, act, u, contact=True, threads=None):
        """Batched rollout. q,qd,act: (E, .) float64 (updated copies
        returned); u: float32 (T, E, n_mus)."""
        q, qd, act = _d(q).copy(), _d(qd).copy(), _d(act).copy()
        u = np.ascontiguousarray(u, dtype=np.float32)
        T, E = u.shape[0], u.shape[1]
        status = np.zeros(E, np.uint32)
        if threads is None:
            threads = max(1, min(len(os.sched_getaffinity(0)), E))
        self.lib.ora_rollout(self.h, E, T, dt, int(contact), q, qd, act, u, status,
                             int(threads))
        return q, qd, act, status


# ------------------------------------------------------------ surrogate MLP
def bf16(v):
    """Round to bfloat16 (nearest even) and back."""
    return _load().ora_bf16(float(v))


def _f(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def mlp_forward(params, x, bf16=True):
    """params = (W1, b1, W2, b2, W3, b3) with W[in][out]; x [B][n0]."""
    W1, b1, W2, b2, W3, b3 = (_f(p) for p in params)
    x = _f(x)
    B, n0 = x.shape
    n1, n2, n3 = W1.shape[1], W2.shape[1], W3.shape[1]
    y = np.zeros((B, n3))
    _load().ora_mlp_forward(B, n0, n1, n2, n3, W1, b1, W2, b2, W3, b3, x, int(bf16), y,
                            None, None, None, None)
    return y


def mlp_grad(params, x, t, mask=None, bf16=True):
    """Loss = mean(mask (y - t)^2) and the gradients of every parameter."""
    W1, b1, W2, b2, W3, b3 = (_f(p) for p in params)
    x, t = _f(x), _f(t)
    B, n0 = x.shape
    n1, n2, n3 = W1.shape[1], W2.shape[1], W3.shape[1]
    g = [np.zeros(p.shape) for p in (W1, b1, W2, b2, W3, b3)]
    mk = None if mask is None else _f(mask)
    loss = _load().ora_mlp_grad(B, n0, n1, n2, n3, W1, b1, W2, b2, W3, b3, x, t,
                                mk.ctypes.data if mk is not None else None, int(bf16), *g)
    return loss, g


def adam(w, m, v, g, lr, b1=0.9, b2=0.999, eps=1e-8, step=1):
    """One Adam step in place on float64 arrays."""
    _load().ora_adam(w.size, w, m, v, np.ascontiguousarray(g, np.float64), lr, b1, b2, eps, step)
