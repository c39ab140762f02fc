"""ctypes binding of libms.so (argument marshalling only).

Every step of the path runs in the library's HIP kernels; this module only
converts a model dict into the C description, hands device pointers of torch
tensors to the C ABI and raises on error status. It fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libms.so")

MS_ST_NONFINITE = 1
MS_ST_NONSPD = 2
MS_ST_FALLBACK = 4
EXC_ARRAY, EXC_IID, EXC_AR1 = 0, 1, 2
SCHED_AUTO, SCHED_FUSED, SCHED_SPLIT = 0, 1, 2
ISSUE_CONCURRENT, ISSUE_CONCURRENT_MOST_WORK, ISSUE_SERIAL = 0, 1, 2

EXPORTED = ("ms_model_create", "ms_model_destroy", "ms_model_info_get",
            "ms_step_batch", "ms_rollout", "ms_step_stages", "ms_model_spans",
            "ms_model_mass_pattern", "ms_last_error", "ms_geometry",
            "ms_surrogate_create", "ms_surrogate_destroy", "ms_surrogate_dims",
            "ms_surrogate_params", "ms_surrogate_grads", "ms_surrogate_set_norm",
            "ms_surrogate_sample", "ms_surrogate_forward", "ms_surrogate_train_step",
            "ms_surrogate_last_error", "ms_rollout_surrogate",
            "ms_batch_create", "ms_batch_destroy", "ms_batch_rollout", "ms_batch_autotune",
            "ms_batch_config", "ms_batch_set_config", "ms_batch_last_error",
            "ms_policy_create", "ms_policy_destroy", "ms_policy_dims", "ms_policy_params",
            "ms_policy_act", "ms_policy_rollout", "ms_surrogate_reserve",
            "ms_surrogate_forward_noalloc", "ms_surrogate_noalloc_max", "ms_policy_reserve",
            "ms_model_set_schedule", "ms_model_get_schedule", "ms_model_reserve",
            "ms_model_set_kernel_timing", "ms_model_kernel_times", "ms_model_set_key_nodes",
            "ms_rollout_record", "ms_surrogate_train", "ms_surrogate_save", "ms_surrogate_load",
            "ms_controller_create", "ms_controller_destroy", "ms_controller_dims",
            "ms_controller_params", "ms_controller_reserve", "ms_controller_step",
            "ms_controller_last_error", "ms_model_set_split_streams", "ms_model_split_parts",
            "ms_rollout_tendon")

_fptr = C.POINTER(C.c_float)
_iptr = C.POINTER(C.c_int32)


class MsDesc(C.Structure):
    _fields_ = [
        ("n_node", C.c_int32), ("parent", _iptr), ("jtype", _iptr),
        ("jpos", _fptr), ("jrot", _fptr), ("axis", _fptr), ("mass", _fptr),
        ("com", _fptr), ("inertia", _fptr), ("damping", _fptr), ("qlo", _fptr),
        ("qhi", _fptr),
        ("n_mus", C.c_int32), ("f0", _fptr), ("l_opt", _fptr), ("l_slack", _fptr),
        ("v_max", _fptr), ("tau_act", _fptr), ("tau_deact", _fptr),
        ("via_start", _iptr), ("via_node", _iptr), ("via_pos", _fptr),
        ("n_con", C.c_int32), ("con_node", _iptr), ("con_pos", _fptr),
        ("con_radius", _fptr), ("contact", C.c_float * 4), ("gravity", C.c_float * 3),
        ("n_eq", C.c_int32), ("eq_start", _iptr), ("eq_dof", _iptr), ("eq_coef", _fptr),
        ("eq_off", _fptr), ("eq_k", C.c_float), ("eq_d", C.c_float)]


class MsInfo(C.Structure):
    _fields_ = [(k, C.c_int32) for k in ("nq", "nv", "n_node", "n_mus", "n_con",
                                         "n_body", "max_dof_depth", "nnz_mass",
                                         "lds_bytes", "lds_shared_bytes")]


class MsOpts(C.Structure):
    _fields_ = [("dt", C.c_float), ("contact", C.c_int32)]


class MsExc(C.Structure):
    _fields_ = [("kind", C.c_int32), ("u", C.c_void_p), ("seed", C.c_uint64),
                ("step0", C.c_int64), ("x", C.c_void_p), ("rho", C.c_float),
                ("s", C.c_float), ("mean", C.c_float)]


class MsRecord(C.Structure):
    _fields_ = [("every", C.c_int32)] + [(k, C.c_void_p) for k in (
        "act", "force", "lm", "vm", "power", "xpos", "xmat", "n_applied")]


class MsTendon(C.Structure):
    _fields_ = [("eps0", C.c_float), ("beta", C.c_float)]


class MsTrainCfg(C.Structure):
    _fields_ = [("n_samples", C.c_int64), ("batch", C.c_int32), ("iters", C.c_int32),
                ("step0", C.c_int32), ("norm_samples", C.c_int32), ("lr0", C.c_float),
                ("lr1", C.c_float), ("seed", C.c_uint64), ("norm_seed", C.c_uint64),
                ("loss", C.c_void_p)]


class MsCtlDesc(C.Structure):
    _fields_ = [("hidden", C.c_int32), ("n_sub", C.c_int32), ("flow_steps", C.c_int32),
                ("flow_dt", C.c_float), ("sigma0", C.c_float), ("n_key", C.c_int32),
                ("key_nodes", C.c_void_p), ("ref_seed", C.c_uint64), ("noise_seed", C.c_uint64),
                ("pi_seed", C.c_uint64), ("flow_seed", C.c_uint64), ("disc_seed", C.c_uint64)]


class MsCtlOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("obs", "a0", "u", "delta", "n_applied")]


class MsBatchState(C.Structure):
    _fields_ = [("q", C.c_void_p), ("qd", C.c_void_p), ("act", C.c_void_p),
                ("status", C.c_void_p)]


class MsStageOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("act", "L", "Ldot", "F", "r", "tau_mus",
                                          "bias_minus_ext", "qdd", "mass")]


_lib = None


def lib():
    """Load libms.so; raise if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp = C.c_void_p
    L.ms_model_create.argtypes = [C.POINTER(MsDesc), C.POINTER(vp)]
    L.ms_model_destroy.argtypes = [vp]
    L.ms_model_destroy.restype = None
    L.ms_model_info_get.argtypes = [vp, C.POINTER(MsInfo)]
    L.ms_model_set_schedule.argtypes = [vp, C.c_int32]
    L.ms_model_get_schedule.argtypes = [vp, _iptr]
    L.ms_model_reserve.argtypes = [vp, C.c_int32]
    L.ms_model_set_split_streams.argtypes = [vp, C.c_int32]
    L.ms_model_split_parts.argtypes = [vp, C.c_int32, _iptr, _iptr]
    L.ms_model_set_kernel_timing.argtypes = [vp, C.c_int32]
    L.ms_model_kernel_times.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int64)]
    L.ms_model_set_key_nodes.argtypes = [vp, C.c_int32, _iptr]
    L.ms_rollout_record.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.POINTER(MsExc), C.c_int32,
                                    C.POINTER(MsOpts), C.POINTER(MsRecord), vp]
    L.ms_rollout_tendon.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, C.POINTER(MsExc),
                                    C.c_int32, C.POINTER(MsOpts), C.POINTER(MsTendon),
                                    C.POINTER(MsRecord), vp]
    L.ms_step_batch.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, C.POINTER(MsOpts), vp]
    L.ms_rollout.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.POINTER(MsExc), C.c_int32,
                             C.POINTER(MsOpts), vp]
    L.ms_step_stages.argtypes = [vp, C.c_int32, vp, vp, vp, vp, C.POINTER(MsOpts),
                                 C.POINTER(MsStageOut), vp]
    L.ms_model_spans.argtypes = [vp, _iptr]
    L.ms_geometry.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.ms_model_mass_pattern.argtypes = [vp, _iptr, _iptr]
    L.ms_last_error.restype = C.c_char_p
    L.ms_surrogate_last_error.restype = C.c_char_p
    L.ms_surrogate_create.argtypes = [vp, C.c_int32, C.c_uint64, C.POINTER(vp)]
    L.ms_surrogate_destroy.argtypes = [vp]
    L.ms_surrogate_destroy.restype = None
    L.ms_surrogate_dims.argtypes = [vp, _iptr]
    L.ms_surrogate_params.argtypes = [vp, C.c_int32] + [_fptr] * 6
    L.ms_surrogate_grads.argtypes = [vp] + [_fptr] * 6
    L.ms_surrogate_set_norm.argtypes = [vp, _fptr, _fptr]
    L.ms_surrogate_sample.argtypes = [vp, C.c_int32, C.c_uint64, C.c_int64, vp, vp]
    L.ms_surrogate_forward.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.ms_surrogate_train_step.argtypes = [vp, C.c_int32, vp, vp, vp, C.c_float, C.c_int32, vp, vp]
    L.ms_surrogate_reserve.argtypes = [vp, C.c_int32]
    L.ms_controller_create.argtypes = [vp, C.POINTER(MsCtlDesc), C.POINTER(vp)]
    L.ms_controller_destroy.argtypes = [vp]
    L.ms_controller_destroy.restype = None
    L.ms_controller_dims.argtypes = [vp, _iptr]
    L.ms_controller_params.argtypes = [vp, C.c_int32, C.c_int32, C.POINTER(_fptr),
                                       C.POINTER(_fptr), _fptr, _fptr]
    L.ms_controller_reserve.argtypes = [vp, C.c_int32]
    L.ms_controller_step.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, C.c_int64, C.c_double,
                                     C.POINTER(MsOpts), vp, vp, C.POINTER(MsCtlOut), vp]
    L.ms_controller_last_error.restype = C.c_char_p
    L.ms_surrogate_train.argtypes = [vp, vp, C.POINTER(MsTrainCfg), vp]
    L.ms_surrogate_save.argtypes = [vp, vp, C.c_size_t, C.POINTER(C.c_size_t)]
    L.ms_surrogate_load.argtypes = [vp, vp, C.c_size_t]
    L.ms_surrogate_forward_noalloc.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.ms_surrogate_noalloc_max.argtypes = [vp]
    L.ms_surrogate_noalloc_max.restype = C.c_int32
    L.ms_policy_reserve.argtypes = [vp, C.c_int32]
    L.ms_rollout_surrogate.argtypes = [vp, vp, C.c_int32, vp, vp, vp, vp, C.POINTER(MsExc),
                                       C.c_int32, C.POINTER(MsOpts), C.c_float, vp, vp]
    L.ms_rollout_surrogate.restype = C.c_int
    L.ms_policy_create.argtypes = [vp, C.c_int32, C.c_int32, C.c_uint64, C.c_uint64, C.POINTER(vp)]
    L.ms_policy_destroy.argtypes = [vp]
    L.ms_policy_destroy.restype = None
    L.ms_policy_dims.argtypes = [vp, _iptr]
    L.ms_policy_params.argtypes = [vp, C.c_int32] + [_fptr] * 6
    L.ms_policy_act.argtypes = [vp, C.c_int32, vp, vp, C.c_double, C.c_int64, vp, vp, vp]
    L.ms_policy_rollout.argtypes = [vp, vp, vp, C.c_int32, vp, vp, vp, vp, C.c_int32, C.c_int32,
                                    C.c_double, C.POINTER(MsOpts), C.c_float, vp, vp, vp]
    for f in ("ms_policy_create", "ms_policy_dims", "ms_policy_params", "ms_policy_act",
              "ms_policy_rollout", "ms_policy_reserve"):
        getattr(L, f).restype = C.c_int
    L.ms_batch_create.argtypes = [C.POINTER(vp), _iptr, C.c_int32, C.POINTER(vp)]
    L.ms_batch_destroy.argtypes = [vp]
    L.ms_batch_destroy.restype = None
    L.ms_batch_rollout.argtypes = [vp, C.POINTER(MsBatchState), C.POINTER(MsExc), C.c_int32,
                                   C.POINTER(MsOpts), vp]
    L.ms_batch_autotune.argtypes = [vp, C.POINTER(MsBatchState), C.POINTER(MsExc), C.c_int32,
                                    C.POINTER(MsOpts), vp]
    L.ms_batch_config.argtypes = [vp, _iptr, _iptr]
    L.ms_batch_set_config.argtypes = [vp, _iptr, C.c_int32]
    L.ms_batch_last_error.restype = C.c_char_p
    for f in ("ms_batch_create", "ms_batch_rollout", "ms_batch_autotune", "ms_batch_config",
              "ms_batch_set_config"):
        getattr(L, f).restype = C.c_int
    for f in ("ms_surrogate_create", "ms_surrogate_dims", "ms_surrogate_params",
              "ms_surrogate_grads", "ms_surrogate_set_norm", "ms_surrogate_sample",
              "ms_surrogate_forward", "ms_surrogate_train_step"):
        getattr(L, f).restype = C.c_int
    for f in ("ms_model_create", "ms_model_info_get", "ms_step_batch", "ms_rollout",
              "ms_step_stages", "ms_model_spans", "ms_model_mass_pattern", "ms_geometry"):
        getattr(L, f).restype = C.c_int
    _lib = L
    return L


class MsError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libms error {code}: {msg}")
        self.code = code


def _check(rc):
    if rc != 0:
        raise MsError(rc, lib().ms_last_error().decode())


def _check_s(rc):
    if rc != 0:
        raise MsError(rc, lib().ms_surrogate_last_error().decode())


def _ptr(a, dtype, ctype):
    return np.ascontiguousarray(a, dtype=dtype).ctypes.data_as(C.POINTER(ctype))


def _dp(t):
    """Device pointer of a torch tensor (or None)."""
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "expected a contiguous device tensor"
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    return C.c_void_p(getattr(stream, "cuda_stream", stream))


class Model:
    """A model compiled into libms device tables."""

    def __init__(self, model: dict):
        L = lib()
        m = model
        self._arrays = {}

        def keep(name, dtype):
            a = np.ascontiguousarray(m[name], dtype=dtype)
            self._arrays[name] = a
            return a.ctypes.data_as(C.POINTER(C.c_float if dtype == np.float32 else C.c_int32))

        d = MsDesc()
        d.n_node = m["n_node"]
        d.parent, d.jtype = keep("parent", np.int32), keep("jtype", np.int32)
        for k in ("jpos", "jrot", "axis", "mass", "com", "inertia", "damping", "qlo", "qhi"):
            setattr(d, k, keep(k, np.float32))
        d.n_mus = m["n_mus"]
        for k in ("f0", "l_opt", "l_slack", "v_max", "tau_act", "tau_deact", "via_pos"):
            setattr(d, k, keep(k, np.float32))
        d.via_start, d.via_node = keep("via_start", np.int32), keep("via_node", np.int32)
        d.n_con = m["n_con"]
        d.con_node = keep("con_node", np.int32)
        d.con_pos, d.con_radius = keep("con_pos", np.float32), keep("con_radius", np.float32)
        d.contact = (C.c_float * 4)(*[float(x) for x in m["contact"]])
        d.gravity = (C.c_float * 3)(*[float(x) for x in m["gravity"]])
        d.n_eq = int(m.get("n_eq", 0))
        if d.n_eq:
            d.eq_start, d.eq_dof = keep("eq_start", np.int32), keep("eq_dof", np.int32)
            d.eq_coef, d.eq_off = keep("eq_coef", np.float32), keep("eq_off", np.float32)
            d.eq_k, d.eq_d = float(m["eq_k"]), float(m["eq_d"])
        h = C.c_void_p()
        _check(L.ms_model_create(C.byref(d), C.byref(h)))
        self.h = h
        info = MsInfo()
        _check(L.ms_model_info_get(h, C.byref(info)))
        self.info = {k: getattr(info, k) for k, _ in MsInfo._fields_}
        self.nq, self.nv, self.n_mus = info.nq, info.nv, info.n_mus
        self.nnz = info.nnz_mass

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ms_model_destroy(self.h)
        except Exception:
            pass

    def set_schedule(self, schedule):
        """SCHED_AUTO, SCHED_FUSED or SCHED_SPLIT (same results, different
        kernels)."""
        _check(lib().ms_model_set_schedule(self.h, int(schedule)))

    def set_split_streams(self, streams):
        """Split schedule: the batch in `streams` (1 to 4) concurrent parts,
        each on a stream of its own; 0 automatic."""
        _check(lib().ms_model_set_split_streams(self.h, int(streams)))

    def split_parts(self, n_env):
        """Env bounds of the concurrent parts a step of n_env envs runs in
        (part h: bounds[h] .. bounds[h + 1])."""
        b = np.zeros(5, np.int32)
        n = np.zeros(1, np.int32)
        _check(lib().ms_model_split_parts(self.h, int(n_env), b.ctypes.data_as(_iptr),
                                          n.ctypes.data_as(_iptr)))
        return [int(x) for x in b[:int(n[0]) + 1]]

    def schedule(self):
        """The schedule steps run with now (SCHED_FUSED or SCHED_SPLIT)."""
        v = C.c_int32()
        _check(lib().ms_model_get_schedule(self.h, C.byref(v)))
        return int(v.value)

    def reserve(self, n_env):
        """Reserve the split schedule's workspace for n_env envs (allocates
        now, so later calls, e.g. inside a graph capture, do not)."""
        _check(lib().ms_model_reserve(self.h, int(n_env)))

    def set_kernel_timing(self, every=1):
        """Record HIP events around the split-schedule kernels of every
        every-th step of each call from now on (0: off)."""
        _check(lib().ms_model_set_kernel_timing(self.h, int(every)))

    def kernel_times(self):
        """(summed ms of the kinematics/dynamics, muscle and factorisation
        kernels, steps timed) since the last call; waits for the events."""
        t = (C.c_double * 3)()
        n = C.c_int64()
        _check(lib().ms_model_kernel_times(self.h, t, C.byref(n)))
        return [float(x) for x in t], int(n.value)

    def spans(self):
        s = np.zeros((self.n_mus, 3), np.int32)
        _check(lib().ms_model_spans(self.h, s.ctypes.data_as(_iptr)))
        return s

    def mass_pattern(self):
        r = np.zeros(self.nnz, np.int32)
        c = np.zeros(self.nnz, np.int32)
        _check(lib().ms_model_mass_pattern(self.h, r.ctypes.data_as(_iptr), c.ctypes.data_as(_iptr)))
        return r, c

    def geometry(self, q, L, r, stream=None):
        """Exact lengths L[n][n_mus] and moment arms r[n][n_mus][3] of poses q."""
        _check(lib().ms_geometry(self.h, q.shape[0], _dp(q), _dp(L), _dp(r), _stream(stream)))

    def step_batch(self, q, qd, act, status, u, dt, contact=True, stream=None):
        n_env = q.shape[0]
        o = MsOpts(dt, int(contact))
        _check(lib().ms_step_batch(self.h, n_env, _dp(q), _dp(qd), _dp(act), _dp(status),
                                   _dp(u), C.byref(o), _stream(stream)))

    def rollout(self, q, qd, act, status, n_steps, dt, contact=True, kind=EXC_ARRAY,
                u=None, seed=0, step0=0, x=None, ar1=(0.0, 0.0, 0.0), stream=None):
        n_env = q.shape[0]
        o = MsOpts(dt, int(contact))
        e = MsExc(kind, _dp(u), seed, step0, _dp(x), float(ar1[0]), float(ar1[1]),
                  float(ar1[2]))
        _check(lib().ms_rollout(self.h, n_env, _dp(q), _dp(qd), _dp(act), _dp(status),
                                C.byref(e), n_steps, C.byref(o), _stream(stream)))

    def rollout_tendon(self, q, qd, act, lm, status, n_steps, dt, contact=True, eps0=0.033,
                       beta=0.1, kind=EXC_ARRAY, u=None, seed=0, step0=0, x=None,
                       ar1=(0.0, 0.0, 0.0), every=1, obs=None, n_applied=None, stream=None):
        """rollout() with compliant tendons; lm (device float32 [n_env][n_mus],
        metres) is the fibre length, advanced with the state. obs, every and
        n_applied record observables as in rollout_record."""
        n_env = q.shape[0]
        o = MsOpts(dt, int(contact))
        e = MsExc(kind, _dp(u), seed, step0, _dp(x), float(ar1[0]), float(ar1[1]),
                  float(ar1[2]))
        t = MsTendon(float(eps0), float(beta))
        rec = None
        if obs or n_applied is not None:
            obs = obs or {}
            rec = MsRecord(int(every), *[_dp(obs.get(k)) for k in
                                         ("act", "force", "lm", "vm", "power", "xpos", "xmat")],
                           _dp(n_applied))
        _check(lib().ms_rollout_tendon(self.h, n_env, _dp(q), _dp(qd), _dp(act), _dp(lm),
                                       _dp(status), C.byref(e), n_steps, C.byref(o),
                                       C.byref(t), C.byref(rec) if rec is not None else None,
                                       _stream(stream)))

    def set_key_nodes(self, nodes):
        """Key nodes whose world frames rollout_record writes."""
        a = np.ascontiguousarray(nodes, np.int32)
        _check(lib().ms_model_set_key_nodes(self.h, len(a), a.ctypes.data_as(_iptr)))

    def rollout_record(self, q, qd, act, status, n_steps, dt, contact=True, kind=EXC_ARRAY,
                       u=None, seed=0, step0=0, x=None, ar1=(0.0, 0.0, 0.0), every=1,
                       obs=None, n_applied=None, stream=None):
        """rollout() that writes the observables named in obs (dict of device
        tensors: act, force, lm, vm, power [n_rec][n_env][n_mus], xpos
        [n_rec][n_env][n_key][3], xmat [..][9]) every `every` steps and adds
        the steps applied to each env to n_applied (uint32/int32 [n_env])."""
        obs = obs or {}
        n_env = q.shape[0]
        o = MsOpts(dt, int(contact))
        e = MsExc(kind, _dp(u), seed, step0, _dp(x), float(ar1[0]), float(ar1[1]),
                  float(ar1[2]))
        r = MsRecord(int(every), *[_dp(obs.get(k)) for k in
                                   ("act", "force", "lm", "vm", "power", "xpos", "xmat")],
                     _dp(n_applied))
        _check(lib().ms_rollout_record(self.h, n_env, _dp(q), _dp(qd), _dp(act), _dp(status),
                                       C.byref(e), n_steps, C.byref(o), C.byref(r),
                                       _stream(stream)))

    def rollout_surrogate(self, sg, q, qd, act, status, n_steps, dt, contact=True, tol=1e-4,
                          fb_count=None, kind=EXC_ARRAY, u=None, seed=0, step0=0, x=None,
                          ar1=(0.0, 0.0, 0.0), stream=None):
        n_env = q.shape[0]
        o = MsOpts(dt, int(contact))
        e = MsExc(kind, _dp(u), seed, step0, _dp(x), float(ar1[0]), float(ar1[1]),
                  float(ar1[2]))
        _check(lib().ms_rollout_surrogate(self.h, sg.h, n_env, _dp(q), _dp(qd), _dp(act),
                                          _dp(status), C.byref(e), n_steps, C.byref(o),
                                          float(tol), _dp(fb_count), _stream(stream)))

    def step_stages(self, q, qd, act, u, dt, contact=True, stream=None):
        import torch
        E = q.shape[0]
        dev = q.device
        nm, nv = self.n_mus, self.nv
        out = dict(act=torch.empty(E, nm, device=dev), L=torch.empty(E, nm, device=dev),
                   Ldot=torch.empty(E, nm, device=dev), F=torch.empty(E, nm, device=dev),
                   r=torch.empty(E, nm, 3, device=dev), tau_mus=torch.empty(E, nv, device=dev),
                   bias_minus_ext=torch.empty(E, nv, device=dev),
                   qdd=torch.empty(E, nv, device=dev),
                   mass=torch.empty(E, self.nnz, dtype=torch.float64, device=dev))
        so = MsStageOut(**{k: _dp(v) for k, v in out.items()})
        o = MsOpts(dt, int(contact))
        _check(lib().ms_step_stages(self.h, E, _dp(q), _dp(qd), _dp(act), _dp(u), C.byref(o),
                                    C.byref(so), _stream(stream)))
        return out


class Surrogate:
    """The library's learned muscle-geometry network bound to a Model."""

    def __init__(self, model: Model, hidden: int = 512, seed: int = 41):
        L = lib()
        self.model = model
        h = C.c_void_p()
        _check_s(L.ms_surrogate_create(model.h, hidden, seed, C.byref(h)))
        self.h = h
        d = np.zeros(4, np.int32)
        _check_s(L.ms_surrogate_dims(h, d.ctypes.data_as(_iptr)))
        self.n_in, self.h1, self.h2, self.n_out = (int(x) for x in d)
        self.shapes = [(self.h1, self.n_in), (self.h1,), (self.h2, self.h1), (self.h2,),
                       (self.n_out, self.h2), (self.n_out,)]

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ms_surrogate_destroy(self.h)
        except Exception:
            pass

    def _bufs(self):
        return [np.zeros(s, np.float32) for s in self.shapes]

    def params(self):
        b = self._bufs()
        _check_s(lib().ms_surrogate_params(self.h, 0, *[x.ctypes.data_as(_fptr) for x in b]))
        return b

    def set_params(self, ps):
        b = [np.ascontiguousarray(p, np.float32).reshape(s) for p, s in zip(ps, self.shapes)]
        _check_s(lib().ms_surrogate_params(self.h, 1, *[x.ctypes.data_as(_fptr) for x in b]))

    def grads(self):
        b = self._bufs()
        _check_s(lib().ms_surrogate_grads(self.h, *[x.ctypes.data_as(_fptr) for x in b]))
        return b

    def set_norm(self, mean, std):
        m = np.ascontiguousarray(mean, np.float32)
        s = np.ascontiguousarray(std, np.float32)
        _check_s(lib().ms_surrogate_set_norm(self.h, m.ctypes.data_as(_fptr), s.ctypes.data_as(_fptr)))

    def save(self, path):
        """Write the network (layer sizes, float32 weights and biases, output
        standardisation) as the library's plain binary blob."""
        n = C.c_size_t()
        _check_s(lib().ms_surrogate_save(self.h, None, 0, C.byref(n)))
        buf = (C.c_ubyte * n.value)()
        _check_s(lib().ms_surrogate_save(self.h, buf, n.value, C.byref(n)))
        with open(path, "wb") as f:
            f.write(bytes(buf))

    def load(self, path):
        """Read a blob written by save() (same layer sizes)."""
        with open(path, "rb") as f:
            data = f.read()
        buf = (C.c_ubyte * len(data)).from_buffer_copy(data)
        _check_s(lib().ms_surrogate_load(self.h, buf, len(data)))

    def train(self, n_samples=10_000_000, batch=8192, iters=1, lr0=1e-2, lr1=1e-5, seed=41,
              norm_samples=8192, norm_seed=40, step0=0, loss=None, stream=None):
        """ms_surrogate_train: Adam on exact labels of sampled poses with a
        cosine learning-rate decay; the output standardisation first when
        norm_samples > 0. loss: device float32 [iters] or None."""
        c = MsTrainCfg(int(n_samples), int(batch), int(iters), int(step0), int(norm_samples),
                       float(lr0), float(lr1), int(seed), int(norm_seed),
                       _dp(loss).value if loss is not None else None)
        _check_s(lib().ms_surrogate_train(self.model.h, self.h, C.byref(c), _stream(stream)))

    def sample(self, q, seed, offset=0, stream=None):
        _check_s(lib().ms_surrogate_sample(self.h, q.shape[0], seed, offset, _dp(q), _stream(stream)))

    def forward(self, q, L, r, stream=None):
        _check_s(lib().ms_surrogate_forward(self.h, q.shape[0], _dp(q), _dp(L), _dp(r),
                                            _stream(stream)))

    def reserve(self, n):
        _check_s(lib().ms_surrogate_reserve(self.h, int(n)))

    def forward_noalloc(self, q, L, r, stream=None):
        _check_s(lib().ms_surrogate_forward_noalloc(self.h, q.shape[0], _dp(q), _dp(L), _dp(r),
                                                    _stream(stream)))

    def noalloc_max(self):
        return int(lib().ms_surrogate_noalloc_max(self.h))

    def train_step(self, q, L, r, lr, step, loss=None, stream=None):
        _check_s(lib().ms_surrogate_train_step(self.h, q.shape[0], _dp(q), _dp(L), _dp(r),
                                               float(lr), int(step), _dp(loss), _stream(stream)))


def _check_b(rc):
    if rc != 0:
        raise MsError(rc, lib().ms_batch_last_error().decode())


class Batch:
    """Envs of several models stepped together (one graph launch per call).

    states: per model a tuple (q, qd, act, status) of device tensors;
    excitations: per model a dict of Model.rollout's excitation arguments
    (kind, u, seed, step0, x, ar1)."""

    def __init__(self, models, n_env):
        L = lib()
        self.models = list(models)
        self.n_env = [int(n) for n in n_env]
        arr = (C.c_void_p * len(self.models))(*[m.h for m in self.models])
        ne = np.asarray(self.n_env, np.int32)
        h = C.c_void_p()
        _check_b(L.ms_batch_create(arr, ne.ctypes.data_as(_iptr), len(self.models), C.byref(h)))
        self.h = h

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ms_batch_destroy(self.h)
        except Exception:
            pass

    def _args(self, states, excitations):
        n = len(self.models)
        st = (MsBatchState * n)()
        ex = (MsExc * n)()
        for i, ((q, qd, act, status), e) in enumerate(zip(states, excitations)):
            st[i] = MsBatchState(_dp(q), _dp(qd), _dp(act), _dp(status))
            ar1 = e.get("ar1", (0.0, 0.0, 0.0))
            ex[i] = MsExc(e.get("kind", EXC_ARRAY), _dp(e.get("u")), e.get("seed", 0),
                          e.get("step0", 0), _dp(e.get("x")), float(ar1[0]), float(ar1[1]),
                          float(ar1[2]))
        return st, ex

    def rollout(self, states, excitations, n_steps, dt, contact=True, stream=None):
        st, ex = self._args(states, excitations)
        o = MsOpts(dt, int(contact))
        _check_b(lib().ms_batch_rollout(self.h, st, ex, n_steps, C.byref(o), _stream(stream)))

    def autotune(self, states, excitations, n_probe, dt, contact=True, stream=None):
        st, ex = self._args(states, excitations)
        o = MsOpts(dt, int(contact))
        _check_b(lib().ms_batch_autotune(self.h, st, ex, n_probe, C.byref(o), _stream(stream)))
        return self.config()

    def config(self):
        w = np.zeros(len(self.models), np.int32)
        mode = np.zeros(1, np.int32)
        _check_b(lib().ms_batch_config(self.h, w.ctypes.data_as(_iptr), mode.ctypes.data_as(_iptr)))
        return w.tolist(), int(mode[0])

    def set_config(self, env_per_wg, issue_mode=ISSUE_CONCURRENT):
        w = np.asarray(env_per_wg, np.int32)
        _check_b(lib().ms_batch_set_config(self.h, w.ctypes.data_as(_iptr), int(issue_mode)))


class Policy:
    """Random-initialised policy network of the library bound to a Model
    (observations of n_ref synthetic reference targets from ref_seed)."""

    def __init__(self, model: Model, hidden: int = 512, n_ref: int = 140, ref_seed: int = 52,
                 seed: int = 51):
        L = lib()
        self.model = model
        h = C.c_void_p()
        _check_s(L.ms_policy_create(model.h, hidden, n_ref, ref_seed, seed, C.byref(h)))
        self.h = h
        d = np.zeros(4, np.int32)
        _check_s(L.ms_policy_dims(h, d.ctypes.data_as(_iptr)))
        self.n_obs, self.n_in, self.hidden, self.n_out = (int(x) for x in d)
        self.shapes = [(self.hidden, self.n_in), (self.hidden,), (self.hidden, self.hidden),
                       (self.hidden,), (self.n_out, self.hidden), (self.n_out,)]

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ms_policy_destroy(self.h)
        except Exception:
            pass

    def params(self):
        b = [np.zeros(s, np.float32) for s in self.shapes]
        _check_s(lib().ms_policy_params(self.h, 0, *[x.ctypes.data_as(_fptr) for x in b]))
        return b

    def reserve(self, n):
        _check_s(lib().ms_policy_reserve(self.h, int(n)))

    def act(self, q, qd, t, u, env0=0, obs=None, stream=None):
        _check_s(lib().ms_policy_act(self.h, q.shape[0], _dp(q), _dp(qd), float(t), int(env0),
                                     _dp(u), _dp(obs), _stream(stream)))

    def rollout(self, q, qd, act, status, n_steps, decim, dt, contact=True, t0=0.0,
                surrogate=None, tol=1e-4, fb_count=None, u_record=None, stream=None):
        o = MsOpts(dt, int(contact))
        _check_s(lib().ms_policy_rollout(self.model.h, self.h,
                                         surrogate.h if surrogate is not None else None,
                                         q.shape[0], _dp(q), _dp(qd), _dp(act), _dp(status),
                                         n_steps, decim, float(t0), C.byref(o), float(tol),
                                         _dp(fb_count), _dp(u_record), _stream(stream)))


def _check_c(rc):
    if rc != 0:
        raise MsError(rc, lib().ms_controller_last_error().decode())


class Controller:
    """The control step around the physics bound to a Model: observation,
    Gaussian initial sampler refined by a flow velocity field, n_sub
    substeps with the excitations held, discriminator reward (random-init
    networks)."""

    def __init__(self, model: Model, keys, hidden=1024, n_sub=10, flow_steps=20, flow_dt=0.05,
                 sigma0=0.1, ref_seed=52, noise_seed=53, pi_seed=54, flow_seed=55, disc_seed=56):
        L = lib()
        self.model = model
        self._keys = np.ascontiguousarray(keys, np.int32)
        d = MsCtlDesc(int(hidden), int(n_sub), int(flow_steps), float(flow_dt), float(sigma0),
                      len(self._keys), self._keys.ctypes.data, ref_seed, noise_seed, pi_seed,
                      flow_seed, disc_seed)
        h = C.c_void_p()
        _check_c(L.ms_controller_create(model.h, C.byref(d), C.byref(h)))
        self.h = h
        dims = np.zeros(6, np.int32)
        _check_c(L.ms_controller_dims(h, dims.ctypes.data_as(_iptr)))
        self.n_obs, self.n_in, self.n_at, self.n_din, self.hidden, self.n_h = (int(x) for x in dims)
        self.n_sub = int(n_sub)

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().ms_controller_destroy(self.h)
        except Exception:
            pass

    def params(self, which):
        """(W1, b1, W2, b2, W3, b3) of network `which` (0 initial sampler, 1
        flow, 2 discriminator) as float32 [out][in]; plus the flow's (action,
        time) block for which = 1 and log_std for which = 0."""
        nm = self.model.n_mus
        h = self.hidden
        ins = [self.n_in if which < 2 else self.n_din, h, h]
        outs = [h, h, 1 if which == 2 else nm]
        W = [np.zeros((o, i), np.float32) for i, o in zip(ins, outs)]
        b = [np.zeros(o, np.float32) for o in outs]
        wat = np.zeros((h, self.n_at), np.float32) if which == 1 else None
        ls = np.zeros(nm, np.float32) if which == 0 else None
        Wp = (_fptr * 3)(*[x.ctypes.data_as(_fptr) for x in W])
        bp = (_fptr * 3)(*[x.ctypes.data_as(_fptr) for x in b])
        _check_c(lib().ms_controller_params(
            self.h, which, 0, Wp, bp, wat.ctypes.data_as(_fptr) if wat is not None else None,
            ls.ctypes.data_as(_fptr) if ls is not None else None))
        out = [W[0], b[0], W[1], b[1], W[2], b[2]]
        return out, wat, ls

    def reserve(self, n_env):
        _check_c(lib().ms_controller_reserve(self.h, int(n_env)))

    def step(self, q, qd, act, status, mstate, ctl_step, t, dt, reward, contact=True, u_in=None,
             out=None, stream=None):
        """One control step; out: dict of device tensors (obs, a0, u, delta,
        n_applied), each optional."""
        out = out or {}
        o = MsOpts(dt, int(contact))
        co = MsCtlOut(*[_dp(out.get(k)) for k in ("obs", "a0", "u", "delta", "n_applied")])
        _check_c(lib().ms_controller_step(self.h, q.shape[0], _dp(q), _dp(qd), _dp(act),
                                          _dp(status), _dp(mstate), int(ctl_step), float(t),
                                          C.byref(o), _dp(u_in), _dp(reward), C.byref(co),
                                          _stream(stream)))
