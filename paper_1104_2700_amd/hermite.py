"""Thin ctypes binding of libhermite (include/hermite.h).

Argument marshalling only: every stage of the hot path runs in the HIP
library.  Device memory comes from torch tensors on the GPU (their
``data_ptr()``); streams are torch's current stream unless one is given.
Importing this module loads ``libhermite.so`` and raises if it is missing --
there is no fallback.

Method names are the C entry points without the ``hermite_`` prefix
(``Context.force_jerk`` calls ``hermite_force_jerk``); the module-level
``lib`` exposes the raw C functions under their own names.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhermite.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        "libhermite.so is not built; run `python -m paper_1104_2700_amd.build` "
        "(no CPU fallback exists)")

lib = ctypes.CDLL(LIB_PATH)

OK, EINVAL, ENODEV, EHIP, ENOMEM, ENONFINITE, ENOTSUP = 0, -1, -2, -3, -4, -5, -6
FP64, MIXED, MIXED_2F, MIXED_SP = 0, 1, 2, 3
DT_PAPER, DT_AARSETH = 0, 1
PRECISIONS = {"fp64": FP64, "mixed": MIXED, "mixed2f": MIXED_2F, "mixed_sp": MIXED_SP}
INT64_MAX = (1 << 63) - 1

_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_d = ctypes.c_double


class CState(ctypes.Structure):
    _fields_ = [("n", _i64), ("tick_bits", _i32), ("reserved0", _i32),
                ("m", _P), ("x", _P), ("v", _P), ("a", _P), ("j", _P),
                ("xp", _P), ("vp", _P), ("pot", _P), ("t", _P), ("dt", _P)]


class CDtParams(ctypes.Structure):
    _fields_ = [("eta", _d), ("form", _i32), ("k_min", _i32), ("k_max", _i32),
                ("reserved0", _i32), ("eta_init", _d)]


class CClusters(ctypes.Structure):
    _fields_ = [("n_clusters", _i32), ("reserved0", _i32), ("max_size", _i64),
                ("offsets", _P), ("eps2", _P)]


class CTuning(ctypes.Structure):
    _fields_ = [("target_lanes", _i32), ("wg_per_cu", _i32),
                ("min_j_per_lane", _i32), ("variant", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_PS, _PD, _PC, _PT = (ctypes.POINTER(CState), ctypes.POINTER(CDtParams),
                      ctypes.POINTER(CClusters), ctypes.POINTER(CTuning))

_SIGS = {
    "hermite_create": ([ctypes.c_int, ctypes.POINTER(_P)]),
    "hermite_destroy": ([_P]),
    "hermite_sync": ([_P, _P]),
    "hermite_select_block": ([_P, _PS, _P, _P, _P, _i64, _P]),
    "hermite_predict": ([_P, _PS, _P, _i64, _P, _P]),
    "hermite_force_jerk": ([_P, _PS, _PC, _P, _P, _i32, _d, ctypes.c_int, _P, _P, _P, _P]),
    "hermite_force_jerk_timed": ([_P, _PS, _PC, _P, _i32, _d, ctypes.c_int, _P, _P, _P, _i32,
                                  ctypes.POINTER(_d), _P]),
    "hermite_force_jerk_noalloc": ([_PS, _PC, _P, _P, _i32, _d, ctypes.c_int, _P, _P, _P, _P]),
    "hermite_correct": ([_P, _PS, _P, _P, _i32, _P, _i64, _P, _P, _P, _PD, _P, _P]),
    "hermite_init_dt": ([_P, _PS, _PD, _P]),
    "hermite_check_finite": ([_P, _PS, _P]),
    "hermite_initialize": ([_P, _PS, _PC, _d, ctypes.c_int, _PD, _P]),
    "hermite_energy": ([_P, _PS, _PC, _d, _P, _P]),
    "hermite_step": ([_P, _PS, _PC, _d, ctypes.c_int, _PD, _i64, ctypes.c_int, _P]),
    "hermite_run": ([_P, _PS, _PC, _d, ctypes.c_int, _PD, _i64, ctypes.c_int, _i32, _i64,
                     ctypes.POINTER(_i64), ctypes.POINTER(_i64), ctypes.POINTER(_i32), _P]),
    "hermite_counters": ([_P, ctypes.POINTER(_i64), _P]),
    "hermite_block_histogram": ([_P, ctypes.POINTER(_i64), _P]),
    "hermite_get_tuning": ([_P, ctypes.c_int, _PT]),
    "hermite_set_mixed_policy": ([_P, ctypes.c_int, _d, _i64]),
    "hermite_get_mixed_policy": ([_P, ctypes.c_int, ctypes.POINTER(_d), ctypes.POINTER(_i64)]),
    "hermite_set_mixed_small_blocks": ([_P, ctypes.c_int, _i64]),
    "hermite_get_mixed_small_blocks": ([_P, ctypes.c_int, ctypes.POINTER(_i64)]),
    "hermite_set_tuning": ([_P, ctypes.c_int, _PT]),
    "hermite_autotune": ([_P, _PS, _PC, _d, ctypes.c_int, _i32, ctypes.c_char_p, _P]),
    "hermite_load_tuning": ([_P, ctypes.c_char_p, ctypes.c_int, _i64, _i32]),
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = ctypes.c_int
lib.hermite_last_error.argtypes = []
lib.hermite_last_error.restype = ctypes.c_char_p


NOALLOC_MAX_ACTIVE = 65536
NOALLOC_MAX_CLUSTERS = 1024


class HermiteError(RuntimeError):
    def __init__(self, code, func):
        msg = lib.hermite_last_error().decode(errors="replace")
        super().__init__("%s failed (%d): %s" % (func, code, msg))
        self.code = code


def _check(rc, func):
    if rc != OK:
        raise HermiteError(rc, func)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def force_jerk_noalloc(s, idx, eps2, precision, acc, jerk, pot=None, n_act_dev=None,
                       n_act_max=None, clusters=None, stream=None):
    """hermite_force_jerk_noalloc: the force sweep with no context and no
    allocation (outputs must be given)."""
    if n_act_max is None:
        n_act_max = s.n if idx is None else int(idx.shape[0])
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    _check(lib.hermite_force_jerk_noalloc(ctypes.byref(s.c()), _cl(clusters), _ptr(idx),
                                          _ptr(n_act_dev), int(n_act_max), float(eps2),
                                          int(precision), _ptr(acc), _ptr(jerk), _ptr(pot),
                                          _stream(stream)), "hermite_force_jerk_noalloc")
    return acc, jerk, pot


class State:
    """Device state of n particles (SoA tensors on ``device``).

    ``x, v, a, j, xp, vp``: float64 (3, n); ``m, pot``: float64 (n,);
    ``t, dt``: int64 (n,) in ticks of 2**-tick_bits.
    """

    def __init__(self, x, v, m, tick_bits=20, device="cuda"):
        dev = torch.device(device)
        f64 = dict(dtype=torch.float64, device=dev)
        self.x = torch.as_tensor(x, **f64).contiguous().clone()
        self.v = torch.as_tensor(v, **f64).contiguous().clone()
        self.m = torch.as_tensor(m, **f64).contiguous().clone()
        n = self.m.shape[0]
        if self.x.shape != (3, n) or self.v.shape != (3, n):
            raise ValueError("x and v must have shape (3, n)")
        self.n = n
        self.tick_bits = int(tick_bits)
        self.a = torch.zeros(3, n, **f64)
        self.j = torch.zeros(3, n, **f64)
        self.xp = torch.zeros(3, n, **f64)
        self.vp = torch.zeros(3, n, **f64)
        self.pot = torch.zeros(n, **f64)
        self.t = torch.zeros(n, dtype=torch.int64, device=dev)
        self.dt = torch.zeros(n, dtype=torch.int64, device=dev)

    def c(self):
        """The hermite_state view of these tensors (pointers, no copies)."""
        s = CState()
        s.n, s.tick_bits = self.n, self.tick_bits
        for k in ("m", "x", "v", "a", "j", "xp", "vp", "pot", "t", "dt"):
            setattr(s, k, getattr(self, k).data_ptr())
        return s

    def clone(self):
        o = State.__new__(State)
        o.n, o.tick_bits = self.n, self.tick_bits
        for k in ("m", "x", "v", "a", "j", "xp", "vp", "pot", "t", "dt"):
            setattr(o, k, getattr(self, k).clone())
        return o

    def copy_from(self, other):
        for k in ("m", "x", "v", "a", "j", "xp", "vp", "pot", "t", "dt"):
            getattr(self, k).copy_(getattr(other, k))

    def to_numpy(self):
        d = {k: getattr(self, k).cpu().numpy() for k in
             ("m", "x", "v", "a", "j", "xp", "vp", "pot", "t", "dt")}
        d["tick_bits"] = self.tick_bits
        return d


class Clusters:
    """Independent clusters: ``offsets`` (C+1,) and per-cluster ``eps2`` (C,)."""

    def __init__(self, offsets, eps2, device="cuda"):
        self.offsets = torch.as_tensor(offsets, dtype=torch.int64, device=device).contiguous()
        self.eps2 = torch.as_tensor(eps2, dtype=torch.float64, device=device).contiguous()
        off = self.offsets.cpu()
        self.n_clusters = int(off.shape[0] - 1)
        self.max_size = int((off[1:] - off[:-1]).max())
        if self.eps2.shape[0] != self.n_clusters:
            raise ValueError("eps2 must have one entry per cluster")

    def c(self):
        c = CClusters()
        c.n_clusters, c.max_size = self.n_clusters, self.max_size
        c.offsets, c.eps2 = self.offsets.data_ptr(), self.eps2.data_ptr()
        return c


def dt_params(eta=0.02, form=DT_PAPER, k_min=3, k_max=20, eta_init=0.0):
    """eta_init: start-up factor of init_dt (0 = the steady factor)."""
    return CDtParams(float(eta), int(form), int(k_min), int(k_max), 0, float(eta_init))


def _cl(clusters):
    return None if clusters is None else ctypes.byref(clusters.c())


class Context:
    """A libhermite context on one HIP device (hermite_create/destroy)."""

    def __init__(self, device=0):
        h = ctypes.c_void_p()
        _check(lib.hermite_create(int(device), ctypes.byref(h)), "hermite_create")
        self.h = h
        self.device = torch.device("cuda", device)

    def close(self):
        if self.h:
            lib.hermite_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- hot path -------------------------------------------------------
    def select_block(self, s: State, idx_out, n_act_dev, T_dev, T_end=INT64_MAX, stream=None):
        _check(lib.hermite_select_block(self.h, ctypes.byref(s.c()), _ptr(idx_out),
                                        _ptr(n_act_dev), _ptr(T_dev), int(T_end),
                                        _stream(stream)), "hermite_select_block")

    def predict(self, s: State, T_dev=None, T_host=0, n_act_dev=None, stream=None):
        _check(lib.hermite_predict(self.h, ctypes.byref(s.c()), _ptr(T_dev), int(T_host),
                                   _ptr(n_act_dev), _stream(stream)), "hermite_predict")

    def force_jerk(self, s: State, idx, eps2, precision=FP64, n_act_dev=None,
                   n_act_max=None, acc=None, jerk=None, pot=None, clusters=None,
                   stream=None):
        """Returns (acc (3, n_act_max), jerk (3, n_act_max), pot (n_act_max,))."""
        if n_act_max is None:
            n_act_max = s.n if idx is None else int(idx.shape[0])
        f64 = dict(dtype=torch.float64, device=s.x.device)
        acc = torch.empty(3, n_act_max, **f64) if acc is None else acc
        jerk = torch.empty(3, n_act_max, **f64) if jerk is None else jerk
        pot = torch.empty(n_act_max, **f64) if pot is None else pot
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        _check(lib.hermite_force_jerk(self.h, ctypes.byref(s.c()), _cl(clusters), _ptr(idx),
                                      _ptr(n_act_dev), int(n_act_max), float(eps2),
                                      int(precision), _ptr(acc), _ptr(jerk), _ptr(pot),
                                      _stream(stream)), "hermite_force_jerk")
        return acc, jerk, pot

    def force_jerk_timed(self, s: State, idx, eps2, precision=FP64, reps=10, acc=None,
                         jerk=None, pot=None, clusters=None, stream=None):
        """Runs the sweep ``reps`` times with HIP events around its phases on
        the launch stream; returns (acc, jerk, pot, ms) where ms holds the
        average milliseconds of the plan kernel, the sweep kernel(s), the
        finishing kernels and the whole call."""
        n_act = s.n if idx is None else int(idx.shape[0])
        f64 = dict(dtype=torch.float64, device=s.x.device)
        acc = torch.empty(3, n_act, **f64) if acc is None else acc
        jerk = torch.empty(3, n_act, **f64) if jerk is None else jerk
        pot = torch.empty(n_act, **f64) if pot is None else pot
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        ms = (ctypes.c_double * 4)()
        _check(lib.hermite_force_jerk_timed(self.h, ctypes.byref(s.c()), _cl(clusters), _ptr(idx),
                                            n_act, float(eps2), int(precision), _ptr(acc),
                                            _ptr(jerk), _ptr(pot), int(reps), ms,
                                            _stream(stream)), "hermite_force_jerk_timed")
        return acc, jerk, pot, {"plan": ms[0], "sweep": ms[1], "finish": ms[2], "total": ms[3]}

    def correct(self, s: State, idx, acc, jerk, pot, params, T_dev=None, T_host=0,
                n_act_dev=None, n_act_max=None, crit_out=None, stream=None):
        if n_act_max is None:
            n_act_max = s.n if idx is None else int(idx.shape[0])
        _check(lib.hermite_correct(self.h, ctypes.byref(s.c()), _ptr(idx), _ptr(n_act_dev),
                                   int(n_act_max), _ptr(T_dev), int(T_host), _ptr(acc),
                                   _ptr(jerk), _ptr(pot), ctypes.byref(params),
                                   _ptr(crit_out), _stream(stream)), "hermite_correct")

    def init_dt(self, s: State, params, stream=None):
        _check(lib.hermite_init_dt(self.h, ctypes.byref(s.c()), ctypes.byref(params),
                                   _stream(stream)), "hermite_init_dt")

    def initialize(self, s: State, eps2, params, precision=FP64, clusters=None, stream=None):
        _check(lib.hermite_initialize(self.h, ctypes.byref(s.c()), _cl(clusters),
                                      float(eps2), int(precision), ctypes.byref(params),
                                      _stream(stream)), "hermite_initialize")

    def energy(self, s: State, eps2, clusters=None, out=None, stream=None):
        """Returns a device tensor [C, 2] of (K, W) per cluster ([1, 2] if single)."""
        C = 1 if clusters is None else clusters.n_clusters
        if out is None:
            out = torch.empty(C, 2, dtype=torch.float64, device=s.x.device)
        _check(lib.hermite_energy(self.h, ctypes.byref(s.c()), _cl(clusters), float(eps2),
                                  _ptr(out), _stream(stream)), "hermite_energy")
        return out

    # -- steps and runs -----------------------------------------------------
    def step(self, s: State, eps2, params, precision=FP64, T_end=INT64_MAX,
             use_graph=False, clusters=None, stream=None):
        _check(lib.hermite_step(self.h, ctypes.byref(s.c()), _cl(clusters), float(eps2),
                                int(precision), ctypes.byref(params), int(T_end),
                                int(bool(use_graph)), _stream(stream)), "hermite_step")

    def run(self, s: State, eps2, params, T_end, precision=FP64, use_graph=True,
            sync_every=64, clusters=None, max_steps=0, stream=None, with_done=False):
        """Integrate to T_end ticks (or max_steps launched steps); returns
        (block steps, interactions) and, with ``with_done``, whether every
        particle reached T_end.  Raises HermiteError with ENONFINITE for a
        non-finite state, or EHIP if the block selection reports a timed-out
        workgroup wait or an inconsistent step-size order."""
        steps, inter, done = _i64(0), _i64(0), _i32(0)
        _check(lib.hermite_run(self.h, ctypes.byref(s.c()), _cl(clusters), float(eps2),
                               int(precision), ctypes.byref(params), int(T_end),
                               int(bool(use_graph)), int(sync_every), int(max_steps),
                               ctypes.byref(steps), ctypes.byref(inter), ctypes.byref(done),
                               _stream(stream)), "hermite_run")
        if with_done:
            return steps.value, inter.value, bool(done.value)
        return steps.value, inter.value

    def block_histogram(self, stream=None):
        """Block steps per active-size bin: [0] n_act = 0, [b] 2^(b-1) <= n_act < 2^b."""
        out = (_i64 * 33)()
        _check(lib.hermite_block_histogram(self.h, out, _stream(stream)),
               "hermite_block_histogram")
        return list(out)

    def check_finite(self, s: State, stream=None):
        """True when every x, v, a, j value is finite (synchronises)."""
        rc = lib.hermite_check_finite(self.h, ctypes.byref(s.c()), _stream(stream))
        if rc == ENONFINITE:
            return False
        _check(rc, "hermite_check_finite")
        return True

    def counters(self, stream=None):
        out = (_i64 * 6)()
        _check(lib.hermite_counters(self.h, out, _stream(stream)), "hermite_counters")
        return dict(zip(("steps", "interactions", "clamped", "T", "n_act", "refined"),
                        list(out)))

    def sync(self, stream=None):
        _check(lib.hermite_sync(self.h, _stream(stream)), "hermite_sync")

    # -- tuning -------------------------------------------------------------
    def get_tuning(self, precision=FP64):
        t = CTuning()
        _check(lib.hermite_get_tuning(self.h, int(precision), ctypes.byref(t)),
               "hermite_get_tuning")
        return t

    def set_mixed_policy(self, precision, near_factor, fp64_below):
        _check(lib.hermite_set_mixed_policy(self.h, int(precision), float(near_factor),
                                            int(fp64_below)), "hermite_set_mixed_policy")

    def get_mixed_policy(self, precision):
        """Returns (near_factor, fp64_below)."""
        f, b = _d(0.0), _i64(0)
        _check(lib.hermite_get_mixed_policy(self.h, int(precision), ctypes.byref(f),
                                            ctypes.byref(b)), "hermite_get_mixed_policy")
        return f.value, b.value

    def set_mixed_small_blocks(self, precision, fp64_inter_below):
        _check(lib.hermite_set_mixed_small_blocks(self.h, int(precision), int(fp64_inter_below)),
               "hermite_set_mixed_small_blocks")

    def get_mixed_small_blocks(self, precision):
        """Interactions below which a mixed sweep is done in FP64."""
        b = _i64(0)
        _check(lib.hermite_get_mixed_small_blocks(self.h, int(precision), ctypes.byref(b)),
               "hermite_get_mixed_small_blocks")
        return b.value

    def set_tuning(self, precision, tuning: CTuning):
        _check(lib.hermite_set_tuning(self.h, int(precision), ctypes.byref(tuning)),
               "hermite_set_tuning")

    def autotune(self, s: State, eps2, precision=FP64, n_act=None, cache_path=None,
                 clusters=None, stream=None):
        """Times launch shapes at s.xp/s.vp and installs the fastest valid one."""
        n_act = s.n if n_act is None else int(n_act)
        path = None if cache_path is None else str(cache_path).encode()
        _check(lib.hermite_autotune(self.h, ctypes.byref(s.c()), _cl(clusters), float(eps2),
                                    int(precision), n_act, path, _stream(stream)),
               "hermite_autotune")
        return self.get_tuning(precision)

    def load_tuning(self, cache_path, precision, n, n_act):
        rc = lib.hermite_load_tuning(self.h, str(cache_path).encode(), int(precision),
                                     int(n), int(n_act))
        return rc == OK
