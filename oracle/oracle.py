"""Plain FP64 CPU oracle for the fourth-order Hermite block-timestep scheme.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this module.  The product
library never calls it, and it shares no code with the GPU path: the
arithmetic lives in ``hermite_oracle.c`` (gcc, -O2 -ffp-contract=off, no
fast-math, Neumaier-compensated ascending-j sums) and this file only moves
numpy arrays in and out and runs the integration procedure in the paper's
order (Section 2, procedure steps 1-9).

State dictionaries use SoA arrays: ``x, v, a, j`` of shape (3, n) float64,
``m`` (n,), ``pot`` (n,), ``t, dt`` (n,) int64 ticks of 2**-tick_bits.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hermite_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Integer codes of the two readings of the Aarseth criterion.
FORM_PAPER = 0     # dt = eta * sqrt(R), as the timestep equation is printed
FORM_AARSETH = 1   # dt = sqrt(eta * R), the classic form


def build(force: bool = False) -> str:
    """Compile the oracle shared library with gcc (strict IEEE binary64)."""
    if (not force and os.path.exists(_LIB)
            and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC)):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    compile_source(_SRC, tmp)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def configure(lib):
    """Declares the C signatures on a loaded oracle library; returns it."""
    d, i64, i32 = ctypes.c_double, ctypes.c_int64, ctypes.c_int
    P = ctypes.c_void_p
    lib.oracle_force.argtypes = [i64, P, P, P, i64, P, d, i64, i64, P, P, P, P]
    lib.oracle_force.restype = None
    lib.oracle_predict.argtypes = [i64, P, P, P, P, P, i64, i32, P, P]
    lib.oracle_predict.restype = None
    lib.oracle_select.argtypes = [i64, P, P, P, P]
    lib.oracle_select.restype = i64
    lib.oracle_aarseth.argtypes = [P, P, P, P, d, i32]
    lib.oracle_aarseth.restype = d
    lib.oracle_quantize.argtypes = [d, i32, i64, i32, i32, i32, P, P]
    lib.oracle_quantize.restype = i64
    lib.oracle_correct.argtypes = ([i64, i64, P, i64, i32] + [P] * 5
                                   + [P] * 7 + [d, i32, i32, i32, P])
    lib.oracle_correct.restype = i64
    lib.oracle_init_dt.argtypes = [i64, P, P, P, P, i32, d, i32, d, i32, i32]
    lib.oracle_init_dt.restype = i64
    lib.oracle_energy.argtypes = [i64, P, P, P, d, P, P, P, P, P, P]
    lib.oracle_energy.restype = None
    lib.oracle_threads.argtypes = [i32]
    lib.oracle_threads.restype = i32
    return lib


def threads(n=0):
    """Sets the oracle's thread count (n >= 1) and returns the count in
    effect; the results do not depend on it (the j order is fixed)."""
    return int(_L().oracle_threads(int(n)))


def compile_source(src_path, out_path):
    """Compiles an oracle C source with the oracle's flags (strict IEEE)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c11", "-Wall", "-o", out_path, src_path, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


def _L():
    global _lib
    if _lib is None:
        _lib = configure(ctypes.CDLL(build()))
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def force(x, v, m, idx, eps2, j_range=None, with_cond=False):
    """Equations (acc), (jrk), (pot) for the particles listed in ``idx``.

    Sums over j in ``j_range`` (default all), excluding j == i.
    Returns ``acc (3, n_act)``, ``jerk (3, n_act)``, ``pot (n_act,)`` and,
    if ``with_cond``, ``cond (3, n_act)`` = sum_j |a_ij|, |jrk_ij|, |phi_ij|.
    """
    x, v, m = _f64(x), _f64(v), _f64(m)
    n = m.shape[0]
    assert x.shape == (3, n) and v.shape == (3, n)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    na = idx.shape[0]
    jb, je = (0, n) if j_range is None else j_range
    acc = np.zeros((3, na)); jrk = np.zeros((3, na)); pot = np.zeros(na)
    cond = np.zeros((3, na)) if with_cond else None
    if na:
        _L().oracle_force(n, _p(x), _p(v), _p(m), na, _p(idx), float(eps2),
                          int(jb), int(je), _p(acc), _p(jrk), _p(pot),
                          _p(cond) if with_cond else None)
    if with_cond:
        return acc, jrk, pot, cond
    return acc, jrk, pot


def predict(x, v, a, j, t, T, tick_bits):
    """Equations (xpred), (vpred) for every particle; dt_i = (T - t_i) ticks."""
    x, v, a, j = _f64(x), _f64(v), _f64(a), _f64(j)
    t = np.ascontiguousarray(t, dtype=np.int64)
    n = t.shape[0]
    xp = np.empty((3, n)); vp = np.empty((3, n))
    _L().oracle_predict(n, _p(x), _p(v), _p(a), _p(j), _p(t), int(T),
                        int(tick_bits), _p(xp), _p(vp))
    return xp, vp


def select(t, dt):
    """Procedure step 1: block time T and the ascending active list."""
    t = np.ascontiguousarray(t, dtype=np.int64)
    dt = np.ascontiguousarray(dt, dtype=np.int64)
    n = t.shape[0]
    idx = np.empty(n, dtype=np.int32)
    T = np.zeros(1, dtype=np.int64)
    na = _L().oracle_select(n, _p(t), _p(dt), _p(T), _p(idx))
    return int(T[0]), idx[:na].copy()


def aarseth(a, j, s, c, eta, form=FORM_PAPER):
    """Equation (timestep) before quantisation, for one particle."""
    a, j, s, c = (_f64(q) for q in (a, j, s, c))
    return _L().oracle_aarseth(_p(a), _p(j), _p(s), _p(c), float(eta), int(form))


def quantize(dt_crit, k_old, T, tick_bits, k_min, k_max):
    """Power-of-two quantisation; returns (dt_ticks, k, clamped)."""
    k = ctypes.c_int(0); cl = ctypes.c_int(0)
    dt = _L().oracle_quantize(float(dt_crit), int(k_old), int(T), int(tick_bits),
                              int(k_min), int(k_max), ctypes.byref(k),
                              ctypes.byref(cl))
    return int(dt), k.value, cl.value


def init_dt(state, eta, form, k_min, k_max, eta_init=0.0):
    """First step sizes eta_s |a|/|j| (t_i = 0; eta_s = eta_init, or the
    steady factor eta / sqrt(eta) when eta_init is 0); returns the
    clamped count."""
    n = state["m"].shape[0]
    return int(_L().oracle_init_dt(n, _p(state["a"]), _p(state["j"]),
                                   _p(state["t"]), _p(state["dt"]),
                                   int(state["tick_bits"]), float(eta), int(form),
                                   float(eta_init), int(k_min), int(k_max)))


def correct(state, idx, T, xp, vp, acc1, jrk1, pot1, eta, form, k_min, k_max,
            crit_out=None):
    """Procedure steps 5-8 for the active list, in place; returns #clamped.

    ``crit_out`` (optional float64 array of length n_act) receives the
    criterion of eq. (timestep) before quantisation.
    """
    n = state["m"].shape[0]
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    acc1, jrk1, pot1 = _f64(acc1), _f64(jrk1), _f64(pot1)
    xp, vp = _f64(xp), _f64(vp)
    return int(_L().oracle_correct(
        n, idx.shape[0], _p(idx), int(T), int(state["tick_bits"]),
        _p(xp), _p(vp), _p(acc1), _p(jrk1), _p(pot1),
        _p(state["x"]), _p(state["v"]), _p(state["a"]), _p(state["j"]),
        _p(state["pot"]), _p(state["t"]), _p(state["dt"]),
        float(eta), int(form), int(k_min), int(k_max),
        _p(crit_out) if crit_out is not None else None))


def energy(x, v, m, eps2):
    """K = 1/2 sum m v^2 and W = 1/2 sum m phi (FP64 potential sweep)."""
    x, v, m = _f64(x), _f64(v), _f64(m)
    n = m.shape[0]
    K = np.zeros(1); W = np.zeros(1)
    phi = np.empty(n); idx = np.empty(n, dtype=np.int32)
    a = np.empty((3, n)); j = np.empty((3, n))
    _L().oracle_energy(n, _p(x), _p(v), _p(m), float(eps2), _p(K), _p(W),
                       _p(phi), _p(idx), _p(a), _p(j))
    return float(K[0]), float(W[0])


def new_state(x, v, m, tick_bits):
    """A state dictionary holding copies of the initial conditions."""
    n = np.asarray(m).shape[0]
    return {
        "x": _f64(x).copy(), "v": _f64(v).copy(), "m": _f64(m).copy(),
        "a": np.zeros((3, n)), "j": np.zeros((3, n)), "pot": np.zeros(n),
        "t": np.zeros(n, dtype=np.int64), "dt": np.zeros(n, dtype=np.int64),
        "tick_bits": int(tick_bits),
    }


def initialize(state, eps2, eta, form, k_min, k_max, eta_init=0.0):
    """t = 0: a full sweep gives a0, j0, pot; then the first step sizes."""
    n = state["m"].shape[0]
    acc, jrk, pot = force(state["x"], state["v"], state["m"],
                          np.arange(n, dtype=np.int32), eps2)
    state["a"][...] = acc
    state["j"][...] = jrk
    state["pot"][...] = pot
    return init_dt(state, eta, form, k_min, k_max, eta_init)


def block_step(state, eps2, eta, form, k_min, k_max, T_end=None):
    """One pass of procedure steps 1-8 (Section 2).

    Returns ``(T, n_act, n_clamped)``; if the next block time is past
    ``T_end`` nothing is changed and ``n_act`` is 0.
    """
    T, idx = select(state["t"], state["dt"])                      # step 1
    if T_end is not None and T > T_end:
        return T, 0, 0
    xp, vp = predict(state["x"], state["v"], state["a"], state["j"],
                     state["t"], T, state["tick_bits"])           # steps 2-3
    acc1, jrk1, pot1 = force(xp, vp, state["m"], idx, eps2)       # step 4
    ncl = correct(state, idx, T, xp, vp, acc1, jrk1, pot1,
                  eta, form, k_min, k_max)                        # steps 5-8
    return T, idx.shape[0], ncl


def run(state, T_end, eps2, eta, form, k_min, k_max, init=True):
    """Integrate until every particle sits at ``T_end`` ticks (step 9 loop).

    Returns a dict with the block-step count, interaction count
    (n_act * n per block step) and clamped-step count.
    """
    n = state["m"].shape[0]
    stats = {"steps": 0, "interactions": 0, "clamped": 0}
    if init:
        stats["clamped"] += initialize(state, eps2, eta, form, k_min, k_max)
        stats["interactions"] += n * n
    while True:
        T, na, ncl = block_step(state, eps2, eta, form, k_min, k_max, T_end)
        if na == 0:
            break
        stats["steps"] += 1
        stats["interactions"] += na * n
        stats["clamped"] += ncl
        if T == T_end:
            break
    return stats
