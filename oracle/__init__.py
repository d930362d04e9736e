"""Serial FP64 CPU oracle for the D2V16 MRT finite-difference LB step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``.  The product package never
imports it.  The arithmetic lives in ``mrtfd_oracle.c`` (plain C, double
precision, one node at a time, in the order the paper states the method);
this module only marshals numpy arrays through ctypes.

Parameters are passed as the plain dict produced by
``paper_1305_4736_amd.workloads`` (grid, rates, b, limiter, boundary kinds
and states); fields are ``(ny, nx)`` arrays with x fastest and ``f`` is
``(16, ny, nx)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mrtfd_oracle.c")
_LIB = os.path.join(_HERE, "libmrtfd_oracle.so")

LIMITERS = {"mc": 0, "minmod": 1, "lw": 2, "upwind": 3}
BC_KINDS = {"periodic": 0, "equilibrium": 1, "outflow": 2, "wall": 3}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, no intrinsics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int), ("ny", ctypes.c_int),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
        ("eta0", ctypes.c_double),
        ("s", ctypes.c_double * 16),
        ("b", ctypes.c_double),
        ("limiter", ctypes.c_int), ("correction", ctypes.c_int),
        ("bc_kind", ctypes.c_int * 4),
        ("bc_state", (ctypes.c_double * 4) * 4),
    ]


_lib = None


def open_library(path: str):
    """Open a build of mrtfd_oracle.c (the default one, or a variant the
    tests compile with a planted mistake to check that the pins catch it)."""
    lib = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    pp = ctypes.POINTER(_Params)
    lib.orc_constants.argtypes = [ctypes.c_double, dp, dp, dp, dp]
    lib.orc_feq_hat.argtypes = [ctypes.c_double] * 5 + [dp]
    lib.orc_feq.argtypes = [ctypes.c_double] * 6 + [dp]
    lib.orc_init.argtypes = [pp, dp, dp, dp, dp, dp]
    lib.orc_advance.argtypes = [pp, dp, ctypes.c_long]
    lib.orc_macros.argtypes = [pp, dp, dp, dp, dp, dp]
    lib.orc_noneq.argtypes = [pp, dp, ctypes.c_int, dp]
    assert lib.orc_sizeof_params() == ctypes.sizeof(_Params)
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = open_library(_LIB)
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _c_params(p: dict) -> _Params:
    c = _Params()
    c.nx, c.ny = int(p["nx"]), int(p["ny"])
    c.dx, c.dy, c.dt = float(p["dx"]), float(p["dy"]), float(p["dt"])
    c.eta0 = float(p.get("eta0", 2.5))
    for k in range(16):
        c.s[k] = float(p["s"][k])
    c.b = float(p["b"])
    c.limiter = LIMITERS[p.get("limiter", "mc")]
    c.correction = 1 if p.get("correction", True) else 0
    for side in range(4):
        bc = p["bc"][side]
        c.bc_kind[side] = BC_KINDS[bc["kind"]]
        st = bc.get("state", (1.0, 0.0, 0.0, 1.0))
        for q in range(4):
            c.bc_state[side][q] = float(st[q])
    return c


def _check(rc, what):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


def constants(eta0: float = 2.5):
    """Velocities (2, 16), M (16, 16), M^-1 (16, 16) and A (16,)."""
    lib = _load()
    v = np.zeros(32)
    M = np.zeros(256)
    Mi = np.zeros(256)
    A = np.zeros(16)
    _check(lib.orc_constants(eta0, _dp(v), _dp(M), _dp(Mi), _dp(A)), "constants")
    return v.reshape(2, 16), M.reshape(16, 16), Mi.reshape(16, 16), A


def feq_hat(rho, jx, jy, e, b):
    out = np.zeros(16)
    _check(_load().orc_feq_hat(rho, jx, jy, e, b, _dp(out)), "feq_hat")
    return out


def feq(rho, ux, uy, T, b, eta0=2.5):
    out = np.zeros(16)
    _check(_load().orc_feq(eta0, b, rho, ux, uy, T, _dp(out)), "feq")
    return out


def _field(a, ny, nx):
    a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx)))
    return a


def init(p: dict, rho, ux, uy, T) -> np.ndarray:
    """f = f^eq(rho, u, T) at every node, then the boundary fill."""
    ny, nx = int(p["ny"]), int(p["nx"])
    args = [_field(a, ny, nx) for a in (rho, ux, uy, T)]
    f = np.zeros((16, ny, nx))
    cp = _c_params(p)
    _check(_load().orc_init(ctypes.byref(cp), *[_dp(a) for a in args], _dp(f)), "init")
    return f


def advance(p: dict, f: np.ndarray, nsteps: int) -> np.ndarray:
    """Return f after ``nsteps`` explicit stages (input is not modified)."""
    ny, nx = int(p["ny"]), int(p["nx"])
    out = np.ascontiguousarray(np.array(f, dtype=np.float64).reshape(16, ny, nx))
    cp = _c_params(p)
    _check(_load().orc_advance(ctypes.byref(cp), _dp(out), int(nsteps)), "advance")
    return out


def run(p: dict, rho, ux, uy, T, nsteps: int) -> np.ndarray:
    return advance(p, init(p, rho, ux, uy, T), nsteps)


def macros(p: dict, f: np.ndarray):
    """(rho, ux, uy, T), each (ny, nx)."""
    ny, nx = int(p["ny"]), int(p["nx"])
    f = np.ascontiguousarray(f, dtype=np.float64)
    outs = [np.zeros((ny, nx)) for _ in range(4)]
    cp = _c_params(p)
    _check(_load().orc_macros(ctypes.byref(cp), _dp(f), *[_dp(o) for o in outs]), "macros")
    return tuple(outs)


def noneq(p: dict, f: np.ndarray, star: bool = False) -> np.ndarray:
    """Delta (star=False) or Delta* (star=True), shape (16, ny, nx)."""
    ny, nx = int(p["ny"]), int(p["nx"])
    f = np.ascontiguousarray(f, dtype=np.float64)
    out = np.zeros((16, ny, nx))
    cp = _c_params(p)
    _check(_load().orc_noneq(ctypes.byref(cp), _dp(f), 1 if star else 0, _dp(out)), "noneq")
    return out
