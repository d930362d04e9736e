"""Python binding of the C ABI in include/mrtfd.h (argument marshalling only).

Every step of the method runs in the gfx950 kernels of ``libmrtfd.so``; this
module converts a parameter dict (see ``workloads``) into ``mrtfd_params``,
passes numpy arrays as host pointers or torch CUDA tensors as device
pointers, and raises on any non-zero status.  There is no fallback: if the
library has not been built the import fails.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MRTFD_LIBRARY selects another build of the same library (e.g. a tuning variant)
LIB_PATH = os.environ.get("MRTFD_LIBRARY") or os.path.join(_HERE, "libmrtfd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build it with `python -m paper_1305_4736_amd.build` "
        "(there is no CPU fallback)")

# The library needs a HIP runtime (libamdhip64.so.7).  PyTorch ships its own
# under that name; load it first when it is installed, so that the process
# holds one HIP runtime that both use (a second copy would bring its own
# device contexts and streams).
try:
    import torch  # noqa: F401
except ImportError:
    pass

_lib = ctypes.CDLL(LIB_PATH)

LIMITERS = {"mc": 0, "minmod": 1, "lw": 2, "upwind": 3}
BC_KINDS = {"periodic": 0, "equilibrium": 1, "outflow": 2, "wall": 3}
PRECISIONS = {"fp64": 0, "fp32": 1}

OK, EINVAL, ENOMEM, EDEVICE, ENONFINITE, ESTATE = 0, -1, -2, -3, -4, -5


class MRTFDError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class NonFiniteError(MRTFDError):
    pass


class _Bc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("rho", ctypes.c_double), ("ux", ctypes.c_double),
                ("uy", ctypes.c_double), ("T", ctypes.c_double)]


class _Params(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dt", ctypes.c_double),
                ("eta0", ctypes.c_double), ("s", ctypes.c_double * 16), ("b", ctypes.c_double),
                ("limiter", ctypes.c_int), ("precision", ctypes.c_int),
                ("energy_flux_correction", ctypes.c_int), ("bc", _Bc * 4)]


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_H = ctypes.c_void_p
_lib.mrtfd_create.argtypes = [ctypes.POINTER(_Params), _vp, ctypes.POINTER(_H)]
_lib.mrtfd_footprint.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_size_t)]
_lib.mrtfd_init.argtypes = [_H, _vp, _vp, _vp, _vp, ctypes.c_int]
_lib.mrtfd_step.argtypes = [_H, ctypes.c_long]
_lib.mrtfd_step_timed.argtypes = [_H, ctypes.c_long, _dp]
_lib.mrtfd_set_steps_per_launch.argtypes = [_H, ctypes.c_int]
_lib.mrtfd_get_steps_per_launch.argtypes = [_H, ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_macros.argtypes = [_H, _vp, _vp, _vp, _vp, ctypes.c_int]
_lib.mrtfd_noneq.argtypes = [_H, ctypes.c_int, _vp, ctypes.c_int]
_lib.mrtfd_get_f.argtypes = [_H, _vp, ctypes.c_int]
_lib.mrtfd_set_f.argtypes = [_H, _vp, ctypes.c_int]
_lib.mrtfd_state_planes.argtypes = [_H, ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_get_state.argtypes = [_H, _vp, ctypes.c_int]
_lib.mrtfd_set_state.argtypes = [_H, _vp, ctypes.c_int]
_lib.mrtfd_sync.argtypes = [_H]
_lib.mrtfd_steps_done.argtypes = [_H]
_lib.mrtfd_steps_done.restype = ctypes.c_long
_lib.mrtfd_destroy.argtypes = [_H]
_lib.mrtfd_last_error.restype = ctypes.c_char_p
_lib.mrtfd_constants.argtypes = [ctypes.c_double, _dp, _dp]


def _check(rc: int):
    if rc != OK:
        msg = _lib.mrtfd_last_error().decode()
        raise (NonFiniteError if rc == ENONFINITE else MRTFDError)(rc, msg)


def c_params(p: dict) -> _Params:
    c = _Params()
    c.nx, c.ny = int(p["nx"]), int(p["ny"])
    c.dx, c.dy, c.dt = float(p["dx"]), float(p["dy"]), float(p["dt"])
    c.eta0 = float(p.get("eta0", 2.5))
    for k in range(16):
        c.s[k] = float(p["s"][k])
    c.b = float(p["b"])
    c.limiter = LIMITERS[p.get("limiter", "mc")]
    c.precision = PRECISIONS[p.get("precision", "fp64")]
    c.energy_flux_correction = 1 if p.get("correction", True) else 0
    for side in range(4):
        bc = p["bc"][side]
        st = bc.get("state", (1.0, 0.0, 0.0, 1.0))
        c.bc[side] = _Bc(BC_KINDS[bc["kind"]], *[float(v) for v in st])
    return c


def footprint(p: dict) -> int:
    out = ctypes.c_size_t(0)
    _check(_lib.mrtfd_footprint(ctypes.byref(c_params(p)), ctypes.byref(out)))
    return int(out.value)


_lib.mrtfd_device_memory.argtypes = [ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)]


def device_memory():
    """(free, total) device memory in bytes."""
    fr, tot = ctypes.c_size_t(0), ctypes.c_size_t(0)
    _check(_lib.mrtfd_device_memory(ctypes.byref(fr), ctypes.byref(tot)))
    return int(fr.value), int(tot.value)


_lib.mrtfd_solve_noalloc.argtypes = [ctypes.POINTER(_Params), _vp, _vp, _vp, _vp, _vp, ctypes.c_long,
                                     _vp, _vp, _vp, _vp]


def solve_noalloc(params: dict, rho, ux, uy, T, nsteps: int, out=None, stream=None):
    """One whole solve with no device allocation (mrtfd_solve_noalloc): device
    tensors in, (rho, ux, uy, T) device tensors out (written into ``out``
    when given).  Asynchronous on `stream` (default: torch's current one)."""
    import torch
    nx, ny = int(params["nx"]), int(params["ny"])
    ins = [_ptr(a, (ny, nx)) for a in (rho, ux, uy, T)]
    if any(d != 1 for _, d, _ in ins):
        raise ValueError("solve_noalloc takes device tensors")
    if out is None:
        out = tuple(torch.empty((ny, nx), dtype=torch.float64, device=rho.device) for _ in range(4))
    outs = [_ptr(a, (ny, nx), writable=True) if a is not None else (None, 1, None) for a in out]
    if stream is None:
        stream = _default_stream()
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    cp = c_params(params)
    _check(_lib.mrtfd_solve_noalloc(ctypes.byref(cp), _vp(int(stream)), *[_vp(p[0]) for p in ins], int(nsteps),
                                    *[_vp(p[0]) if p[0] else None for p in outs]))
    return out


_lib.mrtfd_clock_stamp.argtypes = [_vp, _vp]


def clock_stamp(out, index: int = 0, stream=None):
    """Enqueue a stamp (per XCD: shader-clock cycles, 100 MHz ticks) into row
    `index` of ``out``, an (n, 16) int64 CUDA tensor (zeroed beforehand), on
    `stream` (default: torch's current stream)."""
    if stream is None:
        stream = _default_stream()
    elif hasattr(stream, "cuda_stream"):
        stream = stream.cuda_stream
    if (not _is_device(out) or out.dim() != 2 or out.shape[1] != 16 or out.element_size() != 8
            or not out.is_contiguous() or not 0 <= index < out.shape[0]):
        raise ValueError("out must be a contiguous (n, 16) 64-bit CUDA tensor and index within it")
    _check(_lib.mrtfd_clock_stamp(_vp(int(stream)), _vp(out.data_ptr() + 128 * int(index))))


def clock_mhz(stamps, i0: int = 0, i1: int = 1) -> float:
    """Average core clock (MHz) between two stamps (rows of the (n, 16) array
    read back to the host): the mean over the XCDs that both stamps reached."""
    vals = []
    for x in range(8):
        c0, r0 = stamps[i0][2 * x], stamps[i0][2 * x + 1]
        c1, r1 = stamps[i1][2 * x], stamps[i1][2 * x + 1]
        if r0 > 0 and r1 > r0 and c1 > c0:
            vals.append((c1 - c0) / ((r1 - r0) / 100.0))
    return sum(vals) / len(vals) if vals else float("nan")


def constants(eta0: float = 2.5):
    """Dense M and M^-1 as the kernels apply them (host-only)."""
    M = np.zeros(256)
    Mi = np.zeros(256)
    _check(_lib.mrtfd_constants(eta0, M.ctypes.data_as(_dp), Mi.ctypes.data_as(_dp)))
    return M.reshape(16, 16), Mi.reshape(16, 16)


def _is_device(a) -> bool:
    return hasattr(a, "is_cuda") and bool(a.is_cuda)


def _ptr(a, shape, writable=False):
    """(pointer, on_device, keepalive) for a numpy array or a CUDA tensor."""
    if a is None:
        return None, 0, None
    if _is_device(a):
        import torch
        if a.dtype != torch.float64 or not a.is_contiguous() or tuple(a.shape) != tuple(shape):
            raise ValueError(f"device tensor must be contiguous float64 of shape {shape}")
        return a.data_ptr(), 1, a
    arr = np.asarray(a)
    if writable:
        if arr.dtype != np.float64 or not arr.flags.c_contiguous or arr.shape != tuple(shape):
            raise ValueError(f"host output must be contiguous float64 of shape {shape}")
    else:
        arr = np.ascontiguousarray(np.broadcast_to(arr.astype(np.float64, copy=False), shape))
    return arr.ctypes.data, 0, arr


def _default_stream():
    try:
        import torch
        if torch.cuda.is_available():
            return torch.cuda.current_stream().cuda_stream
    except Exception:
        pass
    return 0


class Solver:
    """One MRT-FD simulation resident on the GPU."""

    def __init__(self, params: dict, stream=None):
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        if stream is None:
            stream = _default_stream()
        elif hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        self.stream = int(stream)
        self._h = _H()
        self._cp = c_params(params)
        _check(_lib.mrtfd_create(ctypes.byref(self._cp), _vp(self.stream), ctypes.byref(self._h)))

    # -- lifecycle ------------------------------------------------------------
    def close(self):
        if self._h:
            _lib.mrtfd_destroy(self._h)
            self._h = _H()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- the path -------------------------------------------------------------
    def init(self, rho, ux, uy, T):
        shp = (self.ny, self.nx)
        ptrs = [_ptr(a, shp) for a in (rho, ux, uy, T)]
        dev = {p[1] for p in ptrs}
        if len(dev) != 1:
            raise ValueError("mix of host and device inputs")
        _check(_lib.mrtfd_init(self._h, *[_vp(p[0]) for p in ptrs], dev.pop()))
        return self

    def step(self, nsteps: int = 1):
        _check(_lib.mrtfd_step(self._h, int(nsteps)))
        return self

    def step_timed(self, nsteps: int) -> float:
        ms = ctypes.c_double(0.0)
        _check(_lib.mrtfd_step_timed(self._h, int(nsteps), ctypes.byref(ms)))
        return ms.value

    @property
    def steps_per_launch(self) -> int:
        """Steps one kernel launch takes: 2 (fused pairs) or 1."""
        k = ctypes.c_int()
        _check(_lib.mrtfd_get_steps_per_launch(self._h, ctypes.byref(k)))
        return k.value

    @steps_per_launch.setter
    def steps_per_launch(self, k: int):
        _check(_lib.mrtfd_set_steps_per_launch(self._h, int(k)))

    def sync(self):
        _check(_lib.mrtfd_sync(self._h))
        return self

    @property
    def steps_done(self) -> int:
        return int(_lib.mrtfd_steps_done(self._h))

    # -- outputs --------------------------------------------------------------
    def macros(self, out=None):
        """(rho, ux, uy, T) as numpy arrays, or written into ``out`` (4
        device tensors / host arrays, any may be None)."""
        shp = (self.ny, self.nx)
        if out is None:
            out = tuple(np.zeros(shp) for _ in range(4))
        ptrs = [_ptr(a, shp, writable=True) for a in out]
        dev = {p[1] for p in ptrs if p[2] is not None}
        on_dev = dev.pop() if dev else 0
        _check(_lib.mrtfd_macros(self._h, *[_vp(p[0]) if p[0] else None for p in ptrs], on_dev))
        return out

    def noneq(self, star: bool = False, out=None):
        shp = (16, self.ny, self.nx)
        if out is None:
            out = np.zeros(shp)
        p, dev, _ = _ptr(out, shp, writable=True)
        _check(_lib.mrtfd_noneq(self._h, 1 if star else 0, _vp(p), dev))
        return out

    def get_f(self, out=None):
        shp = (16, self.ny, self.nx)
        if out is None:
            out = np.zeros(shp)
        p, dev, _ = _ptr(out, shp, writable=True)
        _check(_lib.mrtfd_get_f(self._h, _vp(p), dev))
        return out

    def set_f(self, f):
        p, dev, keep = _ptr(f, (16, self.ny, self.nx))
        _check(_lib.mrtfd_set_f(self._h, _vp(p), dev))
        return self

    @property
    def state_planes(self) -> int:
        """Planes of the bitwise checkpoint: 16, or 20 in FP32 storage."""
        k = ctypes.c_int()
        _check(_lib.mrtfd_state_planes(self._h, ctypes.byref(k)))
        return k.value

    def get_state(self, out=None):
        """The stored state, bit for bit, as (state_planes, ny, nx) doubles."""
        shp = (self.state_planes, self.ny, self.nx)
        if out is None:
            out = np.zeros(shp)
        p, dev, _ = _ptr(out, shp, writable=True)
        _check(_lib.mrtfd_get_state(self._h, _vp(p), dev))
        return out

    def set_state(self, state):
        p, dev, keep = _ptr(state, (self.state_planes, self.ny, self.nx))
        _check(_lib.mrtfd_set_state(self._h, _vp(p), dev))
        return self


# ----------------------------------------------------------------------------
# Batched form

_B = ctypes.c_void_p
_lib.mrtfd_batch_create.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, ctypes.POINTER(_B)]
_lib.mrtfd_batch_destroy.argtypes = [_B]
_lib.mrtfd_batch_add.argtypes = [_B, ctypes.POINTER(_Params), _vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_long,
                                 ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_batch_remove.argtypes = [_B, ctypes.c_int]
_lib.mrtfd_batch_set_steps.argtypes = [_B, ctypes.c_int, ctypes.c_long]
_lib.mrtfd_batch_step.argtypes = [_B, ctypes.c_long]
_lib.mrtfd_batch_set_steps_per_launch.argtypes = [_B, ctypes.c_int]
_lib.mrtfd_batch_get_steps_per_launch.argtypes = [_B, ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_batch_step_timed.argtypes = [_B, ctypes.c_long, _dp]
_lib.mrtfd_batch_steps_done.argtypes = [_B, ctypes.c_int]
_lib.mrtfd_batch_steps_done.restype = ctypes.c_long
_lib.mrtfd_batch_remaining.argtypes = [_B, ctypes.c_int, ctypes.POINTER(ctypes.c_long)]
_lib.mrtfd_batch_rounds.argtypes = [_B, ctypes.POINTER(ctypes.c_long), ctypes.POINTER(ctypes.c_long)]
_lib.mrtfd_batch_pair_rows.argtypes = [_B, ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_batch_macros.argtypes = [_B, ctypes.c_int, _vp, _vp, _vp, _vp, ctypes.c_int]
_lib.mrtfd_batch_get_f.argtypes = [_B, ctypes.c_int, _vp, ctypes.c_int]
_lib.mrtfd_batch_set_f.argtypes = [_B, ctypes.c_int, _vp, ctypes.c_int]
_lib.mrtfd_batch_status.argtypes = [_B, ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_batch_sync.argtypes = [_B]
_lib.mrtfd_batch_shape.argtypes = [_B, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
_lib.mrtfd_batch_autotune.argtypes = [_B, _dp]
_lib.mrtfd_batch_set_shape.argtypes = [_B, ctypes.c_int, ctypes.c_int]

# shape classes of a batch slot (see Batch.set_shape)
SHAPE_CLASSES = {"tile32x8": 0, "tile64x4": 1, "tile128x2": 2, "row256": 3, "strips": 4}


class Batch:
    """Many independent instances advanced together (one precision and one
    limiter per batch)."""

    def __init__(self, capacity: int, precision: str = "fp64", limiter: str = "mc", stream=None):
        if stream is None:
            stream = _default_stream()
        elif hasattr(stream, "cuda_stream"):
            stream = stream.cuda_stream
        self.stream = int(stream)
        self.capacity = int(capacity)
        self.precision, self.limiter = precision, limiter
        self._b = _B()
        self._shapes = {}
        _check(_lib.mrtfd_batch_create(self.capacity, PRECISIONS[precision], LIMITERS[limiter],
                                       _vp(self.stream), ctypes.byref(self._b)))

    def close(self):
        if self._b:
            _lib.mrtfd_batch_destroy(self._b)
            self._b = _B()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def add(self, params: dict, rho, ux, uy, T, nsteps: int = -1) -> int:
        p = dict(params, precision=self.precision, limiter=self.limiter)
        cp = c_params(p)
        shp = (int(p["ny"]), int(p["nx"]))
        ptrs = [_ptr(a, shp) for a in (rho, ux, uy, T)]
        dev = {q[1] for q in ptrs}
        if len(dev) != 1:
            raise ValueError("mix of host and device inputs")
        slot = ctypes.c_int(-1)
        _check(_lib.mrtfd_batch_add(self._b, ctypes.byref(cp), *[_vp(q[0]) for q in ptrs], dev.pop(),
                                    int(nsteps), ctypes.byref(slot)))
        self._shapes[slot.value] = shp
        return slot.value

    def remove(self, slot: int):
        _check(_lib.mrtfd_batch_remove(self._b, int(slot)))
        self._shapes.pop(slot, None)

    def set_steps(self, slot: int, nsteps: int):
        _check(_lib.mrtfd_batch_set_steps(self._b, int(slot), int(nsteps)))

    def step(self, nsteps: int = 1):
        _check(_lib.mrtfd_batch_step(self._b, int(nsteps)))
        return self

    @property
    def steps_per_launch(self) -> int:
        """2: slots that can take two steps per launch in two-step rounds; 1: one."""
        k = ctypes.c_int()
        _check(_lib.mrtfd_batch_get_steps_per_launch(self._b, ctypes.byref(k)))
        return k.value

    @steps_per_launch.setter
    def steps_per_launch(self, k: int):
        _check(_lib.mrtfd_batch_set_steps_per_launch(self._b, int(k)))

    def step_timed(self, nsteps: int) -> float:
        ms = ctypes.c_double(0.0)
        _check(_lib.mrtfd_batch_step_timed(self._b, int(nsteps), ctypes.byref(ms)))
        return ms.value

    def steps_done(self, slot: int) -> int:
        return int(_lib.mrtfd_batch_steps_done(self._b, int(slot)))

    def remaining(self, slot: int) -> int:
        r = ctypes.c_long(0)
        _check(_lib.mrtfd_batch_remaining(self._b, int(slot), ctypes.byref(r)))
        return int(r.value)

    def rounds(self):
        """(one-step rounds, two-step rounds) run so far (diagnostics)."""
        one, two = ctypes.c_long(0), ctypes.c_long(0)
        _check(_lib.mrtfd_batch_rounds(self._b, ctypes.byref(one), ctypes.byref(two)))
        return int(one.value), int(two.value)

    def pair_rows(self) -> int:
        """Band height of the two-step launches as last fitted to the load
        (diagnostics)."""
        rows = ctypes.c_int(0)
        _check(_lib.mrtfd_batch_pair_rows(self._b, ctypes.byref(rows)))
        return int(rows.value)

    def macros(self, slot: int, out=None):
        shp = self._shapes[slot]
        if out is None:
            out = tuple(np.zeros(shp) for _ in range(4))
        ptrs = [_ptr(a, shp, writable=True) for a in out]
        dev = {q[1] for q in ptrs if q[2] is not None}
        on_dev = dev.pop() if dev else 0
        _check(_lib.mrtfd_batch_macros(self._b, int(slot), *[_vp(q[0]) if q[0] else None for q in ptrs], on_dev))
        return out

    def get_f(self, slot: int, out=None):
        shp = (16,) + self._shapes[slot]
        if out is None:
            out = np.zeros(shp)
        p, dev, _ = _ptr(out, shp, writable=True)
        _check(_lib.mrtfd_batch_get_f(self._b, int(slot), _vp(p), dev))
        return out

    def set_f(self, slot: int, f):
        p, dev, keep = _ptr(f, (16,) + self._shapes[slot])
        _check(_lib.mrtfd_batch_set_f(self._b, int(slot), _vp(p), dev))

    def status(self):
        """Per-slot non-finite flags (numpy int array); raises NonFiniteError
        (with .flags) if any slot was flagged since the last check."""
        flags = np.zeros(self.capacity, dtype=np.int32)
        rc = _lib.mrtfd_batch_status(self._b, flags.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
        if rc == ENONFINITE:
            err = NonFiniteError(rc, _lib.mrtfd_last_error().decode())
            err.flags = flags
            raise err
        _check(rc)
        return flags

    def sync(self):
        _check(_lib.mrtfd_batch_sync(self._b))
        return self

    def shape(self, slot: int):
        tx, ty = ctypes.c_int(0), ctypes.c_int(0)
        _check(_lib.mrtfd_batch_shape(self._b, int(slot), ctypes.byref(tx), ctypes.byref(ty)))
        return tx.value, ty.value

    def set_shape(self, slot: int, shape):
        """Force a slot into a shape class (a name of SHAPE_CLASSES or its
        index); the state is kept and every class gives the same result."""
        k = SHAPE_CLASSES[shape] if isinstance(shape, str) else int(shape)
        _check(_lib.mrtfd_batch_set_shape(self._b, int(slot), k))
        return self

    def autotune(self):
        """Measured device time per work unit (microseconds) of the shape
        classes tile32x8, tile64x4, tile128x2, row256, strips (a unit is a
        tile, or a strip row with its bands' halo rows); every slot then gets
        its cheapest class."""
        c = np.zeros(len(SHAPE_CLASSES))
        _check(_lib.mrtfd_batch_autotune(self._b, c.ctypes.data_as(_dp)))
        return c
