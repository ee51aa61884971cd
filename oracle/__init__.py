"""CPU oracle of the MPC-SRD time step: ctypes binding of ``oracle.c``.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` import this package.  It shares no code
with the GPU library and never imports it.

Each wrapper names the part of the paper (arXiv:2406.15236, Sec. II unless
stated) that the C function follows; the C source carries the details.
Lengths are in units of the cell size a.  Position and velocity arrays are
float64 with shape (3, n) (SoA, C-contiguous).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

TAG_SHIFT, TAG_AXIS, TAG_THERMO, TAG_PHANTOM = 1, 2, 3, 4
CELL_FIELDS = ["nfluid", "nphantom", "vx", "vy", "vz", "K", "nx", "ny", "nz",
               "kappa", "Ek", "attempts", "px", "py", "pz", "Kpost"]
CELL_STRIDE = len(CELL_FIELDS)


def build(out: str = LIB_PATH, src: str = _SRC) -> str:
    """Compile the oracle (gcc, -O2 -ffp-contract=off: one IEEE op per written op)."""
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
           "-Wall", "-Wextra", "-I", _HERE, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


class _Params(C.Structure):
    _fields_ = [("L", C.c_int32 * 3), ("walls", C.c_int32), ("mbs", C.c_int32),
                ("amc", C.c_int32), ("fixed", C.c_int32), ("slip", C.c_int32),
                ("h", C.c_double), ("alpha", C.c_double),
                ("kT", C.c_double), ("mass", C.c_double), ("density", C.c_double),
                ("g", C.c_double * 3), ("seed", C.c_uint64), ("uwall", C.c_double),
                ("le_u", C.c_double)]


@dataclass
class Params:
    """One periodic (or z-walled) MPC box.  Lengths in cells, alpha in radians."""
    L: tuple = (16, 16, 16)
    h: float = 0.1
    alpha: float = np.deg2rad(130.0)
    kT: float = 1.0
    mass: float = 1.0
    density: float = 10.0
    seed: int = 1
    mbs: bool = False
    walls: bool = False
    amc: bool = False
    fixed: bool = False
    slip: bool = False
    uwall: float = 0.0
    le_u: float = 0.0
    g: tuple = field(default_factory=lambda: (0.0, 0.0, 0.0))

    def c(self) -> _Params:
        p = _Params()
        p.L[:] = [int(v) for v in self.L]
        p.walls, p.mbs, p.amc = int(self.walls), int(self.mbs), int(self.amc)
        p.fixed = int(self.fixed)
        p.slip = int(self.slip)
        p.uwall = float(self.uwall)
        p.le_u = float(self.le_u)
        p.h, p.alpha, p.kT, p.mass = self.h, self.alpha, self.kT, self.mass
        p.density = self.density
        p.g[:] = [float(v) for v in self.g]
        p.seed = int(self.seed) & 0xFFFFFFFFFFFFFFFF
        return p

    @property
    def ncells(self) -> int:
        lz = self.L[2] + 2 if self.walls else self.L[2]
        return int(self.L[0] * self.L[1] * lz)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or (
                os.path.getmtime(LIB_PATH) < os.path.getmtime(_SRC)):
            build()
        _lib = load(LIB_PATH)
    return _lib


class use_library:
    """Context manager: run the wrappers against another build of the oracle
    (the mutation tests load deliberately broken copies this way)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        lib()
        self.saved = _lib
        _lib = load(self.path)
        return _lib

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved


def load(path: str):
    """Open one build of the oracle and declare its C signatures."""
    L = C.CDLL(path)
    if True:
        P = C.POINTER(_Params)
        u32p, f64p = C.POINTER(C.c_uint32), C.POINTER(C.c_double)
        sig = {
            "orc_philox": (None, [u32p, u32p, u32p]),
            "orc_u24": (C.c_double, [C.c_uint32]),
            "orc_u53": (C.c_double, [C.c_uint32, C.c_uint32]),
            "orc_u53_open": (C.c_double, [C.c_uint32, C.c_uint32]),
            "orc_u32_open": (C.c_double, [C.c_uint32]),
            "orc_shift": (None, [P, C.c_uint64, f64p]),
            "orc_ncells": (C.c_int64, [P]),
            "orc_stream": (C.c_int64, [P, C.c_uint64, C.c_int64, f64p, f64p]),
            "orc_keys": (C.c_int, [P, C.c_uint64, C.c_int64, f64p, u32p]),
            "orc_sort": (None, [C.c_int64, u32p, C.c_int64, u32p, u32p]),
            "orc_wall_fraction": (C.c_double, [P, C.c_double, C.c_int32]),
            "orc_cell_axis": (None, [P, C.c_uint64, C.c_uint32, f64p]),
            "orc_cell_gamma": (C.c_double, [P, C.c_uint64, C.c_uint32, C.c_double,
                                            C.POINTER(C.c_int32)]),
            "orc_phantoms": (C.c_int32, [P, C.c_uint64, C.c_uint32, C.c_double, f64p,
                                         C.c_int32]),
            "orc_rotate": (None, [C.c_double, f64p, f64p, f64p]),
            "orc_collide": (C.c_int, [P, C.c_uint64, C.c_int64, f64p, f64p, u32p, u32p,
                                      C.c_int64, f64p]),
            "orc_reorder": (None, [C.c_int64, f64p, f64p, u32p]),
            "orc_step": (C.c_int, [P, C.c_uint64, C.c_int64, f64p, f64p, C.c_int32,
                                   u32p, u32p, u32p]),
            "orc_observables": (None, [P, C.c_int64, f64p, f64p]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        return L


def _f64(a):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u32(a):
    assert a.dtype == np.uint32 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


def _state(x, v):
    x = np.ascontiguousarray(x, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert x.shape == v.shape and x.shape[0] == 3
    return x, v


# --- random streams ---------------------------------------------------------
def philox(ctr, key):
    """Philox4x32-10 block function (Salmon et al., SC'11)."""
    c = np.asarray(ctr, dtype=np.uint32).copy()
    k = np.asarray(key, dtype=np.uint32).copy()
    out = np.zeros(4, dtype=np.uint32)
    lib().orc_philox(_u32(c), _u32(k), _u32(out))
    return out


def u24(w): return lib().orc_u24(int(w))
def u53(a, b): return lib().orc_u53(int(a), int(b))
def u53_open(a, b): return lib().orc_u53_open(int(a), int(b))
def u32_open(w): return lib().orc_u32_open(int(w))


def shift(p: Params, t: int) -> np.ndarray:
    """Grid shift of step t (Sec. II: lattice shifted before every collision)."""
    s = np.zeros(3)
    lib().orc_shift(C.byref(p.c()), t, _f64(s))
    return s


def cell_axis(p: Params, t: int, key: int) -> np.ndarray:
    n = np.zeros(3)
    lib().orc_cell_axis(C.byref(p.c()), t, key, _f64(n))
    return n


def cell_gamma(p: Params, t: int, key: int, shape: float):
    att = C.c_int32(0)
    g = lib().orc_cell_gamma(C.byref(p.c()), t, key, shape, C.byref(att))
    return g, att.value


def phantoms(p: Params, t: int, key: int, fw: float, max_out: int = 127) -> np.ndarray:
    buf = np.zeros(3 * max_out)
    k = lib().orc_phantoms(C.byref(p.c()), t, key, fw, _f64(buf), max_out)
    return buf[:3 * k].reshape(k, 3)


def wall_fraction(p: Params, sz: float, cz: int) -> float:
    return lib().orc_wall_fraction(C.byref(p.c()), sz, cz)


def rotate(alpha: float, n, u) -> np.ndarray:
    n = np.ascontiguousarray(n, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64)
    out = np.zeros(3)
    lib().orc_rotate(alpha, _f64(n), _f64(u), _f64(out))
    return out


# --- the step, part by part -----------------------------------------------
def stream(p: Params, x, v, t: int = 0):
    """Eq.(1) of step t with periodic wrap (Lees-Edwards offset of time
    (t+1) h) or walls.  Returns (x, v, bounces)."""
    x, v = _state(x, v)
    x, v = x.copy(), v.copy()
    nb = lib().orc_stream(C.byref(p.c()), t, x.shape[1], _f64(x), _f64(v))
    return x, v, int(nb)


def keys(p: Params, t: int, x) -> np.ndarray:
    x = np.ascontiguousarray(x, dtype=np.float64)
    key = np.zeros(x.shape[1], dtype=np.uint32)
    rc = lib().orc_keys(C.byref(p.c()), t, x.shape[1], _f64(x), _u32(key))
    if rc != 0:
        raise ValueError("position outside the box or not finite")
    return key


def sort(key, ncell: int):
    key = np.ascontiguousarray(key, dtype=np.uint32)
    perm = np.zeros(key.size, dtype=np.uint32)
    offset = np.zeros(ncell + 1, dtype=np.uint32)
    lib().orc_sort(key.size, _u32(key), ncell, _u32(perm), _u32(offset))
    return perm, offset


def collide(p: Params, t: int, v, perm, offset, cells: bool = False, x=None):
    """Eq.(2) + MBS (or Eqs. 3-4, SRD+a, which reads the streamed positions x)
    on streamed velocities v (3, n).  Returns v' [, cell table]."""
    v = np.ascontiguousarray(v, dtype=np.float64).copy()
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    offset = np.ascontiguousarray(offset, dtype=np.uint32)
    ncell = offset.size - 1
    co = np.zeros(ncell * CELL_STRIDE) if cells else None
    xp = None
    if x is not None:
        x = np.ascontiguousarray(x, dtype=np.float64)
        xp = _f64(x)
    rc = lib().orc_collide(C.byref(p.c()), t, v.shape[1], xp, _f64(v), _u32(perm),
                           _u32(offset), ncell, _f64(co) if cells else None)
    if rc == -3:
        raise ValueError("a fixed-point summand is outside |x| < 2^37")
    if rc != 0:
        raise ValueError("SRD+a and Lees-Edwards need positions; SRD+a is defined for "
                         "periodic boxes, Lees-Edwards for periodic boxes without SRD+a")
    if cells:
        return v, co.reshape(ncell, CELL_STRIDE)
    return v


def reorder(x, v, perm):
    x, v = _state(x, v)
    x, v = x.copy(), v.copy()
    lib().orc_reorder(x.shape[1], _f64(x), _f64(v), _u32(np.ascontiguousarray(perm, np.uint32)))
    return x, v


def step(p: Params, t: int, x, v, reorder: bool = False, binning: bool = False):
    """One full step t -> t+1.  Returns (x, v) or (x, v, key, perm, offset)."""
    x, v = _state(x, v)
    x, v = x.copy(), v.copy()
    n = x.shape[1]
    key = np.zeros(n, dtype=np.uint32)
    perm = np.zeros(n, dtype=np.uint32)
    offset = np.zeros(p.ncells + 1, dtype=np.uint32)
    rc = lib().orc_step(C.byref(p.c()), t, n, _f64(x), _f64(v), int(bool(reorder)),
                        _u32(key), _u32(perm), _u32(offset))
    if rc == -2:
        raise ValueError("SRD+a is defined for periodic boxes")
    if rc == -3:
        raise ValueError("a fixed-point summand is outside |x| < 2^37")
    if rc != 0:
        raise ValueError("position outside the box or not finite")
    if binning:
        return x, v, key, perm, offset
    return x, v


def run(p: Params, x, v, steps: int, t0: int = 0, reorder_every: int = 0):
    """Advance `steps` steps; reorder after step t when (t+1) % R == 0."""
    for t in range(t0, t0 + steps):
        ro = reorder_every > 0 and (t + 1) % reorder_every == 0
        x, v = step(p, t, x, v, reorder=ro)
    return x, v


def observables(p: Params, v) -> dict:
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(6)
    lib().orc_observables(C.byref(p.c()), v.shape[1], _f64(v), _f64(out))
    return {"P": out[:3].copy(), "E": out[3], "T": out[4], "N": int(out[5])}
