"""MI355X (gfx950) MPC-SRD library: Python binding of the C ABI in include/mpc.h.

The binding only marshals arguments: every step of the MPC step runs in the
HIP kernels of ``libmpc355.so``.  PyTorch provides the device workspace (a
uint8 tensor) and the HIP stream.  If the library is missing, importing works
but every call raises: there is no CPU fallback.

Function names mirror the C ABI (``mpc_create`` -> ``create`` etc.); the
``Sim`` class bundles a handle with its workspace.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

from .build import LIB

FP64, FP32, SPLIT32 = 0, 1, 2
MBS, WALLS_Z, AMC, FIXED_SUMS, SLIP = 1, 2, 4, 8, 16
FORMS = {"fp64": FP64, "fp32": FP32, "split": SPLIT32}
MAX_CELL_PARTICLES = 256

OK, EINVAL, ENOSPACE, ERANGE, EHIP, ESTATE = 0, -1, -2, -3, -4, -5


class MPCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


class Params(C.Structure):
    _fields_ = [("L", C.c_int32 * 3), ("form", C.c_int32), ("flags", C.c_uint32),
                ("reorder_every", C.c_int32), ("a", C.c_double), ("density", C.c_double),
                ("dt", C.c_double), ("alpha", C.c_double), ("kT", C.c_double),
                ("mass", C.c_double), ("g", C.c_double * 3), ("seed", C.c_uint64),
                ("wall_u", C.c_double), ("le_u", C.c_double)]


class Obs(C.Structure):
    _fields_ = [("step", C.c_uint64), ("n", C.c_uint64), ("P", C.c_double * 3),
                ("E", C.c_double), ("T", C.c_double), ("mass_total", C.c_double)]


class KernelTimes(C.Structure):
    _fields_ = [("scan_ms", C.c_double), ("scatter_ms", C.c_double),
                ("collide_ms", C.c_double), ("prologue_ms", C.c_double),
                ("other_ms", C.c_double), ("scan_launches", C.c_uint64),
                ("scatter_launches", C.c_uint64), ("collide_launches", C.c_uint64),
                ("prologue_launches", C.c_uint64)]


SYMBOLS = ["mpc_workspace_bytes", "mpc_create", "mpc_init_state", "mpc_step",
           "mpc_step_profiled", "mpc_set_graph", "mpc_sync", "mpc_observables",
           "mpc_box_info", "mpc_get_step", "mpc_set_step", "mpc_set_state", "mpc_get_state",
           "mpc_get_particles",
           "mpc_get_binning", "mpc_autotune", "mpc_set_tiling", "mpc_get_tiling", "mpc_destroy",
           "mpc_strerror",
           "mpc_last_error", "mpc_probe_copy", "mpc_probe_read", "mpc_run_noalloc"]

_lib = None


def lib():
    """Load libmpc355.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: build it with "
                               "`python -m paper_2406_15236_amd.build` (no CPU fallback)")
        L = C.CDLL(LIB)
        vp, u32p, f64p = C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_double)
        P = C.POINTER(Params)
        sig = {
            "mpc_workspace_bytes": (C.c_int, [P, C.c_int32, C.POINTER(C.c_size_t)]),
            "mpc_create": (C.c_int, [P, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]),
            "mpc_init_state": (C.c_int, [vp, C.c_uint64]),
            "mpc_step": (C.c_int, [vp, C.c_int64]),
            "mpc_step_profiled": (C.c_int, [vp, C.c_int64, C.POINTER(KernelTimes)]),
            "mpc_set_graph": (C.c_int, [vp, C.c_int32]),
            "mpc_sync": (C.c_int, [vp]),
            "mpc_observables": (C.c_int, [vp, C.c_int32, C.POINTER(Obs)]),
            "mpc_box_info": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int64),
                                       C.POINTER(C.c_int64)]),
            "mpc_get_step": (C.c_int, [vp, C.POINTER(C.c_uint64)]),
            "mpc_set_step": (C.c_int, [vp, C.c_uint64]),
            "mpc_set_state": (C.c_int, [vp, C.c_int32, f64p, f64p, C.c_int64]),
            "mpc_get_state": (C.c_int, [vp, C.c_int32, f64p, f64p, C.c_int64]),
            "mpc_get_particles": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int64), C.c_int64,
                                            f64p, f64p]),
            "mpc_get_binning": (C.c_int, [vp, C.c_int32, u32p, u32p, u32p]),
            "mpc_autotune": (C.c_int, [vp, C.c_int32, C.POINTER(C.c_int32),
                                       C.POINTER(C.c_int32)]),
            "mpc_set_tiling": (C.c_int, [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32]),
            "mpc_get_tiling": (C.c_int, [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                         C.POINTER(C.c_int64)]),
            "mpc_destroy": (C.c_int, [vp]),
            "mpc_probe_copy": (C.c_int, [vp, vp, C.c_size_t, C.c_int32, vp]),
            "mpc_run_noalloc": (C.c_int, [P, vp, vp, C.c_int64, C.c_uint64, C.c_int64, vp]),
            "mpc_probe_read": (C.c_int, [vp, C.c_size_t, vp, C.c_size_t, C.c_int32, vp]),
            "mpc_strerror": (C.c_char_p, [C.c_int]),
            "mpc_last_error": (C.c_char_p, [vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype, fn.argtypes = res, args
        _lib = L
    return _lib


def _check(rc: int, handle=None):
    if rc != 0:
        L = lib()
        msg = L.mpc_strerror(rc).decode()
        if handle is not None:
            detail = L.mpc_last_error(handle).decode()
            if detail:
                msg += ": " + detail
        raise MPCError(rc, msg)


def run_noalloc(params, x_ptr: int, v_ptr: int, n: int, step: int, nsteps: int,
                stream_ptr: int):
    """Advance one FP64 box in place in caller-owned device arrays x[3][n],
    v[3][n] with the library's static scratch (no device allocation)."""
    _check(lib().mpc_run_noalloc(C.byref(params), x_ptr, v_ptr, n, step, nsteps, stream_ptr))


def probe_copy(dst_ptr: int, src_ptr: int, nbytes: int, grid: int, stream_ptr: int):
    """Enqueue the HBM copy probe (device pointers)."""
    _check(lib().mpc_probe_copy(dst_ptr, src_ptr, nbytes, grid, stream_ptr))


def probe_read(src_ptr: int, nbytes: int, out_ptr: int, out_bytes: int, grid: int,
               stream_ptr: int):
    """Enqueue the HBM read probe (device pointers)."""
    _check(lib().mpc_probe_read(src_ptr, nbytes, out_ptr, out_bytes, grid, stream_ptr))


def make_params(box: dict, form="fp64", flags: int | None = None, reorder_every: int = 0,
                a: float = 1.0) -> Params:
    """mpc_params from a box description (keys as in synth.config / batch_boxes)."""
    p = Params()
    p.L[:] = [int(v) for v in box["L"]]
    p.form = FORMS[form] if isinstance(form, str) else int(form)
    if flags is None:
        flags = ((MBS if box.get("mbs") else 0) | (WALLS_Z if box.get("walls") else 0)
                 | (AMC if box.get("amc") else 0) | (FIXED_SUMS if box.get("fixed") else 0)
                 | (SLIP if box.get("slip") else 0))
    p.flags = int(flags)
    p.reorder_every = int(reorder_every)
    p.a = float(box.get("a", a))
    p.density = float(box.get("density", 10.0))
    p.dt = float(box.get("h", box.get("dt", 0.1)))
    p.alpha = float(box.get("alpha", math.radians(130.0)))
    p.kT = float(box.get("kT", 1.0))
    p.mass = float(box.get("mass", 1.0))
    p.g[:] = [float(v) for v in box.get("g", (0.0, 0.0, 0.0))]
    p.seed = int(box.get("seed", 1)) & 0xFFFFFFFFFFFFFFFF
    p.wall_u = float(box.get("uwall", 0.0))
    p.le_u = float(box.get("le_u", 0.0))
    return p


def _arr(params):
    if isinstance(params, Params):
        params = [params]
    arr = (Params * len(params))(*params)
    return arr, len(params)


# --- C-ABI mirrors -------------------------------------------------------
def workspace_bytes(params) -> int:
    arr, n = _arr(params)
    out = C.c_size_t(0)
    _check(lib().mpc_workspace_bytes(arr, n, C.byref(out)))
    return int(out.value)


def create(params, workspace_ptr: int, nbytes: int, stream_ptr: int):
    arr, n = _arr(params)
    h = C.c_void_p()
    _check(lib().mpc_create(arr, n, C.c_void_p(workspace_ptr), nbytes,
                            C.c_void_p(stream_ptr), C.byref(h)))
    return h


def _f64(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _u32(a):
    return a.ctypes.data_as(C.POINTER(C.c_uint32))


class Sim:
    """A handle plus the torch-owned device workspace it runs in."""

    def __init__(self, boxes, form="fp64", reorder_every: int = 0, flags: int | None = None,
                 graph: bool = True, device="cuda", a: float = 1.0):
        import torch
        if isinstance(boxes, dict):
            boxes = [boxes]
        self.boxes = boxes
        self.form = form
        self.params = [make_params(b, form, flags, reorder_every, a) for b in boxes]
        self.nbytes = workspace_bytes(self.params)
        self.device = torch.device(device)
        self.workspace = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=self.device)
        self.stream = torch.cuda.current_stream(self.device)
        self.h = create(self.params, self.workspace.data_ptr(), self.nbytes,
                        self.stream.cuda_stream)
        self.set_graph(graph)

    # lifetime
    def close(self):
        if getattr(self, "h", None) is not None:
            _check(lib().mpc_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # calls
    def _c(self, rc):
        _check(rc, self.h)

    def box_info(self, box: int = 0):
        n, c = C.c_int64(0), C.c_int64(0)
        self._c(lib().mpc_box_info(self.h, box, C.byref(n), C.byref(c)))
        return int(n.value), int(c.value)

    def n(self, box: int = 0) -> int:
        return self.box_info(box)[0]

    def init_state(self, seed: int = 1):
        self._c(lib().mpc_init_state(self.h, seed))

    def step(self, nsteps: int = 1):
        self._c(lib().mpc_step(self.h, nsteps))

    def step_profiled(self, nsteps: int, acc: KernelTimes | None = None) -> KernelTimes:
        acc = acc or KernelTimes()
        self._c(lib().mpc_step_profiled(self.h, nsteps, C.byref(acc)))
        return acc

    def set_graph(self, enable):
        """False/0: kernel by kernel; True/1: one-step graph; K > 1: also a
        graph of K consecutive steps."""
        self._c(lib().mpc_set_graph(self.h, int(enable)))

    def sync(self):
        self._c(lib().mpc_sync(self.h))

    def get_step(self) -> int:
        t = C.c_uint64(0)
        self._c(lib().mpc_get_step(self.h, C.byref(t)))
        return int(t.value)

    def set_step(self, t: int):
        self._c(lib().mpc_set_step(self.h, t))

    def observables(self, box: int = 0) -> dict:
        o = Obs()
        self._c(lib().mpc_observables(self.h, box, C.byref(o)))
        return {"step": o.step, "N": o.n, "P": np.array(o.P[:]), "E": o.E, "T": o.T,
                "M": o.mass_total}

    def set_state(self, x, v, box: int = 0):
        x = np.ascontiguousarray(x, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        n = x.shape[1]
        self._c(lib().mpc_set_state(self.h, box, _f64(x), _f64(v), n))

    def get_state(self, box: int = 0):
        n = self.n(box)
        x = np.empty((3, n))
        v = np.empty((3, n))
        self._c(lib().mpc_get_state(self.h, box, _f64(x), _f64(v), n))
        return x, v

    def get_particles(self, idx, box: int = 0):
        """(x, v), each (3, m) FP64: the particles with logical indices idx."""
        idx = np.ascontiguousarray(idx, dtype=np.int64)
        m = idx.size
        x = np.empty((3, m))
        v = np.empty((3, m))
        self._c(lib().mpc_get_particles(self.h, box, idx.ctypes.data_as(C.POINTER(C.c_int64)), m,
                                        _f64(x), _f64(v)))
        return x, v

    def get_binning(self, box: int = 0):
        n, nc = self.box_info(box)
        key = np.empty(n, dtype=np.uint32)
        perm = np.empty(n, dtype=np.uint32)
        off = np.empty(nc + 1, dtype=np.uint32)
        self._c(lib().mpc_get_binning(self.h, box, _u32(key), _u32(perm), _u32(off)))
        return key, perm, off

    def set_tiling(self, tile_cells: int = 0, grid: int = 0, yblock: int = 0, order: int = 0):
        self._c(lib().mpc_set_tiling(self.h, tile_cells, grid, yblock, order))

    def get_tiling(self) -> dict:
        tc, g, yb, od, nt = (C.c_int32(0), C.c_int32(0), C.c_int32(0), C.c_int32(0),
                             C.c_int64(0))
        self._c(lib().mpc_get_tiling(self.h, C.byref(tc), C.byref(g), C.byref(yb), C.byref(od),
                                     C.byref(nt)))
        return {"tile_cells": tc.value, "grid": g.value, "yblock": yb.value, "order": od.value,
                "ntiles": nt.value}

    def autotune(self, trial_steps: int = 3):
        tc, g = C.c_int32(0), C.c_int32(0)
        self._c(lib().mpc_autotune(self.h, trial_steps, C.byref(tc), C.byref(g)))
        return int(tc.value), int(g.value)
