"""FP64 CPU oracle for SE(2)-grid traversability assessment -- TEST INFRASTRUCTURE.

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library: the C source
``seb_oracle.c`` defines its own parameter struct, and this wrapper marshals
plain numpy arrays into it.

The method it implements (Sec. III Eq. 1-3 and Sec. V-B Algorithm 1 of the
paper) is described in the header comment of ``seb_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "seb_oracle.c")
_LIB = os.path.join(_HERE, "libseb_oracle.so")

ST_VALID, ST_CURV, ST_TILT, ST_DEGEN, ST_TRAV = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
               "-fPIC", "-shared", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("res", C.c_double),
        ("n_yaw", C.c_int32), ("fp_length", C.c_double), ("fp_width", C.c_double),
        ("fp_nl", C.c_int32), ("fp_nw", C.c_int32), ("fp_shape", C.c_int32),
        ("kappa_max", C.c_double), ("phi_x_max", C.c_double), ("phi_y_max", C.c_double),
        ("w_kappa", C.c_double), ("w_phi_x", C.c_double), ("w_phi_y", C.c_double),
        ("risk_max", C.c_double), ("min_valid", C.c_int32), ("fit", C.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = C.CDLL(_LIB)
        dp = C.POINTER(C.c_double)
        lib.orc_assess_rect.restype = C.c_int
        lib.orc_assess_rect.argtypes = [C.POINTER(_Params), C.POINTER(C.c_float), C.c_int64,
                                        C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int,
                                        dp, dp, dp, dp, dp, dp, dp,
                                        C.POINTER(C.c_uint8), C.POINTER(C.c_int32), C.c_int]
        lib.orc_assess_list.restype = C.c_int
        lib.orc_assess_list.argtypes = [C.POINTER(_Params), C.POINTER(C.c_float), C.c_int64,
                                        C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_int32), dp, dp, dp, dp, dp, dp, dp,
                                        C.POINTER(C.c_uint8), C.POINTER(C.c_int32), C.c_int]
        lib.orc_reach.restype = C.c_int
        lib.orc_reach.argtypes = [C.POINTER(_Params)] + [C.POINTER(C.c_int32)] * 4
        lib.orc_max_threads.restype = C.c_int
        lib.orc_rho_full.restype = C.c_double
        lib.orc_rho_full.argtypes = [C.POINTER(_Params), C.POINTER(C.c_int32)]
        lib.orc_gate_points.restype = C.c_int
        lib.orc_gate_points.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int,
                                        C.c_int, C.c_int, C.c_double]
        _lib = lib
    return _lib


def _params(p) -> _Params:
    return _Params(int(p.width), int(p.height), float(p.resolution), int(p.n_yaw),
                   float(p.fp_length), float(p.fp_width), int(p.fp_nl), int(p.fp_nw),
                   int(p.fp_shape), float(p.kappa_max), float(p.phi_x_max), float(p.phi_y_max),
                   float(p.w_kappa), float(p.w_phi_x), float(p.w_phi_y), float(p.risk_max),
                   int(p.min_valid), int(p.fit))


@dataclass
class Result:
    z: np.ndarray
    roll: np.ndarray
    pitch: np.ndarray
    risk: np.ndarray
    kappa: np.ndarray
    phi_x: np.ndarray
    phi_y: np.ndarray
    status: np.ndarray
    n_valid: np.ndarray


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _alloc(shape):
    f = lambda: np.empty(shape, dtype=np.float64)
    return Result(f(), f(), f(), f(), f(), f(), f(), np.empty(shape, np.uint8),
                  np.empty(shape, np.int32))


def assess_rect(params, height: np.ndarray, x0: int = 0, y0: int = 0, nx: int | None = None,
                ny: int | None = None, k0: int = 0, nk: int | None = None,
                threads: int = 0) -> Result:
    """Assess states of the rectangle; arrays come back shaped [nk, ny, nx]."""
    lib = _load()
    h = np.ascontiguousarray(height, dtype=np.float32)
    assert h.shape == (params.height, params.width)
    nx = params.width - x0 if nx is None else nx
    ny = params.height - y0 if ny is None else ny
    nk = params.n_yaw - k0 if nk is None else nk
    r = _alloc((nk, ny, nx))
    P = _params(params)
    dp = C.c_double
    rc = lib.orc_assess_rect(C.byref(P), _ptr(h, C.c_float), h.shape[1], x0, y0, nx, ny, k0, nk,
                             _ptr(r.z, dp), _ptr(r.roll, dp), _ptr(r.pitch, dp), _ptr(r.risk, dp),
                             _ptr(r.kappa, dp), _ptr(r.phi_x, dp), _ptr(r.phi_y, dp),
                             _ptr(r.status, C.c_uint8), _ptr(r.n_valid, C.c_int32), threads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return r


def assess_list(params, height: np.ndarray, ix, iy, k, threads: int = 0) -> Result:
    """Assess an explicit list of states; arrays come back with one entry per state."""
    lib = _load()
    h = np.ascontiguousarray(height, dtype=np.float32)
    assert h.shape == (params.height, params.width)
    ix = np.ascontiguousarray(ix, dtype=np.int32)
    iy = np.ascontiguousarray(iy, dtype=np.int32)
    k = np.ascontiguousarray(k, dtype=np.int32)
    n = ix.shape[0]
    r = _alloc((n,))
    P = _params(params)
    dp = C.c_double
    rc = lib.orc_assess_list(C.byref(P), _ptr(h, C.c_float), h.shape[1], n,
                             _ptr(ix, C.c_int32), _ptr(iy, C.c_int32), _ptr(k, C.c_int32),
                             _ptr(r.z, dp), _ptr(r.roll, dp), _ptr(r.pitch, dp), _ptr(r.risk, dp),
                             _ptr(r.kappa, dp), _ptr(r.phi_x, dp), _ptr(r.phi_y, dp),
                             _ptr(r.status, C.c_uint8), _ptr(r.n_valid, C.c_int32), threads)
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    return r


def reach(params) -> tuple[int, int, int, int]:
    """(dx_min, dx_max, dy_min, dy_max): extent of cells any footprint sample reads."""
    lib = _load()
    v = [C.c_int32() for _ in range(4)]
    lib.orc_reach(C.byref(_params(params)), *[C.byref(x) for x in v])
    return tuple(int(x.value) for x in v)


def rho_full(params) -> tuple[float, int]:
    """(rho_full, n_total): 4 det / (D + E)^2 of the complete footprint's exact
    integer scatter, and its sample count."""
    lib = _load()
    n = C.c_int32()
    r = lib.orc_rho_full(C.byref(_params(params)), C.byref(n))
    return float(r), int(n.value)


def max_threads() -> int:
    return int(_load().orc_max_threads())


def gate_points(p, q, min_valid: int, n_total: int, rho_f: float) -> int:
    """Gate of the fit for valid samples at integer body-grid coordinates
    (p[m], q[m]): -1 no fit, 0 fit, 1 near-degenerate fit (Sec. V-B gate
    reading: fewer than half the samples, or rho below rho_full / 16)."""
    lib = _load()
    pa = np.ascontiguousarray(p, dtype=np.int32)
    qa = np.ascontiguousarray(q, dtype=np.int32)
    assert pa.shape == qa.shape and pa.ndim == 1
    return int(lib.orc_gate_points(_ptr(pa, C.c_int32), _ptr(qa, C.c_int32), int(pa.size),
                                   int(min_valid), int(n_total), float(rho_f)))
