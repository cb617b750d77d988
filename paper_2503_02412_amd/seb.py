"""Python binding of libseb.so (include/seb.h): argument marshalling only.

Every step of the assessment runs in the library's HIP kernels; torch is used
for device memory and streams.  Importing this module on a machine without
the built library raises immediately -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libseb.so")

SEB_OK, SEB_ERR_INVALID, SEB_ERR_HIP, SEB_ERR_ALLOC, SEB_ERR_UNSUPPORTED, SEB_ERR_IO = \
    0, -1, -2, -3, -4, -5
ST_VALID, ST_CURV, ST_TILT, ST_DEGEN, ST_TRAV, ST_SURROGATE = 1, 2, 4, 8, 16, 32


class SebError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        super().__init__(f"{where}: status {code} ({detail})")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("width", C.c_int32), ("height", C.c_int32), ("resolution", C.c_double),
        ("n_yaw", C.c_int32), ("fp_length", C.c_double), ("fp_width", C.c_double),
        ("fp_nl", C.c_int32), ("fp_nw", C.c_int32), ("fp_shape", C.c_int32),
        ("kappa_max", C.c_double), ("phi_x_max", C.c_double), ("phi_y_max", C.c_double),
        ("w_kappa", C.c_double), ("w_phi_x", C.c_double), ("w_phi_y", C.c_double),
        ("risk_max", C.c_double), ("min_valid", C.c_int32), ("precision", C.c_int32),
        ("fit", C.c_int32),
    ]


class Out(C.Structure):
    _fields_ = [("z", C.c_void_p), ("roll", C.c_void_p), ("pitch", C.c_void_p),
                ("risk", C.c_void_p), ("status", C.c_void_p)]


class WindowPlan(C.Structure):
    _fields_ = [
        ("old_origin_x", C.c_int64), ("old_origin_y", C.c_int64),
        ("new_origin_x", C.c_int64), ("new_origin_y", C.c_int64),
        ("full_reset", C.c_int32), ("exposed_rows", C.c_int32), ("exposed_cols", C.c_int32),
        ("n_cells_exposed", C.c_int64), ("n_rects", C.c_int32),
        ("rects", (C.c_int32 * 4) * 8), ("n_states", C.c_int64),
    ]


class Scan(C.Structure):
    _fields_ = [("points", C.c_void_p), ("n_points", C.c_int64),
                ("R_B", C.c_double * 9), ("p_B", C.c_double * 3),
                ("R_BS", C.c_double * 9), ("p_BS", C.c_double * 3),
                ("Sigma_R", C.c_double * 9), ("Sigma_B", C.c_double * 9),
                ("sigma_range", C.c_double), ("sigma_angle", C.c_double),
                ("z_min", C.c_double), ("z_max", C.c_double), ("mahalanobis", C.c_double)]


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "seb_validate_config": (C.c_int, [C.POINTER(Config)]),
    "seb_create": (C.c_int, [C.POINTER(Config), C.POINTER(C.c_void_p)]),
    "seb_destroy": (None, [C.c_void_p]),
    "seb_assess_se2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                 C.c_int32, C.c_int32, C.POINTER(Out), C.c_void_p]),
    "seb_window_create": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.POINTER(Out),
                                    C.c_double, C.c_double, C.POINTER(C.c_void_p)]),
    "seb_window_destroy": (None, [C.c_void_p]),
    "seb_window_origin": (C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                    C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "seb_window_reset": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_int64,
                                   C.c_void_p]),
    "seb_window_plan_move": (C.c_int, [C.c_void_p, C.c_double, C.c_double,
                                       C.POINTER(WindowPlan)]),
    "seb_plan_window_move": (C.c_int, [C.POINTER(Config), C.c_int64, C.c_int64, C.c_double,
                                       C.c_double, C.POINTER(WindowPlan)]),
    "seb_update_window": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_void_p, C.c_void_p,
                                    C.POINTER(C.c_int64)]),
    "seb_sdf_se2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                              C.c_void_p, C.c_void_p]),
    "seb_query_se2": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int32, C.c_int32,
                                C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p]),
    "seb_fuser_create": (C.c_int, [C.c_void_p, C.c_int64, C.POINTER(C.c_void_p)]),
    "seb_fuser_destroy": (None, [C.c_void_p]),
    "seb_fuse_scan": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, C.c_int64,
                                C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p]),
    "seb_fuse_scan_static": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                       C.c_int64, C.c_int64, C.c_void_p, C.c_void_p,
                                       C.c_void_p]),
    "seb_raycast_reset": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int64,
                                    C.c_void_p, C.c_double, C.c_void_p, C.c_void_p]),
    "seb_inpaint_nearest": (C.c_int, [C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32,
                                      C.c_int32, C.c_void_p, C.c_int64, C.c_void_p]),
    "seb_strerror": (C.c_char_p, [C.c_int]),
    "seb_last_error": (C.c_char_p, []),
    "seb_version": (C.c_char_p, []),
}


def lib():
    """Load libseb.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        # torch first: the library then binds to the HIP runtime torch already
        # loaded (same SONAME), so device pointers and streams are shared.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2503_02412_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc: int, where: str):
    if rc != SEB_OK:
        raise SebError(rc, where, lib().seb_last_error().decode())


def config(params) -> Config:
    p = params
    return Config(int(p.width), int(p.height), float(p.resolution), int(p.n_yaw),
                  float(p.fp_length), float(p.fp_width), int(p.fp_nl), int(p.fp_nw),
                  int(p.fp_shape), float(p.kappa_max), float(p.phi_x_max), float(p.phi_y_max),
                  float(p.w_kappa), float(p.w_phi_x), float(p.w_phi_y), float(p.risk_max),
                  int(p.min_valid), int(p.precision), int(p.fit))


def validate(params) -> int:
    cfg = config(params)
    return int(lib().seb_validate_config(C.byref(cfg)))


def plan_window_move(params, origin_x: int, origin_y: int, x: float, y: float) -> WindowPlan:
    """Host-only window-move geometry (seb_plan_window_move)."""
    cfg = config(params)
    p = WindowPlan()
    _check(lib().seb_plan_window_move(C.byref(cfg), int(origin_x), int(origin_y), float(x),
                                      float(y), C.byref(p)), "seb_plan_window_move")
    return p


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def alloc_outputs(params, device="cuda"):
    """Five torch tensors [K, H, W] on the device (float32 x4 + uint8 status)."""
    import torch
    shape = (params.n_yaw, params.height, params.width)
    f = lambda: torch.empty(shape, dtype=torch.float32, device=device)
    return {"z": f(), "roll": f(), "pitch": f(), "risk": f(),
            "status": torch.empty(shape, dtype=torch.uint8, device=device)}


def _out_struct(out, params) -> Out:
    K, H, W = params.n_yaw, params.height, params.width
    for name in ("z", "roll", "pitch", "risk", "status"):
        t = out[name]
        if not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != (K, H, W):
            raise ValueError(f"output '{name}' must be a contiguous CUDA tensor [K, H, W]")
    return Out(out["z"].data_ptr(), out["roll"].data_ptr(), out["pitch"].data_ptr(),
               out["risk"].data_ptr(), out["status"].data_ptr())


def _check_map(height, params):
    import torch
    if not (height.is_cuda and height.dtype == torch.float32 and height.dim() == 2):
        raise ValueError("height must be a float32 CUDA tensor [H, W]")
    if tuple(height.shape) != (params.height, params.width) or height.stride(1) != 1:
        raise ValueError("height must be [H, W] with unit column stride")


class Context:
    """Footprint table for one configuration (seb_create / seb_destroy)."""

    def __init__(self, params):
        self.params = params
        self._cfg = config(params)
        h = C.c_void_p()
        _check(lib().seb_create(C.byref(self._cfg), C.byref(h)), "seb_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().seb_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def assess(self, height, out=None, rect=None, stream=None):
        """seb_assess_se2 over rect = (x0, y0, nx, ny) (default: the whole map)."""
        _check_map(height, self.params)
        if out is None:
            out = alloc_outputs(self.params, height.device)
        x0, y0, nx, ny = rect if rect is not None else (0, 0, self.params.width,
                                                         self.params.height)
        o = _out_struct(out, self.params)
        _check(lib().seb_assess_se2(self._h, C.c_void_p(height.data_ptr()), height.stride(0),
                                    x0, y0, nx, ny, C.byref(o), _stream_handle(stream)),
               "seb_assess_se2")
        return out

    def launcher(self, height, out, rect=None, stream=None):
        """A zero-argument callable that issues seb_assess_se2 with the
        arguments marshalled once, here (for launch loops that repeat the same
        call: the host cost per launch is then the C call alone).  Raises
        SebError on a failed launch."""
        _check_map(height, self.params)
        x0, y0, nx, ny = rect if rect is not None else (0, 0, self.params.width,
                                                         self.params.height)
        o = _out_struct(out, self.params)
        fn = lib().seb_assess_se2
        args = (self._h, C.c_void_p(height.data_ptr()), height.stride(0), x0, y0, nx, ny,
                C.byref(o), _stream_handle(stream))
        keep = (height, out, o)

        def launch():
            rc = fn(*args)
            if rc != SEB_OK:
                _check(rc, "seb_assess_se2")
            return keep
        return launch

    def _field(self, t, name, dtype):
        import torch
        p = self.params
        if (t is None or not t.is_cuda or t.dtype != dtype or not t.is_contiguous()
                or tuple(t.shape) != (p.n_yaw, p.height, p.width)):
            raise ValueError(f"{name} must be a contiguous {dtype} CUDA tensor [K, H, W]")
        return C.c_void_p(t.data_ptr())

    def sdf(self, status, cap_cells: int, unknown_is_obstacle: bool = True, ring=(0, 0),
            out=None, stream=None):
        """seb_sdf_se2: signed distance field [K, H, W] (float32, metres) of `status`."""
        import torch
        st = self._field(status, "status", torch.uint8)
        if out is None:
            out = torch.empty(tuple(status.shape), dtype=torch.float32, device=status.device)
        o = self._field(out, "out", torch.float32)
        _check(lib().seb_sdf_se2(self._h, st, int(ring[0]), int(ring[1]), int(cap_cells),
                                 int(bool(unknown_is_obstacle)), o, _stream_handle(stream)),
               "seb_sdf_se2")
        return out

    def query(self, poses, sdf=None, risk=None, ring=(0, 0), out=None, stream=None):
        """seb_query_se2: [n, 8] = (sdf, d/dx, d/dy, d/dtheta, risk, d/dx, d/dy, d/dtheta)
        at poses [n, 3] = (x, y, theta) (float32, logical map metres)."""
        import torch
        if not (poses.is_cuda and poses.dtype == torch.float32 and poses.is_contiguous()
                and poses.dim() == 2 and poses.shape[1] == 3):
            raise ValueError("poses must be a contiguous float32 CUDA tensor [n, 3]")
        fa = None if sdf is None else self._field(sdf, "sdf", torch.float32)
        fb = None if risk is None else self._field(risk, "risk", torch.float32)
        n = poses.shape[0]
        if out is None:
            out = torch.empty((n, 8), dtype=torch.float32, device=poses.device)
        if not (out.is_cuda and out.dtype == torch.float32 and out.is_contiguous()
                and tuple(out.shape) == (n, 8)):
            raise ValueError("out must be a contiguous float32 CUDA tensor [n, 8]")
        _check(lib().seb_query_se2(self._h, fa, fb, int(ring[0]), int(ring[1]),
                                   C.c_void_p(poses.data_ptr()), n, C.c_void_p(out.data_ptr()),
                                   _stream_handle(stream)), "seb_query_se2")
        return out

    def raycast_reset(self, height, origin, points, frames: dict, margin: float = 0.0,
                      n_reset=None, stream=None):
        """seb_raycast_reset: cells standing above a sensor-to-point ray become
        unknown (in place, ring storage of the window at world cell `origin`)."""
        _check_map(height, self.params)
        sc = Fuser.scan_struct(points, dict({"Sigma_R": np.zeros(9), "Sigma_B": np.zeros(9),
                                             "sigma_range": 1.0, "sigma_angle": 0.0,
                                             "z_min": 0.0, "z_max": 0.0, "mahalanobis": 1.0},
                                            **frames))
        ptr = None if n_reset is None else n_reset.data_ptr()
        _check(lib().seb_raycast_reset(self._h, C.c_void_p(height.data_ptr()), height.stride(0),
                                       int(origin[0]), int(origin[1]), C.byref(sc), float(margin),
                                       C.c_void_p(ptr), _stream_handle(stream)),
               "seb_raycast_reset")

    def inpaint(self, height, radius: int, ring=(0, 0), out=None, stream=None):
        """seb_inpaint_nearest: nearest-neighbour fill of unknown cells (a new map)."""
        import torch
        _check_map(height, self.params)
        if out is None:
            out = torch.empty_like(height)
        _check_map(out, self.params)
        _check(lib().seb_inpaint_nearest(self._h, C.c_void_p(height.data_ptr()), height.stride(0),
                                         int(ring[0]), int(ring[1]), int(radius),
                                         C.c_void_p(out.data_ptr()), out.stride(0),
                                         _stream_handle(stream)), "seb_inpaint_nearest")
        return out


class Fuser:
    """Scan fusion into an elevation map (seb_fuser_* / seb_fuse_scan)."""

    def __init__(self, ctx: Context, max_points: int):
        self.ctx = ctx
        h = C.c_void_p()
        _check(lib().seb_fuser_create(ctx._h, int(max_points), C.byref(h)), "seb_fuser_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().seb_fuser_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def scan_struct(points, frames: dict) -> Scan:
        import torch
        if not (points.is_cuda and points.dtype == torch.float32 and points.is_contiguous()
                and points.dim() == 2 and points.shape[1] == 3):
            raise ValueError("points must be a contiguous float32 CUDA tensor [n, 3]")
        d = lambda k, n: (C.c_double * n)(*[float(v) for v in np.asarray(frames[k]).ravel()])
        return Scan(points.data_ptr(), points.shape[0], d("R_B", 9), d("p_B", 3), d("R_BS", 9),
                    d("p_BS", 3), d("Sigma_R", 9), d("Sigma_B", 9), float(frames["sigma_range"]),
                    float(frames["sigma_angle"]), float(frames["z_min"]), float(frames["z_max"]),
                    float(frames["mahalanobis"]))

    def fuse(self, height, variance, origin, points, frames: dict, n_fused=None, stream=None):
        """Fuse a scan (points: float32 CUDA [n, 3], sensor frame) into the ring
        maps height / variance of the window whose logical (0, 0) is world
        cell `origin`."""
        p = self.ctx.params
        _check_map(height, p)
        _check_map(variance, p)
        if height.stride(0) != variance.stride(0):
            raise ValueError("height and variance must share a row stride")
        sc = self.scan_struct(points, frames)
        ptr = None if n_fused is None else n_fused.data_ptr()
        _check(lib().seb_fuse_scan(self._h, C.c_void_p(height.data_ptr()),
                                   C.c_void_p(variance.data_ptr()), height.stride(0),
                                   int(origin[0]), int(origin[1]), C.byref(sc), C.c_void_p(ptr),
                                   _stream_handle(stream)), "seb_fuse_scan")


def fuse_scan_static(ctx: "Context", height, variance, origin, points, frames: dict,
                     n_fused=None, stream=None):
    """seb_fuse_scan_static: Fuser.fuse without a fuser (the library's static
    workspace; maps of at most 2^18 cells, scans of at most 2^18 points)."""
    p = ctx.params
    _check_map(height, p)
    _check_map(variance, p)
    if height.stride(0) != variance.stride(0):
        raise ValueError("height and variance must share a row stride")
    sc = Fuser.scan_struct(points, frames)
    ptr = None if n_fused is None else n_fused.data_ptr()
    _check(lib().seb_fuse_scan_static(ctx._h, C.c_void_p(height.data_ptr()),
                                      C.c_void_p(variance.data_ptr()), height.stride(0),
                                      int(origin[0]), int(origin[1]), C.byref(sc),
                                      C.c_void_p(ptr), _stream_handle(stream)),
           "seb_fuse_scan_static")


class Window:
    """Rolling window over ring storage (seb_window_*)."""

    def __init__(self, ctx: Context, x: float, y: float, ring=None, out=None):
        import torch
        p = ctx.params
        self.ctx = ctx
        self.ring = ring if ring is not None else torch.full(
            (p.height, p.width), float("nan"), dtype=torch.float32, device="cuda")
        self.out = out if out is not None else alloc_outputs(p, self.ring.device)
        o = _out_struct(self.out, p)
        h = C.c_void_p()
        _check(lib().seb_window_create(ctx._h, C.c_void_p(self.ring.data_ptr()),
                                       self.ring.stride(0), C.byref(o), float(x), float(y),
                                       C.byref(h)), "seb_window_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().seb_window_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def origin(self):
        ox, oy, rx, ry = C.c_int64(), C.c_int64(), C.c_int32(), C.c_int32()
        _check(lib().seb_window_origin(self._h, C.byref(ox), C.byref(oy), C.byref(rx),
                                       C.byref(ry)), "seb_window_origin")
        return ox.value, oy.value, rx.value, ry.value

    def reset(self, x, y, heights=None, stream=None):
        ptr, ld = (None, 0) if heights is None else (heights.data_ptr(), heights.stride(0))
        if heights is not None:
            _check_map(heights, self.ctx.params)
        _check(lib().seb_window_reset(self._h, float(x), float(y), C.c_void_p(ptr), ld,
                                      _stream_handle(stream)), "seb_window_reset")

    def plan(self, x, y) -> WindowPlan:
        p = WindowPlan()
        _check(lib().seb_window_plan_move(self._h, float(x), float(y), C.byref(p)),
               "seb_window_plan_move")
        return p

    def update(self, x, y, new_cells=None, stream=None) -> int:
        if new_cells is not None:
            import torch
            need = self.plan(x, y).n_cells_exposed
            if (not new_cells.is_cuda or new_cells.dtype != torch.float32
                    or not new_cells.is_contiguous() or new_cells.numel() < need):
                raise ValueError(f"new_cells must be a contiguous float32 CUDA tensor "
                                 f"with >= {need} elements")
        n = C.c_int64()
        ptr = None if new_cells is None else new_cells.data_ptr()
        _check(lib().seb_update_window(self._h, float(x), float(y), C.c_void_p(ptr),
                                       _stream_handle(stream), C.byref(n)), "seb_update_window")
        return n.value

    def logical(self, name: str):
        """An output (or 'height') un-rotated to logical window order (a copy)."""
        import torch
        _, _, rx, ry = self.origin()
        t = self.ring if name == "height" else self.out[name]
        return torch.roll(t, shifts=(-ry, -rx), dims=(-2, -1))


def version() -> str:
    return lib().seb_version().decode()


# ------------------------------------------------------------ surrogate net

class TrainBatch(C.Structure):
    _fields_ = [
        ("maps", C.c_void_p), ("n_maps", C.c_int32), ("map_h", C.c_int32), ("map_w", C.c_int32),
        ("resolution", C.c_double), ("n_yaw", C.c_int32),
        ("label_z", C.c_void_p), ("label_roll", C.c_void_p), ("label_pitch", C.c_void_p),
        ("label_risk", C.c_void_p), ("samples", C.c_void_p), ("batch", C.c_int32),
    ]


_SIGS.update({
    "seb_net_param_count": (C.c_int64, []),
    "seb_net_create": (C.c_int, [C.c_uint64, C.c_int32, C.POINTER(C.c_void_p)]),
    "seb_net_destroy": (None, [C.c_void_p]),
    "seb_net_get_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "seb_net_set_params": (C.c_int, [C.c_void_p, C.c_void_p]),
    "seb_net_save": (C.c_int, [C.c_void_p, C.c_char_p]),
    "seb_net_load": (C.c_int, [C.c_void_p, C.c_char_p]),
    "seb_net_forward": (C.c_int, [C.c_void_p, C.POINTER(TrainBatch), C.c_void_p, C.c_void_p]),
    "seb_net_train_step": (C.c_int, [C.c_void_p, C.POINTER(TrainBatch), C.c_float, C.c_void_p,
                                     C.c_void_p, C.c_void_p]),
    "seb_net_last_error": (C.c_char_p, []),
})


def _net_check(rc: int, where: str):
    if rc != SEB_OK:
        raise SebError(rc, where, lib().seb_net_last_error().decode())


class Net:
    """The surrogate network (seb_net_*)."""

    def __init__(self, seed: int = 0, max_batch: int = 4096):
        h = C.c_void_p()
        _net_check(lib().seb_net_create(int(seed), int(max_batch), C.byref(h)), "seb_net_create")
        self._h = h
        self.max_batch = max_batch

    @staticmethod
    def param_count() -> int:
        return int(lib().seb_net_param_count())

    def close(self):
        if getattr(self, "_h", None):
            lib().seb_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def params(self):
        import numpy as np
        out = np.empty(self.param_count(), dtype=np.float32)
        _net_check(lib().seb_net_get_params(self._h, out.ctypes.data), "seb_net_get_params")
        return out

    def set_params(self, vec):
        import numpy as np
        v = np.ascontiguousarray(vec, dtype=np.float32)
        if v.size != self.param_count():
            raise ValueError("parameter vector has the wrong length")
        _net_check(lib().seb_net_set_params(self._h, v.ctypes.data), "seb_net_set_params")

    def save(self, path: str):
        _net_check(lib().seb_net_save(self._h, path.encode()), "seb_net_save")

    def load(self, path: str):
        _net_check(lib().seb_net_load(self._h, path.encode()), "seb_net_load")

    @staticmethod
    def _batch(maps, samples, resolution, n_yaw, labels=None) -> TrainBatch:
        import torch
        if not (maps.is_cuda and maps.dtype == torch.float32 and maps.dim() == 3
                and maps.is_contiguous()):
            raise ValueError("maps must be a contiguous float32 CUDA tensor [n, H, W]")
        if not (samples.is_cuda and samples.dtype == torch.int32 and samples.dim() == 2
                and samples.shape[1] == 4 and samples.is_contiguous()):
            raise ValueError("samples must be a contiguous int32 CUDA tensor [B, 4]")
        n, H, W = maps.shape
        s = samples.cpu()
        if samples.shape[0] and (int(s[:, 0].min()) < 0 or int(s[:, 0].max()) >= n
                                 or int(s[:, 1].min()) < 0 or int(s[:, 1].max()) >= H
                                 or int(s[:, 2].min()) < 0 or int(s[:, 2].max()) >= W
                                 or int(s[:, 3].min()) < 0 or int(s[:, 3].max()) >= n_yaw):
            raise ValueError("sample indices out of range")
        ptr = [None] * 4
        if labels is not None:
            for i, k in enumerate(("z", "roll", "pitch", "risk")):
                t = labels[k]
                if tuple(t.shape) != (n, n_yaw, H, W) or not t.is_contiguous() or not t.is_cuda:
                    raise ValueError(f"label '{k}' must be a contiguous CUDA tensor [n, K, H, W]")
                ptr[i] = t.data_ptr()
        return TrainBatch(maps.data_ptr(), n, H, W, float(resolution), int(n_yaw), ptr[0], ptr[1],
                          ptr[2], ptr[3], samples.data_ptr(), samples.shape[0])

    def forward(self, maps, samples, resolution, n_yaw, stream=None):
        import torch
        b = self._batch(maps, samples, resolution, n_yaw)
        y = torch.empty((samples.shape[0], 4), dtype=torch.float32, device=maps.device)
        _net_check(lib().seb_net_forward(self._h, C.byref(b), C.c_void_p(y.data_ptr()),
                                         _stream_handle(stream)), "seb_net_forward")
        return y

    def train_step(self, maps, labels, samples, resolution, n_yaw, lr, loss=None, grad=None,
                   stream=None):
        b = self._batch(maps, samples, resolution, n_yaw, labels)
        _net_check(lib().seb_net_train_step(
            self._h, C.byref(b), C.c_float(lr),
            C.c_void_p(None if loss is None else loss.data_ptr()),
            C.c_void_p(None if grad is None else grad.data_ptr()), _stream_handle(stream)),
            "seb_net_train_step")


_SIGS.update({
    "seb_surrogate_create": (C.c_int, [C.c_void_p, C.POINTER(C.c_void_p)]),
    "seb_surrogate_destroy": (None, [C.c_void_p]),
    "seb_surrogate_infer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                      C.POINTER(Out), C.c_float, C.c_float, C.c_void_p,
                                      C.c_void_p]),
})


class Surrogate:
    """Surrogate inference workspace for one context (seb_surrogate_*)."""

    def __init__(self, ctx: Context):
        h = C.c_void_p()
        _check(lib().seb_surrogate_create(ctx._h, C.byref(h)), "seb_surrogate_create")
        self._h = h
        self.ctx = ctx

    def close(self):
        if getattr(self, "_h", None):
            lib().seb_surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def infer(self, net: "Net", height, out=None, band: float = 0.1, min_known: float = 0.75,
              n_fallback=None, stream=None):
        """seb_surrogate_infer; returns the outputs (n_fallback: optional int32 CUDA tensor)."""
        p = self.ctx.params
        _check_map(height, p)
        if out is None:
            out = alloc_outputs(p, height.device)
        o = _out_struct(out, p)
        nf = None if n_fallback is None else n_fallback.data_ptr()
        _check(lib().seb_surrogate_infer(self._h, net._h, C.c_void_p(height.data_ptr()),
                                         height.stride(0), C.byref(o), C.c_float(band),
                                         C.c_float(min_known), C.c_void_p(nf),
                                         _stream_handle(stream)), "seb_surrogate_infer")
        return out
