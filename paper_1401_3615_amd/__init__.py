"""Python binding of the gfx950 FDK backprojection library (libfdk.so).

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in include/fdk.h.  PyTorch supplies device
memory (tensors) and streams.  If the compiled library is missing, every call
raises; there is no CPU fallback.

Conventions: projection matrices are (N, 3, 4) float64 row-major, projections
(N, H, W) with the column index fastest, volumes (nz, L, L) indexed (z, y, x).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field
from typing import Optional, Sequence

import numpy as np
import torch  # loads the HIP runtime that libfdk.so binds to

from . import _build

__all__ = [
    "FdkError", "Volume", "Geometry", "F32", "F16", "BF16", "TUNE_ADJOINT", "TUNE_BATCHED", "load", "backproject",
    "backproject_noalloc",
    "forwardproject", "backproject_batched", "pack_projections", "set_tile", "get_tile",
    "load_tuning", "set_tuning_entry", "validate", "release_workspace", "abi_version",
    "BackProject", "ForwardProject", "Scan", "profile_enable", "profile_read", "FilterGeometry",
    "filter_projections", "cgls", "sirt", "backproject_streamed", "streamed_plan", "normalize_matrices",
]

F32, F16, BF16 = 0, 1, 2
TUNE_ADJOINT = 3   # tuning slot of the forward projector
TUNE_BATCHED = 4   # tuning slot of the batched persistent launch
_TORCH_DTYPE = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}


class FdkError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_status_name(status)}: {message}")
        self.status = status


class _Volume(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("z_begin", ctypes.c_int32), ("z_count", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("voxel_mm", ctypes.c_double),
                ("origin_mm", ctypes.c_double * 3)]


class _Proj(ctypes.Structure):
    _fields_ = [("n_proj", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("dtype", ctypes.c_int32), ("mats", ctypes.POINTER(ctypes.c_double)),
                ("data", ctypes.c_void_p), ("scale", ctypes.c_void_p)]


class _Scan(ctypes.Structure):
    _fields_ = [("vol", _Volume), ("proj", _Proj), ("volume", ctypes.c_void_p)]


_lib = None


def load():
    """Load libfdk.so from the package directory (raises if it was not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_build.LIB):
        raise FdkError(-3, f"HIP library not built: {_build.LIB} is missing "
                           "(build it with: python -m paper_1401_3615_amd._build)")
    lib = ctypes.CDLL(_build.LIB)
    vp, i32 = ctypes.c_void_p, ctypes.c_int32
    pv, pp, ps = ctypes.POINTER(_Volume), ctypes.POINTER(_Proj), ctypes.POINTER(_Scan)
    sig = {
        "fdk_backproject": ([pv, pp, vp, ctypes.c_int, vp], ctypes.c_int),
        "fdk_backproject_noalloc": ([pv, pp, vp, ctypes.c_int, vp], ctypes.c_int),
        "fdk_forwardproject": ([pv, vp, pp, vp, ctypes.c_int, vp], ctypes.c_int),
        "fdk_backproject_batched": ([ps, i32, ctypes.c_int, vp], ctypes.c_int),
        "fdk_pack_projections": ([vp, i32, i32, i32, i32, vp, vp, vp], ctypes.c_int),
        "fdk_filter_projections": ([ctypes.POINTER(_FilterGeom), vp, vp, i32, vp, vp], ctypes.c_int),
        "fdk_cgls": ([pv, pp, vp, i32, ctypes.c_int, vp, vp], ctypes.c_int),
        "fdk_backproject_streamed": ([pv, pp, vp, i32, i32, ctypes.c_int, vp], ctypes.c_int),
        "fdk_streamed_plan": ([pv, pp, i32, ctypes.POINTER(i32), vp, vp], ctypes.c_int),
        "fdk_sirt": ([pv, pp, vp, i32, ctypes.c_double, i32, vp, vp], ctypes.c_int),
        "fdk_set_tile": ([i32, i32, i32, i32], ctypes.c_int),
        "fdk_get_tile": ([pv, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)],
                         ctypes.c_int),
        "fdk_load_tuning": ([ctypes.c_char_p], i32),
        "fdk_set_tuning_entry": ([i32, i32, i32, i32, i32], ctypes.c_int),
        "fdk_validate": ([pv, pp, ctypes.c_int], ctypes.c_int),
        "fdk_normalize_matrices": ([ctypes.POINTER(ctypes.c_double), i32], ctypes.c_int),
        "fdk_release_workspace": ([], ctypes.c_int),
        "fdk_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "fdk_last_error": ([], ctypes.c_char_p),
        "fdk_abi_version": ([], i32),
        "fdk_profile_enable": ([ctypes.c_int], ctypes.c_int),
        "fdk_profile_read": ([ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64),
                              ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _status_name(st: int) -> str:
    names = {0: "FDK_OK", -1: "FDK_E_INVALID_ARG", -2: "FDK_E_GEOMETRY", -3: "FDK_E_UNSUPPORTED",
             -4: "FDK_E_NOMEM", -5: "FDK_E_DEVICE"}
    return names.get(st, f"status {st}")


def _check(st: int):
    if st != 0:
        raise FdkError(st, load().fdk_last_error().decode())


@dataclass
class Volume:
    """L^3 grid of voxel pitch voxel_mm; origin_mm is the centre of voxel 0
    (default: volume centred on the isocentre).  Buffers hold the planes
    [z_begin, z_begin + z_count)."""
    L: int
    voxel_mm: float
    origin_mm: Optional[Sequence[float]] = None
    z_begin: int = 0
    z_count: Optional[int] = None

    def c(self) -> _Volume:
        v = _Volume()
        v.L = self.L
        v.z_begin = self.z_begin
        v.z_count = self.L - self.z_begin if self.z_count is None else self.z_count
        v.reserved = 0
        v.voxel_mm = self.voxel_mm
        o = self.origin_mm
        if o is None:
            c = -(self.L - 1) * self.voxel_mm / 2.0
            o = (c, c, c)
        v.origin_mm[:] = [float(x) for x in o]
        return v

    @property
    def planes(self) -> int:
        return self.L - self.z_begin if self.z_count is None else self.z_count

    def slab(self, z_begin: int, z_count: int) -> "Volume":
        return Volume(self.L, self.voxel_mm, self.origin_mm, z_begin, z_count)


@dataclass
class Geometry:
    """Projection geometry: one 3x4 matrix per projection and the detector size."""
    mats: np.ndarray
    width: int
    height: int
    _m: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self._m = np.ascontiguousarray(np.asarray(self.mats, dtype=np.float64).reshape(-1, 12))

    @property
    def n_proj(self) -> int:
        return self._m.shape[0]

    def c(self, data=None, dtype=F32, scale=None) -> _Proj:
        p = _Proj()
        p.n_proj = self.n_proj
        p.width = self.width
        p.height = self.height
        p.dtype = dtype
        p.mats = self._m.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        p.data = data
        p.scale = scale
        return p


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def _dev_ptr(t: torch.Tensor, name: str, dtypes=None) -> int:
    if not t.is_cuda:
        raise FdkError(-1, f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise FdkError(-1, f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise FdkError(-3, f"{name} has dtype {t.dtype}")
    return t.data_ptr()


def backproject(proj: torch.Tensor, geom: Geometry, vol: Volume, out: torch.Tensor = None,
                accumulate: bool = False, scale: torch.Tensor = None, stream=None) -> torch.Tensor:
    """fdk_backproject: volume (z_count, L, L) float32 from projections (N, H, W)."""
    lib = load()
    if proj.dtype not in _TORCH_DTYPE:
        raise FdkError(-3, f"projection dtype {proj.dtype}")
    if tuple(proj.shape) != (geom.n_proj, geom.height, geom.width):
        raise FdkError(-1, f"projections {tuple(proj.shape)} do not match geometry "
                           f"{(geom.n_proj, geom.height, geom.width)}")
    if out is None:
        out = torch.empty((vol.planes, vol.L, vol.L), dtype=torch.float32, device=proj.device)
    elif tuple(out.shape) != (vol.planes, vol.L, vol.L) or out.dtype != torch.float32:
        raise FdkError(-1, "output volume has the wrong shape or dtype")
    sp = None
    if scale is not None:
        if scale.numel() != geom.n_proj:
            raise FdkError(-1, "scale must have one entry per projection")
        sp = _dev_ptr(scale, "scale", (torch.float32,))
    v = vol.c()
    p = geom.c(_dev_ptr(proj, "projections"), _TORCH_DTYPE[proj.dtype], sp)
    _check(lib.fdk_backproject(ctypes.byref(v), ctypes.byref(p),
                               _dev_ptr(out, "volume", (torch.float32,)), int(bool(accumulate)),
                               _stream(stream)))
    return out


def backproject_noalloc(proj: torch.Tensor, geom: Geometry, vol: Volume, out: torch.Tensor,
                        accumulate: bool = False, scale: torch.Tensor = None, stream=None) -> torch.Tensor:
    """fdk_backproject_noalloc: fdk_backproject without any device allocation
    (FP32 projections; the caller provides `out`)."""
    lib = load()
    if proj.dtype not in _TORCH_DTYPE:
        raise FdkError(-3, f"projection dtype {proj.dtype}")
    if tuple(proj.shape) != (geom.n_proj, geom.height, geom.width):
        raise FdkError(-1, f"projections {tuple(proj.shape)} do not match geometry "
                           f"{(geom.n_proj, geom.height, geom.width)}")
    if tuple(out.shape) != (vol.planes, vol.L, vol.L) or out.dtype != torch.float32:
        raise FdkError(-1, "output volume has the wrong shape or dtype")
    sp = None
    if scale is not None:
        if scale.numel() != geom.n_proj:
            raise FdkError(-1, "scale must have one entry per projection")
        sp = _dev_ptr(scale, "scale", (torch.float32,))
    v = vol.c()
    p = geom.c(_dev_ptr(proj, "projections"), _TORCH_DTYPE[proj.dtype], sp)
    _check(lib.fdk_backproject_noalloc(ctypes.byref(v), ctypes.byref(p),
                                       _dev_ptr(out, "volume", (torch.float32,)), int(bool(accumulate)),
                                       _stream(stream)))
    return out


def forwardproject(volume: torch.Tensor, geom: Geometry, vol: Volume, out: torch.Tensor = None,
                   accumulate: bool = False, stream=None) -> torch.Tensor:
    """fdk_forwardproject (adjoint of backproject): projections (N, H, W) float32."""
    lib = load()
    if tuple(volume.shape) != (vol.planes, vol.L, vol.L):
        raise FdkError(-1, f"volume {tuple(volume.shape)} does not match the grid")
    if out is None:
        out = torch.empty((geom.n_proj, geom.height, geom.width), dtype=torch.float32,
                          device=volume.device)
    elif tuple(out.shape) != (geom.n_proj, geom.height, geom.width) or out.dtype != torch.float32:
        raise FdkError(-1, "output projections have the wrong shape or dtype")
    v = vol.c()
    p = geom.c()
    _check(lib.fdk_forwardproject(ctypes.byref(v), _dev_ptr(volume, "volume", (torch.float32,)),
                                  ctypes.byref(p), _dev_ptr(out, "projections", (torch.float32,)),
                                  int(bool(accumulate)), _stream(stream)))
    return out


def backproject_streamed(proj: torch.Tensor, geom: Geometry, vol: Volume, slab_planes: int,
                         out: torch.Tensor = None, accumulate: bool = False, scale: torch.Tensor = None,
                         stream=None) -> torch.Tensor:
    """fdk_backproject_streamed: the projection stack may live in host memory
    (pin it for overlap); each z-slab of `slab_planes` planes receives only
    its detector row band.  `out` on the CPU keeps the volume in host memory
    (FDK_STREAM_HOST_VOLUME); default: a new device volume.  The CPU tensors
    must stay alive until the stream has completed."""
    lib = load()
    if proj.dtype not in _TORCH_DTYPE:
        raise FdkError(-3, f"projection dtype {proj.dtype}")
    if tuple(proj.shape) != (geom.n_proj, geom.height, geom.width) or not proj.is_contiguous():
        raise FdkError(-1, "projections must be a contiguous (N, H, W) stack matching the geometry")
    if out is None:
        out = torch.empty((vol.planes, vol.L, vol.L), dtype=torch.float32, device="cuda")
    if tuple(out.shape) != (vol.planes, vol.L, vol.L) or out.dtype != torch.float32 or not out.is_contiguous():
        raise FdkError(-1, "output volume has the wrong shape, dtype or layout")
    sp = None
    if scale is not None:
        if scale.numel() != geom.n_proj:
            raise FdkError(-1, "scale must have one entry per projection")
        sp = _dev_ptr(scale, "scale", (torch.float32,))
    v = vol.c()
    p = geom.c(proj.data_ptr(), _TORCH_DTYPE[proj.dtype], sp)
    flags = 0 if out.is_cuda else 1
    _check(lib.fdk_backproject_streamed(ctypes.byref(v), ctypes.byref(p), out.data_ptr(), int(slab_planes), flags,
                                        int(bool(accumulate)), _stream(stream)))
    return out


def streamed_plan(geom: Geometry, vol: Volume, slab_planes: int):
    """(band_rows (S,), first_rows (S, N)) of fdk_backproject_streamed's slab plan."""
    lib = load()
    v, p = vol.c(), geom.c()
    n = ctypes.c_int32()
    _check(lib.fdk_streamed_plan(ctypes.byref(v), ctypes.byref(p), int(slab_planes), ctypes.byref(n), None, None))
    rows = np.zeros(n.value, dtype=np.int32)
    first = np.zeros((n.value, geom.n_proj), dtype=np.int32)
    _check(lib.fdk_streamed_plan(ctypes.byref(v), ctypes.byref(p), int(slab_planes), ctypes.byref(n),
                                 rows.ctypes.data, first.ctypes.data))
    return rows, first


@dataclass
class Scan:
    proj: torch.Tensor
    geom: Geometry
    vol: Volume
    out: torch.Tensor
    scale: Optional[torch.Tensor] = None


def backproject_batched(scans: Sequence[Scan], accumulate: bool = False, stream=None) -> None:
    """fdk_backproject_batched: all scans in one persistent launch (HIP graph)."""
    lib = load()
    arr = (_Scan * len(scans))()
    for i, s in enumerate(scans):
        if s.proj.dtype not in _TORCH_DTYPE:
            raise FdkError(-3, f"scan {i}: projection dtype {s.proj.dtype}")
        if tuple(s.proj.shape) != (s.geom.n_proj, s.geom.height, s.geom.width):
            raise FdkError(-1, f"scan {i}: projections do not match geometry")
        if tuple(s.out.shape) != (s.vol.planes, s.vol.L, s.vol.L) or s.out.dtype != torch.float32:
            raise FdkError(-1, f"scan {i}: output volume has the wrong shape or dtype")
        arr[i].vol = s.vol.c()
        sp = _dev_ptr(s.scale, "scale", (torch.float32,)) if s.scale is not None else None
        arr[i].proj = s.geom.c(_dev_ptr(s.proj, "projections"), _TORCH_DTYPE[s.proj.dtype], sp)
        arr[i].volume = _dev_ptr(s.out, "volume", (torch.float32,))
    _check(lib.fdk_backproject_batched(arr, len(scans), int(bool(accumulate)), _stream(stream)))


def pack_projections(proj: torch.Tensor, dtype=torch.float16, stream=None):
    """fdk_pack_projections: (packed (N, H, W) float16/bfloat16, scale (N,) float32)."""
    lib = load()
    if proj.dtype != torch.float32 or proj.dim() != 3:
        raise FdkError(-1, "pack_projections expects (N, H, W) float32")
    code = {torch.float16: F16, torch.bfloat16: BF16}.get(dtype)
    if code is None:
        raise FdkError(-3, f"pack dtype {dtype}")
    n, h, w = proj.shape
    packed = torch.empty((n, h, w), dtype=dtype, device=proj.device)
    scale = torch.empty(n, dtype=torch.float32, device=proj.device)
    _check(lib.fdk_pack_projections(_dev_ptr(proj, "projections"), n, w, h, code,
                                    packed.data_ptr(), scale.data_ptr(), _stream(stream)))
    return packed, scale


class _FilterGeom(ctypes.Structure):
    _fields_ = [("n_proj", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("pixel_u_mm", ctypes.c_double), ("pixel_v_mm", ctypes.c_double),
                ("u0", ctypes.c_double), ("v0", ctypes.c_double), ("sdd_mm", ctypes.c_double),
                ("sid_mm", ctypes.c_double), ("angles_rad", ctypes.POINTER(ctypes.c_double)),
                ("scan_range_rad", ctypes.c_double), ("dbeta_rad", ctypes.c_double), ("fan_sign", ctypes.c_double)]


@dataclass
class FilterGeometry:
    """Geometry of FDK preprocessing (fdk_filter_geometry): detector pitch,
    principal point (pixels), distances (mm), gantry angles (rad, from the
    scan start), short-scan range (<= 0: no Parker weights), angular step,
    orientation of the fan angle."""
    angles_rad: np.ndarray
    width: int
    height: int
    pixel_u_mm: float
    pixel_v_mm: float
    u0: float
    v0: float
    sdd_mm: float
    sid_mm: float
    scan_range_rad: float
    dbeta_rad: float
    fan_sign: float = -1.0
    _a: np.ndarray = field(init=False, repr=False)

    def __post_init__(self):
        self._a = np.ascontiguousarray(np.asarray(self.angles_rad, dtype=np.float64).ravel())

    @property
    def n_proj(self) -> int:
        return self._a.shape[0]

    def c(self) -> _FilterGeom:
        g = _FilterGeom()
        g.n_proj, g.width, g.height, g.reserved = self.n_proj, self.width, self.height, 0
        g.pixel_u_mm, g.pixel_v_mm, g.u0, g.v0 = self.pixel_u_mm, self.pixel_v_mm, self.u0, self.v0
        g.sdd_mm, g.sid_mm = self.sdd_mm, self.sid_mm
        g.angles_rad = self._a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        g.scan_range_rad, g.dbeta_rad, g.fan_sign = self.scan_range_rad, self.dbeta_rad, self.fan_sign
        return g


def filter_projections(lineint: torch.Tensor, fgeom: FilterGeometry, dtype=torch.float32,
                       out: torch.Tensor = None, stream=None):
    """FDK preprocessing (cosine and Parker weights, ramp filter along rows)
    of an (N, H, W) FP32 stack on the device.  Returns the filtered stack,
    and for dtype float16 / bfloat16 also the per-projection scale of the
    packed form (None for float32)."""
    lib = load()
    if lineint.dim() != 3 or tuple(lineint.shape) != (fgeom.n_proj, fgeom.height, fgeom.width):
        raise FdkError(-1, f"stack {tuple(lineint.shape)} does not match the filter geometry")
    if dtype not in _TORCH_DTYPE:
        raise FdkError(-3, f"output dtype {dtype}")
    src = _dev_ptr(lineint, "lineint", (torch.float32,))
    if out is None:
        out = torch.empty(tuple(lineint.shape), dtype=dtype, device=lineint.device)
    elif tuple(out.shape) != tuple(lineint.shape):
        raise FdkError(-1, "output stack has the wrong shape")
    dst = _dev_ptr(out, "out", (dtype,))
    scale = None
    if dtype != torch.float32:
        scale = torch.empty(fgeom.n_proj, dtype=torch.float32, device=lineint.device)
    g = fgeom.c()
    _check(lib.fdk_filter_projections(ctypes.byref(g), src, dst, _TORCH_DTYPE[dtype],
                                      scale.data_ptr() if scale is not None else None, _stream(stream)))
    return out, scale


def _solver_args(proj, geom, vol, x0, name):
    if proj.dtype != torch.float32:
        raise FdkError(-3, f"{name} takes float32 projections, got {proj.dtype}")
    if tuple(proj.shape) != (geom.n_proj, geom.height, geom.width):
        raise FdkError(-1, f"projections {tuple(proj.shape)} do not match geometry "
                           f"{(geom.n_proj, geom.height, geom.width)}")
    shape = (vol.planes, vol.L, vol.L)
    if x0 is None:
        out = torch.empty(shape, dtype=torch.float32, device=proj.device)
    else:
        if tuple(x0.shape) != shape or x0.dtype != torch.float32:
            raise FdkError(-1, "start volume has the wrong shape or dtype")
        out = x0.detach().clone().contiguous()
    return out


def cgls(proj: torch.Tensor, geom: Geometry, vol: Volume, n_iter: int, x0: torch.Tensor = None,
         history: bool = False, stream=None):
    """fdk_cgls: n_iter CGLS iterations for min ||A x - p|| with A the
    forward projector.  Returns the volume, and with history=True also the
    float64 tensor of ||r_k||^2, k = 0 .. n_iter."""
    lib = load()
    out = _solver_args(proj, geom, vol, x0, "cgls")
    hist = torch.empty(n_iter + 1, dtype=torch.float64, device=proj.device) if history else None
    v = vol.c()
    p = geom.c(_dev_ptr(proj, "projections"), F32)
    _check(lib.fdk_cgls(ctypes.byref(v), ctypes.byref(p), out.data_ptr(), int(n_iter), int(x0 is not None),
                        hist.data_ptr() if hist is not None else None, _stream(stream)))
    return (out, hist) if history else out


def sirt(proj: torch.Tensor, geom: Geometry, vol: Volume, n_iter: int, lam: float = 1.0,
         x0: torch.Tensor = None, nonneg: bool = False, history: bool = False, stream=None):
    """fdk_sirt: n_iter SIRT updates x += lam C A^T R (p - A x).  Returns the
    volume, and with history=True also ||p - A x_k||^2, k = 0 .. n_iter - 1."""
    lib = load()
    out = _solver_args(proj, geom, vol, x0, "sirt")
    hist = torch.empty(max(n_iter, 1), dtype=torch.float64, device=proj.device) if history else None
    flags = (1 if x0 is not None else 0) | (2 if nonneg else 0)
    v = vol.c()
    p = geom.c(_dev_ptr(proj, "projections"), F32)
    _check(lib.fdk_sirt(ctypes.byref(v), ctypes.byref(p), out.data_ptr(), int(n_iter), float(lam), flags,
                        hist.data_ptr() if hist is not None else None, _stream(stream)))
    return (out, hist[:n_iter]) if history else out


def set_tile(dtype: int, strip: int, waves: int, layout: int = 0) -> None:
    """Pin (strip, waves, layout) for a dtype; (0, 0) restores the automatic choice."""
    _check(load().fdk_set_tile(dtype, strip, waves, layout))


def get_tile(vol: Volume, dtype: int = F32) -> tuple[int, int, int]:
    """(strip, waves, layout) a call with this grid and dtype would use."""
    s, w, lay = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    v = vol.c()
    _check(load().fdk_get_tile(ctypes.byref(v), dtype, ctypes.byref(s), ctypes.byref(w),
                               ctypes.byref(lay)))
    return s.value, w.value, lay.value


def load_tuning(path: str) -> int:
    n = load().fdk_load_tuning(path.encode())
    if n < 0:
        _check(n)
    return n


def set_tuning_entry(dtype: int, size_class: int, strip: int, waves: int, layout: int = 0) -> None:
    _check(load().fdk_set_tuning_entry(dtype, size_class, strip, waves, layout))


def validate(geom: Geometry, vol: Volume, need_data: bool = False, dtype: int = F32) -> None:
    """Host-side argument check (no GPU work); raises FdkError."""
    v = vol.c()
    p = geom.c(1 if need_data else None, dtype)
    _check(load().fdk_validate(ctypes.byref(v), ctypes.byref(p), int(need_data)))


def normalize_matrices(mats) -> np.ndarray:
    """fdk_normalize_matrices on a copy: (N, 3, 4) float64 matrices scaled so
    that ||A[2, :3]|| = 1 and w > 0 at the origin."""
    m = np.array(mats, dtype=np.float64, copy=True).reshape(-1, 12)
    _check(load().fdk_normalize_matrices(m.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), m.shape[0]))
    return m.reshape(-1, 3, 4)


def release_workspace() -> None:
    _check(load().fdk_release_workspace())


def profile_enable(enable: bool = True) -> None:
    """Start (and clear) or stop per-launch HIP-event timing inside the library."""
    _check(load().fdk_profile_enable(int(bool(enable))))


def profile_read(kernel: str) -> tuple[int, float]:
    """(launches, total milliseconds) of one kernel kind since profile_enable."""
    n, ms = ctypes.c_int64(), ctypes.c_double()
    _check(load().fdk_profile_read(kernel.encode(), ctypes.byref(n), ctypes.byref(ms)))
    return n.value, ms.value


def abi_version() -> int:
    return int(load().fdk_abi_version())


class BackProject(torch.autograd.Function):
    """V = B p.  Gradient with respect to p: B^T grad_V (the forward projector)."""

    @staticmethod
    def forward(ctx, proj, geom: Geometry, vol: Volume):
        ctx.geom, ctx.vol = geom, vol
        return backproject(proj.contiguous(), geom, vol)

    @staticmethod
    def backward(ctx, grad_v):
        g = forwardproject(grad_v.contiguous().to(torch.float32), ctx.geom, ctx.vol)
        return g, None, None


class ForwardProject(torch.autograd.Function):
    """p = B^T V.  Gradient with respect to V: B grad_p (the backprojector)."""

    @staticmethod
    def forward(ctx, volume, geom: Geometry, vol: Volume):
        ctx.geom, ctx.vol = geom, vol
        return forwardproject(volume.contiguous(), geom, vol)

    @staticmethod
    def backward(ctx, grad_p):
        g = backproject(grad_p.contiguous().to(torch.float32), ctx.geom, ctx.vol)
        return g, None, None
