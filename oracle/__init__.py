"""FP64 oracle for voxel-driven FDK backprojection and its adjoint.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.

The arithmetic lives in ``fdk_oracle.c`` (plain loops, FP64); this module only
marshals numpy arrays into it.  Matrices are (N, 3, 4) row-major FP64;
projections (N, H, W); volumes (nz, L, L) with index (z, y, x).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdk_oracle.c")
_SRC_FILTER = os.path.join(_HERE, "fdk_filter_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (OpenMP, FP64, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared", "-fPIC",
                        "-std=gnu11", "-o", tmp, _SRC, _SRC_FILTER, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        lib.oracle_backproject.argtypes = [_i64, ctypes.c_double, _dp, _i64, _i64, _i64, _i64,
                                           _i64, _dp, _dp, _i64, _i64, _dp, ctypes.c_int]
        lib.oracle_backproject.restype = None
        lib.oracle_backproject_points.argtypes = [_i64, _ip, ctypes.c_double, _dp, _i64, _i64,
                                                  _i64, _dp, _dp, _dp]
        lib.oracle_backproject_points.restype = None
        lib.oracle_forwardproject.argtypes = [_i64, ctypes.c_double, _dp, _i64, _i64, _i64,
                                              _i64, _i64, _dp, _dp, _dp, ctypes.c_int]
        lib.oracle_forwardproject.restype = None
        lib.oracle_supported_updates.argtypes = [_i64, ctypes.c_double, _dp, _i64, _i64, _i64,
                                                 _i64, _i64, _dp]
        lib.oracle_supported_updates.restype = _i64
        lib.oracle_num_threads.restype = ctypes.c_int
        d = ctypes.c_double
        lib.oracle_parker_weight.argtypes = [d, d, d]
        lib.oracle_parker_weight.restype = d
        lib.oracle_ramp_kernel.argtypes = [_i64, d]
        lib.oracle_ramp_kernel.restype = d
        lib.oracle_fdk_filter.argtypes = [_i64, _i64, _i64, d, d, d, d, d, d, _dp, d, d, d, _dp, _dp]
        lib.oracle_fdk_filter.restype = None
        _lib = lib
    return _lib


def _f64(a) -> np.ndarray:
    if hasattr(a, "detach"):  # torch tensor
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _origin(L, voxel, origin):
    if origin is None:
        o = -(L - 1) * voxel / 2.0
        origin = (o, o, o)
    return np.ascontiguousarray(origin, dtype=np.float64)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def backproject(L: int, voxel: float, mats, proj, origin=None, z_range=None,
                k_range=None, init=None) -> np.ndarray:
    """V = sum_k bilinear(I_k, u/w, v/w) / w^2 over planes z_range=(z0, nz).

    ``init`` (nz, L, L) is accumulated onto when given."""
    lib = _load()
    mats = _f64(mats).reshape(-1, 12)
    proj = _f64(proj)
    N, H, W = proj.shape
    assert mats.shape[0] == N
    z0, nz = (0, L) if z_range is None else z_range
    k0, k1 = (0, N) if k_range is None else k_range
    org = _origin(L, voxel, origin)
    if init is None:
        vol = np.zeros((nz, L, L))
        acc = 0
    else:
        vol = _f64(init).reshape(nz, L, L).copy()
        acc = 1
    lib.oracle_backproject(L, float(voxel), _ptr(org), z0, nz, N, W, H, _ptr(mats), _ptr(proj),
                           k0, k1, _ptr(vol), acc)
    return vol


def backproject_points(xyz, voxel: float, mats, proj, L: int | None = None,
                       origin=None) -> np.ndarray:
    """Backprojection at voxels xyz (P, 3) int (x, y, z), one by one."""
    lib = _load()
    mats = _f64(mats).reshape(-1, 12)
    proj = _f64(proj)
    N, H, W = proj.shape
    pts = np.ascontiguousarray(xyz, dtype=np.int32).reshape(-1, 3)
    if origin is None:
        assert L is not None
    org = _origin(L, voxel, origin)
    out = np.zeros(pts.shape[0])
    lib.oracle_backproject_points(pts.shape[0], pts.ctypes.data_as(_ip), float(voxel), _ptr(org),
                                  N, W, H, _ptr(mats), _ptr(proj), _ptr(out))
    return out


def forwardproject(L: int, voxel: float, mats, vol, W: int, H: int, origin=None,
                   z_range=None, init=None) -> np.ndarray:
    """Adjoint B^T: scatter vol (nz, L, L) onto (N, H, W) detector pixels."""
    lib = _load()
    mats = _f64(mats).reshape(-1, 12)
    N = mats.shape[0]
    z0, nz = (0, L) if z_range is None else z_range
    v = _f64(vol).reshape(nz, L, L)
    org = _origin(L, voxel, origin)
    if init is None:
        out = np.zeros((N, H, W))
        acc = 0
    else:
        out = _f64(init).reshape(N, H, W).copy()
        acc = 1
    lib.oracle_forwardproject(L, float(voxel), _ptr(org), z0, nz, N, W, H, _ptr(mats), _ptr(v),
                              _ptr(out), acc)
    return out


def gradient(L: int, voxel: float, mats, proj, target, origin=None) -> np.ndarray:
    """Gradient of ||B p - V_t||^2 with respect to p: 2 B^T (B p - V_t)."""
    proj = _f64(proj)
    N, H, W = proj.shape
    r = backproject(L, voxel, mats, proj, origin) - _f64(target).reshape(L, L, L)
    return 2.0 * forwardproject(L, voxel, mats, r, W, H, origin)


def supported_updates(L: int, voxel: float, mats, W: int, H: int, origin=None,
                      z_range=None) -> int:
    """Count of (voxel, projection) pairs whose sample touches the detector."""
    lib = _load()
    mats = _f64(mats).reshape(-1, 12)
    N = mats.shape[0]
    z0, nz = (0, L) if z_range is None else z_range
    org = _origin(L, voxel, origin)
    return int(lib.oracle_supported_updates(L, float(voxel), _ptr(org), z0, nz, N, W, H,
                                            _ptr(mats)))


def parker_weight(beta: float, gamma: float, scan_range: float) -> float:
    """Short-scan weight of the ray at fan angle gamma in the view at gantry
    angle beta (Parker 1982); scan_range <= 0 means no weighting."""
    return float(_load().oracle_parker_weight(float(beta), float(gamma), float(scan_range)))


def ramp_kernel(n: int, tau: float) -> float:
    """Band-limited ramp filter tap h(n) at sample spacing tau (Kak & Slaney)."""
    return float(_load().oracle_ramp_kernel(int(n), float(tau)))


def fdk_filter(proj, pixel_u: float, pixel_v: float, u0: float, v0: float, sdd: float, sid: float,
               beta, scan_range: float, dbeta: float, fan_sign: float = -1.0) -> np.ndarray:
    """FDK preprocessing (cosine weight, Parker weight, ramp convolution along
    rows, scale t * dbeta * SID^2) of line integrals proj (N, H, W), FP64,
    direct convolution.  See fdk_filter_oracle.c for the formulas."""
    p = _f64(proj)
    N, H, W = p.shape
    b = _f64(beta).ravel()
    assert b.size == N
    q = np.empty_like(p)
    _load().oracle_fdk_filter(N, W, H, float(pixel_u), float(pixel_v), float(u0), float(v0), float(sdd),
                              float(sid), _ptr(b), float(scan_range), float(dbeta), float(fan_sign),
                              _ptr(p), _ptr(q))
    return q


def rel_l2(x, ref) -> float:
    """||x - ref||_2 / ||ref||_2 in FP64."""
    x = _f64(x).ravel()
    ref = _f64(ref).ravel()
    return float(np.linalg.norm(x - ref) / np.linalg.norm(ref))


def psnr(x, ref) -> float:
    """10 log10((max ref - min ref)^2 / MSE), FP64 over all voxels."""
    x = _f64(x).ravel()
    ref = _f64(ref).ravel()
    mse = float(np.mean((x - ref) ** 2))
    rng = float(ref.max() - ref.min())
    return float("inf") if mse == 0 else 10.0 * np.log10(rng * rng / mse)
