"""Host-side tests of the C ABI (no GPU needed): the library loads, exports
every entry point declared in include/fdk.h, and rejects bad arguments on
the host before touching the device."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import synthetic as S
from tests._common import ROOT, ensure_built


@pytest.fixture(scope="module")
def fdk():
    ensure_built()
    import paper_1401_3615_amd as m
    m.load()
    return m


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "fdk.h")).read()
    return sorted(set(re.findall(r"\b(fdk_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(fdk):
    lib = fdk.load()
    names = declared_symbols()
    assert len(names) >= 13
    for n in names:
        assert hasattr(lib, n), n
    assert fdk.abi_version() == 1


def test_status_strings(fdk):
    lib = fdk.load()
    for code, name in [(0, b"FDK_OK"), (-1, b"FDK_E_INVALID_ARG"), (-2, b"FDK_E_GEOMETRY"),
                       (-3, b"FDK_E_UNSUPPORTED"), (-4, b"FDK_E_NOMEM"), (-5, b"FDK_E_DEVICE")]:
        assert lib.fdk_status_string(code) == name


def _case(L=16, N=4, W=32, H=24):
    mats = S.tiny_cone_matrices(N, W, H, L, 1.0, 0)
    return mats, W, H


def test_validate_accepts_good_geometry(fdk):
    mats, W, H = _case()
    fdk.validate(fdk.Geometry(mats, W, H), fdk.Volume(16, 1.0))


@pytest.mark.parametrize("mutate,status", [
    (lambda v, g: setattr(v, "L", 0), -1),
    (lambda v, g: setattr(v, "voxel_mm", 0.0), -1),
    (lambda v, g: setattr(v, "voxel_mm", float("nan")), -1),
    (lambda v, g: setattr(v, "z_begin", 16), -1),
    (lambda v, g: setattr(v, "z_count", 17), -1),
    (lambda v, g: setattr(v, "origin_mm", (0.0, float("inf"), 0.0)), -1),
    (lambda v, g: setattr(g, "width", 0), -1),
    (lambda v, g: setattr(g, "height", 1 << 23), -1),
])
def test_validate_rejects(fdk, mutate, status):
    mats, W, H = _case()
    g = fdk.Geometry(mats, W, H)
    v = fdk.Volume(16, 1.0, z_begin=0, z_count=16)
    mutate(v, g)
    with pytest.raises(fdk.FdkError) as ei:
        fdk.validate(g, v)
    assert ei.value.status == status


def test_validate_rejects_nonfinite_matrix(fdk):
    mats, W, H = _case()
    mats[2, 1, 3] = np.nan
    with pytest.raises(fdk.FdkError) as ei:
        fdk.validate(fdk.Geometry(mats, W, H), fdk.Volume(16, 1.0))
    assert ei.value.status == -1
    assert "matrix 2" in str(ei.value)


def test_geometry_error_names_projection_and_corner(fdk):
    mats, W, H = _case()
    mats[3] = -mats[3]
    with pytest.raises(fdk.FdkError) as ei:
        fdk.validate(fdk.Geometry(mats, W, H), fdk.Volume(16, 1.0))
    assert ei.value.status == -2
    assert "projection 3" in str(ei.value)


def test_geometry_checked_on_processed_slab_only(fdk):
    """w <= 0 only in planes outside the slab is accepted for that slab."""
    L = 16
    mats = np.zeros((1, 3, 4))
    mats[0, 0, 0] = mats[0, 1, 1] = 1.0
    mats[0, 2, 2] = 1.0  # w = Z: positive only for z > 0 in world terms
    vol_all = fdk.Volume(L, 1.0, origin_mm=(0.0, 0.0, -7.5))
    with pytest.raises(fdk.FdkError):
        fdk.validate(fdk.Geometry(mats, 8, 8), vol_all)
    fdk.validate(fdk.Geometry(mats, 8, 8), vol_all.slab(8, 8))


def test_unsupported_dtype(fdk):
    mats, W, H = _case()
    lib = fdk.load()
    v = fdk.Volume(16, 1.0).c()
    p = fdk.Geometry(mats, W, H).c(data=1, dtype=7)
    assert lib.fdk_validate(ctypes.byref(v), ctypes.byref(p), 1) == -3


def test_invalid_calls_do_not_touch_the_device(fdk):
    """Argument errors are reported before any HIP call (this host has no GPU)."""
    lib = fdk.load()
    mats, W, H = _case()
    v = fdk.Volume(16, 1.0).c()
    p = fdk.Geometry(mats, W, H).c(data=None)
    assert lib.fdk_backproject(ctypes.byref(v), ctypes.byref(p), 1, 0, None) == -1
    assert b"data is NULL" in lib.fdk_last_error()
    p = fdk.Geometry(mats, W, H).c(data=1)
    assert lib.fdk_backproject(ctypes.byref(v), ctypes.byref(p), None, 0, None) == -1
    assert lib.fdk_forwardproject(ctypes.byref(v), None, ctypes.byref(p), 1, 0, None) == -1
    assert lib.fdk_backproject(None, ctypes.byref(p), 1, 0, None) == -1
    assert lib.fdk_backproject_batched(None, 1, 0, None) == -1
    assert lib.fdk_pack_projections(1, 4, 8, 8, 0, 1, 1, None) == -3
    assert lib.fdk_pack_projections(None, 4, 8, 8, 1, 1, 1, None) == -1


def test_batched_reports_failing_scan(fdk):
    lib = fdk.load()
    mats, W, H = _case()
    bad = mats.copy()
    bad[0] = -bad[0]
    arr = (fdk._Scan * 3)()
    keep = []
    for i, m in enumerate([mats, mats, bad]):
        g = fdk.Geometry(m, W, H)
        keep.append(g)
        arr[i].vol = fdk.Volume(16, 1.0).c()
        arr[i].proj = g.c(data=1)
        arr[i].volume = 1
    assert lib.fdk_backproject_batched(arr, 3, 0, None) == -2
    assert b"scan 2" in lib.fdk_last_error()


def test_tiles_and_tuning_file(fdk, tmp_path):
    vol = fdk.Volume(512, 0.5)
    fdk.set_tile(fdk.F16, 4, 1, 1)
    assert fdk.get_tile(vol, fdk.F16) == (4, 1, 1)
    fdk.set_tile(fdk.F16, 0, 0)
    with pytest.raises(fdk.FdkError):
        fdk.set_tile(fdk.F32, 3, 1)
    with pytest.raises(fdk.FdkError):
        fdk.set_tile(fdk.F32, 4, 1, 4)
    f = tmp_path / "tune.txt"
    f.write_text("fdk-tuning 1 gfx950\n# dtype class strip waves layout\n0 9 8 1 0\n1 9 2 2 1\n")
    assert fdk.load_tuning(str(f)) == 2
    assert fdk.get_tile(vol, fdk.F32) == (8, 1, 0)
    assert fdk.get_tile(vol, fdk.F16) == (2, 2, 1)
    stale = tmp_path / "stale.txt"
    stale.write_text("fdk-tuning 0 gfx942\n0 9 4 4 0\n")
    with pytest.raises(fdk.FdkError):
        fdk.load_tuning(str(stale))
    assert fdk.get_tile(vol, fdk.F32) == (8, 1, 0)   # stale file ignored
    bad = tmp_path / "bad.txt"
    bad.write_text("fdk-tuning 1 gfx950\n0 9 5 1 0\n")
    with pytest.raises(fdk.FdkError):
        fdk.load_tuning(str(bad))
    fdk.set_tuning_entry(0, 9, 16, 2, 1)
    assert fdk.get_tile(vol, fdk.F32) == (16, 2, 1)
    for dt in (0, 1):
        fdk.set_tuning_entry(dt, 9, 0, 0)   # restore the built-in choice
    assert fdk.get_tile(vol, fdk.F32) == fdk.get_tile(vol, fdk.F32)


def test_adjoint_tiles(fdk):
    vol = fdk.Volume(256, 1.0)
    assert fdk.get_tile(vol, fdk.TUNE_ADJOINT) == (60, 1, 4)
    for bad in [(16, 3, 4), (509, 8, 4), (0, 1, 4), (16, 4, 3), (16, 4, 1), (5, 1, 0)]:
        with pytest.raises(fdk.FdkError):
            fdk.set_tile(fdk.TUNE_ADJOINT, *bad)
    for good in [(1, 1, 4), (508, 8, 4), (4092, 1, 4), (8, 2, 0)]:
        fdk.set_tile(fdk.TUNE_ADJOINT, *good)
        assert fdk.get_tile(vol, fdk.TUNE_ADJOINT) == good
    fdk.set_tile(fdk.TUNE_ADJOINT, 0, 0)
    assert fdk.get_tile(vol, fdk.TUNE_ADJOINT) == (60, 1, 4)
    # large volumes: two projections per workgroup on 36-row tiles
    assert fdk.get_tile(fdk.Volume(512, 0.5), fdk.TUNE_ADJOINT) == (36, 2, 4)


def test_batched_slot(fdk):
    vol = fdk.Volume(256, 1.0)
    assert fdk.get_tile(vol, fdk.TUNE_BATCHED) == fdk.get_tile(vol, fdk.F32)   # default follows FP32
    fdk.set_tile(fdk.TUNE_BATCHED, 8, 2, 1)
    try:
        assert fdk.get_tile(vol, fdk.TUNE_BATCHED) == (8, 2, 1)
        with pytest.raises(fdk.FdkError):
            fdk.set_tile(fdk.TUNE_BATCHED, 8, 2, 4)
    finally:
        fdk.set_tile(fdk.TUNE_BATCHED, 0, 0)
    with pytest.raises(fdk.FdkError):
        fdk.set_tile(5, 8, 2, 0)   # no such slot


def test_header_struct_layout(fdk):
    """The ctypes mirror has the sizes the C structs have."""
    assert ctypes.sizeof(fdk._Volume) == 48
    assert ctypes.sizeof(fdk._Proj) == 40
    assert ctypes.sizeof(fdk._Scan) == 96


def test_autotune_file_round_trip(fdk, tmp_path):
    """The autotuner's writer produces a file the library's loader accepts."""
    from paper_1401_3615_amd import autotune
    res = [autotune.Result(0, 9, 16, 4, 3, 1000.0), autotune.Result(1, 8, 8, 2, 1, 900.0),
           autotune.Result(3, 8, 16, 2, 4, 400.0)]
    path = tmp_path / "tuned.txt"
    autotune.write(res, str(path))
    assert path.read_text().startswith(f"fdk-tuning {fdk.abi_version()} gfx950\n")
    try:
        assert fdk.load_tuning(str(path)) == 3
        assert fdk.get_tile(fdk.Volume(512, 0.5), fdk.F32) == (16, 4, 3)
        assert fdk.get_tile(fdk.Volume(300, 0.5), fdk.F16) == (8, 2, 1)
        assert fdk.get_tile(fdk.Volume(256, 0.5), fdk.TUNE_ADJOINT) == (16, 2, 4)
    finally:
        for r in res:
            fdk.set_tuning_entry(r.slot, r.size_class, 0, 0)
    for slot in (fdk.F32, fdk.F16, fdk.BF16, fdk.TUNE_ADJOINT):
        for strip, waves, layout in autotune.candidates(slot):
            fdk.set_tile(slot, strip, waves, layout)   # every candidate is a compiled shape
        fdk.set_tile(slot, 0, 0)


def test_filter_validation(fdk):
    """Host-side checks of fdk_filter_projections (no device work)."""
    import numpy as np
    lib = fdk.load()

    def g(**kw):
        base = dict(angles_rad=np.linspace(0, 3.49, 4), width=64, height=8, pixel_u_mm=1.0, pixel_v_mm=1.0,
                    u0=31.5, v0=3.5, sdd_mm=1200.0, sid_mm=750.0, scan_range_rad=3.49, dbeta_rad=0.1,
                    fan_sign=-1.0)
        base.update(kw)
        return fdk.FilterGeometry(**base)

    cases = [(g(width=2049), -1), (g(fan_sign=0.5), -1), (g(sdd_mm=-1.0), -1), (g(pixel_u_mm=float("nan")), -1),
             (g(scan_range_rad=3.2, pixel_u_mm=10.0), -2), (g(width=0), -1)]
    for geom, code in cases:
        c = geom.c()
        assert lib.fdk_filter_projections(ctypes.byref(c), 1, 1, 0, None, None) == code, lib.fdk_last_error()
    c = g().c()
    assert lib.fdk_filter_projections(ctypes.byref(c), None, 1, 0, None, None) == -1
    assert lib.fdk_filter_projections(ctypes.byref(c), 1, 1, 1, None, None) == -1   # packed needs scale_out
    assert lib.fdk_filter_projections(ctypes.byref(c), 1, 1, 7, None, None) == -3
    c.reserved = 1
    assert lib.fdk_filter_projections(ctypes.byref(c), 1, 1, 0, None, None) == -1
    assert lib.fdk_filter_projections(None, 1, 1, 0, None, None) == -1
    assert ctypes.sizeof(fdk._FilterGeom) == 96


def test_solver_validation(fdk):
    """Host-side checks of fdk_cgls / fdk_sirt (no device work)."""
    lib = fdk.load()
    mats, W, H = _case()
    v = fdk.Volume(16, 1.0).c()
    p = fdk.Geometry(mats, W, H).c(1, fdk.F32)
    assert lib.fdk_cgls(ctypes.byref(v), ctypes.byref(p), None, 2, 0, None, None) == -1   # no volume
    assert lib.fdk_cgls(ctypes.byref(v), ctypes.byref(p), 1, -1, 0, None, None) == -1     # n_iter < 0
    assert lib.fdk_sirt(ctypes.byref(v), ctypes.byref(p), 1, 2, 0.0, 0, None, None) == -1  # lambda
    assert lib.fdk_sirt(ctypes.byref(v), ctypes.byref(p), 1, 2, float("nan"), 0, None, None) == -1
    assert lib.fdk_sirt(ctypes.byref(v), ctypes.byref(p), 1, 2, 1.0, 4, None, None) == -1  # flags
    p16 = fdk.Geometry(mats, W, H).c(1, fdk.F16)
    assert lib.fdk_cgls(ctypes.byref(v), ctypes.byref(p16), 1, 2, 0, None, None) == -3
    assert lib.fdk_sirt(ctypes.byref(v), ctypes.byref(p16), 1, 2, 1.0, 0, None, None) == -3
    p0 = fdk.Geometry(mats, W, H).c(None, fdk.F32)
    assert lib.fdk_cgls(ctypes.byref(v), ctypes.byref(p0), 1, 2, 0, None, None) == -1     # no data
    behind = mats.copy()
    behind[1] *= -1.0
    pb = fdk.Geometry(behind, W, H).c(1, fdk.F32)
    assert lib.fdk_cgls(ctypes.byref(v), ctypes.byref(pb), 1, 2, 0, None, None) == -2
    assert lib.fdk_sirt(ctypes.byref(v), ctypes.byref(pb), 1, 2, 1.0, 0, None, None) == -2
    assert b"projection 1" in lib.fdk_last_error()


@pytest.mark.parametrize("tilt,H,slab", [(0.0, 72, 5), (3.0, 72, 8), (0.0, 24, 6), (2.0, 24, 40)])
def test_streamed_plan_covers_every_tap(fdk, tilt, H, slab):
    """Host-side slab plan of fdk_backproject_streamed: every detector row a
    voxel of the slab can sample (floor(iy) .. floor(iy) + 1, with a row of
    slack either side for FP32 coordinates) lies inside the projection's band,
    and every band lies on the detector, so off-detector taps stay off."""
    import numpy as np
    W, L, voxel = 96, 40, 4.0
    carm = S.CArm(12, W, H, pixel=384.0 / W, tilt_deg=tilt)
    mats = S.carm_matrices(carm)
    geom, vol = fdk.Geometry(mats, W, H), fdk.Volume(L, voxel)
    rows, first = fdk.streamed_plan(geom, vol, slab)
    assert len(rows) == -(-L // slab)
    assert np.all(rows >= 1) and np.all(rows <= H)
    assert np.all(first >= 0) and np.all(first + rows[:, None] <= H)
    o = S.default_origin(L, voxel)
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    X = np.stack([o[0] + x * voxel, o[1] + y * voxel, o[2] + z * voxel, np.ones(x.shape)], -1)
    for s in range(len(rows)):
        P = X[s * slab:(s + 1) * slab].reshape(-1, 4)
        for k in range(mats.shape[0]):
            uvw = P @ mats[k].T
            iy = uvw[:, 1] / uvw[:, 2]
            j = np.floor(iy)
            need_lo = np.clip(j - 1, 0, H - 1)
            need_hi = np.clip(j + 2, 0, H - 1)
            on = (iy > -2) & (iy < H + 1)
            assert np.all(need_lo[on] >= first[s, k]), (s, k)
            assert np.all(need_hi[on] < first[s, k] + rows[s]), (s, k)
    if H == 24 and slab < L:
        assert rows.min() < H   # some slab needs only part of the detector


def test_normalize_matrices(fdk):
    """Host-side: unit third row, w > 0 at the origin, projected positions
    unchanged; invalid inputs rejected."""
    import numpy as np
    mats, W, H = _case()
    rng = np.random.default_rng(3)
    scaled = mats * rng.uniform(-5.0, 5.0, size=(mats.shape[0], 1, 1))
    scaled[scaled[:, 2, 3] > 0] *= -1.0          # some with w < 0 at the origin
    out = fdk.normalize_matrices(scaled)
    np.testing.assert_allclose(np.linalg.norm(out[:, 2, :3], axis=1), 1.0, rtol=1e-15)
    assert np.all(out[:, 2, 3] > 0)
    X = np.concatenate([rng.normal(size=(20, 3)) * 4.0, np.ones((20, 1))], 1)
    for k in range(mats.shape[0]):
        a, b = X @ scaled[k].T, X @ out[k].T
        np.testing.assert_allclose(b[:, :2] / b[:, 2:], a[:, :2] / a[:, 2:], rtol=1e-12)
    np.testing.assert_allclose(out, fdk.normalize_matrices(mats), rtol=1e-13, atol=1e-13)
    bad = mats.copy()
    bad[1, 2, :3] = 0.0
    with pytest.raises(fdk.FdkError):
        fdk.normalize_matrices(bad)
    bad = mats.copy()
    bad[0, 0, 0] = float("nan")
    with pytest.raises(fdk.FdkError):
        fdk.normalize_matrices(bad)


def test_empty_and_limit_arguments(fdk):
    """Empty stacks, grids past the size limit and invalid slab sizes are
    rejected on the host."""
    import numpy as np
    lib = fdk.load()
    mats, W, H = _case()
    v = fdk.Volume(16, 1.0).c()
    empty = fdk.Geometry(np.zeros((0, 3, 4)), W, H)
    with pytest.raises(fdk.FdkError) as ei:
        fdk.validate(empty, fdk.Volume(16, 1.0))
    assert ei.value.status == -1
    with pytest.raises(fdk.FdkError) as ei:
        fdk.validate(fdk.Geometry(mats, W, H), fdk.Volume(32769, 1.0, z_count=1))
    assert ei.value.status == -1
    p = fdk.Geometry(mats, W, H).c(1, fdk.F32)
    for slab in (0, -3):
        assert lib.fdk_backproject_streamed(ctypes.byref(v), ctypes.byref(p), 1, slab, 0, 0, None) == -1
    assert lib.fdk_backproject_streamed(ctypes.byref(v), ctypes.byref(p), 1, 4, 2, 0, None) == -1   # flags
    assert lib.fdk_backproject_streamed(ctypes.byref(v), ctypes.byref(p), None, 4, 0, 0, None) == -1
    n = ctypes.c_int32()
    assert lib.fdk_streamed_plan(ctypes.byref(v), ctypes.byref(p), 0, ctypes.byref(n), None, None) == -1


def test_solver_history_must_be_device_memory(fdk):
    import numpy as np
    lib = fdk.load()
    mats, W, H = _case()
    v = fdk.Volume(16, 1.0).c()
    p = fdk.Geometry(mats, W, H).c(1, fdk.F32)
    host = np.zeros(4)
    assert lib.fdk_cgls(ctypes.byref(v), ctypes.byref(p), 1, 2, 0, host.ctypes.data, None) == -1
    assert b"history" in lib.fdk_last_error()
    assert lib.fdk_sirt(ctypes.byref(v), ctypes.byref(p), 1, 2, 1.0, 0, host.ctypes.data, None) == -1


def test_noalloc_limits_checked_on_host(fdk):
    """fdk_backproject_noalloc rejects FP16 data, more than 4096 projections
    and grids whose window table exceeds its scratch array, on the host,
    before any device access (the device pointers here are never touched)."""
    lib = fdk.load()
    fake = ctypes.c_void_p(0x1000)

    def call(L, N, dtype=0, W=32, H=24):
        mats = S.tiny_cone_matrices(N, W, H, L, 16.0 / L, 0)
        g, v = fdk.Geometry(mats, W, H), fdk.Volume(L, 16.0 / L)
        p = g.c(fake, dtype, None)
        return lib.fdk_backproject_noalloc(ctypes.byref(v.c()), ctypes.byref(p), fake, 0, None)

    assert call(16, 4, dtype=1) == -3
    assert call(16, 4097) == -1
    assert b"4096" in lib.fdk_last_error()
    # ceil(2048 / 16)^2 * 300 * 8 bytes = 39.3 MB per 16 planes > 31 MiB
    assert call(2048, 300) == -1
    assert b"window table" in lib.fdk_last_error()
