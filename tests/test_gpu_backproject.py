"""GPU parity of fdk_backproject against the FP64 oracle (through the C ABI)."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from tests._common import ELEM_TOL, REL_L2_FP32, assert_parity, ensure_built, small_carm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def fdk():
    ensure_built()
    import paper_1401_3615_amd as m
    m.load()
    return m


@pytest.fixture(scope="module")
def c0():
    """128^3 @ 0.5 mm from 124 filtered 1248x960 projections (phantom seed 0)."""
    carm = S.CArm(124)
    mats, q = S.filtered_projections(carm, 0, device=DEV)
    return carm, mats, q.contiguous()


def test_c0_fp32_full_volume(fdk, c0):
    carm, mats, q = c0
    L, voxel = 128, 0.5
    geom = fdk.Geometry(mats, carm.width, carm.height)
    out = fdk.backproject(q, geom, fdk.Volume(L, voxel))
    torch.cuda.synchronize()
    ref = oracle.backproject(L, voxel, mats, q.cpu().numpy())
    err = assert_parity(out.cpu().numpy(), ref, what="C0 fp32")
    print(f"C0 128^3x124 fp32 rel L2 {err:.3e} PSNR {oracle.psnr(out.cpu().numpy(), ref):.1f} dB")


@pytest.mark.parametrize("layout", [0, 1, 3])
def test_tilted_carm_general_path(fdk, layout):
    """A C-arm whose depth axis leaves the orbit plane (0.4 degree tilt, as in
    calibrated real systems): w changes along z, so the kernels take 1/w per
    voxel instead of once per strip; full 1248 x 960 detector."""
    carm = S.CArm(31, tilt_deg=0.4)
    mats, q = S.filtered_projections(carm, 11)
    assert np.all(mats[:, 2, 2] != 0.0)
    L, voxel = 72, 3.0
    fdk.set_tile(fdk.F32, 16, 4, layout)
    try:
        out = fdk.backproject(q.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.F32, 0, 0)
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    assert_parity(out.cpu().numpy(), ref, what=f"tilted C-arm layout {layout}")


@pytest.mark.parametrize("strip,waves", [(16, 4), (2, 1)])
@pytest.mark.parametrize("tilt", [0.0, 0.4])
def test_lds_windows_too_large(fdk, strip, waves, tilt):
    """4 mm voxels on the 0.308 mm-pixel detector: every tile's footprint
    exceeds the LDS tile, so every projection goes through the gather pass
    of the LDS kernel (constant-depth and per-voxel variants)."""
    carm = S.CArm(9, tilt_deg=tilt)
    mats, q = S.filtered_projections(carm, 12)
    L, voxel = 40, 4.0
    fdk.set_tile(fdk.F32, strip, waves, 3)
    try:
        out = fdk.backproject(q.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.F32, 0, 0)
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    assert_parity(out.cpu().numpy(), ref, what=f"oversized windows {strip}x{waves} tilt {tilt}")


def test_orbit_plane_geometry_is_constant_w():
    """The default C-arm has w independent of z exactly (the per-strip
    reciprocal path)."""
    mats = S.carm_matrices(S.CArm(8))
    assert np.all(mats[:, 2, 2] == 0.0)


@pytest.mark.parametrize("layout", [0, 1, 2, 3])
@pytest.mark.parametrize("strip,waves", [(2, 1), (2, 4), (4, 1), (4, 2), (8, 1), (8, 4),
                                         (16, 1), (16, 2), (16, 4), (2, 2), (4, 4), (8, 2),
                                         (32, 1), (32, 2), (32, 4)])
def test_every_tile_shape_ragged(fdk, strip, waves, layout):
    """L = 37 (ragged in x, y and z for every shape), odd detector 101 x 77,
    both staged layouts."""
    carm = small_carm(9, 101, 77)
    mats, q = S.filtered_projections(carm, 3)
    L, voxel = 37, 4.0
    geom = fdk.Geometry(mats, carm.width, carm.height)
    vol = fdk.Volume(L, voxel)
    fdk.set_tile(fdk.F32, strip, waves, layout)
    try:
        assert fdk.get_tile(vol, fdk.F32) == (strip, waves, layout)
        out = fdk.backproject(q.to(DEV), geom, vol)
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.F32, 0, 0)
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    assert_parity(out.cpu().numpy(), ref, what=f"tile {strip}x{waves}")


@pytest.mark.parametrize("seed", [1, 2])
def test_edges_partial_and_off_detector(fdk, seed):
    """A volume that overfills a tiny detector: voxels project off it, onto its
    edges and into (-1, 0); white-noise projections."""
    L, W, H, N, voxel = 21, 13, 9, 5, 1.0
    mats = S.tiny_cone_matrices(N, W, H, L, voxel, seed)
    p = S.random_projections(N, H, W, seed)
    geom = fdk.Geometry(mats, W, H)
    out = fdk.backproject(torch.from_numpy(p).to(DEV), geom, fdk.Volume(L, voxel))
    torch.cuda.synchronize()
    ref = oracle.backproject(L, voxel, mats, p)
    # off-detector voxels must be exactly zero
    got = out.cpu().numpy()
    assert np.array_equal(got[ref == 0.0], np.zeros(int((ref == 0.0).sum()), np.float32))
    assert_parity(got, ref, what="tiny cone")


def test_accumulate_and_slabs(fdk):
    carm = small_carm(15, 160, 128)
    mats, q = S.filtered_projections(carm, 4)
    L, voxel = 48, 2.5
    geom = fdk.Geometry(mats, carm.width, carm.height)
    qd = q.to(DEV)
    full = fdk.backproject(qd, geom, fdk.Volume(L, voxel))
    init = torch.randn(L, L, L, device=DEV)
    acc = init.clone()
    fdk.backproject(qd, geom, fdk.Volume(L, voxel), out=acc, accumulate=True)
    # z-slabs of uneven thickness written into views of one buffer
    slabbed = torch.full((L, L, L), float("nan"), device=DEV)
    for z0, nz in [(0, 5), (5, 17), (22, 26)]:
        fdk.backproject(qd, geom, fdk.Volume(L, voxel, z_begin=z0, z_count=nz), out=slabbed[z0:z0 + nz])
    torch.cuda.synchronize()
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    assert_parity(full.cpu().numpy(), ref, what="full")
    assert_parity(acc.cpu().numpy(), ref + init.cpu().numpy().astype(np.float64), what="accumulate")
    # a slab computes its planes as the full launch does (strips may group the
    # planes differently, so only FP32 rounding may differ)
    assert oracle.rel_l2(slabbed.cpu().numpy(), full.cpu().numpy()) < 1e-6


def test_projection_subsets_add_up(fdk):
    """Two calls over projection subsets with accumulate equal one call (to FP32 rounding)."""
    carm = small_carm(12, 128, 96)
    mats, q = S.filtered_projections(carm, 5)
    L, voxel = 32, 3.0
    g_all = fdk.Geometry(mats, carm.width, carm.height)
    g_a = fdk.Geometry(mats[:5], carm.width, carm.height)
    g_b = fdk.Geometry(mats[5:], carm.width, carm.height)
    qd = q.to(DEV)
    vol = fdk.Volume(L, voxel)
    one = fdk.backproject(qd, g_all, vol)
    two = fdk.backproject(qd[:5].contiguous(), g_a, vol)
    fdk.backproject(qd[5:].contiguous(), g_b, vol, out=two, accumulate=True)
    torch.cuda.synchronize()
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    assert_parity(two.cpu().numpy(), ref, what="subsets")
    assert oracle.rel_l2(two.cpu().numpy(), one.cpu().numpy()) < 1e-6


def test_degenerate_sizes(fdk):
    # L = 1, one projection, 1x1 detector: the voxel maps onto the only pixel
    mats = np.array([[[1.0, 0, 0, 0.25], [0, 1.0, 0, -0.5], [0, 0, 0, 2.0]]])
    p = np.array([[[3.0]]], np.float32)
    out = fdk.backproject(torch.from_numpy(p).to(DEV), fdk.Geometry(mats, 1, 1),
                          fdk.Volume(1, 1.0, origin_mm=(0.0, 0.0, 0.0)))
    ref = oracle.backproject(1, 1.0, mats, p, origin=(0.0, 0.0, 0.0))
    torch.cuda.synchronize()
    np.testing.assert_allclose(out.cpu().numpy().ravel(), ref.ravel(), rtol=1e-6)
    assert ref.ravel()[0] != 0.0


def test_all_voxels_off_detector(fdk):
    L, W, H, voxel = 16, 20, 10, 1.0
    mats = S.tiny_cone_matrices(3, W, H, L, voxel, 9)
    mats[:, 0, 3] += 1e6 * mats[:, 2, 3]  # shift u far past the detector
    p = np.ones((3, H, W), np.float32)
    out = torch.full((L, L, L), 7.0, device=DEV)
    fdk.backproject(torch.from_numpy(p).to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel), out=out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0


def test_geometry_error_leaves_output(fdk):
    L, W, H, voxel = 8, 12, 9, 1.0
    mats = S.tiny_cone_matrices(2, W, H, L, voxel, 2)
    mats[1] = -mats[1]  # w < 0 everywhere for projection 1
    out = torch.full((L, L, L), 5.0, device=DEV)
    with pytest.raises(fdk.FdkError) as ei:
        fdk.backproject(torch.ones(2, H, W, device=DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel), out=out)
    assert ei.value.status == -2
    torch.cuda.synchronize()
    assert torch.all(out == 5.0)


def test_scale_argument_fp32(fdk):
    """A per-projection scale multiplies each projection's contribution."""
    carm = small_carm(6, 96, 80)
    mats, q = S.filtered_projections(carm, 6)
    L, voxel = 24, 4.0
    s = np.array([0.5, 2.0, 1.0, 4.0, 0.25, 3.0], np.float32)
    out = fdk.backproject(q.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel),
                          scale=torch.from_numpy(s).to(DEV))
    torch.cuda.synchronize()
    ref = oracle.backproject(L, voxel, mats, q.numpy().astype(np.float64) * s[:, None, None])
    assert_parity(out.cpu().numpy(), ref, what="scale")


def test_non_default_stream(fdk):
    carm = small_carm(8, 128, 96)
    mats, q = S.filtered_projections(carm, 7)
    L, voxel = 40, 2.0
    geom = fdk.Geometry(mats, carm.width, carm.height)
    qd = q.to(DEV)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        out = fdk.backproject(qd, geom, fdk.Volume(L, voxel))
    st.synchronize()
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    assert_parity(out.cpu().numpy(), ref, what="stream")


@pytest.mark.parametrize("L,voxel,W,H,tilt,noise", [(12, 8.0, 160, 128, 0.0, True), (16, 24.0, 48, 40, 0.0, True),
                                                    (16, 12.0, 48, 40, 0.0, True), (10, 30.0, 256, 200, 1.0, False),
                                                    (9, 14.0, 61, 47, 2.0, True)])
def test_small_grid_reads_stack_in_place(fdk, L, voxel, W, H, tilt, noise):
    """Grids with fewer than one voxel per eight projection pixels read the
    FP32 stack in place (no staging): windows inside the detector, volumes
    overfilling it (edge windows, including the first and last image rows),
    footprints larger than the LDS tile (large voxels on a fine detector) and
    an odd width.  White-noise images make any misplaced pixel show; the
    large-footprint case takes filtered phantom projections instead, since
    with samples a hundred pixels from the centre the FP32 rounding of the
    sample position alone moves a white-noise backprojection by about 1e-5
    (relative), for the staged path as much as for this one."""
    carm = S.CArm(30, W, H, pixel=384.0 / W, tilt_deg=tilt)
    assert L ** 3 * 8 < 30 * W * H
    if noise:
        mats = S.carm_matrices(carm)
        proj = S.random_projections(30, H, W, 17)
    else:
        mats, q = S.filtered_projections(carm, 17)
        proj = q.numpy()
    fdk.set_tile(fdk.F32, 16, 4, 3)
    try:
        out = fdk.backproject(torch.from_numpy(proj).to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.F32, 0, 0)
    ref = oracle.backproject(L, voxel, mats, proj)
    assert_parity(out.cpu().numpy(), ref, what=f"in place L={L} W={W}")
