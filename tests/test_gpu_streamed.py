"""Out-of-core backprojection (fdk_backproject_streamed): projections in host
memory streamed to the device one detector row band per z-slab, and volumes
kept in host memory, against the FP64 oracle and against the in-core call."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from tests._common import assert_parity, ensure_built

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def fdk():
    ensure_built()
    import paper_1401_3615_amd as m
    m.load()
    return m


def _case(tilt=2.0, H=48, n=14, W=96, seed=0):
    """A detector only 48 rows high (60 mm at the isocentre): the top and
    bottom slabs of the 128 mm volume reach part of it or none of it."""
    carm = S.CArm(n, W, H, pixel=384.0 / W, tilt_deg=tilt)
    mats = S.carm_matrices(carm)
    proj = torch.from_numpy(S.random_projections(n, H, W, seed))
    return mats, proj


def _incore(fdk, proj, geom, vol, **kw):
    out = fdk.backproject(proj.to(DEV), geom, vol, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("slab", [1, 5, 16, 37])
def test_streamed_matches_oracle_and_incore(fdk, slab):
    mats, proj = _case()
    L, voxel = 37, 128.0 / 37
    geom, vol = fdk.Geometry(mats, 96, 48), fdk.Volume(L, voxel)
    host = proj.pin_memory()
    out = fdk.backproject_streamed(host, geom, vol, slab)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref = oracle.backproject(L, voxel, mats, proj.numpy())
    assert_parity(got, ref, what=f"streamed slab={slab}")
    inc = _incore(fdk, proj, geom, vol)
    assert oracle.rel_l2(got, inc) <= 1e-6


def test_streamed_host_volume_accumulate(fdk):
    mats, proj = _case(seed=1)
    L, voxel = 37, 128.0 / 37
    geom, vol = fdk.Geometry(mats, 96, 48), fdk.Volume(L, voxel)
    init = torch.randn((L, L, L), generator=torch.Generator().manual_seed(2)) * 1e-6
    out = init.clone().pin_memory()
    res = fdk.backproject_streamed(proj.pin_memory(), geom, vol, 6, out=out, accumulate=True)
    torch.cuda.synchronize()
    assert res is out and not out.is_cuda
    ref = oracle.backproject(L, voxel, mats, proj.numpy(), init=init.numpy())
    assert_parity(out.numpy(), ref, what="host volume, accumulate")


def test_streamed_pageable_and_device_sources(fdk):
    """Pageable host memory (copied synchronously by the runtime) and a
    device-resident stack both give the in-core result; a pageable host
    volume too."""
    mats, proj = _case(tilt=0.0, seed=3)
    L, voxel = 32, 4.0
    geom, vol = fdk.Geometry(mats, 96, 48), fdk.Volume(L, voxel)
    inc = _incore(fdk, proj, geom, vol)
    a = fdk.backproject_streamed(proj.clone(), geom, vol, 7)
    b = fdk.backproject_streamed(proj.to(DEV), geom, vol, 7)
    c = torch.empty((L, L, L))
    fdk.backproject_streamed(proj.clone(), geom, vol, 7, out=c)
    torch.cuda.synchronize()
    for name, got in (("pageable", a.cpu().numpy()), ("device", b.cpu().numpy()), ("host volume", c.numpy())):
        assert oracle.rel_l2(got, inc) <= 1e-6, name


def test_streamed_slab_of_a_slab_and_fp16(fdk):
    """A z-range of the grid, streamed in slabs, from an FP16 stack with its
    device scale, against the in-core FP16 call on the same range."""
    mats, proj = _case(seed=4)
    L, voxel = 40, 3.2
    geom = fdk.Geometry(mats, 96, 48)
    part = fdk.Volume(L, voxel).slab(7, 26)
    packed, scale = fdk.pack_projections(proj.to(DEV), torch.float16)
    inc = _incore(fdk, packed, geom, part, scale=scale)
    got = fdk.backproject_streamed(packed.cpu().pin_memory(), geom, part, 9, scale=scale)
    torch.cuda.synchronize()
    assert oracle.rel_l2(got.cpu().numpy(), inc) <= 1e-6


@pytest.mark.parametrize("W", [97, 98, 96])
def test_streamed_device_stack_row_widths(fdk, W):
    """Device-resident FP16 stacks are gathered into bands by a kernel that
    copies rows in 2-, 4- or 16-byte units depending on the row length."""
    carm = S.CArm(10, W, 48, pixel=384.0 / W, tilt_deg=1.0)
    mats = S.carm_matrices(carm)
    proj = torch.from_numpy(S.random_projections(10, 48, W, 6))
    geom, vol = fdk.Geometry(mats, W, 48), fdk.Volume(30, 4.0)
    packed, scale = fdk.pack_projections(proj.to(DEV), torch.float16)
    inc = _incore(fdk, packed, geom, vol, scale=scale)
    got = fdk.backproject_streamed(packed, geom, vol, 4, scale=scale)
    torch.cuda.synchronize()
    assert oracle.rel_l2(got.cpu().numpy(), inc) <= 1e-6


def test_streamed_buffers_grow_between_calls(fdk):
    mats, proj = _case(seed=5)
    geom = fdk.Geometry(mats, 96, 48)
    host = proj.pin_memory()
    for L, slab in ((24, 3), (40, 20), (33, 11)):
        vol = fdk.Volume(L, 128.0 / L)
        got = fdk.backproject_streamed(host, geom, vol, slab, out=torch.empty((L, L, L)).pin_memory())
        torch.cuda.synchronize()
        ref = oracle.backproject(L, 128.0 / L, mats, proj.numpy())
        assert_parity(got.numpy(), ref, what=f"L={L} slab={slab}")


def test_streamed_full_size(fdk):
    """512^3 @ 0.5 mm from 496 x 1248x960 filtered projections in pinned host
    memory, slabs of 64 planes: equal to the in-core call, and to the oracle at
    seeded voxels."""
    carm = S.CArm(496)
    mats, q = S.filtered_projections(carm, seed=0, device=DEV)
    geom, vol = fdk.Geometry(mats, 1248, 960), fdk.Volume(512, 0.5)
    inc = fdk.backproject(q.contiguous(), geom, vol)
    host = q.cpu().pin_memory()
    got = fdk.backproject_streamed(host, geom, vol, 64)
    torch.cuda.synchronize()
    err = float(((got.double() - inc.double()).norm() / inc.double().norm()).item())
    assert err <= 1e-6, err
    rng = np.random.default_rng(11)
    xyz = np.concatenate([rng.integers(0, 512, size=(1500, 3)),
                          np.array([[0, 0, 0], [511, 511, 511], [256, 256, 63], [256, 256, 64], [100, 400, 448]])])
    ref = oracle.backproject_points(xyz, 0.5, mats, host.numpy(), L=512)
    g = got[torch.from_numpy(xyz[:, 2]), torch.from_numpy(xyz[:, 1]), torch.from_numpy(xyz[:, 0])].cpu().numpy()
    scale = np.abs(ref).max()
    assert np.abs(g - ref).max() <= 1e-4 * scale


def test_streamed_waits_for_caller_stream(fdk):
    """A device stack written on the caller's stream just before the call
    (packed there, no host synchronisation in between) is gathered only after
    it is written: the library's copy stream waits for the caller's."""
    mats, proj = _case(tilt=1.0, seed=12)
    L, voxel = 30, 4.0
    geom, vol = fdk.Geometry(mats, 96, 48), fdk.Volume(L, voxel)
    ref = oracle.backproject(L, voxel, mats, proj.numpy())
    src = proj.to(DEV)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        # a long queue of work ahead of the pack keeps it from finishing early
        junk = torch.randn((2048, 2048), device=DEV)
        for _ in range(20):
            junk = junk @ junk
            junk = junk / junk.abs().max()
        stack = src * 2.0
        got = fdk.backproject_streamed(stack, geom, vol, 4, stream=side)
        got2 = fdk.backproject_streamed(stack * 0.5, geom, vol, 7, stream=side)
    side.synchronize()
    assert_parity(got.cpu().numpy(), 2.0 * ref, what="streamed after pack on a side stream")
    assert_parity(got2.cpu().numpy(), ref, what="second call, other slabs")


def test_streamed_many_slabs_repeat(fdk):
    """More slabs than there are cached geometries: repeated calls reuse the
    one table composed for all slabs of a call."""
    mats, proj = _case(seed=13)
    L, voxel = 40, 3.2
    geom, vol = fdk.Geometry(mats, 96, 48), fdk.Volume(L, voxel)
    ref = oracle.backproject(L, voxel, mats, proj.numpy())
    host = proj.pin_memory()
    for _ in range(3):
        got = fdk.backproject_streamed(host, geom, vol, 1)   # 40 slabs
        torch.cuda.synchronize()
        assert_parity(got.cpu().numpy(), ref, what="40 one-plane slabs")
