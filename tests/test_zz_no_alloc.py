"""The allocation-free backprojection (fdk_backproject_noalloc) against the
allocating entry point (fdk_backproject) and the oracle, through the C ABI:
two calls in a row on the one shared scratch array, the second smaller; a
full-size call that runs in several z-chunks; and no growth of the device
memory torch sees."""
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


def _case(n, W, H, seed, tilt=0.0):
    carm = S.CArm(n, W, H, pixel=384.0 / W, tilt_deg=tilt)
    return S.carm_matrices(carm), torch.from_numpy(S.random_projections(n, H, W, seed))


@pytest.mark.parametrize("tilt", [0.0, 1.0])
def test_noalloc_two_calls_second_smaller(fdk, tilt):
    cases = [(48, 2.5, 30, 160, 128, 1), (24, 4.0, 9, 96, 64, 2)]
    for L, voxel, n, W, H, seed in cases:
        mats, q = _case(n, W, H, seed, tilt)
        geom, vol = fdk.Geometry(mats, W, H), fdk.Volume(L, voxel)
        qd = q.to(DEV)
        out = torch.full((L, L, L), float("nan"), device=DEV)
        torch.cuda.synchronize()
        fdk.backproject_noalloc(qd, geom, vol, out)
        ref_entry = fdk.backproject(qd, geom, vol)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        # same samples and weights as the allocating entry point, whose anchors
        # are per tile instead of per lane: only FP32 rounding differs, held to
        # the FP32 bar (on these rough random images it is ~1e-6)
        assert oracle.rel_l2(got, ref_entry.cpu().numpy()) <= 1e-5, f"L={L}: differs from fdk_backproject"
        assert_parity(got, oracle.backproject(L, voxel, mats, q.numpy()), what=f"noalloc L={L}")


def test_noalloc_accumulate_scale_and_slab(fdk):
    L, voxel, n, W, H = 40, 3.0, 12, 128, 96
    mats, q = _case(n, W, H, 3)
    s = np.linspace(-1.5, 2.0, n).astype(np.float32)
    s[4] = 0.0
    geom = fdk.Geometry(mats, W, H)
    part = fdk.Volume(L, voxel).slab(5, 27)
    init = torch.randn((27, L, L), generator=torch.Generator().manual_seed(4))
    out = init.to(DEV)
    fdk.backproject_noalloc(q.to(DEV), geom, part, out, accumulate=True, scale=torch.from_numpy(s).to(DEV))
    torch.cuda.synchronize()
    full = oracle.backproject(L, voxel, mats, q.double().numpy() * s.astype(np.float64)[:, None, None])
    assert_parity(out.cpu().numpy(), full[5:32] + init.numpy(), what="noalloc slab, accumulate, scale")


def test_noalloc_full_size_in_chunks(fdk):
    """512^3 @ 0.5 mm from 496 x 1248x960: the window table of the whole grid
    does not fit the scratch array, so the call runs in z-chunks."""
    carm = S.CArm(496)
    mats, q = S.filtered_projections(carm, seed=0, device=DEV)
    geom, vol = fdk.Geometry(mats, 1248, 960), fdk.Volume(512, 0.5)
    q = q.contiguous()
    out = torch.empty((512, 512, 512), device=DEV)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    fdk.backproject_noalloc(q, geom, vol, out)
    torch.cuda.synchronize()
    assert torch.cuda.memory_allocated() == before
    inc = fdk.backproject(q, geom, vol)
    torch.cuda.synchronize()
    err = float(((out.double() - inc.double()).norm() / inc.double().norm()).item())
    assert err <= 1e-6, err
    rng = np.random.default_rng(12)
    xyz = np.concatenate([rng.integers(0, 512, size=(1500, 3)),
                          np.array([[0, 0, 0], [511, 511, 511], [256, 256, 111], [256, 256, 112], [3, 500, 447]])])
    ref = oracle.backproject_points(xyz, 0.5, mats, q.cpu().numpy(), L=512)
    g = out[torch.from_numpy(xyz[:, 2]), torch.from_numpy(xyz[:, 1]), torch.from_numpy(xyz[:, 0])].cpu().numpy()
    assert np.abs(g - ref).max() <= 1e-4 * np.abs(ref).max()


def test_noalloc_rejects_beyond_limits(fdk):
    mats, q = _case(5, 96, 64, 5)
    geom, vol = fdk.Geometry(mats, 96, 64), fdk.Volume(24, 4.0)
    out = torch.zeros((24, 24, 24), device=DEV)
    with pytest.raises(fdk.FdkError, match="UNSUPPORTED"):
        fdk.backproject_noalloc(q.to(DEV).half(), geom, vol, out)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out).item() == 0
