"""Per-projection factors of any sign: projection k contributes scale[k]
times its stored values, so a zero factor adds nothing and a negative one
subtracts the projection (Listing 1 summed over weighted projections).  Every
sampling path (zero-bordered gathers, LDS windows, the window fallback, the
persistent batched kernel, circular and tilted orbits) is checked against the
oracle run on the scaled values."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from tests._common import assert_parity, ensure_built, small_carm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FACTORS = np.array([0.0, -2.0, 0.5, 1.3], dtype=np.float32)


@pytest.fixture(scope="module")
def fdk():
    ensure_built()
    import paper_1401_3615_amd as m
    m.load()
    return m


def _case(n, W, H, tilt, seed):
    carm = S.CArm(n, W, H, pixel=384.0 / W, tilt_deg=tilt)
    mats = S.carm_matrices(carm)
    q = torch.from_numpy(S.random_projections(n, H, W, seed))
    s = np.resize(FACTORS, n)
    s = np.random.default_rng(seed).permutation(s).astype(np.float32)
    return mats, q, s


def _ref(L, voxel, mats, q, s):
    return oracle.backproject(L, voxel, mats, q.double().numpy() * s.astype(np.float64)[:, None, None])


@pytest.mark.parametrize("layout", [0, 3])
@pytest.mark.parametrize("tilt", [0.0, 1.5])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_scale_any_sign(fdk, layout, tilt, dtype):
    n, W, H, L, voxel = 11, 128, 96, 40, 3.0
    mats, q, s = _case(n, W, H, tilt, seed=40 + layout)
    slot = fdk.F32 if dtype == torch.float32 else fdk.F16
    qd = q.to(dtype)   # the stored values; the oracle reads them back in FP64
    fdk.set_tile(slot, 8, 4, layout)
    try:
        out = fdk.backproject(qd.to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel),
                              scale=torch.from_numpy(s).to(DEV))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(slot, 0, 0)
    ref = _ref(L, voxel, mats, qd.float(), s)
    assert_parity(out.cpu().numpy(), ref, what=f"scale layout={layout} tilt={tilt} {dtype}")


def test_scale_zero_everywhere_gives_zero(fdk):
    n, W, H, L, voxel = 5, 96, 64, 24, 4.0
    mats, q, _ = _case(n, W, H, 0.0, seed=7)
    init = torch.full((L, L, L), 3.0, device=DEV)
    out = fdk.backproject(q.to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel), out=init,
                          accumulate=True, scale=torch.zeros(n, device=DEV))
    torch.cuda.synchronize()
    assert torch.equal(out.cpu(), torch.full((L, L, L), 3.0))


def test_scale_in_window_fallback(fdk):
    """A detector far finer than the voxel grid: the LDS windows overflow and
    the tile falls back to gathers for those projections."""
    n, W, H, L, voxel = 6, 1400, 96, 16, 8.0
    mats, q, s = _case(n, W, H, 0.0, seed=9)
    fdk.set_tile(fdk.F32, 16, 4, 3)
    try:
        out = fdk.backproject(q.to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel),
                              scale=torch.from_numpy(s).to(DEV))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.F32, 0, 0)
    assert_parity(out.cpu().numpy(), _ref(L, voxel, mats, q, s), what="fallback")


def test_scale_batched(fdk):
    specs = [(24, 4.0, 7, 96, 64, 0.0, 50), (20, 5.0, 9, 64, 48, 1.0, 51), (30, 3.0, 5, 128, 96, 0.0, 52)]
    scans, refs = [], []
    for L, voxel, n, W, H, tilt, seed in specs:
        mats, q, s = _case(n, W, H, tilt, seed)
        out = torch.full((L, L, L), float("nan"), device=DEV)
        scans.append(fdk.Scan(q.to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel), out,
                              torch.from_numpy(s).to(DEV)))
        refs.append(_ref(L, voxel, mats, q, s))
    fdk.backproject_batched(scans)
    torch.cuda.synchronize()
    for sc, ref in zip(scans, refs):
        assert_parity(sc.out.cpu().numpy(), ref, what="batched scale")
