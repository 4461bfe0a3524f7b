"""FP16/BF16 projection storage: packing is bit-exact against its definition,
and the packed backprojection meets the FP32 bar against the oracle run on the
dequantised projections (the kernel error); the storage error is stated."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from tests._common import assert_parity, ensure_built, small_carm

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def fdk():
    ensure_built()
    import paper_1401_3615_amd as m
    m.load()
    return m


def bf16_rne_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of FP32 to bfloat16, written from the definition."""
    u = x32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16).astype(np.uint16)
    nan = np.isnan(x32)
    r[nan] = ((u[nan] >> 16) | 0x40).astype(np.uint16)
    return r


@pytest.mark.parametrize("seed", [0, 1])
def test_pack_bit_exact(fdk, seed):
    rng = np.random.default_rng(seed)
    p = (rng.standard_normal((5, 37, 53)) * rng.uniform(1e-3, 1e3, size=(5, 1, 1))).astype(np.float32)
    p[3] = 0.0                       # an all-zero projection gets scale 1
    pd = torch.from_numpy(p).to(DEV)
    h, s = fdk.pack_projections(pd, torch.float16)
    b, sb = fdk.pack_projections(pd, torch.bfloat16)
    torch.cuda.synchronize()
    m = np.abs(p).max(axis=(1, 2))
    expect_s = np.where(m > 0, m * np.float32(2.0 ** -14), np.float32(1.0)).astype(np.float32)
    assert np.array_equal(s.cpu().numpy(), expect_s)
    assert np.array_equal(sb.cpu().numpy(), expect_s)
    q = (p / expect_s[:, None, None]).astype(np.float32)   # IEEE division in FP32
    assert np.array_equal(h.cpu().numpy().view(np.uint16), q.astype(np.float16).view(np.uint16))
    assert np.array_equal(b.cpu().view(torch.int16).numpy().view(np.uint16), bf16_rne_bits(q))
    # bf16 from torch's own conversion agrees
    assert torch.equal(b.cpu(), torch.from_numpy(q).to(torch.bfloat16))


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
def test_packed_backprojection(fdk, dtype):
    carm = small_carm(31, 256, 200)
    mats, q = S.filtered_projections(carm, 8)
    L, voxel = 64, 1.5
    qd = q.to(DEV)
    qp, sc = fdk.pack_projections(qd, dtype)
    geom = fdk.Geometry(mats, carm.width, carm.height)
    out = fdk.backproject(qp, geom, fdk.Volume(L, voxel), scale=sc)
    torch.cuda.synchronize()
    deq = qp.double().cpu().numpy() * sc.double().cpu().numpy()[:, None, None]
    ref_k = oracle.backproject(L, voxel, mats, deq)
    assert_parity(out.cpu().numpy(), ref_k, what=f"{dtype} kernel error")
    ref = oracle.backproject(L, voxel, mats, q.numpy())
    total = oracle.rel_l2(out.cpu().numpy(), ref)
    print(f"{dtype}: total rel L2 {total:.3e}, PSNR {oracle.psnr(out.cpu().numpy(), ref):.1f} dB")
    assert total < (1e-3 if dtype == torch.float16 else 1e-2)


def test_packed_without_scale_is_raw_values(fdk):
    """FP16 data with scale=None is backprojected as stored."""
    carm = small_carm(5, 96, 64)
    mats, q = S.filtered_projections(carm, 9)
    L, voxel = 24, 4.0
    h = (q * (1000.0 / q.abs().max())).to(torch.float16)   # within FP16 range
    out = fdk.backproject(h.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
    torch.cuda.synchronize()
    ref = oracle.backproject(L, voxel, mats, h.double().numpy())
    assert_parity(out.cpu().numpy(), ref, what="fp16 raw")
