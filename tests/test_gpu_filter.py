"""FDK preprocessing on the GPU (fdk_filter_projections) against the FP64
direct-convolution oracle."""
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


def fgeom_of(fdk, carm, fan_sign=-1.0, scan_range=None):
    cu, cv = carm.principal_point
    arc = np.deg2rad(carm.arc_deg)
    return fdk.FilterGeometry(angles_rad=carm.angles_rad(), width=carm.width, height=carm.height,
                              pixel_u_mm=carm.pixel, pixel_v_mm=carm.pixel, u0=cu, v0=cv, sdd_mm=carm.sdd,
                              sid_mm=carm.sid, scan_range_rad=arc if scan_range is None else scan_range,
                              dbeta_rad=arc / max(carm.n_proj - 1, 1), fan_sign=fan_sign)


def oracle_filter(fg, li, rows=None):
    """Oracle on all rows, or on the given rows only (the filter is per row)."""
    args = dict(pixel_u=fg.pixel_u_mm, pixel_v=fg.pixel_v_mm, u0=fg.u0, v0=fg.v0, sdd=fg.sdd_mm,
                sid=fg.sid_mm, beta=fg.angles_rad, scan_range=fg.scan_range_rad, dbeta=fg.dbeta_rad,
                fan_sign=fg.fan_sign)
    if rows is None:
        return oracle.fdk_filter(li, **args)
    out = []
    for j in rows:
        out.append(oracle.fdk_filter(li[:, j:j + 1], **{**args, "v0": fg.v0 - j})[:, 0])
    return np.stack(out, axis=1)


@pytest.mark.parametrize("W,H,N,fan_sign", [(101, 7, 5, -1.0), (64, 6, 4, 1.0), (33, 1, 3, -1.0),
                                            (2, 3, 3, -1.0), (1, 4, 3, 1.0), (257, 5, 3, -1.0),
                                            (3, 2, 3, -1.0), (7, 3, 3, 1.0), (12, 3, 3, -1.0),
                                            (20, 2, 3, 1.0), (1000, 3, 3, -1.0), (10, 3, 3, 1.0)])
def test_filter_matches_oracle(fdk, W, H, N, fan_sign):
    """Ragged widths: FFT sizes 2^k from 4 to 2048 (4 and 8 run every stage
    on its own, from 16 up the first and last stages are fused; log2 M even
    and odd) and 5 * 2^k (20, 40, 80, 640: a radix-5 first stage, with a
    radix-2 stage after it or not); odd row counts (the last row of a projection
    filtered alone), both fan orientations."""
    carm = S.CArm(N, W, H, pixel=max(0.308, 400.0 / W))
    fg = fgeom_of(fdk, carm, fan_sign)
    li = np.random.default_rng(W + H).standard_normal((N, H, W)).astype(np.float32)
    out, sc = fdk.filter_projections(torch.from_numpy(li).to(DEV), fg)
    torch.cuda.synchronize()
    assert sc is None
    ref = oracle_filter(fg, li.astype(np.float64))
    assert_parity(out.cpu().numpy(), ref, what=f"filter W={W} H={H}")


def test_filter_without_short_scan_weights(fdk):
    carm = S.CArm(4, 96, 5, pixel=4.0)
    fg = fgeom_of(fdk, carm, scan_range=0.0)
    li = np.random.default_rng(2).standard_normal((4, 5, 96)).astype(np.float32)
    out, _ = fdk.filter_projections(torch.from_numpy(li).to(DEV), fg)
    torch.cuda.synchronize()
    assert_parity(out.cpu().numpy(), oracle_filter(fg, li.astype(np.float64)), what="no Parker")


def test_filter_full_detector_rows(fdk):
    """1248-pixel rows (FFT size 2560 = 5 x 512) of the benchmark detector, sampled rows
    of a full phantom stack (the oracle filters rows independently)."""
    carm = S.CArm(8)
    mats = S.carm_matrices(carm)
    li = S.project_phantom(mats, carm.width, carm.height, S.ellipsoid_phantom(0), device=DEV).float()
    fg = fgeom_of(fdk, carm)
    out, _ = fdk.filter_projections(li.contiguous(), fg)
    torch.cuda.synchronize()
    rows = [0, 301, 479, 480, 959]
    ref = oracle_filter(fg, li.cpu().numpy().astype(np.float64), rows)
    got = out.cpu().numpy()[:, rows]
    assert_parity(got, ref, what="full detector rows")
    # and the host generator's FFT filter (FP64) on the whole stack
    q_host = S.fdk_filter(li.double(), carm).cpu().numpy()
    err = oracle.rel_l2(out.cpu().numpy(), q_host)
    print(f"GPU filter vs FP64 host filter, 8 x 960 x 1248: rel L2 {err:.2e}")
    assert err < 1e-5


@pytest.mark.parametrize("dtype", [torch.float16, torch.bfloat16])
@pytest.mark.parametrize("n,h,w", [(5, 9, 200), (7, 9, 201), (96, 64, 320), (75, 33, 130)])
def test_filter_packed_output(fdk, dtype, n, h, w):
    """FP16/BF16 output equals packing the FP32 output (scale from the
    per-wave maxima the filter records): odd row counts, a projection size
    that is not a multiple of four or of eight, and many projections whose
    row pairs run on every XCD."""
    carm = S.CArm(n, w, h, pixel=400.0 / w)
    fg = fgeom_of(fdk, carm)
    li = torch.randn(n, h, w, generator=torch.Generator().manual_seed(7)).to(DEV)
    q32, _ = fdk.filter_projections(li, fg)
    qp, sc = fdk.filter_projections(li, fg, dtype=dtype)
    p2, s2 = fdk.pack_projections(q32, dtype)
    torch.cuda.synchronize()
    assert torch.equal(sc, s2)
    assert torch.equal(qp.view(torch.int16), p2.view(torch.int16))


def test_filter_then_backproject_reconstructs(fdk):
    """GPU preprocessing + GPU backprojection of exact phantom line integrals
    reproduce the phantom near the mid-plane (as the FP64 pipeline does)."""
    carm = S.CArm(124, 620, 480, pixel=0.616)
    mats = S.carm_matrices(carm)
    ph = S.ellipsoid_phantom(0)
    li = S.project_phantom(mats, carm.width, carm.height, ph, device=DEV).float().contiguous()
    q, _ = fdk.filter_projections(li, fgeom_of(fdk, carm))
    L, voxel = 64, 1.5
    V = fdk.backproject(q, fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel, z_begin=28, z_count=8))
    torch.cuda.synchronize()
    T = S.voxelize_phantom(ph, L, voxel).numpy()[28:36]
    v = V.cpu().numpy()
    assert v.mean() == pytest.approx(T.mean(), rel=0.02)
    assert oracle.rel_l2(v, T) < 0.10
