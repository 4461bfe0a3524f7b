"""The hand-written adjoint (voxel-driven forward projector) against the
oracle, the dot-product test, finite differences and autograd."""
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


def smooth_volume(L, seed):
    ph = S.ellipsoid_phantom(seed)
    return S.voxelize_phantom(ph, L, 96.0 / L).float()


def test_forwardproject_matches_oracle(fdk):
    carm = small_carm(15, 160, 128)
    mats = S.carm_matrices(carm)
    L, voxel = 48, 2.0
    x = torch.randn(L, L, L, generator=torch.Generator().manual_seed(3))
    out = fdk.forwardproject(x.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
    torch.cuda.synchronize()
    ref = oracle.forwardproject(L, voxel, mats, x.numpy(), carm.width, carm.height)
    assert_parity(out.cpu().numpy(), ref, what="forward projection")


@pytest.mark.parametrize("strip,waves,layout", [(2, 1, 0), (8, 2, 0), (16, 4, 0), (32, 4, 0),
                                                (1, 1, 4), (5, 2, 4), (13, 4, 4), (16, 1, 4), (60, 1, 4), (77, 8, 4), (508, 8, 4)])
def test_forwardproject_every_shape(fdk, strip, waves, layout):
    """Ragged grid (L = 37): direct global scatter for several strip shapes
    and detector tiles of 1 to 77 rows for 1 to 8 projections per
    workgroup."""
    carm = small_carm(9, 101, 77)
    mats = S.carm_matrices(carm)
    L, voxel = 37, 4.0
    x = torch.randn(L, L, L, generator=torch.Generator().manual_seed(5))
    fdk.set_tile(fdk.TUNE_ADJOINT, strip, waves, layout)
    try:
        out = fdk.forwardproject(x.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_ADJOINT, 0, 0)
    ref = oracle.forwardproject(L, voxel, mats, x.numpy(), carm.width, carm.height)
    assert_parity(out.cpu().numpy(), ref, what=f"adjoint {strip}x{waves} layout {layout}")


@pytest.mark.parametrize("rows,group", [(8, 2), (16, 4), (64, 1), (32, 8)])
def test_forwardproject_detector_tiles_wide(fdk, rows, group):
    """Detector tiles of the 1248 x 960 detector, rows x min(1248, 20480 /
    (rows group)) pixels, so all but the first split the columns between
    tiles; group projections share a workgroup; the volume is larger than the
    field of view."""
    carm = S.CArm(5)
    mats = S.carm_matrices(carm)
    L, voxel = 56, 4.5
    x = torch.randn(L, L, L, generator=torch.Generator().manual_seed(8))
    fdk.set_tile(fdk.TUNE_ADJOINT, rows, group, 4)
    try:
        out = fdk.forwardproject(x.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_ADJOINT, 0, 0)
    ref = oracle.forwardproject(L, voxel, mats, x.numpy(), carm.width, carm.height)
    assert_parity(out.cpu().numpy(), ref, what=f"detector tiles {rows} rows x {group}")


@pytest.mark.parametrize("layout", [4, 0])
def test_forwardproject_tilted_carm(fdk, layout):
    """A C-arm tilted by 0.4 degree (w varies along z: per-voxel reciprocal
    path) on the full detector, against the oracle scatter."""
    carm = S.CArm(6, tilt_deg=0.4)
    mats = S.carm_matrices(carm)
    assert np.all(mats[:, 2, 2] != 0.0)
    L, voxel = 48, 5.0
    x = torch.randn(L, L, L, generator=torch.Generator().manual_seed(9))
    fdk.set_tile(fdk.TUNE_ADJOINT, *((16, 1, 4) if layout == 4 else (8, 2, 0)))
    try:
        out = fdk.forwardproject(x.to(DEV), fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel))
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_ADJOINT, 0, 0)
    ref = oracle.forwardproject(L, voxel, mats, x.numpy(), carm.width, carm.height)
    assert_parity(out.cpu().numpy(), ref, what=f"tilted adjoint layout {layout}")


def test_forwardproject_edges_and_accumulate(fdk):
    L, W, H, N, voxel = 19, 13, 9, 4, 1.0
    mats = S.tiny_cone_matrices(N, W, H, L, voxel, 5)
    x = np.random.default_rng(1).standard_normal((L, L, L)).astype(np.float32)
    init = np.random.default_rng(2).standard_normal((N, H, W)).astype(np.float32)
    out = torch.from_numpy(init).to(DEV)
    fdk.forwardproject(torch.from_numpy(x).to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel),
                       out=out, accumulate=True)
    torch.cuda.synchronize()
    ref = oracle.forwardproject(L, voxel, mats, x, W, H) + init.astype(np.float64)
    assert_parity(out.cpu().numpy(), ref, what="forward projection, accumulate")


def test_forwardproject_slab(fdk):
    """A slab forward-projects exactly its planes: slabs add up to the whole."""
    carm = small_carm(6, 96, 80)
    mats = S.carm_matrices(carm)
    L, voxel = 32, 3.0
    x = torch.randn(L, L, L, device=DEV)
    geom = fdk.Geometry(mats, carm.width, carm.height)
    whole = fdk.forwardproject(x, geom, fdk.Volume(L, voxel))
    parts = fdk.forwardproject(x[:10].contiguous(), geom, fdk.Volume(L, voxel, z_begin=0, z_count=10))
    fdk.forwardproject(x[10:].contiguous(), geom, fdk.Volume(L, voxel, z_begin=10, z_count=22),
                       out=parts, accumulate=True)
    torch.cuda.synchronize()
    assert oracle.rel_l2(parts.cpu().numpy(), whole.cpu().numpy()) < 1e-6


def test_dot_product_gpu(fdk):
    """<B p, x> = <p, B^T x> with both operators on the GPU."""
    carm = small_carm(24, 200, 160)
    mats = S.carm_matrices(carm)
    L, voxel = 64, 1.5
    g = torch.Generator(device=DEV)
    g.manual_seed(2)
    x = torch.randn(L, L, L, device=DEV, generator=g)
    p = torch.randn(24, carm.height, carm.width, device=DEV, generator=g)
    geom, vol = fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel)
    Bp = fdk.backproject(p, geom, vol)
    Btx = fdk.forwardproject(x, geom, vol)
    lhs = float((Bp.double() * x.double()).sum())
    rhs = float((p.double() * Btx.double()).sum())
    scale = float(Bp.double().norm() * x.double().norm())
    print(f"dot test: <Bp,x>={lhs:.9e} <p,B^T x>={rhs:.9e} rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * scale


def test_autograd_gradient_and_fd(fdk):
    """loss = ||BP(p) - V_t||^2; the autograd gradient (forward projector)
    matches the oracle's 2 B^T (B p - V_t) and central differences."""
    carm = small_carm(12, 96, 80)
    mats, q = S.filtered_projections(carm, 10)
    L, voxel = 32, 3.0
    geom, vol = fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel)
    Vt = smooth_volume(L, 1)
    p = q.to(DEV).clone().requires_grad_(True)
    V = fdk.BackProject.apply(p, geom, vol)
    loss = ((V - Vt.to(DEV)) ** 2).sum()
    loss.backward()
    g = p.grad.detach().cpu().numpy()
    ref = oracle.gradient(L, voxel, mats, q.numpy(), Vt.numpy())
    assert_parity(g, ref, rel=1e-4, elem=1e-3, what="gradient")
    # loss is exactly quadratic in p: central differences have no truncation error
    rng = np.random.default_rng(4)
    flat = np.flatnonzero(np.abs(ref.ravel()) > 1e-3 * np.abs(ref).max())
    pick = rng.choice(flat, 16, replace=False)
    q64 = q.double().numpy()
    h = 1e-3

    def L_of(pp):
        r = oracle.backproject(L, voxel, mats, pp) - Vt.double().numpy()
        return float((r * r).sum())

    for i in pick:
        e = np.zeros(q64.size)
        e[i] = h
        e = e.reshape(q64.shape)
        fd = (L_of(q64 + e) - L_of(q64 - e)) / (2 * h)
        assert g.ravel()[i] == pytest.approx(fd, rel=2e-3, abs=1e-6 * np.abs(ref).max())


def test_forwardproject_autograd(fdk):
    """ForwardProject's gradient is the backprojection."""
    carm = small_carm(8, 96, 80)
    mats = S.carm_matrices(carm)
    L, voxel = 24, 4.0
    geom, vol = fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel)
    x = torch.randn(L, L, L, device=DEV, requires_grad=True)
    y = torch.randn(8, carm.height, carm.width, device=DEV)
    (fdk.ForwardProject.apply(x, geom, vol) * y).sum().backward()
    ref = oracle.backproject(L, voxel, mats, y.cpu().numpy())
    assert_parity(x.grad.cpu().numpy(), ref, what="ForwardProject.backward")


def test_c3_dot_and_fd_full_size(fdk):
    """The 256^3 x 496 x 1248x960 differentiable configuration: dot test with
    seeded Gaussian x and p, and finite differences at 64 seeded pixels.  The
    loss is quadratic, so its central difference at pixel i with step h is
    exactly 2 <B p - V_t, B e_i>; B e_i comes from the FP64 oracle."""
    carm = S.CArm(496)
    mats = S.carm_matrices(carm)
    L, voxel = 256, 0.5
    geom, vol = fdk.Geometry(mats, carm.width, carm.height), fdk.Volume(L, voxel)
    g = torch.Generator(device=DEV)
    g.manual_seed(2)
    x = torch.randn(L, L, L, device=DEV, generator=g)
    g.manual_seed(3)
    p = torch.randn(496, carm.height, carm.width, device=DEV, generator=g)
    Bp = fdk.backproject(p, geom, vol)
    Btx = fdk.forwardproject(x, geom, vol)
    lhs = float((Bp.double() * x.double()).sum())
    rhs = float((p.double() * Btx.double()).sum())
    scale = float(Bp.double().norm() * x.double().norm())
    print(f"C3 dot test rel {abs(lhs - rhs) / scale:.2e}")
    assert abs(lhs - rhs) <= 1e-5 * scale
    del Btx, x
    # gradient of ||B p - V_t||^2 through autograd, p = filtered phantom seed 0
    mats_q, q = S.filtered_projections(carm, 0, device=DEV)
    Vt = S.voxelize_phantom(S.ellipsoid_phantom(1), L, voxel, device=DEV).float()
    pq = q.clone().requires_grad_(True)
    V = fdk.BackProject.apply(pq, geom, vol)
    loss = ((V - Vt) ** 2).sum()
    loss.backward()
    r = (V.detach() - Vt).double().cpu().numpy()
    grad = pq.grad.detach()
    gscale = float(grad.abs().max())
    rng = np.random.default_rng(4)
    # 64 seeded pixels in the detector region the volume projects onto
    ks = rng.integers(0, 496, 64)
    js = rng.integers(380, 580, 64)
    iss = rng.integers(380, 868, 64)
    for k, j, i in zip(ks, js, iss):
        delta = np.zeros((1, carm.height, carm.width))
        delta[0, j, i] = 1.0
        Be = oracle.backproject(L, voxel, mats[k:k + 1], delta)
        fd = 2.0 * float((r * Be).sum())
        gi = float(grad[k, j, i])
        assert gi == pytest.approx(fd, rel=2e-3, abs=1e-5 * gscale)
