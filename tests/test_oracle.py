"""Pins for the FP64 oracle, each against something other than the oracle itself.

* brute force: the branch-free tent form  val = sum_ij I[j][i] L(ix-i) L(iy-j),
  L(t) = max(0, 1-|t|), summed over *every* pixel, built as a dense matrix B;
* a library routine: with w == 1 (affine matrices) backprojection reduces to
  bilinear resampling with zero extension (scipy.ndimage.map_coordinates,
  order=1, mode='grid-constant');
* closed forms: constant image, exact pixel-centre copy, single-pixel delta;
* invariants: off-detector voxels add exactly 0, linearity, BP(cA)=BP(A)/c^2,
  additivity over projection subsets and z-slabs, projection permutation;
* adjoint: B^T from the dense matrix, the dot-product test, exact-quadratic
  finite differences of ||Bp - V_t||^2;
* the analytic phantom: FDK of exact line integrals reproduces the densities;
* a hand-derived worked example stored under tests/golden/.
"""
import json
import os

import numpy as np
import pytest
from scipy.ndimage import map_coordinates

import oracle
import synthetic as S

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ----------------------------------------------------------------------------- helpers
def centres(L, voxel, origin=None):
    o = S.default_origin(L, voxel) if origin is None else origin
    z, y, x = np.meshgrid(np.arange(L), np.arange(L), np.arange(L), indexing="ij")
    X = np.stack([o[0] + x * voxel, o[1] + y * voxel, o[2] + z * voxel, np.ones_like(x, float)], -1)
    return X.reshape(-1, 4)  # voxel order (z, y, x), x fastest


def dense_B(L, voxel, mats, W, H, origin=None):
    """Dense (L^3, N*H*W) matrix of the tent form over every pixel."""
    X = centres(L, voxel, origin)
    N = mats.shape[0]
    B = np.zeros((X.shape[0], N, H, W))
    ii = np.arange(W)[None, None, :]
    jj = np.arange(H)[None, :, None]
    for k in range(N):
        uvw = X @ mats[k].T
        ix = uvw[:, 0] / uvw[:, 2]
        iy = uvw[:, 1] / uvw[:, 2]
        lx = np.maximum(0.0, 1.0 - np.abs(ix[:, None, None] - ii))
        ly = np.maximum(0.0, 1.0 - np.abs(iy[:, None, None] - jj))
        B[:, k] = lx * ly / (uvw[:, 2] ** 2)[:, None, None]
    return B.reshape(X.shape[0], -1)


def pixel_coords(L, voxel, mats, origin=None):
    X = centres(L, voxel, origin)
    uvw = np.einsum("nrc,pc->npr", mats, X)
    return uvw[..., 0] / uvw[..., 2], uvw[..., 1] / uvw[..., 2], uvw[..., 2]


# ----------------------------------------------------------------------------- brute force
@pytest.mark.parametrize("L,W,H,seed", [(4, 7, 5, 1), (5, 7, 5, 2), (8, 7, 5, 3), (6, 5, 7, 4)])
def test_tent_bruteforce(L, W, H, seed):
    voxel = 1.0
    mats = S.tiny_cone_matrices(3, W, H, L, voxel, seed)
    ix, iy, w = pixel_coords(L, voxel, mats)
    # the case must exercise the edges: voxels projecting into (-1, 0), past W-1, and off
    assert ((ix > -1) & (ix < 0)).any() or ((iy > -1) & (iy < 0)).any()
    assert ((ix > W - 1) & (ix < W)).any() or ((iy > H - 1) & (iy < H)).any()
    assert ((ix <= -1) | (ix >= W) | (iy <= -1) | (iy >= H)).any()
    proj = S.random_projections(3, H, W, seed)
    B = dense_B(L, voxel, mats, W, H)
    ref = (B @ proj.astype(np.float64).ravel()).reshape(L, L, L)
    got = oracle.backproject(L, voxel, mats, proj)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_floor_not_truncation():
    """ix in (-1, 0): tap -1 is zero, tap 0 has weight 1+ix (truncation would give 1-ix)."""
    L, voxel = 1, 1.0
    W, H = 4, 3
    img = np.zeros((1, H, W), np.float32)
    img[0, 1, 0] = 1.0
    # affine map: ix = -0.25, iy = 1 for the single voxel at the origin
    A = np.array([[[0, 0, 0, -0.25], [0, 0, 0, 1.0], [0, 0, 0, 1.0]]])
    got = oracle.backproject(L, voxel, A, img)
    assert got.ravel()[0] == pytest.approx(0.75, abs=1e-15)


# ----------------------------------------------------------------------------- library routine
@pytest.mark.parametrize("seed", [0, 1])
def test_affine_equals_bilinear_resampling(seed):
    rng = np.random.default_rng(seed)
    L, voxel, W, H, N = 9, 0.7, 11, 8, 4
    origin = (-2.0, -1.5, -3.0)
    mats = np.zeros((N, 3, 4))
    for k in range(N):
        mats[k, :2, :3] = rng.uniform(-1.5, 1.5, size=(2, 3))
        mats[k, 0, 3] = rng.uniform(2, 8)
        mats[k, 1, 3] = rng.uniform(1, 6)
        mats[k, 2, 3] = 1.0
    proj = S.random_projections(N, H, W, seed + 10)
    got = oracle.backproject(L, voxel, mats, proj, origin=origin)
    X = centres(L, voxel, origin)
    ref = np.zeros(X.shape[0])
    for k in range(N):
        uv = X @ mats[k, :2].T
        ref += map_coordinates(proj[k].astype(np.float64), [uv[:, 1], uv[:, 0]], order=1,
                               mode="grid-constant", cval=0.0)
    assert np.max(np.abs(got.ravel() - ref)) <= 1e-12 * np.max(np.abs(ref))


# ----------------------------------------------------------------------------- closed forms
def test_constant_image():
    L, voxel, W, H, N = 6, 1.0, 9, 7, 5
    mats = S.tiny_cone_matrices(N, W, H, L, voxel, 7, jitter=0.0)
    c = 2.5
    proj = np.full((N, H, W), c, np.float32)
    got = oracle.backproject(L, voxel, mats, proj).ravel()
    ix, iy, w = pixel_coords(L, voxel, mats)
    inside = ((ix >= 0) & (ix <= W - 1) & (iy >= 0) & (iy <= H - 1)).all(0)
    assert inside.sum() > 10
    expect = (c / w ** 2).sum(0)
    np.testing.assert_allclose(got[inside], expect[inside], rtol=1e-14)


def test_exact_copy():
    """u = x, v = y on voxel indices with w = 2 on every projection:
    every plane receives sum_k I_k / 4."""
    L, voxel, N = 5, 0.5, 3
    origin = (1.0, -2.0, 0.25)
    mats = np.zeros((N, 3, 4))
    for k in range(N):
        # (u, v, w) = 2 * ((X - ox)/voxel, (Y - oy)/voxel, 1)
        mats[k] = 2.0 * np.array([[1 / voxel, 0, 0, -origin[0] / voxel],
                                  [0, 1 / voxel, 0, -origin[1] / voxel],
                                  [0, 0, 0, 1.0]])
    proj = S.random_projections(N, L, L, 5)
    got = oracle.backproject(L, voxel, mats, proj, origin=origin)
    expect = proj.astype(np.float64).sum(0) / 4.0
    for z in range(L):
        np.testing.assert_allclose(got[z], expect, rtol=0, atol=1e-15)


def test_single_pixel_delta_support():
    L, voxel, W, H = 8, 1.0, 7, 5
    mats = S.tiny_cone_matrices(1, W, H, L, voxel, 11)
    img = np.zeros((1, H, W), np.float32)
    img[0, 2, 3] = 1.0
    got = oracle.backproject(L, voxel, mats, img).ravel()
    ix, iy, w = pixel_coords(L, voxel, mats)
    support = (np.abs(ix[0] - 3) < 1) & (np.abs(iy[0] - 2) < 1)
    assert support.any()
    assert np.array_equal(got != 0, support)
    tent = (1 - np.abs(ix[0] - 3)) * (1 - np.abs(iy[0] - 2)) / w[0] ** 2
    np.testing.assert_allclose(got[support], tent[support], rtol=1e-12)


def test_golden_worked_example():
    with open(os.path.join(GOLDEN, "worked_example.json")) as f:
        g = json.load(f)
    got = oracle.backproject(g["L"], g["voxel_mm"], np.array(g["mats"]),
                             np.array(g["proj"], np.float32), origin=g["origin_mm"])
    np.testing.assert_allclose(got.ravel(), np.array(g["expected"]), rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------- invariants
def _cone_case(seed, L=10, W=12, H=9, N=6):
    voxel = 1.0
    mats = S.tiny_cone_matrices(N, W, H, L, voxel, seed)
    proj = S.random_projections(N, H, W, seed + 100)
    return L, voxel, mats, proj


def test_off_detector_adds_exact_zero():
    L, voxel, mats, proj = _cone_case(21)
    N, H, W = proj.shape
    ix, iy, w = pixel_coords(L, voxel, mats)
    off = ((ix <= -1) | (ix >= W) | (iy <= -1) | (iy >= H)).all(0)
    assert off.sum() > 0
    got = oracle.backproject(L, voxel, mats, np.abs(proj) + 1.0).ravel()
    assert np.all(got[off] == 0.0)
    assert np.all(got[~off] > 0.0)


def test_linearity_and_scale():
    L, voxel, mats, p = _cone_case(22)
    q = S.random_projections(*p.shape, 99)
    a, b = 0.75, -1.25
    lhs = oracle.backproject(L, voxel, mats, a * p.astype(np.float64) + b * q.astype(np.float64))
    rhs = a * oracle.backproject(L, voxel, mats, p) + b * oracle.backproject(L, voxel, mats, q)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-13 * np.abs(rhs).max())
    c = 3.0
    base = oracle.backproject(L, voxel, mats, p)
    scaled = oracle.backproject(L, voxel, mats * c, p)
    np.testing.assert_allclose(scaled, base / c ** 2, rtol=0, atol=1e-13 * np.abs(base).max())
    # a weight of 1/w instead of 1/w^2 would give base / c
    assert np.abs(scaled - base / c).max() > 0.1 * np.abs(base).max()


def test_additivity_slabs_and_permutation():
    L, voxel, mats, p = _cone_case(23)
    N = p.shape[0]
    full = oracle.backproject(L, voxel, mats, p)
    part = oracle.backproject(L, voxel, mats, p, k_range=(0, 2))
    part = oracle.backproject(L, voxel, mats, p, k_range=(2, N), init=part)
    np.testing.assert_allclose(part, full, rtol=0, atol=1e-14 * np.abs(full).max())
    slab = np.concatenate([oracle.backproject(L, voxel, mats, p, z_range=(0, 3)),
                           oracle.backproject(L, voxel, mats, p, z_range=(3, L - 3))])
    assert np.array_equal(slab, full)
    perm = np.random.default_rng(0).permutation(N)
    pp = oracle.backproject(L, voxel, mats[perm], p[perm])
    np.testing.assert_allclose(pp, full, rtol=0, atol=1e-14 * np.abs(full).max())


def test_points_match_volume():
    L, voxel, mats, p = _cone_case(24)
    full = oracle.backproject(L, voxel, mats, p)
    rng = np.random.default_rng(3)
    xyz = rng.integers(0, L, size=(50, 3))
    pts = oracle.backproject_points(xyz, voxel, mats, p, L=L)
    np.testing.assert_array_equal(pts, full[xyz[:, 2], xyz[:, 1], xyz[:, 0]])


# ----------------------------------------------------------------------------- adjoint
@pytest.mark.parametrize("L,W,H,seed", [(4, 7, 5, 31), (7, 6, 9, 32)])
def test_adjoint_is_dense_transpose(L, W, H, seed):
    voxel = 1.0
    mats = S.tiny_cone_matrices(3, W, H, L, voxel, seed)
    x = np.random.default_rng(seed).standard_normal((L, L, L))
    B = dense_B(L, voxel, mats, W, H)
    ref = (B.T @ x.ravel()).reshape(3, H, W)
    got = oracle.forwardproject(L, voxel, mats, x, W, H)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_dot_product():
    L, W, H, N, voxel = 16, 32, 24, 5, 1.0
    mats = S.tiny_cone_matrices(N, W, H, L, voxel, 41)
    rng = np.random.default_rng(2)
    x = rng.standard_normal((L, L, L))
    p = rng.standard_normal((N, H, W))
    Bp = oracle.backproject(L, voxel, mats, p)
    Btx = oracle.forwardproject(L, voxel, mats, x, W, H)
    lhs, rhs = float((Bp * x).sum()), float((p * Btx).sum())
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Bp) * np.linalg.norm(x)


def test_gradient_finite_differences():
    """||Bp - V_t||^2 is exactly quadratic in p: central differences have no
    truncation error, so they match 2 B^T (Bp - V_t) up to rounding."""
    L, W, H, N, voxel = 6, 8, 7, 3, 1.0
    mats = S.tiny_cone_matrices(N, W, H, L, voxel, 51)
    rng = np.random.default_rng(5)
    p = rng.standard_normal((N, H, W))
    Vt = rng.standard_normal((L, L, L))
    g = oracle.gradient(L, voxel, mats, p, Vt)

    def loss(pp):
        r = oracle.backproject(L, voxel, mats, pp) - Vt
        return float((r * r).sum())

    h = 1e-3
    for flat in rng.choice(p.size, 12, replace=False):
        e = np.zeros(p.size)
        e[flat] = h
        e = e.reshape(p.shape)
        fd = (loss(p + e) - loss(p - e)) / (2 * h)
        assert fd == pytest.approx(g.ravel()[flat], rel=1e-7, abs=1e-9)


# ----------------------------------------------------------------------------- phantom
def test_fdk_phantom_sanity():
    """FDK of the analytic ellipsoid projections approximates the densities
    near the mid-plane (loose geometry/weighting gate, not a parity gate)."""
    carm = S.CArm(124, 620, 480, pixel=0.616)
    mats = S.carm_matrices(carm)
    ph = S.ellipsoid_phantom(0)
    q = S.fdk_filter(S.project_phantom(mats, carm.width, carm.height, ph), carm)
    L, voxel = 64, 1.5
    V = oracle.backproject(L, voxel, mats, q.numpy())
    T = S.voxelize_phantom(ph, L, voxel).numpy()
    zc = slice(L // 2 - 4, L // 2 + 4)
    assert V[zc].mean() == pytest.approx(T[zc].mean(), rel=0.02)
    assert oracle.rel_l2(V[zc], T[zc]) < 0.10


def test_matrix_layout_listing_form():
    """The listing indexes A column-major (u uses A[0], A[3], A[6], A[9]); the
    row-major P[r][c] = A_cm[r + 3c] gives the same detector coordinates."""
    rng = np.random.default_rng(8)
    P = rng.standard_normal((3, 4))
    A_cm = P.T.ravel()  # A_cm[r + 3c] = P[r][c]
    X = rng.standard_normal(3)
    u = X[0] * A_cm[0] + X[1] * A_cm[3] + X[2] * A_cm[6] + A_cm[9]
    v = X[0] * A_cm[1] + X[1] * A_cm[4] + X[2] * A_cm[7] + A_cm[10]
    w = X[0] * A_cm[2] + X[1] * A_cm[5] + X[2] * A_cm[8] + A_cm[11]
    np.testing.assert_allclose(P @ np.append(X, 1.0), [u, v, w], rtol=1e-14)


def test_supported_update_count_matches_paper_workload():
    """The stored supported-update count of the synthetic 512^3 x 496 C-arm
    workload (written by tests/golden/make_supported_updates.py with the
    oracle) is within 2% of the clipped update count the paper derives for the
    RabbitCT scan (4.39e10, Sec. "Performance Model"), and consistent with the
    oracle's counter on a slab of planes."""
    import json
    import os
    with open(os.path.join(os.path.dirname(__file__), "golden", "supported_updates.json")) as f:
        rec = json.load(f)["512^3 @0.5mm x 496 x 1248x960, 200deg C-arm"]
    assert rec["nominal"] == 512 ** 3 * 496
    assert abs(rec["supported"] / 4.39e10 - 1.0) < 0.02
    # the oracle's counter on a slab stays within that slab's nominal count
    carm = S.CArm(8)
    mats = S.carm_matrices(carm)
    n = oracle.supported_updates(64, 0.5 * 512 / 64, mats, carm.width, carm.height, z_range=(30, 4))
    assert 0 < n <= 64 * 64 * 4 * 8


@pytest.mark.parametrize("L,W,H,seed", [(4, 7, 5, 1), (5, 7, 5, 2), (8, 7, 5, 3), (6, 5, 7, 4)])
def test_supported_updates_bruteforce(L, W, H, seed):
    """The supported-update count (the clipped updates behind the paper's GUp/s,
    Sec. "Performance Model") equals, exactly, the number of (voxel,
    projection) pairs with at least one nonzero entry of the dense tent matrix
    over every pixel, i.e. pairs whose bilinear sample has a tap on the
    detector.  The tiny cones put voxels at ix in (-1, 0) and (W-1, W), which a
    support test of [0, W) or [0, W-1] would miss."""
    voxel = 1.0
    mats = S.tiny_cone_matrices(3, W, H, L, voxel, seed)
    ix, iy, _ = pixel_coords(L, voxel, mats)
    assert (((ix > -1) & (ix < 0)) | ((iy > -1) & (iy < 0))).any()
    assert (((ix > W - 1) & (ix < W)) | ((iy > H - 1) & (iy < H))).any()
    B = dense_B(L, voxel, mats, W, H).reshape(L ** 3, 3, H * W)
    expect = int(np.count_nonzero((B != 0).any(axis=2)))
    assert 0 < expect < L ** 3 * 3
    assert oracle.supported_updates(L, voxel, mats, W, H) == expect
    # per slab of planes, and the slabs add up
    z = L // 2
    Bz = B.reshape(L, L * L, 3, H * W)
    lo = int(np.count_nonzero((Bz[:z] != 0).any(axis=3)))
    hi = int(np.count_nonzero((Bz[z:] != 0).any(axis=3)))
    assert oracle.supported_updates(L, voxel, mats, W, H, z_range=(0, z)) == lo
    assert oracle.supported_updates(L, voxel, mats, W, H, z_range=(z, L - z)) == hi
    assert lo + hi == expect


def test_supported_updates_edges_exact():
    """Single voxels placed by an affine map at chosen detector coordinates:
    a sample at ix in (-1, 0) or (W-1, W) (one tap column on the detector)
    counts, ix = -1 or ix = W exactly (both taps at weight 0 or off) does
    not, and likewise along the rows."""
    W, H = 6, 4
    cases = [((-0.5, 1.0), 1), ((W - 0.5, 1.0), 1), ((-1.0, 1.0), 0), ((float(W), 1.0), 0),
             ((2.0, -0.25), 1), ((2.0, H - 0.75), 1), ((2.0, -1.0), 0), ((2.0, float(H)), 0),
             ((-1.5, 2.0), 0), ((2.5, 1.5), 1), ((-0.999, -0.999), 1)]
    for (u, v), want in cases:
        A = np.array([[[0, 0, 0, u], [0, 0, 0, v], [0, 0, 0, 1.0]]])
        assert oracle.supported_updates(1, 1.0, A, W, H) == want, (u, v)
    # w != 1: the test is on u/w, not on u
    A = np.array([[[0, 0, 0, -0.5 * 3.0], [0, 0, 0, 1.0 * 3.0], [0, 0, 0, 3.0]]])
    assert oracle.supported_updates(1, 1.0, A, W, H) == 1


def test_psnr_and_rel_l2_hand_values():
    """PSNR = 10 log10((max ref - min ref)^2 / MSE) and rel L2 = ||x - ref|| /
    ||ref|| (the quality measures of the paper's benchmark, defined here as
    their textbook forms) on values worked out by hand."""
    ref = np.array([1.0, 2.0, 5.0, -3.0])
    x = np.array([1.0, 4.0, 5.0, -2.0])          # errors 0, 2, 0, 1: MSE = 5/4
    # range 8: 10 log10(64 / 1.25) = 10 log10(51.2)
    assert oracle.psnr(x, ref) == pytest.approx(17.092699609758306, abs=1e-12)
    # ||(0, 2, 0, 1)|| / ||(1, 2, 5, -3)|| = sqrt(5) / sqrt(39)
    assert oracle.rel_l2(x, ref) == pytest.approx(np.sqrt(5.0 / 39.0), rel=1e-14)
    # a constant offset d gives MSE = d^2: PSNR = 20 log10(range / d)
    ref2 = np.linspace(-4.0, 6.0, 101).reshape(101, 1)
    assert oracle.psnr(ref2 + 0.01, ref2) == pytest.approx(60.0, abs=1e-9)
    assert oracle.psnr(ref2 - 0.1, ref2) == pytest.approx(40.0, abs=1e-9)
    # equal inputs: infinite PSNR, zero error
    assert oracle.psnr(ref, ref) == float("inf")
    assert oracle.rel_l2(ref, ref) == 0.0
    # shape does not matter (all voxels in one sum)
    assert oracle.psnr(x.reshape(2, 2), ref.reshape(2, 2)) == oracle.psnr(x, ref)


# ----------------------------------------------------------------------------- FDK preprocessing
def _filter_args(carm):
    cu, cv = carm.principal_point
    arc = np.deg2rad(carm.arc_deg)
    dbeta = arc / (carm.n_proj - 1)
    return dict(pixel_u=carm.pixel, pixel_v=carm.pixel, u0=cu, v0=cv, sdd=carm.sdd, sid=carm.sid,
                beta=carm.angles_rad(), scan_range=arc, dbeta=dbeta, fan_sign=-1.0)


def test_ramp_kernel_frequency_response():
    """The band-limited ramp kernel's DTFT is |f| on the band (Kak & Slaney):
    sum_n h(n) exp(-2 pi i f n) = |f| / tau^2 for |f| <= 1/2 (tau = sample
    spacing); the truncation of the 1/n^2 tail at |n| < 2^14 costs < 1e-5."""
    tau = 0.7
    n = np.arange(-(1 << 14) + 1, 1 << 14)
    h = np.array([oracle.ramp_kernel(int(k), tau) for k in n])
    for f in (0.03, 0.1, 0.25, 0.4, 0.49):
        H = float(np.sum(h * np.cos(2 * np.pi * f * n)))
        assert H * tau * tau == pytest.approx(f, abs=2e-5)
    assert oracle.ramp_kernel(0, tau) > 0 and oracle.ramp_kernel(2, tau) == 0.0 and oracle.ramp_kernel(-3, tau) < 0


def test_parker_weights_complementary_rays():
    """Parker's weights give the two measurements of every ray total weight 1:
    the ray (beta, gamma) is measured again at (beta + pi + 2 gamma, -gamma);
    outside the short scan the weight is 0 and in its middle 1."""
    rng = np.random.default_rng(3)
    R = np.deg2rad(200.0)
    d = (R - np.pi) / 2
    for _ in range(2000):
        g = rng.uniform(-0.9 * d, 0.9 * d)
        b = rng.uniform(0, np.pi + 2 * d)
        b2 = b + np.pi + 2 * g
        if b2 > np.pi + 2 * d:       # the other measurement lies before the scan start
            b2 = b - np.pi + 2 * g
            if b2 < 0:
                continue
        w = oracle.parker_weight(b, g, R) + oracle.parker_weight(b2, -g, R)
        assert w == pytest.approx(1.0, abs=1e-12)
    assert oracle.parker_weight(-0.01, 0.0, R) == 0.0
    assert oracle.parker_weight(np.pi + 2 * d + 0.01, 0.0, R) == 0.0
    assert oracle.parker_weight(np.pi / 2, 0.0, R) == 1.0
    assert oracle.parker_weight(1.0, 0.3, -1.0) == 1.0


def test_filter_is_weighted_linear_convolution():
    """Against numpy's full linear convolution of the weighted rows, with the
    cosine weight computed as the cosine of the angle between the pixel's ray
    and the central ray (vector form)."""
    carm = S.CArm(7, 45, 6, pixel=8.0)
    a = _filter_args(carm)
    p = np.random.default_rng(5).standard_normal((7, 6, 45))
    q = oracle.fdk_filter(p, **a)
    tau = carm.pixel * carm.sid / carm.sdd
    W = 45
    h = np.array([oracle.ramp_kernel(n, tau) for n in range(-(W - 1), W)])
    u = (np.arange(W) - a["u0"]) * carm.pixel
    for k in range(7):
        for j in range(6):
            v = (j - a["v0"]) * carm.pixel
            ray = np.stack([u, np.full(W, v), np.full(W, carm.sdd)], axis=1)
            cosw = ray[:, 2] / np.linalg.norm(ray, axis=1)
            g = -np.arctan2(u, carm.sdd)
            wp = np.array([oracle.parker_weight(a["beta"][k], gg, a["scan_range"]) for gg in g])
            full = np.convolve(p[k, j] * cosw * wp, h)          # length 3W - 2
            ref = full[W - 1:2 * W - 1] * tau * a["dbeta"] * carm.sid ** 2
            np.testing.assert_allclose(q[k, j], ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_filter_matches_fft_implementation():
    """The direct-convolution oracle and the FFT-based host filter of the
    synthetic input generator (an independent implementation) agree."""
    carm = S.CArm(9, 64, 12, pixel=6.0)
    li = np.random.default_rng(6).standard_normal((9, 12, 64))
    import torch
    ref = S.fdk_filter(torch.from_numpy(li), carm).numpy()
    q = oracle.fdk_filter(li, **_filter_args(carm))
    assert oracle.rel_l2(q, ref) < 1e-12


def test_fdk_phantom_sanity_with_oracle_filter():
    """Oracle filter + oracle backprojection of exact ellipsoid line integrals
    reproduce the phantom densities near the mid-plane (the scale constants)."""
    carm = S.CArm(124, 620, 480, pixel=0.616)
    mats = S.carm_matrices(carm)
    ph = S.ellipsoid_phantom(0)
    li = S.project_phantom(mats, carm.width, carm.height, ph).numpy()
    rows = slice(200, 280)                  # the rows the mid-plane slab projects onto
    q = np.zeros_like(li)
    q[:, rows] = oracle.fdk_filter(li[:, rows], **{**_filter_args(carm), "v0": carm.principal_point[1] - 200})
    L, voxel = 64, 1.5
    zc = (L // 2 - 4, 8)
    V = oracle.backproject(L, voxel, mats, q, z_range=zc)
    T = S.voxelize_phantom(ph, L, voxel).numpy()[L // 2 - 4:L // 2 + 4]
    assert V.mean() == pytest.approx(T.mean(), rel=0.02)
    assert oracle.rel_l2(V, T) < 0.10
