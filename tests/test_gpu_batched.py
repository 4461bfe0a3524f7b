"""Batched form: many uneven scans in one persistent launch replayed from a
HIP graph, against one launch per scan and against the oracle."""
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


def make_scans(fdk, specs, dtypes):
    scans, host = [], []
    for (L, voxel, N, W, H, seed), dt in zip(specs, dtypes):
        carm = small_carm(N, W, H)
        mats, q = S.filtered_projections(carm, seed)
        qd = q.to(DEV)
        sc = None
        if dt != torch.float32:
            qd, sc = fdk.pack_projections(qd, dt)
        geom = fdk.Geometry(mats, W, H)
        vol = fdk.Volume(L, voxel)
        out = torch.full((L, L, L), float("nan"), device=DEV)
        scans.append(fdk.Scan(qd, geom, vol, out, sc))
        host.append((L, voxel, mats, q, qd, sc))
    return scans, host


SPECS = [(37, 3.0, 9, 101, 77, 20), (64, 1.5, 17, 160, 128, 21), (24, 4.0, 5, 96, 64, 22),
         (48, 2.0, 13, 128, 96, 23), (20, 5.0, 3, 64, 48, 24)]


def test_batched_matches_single_and_oracle(fdk):
    dts = [torch.float32, torch.float16, torch.float32, torch.bfloat16, torch.float32]
    scans, host = make_scans(fdk, SPECS, dts)
    # the batched launch uses one tile shape for all scans (the batched slot;
    # FP16/BF16 scans keep their own slot's layout); pin it for the single calls
    maxvol = fdk.Volume(max(sp[0] for sp in SPECS), 1.0)
    s, w, lay32 = fdk.get_tile(maxvol, fdk.TUNE_BATCHED)
    lays = {fdk.F32: lay32, fdk.F16: fdk.get_tile(maxvol, fdk.F16)[2], fdk.BF16: fdk.get_tile(maxvol, fdk.BF16)[2]}
    fdk.backproject_batched(scans)
    torch.cuda.synchronize()
    for dt in (fdk.F32, fdk.F16, fdk.BF16):
        fdk.set_tile(dt, s, w, lays[dt])
    try:
        for sc, (L, voxel, mats, q, qd, scale) in zip(scans, host):
            single = fdk.backproject(sc.proj, sc.geom, sc.vol, scale=sc.scale)
            torch.cuda.synchronize()
            # same samples and weights; the persistent kernel rotates each tile's
            # projection order by the device-wide residency instead of the
            # per-XCD one, so only the FP32 summation order differs
            assert oracle.rel_l2(sc.out.cpu().numpy(), single.cpu().numpy()) < 1e-6, \
                "batched differs from one launch per scan"
            if scale is None:
                ref = oracle.backproject(L, voxel, mats, q.numpy())
            else:
                ref = oracle.backproject(L, voxel, mats,
                                         qd.double().cpu().numpy() * scale.double().cpu().numpy()[:, None, None])
            assert_parity(sc.out.cpu().numpy(), ref, what=f"batched L={L}")
    finally:
        for dt in (fdk.F32, fdk.F16, fdk.BF16):
            fdk.set_tile(dt, 0, 0)


def test_graph_replay_restages_new_data(fdk):
    """A second call with the same descriptors replays the captured graph; it
    must see projection data written in between (same pointers)."""
    scans, host = make_scans(fdk, SPECS[:3], [torch.float32] * 3)
    fdk.backproject_batched(scans)
    torch.cuda.synchronize()
    first = [s.out.clone() for s in scans]
    for rep in range(3):
        for s in scans:
            s.proj.mul_(-2.0)
        torch.cuda.synchronize()
        fdk.backproject_batched(scans)
        torch.cuda.synchronize()
        for s, f in zip(scans, first):
            expect = f * (-2.0) ** (rep + 1)
            assert oracle.rel_l2(s.out.cpu().numpy(), expect.cpu().numpy()) < 1e-6


def test_batched_accumulate(fdk):
    scans, host = make_scans(fdk, SPECS[:2], [torch.float32] * 2)
    fdk.backproject_batched(scans)
    torch.cuda.synchronize()
    once = [s.out.clone() for s in scans]
    fdk.backproject_batched(scans, accumulate=True)
    torch.cuda.synchronize()
    for s, o in zip(scans, once):
        assert oracle.rel_l2(s.out.cpu().numpy(), 2 * o.cpu().numpy()) < 1e-6


def test_batched_every_item_once(fdk):
    """Many tiny scans (more work items than persistent workgroups, uneven
    costs): every voxel of every scan is added exactly once.  The call
    accumulates onto zeros, so a work item run twice would double its
    voxels and one never run would leave them zero."""
    specs = [(8 + (i % 5) * 3, 6.0, 1 + (i % 4), 32, 24, 100 + i) for i in range(40)]
    scans = []
    for (L, voxel, N, W, H, seed) in specs:
        carm = small_carm(N, W, H)
        mats = S.carm_matrices(carm)
        ones = torch.ones(N, H, W, device=DEV)
        scans.append(fdk.Scan(ones, fdk.Geometry(mats, W, H), fdk.Volume(L, voxel),
                              torch.zeros((L, L, L), device=DEV)))
    fdk.backproject_batched(scans, accumulate=True)
    torch.cuda.synchronize()
    for s, (L, voxel, N, W, H, seed) in zip(scans, specs):
        ref = oracle.backproject(L, voxel, s.geom.mats, np.ones((N, H, W), np.float32))
        assert_parity(s.out.cpu().numpy(), ref, what=f"tiny scan L={L} N={N}")


def test_autotuner_on_device(fdk, tmp_path):
    """A short tuning run picks valid shapes whose calls still match the oracle."""
    from paper_1401_3615_amd import autotune
    geom = autotune.carm_geometry(12, 256, 200, 1.5)
    res = autotune.tune(geom, [40], slots=(fdk.F32, fdk.TUNE_ADJOINT), reps=1)
    assert {r.slot for r in res} == {fdk.F32, fdk.TUNE_ADJOINT}
    path = tmp_path / "t.txt"
    autotune.write(res, str(path))
    try:
        assert fdk.load_tuning(str(path)) == 2
        vol = fdk.Volume(40, 0.5 * 512 / 40)
        r32 = [r for r in res if r.slot == fdk.F32][0]
        assert fdk.get_tile(vol, fdk.F32) == (r32.strip, r32.waves, r32.layout)
        q = torch.randn(12, 200, 256, generator=torch.Generator().manual_seed(3))
        out = fdk.backproject(q.to(DEV), geom, vol)
        torch.cuda.synchronize()
        ref = oracle.backproject(40, vol.voxel_mm, geom.mats, q.numpy())
        assert_parity(out.cpu().numpy(), ref, what="tuned shape")
    finally:
        for r in res:
            fdk.set_tuning_entry(r.slot, r.size_class, 0, 0)


@pytest.mark.parametrize("layout", [0, 1, 3])
def test_batched_layouts(fdk, layout):
    """The persistent kernel with FP32 scans gathering from plain or quad
    staged images, or sampling LDS windows."""
    scans, host = make_scans(fdk, SPECS, [torch.float32] * len(SPECS))
    fdk.set_tile(fdk.TUNE_BATCHED, 8, 4, layout)
    try:
        fdk.backproject_batched(scans)
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_BATCHED, 0, 0)
    for sc, (L, voxel, mats, q, qd, scale) in zip(scans, host):
        ref = oracle.backproject(L, voxel, mats, q.numpy())
        assert_parity(sc.out.cpu().numpy(), ref, what=f"batched layout {layout} L={L}")


@pytest.mark.parametrize("strip,waves", [(32, 4), (8, 2)])
def test_batched_unstaged_edges_and_large_windows(fdk, strip, waves):
    """FP32 scans sampling LDS windows read the caller's images directly:
    windows at the detector edges (volumes overfilling small detectors, odd
    width) are bounds-checked, and windows larger than the LDS tile (large
    voxels on a fine detector) take the checked gather."""
    specs = [(40, 8.0, 7, 48, 36, 31), (36, 8.0, 5, 256, 192, 32), (33, 6.0, 6, 61, 45, 33),
             (16, 24.0, 9, 48, 40, 34), (16, 12.0, 8, 48, 40, 35)]
    scans, host = make_scans(fdk, specs, [torch.float32] * len(specs))
    fdk.set_tile(fdk.TUNE_BATCHED, strip, waves, 3)
    try:
        fdk.backproject_batched(scans)
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_BATCHED, 0, 0)
    for sc, (L, voxel, mats, q, qd, scale) in zip(scans, host):
        ref = oracle.backproject(L, voxel, mats, q.numpy())
        assert_parity(sc.out.cpu().numpy(), ref, what=f"unstaged L={L} W={sc.geom.width}")


@pytest.mark.parametrize("layout", [3, 0])
def test_batched_mixed_orbits(fdk, layout):
    """A batch mixing circular scans (u and w constant along z) with tilted
    ones (w varies along z): the persistent kernel takes the column walk for
    the circular scans and the per-voxel walk for the tilted ones (layout 3),
    or gathers (layout 0).  Against the oracle and against one launch per
    scan."""
    specs = [(30, 4.0, 9, 128, 96, 0.0, 60), (28, 4.0, 7, 96, 72, 0.4, 61), (24, 5.0, 11, 128, 96, 0.4, 62),
             (32, 3.5, 6, 160, 120, 0.0, 63)]
    scans, refs = [], []
    for L, voxel, n, W, H, tilt, seed in specs:
        carm = S.CArm(n, W, H, pixel=384.0 / W, tilt_deg=tilt)
        mats, q = S.filtered_projections(carm, seed)
        scans.append(fdk.Scan(q.to(DEV), fdk.Geometry(mats, W, H), fdk.Volume(L, voxel),
                              torch.full((L, L, L), float("nan"), device=DEV)))
        refs.append(oracle.backproject(L, voxel, mats, q.numpy()))
    fdk.set_tile(fdk.TUNE_BATCHED, 8, 4, layout)
    fdk.set_tile(fdk.F32, 8, 4, layout)
    try:
        fdk.backproject_batched(scans)
        singles = [fdk.backproject(s.proj, s.geom, s.vol) for s in scans]
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_BATCHED, 0, 0)
        fdk.set_tile(fdk.F32, 0, 0)
    for sc, ref, one, sp in zip(scans, refs, singles, specs):
        got = sc.out.cpu().numpy()
        assert_parity(got, ref, what=f"mixed orbits layout {layout} tilt {sp[5]}")
        assert oracle.rel_l2(got, one.cpu().numpy()) < 1e-6


@pytest.mark.parametrize("tile", [None, (32, 4, 3)])
def test_batched_benchmark_scans(fdk, tile):
    """The batched benchmark's 16 scans at their own sizes (L up to 256, N up
    to 496, 1248x960 or 620x480 detectors, SID 600-800 mm, each with its own
    seeded phantom), with the default tile and with the shape the autotuner
    picks for them; every scan against the oracle at sampled voxels
    (including its corners and centre).  The call accumulates onto zeros: a
    work item run twice would show."""
    specs = S.batched_scan_specs(16, seed=100)
    data = S.batched_phantom_scans(specs, device=DEV)
    scans = []
    for sp, (mats, q) in zip(specs, data):
        scans.append(fdk.Scan(q.contiguous(), fdk.Geometry(mats, sp.width, sp.height), fdk.Volume(sp.L, sp.voxel_mm),
                              torch.zeros((sp.L, sp.L, sp.L), device=DEV)))
    if tile is not None:
        fdk.set_tile(fdk.TUNE_BATCHED, *tile)
    try:
        fdk.backproject_batched(scans, accumulate=True)
        torch.cuda.synchronize()
    finally:
        fdk.set_tile(fdk.TUNE_BATCHED, 0, 0)
    rng = np.random.default_rng(7)
    for i, (sp, sc, (mats, q)) in enumerate(zip(specs, scans, data)):
        L = sp.L
        corners = np.array([[x, y, z] for x in (0, L - 1) for y in (0, L - 1) for z in (0, L - 1)])
        xyz = np.concatenate([rng.integers(0, L, size=(300, 3)), corners, [[L // 2] * 3]])
        ref = oracle.backproject_points(xyz, sp.voxel_mm, mats, q.cpu().numpy().astype(np.float64), L=L)
        idx = torch.as_tensor(xyz.astype(np.int64), device=DEV)
        got = sc.out[idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()
        assert np.all(np.isfinite(got))
        err = oracle.rel_l2(got, ref)
        assert err <= 1e-5, f"scan {i} (L={L}, N={sp.n_proj}, {sp.width}x{sp.height}): rel L2 {err:.3e}"
        assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max(), f"scan {i}: element error"
