"""Large-detector form (the paper's outlook to industrial scanners with
10000 x 10000 pixel projections, over 380 MiB each): projections in pinned
host memory streamed to the device one detector row band per z-slab, into a
z-range of a 4096^2 grid, against the oracle at sampled voxels."""
import numpy as np
import pytest
import torch

import oracle
import synthetic as S
from tests._common import ensure_built

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def fdk():
    ensure_built()
    import paper_1401_3615_amd as m
    m.load()
    return m


def test_xxl_detector_streamed_row_bands(fdk):
    carm = S.xxl_carm(4)
    mats, q = S.filtered_projections(carm, seed=3, device=DEV)
    host = q.cpu().pin_memory()
    del q
    torch.cuda.empty_cache()
    L, voxel, z0, nz = 4096, 0.25, 2000, 96
    geom = fdk.Geometry(mats, carm.width, carm.height)
    part = fdk.Volume(L, voxel).slab(z0, nz)
    rows, first = fdk.streamed_plan(geom, part, 32)
    # each slab reads a band of a few hundred of the 10000 rows
    assert rows.max() < 600, rows
    out = fdk.backproject_streamed(host, geom, part, 32)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    xyz = np.stack([rng.integers(0, L, 600), rng.integers(0, L, 600), rng.integers(z0, z0 + nz, 600)], 1)
    xyz = np.concatenate([xyz, [[2048, 2048, z0], [2048, 2048, z0 + nz - 1], [100, 3000, z0 + 31],
                                [3000, 100, z0 + 32], [0, 0, z0], [L - 1, L - 1, z0 + nz - 1]]]).astype(np.int32)
    ref = oracle.backproject_points(xyz, voxel, mats, host.numpy(), L=L)
    idx = torch.as_tensor(xyz.astype(np.int64), device=DEV)
    got = out[idx[:, 2] - z0, idx[:, 1], idx[:, 0]].double().cpu().numpy()
    assert np.all(np.isfinite(got))
    assert np.abs(ref).max() > 0
    err = oracle.rel_l2(got, ref)
    print(f"10000^2 detector, 4096^2 x {nz} planes: rel L2 over {len(ref)} sampled voxels {err:.3e}, "
          f"band rows per slab {rows.tolist()}")
    assert err <= 1e-5
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
