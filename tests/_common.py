"""Shared helpers for the tests: seeded cases and tolerance checks."""
from __future__ import annotations

import os

import numpy as np

import oracle
import synthetic as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# FP32 bar for backprojection against the FP64 oracle (relative L2 over the
# volume), as required for the FP32 path.  Element-wise, every voxel is also
# held to ELEM_TOL * max|V_oracle|: the FP32 coordinate error of ~1e-4 px times
# the projections' local slope, summed over projections, stays two orders of
# magnitude below the largest voxel on the smooth filtered-phantom data.
REL_L2_FP32 = 1e-5
ELEM_TOL = 1e-4


def ensure_built():
    """Build the HIP library and the oracle if (and only if) nothing is built."""
    from paper_1401_3615_amd import _build
    if not os.path.exists(_build.LIB):
        _build.build_library(force=True)
    oracle.build(force=False)


def small_carm(n_proj, width, height, seed=0, full_width_mm=384.0):
    """A C-arm whose detector keeps the physical 384 mm width with fewer pixels."""
    pixel = full_width_mm / width
    return S.CArm(n_proj, width, height, pixel=pixel)


def phantom_case(carm, seed=0, device="cpu"):
    mats, q = S.filtered_projections(carm, seed, device=device)
    return mats, q


def assert_parity(got, ref, rel=REL_L2_FP32, elem=ELEM_TOL, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite output"
    err = oracle.rel_l2(got, ref)
    scale = np.abs(ref).max()
    maxerr = np.abs(got - ref).max()
    assert err <= rel, f"{what}: rel L2 {err:.3e} > {rel:.1e}"
    assert maxerr <= elem * scale, f"{what}: max error {maxerr:.3e} > {elem:.0e} * {scale:.3e}"
    return err
