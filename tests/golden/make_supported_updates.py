"""Writes supported_updates.json: for each benchmark workload, the number of
(voxel, projection) pairs whose bilinear sample touches the detector (at least
one of its four taps lies on it), counted by the FP64 oracle.  This is the
update count of the paper's GUp/s convention, where the clipping mask removes
voxels that project off the detector (Sec. "Performance Model" counts the
clipped volume once per projection).

Run from the repository root:  python tests/golden/make_supported_updates.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synthetic as S  # noqa: E402

WORKLOADS = {
    "512^3 @0.5mm x 496 x 1248x960, 200deg C-arm": (512, 0.5, S.CArm(496)),
    "512^3 @0.5mm x 496 x 1248x960, 200deg C-arm tilted 0.5deg": (512, 0.5, S.CArm(496, tilt_deg=0.5)),
    "1024^3 @0.25mm x 496 x 1248x960, 200deg C-arm": (1024, 0.25, S.CArm(496)),
}


def main() -> int:
    oracle.build(force=False)
    out = {}
    for name, (L, voxel, carm) in WORKLOADS.items():
        mats = S.carm_matrices(carm)
        n = oracle.supported_updates(L, voxel, mats, carm.width, carm.height)
        out[name] = {"L": L, "voxel_mm": voxel, "n_proj": carm.n_proj, "nominal": L ** 3 * carm.n_proj,
                     "supported": n, "fraction": n / (L ** 3 * carm.n_proj)}
        print(name, out[name], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "supported_updates.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    return 0


if __name__ == "__main__":
    sys.exit(main())
