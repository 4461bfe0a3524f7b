"""Autotuner for the backprojection and forward-projection tile shapes.

For every (tuning slot, volume size class) it times each compiled tile shape
and staged layout on the caller's geometry with random projection data and
keeps the fastest; the result is a tuning file the library reads
(`fdk_load_tuning`, or the FDK_TUNING_FILE environment variable):

    fdk-tuning 1 gfx950
    # slot class strip waves layout   (GUp/s)
    0 9 16 4 3

Slots: 0 FP32, 1 FP16, 2 BF16 (backprojection by projection dtype), 3 the
forward projector, 4 the batched persistent launch (`tune_batched`, timed on
the caller's scans).  Size class = floor(log2(L)).

    python -m paper_1401_3615_amd.autotune --out tuning.txt [--sizes 128,256,512]
        [--slots 0,1,2,3] [--n-proj 124] [--detector 1248x960] [--load]

The command line tunes on a circular C-arm (200 degree short scan, SID 750 mm,
SDD 1200 mm) of the given detector; `tune()` takes any geometry.
"""
from __future__ import annotations

import argparse
import math
import sys
from dataclasses import dataclass

import torch

from . import (F16, F32, BF16, TUNE_ADJOINT, TUNE_BATCHED, FdkError, Geometry, Volume, abi_version,
               backproject, backproject_batched, forwardproject, load, load_tuning, pack_projections, set_tile,
               set_tuning_entry)

BP_STRIPS = (2, 4, 8, 16, 32)
BP_WAVES = (1, 2, 4)
BP_LAYOUTS = (0, 1, 2, 3)
ADJ_SHAPES = [(r, g, 4) for r in (12, 28, 60) for g in (1, 2, 4)] + [(8, 2, 0), (16, 4, 0)]


@dataclass
class Result:
    slot: int
    size_class: int
    strip: int
    waves: int
    layout: int
    gups: float


def size_class(L: int) -> int:
    return int(math.floor(math.log2(L)))


def candidates(slot: int):
    if slot == TUNE_ADJOINT:
        return list(ADJ_SHAPES)
    return [(s, w, lay) for s in BP_STRIPS for w in BP_WAVES for lay in BP_LAYOUTS
            if not (lay == 3 and w == 1 and s <= 4)]


def _time(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(geom: Geometry, sizes, voxel_mm_at_512: float = 0.5, slots=(F32, F16, BF16, TUNE_ADJOINT),
         reps: int = 3, device: str = "cuda:0", log=None) -> list[Result]:
    """Fastest shape per (slot, size class) for `geom`; volumes of edge L use
    voxels of voxel_mm_at_512 * 512 / L (the same field of view)."""
    load()
    gen = torch.Generator(device=device)
    gen.manual_seed(1234)
    N, H, W = geom.n_proj, geom.height, geom.width
    proj = torch.randn((N, H, W), device=device, generator=gen)
    packed = {F16: pack_projections(proj, torch.float16), BF16: pack_projections(proj, torch.bfloat16)}
    results = []
    for L in sizes:
        vol = Volume(L, voxel_mm_at_512 * 512.0 / L)
        out = torch.empty((L, L, L), device=device)
        x = torch.randn((L, L, L), device=device, generator=gen)
        pout = torch.empty((N, H, W), device=device)
        for slot in slots:
            best = None
            for strip, waves, layout in candidates(slot):
                try:
                    set_tile(slot, strip, waves, layout)
                except FdkError:
                    continue
                try:
                    if slot == TUNE_ADJOINT:
                        fn = lambda: forwardproject(x, geom, vol, out=pout)
                    elif slot == F32:
                        fn = lambda: backproject(proj, geom, vol, out=out)
                    else:
                        data, sc = packed[slot]
                        fn = lambda data=data, sc=sc: backproject(data, geom, vol, out=out, scale=sc)
                    ms = _time(fn, reps)
                finally:
                    set_tile(slot, 0, 0)
                gups = L ** 3 * N / (ms * 1e-3) / 1e9
                if best is None or gups > best.gups:
                    best = Result(slot, size_class(L), strip, waves, layout, gups)
            if best is not None:
                results.append(best)
                if log:
                    log(f"slot {slot} L={L}: {best.strip}x{best.waves} layout {best.layout} "
                        f"{best.gups:.1f} GUp/s")
    return results


BATCHED_SHAPES = [(s, w, lay) for s in (8, 16, 32) for w in (2, 4) for lay in (0, 1, 3)]


def tune_batched(scans, candidates=None, reps: int = 2, log=None) -> Result:
    """Fastest (strip, waves, FP32 layout) of the batched persistent launch for
    these scans (each candidate captures its own graph; the first call of a
    candidate is not timed)."""
    load()
    maxL = max(sc.vol.L for sc in scans)
    best = None
    for strip, waves, layout in candidates or BATCHED_SHAPES:
        try:
            set_tile(TUNE_BATCHED, strip, waves, layout)
        except FdkError:
            continue
        try:
            ms = _time(lambda: backproject_batched(scans), reps)
        finally:
            set_tile(TUNE_BATCHED, 0, 0)
        gups = sum(sc.vol.L ** 3 * sc.geom.n_proj for sc in scans) / (ms * 1e-3) / 1e9
        if best is None or gups > best.gups:
            best = Result(TUNE_BATCHED, size_class(maxL), strip, waves, layout, gups)
    if log and best:
        log(f"batched: {best.strip}x{best.waves} layout {best.layout} {best.gups:.1f} GUp/s")
    return best


def write(results, path: str) -> None:
    with open(path, "w") as f:
        f.write(f"fdk-tuning {abi_version()} gfx950\n")
        f.write("# slot class strip waves layout   (GUp/s measured)\n")
        for r in results:
            f.write(f"{r.slot} {r.size_class} {r.strip} {r.waves} {r.layout}   # {r.gups:.1f}\n")


def apply(results) -> None:
    """Install the results into the running library's tuning table."""
    for r in results:
        set_tuning_entry(r.slot, r.size_class, r.strip, r.waves, r.layout)


def carm_geometry(n_proj: int, width: int, height: int, pixel_mm: float, sid: float = 750.0,
                  sdd: float = 1200.0, arc_deg: float = 200.0) -> Geometry:
    """Circular short-scan C-arm about z: P_k = K [R_k | t_k] in FP64."""
    import numpy as np
    f = sdd / pixel_mm
    cu, cv = (width - 1) / 2.0, (height - 1) / 2.0
    K = np.array([[f, 0.0, cu], [0.0, f, cv], [0.0, 0.0, 1.0]])
    mats = np.empty((n_proj, 3, 4))
    for k in range(n_proj):
        th = math.radians(k * arc_deg / max(n_proj - 1, 1))
        c, s = math.cos(th), math.sin(th)
        R = np.array([[-s, c, 0.0], [0.0, 0.0, -1.0], [-c, -s, 0.0]])
        t = -R @ (sid * np.array([c, s, 0.0]))
        mats[k] = K @ np.concatenate([R, t[:, None]], axis=1)
    return Geometry(mats, width, height)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1401_3615_amd.autotune")
    ap.add_argument("--out", required=True)
    ap.add_argument("--sizes", default="128,256,512")
    ap.add_argument("--slots", default="0,1,2,3")
    ap.add_argument("--n-proj", type=int, default=124)
    ap.add_argument("--detector", default="1248x960", help="WIDTHxHEIGHT")
    ap.add_argument("--pixel-mm", type=float, default=0.308)
    ap.add_argument("--load", action="store_true", help="load the written file into the library")
    a = ap.parse_args(argv)
    W, H = (int(v) for v in a.detector.split("x"))
    geom = carm_geometry(a.n_proj, W, H, a.pixel_mm)
    res = tune(geom, [int(s) for s in a.sizes.split(",")], slots=[int(s) for s in a.slots.split(",")],
               log=lambda m: print(m, file=sys.stderr, flush=True))
    write(res, a.out)
    if a.load:
        load_tuning(a.out)
    print(a.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
