#!/usr/bin/env python3
"""Throughput of voxel-driven FDK backprojection on one MI355X.

Headline workload: a 512^3 volume (0.5 mm voxels) backprojected from 496
filtered 1248x960 projections of a seeded ellipsoid phantom on a 200-degree
C-arm short scan (the paper's RabbitCT shapes).  One step is one
fdk_backproject call on FP32 projections (matrix conditioning from the cached
table, zero-padded staging, coefficient fold, backprojection kernel); `value`
is L^3 * N / step time in GUp/s with the projections resident in HBM.

The same JSON line carries the other forms measured on the same GPU: FP16 and
BF16 projection storage, the adjoint (forward projector), the batched
persistent launch of 16 uneven scans against one launch per scan, and the
1024^3 volume processed as z-slabs; plus the roofline of the backprojection
kernel and the FP64 oracle timed on the host cores as the CPU baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--legs ...]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FLOP_PER_UPDATE = 22          # FP operations of one voxel update (FMA = 2): u, v, w 6; ix, iy 2 (plus one
                              # reciprocal, not counted); floor and fraction 2; bilinear 3 sub + 3 FMA = 9;
                              # weight and accumulate 1 mul + 1 FMA = 3
PEAK_FP32_TFLOPS = 157.3      # MI355X published FP32 vector peak
PEAK_FP32_NONPACKED = 78.6    # 256 CU x 64 lanes x 2 (FMA) x 2.4 GHz, without packed FP32
COUNTERS_FILE = os.path.join(ROOT, "profiles", "bp_f32_512x496_counters.json")
KERNEL_SRC = os.path.join(ROOT, "paper_1401_3615_amd", "csrc", "fdk_kernels.hip")
COPY_BYTES = 1 << 30          # calibration kernel traffic each way (profile runs only)


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bp_kernel_name(fdk, vol, geom) -> str:
    """Name of the FP32 backprojection kernel the library launches for `vol`
    (the LDS kernel is instantiated for u and w constant along z (3: zero
    z-coefficients in every matrix's first and third rows), w constant (1) or
    neither (0), and for reading staged images or the caller's stack in
    place, which it does for grids with fewer than one voxel per eight
    projection pixels)."""
    import numpy as np
    strip, waves, layout = fdk.get_tile(vol, fdk.F32)
    if layout == 3:
        m = np.asarray(geom.mats).reshape(-1, 3, 4)
        w_const = bool(np.all(m[:, 2, 2] == 0.0))
        cw = 3 if w_const and bool(np.all(m[:, 0, 2] == 0.0)) else int(w_const)
        pixels = len(m) * geom.width * geom.height
        in_place = vol.planes * vol.L * vol.L * 8 < pixels and os.environ.get("FDK_STAGE_FP32") != "1"
        return f"bp_lds_kernel<float, {strip}, {waves}, {cw}, {str(in_place).lower()}>"
    return f"bp_kernel<float, {layout}, {strip}, {waves}>"


SUPPORTED_FILE = os.path.join(ROOT, "tests", "golden", "supported_updates.json")
HEADLINE_KEY = "512^3 @0.5mm x 496 x 1248x960, 200deg C-arm"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def supported_gups(nominal: int, ms: float):
    """GUp/s over supported updates (count written by the oracle), or None."""
    try:
        with open(SUPPORTED_FILE) as f:
            rec = json.load(f)[HEADLINE_KEY]
    except (OSError, KeyError, ValueError):
        return None
    if rec["nominal"] != nominal:
        return None
    return round(rec["supported"] / (ms * 1e-3) / 1e9, 2)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def time_steps(fn, steps: int, warmup: int, stream):
    """Untimed warm-up, then `steps` calls bracketed by synchronisation and
    HIP events on the launch stream; returns ms per step."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU-oracle baseline leg")
    ap.add_argument("--legs", default="fp16,bf16,tilted,adjoint,iterative,batched,slab1024,streamed,filter,xxl",
                    help="comma list of extra legs (fp16,bf16,tilted,adjoint,iterative,batched,slab1024,"
                         "streamed,filter,xxl) or 'none'")
    ap.add_argument("--profile-only", action="store_true",
                    help="run only warm-up and timed FP32 steps (for profiler runs)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(z-slab sharding across GPUs is described, not built); run with --gpus 1", file=sys.stderr)
        return 2
    legs = set() if args.legs == "none" else set(args.legs.split(","))

    import numpy as np
    import torch

    import paper_1401_3615_amd as fdk
    from paper_1401_3615_amd import _build
    import synthetic as S

    if not os.path.exists(_build.LIB):
        log("library not built; building")
        _build.build_library(force=True)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream()

    # ---------------------------------------------------------------- workload
    L, voxel, N = 512, 0.5, 496
    carm = S.CArm(N)
    t0 = time.time()
    mats, q = S.filtered_projections(carm, seed=0, device=dev)
    q = q.contiguous()
    torch.cuda.synchronize()
    log(f"phantom projections {tuple(q.shape)} generated on the GPU in {time.time() - t0:.1f} s")
    geom = fdk.Geometry(mats, carm.width, carm.height)
    vol = fdk.Volume(L, voxel)
    out = torch.empty((L, L, L), dtype=torch.float32, device=dev)
    updates = L ** 3 * N

    # ---------------------------------------------------------------- FP32 headline
    bp32 = lambda: fdk.backproject(q, geom, vol, out=out)
    fdk.profile_enable(False)
    for _ in range(args.warmup):
        bp32()
    torch.cuda.synchronize()
    fdk.profile_enable(True)
    ms = time_steps(bp32, args.steps, 0, stream)
    n_bp, bp_ms_total = fdk.profile_read("bp")
    n_st, st_ms_total = fdk.profile_read("stage")
    fdk.profile_enable(False)
    bp_kernel_ms = bp_ms_total / max(n_bp, 1)
    stage_ms = st_ms_total / max(n_st, 1)
    value = updates / (ms * 1e-3) / 1e9
    log(f"fp32: {ms:.2f} ms/step, {value:.1f} GUp/s (bp kernel {bp_kernel_ms:.2f} ms, staging {stage_ms:.2f} ms)")
    if args.profile_only:
        # calibration for HBM counters: an elementwise kernel that reads and
        # writes COPY_BYTES each
        src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.bitwise_not(src, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"metric": "fp32_gups", "value": value, "ms_per_step": ms,
                          "kernel": bp_kernel_name(fdk, vol, geom), "copy_bytes_each_way": COPY_BYTES}), flush=True)
        return 0
    vol32 = out.clone()

    extra = {}
    # ---------------------------------------------------------------- FP16 / BF16 storage
    packed = {}
    packed_stacks = {}
    for name, tdt in (("fp16", torch.float16), ("bf16", torch.bfloat16)):
        if name not in legs:
            continue
        pk_ms = time_steps(lambda: fdk.pack_projections(q, tdt), 1, 1, stream)
        qp, sc = fdk.pack_projections(q, tdt)
        fn = lambda qp=qp, sc=sc: fdk.backproject(qp, geom, vol, out=out, scale=sc)
        m = time_steps(fn, args.steps, args.warmup, stream)
        packed[name] = out.clone()
        extra[f"{name}_gups"] = updates / (m * 1e-3) / 1e9
        extra[f"{name}_ms_per_step"] = m
        extra[f"{name}_pack_ms"] = pk_ms
        log(f"{name}: {m:.2f} ms/step, {extra[f'{name}_gups']:.1f} GUp/s (pack {pk_ms:.2f} ms, not in step)")
        if name == "fp16":
            packed_stacks[name] = (qp, sc)   # reused by the 1024^3 FP16 leg
        del qp, sc

    # ---------------------------------------------------------------- FDK preprocessing
    if "filter" in legs:
        # line integrals of the same phantom, filtered on the GPU (cosine, Parker, ramp),
        # against the host generator's FP64 FFT filter
        li = S.project_phantom(mats, carm.width, carm.height, S.ellipsoid_phantom(0), device=dev).float()
        q64 = S.fdk_filter(li.double(), carm)    # FP64 filter of the same FP32 input: the kernel's error
        li = li.contiguous()
        cu, cv = carm.principal_point
        arc = math.radians(carm.arc_deg)
        fg = fdk.FilterGeometry(angles_rad=carm.angles_rad(), width=carm.width, height=carm.height,
                                pixel_u_mm=carm.pixel, pixel_v_mm=carm.pixel, u0=cu, v0=cv, sdd_mm=carm.sdd,
                                sid_mm=carm.sid, scan_range_rad=arc, dbeta_rad=arc / (N - 1), fan_sign=-1.0)
        qf = torch.empty_like(li)
        m = time_steps(lambda: fdk.filter_projections(li, fg, out=qf), args.steps, args.warmup, stream)
        mh = time_steps(lambda: fdk.filter_projections(li, fg, dtype=torch.float16), args.steps, args.warmup,
                        stream)
        fdk.filter_projections(li, fg, out=qf)
        torch.cuda.synchronize()
        err = float(((qf.double() - q64).norm() / q64.norm()).item())
        nbytes = 2 * li.numel() * 4
        extra["filter_ms"] = m
        extra["filter_fp16_ms"] = mh
        extra["filter_gbps"] = nbytes / (m * 1e-3) / 1e9
        extra["filter_rel_l2_vs_fp64"] = float(f"{err:.3e}")
        log(f"filter 496 x 960 x 1248: {m:.2f} ms ({extra['filter_gbps']:.0f} GB/s of 4.75 GB read+write), "
            f"to FP16 {mh:.2f} ms; rel L2 vs FP64 {err:.2e}")
        del li, q64, qf

    # ---------------------------------------------------------------- general path
    if "tilted" in legs:
        # the same workload on a C-arm tilted by 0.5 degree: w varies along z,
        # so the kernel takes 1/w per voxel (as for calibrated real systems)
        carm_t = S.CArm(N, tilt_deg=0.5)
        mats_t, q_t = S.filtered_projections(carm_t, seed=0, device=dev)
        q_t = q_t.contiguous()
        geom_t = fdk.Geometry(mats_t, carm_t.width, carm_t.height)
        m = time_steps(lambda: fdk.backproject(q_t, geom_t, vol, out=out), args.steps, args.warmup, stream)
        extra["tilted_gups"] = updates / (m * 1e-3) / 1e9
        extra["tilted_ms_per_step"] = m
        log(f"fp32, C-arm tilted 0.5 deg (per-voxel 1/w): {m:.2f} ms/step, {extra['tilted_gups']:.1f} GUp/s")
        del q_t

    # ---------------------------------------------------------------- adjoint
    if "adjoint" in legs:
        pout = torch.empty_like(q)
        fn = lambda: fdk.forwardproject(vol32, geom, vol, out=pout)
        m = time_steps(fn, max(1, min(args.steps, 3)), 1, stream)
        extra["adjoint_gups"] = updates / (m * 1e-3) / 1e9
        extra["adjoint_ms_per_step"] = m
        sup = supported_gups(updates, m)
        if sup is not None:
            # four FP64 LDS atomic adds per supported update (a lower bound: samples near a
            # tile edge are scattered by both tiles)
            extra["adjoint_supported_gups"] = sup
            extra["adjoint_lds_atomics_per_s"] = 4.0 * sup * 1e9
        log(f"adjoint 512^3x496: {m:.2f} ms/step, {extra['adjoint_gups']:.1f} GUp/s")
        del pout

    # ---------------------------------------------------------------- iterative reconstruction
    if "iterative" in legs:
        # CGLS and SIRT on the matched pair at 256^3 @ 0.5 mm from the exact line
        # integrals of the phantom (496 x 1248x960); one iteration = one forward
        # and one backprojection (2 L^3 N updates) plus the vector kernels
        Li, voxi = 256, 0.5
        voli = fdk.Volume(Li, voxi)
        li = S.project_phantom(mats, carm.width, carm.height, S.ellipsoid_phantom(0), device=dev).float()
        li = li.contiguous()
        per_it = 2 * Li ** 3 * N
        for name, run in (("cgls", lambda n: fdk.cgls(li, geom, voli, n, history=True)),
                          ("sirt", lambda n: fdk.sirt(li, geom, voli, n, history=True))):
            n_it = 5
            run(1)
            torch.cuda.synchronize()
            m1 = time_steps(lambda: run(1), 2, 0, stream)
            fdk.profile_enable(True)
            m5 = time_steps(lambda: run(n_it), 2, 0, stream)
            parts = {k: fdk.profile_read(k)[1] / 2 for k in ("fp", "bp", "stage", "window", "fold", "iter")}
            fdk.profile_enable(False)
            x, hist = run(n_it)
            torch.cuda.synchronize()
            h = hist.cpu().numpy()
            it_ms = (m5 - m1) / (n_it - 1)
            extra[f"{name}_ms_per_iter"] = it_ms
            extra[f"{name}_gups"] = per_it / (it_ms * 1e-3) / 1e9
            extra[f"{name}_setup_ms"] = m1 - it_ms
            extra[f"{name}_residual_ratio_5"] = float(h[-1] / h[0])
            brk = ", ".join(f"{k} {v / n_it:.2f}" for k, v in parts.items())
            log(f"{name} 256^3 x 496: {it_ms:.2f} ms/iteration ({extra[f'{name}_gups']:.1f} GUp/s over 2 L^3 N), "
                f"setup {m1 - it_ms:.2f} ms; per-iteration ms by kind: {brk}; ||r_5||^2/||r_0||^2 = {h[-1] / h[0]:.3e}")
            del x, hist
        del li

    # ---------------------------------------------------------------- 1024^3 in z-slabs
    if "slab1024" in legs:
        # 1024^3 @ 0.25 mm (4 GiB) in 64-plane z-slabs, each reading only the
        # detector row band it projects onto (a device-to-device copy of the band
        # rows, the band offset folded into the matrices); for comparison the
        # plain per-slab call on the whole stack with 256-plane slabs
        L2, vox2 = 1024, 0.25
        big = torch.empty((L2, L2, L2), dtype=torch.float32, device=dev)
        base = fdk.Volume(L2, vox2)
        m = time_steps(lambda: fdk.backproject_streamed(q, geom, base, 64, out=big), max(1, min(args.steps, 3)), 1,
                       stream)
        slabs = [(z, 256) for z in range(0, L2, 256)]

        def slab_run():
            for z0, nz in slabs:
                fdk.backproject(q, geom, base.slab(z0, nz), out=big[z0:z0 + nz])
        mw = time_steps(slab_run, max(1, min(args.steps, 3)), 1, stream)
        extra["slab1024_gups"] = L2 ** 3 * N / (m * 1e-3) / 1e9
        extra["slab1024_ms_per_step"] = m
        extra["slab1024_whole_stack_slabs256_ms"] = mw
        log(f"1024^3 x 496 in 64-plane z-slabs with row bands: {m:.1f} ms, {extra['slab1024_gups']:.1f} GUp/s "
            f"(whole stack per 256-plane slab: {mw:.1f} ms)")
        # the FP16-projection form of the same volume (FP16 stack packed outside the step)
        qh, sh = packed_stacks.get("fp16") or fdk.pack_projections(q, torch.float16)
        mh = time_steps(lambda: fdk.backproject_streamed(qh, geom, base, 64, out=big, scale=sh),
                        max(1, min(args.steps, 3)), 1, stream)
        extra["slab1024_fp16_gups"] = L2 ** 3 * N / (mh * 1e-3) / 1e9
        extra["slab1024_fp16_ms_per_step"] = mh
        log(f"1024^3 x 496 from FP16 projections, same slabs: {mh:.1f} ms, {extra['slab1024_fp16_gups']:.1f} GUp/s")
        del big, qh, sh

    # ---------------------------------------------------------------- out-of-core
    if "streamed" in legs:
        # the 1024^3 volume with the projection stack in pinned host memory: each
        # 128-plane slab receives only its detector row band over PCIe while the
        # previous slab is backprojected; then the volume kept in host memory too
        L2, vox2, slab = 1024, 0.25, 128
        base = fdk.Volume(L2, vox2)
        host_q = q.cpu().pin_memory()
        rows, _ = fdk.streamed_plan(geom, base, slab)
        h2d = float(rows.sum()) * N * carm.width * 4
        big = torch.empty((L2, L2, L2), dtype=torch.float32, device=dev)
        m = time_steps(lambda: fdk.backproject_streamed(host_q, geom, base, slab, out=big), 2, 1, stream)
        extra["streamed1024_gups"] = L2 ** 3 * N / (m * 1e-3) / 1e9
        extra["streamed1024_ms_per_step"] = m
        extra["streamed1024_h2d_gb"] = h2d / 1e9
        del big
        hv = torch.empty((L2, L2, L2), dtype=torch.float32).pin_memory()
        mh = time_steps(lambda: fdk.backproject_streamed(host_q, geom, base, slab, out=hv), 2, 1, stream)
        extra["streamed1024_host_volume_gups"] = L2 ** 3 * N / (mh * 1e-3) / 1e9
        extra["streamed1024_host_volume_ms_per_step"] = mh
        log(f"1024^3 x 496 streamed from host ({h2d / 1e9:.2f} GB of row bands over PCIe per pass): {m:.1f} ms, "
            f"{extra['streamed1024_gups']:.1f} GUp/s; volume in host memory too: {mh:.1f} ms, "
            f"{extra['streamed1024_host_volume_gups']:.1f} GUp/s")
        del hv, host_q

    # ---------------------------------------------------------------- large detector
    if "xxl" in legs:
        # the paper's outlook to industrial scanners: 8 projections of 10000 x 10000
        # pixels (381 MiB each) in pinned host memory, streamed one detector row
        # band per 32-plane slab into the middle 256 planes of a 4096^2 grid at
        # 0.25 mm (16 GiB on the device)
        xc = S.xxl_carm(8)
        t0 = time.time()
        xm, xq = S.filtered_projections(xc, seed=0, device=dev)
        xhost = xq.cpu().pin_memory()
        del xq
        torch.cuda.empty_cache()
        log(f"xxl: 8 filtered 10000x10000 projections generated in {time.time() - t0:.1f} s")
        xg = fdk.Geometry(xm, xc.width, xc.height)
        xv = fdk.Volume(4096, 0.25).slab(1920, 256)
        xrows, _ = fdk.streamed_plan(xg, xv, 32)
        xh2d = float(xrows.sum()) * 8 * xc.width * 4
        xout = torch.empty((256, 4096, 4096), dtype=torch.float32, device=dev)
        mx = time_steps(lambda: fdk.backproject_streamed(xhost, xg, xv, 32, out=xout), 2, 1, stream)
        xup = 4096 * 4096 * 256 * 8
        extra["xxl_gups"] = xup / (mx * 1e-3) / 1e9
        extra["xxl_ms_per_step"] = mx
        extra["xxl_h2d_gb"] = xh2d / 1e9
        extra["xxl_config"] = "8 x 10000x10000 fp32 projections (pinned host) -> 4096^2 x 256 planes @0.25mm, 32-plane slabs"
        log(f"xxl: 4096^2 x 256 from 8 x 10000x10000 projections in host memory ({xh2d / 1e9:.2f} GB of row bands): "
            f"{mx:.1f} ms, {extra['xxl_gups']:.1f} GUp/s")
        del xout, xhost

    # ---------------------------------------------------------------- batched
    if "batched" in legs:
        # 16 uneven scans, each with the filtered projections of its own seeded phantom
        specs = S.batched_scan_specs(16, seed=100)
        t0 = time.time()
        scans = []
        for sp, (m_i, q_i) in zip(specs, S.batched_phantom_scans(specs, device=dev)):
            scans.append(fdk.Scan(q_i.contiguous(), fdk.Geometry(m_i, sp.width, sp.height),
                                  fdk.Volume(sp.L, sp.voxel_mm),
                                  torch.empty((sp.L, sp.L, sp.L), device=dev)))
        torch.cuda.synchronize()
        log(f"batched: phantom projections of 16 scans generated in {time.time() - t0:.1f} s")
        total = sum(sp.L ** 3 * sp.n_proj for sp in specs)
        # tile shape of the persistent launch from the autotuner, timed on these scans (not in the step)
        from paper_1401_3615_amd import autotune
        t0 = time.time()
        tuned = autotune.tune_batched(scans, reps=2)
        autotune.apply([tuned])
        extra["batched_tile"] = [tuned.strip, tuned.waves, tuned.layout]
        log(f"autotuned batched tile {extra['batched_tile']} in {time.time() - t0:.1f} s")
        mb = time_steps(lambda: fdk.backproject_batched(scans), max(1, args.steps // 2), 1, stream)

        def one_at_a_time():
            for s in scans:
                fdk.backproject(s.proj, s.geom, s.vol, out=s.out)
        mo = time_steps(one_at_a_time, max(1, args.steps // 2), 1, stream)
        extra["batched_gups"] = total / (mb * 1e-3) / 1e9
        extra["batched_one_at_a_time_gups"] = total / (mo * 1e-3) / 1e9
        extra["batched_ms_per_step"] = mb
        log(f"batched 16 scans: {mb:.1f} ms ({extra['batched_gups']:.1f} GUp/s) vs one at a time "
            f"{mo:.1f} ms ({extra['batched_one_at_a_time_gups']:.1f} GUp/s)")
        del scans

    # ---------------------------------------------------------------- roofline
    achieved = FLOP_PER_UPDATE * updates / (bp_kernel_ms * 1e-3) / 1e12
    traffic = None
    if os.path.exists(COUNTERS_FILE):
        with open(COUNTERS_FILE) as f:
            cnt = json.load(f)
        if cnt.get("kernel_source_sha256") == kernel_hash():
            traffic = cnt["hbm_bytes_per_launch"]
    roofline = {"bound": "alu", "achieved": round(achieved, 2), "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4), "traffic": traffic,
                "kernel": bp_kernel_name(fdk, vol, geom), "kernel_ms": round(bp_kernel_ms, 3),
                "flop_per_update": FLOP_PER_UPDATE,
                "frac_of_nonpacked_peak": round(achieved / PEAK_FP32_NONPACKED, 4)}

    # ---------------------------------------------------------------- CPU oracle baseline + accuracy
    cpu = None
    if not args.no_cpu:
        # the FP64 oracle on the whole 512^3 volume (every voxel, every
        # projection) on the host's cores: the CPU baseline and the reference
        # of the accuracy figures
        import oracle
        q64 = q.cpu().numpy().astype(np.float64)
        t0 = time.time()
        ref = oracle.backproject(L, voxel, mats, q64)
        dt = time.time() - t0
        cpu = {"value": round(updates / dt / 1e9, 4), "unit": "GUp/s", "cores": oracle.num_threads(),
               "kind": "oracle", "nproc": os.cpu_count(), "cpu_model": cpu_model(),
               "sample": f"the whole 512^3 x 496 volume ({updates:.4g} updates, {dt:.1f} s)"}
        acc = {}
        for name, v in [("fp32", vol32)] + list(packed.items()):
            got = v.cpu().numpy()
            acc[name] = {"rel_l2": float(f"{oracle.rel_l2(got, ref):.3e}"),
                         "psnr_db": round(oracle.psnr(got, ref), 2)}
        extra["accuracy_vs_oracle"] = acc
        log(f"oracle {cpu['value']} GUp/s on {cpu['cores']} threads ({cpu['nproc']} CPUs, {cpu['cpu_model']}); "
            f"accuracy over all voxels {acc}")
        del q64, ref

    line = {
        "metric": "GUp/s at 512^3 vol x 496 proj: FP32 vs FP16-proj; fwd+adjoint GUp/s",
        "value": round(value, 2),
        "unit": "GUp/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fdk_backproject 512^3 @0.5mm <- 496 x 1248x960 fp32, 200deg C-arm, "
                               "10-ellipsoid phantom seed 0",
                   "L": L, "n_proj": N, "detector": [carm.height, carm.width]},
        "supported_update_fraction_note": "value counts L^3*N nominal updates; supported_gups counts only "
                                          "(voxel, projection) pairs whose sample touches the detector, the "
                                          "paper's convention (count from the oracle)",
        "supported_gups": supported_gups(updates, ms),
        "staging_ms": round(stage_ms, 3),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    # timings and rates to 3 decimals; error figures keep 4 significant digits
    line.update({k: (float(f"{v:.4g}") if "rel_l2" in k else round(v, 3)) if isinstance(v, float) else v
                 for k, v in extra.items()})
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
