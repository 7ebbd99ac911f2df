#!/usr/bin/env python3
"""Benchmark of the MI355X smooth-and-clip (S+C) finder.

One step = one whole S+C run (every kernel pair: smoothing, noise, clip into
the mask) over a cube already resident in HBM.

Default workload (the largest configuration that fits one GPU):
large_2048x2048x4096, one 2048 x 2048 x 4096 float32 cube (64 GiB, spectral
axis slowest) of Gaussian noise whose sigma varies 0.8-1.5 across the field,
a 26-px NaN border (5 % of the voxels) and 20000 mock galaxies; kernels
spatial {0, 3, 6, 9} px x spectral {0, 3, 7, 15, 31} ch; MAD noise on
negative voxels; threshold 3.5; replacement n = 2. It is generated slab by
slab straight into HBM.

Other workloads: plain_1024cube (1024^3, 12 kernels), batch96 (96 uneven
cubes in one graph launch, --batch-mode loop for one run call per cube),
paper_360x360x1464 and paper_1501cube (the shapes of the paper's two speed
tests); --storage f16/bf16 stores the cube noise-scaled in 16 bits inside
each run.

Unless --no-extras is given, the line also carries, measured in the same
process after the headline: the large cube with FP16 storage as a one-cube
graph launch, the 1024^3 workload in FP32 (also as a one-cube graph launch),
the local noise normalisation of that cube (31 px / 31 ch window) and the
linker on its S+C mask.

Prints one JSON line. `value` is voxels per second of whole runs; `roofline`
describes the kernel family with the largest share of device time, timed with
HIP events on the launch stream; `cpu_baseline` times the FP64 oracle on a
slab of the same cube on the host cores (and on one core).
"""
import argparse
import dataclasses
import hashlib
import json
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E peak
METRIC = "S+C voxels/s over all kernels (FP32 vs batched/FP16) at oracle mask match; % HBM peak"


def say(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """Hash of every kernel and host source of the library."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_15789_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".h")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(family: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counter summaries, if
    they were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{family}_{workload}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_src_sha") != kernel_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def upload(spec, torch, synth):
    """Generate a cube slab by slab (about 1 GiB each) straight into HBM."""
    x = torch.empty(spec.shape, dtype=torch.float32, device="cuda")
    slab = max(1, (1 << 28) // (spec.nx * spec.ny))
    for z0 in range(0, spec.nz, slab):
        z1 = min(spec.nz, z0 + slab)
        x[z0:z1].copy_(torch.from_numpy(synth.generate(spec, z0=z0, z1=z1)))
        if spec.nz > 8 * slab and (z0 // slab) % 16 == 15:
            say(f"planes 0-{z1 - 1} generated")
    return x


def count_set(m, torch) -> int:
    """Nonzero voxels of a uint8 mask, a slab at a time (a whole-cube reduction
    would materialise a wider copy)."""
    slab = max(1, (1 << 28) // (m.shape[1] * m.shape[2]))
    return sum(int(torch.count_nonzero(m[z0:z0 + slab]).item())
               for z0 in range(0, m.shape[0], slab))


def roofline(stats, workload, use_traffic=True):
    """The kernel family with the largest device time: algorithmic bytes per
    launch over its mean event-timed launch duration, against the HBM peak."""
    dom = max(stats, key=lambda s: s["total_ms"])
    avg_ms = dom["total_ms"] / dom["launches"]
    per_launch = dom["bytes"] / dom["launches"]
    achieved = per_launch / (avg_ms * 1e-3) / 1e9
    return {"bound": "hbm", "kernel": dom["name"], "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": read_traffic(dom["name"], workload) if use_traffic else None,
            "avg_launch_ms": avg_ms, "alg_bytes_per_launch": per_launch}


def family_gbs(stats):
    return {s["name"]: round(s["bytes"] / (s["total_ms"] * 1e-3) / 1e9, 1)
            for s in stats if s["bytes"] > 0 and s["total_ms"] > 0}


def time_runs(h, wl, xs, masks, steps, warmup, storage, graph, stream, torch):
    """Warm up, then time `steps` whole runs (or batched graph launches)
    between two device synchronisations, with per-launch events on."""
    def step():
        if graph:
            _, noise, s0 = h.run_batch(xs, wl.kernels, wl.threshold, wl.noise_mode,
                                       wl.flux_range, wl.replacement, masks=masks,
                                       stream=stream, storage=storage)
            return noise[0], s0[0]
        for xi, mi in zip(xs, masks):
            _, noise, s0 = h.run(xi, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                                 wl.replacement, mask=mi, stream=stream, storage=storage)
        return noise, s0

    for _ in range(warmup):
        step()
    h.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        noise, s0 = step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    h.profile(False)
    return dt, noise, s0, h.profile_read()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_sample(workload: str, planes: int) -> dict:
    """The FP64 oracle, unchanged, on planes [0, planes) of the workload's
    first cube: every kernel pair, noise measured on the slab."""
    import oracle
    import synth
    wl = synth.workload(workload)
    spec = wl.cubes[0]
    x = synth.generate(spec, z0=0, z1=planes)
    t0 = time.perf_counter()
    oracle.run(x, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range, wl.replacement)
    dt = time.perf_counter() - t0
    return {"voxels": int(x.size), "seconds": dt, "value": x.size / dt}


def cpu_baseline(workload, spec, n_kernels, planes, planes_1t):
    """The oracle on a slab of the same cube on all host threads, and on one
    thread in a child process (OpenMP fixes its thread count at start)."""
    multi = cpu_sample(workload, planes)
    threads = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--cpu-worker",
                        workload, str(planes_1t)], env=env, capture_output=True, text=True,
                       timeout=600)
    one = json.loads(r.stdout.strip().splitlines()[-1]) if r.returncode == 0 else None
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count()
    out = {"value": multi["value"], "unit": "voxels/s", "cores": threads, "kind": "oracle",
           "sample": f"planes 0-{planes - 1} of the same cube ({spec.nx}x{spec.ny}x{planes} "
                     f"voxels, all {n_kernels} kernel pairs, noise measured on the slab: the "
                     f"whole cube is beyond the host's time), {multi['seconds']:.1f} s",
           "cpu_model": cpu_model(), "nproc": nproc}
    if one:
        out["one_thread"] = {"value": one["value"], "unit": "voxels/s",
                             "sample": f"planes 0-{planes_1t - 1} ({one['voxels']} voxels), "
                                       f"{one['seconds']:.1f} s"}
    return out


def extras_repl_off(h, x, m, wl, noise_mode, flux_range, name, stream, torch, out):
    """Replacement off: the run one pair at a time and with fused widths."""
    leg = {"kernels": wl.kernels, "noise": noise_mode, "flux_range": flux_range,
           "replacement": None}
    for fuse in (False, True):
        def one():
            return h.run(x, wl.kernels, wl.threshold, noise_mode, flux_range, -1.0, mask=m,
                         stream=stream, fuse_widths=fuse)
        one()
        h.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            _, noise_f, _ = one()
        torch.cuda.synchronize()
        tf = (time.perf_counter() - t0) / 5
        h.profile(False)
        st = h.profile_read()
        key = "fused" if fuse else "per_pair"
        leg[key] = {"ms": tf * 1e3, "value": x.numel() / tf, "unit": "voxels/s",
                    "family_ms_per_run": {s["name"]: s["total_ms"] / 5 for s in st},
                    "kernel_gbs": family_gbs(st),
                    "noise": [float(v) for v in noise_f]}
        say(f"1024^3 replacement off, {noise_mode}, {key}: {tf * 1e3:.1f} ms")
    out[name] = leg


def extras(sc, torch, synth, stream, large_x=None, large_wl=None):
    """Secondary figures measured in the same process."""
    out = {}
    if large_x is not None:
        # the large cube with FP16 storage, as a one-cube graph launch
        h = sc.SofiaSC(0)
        try:
            m = torch.empty(large_x.shape, dtype=torch.uint8, device="cuda")
            dt, noise, s0, stats = time_runs(h, large_wl, [large_x], [m], 3, 1, "f16", True,
                                             stream, torch)
            out["large_f16_graph"] = {
                "ms_per_step": dt * 1e3 / 3, "value": large_x.numel() * 3 / dt,
                "unit": "voxels/s", "storage": "f16", "batch_mode": "graph",
                "roofline": roofline(stats, large_wl.name, use_traffic=False),
                "noise": [float(v) for v in noise]}
            say(f"large f16 graph: {dt * 1e3 / 3:.1f} ms/step")
            del m
        finally:
            h.close()
        torch.cuda.empty_cache()
    # the 1024^3 workload: S+C in FP32, noise normalisation, linker
    wl = synth.workload("plain_1024cube")
    x = upload(wl.cubes[0], torch, synth)
    m = torch.empty(x.shape, dtype=torch.uint8, device="cuda")
    h = sc.SofiaSC(0)
    try:
        dt, noise, s0, stats = time_runs(h, wl, [x], [m], 10, 2, "f32", False, stream, torch)
        alg = sum(s["bytes"] for s in stats) / 10
        out["plain_1024cube"] = {
            "ms_per_step": dt * 100, "value": x.numel() * 10 / dt, "unit": "voxels/s",
            "roofline": roofline(stats, wl.name),
            "whole_step_hbm_frac": alg / (dt / 10) / 1e9 / HBM_PEAK_GBS,
            "kernel_gbs": family_gbs(stats), "mask_voxels": count_set(m, torch)}
        say(f"1024^3 f32: {dt * 100:.1f} ms/step")
        # the same run as a one-cube graph launch (no launch gaps)
        dt, noise, s0, stats = time_runs(h, wl, [x], [m], 10, 2, "f32", True, stream, torch)
        out["plain_1024cube_graph"] = {
            "ms_per_step": dt * 100, "value": x.numel() * 10 / dt, "unit": "voxels/s",
            "batch_mode": "graph"}
        say(f"1024^3 f32, one-cube graph: {dt * 100:.1f} ms/step")
        # the same run with the sampled-Gaussian spatial kernel (variant G1)
        wlg = dataclasses.replace(wl, name=wl.name + "_gauss", kernels=[
            (f, w, "gauss") if f > 0 else (f, w) for f, w in wl.kernels])
        dt, noise, s0, stats = time_runs(h, wlg, [x], [m], 10, 2, "f32", False, stream, torch)
        out["plain_1024cube_gauss"] = {
            "ms_per_step": dt * 100, "value": x.numel() * 10 / dt, "unit": "voxels/s",
            "kernels": wlg.kernels, "kernel_gbs": family_gbs(stats),
            "family_ms": {s["name"]: s["total_ms"] / s["launches"] for s in stats},
            "noise": [float(v) for v in noise]}
        say(f"1024^3 f32, sampled Gaussian: {dt * 100:.1f} ms/step")
        # replacement off: one pair at a time, and with the pairs that share a
        # spatial kernel fused into shared passes; RMS noise over all voxels,
        # and the workload's own MAD over the negative voxels
        for nm, rg, name in (("std", "all", "plain_1024cube_repl_off_std"),
                             (wl.noise_mode, wl.flux_range, "plain_1024cube_repl_off")):
            extras_repl_off(h, x, m, wl, nm, rg, name, stream, torch, out)
        h.run(x, wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range, wl.replacement,
              mask=m, stream=stream)
        y = torch.empty_like(x)
        h.normalise(x, 31, 31, 16, 16, "mad", "negative", out=y, grid=False)
        h.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            h.normalise(x, 31, 31, 16, 16, "mad", "negative", out=y, grid=False)
        torch.cuda.synchronize()
        tn = (time.perf_counter() - t0) / 5
        h.profile(False)
        st = h.profile_read()
        out["noise_norm_1024cube"] = {
            "window": [31, 31], "grid": [16, 16], "noise": "mad", "flux_range": "negative",
            "ms": tn * 1e3, "value": x.numel() / tn, "unit": "voxels/s",
            "family_ms": {s["name"]: s["total_ms"] / s["launches"] for s in st},
            "roofline": roofline(st, wl.name, use_traffic=False)}
        say(f"noise normalisation: {tn * 1e3:.1f} ms")
        del y
        lab = torch.empty(x.shape, dtype=torch.int32, device="cuda")
        _, n_src, _ = h.link(m, 2, 2, 8, 5, labels=lab, boxes=False)
        h.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            h.link(m, 2, 2, 8, 5, labels=lab, boxes=False)
        torch.cuda.synchronize()
        tl = (time.perf_counter() - t0) / 5
        h.profile(False)
        st = h.profile_read()
        out["linker_1024cube"] = {
            "radius": [2, 2], "min_size": [8, 5], "ms": tl * 1e3, "value": x.numel() / tl,
            "unit": "voxels/s", "sources": n_src,
            "family_ms": {s["name"]: s["total_ms"] / s["launches"] for s in st}}
        say(f"linker: {tl * 1e3:.1f} ms, {n_src} sources")
        # parameterisation and reliability of the linker's detections
        rec = torch.empty(max(n_src, 1) * sc.SOURCE_DTYPE.itemsize, dtype=torch.uint8,
                          device="cuda")
        _, n_kept = h.parameterise(x, lab, n_src, sigma_rms=s0, out=rec)
        h.profile(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            h.parameterise(x, lab, n_src, sigma_rms=s0, out=rec)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - t0) / 5
        h.profile(False)
        st = h.profile_read()
        out["parameterise_1024cube"] = {
            "sources": n_src, "kept": n_kept, "scale": 0.4, "rel_threshold": 0.9,
            "snr_threshold": 2.8, "ms": tp * 1e3, "value": x.numel() / tp,
            "unit": "voxels/s",
            "family_ms": {s["name"]: s["total_ms"] / s["launches"] for s in st},
            "kernel_gbs": family_gbs(st),
            "density_pairs_per_s": {s["name"]: s["voxels"] / (s["total_ms"] * 1e-3)
                                    for s in st if s["name"] == "reliability"
                                    and s["total_ms"] > 0}}
        say(f"parameterisation: {tp * 1e3:.1f} ms, {n_kept} of {n_src} kept")
        del lab, rec
    finally:
        h.close()
    del x, m
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="large_2048x2048x4096")
    ap.add_argument("--cpu-planes", type=int, default=0,
                    help="planes of the oracle's sample (0: sized to the workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"],
                    help="cube storage inside the run (16-bit: noise-scaled copy)")
    ap.add_argument("--batch-mode", default="auto", choices=["auto", "graph", "loop"],
                    help="graph: one sofia_sc_run_batch graph launch per step (all "
                         "cubes); loop: one sofia_sc_run call per cube; auto: graph for "
                         "many-cube workloads, loop otherwise")
    ap.add_argument("--tune", action="store_true",
                    help="autotune the launch shapes on the workload's first cube first")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one plain device copy of the cube (4 B/voxel "
                         "read + write), the calibration kernel for HBM counters")
    ap.add_argument("--cpu-worker", nargs=2, metavar=("WORKLOAD", "PLANES"),
                    help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_worker:
        print(json.dumps(cpu_sample(args.cpu_worker[0], int(args.cpu_worker[1]))), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2106_15789_amd as sc

    wl = synth.workload(args.workload)
    spec = wl.cubes[0]
    batch = len(wl.cubes) > 1
    say(f"generating {args.workload}: {len(wl.cubes)} cube(s), "
        f"{sum(c.n_vox for c in wl.cubes)} voxels")
    xs = []
    for i, c in enumerate(wl.cubes):
        xs.append(upload(c, torch, synth))
        if batch and (i + 1) % 16 == 0:
            say(f"{i + 1} cubes generated")
    masks = [torch.empty(x.shape, dtype=torch.uint8, device=x.device) for x in xs]
    torch.cuda.synchronize()
    h = sc.SofiaSC(0)
    stream = torch.cuda.current_stream()
    graph = args.batch_mode == "graph" or (batch and args.batch_mode == "auto")
    tuned = None
    if args.tune:
        tuned = h.tune_run(xs[0], wl.kernels, wl.threshold, wl.noise_mode, wl.flux_range,
                           wl.replacement, mask=masks[0], stream=stream, storage=args.storage)
        say(f"tuned shapes: {tuned}")
    if args.copy_probe:
        probe = torch.empty_like(xs[0])
        probe.copy_(xs[0])
        torch.cuda.synchronize()
        del probe
    dt, noise, sigma0, stats = time_runs(h, wl, xs, masks, args.steps, args.warmup,
                                         args.storage, graph, stream, torch)
    say(f"timed steps done: {dt * 1e3 / args.steps:.1f} ms/step")

    n_vox = sum(c.n_vox for c in wl.cubes)
    gpu_ms = sum(s["total_ms"] for s in stats)
    alg_bytes_step = sum(s["bytes"] for s in stats) / args.steps
    result = {
        "metric": METRIC,
        "value": n_vox * args.steps / dt,
        "unit": "voxels/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic (seeded Philox noise + Gaussian mock galaxies)",
        "config": {
            "workload": args.workload, "n_cubes": len(wl.cubes),
            "nx": spec.nx, "ny": spec.ny, "nz": spec.nz,
            "kernels": [list(k) for k in wl.kernels], "noise": wl.noise_mode,
            "flux_range": wl.flux_range, "threshold": wl.threshold,
            "replacement": wl.replacement, "storage": args.storage,
            "batch_mode": "graph" if graph else "loop", "nan_border": spec.nan_border,
            "n_gal": spec.n_gal, "shapes": tuned or h.shapes(),
        },
        "roofline": roofline(stats, args.workload, use_traffic=args.storage == "f32"),
        "whole_step_hbm_frac": alg_bytes_step / (dt / args.steps) / 1e9 / HBM_PEAK_GBS,
        "alg_bytes_per_step": alg_bytes_step,
        "kernel_time_share": {s["name"]: round(s["total_ms"] / gpu_ms, 4) for s in stats},
        "kernel_gbs": family_gbs(stats),
        "noise": [float(v) for v in noise],
        "sigma0": float(sigma0),
        "mask_voxels": sum(count_set(m, torch) for m in masks),
        "kernel_src_sha": kernel_source_sha(),
    }
    h.close()
    del masks
    torch.cuda.empty_cache()
    if not args.no_extras:
        big = xs[0] if (not batch and spec.n_vox >= (1 << 33)) else None
        result["extras"] = extras(sc, torch, synth, stream, big, wl if big is not None else None)
    del xs
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        say("cpu baseline")
        # about 10 s of oracle work on all threads and on one thread
        per_plane = spec.nx * spec.ny * len(wl.kernels)
        planes = args.cpu_planes or max(2, -(-32 * (1 << 22) * 20 // per_plane))
        planes_1t = max(1, planes // 16)
        result["cpu_baseline"] = cpu_baseline(args.workload, spec, len(wl.kernels),
                                              min(planes, spec.nz), min(planes_1t, spec.nz))
    else:
        result["cpu_baseline"] = None
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
