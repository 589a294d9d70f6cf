#!/usr/bin/env python3
"""Benchmark of the MBIR hot path on one MI355X.

Default workload (the 3-D volume): 2048 spectral pixels x 256 x 256 A-scans
with a 2-D lateral transform, image 2048 x 256 x 256 complex64 (1 GiB), 5000
seeded point scatterers in a smooth random background, every pixel observed,
1% Gaussian noise, 3-level 3-D Haar l1 with lambda = 0.01 lambda_max,
Kaiser-Bessel J = 6, sigma = 2.

A step is one FISTA iteration: Phi, Phi^H and the Haar prox.  The timed
region is one oct_mbir_solve of --steps iterations with every input resident
in device memory.  Per-stage kernel durations come from HIP events on the
stream the library launches on (torch's current stream); the slowest
single-kernel stage gives the roofline entry.  The full-size B-scan
(2048 x 1000, 50% random mask, TV) is timed too, as an extra key.  The CPU
baseline times the FP64 oracle on a bounded sample of the volume workload on
the host, on one core and on all of them.

Prints one JSON line.
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

METRIC = "Φ+Φᴴ applications/s & HBM GB/s; MBIR iters/s; serving p50/p99 latency"
HBM_PEAK_GBPS = 8000.0
WORKLOAD = "volume_2048x256x256_haar"
BSCAN = "bscan_2048x1000_tv"
SMALL = "bscan_512x64_l1"


def stage_bytes(g, masked: bool, penalty: str) -> dict:
    """Algorithmic HBM bytes of each stage of one FISTA iteration: every pass
    reads its inputs and writes its outputs once.  A volume's 2-D lateral
    transform takes two passes (a 256 x 256 plane does not fit on chip): the
    second axis adds a read and a write of the image (or spectrum) per
    transform.  With every pixel observed (no mask) the solve has no
    residual seam and one column stage: a kernel per column pair that reads
    X1 and the lateral spectrum of y (formed once per solve), keeps the
    residual spectrum on chip and writes the adjoint columns (every unmasked
    workload here fits it)."""
    N = g.batch * g.n_y * g.n_x * g.n_depth
    M = g.batch * g.n_y * g.n_x * g.n_k
    mbits = M / 8.0 if masked else 0.0
    vol = g.lateral_dims == 2
    prox = {"tv": 48.0, "haar": 16.0, "l1": 16.0}[penalty] * N   # v (+ dual) in; z (+ dual) out
    st = {"lat_fwd": 32.0 * N + (16.0 * N if vol else 0.0)}    # z, z_prev in; X1 and x out (+ y pass)
    if masked:
        st["nufft_fwd"] = 8.0 * N + 8.0 * M                     # X1 in; W out
        st["normal"] = 20.0 * M + mbits + (32.0 * M if vol else 0.0)   # W, y, mask in; R out (+ two y passes)
        st["nufft_adj"] = 8.0 * M + 8.0 * N                     # R in; X1 out
    else:
        st["nufft_normal"] = 16.0 * N + 8.0 * M                 # X1, F_lat y in; X1 out (R stays on chip)
    st["lat_update"] = 24.0 * N + (16.0 * N if vol else 0.0)    # X1, x in; v out (+ y pass)
    st["prox"] = prox
    return st


# FP32 vector peak without packed FP32: 256 CUs x 4 SIMDs x 16 lanes x 2 flop
# (FMA) x 2.4 GHz.  The published 157.3 TFLOP/s counts packed FP32, which the
# build disables.
FP32_PEAK_TFLOPS = 256 * 4 * 16 * 2 * 2.4e9 / 1e12


def grad_bytes(g, masked: bool) -> float:
    """Phi + Phi^H (oct_grad): x in, lateral FFT, NUFFT, residual seam,
    adjoint NUFFT, inverse lateral FFT, g out.  A volume's 2-D lateral
    transform takes two passes (a plane does not fit on chip), which adds a
    read and a write of the image twice on each side and of the spectrum
    twice in the seam."""
    N = g.batch * g.n_y * g.n_x * g.n_depth
    M = g.batch * g.n_y * g.n_x * g.n_k
    mbits = M / 8.0 if masked else 0.0
    if g.lateral_dims == 2:
        return 80.0 * N + 68.0 * M + mbits
    return 48.0 * N + 36.0 * M + mbits


def phi_sizes_bench() -> dict:
    """Phi + Phi^H (oct_grad) at the batch (32 x 1024 x 512) and volume
    (2048 x 256 x 256) sizes, random x and y resident on the device, and a
    plain 1 GiB device copy for the attainable bandwidth."""
    import torch
    import paper_2108_01438_amd as P
    import synth
    torch.cuda.set_device(0)
    res = {"metric": "Phi+Phi^H applications/s and algorithmic HBM GB/s", "peak_GBps": HBM_PEAK_GBPS}
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(10):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    res["copy_GBps"] = round(2 * n * 4 / (a.elapsed_time(b) / 10 * 1e-3) / 1e9, 1)
    del src, dst
    for name, reps in (("batch32_1024x512_grad", 20), ("volume_2048x256x256_haar", 5)):
        g = P.Geometry.from_dict(synth.preset(name)["geom"])
        plan = P.Plan(g)
        gen = torch.Generator(device="cuda").manual_seed(5)
        x = torch.randn(g.img_shape, dtype=torch.complex64, device="cuda", generator=gen)
        y = torch.randn(g.meas_shape, dtype=torch.float32, device="cuda", generator=gen)
        gb = torch.empty_like(x)
        rb = torch.empty((), dtype=torch.float64, device="cuda")
        for _ in range(2):
            plan.grad(x, y, gb, rb)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            plan.grad(x, y, gb, rb)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        byt = grad_bytes(g, False)
        res[name] = {"ms": round(ms, 4), "applications_per_s": round(1000.0 / ms, 2),
                     "algorithmic_GB": round(byt / 1e9, 3), "GBps": round(byt / (ms * 1e-3) / 1e9, 1),
                     "frac_of_peak": round(byt / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)}
        print(f"[bench] {name}: {ms:.3f} ms", file=sys.stderr, flush=True)
        plan.close()
        del x, y, gb
    return res


# kernels of the single-kernel stages (a volume's lateral stages take two or
# three launches of the lateral kernel), by the name rocprofv3 reports
STAGE_KERNEL = {
    "nufft_fwd": "nufft_fwd_pair_kernel<6, false, false>",
    "nufft_adj": "nufft_adj_pair_kernel<6, true>",
    "nufft_normal": "nufft_normal_pair_kernel<6, false, 4>",
    "prox": {"tv": "tv2d_tile_kernel<false>", "haar": "haar_kernel<3, 3", "l1": "prox_l1_kernel"},
}
BSCAN_STAGE_KERNEL = {
    "lat_fwd": "lat_kernel<0, false, ",
    "normal": "lat_kernel<3, false, ",
    "lat_update": "lat_kernel<4, false, ",
}
STAGE_SOURCE = {
    "lat_fwd": "oct_lateral.hip", "normal": "oct_lateral.hip", "lat_update": "oct_lateral.hip",
    "nufft_fwd": "oct_nufft.hip", "nufft_adj": "oct_nufft.hip", "nufft_normal": "oct_nufft.hip",
    "prox": "oct_prox.hip",
}


def stage_kernel(stage: str, penalty: str, volume: bool):
    """Kernel (name prefix) of a stage that is one launch, else None."""
    k = STAGE_KERNEL.get(stage)
    if isinstance(k, dict):
        k = k.get(penalty)
    if k is None and not volume:
        k = BSCAN_STAGE_KERNEL.get(stage)
    return k


def source_digest(stage: str) -> str:
    h = hashlib.sha256()
    for f in (STAGE_SOURCE[stage], "oct_fft.h", "oct_common.h"):
        with open(os.path.join(ROOT, "paper_2108_01438_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(workload: str, stage: str):
    """HBM bytes per launch of a stage's kernel from the committed rocprofv3
    counter summary, if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    s = rec.get("stages", {}).get(stage)
    if not s or s.get("source_digest") != source_digest(stage):
        return None
    return float(s["hbm_bytes_per_launch"])


def _counter_rows(d: str):
    """(kernel name, counter name, value, grid size) of every dispatch in the
    rocprofv3 counter-collection CSVs under directory d."""
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                rows.append((r["Kernel_Name"], r["Counter_Name"], float(r["Counter_Value"]),
                             int(r.get("Grid_Size", 0) or 0)))
    return rows


def _kname(k: str) -> str:
    """Kernel name without rocprofv3's 'void ' and anonymous-namespace prefixes."""
    if k.startswith("void "):
        k = k[5:]
    return k.replace("(anonymous namespace)::", "")


def _per_launch(rows, counter: str, prefix: str) -> float:
    """Mean value of a counter per dispatch of the kernels whose name starts
    with prefix."""
    vals = [v for k, c, v, _ in rows if c == counter and _kname(k).startswith(prefix)]
    if not vals:
        raise SystemExit(f"no {counter} rows for {prefix!r}")
    return sum(vals) / len(vals)


def traffic_json(workload: str, penalty: str, volume: bool, fetch_dir: str, write_dir: str,
                 copy_fetch_dir: str, copy_write_dir: str, copy_bytes: int) -> dict:
    """Scaled HBM bytes per launch of the single-kernel stages from two
    rocprofv3 --pmc runs of the bench (FETCH_SIZE, WRITE_SIZE, in KiB per
    dispatch) and the same two counters on a plain device copy of copy_bytes
    each way (the calibration: true bytes / counted bytes)."""
    cf = _per_launch(_counter_rows(copy_fetch_dir), "FETCH_SIZE", "__amd_rocclr_copyBuffer") * 1024.0
    cw = _per_launch(_counter_rows(copy_write_dir), "WRITE_SIZE", "__amd_rocclr_copyBuffer") * 1024.0
    fs, ws = copy_bytes / cf, copy_bytes / cw
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    out = {"workload": workload, "fetch_scale": fs, "write_scale": ws, "copy_bytes_each_way": copy_bytes,
           "stages": {}}
    # the stages of the workload's iteration: the B-scan is masked, the volume fully observed
    stages = (("lat_fwd", "nufft_normal", "lat_update", "prox") if volume else
              ("lat_fwd", "nufft_fwd", "normal", "nufft_adj", "lat_update", "prox"))
    for st in stages:
        k = stage_kernel(st, penalty, volume)
        if k is None:
            continue
        f = _per_launch(fr, "FETCH_SIZE", k) * 1024.0 * fs
        w = _per_launch(wr, "WRITE_SIZE", k) * 1024.0 * ws
        out["stages"][st] = {"kernel": k, "hbm_bytes_per_launch": f + w, "fetch_bytes": f, "write_bytes": w,
                             "source_digest": source_digest(st)}
    return out


def make_workload(P, synth, torch):
    """The full-size B-scan: specimen, mask and unit noise (seeded)."""
    import numpy as np
    pr = synth.preset(BSCAN)
    geom = P.Geometry.from_dict(pr["geom"])
    rng = np.random.default_rng(1)
    x_true = synth.scatterers(rng, geom.img_shape, pr["scatterers"])
    x_true[0, 0] += synth.layers(rng, geom.n_depth, geom.n_x, pr["layers"])
    mask = synth.mask_random_exact(rng, (1, geom.n_x), geom.n_k, geom.n_k // 2)
    noise = synth.standard_normal(rng, geom.meas_shape)
    return geom, pr, x_true, mask, noise


def volume_specimen(synth, shape, pr):
    """The volume's specimen: scatterers in a smooth background whose RMS is 5%
    of the mean scatterer amplitude (seed 2)."""
    import numpy as np
    rng = np.random.default_rng(2)
    x = synth.scatterers(rng, shape, pr["scatterers"])
    x[0] += synth.smooth_field_coarse(rng, shape[1:], 16, pr["field"] * 0.75)
    return x.astype(np.complex64)


def cpu_baseline(slab_y: int = 32) -> dict:
    """The FP64 oracle, as it stands, on one FISTA-Haar iteration of a slab of
    the volume workload (all 2048 depth samples and 256 A-scans along x, slab_y
    of the 256 along y, i.e. 1/8 of the volume), on one thread and on every
    host core; the rate is scaled to the whole volume (time x 256 / slab_y)."""
    import numpy as np
    import oracle as O
    import synth
    pr = synth.preset(WORKLOAD)
    g = O.Geometry(**dict(pr["geom"], n_y=slab_y))
    rng = np.random.default_rng(3)
    x = synth.scatterers(rng, O.img_shape(g), pr["scatterers"] * slab_y // 256)
    y = synth.noisy(O.forward(x, g), synth.standard_normal(rng, O.meas_shape(g)), None, pr["noise"])
    lam = pr["lam"] * O.lambda_max(y, g)
    delta = O.step_size(O.lipschitz(g, None, iters=1))
    scale = pr["geom"]["n_y"] / slab_y
    res = {}
    for nt in (1, os.cpu_count() or 1):
        prev = O.set_workers(nt)
        t0 = time.perf_counter()
        O.fista(y, g, None, O.PEN_HAAR, lam, delta, 1, haar_levels=3)
        res[nt] = time.perf_counter() - t0
        O.set_workers(prev)
    nt = max(res)
    try:
        model = next(l.split(":", 1)[1].strip() for l in open("/proc/cpuinfo") if l.startswith("model name"))
    except (OSError, StopIteration):
        model = "unknown"
    return {"value": 1.0 / (res[nt] * scale), "unit": "MBIR iters/s", "cores": nt, "kind": "oracle",
            "single_core_value": 1.0 / (res[1] * scale),
            "sample": f"one FISTA iteration (Phi, Phi^H, 3-level Haar prox and the objective) of a "
                      f"2048 x 256 x {slab_y} slab of the 2048 x 256 x 256 Haar volume workload "
                      f"(1/{int(scale)} of it; rate scaled by {int(scale)}), NumPy/SciPy FP64: "
                      f"{res[nt]:.1f} s on {nt} threads, {res[1]:.1f} s on one; host: {model}"}


def serving_bench(n_req: int, seed: int = 4, warmup: int = 20, rates=(0.5, 0.8, 1.0), slots: int = 8,
                  budget_gib: int = 200) -> dict:
    """Serving mix (60% B-scans 1024-2048 px x 256-2000 A-scans, 30% volumes
    1024 x 64^2..128^2, 10% 512 x 64 B-scans; random penalty, 50-100
    iterations): `warmup` requests first, then `n_req` requests solved one at
    a time (the sequential rate C), by the continuous-batching server with
    every request queued at once (closed loop), and with Poisson arrivals at
    each rate x C.  Every result of the mix is compared bitwise with its
    sequential solve (SHA-1 of the bytes)."""
    import hashlib
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    from paper_2108_01438_amd.serve import HipExecutor, Request, Server, run_sequential
    rng = np.random.default_rng(seed)
    mix = synth.serving_mix(rng, warmup + n_req)
    reqs, Lcache, plans = [], {}, {}
    t0 = time.perf_counter()
    for i, spec in enumerate(mix):
        r = np.random.default_rng(spec["seed"])
        geo = dict(synth.OPTICS)
        geo.update(spec["geom"])
        g = P.Geometry.from_dict(geo)
        key = tuple(sorted(spec["geom"].items()))
        plan = plans.get(key)
        if plan is None:
            if len(plans) > 16:
                for p_ in plans.values():
                    p_.close()
                plans.clear()
            plan = plans[key] = P.Plan(g)
        x = synth.scatterers(r, g.img_shape, 20).astype(np.complex64)
        y = plan.forward(torch.from_numpy(x).cuda())
        noise = torch.from_numpy(synth.standard_normal(r, g.meas_shape).astype(np.float32)).cuda()
        y = (y + 0.01 * float(y.abs().max().item()) * noise).contiguous()
        lam = spec["lam"] * float(plan.adjoint(y).abs().max().item())
        if key not in Lcache:
            Lcache[key] = plan.lipschitz(50)
        reqs.append(Request(geom=g, y=y.cpu().numpy(), penalty=spec["pen"], lam=lam, iters=spec["iters"],
                            delta=1.0 / (1.05 * Lcache[key])))
        if (i + 1) % 100 == 0:
            print(f"[serving] {i + 1} requests ready ({time.perf_counter() - t0:.0f} s)", file=sys.stderr, flush=True)
    for p_ in plans.values():
        p_.close()
    warm, meas = reqs[:warmup], reqs[warmup:]
    digest = lambda a: hashlib.sha1(np.ascontiguousarray(a).view(np.uint8)).hexdigest()   # noqa: E731
    budget = budget_gib << 30

    ex1 = HipExecutor(slots=1)
    run_sequential(ex1, warm)
    t0 = time.perf_counter()
    alone = []
    for r in meas:
        outs, _ = run_sequential(ex1, [r])
        alone.append(digest(outs[0]))
    t_seq = time.perf_counter() - t0
    ex1.shutdown()
    C = n_req / t_seq
    print(f"[serving] sequential {C:.2f} solves/s", file=sys.stderr, flush=True)

    def serve(arrivals):
        srv = Server(HipExecutor(slots=slots), mem_budget=budget, slots=slots)
        for f in [srv.submit(r) for r in warm]:
            f.result(timeout=600)
        srv.completed.clear()
        t_start = time.perf_counter()
        futs = []
        for r, ta in zip(meas, arrivals):
            dt = t_start + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            futs.append(srv.submit(r))
        outs = [digest(f.result(timeout=900)) for f in futs]
        t_all = time.perf_counter() - t_start
        srv.close()
        st = srv.latency_stats()
        mism = sum(int(a != b) for a, b in zip(alone, outs))
        return {"solves_per_s": round(n_req / t_all, 3), "p50_ms": round(st["p50_s"] * 1e3, 2),
                "p99_ms": round(st["p99_s"] * 1e3, 2), "mean_ms": round(st["mean_s"] * 1e3, 2),
                "alone_vs_mix_mismatches": mism}

    out = {"metric": "serving solves/s with p50/p99 latency (continuous batching vs sequential solves)",
           "warmup_requests": warmup, "requests": n_req, "slots": slots, "mem_budget_GiB": budget_gib,
           "sequential_solves_per_s": round(C, 3), "sequential_mean_ms": round(t_seq / n_req * 1e3, 2)}
    cl = serve([0.0] * n_req)
    out["closed_loop"] = cl
    out["closed_loop_gain"] = round(cl["solves_per_s"] / C, 3)
    print(f"[serving] closed loop {cl}", file=sys.stderr, flush=True)
    for rate in rates:
        arr = np.cumsum(rng.exponential(1.0 / (rate * C), size=n_req))
        res = serve(list(arr))
        res["offered_solves_per_s"] = round(rate * C, 3)
        out[f"poisson_{rate:g}C"] = res
        print(f"[serving] poisson {rate:g} C: {res}", file=sys.stderr, flush=True)
    return out


def table1_bench(search_iters: int = 10, u_range=(-6.0, -0.5), coarse: int = 8) -> dict:
    """Synthetic analogue of Table 1 (Sec. 3.2): NCC (eq. (17)) against the
    fully sampled ISAM image for the direct reconstructions of Figure 1 and, for
    the random / equispaced / partial sub-sampling of Sec. 3.1, the
    interpolated-ISAM baseline and MBIR with TV and with 3-level Haar (the
    substitute for the DT-CWT), each lambda chosen by a golden-section search
    on the NCC, 100 FISTA iterations.  Specimens on the 2048 x 1000 B-scan:
    sparse point scatterers (bead-like) and layered speckle (tissue-like), 1%
    noise; measurements are synthesised with the library's own forward
    operator.  The twelve lambda searches of a specimen run concurrently, one
    plan and stream each; each coarse scan is one batched solve."""
    import concurrent.futures as cf
    import dataclasses
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    from paper_2108_01438_amd.tune import tune_lambda
    import synth
    torch.cuda.set_device(0)
    pr = synth.preset(BSCAN)
    geom = P.Geometry.from_dict(pr["geom"])
    out = {"metric": "NCC vs fully sampled ISAM (eq. (17)); synthetic analogue of Table 1",
           "workload": "B-scan 2048 spectral px x 1000 A-scans, 1% noise, 100 FISTA iterations, "
                       f"lambda = 10^u lambda_max, u in [{u_range[0]}, {u_range[1]}]: {coarse}-point scan, "
                       f"then golden-section search on NCC between the best point's neighbours "
                       f"({search_iters} reductions)",
           "specimens": {}}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for spec in ("beads", "tissue"):
        rng = np.random.default_rng({"beads": 11, "tissue": 12}[spec])
        if spec == "beads":
            x_true = synth.scatterers(rng, geom.img_shape, 500)
        else:
            x_true = np.zeros(geom.img_shape, dtype=np.complex128)
            x_true[0, 0] = synth.layers(rng, geom.n_depth, geom.n_x, 3)
        full = P.Plan(geom)
        xd = torch.from_numpy(x_true.astype(np.complex64)).cuda()
        y_clean = full.forward(xd)
        sigma = pr["noise"] * float(y_clean.abs().max())
        noise = torch.from_numpy(rng.standard_normal(geom.meas_shape).astype(np.float32)).cuda()
        y_full = y_clean + sigma * noise
        ref = full.direct(y_full, "isam")
        row = {"fully_sampled": {k: round(full.ncc(full.direct(y_full, k), ref), 4)
                                 for k in ("axial", "dispersion", "isam")}}
        row["fully_sampled_vs_true"] = {k: round(full.ncc(full.direct(y_full, k), xd), 4)
                                        for k in ("axial", "dispersion", "isam")}
        if spec == "beads":   # kernel times of the direct reconstructions and NCC at this size
            times = {}
            for k in ("axial", "dispersion", "isam", "interp_isam"):
                xo = full.direct(y_full, k)
                torch.cuda.synchronize()
                a.record()
                for _ in range(20):
                    full.direct(y_full, k, x=xo)
                b.record()
                torch.cuda.synchronize()
                times[k] = round(a.elapsed_time(b) / 20, 4)
            t0 = time.perf_counter()
            for _ in range(20):
                full.ncc(ref, ref)
            times["ncc_incl_sync"] = round((time.perf_counter() - t0) / 20 * 1e3, 4)
            out["direct_ms"] = times
        masks = {"random": synth.mask_bernoulli(rng, (1, geom.n_x), geom.n_k, 0.5),
                 "equispaced": synth.mask_equispaced((1, geom.n_x), geom.n_k),
                 "partial": synth.mask_partial((1, geom.n_x), geom.n_k)}
        jobs = []
        for mname, mask in masks.items():
            md = torch.from_numpy(mask.astype(np.float32)[None]).cuda()
            y_m = y_full * md
            pm = P.Plan(geom, mask)
            interp = round(pm.ncc(pm.direct(y_m, "interp_isam"), ref), 4)
            L = pm.lipschitz(50)
            lam_max = float(pm.adjoint(y_m).abs().max())
            row[mname] = {"interp_isam": interp}
            for pen in ("tv", "haar"):
                jobs.append((mname, pen, mask, y_m, 1.0 / (1.05 * L), lam_max))
            pm.close()

        def run(job):
            mname, pen, mask, y_m, delta, lam_max = job
            st = torch.cuda.Stream()
            plan = P.Plan(geom, mask)
            plan_b = P.Plan(dataclasses.replace(geom, batch=coarse), mask)   # the coarse scan as one solve
            with torch.cuda.stream(st):
                r = tune_lambda(plan, y_m, ref, pen, lam_max, delta, iters=100, u_range=u_range,
                                search_iters=search_iters, coarse=coarse, stream=st, batched_plan=plan_b)
            st.synchronize()
            plan.close()
            plan_b.close()
            return mname, pen, r
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=len(jobs)) as ex:
            for mname, pen, r in ex.map(run, jobs):
                row[mname]["mbir_" + pen] = round(r["ncc"], 4)
                row[mname]["lambda_frac_" + pen] = float("%.3g" % (10.0 ** r["u"]))
        row["search_seconds"] = round(time.perf_counter() - t0, 2)
        row["solves"] = len(jobs) * (coarse + search_iters + 3)
        out["specimens"][spec] = row
        full.close()
        print(f"[bench] table1 {spec}: {json.dumps(row)}", file=sys.stderr, flush=True)
    return out


def paper_backward_bench(steps: int = 100, reps: int = 50) -> dict:
    """The paper's backward operator (eq. (10)-(11)) against the exact adjoint on
    the full B-scan: one application each, a FISTA-TV solve of `steps`
    iterations each (each with the step size of its own normal operator), the
    two power-iteration constants and the NCC of each solution with the
    specimen."""
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    torch.cuda.set_device(0)
    geom, pr, x_true, mask, noise = make_workload(P, synth, torch)
    plan = P.Plan(geom, mask)
    mask_d = torch.from_numpy(mask.astype(np.float32)[None]).cuda()
    xt = torch.from_numpy(x_true.astype(np.complex64)).cuda()
    y_clean = plan.forward(xt)
    sigma = pr["noise"] * float(y_clean.abs().max().item())
    y = ((y_clean + sigma * torch.from_numpy(noise.astype(np.float32)).cuda()) * mask_d).contiguous()
    lam = pr["lam"] * float(plan.adjoint(y).abs().max().item())
    xbuf = torch.empty(geom.img_shape, dtype=torch.complex64, device="cuda")

    def timed(fn, n):
        for _ in range(3):
            fn()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(n):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / n

    out = {"workload": "B-scan 2048 spectral px x 1000 A-scans, 50% random mask, TV lambda=0.005 lambda_max, "
                       "10 FGP steps"}
    out["adjoint_ms"] = round(timed(lambda: plan.adjoint(y, xbuf), reps), 5)
    out["adjoint_paper_ms"] = round(timed(lambda: plan.adjoint_paper(y, xbuf), reps), 5)
    for name, pb in (("exact", False), ("paper", True)):
        L = plan.lipschitz(50, seed=0, paper_backward=pb)
        delta = 1.0 / (1.05 * L)
        plan.mbir_solve(y, "tv", lam, 5, delta=delta, tv_inner=10, paper_backward=pb)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        z, info = plan.mbir_solve(y, "tv", lam, steps, delta=delta, tv_inner=10, paper_backward=pb,
                                  objective=True)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"L": round(L, 4), "ms_per_iteration": round(e0.elapsed_time(e1) / steps, 5),
                     "objective_first": round(float(info["objective"][0]), 4),
                     "objective_last": round(float(info["objective"][-1]), 4),
                     "ncc_vs_specimen": round(plan.ncc(z, xt), 5)}
        out[name + "_z"] = z
    ze, zp = out.pop("exact_z"), out.pop("paper_z")
    out["rel_diff_solutions"] = round(float((zp - ze).abs().pow(2).sum().sqrt() / ze.abs().pow(2).sum().sqrt()), 5)
    return out


def penalties_bench(steps: int = 100, reps: int = 20) -> dict:
    """The four regularisers on the full B-scan workload (2048 x 1000, 50%
    random mask): per penalty the prox alone (HIP events, `reps` calls), one
    FISTA solve of `steps` iterations, and the NCC of its result with the
    specimen.  lambda = 0.01 lambda_max (l1, Haar, DT-CWT), 0.005 (TV);
    3 wavelet levels, 10 FGP steps.  Then each step alone on the
    2048 x 256 x 256 volume."""
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    torch.cuda.set_device(0)
    geom, pr, x_true, mask, noise = make_workload(P, synth, torch)
    plan = P.Plan(geom, mask)
    mask_d = torch.from_numpy(mask.astype(np.float32)[None]).cuda()
    xt = torch.from_numpy(x_true.astype(np.complex64)).cuda()
    yc = plan.forward(xt)
    sigma = pr["noise"] * float(yc.abs().max().item())
    y = ((yc + sigma * torch.from_numpy(noise.astype(np.float32)).cuda()) * mask_d).contiguous()
    lmax = float(plan.adjoint(y).abs().max().item())
    delta = 1.0 / (1.05 * plan.lipschitz(50, seed=0))
    v = plan.adjoint(y)
    zbuf = torch.empty_like(v)
    out = {"workload": "B-scan 2048 spectral px x 1000 A-scans, 50% random mask; 3 wavelet levels, 10 FGP steps"}
    for pen, frac in (("l1", 0.01), ("tv", 0.005), ("haar", 0.01), ("dtcwt", 0.01)):
        lam = frac * lmax
        for _ in range(3):
            plan.prox(pen, lam, delta, v, zbuf, haar_levels=3)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            plan.prox(pen, lam, delta, v, zbuf, haar_levels=3)
        b.record()
        torch.cuda.synchronize()
        prox_ms = a.elapsed_time(b) / reps
        plan.mbir_solve(y, pen, lam, 5, delta=delta, tv_inner=10, haar_levels=3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        z, _ = plan.mbir_solve(y, pen, lam, steps, delta=delta, tv_inner=10, haar_levels=3)
        e1.record()
        torch.cuda.synchronize()
        out[pen] = {"lambda_frac": frac, "prox_ms": round(prox_ms, 5),
                    "ms_per_iteration": round(e0.elapsed_time(e1) / steps, 5),
                    "ncc_vs_specimen": round(plan.ncc(z, xt), 5)}
    # the step alone on the 2048 x 256 x 256 volume (random image, tau = 0.01 of its peak)
    del plan, v, zbuf, y, yc, xt
    torch.cuda.empty_cache()
    gv = P.Geometry(n_depth=2048, n_x=256, n_y=256, lateral_dims=2, n_k=2048)
    pv = P.Plan(gv)
    gen = torch.Generator(device="cuda").manual_seed(5)
    vv = torch.randn(gv.img_shape, dtype=torch.complex64, device="cuda", generator=gen)
    zv = torch.empty_like(vv)
    tau = 0.01 * float(vv.abs().max().item())
    vol = {}
    for pen in ("l1", "tv", "haar", "dtcwt"):
        for _ in range(2):
            pv.prox(pen, tau, 1.0, vv, zv, haar_levels=3)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(5):
            pv.prox(pen, tau, 1.0, vv, zv, haar_levels=3)
        b.record()
        torch.cuda.synchronize()
        vol[pen] = round(a.elapsed_time(b) / 5, 4)
    out["volume_2048x256x256_prox_ms"] = vol
    return out


def literal_bench(steps: int = 100, reps: int = 50) -> dict:
    """The paper's literal K, Q, D chain (model 1) against the direct model on a
    B-scan in the paper's sizing (M_k = 2 N_z: 1024 depth samples, 1000 A-scans,
    2048 spectral pixels, 50% random mask, TV): Phi + Phi^H time, a FISTA-TV
    solve of `steps` iterations with each model's own step, the relative
    difference of the two models' measurements of the same specimen, and the NCC
    of each solution with the specimen (data synthesised with the direct model)."""
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    torch.cuda.set_device(0)
    rng = np.random.default_rng(1)
    gd = P.Geometry(n_depth=1024, n_x=1000, n_k=2048)
    gl = P.Geometry(n_depth=1024, n_x=1000, n_k=2048, model=1)
    x_true = synth.scatterers(rng, gd.img_shape, 500)
    x_true[0, 0] += synth.layers(rng, gd.n_depth, gd.n_x, 3)
    mask = synth.mask_random_exact(rng, (1, gd.n_x), gd.n_k, gd.n_k // 2)
    noise = synth.standard_normal(rng, gd.meas_shape)
    xt = torch.from_numpy(x_true.astype(np.complex64)).cuda()
    plans = {"direct": P.Plan(gd, mask), "literal": P.Plan(gl, mask)}
    yd = plans["direct"].forward(xt)
    yl = plans["literal"].forward(xt)
    mask_d = torch.from_numpy(mask.astype(np.float32)[None]).cuda()
    sigma = 0.01 * float(yd.abs().max().item())
    y = ((yd + sigma * torch.from_numpy(noise.astype(np.float32)).cuda()) * mask_d).contiguous()
    out = {"workload": "B-scan 1024 depth x 1000 A-scans, 2048 spectral px (M_k = 2 N_z), 50% random mask, "
                       "TV lambda=0.005 lambda_max, 10 FGP steps; data from the direct model",
           "model_gap_rel": round(float((yl - yd).norm() / yd.norm()), 5)}
    lam = 0.005 * float(plans["direct"].adjoint(y).abs().max().item())
    gbuf = torch.empty(gd.img_shape, dtype=torch.complex64, device="cuda")
    rbuf = torch.empty((), dtype=torch.float64, device="cuda")
    for name, plan in plans.items():
        for _ in range(3):
            plan.grad(xt, y, gbuf, rbuf)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            plan.grad(xt, y, gbuf, rbuf)
        b.record()
        torch.cuda.synchronize()
        L = plan.lipschitz(50, seed=0)
        delta = 1.0 / (1.05 * L)
        plan.mbir_solve(y, "tv", lam, 5, delta=delta, tv_inner=10)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        z, info = plan.mbir_solve(y, "tv", lam, steps, delta=delta, tv_inner=10, objective=True)
        e1.record()
        torch.cuda.synchronize()
        out[name] = {"phi_phih_ms": round(a.elapsed_time(b) / reps, 5), "L": round(L, 3),
                     "ms_per_iteration": round(e0.elapsed_time(e1) / steps, 5),
                     "objective_last": round(float(info["objective"][-1]), 3),
                     "ncc_vs_specimen": round(plan.ncc(z, xt), 5)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--stage-reps", type=int, default=10)
    ap.add_argument("--workload", choices=("volume", "bscan"), default="volume",
                    help="headline workload: the 2048 x 256 x 256 Haar volume (default) or the 2048 x 1000 TV B-scan")
    ap.add_argument("--no-bscan", action="store_true", help="skip the B-scan summaries (full-size TV, small l1) of the volume line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--traffic-json", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR", "COPY_WRITE_DIR"),
                    help="only write profiles/traffic_<workload>.json from rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE "
                         "runs of this bench and of --copy-probe-mib 512")
    ap.add_argument("--serving", type=int, default=0,
                    help="only run the serving benchmark with this many measured requests")
    ap.add_argument("--serving-warmup", type=int, default=20, help="warm-up requests of the serving benchmark")
    ap.add_argument("--serving-slots", type=int, default=8, help="concurrent solves of the serving benchmark")
    ap.add_argument("--table1", action="store_true",
                    help="only run the synthetic analogue of Table 1 (NCC of direct, interpolated and MBIR images)")
    ap.add_argument("--small", action="store_true",
                    help="only the small B-scan's solve latency (launched and graph-replayed)")
    ap.add_argument("--phi-sizes", action="store_true",
                    help="only time Phi + Phi^H at the batch and volume sizes")
    ap.add_argument("--bound", type=float, default=0.0,
                    help="modulus bound of the constraint set C (eq. (16)) as a fraction of max|x_true|; 0 = none")
    ap.add_argument("--penalties", action="store_true",
                    help="only compare the four regularisers (prox time, FISTA time, NCC) on the B-scan workload")
    ap.add_argument("--literal", action="store_true",
                    help="only compare the paper's literal K, Q, D chain with the direct model (M_k = 2 N_z)")
    ap.add_argument("--paper-backward", action="store_true",
                    help="only compare the paper's backward operator with the exact adjoint (cost and solutions)")
    ap.add_argument("--profile-stages", action="store_true",
                    help="only run every stage of the headline workload's FISTA iteration --stage-reps times on "
                         "random data (for counter profiles)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB 5 times (counter calibration)")
    args = ap.parse_args()
    if args.traffic_json:
        wl, pen, vol = (WORKLOAD, "haar", True) if args.workload == "volume" else (BSCAN, "tv", False)
        rec = traffic_json(wl, pen, vol, *args.traffic_json, copy_bytes=512 << 20)
        path = os.path.join(ROOT, "profiles", f"traffic_{wl}.json")
        with open(path, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps(rec))
        return 0
    if args.profile_stages:
        print(json.dumps(profile_stages(args)), flush=True)
        return 0
    if args.copy_probe_mib > 0:
        import torch
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 4, "launches": 5}))
        return 0
    if args.table1:
        print(json.dumps(table1_bench()), flush=True)
        return 0
    if args.small:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(small_line()), flush=True)
        return 0
    if args.phi_sizes:
        print(json.dumps(phi_sizes_bench()), flush=True)
        return 0
    if args.penalties:
        print(json.dumps(penalties_bench(args.steps)), flush=True)
        return 0
    if args.literal:
        print(json.dumps(literal_bench(args.steps)), flush=True)
        return 0
    if args.paper_backward:
        print(json.dumps(paper_backward_bench(args.steps)), flush=True)
        return 0
    if args.serving > 0:
        import torch
        torch.cuda.set_device(0)
        print(json.dumps(serving_bench(args.serving, warmup=args.serving_warmup, slots=args.serving_slots)),
              flush=True)
        return 0
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        return 2

    import torch
    torch.cuda.set_device(0)
    if args.workload == "bscan":
        line = bscan_line(args)
    else:
        line = volume_line(args)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle) ...", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline()
    print(json.dumps(line), flush=True)
    return 0


def profile_stages(args) -> dict:
    """Every stage of one FISTA iteration of the headline workload, --stage-reps
    times each, on random data (the launch shapes of the timed solve)."""
    import torch
    import paper_2108_01438_amd as P
    import synth
    torch.cuda.set_device(0)
    name, pen = (WORKLOAD, "haar") if args.workload == "volume" else (BSCAN, "tv")
    geom = P.Geometry.from_dict(synth.preset(name)["geom"])
    mask = None
    if args.workload != "volume":   # the B-scan's solve sees half of every A-scan (seeded, as its bench)
        import numpy as np
        mask = synth.mask_random_exact(np.random.default_rng(1), (1, geom.n_x), geom.n_k, geom.n_k // 2)
    plan = P.Plan(geom, mask)
    gen = torch.Generator(device="cuda").manual_seed(5)
    y = torch.randn(geom.meas_shape, dtype=torch.float32, device="cuda", generator=gen)
    sb = stage_bytes(geom, mask is not None, pen)
    st = time_stages(plan, pen, y, sb, args.stage_reps)
    plan.close()
    return {"workload": name, "reps": args.stage_reps,
            "stages_ms": {k: round(v["ms"], 5) for k, v in st.items()}}


def time_stages(plan, penalty: str, y, sb: dict, reps: int) -> dict:
    """HIP-event duration of each stage of a FISTA iteration on the plan's own
    buffers (oct_run_stage), on torch's current stream (the launch stream)."""
    import torch
    stages = {}
    for st in sb:   # the stages of the solve's iteration
        for _ in range(3):
            plan.run_stage(st, penalty, y)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        for _ in range(reps):
            plan.run_stage(st, penalty, y)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / reps
        stages[st] = {"ms": ms, "bytes": sb[st], "GBps": sb[st] / (ms * 1e-3) / 1e9}
    return stages


def time_solve(plan, y, penalty: str, lam: float, delta: float, steps: int, warmup: int, **kw):
    """One solve of `steps` iterations after a warm-up solve; ms per
    iteration (the larger of the HIP-event and the host wall-clock time)."""
    import torch
    plan.mbir_solve(y, penalty, lam, max(1, warmup), delta=delta, **kw)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    z, _ = plan.mbir_solve(y, penalty, lam, steps, delta=delta, **kw)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return z, max(e0.elapsed_time(e1), wall * 1e3) / steps


def time_grad(plan, x, y, reps: int) -> float:
    import torch
    gbuf = torch.empty_like(x)
    rbuf = torch.empty((), dtype=torch.float64, device="cuda")
    for _ in range(3):
        plan.grad(x, y, gbuf, rbuf)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        plan.grad(x, y, gbuf, rbuf)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def roofline(workload: str, stages: dict, penalty: str, volume: bool, g, n_inner: int = 10) -> dict:
    """Roofline entry of the slowest single-kernel stage: algorithmic bytes (or,
    for the TV tile kernel, which is bound by FP32 vector arithmetic, flops)
    per launch over its HIP-event launch duration."""
    cand = [st for st in stages if stage_kernel(st, penalty, volume)]
    dom = max(cand, key=lambda k: stages[k]["ms"])
    ms = stages[dom]["ms"]
    base = {"kernel": stage_kernel(dom, penalty, volume), "stage": dom, "traffic": traffic_for(workload, dom),
            "algorithmic_bytes_per_launch": stages[dom]["bytes"], "ms_per_launch": round(ms, 5)}
    if dom == "prox" and penalty == "tv":
        N = g.batch * g.n_y * g.n_x * g.n_depth
        fl = float(N) * (n_inner * TV_FLOPS_PER_STEP + TV_FLOPS_FINAL)
        ach = fl / (ms * 1e-3) / 1e12
        return dict({"bound": "alu", "achieved": round(ach, 2), "peak": round(FP32_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(ach / FP32_PEAK_TFLOPS, 4),
                     "algorithmic_flops_per_launch": fl, "hbm_GBps": round(stages[dom]["GBps"], 1)}, **base)
    ach = stages[dom]["GBps"]
    return dict({"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                 "frac": round(ach / HBM_PEAK_GBPS, 4)}, **base)


# Algorithmic flops of the TV prox per pixel (FMA = 2): per FGP step the
# divergence of r (6), d = v + tau div r (4), grad d (4), q = r + s grad d (8),
# |q|^2 (7), projection (2 + 4), momentum r = p + mom (p - p_old) (12); once at
# the end z = v + tau div p (10).  The TV value (12 more) is computed only when
# the objective is asked for, which the timed solve does not do.
TV_FLOPS_PER_STEP = 47
TV_FLOPS_FINAL = 10


def volume_line(args) -> dict:
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    pr = synth.preset(WORKLOAD)
    geom = P.Geometry.from_dict(pr["geom"])
    x_true = volume_specimen(synth, geom.img_shape, pr)
    plan = P.Plan(geom)
    xt = torch.from_numpy(x_true).cuda()
    del x_true
    y = plan.forward(xt)
    gen = torch.Generator(device="cuda").manual_seed(2)
    sigma = pr["noise"] * float(y.abs().max().item())
    y = (y + sigma * torch.randn(y.shape, dtype=torch.float32, device="cuda", generator=gen)).contiguous()
    lam = pr["lam"] * float(plan.adjoint(y).abs().max().item())
    L = plan.lipschitz(50, seed=0)
    delta = 1.0 / (1.05 * L)
    print(f"[bench] volume ready: lambda={lam:.4g} L={L:.4g}", file=sys.stderr, flush=True)
    z, ms_step = time_solve(plan, y, "haar", lam, delta, args.steps, args.warmup, haar_levels=3)
    print(f"[bench] volume solve: {ms_step:.4f} ms/iteration", file=sys.stderr, flush=True)
    sb = stage_bytes(geom, False, "haar")
    stages = time_stages(plan, "haar", y, sb, args.stage_reps)
    ms_grad = time_grad(plan, z, y, args.stage_reps)
    gb = grad_bytes(geom, False)
    roof = roofline(WORKLOAD, stages, "haar", True, geom)
    del z, xt
    plan.close()
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC,
        "value": round(1000.0 / ms_step, 3),
        "unit": "MBIR iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (complex64; FP64 reductions and momenta)",
        "data": "synthetic (seeded scatterers in a smooth random background, 1% noise, every pixel observed)",
        "config": {"workload": "3-D volume 2048 spectral px x 256 x 256 A-scans, image 2048x256x256 complex64, "
                               "2-D lateral FFT, 3-level 3-D Haar l1 lambda=0.01 lambda_max, KB J=6 sigma=2, "
                               "one FISTA iteration per step",
                   "n_depth": geom.n_depth, "n_x": geom.n_x, "n_y": geom.n_y, "n_k": geom.n_k,
                   "penalty": "haar", "parallelism": "1 GPU"},
        "phi_phih_per_s": round(1000.0 / ms_grad, 2),
        "phi_phih_ms": round(ms_grad, 5),
        "phi_phih_GBps": round(gb / (ms_grad * 1e-3) / 1e9, 1),
        "phi_phih_frac_of_peak": round(gb / (ms_grad * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        "stages": {k: {"ms": round(v["ms"], 5), "GBps": round(v["GBps"], 1)} for k, v in stages.items()},
        "roofline": roof,
    }
    if not args.no_bscan:
        out[BSCAN] = bscan_line(args, extra=True)
        out[SMALL] = small_line()
    return out


def small_line(reps: int = 20) -> dict:
    """The small B-scan (512 x 64, 20 scatterers, 1% noise, l1 lambda = 0.01
    lambda_max, 50 iterations) is launch-bound: the latency of a whole solve,
    launched op by op and replayed from a captured HIP graph of the same calls
    (the replay's result is compared bitwise with the launched solve), and
    Phi + Phi^H applications per second at this size."""
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    pr = synth.preset(SMALL)
    geom = P.Geometry.from_dict(pr["geom"])
    rng = np.random.default_rng(0)
    x_true = synth.scatterers(rng, geom.img_shape, pr["scatterers"])
    plan = P.Plan(geom)
    y = plan.forward(torch.from_numpy(x_true.astype(np.complex64)).cuda())
    noise = torch.from_numpy(rng.standard_normal(tuple(y.shape)).astype(np.float32)).cuda()
    y = (y + pr["noise"] * float(y.abs().max().item()) * noise).contiguous()
    lam = pr["lam"] * float(plan.adjoint(y).abs().max().item())
    delta = 1.0 / (1.05 * plan.lipschitz(50, seed=0))
    iters = pr["iters"]
    z = torch.empty(geom.img_shape, dtype=torch.complex64, device="cuda")

    def solve():
        plan.mbir_solve(y, "l1", lam, iters, delta=delta, x_out=z)

    def latency(fn) -> float:
        ts = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        return float(np.median(ts)) * 1e3

    for _ in range(3):
        solve()
    torch.cuda.synchronize()
    ref = z.clone()
    ms_eager = latency(solve)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        solve()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        solve()
    z.zero_()
    graph.replay()
    torch.cuda.synchronize()
    equal = bool(torch.equal(z, ref))
    ms_graph = latency(graph.replay)
    ms_grad = time_grad(plan, ref, y, 200)
    gb = grad_bytes(geom, False)
    del graph
    plan.close()
    return {
        "workload": "B-scan 512 spectral px x 64 A-scans, 20 scatterers, l1 lambda=0.01 lambda_max, "
                    "50 iterations per solve",
        "solve_ms_launched": round(ms_eager, 4), "solve_ms_graph": round(ms_graph, 4),
        "graph_replay_bitwise_equal": equal,
        "iters_per_s_launched": round(iters * 1000.0 / ms_eager, 1),
        "iters_per_s_graph": round(iters * 1000.0 / ms_graph, 1),
        "phi_phih_ms": round(ms_grad, 5), "phi_phih_per_s": round(1000.0 / ms_grad, 1),
        "phi_phih_GBps": round(gb / (ms_grad * 1e-3) / 1e9, 1),
    }


def bscan_line(args, extra: bool = False) -> dict:
    """The full-size B-scan TV workload: the headline with --workload bscan,
    else a summary under its own key."""
    import numpy as np
    import torch
    import paper_2108_01438_amd as P
    import synth
    geom, pr, x_true, mask, noise = make_workload(P, synth, torch)
    plan = P.Plan(geom, mask)
    mask_d = torch.from_numpy(mask.astype(np.float32)[None]).cuda()
    xt = torch.from_numpy(x_true.astype(np.complex64)).cuda()
    y_clean = plan.forward(xt)
    sigma = pr["noise"] * float(y_clean.abs().max().item())
    y = ((y_clean + sigma * torch.from_numpy(noise.astype(np.float32)).cuda()) * mask_d).contiguous()
    lam = pr["lam"] * float(plan.adjoint(y).abs().max().item())
    L = plan.lipschitz(50, seed=0)
    delta = 1.0 / (1.05 * L)
    bound = args.bound * float(xt.abs().max().item()) if args.bound > 0 else None
    steps = 100 if extra else args.steps
    z, ms_step = time_solve(plan, y, "tv", lam, delta, steps, args.warmup, tv_inner=10, bound=bound)
    print(f"[bench] B-scan solve: {ms_step:.4f} ms/iteration", file=sys.stderr, flush=True)
    sb = stage_bytes(geom, True, "tv")
    stages = time_stages(plan, "tv", y, sb, 50)
    ms_grad = time_grad(plan, z, y, 50)
    gb = grad_bytes(geom, True)
    roof = roofline(BSCAN, stages, "tv", False, geom)
    plan.close()
    summary = {
        "ms_per_iteration": round(ms_step, 5), "iters_per_s": round(1000.0 / ms_step, 2),
        "phi_phih_ms": round(ms_grad, 5), "phi_phih_per_s": round(1000.0 / ms_grad, 1),
        "phi_phih_GBps": round(gb / (ms_grad * 1e-3) / 1e9, 1),
        "stages": {k: {"ms": round(v["ms"], 5), "GBps": round(v["GBps"], 1)} for k, v in stages.items()},
        "roofline": roof,
    }
    if extra:
        summary["workload"] = ("B-scan 2048 spectral px x 1000 A-scans, 50% random mask, isotropic TV "
                               "lambda=0.005 lambda_max, 10 FGP steps, 100 iterations")
        return summary
    out = {
        "metric": METRIC, "value": round(1000.0 / ms_step, 2), "unit": "MBIR iters/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (complex64; FP64 reductions and momenta)",
        "data": "synthetic (seeded scatterers + layered speckle, 1% noise, 50% random mask)",
        "config": {"workload": "B-scan 2048 spectral px x 1000 A-scans, image 2048x1000 complex64, "
                               "isotropic TV lambda=0.005 lambda_max, 10 FGP steps, KB J=6 sigma=2, "
                               "one FISTA iteration per step",
                   "n_depth": geom.n_depth, "n_x": geom.n_x, "n_k": geom.n_k, "penalty": "tv",
                   "parallelism": "1 GPU"},
    }
    out.update({k: v for k, v in summary.items() if k not in ("ms_per_iteration", "iters_per_s")})
    if bound is not None:
        out["config"]["bound"] = f"|x_i| <= {args.bound} max|x_true| (constraint set C)"
    return out


if __name__ == "__main__":
    sys.exit(main())
