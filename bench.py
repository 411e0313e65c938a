"""Benchmark of the StoDIP data-consistency hot path on one MI355X.

A step is one minibatch DC gradient of the MRF subspace operator (forward,
residual, loss and adjoint; Algorithm 1's forward + loss.backward() for the
NUFFT part).  The headline workload is the largest single-GPU one: a 224^3
image x K = 6 subspace channels, a minibatch of 8 of 48 coils, T = 1200
frames x 12 spiral interleaves x 1400 samples (M = 20.16M points), W = 6,
sigma = 2 (448^3 fine grids).

The step is captured once in a HIP graph and the timed steps are replays
(--eager times plain calls instead).  Prints one JSON line: throughput in
nonuniform points x channels per second (M * B * K per fwd+adj), the plain
per-coil/per-channel path beside it (eager calls, on a plan built with the
options the autotuner picks for one coil and one channel), a per-stage
breakdown from HIP events recorded on the library's stream around every
kernel launch of further eager steps, the HBM roofline of the dominant
kernel, the CPU FP64 oracle timed on a bounded sample, and extra rows for
the 160^3 benchmark and the paper-shaped one-coil step.
"""

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

# workload name -> description for the JSON line
WORKLOADS = {
    "c5": "224^3 x K=6 subspace image, 8-of-48 coil minibatch, T=1200 frames x 12 spiral "
          "interleaves x 1400 samples (M=20.16M), KB W=6, sigma=2 (448^3 grid): batched DC "
          "gradient",
    "c4": "160^3 x K=5 subspace image, 4-of-32 coil minibatch, T=1000 frames x 8 spiral "
          "interleaves x 1200 samples (M=9.6M), KB W=6, sigma=2 (320^3 grid): batched DC gradient",
    "paper": "paper-shaped step: 200^3 x K=5 subspace image, 1-of-8 coil minibatch (one coil "
             "per stochastic step), T=880 frames x 28 spiral arms x 876 samples (M=21.59M), "
             "KB W=6, sigma=2 (400^3 grid): DC gradient",
    "small": "latency-bound step: 32^3 x K=5 subspace image, 4-of-8 coil minibatch, T=8 frames "
             "x 1 spiral arm x 1024 samples (M=8192), KB W=6, sigma=2 (64^3 grid): batched DC "
             "gradient",
    "ragged": "ragged volumes in one group call: 128^3 (T=512), 160^3 (T=1000) and "
              "160x192x192 (T=1440), each 8 spiral arms x 1200 samples per frame with its own "
              "trajectory and V, K=5, 4-of-32 coils: batched DC gradient",
}
# member workloads of the ragged group
RAGGED = ["c3r128", "c4", "c3r192"]
HBM_PEAK_GBPS = 8000.0       # MI355X HBM3E
FP32_PEAK_TFLOPS = 157.3     # vector FP32 with packed FMA
FP16_MFMA_PEAK_TFLOPS = 2500.0


def _args():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20,
                    help="points of the CPU oracle sample")
    ap.add_argument("--eager", action="store_true",
                    help="time eager calls instead of replays of the captured step")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c5",
                    help="headline workload (default c5, the largest single-GPU configuration)")
    ap.add_argument("--extra-rows", default="c4,paper",
                    help="comma-separated workloads timed after the headline and reported in "
                         "'extra_rows' ('' for none)")
    ap.add_argument("--extra-steps", type=int, default=10, help="timed steps of an extra row")
    ap.add_argument("--no-plain-tune", action="store_true",
                    help="time the plain path on the batched step's plan instead of a plan "
                         "autotuned for one coil and one channel")
    ap.add_argument("--spread-engine", choices=["auto", "gather", "matrix", "planes"],
                    default="auto")
    ap.add_argument("--point-order", choices=["auto", "cell"], default="auto",
                    help="order of the points in an interpolation tile (plan option)")
    ap.add_argument("--extras", action="store_true",
                    help="also time the calls around the step on the first volume: normal "
                         "operator and CG iterations over all coils, scaled adjoint, full-coil "
                         "DC gradient, TV value/gradient, density compensation")
    ap.add_argument("--autotune", action="store_true",
                    help="build each plan with the options sdn_autotune finds fastest "
                         "(tile, points per item, spreading engine); untimed")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--only-step", action="store_true",
                    help="warmup and timed steps only (no breakdown, plain path, extra rows or "
                         "CPU baseline): for profiler runs")
    return ap.parse_args()


def stage_bytes(g):
    """Algorithmic HBM bytes of one step of each stage (complex64 = 8 B,
    point record = 24 B), for the DC-gradient step."""
    c8 = 8
    P, B, K, M = g["P"], g["B"], g["K"], g["M"]
    nvox = g["Nx"] * g["Ny"] * g["Nz"]
    G = g["nfx"] * g["nfy"] * g["nfz"]
    xline = g["nfx"] * g["Ny"] * g["Nz"]           # x-transformed image lines
    xyplane = g["nfx"] * g["nfy"] * g["Nz"]        # xy-transformed image planes
    return {
        "pre_fftx": c8 * ((K + B) * nvox + P * xline),
        "fft_y": c8 * P * (xline + xyplane),
        "fft_z": c8 * P * (xyplane + G),
        "interp": c8 * (P * G + 2 * B * M) + 24 * M,
        "clear": c8 * P * G,
        "spread": c8 * (P * G + B * M) + 24 * M,
        "ifft_z": c8 * P * (G + xyplane),
        "ifft_y": c8 * P * (xyplane + xline),
        "post_ifftx": c8 * (P * xline + (B + K) * nvox),
    }


# flops of one gridding launch: every nonuniform point meets W^3 cells for
# every (coil, channel) pair, one real weight times one complex value each
# (2 FMAs = 4 flops)
def stage_flops(g, W):
    return {"interp": 4 * W ** 3 * g["M"] * g["P"], "spread": 4 * W ** 3 * g["M"] * g["P"]}


# Kernel sources whose text the committed counter summary was taken from.
_SOURCES = {"interp": "gridops.hip", "spread": "gridops.hip", "pre_fftx": "fft.hip",
            "fft_y": "fft.hip", "fft_z": "fft.hip", "ifft_z": "fft.hip", "ifft_y": "fft.hip",
            "post_ifftx": "fft.hip"}
_HERE = os.path.dirname(os.path.abspath(__file__))


def traffic_file(workload):
    return os.path.join(_HERE, "profiles", f"hbm_traffic_{workload}.txt")


def measured_traffic(stage, workload):
    """HBM bytes per launch of a stage from the committed FETCH_SIZE / WRITE_SIZE
    summary of this workload, or None when there is none or the kernel source
    has changed since the counters were taken."""
    src = os.path.join(_HERE, "paper_2408_02367_amd", "csrc", _SOURCES.get(stage, ""))
    path = traffic_file(workload)
    if not os.path.isfile(path) or not os.path.isfile(src):
        return None
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    for line in open(path):
        parts = dict(kv.split("=", 1) for kv in line.split() if "=" in kv)
        if parts.get("stage") == stage and parts.get("source_sha256") == digest:
            return int(float(parts["hbm_bytes_per_launch"]))
    return None


def cpu_baseline(w, x, smaps, sample):
    """The FP64 oracle's gridding fwd+adj for one (coil, channel) pair of the
    workload: grid stages in full, point stages on a seeded random sample of
    points, extrapolated linearly to all M points."""
    from oracle import gridding
    from oracle.gridding import _WORKERS

    grid = gridding.Grid(w["shape"])
    M = w["traj"].shape[0]
    sel = np.sort(np.random.default_rng(7).choice(M, size=min(sample, M), replace=False))
    pts = w["traj"][sel]
    f = x[0].astype(np.complex128) * smaps[w["coil_idx"][0]].astype(np.complex128)
    t0 = time.perf_counter()
    G = grid.fft(grid.deapodise_pad(f))
    t1 = time.perf_counter()
    u = grid.interp(G, pts)
    t2 = time.perf_counter()
    H = grid.spread(u, pts)
    t3 = time.perf_counter()
    grid.crop_deapodise(grid.ifft(H))
    t4 = time.perf_counter()
    t_grid = (t1 - t0) + (t4 - t3)
    shape_s = "x".join(str(n) for n in w["shape"])
    fine_s = "x".join(str(n) for n in grid.nf)
    t_pts = (t3 - t1) * (M / len(sel))
    return {"value": M / (t_grid + t_pts), "unit": "pts*ch/s", "cores": _WORKERS,
            "kind": "oracle",
            "sample": f"one (coil, channel) fwd+adj of the {shape_s} workload: deapodise/FFT/"
                      f"IFFT/crop on the full {fine_s} grid ({t_grid:.2f} s), interp+spread on "
                      f"{len(sel)} of {M} points ({t3 - t1:.2f} s) scaled to all points",
            "seconds": t4 - t0}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {a.gpus} is not supported (the coil "
              "axis would shard across GPUs, with one all-reduce of the image gradient per "
              "step)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2408_02367_amd as sdn
    import workloads as wl

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    head = measure(a.workload, a, a.steps, a.warmup, dev, torch, sdn, wl, headline=True)
    if a.only_step:
        print(json.dumps(head["out"]), flush=True)
        return
    out = head["out"]
    extras = [n for n in a.extra_rows.split(",") if n.strip() and n.strip() != a.workload]
    if a.extras:
        _log("timing the calls around the step")
        out["extras"] = _extras(head["vols"][0], torch, sdn)
    cpu_w = head["vols"][0]["w"]
    del head
    torch.cuda.empty_cache()
    if extras:
        out["extra_rows"] = []
        for name in extras:
            r = measure(name.strip(), a, min(a.steps, a.extra_steps), min(a.warmup, 2), dev,
                        torch, sdn, wl, headline=False)
            row = r["out"]
            out["extra_rows"].append({k: row[k] for k in (
                "name", "value", "unit", "ms_per_step", "step_ms_p10_p50_p90", "timing",
                "eager_profiled_ms_per_step", "plain_ms_per_step", "speedup_vs_plain",
                "plain_tuned_options", "config", "stages", "plain_stages_ms", "roofline")})
            del r
            torch.cuda.empty_cache()
    if not a.no_cpu_baseline:
        _log("timing the CPU oracle sample")
        out["cpu_baseline"] = cpu_baseline(cpu_w, cpu_w["x"], cpu_w["smaps"], a.cpu_sample)
    print(json.dumps(out), flush=True)


def measure(workload, a, steps, warmup, dev, torch, sdn, wl, headline):
    """Time one workload's DC step (graph replays), its stage breakdown and
    the plain path; returns {"out": the JSON fields, "vols": the volumes}."""
    names = RAGGED if workload == "ragged" else [workload]
    vols = []
    for name in names:
        _log(f"drawing the synthetic workload {name}")
        vols.append(_volume(name, a, dev, torch, sdn, wl))
    K, B = vols[0]["K"], vols[0]["B"]
    P = B * K
    group = sdn.PlanGroup([v["plan"] for v in vols]) if len(vols) > 1 else None

    def step():
        if group is None:
            v = vols[0]
            sdn.mrf_dc_grad(v["plan"], v["x"], v["smaps"], v["ci"], v["V"], v["d"],
                            grad=v["grad"], loss=v["loss"])
        else:
            group.mrf_dc_grad([v["x"] for v in vols], [v["smaps"] for v in vols],
                              [v["ci"] for v in vols], [v["V"] for v in vols],
                              [v["d"] for v in vols])

    _log(f"{workload}: warmup")
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    # the DC step captured once in a HIP graph (the workspace is sized by now,
    # so a step is kernels on the stream only); the timed steps are replays
    graph = None
    if not a.eager:
        graph = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            step()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(graph):
            step()
        for _ in range(2):
            graph.replay()
        torch.cuda.synchronize()
    run = graph.replay if graph is not None else step
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for e0, e1 in ev:
        e0.record()
        run()
        e1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_step = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    ms_step = (t1 - t0) * 1e3 / steps
    M_all = sum(v["M"] for v in vols)
    value = M_all * P / (ms_step * 1e-3)
    _log(f"{workload}: {ms_step:.3f} ms/step")
    v0 = vols[0]
    engine = v0["plan"].spread_engine(B, K)
    config = {"workload": WORKLOADS[workload], "name": workload, "spread_engine": engine,
              "K": K, "B": B, "W": v0["info"]["W"], "sigma": v0["info"]["sigma"],
              "autotuned": bool(a.autotune), "tile": list(v0["info"]["tile"]),
              "point_order": v0["point_order"]}
    if len(vols) == 1:
        config.update({"shape": list(v0["shape"]), "C": v0["C"], "M": v0["M"], "T": v0["T"]})
    else:
        config["volumes"] = [{"shape": list(v["shape"]), "C": v["C"], "M": v["M"], "T": v["T"]}
                             for v in vols]
    out = {
        "metric": "NUFFT fwd+adj nonuniform pts*ch/s (minibatch DC gradient)",
        "name": workload,
        "value": round(value, 1),
        "unit": "pts*ch/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_step, 3),
        "step_ms_p10_p50_p90": [round(float(np.percentile(per_step, q)), 3) for q in (10, 50, 90)],
        "timing": "hipGraph replays of the captured step" if graph is not None else "eager calls",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": ("fp32 (spreading products on the matrix cores from split fp16 hi/lo operands, "
                  "fp32 accumulation)" if engine in ("matrix", "planes") else "fp32"),
        "data": "synthetic",
        "config": config,
    }
    if a.only_step:
        _calibration_copy(a, dev, torch)
        return {"out": out, "vols": vols}

    # per-stage breakdown: eager steps with HIP events around every launch,
    # recorded by the library on the stream it launches on
    _log(f"{workload}: stage breakdown")
    for v in vols:
        v["plan"].profile(True)
        v["plan"].profile_read(reset=True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t2) * 1e3 / steps
    stages = {}
    for v in vols:
        for st, (ms, n) in v["plan"].profile_read(reset=True).items():
            m0, n0 = stages.get(st, (0.0, 0))
            stages[st] = (m0 + ms, n0 + n)
        v["plan"].profile(False)
    out["eager_profiled_ms_per_step"] = round(eager_ms, 3)
    if group is not None:
        # the group call (one interpolation and one spreading launch over all
        # volumes) against the member plans called one after another, both
        # as eager calls
        def loop_step():
            for v in vols:
                sdn.mrf_dc_grad(v["plan"], v["x"], v["smaps"], v["ci"], v["V"], v["d"],
                                grad=v["grad"], loss=v["loss"])

        out["ragged_fused_eager_ms"] = _timed(step, torch, reps=steps)
        out["ragged_member_loop_eager_ms"] = _timed(loop_step, torch, reps=steps)

    # the plain per-coil/per-channel path on the same data, on plans built
    # with the options the autotuner finds fastest for one coil and channel
    plain_ms, plain_stages, tuned_opts = None, None, None
    if a.plain_steps > 0:
        for v in vols:
            v["yp"] = torch.empty_like(v["d"])
            v["xo"] = torch.empty_like(v["x"])
            if a.no_plain_tune:
                v["pplan"] = v["plan"]
            else:
                _log(f"{workload}: autotuning the plain path's plan of {v['name']} (B=K=1)")
                tuned = sdn.autotune(v["traj_d"], v["shape"], 1, 1, frame_of_point=v["frame_d"],
                                     T=v["T"])
                tuned_opts = {k: tuned[k] for k in sdn.TUNED_KEYS}
                v["pplan"] = sdn.Plan(v["traj_d"], v["shape"], frame_of_point=v["frame_d"],
                                      T=v["T"], **tuned_opts)

        def plain_step():
            for v in vols:
                sdn.mrf_forward(v["pplan"], v["x"], v["smaps"], v["ci"], v["V"], out=v["yp"],
                                plain=True)
                sdn.mrf_adjoint(v["pplan"], v["d"], v["smaps"], v["ci"], v["V"], out=v["xo"],
                                plain=True)

        _log(f"{workload}: timing the plain path")
        plain_step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.plain_steps):
            plain_step()
        torch.cuda.synchronize()
        plain_ms = (time.perf_counter() - t0) * 1e3 / a.plain_steps
        # stage breakdown of one more plain step (not part of the timing above)
        for v in vols:
            v["pplan"].profile(True)
            v["pplan"].profile_read(reset=True)
        plain_step()
        plain_stages = {}
        for v in vols:
            for st, (ms, n) in v["pplan"].profile_read(reset=True).items():
                plain_stages[st] = round(plain_stages.get(st, 0.0) + ms, 3)
            v["pplan"].profile(False)
        for v in vols:
            if v["pplan"] is not v["plan"]:
                v["pplan"].close()
            v["pplan"] = None
    _calibration_copy(a, dev, torch)

    # algorithmic bytes and flops of one step per stage, summed over volumes;
    # a single volume's step launches each stage once (or once per coil chunk,
    # whose bytes add up to the same total)
    sb, sf, sl = {}, {}, {}
    W = v0["info"]["W"]
    for v in vols:
        info, shape = v["info"], v["shape"]
        geo = dict(P=P, B=B, K=K, M=v["M"], Nz=shape[0], Ny=shape[1], Nx=shape[2],
                   nfz=info["fine"][0], nfy=info["fine"][1], nfx=info["fine"][2])
        for dct, part in ((sb, stage_bytes(geo)), (sf, stage_flops(geo, W)),
                          # on-chip bytes of the interpolation: every (point,
                          # channel) reads its W^3 cells (8 B each) from LDS
                          (sl, {"interp": 8 * W ** 3 * v["M"] * P})):
            for st, val in part.items():
                dct[st] = dct.get(st, 0) + val
    per_stage = {}
    for st, (ms, n) in stages.items():
        avg = ms / n
        t_step = ms / steps * 1e-3
        per_stage[st] = {"ms_per_step": round(ms / steps, 4), "launches": n,
                         "avg_launch_ms": round(avg, 4)}
        if st in sb:
            per_stage[st]["algo_GBps"] = round(sb[st] / t_step / 1e9, 1)
            per_stage[st]["hbm_frac"] = round(sb[st] / t_step / (HBM_PEAK_GBPS * 1e9), 4)
        if st in sf:
            per_stage[st]["TFLOPs"] = round(sf[st] / t_step / 1e12, 2)
            # against the FP32 vector peak (157.3 TFLOP/s with packed FP32)
            per_stage[st]["fp32_vector_frac"] = round(sf[st] / t_step / (FP32_PEAK_TFLOPS * 1e12), 4)
        if st in sl:
            per_stage[st]["lds_read_TBps"] = round(sl[st] / t_step / 1e12, 1)
    out["stages"] = per_stage
    out["roofline"] = roofline(stages, sb, sf, steps, vols, B, K, engine, workload)
    out["plain_ms_per_step"] = round(plain_ms, 3) if plain_ms else None
    out["speedup_vs_plain"] = round(plain_ms / ms_step, 3) if plain_ms else None
    out["plain_tuned_options"] = tuned_opts
    out["plain_stages_ms"] = plain_stages
    out["torch_peak_mem_GB"] = round(torch.cuda.max_memory_allocated() / 1e9, 2)
    out["plan_workspace_GB"] = round(sum(v["plan"].workspace_size(B, K) for v in vols) / 1e9, 2)
    _log(f"{workload}: plain {plain_ms} ms/step")
    if group is not None:
        group.close()
    return {"out": out, "vols": vols}


def _calibration_copy(a, dev, torch):
    """One fill and one device copy of --calib-copy-mb MiB: known traffic for
    scaling the HBM counters."""
    if a.calib_copy_mb <= 0:
        return
    n = a.calib_copy_mb * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def roofline(stages, sb, sf, steps, vols, B, K, engine, workload):
    """HBM roofline of the dominant kernel (the stage with the most time):
    algorithmic bytes per launch over its average launch time, against
    8 TB/s, with its vector-ALU and matrix-core figures beside it."""
    dom = max((st for st in stages if st in sb), key=lambda st: stages[st][0])
    launches_per_step = stages[dom][1] / steps
    dom_avg_s = stages[dom][0] / stages[dom][1] * 1e-3
    bytes_launch = sb[dom] / launches_per_step
    achieved = bytes_launch / dom_avg_s / 1e9
    r = {"kernel": dom, "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
         "algo_bytes_per_launch": bytes_launch,
         "traffic": measured_traffic(dom, workload),
         "avg_launch_ms": round(dom_avg_s * 1e3, 4)}
    if dom in sf:
        # the gridding kernels sit above the FP32 ridge (864 flop per point and
        # channel against ~30 B): their arithmetic figures beside the HBM ones
        fl = sf[dom] / launches_per_step / dom_avg_s / 1e12
        r["alu"] = {"achieved_TFLOPs": round(fl, 2), "peak_TFLOPs": FP32_PEAK_TFLOPS,
                    "frac": round(fl / FP32_PEAK_TFLOPS, 4),
                    "algo_flops_per_launch": sf[dom] / launches_per_step}
        if dom == "spread" and engine == "matrix":
            # (entry, coil) block products: 64 x 16K outputs per list entry,
            # three split products of 2 flops each
            blocks = sum(v["info"]["nvisit"] for v in vols) * B
            executed = blocks * 64 * 16 * K * 3 * 2 / launches_per_step
            r["mfma"] = {"dtype": "fp16 (split hi/lo), fp32 accumulation",
                         "executed_TFLOPs_upper_bound": round(executed / dom_avg_s / 1e12, 1),
                         "peak_TFLOPs": FP16_MFMA_PEAK_TFLOPS}
        elif dom == "spread" and engine == "planes":
            r["mfma"] = {"dtype": "fp16 (split hi/lo), fp32 accumulation",
                         "peak_TFLOPs": FP16_MFMA_PEAK_TFLOPS,
                         "note": "planes no entry of a batch touches are skipped, so the "
                                 "executed products depend on the list order"}
    return r


def _timed(fn, torch, reps=3):
    """Milliseconds per call of fn (after one untimed call), HIP events on
    the current stream."""
    fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return round(e0.elapsed_time(e1) / reps, 3)


def _extras(v, torch, sdn):
    """Times of the initialisers (all C coils), the full-coil DC gradient, the
    TV penalty and the density compensation on one volume's plan and data."""
    plan, x, smaps, V = v["plan"], v["x"], v["smaps"], v["V"]
    C, M, K = smaps.shape[0], v["M"], v["K"]
    allc = list(range(C))
    y = sdn.mrf_forward(plan, x, smaps, allc, V)          # data of every coil
    torch.cuda.synchronize()
    out = {"coils": C, "channels": K, "points": M}
    out["normal_op_ms"] = _timed(lambda: sdn.mrf_normal(plan, x, smaps, V), torch)
    iters = 4
    t_cg = _timed(lambda: sdn.mrf_cg(plan, y, smaps, V, iterations=iters, K=K), torch, reps=1)
    t_cg0 = _timed(lambda: sdn.mrf_cg(plan, y, smaps, V, iterations=0, K=K), torch, reps=1)
    out["cg_ms_per_iteration"] = round((t_cg - t_cg0) / iters, 3)
    out["cg_setup_ms"] = t_cg0
    out["scaled_adjoint_ms"] = _timed(lambda: sdn.mrf_scaled_adjoint(plan, y, smaps, V), torch)
    grad = torch.empty_like(x)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    out["full_coil_dc_grad_ms"] = _timed(
        lambda: sdn.mrf_dc_grad(plan, x, smaps, allc, V, y, grad=grad, loss=loss), torch)
    out["full_coil_pts_ch_per_s"] = round(M * C * K / (out["full_coil_dc_grad_ms"] * 1e-3), 1)
    out["tv_value_grad_ms"] = _timed(lambda: sdn.tv_grad(plan, x, 1e-3, 1.0), torch)
    nvox = x.numel() // K
    # TV: x read, gradient written (8 B each) per voxel and channel
    out["tv_algo_GBps"] = round(16 * nvox * K / (out["tv_value_grad_ms"] * 1e-3) / 1e9, 1)
    out["dcf_10_iterations_ms"] = _timed(lambda: sdn.dcf_estimate(plan, 10), torch, reps=1)
    return out


def _volume(name, a, dev, torch, sdn, wl):
    """One volume of a workload on the device: plan, images, coil maps, V and
    simulated measurements d = A x_true + 1% noise of the minibatch coils,
    with the evaluation point x a 10% RMS smooth perturbation of x_true."""
    # the minibatch's coil maps only (normalised over all C coils): the step
    # reads no other map, and c5's 48 maps would take 4.3 GB
    w = wl.make(name, minibatch_maps=name not in ("c1",) and not a.extras)
    shape, K, B = w["shape"], w["K"], w["B"]
    M = w["traj"].shape[0]
    x_true = w["x"]
    pert = wl.phantom(shape, K, w["seed"] + 100)
    pert *= 0.1 * np.sqrt(np.mean(np.abs(x_true) ** 2) / np.mean(np.abs(pert) ** 2))
    x_np = (x_true + pert).astype(np.complex64)
    opts = {"spread_engine": a.spread_engine, "point_order": a.point_order}
    traj_d = torch.from_numpy(w["traj"]).to(dev)
    frame_d = torch.from_numpy(w["frame"]).to(dev)
    if a.autotune:
        _log(f"autotuning the plan of {name}")
        tuned = sdn.autotune(traj_d, shape, B, K, frame_of_point=frame_d, T=w["T"])
        opts = {k: tuned[k] for k in sdn.TUNED_KEYS}
    _log(f"building the plan of {name}")
    plan = sdn.Plan(traj_d, shape, frame_of_point=frame_d, T=w["T"], **opts)
    smaps = torch.from_numpy(w["smaps"]).to(dev)
    V = torch.from_numpy(w["V"]).to(dev)
    ci = w["coil_idx"]
    xt = torch.from_numpy(x_true).to(dev)
    y_clean = sdn.mrf_forward(plan, xt, smaps, ci, V)
    torch.cuda.synchronize()
    rms = torch.sqrt(torch.mean(torch.abs(y_clean) ** 2, dim=1)).cpu().numpy()
    noise = wl.complex_noise((B, M), 0.01, rms, w["seed"])
    d = (y_clean + torch.from_numpy(noise).to(dev)).contiguous()
    del y_clean, xt
    x = torch.from_numpy(x_np).to(dev)
    return dict(w=w, name=name, shape=shape, K=K, B=B, C=w["C"], M=M, T=w["T"], plan=plan,
                traj_d=traj_d, frame_d=frame_d,
                point_order=opts.get("point_order", "auto"),
                info=plan.info(), smaps=smaps, V=V, ci=ci, x=x, d=d,
                grad=torch.empty_like(x), loss=torch.empty(1, dtype=torch.float64, device=dev))


if __name__ == "__main__":
    main()
