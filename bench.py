"""Benchmark of the FLoD-3DGS rasterizer hot path on one MI355X.

Step (the timed unit, `value`): one forward render + L1 loss + backward (gradients for
means, log-scales, quaternions, opacity logits and SH) at 1920x1080 over 1,000,000
cluster-scene Gaussians (SH degree 3, FP32), cycling over 8 seeded orbit cameras; each
camera's L1 target is rendered once, before timing, from a perturbed copy of the scene.
Inputs are resident in HBM before timing starts.

Printed: ONE JSON line. Besides the step it reports, each timed the same way (warm-up, then a
timed loop bracketed by device synchronisation):
  render_fps          forward only, same scene and cameras
  stack_1080p         the 5-level stack (40k..2.5M, 4.39M resident): level 5 alone and
                      selective rendering over levels 1..5 with per-view bands 16/8/4/2
  train_720p          forward + L1 + backward at 1280x720 over 500k Gaussians (s_min 0.0125)
  serving             512 Poisson requests (mean gap 2 ms) of mixed resolution and level
                      selection over the resident stack, 4 slots, 32 GiB HBM budget
  roofline            the dominant kernel of the step, from HIP events recorded on the render
                      stream around that kernel inside the timed region
  cpu_baseline        the CPU oracle on a bounded sample of the step's workload
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import hashlib

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP32_VALU_PEAK_TFLOPS = 157.3  # MI355X fp32 vector, TFLOP/s (FMA = 2 FLOP, packed FP32 issue)
# FP32 lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one operation per lane
# per clock (an FMA counts once); the published 157.3 TFLOP/s is this x 2 (FMA) x 2 (packed
# FP32), and this build does not issue packed FP32
LANE_OP_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12

# Algorithmic work of the hot path's steps (the survey's measurement table), per launch, from the
# frame's own counts: N candidates, K instances, P pixels, Pi pairs walked (sum of n_contrib),
# Pi_bl pairs blended. The blend steps are VALU-bound: 20 lane operations per walked pair
# (offset, q, exp, alpha, tests: about 16 VALU and one exp), and in the backward about 51 per pair,
# read here as the walk's 20 for every walked pair plus 31 (transmittance recovery, dL/dalpha, the
# nine components, the suffix update) for every blended one.
OPS_WALK = 20
OPS_BWD_BLENDED = 31
SURVEY_STEPS = {           # step -> the library's timed stages that implement it
    "S2 preprocess": ["preprocess"],
    "S3 scan": ["offsets"],       # the visible-set compaction is the depth sort's first pass
    "S4 duplicate": ["emit"],
    "S5 sort": ["depth_sort", "tile_sort"],
    "S6 ranges": ["ranges"],
    "S7 blend": ["blend"],
    "S8 blend backward": ["blend_bwd"],
    "S9 preprocess backward": ["preprocess_bwd"],
}


def survey_work(step, N, K, P, tiles, pi_walk, pi_blend):
    """(bytes, lane operations) the step must move / execute at minimum."""
    return {
        "S2 preprocess": ((236 + 48) * N, 0.0),
        "S3 scan": (8 * N, 0.0),
        "S4 duplicate": (16 * N + 12 * K, 0.0),
        "S5 sort": (24 * K, 0.0),
        "S6 ranges": (8 * K + 8 * tiles, 0.0),
        "S7 blend": (40 * K + 20 * P, OPS_WALK * pi_walk),
        "S8 blend backward": (40 * K + 20 * P + 12 * P + 36 * K, OPS_WALK * pi_walk + OPS_BWD_BLENDED * pi_blend),
        "S9 preprocess backward": ((236 + 52 + 236) * N, 0.0),
    }[step]


# FP32 operations per (pixel, list entry) pair of the blend kernels counted as FLOPs (an FMA
# counts 2), for the published FP32 peak: every evaluated pair recomputes d, q, exp, o*G and
# the clamp (15); a blended pair adds 9 in the forward (T update, weight, 3 colour FMAs) and
# 46 in the backward (transmittance recovery, dL/dalpha, 9 gradient components, the suffix
# update).
FLOPS_EVAL = 15
FLOPS_BLEND_FWD = 9
FLOPS_BLEND_BWD = 46


# Measured HBM traffic per launch of a kernel, from two rocprofv3 --pmc runs (FETCH_SIZE,
# then WRITE_SIZE) of `bench.py --no-extras --no-cpu --steps 3 --warmup 1`, each counter
# scaled by its reading for a 1 GiB device-to-device copy (profiles/
# step_1080p_1M_hbm_counters.md). A figure holds only for the kernel sources it was taken
# with: the sha256 over the listed files must match, else the traffic is reported as null.
PROFILED_TRAFFIC = {
    "blend_bwd": {"bytes": 367981396, "sha256": "6ca6729009997e3935e52060e165db65d61653b0101d2999188c0c22c6851ced",
                  "sources": ['paper_2408_12894_amd/csrc/backward.hip', 'paper_2408_12894_amd/csrc/blend_common.h', 'paper_2408_12894_amd/csrc/project.h', 'paper_2408_12894_amd/csrc/flod_internal.h']},
}


def profiled_traffic(kernel: str):
    e = PROFILED_TRAFFIC.get(kernel)
    if not e:
        return None
    h = hashlib.sha256()
    for f in e["sources"]:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return e["bytes"] if h.hexdigest() == e["sha256"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=8)
    ap.add_argument("--n", type=int, default=1_000_000, help="Gaussians in the 1080p scene")
    ap.add_argument("--no-extras", action="store_true", help="only the fwd+bwd step")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=512)
    ap.add_argument("--serving-only", action="store_true",
                    help="only the serving runs over the 5-level stack (for kernel traces of serving)")
    ap.add_argument("--trace-overlap", metavar="CSV", default=None,
                    help="only summarise a rocprofv3 kernel-trace CSV: how much kernel time overlaps")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device-to-device 10 times (reference for HBM byte counters)")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def timed(fn, n, warm, sync):
    for i in range(warm):
        fn(i)
    sync()
    t0 = time.perf_counter()
    for i in range(n):
        fn(i)
    sync()
    return (time.perf_counter() - t0) / n


def algorithmic_bytes(stage, N, n_vis, K, P, tiles):
    """Bytes a stage cannot avoid moving in one launch (its reads and writes of each item once)."""
    return {
        "preprocess": (236 + 80) * N,
        "depth_sort": 4 * N + 8 * n_vis + 3 * 2 * 8 * n_vis,   # the first pass reads every candidate's key
        "offsets": 8 * n_vis,
        "emit": 40 * n_vis + 8 * K,
        "tile_sort": 2 * (4 + 16) * K,
        "ranges": 4 * K + 8 * tiles,
        "blend": 44 * K + 20 * P,
        "blend_bwd": 44 * K + 20 * P + 12 * P + 36 * K,
        "preprocess_bwd": (236 + 4 + 36 + 236) * N,
    }[stage]


def copy_bandwidth(torch, mib=1024, reps=10):
    """Device-to-device copy rate in GB/s (bytes read plus bytes written per second) over a
    `mib` MiB buffer, HIP events around `reps` copies."""
    n = mib << 18
    src = torch.ones(n, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    t = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2 * n * 4 / t / 1e9


def cpu_model() -> str:
    try:
        import subprocess
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def serving_bench(stack, count):
    """The serving trace (Poisson arrivals, mean gap 2 ms, mixed resolutions and level
    selections) over the resident stack under a 32 GiB budget: with 4 slots and, as the
    baseline, the same whole trace one request at a time (1 slot); then saturated (every
    request arriving at once) with 1 and 4 slots for the throughput the device sustains."""
    from paper_2408_12894_amd import serving, synth
    budget = 32 << 30
    trace = synth.serving_trace(seed=30, count=count)
    warm = synth.serving_trace(seed=33, count=64)
    mpix = sum(q.camera.width * q.camera.height for q in trace) / 1e6
    servers = {}
    for n in (4, 1):       # long-running servers, warmed up (contexts hold their workspace)
        servers[n] = serving.Server(stack, n_slots=n, budget_bytes=budget)
        servers[n].serve(warm, time_scale=0.0)

    def run(n_slots, time_scale):
        recs, st = servers[n_slots].serve(trace, time_scale=time_scale)
        span = max(r.done for r in recs if r.status == "ok") - min(r.arrival for r in recs)
        st["mpix_per_s"] = mpix / span
        log(f"serving {n_slots} slot(s){' saturated' if time_scale == 0 else ''}: p50 {st['p50_ms']:.2f} ms "
            f"p99 {st['p99_ms']:.2f} ms, {st['throughput_rps']:.0f} req/s, {st['mpix_per_s']:.0f} Mpix/s; device: "
            f"{st.get('device_overlapping', 0)} of {st.get('device_requests', 0)} requests overlap another, "
            f"concurrency {st.get('device_concurrency', float('nan')):.2f}, max in flight "
            f"{st.get('device_max_in_flight', 0)}; reserved peak {st['device_peak_reserved_bytes'] / 2**30:.2f} "
            f"GiB of {budget / 2**30:.0f}")
        return {k: (float(v) if isinstance(v, (float, np.floating)) else v) for k, v in st.items()}

    out = run(4, 1.0)
    out["one_slot"] = run(1, 1.0)
    out["saturated_4_slots"] = run(4, 0.0)
    out["saturated_1_slot"] = run(1, 0.0)
    for srv in servers.values():
        srv.close()
    out["requests"] = count
    out["offered_rps"] = count / max(q.arrival_s for q in trace)
    return out


def trace_overlap(path, include=None):
    """Kernel concurrency in a rocprofv3 kernel trace (CSV): the union of the kernels'
    [start, end) intervals against their sum, the share of that union with two or more kernels
    running, and the most kernels running at once, per queue and overall."""
    import csv
    rows = list(csv.DictReader(open(path)))
    iv = []
    queues = {}
    for r in rows:
        name = r.get("Kernel_Name", "")
        if include and include not in name:
            continue
        a, b = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
        q = r.get("Queue_Id") or r.get("Stream_Id") or "?"
        iv.append((a, b))
        queues[q] = queues.get(q, 0) + 1
    ev = sorted([(a, 1) for a, _ in iv] + [(b, -1) for _, b in iv], key=lambda e: (e[0], e[1]))
    cur = best = 0
    union = multi = 0
    last = None
    for t, d in ev:
        if last is not None:
            if cur > 0:
                union += t - last
            if cur > 1:
                multi += t - last
        cur += d
        best = max(best, cur)
        last = t
    total = sum(b - a for a, b in iv)
    return {"kernels": len(iv), "queues": len(queues), "kernel_time_ms": total / 1e6,
            "busy_ms": union / 1e6, "concurrency": total / union if union else float("nan"),
            "share_of_busy_with_2plus": multi / union if union else float("nan"), "max_concurrent": best}


def main():
    args = parse()
    if args.trace_overlap:
        print(json.dumps(trace_overlap(args.trace_overlap)), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU (got --gpus {args.gpus}); this build runs on a single "
              "MI355X and its multi-GPU sharding is a design only", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2408_12894_amd import render, serving, synth

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration << 18            # float32 elements in MIB mebibytes
        src = torch.ones(n, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(10):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": n * 4, "copies": 10}), flush=True)
        return
    dev = torch.device("cuda:0")
    sync = torch.cuda.synchronize
    bg = (0.0, 0.0, 0.0)
    out_extra = {}
    if args.serving_only:
        stack = [render.GaussianLevel.from_scene(s_, dev) for s_ in synth.level_stack()]
        print(json.dumps({"serving": serving_bench(stack, args.serving_requests)}), flush=True)
        return

    # ------------------------------------------------------------------ 1080p / 1M step
    log(f"1080p scene: {args.n} Gaussians")
    scene = synth.cluster_scene(args.n, seed=1, layout_seed=1)
    cams = synth.orbit_cameras(2, 8, 4.0, 1920, 1080)
    target = scene.copy()
    rng = np.random.default_rng(3)
    target.means = (scene.means + rng.normal(0, 0.01, scene.means.shape)).astype(np.float32)
    target.opacity_logits = (scene.opacity_logits + rng.normal(0, 0.2, scene.n)).astype(np.float32)
    r = render.Renderer(0)
    lv = render.GaussianLevel.from_scene(scene, dev)
    tl = render.GaussianLevel.from_scene(target, dev)
    targets = [r.render_level(tl, c, bg)[0] for c in cams]
    del tl
    params = [t.clone().requires_grad_(True) for t in (lv.means, lv.log_scales, lv.quats, lv.opacity_logits, lv.sh)]

    def train_step(i):
        for p in params:
            p.grad = None
        img = render.rasterize(*params, cams[i % len(cams)], scene.s_min, bg, renderer=r)
        render.l1_loss(img, targets[i % len(cams)], renderer=r).backward()

    log("fwd+bwd step")
    # warm-up with every stage timed, to find the dominant kernel
    r.set_timing(True)
    r.stage_times(reset=True)
    for i in range(args.warmup):
        train_step(i)
    sync()
    warm = r.stage_times(reset=True)
    dom = max((k for k, (ms, c) in warm.items() if c), key=lambda k: warm[k][0] / warm[k][1])
    # timed steps: HIP events only around the dominant kernel (each recorded stage adds two
    # event records to the stream, which would otherwise inflate the step)
    r.set_timing(True, stages=[dom])
    t0 = time.perf_counter()
    for i in range(args.steps):
        train_step(i)
    sync()
    t1 = time.perf_counter()
    dom_live = r.stage_times(reset=True)[dom]
    ms_step = (t1 - t0) * 1e3 / args.steps
    iters_s = 1e3 / ms_step
    # per-stage breakdown from separate steps with every stage timed
    r.set_timing(True)
    for i in range(min(args.steps, 16)):
        train_step(i)
    sync()
    stage = r.stage_times(reset=True)
    r.set_timing(False)

    # workload counts per camera (K, visible, pairs walked and blended)
    Ks, vis, walk, blended = [], [], [], []
    nbl = torch.empty((1080, 1920), dtype=torch.int32, device=dev)
    for c in cams:
        _, _, nc = r.render_level(lv, c, bg, n_blended=nbl)
        s = r.stats()
        Ks.append(s["n_instances"])
        vis.append(s["n_visible"])
        walk.append(int(nc.sum(dtype=torch.int64)))
        blended.append(int(nbl.sum(dtype=torch.int64)))
    v0 = r.view()
    lens = v0["ranges"][:, 1].astype(np.int64) - v0["ranges"][:, 0]
    K, n_vis = float(np.mean(Ks)), float(np.mean(vis))
    Pi_walk, Pi_blend = float(np.mean(walk)), float(np.mean(blended))
    N, P, tiles = scene.n, 1920 * 1080, 120 * 68
    per_stage = {k: {"ms": ms / c} for k, (ms, c) in stage.items() if c}
    for k, v in per_stage.items():
        v["GBs_algorithmic"] = algorithmic_bytes(k, N, n_vis, K, P, tiles) / (v["ms"] * 1e-3) / 1e9
    dom_ms = dom_live[0] / dom_live[1]        # live, inside the timed steps
    # the measured device-to-device copy rate: the HBM rate a stream of reads and writes reaches
    copy_gbs = copy_bandwidth(torch)
    step_of = {st_: name for name, sts in SURVEY_STEPS.items() for st_ in sts}
    if dom in ("blend", "blend_bwd"):
        b_, ops = survey_work(step_of[dom], N, K, P, tiles, Pi_walk, Pi_blend)
        ach = ops / (dom_ms * 1e-3) / 1e12
        per_pair = FLOPS_BLEND_BWD if dom == "blend_bwd" else FLOPS_BLEND_FWD
        flops = FLOPS_EVAL * Pi_walk + per_pair * Pi_blend
        roof = {"kernel": dom, "bound": "alu", "achieved": ach, "peak": LANE_OP_PEAK_TOPS, "unit": "Top/s",
                "frac": ach / LANE_OP_PEAK_TOPS, "traffic": profiled_traffic(dom),
                "algorithmic_ops_per_launch": ops, "pairs_walked": Pi_walk, "pairs_blended": Pi_blend,
                "fp32_flops_per_launch": flops,
                "frac_of_published_fp32": flops / (dom_ms * 1e-3) / 1e12 / FP32_VALU_PEAK_TFLOPS}
    else:
        byts, _ = survey_work(step_of[dom], N, K, P, tiles, Pi_walk, Pi_blend)
        ach = byts / (dom_ms * 1e-3) / 1e9
        roof = {"kernel": dom, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": ach / HBM_PEAK_GBS, "traffic": profiled_traffic(dom), "algorithmic_bytes_per_launch": byts,
                "frac_of_copy": ach / copy_gbs}
    roof["avg_launch_ms"] = dom_ms
    # whole-step roofline over the survey's steps: the larger of the HBM time and the ALU time
    steps = {}
    t_roof = 0.0
    for name, sts in SURVEY_STEPS.items():
        if not all(x in per_stage for x in sts):
            continue
        ms = sum(per_stage[x]["ms"] for x in sts)
        byts, ops = survey_work(name, N, K, P, tiles, Pi_walk, Pi_blend)
        t_b, t_a = byts / (HBM_PEAK_GBS * 1e9), ops / (LANE_OP_PEAK_TOPS * 1e12)
        t_roof += max(t_b, t_a)
        steps[name] = {"ms": round(ms, 4), "bytes": byts, "ops": ops, "GBs": round(byts / (ms * 1e-3) / 1e9, 1),
                       "frac_hbm": round(byts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 3),
                       "frac_copy": round(byts / (ms * 1e-3) / 1e9 / copy_gbs, 3),
                       "roofline_ms": round(1e3 * max(t_b, t_a), 4), "frac": round(1e3 * max(t_b, t_a) / ms, 3)}
        if ops:
            steps[name]["Tops"] = round(ops / (ms * 1e-3) / 1e12, 2)
            steps[name]["frac_alu"] = round(ops / (ms * 1e-3) / 1e12 / LANE_OP_PEAK_TOPS, 3)
    stage_sum_ms = sum(v["ms"] for v in per_stage.values())
    out_extra["step_roofline"] = {"roofline_ms": 1e3 * t_roof, "stages_ms": stage_sum_ms,
                                  "frac_of_stages": 1e3 * t_roof / stage_sum_ms, "frac_of_step": 1e3 * t_roof / ms_step,
                                  "hbm_peak_GBs": HBM_PEAK_GBS, "hbm_copy_GBs": copy_gbs,
                                  "lane_op_peak_Tops": LANE_OP_PEAK_TOPS, "steps": steps}
    log(f"step {ms_step:.3f} ms ({iters_s:.1f} it/s); K={K:.0f} visible={n_vis:.0f} "
        f"pairs walked {Pi_walk:.3g} blended {Pi_blend:.3g}; device copy {copy_gbs:.0f} GB/s")
    log(f"tile list length mean {lens.mean():.0f} p50 {np.median(lens):.0f} p99 {np.percentile(lens, 99):.0f} "
        f"max {lens.max()}")
    for k, v in per_stage.items():
        log(f"  {k:15s} {v['ms']:.3f} ms  {v['GBs_algorithmic']:.0f} GB/s of this design's bytes")
    for name, v in steps.items():
        extra = f", {v['Tops']:.1f} Top/s = {v['frac_alu']:.2f} of {LANE_OP_PEAK_TOPS:.1f}" if "Tops" in v else ""
        log(f"  {name:24s} {v['ms']:.3f} ms  {v['GBs']:.0f} GB/s of the survey's bytes = {v['frac_hbm']:.2f} of "
            f"8 TB/s, {v['frac_copy']:.2f} of the copy rate{extra}; roofline {v['roofline_ms']:.3f} ms "
            f"({v['frac']:.2f})")

    if not args.no_extras:
        # -------------------------------------------------------------- forward FPS
        # as a caller that only renders (the server's renderers too): no backward state kept
        r.keep_backward_state(False)
        t = timed(lambda i: r.render_level(lv, cams[i % 8], bg), 8 * 8, 8, sync)
        out_extra["render_fps"] = 1.0 / t
        # per-frame device time (events on the render stream): 8 cameras x 20 repetitions
        evs = []
        for rep in range(20):
            for c in cams:
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                r.render_level(lv, c, bg)
                e1.record()
                evs.append((e0, e1))
        sync()
        fms = np.array([a.elapsed_time(b) for a, b in evs])
        out_extra["render_frame_ms"] = {"median": float(np.median(fms)), "p10": float(np.percentile(fms, 10)),
                                        "p90": float(np.percentile(fms, 90)), "fps_median": 1e3 / float(np.median(fms))}
        log(f"render: {1e3 * t:.3f} ms/frame ({1 / t:.1f} FPS); device median {np.median(fms):.3f} ms "
            f"p10 {np.percentile(fms, 10):.3f} p90 {np.percentile(fms, 90):.3f}")
        r.keep_backward_state(True)
        del params, targets
        # -------------------------------------------------------------- 720p training step
        tr_scene, tr_target, tr_cam, _ = synth.training_case()
        tr_lv = render.GaussianLevel.from_scene(tr_scene, dev)
        tr_tgt = r.render_level(render.GaussianLevel.from_scene(tr_target, dev), tr_cam, bg)[0]
        tr_params = [t.clone().requires_grad_(True) for t in
                     (tr_lv.means, tr_lv.log_scales, tr_lv.quats, tr_lv.opacity_logits, tr_lv.sh)]

        def tr_step(i):
            for p in tr_params:
                p.grad = None
            img = render.rasterize(*tr_params, tr_cam, tr_scene.s_min, bg, renderer=r)
            render.l1_loss(img, tr_tgt, renderer=r).backward()

        t = timed(tr_step, 30, 5, sync)
        out_extra["train_720p"] = {"iters_s": 1.0 / t, "ms": 1e3 * t, "n_gaussians": tr_scene.n,
                                   "K": r.stats()["n_instances"]}
        log(f"train 720p/500k: {1e3 * t:.3f} ms ({1 / t:.1f} it/s)")
        # one iteration of the level-training loop: render, L1 + SSIM, backward, fused Adam
        from paper_2408_12894_amd import fit
        fl = fit.clone_level(tr_lv)
        opt = fit.LevelAdam(fl)
        fit_grads = {}

        def fit_step(i):
            image, _, _ = r.render_level(fl, tr_cam, bg)
            x = image.detach().requires_grad_(True)
            render.l1_ssim_loss(x, tr_tgt, 0.2, renderer=r).backward()
            fit_grads.update(r.backward(fl, x.grad))
            opt.step(r, fl, fit_grads)

        t = timed(fit_step, 30, 5, sync)
        t_adam = timed(lambda i: opt.step(r, fl, fit_grads), 50, 5, sync)
        adam_bytes = 28 * 59 * fl.n
        out_extra["fit_iter_720p"] = {"iters_s": 1.0 / t, "ms": 1e3 * t, "n_gaussians": fl.n,
                                      "adam_ms": 1e3 * t_adam, "adam_GBs_algorithmic": adam_bytes / t_adam / 1e9}
        log(f"level-training iteration 720p/500k (L1+SSIM, Adam): {1e3 * t:.3f} ms ({1 / t:.1f} it/s); "
            f"Adam {1e3 * t_adam:.3f} ms, {adam_bytes / t_adam / 1e9:.0f} GB/s algorithmic")
        del tr_params, tr_lv, tr_tgt, fl, opt, fit_grads
        # -------------------------------------------------------------- L1 + SSIM loss at 1080p
        g = torch.Generator(device=dev).manual_seed(5)
        ls_x = torch.rand((3, 1080, 1920), device=dev, generator=g).requires_grad_(True)
        ls_y = torch.rand((3, 1080, 1920), device=dev, generator=g)

        def loss_step(i):
            ls_x.grad = None
            render.l1_ssim_loss(ls_x, ls_y, 0.2, renderer=r).backward()

        t = timed(loss_step, 30, 5, sync)
        out_extra["l1_ssim_1080p"] = {"ms_fwd_bwd": 1e3 * t,
                                      "GBs_algorithmic": (3 * 1080 * 1920 * (8 + 12 + 12 + 12)) / t / 1e9}
        log(f"L1+SSIM 1080p fwd+bwd: {1e3 * t:.3f} ms")
        del ls_x, ls_y
        # -------------------------------------------------------------- 5-level stack at 1080p
        log("5-level stack (4.39M resident)")
        stack_scenes = synth.level_stack()
        stack = [render.GaussianLevel.from_scene(s, dev) for s in stack_scenes]
        del stack_scenes
        t_l5 = timed(lambda i: r.render_level(stack[4], cams[i % 8], bg), 16, 8, sync)
        k_l5 = r.stats()["n_instances"]
        t_sel = timed(lambda i: r.render_selective(stack, 1, 5, synth.LEVEL_BANDS, cams[i % 8].campos, cams[i % 8],
                                                   bg), 16, 8, sync)
        _, _, _, cnt = r.render_selective(stack, 1, 5, synth.LEVEL_BANDS, cams[0].campos, cams[0], bg,
                                          with_counts=True)
        sel_counts = cnt.cpu().tolist()
        k_sel = r.stats()["n_instances"]
        per_level = {}
        for l in range(1, 6):
            tl_ = timed(lambda i: r.render_level(stack[l - 1], cams[i % 8], bg), 8, 2, sync)
            per_level[f"L{l}"] = {"fps": 1.0 / tl_, "K_cam0_last": r.stats()["n_instances"]}
        out_extra["stack_1080p"] = {
            "resident_gaussians": int(sum(x.n for x in stack)), "resident_bytes": int(sum(x.nbytes() for x in stack)),
            "max_level_fps": 1.0 / t_l5, "selective_1_5_fps": 1.0 / t_sel,
            "selective_vs_max_level": t_l5 / t_sel, "selected_per_level_cam0": sel_counts,
            "K_max_level": k_l5, "K_selective": k_sel, "per_level": per_level}
        log(f"stack: L5 {1 / t_l5:.1f} FPS, selective[1,5] {1 / t_sel:.1f} FPS, selected {sel_counts}")
        # predetermined selection set around the mean camera position: compact once, render the subset
        centre = np.mean([c.campos for c in cams], axis=0).astype(np.float32)
        t0 = time.perf_counter()
        gsel = r.select_compact(stack, 1, 5, synth.LEVEL_BANDS, centre)
        sync()
        t_compact = time.perf_counter() - t0
        t_pre = timed(lambda i: r.render_merged(gsel, cams[i % 8], bg), 16, 8, sync)
        out_extra["predetermined_1080p"] = {
            "resident_bytes": int(sum(x.nbytes() for x in gsel)), "kept_per_level": [x.n for x in gsel],
            "compact_ms": 1e3 * t_compact, "render_fps": 1.0 / t_pre}
        log(f"predetermined: {sum(x.nbytes() for x in gsel) / 2**30:.3f} GiB resident, compact "
            f"{1e3 * t_compact:.1f} ms, render {1 / t_pre:.1f} FPS")
        del gsel
        # overlap pruning (d_op = s_min / 2) and the eq. 5 transition, levels 1-4
        ops = {}
        for l in range(1, 5):
            lvl = stack[l - 1]
            kept = r.overlap_prune(lvl, lvl.s_min / 2)[1]
            t_pr = timed(lambda i: r.overlap_prune(lvl, lvl.s_min / 2), 5, 1, sync)
            t_tr = timed(lambda i: r.level_transition(lvl, stack[l].s_min), 5, 1, sync)
            ops[f"L{l}"] = {"n": lvl.n, "prune_ms": 1e3 * t_pr, "kept": kept,
                            "transition_ms": 1e3 * t_tr, "transition_GBs": 2 * 236 * lvl.n / t_tr / 1e9}
            log(f"L{l}: prune {1e3 * t_pr:.2f} ms (kept {kept}/{lvl.n}), transition {1e3 * t_tr:.3f} ms")
        out_extra["level_ops"] = ops
        # -------------------------------------------------------------- serving
        if not args.no_serving:
            out_extra["serving"] = serving_bench(stack, args.serving_requests)
        del stack

    out = {
        "metric": "fwd+bwd iters/s & render FPS at 1080p/1M Gaussians; serving p50/p99 latency",
        "value": iters_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "fwd+bwd step, 1920x1080, 1M cluster-scene Gaussians, SH degree 3, 8 orbit cameras",
                   "n_gaussians": N, "width": 1920, "height": 1080, "instances_K": K, "visible": n_vis},
        "roofline": roof,
        "stages_ms": {k: round(v["ms"], 4) for k, v in per_stage.items()},
    }
    out.update(out_extra)

    # ------------------------------------------------------------------ CPU oracle baseline
    if not args.no_cpu:
        import oracle
        threads = len(os.sched_getaffinity(0))
        oracle.set_threads(threads)
        cam = cams[0]
        t0 = time.perf_counter()
        k = oracle.keys(*scene.arrays()[:4], scene.s_min, cam)
        oracle.instances(k)
        order = oracle.depth_order(k)
        t_keys = time.perf_counter() - t0
        rng = np.random.default_rng(7)
        npx = 4096
        pix = np.unique(np.stack([rng.integers(0, 1920, npx), rng.integers(0, 1080, npx)], 1).astype(np.int32), axis=0)
        npx = pix.shape[0]
        t0 = time.perf_counter()
        ref = oracle.image(order, *scene.arrays()[:4], scene.s_min, scene.sh, 3, cam, bg, pix)
        t_img = time.perf_counter() - t0
        w = np.sign(rng.normal(size=(npx, 3))) / (3 * P)
        t0 = time.perf_counter()
        oracle.grad(order, *scene.arrays()[:4], scene.s_min, scene.sh, 3, cam, bg, pix, w)
        t_grad = time.perf_counter() - t0
        t_frame = t_keys + (t_img + t_grad) * P / npx
        # the 2,000-Gaussian 128x128 frame in full: O1 and O2 over every pixel, median of 3
        from paper_2408_12894_amd import synth as _synth
        s1, c1, b1 = _synth.small_forward_case()
        t1 = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.render(s1.arrays(), s1.s_min, c1, b1)
            t1.append(time.perf_counter() - t0)
        out["cpu_baseline"] = {"value": 1.0 / t_frame, "unit": "iters/s", "cores": oracle.get_threads(),
                               "kind": "oracle", "cpu_model": cpu_model(),
                               "sample": f"fwd+bwd step at 1920x1080/1M, camera 0: O1 keys and sorted instance list "
                                         f"in full ({t_keys:.2f} s), O2 image ({t_img:.2f} s) and O3 gradient "
                                         f"({t_grad:.2f} s) on {npx} of {P} pixels, extrapolated per pixel to the "
                                         f"frame",
                               "extrapolated": True,
                               "small_frame_128x128_2k_s": float(np.median(t1))}
        log(f"cpu oracle: {t_frame:.1f} s per step extrapolated ({oracle.get_threads()} threads, {cpu_model()}); "
            f"128x128 / 2k frame {np.median(t1):.3f} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
