#!/usr/bin/env python3
"""Benchmark: graph-captured 2DGS tracking iterations at 640x480 with 300k surfels on one MI355X.

One step is one tracking iteration of the whole hot path: per-surfel preprocessing,
the pair duplication, the tile sort with the tile ranges, and the tracking walk (each
tile's list put in depth order, then the forward blend of colour/depth/normal/
opacity, the tracking loss with its masks and the pose-only backward with the se(3)
pose reduction in one walk), and the AdamW + Exp pose step.  Inputs (a seeded synthetic 6x5x3 m room with 20 boxes, 300,000 surfels,
the target RGB-D frame rendered at the ground-truth pose, a start pose 5 cm / 3 deg
away) are resident in HBM before timing starts.

Printed (one JSON line): iterations/s over the timed steps, ms to converge to
1 cm / 0.5 deg from the same start, the roofline of the dominant kernel (timed
with HIP events in an eager profiled pass of the same loop), and the FP64 CPU
oracle's iterations/s on the host cores over a bounded sample.
"""

from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "fwd+bwd 2DGS iters/s @640x480, 300k surfels; ms to 1cm/0.5deg pose converge"
LR = (6e-3,) * 6  # the library's tracking default (rasterizer.TRACK_LR)
HBM_PEAK_GBS = 8000.0
# Non-packed FP32 VALU issue rate: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz (one lane-op per
# lane per clock; transcendental ops occupy 4 issue slots).
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# VALU lane-op slots per unit of work, counted in the gfx950 code of the blend kernels
# (transcendentals at 4 slots): per evaluated (pixel, surfel) pair (the pairs each pixel
# walks before it terminates, after the per-wave cull) and per composited pair (3D
# branch).  blend_track: the evaluation, then the compositing with the pose-gradient
# terms; blend_fwd: the evaluation, then the 8-channel compositing; blend_bwd (all
# parameters): the evaluation, then the reverse step and the 16 per-surfel terms it
# adds (the wave reduction that carries those additions is not counted).
OPS_PER_UNIT = {"blend_track": (45, 129), "blend_fwd": (43, 20), "blend_bwd": (42, 86)}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def rooms_summary(warm, conv_iter, ms_step):
    """Median ms to converge over the bench room and the extra rooms (unconverged runs
    count 101 iterations), plain and warm-started (proposal time included)."""
    import numpy as np

    rooms = warm.get("more_rooms")
    if not rooms:
        return {}
    plain = [conv_iter or 101] + [c["plain_iters"] or 101 for c in rooms]
    warm_it = [warm["iters_to_converge"] or 101] + [c["warm_iters"] or 101 for c in rooms]
    return {"rooms": len(plain), "median_ms_to_converge_plain": float(np.median(plain)) * ms_step,
            "median_ms_to_converge_warm": warm["warm_start_ms"] + float(np.median(warm_it)) * ms_step,
            "warm_faster_in": int(sum(warm["warm_start_ms"] + w * ms_step < p * ms_step
                                      for p, w in zip(plain, warm_it)))}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def measured_counters(workload, kernel):
    """Per-launch counters of `kernel` (rocprofv3 name) from the committed counter runs
    (profiles/counters.json), if the blend kernels' source is unchanged since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "counters.json")
    src = os.path.join(ROOT, "paper_2506_00970_amd", "csrc", "blend.hip")
    try:
        with open(path) as f:
            rec = json.load(f)
        with open(src, "rb") as f:
            sha = hashlib.sha256(f.read()).hexdigest()
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != sha:
        return None
    return rec.get(workload, {}).get(kernel)


def alu_roofline(kernel, evaluated, covering, ms, measured=None):
    """The VALU roofline of a blend kernel: algorithmic lane-ops per launch (the per-unit
    counts of OPS_PER_UNIT times the launch's evaluated and composited pairs) over its
    average launch time, against the non-packed FP32 issue peak."""
    pe, pc = OPS_PER_UNIT[kernel]
    ops = pe * evaluated + pc * covering
    achieved = ops / (ms * 1e-3) / 1e12
    out = {"bound": "alu", "kernel": kernel, "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "Tops/s",
           "frac": achieved / VALU_PEAK_TOPS, "traffic": None, "units_per_launch": evaluated,
           "ops_per_unit": ops / max(evaluated, 1.0), "avg_launch_ms": ms,
           "ops_model": {"per_evaluated_pair": pe, "per_composited_pair": pc, "evaluated_pairs": evaluated,
                         "covering_pairs": covering},
           "measured": None}
    if measured:
        out["traffic"] = measured.get("fetch_bytes", 0.0) + measured.get("write_bytes", 0.0) or None
        out["measured"] = {k: measured[k] for k in ("valu_busy", "valu_lane_utilisation", "valu_insts",
                                                     "valu_lane_ops", "lds_insts", "lds_bank_conflict_frac",
                                                     "l2_atomics") if k in measured}
        # issued active-lane VALU work over the same launch time
        out["measured"]["issued_frac"] = measured["valu_lane_ops"] / (ms * 1e-3) / 1e12 / VALU_PEAK_TOPS
    return out


def cpu_baseline(room_params, cam, start, tgt_rgb, tgt_depth, budget_s=20.0):
    """The FP64 oracle on the host: tracking iterations (render, loss, pose-only backward, step)."""
    import numpy as np

    import oracle
    from oracle import loss as oloss

    threads = max(1, min(os.cpu_count() or 1, 16))
    pose = start.astype(np.float64)
    st = oloss.AdamState()
    t0 = time.perf_counter()
    iters = 0
    while True:
        o = oracle.render(room_params, cam, pose, nthreads=threads)
        _, d_rgb, d_depth, _ = oloss.tracking_loss(o["rgb"], o["depth"], o["normal"], o["alpha"], tgt_rgb,
                                                   tgt_depth, cam)
        g = oracle.backward(room_params, cam, pose, d_rgb=d_rgb, d_depth=d_depth, nthreads=threads)
        pose, _ = oloss.adamw_pose_step(pose, g["pose_paper"], st, LR)
        iters += 1
        el = time.perf_counter() - t0
        if el >= budget_s or iters >= 50:
            break
    return {"value": iters / el, "unit": "iters/s", "cores": threads, "kind": "oracle",
            "sample": f"{iters} FP64 tracking iterations (render + loss + pose-only backward + AdamW step) "
                      f"of the same 640x480 / 300k workload in {el:.1f} s on {threads} threads of "
                      f"'{cpu_model()}' ({os.cpu_count()} logical CPUs)"}


def map_bench(args):
    """The mapping side: the forward blend with and without per-surfel contributions
    (eq:contribution) on the tracking workload; the mapping loss of one view and a
    mapping iteration over a 5-keyframe window (batched render, each view's loss, the
    batched backward to all surfel parameters); each bookkeeping kernel at map sizes
    against the HBM roofline.  One JSON line."""
    import numpy as np
    import torch

    import synth
    from paper_2506_00970_amd import Rasterizer, mapstate

    dev = torch.device("cuda", 0)
    cam = synth.Camera(640, 480, 525.0, 525.0, 320.0, 240.0)
    log("building the synthetic room")
    room = synth.make_room(args.n, seed=args.seed)
    pose_np = synth.room_camera(room, seed=args.seed)
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    P, pose = to_dev(room.params), to_dev(pose_np.reshape(12))
    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    blend = {}
    for contrib in (False, True):
        r = Rasterizer(device=0, profile=2)
        for _ in range(3):
            r.render_batch([(P, cam, pose)], contribution=contrib)
        torch.cuda.synchronize()
        r.profile(reset=True)
        for _ in range(args.profile_steps):
            r.render_batch([(P, cam, pose)], contribution=contrib)
        fam = r.profile(reset=True)["families"]
        blend["with_contribution" if contrib else "plain"] = {
            k: fam[k]["ms"] / fam[k]["launches"] for k in fam if fam[k]["launches"]}
        del r

    # the mapping loss of one 640x480 view, and a mapping iteration over the window of
    # N_a + N_i = 5 keyframes: batched render, each view's loss, batched full backward
    from paper_2506_00970_amd import maploss

    r = Rasterizer(device=0, profile=2)
    poses = [to_dev(synth.room_camera(room, seed=args.seed + k).reshape(12)) for k in range(5)]
    tposes = [to_dev(synth.perturb_pose(synth.room_camera(room, seed=args.seed + k), 0.02, 1.0, seed=k).reshape(12))
              for k in range(5)]
    targets = []
    for tp in tposes:
        o = r.render(P, cam, tp)
        targets.append((o.rgb.clone(), o.depth.clone()))
    o = r.render(P, cam, poses[0])
    loss_ms = timed(lambda: maploss.mapping_loss(o.rgb, o.depth, o.normal, targets[0][0], targets[0][1], cam),
                    args.profile_steps)

    def mapping_iteration():
        outs = r.render_batch([(P, cam, p) for p in poses])
        grads = []
        for k, out in enumerate(outs):
            _, d_rgb, d_depth, d_normal = maploss.mapping_loss(out.rgb, out.depth, out.normal, targets[k][0],
                                                               targets[k][1], cam)
            grads.append({"d_rgb": d_rgb, "d_depth": d_depth, "d_normal": d_normal})
        r.backward_batch(outs[0].generation, grads, params_grad=True)

    mapping_iteration()
    torch.cuda.synchronize()
    r.profile(reset=True)
    iter_ms = timed(mapping_iteration, args.profile_steps)
    fam = r.profile(reset=True)["families"]
    # with the Adam step over the surfel parameters: the whole iteration on the device.
    # Tiny learning rates keep the timed workload (the map) the same from step to step;
    # the step's cost does not depend on them.
    Pm = P.clone()
    opt = mapstate.ParamAdam(Pm, lr=(1e-7,) * 6)

    def mapping_iteration_with_step():
        outs = r.render_batch([(Pm, cam, p) for p in poses])
        grads = []
        for k, out in enumerate(outs):
            _, d_rgb, d_depth, d_normal = maploss.mapping_loss(out.rgb, out.depth, out.normal, targets[k][0],
                                                               targets[k][1], cam)
            grads.append({"d_rgb": d_rgb, "d_depth": d_depth, "d_normal": d_normal})
        res = r.backward_batch(outs[0].generation, grads, params_grad=True)
        opt.step(Pm, res[0][0])

    Ps, Gs = P.clone(), torch.randn_like(P)
    opt_s = mapstate.ParamAdam(Ps)
    step_ms = timed(lambda: opt_s.step(Ps, Gs), args.profile_steps)
    del Ps, Gs, opt_s
    full_ms = timed(mapping_iteration_with_step, args.profile_steps)
    mapping = {"loss_ms_640x480": loss_ms, "iteration_ms_5_views": iter_ms,
               "iteration_families_ms": {k: fam[k]["ms"] / (args.profile_steps + 1) for k in fam if fam[k]["launches"]},
               "adam_step_ms": step_ms, "adam_step_GB/s": 7 * 60.0 * args.n / (step_ms * 1e-3) / 1e9,
               "iteration_with_adam_ms_5_views": full_ms}
    del r

    kernels = {}
    g = np.random.default_rng(args.seed)
    for n in (1_000_000, 16_000_000):
        log(f"map kernels at {n} splats")
        params = torch.empty((15, n), dtype=torch.float32, device=dev)
        params.normal_()
        ca = torch.rand(n, device=dev)
        cb = torch.rand(n, device=dev)
        closest = torch.from_numpy(g.integers(0, 8, n).astype(np.int32)).to(dev)
        delta = to_dev(np.tile(np.hstack([np.eye(3), np.full((3, 1), 0.01)]).reshape(1, 12), (8, 1)))
        st = mapstate.MapState(n, dev)
        rm = mapstate.prune_mask(ca, closest, 3)
        kept = float(n - int(rm.sum().item()))
        work = torch.empty(max(1, mapstate._lib.load().gs2d_compact_workspace(n)), dtype=torch.int32, device=dev)
        out = torch.empty_like(params)
        n_out = torch.empty(1, dtype=torch.int32, device=dev)
        moved = float(int((closest < 8).sum().item()))
        # algorithmic HBM bytes per call: every input read once, every output written once
        cases = {
            "covisibility": (lambda: mapstate.covisibility_counts(ca, cb), 8.0 * n),
            "prune_mask": (lambda: mapstate.prune_mask(ca, closest, 3), 9.0 * n),
            "compact_15_planes": (lambda: mapstate._lib.check(mapstate._lib.load().gs2d_compact(
                params.data_ptr(), n, 15, n, rm.data_ptr(), out.data_ptr(), n, n_out.data_ptr(), work.data_ptr(),
                mapstate._stream(dev))), 2.0 * n + 2 * 60.0 * kept),
            "state_update": (lambda: st.update(params, ca, pose, 9, inactive_after=5), 48.0 * n),
            "correct": (lambda: mapstate.correct(params, closest, delta), 4.0 * n + 72.0 * moved),
        }
        for name, (fn, nbytes) in cases.items():
            ms = timed(fn, args.profile_steps)
            kernels[f"{name}@{n}"] = {"ms": ms, "algorithmic_bytes": nbytes, "GB/s": nbytes / (ms * 1e-3) / 1e9,
                                      "frac_hbm": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del params, ca, cb, closest, st, rm, work, out
        torch.cuda.empty_cache()
    top = kernels["state_update@16000000"]
    out = {
        "metric": "mapping side: contribution render, mapping loss and iteration, map kernels",
        "value": top["GB/s"], "unit": "GB/s", "n_gpus": 1, "steps": args.profile_steps, "warmup": 1,
        "higher_is_better": True, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"640x480 f=525 views of the {args.n}-surfel synthetic room (forward render with "
                               "contributions; mapping loss; mapping iteration over 5 views: batched render, "
                               "loss, full backward, no optimizer step); map kernels on 1M and 16M random "
                               "splats", "n_surfels": args.n},
        "roofline": {"bound": "hbm", "kernel": "state_update@16M", "achieved": top["GB/s"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": top["frac_hbm"], "traffic": None},
        "blend_ms_per_launch": blend,
        "mapping": mapping,
        "map_kernels": kernels,
    }
    print(json.dumps(out), flush=True)


def _replay_times(graph, reps):
    """Per-replay GPU times (ms) of a captured graph, each bracketed by its own events."""
    import torch

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in ev:
        a.record()
        graph.replay()
        b.record()
    torch.cuda.synchronize()
    return [a.elapsed_time(b) for a, b in ev]


def config1_bench(args):
    """Single frame: 2,000 random surfels at 64x48, forward render, the unmasked L1 over
    colour, depth and normal against a second seeded render, and the backward to all
    surfel parameters and the pose, captured into one graph after the autotuner has
    picked the tile shape and LDS batch; median of 1,000 replays."""
    import numpy as np
    import torch

    import synth
    from paper_2506_00970_amd import Rasterizer

    dev = torch.device("cuda", 0)
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    s, t = synth.random_surfels(2000, seed=0), synth.random_surfels(2000, seed=1)
    cam = s.camera
    r = Rasterizer(device=0)
    tg = r.render(to_dev(t.params), cam, to_dev(t.pose.reshape(12)))
    trgb, tdep, tnrm = tg.rgb.clone(), tg.depth.clone(), tg.normal.clone()
    P, pose = to_dev(s.params), to_dev(s.pose.reshape(12))
    # 12 tiles of 16 x 16: each blend is one tile's walk; the autotuner weighs smaller tiles
    # on the step's own backward (to all surfel parameters)
    tuning = r.autotune(P, cam, pose, full_backward=True)

    def step():
        out = r.render_batch([(P, cam, pose)])[0]
        _, d_rgb, d_depth, d_normal = r.image_loss(cam, out.rgb, out.depth, out.normal, out.alpha, trgb, tdep, tnrm,
                                                   w_rgb=1.0, w_depth=1.0, w_normal=1.0)
        return r.backward_batch(out.generation, [{"d_rgb": d_rgb, "d_depth": d_depth, "d_normal": d_normal}],
                                params_grad=True)

    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(3):
            step()
    st.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        step()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    times = _replay_times(graph, 1000)
    med = float(np.median(times))
    print(json.dumps({
        "metric": "single-frame fwd+bwd (all surfel params + pose) wall time, graph replay, median of 1,000",
        "value": med * 1e3, "unit": "us", "n_gpus": 1, "steps": 1000, "warmup": args.warmup,
        "ms_per_step": med, "higher_is_better": False, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "2,000 random surfels (seed 0), 64x48 f=60, L1 on colour, depth and normal against "
                               "the render of seed 1; render + loss + backward in one HIP graph", "tuning": tuning},
        "mean_us": float(np.mean(times)) * 1e3, "p90_us": float(np.percentile(times, 90)) * 1e3,
        "counts": r.counts()}), flush=True)


def config3_bench(args):
    """Mapping window: 8 keyframes (4 at 640x480, 4 at 1200x680) over a 1M-surfel room;
    the optimised state is the room with its centres jittered by 5 mm and colours by
    0.05, the poses by 2 cm / 1 deg; targets are renders of the true room.  One
    iteration renders the 8 views in one batched launch, forms each view's opacity-
    masked colour + 0.5 depth L1, and runs the batched backward to all 15 surfel
    parameters and the 8 poses; autotuned tile and batch, captured into one graph."""
    import numpy as np
    import torch

    import synth
    from paper_2506_00970_amd import Rasterizer

    dev = torch.device("cuda", 0)
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    cam_s = synth.Camera(640, 480, 525.0, 525.0, 320.0, 240.0)
    cam_l = synth.Camera(1200, 680, 600.0, 600.0, 600.0, 340.0)
    cams = [cam_s] * 4 + [cam_l] * 4
    log("building the 1M-surfel room")
    room = synth.make_room(1_000_000, seed=100)
    gt = [synth.room_camera(room, seed=100 + k) for k in range(8)]
    g = np.random.default_rng(100)
    state = room.params.astype(np.float32).copy()
    state[0:3] += g.normal(0.0, 0.005, state[0:3].shape).astype(np.float32)
    state[12:15] += g.normal(0.0, 0.05, state[12:15].shape).astype(np.float32)
    poses = [synth.perturb_pose(gt[k], 0.02, 1.0, seed=200 + k) for k in range(8)]
    r = Rasterizer(device=0)
    Pgt = to_dev(room.params)
    targets = []
    for k in range(8):
        o = r.render(Pgt, cams[k], to_dev(gt[k].reshape(12)))
        targets.append((o.rgb.clone(), o.depth.clone()))
    del Pgt
    P = to_dev(state)
    pose_t = [to_dev(p.reshape(12)) for p in poses]
    tuning = r.autotune(P, cam_l, pose_t[4], full_backward=True)
    views = [(P, cams[k], pose_t[k]) for k in range(8)]

    def step(rr=r):
        outs = rr.render_batch(views)
        # every view's loss and image gradients in one launch (and one for the reductions)
        _, g = rr.image_loss_batch([{"camera": cams[k], "rgb": o.rgb, "depth": o.depth, "normal": o.normal,
                                     "alpha": o.alpha, "tgt_rgb": targets[k][0], "tgt_depth": targets[k][1]}
                                    for k, o in enumerate(outs)], w_rgb=1.0, w_depth=0.5, opacity_mask=True)
        grads = [{"d_rgb": d_rgb, "d_depth": d_depth} for d_rgb, d_depth, _ in g]
        return rr.backward_batch(outs[0].generation, grads, params_grad=True)

    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        for _ in range(2):
            step()
    st.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=st):
        step()
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    steps = min(args.steps, 50)
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    times = _replay_times(graph, 20)
    # eager passes of the same iteration with the tuned shape: one counting the blend
    # work (its counting kernels are slower), one timing each kernel family with HIP
    # events while running the same kernels as the graph
    tw, th, tb = tuning["tile_w"], tuning["tile_h"], tuning["batch"]
    rc = Rasterizer(device=0, tile=(tw, th), batch=tb, profile=1)
    step(rc)
    rc.profile(reset=True)
    step(rc)
    prof = rc.profile(reset=True)
    rt = Rasterizer(device=0, tile=(tw, th), batch=tb, profile=2)
    step(rt)
    rt.profile(reset=True)
    for _ in range(3):
        step(rt)
    fam = rt.profile(reset=True)["families"]
    torch.cuda.synchronize()
    per_launch = {k: (v["ms"] / v["launches"] if v["launches"] else 0.0) for k, v in fam.items()}
    nf, nb = max(prof["families"]["blend_fwd"]["launches"], 1), max(prof["families"]["blend_bwd"]["launches"], 1)
    roof_bwd = alu_roofline("blend_bwd", prof["bwd_evaluated"] / nb, prof["bwd_covering"] / nb, per_launch["blend_bwd"],
                            measured_counters("map", f"blend_bwd_kernel<{tw}, {th}, false, false, false, false>"))
    roof_fwd = alu_roofline("blend_fwd", prof["fwd_evaluated"] / nf, prof["fwd_covering"] / nf, per_launch["blend_fwd"],
                            measured_counters("map", f"blend_fwd_kernel<{tw}, {th}, false>"))
    print(json.dumps({
        "metric": "mapping-window iterations/s (8 views fwd + bwd to all surfel params and poses), 1M surfels",
        "value": steps / el, "unit": "iters/s", "n_gpus": 1, "steps": steps, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / steps, "higher_is_better": True, "scaling": "weak", "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "8 keyframes (4 x 640x480 f=525, 4 x 1200x680 f=600) of a 1M-surfel synthetic room "
                               "(seed 100), state jittered 5 mm / 0.05 colour, poses 2 cm / 1 deg; opacity-masked "
                               "colour + 0.5 depth L1 per view; one HIP graph per iteration", "tuning": tuning},
        "median_replay_ms": float(np.median(times)), "counts": r.counts(),
        "roofline": roof_bwd, "roofline_forward": roof_fwd, "kernels_ms_per_launch": per_launch}), flush=True)


def config4_bench(args):
    """Batched tracking: 32 independent problems (320x240 .. 1200x680, 50k .. 1M surfels,
    2-8 cm / 1-5 deg starts), 50 graph-captured iterations of all 32 in one launch per
    kernel per iteration; aggregate iterations/s and per-problem convergence."""
    import numpy as np
    import torch

    import synth
    from paper_2506_00970_amd import Rasterizer

    dev = torch.device("cuda", 0)
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)
    res = [(320, 240), (640, 480), (848, 480), (1200, 680)]
    r = Rasterizer(device=0)
    batch, gts = [], []
    log("building 32 rooms")
    for j in range(32):
        g = np.random.default_rng(1000 + j)
        W, H = res[g.integers(0, 4)]
        f = 525.0 * W / 640.0
        cam = synth.Camera(W, H, f, f, W / 2.0, H / 2.0)
        n = int(round(np.exp(g.uniform(np.log(5e4), np.log(1e6)))))
        room = synth.make_room(n, seed=1000 + j)
        gt = synth.room_camera(room, seed=1000 + j)
        start = synth.perturb_pose(gt, g.uniform(0.02, 0.08), g.uniform(1.0, 5.0), seed=2000 + j)
        P = to_dev(room.params)
        tgt = r.render(P, cam, to_dev(gt.reshape(12)))
        batch.append((P, cam, to_dev(start.reshape(12)), tgt.rgb.clone(), tgt.depth.clone()))
        gts.append(gt)
    starts = [b[2].clone() for b in batch]
    r.track_batch(batch, n_iters=args.warmup)
    for b, s0 in zip(batch, starts):
        b[2].copy_(s0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ph, lh = r.track_batch(batch, n_iters=50)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    hist = ph.cpu().numpy().astype(np.float64)
    conv = []
    for j in range(32):
        it = None
        for i in range(hist.shape[0]):
            e_t, e_r = synth.pose_error(hist[i, j].reshape(3, 4), gts[j])
            if e_t < 0.01 and e_r < 0.5:
                it = i + 1
                break
        conv.append(it)
    # learned warm start, for the problems whose frames the network takes (width 80 k and
    # height 60 k: 320x240 and 640x480): one proposal per problem, then the same 50
    # batched iterations from T_0, with each start pose as that problem's fallback; the
    # other problems start where they did
    warm = None
    if os.path.exists(args.weights):
        from paper_2506_00970_amd._lib import TRACK_FELL_BACK
        from paper_2506_00970_amd.warmstart import WarmStartNet

        log("warm-started batched run")
        net = WarmStartNet(max_batch=1)
        net.set_params(torch.from_numpy(np.load(args.weights, allow_pickle=False).astype(np.float32)).to(dev))
        takes = [c.width % 80 == 0 and c.height % 60 == 0 and c.width // 80 == c.height // 60
                 for (_, c, _, _, _) in batch]
        for j in range(32):  # warm-up proposals (first calls size the image workspace)
            if takes[j]:
                net.propose(r, batch[j][0], batch[j][1], starts[j], batch[j][3], batch[j][4])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        wbatch, fbs = [], []
        for j, (P, c, _, trgb, tdep) in enumerate(batch):
            if takes[j]:
                p0, l0 = net.propose(r, P, c, starts[j], trgb, tdep)
                wbatch.append((P, c, p0, trgb, tdep))
                fbs.append((starts[j], l0))
            else:
                wbatch.append((P, c, starts[j].clone(), trgb, tdep))
                fbs.append(None)
        torch.cuda.synchronize()
        prop_ms = 1e3 * (time.perf_counter() - t0)
        wph, _ = r.track_batch(wbatch, n_iters=50, fallbacks=fbs)
        torch.cuda.synchronize()
        kept = [bool(t and not (st & TRACK_FELL_BACK)) for t, st in zip(takes, r.track_status)]
        whist = wph.cpu().numpy().astype(np.float64)
        wconv = []
        for j in range(32):
            it = None
            for i in range(whist.shape[0]):
                e_t, e_r = synth.pose_error(whist[i, j].reshape(3, 4), gts[j])
                if e_t < 0.01 and e_r < 0.5:
                    it = i + 1
                    break
            wconv.append(it)
        sel = [j for j in range(32) if takes[j]]
        warm = {"problems_warm_started": len(sel), "proposals_ms": prop_ms, "iters_to_converge": wconv,
                "converged": sum(c is not None for c in wconv), "kept_t0": sum(kept),
                "converged_of_warm_started": sum(wconv[j] is not None for j in sel),
                "converged_of_warm_started_plain": sum(conv[j] is not None for j in sel)}
    print(json.dumps({
        "metric": "batched tracking: aggregate iterations/s of 32 independent problems, 50 iterations",
        "value": 32 * 50 / el, "unit": "iters/s", "n_gpus": 1, "steps": 50, "warmup": args.warmup,
        "ms_per_step": 1e3 * el / 50, "higher_is_better": True, "scaling": "weak", "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "32 seeded rooms (seeds 1000-1031), 320x240..1200x680, 50k..1M surfels, "
                               "2-8 cm / 1-5 deg starts, tracking loss with masks, lambda_d = 1"},
        "iters_to_converge": conv, "converged": sum(c is not None for c in conv),
        "ms_to_converge_median": float(np.median([c for c in conv if c])) * 1e3 * el / 50 if any(conv) else None,
        "warm_start": warm}),
        flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=300_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--held-out-rooms", type=int, default=9,
                    help="rooms after the bench room on which plain and warm-started convergence are also measured")
    ap.add_argument("--profile-steps", type=int, default=20)
    ap.add_argument("--weights", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                      "paper_2506_00970_amd", "weights", "warm_start.npy"),
                    help="trained warm-start network (FP32 .npy); the warm-started convergence is skipped "
                         "when the file is absent")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run 3 plain device copies of 256 MiB (reference for HBM traffic counters)")
    ap.add_argument("--map", action="store_true",
                    help="measure the mapping side (contribution render, mapping loss and iteration, map kernels)")
    ap.add_argument("--config", type=int, choices=(1, 3, 4),
                    help="measure another workload instead: 1 single frame, 3 mapping window, 4 batched tracking")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); this build has no multi-GPU path: "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.map:
        return map_bench(args)
    if args.config:
        return {1: config1_bench, 3: config3_bench, 4: config4_bench}[args.config](args)

    import numpy as np
    import torch

    import synth
    from paper_2506_00970_amd import Rasterizer

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.calibrate_copy:
        x = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        del x, y
    cam = synth.Camera(640, 480, 525.0, 525.0, 320.0, 240.0)
    log("building the synthetic room")
    room = synth.make_room(args.n, seed=args.seed)
    pose_gt = synth.room_camera(room, seed=args.seed)
    start = synth.perturb_pose(pose_gt, 0.05, 3.0, seed=args.seed + 1)
    to_dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)

    r = Rasterizer(device=0, profile=1)
    P = to_dev(room.params)
    gt = to_dev(pose_gt.reshape(12))
    tgt = r.render(P, cam, gt)
    tgt_rgb, tgt_depth = tgt.rgb.clone(), tgt.depth.clone()
    pose = to_dev(start.reshape(12))
    start_dev = pose.clone()
    torch.cuda.synchronize()

    # convergence: 100 iterations from the start pose, pose history on the device
    log("convergence run")
    pose.copy_(start_dev)
    _, ph, lh = r.track(P, cam, pose, tgt_rgb, tgt_depth, n_iters=100, lr=LR, use_graph=True)
    torch.cuda.synchronize()
    hist = ph.cpu().numpy().astype(np.float64)
    conv_iter = None
    errs = []
    for i in range(hist.shape[0]):
        e_t, e_r = synth.pose_error(hist[i].reshape(3, 4), pose_gt)
        errs.append((e_t, e_r))
        if conv_iter is None and e_t < 0.01 and e_r < 0.5:
            conv_iter = i + 1

    # learned warm start: the proposal's own time, then the same iterations from T_0, with
    # the start pose as the fallback that the first iteration takes if T_0 is worse
    warm = None
    if os.path.exists(args.weights):
        from paper_2506_00970_amd._lib import TRACK_FELL_BACK
        from paper_2506_00970_amd.warmstart import WarmStartNet

        log("warm-started convergence run")
        net = WarmStartNet(max_batch=1)
        net.set_params(torch.from_numpy(np.load(args.weights, allow_pickle=False).astype(np.float32)).to(dev))
        rw = Rasterizer(device=0)
        rw.track(P, cam, pose.copy_(start_dev), tgt_rgb, tgt_depth, n_iters=args.warmup, lr=LR, history=False)
        for _ in range(3):
            net.propose(rw, P, cam, start_dev, tgt_rgb, tgt_depth)
        torch.cuda.synchronize()
        # back-to-back proposals, HIP events on the stream they run on
        reps = 50
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            w_pose, start_loss = net.propose(rw, P, cam, start_dev, tgt_rgb, tgt_depth)
        ev1.record()
        torch.cuda.synchronize()
        warm_ms = ev0.elapsed_time(ev1) / reps
        w0 = w_pose.cpu().numpy().astype(np.float64).reshape(3, 4)
        _, wph, _ = rw.track(P, cam, w_pose, tgt_rgb, tgt_depth, n_iters=100, lr=LR, use_graph=True,
                             fallback=(start_dev, start_loss))
        torch.cuda.synchronize()
        kept = not (rw.track_status[0] & TRACK_FELL_BACK)
        whist = wph.cpu().numpy().astype(np.float64)
        wconv = None
        for i in range(whist.shape[0]):
            e_t, e_r = synth.pose_error(whist[i].reshape(3, 4), pose_gt)
            if e_t < 0.01 and e_r < 0.5:
                wconv = i + 1
                break
        e0 = synth.pose_error(w0, pose_gt)
        warm = {"warm_start_ms": warm_ms, "iters_to_converge": wconv, "kept": kept,
                "error_after_warm_start_cm_deg": [100 * e0[0], e0[1]]}
        # one room says little about a learned proposal: iterations to converge on the
        # next rooms of the same generator too (plain, and warm-started with fallback)
        if args.held_out_rooms > 0:
            from paper_2506_00970_amd.eval_warmstart import run_case

            log(f"warm start on {args.held_out_rooms} more rooms")
            warm["more_rooms"] = [
                {k: c[k] for k in ("seed", "plain_iters", "warm_iters", "kept")}
                for c in (run_case(rw, net, args.seed + k, 100, n_surfels=args.n)
                          for k in range(1, args.held_out_rooms + 1))]
        del rw, net

    # warm-up and timed graph replays
    log("warm-up")
    pose.copy_(start_dev)
    r.track(P, cam, pose, tgt_rgb, tgt_depth, n_iters=args.warmup, lr=LR, use_graph=True, history=False)
    pose.copy_(start_dev)
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    t0 = time.perf_counter()
    r.track(P, cam, pose, tgt_rgb, tgt_depth, n_iters=args.steps, lr=LR, use_graph=True, history=False)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    ms_step = 1e3 * el / args.steps
    value = args.steps / el

    # eager passes of the same loop: one counting the blend work units (the counting
    # kernels are slower), one timing each kernel family with HIP events on the launch
    # stream while running the same kernels as the graph
    log("profiled eager passes")
    pose.copy_(start_dev)
    torch.cuda.synchronize()
    r.profile(reset=True)
    r.track(P, cam, pose, tgt_rgb, tgt_depth, n_iters=args.profile_steps, lr=LR, use_graph=False, history=False)
    prof = r.profile(reset=True)
    counts = r.counts()
    rt = Rasterizer(device=0, profile=2)
    pose.copy_(start_dev)
    rt.track(P, cam, pose, tgt_rgb, tgt_depth, n_iters=2, lr=LR, use_graph=False, history=False)
    rt.profile(reset=True)
    pose.copy_(start_dev)
    rt.track(P, cam, pose, tgt_rgb, tgt_depth, n_iters=args.profile_steps, lr=LR, use_graph=False, history=False)
    fam = rt.profile(reset=True)["families"]
    per_launch = {k: (v["ms"] / v["launches"] if v["launches"] else 0.0) for k, v in fam.items()}
    cfam = prof["families"]  # launches of the counting pass
    n_fwd = cfam["blend_fwd"]["launches"] + cfam["blend_track"]["launches"]
    n_bwd = cfam["blend_bwd"]["launches"]
    # the tracking walk: evaluated pairs, and the pairs it composites with their
    # forward blend, loss and pose-gradient terms
    roofline = alu_roofline("blend_track", prof["fwd_evaluated"] / max(n_fwd, 1), prof["fwd_covering"] / max(n_fwd, 1),
                            per_launch["blend_track"],
                            measured_counters("track", "blend_track_kernel<16, 16, false>"))

    out = {
        "metric": METRIC,
        "value": value,
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
        "config": {"workload": "tracking iteration (fwd + tracking loss + pose-only bwd + AdamW/Exp step), "
                               "640x480 f=525, 300k-surfel synthetic room (6x5x3 m, 20 boxes), start 5 cm / 3 deg",
                   "n_surfels": args.n, "width": 640, "height": 480, "tile": [16, 16], "graph": True,
                   "room_seed": args.seed},
        "ms_to_converge": (conv_iter * ms_step) if conv_iter else None,
        "iters_to_converge": conv_iter,
        "final_error_cm_deg": [100 * errs[-1][0], errs[-1][1]],
        "warm_start": None if warm is None else dict(
            warm, ms_to_converge=(warm["warm_start_ms"] + warm["iters_to_converge"] * ms_step)
            if warm["iters_to_converge"] else None, **rooms_summary(warm, conv_iter, ms_step)),
        "roofline": roofline,
        "kernels_ms_per_launch": per_launch,
        "work": {"fwd_evaluated": prof["fwd_evaluated"] / max(n_fwd, 1),
                 "fwd_covering": prof["fwd_covering"] / max(n_fwd, 1),
                 "bwd_evaluated": prof["bwd_evaluated"] / max(n_bwd, 1),
                 "bwd_covering": prof["bwd_covering"] / max(n_bwd, 1),
                 "n_visible": counts["n_visible"], "n_pairs": counts["n_pairs"]},
    }
    if not args.no_cpu_baseline:
        log("CPU baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline(room.params, cam, start, tgt_rgb.cpu().numpy().astype(np.float64),
                                           tgt_depth.cpu().numpy().astype(np.float64))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
