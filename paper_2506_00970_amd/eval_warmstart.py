"""Plain tracking against warm-started tracking on held-out rooms.

    python -m paper_2506_00970_amd.eval_warmstart --weights paper_2506_00970_amd/weights/warm_start.npy

For each room seed: 300k surfels, the ground-truth camera of that seed, the target
RGB-D frame rendered there, and the start pose moved 5 cm and turned 3 deg.  Plain:
`iters` tracking iterations from the start pose.  Warm: the warm start (network,
Exp, fallback check), then the same iterations from its pose.  Convergence is the
first iteration whose pose is within 1 cm and 0.5 deg of the ground truth; its time
is that many iterations at the measured per-iteration time (plus, for the warm
start, its own measured time).  Prints one JSON line.
"""

from __future__ import annotations

import argparse
import json

import numpy as np
import torch

import synth

from ._lib import TRACK_FELL_BACK
from .rasterizer import Rasterizer
from .warmstart import WarmStartNet

CAMERA = synth.Camera(640, 480, 525.0, 525.0, 320.0, 240.0)
TOL_M, TOL_DEG = 0.01, 0.5


def first_converged(hist: np.ndarray, gt: np.ndarray) -> int | None:
    """1-based index of the first pose in hist [iters, 12] within tolerance, or None."""
    for i, p in enumerate(hist):
        m, deg = synth.pose_error(p.reshape(3, 4), gt)
        if m < TOL_M and deg < TOL_DEG:
            return i + 1
    return None


def time_ms(fn, reps: int = 20) -> float:
    for _ in range(3):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def run_case(rast: Rasterizer, net: WarmStartNet, seed: int, iters: int, n_surfels: int = 300_000,
             trans_m: float = 0.05, rot_deg: float = 3.0) -> dict:
    room = synth.make_room(n_surfels, seed=seed)
    gt = synth.room_camera(room, seed=seed)
    start = synth.perturb_pose(gt, trans_m, rot_deg, seed=seed + 1)
    dev = rast.device
    P = torch.from_numpy(room.params).to(dev)
    tgt = rast.render(P, CAMERA, torch.from_numpy(gt.reshape(12)).to(dev))
    trgb, tdep = tgt.rgb.clone(), tgt.depth.clone()
    s = torch.from_numpy(start.reshape(12).astype(np.float32)).to(dev)
    # plain
    pose = s.clone()
    _, ph, _ = rast.track(P, CAMERA, pose, trgb, tdep, iters)
    plain = first_converged(ph.cpu().numpy(), gt)
    # warm: the proposal, then tracking from T_0 with the start pose as its fallback
    w_pose, start_loss = net.propose(rast, P, CAMERA, s, trgb, tdep)
    w0 = w_pose.clone()
    _, wh, _ = rast.track(P, CAMERA, w_pose, trgb, tdep, iters, fallback=(s, start_loss))
    kept = not (rast.track_status[0] & TRACK_FELL_BACK)
    warm = first_converged(wh.cpu().numpy(), gt)
    err0 = synth.pose_error(start, gt)
    errw = synth.pose_error(w0.cpu().numpy().reshape(3, 4), gt)
    return {"seed": seed, "plain_iters": plain, "warm_iters": warm, "kept": kept,
            "start_err_cm_deg": [err0[0] * 100, err0[1]], "warm_err_cm_deg": [errw[0] * 100, errw[1]],
            "P": P, "trgb": trgb, "tdep": tdep, "start": s}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--weights", required=True)
    ap.add_argument("--seeds", type=int, default=20)
    ap.add_argument("--first-seed", type=int, default=0)
    ap.add_argument("--iters", type=int, default=100)
    ap.add_argument("--time-proposal", type=int, default=0, metavar="N",
                    help="only time N back-to-back proposals on the first room, then exit")
    a = ap.parse_args(argv)
    rast = Rasterizer()
    net = WarmStartNet(max_batch=1)
    theta = np.load(a.weights, allow_pickle=False).astype(np.float32)
    net.set_params(torch.from_numpy(theta).cuda())
    if a.time_proposal:
        c = run_case(rast, net, a.first_seed, a.iters)
        ms = time_ms(lambda: net.propose(rast, c["P"], CAMERA, c["start"], c["trgb"], c["tdep"]), a.time_proposal)
        out = {"seed": a.first_seed, "proposal_ms": ms, "calls": a.time_proposal}
        print(json.dumps(out), flush=True)
        return out
    cases = []
    ms_iter = ms_warm = None
    for seed in range(a.first_seed, a.first_seed + a.seeds):
        c = run_case(rast, net, seed, a.iters)
        if ms_iter is None:  # per-iteration and warm-start times, measured once on the first room
            pose = c["start"].clone()
            ms_iter = time_ms(lambda: rast.track(c["P"], CAMERA, pose.copy_(c["start"]), c["trgb"], c["tdep"],
                                                 a.iters, history=False)) / a.iters
            ms_warm = time_ms(lambda: net.propose(rast, c["P"], CAMERA, c["start"], c["trgb"], c["tdep"]))
        for k in ("P", "trgb", "tdep", "start"):
            del c[k]
        cases.append(c)
        print(json.dumps(c), flush=True)

    def ms(it, warm):
        return None if it is None else it * ms_iter + (ms_warm if warm else 0.0)

    plain_ms = [ms(c["plain_iters"], False) for c in cases]
    warm_ms = [ms(c["warm_iters"], True) for c in cases]

    def stats(v):
        ok = [x for x in v if x is not None]
        return {"median_ms": float(np.median(ok)) if ok else None, "p90_ms": float(np.percentile(ok, 90)) if ok else None,
                "success": len(ok) / len(v)}

    out = {"seeds": [c["seed"] for c in cases], "ms_per_iter": ms_iter, "warm_start_ms": ms_warm,
           "plain": stats(plain_ms), "warm": stats(warm_ms),
           "kept_frac": float(np.mean([c["kept"] for c in cases])),
           "faster_frac": float(np.mean([(w is not None) and (p is None or w < p) for p, w in zip(plain_ms, warm_ms)]))}
    print(json.dumps(out), flush=True)
    return out


if __name__ == "__main__":
    main()
