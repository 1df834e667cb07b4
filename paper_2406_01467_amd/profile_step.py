"""A short, profiler-friendly run of the rasterizer step.

    python -m paper_2406_01467_amd.profile_step [--workload NAME] [--steps K]

Runs, on cuda:0: one plain copy kernel of known size (a float32 multiply by
one over COPY_MIB MiB, so hardware byte counters can be scaled against a
known read + write volume), then K fwd+bwd steps of the workload enqueued
eagerly (one dispatch per kernel, no graph), with the benchmark's loss
gradient (L1 colour + 5 x Eq. 24).  Meant to run under
`rocprofv3 --kernel-trace --stats` or `rocprofv3 --pmc ...`.
"""
from __future__ import annotations

import argparse
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COPY_MIB = 512


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="plain_1600x1064_1m")
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--tile", default="16x16")
    ap.add_argument("--schedule", type=int, default=1)
    ap.add_argument("--batch", type=int, default=0, help="splats staged per round (0: default)")
    ap.add_argument("--wave", type=int, default=0, help="pixels per wave row (0: 8x8 waves)")
    ap.add_argument("--lane-masks", type=int, default=0,
                    help="1: per-lane splat masks on every 8x8 wave of larger tiles")
    ap.add_argument("--copy-mib", type=int, default=COPY_MIB)
    args = ap.parse_args(argv)

    import torch

    import synth
    from paper_2406_01467_amd import Settings
    from paper_2406_01467_amd.batched import BatchedPlan
    from paper_2406_01467_amd.loss import make_grad_fn
    from paper_2406_01467_amd.raster import Rasterizer

    dev = torch.device("cuda:0")
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(f"copy kernel: {args.copy_mib} MiB read, {args.copy_mib} MiB written", flush=True)
    del src, dst

    scene, views = synth.make_workload(args.workload)
    tw, th = (int(x) for x in args.tile.split("x"))
    st = Settings(tile_w=tw, tile_h=th, sh_degree=scene.sh_degree, schedule=args.schedule,
                  batch=args.batch, wave_w=args.wave, lane_masks=args.lane_masks)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)  # noqa: E731
    params = [t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacities),
              t(scene.sh.reshape(scene.n, -1))]
    target = torch.from_numpy(synth.random_targets(views, seed=7)["color"]).to(dev)
    rast = Rasterizer(views, st, dev)
    plan = BatchedPlan(views, st, params, make_grad_fn(rast, target))
    for i in range(args.steps):
        plan.enqueue()
        torch.cuda.synchronize()
        print(f"step {i + 1}/{args.steps} done, pairs {plan.n_pairs()}", flush=True)
    if plan.overflowed():
        raise RuntimeError("pair capacity overflow")


if __name__ == "__main__":
    main()
