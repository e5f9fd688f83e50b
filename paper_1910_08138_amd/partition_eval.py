"""Sub-block partitions compared on the GPU (paper Sec. 5.2): the partition
a scene generator draws (recursive coordinate bisection to the configured
sub-block sizes) against the visibility-graph partitioner with the same
number of sub-blocks, with and without its cost-model pass.

Per partition: tie points and point copies (the intersection and exchange
work), the camera counts of the sub-blocks, the time of one LM step of all
sub-blocks (HIP-graph replays timed with HIP events, median of 5), and on
request a run of the method under the improvement test (outer iterations,
sigma0, camera-centre error).

    python -m paper_1910_08138_amd.partition_eval [--configs 2,3] [--schedule]
"""
from __future__ import annotations

import argparse
import json

import numpy as np

from . import binding, scenes, tune
from .ablation import centre_error


def lm_step_ms(scene, precision=binding.RPBA_MIXED):
    ms, fails = tune.measure(scene, dict(precision=precision), steps=5)
    return ms, fails


def evaluate(scene, name, schedule, log):
    sizes = np.bincount(scene.cam_block, minlength=scene.L)
    L = scene.L
    pairs = np.unique(scene.obs_pt.astype(np.int64) * L + scene.cam_block[scene.obs_cam])
    per_pt = np.bincount(pairs // L, minlength=scene.N)
    row = dict(partition=name, scene=scene.name, M=scene.M, L=int(L), tie_points=int((per_pt >= 2).sum()),
               point_copies=int(per_pt.sum()), min_cams=int(sizes.min()), max_cams=int(sizes.max()))
    for prec, key in ((binding.RPBA_MIXED, "lm_step_ms_mixed"), (binding.RPBA_FP64, "lm_step_ms_fp64")):
        ms, fails = lm_step_ms(scene, prec)
        row[key] = ms
        row[key.replace("ms", "fails")] = fails
    if schedule:
        p, hist = binding.run_ratio_rule(scene, T_max=15, I_max=10, graph=True, precision=binding.RPBA_MIXED)
        st = hist[-1]["int_stats"]
        _, C = p.cameras()
        row.update(outer_iterations=len(hist) - 1, sigma0_px=float(st[1]), centre_error_rel=centre_error(scene, C))
        p.close()
    log(json.dumps(row))
    return row


def run(configs=(2, 3), seed=0, schedule=False, small=False, log=print):
    rows = []
    for cfg in configs:
        s = scenes.config_scene(cfg, seed, small=small)
        rows.append(evaluate(s, "generator (coordinate bisection)", schedule, log))
        blk, _, st = binding.partition(s, s.L, imbalance=0.05)
        rows.append(evaluate(s.repartition(blk, name=s.name), "visibility graph", schedule, log))
        blk, _, st = binding.partition(s, s.L, imbalance=0.05, cost_cams3=1.0, cost_obs=0.0)
        rows.append(evaluate(s.repartition(blk, name=s.name), "visibility graph + cost pass (n^3)", schedule, log))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", default="2,3")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--schedule", action="store_true")
    ap.add_argument("--small", action="store_true")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the partition comparison runs on the GPU"
    binding.load_library()
    run(tuple(int(c) for c in args.configs.split(",")), args.seed, args.schedule, args.small,
        log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
