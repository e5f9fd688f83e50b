"""Autotuner of librpba's launch configuration.

For one problem it times the sub-block LM step (Schur pass, solve,
back-substitution and update of every sub-block, replayed as a HIP graph and
timed with HIP events on the handle's stream) under each candidate
configuration, and keeps the fastest one whose steps all factorise:

  * the Cholesky tile edge (32 or 64) and the factorisation schedule (one
    persistent dataflow launch, or three launches per tile column);
  * then, with the best of those, the lanes per camera-pair block of the
    Schur pass (4, 8 or 16);
  * on the mixed-precision path also the cut between sub-blocks solved
    directly and those solved by block-Jacobi PCG with iterative refinement
    (``pcg_min_cams`` 300, 200 or 150 cameras; None = every sub-block
    direct).

The search is coordinate-wise: each stage keeps the best configuration of
the previous one and varies one choice.

Results are cached in a JSON file keyed by a signature of the problem's shape
(camera, point and observation counts and the sorted sub-block sizes), the
precision and whether the cameras carry intrinsics, so a second run on the
same shape reuses the choice.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np

from . import binding

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "rpba_tune.json")


def signature(scene, precision) -> str:
    sizes = np.sort(np.bincount(scene.cam_block, minlength=scene.L))
    h = hashlib.sha1()
    intr = int(getattr(scene, "cam_f", None) is not None)
    h.update(np.asarray([scene.M, scene.N, scene.K, scene.L, int(precision), intr], dtype=np.int64).tobytes())
    h.update(sizes.astype(np.int64).tobytes())
    return h.hexdigest()[:20]


def stages(precision, intrinsics=False):
    """The candidate configurations of each search stage; a stage's entries
    override the best configuration found so far.  With intrinsics (8 x 8
    camera blocks) the pair pass always takes 8 lanes and every sub-block is
    solved directly, so only the factorisation is searched."""
    out = [[dict(chol_tile=t, chol_schedule=sc, pair_lanes=8, pcg_min_cams=None)
            for t in (64, 32) for sc in (binding.RPBA_CHOL_DATAFLOW, binding.RPBA_CHOL_STEPWISE)]]
    if intrinsics:
        return out
    out.append([dict(pair_lanes=g) for g in (4, 16)])
    if precision == binding.RPBA_MIXED:
        out.append([dict(pcg_min_cams=c) for c in (300, 200, 150)])
    return out


def _options(cand, precision):
    opts = dict(precision=precision, chol_tile=cand["chol_tile"], chol_schedule=cand["chol_schedule"],
                pair_lanes=cand.get("pair_lanes", 8))
    if cand.get("pcg_min_cams") is not None:
        opts.update(solver=binding.RPBA_SOLVER_AUTO, pcg_min_cams=cand["pcg_min_cams"])
    return opts


def measure(scene, opts, steps=5, warmup=2):
    """Milliseconds per LM step (median over `steps` graph replays) and the
    number of sub-block factorisations that failed."""
    import torch
    p = binding.Problem(scene, **opts)
    try:
        p.set_graph(True)
        p.rpba_intersect()
        for _ in range(warmup):
            p.rpba_subblock_lm_step()
        p.sync()
        times, fails = [], 0
        for _ in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(p.stream)
            bs = p.rpba_subblock_lm_step()
            e1.record(p.stream)
            p.sync()
            times.append(e0.elapsed_time(e1))
            fails += int((bs[:, 3] < 0).sum().item())  # a failed factorisation reports -1 iterations
        return float(np.median(times)), fails
    finally:
        del p
        torch.cuda.synchronize()
        torch.cuda.empty_cache()


def tune(scene, precision=binding.RPBA_FP64, cache_path=DEFAULT_CACHE, steps=5, force=False, log=None):
    """Best options for this problem (a dict for binding.Problem) and the
    table of measured candidates."""
    key = signature(scene, precision)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        try:
            with open(cache_path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if not force and key in cache:
        ent = cache[key]
        return _options(ent["choice"], precision), ent["table"]
    table = []
    best = None
    for stage in stages(precision, getattr(scene, "cam_f", None) is not None):
        base = dict(best) if best else {}
        for k in ("ms", "fails"):
            base.pop(k, None)
        for over in stage:
            cand = dict(base, **over)
            t0 = time.time()
            ms, fails = measure(scene, _options(cand, precision), steps=steps)
            row = dict(cand, ms=ms, fails=fails)
            table.append(row)
            if log:
                log(f"tune {cand}: {ms:.3f} ms per LM step ({time.time() - t0:.1f} s)")
            if fails == 0 and (best is None or ms < best["ms"]):
                best = row
    if best is None:
        best = min(table, key=lambda r: r["ms"])
    choice = {k: best[k] for k in ("chol_tile", "chol_schedule", "pair_lanes", "pcg_min_cams") if k in best}
    if cache_path:
        cache[key] = dict(choice=choice, table=table)
        try:
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            with open(cache_path, "w") as f:
                json.dump(cache, f, indent=1)
        except OSError:
            pass
    return _options(choice, precision), table
