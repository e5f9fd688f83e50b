"""Outlier test matrix of the robust estimation (paper Sec. 5.3, and the
comparison of parallel and serial robust estimation in Sec. 6.5,
tab:robust), on seeded synthetic scenes with planted gross errors.

For each share of gross errors (15-40 px displacements on that fraction of
the observations) three runs of the full schedule on the GPU, each under the
improvement test of Sec. 5.4:
  * no robust estimation (the sub-block partition of the scene);
  * the parallel variant on the same partition: after basic convergence the
    observations beyond t_v = 4 are weighted down by 1e-4 at every
    intersection, at the end every point with such an observation is
    eliminated;
  * the serial variant on one block (all cameras, a plain serial bundle
    adjustment): t_v = 3, weighting down after basic convergence, at the end
    the flagged observations deleted and points left in one camera
    eliminated.
Reported per run: outer iterations, observations removed (deleted, or
belonging to an eliminated point) and their share, points eliminated, sigma0
and RMS after the final intersection, the ratio of sigma0 to that of the
non-robust run, the share of planted gross errors removed (recall), the share
of observations removed on points without a gross error, the camera-centre
error after a similarity alignment, the median ratio of the point variances
(sigma0^2 times the trace of the intersection covariance) to those of the
non-robust run, and the wall time.

    python -m paper_1910_08138_amd.robust_matrix [--config 2] [--fracs 0,0.01,0.02,0.05] [--small]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import binding, scenes
from .ablation import centre_error


def removed_mask(scene, weights, status):
    """Observations out of the final adjustment: deleted (weight 0) or of a
    point that is not valid."""
    return (weights == 0.0) | (status[scene.obs_pt] != 0)


def run_one(scene, robust, T_max, I_max):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p, hist = binding.run_ratio_rule(scene, T_max=T_max, I_max=I_max, graph=True, robust=robust)
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    w = p.robust_result()[1] if robust else np.ones(scene.K)
    _, cov, st = p.intersection()
    _, C = p.cameras()
    return dict(p=p, hist=hist, weights=w, status=st, cov=cov, C=C, secs=secs)


def summarise(scene, name, r, base):
    st = r["hist"][-1]["int_stats"]
    rem = removed_mask(scene, r["weights"], r["status"])
    row = dict(variant=name, blocks=int(scene.L), outer_iterations=len(r["hist"]) - 1,
               robust_iterations=int(sum(1 for h in r["hist"][:-1] if h.get("robust"))),
               observations=int(scene.K), removed=int(rem.sum()), removed_pct=100.0 * rem.mean(),
               eliminated_points=int((r["status"] == 4).sum()), sigma0_px=float(st[1]), rms_px=float(st[2]),
               centre_error_rel=centre_error(scene, r["C"]), seconds=r["secs"])
    if scene.outlier is not None and scene.outlier.any():
        bad_pt = np.bincount(scene.obs_pt, weights=scene.outlier.astype(float), minlength=scene.N) > 0
        clean = ~bad_pt[scene.obs_pt]
        row["recall"] = float(rem[scene.outlier].mean())
        row["removed_clean_points_pct"] = 100.0 * float(rem[clean].mean())
    else:
        row["removed_clean_points_pct"] = 100.0 * float(rem.mean())
    if base is not None:
        bst = base["hist"][-1]["int_stats"]
        row["sigma0_ratio"] = float(st[1] / bst[1])
        ok = (r["status"] == 0) & (base["status"] == 0)
        tr = r["cov"][0] + r["cov"][3] + r["cov"][5]
        tb = base["cov"][0] + base["cov"][3] + base["cov"][5]
        ratio = (st[1] ** 2 * tr[ok]) / (bst[1] ** 2 * tb[ok])
        row["variance_ratio_median"] = float(np.median(ratio))
        row["variance_ratio_mean"] = float(ratio.mean())
        row["variance_ratio_std"] = float(ratio.std())
    return row


def run(config=2, seed=0, fracs=(0.0, 0.01, 0.02, 0.05), small=False, T_max=15, I_max=10, log=print):
    import torch
    rows = []
    for frac in fracs:
        s = scenes.config_scene(config, seed, small=small)
        if frac > 0:
            s = scenes.add_gross_errors(s, frac, seed)
        s1 = s.repartition(np.zeros(s.M, dtype=np.int32), name=s.name + "-one-block")
        log(f"scene {s.name}: M={s.M} N={s.N} K={s.K} L={s.L}, gross errors {100 * frac:.1f}%")
        base = run_one(s, False, T_max, I_max)
        for name, sc, robust in (("not robust", s, False), ("parallel, t_v=4", s, "parallel"),
                                 ("serial (one block), t_v=3", s1, "serial")):
            r = base if robust is False else run_one(sc, robust, T_max, I_max)
            row = summarise(sc, name, r, None if robust is False else base)
            row["gross_error_pct"] = 100.0 * frac
            rows.append(row)
            log(json.dumps(row))
            if r is not base:
                r["p"].close()
            torch.cuda.empty_cache()
        base["p"].close()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--fracs", default="0,0.01,0.02,0.05")
    ap.add_argument("--small", action="store_true")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the outlier matrix runs on the GPU"
    binding.load_library()
    run(args.config, args.seed, tuple(float(f) for f in args.fracs.split(",")), small=args.small,
        log=lambda m: print(m, flush=True))


if __name__ == "__main__":
    main()
