"""The method against its ablations and the plain consensus (paper Sec. 6.3
and 6.4, the comparison of tab:ablation), on a seeded synthetic scene.

Every variant runs the schedule the paper uses for its tables: outer
iterations until the improvement test of the reprojection RMS stops them,
inner LM steps per sub-block until the same test stops each sub-block
(rpba_ratio_update, ratio 1.01).  Reported per variant: outer iterations,
final sigma0 and RMS [px] after the final intersection (for the plain
variants, the evaluation at the consensus points), camera-centre error after
a similarity alignment to the truth, and the wall time of the run on the GPU.

    python -m paper_1910_08138_amd.ablation [--config 2] [--seed 0] [--rho 1000]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import binding, scenes

VARIANTS = [("extended", binding.RPBA_VARIANT_EXTENDED), ("extended, weights from all cameras",
                                                           binding.RPBA_VARIANT_ALL_CAMERAS),
            ("extended, scalar weight rho", binding.RPBA_VARIANT_SCALAR),
            ("plain consensus (ADMM)", binding.RPBA_VARIANT_PLAIN),
            ("plain consensus, refined weights", binding.RPBA_VARIANT_PLAIN_REFINED)]


def centre_error(scene, C):
    """RMS distance of the estimated camera centres from the true ones after
    the best similarity transform (Umeyama 1991), relative to the extent."""
    A, B = C.T, scene.cam_C_true.T
    ma, mb = A.mean(0), B.mean(0)
    U, S, Vt = np.linalg.svd((B - mb).T @ (A - ma))
    D = np.diag([1, 1, np.sign(np.linalg.det(U @ Vt))])
    R = U @ D @ Vt
    sc = np.trace(np.diag(S) @ D) / ((A - ma) ** 2).sum()
    Ab = sc * (A - ma) @ R.T + mb
    ext = float(np.linalg.norm(B.max(0) - B.min(0)))
    return float(np.sqrt(((Ab - B) ** 2).sum(1).mean()) / ext)


def run(scene, rho=1000.0, T_max=30, I_max=10, log=print):
    import torch
    rows = []
    for name, var in VARIANTS:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, hist = binding.run_ratio_rule(scene, T_max=T_max, I_max=I_max, graph=True, variant=var, rho=rho)
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        st = hist[-1]["int_stats"]
        _, C = p.cameras()
        row = dict(variant=name, outer_iterations=len(hist) - 1,
                   lm_steps=int(sum(int(h["steps"].max()) for h in hist[:-1])),
                   sigma0_px=float(st[1]), rms_px=float(st[2]), valid_points=int(st[3]),
                   centre_error_rel=centre_error(scene, C), seconds=secs)
        rows.append(row)
        log(json.dumps(row))
        p.close()
        del p
        torch.cuda.empty_cache()
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--rho", type=float, default=1000.0)
    ap.add_argument("--small", action="store_true")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "the ablation runs on the GPU"
    binding.load_library()
    s = scenes.config_scene(args.config, args.seed, small=args.small)
    print(f"scene {s.name}: M={s.M} N={s.N} K={s.K} L={s.L}, noise {s.sigma_px} px, rho {args.rho}", flush=True)
    run(s, rho=args.rho)


if __name__ == "__main__":
    main()
