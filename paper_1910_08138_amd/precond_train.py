"""Training and held-out evaluation of the learned block preconditioner on
the reduced camera systems of the method itself (two compact sub-blocks of
200-300 cameras re-partitioned from the 500-camera aerial scenes, seeds
0-23 for training, 24-27 for validation, 28-31 held out).

Every step runs in librpba's kernels: the harvest (features, inverse factors
of the diagonal blocks, probe products), the network's forward and backward
passes and Adam, and the PCG solves of the evaluation.  Reported on the
held-out seeds: CG iterations and solve time with the learned blocks against
block-Jacobi, and the final RMS of both against direct FP64 Cholesky.

    python -m paper_1910_08138_amd.precond_train [--out weights.npy] [--small]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import binding, precond, scenes

TRAIN, VAL, TEST = range(0, 24), range(24, 28), range(28, 32)


def harvest_seeds(seeds, small, nz, T, I, log):
    import torch
    out = []
    for sd in seeds:
        t0 = time.time()
        s = scenes.config_scene(5, sd, small=small)
        out.append(precond.harvest(s, nz=nz, T=T, I=I, seed=sd))
        log(f"harvest seed {sd}: {out[-1].shape[0]} samples, sub-blocks "
            f"{np.bincount(s.cam_block).tolist()} cameras ({time.time() - t0:.1f} s)")
    return torch.cat(out, 0)


def cholesky_rms(scene, T, I):
    p, hist = binding.run_schedule(scene, T=T, I=I, precision=binding.RPBA_MIXED)
    rms = float(hist[-1]["int_stats"][2])
    p.close()
    return rms


def evaluate_seeds(seeds, W, small, T, I, log, **opts):
    rows = []
    for sd in seeds:
        s = scenes.config_scene(5, sd, small=small)
        it_bj, ms_bj, st_bj = precond.evaluate(s, None, T=T, I=I, **opts)
        it_le, ms_le, st_le = precond.evaluate(s, W, T=T, I=I, **opts)
        rms_ch = cholesky_rms(s, T, I)
        row = dict(seed=sd, cg_iterations_block_jacobi=it_bj, cg_iterations_learned=it_le,
                   iteration_ratio=it_le / it_bj, solve_ms_block_jacobi=ms_bj, solve_ms_learned=ms_le,
                   rms_block_jacobi=float(st_bj[2]), rms_learned=float(st_le[2]), rms_cholesky=rms_ch)
        rows.append(row)
        log(json.dumps(row))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--small", action="store_true", help="80-camera scenes (quick check)")
    ap.add_argument("--nz", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=60)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--out", default=None, help="save the trained FP32 weights (numpy .npy)")
    args = ap.parse_args()
    import torch
    assert torch.cuda.is_available(), "training runs on the GPU"
    binding.load_library()
    log = lambda m: print(m, flush=True)  # noqa: E731
    T, I = 3, 2
    data = harvest_seeds(TRAIN, args.small, args.nz, T, I, log)
    val = harvest_seeds(VAL, args.small, args.nz, T, I, log)
    log(f"training samples {data.shape[0]}, validation samples {val.shape[0]}")
    W, losses = precond.train(data, nz=args.nz, epochs=args.epochs, batch=4096, lr=args.lr, seed=0)
    l0, _ = precond.loss_and_grad(val, args.nz, precond.init_params(0))
    l1, _ = precond.loss_and_grad(val, args.nz, W)
    log(f"training loss {losses[0]:.6f} -> {losses[-1]:.6f}; validation loss block-Jacobi {l0:.6f}, learned {l1:.6f}")
    opts = dict(pcg_maxit=2000, ir_tol=1e-10, ir_maxit=10)
    rows = evaluate_seeds(TEST, W, args.small, T, I, log, **opts)
    it_bj = sum(r["cg_iterations_block_jacobi"] for r in rows)
    it_le = sum(r["cg_iterations_learned"] for r in rows)
    log(json.dumps(dict(held_out_seeds=list(TEST), cg_iterations_block_jacobi=it_bj, cg_iterations_learned=it_le,
                        ratio=it_le / it_bj, train_loss=[losses[0], losses[-1]], val_loss=[l0, l1])))
    if args.out:
        np.save(args.out, W.cpu().numpy().astype(np.float32))
        log(f"weights written to {args.out}")


if __name__ == "__main__":
    main()
