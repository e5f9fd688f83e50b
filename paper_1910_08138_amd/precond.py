"""Harvesting, training and evaluation of the learned block preconditioner.

Every computation runs in librpba's kernels (harvest: feature, inverse-factor
and probe-product kernels; training: forward/backward and Adam kernels); this
module only drives them and holds the tensors.

Data: the reduced camera systems the method itself assembles while adjusting
two-sub-block aerial scenes (200-300 cameras per sub-block at full size).
Probes: Rademacher vectors drawn here (seeded) and passed to the library.
"""
from __future__ import annotations

import numpy as np

from . import binding, scenes


def harvest(scene, nz=4, T=3, I=2, seed=0, device="cuda"):
    """Run the fixed schedule with block-Jacobi PCG on every sub-block and
    collect one sample per camera before each LM step."""
    import torch
    p = binding.Problem(scene, device=device, precision=binding.RPBA_MIXED, solver=binding.RPBA_SOLVER_PCG_BJ)
    gen = torch.Generator(device="cpu").manual_seed(int(seed))
    out = []
    for t in range(T):
        p.rpba_intersect()
        for s in range(I):
            z = (torch.randint(0, 2, (nz, scene.M, 6), generator=gen, dtype=torch.int8).float() * 2 - 1).to(device)
            out.append(p.precond_harvest(z))
            p.rpba_subblock_lm_step()
        p.rpba_consensus()
    p.sync()
    return torch.cat(out, 0)


def init_params(seed=0, device="cuda"):
    """Xavier-uniform hidden layers, zero output layer: the initial network
    outputs zero, i.e. exactly block-Jacobi."""
    import torch
    nf, nh, no = 26, 64, 21
    rng = np.random.default_rng(seed)

    def xav(o, i):
        b = np.sqrt(6.0 / (i + o))
        return rng.uniform(-b, b, size=(o, i))

    parts = [xav(nh, nf).ravel(), np.zeros(nh), xav(nh, nh).ravel(), np.zeros(nh), np.zeros(no * nh), np.zeros(no)]
    W = np.concatenate(parts).astype(np.float32)
    assert W.size == binding.precond_num_params()
    return torch.as_tensor(W, device=device)


def train(samples, nz=4, epochs=20, batch=4096, lr=2e-3, seed=0, W=None, log=None):
    """Adam on mini-batches of a once-shuffled sample set; returns (W, losses)."""
    import torch
    dev = samples.device
    n = samples.shape[0]
    perm = torch.as_tensor(np.random.default_rng(seed).permutation(n), device=dev)
    data = samples.index_select(0, perm).contiguous()
    if W is None:
        W = init_params(seed, dev)
    m = torch.zeros_like(W)
    v = torch.zeros_like(W)
    grad = torch.zeros_like(W)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    bs = min(batch, n)
    scratch = torch.empty(binding.precond_train_scratch_bytes(bs), dtype=torch.uint8, device=dev)
    losses = []
    t = 0
    for ep in range(epochs):
        tot = 0.0
        nb = 0
        for off in range(0, n - bs + 1, bs):
            t += 1
            binding.precond_train_step(data[off:off + bs], nz, W, m, v, t, lr, scratch, grad, loss, apply=True)
            tot += float(loss.item())
            nb += 1
        losses.append(tot / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {losses[-1]:.6f}")
    return W, losses


def loss_and_grad(samples, nz, W):
    import torch
    dev = samples.device
    grad = torch.zeros_like(W)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    scratch = torch.empty(binding.precond_train_scratch_bytes(samples.shape[0]), dtype=torch.uint8, device=dev)
    binding.precond_train_step(samples.contiguous(), nz, W, None, None, 0, 0.0, scratch, grad, loss, apply=False)
    torch.cuda.synchronize()
    return float(loss.item()), grad


def evaluate(scene, W=None, T=3, I=2, **opts):
    """Fixed schedule with PCG on every sub-block; block-Jacobi when W is None,
    else the learned blocks.  Returns (total CG iterations, solve ms, final
    int_stats)."""
    solver = binding.RPBA_SOLVER_PCG_BJ if W is None else binding.RPBA_SOLVER_PCG_LEARNED
    p = binding.Problem(scene, precision=binding.RPBA_MIXED, solver=solver, **opts)
    if W is not None:
        p.set_precond_weights(W)
    p.set_timing(True)
    iters = 0.0
    for t in range(T):
        p.rpba_intersect()
        for s in range(I):
            bs = p.rpba_subblock_lm_step()
            p.sync()
            iters += float(bs[:, 3].sum().item())
        p.rpba_consensus()
    st = p.rpba_intersect()
    p.sync()
    ms = p.timing()["iterative_solve"]["ms"]
    return iters, ms, st.cpu().numpy()
