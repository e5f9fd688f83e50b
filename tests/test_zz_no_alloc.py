"""rpba_precond_train_step_noalloc (the training step that allocates
nothing, its scratch in the library's own device array) against
rpba_precond_train_step (caller workspace), through the C ABI: same loss,
gradient and Adam update, bit for bit (same kernels, same fixed summation
order), on two calls in a row with the second on fewer samples; a sample
count above the maximum is rejected."""
import numpy as np
import pytest

from paper_1910_08138_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1910_08138_amd import binding
    binding.load_library()
    return binding


def _step(rp, fn, samples, nz, W0, t, scratch=None):
    import torch
    W = W0.clone()
    m = torch.full_like(W, 1e-3)
    v = torch.full_like(W, 1e-4)
    grad = torch.zeros_like(W)
    loss = torch.zeros(1, dtype=torch.float32, device=W.device)
    if scratch is None:
        fn(samples, nz, W, m, v, t, 1e-3, grad, loss, apply=True)
    else:
        fn(samples, nz, W, m, v, t, 1e-3, scratch, grad, loss, apply=True)
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in (loss, grad, W, m, v)]


def test_noalloc_training_step_matches_workspace_step(rp):
    import torch
    from paper_1910_08138_amd import precond
    nz = 3
    base = precond.harvest(scenes.config_scene(5, 0, small=True), nz=nz, T=2, I=2, seed=0)
    reps = rp.TRAIN_NOALLOC_MAX_SAMPLES // base.shape[0]
    samples = torch.cat([base] * reps, 0).contiguous()    # close to the maximum
    n = samples.shape[0]
    assert rp.TRAIN_NOALLOC_MAX_SAMPLES // 2 < n <= rp.TRAIN_NOALLOC_MAX_SAMPLES
    rng = np.random.default_rng(1)
    W0 = torch.as_tensor((rng.normal(size=rp.precond_num_params()) * 0.05).astype(np.float32), device="cuda")
    for t, rows in ((1, n), (2, n // 3 + 7)):      # the second call on fewer samples
        sub = samples[:rows].contiguous()
        scratch = torch.empty(rp.precond_train_scratch_bytes(rows), dtype=torch.uint8, device="cuda")
        ref = _step(rp, rp.precond_train_step, sub, nz, W0, t, scratch)
        got = _step(rp, rp.precond_train_step_noalloc, sub, nz, W0, t)
        for name, a, b in zip(("loss", "grad", "W", "m", "v"), got, ref):
            assert np.array_equal(a, b), (t, rows, name, np.abs(a - b).max())
        assert ref[0][0] > 0 and np.abs(ref[1]).max() > 0


def test_noalloc_rejects_too_many_samples(rp):
    import torch
    nz = 1
    stride = 26 + 36 + 12 * nz
    big = torch.zeros((rp.TRAIN_NOALLOC_MAX_SAMPLES + 1, stride), dtype=torch.float32, device="cuda")
    W = torch.zeros(rp.precond_num_params(), dtype=torch.float32, device="cuda")
    g = torch.zeros_like(W)
    with pytest.raises(rp.RpbaError, match="exceed the maximum of 8192"):
        rp.precond_train_step_noalloc(big, nz, W, None, None, 0, 0.0, g, None, apply=False)
