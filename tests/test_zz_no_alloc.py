"""The allocation-free training entry point (rlbm_mlp_train_noalloc) against the
allocating one (rlbm_mlp_train with a caller workspace), through the C ABI: the same
kernels in the same order, so the trained weights and the loss history must be
bit-identical, on two calls in a row (the second on fewer samples, reusing the
library's array) and with the size limit enforced."""
import ctypes

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rlbm.lib()
    return rlbm


def _data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-2.0, 1.0, n).astype(np.float32)
    t = (np.tanh(1.5 * x) + 0.2 * x * x).astype(np.float32)
    return torch.from_numpy(x).cuda(), torch.from_numpy(t).cuda()


def _init_net(rl, x, t):
    net = rl.GuessNet()
    noise = torch.from_numpy(np.random.default_rng(1).standard_normal(rl.MLP_HIDDEN + 1).astype(np.float32)).cuda()
    net.init(x, t, noise)
    return net


def test_noalloc_training_matches_workspace_training(rl):
    L = rl.lib()
    stream = torch.cuda.current_stream()
    s = ctypes.c_void_p(stream.cuda_stream)
    nmax = rl.MLP_NOALLOC_MAX
    for n, iters in ((nmax, 40), (5000, 25)):
        print(f"[no-alloc] n={n} iters={iters}", flush=True)
        x, t = _data(n, seed=n)
        ref = _init_net(rl, x, t)
        got = rl.GuessNet()
        got.w.copy_(ref.w)
        ref_loss = ref.train(x, t, iters=iters, lr=3e-3)
        loss = torch.empty(iters, dtype=torch.float32, device="cuda")
        rc = L.rlbm_mlp_train_noalloc(rl._ptr(got.w), rl._ptr(x), rl._ptr(t), n, iters, ctypes.c_float(3e-3),
                                      rl._ptr(loss), s)
        assert rc == rl.RLBM_OK
        torch.cuda.synchronize()
        assert torch.equal(got.w, ref.w), (n, (got.w - ref.w).abs().max().item())
        assert torch.equal(loss, ref_loss), n
        assert loss[-1].item() < loss[0].item()


def test_noalloc_rejects_too_many_samples(rl):
    L = rl.lib()
    x, t = _data(8, seed=0)
    w = torch.zeros(rl.MLP_FLOATS, dtype=torch.float32, device="cuda")
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.rlbm_mlp_train_noalloc(rl._ptr(w), rl._ptr(x), rl._ptr(t), rl.MLP_NOALLOC_MAX + 1, 1, ctypes.c_float(1e-3),
                                    None, s) \
        == rl.RLBM_EINVAL
    assert L.rlbm_mlp_train_noalloc(rl._ptr(w), rl._ptr(x), rl._ptr(t), 0, 1, ctypes.c_float(1e-3), None, s) \
        == rl.RLBM_EINVAL
