"""The inversion-guess network on the GPU: forward/backward kernels against the FP64
oracle, deterministic gradients, training on pairs from the method's own runs, and
what the trained network gains over the fixed starting point."""
import numpy as np
import pytest
import torch

import workloads
from oracle import mlp as OM

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


def _random_net(rl, seed):
    rng = np.random.default_rng(seed)
    w = np.concatenate([[0.2, 1.7, -0.1, 0.6], rng.standard_normal(3 * rl.MLP_HIDDEN + 1)]).astype(np.float32)
    L = rng.uniform(-1.5, 0.5, 5000).astype(np.float32)
    t = (np.sin(2 * L) + 0.3 * L).astype(np.float32)
    return w, L, t


def test_forward_matches_oracle(rl):
    w, L, t = _random_net(rl, 3)
    net = rl.GuessNet()
    net.w.copy_(torch.from_numpy(w))
    y = net.predict(torch.from_numpy(L).cuda()).cpu().numpy()
    _, mu = OM.forward(w.astype(np.float64), L.astype(np.float64))
    np.testing.assert_allclose(y, mu, rtol=2e-5, atol=2e-5)


def test_gradient_matches_oracle_and_is_deterministic(rl):
    w, L, t = _random_net(rl, 4)
    net = rl.GuessNet()
    net.w.copy_(torch.from_numpy(w))
    xs, ts = torch.from_numpy(L).cuda(), torch.from_numpy(t).cuda()
    loss, grad = net.loss_grad(xs, ts)
    loss2, grad2 = net.loss_grad(xs, ts)
    assert torch.equal(grad, grad2) and torch.equal(loss, loss2)
    ref_loss, ref_grad = OM.loss_grad(w.astype(np.float64), L.astype(np.float64), t.astype(np.float64))
    g = grad.cpu().numpy().astype(np.float64)
    scale = np.abs(ref_grad).max()
    print(f"  grad max abs err / max |grad| = {np.abs(g - ref_grad).max() / scale:.2e}")
    assert np.abs(g - ref_grad).max() <= 1e-4 * scale
    assert abs(loss.item() - ref_loss) <= 1e-4 * ref_loss


def _hotspot_samples(rl, L=128, steps=40, seed=4):
    params, fields = workloads.hotspot_fd(L=L, seed=seed, sigma=L / 32)
    sim = rl.Sim(dict(params, precision="fp32"), {k: v.cuda() for k, v in fields.items()})
    sim.step(steps)
    x, t = sim.inversion_samples()
    sim.close()
    return x.reshape(-1), t.reshape(-1)


@pytest.fixture(scope="module")
def trained(rl):
    """Network trained on (ln r, ln z) pairs from a Fermi-Dirac hot-spot run."""
    x, t = _hotspot_samples(rl)
    net = rl.GuessNet()
    noise = torch.from_numpy(np.random.default_rng(0).standard_normal(rl.MLP_HIDDEN + 1).astype(np.float32)).cuda()
    net.init(x, t, noise)
    losses = net.train(x, t, iters=3000, lr=3e-3).cpu().numpy()
    return net, x, t, losses


def test_training_reduces_loss(rl, trained):
    net, x, t, losses = trained
    print(f"  loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    assert losses[-1] < 1e-3 * losses[0]
    mu = net.predict(x)
    err = (mu - t).abs().max().item()
    print(f"  max |mu_guess - ln z| on the training pairs: {err:.2e}")
    assert err < 0.05


def _run_fd(rl, guess, net, L=256, steps=20, precision="fp64"):
    params, fields = workloads.hotspot_fd(L=L, seed=7, sigma=L / 32)
    p = dict(params, precision=precision, collect_stats=True, guess=guess)
    if guess == "mlp":
        p["mlp"] = net.w
    sim = rl.Sim(p, {k: v.cuda() for k, v in fields.items()})
    sim.step(steps)
    it, solves = sim.inversion_stats()
    flds = {k: v.cpu().numpy() for k, v in sim.fields().items()}
    sim.close()
    return it / solves, flds


def test_network_guess_saves_newton_iterations(rl, trained):
    """Same converged states, fewer Newton iterations per inversion (held-out grid)."""
    net = trained[0]
    it_fixed, f_fixed = _run_fd(rl, "fixed", net)
    it_mlp, f_mlp = _run_fd(rl, "mlp", net)
    print(f"  Newton iterations per inversion: fixed start {it_fixed:.2f}, network start {it_mlp:.2f}")
    assert it_mlp < it_fixed - 1.0
    for k in ("n", "eps", "theta", "z", "ux", "uy"):
        err = np.abs(f_mlp[k] - f_fixed[k]).max() / max(np.abs(f_fixed[k]).max(), 1e-2)
        assert err < 1e-12, (k, err)
