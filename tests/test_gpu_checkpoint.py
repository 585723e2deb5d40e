"""Checkpoint and resume: the post-collision populations are the whole state, so a
run restored from a saved state continues bit for bit."""
import pytest
import torch

import workloads
from conftest import same_bits

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rl():
    from paper_1709_09073_amd import rlbm
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return rlbm


@pytest.mark.parametrize("stats,precision", [("FD", "fp32"), ("MJ", "fp64"), ("BE", "dev16")])
def test_resume_is_bitwise(rl, stats, precision):
    nx, ny, k = 48, 20, 37
    fields = {kk: v.cuda() for kk, v in workloads.smooth_random(nx, ny, seed=9, stats=stats).items()}
    params = dict(nx=nx, ny=ny, stats=stats, precision=precision, tau=0.9, bc=("open", "open", "periodic", "periodic"))
    print(f"[checkpoint] {stats} {precision} {nx}x{ny} {k}+{k} steps", flush=True)
    one = rl.Sim(params, fields)
    one.step(k)
    saved = one.state().clone()
    one.step(k)
    ref = one.state().clone()
    one.close()
    two = rl.Sim(params, fields)
    two.load_state(saved)
    two.step(k)
    got = two.state().clone()
    two.close()
    assert same_bits(got, ref)
