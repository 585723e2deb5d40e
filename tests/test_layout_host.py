"""Host-side conversion between (72, ny, nx) populations and the library's buffer
layouts (no GPU): FP32/FP64 cell records per direction block, and the 16-bit
deviation buffer's views (SNORM16 codes, side values, half scales), as documented in
include/rlbm.h; and bench.py's naming of the kernel it measures."""
import os

import numpy as np
import pytest
import torch

from paper_1709_09073_amd import rlbm


@pytest.mark.parametrize("precision,dtype", [("fp32", torch.float32), ("fp64", torch.float64)])
def test_pack_unpack_round_trip(precision, dtype):
    nx, ny = 7, 5
    f = torch.randn(72, ny, nx, dtype=dtype, generator=torch.Generator().manual_seed(3))
    buf = rlbm.pack_populations(f, precision)
    assert buf.shape == (72 * nx * ny,)
    assert torch.equal(rlbm.unpack_populations(buf, precision, nx, ny), f)


@pytest.mark.parametrize("precision,dtype", [("fp32", torch.float32), ("fp64", torch.float64)])
def test_record_positions(precision, dtype):
    """Byte offsets of direction n, shell k, cell c = y nx + x, in elements."""
    nx, ny = 6, 4
    P = nx * ny
    f = torch.arange(72 * P, dtype=dtype).reshape(72, ny, nx)
    buf = rlbm.pack_populations(f, precision)
    for n, k, x, y in [(0, 0, 0, 0), (3, 5, 2, 3), (11, 3, 5, 1), (7, 4, 1, 2)]:
        c = y * nx + x
        if precision == "fp32":
            idx = n * 6 * P + (4 * c + k if k < 4 else 4 * P + 2 * c + (k - 4))
        else:
            idx = n * 6 * P + (k // 2) * 2 * P + 2 * c + (k % 2)
        assert buf[idx] == f[6 * n + k, y, x]


def test_dev16_views_layout():
    nx, ny = 5, 3
    P = nx * ny
    raw = torch.zeros(192 * P, dtype=torch.uint8)
    dev = torch.arange(72 * P, dtype=torch.int16) - 500
    side = torch.arange(8 * P, dtype=torch.float32) + 0.5
    scale = (torch.arange(6 * P, dtype=torch.float32) * 0.25).half()
    raw[:144 * P] = dev.view(torch.uint8)
    rec = raw[144 * P:].view(P, 48)
    rec[:, :32] = side.view(P, 8).contiguous().view(torch.uint8).view(P, 32)
    rec[:, 32:44] = scale.view(P, 6).contiguous().view(torch.uint8).view(P, 12)
    d, s, sc = rlbm.dev16_views(raw.view(torch.float32), nx, ny)
    for n, k, x, y in [(0, 0, 0, 0), (4, 5, 3, 2), (11, 1, 4, 1)]:
        c = y * nx + x
        assert d[6 * n + k, y, x] == dev[n * 6 * P + 6 * c + k]
    for j, x, y in [(0, 0, 0), (7, 4, 2), (5, 2, 1)]:
        c = y * nx + x
        assert s[j, y, x] == side[8 * c + j]
    for j, x, y in [(0, 0, 0), (5, 4, 2), (3, 2, 1)]:
        c = y * nx + x
        assert sc[j, y, x] == scale[6 * c + j]


def test_bench_names_the_step_kernel_and_ties_traffic_to_source_and_tile():
    """bench.py names the kernel its roofline describes (staged pull for FP32 and
    16-bit populations on tiles whose halo fits 512 cells, direct otherwise) and
    reports recorded HBM traffic only for the kernel source and tile it was taken on."""
    import json
    import bench
    fd = dict(stats="FD", bc=("open",) * 4)
    assert bench.step_kernel(fd, "fp32", 5, (64, 4), False) == "k_step_staged<1, float>"
    assert bench.step_kernel(fd, "dev16", 5, (16, 16), False) == "k_step_staged<1, Dev16>"
    assert bench.step_kernel(fd, "dev16", 5, (128, 2), False) == "k_step<1, Dev16, float, 5, false>"
    assert bench.step_kernel(fd, "fp64", 5, (32, 8), False) == "k_step<1, double, double, 5, false>"
    assert bench.step_kernel(dict(stats="MJ"), "fp32", 3, (32, 8), False) == "k_step<0, float, float, 3, false>"
    forced = dict(stats="MJ", force=(1e-8, 0.0), bc=("periodic", "periodic", "wall_neq", "wall_neq"))
    assert bench.step_kernel(forced, "fp32", 5, (64, 4), False) == "k_step<0, float, float, 5, true>"
    assert bench.step_kernel(dict(stats="MJ"), "fp32", 5, (32, 8), True).startswith("k_step_tiles<0, float, float>")
    from conftest import ROOT
    with open(os.path.join(ROOT, "profiles", "hbm_traffic.json")) as fh:
        rec = json.load(fh)
    for key, r in rec.items():
        workload, precision = key.split("/")
        tile = tuple(int(v) for v in r["tile"].split("x"))
        other = (256, 1) if tile != (256, 1) else (128, 2)
        if r["source_sha256"] == bench.kernel_source_hash():
            assert bench.recorded_traffic(workload, precision, tile) == r["traffic_bytes_per_launch"]
        assert bench.recorded_traffic(workload, precision, other) is None
