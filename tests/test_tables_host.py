"""The constant tables compiled into the library are exactly what the generator
writes: regenerating csrc/rlbm_tables.h (quadrature nodes and weights, separable
projector, g_nu Taylor tables, zeta values) reproduces the committed header byte
for byte, so no hand edit or stale table reaches the kernels."""
import os

from paper_1709_09073_amd import gen_tables

HEADER = os.path.join(os.path.dirname(gen_tables.__file__), "csrc", "rlbm_tables.h")


def test_generated_header_matches_committed(tmp_path):
    out = tmp_path / "rlbm_tables.h"
    gen_tables.emit(str(out))
    with open(HEADER) as fh:
        committed = fh.read()
    assert out.read_text() == committed
