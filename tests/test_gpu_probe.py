"""The VALU issue probe behind the roofline's issue model (bench.py --valu-probe) runs on the GPU:
every kind returns a positive time and a cycle count per instruction, at a reduced size."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_valu_probe_small():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import bench
    print("valu probe: 256 blocks x 64 iterations", flush=True)
    out = bench.valu_probe(blocks=256, iters=64, reps=1)
    names = [r["probe"] for r in out["valu_probe"]]
    assert names[:6] == [n for n, _ in bench.VALU_PROBE_KINDS]
    for r in out["valu_probe"]:
        c = r["cycles_per_wave_instruction_per_simd_at_2.4GHz"]
        assert r["ms"] > 0 and math.isfinite(c) and c > 0, r
