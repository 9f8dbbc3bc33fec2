"""The benchmark's command line: one GPU only, with a message otherwise."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_adjoint_units_from_hit_bits():
    """The adjoint's work units: with tau = 1 a blocked sample is neither
    drawn nor evaluated, and a pair with both rays blocked skips its Philox
    blocks; with tau < 1 every sample is drawn and every traced ray evaluated."""
    import types
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import bench
    # two pixels, spp 3 (one word each): pixel 0 pairs (both, light only,
    # none), pixel 1 pairs (bsdf only, both, none)
    words = np.array([[0b000111, 0b001110]], np.uint32)
    hb = torch.from_numpy(words.view(np.int32))
    stats = {"valid_pixels": 2, "rays_traced": 10, "rays_hit": 6}
    u = bench.adjoint_units(hb, stats, types.SimpleNamespace(tau=1.0, spp=3))
    assert u == {"pairs_drawn": 4, "light_draws": 3, "bsdf_draws": 3, "evaluated_directions": 4}
    u = bench.adjoint_units(hb, stats, types.SimpleNamespace(tau=0.5, spp=3))
    assert u == {"pairs_drawn": 6, "light_draws": 6, "bsdf_draws": 6, "evaluated_directions": 10}
