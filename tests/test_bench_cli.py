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
    """The adjoint's work units: the live samples (with tau = 1 those not
    blocked) are drawn and evaluated, a pair draws its first Philox block
    once; without tracing every sample is drawn."""
    import types
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    import bench
    # two pixels, spp 3 (one word each).  Live: pixel 0 pairs (both, light,
    # bsdf), pixel 1 pairs (both, both, none); blocked: pixel 0 pairs (both,
    # light, none), pixel 1 pairs (bsdf, none, none)
    live = torch.from_numpy(np.array([[0b100111, 0b001111]], np.uint32).view(np.int32))
    hb = torch.from_numpy(np.array([[0b000111, 0b000010]], np.uint32).view(np.int32))
    stats = {"valid_pixels": 2, "rays_traced": 10, "rays_hit": 6}
    u = bench.adjoint_units(hb, live, stats, types.SimpleNamespace(tau=1.0, spp=3))
    # needed: pixel 0 (none, none, bsdf), pixel 1 (light, both, none)
    assert u == {"pairs_drawn": 3, "light_draws": 2, "bsdf_draws": 2, "evaluated_directions": 4}
    u = bench.adjoint_units(hb, live, stats, types.SimpleNamespace(tau=0.5, spp=3))
    assert u == {"pairs_drawn": 5, "light_draws": 4, "bsdf_draws": 4, "evaluated_directions": 8}
    u = bench.adjoint_units(hb, None, stats, types.SimpleNamespace(tau=0.0, spp=3))
    assert u == {"pairs_drawn": 6, "light_draws": 6, "bsdf_draws": 6, "evaluated_directions": 10}
