"""The allocation-free image loss (mcdi_image_loss_noalloc, static device
scratch) against the allocating entry point mcdi_image_loss, through the C
ABI: two calls in a row, the second on a smaller input, each equal bit for
bit to the allocating call on the same inputs (the same kernels, a
fixed-order reduction); sizes beyond the static scratch are refused before
anything is enqueued."""

import ctypes as C

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _inputs(n, seed):
    g = torch.Generator().manual_seed(seed)
    kd = torch.rand((3, n), generator=g)
    c_d = torch.exp(torch.randn((3, n), generator=g))
    c_s = torch.rand((3, n), generator=g) * 0.3
    ref = torch.exp(torch.randn((3, n), generator=g))
    c_d[0, :: 97] = -0.5          # negative lighting: clamped by the tonemap, no gradient
    mask = (torch.rand(n, generator=g) < 0.8).to(torch.uint8)
    return [t.cuda().contiguous() for t in (kd, c_d, c_s, ref)] + [mask.cuda()]


def _both(n, seed):
    import paper_2206_03380_amd as M
    kd, c_d, c_s, ref, mask = _inputs(n, seed)
    a = M.image_loss(kd, c_d, c_s, ref, mask, 0.15)
    b = M.image_loss(kd, c_d, c_s, ref, mask, 0.15, noalloc=True)
    torch.cuda.synchronize()
    return a, b


def test_noalloc_equals_allocating_entry_point():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    # first a large call, then a smaller one: the static scratch keeps the
    # first call's partial sums, which the second must not pick up
    for n, seed in ((1_300_001, 1), (5_003, 2)):
        print("noalloc image loss: n =", n, flush=True)
        a, b = _both(n, seed)
        for x, y in zip(a, b):
            assert torch.equal(x, y), (n, x.flatten()[:4], y.flatten()[:4])
        assert torch.isfinite(a[0]).all() and float(a[0][2]) > 0.0


def test_noalloc_rejects_sizes_beyond_the_static_scratch():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2206_03380_amd import _lib as L
    lib = L.lib()
    d = C.c_void_p(16)     # never dereferenced: validation fails first
    st = lib.mcdi_image_loss_noalloc(d, d, d, d, d, 600_000_000, C.c_float(0.15), d, None, None, None, None)
    assert st == L.MCDI_E_UNSUPPORTED
    assert b"static" in lib.mcdi_last_error()
    st = lib.mcdi_image_loss_noalloc(d, d, d, d, d, 0, C.c_float(0.15), d, None, None, None, None)
    assert st == L.MCDI_E_INVALID
