"""Image loss of the composed image (appendix A): oracle pins on the CPU and
HIP parity on the GPU."""

import numpy as np
import pytest

from oracle import loss as OL

RNG = np.random.Generator(np.random.PCG64(1541))


def test_srgb_transfer_pins():
    # end points and the standard's decoding function as an inverse
    assert OL.srgb(0.0) == 0.0 and abs(OL.srgb(1.0) - 1.0) < 1e-15
    y = np.linspace(0.0, 1.0, 1001)
    enc = OL.srgb(y)
    dec = np.where(enc <= 0.04045, enc / 12.92, ((enc + 0.055) / 1.055) ** 2.4)
    assert np.allclose(dec, y, atol=2e-6)           # the standard's 2e-5 seam at 0.0031308
    assert np.all(np.diff(enc) > 0)
    # derivative against central differences away from the seam
    yy = np.concatenate([np.linspace(1e-4, 0.003, 50), np.linspace(0.004, 4.0, 200)])
    h = 1e-7
    fd = (OL.srgb(yy + h) - OL.srgb(yy - h)) / (2 * h)
    assert np.allclose(OL.srgb_d(yy), fd, rtol=1e-6)


def test_tonemap_derivative_and_clamp():
    x = np.concatenate([np.linspace(1e-3, 50, 300)])
    h = 1e-6
    fd = (OL.tonemap(x + h) - OL.tonemap(x - h)) / (2 * h)
    assert np.allclose(OL.tonemap_d(x), fd, rtol=1e-6)
    assert np.all(OL.tonemap(np.array([-1.0, -5.0])) == 0) and np.all(OL.tonemap_d(np.array([-1.0])) == 0)


def test_loss_hand_case():
    kd = np.full((3, 1), 0.5)
    cd = np.ones((3, 1))
    cs = np.zeros((3, 1))
    ref = np.full((3, 1), 0.5)
    li, ll, gkd, gcd, gcs = OL.image_loss(kd, cd, cs, ref, np.ones(1), w_light=0.15)
    assert li == 0.0 and np.all(gkd == 0)
    expect = abs(OL.srgb(np.log(2.0)) - OL.srgb(np.log(1.5)))
    assert abs(ll - expect) < 1e-15
    # gradient of the light term only: sign(+) * T'(1) / 3 * w
    assert np.allclose(gcs[:, 0], 0.15 / 3 * OL.tonemap_d(1.0))


def test_loss_hand_case_coloured_reference():
    """A reference whose channels differ: the image term is the mean over the
    three channels of |T(c) - T(ref)|, and the light term compares the mean
    of T(c_d + c_s) with the largest channel of T(ref), which is T(1) here,
    so it vanishes.  A second, masked pixel changes nothing and gets no
    gradient."""
    kd = np.array([[1.0, 0.3], [1.0, 0.3], [1.0, 0.3]])
    cd = np.ones((3, 2))
    cs = np.zeros((3, 2))
    ref = np.array([[0.2, 5.0], [0.5, 5.0], [1.0, 5.0]])
    li, ll, gkd, gcd, gcs = OL.image_loss(kd, cd, cs, ref, np.array([1, 0]), w_light=0.15)
    T = lambda x: OL.srgb(np.log(x + 1.0))  # noqa: E731
    assert abs(li - (abs(T(1.0) - T(0.2)) + abs(T(1.0) - T(0.5))) / 3) < 1e-15
    assert abs(ll) < 1e-15
    assert np.all(gkd[:, 1] == 0) and np.all(gcd[:, 1] == 0) and np.all(gcs[:, 1] == 0)


def test_loss_gradients_match_finite_differences():
    n = 40
    kd, cd, cs, ref = (RNG.uniform(0.05, 2.0, (3, n)) for _ in range(4))
    mask = RNG.random(n) < 0.8
    li, ll, gkd, gcd, gcs = OL.image_loss(kd, cd, cs, ref, mask)
    total = lambda a, b, c: (lambda r: r[0] + 0.15 * r[1])(OL.image_loss(a, b, c, ref, mask))  # noqa: E731
    h = 1e-7
    for arr, g in ((kd, gkd), (cd, gcd), (cs, gcs)):
        for (c, k) in [(0, 3), (1, 7), (2, 11), (0, 20), (2, 33)]:
            p = arr.copy(); p[c, k] += h
            m = arr.copy(); m[c, k] -= h
            args_p = [p if arr is x else x for x in (kd, cd, cs)]
            args_m = [m if arr is x else x for x in (kd, cd, cs)]
            fd = (total(*args_p) - total(*args_m)) / (2 * h)
            assert abs(fd - g[c, k]) < 1e-6 * max(1.0, abs(fd)), (c, k, fd, g[c, k])


@pytest.mark.gpu
@pytest.mark.parametrize("n", [1, 257, 100_003, 1_300_001])
def test_image_loss_gpu_parity(n):
    """n = 1, a ragged tail, several blocks, and more pixels than one pass of
    the grid-stride loop covers."""
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_03380_amd as M
    rng = np.random.Generator(np.random.PCG64(1541 + n))
    kd = rng.uniform(0.0, 1.0, (3, n)).astype(np.float32)
    cd = rng.lognormal(0, 1, (3, n)).astype(np.float32)
    cs = rng.lognormal(-1, 1, (3, n)).astype(np.float32)
    ref = rng.lognormal(0, 1, (3, n)).astype(np.float32)
    cs[:, :10] = -0.5                    # negative radiance: clamped
    cd[:, 10:20] = 1e-6                  # tiny radiance: log(1 + x) near 0, linear sRGB segment
    cs[:, 10:20] = 0.0
    mask = (rng.random(n) < 0.9).astype(np.uint8)
    mask[0] = 1
    print("image loss parity n=%d" % n, flush=True)
    t = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    loss, gkd, gcd, gcs = M.image_loss(t(kd), t(cd), t(cs), t(ref), t(mask))
    torch.cuda.synchronize()
    li, ll, okd, ocd, ocs = OL.image_loss(kd, cd, cs, ref, mask)
    lo = loss.cpu().numpy()
    assert abs(lo[0] - li) <= 1e-5 * li and abs(lo[1] - ll) <= 1e-5 * ll
    assert abs(lo[2] - (li + 0.15 * ll)) <= 1e-5 * (li + 0.15 * ll)
    # sign decisions taken in FP32 on the device: exclude near-ties
    c = kd.astype(np.float64) * cd + cs
    tie = np.abs(OL.tonemap(c) - OL.tonemap(ref)) < 1e-5
    lsum = cd.astype(np.float64) + cs
    tie_l = np.abs(OL.tonemap(lsum).mean(0) - OL.tonemap(ref).max(0)) < 1e-5
    ok = ~tie.any(0) & ~tie_l
    assert ok.mean() > 0.999 or n < 1000
    for g, o in ((gkd, okd), (gcd, ocd), (gcs, ocs)):
        gg = g.cpu().numpy().astype(np.float64)[:, ok]
        oo = o[:, ok]
        assert np.allclose(gg, oo, rtol=1e-4, atol=1e-6 * np.abs(oo).max())
    # deterministic
    loss2 = M.image_loss(t(kd), t(cd), t(cs), t(ref), t(mask))[0]
    assert torch.equal(loss, loss2)


@pytest.mark.gpu
def test_image_loss_autograd():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2206_03380_amd as M
    n = 5000
    rng = np.random.Generator(np.random.PCG64(77))
    kd, cd, cs, ref = (torch.from_numpy(rng.uniform(0.01, 2.0, (3, n)).astype(np.float32)).cuda() for _ in range(4))
    mask = torch.from_numpy((rng.random(n) < 0.9).astype(np.uint8)).cuda()
    kd.requires_grad_(True)
    cd.requires_grad_(True)
    cs.requires_grad_(True)
    L = M.ImageLoss.apply(kd, cd, cs, ref, mask, 0.15)
    (2.0 * L).backward()
    loss, gkd, gcd, gcs = M.image_loss(kd.detach(), cd.detach(), cs.detach(), ref, mask)
    assert torch.equal(L.detach(), loss[2])
    assert torch.equal(kd.grad, 2.0 * gkd) and torch.equal(cd.grad, 2.0 * gcd) and torch.equal(cs.grad, 2.0 * gcs)
