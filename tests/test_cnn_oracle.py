"""Pins of the FP64 CPU reference of the scheduler CNN (oracle/cnn.py)."""
import numpy as np
import pytest
from scipy import ndimage

from oracle import cnn


def test_conv3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(4, 5, 6, 1))
    w = rng.normal(size=(1, 1, 27))
    y = cnn.conv3(x, w, np.zeros(1))[..., 0]
    ref = ndimage.correlate(x[..., 0], w[0, 0].reshape(3, 3, 3), mode="constant", cval=0.0)
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)


def test_conv3_channel_mixing_and_bias():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(3, 4, 4, 3))
    w = rng.normal(size=(2, 3, 27))
    b = np.array([0.5, -1.0])
    y = cnn.conv3(x, w, b)
    for co in range(2):
        ref = b[co] + sum(ndimage.correlate(x[..., ci], w[co, ci].reshape(3, 3, 3), mode="constant")
                          for ci in range(3))
        np.testing.assert_allclose(y[..., co], ref, rtol=1e-12, atol=1e-12)


def test_bce_matches_log_sigmoid_form():
    z = np.array([-30.0, -2.0, 0.0, 3.0, 25.0])
    t = np.array([0.0, 1.0, 1.0, 0.0, 1.0])
    m = np.array([1.0, 1.0, 0.0, 1.0, 1.0])
    loss, gz = cnn.bce_loss(z, t, m)
    sig = 1 / (1 + np.exp(-z))
    per = -(t * np.log(np.clip(sig, 1e-300, None)) + (1 - t) * np.log(np.clip(1 - sig, 1e-300, None)))
    assert abs(loss - (per * m).sum() / m.sum()) < 1e-9
    np.testing.assert_allclose(gz, (sig - t) * m / m.sum(), rtol=1e-12)


@pytest.mark.parametrize("dims", [(1, 5, 6), (3, 4, 3)])
def test_gradients_match_finite_differences(dims):
    C = 3
    rng = np.random.default_rng(2)
    p = rng.normal(scale=0.4, size=cnn.num_params(C))
    x = rng.normal(size=dims + (6,))
    t = (rng.uniform(size=dims) < 0.5).astype(float)
    m = (rng.uniform(size=dims) < 0.8).astype(float)
    _, g = cnn.loss_and_grad(p, x, t, m, C)
    h = 1e-6
    idx = rng.choice(p.size, size=40, replace=False)
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = cnn.loss_and_grad(p + e, x, t, m, C)
        lm, _ = cnn.loss_and_grad(p - e, x, t, m, C)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_param_count():
    assert cnn.num_params(16) == 16 * 3 * 27 + 16 + 16 * 16 * 27 + 16 + 16 * 27 + 1


def test_bf16_round_matches_torch_conversion():
    """bfloat16 rounding against torch's float32 -> bfloat16 cast (round to
    nearest even), on random values over many binades and on exact ties."""
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(7)
    x = (rng.normal(size=20000) * np.exp2(rng.integers(-40, 40, size=20000))).astype(np.float32)
    one = np.float32(1.0)
    ties = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, -(1 + 2.0 ** -8), 3 * 2.0 ** -9 + 2.0 ** -1,
                     255.5, 256.0 + 1.0, 0.0, -0.0, one], dtype=np.float32)
    for v in (x, ties):
        want = torch.from_numpy(v).to(torch.bfloat16).to(torch.float32).numpy()
        got = cnn.bf16_round(v)
        assert (got == want).all()
    # ties go to the even significand
    assert cnn.bf16_round(np.float32(1 + 2.0 ** -8)) == 1.0
    assert cnn.bf16_round(np.float32(1 + 3 * 2.0 ** -8)) == np.float32(1 + 2.0 ** -6)


def test_conv3_bf16_sums_in_the_stated_order():
    """One voxel summed by a plain float32 loop in the stated order (bias,
    taps, channels) gives every bit of conv3_bf16, on values where the order
    of float32 sums matters."""
    rng = np.random.default_rng(8)
    x = cnn.bf16_round((rng.normal(size=(3, 3, 4, 2)) * np.exp2(rng.integers(-12, 12, size=(3, 3, 4, 2))))
                       .astype(np.float32))
    w = cnn.bf16_round(rng.normal(size=(2, 2, 27)).astype(np.float32))
    b = rng.normal(size=2).astype(np.float32)
    y = cnn.conv3_bf16(x, w, b)
    for (z, yy, xx) in ((1, 1, 1), (0, 2, 3), (2, 0, 0)):
        for co in range(2):
            acc = np.float32(b[co])
            for t, (dz, dy, dx) in enumerate(cnn.TAPS):
                zz, y2, x2 = z + dz, yy + dy, xx + dx
                if 0 <= zz < 3 and 0 <= y2 < 3 and 0 <= x2 < 4:
                    for ci in range(2):
                        acc = np.float32(acc + np.float32(x[zz, y2, x2, ci] * w[co, ci, t]))
            assert acc == y[z, yy, xx, co]
    # and the order does matter here: a float64 sum rounded once differs somewhere
    exact = cnn.conv3(x.astype(np.float64), w.astype(np.float64), b.astype(np.float64))
    assert (exact.astype(np.float32) != y).any()


def test_forward_bf16_equals_the_exact_forward_on_exact_values():
    """With small-integer inputs and weights every float32 sum is exact, so
    the bf16 forward is the FP64 forward with each layer's output rounded to
    bfloat16 after its ReLU."""
    C = 3
    rng = np.random.default_rng(9)
    q = dict(w1=rng.integers(-2, 3, size=(C, 3, 27)), b1=rng.integers(-3, 4, size=C),
             w2=rng.integers(-1, 2, size=(C, C, 27)), b2=rng.integers(-3, 4, size=C),
             w3=rng.integers(-1, 2, size=(1, C, 27)), b3=rng.integers(-3, 4, size=1))
    q = {k: v.astype(np.float64) for k, v in q.items()}
    p = cnn.pack(q)
    x = rng.integers(-3, 4, size=(3, 5, 4, 6)).astype(np.float64)
    r = lambda a: cnn.bf16_round(a.astype(np.float32)).astype(np.float64)
    h1 = r(np.maximum(cnn.conv3(x[..., :3], q["w1"], q["b1"]), 0))
    h2 = r(np.maximum(cnn.conv3(h1, q["w2"], q["b2"]), 0))
    want = r(cnn.conv3(h2, q["w3"], q["b3"]))[..., 0]
    got = cnn.forward_bf16(p, x, C)
    assert (got == want).all()
    # the rounding is really taken: without it the logits differ
    z, _ = cnn.forward(p, x, C)
    assert (z != got).any()
