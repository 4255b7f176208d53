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
