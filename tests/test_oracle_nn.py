"""Pins of the FP64 network reference (oracle/nn_ref.py): the forward
convolution against scipy's correlate, every backward pass and the whole
network's gradient against central finite differences."""
import numpy as np
import pytest
from scipy.signal import correlate

from oracle import nn_ref as R


def test_conv3x3_matches_scipy_correlate():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 5, 6, 3))
    w = rng.standard_normal((3, 3, 3, 4))
    b = rng.standard_normal(4)
    y = R.conv3x3(x, w, b)
    for n in range(2):
        for o in range(4):
            ref = b[o] + sum(correlate(x[n, :, :, k], w[:, :, k, o], mode="same", method="direct")
                             for k in range(3))
            assert np.abs(y[n, :, :, o] - ref).max() < 1e-12


def _fd(f, arr, idx, eps=1e-6):
    old = arr[idx]
    arr[idx] = old + eps
    fp = f()
    arr[idx] = old - eps
    fm = f()
    arr[idx] = old
    return (fp - fm) / (2 * eps)


def test_conv3x3_backward_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 4, 5, 2))
    w = rng.standard_normal((3, 3, 2, 3))
    b = rng.standard_normal(3)
    dy = rng.standard_normal((2, 4, 5, 3))
    dx, dw, db = R.conv3x3_backward(x, w, dy)
    loss = lambda: float((R.conv3x3(x, w, b) * dy).sum())
    for idx in [(0, 0, 0, 0), (1, 3, 4, 1), (0, 2, 1, 1)]:
        assert abs(_fd(loss, x, idx) - dx[idx]) < 1e-6
    for idx in [(0, 0, 0, 0), (2, 1, 1, 2), (1, 2, 0, 1)]:
        assert abs(_fd(loss, w, idx) - dw[idx]) < 1e-6
    for o in range(3):
        assert abs(_fd(loss, b, (o,)) - db[o]) < 1e-6


def test_pool_and_upsample_are_adjoint_pairs():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 6, 4, 3))
    y = rng.standard_normal((2, 3, 2, 3))
    assert abs((R.avgpool2(x) * y).sum() - (x * R.avgpool2_backward(y)).sum()) < 1e-12
    assert abs((R.upsample2(y) * x).sum() - (y * R.upsample2_backward(x)).sum()) < 1e-12
    assert np.allclose(R.avgpool2(np.ones((1, 4, 4, 1))), 1.0)


def test_mse_gradient():
    rng = np.random.default_rng(3)
    y = rng.standard_normal((1, 3, 3, 2))
    t = rng.standard_normal((1, 3, 3, 2))
    m = (rng.uniform(size=(1, 3, 3, 2)) > 0.3).astype(float)
    _, g = R.mse(y, t, m)
    for idx in [(0, 0, 0, 0), (0, 2, 1, 1)]:
        assert abs(_fd(lambda: R.mse(y, t, m)[0], y, idx) - g[idx]) < 1e-8


@pytest.mark.parametrize("chans", [(2, 3), (2, 3, 4)])
def test_unet_gradient_finite_differences(chans):
    rng = np.random.default_rng(4)
    net = R.UNet(cin=2, cout=2, chans=chans, rng=rng)
    for w, b in net.params:
        b += 0.1 * rng.standard_normal(b.shape)  # keep ReLUs away from 0
    x = rng.standard_normal((1, 8, 8, 2))
    t = rng.standard_normal((1, 8, 8, 2))
    m = np.ones_like(t)

    def loss():
        y, _ = net.forward(x)
        return R.mse(y, t, m)[0]

    y, tape = net.forward(x)
    _, dy = R.mse(y, t, m)
    grads, dx = net.backward(tape, dy)
    for k in (0, len(net.params) // 2, len(net.params) - 1):
        w, b = net.params[k]
        dw, db = grads[k]
        idx = tuple(int(i) for i in np.unravel_index(np.argmax(np.abs(dw)), dw.shape))
        assert abs(_fd(loss, w, idx) - dw[idx]) < 1e-6 * max(1.0, abs(dw[idx]))
        assert abs(_fd(loss, b, (0,)) - db[0]) < 1e-6 * max(1.0, abs(db[0]))
    idx = (0, 3, 4, 1)
    assert abs(_fd(loss, x, idx) - dx[idx]) < 1e-6
