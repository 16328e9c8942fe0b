"""FP64 CPU reference of the warm-start network's layers (test infrastructure).

TEST INFRASTRUCTURE ONLY: the GPU network kernels are checked against these
plain numpy definitions; nothing in the product path imports this module.

Tensors are NHWC (batch, height, width, channels).  Every backward pass is
the derivative of its forward pass written out by hand; the pins in
tests/test_oracle_nn.py check each one against central finite differences
and the forward convolution against scipy's correlate.

Layers:
  conv3x3(x, w, b)   y[n,i,j,o] = b[o] + sum_{a,c,k} w[a,c,k,o] x[n,i+a-1,j+c-1,k]
                     with zero padding; w is [3][3][Cin][Cout] here (the GPU
                     library keeps its own [tap][Cout][Cin] order)
  relu, avgpool2 (2x2 mean), upsample2 (nearest), concat (channels),
  masked MSE loss.
"""
from __future__ import annotations

import numpy as np


def conv3x3(x, w, b=None):
    n, h, wd, ci = x.shape
    co = w.shape[3]
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    y = np.zeros((n, h, wd, co))
    for a in range(3):
        for c in range(3):
            y += np.einsum("nijk,ko->nijo", xp[:, a:a + h, c:c + wd, :], w[a, c])
    if b is not None:
        y += b
    return y


def conv3x3_backward(x, w, dy):
    """Gradients (dx, dw, db) of sum(dy * conv3x3(x, w, b))."""
    n, h, wd, ci = x.shape
    xp = np.zeros((n, h + 2, wd + 2, ci))
    xp[:, 1:-1, 1:-1, :] = x
    dxp = np.zeros_like(xp)
    dw = np.zeros_like(w)
    for a in range(3):
        for c in range(3):
            dw[a, c] = np.einsum("nijk,nijo->ko", xp[:, a:a + h, c:c + wd, :], dy)
            dxp[:, a:a + h, c:c + wd, :] += np.einsum("nijo,ko->nijk", dy, w[a, c])
    db = dy.sum(axis=(0, 1, 2))
    return dxp[:, 1:-1, 1:-1, :], dw, db


def relu(x):
    return np.maximum(x, 0.0)


def relu_backward(y, dy):
    """y is the ReLU output; its positive entries pass the gradient."""
    return dy * (y > 0)


def avgpool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def avgpool2_backward(dy):
    return np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2) / 4.0


def upsample2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def upsample2_backward(dy):
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def mse(y, target, mask):
    """Mean over masked entries of (y - target)^2 and its gradient."""
    d = (y - target) * mask
    cnt = mask.sum()
    return float((d * d).sum() / cnt), 2.0 * d / cnt


class UNet:
    """The warm-start network in FP64: levels of two conv3x3 + ReLU, 2x2
    average pooling down, nearest upsampling and channel concatenation up,
    a final conv3x3 without activation.  chans[l] channels at level l."""

    def __init__(self, cin, cout, chans, rng):
        self.chans = list(chans)
        self.params = []  # (w, b) pairs in layer order
        L = len(chans)

        def add(ci, co):
            std = np.sqrt(2.0 / (9 * ci))
            self.params.append([rng.standard_normal((3, 3, ci, co)) * std, np.zeros(co)])

        prev = cin
        for lvl in range(L):
            add(prev, chans[lvl])
            add(chans[lvl], chans[lvl])
            prev = chans[lvl]
        for lvl in range(L - 2, -1, -1):
            add(prev + chans[lvl], chans[lvl])
            add(chans[lvl], chans[lvl])
            prev = chans[lvl]
        add(prev, cout)

    def forward(self, x):
        """Returns the output and the tape needed by backward."""
        tape = []
        P = self.params
        k = 0
        skips = []
        h = x
        L = len(self.chans)
        for lvl in range(L):
            if lvl > 0:
                h = avgpool2(h)
            for _ in range(2):
                y = relu(conv3x3(h, *P[k]))
                tape.append((h, k, y))
                h = y
                k += 1
            skips.append(h)
        for lvl in range(L - 2, -1, -1):
            h = np.concatenate([upsample2(h), skips[lvl]], axis=3)
            for _ in range(2):
                y = relu(conv3x3(h, *P[k]))
                tape.append((h, k, y))
                h = y
                k += 1
        y = conv3x3(h, *P[k])
        tape.append((h, k, None))
        return y, tape

    def backward(self, tape, dy):
        """Gradients [(dw, db)] of sum(dy * output), layer order."""
        grads = [None] * len(self.params)
        L = len(self.chans)
        P = self.params
        ti = len(tape) - 1
        h_in, k, _ = tape[ti]
        dh, dw, db = conv3x3_backward(h_in, P[k][0], dy)
        grads[k] = (dw, db)
        ti -= 1
        dskips = [None] * L
        for lvl in range(0, L - 1):
            for _ in range(2):
                h_in, k, y = tape[ti]
                dz = relu_backward(y, dh)
                dh, dw, db = conv3x3_backward(h_in, P[k][0], dz)
                grads[k] = (dw, db)
                ti -= 1
            # the concat input was [upsampled level lvl+1 | skip lvl]
            up_ch = dh.shape[3] - self.chans[lvl]
            dskips[lvl] = dh[..., up_ch:]
            dh = upsample2_backward(dh[..., :up_ch])
        for lvl in range(L - 1, -1, -1):
            if dskips[lvl] is not None and lvl < L - 1:
                dh = dh + dskips[lvl]
            for _ in range(2):
                h_in, k, y = tape[ti]
                dz = relu_backward(y, dh)
                dh, dw, db = conv3x3_backward(h_in, P[k][0], dz)
                grads[k] = (dw, db)
                ti -= 1
            if lvl > 0:
                dh = avgpool2_backward(dh)
        return grads, dh
