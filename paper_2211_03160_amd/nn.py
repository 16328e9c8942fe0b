"""The warm-start network on the GPU: a U-Net whose layers, gradients and
Adam updates all run in the BF16 MFMA kernels of include/lbm_nn.h.

PyTorch holds the tensors (device memory) and the stream; every arithmetic
step is a library call.  Activations and their gradients are BF16 (stored
as int16 tensors of raw bits), NHWC; weights are FP32 masters with BF16
copies in the [tap][cout][cin] order of the kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import lbm as _lbm

NN_EXPORTS = ["lbm_nn_conv3x3", "lbm_nn_conv3x3_flip", "lbm_nn_conv3x3_wgrad",
              "lbm_nn_relu_backward", "lbm_nn_avgpool2", "lbm_nn_avgpool2_backward",
              "lbm_nn_upsample2", "lbm_nn_upsample2_backward", "lbm_nn_copy_channels",
              "lbm_nn_mse", "lbm_nn_adam", "lbm_nn_to_bf16", "lbm_nn_to_f32",
              "lbm_nn_last_error"]

_ready = False


def lib():
    global _ready
    L = _lbm.lib()
    if not _ready:
        P, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        f32 = C.c_float
        L.lbm_nn_conv3x3.argtypes = [P, i32, i32, i32, i32, P, P, i32, i32, P, P]
        L.lbm_nn_conv3x3_flip.argtypes = [P, i32, i32, P, P]
        L.lbm_nn_conv3x3_wgrad.argtypes = [P, P, i32, i32, i32, i32, i32, P, i32, P, P, P]
        L.lbm_nn_relu_backward.argtypes = [P, P, P, i64, P]
        for n in ("lbm_nn_avgpool2", "lbm_nn_avgpool2_backward", "lbm_nn_upsample2",
                  "lbm_nn_upsample2_backward"):
            getattr(L, n).argtypes = [P, i32, i32, i32, i32, P, P]
        L.lbm_nn_copy_channels.argtypes = [P, i32, i32, P, i32, i32, i32, i64, i32, P]
        L.lbm_nn_mse.argtypes = [P, i32, P, P, i64, i32, C.c_double, P, P, P, P]
        L.lbm_nn_adam.argtypes = [P, P, P, P, i64, f32, f32, f32, f32, i32, P, P]
        L.lbm_nn_to_bf16.argtypes = [P, P, i64, P]
        L.lbm_nn_to_f32.argtypes = [P, P, i64, P]
        L.lbm_nn_last_error.restype = C.c_char_p
        for n in NN_EXPORTS[:-1]:
            getattr(L, n).restype = C.c_int32
        _ready = True
    return L


def _check(st):
    if st != 0:
        raise _lbm.LBMError(st, lib().lbm_nn_last_error().decode())


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def empty_bf16(*shape):
    import torch
    return torch.empty(*shape, dtype=torch.int16, device="cuda")


def to_bf16(x):
    """FP32 device tensor -> BF16 bits (int16 tensor of the same shape)."""
    import torch
    x = x.contiguous().float()
    y = torch.empty(x.shape, dtype=torch.int16, device="cuda")
    _check(lib().lbm_nn_to_bf16(_p(x), _p(y), x.numel(), _s()))
    return y


def to_f32(x):
    import torch
    y = torch.empty(x.shape, dtype=torch.float32, device="cuda")
    _check(lib().lbm_nn_to_f32(_p(x), _p(y), x.numel(), _s()))
    return y


def conv3x3(x, wt, bias, cout, relu):
    n, h, w, cin = x.shape
    y = empty_bf16(n, h, w, cout)
    _check(lib().lbm_nn_conv3x3(_p(x), n, h, w, cin, _p(wt), _p(bias), cout, int(relu), _p(y), _s()))
    return y


def conv3x3_flip(wt, cin, cout):
    wf = empty_bf16(9, cin, cout)
    _check(lib().lbm_nn_conv3x3_flip(_p(wt), cin, cout, _p(wf), _s()))
    return wf


def conv3x3_wgrad(x, dz, cout, dw, db):
    import torch
    n, h, w, cin = x.shape
    P = n * h * w
    chunks = int(max(1, min(64, P // 2048)))
    partial = torch.empty(chunks * 9 * cout * cin, dtype=torch.float32, device="cuda")
    _check(lib().lbm_nn_conv3x3_wgrad(_p(x), _p(dz), n, h, w, cin, cout, _p(partial), chunks,
                                      _p(dw), _p(db), _s()))


def relu_backward(y, dy):
    dz = empty_bf16(*y.shape)
    _check(lib().lbm_nn_relu_backward(_p(y), _p(dy), _p(dz), y.numel(), _s()))
    return dz


def avgpool2(x):
    n, h, w, c = x.shape
    y = empty_bf16(n, h // 2, w // 2, c)
    _check(lib().lbm_nn_avgpool2(_p(x), n, h, w, c, _p(y), _s()))
    return y


def avgpool2_backward(dy):
    n, h, w, c = dy.shape
    dx = empty_bf16(n, 2 * h, 2 * w, c)
    _check(lib().lbm_nn_avgpool2_backward(_p(dy), n, 2 * h, 2 * w, c, _p(dx), _s()))
    return dx


def upsample2(x):
    n, h, w, c = x.shape
    y = empty_bf16(n, 2 * h, 2 * w, c)
    _check(lib().lbm_nn_upsample2(_p(x), n, h, w, c, _p(y), _s()))
    return y


def upsample2_backward(dy):
    n, h2, w2, c = dy.shape
    dx = empty_bf16(n, h2 // 2, w2 // 2, c)
    _check(lib().lbm_nn_upsample2_backward(_p(dy), n, h2 // 2, w2 // 2, c, _p(dx), _s()))
    return dx


def copy_channels(src, soff, dst, doff, cc, accumulate=False):
    pixels = src.numel() // src.shape[-1]
    _check(lib().lbm_nn_copy_channels(_p(src), src.shape[-1], soff, _p(dst), dst.shape[-1], doff,
                                      cc, pixels, int(accumulate), _s()))


def concat(a, b):
    out = empty_bf16(*a.shape[:-1], a.shape[-1] + b.shape[-1])
    copy_channels(a, 0, out, 0, a.shape[-1])
    copy_channels(b, 0, out, a.shape[-1], b.shape[-1])
    return out


def mse(y, target, mask, with_grad=True):
    """Masked MSE of y (BF16 [..., cy]) against FP32 target/mask [..., used]."""
    import torch
    cy = y.shape[-1]
    used = target.shape[-1]
    pixels = y.numel() // cy
    count = float(mask.sum().item())
    dy = empty_bf16(*y.shape) if with_grad else None
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    scratch = torch.empty(1024, dtype=torch.float32, device="cuda")
    _check(lib().lbm_nn_mse(_p(y), cy, _p(target), _p(mask), pixels, used, count, _p(dy),
                            _p(loss), _p(scratch), _s()))
    return loss, dy


class UNet:
    """U-Net with len(chans) levels: two conv3x3 + ReLU per level, 2x2 mean
    pooling down, nearest upsampling + channel concatenation up, a final
    conv3x3 to `cout` channels.  Weights drawn from numpy's generator with
    the given seed (He-normal), biases zero."""

    def __init__(self, cin=16, cout=16, chans=(32, 64, 128, 256), seed=0):
        import torch
        self.cin, self.cout, self.chans = cin, cout, tuple(chans)
        rng = np.random.default_rng(seed)
        shapes = []
        prev = cin
        L = len(chans)
        for lvl in range(L):
            shapes += [(prev, chans[lvl]), (chans[lvl], chans[lvl])]
            prev = chans[lvl]
        for lvl in range(L - 2, -1, -1):
            shapes += [(prev + chans[lvl], chans[lvl]), (chans[lvl], chans[lvl])]
            prev = chans[lvl]
        shapes.append((prev, cout))
        self.layers = []
        for ci, co in shapes:
            w = rng.standard_normal((9, co, ci)).astype(np.float32) * np.float32(np.sqrt(2.0 / (9 * ci)))
            lay = {"ci": ci, "co": co,
                   "w": torch.from_numpy(w).cuda(), "b": torch.zeros(co, device="cuda")}
            lay["wbf"] = to_bf16(lay["w"])
            for k in ("mw", "vw", "gw"):
                lay[k] = torch.zeros_like(lay["w"])
            for k in ("mb", "vb", "gb"):
                lay[k] = torch.zeros_like(lay["b"])
            self.layers.append(lay)
        self.steps = 0

    def set_weights(self, ws, bs):
        """Load FP32 weights [9][co][ci] and biases (numpy) into every layer."""
        import torch
        for lay, w, b in zip(self.layers, ws, bs):
            lay["w"].copy_(torch.from_numpy(np.ascontiguousarray(w, np.float32)))
            lay["b"].copy_(torch.from_numpy(np.ascontiguousarray(b, np.float32)))
            lay["wbf"] = to_bf16(lay["w"])

    def forward(self, x):
        """x: BF16 [n, h, w, cin] (h, w divisible by 2^(levels-1)).
        Returns (y, tape)."""
        tape = []
        k = 0
        skips = []
        h = x
        L = len(self.chans)
        for lvl in range(L):
            if lvl > 0:
                h = avgpool2(h)
            for _ in range(2):
                lay = self.layers[k]
                y = conv3x3(h, lay["wbf"], lay["b"], lay["co"], True)
                tape.append((h, k, y))
                h, k = y, k + 1
            skips.append(h)
        for lvl in range(L - 2, -1, -1):
            h = concat(upsample2(h), skips[lvl])
            for _ in range(2):
                lay = self.layers[k]
                y = conv3x3(h, lay["wbf"], lay["b"], lay["co"], True)
                tape.append((h, k, y))
                h, k = y, k + 1
        lay = self.layers[k]
        y = conv3x3(h, lay["wbf"], lay["b"], lay["co"], False)
        tape.append((h, k, None))
        return y, tape

    def _layer_backward(self, h_in, k, dz, need_dx=True):
        lay = self.layers[k]
        conv3x3_wgrad(h_in, dz, lay["co"], lay["gw"], lay["gb"])
        if not need_dx:
            return None
        wf = conv3x3_flip(lay["wbf"], lay["ci"], lay["co"])
        return conv3x3(dz, wf, None, lay["ci"], False)

    def backward(self, tape, dy):
        """Fills every layer's gw, gb with the gradient of sum(dy * y)."""
        L = len(self.chans)
        ti = len(tape) - 1
        h_in, k, _ = tape[ti]
        dh = self._layer_backward(h_in, k, dy)
        ti -= 1
        dskips = [None] * L
        for lvl in range(0, L - 1):
            for _ in range(2):
                h_in, k, y = tape[ti]
                dh = self._layer_backward(h_in, k, relu_backward(y, dh))
                ti -= 1
            up_ch = dh.shape[-1] - self.chans[lvl]
            dskip = empty_bf16(*dh.shape[:-1], self.chans[lvl])
            copy_channels(dh, up_ch, dskip, 0, self.chans[lvl])
            dup = empty_bf16(*dh.shape[:-1], up_ch)
            copy_channels(dh, 0, dup, 0, up_ch)
            dskips[lvl] = dskip
            dh = upsample2_backward(dup)
        for lvl in range(L - 1, -1, -1):
            if lvl < L - 1:
                copy_channels(dskips[lvl], 0, dh, 0, dh.shape[-1], accumulate=True)
            for j in range(2):
                h_in, k, y = tape[ti]
                last = lvl == 0 and j == 1
                dh = self._layer_backward(h_in, k, relu_backward(y, dh), need_dx=not last)
                ti -= 1
            if lvl > 0:
                dh = avgpool2_backward(dh)

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.steps += 1
        for lay in self.layers:
            _check(lib().lbm_nn_adam(_p(lay["w"]), _p(lay["gw"]), _p(lay["mw"]), _p(lay["vw"]),
                                     lay["w"].numel(), lr, beta1, beta2, eps, self.steps,
                                     _p(lay["wbf"]), _s()))
            _check(lib().lbm_nn_adam(_p(lay["b"]), _p(lay["gb"]), _p(lay["mb"]), _p(lay["vb"]),
                                     lay["b"].numel(), lr, beta1, beta2, eps, self.steps, None, _s()))

    def state(self):
        return {"cin": self.cin, "cout": self.cout, "chans": list(self.chans), "steps": self.steps,
                "w": [l["w"].cpu().numpy() for l in self.layers],
                "b": [l["b"].cpu().numpy() for l in self.layers]}
