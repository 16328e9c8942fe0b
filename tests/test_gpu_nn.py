"""GPU network kernels (include/lbm_nn.h) against the FP64 reference of
oracle/nn_ref.py, on BF16-exact inputs and weights.

Tolerances: outputs stored as BF16 carry a relative rounding of 2^-8; FP32
accumulation adds ~1e-6 of the sum of |terms|.  Weight gradients are FP32
sums of exact BF16 products.  The whole-network gradient passes through ten
BF16 roundings of activations and gradients and is compared normwise."""
import numpy as np
import pytest

from oracle import nn_ref as R

pytestmark = pytest.mark.gpu

BF = 2.0 ** -8


def _bf(a):
    """Round an FP32/FP64 numpy array to BF16 values (nearest even)."""
    u = np.asarray(a, np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _dev_bf16(a):
    import torch
    from paper_2211_03160_amd import nn
    return nn.to_bf16(torch.from_numpy(np.asarray(a, np.float32)).cuda())


def _host(t):
    from paper_2211_03160_amd import nn
    return nn.to_f32(t).cpu().numpy().astype(np.float64)


def _w_gpu_to_ref(w):  # [9][co][ci] -> [3][3][ci][co]
    co, ci = w.shape[1], w.shape[2]
    return w.reshape(3, 3, co, ci).transpose(0, 1, 3, 2)


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 7, 9, 16, 16), (1, 16, 16, 32, 64), (3, 5, 4, 48, 32),
                                         (1, 17, 17, 16, 128)])
@pytest.mark.parametrize("relu", [0, 1])
def test_conv3x3_forward(n, h, w, ci, co, relu):
    import torch
    from paper_2211_03160_amd import nn
    rng = np.random.default_rng(ci + co + relu)
    x = _bf(rng.standard_normal((n, h, w, ci)))
    wt = _bf(rng.standard_normal((9, co, ci)) * 0.2)
    b = rng.standard_normal(co).astype(np.float32)
    y = nn.conv3x3(_dev_bf16(x), _dev_bf16(wt), torch.from_numpy(b).cuda(), co, relu)
    ref = R.conv3x3(x, _w_gpu_to_ref(wt), b.astype(np.float64))
    if relu:
        ref = R.relu(ref)
    scale = R.conv3x3(np.abs(x), np.abs(_w_gpu_to_ref(wt))) + np.abs(b)
    err = np.abs(_host(y) - ref)
    assert np.all(err <= BF * np.abs(ref) + 1e-5 * scale), err.max()


@pytest.mark.parametrize("n,h,w,ci,co", [(2, 6, 5, 16, 32), (1, 12, 12, 96, 32), (2, 8, 8, 64, 16),
                                         (4, 40, 40, 48, 48), (1, 20, 30, 32, 256)])
def test_conv3x3_gradients(n, h, w, ci, co):
    import torch
    from paper_2211_03160_amd import nn
    rng = np.random.default_rng(7 + ci)
    x = _bf(rng.standard_normal((n, h, w, ci)))
    wt = _bf(rng.standard_normal((9, co, ci)) * 0.2)
    dz = _bf(rng.standard_normal((n, h, w, co)))
    dx_ref, dw_ref, db_ref = R.conv3x3_backward(x, _w_gpu_to_ref(wt), dz)
    xd, wd, dzd = _dev_bf16(x), _dev_bf16(wt), _dev_bf16(dz)
    dx = nn.conv3x3(dzd, nn.conv3x3_flip(wd, ci, co), None, ci, False)
    scale_x = R.conv3x3_backward(np.abs(x), np.abs(_w_gpu_to_ref(wt)), np.abs(dz))[0]
    assert np.all(np.abs(_host(dx) - dx_ref) <= BF * np.abs(dx_ref) + 1e-5 * scale_x)
    dw = torch.zeros((9, co, ci), device="cuda")
    db = torch.zeros(co, device="cuda")
    nn.conv3x3_wgrad(xd, dzd, co, dw, db)
    dw_h = dw.cpu().numpy().reshape(3, 3, co, ci).transpose(0, 1, 3, 2)
    scale_w = R.conv3x3_backward(np.abs(x), np.abs(_w_gpu_to_ref(wt)), np.abs(dz))[1]
    assert np.all(np.abs(dw_h - dw_ref) <= 1e-5 * scale_w + 1e-6)
    assert np.all(np.abs(db.cpu().numpy() - db_ref) <= 1e-5 * np.abs(dz).sum(axis=(0, 1, 2)) + 1e-6)


def test_pool_upsample_relu_and_copies():
    from paper_2211_03160_amd import nn
    rng = np.random.default_rng(3)
    x = _bf(rng.standard_normal((2, 8, 6, 32)))
    xd = _dev_bf16(x)
    assert np.all(np.abs(_host(nn.avgpool2(xd)) - R.avgpool2(x)) <= BF * np.abs(R.avgpool2(x)) + 1e-30)
    y = _bf(rng.standard_normal((2, 4, 3, 32)))
    yd = _dev_bf16(y)
    assert np.array_equal(_host(nn.upsample2(yd)), R.upsample2(y))
    assert np.allclose(_host(nn.avgpool2_backward(yd)), R.avgpool2_backward(y), rtol=BF, atol=0)
    ub = _host(nn.upsample2_backward(xd))
    assert np.all(np.abs(ub - R.upsample2_backward(x)) <= BF * np.abs(R.upsample2_backward(x)) + 1e-30)
    r = R.relu(x)
    dz = _host(nn.relu_backward(_dev_bf16(r), _dev_bf16(y.repeat(2, 1).repeat(2, 2))))
    assert np.array_equal(dz, R.relu_backward(r, y.repeat(2, 1).repeat(2, 2)))
    c = nn.concat(xd, _dev_bf16(x[..., :16]))
    ch = _host(c)
    assert np.array_equal(ch[..., :32], x) and np.array_equal(ch[..., 32:], x[..., :16])


def test_mse_and_adam():
    import torch
    from paper_2211_03160_amd import nn
    rng = np.random.default_rng(5)
    y = _bf(rng.standard_normal((2, 6, 6, 16)))
    t = rng.standard_normal((2, 6, 6, 3)).astype(np.float32)
    m = (rng.uniform(size=(2, 6, 6, 3)) > 0.2).astype(np.float32)
    loss, dy = nn.mse(_dev_bf16(y), torch.from_numpy(t).cuda(), torch.from_numpy(m).cuda())
    ref, g = R.mse(y[..., :3], t.astype(np.float64), m.astype(np.float64))
    assert abs(float(loss.item()) - ref) <= 1e-5 * ref
    dyh = _host(dy)
    assert np.all(np.abs(dyh[..., :3] - g) <= BF * np.abs(g) + 1e-12) and not dyh[..., 3:].any()
    # Adam, two steps, against the update rule written out in numpy
    w = rng.standard_normal(1000).astype(np.float32)
    gs = [rng.standard_normal(1000).astype(np.float32) for _ in range(2)]
    wd = torch.from_numpy(w.copy()).cuda()
    md = torch.zeros_like(wd)
    vd = torch.zeros_like(wd)
    wm, mm, vm = w.astype(np.float64), np.zeros(1000), np.zeros(1000)
    for step, g in enumerate(gs, 1):
        gd = torch.from_numpy(g).cuda()
        nn._check(nn.lib().lbm_nn_adam(nn._p(wd), nn._p(gd), nn._p(md), nn._p(vd), 1000, 1e-2, 0.9, 0.999,
                                       1e-8, step, None, nn._s()))
        mm = 0.9 * mm + 0.1 * g
        vm = 0.999 * vm + 0.001 * g.astype(np.float64) ** 2
        wm = wm - 1e-2 * (mm / (1 - 0.9 ** step)) / (np.sqrt(vm / (1 - 0.999 ** step)) + 1e-8)
    assert np.abs(wd.cpu().numpy() - wm).max() < 1e-5


@pytest.mark.parametrize("chans", [(16, 32), (16, 32, 48)])
def test_unet_gradient_matches_reference(chans):
    """The GPU network's loss gradient for every layer against the FP64
    reference network with the same (BF16-exact) weights and input."""
    import torch
    from paper_2211_03160_amd import nn
    net = nn.UNet(cin=16, cout=16, chans=chans, seed=3)
    rng = np.random.default_rng(11)
    ws = [_bf(l["w"].cpu().numpy()) for l in net.layers]
    bs = [0.05 * rng.standard_normal(l["co"]).astype(np.float32) for l in net.layers]
    net.set_weights(ws, bs)
    ref = R.UNet(cin=16, cout=16, chans=chans, rng=np.random.default_rng(0))
    for k, (w, b) in enumerate(zip(ws, bs)):
        ref.params[k] = [_w_gpu_to_ref(w), b.astype(np.float64)]
    x = _bf(rng.standard_normal((2, 16, 16, 16)))
    t = rng.standard_normal((2, 16, 16, 3))
    m = np.ones_like(t)
    y, tape = net.forward(_dev_bf16(x))
    yr, tr = ref.forward(x)
    rel_y = np.linalg.norm(_host(y)[..., :3] - yr[..., :3]) / np.linalg.norm(yr[..., :3])
    loss, dy = nn.mse(y, torch.from_numpy(t.astype(np.float32)).cuda(),
                      torch.from_numpy(m.astype(np.float32)).cuda())
    net.backward(tape, dy)
    _, gref = R.mse(yr[..., :3], t, m)
    g16 = np.zeros_like(yr)
    g16[..., :3] = gref
    grads, _ = ref.backward(tr, g16)
    worst = 0.0
    for k, lay in enumerate(net.layers):
        gw = lay["gw"].cpu().numpy().reshape(3, 3, lay["co"], lay["ci"]).transpose(0, 1, 3, 2)
        rel = np.linalg.norm(gw - grads[k][0]) / np.linalg.norm(grads[k][0])
        relb = np.linalg.norm(lay["gb"].cpu().numpy() - grads[k][1]) / np.linalg.norm(grads[k][1])
        worst = max(worst, rel, relb)
    print(f"chans {chans}: forward rel {rel_y:.2e}, worst layer gradient rel {worst:.2e}", flush=True)
    assert rel_y < 2e-2
    assert worst < 5e-2
