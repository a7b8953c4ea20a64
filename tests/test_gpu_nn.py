"""GPU tests of the warm-start network kernels (include/lbm_nn.h) against
plain PyTorch CPU references.

Operands the matrix cores read are rounded to BF16 on both sides, so the
remaining differences are FP32 accumulation order (and, for BF16 outputs,
one rounding of the result)."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from paper_2103_02119_amd import nn as K
from paper_2103_02119_amd import warmstart as WS

import nn_reference as REF

pytestmark = pytest.mark.gpu


def announce(*args):
    print("case:", *args, flush=True)


def r16(x):
    """Round to BF16 and back (float64)."""
    return torch.as_tensor(x).to(torch.bfloat16).to(torch.float64)


def dev_bf16(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.float32)).to(torch.bfloat16).cuda().reshape(-1)


def dev_f32(x):
    return torch.as_tensor(np.ascontiguousarray(x, np.float32)).cuda().reshape(-1)


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-30))


SHAPES = [(2, 16, 24, 16, 8, 40), (1, 10, 13, 8, 0, 32), (3, 8, 8, 32, 64, 64)]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3x3_forward(shape):
    n, h, w, c1, c2, cout = shape
    announce("conv fwd", shape)
    g = np.random.default_rng(1)
    x1 = g.standard_normal((n, h, w, c1))
    x2 = g.standard_normal((n, h, w, c2)) if c2 else None
    W = g.standard_normal((9 * (c1 + c2), cout)) * 0.2
    b = g.standard_normal(cout)
    wt = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    wd = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    K.lbm_nn_cast_weights(dev_f32(W), c1 + c2, cout, wt, wd)
    for relu in (False, True):
        y = torch.empty(n * h * w * cout, dtype=torch.bfloat16, device="cuda")
        K.lbm_nn_conv3x3_fwd(dev_bf16(x1), c1, dev_bf16(x2) if c2 else None, c2, n, h, w, wt,
                             dev_f32(b), cout, relu, y)
        x = np.concatenate([x1, x2], -1) if c2 else x1
        ref = F.conv2d(r16(x).permute(0, 3, 1, 2), r16(REF.w_torch(W, c1 + c2, cout)),
                       torch.as_tensor(np.float32(b).astype(np.float64)), padding=1)
        if relu:
            ref = F.relu(ref)
        ref = ref.permute(0, 2, 3, 1).numpy()
        got = y.float().cpu().numpy().reshape(ref.shape)
        # one BF16 rounding of the result (and FP32 accumulation order)
        assert np.all(np.abs(got - ref) <= 2.0 ** -7 * np.abs(ref) + 1e-5)


@pytest.mark.parametrize("shape", SHAPES)
def test_conv3x3_data_gradient(shape):
    n, h, w, c1, c2, cout = shape
    announce("conv dgrad", shape)
    g = np.random.default_rng(2)
    C = c1 + c2
    W = g.standard_normal((9 * C, cout)) * 0.2
    gy = g.standard_normal((n, h, w, cout))
    wt = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    wd = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    K.lbm_nn_cast_weights(dev_f32(W), C, cout, wt, wd)
    prior1 = g.standard_normal((n, h, w, c1))
    gx1 = dev_f32(prior1)
    gx2 = dev_f32(np.zeros((n, h, w, c2))) if c2 else None
    ref = torch.nn.grad.conv2d_input((n, C, h, w), r16(REF.w_torch(W, C, cout)),
                                     r16(gy).permute(0, 3, 1, 2), padding=1)
    ref = ref.permute(0, 2, 3, 1).numpy()
    for acc in (False, True):
        K.lbm_nn_conv3x3_dgrad(dev_f32(gy), n, h, w, cout, wd, gx1, c1, gx2, c2, acc)
        got1 = gx1.cpu().numpy().reshape(n, h, w, c1)
        expect1 = ref[..., :c1] + (ref[..., :c1] if acc else 0.0)
        assert rel(got1, expect1) < 1e-5
        if c2:
            assert rel(gx2.cpu().numpy().reshape(n, h, w, c2), ref[..., c1:] * (2 if acc else 1)) < 1e-5


@pytest.mark.parametrize("shape", SHAPES + [(4, 64, 128, 32, 0, 32)])
def test_conv3x3_weight_gradient(shape):
    n, h, w, c1, c2, cout = shape
    announce("conv wgrad", shape)
    g = np.random.default_rng(3)
    C = c1 + c2
    x1 = g.standard_normal((n, h, w, c1))
    x2 = g.standard_normal((n, h, w, c2)) if c2 else None
    gy = g.standard_normal((n, h, w, cout))
    gw = torch.empty(9 * C * cout, dtype=torch.float32, device="cuda")
    gb = torch.empty(cout, dtype=torch.float32, device="cuda")
    work = torch.empty(K.lbm_nn_conv3x3_wgrad_work(c1, c2, n, h, w, cout) // 4 + 1,
                       dtype=torch.float32, device="cuda")
    K.lbm_nn_conv3x3_wgrad(dev_bf16(x1), c1, dev_bf16(x2) if c2 else None, c2, n, h, w,
                           dev_f32(gy), cout, gw, gb, work)
    x = np.concatenate([x1, x2], -1) if c2 else x1
    ref = torch.nn.grad.conv2d_weight(r16(x).permute(0, 3, 1, 2), (cout, C, 3, 3),
                                      r16(gy).permute(0, 3, 1, 2), padding=1)
    ref = ref.permute(2, 3, 1, 0).reshape(9 * C, cout).numpy()
    assert rel(gw.cpu().numpy().reshape(9 * C, cout), ref) < 1e-5
    assert rel(gb.cpu().numpy(), np.float32(gy).astype(np.float64).sum((0, 1, 2))) < 1e-5


def test_pool_upsample_relu_head_mse_adam_and_casts():
    announce("elementwise")
    g = np.random.default_rng(4)
    n, h, w, c = 2, 8, 12, 16
    x = np.float32(r16(g.standard_normal((n, h, w, c))).numpy())
    y = torch.empty(n * h * w * c // 4, dtype=torch.bfloat16, device="cuda")
    K.lbm_nn_avgpool2_fwd(dev_bf16(x), n, h, w, c, y)
    ref = r16(x.reshape(n, h // 2, 2, w // 2, 2, c).mean((2, 4))).numpy()
    assert np.array_equal(y.float().cpu().numpy().reshape(ref.shape), ref)
    gy = g.standard_normal((n, h // 2, w // 2, c))
    gx = dev_f32(np.ones((n, h, w, c)))
    K.lbm_nn_avgpool2_bwd(dev_f32(gy), n, h, w, c, gx, True)
    ref = 1.0 + np.repeat(np.repeat(np.float32(gy), 2, 1), 2, 2) / 4
    assert rel(gx.cpu().numpy().reshape(ref.shape), ref) < 1e-7
    up = torch.empty(n * 4 * h * w * c, dtype=torch.bfloat16, device="cuda")
    K.lbm_nn_upsample2_fwd(dev_bf16(x), n, h, w, c, up)
    assert np.array_equal(up.float().cpu().numpy().reshape(n, 2 * h, 2 * w, c),
                          np.repeat(np.repeat(x, 2, 1), 2, 2))
    gu = np.float32(g.standard_normal((n, 2 * h, 2 * w, c)))
    gd = torch.empty(n * h * w * c, dtype=torch.float32, device="cuda")
    K.lbm_nn_upsample2_bwd(dev_f32(gu), n, h, w, c, gd)
    assert rel(gd.cpu().numpy().reshape(n, h, w, c),
               gu.reshape(n, h, 2, w, 2, c).astype(np.float64).sum((2, 4))) < 1e-6
    # ReLU backward from the BF16 output
    yv = np.float32(r16(g.standard_normal(1000)).numpy())
    gv = np.float32(g.standard_normal(1000))
    out = torch.empty(1000, dtype=torch.float32, device="cuda")
    K.lbm_nn_relu_bwd(dev_f32(gv), dev_bf16(yv), out)
    assert np.array_equal(out.cpu().numpy(), np.where(yv > 0, gv, 0.0).astype(np.float32))
    # 1x1 head
    m, cin, cout = 3000, 32, 3
    xh = np.float32(r16(g.standard_normal((m, cin))).numpy())
    wh, bh = np.float32(g.standard_normal((cin, cout))), np.float32(g.standard_normal(cout))
    yh = torch.empty(m * cout, dtype=torch.float32, device="cuda")
    K.lbm_nn_conv1x1_fwd(dev_bf16(xh), m, cin, dev_f32(wh), dev_f32(bh), cout, yh)
    assert rel(yh.cpu().numpy().reshape(m, cout), xh.astype(np.float64) @ wh + bh) < 1e-6
    gyh = np.float32(g.standard_normal((m, cout)))
    gxh = torch.empty(m * cin, dtype=torch.float32, device="cuda")
    gwh = torch.empty(cin * cout, dtype=torch.float32, device="cuda")
    gbh = torch.empty(cout, dtype=torch.float32, device="cuda")
    work = torch.empty(K.lbm_nn_conv1x1_work(m, cin, cout) // 4 + 1, dtype=torch.float32, device="cuda")
    K.lbm_nn_conv1x1_bwd(dev_bf16(xh), dev_f32(gyh), m, cin, dev_f32(wh), cout, gxh, gwh, gbh, work)
    assert rel(gxh.cpu().numpy().reshape(m, cin), gyh.astype(np.float64) @ wh.T) < 1e-6
    assert rel(gwh.cpu().numpy().reshape(cin, cout), xh.T.astype(np.float64) @ gyh) < 1e-5
    assert rel(gbh.cpu().numpy(), gyh.astype(np.float64).sum(0)) < 1e-5
    # masked MSE
    pred, tgt = np.float32(g.standard_normal((m, cout))), np.float32(g.standard_normal((m, cout)))
    fl = (g.random(m) > 0.3).astype(np.uint8)
    cw = np.float32([1.0, 2.0, 0.5])
    grad = torch.empty(m * cout, dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    work = torch.empty(K.lbm_nn_mse_work(m, cout) // 4 + 1, dtype=torch.float32, device="cuda")
    count = float(fl.sum())
    K.lbm_nn_mse(dev_f32(pred), dev_f32(tgt), torch.as_tensor(fl).cuda(), m, cout, dev_f32(cw),
                 count, grad, loss, work)
    d = (pred - tgt).astype(np.float64)
    assert abs(loss.item() - (cw * d ** 2 * fl[:, None]).sum() / count) < 1e-5 * loss.item()
    assert rel(grad.cpu().numpy().reshape(m, cout), 2 * cw * d * fl[:, None] / count) < 1e-6
    # Adam, two steps
    p0, g1, g2 = (np.float32(g.standard_normal(500)) for _ in range(3))
    p, mm, vv = dev_f32(p0), dev_f32(np.zeros(500)), dev_f32(np.zeros(500))
    K.lbm_nn_adam(p, dev_f32(g1), mm, vv, 1e-2, 0.9, 0.999, 1e-8, 1)
    K.lbm_nn_adam(p, dev_f32(g2), mm, vv, 1e-2, 0.9, 0.999, 1e-8, 2)
    m1 = 0.1 * g1.astype(np.float64)
    v1 = 0.001 * g1.astype(np.float64) ** 2
    q = p0 - 1e-2 * (m1 / 0.1) / (np.sqrt(v1 / 0.001) + 1e-8)
    m2 = 0.9 * m1 + 0.1 * g2
    v2 = 0.999 * v1 + 0.001 * g2.astype(np.float64) ** 2
    q = q - 1e-2 * (m2 / (1 - 0.81)) / (np.sqrt(v2 / (1 - 0.999 ** 2)) + 1e-8)
    assert rel(p.cpu().numpy(), q) < 1e-5
    # casts
    W = np.float32(g.standard_normal((9 * 24, 40)))
    wt = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    wd = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    K.lbm_nn_cast_weights(dev_f32(W), 24, 40, wt, wd)
    Wr = r16(W).numpy().reshape(3, 3, 24, 40)
    assert np.array_equal(wt.float().cpu().numpy().reshape(40, 9 * 24), Wr.reshape(9 * 24, 40).T)
    assert np.array_equal(wd.float().cpu().numpy().reshape(24, 9, 40), Wr.reshape(9, 24, 40).transpose(1, 0, 2))
    xb = torch.empty(W.size, dtype=torch.bfloat16, device="cuda")
    K.lbm_nn_cast_bf16(dev_f32(W), xb)
    assert np.array_equal(xb.float().cpu().numpy().reshape(W.shape), r16(W).numpy())


def _net_and_data(N=2, H=32, W=64, seed=11):
    net = WS.WarmStartNet(H=H, W=W, batch=N, seed=seed)
    g = np.random.default_rng(seed)
    X = np.stack([WS.input_planes((g.random((H, W)) > 0.9).astype(np.uint8),
                                  float(g.uniform(100, 5000)), float(g.choice([0.25, 0.5, 1.0])))
                  for _ in range(N)])
    T = np.float32(g.standard_normal((N, H, W, 3)) * 0.5)
    Fm = (X[..., 0] == 0).astype(np.uint8)
    return net, X, T, Fm


def test_whole_network_gradients_against_cpu_autograd():
    """Loss and every parameter gradient of the full encoder-decoder against
    FP64 CPU autograd with BF16 rounding at the same places; the GPU also
    rounds the backward's matrix-core operands (gradients) to BF16, which the
    reference does not, hence the per-tensor relative L2 bound."""
    announce("network gradients")
    net, X, T, Fm = _net_and_data()
    N, H, W = net.N, net.H, net.W
    count = float(Fm.sum())
    pred = net.forward(dev_f32(X))
    net.loss_grad(dev_f32(T), torch.as_tensor(Fm).cuda().reshape(-1), count,
                  torch.ones(3, dtype=torch.float32, device="cuda"))
    net.backward(net.gpred)
    torch.cuda.synchronize()
    st = net.state()
    params = {k: torch.tensor(np.float64(v), requires_grad=True) for k, v in st.items()}
    ref_pred = REF.forward(params, np.float64(X))
    loss = REF.masked_mse(ref_pred, np.float64(T), Fm, count)
    loss.backward()
    assert abs(net.loss.item() - loss.item()) < 2e-3 * loss.item()
    assert rel(pred.cpu().numpy().reshape(N, H, W, 3), ref_pred.detach().numpy()) < 2e-2
    grads = {cv.name: (cv.gW, cv.gb) for cv in net.layers()}
    grads["head"] = (net.hgW, net.hgb)
    for name, (gW, gb) in grads.items():
        for tag, gd in (("W", gW), ("b", gb)):
            ref = params[f"{name}.{tag}"].grad.numpy().reshape(-1)
            got = gd.cpu().numpy().reshape(-1).astype(np.float64)
            err = np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-30)
            cos = got @ ref / max(np.linalg.norm(got) * np.linalg.norm(ref), 1e-30)
            assert err < 3e-2 and cos > 0.999, (name, tag, err, cos)


def test_training_reduces_the_loss():
    announce("training")
    net, X, T, Fm = _net_and_data(N=4, seed=12)
    # a smooth target the network can fit
    H, W = net.H, net.W
    yy, xx = np.meshgrid(np.linspace(0, 1, H), np.linspace(0, 1, W), indexing="ij")
    T = np.float32(np.stack([np.sin(3 * xx) * np.cos(2 * yy) * (1 + 0.3 * k) for k in range(4)])[..., None]
                   * np.array([1.0, -0.5, 0.25]))
    tr = WS.Trainer(net, X, T, Fm)
    first = tr.epoch(2e-3)
    for _ in range(60):
        last = tr.epoch(2e-3)
    assert np.isfinite(last) and last < 0.2 * first, (first, last)
