"""Plain PyTorch CPU reference of the warm-start network (FP64 autograd).

Used only by the tests.  It follows the network's definition directly
(torch.nn.functional conv2d / avg_pool2d / interpolate / relu) and rounds to
BF16 exactly where the GPU path stores BF16: every 3x3 weight, every
activation a 3x3 convolution or the head reads.  Gradients pass those
roundings straight through."""
import numpy as np
import torch
import torch.nn.functional as F

LEVELS = (32, 64, 128, 256)


def bf16(x):
    return x + (x.to(torch.bfloat16).to(x.dtype) - x).detach()


def w_torch(W, C, cout):
    """Our W[k = (3 i + j) C + ci][co] -> torch's [co][ci][i][j]."""
    return torch.as_tensor(np.asarray(W, np.float64)).reshape(3, 3, C, cout).permute(3, 2, 0, 1)


def conv3(x, W, b, relu=True):
    """x: [N][C][H][W] float64; W in our layout (torch tensor with grad)."""
    C = x.shape[1]
    cout = W.shape[1]
    wt = bf16(W.reshape(3, 3, C, cout).permute(3, 2, 0, 1))
    y = F.conv2d(bf16(x), wt, b, padding=1)
    return F.relu(y) if relu else y


def forward(params, x0, levels=LEVELS):
    """params: dict name -> torch float64 tensors (requires_grad as wanted);
    x0: [N][H][W][8] float64 numpy.  Returns the prediction [N][H][W][3]."""
    x = torch.as_tensor(x0).permute(0, 3, 1, 2)
    acts = {}
    h = x
    for l in range(4):
        h = bf16(conv3(h, params[f"e{l}a.W"], params[f"e{l}a.b"]))
        h = bf16(conv3(h, params[f"e{l}b.W"], params[f"e{l}b.b"]))
        acts[l] = h
        if l < 3:
            h = bf16(F.avg_pool2d(h, 2))
    low = acts[3]
    for l in (2, 1, 0):
        up = F.interpolate(low, scale_factor=2, mode="nearest")
        h = bf16(conv3(torch.cat([acts[l], up], 1), params[f"d{l}a.W"], params[f"d{l}a.b"]))
        low = bf16(conv3(h, params[f"d{l}b.W"], params[f"d{l}b.b"]))
    y = torch.einsum("nchw,co->nhwo", low, params["head.W"]) + params["head.b"]
    return y


def masked_mse(pred, target, fluid, count):
    t = torch.as_tensor(target)
    f = torch.as_tensor(fluid.astype(np.float64))[..., None]
    return (((pred - t) ** 2) * f).sum() / count
