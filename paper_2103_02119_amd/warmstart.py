"""Learned warm start for steady lattice Boltzmann runs.

A 4-level convolutional encoder-decoder (32, 64, 128, 256 channels; skip
connections by channel concatenation; 2 x 2 average pooling down, nearest
upsampling up; two 3x3 ReLU convolutions per level and a 1x1 head) maps
  input  (per node): solid flag, Re, aspect ratio a, x / W, y / H (BF16)
  output (per node): (rho - 1) / s_rho, ux / U, uy / U           (FP32)
for lid-driven cavities with rectangular obstacles.  Its prediction is the
initial state of the lattice (lbm_set_fields); the lattice Boltzmann run
then converges from it, so the scheme itself decides the answer and the
network only shortens the way there.

Every forward, backward and optimizer step runs in the HIP kernels of
include/lbm_nn.h (3x3 convolutions on the matrix cores in BF16 with FP32
accumulation); torch only allocates the device buffers.
"""
from __future__ import annotations

import time

import numpy as np

from . import lbm as L
from . import nn as K

LEVELS = (32, 64, 128, 256)
CIN = 8          # solid, Re, a, x, y and three zero channels (3x3 layers need multiples of 8)
COUT = 3
RE_MID, RE_HALF = 2550.0, 2450.0   # Re in [100, 5000] -> [-1, 1]


class Conv3:
    """One 3x3 convolution + ReLU with its parameters and optimizer state."""

    def __init__(self, name, c1, c2, cout, torch, gen):
        self.name, self.c1, self.c2, self.cout = name, c1, c2, cout
        C = c1 + c2
        std = np.sqrt(2.0 / (9 * C))
        w = gen.normal(0.0, std, size=(9 * C, cout)).astype(np.float32)
        dev = "cuda"
        self.W = torch.from_numpy(w).to(dev)
        self.b = torch.zeros(cout, dtype=torch.float32, device=dev)
        self.gW = torch.zeros_like(self.W)
        self.gb = torch.zeros_like(self.b)
        self.mW, self.vW = torch.zeros_like(self.W), torch.zeros_like(self.W)
        self.mb, self.vb = torch.zeros_like(self.b), torch.zeros_like(self.b)
        self.WT = torch.empty(9 * C * cout, dtype=torch.bfloat16, device=dev)
        self.WD = torch.empty(9 * C * cout, dtype=torch.bfloat16, device=dev)

    def params(self):
        return [(self.W, self.gW, self.mW, self.vW), (self.b, self.gb, self.mb, self.vb)]


class WarmStartNet:
    """The encoder-decoder on device buffers for a fixed batch shape."""

    def __init__(self, H=128, W=256, batch=8, seed=2103, levels=LEVELS):
        import torch

        self.torch = torch
        if H % 8 or W % 8:
            raise ValueError("H and W must be multiples of 8 (three 2x poolings)")
        self.H, self.W, self.N = H, W, batch
        self.levels = levels
        gen = np.random.Generator(np.random.PCG64(seed))
        c = levels
        self.enc = [[Conv3("e0a", CIN, 0, c[0], torch, gen), Conv3("e0b", c[0], 0, c[0], torch, gen)]]
        for l in range(1, 4):
            self.enc.append([Conv3(f"e{l}a", c[l - 1], 0, c[l], torch, gen),
                             Conv3(f"e{l}b", c[l], 0, c[l], torch, gen)])
        self.dec = {}
        for l in (2, 1, 0):
            self.dec[l] = [Conv3(f"d{l}a", c[l], c[l + 1], c[l], torch, gen),
                           Conv3(f"d{l}b", c[l], 0, c[l], torch, gen)]
        hw = gen.normal(0.0, np.sqrt(1.0 / c[0]) * 0.1, size=(c[0], COUT)).astype(np.float32)
        self.hW = torch.from_numpy(hw).cuda()
        self.hb = torch.zeros(COUT, dtype=torch.float32, device="cuda")
        self.hgW, self.hgb = torch.zeros_like(self.hW), torch.zeros_like(self.hb)
        self.hmW, self.hvW = torch.zeros_like(self.hW), torch.zeros_like(self.hW)
        self.hmb, self.hvb = torch.zeros_like(self.hb), torch.zeros_like(self.hb)
        self.step_count = 0
        self._alloc()
        self.cast()

    # ------------------------------------------------------------ buffers
    def layers(self):
        out = [cv for lv in self.enc for cv in lv]
        for l in (2, 1, 0):
            out += self.dec[l]
        return out

    def _res(self, l):
        return self.H >> l, self.W >> l

    def _alloc(self):
        t = self.torch
        N, c = self.N, self.levels
        bf = dict(dtype=t.bfloat16, device="cuda")
        f32 = dict(dtype=t.float32, device="cuda")
        A, G = {}, {}

        def act(name, l, ch):
            h, w = self._res(l)
            A[name] = t.empty(N * h * w * ch, **bf)
            G[name] = t.empty(N * h * w * ch, **f32)

        act("x0", 0, CIN)
        for l in range(4):
            act(f"e{l}a", l, c[l])
            act(f"e{l}b", l, c[l])
            if l < 3:
                act(f"p{l}", l + 1, c[l])
        for l in (2, 1, 0):
            act(f"u{l}", l, c[l + 1])
            act(f"d{l}a", l, c[l])
            act(f"d{l}b", l, c[l])
        self.A, self.G = A, G
        M0 = N * self.H * self.W
        self.pred = t.empty(M0 * COUT, **f32)
        self.gpred = t.empty(M0 * COUT, **f32)
        self.gz = t.empty(M0 * max(c[0], 1) * 2, **f32)   # pre-activation gradient scratch
        work = 0
        for cv in self.layers():
            l = int(cv.name[1])
            h, w = self._res(l)
            work = max(work, K.lbm_nn_conv3x3_wgrad_work(cv.c1, cv.c2, N, h, w, cv.cout))
        work = max(work, K.lbm_nn_conv1x1_work(M0, c[0], COUT), K.lbm_nn_mse_work(M0, COUT))
        self.work = t.empty(work // 4 + 1, **f32)
        self.loss = t.zeros(1, **f32)

    def _gz(self, n):
        return self.gz[:n] if n <= self.gz.numel() else self._grow(n)

    def _grow(self, n):
        self.gz = self.torch.empty(n, dtype=self.torch.float32, device="cuda")
        return self.gz

    def cast(self):
        for cv in self.layers():
            K.lbm_nn_cast_weights(cv.W, cv.c1 + cv.c2, cv.cout, cv.WT, cv.WD)

    # ------------------------------------------------------------ forward
    def _conv(self, cv, x1, x2, y, l):
        h, w = self._res(l)
        K.lbm_nn_conv3x3_fwd(x1, cv.c1, x2, cv.c2, self.N, h, w, cv.WT, cv.b, cv.cout, True, y)

    def forward(self, x0_f32):
        """x0_f32: device FP32 [N * H * W * CIN]; returns the FP32 prediction
        [N * H * W * 3] (a view of an internal buffer)."""
        A, N = self.A, self.N
        K.lbm_nn_cast_bf16(x0_f32, A["x0"])
        prev = A["x0"]
        for l in range(4):
            a, b = self.enc[l]
            self._conv(a, prev, None, A[f"e{l}a"], l)
            self._conv(b, A[f"e{l}a"], None, A[f"e{l}b"], l)
            if l < 3:
                h, w = self._res(l)
                K.lbm_nn_avgpool2_fwd(A[f"e{l}b"], N, h, w, self.levels[l], A[f"p{l}"])
                prev = A[f"p{l}"]
        low = A["e3b"]
        for l in (2, 1, 0):
            h, w = self._res(l + 1)
            K.lbm_nn_upsample2_fwd(low, N, h, w, self.levels[l + 1], A[f"u{l}"])
            a, b = self.dec[l]
            self._conv(a, A[f"e{l}b"], A[f"u{l}"], A[f"d{l}a"], l)
            self._conv(b, A[f"d{l}a"], None, A[f"d{l}b"], l)
            low = A[f"d{l}b"]
        M0 = N * self.H * self.W
        K.lbm_nn_conv1x1_fwd(low, M0, self.levels[0], self.hW, self.hb, COUT, self.pred)
        return self.pred

    # ------------------------------------------------------------ backward
    def _conv_bwd(self, cv, x1, x2, y, gy, gx1, gx2, l, accumulate=False):
        """gy: gradient w.r.t. the layer's (post-ReLU) output y."""
        h, w = self._res(l)
        n = self.N * h * w * cv.cout
        gz = self._gz(n)
        K.lbm_nn_relu_bwd(gy[:n], y, gz)
        K.lbm_nn_conv3x3_wgrad(x1, cv.c1, x2, cv.c2, self.N, h, w, gz, cv.cout, cv.gW, cv.gb,
                               self.work)
        if gx1 is not None:
            K.lbm_nn_conv3x3_dgrad(gz, self.N, h, w, cv.cout, cv.WD, gx1, cv.c1, gx2, cv.c2,
                                   accumulate)

    def backward(self, gpred):
        """Parameter gradients of the loss whose gradient w.r.t. the
        prediction is gpred (device FP32 [N * H * W * 3]): the forward's steps
        in reverse, finest decoder level first, then the encoder from the
        bottom up (each skip's gradient is written by its decoder level and
        completed by the pooling path)."""
        A, G, N, c = self.A, self.G, self.N, self.levels
        M0 = N * self.H * self.W
        K.lbm_nn_conv1x1_bwd(A["d0b"], gpred, M0, c[0], self.hW, COUT, G["d0b"], self.hgW,
                             self.hgb, self.work)
        for l in (0, 1, 2):
            a, b = self.dec[l]
            self._conv_bwd(b, A[f"d{l}a"], None, A[f"d{l}b"], G[f"d{l}b"], G[f"d{l}a"], None, l)
            self._conv_bwd(a, A[f"e{l}b"], A[f"u{l}"], A[f"d{l}a"], G[f"d{l}a"], G[f"e{l}b"],
                           G[f"u{l}"], l)
            h, w = self._res(l + 1)
            below = "e3b" if l == 2 else f"d{l + 1}b"
            K.lbm_nn_upsample2_bwd(G[f"u{l}"], N, h, w, c[l + 1], G[below])
        for l in (3, 2, 1, 0):
            a, b = self.enc[l]
            self._conv_bwd(b, A[f"e{l}a"], None, A[f"e{l}b"], G[f"e{l}b"], G[f"e{l}a"], None, l)
            if l > 0:
                self._conv_bwd(a, A[f"p{l - 1}"], None, A[f"e{l}a"], G[f"e{l}a"], G[f"p{l - 1}"],
                               None, l)
                h, w = self._res(l - 1)
                K.lbm_nn_avgpool2_bwd(G[f"p{l - 1}"], N, h, w, c[l - 1], G[f"e{l - 1}b"], True)
            else:
                self._conv_bwd(a, A["x0"], None, A["e0a"], G["e0a"], None, None, 0)

    # ------------------------------------------------------------ loss and update
    def loss_grad(self, target, fluid, count, cw):
        """Masked MSE of the last forward against target (device FP32
        [N * H * W * 3]) over fluid pixels (device uint8 [N * H * W]);
        leaves d loss / d pred in self.gpred and the loss in self.loss."""
        M0 = self.N * self.H * self.W
        K.lbm_nn_mse(self.pred, target, fluid, M0, COUT, cw, count, self.gpred, self.loss,
                     self.work)
        return self.gpred

    def all_params(self):
        out = []
        for cv in self.layers():
            out += cv.params()
        out += [(self.hW, self.hgW, self.hmW, self.hvW), (self.hb, self.hgb, self.hmb, self.hvb)]
        return out

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8):
        self.step_count += 1
        for p, g, m, v in self.all_params():
            K.lbm_nn_adam(p, g, m, v, lr, b1, b2, eps, self.step_count)
        self.cast()

    # ------------------------------------------------------------ weights
    def state(self):
        out = {}
        for cv in self.layers():
            out[cv.name + ".W"] = cv.W.cpu().numpy()
            out[cv.name + ".b"] = cv.b.cpu().numpy()
        out["head.W"] = self.hW.cpu().numpy()
        out["head.b"] = self.hb.cpu().numpy()
        return out

    def load_state(self, st):
        t = self.torch
        for cv in self.layers():
            cv.W.copy_(t.from_numpy(np.asarray(st[cv.name + ".W"], np.float32)))
            cv.b.copy_(t.from_numpy(np.asarray(st[cv.name + ".b"], np.float32)))
        self.hW.copy_(t.from_numpy(np.asarray(st["head.W"], np.float32)))
        self.hb.copy_(t.from_numpy(np.asarray(st["head.b"], np.float32)))
        self.cast()


# ---------------------------------------------------------------- data

def input_planes(mask, Re, a):
    """FP32 [H, W, CIN] network input of one case: solid flag, normalized Re
    and aspect ratio, node coordinates in [0, 1], zero padding."""
    H, W = mask.shape
    x = np.zeros((H, W, CIN), np.float32)
    x[..., 0] = mask != 0
    x[..., 1] = (Re - RE_MID) / RE_HALF
    x[..., 2] = (a - 0.5) / 0.5
    x[..., 3] = (np.arange(W, dtype=np.float32)[None, :] + 0.5) / W
    x[..., 4] = (np.arange(H, dtype=np.float32)[:, None] + 0.5) / H
    return x


class Scales:
    """Output normalization: (rho - 1) / s_rho, u / U."""

    def __init__(self, s_rho, U):
        self.s_rho, self.U = float(s_rho), float(U)

    def encode(self, rho, ux, uy):
        return np.stack([(rho - 1.0) / self.s_rho, ux / self.U, uy / self.U], -1).astype(np.float32)

    def decode(self, y):
        return 1.0 + self.s_rho * y[..., 0], self.U * y[..., 1], self.U * y[..., 2]


def cavity_cases(params, nx, ny, U):
    """lbm_case list for dicts with keys Re, r (lid-driven cavities)."""
    from . import workloads as Wk
    return [Wk.cavity_case(nx, ny, p["r"], p["Re"], U) for p in params]


def generate(params, masks, nx, ny, U, precision, tol, check_every, max_steps, log=None):
    """Steady fields of cavities with obstacles from the batched solver.
    Returns (rho, ux, uy) arrays [n, ny, nx], the per-case steps (-1 blown up,
    -2 not converged at max_steps) and the wall time."""
    cases = cavity_cases(params, nx, ny, U)
    b = L.Batch(cases, precision=precision)
    for c, m in enumerate(masks):
        b.set_mask(c, m)
    b.autotune(2)
    t0 = time.perf_counter()
    steps = np.full(len(cases), -2, np.int64)
    done = 0
    while done < max_steps:
        n = min(max_steps - done, check_every * 20)
        got = b.run_to_steady(tol, check_every, n)
        for c in range(len(cases)):
            if steps[c] == -2 and got[c] != -2:
                steps[c] = got[c] + done if got[c] > 0 else got[c]
        done += n
        if log:
            log(f"generate: {done} steps, {int((steps > 0).sum())} converged, "
                f"{int((steps == -1).sum())} blew up, {time.perf_counter() - t0:.1f} s")
        if (steps != -2).all():
            break
    rho = np.empty((len(cases), ny, nx))
    ux, uy = np.empty_like(rho), np.empty_like(rho)
    for c in range(len(cases)):
        rho[c], ux[c], uy[c] = b.moments(c)
    wall = time.perf_counter() - t0
    b.close()
    return rho, ux, uy, steps, wall


class Trainer:
    """Keeps a dataset on the device and trains a WarmStartNet on it."""

    def __init__(self, net, X, T, F, seed=7):
        import torch

        self.net, self.torch = net, torch
        self.X = torch.from_numpy(np.ascontiguousarray(X, np.float32)).cuda()
        self.T = torch.from_numpy(np.ascontiguousarray(T, np.float32)).cuda()
        self.Fh = np.ascontiguousarray(F, np.uint8)
        self.F = torch.from_numpy(self.Fh).cuda()
        self.n = X.shape[0]
        self.gen = np.random.Generator(np.random.PCG64(seed))
        N, H, W = net.N, net.H, net.W
        self.xb = torch.empty(N * H * W * CIN, dtype=torch.float32, device="cuda")
        self.tb = torch.empty(N * H * W * COUT, dtype=torch.float32, device="cuda")
        self.fb = torch.empty(N * H * W, dtype=torch.uint8, device="cuda")
        self.cw = torch.ones(COUT, dtype=torch.float32, device="cuda")

    def _batch(self, idx):
        N, H, W = self.net.N, self.net.H, self.net.W
        for j, i in enumerate(idx):
            self.xb[j * H * W * CIN:(j + 1) * H * W * CIN].copy_(self.X[i].reshape(-1))
            self.tb[j * H * W * COUT:(j + 1) * H * W * COUT].copy_(self.T[i].reshape(-1))
            self.fb[j * H * W:(j + 1) * H * W].copy_(self.F[i].reshape(-1))
        return float(self.Fh[idx].sum())

    def epoch(self, lr):
        N = self.net.N
        perm = self.gen.permutation(self.n)
        losses = []
        for s in range(0, self.n - N + 1, N):
            idx = perm[s:s + N]
            count = self._batch(idx)
            self.net.forward(self.xb)
            self.net.loss_grad(self.tb, self.fb, count, self.cw)
            self.net.backward(self.net.gpred)
            self.net.adam(lr)
            losses.append(self.net.loss.clone())
        self.torch.cuda.synchronize()
        return float(self.torch.stack([v.clone() for v in losses]).mean()) if losses else float("nan")

    def evaluate(self, X, T, F):
        """Mean masked MSE on held-out data."""
        net = self.net
        N, H, W = net.N, net.H, net.W
        tot, cnt = 0.0, 0
        for s in range(0, X.shape[0] - N + 1, N):
            pred = predict_raw(net, X[s:s + N])
            d = (pred - T[s:s + N]) ** 2 * F[s:s + N, ..., None]
            tot += float(d.sum())
            cnt += int(F[s:s + N].sum())
        return tot / max(cnt, 1)


def predict_raw(net, X):
    """Network output [n, H, W, 3] for inputs X [n, H, W, CIN] (n <= batch)."""
    t = net.torch
    N, H, W = net.N, net.H, net.W
    n = X.shape[0]
    xb = np.zeros((N, H, W, CIN), np.float32)
    xb[:n] = X
    x = t.from_numpy(xb).cuda().reshape(-1)
    y = net.forward(x)
    return y.reshape(N, H, W, COUT)[:n].cpu().numpy()
