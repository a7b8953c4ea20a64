"""Learned warm start for steady lattice Boltzmann runs.

A 4-level convolutional encoder-decoder (32, 64, 128, 256 channels; skip
connections by channel concatenation; 2 x 2 average pooling down, nearest
upsampling up; two 3x3 ReLU convolutions per level and a 1x1 head) maps
  input  (per node): solid flag, Re, aspect ratio a, x / W, y / H,
                     distance to the nearest solid or wall         (BF16)
  output (per node): (rho - 1) cs2 / U^2, ux / U, uy / U          (FP32)
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
CIN = 8          # solid, Re, a, x, y, wall distance and two zero channels (multiples of 8)
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

def wall_distance(mask, a):
    """Distance (lattice x units) from each node to the nearest solid node or
    cavity wall (walls half a node beyond the outer rows and columns)."""
    from scipy.ndimage import distance_transform_edt

    H, W = mask.shape
    fluid = np.zeros((H + 2, W + 2), bool)
    fluid[1:-1, 1:-1] = mask == 0
    d = distance_transform_edt(fluid, sampling=(a, 1.0))[1:-1, 1:-1]
    # a wall lies half a spacing from the outer nodes, not a full one
    return np.maximum(d - 0.5 * min(a, 1.0), 0.0) * (mask == 0)


def input_planes(mask, Re, a):
    """FP32 [H, W, CIN] network input of one case: solid flag, normalized Re
    and aspect ratio, node coordinates in [0, 1], distance to the nearest
    solid or wall (/32), zero padding."""
    H, W = mask.shape
    x = np.zeros((H, W, CIN), np.float32)
    x[..., 0] = mask != 0
    x[..., 1] = (Re - RE_MID) / RE_HALF
    x[..., 2] = (a - 0.5) / 0.5
    x[..., 3] = (np.arange(W, dtype=np.float32)[None, :] + 0.5) / W
    x[..., 4] = (np.arange(H, dtype=np.float32)[:, None] + 0.5) / H
    x[..., 5] = wall_distance(mask, a) / 32.0
    return x


class Scales:
    """Output normalization: the pressure coefficient (rho - 1) cs2 / U^2
    (p = rho cs2) and u / U; cs2 differs between aspect ratios, the pressure
    coefficient does not."""

    def __init__(self, U):
        self.U = float(U)

    def encode(self, rho, ux, uy, cs2):
        c = np.asarray(cs2, np.float64).reshape(-1, *([1] * (rho.ndim - 1))) if rho.ndim == 3 else cs2
        return np.stack([(rho - 1.0) * c / self.U ** 2, ux / self.U, uy / self.U], -1).astype(np.float32)

    def decode(self, y, cs2):
        return 1.0 + y[..., 0] * self.U ** 2 / cs2, self.U * y[..., 1], self.U * y[..., 2]


def cavity_cases(params, nx, ny, U):
    """lbm_case list for dicts with keys Re, r (lid-driven cavities, the
    sound speed of the paper's cavity runs)."""
    from . import workloads as Wk
    return [Wk.cavity_case(nx, ny, p["r"], p["Re"], U, cs2=Wk.cavity_cs2(p["r"])) for p in params]


def generate(params, masks, nx, ny, U, precision, tol, check_every, max_steps, log=None):
    """Steady fields of cavities with obstacles from the batched solver.
    Returns (rho, ux, uy) arrays [n, ny, nx], the per-case steps (-1 blown up,
    -2 not converged at max_steps) and the wall time."""
    cases = cavity_cases(params, nx, ny, U)
    t0 = time.perf_counter()
    b = L.Batch(cases, precision=precision)
    for c, m in enumerate(masks):
        b.set_mask(c, m)
    b.autotune(2)
    if log:
        log(f"generate: {len(cases)} cases set up in {time.perf_counter() - t0:.1f} s, "
            f"launch shape {b.launch_shape()}")
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


# ---------------------------------------------------------------- pipeline

def _log_default(msg):
    print(msg, flush=True)


def build_dataset(params, nx=256, ny=128, U=0.05, precision=L.LBM_FP32_DEV, tol=2e-6,
                  check_every=1000, max_steps=150_000, log=_log_default):
    """Steady cavity fields for the given case parameters (dicts Re, r,
    mask_seed) from the batched solver; keeps the converged cases.  Returns
    (X [n, ny, nx, CIN], fields (rho, ux, uy) [n, ny, nx] each, masks, kept
    parameter dicts, generation info)."""
    from . import inputs as I

    masks = [I.cavity_obstacles(nx, ny, p["mask_seed"]) for p in params]
    rho, ux, uy, steps, wall = generate(params, masks, nx, ny, U, precision, tol, check_every,
                                        max_steps, log=log)
    keep = np.nonzero(steps > 0)[0]
    X = np.stack([input_planes(masks[i], params[i]["Re"], params[i]["r"]) for i in keep])
    info = dict(cases=len(params), converged=int(len(keep)), blew_up=int((steps == -1).sum()),
                not_converged=int((steps == -2).sum()), seconds=round(wall, 2), tol=tol,
                median_steps=int(np.median(steps[keep])) if len(keep) else None)
    return X, (rho[keep], ux[keep], uy[keep]), [masks[i] for i in keep], [params[i] for i in keep], info


def train(net, X, T, F, epochs, lr_max=1e-3, lr_min=2e-5, val=None, channel_weights=(0.25, 1, 1),
          seconds=None, log=_log_default):
    """Adam with a cosine learning-rate schedule; returns the loss history.
    The pressure channel is weighted down: an initial density error costs
    the lattice run little, a velocity error much more.  With `seconds` the
    epoch count is cut to what fits that time, judged from the first epoch."""
    tr = Trainer(net, X, T, F)
    tr.cw.copy_(net.torch.tensor(channel_weights, dtype=net.torch.float32))
    hist = []
    t0 = time.perf_counter()
    e = 0
    while e < epochs:
        if seconds and e == 1:
            per = time.perf_counter() - t0
            epochs = max(2, min(epochs, int(seconds / per)))
            log(f"train: {per:.1f} s per epoch, {epochs} epochs fit {seconds:.0f} s")
        lr = lr_min + 0.5 * (lr_max - lr_min) * (1 + np.cos(np.pi * e / max(epochs - 1, 1)))
        loss = tr.epoch(lr)
        rec = dict(epoch=e, lr=float(lr), loss=loss)
        if val is not None and (e % 10 == 9 or e == epochs - 1):
            rec["val"] = tr.evaluate(*val)
        hist.append(rec)
        if e % 10 == 9 or e == epochs - 1:
            log(f"train: epoch {e + 1}/{epochs} loss {loss:.4g}"
                + (f" val {rec['val']:.4g}" if "val" in rec else "") + f" {time.perf_counter() - t0:.1f} s")
        e += 1
    return hist, time.perf_counter() - t0


def predict_fields(net, scales, masks, params):
    """Predicted (rho, ux, uy) [ny, nx] per case; solid nodes at rest."""
    out = []
    X = np.stack([input_planes(m, p["Re"], p["r"]) for m, p in zip(masks, params)])
    for s in range(0, len(X), net.N):
        y = predict_raw(net, X[s:s + net.N])
        from . import workloads as Wk
        for j in range(y.shape[0]):
            rho, ux, uy = scales.decode(y[j].astype(np.float64), Wk.cavity_cs2(params[s + j]["r"]))
            solid = masks[s + j] != 0
            rho[solid], ux[solid], uy[solid] = 1.0, 0.0, 0.0
            out.append((rho, ux, uy))
    return out


SETTLE_STEPS = 50   # steps before the smoothing step of a start from fields
CONSISTENT_STEPS = 100  # steps of the consistent start (velocity held at the prediction)


MODES = ("cold", "cold+smooth", "warm", "warm+smooth")
# further starts that warm_vs_cold knows (not run by default)
EXTRA_MODES = ("consistent", "consistent+smooth")


def consistent_start(b, pred, masks, steps=CONSISTENT_STEPS):
    """A start consistent with the predicted velocity in the manner of Mei,
    Luo, Lallemand and d'Humieres (Comput. Fluids 2006): from the predicted
    fields at equilibrium, take `steps` steps, after each one moving every
    fluid node's equilibrium part back to the predicted velocity at the
    node's current density, f <- f + feq(rho, u_pred) - feq(rho, u); the
    density and the non-equilibrium parts develop, the velocity stays.
    Equilibria come from the library (lbm_batch_set_fields), so this runs
    through the public API only."""
    for _ in range(steps):
        b.step(1)
        for c, (_, ux_p, uy_p) in enumerate(pred):
            rho, ux, uy = b.moments(c)
            f = b.get_populations(c)
            b.set_fields(c, rho, ux, uy)
            f_now = b.get_populations(c)
            b.set_fields(c, rho, ux_p, uy_p)
            f_pred = b.get_populations(c)
            fluid = (masks[c] == 0)[None]
            b.set_populations(c, np.where(fluid, f + (f_pred - f_now), f))


def _compare(res, ref, mode):
    """Steps of `mode` against `ref` over the cases both reached."""
    both = (res[ref]["steps"] > 0) & (res[mode]["steps"] > 0)
    sc, sw = res[ref]["steps"][both], res[mode]["steps"][both]
    return dict(compared=int(both.sum()), steps_total=int(sw.sum()),
                ref_steps_total=int(sc.sum()),
                step_speedup_total=float(sc.sum() / max(sw.sum(), 1)),
                step_speedup_median=float(np.median(sc / sw)) if len(sc) else None,
                step_speedup_range=[float((sc / sw).min()), float((sc / sw).max())]
                if len(sc) else None)


def warm_vs_cold(net, scales, params, nx=256, ny=128, U=0.05, tol=1e-8, check_every=1000,
                 max_steps=400_000, modes=None, log=_log_default):
    """Steps and wall time to a per-step residual of tol (FP64; the plain
    lattice Boltzmann scheme decides convergence) for the same cases started
      cold        from rest,
      cold+smooth from rest, with one smoothing step after SETTLE_STEPS,
      warm        from the network's prediction (lbm_set_fields),
      warm+smooth from the prediction, with the smoothing step,
      consistent, consistent+smooth  (on request) from the prediction made
                  consistent by consistent_start, without and with the
                  smoothing step.
    An equilibrium start from any field that is not the scheme's own steady
    state excites the undamped staggered-momentum mode of the D2Q9 streaming;
    the smoothing step (mean of two consecutive states) removes it.  Each
    variant advances all cases as one batch."""
    import torch

    from . import inputs as I

    masks = [I.cavity_obstacles(nx, ny, p["mask_seed"]) for p in params]
    res = {}
    for mode in (modes or MODES):
        b = L.Batch(cavity_cases(params, nx, ny, U), precision=L.LBM_FP64)
        for c, m in enumerate(masks):
            b.set_mask(c, m)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        extra = 0
        if mode.startswith(("warm", "consistent")):
            pred = predict_fields(net, scales, masks, params)
            for c, (rho, ux, uy) in enumerate(pred):
                b.set_fields(c, rho, ux, uy)
            if mode.startswith("consistent"):
                consistent_start(b, pred, masks)
                extra += CONSISTENT_STEPS
        t_inf = time.perf_counter() - t0
        if mode.endswith("smooth"):
            b.step(SETTLE_STEPS)
            b.smooth_step()
            extra += SETTLE_STEPS + 1
        steps = b.run_to_steady(tol, check_every, max_steps)
        steps = np.where(steps > 0, steps + extra, steps)
        wall = time.perf_counter() - t0
        b.close()
        res[mode] = dict(steps=steps, seconds=wall, inference_seconds=t_inf)
        log(f"{mode}: {int((steps > 0).sum())}/{len(params)} reached {tol:g} in {wall:.1f} s")
    out = dict(tol=tol, cases=len(params), settle_steps=SETTLE_STEPS, check_every=check_every,
               max_steps=max_steps)
    for mode, r in res.items():
        out[mode] = dict(reached=int((r["steps"] > 0).sum()), seconds=round(r["seconds"], 3))
        if mode.startswith("warm"):
            out["inference_seconds"] = round(r["inference_seconds"], 3)
        if mode.startswith("consistent"):
            out[mode]["start_seconds"] = round(r["inference_seconds"], 3)
    # against the plain scheme from rest
    if "cold" in res:
        for mode in res:
            if mode != "cold":
                out[mode]["vs_cold"] = _compare(res, "cold", mode)
    # the network's own gain: the same start-up treatment with and without
    # it; the consistent start against the equilibrium start of the same
    # prediction
    for key, warm, cold in (("network_gain", "warm+smooth", "cold+smooth"),
                            ("network_gain", "warm", "cold"),
                            ("consistent_gain", "consistent+smooth", "warm+smooth"),
                            ("consistent_gain", "consistent", "warm")):
        if warm in res and cold in res:
            c = _compare(res, cold, warm)
            c["wall_speedup"] = float(res[cold]["seconds"] / res[warm]["seconds"])
            out[f"{key}_{warm}_vs_{cold}"] = c
    out["per_case"] = [dict(Re=round(p["Re"], 1), r=p["r"],
                            **{m: int(res[m]["steps"][c]) for m in res}) for c, p in enumerate(params)]
    return out


def build_dataset_budget(target, gen_batch, seconds, seed, re_range, nx, ny, precision, tol,
                         max_steps, log=_log_default):
    """build_dataset over successive batches of gen_batch seeded cases until
    `target` fields have converged or `seconds` have passed (checked between
    batches); the cases are the first ones of one seeded sequence, so a
    larger budget extends a smaller one's dataset."""
    from . import inputs as I

    t0 = time.perf_counter()
    parts, infos = [], []
    allp = I.warmstart_cases(gen_batch * 64, seed=seed, re_range=re_range)
    k = 0
    while True:
        params = allp[k * gen_batch:(k + 1) * gen_batch]
        parts.append(build_dataset(params, nx=nx, ny=ny, precision=precision, tol=tol,
                                   max_steps=max_steps, log=log))
        infos.append(parts[-1][4])
        k += 1
        got = sum(p[0].shape[0] for p in parts)
        log(f"dataset: {got} fields from {k * gen_batch} cases, {time.perf_counter() - t0:.0f} s")
        if got >= target or time.perf_counter() - t0 > seconds or k * gen_batch >= len(allp):
            break
    X = np.concatenate([p[0] for p in parts])
    fields = tuple(np.concatenate([p[1][i] for p in parts]) for i in range(3))
    masks = [m for p in parts for m in p[2]]
    kept = [q for p in parts for q in p[3]]
    keys = ("cases", "converged", "blew_up", "not_converged")
    info = {key: int(sum(i[key] for i in infos)) for key in keys}
    info.update(seconds=round(time.perf_counter() - t0, 2), tol=tol, batches=k,
                median_steps=int(np.median([i["median_steps"] for i in infos if i["median_steps"]]))
                if any(i["median_steps"] for i in infos) else None)
    return X, fields, masks, kept, info


def save_weights(net, scales, path):
    """The trained network's parameters: 3x3 and head weights rounded to BF16
    (the precision the forward pass uses them in) and stored as their raw
    16-bit patterns, biases in FP32.  numpy .npz, no pickled objects."""
    import torch

    out = {"U": np.float64(scales.U), "levels": np.asarray(net.levels, np.int32)}
    for k, v in net.state().items():
        if k.endswith(".W"):
            bf = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(torch.bfloat16)
            out[k] = bf.view(torch.int16).numpy().view(np.uint16)
        else:
            out[k] = np.asarray(v, np.float32)
    np.savez_compressed(path, **out)


def load_weights(path, batch=16, H=128, W=256):
    """A WarmStartNet (device buffers for `batch` inputs of H x W) and its
    output scales from save_weights' file."""
    import torch

    with np.load(path, allow_pickle=False) as z:
        levels = tuple(int(c) for c in z["levels"])
        net = WarmStartNet(H=H, W=W, batch=batch, levels=levels)
        st = {}
        for k in z.files:
            if k in ("U", "levels"):
                continue
            v = z[k]
            if v.dtype == np.uint16:
                v = torch.from_numpy(v.view(np.int16)).view(torch.bfloat16).float().numpy()
            st[k] = v
        net.load_state(st)
        return net, Scales(float(z["U"]))


def run_pipeline(n_train=3200, n_test=64, epochs=120, batch=16, seed=2103, test_seed=77,
                 out_dir=None, nx=256, ny=128, gen_max_steps=150_000, eval_max_steps=400_000,
                 re_range=(100.0, 5000.0), gen_precision=L.LBM_FP32_DEV, gen_tol=2e-6,
                 target_fields=None, gen_seconds=None, gen_batch=1600, train_seconds=None,
                 log=_log_default):
    """Generate steady fields with the batched solver, train the network on
    them, then compare cold and warm starts on unseen cases.  With
    target_fields the generation runs in batches of gen_batch cases until
    that many fields have converged or gen_seconds have passed."""
    import json
    import os

    from . import inputs as I

    t0 = time.perf_counter()
    if target_fields:
        X, (rho, ux, uy), masks, kept, gen_info = build_dataset_budget(
            target_fields, gen_batch, gen_seconds or 1e9, seed, re_range, nx, ny, gen_precision,
            gen_tol, gen_max_steps, log=log)
    else:
        params = I.warmstart_cases(n_train, seed=seed, re_range=re_range)
        X, (rho, ux, uy), masks, kept, gen_info = build_dataset(params, nx=nx, ny=ny,
                                                                precision=gen_precision,
                                                                tol=gen_tol,
                                                                max_steps=gen_max_steps, log=log)
    log(f"dataset: {gen_info}")
    from . import workloads as Wk

    fluid = (X[..., 0] == 0).astype(np.uint8)
    scales = Scales(0.05)
    T = scales.encode(rho, ux, uy, [Wk.cavity_cs2(p["r"]) for p in kept])
    nval = max(batch, len(X) // 10)
    net = WarmStartNet(H=X.shape[1], W=X.shape[2], batch=batch, seed=seed)
    hist, t_train = train(net, X[nval:], T[nval:], fluid[nval:], epochs,
                          val=(X[:nval], T[:nval], fluid[:nval]), seconds=train_seconds, log=log)
    if out_dir:
        os.makedirs(out_dir, exist_ok=True)
        save_weights(net, scales, os.path.join(out_dir, "warmstart_weights.npz"))
        log(f"weights saved to {out_dir}")
    test = I.warmstart_cases(n_test, seed=test_seed, re_range=re_range)
    cmp = (warm_vs_cold(net, scales, test, nx=nx, ny=ny, max_steps=eval_max_steps, log=log)
           if n_test else None)
    # the validation error of predicting the rest state (all zeros), over the
    # same whole batches that the validation loss covers
    nv = (nval // batch) * batch
    val_zero = float((T[:nv] ** 2 * fluid[:nv, ..., None]).sum() / max(int(fluid[:nv].sum()), 1))
    metrics = dict(dataset=gen_info, train_samples=int(len(X) - nval),
                   val_samples=int(nval), epochs=len(hist), batch=batch,
                   train_seconds=round(t_train, 2), final_loss=hist[-1]["loss"],
                   final_val=hist[-1].get("val"), val_zero_prediction=val_zero, warm_vs_cold=cmp,
                   total_seconds=round(time.perf_counter() - t0, 1))
    if out_dir:
        with open(os.path.join(out_dir, "warmstart_metrics.json"), "w") as fh:
            json.dump(dict(metrics, history=hist), fh, indent=1)
    return metrics, net, scales


WEIGHTS = __import__("os").path.join(__import__("os").path.dirname(__file__),
                                     "warmstart_cavity_256x128.npz")


def evaluate(weights=WEIGHTS, n_test=64, test_seed=77, max_steps=400_000, modes=None,
             log=_log_default):
    """warm_vs_cold for n_test unseen seeded cases with saved weights."""
    from . import inputs as I

    net, scales = load_weights(weights)
    test = I.warmstart_cases(n_test, seed=test_seed)
    return warm_vs_cold(net, scales, test, max_steps=max_steps, modes=modes, log=log)


def conv_flops(net):
    """Multiply-adds x 2 of the network's 3x3 convolutions for one forward
    pass of its batch (the pooling, upsampling, head and loss are left out)."""
    total = 0
    for cv in net.layers():
        h, w = net._res(int(cv.name[1]))
        total += 2 * net.N * h * w * 9 * (cv.c1 + cv.c2) * cv.cout
    return total


def nn_throughput(batch=16, reps=20, H=128, W=256, seed=5):
    """Rate of the network's kernels on seeded random inputs: forward passes,
    and whole training steps (forward, masked MSE, backward, Adam), timed
    between device synchronizations.  A training step runs the 3x3
    convolutions three times (forward, data gradient except for the first
    layer, weight gradient)."""
    import torch

    net = WarmStartNet(H, W, batch, seed=seed)
    g = np.random.Generator(np.random.PCG64(seed))
    M0 = batch * H * W
    x0 = torch.from_numpy(g.uniform(-1, 1, M0 * CIN).astype(np.float32)).cuda()
    tgt = torch.from_numpy(g.normal(0, 1, M0 * COUT).astype(np.float32)).cuda()
    fluid = torch.ones(M0, dtype=torch.uint8, device="cuda")
    cw = torch.tensor((0.25, 1.0, 1.0), dtype=torch.float32, device="cuda")

    def train_step():
        net.forward(x0)
        net.loss_grad(tgt, fluid, M0, cw)
        net.backward(net.gpred)
        net.adam(1e-4)

    net.forward(x0)
    train_step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.forward(x0)
    torch.cuda.synchronize()
    fwd = (time.perf_counter() - t0) / reps
    t0 = time.perf_counter()
    for _ in range(reps):
        train_step()
    torch.cuda.synchronize()
    step = (time.perf_counter() - t0) / reps
    f = conv_flops(net)
    first = net.enc[0][0]
    f_first = 2 * batch * H * W * 9 * (first.c1 + first.c2) * first.cout
    f_step = 3 * f - f_first
    return dict(batch=batch, H=H, W=W, conv_gflop_forward=round(f / 1e9, 2),
                forward_ms=round(1e3 * fwd, 3), forward_tflops=round(f / fwd / 1e12, 1),
                train_step_ms=round(1e3 * step, 3), train_step_tflops=round(f_step / step / 1e12, 1),
                samples_per_s=round(batch / step, 1), peak_bf16_tflops=2500.0)


if __name__ == "__main__":
    import argparse
    import json

    ap = argparse.ArgumentParser(description="train and evaluate the learned warm start")
    ap.add_argument("--train-cases", type=int, default=3200)
    ap.add_argument("--target-fields", type=int, default=0,
                    help="generate batches of cases until this many fields converged")
    ap.add_argument("--gen-seconds", type=float, default=0.0,
                    help="stop generating new batches after this many seconds")
    ap.add_argument("--gen-max-steps", type=int, default=150_000)
    ap.add_argument("--test-cases", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=120)
    ap.add_argument("--train-seconds", type=float, default=0.0,
                    help="cut the epoch count to what fits this time")
    ap.add_argument("--gen-batch", type=int, default=1600)
    ap.add_argument("--out", default=None)
    ap.add_argument("--eval-only", default=None, metavar="WEIGHTS",
                    help="skip training: evaluate saved weights on --test-cases unseen cases")
    ap.add_argument("--nn-throughput", action="store_true",
                    help="time the network's forward pass and training step (batch 16) and exit")
    ap.add_argument("--modes", default=",".join(MODES),
                    help="starts to evaluate, comma-separated, of " + ", ".join(MODES + EXTRA_MODES))
    a = ap.parse_args()
    if a.nn_throughput:
        print(json.dumps(nn_throughput()), flush=True)
    elif a.eval_only:
        modes = tuple(m for m in a.modes.split(",") if m)
        unknown = [m for m in modes if m not in MODES + EXTRA_MODES]
        if unknown:
            ap.error(f"unknown modes {unknown}")
        cmp = evaluate(a.eval_only, a.test_cases, modes=modes, log=lambda m: print(m, flush=True))
        if a.out:
            import os
            os.makedirs(a.out, exist_ok=True)
            with open(os.path.join(a.out, "warmstart_eval.json"), "w") as fh:
                json.dump(cmp, fh, indent=1)
        print(json.dumps({k: v for k, v in cmp.items() if k != "per_case"}), flush=True)
    else:
        m, _, _ = run_pipeline(a.train_cases, a.test_cases, a.epochs, out_dir=a.out,
                               target_fields=a.target_fields or None,
                               gen_seconds=a.gen_seconds or None, gen_max_steps=a.gen_max_steps,
                               gen_batch=a.gen_batch, train_seconds=a.train_seconds or None)
        m = dict(m)
        if m["warm_vs_cold"]:
            m["warm_vs_cold"] = {k: v for k, v in m["warm_vs_cold"].items() if k != "per_case"}
        print(json.dumps(m), flush=True)
