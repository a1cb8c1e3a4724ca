"""Python binding of the learned window surrogate (include/sg.h).

Argument marshalling only; forward, loss, backward and Adam run in the HIP
kernels of csrc/sg.hip."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check
from .lbm import _ptr, _stream_ptr

# (name, cin, cout) in parameter order; mirrors the library's layer table
LAYERS = [("in", 32, 32), ("e0a", 32, 32), ("e0b", 32, 32), ("e1a", 32, 64), ("e1b", 64, 64),
          ("e2a", 64, 128), ("e2b", 128, 128), ("e3a", 128, 128), ("e3b", 128, 128),
          ("d2a", 128, 128), ("d2b", 128, 64), ("d1a", 64, 64), ("d1b", 64, 32),
          ("d0a", 32, 32), ("d0b", 32, 32), ("out", 32, 32)]
NBASIS = 4


class SgConfig(ctypes.Structure):
    _fields_ = [("batch", ctypes.c_int32), ("height", ctypes.c_int32), ("width", ctypes.c_int32),
                ("split", ctypes.c_int32), ("train", ctypes.c_int32)]


def param_count():
    return int(_lib.load().sg_param_count())


def pack_params(P):
    """dict name.w [co][ci][3][3], name.a [co][4] -> flat float32 vector."""
    parts = []
    for name, ci, co in LAYERS:
        parts.append(np.asarray(P[name + ".w"], dtype=np.float64).reshape(-1))
        parts.append(np.asarray(P[name + ".a"], dtype=np.float64).reshape(-1))
    return np.concatenate(parts)


def unpack_params(v):
    out, o = {}, 0
    v = np.asarray(v)
    for name, ci, co in LAYERS:
        n = co * ci * 9
        out[name + ".w"] = v[o:o + n].reshape(co, ci, 3, 3)
        o += n
        out[name + ".a"] = v[o:o + co * NBASIS].reshape(co, NBASIS)
        o += co * NBASIS
    return out


def init_params(seed=0, out_scale=0.0):
    """Seeded initial parameters: He-like weights, FiLM gains 1, the output
    layer scaled by out_scale (0: the network starts as the identity map)."""
    g = np.random.default_rng(seed)
    P = {}
    for name, ci, co in LAYERS:
        w = g.standard_normal((co, ci, 3, 3)) / np.sqrt(9 * ci)
        if name == "out":
            w *= out_scale
        a = np.zeros((co, NBASIS))
        a[:, 0] = 1.0
        P[name + ".w"], P[name + ".a"] = w, a
    return P


class Surrogate:
    def __init__(self, batch, height, width, split=3, train=False, device="cuda:0"):
        L = _lib.load()
        self.L = L
        self.device = torch.device(device)
        self.cfg = SgConfig(int(batch), int(height), int(width), int(split), int(bool(train)))
        self.batch, self.H, self.W = int(batch), int(height), int(width)
        nbytes = L.sg_workspace_bytes(ctypes.byref(self.cfg))
        if nbytes == 0:
            h = ctypes.c_void_p()
            check(L.sg_create(ctypes.byref(self.cfg), ctypes.c_void_p(256), 0, None,
                              ctypes.byref(h)))
            raise RuntimeError("invalid surrogate configuration")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            h = ctypes.c_void_p()
            check(L.sg_create(ctypes.byref(self.cfg), ctypes.c_void_p(self.ws.data_ptr() + off),
                              nbytes, _stream_ptr(self.device), ctypes.byref(h)))
        self.ctx = h
        self.nparam = param_count()

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.L.sg_destroy(ctx)
            self.ctx = None

    def set_conv_mode(self, mode):
        """0: LDS-tiled convolutions where they apply (default); 1: direct only."""
        check(self.L.sg_set_conv_mode(self.ctx, int(mode)))
        return self

    def set_params(self, v):
        t = torch.as_tensor(np.asarray(v, dtype=np.float32) if not torch.is_tensor(v) else v)
        t = t.to(self.device, torch.float32).contiguous()
        if t.numel() != self.nparam:
            raise ValueError("expected %d parameters" % self.nparam)
        check(self.L.sg_set_params(self.ctx, _ptr(t)))
        torch.cuda.synchronize(self.device)
        return self

    def get_params(self):
        t = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        check(self.L.sg_get_params(self.ctx, _ptr(t)))
        return t

    def get_grads(self):
        t = torch.empty(self.nparam, dtype=torch.float32, device=self.device)
        check(self.L.sg_get_grads(self.ctx, _ptr(t)))
        return t

    def _check_in(self, x, c):
        if x.dtype != torch.float32 or not x.is_cuda or not x.is_contiguous():
            raise ValueError("contiguous float32 device tensor expected")
        if x.dim() != 4 or x.shape[1] != c or x.shape[2] != self.H or x.shape[3] != self.W:
            raise ValueError("shape [B][%d][%d][%d] expected" % (c, self.H, self.W))
        if x.shape[0] > self.batch:
            raise ValueError("batch too large")

    def forward(self, x, circular=True, out=None):
        self._check_in(x, 8)
        if out is None:
            out = torch.empty((x.shape[0], 5, self.H, self.W), dtype=torch.float32,
                              device=self.device)
        check(self.L.sg_forward(self.ctx, _ptr(x), x.shape[0], int(bool(circular)), _ptr(out)))
        return out

    def train_step(self, x, target, circular=True, lr=1e-3, want_loss=True):
        self._check_in(x, 8)
        self._check_in(target, 5)
        loss = ctypes.c_double()
        check(self.L.sg_train_step(self.ctx, _ptr(x), _ptr(target), x.shape[0],
                                   int(bool(circular)), ctypes.c_float(lr),
                                   ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


LEVELS = [0, 0, 0, 1, 1, 2, 2, 3, 3, 2, 2, 1, 1, 0, 0, 0]  # resolution level of each layer


def forward_flops(B, H, W, padded=False):
    """Multiply-add FLOPs of one forward (the 3x3 convolutions) on the
    network's own channels (5 real input fields into the first layer, 5 real
    outputs of the last), or as the kernels run them (padded=True: 32
    channels there; one matrix-core pass)."""
    tot = 0
    for (name, ci, co), lv in zip(LAYERS, LEVELS):
        if not padded:
            ci = 5 if name == "in" else ci
            co = 5 if name == "out" else co
        tot += 2 * 9 * ci * co * (H >> lv) * (W >> lv)
    return B * tot


def main():
    """Time the forward pass: python -m paper_2408_01081_amd.surrogate B H W
    [conv_mode] [weights.npy] (median of 20 calls after 3 warm-up calls), or
    a training step (forward + backward + Adam, learning rate 1e-6):
    python -m paper_2408_01081_amd.surrogate train B H W (mean of 10 steps
    after 3 warm-up steps)."""
    import os
    import sys
    if sys.argv[1] == "train":
        B, H, W = (int(a) for a in sys.argv[2:5])
        net = Surrogate(B, H, W, split=3, train=True)
        net.set_params(np.load(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                            "weights", "surrogate.npy"), allow_pickle=False))
        g = torch.Generator(device=net.device).manual_seed(0)
        x = torch.randn(B, 8, H, W, device=net.device, generator=g)
        x[:, 5], x[:, 6], x[:, 7] = 0.5, 1.0, 1.0
        y = x[:, :5] + 0.01 * torch.randn(B, 5, H, W, device=net.device, generator=g)
        for _ in range(3):
            net.train_step(x, y, lr=1e-6, want_loss=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            net.train_step(x, y, lr=1e-6, want_loss=False)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 10
        fl = 3 * forward_flops(B, H, W)
        print("train step B=%d %dx%d: %.4f ms, %.1f TFLOP/s of the network's own FLOPs "
              "counted as 3 forward passes (%.1f%% of the 2.5 PFLOP/s BF16 peak)"
              % (B, H, W, ms, fl / ms / 1e9, fl / ms / 1e9 / 25.0), flush=True)
        return
    B, H, W = (int(a) for a in sys.argv[1:4])
    mode = int(sys.argv[4]) if len(sys.argv) > 4 else 0
    path = sys.argv[5] if len(sys.argv) > 5 else os.path.join(
        os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate.npy")
    net = Surrogate(B, H, W, split=3)
    net.set_params(np.load(path, allow_pickle=False))
    net.set_conv_mode(mode)
    x = torch.randn(B, 8, H, W, device=net.device)
    x[:, 5], x[:, 6], x[:, 7] = 0.5, 1.0, 1.0
    for _ in range(3):
        net.forward(x)
    times = []
    for _ in range(20):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        net.forward(x)
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    ms = float(np.median(times))
    fl, flp = forward_flops(B, H, W), forward_flops(B, H, W, padded=True)
    print("forward B=%d %dx%d conv_mode %d: %.4f ms, %.1f TFLOP/s of the network's own FLOPs "
          "(%.1f%% of the 2.5 PFLOP/s BF16 peak); the kernels issue %.1f TFLOP/s (3 hi/lo "
          "passes over padded channels)"
          % (B, H, W, mode, ms, fl / ms / 1e9, fl / ms / 1e9 / 25.0, 3 * flp / ms / 1e9),
          flush=True)


if __name__ == "__main__":
    main()
