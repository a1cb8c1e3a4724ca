"""Python binding of the batched-lattice C ABI (lbm_batch_* in include/lbm.h).

Instances of uneven size, boundary type and material are advanced together;
fields move in and out as packed 1-D tensors (instance i's [c][ny][nx] block
starts at c * node_offset(i))."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import LbmParams, check
from .lbm import _ptr, _stream_ptr


class Batch:
    def __init__(self, instances, device="cuda:0"):
        """instances: iterable of dicts with keys nx, ny, dx, dt, lam, mu, rho,
        bc and optionally model."""
        self.L = _lib.load()
        self.device = torch.device(device)
        inst = list(instances)
        self.n = len(inst)
        arr = (LbmParams * self.n)()
        for i, p in enumerate(inst):
            arr[i] = LbmParams(int(p["nx"]), int(p["ny"]), float(p["dx"]), float(p["dt"]),
                               float(p["lam"]), float(p["mu"]), float(p["rho"]), int(p["bc"]),
                               int(p.get("model", 0)), 0)
        self._params = arr
        self.shapes = [(int(p["ny"]), int(p["nx"])) for p in inst]
        nbytes = self.L.lbm_batch_workspace_bytes(self.n, ctypes.cast(arr, ctypes.c_void_p))
        if nbytes == 0:
            h = ctypes.c_void_p()
            check(self.L.lbm_batch_create(self.n, ctypes.cast(arr, ctypes.c_void_p),
                                          ctypes.c_void_p(256), 0, None, ctypes.byref(h)))
            raise RuntimeError("invalid batch parameters")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            h = ctypes.c_void_p()
            check(self.L.lbm_batch_create(self.n, ctypes.cast(arr, ctypes.c_void_p),
                                          ctypes.c_void_p(self.ws.data_ptr() + off), nbytes,
                                          _stream_ptr(self.device), ctypes.byref(h)))
        self.ctx = h
        self.offsets = [int(self.L.lbm_batch_node_offset(self.ctx, i)) for i in range(self.n + 1)]
        self.total_nodes = self.offsets[-1]
        self._keep = []
        self._walls = {}

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.L.lbm_batch_destroy(ctx)
            self.ctx = None

    # -- packing ----------------------------------------------------------------
    def pack(self, arrays, dtype=torch.float64):
        """List of per-instance [c][ny][nx] arrays -> packed device tensor."""
        parts = [torch.as_tensor(np.ascontiguousarray(a)).reshape(-1) if isinstance(a, np.ndarray)
                 else a.reshape(-1) for a in arrays]
        return torch.cat(parts).to(self.device, dtype).contiguous()

    def unpack(self, packed, ncomp):
        out = []
        for i, (ny, nx) in enumerate(self.shapes):
            a = ncomp * self.offsets[i]
            out.append(packed[a:a + ncomp * ny * nx].reshape(ncomp, ny, nx))
        return out

    # -- state --------------------------------------------------------------------
    def init(self, v0, sigma0):
        v0 = v0.to(self.device, torch.float64).contiguous()
        s0 = sigma0.to(self.device, torch.float64).contiguous()
        if v0.numel() != 2 * self.total_nodes or s0.numel() != 3 * self.total_nodes:
            raise ValueError("packed field sizes do not match the batch")
        check(self.L.lbm_batch_init(self.ctx, _ptr(v0), _ptr(s0)))
        self._keep = [v0, s0]
        return self

    def init_fields_f32(self, fields):
        f = fields.to(self.device, torch.float32).contiguous()
        if f.numel() != 5 * self.total_nodes:
            raise ValueError("packed field size does not match the batch")
        check(self.L.lbm_batch_init_fields_f32(self.ctx, _ptr(f)))
        self._keep = [f]
        return self

    def set_wall_velocity(self, i, W, T):
        if W is None or W.shape[0] == 0:
            check(self.L.lbm_batch_set_wall_velocity(self.ctx, i, 0, None, None, 0))
            self._walls.pop(i, None)
            return self
        W = W.to(self.device, torch.float32).contiguous()
        T = T.to(self.device, torch.float32).contiguous()
        check(self.L.lbm_batch_set_wall_velocity(self.ctx, i, W.shape[0], _ptr(W), _ptr(T),
                                                 T.shape[0]))
        self._walls[i] = (W, T)
        return self

    def step(self, n=1, graph=True):
        fn = self.L.lbm_batch_step if graph else self.L.lbm_batch_step_eager
        check(fn(self.ctx, int(n)))
        return self

    @property
    def tblock_config(self):
        """Temporally blocked variant in use (T steps per launch), -1 = none."""
        i = ctypes.c_int32()
        check(self.L.lbm_batch_get_tblock_config(self.ctx, ctypes.byref(i)))
        return i.value

    @tblock_config.setter
    def tblock_config(self, index):
        check(self.L.lbm_batch_set_tblock_config(self.ctx, int(index)))

    def tblock_configs(self):
        out = []
        for i in range(self.L.lbm_batch_tblock_config_count()):
            t, sr, nt, pf = (ctypes.c_int32() for _ in range(4))
            check(self.L.lbm_batch_tblock_config_info(i, ctypes.byref(t), ctypes.byref(sr),
                                                      ctypes.byref(nt), ctypes.byref(pf)))
            out.append({"index": i, "steps": t.value, "seg_rows": sr.value,
                        "nontemporal": nt.value, "prefetch": pf.value})
        return out

    def autotune(self, reps=5):
        """Select the fastest of single steps and the blocked variants (state
        unchanged); returns (index, ms per step)."""
        i, ms = ctypes.c_int32(), ctypes.c_double()
        check(self.L.lbm_batch_autotune(self.ctx, int(reps), ctypes.byref(i), ctypes.byref(ms)))
        return i.value, ms.value

    @property
    def steps(self):
        return int(self.L.lbm_batch_step_count(self.ctx))

    def moments(self, out=None, system=False):
        if out is None:
            out = torch.empty(5 * self.total_nodes, dtype=torch.float32, device=self.device)
        if (out.numel() != 5 * self.total_nodes or out.dtype != torch.float32
                or not out.is_contiguous() or not out.is_cuda):
            raise ValueError("out must be a contiguous float32 tensor of 5 * total_nodes "
                             "elements on the batch's device")
        fn = self.L.lbm_batch_moments_U if system else self.L.lbm_batch_moments
        check(fn(self.ctx, _ptr(out)))
        return out

    def energy(self):
        out = (ctypes.c_double * self.n)()
        check(self.L.lbm_batch_energy(self.ctx, out))
        return np.array(out[:])

    def rel_l2_fields(self, fields):
        f = fields.to(self.device, torch.float32).contiguous()
        out = (ctypes.c_double * self.n)()
        check(self.L.lbm_batch_rel_l2_fields(self.ctx, _ptr(f), out))
        return np.array(out[:])

    def rel_l2_pair(self, a, b):
        """Per-instance ||U(a) - U(b)|| / ||U(b)|| of two packed FP32 field
        arrays (v, sigma_bar), U from each instance's material; no state."""
        fa = a.to(self.device, torch.float32).contiguous()
        fb = b.to(self.device, torch.float32).contiguous()
        if fa.numel() != 5 * self.total_nodes or fb.numel() != 5 * self.total_nodes:
            raise ValueError("packed field sizes do not match the batch")
        out = (ctypes.c_double * self.n)()
        check(self.L.lbm_batch_rel_l2_pair(self.ctx, _ptr(fa), _ptr(fb), out))
        return np.array(out[:])


def rel_l2_pair_static(instances, a, b, device="cuda:0"):
    """lbm_rel_l2_pair_static: per-instance ||U(a) - U(b)|| / ||U(b)|| of
    packed FP32 fields for the instances described by `instances` (dicts as
    for Batch), with no batch, workspace or device allocation."""
    L = _lib.load()
    inst = list(instances)
    arr = (LbmParams * len(inst))()
    for i, p in enumerate(inst):
        arr[i] = LbmParams(int(p["nx"]), int(p["ny"]), float(p["dx"]), float(p["dt"]),
                           float(p["lam"]), float(p["mu"]), float(p["rho"]), int(p["bc"]),
                           int(p.get("model", 0)), 0)
    dev = torch.device(device)
    fa = a.to(dev, torch.float32).contiguous()
    fb = b.to(dev, torch.float32).contiguous()
    nodes = sum(int(p["nx"]) * int(p["ny"]) for p in inst)
    if fa.numel() != 5 * nodes or fb.numel() != 5 * nodes:
        raise ValueError("packed field sizes do not match the instances")
    out = (ctypes.c_double * len(inst))()
    with torch.cuda.device(dev):
        check(L.lbm_rel_l2_pair_static(len(inst), ctypes.cast(arr, ctypes.c_void_p), _ptr(fa),
                                       _ptr(fb), out, _stream_ptr(dev)))
    return np.array(out[:])
