"""Python binding of the exact linear window operator (lbm_wop_* in
include/lbm.h): the 16-step window map of a periodic lattice as one
convolution, built from the library's own lattice steps on unit deltas and
applied by its matrix-core kernel.  Argument marshalling only."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import LbmParams, check
from .lbm import PERIODIC, _ptr, _stream_ptr

STEPS = 16
SIDE = 2 * (STEPS + 1) + 1


class WindowOperator:
    """The window operator of a periodic nx x ny lattice with Lame constants
    lam, mu, density rho, spacing dx and time step dt."""

    def __init__(self, nx, ny, dx, dt, lam, mu, rho, device="cuda:0"):
        self.L = _lib.load()
        self.device = torch.device(device)
        self.nx, self.ny = int(nx), int(ny)
        self.params = LbmParams(self.nx, self.ny, float(dx), float(dt), float(lam), float(mu),
                                float(rho), PERIODIC, 0, 0)
        nb = self.L.lbm_wop_scratch_bytes(ctypes.byref(self.params))
        if nb == 0:
            raise ValueError("no window operator for these parameters (periodic, mu > 0, "
                             "CFL-like condition)")
        with torch.cuda.device(self.device):
            scratch = torch.empty(nb + 256, dtype=torch.uint8, device=self.device)
            off = (-scratch.data_ptr()) % 256
            self.G = torch.empty((SIDE, SIDE, 5, 5), dtype=torch.float32, device=self.device)
            self.op = torch.empty(self.L.lbm_wop_operand_bytes() // 4, dtype=torch.float32,
                                  device=self.device)
            check(self.L.lbm_wop_build(ctypes.byref(self.params), _ptr(self.G), _ptr(self.op),
                                       ctypes.c_void_p(scratch.data_ptr() + off), nb,
                                       _stream_ptr(self.device)))
            torch.cuda.current_stream(self.device).synchronize()
        del scratch

    def apply(self, x, out=None):
        """x: [B][5][ny][nx] float32 fields (v, sigma_bar) on the device ->
        the fields 16 lattice steps later."""
        if x.dim() != 4 or x.shape[1:] != (5, self.ny, self.nx):
            raise ValueError("expected [B][5][%d][%d] fields" % (self.ny, self.nx))
        if x.dtype != torch.float32 or not x.is_contiguous() or x.device != self.device:
            raise ValueError("contiguous float32 fields on the operator's device expected")
        if out is None:
            out = torch.empty_like(x)
        if out.shape != x.shape or out.dtype != torch.float32 or not out.is_contiguous():
            raise ValueError("out must match x")
        check(self.L.lbm_wop_apply(ctypes.byref(self.params), _ptr(self.op), _ptr(x), _ptr(out),
                                   int(x.shape[0]), _stream_ptr(self.device)))
        return out


class WindowSurrogate:
    """The exact operator in the place of the learned surrogate of the
    serving rollout (same call as Surrogate.forward: inputs [B][8][H][W]
    with the material in channels 5..7, which the operator was built for)."""

    def __init__(self, op: WindowOperator):
        self.op = op
        self.H, self.W = op.ny, op.nx
        self._x = None

    def forward(self, x, circular=True, out=None):
        if not circular:
            raise ValueError("the exact window operator covers periodic windows only")
        f = x[:, :5]
        if not f.is_contiguous():
            if self._x is None or self._x.shape != f.shape:
                self._x = torch.empty(f.shape, dtype=torch.float32, device=x.device)
            self._x.copy_(f)
            f = self._x
        if out is not None and not out.is_contiguous():
            y = self.op.apply(f)
            out.copy_(y)
            return out
        return self.op.apply(f, out=out)
