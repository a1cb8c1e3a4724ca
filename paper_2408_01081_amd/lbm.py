"""Python binding of the single-lattice C ABI (include/lbm.h).

PyTorch provides the device memory (workspace, inputs, outputs) and the HIP
stream; all computation happens in the library's kernels."""
from __future__ import annotations

import ctypes

import torch

from . import _lib
from ._lib import LbmParams, check

PERIODIC, DIRICHLET = 0, 1
PLANE_STRAIN, PLANE_STRESS, CONTINUUM_2D = 0, 1, 2
PLANE_LAYOUT, DISPLACEMENT, ALLOW_UNSTABLE = 1, 2, 4


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return ctypes.c_void_p(t.data_ptr())


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Lattice:
    """One lattice problem on one GPU.

    Parameters follow ``lbm_params``: nodes ``nx`` x ``ny``, spacing ``dx``,
    time step ``dt``, Lame constants ``lam`` and ``mu``, density ``rho``,
    boundary ``bc`` (PERIODIC or DIRICHLET) and material ``model``;
    ``displacement`` reserves the displacement state (``init_displacement``);
    ``allow_unstable`` accepts parameters beyond the CFL-like limit."""

    def __init__(self, nx, ny, dx, dt, lam, mu, rho, bc=PERIODIC, model=PLANE_STRAIN,
                 device="cuda:0", plane_layout=False, displacement=False, allow_unstable=False):
        self.L = _lib.load()
        self.device = torch.device(device)
        self.nx, self.ny, self.bc = int(nx), int(ny), int(bc)
        flags = ((PLANE_LAYOUT if plane_layout else 0) | (DISPLACEMENT if displacement else 0)
                 | (ALLOW_UNSTABLE if allow_unstable else 0))
        self.params = LbmParams(int(nx), int(ny), float(dx), float(dt), float(lam), float(mu),
                                float(rho), int(bc), int(model), flags)
        nbytes = self.L.lbm_workspace_bytes(ctypes.byref(self.params))
        if nbytes == 0:
            # re-run create to get the precise validation error
            h = ctypes.c_void_p()
            check(self.L.lbm_create(ctypes.byref(self.params), ctypes.c_void_p(256), 0, None,
                                    ctypes.byref(h)))
            raise RuntimeError("invalid parameters")
        with torch.cuda.device(self.device):
            self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            off = (-self.ws.data_ptr()) % 256
            self._ws_ptr = ctypes.c_void_p(self.ws.data_ptr() + off)
            h = ctypes.c_void_p()
            check(self.L.lbm_create(ctypes.byref(self.params), self._ws_ptr, nbytes,
                                    _stream_ptr(self.device), ctypes.byref(h)))
        self.ctx = h
        self._keep = []  # inputs that must outlive queued kernels
        kK, km, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        check(self.L.lbm_lattice_constants(self.ctx, ctypes.byref(kK), ctypes.byref(km),
                                           ctypes.byref(c)))
        self.kK, self.km, self.c = kK.value, km.value, c.value

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx:
            try:
                torch.cuda.synchronize(self.device)
            except Exception:
                pass
            self.L.lbm_destroy(ctx)
            self.ctx = None

    # -- state set-up --------------------------------------------------------
    def init(self, v0, sigma0, grad=None):
        """Second-order initialisation from physical fields (float64 device
        tensors [2][ny][nx], [3][ny][nx], optional [2][5][ny][nx])."""
        ts = [t.to(self.device, torch.float64).contiguous() if t is not None else None
              for t in (v0, sigma0, grad)]
        self._check_shape(ts[0], (2, self.ny, self.nx))
        self._check_shape(ts[1], (3, self.ny, self.nx))
        if ts[2] is not None:
            self._check_shape(ts[2], (2, 5, self.ny, self.nx))
        check(self.L.lbm_init(self.ctx, _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2])))
        self._keep = ts
        return self

    def init_from_gradient(self, v0, gradu0, grad=None):
        """Second-order initialisation from the initial velocity [2][ny][nx]
        and displacement gradient [4][ny][nx] (du_x/dx, du_x/dy, du_y/dx,
        du_y/dy), optional exact d/dx, d/dy of these six fields
        [2][6][ny][nx]; float64.  Needed for mu = 0, where the stress does
        not determine U0."""
        ts = [t.to(self.device, torch.float64).contiguous() if t is not None else None
              for t in (v0, gradu0, grad)]
        self._check_shape(ts[0], (2, self.ny, self.nx))
        self._check_shape(ts[1], (4, self.ny, self.nx))
        if ts[2] is not None:
            self._check_shape(ts[2], (2, 6, self.ny, self.nx))
        check(self.L.lbm_init_from_gradient(self.ctx, _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2])))
        self._keep = ts
        return self

    def set_populations(self, f):
        t = f.to(self.device, torch.float32).contiguous()
        self._check_shape(t, (4, 5, self.ny, self.nx))
        check(self.L.lbm_set_populations(self.ctx, _ptr(t)))
        self._keep = [t]
        return self

    def set_wall_velocity(self, W, T):
        """Separable wall data: W [R][2(nx+ny)][2], T [nsteps][R] (float32)."""
        if W is None or W.shape[0] == 0:
            check(self.L.lbm_set_wall_velocity(self.ctx, 0, None, None, 0))
            self._wall = None
            return self
        W = W.to(self.device, torch.float32).contiguous()
        T = T.to(self.device, torch.float32).contiguous()
        R = W.shape[0]
        if W.shape != (R, 2 * (self.nx + self.ny), 2) or T.dim() != 2 or T.shape[1] != R:
            raise ValueError("bad wall table shapes")
        check(self.L.lbm_set_wall_velocity(self.ctx, R, _ptr(W), _ptr(T), T.shape[0]))
        self._wall = (W, T)
        return self

    def set_body_force(self, X, Y, T):
        """Separable body load b_bar = rho b: X [R][2][nx], Y [R][ny],
        T [nsteps+1][R] (float32); R = 0 or X None removes it."""
        if X is None or X.shape[0] == 0:
            check(self.L.lbm_set_body_force(self.ctx, 0, None, None, None, 0))
            self._force = None
            return self
        X, Y, T = (t.to(self.device, torch.float32).contiguous() for t in (X, Y, T))
        R = X.shape[0]
        if (X.shape != (R, 2, self.nx) or Y.shape != (R, self.ny) or T.dim() != 2
                or T.shape[1] != R or T.shape[0] < 1):
            raise ValueError("bad body load table shapes")
        check(self.L.lbm_set_body_force(self.ctx, R, _ptr(X), _ptr(Y), _ptr(T), T.shape[0] - 1))
        self._force = (X, Y, T)
        return self

    def init_displacement(self, u0):
        """Start the trapezoidal displacement output from u0 [2][ny][nx]."""
        t = u0.to(self.device, torch.float64).contiguous()
        self._check_shape(t, (2, self.ny, self.nx))
        check(self.L.lbm_init_displacement(self.ctx, _ptr(t)))
        self._keep = list(self._keep) + [t]
        return self

    def displacement(self, out=None):
        """u(t_n) float32 [2][ny][nx]."""
        out = self._out(out, (2, self.ny, self.nx))
        check(self.L.lbm_displacement(self.ctx, _ptr(out)))
        return out

    def set_reference(self, X, Y, T):
        """Exact outputs for the error norms: X [R][7][nx], Y [R][ny],
        T [nsteps+1][R] (float64); components u_x, u_y, v_x, v_y,
        sigma_xx, sigma_yy, sigma_xy."""
        if X is None or X.shape[0] == 0:
            check(self.L.lbm_set_reference(self.ctx, 0, None, None, None, 0))
            self._ref = None
            return self
        X, Y, T = (t.to(self.device, torch.float64).contiguous() for t in (X, Y, T))
        R = X.shape[0]
        if (X.shape != (R, 7, self.nx) or Y.shape != (R, self.ny) or T.dim() != 2
                or T.shape[1] != R or T.shape[0] < 1):
            raise ValueError("bad reference table shapes")
        check(self.L.lbm_set_reference(self.ctx, R, _ptr(X), _ptr(Y), _ptr(T), T.shape[0] - 1))
        self._ref = (X, Y, T)
        return self

    def track_errors(self, on=True):
        check(self.L.lbm_error_track(self.ctx, int(bool(on))))
        return self

    def error_norms(self):
        """Space-time norms of Section 6.1 over the tracked levels, per group
        ('u', 'v', 's' for Cauchy stress): L2, L2rel, Linf, Linfrel."""
        import math
        buf = (ctypes.c_double * 10)()
        check(self.L.lbm_error_sums(self.ctx, buf))
        w = self.params.dx ** 2 * self.params.dt
        out = {"levels": int(buf[9])}
        for gi, name in enumerate(("u", "v", "s")):
            e2, x2, einf = buf[3 * gi], buf[3 * gi + 1], buf[3 * gi + 2]
            out[name] = {"L2": math.sqrt(w * e2), "L2rel": math.sqrt(e2 / x2) if x2 else None,
                         "Linf": einf, "Linfrel": einf / math.sqrt(w * x2) if x2 else None}
        return out

    # -- stepping and output ---------------------------------------------------
    def step(self, n=1):
        check(self.L.lbm_step(self.ctx, int(n)))
        return self

    @property
    def steps(self):
        return int(self.L.lbm_step_count(self.ctx))

    def moments(self, out=None):
        """(v_x, v_y, sigma_xx, sigma_yy, sigma_xy) float32 [5][ny][nx]."""
        out = self._out(out, (5, self.ny, self.nx))
        check(self.L.lbm_moments(self.ctx, _ptr(out)))
        return out

    def moments_U(self, out=None):
        out = self._out(out, (5, self.ny, self.nx))
        check(self.L.lbm_moments_U(self.ctx, _ptr(out)))
        return out

    def populations(self, out=None):
        out = self._out(out, (4, 5, self.ny, self.nx))
        check(self.L.lbm_populations(self.ctx, _ptr(out)))
        return out

    def energy(self):
        r = ctypes.c_double()
        check(self.L.lbm_energy(self.ctx, ctypes.byref(r)))
        return r.value

    def rel_l2(self, refU):
        t = refU.to(self.device, torch.float64).contiguous()
        self._check_shape(t, (5, self.ny, self.nx))
        r = ctypes.c_double()
        check(self.L.lbm_rel_l2(self.ctx, _ptr(t), ctypes.byref(r)))
        return r.value

    # -- launch configurations / autotuner --------------------------------------
    @property
    def step_config(self):
        i = ctypes.c_int32()
        check(self.L.lbm_get_step_config(self.ctx, ctypes.byref(i)))
        return i.value

    @step_config.setter
    def step_config(self, index):
        check(self.L.lbm_set_step_config(self.ctx, int(index)))

    @property
    def tblock_config(self):
        """Temporally blocked variant in use (T steps per launch), -1 = none."""
        i = ctypes.c_int32()
        check(self.L.lbm_get_tblock_config(self.ctx, ctypes.byref(i)))
        return i.value

    @tblock_config.setter
    def tblock_config(self, index):
        check(self.L.lbm_set_tblock_config(self.ctx, int(index)))

    def set_tblock_split(self, mode):
        """Split blocked launches of a Dirichlet lattice (interior with the
        periodic kernel's code, wall band with the Dirichlet rule, one
        launch): -1 (the default) or 1 wherever a split kernel exists and
        the lattice allows, 0 never."""
        check(self.L.lbm_set_tblock_split(self.ctx, int(mode)))

    def tblock_split_active(self, index):
        """Whether launches of blocked variant `index` run split now."""
        return int(self.L.lbm_tblock_split_active(self.ctx, int(index))) == 1

    def select_for_steps(self, n):
        """Select the launch configuration cheapest for runs of n steps
        (from the last autotune's launch times); returns the blocked variant
        (-1: single steps)."""
        i = ctypes.c_int32()
        check(self.L.lbm_select_for_steps(self.ctx, int(n), ctypes.byref(i)))
        return i.value

    def tblock_remainder(self, r):
        """The blocked variant `step` launches for the last r steps of a run
        (-1: none)."""
        i = ctypes.c_int32()
        check(self.L.lbm_get_tblock_remainder(self.ctx, int(r), ctypes.byref(i)))
        return i.value

    @property
    def steps_per_launch(self):
        """Time steps per launch lbm_step uses for this lattice as configured."""
        return int(self.L.lbm_steps_per_launch(self.ctx))

    def tblock_configs(self):
        out = []
        for i in range(self.L.lbm_tblock_config_count()):
            t, sr, nt, pf = (ctypes.c_int32() for _ in range(4))
            check(self.L.lbm_tblock_config_info(i, ctypes.byref(t), ctypes.byref(sr),
                                                ctypes.byref(nt), ctypes.byref(pf)))
            out.append({"index": i, "steps": t.value, "seg_rows": sr.value,
                        "nontemporal": nt.value, "prefetch": pf.value})
        return out

    def time_tblock_config(self, index, reps=20):
        """Average ms of one launch (T steps) of blocked variant `index`."""
        ms = ctypes.c_double()
        check(self.L.lbm_time_tblock_config(self.ctx, int(index), int(reps), ctypes.byref(ms)))
        return ms.value

    def valid_step_configs(self):
        return [i for i, c in enumerate(step_configs()) if c["valid_for"](self.nx)]

    def time_step_config(self, index, reps=20):
        ms = ctypes.c_double()
        check(self.L.lbm_time_step_config(self.ctx, int(index), int(reps), ctypes.byref(ms)))
        return ms.value

    def autotune(self, reps=20, use_cache=True):
        """Pick the fastest launch configuration for this grid (state unchanged)."""
        i, ms = ctypes.c_int32(), ctypes.c_double()
        check(self.L.lbm_autotune(self.ctx, int(reps), int(bool(use_cache)), ctypes.byref(i),
                                  ctypes.byref(ms)))
        return i.value, ms.value

    # -- helpers ---------------------------------------------------------------
    def _out(self, out, shape):
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=self.device)
        self._check_shape(out, shape)
        if out.dtype != torch.float32:
            raise ValueError("float32 output expected")
        return out

    @staticmethod
    def _check_shape(t, shape):
        if tuple(t.shape) != tuple(shape):
            raise ValueError("shape %s expected, got %s" % (shape, tuple(t.shape)))


def step_configs():
    """Descriptions of the step kernel's launch configurations."""
    L = _lib.load()
    out = []
    for i in range(L.lbm_step_config_count()):
        v, t, n, x = (ctypes.c_int32() for _ in range(4))
        check(L.lbm_step_config_info(i, ctypes.byref(v), ctypes.byref(t), ctypes.byref(n),
                                     ctypes.byref(x)))
        vec, xm = v.value, x.value
        out.append({"index": i, "vec": vec, "threads": t.value, "nontemporal": n.value,
                    "shuffle": xm,
                    "valid_for": (lambda nx, vec=vec, xm=xm:
                                  nx % vec == 0 and (xm == 0 or nx % (64 * vec) == 0))})
    return out


def copy_f32(dst, src):
    """Plain streaming copy kernel (bandwidth reference)."""
    if dst.numel() != src.numel() or dst.dtype != torch.float32 or src.dtype != torch.float32:
        raise ValueError("float32 tensors of equal size expected")
    check(_lib.load().lbm_copy_f32(_ptr(dst), _ptr(src), src.numel(), _stream_ptr(src.device)))
