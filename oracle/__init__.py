"""FP64 CPU oracle of the vectorial lattice Boltzmann scheme for 2D linear
elastodynamics (arXiv 2408.01081).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package.  It shares no code with the HIP
library (``paper_2408_01081_amd``) and never imports it.

The scheme's arithmetic lives in ``lbm_oracle.c`` (plain C, double precision,
OpenMP); this module builds it, loads it with ctypes and adds the problem
set-up (Section 2), the conversions between physical fields and the
first-order system's variables (Eq. ic_vector, Eq. sigma_num) and the error
norms of Section 6.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lib = None

PERIODIC, DIRICHLET = 0, 1


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        L.orc_step.argtypes = [i, i, i, d, d, d, dp, dp, dp, dp, dp, dp, dp, dp]
        L.orc_step.restype = None
        L.orc_moments.argtypes = [i, i, dp, dp, dp]
        L.orc_init.argtypes = [i, i, i, d, d, dp, dp, dp, dp, dp]
        L.orc_norm_weights.argtypes = [d, d, dp]
        L.orc_norm_weights.restype = i
        L.orc_energy.argtypes = [i, i, d, d, dp]
        L.orc_energy.restype = d
        L.orc_wall_link.argtypes = [i, i, i, i, i]
        L.orc_wall_link.restype = i
        L.orc_run.argtypes = [i, i, i, d, d, dp, dp, dp, ctypes.c_long]
        L.orc_set_printed_wall_source.argtypes = [d]
        L.orc_threads.restype = i
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# ---------------------------------------------------------------------------
# Set-up (Section 2.1 / 2.3 / 3.1, Eq. stab_cond)
# ---------------------------------------------------------------------------
class CFLError(ValueError):
    pass


class Setup:
    """Grid, material and step of one problem, reduced to lattice units.

    c_K from the material model (Eq. 2D / plane_strain / plane_stress written
    with Lame's lambda: c_K^2 = (lambda+mu)/rho for plane strain and a 2D
    continuum, lambda -> 2 lambda mu/(lambda+2mu) for plane stress),
    c_mu^2 = mu/rho (Eq. all), lattice speed c = dx/dt, Courant numbers
    kK = c_K/c and km = c_mu/c.  Rejects 2 sqrt(kK^2 + km^2) >= 1
    (Eq. stab_cond) unless allow_unstable is set."""

    def __init__(self, nx, ny, dx, dt, lam, mu, rho, bc, model="plane_strain",
                 allow_unstable=False):
        if nx < 1 or ny < 1 or dx <= 0 or dt <= 0 or rho <= 0 or mu < 0:
            raise ValueError("bad problem parameters")
        if model == "plane_stress":
            lam = 2.0 * lam * mu / (lam + 2.0 * mu)
        cK2 = (lam + mu) / rho
        if cK2 <= 0:
            raise ValueError("lambda + mu must be positive")
        self.nx, self.ny, self.dx, self.dt, self.rho, self.bc = nx, ny, dx, dt, rho, bc
        self.cK, self.cmu = math.sqrt(cK2), math.sqrt(mu / rho)
        self.c = dx / dt
        self.kK, self.km = self.cK / self.c, self.cmu / self.c
        self.cfl = 2.0 * math.hypot(self.kK, self.km)
        if self.cfl >= 1.0 and not allow_unstable:
            raise CFLError("2 sqrt(cK^2+cmu^2)/c = %.4f >= 1" % self.cfl)

    @staticmethod
    def from_speeds(nx, ny, dx, dt, cK2, cmu2, bc, allow_unstable=False):
        """Set-up from (c_K^2, c_mu^2) with rho = 1 (the paper's Section 6)."""
        return Setup(nx, ny, dx, dt, cK2 - cmu2, cmu2, 1.0, bc, allow_unstable=allow_unstable)

    # -- physical fields <-> first-order system variables -----------------
    def U_from_fields(self, v, sb):
        """U = (v_x, v_y, j_s, j_d, j_xy) from velocity and Cauchy stress.

        Inverts Eq. sigma_num with sigma = sigma_bar / rho:
        j_s = -(s_xx + s_yy)/(2 c_K), j_d = -(s_xx - s_yy)/(2 c_mu),
        j_xy = -s_xy / c_mu  (needs c_mu > 0)."""
        s = np.asarray(sb) / self.rho
        U = np.empty((5,) + np.shape(v)[1:])
        U[0], U[1] = v[0], v[1]
        U[2] = -(s[0] + s[1]) / (2.0 * self.cK)
        U[3] = -(s[0] - s[1]) / (2.0 * self.cmu)
        U[4] = -s[2] / self.cmu
        return U

    def fields_from_U(self, U):
        """(v, sigma_bar) from U (Eq. sigma_num times rho)."""
        v = np.array(U[:2])
        sb = -self.rho * np.stack([self.cK * U[2] + self.cmu * U[3],
                                   self.cK * U[2] - self.cmu * U[3],
                                   self.cmu * U[4]])
        return v, sb

    def U_from_displacement_gradient(self, v, gradu):
        """Eq. ic_vector: U0 from v0 and grad u0 (gradu[a][b] = d u_a / d x_b)."""
        U = np.empty((5,) + np.shape(v)[1:])
        U[0], U[1] = v[0], v[1]
        U[2] = -self.cK * (gradu[0][0] + gradu[1][1])
        U[3] = -self.cmu * (gradu[0][0] - gradu[1][1])
        U[4] = -self.cmu * (gradu[1][0] + gradu[0][1])
        return U

    def wall_count(self):
        return 2 * (self.nx + self.ny)

    def wall_points(self):
        """Midpoints x_b = x - e_ij dx / 2 of the missing links, in the
        oracle's link order (left, right, bottom, top)."""
        nx, ny, dx = self.nx, self.ny, self.dx
        ys = (np.arange(ny) + 0.5) * dx
        xs = (np.arange(nx) + 0.5) * dx
        xb = np.concatenate([xs[0] - 0.5 * dx + 0 * ys, xs[-1] + 0.5 * dx + 0 * ys, xs, xs])
        yb = np.concatenate([ys, ys, ys[0] - 0.5 * dx + 0 * xs, ys[-1] + 0.5 * dx + 0 * xs])
        return xb, yb

    def nodes(self):
        xs = (np.arange(self.nx) + 0.5) * self.dx
        ys = (np.arange(self.ny) + 0.5) * self.dx
        return np.meshgrid(xs, ys)


# ---------------------------------------------------------------------------
# Thin wrappers over the C routines
# ---------------------------------------------------------------------------
def init_populations(s: Setup, U0, UX=None, UY=None, Bhat0=None):
    f = np.empty((4, 5, s.ny, s.nx))
    c = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    U0, UX, UY, Bhat0 = c(U0), c(UX), c(UY), c(Bhat0)
    lib().orc_init(s.nx, s.ny, s.bc, s.kK, s.km, _p(U0), _p(UX), _p(UY), _p(Bhat0), _p(f))
    return f


def step(s: Setup, f, Bhat=None, wall=None, ustar=None, want_U=False, want_u=False):
    """One time step: returns (f_next, U(t_n) or None, u(t_n) or None)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    fn = np.empty_like(f)
    fs = np.empty_like(f)
    U = np.empty((5, s.ny, s.nx)) if want_U else None
    u = np.empty((2, s.ny, s.nx)) if (want_u and ustar is not None) else None
    Bhat = None if Bhat is None else np.ascontiguousarray(Bhat, dtype=np.float64)
    wall = None if wall is None else np.ascontiguousarray(wall, dtype=np.float64)
    lib().orc_step(s.nx, s.ny, s.bc, s.kK, s.km, s.dt, _p(f), _p(fn), _p(Bhat), _p(wall),
                   _p(ustar), _p(u), _p(U), _p(fs))
    return fn, U, u


def moments(s: Setup, f, Bhat=None):
    U = np.empty((5, s.ny, s.nx))
    Bhat = None if Bhat is None else np.ascontiguousarray(Bhat, dtype=np.float64)
    lib().orc_moments(s.nx, s.ny, _p(np.ascontiguousarray(f)), _p(Bhat), _p(U))
    return U


def norm_weights(kK, km):
    out = np.empty((4, 5, 5))
    if lib().orc_norm_weights(kK, km, _p(out)):
        raise np.linalg.LinAlgError("singular g_ij")
    return out


def energy(s: Setup, f):
    """||f||_P^2 (Definition grid_norm, Eq. def_symmetrizer)."""
    return lib().orc_energy(s.nx, s.ny, s.kK, s.km, _p(np.ascontiguousarray(f)))


def run_free(s: Setup, f, nsteps):
    """Advance nsteps with B = 0 and homogeneous (or periodic) boundaries."""
    f = np.ascontiguousarray(f, dtype=np.float64).copy()
    w, fs = np.empty_like(f), np.empty_like(f)
    lib().orc_run(s.nx, s.ny, s.bc, s.kK, s.km, _p(f), _p(w), _p(fs), int(nsteps))
    return f


# ---------------------------------------------------------------------------
# A whole simulation driven by closed-form data (Section 6.1 recipe)
# ---------------------------------------------------------------------------
class Simulation:
    """Initial data -> populations (Eq. ic_second) -> steps (Section 3.6).

    v0, sb0       physical initial velocity [2] and Cauchy stress [3] fields
    dfields       optional exact spatial derivatives [2][5] of (v, sigma_bar)
                  (physical); otherwise central differences are used
    gradu0        optional displacement gradient [2][2] (d u_a / d x_b) of u0:
                  U0 then follows Eq. ic_vector from (v0, gradu0) and sb0 is
                  not used (needed for c_mu = 0, where the stress does not
                  determine j_d, j_xy); dfields then holds the exact
                  derivatives [2] of (v0, gradu0) in the same nesting
    u0            optional initial displacement; enables the trapezoidal
                  displacement output (Eq. trapezoidal) with u*(0) = u0 - dt/2 v(0)
    body(t)       optional physical body load b_bar(t) on the nodes, [2][ny][nx]
    wall(t)       optional du_D/dt at the wall midpoints, [L][2]
    """

    def __init__(self, s: Setup, v0, sb0, dfields=None, u0=None, body=None, wall=None,
                 init_correction=True, gradu0=None):
        self.s, self.body, self.wall = s, body, wall
        self.n = 0
        UX = UY = None
        if gradu0 is not None:
            # Eq. ic_vector (linear: derivatives map the same way)
            U0 = s.U_from_displacement_gradient(v0, gradu0)
            if dfields is not None:
                UX = s.U_from_displacement_gradient(*dfields[0]) * s.dx
                UY = s.U_from_displacement_gradient(*dfields[1]) * s.dx
        else:
            U0 = s.U_from_fields(v0, sb0)
            if dfields is not None:
                UX = s.U_from_fields(dfields[0][:2], dfields[0][2:]) * s.dx
                UY = s.U_from_fields(dfields[1][:2], dfields[1][2:]) * s.dx
        B0 = self.bhat(0.0)
        if init_correction:
            self.f = init_populations(s, U0, UX, UY, B0)
        else:
            # ablation: equilibrium populations only (no dt/8 correction term)
            z = np.zeros_like(U0)
            self.f = init_populations(s, U0, z, z, None)
        self.ustar = None
        if u0 is not None:
            self.ustar = np.ascontiguousarray(np.array(u0, dtype=np.float64) - 0.5 * s.dt * U0[:2])

    def bhat(self, t):
        if self.body is None:
            return None
        return np.ascontiguousarray(self.s.dt * np.asarray(self.body(t)) / self.s.rho)

    def t(self):
        return self.n * self.s.dt

    def U(self):
        return moments(self.s, self.f, self.bhat(self.t()))

    def advance(self, nsteps=1, record=None):
        """Advance; ``record(n, U, u)`` is called with the collision-stage
        outputs of every step (times t_n, n = current..current+nsteps-1)."""
        s = self.s
        for _ in range(nsteps):
            tn = self.t()
            w = None if self.wall is None else self.wall(tn + 0.5 * s.dt)
            fn, U, u = step(s, self.f, self.bhat(tn), w, self.ustar, want_U=record is not None,
                            want_u=record is not None)
            if record is not None:
                record(self.n, U, u)
            self.f = fn
            self.n += 1
        return self

    def displacement(self):
        """u(t_n) = u* + dt/2 v(t_n) (Section 3.5)."""
        U = self.U()
        return self.ustar + 0.5 * self.s.dt * U[:2]


# ---------------------------------------------------------------------------
# Error norms of Section 6.1 / 6.2
# ---------------------------------------------------------------------------
class SpaceTimeNorms:
    """Accumulates L2 = (dx^2 dt sum |e|^2)^(1/2) and Linf over G x T and the
    matching norms of the exact solution (for L2rel / Linfrel)."""

    def __init__(self, dx, dt):
        self.w = dx * dx * dt
        self.e2 = {}
        self.x2 = {}
        self.einf = {}

    def add(self, name, num, exact):
        e = np.asarray(num) - np.asarray(exact)
        self.e2[name] = self.e2.get(name, 0.0) + self.w * float(np.sum(e * e))
        self.x2[name] = self.x2.get(name, 0.0) + self.w * float(np.sum(np.asarray(exact) ** 2))
        self.einf[name] = max(self.einf.get(name, 0.0), float(np.abs(e).max()))

    def L2(self, name):
        return math.sqrt(self.e2[name])

    def L2rel(self, name):
        return math.sqrt(self.e2[name] / self.x2[name])

    def Linfrel(self, name):
        return self.einf[name] / math.sqrt(self.x2[name])


def rel_l2(a, b):
    """||a - b||_2 / ||b||_2 over all entries (FP64)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.sqrt(np.sum((a - b) ** 2) / np.sum(b * b)))
