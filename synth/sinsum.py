"""Closed-form problem data built from finite sums of sinusoids.

A ``SinSum`` is  s(x, y, t) = sum_k A_k * sin(a_k x + b_k y + w_k t + p_k).
The set is closed under differentiation (d/dx multiplies A by a and shifts the
phase by pi/2) and under products (product-to-sum identities), so every
manufactured solution the paper uses (Section 6, Eq. periodic_moving and the
stability-test data) and every textbook plane wave can be written exactly and
differentiated exactly.

This module describes *problems*, not the lattice Boltzmann scheme: the
elastodynamic PDE (Eq. teq with the material law Eq. cauchy), the manufactured
body force / initial / boundary data of Section 6.1, and plane-wave solutions.
It holds none of the scheme's arithmetic.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

HALF_PI = 0.5 * math.pi


class SinSum:
    """Sum of sinusoids  sum_k A_k sin(a_k x + b_k y + w_k t + p_k)."""

    __slots__ = ("terms",)

    def __init__(self, terms=None):
        t = np.zeros((0, 5)) if terms is None else np.asarray(terms, dtype=np.float64).reshape(-1, 5)
        self.terms = t

    # -- constructors ---------------------------------------------------------
    @staticmethod
    def sin(a=0.0, b=0.0, w=0.0, p=0.0, amp=1.0):
        return SinSum([[amp, a, b, w, p]])

    @staticmethod
    def cos(a=0.0, b=0.0, w=0.0, p=0.0, amp=1.0):
        return SinSum([[amp, a, b, w, p + HALF_PI]])

    @staticmethod
    def const(c):
        return SinSum([[c, 0.0, 0.0, 0.0, HALF_PI]])

    # -- algebra --------------------------------------------------------------
    def __add__(self, other):
        if not isinstance(other, SinSum):
            other = SinSum.const(float(other))
        return SinSum(np.vstack([self.terms, other.terms]))

    __radd__ = __add__

    def __neg__(self):
        t = self.terms.copy()
        t[:, 0] *= -1.0
        return SinSum(t)

    def __sub__(self, other):
        return self + (-other)

    def __rsub__(self, other):
        return (-self) + other

    def __mul__(self, other):
        if isinstance(other, SinSum):
            out = []
            # sin(u) sin(v) = 1/2 [sin(u - v + pi/2) - sin(u + v + pi/2)]
            for A1, a1, b1, w1, p1 in self.terms:
                for A2, a2, b2, w2, p2 in other.terms:
                    h = 0.5 * A1 * A2
                    out.append([h, a1 - a2, b1 - b2, w1 - w2, p1 - p2 + HALF_PI])
                    out.append([-h, a1 + a2, b1 + b2, w1 + w2, p1 + p2 + HALF_PI])
            return SinSum(out)
        t = self.terms.copy()
        t[:, 0] *= float(other)
        return SinSum(t)

    __rmul__ = __mul__

    def simplified(self, rtol: float = 1e-14) -> "SinSum":
        """Merge terms of equal frequency (a, b, w) by phasor addition."""
        groups = {}
        for A, a, b, w, p in self.terms:
            if (a, b, w) < (0.0, 0.0, 0.0) and (a, b, w) != (0.0, 0.0, 0.0):
                a, b, w, p = -a, -b, -w, math.pi - p  # sin(-th + p) = sin(th + pi - p)
            key = (round(a, 12), round(b, 12), round(w, 12))
            z = groups.get(key, (0j, (a, b, w)))
            groups[key] = (z[0] + A * complex(math.cos(p), math.sin(p)), z[1])
        if not groups:
            return SinSum()
        amax = max(abs(z) for z, _ in groups.values())
        out = [[abs(z), a, b, w, math.atan2(z.imag, z.real)]
               for z, (a, b, w) in groups.values() if abs(z) > rtol * amax]
        return SinSum(out)

    def d(self, var: str) -> "SinSum":
        col = {"x": 1, "y": 2, "t": 3}[var]
        t = self.terms.copy()
        t[:, 0] *= t[:, col]
        t[:, 4] += HALF_PI
        keep = t[:, 0] != 0.0
        return SinSum(t[keep])

    # -- evaluation -----------------------------------------------------------
    def __call__(self, x, y, t=0.0):
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        shape = np.broadcast(x, y, np.asarray(t)).shape
        out = np.zeros(shape)
        for A, a, b, w, p in self.terms:
            out += A * np.sin(a * x + b * y + w * t + p)
        return out

    def on_grid(self, xs, ys, t=0.0):
        """Evaluate on the tensor grid ys x xs (array [len(ys)][len(xs)]) with
        sin(ax + by + c) = sin(ax + c) cos(by) + cos(ax + c) sin(by)."""
        xs = np.asarray(xs, dtype=np.float64)
        ys = np.asarray(ys, dtype=np.float64)
        out = np.zeros((len(ys), len(xs)))
        for A, a, b, w, p in self.terms:
            ph = a * xs + (w * t + p)
            out += np.outer(np.cos(b * ys), A * np.sin(ph))
            out += np.outer(np.sin(b * ys), A * np.cos(ph))
        return out

    def separable_in_time(self, x, y):
        """Split s(x_b, t) = sum_r W_r(x_b) T_r(t) at fixed points.

        Uses sin(th + w t) = sin(th) cos(w t) + cos(th) sin(w t), i.e. rank 2
        per term.  Returns (W [2K, npts], freqs [K]) where the time functions
        are cos(w_k t) (row 2k) and sin(w_k t) (row 2k+1)."""
        x = np.asarray(x, dtype=np.float64)
        y = np.asarray(y, dtype=np.float64)
        K = len(self.terms)
        W = np.zeros((2 * K,) + np.broadcast(x, y).shape)
        for k, (A, a, b, w, p) in enumerate(self.terms):
            th = a * x + b * y + p
            W[2 * k] = A * np.sin(th)
            W[2 * k + 1] = A * np.cos(th)
        return W, self.terms[:, 3].copy()


@dataclass
class Material:
    """Density-scaled wave speeds of Eq. cauchy: c_K^2 and c_mu^2 (Section 2.1)."""

    cK2: float
    cmu2: float
    rho: float = 1.0

    @staticmethod
    def from_lame(lam: float, mu: float, rho: float, model: str = "plane_strain") -> "Material":
        """Eq. 2D / plane_strain / plane_stress with the bulk modulus written
        through Lame's lambda: plane strain (3D lambda) and a 2D continuum
        (2D lambda) both give c_K^2 = (lambda + mu)/rho; plane stress replaces
        lambda by 2 lambda mu / (lambda + 2 mu)."""
        if model == "plane_stress":
            lam = 2.0 * lam * mu / (lam + 2.0 * mu)
        elif model not in ("plane_strain", "continuum_2d"):
            raise ValueError(model)
        return Material((lam + mu) / rho, mu / rho, rho)


class Elastodynamics:
    """Exact fields of a displacement u_hat = (ux, uy) given as SinSums.

    Everything here is the continuum problem of Section 2 / Section 6.1:
    velocity, density-scaled stress (Eq. cauchy), Cauchy stress, and the
    manufactured body load b = d_t^2 u - div sigma."""

    def __init__(self, ux: SinSum, uy: SinSum, mat: Material):
        self.ux, self.uy, self.mat = ux, uy, mat
        cK2, cm2 = mat.cK2, mat.cmu2
        div = ux.d("x") + uy.d("y")
        dev = ux.d("x") - uy.d("y")
        self.sxx = div * cK2 + dev * cm2  # sigma = sigma_bar / rho
        self.syy = div * cK2 - dev * cm2
        self.sxy = (uy.d("x") + ux.d("y")) * cm2
        self.vx, self.vy = ux.d("t"), uy.d("t")
        self.bx = ux.d("t").d("t") - self.sxx.d("x") - self.sxy.d("y")
        self.by = uy.d("t").d("t") - self.sxy.d("x") - self.syy.d("y")
        for name in ("ux", "uy", "sxx", "syy", "sxy", "vx", "vy", "bx", "by"):
            setattr(self, name, getattr(self, name).simplified())

    def fields(self, x, y, t):
        """(v [2], sigma_bar [3], u [2]) physical fields at points."""
        r = self.mat.rho
        v = np.stack([self.vx(x, y, t), self.vy(x, y, t)])
        sb = r * np.stack([self.sxx(x, y, t), self.syy(x, y, t), self.sxy(x, y, t)])
        u = np.stack([self.ux(x, y, t), self.uy(x, y, t)])
        return v, sb, u

    def fields_on_grid(self, xs, ys, t):
        """Like fields() on the tensor grid ys x xs, via separable evaluation."""
        r = self.mat.rho
        g = lambda s: s.on_grid(xs, ys, t)
        v = np.stack([g(self.vx), g(self.vy)])
        sb = r * np.stack([g(self.sxx), g(self.syy), g(self.sxy)])
        return v, sb

    def field_gradients(self, x, y, t):
        """d/dx and d/dy of (vx, vy, sbxx, sbyy, sbxy): array [2][5][...]."""
        r = self.mat.rho
        comps = [self.vx, self.vy, self.sxx * r, self.syy * r, self.sxy * r]
        return np.stack([np.stack([c.d(a)(x, y, t) for c in comps]) for a in ("x", "y")])

    def displacement_gradient(self, x, y, t):
        """(du_x/dx, du_x/dy, du_y/dx, du_y/dy) at points, array [4][...]."""
        return np.stack([self.ux.d("x")(x, y, t), self.ux.d("y")(x, y, t),
                         self.uy.d("x")(x, y, t), self.uy.d("y")(x, y, t)])

    def gradient_field_derivatives(self, x, y, t):
        """d/dx and d/dy of (v_x, v_y, du_x/dx, du_x/dy, du_y/dx, du_y/dy):
        array [2][6][...]."""
        comps = [self.vx, self.vy, self.ux.d("x"), self.ux.d("y"), self.uy.d("x"),
                 self.uy.d("y")]
        return np.stack([np.stack([c.d(a)(x, y, t) for c in comps]) for a in ("x", "y")])

    def body_force(self, x, y, t):
        """Physical body load b_bar = rho * b, array [2][...]."""
        r = self.mat.rho
        return r * np.stack([self.bx(x, y, t), self.by(x, y, t)])

    def has_body_force(self, tol=1e-12) -> bool:
        xs = np.linspace(0.013, 0.97, 7)
        X, Y = np.meshgrid(xs, xs)
        return float(np.abs(self.body_force(X, Y, 0.37)).max()) > tol


def plane_wave(kx: float, ky: float, amp: float, phase: float, kind: str, mat: Material):
    """Textbook plane wave solving Eq. teq with b = 0.

    P wave: polarisation along k, omega = sqrt(cK^2 + cmu^2) |k|.
    S wave: polarisation normal to k, omega = cmu |k|.
    Returns (ux, uy) SinSums of u = amp * d * sin(k.x - omega t + phase)."""
    kn = math.hypot(kx, ky)
    if kn == 0.0:
        raise ValueError("zero wavenumber")
    if kind == "P":
        d = (kx / kn, ky / kn)
        om = math.sqrt(mat.cK2 + mat.cmu2) * kn
    elif kind == "S":
        d = (-ky / kn, kx / kn)
        om = math.sqrt(mat.cmu2) * kn
    else:
        raise ValueError(kind)
    s = SinSum.sin(kx, ky, -om, phase)
    return s * (amp * d[0]), s * (amp * d[1])


def periodic_moving_solution() -> tuple[SinSum, SinSum]:
    """The L-periodic manufactured displacement of Eq. periodic_moving."""
    pi = math.pi
    ux = (SinSum.sin(4 * pi, 0, -4 * pi * 0.3) * SinSum.cos(0, 2 * pi, -2 * pi * 0.8)
          * SinSum.sin(0, 0, 4 * pi, -4 * pi * 0.1))
    uy = (SinSum.cos(4 * pi, 0, -4 * pi * 0.7) * SinSum.sin(0, 2 * pi, -2 * pi * 0.1)
          * SinSum.cos(0, 0, 4 * pi, 4 * pi * 0.4))
    return ux, uy


def stability_test_solution() -> tuple[SinSum, SinSum]:
    """Initial data of the homogeneous-Dirichlet stability test (Section 6.2):
    u0 = sin(4 pi x) sin(2 pi y) (sin 4pi(t-0.1), sin 4pi(t+0.4)) read at t = 0,
    v0 = its time derivative at t = 0.  Zero on the boundary of the unit square."""
    pi = math.pi
    s = SinSum.sin(4 * pi) * SinSum.sin(0, 2 * pi)
    return s * SinSum.sin(0, 0, 4 * pi, -4 * pi * 0.1), s * SinSum.sin(0, 0, 4 * pi, 4 * pi * 0.4)


def standing_mms_solution() -> tuple[SinSum, SinSum]:
    """Smooth manufactured displacement u = sin(2 pi x) cos(2 pi y) cos(2 pi t)
    in both components (requires a matching body load)."""
    pi = math.pi
    s = SinSum.sin(2 * pi) * SinSum.cos(0, 2 * pi) * SinSum.cos(0, 0, 2 * pi)
    return s, s * 1.0
