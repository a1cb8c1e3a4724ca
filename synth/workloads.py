"""Seeded synthetic workloads shared by the oracle tests, the GPU tests and the
benchmark.  Only inputs are produced here (grids, materials, initial fields,
wall data); nothing in this module performs a lattice Boltzmann operation.

All randomness is numpy ``Generator(PCG64(seed))`` on the host.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .sinsum import Elastodynamics, Material, SinSum, plane_wave

PERIODIC, DIRICHLET = 0, 1


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def node_coords(nx: int, ny: int, dx: float):
    """Cell-centred node positions ((k+1/2)dx, (l+1/2)dx), arrays [ny][nx]."""
    xs = (np.arange(nx) + 0.5) * dx
    ys = (np.arange(ny) + 0.5) * dx
    X, Y = np.meshgrid(xs, ys)
    return X, Y


def wall_points(nx: int, ny: int, dx: float):
    """Wall-link midpoints in the library's link order.

    Links [0, ny): left wall x = 0, node (0, l).
    Links [ny, 2ny): right wall x = nx dx, node (nx-1, l).
    Links [2ny, 2ny+nx): bottom wall y = 0, node (k, 0).
    Links [2ny+nx, 2ny+2nx): top wall y = ny dx, node (k, ny-1).
    Returns (xb, yb) arrays of length 2(nx+ny)."""
    ys = (np.arange(ny) + 0.5) * dx
    xs = (np.arange(nx) + 0.5) * dx
    xb = np.concatenate([np.zeros(ny), np.full(ny, nx * dx), xs, xs])
    yb = np.concatenate([ys, ys, np.zeros(nx), np.full(nx, ny * dx)])
    return xb, yb


def poisson_lame(nu: float, mu: float = 1.0) -> float:
    """Lame lambda for Poisson ratio nu at shear modulus mu."""
    return 2.0 * mu * nu / (1.0 - 2.0 * nu)


def dt_at_cfl_fraction(dx: float, mat: Material, frac: float = 0.5) -> float:
    """Time step at which 2 sqrt(cK^2 + cmu^2) / (dx/dt) equals ``frac``."""
    cP = math.sqrt(mat.cK2 + mat.cmu2)
    return frac * dx / (2.0 * cP)


@dataclass
class Problem:
    """One lattice problem: grid, material, step, and exact/initial data."""

    nx: int
    ny: int
    dx: float
    dt: float
    lam: float
    mu: float
    rho: float
    bc: int
    sol: Elastodynamics | None = None  # exact solution (closed form) if any
    v0: np.ndarray | None = None       # [2][ny][nx] physical initial velocity
    sb0: np.ndarray | None = None      # [3][ny][nx] physical initial Cauchy stress
    meta: dict = field(default_factory=dict)

    @property
    def mat(self) -> Material:
        return Material.from_lame(self.lam, self.mu, self.rho)

    def initial_fields(self):
        if self.v0 is not None:
            return self.v0, self.sb0
        xs = (np.arange(self.nx) + 0.5) * self.dx
        ys = (np.arange(self.ny) + 0.5) * self.dx
        return self.sol.fields_on_grid(xs, ys, 0.0)

    def exact(self, t: float):
        X, Y = node_coords(self.nx, self.ny, self.dx)
        return self.sol.fields(X, Y, t)

    def wall_velocity(self, t: float) -> np.ndarray:
        """du_D/dt at wall midpoints, [L][2]; zero when there is no solution."""
        L = 2 * (self.nx + self.ny)
        if self.sol is None:
            return np.zeros((L, 2))
        xb, yb = wall_points(self.nx, self.ny, self.dx)
        return np.stack([self.sol.vx(xb, yb, t), self.sol.vy(xb, yb, t)], axis=1)

    def body_table(self, nsteps: int):
        """Body load table of the solution's manufactured load; see
        separable_body_table.  R = 0 when the solution needs no load."""
        return separable_body_table(self.sol, self.nx, self.ny, self.dx, self.dt, nsteps)

    def reference_table(self, nsteps: int):
        """Exact outputs for the error norms; see separable_reference_table."""
        return separable_reference_table(self.sol, self.nx, self.ny, self.dx, self.dt, nsteps)

    def wall_table(self, nsteps: int, step0: int = 0):
        """Separable wall velocity du_D/dt(x_b, t_n + dt/2) = sum_r W[r] T[n][r].

        Returns (W [R][L][2] float64, T [nsteps][R] float64); R = 0 when the
        boundary data are homogeneous."""
        L = 2 * (self.nx + self.ny)
        if self.sol is None or self.bc != DIRICHLET:
            return np.zeros((0, L, 2)), np.zeros((nsteps, 0))
        xb, yb = wall_points(self.nx, self.ny, self.dx)
        comps = [self.sol.vx, self.sol.vy]
        Ws, Ts = [], []
        tn = (np.arange(step0, step0 + nsteps) + 0.5) * self.dt
        for ci, s in enumerate(comps):
            if len(s.terms) == 0:
                continue
            W, w = s.separable_in_time(xb, yb)
            for k in range(len(w)):
                for r, fn in ((2 * k, np.cos), (2 * k + 1, np.sin)):
                    Wr = np.zeros((L, 2))
                    Wr[:, ci] = W[r]
                    Ws.append(Wr)
                    Ts.append(fn(w[k] * tn))
        return np.stack(Ws), np.stack(Ts, axis=1)


def oscillating_walls(nx: int, ny: int, dt: float, nsteps: int, rank: int = 4,
                      amp: float = 1e-2, seed: int = 0):
    """Seeded separable wall velocities for a Dirichlet rectangle (driven
    walls, no exact solution behind them): W [rank][L][2] with L = 2 (nx +
    ny) links (left wall rows, right wall rows, bottom columns, top columns),
    each component a short random Fourier series of the link position of
    amplitude ~amp; T [nsteps][rank] = cos / sin (omega_r t_n), t_n = (n +
    1/2) dt, omega_r / 2 pi uniform in [0.5, 4].  float64."""
    rng = np.random.default_rng(seed)
    L = 2 * (nx + ny)
    s = np.arange(L) / L
    W = np.zeros((rank, L, 2))
    for r in range(rank):
        for c in range(2):
            k = rng.integers(1, 6, size=3)
            ph = rng.uniform(0.0, 2 * np.pi, size=3)
            a = rng.normal(size=3)
            W[r, :, c] = amp * sum(a[j] * np.sin(2 * np.pi * k[j] * s + ph[j]) for j in range(3))
    om = 2 * np.pi * rng.uniform(0.5, 4.0, size=rank)
    tn = (np.arange(nsteps) + 0.5) * dt
    T = np.stack([np.cos(om[r] * tn) if r % 2 == 0 else np.sin(om[r] * tn)
                  for r in range(rank)], axis=1)
    return W, T


def separable_table(comps, nx: int, ny: int, dx: float, dt: float, nsteps: int):
    """Fields given as SinSums, comps = [(SinSum, scale), ...] (component c is
    scale_c * comps[c][0]), at the nodes and levels t_n = n dt, n = 0..nsteps,
    as a sum of products of a function of x, of y and of t:
      field_c(x_k, y_l, t_n) = sum_r X[r][c][k] Y[r][l] T[n][r].

    Each term A sin(al + be + ga) (al = a x + p, be = b y, ga = w t) splits into
    four products by the addition theorem:
      sin al cos be cos ga + cos al sin be cos ga
      + cos al cos be sin ga - sin al sin be sin ga.
    Returns float64 (X [R][C][nx], Y [R][ny], T [nsteps+1][R])."""
    C = len(comps)
    xs = (np.arange(nx) + 0.5) * dx
    ys = (np.arange(ny) + 0.5) * dx
    tn = np.arange(nsteps + 1) * dt
    Xs, Ys, Ts = [], [], []
    for comp, (s, scale) in enumerate(comps):
        for A, a, b, w, p in s.terms:
            al, be, ga = a * xs + p, b * ys, w * tn
            for fx, fy, ft, sign in ((np.sin, np.cos, np.cos, 1.0), (np.cos, np.sin, np.cos, 1.0),
                                     (np.cos, np.cos, np.sin, 1.0), (np.sin, np.sin, np.sin, -1.0)):
                Xr = np.zeros((C, nx))
                Xr[comp] = sign * scale * A * fx(al)
                Xs.append(Xr)
                Ys.append(fy(be))
                Ts.append(ft(ga))
    if not Xs:
        return np.zeros((0, C, nx)), np.zeros((0, ny)), np.zeros((nsteps + 1, 0))
    return np.stack(Xs), np.stack(Ys), np.stack(Ts, axis=1)


def separable_body_table(sol: Elastodynamics | None, nx: int, ny: int, dx: float, dt: float,
                         nsteps: int):
    """The physical body load b_bar = rho b of ``sol`` in the form of
    separable_table (two components); R = 0 without a load."""
    if sol is None or not sol.has_body_force():
        return np.zeros((0, 2, nx)), np.zeros((0, ny)), np.zeros((nsteps + 1, 0))
    r = sol.mat.rho
    return separable_table([(sol.bx, r), (sol.by, r)], nx, ny, dx, dt, nsteps)


def separable_reference_table(sol: Elastodynamics, nx: int, ny: int, dx: float, dt: float,
                              nsteps: int):
    """The exact outputs of ``sol`` (u_x, u_y, v_x, v_y and the Cauchy stress
    sigma_bar = rho sigma: xx, yy, xy) in the form of separable_table."""
    r = sol.mat.rho
    comps = [(sol.ux, 1.0), (sol.uy, 1.0), (sol.vx, 1.0), (sol.vy, 1.0),
             (sol.sxx, r), (sol.syy, r), (sol.sxy, r)]
    return separable_table(comps, nx, ny, dx, dt, nsteps)


def plane_wave_superposition(seed: int, mat: Material, nwaves: int = 8, kmax: int = 16,
                             lengths=(1.0, 1.0)):
    """Seeded sum of P and S plane waves with integer wavenumbers |m| <= kmax
    (periodic on a rectangle of the given side lengths), velocity amplitude ~1."""
    g = rng(seed)
    Lx, Ly = lengths
    ux, uy = SinSum(), SinSum()
    waves = []
    while len(waves) < nwaves:
        m = int(g.integers(-kmax, kmax + 1))
        n = int(g.integers(-kmax, kmax + 1))
        if m == 0 and n == 0 or m * m + n * n > kmax * kmax:
            continue
        kind = "P" if g.random() < 0.5 else "S"
        kx, ky = 2 * math.pi * m / Lx, 2 * math.pi * n / Ly
        kn = math.hypot(kx, ky)
        om = (math.sqrt(mat.cK2 + mat.cmu2) if kind == "P" else math.sqrt(mat.cmu2)) * kn
        amp = float(g.uniform(0.5, 1.0)) / om
        ph = float(g.uniform(0, 2 * math.pi))
        a, b = plane_wave(kx, ky, amp, ph, kind, mat)
        ux, uy = ux + a, uy + b
        waves.append((m, n, kind, amp, ph))
    return ux, uy, waves


def plane_wave_problem(nx, ny, bc, seed, nu=None, rho=1.0, mu=1.0, cfl=0.5, nwaves=8, kmax=16,
                       dx=None):
    """Grid problem whose exact solution is a seeded plane-wave superposition.

    The domain is (0, nx dx) x (0, ny dx); dx defaults to 1/max(nx, ny)... the
    wavenumbers are integer multiples of 2 pi / side so the data are periodic."""
    g = rng(seed + 7919)
    if nu is None:
        nu = float(g.uniform(0.0, 0.49))
    lam = poisson_lame(nu, mu)
    if dx is None:
        dx = 1.0 / max(nx, ny)
    mat = Material.from_lame(lam, mu, rho)
    ux, uy, waves = plane_wave_superposition(seed, mat, nwaves, kmax, (nx * dx, ny * dx))
    dt = dt_at_cfl_fraction(dx, mat, cfl)
    p = Problem(nx, ny, dx, dt, lam, mu, rho, bc, Elastodynamics(ux, uy, mat),
                meta={"nu": nu, "waves": waves, "seed": seed})
    return p


def gaussian_random_field(g: np.random.Generator, ny: int, nx: int, ell: float,
                          nfields: int = 1) -> np.ndarray:
    """Periodic Gaussian random fields: white noise convolved with a periodic
    Gaussian of standard deviation ell/sqrt(2) cells (covariance length ell),
    normalised to zero mean and unit sample variance.  Shape [nfields][ny][nx]."""
    import scipy.fft as sfft
    noise = g.standard_normal((nfields, ny, nx))
    s = ell / math.sqrt(2.0)
    kx = 2 * math.pi * np.fft.rfftfreq(nx)
    ky = 2 * math.pi * np.fft.fftfreq(ny)
    filt = np.exp(-0.5 * s * s * (ky[:, None] ** 2 + kx[None, :] ** 2))
    f = sfft.irfft2(sfft.rfft2(noise, workers=-1) * filt, s=(ny, nx), workers=-1)
    f -= f.mean(axis=(1, 2), keepdims=True)
    f /= f.std(axis=(1, 2), keepdims=True)
    return f


def wall_taper(ny: int, nx: int, width: float) -> np.ndarray:
    """Smooth factor that vanishes at the four walls and is 1 beyond ``width``
    cells from them (sin^2 ramp)."""
    def ramp(n):
        d = np.minimum(np.arange(n) + 0.5, n - (np.arange(n) + 0.5))
        r = np.clip(d / max(width, 1e-12), 0.0, 1.0)
        return np.sin(0.5 * math.pi * r) ** 2
    return ramp(ny)[:, None] * ramp(nx)[None, :]


def random_material(g: np.random.Generator, rho_range=(0.5, 2.0), nu_range=(0.0, 0.49),
                    mu: float = 1.0):
    nu = float(g.uniform(*nu_range))
    rho = float(g.uniform(*rho_range))
    return poisson_lame(nu, mu), mu, rho, nu


def grf_problem(nx, ny, bc, seed, ell=None, rho_range=(0.5, 2.0), cfl=0.5, dx=1.0):
    """Problem with Gaussian-random-field initial velocity and stress (no
    closed-form solution).  Dirichlet instances taper the fields to zero at the
    walls (homogeneous boundary data)."""
    g = rng(seed)
    lam, mu, rho, nu = random_material(g, rho_range)
    if ell is None:
        ell = float(g.uniform(8.0, 32.0))
    f = gaussian_random_field(g, ny, nx, ell, 5)
    if bc == DIRICHLET:
        f = f * wall_taper(ny, nx, ell)
    mat = Material.from_lame(lam, mu, rho)
    dt = dt_at_cfl_fraction(dx, mat, cfl)
    # velocity ~ unit variance; stress scaled by rho * c_P so both parts of the
    # state have comparable magnitude in the first-order system's variables.
    sc = rho * math.sqrt(mat.cK2 + mat.cmu2)
    return Problem(nx, ny, dx, dt, lam, mu, rho, bc, None, v0=f[:2].copy(), sb0=f[2:] * sc,
                   meta={"nu": nu, "ell": ell, "seed": seed})


def random_populations(seed: int, nx: int, ny: int) -> np.ndarray:
    """Seeded standard-normal population array [4][5][ny][nx] (for invariant
    and parity tests that start from an arbitrary lattice state)."""
    return rng(seed).standard_normal((4, 5, ny, nx))


def batched_instances(n: int, seed: int, side=(64, 512), rho_range=(0.5, 2.0), cfl=0.5,
                      dirichlet_fraction=0.5):
    """Seeded batch of GRF problems: side lengths uniform in [side], non-square,
    the first round(n * dirichlet_fraction) of a seeded permutation Dirichlet,
    Poisson ratio U[0, 0.49], mu = 1, rho uniform in rho_range, time step at
    ``cfl`` of the CFL-like limit, GRF length scale U[8, 32] cells."""
    g = rng(seed)
    order = g.permutation(n)
    nd = int(round(n * dirichlet_fraction))
    bcs = np.zeros(n, dtype=int)
    bcs[order[:nd]] = DIRICHLET
    probs = []
    for i in range(n):
        nx = int(g.integers(side[0], side[1] + 1))
        ny = int(g.integers(side[0], side[1] + 1))
        probs.append(grf_problem(nx, ny, int(bcs[i]), seed=seed * 100003 + i,
                                 rho_range=rho_range, cfl=cfl))
    return probs
