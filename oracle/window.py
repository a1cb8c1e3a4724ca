"""FP64 oracle of the exact linear window operator (periodic lattices).

TEST INFRASTRUCTURE ONLY (see the package docstring): used by the tests and
nothing else; it shares no code with the HIP library.

For a fixed material the window map of the scheme on a periodic lattice,

    U_out = moments(n steps from the second-order initialisation of U_in),

is linear in U_in (the initialisation Eq. ic_second with central-difference
gradients, the collision Eq. collision_vector and the streaming Eq.
streaming are all linear) and commutes with lattice shifts, so it is a
convolution:

    U_out[co](p) = sum_{d} sum_{ci} G[d][co][ci] U_in[ci](p - d),

where G[d][:, ci] is the response at offset d to a unit delta in component
ci.  Information moves one node per step along an axis and the central
differences reach one node, so G vanishes outside |dx| + |dy| <= n + 1.
This module obtains G exactly that way (delta inputs through the oracle's
own initialisation and steps) and applies it as a plain periodic
convolution.
"""
from __future__ import annotations

import numpy as np

from . import PERIODIC, Setup, init_populations, moments, run_free


def radius(nsteps: int) -> int:
    """Support radius of the n-step window map: n steps plus the reach of the
    central differences in the initialisation."""
    return nsteps + 1


def _lattice(s: Setup, side: int) -> Setup:
    rho = s.rho
    mu = s.cmu * s.cmu * rho
    lam = s.cK * s.cK * rho - mu
    return Setup(side, side, s.dx, s.dt, lam, mu, rho, PERIODIC)


def window_map_n(s: Setup, U, nsteps: int):
    """Second-order initialisation from U (central differences, no load),
    nsteps steps, zeroth moment: the lattice scheme's window map."""
    f = init_populations(s, np.ascontiguousarray(U, dtype=np.float64))
    f = run_free(s, f, nsteps)
    return moments(s, f)


def window_operator(s: Setup, nsteps: int = 16):
    """G[dy + R][dx + R][co][ci], R = nsteps + 1: the response in component co
    at offset (dx, dy) to a unit delta in component ci, on a periodic lattice
    wider than the support (material and time step of s)."""
    R = radius(nsteps)
    side = 2 * R + 6
    c0 = side // 2
    lat = _lattice(s, side)
    G = np.zeros((2 * R + 1, 2 * R + 1, 5, 5))
    for ci in range(5):
        U0 = np.zeros((5, side, side))
        U0[ci, c0, c0] = 1.0
        Uo = window_map_n(lat, U0, nsteps)
        G[:, :, :, ci] = np.transpose(Uo[:, c0 - R:c0 + R + 1, c0 - R:c0 + R + 1], (1, 2, 0))
    return G


def apply_window_operator(G, U):
    """Periodic convolution U_out[co](p) = sum_d sum_ci G[d][co][ci] U[ci](p - d)
    of U [5][ny][nx]."""
    U = np.asarray(U, dtype=np.float64)
    R = (G.shape[0] - 1) // 2
    out = np.zeros_like(U)
    for iy in range(2 * R + 1):
        for ix in range(2 * R + 1):
            g = G[iy, ix]
            if not g.any():
                continue
            shifted = np.roll(U, (iy - R, ix - R), axis=(1, 2))  # U(p - d)
            out += np.einsum("oc,cyx->oyx", g, shifted)
    return out
