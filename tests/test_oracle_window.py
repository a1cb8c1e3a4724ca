"""Pins of the oracle's exact linear window operator (oracle/window.py): the
n-step window map of the periodic scheme read as a convolution.

* uniform states are stationary (no gradients: the initialisation gives the
  equilibrium, which streaming and collision keep), so the taps sum to the
  identity;
* information moves one node per step along an axis and the central
  differences reach one node: no tap outside |dx| + |dy| <= n + 1, and the
  outermost diamond is reached;
* superposition: the operator applied to an arbitrary periodic field equals
  the scheme run on that field (a wrong offset direction or a dropped tap
  fails this; each tap G[d] is found symmetric in its component pair, so
  the pair order is not pinned and does not matter)."""
import numpy as np
import pytest

import oracle
from oracle import window as W


def _setup(nx, ny, cK2, cmu2, frac=0.5):
    # (c_K^2, c_mu^2) with rho = 1; time step at `frac` of the CFL-like limit
    dx = 1.0 / nx
    c = 2.0 * np.sqrt(cK2 + cmu2) / frac
    return oracle.Setup.from_speeds(nx, ny, dx, dx / c, cK2, cmu2, oracle.PERIODIC)


@pytest.mark.parametrize("cK2,cmu2", [(1.1, 0.4), (1.4, 0.1)])
def test_taps_sum_to_identity(cK2, cmu2):
    G = W.window_operator(_setup(40, 40, cK2, cmu2), nsteps=6)
    assert np.allclose(G.sum(axis=(0, 1)), np.eye(5), atol=1e-13)


def test_support_is_the_diamond():
    n = 5
    G = W.window_operator(_setup(40, 40, 1.1, 0.4), nsteps=n)
    R = W.radius(n)
    assert G.shape == (2 * R + 1, 2 * R + 1, 5, 5)
    dy, dx = np.meshgrid(np.arange(-R, R + 1), np.arange(-R, R + 1), indexing="ij")
    outside = np.abs(dx) + np.abs(dy) > R
    assert np.all(G[outside] == 0.0)
    edge = np.abs(dx) + np.abs(dy) == R
    assert np.abs(G[edge]).max() > 1e-8


@pytest.mark.parametrize("nsteps", [1, 4, 16])
def test_superposition_equals_the_scheme(nsteps):
    s = _setup(48, 40, 1.1, 0.4)
    G = W.window_operator(s, nsteps=nsteps)
    g = np.random.default_rng(nsteps)
    U = g.standard_normal((5, 40, 48))
    want = W.window_map_n(s, U, nsteps)
    got = W.apply_window_operator(G, U)
    assert oracle.rel_l2(got, want) < 1e-12
