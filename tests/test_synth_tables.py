"""The separable tables handed to the library (body load, wall velocity)
reproduce the closed-form data they are built from (addition theorems only;
no scheme arithmetic is involved)."""
import math

import numpy as np
import pytest

import synth


def _problem(sol_fn, mat, N, bc):
    ux, uy = sol_fn()
    e = synth.Elastodynamics(ux, uy, mat)
    dx = 1.0 / N
    lam, mu = (mat.cK2 - mat.cmu2) * mat.rho, mat.cmu2 * mat.rho
    return synth.Problem(N, N + 3, dx, 0.3 * dx, lam, mu, mat.rho, bc, sol=e)


@pytest.mark.parametrize("sol_fn", [synth.standing_mms_solution, synth.periodic_moving_solution])
def test_body_table_sums_to_body_load(sol_fn):
    mat = synth.Material(1.1, 0.4, 1.7)
    prob = _problem(sol_fn, mat, 24, synth.PERIODIC)
    X, Y, T = prob.body_table(9)
    assert X.shape[1:] == (2, prob.nx) and Y.shape == (X.shape[0], prob.ny)
    assert T.shape == (10, X.shape[0])
    Xn, Yn = synth.node_coords(prob.nx, prob.ny, prob.dx)
    for n in (0, 4, 9):
        got = np.einsum("rak,rl,r->alk", X, Y, T[n])
        want = prob.sol.body_force(Xn, Yn, n * prob.dt)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_body_table_empty_without_load():
    mat = synth.Material(1.1, 0.4, 1.0)
    pw = lambda: synth.plane_wave(2 * math.pi, 0.0, 0.1, 0.2, "P", mat)
    prob = _problem(pw, mat, 16, synth.PERIODIC)
    X, Y, T = prob.body_table(5)
    assert X.shape == (0, 2, 16) and Y.shape == (0, 19) and T.shape == (6, 0)


def test_wall_table_sums_to_wall_velocity():
    mat = synth.Material(1.1, 0.4, 1.0)
    prob = _problem(synth.periodic_moving_solution, mat, 20, synth.DIRICHLET)
    W, T = prob.wall_table(7, step0=3)
    for n in (0, 6):
        got = np.einsum("rlc,r->lc", W, T[n])
        want = prob.wall_velocity((3 + n + 0.5) * prob.dt)
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_reference_table_sums_to_exact_outputs():
    mat = synth.Material(1.1, 0.4, 1.7)
    prob = _problem(synth.periodic_moving_solution, mat, 20, synth.DIRICHLET)
    X, Y, T = prob.reference_table(6)
    assert X.shape[1:] == (7, prob.nx) and T.shape == (7, X.shape[0])
    Xn, Yn = synth.node_coords(prob.nx, prob.ny, prob.dx)
    for n in (0, 6):
        got = np.einsum("rck,rl,r->clk", X, Y, T[n])
        v, sb, u = prob.sol.fields(Xn, Yn, n * prob.dt)
        want = np.concatenate([u, v, sb])
        assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()
