"""Invariants of the oracle that hold exactly (to roundoff) by the paper's
analysis: initialisation identity, energy isometry (Props. stab_periodic and
stability_dbc), conservation, brute-force transition matrices on tiny grids,
exact rigid translation through Dirichlet walls, and agreement with the
independent Fourier-space evolution."""
import json
import os

import numpy as np
import pytest

import oracle
from oracle import Setup, spectral

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_init_zeroth_moment_identity():
    # Eq. ic_second: the dt/8 correction has zero zeroth moment except the
    # -B/2 part, so sum_ij f_ij(0) + dt/2 B = U0 exactly (Section 4.2)
    s = Setup(16, 12, 1 / 16, 1 / 48, 1.0, 0.5, 1.3, oracle.PERIODIC)
    g = np.random.default_rng(0)
    U0 = g.standard_normal((5, 12, 16))
    UX = g.standard_normal((5, 12, 16))
    UY = g.standard_normal((5, 12, 16))
    B0 = g.standard_normal((2, 12, 16))
    f = oracle.init_populations(s, U0, UX, UY, B0)
    tot = f.sum(0)
    tot[:2] += 0.5 * B0
    assert np.abs(tot - U0).max() < 1e-14


def test_uniform_state_initialises_to_equilibrium():
    s = Setup(6, 5, 0.1, 0.01, 2.0, 1.0, 1.0, oracle.DIRICHLET)
    U0 = np.zeros((5, 5, 6)) + np.array([0.3, -0.2, 0.7, 0.1, -0.4])[:, None, None]
    f = oracle.init_populations(s, U0)   # central differences vanish
    feq = spectral.g_blocks(s.kK, s.km) @ U0[:, 0, 0]  # f_eq = g_ij U (Eq. stability_linear)
    assert np.allclose(f[:, :, 2, 3], feq, atol=1e-15)


@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.DIRICHLET])
@pytest.mark.parametrize("cK2,cmu2", [(1.1, 0.4), (1.4, 0.1), (0.2, 1.3)])
def test_energy_isometry_random_state(bc, cK2, cmu2):
    # ||f||_P is constant for b = 0 with periodic or homogeneous Dirichlet
    # boundaries (Props. stab_periodic, stability_dbc); the paper reports a
    # maximal relative drift of 3.4e-15 (Section 6.2)
    s = Setup.from_speeds(24, 20, 1 / 160, 1 / 400, cK2, cmu2, bc)
    f = np.random.default_rng(7).standard_normal((4, 5, 20, 24))
    E0 = oracle.energy(s, f)
    f2 = oracle.run_free(s, f, 10000)
    assert abs(oracle.energy(s, f2) - E0) / E0 < 1e-13


def test_paper_stability_run_drift():
    # Section 6.2: homogeneous Dirichlet, unit square, dx = 1/160,
    # dt = 1/400, (cK^2, cmu^2) = (1.1, 0.4), b = 0, t_f = 10 T (4000 steps)
    gold = json.load(open(os.path.join(GOLDEN, "paper_stability_test.json")))
    import synth
    s = Setup.from_speeds(160, 160, gold["dx"], gold["dt"], gold["cK2"], gold["cmu2"],
                          oracle.DIRICHLET)
    assert abs(s.cfl - gold["cfl_ratio"]) < 0.005
    mat = synth.Material(gold["cK2"], gold["cmu2"], 1.0)
    ux, uy = synth.stability_test_solution()
    e = synth.Elastodynamics(ux, uy, mat)
    X, Y = s.nodes()
    v0, sb0, u0 = e.fields(X, Y, 0.0)
    sim = oracle.Simulation(s, v0, sb0, e.field_gradients(X, Y, 0.0))
    E0 = oracle.energy(s, sim.f)
    drift = 0.0
    f = sim.f
    for _ in range(gold["steps"] // 100):
        f = oracle.run_free(s, f, 100)
        drift = max(drift, abs(oracle.energy(s, f) - E0) / E0)
    assert drift < 10 * gold["max_rel_drift"]


def test_unstable_parameters_diverge():
    # ratio 1.01 (Section 6.2: (1.2, 0.4) at c = 2.5) diverges within a few
    # hundred steps; ratio 0.98 stays flat
    g = np.random.default_rng(11)
    f0 = g.standard_normal((4, 5, 40, 40))
    for cK2, grows in ((1.1, False), (1.2, True)):
        s = Setup.from_speeds(40, 40, 1 / 160, 1 / 400, cK2, 0.4, oracle.DIRICHLET,
                              allow_unstable=True)
        f = oracle.run_free(s, f0, 500)
        ratio = np.sum(f * f) / np.sum(f0 * f0)
        assert (ratio > 1e6) == grows, (cK2, ratio)


def test_spectral_radius_at_paper_points():
    # one-step amplification: exactly 1 below the limit, > 1 above
    c = 2.5
    for cK2, stable in ((1.1, True), (1.2, False)):
        kK, km = np.sqrt(cK2) / c, np.sqrt(0.4) / c
        r = spectral.spectral_radius_periodic(kK, km, 16)
        if stable:
            assert abs(r - 1.0) < 1e-9
        else:
            assert r > 1.01


def test_periodic_sum_conserved():
    s = Setup.from_speeds(13, 9, 0.1, 0.03, 1.5, 0.5, oracle.PERIODIC)
    f = np.random.default_rng(2).standard_normal((4, 5, 9, 13))
    f2 = oracle.run_free(s, f, 137)
    assert np.allclose(f2.sum(axis=(0, 2, 3)), f.sum(axis=(0, 2, 3)), atol=1e-11)


@pytest.mark.parametrize("nx,ny", [(7, 5), (8, 8), (1, 6), (5, 1), (2, 3)])
def test_matches_fourier_space_evolution(nx, ny):
    # independent second implementation: (S(k) C)^n per wavenumber
    s = Setup.from_speeds(nx, ny, 0.1, 0.036, 1.3, 0.35, oracle.PERIODIC)
    f0 = np.random.default_rng(nx * 10 + ny).standard_normal((4, 5, ny, nx))
    n = 23
    a = oracle.run_free(s, f0, n)
    b = spectral.evolve_periodic(f0, s.kK, s.km, n)
    assert np.abs(a - b).max() < 1e-12 * max(1.0, np.abs(b).max())


def _transition_matrix(s):
    n = 20 * s.nx * s.ny
    M = np.empty((n, n))
    for col in range(n):
        e = np.zeros(n)
        e[col] = 1.0
        fn, _, _ = oracle.step(s, e.reshape(4, 5, s.ny, s.nx))
        M[:, col] = fn.reshape(n)
    return M


def _weight_matrix(s):
    k = oracle.norm_weights(s.kK, s.km)
    n = s.nx * s.ny
    K = np.zeros((20 * n, 20 * n))
    for q in range(4):
        for node in range(n):
            idx = [(q * 5 + c) * n + node for c in range(5)]
            K[np.ix_(idx, idx)] = k[q]
    return K


@pytest.mark.parametrize("bc", [oracle.PERIODIC, oracle.DIRICHLET])
@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 3), (2, 2), (3, 2), (4, 3), (3, 4)])
def test_brute_force_isometry_tiny_grids(bc, nx, ny):
    # assemble the full one-step map and check M^T K M = K, i.e. the scheme
    # is an isometry of the weighted grid norm for every state, including all
    # corner and single-row configurations of the wall rule
    s = Setup.from_speeds(nx, ny, 0.1, 0.04, 1.1, 0.4, bc)
    M = _transition_matrix(s)
    K = _weight_matrix(s)
    assert np.allclose(M.T @ K @ M, K, atol=1e-12)
    # and the map is invertible with M^{-1} = K^{-1} M^T K
    assert np.allclose(np.linalg.solve(K, M.T @ K) @ M, np.eye(len(M)), atol=1e-11)


@pytest.mark.parametrize("printed,exact", [(0.0, True), (1.0, True), (2.5, False)])
def test_rigid_translation_through_walls(printed, exact):
    # a uniform velocity with u_D moving at that velocity is an exact solution
    # (zero strain); the wall rule must reproduce it to roundoff.  This pins
    # the source rows 3-5 of Eq. bc_s to the Courant-number form; the
    # literally printed c_K, c_mu form agrees only when c = 1.
    c = 2.5 if printed != 1.0 else 1.0
    s = Setup.from_speeds(9, 7, 0.1, 0.1 / c, 0.02 * c * c, 0.01 * c * c, oracle.DIRICHLET)
    vel = np.array([0.7, -0.3])
    U0 = np.zeros((5, 7, 9))
    U0[0], U0[1] = vel[0], vel[1]
    f = oracle.init_populations(s, U0)
    wall = np.tile(vel, (s.wall_count(), 1))
    oracle.lib().orc_set_printed_wall_source(c if printed else 0.0)
    try:
        for _ in range(25):
            f, _, _ = oracle.step(s, f, wall=wall)
    finally:
        oracle.lib().orc_set_printed_wall_source(0.0)
    err = np.abs(oracle.moments(s, f) - U0).max()
    assert (err < 1e-13) == exact, err


@pytest.mark.parametrize("nx,ny,n", [(48, 32, 150), (40, 40, 333)])
def test_plane_wave_reference_matches_c_oracle(nx, ny, n):
    # per-mode exact discrete evolution (used for full-size GPU parity)
    # equals the C oracle run on the whole grid
    import synth
    prob = synth.plane_wave_problem(nx, ny, synth.PERIODIC, seed=4, nwaves=5, kmax=6)
    s = Setup(nx, ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, oracle.PERIODIC)
    v0, sb0 = prob.initial_fields()
    sim = oracle.Simulation(s, v0, sb0)
    sim.advance(n)
    want = sim.U()
    g = np.random.default_rng(0)
    iy = g.integers(0, ny, 300)
    ix = g.integers(0, nx, 300)
    got = spectral.plane_wave_reference(s, prob.sol, n, iy, ix)
    assert np.abs(got - want[:, iy, ix]).max() < 1e-11 * np.abs(want).max()
