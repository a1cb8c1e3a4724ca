"""Pins of the oracle's local algebra against facts the paper fixes (Section 5)
and against an independent matrix-form assembly (oracle/spectral.py)."""
import math

import numpy as np
import pytest

import oracle
from oracle import Setup, spectral

D = np.diag([-1.0, -1.0, 1.0, 1.0, 1.0])
KAPPAS = [(0.2165, 0.125), (0.35, 0.1), (0.05, 0.45), (0.3, 0.3), (0.48, 0.01)]


@pytest.mark.parametrize("kK,km", KAPPAS)
def test_flux_matrices_symmetric_and_g_sum(kK, km):
    # Eq. stability_linear: A_x, A_y symmetric; sum_ij g_ij = I
    Ax, Ay = spectral.flux_matrices(kK, km)
    assert np.array_equal(Ax, Ax.T) and np.array_equal(Ay, Ay.T)
    g = spectral.g_blocks(kK, km)
    assert np.allclose(g.sum(0), np.eye(5), atol=1e-15)


@pytest.mark.parametrize("kK,km", KAPPAS)
def test_G_projector_and_collision_spectrum(kK, km):
    # G^2 = G (Section 5.2), spec(J) = {-omega, 0} with J = omega (G - I),
    # and at omega = 2 the collision I + J is an involution.
    G = spectral.G_matrix(kK, km)
    assert np.allclose(G @ G, G, atol=1e-14)
    J = 2.0 * (G - np.eye(20))
    ev = np.linalg.eigvals(J)
    assert np.all(np.minimum(np.abs(ev), np.abs(ev + 2.0)) < 1e-12)
    C = spectral.collision_matrix(kK, km)
    assert np.allclose(C @ C, np.eye(20), atol=1e-13)


@pytest.mark.parametrize("kK,km", KAPPAS)
def test_g_eigenvalues_closed_form(kK, km):
    # eig(g_ij) = 1/4 + 1/2 {0, +-sqrt(kK^2 + km^2), +-km}: positive iff Eq. stab_cond
    a = math.hypot(kK, km)
    want = np.sort([0.25, 0.25 + a / 2, 0.25 - a / 2, 0.25 + km / 2, 0.25 - km / 2])
    for g in spectral.g_blocks(kK, km):
        assert np.allclose(np.sort(np.linalg.eigvalsh(g)), want, atol=1e-14)


@pytest.mark.parametrize("kK,km", KAPPAS)
def test_norm_weights_inverse_and_reflection(kK, km):
    # C oracle's k_ij equal g_ij^{-1} from the independent assembly, and
    # k_{-i-j} = D^T k_ij D (Section 5.3)
    k = oracle.norm_weights(kK, km)
    g = spectral.g_blocks(kK, km)
    for q in range(4):
        assert np.allclose(k[q] @ g[q], np.eye(5), atol=1e-12)
        assert np.allclose(k[(q + 2) % 4], D.T @ k[q] @ D, atol=1e-12)
        assert np.all(np.linalg.eigvalsh(k[q]) > 0)


@pytest.mark.parametrize("kK,km", KAPPAS)
def test_C_collision_matches_matrix_form(kK, km):
    # A 1x1 periodic lattice streams every population onto itself, so one
    # oracle step is exactly the collision; compare with I + 2(G - I).
    s = Setup.from_speeds(1, 1, 1.0, 1.0, kK ** 2, km ** 2, oracle.PERIODIC)
    s.kK, s.km = kK, km
    g = np.random.default_rng(3)
    f = g.standard_normal((4, 5, 1, 1))
    fn, _, _ = oracle.step(s, f)
    want = spectral.collision_matrix(kK, km) @ f.reshape(20)
    assert np.allclose(fn.reshape(20), want, atol=1e-14)


def test_collision_conserves_moment_plus_force():
    # sum_ij f*_ij = sum_ij f_ij + dt B (omega = 2, Eq. cond_eq)
    s = Setup.from_speeds(1, 1, 1.0, 1.0, 0.05, 0.01, oracle.PERIODIC)
    g = np.random.default_rng(4)
    f = g.standard_normal((4, 5, 1, 1))
    B = g.standard_normal((2, 1, 1))
    fn, U, _ = oracle.step(s, f, Bhat=B, want_U=True)
    tot = f.sum(0)
    tot[:2] += B
    assert np.allclose(fn.sum(0), tot, atol=1e-14)
    assert np.allclose(U[:2], f.sum(0)[:2] + 0.5 * B, atol=1e-15)


def test_cfl_rejection():
    # Eq. stab_cond: the paper's pair (1.1, 0.4) at c = 2.5 is admissible,
    # (1.2, 0.4) is not (Section 6.2)
    s = Setup.from_speeds(8, 8, 1 / 160, 1 / 400, 1.1, 0.4, oracle.DIRICHLET)
    assert abs(s.cfl - 0.98) < 0.005
    with pytest.raises(oracle.CFLError):
        Setup.from_speeds(8, 8, 1 / 160, 1 / 400, 1.2, 0.4, oracle.DIRICHLET)


def test_material_models():
    # plane strain / 2D continuum share c_K^2 = (lambda + mu)/rho; plane stress
    # with the bulk modulus K = lambda + 2 mu/3 gives 9 K mu / ((3K + 4mu) rho)
    lam, mu, rho = 1.3, 0.7, 1.9
    s1 = Setup(4, 4, 1.0, 0.1, lam, mu, rho, 0)
    assert math.isclose(s1.cK ** 2, (3 * (lam + 2 * mu / 3) + mu) / (3 * rho))
    s2 = Setup(4, 4, 1.0, 0.1, lam, mu, rho, 0, model="plane_stress")
    K = lam + 2 * mu / 3
    assert math.isclose(s2.cK ** 2, 9 * K * mu / ((3 * K + 4 * mu) * rho))
    assert math.isclose(s2.cmu ** 2, mu / rho)


def test_field_conversion_roundtrip():
    s = Setup(4, 3, 1.0, 0.1, 1.0, 0.5, 1.7, 0)
    g = np.random.default_rng(5)
    v = g.standard_normal((2, 3, 4))
    sb = g.standard_normal((3, 3, 4))
    v2, sb2 = s.fields_from_U(s.U_from_fields(v, sb))
    assert np.allclose(v2, v) and np.allclose(sb2, sb)
