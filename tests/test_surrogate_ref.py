"""Pins of the FP64 surrogate reference: convolution against scipy's
correlation, adjoint identities, and finite-difference gradients of the whole
network loss."""
import math

import numpy as np
import pytest
from scipy import signal

from oracle import surrogate_ref as S


@pytest.mark.parametrize("circular", [True, False])
def test_conv_matches_scipy(circular):
    g = np.random.default_rng(0)
    x = g.standard_normal((2, 8, 6, 3))
    w = g.standard_normal((4, 3, 3, 3))
    z = S.conv3x3(x, w, circular)
    for b in range(2):
        for o in range(4):
            ref = np.zeros((8, 6))
            for i in range(3):
                img = x[b, :, :, i]
                if circular:
                    img = np.pad(img, 1, mode="wrap")
                    ref += signal.correlate2d(img, w[o, i], mode="valid")
                else:
                    ref += signal.correlate2d(img, w[o, i], mode="same", boundary="fill")
            assert np.allclose(z[b, :, :, o], ref, atol=1e-12)


@pytest.mark.parametrize("circular", [True, False])
def test_conv_backward_is_adjoint(circular):
    g = np.random.default_rng(1)
    x = g.standard_normal((2, 5, 4, 3))
    w = g.standard_normal((2, 3, 3, 3))
    gz = g.standard_normal((2, 5, 4, 2))
    gx, gw = S.conv3x3_backward(x, w, gz, circular)
    # <conv(x), gz> = <x, gx>  and  d<conv(x;w), gz>/dw = gw
    assert abs(np.sum(S.conv3x3(x, w, circular) * gz) - np.sum(x * gx)) < 1e-10
    dw = g.standard_normal(w.shape)
    lhs = np.sum(S.conv3x3(x, dw, circular) * gz)
    assert abs(lhs - np.sum(dw * gw)) < 1e-10


def test_pool_up_adjoints():
    g = np.random.default_rng(2)
    x = g.standard_normal((1, 4, 6, 2))
    y = g.standard_normal((1, 2, 3, 2))
    assert abs(np.sum(S.pool2(x) * y) - np.sum(x * S.pool2_backward(y))) < 1e-12
    assert abs(np.sum(S.up2(y) * x) - np.sum(y * S.up2_backward(x))) < 1e-12


def test_field_conversion_roundtrip():
    g = np.random.default_rng(3)
    inp = _input(g, 2, 16, 16)
    cK, cm, rho = S.material_speeds(inp)
    f = inp[:, :5]
    assert np.allclose(S.U_to_fields(S.fields_to_U(f, cK, cm, rho), cK, cm, rho), f)


def _input(g, B, H, W):
    inp = np.zeros((B, 8, H, W))
    inp[:, :5] = g.standard_normal((B, 5, H, W))
    nu = g.uniform(0, 0.49, B)
    lam = 2 * nu / (1 - 2 * nu)
    rho = g.uniform(0.5, 2.0, B)
    inp[:, 5] = lam[:, None, None]
    inp[:, 6] = 1.0
    inp[:, 7] = rho[:, None, None]
    return inp


@pytest.mark.parametrize("circular", [True, False])
def test_network_gradient_finite_differences(circular):
    g = np.random.default_rng(4)
    inp = _input(g, 2, 16, 16)
    tgt = inp[:, :5] + 0.1 * g.standard_normal((2, 5, 16, 16))
    P = S.init_params(seed=5)
    for k in P:
        if k.endswith(".a"):
            P[k] = P[k] + 0.2 * g.standard_normal(P[k].shape)
    fw = S.Forward(P, inp, circular)
    fw.loss(tgt)
    G = fw.backward()
    for key in ("in.w", "e1a.w", "e3b.w", "d1b.w", "out.w", "e2a.a", "out.a", "d0a.a"):
        idx = tuple(g.integers(0, n) for n in P[key].shape)
        h = 1e-6 * max(1.0, abs(P[key][idx]))
        P[key][idx] += h
        lp = S.Forward(P, inp, circular).loss(tgt)
        P[key][idx] -= 2 * h
        lm = S.Forward(P, inp, circular).loss(tgt)
        P[key][idx] += h
        fd = (lp - lm) / (2 * h)
        assert abs(fd - G[key][idx]) <= 1e-6 * max(abs(fd), 1e-8) + 1e-11, (key, fd, G[key][idx])


def test_identity_network_reproduces_input():
    # zero output layer: the surrogate returns its input fields exactly
    g = np.random.default_rng(6)
    inp = _input(g, 2, 16, 16)
    P = S.init_params(seed=1)
    P["out.w"][:] = 0
    fw = S.Forward(P, inp, True)
    assert np.allclose(fw.out, inp[:, :5], atol=1e-12)


def test_chebyshev_basis_is_cos_n_theta():
    # T_n(cos theta) = cos(n theta): catches a wrong recurrence or order
    theta = np.linspace(0.0, math.pi, 37)
    T = S.chebyshev(np.cos(theta))
    assert T.shape == (37, S.NBASIS)
    for n in range(S.NBASIS):
        assert np.allclose(T[:, n], np.cos(n * theta), atol=1e-14), n


def _material_input(theta, rho=1.3):
    # per-sample material with atan2(c_mu, c_K) = theta and c_K^2 + c_mu^2 = 2
    cK, cm = math.sqrt(2) * math.cos(theta), math.sqrt(2) * math.sin(theta)
    inp = np.zeros((1, 8, 4, 4))
    inp[:, 6] = rho * cm * cm             # mu
    inp[:, 5] = rho * cK * cK - inp[:, 6]  # lambda (c_K^2 = (lambda + mu) / rho)
    inp[:, 7] = rho
    return inp


def test_conditioning_maps_the_angle_range_to_unit_interval():
    # the end points of the angle range go to -1 and +1, its midpoint to 0,
    # and the map is affine in theta in between
    lo, hi = S.THETA_LO, S.THETA_HI
    for theta, want in ((lo, -1.0), (hi, 1.0), (0.5 * (lo + hi), 0.0),
                        (lo + 0.25 * (hi - lo), -0.5)):
        assert abs(S.conditioning(_material_input(theta))[0] - want) < 1e-12, theta


def test_pool_and_upsample_values():
    # 2 x 2 means and nearest-neighbour copies, on a known array
    x = np.arange(16.0).reshape(1, 4, 4, 1)
    assert np.array_equal(S.pool2(x)[0, :, :, 0], [[2.5, 4.5], [10.5, 12.5]])
    y = np.array([[1.0, 2.0], [3.0, 4.0]]).reshape(1, 2, 2, 1)
    assert np.array_equal(S.up2(y)[0, :, :, 0], [[1, 1, 2, 2], [1, 1, 2, 2],
                                                  [3, 3, 4, 4], [3, 3, 4, 4]])


def test_fields_to_U_matches_oracle_conversion():
    # the surrogate's pre-map and the lattice oracle's conversion (pinned by
    # the oracle tests through Eq. sigma_num) agree for per-sample materials
    import oracle
    g = np.random.default_rng(8)
    inp = _input(g, 3, 6, 5)
    cK, cm, rho = S.material_speeds(inp)
    U = S.fields_to_U(inp[:, :5], cK, cm, rho)
    for b in range(3):
        lam, mu, r = inp[b, 5, 0, 0], inp[b, 6, 0, 0], inp[b, 7, 0, 0]
        s = oracle.Setup(5, 6, 1.0, 0.01, lam, mu, r, oracle.PERIODIC)
        want = s.U_from_fields(inp[b, :2], inp[b, 2:5])
        assert np.allclose(U[b], want, rtol=1e-13, atol=1e-13), b


def test_adam_constant_gradient_moves_lr_per_step():
    # with a constant gradient g the bias-corrected moments are exactly g and
    # g^2 at every step, so each step moves by lr g / (|g| + eps): after n
    # steps P = P0 - n lr g / (|g| + eps) (a missing or wrong bias correction
    # makes the early steps shorter or longer)
    g = np.random.default_rng(9)
    grad = g.standard_normal((7, 3))
    P = {"w": g.standard_normal((7, 3))}
    P0 = P["w"].copy()
    M, V = {"w": np.zeros((7, 3))}, {"w": np.zeros((7, 3))}
    lr, eps = 1e-2, 1e-8
    for n in range(1, 6):
        S.adam_update(P, {"w": grad}, M, V, n, lr, eps=eps)
        want = P0 - n * lr * grad / (np.abs(grad) + eps)
        assert np.allclose(P["w"], want, rtol=0, atol=1e-13), n
