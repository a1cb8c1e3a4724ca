"""FP64 CPU reference of the learned window surrogate (forward, loss and
backward), used to check the HIP kernels.

TEST INFRASTRUCTURE ONLY (see the package docstring).  The surrogate is not
part of the paper: it is a small convolutional time-stepper that maps the
macroscopic fields of a lattice (velocity and Cauchy stress, plus Lame
constants and density) to the fields 16 lattice steps later.  Parity against
the paper is therefore unpinned; this reference is pinned instead (tests) by
scipy's correlation routine, adjoint identities and finite-difference
gradients, T_n(cos theta) = cos(n theta) for the Chebyshev basis and the end
points of the conditioning map, known values of pooling and up-sampling, the
field conversion against the lattice oracle's (Eq. sigma_num), and the
closed form of Adam under a constant gradient (n steps move n lr g/(|g|+eps)).

Network (everything in float64 here):
  pre    physical fields -> first-order system variables U (inverse of
         Eq. sigma_num), divided by the per-sample RMS s of U; channels padded
         to 32 with zeros.  Conditioning scalar t in [-1, 1] from the angle
         theta = atan2(c_mu, c_K) (the time step is taken at half the CFL-like
         limit, so theta fixes both Courant numbers).
  body   linear U-Net without biases or activations: 3x3 convolutions (circular
         padding for periodic, zero padding for Dirichlet data), two per level
         on 4 levels (32, 64, 128, 128 channels), 2x2 average pooling down,
         nearest-neighbour up-sampling plus an additive skip on the way up;
         every convolution output channel c of sample b is multiplied by
         gamma[b, c] = sum_m a[c, m] T_m(t_b) (Chebyshev T_0..T_3).
  post   U' = U + s * y[..., :5]; back to physical fields.
  loss   mean over (b, c < 5, pixels) of (y[..., :5] - (U_target - U)/s)^2.
"""
from __future__ import annotations

import math

import numpy as np

NBASIS = 4
CPAD = 32
THETA_LO = math.radians(8.0)
THETA_HI = math.radians(45.0)

# (name, cin, cout, level); level 0 is full resolution
LAYERS = [("in", 32, 32, 0), ("e0a", 32, 32, 0), ("e0b", 32, 32, 0),
          ("e1a", 32, 64, 1), ("e1b", 64, 64, 1),
          ("e2a", 64, 128, 2), ("e2b", 128, 128, 2),
          ("e3a", 128, 128, 3), ("e3b", 128, 128, 3),
          ("d2a", 128, 128, 2), ("d2b", 128, 64, 2),
          ("d1a", 64, 64, 1), ("d1b", 64, 32, 1),
          ("d0a", 32, 32, 0), ("d0b", 32, 32, 0), ("out", 32, 32, 0)]


def chebyshev(t, n=NBASIS):
    T = [np.ones_like(t), t]
    for _ in range(2, n):
        T.append(2 * t * T[-1] - T[-2])
    return np.stack(T[:n], axis=-1)


def init_params(seed=0, scale=1.0):
    """Weights [cout][cin][3][3] and FiLM coefficients [cout][NBASIS]."""
    g = np.random.default_rng(seed)
    P = {}
    for name, ci, co, _ in LAYERS:
        fan = 9 * ci
        P[name + ".w"] = g.standard_normal((co, ci, 3, 3)) * scale / math.sqrt(fan)
        a = np.zeros((co, NBASIS))
        a[:, 0] = 1.0
        P[name + ".a"] = a
    return P


# ---------------------------------------------------------------------------
# primitives (NHWC, float64)
# ---------------------------------------------------------------------------
def conv3x3(x, w, circular):
    """z[b,y,x,o] = sum_{i,dy,dx} w[o,i,dy+1,dx+1] x[b,y+dy,x+dx,i]."""
    B, H, W, C = x.shape
    if circular:
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="wrap")
    else:
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    z = np.zeros((B, H, W, w.shape[0]))
    for ky in range(3):
        for kx in range(3):
            z += xp[:, ky:ky + H, kx:kx + W, :] @ w[:, :, ky, kx].T
    return z


def conv3x3_backward(x, w, gz, circular):
    """Gradients of conv3x3 w.r.t. x and w given gz = dL/dz."""
    B, H, W, C = x.shape
    if circular:
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)), mode="wrap")
    else:
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    gw = np.zeros_like(w)
    gxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            win = xp[:, ky:ky + H, kx:kx + W, :]
            gw[:, :, ky, kx] = np.einsum("bhwo,bhwi->oi", gz, win)
            gxp[:, ky:ky + H, kx:kx + W, :] += gz @ w[:, :, ky, kx]
    if circular:
        gx = gxp[:, 1:-1, 1:-1, :].copy()
        gx[:, -1, :, :] += gxp[:, 0, 1:-1, :]
        gx[:, 0, :, :] += gxp[:, -1, 1:-1, :]
        gx[:, :, -1, :] += gxp[:, 1:-1, 0, :]
        gx[:, :, 0, :] += gxp[:, 1:-1, -1, :]
        gx[:, -1, -1, :] += gxp[:, 0, 0, :]
        gx[:, -1, 0, :] += gxp[:, 0, -1, :]
        gx[:, 0, -1, :] += gxp[:, -1, 0, :]
        gx[:, 0, 0, :] += gxp[:, -1, -1, :]
    else:
        gx = gxp[:, 1:-1, 1:-1, :].copy()
    return gx, gw


def pool2(x):
    B, H, W, C = x.shape
    return x.reshape(B, H // 2, 2, W // 2, 2, C).mean(axis=(2, 4))


def pool2_backward(g):
    return np.repeat(np.repeat(g, 2, axis=1), 2, axis=2) * 0.25


def up2(x):
    return np.repeat(np.repeat(x, 2, axis=1), 2, axis=2)


def up2_backward(g):
    B, H, W, C = g.shape
    return g.reshape(B, H // 2, 2, W // 2, 2, C).sum(axis=(2, 4))


# ---------------------------------------------------------------------------
# pre / post
# ---------------------------------------------------------------------------
def material_speeds(inp):
    """inp [B][8][H][W]: channel 5 = lambda, 6 = mu, 7 = rho (per pixel)."""
    lam, mu, rho = inp[:, 5], inp[:, 6], inp[:, 7]
    cK = np.sqrt((lam + mu) / rho)
    cm = np.sqrt(mu / rho)
    return cK, cm, rho


def fields_to_U(f, cK, cm, rho):
    """f [B][5][H][W] physical (v, sigma_bar) -> U [B][5][H][W]."""
    s = f[:, 2:] / rho[:, None]
    U = np.empty_like(f)
    U[:, 0], U[:, 1] = f[:, 0], f[:, 1]
    U[:, 2] = -(s[:, 0] + s[:, 1]) / (2 * cK)
    U[:, 3] = -(s[:, 0] - s[:, 1]) / (2 * cm)
    U[:, 4] = -s[:, 2] / cm
    return U


def U_to_fields(U, cK, cm, rho):
    f = np.empty_like(U)
    f[:, 0], f[:, 1] = U[:, 0], U[:, 1]
    f[:, 2] = -rho * (cK * U[:, 2] + cm * U[:, 3])
    f[:, 3] = -rho * (cK * U[:, 2] - cm * U[:, 3])
    f[:, 4] = -rho * cm * U[:, 4]
    return f


def conditioning(inp):
    cK, cm, _ = material_speeds(inp)
    theta = np.arctan2(cm.mean(axis=(1, 2)), cK.mean(axis=(1, 2)))
    return 2 * (theta - THETA_LO) / (THETA_HI - THETA_LO) - 1


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
class Forward:
    """Forward pass with everything kept for the backward pass."""

    def __init__(self, P, inp, circular):
        self.P, self.circular = P, circular
        cK, cm, rho = material_speeds(inp)
        self.cK, self.cm, self.rho = cK, cm, rho
        U = fields_to_U(inp[:, :5], cK, cm, rho)
        self.U = U
        self.s = np.sqrt(np.mean(U ** 2, axis=(1, 2, 3)))
        self.t = conditioning(inp)
        self.T = chebyshev(self.t)                       # [B][NBASIS]
        B, _, H, W = inp.shape
        x0 = np.zeros((B, H, W, CPAD))
        x0[..., :5] = np.transpose(U / self.s[:, None, None, None], (0, 2, 3, 1))
        self.x0 = x0
        self.z, self.gam, self.xin = {}, {}, {}
        y = {}

        def conv(name, x):
            self.xin[name] = x
            z = conv3x3(x, P[name + ".w"], circular)
            gam = self.T @ P[name + ".a"].T              # [B][cout]
            self.z[name], self.gam[name] = z, gam
            y[name] = z * gam[:, None, None, :]
            return y[name]

        h = conv("in", x0)
        h = conv("e0a", h)
        s0 = conv("e0b", h)
        h = conv("e1a", pool2(s0))
        s1 = conv("e1b", h)
        h = conv("e2a", pool2(s1))
        s2 = conv("e2b", h)
        h = conv("e3a", pool2(s2))
        h = conv("e3b", h)
        h = conv("d2a", up2(h) + s2)
        h = conv("d2b", h)
        h = conv("d1a", up2(h) + s1)
        h = conv("d1b", h)
        h = conv("d0a", up2(h) + s0)
        h = conv("d0b", h)
        yo = conv("out", h)
        self.y = y
        self.yout = yo[..., :5]                          # [B][H][W][5]
        Unew = U + self.s[:, None, None, None] * np.transpose(self.yout, (0, 3, 1, 2))
        self.Unew = Unew
        self.out = U_to_fields(Unew, cK, cm, rho)

    def loss(self, target):
        Ut = fields_to_U(target, self.cK, self.cm, self.rho)
        d = np.transpose(self.yout, (0, 3, 1, 2)) - (Ut - self.U) / self.s[:, None, None, None]
        self.diff = d
        return float(np.mean(d ** 2))

    def backward(self):
        """Gradients of the loss w.r.t. every parameter (dict like P)."""
        P, circ = self.P, self.circular
        B, _, H, W = self.U.shape
        G = {}
        g = np.zeros((B, H, W, CPAD))
        g[..., :5] = np.transpose(2 * self.diff / self.diff.size, (0, 2, 3, 1))

        def conv_back(name, gy):
            z, gam = self.z[name], self.gam[name]
            G[name + ".a"] = np.einsum("bc,bm->cm", np.einsum("bhwc,bhwc->bc", gy, z), self.T)
            gz = gy * gam[:, None, None, :]
            gx, gw = conv3x3_backward(self.xin[name], P[name + ".w"], gz, circ)
            G[name + ".w"] = gw
            return gx

        h = conv_back("out", g)
        h = conv_back("d0b", h)
        gu0 = conv_back("d0a", h)           # d/d(up2(d1b) + s0)
        h = conv_back("d1b", up2_backward(gu0))
        gu1 = conv_back("d1a", h)
        h = conv_back("d2b", up2_backward(gu1))
        gu2 = conv_back("d2a", h)
        h = conv_back("e3b", up2_backward(gu2))
        h = conv_back("e3a", h)
        gs2 = pool2_backward(h) + gu2
        h = conv_back("e2b", gs2)
        h = conv_back("e2a", h)
        gs1 = pool2_backward(h) + gu1
        h = conv_back("e1b", gs1)
        h = conv_back("e1a", h)
        gs0 = pool2_backward(h) + gu0
        h = conv_back("e0b", gs0)
        h = conv_back("e0a", h)
        conv_back("in", h)
        return G


def adam_update(P, G, M, V, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected), in place."""
    for k in P:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        V[k] = b2 * V[k] + (1 - b2) * G[k] ** 2
        mh = M[k] / (1 - b1 ** step)
        vh = V[k] / (1 - b2 ** step)
        P[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
