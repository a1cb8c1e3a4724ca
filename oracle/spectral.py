"""Second, independent evolution of the periodic scheme in Fourier space.

TEST INFRASTRUCTURE ONLY (see the package docstring).

On a periodic lattice the scheme is linear and shift invariant, so each
discrete wavenumber evolves on its own: collision is the 20x20 matrix
I + omega (G - I) of Eq. collision_vector with G built from the blocks
g_ij = 1/4 I + 1/(2c)(i A_x + j A_y) of Eq. stability_linear, and streaming
multiplies population (i,j) by exp(-i k.e_ij) (a pull from x - e_ij).  This
module assembles those matrices directly from the paper's matrix form, in
numpy, without calling the C oracle, so agreement between the two is a
genuine cross-check of both.
"""
from __future__ import annotations

import numpy as np

E = np.array([[1, 0], [0, 1], [-1, 0], [0, -1]])


def flux_matrices(kK: float, km: float):
    """A_x / c and A_y / c of Eq. stability_linear (Courant-number form)."""
    Ax = np.zeros((5, 5))
    Ay = np.zeros((5, 5))
    Ax[0, 2] = Ax[2, 0] = kK
    Ax[0, 3] = Ax[3, 0] = km
    Ax[1, 4] = Ax[4, 1] = km
    Ay[0, 4] = Ay[4, 0] = km
    Ay[1, 2] = Ay[2, 1] = kK
    Ay[1, 3] = Ay[3, 1] = -km
    return Ax, Ay


def g_blocks(kK: float, km: float):
    Ax, Ay = flux_matrices(kK, km)
    return np.stack([0.25 * np.eye(5) + 0.5 * (i * Ax + j * Ay) for i, j in E])


def G_matrix(kK: float, km: float):
    g = g_blocks(kK, km)
    return np.concatenate([np.concatenate([g[q]] * 4, axis=1) for q in range(4)], axis=0)


def collision_matrix(kK: float, km: float, omega: float = 2.0):
    return np.eye(20) + omega * (G_matrix(kK, km) - np.eye(20))


def evolve_periodic(f0: np.ndarray, kK: float, km: float, nsteps: int, omega: float = 2.0):
    """f0 [4][5][ny][nx] -> populations after nsteps (pre-collision), exactly
    as the lattice scheme with periodic wrap and no body load."""
    _, _, ny, nx = f0.shape
    C = collision_matrix(kK, km, omega)
    fh = np.fft.fft2(f0.reshape(20, ny, nx))              # [20][ny][nx]
    ky = np.fft.fftfreq(ny) * 2 * np.pi
    kx = np.fft.fftfreq(nx) * 2 * np.pi
    out = np.empty_like(fh)
    for a in range(ny):
        for b in range(nx):
            ph = np.exp(-1j * (E[:, 0] * kx[b] + E[:, 1] * ky[a]))
            S = np.diag(np.repeat(ph, 5))
            M = np.linalg.matrix_power(S @ C, nsteps)
            out[:, a, b] = M @ fh[:, a, b]
    return np.real(np.fft.ifft2(out)).reshape(4, 5, ny, nx)


def spectral_radius_periodic(kK: float, km: float, n: int = 16, omega: float = 2.0) -> float:
    """max over the n x n discrete wavenumbers of the one-step amplification
    matrix's spectral radius."""
    C = collision_matrix(kK, km, omega)
    k = np.fft.fftfreq(n) * 2 * np.pi
    r = 0.0
    for a in k:
        for b in k:
            ph = np.exp(-1j * (E[:, 0] * b + E[:, 1] * a))
            M = np.diag(np.repeat(ph, 5)) @ C
            r = max(r, float(np.abs(np.linalg.eigvals(M)).max()))
    return r


# ---------------------------------------------------------------------------
# Exact discrete evolution of periodic plane-wave data at any grid size
# ---------------------------------------------------------------------------
def _mode_table(fields):
    """Fourier content of real fields given as SinSums at t = 0.

    Returns {(a, b): complex[nf]} such that field_i(x, y) =
    Re(sum_k C_k[i] exp(i (a x + b y)))."""
    table = {}
    nf = len(fields)
    for i, s in enumerate(fields):
        for A, a, b, w, p in s.simplified().terms:
            z = -1j * A * np.exp(1j * p)       # A sin(th + p) = Re(-i A e^{ip} e^{i th})
            if (a, b) < (0.0, 0.0):
                a, b, z = -a, -b, np.conj(z)   # Re(z e^{-i th}) = Re(conj(z) e^{i th})
            key = (round(a, 9), round(b, 9))
            if key not in table:
                table[key] = (a, b, np.zeros(nf, dtype=complex))
            table[key][2][i] += z
    return table


def plane_wave_reference(setup, sol, nsteps: int, iy, ix):
    """U(t_n) of the lattice scheme with central-difference initialisation,
    for periodic plane-wave data, at the nodes (iy, ix).

    The scheme is linear and shift invariant on a periodic lattice, so every
    Fourier mode exp(i k.x) of the initial data evolves alone.  For each mode
    the initial populations are obtained from the C oracle's initialisation
    (Eq. ic_second) on a 5x5 patch (the centre node sees only interior central
    differences), split into real and imaginary parts; the amplitudes are
    advanced by (S(k) C)^n and summed at the requested nodes."""
    import oracle  # the C oracle, for the initialisation on a patch

    r = setup.rho
    fields = [sol.vx, sol.vy, sol.sxx * r, sol.syy * r, sol.sxy * r]
    table = _mode_table(fields)
    dx = setup.dx
    C = collision_matrix(setup.kK, setup.km)
    patch = oracle.Setup(5, 5, dx, setup.dt, (setup.cK ** 2 - setup.cmu ** 2) * r,
                         setup.cmu ** 2 * r, r, oracle.DIRICHLET)
    xs = (np.arange(5) + 0.5) * dx
    PX, PY = np.meshgrid(xs, xs)
    xc, yc = xs[2], xs[2]
    iy = np.asarray(iy)
    ix = np.asarray(ix)
    X = (ix + 0.5) * dx
    Y = (iy + 0.5) * dx
    out = np.zeros((5,) + iy.shape)
    for a, b, Ck in table.values():
        ph = np.exp(1j * (a * PX + b * PY))
        parts = []
        for comp in (np.real, np.imag):
            v = np.stack([comp(Ck[i] * ph) for i in range(2)])
            sb = np.stack([comp(Ck[i] * ph) for i in range(2, 5)])
            U0 = setup.U_from_fields(v, sb)
            parts.append(oracle.init_populations(patch, U0)[:, :, 2, 2].reshape(20))
        amp = (parts[0] + 1j * parts[1]) * np.exp(-1j * (a * xc + b * yc))
        phase = np.exp(-1j * (E[:, 0] * a * dx + E[:, 1] * b * dx))
        M = np.diag(np.repeat(phase, 5)) @ C
        an = np.linalg.matrix_power(M, nsteps) @ amp
        Un = an.reshape(4, 5).sum(0)
        out += np.real(Un[:, None] * np.exp(1j * (a * X + b * Y)).reshape(1, -1)).reshape(out.shape)
    return out
