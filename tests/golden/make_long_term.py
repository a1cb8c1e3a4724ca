"""Writes long_term_oracle.json: the FP64 oracle on the long-term test of
Section 6.2 (manufactured solution Eq. periodic_moving with its body load and
time-dependent Dirichlet walls on the unit square, (dx, dt) = (1/160, 1/400),
10^6 steps), for the stable pair (c_K^2, c_mu^2) = (1.1, 0.4) and, over the
first few hundred steps, the unstable pair (1.2, 0.4).

Recorded at checkpoints: the space-only relative L2 displacement error
L2rel^Omega(e^u) against the exact solution, the squared weighted norm
||f||_P^2 of the pre-collision populations, and at the last checkpoint the
numerical and exact displacement along the horizontal row l = 80.

Calls only oracle/ and synth/.  About half an hour on 4 cores:
    OMP_NUM_THREADS=4 python tests/golden/make_long_term.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

N, DX, DT = 160, 1.0 / 160, 1.0 / 400
STABLE_STEPS = [1000, 10000, 100000, 250000, 500000, 750000, 1000000]
UNSTABLE_STEPS = [100, 200, 300, 400, 500]
CUT_ROW = 80


def run(cK2, cmu2, checkpoints, allow_unstable):
    mat = synth.Material(cK2, cmu2, 1.0)
    e = synth.Elastodynamics(*synth.periodic_moving_solution(), mat)
    s = oracle.Setup.from_speeds(N, N, DX, DT, cK2, cmu2, oracle.DIRICHLET,
                                 allow_unstable=allow_unstable)
    X, Y = s.nodes()
    xb, yb = s.wall_points()
    # body load b_bar = rho b from its separable form (the same closed form,
    # evaluated as a small matrix product per step)
    BX, BY, _ = synth.separable_body_table(e, N, N, DX, DT, 0)
    terms = [(A, w, p) for s_ in (e.bx, e.by) for A, a, b, w, p in s_.terms]
    R = BX.shape[0]
    Xf = BX.reshape(R, 2 * N)

    def time_row(t):
        out = np.empty(R)
        r = 0
        for _, w, _p in terms:
            ga = w * t
            out[r:r + 4] = (np.cos(ga), np.cos(ga), np.sin(ga), np.sin(ga))
            r += 4
        return out

    def body(t):
        B = BY.T @ (Xf * time_row(t)[:, None])        # [ny][2 nx]
        return np.ascontiguousarray(B.reshape(N, 2, N).transpose(1, 0, 2))

    ref = e.body_force(X, Y, 0.37)
    assert np.abs(body(0.37) - ref).max() <= 1e-12 * np.abs(ref).max()
    wall = lambda t: np.stack([e.vx(xb, yb, t), e.vy(xb, yb, t)], 1)
    v0, sb0, u0 = e.fields(X, Y, 0.0)
    sim = oracle.Simulation(s, v0, sb0, e.field_gradients(X, Y, 0.0), u0, body=body, wall=wall)
    out = {"steps": [], "l2rel_u": [], "energy": []}
    t0 = time.time()
    for n in checkpoints:
        sim.advance(n - sim.n)
        u = sim.displacement()
        ue = np.stack([e.ux(X, Y, sim.t()), e.uy(X, Y, sim.t())])
        err = float(np.sqrt(((u - ue) ** 2).sum() / (ue ** 2).sum()))
        out["steps"].append(n)
        out["l2rel_u"].append(err)
        out["energy"].append(float(oracle.energy(s, sim.f)))
        print("cK2=%.1f step %d: L2rel_u %.6e  (%.0f s)" % (cK2, n, err, time.time() - t0),
              flush=True)
    out["cut_row"] = CUT_ROW
    out["cut_u"] = u[:, CUT_ROW, :].tolist()
    out["cut_exact"] = ue[:, CUT_ROW, :].tolist()
    return out


def main():
    doc = {
        "_source": "arXiv 2408.01081, Section 6.2, long-term test (Eq. periodic_moving, "
                   "Dirichlet unit square, (dx, dt) = (1/160, 1/400), t_f = 2500 T = 10^6 steps); "
                   "values computed by the FP64 oracle with this script",
        "command": "OMP_NUM_THREADS=4 python tests/golden/make_long_term.py",
        "nx": N, "ny": N, "dx": DX, "dt": DT, "rho": 1.0,
        "stable": dict(cK2=1.1, cmu2=0.4, **run(1.1, 0.4, STABLE_STEPS, False)),
        "unstable": dict(cK2=1.2, cmu2=0.4, **run(1.2, 0.4, UNSTABLE_STEPS, True)),
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long_term_oracle.json")
    json.dump(doc, open(path, "w"), indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
