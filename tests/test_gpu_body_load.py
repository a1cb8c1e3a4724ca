"""Body load (Eq. cond_eq: U_num = sum f + B_hat / 2, B_hat = dt b_bar / rho)
and the trapezoidal displacement output (Section 3.5) on the HIP path,
against the FP64 oracle on manufactured solutions (Section 6.1) and against
the exact solution (second-order convergence).

Tolerance: as for the load-free path, FP32 populations accumulate about
2e-6 relative error over 1000 steps; the load table is FP32 too (relative
rounding ~1e-7 of B_hat per step), so the parity bar stays rel-L2 <= 1e-5."""
import numpy as np
import pytest

import oracle
import synth

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _mms(N, bc, sol_fn, mat, dt, ny=None):
    ux, uy = sol_fn()
    e = synth.Elastodynamics(ux, uy, mat)
    dx = 1.0 / N
    lam, mu = (mat.cK2 - mat.cmu2) * mat.rho, mat.cmu2 * mat.rho
    return synth.Problem(N, ny or N, dx, dt(dx), lam, mu, mat.rho, bc, sol=e)


def _run(prob, nsteps, tblock=None, with_disp=True):
    """GPU lattice and oracle simulation of prob, both advanced nsteps."""
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    e = prob.sol
    X, Y = synth.node_coords(prob.nx, prob.ny, prob.dx)
    v0, sb0, u0 = e.fields(X, Y, 0.0)
    grad = e.field_gradients(X, Y, 0.0)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                  displacement=with_disp)
    BX, BY, BT = prob.body_table(nsteps)
    assert BX.shape[0] > 0
    lat.set_body_force(*(torch.from_numpy(a) for a in (BX, BY, BT)))
    lat.init(torch.from_numpy(v0), torch.from_numpy(sb0), torch.from_numpy(grad))
    if with_disp:
        lat.init_displacement(torch.from_numpy(u0))
    if prob.bc == synth.DIRICHLET:
        W, T = prob.wall_table(nsteps)
        lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
    if tblock is not None:
        lat.tblock_config = tblock
    s = oracle.Setup(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    xb, yb = s.wall_points()
    wall = (lambda t: np.stack([e.vx(xb, yb, t), e.vy(xb, yb, t)], 1)) if prob.bc else None
    sim = oracle.Simulation(s, v0, sb0, grad, u0 if with_disp else None,
                            body=lambda t: e.body_force(X, Y, t), wall=wall)
    return lat, sim, s


@gpu
@pytest.mark.parametrize("bc,N,ny", [(synth.PERIODIC, 64, 64), (synth.PERIODIC, 67, 33),
                                     (synth.DIRICHLET, 40, 40), (synth.DIRICHLET, 37, 70)])
def test_init_with_load_matches_oracle(bc, N, ny):
    mat = synth.Material.from_lame(1.0, 0.5, 1.3)
    prob = _mms(N, bc, synth.standing_mms_solution, mat,
                lambda dx: synth.dt_at_cfl_fraction(dx, mat, 0.5), ny=ny)
    lat, sim, s = _run(prob, 1)
    got = lat.populations().double().cpu().numpy()
    assert np.abs(got - sim.f).max() < 1e-6 * np.abs(sim.f).max()
    U = lat.moments_U().double().cpu().numpy()
    assert oracle.rel_l2(U, sim.U()) < 1e-6
    u = lat.displacement().double().cpu().numpy()
    assert oracle.rel_l2(u, sim.displacement()) < 1e-6


# The standing solution's displacement carries cos(2 pi t): with dt = 0.4 dx
# on 64 nodes, 1000 steps end at t = 6.25, a zero of u, where any absolute
# error (including the FP32 error of v integrated over 1000 steps) is huge
# relative to |u|; 900 steps end at cos = -0.71.  Every case also bounds the
# displacement error relative to the initial displacement.
@gpu
@pytest.mark.parametrize("bc,N,ny,nsteps,sol", [
    (synth.PERIODIC, 64, 64, 900, "standing"),
    (synth.PERIODIC, 96, 50, 400, "moving"),
    (synth.DIRICHLET, 40, 40, 1000, "moving"),
    (synth.DIRICHLET, 53, 29, 300, "standing"),
])
def test_many_steps_with_load_and_displacement(bc, N, ny, nsteps, sol):
    torch = _torch()
    fn = synth.standing_mms_solution if sol == "standing" else synth.periodic_moving_solution
    mat = synth.Material(1.1, 0.4, 0.8)
    prob = _mms(N, bc, fn, mat, lambda dx: 0.4 * dx, ny=ny)
    # a blocked variant is selected but steps with a load run one per launch
    lat, sim, s = _run(prob, nsteps, tblock=10)
    lat.step(nsteps - 7)
    lat.step(7)
    sim.advance(nsteps)
    Uo = sim.U()
    U = lat.moments_U().double().cpu().numpy()
    err = oracle.rel_l2(U, Uo)
    u = lat.displacement().double().cpu().numpy()
    uerr = oracle.rel_l2(u, sim.displacement())
    print("%s bc=%d %dx%d n=%d: rel-L2 U %.3e u %.3e" % (sol, bc, N, ny, nsteps, err, uerr))
    assert err < 1e-5 and uerr < 1e-5
    u0 = prob.sol.fields(*synth.node_coords(prob.nx, prob.ny, prob.dx), 0.0)[2]
    assert np.sqrt(((u - sim.displacement()) ** 2).sum() / (u0 ** 2).sum()) < 1e-5
    # physical moments, device reductions and pre-collision populations at
    # the same level, all with B_hat(t_n)
    # (the physical moments map back to U: compared in U's balanced units,
    # since sigma_bar alone can be small next to the error in v)
    m = lat.moments().double().cpu().numpy()
    assert oracle.rel_l2(s.U_from_fields(m[:2], m[2:]), Uo) < 1e-5
    dev = lat.rel_l2(torch.from_numpy(Uo))
    assert abs(dev - err) <= 1e-3 * err + 1e-12
    f = lat.populations().double().cpu().numpy()
    assert oracle.rel_l2(f, sim.f) < 1e-5
    Ef = oracle.energy(s, f)
    assert abs(lat.energy() - Ef) <= 1e-6 * Ef


@gpu
def test_load_without_displacement():
    mat = synth.Material(1.1, 0.4, 1.0)
    prob = _mms(48, synth.PERIODIC, synth.periodic_moving_solution, mat, lambda dx: 0.4 * dx)
    lat, sim, s = _run(prob, 300, with_disp=False)
    lat.step(300)
    sim.advance(300)
    assert oracle.rel_l2(lat.moments_U().double().cpu().numpy(), sim.U()) < 1e-5
    with pytest.raises(RuntimeError):
        lat.displacement()


@gpu
def test_second_order_against_exact_solution():
    # standing manufactured solution on the periodic unit square at half the
    # CFL-like limit, fixed end time: 100/200/400 steps on 32/64/128 nodes
    mat = synth.Material.from_lame(1.0, 0.5, 1.0)
    errs = []
    for N, n in ((32, 100), (64, 200), (128, 400)):
        prob = _mms(N, synth.PERIODIC, synth.standing_mms_solution, mat,
                    lambda dx: synth.dt_at_cfl_fraction(dx, mat, 0.5))
        lat, _, s = _run(prob, n)
        lat.step(n)
        X, Y = synth.node_coords(N, N, prob.dx)
        v, sb, ue = prob.sol.fields(X, Y, n * prob.dt)
        u = lat.displacement().double().cpu().numpy()
        m = lat.moments().double().cpu().numpy()
        errs.append((oracle.rel_l2(u, ue), oracle.rel_l2(m[2:], sb)))
    print("final-time rel-L2 (u, sigma):", errs)
    for k in range(2):
        for a, b in zip(errs, errs[1:]):
            assert 3.8 < a[k] / b[k] < 4.2, errs


@gpu
def test_load_and_displacement_errors():
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    mat = synth.Material(1.1, 0.4, 1.0)
    prob = _mms(16, synth.PERIODIC, synth.standing_mms_solution, mat, lambda dx: 0.4 * dx)
    lat, _, _ = _run(prob, 5)
    lat.step(5)
    with pytest.raises(RuntimeError):
        lat.step(1)          # load table ends at t_5
    with pytest.raises(ValueError):
        lat.set_body_force(torch.zeros(2, 2, 16), torch.zeros(2, 15), torch.zeros(4, 2))
    # the displacement state must be started before stepping
    lat2 = Lattice(16, 16, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, synth.PERIODIC,
                   displacement=True)
    lat2.set_populations(torch.zeros(4, 5, 16, 16))
    with pytest.raises(RuntimeError):
        lat2.step(1)
    # and needs the flag
    lat3 = Lattice(16, 16, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, synth.PERIODIC)
    lat3.set_populations(torch.zeros(4, 5, 16, 16))
    with pytest.raises(RuntimeError):
        lat3.init_displacement(torch.zeros(2, 16, 16, dtype=torch.float64))
    # removing the load returns to the plain path
    lat.set_body_force(None, None, None)
    lat.step(3)


def _random_load(g, R, nx, ny, nsteps):
    """A seeded separable load table of rank R (arbitrary, not a solution's)."""
    return (0.5 * g.standard_normal((R, 2, nx)), g.standard_normal((R, ny)),
            g.standard_normal((nsteps + 1, R)))


@gpu
@pytest.mark.parametrize("bc,N,ny", [(synth.PERIODIC, 130, 64), (synth.PERIODIC, 70, 45),
                                     (synth.DIRICHLET, 300, 70), (synth.DIRICHLET, 61, 37)])
@pytest.mark.parametrize("R", [1, 5, 16, 17, 32, 33])
def test_blocked_steps_with_load_bitwise_equal_single_steps(bc, N, ny, R):
    # with a load of rank <= 32 and no displacement state the blocked kernel
    # steps T per launch (kernels for 16 and 32 ranks, the ranks below padded
    # with terms that add exactly nothing); rank 33 runs one step per launch;
    # every launch variant, through each load variant, gives the single-step
    # state bit for bit (Dirichlet with moving walls)
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(N, ny, bc, seed=23, kmax=3)
    v0, sb0 = prob.initial_fields()
    nsteps = 37
    g = np.random.default_rng(R)
    BX, BY, BT = (torch.from_numpy(a) for a in _random_load(g, R, N, ny, nsteps))
    W, T = prob.wall_table(nsteps)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    lat.set_body_force(BX, BY, BT)
    ref = None
    for cfg in [-1] + [c["index"] for c in lat.tblock_configs()]:
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        if bc == synth.DIRICHLET:
            lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg
        lat.step(11).step(nsteps - 11)
        f = lat.populations()
        if ref is None:
            ref = f
            assert torch.isfinite(f).all()
        else:
            assert torch.equal(f.view(torch.int32), ref.view(torch.int32)), cfg


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
def test_blocked_steps_with_load_match_oracle(bc):
    # the standing solution's load has rank 16 for these Lame parameters, so
    # the blocked kernel takes it (no displacement state)
    mat = synth.Material.from_lame(1.0, 0.5, 1.0)
    prob = _mms(64, bc, synth.standing_mms_solution, mat,
                lambda dx: synth.dt_at_cfl_fraction(dx, mat, 0.5), ny=48)
    assert prob.body_table(1)[0].shape[0] == 16
    lat, sim, s = _run(prob, 300, tblock=40 if bc == synth.PERIODIC else 19, with_disp=False)
    lat.step(296).step(4)
    sim.advance(300)
    err = oracle.rel_l2(lat.moments_U().double().cpu().numpy(), sim.U())
    print("blocked with load, bc=%d: rel-L2 %.3e" % (bc, err))
    assert err < 1e-5


@gpu
@pytest.mark.parametrize("bc,N,ny", [(synth.PERIODIC, 130, 64), (synth.DIRICHLET, 300, 70),
                                     (synth.DIRICHLET, 61, 37)])
@pytest.mark.parametrize("R", [0, 5, 16, 24])
def test_blocked_steps_with_displacement_bitwise_equal_single_steps(bc, N, ny, R):
    # with the FP64 displacement state (and a load of rank <= 16, or none)
    # the blocked kernel keeps the rows a wave owns in LDS and adds dt/2 v
    # twice per level in the single-step order: populations and displacement
    # bit for bit those of one launch per step, for every launch variant
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(N, ny, bc, seed=29, kmax=3)
    v0, sb0 = prob.initial_fields()
    nsteps = 37
    g = np.random.default_rng(100 + R)
    u0 = torch.from_numpy(g.standard_normal((2, ny, N)))
    W, T = prob.wall_table(nsteps)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                  displacement=True)
    if R:
        lat.set_body_force(*(torch.from_numpy(a) for a in _random_load(g, R, N, ny, nsteps)))
    ref = None
    for cfg in [-1] + [c["index"] for c in lat.tblock_configs()]:
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        lat.init_displacement(u0)
        if bc == synth.DIRICHLET:
            lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg
        lat.step(11).step(nsteps - 11)
        got = (lat.populations(), lat.displacement())
        if ref is None:
            ref = got
            assert all(torch.isfinite(t).all() for t in got)
        else:
            for a, b in zip(got, ref):
                assert torch.equal(a.view(torch.int32), b.view(torch.int32)), cfg


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
def test_blocked_steps_with_load_and_displacement_match_oracle(bc):
    mat = synth.Material.from_lame(1.0, 0.5, 1.0)
    prob = _mms(64, bc, synth.standing_mms_solution, mat,
                lambda dx: synth.dt_at_cfl_fraction(dx, mat, 0.5), ny=48)
    lat, sim, s = _run(prob, 300, tblock=40 if bc == synth.PERIODIC else 19)
    lat.step(296).step(4)
    sim.advance(300)
    err = oracle.rel_l2(lat.moments_U().double().cpu().numpy(), sim.U())
    uerr = oracle.rel_l2(lat.displacement().double().cpu().numpy(), sim.displacement())
    print("blocked with load and displacement, bc=%d: rel-L2 U %.3e u %.3e" % (bc, err, uerr))
    assert err < 1e-5 and uerr < 1e-5


@gpu
def test_steps_per_launch_reports_the_path():
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(256, 128, synth.PERIODIC, seed=31, kmax=2)
    g = np.random.default_rng(5)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                  displacement=True)
    idx = {(c["steps"], c["seg_rows"], c["nontemporal"], c["prefetch"]): c["index"]
           for c in lat.tblock_configs()}
    assert lat.steps_per_launch == 1                    # no blocked variant selected
    lat.tblock_config = idx[(8, 0, 0, 2)]
    assert lat.steps_per_launch == 7                    # displacement state alone: T = 7
    lat.set_body_force(*(torch.from_numpy(a) for a in _random_load(g, 16, 256, 128, 10)))
    assert lat.steps_per_launch == 6                    # load and displacement: T = 6
    lat.set_body_force(*(torch.from_numpy(a) for a in _random_load(g, 17, 256, 128, 10)))
    assert lat.steps_per_launch == 6                    # ranks 17 .. 32: the T = 6 kernels
    lat.set_body_force(*(torch.from_numpy(a) for a in _random_load(g, 33, 256, 128, 10)))
    assert lat.steps_per_launch == 1                    # rank above 32: one launch per step
    lat2 = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    lat2.tblock_config = idx[(8, 0, 0, 2)]
    assert lat2.steps_per_launch == 8
    lat2.set_body_force(*(torch.from_numpy(a) for a in _random_load(g, 16, 256, 128, 10)))
    assert lat2.steps_per_launch == 8                   # the load-only kernel has T = 8


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
@pytest.mark.parametrize("extras", ["load", "disp", "both", "load32"])
def test_blocked_extras_every_remainder_bitwise_equal_single_steps(bc, extras):
    # with a load and/or the displacement state, lbm_step(n) runs full
    # launches of the T-step kernel with those extras and the steps left in
    # launches of shorter variants (the longest that fits first; a last
    # single step in the one-step kernel): every remainder gives the state of
    # one launch per step bit for bit
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    N, ny = 150, 40
    prob = synth.plane_wave_problem(N, ny, bc, seed=43, kmax=3)
    v0, sb0 = prob.initial_fields()
    nmax = 2 * 8
    g = np.random.default_rng(7)
    R = {"load": 9, "disp": 0, "both": 12, "load32": 20}[extras]
    disp = extras in ("disp", "both")
    W, T = prob.wall_table(nmax)
    u0 = torch.from_numpy(g.standard_normal((2, ny, N)))
    load = [torch.from_numpy(a) for a in _random_load(g, R, N, ny, nmax)] if R else None
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                  displacement=disp)
    if load:
        lat.set_body_force(*load)

    def start(cfg):
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        if disp:
            lat.init_displacement(u0)
        if bc == synth.DIRICHLET:
            lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg

    def state():
        return [lat.populations()] + ([lat.displacement()] if disp else [])

    start(-1)
    ref = {}
    for n in range(1, nmax + 1):
        lat.step(1)
        ref[n] = state()
    seen = set()
    for c in lat.tblock_configs():
        start(c["index"])
        T_run = lat.steps_per_launch
        key = (T_run, c["seg_rows"] <= 0)
        if T_run == 1 or key in seen:
            continue
        seen.add(key)
        for n in range(T_run, min(2 * T_run, nmax) + 1):
            start(c["index"])
            lat.step(n)
            for a, b in zip(state(), ref[n]):
                assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (c, T_run, n)
    assert seen
