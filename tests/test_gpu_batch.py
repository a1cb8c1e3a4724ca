"""Batched lattices: bitwise identical to stepping each instance alone, graph
and eager launches agree, per-instance reductions and the FP32-field
re-initialisation used by the judge."""
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


def _problems():
    probs = [synth.plane_wave_problem(67, 45, synth.PERIODIC, seed=1, kmax=3),
             synth.plane_wave_problem(300, 129, synth.DIRICHLET, seed=2, kmax=4),
             synth.grf_problem(64, 64, synth.PERIODIC, seed=3),
             synth.grf_problem(97, 130, synth.DIRICHLET, seed=4),
             synth.plane_wave_problem(5, 3, synth.DIRICHLET, seed=5, kmax=1),
             synth.grf_problem(512, 77, synth.PERIODIC, seed=6, ell=12.0)]
    return probs


def _params(p):
    return dict(nx=p.nx, ny=p.ny, dx=p.dx, dt=p.dt, lam=p.lam, mu=p.mu, rho=p.rho, bc=p.bc)


@gpu
def test_batch_bitwise_equals_single_instances():
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    from paper_2408_01081_amd.lbm import Lattice
    probs = _problems()
    nsteps = 37
    b = Batch([_params(p) for p in probs])
    fields = [p.initial_fields() for p in probs]
    b.init(b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields]))
    tables = {}
    for i, p in enumerate(probs):
        if p.bc == synth.DIRICHLET and p.sol is not None:
            W, T = p.wall_table(nsteps)
            tables[i] = (torch.from_numpy(W), torch.from_numpy(T))
            b.set_wall_velocity(i, *tables[i])
    b.step(20).step(nsteps - 20)
    got = [u.cpu().numpy() for u in b.unpack(b.moments(system=True), 5)]
    for i, p in enumerate(probs):
        lat = Lattice(p.nx, p.ny, p.dx, p.dt, p.lam, p.mu, p.rho, p.bc)
        lat.init(torch.from_numpy(fields[i][0]), torch.from_numpy(fields[i][1]))
        if i in tables:
            lat.set_wall_velocity(*tables[i])
        lat.step(nsteps)
        want = lat.moments_U().cpu().numpy()
        assert np.array_equal(got[i].view(np.uint32), want.view(np.uint32)), i


@gpu
def test_batch_graph_equals_eager_and_oracle():
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = _problems()
    fields = [p.initial_fields() for p in probs]
    out = []
    for graph in (True, False):
        b = Batch([_params(p) for p in probs])
        b.init(b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields]))
        for k in range(3):
            b.step(11, graph=graph)
        out.append(b.moments().cpu().numpy())
    assert np.array_equal(out[0], out[1])
    # one instance against the oracle (homogeneous walls for the GRF ones)
    p = probs[3]
    s = oracle.Setup(p.nx, p.ny, p.dx, p.dt, p.lam, p.mu, p.rho, p.bc)
    sim = oracle.Simulation(s, *fields[3])
    sim.advance(33)
    v, sb = s.fields_from_U(sim.U())
    got = b.unpack(torch.from_numpy(out[1]), 5)[3].numpy().astype(np.float64)
    assert oracle.rel_l2(got, np.concatenate([v, sb])) < 1e-5


@gpu
def test_batch_energy_and_judge_norm():
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = [p for p in _problems() if p.sol is None]   # homogeneous data: energy conserved
    fields = [p.initial_fields() for p in probs]
    b = Batch([_params(p) for p in probs])
    b.init(b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields]))
    E0 = b.energy()
    b.step(50)
    E1 = b.energy()
    assert np.all(np.abs(E1 - E0) / E0 < 1e-5)
    for i, p in enumerate(probs):
        s = oracle.Setup(p.nx, p.ny, p.dx, p.dt, p.lam, p.mu, p.rho, p.bc)
        sim = oracle.Simulation(s, *fields[i])
        assert abs(oracle.energy(s, sim.f) - E0[i]) / E0[i] < 1e-6
    m = b.moments()
    r0 = b.rel_l2_fields(m)
    assert np.all(r0 < 1e-6)
    # a known relative perturbation of one instance's fields is measured
    mm = b.unpack(m.clone(), 5)
    U = [u.double().cpu().numpy() for u in b.unpack(b.moments(system=True), 5)]
    pert = m.clone()
    pp = b.unpack(pert, 5)
    pp[1][:2] *= 1.001          # velocity part of instance 1 only
    r = b.rel_l2_fields(pert)
    want = 1e-3 * np.sqrt(np.sum(U[1][:2] ** 2) / np.sum(U[1] ** 2))
    assert abs(r[1] - want) < 1e-3 * want + 1e-7
    assert r[0] < 1e-6 and r[2] < 1e-6
    del mm


@gpu
def test_batch_reinit_from_fp32_fields():
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = _problems()
    fields = [p.initial_fields() for p in probs]
    b1 = Batch([_params(p) for p in probs])
    b1.init(b1.pack([f[0] for f in fields]), b1.pack([f[1] for f in fields]))
    packed5 = b1.pack([np.concatenate([f[0], f[1]]) for f in fields], dtype=torch.float32)
    b2 = Batch([_params(p) for p in probs])
    b2.init_fields_f32(packed5)
    # the FP64 path from FP32-rounded inputs differs only by the input rounding
    m1 = b1.moments().double().cpu().numpy()
    m2 = b2.moments().double().cpu().numpy()
    assert oracle.rel_l2(m2, m1) < 1e-6


@gpu
def test_batch_blocked_variants_bitwise_equal_single_steps():
    # every temporally blocked variant, graph and eager, with step counts that
    # leave a remainder of single steps; walls at rest
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = _problems()
    fields = [p.initial_fields() for p in probs]
    b = Batch([_params(p) for p in probs])
    v0, s0 = b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields])
    b.init(v0, s0).step(23, graph=False)
    ref = b.moments(system=True).cpu().numpy()
    for c in b.tblock_configs():
        b.tblock_config = c["index"]
        for graph in (True, False):
            b.init(v0, s0)
            b.step(9, graph=graph).step(14, graph=graph)
            got = b.moments(system=True).cpu().numpy()
            assert b.steps == 23
            assert np.array_equal(got.view(np.uint32), ref.view(np.uint32)), (c, graph)


@gpu
def test_batch_remainder_launches_bitwise_equal_single_steps():
    # a run of n steps ends with one launch of an (n mod T)-step variant:
    # every remainder of the T = 6 and T = 7 variants, graph and eager, with
    # the variant for the last steps picked by shape (no launch times yet) and
    # by the autotuner's launch times
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = _problems()
    fields = [p.initial_fields() for p in probs]
    b = Batch([_params(p) for p in probs])
    v0, s0 = b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields])
    b.init(v0, s0)
    ref = {}
    for n in range(1, 14):
        b.step(1, graph=False)
        ref[n] = b.moments(system=True).cpu().numpy()
    long = [c["index"] for c in b.tblock_configs() if c["steps"] >= 6]
    assert long

    def check_all():
        for idx in long:
            T = b.tblock_configs()[idx]["steps"]
            b.tblock_config = idx
            for n in range(T + 1, 2 * T):
                for graph in (True, False):
                    b.init(v0, s0)
                    b.step(n, graph=graph)
                    got = b.moments(system=True).cpu().numpy()
                    assert b.steps == n
                    assert np.array_equal(got.view(np.uint32), ref[n].view(np.uint32)), \
                        (idx, n, graph)

    check_all()
    b.init(v0, s0)
    b.autotune(reps=1)
    check_all()


@gpu
def test_batch_blocked_variants_with_moving_walls_bitwise_equal_single_lattices():
    # instances with moving walls (different ranks and sizes) beside periodic
    # and resting-wall ones: every blocked variant, graph and eager, gives
    # each single lattice's result with the same wall data bit for bit
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    from paper_2408_01081_amd.lbm import Lattice
    probs = [synth.plane_wave_problem(300, 129, synth.DIRICHLET, seed=2, kmax=4),
             synth.plane_wave_problem(64, 64, synth.PERIODIC, seed=3, kmax=2),
             synth.plane_wave_problem(130, 71, synth.DIRICHLET, seed=5, kmax=3),
             synth.plane_wave_problem(97, 40, synth.DIRICHLET, seed=7, kmax=2)]
    nsteps = 23
    walls = [p.wall_table(nsteps + 9) if i != 3 and p.bc == synth.DIRICHLET else None
             for i, p in enumerate(probs)]
    fields = [p.initial_fields() for p in probs]
    want = []
    for p, f, w in zip(probs, fields, walls):
        lat = Lattice(p.nx, p.ny, p.dx, p.dt, p.lam, p.mu, p.rho, p.bc)
        lat.init(torch.from_numpy(f[0]), torch.from_numpy(f[1]))
        if w is not None:
            lat.set_wall_velocity(torch.from_numpy(w[0]), torch.from_numpy(w[1]))
        lat.step(nsteps)
        want.append(lat.moments_U().cpu().numpy().reshape(-1))
    want = np.concatenate(want)
    b = Batch([_params(p) for p in probs])
    v0, s0 = b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields])
    for i, w in enumerate(walls):
        if w is not None:
            b.set_wall_velocity(i, torch.from_numpy(w[0]).cuda(), torch.from_numpy(w[1]).cuda())
    for idx in [-1] + [c["index"] for c in b.tblock_configs()]:
        b.tblock_config = idx
        for graph in (True, False):
            b.init(v0, s0)
            b.step(9, graph=graph).step(nsteps - 9, graph=graph)
            got = b.moments(system=True).cpu().numpy()
            assert np.array_equal(got.view(np.uint32), want.view(np.uint32)), (idx, graph)
    # the autotuner times blocked variants with the walls too
    b.init(v0, s0)
    idx, ms = b.autotune(reps=2)
    assert -1 <= idx < len(b.tblock_configs()) and ms > 0


@gpu
def test_batch_autotune_keeps_state():
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = _problems()
    fields = [p.initial_fields() for p in probs]
    b = Batch([_params(p) for p in probs])
    b.init(b.pack([f[0] for f in fields]), b.pack([f[1] for f in fields])).step(3)
    before = b.moments(system=True).cpu().numpy()
    idx, ms = b.autotune(reps=3)
    assert -1 <= idx < len(b.tblock_configs()) and ms > 0
    assert b.tblock_config == idx and b.steps == 3
    assert np.array_equal(b.moments(system=True).cpu().numpy(), before)


@gpu
def test_batch_rel_l2_pair_of_field_arrays():
    # per-instance ||U(a) - U(b)|| / ||U(b)|| with each instance's material
    # (no lattice state involved), against the oracle's field conversion
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    probs = _problems()
    b = Batch([_params(p) for p in probs])
    g = np.random.default_rng(12)
    fa = [g.standard_normal((5, p.ny, p.nx)) for p in probs]
    fb = [f + 0.01 * (i + 1) * g.standard_normal(f.shape) for i, f in enumerate(fa)]
    got = b.rel_l2_pair(b.pack(fa, torch.float32), b.pack(fb, torch.float32))
    for i, p in enumerate(probs):
        s = oracle.Setup(p.nx, p.ny, p.dx, p.dt, p.lam, p.mu, p.rho, p.bc)
        a32, b32 = (np.asarray(x, dtype=np.float32).astype(np.float64) for x in (fa[i], fb[i]))
        Ua, Ub = s.U_from_fields(a32[:2], a32[2:]), s.U_from_fields(b32[:2], b32[2:])
        want = np.sqrt(np.sum((Ua - Ub) ** 2) / np.sum(Ub ** 2))
        assert abs(got[i] - want) <= 1e-12 * want, (i, got[i], want)
