"""Launch configurations of the step kernel: every valid configuration gives a
bitwise-identical lattice state (same per-node FP32 arithmetic), and the
autotuner leaves the state unchanged."""
import numpy as np
import pytest

import synth

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
@pytest.mark.parametrize("nx,ny", [(512, 24), (320, 19), (66, 30), (1024, 8), (63, 5)])
def test_all_configs_bitwise_identical(bc, nx, ny):
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(nx, ny, bc, seed=11, kmax=3)
    v0, sb0 = prob.initial_fields()
    W, T = prob.wall_table(40)
    ref = None
    for plane_layout in (False, True):
        lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                      plane_layout=plane_layout)
        configs = lat.valid_step_configs()
        assert configs, "no valid configuration"
        for i in configs:
            lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
            if bc == synth.DIRICHLET:
                lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
            lat.step_config = i
            lat.step(40)
            f = lat.populations().cpu().numpy()
            if ref is None:
                ref = f
            else:
                assert np.array_equal(f.view(np.uint32), ref.view(np.uint32)), (plane_layout, i)


@gpu
def test_autotune_keeps_state_and_picks_valid_config():
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(512, 64, synth.PERIODIC, seed=1)
    v0, sb0 = prob.initial_fields()
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    lat.init(torch.from_numpy(v0), torch.from_numpy(sb0)).step(3)
    before = lat.populations().cpu().numpy()
    idx, ms = lat.autotune(reps=3, use_cache=False)
    assert idx in lat.valid_step_configs() and ms > 0
    assert lat.step_config == idx
    after = lat.populations().cpu().numpy()
    assert np.array_equal(before, after)
    # a second call hits the in-process cache
    idx2, ms2 = lat.autotune(reps=3, use_cache=True)
    assert idx2 == idx and ms2 < 0


_TUNE_SCRIPT = r"""
import json, sys
import torch
sys.path.insert(0, sys.argv[1])
import synth
from paper_2408_01081_amd.lbm import Lattice
prob = synth.plane_wave_problem(2048, 512, synth.PERIODIC, seed=3, kmax=4)
v0, sb0 = (torch.from_numpy(a).cuda() for a in prob.initial_fields())
lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
lat.init(v0, sb0)
idx, ms = lat.autotune(reps=2, use_cache=True)
print(json.dumps({"ms": ms, "step": lat.step_config, "tb": lat.tblock_config,
                  "T": lat.steps_per_launch,
                  "rem": [lat.tblock_remainder(r) for r in range(2, 9)]}))
"""


@gpu
def test_autotune_cache_file_keeps_every_choice(tmp_path):
    # the choices, including the variants for the last steps of a run, go
    # to the file named by LBM_AUTOTUNE_CACHE: a fresh process that reads it
    # (the file is read once per process) launches the same kernels
    _torch()
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, LBM_AUTOTUNE_CACHE=str(tmp_path / "tune.txt"))
    outs = []
    for _ in range(2):
        r = subprocess.run([sys.executable, "-c", _TUNE_SCRIPT, root], env=env,
                           capture_output=True, text=True, timeout=180)
        assert r.returncode == 0, r.stderr[-2000:]
        outs.append(json.loads(r.stdout.strip().splitlines()[-1]))
    first, second = outs
    assert first["ms"] > 0 and second["ms"] == -1      # timed, then read from the file
    assert (second["step"], second["tb"]) == (first["step"], first["tb"])
    assert first["tb"] >= 0                             # blocking wins on this grid
    assert second["rem"] == first["rem"]
    for r in range(2, first["T"]):
        assert first["rem"][r - 2] >= 0, (r, first["rem"])


@gpu
def test_select_for_steps():
    # the configuration cheapest for runs of n steps, from the autotuner's
    # launch times: on 4096^2 a 20-step run takes two 10-step launches
    # (T = 8, the fastest per step, needs a third launch for the last 4
    # steps); without launch times the selection stays; the state is
    # bitwise that of single steps whatever is selected
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(4096, 4096, synth.PERIODIC, seed=5, kmax=4)
    v0, sb0 = (torch.from_numpy(a).cuda() for a in prob.initial_fields())
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    lat.init(v0, sb0)
    lat.tblock_config = 3
    assert lat.select_for_steps(20) == 3 == lat.tblock_config   # no launch times yet
    lat.autotune(reps=3, use_cache=False)
    steps = {c["index"]: c["steps"] for c in lat.tblock_configs()}
    per_step = lat.tblock_config
    assert per_step >= 0
    idx = lat.select_for_steps(20)
    assert idx == lat.tblock_config and 20 % steps[idx] == 0, (idx, per_step)
    if 20 % steps[per_step]:
        assert idx != per_step
    lat.init(v0, sb0)
    lat.step(20)
    got = lat.populations()
    lat.init(v0, sb0)
    lat.tblock_config = -1
    lat.step(20)
    assert torch.equal(got.view(torch.int32), lat.populations().view(torch.int32))
    for n in (1, 7, 840):
        i = lat.select_for_steps(n)
        assert i == lat.tblock_config and -1 <= i < len(steps)


@gpu
def test_copy_kernel():
    torch = _torch()
    from paper_2408_01081_amd.lbm import copy_f32
    a = torch.randn(1 << 20, device="cuda")
    b = torch.empty_like(a)
    copy_f32(b, a)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
@pytest.mark.parametrize("nx,ny,plane", [(512, 96, False), (300, 70, False), (64, 64, False),
                                         (61, 7, False), (1, 5, False), (130, 1, False),
                                         (2, 2, False), (1024, 33, False), (300, 70, True),
                                         (61, 7, True)])
def test_blocked_kernels_bitwise_equal_single_steps(bc, nx, ny, plane):
    # temporal blocking changes where values live, not the arithmetic (both
    # population layouts)
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(nx, ny, bc, seed=13, kmax=2)
    v0, sb0 = prob.initial_fields()
    nsteps = 23                       # odd: the last step is a single step
    W, T = prob.wall_table(nsteps)
    ref = None
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                  plane_layout=plane)
    for cfg2 in [-1] + [c["index"] for c in lat.tblock_configs()]:
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        if bc == synth.DIRICHLET:
            lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg2
        lat.step(5).step(nsteps - 5)
        f = lat.populations().cpu().numpy()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f.view(np.uint32), ref.view(np.uint32)), cfg2


# (T, nontemporal, prefetch) of the variants that have a split kernel
_SPLIT_KERNELS = {(7, 0, 1), (7, 0, 2), (6, 0, 1), (6, 0, 2), (5, 0, 1)}


def _split_expected(nx, ny, c):
    # a split kernel for the variant; the interior strips
    # [1, (nx - T) // (64 - 2T)) one or more; 16 wall rows at the top and
    # bottom leaving interior rows
    T = c["steps"]
    return ((T, c["nontemporal"], c["prefetch"]) in _SPLIT_KERNELS
            and (nx - T) // (64 - 2 * T) > 1 and ny >= 33)


@gpu
@pytest.mark.parametrize("nx,ny,plane", [(512, 96, False), (200, 130, False), (130, 33, False),
                                         (1030, 33, False), (300, 70, True), (120, 35, False),
                                         (2048, 1024, False)])
def test_split_dirichlet_launches_bitwise_equal(nx, ny, plane):
    # a split launch (interior with the periodic kernel's code, wall band
    # with the Dirichlet rule, in one grid) gives the unsplit launch's result
    # bit for bit, with moving walls, for every variant
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(nx, ny, synth.DIRICHLET, seed=29, kmax=2)
    v0, sb0 = prob.initial_fields()
    nsteps = 19
    W, T = prob.wall_table(nsteps)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc,
                  plane_layout=plane)

    def run(cfg2, mode):
        lat.set_tblock_split(mode)
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg2
        lat.step(3).step(nsteps - 3)
        return lat.populations().cpu().numpy().view(np.uint32)

    ref = run(-1, 0)
    split_seen = 0
    for c in lat.tblock_configs():
        i = c["index"]
        lat.set_tblock_split(1)
        active = lat.tblock_split_active(i)
        assert active == _split_expected(nx, ny, c), (i, c["steps"])
        split_seen += active
        lat.set_tblock_split(0)
        assert not lat.tblock_split_active(i)
        lat.set_tblock_split(-1)
        assert lat.tblock_split_active(i) == active
        for mode in (1, 0, -1):
            f = run(i, mode)
            assert np.array_equal(f, ref), (i, mode)
    print("%dx%d: %d variants split" % (nx, ny, split_seen))
    lat.set_tblock_split(-1)
    with pytest.raises(RuntimeError):
        lat.set_tblock_split(2)


@gpu
@pytest.mark.parametrize("bc,nx,ny", [(synth.PERIODIC, 4096, 4096), (synth.PERIODIC, 4096, 2000),
                                      (synth.DIRICHLET, 4096, 2000)])
def test_whole_device_blocked_variants_bitwise_equal_single_steps(bc, nx, ny):
    # variants sized to the resident wave slots, on the full-size grid and on
    # one whose last segment is short
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(nx, ny, bc, seed=19, kmax=3)
    v0, sb0 = prob.initial_fields()
    nsteps = 17
    W, T = prob.wall_table(nsteps)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    ref = None
    cfgs = [c["index"] for c in lat.tblock_configs() if c["seg_rows"] <= 0]
    assert cfgs
    for cfg2 in [-1] + cfgs:
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        if bc == synth.DIRICHLET:
            lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg2
        lat.step(nsteps)
        f = lat.populations()
        if ref is None:
            ref = f
        else:
            assert torch.equal(f.view(torch.int32), ref.view(torch.int32)), cfg2
    del ref, f, lat
    torch.cuda.empty_cache()


@gpu
def test_blocked_kernels_across_wall_table_chunks():
    # lbm_step sums wall velocities in chunks of up to 420 steps: runs longer than a
    # chunk, split at odd places, stay bitwise equal to single steps
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(70, 45, synth.DIRICHLET, seed=17, kmax=3)
    v0, sb0 = prob.initial_fields()
    nsteps = 431 + 419
    W, T = prob.wall_table(nsteps)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    ref = None
    seen = set()
    for c in [{"index": -1, "steps": 1}] + lat.tblock_configs():
        if c["steps"] in seen:
            continue
        seen.add(c["steps"])
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = c["index"]
        lat.step(431).step(419)
        assert lat.steps == nsteps
        f = lat.populations().cpu().numpy()
        if ref is None:
            ref = f
        else:
            assert np.array_equal(f.view(np.uint32), ref.view(np.uint32)), c


@gpu
def test_blocked_kernels_match_oracle_dirichlet_walls():
    torch = _torch()
    import oracle
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(200, 130, synth.DIRICHLET, seed=14, kmax=4)
    v0, sb0 = prob.initial_fields()
    n = 300
    W, T = prob.wall_table(n)
    s = oracle.Setup(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    sim = oracle.Simulation(s, v0, sb0, wall=prob.wall_velocity)
    sim.advance(n)
    ref = sim.U()
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    for c in lat.tblock_configs():
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = c["index"]
        lat.step(n)
        U = lat.moments_U().double().cpu().numpy()
        assert oracle.rel_l2(U, ref) < 1e-5, c


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
def test_every_remainder_bitwise_equal_single_steps(bc):
    # lbm_step(n) with a T-step variant runs floor(n / T) full launches and
    # the r = n mod T steps left in one launch of an r-step variant (r >= 2)
    # or of the single-step kernel: for every T and every r, both launch
    # shapes per T (fixed segments and one wave per resident slot), the state
    # is the single-step state bit for bit (Dirichlet with moving walls)
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    prob = synth.plane_wave_problem(203, 71, bc, seed=37, kmax=3)
    v0, sb0 = prob.initial_fields()
    nmax = 3 * 8
    W, T = prob.wall_table(nmax)
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)

    def start(cfg):
        lat.init(torch.from_numpy(v0), torch.from_numpy(sb0))
        if bc == synth.DIRICHLET:
            lat.set_wall_velocity(torch.from_numpy(W), torch.from_numpy(T))
        lat.tblock_config = cfg

    start(-1)
    ref = {0: lat.populations()}
    for n in range(1, nmax + 1):
        lat.step(1)
        ref[n] = lat.populations()
    picks = {}
    for c in lat.tblock_configs():
        picks.setdefault((c["steps"], c["seg_rows"] <= 0), c["index"])
    for (steps, _), cfg in sorted(picks.items()):
        for n in range(steps, 2 * steps + 1) if steps < 8 else range(8, nmax + 1):
            start(cfg)
            lat.step(n)
            got = lat.populations()
            assert torch.equal(got.view(torch.int32), ref[n].view(torch.int32)), (cfg, steps, n)


@gpu
def test_blocked_kernel_on_lattice_beyond_32_bit_row_offsets():
    # 8192^2 row-major: row byte offsets reach 5.4 GB, past 2^32; the blocked
    # kernel forms row addresses in 64 bits and gives the single-step state
    # bit for bit (8 + 8 steps and a 3-step launch for the rest)
    torch = _torch()
    from paper_2408_01081_amd.lbm import Lattice
    N = 8192
    prob = synth.plane_wave_problem(N, N, synth.PERIODIC, seed=41, kmax=4)
    v0, sb0 = (torch.from_numpy(a).cuda() for a in prob.initial_fields())
    lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    idx = {(c["steps"], c["seg_rows"], c["nontemporal"], c["prefetch"]): c["index"]
           for c in lat.tblock_configs()}
    out = []
    for cfg in (-1, idx[(8, 0, 0, 2)]):
        lat.init(v0, sb0)
        lat.tblock_config = cfg
        lat.step(19)
        out.append(lat.moments_U())
    del lat
    assert torch.isfinite(out[0]).all()
    assert torch.equal(out[0].view(torch.int32), out[1].view(torch.int32))
