"""Surrogate + judge rollout logic: with every window rejected the result is
the lattice window chain; with every window accepted it is the surrogate
chain; a mixed run only ever returns accepted surrogate outputs or lattice
replays.  Also the training-data generator's windows restart exactly like
the judge's replays."""
import numpy as np
import pytest

import synth

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _problem(bc=synth.DIRICHLET):
    return synth.grf_problem(128, 64, bc, seed=21, ell=10.0)


def _lbm_chain(prob, f0, nwin):
    torch = _torch()
    from paper_2408_01081_amd.batch import Batch
    b = Batch([dict(nx=prob.nx, ny=prob.ny, dx=prob.dx, dt=prob.dt, lam=prob.lam, mu=prob.mu,
                    rho=prob.rho, bc=prob.bc)])
    m = f0.reshape(-1).clone()
    for _ in range(nwin):
        b.init_fields_f32(m)
        b.step(16)
        m = b.moments()
    return m.view(5, prob.ny, prob.nx)


@gpu
@pytest.mark.parametrize("bc", [synth.PERIODIC, synth.DIRICHLET])
def test_rollout_all_rejected_is_lattice_chain(bc):
    torch = _torch()
    from paper_2408_01081_amd.serve import Rollout
    from paper_2408_01081_amd.surrogate import Surrogate, init_params, pack_params
    prob = _problem(bc)
    net = Surrogate(1, prob.ny, prob.nx, split=3)
    net.set_params(pack_params(init_params(1, 0.05)).astype(np.float32))
    f0 = torch.cat([torch.from_numpy(prob.v0), torch.from_numpy(prob.sb0)]).float().cuda()
    ro = Rollout(net, prob, chunk=4, tol=-1.0)
    out, st = ro.run(f0, 7)
    assert st["accepted"] == 0 and st["fallbacks"] == 7
    ref = _lbm_chain(prob, f0, 7)
    assert torch.equal(out, ref)


@gpu
def test_rollout_all_accepted_is_surrogate_chain():
    torch = _torch()
    from paper_2408_01081_amd.serve import Rollout
    from paper_2408_01081_amd.surrogate import Surrogate, init_params, pack_params
    prob = _problem()
    net = Surrogate(1, prob.ny, prob.nx, split=3)
    net.set_params(pack_params(init_params(2, 0.05)).astype(np.float32))
    f0 = torch.cat([torch.from_numpy(prob.v0), torch.from_numpy(prob.sb0)]).float().cuda()
    ro = Rollout(net, prob, chunk=3, tol=1e30)
    out, st = ro.run(f0, 7)
    assert st["accepted"] == 7 and st["fallbacks"] == 0
    x = torch.zeros((1, 8, prob.ny, prob.nx), device="cuda")
    x[0, :5] = f0
    x[0, 5], x[0, 6], x[0, 7] = prob.lam, prob.mu, prob.rho
    for _ in range(7):
        y = net.forward(x, circular=False)
        x[0, :5] = y[0]
    assert torch.equal(out, x[0, :5])


@gpu
def test_rollout_mixed_returns_valid_states():
    torch = _torch()
    from paper_2408_01081_amd.serve import Rollout
    from paper_2408_01081_amd.surrogate import Surrogate, init_params, pack_params
    prob = _problem()
    net = Surrogate(1, prob.ny, prob.nx, split=3)
    # the identity map: windows where the fields barely move are accepted
    net.set_params(pack_params(init_params(3, 0.0)).astype(np.float32))
    f0 = torch.cat([torch.from_numpy(prob.v0), torch.from_numpy(prob.sb0)]).float().cuda()
    acc = []
    for tol in (0.0, 0.05, 0.2, 0.6, 1e30):
        ro = Rollout(net, prob, chunk=4, tol=tol)
        out, st = ro.run(f0, 6)
        # every window is either accepted or replaced by its replay
        assert st["accepted"] + st["fallbacks"] == 6, st
        # the judged errors include each rejected window's: the largest is
        # above the tolerance exactly when some window fell back
        assert (st["fallbacks"] == 0) == (st["window_err_max"] <= tol), (tol, st)
        assert torch.isfinite(out).all()
        acc.append(st["accepted"])
    # nothing passes a zero tolerance, everything an infinite one
    assert acc[0] == 0 and acc[-1] == 6, acc


@gpu
def test_training_windows_restart_like_the_judge():
    torch = _torch()
    from paper_2408_01081_amd.train import generate
    data, mat, bc = generate(3, side=128, windows=3, bc=synth.PERIODIC, seed=9, chunk=2)
    # window 2 -> 3 of trajectory 1 equals a judge replay from snapshot 2
    import synth as S
    p = S.grf_problem(128, 128, synth.PERIODIC, seed=9 * 1000003 + 1)
    ref = _lbm_chain(p, data[1, 2].reshape(-1), 1)
    assert torch.equal(ref, data[1, 3])
