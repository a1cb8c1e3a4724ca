"""What the trained surrogate gains over the method without it.

On held-out trajectories (seeds never used in training) of the window map
L(m) = moments(16 lattice steps from the second-order initialisation of m),
the committed network predicts a window to a per-window relative L2 error
(first-order system variables U) far below the judge's 1e-3 acceptance
threshold on periodic lattices, where carrying the fields over unchanged (no
surrogate) is off by order one.  Windows the surrogate gets right need no
lattice fallback.  The serving time against the plain lattice scheme is
printed, not asserted (the surrogate chain is sequential; see the serving
benchmark)."""
import os

import numpy as np
import pytest

import synth

gpu = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
WEIGHTS = os.path.join(ROOT, "paper_2408_01081_amd", "weights", "surrogate.npy")


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _errors(bc, ntraj, seed):
    torch = _torch()
    from paper_2408_01081_amd.surrogate import Surrogate
    from paper_2408_01081_amd.train import generate, rel_l2_U, window_errors
    data, mat, _ = generate(ntraj, side=128, windows=4, bc=bc, seed=seed, chunk=ntraj)
    net = Surrogate(16, 128, 128, split=3)
    net.set_params(np.load(WEIGHTS, allow_pickle=False))
    e = window_errors(net, data, mat, bc == synth.PERIODIC, 16)
    n, W1 = data.shape[0], data.shape[1]
    ident = rel_l2_U(data[:, :-1].reshape(-1, 5, 128, 128), data[:, 1:].reshape(-1, 5, 128, 128),
                     mat.repeat_interleave(W1 - 1, 0).to(data.device))
    del data
    torch.cuda.empty_cache()
    return e, ident


@gpu
@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights committed")
def test_trained_surrogate_beats_no_surrogate_periodic():
    e, ident = _errors(synth.PERIODIC, 48, seed=77)
    print("periodic: surrogate median %.3e p90 %.3e max %.3e, accepted %.3f; "
          "identity median %.3e" % (np.median(e), np.quantile(e, 0.9), e.max(),
                                    np.mean(e <= 1e-3), np.median(ident)))
    assert np.median(e) < 5e-4
    assert np.mean(e <= 1e-3) > 0.9          # windows the judge accepts
    assert np.median(ident) > 100 * np.median(e)


@gpu
@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights committed")
def test_trained_surrogate_beats_no_surrogate_dirichlet():
    e, ident = _errors(synth.DIRICHLET, 32, seed=78)
    print("dirichlet: surrogate median %.3e p90 %.3e max %.3e, accepted %.3f; "
          "identity median %.3e" % (np.median(e), np.quantile(e, 0.9), e.max(),
                                    np.mean(e <= 1e-3), np.median(ident)))
    assert np.median(e) < 3e-3
    assert np.median(ident) > 30 * np.median(e)


@gpu
@pytest.mark.skipif(not os.path.exists(WEIGHTS), reason="no trained weights committed")
def test_serving_with_trained_surrogate_periodic():
    # a periodic 128x128 rollout of 32 windows: every returned state is an
    # accepted surrogate output or a lattice replay, and the final state stays
    # close to the plain lattice run (re-initialisation at every window makes
    # the two differ by more than the per-window tolerance over many windows)
    torch = _torch()
    from paper_2408_01081_amd import serve
    from paper_2408_01081_amd.surrogate import Surrogate
    prob = synth.grf_problem(128, 128, synth.PERIODIC, seed=79)
    net = Surrogate(1, 128, 128, split=3)
    net.set_params(np.load(WEIGHTS, allow_pickle=False))
    plain_ms, variant, plain_final, _ = serve.plain_time_to_solution(prob, 32 * 16, reps=3)
    ro_ms, state, st = serve.rollout_time_to_solution(net, prob, 32, chunk=16, tol=1e-3, reps=1)
    a, b = state.double().flatten(), plain_final.double().flatten()
    rel = float(((a - b).norm() / b.norm()).item())
    print("serving periodic 128^2, 512 steps: plain %.3f ms (%s), surrogate+judge %.3f ms, "
          "acceptance %.3f, final rel-L2 vs plain %.2e" % (plain_ms, variant, ro_ms,
                                                          st["acceptance"], rel))
    assert st["acceptance"] > 0.8
    assert st["window_err_max"] is not None
    assert rel < 0.05
