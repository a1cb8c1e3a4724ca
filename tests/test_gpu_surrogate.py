"""Surrogate kernels (forward, loss gradient, Adam) against the FP64 CPU
reference in oracle/surrogate_ref.py on the same seeded inputs and
parameters.

Tolerances: with hi/lo BF16 operands (split 3) the products carry ~16
significant bits and accumulate in FP32, so outputs agree to ~1e-5 relative
and gradients to ~1e-4; with plain BF16 operands (split 1) each operand is
rounded to 8 bits (relative 2^-9 = 2e-3 per rounding)."""
import numpy as np
import pytest

from oracle import surrogate_ref as R

gpu = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _inputs(seed, B, H, W):
    g = np.random.default_rng(seed)
    import synth
    inp = np.zeros((B, 8, H, W))
    for b in range(B):
        f = synth.gaussian_random_field(g, H, W, float(g.uniform(6, 16)), 5)
        inp[b, :5] = f
        nu = g.uniform(0, 0.49)
        inp[b, 5] = 2 * nu / (1 - 2 * nu)
        inp[b, 6] = 1.0
        inp[b, 7] = g.uniform(0.5, 2.0)
    tgt = inp[:, :5] + 0.05 * g.standard_normal((B, 5, H, W))
    return inp, tgt


def _params(seed):
    from paper_2408_01081_amd import surrogate as S
    P = S.init_params(seed=seed, out_scale=0.3)
    g = np.random.default_rng(seed + 1)
    for k in P:
        if k.endswith(".a"):
            P[k] = P[k] + 0.1 * g.standard_normal(P[k].shape)
    return P


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


@gpu
@pytest.mark.parametrize("split,circular", [(3, True), (3, False), (1, True)])
def test_forward_matches_reference(split, circular):
    torch = _torch()
    from paper_2408_01081_amd import surrogate as S
    B, H, W = 3, 64, 128
    inp, _ = _inputs(1, B, H, W)
    P = _params(2)
    net = S.Surrogate(B, H, W, split=split)
    net.set_params(S.pack_params(P))
    x = torch.from_numpy(inp.astype(np.float32)).cuda()
    out = net.forward(x, circular=circular).double().cpu().numpy()
    # reference on the FP32-rounded input and parameters
    P32 = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    ref = R.Forward(P32, inp.astype(np.float32).astype(np.float64), circular)
    d_out = out - inp[:, :5]
    d_ref = ref.out - inp[:, :5]
    err = _rel(d_out, d_ref)   # relative to the network's correction
    print("split %d circular %d: forward rel err of the correction %.2e" % (split, circular, err))
    assert err < (1e-4 if split == 3 else 3e-2)
    if split == 3:
        assert _rel(out, ref.out) < 1e-5


@gpu
@pytest.mark.parametrize("circular", [True, False])
def test_gradients_match_reference(circular):
    torch = _torch()
    from paper_2408_01081_amd import surrogate as S
    B, H, W = 2, 64, 128
    inp, tgt = _inputs(3, B, H, W)
    P = _params(4)
    net = S.Surrogate(B, H, W, split=3, train=True)
    net.set_params(S.pack_params(P))
    x = torch.from_numpy(inp.astype(np.float32)).cuda()
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    loss = net.train_step(x, t, circular=circular, lr=0.0)
    G = S.unpack_params(net.get_grads().double().cpu().numpy())
    P32 = {k: v.astype(np.float32).astype(np.float64) for k, v in P.items()}
    ref = R.Forward(P32, inp.astype(np.float32).astype(np.float64), circular)
    lref = ref.loss(tgt.astype(np.float32).astype(np.float64))
    assert abs(loss - lref) / lref < 1e-5
    Gr = ref.backward()
    worst = 0.0
    for k in Gr:
        e = _rel(G[k], Gr[k])
        worst = max(worst, e)
        assert e < 1e-3, (k, e)
    print("worst gradient block rel err %.2e" % worst)


@gpu
def test_adam_step_matches_reference_and_loss_decreases():
    torch = _torch()
    from paper_2408_01081_amd import surrogate as S
    B, H, W = 2, 64, 128
    inp, tgt = _inputs(5, B, H, W)
    P = _params(6)
    net = S.Surrogate(B, H, W, split=3, train=True)
    v0 = S.pack_params(P).astype(np.float32)
    net.set_params(v0)
    x = torch.from_numpy(inp.astype(np.float32)).cuda()
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    lr = 1e-3
    # the FP64 reference Adam (bias-corrected moments) fed the kernel's own
    # gradient of each step, over several steps
    Pr = {"v": v0.astype(np.float64)}
    M, V = {"v": np.zeros_like(Pr["v"])}, {"v": np.zeros_like(Pr["v"])}
    for step in range(1, 5):
        net.train_step(x, t, circular=True, lr=lr)
        g = net.get_grads().double().cpu().numpy()
        R.adam_update(Pr, {"v": g}, M, V, step, lr)
        v = net.get_params().double().cpu().numpy()
        assert np.max(np.abs(v - Pr["v"])) < 1e-6 + 1e-5 * lr, step
    losses = [net.train_step(x, t, circular=True, lr=lr) for _ in range(30)]
    assert losses[-1] < 0.5 * losses[0], losses


@gpu
@pytest.mark.parametrize("split,circular,B,H,W", [(3, True, 1, 256, 256), (3, False, 2, 128, 256),
                                                  (3, True, 32, 64, 128), (1, False, 4, 64, 128)])
def test_tiled_and_direct_convolutions_agree(split, circular, B, H, W):
    # the LDS-tiled convolution (blocks of 4 x 64, 1 x 64, 2 x 32 and 4 x 16
    # pixels across these shapes) and the direct one compute the same products; only the FP32 summation order of
    # the reduction slices may differ (with plain BF16 operands such a
    # difference can flip the rounding of the next layer's operand, so the
    # bound is that of the split-1 reference comparison)
    torch = _torch()
    from paper_2408_01081_amd import surrogate as S
    inp, _ = _inputs(5, B, H, W)
    P = _params(6)
    x = torch.from_numpy(inp.astype(np.float32)).cuda()
    outs = []
    for mode in (0, 1):
        net = S.Surrogate(B, H, W, split=split)
        net.set_params(S.pack_params(P))
        net.set_conv_mode(mode)
        outs.append(net.forward(x, circular=circular).double().cpu().numpy())
        del net
    err = _rel(outs[0] - inp[:, :5], outs[1] - inp[:, :5])
    print("tiled vs direct, split %d: rel diff of the correction %.2e" % (split, err))
    assert err < (1e-5 if split == 3 else 3e-2)


@gpu
@pytest.mark.parametrize("circular", [True, False])
def test_tiled_and_direct_weight_gradients_agree(circular):
    # the LDS-staged weight gradient (blocks of 64 pixels: one row segment at
    # the 128- and 64-wide levels, 2 and 4 whole rows at the 32- and 16-wide
    # ones) and the direct kernel sum the same products in another order
    torch = _torch()
    from paper_2408_01081_amd import surrogate as S
    B, H, W = 8, 128, 128
    inp, tgt = _inputs(7, B, H, W)
    P = _params(8)
    x = torch.from_numpy(inp.astype(np.float32)).cuda()
    t = torch.from_numpy(tgt.astype(np.float32)).cuda()
    grads = []
    for mode in (0, 1):
        net = S.Surrogate(B, H, W, split=3, train=True)
        net.set_params(S.pack_params(P))
        net.set_conv_mode(mode)
        net.train_step(x, t, circular=circular, lr=0.0)
        grads.append(S.unpack_params(net.get_grads().double().cpu().numpy()))
        del net
    worst = max(_rel(grads[0][k], grads[1][k]) for k in grads[0])
    print("tiled vs direct weight gradients: worst block rel diff %.2e" % worst)
    assert worst < 1e-4
