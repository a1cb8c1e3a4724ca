"""Training data from the batched lattice Boltzmann path, and training of the
window surrogate on the GPU with its own forward/backward kernels.

Window map (what the surrogate learns and what the judge replays):
    L(m) = moments(16 lattice steps from the second-order initialisation of m)
where m are the macroscopic fields (v, Cauchy stress).  A trajectory is
m_0, m_1 = L(m_0), m_2 = L(m_1), ...: every window restarts from the
previous window's moments, exactly as the judge does during serving.

Command line (writes the trained parameters as a float32 .npy file):
    python -m paper_2408_01081_amd.train --out weights.npy --minutes 6
"""
from __future__ import annotations

import argparse
import math
import os
import sys
import time

import numpy as np
import torch

from .batch import Batch
from .surrogate import Surrogate, init_params, pack_params

K_WINDOW = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _instances(probs):
    return [dict(nx=p.nx, ny=p.ny, dx=p.dx, dt=p.dt, lam=p.lam, mu=p.mu, rho=p.rho, bc=p.bc)
            for p in probs]


def generate(n_traj, side=128, windows=16, bc=0, seed=4, chunk=512, device="cuda:0"):
    """Trajectories of the judge-consistent window map on seeded GRF data.

    Returns (fields [n][windows+1][5][side][side] float32 on the device,
    material [n][3] = (lambda, mu, rho) float32, bc)."""
    import synth
    dev = torch.device(device)
    data = torch.empty((n_traj, windows + 1, 5, side, side), dtype=torch.float32, device=dev)
    mat = torch.empty((n_traj, 3), dtype=torch.float32)
    done = 0
    while done < n_traj:
        n = min(chunk, n_traj - done)
        probs = [synth.grf_problem(side, side, bc, seed=seed * 1000003 + done + i)
                 for i in range(n)]
        b = Batch(_instances(probs), device=dev)
        v0 = b.pack([p.v0 for p in probs])
        s0 = b.pack([p.sb0 for p in probs])
        b.init(v0, s0)
        snap = torch.cat([v0.view(n, 2, side, side), s0.view(n, 3, side, side)], dim=1)
        data[done:done + n, 0] = snap.float()
        m = b.moments()
        for w in range(windows):
            b.step(K_WINDOW)
            b.moments(out=m)
            data[done:done + n, w + 1] = m.view(n, 5, side, side)
            if w + 1 < windows:
                b.init_fields_f32(m)          # judge-consistent restart
        for i, p in enumerate(probs):
            mat[done + i] = torch.tensor([p.lam, p.mu, p.rho])
        done += n
        del b
    torch.cuda.synchronize(dev)
    return data, mat, bc


def pairs_of(data):
    """Training pairs of a trajectory set: inputs data[:, w], targets
    data[:, w + 1] (views, no copy)."""
    return data[:, :-1], data[:, 1:]


def assemble(inp, tgt, mat, idx, widx, out_in, out_tgt):
    """Input [B][8][H][W] (fields inp[idx, widx], material channels) and
    target [B][5][H][W] (tgt[idx, widx]) for pair sets of [n][W][5][H][W]."""
    B = len(idx)
    it = torch.as_tensor(idx, device=inp.device)
    wt = torch.as_tensor(widx, device=inp.device)
    out_in[:B, :5] = inp[it, wt]
    out_tgt[:B] = tgt[it, wt]
    m = mat.to(inp.device)[it]
    out_in[:B, 5:] = m[:, :, None, None]


def pushforward(net, inp, mat, bc, batch, chain=False, chunk=512):
    """Pairs on the states a rollout of the surrogate visits: y and its image
    under the judge's window map L(y) = moments(16 steps from the FP64
    re-initialisation of y), with the trajectory's material, dx = 1 and the
    time step at half the CFL-like limit (as generate() draws them).  y =
    net(x) for every input x of the pair set, or (chain) the network's own
    chain from each trajectory's first input, y_w = net^(w+1)(x_0), the
    states of a rollout in which every window is accepted.  Returns
    (y, L(y)), each [n][W][5][H][H] float32 on the device."""
    import synth
    n, W, H = inp.shape[0], inp.shape[1], inp.shape[3]
    dev = inp.device
    pin = torch.empty((n, W, 5, H, H), dtype=torch.float32, device=dev)
    ptg = torch.empty_like(pin)
    xin = torch.empty((batch, 8, H, H), dtype=torch.float32, device=dev)
    tgt = torch.empty((batch, 5, H, H), dtype=torch.float32, device=dev)
    if chain:
        for w in range(W):
            src = inp[:, 0] if w == 0 else pin[:, w - 1]
            for k in range(0, n, batch):
                B = min(batch, n - k)
                xin[:B, :5] = src[k:k + B]
                xin[:B, 5:] = mat[k:k + B].to(dev)[:, :, None, None]
                pin[k:k + B, w] = net.forward(xin[:B], circular=(bc == 0))
    else:
        pairs = [(i, w) for i in range(n) for w in range(W)]
        for k in range(0, len(pairs), batch):
            pp = pairs[k:k + batch]
            B = len(pp)
            it, wt = [p[0] for p in pp], [p[1] for p in pp]
            assemble(inp, inp, mat, it, wt, xin, tgt)
            pin[torch.as_tensor(it, device=dev), torch.as_tensor(wt, device=dev)] = \
                net.forward(xin[:B], circular=(bc == 0))
    for c0 in range(0, n, chunk):
        c1 = min(n, c0 + chunk)
        insts = []
        for lam, mu, rho in mat[c0:c1].double().cpu().numpy():
            m = synth.Material.from_lame(float(lam), float(mu), float(rho))
            insts.append(dict(nx=H, ny=H, dx=1.0, dt=synth.dt_at_cfl_fraction(1.0, m, 0.5),
                              lam=float(lam), mu=float(mu), rho=float(rho), bc=int(bc)))
        b = Batch(insts, device=dev)
        mo = torch.empty((c1 - c0, 5, H, H), dtype=torch.float32, device=dev)
        for w in range(W):
            b.init_fields_f32(pin[c0:c1, w].contiguous())
            b.step(K_WINDOW)
            b.moments(out=mo.view(-1))
            ptg[c0:c1, w] = mo
        del b
    torch.cuda.synchronize(dev)
    return pin, ptg


def window_errors(net, data, mat, circular, batch, max_pairs=4096, seed=0):
    """Per-window relative L2 error (system variables U, FP64 on the device)
    of the surrogate against the lattice window map, on up to max_pairs
    (trajectory, window) pairs."""
    return pair_errors(net, *pairs_of(data), mat, circular, batch, max_pairs, seed)


def pair_errors(net, inp, tgt_set, mat, circular, batch, max_pairs=4096, seed=0):
    """Per-pair relative L2 error (system variables U) of the surrogate on up
    to max_pairs pairs of a pair set."""
    n, W = inp.shape[0], inp.shape[1]
    g = np.random.default_rng(seed)
    pairs = [(i, w) for i in range(n) for w in range(W)]
    if len(pairs) > max_pairs:
        sel = g.choice(len(pairs), max_pairs, replace=False)
        pairs = [pairs[k] for k in sel]
    H = inp.shape[3]
    xin = torch.empty((batch, 8, H, H), dtype=torch.float32, device=inp.device)
    tgt = torch.empty((batch, 5, H, H), dtype=torch.float32, device=inp.device)
    errs = []
    for k in range(0, len(pairs), batch):
        pp = pairs[k:k + batch]
        B = len(pp)
        assemble(inp, tgt_set, mat, [p[0] for p in pp], [p[1] for p in pp], xin, tgt)
        out = net.forward(xin[:B], circular=circular)
        errs.append(rel_l2_U(out, tgt[:B], xin[:B, 5:]))
    return np.concatenate(errs)


def rel_l2_U(a, b, material, chunk=64):
    """||U(a) - U(b)|| / ||U(b)|| per sample, U = first-order system variables
    of each sample's material, computed by the library (lbm_batch_rel_l2_pair:
    a batch of field-only instances, no lattice state).  a, b: [B][5][H][W]
    fields (v, sigma_bar); material: per sample [B][3] or per pixel
    [B][3][H][W] (lambda, mu, rho, constant over the window)."""
    mt = material if material.dim() == 2 else material[:, :, 0, 0]
    mt = mt.double().cpu().numpy()
    Bn, _, H, W = a.shape
    out = []
    for k in range(0, Bn, chunk):
        insts = []
        for lam, mu, rho in mt[k:k + chunk]:
            # any admissible time step: only the material enters U
            cmax = math.sqrt((lam + 2.0 * mu) / rho)  # sqrt(c_K^2 + c_mu^2)
            insts.append(dict(nx=W, ny=H, dx=1.0, dt=0.25 / cmax, lam=float(lam), mu=float(mu),
                              rho=float(rho), bc=0))
        batch = Batch(insts, device=a.device)
        out.append(batch.rel_l2_pair(a[k:k + chunk].reshape(-1), b[k:k + chunk].reshape(-1)))
    return np.concatenate(out)


def train(net, sets, minutes, batch, lr0=1e-3, lr_end=2e-5, seed=0, log_every=100,
          max_steps=None, spike=1000.0):
    """Adam with a cosine learning-rate decay over the time budget.  sets is
    a list of (inputs, targets, mat, bc) pair sets ([n][W][5][H][W] each);
    batches alternate between them.

    The network is linear in the fields and has no saturation, so an unlucky
    update can make it diverge: every log_every steps the loss is checked, the
    parameters of the last healthy check are kept on the device, and a loss
    above `spike` times the best smoothed loss (or non-finite) restores them
    and halves the learning rate.  Returns the parameters with the lowest
    smoothed loss."""
    g = np.random.default_rng(seed)
    H = sets[0][0].shape[3]
    dev = sets[0][0].device
    xin = torch.empty((batch, 8, H, H), dtype=torch.float32, device=dev)
    tgt = torch.empty((batch, 5, H, H), dtype=torch.float32, device=dev)
    t0 = time.time()
    budget = minutes * 60.0
    step, hist = 0, []
    good = net.get_params().clone()
    best_params, best = good.clone(), float("inf")
    smooth, scale, restores = None, 1.0, 0
    while True:
        el = time.time() - t0
        if el > budget or (max_steps and step >= max_steps):
            break
        frac = min(1.0, el / budget)
        lr = scale * (lr_end + 0.5 * (lr0 - lr_end) * (1 + math.cos(math.pi * frac)))
        inp, tg, mat, bc = sets[step % len(sets)]
        idx = g.integers(0, inp.shape[0], batch)
        widx = g.integers(0, inp.shape[1], batch)
        assemble(inp, tg, mat, idx, widx, xin, tgt)
        check = (step % log_every) == 0
        loss = net.train_step(xin, tgt, circular=(bc == 0), lr=lr, want_loss=check)
        if check:
            if not math.isfinite(loss) or (smooth is not None and loss > spike * max(best, 1e-12)):
                net.set_params(good)           # back to the last healthy parameters
                scale *= 0.5
                restores += 1
                log("step %6d  loss %.3e: restored, lr scale %.3g" % (step, loss, scale))
            else:
                smooth = loss if smooth is None else 0.8 * smooth + 0.2 * loss
                good = net.get_params().clone()
                if smooth < best:
                    best, best_params = smooth, good.clone()
            hist.append((step, round(time.time() - t0, 1), loss, lr))
            if (step // log_every) % 5 == 0:
                log("step %6d  t %6.1fs  loss %.3e  smooth %.3e  lr %.2e" %
                    (step, time.time() - t0, loss, smooth if smooth else float("nan"), lr))
        step += 1
    torch.cuda.synchronize(dev)
    net.set_params(best_params)
    return step, hist, {"restores": restores, "best_smoothed_loss": best}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--minutes", type=float, default=6.0)
    ap.add_argument("--n-periodic", type=int, default=4096)
    ap.add_argument("--n-dirichlet", type=int, default=1024)
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--windows", type=int, default=16)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--split", type=int, default=3)
    ap.add_argument("--lr", type=float, default=5e-4)
    ap.add_argument("--init", default="")
    ap.add_argument("--report", default="")
    ap.add_argument("--seed-periodic", type=int, default=4)
    ap.add_argument("--seed-dirichlet", type=int, default=5)
    ap.add_argument("--pushforward-rounds", type=int, default=0,
                    help="split the time into this many rounds, each training on the "
                         "trajectory pairs and on pairs (y, L(y)) of the network's own "
                         "outputs y (recomputed at the start of every round)")
    ap.add_argument("--chain", action="store_true",
                    help="with --pushforward-rounds: y along the network's own chain from "
                         "each trajectory's first state (a rollout's states)")
    args = ap.parse_args()
    t0 = time.time()
    sets = []
    if args.n_periodic:
        sets.append(generate(args.n_periodic, args.side, args.windows, bc=0,
                             seed=args.seed_periodic))
    if args.n_dirichlet:
        sets.append(generate(args.n_dirichlet, args.side, args.windows, bc=1,
                             seed=args.seed_dirichlet))
    t_gen = time.time() - t0
    log("data: %s in %.1fs" % ([tuple(s[0].shape) for s in sets], t_gen))
    # hold out the last 1/8 of every set for validation
    train_sets, val_sets = [], []
    for data, mat, bc in sets:
        nv = max(1, data.shape[0] // 8)
        train_sets.append((data[:-nv], mat[:-nv], bc))
        val_sets.append((data[-nv:], mat[-nv:], bc))
    net = Surrogate(args.batch, args.side, args.side, split=args.split, train=True)
    p0 = np.load(args.init, allow_pickle=False) if args.init else pack_params(init_params(0, 0.0))
    net.set_params(p0.astype(np.float32))
    trajs = [(*pairs_of(d), m, bc) for d, m, bc in train_sets]
    rounds = max(1, args.pushforward_rounds)
    steps, hist, info = 0, [], {}
    for r in range(rounds):
        sets_r = list(trajs)
        if args.pushforward_rounds:
            t1 = time.time()
            for inp, tg, m, bc in trajs:
                sets_r.append((*pushforward(net, inp, m, bc, args.batch, chain=args.chain), m,
                               bc))
            log("round %d: pushforward pairs in %.1fs" % (r, time.time() - t1))
        s_r, h_r, info = train(net, sets_r, args.minutes / rounds, args.batch, lr0=args.lr)
        steps += s_r
        hist += [(steps - s_r + h[0],) + tuple(h[1:]) for h in h_r]
        sets_r = None
    params = net.get_params().cpu().numpy()
    np.save(args.out, params, allow_pickle=False)
    rep = {"steps": steps, "minutes": args.minutes, "data_seconds": round(t_gen, 1),
           "pushforward_rounds": args.pushforward_rounds,
           "history": hist[::max(1, len(hist) // 40)], "validation": {}, **info}
    for data, mat, bc in val_sets:
        e = window_errors(net, data, mat, bc == 0, args.batch)
        # the second window of a surrogate chain: the network on its own
        # outputs, against the window map of those outputs (the judge's test
        # in a rollout)
        pin, ptg = pushforward(net, data[:, :-1], mat, bc, args.batch)
        e2 = pair_errors(net, pin, ptg, mat, bc == 0, args.batch)
        # and along the network's own chain (a fully accepted rollout)
        pin, ptg = pushforward(net, data[:, :-1], mat, bc, args.batch, chain=True)
        e3 = pair_errors(net, pin, ptg, mat, bc == 0, args.batch)
        ec = pair_errors(net, pin[:, -1:], ptg[:, -1:], mat, bc == 0, args.batch)
        del pin, ptg
        rep["validation"]["periodic" if bc == 0 else "dirichlet"] = {
            "pairs": int(len(e)), "median": float(np.median(e)), "p90": float(np.quantile(e, 0.9)),
            "max": float(e.max()), "frac_le_1e-3": float(np.mean(e <= 1e-3)),
            "on_own_outputs": {"median": float(np.median(e2)),
                               "p90": float(np.quantile(e2, 0.9)),
                               "frac_le_1e-3": float(np.mean(e2 <= 1e-3))},
            "along_own_chain": {"median": float(np.median(e3)),
                                "p90": float(np.quantile(e3, 0.9)),
                                "frac_le_1e-3": float(np.mean(e3 <= 1e-3)),
                                "last_window_median": float(np.median(ec))}}
        # the identity map (no surrogate) for scale
        ident = rel_l2_U(data[:, :-1].reshape(-1, 5, args.side, args.side)[:512],
                         data[:, 1:].reshape(-1, 5, args.side, args.side)[:512],
                         mat.repeat_interleave(data.shape[1] - 1, 0)[:512].to(data.device))
        # (the identity map = persistence, i.e. no surrogate at all)
        rep["validation"]["periodic" if bc == 0 else "dirichlet"]["identity_median"] = \
            float(np.median(ident))
    log(rep["validation"])
    if args.report:
        import json
        json.dump(rep, open(args.report, "w"), indent=1)


if __name__ == "__main__":
    main()
