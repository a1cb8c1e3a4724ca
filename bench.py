#!/usr/bin/env python3
"""Benchmark of the FP32 lattice Boltzmann step on one MI355X.

Workload (one "step"): one time step of a 4096^2 periodic lattice plus one
time step of a 2048x1024 Dirichlet lattice with time-dependent manufactured
boundary displacement; Poisson ratio from a seed, mu = 1, rho = 1, time step at
half the CFL-like limit; initial data are seeded plane-wave superpositions
(exact solutions, b = 0).  Inputs are resident in HBM before timing starts.

Prints one JSON line: GLUPS (lattice node updates per second, both lattices),
the dominant kernel's achieved HBM bandwidth against the 8 TB/s peak, the FP64
oracle's throughput on a bounded CPU sample, and the rel-L2 of the final
periodic state against the exact discrete FP64 evolution.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "GLUPS + % HBM peak; surrogate vs plain LBM time at rel-L2 <= 1e-3"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = 160  # 20 FP32 populations read + 20 written per node update


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-parity", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=30)
    ap.add_argument("--batch-instances", type=int, default=512)
    ap.add_argument("--batch-steps", type=int, default=2000)
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--no-load-leg", action="store_true")
    ap.add_argument("--surrogate-weights", default=os.path.join(
        ROOT, "paper_2408_01081_amd", "weights", "surrogate.npy"))
    ap.add_argument("--step-configs", default="",
                    help="force single-step launch configurations 'P,D' (periodic, Dirichlet) "
                         "instead of autotuning, e.g. to profile what a timed run chose")
    ap.add_argument("--tblock-configs", default="",
                    help="with --step-configs: temporally blocked variants 'P,D' (-1 = single "
                         "steps only)")
    return ap.parse_args()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the lattice workload is measured on one "
              "GPU's share; runs over several GPUs are not supported (asked for --gpus %d)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2408_01081_amd.lbm import Lattice

    dev = torch.device("cuda:0")
    K, W = args.steps, args.warmup
    total = K + W

    # ---- problems (config: 4096^2 periodic + 2048x1024 Dirichlet) -----------
    t0 = time.time()
    per = synth.plane_wave_problem(4096, 4096, synth.PERIODIC, seed=2)
    dir_ = synth.plane_wave_problem(2048, 1024, synth.DIRICHLET, seed=2, dx=1.0 / 1024)
    # both lattices on the current stream, one after the other: each kernel's
    # launch duration is then its own (two streams overlapped the lattices'
    # launches by about 2% of the step time and blurred the per-kernel times)
    lats, fields = [], []
    for prob in (per, dir_):
        v0, sb0 = prob.initial_fields()
        v0, sb0 = torch.from_numpy(v0).to(dev), torch.from_numpy(sb0).to(dev)
        lat = Lattice(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
        lat.init(v0, sb0)
        if prob.bc == synth.DIRICHLET:
            Wt, Tt = prob.wall_table(max(total, RERANK_STEPS + 64))
            lat.set_wall_velocity(torch.from_numpy(Wt).to(dev), torch.from_numpy(Tt).to(dev))
        lats.append(lat)
        fields.append((v0, sb0))
    torch.cuda.synchronize()
    log("setup %.1fs" % (time.time() - t0))

    nodes = per.nx * per.ny + dir_.nx * dir_.ny
    # launch configuration chosen by the autotuner (state-preserving): the best
    # single-step configuration and, when faster per step, a two-step variant
    from paper_2408_01081_amd.lbm import step_configs
    cfgs = step_configs()
    tuned = []
    per_step_pick = []  # the autotuner's blocked variant (fastest per step), before the re-rank
    forced = [int(v) for v in args.step_configs.split(",")] if args.step_configs else None
    forced2 = [int(v) for v in args.tblock_configs.split(",")] if args.tblock_configs else None
    for li, lat in enumerate(lats):
        if forced:
            # the autotuner's choices for the launches that take the steps after
            # the last full one (it times every variant), then the forced ones
            lat.autotune(reps=3, use_cache=True)
            lat.step_config = forced[li]
            lat.tblock_config = forced2[li] if forced2 else -1
        else:
            lat.autotune(reps=10, use_cache=True)
            per_step_pick.append(lat.tblock_config)
            lat.select_for_steps(min(K, RERANK_STEPS))   # cheapest for the run length
            rerank(lat, fields[li], min(K, RERANK_STEPS))
        idx, idx2 = lat.step_config, lat.tblock_config
        c = cfgs[idx]
        t = {"lattice": "%dx%d" % (lat.nx, lat.ny), "config": idx, "vec": c["vec"],
             "threads": c["threads"], "nontemporal": c["nontemporal"], "shuffle": c["shuffle"],
             "tblock_config": idx2}
        if idx2 >= 0:
            t["tblock"] = next(k for k in lat.tblock_configs() if k["index"] == idx2)
        tuned.append(t)
    fields = None  # the initial fields were kept for the re-rank only
    log("autotuned: %s" % tuned)
    if forced:
        # without the autotuner nothing has launched the kernels of the timed
        # region yet: run one full launch and the launch for the steps after
        # the last full one (untimed set-up), so no first-launch cost of a
        # kernel falls into the timed region
        for lat in lats:
            T = lat.steps_per_launch
            lat.step(T + K % T)
    for lat in lats:
        lat.step(W)
    torch.cuda.synchronize()

    # ---- timed region ----------------------------------------------------------
    # each lattice's K steps, as lbm_step runs them: full launches of T steps,
    # then one launch for the K mod T steps left; events on the stream the
    # kernels run on mark the full launches apart from the rest, and each full
    # launch of the periodic lattice on its own, so the dominant kernel's
    # average launch time comes from its own launches (without the gaps
    # between them)
    stream = torch.cuda.current_stream(dev)
    E = lambda: torch.cuda.Event(enable_timing=True)
    start, end = E(), E()
    ev = [[E(), E(), E()], [E(), E(), E()]]
    Ts = [lat.steps_per_launch for lat in lats]
    lev = [(E(), E()) for _ in range(K // Ts[0])]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for li, lat in enumerate(lats):
        full = K // Ts[li] * Ts[li]
        ev[li][0].record(stream)
        if li == 0:
            for a0, a1 in lev:
                a0.record(stream)
                lat.step(Ts[0])
                a1.record(stream)
        else:
            lat.step(full)
        ev[li][1].record(stream)
        lat.step(K - full)
        ev[li][2].record(stream)
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = start.elapsed_time(end)
    ms_per_step = ms_total / K
    glups = nodes * K / (ms_total * 1e-3) / 1e9
    log("timed: %d steps in %.3f s (events %.3f s)" % (K, wall, ms_total * 1e-3))

    # ---- dominant kernel: the 4096^2 periodic lattice's kernel -----------------
    # Its average launch duration comes from the periodic lattice's part of the
    # timed region (HIP events on the stream its kernels run on).  Algorithmic bytes
    # per launch: every node's 20 FP32 populations read once and written once
    # (160 B per node), for one time step (k_step) or T (k_tblock).
    per_lat = lats[0]
    blocked = tuned[0]["tblock_config"] >= 0
    T = Ts[0]
    assert T == (tuned[0]["tblock"]["steps"] if blocked else 1)
    launches = K // T
    if launches > 0:
        kern_ms = sum(a0.elapsed_time(a1) for a0, a1 in lev) / launches
        kern_src = ("HIP events around each of the %d full launches of the timed region "
                    "(mean)" % launches)
    else:  # fewer timed steps than one launch takes: time the launch apart
        kern_ms = (per_lat.time_tblock_config(tuned[0]["tblock_config"], 20) if blocked
                   else per_lat.time_step_config(tuned[0]["config"], 20))
        kern_src = "20 launches timed apart (the timed region has no full launch)"
    rest = K - launches * T
    alg_bytes = BYTES_PER_LUP * per.nx * per.ny
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    kname = "k_tblock" if blocked else "k_step"
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname, launch_key(tuned[0])),
                "kernel": "%s (periodic 4096x4096, %s)" % (
                    kname, ("blocked variant %d, %d steps per launch"
                            % (tuned[0]["tblock_config"], T)) if blocked
                    else ("config %d" % tuned[0]["config"])),
                "kernel_ms": round(kern_ms, 5), "kernel_ms_from": kern_src,
                "full_launches_ms_per_launch": (
                    round(ev[0][0].elapsed_time(ev[0][1]) / launches, 5) if launches else None),
                "launches": launches, "steps_per_launch": T,
                "steps_after_full_launches": {
                    "steps": rest, "ms": round(ev[0][1].elapsed_time(ev[0][2]), 5),
                    "launch": ("none" if rest == 0 else "single-step kernel" if rest == 1
                               else "one %d-step blocked launch" % rest)},
                "kernel_glups": round(T * per.nx * per.ny / kern_ms / 1e6, 2),
                "algorithmic_bytes_per_launch": alg_bytes}
    if blocked:
        # the best single-step kernel on the same lattice, for comparison: its
        # bandwidth fraction is the kernel-quality figure of the one-step form
        ms1 = per_lat.time_step_config(tuned[0]["config"], reps=50)
        roofline["single_step_reference"] = {
            "kernel": "k_step (config %d)" % tuned[0]["config"], "ms": round(ms1, 5),
            "GB/s": round(alg_bytes / (ms1 * 1e-3) / 1e9, 1),
            "frac": round(alg_bytes / (ms1 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "glups": round(per.nx * per.ny / ms1 / 1e6, 2)}
        # the variant fastest per step, where the run length made the re-rank
        # choose another one (e.g. T = 10 for 20-step runs against T = 8)
        pick = per_step_pick[0] if per_step_pick else -1
        if pick >= 0 and pick != tuned[0]["tblock_config"]:
            ms8 = per_lat.time_tblock_config(pick, 20)
            Tp = next(k["steps"] for k in per_lat.tblock_configs() if k["index"] == pick)
            roofline["per_step_best_reference"] = {
                "kernel": "k_tblock (blocked variant %d, %d steps per launch), the tuner's fastest "
                          "per step" % (pick, Tp),
                "ms": round(ms8, 5), "ms_per_step": round(ms8 / Tp, 5),
                "GB/s": round(alg_bytes / (ms8 * 1e-3) / 1e9, 1),
                "frac": round(alg_bytes / (ms8 * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "glups": round(Tp * per.nx * per.ny / ms8 / 1e6, 2),
                "selected_ms_per_step": round(kern_ms / T, 5)}
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    # ---- reference: plain streaming copy of one population buffer -------------
    from paper_2408_01081_amd.lbm import copy_f32
    nflt = 20 * per.nx * per.ny
    src = torch.ones(nflt, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        copy_f32(dst, src)
    a.record(stream)
    for _ in range(20):
        copy_f32(dst, src)
    b.record(stream)
    torch.cuda.synchronize()
    copy_ms = a.elapsed_time(b) / 20
    copy_ref = {"kernel": "k_copy (16 B/lane, nontemporal stores)",
                "bytes_per_launch": 8 * nflt, "ms": round(copy_ms, 5),
                "GB/s": round(8 * nflt / (copy_ms * 1e-3) / 1e9, 1)}
    roofline["copy_reference"] = copy_ref
    del src, dst

    # ---- parity of the final periodic state vs the exact FP64 evolution -------
    parity = None
    if not args.no_parity:
        try:
            parity = periodic_parity(per, per_lat)
        except Exception as ex:  # reported, never hidden
            parity = {"error": repr(ex)}

    del lats, per_lat
    torch.cuda.empty_cache()

    # ---- the step with a body load and the displacement output ----------------
    with_load = with_load_blocked = with_load_single = None
    if not args.no_load_leg:
        tb = tuned[0]["tblock_config"]
        legs = {}
        for key, kw in (("disp", dict(nsteps=400, disp=True, tblock=tb)),
                        ("load", dict(nsteps=400, disp=False, tblock=tb)),
                        ("single", dict(nsteps=200, disp=True, tblock=-1))):
            try:
                legs[key] = load_leg(**kw)
            except Exception as ex:  # reported, never hidden
                legs[key] = {"error": repr(ex)}
        with_load, with_load_blocked, with_load_single = legs["disp"], legs["load"], legs["single"]

    # ---- batched instances: one hipGraph launch of many steps ------------------
    batched = None
    if args.batch_instances > 0 and args.batch_steps > 0:
        batched = batched_leg(args.batch_instances, args.batch_steps)

    # ---- learned surrogate: MFMA throughput and surrogate + judge rollout -----
    surrogate = None
    if not args.no_surrogate:
        try:
            surrogate = surrogate_leg(args.surrogate_weights)
        except Exception as ex:  # reported, never hidden
            surrogate = {"error": repr(ex)}

    # ---- CPU baseline: the FP64 oracle on a bounded sample ---------------------
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(per, dir_, args.cpu_sample_steps)

    out = {
        "metric": METRIC, "value": round(glups, 3), "unit": "GLUPS", "n_gpus": 1,
        "steps": K, "warmup": W, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "plain LBM FP32: periodic 4096x4096 + Dirichlet 2048x1024 "
                               "(time-dependent manufactured walls), plane-wave data, "
                               "nu seeded (%.4f / %.4f), rho = 1, half CFL limit" %
                               (per.meta["nu"], dir_.meta["nu"]),
                   "nodes_per_step": nodes, "precision": "FP32 populations, FP64 init",
                   "step_configs": tuned},
        "hbm_frac": roofline["frac"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
        "with_load_and_displacement": with_load,
        "with_load": with_load_blocked,
        "with_load_and_displacement_one_launch_per_step": with_load_single,
        "batched": batched,
        "surrogate": surrogate,
        "wall_s": round(wall, 3),
    }
    print(json.dumps(out), flush=True)


def launch_key(t):
    """Launch properties the stored counter results are keyed on."""
    if t["tblock_config"] >= 0:
        b = t["tblock"]
        return "T=%d seg=%d nt=%d pf=%d" % (b["steps"], b["seg_rows"], b["nontemporal"],
                                           b["prefetch"])
    return "vec=%d threads=%d nt=%d shuffle=%d" % (t["vec"], t["threads"], t["nontemporal"],
                                                   t["shuffle"])


RERANK_STEPS = 840  # steps each candidate of the re-rank is timed for


def rerank(lat, fields, run_steps, top=4):
    """The autotuner times repeated launches from one buffer, which on grids
    smaller than the device's last-level cache stays resident there; real
    stepping alternates two buffers, and a run of n steps pays for the launch
    that takes the n mod T steps after the last full one.  Time the
    autotuner's choice and the blocked variants its launch timing ranks best
    per step by stepping runs of the benchmark's own length (run_steps steps
    per call, repeated up to RERANK_STEPS steps), keep the fastest, and
    re-initialise the lattice (state and step count as before)."""
    import torch
    per_step = sorted((lat.time_tblock_config(c["index"], 5) / c["steps"], c["index"])
                      for c in lat.tblock_configs())
    cands = [lat.tblock_config] + [i for _, i in per_step[:top] if i != lat.tblock_config]
    reps = max(1, RERANK_STEPS // run_steps)
    best = None
    for idx in cands:
        lat.init(*fields)
        lat.tblock_config = idx
        lat.step(64)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            lat.step(run_steps)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        if best is None or ms < best[0]:
            best = (ms, idx)
    lat.init(*fields)
    lat.tblock_config = best[1]
    torch.cuda.synchronize()


def measured_traffic(kname, launch):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, if one was taken on the current device code of that
    kernel and on the launch configuration this run uses."""
    path = os.path.join(ROOT, "profiles", "%s_periodic_4096_traffic.json" % kname)
    if not os.path.exists(path):
        return None
    try:
        from paper_2408_01081_amd import build as B
        h = B.kernel_hash(kname)
        for e in json.load(open(path)).get("entries", []):
            if e.get("source_sha256") == h and e.get("launch") == launch:
                return e.get("bytes_per_launch")
    except Exception:
        return None
    return None


def periodic_parity(prob, lat, nsample=4096):
    import numpy as np

    import oracle
    from oracle import spectral
    n = lat.steps
    s = oracle.Setup(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, prob.bc)
    g = np.random.default_rng(123)
    iy = g.integers(0, prob.ny, nsample)
    ix = g.integers(0, prob.nx, nsample)
    want = spectral.plane_wave_reference(s, prob.sol, n, iy, ix)
    U = lat.moments_U()
    import torch
    got = U[:, torch.from_numpy(iy).to(U.device), torch.from_numpy(ix).to(U.device)]
    got = got.double().cpu().numpy()
    return {"against": "exact FP64 discrete evolution (per Fourier mode) of the same scheme",
            "lattice": "periodic 4096x4096", "steps": n, "nodes_sampled": nsample,
            "rel_l2": float(np.sqrt(np.sum((got - want) ** 2) / np.sum(want ** 2)))}


def batched_leg(n, nsteps):
    """n seeded instances (sides U[64, 512], half Dirichlet, per-instance
    material and time step, GRF data) advanced nsteps in one hipGraph launch."""
    import torch

    import synth
    from paper_2408_01081_amd.batch import Batch
    t0 = time.time()
    probs = synth.batched_instances(n, seed=3)
    b = Batch([dict(nx=p.nx, ny=p.ny, dx=p.dx, dt=p.dt, lam=p.lam, mu=p.mu, rho=p.rho, bc=p.bc)
               for p in probs])
    b.init(b.pack([p.v0 for p in probs]), b.pack([p.sb0 for p in probs]))
    E0 = b.energy()
    tb, tb_ms = b.autotune(reps=5)   # single steps or a temporally blocked variant
    b.step(nsteps)            # builds (and caches) the graph, warms up
    torch.cuda.synchronize()
    log("batched setup + first graph %.1fs" % (time.time() - t0))
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(nsteps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    E1 = b.energy()
    nodes = b.total_nodes
    import numpy as np
    drift = float(np.max(np.abs(E1 - E0) / E0))
    out = {"workload": "%d instances, sides U[64,512], %d Dirichlet (homogeneous walls), "
                       "nu U[0,0.49], rho U[0.5,2], GRF data, FP32" %
                       (n, sum(p.bc for p in probs)),
           "nodes": nodes, "steps": nsteps, "graph_launches": 1, "ms": round(ms, 3),
           "GLUPS": round(nodes * nsteps / (ms * 1e-3) / 1e9, 3),
           "tblock": b.tblock_configs()[tb] if tb >= 0 else None,
           "algorithmic_GB/s": round(160 * nodes * nsteps / steps_per_launch(b, tb)
                                     / (ms * 1e-3) / 1e9, 1),
           "max_rel_energy_drift": drift}
    # the same instances with moving walls on every Dirichlet one (seeded
    # rank-4 separable data): blocked launches read per-launch wall tables;
    # the graph of each call is built inside the timed call
    dev = torch.device("cuda")
    for i, p in enumerate(probs):
        if p.bc == synth.DIRICHLET:
            W, T = synth.oscillating_walls(p.nx, p.ny, p.dt, 3 * nsteps + 64, rank=4,
                                           seed=1000 + i)
            b.set_wall_velocity(i, torch.from_numpy(W).float().to(dev),
                                torch.from_numpy(T).float().to(dev))
    mw = {}
    for label, cfg in (("tuned", None), ("single_steps", -1)):
        b.init(b.pack([p.v0 for p in probs]), b.pack([p.sb0 for p in probs]))
        if cfg is None:
            cfg, _ = b.autotune(reps=3)
        else:
            b.tblock_config = cfg
        torch.cuda.synchronize()
        e0.record(stream)
        b.step(nsteps)
        e1.record(stream)
        torch.cuda.synchronize()
        msw = e0.elapsed_time(e1)
        mw[label] = {"ms": round(msw, 3), "GLUPS": round(nodes * nsteps / (msw * 1e-3) / 1e9, 3),
                     "tblock": b.tblock_configs()[cfg] if cfg >= 0 else None}
    out["moving_walls"] = {"walls": "rank-4 separable wall velocities on the %d Dirichlet "
                                    "instances, %d steps" % (sum(p.bc for p in probs), nsteps),
                           **mw}
    return out


def load_leg(nsteps=200, disp=True, tblock=None):
    """The 4096^2 periodic lattice stepped with a body load (the standing
    manufactured solution's, separable, rank 16), with or without the FP64
    displacement state, blocked variant `tblock` selected (-1: one launch per
    step): the optional outputs' cost, reported beside the plain step."""
    import numpy as np
    import torch

    import synth
    from paper_2408_01081_amd.lbm import Lattice
    N = 4096
    mat = synth.Material.from_lame(1.0, 0.5, 1.0)
    e = synth.Elastodynamics(*synth.standing_mms_solution(), mat)
    dx = 1.0 / N
    prob = synth.Problem(N, N, dx, synth.dt_at_cfl_fraction(dx, mat, 0.5), 1.0, 0.5, 1.0,
                         synth.PERIODIC, sol=e)
    dev = torch.device("cuda:0")
    lat = Lattice(N, N, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho, synth.PERIODIC,
                  displacement=disp)
    if tblock is not None:
        lat.tblock_config = tblock
    BX, BY, BT = prob.body_table(2 * nsteps + 10)
    lat.set_body_force(*(torch.from_numpy(a).to(dev) for a in (BX, BY, BT)))
    v0, sb0 = prob.initial_fields()
    lat.init(torch.from_numpy(v0).to(dev), torch.from_numpy(sb0).to(dev))
    if disp:
        X, Y = synth.node_coords(N, N, dx)
        lat.init_displacement(torch.from_numpy(np.stack([e.ux(X, Y, 0.0),
                                                         e.uy(X, Y, 0.0)])).to(dev))
    lat.step(10)
    stream = torch.cuda.current_stream(dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    lat.step(nsteps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / nsteps
    T = lat.steps_per_launch
    extra = " + FP64 displacement state" if disp else ""
    per_launch = BYTES_PER_LUP + (32 if disp else 0)  # B per node and launch
    out = {"workload": "periodic 4096x4096, body load of rank %d (standing manufactured "
                       "solution)%s, %d step(s) per launch" % (BX.shape[0], extra, T),
           "kernel": ("k_tblock with load%s" % (" and displacement" if disp else "")) if T > 1
           else "k_step_ext",
           "steps": nsteps, "ms_per_step": round(ms, 5), "GLUPS": round(N * N / ms / 1e6, 2),
           "steps_per_launch": T,
           "algorithmic_bytes_per_node_update": round(per_launch / T, 2)}
    if T == 1:
        alg = per_launch * N * N
        out["algorithmic_GB/s"] = round(alg / (ms * 1e-3) / 1e9, 1)
        out["frac"] = round(alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
    del lat
    torch.cuda.empty_cache()
    return out


def steps_per_launch(b, tb):
    return b.tblock_configs()[tb]["steps"] if tb >= 0 else 1


BF16_PEAK_TFLOPS = 2500.0
FP32_MFMA_PEAK_TFLOPS = 157.3


def unet_flops(H, W, B, padded=False):
    """Multiply-add FLOPs of one U-Net forward (3x3 convolutions only), on
    the network's own channels (5 real input fields into the first layer, 5
    real outputs of the last), or as the kernels run them (padded=True: 32
    channels there, one matrix-core pass)."""
    from paper_2408_01081_amd.surrogate import forward_flops
    return forward_flops(B, H, W, padded=padded)


def window_op_tiles(H, W, B):
    """(matrix tiles per wave, column tiles per workgroup) that lbm_wop_apply
    picks for B windows of H x W: 2, 2 where that gives >= 512 workgroups,
    else 2, 1 where that does, else 1, 2, else 1, 1, each only while it
    computes at most 15% more columns than 16-column granularity."""
    ty = (H + 2) // 3
    c16 = (W + 15) // 16 * 16
    def ok(cols, min_wgs):
        n = (W + cols - 1) // cols
        return n * cols * 100 <= c16 * 115 and n * ty * B >= min_wgs
    if ok(64, 512):
        return 2, 2
    if ok(32, 512):
        return 2, 1
    if ok(32, 0):
        return 1, 2
    return 1, 1


def window_op_flops(H, W, B):
    """(useful, issued) FLOPs of one application of the exact window
    operator: 2 x 5 x 5 per tap of the diamond |dx| + |dy| <= 17 (613 taps)
    per output node, and what the matrix-core kernel issues (16 x 16 x 4
    products, 5 x 48 x 4 = 960 per tile of 16 columns x 3 rows, padding
    included, over the columns of the workgroups window_op_tiles gives)."""
    R = 17
    taps = 2 * R * R + 2 * R + 1
    useful = 2 * taps * 25 * H * W * B
    mt, nct = window_op_tiles(H, W, B)
    cols = 16 * mt * nct
    tiles = ((W + cols - 1) // cols) * mt * nct * ((H + 2) // 3) * B
    issued = 2 * 16 * 16 * 4 * 960 * tiles
    return useful, issued


def surrogate_leg(weights_path):
    """MFMA throughput of the surrogate kernels and the serving comparison on
    a 256x256 Dirichlet lattice: 4096 steps as 256 windows of 16 steps."""
    import numpy as np
    import torch

    import synth
    from paper_2408_01081_amd import serve
    from paper_2408_01081_amd.surrogate import Surrogate, init_params, pack_params
    out = {}
    trained = os.path.exists(weights_path)
    params = (np.load(weights_path, allow_pickle=False) if trained
              else pack_params(init_params(0, 0.0)).astype(np.float32))
    out["weights"] = os.path.relpath(weights_path, ROOT) if trained else "untrained (identity)"
    # forward throughput at the serving size and training-step throughput
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for (B, H, split) in ((1, 256, 3), (32, 128, 3)):
        net = Surrogate(B, H, H, split=split)
        net.set_params(params)
        x = torch.randn(B, 8, H, H, device="cuda")
        x[:, 5], x[:, 6], x[:, 7] = 0.5, 1.0, 1.0
        for _ in range(3):
            net.forward(x)
        e0.record()
        for _ in range(20):
            net.forward(x)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 20
        fl = unet_flops(H, H, B)
        flp = unet_flops(H, H, B, padded=True)
        out["forward_b%d_%d" % (B, H)] = {
            "ms": round(ms, 4), "GFLOP": round(fl / 1e9, 2),
            "TFLOP/s": round(fl / ms / 1e9, 2),
            "frac_of_bf16_peak": round(fl / ms / 1e9 / BF16_PEAK_TFLOPS, 4),
            "note": "FLOP of the network's own channels, one pass; the kernels run %d BF16 "
                    "matrix-core passes (hi/lo split) over padded channels: %.1f TFLOP/s issued"
                    % (split, split * flp / ms / 1e9)}
        del net
    # training step (forward, loss, backward, Adam) at the training shape
    B, H = 32, 128
    net = Surrogate(B, H, H, split=3, train=True)
    net.set_params(params)
    x = torch.randn(B, 8, H, H, device="cuda")
    x[:, 5], x[:, 6], x[:, 7] = 0.5, 1.0, 1.0
    tgt = x[:, :5].contiguous()
    for _ in range(3):
        net.train_step(x, tgt, lr=0.0, want_loss=False)
    e0.record()
    for _ in range(10):
        net.train_step(x, tgt, lr=0.0, want_loss=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / 10
    fl = 3 * unet_flops(H, H, B)  # forward + data gradients + weight gradients
    out["train_step_b%d_%d" % (B, H)] = {
        "ms": round(ms, 4), "GFLOP": round(fl / 1e9, 2), "TFLOP/s": round(fl / ms / 1e9, 2),
        "frac_of_bf16_peak": round(fl / ms / 1e9 / BF16_PEAK_TFLOPS, 4),
        "note": "forward + backward (data and weight gradients of every convolution) + Adam; "
                "FLOP of the network's own channels counted as three forward passes, one "
                "matrix-core pass each"}
    del net
    out["window_operator"] = window_operator_leg()
    # serving comparison (C5 shape): seeded material and GRF data
    prob = synth.grf_problem(256, 256, synth.DIRICHLET, seed=5)
    plain_ms, variant, plain_final, variants = serve.plain_time_to_solution(prob, 4096, reps=3)
    net = Surrogate(1, 256, 256, split=3)
    net.set_params(params)
    ro_ms, state, st = serve.rollout_time_to_solution(net, prob, 256, chunk=32, tol=1e-3,
                                                      reps=1)
    a = state.double().flatten()
    bref = plain_final.double().flatten()
    out["serving"] = {
        "workload": "256x256 Dirichlet, nu %.3f rho %.3f, GRF data, 4096 steps = 256 windows of 16"
                    % (prob.meta["nu"], prob.lam * 0 + prob.rho),
        "plain_lbm_ms": round(plain_ms, 3), "plain_variant": variant,
        "plain_variants_ms": {k: round(v, 3) for k, v in variants.items()},
        "surrogate_judge_ms": round(ro_ms, 2),
        "speedup_vs_plain": round(plain_ms / ro_ms, 4),
        "tolerance": 1e-3, **st,
        "final_rel_l2_vs_plain_fields": float(((a - bref).norm() / bref.norm()).item())}
    return out


def _omp_threads(n):
    """Set the OpenMP thread count of the oracle's runtime (the system
    libgomp the C oracle links); returns the previous count."""
    import ctypes
    g = ctypes.CDLL("libgomp.so.1")
    old = g.omp_get_max_threads()
    g.omp_set_num_threads(int(n))
    return old


def window_operator_leg():
    """The exact linear window operator (16 lattice steps of a periodic
    lattice as one FP32 matrix-core convolution): build and apply times, its
    rate against the FP32 matrix-core peak, 16 lattice steps of the same
    lattice, and the serving comparison on a periodic 256x256 problem with
    the operator in the surrogate's place."""
    import numpy as np
    import torch

    import synth
    from paper_2408_01081_amd import serve
    from paper_2408_01081_amd.window import WindowOperator, WindowSurrogate
    out = {}
    prob = synth.grf_problem(256, 256, synth.PERIODIC, seed=5)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    op = WindowOperator(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho)
    out["build_ms"] = round((time.perf_counter() - t0) * 1e3, 2)
    for B, H in ((1, 256), (32, 128)):
        o = op if H == 256 else WindowOperator(H, H, prob.dx, prob.dt, prob.lam, prob.mu,
                                               prob.rho)
        x = torch.randn(B, 5, H, H, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            o.apply(x, out=y)
        e0.record()
        for _ in range(50):
            o.apply(x, out=y)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 50
        useful, issued = window_op_flops(H, H, B)
        out["apply_b%d_%d" % (B, H)] = {
            "ms": round(ms, 4), "GFLOP": round(useful / 1e9, 3),
            "TFLOP/s": round(useful / ms / 1e9, 2),
            "frac_of_fp32_mfma_peak": round(useful / ms / 1e9 / FP32_MFMA_PEAK_TFLOPS, 4),
            "issued_TFLOP/s": round(issued / ms / 1e9, 2),
            "issued_frac": round(issued / ms / 1e9 / FP32_MFMA_PEAK_TFLOPS, 4)}
    plain_ms, variant, plain_final, variants = serve.plain_time_to_solution(prob, 4096, reps=3)
    ro_ms, state, st = serve.rollout_time_to_solution(WindowSurrogate(op), prob, 256, chunk=32,
                                                      tol=1e-3, reps=3)
    a = state.double().flatten()
    bref = plain_final.double().flatten()
    out["serving_periodic"] = {
        "workload": "256x256 periodic, nu %.3f rho %.3f, GRF data, 4096 steps = 256 windows "
                    "of 16, the exact operator in the surrogate's place"
                    % (prob.meta["nu"], prob.rho),
        "plain_lbm_ms": round(plain_ms, 3), "plain_variant": variant,
        "plain_ms_per_16_steps": round(plain_ms / 256, 4),
        "operator_judge_ms": round(ro_ms, 3), "speedup_vs_plain": round(plain_ms / ro_ms, 4),
        "tolerance": 1e-3, **st,
        "final_rel_l2_vs_plain_fields": float(((a - bref).norm() / bref.norm()).item())}
    return out


def cpu_baseline(per, dir_, nsteps, single_steps=4):
    """Time the FP64 oracle (as it stands) on a bounded sample of the same
    workload: nsteps steps of each lattice from its initial state on all of
    the host's cores, then single_steps steps of each on one core.  The
    periodic lattice runs the oracle's C step loop; the Dirichlet lattice
    steps through the oracle's per-step driver with the benchmark's
    time-dependent wall velocities (summed from the closed form every step)."""
    import oracle

    def sample(n):
        t_total, lups = 0.0, 0
        for prob in (per, dir_):
            s = oracle.Setup(prob.nx, prob.ny, prob.dx, prob.dt, prob.lam, prob.mu, prob.rho,
                             prob.bc)
            v0, sb0 = prob.initial_fields()
            if prob.bc == oracle.DIRICHLET:
                sim = oracle.Simulation(s, v0, sb0, wall=prob.wall_velocity)
                del v0, sb0
                t0 = time.perf_counter()
                sim.advance(n)
                t_total += time.perf_counter() - t0
                del sim
            else:
                f = oracle.init_populations(s, s.U_from_fields(v0, sb0))
                del v0, sb0
                t0 = time.perf_counter()
                oracle.run_free(s, f, n)
                t_total += time.perf_counter() - t0
                del f
            lups += prob.nx * prob.ny * n
        return lups / t_total / 1e9, t_total

    cores = int(oracle.lib().orc_threads())
    all_glups, all_s = sample(nsteps)
    old = _omp_threads(1)
    try:
        one_glups, one_s = sample(single_steps)
    finally:
        _omp_threads(old)
    return {"value": round(all_glups, 5), "unit": "GLUPS", "cores": cores, "kind": "oracle",
            "sample": "%d steps of each lattice (4096x4096 periodic; 2048x1024 Dirichlet with "
                      "the benchmark's rank-30 time-dependent walls), FP64, step loop only"
                      % nsteps,
            "seconds": round(all_s, 2),
            "single_core": {"value": round(one_glups, 6), "unit": "GLUPS", "cores": 1,
                            "sample": "%d steps of each lattice, same data" % single_steps,
                            "seconds": round(one_s, 2)}}


if __name__ == "__main__":
    main()
