#!/usr/bin/env python3
"""Throughput of the GRPIC hot path on one MI355X.

A step is one full pass of the method over the particles: for the default
workload (the full PIC cycle) the Maxwell sub-steps 1-4, field gather and
hybrid push, deposit, and sub-steps 7-10.  Prints one JSON line with the
particle-steps/s of the whole job, the roofline of the dominant kernel (from
HIP-event timings taken by the library on its own stream) and the CPU oracle
timed on a bounded sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SEED = 2602074520
PEAK_FP64_TFLOPS = 78.6     # MI355X FP64 vector (256 CUs x 2.4 GHz x 128 FLOP/clk)
PEAK_HBM_GBS = 8000.0       # MI355X HBM3E

# Algorithmic FP64 operations per particle, measured on the oracle compiled
# with a counting scalar type (oracle/flopcount.cpp, split-monopole and
# neutral-orbit workloads): additions, subtractions and multiplications count
# one each, and so do divisions, square roots and sin/cos/exp/log calls (their
# numbers are listed apart by the counter).  The counts follow the method as
# the oracle writes it, e.g. the deposit weights evaluate sqrt(gamma) at all
# 4 x 16 trapezoid points with their own sin/cos, where the kernel shares the
# 7 x 7 distinct samples; the kernel's own shared-sample formulation needs
# fewer operations (FLOP_KERNEL_* below, counted by hand on its formulas).
FLOP_RK4_GRID = 1779     # RK4 step with the six fields gathered at every stage
FLOP_RK4_NOGRID = 959    # RK4 step of a neutral particle (no fields)
FLOP_ENERGY = 55         # e = alpha Gamma - beta^r u_r at one state
FLOP_WEIGHTS = 1311      # deposit weights of a position (eqs. v1-v5)
FLOP_IMR_ITER = 455      # one Picard iteration of eq. imr1 (gather included)
FLOP_NEWTON_ITER = 3400  # one Newton iteration (seven evaluations, 6 x 6 solve)
FLOP_HAM_ITER = 3680     # one discrete-gradient iteration (six orderings)
FLOP_GATHER = 145        # one metric-weighted gather of the six components
FLOP_SWITCH = 2 * FLOP_ENERGY + 3
# hand counts of the kernel's formulation (shared samples, factored forms)
FLOP_KERNEL_RK4_GRID = 4 * (89 + 76 + 93) + 90
FLOP_KERNEL_WEIGHTS = 610
# algorithmic HBM bytes per particle of the explicit push pass of a charged
# particle under Hyb2: state in/out (2 x 48), q/m, flags in/out, herr out,
# iterations, old position (2 x 8) + dphi (FP32), new weights (three
# stored in 4 B fixed point, the fourth is their complement) + cell (a
# neutral particle also reads H0, Hyb1 herr)
BYTES_PUSH = 48 + 1 + 1 + 48 + 1 + 8 + 1 + 20 + 12 + 4
# deposit per particle: old/new weights (three each, 4 B fixed point) and
# cells, q/m, w, dphi (FP32), flags
BYTES_DEPOSIT = 12 + 12 + 4 + 4 + 1 + 8 + 4 + 1
# one launch of the Maxwell group (sub-steps 1-4, or 7-10) per cell: about 65
# FP32 arrays read or written (two constitutive updates with their metric
# coefficient tables and two curl updates)
BYTES_FIELDS_PER_CELL = 65 * 4
# the paper's current (deposit mode "paper"), per particle: r, theta, u_r,
# u_theta, u_phi, w (FP64), q/m and flags, node weights W1..W3 (4 B fixed
# point) and cell
BYTES_DEPOSIT_PAPER = 6 * 8 + 1 + 1 + 12 + 4
# divergence cleaning, per node and chain: every Jacobi sweep reads phi, the
# source and the two face coefficients and writes phi (5 x 8 B); the source
# and correction kernels about 100 B more
BYTES_CLEAN_SWEEP = 40
BYTES_CLEAN_FIXED = 100


# Kernel per timing group, as named in rocprofv3 traces, and the source files
# that determine its code: a committed counter summary is only used while its
# recorded hash of these files still matches.
GROUP_KERNEL = {"push": "k_push_explicit", "implicit": "k_push_implicit",
                "deposit": "k_deposit", "fields": "k_ampere", "sort": "k_tile_scatter",
                "clean": "k_clean_jacobi"}
GROUP_SOURCES = {"push": "push.hip", "implicit": "push.hip", "deposit": "deposit.hip",
                 "fields": "maxwell.hip", "sort": "particles.hip", "clean": "clean.hip"}


def kernel_source_hash(group):
    import hashlib
    h = hashlib.sha256()
    src = os.path.join(ROOT, "paper_2602_07452_amd", "csrc")
    files = [GROUP_SOURCES[group]] + sorted(f for f in os.listdir(src) if f.endswith(".hpp"))
    for f in files:
        with open(os.path.join(src, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    with open(os.path.join(ROOT, "include", "grpic.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()


def counter_traffic(group, workload, particles):
    """HBM bytes per launch of a timing group's kernel from the committed
    FETCH_SIZE / WRITE_SIZE summary (each counter scaled by its copy-kernel
    calibration factor); None when there is no summary for this workload or
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{group}_{workload}_counters.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != kernel_source_hash(group):
        return None
    if int(kv.get("particles", -1)) != particles:
        return None
    fetch = float(kv["fetch_kib_per_launch"]) * 1024 * float(kv["fetch_factor"])
    write = float(kv["write_kib_per_launch"]) * 1024 * float(kv["write_factor"])
    return fetch + write


def rplus(a):
    return 1.0 + np.sqrt(1.0 - a * a)


WORKLOADS = {
    "c3": dict(
        desc=("full PIC cycle, plasma-filled Wald magnetosphere: Kerr a=0.99 started "
              "with the a=0 Wald field (grid E=0, D=-beta x B/alpha), "
              "1024x1024 (r,theta) grid r in [0.9 r+, 20], absorbing layer from 18, "
              "2^24 e+/e- macro-particles uniform in proper volume, Maxwell-Juettner "
              "Theta=0.1, FDTD + gather + Hyb2 push (RK4 -> IMR) + conserving deposit"),
        a=0.99, nr=1024, nth=1024, r_out=20.0, n=1 << 24, mode="evolve",
        pusher="hyb2", thr=1e-13, theta=0.1, r_abs=18.0, a_field=0.0),
    "c5": dict(
        desc=("full PIC cycle, split-monopole magnetosphere: Kerr a=0.9, 2048x2048 (r,theta) "
              "grid r in [0.9 r+, 100], absorbing layer from 90, 2^27 e+/e- macro-particles "
              "uniform in proper volume, Maxwell-Juettner Theta=0.05, FDTD + gather + Hyb2 "
              "push (RK4 -> IMR, learned guess) + conserving deposit, step replayed as a "
              "hipGraph"),
        a=0.9, nr=2048, nth=2048, r_out=100.0, n=1 << 27, mode="evolve", fields="monopole",
        pusher="hyb2", thr=1e-13, theta=0.05, r_abs=90.0, graph=1, guess="mlp"),
    "c1": dict(
        desc=("neutral test particles in Schwarzschild (a=0), no fields: 1024 particles, "
              "r in [6, 20], theta in [pi/4, 3pi/4], even ids circular, odd ids eccentric, "
              "dt=0.01, Hyb2 (RK4 -> Hamiltonian discrete gradient) at 1e-15"),
        a=0.0, nr=0, nth=0, r_out=1e9, n=1024, mode="none", pusher="hyb2", thr=1e-15,
        dt=0.01, theta=0.1),
    "c2": dict(
        desc=("charged test particles in the Kerr a=0.9 Wald field (B0=1) on a "
              "512x512 grid, r in [0.9 r+, 50]: 2^20 particles, q/m=+-1, |u|~U[0,1] "
              "isotropic, gather + Hyb2 push (RK4 -> IMR), dt=0.01, no deposit"),
        a=0.9, nr=512, nth=512, r_out=50.0, n=1 << 20, mode="static",
        pusher="hyb2", thr=1e-13, theta=1.0, dt=0.01),
}


def make_context(G, W, n=None, push_wps=0, persistent_waves=0):
    a = W["a"]
    rp = rplus(a)
    evolve = W["mode"] == "evolve"
    n = W["n"] if n is None else n
    if W["mode"] == "none":
        # test particles without fields (circular and eccentric orbits)
        cfg = G.config_default(a=a, dt=W["dt"], pusher=G.PUSH_HYB2, hyb_threshold=W["thr"],
                               max_particles=n, r_remove_in=rp, guess=G.GUESS_RK4)
        ctx = G.Context(cfg)
        ctx.init_particles(G.INIT_ORBITS, n, SEED + 1, 6.0, 20.0, np.pi / 4, 3 * np.pi / 4,
                           W["theta"])
        return ctx, cfg
    cfg = G.config_default(
        a=a, nr=W["nr"], nth=W["nth"], r_in=0.9 * rp, r_out=W["r_out"],
        field_mode=G.FIELDS_EVOLVE if evolve else G.FIELDS_STATIC,
        pusher=G.PUSH_HYB2, hyb_threshold=W["thr"], max_particles=n,
        r_remove_in=rp, r_remove_out=W["r_out"], reflect=1,
        r_abs=W.get("r_abs", 0.0), chi0=1e4 if evolve else 0.0, lambda_abs=5.0,
        guess=G.GUESS_MLP if W.get("guess") == "mlp" else G.GUESS_RK4,
        sort_every=W.get("sort_every", 50),
        push_waves_per_simd=push_wps,
        deposit_mode=G.DEPOSIT_PAPER if W.get("deposit") == "paper" else G.DEPOSIT_CONSERVING,
        clean_every=W.get("clean_every", 0), clean_iters=W.get("clean_iters", 500),
        inj_every=W.get("inj_every", 0), inj_r0=rp, inj_r1=6.0, inj_mult=3.0,
        inj_density=5.0, inj_theta=0.5, inj_seed=SEED + 7,
        solver=G.SOLVER_NEWTON if W.get("solver") == "newton" else G.SOLVER_PICARD)
    if persistent_waves:
        cfg.persistent_waves = persistent_waves
    cfg.dt = 0.5 * G.cfl_dt(cfg) if evolve else W["dt"]
    ctx = G.Context(cfg)
    if W.get("fields") == "monopole":
        ctx.set_fields_split_monopole(1.0, 1e3)
    else:
        ctx.set_fields_wald(1.0, a_field=W.get("a_field"))
    if evolve:
        # weight: plasma frequency omega_p dt = 0.05 at the mean density
        # (4 pi n q^2/m = omega_p^2, n = N w / V, V ~ proper shell volume)
        r0, r1 = rp, W["r_abs"]
        vol = 4.0 * np.pi / 3.0 * (r1 ** 3 - r0 ** 3)
        w = (0.05 / cfg.dt) ** 2 * vol / (4.0 * np.pi * n)
        ctx.init_particles(G.INIT_SHELL_MJ, n, SEED + 3, r0, r1, cfg.theta0,
                           np.pi - cfg.theta0, W["theta"], w=w)
    else:
        ctx.init_particles(G.INIT_SHELL_ISO, n, SEED + 2, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, W["theta"])
    return ctx, cfg


def herr_percentiles(hist):
    c = np.cumsum(hist)
    if c[-1] == 0:
        return {}
    out = {}
    for q in (50, 90, 99):
        b = int(np.searchsorted(c, q / 100.0 * c[-1]))
        out[f"p{q}"] = float(10 ** ((b + 1) / 2.0 - 30.0))  # upper bin edge
    return out


def cpu_baseline(W, cfg, sample_particles, sample_steps):
    """The oracle on the host cores: the particle part (push + deposit) on a
    particle sample and the grid part of a step, combined for the full
    workload's particle count."""
    import oracle as O
    nthreads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    if W["mode"] == "none":
        p = O.init_particles(O.INIT_ORBITS, cfg.a, SEED + 1, W["n"], 6.0, 20.0, np.pi / 4,
                             3 * np.pi / 4, W["theta"])
        P = O.push_params(cfg.a, cfg.dt, pusher=O.HYB2, guess=O.GUESS_RK4,
                          thr=cfg.hyb_threshold, tol=cfg.tol, kmax=cfg.kmax,
                          field_kind=O.FIELDS_NONE, r_min=cfg.r_remove_in, r_max=1e30,
                          th_lo=-1.0, th_hi=10.0)
        t0 = time.perf_counter()
        for _ in range(sample_steps):
            O.push(P, p)
        t = time.perf_counter() - t0
        return {"value": W["n"] * sample_steps / t, "unit": "particle-steps/s",
                "cores": nthreads, "kind": "oracle",
                "sample": f"all {W['n']} particles x {sample_steps} steps"}
    g = O.Grid(cfg.a, cfg.nr, cfg.nth, cfg.r_in, cfg.r_out, cfg.theta0)
    if W.get("fields") == "monopole":
        D, B = O.split_monopole_grid(g, 1.0, 1e3)
    else:
        D, B = O.wald_grid(g, 1.0, a_field=W.get("a_field"))
    G6 = [g.densitize(c, D[c]) for c in range(3)] + [g.densitize(3 + c, B[c]) for c in range(3)]
    evolve = W["mode"] == "evolve"
    if evolve:
        p = O.init_particles(O.INIT_SHELL_MJ, cfg.a, SEED + 3, sample_particles,
                             rplus(cfg.a), W["r_abs"], cfg.theta0, np.pi - cfg.theta0,
                             W["theta"], w=1e-6)
    else:
        p = O.init_particles(O.INIT_SHELL_ISO, cfg.a, SEED + 2, sample_particles, 2.0, 30.0,
                             cfg.theta0, np.pi - cfg.theta0, W["theta"])
    P = O.push_params(cfg.a, cfg.dt, pusher=O.HYB2, guess=O.GUESS_RK4, thr=cfg.hyb_threshold,
                      tol=cfg.tol, kmax=cfg.kmax, field_kind=O.FIELDS_GRID,
                      r_min=cfg.r_remove_in, r_max=cfg.r_remove_out, th_lo=cfg.theta0,
                      th_hi=np.pi - cfg.theta0)
    t0 = time.perf_counter()
    for _ in range(sample_steps):
        old = p.state()[:, :3].copy()
        alive0 = (p.flags & 1) != 0
        O.push(P, p, grid=g, G=G6)
        if evolve:
            alive = alive0 & ((p.flags & 1) != 0)
            O.deposit(g, cfg.dt, old, p.state()[:, :3], p.qm * p.w, alive.astype(np.int32))
    t_part = (time.perf_counter() - t0) / (sample_steps * sample_particles)
    # the same particle work on one thread (a sixteenth of the sample)
    t_part1 = None
    try:
        import ctypes
        gomp = ctypes.CDLL("libgomp.so.1")
        n1 = max(sample_particles // 16, 1024)
        q = O.Particles(n1)
        for k in ("r", "th", "ph", "ur", "uth", "uph", "qm", "w", "H0", "herr"):
            getattr(q, k)[:] = getattr(p, k)[:n1]
        q.flags[:] = p.flags[:n1]
        gomp.omp_set_num_threads(1)
        t0 = time.perf_counter()
        for _ in range(sample_steps):
            old = q.state()[:, :3].copy()
            alive0 = (q.flags & 1) != 0
            O.push(P, q, grid=g, G=G6)
            if evolve:
                alive = alive0 & ((q.flags & 1) != 0)
                O.deposit(g, cfg.dt, old, q.state()[:, :3], q.qm * q.w, alive.astype(np.int32))
        t_part1 = (time.perf_counter() - t0) / (sample_steps * n1)
        gomp.omp_set_num_threads(nthreads)
    except OSError:
        pass
    t_grid = 0.0
    if evolve:
        F = O.Fields.uniform_levels(g, D, B)
        t1 = time.perf_counter()
        O.pic_step(P, g, F, None, absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
        t_grid = time.perf_counter() - t1
    n_full = W["n"]
    rate = n_full / (t_grid + n_full * t_part)
    extra = {}
    if t_part1 is not None:
        extra = {"value_1thread": n_full / (t_grid + n_full * t_part1),
                 "t_particle_1thread_s": t_part1}
    return {"value": rate, "unit": "particle-steps/s", "cores": nthreads, "kind": "oracle",
            **extra,
            "sample": (f"{sample_particles} particles x {sample_steps} steps of push"
                       + (" + deposit, plus one full grid step (Maxwell sub-steps) on the "
                          f"{cfg.nr}x{cfg.nth} grid; rate = N / (t_grid + N t_particle) for "
                          f"N = {n_full}" if evolve else f"; rate for N = {n_full}")),
            "t_particle_s": t_part, "t_grid_s": t_grid}


# the a.0 rows of Table 2 (Sec. 3.1.2): scheme, Delta t_RK4, Delta t_Ham, threshold
TABLE2_A0 = (("RK4", "rk4", 0.05, 0.0, 0.0), ("Ham", "ham", 0.0, 1.0, 0.0),
             ("Hyb1", "hyb1", 0.08, 1.0, 1.5), ("Hyb2", "hyb2", 0.5, 1.0, 1e-15))


def table2_runs(G, W, t_end):
    """The hybrid experiment of Sec. 3.1.2 on the test-particle workload:
    every scheme of the a.0 rows of Table 2 with its own step lengths, each
    particle run on its own clock to t_end.  Reports the wall time, the
    particle-steps taken and the energy violation |H - H0|/H0 at t_end."""
    pushers = {"rk4": G.PUSH_RK4, "ham": G.PUSH_HAM, "hyb1": G.PUSH_HYB1,
               "hyb2": G.PUSH_HYB2}
    n = W["n"]
    out = {"t_end": t_end, "particles": n, "schemes": {}}
    for name, key, dt_rk, dt_ham, thr in TABLE2_A0:
        dt = dt_rk if dt_rk > 0 else dt_ham
        cfg = G.config_default(a=W["a"], dt=dt, dt_implicit=dt_ham, t_end=t_end,
                               pusher=pushers[key], hyb_threshold=thr, max_particles=n,
                               r_remove_in=rplus(W["a"]))
        with G.Context(cfg) as ctx:
            ctx.init_particles(G.INIT_ORBITS, n, SEED + 1, 6.0, 20.0, np.pi / 4,
                               3 * np.pi / 4, W["theta"])
            # enough steps for the clock that only takes the shorter step
            nsteps = int(np.ceil(t_end / min(dt, dt_ham if dt_ham > 0 else dt))) + 1
            ctx.sync()
            t0 = time.perf_counter()
            ctx.step(nsteps)
            ctx.sync()
            wall = time.perf_counter() - t0
            d = ctx.diagnostics()
            P = ctx.get_particles()
            t = ctx.get_times()
        alive = (P["flags"] & G.FLAG_ALIVE) != 0
        assert np.all(t[alive] == t_end)
        h = P["herr"][alive]
        out["schemes"][name] = {
            "dt_rk4": dt_rk or None, "dt_ham": dt_ham or None, "threshold": thr or None,
            "launches": nsteps, "wall_s": wall, "implicit_particle_steps": int(d["implicit_steps"]),
            "herr_max": float(h.max()), "herr_median": float(np.median(h)),
            "alive": int(alive.sum())}
        print(f"[bench] Table 2 {name}: {wall:.3f} s, |H-H0|/H0 max {h.max():.2e} "
              f"median {np.median(h):.2e}", file=sys.stderr, flush=True)
    return out


def pusher_cost_ratios(G, W, n=1 << 20, dt=0.1, steps=100):
    """The paper's only timing statement (Sec. 3.1, neutral orbits at
    dt = 0.1): wall time of the implicit midpoint rule and of the
    discrete-gradient scheme relative to RK4.  Here per particle-step on the
    GPU, 2^20 particles of the test-particle distribution, each pusher
    alone."""
    out = {"particles": n, "dt": dt, "steps": steps}
    for name, pusher in (("rk4", G.PUSH_RK4), ("imr", G.PUSH_IMR), ("ham", G.PUSH_HAM)):
        cfg = G.config_default(a=W["a"], dt=dt, pusher=pusher, max_particles=n,
                               r_remove_in=rplus(W["a"]))
        with G.Context(cfg) as ctx:
            ctx.init_particles(G.INIT_ORBITS, n, SEED + 1, 6.0, 20.0, np.pi / 4,
                               3 * np.pi / 4, W["theta"])
            ctx.step(5)
            ctx.sync()
            d0 = ctx.diagnostics()
            t0 = time.perf_counter()
            ctx.step(steps)
            ctx.sync()
            t = time.perf_counter() - t0
            d1 = ctx.diagnostics()
        it = (d1["iter_hist"] - d0["iter_hist"]) @ np.arange(len(d1["iter_hist"]))
        impl = d1["implicit_steps"] - d0["implicit_steps"]
        out[name] = {"particle_steps_per_s": d1["alive"] * steps / t, "ms_per_step": t * 1e3 / steps,
                     "mean_iterations": float(it / impl) if impl else None}
    out["imr_over_rk4"] = out["imr"]["ms_per_step"] / out["rk4"]["ms_per_step"]
    out["ham_over_rk4"] = out["ham"]["ms_per_step"] / out["rk4"]["ms_per_step"]
    print(f"[bench] pusher cost ratios: IMR/RK4 {out['imr_over_rk4']:.2f}, "
          f"Ham/RK4 {out['ham_over_rk4']:.2f}", file=sys.stderr, flush=True)
    return out


def learned_vs_plain(G, steps, n=1 << 20, dt=0.01, collect_steps=4, epochs=20):
    """The charged test-particle workload (Kerr a=0.9, Wald field on 512^2,
    2^20 particles) with the implicit midpoint pusher on every particle,
    started from z^n (plain) and from the learned guess.  The network is
    trained on the GPU on the converged steps of collect_steps steps of the
    same workload (other seed).  Both runs converge to the same states, so
    their H errors agree; the rate counts particle-steps per second."""
    a = 0.9
    rp = rplus(a)

    def cfg(guess):
        return G.config_default(a=a, nr=512, nth=512, r_in=0.9 * rp, r_out=50.0, dt=dt,
                                field_mode=G.FIELDS_STATIC, pusher=G.PUSH_IMR,
                                max_particles=n, r_remove_in=rp, r_remove_out=50.0,
                                reflect=1, guess=guess)

    def init(ctx, c, seed):
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, n, seed, 2.0, 30.0, c.theta0,
                           np.pi - c.theta0, 1.0)

    c = cfg(G.GUESS_MLP)
    with G.Context(c) as ctx:
        init(ctx, c, SEED + 2)
        ctx.mlp_collect(collect_steps * n)
        ctx.step(collect_steps)
        ctx.mlp_collect(0)
        samples = ctx.mlp_num_samples()
        t0 = time.perf_counter()
        loss = ctx.mlp_train(epochs=epochs, batch=4096, lr=3e-3, lr_final=3e-5, seed=7)
        t_train = time.perf_counter() - t0
        net = ctx.mlp_get()
    out = {"workload": ("charged test particles, Kerr a=0.9, Wald B0=1 on 512x512, "
                        f"2^20 particles, implicit midpoint on every particle, dt={dt}"),
           "train": {"samples": samples, "epochs": epochs, "batch": 4096,
                     "loss_first_epoch": float(loss[0]), "loss_last_epoch": float(loss[-1]),
                     "seconds": t_train}}
    def run(guess, tol=None, theta=None):
        c = cfg(guess)
        if tol is not None:
            c.tol = tol
        with G.Context(c) as ctx:
            init(ctx, c, SEED + 9)
            if theta is not None:
                ctx.mlp_set(*theta)
            ctx.step(2)
            ctx.sync()
            d0 = ctx.diagnostics()
            t0 = time.perf_counter()
            ctx.step(steps)
            ctx.sync()
            t1 = time.perf_counter()
            d1 = ctx.diagnostics()
            # kernel times per step, over three more steps
            ctx.enable_timing(True)
            ctx.reset_timings()
            ctx.step(3)
            ctx.sync()
            tim = ctx.timings()
        h = d1["iter_hist"] - d0["iter_hist"]
        return {"value": n * steps / (t1 - t0), "unit": "particle-steps/s",
                "mean_iterations": float(h @ np.arange(len(h)) / max(h.sum(), 1)),
                "h_error": herr_percentiles(d1["herr_hist"]),
                "not_converged": int(d1["noconv"] - d0["noconv"]),
                "implicit_ms_per_step": tim.get("implicit", (0.0, 0))[0] / 3,
                "guess_ms_per_step": tim.get("guess", (0.0, 0))[0] / 3}

    out["plain"] = run(G.GUESS_PLAIN)
    out["learned"] = run(G.GUESS_MLP, theta=net)
    out["speedup"] = out["learned"]["value"] / out["plain"]["value"]
    # What any guess of BF16 accuracy could gain here.  The Picard iteration
    # contracts its error by rho per iteration: rho from the mean counts at
    # two stopping tolerances (1e-13 and 1e-10, three decades apart).  A
    # guess correcting the Euler step to the 2^-9 relative accuracy of BF16
    # starts log10(512) / log10(1/rho) iterations and one evaluation (the
    # Euler base) ahead of z^n; it costs the base's evaluation plus the
    # network.  c_iter: implicit-pass time per particle-iteration of the
    # plain run; the network's cost is the guess kernel's time per particle
    # in those units (it includes the base's evaluation and the features).
    loose = run(G.GUESS_PLAIN, tol=1e-10)
    k13, k10 = out["plain"]["mean_iterations"], loose["mean_iterations"]
    rho = 10.0 ** (-3.0 / max(k13 - k10, 1e-9))
    floor_its = max(1.0, k13 - 1.0 - np.log10(512.0) / np.log10(1.0 / rho))
    c_iter = out["plain"]["implicit_ms_per_step"] / max(k13, 1e-9)
    net_cost = out["learned"]["guess_ms_per_step"] / c_iter if c_iter > 0 else None
    out["bound"] = {
        "rho": rho, "mean_iterations_tol_1e-10": k10,
        "iterations_floor_bf16_guess": floor_its,
        "speedup_max_free_network": k13 / (1.0 + floor_its),
        "network_cost_iterations": net_cost,
        "speedup_max_with_measured_network": (k13 / (net_cost + floor_its)
                                              if net_cost is not None else None)}
    return out


def timed_steps(ctx, steps, timing):
    """Run `steps` steps between two stream synchronisations; with timing, the
    library's HIP events time each kernel group on its stream.  Particle-steps
    count the particles alive at the start and at the end (mean)."""
    ctx.enable_timing(timing)
    ctx.reset_timings()
    ctx.sync()
    d0 = ctx.diagnostics()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.sync()
    t1 = time.perf_counter()
    d1 = ctx.diagnostics()
    tim = ctx.timings() if timing else {}
    ctx.enable_timing(False)
    alive = 0.5 * (d0["alive"] + d1["alive"])
    return {"steps": steps, "seconds": t1 - t0, "d0": d0, "d1": d1, "tim": tim,
            "alive": alive, "value": alive * steps / (t1 - t0),
            "ms_step": (t1 - t0) * 1e3 / max(steps, 1)}


def warm_and_time(ctx, args, graph, W):
    """Warmup steps, the autotuner's trials (real, untimed steps), then the
    timed steps; returns the timed run and the autotuner's choice."""
    ctx.use_graph(graph)
    ctx.step(args.warmup)
    ctx.sync()
    tune = None
    if not args.no_autotune:
        tune = ctx.autotune(3)
        print(f"[bench] autotune: {tune}", file=sys.stderr, flush=True)
    run = timed_steps(ctx, args.steps, timing=not graph)
    return run, tune


def flop_counts(W, run):
    """Algorithmic FP64 operations of the explicit and implicit pushes over a
    run, from the per-particle counts and the run's scheme and iteration
    statistics."""
    d0, d1 = run["d0"], run["d1"]
    steps, alive = run["steps"], run["alive"]
    impl = d1["implicit_steps"] - d0["implicit_steps"]
    iters = (d1["iter_hist"] - d0["iter_hist"]) @ np.arange(len(d1["iter_hist"]))
    evolve = W["mode"] == "evolve"
    grid = W["mode"] != "none"
    flop_rk4 = FLOP_RK4_GRID if grid else FLOP_RK4_NOGRID
    if not grid:
        flop_iter = FLOP_HAM_ITER  # neutral particles: discrete gradient
    elif W.get("solver") == "newton":
        flop_iter = FLOP_NEWTON_ITER
    else:
        flop_iter = FLOP_IMR_ITER
    return {
        "push": steps * alive * (flop_rk4 + FLOP_SWITCH) +
        (steps * alive - impl) * (FLOP_WEIGHTS if evolve else 0),
        "implicit": iters * flop_iter + impl * (FLOP_SWITCH + (FLOP_WEIGHTS if evolve else 0)),
        # the same work counted on the kernel's own shared-sample formulation
        "push_kernel_count": steps * alive * ((FLOP_KERNEL_RK4_GRID if grid else flop_rk4) +
                                              FLOP_SWITCH) +
        (steps * alive - impl) * (FLOP_KERNEL_WEIGHTS if evolve else 0),
    }, impl, iters


def roofline(W, run, workload):
    """Each kernel group's achieved rate against its bound, from the HIP-event
    timings of `run` (None without timings); the dominant group is the top
    level."""
    tim = run["tim"]
    if not tim:
        return None
    flops, _, _ = flop_counts(W, run)
    alive = run["alive"]
    paper = W.get("deposit") == "paper"
    bytes_dep = BYTES_DEPOSIT_PAPER if paper else BYTES_DEPOSIT
    # counter summaries are taken on the default configuration of a workload
    wl_key = workload + ("_paper" if paper else "") + \
        ("_clean" if W.get("clean_every") else "") + ("_inject" if W.get("inj_every") else "") + \
        ("_newton" if W.get("solver") == "newton" else "")
    nodes = (W["nr"] + 1) * (W["nth"] + 1)
    groups = {}
    for grp in ("push", "implicit", "deposit", "fields", "clean"):
        cnt_g = tim.get(grp, (0.0, 0))[1]
        if cnt_g == 0:
            continue
        avg_g = tim[grp][0] / cnt_g * 1e-3
        if grp in ("push", "implicit"):
            a_g = flops[grp] / cnt_g / avg_g / 1e12
            groups[grp] = {"bound": "alu", "achieved": a_g, "peak": PEAK_FP64_TFLOPS,
                           "unit": "TFLOP/s", "frac": a_g / PEAK_FP64_TFLOPS,
                           "flop_per_launch": flops[grp] / cnt_g,
                           "flop_count": "oracle, counting scalar type"}
            if grp == "push":
                groups[grp]["frac_kernel_count"] = \
                    flops["push_kernel_count"] / cnt_g / avg_g / 1e12 / PEAK_FP64_TFLOPS
        else:
            nb = {"deposit": bytes_dep * alive,
                  "fields": BYTES_FIELDS_PER_CELL * W["nr"] * W["nth"],
                  "clean": 2 * nodes * (BYTES_CLEAN_SWEEP * W.get("clean_iters", 500) +
                                        BYTES_CLEAN_FIXED)}[grp]
            a_g = nb / avg_g / 1e9
            groups[grp] = {"bound": "hbm", "achieved": a_g, "peak": PEAK_HBM_GBS,
                           "unit": "GB/s", "frac": a_g / PEAK_HBM_GBS,
                           "bytes_per_launch": nb}
        groups[grp]["avg_launch_ms"] = avg_g * 1e3
        groups[grp]["launches"] = cnt_g
        groups[grp]["traffic"] = counter_traffic(grp, wl_key, W["n"])
    ms = {g: tim[g][0] for g in groups if g != "clean"}
    dom = max(ms, key=ms.get)
    roof = {"kernel": dom, **groups[dom]}
    roof["algorithmic_bytes"] = (BYTES_PUSH * alive if dom == "push" else
                                 groups[dom].get("bytes_per_launch"))
    roof["groups"] = groups
    roof["kernel_ms_per_step"] = {k: v[0] / max(run["steps"], 1) for k, v in tim.items()
                                  if v[1] > 0}
    return roof


def plain_guess_run(G, W, args, pre_steps):
    """The same workload with the plain start of the implicit iteration (the
    hybrid's RK4 result, no network), run through the same number of steps
    before its timed region, for the learned-vs-plain comparison."""
    Wp = dict(W)
    Wp.pop("guess", None)
    ctx, _ = make_context(G, Wp, push_wps=args.push_wps,
                          persistent_waves=args.persistent_waves)
    try:
        if pre_steps:
            ctx.step(pre_steps)
        run, _ = warm_and_time(ctx, args, bool(args.graph or W.get("graph", 0)), Wp)
    finally:
        ctx.close()
    d0, d1 = run["d0"], run["d1"]
    impl = d1["implicit_steps"] - d0["implicit_steps"]
    iters = (d1["iter_hist"] - d0["iter_hist"]) @ np.arange(len(d1["iter_hist"]))
    return {"value": run["value"], "unit": "particle-steps/s", "ms_per_step": run["ms_step"],
            "implicit_fraction": impl / max(run["steps"] * run["alive"], 1),
            "mean_implicit_iterations": float(iters / max(impl, 1)),
            "h_error": herr_percentiles(d1["herr_hist"])}


def copy_calibration(nbytes):
    """One device-to-device copy of nbytes with the HIP runtime's own blit
    kernel: a kernel of known traffic for scaling the FETCH_SIZE / WRITE_SIZE
    counters."""
    import ctypes as C
    hip = C.CDLL("libamdhip64.so")
    a, b = C.c_void_p(), C.c_void_p()
    assert hip.hipMalloc(C.byref(a), C.c_size_t(nbytes)) == 0
    assert hip.hipMalloc(C.byref(b), C.c_size_t(nbytes)) == 0
    assert hip.hipMemset(a, 1, C.c_size_t(nbytes)) == 0
    for _ in range(3):
        assert hip.hipMemcpy(b, a, C.c_size_t(nbytes), 3) == 0  # device to device
    assert hip.hipDeviceSynchronize() == 0
    hip.hipFree(a)
    hip.hipFree(b)
    print(json.dumps({"copy_calibration_bytes": nbytes}))


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--particles", type=int, default=0, help="override particle count")
    ap.add_argument("--graph", type=int, default=0, help="replay the step as a hipGraph")
    ap.add_argument("--push-wps", type=int, default=0, help="explicit-push waves per SIMD")
    ap.add_argument("--sort-every", type=int, default=0,
                    help="steps between particle re-sorts (0: the workload's value)")
    ap.add_argument("--persistent-waves", type=int, default=0,
                    help="implicit-pass waves per CU (0: library default)")
    ap.add_argument("--deposit", choices=("conserving", "paper"), default="conserving",
                    help="deposit mode of the full-cycle workloads (paper: Sec. 2.3 current)")
    ap.add_argument("--clean-every", type=int, default=0,
                    help="divergence cleaning after every N-th step (Sec. 2.4; 0: never)")
    ap.add_argument("--clean-iters", type=int, default=500)
    ap.add_argument("--solver", choices=("picard", "newton"), default="picard",
                    help="implicit midpoint solver (Newton: Sec. 2.2.2)")
    ap.add_argument("--inject-every", type=int, default=0,
                    help="pair injection (Sec. 3.3: r+ <= r <= 6, multiplicity 3, density "
                         "5 n_GJ, Theta 0.5) after every N-th step (0: never)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probe", action="store_true",
                    help="skip the measured FP64-FMA and copy ceilings")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20)
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch settings (no autotuner trials)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-vs-plain guess comparison")
    ap.add_argument("--learned-steps", type=int, default=20)
    ap.add_argument("--learned-dt", type=float, nargs="+", default=[0.01, 0.03, 0.1],
                    help="time steps of the learned-vs-plain comparison on the charged "
                         "test-particle workload")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the plain-start run of a learned-guess workload")
    ap.add_argument("--roofline-steps", type=int, default=20,
                    help="eager steps timed per kernel group after graph-replayed steps")
    ap.add_argument("--table2-t", type=float, default=1000.0,
                    help="end time of the Table 2 scheme runs (workload c1; 0 skips them)")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="only run a device copy of this many bytes (counter scale)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (--gpus {args.gpus} requested); the path "
              "is built and measured on a single MI355X", file=sys.stderr)
        sys.exit(2)

    import paper_2602_07452_amd as G
    W = dict(WORKLOADS[args.workload])
    if args.particles:
        W["n"] = args.particles
    if args.sort_every:
        W["sort_every"] = args.sort_every
    if args.solver != "picard":
        W["solver"] = args.solver
        W["desc"] += f"; {args.solver} solver for the implicit midpoint rule"
    if args.inject_every:
        if W["mode"] != "evolve":
            print("--inject-every needs a full-cycle workload (c3, c5)", file=sys.stderr)
            sys.exit(2)
        W["inj_every"] = args.inject_every
        W["desc"] += (f"; pair injection every {args.inject_every} steps in r+ <= r <= 6 "
                      "(multiplicity 3, 5 n_GJ per pair, Theta 0.5)")
    if args.deposit != "conserving" or args.clean_every:
        if W["mode"] != "evolve":
            print("--deposit/--clean-every need a full-cycle workload (c3, c5)", file=sys.stderr)
            sys.exit(2)
        W["deposit"], W["clean_every"] = args.deposit, args.clean_every
        W["clean_iters"] = args.clean_iters
        W["desc"] += (f"; {args.deposit} deposit" +
                      (f", cleaning every {args.clean_every} steps ({args.clean_iters} "
                       "Jacobi sweeps)" if args.clean_every else ""))
    ctx, cfg = make_context(G, W, push_wps=args.push_wps,
                            persistent_waves=args.persistent_waves)
    print(f"[bench] workload {args.workload}: n={W['n']} dt={cfg.dt:.3e}", file=sys.stderr,
          flush=True)
    graph = bool(args.graph or W.get("graph", 0))
    mlp_info = None
    pre_steps = 0
    if W.get("guess") == "mlp":
        # learned guess: trained on the GPU on the converged implicit steps of
        # the first warmup steps (RK4 result corrected by the network)
        pre_steps = max(args.warmup // 2, 4)
        t0 = time.perf_counter()
        ctx.mlp_collect(1 << 24)
        ctx.step(pre_steps)
        ctx.mlp_collect(0)
        loss = ctx.mlp_train(epochs=8, batch=4096, lr=3e-3, lr_final=3e-5, seed=7)
        mlp_info = {"samples": ctx.mlp_num_samples(), "epochs": 8,
                    "loss_first_epoch": float(loss[0]), "loss_last_epoch": float(loss[-1]),
                    "collect_and_train_s": time.perf_counter() - t0}
    run, tune = warm_and_time(ctx, args, graph, W)
    value, ms_step = run["value"], run["ms_step"]
    print(f"[bench] {ms_step:.3f} ms/step, {value:.4e} particle-steps/s", file=sys.stderr,
          flush=True)
    # roofline: HIP-event timing of each kernel group on the library's stream.
    # Events cannot be placed between the kernels of a replayed graph, so with
    # graph replay the groups are timed over eager steps of the same kernels
    # that follow the timed region.
    if graph:
        ctx.use_graph(False)
        rl = timed_steps(ctx, max(1, min(args.steps, args.roofline_steps)), timing=True)
    else:
        rl = run
    roof = roofline(W, rl, args.workload)
    if roof is not None and graph:
        roof["timing"] = (f"HIP events over {rl['steps']} eager steps after the "
                          f"{args.steps} graph-replayed timed steps")

    peaks = None
    if not args.no_probe:
        # the achievable ceilings of this device, next to the published peaks
        peaks = ctx.probe_peaks()
        print(f"[bench] measured ceilings: FP64 FMA {peaks['fp64_fma_tflops']:.1f} TFLOP/s, "
              f"copy {peaks['copy_tbs']:.2f} TB/s", file=sys.stderr, flush=True)
        if roof is not None:
            for gd in [roof] + list(roof["groups"].values()):
                ceil = (peaks["fp64_fma_tflops"] if gd["bound"] == "alu"
                        else peaks["copy_tbs"] * 1e3)
                gd["frac_of_measured"] = gd["achieved"] / ceil
    ctx.close()
    d0, d1 = run["d0"], run["d1"]
    impl = d1["implicit_steps"] - d0["implicit_steps"]
    iters = (d1["iter_hist"] - d0["iter_hist"]) @ np.arange(len(d1["iter_hist"]))
    grid = W["mode"] != "none"
    plain = None
    if mlp_info is not None and not args.no_plain:
        # learned vs plain on the workload itself: the same run with the
        # iteration started from the RK4 result alone
        print("[bench] same workload, plain implicit start", file=sys.stderr, flush=True)
        plain = plain_guess_run(G, W, args, pre_steps)
        plain["learned_over_plain"] = value / plain["value"]
        print(f"[bench] plain start: {plain['ms_per_step']:.3f} ms/step "
              f"(learned/plain {plain['learned_over_plain']:.3f})", file=sys.stderr, flush=True)
    table2 = ratios = None
    if args.workload == "c1" and args.table2_t > 0:
        table2 = table2_runs(G, W, args.table2_t)
        ratios = pusher_cost_ratios(G, W)
    learned = None
    if not args.no_learned:
        print("[bench] learned vs plain implicit guess", file=sys.stderr, flush=True)
        learned = {f"dt={dt:g}": learned_vs_plain(G, args.learned_steps, dt=dt)
                   for dt in args.learned_dt}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample", file=sys.stderr, flush=True)
        cpu = cpu_baseline(W, cfg, args.cpu_sample, args.cpu_steps)

    out = {
        "metric": "particle-steps/s (gather+push+deposit) at fixed H error; learned vs plain guess",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64 particles / f32 fields" if grid else "f64",
        "data": "synthetic",
        "config": {"workload": W["desc"], "particles": W["n"], "grid": [W["nr"], W["nth"]],
                   "dt": cfg.dt,
                   "pusher": ("Hyb2 (RK4 -> IMR)" if grid
                              else "Hyb2 (RK4 -> Hamiltonian discrete gradient)"),
                   "threshold": cfg.hyb_threshold,
                   "guess": ("RK4 result + learned correction" if mlp_info else "RK4 result"),
                   "precision": ("FP64 particle state, metric, push and energy check; FP32 "
                                 "field storage, Maxwell arithmetic and J/rho outputs; int64 "
                                 "fixed-point deposit sums") if grid else "FP64",
                   "graph": graph, "sort_every": cfg.sort_every,
                   "tile": [cfg.tile_r, cfg.tile_th]},
        "implicit_fraction": impl / max(args.steps * run["alive"], 1),
        "mean_implicit_iterations": float(iters / max(impl, 1)),
        "h_error": herr_percentiles(d1["herr_hist"]),
        "deposit_fallback_blocks": int(d1["deposit_fallback"] - d0["deposit_fallback"]),
        "deposit_outside_box": int(d1["deposit_outside"] - d0["deposit_outside"]),
        "roofline": roof,
        "measured_peaks": peaks,
        "autotune": tune,
        "learned_guess_training": mlp_info,
        "plain_guess": plain,
        "learned_guess": learned,
        "table2_a0": table2,
        "pusher_cost_ratios": ratios,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
