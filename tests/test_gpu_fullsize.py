"""Parity at the full benchmark sizes, in the launch configuration bench.py
times: a seeded sample of particles is pushed one by one by the oracle (with
the GPU's own FP32 fields) and compared with the GPU step; the deposit and the
field update are checked through properties that hold at any size (discrete
charge continuity, div B unchanged by the step)."""
import numpy as np
import pytest

import bench
import oracle as O
import paper_2602_07452_amd as G
from gpu_common import TOL_STATE, compare_push, oracle_grid, push_params_from, rplus

pytestmark = pytest.mark.gpu

NSAMPLE = 512


def _fields6(ctx):
    return ([ctx.get_field(G.LEVEL_DH1, c).astype(np.float64) for c in range(3)],
            [ctx.get_field(G.LEVEL_BH, c).astype(np.float64) for c in range(3)])


def _check_full_size(workload, learned):
    W = dict(bench.WORKLOADS[workload])
    if not learned:
        W.pop("guess", None)
    ctx, cfg = bench.make_context(G, W)
    try:
        ctx.use_graph(bool(W.get("graph", 0)))
        if W.get("guess") == "mlp":
            ctx.mlp_collect(1 << 20)
            ctx.step(2)
            ctx.mlp_collect(0)
            ctx.mlp_train(epochs=2, batch=4096, seed=3)
        ctx.step(2)  # not a multiple of the sort interval: ids keep their slots
        n = ctx.num_particles()
        rng = np.random.default_rng(2602074520 + 17)
        ids = np.sort(rng.choice(n, NSAMPLE, replace=False))
        before = ctx.sample_particles(ids)
        Dh, _ = _fields6(ctx)
        rho0 = ctx.get_field(G.LEVEL_J, 3).astype(np.float64)
        g0, b0, _ = ctx.field_diagnostics()
        ctx.step(1)
        after = ctx.sample_particles(ids)
        _, Bh = _fields6(ctx)
        J = [ctx.get_field(G.LEVEL_J, c).astype(np.float64) for c in range(4)]
        g1, b1, _ = ctx.field_diagnostics()
    finally:
        ctx.close()
    g = oracle_grid(cfg)
    # particles: the oracle pushes the sample with the GPU's D^{n+3/2} (input
    # level) and B^{n+3/2} (rebuilt by the step)
    err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_GRID),
                          grid=g, G6=Dh + Bh)
    assert err <= TOL_STATE
    alive = (before["flags"] & G.FLAG_ALIVE) != 0
    assert alive.sum() > 0.9 * NSAMPLE
    # deposit: discrete continuity of the FP32 rho and J at interior nodes
    Lr = np.diff(g.rh)
    res = (J[3] - rho0)[1:-1, 1:-1] / cfg.dt
    res += (J[0][1:-1, 1:] - J[0][1:-1, :-1]) / Lr[None, :]
    res += (J[1][1:, 1:-1] - J[1][:-1, 1:-1]) / (g.tn[1] - g.tn[0])
    mask = g.rn[1:-1] > rplus(cfg.a) + 6 * (g.rn[1] - g.rn[0])
    scale = np.abs(J[3]).max() / cfg.dt
    assert np.abs(res[:, mask]).max() < 1e-5 * scale
    # fields: the update keeps div B (densitized, eq. m2) at its level; FP32
    # storage adds round-off of the order of the field over the cell size
    bscale = max(np.abs(b).max() for b in Bh) / min(np.diff(g.rn).min(), g.tn[1] - g.tn[0])
    assert b1 <= 2.0 * b0 + 1e-6 * bscale


def test_full_size_plasma_wald():
    """2^24 particles on 1024^2 (the bench workload)."""
    _check_full_size("c3", learned=False)


def test_full_size_split_monopole_learned_graph():
    """2^27 particles on 2048^2 with the learned guess and graph replay."""
    _check_full_size("c5", learned=True)


def test_full_size_charged_test_particles():
    """2^20 charged test particles in the static Wald grid field (Hyb2 with the
    RK4 result as first iterate), sampled."""
    W = dict(bench.WORKLOADS["c2"])
    ctx, cfg = bench.make_context(G, W)
    try:
        G6 = [ctx.get_field(G.LEVEL_DH1, c).astype(np.float64) for c in range(3)] + \
             [ctx.get_field(G.LEVEL_BH, c).astype(np.float64) for c in range(3)]
        ctx.step(3)
        rng = np.random.default_rng(2602074520 + 18)
        ids = np.sort(rng.choice(ctx.num_particles(), NSAMPLE, replace=False))
        before = ctx.sample_particles(ids)
        ctx.step(1)
        after = ctx.sample_particles(ids)
    finally:
        ctx.close()
    err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_GRID),
                          grid=oracle_grid(cfg), G6=G6)
    assert err <= TOL_STATE


def test_full_size_neutral_test_particles():
    """All 1024 neutral particles of the Schwarzschild test-particle workload,
    one Hyb2 step (RK4 -> discrete gradient) after 20."""
    W = dict(bench.WORKLOADS["c1"])
    ctx, cfg = bench.make_context(G, W)
    try:
        ctx.step(20)
        before = ctx.get_particles()
        ctx.step(1)
        after = ctx.get_particles()
    finally:
        ctx.close()
    err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_NONE))
    assert err <= TOL_STATE
