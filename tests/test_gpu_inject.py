"""Pair injection (Sec. 3.3) on the GPU, through the C ABI, against the
oracle: into electrovacuum, after steps (cells that kept their plasma are
skipped), at a capacity limit, and on a schedule inside a running PIC loop
(Gauss's law kept by the co-located pairs, graph replay equal to eager
steps)."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import levels, oracle_grid, rplus

pytestmark = pytest.mark.gpu

SEED = 2602074520


def _cfg(cap=60000, every=0, a=0.9):
    cfg = G.config_default(a=a, nr=40, nth=32, r_in=0.9 * rplus(a), r_out=12.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-9, max_particles=cap, r_remove_in=rplus(a),
                           r_remove_out=12.0, reflect=1, r_abs=11.0, chi0=1e4,
                           lambda_abs=5.0, tile_r=16, tile_th=16, guess=G.GUESS_RK4,
                           inj_every=every, inj_r0=2.0, inj_r1=6.0, inj_mult=3.0,
                           inj_density=5.0, inj_theta=0.5, inj_seed=SEED + 70, sort_every=4)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _params(cfg):
    return O.InjectParams(cfg.inj_r0, cfg.inj_r1, cfg.inj_mult, cfg.inj_density,
                          cfg.inj_theta, cfg.inj_seed)


def _oracle_inject(cfg, g, ctx, event, room=None):
    """The oracle's injection from the GPU's state (B of the integer chain,
    particles in id order)."""
    S = levels(ctx)
    B = [g.densitize(3 + c, S[G.LEVEL_BN][c].astype(np.float64), -1) for c in range(2)]
    P = ctx.get_particles()
    p = O.Particles(len(P["r"]))
    for k in ("r", "th", "ph", "ur", "uth", "uph", "qm", "w", "H0"):
        getattr(p, k)[:] = P[k]
    p.flags[:] = P["flags"]
    room = cfg.max_particles - p.n if room is None else room
    return O.inject(g, _params(cfg), event, B, p, room), p.n


def _compare_new(P, q, n0):
    new = np.arange(n0, len(P["r"]))
    assert len(P["r"]) == q.n
    for k in ("r", "th", "ph"):
        assert np.allclose(P[k][new], getattr(q, k)[n0:], rtol=1e-14, atol=0), k
    for k in ("ur", "uth", "uph"):
        assert np.allclose(P[k][new], getattr(q, k)[n0:], rtol=1e-12, atol=1e-13), k
    assert np.array_equal(P["qm"][new], q.qm[n0:])
    assert np.allclose(P["w"][new], q.w[n0:], rtol=1e-12, atol=0)
    assert np.allclose(P["H0"][new], q.H0[n0:], rtol=1e-13, atol=0)
    assert np.all(P["flags"][new] == G.FLAG_ALIVE)


def test_injection_into_vacuum_matches_oracle():
    cfg = _cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=0.0)
        q, n0 = _oracle_inject(cfg, g, ctx, 0)
        added = ctx.inject()
        P = ctx.get_particles()
        rho = ctx.get_field(G.LEVEL_J, 3)
    assert n0 == 0 and added == q.n > 1000
    _compare_new(P, q, 0)
    assert np.abs(rho).max() == 0.0  # nothing deposited by the injection itself


def test_injection_after_steps_matches_oracle():
    """Inject, move the plasma for a few steps, inject again: only cells
    whose density fell below the multiplicity get a new pair."""
    cfg = _cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=0.0)
        first = ctx.inject()
        ctx.step(6)
        q, n0 = _oracle_inject(cfg, g, ctx, 6)
        added = ctx.inject()
        P = ctx.get_particles()
    assert n0 == first and 0 < added < first
    _compare_new(P, q, n0)


def test_injection_at_the_capacity_limit():
    cfg = _cfg(cap=101)
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=0.0)
        q, _ = _oracle_inject(cfg, g, ctx, 0)
        assert ctx.inject() == 100
        P = ctx.get_particles()
        assert ctx.inject() == 0  # full
    _compare_new(P, q, 0)


def test_scheduled_injection_keeps_gauss_and_graph_replay():
    """Injection every 5 steps inside the PIC loop: the co-located pairs
    leave rho and so Gauss's law untouched (conserving deposit), and the
    run replayed as graphs equals the eager run bit for bit.  The Gauss
    residual is formed from the FP32 D and rho arrays, whose rounding alone
    moves it (the same 20 steps without any particle): the plasma may move
    it by no more than twice that floor, far below the residual one
    uncompensated injected charge would leave."""
    runs = {}
    for graph, every in ((False, 5), (True, 5), (False, 0)):
        cfg = _cfg(every=every)
        g = oracle_grid(cfg)
        with G.Context(cfg) as ctx:
            ctx.set_fields_wald(1.0, a_field=0.0)
            ctx.use_graph(graph)
            S0 = levels(ctx)
            ctx.step(20)
            S1 = levels(ctx)
            runs[graph, every] = (ctx.get_particles(), S0, S1, ctx.num_particles())
    (P0, S0, S_e, n_e), (P1, _, S_g, n_g) = runs[False, 5], runs[True, 5]
    _, V0, V1, n_v = runs[False, 0]
    assert n_e == n_g > 0 and n_v == 0
    for k in P0:
        assert np.array_equal(P0[k], P1[k]), k
    for lev in S_e:
        for c in range(len(S_e[lev])):
            assert np.array_equal(S_e[lev][c], S_g[lev][c])
    inner = (g.rn > 2.0) & (g.rn < cfg.r_abs - 1.0)

    def residual(S):
        D = [g.densitize(c, S[G.LEVEL_DN][c].astype(np.float64), -1) for c in range(3)]
        return O.gauss_residual(g, D, S[G.LEVEL_J][3].astype(np.float64))[:, inner]

    drift = np.abs(residual(S_e) - residual(S0)).max()
    floor = np.abs(residual(V1) - residual(V0)).max()
    assert 0.0 < floor < 1e-3 * max(np.abs(residual(S0)).max(), 1e-6)
    assert drift <= 2.0 * floor + 1e-7, (drift, floor)
