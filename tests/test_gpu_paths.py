"""Paths that production runs take rarely and the other parity tests do not
reach, against the oracle: the implicit iteration stopped at its cap
(non-convergence, Sec. 2.2.2), the restart from z^n when the iteration from
the learned guess does not converge, and the deposit's overflow paths
(Sec. 2.3): the second pass over short segments, the global-atomic
fallback and the particles outside their planned box in the conserving
deposit, and the global fallback of the paper's current."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import (TOL_STATE, compare_push, gpu_fields_as_G, levels, norm_err,
                        oracle_grid, oracle_particles, push_params_from, rplus, state_err)

pytestmark = pytest.mark.gpu

SEED = 2602074520
TOL_DEP = 1e-6


# ------------------------------------------------------- non-convergence
def _wald_cfg(pusher, kmax, guess, n=4096, thr=1e-13):
    a = 0.9
    return G.config_default(a=a, nr=48, nth=40, r_in=0.9 * rplus(a), r_out=50.0, dt=0.01,
                            field_mode=G.FIELDS_STATIC, pusher=pusher, hyb_threshold=thr,
                            kmax=kmax, guess=guess, max_particles=n, r_remove_in=rplus(a),
                            r_remove_out=50.0, reflect=1, tile_r=16, tile_th=16)


def _wald_step(cfg, seed, net=None):
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, cfg.max_particles, seed, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, 1.0)
        if net is not None:
            ctx.mlp_set(*net)
        G6 = gpu_fields_as_G(ctx)
        before = ctx.get_particles()
        d0 = ctx.diagnostics()
        ctx.step(1)
        after = ctx.get_particles()
        d1 = ctx.diagnostics()
    return G6, before, after, d1["noconv"] - d0["noconv"]


def _oracle_step(cfg, before, G6, **kw):
    P = push_params_from(cfg, O.FIELDS_GRID)
    for k, v in kw.items():
        setattr(P, k, v)
    p = oracle_particles(before)
    O.push(P, p, grid=oracle_grid(cfg), G=G6)
    return p


@pytest.mark.parametrize("kmax", [1, 5])
def test_implicit_cap_flags_match_oracle(kmax):
    """IMR from z^n stopped after kmax iterations: the GPU returns the last
    iterate, the not-converged flag and the count as the oracle does, and
    counts the stops."""
    cfg = _wald_cfg(G.PUSH_IMR, kmax, G.GUESS_PLAIN)
    G6, before, after, noconv = _wald_step(cfg, SEED + 100 + kmax)
    p = _oracle_step(cfg, before, G6)
    alive = (before["flags"] & G.FLAG_ALIVE) != 0
    assert (state_err(after["z"][alive], p.state()[alive]) <= TOL_STATE).all()
    gnc = (after["flags"] & G.FLAG_NOCONV) != 0
    onc = (p.flags & O.NOCONV) != 0
    assert np.array_equal(gnc[alive], onc[alive])
    assert np.array_equal(after["iters"][alive], p.iters[alive])
    assert noconv == int(gnc[alive].sum())
    if kmax == 1:
        assert gnc[alive].all()  # one iteration from z^n never meets 1e-13
    else:
        assert 0 < gnc[alive].sum() < alive.sum()


def test_hybrid_cap_flags_match_oracle():
    """Hyb2 with the RK4 result as first iterate and a cap of two: a mix of
    converged and stopped implicit redos, equal to the oracle's."""
    cfg = _wald_cfg(G.PUSH_HYB2, 2, G.GUESS_RK4, thr=1e-15)
    G6, before, after, noconv = _wald_step(cfg, SEED + 104)
    err, p = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_GRID),
                          grid=oracle_grid(cfg), G6=G6)
    alive = (before["flags"] & G.FLAG_ALIVE) != 0
    same = ((after["flags"] & G.FLAG_IMPLICIT) != 0) == ((p.flags & O.IMPLICIT) != 0)
    sel = alive & same
    gnc = (after["flags"] & G.FLAG_NOCONV) != 0
    assert np.array_equal(gnc[sel], ((p.flags & O.NOCONV) != 0)[sel])
    assert np.array_equal(after["iters"][sel], p.iters[sel])
    assert gnc[sel].sum() > 0 and noconv == int(gnc[alive].sum())


def _bad_net(seed=5):
    """A network whose guess is far from the step (outputs of order one in
    every component of the state): the iteration from it cannot meet the
    tolerance within a small cap."""
    rng = np.random.default_rng(seed)
    theta = rng.normal(0.0, 0.5, G.MLP_NPARAM).astype(np.float32)
    return theta, np.zeros(14, np.float32), np.ones(14, np.float32), np.ones(6, np.float32)


@pytest.mark.parametrize("kmax", [1, 2])
def test_learned_guess_restart_matches_plain_oracle(kmax):
    """IMR from a far-off learned guess with a cap of kmax: the iteration from
    the guess stops unconverged, the particle restarts from z^n, and its
    result, flags and count (kmax + the restart's iterations) are the
    oracle's plain iteration from z^n."""
    cfg = _wald_cfg(G.PUSH_IMR, kmax, G.GUESS_MLP)
    G6, before, after, noconv = _wald_step(cfg, SEED + 110 + kmax, net=_bad_net())
    p = _oracle_step(cfg, before, G6)
    alive = (before["flags"] & G.FLAG_ALIVE) != 0
    assert (state_err(after["z"][alive], p.state()[alive]) <= TOL_STATE).all()
    gnc = (after["flags"] & G.FLAG_NOCONV) != 0
    assert np.array_equal(gnc[alive], ((p.flags & O.NOCONV) != 0)[alive])
    assert np.array_equal(after["iters"][alive], p.iters[alive] + kmax)
    assert noconv == int(gnc[alive].sum())


# ------------------------------------------------------ deposit overflow
def _pic_cfg(n, nr, nth, tile_r, tile_th, mode=G.DEPOSIT_CONSERVING, **kw):
    a = 0.99
    cfg = G.config_default(a=a, nr=nr, nth=nth, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-9, max_particles=n,
                           r_remove_in=rplus(a), r_remove_out=20.0, reflect=1,
                           r_abs=18.0, chi0=1e4, lambda_abs=5.0, tile_r=tile_r,
                           tile_th=tile_th, deposit_mode=mode, guess=G.GUESS_RK4, **kw)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _deposit_matches(cfg, P0, P1, S1):
    g = oracle_grid(cfg)
    alive = ((P0["flags"] & 1) != 0) & ((P1["flags"] & 1) != 0)
    old = np.stack([P0["r"], P0["th"], P0["ph"]], axis=1)
    new = np.stack([P1["r"], P1["th"], P1["ph"]], axis=1)
    rho, Jr, Jt, Jp = O.deposit(g, cfg.dt, old, new, P0["qm"] * P0["w"],
                                alive.astype(np.int32))
    errs = {name: norm_err(S1[G.LEVEL_J][c], want)
            for name, c, want in (("Jr", 0, Jr), ("Jt", 1, Jt), ("Jp", 2, Jp), ("rho", 3, rho))}
    assert max(errs.values()) < TOL_DEP, errs
    assert np.abs(Jr).max() > 0 and np.abs(Jt).max() > 0


def test_deposit_global_fallback_matches_oracle():
    """One sort tile covering the whole 64 x 64 grid: every chunk and every
    2048-particle segment of randomly placed particles spans the grid's
    65 x 65 nodes, more than the 2048 LDS bins, so the deposit goes through
    its second pass and then its global atomics."""
    cfg = _pic_cfg(20000, 64, 64, 64, 64)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 120, rplus(cfg.a),
                           18.0, cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        ctx.step(1)
        P0 = ctx.get_particles()
        d0 = ctx.diagnostics()
        ctx.step(1)
        d1 = ctx.diagnostics()
        P1, S1 = ctx.get_particles(), levels(ctx)
    assert d1["deposit_fallback"] - d0["deposit_fallback"] > 0
    _deposit_matches(cfg, P0, P1, S1)


def test_deposit_second_pass_of_injected_particles_matches_oracle():
    """Injected pairs are appended in cell-index order (theta row, then
    radius) after the sorted particles and take equal chunks of 8192: such a
    chunk spans all 64 rows of the grid (a box of far more than 2048 nodes),
    so it is redone in segments of 2048 particles, 16 rows each, which fit
    the LDS bins: no block falls back to global atomics."""
    cfg = _pic_cfg(12000, 64, 64, 16, 16, inj_r0=1.0, inj_r1=25.0, inj_mult=3.0,
                   inj_density=5.0, inj_theta=0.5, inj_seed=SEED + 7)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=0.0)
        ctx.init_particles(G.INIT_SHELL_MJ, 2048, SEED + 121, rplus(cfg.a), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=1e-6)
        ctx.step(1)
        n0 = ctx.num_particles()
        added = ctx.inject()
        P0 = ctx.get_particles()
        d0 = ctx.diagnostics()
        ctx.step(1)
        d1 = ctx.diagnostics()
        P1, S1 = ctx.get_particles(), levels(ctx)
    assert added >= 8192
    # the first chunk of appended particles spans more than the LDS bins
    g = oracle_grid(cfg)
    first = slice(n0, n0 + 8192)
    rows = np.searchsorted(g.tn, P0["th"][first])
    cols = np.searchsorted(g.rn, P0["r"][first])
    assert (np.ptp(rows) + 2) * (np.ptp(cols) + 2) > 2048
    assert d1["deposit_fallback"] == d0["deposit_fallback"]
    _deposit_matches(cfg, P0, P1, S1)


def test_deposit_outside_the_planned_box_matches_oracle():
    """The sort plans a node box for each deposit chunk (its tiles widened
    by a margin); a particle that has left that box since the sort is
    deposited through global atomics.  No re-sort for 200 steps of hot
    plasma on a 128 x 128 grid of 16 x 16 tiles lets particles near the
    horizon, where the cells are small, drift out of their boxes: the GPU
    counts them, and the deposit of the next step is the oracle's."""
    cfg = _pic_cfg(20000, 128, 128, 16, 16, sort_every=0)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 123, rplus(cfg.a),
                           18.0, cfg.theta0, np.pi - cfg.theta0, 1.0, w=2e-3)
        ctx.step(200)
        P0 = ctx.get_particles()
        d0 = ctx.diagnostics()
        ctx.step(1)
        d1 = ctx.diagnostics()
        P1, S1 = ctx.get_particles(), levels(ctx)
    outside = d1["deposit_outside"] - d0["deposit_outside"]
    print(f"particles outside their planned box in the last step: {outside}")
    assert outside > 0
    assert d1["deposit_fallback"] == d0["deposit_fallback"]
    _deposit_matches(cfg, P0, P1, S1)


def test_paper_current_global_fallback_matches_oracle():
    """The paper's current (deposit mode PAPER) with one sort tile over the
    whole grid: its equal chunks of randomly placed particles miss the LDS
    bins and use global atomics."""
    cfg = _pic_cfg(20000, 64, 64, 64, 64, mode=G.DEPOSIT_PAPER)
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=0.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 122, rplus(cfg.a),
                           18.0, cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        d0 = ctx.diagnostics()
        ctx.step(2)
        d1 = ctx.diagnostics()
        P, S = ctx.get_particles(), levels(ctx)
    assert d1["deposit_fallback"] - d0["deposit_fallback"] > 0
    alive = ((P["flags"] & G.FLAG_ALIVE) != 0).astype(np.int32)
    rho, Jr, Jt, Jp = O.deposit_paper(g, P["z"], P["qm"] * P["w"], alive)
    errs = {name: norm_err(S[G.LEVEL_J][c], want)
            for name, c, want in (("Jr", 0, Jr), ("Jt", 1, Jt), ("Jp", 2, Jp), ("rho", 3, rho))}
    assert max(errs.values()) < TOL_DEP, errs
