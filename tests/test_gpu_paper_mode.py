"""The paper's own current (Sec. 2.3) and divergence cleaning (Sec. 2.4) on
the GPU, through the C ABI, against the oracle: the deposit at the loaded
and at the pushed state, a full paper-mode step, the Jacobi cleaning of
both D chains, and the scheduled cleaning holding Gauss's law."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import (TOL_STATE, compare_push, field_errors, levels, norm_err, oracle_fields,
                        oracle_grid, oracle_particles, push_params_from, rplus)

pytestmark = pytest.mark.gpu

SEED = 2602074520
TOL_DEP = 1e-6  # FP32 output of FP64 sums (as for the conserving deposit)


def _cfg(n=3000, clean_every=0, mode=G.DEPOSIT_PAPER, a=0.99):
    cfg = G.config_default(a=a, nr=40, nth=32, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-9, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=20.0, reflect=1, r_abs=18.0, chi0=1e4,
                           lambda_abs=5.0, tile_r=16, tile_th=16, deposit_mode=mode,
                           clean_every=clean_every, clean_iters=500, guess=G.GUESS_RK4)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _init(ctx, cfg, seed=SEED + 60):
    ctx.set_fields_wald(1.0, a_field=0.0)
    ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, seed, rplus(cfg.a), 18.0,
                       cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)


def _deposit_errors(g, P, S):
    alive = ((P["flags"] & G.FLAG_ALIVE) != 0).astype(np.int32)
    rho, Jr, Jt, Jp = O.deposit_paper(g, P["z"], P["qm"] * P["w"], alive)
    return {name: norm_err(S[G.LEVEL_J][c], want)
            for name, c, want in (("Jr", 0, Jr), ("Jt", 1, Jt), ("Jp", 2, Jp), ("rho", 3, rho))}


def test_paper_current_matches_oracle():
    """At the loaded state (the J^{n+1} of the first step) and after two
    steps (J^{n+2} at the pushed state)."""
    cfg = _cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        _init(ctx, cfg)
        P0, S0 = ctx.get_particles(), levels(ctx)
        ctx.step(2)
        P2, S2 = ctx.get_particles(), levels(ctx)
    for P, S in ((P0, S0), (P2, S2)):
        errs = _deposit_errors(g, P, S)
        assert max(errs.values()) < TOL_DEP, errs
    assert np.abs(S2[G.LEVEL_J][0]).max() > 0 and np.abs(S2[G.LEVEL_J][1]).max() > 0


def test_paper_mode_full_step_matches_oracle():
    cfg = _cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        _init(ctx, cfg)
        ctx.step(2)
        S0, P0 = levels(ctx), ctx.get_particles()
        ctx.step(1)
        S1, P1 = levels(ctx), ctx.get_particles()
    F = oracle_fields(g, S0)
    P = push_params_from(cfg, O.FIELDS_GRID)
    P.deposit_mode = O.DEPOSIT_PAPER
    O.pic_step(P, g, F, oracle_particles(P0), absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    assert not field_errors(g, F, S1)
    G6 = [S0[G.LEVEL_DH1][c].astype(np.float64) for c in range(3)] + \
         [S1[G.LEVEL_BH][c].astype(np.float64) for c in range(3)]
    err, _ = compare_push(cfg, P0, P1, P, grid=g, G6=G6)
    assert err <= TOL_STATE
    errs = _deposit_errors(g, P1, S1)
    assert max(errs.values()) < TOL_DEP, errs


@pytest.mark.parametrize("iters", [1, 37, 500])
def test_cleaning_matches_oracle(iters):
    """Both chains: the integer chain against rho, the half chain against
    1.5 rho - 0.5 rho_prev; everything else untouched."""
    cfg = _cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        _init(ctx, cfg)
        ctx.step(3)
        S0 = levels(ctx)
        g0, _, _ = ctx.field_diagnostics()
        ctx.clean(iters)
        S1 = levels(ctx)
        g1, _, _ = ctx.field_diagnostics()
    rho = S0[G.LEVEL_J][3].astype(np.float64)
    rho_prev = S0[G.LEVEL_JPREV][3].astype(np.float64)
    for lev, rr in ((G.LEVEL_DN, rho), (G.LEVEL_DH1, 1.5 * rho - 0.5 * rho_prev)):
        D = [g.densitize(c, S0[lev][c].astype(np.float64), -1) for c in range(3)]
        Dc, _ = O.div_clean(g, D, rr, iters)
        for c in range(3):
            want = g.densitize(c, Dc[c])
            assert norm_err(S1[lev][c], want) < 1e-6, (lev, c)
            # the correction itself, against its own size
            d_gpu = S1[lev][c].astype(np.float64) - S0[lev][c]
            d_orc = want - g.densitize(c, D[c])
            scale = max(np.abs(d_orc).max(), 1e-7 * np.abs(want).max())
            assert np.abs(d_gpu - d_orc).max() <= 1e-2 * scale + 2e-7 * np.abs(want).max()
    for lev in (G.LEVEL_DH0, G.LEVEL_BM, G.LEVEL_BN, G.LEVEL_BH, G.LEVEL_J, G.LEVEL_JPREV):
        for c in range(len(S0[lev])):
            assert np.array_equal(S0[lev][c], S1[lev][c])
    if iters == 500:
        assert g1 < 0.2 * g0


def test_scheduled_cleaning_holds_gauss():
    """Sec. 2.4's schedule (every 25 steps, 500 sweeps; here every 5 steps on
    a small grid): over 20 steps the conserving deposit keeps the Gauss
    residual of the integer chain inside the absorbing layer's radius (up to
    FP32 round-off), the paper's
    current lets it drift, and the cleaned paper-mode run ends with a
    residual well below the uncleaned one.  Particles start away from the
    horizon, so none is removed (a removal takes charge away without a
    current)."""
    out = {}
    for name, mode, every in (("conserving", G.DEPOSIT_CONSERVING, 0),
                              ("paper", G.DEPOSIT_PAPER, 0),
                              ("paper+clean", G.DEPOSIT_PAPER, 5)):
        cfg = _cfg(mode=mode, clean_every=every)
        g = oracle_grid(cfg)
        with G.Context(cfg) as ctx:
            ctx.set_fields_wald(1.0, a_field=0.0)
            ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 61, 3.0, 14.0,
                               cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
            S0 = levels(ctx)
            ctx.step(20)
            S1 = levels(ctx)
            assert ctx.diagnostics()["removed"] == 0
        # nodes outside the absorbing layer (its damping of D does not keep
        # Gauss's law in either mode)
        inner = (g.rn > 2.0) & (g.rn < cfg.r_abs - 2.0)
        res = [O.gauss_residual(g, [g.densitize(c, S[G.LEVEL_DN][c].astype(np.float64), -1)
                                    for c in range(3)], S[G.LEVEL_J][3].astype(np.float64))
               [:, inner] for S in (S0, S1)]
        out[name] = (np.abs(res[1] - res[0]).max(), np.abs(res[1]).max())
    print({k: f"drift {v[0]:.3e}, residual {v[1]:.3e}" for k, v in out.items()})
    assert out["paper"][0] > 30 * out["conserving"][0]
    assert out["paper+clean"][1] < 0.2 * out["paper"][1]


def test_cleaning_needs_evolving_fields():
    cfg = G.config_default(a=0.9, nr=16, nth=16, r_in=1.3, r_out=10.0,
                           field_mode=G.FIELDS_STATIC, max_particles=16)
    with G.Context(cfg) as ctx:
        with pytest.raises(G.GrpicError):
            ctx.clean(10)
