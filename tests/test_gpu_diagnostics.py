"""Grid diagnostics (Gauss residual, div B, the Poynting luminosity P_BZ of
eq. Pbz) on the GPU against the oracle, for one state and as a time series
over a multi-step run (the parity protocol for multi-step runs compares
statistics such as P_BZ(r) rather than particle trajectories)."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import levels, oracle_fields, oracle_grid, oracle_particles, push_params_from, rplus

pytestmark = pytest.mark.gpu

SEED = 2602074520


def _cfg(n=2048, a=0.9):
    cfg = G.config_default(a=a, nr=48, nth=40, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-13, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=20.0, reflect=1, r_abs=18.0, chi0=1e4,
                           lambda_abs=5.0, tile_r=16, tile_th=16, guess=G.GUESS_RK4)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _plain(g, S, lev, off):
    return [g.densitize(off + c, S[lev][c].astype(np.float64), -1) for c in range(3)]


def test_field_diagnostics_match_oracle():
    cfg = _cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 80, rplus(cfg.a), 16.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        ctx.step(5)
        gmax, bmax, pbz = ctx.field_diagnostics()
        S = levels(ctx)
    D, B = _plain(g, S, G.LEVEL_DN, 0), _plain(g, S, G.LEVEL_BN, 3)
    rho = S[G.LEVEL_J][3].astype(np.float64)
    go = np.abs(O.gauss_residual(g, D, rho)).max()
    bo = np.abs(O.div_B(g, B)).max()
    po = O.poynting(g, D, B)
    assert abs(gmax - go) <= 1e-5 * go
    # the sampled Wald field carries a truncation-level div B (constant in
    # time on the Yee grid)
    assert abs(bmax - bo) <= 1e-5 * bo
    assert np.abs(pbz - po).max() <= 1e-5 * np.abs(po).max()
    assert np.abs(po).max() > 0


def test_pbz_time_series_matches_oracle():
    """Split monopole with a pair plasma, 30 steps: the GPU (FP32 fields)
    and the oracle (FP64 fields from the same initial arrays, its own
    particles) give the same P_BZ(r) at every step."""
    cfg = _cfg()
    g = oracle_grid(cfg)
    steps = 30
    series_gpu = []
    with G.Context(cfg) as ctx:
        ctx.set_fields_split_monopole(1.0, 1e3)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 81, rplus(cfg.a), 16.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.05, w=1e-3)
        S0 = levels(ctx)
        P0 = ctx.get_particles()
        for _ in range(steps):
            ctx.step(1)
            series_gpu.append(ctx.field_diagnostics()[2])
    F = oracle_fields(g, S0)
    p = oracle_particles(P0)
    P = push_params_from(cfg, O.FIELDS_GRID)
    series_orc = []
    for _ in range(steps):
        O.pic_step(P, g, F, p, absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
        series_orc.append(O.poynting(g, F.Dn, F.Bn))
    sg, so = np.array(series_gpu), np.array(series_orc)
    scale = np.abs(so).max()
    assert scale > 0
    err = np.abs(sg - so).max(axis=1) / scale
    print(f"P_BZ(r) time series: max relative difference {err.max():.2e} over {steps} steps")
    assert err.max() < 1e-4


def _herr_bins(v):
    """Host bins of energy violations, floor(2 (log10 v + 30)) clamped to
    [0, 63]; 0 for v < 1e-30 or NaN."""
    v = np.asarray(v, np.float64)
    ok = v >= 1e-30
    b = np.zeros(v.shape, np.int64)
    b[ok] = np.floor(2.0 * (np.log10(np.minimum(v[ok], 1e30)) + 30.0)).astype(np.int64)
    return np.clip(b, 0, G.HIST_BINS - 1)


def test_particle_census_matches_the_particle_arrays():
    """The alive count and the energy-violation histogram of the diagnostics
    are those of the particle arrays after the last step (a hot plasma up to
    the outer edge, so that particles are removed and some steps are taken
    implicitly).  The device bins with an FP32 logarithm: a value within
    1e-6 of a bin edge may land on either side."""
    cfg = _cfg(n=4096)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 81, rplus(cfg.a), 19.9,
                           cfg.theta0, np.pi - cfg.theta0, 1.0, w=2e-3)
        d = ctx.diagnostics()
        assert d["alive"] == cfg.max_particles and d["herr_hist"][0] == cfg.max_particles
        for _ in range(3):
            ctx.step(4)
            d = ctx.diagnostics()
            P = ctx.get_particles()
            alive = (P["flags"] & G.FLAG_ALIVE) != 0
            assert d["alive"] == int(alive.sum())
            v = P["herr"][alive]
            lo, hi = _herr_bins(v * (1.0 - 1e-6)), _herr_bins(v * (1.0 + 1e-6))
            sure = np.bincount(lo[lo == hi], minlength=G.HIST_BINS)
            h = d["herr_hist"]
            assert h.sum() == alive.sum()
            assert np.all(h >= sure) and (h - sure).sum() == int((lo != hi).sum())
        assert d["removed"] > 0 and d["implicit_steps"] > 0
        assert alive.sum() < cfg.max_particles
