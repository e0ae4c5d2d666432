"""Edge and degenerate cases of the GPU path against the oracle: particles
exactly on grid nodes, half points and the theta edges; an empty particle
set; neutral and charged particles together in grid fields (the
discrete-gradient implicit pass with a grid); the non-rotating hole a = 0."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import (TOL_STATE, compare_push, gpu_fields_as_G, norm_err, oracle_grid,
                        oracle_particles, push_params_from, rplus)
from gpu_common import field_errors as _field_errors
from gpu_common import levels as _levels
from gpu_common import oracle_fields as _oracle_fields

pytestmark = pytest.mark.gpu

SEED = 2602074520


def _pic_cfg(a=0.99, n=2048, nr=40, nth=32):
    cfg = G.config_default(a=a, nr=nr, nth=nth, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-9, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=20.0, reflect=1, r_abs=18.0, chi0=1e4,
                           lambda_abs=5.0, tile_r=16, tile_th=16)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _grid_point_particles(ctx, cfg):
    """e+/e- pairs placed exactly on nodes, half points, the theta edges and
    one ulp below nodes, with small random momenta."""
    rn, rh, tn, th = ctx.grid_coords()
    rng = np.random.default_rng(SEED + 30)
    inside = lambda r: r > rplus(cfg.a) * 1.05 and r < 17.0
    pts = []
    for i in range(2, cfg.nr - 2, 3):
        for j in range(0, cfg.nth + 1, 4):
            for r, t in ((rn[i], tn[j]), (rh[i], tn[j]), (rn[i], th[min(j, cfg.nth - 1)]),
                         (np.nextafter(rn[i], 0.0), tn[j]), (rn[i], np.nextafter(tn[j], 0.0))):
                if inside(r) and cfg.theta0 <= t <= np.pi - cfg.theta0:
                    pts.append((r, t))
    pts = np.array(pts[: cfg.max_particles // 2])
    m = len(pts)
    z = np.zeros((2 * m, 6))
    z[0::2, 0] = z[1::2, 0] = pts[:, 0]
    z[0::2, 1] = z[1::2, 1] = pts[:, 1]
    z[:, 2] = rng.uniform(0, 2 * np.pi, 2 * m)
    z[:, 3:] = rng.normal(0, 0.05, (2 * m, 3))
    qm = np.tile([1.0, -1.0], m)
    return z, qm


def test_particles_on_nodes_and_edges():
    cfg = _pic_cfg()
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        z, qm = _grid_point_particles(ctx, cfg)
        ctx.load_particles(z, qm, w=np.full(len(qm), 1e-3))
        S0 = _levels(ctx)
        P0 = ctx.get_particles()
        ctx.step(1)
        S1 = _levels(ctx)
        P1 = ctx.get_particles()
    assert len(qm) > 100
    # initial charge of co-located pairs cancels exactly
    assert np.abs(S0[G.LEVEL_J][3]).max() == 0.0
    G6 = [S0[G.LEVEL_DH1][c].astype(np.float64) for c in range(3)] + \
         [S1[G.LEVEL_BH][c].astype(np.float64) for c in range(3)]
    err, _ = compare_push(cfg, P0, P1, push_params_from(cfg, O.FIELDS_GRID), grid=g, G6=G6)
    assert err <= TOL_STATE
    alive = ((P0["flags"] & 1) != 0) & ((P1["flags"] & 1) != 0)
    old = np.stack([P0["r"], P0["th"], P0["ph"]], axis=1)
    new = np.stack([P1["r"], P1["th"], P1["ph"]], axis=1)
    rho, Jr, Jt, Jp = O.deposit(g, cfg.dt, old, new, P0["qm"] * P0["w"], alive.astype(np.int32))
    for got, want in ((S1[G.LEVEL_J][3], rho), (S1[G.LEVEL_J][0], Jr),
                      (S1[G.LEVEL_J][1], Jt), (S1[G.LEVEL_J][2], Jp)):
        assert norm_err(got, want) < 1e-6
    # and the field update around them
    F = _oracle_fields(g, S0)
    O.pic_step(push_params_from(cfg, O.FIELDS_GRID), g, F, oracle_particles(P0),
               absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    assert not _field_errors(g, F, S1)


def test_empty_particle_set_evolves_vacuum_fields():
    cfg = _pic_cfg(n=64)
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        assert ctx.num_particles() == 0
        S0 = _levels(ctx)
        ctx.step(1)
        S1 = _levels(ctx)
        d = ctx.diagnostics()
    assert d["alive"] == 0 and d["implicit_steps"] == 0
    assert all(np.abs(S1[G.LEVEL_J][c]).max() == 0.0 for c in range(4))
    F = _oracle_fields(g, S0)
    O.pic_step(push_params_from(cfg, O.FIELDS_GRID), g, F, None,
               absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    assert not _field_errors(g, F, S1)


def test_neutral_and_charged_particles_in_grid_fields():
    """Hyb2 with neutral particles among charged ones in the static Wald grid
    field: neutral rejects go to the discrete-gradient scheme, charged ones
    to the implicit midpoint rule, in one implicit pass."""
    a = 0.9
    n = 3000
    cfg = G.config_default(a=a, nr=64, nth=48, r_in=0.9 * rplus(a), r_out=50.0, dt=0.05,
                           field_mode=G.FIELDS_STATIC, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-12, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=50.0, reflect=1, guess=G.GUESS_RK4)
    g = oracle_grid(cfg)
    p = O.init_particles(O.INIT_SHELL_ISO, a, SEED + 31, n, 2.0, 30.0, cfg.theta0,
                         np.pi - cfg.theta0, 1.0)
    qm = p.qm.copy()
    qm[::3] = 0.0
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.load_particles(p.state(), qm)
        G6 = gpu_fields_as_G(ctx)
        ctx.step(1)
        before = ctx.get_particles()
        ctx.step(1)
        after = ctx.get_particles()
    err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_GRID),
                          grid=g, G6=G6)
    assert err <= TOL_STATE
    impl = (after["flags"] & G.FLAG_IMPLICIT) != 0
    neutral = before["qm"] == 0
    assert impl[neutral].any() and impl[~neutral].any()
    assert (~impl[neutral]).any() and (~impl[~neutral]).any()


def test_schwarzschild_full_step():
    """a = 0: the Wald field reduces to a uniform field in Schwarzschild
    (App. B.1); one full cycle matches the oracle."""
    cfg = _pic_cfg(a=0.0, n=3000)
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 32, rplus(0.0), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        ctx.step(2)
        S0 = _levels(ctx)
        P0 = ctx.get_particles()
        ctx.step(1)
        S1 = _levels(ctx)
        P1 = ctx.get_particles()
    F = _oracle_fields(g, S0)
    O.pic_step(push_params_from(cfg, O.FIELDS_GRID), g, F, oracle_particles(P0),
               absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    assert not _field_errors(g, F, S1)
    G6 = [S0[G.LEVEL_DH1][c].astype(np.float64) for c in range(3)] + \
         [S1[G.LEVEL_BH][c].astype(np.float64) for c in range(3)]
    err, _ = compare_push(cfg, P0, P1, push_params_from(cfg, O.FIELDS_GRID), grid=g, G6=G6)
    assert err <= TOL_STATE


def test_schwarzschild_wald_start_full_steps():
    """Sec. 3.3: a = 0.999 spacetime started with the a = 0 Wald field (grid
    E_i = 0, D = -beta x B / alpha) and a pair plasma; the initial fields
    match the oracle's, then one full cycle after two steps matches too."""
    cfg = _pic_cfg(a=0.999, n=3000)
    g = oracle_grid(cfg)
    D, B = O.wald_grid(g, 1.0, a_field=0.0)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=0.0)
        for lev in (G.LEVEL_DN, G.LEVEL_BN):
            arrs, off = (D, 0) if lev == G.LEVEL_DN else (B, 3)
            for c in range(3):
                assert norm_err(ctx.get_field(lev, c), g.densitize(off + c, arrs[c])) < 1e-6
        assert np.abs(ctx.get_field(G.LEVEL_BN, 2)).max() == 0.0  # B^phi = 0
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 33, rplus(cfg.a), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        ctx.step(2)
        S0 = _levels(ctx)
        P0 = ctx.get_particles()
        ctx.step(1)
        S1 = _levels(ctx)
        P1 = ctx.get_particles()
    F = _oracle_fields(g, S0)
    O.pic_step(push_params_from(cfg, O.FIELDS_GRID), g, F, oracle_particles(P0),
               absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    assert not _field_errors(g, F, S1)
    G6 = [S0[G.LEVEL_DH1][c].astype(np.float64) for c in range(3)] + \
         [S1[G.LEVEL_BH][c].astype(np.float64) for c in range(3)]
    err, _ = compare_push(cfg, P0, P1, push_params_from(cfg, O.FIELDS_GRID), grid=g, G6=G6)
    assert err <= TOL_STATE


def test_zero_dt_is_half_the_courant_limit():
    """dt = 0 with a grid resolves to half the Courant limit (grpic_cfl_dt);
    the context reports the resolved configuration."""
    cfg = _pic_cfg(n=64)
    want = 0.5 * G.cfl_dt(cfg)
    cfg.dt = 0.0
    with G.Context(cfg) as ctx:
        assert ctx.cfg.dt == want and ctx.get_config().dt == want
        ctx.set_fields_wald(1.0)
        ctx.step(1)
    cfg = G.config_default(a=0.0, dt=0.0, max_particles=8)  # no grid: dt needed
    with pytest.raises(G.GrpicError):
        G.Context(cfg)


def test_time_step_above_the_courant_limit_is_refused():
    """grpic_create refuses a full-cycle configuration whose dt exceeds the
    grid's Courant limit (GRPIC_E_CFL) and accepts one just below it."""
    cfg = _pic_cfg(n=64)
    lim = G.cfl_dt(cfg)
    cfg.dt = 1.01 * lim
    with pytest.raises(G.GrpicError, match="error -2"):
        G.Context(cfg)
    cfg.dt = 0.99 * lim
    with G.Context(cfg) as ctx:
        assert ctx.get_config().dt == cfg.dt


def test_nonfinite_particle_is_removed_and_isolated():
    """A particle whose step gives a non-finite state is flagged, counted and
    removed; it deposits nothing, the fields stay finite, and every other
    particle steps as the oracle says."""
    cfg = _pic_cfg(n=2000)
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 34, rplus(cfg.a), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        P = ctx.get_particles()
        z = P["z"].copy()
        z[11, 3] = np.nan
        z[500, 5] = np.inf
        ctx.load_particles(z, P["qm"], P["w"], H0=P["H0"])
        S0 = _levels(ctx)
        P0 = ctx.get_particles()
        ctx.step(1)
        P1 = ctx.get_particles()
        S1 = _levels(ctx)
        d = ctx.diagnostics()
    bad = np.zeros(len(z), bool)
    bad[[11, 500]] = True
    assert np.all(P1["flags"][bad] == G.FLAG_REMOVED | G.FLAG_NONFINITE)
    assert d["nonfinite"] == 2
    for lev in S1:
        for c in range(len(S1[lev])):
            assert np.all(np.isfinite(S1[lev][c]))
    G6 = [S0[G.LEVEL_DH1][c].astype(np.float64) for c in range(3)] + \
         [S1[G.LEVEL_BH][c].astype(np.float64) for c in range(3)]
    keep = lambda D: {k: v[~bad] for k, v in D.items()}
    err, _ = compare_push(cfg, keep(P0), keep(P1), push_params_from(cfg, O.FIELDS_GRID),
                          grid=g, G6=G6)
    assert err <= TOL_STATE
