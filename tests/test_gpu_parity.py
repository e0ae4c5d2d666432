"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the
same seeded inputs.  Sizes span several tiles and a ragged tail while the
oracle finishes in seconds."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import (TOL_FIELD, TOL_STATE, compare_push, gpu_fields_as_G,
                        norm_err, oracle_grid, push_params_from, rplus, state_err)

pytestmark = pytest.mark.gpu

SEED = 2602074520


# --------------------------------------------------------------- neutral
@pytest.fixture(scope="module")
def orbits():
    n = 1000  # ragged: not a multiple of the 256-thread block
    cfg = G.config_default(a=0.0, dt=0.05, max_particles=n, r_remove_in=2.0)
    with G.Context(cfg) as ctx:
        ctx.init_particles(G.INIT_ORBITS, n, SEED + 1, 6.0, 20.0, np.pi / 4,
                           3 * np.pi / 4, 0.1)
        P = ctx.get_particles()
    return cfg, P


def test_orbit_initial_data_matches_oracle(orbits):
    cfg, P = orbits
    p = O.init_particles(O.INIT_ORBITS, 0.0, SEED + 1, len(P["r"]), 6.0, 20.0,
                         np.pi / 4, 3 * np.pi / 4, 0.1)
    assert (state_err(P["z"], p.state()) <= 1e-14).all()
    assert np.allclose(P["H0"], p.H0, rtol=1e-14, atol=0)


@pytest.mark.parametrize("pusher,thr", [(G.PUSH_RK4, 0.0), (G.PUSH_IMR, 0.0),
                                        (G.PUSH_HAM, 0.0), (G.PUSH_HYB1, 1.5),
                                        (G.PUSH_HYB2, 1e-15)])
def test_neutral_pushers_one_step(orbits, pusher, thr):
    cfg0, P0 = orbits
    cfg = G.config_default(a=0.0, dt=0.05, max_particles=len(P0["r"]), pusher=pusher,
                           hyb_threshold=thr, r_remove_in=2.0)
    with G.Context(cfg) as ctx:
        ctx.load_particles(P0["z"], P0["qm"], P0["w"], H0=P0["H0"])
        before = ctx.get_particles()
        ctx.step(1)
        after = ctx.get_particles()
    err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_NONE))
    assert err <= TOL_STATE


@pytest.mark.parametrize("pusher,dt,dt_im,thr,t_end", [
    (G.PUSH_HYB2, 0.5, 1.0, 1e-15, 4.3),   # Table 2, a.0 row
    (G.PUSH_HYB1, 0.08, 1.0, 1.5, 1.0),    # Table 2, a.0 row
    (G.PUSH_HAM, 1.0, 1.0, 0.0, 3.5)])
def test_own_step_lengths_match_oracle(orbits, pusher, dt, dt_im, thr, t_end):
    """Steps of their own length (Sec. 3.1.2, Table 2): every step of the
    run to t_end against the oracle from the GPU's state and clocks; the
    clocks agree bit for bit, the clipped last steps land on t_end, and the
    particles then stay."""
    cfg0, P0 = orbits
    cfg = G.config_default(a=0.0, dt=dt, dt_implicit=dt_im, t_end=t_end,
                           max_particles=len(P0["r"]), pusher=pusher, hyb_threshold=thr,
                           r_remove_in=2.0)
    Pp = push_params_from(cfg, O.FIELDS_NONE)
    impl = expl = 0
    with G.Context(cfg) as ctx:
        ctx.load_particles(P0["z"], P0["qm"], P0["w"], H0=P0["H0"])
        assert np.all(ctx.get_times() == 0.0)
        for _ in range(100):
            before, t0 = ctx.get_particles(), ctx.get_times()
            alive = (before["flags"] & 1) != 0
            if np.all(t0[alive] == t_end):
                break
            ctx.step(1)
            after, t1 = ctx.get_particles(), ctx.get_times()
            _, p = compare_push(cfg, before, after, Pp, t=t0)
            assert np.array_equal(t1[alive], p.t[alive])
            moved = alive & (t0 < t_end)
            step_impl = (after["flags"] & G.FLAG_IMPLICIT) != 0
            impl += int((moved & step_impl).sum())
            expl += int((moved & ~step_impl).sum())
        else:
            raise AssertionError("clocks did not reach t_end")
        ctx.step(1)
        still = ctx.get_particles()
        assert np.array_equal(still["z"][alive], before["z"][alive])
        assert np.all(still["flags"][alive] == G.FLAG_ALIVE)
        assert np.all(still["iters"][alive] == 0)
        assert ctx.diagnostics()["alive"] == int(alive.sum())
    if pusher != G.PUSH_HAM:
        assert impl > 0 and expl > 0


def test_neutral_hybrid_many_steps_statistics(orbits):
    """40 Hyb2 steps at the a = 0 Table 2 threshold (1e-15, at the rounding
    level of the switch value, so individual choices are ties): the GPU keeps
    every particle's energy violation at the threshold up to the implicit
    scheme's round-off drift and uses the implicit scheme about as often as
    the oracle."""
    cfg0, P0 = orbits
    cfg = G.config_default(a=0.0, dt=0.05, max_particles=len(P0["r"]),
                           pusher=G.PUSH_HYB2, hyb_threshold=1e-15, r_remove_in=2.0)
    Pp = push_params_from(cfg, O.FIELDS_NONE)
    from gpu_common import oracle_particles
    with G.Context(cfg) as ctx:
        ctx.load_particles(P0["z"], P0["qm"], P0["w"], H0=P0["H0"])
        p = oracle_particles(ctx.get_particles())
        n_orc = 0
        for _ in range(40):
            O.push(Pp, p)
            n_orc += int(((p.flags & O.IMPLICIT) != 0).sum())
        ctx.step(40)
        after = ctx.get_particles()
        d = ctx.diagnostics()
    alive = (after["flags"] & 1) != 0
    e = np.array([O.energy(0.0, z) for z in after["z"][alive]])
    viol = np.abs(e / after["H0"][alive] - 1.0)
    assert viol.max() < 1e-15 + 1e-13
    assert d["steps"] == 40
    assert abs(d["implicit_steps"] - n_orc) <= 0.05 * max(n_orc, 1) + 20


# ------------------------------------------------------- static Wald field
def _wald_cfg(pusher, thr=0.0, n=3000, nr=64, nth=48, dt=0.02, guess=G.GUESS_PLAIN):
    a = 0.9
    return G.config_default(a=a, nr=nr, nth=nth, r_in=0.9 * rplus(a), r_out=50.0,
                            dt=dt, field_mode=G.FIELDS_STATIC, pusher=pusher,
                            hyb_threshold=thr, max_particles=n, r_remove_in=rplus(a),
                            r_remove_out=50.0, reflect=1, guess=guess)


@pytest.mark.parametrize("a_field", [None, 0.0, 0.5])
def test_wald_grid_fields_match_oracle(a_field):
    """Wald field of the spacetime's spin (default), the Schwarzschild-Wald
    start (a_field = 0, Sec. 3.3) and a third spin, on every Yee subgrid."""
    cfg = _wald_cfg(G.PUSH_RK4)
    g = oracle_grid(cfg)
    D, B = O.wald_grid(g, 1.0, a_field=a_field)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0, a_field=a_field)
        for lev, arrs, off in ((G.LEVEL_DH1, D, 0), (G.LEVEL_BH, B, 3), (G.LEVEL_DN, D, 0),
                               (G.LEVEL_BM, B, 3)):
            for c in range(3):
                want = g.densitize(off + c, arrs[c])
                assert norm_err(ctx.get_field(lev, c), want) < 1e-6


@pytest.mark.parametrize("pusher,thr,guess", [(G.PUSH_RK4, 0.0, G.GUESS_PLAIN),
                                              (G.PUSH_IMR, 0.0, G.GUESS_PLAIN),
                                              (G.PUSH_HYB2, 1e-13, G.GUESS_PLAIN),
                                              (G.PUSH_HYB2, 1e-13, G.GUESS_RK4),
                                              (G.PUSH_HYB1, 0.5, G.GUESS_PLAIN)])
def test_charged_static_wald_one_step(pusher, thr, guess):
    cfg = _wald_cfg(pusher, thr, guess=guess)
    g = oracle_grid(cfg)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, cfg.max_particles, SEED + 2, 2.0, 30.0,
                           cfg.theta0, np.pi - cfg.theta0, 1.0)
        G6 = gpu_fields_as_G(ctx)
        ctx.step(2)  # a history for Hyb1's rate
        before = ctx.get_particles()
        ctx.step(1)
        after = ctx.get_particles()
    err, p = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_GRID),
                          grid=g, G6=G6)
    assert err <= TOL_STATE
    if pusher == G.PUSH_HYB2:
        frac = ((after["flags"] & G.FLAG_IMPLICIT) != 0).mean()
        assert 0.0 < frac < 1.0


@pytest.mark.parametrize("pusher,thr", [(G.PUSH_IMR, 0.0), (G.PUSH_HYB2, 1e-13)])
def test_newton_solver_matches_oracle_and_picard(pusher, thr):
    """Newton's method (solver NEWTON) against the oracle's Newton, and the
    same solution as the Picard iteration in fewer iterations (dt = 0.1)."""
    out = {}
    for solver in (G.SOLVER_NEWTON, G.SOLVER_PICARD):
        cfg = _wald_cfg(pusher, thr, dt=0.1)
        cfg.solver = solver
        g = oracle_grid(cfg)
        with G.Context(cfg) as ctx:
            ctx.set_fields_wald(1.0)
            ctx.init_particles(G.INIT_SHELL_ISO, cfg.max_particles, SEED + 2, 2.0, 30.0,
                               cfg.theta0, np.pi - cfg.theta0, 1.0)
            G6 = gpu_fields_as_G(ctx)
            before = ctx.get_particles()
            ctx.step(1)
            after = ctx.get_particles()
        if solver == G.SOLVER_NEWTON:
            err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_GRID),
                                  grid=g, G6=G6)
            assert err <= TOL_STATE
        out[solver] = after
    n, p = out[G.SOLVER_NEWTON], out[G.SOLVER_PICARD]
    both = ((n["flags"] & p["flags"] & G.FLAG_IMPLICIT) != 0)
    assert both.sum() > 100
    assert np.all(state_err(n["z"][both], p["z"][both]) <= 2e-12)
    assert n["iters"][both].mean() < 0.7 * p["iters"][both].mean()


def test_newton_solver_neutral_orbits(orbits):
    """The implicit midpoint rule by Newton's method for geodesics."""
    cfg0, P0 = orbits
    cfg = G.config_default(a=0.0, dt=0.05, max_particles=len(P0["r"]), pusher=G.PUSH_IMR,
                           r_remove_in=2.0, solver=G.SOLVER_NEWTON)
    with G.Context(cfg) as ctx:
        ctx.load_particles(P0["z"], P0["qm"], P0["w"], H0=P0["H0"])
        before = ctx.get_particles()
        ctx.step(1)
        after = ctx.get_particles()
    err, _ = compare_push(cfg, before, after, push_params_from(cfg, O.FIELDS_NONE))
    assert err <= TOL_STATE


def test_shell_initial_data_matches_oracle():
    cfg = _wald_cfg(G.PUSH_RK4, n=2000)
    with G.Context(cfg) as ctx:
        ctx.init_particles(G.INIT_SHELL_ISO, 2000, SEED + 3, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, 1.0)
        P = ctx.get_particles()
    p = O.init_particles(O.INIT_SHELL_ISO, cfg.a, SEED + 3, 2000, 2.0, 30.0, cfg.theta0,
                         np.pi - cfg.theta0, 1.0)
    assert (state_err(P["z"], p.state()) <= 1e-12).all()
    assert np.array_equal(P["qm"], p.qm)


# ------------------------------------------------------------- full PIC
def _pic_cfg(n=4000, nr=48, nth=40):
    a = 0.99
    cfg = G.config_default(a=a, nr=nr, nth=nth, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-9, max_particles=n,
                           r_remove_in=rplus(a), r_remove_out=20.0, reflect=1,
                           r_abs=18.0, chi0=1e4, lambda_abs=5.0, tile_r=16, tile_th=16)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _gpu_state(ctx):
    S = {lev: [ctx.get_field(lev, c) for c in range(4 if lev >= G.LEVEL_J else 3)]
         for lev in range(8)}
    return S, ctx.get_particles()


def _oracle_fields(g, S):
    F = O.Fields(g)
    dd = lambda lev, off: [g.densitize(off + c, S[lev][c].astype(np.float64), -1)
                           for c in range(3)]
    F.Dn, F.Dh0, F.Dh1 = dd(G.LEVEL_DN, 0), dd(G.LEVEL_DH0, 0), dd(G.LEVEL_DH1, 0)
    F.Bm, F.Bn, F.Bh = dd(G.LEVEL_BM, 3), dd(G.LEVEL_BN, 3), dd(G.LEVEL_BH, 3)
    F.Jprev = [S[G.LEVEL_J][c].astype(np.float64) for c in range(3)]
    F.rho = S[G.LEVEL_J][3].astype(np.float64)
    return F


@pytest.fixture(scope="module")
def pic_run():
    cfg = _pic_cfg()
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 4, rplus(cfg.a),
                           18.0, cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        ctx.step(3)
        S0, P0 = _gpu_state(ctx)
        ctx.step(1)
        S1, P1 = _gpu_state(ctx)
    return cfg, S0, P0, S1, P1


def test_full_step_fields_match_oracle(pic_run):
    cfg, S0, P0, S1, P1 = pic_run
    g = oracle_grid(cfg)
    F = _oracle_fields(g, S0)
    p = __import__("gpu_common").oracle_particles(P0)
    O.pic_step(push_params_from(cfg, O.FIELDS_GRID), g, F, p,
               absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    errs = {}
    for name, lev, arrs, off in (("Dn", G.LEVEL_DN, F.Dn, 0), ("Dh0", G.LEVEL_DH0, F.Dh0, 0),
                                 ("Dh1", G.LEVEL_DH1, F.Dh1, 0), ("Bm", G.LEVEL_BM, F.Bm, 3),
                                 ("Bn", G.LEVEL_BN, F.Bn, 3), ("Bh", G.LEVEL_BH, F.Bh, 3)):
        for c in range(3):
            errs[f"{name}{c}"] = norm_err(S1[lev][c], g.densitize(off + c, arrs[c]))
    for c in range(3):
        errs[f"J{c}"] = norm_err(S1[G.LEVEL_J][c], F.Jprev[c])
    errs["rho"] = norm_err(S1[G.LEVEL_J][3], F.rho)
    bad = {k: v for k, v in errs.items() if not v <= TOL_FIELD}
    assert not bad, bad


def test_full_step_particles_match_oracle(pic_run):
    """Particle parity at 1e-12: the oracle pushes with the GPU's own FP32
    D^{n+3/2} (input level) and B^{n+3/2} (rebuilt by the step)."""
    cfg, S0, P0, S1, P1 = pic_run
    g = oracle_grid(cfg)
    G6 = [S0[G.LEVEL_DH1][c].astype(np.float64) for c in range(3)] + \
         [S1[G.LEVEL_BH][c].astype(np.float64) for c in range(3)]
    err, _ = compare_push(cfg, P0, P1, push_params_from(cfg, O.FIELDS_GRID), grid=g, G6=G6)
    assert err <= TOL_STATE


def test_full_step_deposit_matches_oracle(pic_run):
    """Deposit of the GPU's own move (same old/new positions) vs the oracle."""
    cfg, S0, P0, S1, P1 = pic_run
    g = oracle_grid(cfg)
    alive = ((P0["flags"] & 1) != 0) & ((P1["flags"] & 1) != 0)
    old = np.stack([P0["r"], P0["th"], P0["ph"]], axis=1)
    new = np.stack([P1["r"], P1["th"], P1["ph"]], axis=1)
    rho, Jr, Jt, Jp = O.deposit(g, cfg.dt, old, new, P0["qm"] * P0["w"], alive.astype(np.int32))
    for got, want in ((S1[G.LEVEL_J][3], rho), (S1[G.LEVEL_J][0], Jr),
                      (S1[G.LEVEL_J][1], Jt), (S1[G.LEVEL_J][2], Jp)):
        assert norm_err(got, want) < 1e-6


def test_deposit_is_charge_conserving_on_gpu(pic_run):
    """Discrete continuity of the GPU's rho and J (FP32 outputs) at interior
    nodes away from the horizon."""
    cfg, S0, P0, S1, P1 = pic_run
    g = oracle_grid(cfg)
    rho0, rho1 = S0[G.LEVEL_J][3].astype(np.float64), S1[G.LEVEL_J][3].astype(np.float64)
    Jr, Jt = S1[G.LEVEL_J][0].astype(np.float64), S1[G.LEVEL_J][1].astype(np.float64)
    nr, nth = cfg.nr, cfg.nth
    Lr = np.diff(g.rh)
    res = (rho1 - rho0)[1:-1, 1:-1] / cfg.dt
    res += (Jr[1:-1, 1:] - Jr[1:-1, :-1]) / Lr[None, :]
    res += (Jt[1:, 1:-1] - Jt[:-1, 1:-1]) / (g.tn[1] - g.tn[0])
    mask = g.rn[1:-1][None, :] > rplus(cfg.a) + 2 * (g.rn[1] - g.rn[0]) * 3
    scale = np.abs(rho1).max() / cfg.dt
    assert np.abs(res[:, mask[0]]).max() < 1e-5 * scale


def test_full_step_is_deterministic():
    """Two runs from the same inputs give bitwise identical grids and particles
    (fixed-point deposit sums do not depend on the atomic order)."""
    cfg = _pic_cfg(n=3000)
    outs = []
    for _ in range(2):
        with G.Context(cfg) as ctx:
            ctx.set_fields_wald(1.0)
            ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 5, rplus(cfg.a),
                               18.0, cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
            ctx.step(3)
            outs.append(_gpu_state(ctx))
    (Sa, Pa), (Sb, Pb) = outs
    for lev in Sa:
        for a, b in zip(Sa[lev], Sb[lev]):
            assert np.array_equal(a, b)
    assert np.array_equal(Pa["z"], Pb["z"])


def _rows(P):
    """Particle records in a canonical order (the tile sort permutes them)."""
    M = np.column_stack([P["z"], P["qm"], P["w"], P["H0"], P["flags"], P["iters"]])
    return M[np.lexsort(M.T[::-1])]


def test_autotune_keeps_results():
    """The autotuner only changes launch settings and the particle order: the
    grids after its trial steps equal, bit for bit, those of the same number
    of steps with the default settings, and so do the particle records."""
    cfg = _pic_cfg(n=6000, nr=64, nth=48)
    outs, steps = [], None
    for tune in (True, False):
        with G.Context(cfg) as ctx:
            ctx.set_fields_wald(1.0)
            ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 7, rplus(cfg.a),
                               18.0, cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
            if tune:
                r = ctx.autotune(1)
                steps = r["steps"]
                assert r["trials"] >= 8 and r["ms_best"] <= r["ms_start"]
                assert (r["tile_r"], r["tile_th"]) in ((16, 16), (32, 16), (32, 32), (64, 16),
                                                      (64, 32))
                assert r["persistent_waves"] in (4, 8, 16, 32)
            else:
                ctx.step(steps)
            outs.append(_gpu_state(ctx))
    (Sa, Pa), (Sb, Pb) = outs
    for lev in Sa:
        for a, b in zip(Sa[lev], Sb[lev]):
            assert np.array_equal(a, b)
    assert np.array_equal(_rows(Pa), _rows(Pb))


def test_graph_replay_equals_eager():
    cfg = _pic_cfg(n=3000)
    outs = []
    for graph in (False, True):
        with G.Context(cfg) as ctx:
            ctx.set_fields_wald(1.0)
            ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 6, rplus(cfg.a),
                               18.0, cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
            ctx.use_graph(graph)
            ctx.step(4)
            ctx.sync()
            outs.append(_gpu_state(ctx))
    (Sa, Pa), (Sb, Pb) = outs
    for lev in Sa:
        for a, b in zip(Sa[lev], Sb[lev]):
            assert np.array_equal(a, b)
    assert np.array_equal(Pa["z"], Pb["z"])


def test_mj_initial_data_matches_oracle():
    cfg = _pic_cfg(n=2000)
    with G.Context(cfg) as ctx:
        ctx.init_particles(G.INIT_SHELL_MJ, 2000, SEED + 7, rplus(cfg.a), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=1.0)
        P = ctx.get_particles()
    p = O.init_particles(O.INIT_SHELL_MJ, cfg.a, SEED + 7, 2000, rplus(cfg.a), 18.0,
                         cfg.theta0, np.pi - cfg.theta0, 0.1)
    assert (state_err(P["z"], p.state()) <= 1e-12).all()
