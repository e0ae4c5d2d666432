"""Snapshots through the C ABI (grpic_get_state / grpic_set_state): a run
restored from a snapshot into a fresh context continues exactly as the
uninterrupted run (the deposit sums are order-independent integers, so
every field and particle is bit-identical), in every field mode; snapshots
of another grid, or damaged ones, are refused."""
import numpy as np
import pytest

import paper_2602_07452_amd as G
from gpu_common import rplus

pytestmark = pytest.mark.gpu

SEED = 2602074520


def _pic_cfg(n=3000, sort_every=3):
    a = 0.99
    cfg = G.config_default(a=a, nr=40, nth=32, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-10, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=20.0, reflect=1, r_abs=18.0, chi0=1e4,
                           lambda_abs=5.0, tile_r=16, tile_th=16, sort_every=sort_every,
                           guess=G.GUESS_RK4)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    return cfg


def _everything(ctx):
    out = {"particles": ctx.get_particles(), "diag": ctx.diagnostics()}
    if ctx.cfg.field_mode != G.FIELDS_NONE:
        out["fields"] = {(lev, c): ctx.get_field(lev, c)
                         for lev in range(8) for c in range(4 if lev >= G.LEVEL_J else 3)}
    return out


def _assert_identical(x, y):
    for k in x["particles"]:
        assert np.array_equal(x["particles"][k], y["particles"][k]), k
    for k in x["diag"]:
        assert np.array_equal(x["diag"][k], y["diag"][k]), k
    for k in x.get("fields", {}):
        assert np.array_equal(x["fields"][k], y["fields"][k]), k


def _resume_matches(cfg, setup, before=4, after=5, graph=False):
    with G.Context(cfg) as ctx:
        setup(ctx)
        ctx.step(before)
        n = ctx.num_particles()
        snap = ctx.get_state()
        ctx.step(after)
        want = _everything(ctx)
    h = G.state_header(snap)
    assert h.magic == b"GRPICST" and h.version == 2 and h.bytes == snap.size
    assert h.steps == before and h.n == n
    with G.Context(cfg) as ctx:
        ctx.set_state(snap)
        assert np.array_equal(ctx.get_state(), snap)  # restore is lossless
        ctx.use_graph(graph)
        ctx.step(after)
        got = _everything(ctx)
    _assert_identical(want, got)
    return want


def test_full_pic_run_resumes_exactly():
    """Full cycle with Hyb2 (some particles implicit) and sorts every three
    steps on both sides of the snapshot; the resumed run replays graphs."""
    cfg = _pic_cfg()

    def setup(ctx):
        ctx.set_fields_wald(1.0, a_field=0.0)
        ctx.init_particles(G.INIT_SHELL_MJ, cfg.max_particles, SEED + 50, rplus(cfg.a), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)

    want = _resume_matches(cfg, setup, graph=True)
    d = want["diag"]
    assert d["steps"] == 9 and d["implicit_steps"] > 0
    assert np.abs(want["fields"][(G.LEVEL_J, 3)]).max() > 0


def test_static_field_run_resumes_exactly():
    a = 0.9
    cfg = G.config_default(a=a, nr=64, nth=48, r_in=0.9 * rplus(a), r_out=50.0, dt=0.02,
                           field_mode=G.FIELDS_STATIC, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-12, max_particles=2000, r_remove_in=rplus(a),
                           r_remove_out=50.0, reflect=1, guess=G.GUESS_RK4, sort_every=2)

    def setup(ctx):
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, cfg.max_particles, SEED + 51, 2.0, 30.0,
                           cfg.theta0, np.pi - cfg.theta0, 1.0)

    _resume_matches(cfg, setup)


def test_neutral_orbits_resume_exactly():
    """No grid: Hyb2 with the discrete-gradient fallback."""
    n = 1000
    cfg = G.config_default(a=0.0, dt=0.05, max_particles=n, r_remove_in=2.0,
                           pusher=G.PUSH_HYB2, hyb_threshold=1e-15)

    def setup(ctx):
        ctx.init_particles(G.INIT_ORBITS, n, SEED + 52, 6.0, 20.0, np.pi / 4,
                           3 * np.pi / 4, 0.1)

    want = _resume_matches(cfg, setup)
    assert want["diag"]["implicit_steps"] > 0


def test_snapshot_of_another_grid_or_damaged_is_refused():
    cfg = _pic_cfg(n=512)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_MJ, 512, SEED + 53, rplus(cfg.a), 18.0,
                           cfg.theta0, np.pi - cfg.theta0, 0.1, w=2e-3)
        snap = ctx.get_state()
        state0 = _everything(ctx)
        for bad in (snap[:-1], snap[:100]):
            with pytest.raises(G.GrpicError):
                ctx.set_state(bad)
        broken = snap.copy()
        broken[0] ^= 1
        with pytest.raises(G.GrpicError):
            ctx.set_state(broken)
        _assert_identical(state0, _everything(ctx))  # refused: nothing changed
    other = _pic_cfg(n=512)
    other.nth = 40
    other.dt = 0.5 * G.cfl_dt(other)
    with G.Context(other) as ctx:
        with pytest.raises(G.GrpicError):
            ctx.set_state(snap)
    small = _pic_cfg(n=256)
    small.dt = cfg.dt
    with G.Context(small) as ctx:
        with pytest.raises(G.GrpicError):
            ctx.set_state(snap)
