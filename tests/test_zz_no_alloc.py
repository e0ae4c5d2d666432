"""The allocation-free grid diagnostics (grpic_field_diagnostics_noalloc)
against the allocating entry point, through the C ABI: two calls in a row on
one GPU, the second on a smaller grid with smaller maxima (so maxima left in
the shared scratch by the first call would show), each compared bitwise with
grpic_field_diagnostics on the same state."""
import numpy as np
import pytest

import paper_2602_07452_amd as G
from gpu_common import rplus

pytestmark = pytest.mark.gpu

SEED = 2602074520


def _ctx(nr, nth, B0, n, seed):
    a = 0.9
    cfg = G.config_default(a=a, nr=nr, nth=nth, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-13, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=20.0, reflect=1, r_abs=18.0, chi0=1e4,
                           lambda_abs=5.0, tile_r=16, tile_th=16, guess=G.GUESS_RK4)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    ctx = G.Context(cfg)
    ctx.set_fields_wald(B0)
    ctx.init_particles(G.INIT_SHELL_MJ, n, seed, rplus(a), 16.0, cfg.theta0,
                       np.pi - cfg.theta0, 0.1, w=2e-3)
    ctx.step(3)
    return ctx


def _same(x, y):
    gx, bx, px = x
    gy, by, py = y
    assert gx == gy and bx == by
    assert np.array_equal(px, py)


def test_noalloc_diagnostics_equal_the_allocating_ones():
    big = _ctx(96, 80, 40.0, 8192, SEED + 90)
    small = _ctx(40, 32, 1.0, 2048, SEED + 91)
    try:
        first = big.field_diagnostics_noalloc()
        print(f"noalloc call 1 (96x80): gauss {first[0]:.3e} divB {first[1]:.3e}", flush=True)
        _same(first, big.field_diagnostics())
        second = small.field_diagnostics_noalloc()
        print(f"noalloc call 2 (40x32): gauss {second[0]:.3e} divB {second[1]:.3e}",
              flush=True)
        ref = small.field_diagnostics()
        _same(second, ref)
        # the first call's maxima were larger: the second cleared them
        assert first[0] > second[0] and first[1] > second[1]
        assert len(second[2]) == 41 and np.abs(ref[2]).max() > 0
        # the same state again gives the same values (nothing carried over)
        _same(big.field_diagnostics_noalloc(), first)
    finally:
        big.close()
        small.close()


def test_noalloc_diagnostics_refuse_grids_beyond_the_scratch():
    a = 0.9
    cfg = G.config_default(a=a, nr=16385, nth=2, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_STATIC, max_particles=0)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        with pytest.raises(G.GrpicError, match="16384"):
            ctx.field_diagnostics_noalloc()
        # the allocating entry point handles the same grid
        assert len(ctx.field_diagnostics()[2]) == 16386
