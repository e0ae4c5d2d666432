"""Error of FP32 field storage (a project extension): the GPU stores and
gathers fields in FP32, the oracle here runs with FP64 fields.  The parity
tests compare with the oracle in FP32-field mode (same rounded arrays); these
tests state what the rounding itself costs, and bound it."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import norm_err, oracle_grid, oracle_particles, push_params_from, rplus, state_err

pytestmark = pytest.mark.gpu

SEED = 2602074520


def test_fp32_field_storage_error_on_particles():
    """One Hyb2 step of charged particles in the Wald grid field: GPU (FP32
    fields) against the oracle with the FP64 field values."""
    a = 0.9
    n = 4000
    cfg = G.config_default(a=a, nr=128, nth=96, r_in=0.9 * rplus(a), r_out=50.0, dt=0.01,
                           field_mode=G.FIELDS_STATIC, pusher=G.PUSH_RK4, max_particles=n,
                           r_remove_in=rplus(a), r_remove_out=50.0, reflect=1)
    g = oracle_grid(cfg)
    D, B = O.wald_grid(g, 1.0)
    G64 = [g.densitize(c, D[c]) for c in range(3)] + [g.densitize(3 + c, B[c]) for c in range(3)]
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, n, SEED + 2, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, 1.0)
        before = ctx.get_particles()
        ctx.step(1)
        after = ctx.get_particles()
    p = oracle_particles(before)
    O.push(push_params_from(cfg, O.FIELDS_GRID), p, grid=g, G=G64)
    alive = (before["flags"] & 1) != 0
    dz = state_err(after["z"][alive], p.state()[alive])
    # relative to the step itself: the field error enters through dt F
    step = np.abs(after["z"][alive] - before["z"][alive]).max(axis=0)
    rel_step = (np.abs(after["z"][alive] - p.state()[alive]).max(axis=0) /
                np.maximum(step, 1e-300))
    print(f"FP32-field storage: max state error {dz.max():.3e} (relative to max(|z|,1)); "
          f"per component relative to the step {np.array2string(rel_step, precision=2)}")
    assert dz.max() < 1e-8
    assert rel_step.max() < 1e-5


def test_fp32_field_storage_error_on_the_full_step():
    """One full PIC step from FP64-exact initial data: GPU fields (FP32) and
    the oracle's (FP64) after the step."""
    a = 0.99
    cfg = G.config_default(a=a, nr=48, nth=40, r_in=0.9 * rplus(a), r_out=20.0,
                           field_mode=G.FIELDS_EVOLVE, pusher=G.PUSH_HYB2, hyb_threshold=1e-9,
                           max_particles=4000, r_remove_in=rplus(a), r_remove_out=20.0,
                           reflect=1, r_abs=18.0, chi0=1e4, lambda_abs=5.0)
    cfg.dt = 0.5 * G.cfl_dt(cfg)
    g = oracle_grid(cfg)
    D, B = O.wald_grid(g, 1.0)
    p = O.init_particles(O.INIT_SHELL_MJ, a, SEED + 4, 4000, rplus(a), 18.0, cfg.theta0,
                         np.pi - cfg.theta0, 0.1, w=2e-3)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.load_particles(p.state(), p.qm, w=p.w)
        ctx.step(1)
        Dn = [ctx.get_field(G.LEVEL_DN, c) for c in range(3)]
        Bn = [ctx.get_field(G.LEVEL_BN, c) for c in range(3)]
        rho = ctx.get_field(G.LEVEL_J, 3)
    F = O.Fields.uniform_levels(g, D, B)
    q = p.copy()
    # first deposit of the oracle's own run: rho^{n+1} at the loaded positions
    O.pic_step(push_params_from(cfg, O.FIELDS_GRID), g, F, q,
               absorber=[cfg.r_abs, cfg.chi0, cfg.lambda_abs])
    errs = {f"D{c}": norm_err(Dn[c], g.densitize(c, F.Dn[c])) for c in range(3)}
    errs.update({f"B{c}": norm_err(Bn[c], g.densitize(3 + c, F.Bn[c])) for c in range(3)})
    print("FP32-field storage, one full step, relative max-norm field errors: " +
          ", ".join(f"{k} {v:.2e}" for k, v in errs.items()))
    assert max(errs.values()) < 1e-5
