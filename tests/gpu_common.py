"""Shared helpers of the GPU parity tests: build matching GPU contexts and
oracle states, compare with the stated tolerances."""
import numpy as np

import oracle as O
import paper_2602_07452_amd as G

# parity bars
TOL_STATE = 1e-12   # FP64 particle state, per component, relative to max(|z|, 1)
TOL_FIELD = 1e-5    # FP32 field arrays, max-norm relative
TIE = 1e-9          # hybrid decisions within this relative band of the threshold
# rounding uncertainty of a switch value (an energy difference relative to
# the energy, a few dozen FP64 operations): decisions this close to the
# threshold are ties as well
V_NOISE = 32 * 2.0 ** -52


def rplus(a):
    return 1.0 + np.sqrt(1.0 - a * a)


def state_err(z_gpu, z_orc):
    sc = np.maximum(np.abs(z_orc), 1.0)
    return np.abs(z_gpu - z_orc) / sc


def norm_err(a_gpu, a_orc):
    den = np.abs(a_orc).max()
    if den == 0.0:
        return np.abs(a_gpu).max()
    return np.abs(np.asarray(a_gpu, np.float64) - a_orc).max() / den


def oracle_particles(P):
    """oracle.Particles from a GPU get_particles() dict."""
    p = O.Particles(len(P["r"]))
    for k in ("r", "th", "ph", "ur", "uth", "uph", "qm", "w", "H0", "herr"):
        getattr(p, k)[:] = P[k]
    p.flags[:] = P["flags"] & O.ALIVE
    return p


def gpu_fields_as_G(ctx):
    """The six densitized FP32 arrays the push reads (D^{n+3/2}, B^{n+3/2}),
    as float64 for the oracle's FP32-field mode."""
    return [ctx.get_field(G.LEVEL_DH1, c).astype(np.float64) for c in range(3)] + \
           [ctx.get_field(G.LEVEL_BH, c).astype(np.float64) for c in range(3)]


def oracle_grid(cfg):
    return O.Grid(cfg.a, cfg.nr, cfg.nth, cfg.r_in, cfg.r_out, cfg.theta0)


def push_params_from(cfg, field_kind):
    return O.push_params(cfg.a, cfg.dt, pusher=cfg.pusher, guess=cfg.guess,
                         thr=cfg.hyb_threshold, tol=cfg.tol, kmax=cfg.kmax,
                         field_kind=field_kind, r_min=cfg.r_remove_in,
                         r_max=cfg.r_remove_out,
                         th_lo=cfg.theta0 if cfg.reflect else -1.0,
                         th_hi=np.pi - cfg.theta0 if cfg.reflect else 10.0,
                         ham_eps=cfg.ham_eps, dt_impl=cfg.dt_implicit, t_end=cfg.t_end,
                         deposit_mode=cfg.deposit_mode, solver=cfg.solver)


def compare_push(cfg, before, after, P, grid=None, G6=None, tol=TOL_STATE, t=None):
    """Run the oracle push from `before` (GPU particle dict; t: the particle
    clocks before the step, if any) and compare with the GPU result `after`.
    Hybrid decisions inside the tie band are re-run in the oracle with the
    GPU's choice.  Returns the max error and the oracle's particles."""
    p = oracle_particles(before)
    if t is not None:
        p.t = np.array(t, np.float64)
    O.push(P, p, grid=grid, G=G6)
    gpu_impl = (after["flags"] & G.FLAG_IMPLICIT) != 0
    orc_impl = (p.flags & O.IMPLICIT) != 0
    mismatch = np.nonzero((gpu_impl != orc_impl) & ((before["flags"] & 1) != 0))[0]
    if len(mismatch):
        c = p.crit[mismatch]
        noise = np.full(len(mismatch), V_NOISE)
        if P.pusher == O.HYB1:
            prev = before["herr"][mismatch]
            noise = V_NOISE * (1.0 + np.abs(c) * P.dt) / (P.dt * np.maximum(prev, 2.0 ** -52))
        band = np.abs(c - P.thr) <= np.maximum(TIE * abs(P.thr), noise)
        assert band.all(), f"hybrid choice differs outside the tie band: {c[~band][:5]}"
        force = np.full(len(before["r"]), -1, np.int32)
        force[mismatch] = gpu_impl[mismatch].astype(np.int32)
        p = oracle_particles(before)
        if t is not None:
            p.t = np.array(t, np.float64)
        O.push(P, p, grid=grid, G=G6, force=force)
    alive = (before["flags"] & 1) != 0
    err = state_err(after["z"][alive], p.state()[alive])
    assert np.array_equal(after["flags"][alive] & (G.FLAG_ALIVE | G.FLAG_REMOVED),
                          p.flags[alive] & (O.ALIVE | O.REMOVED))
    assert (err <= tol).all(), f"max state error {err.max():.3e}"
    # the switch value is a small difference of energies: its rounding noise
    # is absolute (a few ulp of e), plus what the 1e-12 state bar allows
    herr_ok = np.abs(after["herr"][alive] - p.herr[alive]) <= 1e-11 + 1e-6 * np.abs(p.herr[alive])
    assert herr_ok.all(), np.abs(after["herr"][alive] - p.herr[alive]).max()
    return float(err.max()), p


def levels(ctx):
    """Every field level of the context (host copies)."""
    return {lev: [ctx.get_field(lev, c) for c in range(4 if lev >= G.LEVEL_J else 3)]
            for lev in range(8)}


def oracle_fields(g, S):
    """Oracle fields (plain values) from the GPU levels S."""
    F = O.Fields(g)
    dd = lambda lev, off: [g.densitize(off + c, S[lev][c].astype(np.float64), -1)
                           for c in range(3)]
    F.Dn, F.Dh0, F.Dh1 = dd(G.LEVEL_DN, 0), dd(G.LEVEL_DH0, 0), dd(G.LEVEL_DH1, 0)
    F.Bm, F.Bn, F.Bh = dd(G.LEVEL_BM, 3), dd(G.LEVEL_BN, 3), dd(G.LEVEL_BH, 3)
    F.Jprev = [S[G.LEVEL_J][c].astype(np.float64) for c in range(3)]
    F.rho = S[G.LEVEL_J][3].astype(np.float64)
    return F


def field_errors(g, F, S1):
    """Components of the GPU levels S1 off the oracle fields F by more than
    TOL_FIELD (relative max norm)."""
    errs = {}
    for name, lev, arrs, off in (("Dn", G.LEVEL_DN, F.Dn, 0), ("Dh0", G.LEVEL_DH0, F.Dh0, 0),
                                 ("Dh1", G.LEVEL_DH1, F.Dh1, 0), ("Bm", G.LEVEL_BM, F.Bm, 3),
                                 ("Bn", G.LEVEL_BN, F.Bn, 3), ("Bh", G.LEVEL_BH, F.Bh, 3)):
        for c in range(3):
            errs[f"{name}{c}"] = norm_err(S1[lev][c], g.densitize(off + c, arrs[c]))
    return {k: v for k, v in errs.items() if not v <= TOL_FIELD}
