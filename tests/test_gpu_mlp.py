"""The learned implicit guess (project extension) on the GPU, through the C
ABI: the BF16 matrix-core network and its gradient against the FP64 oracle
network with the same BF16-rounded weights; the training samples the
implicit pass collects against the oracle's features and converged steps;
and what the trained guess gains over the plain start of the iteration."""
import numpy as np
import pytest

import oracle as O
import paper_2602_07452_amd as G
from gpu_common import gpu_fields_as_G, oracle_grid, push_params_from, rplus, state_err

pytestmark = pytest.mark.gpu

SEED = 2602074520
NPAR = G.MLP_NPARAM
# blocks of the packed parameter vector
BLOCKS = {"W1": (0, 896), "b1": (896, 960), "W2": (960, 5056), "b2": (5056, 5120),
          "W3": (5120, 5504), "b3": (5504, 5510)}

# BF16 keeps 8 significant bits (unit roundoff 2^-9 ~ 2e-3).  The GPU rounds
# the weights (the oracle gets the same rounded weights) and also the inputs
# of every product (hidden activations, back-propagated errors); sums of 64
# such terms with mixed signs carry a relative error of a few 1e-3, so the
# outputs are compared at 1e-2 and the gradients (one more rounded product
# chain) at 2e-2, in norm.
TOL_FWD = 1e-2
TOL_GRAD = 2e-2


def bf16_round(x):
    """FP32 values rounded to the nearest BF16 (ties to even)."""
    u = np.ascontiguousarray(x, np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def random_theta(rng):
    th = np.zeros(NPAR, np.float32)
    for k, fan in (("W1", 14), ("b1", 14), ("W2", 64), ("b2", 64), ("W3", 64), ("b3", 64)):
        a, b = BLOCKS[k]
        th[a:b] = rng.uniform(-1, 1, b - a) / np.sqrt(fan)
    return th


def oracle_theta(th):
    """The parameters the GPU computes with: BF16 weights, FP32 biases."""
    t = th.astype(np.float32).copy()
    for k in ("W1", "W2", "W3"):
        a, b = BLOCKS[k]
        t[a:b] = bf16_round(t[a:b])
    return t.astype(np.float64)


def rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b)


@pytest.fixture
def net_ctx():
    cfg = G.config_default(a=0.9, max_particles=64)
    with G.Context(cfg) as ctx:
        yield ctx


def test_forward_matches_oracle(net_ctx):
    rng = np.random.default_rng(SEED + 40)
    th = random_theta(rng)
    net_ctx.mlp_set(th, np.zeros(14), np.ones(14), np.ones(6))
    n = 1000  # 16 blocks of 64 rows and a ragged tail
    X = bf16_round(rng.normal(size=(n, 14)))
    Y = net_ctx.mlp_forward(X)
    Yo = O.mlp_forward(oracle_theta(th), X.astype(np.float64))
    assert rel(Y, Yo) <= TOL_FWD
    for o in range(6):  # every output column, so a swapped column fails
        assert rel(Y[:, o], Yo[:, o]) <= 2 * TOL_FWD


def test_gradient_matches_oracle(net_ctx):
    rng = np.random.default_rng(SEED + 41)
    th = random_theta(rng)
    net_ctx.mlp_set(th, np.zeros(14), np.ones(14), np.ones(6))
    n = 777
    X = bf16_round(rng.normal(size=(n, 14)))
    T = rng.normal(size=(n, 6)).astype(np.float32)
    loss, g = net_ctx.mlp_loss_grad(X, T)
    lo, go = O.mlp_loss_grad(oracle_theta(th), X.astype(np.float64), T.astype(np.float64))
    assert abs(loss - lo) <= TOL_FWD * lo
    for k, (a, b) in BLOCKS.items():
        assert rel(g[a:b], go[a:b]) <= TOL_GRAD, k


def test_set_get_roundtrip(net_ctx):
    rng = np.random.default_rng(SEED + 42)
    th = random_theta(rng)
    mean, inv, sc = rng.normal(size=14), rng.uniform(0.5, 2, 14), rng.uniform(0.1, 1, 6)
    net_ctx.mlp_set(th, mean, inv, sc)
    th2, m2, i2, s2 = net_ctx.mlp_get()
    assert np.array_equal(th2, th) and np.array_equal(m2, mean.astype(np.float32))
    assert np.array_equal(i2, inv.astype(np.float32)) and np.array_equal(s2, sc.astype(np.float32))


# ------------------------------------------------------------ samples
def _wald_imr_cfg(n, guess=G.GUESS_MLP, dt=0.02):
    a = 0.9
    return G.config_default(a=a, nr=64, nth=48, r_in=0.9 * rplus(a), r_out=50.0, dt=dt,
                            field_mode=G.FIELDS_STATIC, pusher=G.PUSH_IMR,
                            max_particles=n, r_remove_in=rplus(a), r_remove_out=50.0,
                            reflect=1, guess=guess)


def _row_keys(Z32):
    return {Z32[i].tobytes(): i for i in range(len(Z32))}


def test_collected_samples_match_oracle():
    n = 3000
    cfg = _wald_imr_cfg(n)
    g = oracle_grid(cfg)
    P = push_params_from(cfg, O.FIELDS_GRID)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, n, SEED + 2, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, 1.0)
        G6 = gpu_fields_as_G(ctx)
        before = ctx.get_particles()
        ctx.mlp_collect(10 * n)
        ctx.step(1)
        X, T, valid = ctx.mlp_get_samples()
    alive = (before["flags"] & G.FLAG_ALIVE) != 0
    assert len(X) == alive.sum() and valid.all()
    keys = _row_keys(before["z"].astype(np.float32))
    rows = [keys[X[v, :6].tobytes()] for v in range(len(X))]
    assert len(set(rows)) == len(rows)  # every particle exactly once
    colmax = np.abs(X).max(axis=0)
    for v in range(0, len(X), 7):  # a sample of the rows, spread over the queue
        k = rows[v]
        z, qm = before["z"][k], before["qm"][k]
        D, B = O.gather(g, G6, z[0], z[1])
        m = O.metric(cfg.a, z[0], z[1])
        feat = np.concatenate([z, qm * D, qm * B, [m[0], m[1]]])
        assert np.all(np.abs(X[v] - feat) <= 1.2e-7 * np.abs(feat) + 1e-12 * colmax), v
        ze = z + cfg.dt * O.rhs(cfg.a, qm, z, D, B)
        zi, it, _ = O.step_imr(P, qm, z, guess=ze, grid=g, G=G6)
        t = zi - ze
        assert np.all(np.abs(T[v] - t) <= 1e-6 * np.abs(t) + 1e-11 * np.maximum(np.abs(z), 1)), v


@pytest.mark.parametrize("guess", [G.GUESS_RK4, G.GUESS_MLP])
def test_collected_hybrid_samples_match_oracle(guess):
    """Hyb2 passes its rejected particles to the implicit pass with the RK4
    result as the base of the guess.  The samples collected from them carry
    the network's features at z^n (z^n, q/m D, q/m B, alpha, beta^r) and,
    as target, the converged step minus the RK4 result, both as the oracle
    computes them; with the learned guess configured or not."""
    n = 3000
    a = 0.9
    cfg = G.config_default(a=a, nr=64, nth=48, r_in=0.9 * rplus(a), r_out=50.0, dt=0.02,
                           field_mode=G.FIELDS_STATIC, pusher=G.PUSH_HYB2,
                           hyb_threshold=1e-15, max_particles=n, r_remove_in=rplus(a),
                           r_remove_out=50.0, reflect=1, guess=guess)
    g = oracle_grid(cfg)
    P = push_params_from(cfg, O.FIELDS_GRID)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, n, SEED + 3, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, 1.0)
        G6 = gpu_fields_as_G(ctx)
        before = ctx.get_particles()
        ctx.mlp_collect(10 * n)
        ctx.step(1)
        after = ctx.get_particles()
        X, T, valid = ctx.mlp_get_samples()
    implicit = (after["flags"] & G.FLAG_IMPLICIT) != 0
    assert 0 < len(X) == implicit.sum() < n and valid.all()
    keys = _row_keys(before["z"].astype(np.float32))
    rows = [keys[X[v, :6].tobytes()] for v in range(len(X))]
    assert len(set(rows)) == len(rows) and implicit[rows].all()
    colmax = np.abs(X).max(axis=0)
    for v in range(0, len(X), max(1, len(X) // 200)):
        k = rows[v]
        z, qm = before["z"][k], before["qm"][k]
        D, B = O.gather(g, G6, z[0], z[1])
        m = O.metric(cfg.a, z[0], z[1])
        feat = np.concatenate([z, qm * D, qm * B, [m[0], m[1]]])
        assert np.all(np.abs(X[v] - feat) <= 1.2e-7 * np.abs(feat) + 1e-12 * colmax), v
        zr, _ = O.step_rk4(P, qm, z, grid=g, G=G6)
        zi, it, _ = O.step_imr(P, qm, z, guess=zr, grid=g, G=G6)
        t = zi - zr
        assert np.all(np.abs(T[v] - t) <= 1e-6 * np.abs(t) + 1e-11 * np.maximum(np.abs(z), 1)), v


# ------------------------------------------------------------ effect
def _mean_iters(d0, d1):
    h = d1["iter_hist"] - d0["iter_hist"]
    return (h @ np.arange(len(h))) / max(h.sum(), 1)


def test_trained_guess_cuts_iterations_and_keeps_the_result():
    """Train on 4 steps of 2^14 particles, then advance fresh particles with
    the plain start (z^n) and with the learned guess: the iteration converges
    to the same states (the fixed point does not depend on the start) in
    fewer iterations."""
    n = 1 << 14
    cfg = _wald_imr_cfg(n)
    with G.Context(cfg) as ctx:
        ctx.set_fields_wald(1.0)
        ctx.init_particles(G.INIT_SHELL_ISO, n, SEED + 2, 2.0, 30.0, cfg.theta0,
                           np.pi - cfg.theta0, 1.0)
        ctx.mlp_collect(4 * n)
        ctx.step(4)
        ctx.mlp_collect(0)
        assert ctx.mlp_num_samples() > 3 * n
        loss = ctx.mlp_train(epochs=30, batch=4096, lr=3e-3, lr_final=3e-5, seed=7)
        net = ctx.mlp_get()
    assert np.all(np.isfinite(loss)) and loss[-1] < 0.5 * loss[0]
    res = {}
    for name, guess in (("plain", G.GUESS_PLAIN), ("mlp", G.GUESS_MLP)):
        c = _wald_imr_cfg(n, guess=guess)
        with G.Context(c) as ctx:
            ctx.set_fields_wald(1.0)
            ctx.init_particles(G.INIT_SHELL_ISO, n, SEED + 9, 2.0, 30.0, c.theta0,
                               np.pi - c.theta0, 1.0)
            if guess == G.GUESS_MLP:
                ctx.mlp_set(*net)
            d0 = ctx.diagnostics()
            ctx.step(3)
            d1 = ctx.diagnostics()
            P = ctx.get_particles()
        res[name] = (P, _mean_iters(d0, d1), d1["noconv"] - d0["noconv"])
    (Pp, ip, ncp), (Pm, im, ncm) = res["plain"], res["mlp"]
    print(f"mean iterations plain {ip:.3f} learned {im:.3f}; loss {loss[0]:.3e} -> {loss[-1]:.3e}")
    assert ncp == 0 and ncm == 0
    assert np.array_equal(Pp["flags"], Pm["flags"])
    both = (Pp["flags"] & G.FLAG_ALIVE) != 0
    assert state_err(Pm["z"][both], Pp["z"][both]).max() <= 1e-11
    assert im < ip - 0.5
