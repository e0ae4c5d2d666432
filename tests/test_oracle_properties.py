"""Property tests of the oracle over generated inputs (hypothesis): the
invariants the method guarantees at any position, move and state, beyond
the fixed seeds of the pin tests."""
import numpy as np
from hypothesis import given, settings, strategies as st

import oracle as O

A_SPIN = st.sampled_from([0.0, 0.5, 0.9, 0.99])
UNIT = st.floats(0.0, 1.0, allow_nan=False)
SETTINGS = settings(max_examples=40, deadline=None)


def _grid(a):
    rp = 1 + np.sqrt(1 - a * a)
    return O.Grid(a, 12, 10, 0.9 * rp, 15.0)


@SETTINGS
@given(a=A_SPIN, p=st.integers(0, 11), q=st.integers(0, 9), fr=UNIT, ft=UNIT)
def test_weights_are_a_partition_of_unity(a, p, q, fr, ft):
    """eqs. v1-v5 at any point of any cell: four non-negative weights that
    sum to one, and a node's weight is 1 at the node itself."""
    g = _grid(a)
    r = g.rn[p] + fr * (g.rn[p + 1] - g.rn[p])
    th = g.tn[q] + ft * (g.tn[q + 1] - g.tn[q])
    W = O.dep_weights(g, r, th, p, q)
    assert np.all(W >= -1e-15) and abs(W.sum() - 1.0) < 1e-14
    if fr == 0.0 and ft == 0.0:
        assert abs(W[0] - 1.0) < 1e-14


@SETTINGS
@given(a=A_SPIN, n=st.integers(1, 6), seed=st.integers(0, 2 ** 32 - 1),
       reach=st.floats(0.01, 2.5))
def test_deposit_is_charge_conserving_for_any_moves(a, n, seed, reach):
    """Sec. 2.3 with the conserving current: for any set of straight moves
    (crossing up to a few cells in both directions) the discrete continuity
    equation holds at every node and the total charge is the particles'."""
    g = _grid(a)
    rng = np.random.default_rng(seed)
    lo, hi = g.rn[0] * 1.001, g.rn[-1] * 0.999
    old = np.c_[rng.uniform(lo, hi, n), rng.uniform(g.th0, np.pi - g.th0, n),
                rng.uniform(0, 6, n)]
    step = np.c_[rng.uniform(-reach, reach, n), rng.uniform(-0.3, 0.3, n) * reach,
                 rng.uniform(-1, 1, n)]
    new = old + step
    new[:, 0] = np.clip(new[:, 0], lo, hi)
    new[:, 1] = np.clip(new[:, 1], g.th0 + 1e-9, np.pi - g.th0 - 1e-9)
    qw = rng.choice([-1.0, 1.0], n) * rng.uniform(0.5, 2.0, n)
    dt = 0.3
    rho0 = O.deposit(g, dt, old, old, qw)[0]
    rho1, Jr, Jt, _ = O.deposit(g, dt, old, new, qw)
    Lr = np.r_[g.rh[0] - g.rn[0], np.diff(g.rh), g.rn[-1] - g.rh[-1]]
    dth = g.tn[1] - g.tn[0]
    Lt = np.r_[0.5 * dth, np.full(g.nth - 1, dth), 0.5 * dth]
    res = (rho1 - rho0) / dt
    Jr_p = np.zeros((g.nth + 1, g.nr + 2))
    Jr_p[:, 1:-1] = Jr
    Jt_p = np.zeros((g.nth + 2, g.nr + 1))
    Jt_p[1:-1, :] = Jt
    res += (Jr_p[:, 1:] - Jr_p[:, :-1]) / Lr[None, :]
    res += (Jt_p[1:, :] - Jt_p[:-1, :]) / Lt[:, None]
    scale = max(np.abs(rho1).max(), np.abs(rho0).max()) / dt
    assert np.abs(res).max() <= 1e-11 * scale
    Q = (rho1 * 2 * np.pi * Lr[None, :] * Lt[:, None]).sum()
    assert abs(Q - qw.sum()) <= 1e-12 * np.abs(qw).sum()


@SETTINGS
@given(a=A_SPIN, r=st.floats(2.5, 12.0), th=st.floats(0.3, 2.8),
       u=st.lists(st.floats(-2.0, 2.0), min_size=3, max_size=3),
       qm=st.sampled_from([-1.0, 0.0, 1.0]))
def test_implicit_midpoint_is_time_reversible(a, r, th, u, qm):
    """eq. imr1 is symmetric: a step with +dt followed by one with -dt
    returns to the start (to the iteration tolerance) for any state, charged
    in the Wald field or neutral."""
    z0 = np.array([r, th, 0.4, *u])
    kw = dict(field_kind=O.FIELDS_WALD, B0=1.0, tol=1e-14, kmax=200)
    z1, k1, _ = O.step_imr(O.push_params(a, 0.02, **kw), qm, z0)
    z2, k2, _ = O.step_imr(O.push_params(a, -0.02, **kw), qm, z1)
    assert k1 > 0 and k2 > 0
    assert np.all(np.abs(z2 - z0) <= 1e-12 * np.maximum(np.abs(z0), 1.0))


@SETTINGS
@given(a=A_SPIN, r=st.floats(2.5, 12.0), th=st.floats(0.3, 2.8),
       u=st.lists(st.floats(-2.0, 2.0), min_size=3, max_size=3))
def test_discrete_gradient_conserves_energy_for_any_state(a, r, th, u):
    """Sec. 2.2.3: the discrete-gradient step keeps H to round-off and u_phi
    exactly, from any neutral state."""
    z0 = np.array([r, th, 0.1, *u])
    z1, k = O.step_ham(O.push_params(a, 0.1, tol=1e-14, kmax=200), z0)
    assert k > 0
    H0, H1 = O.energy(a, z0), O.energy(a, z1)
    assert abs(H1 - H0) <= 1e-13 * abs(H0)
    assert z1[5] == z0[5]
